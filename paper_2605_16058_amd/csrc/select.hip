// Rank selection.
//  t-SVDM-I  (Section 3.3): the same rank k on every slice.
//  t-SVDM-II (Algorithm 2): sort all squared singular values ascending, take
//  cumulative sums, find the largest J with w_J / W < eps^2, threshold
//  tau = v_J and keep, per slice, the values strictly above tau.
//
// The squared values are FP64 and non-negative, so their IEEE bit patterns
// sort as unsigned integers: a bitonic network on uint64 keys (LDS tiles of
// 2048 plus global merge steps) gives the ascending order.  Sums are
// double-double with a fixed combination order and are rounded once, so J
// is deterministic and equals the exact-arithmetic answer except within
// ~1e-30 relative of a tie.
#include <mutex>
#include <string>

#include "common.h"
#include "kernels.h"

namespace tsvdm {

namespace {

constexpr int LTILE = 2048;   // keys sorted per LDS tile
constexpr int LTHREADS = 512;

__device__ __forceinline__ unsigned long long key_of(double v) {
    if (!(v >= 0.0)) v = (v != v) ? __longlong_as_double(0x7ff0000000000000ll) : 0.0;  // NaN -> +inf, negatives -> 0
    v = v + 0.0;  // -0 -> +0
    return (unsigned long long)__double_as_longlong(v);
}

__global__ void sel_fill(const double* __restrict__ s2, int64_t N, int64_t Np,
                         unsigned long long* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Np) keys[i] = i < N ? key_of(s2[i]) : ~0ull;
}

__device__ __forceinline__ void cmp_swap(unsigned long long& a, unsigned long long& b, bool up) {
    if ((a > b) == up) { unsigned long long t = a; a = b; b = t; }
}

// Sort every LDS tile completely (k = 2 .. tile), or, with k_fixed > 0,
// finish the merge stage k_fixed for all strides j < tile.
__global__ __launch_bounds__(LTHREADS) void sel_bitonic_local(unsigned long long* __restrict__ keys,
                                                              int64_t Np, int tile, int64_t k_fixed) {
    __shared__ unsigned long long sk[LTILE];
    const int64_t base = (int64_t)blockIdx.x * tile;
    for (int i = threadIdx.x; i < tile; i += LTHREADS) sk[i] = keys[base + i];
    __syncthreads();
    const int64_t k_lo = k_fixed > 0 ? k_fixed : 2;
    const int64_t k_hi = k_fixed > 0 ? k_fixed : tile;
    for (int64_t k = k_lo; k <= k_hi; k <<= 1) {
        for (int64_t j = (k_fixed > 0 ? tile / 2 : k / 2); j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < tile / 2; t += LTHREADS) {
                const int64_t i = 2 * j * (t / j) + (t % j);  // lower index of the pair
                const int64_t gi = base + i;
                const bool up = (gi & k) == 0;
                cmp_swap(sk[i], sk[i + j], up);
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < tile; i += LTHREADS) keys[base + i] = sk[i];
}

__global__ void sel_bitonic_global(unsigned long long* __restrict__ keys, int64_t Np, int64_t k,
                                   int64_t j) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= Np / 2) return;
    const int64_t i = 2 * j * (t / j) + (t % j);
    const bool up = (i & k) == 0;
    unsigned long long a = keys[i], b = keys[i + j];
    if ((a > b) == up) { keys[i] = b; keys[i + j] = a; }
}

constexpr int STHREADS = 1024;

// Inclusive scan of the STHREADS double-double values (hi, lo) in LDS by
// the whole workgroup: entry t becomes x_0 + ... + x_t, in a fixed tree
// order (step d adds the entry d places earlier).
__device__ void dd_block_scan(double* hi, double* lo, int t) {
    for (int d = 1; d < STHREADS; d <<= 1) {
        const bool has = t >= d;
        dd u = {0.0, 0.0};
        if (has) u = dd{hi[t - d], lo[t - d]};
        const dd v = {hi[t], lo[t]};
        __syncthreads();
        if (has) {
            const dd w = dd_add(u, v);
            hi[t] = w.hi;
            lo[t] = w.lo;
        }
        __syncthreads();
    }
}

// Single-workgroup scan over the N sorted values (N <= a few million).
// Scan of N ascending keys by one workgroup of STHREADS threads, thread t
// owning the t-th contiguous segment; writes stats = {tau, discarded, W, J}.
__device__ void sel_scan_body(const unsigned long long* __restrict__ keys, int64_t N, double eps,
                              double* __restrict__ stats) {
    __shared__ double shi[STHREADS], slo[STHREADS];
    __shared__ unsigned long long J_acc;
    __shared__ double tau_s;
    const int t = threadIdx.x;
    const int64_t seg = (N + STHREADS - 1) / STHREADS;
    const int64_t b0 = (int64_t)t * seg;
    const int64_t b1 = (b0 + seg < N) ? b0 + seg : N;
    if (t == 0) J_acc = 0ull;

    // The segment loops load eight keys at a time and take them in order.
    auto key = [&](int64_t j) { return __longlong_as_double((long long)keys[j]); };

    // pass 1: segment sums, their prefix sums and the total W
    dd acc = {0.0, 0.0};
    int64_t j = b0;
    for (; j + 8 <= b1; j += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = key(j + q);
#pragma unroll
        for (int q = 0; q < 8; ++q) acc = dd_add_d(acc, v[q]);
    }
    for (; j < b1; ++j) acc = dd_add_d(acc, key(j));
    shi[t] = acc.hi; slo[t] = acc.lo;
    __syncthreads();
    dd_block_scan(shi, slo, t);
    const dd pre = t > 0 ? dd{shi[t - 1], slo[t - 1]} : dd{0.0, 0.0};   // sum of earlier segments
    const double W = dd_round(dd{shi[STHREADS - 1], slo[STHREADS - 1]});
    const double eps2 = eps * eps;

    // pass 2: J = #{ j : w_j / W < eps^2 }  (w is non-decreasing); an
    // integer count, so the order of the additions does not matter
    long long c = 0;
    bool go = W > 0.0;
    dd w = pre;
    for (j = b0; go && j + 8 <= b1; j += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = key(j + q);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (!go) break;
            w = dd_add_d(w, v[q]);
            if (dd_round(w) / W < eps2) ++c; else go = false;
        }
    }
    for (; go && j < b1; ++j) {
        w = dd_add_d(w, key(j));
        if (dd_round(w) / W < eps2) ++c; else go = false;
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((t & 63) == 0 && c != 0) atomicAdd(&J_acc, (unsigned long long)c);
    __syncthreads();
    const long long J = (long long)J_acc;
    if (t == 0) {
        double tau;
        if (W == 0.0) tau = 0.0;                         // zero tensor: drop everything
        else if (J == 0) tau = -__longlong_as_double(0x7ff0000000000000ll);  // keep everything
        else tau = __longlong_as_double((long long)keys[J - 1]);
        tau_s = tau;
    }
    __syncthreads();
    // pass 3: discarded energy = sum of values <= tau (segment sums, then
    // the same tree as pass 1)
    const double tau = tau_s;
    dd d = {0.0, 0.0};
    go = true;
    for (j = b0; go && j + 8 <= b1; j += 8) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = key(j + q);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (!go) break;
            if (v[q] <= tau) d = dd_add_d(d, v[q]); else go = false;
        }
    }
    for (; go && j < b1; ++j) {
        const double v = key(j);
        if (v <= tau) d = dd_add_d(d, v); else go = false;
    }
    shi[t] = d.hi; slo[t] = d.lo;
    __syncthreads();
    dd_block_scan(shi, slo, t);
    if (t == 0) {
        stats[0] = tau;
        stats[1] = dd_round(dd{shi[STHREADS - 1], slo[STHREADS - 1]});
        stats[2] = W;
        stats[3] = (double)J;
    }
    __syncthreads();
}

__global__ __launch_bounds__(STHREADS) void sel_scan(const unsigned long long* __restrict__ keys,
                                                     int64_t N, double eps, double* __restrict__ stats) {
    sel_scan_body(keys, N, eps, stats);
}

// Batched selection, one workgroup per tensor: t-SVDM-I writes the fixed
// ranks; t-SVDM-II sorts the tensor's squared values with a bitonic network
// in its global scratch, scans them and counts per slice.
__global__ __launch_bounds__(STHREADS) void sel_batch(const SelTensor* __restrict__ jobs) {
    const SelTensor j = jobs[blockIdx.x];
    const int t = threadIdx.x;
    const int64_t r = j.r, n = j.n;
    if (j.mode == 1) {
        const int64_t kk = j.k < r ? j.k : r;
        for (int64_t i = t; i < n; i += STHREADS) j.rho[i] = (int32_t)kk;
        for (int64_t i = t; i <= n; i += STHREADS) j.offsets[i] = i * kk;
        return;
    }
    const int64_t N = r * n, Np = j.np2;
    unsigned long long* keys = j.keys;
    for (int64_t i = t; i < Np; i += STHREADS) keys[i] = i < N ? key_of(j.s2[i]) : ~0ull;
    __syncthreads();
    for (int64_t k = 2; k <= Np; k <<= 1) {
        for (int64_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (int64_t q = t; q < Np / 2; q += STHREADS) {
                const int64_t i = 2 * jj * (q / jj) + (q % jj);
                const bool up = (i & k) == 0;
                const unsigned long long a = keys[i], b = keys[i + jj];
                if ((a > b) == up) { keys[i] = b; keys[i + jj] = a; }
            }
            __syncthreads();
        }
    }
    sel_scan_body(keys, N, j.eps, j.stats);
    const double tau = j.stats[0];
    for (int64_t i = t; i < n; i += STHREADS) {
        int c = 0;
        for (int64_t q = 0; q < r; ++q) c += (j.s2[i * r + q] > tau) ? 1 : 0;
        j.rho[i] = c;
    }
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int64_t i = 0; i < n; ++i) { j.offsets[i] = run; run += j.rho[i]; }
        j.offsets[n] = run;
    }
}

__global__ void sel_rank(const double* __restrict__ s2, int64_t r, int64_t n,
                         const double* __restrict__ stats, int32_t* __restrict__ rho) {
    const int64_t i = blockIdx.x;  // slice
    if (i >= n) return;
    const double tau = stats[0];
    int c = 0;
    for (int64_t j = threadIdx.x; j < r; j += blockDim.x) c += (s2[i * r + j] > tau) ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    __shared__ int part[16];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += part[w];
        rho[i] = tot;
    }
}

// offsets[i] = sum_{j < i} rho[j], offsets[n] = total (single workgroup)
__global__ __launch_bounds__(1024) void sel_offsets(const int32_t* __restrict__ rho, int64_t n,
                                                    int64_t* __restrict__ offsets) {
    __shared__ long long part[1024];
    const int t = threadIdx.x;
    const int64_t seg = (n + 1023) / 1024;
    const int64_t b0 = (int64_t)t * seg, b1 = (b0 + seg < n) ? b0 + seg : n;
    long long s = 0;
    for (int64_t i = b0; i < b1; ++i) s += rho[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        long long run = 0;
        for (int i = 0; i < 1024; ++i) { long long v = part[i]; part[i] = run; run += v; }
        offsets[n] = run;
    }
    __syncthreads();
    long long run = part[t];
    for (int64_t i = b0; i < b1; ++i) { offsets[i] = run; run += rho[i]; }
}

__global__ void sel_fixed(int64_t kk, int64_t n, int32_t* __restrict__ rho,
                          int64_t* __restrict__ offsets) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rho[i] = (int32_t)kk;
    if (i <= n) offsets[i] = i * kk;
}

int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

size_t select_workspace_bytes(int64_t r, int64_t n) {
    Carver cv(nullptr);
    cv.carve<unsigned long long>((size_t)next_pow2(r * n < 2 ? 2 : r * n));
    return cv.total();
}

int run_truncate_tol(const double* s2, int64_t r, int64_t n, double eps, int32_t* rho,
                     int64_t* offsets, double* stats, void* ws, hipStream_t st) {
    const int64_t N = r * n;
    const int64_t Np = next_pow2(N < 2 ? 2 : N);
    Carver cv(ws);
    unsigned long long* keys = cv.carve<unsigned long long>((size_t)Np);
    sel_fill<<<(unsigned)((Np + 255) / 256), 256, 0, st>>>(s2, N, Np, keys);
    TSVDM_LAUNCH_CHECK();
    const int tile = (int)(Np < LTILE ? Np : LTILE);
    sel_bitonic_local<<<(unsigned)(Np / tile), LTHREADS, 0, st>>>(keys, Np, tile, 0);
    TSVDM_LAUNCH_CHECK();
    for (int64_t k = 2 * (int64_t)tile; k <= Np; k <<= 1) {
        for (int64_t j = k / 2; j >= tile; j >>= 1) {
            sel_bitonic_global<<<(unsigned)((Np / 2 + 255) / 256), 256, 0, st>>>(keys, Np, k, j);
            TSVDM_LAUNCH_CHECK();
        }
        sel_bitonic_local<<<(unsigned)(Np / tile), LTHREADS, 0, st>>>(keys, Np, tile, k);
        TSVDM_LAUNCH_CHECK();
    }
    sel_scan<<<1, STHREADS, 0, st>>>(keys, N, eps, stats);
    TSVDM_LAUNCH_CHECK();
    sel_rank<<<(unsigned)n, 256, 0, st>>>(s2, r, n, stats, rho);
    TSVDM_LAUNCH_CHECK();
    sel_offsets<<<1, 1024, 0, st>>>(rho, n, offsets);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

// Selection without allocation: the sort keys live in a fixed device array
// (8 MiB, 2^20 keys) that every call on a GPU shares.  sel_fill rewrites all
// the keys a call uses (padding included), so nothing needs clearing between
// calls; calls that overlap on one GPU race on the array.
constexpr int64_t STATIC_SELECT_KEYS = (int64_t)1 << 20;
static __device__ __align__(256) unsigned long long scratch[STATIC_SELECT_KEYS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

int64_t static_select_max_keys() { return STATIC_SELECT_KEYS; }

int run_truncate_tol_static(const double* s2, int64_t r, int64_t n, double eps, int32_t* rho,
                            int64_t* offsets, double* stats, hipStream_t st) {
    if (next_pow2(r * n < 2 ? 2 : r * n) > STATIC_SELECT_KEYS) {
        set_error("r*n = " + std::to_string(r * n) + " exceeds the fixed selection scratch (" +
                  std::to_string(STATIC_SELECT_KEYS) + " keys)");
        return TSVDM_E_SHAPE;
    }
    int dev = 0;
    TSVDM_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device ordinal out of range for the fixed selection scratch");
        return TSVDM_E_ARG;
    }
    void* ptr = nullptr;
    {
        // once per device, with that device current: the device address of
        // this GPU's copy of the array (the host symbol is not an address)
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            TSVDM_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            g_scratch_ptr[dev] = p;
        }
        ptr = g_scratch_ptr[dev];
    }
    return run_truncate_tol(s2, r, n, eps, rho, offsets, stats, ptr, st);
}

int run_truncate_rank(int64_t k, int64_t r, int64_t n, int32_t* rho, int64_t* offsets,
                      hipStream_t st) {
    const int64_t kk = k < r ? k : r;
    sel_fixed<<<(unsigned)((n + 1 + 255) / 256), 256, 0, st>>>(kk, n, rho, offsets);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_select_batch(const SelTensor* jobs, int ntensors, hipStream_t st) {
    sel_batch<<<(unsigned)ntensors, STHREADS, 0, st>>>(jobs);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int64_t select_np2(int64_t N) { return next_pow2(N < 2 ? 2 : N); }

}  // namespace tsvdm

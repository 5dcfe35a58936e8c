// Slice-wise SVD by one-sided block Jacobi (Algorithm 1's per-slice SVD;
// Section 3.2 "parallel slices" design carried to the GPU).
//
// Each frontal slice contributes r = min(m, p) vectors of length L = max(m, p)
// (columns if m >= p, rows otherwise).  The r vectors are split into blocks of
// b = NB2/2 and a sweep pairs every two blocks once, using the circle
// (round-robin) tournament so that the nb/2 pairs of one round are disjoint
// and run as independent workgroups.  For a pair the workgroup
//   1. forms the NB2 x NB2 Gram matrix H of its vectors on MFMA,
//   2. measures max |cos| between its vectors from H (FP64) and, if that is
//      above tol, diagonalises H with one cyclic Jacobi sweep in FP64 (LDS),
//   3. applies the accumulated rotation Q to its vectors and to the matching
//      columns of W on MFMA:  vectors <- Q^T vectors,  W <- W Q.
// Vectors stay at their positions (no reordering inside a pair), which keeps
// the tournament's pair coverage intact.  A slice is converged once a whole
// sweep saw max |cos| <= tol; later rounds return at once for it.
#include <mutex>
#include <type_traits>
#include <vector>

#include "angle.h"
#include "common.h"
#include "kernels.h"

namespace tsvdm {

// ---------------------------------------------------------------- statistics
namespace {
std::mutex g_stats_mu;
bool g_stats_on = false;
int64_t g_launches = 0, g_pairs_gram = 0, g_pairs_rot = 0;
double g_ms = 0.0, g_flops = 0.0, g_bytes = 0.0;
int g_width = 0;
}  // namespace

bool stats_enabled() {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    return g_stats_on;
}
void stats_set(bool on) {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    g_stats_on = on;
}
void stats_reset() {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    g_launches = g_pairs_gram = g_pairs_rot = 0;
    g_ms = g_flops = g_bytes = 0.0;
}
// counters: {gram-only pairs, rotating pairs, flops, bytes} as read back
static void stats_add_counters(int64_t launches, double ms, const unsigned long long* c, int width) {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    g_launches += launches;
    g_ms += ms;
    g_pairs_gram += (int64_t)c[0];
    g_pairs_rot += (int64_t)c[1];
    g_flops += (double)c[2];
    g_bytes += (double)c[3];
    g_width = width;
}
// a kernel timed by its caller (no pair counters): the in-LDS Jacobi
void stats_add_launch(int64_t launches, double ms) {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    g_launches += launches;
    g_ms += ms;
    g_width = 0;
}
void stats_get(int64_t* launches, double* ms, int64_t* pg, int64_t* pr, int32_t* width,
               double* flops, double* bytes) {
    std::lock_guard<std::mutex> lk(g_stats_mu);
    if (launches) *launches = g_launches;
    if (ms) *ms = g_ms;
    if (pg) *pg = g_pairs_gram;
    if (pr) *pr = g_pairs_rot;
    if (width) *width = g_width;
    if (flops) *flops = g_flops;
    if (bytes) *bytes = g_bytes;
}

namespace {

// Pair statistics (gram-only pairs, rotating pairs, flops, bytes) are summed
// into PC_BINS bins one 128-byte line apart, bin = workgroup index mod
// PC_BINS: a single set of counters, hit by every workgroup of a launch,
// serialised the atomics and took a quarter of a launch of short pairs.
// They are kept only while statistics are switched on.
constexpr int PC_BINS = 64, PC_STRIDE = 16;
constexpr int PC_WORDS = PC_BINS * PC_STRIDE;

// Skipping pairs found orthogonal whose blocks have not changed since.
// Per slice, trk[0, nbe) counts the rotations that changed each block, and
// trk[nbe + 2 q], trk[nbe + 2 q + 1] hold the two blocks' counts when pair q
// (blocks lo < hi, q = hi (hi - 1) / 2 + lo) last measured every cosine <=
// tol (-1: never).  A pair whose counts still match has the same vectors,
// so the same Gram matrix and the same outcome (no rotation): it returns at
// once.  nbe^2 words per slice.
__device__ __forceinline__ int track_pair(int lo, int hi) { return hi * (hi - 1) / 2 + lo; }

// sum the bins of a copied counter block
void pc_sum(const unsigned long long* bins, unsigned long long* out) {
    for (int k = 0; k < 4; ++k) out[k] = 0ull;
    for (int b = 0; b < PC_BINS; ++b)
        for (int k = 0; k < 4; ++k) out[k] += bins[b * PC_STRIDE + k];
}

__device__ __forceinline__ int circle_player(int seat, int round, int N) {
    return seat == 0 ? 0 : ((seat - 1 + round) % (N - 1)) + 1;
}

// Inner sweep orderings over the NB2 vectors of a block pair, in seat
// order: pair k always sits on seats (k, partner_seat(k)) and the vectors
// move between seats after every step.  Full sweep: circle tournament, seat
// k meets seat NB2-1-k, seat 0 fixed, the others advance one seat (the
// vector on seat j >= 2 moves to j-1, seat 1 to NB2-1).  Cross sweep (both
// blocks already orthogonal inside): seat k (vector k of the first block)
// meets seat b+k, the second block's vectors advance cyclically.
template <int NB2>
__device__ __forceinline__ int partner_seat(bool cross, int k) {
    return cross ? NB2 / 2 + k : NB2 - 1 - k;
}
// seat after one step of the vector on seat j
template <int NB2>
__device__ __forceinline__ int next_seat(bool cross, int j) {
    constexpr int B = NB2 / 2;
    if (cross) return j < B ? j : (j == B ? NB2 - 1 : j - 1);
    return j == 0 ? 0 : (j == 1 ? NB2 - 1 : j - 1);
}
// seat one step earlier of the vector on seat j
template <int NB2>
__device__ __forceinline__ int prev_seat(bool cross, int j) {
    constexpr int B = NB2 / 2;
    if (cross) return j < B ? j : (j == NB2 - 1 ? B : j + 1);
    return j == 0 ? 0 : (j == NB2 - 1 ? 1 : j + 1);
}
// pair on seat j and whether j is its first seat
template <int NB2>
__device__ __forceinline__ int seat_pair(bool cross, int j, bool& first) {
    constexpr int B = NB2 / 2;
    first = j < B;
    return first ? j : (cross ? j - B : NB2 - 1 - j);
}

// Packed symmetric storage of the pair Gram matrix: (a, b) and (b, a) share
// one slot.
__device__ __forceinline__ int sym_idx(int a, int b) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return hi * (hi + 1) / 2 + lo;
}

// W = I and a clean control word per slice; slices outside `run` (when
// given) keep their W and start as done, so no round touches them.
template <class T>
__global__ void jacobi_init(T* __restrict__ W, int64_t r, int64_t n, JacobiCtl* __restrict__ ctl,
                            int* __restrict__ remaining, int max_sweeps,
                            unsigned long long* __restrict__ pair_counts,
                            int32_t* __restrict__ status, const int32_t* __restrict__ run,
                            int32_t* __restrict__ track, int nbe) {
    // W = I: workgroups take whole columns (one index division per column),
    // threads run down the column
    const int64_t cols = W ? r * n : 0;   // W == nullptr: no accumulated rotations
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t col = blockIdx.x; col < cols; col += gridDim.x) {
        const int64_t s = col / r, c = col - s * r;
        if (run && !run[s]) continue;
        T* const w = W + col * r;
        for (int64_t row = threadIdx.x; row < r; row += blockDim.x) w[row] = (row == c) ? T(1) : T(0);
    }
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += stride) {
        JacobiCtl c;
        c.maxcos_bits = 0ull; c.done = (run && !run[idx]) ? 1 : 0; c.sweeps = 0; c.nonfinite = 0; c.pad = 0;
        ctl[idx] = c;
    }
    // pair records: every block unchanged (0), no pair found orthogonal yet
    const int64_t tw = (int64_t)nbe * nbe;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n * tw; idx += stride)
        track[idx] = idx % tw < nbe ? 0 : -1;
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < max_sweeps; i += blockDim.x) remaining[i] = 0;
        for (int i = threadIdx.x; i < PC_WORDS; i += blockDim.x) pair_counts[i] = 0ull;
        if (threadIdx.x == 0) *status = TSVDM_OK;
    }
}

// Shared-memory layout of one pair.  Both MFMA phases stream the L
// positions in tiles of PT, each wave through its own staging region of STG
// elements (enough for either phase's layout).  The pair Gram matrix H
// lives in the same region afterwards as two packed symmetric buffers (one
// per parity of the inner step; FP32 for FP32 vectors, which keeps a
// workgroup under 40 KB so that four share a compute unit, FP64 otherwise);
// while the first is being written, the
// partial sums of every Gram tile from the three waves that do not own it
// sit right behind it.  Q is stored
// transposed (row a =
// column a of Q) with the 16-byte groups of row a XOR-swizzled by a, so that
// row accesses are 16-byte vectors and column reads of 16 rows hit distinct
// banks.
template <class T, int NB2>
struct RoundCfg {
    static constexpr int VW = 16 / sizeof(T);                  // elements per 16-byte access
    static constexpr int PT = 16;                              // positions per tile
    static constexpr int STG = PT * (NB2 + 16);                // staging elements per wave
    static constexpr int NT = NB2 / 16;                        // 16x16 tiles per dimension
    static constexpr int NPH = NB2 / 2;                        // rotations per inner step
    static constexpr int NH = NB2 * (NB2 + 1) / 2;             // packed symmetric H
    static constexpr int SWM = (NB2 / VW < 16 ? NB2 / VW : 16) - 1;  // Q swizzle mask
    // storage type of H between the steps of the inner sweep (the
    // arithmetic on it is FP64 either way)
    typedef typename std::conditional<sizeof(T) == 4, float, double>::type HT;
    static constexpr size_t stg_bytes = sizeof(T) * 4 * STG;
    static constexpr size_t hs_bytes = sizeof(HT) * 2 * NH;
    static constexpr size_t r1 = (stg_bytes > hs_bytes) ? stg_bytes : hs_bytes;
    static constexpr size_t q_bytes = sizeof(T) * NB2 * NB2;
    // three partial sums per Gram tile, parked behind the first H buffer
    static constexpr int NTT = NT * (NT + 1) / 2;
    static constexpr size_t rp_off = (sizeof(HT) * NH + 15) / 16 * 16;
    static constexpr size_t rp_end = rp_off + sizeof(T) * 3 * NTT * 256;
    static constexpr size_t total = (r1 + q_bytes > rp_end) ? r1 + q_bytes : rp_end;
    // LDS of one workgroup (the region above plus the rotations and the
    // reductions, in 512-byte allocation units) and the waves per SIMD the
    // kernel is compiled for: three workgroups per compute unit when the LDS
    // allows it, else two; four for the FP32 pairs of 64 vectors
    // (OCC4 below)
    static constexpr size_t lds_bytes = ((total + 15) / 16 * 16 + NB2 * 16 + 80 + 511) / 512 * 512;
    static constexpr int WAVES = (3 * lds_bytes <= 160 * 1024) ? 3 : 2;
    // Q^T[a][c] = Q[c][a]
    static __device__ __forceinline__ int q_idx(int a, int c) { return a * NB2 + (c ^ ((a & SWM) * VW)); }
};

// FP32 pairs of 64 vectors run four workgroups per compute unit: their
// 40 KB of LDS allow it, and with Q read from LDS in the vector update and
// one H block in registers at a time in the inner sweep the interior
// instances fit the 128 registers a lane then has.  The instances with
// checked loads spill a few registers at that budget and still gain from
// the fourth workgroup.
template <class T, int NB2>
struct RoundOcc {
    static constexpr bool OCC4 = sizeof(T) == 4 && NB2 == 64;
    static constexpr int WAVES = OCC4 ? 4 : RoundCfg<T, NB2>::WAVES;
};

// (c, s) of one rotation as the vectors see it: the angle is computed in
// FP64 and rounded to the working precision, and H is rotated in FP64 with
// the same rounded pair (kept as exact doubles), so that H stays the Gram
// matrix of the vectors the rotations actually produce, up to the rounding
// of its storage (FP32 for FP32 vectors, whose own rounding is as large).
template <class T>
__device__ __forceinline__ double2 rot_make(double c, double s) {
    return make_double2((double)(T)c, (double)(T)s);
}

template <class T, int NB2>
struct RoundShared {
    __align__(16) char smem[RoundCfg<T, NB2>::total];
    double2 rot_cs[2][NB2 / 2];   // (c, s) of each rotation, per parity of the inner step
    double red_mx[4], red_mw[4];  // per-wave convergence measure: across / inside the blocks
    int red_nf[4];                // per-wave: a NaN or Inf was met
};

// INT: every pair of the slice is interior (r a multiple of b with an even
// block count, 16-byte aligned vectors and W columns, L and r multiples of
// the tile), so that the MFMA phases need no checked loads or stores.
template <class T, int NB2, bool ROWS, bool INT = false>
__device__ __forceinline__ void round_body(RoundShared<T, NB2>& sh, T* __restrict__ Ab,
                                           T* __restrict__ Wb, const SliceGeom& g, int nbe, int rnd,
                                           int k, JacobiCtl* __restrict__ ctl_s, double tol,
                                           int vec_a, int vec_w,
                                           unsigned long long* __restrict__ pair_counts,
                                           int32_t* __restrict__ trk) {
    typedef RoundCfg<T, NB2> C;
    typedef typename Acc<T>::type AccT;
    constexpr int B = NB2 / 2, VW = C::VW;
    constexpr int NT = C::NT, NH = C::NH;

    char* smem = sh.smem;

    T* Ts = reinterpret_cast<T*>(smem);                           // [4][STG] per-wave staging
    typedef typename C::HT HT;
    HT* H0 = reinterpret_cast<HT*>(smem);                         // [2][NH] packed H (phase 2)
    T* Qs = reinterpret_cast<T*>(smem + C::r1);                   // [NB2][NB2] Q^T, swizzled

    const int I = circle_player(k, rnd, nbe);
    const int J = circle_player(nbe - 1 - k, rnd, nbe);
    const int64_t r = g.r, L = g.L;
    // unchanged since this pair found its vectors orthogonal: nothing to do
    const int blo = I < J ? I : J, bhi = I < J ? J : I;
    int32_t* const trk_pair = trk + nbe + 2 * track_pair(blo, bhi);
    const int32_t ver_lo = trk[blo], ver_hi = trk[bhi];
    if (trk_pair[0] == ver_lo && trk_pair[1] == ver_hi) return;   // uniform across the block

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;

    auto gidx = [&](int a) -> int64_t { return a < B ? (int64_t)I * B + a : (int64_t)J * B + (a - B); };

    // ---- position tiles.  Wave w takes the tiles w, w + 4, ... of PT
    // positions, loads the 2b values of a tile into registers one tile
    // ahead, stages them in its own LDS region and runs its MFMAs from there,
    // so the waves of one phase never wait for each other.  Load u of a lane
    // covers VW consecutive elements along the contiguous direction: the
    // positions for column families, the vector index for row families (a
    // block of b rows is contiguous, b % VW == 0).
    constexpr int PT = C::PT;
    constexpr int NA = NB2 * PT / (VW * 64);                  // 16-byte loads per lane and tile
    T* const stg = Ts + wave * C::STG;
    T pre[NA][VW];
    // (vector c, position tt) of the first element of load u
    auto origin = [&](bool rw, int u, int& c, int& tt) {
        const int e = lane + 64 * u;
        if (!rw) { c = e / (PT / VW); tt = (e % (PT / VW)) * VW; }
        else { c = (e % (NB2 / VW)) * VW; tt = e / (NB2 / VW); }
    };
    auto load_tile = [&](bool rw, const T* base, int64_t vs, int64_t es, int64_t len, bool vec,
                         int64_t t0) {
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            int c, tt;
            origin(rw, u, c, tt);
            const int64_t gi = gidx(c), t = t0 + tt;
            const bool full = rw ? (t < len && vec && gi + VW <= r) : (gi < r && vec && t + VW <= len);
            const T* src = rw ? base + gi + t * es : base + gi * vs + t;
            if (full) {
                if constexpr (sizeof(T) == 4) {
                    const float4 x = *reinterpret_cast<const float4*>(src);
                    pre[u][0] = x.x; pre[u][1] = x.y; pre[u][2] = x.z; pre[u][3] = x.w;
                } else {
                    const double2 x = *reinterpret_cast<const double2*>(src);
                    pre[u][0] = x.x; pre[u][1] = x.y;
                }
            } else {
#pragma unroll
                for (int q = 0; q < VW; ++q) {
                    const bool ok = rw ? (t < len && gi + q < r) : (gi < r && t + q < len);
                    pre[u][q] = ok ? src[q] : T(0);
                }
            }
        }
    };

    // ---------------- phase 1: Gram matrix H of the pair (MFMA)
    // Each wave sums its own tiles into a partial Gram matrix, forming only
    // the NT (NT + 1) / 2 tiles on and above the diagonal from NT operand
    // fragments per four positions.  Staging rows are padded so that the
    // fragment reads of each half wave (a quarter wave for FP64) hit the 32
    // LDS banks once: column families keep one vector per row of PT + 2
    // (FP64: PT + 1) elements, row families one position per row of NB2 + 16.
    // Each MFMA sums four consecutive positions (summing positions in a
    // strided order within one MFMA was measured to leave the FP32 results
    // several times further from the FP64 ones on smooth inputs).
    constexpr int NTT = C::NTT;
    constexpr int GPC = PT + (sizeof(T) == 4 ? 2 : 1), GPR = NB2 + 16;
    AccT hacc[NTT];
#pragma unroll
    for (int q = 0; q < NTT; ++q) hacc[q] = zero4<AccT>();
    {
        const int64_t ntile = (L + PT - 1) / PT;
        // stage a tile from registers into the wave's LDS region
        auto stage = [&](T (&cur)[NA][VW]) {
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                int c, tt;
                origin(ROWS, u, c, tt);
                if (ROWS) {
                    T* const dst = stg + tt * GPR + c;
                    if constexpr (sizeof(T) == 4)
                        *reinterpret_cast<float4*>(dst) = make_float4(cur[u][0], cur[u][1], cur[u][2], cur[u][3]);
                    else
                        *reinterpret_cast<double2*>(dst) = make_double2(cur[u][0], cur[u][1]);
                } else {
                    // rows of PT + 2 floats are 8-byte aligned only
                    T* const dst = stg + c * GPC + tt;
                    if constexpr (sizeof(T) == 4) {
                        *reinterpret_cast<float2*>(dst) = make_float2(cur[u][0], cur[u][1]);
                        *reinterpret_cast<float2*>(dst + 2) = make_float2(cur[u][2], cur[u][3]);
                    } else {
                        dst[0] = cur[u][0];
                        dst[1] = cur[u][1];
                    }
                }
            }
            // the wave's own LDS stores before its reads (LDS is in order per wave)
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        };
        auto gram_mfma = [&]() {
#pragma unroll
            for (int kk = 0; kk < PT; kk += 4) {
                T f[NT];
#pragma unroll
                for (int i = 0; i < NT; ++i)
                    f[i] = ROWS ? stg[(kk + lg) * GPR + 16 * i + lr] : stg[(16 * i + lr) * GPC + kk + lg];
                int q = 0;
#pragma unroll
                for (int i = 0; i < NT; ++i) {
#pragma unroll
                    for (int j = i; j < NT; ++j, ++q) hacc[q] = mfma(f[i], f[j], hacc[q]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        };
        int64_t tile = wave;
        // Interior tiles of a pair of whole, 16-byte aligned blocks run a
        // branch-free pipeline with two tiles in flight per wave: exactly NA
        // unchecked 16-byte loads per tile (the prefetch index is clamped to
        // the last interior tile, whose extra loads hit L2), so that the wait
        // for a tile counts only the loads issued after it.
        const int64_t nint = (INT || ((int64_t)I * B + B <= r && (int64_t)J * B + B <= r && vec_a != 0)) ? L / PT : 0;
        if (tile < nint) {
            auto fast = [&](T (&dst)[NA][VW], int64_t tl) {
                const int64_t t0 = (tl < nint ? tl : nint - 1) * PT;
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    int c, tt;
                    origin(ROWS, u, c, tt);
                    const int64_t gi = gidx(c), t = t0 + tt;
                    const T* src = ROWS ? Ab + gi + t * g.es : Ab + gi * g.vs + t;
                    if constexpr (sizeof(T) == 4) {
                        const float4 x = *reinterpret_cast<const float4*>(src);
                        dst[u][0] = x.x; dst[u][1] = x.y; dst[u][2] = x.z; dst[u][3] = x.w;
                    } else {
                        const double2 x = *reinterpret_cast<const double2*>(src);
                        dst[u][0] = x.x; dst[u][1] = x.y;
                    }
                }
            };
            T pre2[NA][VW];
            fast(pre, tile);
            fast(pre2, tile + 4);
            for (; tile + 4 < nint; tile += 8) {
                stage(pre);
                fast(pre, tile + 8);
                __builtin_amdgcn_sched_barrier(0);   // loads ahead of the MFMAs
                gram_mfma();
                stage(pre2);
                fast(pre2, tile + 12);
                __builtin_amdgcn_sched_barrier(0);
                gram_mfma();
            }
            if (tile < nint) {
                stage(pre);
                gram_mfma();
                tile += 4;
            }
        }
        // the rest (a partial last tile, or every tile of a pair with a
        // partial block): checked loads, one tile ahead
        if constexpr (!INT) {
            if (tile < ntile) load_tile(ROWS, Ab, g.vs, g.es, L, vec_a != 0, tile * PT);
            for (; tile < ntile; tile += 4) {
                stage(pre);
                if (tile + 4 < ntile) load_tile(ROWS, Ab, g.vs, g.es, L, vec_a != 0, (tile + 4) * PT);
                gram_mfma();
            }
        }
    }
    // Tile q of the Gram matrix belongs to wave q % 4.  Every wave parks its
    // partial sums of the tiles it does not own in LDS in lane order (over
    // the staging regions, hence the barrier first, and clear of the H
    // buffer the owners fill while others still read them); each owner adds
    // the four partials of its tiles in wave order 0..3, so the result does
    // not depend on timing, writes them into the packed H and, once
    // every diagonal is there, forms the convergence measure of its tiles:
    // the largest |cos| = |h_ac| / (||a|| ||c||) over valid vector pairs,
    // kept separately for pairs inside one block and pairs across the two
    // blocks.  The four per-wave maxima meet in LDS.
    T* const Rp = reinterpret_cast<T*>(smem + C::rp_off);         // [NTT][3][4][64]
    auto slot = [&](int q, int w) {                               // w != q % 4
        const int o = q & 3;
        const int k = w - (w > o ? 1 : 0);
        return Rp + (q * 3 + (k < 2 ? k : 2)) * 256;
    };
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NTT; ++q) {
        if ((q & 3) == wave) continue;
        T* const Rw = slot(q, wave);
#pragma unroll
        for (int v = 0; v < 4; ++v) Rw[v * 64 + lane] = hacc[q][v];
    }
    __syncthreads();
    {
        int q = 0;
#pragma unroll
        for (int i = 0; i < NT; ++i) {
#pragma unroll
            for (int j = i; j < NT; ++j, ++q) {
                if ((q & 3) != wave) continue;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int a = i * 16 + mfma_row<T>(lg, v), c = j * 16 + lr;
                    double h = 0.0;
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        const double x = (w == wave) ? (double)hacc[q][v] : (double)slot(q, w)[v * 64 + lane];
                        h = (w == 0) ? x : h + x;
                    }
                    if (a <= c) H0[sym_idx(a, c)] = h;
                }
            }
        }
    }
    __syncthreads();
    {
        // 1 / ||vector a||, 0 for padding and zero vectors so they never
        // count; norms below 2^-500 are scaled by a power of two first
        auto rnorm = [&](int a) -> double {
            const double d = H0[sym_idx(a, a)];
            const bool tiny = d < 0x1p-1000;
            const double y = rsq_nr(tiny ? d * 0x1p1000 : d) * (tiny ? 0x1p500 : 1.0);
            return (gidx(a) < r && d > 0.0) ? y : 0.0;
        };
        double mx = 0.0, mw = 0.0;
        bool nf = false;
        int q = 0;
#pragma unroll
        for (int i = 0; i < NT; ++i) {
#pragma unroll
            for (int j = i; j < NT; ++j, ++q) {
                if ((q & 3) != wave) continue;
                const double rc = rnorm(j * 16 + lr);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int a = i * 16 + mfma_row<T>(lg, v), c = j * 16 + lr;
                    const double h = H0[sym_idx(a, c)];
                    nf = nf || (a <= c && !isfinite(h));
                    const double cs = (a < c) ? fabs(h) * rnorm(a) * rc : 0.0;
                    if ((a < B) != (c < B)) mx = fmax(mx, cs);
                    else mw = fmax(mw, cs);
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            mx = fmax(mx, __shfl_xor(mx, off));
            mw = fmax(mw, __shfl_xor(mw, off));
        }
        const bool any_nf = __any(nf);
        if (lane == 0) { sh.red_mx[wave] = mx; sh.red_mw[wave] = mw; sh.red_nf[wave] = any_nf ? 1 : 0; }
    }
    __syncthreads();
    const double mcx = fmax(fmax(sh.red_mx[0], sh.red_mx[1]), fmax(sh.red_mx[2], sh.red_mx[3]));
    const double mcw = fmax(fmax(sh.red_mw[0], sh.red_mw[1]), fmax(sh.red_mw[2], sh.red_mw[3]));
    const double mc = fmax(mcx, mcw);
    const bool nonfinite = (sh.red_nf[0] | sh.red_nf[1] | sh.red_nf[2] | sh.red_nf[3]) != 0;
    const bool rotate = !nonfinite && (mc > tol);
    // A sweep over the b*b cross pairs only (b steps of b disjoint rotations
    // instead of 2b-1 steps) when both blocks are orthogonal inside, or, in
    // slices of at least 12 blocks, when their largest inside cosine is
    // below the largest cross cosine: a threshold strategy that leaves the
    // smaller inside pairs to a later meeting of the block.  Convergence is
    // still declared only when every cosine of a sweep is below tol.  With
    // many blocks a block meets enough others per sweep that this removes
    // 40-45% of the inner steps at the same sweep count (Gaussian and
    // low-rank-plus-noise slices, 13-16 blocks); with 5-8 blocks it costs
    // one or two more sweeps, which outweighs the saving.
    const bool cross_only = !(mcw > tol) || (nbe >= 12 && mcw < mcx);
    if (tid == 0) {
        if (nonfinite) atomicExch(&ctl_s->nonfinite, 1);
        else atomicMax(&ctl_s->maxcos_bits, (unsigned long long)__double_as_longlong(mc));
        // algorithmic work of this pair over its w valid vectors: Gram
        // 2 w^2 L flops and w L elements read; rotation 2 w^2 (L + r) flops
        // and 2 w (L + r) elements read and written
        const int64_t nI = (int64_t)I * B < r ? ((int64_t)I * B + B <= r ? B : r - (int64_t)I * B) : 0;
        const int64_t nJ = (int64_t)J * B < r ? ((int64_t)J * B + B <= r ? B : r - (int64_t)J * B) : 0;
        const unsigned long long w = (unsigned long long)(nI + nJ);
        unsigned long long fl = 2ull * w * w * (unsigned long long)L;
        unsigned long long by = w * (unsigned long long)L * sizeof(T);
        if (rotate) {
            const unsigned long long lw = (unsigned long long)(Wb ? L + r : L);   // no W: vectors only
            fl += 2ull * w * w * lw;
            by += 2ull * w * lw * sizeof(T);
        }
        if (pair_counts) {
            unsigned long long* const pc = pair_counts + (blockIdx.x % PC_BINS) * PC_STRIDE;
            atomicAdd(&pc[rotate ? 1 : 0], 1ull);
            atomicAdd(&pc[2], fl);
            atomicAdd(&pc[3], by);
        }
    }
    if (!rotate) {   // uniform across the block
        if (!nonfinite && tid == 0) {
            trk_pair[0] = ver_lo;
            trk_pair[1] = ver_hi;
        }
        return;
    }
    // FP64: the first vector tile of the update is in flight during the
    // inner sweep (FP32 has no registers to spare there)
    constexpr bool EARLY = sizeof(T) == 8;
    if (EARLY && wave < (L + PT - 1) / PT) load_tile(ROWS, Ab, g.vs, g.es, L, vec_a != 0, wave * PT);

    // ---------------- phase 2: one cyclic Jacobi sweep on H (FP64 angles)
    // H is kept in seat order (pair k on seats (k, partner_seat(k)) at every
    // step), double-buffered: step s reads buffer s&1 and writes
    // H_{s+1} = J_s^T H_s J_s into the other buffer, each element already on
    // the seats its vectors take at step s+1.  Every LDS index of the sweep is
    // therefore fixed per thread, and one barrier per step suffices.  The last
    // NPH threads compute the rotations of step s+1 meanwhile: the three
    // entries of H_{s+1} they need follow from H_s and the rotations of step
    // s.  The other threads rotate the 2x2 seat blocks (k1 <= k2); every thread
    // rotates a segment of two rows of Q^T (rows in vector order).  Padding
    // vectors are zero, so their rotations are the identity.
    constexpr int NPH = C::NPH;
    constexpr int NBT = 192;                           // threads rotating H blocks (waves 0-2)
    constexpr int NBLK = NPH * (NPH + 1) / 2;
    constexpr int HB = (NBLK + NBT - 1) / NBT;
    constexpr int TPP = 256 / NPH;                     // threads per Q row pair
    constexpr int EPT = NB2 / TPP;                     // Q entries per thread and row
    constexpr int GW = EPT < VW ? EPT : VW;            // Q entries per LDS access
    constexpr int NG = EPT / GW;                       // accesses per row, TPP * GW entries apart
    typedef T QVec __attribute__((ext_vector_type(GW)));
    for (int e = tid; e < NB2 * NB2; e += 256) {
        const int a = e / NB2, c = e % NB2;
        Qs[C::q_idx(a, c)] = (a == c) ? T(1) : T(0);
    }
    const bool cross = cross_only;
    const bool angle_thread = tid >= 256 - NPH;        // the upper lanes of wave 3
    const int ka = tid - (256 - NPH);
    // this thread's H blocks: pairs k1 <= k2; byte offsets (read | write <<
    // 16) into an H buffer and byte offsets of the two rotations
    constexpr int HS = sizeof(HT);
    int bk1[HB], bk2[HB], rw[HB][4], ro1[HB], ro2[HB];
#pragma unroll
    for (int b = 0; b < HB; ++b) {
        const int bi = tid + NBT * b;
        int k2 = (int)((sqrtf(8.0f * (float)bi + 1.0f) - 1.0f) * 0.5f);
        while (k2 > 0 && k2 * (k2 + 1) / 2 > bi) --k2;
        while ((k2 + 1) * (k2 + 2) / 2 <= bi) ++k2;
        const bool use = tid < NBT && bi < NBLK;
        const int k1 = use ? bi - k2 * (k2 + 1) / 2 : 0;
        if (!use) k2 = 0;
        bk1[b] = use ? k1 : -1;
        bk2[b] = k2;
        const int u0 = k1, u1 = partner_seat<NB2>(cross, k1);
        const int v0 = k2, v1 = partner_seat<NB2>(cross, k2);
        const int nu0 = next_seat<NB2>(cross, u0), nu1 = next_seat<NB2>(cross, u1);
        const int nv0 = next_seat<NB2>(cross, v0), nv1 = next_seat<NB2>(cross, v1);
        rw[b][0] = HS * sym_idx(u0, v0) | (HS * sym_idx(nu0, nv0) << 16);
        rw[b][1] = HS * sym_idx(u0, v1) | (HS * sym_idx(nu0, nv1) << 16);
        rw[b][2] = HS * sym_idx(u1, v0) | (HS * sym_idx(nu1, nv0) << 16);
        rw[b][3] = HS * sym_idx(u1, v1) | (HS * sym_idx(nu1, nv1) << 16);
        ro1[b] = 16 * k1;
        ro2[b] = 16 * k2;
    }
    // angle threads: where the two vectors of pair ka at step s+1 sat at step s
    int akp = 0, akq = 0;
    bool afp = true, afq = true;
    if (angle_thread) {
        const int sa = prev_seat<NB2>(cross, ka), sb = prev_seat<NB2>(cross, partner_seat<NB2>(cross, ka));
        akp = seat_pair<NB2>(cross, sa, afp);
        akq = seat_pair<NB2>(cross, sb, afq);
        const int p = ka, q = partner_seat<NB2>(cross, ka);
        double c, sn;
        jacobi_angle(H0[sym_idx(p, p)], H0[sym_idx(q, q)], H0[sym_idx(p, q)], true, c, sn);
        sh.rot_cs[0][ka] = rot_make<T>(c, sn);
    }
    // Q rows of pair qk: the vectors on its seats, advanced every step (the
    // vector on a moving seat goes up by one, NB2-1 wrapping round to 1 in
    // a full sweep, to b in a cross sweep)
    const int qk = tid / TPP, qc0 = (tid % TPP) * GW;
    const int qsa = qk, qsb = partner_seat<NB2>(cross, qk);
    int qp = qsa, qq = qsb;   // step 0: vector = seat
    const bool qp_moves = cross ? false : qsa != 0;
    auto advance = [&](int v) { return v == NB2 - 1 ? (cross ? B : 1) : v + 1; };
    const int nsteps = cross ? B : NB2 - 1;
    __syncthreads();
    // The step loop runs two steps per iteration, so that the buffer of
    // each step is a compile-time offset of the LDS accesses.
    auto one_step = [&](auto parity, int step) {
        constexpr int cb = decltype(parity)::value;
        const char* __restrict__ Hc = reinterpret_cast<const char*>(H0 + cb * NH);
        char* __restrict__ Hn = reinterpret_cast<char*>(H0 + (cb ^ 1) * NH);
        const double2* rcs = sh.rot_cs[cb];
        const char* rcb = reinterpret_cast<const char*>(rcs);
        // ---- this thread's Q segments (rotated at the end of the step):
        // loaded first, so that their latency overlaps the H work
        QVec vp[NG], vq[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            vp[g] = *reinterpret_cast<const QVec*>(&Qs[C::q_idx(qp, qc0 + g * TPP * GW)]);
            vq[g] = *reinterpret_cast<const QVec*>(&Qs[C::q_idx(qq, qc0 + g * TPP * GW)]);
        }
        const double2 rq = rcs[qk];
        // ---- rotations of step s+1 (angle threads, wave 3): first, so that
        // their registers are free again for the H blocks of waves 0-2
        if (angle_thread && step + 1 < nsteps) {
            const int xa = akp, xb = partner_seat<NB2>(cross, akp);
            const int ya = akq, yb = partner_seat<NB2>(cross, akq);
            const HT* Hd = reinterpret_cast<const HT*>(Hc);
            double h[10];
            h[0] = Hd[sym_idx(xa, xa)]; h[1] = Hd[sym_idx(xa, xb)]; h[2] = Hd[sym_idx(xb, xb)];
            h[3] = Hd[sym_idx(ya, ya)]; h[4] = Hd[sym_idx(ya, yb)]; h[5] = Hd[sym_idx(yb, yb)];
            h[6] = Hd[sym_idx(xa, ya)]; h[7] = Hd[sym_idx(xa, yb)];
            h[8] = Hd[sym_idx(xb, ya)]; h[9] = Hd[sym_idx(xb, yb)];
            const double2 rx = rcs[akp], ry = rcs[akq];
            // new vector = a0 * (first of its pair) + a1 * (second)
            const double a0 = afp ? rx.x : rx.y, a1 = afp ? -rx.y : rx.x;
            const double b0 = afq ? ry.x : ry.y, b1 = afq ? -ry.y : ry.x;
            const double app = a0 * (a0 * h[0] + a1 * h[1]) + a1 * (a0 * h[1] + a1 * h[2]);
            const double aqq = b0 * (b0 * h[3] + b1 * h[4]) + b1 * (b0 * h[4] + b1 * h[5]);
            const double apq = a0 * (b0 * h[6] + b1 * h[7]) + a1 * (b0 * h[8] + b1 * h[9]);
            double c, sn;
            jacobi_angle(app, aqq, apq, true, c, sn);
            sh.rot_cs[cb ^ 1][ka] = rot_make<T>(c, sn);
        }
        // ---- H <- J^T H J on this thread's 2x2 blocks, written on the next
        // seats; all of the thread's blocks (up to three) loaded before any is
        // rotated, so that the step waits for LDS once
        constexpr int HG = RoundOcc<T, NB2>::OCC4 ? 1 : 3;
#pragma unroll
        for (int b0 = 0; b0 < HB; b0 += HG) {
            double hv[HG][4];
            double2 r1[HG], r2[HG];
#pragma unroll
            for (int u = 0; u < HG; ++u) {
                const int b = b0 + u;
                if (b < HB && bk1[b] >= 0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) hv[u][e] = *reinterpret_cast<const HT*>(Hc + (rw[b][e] & 0xffff));
                    r1[u] = *reinterpret_cast<const double2*>(rcb + ro1[b]);
                    r2[u] = *reinterpret_cast<const double2*>(rcb + ro2[b]);
                }
            }
#pragma unroll
            for (int u = 0; u < HG; ++u) {
                const int b = b0 + u;
                if (b >= HB || bk1[b] < 0) continue;
                const double c1 = r1[u].x, s1 = r1[u].y, c2 = r2[u].x, s2 = r2[u].y;
                const double t0 = c2 * hv[u][0] - s2 * hv[u][1], t1 = s2 * hv[u][0] + c2 * hv[u][1];
                const double t2 = c2 * hv[u][2] - s2 * hv[u][3], t3 = s2 * hv[u][2] + c2 * hv[u][3];
                *reinterpret_cast<HT*>(Hn + (rw[b][0] >> 16)) = c1 * t0 - s1 * t2;
                *reinterpret_cast<HT*>(Hn + (rw[b][1] >> 16)) = c1 * t1 - s1 * t3;
                if (bk1[b] != bk2[b]) *reinterpret_cast<HT*>(Hn + (rw[b][2] >> 16)) = s1 * t0 + c1 * t2;
                *reinterpret_cast<HT*>(Hn + (rw[b][3] >> 16)) = s1 * t1 + c1 * t3;
            }
        }
        // ---- Q <- Q J: rows qp, qq of Q^T, groups of GW entries at qc0,
        // qc0 + TPP GW, ...; the TPP threads of a row pair cover consecutive
        // groups at every access, so the accesses hit distinct banks
        {
            const T c = (T)rq.x, sn = (T)rq.y;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                *reinterpret_cast<QVec*>(&Qs[C::q_idx(qp, qc0 + g * TPP * GW)]) = c * vp[g] - sn * vq[g];
                *reinterpret_cast<QVec*>(&Qs[C::q_idx(qq, qc0 + g * TPP * GW)]) = sn * vp[g] + c * vq[g];
            }
            if (qp_moves) qp = advance(qp);
            qq = advance(qq);
        }
        __syncthreads();
    };
    for (int step = 0; step < nsteps; step += 2) {
        one_step(std::integral_constant<int, 0>(), step);
        if (step + 1 < nsteps) one_step(std::integral_constant<int, 1>(), step + 1);
    }

    // ---------------- phase 3: vectors <- Q^T vectors, W <- W Q (MFMA)
    // Each wave owns the 16-position tiles wave, wave+4, ... of the vectors:
    // it stages the 2b values of a tile in its own LDS region, multiplies by
    // Q (shared, read-only here) and stores the result straight back to the
    // same positions, so the waves never wait for each other.  Column
    // families give D = Q^T old (MFMA lanes along positions), row families
    // D^T = old^T Q (lanes along the contiguous vector index); either way
    // 16 lanes store 64 contiguous bytes.
    // In FP32 the MFMA operand fragments of Q (Q[c][a] for c = kk + lg,
    // a = 16 ta + lr) stay in registers for both products, NB2 / 4 x NT
    // values a lane; FP64 reads them from LDS (its registers are full).
    constexpr bool QREG = sizeof(T) == 4 && !RoundOcc<T, NB2>::OCC4;
    T qf[QREG ? NB2 / 4 : 1][NT];
    if constexpr (QREG) {
#pragma unroll
        for (int kq = 0; kq < NB2 / 4; ++kq) {
#pragma unroll
            for (int ta = 0; ta < NT; ++ta) qf[kq][ta] = Qs[C::q_idx(ta * 16 + lr, 4 * kq + lg)];
        }
    }
    // The W columns follow the vectors: the last vector tile of a wave
    // already loads the wave's first W tile (where registers allow), so
    // that its latency overlaps the MFMAs of the vectors.
    const int64_t ntile_w = (r + PT - 1) / PT;
    // Returns whether the wave's first W tile is already in registers.
    auto update = [&](auto rows_tag, T* base, int64_t vs, int64_t es, int64_t len, bool vec,
                      bool preloaded, bool next_w) -> bool {
        constexpr bool RW = decltype(rows_tag)::value;
        constexpr int PLD = RW ? PT + 1 : PT;                  // odd stride spreads transposed stores
        const int64_t ntile = (len + PT - 1) / PT;
        int64_t tile = wave;
        const bool any = tile < ntile;
        if constexpr (INT) {
            // Interior slices: a branch-free loop with exactly NA unchecked
            // 16-byte loads per iteration (the next tile, at the end an
            // unused reload of the current one) and unchecked stores.  (The
            // W tile prefetch of the checked loop does not fit the registers
            // here.)
            auto fast = [&](bool rw, const T* b, int64_t vs_, int64_t es_, int64_t t0) {
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    int c, tt;
                    origin(rw, u, c, tt);
                    const int64_t gi = gidx(c), t = t0 + tt;
                    const T* src = rw ? b + gi + t * es_ : b + gi * vs_ + t;
                    if constexpr (sizeof(T) == 4) {
                        const float4 x = *reinterpret_cast<const float4*>(src);
                        pre[u][0] = x.x; pre[u][1] = x.y; pre[u][2] = x.z; pre[u][3] = x.w;
                    } else {
                        const double2 x = *reinterpret_cast<const double2*>(src);
                        pre[u][0] = x.x; pre[u][1] = x.y;
                    }
                }
            };
            auto tile_step = [&](int64_t tile) {
#pragma unroll
                for (int u = 0; u < NA; ++u) {
                    int c, tt;
                    origin(RW, u, c, tt);
                    if (!RW) {
                        T* const dst = stg + c * PLD + tt;
                        if constexpr (sizeof(T) == 4)
                            *reinterpret_cast<float4*>(dst) = make_float4(pre[u][0], pre[u][1], pre[u][2], pre[u][3]);
                        else
                            *reinterpret_cast<double2*>(dst) = make_double2(pre[u][0], pre[u][1]);
                    } else {
#pragma unroll
                        for (int q = 0; q < VW; ++q) stg[(c + q) * PLD + tt] = pre[u][q];
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                fast(RW, base, vs, es, (tile + 4 < ntile ? tile + 4 : tile) * PT);
                // keep the loads of the next tile ahead of this tile's MFMAs
                __builtin_amdgcn_sched_barrier(0);
                AccT acc[NT];
#pragma unroll
                for (int ta = 0; ta < NT; ++ta) acc[ta] = zero4<AccT>();
#pragma unroll
                for (int kk = 0; kk < NB2; kk += 4) {
                    const T b = stg[(kk + lg) * PLD + lr];
#pragma unroll
                    for (int ta = 0; ta < NT; ++ta) {
                        const T q = QREG ? qf[QREG ? kk / 4 : 0][ta] : Qs[C::q_idx(ta * 16 + lr, kk + lg)];
                        acc[ta] = RW ? mfma(b, q, acc[ta]) : mfma(q, b, acc[ta]);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                const int64_t t0 = tile * PT;
#pragma unroll
                for (int ta = 0; ta < NT; ++ta) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (!RW) base[gidx(ta * 16 + mfma_row<T>(lg, v)) * vs + t0 + lr] = acc[ta][v];
                        else base[gidx(ta * 16 + lr) + (t0 + mfma_row<T>(lg, v)) * es] = acc[ta][v];
                    }
                }
            };
            // the first tile peeled off, so that the loop is entered only
            // after a tile's loads and stores, like every later iteration:
            // the wait at its top then counts the loads alone
            if (any) {
                if (!preloaded) fast(RW, base, vs, es, tile * PT);
                tile_step(tile);
                for (tile += 4; tile < ntile; tile += 4) tile_step(tile);
            }
            return false;
        }
        if (tile < ntile && !preloaded) load_tile(RW, base, vs, es, len, vec, tile * PT);
        for (; tile < ntile; tile += 4) {
            // stage the tile: stg[c * PLD + t]
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                int c, tt;
                origin(RW, u, c, tt);
                if (!RW) {
                    T* const dst = stg + c * PLD + tt;
                    if constexpr (sizeof(T) == 4)
                        *reinterpret_cast<float4*>(dst) = make_float4(pre[u][0], pre[u][1], pre[u][2], pre[u][3]);
                    else
                        *reinterpret_cast<double2*>(dst) = make_double2(pre[u][0], pre[u][1]);
                } else {
#pragma unroll
                    for (int q = 0; q < VW; ++q) stg[(c + q) * PLD + tt] = pre[u][q];
                }
            }
            // the wave's own LDS stores before its reads (LDS is in order per wave)
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            if (tile + 4 < ntile) load_tile(RW, base, vs, es, len, vec, (tile + 4) * PT);
            else if (next_w && wave < ntile_w) load_tile(false, Wb, r, 1, r, vec_w != 0, wave * PT);
            __builtin_amdgcn_sched_barrier(0);   // loads ahead of the MFMAs
            AccT acc[NT];
#pragma unroll
            for (int ta = 0; ta < NT; ++ta) acc[ta] = zero4<AccT>();
#pragma unroll
            for (int kk = 0; kk < NB2; kk += 4) {
                const T b = stg[(kk + lg) * PLD + lr];                  // old[c][t]
#pragma unroll
                for (int ta = 0; ta < NT; ++ta) {
                    const T q = QREG ? qf[QREG ? kk / 4 : 0][ta] : Qs[C::q_idx(ta * 16 + lr, kk + lg)];
                    acc[ta] = RW ? mfma(b, q, acc[ta]) : mfma(q, b, acc[ta]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            const int64_t t0 = tile * PT;
#pragma unroll
            for (int ta = 0; ta < NT; ++ta) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (!RW) {
                        const int64_t gi = gidx(ta * 16 + mfma_row<T>(lg, v)), t = t0 + lr;
                        if (gi < r && t < len) base[gi * vs + t] = acc[ta][v];
                    } else {
                        const int64_t gi = gidx(ta * 16 + lr), t = t0 + mfma_row<T>(lg, v);
                        if (gi < r && t < len) base[gi + t * es] = acc[ta][v];
                    }
                }
            }
        }
        return next_w && any;
    };
    constexpr bool NEXTW = ROWS || sizeof(T) == 8;   // FP32 column families: no registers to spare
    const bool w_pre = update(std::integral_constant<bool, ROWS>(), Ab, g.vs, g.es, L, vec_a != 0, EARLY,
                              NEXTW && Wb != nullptr);
    // W == nullptr: the caller needs no accumulated rotations (uniform branch)
    if (Wb) update(std::integral_constant<bool, false>(), Wb, r, 1, r, vec_w != 0, w_pre, false);
    // both blocks changed (read by later launches only: each block belongs
    // to one pair per round)
    if (tid == 0) {
        trk[blo] = ver_lo + 1;
        trk[bhi] = ver_hi + 1;
    }
}

// The LDS of a workgroup is what the waves-per-SIMD figure assumes: FP32
// pairs of 64 vectors run four workgroups per 160 KB compute unit, FP64 pairs
// of 64 vectors two.
template <class T, int NB2>
constexpr bool lds_fits() {
    return sizeof(RoundShared<T, NB2>) <= RoundCfg<T, NB2>::lds_bytes &&
           RoundOcc<T, NB2>::WAVES * RoundCfg<T, NB2>::lds_bytes <= 160 * 1024;
}
static_assert(lds_fits<float, 32>() && lds_fits<float, 64>() && lds_fits<double, 32>() && lds_fits<double, 64>(),
              "LDS budget of jacobi_round");
static_assert(RoundOcc<float, 64>::WAVES == 4 && RoundCfg<float, 64>::WAVES == 3 &&
              RoundCfg<double, 64>::WAVES == 2, "workgroups per compute unit");

// One round for every (slice, pair) of a tensor of identical slices.
template <class T, int NB2, bool ROWS, bool INT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RoundOcc<T, NB2>::WAVES)))
void jacobi_round(T* __restrict__ A, T* __restrict__ W, SliceGeom g,
                                                    int nbe, int rnd, JacobiCtl* __restrict__ ctl,
                                                    double tol, int vec_a, int vec_w,
                                                    unsigned long long* __restrict__ pair_counts,
                                                    int32_t* __restrict__ track) {
    __shared__ RoundShared<T, NB2> sh;
    const int npairs = nbe / 2;
    const int64_t s = blockIdx.x / npairs;
    const int k = blockIdx.x % npairs;
    if (ctl[s].done) return;
    round_body<T, NB2, ROWS, INT>(sh, A + s * g.m * g.p, W ? W + s * g.r * g.r : nullptr, g, nbe, rnd, k,
                                  ctl + s, tol, vec_a, vec_w, pair_counts, track + s * nbe * nbe);
}

// One step of the global round counter t for a batch of slices of any
// shapes: task = (slice, pair); slice s is in round t mod (nbe_s - 1) of its
// own tournament, so slices with fewer blocks simply run more sweeps.
template <class T, int NB2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RoundOcc<T, NB2>::WAVES)))
void jacobi_round_batch(const BatchSlice* __restrict__ sl,
                                                          const int2* __restrict__ tasks, int t,
                                                          JacobiCtl* __restrict__ ctl,
                                                          unsigned long long* __restrict__ pair_counts) {
    __shared__ RoundShared<T, NB2> sh;
    const int2 tk = tasks[blockIdx.x];
    if (ctl[tk.x].done) return;
    const BatchSlice d = sl[tk.x];
    const int rnd = t % (d.nbe - 1);
    if (d.g.rows)
        round_body<T, NB2, true>(sh, static_cast<T*>(d.A), static_cast<T*>(d.W), d.g, d.nbe, rnd,
                                 tk.y, ctl + tk.x, d.tol, d.vec_a, d.vec_w, pair_counts, d.track);
    else
        round_body<T, NB2, false>(sh, static_cast<T*>(d.A), static_cast<T*>(d.W), d.g, d.nbe, rnd,
                                  tk.y, ctl + tk.x, d.tol, d.vec_a, d.vec_w, pair_counts, d.track);
}

// end of a sweep for the slices whose tournament finished a sweep at step t;
// remaining counts the slices still running after step t
__global__ void jacobi_sweep_end_batch(const BatchSlice* __restrict__ sl, int64_t nslices, int t,
                                       JacobiCtl* __restrict__ ctl, int* __restrict__ remaining) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nslices) return;
    const int nr = sl[i].nbe - 1;
    JacobiCtl c = ctl[i];
    if (c.done) return;
    if (t % nr != nr - 1) {
        atomicAdd(remaining, 1);
        return;
    }
    c.sweeps += 1;
    const double mc = __longlong_as_double((long long)c.maxcos_bits);
    if (c.nonfinite || mc <= sl[i].tol) c.done = 1;
    else atomicAdd(remaining, 1);
    c.maxcos_bits = 0ull;
    ctl[i] = c;
}

// W = I (slices that accumulate rotations) and a clean control word for
// every slice of a batch
template <class T>
__global__ void jacobi_init_batch(const BatchSlice* __restrict__ sl, JacobiCtl* __restrict__ ctl,
                                  int* __restrict__ remaining, int max_steps,
                                  unsigned long long* __restrict__ pair_counts,
                                  int32_t* __restrict__ status) {
    const BatchSlice d = sl[blockIdx.x];
    const int64_t r = d.g.r;
    T* W = static_cast<T*>(d.W);
    if (W)
        for (int64_t e = threadIdx.x; e < r * r; e += blockDim.x) W[e] = (e % r == e / r) ? T(1) : T(0);
    for (int e = threadIdx.x; e < d.nbe * d.nbe; e += blockDim.x) d.track[e] = e < d.nbe ? 0 : -1;
    if (threadIdx.x == 0) {
        JacobiCtl c;
        c.maxcos_bits = 0ull; c.done = 0; c.sweeps = 0; c.nonfinite = 0; c.pad = 0;
        ctl[blockIdx.x] = c;
    }
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < max_steps; i += blockDim.x) remaining[i] = 0;
        for (int i = threadIdx.x; i < PC_WORDS; i += blockDim.x) pair_counts[i] = 0ull;
        if (threadIdx.x == 0) *status = TSVDM_OK;
    }
}

// squared norms of every slice's final vectors, one workgroup per slice
// Sum of squares of x[0], x[s], ..., x[(n - 1) s] in FP64, accumulated in
// that order; eight loads are in flight at a time (a loop with one load per
// iteration waits for every load).
template <class T>
__device__ __forceinline__ double sumsq_strided(const T* __restrict__ x, int64_t s, int64_t n) {
    double acc = 0.0;
    int64_t t = 0;
    for (; t + 8 <= n; t += 8) {
        T v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = x[(t + q) * s];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double e = (double)v[q];
            acc = fma(e, e, acc);
        }
    }
    for (; t < n; ++t) {
        const double e = (double)x[t * s];
        acc = fma(e, e, acc);
    }
    return acc;
}

template <class T>
__global__ __launch_bounds__(256) void jacobi_norms_batch(const BatchSlice* __restrict__ sl) {
    const BatchSlice d = sl[blockIdx.x];
    const T* A = static_cast<const T*>(d.A);
    const SliceGeom g = d.g;
    if (g.rows) {
        for (int64_t j = threadIdx.x; j < g.r; j += blockDim.x) d.s2[j] = sumsq_strided(A + j, g.es, g.L);
    } else {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int64_t j = wave; j < g.r; j += 4) {
            const T* x = A + j * g.vs;
            double acc = lane < g.L ? sumsq_strided(x + lane, 64, (g.L - lane + 63) / 64) : 0.0;
            for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
            if (lane == 0) d.s2[j] = acc;
        }
    }
}

__global__ void jacobi_sweep_end(JacobiCtl* __restrict__ ctl, int64_t n, double tol,
                                 int* __restrict__ remaining) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    JacobiCtl c = ctl[i];
    if (c.done) return;
    c.sweeps += 1;
    const double mc = __longlong_as_double((long long)c.maxcos_bits);
    if (c.nonfinite || mc <= tol) c.done = 1;
    else atomicAdd(remaining, 1);
    c.maxcos_bits = 0ull;
    ctl[i] = c;
}

// squared norms of the final vectors, FP64, fixed summation order
template <class T>
__global__ __launch_bounds__(256) void jacobi_norms_rows(const T* __restrict__ A, SliceGeom g,
                                                         double* __restrict__ s2,
                                                         const int32_t* __restrict__ run) {
    // rows case (vs = 1, es = m): thread per vector, coalesced across threads
    const int64_t s = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.r || (run && !run[s])) return;
    const T* Ab = A + s * g.m * g.p;
    s2[s * g.r + j] = sumsq_strided(Ab + j, g.es, g.L);
}

template <class T>
__global__ __launch_bounds__(256) void jacobi_norms_cols(const T* __restrict__ A, SliceGeom g,
                                                         int64_t total_vectors,
                                                         double* __restrict__ s2,
                                                         const int32_t* __restrict__ run) {
    // columns case: one wavefront per contiguous vector
    const int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= total_vectors) return;
    const int64_t s = v / g.r, j = v % g.r;
    if (run && !run[s]) return;
    const T* x = A + s * g.m * g.p + j * g.vs;
    double acc = lane < g.L ? sumsq_strided(x + lane, 64, (g.L - lane + 63) / 64) : 0.0;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) s2[s * g.r + j] = acc;
}

__global__ void jacobi_finish(const JacobiCtl* __restrict__ ctl, int64_t n,
                              int32_t* __restrict__ status) {
    __shared__ int nf, nc;
    if (threadIdx.x == 0) { nf = 0; nc = 0; }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        if (ctl[i].nonfinite) atomicOr(&nf, 1);
        else if (!ctl[i].done) atomicOr(&nc, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *status = nf ? TSVDM_E_NONFINITE : (nc ? TSVDM_E_NOCONV : TSVDM_OK);
}

// Pinned host slots for the per-sweep counts of unconverged slices: one set
// per host thread, allocated on first use and kept for the life of the
// process (nullptr if pinned memory is unavailable).
int* poll_slots() {
    static thread_local int* slots = nullptr;
    static thread_local bool tried = false;
    if (!tried) {
        tried = true;
        if (hipHostMalloc((void**)&slots, 1024 * sizeof(int), hipHostMallocDefault) != hipSuccess) slots = nullptr;
    }
    return slots;
}

template <class T, int NB2>
int jacobi_impl(T* A, int64_t m, int64_t p, int64_t n, T* W, double* s2, int32_t* status,
                const JacobiOpts& o, void* ws, hipStream_t st) {
    static_assert(NB2 >= 32, "the workspace holds pair records for blocks of 16 vectors or more");
    const SliceGeom g = slice_geom(m, p);
    Carver cv(ws);
    JacobiCtl* ctl = cv.carve<JacobiCtl>((size_t)n);
    int* remaining = cv.carve<int>((size_t)o.max_sweeps);
    unsigned long long* pair_counts = cv.carve<unsigned long long>(PC_WORDS);
    constexpr int B = NB2 / 2;
    const int nb = (int)((g.r + B - 1) / B);
    const int nbe = nb + (nb & 1);
    int32_t* track = cv.carve<int32_t>((size_t)(n * nbe * nbe));
    const bool stats = stats_enabled();
    unsigned long long* const pcount = stats ? pair_counts : nullptr;   // counted only for statistics
    std::vector<hipEvent_t> evs;

    int64_t gblocks = g.r * n;   // one workgroup per column of W (grid-stride beyond the cap)
    if (gblocks < (n * nbe * nbe + 255) / 256) gblocks = (n * nbe * nbe + 255) / 256;
    if (gblocks > 65535 * 16) gblocks = 65535 * 16;
    if (gblocks < 1) gblocks = 1;
    jacobi_init<T><<<(unsigned)gblocks, 256, 0, st>>>(o.w_given ? nullptr : W, g.r, n, ctl, remaining,
                                                      o.max_sweeps, pair_counts, status, o.run,
                                                      track, nbe);
    TSVDM_LAUNCH_CHECK();

    const int npairs = nbe / 2;
    const int64_t blocks = n * npairs;
    constexpr int VW = 16 / (int)sizeof(T);
    // 16-byte accesses need every vector (columns) / every row stride (rows)
    // to start on a multiple of VW elements
    const int vec_a = (g.m % VW == 0) ? 1 : 0;
    const int vec_w = (g.r % VW == 0) ? 1 : 0;
    TSVDM_REQUIRE(blocks < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many slice pairs for one launch");
    // every pair interior: whole blocks, an even block count (no padding
    // block), 16-byte aligned accesses, L and r multiples of the tile
    const bool interior = g.r % B == 0 && nb % 2 == 0 && vec_a && vec_w && g.L % 16 == 0 && g.r % 16 == 0;
    int64_t launches = 0;
    // The host poll runs one sweep behind: sweep s's count is copied into
    // pinned memory and read once sweep s + 1 is queued, so the GPU does not
    // idle while the host waits.  A sweep queued after convergence finds
    // every slice done; its launches return at once and change nothing.
    int* poll = o.host_poll ? poll_slots() : nullptr;
    hipEvent_t pev[2] = {nullptr, nullptr};
    int last = -1;
    if (poll) {
        TSVDM_HIP_CHECK(hipEventCreateWithFlags(&pev[0], hipEventDisableTiming));
        TSVDM_HIP_CHECK(hipEventCreateWithFlags(&pev[1], hipEventDisableTiming));
    }
    for (int sweep = 0; sweep < o.max_sweeps; ++sweep) {
        if (stats) {
            hipEvent_t e0, e1;
            TSVDM_HIP_CHECK(hipEventCreate(&e0));
            TSVDM_HIP_CHECK(hipEventCreate(&e1));
            evs.push_back(e0);
            evs.push_back(e1);
            TSVDM_HIP_CHECK(hipEventRecord(e0, st));
        }
        for (int rnd = 0; rnd < nbe - 1; ++rnd) {
            if (g.rows && interior)
                jacobi_round<T, NB2, true, true><<<(unsigned)blocks, 256, 0, st>>>(
                    A, W, g, nbe, rnd, ctl, o.tol, vec_a, vec_w, pcount, track);
            else if (g.rows)
                jacobi_round<T, NB2, true, false><<<(unsigned)blocks, 256, 0, st>>>(
                    A, W, g, nbe, rnd, ctl, o.tol, vec_a, vec_w, pcount, track);
            else if (interior)
                jacobi_round<T, NB2, false, true><<<(unsigned)blocks, 256, 0, st>>>(
                    A, W, g, nbe, rnd, ctl, o.tol, vec_a, vec_w, pcount, track);
            else
                jacobi_round<T, NB2, false, false><<<(unsigned)blocks, 256, 0, st>>>(
                    A, W, g, nbe, rnd, ctl, o.tol, vec_a, vec_w, pcount, track);
            TSVDM_LAUNCH_CHECK();
            ++launches;
        }
        if (stats) TSVDM_HIP_CHECK(hipEventRecord(evs.back(), st));
        jacobi_sweep_end<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(ctl, n, o.tol, remaining + sweep);
        TSVDM_LAUNCH_CHECK();
        if (poll) {
            TSVDM_HIP_CHECK(hipMemcpyAsync(poll + sweep, remaining + sweep, sizeof(int),
                                           hipMemcpyDeviceToHost, st));
            TSVDM_HIP_CHECK(hipEventRecord(pev[sweep & 1], st));
            last = sweep;
            if (sweep >= 1) {
                TSVDM_HIP_CHECK(hipEventSynchronize(pev[(sweep - 1) & 1]));
                if (poll[sweep - 1] == 0) break;
            }
        } else if (o.host_poll) {
            int left = -1;
            TSVDM_HIP_CHECK(hipMemcpyAsync(&left, remaining + sweep, sizeof(int),
                                           hipMemcpyDeviceToHost, st));
            TSVDM_HIP_CHECK(hipStreamSynchronize(st));
            if (left == 0) break;
        }
    }
    if (!g.rows) {
        const int64_t tv = g.r * n;
        jacobi_norms_cols<T><<<(unsigned)((tv + 3) / 4), 256, 0, st>>>(A, g, tv, s2, o.run);
    } else {
        dim3 grid((unsigned)((g.r + 255) / 256), (unsigned)n);
        jacobi_norms_rows<T><<<grid, 256, 0, st>>>(A, g, s2, o.run);
    }
    TSVDM_LAUNCH_CHECK();
    jacobi_finish<<<1, 256, 0, st>>>(ctl, n, status);
    TSVDM_LAUNCH_CHECK();
    if (poll) {
        // no copy into the pinned slots may be in flight once this returns
        // (the next call on this thread reuses them); the kernels queued
        // above keep the GPU busy meanwhile
        if (last >= 0) TSVDM_HIP_CHECK(hipEventSynchronize(pev[last & 1]));
        (void)hipEventDestroy(pev[0]);
        (void)hipEventDestroy(pev[1]);
    }
    if (stats) {
        std::vector<unsigned long long> bins(PC_WORDS);
        unsigned long long pc[4];
        TSVDM_HIP_CHECK(hipMemcpyAsync(bins.data(), pair_counts, sizeof(unsigned long long) * PC_WORDS,
                                       hipMemcpyDeviceToHost, st));
        TSVDM_HIP_CHECK(hipStreamSynchronize(st));
        pc_sum(bins.data(), pc);
        double ms = 0.0;
        for (size_t i = 0; i + 1 < evs.size(); i += 2) {
            float t = 0.f;
            TSVDM_HIP_CHECK(hipEventElapsedTime(&t, evs[i], evs[i + 1]));
            ms += t;
        }
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
        stats_add_counters(launches, ms, pc, NB2);
    }
    return TSVDM_OK;
}

template <class T>
int jacobi_batch_impl(const BatchSlice* sl, int64_t nslices, const int2* tasks,
                      const int64_t* group, int max_steps, int host_poll, void* ctl_ws,
                      int32_t* status, hipStream_t st) {
    Carver cv(ctl_ws);
    JacobiCtl* ctl = cv.carve<JacobiCtl>((size_t)nslices);
    int* remaining = cv.carve<int>((size_t)max_steps);
    unsigned long long* pair_counts = cv.carve<unsigned long long>(PC_WORDS);
    TSVDM_REQUIRE(nslices < ((int64_t)1 << 31) && group[0] < ((int64_t)1 << 31) &&
                      group[1] < ((int64_t)1 << 31),
                  TSVDM_E_SHAPE, "batch too large for one launch");
    jacobi_init_batch<T><<<(unsigned)nslices, 256, 0, st>>>(sl, ctl, remaining, max_steps,
                                                           pair_counts, status);
    TSVDM_LAUNCH_CHECK();
    const bool stats = stats_enabled();
    unsigned long long* const pcount = stats ? pair_counts : nullptr;   // counted only for statistics
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        TSVDM_HIP_CHECK(hipEventCreate(&e0));
        TSVDM_HIP_CHECK(hipEventCreate(&e1));
        TSVDM_HIP_CHECK(hipEventRecord(e0, st));
    }
    int64_t launches = 0;
    const unsigned sblocks = (unsigned)((nslices + 255) / 256);
    // Poll every 4 steps, one poll behind (as in the single-tensor loop):
    // poll k's count goes to pinned slot k mod 2 and is read once poll k + 1
    // is queued; steps queued after convergence find every slice done.
    int* poll = host_poll ? poll_slots() : nullptr;
    hipEvent_t pev[2] = {nullptr, nullptr};
    int lastk = -1;
    if (poll) {
        TSVDM_HIP_CHECK(hipEventCreateWithFlags(&pev[0], hipEventDisableTiming));
        TSVDM_HIP_CHECK(hipEventCreateWithFlags(&pev[1], hipEventDisableTiming));
    }
    for (int t = 0; t < max_steps; ++t) {
        // both pair widths see the same round counter t
        if (group[0] > 0) {
            jacobi_round_batch<T, 32><<<(unsigned)group[0], 256, 0, st>>>(sl, tasks, t, ctl, pcount);
            TSVDM_LAUNCH_CHECK();
            ++launches;
        }
        if (group[1] > 0) {
            jacobi_round_batch<T, 64><<<(unsigned)group[1], 256, 0, st>>>(sl, tasks + group[0], t, ctl,
                                                                         pcount);
            TSVDM_LAUNCH_CHECK();
            ++launches;
        }
        jacobi_sweep_end_batch<<<sblocks, 256, 0, st>>>(sl, nslices, t, ctl, remaining + t);
        TSVDM_LAUNCH_CHECK();
        if (poll && (t % 4 == 3)) {
            const int k = t / 4;
            TSVDM_HIP_CHECK(hipMemcpyAsync(poll + (k & 1), remaining + t, sizeof(int),
                                           hipMemcpyDeviceToHost, st));
            TSVDM_HIP_CHECK(hipEventRecord(pev[k & 1], st));
            lastk = k;
            if (k >= 1) {
                TSVDM_HIP_CHECK(hipEventSynchronize(pev[(k - 1) & 1]));
                if (poll[(k - 1) & 1] == 0) break;
            }
        } else if (host_poll && (t % 4 == 3)) {
            int left = -1;
            TSVDM_HIP_CHECK(hipMemcpyAsync(&left, remaining + t, sizeof(int), hipMemcpyDeviceToHost, st));
            TSVDM_HIP_CHECK(hipStreamSynchronize(st));
            if (left == 0) break;
        }
    }
    if (stats) TSVDM_HIP_CHECK(hipEventRecord(e1, st));
    jacobi_norms_batch<T><<<(unsigned)nslices, 256, 0, st>>>(sl);
    TSVDM_LAUNCH_CHECK();
    jacobi_finish<<<1, 256, 0, st>>>(ctl, nslices, status);
    TSVDM_LAUNCH_CHECK();
    if (poll) {
        // no copy into the pinned slots may be in flight once this returns
        if (lastk >= 0) TSVDM_HIP_CHECK(hipEventSynchronize(pev[lastk & 1]));
        (void)hipEventDestroy(pev[0]);
        (void)hipEventDestroy(pev[1]);
    }
    if (stats) {
        std::vector<unsigned long long> bins(PC_WORDS);
        unsigned long long pc[4];
        TSVDM_HIP_CHECK(hipMemcpyAsync(bins.data(), pair_counts, sizeof(unsigned long long) * PC_WORDS,
                                       hipMemcpyDeviceToHost, st));
        TSVDM_HIP_CHECK(hipStreamSynchronize(st));
        pc_sum(bins.data(), pc);
        float ms = 0.f;
        TSVDM_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        // one pair width for the statistics only when the batch has one
        const int width = group[0] > 0 && group[1] > 0 ? 0 : (group[1] > 0 ? 64 : 32);
        stats_add_counters(launches, ms, pc, width);
    }
    return TSVDM_OK;
}

}  // namespace

size_t jacobi_batch_ctl_bytes(int64_t nslices, int max_steps) {
    Carver cv(nullptr);
    cv.carve<JacobiCtl>((size_t)nslices);
    cv.carve<int>((size_t)max_steps);
    cv.carve<unsigned long long>(PC_WORDS);
    return cv.total();
}

int run_jacobi_batch(int dt, const BatchSlice* sl, int64_t nslices, const int2* tasks,
                     const int64_t* group, int max_steps, int host_poll, void* ctl_ws,
                     int32_t* status, hipStream_t st) {
    if (dt == TSVDM_F64)
        return jacobi_batch_impl<double>(sl, nslices, tasks, group, max_steps, host_poll, ctl_ws, status, st);
    return jacobi_batch_impl<float>(sl, nslices, tasks, group, max_steps, host_poll, ctl_ws, status, st);
}

size_t jacobi_workspace_bytes(int64_t r, int64_t n) {
    // the pair records are sized for the narrowest block (16 vectors)
    const int64_t nb = (r + 15) / 16, nbe = nb + (nb & 1);
    Carver cv(nullptr);
    cv.carve<JacobiCtl>((size_t)n);
    cv.carve<int>(1024);
    cv.carve<unsigned long long>(PC_WORDS);
    cv.carve<int32_t>((size_t)(n * nbe * nbe));
    return cv.total();
}

JacobiOpts jacobi_default_opts(int64_t m, int64_t p, int dt) {
    const SliceGeom g = slice_geom(m, p);
    JacobiOpts o;
    o.block = (g.r >= 256) ? 64 : 32;
    o.max_sweeps = 40;
    const double eps = dt == TSVDM_F64 ? 1.1102230246251565e-16 : 5.9604644775390625e-08;
    const double c = 8.0 * sqrt((double)(g.L > 1 ? g.L : 1)) * eps;
    o.tol = dt == TSVDM_F64 ? fmax(c, 1e-14) : fmax(c, 2e-6);
    o.host_poll = 1;
    return o;
}

int run_jacobi(void* A, int dt, int64_t m, int64_t p, int64_t n, void* W, double* s2,
               int32_t* status, const JacobiOpts& o, void* ws, hipStream_t st) {
    TSVDM_REQUIRE(o.block == 32 || o.block == 64, TSVDM_E_ARG, "block must be 16 or 32 (pair width 32 or 64)");
    TSVDM_REQUIRE(o.max_sweeps >= 1 && o.max_sweeps <= 1024, TSVDM_E_ARG, "max_sweeps must be in [1, 1024]");
    if (dt == TSVDM_F64) {
        if (o.block == 32)
            return jacobi_impl<double, 32>(static_cast<double*>(A), m, p, n, static_cast<double*>(W), s2, status, o, ws, st);
        return jacobi_impl<double, 64>(static_cast<double*>(A), m, p, n, static_cast<double*>(W), s2, status, o, ws, st);
    }
    if (dt == TSVDM_F32) {
        if (o.block == 32)
            return jacobi_impl<float, 32>(static_cast<float*>(A), m, p, n, static_cast<float*>(W), s2, status, o, ws, st);
        return jacobi_impl<float, 64>(static_cast<float*>(A), m, p, n, static_cast<float*>(W), s2, status, o, ws, st);
    }
    set_error("slice SVD supports F64 and F32 only");
    return TSVDM_E_UNSUPPORTED;
}

}  // namespace tsvdm

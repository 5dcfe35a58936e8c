// Factor emission and the variable-rank reconstruction GEMM.
//
// Algorithm 2 keeps, per slice i, the rho_i leading left singular vectors and
// G_i = S_i V_i^T restricted to them; Section 3.4 stores them without padding
// (slice i owns exactly m*rho_i and p*rho_i entries).  The Jacobi output holds
// the vectors unsorted, so each slice first sorts its squared singular values
// (descending, ties by index) in LDS and then gathers the kept triplets.
// The reconstruction C-hat_i = U_i G_i is a batched GEMM whose inner size
// rho_i varies per slice.
#include "common.h"
#include "kernels.h"

namespace tsvdm {

namespace {

constexpr int PMAX = 4096;  // largest r handled by the in-LDS sort

// perm[s*r + c] = index of the c-th largest s2 of slice s; S_pk gets the
// singular values of the kept triplets (positions first .. first+rho-1 of the
// descending order).
template <class T>
__global__ __launch_bounds__(1024) void pack_sort(const double* __restrict__ s2, int64_t r,
                                                  int64_t n, const int32_t* __restrict__ rho,
                                                  const int64_t* __restrict__ offsets,
                                                  int64_t capacity, int first,
                                                  int32_t* __restrict__ perm, T* __restrict__ S_pk,
                                                  int32_t* __restrict__ status) {
    __shared__ unsigned long long key[PMAX];
    __shared__ int idx[PMAX];
    const int64_t s = blockIdx.x;
    int np = 1;
    while (np < r) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        if (i < r) {
            double v = s2[s * r + i];
            if (!(v >= 0.0)) v = 0.0;
            v += 0.0;
            key[i] = ~(unsigned long long)__double_as_longlong(v);  // ascending key = descending value
        } else {
            key[i] = ~0ull;
        }
        idx[i] = i;
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < np / 2; t += blockDim.x) {
                const int i = 2 * j * (t / j) + (t % j);
                const bool up = (i & k) == 0;
                const unsigned long long ka = key[i], kb = key[i + j];
                const int ia = idx[i], ib = idx[i + j];
                const bool gt = (ka > kb) || (ka == kb && ia > ib);
                if (gt == up) { key[i] = kb; key[i + j] = ka; idx[i] = ib; idx[i + j] = ia; }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < r; i += blockDim.x) perm[s * r + i] = idx[i];
    const int64_t off = offsets[s];
    const int kr = rho[s];
    for (int c = threadIdx.x; c < kr; c += blockDim.x) {
        if (off + kr <= capacity && first + c < r) {
            double v = s2[s * r + idx[first + c]];
            S_pk[off + c] = static_cast<T>(sqrt(v > 0.0 ? v : 0.0));
        }
    }
    if (s == 0 && threadIdx.x == 0 && offsets[n] > capacity) *status = TSVDM_E_CAPACITY;
}

// Gather kept vectors into U_pk (m x rho) and G_pk (rho x p) of each slice.
// Workgroup x of a slice takes the U columns c = x, x + gridDim.x, ... and
// the G columns b = x, x + gridDim.x, ...; its threads run along the
// column, so no element needs an index division.
template <class T>
__global__ __launch_bounds__(256) void pack_copy(const T* __restrict__ A, const T* __restrict__ W,
                                                 const double* __restrict__ s2, SliceGeom g,
                                                 const int32_t* __restrict__ rho,
                                                 const int64_t* __restrict__ offsets,
                                                 int64_t capacity, int first,
                                                 const int32_t* __restrict__ perm,
                                                 T* __restrict__ U_pk, T* __restrict__ G_pk) {
    const int64_t s = blockIdx.y;
    const int64_t kr = rho[s];
    const int64_t off = offsets[s];
    if (kr <= 0 || off + kr > capacity) return;  // an overflowing slice is not written
    const int64_t m = g.m, p = g.p, r = g.r;
    const T* Ab = A + s * m * p;
    const T* Wb = W + s * r * r;
    const double* s2b = s2 + s * r;
    const int32_t* pr = perm + s * r + first;
    const bool rows = g.rows != 0;  // m < p: vectors are rows, W holds U
    const int t = threadIdx.x;
    T* const Uo = U_pk + m * off;
    T* const Go = G_pk + p * off;
    for (int64_t c = blockIdx.x; c < kr; c += gridDim.x) {
        const int64_t j = pr[c];
        T* const u = Uo + c * m;
        if (rows) {
            const T* w = Wb + j * r;
            for (int64_t a = t; a < m; a += blockDim.x) u[a] = w[a];
        } else {
            const double sg = sqrt(fmax(s2b[j], 0.0));
            const T* x = Ab + j * m;
            for (int64_t a = t; a < m; a += blockDim.x)
                u[a] = sg > 0.0 ? static_cast<T>((double)x[a] / sg) : T(0);
        }
    }
    for (int64_t b = blockIdx.x; b < p; b += gridDim.x) {
        T* const gcol = Go + b * kr;   // G_pk is kr x p, leading dim kr
        if (rows) {
            const T* x = Ab + b * m;
            for (int64_t c = t; c < kr; c += blockDim.x) gcol[c] = x[pr[c]];
        } else {
            for (int64_t c = t; c < kr; c += blockDim.x) {
                const int64_t j = pr[c];
                const double sg = sqrt(fmax(s2b[j], 0.0));
                gcol[c] = static_cast<T>(sg * (double)Wb[b + j * r]);
            }
        }
    }
}

// C(:,:,s) = U_pk_s (m x rho_s) * G_pk_s (rho_s x p), computed as
// C^T = G^T U^T so that MFMA output lanes run along the rows of C.
// K chunk of the low-rank product staged in LDS.
constexpr int LR_KC = 32;
template <class T, int BW>
struct LowrankShared {
    T Us[LR_KC][64 + 1];  // [c][a]
    T Gs[BW][LR_KC + 1];  // [b][c]
};

// Output tile (ta, tb) of one slice, 64 rows by BW (64 or 128) columns:
// Cb (m x p) = Ub (m x kr) * Gb (kr x p).  Each wave holds BW / 64 strips
// of 16 columns against all 64 rows.  The next K chunk is loaded into
// registers while the MFMAs of the current one run; every sum runs over k
// in increasing order, four terms per MFMA, whatever BW is.
template <class T, int BW>
__device__ __forceinline__ void lowrank_tile(LowrankShared<T, BW>& sh, const T* __restrict__ Ub,
                                             const T* __restrict__ Gb, int64_t m, int64_t p,
                                             int64_t kr, T* __restrict__ Cb, int ta, int tb) {
    typedef typename Acc<T>::type AccT;
    constexpr int KC = LR_KC;
    constexpr int NF = BW / 64;           // 16-column strips per wave
    constexpr int PU = KC * 64 / 256;     // U elements per thread and chunk
    constexpr int PG = KC * BW / 256;     // G elements per thread and chunk
    auto& Us = sh.Us;
    auto& Gs = sh.Gs;
    const int64_t a0 = (int64_t)ta * 64, b0 = (int64_t)tb * BW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    AccT acc[NF][4];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[f][t] = zero4<AccT>();
    T ur[PU], gr[PG];
    auto load = [&](int64_t c0) {
#pragma unroll
        for (int i = 0; i < PU; ++i) {
            const int e = tid + 256 * i;
            const int a = e & 63, c = e >> 6;
            ur[i] = (a0 + a < m && c0 + c < kr) ? Ub[(a0 + a) + (c0 + c) * m] : T(0);
        }
#pragma unroll
        for (int i = 0; i < PG; ++i) {
            const int e = tid + 256 * i;
            const int cg = e % KC, b = e / KC;
            gr[i] = (b0 + b < p && c0 + cg < kr) ? Gb[(c0 + cg) + (b0 + b) * kr] : T(0);
        }
    };
    if (kr > 0) load(0);
    for (int64_t c0 = 0; c0 < kr; c0 += KC) {
#pragma unroll
        for (int i = 0; i < PU; ++i) {
            const int e = tid + 256 * i;
            Us[e >> 6][e & 63] = ur[i];
        }
#pragma unroll
        for (int i = 0; i < PG; ++i) {
            const int e = tid + 256 * i;
            Gs[e / KC][e % KC] = gr[i];
        }
        __syncthreads();
        if (c0 + KC < kr) load(c0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            T av[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) av[f] = Gs[(wave * NF + f) * 16 + lr][kk + lg];  // A = G^T
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                T bv = Us[kk + lg][t * 16 + lr];  // B = U^T : k = c, col a
#pragma unroll
                for (int f = 0; f < NF; ++f) acc[f][t] = mfma(av[f], bv, acc[f][t]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t a = a0 + t * 16 + lr;
        if (a >= m) continue;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t b = b0 + (wave * NF + f) * 16 + mfma_row<T>(lg, v);
                if (b < p) Cb[a + b * m] = acc[f][t][v];
            }
    }
}

template <class T>
struct LowrankCfg {
    static constexpr int WAVES = sizeof(T) == 4 ? 2 : 1;   // waves per SIMD the registers allow
};

template <class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LowrankCfg<T>::WAVES)))
void lowrank_gemm(const T* __restrict__ U_pk,
                                                    const T* __restrict__ G_pk, int64_t m,
                                                    int64_t p, const int32_t* __restrict__ rho,
                                                    const int64_t* __restrict__ offsets,
                                                    int64_t capacity, T* __restrict__ C,
                                                    int tiles_a) {
    __shared__ LowrankShared<T, 128> sh;
    const int64_t s = blockIdx.y;
    const int ta = blockIdx.x % tiles_a, tb = blockIdx.x / tiles_a;
    const int64_t off = offsets[s];
    const int64_t kr = (off + rho[s] <= capacity) ? rho[s] : 0;  // unwritten slices read as 0
    lowrank_tile<T, 128>(sh, U_pk + m * off, G_pk + p * off, m, p, kr, C + s * m * p, ta, tb);
}

// Batched form: task = (slice, tile a, tile b) over PackSlice descriptors.
template <class T>
__global__ __launch_bounds__(256) void lowrank_gemm_batch(const PackSlice* __restrict__ ps,
                                                          const int4* __restrict__ tasks) {
    __shared__ LowrankShared<T, 64> sh;
    const int4 tk = tasks[blockIdx.x];
    const PackSlice d = ps[tk.x];
    const int64_t m = d.g.m, p = d.g.p;
    const int64_t off = *d.off;
    const int64_t kr = (off + *d.rho <= d.capacity) ? *d.rho : 0;
    lowrank_tile<T, 64>(sh, static_cast<const T*>(d.U_pk) + m * off,
                    static_cast<const T*>(d.G_pk) + p * off, m, p, kr, static_cast<T*>(d.C),
                    tk.y, tk.z);
}

// Batched pack, one workgroup per slice: sort the slice's squared singular
// values (descending, ties by index) in LDS, then gather its kept triplets.
template <class T>
__global__ __launch_bounds__(1024) void pack_batch(const PackSlice* __restrict__ ps) {
    __shared__ unsigned long long key[PMAX];
    __shared__ int idx[PMAX];
    const PackSlice d = ps[blockIdx.x];
    const SliceGeom g = d.g;
    const int64_t r = g.r, m = g.m, p = g.p;
    int np = 1;
    while (np < r) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        if (i < r) {
            double v = d.s2[i];
            if (!(v >= 0.0)) v = 0.0;
            v += 0.0;
            key[i] = ~(unsigned long long)__double_as_longlong(v);
        } else {
            key[i] = ~0ull;
        }
        idx[i] = i;
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < np / 2; t += blockDim.x) {
                const int i = 2 * j * (t / j) + (t % j);
                const bool up = (i & k) == 0;
                const unsigned long long ka = key[i], kb = key[i + j];
                const int ia = idx[i], ib = idx[i + j];
                const bool gt = (ka > kb) || (ka == kb && ia > ib);
                if (gt == up) { key[i] = kb; key[i + j] = ka; idx[i] = ib; idx[i + j] = ia; }
            }
            __syncthreads();
        }
    }
    const int64_t kr = *d.rho, off = *d.off;
    if (kr <= 0) return;
    if (off + kr > d.capacity) {
        if (threadIdx.x == 0) atomicExch(d.status, (int32_t)TSVDM_E_CAPACITY);
        return;
    }
    const T* Ab = static_cast<const T*>(d.A);
    const T* Wb = static_cast<const T*>(d.W);
    T* U = static_cast<T*>(d.U_pk) + m * off;
    T* G = static_cast<T*>(d.G_pk) + p * off;
    T* S = static_cast<T*>(d.S_pk) + off;
    for (int c = threadIdx.x; c < kr; c += blockDim.x)
        S[c] = static_cast<T>(sqrt(fmax(d.s2[idx[c]], 0.0)));
    const bool rows = g.rows != 0;
    for (int64_t e = threadIdx.x; e < kr * m; e += blockDim.x) {
        const int64_t a = e % m, c = e / m, j = idx[c];
        T v;
        if (rows) {
            v = Wb[j * r + a];
        } else {
            const double sg = sqrt(fmax(d.s2[j], 0.0));
            v = sg > 0.0 ? static_cast<T>((double)Ab[a + j * m] / sg) : T(0);
        }
        U[e] = v;
    }
    for (int64_t e = threadIdx.x; e < kr * p; e += blockDim.x) {
        const int64_t c = e % kr, b = e / kr, j = idx[c];
        T v;
        if (rows) {
            v = Ab[j + b * m];
        } else {
            const double sg = sqrt(fmax(d.s2[j], 0.0));
            v = static_cast<T>(sg * (double)Wb[b + j * r]);
        }
        G[e] = v;
    }
}

template <class T>
int pack_impl(const void* A, const void* W, const double* s2, int64_t m, int64_t p, int64_t n,
              const int32_t* rho, const int64_t* offsets, int64_t capacity, int first,
              void* U_pk, void* G_pk, void* S_pk, int32_t* status, void* ws, hipStream_t st) {
    const SliceGeom g = slice_geom(m, p);
    TSVDM_REQUIRE(g.r <= PMAX, TSVDM_E_SHAPE, "min(m, p) above 4096 is not supported by pack");
    Carver cv(ws);
    int32_t* perm = cv.carve<int32_t>((size_t)(g.r * n));
    pack_sort<T><<<(unsigned)n, 1024, 0, st>>>(s2, g.r, n, rho, offsets, capacity, first, perm,
                                                static_cast<T*>(S_pk), status);
    TSVDM_LAUNCH_CHECK();
    dim3 grid(64, (unsigned)n);
    pack_copy<T><<<grid, 256, 0, st>>>(static_cast<const T*>(A), static_cast<const T*>(W), s2, g,
                                       rho, offsets, capacity, first, perm,
                                       static_cast<T*>(U_pk), static_cast<T*>(G_pk));
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

}  // namespace

int run_pack_sort_f32(const double* s2, int64_t r, int64_t n, const int32_t* rho,
                      const int64_t* offsets, int64_t capacity, int32_t* perm, float* S_pk,
                      int32_t* status, hipStream_t st) {
    TSVDM_REQUIRE(r <= PMAX, TSVDM_E_SHAPE, "min(m, p) above 4096 is not supported by pack");
    pack_sort<float><<<(unsigned)n, 1024, 0, st>>>(s2, r, n, rho, offsets, capacity, 0, perm, S_pk, status);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

size_t pack_workspace_bytes(int64_t m, int64_t p, int64_t n) {
    const SliceGeom g = slice_geom(m, p);
    Carver cv(nullptr);
    cv.carve<int32_t>((size_t)(g.r * n));
    return cv.total();
}

int run_pack_from(const void* A, const void* W, const double* s2, int dt, int64_t m, int64_t p,
                  int64_t n, const int32_t* rho, const int64_t* offsets, int64_t capacity,
                  int first, void* U_pk, void* G_pk, void* S_pk, int32_t* status, void* ws,
                  hipStream_t st) {
    if (dt == TSVDM_F64)
        return pack_impl<double>(A, W, s2, m, p, n, rho, offsets, capacity, first, U_pk, G_pk,
                                 S_pk, status, ws, st);
    if (dt == TSVDM_F32)
        return pack_impl<float>(A, W, s2, m, p, n, rho, offsets, capacity, first, U_pk, G_pk,
                                S_pk, status, ws, st);
    set_error("pack supports F64 and F32 only");
    return TSVDM_E_UNSUPPORTED;
}

int run_pack(const void* A, const void* W, const double* s2, int dt, int64_t m, int64_t p,
             int64_t n, const int32_t* rho, const int64_t* offsets, int64_t capacity,
             void* U_pk, void* G_pk, void* S_pk, int32_t* status, void* ws, hipStream_t st) {
    return run_pack_from(A, W, s2, dt, m, p, n, rho, offsets, capacity, 0, U_pk, G_pk, S_pk,
                         status, ws, st);
}

int run_lowrank_gemm(const void* U_pk, const void* G_pk, int dt, int64_t m, int64_t p,
                     int64_t n, const int32_t* rho, const int64_t* offsets, int64_t capacity,
                     void* C, hipStream_t st) {
    // 64 x 128 output tiles (rows a of m, columns b of p)
    const int ta = (int)((m + 63) / 64), tb = (int)((p + 127) / 128);
    TSVDM_REQUIRE((int64_t)ta * tb < ((int64_t)1 << 31) && n < 65536, TSVDM_E_SHAPE,
                  "reconstruction grid too large");
    dim3 grid((unsigned)(ta * tb), (unsigned)n);
    if (dt == TSVDM_F64) {
        lowrank_gemm<double><<<grid, 256, 0, st>>>(static_cast<const double*>(U_pk),
                                                   static_cast<const double*>(G_pk), m, p, rho,
                                                   offsets, capacity, static_cast<double*>(C), ta);
    } else if (dt == TSVDM_F32) {
        lowrank_gemm<float><<<grid, 256, 0, st>>>(static_cast<const float*>(U_pk),
                                                  static_cast<const float*>(G_pk), m, p, rho,
                                                  offsets, capacity, static_cast<float*>(C), ta);
    } else {
        set_error("reconstruction supports F64 and F32 only");
        return TSVDM_E_UNSUPPORTED;
    }
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_pack_batch(int dt, const PackSlice* ps, int64_t nslices, hipStream_t st) {
    TSVDM_REQUIRE(nslices < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many slices");
    if (dt == TSVDM_F64) pack_batch<double><<<(unsigned)nslices, 1024, 0, st>>>(ps);
    else pack_batch<float><<<(unsigned)nslices, 1024, 0, st>>>(ps);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_lowrank_batch(int dt, const PackSlice* ps, const int4* tasks, int64_t ntasks,
                      hipStream_t st) {
    TSVDM_REQUIRE(ntasks < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many reconstruction tiles");
    if (dt == TSVDM_F64) lowrank_gemm_batch<double><<<(unsigned)ntasks, 256, 0, st>>>(ps, tasks);
    else lowrank_gemm_batch<float><<<(unsigned)ntasks, 256, 0, st>>>(ps, tasks);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

}  // namespace tsvdm

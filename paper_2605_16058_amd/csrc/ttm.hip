// Mode-3 tensor-times-matrix on MFMA (Section 2.1; Section 3.1).
//
// For a column-major m x p x n tensor the mode-3 unfolding is the (mp) x n
// matrix X whose column l is frontal slice l, so Y = X x_3 op(M) is the single
// GEMM  Y[row, i] = sum_l X[row, l] * op(M)[i, l]  with a huge row count
// R = mp and small N = K = n.  For a mode k of an order-d tensor the same
// GEMM runs on each of the P = n_{k+1} ... n_d contiguous blocks of
// R = n_1 ... n_{k-1} rows (Section 3.1, middle-mode TTM), blockIdx.y
// selecting the block.  Each workgroup computes a TR-row x TI-slice
// tile of Y in the transposed orientation Y^T = op(M) X^T so that the MFMA
// output lanes run along tensor rows and the stores coalesce.  Three tile
// shapes share one body (64x64, 128x32, 256x16: every wave owns 16 slices
// and four 16-row MFMA tiles); narrow shapes waste less work when n is small.
#include "common.h"
#include "kernels.h"

namespace tsvdm {

namespace {

// tile shape codes of the C ABI: 1 = 64x64, 2 = 128x32, 3 = 256x16
template <int SHAPE>
struct TileShape {
    static constexpr int TI = 64 >> (SHAPE - 1);  // output slices per workgroup
    static constexpr int TR = 64 << (SHAPE - 1);  // rows of the unfolding per workgroup
    static constexpr int WI = TI / 16;            // waves along slices
    static constexpr int WROWS = TR / (4 / WI);   // rows per wave (always 64)
};

int default_tile(int64_t n) { return n <= 16 ? 3 : (n <= 32 ? 2 : 1); }

// Tt[i*n + l] = scale * op(M)[i, l], stored in the LDS staging type.
template <class ST>
__global__ void ttm_prep(const double* __restrict__ M, int n, int transpose,
                         double scale, ST* __restrict__ Tt) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    int i = (int)(idx / n), l = (int)(idx % n);
    double v = transpose ? M[l + (int64_t)i * n] : M[i + (int64_t)l * n];
    Tt[idx] = static_cast<ST>(scale * v);
}

// KIND 0: plain MFMA in CT (double or float), K step 4.
// KIND 1: BF16 operands, FP32 accumulate, K step 32.
// KIND 2: split BF16 (hi*hi + hi*lo + lo*hi), FP32 accumulate, K step 32.
template <class CT, int KIND, int SHAPE>
struct TtmShared {
    static constexpr int KC = (KIND == 0) ? 16 : 32;
    CT Xs[KC][TileShape<SHAPE>::TR + 1];   // [l][row]
    CT Ts[TileShape<SHAPE>::TI][KC + 1];   // [i][l]
};

// Output tile (row tile rt, slice tile ct) of Y = X x_3 op(M).
template <class CT, int KIND, int SHAPE>
__device__ __forceinline__ void ttm_tile(TtmShared<CT, KIND, SHAPE>& sh, const void* __restrict__ X, int xdt,
                                         void* __restrict__ Y, int ydt, int64_t R, int n,
                                         const CT* __restrict__ Tt, int64_t rt, int ct) {
    constexpr int KC = TtmShared<CT, KIND, SHAPE>::KC;
    constexpr int TR = TileShape<SHAPE>::TR, TI = TileShape<SHAPE>::TI, WI = TileShape<SHAPE>::WI;
    typedef typename Acc<CT>::type AccT;
    auto& Xs = sh.Xs;
    auto& Ts = sh.Ts;
    const int64_t row0 = rt * TR;
    const int i0 = ct * TI;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int wi = wave % WI;                                // slice group of this wave
    const int wr0 = (wave / WI) * TileShape<SHAPE>::WROWS;  // first tile row of this wave

    AccT acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = zero4<AccT>();

    for (int l0 = 0; l0 < n; l0 += KC) {
        // stage X[row0 .. row0+TR-1, l0 .. l0+KC-1], coalesced along rows
#pragma unroll
        for (int e = tid; e < KC * TR; e += 256) {
            int r = e & (TR - 1), l = e / TR;
            int64_t row = row0 + r;
            int lg_ = l0 + l;
            CT v = 0;
            if (row < R && lg_ < n) v = ldg_as<CT>(X, row + (int64_t)lg_ * R, xdt);
            Xs[l][r] = v;
        }
        // stage op(M) block [i0 .. i0+TI-1, l0 .. l0+KC-1]
#pragma unroll
        for (int e = tid; e < KC * TI; e += 256) {
            int l = e % KC, i = e / KC;
            CT v = 0;
            if (i0 + i < n && l0 + l < n) v = Tt[(int64_t)(i0 + i) * n + l0 + l];
            Ts[i][l] = v;
        }
        __syncthreads();

        const int irow = wi * 16 + lr;  // output slice (A-operand row)
        if constexpr (KIND == 0) {
#pragma unroll
            for (int kk = 0; kk < KC; kk += 4) {
                CT a = Ts[irow][kk + lg];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    CT b = Xs[kk + lg][wr0 + t * 16 + lr];
                    acc[t] = mfma(a, b, acc[t]);
                }
            }
        } else {
            v8bf ahi, alo;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float x = Ts[irow][lg * 8 + e];
                __bf16 h = to_bf16(x);
                ahi[e] = h;
                alo[e] = to_bf16(x - static_cast<float>(h));
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                v8bf bhi, blo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    float x = Xs[lg * 8 + e][wr0 + t * 16 + lr];
                    __bf16 h = to_bf16(x);
                    bhi[e] = h;
                    blo[e] = to_bf16(x - static_cast<float>(h));
                }
                acc[t] = mfma_bf16(ahi, bhi, acc[t]);
                if constexpr (KIND == 2) {
                    acc[t] = mfma_bf16(ahi, blo, acc[t]);
                    acc[t] = mfma_bf16(alo, bhi, acc[t]);
                }
            }
        }
        __syncthreads();
    }

    // D lane layout: slice i0 + 16*wi + mfma row, row row0 + wr0 + 16*t + lr
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int64_t row = row0 + wr0 + t * 16 + lr;
        if (row >= R) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int i = i0 + wi * 16 + mfma_row<CT>(lg, v);
            if (i < n) stg_as(Y, row + (int64_t)i * R, ydt, (double)acc[t][v]);
        }
    }
}

template <class CT, int KIND, int SHAPE>
__global__ __launch_bounds__(256) void ttm_kernel(
    const void* __restrict__ X, int xdt, void* __restrict__ Y, int ydt,
    int64_t R, int n, const CT* __restrict__ Tt, int n_ct, int64_t n_rt) {
    __shared__ TtmShared<CT, KIND, SHAPE> sh;
    // block blockIdx.y of R x n elements
    const int64_t boff = (int64_t)blockIdx.y * R * n;
    X = static_cast<const char*>(X) + boff * (xdt == TSVDM_F64 ? 8 : 4);
    Y = static_cast<char*>(Y) + boff * (ydt == TSVDM_F64 ? 8 : 4);
    // XCD-aware block mapping: the n_ct column tiles of one row tile share
    // blockIdx % 8 (the same XCD and L2) and are dispatched together.
    const int64_t bid = blockIdx.x;
    const int64_t xcd = bid & 7, local = bid >> 3;
    const int64_t rt = (local / n_ct) * 8 + xcd;
    const int ct = (int)(local % n_ct);
    if (rt >= n_rt) return;
    ttm_tile<CT, KIND, SHAPE>(sh, X, xdt, Y, ydt, R, n, Tt, rt, ct);
}

// Batched form: task = (problem, row tile, slice tile), all of one shape.
template <class CT, int KIND, int SHAPE>
__global__ __launch_bounds__(256) void ttm_kernel_batch(const TtmProblem* __restrict__ probs,
                                                        const int4* __restrict__ tasks,
                                                        int xdt, int ydt) {
    __shared__ TtmShared<CT, KIND, SHAPE> sh;
    const int4 tk = tasks[blockIdx.x];
    const TtmProblem pr = probs[tk.x];
    ttm_tile<CT, KIND, SHAPE>(sh, pr.X, xdt, pr.Y, ydt, pr.R, pr.n,
                              static_cast<const CT*>(pr.Tt), (int64_t)tk.y, tk.z);
}

template <class ST>
__global__ void ttm_prep_batch(const TtmProblem* __restrict__ probs, int nprob, int transpose) {
    const TtmProblem pr = probs[blockIdx.x];
    const int n = pr.n;
    ST* Tt = static_cast<ST*>(pr.Tt);
    for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += blockDim.x) {
        const int i = (int)(idx / n), l = (int)(idx % n);
        const double v = transpose ? pr.M[l + (int64_t)i * n] : pr.M[i + (int64_t)l * n];
        Tt[idx] = static_cast<ST>(pr.scale * v);
    }
}

template <class CT, int KIND, int SHAPE>
int launch_tiles(const void* X, int xdt, void* Y, int ydt, int64_t R, int n, int64_t P,
                 const CT* Tt, hipStream_t st) {
    constexpr int TR = TileShape<SHAPE>::TR, TI = TileShape<SHAPE>::TI;
    int n_ct = (n + TI - 1) / TI;
    int64_t n_rt = (R + TR - 1) / TR;
    int64_t n_rt8 = (n_rt + 7) / 8 * 8;
    int64_t blocks = n_rt8 * n_ct;
    TSVDM_REQUIRE(blocks < (int64_t)1 << 31, TSVDM_E_SHAPE, "tensor too large for one launch");
    const size_t xes = xdt == TSVDM_F64 ? 8 : 4, yes = ydt == TSVDM_F64 ? 8 : 4;
    for (int64_t p0 = 0; p0 < P; p0 += 65535) {
        const int64_t pc = P - p0 < 65535 ? P - p0 : 65535;
        const void* Xp = static_cast<const char*>(X) + (size_t)(p0 * R * n) * xes;
        void* Yp = static_cast<char*>(Y) + (size_t)(p0 * R * n) * yes;
        ttm_kernel<CT, KIND, SHAPE><<<dim3((unsigned)blocks, (unsigned)pc), 256, 0, st>>>(
            Xp, xdt, Yp, ydt, R, n, Tt, n_ct, n_rt);
        TSVDM_LAUNCH_CHECK();
    }
    return TSVDM_OK;
}

template <class CT, int KIND>
int launch_ttm(const void* X, int xdt, void* Y, int ydt, int64_t R, int n, int64_t P,
               const double* M, int transpose, double scale, int tile, void* ws,
               hipStream_t st) {
    CT* Tt = static_cast<CT*>(ws);
    int64_t nn = (int64_t)n * n;
    ttm_prep<CT><<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(M, n, transpose, scale, Tt);
    TSVDM_LAUNCH_CHECK();
    switch (tile ? tile : default_tile(n)) {
        case 1: return launch_tiles<CT, KIND, 1>(X, xdt, Y, ydt, R, n, P, Tt, st);
        case 2: return launch_tiles<CT, KIND, 2>(X, xdt, Y, ydt, R, n, P, Tt, st);
        case 3: return launch_tiles<CT, KIND, 3>(X, xdt, Y, ydt, R, n, P, Tt, st);
        default: set_error("unknown transform tile shape"); return TSVDM_E_ARG;
    }
}

template <class CT, int KIND>
int launch_batch(const TtmProblem* probs, const int4* tasks, const int64_t* group, int xdt,
                 int ydt, hipStream_t st) {
    int64_t o = 0;
    for (int sh = 1; sh <= 3; ++sh) {
        const int64_t cnt = group[sh - 1];
        if (cnt > 0) {
            if (sh == 1) ttm_kernel_batch<CT, KIND, 1><<<(unsigned)cnt, 256, 0, st>>>(probs, tasks + o, xdt, ydt);
            else if (sh == 2) ttm_kernel_batch<CT, KIND, 2><<<(unsigned)cnt, 256, 0, st>>>(probs, tasks + o, xdt, ydt);
            else ttm_kernel_batch<CT, KIND, 3><<<(unsigned)cnt, 256, 0, st>>>(probs, tasks + o, xdt, ydt);
            TSVDM_LAUNCH_CHECK();
        }
        o += cnt;
    }
    return TSVDM_OK;
}

}  // namespace

size_t ttm_workspace_bytes(int64_t n) { return align_up((size_t)(n * n) * sizeof(double)); }

int run_ttm_mode(const void* X, int xdt, void* Y, int ydt, int64_t R, int64_t n, int64_t P,
                 const double* M, int transpose, double scale, int compute, int tile, void* ws,
                 hipStream_t st) {
    switch (compute) {
        case TSVDM_F64:
            return launch_ttm<double, 0>(X, xdt, Y, ydt, R, (int)n, P, M, transpose, scale, tile, ws, st);
        case TSVDM_F32:
            return launch_ttm<float, 0>(X, xdt, Y, ydt, R, (int)n, P, M, transpose, scale, tile, ws, st);
        case TSVDM_BF16:
            return launch_ttm<float, 1>(X, xdt, Y, ydt, R, (int)n, P, M, transpose, scale, tile, ws, st);
        case TSVDM_BF16X3:
            return launch_ttm<float, 2>(X, xdt, Y, ydt, R, (int)n, P, M, transpose, scale, tile, ws, st);
        default:
            set_error("unsupported compute dtype for the transform");
            return TSVDM_E_UNSUPPORTED;
    }
}

int run_ttm(const void* X, int xdt, void* Y, int ydt, int64_t m, int64_t p, int64_t n,
            const double* M, int transpose, double scale, int compute, int tile, void* ws,
            hipStream_t st) {
    return run_ttm_mode(X, xdt, Y, ydt, m * p, n, 1, M, transpose, scale, compute, tile, ws, st);
}

int ttm_resolve_tile(int tile, int64_t n) { return tile ? tile : default_tile(n); }

void ttm_tile_counts(int tile, int64_t R, int64_t n, int64_t* n_rt, int* n_ct) {
    const int sh = ttm_resolve_tile(tile, n);
    const int ti = 64 >> (sh - 1), tr = 64 << (sh - 1);
    *n_rt = (R + tr - 1) / tr;
    *n_ct = (int)((n + ti - 1) / ti);
}

int run_ttm_batch(const TtmProblem* probs, int nprob, const int4* tasks, const int64_t* group,
                  int xdt, int ydt, int compute, int transpose, hipStream_t st) {
    TSVDM_REQUIRE(group[0] + group[1] + group[2] < ((int64_t)1 << 31), TSVDM_E_SHAPE,
                  "too many transform tiles");
    switch (compute) {
        case TSVDM_F64:
            ttm_prep_batch<double><<<nprob, 256, 0, st>>>(probs, nprob, transpose);
            TSVDM_LAUNCH_CHECK();
            return launch_batch<double, 0>(probs, tasks, group, xdt, ydt, st);
        case TSVDM_F32:
            ttm_prep_batch<float><<<nprob, 256, 0, st>>>(probs, nprob, transpose);
            TSVDM_LAUNCH_CHECK();
            return launch_batch<float, 0>(probs, tasks, group, xdt, ydt, st);
        case TSVDM_BF16:
            ttm_prep_batch<float><<<nprob, 256, 0, st>>>(probs, nprob, transpose);
            TSVDM_LAUNCH_CHECK();
            return launch_batch<float, 1>(probs, tasks, group, xdt, ydt, st);
        case TSVDM_BF16X3:
            ttm_prep_batch<float><<<nprob, 256, 0, st>>>(probs, nprob, transpose);
            TSVDM_LAUNCH_CHECK();
            return launch_batch<float, 2>(probs, tasks, group, xdt, ydt, st);
        default:
            set_error("unsupported compute dtype for the transform");
            return TSVDM_E_UNSUPPORTED;
    }
}

}  // namespace tsvdm

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
// output lanes run along tensor rows and the stores coalesce.  Seven tile
// shapes share one body (every wave owns four 16-row MFMA tiles and 16, 32
// or 64 slices): narrow shapes waste less work when n is small, and wider
// waves read each LDS operand value once for more MFMAs.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace tsvdm {

namespace {

// tile shape codes of the C ABI (output slices x rows per workgroup, slices
// per wave; the waves own 64 rows each but in shape 8): 1 = 64x64, 2 =
// 32x128, 3 = 16x256 (16 slices per wave), 4 = 64x128, 5 = 32x256 (32), 6 =
// 128x128, 7 = 64x256 (64), 8 = 64x64 as 2 x 2 waves of 32 slices x 32
// rows.  A wider wave reads each LDS operand value once for more MFMAs.
__host__ __device__ constexpr int shape_ti(int s) {
    return s == 1 ? 64 : s == 2 ? 32 : s == 3 ? 16 : s == 4 ? 64 : s == 5 ? 32 : s == 6 ? 128 : 64;
}
__host__ __device__ constexpr int shape_tr(int s) {
    return s == 1 ? 64 : s == 2 ? 128 : s == 3 ? 256 : s == 4 ? 128 : s == 5 ? 256 : s == 6 ? 128 : s == 7 ? 256 : 64;
}
__host__ __device__ constexpr int shape_ws(int s) { return s <= 3 ? 16 : s <= 5 ? 32 : s <= 7 ? 64 : 32; }
__host__ __device__ constexpr int shape_wr(int s) { return s == 8 ? 32 : 64; }
template <int SHAPE>
struct TileShape {
    static constexpr int TI = shape_ti(SHAPE);        // output slices per workgroup
    static constexpr int TR = shape_tr(SHAPE);        // rows of the unfolding per workgroup
    static constexpr int WS = shape_ws(SHAPE);        // slices per wave
    static constexpr int NS = WS / 16;                // 16-slice MFMA tiles per wave
    static constexpr int WI = TI / WS;                // waves along slices
    static constexpr int WROWS = shape_wr(SHAPE);     // rows per wave
    static constexpr int NR = WROWS / 16;             // 16-row MFMA tiles per wave
    static_assert(WI * (TR / WROWS) == 4, "four waves");
};

// tile = 0: by n; FP32-operand forms take the wide waves once n > 32, the
// FP64 form (no registers for them) the 2 x 2 waves of 32 x 32
int default_tile(int64_t n, int compute) {
    if (n <= 16) return 3;
    if (n <= 32) return 2;
    if (compute == TSVDM_F64) return 8;
    return n <= 64 ? 4 : 6;
}

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
// Two stages of the K chunk: the next chunk is loaded into registers while
// the MFMAs consume the current one, then written to the other stage, so a
// chunk costs one barrier.  X rows are padded by 16 floats / 8 doubles, so
// that the two 16-lane row groups of an MFMA operand read hit disjoint banks.
template <class CT, int KIND, int SHAPE>
struct TtmShared {
    static constexpr int KC = (KIND == 0) ? 16 : 32;
    static constexpr int TR = TileShape<SHAPE>::TR, TI = TileShape<SHAPE>::TI;
    static constexpr int XLD = TR + (sizeof(CT) == 4 ? 16 : 8);
    CT Xs[2][KC][XLD];        // [stage][l][row]
    CT Ts[2][TI][KC + 1];     // [stage][i][l]
};

// Output tile (row tile rt, slice tile ct) of Y = X x_3 op(M); XT is the
// input element type.  VEC: R is a multiple of the 16-byte vector and X is
// 16-byte aligned, so that X loads as 16-byte vectors of consecutive rows.
template <class CT, class XT, int KIND, int SHAPE, bool VEC>
__device__ __forceinline__ void ttm_tile(TtmShared<CT, KIND, SHAPE>& sh, const XT* __restrict__ X,
                                         void* __restrict__ Y, int ydt, int64_t R, int n,
                                         const CT* __restrict__ Tt, int64_t rt, int ct) {
    typedef TtmShared<CT, KIND, SHAPE> S;
    constexpr int KC = S::KC, TR = S::TR, TI = S::TI;
    constexpr int WI = TileShape<SHAPE>::WI, WS = TileShape<SHAPE>::WS, NS = TileShape<SHAPE>::NS;
    constexpr int VW = VEC ? 16 / (int)sizeof(XT) : 1;     // X values per load
    constexpr int NXE = KC * TR / (256 * VW);              // X loads per thread and chunk
    constexpr int NTE = TI * KC / 256;                     // op(M) values per thread and chunk
    static_assert(NXE >= 1 && NTE >= 1, "tile too small for the staging map");
    typedef typename Acc<CT>::type AccT;
    const int64_t row0 = rt * TR;
    const int i0 = ct * TI;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int wi = wave % WI;                                // slice group of this wave
    const int wr0 = (wave / WI) * TileShape<SHAPE>::WROWS;  // first tile row of this wave

    constexpr int NR = TileShape<SHAPE>::NR;
    AccT acc[NS][NR];
#pragma unroll
    for (int u = 0; u < NS; ++u)
#pragma unroll
        for (int t = 0; t < NR; ++t) acc[u][t] = zero4<AccT>();

    // This thread's staging elements: X load k covers rows r .. r + VW - 1
    // of column l, consecutive threads along the rows; op(M) value k is
    // (slice i, column l), consecutive threads along l.  Rows and slices
    // outside the tensor are loaded from an index clamped into it (R >= VW)
    // and zeroed only when stored, so that nothing waits for the loads
    // before the MFMAs of the current chunk; the addresses are formed once
    // and advanced by a scalar offset per chunk (columns are clamped only in
    // a last, partial chunk).
    const XT* xb[NXE];
    const CT* tb[NTE];
    bool xok[NXE], tok[NTE];
#pragma unroll
    for (int k = 0; k < NXE; ++k) {
        const int e = tid + 256 * k;
        const int l = e / (TR / VW), r = (e % (TR / VW)) * VW;
        const int64_t row = row0 + r;
        xok[k] = row < R;
        xb[k] = X + (row < R ? row : R - VW) + (int64_t)l * R;
    }
#pragma unroll
    for (int k = 0; k < NTE; ++k) {
        const int e = tid + 256 * k;
        const int l = e % KC, i = e / KC;
        tok[k] = i0 + i < n;
        tb[k] = Tt + (int64_t)(i0 + i < n ? i0 + i : n - 1) * n + l;
    }
    // every row and slice of the tile inside the tensor: only the columns
    // of a partial last chunk are zeroed
    const bool inner = row0 + TR <= R && i0 + TI <= n;
    // FP64: two register sets, chunk c + 2 loaded while chunk c + 1 waits to
    // be stored, so each load has a whole chunk of MFMAs to arrive (FP32 has
    // no registers to spare for it: its wide tiles would lose waves)
    constexpr int PF = sizeof(CT) == 8 ? 2 : 1;
    XT xv[PF][NXE][VW];
    CT tv[PF][NTE];
    bool lok[PF][NXE], ltok[PF][NTE];
    auto load = [&](auto S, int l0) {
        constexpr int s = decltype(S)::value;
        const bool full = l0 + KC <= n;
#pragma unroll
        for (int k = 0; k < NXE; ++k) {
            const XT* src = xb[k] + (int64_t)l0 * R;
            lok[s][k] = true;
            if (!full) {
                const int l = (tid + 256 * k) / (TR / VW);
                lok[s][k] = l0 + l < n;
                if (!lok[s][k]) src = xb[k] + (int64_t)(n - 1 - l) * R;
            }
            if constexpr (VW == 4) {
                const float4 x = *reinterpret_cast<const float4*>(src);
                xv[s][k][0] = x.x; xv[s][k][1] = x.y; xv[s][k][2] = x.z; xv[s][k][3] = x.w;
            } else if constexpr (VW == 2) {
                const double2 x = *reinterpret_cast<const double2*>(src);
                xv[s][k][0] = x.x; xv[s][k][1] = x.y;
            } else {
                xv[s][k][0] = *src;
            }
        }
#pragma unroll
        for (int k = 0; k < NTE; ++k) {
            const CT* src = tb[k] + l0;
            ltok[s][k] = true;
            if (!full) {
                const int l = (tid + 256 * k) % KC;
                ltok[s][k] = l0 + l < n;
                if (!ltok[s][k]) src = tb[k] + (n - 1 - l);
            }
            tv[s][k] = *src;
        }
    };
    auto store = [&](auto S, int stg) {
        constexpr int s = decltype(S)::value;
#pragma unroll
        for (int k = 0; k < NXE; ++k) {
            const int e = tid + 256 * k;
            CT* dst = &sh.Xs[stg][e / (TR / VW)][(e % (TR / VW)) * VW];
            const bool ok = (inner || xok[k]) && lok[s][k];
#pragma unroll
            for (int q = 0; q < VW; ++q) dst[q] = ok ? static_cast<CT>(xv[s][k][q]) : CT(0);
        }
#pragma unroll
        for (int k = 0; k < NTE; ++k) {
            const int e = tid + 256 * k;
            sh.Ts[stg][e / KC][e % KC] = ((inner || tok[k]) && ltok[s][k]) ? tv[s][k] : CT(0);
        }
    };

    const int irow = wi * WS + lr;  // output slice (A-operand row) of the wave's first slice tile
    const int nchunk = (n + KC - 1) / KC;
    typedef std::integral_constant<int, 0> S0;
    typedef std::integral_constant<int, 1> S1;
    auto compute = [&](int stg) {
        const auto& Xs = sh.Xs[stg];
        const auto& Ts = sh.Ts[stg];
        if constexpr (KIND == 0) {
            // every operand of the chunk read before the first MFMA, so that
            // the LDS latency is paid once per chunk
            CT af[KC / 4][NS], bf[KC / 4][NR];
#pragma unroll
            for (int kq = 0; kq < KC / 4; ++kq) {
#pragma unroll
                for (int u = 0; u < NS; ++u) af[kq][u] = Ts[irow + 16 * u][4 * kq + lg];
#pragma unroll
                for (int t = 0; t < NR; ++t) bf[kq][t] = Xs[4 * kq + lg][wr0 + t * 16 + lr];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int kq = 0; kq < KC / 4; ++kq) {
#pragma unroll
                for (int u = 0; u < NS; ++u)
#pragma unroll
                    for (int t = 0; t < NR; ++t) acc[u][t] = mfma(af[kq][u], bf[kq][t], acc[u][t]);
            }
        } else {
            v8bf ahi[NS], alo[NS];
#pragma unroll
            for (int u = 0; u < NS; ++u)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    float x = Ts[irow + 16 * u][lg * 8 + e];
                    __bf16 h = to_bf16(x);
                    ahi[u][e] = h;
                    alo[u][e] = to_bf16(x - static_cast<float>(h));
                }
#pragma unroll
            for (int t = 0; t < NR; ++t) {
                v8bf bhi, blo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    float x = Xs[lg * 8 + e][wr0 + t * 16 + lr];
                    __bf16 h = to_bf16(x);
                    bhi[e] = h;
                    blo[e] = to_bf16(x - static_cast<float>(h));
                }
#pragma unroll
                for (int u = 0; u < NS; ++u) {
                    acc[u][t] = mfma_bf16(ahi[u], bhi, acc[u][t]);
                    if constexpr (KIND == 2) {
                        acc[u][t] = mfma_bf16(ahi[u], blo, acc[u][t]);
                        acc[u][t] = mfma_bf16(alo[u], bhi, acc[u][t]);
                    }
                }
            }
        }
    };
    // chunk c in LDS stage c & 1
    load(S0{}, 0);
    store(S0{}, 0);
    if constexpr (PF == 2) {
        // register set s holds chunk c + 1 during step c when c & 1 == s
        if (nchunk > 1) load(S0{}, KC);
        __syncthreads();
        auto step = [&](auto S, int c) {
            constexpr int s = decltype(S)::value;
            if (c + 2 < nchunk) load(std::integral_constant<int, 1 - s>{}, (c + 2) * KC);
            compute(c & 1);
            if (c + 1 < nchunk) store(S, (c + 1) & 1);
            __syncthreads();
        };
        for (int c = 0; c < nchunk; c += 2) {
            step(S0{}, c);
            if (c + 1 < nchunk) step(S1{}, c + 1);
        }
    } else {
        __syncthreads();
        for (int c = 0; c < nchunk; ++c) {
            if (c + 1 < nchunk) load(S0{}, (c + 1) * KC);
            compute(c & 1);
            if (c + 1 < nchunk) store(S0{}, (c + 1) & 1);
            __syncthreads();
        }
    }

    // D lane layout: slice i0 + WS*wi + 16*u + mfma row, row row0 + wr0 + 16*t + lr
#pragma unroll
    for (int t = 0; t < NR; ++t) {
        int64_t row = row0 + wr0 + t * 16 + lr;
        if (row >= R) continue;
#pragma unroll
        for (int u = 0; u < NS; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                int i = i0 + wi * WS + 16 * u + mfma_row<CT>(lg, v);
                if (i < n) stg_as(Y, row + (int64_t)i * R, ydt, (double)acc[u][t][v]);
            }
    }
}

template <class CT, class XT, int KIND, int SHAPE, bool VEC>
__global__ __launch_bounds__(256) void ttm_kernel(
    const XT* __restrict__ X, void* __restrict__ Y, int ydt,
    int64_t R, int n, const CT* __restrict__ Tt, int n_ct, int64_t n_rt) {
    __shared__ TtmShared<CT, KIND, SHAPE> sh;
    // block blockIdx.y of R x n elements
    const int64_t boff = (int64_t)blockIdx.y * R * n;
    X += boff;
    Y = static_cast<char*>(Y) + boff * (ydt == TSVDM_F64 ? 8 : 4);
    // XCD-aware block mapping: the n_ct column tiles of one row tile share
    // blockIdx % 8 (the same XCD and L2) and are dispatched together.
    const int64_t bid = blockIdx.x;
    const int64_t xcd = bid & 7, local = bid >> 3;
    const int64_t rt = (local / n_ct) * 8 + xcd;
    const int ct = (int)(local % n_ct);
    if (rt >= n_rt) return;
    ttm_tile<CT, XT, KIND, SHAPE, VEC>(sh, X, Y, ydt, R, n, Tt, rt, ct);
}

// Batched form: task = (problem, row tile, slice tile), all of one shape;
// element loads (the problems' row counts and alignments differ).
template <class CT, class XT, int KIND, int SHAPE>
__global__ __launch_bounds__(256) void ttm_kernel_batch(const TtmProblem* __restrict__ probs,
                                                        const int4* __restrict__ tasks, int ydt) {
    __shared__ TtmShared<CT, KIND, SHAPE> sh;
    const int4 tk = tasks[blockIdx.x];
    const TtmProblem pr = probs[tk.x];
    ttm_tile<CT, XT, KIND, SHAPE, false>(sh, static_cast<const XT*>(pr.X), pr.Y, ydt, pr.R, pr.n,
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

template <class CT, class XT, int KIND, int SHAPE>
int launch_tiles(const void* X, void* Y, int ydt, int64_t R, int n, int64_t P,
                 const CT* Tt, hipStream_t st) {
    constexpr int TR = TileShape<SHAPE>::TR, TI = TileShape<SHAPE>::TI;
    int n_ct = (n + TI - 1) / TI;
    int64_t n_rt = (R + TR - 1) / TR;
    int64_t n_rt8 = (n_rt + 7) / 8 * 8;
    int64_t blocks = n_rt8 * n_ct;
    TSVDM_REQUIRE(blocks < (int64_t)1 << 31, TSVDM_E_SHAPE, "tensor too large for one launch");
    const size_t yes = ydt == TSVDM_F64 ? 8 : 4;
    // every block of R x n elements starts 16-byte aligned when X does and R
    // is a multiple of the vector
    const bool vec = R % (int64_t)(16 / sizeof(XT)) == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0;
    for (int64_t p0 = 0; p0 < P; p0 += 65535) {
        const int64_t pc = P - p0 < 65535 ? P - p0 : 65535;
        const XT* Xp = static_cast<const XT*>(X) + (size_t)(p0 * R * n);
        void* Yp = static_cast<char*>(Y) + (size_t)(p0 * R * n) * yes;
        const dim3 grid((unsigned)blocks, (unsigned)pc);
        if (vec)
            ttm_kernel<CT, XT, KIND, SHAPE, true><<<grid, 256, 0, st>>>(Xp, Yp, ydt, R, n, Tt, n_ct, n_rt);
        else
            ttm_kernel<CT, XT, KIND, SHAPE, false><<<grid, 256, 0, st>>>(Xp, Yp, ydt, R, n, Tt, n_ct, n_rt);
        TSVDM_LAUNCH_CHECK();
    }
    return TSVDM_OK;
}

template <class CT, class XT, int KIND>
int launch_shape(const void* X, void* Y, int ydt, int64_t R, int n, int64_t P, const CT* Tt,
                 int tile, hipStream_t st) {
    const int compute = KIND == 1 ? TSVDM_BF16 : KIND == 2 ? TSVDM_BF16X3 : sizeof(CT) == 8 ? TSVDM_F64 : TSVDM_F32;
    switch (tile ? tile : default_tile(n, compute)) {
        case 1: return launch_tiles<CT, XT, KIND, 1>(X, Y, ydt, R, n, P, Tt, st);
        case 2: return launch_tiles<CT, XT, KIND, 2>(X, Y, ydt, R, n, P, Tt, st);
        case 3: return launch_tiles<CT, XT, KIND, 3>(X, Y, ydt, R, n, P, Tt, st);
        case 4: return launch_tiles<CT, XT, KIND, 4>(X, Y, ydt, R, n, P, Tt, st);
        case 5: return launch_tiles<CT, XT, KIND, 5>(X, Y, ydt, R, n, P, Tt, st);
        case 6: return launch_tiles<CT, XT, KIND, 6>(X, Y, ydt, R, n, P, Tt, st);
        case 7: return launch_tiles<CT, XT, KIND, 7>(X, Y, ydt, R, n, P, Tt, st);
        case 8: return launch_tiles<CT, XT, KIND, 8>(X, Y, ydt, R, n, P, Tt, st);
        default: set_error("unknown transform tile shape"); return TSVDM_E_ARG;
    }
}

template <class CT, int KIND>
int launch_ttm(const void* X, int xdt, void* Y, int ydt, int64_t R, int n, int64_t P,
               const double* M, int transpose, double scale, int tile, void* ws,
               hipStream_t st) {
    CT* Tt = static_cast<CT*>(ws);
    int64_t nn = (int64_t)n * n;
    ttm_prep<CT><<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(M, n, transpose, scale, Tt);
    TSVDM_LAUNCH_CHECK();
    if (xdt == TSVDM_F64) return launch_shape<CT, double, KIND>(X, Y, ydt, R, n, P, Tt, tile, st);
    return launch_shape<CT, float, KIND>(X, Y, ydt, R, n, P, Tt, tile, st);
}

template <class CT, class XT, int KIND>
int launch_batch_x(const TtmProblem* probs, const int4* tasks, const int64_t* group, int ydt,
                   hipStream_t st) {
    int64_t o = 0;
    for (int sh = 1; sh <= TTM_SHAPES; ++sh) {
        const int64_t cnt = group[sh - 1];
        if (cnt > 0) {
            const unsigned g = (unsigned)cnt;
            switch (sh) {
                case 1: ttm_kernel_batch<CT, XT, KIND, 1><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
                case 2: ttm_kernel_batch<CT, XT, KIND, 2><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
                case 3: ttm_kernel_batch<CT, XT, KIND, 3><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
                case 4: ttm_kernel_batch<CT, XT, KIND, 4><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
                case 5: ttm_kernel_batch<CT, XT, KIND, 5><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
                case 6: ttm_kernel_batch<CT, XT, KIND, 6><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
                case 7: ttm_kernel_batch<CT, XT, KIND, 7><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
                default: ttm_kernel_batch<CT, XT, KIND, 8><<<g, 256, 0, st>>>(probs, tasks + o, ydt); break;
            }
            TSVDM_LAUNCH_CHECK();
        }
        o += cnt;
    }
    return TSVDM_OK;
}

template <class CT, int KIND>
int launch_batch(const TtmProblem* probs, const int4* tasks, const int64_t* group, int xdt,
                 int ydt, hipStream_t st) {
    if (xdt == TSVDM_F64) return launch_batch_x<CT, double, KIND>(probs, tasks, group, ydt, st);
    return launch_batch_x<CT, float, KIND>(probs, tasks, group, ydt, st);
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

int ttm_resolve_tile(int tile, int64_t n, int compute) { return tile ? tile : default_tile(n, compute); }

void ttm_tile_counts(int shape, int64_t R, int64_t n, int64_t* n_rt, int* n_ct) {
    const int ti = shape_ti(shape), tr = shape_tr(shape);
    *n_rt = (R + tr - 1) / tr;
    *n_ct = (int)((n + ti - 1) / ti);
}

int run_ttm_batch(const TtmProblem* probs, int nprob, const int4* tasks, const int64_t* group,
                  int xdt, int ydt, int compute, int transpose, hipStream_t st) {
    int64_t total = 0;
    for (int s = 0; s < TTM_SHAPES; ++s) total += group[s];
    TSVDM_REQUIRE(total < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many transform tiles");
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

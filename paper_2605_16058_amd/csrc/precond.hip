// Slice SVDs of the mixed (FP32) path by way of the FP64 Gram matrix.
//
// A slice has r = min(m, p) Jacobi vectors x_v of length L = max(m, p): its
// rows when it is wide (m < p), its columns when it is tall.  Instead of
// rotating those long vectors, the slice is first reduced to an r x r
// triangular factor (Section 3.2 leaves the slice SVD method open; this is
// the Gram-matrix route for slices of any aspect ratio):
//   1. G = X X^T (r x r) in FP64 on MFMA.  Products of FP32 inputs are exact
//      in FP64, so G carries only the FP64 rounding of its sums.
//   2. L L^T = G + s I (Cholesky in FP64), s = (L + r) u64 trace(G): the
//      shift, about the size of G's own rounding, keeps the factorisation
//      defined for rank-deficient slices; a pivot that rounding still leaves
//      <= 0 gives a zero column.
//   3. One-sided Jacobi (FP32 vectors, FP64 angles) on the columns of L
//      without accumulating rotations: L Q = B with orthogonal columns, so
//      G + s I = B B^T and the normalised columns of B are the eigenvectors
//      of G, i.e. the singular vectors of the slice on its short side, with
//      sigma_j^2 = ||b_j||^2 - s.
//   4. Factors: wide (short side = U): G_i = U_rho^T A_hat_i; tall (short
//      side = V): G_i = S V_rho^T and U_i = A_hat_i V_rho S^-1, one product
//      with the slice itself.
// Eigenvalues of the FP64 Gram carry absolute errors of order u64 ||G||, so
// sigma_j moves by at most about u64 sigma_max^2 / sigma_j, and by
// sqrt(u64) sigma_max as sigma_j -> 0: far inside the FP32 path's value
// bound (2e-5 sigma_max).  The FP64 path does not use this form.
// Against rotating the slice itself, each Jacobi pair touches vectors of
// length r instead of L and no rotation matrix: for the 512 x 1024 climate
// slices 2 w^2 (2 r) instead of 2 w^2 (2 L + r) flops per rotating pair.
#include <mutex>

#include "angle.h"
#include "common.h"
#include "kernels.h"

namespace tsvdm {

namespace {

constexpr int GK = 16;   // positions per K chunk of the Gram
constexpr int CB = 16;   // Cholesky panel width
constexpr int FK = 32;   // vector indices per K chunk of the factor product

// lower-triangle tile q -> (ti, tj) with ti >= tj
__device__ __forceinline__ void tri_tile(int q, int& ti, int& tj) {
    int i = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= q) ++i;
    while (i * (i + 1) / 2 > q) --i;
    ti = i;
    tj = q - i * (i + 1) / 2;
}

// G(i, j) = sum_t X(i, t) X(j, t) for the 64 x 64 tile (ti, tj), ti >= tj,
// of slice blockIdx.x / ntri; X(v, t) = A[v vs + t es].  Wave w computes the
// rows j of 16 w .. 16 w + 15 of the transposed tile against all 64 i, so
// that the stores run along i (G is column-major: G[i + j r]).  The next K
// chunk is loaded into registers while the MFMAs of the current one run;
// two LDS buffers, one barrier per chunk.
template <class T>
__device__ __forceinline__ void gram_tile(const T* __restrict__ X, const SliceGeom& g, int ti, int tj,
                                          double* __restrict__ Gs) {
    __shared__ double sa[2][64][GK + 1];   // operand rows i
    __shared__ double sb[2][64][GK + 1];   // operand rows j
    const int64_t r = g.r, L = g.L, vs = g.vs, es = g.es;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
    const int64_t i0 = (int64_t)ti * 64, j0 = (int64_t)tj * 64;
    const bool rows = g.rows != 0;
    // this thread's four elements: rows -> one position, four consecutive
    // vectors; columns -> one vector, four consecutive positions
    const int v0 = rows ? (tid & 15) * 4 : (tid >> 2);
    const int t0 = rows ? (tid >> 4) : (tid & 3) * 4;
    const bool vec = (g.m % 4) == 0;   // 16-byte alignment of every group of four
    T ra[4], rb[4];
    auto load1 = [&](int64_t base_v, int64_t tc, T* out) {
        const int64_t v = base_v + v0, t = tc + t0;
        const T* src = X + v * vs + t * es;
        const bool full = rows ? (v + 3 < r && t < L) : (v < r && t + 3 < L);
        if (vec && full) {
            if constexpr (sizeof(T) == 4) {
                const float4 x = *reinterpret_cast<const float4*>(src);
                out[0] = x.x; out[1] = x.y; out[2] = x.z; out[3] = x.w;
            } else {
                const double2 x = *reinterpret_cast<const double2*>(src);
                const double2 y = *reinterpret_cast<const double2*>(src + 2);
                out[0] = x.x; out[1] = x.y; out[2] = y.x; out[3] = y.y;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t vq = rows ? v + q : v, tq = rows ? t : t + q;
                out[q] = (vq < r && tq < L) ? X[vq * vs + tq * es] : T(0);
            }
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int v = rows ? v0 + q : v0, t = rows ? t0 : t0 + q;
            sa[buf][v][t] = (double)ra[q];
            sb[buf][v][t] = (double)rb[q];
        }
    };
    v4d acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = zero4<v4d>();
    load1(i0, 0, ra);
    load1(j0, 0, rb);
    int buf = 0;
    for (int64_t tc = 0; tc < L; tc += GK) {
        put(buf);
        __syncthreads();
        if (tc + GK < L) {
            load1(i0, tc + GK, ra);
            load1(j0, tc + GK, rb);
        }
#pragma unroll
        for (int kk = 0; kk < GK; kk += 4) {
            const double a = sb[buf][16 * wave + lr][kk + lg];   // A(row j, k)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = mfma_f64(a, sa[buf][16 * c + lr][kk + lg], acc[c]);
        }
        buf ^= 1;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t i = i0 + 16 * c + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t j = j0 + 16 * wave + mfma_row<double>(lg, v);
            if (i < r && j < r) Gs[i + j * r] = acc[c][v];
        }
    }
}

template <class T>
__global__ __launch_bounds__(256) void pc_gram(const T* __restrict__ A, SliceGeom g, int ntri,
                                               double* __restrict__ G) {
    const int64_t s = blockIdx.x / ntri;
    int ti, tj;
    tri_tile((int)(blockIdx.x % ntri), ti, tj);
    gram_tile(A + s * g.m * g.p, g, ti, tj, G + s * g.r * g.r);
}

// batch: task (Gram slice, lower-triangle tile)
__global__ __launch_bounds__(256) void pc_gram_batch(const GramSlice* __restrict__ gs,
                                                     const int2* __restrict__ tasks) {
    const int2 t = tasks[blockIdx.x];
    const GramSlice d = gs[t.x];
    int ti, tj;
    tri_tile(t.y, ti, tj);
    gram_tile(d.A, d.g, ti, tj, d.G);
}

// P (G + s I) P^T = L L^T for the slice blockIdx.x, with diagonal pivoting:
// column k of L takes the remaining row with the largest updated diagonal
// (ties: the lowest position), so L's columns come in decreasing order of
// what they add.  Output B (r x r, column-major): column k of L with its rows
// at their original indices, so B B^T = G + s I, and B^T B = L^T L.  The
// Jacobi then orthogonalises the columns of B: with pivoting, L^T L is far
// closer to diagonal than G (the effect of the pivoted factor on one-sided
// Jacobi that Drmac and Veselic analyse), and on the test spectra the
// rounds need about a quarter fewer sweeps and rotations.
// Right-looking with panels of CB columns.  The trailing matrix keeps only
// the remaining rows, compacted in their original order, in column-major
// storage with leading dimension equal to its size (strict lower triangle;
// the updated diagonal lives in LDS): G itself at first, then alternately
// Ws and G (G is overwritten).  Per panel: CB pivot steps, then the panel's
// columns to B and one MFMA update of the remaining trailing matrix into
// the other buffer.  A pivot step is one barrier: every wave finds the
// pivot itself (an argmax over the whole diagonal, the same order in every
// wave), then the threads compute the new column (the trailing column of
// the pivot minus the panel's earlier columns).  So that a wave still
// searching never sees the step's own writes, the diagonal alternates
// between two LDS buffers and a pivot's mark carries its step.  A pivot <= 0 (rounding of a singular G + s I) gives a zero
// column; non-finite values stay non-finite.  Fixed operation order: the
// result does not depend on timing.
// Threads of a Cholesky workgroup (one workgroup per slice).  A launch of
// few slices, no more than the compute units can hold at once, relies on
// the waves of one workgroup to hide the latency of the trailing update's
// loads: sixteen waves for fewer than CHOL_WIDE_MAX slices of more than 256
// rows (0.68 ms less than four over 256 slices of 512, 7.2 ms less over 64
// of 1024).  A launch of many slices has the workgroups for that, and four
// waves keep its idle lanes and redundant pivot searches down (sixteen cost
// 4.2 ms over 3,566 slices of 257-384 rows, 18 ms over 49,640 of 73).  The
// trace keeps its four-wave summation order either way: the results are
// the same bits.
constexpr int64_t CHOL_WIDE_MAX = 512;
constexpr bool chol_wide(int64_t r, int64_t slices) { return r > 256 && slices < CHOL_WIDE_MAX; }

template <int MAXR, class OT, int NT>
__device__ __forceinline__ void chol_slice(double* __restrict__ Gs, int64_t r, double cshift,
                                           double* __restrict__ Ws, OT* __restrict__ Os,
                                           double* __restrict__ shift_out) {
    constexpr int PLD = CB + 1;                // column CB: the updated diagonal (even steps)
    constexpr int NW = NT / 64;
    constexpr int PER = (MAXR + NT - 1) / NT;  // positions per thread
    __shared__ double P[MAXR * PLD];           // panel columns by trailing position
    __shared__ double dodd[MAXR];              // the updated diagonal after odd steps
    __shared__ int opos[MAXR];                 // original index of each position
    __shared__ int keep[MAXR];                 // 0: remaining, c + 1: pivot of step c of this panel
    __shared__ int oldp[MAXR];                 // after a panel: old position of each new one
    __shared__ double rv[4];
    __shared__ int scan_w[NW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
    const int R = (int)r;
    // trace in a fixed order (the first four waves, 256 lanes)
    if (wave < 4) {
        double tr = 0.0;
        for (int j = tid; j < R; j += 256) tr += Gs[(int64_t)j * (R + 1)];
        for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off);
        if (lane == 0) rv[wave] = tr;
    }
    __syncthreads();
    const double sh = cshift * ((rv[0] + rv[1]) + (rv[2] + rv[3]));
    if (tid == 0) *shift_out = sh;
    for (int a = tid; a < R; a += NT) {
        opos[a] = a;
        P[a * PLD + CB] = Gs[(int64_t)a * (R + 1)] + sh;
    }
    // B starts at zero: a panel writes only the rows still remaining
    for (int64_t e = tid; e < (int64_t)R * R; e += NT) Os[e] = OT(0);
    __syncthreads();
    double* To = Gs;   // trailing matrix, strict lower triangle, leading dimension ldo
    double* Tn = Ws;
    int64_t ldo = R;
    int n = R, k = 0;
    while (n > 0) {
        const int nc = n < CB ? n : CB;   // nc < CB only for the last panel
        for (int a = tid; a < n; a += NT) keep[a] = 0;
        __syncthreads();
        for (int c = 0; c < nc; ++c) {
            // the updated diagonal: read from one buffer, written to the other
            const double* dcur = (c & 1) ? dodd : P + CB;
            double* dnxt = (c & 1) ? P + CB : dodd;
            const int dst = (c & 1) ? 1 : PLD;   // stride of dcur
            const int dsn = (c & 1) ? PLD : 1;   // stride of dnxt
            // 1. pivot, in every wave: the largest updated diagonal among the
            //    remaining rows (ties: the lowest position; NaN counts as
            //    -inf; some row always remains).  A mark c + 1 is this
            //    step's own pivot, set by a faster wave: still a candidate.
            double bv = -INFINITY;
            int bi = 0x7fffffff;
            for (int a = lane; a < n; a += 64) {
                const int kp = keep[a];
                if (kp != 0 && kp <= c) continue;
                double v = dcur[a * dst];
                v = (v == v) ? v : -INFINITY;
                if (v > bv || (v == bv && a < bi)) { bv = v; bi = a; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int oi = __shfl_xor(bi, off);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            const int q = bi;
            // 2. column c: l_a = (T(a, q) - sum_{c' < c} l_a,c' l_q,c') / l_qq
            // a pivot <= 0 gives a zero column; NaN and Inf travel on (x 0)
            // so that the Jacobi reports them
            const double dq = dcur[q * dst];
            const double lqq = dq > 0.0 ? sqrt(dq) : dq * 0.0;
            for (int a = tid; a < n; a += NT) {
                if (a == q) {
                    P[a * PLD + c] = lqq;
                    keep[a] = c + 1;
                } else if (keep[a]) {
                    P[a * PLD + c] = 0.0;   // pivoted earlier in this panel
                } else {
                    // the trailing entry's load is issued first and the
                    // panel's dot product (two chains) runs while it travels
                    const double tq = a > q ? To[a + (int64_t)q * ldo] : To[q + (int64_t)a * ldo];
                    double d0 = 0.0, d1 = 0.0;
                    int cc = 0;
                    for (; cc + 1 < c; cc += 2) {
                        d0 = fma(P[a * PLD + cc], P[q * PLD + cc], d0);
                        d1 = fma(P[a * PLD + cc + 1], P[q * PLD + cc + 1], d1);
                    }
                    if (cc < c) d0 = fma(P[a * PLD + cc], P[q * PLD + cc], d0);
                    const double t = tq - (d0 + d1);
                    const double l = lqq > 0.0 ? t / lqq : t * 0.0;
                    P[a * PLD + c] = l;
                    dnxt[a * dsn] = dcur[a * dst] - l * l;
                }
            }
            __syncthreads();
        }
        // 3. the panel's columns of B, rows at their original indices (the
        //    rows factored in earlier panels keep their zeros)
        for (int c = 0; c < nc; ++c)
            for (int a = tid; a < n; a += NT) Os[opos[a] + (int64_t)(k + c) * R] = (OT)P[a * PLD + c];
        // 4. new positions of the remaining rows (order kept): thread tid
        //    takes positions [tid PER, tid PER + PER)
        const int nn = n - nc;
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int a = tid * PER + j;
            if (a < n && keep[a] == 0) ++cnt;
        }
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off);
            if (lane >= off) incl += y;
        }
        if (lane == 63) scan_w[wave] = incl;
        __syncthreads();
        int base = incl - cnt;
        for (int w = 0; w < wave; ++w) base += scan_w[w];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int a = tid * PER + j;
            if (a < n) {
                if (keep[a] == 0) {
                    oldp[base] = a;
                    ++base;
                }
            }
        }
        __syncthreads();
        // 5. Tn(a, b) = To(oldp a, oldp b) - sum_c P(oldp a, c) P(oldp b, c)
        //    for a > b < nn (only after a full panel: nn > 0 implies nc = CB).
        //    16 x 16 tiles of the lower triangle, four per wave at a time
        //    (tiles t0, t0 + NW, t0 + 2 NW, t0 + 3 NW for wave t0),
        //    their loads issued before the MFMAs; lane (lr, lg) holds rows
        //    16 ta + lr of columns 16 tb + lg + 4 v, so a store instruction
        //    writes 16 consecutive rows of four columns.
        if (nn > 1) {
            const int nt = (nn + 15) / 16, ntri = nt * (nt + 1) / 2;
            for (int t0 = wave; t0 < ntri; t0 += 4 * NW) {
                double tv[4][4];
                v4d acc[4];
                int ra[4], cb[4];
                bool vt[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int tq = t0 + NW * u;
                    int ti = 0, tj = 0;
                    vt[u] = tq < ntri;
                    if (vt[u]) tri_tile(tq, ti, tj);
                    ra[u] = 16 * ti + lr;   // this lane's row (new position)
                    cb[u] = 16 * tj;        // the tile's first column
                    const bool va = vt[u] && ra[u] < nn;
                    const int oa = va ? oldp[ra[u]] : 0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int b = cb[u] + lg + 4 * v;
                        tv[u][v] = (va && b < ra[u]) ? To[oa + (int64_t)oldp[b] * ldo] : 0.0;
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int rb = cb[u] + lr;   // the tile column this lane feeds
                    const bool va = vt[u] && ra[u] < nn, vb = vt[u] && rb < nn;
                    const int oa = va ? oldp[ra[u]] : 0, ob = vb ? oldp[rb] : 0;
                    v4d z = zero4<v4d>();
#pragma unroll
                    for (int s4 = 0; s4 < CB / 4; ++s4) {
                        const double xa = vb ? P[ob * PLD + 4 * s4 + lg] : 0.0;   // A(lr, k): column rows
                        const double xb = va ? P[oa * PLD + 4 * s4 + lg] : 0.0;   // B(k, lr): tile rows
                        z = mfma_f64(xa, xb, z);
                    }
                    acc[u] = z;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!vt[u] || ra[u] >= nn) continue;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int b = cb[u] + lg + 4 * v;
                        if (b < ra[u]) Tn[ra[u] + (int64_t)b * nn] = tv[u][v] - acc[u][v];
                    }
                }
            }
        }
        __syncthreads();
        // 6. per-position data to the new positions (through registers)
        int ov[PER];
        double dv[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int a = tid + NT * j;
            if (a < nn) {
                ov[j] = opos[oldp[a]];
                dv[j] = P[oldp[a] * PLD + CB];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int a = tid + NT * j;
            if (a < nn) {
                opos[a] = ov[j];
                P[a * PLD + CB] = dv[j];
            }
        }
        __syncthreads();
        double* const nxt = (Tn == Ws) ? Gs : Ws;
        To = Tn;
        Tn = nxt;
        ldo = nn;
        n = nn;
        k += nc;
    }
}

template <int MAXR, class OT, int NT>
__global__ __launch_bounds__(NT) void pc_chol(double* __restrict__ G, int64_t r, double cshift,
                                               double* __restrict__ Lw, OT* __restrict__ Lo,
                                               double* __restrict__ shift) {
    const int64_t s = blockIdx.x;
    chol_slice<MAXR, OT, NT>(G + s * r * r, r, cshift, Lw + s * r * r, Lo + s * r * r, shift + s);
}

// batch: one workgroup per Gram slice listed (one size class, r <= MAXR)
template <int MAXR, int NT>
__global__ __launch_bounds__(NT) void pc_chol_batch(const GramSlice* __restrict__ gs,
                                                     const int* __restrict__ list) {
    const GramSlice d = gs[list[blockIdx.x]];
    const double cshift = (double)(d.g.L + d.g.r) * 1.1102230246251565e-16;
    chol_slice<MAXR, float, NT>(d.G, d.g.r, cshift, d.Lw, d.B, d.shift);
}

// seat -> player of the circle tournament over N (even) players in round
// `round` (seat 0 fixed, the others advance one seat per round)
__device__ __forceinline__ int lds_player(int seat, int round, int N) {
    if (seat == 0) return 0;
    int t = seat - 1 + round;
    if (t >= N - 1) t -= N - 1;
    return t + 1;
}

// x from lane (lane ^ 1), (lane ^ 2), or its mirror in the 8- or 16-lane
// row, by DPP (two 32-bit moves for a double)
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 16 lanes of a DPP row.  Every step adds the value of a
// partner lane under an involution (xor 1, xor 2, mirror in 8, mirror in
// 16), so the two lanes of a pair add the same two numbers and, addition
// being commutative, every lane ends with the same bits.
__device__ __forceinline__ double row_sum16(double x) {
    x += dpp_move<0xB1>(x);    // quad_perm [1, 0, 3, 2]
    x += dpp_move<0x4E>(x);    // quad_perm [2, 3, 0, 1]
    x += dpp_move<0x141>(x);   // row_half_mirror
    x += dpp_move<0x140>(x);   // row_mirror
    return x;
}

// One-sided Jacobi held in LDS for factors of at most RMAX columns: the
// r x r factor of slice blockIdx.x stays in LDS (r x (r + 1) floats,
// dynamic) for all its sweeps: one workgroup per slice, no launch per
// round.  A round of the circle tournament pairs the columns disjointly;
// sixteen groups of 16 lanes (one DPP row each) take its pairs, group g
// the pairs g, g + 16, ..., two at a time so that their latencies overlap
// (a wave skips the pair slots none of its four groups has, so that at
// r = 73, 37 pairs, two waves work on three pairs and two on two): the
// three dot products in FP64
// from exact FP32 products (lane i holds elements i, i + 16, ...), summed
// over the row by DPP, the FP64 angle and the FP32 rotation of the two
// columns; one barrier per round.  The slice has converged after the first
// sweep whose largest |cos| is <= tol; one more sweep then rotates every
// pair not orthogonal to rounding, because the short-side vectors' residual
// non-orthogonality is amplified by sigma_i / sigma_j in the long-side
// factor (U = A V / sigma for tall slices, V = G^T / sigma for wide ones).
// Then s2 = max(||b_j||^2 - shift, 0) in FP64 and flag = 0 (converged), 1
// (sweep limit) or 2 (NaN / Inf met).
template <int RMAX>
__device__ __forceinline__ void jacobi_lds_slice(float* __restrict__ Bs, int rr, double tol, int max_sweeps,
                                                 double shs, double* __restrict__ s2s,
                                                 int32_t* __restrict__ flag_out) {
    constexpr int E = RMAX / 16;     // elements per lane and column
    extern __shared__ float X[];     // column j at X[j * RP]
    __shared__ double gmax[16];
    __shared__ int gbad[16];
    const int tid = threadIdx.x, grp = tid >> 4, l = tid & 15;
    const int grp0 = grp & ~3;       // first group of this wave
    const int RP = rr + 1;
    for (int idx = tid; idx < rr * rr; idx += 256) {
        const int j = idx / rr, i = idx - j * rr;
        X[j * RP + i] = Bs[idx];
    }
    __syncthreads();
    const int R = rr + (rr & 1);
    const int NP = R / 2;            // pairs per round
    bool conv = false, bad = false, polish = false;
    for (int sw = 0; sw < max_sweeps + 1; ++sw) {
        if (sw == max_sweeps && !conv) break;
        const double thr = polish ? 0.0 : tol;
        double mx = 0.0;
        for (int rnd = 0; rnd < R - 1; ++rnd) {
            for (int k0 = 0; grp0 + k0 < NP; k0 += 32) {
                // this group's pairs grp + k0 and grp + k0 + 16 of the round
                // (either may be the padding player's or absent): uniform in
                // the group; slot u is worked on by the wave when one of its
                // groups has it
                int pp[2], qq[2];
                bool use[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int k = grp + k0 + 16 * u;
                    pp[u] = lds_player(k, rnd, R);
                    qq[u] = lds_player(R - 1 - k, rnd, R);
                    use[u] = k < NP && pp[u] < rr && qq[u] < rr;
                }
                float vp[2][E], vq[2][E];
                double app[2], aqq[2], apq[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (grp0 + k0 + 16 * u >= NP) continue;
                    const float* xp = X + (use[u] ? pp[u] : 0) * RP;
                    const float* xq = X + (use[u] ? qq[u] : 0) * RP;
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int i = l + 16 * e;
                        const bool ok = use[u] && i < rr;
                        vp[u][e] = ok ? xp[i] : 0.0f;
                        vq[u][e] = ok ? xq[i] : 0.0f;
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (grp0 + k0 + 16 * u >= NP) continue;
                    double a0 = 0.0, b0 = 0.0, c0 = 0.0;
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const double a = vp[u][e], b = vq[u][e];
                        a0 = fma(a, a, a0);
                        b0 = fma(b, b, b0);
                        c0 = fma(a, b, c0);
                    }
                    app[u] = row_sum16(a0);
                    aqq[u] = row_sum16(b0);
                    apq[u] = row_sum16(c0);
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (!use[u]) continue;
                    if (!(app[u] + aqq[u] + fabs(apq[u]) < INFINITY)) { bad = true; continue; }
                    const double den = app[u] * aqq[u];
                    const double cs = den > 0.0 ? fabs(apq[u]) / sqrt(den) : 0.0;
                    mx = fmax(mx, cs);
                    if (cs > thr) {
                        double c, sn;
                        jacobi_angle(app[u], aqq[u], apq[u], true, c, sn);
                        const float cf = (float)c, sf = (float)sn;
                        float* xp = X + pp[u] * RP;
                        float* xq = X + qq[u] * RP;
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const int i = l + 16 * e;
                            if (i < rr) {
                                xp[i] = cf * vp[u][e] - sf * vq[u][e];
                                xq[i] = sf * vp[u][e] + cf * vq[u][e];
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (l == 0) { gmax[grp] = mx; gbad[grp] = bad ? 1 : 0; }
        __syncthreads();
        double m = 0.0;
        int anybad = 0;
        for (int g2 = 0; g2 < 16; ++g2) { m = fmax(m, gmax[g2]); anybad |= gbad[g2]; }
        __syncthreads();   // gmax is rewritten by the next sweep
        if (anybad) { bad = true; break; }
        if (polish) break;
        conv = m <= tol;
        polish = conv;
    }
    // squared norms (fixed order: lane sums, then the row sum) and the
    // factor back to memory
    for (int j = grp; j < rr; j += 16) {
        double a = 0.0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = l + 16 * e;
            if (i < rr) { const double v = X[j * RP + i]; a = fma(v, v, a); }
        }
        a = row_sum16(a);
        if (l == 0) { const double v = a - shs; s2s[j] = v > 0.0 ? v : 0.0; }
    }
    for (int idx = tid; idx < rr * rr; idx += 256) {
        const int j = idx / rr, i = idx - j * rr;
        Bs[idx] = X[j * RP + i];
    }
    if (tid == 0) *flag_out = bad ? 2 : (conv ? 0 : 1);
}

template <int RMAX>
__global__ __launch_bounds__(256) void pc_jacobi_lds(float* __restrict__ B, int64_t r, double tol,
                                                     int max_sweeps, const double* __restrict__ shift,
                                                     double* __restrict__ s2, int32_t* __restrict__ flag) {
    const int64_t s = blockIdx.x;
    jacobi_lds_slice<RMAX>(B + s * r * r, (int)r, tol, max_sweeps, shift[s], s2 + s * r, flag + s);
}

// batch: the Gram slices listed in `list` (one size class of r)
template <int RMAX>
__global__ __launch_bounds__(256) void pc_jacobi_lds_batch(const GramSlice* __restrict__ gs,
                                                           const int* __restrict__ list, int max_sweeps) {
    const GramSlice d = gs[list[blockIdx.x]];
    jacobi_lds_slice<RMAX>(d.B, (int)d.g.r, d.tol, max_sweeps, *d.shift, d.s2, d.flag);
}

// batch: status word from the Gram slices' flags
__global__ void pc_gram_status(const GramSlice* __restrict__ gs, int64_t n, int32_t* __restrict__ status) {
    __shared__ int nf, nc;
    if (threadIdx.x == 0) { nf = 0; nc = 0; }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int f = *gs[i].flag;
        if (f == 2) atomicOr(&nf, 1);
        else if (f == 1) atomicOr(&nc, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *status = nf ? TSVDM_E_NONFINITE : (nc ? TSVDM_E_NOCONV : TSVDM_OK);
}

__global__ void pc_flags_status(const int32_t* __restrict__ flag, int64_t n, int32_t* __restrict__ status) {
    __shared__ int nf, nc;
    if (threadIdx.x == 0) { nf = 0; nc = 0; }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        if (flag[i] == 2) atomicOr(&nf, 1);
        else if (flag[i] == 1) atomicOr(&nc, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *status = nf ? TSVDM_E_NONFINITE : (nc ? TSVDM_E_NOCONV : TSVDM_OK);
}

// s2 <- max(s2 - shift, 0) per slice: squared singular values of the slice
// from the squared norms of B (||b_j||^2 = sigma_j^2 + s).
__global__ void pc_unshift(double* __restrict__ s2, const double* __restrict__ shift, int64_t r,
                           int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= r * n) return;
    const double v = s2[idx] - shift[idx / r];
    s2[idx] = v > 0.0 ? v : 0.0;
}

// batch: pc_unshift for Gram slices whose Jacobi ran in the block rounds,
// one workgroup per slice
__global__ __launch_bounds__(256) void pc_unshift_batch(const GramSlice* __restrict__ gs) {
    const GramSlice d = gs[blockIdx.x];
    const double sh = *d.shift;
    for (int64_t j = threadIdx.x; j < d.g.r; j += blockDim.x) {
        const double v = d.s2[j] - sh;
        d.s2[j] = v > 0.0 ? v : 0.0;
    }
}

// Preconditioned rotation form: W (r x r per slice) = the columns of B
// scaled to unit norm.  A zero column comes only from a zero slice (the
// shift then is 0 and so is every column): it becomes the unit vector e_j,
// so that W = I there.  A non-finite norm sets *flag to TSVDM_E_NONFINITE
// unless it already holds a condition.
template <class BT, class T>
__global__ __launch_bounds__(256) void pc_normalize(const BT* __restrict__ B, int64_t r, T* __restrict__ W,
                                                    int32_t* __restrict__ flag) {
    __shared__ double red[256];
    const int64_t j = blockIdx.x, s = blockIdx.y;
    const BT* b = B + s * r * r + j * r;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < r; i += 256) {
        const double x = (double)b[i];
        acc = fma(x, x, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double n2 = red[0];
    const bool ok = n2 > 0.0 && isfinite(n2);
    if (!isfinite(n2) && threadIdx.x == 0) atomicCAS(flag, (int32_t)TSVDM_OK, (int32_t)TSVDM_E_NONFINITE);
    const double inv = ok ? 1.0 / sqrt(n2) : 0.0;
    T* w = W + s * r * r + j * r;
    if (n2 == 0.0)
        for (int64_t i = threadIdx.x; i < r; i += 256) w[i] = i == j ? T(1) : T(0);
    else
        for (int64_t i = threadIdx.x; i < r; i += 256) w[i] = (T)((double)b[i] * inv);
}

// In place on C = W^T W (lower triangle read): S = (3 I - C) / 2 in both
// triangles.  One Newton-Schulz step W <- W S maps W^T W = I + E to
// I - (3/4) E^2 + O(E^3): W converges quadratically to the orthogonal polar
// factor of the starting W.  Thread (i >= j) reads only its own element.
__global__ void pc_ns_coef(double* __restrict__ C, int64_t r, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r * r * n) return;
    const int64_t s = e / (r * r), rem = e - s * r * r, j = rem / r, i = rem - j * r;
    if (i < j) return;
    double* c = C + s * r * r;
    const double v = c[i + j * r];
    const double out = i == j ? 0.5 * (3.0 - v) : -0.5 * v;
    c[i + j * r] = out;
    c[j + i * r] = out;
}

// Before the last Newton-Schulz step: rho[s] = r where max |C - I| (lower
// triangle of C = W^T W) exceeds thr, else 0 (the step's product then
// leaves that slice to pc_ns_keep); one workgroup per slice.
__global__ __launch_bounds__(256) void pc_ns_check(const double* __restrict__ C, int64_t r, double thr,
                                                   int32_t* __restrict__ rho) {
    __shared__ double red[4];
    const int64_t s = blockIdx.x;
    const double* c = C + s * r * r;
    double mx = 0.0;
    for (int64_t e = threadIdx.x; e < r * r; e += 256) {
        const int64_t j = e / r, i = e - j * r;
        if (i >= j) {
            const double d = fabs(c[e] - (i == j ? 1.0 : 0.0));
            mx = (d > mx || d != d) ? d : mx;   // NaN wins: the step then runs and keeps it
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(mx, off);
        mx = (o > mx || o != o) ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < 4; ++w) m = (red[w] > m || red[w] != red[w]) ? red[w] : m;
        rho[s] = (m > thr || m != m) ? (int32_t)r : 0;
    }
}

// W_next = W_cur for the slices whose last step was skipped (rho[s] == 0)
__global__ void pc_ns_keep(const double* __restrict__ cur, double* __restrict__ nxt,
                           const int32_t* __restrict__ rho, int64_t r, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r * r * n) return;
    if (rho[e / (r * r)] == 0) nxt[e] = cur[e];
}

// Ut = W^T per r x r slice
template <class T>
__global__ void pc_transpose(const T* __restrict__ W, int64_t r, int64_t n, T* __restrict__ Ut) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= r * r * n) return;
    const int64_t s = e / (r * r), rem = e - s * r * r, j = rem / r, i = rem - j * r;
    Ut[s * r * r + j + i * r] = W[e];
}

// rho[i] = r, off[i] = i r: every slice's full-rank block for the product
// that applies W to the slice
__global__ void pc_rank_full(int32_t* __restrict__ rho, int64_t* __restrict__ off, int64_t r, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rho[i] = (int32_t)r;
    if (i <= n) off[i] = i * r;
}

// status <- the first stage's condition when the second reported none
__global__ void pc_merge_status(int32_t* __restrict__ status, const int32_t* __restrict__ first) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && *status == TSVDM_OK) *status = *first;
}

// Short-side factor from B: kept column c (sorted position c, index j =
// perm[c]) is b_j / ||b_j||, ||b_j||^2 = s2_j + shift.  Wide slices: column
// c of U_pk (m x rho); tall slices: row c of G_pk (rho x p) scaled by sigma_c.
__global__ __launch_bounds__(256) void pc_pack_short(const float* __restrict__ B, const double* __restrict__ s2,
                                                     const double* __restrict__ shift, SliceGeom g,
                                                     const int32_t* __restrict__ rho,
                                                     const int64_t* __restrict__ offsets, int64_t capacity,
                                                     const int32_t* __restrict__ perm,
                                                     float* __restrict__ U_pk, float* __restrict__ G_pk) {
    const int64_t s = blockIdx.y;
    const int64_t kr = rho[s], off = offsets[s], r = g.r;
    if (kr <= 0 || off + kr > capacity) return;
    const float* Bs = B + s * r * r;
    const double* s2b = s2 + s * r;
    const double shs = shift[s];
    const int32_t* pr = perm + s * r;
    for (int64_t c = blockIdx.x; c < kr; c += gridDim.x) {
        const int64_t j = pr[c];
        const double sg2 = s2b[j] > 0.0 ? s2b[j] : 0.0;
        const double nb = sqrt(sg2 + shs);
        const double scale = nb > 0.0 ? (g.rows ? 1.0 : sqrt(sg2)) / nb : 0.0;
        const float* b = Bs + j * r;
        if (g.rows) {
            float* u = U_pk + g.m * off + c * g.m;
            for (int64_t a = threadIdx.x; a < r; a += blockDim.x) u[a] = (float)((double)b[a] * scale);
        } else {
            float* gr = G_pk + g.p * off + c;   // row c of the kr x p block (leading dim kr)
            for (int64_t t = threadIdx.x; t < r; t += blockDim.x) gr[t * kr] = (float)((double)b[t] * scale);
        }
    }
}

// Long-side factor by one product with the slice:
//   wide: G_pk(c, t) = sum_v u_c(v) X(v, t)            (rho x p, leading dim rho)
//   tall: U_pk(t, c) = sum_v X(v, t) v_c(v) / sigma_c  (m x rho)
// with u_c = v_c = b_perm(c) / ||b_perm(c)|| and X(v, t) = A[v vs + t es].
// Tile: 64 kept columns c x 64 positions t; wave w owns the output rows
// 16 w .. 16 w + 15 against all 64 columns, the MFMA output lanes running
// along the stored contiguous index (c for wide, t for tall).  K chunks of
// FK vector indices v, loaded into registers one chunk ahead.
template <bool ROWS>
__device__ __forceinline__ void factor_tile(const float* __restrict__ X, const float* __restrict__ Bs,
                                            const double* __restrict__ s2s, double shs, const SliceGeom& g,
                                            int64_t kr, int64_t off, int64_t capacity,
                                            const int32_t* __restrict__ perm_s, int tc_idx, int tt_idx,
                                            float* __restrict__ out) {
    __shared__ float sx[2][64][FK + 1];   // X(v, t): [t][v]
    __shared__ float sbk[2][64][FK + 1];  // b_perm(c)(v): [c][v]
    __shared__ double scl[64];
    __shared__ int jc[64];
    const int64_t c0 = (int64_t)tc_idx * 64, t0 = (int64_t)tt_idx * 64;
    if (kr <= 0 || off + kr > capacity || c0 >= kr) return;
    const int64_t r = g.r, L = g.L, vs = g.vs, es = g.es;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
    if (tid < 64) {
        const int64_t c = c0 + tid;
        int j = 0;
        double sc = 0.0;
        if (c < kr) {
            j = perm_s[c];
            const double sg2 = s2s[j] > 0.0 ? s2s[j] : 0.0;
            const double nb = sqrt(sg2 + shs);
            const double sg = sqrt(sg2);
            sc = nb > 0.0 ? (ROWS ? 1.0 / nb : (sg > 0.0 ? 1.0 / (nb * sg) : 0.0)) : 0.0;
        }
        jc[tid] = j;
        scl[tid] = sc;
    }
    __syncthreads();
    // loads: 64 x FK elements per operand, 8 per thread (two groups of four)
    float rx[8], rbv[8];
    const bool vec = (g.m % 4) == 0 && (r % 4) == 0;
    auto load = [&](int64_t vc) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + 256 * h;           // 512 groups of four
            // X: rows (vs = 1) -> four consecutive v at one t; columns (es = 1)
            // -> four consecutive t at one v
            int v, t;
            if (ROWS) { v = (e % (FK / 4)) * 4; t = e / (FK / 4); }
            else { t = (e % 16) * 4; v = e / 16; }
            const int64_t gv = vc + v, gt = t0 + t;
            const float* src = X + gv * vs + gt * es;
            const bool full = ROWS ? (gv + 3 < r && gt < L) : (gv < r && gt + 3 < L);
            if (vec && full) {
                const float4 x4 = *reinterpret_cast<const float4*>(src);
                rx[4 * h] = x4.x; rx[4 * h + 1] = x4.y; rx[4 * h + 2] = x4.z; rx[4 * h + 3] = x4.w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t vq = ROWS ? gv + q : gv, tq = ROWS ? gt : gt + q;
                    rx[4 * h + q] = (vq < r && tq < L) ? X[vq * vs + tq * es] : 0.0f;
                }
            }
            // B: column perm(c), four consecutive v
            const int c = e / (FK / 4), vb = (e % (FK / 4)) * 4;
            const int64_t gvb = vc + vb;
            const bool okc = c0 + c < kr;
            const float* bsrc = Bs + (int64_t)jc[c] * r + gvb;
            if (vec && okc && gvb + 3 < r) {
                const float4 b4 = *reinterpret_cast<const float4*>(bsrc);
                rbv[4 * h] = b4.x; rbv[4 * h + 1] = b4.y; rbv[4 * h + 2] = b4.z; rbv[4 * h + 3] = b4.w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) rbv[4 * h + q] = (okc && gvb + q < r) ? bsrc[q] : 0.0f;
            }
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + 256 * h;
            int v, t;
            if (ROWS) { v = (e % (FK / 4)) * 4; t = e / (FK / 4); }
            else { t = (e % 16) * 4; v = e / 16; }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (ROWS) sx[buf][t][v + q] = rx[4 * h + q];
                else sx[buf][t + q][v] = rx[4 * h + q];
            }
            const int c = e / (FK / 4), vb = (e % (FK / 4)) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) sbk[buf][c][vb + q] = rbv[4 * h + q];
        }
    };
    v4f acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = zero4<v4f>();
    load(0);
    int buf = 0;
    for (int64_t vc = 0; vc < r; vc += FK) {
        put(buf);
        __syncthreads();
        if (vc + FK < r) load(vc + FK);
#pragma unroll
        for (int kk = 0; kk < FK; kk += 4) {
            if (ROWS) {
                // D(t, c): output lanes along c
                const float a = sx[buf][16 * wave + lr][kk + lg];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = mfma_f32(a, sbk[buf][16 * c + lr][kk + lg], acc[c]);
            } else {
                // D(c, t): output lanes along t
                const float a = sbk[buf][16 * wave + lr][kk + lg];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = mfma_f32(a, sx[buf][16 * c + lr][kk + lg], acc[c]);
            }
        }
        buf ^= 1;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * wave + mfma_row<float>(lg, v), col = 16 * q + lr;
            if (ROWS) {
                // row = t, col = c: G_pk[p off + c + t kr]
                const int64_t t = t0 + row, c = c0 + col;
                if (t < L && c < kr) out[g.p * off + c + t * kr] = (float)((double)acc[q][v] * scl[col]);
            } else {
                // row = c, col = t: U_pk[m off + t + c m]
                const int64_t c = c0 + row, t = t0 + col;
                if (t < L && c < kr) out[g.m * off + t + c * g.m] = (float)((double)acc[q][v] * scl[row]);
            }
        }
    }
}

template <bool ROWS>
__global__ __launch_bounds__(256) void pc_factor(const float* __restrict__ A, const float* __restrict__ B,
                                                 const double* __restrict__ s2,
                                                 const double* __restrict__ shift, SliceGeom g,
                                                 const int32_t* __restrict__ rho,
                                                 const int64_t* __restrict__ offsets, int64_t capacity,
                                                 const int32_t* __restrict__ perm, int tiles_t,
                                                 float* __restrict__ out) {
    const int64_t s = blockIdx.y, r = g.r;
    factor_tile<ROWS>(A + s * g.m * g.p, B + s * r * r, s2 + s * r, shift[s], g, rho[s], offsets[s],
                      capacity, perm + s * r, (int)(blockIdx.x / tiles_t), (int)(blockIdx.x % tiles_t), out);
}

// batch: task (Gram slice, output tile); wide slices write G_pk, tall U_pk
__global__ __launch_bounds__(256) void pc_factor_batch(const GramSlice* __restrict__ gs,
                                                       const PackSlice* __restrict__ ps,
                                                       const int4* __restrict__ tasks) {
    const int4 t = tasks[blockIdx.x];
    const GramSlice d = gs[t.x];
    const PackSlice q = ps[t.x];
    if (d.g.rows)
        factor_tile<true>(d.A, d.B, d.s2, *d.shift, d.g, *q.rho, *q.off, q.capacity, d.perm, t.y, t.z,
                          static_cast<float*>(q.G_pk));
    else
        factor_tile<false>(d.A, d.B, d.s2, *d.shift, d.g, *q.rho, *q.off, q.capacity, d.perm, t.y, t.z,
                           static_cast<float*>(q.U_pk));
}

// batch: per Gram slice, the descending order of its squared singular
// values (ties by index, the order of pack_sort), its kept singular values
// and short-side factor (as pc_pack_short); a slice whose block would pass
// the capacity is not written and sets the status.
__global__ __launch_bounds__(256) void pc_pack_batch(const GramSlice* __restrict__ gs,
                                                     const PackSlice* __restrict__ ps) {
    __shared__ unsigned long long key[GRAM_MAX_R];
    __shared__ int idx[GRAM_MAX_R];
    const GramSlice d = gs[blockIdx.x];
    const PackSlice q = ps[blockIdx.x];
    const int r = (int)d.g.r;
    int np = 1;
    while (np < r) np <<= 1;
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        if (i < r) {
            double v = d.s2[i];
            if (!(v >= 0.0)) v = 0.0;
            v += 0.0;
            key[i] = ~(unsigned long long)__double_as_longlong(v);   // ascending key = descending value
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
    for (int i = threadIdx.x; i < r; i += blockDim.x) d.perm[i] = idx[i];
    const int64_t kr = *q.rho, off = *q.off;
    if (kr <= 0) return;
    if (off + kr > q.capacity) {
        if (threadIdx.x == 0) atomicExch(q.status, (int32_t)TSVDM_E_CAPACITY);
        return;
    }
    float* S = static_cast<float*>(q.S_pk) + off;
    for (int c = threadIdx.x; c < kr; c += blockDim.x) {
        const double v = d.s2[idx[c]];
        S[c] = (float)sqrt(v > 0.0 ? v : 0.0);
    }
    const double shs = *d.shift;
    for (int64_t c = 0; c < kr; ++c) {
        const int j = idx[c];
        const double sg2 = d.s2[j] > 0.0 ? d.s2[j] : 0.0;
        const double nb = sqrt(sg2 + shs);
        const double scale = nb > 0.0 ? (d.g.rows ? 1.0 : sqrt(sg2)) / nb : 0.0;
        const float* b = d.B + (int64_t)j * r;
        if (d.g.rows) {
            float* u = static_cast<float*>(q.U_pk) + d.g.m * off + c * d.g.m;
            for (int a = threadIdx.x; a < r; a += blockDim.x) u[a] = (float)((double)b[a] * scale);
        } else {
            float* gr = static_cast<float*>(q.G_pk) + d.g.p * off + c;
            for (int t = threadIdx.x; t < r; t += blockDim.x) gr[t * kr] = (float)((double)b[t] * scale);
        }
    }
}


// The in-LDS Jacobi keeps r x (r + 1) floats of dynamic LDS; each size
// class is allowed the most its largest r needs, once per process.
constexpr int LDS_CLASSES = 4;
constexpr int LDS_RMAX[LDS_CLASSES] = {32, 64, 96, 128};
static_assert(GRAM_LDS_MAX_R <= LDS_RMAX[LDS_CLASSES - 1], "in-LDS limit beyond the largest class");
static_assert(GRAM_LDS_CLASSES == LDS_CLASSES, "class count differs from the header");
// the Cholesky's static LDS panel is sized by its class's largest r
constexpr int CHOL_RMAX[GRAM_CHOL_CLASSES] = {128, 256, 512, 1024};
static_assert(CHOL_RMAX[GRAM_CHOL_CLASSES - 1] == GRAM_MAX_R, "largest Cholesky class differs from the limit");

template <int RMAX>
hipError_t allow_lds() {
    const int bytes = RMAX * (RMAX + 1) * (int)sizeof(float);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&pc_jacobi_lds<RMAX>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&pc_jacobi_lds_batch<RMAX>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

std::mutex g_lds_mu;
bool g_lds_ready = false;

template <int RMAX>
int launch_lds_bucket(float* B, int64_t r, int64_t n, double tol, int max_sweeps, const double* shift,
                      double* s2, int32_t* flag, hipStream_t st) {
    const size_t bytes = (size_t)r * (size_t)(r + 1) * sizeof(float);
    pc_jacobi_lds<RMAX><<<(unsigned)n, 256, bytes, st>>>(B, r, tol, max_sweeps, shift, s2, flag);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int launch_jacobi_lds(float* B, int64_t r, int64_t n, double tol, int max_sweeps, const double* shift,
                      double* s2, int32_t* flag, hipStream_t st) {
    const int rc = gram_lds_prepare();
    if (rc) return rc;
    if (r <= 32) return launch_lds_bucket<32>(B, r, n, tol, max_sweeps, shift, s2, flag, st);
    if (r <= 64) return launch_lds_bucket<64>(B, r, n, tol, max_sweeps, shift, s2, flag, st);
    if (r <= 96) return launch_lds_bucket<96>(B, r, n, tol, max_sweeps, shift, s2, flag, st);
    return launch_lds_bucket<128>(B, r, n, tol, max_sweeps, shift, s2, flag, st);
}

}  // namespace

int gram_lds_prepare() {
    std::lock_guard<std::mutex> lk(g_lds_mu);
    if (g_lds_ready) return TSVDM_OK;
    TSVDM_HIP_CHECK(allow_lds<32>());
    TSVDM_HIP_CHECK(allow_lds<64>());
    TSVDM_HIP_CHECK(allow_lds<96>());
    TSVDM_HIP_CHECK(allow_lds<128>());
    g_lds_ready = true;
    return TSVDM_OK;
}

int gram_lds_class(int64_t r) {
    for (int c = 0; c < LDS_CLASSES; ++c)
        if (r <= LDS_RMAX[c]) return c;
    return -1;
}

int gram_chol_class(int64_t r) {
    for (int c = 0; c < GRAM_CHOL_CLASSES; ++c)
        if (r <= CHOL_RMAX[c]) return c;
    return -1;
}

double gram_tol(int64_t r) { return jacobi_default_opts(r, r, TSVDM_F32).tol; }

int run_gram_prep_batch(const GramSlice* gs, int64_t ngram, const int2* gram_tasks, int64_t ntasks,
                        const int* lists, const int64_t* class_off, const int64_t* class_cnt,
                        hipStream_t st) {
    TSVDM_REQUIRE(ntasks < ((int64_t)1 << 31) && ngram < ((int64_t)1 << 31), TSVDM_E_SHAPE,
                  "too many Gram slices for one launch");
    if (ngram == 0) return TSVDM_OK;
    pc_gram_batch<<<(unsigned)ntasks, 256, 0, st>>>(gs, gram_tasks);
    TSVDM_LAUNCH_CHECK();
    for (int c = 0; c < GRAM_CHOL_CLASSES; ++c) {
        if (!class_cnt[c]) continue;
        const int* list = lists + class_off[c];
        const unsigned cnt = (unsigned)class_cnt[c];
        switch (CHOL_RMAX[c]) {
            case 128: pc_chol_batch<128, 256><<<cnt, 256, 0, st>>>(gs, list); break;
            case 256: pc_chol_batch<256, 256><<<cnt, 256, 0, st>>>(gs, list); break;
            case 512:
                if (chol_wide(512, cnt)) pc_chol_batch<512, 1024><<<cnt, 1024, 0, st>>>(gs, list);
                else pc_chol_batch<512, 256><<<cnt, 256, 0, st>>>(gs, list);
                break;
            default:
                if (chol_wide(1024, cnt)) pc_chol_batch<1024, 1024><<<cnt, 1024, 0, st>>>(gs, list);
                else pc_chol_batch<1024, 256><<<cnt, 256, 0, st>>>(gs, list);
                break;
        }
        TSVDM_LAUNCH_CHECK();
    }
    return TSVDM_OK;
}

int run_gram_unshift_batch(const GramSlice* gs, int64_t n, hipStream_t st) {
    TSVDM_REQUIRE(n < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many Gram slices for one launch");
    if (n == 0) return TSVDM_OK;
    pc_unshift_batch<<<(unsigned)n, 256, 0, st>>>(gs);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_gram_lds_batch(const GramSlice* gs, const int* lists, const int64_t* class_off,
                       const int64_t* class_cnt, const int* class_maxr, int max_sweeps,
                       const GramSlice* gs_lds, int64_t n_lds, int32_t* status, hipStream_t st) {
    TSVDM_REQUIRE(n_lds < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many Gram slices for one launch");
    if (n_lds == 0) return TSVDM_OK;
    for (int c = 0; c < LDS_CLASSES; ++c) {
        if (!class_cnt[c]) continue;
        const size_t bytes = (size_t)class_maxr[c] * (size_t)(class_maxr[c] + 1) * sizeof(float);
        const int* list = lists + class_off[c];
        const unsigned cnt = (unsigned)class_cnt[c];
        switch (LDS_RMAX[c]) {
            case 32: pc_jacobi_lds_batch<32><<<cnt, 256, bytes, st>>>(gs, list, max_sweeps); break;
            case 64: pc_jacobi_lds_batch<64><<<cnt, 256, bytes, st>>>(gs, list, max_sweeps); break;
            case 96: pc_jacobi_lds_batch<96><<<cnt, 256, bytes, st>>>(gs, list, max_sweeps); break;
            default: pc_jacobi_lds_batch<128><<<cnt, 256, bytes, st>>>(gs, list, max_sweeps); break;
        }
        TSVDM_LAUNCH_CHECK();
    }
    pc_gram_status<<<1, 256, 0, st>>>(gs_lds, n_lds, status);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_gram_pack_batch(const GramSlice* gs, const PackSlice* ps, int64_t ngram, const int4* ftasks,
                        int64_t nft, hipStream_t st) {
    TSVDM_REQUIRE(nft < ((int64_t)1 << 31) && ngram < ((int64_t)1 << 31), TSVDM_E_SHAPE,
                  "too many Gram slices for one launch");
    if (ngram == 0) return TSVDM_OK;
    pc_pack_batch<<<(unsigned)ngram, 256, 0, st>>>(gs, ps);
    TSVDM_LAUNCH_CHECK();
    if (nft > 0) {
        pc_factor_batch<<<(unsigned)nft, 256, 0, st>>>(gs, ps, ftasks);
        TSVDM_LAUNCH_CHECK();
    }
    return TSVDM_OK;
}


size_t gram_svd_workspace_bytes(int64_t m, int64_t p, int64_t n) {
    const SliceGeom g = slice_geom(m, p);
    Carver cv(nullptr);
    cv.carve<double>((size_t)(g.r * g.r * n));   // G
    cv.carve<double>((size_t)(g.r * g.r * n));   // second trailing-matrix buffer of the Cholesky
    return cv.total() + jacobi_workspace_bytes(g.r, n);
}


// G = X X^T (FP64) and the pivoted, shifted Cholesky factor of every slice,
// P (G + s I) P^T = L L^T: B = P^T L in OT (B B^T = G + s I), s per slice.
// G and Lw are the factorisation's workspace (G is overwritten).
template <class T, class OT>
int gram_factor(const T* A_hat, const SliceGeom& g, int64_t n, double* G, double* Lw, OT* B,
                double* shift, hipStream_t st) {
    const int64_t r = g.r;
    const int nt = (int)((r + 63) / 64);
    const int ntri = nt * (nt + 1) / 2;
    TSVDM_REQUIRE((int64_t)ntri * n < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many Gram tiles");
    pc_gram<T><<<(unsigned)(ntri * n), 256, 0, st>>>(A_hat, g, ntri, G);
    TSVDM_LAUNCH_CHECK();
    const double cshift = (double)(g.L + r) * 1.1102230246251565e-16;
    const bool wide = chol_wide(r, n);
    if (r <= 128) pc_chol<128, OT, 256><<<(unsigned)n, 256, 0, st>>>(G, r, cshift, Lw, B, shift);
    else if (r <= 256) pc_chol<256, OT, 256><<<(unsigned)n, 256, 0, st>>>(G, r, cshift, Lw, B, shift);
    else if (r <= 512 && wide) pc_chol<512, OT, 1024><<<(unsigned)n, 1024, 0, st>>>(G, r, cshift, Lw, B, shift);
    else if (r <= 512) pc_chol<512, OT, 256><<<(unsigned)n, 256, 0, st>>>(G, r, cshift, Lw, B, shift);
    else if (wide) pc_chol<1024, OT, 1024><<<(unsigned)n, 1024, 0, st>>>(G, r, cshift, Lw, B, shift);
    else pc_chol<1024, OT, 256><<<(unsigned)n, 256, 0, st>>>(G, r, cshift, Lw, B, shift);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_gram_svd(const float* A_hat, int64_t m, int64_t p, int64_t n, float* B, double* s2,
                 double* shift, int32_t* status, const JacobiOpts& o, int jacobi, void* ws,
                 hipStream_t st) {
    const SliceGeom g = slice_geom(m, p);
    const int64_t r = g.r;
    TSVDM_REQUIRE(r <= GRAM_MAX_R, TSVDM_E_SHAPE, "min(m, p) must be <= 1024 for the Gram form");
    Carver cv(ws);
    double* G = cv.carve<double>((size_t)(r * r * n));
    double* Lw = cv.carve<double>((size_t)(r * r * n));
    void* jws = static_cast<char*>(ws) + cv.total();
    const int rc0 = gram_factor<float, float>(A_hat, g, n, G, Lw, B, shift, st);
    if (rc0) return rc0;
    // one-sided Jacobi on the columns of L (r x r), no accumulated rotations:
    // held in LDS, or the block rounds streaming through HBM
    const bool lds = jacobi == TSVDM_GRAM_LDS || (jacobi == TSVDM_GRAM_AUTO && r <= GRAM_LDS_MAX_R);
    TSVDM_REQUIRE(!lds || r <= GRAM_LDS_MAX_R, TSVDM_E_SHAPE, "the in-LDS Jacobi needs min(m, p) <= 128");
    TSVDM_REQUIRE(!lds || n < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many slices for one launch");
    if (lds) {
        int32_t* flag = static_cast<int32_t*>(jws);
        const bool stats = stats_enabled();
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (stats) {
            TSVDM_HIP_CHECK(hipEventCreate(&e0));
            TSVDM_HIP_CHECK(hipEventCreate(&e1));
            TSVDM_HIP_CHECK(hipEventRecord(e0, st));
        }
        int rc2 = launch_jacobi_lds(B, r, n, o.tol, o.max_sweeps, shift, s2, flag, st);
        if (rc2) return rc2;
        if (stats) {
            TSVDM_HIP_CHECK(hipEventRecord(e1, st));
            TSVDM_HIP_CHECK(hipEventSynchronize(e1));
            float t = 0.f;
            TSVDM_HIP_CHECK(hipEventElapsedTime(&t, e0, e1));
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            stats_add_launch(1, t);
        }
        pc_flags_status<<<1, 256, 0, st>>>(flag, n, status);
        TSVDM_LAUNCH_CHECK();
        return TSVDM_OK;
    }
    int rc = run_jacobi(B, TSVDM_F32, r, r, n, nullptr, s2, status, o, jws, st);
    if (rc) return rc;
    pc_unshift<<<(unsigned)((r * n + 255) / 256), 256, 0, st>>>(s2, shift, r, n);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_gram_pack(const float* A_hat, const float* B, const double* s2, const double* shift,
                  int64_t m, int64_t p, int64_t n, const int32_t* rho, const int64_t* offsets,
                  int64_t capacity, float* U_pk, float* G_pk, float* S_pk, int32_t* status,
                  void* ws, hipStream_t st) {
    const SliceGeom g = slice_geom(m, p);
    const int64_t r = g.r;
    int32_t* perm = static_cast<int32_t*>(ws);
    int rc = run_pack_sort_f32(s2, r, n, rho, offsets, capacity, perm, S_pk, status, st);
    if (rc) return rc;
    TSVDM_REQUIRE(n < 65536, TSVDM_E_SHAPE, "n must be below 65536");
    dim3 gs((unsigned)(r < 256 ? r : 256), (unsigned)n);
    pc_pack_short<<<gs, 256, 0, st>>>(B, s2, shift, g, rho, offsets, capacity, perm, U_pk, G_pk);
    TSVDM_LAUNCH_CHECK();
    const int tiles_c = (int)((r + 63) / 64), tiles_t = (int)((g.L + 63) / 64);
    TSVDM_REQUIRE((int64_t)tiles_c * tiles_t < ((int64_t)1 << 31), TSVDM_E_SHAPE, "factor grid too large");
    dim3 gf((unsigned)(tiles_c * tiles_t), (unsigned)n);
    if (g.rows)
        pc_factor<true><<<gf, 256, 0, st>>>(A_hat, B, s2, shift, g, rho, offsets, capacity, perm, tiles_t, G_pk);
    else
        pc_factor<false><<<gf, 256, 0, st>>>(A_hat, B, s2, shift, g, rho, offsets, capacity, perm, tiles_t, U_pk);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

size_t precond_svd_workspace_bytes(int64_t m, int64_t p, int64_t n, int dt) {
    const SliceGeom g = slice_geom(m, p);
    const size_t e = dt == TSVDM_F64 ? 8 : 4;
    const size_t rr = (size_t)(g.r * g.r * n);
    Carver cv(nullptr);
    cv.carve<double>(rr);                  // G, then W^T W and S
    cv.carve<double>(rr);                  // second Cholesky buffer, then the Newton-Schulz iterate
    cv.carve<float>(rr);                   // B (FP32 factor)
    cv.carve<char>(g.rows ? rr * e : 1);   // W^T (wide slices)
    cv.carve<double>((size_t)n);           // shifts
    cv.carve<int32_t>((size_t)n);          // full ranks
    cv.carve<int64_t>((size_t)n + 1);      // their offsets
    cv.carve<int32_t>(1);                  // first-stage status
    return cv.total() + jacobi_workspace_bytes(g.r, n);
}

namespace {

// FP64 slices (T = double)
template <class T>
int precond_impl(const T* A_hat, int dt, int64_t m, int64_t p, int64_t n, T* X, T* W, double* s2,
                 int32_t* status, const JacobiOpts& o, void* ws, hipStream_t st) {
    static_assert(sizeof(T) == 8, "the preconditioned form runs FP64 slices");
    const SliceGeom g = slice_geom(m, p);
    const int64_t r = g.r;
    TSVDM_REQUIRE(r <= GRAM_MAX_R, TSVDM_E_SHAPE, "min(m, p) must be <= 1024 for the preconditioned form");
    TSVDM_REQUIRE(n < 65536, TSVDM_E_SHAPE, "n must be below 65536");
    const size_t rr = (size_t)(r * r * n);
    Carver cv(ws);
    double* G = cv.carve<double>(rr);
    double* Lw = cv.carve<double>(rr);
    float* B = cv.carve<float>(rr);
    T* Ut = cv.carve<T>(g.rows ? rr : 1);
    double* shift = cv.carve<double>((size_t)n);
    int32_t* rho = cv.carve<int32_t>((size_t)n);
    int64_t* off = cv.carve<int64_t>((size_t)n + 1);
    int32_t* s1 = cv.carve<int32_t>(1);
    void* jws = static_cast<char*>(ws) + cv.total();
    // 1. the FP32 Gram form's factor and its Jacobi (no accumulator): B's
    //    unit columns are the short-side singular vectors to the FP32
    //    Jacobi's tolerance (and the FP64 Gram's rounding)
    int rc = gram_factor<T, float>(A_hat, g, n, G, Lw, B, shift, st);
    if (rc) return rc;
    JacobiOpts o1 = jacobi_default_opts(r, r, TSVDM_F32);
    o1.block = o.block;
    o1.max_sweeps = o.max_sweeps;
    o1.host_poll = o.host_poll;
    rc = run_jacobi(B, TSVDM_F32, r, r, n, nullptr, s2, s1, o1, jws, st);
    if (rc) return rc;
    // (into Lw, so that the third Newton-Schulz step below ends in W)
    pc_normalize<float, double><<<dim3((unsigned)r, (unsigned)n), 256, 0, st>>>(B, r, Lw, s1);
    TSVDM_LAUNCH_CHECK();
    // 2. W orthonormal to the working precision: its cosines are <= the
    //    FP32 tol (~1e-5), so ||W^T W - I|| <= r tol < 0.02 and three
    //    Newton-Schulz steps take it below 1e-18 (0.02 -> 3e-4 -> 7e-8 ->
    //    4e-15 at worst, then rounding); the rotation form in step 4 then
    //    applies an orthogonal W, so its result keeps its own accuracy.
    //    W^T W by the Gram kernel (the columns of W as vectors), W S by the
    //    factor product with every slice at full rank.  The third step runs
    //    only on the slices whose max |W^T W - I| still exceeds 32 sqrt(r)
    //    u64, the size of the FP64 rounding of W^T W itself (a step cannot
    //    go below it); the usual FP32 tolerances leave every slice there
    //    after two.
    pc_rank_full<<<(unsigned)((n + 256) / 256), 256, 0, st>>>(rho, off, r, n);
    TSVDM_LAUNCH_CHECK();
    {
        const SliceGeom gw = slice_geom(r, r);
        const int nt = (int)((r + 63) / 64);
        const int ntri = nt * (nt + 1) / 2;
        TSVDM_REQUIRE((int64_t)ntri * n < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many Gram tiles");
        const unsigned eb = (unsigned)((r * r * n + 255) / 256);
        double* cur = Lw;
        double* nxt = W;
        const double thr = 32.0 * sqrt((double)r) * 1.1102230246251565e-16;
        for (int it = 0; it < 3; ++it) {   // Lw -> W -> Lw -> W
            pc_gram<double><<<(unsigned)(ntri * n), 256, 0, st>>>(cur, gw, ntri, G);
            TSVDM_LAUNCH_CHECK();
            if (it == 2) {
                pc_ns_check<<<(unsigned)n, 256, 0, st>>>(G, r, thr, rho);
                TSVDM_LAUNCH_CHECK();
            }
            pc_ns_coef<<<eb, 256, 0, st>>>(G, r, n);
            TSVDM_LAUNCH_CHECK();
            rc = run_lowrank_gemm(cur, G, TSVDM_F64, r, r, n, rho, off, r * n, nxt, st);
            if (rc) return rc;
            if (it == 2) {
                pc_ns_keep<<<eb, 256, 0, st>>>(cur, nxt, rho, r, n);
                TSVDM_LAUNCH_CHECK();
            }
            double* const t = cur;
            cur = nxt;
            nxt = t;
        }
        // every slice at full rank again for the product with the slice
        pc_rank_full<<<(unsigned)((n + 256) / 256), 256, 0, st>>>(rho, off, r, n);
        TSVDM_LAUNCH_CHECK();
        if (g.rows) {
            pc_transpose<double><<<eb, 256, 0, st>>>(W, r, n, Ut);
            TSVDM_LAUNCH_CHECK();
        }
    }
    // 3. the slice rotated by W: X = W^T A (wide) or A W (tall)
    if (g.rows) rc = run_lowrank_gemm(Ut, A_hat, dt, m, p, n, rho, off, r * n, X, st);
    else rc = run_lowrank_gemm(A_hat, W, dt, m, p, n, rho, off, r * n, X, st);
    if (rc) return rc;
    // 4. the rotation form on X, accumulating into W: its first sweeps find
    //    the vectors nearly orthogonal already
    JacobiOpts o2 = o;
    o2.w_given = 1;
    rc = run_jacobi(X, dt, m, p, n, W, s2, status, o2, jws, st);
    if (rc) return rc;
    pc_merge_status<<<1, 64, 0, st>>>(status, s1);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

}  // namespace

int run_precond_svd(const void* A_hat, int dt, int64_t m, int64_t p, int64_t n, void* X, void* W,
                    double* s2, int32_t* status, const JacobiOpts& o, void* ws, hipStream_t st) {
    TSVDM_REQUIRE(dt == TSVDM_F64, TSVDM_E_UNSUPPORTED, "the preconditioned form runs FP64 slices");
    return precond_impl<double>(static_cast<const double*>(A_hat), dt, m, p, n, static_cast<double*>(X),
                                static_cast<double*>(W), s2, status, o, ws, st);
}

}  // namespace tsvdm

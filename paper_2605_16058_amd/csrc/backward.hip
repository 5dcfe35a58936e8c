// Adjoint of the truncation loss L(A, M) = sum_i sum_{j>k} sigma_ij^2 of the
// slices of A x_3 M (for orthogonal M, L = ||A - A_k||_F^2, Section 2.3).
// Not in the paper; derived: with R-hat_i the rank-k tail of slice i,
//   dL/dA = 2 R-hat x_3 M^T,   dL/dM = 2 R-hat_(3) A_(3)^T.
// The slice factors are recomputed (transform + Jacobi), never stored by
// the forward call.
#include "common.h"
#include "kernels.h"

namespace tsvdm {

namespace {

// part[split][i + l*n] = sum over the split's rows of P[row, i] * Q[row, l]
template <class T>
__global__ __launch_bounds__(256) void tsmm_partial(const T* __restrict__ P, const void* __restrict__ Q,
                                                    int qdt, int64_t R, int n, int64_t rps,
                                                    int tiles, double* __restrict__ part) {
    typedef typename Acc<T>::type AccT;
    constexpr int KC = 16;
    __shared__ T Ps[KC][64 + 1];
    __shared__ T Qs[KC][64 + 1];
    const int ti = blockIdx.x % tiles, tl = blockIdx.x / tiles;
    const int64_t split = blockIdx.y;
    const int i0 = ti * 64, l0 = tl * 64;
    const int64_t r0 = split * rps;
    const int64_t r1 = (r0 + rps < R) ? r0 + rps : R;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    AccT acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = zero4<AccT>();
    for (int64_t c0 = r0; c0 < r1; c0 += KC) {
        for (int e = tid; e < KC * 64; e += 256) {
            const int k = e % KC, i = e / KC;
            const int64_t row = c0 + k;
            T pv = 0, qv = 0;
            if (row < r1 && i0 + i < n) pv = P[row + (int64_t)(i0 + i) * R];
            if (row < r1 && l0 + i < n) qv = ldg_as<T>(Q, row + (int64_t)(l0 + i) * R, qdt);
            Ps[k][i] = pv;
            Qs[k][i] = qv;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            T a = Ps[kk + lg][wave * 16 + lr];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                T b = Qs[kk + lg][t * 16 + lr];
                acc[t] = mfma(a, b, acc[t]);
            }
        }
        __syncthreads();
    }
    double* out = part + split * (int64_t)n * n;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int l = l0 + t * 16 + lr;
        if (l >= n) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + wave * 16 + mfma_row<T>(lg, v);
            if (i < n) out[i + (int64_t)l * n] = (double)acc[t][v];
        }
    }
}

__global__ void tsmm_final(const double* __restrict__ part, int64_t splits, int n, double scale,
                           double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nn = (int64_t)n * n;
    if (e >= nn) return;
    double s = 0.0;
    for (int64_t k = 0; k < splits; ++k) s += part[k * nn + e];
    out[e] = scale * s;
}

// loss = sum over slices of the squared singular values at sorted positions
// first .. r-1 (the tail), combined in a fixed order.
__global__ __launch_bounds__(256) void tail_loss(const double* __restrict__ s2,
                                                 const int32_t* __restrict__ perm, int64_t r,
                                                 int64_t n, int64_t first,
                                                 double* __restrict__ loss) {
    __shared__ double part[256];
    double acc = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += 256) {
        double t = 0.0;
        for (int64_t c = first; c < r; ++c) t += s2[s * r + perm[s * r + c]];
        acc += t;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0;
        for (int i = 0; i < 256; ++i) x += part[i];
        *loss = x;
    }
}

struct BwdLayout {
    void* Ahat; void* W; double* s2; void* jws; int32_t* rho; int64_t* offsets;
    void* Upk; void* Gpk; void* Spk; int32_t* perm; void* Rhat; double* Mt; double* part;
    int64_t splits, rps;
    size_t total;
};

BwdLayout bwd_layout(void* ws, int64_t m, int64_t p, int64_t n, int dt) {
    const SliceGeom g = slice_geom(m, p);
    const size_t es = dt == TSVDM_F64 ? 8 : 4;
    const int64_t R = m * p;
    BwdLayout L;
    int64_t rps = (R + 1023) / 1024;
    if (rps < 1024) rps = 1024;
    rps = (rps + 15) / 16 * 16;
    L.rps = rps;
    L.splits = (R + rps - 1) / rps;
    Carver cv(ws);
    L.Ahat = cv.carve<char>((size_t)(R * n) * es);
    L.W = cv.carve<char>((size_t)(g.r * g.r * n) * es);
    L.s2 = cv.carve<double>((size_t)(g.r * n));
    L.jws = cv.carve<char>(jacobi_workspace_bytes(g.r, n));
    L.rho = cv.carve<int32_t>((size_t)n);
    L.offsets = cv.carve<int64_t>((size_t)n + 1);
    L.Upk = cv.carve<char>((size_t)(m * g.r * n) * es);
    L.Gpk = cv.carve<char>((size_t)(p * g.r * n) * es);
    L.Spk = cv.carve<char>((size_t)(g.r * n) * es);
    L.perm = cv.carve<int32_t>((size_t)(g.r * n));
    L.Rhat = cv.carve<char>((size_t)(R * n) * es);
    L.Mt = cv.carve<double>((size_t)(n * n));
    L.part = cv.carve<double>((size_t)(L.splits * n * n));
    L.total = cv.total();
    return L;
}

}  // namespace

size_t backward_workspace_bytes(int64_t m, int64_t p, int64_t n, int dt) {
    return bwd_layout(nullptr, m, p, n, dt).total;
}

int run_backward(const void* A, int dt, int64_t m, int64_t p, int64_t n, const double* M,
                 int64_t k, double g, void* dA, double* dM, double* loss, int32_t* status,
                 void* ws, hipStream_t st) {
    const SliceGeom geo = slice_geom(m, p);
    BwdLayout L = bwd_layout(ws, m, p, n, dt);
    const int64_t kk = k < geo.r ? k : geo.r;
    const int64_t tail = geo.r - kk;
    int rc;
    rc = run_ttm(A, dt, L.Ahat, dt, m, p, n, M, 0, 1.0, dt, 0, L.Mt, st);
    if (rc) return rc;
    JacobiOpts o = jacobi_default_opts(m, p, dt);
    rc = run_jacobi(L.Ahat, dt, m, p, n, L.W, L.s2, status, o, L.jws, st);
    if (rc) return rc;
    rc = run_truncate_rank(tail, geo.r, n, L.rho, L.offsets, st);
    if (rc) return rc;
    // pack the tail (positions kk .. r-1 of the descending order); the pack
    // workspace is the perm array
    rc = run_pack_from(L.Ahat, L.W, L.s2, dt, m, p, n, L.rho, L.offsets, tail * n, (int)kk,
                       L.Upk, L.Gpk, L.Spk, status, L.perm, st);
    if (rc) return rc;
    if (loss) {
        tail_loss<<<1, 256, 0, st>>>(L.s2, L.perm, geo.r, n, kk, loss);
        TSVDM_LAUNCH_CHECK();
    }
    if (!dA && !dM) return TSVDM_OK;
    rc = run_lowrank_gemm(L.Upk, L.Gpk, dt, m, p, n, L.rho, L.offsets, tail * n, L.Rhat, st);
    if (rc) return rc;
    if (dA) {
        rc = run_ttm(L.Rhat, dt, dA, dt, m, p, n, M, 1, 2.0 * g, dt, 0, L.Mt, st);
        if (rc) return rc;
    }
    if (dM) {
        const int tiles = (int)((n + 63) / 64);
        dim3 grid((unsigned)(tiles * tiles), (unsigned)L.splits);
        const int64_t R = m * p;
        if (dt == TSVDM_F64)
            tsmm_partial<double><<<grid, 256, 0, st>>>(static_cast<const double*>(L.Rhat), A, dt, R,
                                                       (int)n, L.rps, tiles, L.part);
        else
            tsmm_partial<float><<<grid, 256, 0, st>>>(static_cast<const float*>(L.Rhat), A, dt, R,
                                                      (int)n, L.rps, tiles, L.part);
        TSVDM_LAUNCH_CHECK();
        tsmm_final<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(L.part, L.splits, (int)n,
                                                                    2.0 * g, dM);
        TSVDM_LAUNCH_CHECK();
    }
    return TSVDM_OK;
}

}  // namespace tsvdm

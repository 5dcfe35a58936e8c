// extern "C" entry points of libtsvdm: argument validation (before any
// launch), workspace sizing and dispatch to the kernels.
#include <cmath>
#include <string>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace tsvdm {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

namespace {

constexpr int64_t kMaxDim = (int64_t)1 << 31;

int check_shape(int64_t m, int64_t p, int64_t n) {
    TSVDM_REQUIRE(m > 0 && p > 0 && n > 0, TSVDM_E_SHAPE, "m, p and n must be positive");
    TSVDM_REQUIRE(m < kMaxDim && p < kMaxDim && n < 65536, TSVDM_E_SHAPE,
                  "m, p must be < 2^31 and n < 65536");
    TSVDM_REQUIRE(m * p <= ((int64_t)1 << 40) / n, TSVDM_E_SHAPE, "tensor too large");
    return TSVDM_OK;
}

bool io_dtype(int dt) { return dt == TSVDM_F64 || dt == TSVDM_F32; }

int check_ws(void* ws, size_t have, size_t need) {
    if (need == 0) return TSVDM_OK;
    TSVDM_REQUIRE(ws != nullptr, TSVDM_E_ARG, "workspace pointer is NULL");
    if (have < need) {
        set_error("workspace too small: " + std::to_string(have) + " < " + std::to_string(need) +
                  " bytes");
        return TSVDM_E_WORKSPACE;
    }
    return TSVDM_OK;
}

#define TSVDM_TRY(expr)              \
    do {                             \
        int rc_ = (expr);            \
        if (rc_ != TSVDM_OK) return rc_; \
    } while (0)

size_t esize(int dt) { return dt == TSVDM_F64 ? 8 : 4; }

size_t reconstruct_bytes(int64_t m, int64_t p, int64_t n, int dt) {
    Carver cv(nullptr);
    cv.carve<char>((size_t)(m * p * n) * esize(dt));
    cv.carve<char>(ttm_workspace_bytes(n));
    return cv.total();
}

}  // namespace
}  // namespace tsvdm

using namespace tsvdm;

extern "C" {

int tsvdm_version(void) { return 10000; }

const char* tsvdm_last_error(void) { return g_last_error.c_str(); }

int tsvdm_check_transform(const double* M, int64_t n, double tol, double* scale_sq) {
    clear_error();
    TSVDM_REQUIRE(M != nullptr, TSVDM_E_ARG, "M is NULL");
    TSVDM_REQUIRE(n > 0 && n < 65536, TSVDM_E_SHAPE, "n must be in [1, 65535]");
    TSVDM_REQUIRE(tol >= 0.0, TSVDM_E_ARG, "tol must be >= 0");
    // G = M^T M, column-major M
    std::vector<double> G((size_t)(n * n));
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = 0; b <= a; ++b) {
            double s = 0.0;
            for (int64_t i = 0; i < n; ++i) s += M[i + a * n] * M[i + b * n];
            G[a + b * n] = s;
            G[b + a * n] = s;
        }
    double c2 = 0.0;
    for (int64_t a = 0; a < n; ++a) c2 += G[a + a * n];
    c2 /= (double)n;
    if (!std::isfinite(c2) || c2 <= 0.0) {
        set_error("M must be a nonzero multiple of an orthogonal matrix");
        return TSVDM_E_NOT_ORTHO;
    }
    double dev = 0.0;
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = 0; b < n; ++b) {
            const double d = std::fabs(G[a + b * n] / c2 - (a == b ? 1.0 : 0.0));
            if (!(d <= dev)) dev = d;  // NaN propagates
        }
    if (!(dev <= tol)) {
        set_error("M is not a multiple of an orthogonal matrix (max |M^T M / c^2 - I| = " +
                  std::to_string(dev) + ")");
        return TSVDM_E_NOT_ORTHO;
    }
    if (scale_sq) *scale_sq = c2;
    return TSVDM_OK;
}

// ------------------------------------------------------------- transform

int tsvdm_transform_workspace_size(int64_t n, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_REQUIRE(n > 0 && n < 65536, TSVDM_E_SHAPE, "n must be in [1, 65535]");
    *bytes = ttm_workspace_bytes(n);
    return TSVDM_OK;
}

int tsvdm_transform(const void* X, int x_dtype, void* Y, int y_dtype, int64_t m, int64_t p,
                    int64_t n, const double* M, int transpose, double scale, int compute,
                    int tile, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(X && Y && M, TSVDM_E_ARG, "X, Y and M must be non-NULL");
    TSVDM_REQUIRE(X != Y, TSVDM_E_ARG, "Y must not alias X");
    TSVDM_REQUIRE(io_dtype(x_dtype) && io_dtype(y_dtype), TSVDM_E_UNSUPPORTED,
                  "x_dtype and y_dtype must be F64 or F32");
    TSVDM_REQUIRE(compute >= TSVDM_F64 && compute <= TSVDM_BF16X3, TSVDM_E_UNSUPPORTED,
                  "unknown compute dtype");
    TSVDM_REQUIRE(!(compute >= TSVDM_BF16 && y_dtype != TSVDM_F32), TSVDM_E_UNSUPPORTED,
                  "BF16 compute writes F32 output only");
    TSVDM_REQUIRE(transpose == 0 || transpose == 1, TSVDM_E_ARG, "transpose must be 0 or 1");
    TSVDM_REQUIRE(std::isfinite(scale), TSVDM_E_ARG, "scale must be finite");
    TSVDM_REQUIRE(tile >= 0 && tile <= TTM_SHAPES, TSVDM_E_ARG, "tile must be in [0, 8]");
    TSVDM_TRY(check_ws(ws, ws_bytes, ttm_workspace_bytes(n)));
    return run_ttm(X, x_dtype, Y, y_dtype, m, p, n, M, transpose, scale, compute, tile, ws,
                   as_stream(stream));
}

int tsvdm_transform_mode(const void* X, int x_dtype, void* Y, int y_dtype, int32_t d,
                         const int64_t* dims, int32_t k, const double* M, int transpose,
                         double scale, int compute, int tile, void* ws, size_t ws_bytes,
                         void* stream) {
    clear_error();
    TSVDM_REQUIRE(dims != nullptr, TSVDM_E_ARG, "dims is NULL");
    TSVDM_REQUIRE(d >= 3 && d <= 32, TSVDM_E_SHAPE, "d must be in [3, 32]");
    TSVDM_REQUIRE(k >= 3 && k <= d, TSVDM_E_ARG, "k must be in [3, d]");
    int64_t R = 1, P = 1;
    for (int i = 0; i < d; ++i) {
        TSVDM_REQUIRE(dims[i] >= 1 && dims[i] < ((int64_t)1 << 31), TSVDM_E_SHAPE,
                      "every dimension must be in [1, 2^31)");
        int64_t& acc = (i + 1 < k) ? R : P;
        if (i + 1 == k) continue;
        TSVDM_REQUIRE(acc <= (((int64_t)1 << 46) / dims[i]), TSVDM_E_SHAPE, "tensor too large");
        acc *= dims[i];
    }
    const int64_t n = dims[k - 1];
    TSVDM_REQUIRE(n < 65536, TSVDM_E_SHAPE, "n_k must be below 65536");
    TSVDM_REQUIRE(R <= (((int64_t)1 << 46) / n) / P, TSVDM_E_SHAPE, "tensor too large");
    TSVDM_REQUIRE(X && Y && M, TSVDM_E_ARG, "X, Y and M must be non-NULL");
    TSVDM_REQUIRE(X != Y, TSVDM_E_ARG, "Y must not alias X");
    TSVDM_REQUIRE(io_dtype(x_dtype) && io_dtype(y_dtype), TSVDM_E_UNSUPPORTED,
                  "x_dtype and y_dtype must be F64 or F32");
    TSVDM_REQUIRE(compute >= TSVDM_F64 && compute <= TSVDM_BF16X3, TSVDM_E_UNSUPPORTED,
                  "unknown compute dtype");
    TSVDM_REQUIRE(!(compute >= TSVDM_BF16 && y_dtype != TSVDM_F32), TSVDM_E_UNSUPPORTED,
                  "BF16 compute writes F32 output only");
    TSVDM_REQUIRE(transpose == 0 || transpose == 1, TSVDM_E_ARG, "transpose must be 0 or 1");
    TSVDM_REQUIRE(std::isfinite(scale), TSVDM_E_ARG, "scale must be finite");
    TSVDM_REQUIRE(tile >= 0 && tile <= TTM_SHAPES, TSVDM_E_ARG, "tile must be in [0, 8]");
    TSVDM_TRY(check_ws(ws, ws_bytes, ttm_workspace_bytes(n)));
    return run_ttm_mode(X, x_dtype, Y, y_dtype, R, n, P, M, transpose, scale, compute, tile, ws,
                        as_stream(stream));
}

int tsvdm_transform_dct(const void* X, int x_dtype, void* Y, int y_dtype, int32_t d,
                        const int64_t* dims, int32_t k, int inverse, int compute, void* stream) {
    clear_error();
    TSVDM_REQUIRE(dims != nullptr, TSVDM_E_ARG, "dims is NULL");
    TSVDM_REQUIRE(d >= 3 && d <= 32, TSVDM_E_SHAPE, "d must be in [3, 32]");
    TSVDM_REQUIRE(k >= 3 && k <= d, TSVDM_E_ARG, "k must be in [3, d]");
    int64_t R = 1, P = 1;
    for (int i = 0; i < d; ++i) {
        TSVDM_REQUIRE(dims[i] >= 1 && dims[i] < ((int64_t)1 << 31), TSVDM_E_SHAPE,
                      "every dimension must be in [1, 2^31)");
        int64_t& acc = (i + 1 < k) ? R : P;
        if (i + 1 == k) continue;
        TSVDM_REQUIRE(acc <= (((int64_t)1 << 46) / dims[i]), TSVDM_E_SHAPE, "tensor too large");
        acc *= dims[i];
    }
    const int64_t n = dims[k - 1];
    TSVDM_REQUIRE(n >= 2 && n <= 1024 && (n & (n - 1)) == 0, TSVDM_E_SHAPE,
                  "n_k must be a power of two in [2, 1024]");
    TSVDM_REQUIRE(R < ((int64_t)1 << 31), TSVDM_E_SHAPE,
                  "the dimensions before mode k must multiply to below 2^31");
    TSVDM_REQUIRE(R <= (((int64_t)1 << 46) / n) / P, TSVDM_E_SHAPE, "tensor too large");
    TSVDM_REQUIRE(X && Y, TSVDM_E_ARG, "X and Y must be non-NULL");
    TSVDM_REQUIRE(X != Y, TSVDM_E_ARG, "Y must not alias X");
    TSVDM_REQUIRE(io_dtype(x_dtype) && io_dtype(y_dtype), TSVDM_E_UNSUPPORTED,
                  "x_dtype and y_dtype must be F64 or F32");
    TSVDM_REQUIRE(compute == TSVDM_F64 || compute == TSVDM_F32, TSVDM_E_UNSUPPORTED,
                  "compute must be F64 or F32");
    TSVDM_REQUIRE(inverse == 0 || inverse == 1, TSVDM_E_ARG, "inverse must be 0 or 1");
    return run_dct_mode(X, x_dtype, Y, y_dtype, R, n, P, inverse, compute, as_stream(stream));
}

// ------------------------------------------------------------- slice SVD

int tsvdm_slice_svd_workspace_size(int64_t m, int64_t p, int64_t n, int dtype, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    *bytes = jacobi_workspace_bytes(m < p ? m : p, n);
    return TSVDM_OK;
}

int tsvdm_slice_svd(void* A_hat, int dtype, int64_t m, int64_t p, int64_t n, void* W, double* s2,
                    int32_t* status, int block, int max_sweeps, double tol, int host_poll,
                    void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A_hat && W && s2 && status, TSVDM_E_ARG, "A_hat, W, s2 and status must be non-NULL");
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    TSVDM_REQUIRE(block == 0 || block == 16 || block == 32, TSVDM_E_ARG, "block must be 0, 16 or 32");
    TSVDM_REQUIRE(max_sweeps >= 0 && max_sweeps <= 1000, TSVDM_E_ARG, "max_sweeps must be in [0, 1000]");
    TSVDM_REQUIRE(tol >= 0.0 && tol < 1.0 && std::isfinite(tol), TSVDM_E_ARG, "tol must lie in [0, 1)");
    TSVDM_REQUIRE(host_poll == 0 || host_poll == 1, TSVDM_E_ARG, "host_poll must be 0 or 1");
    TSVDM_TRY(check_ws(ws, ws_bytes, jacobi_workspace_bytes(m < p ? m : p, n)));
    JacobiOpts o = jacobi_default_opts(m, p, dtype);
    if (block) o.block = 2 * block;
    if (max_sweeps) o.max_sweeps = max_sweeps;
    if (tol > 0.0) o.tol = tol;
    o.host_poll = host_poll;
    return run_jacobi(A_hat, dtype, m, p, n, W, s2, status, o, ws, as_stream(stream));
}

int tsvdm_slice_svd_precond_workspace_size(int64_t m, int64_t p, int64_t n, int dtype, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(dtype == TSVDM_F64, TSVDM_E_UNSUPPORTED, "dtype must be F64");
    TSVDM_REQUIRE(std::min(m, p) <= GRAM_MAX_R, TSVDM_E_SHAPE, "min(m, p) must be <= 1024");
    *bytes = precond_svd_workspace_bytes(m, p, n, dtype);
    return TSVDM_OK;
}

int tsvdm_slice_svd_precond(const void* A_hat, int dtype, int64_t m, int64_t p, int64_t n, void* X,
                            void* W, double* s2, int32_t* status, int block, int max_sweeps,
                            double tol, int host_poll, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A_hat && X && W && s2 && status, TSVDM_E_ARG, "A_hat, X, W, s2 and status must be non-NULL");
    TSVDM_REQUIRE(A_hat != X, TSVDM_E_ARG, "X must not alias A_hat");
    TSVDM_REQUIRE(dtype == TSVDM_F64, TSVDM_E_UNSUPPORTED, "dtype must be F64");
    TSVDM_REQUIRE(std::min(m, p) <= GRAM_MAX_R, TSVDM_E_SHAPE, "min(m, p) must be <= 1024");
    TSVDM_REQUIRE(n < 65536, TSVDM_E_SHAPE, "n must be below 65536");
    TSVDM_REQUIRE(block == 0 || block == 16 || block == 32, TSVDM_E_ARG, "block must be 0, 16 or 32");
    TSVDM_REQUIRE(max_sweeps >= 0 && max_sweeps <= 1000, TSVDM_E_ARG, "max_sweeps must be in [0, 1000]");
    TSVDM_REQUIRE(tol >= 0.0 && tol < 1.0 && std::isfinite(tol), TSVDM_E_ARG, "tol must lie in [0, 1)");
    TSVDM_REQUIRE(host_poll == 0 || host_poll == 1, TSVDM_E_ARG, "host_poll must be 0 or 1");
    TSVDM_TRY(check_ws(ws, ws_bytes, precond_svd_workspace_bytes(m, p, n, dtype)));
    JacobiOpts o = jacobi_default_opts(m, p, dtype);
    if (block) o.block = 2 * block;
    if (max_sweeps) o.max_sweeps = max_sweeps;
    if (tol > 0.0) o.tol = tol;
    o.host_poll = host_poll;
    return run_precond_svd(A_hat, dtype, m, p, n, X, W, s2, status, o, ws, as_stream(stream));
}

int tsvdm_slice_svd_gram_workspace_size(int64_t m, int64_t p, int64_t n, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_TRY(check_shape(m, p, n));
    *bytes = gram_svd_workspace_bytes(m, p, n);
    return TSVDM_OK;
}

int tsvdm_slice_svd_gram(const void* A_hat, int64_t m, int64_t p, int64_t n, void* B, double* s2,
                         double* shift, int32_t* status, int block, int max_sweeps, double tol,
                         int jacobi, int host_poll, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A_hat && B && s2 && shift && status, TSVDM_E_ARG,
                  "A_hat, B, s2, shift and status must be non-NULL");
    TSVDM_REQUIRE(A_hat != B, TSVDM_E_ARG, "B must not alias A_hat");
    TSVDM_REQUIRE(std::min(m, p) <= GRAM_MAX_R, TSVDM_E_SHAPE, "min(m, p) must be <= 1024");
    TSVDM_REQUIRE(block == 0 || block == 16 || block == 32, TSVDM_E_ARG, "block must be 0, 16 or 32");
    TSVDM_REQUIRE(max_sweeps >= 0 && max_sweeps <= 1000, TSVDM_E_ARG, "max_sweeps must be in [0, 1000]");
    TSVDM_REQUIRE(tol >= 0.0 && tol < 1.0 && std::isfinite(tol), TSVDM_E_ARG, "tol must lie in [0, 1)");
    TSVDM_REQUIRE(host_poll == 0 || host_poll == 1, TSVDM_E_ARG, "host_poll must be 0 or 1");
    TSVDM_REQUIRE(jacobi == TSVDM_GRAM_AUTO || jacobi == TSVDM_GRAM_ROUNDS || jacobi == TSVDM_GRAM_LDS,
                  TSVDM_E_ARG, "jacobi must be TSVDM_GRAM_AUTO, _ROUNDS or _LDS");
    TSVDM_REQUIRE(jacobi != TSVDM_GRAM_LDS || std::min(m, p) <= GRAM_LDS_MAX_R, TSVDM_E_SHAPE,
                  "TSVDM_GRAM_LDS needs min(m, p) <= 128");
    TSVDM_TRY(check_ws(ws, ws_bytes, gram_svd_workspace_bytes(m, p, n)));
    const int64_t r = std::min(m, p);
    JacobiOpts o = jacobi_default_opts(r, r, TSVDM_F32);
    if (block) o.block = 2 * block;
    if (max_sweeps) o.max_sweeps = max_sweeps;
    if (tol > 0.0) o.tol = tol;
    o.host_poll = host_poll;
    return run_gram_svd(static_cast<const float*>(A_hat), m, p, n, static_cast<float*>(B), s2, shift,
                        status, o, jacobi, ws, as_stream(stream));
}

int tsvdm_pack_gram(const void* A_hat, const void* B, const double* s2, const double* shift,
                    int64_t m, int64_t p, int64_t n, const int32_t* rho, const int64_t* offsets,
                    int64_t capacity, void* U_pk, void* G_pk, void* S_pk, int32_t* status, void* ws,
                    size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A_hat && B && s2 && shift && rho && offsets && status, TSVDM_E_ARG,
                  "A_hat, B, s2, shift, rho, offsets and status must be non-NULL");
    TSVDM_REQUIRE(capacity >= 0, TSVDM_E_ARG, "capacity must be >= 0");
    TSVDM_REQUIRE(capacity == 0 || (U_pk && G_pk && S_pk), TSVDM_E_ARG,
                  "U_pk, G_pk and S_pk must be non-NULL when capacity > 0");
    TSVDM_REQUIRE(std::min(m, p) <= GRAM_MAX_R, TSVDM_E_SHAPE, "min(m, p) must be <= 1024");
    TSVDM_TRY(check_ws(ws, ws_bytes, pack_workspace_bytes(m, p, n)));
    return run_gram_pack(static_cast<const float*>(A_hat), static_cast<const float*>(B), s2, shift,
                         m, p, n, rho, offsets, capacity, static_cast<float*>(U_pk),
                         static_cast<float*>(G_pk), static_cast<float*>(S_pk), status, ws,
                         as_stream(stream));
}

// ------------------------------------------------------------- truncation

int tsvdm_truncate_rank(int64_t k, int64_t r, int64_t n, int32_t* rho, int64_t* offsets,
                        void* stream) {
    clear_error();
    TSVDM_REQUIRE(rho && offsets, TSVDM_E_ARG, "rho and offsets must be non-NULL");
    TSVDM_REQUIRE(k >= 1, TSVDM_E_ARG, "k must be >= 1");
    TSVDM_REQUIRE(r >= 1 && r < kMaxDim && n >= 1 && n < ((int64_t)1 << 31), TSVDM_E_SHAPE,
                  "r and n must be positive");
    return run_truncate_rank(k, r, n, rho, offsets, as_stream(stream));
}

int tsvdm_truncate_tol_workspace_size(int64_t r, int64_t n, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_REQUIRE(r >= 1 && n >= 1 && r * n <= ((int64_t)1 << 30), TSVDM_E_SHAPE,
                  "r*n must be in [1, 2^30]");
    *bytes = select_workspace_bytes(r, n);
    return TSVDM_OK;
}

int tsvdm_truncate_tol(const double* s2, int64_t r, int64_t n, double eps, int32_t* rho,
                       int64_t* offsets, double* stats, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_REQUIRE(s2 && rho && offsets && stats, TSVDM_E_ARG,
                  "s2, rho, offsets and stats must be non-NULL");
    TSVDM_REQUIRE(r >= 1 && n >= 1 && r * n <= ((int64_t)1 << 30) && n < 65536, TSVDM_E_SHAPE,
                  "r*n must be in [1, 2^30] and n < 65536");
    TSVDM_REQUIRE(eps > 0.0 && eps < 1.0, TSVDM_E_ARG, "eps must lie in (0, 1)");
    TSVDM_TRY(check_ws(ws, ws_bytes, select_workspace_bytes(r, n)));
    return run_truncate_tol(s2, r, n, eps, rho, offsets, stats, ws, as_stream(stream));
}

int tsvdm_truncate_tol_noalloc(const double* s2, int64_t r, int64_t n, double eps, int32_t* rho,
                               int64_t* offsets, double* stats, void* stream) {
    clear_error();
    TSVDM_REQUIRE(s2 && rho && offsets && stats, TSVDM_E_ARG,
                  "s2, rho, offsets and stats must be non-NULL");
    TSVDM_REQUIRE(r >= 1 && n >= 1 && r * n <= static_select_max_keys() && n < 65536, TSVDM_E_SHAPE,
                  "r*n must be in [1, " + std::to_string(static_select_max_keys()) + "] and n < 65536");
    TSVDM_REQUIRE(eps > 0.0 && eps < 1.0, TSVDM_E_ARG, "eps must lie in (0, 1)");
    return run_truncate_tol_static(s2, r, n, eps, rho, offsets, stats, as_stream(stream));
}

int tsvdm_slice_svd_subset(void* A_hat, int dtype, int64_t m, int64_t p, int64_t n, void* W,
                           double* s2, int32_t* status, const int32_t* run, int block,
                           int max_sweeps, double tol, int host_poll, void* ws, size_t ws_bytes,
                           void* stream) {
    clear_error();
    TSVDM_REQUIRE(run != nullptr, TSVDM_E_ARG, "run must be non-NULL");
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A_hat && W && s2 && status, TSVDM_E_ARG, "A_hat, W, s2 and status must be non-NULL");
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    TSVDM_REQUIRE(block == 0 || block == 16 || block == 32, TSVDM_E_ARG, "block must be 0, 16 or 32");
    TSVDM_REQUIRE(max_sweeps >= 0 && max_sweeps <= 1000, TSVDM_E_ARG, "max_sweeps must be in [0, 1000]");
    TSVDM_REQUIRE(tol >= 0.0 && tol < 1.0 && std::isfinite(tol), TSVDM_E_ARG, "tol must lie in [0, 1)");
    TSVDM_REQUIRE(host_poll == 0 || host_poll == 1, TSVDM_E_ARG, "host_poll must be 0 or 1");
    TSVDM_TRY(check_ws(ws, ws_bytes, jacobi_workspace_bytes(m < p ? m : p, n)));
    JacobiOpts o = jacobi_default_opts(m, p, dtype);
    if (block) o.block = 2 * block;
    if (max_sweeps) o.max_sweeps = max_sweeps;
    if (tol > 0.0) o.tol = tol;
    o.host_poll = host_poll;
    o.run = run;
    return run_jacobi(A_hat, dtype, m, p, n, W, s2, status, o, ws, as_stream(stream));
}

int tsvdm_slice_energy(const void* A_hat, int dtype, int64_t m, int64_t p, int64_t n, double* E,
                       void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A_hat && E, TSVDM_E_ARG, "A_hat and E must be non-NULL");
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    return run_slice_energy(A_hat, dtype, m, p, n, E, as_stream(stream));
}

int tsvdm_certify_lump(const double* E, const int32_t* computed, double* s2, int64_t r, int64_t n,
                       void* stream) {
    clear_error();
    TSVDM_REQUIRE(E && computed && s2, TSVDM_E_ARG, "E, computed and s2 must be non-NULL");
    TSVDM_REQUIRE(r >= 1 && n >= 1 && r <= (((int64_t)1 << 46) / n), TSVDM_E_SHAPE,
                  "r and n must be positive (r*n below 2^46)");
    return run_lump_s2(E, computed, s2, r, n, as_stream(stream));
}

int tsvdm_certify_check(const double* E, const double* stats, int32_t* computed, int32_t* run_next,
                        int64_t n, int force, int32_t* certified, void* stream) {
    clear_error();
    TSVDM_REQUIRE(E && stats && computed && run_next && certified, TSVDM_E_ARG,
                  "E, stats, computed, run_next and certified must be non-NULL");
    TSVDM_REQUIRE(n >= 1, TSVDM_E_SHAPE, "n must be positive");
    TSVDM_REQUIRE(force == 0 || force == 1, TSVDM_E_ARG, "force must be 0 or 1");
    TSVDM_REQUIRE((const void*)computed != (const void*)run_next, TSVDM_E_ARG,
                  "computed and run_next must be distinct");
    return run_certify(E, stats, computed, run_next, n, force, certified, as_stream(stream));
}

// ------------------------------------------------------------- pack

int tsvdm_pack_workspace_size(int64_t m, int64_t p, int64_t n, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_TRY(check_shape(m, p, n));
    *bytes = pack_workspace_bytes(m, p, n);
    return TSVDM_OK;
}

int tsvdm_pack(const void* A_hat, const void* W, const double* s2, int dtype, int64_t m,
               int64_t p, int64_t n, const int32_t* rho, const int64_t* offsets,
               int64_t capacity, void* U_pk, void* G_pk, void* S_pk, int32_t* status, void* ws,
               size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A_hat && W && s2 && rho && offsets && status, TSVDM_E_ARG,
                  "A_hat, W, s2, rho, offsets and status must be non-NULL");
    TSVDM_REQUIRE(capacity >= 0, TSVDM_E_ARG, "capacity must be >= 0");
    TSVDM_REQUIRE(capacity == 0 || (U_pk && G_pk && S_pk), TSVDM_E_ARG,
                  "U_pk, G_pk and S_pk must be non-NULL when capacity > 0");
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    TSVDM_REQUIRE(std::min(m, p) <= 4096, TSVDM_E_SHAPE, "min(m, p) must be <= 4096");
    TSVDM_TRY(check_ws(ws, ws_bytes, pack_workspace_bytes(m, p, n)));
    return run_pack(A_hat, W, s2, dtype, m, p, n, rho, offsets, capacity, U_pk, G_pk, S_pk,
                    status, ws, as_stream(stream));
}

// ------------------------------------------------------------- reconstruct

int tsvdm_reconstruct_workspace_size(int64_t m, int64_t p, int64_t n, int dtype, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    *bytes = reconstruct_bytes(m, p, n, dtype);
    return TSVDM_OK;
}

int tsvdm_reconstruct(const void* U_pk, const void* G_pk, int dtype, int64_t m, int64_t p,
                      int64_t n, const int32_t* rho, const int64_t* offsets, int64_t capacity,
                      const double* M, double scale, void* A_rec, int out_dtype, int compute,
                      int tile, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(rho && offsets && M && A_rec, TSVDM_E_ARG,
                  "rho, offsets, M and A_rec must be non-NULL");
    TSVDM_REQUIRE(capacity >= 0, TSVDM_E_ARG, "capacity must be >= 0");
    TSVDM_REQUIRE(capacity == 0 || (U_pk && G_pk), TSVDM_E_ARG,
                  "U_pk and G_pk must be non-NULL when capacity > 0");
    TSVDM_REQUIRE(io_dtype(dtype) && io_dtype(out_dtype), TSVDM_E_UNSUPPORTED,
                  "dtype and out_dtype must be F64 or F32");
    TSVDM_REQUIRE(compute >= TSVDM_F64 && compute <= TSVDM_BF16X3, TSVDM_E_UNSUPPORTED,
                  "unknown compute dtype");
    TSVDM_REQUIRE(!(compute >= TSVDM_BF16 && out_dtype != TSVDM_F32), TSVDM_E_UNSUPPORTED,
                  "BF16 compute writes F32 output only");
    TSVDM_REQUIRE(std::isfinite(scale), TSVDM_E_ARG, "scale must be finite");
    TSVDM_REQUIRE(tile >= 0 && tile <= TTM_SHAPES, TSVDM_E_ARG, "tile must be in [0, 8]");
    const size_t need = reconstruct_bytes(m, p, n, dtype);
    TSVDM_TRY(check_ws(ws, ws_bytes, need));
    Carver cv(ws);
    void* C = cv.carve<char>((size_t)(m * p * n) * esize(dtype));
    void* tws = cv.carve<char>(ttm_workspace_bytes(n));
    hipStream_t st = as_stream(stream);
    TSVDM_TRY(run_lowrank_gemm(U_pk, G_pk, dtype, m, p, n, rho, offsets, capacity, C, st));
    return run_ttm(C, dtype, A_rec, out_dtype, m, p, n, M, 1, scale, compute, tile, tws, st);
}

int tsvdm_lowrank(const void* U_pk, const void* G_pk, int dtype, int64_t m, int64_t p, int64_t n,
                  const int32_t* rho, const int64_t* offsets, int64_t capacity, void* C,
                  void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(rho && offsets && C, TSVDM_E_ARG, "rho, offsets and C must be non-NULL");
    TSVDM_REQUIRE(capacity >= 0, TSVDM_E_ARG, "capacity must be >= 0");
    TSVDM_REQUIRE(capacity == 0 || (U_pk && G_pk), TSVDM_E_ARG,
                  "U_pk and G_pk must be non-NULL when capacity > 0");
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    return run_lowrank_gemm(U_pk, G_pk, dtype, m, p, n, rho, offsets, capacity, C, as_stream(stream));
}

// ------------------------------------------------------------- error report

int tsvdm_error_workspace_size(int64_t count, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_REQUIRE(count > 0, TSVDM_E_SHAPE, "count must be positive");
    *bytes = error_workspace_bytes(count);
    return TSVDM_OK;
}

int tsvdm_error(const void* A, int a_dtype, const void* B, int b_dtype, int64_t count,
                double* out, void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_REQUIRE(A && B && out, TSVDM_E_ARG, "A, B and out must be non-NULL");
    TSVDM_REQUIRE(count > 0, TSVDM_E_SHAPE, "count must be positive");
    TSVDM_REQUIRE(io_dtype(a_dtype) && io_dtype(b_dtype), TSVDM_E_UNSUPPORTED,
                  "dtypes must be F64 or F32");
    TSVDM_TRY(check_ws(ws, ws_bytes, error_workspace_bytes(count)));
    return run_error(A, a_dtype, B, b_dtype, count, out, ws, as_stream(stream));
}

// ------------------------------------------------------------- adjoint

int tsvdm_backward_workspace_size(int64_t m, int64_t p, int64_t n, int dtype, size_t* bytes) {
    clear_error();
    TSVDM_REQUIRE(bytes != nullptr, TSVDM_E_ARG, "bytes is NULL");
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    *bytes = backward_workspace_bytes(m, p, n, dtype);
    return TSVDM_OK;
}

int tsvdm_backward(const void* A, int dtype, int64_t m, int64_t p, int64_t n, const double* M,
                   int64_t k, double g, void* dA, double* dM, double* loss, int32_t* status,
                   void* ws, size_t ws_bytes, void* stream) {
    clear_error();
    TSVDM_TRY(check_shape(m, p, n));
    TSVDM_REQUIRE(A && M && status, TSVDM_E_ARG, "A, M and status must be non-NULL");
    TSVDM_REQUIRE(io_dtype(dtype), TSVDM_E_UNSUPPORTED, "dtype must be F64 or F32");
    TSVDM_REQUIRE(k >= 1, TSVDM_E_ARG, "k must be >= 1");
    TSVDM_REQUIRE(std::isfinite(g), TSVDM_E_ARG, "g must be finite");
    TSVDM_REQUIRE(std::min(m, p) <= 4096, TSVDM_E_SHAPE, "min(m, p) must be <= 4096");
    TSVDM_TRY(check_ws(ws, ws_bytes, backward_workspace_bytes(m, p, n, dtype)));
    return run_backward(A, dtype, m, p, n, M, k, g, dA, dM, loss, status, ws, as_stream(stream));
}

// ------------------------------------------------------------- statistics

int tsvdm_stats_enable(int on) {
    clear_error();
    TSVDM_REQUIRE(on == 0 || on == 1, TSVDM_E_ARG, "on must be 0 or 1");
    stats_set(on != 0);
    return TSVDM_OK;
}

int tsvdm_stats_reset(void) {
    clear_error();
    stats_reset();
    return TSVDM_OK;
}

int tsvdm_stats_get(int64_t* launches, double* ms, int64_t* pairs_gram, int64_t* pairs_rot,
                    int32_t* pair_width, double* flops, double* bytes) {
    clear_error();
    stats_get(launches, ms, pairs_gram, pairs_rot, pair_width, flops, bytes);
    return TSVDM_OK;
}

}  // extern "C"

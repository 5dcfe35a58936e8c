/*
 * tsvdm.h -- C ABI of the MI355X (gfx950) star-M truncated tensor SVD.
 *
 * The library computes the data-parallel hot path of the star-M t-SVD
 * (Hussain et al., "High-Performance star-M SVD for Big Data Compression"):
 *
 *   transform      A-hat = A x_3 M                      Section 2.1, Algorithm 1
 *   slice SVDs     A-hat_i = U_i S_i V_i^T, i = 1..n     Algorithm 1, Section 3.2
 *   truncation     t-SVDM-I: rank k on every slice       Section 3.3
 *                  t-SVDM-II: global tolerance eps       Algorithm 2
 *   factors        U_i(:, 1:rho_i), s_i, G_i = S V^T     Algorithm 2, Section 3.4
 *   reconstruct    A_rho = (U_i G_i)_i x_3 M^{-1}        Section 2.1
 *   adjoint        d/dA and d/dM of the truncation loss  (not in the paper)
 *
 * Conventions (all entry points)
 * ------------------------------
 *  - Tensors are column-major (Section 3): element (a, b, i) of an m x p x n
 *    tensor is at offset a + b*m + i*m*p, so frontal slice i is a contiguous
 *    m x p column-major matrix.  r = min(m, p).
 *  - Every data pointer is a DEVICE pointer owned by the caller.  The library
 *    never frees caller memory and keeps no pointer after a call returns
 *    (batch plans keep only host data and graph objects).
 *  - M (device, FP64) is used as given by tsvdm_transform, tsvdm_transform_mode
 *    and tsvdm_reconstruct: these calls cannot read device memory before
 *    launching, so they do not check it.  Check a transform once on the host
 *    with tsvdm_check_transform (Algorithm 2 requires M = c*Q with Q
 *    orthogonal; a matrix that is not gives a silently wrong A_rho) and pass
 *    the back-transform scale 1/c^2 it returns.
 *  - Every compute call is enqueued on `stream` (a hipStream_t passed as
 *    void*; NULL = the default stream) and returns before the work finishes.
 *    Results are valid after the stream is synchronised.
 *  - Errors that can be seen on the host (bad sizes, null pointers, a too
 *    small workspace, an unsupported dtype) return a negative tsvdm_status
 *    BEFORE anything is launched; tsvdm_last_error() then holds a message
 *    (thread-local).  Conditions seen on the device (Jacobi not converged,
 *    a non-finite value, an undersized packed output) are written as a
 *    tsvdm_status into the caller's device status word and never abort.
 *  - Workspace: each entry point that needs scratch memory takes (ws, ws_bytes);
 *    the required size comes from the matching *_workspace_size query.
 *    Workspace contents need not be initialised and are not preserved.
 *  - Calls that share a workspace or outputs must not overlap in time.
 */
#ifndef TSVDM_H
#define TSVDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TSVDM_OK = 0,
    TSVDM_E_ARG = -1,         /* null pointer, bad flag or tolerance        */
    TSVDM_E_SHAPE = -2,       /* a size is <= 0 or too large                */
    TSVDM_E_NOT_ORTHO = -3,   /* M is not a multiple of an orthogonal matrix */
    TSVDM_E_WORKSPACE = -4,   /* ws_bytes smaller than the query returned    */
    TSVDM_E_NOCONV = -5,      /* (device) Jacobi hit max_sweeps             */
    TSVDM_E_NONFINITE = -6,   /* (device) NaN or Inf met                    */
    TSVDM_E_HIP = -7,         /* a HIP runtime call failed                  */
    TSVDM_E_UNSUPPORTED = -8, /* dtype or option not available              */
    TSVDM_E_CAPACITY = -9     /* (device) packed output smaller than sum rho */
} tsvdm_status;

/* Element types.  BF16X3 is a compute mode only: each FP32 operand x is split
 * into hi = bf16(x) and lo = bf16(x - hi), and the product is formed from the
 * three MFMA products hi*hi + hi*lo + lo*hi with FP32 accumulation. */
typedef enum {
    TSVDM_F64 = 0,
    TSVDM_F32 = 1,
    TSVDM_BF16 = 2,
    TSVDM_BF16X3 = 3
} tsvdm_dtype;

/* --------------------------------------------------------------------- */
/* library                                                               */
/* --------------------------------------------------------------------- */

/* Library version as 10000*major + 100*minor + patch. */
int tsvdm_version(void);

/* Message of the last failing call on this thread ("" if none).  The string
 * stays valid until the next tsvdm_* call on the same thread. */
const char* tsvdm_last_error(void);

/* Host-side check that the n x n column-major FP64 matrix M_host is c*Q with
 * Q orthogonal: max |M^T M / c^2 - I| <= tol with c^2 = mean(diag(M^T M)).
 * Algorithm 2 requires such an M and Section 3 restricts to orthonormal M.
 * On success writes c^2 to *scale_sq (may be NULL) and returns TSVDM_OK,
 * else TSVDM_E_NOT_ORTHO.  Reads host memory only; launches nothing. */
int tsvdm_check_transform(const double* M_host, int64_t n, double tol,
                          double* scale_sq);

/* --------------------------------------------------------------------- */
/* mode-3 transform (Section 2.1; Section 3.1, last-mode TTM as one GEMM) */
/* --------------------------------------------------------------------- */

/* Y = X x_3 (scale * op(M)):  Y(:,:,i) = scale * sum_l op(M)[i,l] X(:,:,l),
 * op(M) = M (transpose = 0) or M^T (transpose = 1).  The forward transform
 * is (transpose = 0, scale = 1); the back-transform of an orthonormal M is
 * (transpose = 1, scale = 1) and of M = c*Q is (1, 1/c^2).
 *   X        device, x_dtype (F64 or F32), m*p*n elements, column-major.
 *   Y        device, y_dtype (F64 or F32), m*p*n elements; must not alias X.
 *   M        device, FP64, n x n column-major.
 *   compute  F64: FP64 MFMA; F32: FP32 MFMA; BF16 / BF16X3: BF16 MFMA with
 *            FP32 accumulation (y_dtype must then be F32).
 *   tile     workgroup tile of the (mp) x n output, rows x slices:
 *            TSVDM_TILE_64x64, TSVDM_TILE_128x32, TSVDM_TILE_256x16 (16
 *            slices per wave), TSVDM_TILE_128x64, TSVDM_TILE_256x32 (32),
 *            TSVDM_TILE_128x128, TSVDM_TILE_256x64 (64),
 *            TSVDM_TILE_64x64_2x2 (four waves of 32 rows x 32 slices), or
 *            TSVDM_TILE_AUTO: 256x16 for n <= 16, 128x32 for n <= 32, else
 *            64x64_2x2 for F64 and, for the FP32-operand forms, 128x64 up
 *            to n = 64 and 128x128 above.  Every tile gives the same
 *            result; only the speed differs.
 * ws: tsvdm_transform_workspace_size bytes (holds op(M) in compute type). */
enum {
    TSVDM_TILE_AUTO = 0,
    TSVDM_TILE_64x64 = 1,
    TSVDM_TILE_128x32 = 2,
    TSVDM_TILE_256x16 = 3,
    TSVDM_TILE_128x64 = 4,
    TSVDM_TILE_256x32 = 5,
    TSVDM_TILE_128x128 = 6,
    TSVDM_TILE_256x64 = 7,
    TSVDM_TILE_64x64_2x2 = 8
};
int tsvdm_transform_workspace_size(int64_t n, size_t* bytes);
int tsvdm_transform(const void* X, int x_dtype, void* Y, int y_dtype,
                    int64_t m, int64_t p, int64_t n,
                    const double* M, int transpose, double scale,
                    int compute, int tile, void* ws, size_t ws_bytes, void* stream);

/* Mode-k transform of an order-d tensor (Section 2.1, footnote: every mode
 * k >= 3 has its own transform; Section 3.1, middle-mode TTM):
 * Y = X x_k (scale * op(M)) for 3 <= k <= d, where dims (host, d entries)
 * holds n_1 ... n_d and X, Y (device, column-major, prod(dims) elements,
 * no aliasing) keep mode 1 fastest.  The tensor is the P = n_{k+1}...n_d
 * contiguous blocks of the (n_1...n_{k-1}) x n_k matrix; all blocks run as
 * one launch (k = d is the last-mode case, P = 1).  M: device FP64 n_k x n_k
 * column-major.  x_dtype, y_dtype, transpose, scale, compute and tile as in
 * tsvdm_transform; ws: tsvdm_transform_workspace_size(n_k) bytes.  A 3-way
 * tensor with k = 3 is exactly tsvdm_transform. */
int tsvdm_transform_mode(const void* X, int x_dtype, void* Y, int y_dtype,
                         int32_t d, const int64_t* dims, int32_t k,
                         const double* M, int transpose, double scale,
                         int compute, int tile, void* ws, size_t ws_bytes, void* stream);

/* Fast mode-k transform by the orthonormal DCT-II C (C_qj = s_q cos(pi q
 * (2j + 1) / (2 n_k)), s_0 = sqrt(1/n_k), s_q = sqrt(2/n_k)): Y = X x_k C
 * (inverse = 0) or Y = X x_k C^T = X x_k C^-1 (inverse = 1), computed by an
 * FFT in O(log n_k) work per element instead of the dense product's O(n_k)
 * (Section 2.2, choice of M: the DCT applies in O(n log n); Section 5,
 * operator transforms for the TTM stage).  The result equals
 * tsvdm_transform_mode with M = C (scale 1) up to rounding.
 *   X, Y     device, column-major, prod(dims) elements, no aliasing.
 *   d, dims, k  as in tsvdm_transform_mode (d = 3, k = 3: the 3-way case).
 *   n_k      a power of two in [2, 1024]; the product of the dimensions
 *            before mode k below 2^31.
 *   compute  TSVDM_F64 or TSVDM_F32: the FFT's arithmetic (twiddles are
 *            computed in FP64 and rounded once).
 * No workspace.  Errors: TSVDM_E_SHAPE for an unsupported n_k, the others
 * as in tsvdm_transform_mode. */
int tsvdm_transform_dct(const void* X, int x_dtype, void* Y, int y_dtype,
                        int32_t d, const int64_t* dims, int32_t k, int inverse,
                        int compute, void* stream);

/* --------------------------------------------------------------------- */
/* slice SVDs (Algorithm 1; Section 3.2)                                 */
/* --------------------------------------------------------------------- */

/* One-sided block Jacobi SVD of every frontal slice of A_hat (m x p x n,
 * dtype F64 or F32), in place.
 * The r = min(m, p) "Jacobi vectors" are the columns of the slice when
 * m >= p and its rows when m < p.  On return:
 *   A_hat    the vectors are mutually orthogonal: for m >= p column j of
 *            slice i is sigma_j u_j; for m < p row j is sigma_j v_j^T.
 *   W        (r x r x n, same dtype) the accumulated rotations: V when
 *            m >= p, U when m < p (so A_hat_i = U (S V^T) or (U S) V^T).
 *   s2       (r x n, FP64) squared norms of the final vectors, i.e. the
 *            squared singular values in the same (unsorted) order.
 *   status   (device int32, 1 element) TSVDM_OK or TSVDM_E_NOCONV /
 *            TSVDM_E_NONFINITE.
 * Options:
 *   block    Jacobi block width b (16 or 32; 0 = 32 when min(m, p) >= 256,
 *            else 16).
 *   max_sweeps  sweep limit (0 = 40).
 *   tol      convergence threshold on |cos| between any two vectors, tested
 *            in FP64 (0 = default: 1e-14 for F64, 2e-6 for F32).
 *   host_poll   1: read the count of unconverged slices after every sweep
 *            and stop early; the host reads sweep s's count once sweep
 *            s + 1 is queued (so at most one sweep that changes nothing
 *            runs after convergence) and waits for the last count before
 *            returning; not usable under stream capture.  0: launch
 *            max_sweeps sweeps whose kernels return at once after
 *            convergence (graph-capturable).  Results are the same bits
 *            either way.
 * Rotation angles, the convergence test and s2 are computed in FP64 for
 * both dtypes.  A block pair whose vectors measured every |cos| <= tol, and
 * neither of whose blocks has rotated since, is skipped when it meets again
 * (its Gram matrix would be the same bits, so it would not rotate); ws holds
 * these records, (ceil(r / 16) rounded up to even)^2 int32 per slice, beside
 * the per-slice control words. */
int tsvdm_slice_svd_workspace_size(int64_t m, int64_t p, int64_t n, int dtype,
                                   size_t* bytes);
int tsvdm_slice_svd(void* A_hat, int dtype, int64_t m, int64_t p, int64_t n,
                    void* W, double* s2, int32_t* status,
                    int block, int max_sweeps, double tol, int host_poll,
                    void* ws, size_t ws_bytes, void* stream);

/* Slice SVDs by the rotation form, preconditioned by the Gram form
 * (Algorithm 1's slice SVDs; Section 3.2 leaves their method open), in FP64
 * with the rotation form's accuracy.  With r = min(m, p):
 *   1. the Gram form of tsvdm_slice_svd_gram (FP64 Gram matrix, pivoted
 *      shifted Cholesky factor, FP32 Jacobi on its columns to the FP32
 *      tol): unit columns W (r x r, FP64), approximating the short-side
 *      singular vectors, with cosines <= that tol;
 *   2. W made orthonormal to FP64 rounding by Newton-Schulz steps
 *      W <- W (3 I - W^T W) / 2 (quadratic from ||W^T W - I|| <= r tol):
 *      two, and a third on the slices still above the rounding level;
 *   3. X = W^T A_hat (m < p) or A_hat W (m >= p), one GEMM per slice;
 *   4. the one-sided Jacobi of tsvdm_slice_svd on X with W as its starting
 *      accumulator: X and W then hold exactly what tsvdm_slice_svd leaves
 *      in A_hat and W (the same layouts, the same convergence test on the
 *      vectors themselves), in fewer sweeps of the long vectors.
 * dtype: TSVDM_F64 only.
 * A_hat is only read; X (m x p x n, dtype) receives the orthogonalised
 * vectors, W (r x r x n) the accumulated rotation, s2 (r x n, FP64) the
 * squared singular values (unsorted), status TSVDM_OK, TSVDM_E_NOCONV or
 * TSVDM_E_NONFINITE (either stage).  block, max_sweeps, tol and host_poll
 * as in tsvdm_slice_svd (step 1 takes its default tol for vectors of length
 * r).  min(m, p) <= TSVDM_GRAM_MAX_R, n < 65536.
 * ws: tsvdm_slice_svd_precond_workspace_size bytes. */
int tsvdm_slice_svd_precond_workspace_size(int64_t m, int64_t p, int64_t n, int dtype,
                                           size_t* bytes);
int tsvdm_slice_svd_precond(const void* A_hat, int dtype, int64_t m, int64_t p, int64_t n,
                            void* X, void* W, double* s2, int32_t* status, int block,
                            int max_sweeps, double tol, int host_poll, void* ws,
                            size_t ws_bytes, void* stream);

/* Slice SVDs of an FP32 tensor through the FP64 Gram matrix, for the
 * mixed-precision path (Algorithm 1's slice SVDs; Section 3.2 leaves the
 * slice SVD method open).  With r = min(m, p) and X the r Jacobi vectors of
 * a slice (its rows when m < p, its columns otherwise):
 *   G = X X^T in FP64 (exact FP32 products, FP64 sums), then the Cholesky
 *   factor L L^T = G + s I with s = (max(m, p) + r) * 2^-53 * trace(G)
 *   (a pivot that rounding leaves <= 0 gives a zero column), then the
 *   one-sided Jacobi of tsvdm_slice_svd on the columns of L in FP32 with
 *   FP64 angles, accumulating no rotations: L Q = B.
 * Outputs (A_hat is only read and must stay unchanged for tsvdm_pack_gram):
 *   B      (r x r x n, F32, column-major per slice) the orthogonal columns:
 *          b_j / ||b_j|| are the singular vectors of the slice on its short
 *          side (U when m < p, V otherwise), ||b_j||^2 = sigma_j^2 + s;
 *   s2     (r x n, FP64) sigma_j^2 = max(||b_j||^2 - s, 0), unsorted;
 *   shift  (n, FP64) s of each slice;
 *   status as in tsvdm_slice_svd.
 * The eigenvalues of the FP64 Gram matrix carry absolute errors of order
 * 2^-53 ||G||, so sigma_j is accurate to about 2^-53 sigma_max^2 / sigma_j
 * (2^-26.5 sigma_max as sigma_j -> 0), well inside FP32 accuracy; this form
 * is for FP32 results only.  min(m, p) <= TSVDM_GRAM_MAX_R.  block,
 * max_sweeps, tol (default tol from the vector length r) and host_poll as in
 * tsvdm_slice_svd.  jacobi (tsvdm_gram_jacobi) places the Jacobi on L:
 *   TSVDM_GRAM_ROUNDS  the block rounds of tsvdm_slice_svd, L in HBM;
 *   TSVDM_GRAM_LDS     one workgroup per slice runs every sweep with L held
 *                      in LDS, scalar pairs in a cyclic tournament (block
 *                      unused); needs r <= TSVDM_GRAM_LDS_MAX_R;
 *   TSVDM_GRAM_AUTO    LDS for r <= TSVDM_GRAM_LDS_MAX_R, else the rounds.
 * The two placements give different rounding (both within the bound above).
 * ws: tsvdm_slice_svd_gram_workspace_size bytes (holds G and L in FP64). */
#define TSVDM_GRAM_MAX_R 1024
#define TSVDM_GRAM_LDS_MAX_R 128
typedef enum { TSVDM_GRAM_AUTO = 0, TSVDM_GRAM_ROUNDS = 1, TSVDM_GRAM_LDS = 2 } tsvdm_gram_jacobi;
int tsvdm_slice_svd_gram_workspace_size(int64_t m, int64_t p, int64_t n, size_t* bytes);
int tsvdm_slice_svd_gram(const void* A_hat, int64_t m, int64_t p, int64_t n, void* B,
                         double* s2, double* shift, int32_t* status, int block, int max_sweeps,
                         double tol, int jacobi, int host_poll, void* ws, size_t ws_bytes,
                         void* stream);

/* Slice SVDs of a subset: as tsvdm_slice_svd, but only the slices with
 * run[i] != 0 (run: device int32[n]) are computed; every other slice keeps
 * its A_hat, W and s2 entries untouched, so several calls can fill one set
 * of outputs.  Used by the certified t-SVDM-II selection below. */
int tsvdm_slice_svd_subset(void* A_hat, int dtype, int64_t m, int64_t p, int64_t n,
                           void* W, double* s2, int32_t* status, const int32_t* run,
                           int block, int max_sweeps, double tol, int host_poll,
                           void* ws, size_t ws_bytes, void* stream);

/* --------------------------------------------------------------------- */
/* truncation                                                            */
/* --------------------------------------------------------------------- */

/* t-SVDM-I (Section 3.3): rho[i] = min(k, r) for every slice and
 * offsets[i] = sum_{j<i} rho[j] (n+1 entries, offsets[n] = total).
 * rho: device int32[n]; offsets: device int64[n+1]. */
int tsvdm_truncate_rank(int64_t k, int64_t r, int64_t n,
                        int32_t* rho, int64_t* offsets, void* stream);

/* t-SVDM-II (Algorithm 2).  s2: device FP64 [r x n] squared singular values
 * (any order within a slice).  With v the ascending sort of all n*r values,
 * w_J = v_1 + ... + v_J and W = the sum of all values:
 *   J   = the largest J with w_J / W < eps*eps  (J = 0 if none),
 *   tau = v_J (-inf if J = 0),
 *   rho[i] = #{ j : s2[j + i*r] > tau }  (every value equal to tau dropped).
 * Sums are double-double (about 106-bit) and rounded once to FP64, so the
 * decision matches exact arithmetic except within ~1e-30 of a tie.  A zero
 * tensor (W = 0) gives rho = 0.
 * stats (device FP64[4]): tau, discarded energy (sum of dropped values),
 * W, and J (as a double).  eps must lie in (0, 1). */
int tsvdm_truncate_tol_workspace_size(int64_t r, int64_t n, size_t* bytes);
int tsvdm_truncate_tol(const double* s2, int64_t r, int64_t n, double eps,
                       int32_t* rho, int64_t* offsets, double* stats,
                       void* ws, size_t ws_bytes, void* stream);

/* t-SVDM-II selection that allocates nothing, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and errors as
 * tsvdm_truncate_tol without the workspace: the sort keys live in a fixed
 * device array of 2^20 keys (8 MiB per GPU, held until the process ends),
 * so r*n must not exceed 1048576 (else TSVDM_E_SHAPE before any launch).
 * Every call on one GPU shares that array: calls that overlap in time on
 * the same GPU (different streams, threads or processes' shared contexts)
 * race and must be serialised by the caller.  No hipMalloc or hipFree is
 * made; the array's device address is looked up once per device on the
 * first call there. */
int tsvdm_truncate_tol_noalloc(const double* s2, int64_t r, int64_t n, double eps,
                               int32_t* rho, int64_t* offsets, double* stats, void* stream);

/* Certified t-SVDM-II selection (Algorithm 2; Section 4.1: t-SVDM-II
 * discards many slices entirely).  A slice i without an SVD enters the
 * selection as one value, its energy E_i = ||A_hat_i||_F^2 (all its squared
 * singular values are <= E_i and sum to it).  If after tsvdm_truncate_tol
 * every such E_i is strictly below tau, the selection, tau and every rank are
 * exactly those of the full selection (totals agree to rounding: the
 * energies stand in for sums of squared singular values) and those slices
 * get rank 0; otherwise the slices with E_i >= tau need their SVD and the
 * selection is repeated.  One round:
 *   tsvdm_slice_svd_subset(run) -> tsvdm_certify_lump -> tsvdm_truncate_tol
 *   -> tsvdm_certify_check (certified, or run = the slices to add).
 * tsvdm_slice_energy: E[i] = sum of squares of slice i (device FP64[n]),
 *   FP64, fixed summation order.
 * tsvdm_certify_lump: s2[:, i] = (E_i, 0, ..., 0) for computed[i] == 0
 *   (s2: device FP64 [r x n]; computed: device int32[n]).
 * tsvdm_certify_check: certified (device int32[1]) = every E_i with
 *   computed[i] == 0 is finite and < stats[0] (tau, from tsvdm_truncate_tol);
 *   run_next[i] = 1 for those that are not, and computed[i] becomes 1 for
 *   them.  force = 1 instead moves every uncomputed slice into run_next (and
 *   computed) and reports certified = 0: the full computation. */
int tsvdm_slice_energy(const void* A_hat, int dtype, int64_t m, int64_t p, int64_t n,
                       double* E, void* stream);
int tsvdm_certify_lump(const double* E, const int32_t* computed, double* s2,
                       int64_t r, int64_t n, void* stream);
int tsvdm_certify_check(const double* E, const double* stats, int32_t* computed,
                        int32_t* run_next, int64_t n, int force, int32_t* certified,
                        void* stream);

/* --------------------------------------------------------------------- */
/* factor emission (Algorithm 2's final loop; Section 3.4 packed layout) */
/* --------------------------------------------------------------------- */

/* From the output of tsvdm_slice_svd, write for each slice i the rho[i]
 * leading triplets in descending sigma order, packed without padding:
 *   U_pk : column-major m x rho_i block at element offset m*offsets[i]
 *   G_pk : column-major rho_i x p block (G_i = S_i V_i^T) at p*offsets[i]
 *   S_pk : rho_i singular values at offsets[i]
 * All three in `dtype` (the dtype of A_hat / W).  capacity = number of
 * triplets the buffers hold (U_pk has m*capacity elements, ...); if
 * offsets[n] > capacity nothing beyond capacity is written and *status is
 * set to TSVDM_E_CAPACITY.  A kept singular value that is exactly 0 (only
 * possible for t-SVDM-I) gets a zero column in U_pk.
 * ws: tsvdm_pack_workspace_size bytes. */
int tsvdm_pack_workspace_size(int64_t m, int64_t p, int64_t n, size_t* bytes);
int tsvdm_pack(const void* A_hat, const void* W, const double* s2, int dtype,
               int64_t m, int64_t p, int64_t n,
               const int32_t* rho, const int64_t* offsets, int64_t capacity,
               void* U_pk, void* G_pk, void* S_pk, int32_t* status,
               void* ws, size_t ws_bytes, void* stream);

/* tsvdm_pack for the output of tsvdm_slice_svd_gram (F32): the same packed
 * layout, capacity rule and status.  For kept triplet c (descending sigma,
 * index j): u_c = b_j / ||b_j|| and G_i = U_rho^T A_hat_i when m < p;
 * v_c = b_j / ||b_j||, G_i row c = sigma_c v_c^T and u_c = A_hat_i v_c /
 * sigma_c (a zero column when sigma_c = 0) otherwise: one product with the
 * slice gives the long-side factor.  ws: tsvdm_pack_workspace_size bytes. */
int tsvdm_pack_gram(const void* A_hat, const void* B, const double* s2, const double* shift,
                    int64_t m, int64_t p, int64_t n, const int32_t* rho, const int64_t* offsets,
                    int64_t capacity, void* U_pk, void* G_pk, void* S_pk, int32_t* status,
                    void* ws, size_t ws_bytes, void* stream);

/* --------------------------------------------------------------------- */
/* reconstruction (Section 2.1, third step of the star-M product)        */
/* --------------------------------------------------------------------- */

/* C_hat_i = U_pk_i * G_pk_i (variable-rank batched GEMM, `dtype`), then
 * A_rec = C_hat x_3 (scale * M^T) written in out_dtype (F64 or F32);
 * scale = 1 for orthonormal M, 1/c^2 for M = c*Q.  U_pk, G_pk use the
 * packed layout of tsvdm_pack with the same `capacity`; a slice whose block
 * would end beyond capacity contributes zero.  C_hat lives in the workspace
 * (m*p*n elements of `dtype`).  compute and tile select the back-TTM
 * arithmetic and tile shape as in tsvdm_transform. */
int tsvdm_reconstruct_workspace_size(int64_t m, int64_t p, int64_t n,
                                     int dtype, size_t* bytes);
int tsvdm_reconstruct(const void* U_pk, const void* G_pk, int dtype,
                      int64_t m, int64_t p, int64_t n,
                      const int32_t* rho, const int64_t* offsets, int64_t capacity,
                      const double* M, double scale, void* A_rec,
                      int out_dtype, int compute, int tile,
                      void* ws, size_t ws_bytes, void* stream);

/* C (device, m*p*n elements of dtype, column-major) with slice i equal to
 * U_pk_i * G_pk_i (variable-rank batched GEMM, Section 2.1 third step in
 * the transform domain), i.e. the first half of tsvdm_reconstruct without
 * the back-transform: order-d tensors apply their back-transforms mode by
 * mode with tsvdm_transform_mode.  Arguments as in tsvdm_reconstruct; no
 * workspace. */
int tsvdm_lowrank(const void* U_pk, const void* G_pk, int dtype,
                  int64_t m, int64_t p, int64_t n,
                  const int32_t* rho, const int64_t* offsets, int64_t capacity,
                  void* C, void* stream);

/* --------------------------------------------------------------------- */
/* error report                                                          */
/* --------------------------------------------------------------------- */

/* out (device FP64[2]) = { sum (A - B)^2, sum A^2 } over `count` elements,
 * accumulated in FP64 in a fixed order (deterministic).  A, B are F64 or
 * F32 (independently).  ws: tsvdm_error_workspace_size bytes. */
int tsvdm_error_workspace_size(int64_t count, size_t* bytes);
int tsvdm_error(const void* A, int a_dtype, const void* B, int b_dtype,
                int64_t count, double* out, void* ws, size_t ws_bytes,
                void* stream);

/* --------------------------------------------------------------------- */
/* adjoint of the truncation loss (not in the paper)                     */
/* --------------------------------------------------------------------- */

/* L(A, M) = sum_i sum_{j > k} sigma_ij^2 with sigma the singular values of
 * the slices of A x_3 M (for orthogonal M, L = ||A - A_k||_F^2).  With
 * R-hat_i the rank-k tail of slice i (recomputed here: transform, Jacobi,
 * tail reconstruction; the factors are not stored between calls):
 *   dA = 2 g * (R-hat x_3 M^T)            (m x p x n, `dtype`; may be NULL)
 *   dM = 2 g * R-hat_(3) A_(3)^T          (n x n FP64 column-major; may be NULL)
 *   loss (device FP64[1]) = L.
 * A: device, F32 or F64 (dtype also selects the compute precision).
 * M: device FP64 n x n.  Requires sigma_k > sigma_{k+1} in every slice for
 * the gradient to exist (not checked).  status as in tsvdm_slice_svd. */
int tsvdm_backward_workspace_size(int64_t m, int64_t p, int64_t n, int dtype,
                                  size_t* bytes);
int tsvdm_backward(const void* A, int dtype, int64_t m, int64_t p, int64_t n,
                   const double* M, int64_t k, double g,
                   void* dA, double* dM, double* loss, int32_t* status,
                   void* ws, size_t ws_bytes, void* stream);

/* --------------------------------------------------------------------- */
/* batches of independent tensors of any shapes                          */
/* --------------------------------------------------------------------- */

/* One tensor of a batch: t-SVDM-I (mode 1, rank k) or t-SVDM-II (mode 2,
 * tolerance eps) end to end.  All pointers are device pointers owned by the
 * caller; outputs use the layouts of tsvdm_pack / tsvdm_reconstruct and are
 * written in the batch's compute dtype (A_rec, U_pk, G_pk, S_pk). */
typedef struct {
    int64_t m, p, n;
    const void* A;        /* input tensor, in_dtype, column-major              */
    const double* M;      /* n x n FP64 column-major, a multiple of orthogonal  */
    double inv_scale;     /* back-transform scale 1/c^2 (1 for orthonormal M)   */
    int32_t mode;         /* 1 = t-SVDM-I, 2 = t-SVDM-II                        */
    int32_t block;        /* Jacobi block width of its slices: 16, 32, or 0 to  */
                          /* take the plan's (see tsvdm_batch_plan_create)      */
    int64_t k;            /* mode 1 rank (>= 1, clamped to r)                   */
    double eps;           /* mode 2 tolerance, in (0, 1)                        */
    int32_t* rho;         /* out: int32[n] ranks                                */
    int64_t* offsets;     /* out: int64[n+1] packed offsets                     */
    double* stats;        /* out: FP64[4] (tau, discarded, total, J) or NULL    */
    void* U_pk;           /* out: packed factors; NULL = kept in the workspace  */
    void* G_pk;
    void* S_pk;
    int64_t capacity;     /* triplets U_pk/G_pk/S_pk hold (ignored when NULL)   */
    void* A_rec;          /* out: reconstruction m*p*n, or NULL to skip it      */
    double* err;          /* out: FP64[2] {sum (A-A_rec)^2, sum A^2} or NULL    */
    int32_t ttm_tile;     /* transform tile shape (TSVDM_TILE_*) of both TTMs   */
    int32_t reserved;     /* must be 0                                          */
} tsvdm_batch_item;

typedef struct tsvdm_batch_plan_s* tsvdm_batch_plan;

/* Build a plan for `count` items: validates every item, lays out the
 * workspace (returned in *ws_bytes) and the per-stage task tables (transform
 * tiles, Jacobi (slice, block-pair) tasks, per-tensor selection, per-slice
 * packing, reconstruction tiles), which live in the caller's workspace: the
 * plan owns only host data (a pinned host copy of the tables) and graph
 * objects, never device memory.  in_dtype: F32 or F64 input; dtype: F64 or F32 Jacobi / factor /
 * output type; ttm_compute as in tsvdm_transform; block: the Jacobi block
 * width (16 or 32) of items whose own block is 0; block 0 leaves those
 * items at the default (32 when the largest min(m, p) of the batch is at
 * least 256, else 16).  Items of different widths run as two launches per
 * round step.  max_sweeps 0 = 40.  Host errors return before anything is
 * launched.
 * In an F32 plan, items with min(m, p) <= TSVDM_GRAM_MAX_R take the Gram
 * form of tsvdm_slice_svd_gram / tsvdm_pack_gram, every other item the
 * block-rotation form of tsvdm_slice_svd / tsvdm_pack (F64 plans: the
 * rotation form only).  The Gram form's Jacobi is TSVDM_GRAM_LDS when every
 * item of the plan has min(m, p) <= TSVDM_GRAM_LDS_MAX_R, else
 * TSVDM_GRAM_ROUNDS.  Each item's results equal those calls' bits at the
 * item's block width and that placement. */
int tsvdm_batch_plan_create(const tsvdm_batch_item* items, int32_t count, int in_dtype,
                            int dtype, int ttm_compute, int block, int max_sweeps,
                            tsvdm_batch_plan* plan, size_t* ws_bytes);

/* Run the whole batch on `stream`: one launch per stage covers every tensor
 * (the Jacobi stage launches once per step of a global round counter; each
 * slice follows its own tournament).  host_poll = 1 reads a device counter
 * every 4 rounds, one reading behind the queued work, and stops when all
 * slices converged; host_poll = 0 runs the fixed number of steps (kernels
 * of converged slices return at once).  Results are the same bits either
 * way.
 * Every run first copies the plan's task tables (pinned host memory) into
 * the workspace on `stream`, so the workspace need not be preserved between
 * runs; the first run with a new workspace address rebuilds the tables
 * (synchronising the device once, since tables embed workspace addresses).
 * use_graph = 1 captures the run (host_poll forced to 0) into a hipGraph on
 * the first call for this (workspace, stream) and replays it afterwards
 * (the table copy is a copy node of the graph).
 * status (device int32[1]): TSVDM_OK or the first device-side condition. */
int tsvdm_batch_run(tsvdm_batch_plan plan, void* ws, size_t ws_bytes, int host_poll,
                    int use_graph, int32_t* status, void* stream);

/* Release the plan, its pinned host tables and any captured graph. */
int tsvdm_batch_plan_destroy(tsvdm_batch_plan plan);

/* --------------------------------------------------------------------- */
/* kernel statistics (for roofline reporting)                            */
/* --------------------------------------------------------------------- */

/* With statistics on, tsvdm_slice_svd records HIP events on its stream
 * around the Jacobi round launches of every sweep, and at the end of the
 * call waits for them and copies the device pair counters to the host (one
 * extra synchronisation per call).  Totals accumulate process-wide until
 * tsvdm_stats_reset:
 *   launches    Jacobi round kernels launched,
 *   ms          summed event time over those launches (includes the small
 *               gaps between back-to-back launches),
 *   pairs_gram  block pairs that only formed their Gram matrix (converged),
 *   pairs_rot   block pairs that also rotated their vectors (pairs skipped
 *               as unchanged since they last converged count in neither),
 *   pair_width  2b of the last call (the rows of each pair's Gram matrix;
 *               0 after a batch that mixed both widths),
 *   flops       algorithmic flops of those pairs over their w valid vectors:
 *               2 w^2 L (Gram) + 2 w^2 (L + r) (rotation, when rotating),
 *   bytes       algorithmic bytes: w L e (Gram read) + 2 w (L + r) e
 *               (rotation read and write), e = element size.
 * Any pointer may be NULL.  Thread-safe; host only. */
int tsvdm_stats_enable(int on);
int tsvdm_stats_reset(void);
int tsvdm_stats_get(int64_t* launches, double* ms, int64_t* pairs_gram,
                    int64_t* pairs_rot, int32_t* pair_width, double* flops, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* TSVDM_H */

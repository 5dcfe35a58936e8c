// Host-side launchers implemented in the .hip translation units.
#pragma once

#include "common.h"

namespace tsvdm {

// ---- batch descriptors (device-resident tables built by the batch plan)
struct TtmProblem {       // Y = X x_3 (scale * op(M)) for one tensor
    const void* X;
    void* Y;
    const double* M;
    void* Tt;             // n*n staging of scale*op(M) in the compute type
    int64_t R;            // m*p
    int n;
    int pad;
    double scale;
};

struct BatchSlice {       // one frontal slice for the batched Jacobi
    void* A;              // slice base (m*p elements)
    void* W;              // r*r rotation accumulator, or null (none kept)
    double* s2;           // r squared singular values
    SliceGeom g;
    int nbe;              // block count padded to even
    int vec_a, vec_w;
    int tensor;
    double tol;           // convergence threshold on |cos|
    int32_t* track;       // nbe^2 pair records (changed blocks, orthogonal pairs)
};

struct PackSlice {        // one slice for batched packing and reconstruction
    const void* A;        // orthogonalised vectors (Jacobi output)
    const void* W;        // rotation accumulator
    const double* s2;     // r squared singular values
    SliceGeom g;
    const int32_t* rho;   // &rho[i] of its tensor
    const int64_t* off;   // &offsets[i] of its tensor
    void* U_pk;           // tensor-level packed outputs
    void* G_pk;
    void* S_pk;
    int64_t capacity;
    void* C;              // reconstruction target slice (m*p)
    int32_t* status;
};

// Gram form (FP32): FP64 Gram, shifted Cholesky factor, one-sided Jacobi on
// the factor.  min(m, p) <= GRAM_MAX_R; the Jacobi runs in LDS (one
// workgroup per slice) for r <= GRAM_LDS_MAX_R, else in the block rounds.
constexpr int GRAM_MAX_R = TSVDM_GRAM_MAX_R;
constexpr int GRAM_LDS_MAX_R = TSVDM_GRAM_LDS_MAX_R;
constexpr int GRAM_LDS_CLASSES = 4;    // in-LDS size classes (r <= 32, 64, 96, 128)
constexpr int GRAM_CHOL_CLASSES = 4;   // Cholesky size classes (r <= 128, 256, 512, 1024)
struct GramSlice {        // one slice of a batch on the Gram form
    const float* A;       // A-hat slice (m x p), read only
    float* B;             // r x r factor, then its orthogonalised columns
    double* G;            // r x r FP64 Gram matrix (workspace; overwritten by the Cholesky)
    double* Lw;           // r x r FP64 workspace of the Cholesky
    double* s2;           // r squared singular values
    double* shift;        // the Cholesky shift of the slice
    int32_t* flag;        // in-LDS Jacobi: 0 converged, 1 sweep limit, 2 NaN / Inf
    int32_t* perm;        // r: descending order of s2
    SliceGeom g;
    double tol;           // convergence threshold on |cos|
};
// G and the Cholesky factor of every Gram slice; lists: Gram slice indices
// grouped by Cholesky size class (host offsets and counts)
int run_gram_prep_batch(const GramSlice* gs, int64_t ngram, const int2* gram_tasks, int64_t ntasks,
                        const int* lists, const int64_t* class_off, const int64_t* class_cnt,
                        hipStream_t st);
// s2 <- max(s2 - shift, 0) for n Gram slices whose Jacobi ran in the rounds
int run_gram_unshift_batch(const GramSlice* gs, int64_t n, hipStream_t st);
// in-LDS Jacobi of the listed slices (grouped by in-LDS size class, with the
// largest r per class); status from the flags of gs_lds[0, n_lds)
int run_gram_lds_batch(const GramSlice* gs, const int* lists, const int64_t* class_off,
                       const int64_t* class_cnt, const int* class_maxr, int max_sweeps,
                       const GramSlice* gs_lds, int64_t n_lds, int32_t* status, hipStream_t st);
int run_gram_pack_batch(const GramSlice* gs, const PackSlice* ps, int64_t ngram, const int4* ftasks,
                        int64_t nft, hipStream_t st);
int gram_lds_class(int64_t r);          // in-LDS size class of r (0..3)
int gram_chol_class(int64_t r);         // Cholesky size class of r (0..3)
int gram_lds_prepare();                 // allow the dynamic LDS of every class (host, not under capture)
double gram_tol(int64_t r);             // default convergence threshold of the Gram form

int run_pack_batch(int dt, const PackSlice* ps, int64_t nslices, hipStream_t st);
int run_lowrank_batch(int dt, const PackSlice* ps, const int4* tasks, int64_t ntasks,
                      hipStream_t st);

struct SelTensor {        // one tensor's rank selection
    const double* s2;     // r*n squared singular values (slice-major)
    int32_t* rho;
    int64_t* offsets;     // n+1
    double* stats;        // 4 or NULL
    unsigned long long* keys;  // np2 scratch (t-SVDM-II)
    int64_t r, n, np2;
    int mode;             // 1: fixed rank k, 2: tolerance eps
    int pad;
    int64_t k;
    double eps;
};
int run_select_batch(const SelTensor* st_dev, int ntensors, hipStream_t st);
int64_t select_np2(int64_t N);

struct ErrJob {           // sum (A - B)^2 and sum A^2 of one tensor
    const void* A;
    const void* B;
    int64_t count;
    double* out;          // 2 doubles
    double* part;         // 2 * ERR_SEGS doubles
};
constexpr int ERR_SEGS = 64;
int run_error_batch(int adt, int bdt, const ErrJob* jobs, int njobs, hipStream_t st);

size_t jacobi_batch_ctl_bytes(int64_t nslices, int max_steps);
// tasks sorted by pair width: group[0] tasks of width 32, then group[1] of 64
int run_jacobi_batch(int dt, const BatchSlice* sl, int64_t nslices, const int2* tasks,
                     const int64_t* group, int max_steps, int host_poll, void* ctl_ws,
                     int32_t* status, hipStream_t st);

// ---- transform (ttm.hip)
size_t ttm_workspace_bytes(int64_t n);
// tile: 1 = 64 rows x 64 slices, 2 = 128 x 32, 3 = 256 x 16, 4 = 128 x 64,
// 5 = 256 x 32, 6 = 128 x 128, 7 = 256 x 64, 8 = 64 x 64 in 2 x 2 waves,
// 0 = by n and compute type
constexpr int TTM_SHAPES = 8;
int ttm_resolve_tile(int tile, int64_t n, int compute);
void ttm_tile_counts(int shape, int64_t R, int64_t n, int64_t* n_rt, int* n_ct);
// tasks sorted by tile shape; group[s] = task count of shape s + 1 (TTM_SHAPES entries)
int run_ttm_batch(const TtmProblem* probs, int nprob, const int4* tasks, const int64_t* group,
                  int xdt, int ydt, int compute, int transpose, hipStream_t st);
int run_ttm(const void* X, int xdt, void* Y, int ydt, int64_t m, int64_t p, int64_t n,
            const double* M, int transpose, double scale, int compute, int tile, void* ws,
            hipStream_t st);
// Fast orthonormal DCT-II (inverse: its transpose) along the middle index
// of R x n x P (column-major); n a power of two in [2, 1024]; compute F32 or
// F64 (the FFT arithmetic); inputs / outputs F32 or F64.
int run_dct_mode(const void* X, int xdt, void* Y, int ydt, int64_t R, int64_t n, int64_t P,
                 int inverse, int compute, hipStream_t st);
// P consecutive blocks of R x n elements, each Y_b = X_b x_last (scale * op(M))
int run_ttm_mode(const void* X, int xdt, void* Y, int ydt, int64_t R, int64_t n, int64_t P,
                 const double* M, int transpose, double scale, int compute, int tile, void* ws,
                 hipStream_t st);

// ---- slice SVD (jacobi.hip)
struct JacobiCtl {
    unsigned long long maxcos_bits;  // max |cos| seen in the current sweep (FP64 bits)
    int done;                        // 1 once a sweep saw max |cos| <= tol
    int sweeps;                      // sweeps completed
    int nonfinite;                   // a NaN/Inf was met
    int pad;
};

struct JacobiOpts {
    int block;        // 2b, the pair width (32 or 64)
    int max_sweeps;
    double tol;
    int host_poll;
    // device int32[n] or null: slices with run[i] == 0 are left untouched
    // (their A, W and s2 keep whatever they hold)
    const int32_t* run = nullptr;
    // 1: W already holds the slices' starting rotation (not reset to I)
    int w_given = 0;
};

size_t jacobi_workspace_bytes(int64_t r, int64_t n);   // r = min(m, p)
// Gram form of the FP32 slice SVDs (precond.hip)
size_t gram_svd_workspace_bytes(int64_t m, int64_t p, int64_t n);
// jacobi: TSVDM_GRAM_AUTO / ROUNDS / LDS (checked by the caller)
int run_gram_svd(const float* A_hat, int64_t m, int64_t p, int64_t n, float* B, double* s2,
                 double* shift, int32_t* status, const JacobiOpts& o, int jacobi, void* ws,
                 hipStream_t st);
// Preconditioned rotation form: the Gram form's vectors rotate the slice
// (X = W^T A or A W) and the rotation form finishes on X from W
size_t precond_svd_workspace_bytes(int64_t m, int64_t p, int64_t n, int dt);
int run_precond_svd(const void* A_hat, int dt, int64_t m, int64_t p, int64_t n, void* X, void* W,
                    double* s2, int32_t* status, const JacobiOpts& o, void* ws, hipStream_t st);
int run_gram_pack(const float* A_hat, const float* B, const double* s2, const double* shift,
                  int64_t m, int64_t p, int64_t n, const int32_t* rho, const int64_t* offsets,
                  int64_t capacity, float* U_pk, float* G_pk, float* S_pk, int32_t* status,
                  void* ws, hipStream_t st);
int run_pack_sort_f32(const double* s2, int64_t r, int64_t n, const int32_t* rho,
                      const int64_t* offsets, int64_t capacity, int32_t* perm, float* S_pk,
                      int32_t* status, hipStream_t st);
bool stats_enabled();
void stats_add_launch(int64_t launches, double ms);
void stats_set(bool on);
void stats_reset();
void stats_get(int64_t* launches, double* ms, int64_t* pairs_gram, int64_t* pairs_rot,
               int32_t* width, double* flops, double* bytes);
int run_jacobi(void* A, int dt, int64_t m, int64_t p, int64_t n, void* W, double* s2,
               int32_t* status, const JacobiOpts& o, void* ws, hipStream_t st);
JacobiOpts jacobi_default_opts(int64_t m, int64_t p, int dt);

// ---- certified rank selection (certify.hip)
int run_slice_energy(const void* A, int dt, int64_t m, int64_t p, int64_t n, double* E,
                     hipStream_t st);
int run_lump_s2(const double* E, const int32_t* computed, double* s2, int64_t r, int64_t n,
                hipStream_t st);
int run_certify(const double* E, const double* stats, int32_t* computed, int32_t* run_next,
                int64_t n, int force, int32_t* certified, hipStream_t st);

// ---- selection (select.hip)
size_t select_workspace_bytes(int64_t r, int64_t n);
int64_t static_select_max_keys();
int run_truncate_tol_static(const double* s2, int64_t r, int64_t n, double eps, int32_t* rho,
                            int64_t* offsets, double* stats, hipStream_t st);
int run_truncate_tol(const double* s2, int64_t r, int64_t n, double eps, int32_t* rho,
                     int64_t* offsets, double* stats, void* ws, hipStream_t st);
int run_truncate_rank(int64_t k, int64_t r, int64_t n, int32_t* rho, int64_t* offsets,
                      hipStream_t st);

// ---- packing and reconstruction (pack.hip)
size_t pack_workspace_bytes(int64_t m, int64_t p, int64_t n);
int run_pack(const void* A, const void* W, const double* s2, int dt, int64_t m, int64_t p,
             int64_t n, const int32_t* rho, const int64_t* offsets, int64_t capacity,
             void* U_pk, void* G_pk, void* S_pk, int32_t* status, void* ws, hipStream_t st);
int run_lowrank_gemm(const void* U_pk, const void* G_pk, int dt, int64_t m, int64_t p,
                     int64_t n, const int32_t* rho, const int64_t* offsets, int64_t capacity,
                     void* C, hipStream_t st);
int run_pack_from(const void* A, const void* W, const double* s2, int dt, int64_t m, int64_t p,
                  int64_t n, const int32_t* rho, const int64_t* offsets, int64_t capacity,
                  int first, void* U_pk, void* G_pk, void* S_pk, int32_t* status, void* ws,
                  hipStream_t st);

// ---- reductions (reduce.hip)
size_t error_workspace_bytes(int64_t count);
int run_error(const void* A, int adt, const void* B, int bdt, int64_t count, double* out,
              void* ws, hipStream_t st);

// ---- adjoint (backward.hip)
size_t backward_workspace_bytes(int64_t m, int64_t p, int64_t n, int dt);
int run_backward(const void* A, int dt, int64_t m, int64_t p, int64_t n, const double* M,
                 int64_t k, double g, void* dA, double* dM, double* loss, int32_t* status,
                 void* ws, hipStream_t st);

}  // namespace tsvdm

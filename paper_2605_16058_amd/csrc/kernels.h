// Host-side launchers implemented in the .hip translation units.
#pragma once

#include "common.h"

namespace tsvdm {

// ---- transform (ttm.hip)
size_t ttm_workspace_bytes(int64_t n);
int run_ttm(const void* X, int xdt, void* Y, int ydt, int64_t m, int64_t p, int64_t n,
            const double* M, int transpose, double scale, int compute, void* ws,
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
};

size_t jacobi_workspace_bytes(int64_t n);
bool stats_enabled();
void stats_set(bool on);
void stats_reset();
void stats_add(int64_t launches, double ms, int64_t pairs_gram, int64_t pairs_rot, int width);
void stats_get(int64_t* launches, double* ms, int64_t* pairs_gram, int64_t* pairs_rot,
               int32_t* width);
int run_jacobi(void* A, int dt, int64_t m, int64_t p, int64_t n, void* W, double* s2,
               int32_t* status, const JacobiOpts& o, void* ws, hipStream_t st);
JacobiOpts jacobi_default_opts(int64_t m, int64_t p, int dt);

// ---- selection (select.hip)
size_t select_workspace_bytes(int64_t r, int64_t n);
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

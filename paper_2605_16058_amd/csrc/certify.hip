// Certified rank selection for t-SVDM-II: slices whose whole energy is
// provably below the threshold need no SVD.
//
// Algorithm 2 keeps, in every slice, the squared singular values above tau,
// where tau is the largest of the smallest values whose running sum stays
// below eps^2 times the total; Section 4.1 observes that t-SVDM-II discards
// many slices entirely.  The selection needs only the values above tau and,
// for the rest, their sum: a slice i whose SVD is not computed stands in the
// sorted list as one value, its energy E_i = ||A_i||_F^2 (the sum of its
// squared singular values, each of which is <= E_i).  If afterwards every
// such stand-in lies strictly below the tau found, then every value of
// those slices lies below it too, all of them come before tau in the sorted
// order with the right total, and tau and every rank are exactly those of
// the full selection (those slices get rank 0).  Otherwise the slices whose
// stand-in reached tau get their SVD and the selection is repeated.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "common.h"
#include "kernels.h"

namespace tsvdm {
namespace {

constexpr int ETHREADS = 256;

// E[i] = sum of the squares of slice i in FP64: one workgroup per slice,
// every thread a fixed strided share, then a fixed reduction tree, so the
// result does not depend on timing.
template <class T>
__global__ __launch_bounds__(ETHREADS) void slice_energy(const T* __restrict__ A, int64_t mp,
                                                         double* __restrict__ E) {
    __shared__ double part[ETHREADS];
    const T* x = A + (int64_t)blockIdx.x * mp;
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < mp; e += ETHREADS) {
        const double v = (double)x[e];
        acc = fma(v, v, acc);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = ETHREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) E[blockIdx.x] = part[0];
}

// Stand-ins of the slices without an SVD: s2[:, i] = (E_i, 0, ..., 0).
__global__ void lump_s2(const double* __restrict__ E, const int32_t* __restrict__ computed,
                        double* __restrict__ s2, int64_t r, int64_t n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= r * n) return;
    const int64_t i = idx / r, j = idx % r;
    if (computed[i]) return;
    s2[idx] = (j == 0) ? E[i] : 0.0;
}

// certified = every stand-in finite and strictly below tau (stats[0]);
// run_next[i] = 1 for the stand-ins that are not (all of them with force),
// which join `computed`.
__global__ void certify(const double* __restrict__ E, const double* __restrict__ stats,
                        int32_t* __restrict__ computed, int32_t* __restrict__ run_next, int64_t n,
                        int force, int32_t* __restrict__ certified) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const double tau = stats[0];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        int nx = 0;
        if (!computed[i]) {
            const double e = E[i];
            if (force || !(e < tau)) {   // also true for NaN
                nx = 1;
                computed[i] = 1;
                atomicOr(&bad, 1);
            }
        }
        run_next[i] = nx;
    }
    __syncthreads();
    if (threadIdx.x == 0) *certified = (bad || force) ? 0 : 1;
}

}  // namespace

int run_slice_energy(const void* A, int dt, int64_t m, int64_t p, int64_t n, double* E,
                     hipStream_t st) {
    if (n == 0) return TSVDM_OK;
    const int64_t mp = m * p;
    for (int64_t s0 = 0; s0 < n; s0 += ((int64_t)1 << 30)) {
        const int64_t cnt = (n - s0) < ((int64_t)1 << 30) ? (n - s0) : ((int64_t)1 << 30);
        if (dt == TSVDM_F64)
            slice_energy<double><<<(unsigned)cnt, ETHREADS, 0, st>>>(
                static_cast<const double*>(A) + s0 * mp, mp, E + s0);
        else
            slice_energy<float><<<(unsigned)cnt, ETHREADS, 0, st>>>(
                static_cast<const float*>(A) + s0 * mp, mp, E + s0);
        TSVDM_LAUNCH_CHECK();
    }
    return TSVDM_OK;
}

int run_lump_s2(const double* E, const int32_t* computed, double* s2, int64_t r, int64_t n,
                hipStream_t st) {
    const int64_t total = r * n;
    if (total == 0) return TSVDM_OK;
    const int64_t blocks = (total + 255) / 256;
    TSVDM_REQUIRE(blocks < ((int64_t)1 << 31), TSVDM_E_SHAPE, "too many values");
    lump_s2<<<(unsigned)blocks, 256, 0, st>>>(E, computed, s2, r, n);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

int run_certify(const double* E, const double* stats, int32_t* computed, int32_t* run_next,
                int64_t n, int force, int32_t* certified, hipStream_t st) {
    certify<<<1, 1024, 0, st>>>(E, stats, computed, run_next, n, force, certified);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

}  // namespace tsvdm

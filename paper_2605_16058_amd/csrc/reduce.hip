// Error report: sum (A - B)^2 and sum A^2 in FP64 with a fixed reduction
// order, so repeated runs give bit-identical results.
#include "common.h"
#include "kernels.h"

namespace tsvdm {

namespace {

constexpr int RBLOCKS = 1024;
constexpr int RTHREADS = 256;

// Thread's share of sum (A - B)^2 and sum A^2 over [i0, end) with stride
// RTHREADS, in FP64.  Eight elements' loads are issued together; the sums
// take the elements in the same order as one at a time.
template <class TA, class TB>
__device__ __forceinline__ void err_range(const TA* __restrict__ A, const TB* __restrict__ B, int64_t i0,
                                          int64_t end, double& d2, double& a2) {
    int64_t i = i0;
    for (; i + 7 * RTHREADS < end; i += 8 * RTHREADS) {
        TA av[8];
        TB bv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            av[q] = A[i + q * RTHREADS];
            bv[q] = B[i + q * RTHREADS];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const double a = (double)av[q];
            const double d = a - (double)bv[q];
            d2 = fma(d, d, d2);
            a2 = fma(a, a, a2);
        }
    }
    for (; i < end; i += RTHREADS) {
        const double a = (double)A[i];
        const double d = a - (double)B[i];
        d2 = fma(d, d, d2);
        a2 = fma(a, a, a2);
    }
}

template <class TA, class TB>
__global__ __launch_bounds__(RTHREADS) void err_partial(const TA* __restrict__ A,
                                                        const TB* __restrict__ B, int64_t count,
                                                        double* __restrict__ part) {
    // block b owns the contiguous range [b*seg, (b+1)*seg)
    const int64_t seg = (count + RBLOCKS - 1) / RBLOCKS;
    const int64_t b0 = (int64_t)blockIdx.x * seg;
    const int64_t b1 = (b0 + seg < count) ? b0 + seg : count;
    double d2 = 0.0, a2 = 0.0;
    err_range(A, B, b0 + threadIdx.x, b1, d2, a2);
    for (int off = 32; off > 0; off >>= 1) {
        d2 += __shfl_xor(d2, off);
        a2 += __shfl_xor(a2, off);
    }
    __shared__ double sd[RTHREADS / 64], sa[RTHREADS / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sd[w] = d2; sa[w] = a2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int i = 0; i < RTHREADS / 64; ++i) { x += sd[i]; y += sa[i]; }
        part[2 * blockIdx.x] = x;
        part[2 * blockIdx.x + 1] = y;
    }
}

__global__ void err_final(const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double x = 0.0, y = 0.0;
    for (int i = 0; i < RBLOCKS; ++i) { x += part[2 * i]; y += part[2 * i + 1]; }
    out[0] = x;
    out[1] = y;
}

template <class TA, class TB>
void launch_err(const void* A, const void* B, int64_t count, double* part, hipStream_t st) {
    err_partial<TA, TB><<<RBLOCKS, RTHREADS, 0, st>>>(static_cast<const TA*>(A),
                                                      static_cast<const TB*>(B), count, part);
}

}  // namespace

size_t error_workspace_bytes(int64_t) { return align_up(sizeof(double) * 2 * RBLOCKS); }

int run_error(const void* A, int adt, const void* B, int bdt, int64_t count, double* out,
              void* ws, hipStream_t st) {
    double* part = static_cast<double*>(ws);
    if (adt == TSVDM_F64 && bdt == TSVDM_F64) launch_err<double, double>(A, B, count, part, st);
    else if (adt == TSVDM_F64 && bdt == TSVDM_F32) launch_err<double, float>(A, B, count, part, st);
    else if (adt == TSVDM_F32 && bdt == TSVDM_F64) launch_err<float, double>(A, B, count, part, st);
    else if (adt == TSVDM_F32 && bdt == TSVDM_F32) launch_err<float, float>(A, B, count, part, st);
    else {
        set_error("error report supports F64 and F32 only");
        return TSVDM_E_UNSUPPORTED;
    }
    TSVDM_LAUNCH_CHECK();
    err_final<<<1, 64, 0, st>>>(part, out);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

namespace {

// task = (job, segment): segment s of job j covers [s*seg, (s+1)*seg)
template <class TA, class TB>
__global__ __launch_bounds__(RTHREADS) void err_partial_batch(const ErrJob* __restrict__ jobs) {
    const ErrJob jb = jobs[blockIdx.y];
    const TA* A = static_cast<const TA*>(jb.A);
    const TB* B = static_cast<const TB*>(jb.B);
    const int64_t seg = (jb.count + ERR_SEGS - 1) / ERR_SEGS;
    const int64_t b0 = (int64_t)blockIdx.x * seg;
    const int64_t b1 = (b0 + seg < jb.count) ? b0 + seg : jb.count;
    double d2 = 0.0, a2 = 0.0;
    err_range(A, B, b0 + threadIdx.x, b1, d2, a2);
    for (int off = 32; off > 0; off >>= 1) {
        d2 += __shfl_xor(d2, off);
        a2 += __shfl_xor(a2, off);
    }
    __shared__ double sd[RTHREADS / 64], sa[RTHREADS / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { sd[w] = d2; sa[w] = a2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0, y = 0.0;
        for (int i = 0; i < RTHREADS / 64; ++i) { x += sd[i]; y += sa[i]; }
        jb.part[2 * blockIdx.x] = x;
        jb.part[2 * blockIdx.x + 1] = y;
    }
}

__global__ void err_final_batch(const ErrJob* __restrict__ jobs, int njobs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= njobs) return;
    const ErrJob jb = jobs[j];
    double x = 0.0, y = 0.0;
    for (int i = 0; i < ERR_SEGS; ++i) { x += jb.part[2 * i]; y += jb.part[2 * i + 1]; }
    jb.out[0] = x;
    jb.out[1] = y;
}

}  // namespace

int run_error_batch(int adt, int bdt, const ErrJob* jobs, int njobs, hipStream_t st) {
    dim3 grid(ERR_SEGS, (unsigned)njobs);
    if (adt == TSVDM_F64 && bdt == TSVDM_F64) err_partial_batch<double, double><<<grid, RTHREADS, 0, st>>>(jobs);
    else if (adt == TSVDM_F64) err_partial_batch<double, float><<<grid, RTHREADS, 0, st>>>(jobs);
    else if (bdt == TSVDM_F64) err_partial_batch<float, double><<<grid, RTHREADS, 0, st>>>(jobs);
    else err_partial_batch<float, float><<<grid, RTHREADS, 0, st>>>(jobs);
    TSVDM_LAUNCH_CHECK();
    err_final_batch<<<(unsigned)((njobs + 63) / 64), 64, 0, st>>>(jobs, njobs);
    TSVDM_LAUNCH_CHECK();
    return TSVDM_OK;
}

}  // namespace tsvdm

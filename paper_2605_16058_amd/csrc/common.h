// Internal helpers shared by the HIP translation units of libtsvdm.
// Not part of the public ABI (include/tsvdm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "../../include/tsvdm.h"

namespace tsvdm {

// ---------------------------------------------------------------- errors

// Thread-local message behind tsvdm_last_error().
void set_error(const std::string& msg);
void clear_error();

#define TSVDM_HIP_CHECK(expr)                                                    \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) {                                                  \
            ::tsvdm::set_error(std::string("HIP error in " #expr ": ") +         \
                               hipGetErrorString(e_));                           \
            return TSVDM_E_HIP;                                                  \
        }                                                                        \
    } while (0)

#define TSVDM_REQUIRE(cond, code, msg)                                           \
    do {                                                                         \
        if (!(cond)) {                                                           \
            ::tsvdm::set_error(msg);                                             \
            return (code);                                                       \
        }                                                                        \
    } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Check the last kernel launch; used right after <<<>>> launches.
#define TSVDM_LAUNCH_CHECK() TSVDM_HIP_CHECK(hipGetLastError())

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// A bump allocator over the caller's workspace: carve() returns aligned
// sub-buffers; total() is the size needed (for the *_workspace_size queries).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <class T>
    T* carve(size_t count) {
        off = align_up(off);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t total() const { return align_up(off); }
};

// ------------------------------------------------------------- MFMA types

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// 16x16 MFMA tiles on a 64-lane wavefront (CDNA3/CDNA4 layout):
//   A (16 x K) : lane L holds row  L % 16, k-group L / 16
//   B (K x 16) : lane L holds col  L % 16, k-group L / 16
//   D (16 x 16): lane L holds rows 4*(L/16) + {0,1,2,3} of column L % 16
// For the 16x16x4 shapes a k-group is one k; for 16x16x32 bf16 it is eight
// consecutive k.  A and B always use the same k mapping, so any permutation
// of k inside a group is harmless.
// The D row of element v differs by type (measured on gfx950):
//   f32 / bf16 (FP32 accumulators): row 4*(L/16) + v
//   f64:                            row (L/16) + 4*v
template <class T> __device__ __forceinline__ int mfma_row(int lg, int v);
template <> __device__ __forceinline__ int mfma_row<float>(int lg, int v) { return 4 * lg + v; }
template <> __device__ __forceinline__ int mfma_row<double>(int lg, int v) { return lg + 4 * v; }
__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <class T> struct Acc;
template <> struct Acc<double> { typedef v4d type; };
template <> struct Acc<float> { typedef v4f type; };

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) { return mfma_f64(a, b, c); }
__device__ __forceinline__ v4f mfma(float a, float b, v4f c) { return mfma_f32(a, b, c); }

template <class V>
__device__ __forceinline__ V zero4() {
    V z;
    z[0] = 0; z[1] = 0; z[2] = 0; z[3] = 0;
    return z;
}

// ------------------------------------------------------------ load / store

template <class T> __device__ __forceinline__ T ldg_as(const void* p, int64_t i, int dt);

template <>
__device__ __forceinline__ double ldg_as<double>(const void* p, int64_t i, int dt) {
    return dt == TSVDM_F64 ? static_cast<const double*>(p)[i]
                           : static_cast<double>(static_cast<const float*>(p)[i]);
}
template <>
__device__ __forceinline__ float ldg_as<float>(const void* p, int64_t i, int dt) {
    return dt == TSVDM_F64 ? static_cast<float>(static_cast<const double*>(p)[i])
                           : static_cast<const float*>(p)[i];
}

__device__ __forceinline__ void stg_as(void* p, int64_t i, int dt, double v) {
    if (dt == TSVDM_F64) static_cast<double*>(p)[i] = v;
    else static_cast<float*>(p)[i] = static_cast<float>(v);
}

// round-to-nearest-even FP32 -> BF16
__device__ __forceinline__ __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }

// ------------------------------------------------------ double-double sums

struct dd { double hi, lo; };

__device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double err = (a - (s - bb)) + (b - bb);
    return {s, err};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_add_d(dd a, double b) {
    dd s = two_sum(a.hi, b);
    s.lo += a.lo;
    return two_sum(s.hi, s.lo);
}
__device__ __forceinline__ double dd_round(dd a) { return a.hi + a.lo; }

// Slice geometry: r = min(m, p) Jacobi vectors of length L = max(m, p).
// Element t of vector j of a slice lives at j*vs + t*es.
// `rows` says which orientation holds (it cannot be inferred from es: for
// m = 1 the rows have element stride 1).
struct SliceGeom {
    int64_t m, p, r, L, vs, es;
    int rows;
};
__host__ __device__ inline SliceGeom slice_geom(int64_t m, int64_t p) {
    SliceGeom g;
    g.m = m; g.p = p;
    if (m >= p) { g.r = p; g.L = m; g.vs = m; g.es = 1; g.rows = 0; }   // columns
    else        { g.r = m; g.L = p; g.vs = 1; g.es = m; g.rows = 1; }   // rows
    return g;
}

}  // namespace tsvdm

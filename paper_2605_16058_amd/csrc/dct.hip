// Fast orthonormal DCT-II along one mode of a column-major tensor: the
// operator form of the mode product for M = C, the orthonormal DCT-II.
// Section 2.2 (choice of M) notes that the DCT applies in O(n log n);
// Section 3.1 runs every transform as a dense TTM, and Section 5 leaves
// operator transforms for the TTM stage as future work.
//
// Forward, Y = X x_k C:  Y_q = s_q sum_j x_j cos(pi q (2j + 1) / (2n)),
//   s_0 = sqrt(1/n), s_q = sqrt(2/n).  With v_j = x_{2j}, v_{n-1-j} = x_{2j+1}
//   (j < n/2) and V = DFT_n(v):  Y_q = s_q Re(exp(-i pi q / (2n)) V_q).
// Inverse, Y = X x_k C^T (C is orthogonal): with t_q = x_q / s_q,
//   V_q = exp(i pi q / (2n)) (t_q - i t_{n-q})  (t_n = 0),  v = IDFT_n(V)
//   (real), then y_{2j} = v_j, y_{2j+1} = v_{n-1-j}.
// DFT_n runs as a four-step FFT, n = n1 n2: n2 length-n1 DFTs in registers
// (one per thread), a twiddle multiply, a transpose through LDS and n1
// length-n2 DFTs in registers.  The inverse DFT is conj(DFT(conj(V))) / n.
// Work per element ~ 5 log2(n) flops against the dense product's 2n; one
// read and one write of every element, so the kernel is HBM bound.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"
#include "kernels.h"

namespace tsvdm {
namespace {

template <class CT>
struct Cx {
    CT re, im;
};

template <class CT>
__device__ __forceinline__ Cx<CT> cmul(Cx<CT> a, Cx<CT> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }
constexpr int bitrev(int x, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

// Geometry for n = 2^L: n1 = 2^ceil(L/2) threads per tube, n2 = n / n1; TB
// tubes per workgroup (at most 512 threads; 32 tubes make every access of
// a wave 128 contiguous bytes per index), halved until the padded tile and
// the three twiddle tables (5n values) fit in 80 KB of LDS.
template <class CT, int L>
struct DctCfg {
    static constexpr int n = 1 << L;
    static constexpr int n1 = 1 << ((L + 1) / 2);
    static constexpr int n2 = n / n1;
    static constexpr size_t lds(int tb) { return ((size_t)tb * (n + 1) * 2 + (size_t)5 * n) * sizeof(CT); }
    static constexpr int fit(int tb) { return (tb > 1 && lds(tb) > 81920) ? fit(tb / 2) : tb; }
    static_assert(lds(1) <= 81920, "transform length too large for the LDS");
    static constexpr int TB = fit(512 / n1 < 32 ? 512 / n1 : 32);
    static constexpr int THREADS = TB * n1;
};

// In-register DFT of length N (power of two): radix-2 decimation in time on
// inputs stored in bit-reversed order; w[m] = exp(-2 pi i m / N), m < N/2.
template <class CT, int N>
__device__ __forceinline__ void dft_regs(Cx<CT> (&x)[N], const Cx<CT> (&w)[N / 2 > 0 ? N / 2 : 1]) {
#pragma unroll
    for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
        for (int i = 0; i < N; i += len) {
#pragma unroll
            for (int j = 0; j < len / 2; ++j) {
                const Cx<CT> u = x[i + j];
                const Cx<CT> v = (j == 0) ? x[i + j + len / 2] : cmul(x[i + j + len / 2], w[j * (N / len)]);
                x[i + j] = {u.re + v.re, u.im + v.im};
                x[i + j + len / 2] = {u.re - v.re, u.im - v.im};
            }
        }
    }
}

// The stages of one workgroup's tube block.  Thread (tube, sub) loads and
// transforms the step-1 inputs q = n2 j1 + sub (sub < n2) of its tube and
// the step-4 outputs q = sub + n1 k2.
template <class IT, class CT, int L, bool INV>
struct DctStages {
    typedef DctCfg<CT, L> C;
    static constexpr int n = C::n, n1 = C::n1, n2 = C::n2;
    // raw inputs per thread: x at the reordered positions (forward), or x_q
    // and x_{n-q} (inverse; for q = 0 the second is x_0 and is not used)
    static constexpr int NIN = INV ? 2 * n1 : n1;

    __device__ static __forceinline__ void load(IT (&raw)[NIN], const IT* __restrict__ in, int64_t R, int sub) {
#pragma unroll
        for (int j1 = 0; j1 < n1; ++j1) {
            const int q = n2 * j1 + sub;
            if (!INV) {
                const int src = (q < n / 2) ? 2 * q : 2 * (n - 1 - q) + 1;
                raw[j1] = in[(int64_t)src * R];
            } else {
                raw[j1] = in[(int64_t)q * R];
                raw[n1 + j1] = in[(int64_t)((n - q) & (n - 1)) * R];
            }
        }
    }

    // step 1a: the inputs v[n2 j1 + sub] of the thread's length-n1 DFT as
    // complex values, placed in bit-reversed order
    __device__ static __forceinline__ void prep(const IT (&raw)[NIN], int sub, const Cx<CT>* pw,
                                                const CT* isc, Cx<CT> (&x1)[n1]) {
#pragma unroll
        for (int j1 = 0; j1 < n1; ++j1) {
            const int q = n2 * j1 + sub;
            Cx<CT> v;
            if (!INV) {
                v = {(CT)raw[j1], CT(0)};
            } else {
                // conj(V_q) with V_q = pw_q (t_q - i t_{n-q})
                const CT tq = (CT)raw[j1] * isc[q];
                const CT tr = (q == 0) ? CT(0) : (CT)raw[n1 + j1] * isc[n - q];
                const Cx<CT> p = pw[q];
                const Cx<CT> V = {p.re * tq + p.im * tr, p.im * tq - p.re * tr};
                v = {V.re, -V.im};
            }
            x1[bitrev(j1, ilog2(n1))] = v;
        }
    }

    // step 1b: the DFT over j1 in registers, the twiddles, and the write
    // into the LDS row
    __device__ static __forceinline__ void first(Cx<CT> (&x1)[n1], int sub, const Cx<CT>* tw, Cx<CT>* row) {
        Cx<CT> w1[n1 / 2 > 0 ? n1 / 2 : 1];
#pragma unroll
        for (int m = 0; m < n1 / 2; ++m) w1[m] = tw[m * n2];
        dft_regs<CT, n1>(x1, w1);
#pragma unroll
        for (int k1 = 0; k1 < n1; ++k1) {
            const Cx<CT> t = (sub * k1 == 0) ? x1[k1] : cmul(x1[k1], tw[(sub * k1) % n]);
            row[sub * n1 + k1] = t;
        }
    }

    // step 4 (all threads): DFT over j2 of the transposed row; output
    // q = sub + n1 k2, then the DCT post-twiddle (forward) or the
    // reordering (inverse) and the stores
    template <class OT>
    __device__ static __forceinline__ void second(int sub, const Cx<CT>* tw, const Cx<CT>* pw,
                                                  const Cx<CT>* row, bool valid, OT* __restrict__ out,
                                                  int64_t R) {
        Cx<CT> w2[n2 / 2 > 0 ? n2 / 2 : 1];
#pragma unroll
        for (int m = 0; m < n2 / 2; ++m) w2[m] = tw[m * n1];
        Cx<CT> x4[n2];
#pragma unroll
        for (int j2 = 0; j2 < n2; ++j2) x4[bitrev(j2, ilog2(n2))] = row[j2 * n1 + sub];
        dft_regs<CT, n2>(x4, w2);
        if (!valid) return;
#pragma unroll
        for (int k2 = 0; k2 < n2; ++k2) {
            const int q = sub + n1 * k2;
            if (!INV) {
                const Cx<CT> p = pw[q];
                out[(int64_t)q * R] = (OT)(p.re * x4[k2].re - p.im * x4[k2].im);
            } else {
                // v_q = Re(conj(DFT(conj V))_q) / n = Re(DFT(conj V)_q) / n
                const int dst = (q < n / 2) ? 2 * q : 2 * (n - 1 - q) + 1;
                out[(int64_t)dst * R] = (OT)(x4[k2].re * (CT(1) / CT(n)));
            }
        }
    }
};

// Twiddle tables of one workgroup, FP64 sincospi rounded to CT.
template <class CT, int L, bool INV>
__device__ __forceinline__ void dct_tables(Cx<CT>* tw, Cx<CT>* pw, CT* isc) {
    constexpr int n = 1 << L;
    for (int q = threadIdx.x; q < n; q += (int)blockDim.x) {
        double s, c;
        sincospi(-2.0 * q / n, &s, &c);
        tw[q] = {(CT)c, (CT)s};
        const double sq = (q == 0) ? sqrt(1.0 / n) : sqrt(2.0 / n);
        if (!INV) {
            sincospi(-0.5 * q / n, &s, &c);
            pw[q] = {(CT)(sq * c), (CT)(sq * s)};
        } else {
            sincospi(0.5 * q / n, &s, &c);
            pw[q] = {(CT)c, (CT)s};
            isc[q] = (CT)(1.0 / sq);
        }
    }
}

// One tube block (TB tubes from row blockIdx.x TB) per workgroup, tubes
// past R masked.  A thread issues all of its loads together before any
// arithmetic (one branch on the tube's validity, none per element), so
// that their latencies overlap.
template <class IT, class OT, class CT, int L, bool INV>
__global__ __launch_bounds__((DctCfg<CT, L>::THREADS)) void dct_kernel(const IT* __restrict__ X,
                                                                     OT* __restrict__ Y, int64_t R,
                                                                     int64_t b0) {
    typedef DctCfg<CT, L> C;
    typedef DctStages<IT, CT, L, INV> S;
    constexpr int n = C::n, n2 = C::n2, TB = C::TB;
    __shared__ Cx<CT> buf[TB * (n + 1)];
    __shared__ Cx<CT> tw[n];     // exp(-2 pi i q / n)
    __shared__ Cx<CT> pw[n];     // forward: s_q exp(-i pi q / (2n)); inverse: exp(i pi q / (2n))
    __shared__ CT isc[n];        // inverse: 1 / s_q
    dct_tables<CT, L, INV>(tw, pw, isc);
    __syncthreads();

    const int tid = threadIdx.x;
    const int tube = tid % TB, sub = tid / TB;
    const int64_t a = (int64_t)blockIdx.x * TB + tube;
    const bool valid = a < R;
    const int64_t blk = b0 + blockIdx.y;
    Cx<CT>* const row = buf + tube * (n + 1);
    if (sub < n2) {
        IT raw[S::NIN];
#pragma unroll
        for (int i = 0; i < S::NIN; ++i) raw[i] = IT(0);
        if (valid) S::load(raw, X + blk * R * n + a, R, sub);
        Cx<CT> x1[C::n1];
        S::prep(raw, sub, pw, isc, x1);
        S::first(x1, sub, tw, row);
    }
    __syncthreads();
    S::second(sub, tw, pw, row, valid, Y + blk * R * n + a, R);
}

template <class IT, class OT, class CT, int L, bool INV>
void launch_dct(const void* X, void* Y, int64_t R, int64_t P, hipStream_t st) {
    typedef DctCfg<CT, L> C;
    const int64_t gx = (R + C::TB - 1) / C::TB;   // below 2^31: checked by the caller
    for (int64_t b0 = 0; b0 < P; b0 += 65535) {
        const int64_t gy = (P - b0) < 65535 ? (P - b0) : 65535;
        hipLaunchKernelGGL((dct_kernel<IT, OT, CT, L, INV>), dim3((unsigned)gx, (unsigned)gy),
                           dim3(C::THREADS), 0, st, static_cast<const IT*>(X), static_cast<OT*>(Y), R,
                           b0);
    }
}

template <class IT, class OT, class CT, bool INV>
int dct_dispatch(int L, const void* X, void* Y, int64_t R, int64_t P, hipStream_t st) {
    switch (L) {
        case 1: launch_dct<IT, OT, CT, 1, INV>(X, Y, R, P, st); break;
        case 2: launch_dct<IT, OT, CT, 2, INV>(X, Y, R, P, st); break;
        case 3: launch_dct<IT, OT, CT, 3, INV>(X, Y, R, P, st); break;
        case 4: launch_dct<IT, OT, CT, 4, INV>(X, Y, R, P, st); break;
        case 5: launch_dct<IT, OT, CT, 5, INV>(X, Y, R, P, st); break;
        case 6: launch_dct<IT, OT, CT, 6, INV>(X, Y, R, P, st); break;
        case 7: launch_dct<IT, OT, CT, 7, INV>(X, Y, R, P, st); break;
        case 8: launch_dct<IT, OT, CT, 8, INV>(X, Y, R, P, st); break;
        case 9: launch_dct<IT, OT, CT, 9, INV>(X, Y, R, P, st); break;
        case 10: launch_dct<IT, OT, CT, 10, INV>(X, Y, R, P, st); break;
        default: return TSVDM_E_SHAPE;
    }
    return TSVDM_OK;
}

template <class IT, class OT, class CT>
int dct_typed(int L, int inverse, const void* X, void* Y, int64_t R, int64_t P, hipStream_t st) {
    return inverse ? dct_dispatch<IT, OT, CT, true>(L, X, Y, R, P, st)
                   : dct_dispatch<IT, OT, CT, false>(L, X, Y, R, P, st);
}

}  // namespace

int run_dct_mode(const void* X, int xdt, void* Y, int ydt, int64_t R, int64_t n, int64_t P,
                 int inverse, int compute, hipStream_t st) {
    int L = 0;
    while ((int64_t(1) << L) < n) ++L;
    if ((int64_t(1) << L) != n || L < 1 || L > 10) return TSVDM_E_SHAPE;
    if (R == 0 || P == 0) return TSVDM_OK;
    if (R >= ((int64_t)1 << 31)) {   // the grid holds ceil(R / tubes per workgroup) <= R workgroups
        set_error("dct: the rows before the transformed mode must number below 2^31");
        return TSVDM_E_SHAPE;
    }
    int rc;
    if (compute == TSVDM_F32) {
        if (xdt == TSVDM_F32 && ydt == TSVDM_F32) rc = dct_typed<float, float, float>(L, inverse, X, Y, R, P, st);
        else if (xdt == TSVDM_F32 && ydt == TSVDM_F64) rc = dct_typed<float, double, float>(L, inverse, X, Y, R, P, st);
        else if (xdt == TSVDM_F64 && ydt == TSVDM_F32) rc = dct_typed<double, float, float>(L, inverse, X, Y, R, P, st);
        else rc = dct_typed<double, double, float>(L, inverse, X, Y, R, P, st);
    } else {
        if (xdt == TSVDM_F32 && ydt == TSVDM_F32) rc = dct_typed<float, float, double>(L, inverse, X, Y, R, P, st);
        else if (xdt == TSVDM_F32 && ydt == TSVDM_F64) rc = dct_typed<float, double, double>(L, inverse, X, Y, R, P, st);
        else if (xdt == TSVDM_F64 && ydt == TSVDM_F32) rc = dct_typed<double, float, double>(L, inverse, X, Y, R, P, st);
        else rc = dct_typed<double, double, double>(L, inverse, X, Y, R, P, st);
    }
    if (rc != TSVDM_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error(std::string("dct launch: ") + hipGetErrorString(e));
        return TSVDM_E_HIP;
    }
    return TSVDM_OK;
}

}  // namespace tsvdm

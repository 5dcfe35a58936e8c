// FP64 Jacobi rotation angle shared by the slice-SVD kernels.
#ifndef TSVDM_ANGLE_H
#define TSVDM_ANGLE_H

#include "common.h"

namespace tsvdm {

// FP64 reciprocal and reciprocal square root: the hardware estimates
// refined by two Newton steps each (quadratic convergence from about 23
// correct bits), for arguments in [1, 4] where no scaling is needed.
static __device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    return fma(fma(-x, y, 1.0), y, y);
}
static __device__ __forceinline__ double rsq_nr(double x) {
    const double h = 0.5 * x;
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// Rotation (c, s) annihilating apq of the symmetric 2x2 [app apq; apq aqq]
// in FP64 (the classical Jacobi angle, tan 2theta = 2 apq / (aqq - app),
// smaller root): with d = aqq - app and e = 2 apq scaled by max(|d|, |e|),
//   t = sign(d) e / (|d| + sqrt(d^2 + e^2)),  c = 1 / sqrt(1 + t^2),  s = c t,
// so every square root and reciprocal has an argument in [1, 2] and
// c^2 + s^2 = 1 to rounding.  new_p = c p - s q, new_q = s p + c q.
// Identity when invalid or when |apq| <= 1e-18 sqrt(|app aqq|).
static __device__ __forceinline__ void jacobi_angle(double app, double aqq, double apq, bool valid,
                                             double& c, double& s) {
    c = 1.0;
    s = 0.0;
    // the threshold needs no accuracy: unrefined hardware square roots
    const double a = fmax(fabs(app), 1e-300), b = fmax(fabs(aqq), 1e-300);
    const double thr = 1e-18 * (a * __builtin_amdgcn_rsq(a)) * (b * __builtin_amdgcn_rsq(b));
    if (valid && fabs(apq) > thr) {
        const double d = aqq - app, e = 2.0 * apq;
        const double inv = rcp_nr(fmax(fabs(d), fabs(e)));
        const double dn = d * inv, en = e * inv;     // max(|dn|, |en|) = 1
        const double q2 = fma(dn, dn, en * en);      // in [1, 2]
        const double h = q2 * rsq_nr(q2);
        const double t = copysign(1.0, dn) * en * rcp_nr(fabs(dn) + h);
        c = rsq_nr(fma(t, t, 1.0));
        s = c * t;
    }
}

}  // namespace tsvdm

#endif  // TSVDM_ANGLE_H

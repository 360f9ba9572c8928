// Device-side helpers shared by the xTC kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xtc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kPairTile = 128;   // pair-column padding unit (xtc_pair_ld)
constexpr int kGridPad = 128;    // grid-row padding unit of the prepared operands

// Jastrow parameters as kernels see them.  dcoef[k] = (k+1) coef[k], so the
// power-form derivative is a Horner polynomial in t = r/(1+r); entries beyond
// ncoef are zero, so all 16 terms are evaluated (leading zero terms leave the
// Horner value exactly unchanged) without a data-dependent loop.
struct JasDev {
    int32_t kind;    // 0 Pade, 1 power
    int32_t ncoef;
    double b;
    double dcoef[16];
    double d2coef[16];   // (k+2)(k+1) coef[k+1]: u''(t) as a Horner polynomial
    // the same parameters rounded to FP32 (reduced-precision forms; kernel
    // arguments, so they stay in scalar registers)
    float fb;
    float fdcoef[16];
    float fd2coef[16];
};

// 1/sqrt(x) and 1/x in FP64 from the hardware approximations (v_rsq_f64,
// v_rcp_f64) refined by two Newton steps each (each step squares the
// relative error), for x > 0 and finite: a few ulp, against the longer
// correctly rounded sequences the compiler emits for sqrt and division.
__device__ __forceinline__ double rsq_f64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    y = y * fma(-hx, y * y, 1.5);
    y = y * fma(-hx, y * y, 1.5);
    return y;
}
__device__ __forceinline__ double rcp_f64(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = y * fma(-x, y, 2.0);
    y = y * fma(-x, y, 2.0);
    return y;
}

// u'(r)/r for the electron-electron Jastrow, from r^2; exactly 0 at r^2 == 0
// (coincident points: the gradient of an isotropic function is taken as 0).
//   Pade : u = r/(2(1+br))      -> u'/r = 1 / (2 r (1+br)^2)
//   power: u = sum c_k t^k      -> u'/r = (sum k c_k t^(k-1)) / (r (1+r)^2)
template <int KIND>
__device__ __forceinline__ double du_over_r(double r2, const JasDev& J) {
    const double s = rsq_f64(r2);                 // 1/r (not finite at r2 == 0: selected away)
    const double r = r2 * s;
    double f;
    if constexpr (KIND == 0) {
        const double it = rcp_f64(fma(J.b, r, 1.0));
        f = 0.5 * s * it * it;
    } else {
        const double q = rcp_f64(1.0 + r);
        const double t = r * q;
        double p = J.dcoef[15];
#pragma unroll
        for (int k = 14; k >= 0; --k) p = fma(p, t, J.dcoef[k]);
        f = p * q * q * s;
    }
    return r2 > 0.0 ? f : 0.0;
}

__device__ __forceinline__ int pair_index(int p, int q, int N) {
    // p <= q
    return p * N - (p * (p - 1)) / 2 + (q - p);
}

__device__ __forceinline__ int pair_sym(int p, int q, int N) {
    return p <= q ? pair_index(p, q, N) : pair_index(q, p, N);
}

}  // namespace xtc

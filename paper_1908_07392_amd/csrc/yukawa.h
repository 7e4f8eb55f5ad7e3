/*
 * yukawa.h -- scalar arithmetic of the modified-Helmholtz (Yukawa) layer
 * potentials, shared by the HIP kernels of this library.
 *
 *   G(x,y)      = K0(alpha r) / (2 pi)                       (single layer)
 *   dG/dn_y     = alpha K1(alpha r) (x-y).n_y / (2 pi r)     (double layer)
 *
 * K0(alpha r)/(2 pi) is the Yukawa part of the paper's modified-biharmonic
 * Green's function (Sec. 2 and App. B).  Two evaluators are provided:
 *
 *  * k01_*      : K0 and alpha K1(alpha r)/r for the far-field tiles
 *                 (z <= 2: log-split small-argument form of App. C with
 *                 fitted polynomials; z > 2: exp(-z)/sqrt(z) times a fitted
 *                 polynomial in 4/z - 1; coefficients in constants.h).
 *  * split_k01  : the kernel-split pieces of Sec. 4.1,
 *                 K0 = K0^S - I0 log z,  K1 = K1^S + I1 log z + 1/z,
 *                 returned as I0, K0^S, I1/z and K1^S/z (series of App. C),
 *                 used by the near-field quadrature.
 */
#pragma once
#include <hip/hip_runtime.h>

#include "constants.h"

namespace mhlp {

constexpr double PI = 3.14159265358979323846264338328;
constexpr double INV_2PI = 0.159154943091895335768883763373;
constexpr double LN2 = 0.693147180559945309417232121458;
constexpr double EULER_G = 0.577215664901532860606512090082;

template <int N, typename T>
__host__ __device__ __forceinline__ T horner(const T (&c)[N], T x)
{
    T v = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) v = fma(v, x, c[i]);
    return v;
}

/* ---------------------------------------------------------------------- */
/* Far-field kernel values, FP64.                                          */
/*   out.k0   = K0(z)                                                       */
/*   out.ak1r = alpha K1(z) / r          (z = alpha r)                      */
/* ---------------------------------------------------------------------- */
struct K01 {
    double k0;
    double ak1r;
};

/* r2 = |x-y|^2 > 0; a = alpha, a2q = alpha^2/4, a4 = 4/alpha */
template <bool SLP, bool DLP>
__host__ __device__ __forceinline__ K01 k01_fp64(double r2, double a, double a2q, double a4)
{
    K01 o{0.0, 0.0};
    const double q = a2q * r2; /* z^2/4 */
    if (q <= 1.0) {
        const double lq = log(q); /* 2 log(z/2) */
        if (SLP) o.k0 = fma(-0.5 * lq, horner(KS_I0, q), horner(KS_R0, q));
        if (DLP) {
            /* alpha K1/r = alpha^2 K1/z = 1/r^2 + alpha^2 (log(z/2) I1/z - R1/4) */
            const double t = fma(0.5 * lq, horner(KS_I1Z, q), -0.25 * horner(KS_R1, q));
            o.ak1r = fma(4.0 * a2q, t, 1.0 / r2);
        }
    } else {
        const double r = sqrt(r2);
        const double z = a * r;
        const double u = a4 / r - 1.0;
        const double e = exp(-z) / sqrt(z);
        if (SLP) o.k0 = e * horner(KL0, u);
        if (DLP) o.ak1r = a * e * horner(KL1, u) / r;
    }
    return o;
}

/* ---------------------------------------------------------------------- */
/* Far-field kernel values, FP32 (mixed-precision far field).               */
/* Same two regimes with the FP32 fits; exp/log/rsqrt/rcp are the hardware  */
/* single-precision instructions.  Below e^{-87} the FP32 result flushes to */
/* zero, far below the FP32 resolution of any potential it is summed into.  */
/* ---------------------------------------------------------------------- */
struct K01f {
    float k0;
    float ak1r;
};

template <bool SLP, bool DLP>
__device__ __forceinline__ K01f k01_fp32(float r2, float a, float a2q, float a4)
{
    K01f o{0.0f, 0.0f};
    const float q = a2q * r2;
    if (q <= 1.0f) {
        const float lq = __logf(q);
        if (SLP) o.k0 = fmaf(-0.5f * lq, horner(KSF_I0, q), horner(KSF_R0, q));
        if (DLP) {
            const float t = fmaf(0.5f * lq, horner(KSF_I1Z, q), -0.25f * horner(KSF_R1, q));
            o.ak1r = fmaf(4.0f * a2q, t, __frcp_rn(r2));
        }
    } else {
        const float ri = __frsqrt_rn(r2);
        const float r = r2 * ri;
        const float z = a * r;
        const float u = fmaf(a4, ri, -1.0f);
        const float e = __expf(-z) * __frsqrt_rn(z);
        if (SLP) o.k0 = e * horner(KLF0, u);
        if (DLP) o.ak1r = a * e * horner(KLF1, u) * ri;
    }
    return o;
}

/* ---------------------------------------------------------------------- */
/* Kernel-split pieces (paper Sec. 4.1, App. C), any moderate z >= 0.       */
/*   I0(z), K0S = K0 + I0 log z, I1z = I1(z)/z, K1Sz = (K1 - I1 log z - 1/z)/z */
/* Power series in q = z^2/4 with psi(n+1) = -gamma + sum_{k<=n} 1/k.        */
/* ---------------------------------------------------------------------- */
struct Split {
    double i0, k0s, i1z, k1sz;
};

__host__ __device__ inline Split split_k01(double z)
{
    const double q = 0.25 * z * z;
    double a = 1.0, b = 1.0; /* q^n/(n!)^2 and q^n/(n!(n+1)!) */
    double p1 = -EULER_G, p2 = 1.0 - EULER_G;
    double si0 = 0.0, si1 = 0.0, sr0 = 0.0, sr1 = 0.0;
    for (int n = 0; n < 80; ++n) {
        si0 += a;
        si1 += b;
        sr0 = fma(p1, a, sr0);
        sr1 = fma(p1 + p2, b, sr1);
        if (a <= 1e-18 * si0 && b <= 1e-18 * si1) break;
        const double n1 = n + 1.0;
        a *= q / (n1 * n1);
        b *= q / (n1 * (n1 + 1.0));
        p1 += 1.0 / n1;
        p2 += 1.0 / (n1 + 1.0);
    }
    Split s;
    s.i0 = si0;
    s.i1z = 0.5 * si1;
    /* K0 = -log(z/2) I0 + R0  =>  K0 + I0 log z = I0 log 2 + R0 */
    s.k0s = fma(LN2, si0, sr0);
    /* K1 = 1/z + log(z/2) I1 - (z/4) R1  =>  (K1 - I1 log z - 1/z)/z = -log2 I1/z - R1/4 */
    s.k1sz = fma(-LN2, s.i1z, -0.25 * sr1);
    return s;
}

/* ---------------------------------------------------------------------- */
/* Minimal complex arithmetic                                               */
/* ---------------------------------------------------------------------- */
struct cplx {
    double re, im;
};
__host__ __device__ __forceinline__ cplx mk(double r, double i) { return cplx{r, i}; }
__host__ __device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__host__ __device__ __forceinline__ cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__host__ __device__ __forceinline__ cplx operator-(cplx a) { return {-a.re, -a.im}; }
__host__ __device__ __forceinline__ cplx operator*(cplx a, cplx b)
{
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__host__ __device__ __forceinline__ cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
__host__ __device__ __forceinline__ cplx operator*(cplx a, double s) { return {s * a.re, s * a.im}; }
__host__ __device__ __forceinline__ double cabs2(cplx a) { return fma(a.re, a.re, a.im * a.im); }
__host__ __device__ __forceinline__ double cabs(cplx a) { return hypot(a.re, a.im); }
__host__ __device__ __forceinline__ cplx conj(cplx a) { return {a.re, -a.im}; }
__host__ __device__ inline cplx operator/(cplx a, cplx b)
{
    /* scaled division (Smith) */
    if (fabs(b.re) >= fabs(b.im)) {
        double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    double r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__host__ __device__ inline cplx clog(cplx a) { return {log(cabs(a)), atan2(a.im, a.re)}; }
__host__ __device__ inline cplx csqrt(cplx a)
{
    double m = cabs(a);
    if (m == 0.0) return {0.0, 0.0};
    double re = sqrt(0.5 * (m + fabs(a.re)));
    double im = 0.5 * a.im / re;
    if (a.re >= 0.0) return {re, im};
    return {fabs(im), a.im >= 0.0 ? re : -re};
}

} // namespace mhlp

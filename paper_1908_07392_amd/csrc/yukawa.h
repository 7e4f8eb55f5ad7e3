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
/* Far-field kernel values, FP64, device-lean version for the tile kernels.  */
/* Same regimes and coefficients as k01_fp64 with lean elementary functions: */
/*  * 1/sqrt and 1/x: hardware v_rsq_f64 / v_rcp_f64 estimates refined by    */
/*    one Newton-type step (third order for rsq, two steps for rcp);         */
/*  * e^{-z}: Cody-Waite reduction z = n ln2 - r, |r| <= ln2/2, degree-13    */
/*    Taylor polynomial (truncation 4e-18), scaling by 2^-n (ldexp);         */
/*  * log q, 0 < q <= 1: q = m 2^e with m in [sqrt(1/2), sqrt(2)),           */
/*    log m = 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.1716, series to s^21.     */
/* ---------------------------------------------------------------------- */
constexpr double LN2_HI = 6.93147180369123816490e-01; /* ln 2 split: hi has 32 bits */
constexpr double LN2_LO = 1.90821492927058770002e-10;
constexpr double LOG2E = 1.44269504088896338700e+00;
constexpr double SQRT_HALF = 0.707106781186547524401;
/* 1/k!, k = 0..13 */
static constexpr double EXP_T[14] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0, 1.0 / 720.0, 1.0 / 5040.0,
                                     1.0 / 40320.0, 1.0 / 362880.0, 1.0 / 3628800.0, 1.0 / 39916800.0,
                                     1.0 / 479001600.0, 1.0 / 6227020800.0};
/* 1/(2k+1), k = 0..10 */
static constexpr double ATANH_T[11] = {1.0, 1.0 / 3.0, 1.0 / 5.0, 1.0 / 7.0, 1.0 / 9.0, 1.0 / 11.0,
                                       1.0 / 13.0, 1.0 / 15.0, 1.0 / 17.0, 1.0 / 19.0, 1.0 / 21.0};

/* Coefficient tables of the far-field kernel values, in the constant
   address space.  The tile kernels fetch the table pointer through
   far_table() once per pair of sources: the empty asm makes the pointer
   opaque, so the compiler cannot hoist the (scalar) loads of the
   coefficients out of the source loop into vector registers.  Each
   coefficient then reaches its v_fma_f64 as a scalar-register operand, and
   the vector register file holds only per-lane state (about 110 instead of
   about 200 registers in the fused kernel: 4 instead of 2 waves per SIMD). */
#define MHLP_CAS __attribute__((address_space(4)))
struct FarTable {
    double kl0[23], kl1[23], expt[14], atanh[11], ks_i0[12], ks_r0[13], ks_i1z[12], ks_r1[13];
};

constexpr FarTable make_far_table()
{
    FarTable t{};
    for (int i = 0; i < 23; ++i) t.kl0[i] = KL0[i], t.kl1[i] = KL1[i];
    for (int i = 0; i < 14; ++i) t.expt[i] = EXP_T[i];
    for (int i = 0; i < 11; ++i) t.atanh[i] = ATANH_T[i];
    for (int i = 0; i < 12; ++i) t.ks_i0[i] = KS_I0[i], t.ks_i1z[i] = KS_I1Z[i];
    for (int i = 0; i < 13; ++i) t.ks_r0[i] = KS_R0[i], t.ks_r1[i] = KS_R1[i];
    return t;
}

static __constant__ FarTable FAR_TAB = make_far_table();

typedef const MHLP_CAS FarTable *FarTab;

__device__ __forceinline__ FarTab far_table()
{
    FarTab T = (FarTab)&FAR_TAB;
    asm volatile("" : "+s"(T));
    return T;
}

template <int N>
__device__ __forceinline__ double hornerc(const MHLP_CAS double *c, double x)
{
    double v = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) v = fma(v, x, c[i]);
    return v;
}

/* value and first derivative of the polynomial */
template <int N>
__device__ __forceinline__ double hornercd(const MHLP_CAS double *c, double x, double &d)
{
    double v = c[N - 1];
    d = 0.0;
#pragma unroll
    for (int i = N - 2; i >= 0; --i) {
        d = fma(d, x, v);
        v = fma(v, x, c[i]);
    }
    return v;
}

__device__ __forceinline__ double lean_rsq(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

__device__ __forceinline__ double lean_rcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ double lean_exp_neg(FarTab T, double z)
{
    const double n = rint(z * LOG2E);
    double r = fma(n, LN2_HI, -z);
    r = fma(n, LN2_LO, r);
    return ldexp(hornerc<14>(T->expt, r), -(int)n);
}

__device__ __forceinline__ double lean_log01(FarTab T, double q)
{
    int e;
    double m = frexp(q, &e);
    const bool lo = m < SQRT_HALF;
    m = lo ? 2.0 * m : m;
    e -= lo ? 1 : 0;
    const double s = (m - 1.0) * lean_rcp(m + 1.0);
    const double p = hornerc<11>(T->atanh, s * s);
    const double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, 2.0 * s * p));
}

/* K0(z) and alpha K1(z)/r for the far-field tiles.  When both layers are
   wanted, K1 is taken from the derivative of the K0 fits (K1 = -K0'):
     z > 2 : K0 = E P0(u), K1 = E [P0 (1 + 1/(2z)) + (4/z^2) P0'(u)],
             E = e^{-z}/sqrt(z), u = 4/z - 1;
     z <= 2: K1 = I0/z + (z/4) log(q) I0'(q) - (z/2) R0'(q), q = z^2/4,
   which halves the coefficient tables (max rel. error 3e-15 vs 5e-16 for the
   separate fits; measured against mpmath).  ia = 1/alpha.
   k01_far_big evaluates the z > 2 form for any r2 > 0 (finite or inf/nan
   garbage when z <= 2); k01_far_small is the z <= 2 form.  k01_far2 takes
   two pairs: both big forms straight-line (independent instruction streams
   the scheduler interleaves) on lanes where either pair needs it, then the
   small form on lanes that need it, overwriting the big values. */
template <bool SLP, bool DLP>
__device__ __forceinline__ K01 k01_far_big(FarTab T, double r2, double a, double a4, double ia)
{
    K01 o{0.0, 0.0};
    const double ri = lean_rsq(r2);
    const double z = a * (r2 * ri);
    const double u = fma(a4, ri, -1.0);
    const double e = lean_exp_neg(T, z) * lean_rsq(z);
    if (SLP && DLP) {
        double dp;
        const double p = hornercd<23>(T->kl0, u, dp);
        o.k0 = e * p;
        const double iz = ia * ri; /* 1/z */
        const double k1 = e * fma(4.0 * iz * iz, dp, p * fma(0.5, iz, 1.0));
        o.ak1r = a * k1 * ri;
    } else if (SLP) {
        o.k0 = e * hornerc<23>(T->kl0, u);
    } else {
        o.ak1r = a * e * hornerc<23>(T->kl1, u) * ri;
    }
    return o;
}

template <bool SLP, bool DLP>
__device__ __forceinline__ K01 k01_far_small(FarTab T, double r2, double a2q)
{
    K01 o{0.0, 0.0};
    const double q = a2q * r2; /* z^2/4 */
    const double lq = lean_log01(T, q); /* 2 log(z/2) */
    if (SLP && DLP) {
        double di0, dr0;
        const double i0 = hornercd<12>(T->ks_i0, q, di0);
        const double r0 = hornercd<13>(T->ks_r0, q, dr0);
        o.k0 = fma(-0.5 * lq, i0, r0);
        /* alpha^2 K1/z = I0/r^2 + alpha^2 (lq I0'/4 - R0'/2) */
        o.ak1r = fma(4.0 * a2q, fma(0.25 * lq, di0, -0.5 * dr0), i0 * lean_rcp(r2));
    } else if (SLP) {
        o.k0 = fma(-0.5 * lq, hornerc<12>(T->ks_i0, q), hornerc<13>(T->ks_r0, q));
    } else {
        const double t = fma(0.5 * lq, hornerc<12>(T->ks_i1z, q), -0.25 * hornerc<13>(T->ks_r1, q));
        o.ak1r = fma(4.0 * a2q, t, lean_rcp(r2));
    }
    return o;
}

struct FarConst {
    double a, a2q, a4, ia; /* alpha, alpha^2/4, 4/alpha, 1/alpha */
};

__device__ __forceinline__ FarConst far_const(double alpha)
{
    return FarConst{alpha, 0.25 * alpha * alpha, 4.0 / alpha, 1.0 / alpha};
}

template <bool SLP, bool DLP>
__device__ __forceinline__ void k01_far2(FarTab T, const FarConst &c, double r2a, double r2b, K01 &oa, K01 &ob)
{
    const bool sa = c.a2q * r2a <= 1.0, sb = c.a2q * r2b <= 1.0;
    if (!(sa && sb)) {
        oa = k01_far_big<SLP, DLP>(T, r2a, c.a, c.a4, c.ia);
        ob = k01_far_big<SLP, DLP>(T, r2b, c.a, c.a4, c.ia);
    }
    if (sa || sb) {
        if (sa) oa = k01_far_small<SLP, DLP>(T, r2a, c.a2q);
        if (sb) ob = k01_far_small<SLP, DLP>(T, r2b, c.a2q);
    }
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

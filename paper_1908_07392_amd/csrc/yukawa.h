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
    double ri2; /* 1/r^2 (far-field evaluators only; dropped where unused) */
};

/* r2 = |x-y|^2 > 0; a = alpha, a2q = alpha^2/4, a4 = 4/alpha */
template <bool SLP, bool DLP>
__host__ __device__ __forceinline__ K01 k01_fp64(double r2, double a, double a2q, double a4)
{
    K01 o{0.0, 0.0, 0.0};
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
/*  * e^{-z}, z >= 0: Cody-Waite reduction z = k ln2/64 - r, |r| <= ln2/128,*/
/*    a table of 2^{-j/64} (Tang's table-driven method), degree-5 Taylor     */
/*    polynomial (truncation 4e-17), scaling by 2^-(k/64) (ldexp);           */
/*  * log q, 0 < q <= 1: q = m 2^e with m in [sqrt(1/2), sqrt(2)),           */
/*    log m = 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.1716, series to s^21.     */
/* ---------------------------------------------------------------------- */
constexpr double LN2_HI = 6.93147180369123816490e-01; /* ln 2 split: hi has 32 bits */
constexpr double LN2_LO = 1.90821492927058770002e-10;
constexpr double LOG2E = 1.44269504088896338700e+00;
constexpr double SQRT_HALF = 0.707106781186547524401;
/* 1/k!, k = 0..5 */
static constexpr double EXP_T[6] = {1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0, 1.0 / 120.0};
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
/* the fine pieces: KQ_NB single pieces z in (KQ_B[k], KQ_B[k+1]] (k < KQ_NB,
   the last unbounded) and KQ_NB - 1 pieces spanning two neighbours,
   z in (KQ_B[s], KQ_B[s+2]] (k = KQ_NB + s); coefficient counts of the K0 and
   K1 fits */
constexpr int KQ_NB = 8, KQ_NP = 2 * KQ_NB - 1;
constexpr int KQ_N0[KQ_NP] = {11, 10, 10, 9, 8, 8, 7, 7, 13, 13, 12, 11, 10, 9, 8};
constexpr int KQ_N1[KQ_NP] = {11, 10, 10, 9, 8, 8, 7, 7, 13, 13, 12, 11, 10, 9, 8};
/* the coefficient counts above against the generated tables */
template <int K, size_t N0, size_t N1>
constexpr bool kq_sizes(const double (&)[N0], const double (&)[N1])
{
    return N0 == (size_t)KQ_N0[K] && N1 == (size_t)KQ_N1[K];
}
static_assert(kq_sizes<0>(KQ0_0, KQ1_0) && kq_sizes<1>(KQ0_1, KQ1_1) && kq_sizes<2>(KQ0_2, KQ1_2) &&
                  kq_sizes<3>(KQ0_3, KQ1_3) && kq_sizes<4>(KQ0_4, KQ1_4) && kq_sizes<5>(KQ0_5, KQ1_5) &&
                  kq_sizes<6>(KQ0_6, KQ1_6) && kq_sizes<7>(KQ0_7, KQ1_7) && kq_sizes<8>(KQ0_8, KQ1_8) &&
                  kq_sizes<9>(KQ0_9, KQ1_9) && kq_sizes<10>(KQ0_10, KQ1_10) && kq_sizes<11>(KQ0_11, KQ1_11) &&
                  kq_sizes<12>(KQ0_12, KQ1_12) && kq_sizes<13>(KQ0_13, KQ1_13) && kq_sizes<14>(KQ0_14, KQ1_14),
              "fine-piece coefficient counts differ from the generated tables");
static_assert(sizeof(KQF0[0]) == 6 * sizeof(float) && sizeof(KQF1[0]) == 6 * sizeof(float),
              "FP32 fine pieces are padded to 6 coefficients");
static_assert(sizeof(KP0M) == 12 * sizeof(double) && sizeof(KP0X) == 10 * sizeof(double) &&
                  sizeof(KP1M) == 11 * sizeof(double) && sizeof(KP1X) == 9 * sizeof(double),
              "middle and far piece lengths differ from the generated tables");
struct FarTable {
    double kp0n[17], kp0f[16], kp1n[15], kp1f[14], kl0[23], expt[6], atanh[11], ks_i0[12], ks_r0[13], ks_i1z[12],
        ks_r1[13];
    double exp2nj[64]; /* 2^(-j/64) */
    double kp0m[12], kp0x[10], kp1m[11], kp1x[9]; /* the z > 6 piece split at z = 20 */
    double kq0[15][13], kq1[15][13];               /* the fine pieces (KQ0_k, KQ1_k), zero padded */
    double kqb[15];                                /* their constant v offsets (-2 - ulo - uhi)/(uhi - ulo) */
    double stk[6][14]; /* stresslet smooth parts T1S, T2S, T3S, T1L, T2L, T3L in q = z^2/4 <= 1 */
};

constexpr FarTable make_far_table()
{
    FarTable t{};
    for (int i = 0; i < 23; ++i) t.kl0[i] = KL0[i];
    for (int i = 0; i < 17; ++i) t.kp0n[i] = KP0N[i];
    for (int i = 0; i < 16; ++i) t.kp0f[i] = KP0F[i];
    for (int i = 0; i < 15; ++i) t.kp1n[i] = KP1N[i];
    for (int i = 0; i < 14; ++i) t.kp1f[i] = KP1F[i];
    for (int i = 0; i < 12; ++i) t.kp0m[i] = KP0M[i];
    for (int i = 0; i < 10; ++i) t.kp0x[i] = KP0X[i];
    for (int i = 0; i < 11; ++i) t.kp1m[i] = KP1M[i];
    for (int i = 0; i < 9; ++i) t.kp1x[i] = KP1X[i];
    const double *q0[KQ_NP] = {KQ0_0, KQ0_1, KQ0_2, KQ0_3,  KQ0_4,  KQ0_5,  KQ0_6, KQ0_7,
                               KQ0_8, KQ0_9, KQ0_10, KQ0_11, KQ0_12, KQ0_13, KQ0_14};
    const double *q1[KQ_NP] = {KQ1_0, KQ1_1, KQ1_2, KQ1_3,  KQ1_4,  KQ1_5,  KQ1_6, KQ1_7,
                               KQ1_8, KQ1_9, KQ1_10, KQ1_11, KQ1_12, KQ1_13, KQ1_14};
    for (int k = 0; k < KQ_NP; ++k) {
        for (int i = 0; i < KQ_N0[k]; ++i) t.kq0[k][i] = q0[k][i];
        for (int i = 0; i < KQ_N1[k]; ++i) t.kq1[k][i] = q1[k][i];
        t.kqb[k] = (-2.0 - KQ_ULO[k] - KQ_UHI[k]) / (KQ_UHI[k] - KQ_ULO[k]);
    }
    for (int i = 0; i < 6; ++i) t.expt[i] = EXP_T[i];
    for (int i = 0; i < 64; ++i) t.exp2nj[i] = EXP2_NJ[i];
    for (int i = 0; i < 11; ++i) t.atanh[i] = ATANH_T[i];
    for (int i = 0; i < 12; ++i) t.ks_i0[i] = KS_I0[i], t.ks_i1z[i] = KS_I1Z[i];
    for (int i = 0; i < 13; ++i) t.ks_r0[i] = KS_R0[i], t.ks_r1[i] = KS_R1[i];
    for (int i = 0; i < 14; ++i) {
        t.stk[0][i] = STK_S1[i], t.stk[1][i] = STK_S2[i], t.stk[2][i] = STK_S3[i];
        t.stk[3][i] = STK_L1[i], t.stk[4][i] = STK_L2[i], t.stk[5][i] = STK_L3[i];
    }
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
    /* first step written out (d would start as fma(0, x, c[N-1]), which the
       compiler may not fold) */
    d = c[N - 1];
    double v = fma(c[N - 1], x, c[N - 2]);
#pragma unroll
    for (int i = N - 3; i >= 0; --i) {
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

/* e^{-z} for z >= 0: k = round(64 z log2 e), r = k ln2/64 - z with
   |r| <= ln2/128 (+ rounding), e^{-z} = 2^{-(k >> 6)} 2^{-(k & 63)/64} e^r
   (Tang's table-driven reduction: the table entry is a per-lane load, and the
   Taylor polynomial of e^r needs 6 terms, truncation below 4e-17 relative;
   the reduction by ln 2 alone needs 14).  k comes from adding 1.5 * 2^52,
   whose low word then holds it as an integer; k ln2/64 is exact in its high
   part (LN2_HI has 21 trailing zero bits, k < 2^21 for z < 2e4, and e^{-z}
   underflows to zero long before). */
__device__ __forceinline__ double lean_exp_neg(FarTab T, double z)
{
    constexpr double SHIFT = 6755399441055744.0; /* 1.5 * 2^52 */
    const double t = fma(z, 64.0 * LOG2E, SHIFT);
    const double kd = t - SHIFT;
    double r = fma(kd, LN2_HI / 64.0, -z);
    r = fma(kd, LN2_LO / 64.0, r);
    const int k = __double2loint(t);
    return ldexp(T->exp2nj[k & 63] * hornerc<6>(T->expt, r), -(k >> 6));
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

/* K0(z) and alpha K1(z)/r for the far-field tiles.
     z > 2 : K_nu = E P(v), E = e^{-z}/sqrt(z), u = 4/z - 1, on two pieces:
             z <= 6 (v = 1.5 u - 0.5) and z > 6 (v = 3 u + 2), v in [-1, 1];
             with both layers, K1 = -K0' = E [P0 (1 + 1/(2z)) + (4/z^2) dP0/du]
             from the K0 pieces (degree 16 / 15; K1 alone: degree 14 / 13);
     z <= 2: K1 = I0/z + (z/4) log(q) I0'(q) - (z/2) R0'(q), q = z^2/4.
   Max rel. error of the z > 2 pieces 1.2e-16 for K0 and K1 (40-digit check).
   The K1R form (the potentials' tiles) splits the z > 6 piece again at
   z = 20 (degree 11 / 9 for K0, 10 / 8 for K1; 1.7e-16), which shortens the
   polynomials of the far pairs, and takes K1 from its own fits with both
   layers too: two independent chains of N0 + N1 - 2 FMA against 2 N0 - 3 and
   a combining step for K1 from the K0 fit's derivative.
   k01_far_small is the z <= 2 form.  k01_far2 takes two sources: the z > 2
   forms straight-line for both (independent instruction streams the
   scheduler interleaves) on lanes where either needs it, with the common
   piece when both fall on the same side of z = 6, then the z <= 2 form on
   the lanes that need it, overwriting the other values. */
struct FarConst {
    double a, a2q, a4, ia; /* alpha, alpha^2/4, 4/alpha, 1/alpha */
    double vn;             /* 6/alpha: v = vn/r - 2 on 2 < z <= 6 */
    /* pieces 6 < z <= 20 (v = vm/r + om) and z > 20 (v = vx/r - 1): with
       u = 4/z - 1 on [-0.8, -1/3] and [-1, -0.8], v = (30u + 17)/7 and 10u + 9 */
    double vm, om, vx;
};

__device__ __forceinline__ FarConst far_const(double alpha)
{
    const double ia = 1.0 / alpha;
    return FarConst{alpha, 0.25 * alpha * alpha, 4.0 / alpha, ia, 6.0 * ia, 120.0 / 7.0 * ia, -13.0 / 7.0, 40.0 * ia};
}

/* polynomial of the two-piece form (value and d/du) at 1/r = ri */
template <bool SLP, bool DLP, bool FAR>
__device__ __forceinline__ double far_piece(FarTab T, const FarConst &c, double ri, double &dpdu)
{
    /* v = 3u + 2 = (12/alpha) ri - 1 (far);  v = 1.5u - 0.5 = (6/alpha) ri - 2 (near) */
    const double v = FAR ? fma(3.0 * c.a4, ri, -1.0) : fma(1.5 * c.a4, ri, -2.0);
    if (SLP && DLP) {
        double d;
        const double p = FAR ? hornercd<16>(T->kp0f, v, d) : hornercd<17>(T->kp0n, v, d);
        dpdu = d * (FAR ? 3.0 : 1.5);
        return p;
    }
    dpdu = 0.0;
    if (SLP) return FAR ? hornerc<16>(T->kp0f, v) : hornerc<17>(T->kp0n, v);
    return FAR ? hornerc<14>(T->kp1f, v) : hornerc<15>(T->kp1n, v);
}

/* the K1R pieces: P = 0 for 2 < z <= 6, 1 for 6 < z <= 20, 2 for z > 20;
   the K0 fit's value at 1/r = ri and, with both layers, the K1 fit's value in
   p1 (two independent chains: fewer FMA than K1 from the K0 fit's derivative) */
template <bool SLP, bool DLP, int P>
__device__ __forceinline__ double far_piece3(FarTab T, const FarConst &c, double ri, double &p1)
{
    const double v = P == 0 ? fma(c.vn, ri, -2.0) : P == 1 ? fma(c.vm, ri, c.om) : fma(c.vx, ri, -1.0);
    if (SLP && DLP) {
        p1 = P == 0 ? hornerc<15>(T->kp1n, v) : P == 1 ? hornerc<11>(T->kp1m, v) : hornerc<9>(T->kp1x, v);
        return P == 0 ? hornerc<17>(T->kp0n, v) : P == 1 ? hornerc<12>(T->kp0m, v) : hornerc<10>(T->kp0x, v);
    }
    p1 = 0.0;
    if (SLP) return P == 0 ? hornerc<17>(T->kp0n, v) : P == 1 ? hornerc<12>(T->kp0m, v) : hornerc<10>(T->kp0x, v);
    return P == 0 ? hornerc<15>(T->kp1n, v) : P == 1 ? hornerc<11>(T->kp1m, v) : hornerc<9>(T->kp1x, v);
}

/* K1R = false: out.ak1r = alpha K1(z)/r, with both layers from the K0 piece
   as K1/E = P (1 + 1/(2z)) + (4/z^2) dP/du.  K1R = true: out.ak1r = K1(z)/r
   (the caller scales its dipoles by alpha); with both layers dpdu then holds
   the K1 fit's value at the pair. */
template <bool SLP, bool DLP, bool K1R = false>
__device__ __forceinline__ K01 far_finish(const FarConst &c, double ri, double z, double e, double p, double dpdu)
{
    K01 o{0.0, 0.0, ri * ri};
    if (SLP && DLP) {
        o.k0 = e * p;
        if (K1R) {
            o.ak1r = (e * ri) * dpdu; /* dpdu: the piece's K1 fit value */
        } else {
            const double iz = c.ia * ri; /* 1/z */
            const double k1 = e * fma(4.0 * iz * iz, dpdu, p * fma(0.5, iz, 1.0));
            o.ak1r = c.a * k1 * ri;
        }
    } else if (SLP) {
        o.k0 = e * p;
    } else {
        o.ak1r = K1R ? e * p * ri : c.a * e * p * ri;
    }
    (void)z;
    return o;
}

/* z <= 2.  K1R: out.ak1r = K1(z)/r (the alpha^2 K1/z form over alpha). */
template <bool SLP, bool DLP, bool K1R = false>
__device__ __forceinline__ K01 k01_far_small(FarTab T, double r2, const FarConst &c)
{
    K01 o{0.0, 0.0, lean_rcp(r2)};
    const double q = c.a2q * r2; /* z^2/4 */
    const double lq = lean_log01(T, q); /* 2 log(z/2) */
    const double s = K1R ? c.a : 4.0 * c.a2q;      /* alpha^2, over alpha with K1R */
    const double ri2 = K1R ? o.ri2 * c.ia : o.ri2; /* 1/r^2, over alpha with K1R */
    if (SLP && DLP) {
        double di0, dr0;
        const double i0 = hornercd<12>(T->ks_i0, q, di0);
        const double r0 = hornercd<13>(T->ks_r0, q, dr0);
        o.k0 = fma(-0.5 * lq, i0, r0);
        /* alpha^2 K1/z = I0/r^2 + alpha^2 (lq I0'/4 - R0'/2) */
        o.ak1r = fma(s, fma(0.25 * lq, di0, -0.5 * dr0), i0 * ri2);
    } else if (SLP) {
        o.k0 = fma(-0.5 * lq, hornerc<12>(T->ks_i0, q), hornerc<13>(T->ks_r0, q));
    } else {
        const double t = fma(0.5 * lq, hornerc<12>(T->ks_i1z, q), -0.25 * hornerc<13>(T->ks_r1, q));
        o.ak1r = fma(s, t, ri2);
    }
    return o;
}

/* PIECES = false (K0 only): one degree-22 fit over all z > 2 in u = 4/z - 1,
   for launches whose lanes often straddle z = 6 (targets in no spatial order) */
/* the z > 2 forms for two sources, straight-line (see k01_far2) */
template <bool SLP, bool DLP, bool PIECES = true, bool K1R = false>
__device__ __forceinline__ void k01_far2_big(FarTab T, const FarConst &c, double r2a, double r2b, K01 &oa, K01 &ob)
{
    static_assert(PIECES || (SLP && !DLP), "the single fit serves the single layer only");
    const double ria = lean_rsq(r2a), rib = lean_rsq(r2b);
    const double za = c.a * (r2a * ria), zb = c.a * (r2b * rib);
    const double ea = lean_exp_neg(T, za) * lean_rsq(za), eb = lean_exp_neg(T, zb) * lean_rsq(zb);
    const bool fa = za > 6.0, fb = zb > 6.0;
    double pa, pb, da = 0.0, db = 0.0;
    if (!PIECES) {
        pa = hornerc<23>(T->kl0, fma(c.a4, ria, -1.0));
        pb = hornerc<23>(T->kl0, fma(c.a4, rib, -1.0));
    } else if (K1R) {
        /* three pieces; both sources in one piece run straight-line */
        const bool xa = za > 20.0, xb = zb > 20.0;
        if (xa && xb) {
            pa = far_piece3<SLP, DLP, 2>(T, c, ria, da);
            pb = far_piece3<SLP, DLP, 2>(T, c, rib, db);
        } else if (fa && fb && !xa && !xb) {
            pa = far_piece3<SLP, DLP, 1>(T, c, ria, da);
            pb = far_piece3<SLP, DLP, 1>(T, c, rib, db);
        } else if (!fa && !fb) {
            pa = far_piece3<SLP, DLP, 0>(T, c, ria, da);
            pb = far_piece3<SLP, DLP, 0>(T, c, rib, db);
        } else {
            if (xa)
                pa = far_piece3<SLP, DLP, 2>(T, c, ria, da);
            else if (fa)
                pa = far_piece3<SLP, DLP, 1>(T, c, ria, da);
            else
                pa = far_piece3<SLP, DLP, 0>(T, c, ria, da);
            if (xb)
                pb = far_piece3<SLP, DLP, 2>(T, c, rib, db);
            else if (fb)
                pb = far_piece3<SLP, DLP, 1>(T, c, rib, db);
            else
                pb = far_piece3<SLP, DLP, 0>(T, c, rib, db);
        }
    } else if (fa && fb) {
        pa = far_piece<SLP, DLP, true>(T, c, ria, da);
        pb = far_piece<SLP, DLP, true>(T, c, rib, db);
    } else if (!fa && !fb) {
        pa = far_piece<SLP, DLP, false>(T, c, ria, da);
        pb = far_piece<SLP, DLP, false>(T, c, rib, db);
    } else {
        if (fa)
            pa = far_piece<SLP, DLP, true>(T, c, ria, da);
        else
            pa = far_piece<SLP, DLP, false>(T, c, ria, da);
        if (fb)
            pb = far_piece<SLP, DLP, true>(T, c, rib, db);
        else
            pb = far_piece<SLP, DLP, false>(T, c, rib, db);
    }
    oa = far_finish<SLP, DLP, K1R>(c, ria, za, ea, pa, da);
    ob = far_finish<SLP, DLP, K1R>(c, rib, zb, eb, pb, db);
}

/* The fine piece K at 1/r = ri: the K0 (SLP) or K1 (DLP) fit's value and,
   with both layers, the K1 fit's value in dpdu as far_finish<.., K1R> takes it.  v = qa ri + qb with qa = (4/alpha) w,
   w = 2/(uhi - ulo), and qk = (4/alpha^2) w.  A plan keeps the qa of every
   piece, then every qk, in device memory (fine_scales); fine_q reads the two
   of piece K through an opaque pointer, once per panel, into scalar
   registers (the compiler cannot hoist the reads of all pieces out of the
   loops, where they would stay live). */
__host__ inline void fine_scales(double alpha, double *q)
{
    for (int k = 0; k < KQ_NP; ++k) {
        const double w = 2.0 / (KQ_UHI[k] - KQ_ULO[k]);
        q[k] = 4.0 / alpha * w;
        q[KQ_NP + k] = 4.0 / (alpha * alpha) * w;
    }
}

template <int K>
__device__ __forceinline__ void fine_q(const double *fq, double &qa, double &qk)
{
    const MHLP_CAS double *q = (const MHLP_CAS double *)fq;
    asm volatile("" : "+s"(q));
    qa = q[K];
    qk = q[KQ_NP + K];
}

template <bool SLP, bool DLP, int K>
__device__ __forceinline__ double far_piece_fine(FarTab T, double qa, double qk, double ri, double &dpdu)
{
    const double v = fma(qa, ri, T->kqb[K]);
    if (SLP && DLP) { /* both layers: the K1 fit's value in dpdu, as far_finish<.., K1R> takes it */
        dpdu = hornerc<KQ_N1[K]>(T->kq1[K], v);
        (void)qk;
        return hornerc<KQ_N0[K]>(T->kq0[K], v);
    }
    dpdu = 0.0;
    if (SLP) return hornerc<KQ_N0[K]>(T->kq0[K], v);
    return hornerc<KQ_N1[K]>(T->kq1[K], v);
}

/* K0 and K1(z)/r (the K1R form) of two sources whose pairs are known to lie in
   one piece: PC = 0..KQ_NP-1 the fine pieces, PC = -1 z <= 2 (k01_far_small).  The
   arithmetic of k01_far2's z > 2 form with the fine piece's polynomial and
   without any per-pair selection: for launches that classify a whole wave
   against a panel beforehand (qa, qk: the piece's scales from fine_q). */
template <bool SLP, bool DLP, int PC>
__device__ __forceinline__ void k01_far2_fixed(FarTab T, const FarConst &c, double qa, double qk, double r2a,
                                               double r2b, K01 &oa, K01 &ob)
{
    if constexpr (PC < 0) {
        oa = k01_far_small<SLP, DLP, true>(T, r2a, c);
        ob = k01_far_small<SLP, DLP, true>(T, r2b, c);
        return;
    }
    constexpr int P = PC < 0 ? 0 : PC;
    const double ria = lean_rsq(r2a), rib = lean_rsq(r2b);
    const double za = c.a * (r2a * ria), zb = c.a * (r2b * rib);
    const double ea = lean_exp_neg(T, za) * lean_rsq(za), eb = lean_exp_neg(T, zb) * lean_rsq(zb);
    double da = 0.0, db = 0.0;
    const double pa = far_piece_fine<SLP, DLP, P>(T, qa, qk, ria, da);
    const double pb = far_piece_fine<SLP, DLP, P>(T, qa, qk, rib, db);
    oa = far_finish<SLP, DLP, true>(c, ria, za, ea, pa, da);
    ob = far_finish<SLP, DLP, true>(c, rib, zb, eb, pb, db);
}

/* PIECES = false (K0 only): one degree-22 fit over all z > 2 in u = 4/z - 1,
   for launches whose lanes often straddle z = 6 (targets in no spatial order) */
template <bool SLP, bool DLP, bool PIECES = true, bool K1R = false>
__device__ __forceinline__ void k01_far2(FarTab T, const FarConst &c, double r2a, double r2b, K01 &oa, K01 &ob)
{
    const bool sa = c.a2q * r2a <= 1.0, sb = c.a2q * r2b <= 1.0;
    if (!(sa && sb)) k01_far2_big<SLP, DLP, PIECES, K1R>(T, c, r2a, r2b, oa, ob);
    if (sa || sb) {
        if (sa) oa = k01_far_small<SLP, DLP, K1R>(T, r2a, c);
        if (sb) ob = k01_far_small<SLP, DLP, K1R>(T, r2b, c);
    }
}

/* alpha^2 T1, alpha^4 T2, alpha^2 T3 of the stresslet for two sources (far
   tiles): closed forms from the z > 2 values of K0 and alpha K1/r, and for
   z <= 2 the split T = TS + TL log z (+ the explicit terms of T2) with TS, TL
   fitted in q = z^2/4 (the closed forms cancel there).  al2 = alpha^2,
   ial2 = 1/alpha^2. */
__device__ __forceinline__ void stk_closed(double al2, double ial2, double r2, double ri2, double k0, double ak1r,
                                           double *A)
{
    const double w = al2 * r2;    /* z^2 */
    const double zk1 = ak1r * r2; /* z K1 */
    const double ri4 = ri2 * ri2;
    A[0] = (-INV_2PI * ial2) * ri4 * fma(2.0 * w, k0, fma(w + 4.0, zk1, -4.0));
    A[1] = (ial2 * (1.0 / PI)) * ri4 * ri2 * fma(4.0 * w, k0, fma(w + 8.0, zk1, -8.0));
    A[2] = INV_2PI * ri2 * (zk1 - 1.0);
}

__device__ __forceinline__ void stk_small(FarTab T, const FarConst &c, double al2, double r2, double *A)
{
    const double q = c.a2q * r2;
    const double lz = fma(0.5, lean_log01(T, q), LN2); /* log z = log(q)/2 + log 2 */
    const double ri2 = lean_rcp(r2);
    const double t1 = fma(hornerc<14>(T->stk[3], q), lz, hornerc<14>(T->stk[0], q));
    const double t2 = fma(hornerc<14>(T->stk[4], q), lz, hornerc<14>(T->stk[1], q));
    const double t3 = fma(hornerc<14>(T->stk[5], q), lz, hornerc<14>(T->stk[2], q));
    A[0] = al2 * t1;
    A[1] = fma(al2 * al2, t2, ri2 * fma(al2, 1.0 / (8.0 * PI), -ri2 * (1.0 / PI)));
    A[2] = al2 * t3;
}

__device__ __forceinline__ void stk_far2(FarTab T, const FarConst &c, double al2, double ial2, double r2a,
                                         double r2b, double *Aa, double *Ab)
{
    const bool sa = c.a2q * r2a <= 1.0, sb = c.a2q * r2b <= 1.0;
    if (!(sa && sb)) {
        K01 oa, ob; /* three pieces, K1(z)/r; alpha K1/r for the closed forms */
        k01_far2_big<true, true, true, true>(T, c, r2a, r2b, oa, ob);
        stk_closed(al2, ial2, r2a, oa.ri2, oa.k0, c.a * oa.ak1r, Aa);
        stk_closed(al2, ial2, r2b, ob.ri2, ob.k0, c.a * ob.ak1r, Ab);
    }
    if (sa || sb) {
        if (sa) stk_small(T, c, al2, r2a, Aa);
        if (sb) stk_small(T, c, al2, r2b, Ab);
    }
}

/* stk_far2 for two sources of a panel whose pairs all fall in piece PC of the
   plan's (wave, panel) class table: a fine piece (the closed forms from its
   K0 and K1 fits), -1 (every z <= 2: the fitted smooth parts) or KQ_NP (the
   per-pair selection of stk_far2) */
template <int PC>
__device__ __forceinline__ void stk_far2_pc(FarTab T, const FarConst &c, double qa, double qk, double al2,
                                            double ial2, double r2a, double r2b, double *Aa, double *Ab)
{
    if constexpr (PC < 0) {
        stk_small(T, c, al2, r2a, Aa);
        stk_small(T, c, al2, r2b, Ab);
    } else if constexpr (PC >= KQ_NP) {
        stk_far2(T, c, al2, ial2, r2a, r2b, Aa, Ab);
    } else {
        K01 oa, ob; /* K1(z)/r; alpha K1/r for the closed forms */
        k01_far2_fixed<true, true, PC>(T, c, qa, qk, r2a, r2b, oa, ob);
        stk_closed(al2, ial2, r2a, oa.ri2, oa.k0, c.a * oa.ak1r, Aa);
        stk_closed(al2, ial2, r2b, ob.ri2, ob.k0, c.a * ob.ak1r, Ab);
    }
    (void)qa;
    (void)qk;
}

/* A_k and B_k = A_k'(r)/r of the stresslet (target gradient) for two
   sources of a far tile.  z > 2: B from K0, alpha K1/r and A,
     B1 = (alpha^2 K0/(2 pi) - 4 A1)/r^2, B2 = -(alpha^2 K0 + 2 alpha K1/r)/(pi r^4) - 6 A2/r^2,
     B3 = -(alpha^2 K0/(2 pi) + 2 A3)/r^2;
   z <= 2: B = 2 d A/d(r^2) from the fitted smooth parts (d/dw = d/(4 dq),
   w = z^2) and the explicit terms of A2. */
__device__ __forceinline__ void stk_closed_ab(double al2, double ial2, double r2, double ri2, double k0, double ak1r,
                                              double *A, double *B)
{
    stk_closed(al2, ial2, r2, ri2, k0, ak1r, A);
    const double ak0 = al2 * k0;
    B[0] = ri2 * fma(INV_2PI, ak0, -4.0 * A[0]);
    B[1] = -ri2 * fma(ri2 * (1.0 / PI), fma(2.0, ak1r, ak0), 6.0 * A[1]);
    B[2] = -ri2 * fma(INV_2PI, ak0, 2.0 * A[2]);
}

__device__ __forceinline__ void stk_small_ab(FarTab T, const FarConst &c, double al2, double r2, double *A, double *B)
{
    const double q = c.a2q * r2;
    const double lz = fma(0.5, lean_log01(T, q), LN2);
    const double ri2 = lean_rcp(r2);
    const double sc[3] = {al2, al2 * al2, al2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double dS, dL;
        const double tS = hornercd<14>(T->stk[k], q, dS);
        const double tL = hornercd<14>(T->stk[3 + k], q, dL);
        A[k] = sc[k] * fma(tL, lz, tS);
        B[k] = sc[k] * fma(0.5 * al2, fma(dL, lz, dS), tL * ri2);
    }
    const double ri4 = ri2 * ri2;
    A[1] += ri2 * fma(al2, 1.0 / (8.0 * PI), -ri2 * (1.0 / PI));
    B[1] += ri4 * fma(al2, -1.0 / (4.0 * PI), 4.0 * ri2 * (1.0 / PI));
}

__device__ __forceinline__ void stk_far2_ab(FarTab T, const FarConst &c, double al2, double ial2, double r2a,
                                            double r2b, double *Aa, double *Ba, double *Ab, double *Bb)
{
    const bool sa = c.a2q * r2a <= 1.0, sb = c.a2q * r2b <= 1.0;
    if (!(sa && sb)) {
        K01 oa, ob; /* three pieces, K1(z)/r; alpha K1/r for the closed forms */
        k01_far2_big<true, true, true, true>(T, c, r2a, r2b, oa, ob);
        stk_closed_ab(al2, ial2, r2a, oa.ri2, oa.k0, c.a * oa.ak1r, Aa, Ba);
        stk_closed_ab(al2, ial2, r2b, ob.ri2, ob.k0, c.a * ob.ak1r, Ab, Bb);
    }
    if (sa || sb) {
        if (sa) stk_small_ab(T, c, al2, r2a, Aa, Ba);
        if (sb) stk_small_ab(T, c, al2, r2b, Ab, Bb);
    }
}

/* stk_far2_ab for two sources of a panel in piece PC of the class table (as
   stk_far2_pc) */
template <int PC>
__device__ __forceinline__ void stk_far2_ab_pc(FarTab T, const FarConst &c, double qa, double qk, double al2,
                                               double ial2, double r2a, double r2b, double *Aa, double *Ba,
                                               double *Ab, double *Bb)
{
    if constexpr (PC < 0) {
        stk_small_ab(T, c, al2, r2a, Aa, Ba);
        stk_small_ab(T, c, al2, r2b, Ab, Bb);
    } else if constexpr (PC >= KQ_NP) {
        stk_far2_ab(T, c, al2, ial2, r2a, r2b, Aa, Ba, Ab, Bb);
    } else {
        K01 oa, ob;
        k01_far2_fixed<true, true, PC>(T, c, qa, qk, r2a, r2b, oa, ob);
        stk_closed_ab(al2, ial2, r2a, oa.ri2, oa.k0, c.a * oa.ak1r, Aa, Ba);
        stk_closed_ab(al2, ial2, r2b, ob.ri2, ob.k0, c.a * ob.ak1r, Ab, Bb);
    }
    (void)qa;
    (void)qk;
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

/* The FP32 fits of the fine pieces (coefficient counts of KQF0 / KQF1) for
   the mixed-precision far field on the plan's (wave, panel) class table:
   PC a fine piece (z > 2: e^{-z} z^{-1/2} times the piece's fit in
   v = (2u - ulo - uhi)/(uhi - ulo), u = 4/z - 1), -1 (every pair z <= 2: the
   series form), KQ_NP (the per-pair choice of k01_fp32). */
constexpr int KQF_N0[KQ_NP] = {5, 5, 4, 4, 4, 3, 3, 3, 6, 6, 5, 4, 4, 4, 4};
constexpr int KQF_N1[KQ_NP] = {5, 4, 4, 4, 4, 4, 3, 3, 5, 5, 5, 5, 4, 4, 3};

constexpr bool kqf_counts_ok()
{
    for (int k = 0; k < KQ_NP; ++k) {
        if (KQF0[k][KQF_N0[k] - 1] == 0.0f || KQF1[k][KQF_N1[k] - 1] == 0.0f) return false;
        for (int i = KQF_N0[k]; i < 6; ++i)
            if (KQF0[k][i] != 0.0f) return false;
        for (int i = KQF_N1[k]; i < 6; ++i)
            if (KQF1[k][i] != 0.0f) return false;
    }
    return true;
}
static_assert(kqf_counts_ok(), "KQF_N0 / KQF_N1 differ from the generated FP32 fine pieces");

template <int N>
__device__ __forceinline__ float horner_f(const float *c, float x)
{
    float v = c[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) v = fmaf(v, x, c[i]);
    return v;
}

template <bool SLP, bool DLP, int PC>
__device__ __forceinline__ K01f k01_fp32_pc(float r2, float a, float a2q, float a4)
{
    if constexpr (PC < 0 || PC >= KQ_NP) {
        if constexpr (PC < 0) {
            K01f o{0.0f, 0.0f};
            const float q = a2q * r2;
            const float lq = __logf(q);
            if (SLP) o.k0 = fmaf(-0.5f * lq, horner(KSF_I0, q), horner(KSF_R0, q));
            if (DLP) {
                const float t = fmaf(0.5f * lq, horner(KSF_I1Z, q), -0.25f * horner(KSF_R1, q));
                o.ak1r = fmaf(4.0f * a2q, t, __frcp_rn(r2));
            }
            return o;
        } else {
            return k01_fp32<SLP, DLP>(r2, a, a2q, a4);
        }
    } else {
        /* v = (4/alpha) w ri + b, w = 2/(uhi - ulo), b = -(2 + ulo + uhi)/(uhi - ulo) */
        constexpr float w = (float)(2.0 / (KQ_UHI[PC] - KQ_ULO[PC]));
        constexpr float b = (float)((-2.0 - KQ_ULO[PC] - KQ_UHI[PC]) / (KQ_UHI[PC] - KQ_ULO[PC]));
        K01f o{0.0f, 0.0f};
        const float ri = __frsqrt_rn(r2);
        const float z = a * (r2 * ri);
        const float v = fmaf(a4 * w, ri, b);
        const float e = __expf(-z) * __frsqrt_rn(z);
        if (SLP) o.k0 = e * horner_f<KQF_N0[PC]>(KQF0[PC], v);
        if (DLP) o.ak1r = a * e * horner_f<KQF_N1[PC]>(KQF1[PC], v) * ri;
        return o;
    }
}

/* ---------------------------------------------------------------------- */
/* Kernel-split pieces (paper Sec. 4.1, App. C), any moderate z >= 0.       */
/*   I0(z), K0S = K0 + I0 log z, I1z = I1(z)/z, K1Sz = (K1 - I1 log z - 1/z)/z */
/* Power series in q = z^2/4 with psi(n+1) = -gamma + sum_{k<=n} 1/k.        */
/* ---------------------------------------------------------------------- */
struct Split {
    double i0, k0s, i1z, k1sz;
};

/* With the target gradient the double layer also needs d/dq of I1z and K1Sz
   (q = z^2/4): i1z_q = (1/2) sum_{n>=1} n q^(n-1)/(n!(n+1)!), and the same
   with the psi weights for K1Sz; the n-th derivative coefficient is the
   (n-1)-th value coefficient divided by n+1. */
struct SplitG {
    Split s;
    double i1z_q, k1sz_q;
};

template <bool GRAD>
__host__ __device__ inline void split_series(double z, Split &s, double *i1z_q, double *k1sz_q)
{
    const double q = 0.25 * z * z;
    double a = 1.0, b = 1.0; /* q^n/(n!)^2 and q^n/(n!(n+1)!) */
    double p1 = -EULER_G, p2 = 1.0 - EULER_G;
    double si0 = 0.0, si1 = 0.0, sr0 = 0.0, sr1 = 0.0, sd1 = 0.0, sdr1 = 0.0;
    for (int n = 0; n < 80; ++n) {
        si0 += a;
        si1 += b;
        sr0 = fma(p1, a, sr0);
        sr1 = fma(p1 + p2, b, sr1);
        const double n1 = n + 1.0;
        if (GRAD) {
            /* term n+1 of the derivative series: q^n/(n!(n+2)!) = b/(n+2) with
               the psi weights of index n+1 */
            const double c = b / (n1 + 1.0);
            sd1 += c;
            sdr1 = fma(p1 + p2 + 1.0 / n1 + 1.0 / (n1 + 1.0), c, sdr1);
        }
        if (a <= 1e-18 * si0 && b <= 1e-18 * si1) break;
        a *= q / (n1 * n1);
        b *= q / (n1 * (n1 + 1.0));
        p1 += 1.0 / n1;
        p2 += 1.0 / (n1 + 1.0);
    }
    s.i0 = si0;
    s.i1z = 0.5 * si1;
    /* K0 = -log(z/2) I0 + R0  =>  K0 + I0 log z = I0 log 2 + R0 */
    s.k0s = fma(LN2, si0, sr0);
    /* K1 = 1/z + log(z/2) I1 - (z/4) R1  =>  (K1 - I1 log z - 1/z)/z = -log2 I1/z - R1/4 */
    s.k1sz = fma(-LN2, s.i1z, -0.25 * sr1);
    if (GRAD) {
        *i1z_q = 0.5 * sd1;
        *k1sz_q = fma(-LN2, *i1z_q, -0.25 * sdr1);
    }
}

__host__ __device__ inline Split split_k01(double z)
{
    Split s;
    split_series<false>(z, s, nullptr, nullptr);
    return s;
}

__host__ __device__ inline SplitG split_k01_grad(double z)
{
    SplitG g;
    split_series<true>(z, g.s, &g.i1z_q, &g.k1sz_q);
    return g;
}

/* ---------------------------------------------------------------------- */
/* Stresslet functions of the modified-Stokes double layer (App. B, C).     */
/*   T1 = -(2 z^2 K0 + (z^2 + 4) z K1 - 4)/(2 pi z^4)                         */
/*   T2 = (4 z^2 K0 + (z^2 + 8) z K1 - 8)/(pi z^6)                            */
/*   T3 = (z K1 - 1)/(2 pi z^2)                                              */
/* and their kernel split (Sec. 4.1)                                          */
/*   T1 = T1S + T1L log z,  T3 = T3S + T3L log z,                             */
/*   T2 = T2S + T2L log z + 1/(8 pi z^2) - 1/(pi z^4),                         */
/* the smooth parts from the power series of App. C with the log z factor     */
/* taken out of its coefficients:                                             */
/*   k0(n) = (psi(n+1) + log 2 - log z) a_n,  a_n = 1/(4^n n!^2),              */
/*   k1(n) = (2 log z - 2 log 2 - psi(n+1) - psi(n+2)) b_n,                    */
/*   b_n = 1/(4^(n+1) n! (n+1)!),                                             */
/*   T1 = -(1/2pi) sum_{n>=1} (2 k0(n) + 4 k1(n) + k1(n-1)) z^(2n-2),           */
/*   T2 - (explicit) = (1/pi) sum_{n>=2} (4 k0(n) + 8 k1(n) + k1(n-1)) z^(2n-4), */
/*   T3 = (1/2pi) sum_{n>=0} k1(n) z^(2n).                                    */
/* ---------------------------------------------------------------------- */
struct StkSplit {
    double s[3], l[3];   /* T1S, T2S, T3S and T1L, T2L, T3L                    */
    double ds[3], dl[3]; /* their derivatives with respect to w = z^2 (GRAD) */
};

template <bool GRAD>
__host__ __device__ inline StkSplit stresslet_split_t(double z)
{
    const double w = z * z;
    double a = 1.0, b = 0.25;                       /* a_n, b_n */
    double psi = -EULER_G, psi1 = 1.0 - EULER_G;    /* psi(n+1), psi(n+2) */
    double pw = 1.0, pw1 = 0.0, pw2 = 0.0, pw3 = 0.0; /* w^n, w^(n-1), w^(n-2), w^(n-3) */
    double k1s_prev = 0.0, k1l_prev = 0.0;
    double t1s = 0.0, t1l = 0.0, t2s = 0.0, t2l = 0.0, t3s = 0.0, t3l = 0.0;
    double d1s = 0.0, d1l = 0.0, d2s = 0.0, d2l = 0.0, d3s = 0.0, d3l = 0.0;
    for (int n = 0; n < 64; ++n) {
        const double k0s = (psi + LN2) * a, k0l = -a;
        const double k1s = -(2.0 * LN2 + psi + psi1) * b, k1l = 2.0 * b;
        const double e3s = k1s * pw, e3l = k1l * pw;
        t3s += e3s;
        t3l += e3l;
        if (GRAD && n >= 1) {
            d3s += n * k1s * pw1;
            d3l += n * k1l * pw1;
        }
        double e1 = 0.0, e2 = 0.0;
        if (n >= 1) {
            const double c1s = 2.0 * k0s + 4.0 * k1s + k1s_prev, c1l = 2.0 * k0l + 4.0 * k1l + k1l_prev;
            e1 = c1s * pw1;
            t1s += e1;
            t1l += c1l * pw1;
            if (GRAD && n >= 2) {
                d1s += (n - 1.0) * c1s * pw2;
                d1l += (n - 1.0) * c1l * pw2;
            }
        }
        if (n >= 2) {
            const double c2s = 4.0 * k0s + 8.0 * k1s + k1s_prev, c2l = 4.0 * k0l + 8.0 * k1l + k1l_prev;
            e2 = c2s * pw2;
            t2s += e2;
            t2l += c2l * pw2;
            if (GRAD && n >= 3) {
                d2s += (n - 2.0) * c2s * pw3;
                d2l += (n - 2.0) * c2l * pw3;
            }
        }
        if (n >= 4 && fabs(e1) <= 1e-18 * fabs(t1s) && fabs(e2) <= 1e-18 * fabs(t2s) &&
            fabs(e3s) <= 1e-18 * fabs(t3s))
            break;
        k1s_prev = k1s;
        k1l_prev = k1l;
        const double n1 = n + 1.0;
        a *= 1.0 / (4.0 * n1 * n1);
        b *= 1.0 / (4.0 * n1 * (n1 + 1.0));
        psi += 1.0 / n1;
        psi1 += 1.0 / (n1 + 1.0);
        pw3 = pw2;
        pw2 = pw1;
        pw1 = pw;
        pw *= w;
    }
    StkSplit o;
    o.s[0] = -INV_2PI * t1s;
    o.l[0] = -INV_2PI * t1l;
    o.s[1] = t2s / PI;
    o.l[1] = t2l / PI;
    o.s[2] = INV_2PI * t3s;
    o.l[2] = INV_2PI * t3l;
    o.ds[0] = -INV_2PI * d1s;
    o.dl[0] = -INV_2PI * d1l;
    o.ds[1] = d2s / PI;
    o.dl[1] = d2l / PI;
    o.ds[2] = INV_2PI * d3s;
    o.dl[2] = INV_2PI * d3l;
    return o;
}

__host__ __device__ inline StkSplit stresslet_split(double z) { return stresslet_split_t<false>(z); }

/* alpha^2 T1, alpha^4 T2, alpha^2 T3 at a source-target pair with r^2 = r2
   (1/r^2 = ri2) from K0 and alpha K1(alpha r)/r (far-field values): closed
   forms for z > 2, the split series for z <= 2 (the closed forms cancel).
   a2 = alpha^2, ia2 = 1/alpha^2. */
__host__ __device__ inline void stresslet_scaled(double a2, double ia2, double r2, double ri2, double k0, double ak1r,
                                                 double *A)
{
    const double w = a2 * r2; /* z^2 */
    if (w > 4.0) {
        const double zk1 = ak1r * r2; /* z K1 */
        const double ri4 = ri2 * ri2;
        A[0] = (-INV_2PI * ia2) * ri4 * fma(2.0 * w, k0, fma(w + 4.0, zk1, -4.0));
        A[1] = (ia2 / PI) * ri4 * ri2 * fma(4.0 * w, k0, fma(w + 8.0, zk1, -8.0));
        A[2] = INV_2PI * ri2 * (zk1 - 1.0);
        return;
    }
    const StkSplit t = stresslet_split(sqrt(w));
    const double lz = 0.5 * log(w);
    A[0] = a2 * fma(t.l[0], lz, t.s[0]);
    A[1] = a2 * a2 * fma(t.l[1], lz, t.s[1]) + a2 * ri2 / (8.0 * PI) - ri2 * ri2 / PI;
    A[2] = a2 * fma(t.l[2], lz, t.s[2]);
}

/* Near-field values of A_k = a_k T_k(alpha r) and B_k = A_k'(r)/r (the radial
   derivative over r), a = (alpha^2, alpha^4, alpha^2), for the target gradient:
   z > 2 from K0, alpha K1/r:
     B1 = (alpha^2 K0/(2 pi) - 4 A1)/r^2,
     B2 = -(alpha^2 K0 + 2 alpha K1/r)/(pi r^4) - 6 A2/r^2,
     B3 = -(alpha^2 K0/(2 pi) + 2 A3)/r^2
   (from T1' = K0/(2 pi z) - 4 T1/z, T2' = -(z K0 + 2 K1)/(pi z^4) - 6 T2/z,
   T3' = -K0/(2 pi z) - 2 T3/z); z <= 2 from the split series and its
   derivative in w = z^2 (B = 2 dA/d(r^2)). */
__host__ __device__ inline void stk_AB(double alpha, double r2, double k0, double ak1r, double *A, double *B)
{
    const double a2 = alpha * alpha, w = a2 * r2, ri2 = 1.0 / r2;
    if (w > 4.0) {
        stresslet_scaled(a2, 1.0 / a2, r2, ri2, k0, ak1r, A);
        B[0] = ri2 * fma(a2 * INV_2PI, k0, -4.0 * A[0]);
        B[1] = -ri2 * ri2 / PI * fma(a2, k0, 2.0 * ak1r) - 6.0 * A[1] * ri2;
        B[2] = -ri2 * fma(a2 * INV_2PI, k0, 2.0 * A[2]);
        return;
    }
    const StkSplit t = stresslet_split_t<true>(sqrt(w));
    const double lz = 0.5 * log(w);
    const double sc[3] = {a2, a2 * a2, a2};
    for (int k = 0; k < 3; ++k) {
        A[k] = sc[k] * fma(t.l[k], lz, t.s[k]);
        /* d/d(r^2) = a2 d/dw;  d(TL log z)/dw = dTL log z + TL/(2w) */
        B[k] = 2.0 * sc[k] * a2 * (fma(t.dl[k], lz, t.ds[k]) + 0.5 * t.l[k] / w);
    }
    A[1] += a2 * ri2 / (8.0 * PI) - ri2 * ri2 / PI;
    B[1] += -a2 * ri2 * ri2 / (4.0 * PI) + 4.0 * ri2 * ri2 * ri2 / PI;
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

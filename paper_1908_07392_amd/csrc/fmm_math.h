/* Special-function helpers of the FMM (host and device): scaled modified
   Bessel functions I_n(x)/s^n, the local-expansion sum at a point, and the
   translation-table rows (outgoing K_n and regular I_n functions of a shift).
   See fmm.h for the expansions they serve. */
#pragma once

namespace mhlp {

/* I_0 by its power series sum_k (x^2/4)^k / (k!)^2 (all terms positive). */
__host__ __device__ inline double fmm_i0_series(double x)
{
    const double t = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= t / ((double)k * (double)k);
        sum += term;
        if (term < 1e-18 * sum && k > 0.5 * x) break;
    }
    return sum;
}

/* Start of the backward sweeps below: far enough above nmax that the minimal
   solution I_n of the recurrence dominates to rounding at nmax. */
__host__ __device__ inline int fmm_ntop(int nmax, double x) { return nmax + 20 + (int)(x + 10.0 * sqrt(x + 1.0)); }

/* I~_n = I_n(x) / s^n for n = 0..nmax (x >= 0, 0 < s <= 1) into o[n * stride].
   The scaled recurrence I~_{n-1} = (2 n s/x) I~_n + s^2 I~_{n+1} (from
   I_{n-1} - I_{n+1} = (2n/x) I_n; backward it is stable for I_n) gives the ratios
   r_n = I~_n / I~_{n-1} = 1/(2 n s/x + s^2 r_{n+1}) by a backward continued
   fraction (bounded, no overflow for small x/s); then I~_n = I~_{n-1} r_n from
   I~_0 = I_0(x). */
__host__ __device__ inline void fmm_iscaled_store(double x, double s, int nmax, double *o, int stride)
{
    if (!(x > 0.0)) {
        o[0] = 1.0;
        for (int n = 1; n <= nmax; ++n) o[n * stride] = 0.0;
        return;
    }
    const double c = 2.0 * s / x, s2 = s * s;
    double r = 0.0;
    for (int n = fmm_ntop(nmax, x); n > nmax; --n) r = 1.0 / fma(c, (double)n, s2 * r);
    for (int n = nmax; n >= 1; --n) {
        r = 1.0 / fma(c, (double)n, s2 * r);
        o[n * stride] = r;
    }
    double v = fmm_i0_series(x);
    o[0] = v;
    for (int n = 1; n <= nmax; ++n) {
        v *= o[n * stride];
        o[n * stride] = v;
    }
}

__host__ __device__ inline cplx cpow_unit(cplx u, int k)
{
    cplx r = mk(1.0, 0.0);
    const cplx b = k >= 0 ? u : conj(u);
    for (int j = 0; j < (k >= 0 ? k : -k); ++j) r = r * b;
    return r;
}

struct FmmRow {
    double bx, by; /* the shift vector (M2L: c_t - c_s; shifts: c_child - c_parent) */
    double s;      /* scale of the row's functions */
    int64_t off;   /* output offset (cplx) */
    int kind;      /* 0: O~_k, 1: R~_k, k = -2p..p */
};

/* one table row: tab[off + j], j = 0..3p, holds O~_k or R~_k of the shift at
   order k = j - 2p; mag: scratch of 2p + 1 doubles */
__host__ __device__ inline void fmm_table_row(const FmmRow &R, int p, double alpha, cplx *tab, double *mag)
{
    const int nmax = 2 * p;
    const double rr = sqrt(R.bx * R.bx + R.by * R.by);
    const double x = alpha * rr;
    const cplx u = rr > 0.0 ? mk(R.bx / rr, R.by / rr) : mk(1.0, 0.0);
    if (R.kind == 0) {
        /* K~_j = K_j(x) s^j by the upward recurrence (stable for K_n) */
        const K01 o = k01_fp64<true, true>(rr * rr, alpha, 0.25 * alpha * alpha, 4.0 / alpha);
        double km = o.k0, k = R.s * o.ak1r * rr / alpha;
        mag[0] = km;
        if (nmax >= 1) mag[1] = k;
        const double c = 2.0 * R.s / x, s2 = R.s * R.s;
        for (int j = 1; j < nmax; ++j) {
            const double kp = fma(c * j, k, s2 * km);
            km = k;
            k = kp;
            mag[j + 1] = k;
        }
    } else {
        fmm_iscaled_store(x, R.s, nmax, mag, 1);
    }
    for (int j = 0; j <= 3 * p; ++j) {
        const int kk = j - 2 * p;
        const double m = mag[kk >= 0 ? kk : -kk];
        const cplx e = cpow_unit(u, kk);
        tab[R.off + j] = mk(m * e.re, m * e.im);
    }
}

/* Local expansions at a point: acc_f = Re(L~f_0 I~_0) + 2 Re sum_{n=1..p} L~f_n I~_n u^n
   for the fields f whose flag is set (x = alpha |z - c|, u = (z - c)/|z - c|).
   One unnormalised backward sweep of the recurrence (rescaled by 1e-200 when it
   grows past 1e200) accumulates every field; the result is scaled by I_0(x)/v_0. */
template <bool F0, bool F1>
__host__ __device__ inline void fmm_l2p(const cplx *L0, const cplx *L1, int p, double x, double s, cplx u, double *acc)
{
    acc[0] = acc[1] = 0.0;
    if (!(x > 0.0)) {
        if (F0) acc[0] = L0[0].re;
        if (F1) acc[1] = L1[0].re;
        return;
    }
    const double c = 2.0 * s / x, s2 = s * s;
    double vp = 0.0, v = 1.0;
    for (int n = fmm_ntop(p, x); n > p; --n) {
        const double vm = fma(c * n, v, s2 * vp);
        vp = v;
        v = vm;
        if (v > 1e200) {
            v *= 1e-200;
            vp *= 1e-200;
        }
    }
    cplx e = cpow_unit(u, p);
    const cplx ub = conj(u);
    double a0 = 0.0, a1 = 0.0;
    for (int n = p; n >= 0; --n) {
        const double w = n == 0 ? v : 2.0 * v;
        if (F0) a0 = fma(w, (L0[n] * e).re, a0);
        if (F1) a1 = fma(w, (L1[n] * e).re, a1);
        if (n == 0) break;
        const double vm = fma(c * n, v, s2 * vp);
        vp = v;
        v = vm;
        e = e * ub;
        if (v > 1e200) {
            v *= 1e-200;
            vp *= 1e-200;
            a0 *= 1e-200;
            a1 *= 1e-200;
        }
    }
    const double f = fmm_i0_series(x) / v;
    acc[0] = a0 * f;
    acc[1] = a1 * f;
}

} // namespace mhlp

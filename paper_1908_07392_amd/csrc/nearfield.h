/*
 * nearfield.h -- near-field correction weights for one (target, panel) pair.
 *
 * Follows the paper's Sec. 4 ("Quadrature details"): the kernel is split into
 * a smooth part, a smooth function times log|r| and (double layer only) a
 * smooth function times the Laplace/Cauchy kernel (x-y).n/|r|^2 (Sec. 4.1);
 * the singular parts are integrated by interpolatory quadrature with exact
 * moments (Sec. 4.3); targets are classified by the Bernstein radius of
 * their preimage, with 16-point Gauss-Legendre for rho >= 3.5, a 32-point
 * upsampled rule for sqrt(3.5) <= rho < 3.5 and kernel split on the upsampled
 * panel below (Sec. 4.5.3); on-surface targets use kernel split for the log
 * part on the 16 nodes with the curvature limit for the Cauchy part (Sec.
 * 4.2, 4.5.2); panels with alpha h > 4.5 are subdivided towards the target
 * and the subpanel weights folded back to the 16 nodes by interpolation
 * (Sec. 4.5.4).
 *
 * Difference from the paper's formulation: the interpolation variable is the
 * panel parameter t (a straight segment) rather than the complex coordinate
 * tau.  With t* the complex preimage of the target, tau(t) - z =
 * (t - t*) Q(t) where Q is the divided difference of the panel polynomial, so
 *    log|tau - z|          = log|t - t*| + log|Q(t)|,
 *    dtau / (tau - z)      = [tau'(t)/Q(t)] dt / (t - t*),
 * and the moments int t^k log(t - t*) dt, int t^k/(t - t*) dt are taken over
 * [-1, 1], where the principal logarithm is continuous whenever t* is off the
 * segment (no winding corrections).
 *
 * All weights multiply the density at the panel's 16 nodes; they REPLACE the
 * panel's direct 16-point contribution (the far-field kernels skip listed
 * panels).  Arithmetic is FP64 throughout.
 */
#pragma once
#include "yukawa.h"

namespace mhlp {

struct NearParams {
    double rho_direct; /* 3.5: 16-point rule accurate at or beyond        */
    double rho_split;  /* sqrt(3.5): kernel split below                    */
    double ah_max;     /* 4.5: largest alpha h a split panel may have      */
    double far_exp;    /* 40: a subpanel with alpha*dist beyond is direct   */
};

/* p(t), p'(t), p''(t) of the Legendre series sum_m a_m P_m(t), complex t. */
__host__ __device__ inline void leg_eval(const cplx *a, cplx t, cplx &p, cplx &dp, cplx *d2p = nullptr)
{
    cplx P0 = mk(1.0, 0.0), P1 = t;
    cplx D0 = mk(0.0, 0.0), D1 = mk(1.0, 0.0);
    cplx E0 = mk(0.0, 0.0), E1 = mk(0.0, 0.0);
    p = a[0] + a[1] * P1;
    dp = a[1];
    cplx d2 = mk(0.0, 0.0);
    for (int m = 1; m < 15; ++m) {
        const double c1 = (2.0 * m + 1.0) / (m + 1.0), c0 = m / (m + 1.0);
        cplx P2 = c1 * (t * P1) - c0 * P0;
        cplx D2 = D0 + (2.0 * m + 1.0) * P1;
        cplx E2 = E0 + (2.0 * m + 1.0) * D1;
        p = p + a[m + 1] * P2;
        dp = dp + a[m + 1] * D2;
        d2 = d2 + a[m + 1] * E2;
        P0 = P1; P1 = P2;
        D0 = D1; D1 = D2;
        E0 = E1; E1 = E2;
    }
    if (d2p) *d2p = d2;
}

/* Divided difference (p(t) - p(s)) / (t - s) of the Legendre series, computed
   without cancellation: with D_m = (P_m(t) - P_m(s))/(t - s),
   D_0 = 0, D_1 = 1, (m+1) D_{m+1} = (2m+1) (P_m(t) + s D_m) - m D_{m-1}.    */
__host__ __device__ inline cplx leg_divdiff(const cplx *a, cplx t, cplx s)
{
    cplx P0 = mk(1.0, 0.0), P1 = t;
    cplx D0 = mk(0.0, 0.0), D1 = mk(1.0, 0.0);
    cplx acc = a[1];
    for (int m = 1; m < 15; ++m) {
        const double c1 = (2.0 * m + 1.0) / (m + 1.0), c0 = m / (m + 1.0);
        cplx D2 = c1 * (P1 + s * D1) - c0 * D0;
        cplx P2 = c1 * (t * P1) - c0 * P0;
        acc = acc + a[m + 1] * D2;
        P0 = P1; P1 = P2;
        D0 = D1; D1 = D2;
    }
    return acc;
}

/* First and Hermite second divided differences of the Legendre series,
   Q = p[t, s] and R = p[t, t, s], so that p(t) - p(s) = (t - s) Q and
   p'(t) = Q + (t - s) R, from the Leibniz rule (x f)[t,t,s] = t f[t,t,s] +
   f[t,s] applied to the three-term recurrence:
   (m+1) E_{m+1} = (2m+1) (t E_m + D_m) - m E_{m-1},  E_0 = E_1 = 0.       */
__host__ __device__ inline void leg_divdiff2(const cplx *a, double t, double s, cplx &Q, cplx &R)
{
    double P0 = 1.0, P1 = t, D0 = 0.0, D1 = 1.0, E0 = 0.0, E1 = 0.0;
    Q = a[1];
    R = mk(0.0, 0.0);
    for (int m = 1; m < 15; ++m) {
        const double c1 = (2.0 * m + 1.0) / (m + 1.0), c0 = m / (m + 1.0);
        const double E2 = c1 * (t * E1 + D1) - c0 * E0;
        const double D2 = c1 * (P1 + s * D1) - c0 * D0;
        const double P2 = c1 * (t * P1) - c0 * P0;
        Q = Q + D2 * a[m + 1];
        R = R + E2 * a[m + 1];
        P0 = P1; P1 = P2;
        D0 = D1; D1 = D2;
        E0 = E1; E1 = E2;
    }
}

/* Newton iteration for the complex preimage t* with p(t*) = z.  The attainable
   accuracy of t* is about eps |z| / |p'|, so convergence is declared once the
   step is below 1e-12 and two more steps polish t* to that floor.  Returns
   false only if the iteration leaves the region |t| < 1000 or never reaches
   the 1e-12 step size. */
__host__ __device__ inline bool preimage(const cplx *a, cplx z, cplx t0, cplx &t)
{
    t = t0;
    int polish = -1;
    for (int it = 0; it < 60; ++it) {
        cplx p, dp;
        leg_eval(a, t, p, dp);
        const cplx dt = (p - z) / dp;
        t = t - dt;
        if (!(cabs2(t) < 1e6)) return false;
        if (polish >= 0) {
            if (++polish == 2) return true;
        } else if (cabs2(dt) < 1e-24 * (1.0 + cabs2(t))) {
            polish = 0;
        }
    }
    return polish >= 0;
}

/* Bernstein radius rho(t) = |t +- sqrt(t^2 - 1)| >= 1. */
__host__ __device__ inline double bernstein_rho(cplx t)
{
    cplx w = csqrt(t * t - mk(1.0, 0.0));
    double r1 = cabs(t + w), r2 = cabs(t - w);
    return r1 > r2 ? r1 : r2;
}

/* Legendre moments over the segment [-1, 1] with pole / branch point s off
   the segment (or real outside it):
     MC[m] = int P_m(t) / (t - s) dt,        m = 0..N
     ML[m] = int P_m(t) log(t - s) dt,       m = 0..N-1
   MC[m] = -2 Q_m(s) is the minimal solution of the Legendre recurrence
   (m+1) M_{m+1} = (2m+1) s M_m - m M_{m-1} (m >= 1, M_1 = s M_0 + 2):
   forward recursion close to the segment (Bernstein radius < 1.05, where the
   error growth rho^(2m) is mild), Miller's backward recursion otherwise,
   normalised by M_0 = log((1 - s)/(-1 - s)).  Log moments by parts with the
   antiderivative (P_{m+1} - P_{m-1})/(2m+1) of P_m, which vanishes at +-1:
     ML[0] = (1-s) log(1-s) - (-1-s) log(-1-s) - 2,
     ML[m] = -(MC[m+1] - MC[m-1]) / (2m+1).
   The principal logarithm is continuous along the segment for such s.       */
template <int N>
__host__ __device__ inline void legendre_moments(cplx s, double rho, cplx *MC, cplx *ML)
{
    const cplx la = clog(mk(-1.0, 0.0) - s);
    const cplx lb = clog(mk(1.0, 0.0) - s);
    const cplx m0 = lb - la;
    if (rho < 1.05) {
        MC[0] = m0;
        MC[1] = s * m0 + mk(2.0, 0.0);
        for (int m = 1; m < N; ++m)
            MC[m + 1] = (1.0 / (m + 1.0)) * ((2.0 * m + 1.0) * (s * MC[m]) - (double)m * MC[m - 1]);
    } else {
        int K = N + 1 + (int)ceil(40.0 / log(rho * rho));
        if (K > 4000) K = 4000;
        cplx y1 = mk(0.0, 0.0), y0 = mk(1e-30, 0.0); /* y_{m+1}, y_m */
        for (int m = K; m >= 1; --m) {
            cplx ym1 = (1.0 / m) * ((2.0 * m + 1.0) * (s * y0) - (m + 1.0) * y1);
            y1 = y0;
            y0 = ym1;
            if (m - 1 <= N) MC[m - 1] = y0;
            if (cabs2(y0) > 1e200) { /* rescale the running solution */
                y0 = 1e-100 * y0;
                y1 = 1e-100 * y1;
                for (int j = m - 1; j <= N && j <= K; ++j) MC[j] = 1e-100 * MC[j];
            }
        }
        const cplx f = m0 / MC[0];
        for (int m = 0; m <= N; ++m) MC[m] = f * MC[m];
    }
    ML[0] = (mk(1.0, 0.0) - s) * lb - (mk(-1.0, 0.0) - s) * la - mk(2.0, 0.0);
    for (int m = 1; m < N; ++m) ML[m] = (-1.0 / (2.0 * m + 1.0)) * (MC[m + 1] - MC[m - 1]);
}

/* Same for real s strictly inside (-1, 1) (target on the curve inside the
   rule's interval): principal-value Cauchy moments and int P_m log|t - s| dt.
   Forward recursion is stable there (both solutions oscillate).            */
template <int N>
__host__ __device__ inline void legendre_moments_real(double s, double *MC, double *ML)
{
    const double l1 = log(1.0 - s), l2 = log(1.0 + s);
    MC[0] = l1 - l2;
    MC[1] = s * MC[0] + 2.0;
    for (int m = 1; m < N; ++m) MC[m + 1] = ((2.0 * m + 1.0) * s * MC[m] - m * MC[m - 1]) / (m + 1.0);
    ML[0] = (1.0 - s) * l1 + (1.0 + s) * l2 - 2.0;
    for (int m = 1; m < N; ++m) ML[m] = -(MC[m + 1] - MC[m - 1]) / (2.0 * m + 1.0);
}

/* Node weights of the N-point Gauss-Legendre rule reproducing the moments
   exactly for polynomials of degree < N: w_k = sum_m lambda_k (2m+1)/2
   P_m(t_k) M_m (discrete orthogonality of the Legendre polynomials). */
template <int N, typename T>
__host__ __device__ inline void moments_to_weights(const double *legw, const T *M, T *w)
{
    for (int k = 0; k < N; ++k) {
        T acc = M[0] * legw[k * N];
        for (int m = 1; m < N; ++m) acc = acc + M[m] * legw[k * N + m];
        w[k] = acc;
    }
}

/* Lagrange basis of the 16 Gauss-Legendre nodes at real t (barycentric). */
__host__ __device__ inline void lagrange16(double t, double *l)
{
    double s = 0.0;
    for (int j = 0; j < 16; ++j) {
        double d = t - GL16_T[j];
        if (d == 0.0) {
            for (int k = 0; k < 16; ++k) l[k] = (k == j) ? 1.0 : 0.0;
            return;
        }
        l[j] = BARY16[j] / d;
        s += l[j];
    }
    const double is = 1.0 / s;
    for (int j = 0; j < 16; ++j) l[j] *= is;
}

/* Per-node kernel pieces for the rule on one (sub)panel. */
struct NodeGeo {
    cplx tau, dtau; /* position, derivative w.r.t. the local parameter */
    double w;       /* quadrature weight |dtau| lambda                 */
};

__host__ __device__ inline double xmy_dot_n(cplx z, const NodeGeo &g)
{
    /* (x - y).n with n = i dtau/|dtau|:  -(Re(conj(tau - z) * i dtau))/|dtau| */
    cplx d = g.tau - z;
    cplx in = mk(-g.dtau.im, g.dtau.re);
    return -(d.re * in.re + d.im * in.im) / cabs(g.dtau);
}

/* Direct (plain quadrature) weights at one node; returns SLP and DLP weights. */
__host__ __device__ inline void direct_node(cplx z, const NodeGeo &g, double alpha, double &ws, double &wd)
{
    const double r2 = cabs2(g.tau - z);
    const K01 o = k01_fp64<true, true>(r2, alpha, 0.25 * alpha * alpha, 4.0 / alpha);
    ws = INV_2PI * o.k0 * g.w;
    wd = INV_2PI * o.ak1r * xmy_dot_n(z, g) * g.w;
}

/* Fold node weights of a rule with NQ nodes on [ta, tb] of the parent panel
   back to the parent's 16 nodes. */
template <int NQ>
__host__ __device__ inline void fold_add(const double *tq, double ta, double tb, const double *WS, const double *WD,
                                         double *Ws, double *Wd)
{
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    for (int k = 0; k < NQ; ++k) {
        double l[16];
        lagrange16(mid + half * tq[k], l);
        for (int j = 0; j < 16; ++j) {
            Ws[j] = fma(l[j], WS[k], Ws[j]);
            Wd[j] = fma(l[j], WD[k], Wd[j]);
        }
    }
}

/* Geometry of the rule with NQ nodes on [ta, tb] of the parent panel. */
template <int NQ>
__host__ __device__ inline void rule_geo(const cplx *a, const double *tq, const double *wq, double ta, double tb,
                                         NodeGeo *g)
{
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    for (int k = 0; k < NQ; ++k) {
        cplx p, dp;
        leg_eval(a, mk(mid + half * tq[k], 0.0), p, dp);
        g[k].tau = p;
        g[k].dtau = half * dp;
        g[k].w = wq[k] * cabs(g[k].dtau);
    }
}

/* Plain NQ-point rule on [ta, tb], folded into the 16 weights. */
template <int NQ>
__host__ __device__ inline void leaf_direct(const cplx *a, const double *tq, const double *wq, double ta, double tb,
                                            cplx z, double alpha, double *Ws, double *Wd)
{
    NodeGeo g[NQ];
    double WS[NQ], WD[NQ];
    rule_geo<NQ>(a, tq, wq, ta, tb, g);
    for (int k = 0; k < NQ; ++k) direct_node(z, g[k], alpha, WS[k], WD[k]);
    fold_add<NQ>(tq, ta, tb, WS, WD, Ws, Wd);
}

/* Kernel split on the 32-point upsampled rule of [ta, tb] for a target with
   parent preimage tstar (complex, off the segment or on the real axis outside
   it). */
__host__ __device__ inline void leaf_split32(const cplx *a, double ta, double tb, cplx z, cplx tstar, double alpha,
                                             double *Ws, double *Wd)
{
    constexpr int NQ = 32;
    NodeGeo g[NQ];
    double WS[NQ], WD[NQ];
    rule_geo<NQ>(a, GL32_T, GL32_W, ta, tb, g);
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    cplx MC[NQ + 1], ML[NQ], pc[NQ], pl[NQ];
    legendre_moments<NQ>(ss, bernstein_rho(ss), MC, ML);
    moments_to_weights<NQ>(LEGW32, MC, pc); /* Cauchy weights */
    moments_to_weights<NQ>(LEGW32, ML, pl); /* log weights    */
    const double la = log(alpha);
    const double a2 = alpha * alpha;
    for (int k = 0; k < NQ; ++k) {
        const cplx tk = mk(mid + half * GL32_T[k], 0.0);
        const cplx Q = half * leg_divdiff(a, tk, tstar); /* (tau - z)/(s - s*) */
        const double sp_ = cabs(g[k].dtau);
        const double logw = fma(sp_, pl[k].re, g[k].w * log(cabs(Q)));
        const double r = cabs(g[k].tau - z);
        const Split s = split_k01(alpha * r);
        const double xn = xmy_dot_n(z, g[k]);
        WS[k] = INV_2PI * (fma(-s.i0, la, s.k0s) * g[k].w - s.i0 * logw);
        const double Sd = a2 * fma(s.i1z, la, s.k1sz), Ld = a2 * s.i1z;
        const cplx cw = pc[k] * (g[k].dtau / Q);
        WD[k] = INV_2PI * (xn * fma(Sd, g[k].w, Ld * logw) + cw.im);
    }
    fold_add<NQ>(GL32_T, ta, tb, WS, WD, Ws, Wd);
}

/* Target on the curve at real local parameter sstar strictly inside the rule's
   interval, not at a node (NQ = 32), or exactly at node `at` (NQ = 16, the
   panel's own nodes).  Log part by kernel split with real moments; smooth and
   Cauchy parts by the plain rule (smooth on the curve), with the on-curve
   limits at a node: G^S(0) for the single layer and kappa/(4 pi) for the
   double layer. */
template <int NQ>
__host__ __device__ inline void leaf_oncurve(const cplx *a, const double *tq, const double *wq, double ta, double tb,
                                             cplx z, double tstar, int at, double alpha, double *Ws, double *Wd)
{
    NodeGeo g[NQ];
    double WS[NQ], WD[NQ];
    rule_geo<NQ>(a, tq, wq, ta, tb, g);
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const double ss = (tstar - mid) / half;
    double MC[NQ + 1], ML[NQ], pl[NQ];
    legendre_moments_real<NQ>(ss, MC, ML);
    moments_to_weights<NQ>(NQ == 16 ? LEGW16 : LEGW32, ML, pl);
    const double la = log(alpha);
    const double a2 = alpha * alpha;
    for (int k = 0; k < NQ; ++k) {
        const double sp_ = cabs(g[k].dtau);
        if (k == at) {
            /* on-curve limits at the target node */
            cplx p, dp, d2;
            leg_eval(a, mk(tstar, 0.0), p, dp, &d2);
            const double sp1 = cabs(dp);
            const double kappa = (dp.re * d2.im - dp.im * d2.re) / (sp1 * sp1 * sp1);
            const double logw = fma(sp_, pl[k], g[k].w * log(half * sp1));
            const Split s0 = split_k01(0.0);
            WS[k] = INV_2PI * (fma(-s0.i0, la, s0.k0s) * g[k].w - s0.i0 * logw);
            WD[k] = 0.5 * INV_2PI * kappa * g[k].w;
            continue;
        }
        /* target on the curve: form y - x, (x - y).n and |y - x|^2 from divided
           differences so that no cancellation occurs near the target */
        const double tk = mid + half * tq[k];
        const double dl = tk - tstar;
        cplx Qp, Rp;
        leg_divdiff2(a, tk, tstar, Qp, Rp);
        const double qq = cabs2(Qp);
        const double r2 = dl * dl * qq;
        const double r = sqrt(r2);
        const double spp = cabs(Qp + dl * Rp);            /* |p'(t_k)| */
        const double xr = (Qp.re * Rp.im - Qp.im * Rp.re) / (qq * spp); /* (x-y).n / r^2 */
        const double xn = xr * r2;
        const double logw = fma(sp_, pl[k], g[k].w * log(half * sqrt(qq)));
        const Split s = split_k01(alpha * r);
        WS[k] = INV_2PI * (fma(-s.i0, la, s.k0s) * g[k].w - s.i0 * logw);
        const double Sd = a2 * fma(s.i1z, la, s.k1sz), Ld = a2 * s.i1z;
        WD[k] = INV_2PI * (xn * fma(Sd, g[k].w, Ld * logw) + xr * g[k].w);
    }
    if (NQ == 16 && ta == -1.0 && tb == 1.0) {
        for (int j = 0; j < 16; ++j) {
            Ws[j] += WS[j];
            Wd[j] += WD[j];
        }
    } else {
        fold_add<NQ>(tq, ta, tb, WS, WD, Ws, Wd);
    }
}

/* Estimated arclength of [ta, tb] of the parent panel of arclength h. */
__host__ __device__ inline double sub_len(double h, double ta, double tb) { return 0.5 * h * (tb - ta); }

/* One interval of the (possibly subdivided) parent: classify by the Bernstein
   radius of the target's local preimage and apply the matching rule. */
__host__ __device__ inline void leaf_apply(const cplx *a, double ta, double tb, cplx z, cplx tstar, double alpha,
                                           const NearParams &P, double *Ws, double *Wd)
{
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    const double rho = bernstein_rho(ss);
    if (rho >= P.rho_direct)
        leaf_direct<16>(a, GL16_T, GL16_W, ta, tb, z, alpha, Ws, Wd);
    else if (rho >= P.rho_split)
        leaf_direct<32>(a, GL32_T, GL32_W, ta, tb, z, alpha, Ws, Wd);
    else
        leaf_split32(a, ta, tb, z, tstar, alpha, Ws, Wd);
}

/* Recursive bisection of [ta, tb] towards the target until every piece either
   satisfies alpha h <= ah_max or is far enough that its contribution is below
   exp(-far_exp) of the kernel at the target's distance scale; leaf(a, b) is
   called for every final piece. */
template <class Leaf>
__host__ __device__ inline void subdivide_t(const cplx *a, double h, double ta, double tb, cplx z, cplx tstar,
                                            double alpha, const NearParams &P, Leaf &&leaf)
{
    double st_a[64], st_b[64];
    int top = 0;
    st_a[top] = ta;
    st_b[top] = tb;
    ++top;
    while (top > 0) {
        --top;
        const double a0 = st_a[top], b0 = st_b[top];
        const double hs = sub_len(h, a0, b0);
        bool is_leaf = alpha * hs <= P.ah_max || top >= 60 || (b0 - a0) < 1e-12;
        if (!is_leaf) {
            const double mid = 0.5 * (a0 + b0), half = 0.5 * (b0 - a0);
            const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
            if (bernstein_rho(ss) >= P.rho_direct) {
                cplx pm, dpm;
                leg_eval(a, mk(mid, 0.0), pm, dpm);
                const double dist = cabs(pm - z) - 0.5 * hs;
                if (alpha * dist >= P.far_exp) is_leaf = true;
            }
        }
        if (is_leaf) {
            leaf(a0, b0);
        } else {
            const double m = 0.5 * (a0 + b0);
            st_a[top] = a0; st_b[top] = m; ++top;
            st_a[top] = m; st_b[top] = b0; ++top;
        }
    }
}

__host__ __device__ inline void subdivide(const cplx *a, double h, double ta, double tb, cplx z, cplx tstar,
                                          double alpha, const NearParams &P, double *Ws, double *Wd)
{
    subdivide_t(a, h, ta, tb, z, tstar, alpha, P,
                [&](double a0, double b0) { leaf_apply(a, a0, b0, z, tstar, alpha, P, Ws, Wd); });
}

/* Correction weights of target z against a panel with Legendre coefficients a
   (position) and arclength h.  self: index of the node of this panel that the
   target is (on-surface evaluation), or -1; tstar: preimage of the target
   (for self, the node's parameter). */
__host__ __device__ inline void pair_weights(const cplx *a, double h, cplx z, int self, cplx tstar, double alpha,
                                             const NearParams &P, double *Ws, double *Wd)
{
    for (int j = 0; j < 16; ++j) Ws[j] = Wd[j] = 0.0;
    if (self >= 0) {
        const double ts = GL16_T[self];
        if (alpha * h <= P.ah_max) {
            /* upsampled: the 32-point rule integrates (degree-15 density) x
               (smooth kernel factor) x log exactly to rounding */
            leaf_oncurve<32>(a, GL32_T, GL32_W, -1.0, 1.0, z, ts, -1, alpha, Ws, Wd);
            return;
        }
        /* central piece holding the target, then the rest subdivided */
        const double d = P.ah_max / (alpha * h);
        const double c0 = ts - d > -1.0 ? ts - d : -1.0;
        const double c1 = ts + d < 1.0 ? ts + d : 1.0;
        leaf_oncurve<32>(a, GL32_T, GL32_W, c0, c1, z, ts, -1, alpha, Ws, Wd);
        if (c0 > -1.0) subdivide(a, h, -1.0, c0, z, mk(ts, 0.0), alpha, P, Ws, Wd);
        if (c1 < 1.0) subdivide(a, h, c1, 1.0, z, mk(ts, 0.0), alpha, P, Ws, Wd);
        return;
    }
    if (alpha * h <= P.ah_max)
        leaf_apply(a, -1.0, 1.0, z, tstar, alpha, P, Ws, Wd);
    else
        subdivide(a, h, -1.0, 1.0, z, tstar, alpha, P, Ws, Wd);
}

/* ====================================================================== */
/* Target gradients (Sec. 4.4 restated for the scalar kernel).             */
/* ====================================================================== */
/* With e = x - y, r = |e|, n = n_y and the split alpha K1(alpha r)/r =
   S(r^2) + L(r^2) log r + 1/r^2 (the double-layer split of Sec. 4.1:
   S = alpha^2 (K1^S/z + (I1/z) log alpha), L = alpha^2 I1/z, z = alpha r),
     grad_x G       = -(1/2pi) e [S + L log r + 1/r^2],
     grad_x dG/dn_y = (1/2pi) grad_x [(e.n) (S + L log r + 1/r^2)]
                    = (1/2pi) { [n S + 2 (e.n) S' e]
                              + [n L + 2 (e.n) L' e] log r
                              + (e.n) L e / r^2
                              + grad_x (e.n)/r^2 },          ' = d/d(r^2).
   Each bracket is smooth, smooth times log r, smooth times the Cauchy-type
   vector e/r^2, or the gradient of the Laplace double layer.  In complex
   notation (vector (v1, v2) <-> v1 + i v2, tau - z = (s - s*) Q(s) on the
   local parameter s, ds_arc = |tau'| ds):
     int f e/r^2 ds_arc = -conj( int f |tau'| / Q  ds/(s - s*) )   (f real),
     int mu (e.n)/r^2 ds_arc = Im F(z),  F(z) = int mu dtau/(tau - z),
     grad Im F = (Im F', Re F'),  F'(z) = int mu tau'/Q^2 ds/(s - s*)^2.
   F' has a (tau - z)^-2 singularity.  As the paper does for its highest
   order term, it is lowered by parts on every interval [ta, tb] of the rule:
     int mu tau' ds/(tau - z)^2 = [-mu/(tau - z)]_ta^tb + int mu'(s) ds/(tau - z),
   where mu' is the derivative of the panel's degree-15 density interpolant
   (exact), so only Cauchy and log moments are needed, integrated through the
   interpolatory weights of the upsampled rule (Sec. 4.3).
   Weight blocks: W[0], W[1] = d/dx1, d/dx2 of S; W[2], W[3] = of D.       */

/* Derivatives l_j'(t) of the Lagrange basis of the 16 Gauss-Legendre nodes at
   real t, from the Legendre form l_j = sum_m LEGC[m][j] P_m and
   P'_{m+1} = P'_{m-1} + (2m+1) P_m. */
__host__ __device__ inline void lagrange16_deriv(double t, double *dl)
{
    double P0 = 1.0, P1 = t, D0 = 0.0, D1 = 1.0;
    for (int j = 0; j < 16; ++j) dl[j] = LEGC[16 + j];
    for (int m = 1; m < 15; ++m) {
        const double P2 = ((2.0 * m + 1.0) * t * P1 - m * P0) / (m + 1.0);
        const double D2 = D0 + (2.0 * m + 1.0) * P1;
        for (int j = 0; j < 16; ++j) dl[j] = fma(LEGC[(m + 1) * 16 + j], D2, dl[j]);
        P0 = P1; P1 = P2;
        D0 = D1; D1 = D2;
    }
}

/* Direct (plain quadrature) gradient weights at one node. */
__host__ __device__ inline void direct_node_grad(cplx z, const NodeGeo &g, double alpha, double *w4)
{
    const cplx e = z - g.tau;
    const double r2 = cabs2(e);
    const K01 o = k01_fp64<true, true>(r2, alpha, 0.25 * alpha * alpha, 4.0 / alpha);
    const double sp_ = cabs(g.dtau);
    const double nx = -g.dtau.im / sp_, ny = g.dtau.re / sp_;
    const double en = e.re * nx + e.im * ny;
    const double b = en * fma(alpha * alpha, o.k0, 2.0 * o.ak1r) / r2;
    const double c = INV_2PI * g.w;
    w4[0] = -c * o.ak1r * e.re;
    w4[1] = -c * o.ak1r * e.im;
    w4[2] = c * fma(o.ak1r, nx, -b * e.re);
    w4[3] = c * fma(o.ak1r, ny, -b * e.im);
}

/* Fold NW blocks of node weights of a rule with NQ nodes on [ta, tb] of the
   parent panel back to the parent's 16 nodes. */
template <int NQ, int NW>
__host__ __device__ inline void fold_add_n(const double *tq, double ta, double tb, const double (*WQ)[NQ],
                                           double (*W)[16])
{
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    for (int k = 0; k < NQ; ++k) {
        double l[16];
        lagrange16(mid + half * tq[k], l);
        for (int b = 0; b < NW; ++b)
            for (int j = 0; j < 16; ++j) W[b][j] = fma(l[j], WQ[b][k], W[b][j]);
    }
}

template <int NQ>
__host__ __device__ inline void leaf_direct_grad(const cplx *a, const double *tq, const double *wq, double ta,
                                                 double tb, cplx z, double alpha, double (*W)[16])
{
    NodeGeo g[NQ];
    double WQ[4][NQ];
    rule_geo<NQ>(a, tq, wq, ta, tb, g);
    for (int k = 0; k < NQ; ++k) {
        double w4[4];
        direct_node_grad(z, g[k], alpha, w4);
        for (int b = 0; b < 4; ++b) WQ[b][k] = w4[b];
    }
    fold_add_n<NQ, 4>(tq, ta, tb, WQ, W);
}

/* Kernel split on the 32-point upsampled rule of [ta, tb] (target off the
   curve, complex parent preimage tstar). */
__host__ __device__ inline void leaf_split32_grad(const cplx *a, double ta, double tb, cplx z, cplx tstar,
                                                  double alpha, double (*W)[16])
{
    constexpr int NQ = 32;
    NodeGeo g[NQ];
    double WQ[4][NQ];
    cplx WF[16]; /* weights of F'(z) on the parent's 16 nodes */
    rule_geo<NQ>(a, GL32_T, GL32_W, ta, tb, g);
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    cplx MC[NQ + 1], ML[NQ], pc[NQ], pl[NQ];
    legendre_moments<NQ>(ss, bernstein_rho(ss), MC, ML);
    moments_to_weights<NQ>(LEGW32, MC, pc); /* (s - s*)^-1 */
    moments_to_weights<NQ>(LEGW32, ML, pl); /* log(s - s*)  */
    /* end-point terms of F' by parts: mu(ta)/(tau(ta) - z) - mu(tb)/(tau(tb) - z) */
    {
        double la_[16], lb_[16];
        cplx pa, pb, dpa, dpb;
        leg_eval(a, mk(ta, 0.0), pa, dpa);
        leg_eval(a, mk(tb, 0.0), pb, dpb);
        lagrange16(ta, la_);
        lagrange16(tb, lb_);
        const cplx ia = mk(1.0, 0.0) / (pa - z), ib = mk(1.0, 0.0) / (pb - z);
        for (int j = 0; j < 16; ++j) WF[j] = la_[j] * ia - lb_[j] * ib;
    }
    const double la = log(alpha);
    const double a2 = alpha * alpha, a4q = 0.25 * a2 * a2;
    for (int k = 0; k < NQ; ++k) {
        const double tkr = mid + half * GL32_T[k];
        const cplx Q = half * leg_divdiff(a, mk(tkr, 0.0), tstar); /* (tau - z)/(s - s*) */
        const double sp_ = cabs(g[k].dtau);
        const double logw = fma(sp_, pl[k].re, g[k].w * log(cabs(Q)));
        const cplx e = z - g[k].tau;
        const SplitG sg = split_k01_grad(alpha * cabs(e));
        const double S = a2 * fma(sg.s.i1z, la, sg.s.k1sz), L = a2 * sg.s.i1z;
        const double Sq = a4q * fma(sg.i1z_q, la, sg.k1sz_q), Lq = a4q * sg.i1z_q;
        const double nx = -g[k].dtau.im / sp_, ny = g[k].dtau.re / sp_;
        const double en = e.re * nx + e.im * ny;
        const double Aw = fma(S, g[k].w, L * logw);          /* smooth + log, order 0 */
        const double Bw = 2.0 * en * fma(Sq, g[k].w, Lq * logw); /* from S', L'       */
        const cplx iQ = mk(1.0, 0.0) / Q;
        const cplx cS = (sp_ * pc[k]) * iQ;                    /* Cauchy, |tau'|/Q   */
        WQ[0][k] = INV_2PI * fma(-e.re, Aw, cS.re);
        WQ[1][k] = INV_2PI * fma(-e.im, Aw, -cS.im);
        WQ[2][k] = INV_2PI * (fma(nx, Aw, Bw * e.re) - en * L * cS.re);
        WQ[3][k] = INV_2PI * (fma(ny, Aw, Bw * e.im) + en * L * cS.im);
        /* by-parts integral: Cauchy weight times dmu/ds = half dmu/dt */
        double dl[16];
        lagrange16_deriv(tkr, dl);
        const cplx cD = (half * pc[k]) * iQ;
        for (int j = 0; j < 16; ++j) WF[j] = WF[j] + dl[j] * cD;
    }
    fold_add_n<NQ, 4>(GL32_T, ta, tb, WQ, W);
    /* grad Im F = (Im F', Re F') */
    for (int j = 0; j < 16; ++j) {
        W[2][j] = fma(INV_2PI, WF[j].im, W[2][j]);
        W[3][j] = fma(INV_2PI, WF[j].re, W[3][j]);
    }
}

__host__ __device__ inline void leaf_apply_grad(const cplx *a, double ta, double tb, cplx z, cplx tstar,
                                                double alpha, const NearParams &P, double (*W)[16])
{
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    const double rho = bernstein_rho(ss);
    if (rho >= P.rho_direct)
        leaf_direct_grad<16>(a, GL16_T, GL16_W, ta, tb, z, alpha, W);
    else if (rho >= P.rho_split)
        leaf_direct_grad<32>(a, GL32_T, GL32_W, ta, tb, z, alpha, W);
    else
        leaf_split32_grad(a, ta, tb, z, tstar, alpha, W);
}

/* Gradient correction weights of an off-curve target z against a panel
   (same tiers and subdivision as the potentials). */
__host__ __device__ inline void pair_grad_weights(const cplx *a, double h, cplx z, cplx tstar, double alpha,
                                                  const NearParams &P, double (*W)[16])
{
    for (int b = 0; b < 4; ++b)
        for (int j = 0; j < 16; ++j) W[b][j] = 0.0;
    if (alpha * h <= P.ah_max)
        leaf_apply_grad(a, -1.0, 1.0, z, tstar, alpha, P, W);
    else
        subdivide_t(a, h, -1.0, 1.0, z, tstar, alpha, P,
                    [&](double a0, double b0) { leaf_apply_grad(a, a0, b0, z, tstar, alpha, P, W); });
}

/* ====================================================================== */
/* Modified-Stokes double layer (the paper's BIE kernel, Sec. 4.1-4.3).    */
/* ====================================================================== */
/* D_ij(x, y) = -T_jik(x, y) n_k(y) with r = x - y:
     D_ij = -[A1 (n_i r_j + r_i n_j + d_ij (r.n)) + A2 r_i r_j (r.n) + A3 r_i n_j],
   A1 = alpha^2 T1, A2 = alpha^4 T2, A3 = alpha^2 T3 (z = alpha |r|).  With the
   split of T1..T3 (Sec. 4.1) the kernel is
     D = D[A^S] + D[A^L] log|r| - (alpha^2/8pi) r_i r_j (r.n)/|r|^2
         + (1/pi) r_i r_j (r.n)/|r|^4,
   A^S = (alpha^2 (T1S + T1L log alpha), alpha^4 (T2S + T2L log alpha), ...),
   A^L = (alpha^2 T1L, alpha^4 T2L, alpha^2 T3L).  The first two terms are
   smooth and smooth times log; the third is a smooth factor times the
   Laplace double-layer kernel (r.n)/|r|^2, integrated as Im of a Cauchy
   integral (Sec. 4.3); the fourth is the Stokes stresslet, whose complex
   form (Sec. 4.3; e = tau - z, omega = mu_1 + i mu_2, nu = n_1 + i n_2) is
     int (mu.e) e (e.n)/|e|^4 dS = -(1/2) int omega Im(dtau/e)
        + (1/4i) conj(int omega conj(nu)^2 dtau/e)
        + (1/4i) conj(int omega conj(e) dtau/e^2),
   and r = -e flips its sign.  The (tau - z)^-2 integral is lowered by parts
   as for the gradients: int f dtau/e^2 = [-f/e] + int f'(s) ds/e with
   f = omega conj(e), f' = omega' conj(e) + omega conj(tau'), the density's
   derivative taken from its degree-15 interpolant.
   Weight blocks: W[0..3] = D11, D12, D21, D22 on the panel's 16 nodes.       */

__host__ __device__ inline void stk_tensor(double rx, double ry, double nx, double ny, const double *A, double *D)
{
    const double rn = rx * nx + ry * ny;
    D[0] = -(A[0] * (2.0 * nx * rx + rn) + A[1] * rx * rx * rn + A[2] * rx * nx);
    D[1] = -(A[0] * (nx * ry + rx * ny) + A[1] * rx * ry * rn + A[2] * rx * ny);
    D[2] = -(A[0] * (ny * rx + ry * nx) + A[1] * ry * rx * rn + A[2] * ry * nx);
    D[3] = -(A[0] * (2.0 * ny * ry + rn) + A[1] * ry * ry * rn + A[2] * ry * ny);
}

/* conj(B omega) as a real 2x2 block acting on (mu_1, mu_2), added to W[.][j] */
__host__ __device__ inline void add_conj_block(cplx B, double (*W)[16], int j)
{
    W[0][j] += B.re;
    W[1][j] -= B.im;
    W[2][j] -= B.im;
    W[3][j] -= B.re;
}

/* split coefficients A^S, A^L at distance r */
__host__ __device__ inline void stk_split_coeffs(double alpha, double r, double *AS, double *AL)
{
    const StkSplit t = stresslet_split(alpha * r);
    const double la = log(alpha), a2 = alpha * alpha, sc[3] = {a2, a2 * a2, a2};
    for (int i = 0; i < 3; ++i) {
        AS[i] = sc[i] * fma(t.l[i], la, t.s[i]);
        AL[i] = sc[i] * t.l[i];
    }
}

__host__ __device__ inline void direct_node_stokes(cplx z, const NodeGeo &g, double alpha, double *w4)
{
    const cplx e = z - g.tau; /* r = x - y */
    const double r2 = cabs2(e);
    const K01 o = k01_fp64<true, true>(r2, alpha, 0.25 * alpha * alpha, 4.0 / alpha);
    double A[3];
    stresslet_scaled(alpha * alpha, 1.0 / (alpha * alpha), r2, 1.0 / r2, o.k0, o.ak1r, A);
    const double sp_ = cabs(g.dtau);
    double D[4];
    stk_tensor(e.re, e.im, -g.dtau.im / sp_, g.dtau.re / sp_, A, D);
    for (int b = 0; b < 4; ++b) w4[b] = D[b] * g.w;
}

template <int NQ>
__host__ __device__ inline void leaf_direct_stokes(const cplx *a, const double *tq, const double *wq, double ta,
                                                   double tb, cplx z, double alpha, double (*W)[16])
{
    NodeGeo g[NQ];
    double WQ[4][NQ];
    rule_geo<NQ>(a, tq, wq, ta, tb, g);
    for (int k = 0; k < NQ; ++k) {
        double w4[4];
        direct_node_stokes(z, g[k], alpha, w4);
        for (int b = 0; b < 4; ++b) WQ[b][k] = w4[b];
    }
    fold_add_n<NQ, 4>(tq, ta, tb, WQ, W);
}

/* Kernel split on the 32-point upsampled rule of [ta, tb] for a target off the
   interval (complex parent preimage tstar, or real outside [ta, tb]). */
__host__ __device__ inline void leaf_split32_stokes(const cplx *a, double ta, double tb, cplx z, cplx tstar,
                                                    double alpha, double (*W)[16])
{
    constexpr int NQ = 32;
    NodeGeo g[NQ];
    double WQ[4][NQ];
    cplx WB[16]; /* conj(WB omega): the by-parts stresslet term on the parent nodes */
    rule_geo<NQ>(a, GL32_T, GL32_W, ta, tb, g);
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    cplx MC[NQ + 1], ML[NQ], pc[NQ], pl[NQ];
    legendre_moments<NQ>(ss, bernstein_rho(ss), MC, ML);
    moments_to_weights<NQ>(LEGW32, MC, pc);
    moments_to_weights<NQ>(LEGW32, ML, pl);
    const cplx cf = mk(0.0, -0.25 / PI); /* -i/(4 pi) */
    /* end-point terms of the by-parts integral: [-omega conj(e)/e]_ta^tb */
    {
        double la_[16], lb_[16];
        cplx pa, pb, dpa, dpb;
        leg_eval(a, mk(ta, 0.0), pa, dpa);
        leg_eval(a, mk(tb, 0.0), pb, dpb);
        lagrange16(ta, la_);
        lagrange16(tb, lb_);
        const cplx ea = pa - z, eb = pb - z;
        const cplx qa = conj(ea) / ea, qb = conj(eb) / eb;
        for (int j = 0; j < 16; ++j) WB[j] = cf * (la_[j] * qa - lb_[j] * qb);
    }
    const double a2 = alpha * alpha;
    for (int k = 0; k < NQ; ++k) {
        const double tkr = mid + half * GL32_T[k];
        const cplx Q = half * leg_divdiff(a, mk(tkr, 0.0), tstar); /* (tau - z)/(s - s*) */
        const double sp_ = cabs(g[k].dtau);
        const double logw = fma(sp_, pl[k].re, g[k].w * log(cabs(Q)));
        const cplx r = z - g[k].tau; /* x - y */
        const cplx nu = mk(-g[k].dtau.im / sp_, g[k].dtau.re / sp_);
        double AS[3], AL[3], Ds[4], Dl[4];
        stk_split_coeffs(alpha, cabs(r), AS, AL);
        stk_tensor(r.re, r.im, nu.re, nu.im, AS, Ds);
        stk_tensor(r.re, r.im, nu.re, nu.im, AL, Dl);
        const cplx iQ = mk(1.0, 0.0) / Q;
        const cplx cdt = pc[k] * (g[k].dtau * iQ); /* weight of int f dtau/(tau - z) */
        const double cw = cdt.im;                 /* Laplace double layer */
        /* -(alpha^2/8pi) r_i r_j (r.n)/|r|^2  and  (1/2pi) omega Im(dtau/e) */
        const double c8 = -a2 / (8.0 * PI) * cw, c2 = 0.5 / PI * cw;
        WQ[0][k] = fma(Ds[0], g[k].w, Dl[0] * logw) + c8 * r.re * r.re + c2;
        WQ[1][k] = fma(Ds[1], g[k].w, Dl[1] * logw) + c8 * r.re * r.im;
        WQ[2][k] = fma(Ds[2], g[k].w, Dl[2] * logw) + c8 * r.im * r.re;
        WQ[3][k] = fma(Ds[3], g[k].w, Dl[3] * logw) + c8 * r.im * r.im + c2;
        /* conj((-i/4pi) int omega conj(nu)^2 dtau/e) at this node, and the
           omega conj(tau') part of the by-parts integrand */
        const cplx nb2 = conj(nu * nu);
        const cplx B1 = cf * (nb2 * cdt);
        const cplx B2 = cf * (pc[k] * conj(g[k].dtau) * iQ);
        WQ[0][k] += B1.re + B2.re;
        WQ[1][k] -= B1.im + B2.im;
        WQ[2][k] -= B1.im + B2.im;
        WQ[3][k] -= B1.re + B2.re;
        /* omega' conj(e) part: the density derivative on the parent nodes */
        double dl[16];
        lagrange16_deriv(tkr, dl);
        const cplx cD = cf * ((half * pc[k]) * (conj(mk(0.0, 0.0) - r) * iQ)); /* conj(e) = -conj(r) */
        for (int j = 0; j < 16; ++j) WB[j] = WB[j] + dl[j] * cD;
    }
    fold_add_n<NQ, 4>(GL32_T, ta, tb, WQ, W);
    for (int j = 0; j < 16; ++j) add_conj_block(WB[j], W, j);
}

/* Target on the curve at real local parameter sstar inside the rule's interval
   (not at one of its nodes): the log part by kernel split with real moments;
   the Cauchy-type and stresslet terms are smooth on the curve and taken by the
   plain rule, with (x - y) and (x - y).n/|x - y|^2 from divided differences. */
__host__ __device__ inline void leaf_oncurve_stokes(const cplx *a, double ta, double tb, double tstar, double alpha,
                                                    double (*W)[16])
{
    constexpr int NQ = 32;
    NodeGeo g[NQ];
    double WQ[4][NQ];
    rule_geo<NQ>(a, GL32_T, GL32_W, ta, tb, g);
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const double ss = (tstar - mid) / half;
    double MC[NQ + 1], ML[NQ], pl[NQ];
    legendre_moments_real<NQ>(ss, MC, ML);
    moments_to_weights<NQ>(LEGW32, ML, pl);
    const double a2 = alpha * alpha;
    for (int k = 0; k < NQ; ++k) {
        const double sp_ = cabs(g[k].dtau);
        const double tk = mid + half * GL32_T[k];
        const double dl = tk - tstar;
        cplx Qp, Rp;
        leg_divdiff2(a, tk, tstar, Qp, Rp);
        const double qq = cabs2(Qp);
        const double r2 = dl * dl * qq;
        const double spp = cabs(Qp + dl * Rp);
        const double xr = (Qp.re * Rp.im - Qp.im * Rp.re) / (qq * spp); /* (x-y).n / r^2 */
        const cplx r = (-dl) * Qp;                                       /* x - y */
        const double ux = Qp.re * Qp.re / qq, uxy = Qp.re * Qp.im / qq, uy = Qp.im * Qp.im / qq; /* r^ r^ */
        const double logw = fma(sp_, pl[k], g[k].w * log(half * sqrt(qq)));
        const double nx = -g[k].dtau.im / sp_, ny = g[k].dtau.re / sp_;
        double AS[3], AL[3], Ds[4], Dl[4];
        stk_split_coeffs(alpha, sqrt(r2), AS, AL);
        stk_tensor(r.re, r.im, nx, ny, AS, Ds);
        stk_tensor(r.re, r.im, nx, ny, AL, Dl);
        /* -(alpha^2/8pi) r_i r_j xr + (1/pi) r^_i r^_j xr */
        const double cq = xr * (1.0 / PI - a2 / (8.0 * PI) * r2);
        WQ[0][k] = fma(Ds[0], g[k].w, Dl[0] * logw) + cq * ux * g[k].w;
        WQ[1][k] = fma(Ds[1], g[k].w, Dl[1] * logw) + cq * uxy * g[k].w;
        WQ[2][k] = fma(Ds[2], g[k].w, Dl[2] * logw) + cq * uxy * g[k].w;
        WQ[3][k] = fma(Ds[3], g[k].w, Dl[3] * logw) + cq * uy * g[k].w;
    }
    fold_add_n<NQ, 4>(GL32_T, ta, tb, WQ, W);
}

__host__ __device__ inline void leaf_apply_stokes(const cplx *a, double ta, double tb, cplx z, cplx tstar,
                                                  double alpha, const NearParams &P, double (*W)[16])
{
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    const double rho = bernstein_rho(ss);
    if (rho >= P.rho_direct)
        leaf_direct_stokes<16>(a, GL16_T, GL16_W, ta, tb, z, alpha, W);
    else if (rho >= P.rho_split)
        leaf_direct_stokes<32>(a, GL32_T, GL32_W, ta, tb, z, alpha, W);
    else
        leaf_split32_stokes(a, ta, tb, z, tstar, alpha, W);
}

/* Stresslet correction weights of target z against a panel; self: node of
   this panel that the target is (on-surface), or -1 (same tiers, subdivision
   and on-curve treatment as the scalar double layer). */
__host__ __device__ inline void pair_stokes_weights(const cplx *a, double h, cplx z, int self, cplx tstar,
                                                    double alpha, const NearParams &P, double (*W)[16])
{
    for (int b = 0; b < 4; ++b)
        for (int j = 0; j < 16; ++j) W[b][j] = 0.0;
    auto leaf = [&](double a0, double b0) { leaf_apply_stokes(a, a0, b0, z, tstar, alpha, P, W); };
    if (self >= 0) {
        const double ts = GL16_T[self];
        if (alpha * h <= P.ah_max) {
            leaf_oncurve_stokes(a, -1.0, 1.0, ts, alpha, W);
            return;
        }
        const double d = P.ah_max / (alpha * h);
        const double c0 = ts - d > -1.0 ? ts - d : -1.0;
        const double c1 = ts + d < 1.0 ? ts + d : 1.0;
        leaf_oncurve_stokes(a, c0, c1, ts, alpha, W);
        if (c0 > -1.0) subdivide_t(a, h, -1.0, c0, z, tstar, alpha, P, leaf);
        if (c1 < 1.0) subdivide_t(a, h, c1, 1.0, z, tstar, alpha, P, leaf);
        return;
    }
    if (alpha * h <= P.ah_max)
        leaf(-1.0, 1.0);
    else
        subdivide_t(a, h, -1.0, 1.0, z, tstar, alpha, P, leaf);
}

/* ---------------------------------------------------------------------- */
/* Target gradient of the stresslet double layer (Sec. 4.4).               */
/* ---------------------------------------------------------------------- */
/* With A_k(r) as above and B_k = A_k'(|r|)/|r|,
     d/dx_l D_ij = -[ r_l (B1 P1 + B2 P2 + B3 P3)_ij + A1 dP1_ijl + A2 dP2_ijl + A3 dP3_ijl ],
   P1 = n_i r_j + r_i n_j + d_ij (r.n), P2 = r_i r_j (r.n), P3 = r_i n_j,
   dP1 = n_i d_jl + d_il n_j + d_ij n_l, dP2 = d_il r_j (r.n) + r_i d_jl (r.n) + r_i r_j n_l, dP3 = d_il n_j.
   Split (Sec. 4.1, 4.4): with A_k = A_k^S + A_k^L log|r| + (explicit terms of A2),
     smooth    -[r_l sum B^S P + sum A^S dP]
     log       -[r_l sum B^L P + sum A^L dP] log|r|        (B^S, B^L = 2 d/d(r^2))
     Cauchy    -(sum A^L P)_ij r_l/|r|^2                  (vector Cauchy kernel, as for grad S)
     d_l of -(alpha^2/8pi) r_i r_j (r.n)/|r|^2:
         -(alpha^2/8pi) [(d_il r_j + r_i d_jl) (r.n)/|r|^2 + r_i r_j d_l((r.n)/|r|^2)],
       the second a frozen smooth factor times the Laplace double-layer gradient
       (Im F', Re F'), F' = int f dtau/(tau - z)^2 by (s - s*)^-2 moments;
     d_l of (1/pi) r_i r_j (r.n)/|r|^4 (Stokes stresslet): with u = -(1/pi) I(z) and
       I the complex form of the double layer (see above),
         dI/dz  = (i/2) Re H1(omega),
         dI/dzb = (1/4i) conj(H1(conj omega)) + (1/4i) conj(H1(omega conj(nu)^2))
                  + (1/2i) conj(H2(omega conj(e))),
       H1(f) = int f dtau/e^2, H2(f) = int f dtau/e^3, lowered once by parts:
       H2(f) = [-f/(2 e^2)] + (1/2) int f'(s) ds/e^2, and d/dx = d/dz + d/dzb,
       d/dy = i (d/dz - d/dzb).
   Weight blocks: W[(2i + l) 2 + j] = d/dx_l of u_i per mu_j, on the panel's 16 nodes. */

/* MH[m] = int P_m(t)/(t - s)^2 dt, m = 0..N-1, from the Cauchy moments MC
   (m = 0..N-2): by parts, MH_m = B_m + int P_m'/(t - s) dt with
   B_m = -1/(1 - s) - (-1)^m/(1 + s); P_{m+1}' - P_{m-1}' = (2m+1) P_m and
   B_{m+1} = B_{m-1} give MH_{m+1} = MH_{m-1} + (2m+1) MC_m,
   MH_0 = B_0, MH_1 = B_1 + MC_0. */
template <int N>
__host__ __device__ inline void hyper_moments(cplx s, const cplx *MC, cplx *MH)
{
    const cplx ia = mk(1.0, 0.0) / (mk(1.0, 0.0) - s), ib = mk(1.0, 0.0) / (mk(1.0, 0.0) + s);
    MH[0] = -(ia + ib);
    MH[1] = (ib - ia) + MC[0];
    for (int m = 1; m + 1 < N; ++m) MH[m + 1] = MH[m - 1] + (2.0 * m + 1.0) * MC[m];
}

/* G[(2i+l)2+j] = r_l (sum_k B_k P_k)_ij + sum_k A_k dP_k,ijl (no sign) */
__host__ __device__ inline void stk_dtensor(double rx, double ry, double nx, double ny, const double *A,
                                            const double *B, double *G)
{
    const double r[2] = {rx, ry}, n[2] = {nx, ny};
    const double rn = rx * nx + ry * ny;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const double dij = i == j ? 1.0 : 0.0;
            const double P = B[0] * (n[i] * r[j] + r[i] * n[j] + dij * rn) + B[1] * r[i] * r[j] * rn + B[2] * r[i] * n[j];
            for (int l = 0; l < 2; ++l) {
                const double dil = i == l ? 1.0 : 0.0, djl = j == l ? 1.0 : 0.0;
                G[(2 * i + l) * 2 + j] = r[l] * P + A[0] * (n[i] * djl + dil * n[j] + dij * n[l]) +
                                         A[1] * (dil * r[j] * rn + r[i] * djl * rn + r[i] * r[j] * n[l]) +
                                         A[2] * dil * n[j];
            }
        }
}

/* adds  u_l += a omega + conj(b omega)  (u = u1 + i u2, omega = mu1 + i mu2) for
   derivative direction l to the eight real weights w8 of one node */
__host__ __device__ inline void add_ab(cplx a, cplx b, int l, double *w8, int stride)
{
    w8[((0 + l) * 2 + 0) * stride] += a.re + b.re;
    w8[((0 + l) * 2 + 1) * stride] += -a.im - b.im;
    w8[((2 + l) * 2 + 0) * stride] += a.im - b.im;
    w8[((2 + l) * 2 + 1) * stride] += a.re - b.re;
}

/* the Stokes-stresslet part of the gradient for a coefficient pair of dI/dz
   (az, bz) and dI/dzb (azb, bzb): d/dx u = -(1/pi)(dI/dz + dI/dzb),
   d/dy u = -(i/pi)(dI/dz - dI/dzb) */
__host__ __device__ inline void add_stresslet_grad(cplx az, cplx bz, cplx azb, cplx bzb, double *w8, int stride)
{
    const double ip = 1.0 / PI;
    add_ab(-ip * (az + azb), -ip * (bz + bzb), 0, w8, stride);
    add_ab(mk(0.0, -ip) * (az - azb), mk(0.0, ip) * (bz - bzb), 1, w8, stride);
}

__host__ __device__ inline void direct_node_stokes_grad(cplx z, const NodeGeo &g, double alpha, double *w8)
{
    const cplx r = z - g.tau;
    const double r2 = cabs2(r);
    const K01 o = k01_fp64<true, true>(r2, alpha, 0.25 * alpha * alpha, 4.0 / alpha);
    double A[3], B[3], G[8];
    stk_AB(alpha, r2, o.k0, o.ak1r, A, B);
    const double sp_ = cabs(g.dtau);
    stk_dtensor(r.re, r.im, -g.dtau.im / sp_, g.dtau.re / sp_, A, B, G);
    for (int b = 0; b < 8; ++b) w8[b] = -G[b] * g.w;
}

template <int NQ>
__host__ __device__ inline void leaf_direct_stokes_grad(const cplx *a, const double *tq, const double *wq, double ta,
                                                        double tb, cplx z, double alpha, double (*W)[16])
{
    NodeGeo g[NQ];
    double WQ[8][NQ];
    rule_geo<NQ>(a, tq, wq, ta, tb, g);
    for (int k = 0; k < NQ; ++k) {
        double w8[8];
        direct_node_stokes_grad(z, g[k], alpha, w8);
        for (int b = 0; b < 8; ++b) WQ[b][k] = w8[b];
    }
    fold_add_n<NQ, 8>(tq, ta, tb, WQ, W);
}

__host__ __device__ inline void leaf_split32_stokes_grad(const cplx *a, double ta, double tb, cplx z, cplx tstar,
                                                         double alpha, double (*W)[16])
{
    constexpr int NQ = 32;
    NodeGeo g[NQ];
    double WQ[8][NQ];
    cplx PB[16]; /* dI/dzb, conj part, on the parent nodes (H2 by parts) */
    rule_geo<NQ>(a, GL32_T, GL32_W, ta, tb, g);
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    cplx MC[NQ + 1], ML[NQ], MH[NQ], pc[NQ], pl[NQ], ph[NQ];
    legendre_moments<NQ>(ss, bernstein_rho(ss), MC, ML);
    hyper_moments<NQ>(ss, MC, MH);
    moments_to_weights<NQ>(LEGW32, MC, pc);
    moments_to_weights<NQ>(LEGW32, ML, pl);
    moments_to_weights<NQ>(LEGW32, MH, ph);
    const cplx i2 = mk(0.0, 0.5), i4 = mk(0.0, 0.25);
    /* end points of H2 by parts: [-omega conj(e)/(2 e^2)]_ta^tb, times (i/2) in dI/dzb */
    {
        double la_[16], lb_[16];
        cplx pa, pb, dpa, dpb;
        leg_eval(a, mk(ta, 0.0), pa, dpa);
        leg_eval(a, mk(tb, 0.0), pb, dpb);
        lagrange16(ta, la_);
        lagrange16(tb, lb_);
        const cplx ea = pa - z, eb = pb - z;
        const cplx qa = conj(ea) / (2.0 * (ea * ea)), qb = conj(eb) / (2.0 * (eb * eb));
        for (int j = 0; j < 16; ++j) PB[j] = i2 * (la_[j] * qa - lb_[j] * qb);
    }
    const double la = log(alpha), a2 = alpha * alpha, c8 = -a2 / (8.0 * PI);
    const double sc[3] = {a2, a2 * a2, a2};
    for (int k = 0; k < NQ; ++k) {
        const double tkr = mid + half * GL32_T[k];
        const cplx Q = half * leg_divdiff(a, mk(tkr, 0.0), tstar);
        const double sp_ = cabs(g[k].dtau);
        const double logw = fma(sp_, pl[k].re, g[k].w * log(cabs(Q)));
        const cplx r = z - g[k].tau; /* x - y */
        const cplx e = -r;           /* tau - z */
        const double nx = -g[k].dtau.im / sp_, ny = g[k].dtau.re / sp_;
        const cplx nu = mk(nx, ny);
        const StkSplit t = stresslet_split_t<true>(alpha * cabs(r));
        double AS[3], AL[3], BS[3], BL[3];
        for (int q = 0; q < 3; ++q) {
            AS[q] = sc[q] * fma(t.l[q], la, t.s[q]);
            AL[q] = sc[q] * t.l[q];
            BS[q] = 2.0 * sc[q] * a2 * fma(t.dl[q], la, t.ds[q]);
            BL[q] = 2.0 * sc[q] * a2 * t.dl[q];
        }
        double Gs[8], Gl[8];
        stk_dtensor(r.re, r.im, nx, ny, AS, BS, Gs);
        stk_dtensor(r.re, r.im, nx, ny, AL, BL, Gl);
        double w8[8];
        for (int b = 0; b < 8; ++b) w8[b] = -fma(Gs[b], g[k].w, Gl[b] * logw);
        const cplx iQ = mk(1.0, 0.0) / Q;
        const cplx cS = (sp_ * pc[k]) * iQ;        /* int f ds/(tau - z) */
        const double cw = (pc[k] * (g[k].dtau * iQ)).im; /* Laplace double layer */
        const cplx h = ph[k] * (g[k].dtau * (iQ * iQ));    /* int f dtau/(tau - z)^2 */
        const double rv[2] = {r.re, r.im}, n[2] = {nx, ny};
        const double rn = r.re * nx + r.im * ny;
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                const double dij = i == j ? 1.0 : 0.0;
                /* Cauchy part of the log term: -(sum A^L P)_ij r_l/|r|^2 */
                const double M = AL[0] * (n[i] * rv[j] + rv[i] * n[j] + dij * rn) + AL[1] * rv[i] * rv[j] * rn +
                                 AL[2] * rv[i] * n[j];
                w8[(2 * i + 0) * 2 + j] += cS.re * M;
                w8[(2 * i + 1) * 2 + j] -= cS.im * M;
                /* -(alpha^2/8pi) [(d_il r_j + r_i d_jl) (r.n)/|r|^2 + r_i r_j d_l((r.n)/|r|^2)] */
                for (int l = 0; l < 2; ++l) {
                    const double dil = i == l ? 1.0 : 0.0, djl = j == l ? 1.0 : 0.0;
                    w8[(2 * i + l) * 2 + j] += c8 * (dil * rv[j] + rv[i] * djl) * cw;
                }
                w8[(2 * i + 0) * 2 + j] += c8 * rv[i] * rv[j] * h.im;
                w8[(2 * i + 1) * 2 + j] += c8 * rv[i] * rv[j] * h.re;
            }
        /* Stokes stresslet: node terms of dI/dz and dI/dzb */
        const cplx az = i4 * h, bz = -(i4 * h);
        const cplx azb = -(i4 * conj(h));
        const cplx bzb = i4 * (h * conj(nu * nu)) + i2 * (0.5 * (ph[k] * (conj(g[k].dtau) * (iQ * iQ))));
        add_stresslet_grad(az, bz, azb, bzb, w8, 1);
        for (int b = 0; b < 8; ++b) WQ[b][k] = w8[b];
        /* omega' conj(e) part of H2 by parts (parent nodes) */
        double dl[16];
        lagrange16_deriv(tkr, dl);
        const cplx cD = i2 * (0.5 * half * (ph[k] * (conj(e) * (iQ * iQ))));
        for (int j = 0; j < 16; ++j) PB[j] = PB[j] + dl[j] * cD;
    }
    fold_add_n<NQ, 8>(GL32_T, ta, tb, WQ, W);
    for (int j = 0; j < 16; ++j) add_stresslet_grad(mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), PB[j], &W[0][j], 16);
}

__host__ __device__ inline void leaf_apply_stokes_grad(const cplx *a, double ta, double tb, cplx z, cplx tstar,
                                                       double alpha, const NearParams &P, double (*W)[16])
{
    const double mid = 0.5 * (ta + tb), half = 0.5 * (tb - ta);
    const cplx ss = (1.0 / half) * (tstar - mk(mid, 0.0));
    const double rho = bernstein_rho(ss);
    if (rho >= P.rho_direct)
        leaf_direct_stokes_grad<16>(a, GL16_T, GL16_W, ta, tb, z, alpha, W);
    else if (rho >= P.rho_split)
        leaf_direct_stokes_grad<32>(a, GL32_T, GL32_W, ta, tb, z, alpha, W);
    else
        leaf_split32_stokes_grad(a, ta, tb, z, tstar, alpha, W);
}

/* Stresslet-gradient correction weights of an off-curve target (8 blocks). */
__host__ __device__ inline void pair_stokes_grad_weights(const cplx *a, double h, cplx z, cplx tstar, double alpha,
                                                         const NearParams &P, double (*W)[16])
{
    for (int b = 0; b < 8; ++b)
        for (int j = 0; j < 16; ++j) W[b][j] = 0.0;
    auto leaf = [&](double a0, double b0) { leaf_apply_stokes_grad(a, a0, b0, z, tstar, alpha, P, W); };
    if (alpha * h <= P.ah_max)
        leaf(-1.0, 1.0);
    else
        subdivide_t(a, h, -1.0, 1.0, z, tstar, alpha, P, leaf);
}

} // namespace mhlp

/*
 * mhlp_oracle.c -- plain, slow, FP64 CPU oracle for the modified-Helmholtz
 * (Yukawa) layer potentials.  TEST INFRASTRUCTURE ONLY: nothing in the HIP
 * library includes, links or calls this file; it shares no code with it.
 *
 * What it computes (af Klinteberg, Askham & Kropinski, "A fast integral
 * equation method for the two-dimensional Navier-Stokes equations"):
 *
 *   SLP  u(x) = int_Gamma G(x,y) sigma(y) dS_y,   G = K0(alpha r) / (2 pi)
 *   DLP  u(x) = int_Gamma dG/dn_y mu(y) dS_y
 *             = int_Gamma alpha K1(alpha r) (x-y).n_y / (2 pi r) mu(y) dS_y
 *
 * and the target gradients of both (Sec. 4.4, the near-boundary gradient,
 * restated for the scalar kernel; r = |x - y|, A = alpha K1(alpha r)/r):
 *
 *   grad_x G       = A (y - x) / (2 pi)
 *   grad_x dG/dn_y = [A n_y - ((y-x).n_y)(y - x)(alpha^2 K0 + 2A)/r^2] / (2 pi)
 *
 * (from K0' = -K1 and (K1(z)/z)' = -(K0(z) + 2 K1(z)/z)/z).
 *
 * The modified-Stokes double layer of Sec. 3.2 (the paper's own BIE):
 *
 *   D[mu]_i(x) = int_Gamma D_ij(x,y) mu_j(y) dS_y,  D_ij = -T_jik(x,y) n_k(y),
 *   T_ijk = a^2 T1 (d_jk r_i + d_ik r_j + d_ij r_k) + a^4 T2 r_i r_j r_k + a^2 T3 d_ik r_j,
 *
 * r = x - y, with T1..T3 of App. B (closed forms in K0, K1 for z > 1.5, the
 * power series of App. C below), and the on-surface operator
 * (1/2) mu + D_pv mu + W mu, W mu = n (int mu.n dS) / |Gamma| (Sec. 2.2).
 *
 * K0(alpha r)/(2 pi) is the scalar Yukawa piece of the paper's modified
 * biharmonic Green's function (Sec. 2, eq. for G; App. B).  The boundary is the
 * composite 16-point Gauss-Legendre panel discretisation of Sec. 3.2, and the
 * density on a panel is the degree-15 interpolant of its nodal values.  The
 * panel itself is taken as the degree-15 polynomial curve through its 16 nodes.
 *
 * The oracle evaluates the *exact* panel integral of that interpolant for
 * every panel close to the target (adaptive Gauss-Legendre bisection; graded
 * meshes towards a target lying on the panel), and the plain 16-point
 * Gauss-Legendre sum for every other panel -- the discretised layer potential
 * of Sec. 3.2 that the kernel-split quadrature of Sec. 4 approximates.  It does
 * not use kernel splitting, upsampling tiers, panel merging or subdivision.
 *
 * Bessel functions: power series of App. C for z <= 2; for z > 2 the integral
 * representation K_nu(z) = int_0^inf exp(-z cosh u) cosh(nu u) du (DLMF 10.32.9)
 * by the trapezoid rule.
 *
 * Conventions: normals n = i tau'/|tau'| (into the domain when the domain lies
 * to the left of the curve direction); the on-surface operator is
 * (1/2) mu + D_pv mu (interior limit, jump relation of the paper's Lemma on
 * jump conditions).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define NPAN 16
#ifndef ORC_RTOL
#define ORC_RTOL 1e-14
#endif
/* the gradient integrals near the curve converge more slowly on the accepted
   pieces; a tighter test keeps their exact panel integrals at ~1e-13 of the
   weights (checked against 30-digit quadrature) */
#ifndef ORC_RTOL_GRAD
#define ORC_RTOL_GRAD 1e-15
#endif
#define TWO_PI 6.283185307179586476925286766559
#define EULER_GAMMA 0.57721566490153286060651209008240243

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rules by Newton iteration on P_n (textbook)               */
/* ------------------------------------------------------------------------ */
static void gauss_legendre(int n, double *t, double *w)
{
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        t[n - 1 - i] = x; /* ascending */
        w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
}

static double GL16_T[16], GL16_W[16], GL32_T[32], GL32_W[32];
static double BARY_W[16];       /* barycentric weights of the 16 nodes */
static long double BARY_W_L[16];
static long double DIFF_L[16][16];  /* differentiation matrix at the nodes */
static int g_init = 0;

static void init_rules(void)
{
    if (g_init) return;
    gauss_legendre(16, GL16_T, GL16_W);
    gauss_legendre(32, GL32_T, GL32_W);
    for (int j = 0; j < 16; ++j) {
        long double p = 1.0L;
        for (int k = 0; k < 16; ++k)
            if (k != j) p *= ((long double)GL16_T[j] - (long double)GL16_T[k]);
        BARY_W_L[j] = 1.0L / p;
        BARY_W[j] = (double)BARY_W_L[j];
    }
    for (int i = 0; i < 16; ++i) {
        long double s = 0.0L;
        for (int j = 0; j < 16; ++j) {
            if (j == i) continue;
            DIFF_L[i][j] = (BARY_W_L[j] / BARY_W_L[i]) / ((long double)GL16_T[i] - (long double)GL16_T[j]);
            s += DIFF_L[i][j];
        }
        DIFF_L[i][i] = -s;
    }
    g_init = 1;
}

void orc_gauss_legendre(int n, double *t, double *w) { gauss_legendre(n, t, w); }

/* ------------------------------------------------------------------------ */
/* Modified Bessel functions K0, K1                                          */
/* ------------------------------------------------------------------------ */
static void k01_series(double z, double *k0, double *k1)
{
    /* App. C: with q = z^2/4,
       I0 = sum q^n/(n!)^2,  I1 = (z/2) sum q^n/(n!(n+1)!)
       K0 = -log(z/2) I0 + sum psi(n+1) q^n/(n!)^2
       K1 = 1/z + log(z/2) I1 - (z/4) sum (psi(n+1)+psi(n+2)) q^n/(n!(n+1)!)
       psi(1) = -gamma, psi(n+1) = psi(n) + 1/n.                              */
    double q = 0.25 * z * z;
    double lz = log(0.5 * z);
    double a = 1.0;          /* q^n/(n!)^2      */
    double b = 1.0;          /* q^n/(n!(n+1)!)  */
    double psi1 = -EULER_GAMMA;          /* psi(n+1) */
    double psi2 = psi1 + 1.0;            /* psi(n+2) */
    double si0 = 0.0, si1 = 0.0, sk0 = 0.0, sk1 = 0.0;
    for (int n = 0; n < 60; ++n) {
        si0 += a;
        si1 += b;
        sk0 += psi1 * a;
        sk1 += (psi1 + psi2) * b;
        if (a < 1e-18 * si0 && n > 2) break;
        a *= q / ((n + 1.0) * (n + 1.0));
        b *= q / ((n + 1.0) * (n + 2.0));
        psi1 += 1.0 / (n + 1.0);
        psi2 += 1.0 / (n + 2.0);
    }
    double i1 = 0.5 * z * si1;
    *k0 = -lz * si0 + sk0;
    *k1 = 1.0 / z + lz * i1 - 0.25 * z * sk1;
}

static void k01_integral(double z, double *k0, double *k1)
{
    /* K_nu(z) = e^{-z} int_0^inf exp(-z (cosh u - 1)) cosh(nu u) du, trapezoid
       rule with step H (exponentially convergent for this entire integrand). */
    /* the integrand is close to a Gaussian of width 1/sqrt(z) for large z */
    const double H = fmin(0.125, 0.5 / sqrt(z));
    double s0 = 0.5, s1 = 0.5;
    for (int k = 1; k < 4000; ++k) {
        double u = k * H;
        double sh = sinh(0.5 * u);
        double cm1 = 2.0 * sh * sh; /* cosh(u) - 1 without cancellation */
        double c = 1.0 + cm1;
        double e = z * cm1;
        if (e > 46.0) break;
        double v = exp(-e);
        s0 += v;
        s1 += v * c;
    }
    if (z > 740.0) {
        *k0 = 0.0;
        *k1 = 0.0;
        return;
    }
    double ez = exp(-z) * H;
    *k0 = ez * s0;
    *k1 = ez * s1;
}

/* The same two representations in long double (64-bit significand), used by
   the gradient integrand: near the curve the gradient integrals cancel by a
   factor ~h/d, so the kernel values must carry more than double precision
   for the exact panel integrals to stay accurate to double rounding. */
#define EULER_GAMMA_L 0.57721566490153286060651209008240243L
static void k01_series_ld(long double z, long double *k0, long double *k1)
{
    long double q = 0.25L * z * z;
    long double lz = logl(0.5L * z);
    long double a = 1.0L, b = 1.0L;
    long double psi1 = -EULER_GAMMA_L, psi2 = psi1 + 1.0L;
    long double si0 = 0.0L, si1 = 0.0L, sk0 = 0.0L, sk1 = 0.0L;
    for (int n = 0; n < 80; ++n) {
        si0 += a;
        si1 += b;
        sk0 += psi1 * a;
        sk1 += (psi1 + psi2) * b;
        if (a < 1e-22L * si0 && n > 2) break;
        a *= q / ((n + 1.0L) * (n + 1.0L));
        b *= q / ((n + 1.0L) * (n + 2.0L));
        psi1 += 1.0L / (n + 1.0L);
        psi2 += 1.0L / (n + 2.0L);
    }
    long double i1 = 0.5L * z * si1;
    *k0 = -lz * si0 + sk0;
    *k1 = 1.0L / z + lz * i1 - 0.25L * z * sk1;
}

static void k01_integral_ld(long double z, long double *k0, long double *k1)
{
    const long double H = fminl(0.125L, 0.4L / sqrtl(z));
    long double s0 = 0.5L, s1 = 0.5L;
    for (int k = 1; k < 8000; ++k) {
        long double u = k * H;
        long double sh = sinhl(0.5L * u);
        long double cm1 = 2.0L * sh * sh;
        long double e = z * cm1;
        if (e > 52.0L) break;
        long double v = expl(-e);
        s0 += v;
        s1 += v * (1.0L + cm1);
    }
    long double ez = expl(-z) * H;
    *k0 = ez * s0;
    *k1 = ez * s1;
}

static void bessel_k01_ld(long double z, long double *k0, long double *k1)
{
    if (z <= 2.0L)
        k01_series_ld(z, k0, k1);
    else
        k01_integral_ld(z, k0, k1);
}

void orc_bessel_k01(double z, double *k0, double *k1)
{
    if (z <= 2.0)
        k01_series(z, k0, k1);
    else
        k01_integral(z, k0, k1);
}

/* ------------------------------------------------------------------------ */
/* Panel interpolation                                                       */
/* ------------------------------------------------------------------------ */
typedef struct {
    double x[16], y[16];     /* node positions            */
    double dx[16], dy[16];   /* derivative of the degree-15 interpolant at nodes */
    long double dxl[16], dyl[16];
    double h;                /* arclength of the panel (16-pt GL)              */
} panel_t;

static void panel_setup(panel_t *p, const double *x, const double *y)
{
    memcpy(p->x, x, 16 * sizeof(double));
    memcpy(p->y, y, 16 * sizeof(double));
    double h = 0.0;
    for (int i = 0; i < 16; ++i) {
        long double sx = 0.0L, sy = 0.0L;
        for (int j = 0; j < 16; ++j) {
            sx += DIFF_L[i][j] * x[j];
            sy += DIFF_L[i][j] * y[j];
        }
        p->dxl[i] = sx;
        p->dyl[i] = sy;
        p->dx[i] = (double)sx;
        p->dy[i] = (double)sy;
        h += GL16_W[i] * hypot(p->dx[i], p->dy[i]);
    }
    p->h = h;
}

/* Integrand context.  The panel parameter is written t = tref + s, where tref
   is the target's own node parameter when the target lies on the panel (and
   0 otherwise), so that t - t_self = s is never formed by cancellation.   */
typedef struct {
    const panel_t *p;
    double tx, ty;
    double ox[16], oy[16];   /* x_j - target */
    double dref[16];         /* tref - t_j   */
    int self;                /* node index of the target on this panel, or -1 */
    double alpha;
    int grad;                /* 0: potentials (32 values), 1: gradients (64), 2: stresslet (64),
                                3: stresslet target gradient (128) */
    int nf;                  /* values per evaluation: 32 or 64              */
} integrand_t;

#define MAXF 128

/* Lagrange basis l_j(t) of the 16 nodes at t = tref + s (barycentric form).
   Long double: the normal component (x-y).n of a target lying on or beside
   the curve is a small difference of interpolated quantities.            */
static void lagrange(const integrand_t *c, double s, long double *l)
{
    long double den[16];
    for (int j = 0; j < 16; ++j) {
        den[j] = (j == c->self) ? (long double)s : ((long double)c->dref[j] + (long double)s);
        if (den[j] == 0.0) {
            for (int k = 0; k < 16; ++k) l[k] = (k == j) ? 1.0 : 0.0;
            return;
        }
    }
    long double sum = 0.0L;
    for (int j = 0; j < 16; ++j) {
        l[j] = (long double)BARY_W_L[j] / den[j];
        sum += l[j];
    }
    for (int j = 0; j < 16; ++j) l[j] /= sum;
}

/* Stresslet functions of App. B, long double:
     T1 = -(2 z^2 K0 + (z^2 + 4) z K1 - 4)/(2 pi z^4),
     T2 = (4 z^2 K0 + (z^2 + 8) z K1 - 8)/(pi z^6),
     T3 = (z K1 - 1)/(2 pi z^2)
   for z > 1.5; below, the power series of App. C with
     k0(n) = (psi(n+1) - log(z/2)) / (4^n n!^2),
     k1(n) = (2 log(z/2) - psi(n+1) - psi(n+2)) / (4^(n+1) n! (n+1)!),
     T1 = -(1/2pi) sum_{n>=1} (2 k0(n) + 4 k1(n) + k1(n-1)) z^(2n-2),
     T2 = -1/(pi z^4) + 1/(8 pi z^2) + (1/pi) sum_{n>=2} (4 k0(n) + 8 k1(n) + k1(n-1)) z^(2n-4),
     T3 = (1/2pi) sum_{n>=0} k1(n) z^(2n).                                   */
static void stresslet_T(long double z, long double *T1, long double *T2, long double *T3)
{
    const long double PI_L = 3.14159265358979323846264338327950288L;
    if (z > 1.5L) {
        long double k0, k1;
        bessel_k01_ld(z, &k0, &k1);
        long double z2 = z * z;
        *T1 = -(2.0L * z2 * k0 + (z2 + 4.0L) * z * k1 - 4.0L) / (2.0L * PI_L * z2 * z2);
        *T2 = (4.0L * z2 * k0 + (z2 + 8.0L) * z * k1 - 8.0L) / (PI_L * z2 * z2 * z2);
        *T3 = (z * k1 - 1.0L) / (2.0L * PI_L * z2);
        return;
    }
    const long double L = logl(0.5L * z), z2 = z * z;
    long double k0[40], k1[40];
    long double psi = -EULER_GAMMA_L; /* psi(n+1) */
    long double f0 = 1.0L, f1 = 0.25L; /* 1/(4^n n!^2), 1/(4^(n+1) n! (n+1)!) */
    for (int n = 0; n < 40; ++n) {
        const long double psi2 = psi + 1.0L / (n + 1.0L);
        k0[n] = (psi - L) * f0;
        k1[n] = (2.0L * L - psi - psi2) * f1;
        psi = psi2;
        f0 /= 4.0L * (n + 1.0L) * (n + 1.0L);
        f1 /= 4.0L * (n + 1.0L) * (n + 2.0L);
    }
    long double s1 = 0.0L, s2 = 0.0L, s3 = 0.0L, zp;
    zp = 1.0L; /* z^(2n-2) from n = 1 */
    for (int n = 1; n < 40; ++n, zp *= z2) s1 += (2.0L * k0[n] + 4.0L * k1[n] + k1[n - 1]) * zp;
    zp = 1.0L; /* z^(2n-4) from n = 2 */
    for (int n = 2; n < 40; ++n, zp *= z2) s2 += (4.0L * k0[n] + 8.0L * k1[n] + k1[n - 1]) * zp;
    zp = 1.0L;
    for (int n = 0; n < 40; ++n, zp *= z2) s3 += k1[n] * zp;
    *T1 = -s1 / (2.0L * PI_L);
    *T2 = -1.0L / (PI_L * z2 * z2) + 1.0L / (8.0L * PI_L * z2) + s2 / PI_L;
    *T3 = s3 / (2.0L * PI_L);
}

/* Derivatives T1'..T3' (d/dz): for z > 1.5 from K0' = -K1, (z K1)' = -z K0:
     T1' = K0/(2 pi z) - 4 T1/z,  T2' = -(z K0 + 2 K1)/(pi z^4) - 6 T2/z,
     T3' = -K0/(2 pi z) - 2 T3/z;
   below, the App. C series differentiated term by term (d log(z/2)/dz = 1/z). */
static void stresslet_dT(long double z, long double *dT1, long double *dT2, long double *dT3)
{
    const long double PI_L = 3.14159265358979323846264338327950288L;
    long double T1, T2, T3;
    stresslet_T(z, &T1, &T2, &T3);
    if (z > 1.5L) {
        long double k0, k1;
        bessel_k01_ld(z, &k0, &k1);
        *dT1 = k0 / (2.0L * PI_L * z) - 4.0L * T1 / z;
        *dT2 = -(z * k0 + 2.0L * k1) / (PI_L * z * z * z * z) - 6.0L * T2 / z;
        *dT3 = -k0 / (2.0L * PI_L * z) - 2.0L * T3 / z;
        return;
    }
    const long double L = logl(0.5L * z), z2 = z * z;
    long double a[40], b[40], k0[40], k1[40];
    long double psi = -EULER_GAMMA_L, f0 = 1.0L, f1 = 0.25L;
    for (int n = 0; n < 40; ++n) {
        const long double psi2 = psi + 1.0L / (n + 1.0L);
        a[n] = f0;
        b[n] = f1;
        k0[n] = (psi - L) * f0;
        k1[n] = (2.0L * L - psi - psi2) * f1;
        psi = psi2;
        f0 /= 4.0L * (n + 1.0L) * (n + 1.0L);
        f1 /= 4.0L * (n + 1.0L) * (n + 2.0L);
    }
    /* d/dz [c_n z^p] = (dc_n/dL) z^(p-1) + p c_n z^(p-1), dk0/dL = -a_n, dk1/dL = 2 b_n */
    long double s1 = 0.0L, s2 = 0.0L, s3 = 0.0L, zp;
    zp = 1.0L / z; /* z^(2n-3) from n = 1 */
    for (int n = 1; n < 40; ++n, zp *= z2) {
        const long double c = 2.0L * k0[n] + 4.0L * k1[n] + k1[n - 1];
        const long double dc = -2.0L * a[n] + 8.0L * b[n] + 2.0L * b[n - 1];
        s1 += (dc + (2.0L * n - 2.0L) * c) * zp;
    }
    zp = 1.0L / z; /* z^(2n-5) from n = 2 */
    for (int n = 2; n < 40; ++n, zp *= z2) {
        const long double c = 4.0L * k0[n] + 8.0L * k1[n] + k1[n - 1];
        const long double dc = -4.0L * a[n] + 16.0L * b[n] + 2.0L * b[n - 1];
        s2 += (dc + (2.0L * n - 4.0L) * c) * zp;
    }
    zp = 1.0L / z; /* z^(2n-1) from n = 0 */
    for (int n = 0; n < 40; ++n, zp *= z2) s3 += (2.0L * b[n] + 2.0L * n * k1[n]) * zp;
    *dT1 = -s1 / (2.0L * PI_L);
    *dT2 = 4.0L / (PI_L * z2 * z2 * z) - 1.0L / (4.0L * PI_L * z2 * z) + s2 / PI_L;
    *dT3 = s3 / (2.0L * PI_L);
}

void orc_stresslet_dT(double z, double *T)
{
    long double a, b, c;
    stresslet_dT(z, &a, &b, &c);
    T[0] = (double)a;
    T[1] = (double)b;
    T[2] = (double)c;
}

/* Target gradient of the stresslet double layer kernel:
   dD[(2 i + l) 2 + j] = d/dx_l D_ij(x, y), r = x - y, n = n_y, with
   A_k = a_k T_k(z), B_k = A_k'(|r|)/|r| = a_k alpha T_k'(z)/|r|, a = (alpha^2, alpha^4, alpha^2):
   d_l D_ij = -[ r_l (B1 P1_ij + B2 P2_ij + B3 P3_ij)
                 + A1 (n_i d_jl + d_il n_j + d_ij n_l)
                 + A2 (d_il r_j (r.n) + r_i d_jl (r.n) + r_i r_j n_l) + A3 d_il n_j ],
   P1 = n_i r_j + r_i n_j + d_ij (r.n), P2 = r_i r_j (r.n), P3 = r_i n_j. */
static void stresslet_dD(long double rx, long double ry, long double nx, long double ny, long double alpha,
                         long double *dD)
{
    const long double r2 = rx * rx + ry * ry, r = sqrtl(r2), z = alpha * r;
    long double T1, T2, T3, d1, d2, d3;
    stresslet_T(z, &T1, &T2, &T3);
    stresslet_dT(z, &d1, &d2, &d3);
    const long double a2 = alpha * alpha, a4 = a2 * a2;
    const long double A[3] = {a2 * T1, a4 * T2, a2 * T3};
    const long double B[3] = {a2 * alpha * d1 / r, a4 * alpha * d2 / r, a2 * alpha * d3 / r};
    const long double rv[2] = {rx, ry}, nv[2] = {nx, ny};
    const long double rn = rx * nx + ry * ny;
    for (int i = 0; i < 2; ++i)
        for (int l = 0; l < 2; ++l)
            for (int j = 0; j < 2; ++j) {
                const long double dij = i == j, dil = i == l, djl = j == l;
                const long double P1 = nv[i] * rv[j] + rv[i] * nv[j] + dij * rn;
                const long double P2 = rv[i] * rv[j] * rn, P3 = rv[i] * nv[j];
                const long double v = rv[l] * (B[0] * P1 + B[1] * P2 + B[2] * P3) +
                                      A[0] * (nv[i] * djl + dil * nv[j] + dij * nv[l]) +
                                      A[1] * (dil * rv[j] * rn + rv[i] * djl * rn + rv[i] * rv[j] * nv[l]) +
                                      A[2] * dil * nv[j];
                dD[(2 * i + l) * 2 + j] = -v;
            }
}

void orc_stresslet_T(double z, double *T)
{
    long double a, b, c;
    stresslet_T(z, &a, &b, &c);
    T[0] = (double)a;
    T[1] = (double)b;
    T[2] = (double)c;
}

/* D_ij(x, y) of the modified-Stokes double layer for r = x - y, n = n_y. */
static void stresslet_D(long double rx, long double ry, long double nx, long double ny, long double alpha,
                        long double D[2][2])
{
    const long double r2 = rx * rx + ry * ry;
    long double T1, T2, T3;
    stresslet_T(alpha * sqrtl(r2), &T1, &T2, &T3);
    const long double a2 = alpha * alpha, a4 = a2 * a2;
    const long double r[2] = {rx, ry}, n[2] = {nx, ny};
    const long double rn = rx * nx + ry * ny;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            D[i][j] = -a2 * T1 * (n[i] * r[j] + r[i] * n[j] + (i == j ? rn : 0.0L)) - a4 * T2 * r[i] * r[j] * rn -
                      a2 * T3 * r[i] * n[j];
}

/* Integrand: for a target and panel parameter t = tref + s, the values
   potentials: F[j] = G(x, y(t)) l_j(t) |y'(t)|,  F[16+j] = dG/dn_y l_j(t) |y'(t)|;
   gradients:  F[j], F[16+j] = d/dx1, d/dx2 of G(x, y(t)), F[32+j], F[48+j] the
               same of dG/dn_y, each times l_j(t) |y'(t)|;
   stresslet:  F[(2i+j)16 + l] = D_ij(x, y(t)) l_l(t) |y'(t)|.
   Differences y(t)-x are formed as sum_j l_j(t)(x_j - x) so that a target on
   the panel keeps full relative accuracy near its own node.              */
static void integrand(const integrand_t *c, double s, long double *F)
{
    long double l[16];
    lagrange(c, s, l);
    long double rx = 0.0L, ry = 0.0L, dx = 0.0L, dy = 0.0L;
    for (int j = 0; j < 16; ++j) {
        rx += l[j] * c->ox[j];
        ry += l[j] * c->oy[j];
        dx += l[j] * c->p->dxl[j];
        dy += l[j] * c->p->dyl[j];
    }
    /* y - x = (rx, ry);  (x - y).n_y |y'| = (x - y).(-dy, dx) = rx dy - ry dx */
    long double xmyn = rx * dy - ry * dx;
    if (c->grad == 3) {
        /* stresslet gradient: F[b 16 + k] = dD[b] l_k |y'|, b = (2i + l) 2 + j */
        long double speed = sqrtl(dx * dx + dy * dy);
        long double dD[8];
        stresslet_dD(-rx, -ry, -dy / speed, dx / speed, c->alpha, dD);
        for (int b = 0; b < 8; ++b)
            for (int k = 0; k < 16; ++k) F[b * 16 + k] = dD[b] * speed * l[k];
        return;
    }
    if (c->grad == 2) {
        /* stresslet: F[(2i+j)16 + l] = D_ij l_l |y'|, r = x - y = -(rx, ry) */
        long double speed = sqrtl(dx * dx + dy * dy);
        long double D[2][2];
        stresslet_D(-rx, -ry, -dy / speed, dx / speed, c->alpha, D);
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 16; ++k) F[(2 * i + j) * 16 + k] = D[i][j] * speed * l[k];
        return;
    }
    if (!c->grad) {
        double r = (double)sqrtl(rx * rx + ry * ry);
        double speed = (double)sqrtl(dx * dx + dy * dy);
        double k0, k1;
        orc_bessel_k01(c->alpha * r, &k0, &k1);
        double gs = k0 / TWO_PI * speed;
        double gd = c->alpha * k1 / (TWO_PI * r) * (double)xmyn;
        for (int j = 0; j < 16; ++j) {
            F[j] = gs * (double)l[j];
            F[16 + j] = gd * (double)l[j];
        }
        return;
    }
    /* A = alpha K1/r, B = (alpha^2 K0 + 2A)/r^2; with d = y - x,
       grad G = A d/(2 pi), grad dG/dn = (A n - (d.n) d B)/(2 pi), and
       -(d.n)|y'| = xmyn, n |y'| = (-dy, dx).  All in long double. */
    const long double al = c->alpha, tp = 2.0L * 3.14159265358979323846264338327950288L;
    long double r2 = rx * rx + ry * ry, r = sqrtl(r2);
    long double speed = sqrtl(dx * dx + dy * dy);
    long double k0, k1;
    bessel_k01_ld(al * r, &k0, &k1);
    long double A = al * k1 / r;
    long double B = (al * al * k0 + 2.0L * A) / r2;
    long double v[4];
    v[0] = A * rx * speed / tp;
    v[1] = A * ry * speed / tp;
    v[2] = (-A * dy + xmyn * rx * B) / tp;
    v[3] = (A * dx + xmyn * ry * B) / tp;
    for (int k = 0; k < 4; ++k)
        for (int j = 0; j < 16; ++j) F[16 * k + j] = v[k] * l[j];
}

static void gl_rule(const integrand_t *c, int n, const double *T, const double *W, double a, double b,
                    long double *I, long double *Iabs)
{
    double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    long double F[MAXF];
    const int nf = c->nf;
    for (int k = 0; k < nf; ++k) {
        I[k] = 0.0L;
        if (Iabs) Iabs[k] = 0.0L;
    }
    for (int i = 0; i < n; ++i) {
        integrand(c, mid + half * T[i], F);
        long double w = (long double)W[i] * half;
        for (int k = 0; k < nf; ++k) {
            I[k] += w * F[k];
            if (Iabs) Iabs[k] += w * fabsl(F[k]);
        }
    }
}

/* Adaptive bisection: accept the 32-point value on [a,b] when the 16-point
   value agrees with it to `rtol` relative (per component, relative to the
   integral of |F| over [a,b]) or to `fl` absolute (per kernel, i.e. per block
   of 16 components); the accepted 32-point value is then accurate to
   rounding.  The absolute floor bounds the work where rounding in the node
   positions of a tiny interval next to a near-singularity exceeds the
   relative test.  `absacc` (optional) collects the integral of |F| over the
   accepted pieces.                                                        */
typedef struct { double a, b; int d; } seg_t;
/* Pieces accepted only because the bisection ran out of stack or of visits
   (not converged).  Every public entry point that integrates clears the count
   and returns ORC_ERR_QUAD when it is nonzero at the end.  Pieces accepted at
   depth 60 or below 1e-17 in width are not counted: they only arise next to a
   target on the panel (graded towards it), where they hold a negligible part
   of the integral. */
static long orc_quad_unconverged = 0;
#define ORC_ERR_QUAD (-3)
static void adaptive(const integrand_t *c, double a, double b, double rtol, const double *fl, long double *acc,
                     long double *absacc)
{
    seg_t stack[128];
    int top = 0, visited = 0;
    const int nf = c->nf;
    stack[top++] = (seg_t){a, b, 0};
    while (top > 0) {
        seg_t s = stack[--top];
        ++visited;
        long double I16[MAXF], I32[MAXF], A32[MAXF];
        gl_rule(c, 16, GL16_T, GL16_W, s.a, s.b, I16, NULL);
        gl_rule(c, 32, GL32_T, GL32_W, s.a, s.b, I32, A32);
        int ok = 1;
        for (int k = 0; k < nf; ++k) {
            double e = (double)fabsl(I16[k] - I32[k]);
            if (e > rtol * (double)A32[k] && e > fl[k >> 4] && e > 1e-300) {
                ok = 0;
                break;
            }
        }
        const int starved = !(ok || s.d >= 60 || (s.b - s.a) < 1e-17) && (top > 124 || visited > 200000);
        if (starved) {
#pragma omp atomic
            ++orc_quad_unconverged;
        }
        if (ok || s.d >= 60 || (s.b - s.a) < 1e-17 || starved) {
            for (int k = 0; k < nf; ++k) acc[k] += I32[k];
            if (absacc)
                for (int k = 0; k < nf; ++k) absacc[k] += A32[k];
        } else {
            double m = 0.5 * (s.a + s.b);
            stack[top++] = (seg_t){m, s.b, s.d + 1};
            stack[top++] = (seg_t){s.a, m, s.d + 1};
        }
    }
}

/* Two passes over the pieces [cuts[q], cuts[q+1]]: a loose one (1e-8) that
   measures the pair's scale S (max over basis functions of int |F|, per
   kernel), then the accurate one with absolute floor 2e-16 S.  The loose
   pass itself uses a floor of 1e-12 of a 32-point estimate of that scale. */
static void integrate_pieces(const integrand_t *c, const double *cuts, int ncut, double *W)
{
    const int nf = c->nf, nk = c->nf / 16;
    long double tmp[MAXF], ab[MAXF], acc[MAXF];
    double fl0[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, fl[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    /* the accurate pass of the gradient kernels (long double arithmetic) is
       judged against a finer floor */
    const double floor_rel = (c->grad == 1 || c->grad == 3) ? 2e-18 : 2e-16;
    for (int k = 0; k < nf; ++k) tmp[k] = ab[k] = acc[k] = 0.0L;
    for (int q = 0; q + 1 < ncut; ++q) {
        long double I[MAXF], A[MAXF];
        gl_rule(c, 32, GL32_T, GL32_W, cuts[q], cuts[q + 1], I, A);
        for (int k = 0; k < nf; ++k) fl0[k >> 4] = fmax(fl0[k >> 4], (double)A[k]);
    }
    for (int b = 0; b < nk; ++b) fl0[b] *= 1e-12;
    for (int q = 0; q + 1 < ncut; ++q) adaptive(c, cuts[q], cuts[q + 1], 1e-8, fl0, tmp, ab);
    for (int k = 0; k < nf; ++k) fl[k >> 4] = fmax(fl[k >> 4], (double)ab[k]);
    for (int b = 0; b < nk; ++b) fl[b] *= floor_rel;
    for (int q = 0; q + 1 < ncut; ++q)
        adaptive(c, cuts[q], cuts[q + 1], (c->grad == 1 || c->grad == 3) ? ORC_RTOL_GRAD : ORC_RTOL, fl, acc, NULL);
    for (int k = 0; k < nf; ++k) W[k] = (double)acc[k];
}

/* Exact panel weights W[0..15] (SLP) and W[16..31] (DLP) of target (tx,ty)
   against panel p; with grad, W[0..63] = d/dx1, d/dx2 of the SLP, then of the
   DLP.  If self >= 0 the target is node `self` of this panel and
   the integral is split there with geometric grading towards it.          */
static void panel_exact_k(const panel_t *p, double tx, double ty, double alpha, int self, int grad, double *W)
{
    integrand_t c;
    c.grad = grad;
    c.nf = grad == 3 ? 128 : grad ? 64 : 32; /* 2, 4 or 8 blocks of 16 */
    c.p = p;
    c.tx = tx;
    c.ty = ty;
    c.alpha = alpha;
    for (int j = 0; j < 16; ++j) {
        c.ox[j] = p->x[j] - tx;
        c.oy[j] = p->y[j] - ty;
    }
    c.self = self;
    double tref = (self >= 0) ? GL16_T[self] : 0.0;
    for (int j = 0; j < 16; ++j) c.dref[j] = tref - GL16_T[j];
    if (self >= 0) {
        c.ox[self] = 0.0;
        c.oy[self] = 0.0;
    }
    if (self < 0) {
        double cuts[2] = {-1.0, 1.0};
        integrate_pieces(&c, cuts, 2, W);
        return;
    }
    /* target on the panel: pieces graded geometrically towards it, in the
       local coordinate s = t - t_self */
    double ts = GL16_T[self];
    enum { LEV = 56 };
    double cuts[2 * LEV + 2];
    int nc = 0;
    for (int k = 0; k < LEV; ++k) cuts[nc++] = (-1.0 - ts) * ldexp(1.0, -k);
    cuts[nc++] = 0.0;
    for (int k = LEV - 1; k >= 0; --k) cuts[nc++] = (1.0 - ts) * ldexp(1.0, -k);
    integrate_pieces(&c, cuts, nc, W);
}

static void panel_exact(const panel_t *p, double tx, double ty, double alpha, int self, double *W)
{
    panel_exact_k(p, tx, ty, alpha, self, 0, W);
}

/* direct 16-point weights: K(x, y_j) |y'(t_j)| lambda_j */
static void panel_direct(const panel_t *p, double tx, double ty, double alpha, double *W)
{
    for (int j = 0; j < 16; ++j) {
        double rx = p->x[j] - tx, ry = p->y[j] - ty;
        double r = hypot(rx, ry);
        double k0, k1;
        orc_bessel_k01(alpha * r, &k0, &k1);
        double speed = hypot(p->dx[j], p->dy[j]);
        double xmyn = rx * p->dy[j] - ry * p->dx[j];
        W[j] = k0 / TWO_PI * speed * GL16_W[j];
        W[16 + j] = alpha * k1 / (TWO_PI * r) * xmyn * GL16_W[j];
    }
}

/* direct 16-point gradient weights (same layout as the exact ones) */
static void panel_direct_grad(const panel_t *p, double tx, double ty, double alpha, double *W)
{
    for (int j = 0; j < 16; ++j) {
        double rx = p->x[j] - tx, ry = p->y[j] - ty;
        double r = hypot(rx, ry);
        double k0, k1;
        orc_bessel_k01(alpha * r, &k0, &k1);
        double speed = hypot(p->dx[j], p->dy[j]);
        double xmyn = rx * p->dy[j] - ry * p->dx[j];
        double A = alpha * k1 / r;
        double B = (alpha * alpha * k0 + 2.0 * A) / (r * r);
        double w = GL16_W[j] / TWO_PI;
        W[j] = A * rx * speed * w;
        W[16 + j] = A * ry * speed * w;
        W[32 + j] = (-A * p->dy[j] + xmyn * rx * B) * w;
        W[48 + j] = (A * p->dx[j] + xmyn * ry * B) * w;
    }
}

/* direct 16-point stresslet weights (same layout as the exact ones) */
static void panel_direct_stokes(const panel_t *p, double tx, double ty, double alpha, double *W)
{
    for (int j = 0; j < 16; ++j) {
        long double speed = sqrtl(p->dxl[j] * p->dxl[j] + p->dyl[j] * p->dyl[j]);
        long double D[2][2];
        stresslet_D((long double)tx - p->x[j], (long double)ty - p->y[j], -p->dyl[j] / speed, p->dxl[j] / speed,
                     alpha, D);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) W[(2 * a + b) * 16 + j] = (double)(D[a][b] * speed * GL16_W[j]);
    }
}

/* direct 16-point weights of the stresslet gradient (128 values) */
static void panel_direct_stokes_grad(const panel_t *p, double tx, double ty, double alpha, double *W)
{
    for (int j = 0; j < 16; ++j) {
        long double speed = sqrtl(p->dxl[j] * p->dxl[j] + p->dyl[j] * p->dyl[j]);
        long double dD[8];
        stresslet_dD((long double)tx - p->x[j], (long double)ty - p->y[j], -p->dyl[j] / speed, p->dxl[j] / speed,
                     alpha, dD);
        for (int b = 0; b < 8; ++b) W[b * 16 + j] = (double)(dD[b] * speed * GL16_W[j]);
    }
}

static int panel_is_near(const panel_t *p, double tx, double ty)
{
    double lim = 2.0 * p->h;
    for (int j = 0; j < 16; ++j)
        if (hypot(p->x[j] - tx, p->y[j] - ty) < lim) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                       */
/* ------------------------------------------------------------------------ */
static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Weights of one target against one panel (W: 32 doubles). mode: 0 auto,
   1 force exact, 2 force direct.  self: node index of the target on this
   panel, or -1. */
int orc_panel_weights(const double *x, const double *y, int64_t panel, double tx, double ty, double alpha,
                      int self, int mode, double *W)
{
    orc_quad_unconverged = 0;
    init_rules();
    panel_t p;
    panel_setup(&p, x + 16 * panel, y + 16 * panel);
    if (mode == 2 && self < 0)
        panel_direct(&p, tx, ty, alpha, W);
    else if (mode == 1 || self >= 0 || panel_is_near(&p, tx, ty))
        panel_exact(&p, tx, ty, alpha, self, W);
    else
        panel_direct(&p, tx, ty, alpha, W);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Layer potentials at m targets.  tgt_node[i] >= 0 marks target i as boundary
   node tgt_node[i] (its own panel is then integrated with the singular split);
   pass NULL for off-surface targets.  sigma/mu/u_slp/u_dlp may be NULL. */
int orc_eval(const double *x, const double *y, int64_t n_panels, const double *sigma, const double *mu,
             double alpha, const double *tx, const double *ty, int64_t m, const int64_t *tgt_node,
             double *u_slp, double *u_dlp, int nthreads)
{
    orc_quad_unconverged = 0;
    init_rules();
    if (alpha <= 0.0 || n_panels <= 0 || m < 0) return -1;
    panel_t *P = (panel_t *)malloc(sizeof(panel_t) * (size_t)n_panels);
    if (!P) return -2;
    for (int64_t p = 0; p < n_panels; ++p) panel_setup(&P[p], x + 16 * p, y + 16 * p);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < m; ++i) {
        long double us = 0.0L, ud = 0.0L;
        int64_t node = tgt_node ? tgt_node[i] : -1;
        for (int64_t p = 0; p < n_panels; ++p) {
            double W[32];
            int self = (node >= 0 && node / 16 == p) ? (int)(node % 16) : -1;
            if (self >= 0 || panel_is_near(&P[p], tx[i], ty[i]))
                panel_exact(&P[p], tx[i], ty[i], alpha, self, W);
            else
                panel_direct(&P[p], tx[i], ty[i], alpha, W);
            for (int j = 0; j < 16; ++j) {
                if (sigma) us += (long double)W[j] * sigma[16 * p + j];
                if (mu) ud += (long double)W[16 + j] * mu[16 * p + j];
            }
        }
        if (u_slp) u_slp[i] = (double)us;
        if (u_dlp) u_dlp[i] = (double)ud;
    }
    free(P);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Gradient weights of one off-surface target against one panel (W: 64
   doubles, blocks d/dx1 SLP, d/dx2 SLP, d/dx1 DLP, d/dx2 DLP).  mode: 0 auto,
   1 force exact, 2 force direct. */
int orc_panel_grad_weights(const double *x, const double *y, int64_t panel, double tx, double ty, double alpha,
                           int mode, double *W)
{
    orc_quad_unconverged = 0;
    init_rules();
    panel_t p;
    panel_setup(&p, x + 16 * panel, y + 16 * panel);
    if (mode == 2)
        panel_direct_grad(&p, tx, ty, alpha, W);
    else if (mode == 1 || panel_is_near(&p, tx, ty))
        panel_exact_k(&p, tx, ty, alpha, -1, 1, W);
    else
        panel_direct_grad(&p, tx, ty, alpha, W);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Gradients of S[sigma] and D[mu] at m off-surface targets (targets must not
   lie on the curve).  Outputs (any may be NULL with its density):
   gsx, gsy = grad S[sigma];  gdx, gdy = grad D[mu]. */
int orc_eval_grad(const double *x, const double *y, int64_t n_panels, const double *sigma, const double *mu,
                  double alpha, const double *tx, const double *ty, int64_t m, double *gsx, double *gsy,
                  double *gdx, double *gdy, int nthreads)
{
    orc_quad_unconverged = 0;
    init_rules();
    if (alpha <= 0.0 || n_panels <= 0 || m < 0) return -1;
    panel_t *P = (panel_t *)malloc(sizeof(panel_t) * (size_t)n_panels);
    if (!P) return -2;
    for (int64_t p = 0; p < n_panels; ++p) panel_setup(&P[p], x + 16 * p, y + 16 * p);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < m; ++i) {
        long double a[4] = {0.0L, 0.0L, 0.0L, 0.0L};
        for (int64_t p = 0; p < n_panels; ++p) {
            double W[64];
            if (panel_is_near(&P[p], tx[i], ty[i]))
                panel_exact_k(&P[p], tx[i], ty[i], alpha, -1, 1, W);
            else
                panel_direct_grad(&P[p], tx[i], ty[i], alpha, W);
            for (int j = 0; j < 16; ++j) {
                if (sigma) {
                    a[0] += (long double)W[j] * sigma[16 * p + j];
                    a[1] += (long double)W[16 + j] * sigma[16 * p + j];
                }
                if (mu) {
                    a[2] += (long double)W[32 + j] * mu[16 * p + j];
                    a[3] += (long double)W[48 + j] * mu[16 * p + j];
                }
            }
        }
        if (gsx) gsx[i] = (double)a[0];
        if (gsy) gsy[i] = (double)a[1];
        if (gdx) gdx[i] = (double)a[2];
        if (gdy) gdy[i] = (double)a[3];
    }
    free(P);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Stresslet weights of one target against one panel (W: 64 doubles, block
   2i+j = D_ij).  self: node of the target on this panel or -1.  mode: 0 auto,
   1 exact, 2 direct. */
int orc_stokes_panel_weights(const double *x, const double *y, int64_t panel, double tx, double ty, double alpha,
                             int self, int mode, double *W)
{
    orc_quad_unconverged = 0;
    init_rules();
    panel_t p;
    panel_setup(&p, x + 16 * panel, y + 16 * panel);
    if (mode == 2 && self < 0)
        panel_direct_stokes(&p, tx, ty, alpha, W);
    else if (mode == 1 || self >= 0 || panel_is_near(&p, tx, ty))
        panel_exact_k(&p, tx, ty, alpha, self, 2, W);
    else
        panel_direct_stokes(&p, tx, ty, alpha, W);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Modified-Stokes double layer D[mu] at m targets (mu1, mu2: the density's
   components at the N nodes; u1, u2: outputs).  tgt_node[i] >= 0 marks target
   i as that boundary node (principal value, no 1/2 mu term); NULL for
   off-surface targets. */
int orc_stokes_eval(const double *x, const double *y, int64_t n_panels, const double *mu1, const double *mu2,
                    double alpha, const double *tx, const double *ty, int64_t m, const int64_t *tgt_node,
                    double *u1, double *u2, int nthreads)
{
    orc_quad_unconverged = 0;
    init_rules();
    if (alpha <= 0.0 || n_panels <= 0 || m < 0) return -1;
    panel_t *P = (panel_t *)malloc(sizeof(panel_t) * (size_t)n_panels);
    if (!P) return -2;
    for (int64_t p = 0; p < n_panels; ++p) panel_setup(&P[p], x + 16 * p, y + 16 * p);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < m; ++i) {
        long double a1 = 0.0L, a2 = 0.0L;
        int64_t node = tgt_node ? tgt_node[i] : -1;
        for (int64_t p = 0; p < n_panels; ++p) {
            double W[64];
            int self = (node >= 0 && node / 16 == p) ? (int)(node % 16) : -1;
            if (self >= 0 || panel_is_near(&P[p], tx[i], ty[i]))
                panel_exact_k(&P[p], tx[i], ty[i], alpha, self, 2, W);
            else
                panel_direct_stokes(&P[p], tx[i], ty[i], alpha, W);
            for (int j = 0; j < 16; ++j) {
                const long double m1 = mu1[16 * p + j], m2 = mu2[16 * p + j];
                a1 += (long double)W[j] * m1 + (long double)W[16 + j] * m2;
                a2 += (long double)W[32 + j] * m1 + (long double)W[48 + j] * m2;
            }
        }
        u1[i] = (double)a1;
        u2[i] = (double)a2;
    }
    free(P);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Stresslet-gradient weights of one off-surface target against one panel
   (W: 128 doubles, block (2i + l) 2 + j = d/dx_l D_ij).  mode: 0 auto,
   1 exact, 2 direct. */
int orc_stokes_grad_panel_weights(const double *x, const double *y, int64_t panel, double tx, double ty,
                                  double alpha, int mode, double *W)
{
    orc_quad_unconverged = 0;
    init_rules();
    panel_t p;
    panel_setup(&p, x + 16 * panel, y + 16 * panel);
    if (mode == 2)
        panel_direct_stokes_grad(&p, tx, ty, alpha, W);
    else if (mode == 1 || panel_is_near(&p, tx, ty))
        panel_exact_k(&p, tx, ty, alpha, -1, 3, W);
    else
        panel_direct_stokes_grad(&p, tx, ty, alpha, W);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Target gradient of the stresslet double layer at m off-surface targets:
   g[c * m + i] = d/dx_l u_a(x_i) for c = 2a + l (du1/dx1, du1/dx2, du2/dx1,
   du2/dx2). */
int orc_stokes_grad_eval(const double *x, const double *y, int64_t n_panels, const double *mu1, const double *mu2,
                         double alpha, const double *tx, const double *ty, int64_t m, double *g, int nthreads)
{
    orc_quad_unconverged = 0;
    init_rules();
    if (alpha <= 0.0 || n_panels <= 0 || m < 0) return -1;
    panel_t *P = (panel_t *)malloc(sizeof(panel_t) * (size_t)n_panels);
    if (!P) return -2;
    for (int64_t p = 0; p < n_panels; ++p) panel_setup(&P[p], x + 16 * p, y + 16 * p);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 2)
    for (int64_t i = 0; i < m; ++i) {
        long double acc[4] = {0.0L, 0.0L, 0.0L, 0.0L};
        for (int64_t p = 0; p < n_panels; ++p) {
            double W[128];
            if (panel_is_near(&P[p], tx[i], ty[i]))
                panel_exact_k(&P[p], tx[i], ty[i], alpha, -1, 3, W);
            else
                panel_direct_stokes_grad(&P[p], tx[i], ty[i], alpha, W);
            for (int c = 0; c < 4; ++c)
                for (int k = 0; k < 16; ++k)
                    acc[c] += (long double)W[(2 * c) * 16 + k] * mu1[16 * p + k] +
                              (long double)W[(2 * c + 1) * 16 + k] * mu2[16 * p + k];
        }
        for (int c = 0; c < 4; ++c) g[c * m + i] = (double)acc[c];
    }
    free(P);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Dense on-surface principal-value stresslet matrix (2N x 2N, row-major):
   row a N + i (component a at node i), column b N + j. */
int orc_stokes_matrix(const double *x, const double *y, int64_t n_panels, double alpha, double *Dm, int nthreads)
{
    orc_quad_unconverged = 0;
    init_rules();
    if (alpha <= 0.0 || n_panels <= 0) return -1;
    int64_t N = 16 * n_panels;
    panel_t *P = (panel_t *)malloc(sizeof(panel_t) * (size_t)n_panels);
    if (!P) return -2;
    for (int64_t p = 0; p < n_panels; ++p) panel_setup(&P[p], x + 16 * p, y + 16 * p);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t p = 0; p < n_panels; ++p) {
            double W[64];
            int self = (i / 16 == p) ? (int)(i % 16) : -1;
            if (self >= 0 || panel_is_near(&P[p], x[i], y[i]))
                panel_exact_k(&P[p], x[i], y[i], alpha, self, 2, W);
            else
                panel_direct_stokes(&P[p], x[i], y[i], alpha, W);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    for (int j = 0; j < 16; ++j) Dm[(a * N + i) * 2 * N + b * N + 16 * p + j] = W[(2 * a + b) * 16 + j];
        }
    }
    free(P);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* Dense on-surface matrices (row-major N x N): S (SLP) and D (DLP, principal
   value, WITHOUT the 1/2 identity).  Either output may be NULL. */
int orc_assemble_onsurface(const double *x, const double *y, int64_t n_panels, double alpha, double *S,
                           double *D, int nthreads)
{
    orc_quad_unconverged = 0;
    init_rules();
    if (alpha <= 0.0 || n_panels <= 0) return -1;
    int64_t N = 16 * n_panels;
    panel_t *P = (panel_t *)malloc(sizeof(panel_t) * (size_t)n_panels);
    if (!P) return -2;
    for (int64_t p = 0; p < n_panels; ++p) panel_setup(&P[p], x + 16 * p, y + 16 * p);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t p = 0; p < n_panels; ++p) {
            double W[32];
            int self = (i / 16 == p) ? (int)(i % 16) : -1;
            if (self >= 0 || panel_is_near(&P[p], x[i], y[i]))
                panel_exact(&P[p], x[i], y[i], alpha, self, W);
            else
                panel_direct(&P[p], x[i], y[i], alpha, W);
            for (int j = 0; j < 16; ++j) {
                if (S) S[i * N + 16 * p + j] = W[j];
                if (D) D[i * N + 16 * p + j] = W[16 + j];
            }
        }
    }
    free(P);
    return orc_quad_unconverged ? ORC_ERR_QUAD : 0;
}

/* ------------------------------------------------------------------------ */
/* GMRES (Saad & Schultz), modified Gram-Schmidt, Givens rotations, restarts. */
/* A is dense row-major n x n.  Stops on the true relative residual           */
/* ||b - A x|| / ||b|| <= tol.  x holds the initial guess on entry.           */
/* ------------------------------------------------------------------------ */
static void matvec(const double *A, int64_t n, const double *v, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        long double s = 0.0L;
        const double *row = A + i * n;
        for (int64_t j = 0; j < n; ++j) s += (long double)row[j] * v[j];
        out[i] = (double)s;
    }
}

static double norm2(const double *v, int64_t n)
{
    long double s = 0.0L;
    for (int64_t i = 0; i < n; ++i) s += (long double)v[i] * v[i];
    return sqrt((double)s);
}

int orc_gmres(const double *A, int64_t n, const double *b, double *x, double tol, int restart, int max_iter,
              int *iters_out, double *relres_out, int nthreads)
{
    set_threads(nthreads);
    int m = restart;
    double *V = (double *)calloc((size_t)(m + 1) * n, sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)calloc(m, sizeof(double)), *sn = (double *)calloc(m, sizeof(double));
    double *g = (double *)calloc(m + 1, sizeof(double)), *yv = (double *)calloc(m, sizeof(double));
    double *r = (double *)calloc(n, sizeof(double)), *w = (double *)calloc(n, sizeof(double));
    double bn = norm2(b, n);
    int iters = 0;
    double rel = 0.0;
    if (bn == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        goto done;
    }
    for (;;) {
        matvec(A, n, x, w);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
        double beta = norm2(r, n);
        rel = beta / bn;
        if (rel <= tol || iters >= max_iter) break;
        for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int k = 0; k <= m; ++k) g[k] = 0.0;
        g[0] = beta;
        int k;
        for (k = 0; k < m && iters < max_iter; ++k) {
            ++iters;
            matvec(A, n, V + (int64_t)k * n, w);
            for (int j = 0; j <= k; ++j) {
                long double s = 0.0L;
                const double *vj = V + (int64_t)j * n;
                for (int64_t i = 0; i < n; ++i) s += (long double)vj[i] * w[i];
                H[j * m + k] = (double)s;
                for (int64_t i = 0; i < n; ++i) w[i] -= H[j * m + k] * vj[i];
            }
            double hn = norm2(w, n);
            H[(k + 1) * m + k] = hn;
            if (hn > 0.0)
                for (int64_t i = 0; i < n; ++i) V[(int64_t)(k + 1) * n + i] = w[i] / hn;
            for (int j = 0; j < k; ++j) {
                double a = H[j * m + k], c = H[(j + 1) * m + k];
                H[j * m + k] = cs[j] * a + sn[j] * c;
                H[(j + 1) * m + k] = -sn[j] * a + cs[j] * c;
            }
            double a = H[k * m + k], c = H[(k + 1) * m + k];
            double den = hypot(a, c);
            cs[k] = a / den;
            sn[k] = c / den;
            H[k * m + k] = den;
            H[(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            if (fabs(g[k + 1]) / bn <= 0.5 * tol || hn == 0.0) {
                ++k;
                break;
            }
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * yv[j];
            yv[i] = s / H[i * m + i];
        }
        for (int j = 0; j < k; ++j)
            for (int64_t i = 0; i < n; ++i) x[i] += yv[j] * V[(int64_t)j * n + i];
    }
done:
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = rel;
    free(V); free(H); free(cs); free(sn); free(g); free(yv); free(r); free(w);
    return rel <= tol ? 0 : 1;
}

/* ------------------------------------------------------------------------ */
/* Volume all-pairs sum with self-cell correction (trapezoid grid).           */
/* u_i = sum_{j != i} K0(alpha |x_i - x_j|)/(2 pi) w_j f_j + (w_i/h^2) Wcell f_i */
/* Wcell = int over the h x h cell centred at the target of K0(alpha|x|)/(2pi)  */
/*       = (1/2pi) 8 int_0^{pi/4} (1 - a K1(a))/alpha^2 dtheta,                  */
/*         a = alpha h / (2 cos theta)   (uses int_0^R K0(alpha s) s ds           */
/*                                        = (1 - alpha R K1(alpha R))/alpha^2).   */
/* ------------------------------------------------------------------------ */
double orc_self_cell(double alpha, double h)
{
    init_rules();
    /* composite 32-point GL on [0, pi/4] split in 8 pieces (smooth integrand) */
    double acc = 0.0;
    const int P = 8;
    double L = M_PI / 4.0;
    for (int q = 0; q < P; ++q) {
        double a0 = L * q / P, a1 = L * (q + 1) / P;
        double mid = 0.5 * (a0 + a1), half = 0.5 * (a1 - a0);
        for (int i = 0; i < 32; ++i) {
            double th = mid + half * GL32_T[i];
            double R = 0.5 * h / cos(th);
            double k0, k1;
            orc_bessel_k01(alpha * R, &k0, &k1);
            acc += GL32_W[i] * half * (1.0 - alpha * R * k1) / (alpha * alpha);
        }
    }
    return 8.0 * acc / TWO_PI;
}

int orc_volume_eval(const double *x, const double *y, const double *w, const double *f, int64_t n, double alpha,
                    double h, const int64_t *idx, int64_t m, double *out, int nthreads)
{
    init_rules();
    double wc = orc_self_cell(alpha, h);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < m; ++q) {
        int64_t i = idx[q];
        long double s = 0.0L;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r = hypot(x[i] - x[j], y[i] - y[j]);
            double k0, k1;
            orc_bessel_k01(alpha * r, &k0, &k1);
            s += (long double)(k0 / TWO_PI * w[j] * f[j]);
        }
        s += (long double)(w[i] / (h * h) * wc * f[i]);
        out[q] = (double)s;
    }
    return 0;
}

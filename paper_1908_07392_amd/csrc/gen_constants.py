"""Generate ``constants.h``: Gauss-Legendre rules, interpolation matrices and the
polynomial coefficients of the device K0/K1 evaluators.

Run:  python paper_1908_07392_amd/csrc/gen_constants.py   (needs mpmath, numpy)

Device K0/K1 (modified Bessel functions of the second kind):
* z <= 2: the log-split form of the small-argument expansions (paper, App. C;
  DLMF 10.31): with q = z^2/4,
      K0(z) = -log(z/2) I0(z) + R0(q),
      K1(z) = 1/z + log(z/2) I1(z) - (z/4) R1(q),
  where I0, I1(z)/z, R0, R1 are entire in q; each is stored as a Chebyshev-
  economised polynomial in q on [0, 1], fitted here in 40-digit arithmetic.
* z > 2: e^z sqrt(z) K_nu(z) is smooth in u = 4/z - 1 in (-1, 1]; it is stored
  as a polynomial in u (Chebyshev interpolant of degree 22 for FP64 and 9 for
  FP32, converted to monomial form; coefficients stay O(1)).
* z > 2, two pieces for the FP64 far-field tiles: z in [2, 6] (u in [-1/3, 1],
  local v = 1.5 u - 0.5) and z >= 6 (u in (-1, -1/3], v = 3 u + 2); K0 to degree
  16 / 15 so that K1 = -K0' taken from the derivative of the fit is also
  accurate, K1 alone to degree 14 / 13.
* z > 6 split again at z = 20 (KP0M / KP0X, KP1M / KP1X): each of K0 and K1
  fitted on its own (the kernels that take these pieces evaluate K1 from its
  fit, not from K0's derivative), degree 11 / 9 and 10 / 8.
* z > 2, eight finer pieces split at z = 3, 4.5, 7, 12, 20, 40, 100 and the
  seven pieces spanning two neighbours (KQ0_k for K0, KQ1_k for K1, each a fit
  of its own), degrees 12 down to 6 from the 1.2e-16 requirement on the value;
  KQF0 / KQF1 the same pieces in FP32 (degrees 5 down to 2, about 1e-7).
"""
import os

import mpmath as mp
import numpy as np

mp.mp.dps = 40
HERE = os.path.dirname(os.path.abspath(__file__))


def cheb_fit_mono(f, deg, lo, hi):
    """Chebyshev interpolant of f on [lo, hi] (degree deg), returned as monomial
    coefficients in v = (2x - lo - hi)/(hi - lo)."""
    N = deg + 1
    xs = [(mp.mpf(hi) + lo) / 2 + (mp.mpf(hi) - lo) / 2 * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / N) for k in range(N)]
    ys = [f(x) for x in xs]
    c = [2 * mp.fsum(ys[j] * mp.cos(mp.pi * k * (j + mp.mpf(1) / 2) / N) for j in range(N)) / N for k in range(N)]
    c[0] /= 2
    T = [[mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]]
    for k in range(2, N):
        a = [mp.mpf(0)] + [2 * v for v in T[-1]]
        b = T[-2] + [mp.mpf(0)] * (len(a) - len(T[-2]))
        T.append([x - y for x, y in zip(a, b)])
    m = [mp.mpf(0)] * N
    for k in range(N):
        for i, v in enumerate(T[k]):
            m[i] += c[k] * v
    return m


def large_fn(nu):
    def f(u):
        if u + 1 < mp.mpf("1e-30"):
            return mp.sqrt(mp.pi / 2)
        z = 4 / (u + 1)
        return mp.e ** z * mp.sqrt(z) * mp.besselk(nu, z)
    return f


def small_fns():
    def I0(q):
        z = 2 * mp.sqrt(q)
        return mp.besseli(0, z)

    def I1z(q):
        z = 2 * mp.sqrt(q)
        return mp.mpf(1) / 2 if q == 0 else mp.besseli(1, z) / z

    def R0(q):
        if q == 0:
            return -mp.euler
        z = 2 * mp.sqrt(q)
        return mp.besselk(0, z) + mp.log(z / 2) * mp.besseli(0, z)

    def R1(q):
        # K1 = 1/z + log(z/2) I1 - (z/4) R1
        if q == 0:
            return 1 - 2 * mp.euler
        z = 2 * mp.sqrt(q)
        return (1 / z + mp.log(z / 2) * mp.besseli(1, z) - mp.besselk(1, z)) * 4 / z
    return dict(I0=I0, I1Z=I1z, R0=R0, R1=R1)


def stokes_small_fns():
    """Smooth parts of the stresslet functions (paper Sec. 4.1, App. B) as
    functions of q = z^2/4:  T1 = T1S + T1L log z,  T3 = T3S + T3L log z,
    T2 = T2S + T2L log z + 1/(8 pi z^2) - 1/(pi z^4); evaluated from the closed
    forms in 40-digit arithmetic (Chebyshev nodes are interior, q > 0)."""
    def zq(q):
        return 2 * mp.sqrt(q)

    def T(z):
        K0, K1 = mp.besselk(0, z), mp.besselk(1, z)
        return (-(2 * z ** 2 * K0 + (z ** 2 + 4) * z * K1 - 4) / (2 * mp.pi * z ** 4),
                (4 * z ** 2 * K0 + (z ** 2 + 8) * z * K1 - 8) / (mp.pi * z ** 6),
                (z * K1 - 1) / (2 * mp.pi * z ** 2))

    def TL(z):
        I0, I1 = mp.besseli(0, z), mp.besseli(1, z)
        return ((2 * z * I0 - (z ** 2 + 4) * I1) / (2 * mp.pi * z ** 3),
                ((z ** 2 + 8) * I1 - 4 * z * I0) / (mp.pi * z ** 5),
                I1 / (2 * mp.pi * z))

    def S(i):
        def f(q):
            with mp.workdps(80):
                z = zq(mp.mpf(q))
                t, tl = T(z), TL(z)
                v = t[i] - tl[i] * mp.log(z)
                if i == 1:
                    v -= 1 / (8 * mp.pi * z ** 2) - 1 / (mp.pi * z ** 4)
                return +v
        return f

    def L(i):
        def f(q):
            with mp.workdps(80):
                return +TL(zq(mp.mpf(q)))[i]
        return f
    return {f"STK_S{i + 1}": S(i) for i in range(3)} | {f"STK_L{i + 1}": L(i) for i in range(3)}


def check_abs(coef, f):
    qs = np.linspace(1e-6, 1, 400)
    cc = np.array([float(c) for c in coef])
    v = np.zeros_like(qs)
    for a in cc[::-1]:
        v = v * qs + a
    ref = np.array([float(f(mp.mpf(q))) for q in qs])
    return float(np.max(np.abs(v - ref)) / np.max(np.abs(ref)))


def mono_in_q(f, deg):
    """Fit on q in [0, 1] with v = 2q - 1, then expand to powers of q."""
    m = cheb_fit_mono(f, deg, 0, 1)
    # p(v) with v = 2q - 1  ->  coefficients in q
    N = len(m)
    out = [mp.mpf(0)] * N
    for i, a in enumerate(m):
        # (2q - 1)^i
        for k in range(i + 1):
            out[k] += a * mp.binomial(i, k) * (2 ** k) * (-1) ** (i - k)
    return out


def check_small(coef, f, dtype):
    qs = np.linspace(0, 1, 400)
    v = np.zeros_like(qs, dtype=dtype)
    cc = np.array([float(c) for c in coef], dtype=dtype)
    for a in cc[::-1]:
        v = (v * qs.astype(dtype) + a).astype(dtype)
    ref = np.array([float(f(mp.mpf(q))) for q in qs])
    return float(np.max(np.abs(v - ref) / np.abs(ref)))


def check_large(coef, f, dtype):
    us = np.linspace(-0.9999, 1.0, 400)
    v = np.zeros_like(us, dtype=dtype)
    cc = np.array([float(c) for c in coef], dtype=dtype)
    for a in cc[::-1]:
        v = (v * us.astype(dtype) + a).astype(dtype)
    ref = np.array([float(f(mp.mpf(u))) for u in us])
    return float(np.max(np.abs(v - ref) / np.abs(ref)))


def check_piece(coef, nu, lo, hi, with_derivative):
    """max rel. error of K_nu (and of K1 from the derivative of a K0 fit) on a piece"""
    dvdu = 2.0 / (hi - lo)
    e0 = e1 = 0.0
    for x in np.linspace(0.0, 1.0, 200):
        u = mp.mpf(lo) + (mp.mpf(hi) - lo) * mp.mpf(x)
        if u <= -1:
            u = mp.mpf(-1) + mp.mpf("1e-6")
        z = 4 / (u + 1)
        v = (2 * u - lo - hi) / (mp.mpf(hi) - lo)
        p = mp.fsum(c * v ** i for i, c in enumerate(coef))
        E = mp.e ** (-z) / mp.sqrt(z)
        e0 = max(e0, float(abs(E * p / mp.besselk(nu, z) - 1)))
        if with_derivative:
            dp = mp.fsum(i * c * v ** (i - 1) for i, c in enumerate(coef) if i) * dvdu
            k1 = E * (p * (1 + 1 / (2 * z)) + (4 / z ** 2) * dp)
            e1 = max(e1, float(abs(k1 / mp.besselk(1, z) - 1)))
    return e0, e1


def check_piece32(coef, nu, lo, hi):
    """max rel. error of a fine-piece fit evaluated in float32 over its v range"""
    vs = np.linspace(-1.0, 1.0, 301)
    cc = np.array([float(c) for c in coef], dtype=np.float32)
    p = np.zeros_like(vs, dtype=np.float32)
    for a in cc[::-1]:
        p = (p * vs.astype(np.float32) + a).astype(np.float32)
    worst = 0.0
    for v, pv in zip(vs, p):
        u = (mp.mpf(v) * (mp.mpf(hi) - lo) + lo + hi) / 2
        if u <= -1:
            u = mp.mpf(-1) + mp.mpf("1e-6")
        worst = max(worst, abs(float(pv) / float(large_fn(nu)(u)) - 1))
    return worst


def fmt(name, vals, ctype="double"):
    suffix = "" if ctype == "double" else "f"
    body = ",\n    ".join(f"{mp.nstr(v, 20, min_fixed=-1, max_fixed=-1)}{suffix}" if ctype == "double" else
                         f"{float(v):.9e}f" for v in vals)
    return f"static constexpr {ctype} {name}[{len(vals)}] = {{\n    {body}}};\n"


def main():
    out = ["/* Generated by gen_constants.py -- do not edit. */", "#pragma once", ""]
    # Gauss-Legendre rules
    for n in (16, 32):
        t, w = np.polynomial.legendre.leggauss(n)
        out.append(f"/* {n}-point Gauss-Legendre nodes (ascending) and weights on [-1, 1] */")
        out.append(fmt(f"GL{n}_T", [mp.mpf(float(x)) for x in t]))
        out.append(fmt(f"GL{n}_W", [mp.mpf(float(x)) for x in w]))
    # barycentric weights of the 16 nodes and the 32x16 upsampling matrix
    t16, _ = np.polynomial.legendre.leggauss(16)
    t32, _ = np.polynomial.legendre.leggauss(32)
    bw = []
    for j in range(16):
        p = mp.mpf(1)
        for k in range(16):
            if k != j:
                p *= (mp.mpf(float(t16[j])) - mp.mpf(float(t16[k])))
        bw.append(1 / p)
    bmax = max(abs(b) for b in bw)
    out.append("/* barycentric weights of the 16 Gauss-Legendre nodes (normalised to max 1) */")
    out.append(fmt("BARY16", [b / bmax for b in bw]))
    up = []
    for k in range(32):
        tk = mp.mpf(float(t32[k]))
        row = []
        for j in range(16):
            v = mp.mpf(1)
            for m in range(16):
                if m != j:
                    v *= (tk - mp.mpf(float(t16[m]))) / (mp.mpf(float(t16[j])) - mp.mpf(float(t16[m])))
            row.append(v)
        up.extend(row)
    out.append("/* UP32[k*16+j] = l_j(t32_k): Lagrange basis of the 16 nodes at the 32 nodes */")
    out.append(fmt("UP32", up))
    # Legendre coefficients of the degree-15 interpolant from nodal values:
    # a_m = (2m+1)/2 sum_j lambda_j P_m(t_j) f_j  (exact for degree <= 15)
    t16m = [mp.mpf(float(x)) for x in t16]
    w16m = [mp.mpf(float(x)) for x in np.polynomial.legendre.leggauss(16)[1]]
    legc = []
    for m in range(16):
        for j in range(16):
            legc.append((2 * m + 1) / mp.mpf(2) * w16m[j] * mp.legendre(m, t16m[j]))
    out.append("/* LEGC[m*16+j]: Legendre coefficient m of the interpolant = sum_j LEGC[m*16+j] f_j */")
    out.append(fmt("LEGC", legc))
    # discrete Legendre transforms: weights w_k = sum_m LEGW[k*n+m] M_m for moments M_m = int P_m(t) K(t) dt
    for n in (16, 32):
        tn, wn = np.polynomial.legendre.leggauss(n)
        tab = []
        for k in range(n):
            tk = mp.mpf(float(tn[k]))
            for m in range(n):
                tab.append(mp.mpf(float(wn[k])) * (2 * m + 1) / mp.mpf(2) * mp.legendre(m, tk))
        out.append(f"/* LEGW{n}[k*{n}+m] = lambda_k (2m+1)/2 P_m(t_k): moments -> node weights, {n}-point rule */")
        out.append(fmt(f"LEGW{n}", tab))

    # Bessel coefficients
    fs = small_fns()
    report = []
    for nm, deg64, deg32 in (("I0", 11, 6), ("I1Z", 11, 6), ("R0", 12, 7), ("R1", 12, 7)):
        c64 = mono_in_q(fs[nm], deg64)
        c32 = mono_in_q(fs[nm], deg32)
        report.append((nm, check_small(c64, fs[nm], np.float64), check_small(c32, fs[nm], np.float32)))
        out.append(f"/* {nm}(q), q = z^2/4 in [0, 1] */")
        out.append(fmt(f"KS_{nm}", c64))
        out.append(fmt(f"KSF_{nm}", c32, "float"))
    for nu in (0, 1):
        c64 = cheb_fit_mono(large_fn(nu), 22, -1, 1)
        c32 = cheb_fit_mono(large_fn(nu), 9, -1, 1)
        report.append((f"KL{nu}", check_large(c64, large_fn(nu), np.float64),
                       check_large(c32, large_fn(nu), np.float32)))
        out.append(f"/* e^z sqrt(z) K{nu}(z) as a polynomial in u = 4/z - 1, z >= 2 */")
        out.append(fmt(f"KL{nu}", c64))
        out.append(fmt(f"KLF{nu}", c32, "float"))
    us = mp.mpf(4) / 6 - 1
    ux = mp.mpf(4) / 20 - 1
    # two pieces split at z = 6 (N: 2 < z <= 6, F: z > 6), and the far piece
    # split again at z = 20 (M: 6 < z <= 20, X: z > 20) for shorter polynomials
    for name, nu, deg, lo, hi, der in (("KP0N", 0, 16, us, 1, True), ("KP0F", 0, 15, -1, us, True),
                                       ("KP1N", 1, 14, us, 1, False), ("KP1F", 1, 13, -1, us, False),
                                       ("KP0M", 0, 11, ux, us, False), ("KP0X", 0, 9, -1, ux, False),
                                       ("KP1M", 1, 10, ux, us, False), ("KP1X", 1, 8, -1, ux, False)):
        c = cheb_fit_mono(large_fn(nu), deg, lo, hi)
        e0, e1 = check_piece(c, nu, lo, hi, der)
        report.append((name, e0, e1))
        out.append(f"/* e^z sqrt(z) K{nu}(z) on u in [{float(lo):.4f}, {float(hi):.4f}] (u = 4/z - 1), as a polynomial"
                   f" in v = (2u - lo - hi)/(hi - lo) */")
        out.append(fmt(name, c))
    # finer pieces for launches that classify whole waves against a panel: eight
    # pieces z in (B_k, B_k+1] (k = 0..7) and seven pieces spanning two of them,
    # z in (B_s, B_s+2] (k = 8 + s), for waves whose pairs straddle one boundary;
    # u in [4/B_hi - 1, 4/B_lo - 1]; K0 (KQ0_k) and K1 (KQ1_k) each fitted on its
    # own, degrees from the 1.2e-16 requirement on the value
    bnd = [mp.mpf(2), mp.mpf(3), mp.mpf("4.5"), mp.mpf(7), mp.mpf(12), mp.mpf(20), mp.mpf(40), mp.mpf(100), mp.inf]
    spans = [(k, k + 1) for k in range(8)] + [(k, k + 2) for k in range(7)]
    d0 = [10, 9, 9, 8, 7, 7, 6, 6, 12, 12, 11, 10, 9, 8, 7]
    d1 = [10, 9, 9, 8, 7, 7, 6, 6, 12, 12, 11, 10, 9, 8, 7]
    ulo_all, uhi_all = [], []
    for k, (a, b) in enumerate(spans):
        hi = 4 / bnd[a] - 1
        lo = 4 / bnd[b] - 1 if bnd[b] != mp.inf else mp.mpf(-1)
        ulo_all.append(lo)
        uhi_all.append(hi)
        for nu, deg, der in ((0, d0[k], False), (1, d1[k], False)):
            name = f"KQ{nu}_{k}"
            c = cheb_fit_mono(large_fn(nu), deg, lo, hi)
            e0, e1 = check_piece(c, nu, lo, hi, der)
            report.append((name, e0, e1))
            out.append(f"/* e^z sqrt(z) K{nu}(z) on u in [{float(lo):.6f}, {float(hi):.6f}] (u = 4/z - 1), piece {k} of the"
                       f" fine set, as a polynomial in v = (2u - lo - hi)/(hi - lo) */")
            out.append(fmt(name, c))
    # FP32 fits of the same pieces for the mixed-precision far field, degrees
    # from about 1e-7 relative error in float32 evaluation (the whole-range
    # FP32 fits reach 8.7e-8 / 6.6e-8 at degree 9), zero padded to 6 coefficients
    d0f = [4, 4, 3, 3, 3, 2, 2, 2, 5, 5, 4, 3, 3, 3, 3]
    d1f = [4, 3, 3, 3, 3, 3, 2, 2, 4, 4, 4, 4, 3, 3, 2]
    for nu, dd in ((0, d0f), (1, d1f)):
        rows = []
        for k, (a, b) in enumerate(spans):
            hi = 4 / bnd[a] - 1
            lo = 4 / bnd[b] - 1 if bnd[b] != mp.inf else mp.mpf(-1)
            c = cheb_fit_mono(large_fn(nu), dd[k], lo, hi)
            report.append((f"KQF{nu}_{k}", check_piece32(c, nu, lo, hi), 0.0))
            rows.append([float(x) for x in c] + [0.0] * (6 - len(c)))
        out.append(f"/* FP32 e^z sqrt(z) K{nu}(z) on the fine pieces (as KQ{nu}_k), degrees "
                   + ", ".join(str(d) for d in dd) + ", zero padded */")
        body = ",\n    ".join("{" + ", ".join(f"{v:.9e}f" for v in r) + "}" for r in rows)
        out.append(f"static constexpr float KQF{nu}[15][6] = {{\n    {body}}};\n")
    out.append("/* fine pieces: the z boundaries, and the u range of each piece (0..7 single, 8..14 double) */")
    out.append(fmt("KQ_B", bnd[:8]))
    out.append(fmt("KQ_ULO", ulo_all))
    out.append(fmt("KQ_UHI", uhi_all))
    for nm, f in stokes_small_fns().items():
        c = mono_in_q(f, 13)
        report.append((nm, check_abs(c, f), 0.0))
        out.append(f"/* {nm}(q), q = z^2/4 in [0, 1]: smooth part of the stresslet function (max-abs fit) */")
        out.append(fmt(nm, c))
    # 2^(-j/64), j = 0..63, correctly rounded: the table of the exponential's
    # reduction by ln2/64 (Tang's table-driven method)
    out.append("/* 2^(-j/64), j = 0..63 (correctly rounded) */")
    out.append(fmt("EXP2_NJ", [mp.mpf(2) ** (-mp.mpf(j) / 64) for j in range(64)]))
    with open(os.path.join(HERE, "constants.h"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    for r in report:
        print("%-4s rel err %.2e   %.2e  (fp64 / fp32, or K / K1 from the derivative)" % r)


if __name__ == "__main__":
    main()

"""Pins of the oracle's target gradients of the layer potentials (the
near-boundary gradient of Sec. 4.4, restated for the scalar Yukawa kernel).

Every expected value comes from outside the oracle's gradient code: circle
closed forms (Graf's addition theorem differentiated in polar coordinates),
the gradient of Green's representation of a Yukawa solution, a brute-force
composite quadrature of one panel with scipy Bessel functions, and a
fourth-order finite difference of the oracle's potentials (pinned on their
own elsewhere).

Near the curve the gradient of a layer potential at distance d is the sum of
contributions of size ~ 1/d that cancel to O(1): its rounding-level error grows
like eps h/d, which the tolerances of the closest targets allow for.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
from paper_1908_07392_amd import workloads as wl


# ---------------------------------------------------------------------------
# Circle: S[cos n.] = A_S f(alpha r) cos(n theta), D[cos n.] = A_D f(alpha r) cos(n theta)
#   inside:  f = I_n, A_S = R K_n(aR), A_D = -aR K_n'(aR)
#   outside: f = K_n, A_S = R I_n(aR), A_D = -aR I_n'(aR)
# grad = (u_r cos - u_t sin, u_r sin + u_t cos), u_r = A a f' cos(n th), u_t = -(n/r) A f sin(n th)
# Products of exponentially scaled functions keep alpha = 500 in range.
# ---------------------------------------------------------------------------
def _circle_grad(alpha, R, n, tx, ty):
    r = np.hypot(tx, ty)
    th = np.arctan2(ty, tx)
    a = alpha
    inside = r < R
    # scaled: I_n(x) = ive e^x, K_n(x) = kve e^-x, derivatives by the recurrences
    ive = lambda m, x: sp.ive(m, x)
    kve = lambda m, x: sp.kve(m, x)
    ivpe = lambda x: 0.5 * (ive(n - 1, x) + ive(n + 1, x))
    kvpe = lambda x: -0.5 * (kve(n - 1, x) + kve(n + 1, x))
    x, y = a * r, a * R
    e_in = np.exp(np.where(inside, x - y, y - x))  # e^{x-y} inside, e^{y-x} outside
    fS = np.where(inside, R * kve(n, y) * ive(n, x), R * ive(n, y) * kve(n, x)) * e_in
    fSp = np.where(inside, R * kve(n, y) * a * ivpe(x), R * ive(n, y) * a * kvpe(x)) * e_in
    fD = np.where(inside, -y * kvpe(y) * ive(n, x), -y * ivpe(y) * kve(n, x)) * e_in
    fDp = np.where(inside, -y * kvpe(y) * a * ivpe(x), -y * ivpe(y) * a * kvpe(x)) * e_in

    def grad(f, fp):
        ur = fp * np.cos(n * th)
        ut = -(n / r) * f * np.sin(n * th)
        return np.array([ur * np.cos(th) - ut * np.sin(th), ur * np.sin(th) + ut * np.cos(th)])

    return grad(fS, fSp), grad(fD, fDp)


def _circle_targets(radii, n_theta=6, seed=1):
    th = np.random.default_rng(seed).uniform(0, 2 * math.pi, n_theta)
    T, RR = np.meshgrid(th, np.asarray(radii))
    return (RR * np.cos(T)).ravel(), (RR * np.sin(T)).ravel(), RR.ravel()


@pytest.mark.parametrize("alpha,panels,n", [(2.0, 32, 0), (10.0, 48, 3), (50.0, 96, 5), (500.0, 256, 2)])
def test_circle_gradient_closed_form(alpha, panels, n):
    R = 1.0
    g = wl.discretize(wl.Curve("circle", R=R), panels)
    dens = np.cos(n * g.theta)
    tx, ty, rr = _circle_targets([0.5, 0.9, 0.99, 0.999, 1.001, 1.01, 1.2])
    gs, gd = oracle.eval_gradients(g.x, g.y, alpha, tx, ty, sigma=dens, mu=dens)
    cs, cd = _circle_grad(alpha, R, n, tx, ty)
    scale_s, scale_d = np.abs(cs).max(), np.abs(cd).max()
    assert np.abs(gs - cs).max() < 1e-11 * scale_s
    assert np.abs(gd - cd).max() < 1e-11 * scale_d
    # the gradient of D jumps across the curve by the tangential derivative of
    # the density; of S by the density itself (normal component): both sides differ
    assert np.abs(cd[:, rr == 0.999] - cd[:, rr == 1.001]).max() > 1e-3 * scale_d or n == 0


def test_circle_gradient_very_near():
    # d = 1e-5 R on both sides: rounding-level error of size eps h/d
    alpha, R, n = 10.0, 1.0, 3
    g = wl.discretize(wl.Curve("circle", R=R), 48)
    dens = np.cos(n * g.theta)
    tx, ty, _ = _circle_targets([1.0 - 1e-5, 1.0 + 1e-5])
    gs, gd = oracle.eval_gradients(g.x, g.y, alpha, tx, ty, sigma=dens, mu=dens)
    cs, cd = _circle_grad(alpha, R, n, tx, ty)
    assert np.abs(gs - cs).max() < 1e-11 * np.abs(cs).max()
    assert np.abs(gd - cd).max() < 1e-9 * np.abs(cd).max()


# ---------------------------------------------------------------------------
# Green's representation u = D[u] - S[du/dn] (inward normal) differentiated:
#   grad u = grad D[u] - grad S[du/dn] inside, 0 outside,
# for u = sum_k c_k K0(alpha |x - x_k|) with the sources x_k outside.
# ---------------------------------------------------------------------------
def _point_sources(alpha, x, y, zs, cs):
    u = np.zeros_like(x)
    gx = np.zeros_like(x)
    gy = np.zeros_like(x)
    for z, c in zip(zs, cs):
        dx, dy = x - z.real, y - z.imag
        rho = np.hypot(dx, dy)
        k1 = sp.k1(alpha * rho)
        u += c * sp.k0(alpha * rho)
        gx -= c * alpha * k1 * dx / rho
        gy -= c * alpha * k1 * dy / rho
    return u, gx, gy


@pytest.mark.parametrize("alpha,panels,tol_near", [(5.0, 96, 2e-9), (50.0, 128, 1e-11)])
def test_green_identity_gradient_starfish(alpha, panels, tol_near):
    curve = wl.starfish_curve()
    g = wl.discretize(curve, panels)
    zs = np.array([2.4 + 0.5j, -0.6 - 2.5j])
    cs = np.array([1.0, -0.7])
    ub, gbx, gby = _point_sources(alpha, g.x, g.y, zs, cs)
    nx, ny = g.normals
    dudn = gbx * nx + gby * ny
    th = np.random.default_rng(3).uniform(0, 2 * math.pi, 8)
    zc, dzc, _ = curve.eval(th)
    nrm = 1j * dzc / np.abs(dzc)
    dists = (1e-1, 1e-2, 1e-3, 1e-4)
    pts = np.concatenate([zc + d * nrm for d in dists] + [np.array([0.2 + 0.1j, -0.4 + 0.3j])])
    gs, gd = oracle.eval_gradients(g.x, g.y, alpha, pts.real, pts.imag, sigma=dudn, mu=ub)
    _, ex, ey = _point_sources(alpha, pts.real, pts.imag, zs, cs)
    err = np.abs(np.array([gd[0] - gs[0] - ex, gd[1] - gs[1] - ey])).max(axis=0)
    scale = np.abs(np.array([gbx, gby])).max()  # scale of the boundary data
    assert err[:16].max() < 1e-11 * scale
    assert err[-2:].max() < 1e-11 * scale
    assert err[16:-2].max() < tol_near * scale
    # exterior targets: the representation and its gradient vanish
    ext = zc - 1e-2 * nrm
    gs, gd = oracle.eval_gradients(g.x, g.y, alpha, ext.real, ext.imag, sigma=dudn, mu=ub)
    assert np.abs(gd - gs).max() < 1e-10 * scale


# ---------------------------------------------------------------------------
# One panel of an ellipse, brute force: composite 20-point GL on a geometric
# mesh towards the closest point, numpy Legendre interpolation, scipy K0/K1.
# ---------------------------------------------------------------------------
def _bruteforce_panel_grad(x, y, tx, ty, alpha):
    leg = np.polynomial.legendre
    t16, _ = leg.leggauss(16)
    Vinv = np.linalg.inv(leg.legvander(t16, 15))
    cx, cy = Vinv @ x, Vinv @ y
    dcx, dcy = leg.legder(cx), leg.legder(cy)
    tt = np.linspace(-1, 1, 20001)
    t0 = tt[np.argmin(np.hypot(leg.legval(tt, cx) - tx, leg.legval(tt, cy) - ty))]
    for _ in range(30):  # Newton on the squared distance for the closest point
        px, py = leg.legval(t0, cx) - tx, leg.legval(t0, cy) - ty
        dx, dy = leg.legval(t0, dcx), leg.legval(t0, dcy)
        ddx, ddy = leg.legval(t0, leg.legder(dcx)), leg.legval(t0, leg.legder(dcy))
        t0 = float(np.clip(t0 - (px * dx + py * dy) / (dx * dx + dy * dy + px * ddx + py * ddy), -1, 1))
    g = np.unique(np.concatenate([t0 + (1 - t0) * 0.5 ** np.arange(0, 50),
                                  t0 - (1 + t0) * 0.5 ** np.arange(0, 50), np.linspace(-1, 1, 9)]))
    g = g[(g >= -1) & (g <= 1)]
    tg, wg = leg.leggauss(20)
    W = np.zeros((4, 16))
    for a, b in zip(g[:-1], g[1:]):
        t = 0.5 * (a + b) + 0.5 * (b - a) * tg
        w = 0.5 * (b - a) * wg
        L = leg.legvander(t, 15) @ Vinv
        px, py = leg.legval(t, cx), leg.legval(t, cy)
        dx, dy = leg.legval(t, dcx), leg.legval(t, dcy)
        # differentiate G(x, y) = K0(alpha |x - y|)/2pi and dG/dn_y in the target x
        ex, ey = tx - px, ty - py
        r = np.hypot(ex, ey)
        speed = np.hypot(dx, dy)
        nx, ny = -dy / speed, dx / speed
        K0, K1, K1p = sp.k0(alpha * r), sp.k1(alpha * r), sp.kvp(1, alpha * r)
        # G_x = -alpha K1 e/r ;  F = alpha K1(alpha r)/r (e.n):  grad F = F'(r) e/r (e.n) + (alpha K1/r) n
        dFdr = alpha * (alpha * K1p * r - K1) / r ** 2
        en = ex * nx + ey * ny
        comps = [-alpha * K1 * ex / r, -alpha * K1 * ey / r,
                 dFdr * ex / r * en + alpha * K1 / r * nx, dFdr * ey / r * en + alpha * K1 / r * ny]
        for k in range(4):
            W[k] += (L * (comps[k] / (2 * np.pi) * speed * w)[:, None]).sum(0)
    return W


@pytest.mark.parametrize("dist,tol", [(0.3, 1e-12), (1e-2, 1e-12), (1e-4, 5e-11)])
def test_panel_gradient_weights_bruteforce(dist, tol):
    # the brute force forms y - x in double: at d = 1e-4 its own rounding, amplified
    # by the 1/r^2 kernel of the double-layer gradient, is ~1e-11 of the weights
    curve = wl.Curve("ellipse", a=1.3, b=0.7)
    g = wl.discretize(curve, 12)
    p = 4
    sl = slice(16 * p, 16 * p + 16)
    th = 0.5 * (g.theta[sl][6] + g.theta[sl][7])
    z, dz, _ = curve.eval(th)
    pt = z + dist * 1j * dz / abs(dz)
    for alpha in (3.0, 40.0):
        W = oracle.panel_grad_weights(g.x, g.y, p, pt.real, pt.imag, alpha, mode=1)
        B = _bruteforce_panel_grad(g.x[sl], g.y[sl], pt.real, pt.imag, alpha)
        for k in range(4):
            assert np.max(np.abs(W[k] - B[k])) < tol * np.max(np.abs(B[k])), (alpha, k)


def test_gradient_matches_finite_differences_of_potentials():
    # fourth-order central differences of the oracle's (separately pinned) potentials
    alpha = 10.0
    g = wl.discretize(wl.starfish_curve(), 48)
    rng = np.random.default_rng(8)
    sigma = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 5))
    mu = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 5))
    pts = np.array([0.1 + 0.2j, -0.5 + 0.1j, 0.3 - 0.6j, 1.1 + 0.05j])
    gs, gd = oracle.eval_gradients(g.x, g.y, alpha, pts.real, pts.imag, sigma=sigma, mu=mu)
    h = 1e-3
    for ax in (0, 1):
        vals = []
        for k in (-2, -1, 1, 2):
            tx = pts.real + (k * h if ax == 0 else 0.0)
            ty = pts.imag + (k * h if ax == 1 else 0.0)
            vals.append(oracle.eval_potentials(g.x, g.y, alpha, tx, ty, sigma=sigma, mu=mu))
        for lay, ref in ((0, gs), (1, gd)):
            f = [v[lay] for v in vals]
            fd = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * h)
            assert np.abs(fd - ref[ax]).max() < 1e-8 * np.abs(ref).max(), (ax, lay)

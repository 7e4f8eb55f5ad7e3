"""Pins of the SISDC oracle (Sec. 3.3) on the periodic box: the quadrature
weights integrate polynomials of degree p exactly; the Taylor-Green vortex (its
advection is a pure gradient, taken by the pressure) decays exactly as
e^{-2t/Re} and the error falls at order K; a genuinely nonlinear flow
self-converges at order K.  A dropped quadrature term, a dropped -L_{m+1} term
or a missing Re in the quadrature term each breaks an order.  The sign of the
advection difference in the corrections changes only the error constant (each
sweep still gains an order), so the orders cannot fix it.  It is pinned by an
exact reduction instead: a plane shear wave carried by a uniform flow,
u = U0 + Re(a e^{ik.x}) e with e perpendicular to k, is a solution of the full
Navier-Stokes equations whose advection (u.grad)u = (U0.grad)u is linear (the
wave's self-advection vanishes identically), so one oracle step must equal the
semi-implicit deferred correction of the scalar equation
a' = lambda_E a + lambda_I a (lambda_E = -i k.U0 explicit, lambda_I = -|k|^2/Re
implicit), written here in the u-form of the paper's correction equation
(explicit Euler on the change of the explicit term, implicit Euler on the
change of the implicit term, plus the spectral integral of the previous sweep)
with its own quadrature weights.  With k.U0 dts = 0.5 a flipped sign moves the
result by ~1e-3 of |a|.
"""
import numpy as np
import pytest

from oracle import sisdc_oracle as S


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_quadrature_weights_are_exact_for_polynomials(p):
    q = S.quadrature_weights(p)
    t = np.arange(p + 1, dtype=float)
    for m in range(p):
        for d in range(p + 1):
            exact = ((m + 1.0) ** (d + 1) - m ** (d + 1.0)) / (d + 1)
            assert abs(q[m] @ t ** d - exact) <= 1e-13 * max(1.0, exact)


def _grid(M, Lb=2 * np.pi):
    g = np.arange(M) * Lb / M
    return np.meshgrid(g, g, indexing="xy")


def _run(u0, g0, L0, Re, T, n, K, Lb):
    u, g, L = u0, g0, L0
    for _ in range(n):
        u, g, L = S.step(u, g, L, Re, T / n, K, Lb)
    return u


@pytest.mark.parametrize("K", [2, 3, 4])
def test_taylor_green_decay_at_order_K(K):
    M, Re, T = 32, 10.0, 0.5
    X, Y = _grid(M)
    u0 = np.stack([np.sin(X) * np.cos(Y), -np.cos(X) * np.sin(Y)])
    g0 = np.stack([np.cos(X) * np.cos(Y), -np.sin(X) * np.sin(Y), np.sin(X) * np.sin(Y), -np.cos(X) * np.cos(Y)])
    L0 = -2.0 * u0
    exact = u0 * np.exp(-2.0 * T / Re)
    errs = [np.abs(_run(u0, g0, L0, Re, T, n, K, 2 * np.pi) - exact).max() for n in (2, 4)]
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - K) < 0.25, (K, errs, rate)


def _random_flow(M, seed, kmax=3):
    rng = np.random.default_rng(seed)
    X, Y = _grid(M)
    u1 = np.zeros_like(X)
    u2 = np.zeros_like(X)
    g = np.zeros((4,) + X.shape)
    lap = np.zeros((2,) + X.shape)
    for _ in range(6):
        m, n = rng.integers(-kmax, kmax + 1, 2)
        if m == 0 and n == 0:
            continue
        c, ph = rng.standard_normal(), rng.uniform(0, 2 * np.pi)
        th = m * X + n * Y + ph
        # psi = c cos th, u = (psi_y, -psi_x)
        u1 += -c * n * np.sin(th)
        u2 += c * m * np.sin(th)
        g[0] += -c * n * m * np.cos(th)
        g[1] += -c * n * n * np.cos(th)
        g[2] += c * m * m * np.cos(th)
        g[3] += c * m * n * np.cos(th)
        lap[0] += c * n * (m * m + n * n) * np.sin(th)
        lap[1] += -c * m * (m * m + n * n) * np.sin(th)
    u = np.stack([u1, u2])
    sc = 1.0 / np.abs(u).max()  # |u| = 1: the advection is resolved by the steps used below
    return sc * u, sc * g, sc * lap


@pytest.mark.parametrize("K", [2, 3])
def test_nonlinear_flow_self_converges_at_order_K(K):
    M, Re, T = 24, 20.0, 0.2
    u0, g0, L0 = _random_flow(M, seed=K)
    ref = _run(u0, g0, L0, Re, T, 64, 4, 2 * np.pi)
    errs = [np.abs(_run(u0, g0, L0, Re, T, n, K, 2 * np.pi) - ref).max() for n in (4, 8)]
    rate = np.log2(errs[0] / errs[1])
    assert abs(rate - K) < 0.35, (K, errs, rate)


def _sdc_scalar(a0, zE, zI, p, K):
    """Semi-implicit deferred correction of a' = (lE + lI) a over one step of p
    equal substeps (zE = dts lE, zI = dts lI), K - 1 correction sweeps, in the
    u-form: new_{m+1} = new_m + zE (new_m - old_m) + zI (new_{m+1} - old_{m+1})
    + sum_j w_mj (zE + zI) old_j, with w_mj = (1/dts) times the integral over
    substep m of the Lagrange basis of node j (Gauss-Legendre, exact)."""
    gt, gw = np.polynomial.legendre.leggauss(8)
    nodes = np.arange(p + 1, dtype=float)
    w = np.zeros((p, p + 1))
    for m in range(p):
        t = m + 0.5 * (gt + 1.0)
        for j in range(p + 1):
            lj = np.prod([(t - nodes[i]) / (nodes[j] - nodes[i]) for i in range(p + 1) if i != j], axis=0)
            w[m, j] = 0.5 * np.sum(gw * lj)
    a = [a0]
    for m in range(p):  # first sweep: IMEX Euler
        a.append(a[m] * (1.0 + zE) / (1.0 - zI))
    for _ in range(K - 1):
        b = [a0]
        for m in range(p):
            rhs = b[m] + zE * (b[m] - a[m]) - zI * a[m + 1] + sum(w[m, j] * (zE + zI) * a[j] for j in range(p + 1))
            b.append(rhs / (1.0 - zI))
        a = b
    return a[p]


@pytest.mark.parametrize("K", [3, 4, 5])
def test_shear_wave_step_equals_scalar_deferred_correction(K):
    M, Re, Lb = 16, 25.0, 2 * np.pi
    X, Y = _grid(M)
    k = np.array([1.0, 2.0])
    e = np.array([2.0, -1.0]) / np.sqrt(5.0)
    U0 = np.array([0.9, 0.55])
    A = 0.3
    p = K - 1
    dts = 0.5 / float(k @ U0)  # k.U0 dts = 0.5
    dt = p * dts
    th = k[0] * X + k[1] * Y
    u0 = np.stack([U0[0] + A * e[0] * np.cos(th), U0[1] + A * e[1] * np.cos(th)])
    g0 = np.stack([-A * e[0] * k[0] * np.sin(th), -A * e[0] * k[1] * np.sin(th),
                   -A * e[1] * k[0] * np.sin(th), -A * e[1] * k[1] * np.sin(th)])
    L0 = np.stack([-(k @ k) * A * e[0] * np.cos(th), -(k @ k) * A * e[1] * np.cos(th)])
    u, _, _ = S.step(u0, g0, L0, Re, dt, K, Lb)
    a = _sdc_scalar(A + 0j, -1j * float(k @ U0) * dts, -(k @ k) / Re * dts, p, K)
    expect = np.stack([U0[0] + e[0] * np.real(a * np.exp(1j * th)), U0[1] + e[1] * np.real(a * np.exp(1j * th))])
    err = np.abs(u - expect).max()
    assert err < 1e-13 * A, (K, err)
    # the step is far from the exact flow: the comparison is with the scheme, not the solution
    exact = np.exp((-1j * float(k @ U0) - (k @ k) / Re) * dt) * A
    assert abs(a - exact) > 1e-4 * A

"""Pins of the SISDC oracle (Sec. 4.3) on the periodic box: the quadrature
weights integrate polynomials of degree p exactly; the Taylor-Green vortex (its
advection is a pure gradient, taken by the pressure) decays exactly as
e^{-2t/Re} and the error falls at order K; a genuinely nonlinear flow
self-converges at order K.  A dropped quadrature term, a dropped -L_{m+1} term
or a missing Re in the quadrature term each breaks an order.  The sign of the
advection difference in the corrections changes only the error constant (each
sweep still gains an order), so no pin here fixes it; it follows the paper's
correction equation, and the GPU step is compared with this oracle.
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

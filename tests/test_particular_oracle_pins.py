"""Pins of the particular-solution oracle (Sec. 2.1 Fourier multiplier, Sec.
3.1.2 grid and type-2 evaluation) against what the PDE fixes on trigonometric
polynomials: a divergence-free field u is recovered from F = (alpha^2 - Delta) u,
a gradient forcing produces no velocity (it is taken by the pressure), a
constant forcing gives F/alpha^2, the computed field solves
(alpha^2 - Delta) u + grad p = F with div u = 0, and its gradient and
off-grid values equal the analytic ones.  A dropped projection, a wrong sign of
k or a missing 1/M^2 each fails one of them.
"""
import numpy as np
import pytest

from oracle import particular_oracle as P

X0, Y0, LB, M = -1.5, -1.2, 3.0, 64


def _grid():
    g = np.arange(M) * LB / M
    X, Y = np.meshgrid(X0 + g, Y0 + g, indexing="xy")
    return X, Y


def _trig_stream(rng, nmodes=6, kmax=7):
    """psi = sum c cos(k.x' + phase) with x' = x - x0; returns psi, grad psi, Hessian and Laplacian makers."""
    modes = [(int(rng.integers(-kmax, kmax + 1)), int(rng.integers(-kmax, kmax + 1))) for _ in range(nmodes)]
    cs = rng.standard_normal(nmodes)
    ph = rng.uniform(0, 2 * np.pi, nmodes)
    w = 2 * np.pi / LB

    def fields(x, y):
        u1 = np.zeros_like(x)
        u2 = np.zeros_like(x)
        d = {k: np.zeros_like(x) for k in ("u1x", "u1y", "u2x", "u2y")}
        lap_fac = []
        for (m, n), c, p in zip(modes, cs, ph):
            th = w * (m * (x - X0) + n * (y - Y0)) + p
            kx, ky = w * m, w * n
            # psi = c cos th; u = (d psi/dy, -d psi/dx)
            s, co = np.sin(th), np.cos(th)
            u1 += -c * ky * s
            u2 += c * kx * s
            d["u1x"] += -c * ky * kx * co
            d["u1y"] += -c * ky * ky * co
            d["u2x"] += c * kx * kx * co
            d["u2y"] += c * kx * ky * co
            lap_fac.append(kx * kx + ky * ky)
        return u1, u2, d

    def forcing(x, y, alpha):
        f1 = np.zeros_like(x)
        f2 = np.zeros_like(x)
        for (m, n), c, p in zip(modes, cs, ph):
            th = w * (m * (x - X0) + n * (y - Y0)) + p
            kx, ky = w * m, w * n
            fac = alpha * alpha + kx * kx + ky * ky
            f1 += -c * ky * np.sin(th) * fac
            f2 += c * kx * np.sin(th) * fac
        return f1, f2

    return fields, forcing


@pytest.mark.parametrize("alpha", [0.7, 5.0, 60.0])
def test_divergence_free_field_recovered_with_gradient_and_point_values(alpha):
    rng = np.random.default_rng(int(alpha * 10))
    fields, forcing = _trig_stream(rng)
    X, Y = _grid()
    F1, F2 = forcing(X, Y, alpha)
    u1h, u2h = P.particular(F1, F2, alpha, LB)
    u1, u2, d = fields(X, Y)
    scale = max(np.abs(u1).max(), np.abs(u2).max())
    assert np.abs(P.grid_values(u1h) - u1).max() <= 1e-13 * scale
    assert np.abs(P.grid_values(u2h) - u2).max() <= 1e-13 * scale
    g1x, g1y = P.grid_gradient(u1h, LB)
    g2x, g2y = P.grid_gradient(u2h, LB)
    gs = max(np.abs(v).max() for v in d.values())
    for got, ref in ((g1x, d["u1x"]), (g1y, d["u1y"]), (g2x, d["u2x"]), (g2y, d["u2y"])):
        assert np.abs(got - ref).max() <= 1e-12 * gs
    px, py = X0 + LB * rng.uniform(0, 1, 40), Y0 + LB * rng.uniform(0, 1, 40)
    r1, r2, _ = fields(px, py)
    assert np.abs(P.point_values(u1h, LB, X0, Y0, px, py) - r1).max() <= 1e-13 * scale
    assert np.abs(P.point_values(u2h, LB, X0, Y0, px, py) - r2).max() <= 1e-13 * scale


def test_gradient_forcing_is_taken_by_the_pressure_and_constants_scale():
    rng = np.random.default_rng(3)
    X, Y = _grid()
    w = 2 * np.pi / LB
    phi_x = np.zeros_like(X)
    phi_y = np.zeros_like(X)
    for _ in range(5):
        m, n = rng.integers(-6, 7, 2)
        c, p = rng.standard_normal(), rng.uniform(0, 2 * np.pi)
        th = w * (m * (X - X0) + n * (Y - Y0)) + p
        phi_x += -c * w * m * np.sin(th)
        phi_y += -c * w * n * np.sin(th)
    u1h, u2h = P.particular(phi_x, phi_y, 3.0, LB)
    assert np.abs(P.grid_values(u1h)).max() <= 1e-14 * np.abs(phi_x).max()
    assert np.abs(P.grid_values(u2h)).max() <= 1e-14 * np.abs(phi_y).max()
    c1, c2 = 0.7, -1.3
    u1h, u2h = P.particular(np.full((M, M), c1), np.full((M, M), c2), 3.0, LB)
    assert np.allclose(P.grid_values(u1h), c1 / 9.0, rtol=0, atol=1e-15)
    assert np.allclose(P.grid_values(u2h), c2 / 9.0, rtol=0, atol=1e-15)


def test_solution_satisfies_the_modified_stokes_system():
    # a generic trigonometric forcing (not divergence-free): the returned u and the
    # pressure p^ = -i k.F^/|k|^2 satisfy (alpha^2 + |k|^2) u^ + i k p^ = F^ and k.u^ = 0
    rng = np.random.default_rng(4)
    X, Y = _grid()
    w = 2 * np.pi / LB
    F1 = np.zeros_like(X)
    F2 = np.zeros_like(X)
    for _ in range(8):
        m, n = rng.integers(-9, 10, 2)
        th = w * (m * (X - X0) + n * (Y - Y0)) + rng.uniform(0, 2 * np.pi)
        F1 += rng.standard_normal() * np.cos(th)
        F2 += rng.standard_normal() * np.sin(th)
    alpha = 2.5
    u1h, u2h = P.particular(F1, F2, alpha, LB)
    K1, K2, nyq = P.wavenumbers(M, LB)
    f1, f2 = P.coefficients(F1), P.coefficients(F2)
    k2 = K1 ** 2 + K2 ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        ph = np.where(k2 > 0, -1j * (K1 * f1 + K2 * f2) / k2, 0.0)
    ok = ~nyq
    r1 = (alpha ** 2 + k2) * u1h + 1j * K1 * ph - f1
    r2 = (alpha ** 2 + k2) * u2h + 1j * K2 * ph - f2
    sc = max(np.abs(f1).max(), np.abs(f2).max())
    assert np.abs(r1[ok]).max() <= 1e-14 * sc and np.abs(r2[ok]).max() <= 1e-14 * sc
    assert np.abs((K1 * u1h + K2 * u2h)[ok]).max() <= 1e-14 * sc

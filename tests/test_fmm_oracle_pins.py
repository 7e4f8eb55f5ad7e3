"""Pins of the FMM oracle (Sec. 3.2.1, scalar Yukawa sums) against what the
mathematics fixes: the closed-form kernel K0 and its dipole alpha K1(alpha r)
(x - y).d/r (scipy), field preservation under each translation, the direct
sum it approximates (within the truncation error, with geometric convergence
in p), exactness when every pair is direct, and the independent C oracle's
volume sum.  A flipped (-1)^l in M2L, R_{n+k} for R_{n-k} in M2M, R_{m-l} for
R_{l-m} in L2L or a swapped conj(d)/d in the dipole expansion each fails one of
the first two tests.
"""
import numpy as np
import pytest
import scipy.special as sp

import oracle
from oracle import fmm_oracle as F


def _closed_form(x, ys, q, d, alpha):
    e = x - ys
    r = np.abs(e)
    return np.sum(q * sp.k0(alpha * r)) + np.sum(alpha * sp.k1(alpha * r) * (e.real * d.real + e.imag * d.imag) / r)


@pytest.mark.parametrize("alpha", [0.3, 4.0, 30.0])
def test_expansions_of_charges_and_dipoles_match_the_kernel(alpha):
    rng = np.random.default_rng(7)
    c = 0.2 - 0.1j
    ys = c + 0.1 * (rng.uniform(-1, 1, 6) + 1j * rng.uniform(-1, 1, 6))
    q = rng.standard_normal(6)
    d = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    xs = c + 0.6 * np.exp(2j * np.pi * rng.uniform(0, 1, 9)) * rng.uniform(1.0, 3.0, 9)
    for qq, dd in ((q, 0 * d), (0 * q, d), (q, d)):
        M = F.form_multipole(c, ys, qq, dd, alpha, 40)
        got = F.eval_multipole(M, c, xs, alpha)
        ref = np.array([_closed_form(x, ys, qq, dd, alpha) for x in xs])
        assert np.abs(got.imag).max() <= 1e-14 * np.abs(ref).max()
        assert np.abs(got.real - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("alpha", [0.3, 4.0, 30.0])
def test_translations_preserve_the_field(alpha):
    rng = np.random.default_rng(8)
    p = 40
    cc, cp = 0.05 + 0.05j, 0.0 + 0.0j  # child and parent centres
    ys = cc + 0.04 * (rng.uniform(-1, 1, 5) + 1j * rng.uniform(-1, 1, 5))
    q = rng.standard_normal(5)
    d = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    Mc = F.form_multipole(cc, ys, q, d, alpha, p)
    xs = 0.9 * np.exp(2j * np.pi * rng.uniform(0, 1, 7))
    ref = np.array([_closed_form(x, ys, q, d, alpha) for x in xs])
    # M2M: the shifted multipole gives the same field outside the parent
    Mp = Mc @ F.m2m_matrix(cc - cp, alpha, p)
    assert np.abs(F.eval_multipole(Mp, cp, xs, alpha).real - ref).max() <= 1e-13 * np.abs(ref).max()
    # M2L: the local expansion about a distant centre reproduces the field near it
    ct = 0.8 + 0.3j
    xt = ct + 0.1 * (rng.uniform(-1, 1, 7) + 1j * rng.uniform(-1, 1, 7))
    reft = np.array([_closed_form(x, ys, q, d, alpha) for x in xt])
    Lt = Mp @ F.m2l_matrix(ct - cp, alpha, p)
    assert np.abs(F.eval_local(Lt, ct, xt, alpha).real - reft).max() <= 1e-13 * np.abs(reft).max()
    # L2L: the shifted local expansion gives the same field near the child centre
    cl = ct + 0.05 - 0.05j
    xl = cl + 0.04 * (rng.uniform(-1, 1, 7) + 1j * rng.uniform(-1, 1, 7))
    refl = np.array([_closed_form(x, ys, q, d, alpha) for x in xl])
    Ll = Lt @ F.l2l_matrix(cl - ct, alpha, p)
    assert np.abs(F.eval_local(Ll, cl, xl, alpha).real - refl).max() <= 1e-13 * np.abs(refl).max()


@pytest.mark.parametrize("alpha", [0.5, 5.0, 40.0])
def test_fmm_matches_the_direct_sum_and_converges_geometrically(alpha):
    rng = np.random.default_rng(9)
    n = 500
    # a uniform cloud plus a tight cluster (boxes of very different occupancy)
    sx = np.concatenate([rng.uniform(-1, 1, n - 100), 0.3 + 0.02 * rng.standard_normal(100)])
    sy = np.concatenate([rng.uniform(-1, 1, n - 100), -0.4 + 0.02 * rng.standard_normal(100)])
    tx, ty = rng.uniform(-1.1, 1.1, 200), rng.uniform(-1.1, 1.1, 200)
    q = rng.standard_normal(n)
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ref = F.direct(sx, sy, tx, ty, alpha, q=q, d=d)
    scale = np.abs(ref).max()
    errs = [np.abs(F.fmm(sx, sy, tx, ty, alpha, p, 4, q=q, d=d) - ref).max() / scale for p in (10, 20, 30, 40)]
    assert errs[-1] < 1e-14
    for a, b in zip(errs[:-1], errs[1:]):
        assert b < 1e-2 * a or b < 1e-14  # at least two digits per ten orders


def test_all_direct_levels_are_the_direct_sum():
    rng = np.random.default_rng(10)
    sx, sy = rng.uniform(-1, 1, 300), rng.uniform(-1, 1, 300)
    q = rng.standard_normal(300)
    d = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    ref = F.direct(sx, sy, sx, sy, 3.0, q=q, d=d)  # targets = sources, self skipped
    for level in (0, 1):
        got = F.fmm(sx, sy, sx, sy, 3.0, 5, level, q=q, d=d)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_exclusion_rule_in_the_direct_part():
    # 20 compact "panels" of 16 sources (segments of length 0.05); each target
    # lies within 0.02 of one panel and skips it, so every skipped source is in
    # the target's 3x3 leaf neighbourhood (leaf side 0.25), as near panels are
    rng = np.random.default_rng(11)
    c = rng.uniform(-0.9, 0.9, 20) + 1j * rng.uniform(-0.9, 0.9, 20)
    t = np.exp(2j * np.pi * rng.uniform(0, 1, 20))
    s16 = np.linspace(-0.025, 0.025, 16)
    ys = (c[:, None] + t[:, None] * s16[None, :]).ravel()
    sx, sy = ys.real, ys.imag
    panel = np.arange(320) // 16
    own = rng.integers(0, 20, 50)
    xt = c[own] + 0.02 * np.exp(2j * np.pi * rng.uniform(0, 1, 50))
    tx, ty = xt.real, xt.imag
    q = rng.standard_normal(320)

    def excl(i, js):
        return panel[js] == own[i]
    got = F.fmm(sx, sy, tx, ty, 8.0, 40, 3, q=q, exclude=excl)
    ref = F.direct(sx, sy, tx, ty, 8.0, q=q, exclude=excl)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_volume_sum_against_the_c_oracle():
    # a 40 x 40 trapezoid grid on [-1.5, 1.5]^2 with a Gaussian density, alpha 20:
    # (1/2pi) FMM sum over j != i plus the self-cell term equals the C oracle's volume sum
    n1 = 40
    g = np.linspace(-1.5, 1.5, n1)
    h = g[1] - g[0]
    X, Y = np.meshgrid(g, g, indexing="xy")
    x, y = X.ravel(), Y.ravel()
    w1 = np.full(n1, h)
    w1[[0, -1]] *= 0.5
    w = np.outer(w1, w1).ravel()
    f = np.exp(-((x - 0.3) ** 2 + (y + 0.2) ** 2) / 0.2)
    alpha = 20.0
    idx = np.arange(0, x.size, 7)
    ref = oracle.volume_eval(x, y, w, f, alpha, h, idx)
    phi = F.fmm(x, y, x[idx], y[idx], alpha, 40, 3, q=w * f)
    got = phi / (2 * np.pi) + oracle.self_cell(alpha, h) * w[idx] / h ** 2 * f[idx]
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()

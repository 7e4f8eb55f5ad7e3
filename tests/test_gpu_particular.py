"""GPU parity of the particular solution on a periodic box (Sec. 2.1 multiplier,
Sec. 3.1.2 grid FFTs, Fourier gradient, type-2 sums at points) against the FP64
oracle, and one full implicit modified-Stokes step (particular solution +
boundary values at the nodes + second-kind BIE + GMRES + double layer at the
interior grid points) against a manufactured solution.

Bars: grid values, gradient and point values 1e-12 relative to the largest
oracle value (the non-uniform FFT's point values are ~1e-14 of sum |u^| from
the exact sums, well inside it); the implicit step 1e-9 relative to the solution's size (GMRES to
1e-12, the boundary discretisation resolved to ~1e-11).
"""
import numpy as np
import pytest
import scipy.special as sp
import torch

from oracle import particular_oracle as PO
from paper_1908_07392_amd import mhlp
from paper_1908_07392_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _forcing(x0, y0, Lb, M, seed, nb=5, width=(0.08, 0.2)):
    """sum of Gaussian bumps well inside the box (below 1e-17 at its edge): smooth and periodic"""
    rng = np.random.default_rng(seed)
    g = np.arange(M) * Lb / M
    X, Y = np.meshgrid(x0 + g, y0 + g, indexing="xy")
    F = np.zeros((2, M, M))
    for _ in range(nb):
        c = np.array([x0, y0]) + Lb * rng.uniform(0.3, 0.7, 2)
        s = rng.uniform(*width)
        bump = np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * s * s))
        F[0] += rng.standard_normal() * bump
        F[1] += rng.standard_normal() * bump
    return F, X, Y


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("M,alpha", [(64, 3.0), (256, 20.0), (512, 300.0)])
def test_particular_solution_vs_oracle(M, alpha, method):
    # method 0: direct type-2 sums at the points; 1: the non-uniform FFT
    x0, y0, Lb = -1.6, -1.5, 3.1
    F, X, Y = _forcing(x0, y0, Lb, M, seed=M)
    box = mhlp.Box(M, x0, y0, Lb, alpha)
    box.set_point_method(method)
    rng = np.random.default_rng(5)
    px, py = x0 + Lb * rng.uniform(0, 1, 333), y0 + Lb * rng.uniform(0, 1, 333)  # ragged against the blocks
    u, g, up = box.particular(_t(F), want_u=True, want_grad=True, px=_t(px), py=_t(py))
    u1h, u2h = PO.particular(F[0], F[1], alpha, Lb)
    ref_u = np.stack([PO.grid_values(u1h), PO.grid_values(u2h)])
    ref_g = np.stack([*PO.grid_gradient(u1h, Lb), *PO.grid_gradient(u2h, Lb)])
    ref_p = np.stack([PO.point_values(u1h, Lb, x0, y0, px, py), PO.point_values(u2h, Lb, x0, y0, px, py)])
    eu, eg, ep = _rel(u.cpu().numpy(), ref_u), _rel(g.cpu().numpy(), ref_g), _rel(up.cpu().numpy(), ref_p)
    print(f"M={M} alpha={alpha} method={method}: u {eu:.2e} grad {eg:.2e} points {ep:.2e}")
    assert eu < 1e-12 and eg < 1e-12 and ep < 1e-12
    # partial requests: points only, gradient only
    _, _, up2 = box.particular(_t(F), want_u=False, px=_t(px), py=_t(py))
    assert _rel(up2.cpu().numpy(), up.cpu().numpy()) == 0.0
    _, g2, _ = box.particular(_t(F), want_u=False, want_grad=True)
    assert _rel(g2.cpu().numpy(), g.cpu().numpy()) == 0.0


def _stokeslets(alpha, x, y, sources):
    u = np.zeros((2, np.size(x)))
    for x0, Fv in sources:
        rx, ry = x - x0.real, y - x0.imag
        z = alpha * np.hypot(rx, ry)
        K0, K1 = sp.k0(z), sp.k1(z)
        S1 = (z * z * K0 + z * K1 - 1) / (2 * np.pi * z * z)
        S2 = -(z * z * K0 + 2 * z * K1 - 2) / (2 * np.pi * z ** 4)
        rF = rx * Fv[0] + ry * Fv[1]
        u += np.array([S1 * Fv[0] + alpha ** 2 * S2 * rx * rF, S1 * Fv[1] + alpha ** 2 * S2 * ry * rF])
    return u


@pytest.mark.parametrize("alpha", [5.0, 40.0])
def test_full_implicit_step_manufactured(alpha):
    """u = u^P + w in the starfish, w the flow of two exterior modified stokeslets:
    the step takes F (box grid) and g = u on the boundary, and must return u at the
    interior grid points."""
    x0, y0, Lb, M = -1.6, -1.6, 3.2, 256
    curve = wl.starfish_curve()
    geo = wl.discretize(curve, 96)
    F, X, Y = _forcing(x0, y0, Lb, M, seed=int(alpha), width=(0.1, 0.18))
    sources = [(2.2 + 0.4j, (1.0, 0.3)), (-0.5 - 2.1j, (-0.4, 0.8))]
    u1h, u2h = PO.particular(F[0], F[1], alpha, Lb)
    # boundary data from the oracle's particular solution plus the stokeslet flow
    g = np.stack([PO.point_values(u1h, Lb, x0, y0, geo.x, geo.y), PO.point_values(u2h, Lb, x0, y0, geo.x, geo.y)])
    g += _stokeslets(alpha, geo.x, geo.y, sources)
    inside = curve.contains(X.ravel(), Y.ravel()) if hasattr(curve, "contains") else None
    if inside is None:
        r = np.hypot(X.ravel(), Y.ravel())
        th = np.arctan2(Y.ravel(), X.ravel())
        inside = r < (1 + 0.3 * np.cos(5 * th)) * 0.97  # interior points at least ~3% of r inside
    ix = np.flatnonzero(inside)
    tx, ty = X.ravel()[ix], Y.ravel()[ix]
    # --- the step on the GPU ---
    box = mhlp.Box(M, x0, y0, Lb, alpha)
    G = mhlp.Geometry(_t(geo.node_soa()))
    on = mhlp.Plan(G, alpha, stokes=True)
    off = mhlp.Plan(G, alpha, _t(tx), _t(ty), stokes=True)
    u, _, ub = box.particular(_t(F), px=_t(geo.x), py=_t(geo.y))
    mu, info = mhlp.stokes_gmres_solve(on, _t(g) - ub, tol=1e-12, restart=100)
    uh = mhlp.stokes_eval(off, mu)
    total = u.reshape(2, -1)[:, ix] + uh
    torch.cuda.synchronize()
    ref = np.stack([PO.grid_values(u1h).ravel()[ix], PO.grid_values(u2h).ravel()[ix]]) + _stokeslets(alpha, tx, ty,
                                                                                                      sources)
    err = _rel(total.cpu().numpy(), ref)
    print(f"alpha={alpha}: GMRES {info['iters']} its, {ix.size} interior grid points, step error {err:.2e}")
    assert info["converged"] and err < 1e-9


def test_box_argument_errors():
    for M in (8, 100, 4096):
        with pytest.raises(mhlp.MhlpError):
            mhlp.Box(M, 0.0, 0.0, 1.0, 1.0)
    with pytest.raises(mhlp.MhlpError):
        mhlp.Box(64, 0.0, 0.0, 0.0, 1.0)
    with pytest.raises(mhlp.MhlpError):
        mhlp.Box(64, 0.0, 0.0, 1.0, -1.0)
    box = mhlp.Box(32, 0.0, 0.0, 1.0, 2.0)
    with pytest.raises(mhlp.MhlpError):
        box.particular(_t(np.zeros((2, 32, 32))), want_u=False)  # nothing requested
    with pytest.raises(mhlp.MhlpError):
        box.particular(_t(np.zeros((2, 16, 16))))  # wrong size
    with pytest.raises(mhlp.MhlpError):
        box.set_point_method(2)
    with pytest.raises(mhlp.MhlpError):
        mhlp.Box(2048, 0.0, 0.0, 1.0, 1.0).set_point_method(1)  # the NUFFT serves M <= 1024
    # a constant forcing gives F/alpha^2 everywhere, also at points
    u, _, up = box.particular(_t(np.ones((2, 32, 32))), px=_t([0.3]), py=_t([0.9]))
    assert np.allclose(u.cpu().numpy(), 0.25, atol=1e-15) and np.allclose(up.cpu().numpy(), 0.25, atol=1e-15)

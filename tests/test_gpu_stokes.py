"""GPU parity of the modified-Stokes double layer (the paper's BIE kernel) and
its on-surface operator 1/2 I + D + W and GMRES, through the C ABI, against
the FP64 oracle.

Tolerance: relative to the largest |oracle value| of the compared set, 1e-11
for potentials and operator; GMRES to a true residual of 1e-10 and within
1e-8 of the oracle's dense LU solve.
"""
import math

import numpy as np
import pytest
import scipy.special as sp
import torch

import oracle
from paper_1908_07392_amd import mhlp
from paper_1908_07392_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def _density(g, seed, nmax=6):
    rng = np.random.default_rng(seed)
    return np.stack([wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, nmax)) for _ in range(2)])


def stokeslet_field(alpha, x, y, sources):
    u = np.zeros((2, np.size(x)))
    for x0, F in sources:
        rx, ry = x - x0.real, y - x0.imag
        z = alpha * np.hypot(rx, ry)
        K0, K1 = sp.k0(z), sp.k1(z)
        S1 = (z * z * K0 + z * K1 - 1) / (2 * np.pi * z * z)
        S2 = -(z * z * K0 + 2 * z * K1 - 2) / (2 * np.pi * z ** 4)
        rF = rx * F[0] + ry * F[1]
        u += np.array([S1 * F[0] + alpha ** 2 * S2 * rx * rF, S1 * F[1] + alpha ** 2 * S2 * ry * rF])
    return u


@pytest.mark.parametrize("alpha", [5.0, 50.0, 500.0])
def test_stokes_near_targets_vs_oracle(alpha):
    curve = wl.starfish_curve()
    g = wl.discretize(curve, 64)
    mu = _density(g, 3)
    rng = np.random.default_rng(int(alpha))
    th = rng.uniform(0, 2 * math.pi, 11)
    z, dz, _ = curve.eval(th)
    nrm = 1j * dz / np.abs(dz)
    pts = np.concatenate([z + d * nrm for d in (3e-2, 1e-3, 1e-6, -1e-3, -3e-2)]
                         + [rng.uniform(-0.5, 0.5, 11) + 1j * rng.uniform(-0.5, 0.5, 11)])  # 66: ragged tiles
    P = mhlp.Plan(mhlp.Geometry(_t(g.node_soa())), alpha, _t(pts.real), _t(pts.imag), stokes=True)
    u = mhlp.stokes_eval(P, _t(mu)).cpu().numpy()
    ref = oracle.stokes_eval(g.x, g.y, alpha, pts.real, pts.imag, mu)
    e = _rel(u, ref)
    print(f"alpha={alpha} pairs={P.n_near_pairs} stokes D err {e:.2e}")
    assert e < 1e-11


@pytest.mark.parametrize("alpha", [5.0, 50.0, 500.0])
@pytest.mark.parametrize("n_panels", [32, 33])
def test_stokes_onsurface_operator_vs_oracle(alpha, n_panels):
    """The on-surface operator (each unordered far pair evaluated once) against
    the oracle's dense matrices; 33 panels leave a ragged last row block."""
    g = wl.discretize(wl.starfish_curve(), n_panels)
    mu = _density(g, 5)
    Dm = oracle.stokes_matrix(g.x, g.y, alpha)
    nx, ny = g.normals
    B = oracle.stokes_bie_matrix(Dm, g.weights, nx, ny)
    P = mhlp.Plan(mhlp.Geometry(_t(g.node_soa())), alpha, stokes=True)
    out = mhlp.stokes_apply_bie(P, _t(mu)).cpu().numpy()
    pv = mhlp.stokes_eval(P, _t(mu)).cpu().numpy()
    e1 = _rel(out.ravel(), B @ mu.ravel())
    e2 = float(np.max(np.abs(pv.ravel() - Dm @ mu.ravel())) / np.max(np.abs(mu)))
    print(f"alpha={alpha} pairs={P.n_near_pairs} bie {e1:.2e} D_pv {e2:.2e}")
    assert e1 < 1e-11 and e2 < 1e-11


@pytest.mark.parametrize("alpha", [3.0, 20.0])
def test_stokes_gmres_reproduces_stokeslet_flow(alpha):
    curve = wl.starfish_curve()
    g = wl.discretize(curve, 64)
    sources = [(2.2 + 0.4j, (1.0, 0.3)), (-0.5 - 2.1j, (-0.4, 0.8))]
    gb = stokeslet_field(alpha, g.x, g.y, sources)
    G = mhlp.Geometry(_t(g.node_soa()))
    P = mhlp.Plan(G, alpha, stokes=True)
    mu, info = mhlp.stokes_gmres_solve(P, _t(gb), tol=1e-10, restart=100)
    print(f"alpha={alpha} stokes GMRES {info}")
    assert info["converged"] and info["rel_residual"] <= 1e-10
    # the true residual through the operator
    r = mhlp.stokes_apply_bie(P, mu).cpu().numpy() - gb
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(gb)
    # against the oracle's dense solve
    nx, ny = g.normals
    B = oracle.stokes_bie_matrix(oracle.stokes_matrix(g.x, g.y, alpha), g.weights, nx, ny)
    ref = np.linalg.solve(B, gb.ravel())
    assert _rel(mu.cpu().numpy().ravel(), ref) < 1e-8
    # the represented flow inside is the stokeslet field
    th = np.array([0.3, 1.7, 4.0])
    z, dz, _ = curve.eval(th)
    nrm = 1j * dz / np.abs(dz)
    pts = np.concatenate([[0.1 + 0.2j, -0.3 + 0.5j], z + 0.1 * nrm, z + 1e-3 * nrm])
    Q = mhlp.Plan(G, alpha, _t(pts.real), _t(pts.imag), stokes=True)
    u = mhlp.stokes_eval(Q, mu).cpu().numpy()
    err = np.abs(u - stokeslet_field(alpha, pts.real, pts.imag, sources)).max() / np.abs(gb).max()
    print(f"  flow error {err:.2e}")
    assert err < 1e-9


def test_stokes_split_shapes_restart_and_autotune():
    g = wl.discretize(wl.starfish_curve(), 64)
    mu = _density(g, 7)
    tx, ty = wl.grid_targets(37, -1.3, 1.3)
    G = mhlp.Geometry(_t(g.node_soa()))
    P = mhlp.Plan(G, 20.0, _t(tx), _t(ty), stokes=True)
    ref = mhlp.stokes_eval(P, _t(mu)).cpu().numpy()
    base = P.nsplit
    for ns in (1, 3, 16):
        P.set_split(ns)
        assert _rel(mhlp.stokes_eval(P, _t(mu)).cpu().numpy(), ref) < 1e-13
    P.set_split(base)
    best, ms, table = P.autotune(layers=6, reps=2)
    assert best in table and P.nsplit == best
    assert _rel(mhlp.stokes_eval(P, _t(mu)).cpu().numpy(), ref) < 1e-13
    # restarts and replayed step graphs on the 2N system
    on = mhlp.Plan(G, 20.0, stokes=True)
    gb = _density(g, 8)
    sols = []
    for restart in (3, 7, 100):
        m, info = mhlp.stokes_gmres_solve(on, _t(gb), tol=1e-10, restart=restart, max_iter=500)
        assert info["converged"] and info["rel_residual"] <= 1e-10, (restart, info)
        sols.append(m.cpu().numpy())
    for s in sols[1:]:
        assert _rel(s, sols[0]) < 1e-8


def test_stokes_plan_kinds_are_not_mixed():
    g = wl.discretize(wl.starfish_curve(), 16)
    G = mhlp.Geometry(_t(g.node_soa()))
    stk = mhlp.Plan(G, 5.0, stokes=True)
    sca = mhlp.Plan(G, 5.0)
    d1 = _t(np.ones(g.n_nodes))
    d2 = _t(np.ones((2, g.n_nodes)))
    with pytest.raises(mhlp.MhlpError):
        mhlp.apply_bie(stk, d1)
    with pytest.raises(mhlp.MhlpError):
        mhlp.gmres_solve(stk, d1)
    with pytest.raises(mhlp.MhlpError):
        mhlp.stokes_apply_bie(sca, d2)
    with pytest.raises(mhlp.MhlpError):
        mhlp.stokes_gmres_solve(sca, d2)
    off = mhlp.Plan(G, 5.0, _t([0.1]), _t([0.2]), stokes=True)
    with pytest.raises(mhlp.MhlpError):
        mhlp.stokes_apply_bie(off, d2)  # the operator needs an on-surface plan
    u = mhlp.stokes_eval(off, d2).cpu().numpy()  # single target
    assert _rel(u, oracle.stokes_eval(g.x, g.y, 5.0, [0.1], [0.2], np.ones((2, g.n_nodes)))) < 1e-8


def test_stokes_config2_full_size_sampled():
    """Full-size workload: starfish 256x16, the 109,314 interior targets of the
    512^2 grid; sampled targets including the 40 closest to the curve."""
    cfg = wl.config2()
    g = cfg["geom"]
    tx, ty = cfg["tx"], cfg["ty"]
    G = mhlp.Geometry(_t(g.node_soa()))
    mu = _density(g, 11, nmax=12)
    rng = np.random.default_rng(14)
    dist = np.min(np.abs((tx + 1j * ty)[:, None] - (g.x + 1j * g.y)[None, ::7]), axis=1)
    idx = np.unique(np.concatenate([rng.choice(tx.size, 100, replace=False), np.argsort(dist)[:40]]))
    for alpha in cfg["alphas"]:
        P = mhlp.Plan(G, alpha, _t(tx), _t(ty), stokes=True)
        u = mhlp.stokes_eval(P, _t(mu)).cpu().numpy()[:, idx]
        ref = oracle.stokes_eval(g.x, g.y, alpha, tx[idx], ty[idx], mu)
        e = _rel(u, ref)
        print(f"config2 stokes alpha={alpha} pairs={P.n_near_pairs} err {e:.2e}")
        assert e < 1e-11


def test_stokes_onsurface_config2_full_size_sampled():
    """The on-surface stresslet operator on the config-2 boundary (N = 4096,
    the size its GMRES runs at): principal-value D mu at sampled nodes (random,
    and the first and last node of panels) against the oracle, and the BIE
    operator with mu/2 and the flux term n(x) (integral of mu.n dS)/|Gamma|."""
    cfg = wl.config2()
    g = cfg["geom"]
    G = mhlp.Geometry(_t(g.node_soa()))
    mu = _density(g, 12, nmax=12)
    rng = np.random.default_rng(15)
    idx = np.unique(np.concatenate([rng.choice(g.n_nodes, 120, replace=False), np.arange(0, g.n_nodes, 16)[::9],
                                    np.arange(15, g.n_nodes, 16)[::9]]))
    nx, ny = g.normals
    flux = np.sum(g.weights * (mu[0] * nx + mu[1] * ny)) / np.sum(g.weights)
    for alpha in cfg["alphas"]:
        P = mhlp.Plan(G, alpha, stokes=True)
        pv = mhlp.stokes_eval(P, _t(mu)).cpu().numpy()[:, idx]
        bie = mhlp.stokes_apply_bie(P, _t(mu)).cpu().numpy().reshape(2, -1)[:, idx]
        ref = oracle.stokes_eval(g.x, g.y, alpha, g.x[idx], g.y[idx], mu, tgt_node=idx)
        refb = ref + 0.5 * mu[:, idx] + flux * np.stack([nx[idx], ny[idx]])
        e1 = float(np.max(np.abs(pv - ref)) / np.max(np.abs(mu)))
        e2 = float(np.max(np.abs(bie - refb)) / np.max(np.abs(mu)))
        print(f"config2 on-surface stokes alpha={alpha} D_pv {e1:.2e} bie {e2:.2e}")
        assert e1 < 1e-11 and e2 < 1e-11

"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (relative to the largest |oracle value| of the compared set):
  * off-surface potentials, FP64: 1e-11 (near-field quadrature error of the
    kernel-split rule is ~1e-13..1e-12; rounding of the direct sums ~1e-14);
  * on-surface operator, FP64: 1e-11 (the on-surface double layer is
    conditioned at ~1e-13 w.r.t. 1-ulp node rounding; see the oracle pins);
  * GMRES: true relative residual <= tol and solution within 1e-9 of the
    oracle's dense solve.
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


def _geom(g):
    return mhlp.Geometry(_t(g.node_soa()))


def _relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


def test_config1_circle_vs_oracle_and_closed_form():
    c = wl.config1()
    g = c["geom"]
    G = _geom(g)
    P = mhlp.Plan(G, c["alpha"], _t(c["tx"]), _t(c["ty"]))
    sig = _t(c["sigma"])
    us, ud = mhlp.eval_layer(P, sigma=sig, mu=sig)
    torch.cuda.synchronize()
    us, ud = us.cpu().numpy(), ud.cpu().numpy()
    os_, od = oracle.eval_potentials(g.x, g.y, c["alpha"], c["tx"], c["ty"], sigma=c["sigma"], mu=c["sigma"])
    print("config1 near pairs", P.n_near_pairs, "slp err", _relerr(us, os_), "dlp err", _relerr(ud, od))
    assert _relerr(us, os_) < 1e-11
    assert _relerr(ud, od) < 1e-11
    # closed form (Graf's addition theorem)
    r = np.hypot(c["tx"], c["ty"])
    th = np.arctan2(c["ty"], c["tx"])
    n = np.arange(len(c["coeffs"]))
    E = np.exp(1j * np.outer(th, n))
    In = sp.iv(n[None, :], c["alpha"] * r[:, None])
    slp = np.real((E * In * sp.kv(n, c["alpha"])) @ c["coeffs"])
    dlp = np.real((E * (-c["alpha"]) * In * sp.kvp(n, c["alpha"])) @ c["coeffs"])
    assert _relerr(us, slp) < 1e-11
    assert _relerr(ud, dlp) < 1e-11


def _near_targets(curve, rng, n_each=12):
    th = rng.uniform(0, 2 * math.pi, n_each)
    z, dz, _ = curve.eval(th)
    nrm = 1j * dz / np.abs(dz)
    pts = []
    for d in (3e-2, 1e-3, 1e-5, 1e-8):
        pts.append(z + d * nrm)
    pts.append(rng.uniform(-0.5, 0.5, n_each) + 1j * rng.uniform(-0.5, 0.5, n_each))
    p = np.concatenate(pts)
    return p.real.copy(), p.imag.copy()


@pytest.mark.parametrize("alpha", [5.0, 50.0, 500.0])
def test_starfish_near_targets_vs_oracle(alpha):
    rng = np.random.default_rng(21)
    curve = wl.starfish_curve()
    g = wl.discretize(curve, 64)
    tx, ty = _near_targets(curve, rng)  # 60 targets: ragged w.r.t. the 256-thread tiles
    sigma = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    mu = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    G = _geom(g)
    P = mhlp.Plan(G, alpha, _t(tx), _t(ty))
    us, ud = mhlp.eval_layer(P, sigma=_t(sigma), mu=_t(mu))
    torch.cuda.synchronize()
    os_, od = oracle.eval_potentials(g.x, g.y, alpha, tx, ty, sigma=sigma, mu=mu)
    es, ed = _relerr(us.cpu().numpy(), os_), _relerr(ud.cpu().numpy(), od)
    print(f"alpha={alpha} pairs={P.n_near_pairs} slp {es:.2e} dlp {ed:.2e}")
    assert es < 1e-11 and ed < 1e-11


@pytest.mark.parametrize("alpha", [5.0, 50.0, 500.0])
def test_onsurface_operator_vs_oracle(alpha):
    rng = np.random.default_rng(5)
    g = wl.discretize(wl.starfish_curve(), 48)
    mu = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 6))
    S, D = oracle.onsurface_matrices(g.x, g.y, alpha, want_slp=True)
    G = _geom(g)
    P = mhlp.Plan(G, alpha)
    out = mhlp.apply_bie(P, _t(mu)).cpu().numpy()
    ref = oracle.apply_bie(D, mu)
    us, ud = mhlp.eval_layer(P, sigma=_t(mu), mu=_t(mu))
    # the principal-value D tends to 0 as alpha grows (eigenvalues of 1/2 I + D tend to 1/2),
    # so its error is measured against the scale of the operator's action, max|mu|
    e1, e2 = _relerr(out, ref), _relerr(us.cpu().numpy(), S @ mu)
    e3 = float(np.max(np.abs(ud.cpu().numpy() - D @ mu)) / np.max(np.abs(mu)))
    print(f"alpha={alpha} pairs={P.n_near_pairs} bie {e1:.2e} slp {e2:.2e} dlp {e3:.2e}")
    assert e1 < 1e-11 and e2 < 1e-11 and e3 < 1e-11


@pytest.mark.parametrize("alpha", [5.0, 50.0, 500.0])
def test_onsurface_ragged_blocks_vs_oracle(alpha):
    """An on-surface plan whose N (33 panels, 528 nodes) is not a multiple of the
    256-row tiles of the symmetric operator: apply_bie, the principal-value D of
    a density alone (eval_dlp: the symmetric tiles without the 1/2 term), S alone
    and the fused SLP + DLP (plain tiles) against the oracle's dense matrices."""
    rng = np.random.default_rng(55)
    g = wl.discretize(wl.starfish_curve(), 33)
    mu = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 6))
    sig = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 6))
    S, D = oracle.onsurface_matrices(g.x, g.y, alpha, want_slp=True)
    P = mhlp.Plan(_geom(g), alpha)
    scale = np.max(np.abs(mu))
    e_bie = _relerr(mhlp.apply_bie(P, _t(mu)).cpu().numpy(), oracle.apply_bie(D, mu))
    e_dlp = float(np.max(np.abs(mhlp.eval_dlp(P, _t(mu)).cpu().numpy() - D @ mu)) / scale)
    e_slp = _relerr(mhlp.eval_slp(P, _t(sig)).cpu().numpy(), S @ sig)
    us, ud = mhlp.eval_layer(P, sigma=_t(sig), mu=_t(mu))
    e_fs = _relerr(us.cpu().numpy(), S @ sig)
    e_fd = float(np.max(np.abs(ud.cpu().numpy() - D @ mu)) / scale)
    print(f"alpha={alpha} N={g.n_nodes} bie {e_bie:.2e} dlp {e_dlp:.2e} slp {e_slp:.2e} fused {e_fs:.2e}/{e_fd:.2e}")
    assert max(e_bie, e_dlp, e_slp, e_fs, e_fd) < 1e-11


def test_gmres_circle_modal():
    R, alpha = 1.0, 10.0
    g = wl.discretize(wl.Curve("circle", R=R), 32)
    x = alpha * R

    def lam(n):
        return x * sp.ive(n, x) * 0.5 * (sp.kve(n - 1, x) + sp.kve(n + 1, x))

    b = np.cos(3 * g.theta) + 0.5 * np.sin(7 * g.theta)
    P = mhlp.Plan(_geom(g), alpha)
    mu, info = mhlp.gmres_solve(P, _t(b), tol=1e-12)
    exact = np.cos(3 * g.theta) / lam(3) + 0.5 * np.sin(7 * g.theta) / lam(7)
    print(info)
    assert info["converged"] and info["rel_residual"] <= 1e-12
    assert np.max(np.abs(mu.cpu().numpy() - exact)) < 1e-10


@pytest.mark.parametrize("alpha", [5.0, 500.0])
def test_gmres_starfish_vs_oracle_solve(alpha):
    g = wl.discretize(wl.starfish_curve(), 40)
    _, D = oracle.onsurface_matrices(g.x, g.y, alpha)
    A = 0.5 * np.eye(g.n_nodes) + D
    zs = np.array([2.0 * np.exp(0.4j), 2.0 * np.exp(2.9j)])
    b, _ = wl.point_source_data(g.x, g.y, alpha, zs, np.array([1.0, -0.7]))
    b = b / np.max(np.abs(b))
    ref = np.linalg.solve(A, b)
    P = mhlp.Plan(_geom(g), alpha)
    mu, info = mhlp.gmres_solve(P, _t(b), tol=1e-10)
    print(info)
    assert info["converged"] and info["rel_residual"] <= 1e-10
    assert _relerr(mu.cpu().numpy(), ref) < 1e-8


def test_config2_full_size_sampled():
    """Full config-2 target set at alpha=50: the launch the benchmark times,
    checked on sampled targets (nearest to the boundary and random)."""
    c = wl.config2(alphas=(50.0,))
    g = c["geom"]
    alpha = 50.0
    rng = np.random.default_rng(2)
    sigma = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    mu = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    G = _geom(g)
    P = mhlp.Plan(G, alpha, _t(c["tx"]), _t(c["ty"]))
    us, ud = mhlp.eval_layer(P, sigma=_t(sigma), mu=_t(mu))
    us, ud = us.cpu().numpy(), ud.cpu().numpy()
    # sample: 64 closest to the boundary + 64 random
    curve = wl.starfish_curve()
    dist = curve.radius_at(np.arctan2(c["ty"], c["tx"])) - np.hypot(c["tx"], c["ty"])
    idx = np.concatenate([np.argsort(dist)[:64], rng.choice(len(dist), 64, replace=False)])
    os_, od = oracle.eval_potentials(g.x, g.y, alpha, c["tx"][idx], c["ty"][idx], sigma=sigma, mu=mu)
    es, ed = _relerr(us[idx], os_), _relerr(ud[idx], od)
    print(f"config2 M={P.n_targets} pairs={P.n_near_pairs} slp {es:.2e} dlp {ed:.2e}")
    assert es < 1e-11 and ed < 1e-11
    assert np.all(np.isfinite(us)) and np.all(np.isfinite(ud))


def test_edge_single_panel_and_single_target():
    g = wl.discretize(wl.Curve("ellipse", a=1.0, b=0.6), 1)
    tx, ty = np.array([0.1]), np.array([0.05])
    P = mhlp.Plan(_geom(g), 3.0, _t(tx), _t(ty))
    sig = np.cos(g.theta)
    us, ud = mhlp.eval_layer(P, sigma=_t(sig), mu=_t(sig))
    os_, od = oracle.eval_potentials(g.x, g.y, 3.0, tx, ty, sigma=sig, mu=sig)
    assert _relerr(us.cpu().numpy(), os_) < 1e-11 and _relerr(ud.cpu().numpy(), od) < 1e-11


def test_invalid_arguments_raise():
    g = wl.discretize(wl.Curve("circle"), 4)
    G = _geom(g)
    with pytest.raises(mhlp.MhlpError):
        mhlp.Plan(G, -1.0)
    P = mhlp.Plan(G, 2.0, _t(np.array([0.0])), _t(np.array([0.0])))
    with pytest.raises(mhlp.MhlpError):
        mhlp.apply_bie(P, _t(np.zeros(g.n_nodes)))


# ---------------------------------------------------------------------------
# Mixed precision: FP32 far field, FP64 near field / identity / Arnoldi.
# Tolerance 1e-6 relative to max|u| for potentials (FP32 kernel values carry
# ~1e-7 relative error); solves are still judged by the FP64 residual at 1e-10.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("alpha", [5.0, 50.0, 500.0])
def test_mixed_precision_potentials(alpha):
    rng = np.random.default_rng(31)
    curve = wl.starfish_curve()
    g = wl.discretize(curve, 64)
    tx, ty = _near_targets(curve, rng)
    tx = np.concatenate([tx, rng.uniform(-0.6, 0.6, 300)])
    ty = np.concatenate([ty, rng.uniform(-0.6, 0.6, 300)])
    sigma = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    G = _geom(g)
    P = mhlp.Plan(G, alpha, _t(tx), _t(ty))
    us, ud = mhlp.eval_layer(P, sigma=_t(sigma), mu=_t(sigma), precision=mhlp.MIXED)
    os_, od = oracle.eval_potentials(g.x, g.y, alpha, tx, ty, sigma=sigma, mu=sigma)
    es, ed = _relerr(us.cpu().numpy(), os_), _relerr(ud.cpu().numpy(), od)
    print(f"mixed alpha={alpha} slp {es:.2e} dlp {ed:.2e}")
    assert es < 1e-6 and ed < 1e-6


@pytest.mark.parametrize("alpha", [5.0, 50.0])
def test_mixed_precision_gmres(alpha):
    g = wl.discretize(wl.starfish_curve(), 64)
    zs = np.array([2.0 * np.exp(0.4j), 2.0 * np.exp(2.9j), 2.0 * np.exp(4.4j)])
    b, _ = wl.point_source_data(g.x, g.y, alpha, zs, np.array([1.0, -0.7, 0.3]))
    b = b / np.max(np.abs(b))
    P = mhlp.Plan(_geom(g), alpha)
    mu64, i64 = mhlp.gmres_solve(P, _t(b), tol=1e-10)
    mu32, i32 = mhlp.gmres_solve(P, _t(b), tol=1e-10, precision=mhlp.MIXED)
    print("fp64", i64, "mixed", i32)
    assert i32["converged"] and i32["rel_residual"] <= 1e-10
    assert _relerr(mu32.cpu().numpy(), mu64.cpu().numpy()) < 1e-8


# ---------------------------------------------------------------------------
# Volume all-pairs sum with self-cell correction (dense stress case)
# ---------------------------------------------------------------------------
def test_volume_small_grid_full():
    n, alpha = 20, 20.0
    gx = np.linspace(-1.5, 1.5, n)
    h = gx[1] - gx[0]
    X, Y = np.meshgrid(gx, gx)
    w1 = np.full(n, h)
    w1[[0, -1]] = h / 2
    W = np.outer(w1, w1).ravel()
    f = (np.cos(2 * X) + Y ** 2).ravel()
    x, y = X.ravel(), Y.ravel()
    u, wc = mhlp.volume_eval(_t(x), _t(y), _t(W), _t(f), alpha, h)
    ref = oracle.volume_eval(x, y, W, f, alpha, h, np.arange(n * n))
    assert abs(wc - oracle.self_cell(alpha, h)) < 1e-14 * abs(wc)
    assert _relerr(u.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-6)])
def test_volume_config3_sampled(precision, tol):
    c = wl.config3()
    u, _ = mhlp.volume_eval(_t(c["x"]), _t(c["y"]), _t(c["w"]), _t(c["f"]), c["alpha"], c["h"], precision=precision)
    idx = c["sample"][:48]
    ref = oracle.volume_eval(c["x"], c["y"], c["w"], c["f"], c["alpha"], c["h"], idx)
    err = _relerr(u.cpu().numpy()[idx], ref)
    print(f"volume precision={precision} sampled rel err {err:.2e}")
    assert err < tol


# ---------------------------------------------------------------------------
# Batched solves: batched == unbatched per system (1e-12), each residual judged
# ---------------------------------------------------------------------------
def _batch_geoms():
    specs = [(wl.Curve("circle", R=0.8), 8, 1.0), (wl.Curve("ellipse", a=1.3, b=0.6), 20, 7.0),
             (wl.Curve("starfish", R=1.0, A=0.2, k=3), 40, 60.0), (wl.Curve("ellipse", a=0.7, b=1.1), 13, 300.0),
             (wl.Curve("starfish", R=1.0, A=0.25, k=7), 33, 1000.0)]
    return [(wl.discretize(c, npan), a) for c, npan, a in specs]


def test_batch_apply_matches_single():
    rng = np.random.default_rng(8)
    geoms = _batch_geoms()
    plans = [mhlp.Plan(_geom(g), a) for g, a in geoms]
    B = mhlp.Batch(plans, 3)
    vecs = []
    for (g, a) in geoms:
        for r in range(3):
            vecs.append(_t(wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 6))))
    out = B.unpack(B.apply(B.pack(vecs)))
    k = 0
    refs = []
    for p in plans:
        for r in range(3):
            ref = mhlp.apply_bie(p, vecs[k])
            refs.append(ref.cpu().numpy())
            assert _relerr(out[k].cpu().numpy(), refs[-1]) < 1e-12
            k += 1
    # every launch shape the autotuner may pick gives the same operator: block
    # targets, 1 or 2 targets per lane, 128 or 256 sources per LDS stage
    for tpl in (1, 2):
        for src in (128, 256):
            for target in (512, 16384):
                B.set_tile(target, tpl, src)
                out2 = B.unpack(B.apply(B.pack(vecs)))
                for k in range(len(vecs)):
                    assert _relerr(out2[k].cpu().numpy(), refs[k]) < 1e-12, (tpl, src, target, k)
    target, ms = B.autotune(reps=2)
    assert target in (512, 1024, 2048, 4096, 8192, 16384) and ms > 0
    tile = B.tile()
    assert len(tile["candidates"]) == 24 and tile["targets_per_lane"] in (1, 2)
    assert tile["sources_per_stage"] in (128, 256) and tile["target"] == target
    out2 = B.unpack(B.apply(B.pack(vecs)))
    for k in range(len(vecs)):
        assert _relerr(out2[k].cpu().numpy(), refs[k]) < 1e-12


def test_batch_gmres_matches_single():
    rng = np.random.default_rng(9)
    geoms = _batch_geoms()
    plans = [mhlp.Plan(_geom(g), a) for g, a in geoms]
    B = mhlp.Batch(plans, 2)
    rhs = []
    for (g, a) in geoms:
        for r in range(2):
            rhs.append(_t(wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))))
    mu, infos = B.gmres(B.pack(rhs), tol=1e-10)
    sols = B.unpack(mu)
    k = 0
    for p in plans:
        for r in range(2):
            assert infos[k]["converged"] and infos[k]["rel_residual"] <= 1e-10, infos[k]
            ref, info = mhlp.gmres_solve(p, rhs[k], tol=1e-10)
            # both solutions have residual <= 1e-10; condition of (1/2 I + D) is O(1)
            assert _relerr(sols[k].cpu().numpy(), ref.cpu().numpy()) < 1e-9
            k += 1


@pytest.mark.parametrize("restart", [2, 5])
def test_batch_gmres_restarts_and_warm_start(restart):
    """Several restart cycles of the lockstep solve, then a warm start in which
    one system's guess is rejected (replaced by zero) and the others are kept."""
    rng = np.random.default_rng(19)
    geoms = _batch_geoms()
    plans = [mhlp.Plan(_geom(g), a) for g, a in geoms]
    B = mhlp.Batch(plans, 2)
    rhs = []
    for (g, a) in geoms:
        for r in range(2):
            rhs.append(_t(wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))))
    gb = B.pack(rhs)
    mu, infos = B.gmres(gb, tol=1e-10, restart=restart, max_iter=400)
    sols = B.unpack(mu)
    refs = []
    k = 0
    for p in plans:
        for r in range(2):
            assert infos[k]["converged"] and infos[k]["rel_residual"] <= 1e-10, infos[k]
            if restart == 2:
                assert infos[k]["restarts"] >= 1
            ref, _ = mhlp.gmres_solve(p, rhs[k], tol=1e-10)
            refs.append(ref)
            assert _relerr(sols[k].cpu().numpy(), ref.cpu().numpy()) < 1e-9
            k += 1
    guesses = [0.999 * x for x in refs]
    guesses[3] = 1e6 * torch.ones_like(refs[3])
    mu2, infos2 = B.gmres(gb, x0=B.pack(guesses), tol=1e-10, restart=restart, max_iter=400)
    sols2 = B.unpack(mu2)
    for k in range(len(rhs)):
        assert infos2[k]["converged"] and infos2[k]["rel_residual"] <= 1e-10
        assert infos2[k]["used_x0"] == (0 if k == 3 else 1)
        assert _relerr(sols2[k].cpu().numpy(), refs[k].cpu().numpy()) < 1e-9
    assert max(i["iters"] for i in infos2) <= max(i["iters"] for i in infos)


def test_zero_rhs_and_exact_initial_guess():
    g = wl.discretize(wl.starfish_curve(), 24)
    P = mhlp.Plan(_geom(g), 12.0)
    z = torch.zeros(g.n_nodes, dtype=torch.float64, device=DEV)
    mu, info = mhlp.gmres_solve(P, z, tol=1e-10)
    assert info["converged"] and info["iters"] == 0 and float(mu.abs().max()) == 0.0
    b = _t(wl.fourier_density(g.theta, wl.random_fourier_coeffs(np.random.default_rng(4), 6)))
    x, info = mhlp.gmres_solve(P, b, tol=1e-12)
    # restarting from the converged solution needs no Arnoldi step
    x2, info2 = mhlp.gmres_solve(P, b, x0=x, tol=1e-10)
    assert info2["converged"] and info2["iters"] == 0 and info2["used_x0"] == 1
    assert torch.equal(x, x2)


@pytest.mark.parametrize("alpha", [0.05, 2000.0])
def test_extreme_alpha_vs_oracle(alpha):
    """alpha -> 0 (every pair in the z <= 2 series branch) and alpha h >> 4.5
    (subdivided near panels, K0 underflow for most far pairs)."""
    rng = np.random.default_rng(31)
    curve = wl.starfish_curve()
    g = wl.discretize(curve, 48)
    tx, ty = _near_targets(curve, rng)
    sigma = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    P = mhlp.Plan(_geom(g), alpha, _t(tx), _t(ty))
    us, ud = mhlp.eval_layer(P, sigma=_t(sigma), mu=_t(sigma))
    os_, od = oracle.eval_potentials(g.x, g.y, alpha, tx, ty, sigma=sigma, mu=sigma)
    assert _relerr(us.cpu().numpy(), os_) < 1e-11 and _relerr(ud.cpu().numpy(), od) < 1e-11


def test_nonfinite_targets_rejected():
    g = wl.discretize(wl.Curve("circle"), 4)
    G = _geom(g)
    with pytest.raises(mhlp.MhlpError):
        mhlp.Plan(G, 3.0, _t([0.1, np.nan]), _t([0.0, 0.2]))
    with pytest.raises(mhlp.MhlpError):
        mhlp.Plan(G, 3.0, _t([0.1, np.inf]), _t([0.0, 0.2]))


def test_zero_rhs_and_loose_tolerance_paths():
    """||g|| stays on the device for FP64 solves from zero: a zero right-hand side
    (scalar and stresslet) ends at the first read of the state with x = 0; a
    tolerance of at least 1 is met by the zero guess before any step; a zero
    right-hand side after a nonzero one reuses the same plan cleanly."""
    g = wl.discretize(wl.starfish_curve(), 24)
    G = _geom(g)
    P = mhlp.Plan(G, 12.0)
    b = _t(wl.fourier_density(g.theta, wl.random_fourier_coeffs(np.random.default_rng(5), 6)))
    x, info = mhlp.gmres_solve(P, b, tol=1e-10)
    assert info["converged"] and info["iters"] > 0
    z = torch.zeros(g.n_nodes, dtype=torch.float64, device=DEV)
    mu, info = mhlp.gmres_solve(P, z, tol=1e-10)
    assert info["converged"] and info["iters"] == 0 and info["restarts"] == 0 and float(mu.abs().max()) == 0.0
    mu, info = mhlp.gmres_solve(P, b, tol=1.5)
    assert info["converged"] and info["iters"] == 0 and float(mu.abs().max()) == 0.0
    x2, info = mhlp.gmres_solve(P, b, tol=1e-10)
    assert torch.equal(x, x2)
    S = mhlp.Plan(G, 12.0, stokes=True)
    z2 = torch.zeros(2 * g.n_nodes, dtype=torch.float64, device=DEV)
    mu, info = mhlp.stokes_gmres_solve(S, z2, tol=1e-10)
    assert info["converged"] and info["iters"] == 0 and float(mu.abs().max()) == 0.0


@pytest.mark.parametrize("n_panels,restart", [(2304, 100), (4160, 100), (4160, 4)])
def test_gmres_long_vectors_circle_modal(n_panels, restart):
    """N = 36,864 nodes: Gram-Schmidt over element slices of 512 (several
    elements per thread, 72 slices) from the first step; N = 66,560: also the
    multi-kernel start of a zero-guess solve (vectors beyond the one-block
    start kernel), unrestarted and restarted every 4 steps (each cycle's end
    on the device, the next cycle from its residual).  A right-hand side with
    sixteen Fourier modes on the circle, whose exact solution divides each mode
    by its eigenvalue of 1/2 I + D."""
    R, alpha = 1.0, 10.0
    g = wl.discretize(wl.Curve("circle", R=R), n_panels)
    x = alpha * R

    def lam(n):
        return x * sp.ive(n, x) * 0.5 * (sp.kve(n - 1, x) + sp.kve(n + 1, x))

    rng = np.random.default_rng(11)
    a, c = rng.standard_normal(16), rng.standard_normal(16)
    b = sum(a[n] * np.cos(n * g.theta) + c[n] * np.sin(n * g.theta) for n in range(16))
    exact = sum((a[n] * np.cos(n * g.theta) + c[n] * np.sin(n * g.theta)) / lam(n) for n in range(16))
    P = mhlp.Plan(_geom(g), alpha)
    mu, info = mhlp.gmres_solve(P, _t(b), tol=1e-12, restart=restart, max_iter=400)
    print(n_panels, restart, info)
    assert g.n_nodes == 16 * n_panels and info["converged"] and info["iters"] >= 5
    assert info["rel_residual"] <= 1e-12
    if restart < info["iters"]:
        assert info["restarts"] >= 2
    assert np.max(np.abs(mu.cpu().numpy() - exact)) < 1e-9 * np.max(np.abs(exact))


def test_gmres_chunk_history_does_not_change_results():
    """A plan sizes the first chunk of a solve from its previous solve (which
    may have needed more or fewer steps) and appends the end of the cycle to
    chunks expected to finish it.  Solving a harder, an easier and the harder
    system again on one plan, restarted and unrestarted, in FP64 and mixed
    precision, gives bit for bit the results and counts of the same solves on
    fresh plans, and the FP64 solutions meet the oracle's dense solve."""
    alpha = 5.0
    g = wl.discretize(wl.starfish_curve(), 40)
    _, D = oracle.onsurface_matrices(g.x, g.y, alpha)
    A = 0.5 * np.eye(g.n_nodes) + D
    zs = np.array([2.0 * np.exp(0.4j), 2.0 * np.exp(2.9j), 1.6 * np.exp(4.4j)])
    hard, _ = wl.point_source_data(g.x, g.y, alpha, zs, np.array([1.0, -0.7, 0.5]))
    hard = hard / np.max(np.abs(hard))
    easy = np.cos(g.theta)
    G = _geom(g)
    for precision in (mhlp.FP64, mhlp.MIXED):
        for restart in (200, 4):
            P = mhlp.Plan(G, alpha)
            counts = []
            for b in (hard, easy, hard, easy):
                mu, info = mhlp.gmres_solve(P, _t(b), tol=1e-10, restart=restart, precision=precision)
                ref, rinfo = mhlp.gmres_solve(mhlp.Plan(G, alpha), _t(b), tol=1e-10, restart=restart,
                                              precision=precision)
                assert info["converged"] and info["rel_residual"] <= 1e-10
                assert (info["iters"], info["restarts"]) == (rinfo["iters"], rinfo["restarts"])
                assert torch.equal(mu, ref)
                if precision == mhlp.FP64:
                    assert _relerr(mu.cpu().numpy(), np.linalg.solve(A, b)) < 1e-8
                counts.append(info["iters"])
            print(precision, restart, counts)
            assert counts[0] > counts[1]  # the history both over- and undershoots

"""Targets next to panel edges (Sec. 4.5.3, the second special case: a target
near the junction of two panels, for which the paper merges the two panels).
This build does not merge panels; each of the two panels is corrected on its
own in the parameter plane.  The test places targets at distances
0.05 h, 5e-3 h, 1e-4, 1e-6, 1e-8 and 1e-9 from eight panel junctions of the
starfish, along the normal and along directions tilted 45 degrees towards
either neighbouring panel, on both sides of the curve (inside and outside the
domain), and compares the single and double layers with the oracle's exact
panel integrals at alpha = 5, 50 and 500.

Bar.  Next to a junction the discretised double layer is ill-conditioned with
respect to the panel geometry: the two panel polynomials meet only up to their
interpolation error (7.6e-16 apart at a 64-panel starfish junction, measured
in 40-digit arithmetic), and a target at distance d from the junction sees an
endpoint shift delta as an angle delta/d, i.e. a change of about
delta |mu| / (2 pi d) in each panel's contribution.  Any FP64 representation of
the panels (rounding of their coefficients and of the target frame, a few ulps
of the panel length h) therefore fixes the result only to ~eps h / d.  The bar
is max(1e-11, 30 eps h / d) of max |u|: 1e-11 down to d ~ 7e-4 h, 9e-7 at
d = 1e-9.  (The oracle integrates in long double; at d = 1e-9 it agrees with a
40-digit quadrature of the same panels to 4e-10.)  Away from junctions the
near-target tests of test_gpu_parity hold 1e-11 down to d = 1e-8."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1908_07392_amd import mhlp
from paper_1908_07392_amd import workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def _edge_targets(curve, g, n_panels, junctions):
    """Targets around the junctions (curve points at the equal-arclength breakpoints)."""
    bps, L = wl._arclength_breakpoints(curve, n_panels)
    h = L / n_panels
    pts, dist = [], []
    for p in junctions:
        z, dz, _ = curve.eval(np.array([bps[p]]))
        z, tau = complex(z[0]), complex(dz[0]) / abs(complex(dz[0]))
        nrm = 1j * tau  # into the domain
        dirs = [nrm * np.exp(1j * a) for a in (0.0, math.pi / 4, -math.pi / 4)]
        dirs += [-d for d in dirs]  # the other side of the curve
        for d in (0.05 * h, 5e-3 * h, 1e-4, 1e-6, 1e-8, 1e-9):
            for v in dirs:
                pts.append(z + d * v)
                dist.append(d)
    p = np.array(pts)
    return p.real.copy(), p.imag.copy(), np.array(dist), h


@pytest.mark.parametrize("alpha", [5.0, 50.0, 500.0])
def test_targets_next_to_panel_edges_vs_oracle(alpha):
    rng = np.random.default_rng(int(alpha) + 40)
    curve = wl.starfish_curve()
    n_panels = 64
    g = wl.discretize(curve, n_panels)
    junctions = sorted(rng.choice(n_panels, 8, replace=False))
    tx, ty, dist, h = _edge_targets(curve, g, n_panels, junctions)
    sigma = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    mu = wl.fourier_density(g.theta, wl.random_fourier_coeffs(rng, 8))
    print(f"edge targets alpha={alpha} M={tx.size} junctions {junctions}", flush=True)
    P = mhlp.Plan(mhlp.Geometry(_t(g.node_soa())), alpha, _t(tx), _t(ty))
    us, ud = mhlp.eval_layer(P, sigma=_t(sigma), mu=_t(mu))
    us, ud = us.cpu().numpy(), ud.cpu().numpy()
    os_, od = oracle.eval_potentials(g.x, g.y, alpha, tx, ty, sigma=sigma, mu=mu)
    es = np.abs(us - os_) / np.max(np.abs(os_))
    ed = np.abs(ud - od) / np.max(np.abs(od))
    bar = np.maximum(1e-11, 30 * np.finfo(float).eps * h / dist)
    for d in np.unique(dist)[::-1]:
        m = dist == d
        print(f"  d = {d:.1e}: slp {es[m].max():.2e} dlp {ed[m].max():.2e} (bar {bar[m][0]:.1e})", flush=True)
    k = int(np.argmax(np.maximum(es, ed) / bar))
    print(f"  near pairs {P.n_near_pairs}; closest to the bar: target {k} at d = {dist[k]:.1e}", flush=True)
    assert np.all(es <= bar) and np.all(ed <= bar)
    assert np.all(es[dist >= 1e-4] < 1e-11) and np.all(ed[dist >= 1e-4] < 1e-11)

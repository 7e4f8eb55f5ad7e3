"""Seeded synthetic workloads for the modified-Helmholtz layer-potential path.

This module generates *inputs only*: closed curves, their composite
16-point Gauss-Legendre panel discretisation with panels of equal arclength
(paper, Sec. 3.2 "Computing the homogeneous correction"), densities, target
point sets and Dirichlet data.  It contains none of the layer-potential,
quadrature-correction or solver arithmetic; both the HIP library and the CPU
oracle consume what it produces.

Geometry conventions
--------------------
* Every curve is oriented with the domain on its left: the outer boundary runs
  counter-clockwise, holes run clockwise.  The unit normal ``n = i tau'/|tau'|``
  then points into the domain (the paper's inward normal).
* A panel is the image of ``t in [-1, 1]`` under a map that is affine in the
  curve parameter ``theta``; breakpoints in ``theta`` are placed so that all
  panels of a curve have equal arclength.
* Node arrays are structure-of-arrays, panel-major, ``t`` ascending inside a
  panel: ``x, y, dx/dt, dy/dt, d2x/dt2, d2y/dt2``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import special as _sp

NODES_PER_PANEL = 16


# --------------------------------------------------------------------------------------
# analytic curves
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class Curve:
    """Closed analytic curve ``z(theta)``, ``theta in [0, 2 pi)``.

    kind: 'circle' (radius R), 'ellipse' (semi-axes a, b) or 'starfish'
    (``r(theta) = R (1 + A cos(k (theta - rot)))``).  ``orient`` = +1 runs
    counter-clockwise, -1 clockwise (holes).
    """

    kind: str
    center: complex = 0j
    R: float = 1.0
    a: float = 1.0
    b: float = 1.0
    A: float = 0.0
    k: int = 5
    rot: float = 0.0
    orient: int = 1

    def _base(self, th):
        th = np.asarray(th, dtype=np.float64)
        e = np.exp(1j * th)
        if self.kind == "circle":
            z = self.R * e
            dz = 1j * self.R * e
            d2z = -self.R * e
        elif self.kind == "ellipse":
            c, s = np.cos(th), np.sin(th)
            z = self.a * c + 1j * self.b * s
            dz = -self.a * s + 1j * self.b * c
            d2z = -self.a * c - 1j * self.b * s
        elif self.kind == "starfish":
            ph = self.k * (th - self.rot)
            r = self.R * (1.0 + self.A * np.cos(ph))
            dr = -self.R * self.A * self.k * np.sin(ph)
            d2r = -self.R * self.A * self.k * self.k * np.cos(ph)
            z = r * e
            dz = (dr + 1j * r) * e
            d2z = (d2r + 2j * dr - r) * e
        else:
            raise ValueError(f"unknown curve kind {self.kind!r}")
        return z, dz, d2z

    def eval(self, th):
        """Return ``z, dz/dtheta, d2z/dtheta2`` (complex) honouring the orientation."""
        th = np.asarray(th, dtype=np.float64)
        if self.orient >= 0:
            z, dz, d2z = self._base(th)
        else:
            z, dz, d2z = self._base(-th)
            dz = -dz
        return z + self.center, dz, d2z

    def radius_at(self, th):
        """Polar radius about the centre (circle/starfish) used for inside tests."""
        th = np.asarray(th, dtype=np.float64)
        if self.kind == "circle":
            return np.full_like(th, self.R)
        if self.kind == "starfish":
            return self.R * (1.0 + self.A * np.cos(self.k * (th - self.rot)))
        raise ValueError("radius_at is defined for star-shaped polar curves only")

    def contains(self, x, y):
        """Analytic inside test (strict) for circle, starfish and ellipse."""
        dx = np.asarray(x) - self.center.real
        dy = np.asarray(y) - self.center.imag
        if self.kind == "ellipse":
            return (dx / self.a) ** 2 + (dy / self.b) ** 2 < 1.0
        th = np.arctan2(dy, dx)
        return np.hypot(dx, dy) < self.radius_at(th)


def _gl(n):
    t, lam = np.polynomial.legendre.leggauss(n)
    return t, lam


def _arclength_breakpoints(curve: Curve, n_panels: int, n_fine: int = 512):
    """Breakpoints ``theta_0=0 < ... < theta_P = 2 pi`` with equal arclength."""
    tg, lg = _gl(24)
    edges = np.linspace(0.0, 2.0 * math.pi, n_fine + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    th = mid[:, None] + half[:, None] * tg[None, :]
    _, dz, _ = curve.eval(th)
    seg = (np.abs(dz) * lg[None, :]).sum(axis=1) * half
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    L = cum[-1]

    def s_from(i0, th1):
        a = edges[i0]
        h = 0.5 * (th1 - a)
        _, d, _ = curve.eval(a + h * (tg + 1.0))
        return cum[i0] + h * float((np.abs(d) * lg).sum())

    bps = np.empty(n_panels + 1)
    bps[0], bps[-1] = 0.0, 2.0 * math.pi
    for p in range(1, n_panels):
        s_t = L * p / n_panels
        i0 = int(np.searchsorted(cum, s_t, side="right") - 1)
        i0 = min(max(i0, 0), n_fine - 1)
        th1 = edges[i0] + (s_t - cum[i0]) / max(seg[i0], 1e-300) * (edges[i0 + 1] - edges[i0])
        for _ in range(50):
            f = s_from(i0, th1) - s_t
            _, d, _ = curve.eval(th1)
            step = f / abs(complex(d))
            th1 -= step
            if abs(step) < 1e-15:
                break
        bps[p] = th1
    return bps, L


@dataclasses.dataclass
class Geometry:
    """Panel discretisation of one or more closed curves (multiply connected allowed)."""

    curves: list
    panels_per_curve: list
    x: np.ndarray
    y: np.ndarray
    dx: np.ndarray
    dy: np.ndarray
    d2x: np.ndarray
    d2y: np.ndarray
    theta: np.ndarray          # curve parameter at each node
    curve_of_node: np.ndarray  # int32 curve index per node
    gl_t: np.ndarray           # 16 Gauss-Legendre nodes on [-1, 1]
    gl_w: np.ndarray           # 16 Gauss-Legendre weights
    lengths: np.ndarray        # arclength of each curve
    theta_w: np.ndarray = None  # quadrature weight in theta (half panel span in theta x GL weight)
    panel_theta: np.ndarray = None  # [Np][2] curve parameter at the panel ends (t = -1, t = 1)

    @property
    def n_nodes(self) -> int:
        return int(self.x.size)

    @property
    def n_panels(self) -> int:
        return self.n_nodes // NODES_PER_PANEL

    @property
    def curve_panel_offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.panels_per_curve)]).astype(np.int32)

    @property
    def curve_node_ptr(self) -> np.ndarray:
        """Node ranges of the curves: curve c owns nodes ptr[c]..ptr[c+1]-1."""
        return (self.curve_panel_offsets * NODES_PER_PANEL).astype(np.int64)

    @property
    def speed(self) -> np.ndarray:
        return np.hypot(self.dx, self.dy)

    @property
    def weights(self) -> np.ndarray:
        """Nystrom weights ``w_m = |y'(t_j)| lambda_j``."""
        return self.speed * np.tile(self.gl_w, self.n_panels)

    @property
    def normals(self):
        """Unit normal ``i tau'/|tau'|`` (into the domain)."""
        s = self.speed
        return -self.dy / s, self.dx / s

    def node_soa(self) -> np.ndarray:
        """``[6][N]`` float64: x, y, dx/dt, dy/dt, d2x/dt2, d2y/dt2."""
        return np.ascontiguousarray(np.stack([self.x, self.y, self.dx, self.dy, self.d2x, self.d2y]))

    def panel_ends(self) -> np.ndarray:
        """``[4][Np]`` float64: xa, ya, xb, yb, the curve points at the panel ends."""
        offs = self.curve_panel_offsets
        out = np.empty((4, self.n_panels))
        for c, curve in enumerate(self.curves):
            sl = slice(offs[c], offs[c + 1])
            za, _, _ = curve.eval(self.panel_theta[sl, 0])
            zb, _, _ = curve.eval(self.panel_theta[sl, 1])
            out[:, sl] = [za.real, za.imag, zb.real, zb.imag]
        return out

    def contains(self, x, y):
        """Inside the domain: inside the outer curve (index 0) and outside every hole."""
        inside = self.curves[0].contains(x, y)
        for c in self.curves[1:]:
            inside &= ~c.contains(x, y)
        return inside


def discretize(curves, panels_per_curve) -> Geometry:
    """Composite 16-point Gauss-Legendre discretisation, equal-arclength panels."""
    if isinstance(curves, Curve):
        curves = [curves]
    if np.isscalar(panels_per_curve):
        panels_per_curve = [int(panels_per_curve)] * len(curves)
    t, lam = _gl(NODES_PER_PANEL)
    xs, ys, dxs, dys, d2xs, d2ys, ths, cid, lens, thw, pth = [], [], [], [], [], [], [], [], [], [], []
    for ci, (c, npan) in enumerate(zip(curves, panels_per_curve)):
        bps, L = _arclength_breakpoints(c, int(npan))
        a, b = bps[:-1], bps[1:]
        half = 0.5 * (b - a)
        th = a[:, None] + half[:, None] * (t[None, :] + 1.0)
        z, dz, d2z = c.eval(th)
        dzt = dz * half[:, None]
        d2zt = d2z * (half[:, None] ** 2)
        xs.append(z.real.ravel()); ys.append(z.imag.ravel())
        dxs.append(dzt.real.ravel()); dys.append(dzt.imag.ravel())
        d2xs.append(d2zt.real.ravel()); d2ys.append(d2zt.imag.ravel())
        ths.append(th.ravel()); cid.append(np.full(th.size, ci, dtype=np.int32))
        thw.append((half[:, None] * lam[None, :]).ravel())
        pth.append(np.stack([a, b], axis=1))
        lens.append(L)
    cat = np.concatenate
    return Geometry(list(curves), [int(p) for p in panels_per_curve], cat(xs), cat(ys), cat(dxs), cat(dys),
                    cat(d2xs), cat(d2ys), cat(ths), cat(cid), t, lam, np.asarray(lens), cat(thw), cat(pth))


# --------------------------------------------------------------------------------------
# densities, targets, data
# --------------------------------------------------------------------------------------
def fourier_density(theta, coeffs):
    """``Re sum_n c_n exp(i n theta)`` for complex coefficients c_0..c_{K-1}."""
    n = np.arange(len(coeffs))
    return np.real(np.exp(1j * np.outer(theta, n)) @ np.asarray(coeffs, dtype=np.complex128))


def random_fourier_coeffs(rng, nmax=8):
    return rng.standard_normal(nmax + 1) + 1j * rng.standard_normal(nmax + 1)


def grid_targets(n, lo, hi):
    g = np.linspace(lo, hi, n)
    X, Y = np.meshgrid(g, g, indexing="xy")
    return X.ravel(), Y.ravel()


def point_source_data(x, y, alpha, zs, cs, shift=None):
    """``sum_k c_k K0(alpha |x - z_k|)`` evaluated as ``exp(-alpha (d - shift))``-scaled
    values so that large alpha does not underflow.  Returns (values, shift)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = np.stack([np.hypot(x - z.real, y - z.imag) for z in zs])
    if shift is None:
        shift = float(d.min())
    v = np.zeros_like(x)
    for k in range(len(zs)):
        v += cs[k] * _sp.kve(0, alpha * d[k]) * np.exp(-alpha * (d[k] - shift))
    return v, shift


# --------------------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------------------
def config1(seed=1001):
    """Circle R=1, 64 panels x 16 nodes, alpha=10, Fourier density n=0..8,
    targets: 64x64 grid on [-1,1]^2 with r < 0.95."""
    rng = np.random.default_rng(seed)
    geom = discretize(Curve("circle", R=1.0), 64)
    c = random_fourier_coeffs(rng, 8)
    sigma = fourier_density(geom.theta, c)
    tx, ty = grid_targets(64, -1.0, 1.0)
    keep = np.hypot(tx, ty) < 0.95
    return dict(name="circle-64x16-alpha10", geom=geom, alpha=10.0, coeffs=c, sigma=sigma,
                tx=tx[keep].copy(), ty=ty[keep].copy())


def starfish_curve():
    return Curve("starfish", R=1.0, A=0.3, k=5)


def config2(seed=1002, alphas=(5.0, 50.0, 500.0), grid=512):
    """Starfish r=1+0.3cos(5 theta), 256 panels x 16 nodes, Dirichlet data from 8 point
    sources on radius 2, interior targets of a grid x grid mesh on [-1.4, 1.4]^2."""
    rng = np.random.default_rng(seed)
    curve = starfish_curve()
    geom = discretize(curve, 256)
    beta = rng.uniform(0.0, 2.0 * math.pi, 8)
    zs = 2.0 * np.exp(1j * beta)
    cs = rng.standard_normal(8)
    tx, ty = grid_targets(grid, -1.4, 1.4)
    keep = curve.contains(tx, ty)
    tx, ty = tx[keep].copy(), ty[keep].copy()
    data = {}
    for a in alphas:
        g, shift = point_source_data(geom.x, geom.y, a, zs, cs)
        scale = float(np.max(np.abs(g)))
        data[a] = dict(g=g / scale, shift=shift, scale=scale)
    return dict(name=f"starfish-256x16-grid{grid}", geom=geom, alphas=tuple(alphas), zs=zs, cs=cs,
                tx=tx, ty=ty, data=data)


def config2_exact(cfg, alpha, x, y):
    """Exact interior solution matching the normalised Dirichlet data of config2."""
    d = cfg["data"][alpha]
    v, _ = point_source_data(x, y, alpha, cfg["zs"], cfg["cs"], shift=d["shift"])
    return v / d["scale"]


def config3(seed=1003, n=256, alpha=20.0):
    """256x256 tensor grid on [-1.5,1.5]^2 with trapezoid weights; forcing is a sum of 16
    Gaussian bumps."""
    rng = np.random.default_rng(seed)
    g = np.linspace(-1.5, 1.5, n)
    h = g[1] - g[0]
    X, Y = np.meshgrid(g, g, indexing="xy")
    w1 = np.full(n, h)
    w1[0] = w1[-1] = 0.5 * h
    W = np.outer(w1, w1)
    cb = rng.uniform(-1.5, 1.5, (16, 2))
    sb = rng.uniform(0.05, 0.3, 16)
    ab = rng.standard_normal(16)
    f = np.zeros_like(X)
    for b in range(16):
        f += ab[b] * np.exp(-((X - cb[b, 0]) ** 2 + (Y - cb[b, 1]) ** 2) / (2 * sb[b] ** 2))
    sub = rng.choice(n * n, 2048, replace=False)
    return dict(name=f"volume-grid{n}-alpha{alpha:g}", x=X.ravel().copy(), y=Y.ravel().copy(),
                w=W.ravel().copy(), f=f.ravel().copy(), h=float(h), alpha=alpha, sample=np.sort(sub))


def config4(seed=1004, n_geom=64, panels_range=(32, 512)):
    """Batch of ellipses (even index) and starfish (odd index) with random panel counts,
    log-uniform alpha in [1, 1000] and four Fourier right-hand sides each."""
    rng = np.random.default_rng(seed)
    out = []
    for gi in range(n_geom):
        if gi % 2 == 0:
            a, b = rng.uniform(0.5, 1.5, 2)
            c = Curve("ellipse", a=float(a), b=float(b))
        else:
            k = int(rng.integers(3, 8))
            A = float(rng.uniform(0.1, 0.3))
            c = Curve("starfish", R=1.0, A=A, k=k)
        npan = int(rng.integers(panels_range[0], panels_range[1] + 1))
        alpha = float(10.0 ** rng.uniform(0.0, 3.0))
        geom = discretize(c, npan)
        rhs = np.stack([fourier_density(geom.theta, random_fourier_coeffs(rng, 8)) for _ in range(4)])
        out.append(dict(curve=c, geom=geom, alpha=alpha, rhs=rhs))
    return out


def config5_geometry(seed=1005):
    """Outer circle R=2 (512 panels, CCW) and three clockwise starfish holes of radius 0.3."""
    rng = np.random.default_rng(seed)
    curves = [Curve("circle", R=2.0)]
    for j in range(3):
        ang = 2.0 * math.pi * j / 3.0
        curves.append(Curve("starfish", center=complex(math.cos(ang), math.sin(ang)), R=0.3, A=0.3, k=5,
                            rot=float(rng.uniform(0.0, 2.0 * math.pi)), orient=-1))
    geom = discretize(curves, [512, 128, 128, 128])
    return geom, rng


def config5(seed=1005, n_steps=200, n_modes=32):
    """Time series of Dirichlet data on the multiply connected config-5 geometry."""
    geom, rng = config5_geometry(seed)
    nc = len(geom.curves)
    a = rng.standard_normal((nc, n_modes))
    phi = rng.uniform(0.0, 2.0 * math.pi, (nc, n_modes))
    om = rng.uniform(-0.1, 0.1, (nc, n_modes))
    n = np.arange(1, n_modes + 1)
    g = np.zeros((n_steps, geom.n_nodes))
    for c in range(nc):
        sel = geom.curve_of_node == c
        t = geom.theta[sel]
        for s in range(n_steps):
            ph = np.outer(t, n) + phi[c][None, :] + om[c][None, :] * s
            g[s, sel] = (np.cos(ph) * (a[c] / n ** 2)[None, :]).sum(axis=1)
    return dict(name="multiply-connected-1280x16-alpha30", geom=geom, alpha=30.0, g=g)

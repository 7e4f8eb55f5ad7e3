"""Plain FP64 CPU fast multipole method for the Yukawa sums of the layer
potentials (Sec. 3.2.1, "Fast summation"), restricted to the scalar kernel.

TEST INFRASTRUCTURE ONLY: imported by the test suite; the HIP library never
imports, links or calls it, and the two share no code.

What it computes.  For charges q_j and dipole vectors d_j at sources y_j,

    phi(x_i) = sum_j [ q_j K0(alpha |x_i - y_j|) + d_j . grad_y K0(alpha |x_i - y_j|) ]

over all pairs the caller does not exclude; (1/2pi) phi is the far field of the
single layer (q = w sigma) and the double layer (d = w mu n).  The exact result
is the direct sum; the FMM approximates it by truncated separation-of-variables
expansions, and this module takes the method's steps in order on a uniform
quadtree (Sec. 3.2.1, "Tree structure" and "Form multipole and form local").

Expansions (the paper's multipole / local expansions restricted to fields of
the modified Helmholtz kernel).  With z = x - c in polar form r e^{i theta}
and every integer n (K_{-n} = K_n, I_{-n} = I_n):
    O_n(z) = K_n(alpha r) e^{i n theta}   (outgoing; the K_n part of the
                                           paper's multipole basis),
    R_n(z) = I_n(alpha r) e^{i n theta}   (regular; I_n = P_n + (alpha r/2)^|n|/|n|!
                                           lies in the span of the local basis).
    multipole about c:  phi(x) = sum_n M_n O_n(x - c)   (|x - c| beyond the sources)
    local about c:      phi(x) = sum_n L_n R_n(x - c)   (|x - c| inside the source-free disc)
Graf's addition theorem gives K0(alpha |x - y|) = sum_n O_n(x - c) R_{-n}(y - c),
and with (d/dx + i d/dy) R_m = alpha R_{m+1}, (d/dx - i d/dy) R_m = alpha R_{m-1},
d . grad = (conj(d) (d/dx + i d/dy) + d (d/dx - i d/dy))/2 (d = d1 + i d2):
    charge  q at y:  M_n += q R_{-n}(y - c)
    dipole  d at y:  M_n += (alpha/2) [conj(d) R_{1-n}(y - c) + d R_{-1-n}(y - c)]
Translations (the same theorem for the outgoing and regular families):
    M2M  (child c' -> parent c):   M_k  = sum_n M'_n R_{n-k}(c' - c)
    M2L  (source c_s -> target c_t): L_l = (-1)^l sum_n M_n O_{n-l}(c_t - c_s)
    L2L  (parent c -> child c'):   L'_m = sum_l L_l R_{l-m}(c' - c)
    L2P: phi(x) = sum_l L_l R_l(x - c)
Truncation keeps |n| <= p on every expansion (p = 40 in the paper).

Tree.  Root square: centre at the midpoint of the bounding box of all sources
and targets, side S = (largest extent) (1 + 2^-20) (S = 1 when all points
coincide); level l has 4^l boxes of side S/2^l; a point's leaf box has
ix = floor((x - (cx - S/2)) / (S/2^L)), clamped to [0, 2^L - 1] (same for y).
Each leaf interacts directly (P2P) with the sources of its 3x3 neighbourhood;
every other source box reaches it through the interaction lists (children of
the parent's neighbours that are not neighbours) at levels 2..L.

Bessel functions are scipy's (a library primitive); expansions are not scaled,
so the parameters must keep I_n and K_n in range (checked: a non-finite
expansion raises).
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp


def root_box(x, y):
    """(cx, cy, S) of the root square of the point set."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xmin, xmax, ymin, ymax = x.min(), x.max(), y.min(), y.max()
    cx, cy = 0.5 * (xmin + xmax), 0.5 * (ymin + ymax)
    ext = max(xmax - xmin, ymax - ymin)
    S = ext * (1.0 + 2.0 ** -20) if ext > 0 else 1.0
    return cx, cy, S


def leaf_index(x, y, box, level):
    """(ix, iy) leaf coordinates of points."""
    cx, cy, S = box
    side = S / 2.0 ** level
    nb = 2 ** level
    ix = np.clip(np.floor((np.asarray(x) - (cx - 0.5 * S)) / side).astype(np.int64), 0, nb - 1)
    iy = np.clip(np.floor((np.asarray(y) - (cy - 0.5 * S)) / side).astype(np.int64), 0, nb - 1)
    return ix, iy


def box_center(box, level, ix, iy):
    cx, cy, S = box
    side = S / 2.0 ** level
    return (cx - 0.5 * S + (ix + 0.5) * side) + 1j * (cy - 0.5 * S + (iy + 0.5) * side)


def R(n, z, alpha):
    """Regular functions R_n(z) = I_n(alpha |z|) e^{i n arg z}; n an int array, z complex (broadcast)."""
    z = np.asarray(z, dtype=np.complex128)
    n = np.asarray(n)
    r = np.abs(z)
    th = np.angle(z)
    return sp.iv(np.abs(n), alpha * r) * np.exp(1j * n * th)


def O(n, z, alpha):
    """Outgoing functions O_n(z) = K_n(alpha |z|) e^{i n arg z}."""
    z = np.asarray(z, dtype=np.complex128)
    n = np.asarray(n)
    r = np.abs(z)
    th = np.angle(z)
    return sp.kv(np.abs(n), alpha * r) * np.exp(1j * n * th)


def _finite(a, what):
    if not np.all(np.isfinite(a)):
        raise FloatingPointError(f"{what}: expansion out of floating-point range for these parameters")
    return a


def form_multipole(c, ys, q, d, alpha, p):
    """Multipole coefficients M_n, n = -p..p, about c of charges q and dipoles d (complex) at ys."""
    n = np.arange(-p, p + 1)
    w = ys[:, None] - c
    M = np.zeros(2 * p + 1, dtype=np.complex128)
    if q is not None:
        M += (q[:, None] * R(-n[None, :], w, alpha)).sum(axis=0)
    if d is not None:
        M += 0.5 * alpha * (np.conj(d)[:, None] * R(1 - n[None, :], w, alpha)
                            + d[:, None] * R(-1 - n[None, :], w, alpha)).sum(axis=0)
    return _finite(M, "P2M")


def eval_multipole(M, c, xs, alpha):
    p = (M.size - 1) // 2
    n = np.arange(-p, p + 1)
    return (M[None, :] * O(n[None, :], xs[:, None] - c, alpha)).sum(axis=1)


def m2m_matrix(a, alpha, p):
    """T[n, k] with M_k = sum_n M'_n T[n, k], shift a = c_child - c_parent."""
    n = np.arange(-p, p + 1)
    return _finite(R(n[:, None] - n[None, :], a, alpha), "M2M")


def m2l_matrix(b, alpha, p):
    """T[n, l] with L_l = sum_n M_n T[n, l], b = c_target - c_source."""
    n = np.arange(-p, p + 1)
    return _finite(((-1.0) ** np.abs(n))[None, :] * O(n[:, None] - n[None, :], b, alpha), "M2L")


def l2l_matrix(a, alpha, p):
    """T[l, m] with L'_m = sum_l L_l T[l, m], shift a = c_child - c_parent."""
    n = np.arange(-p, p + 1)
    return _finite(R(n[:, None] - n[None, :], a, alpha), "L2L")


def eval_local(L, c, xs, alpha):
    p = (L.size - 1) // 2
    n = np.arange(-p, p + 1)
    return (L[None, :] * R(n[None, :], xs[:, None] - c, alpha)).sum(axis=1)


def direct_pairs(x, ys, q, d, alpha):
    """sum over the given sources of q K0 + d . grad_y K0 at target x (complex x, ys; d complex)."""
    e = x - ys
    r = np.abs(e)
    out = 0.0
    if q is not None:
        out = out + np.sum(q * sp.k0(alpha * r))
    if d is not None:
        # d . grad_y K0(alpha |x - y|) = alpha K1(alpha r) (x - y) . d / r
        out = out + np.sum(alpha * sp.k1(alpha * r) * (e.real * d.real + e.imag * d.imag) / r)
    return out


def fmm(sx, sy, tx, ty, alpha, p, level, q=None, d=None, exclude=None):
    """phi at the targets by the FMM on a uniform quadtree with leaves at `level`.

    q: charges [N] or None; d: dipoles [N] complex (d1 + i d2) or None.
    exclude(i, src_index_array) -> boolean mask of sources skipped for target i
    in the direct (P2P) part; None skips coincident points only."""
    sx, sy, tx, ty = (np.asarray(a, dtype=np.float64) for a in (sx, sy, tx, ty))
    ys = sx + 1j * sy
    xs = tx + 1j * ty
    q = None if q is None else np.asarray(q, dtype=np.float64)
    d = None if d is None else np.asarray(d, dtype=np.complex128)
    box = root_box(np.concatenate([sx, tx]), np.concatenate([sy, ty]))
    L = int(level)
    nb = 2 ** L
    six, siy = leaf_index(sx, sy, box, L)
    tix, tiy = leaf_index(tx, ty, box, L)
    src_of = {}
    for j, key in enumerate(zip(six.tolist(), siy.tolist())):
        src_of.setdefault(key, []).append(j)
    src_of = {k: np.array(v) for k, v in src_of.items()}
    K = 2 * p + 1
    # translation matrices depend only on the level and the box offset
    cache = {}

    def shift(kind, lev, a):
        key = (kind, lev, round(a.real / (S / 2.0 ** lev) * 4), round(a.imag / (S / 2.0 ** lev) * 4))
        if key not in cache:
            cache[key] = {"m2m": m2m_matrix, "m2l": m2l_matrix, "l2l": l2l_matrix}[kind](a, alpha, p)
        return cache[key]

    S = box[2]
    # upward pass: multipoles at the leaves, then M2M to level 2
    mp = {L: {}}
    for (ix, iy), js in src_of.items():
        c = box_center(box, L, ix, iy)
        mp[L][(ix, iy)] = form_multipole(c, ys[js], None if q is None else q[js], None if d is None else d[js],
                                         alpha, p)
    for lev in range(L - 1, 1, -1):
        mp[lev] = {}
        for (ix, iy), Mc in mp[lev + 1].items():
            par = (ix // 2, iy // 2)
            a = box_center(box, lev + 1, ix, iy) - box_center(box, lev, *par)
            acc = mp[lev].setdefault(par, np.zeros(K, dtype=np.complex128))
            acc += Mc @ shift("m2m", lev, a)
    # downward pass: M2L over interaction lists, L2L to the children
    loc = {}
    for lev in range(2, L + 1):
        nl = 2 ** lev
        loc[lev] = {}
        for ix in range(nl):
            for iy in range(nl):
                Lc = np.zeros(K, dtype=np.complex128)
                if lev > 2:
                    Lp = loc[lev - 1].get((ix // 2, iy // 2))
                    if Lp is not None:
                        a = box_center(box, lev, ix, iy) - box_center(box, lev - 1, ix // 2, iy // 2)
                        Lc = Lp @ shift("l2l", lev, a)
                px, py = ix // 2, iy // 2
                for jx in range(2 * (px - 1), 2 * (px + 1) + 2):
                    for jy in range(2 * (py - 1), 2 * (py + 1) + 2):
                        if not (0 <= jx < nl and 0 <= jy < nl):
                            continue
                        if max(abs(jx - ix), abs(jy - iy)) < 2:
                            continue
                        Ms = mp.get(lev, {}).get((jx, jy))
                        if Ms is None:
                            continue
                        b = box_center(box, lev, ix, iy) - box_center(box, lev, jx, jy)
                        Lc = Lc + Ms @ shift("m2l", lev, b)
                loc[lev][(ix, iy)] = _finite(Lc, "M2L")
    # leaves: local expansion plus direct sums over the 3x3 neighbourhood
    phi = np.zeros(xs.size)
    for i in range(xs.size):
        ix, iy = int(tix[i]), int(tiy[i])
        val = 0.0 + 0.0j
        if L >= 2:
            val += eval_local(loc[L][(ix, iy)], box_center(box, L, ix, iy), xs[i:i + 1], alpha)[0]
        js = [src_of[(jx, jy)] for jx in range(ix - 1, ix + 2) for jy in range(iy - 1, iy + 2)
              if (jx, jy) in src_of]
        if js:
            js = np.concatenate(js)
            skip = (np.abs(xs[i] - ys[js]) == 0) if exclude is None else exclude(i, js)
            js = js[~skip]
            val += direct_pairs(xs[i], ys[js], None if q is None else q[js], None if d is None else d[js], alpha)
        phi[i] = val.real
    return phi


def direct(sx, sy, tx, ty, alpha, q=None, d=None, exclude=None):
    """The exact sum the FMM approximates (same exclusion rule)."""
    ys = np.asarray(sx) + 1j * np.asarray(sy)
    xs = np.asarray(tx) + 1j * np.asarray(ty)
    q = None if q is None else np.asarray(q, dtype=np.float64)
    d = None if d is None else np.asarray(d, dtype=np.complex128)
    out = np.zeros(xs.size)
    allj = np.arange(ys.size)
    for i in range(xs.size):
        skip = (np.abs(xs[i] - ys) == 0) if exclude is None else exclude(i, allj)
        js = allj[~skip]
        out[i] = direct_pairs(xs[i], ys[js], None if q is None else q[js], None if d is None else d[js], alpha).real
    return out

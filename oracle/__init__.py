"""Plain FP64 CPU oracle for the modified-Helmholtz layer-potential path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
CPU-baseline leg of the benchmark may import this package.  The HIP library
never imports, links or calls it, and the two share no code.

The arithmetic lives in ``mhlp_oracle.c`` (header comment there gives the
definitions and the paper passages they follow); this module is the ctypes
marshalling around it plus a small numpy MLP reference.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhlp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-D_GNU_SOURCE",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_bessel_k01.argtypes = [ctypes.c_double, _D, _D]
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, _D, _D]
        L.orc_panel_weights.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int, _D]
        L.orc_eval.argtypes = [_D, _D, ctypes.c_int64, _D, _D, ctypes.c_double, _D, _D, ctypes.c_int64, _I64,
                               _D, _D, ctypes.c_int]
        L.orc_panel_grad_weights.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int, _D]
        L.orc_eval_grad.argtypes = [_D, _D, ctypes.c_int64, _D, _D, ctypes.c_double, _D, _D, ctypes.c_int64,
                                    _D, _D, _D, _D, ctypes.c_int]
        L.orc_stresslet_T.argtypes = [ctypes.c_double, _D]
        L.orc_stokes_panel_weights.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_int, _D]
        L.orc_stokes_eval.argtypes = [_D, _D, ctypes.c_int64, _D, _D, ctypes.c_double, _D, _D, ctypes.c_int64,
                                      _I64, _D, _D, ctypes.c_int]
        L.orc_stresslet_dT.argtypes = [ctypes.c_double, _D]
        L.orc_stokes_grad_panel_weights.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, ctypes.c_int, _D]
        L.orc_stokes_grad_eval.argtypes = [_D, _D, ctypes.c_int64, _D, _D, ctypes.c_double, _D, _D, ctypes.c_int64,
                                           _D, ctypes.c_int]
        L.orc_stokes_matrix.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_double, _D, ctypes.c_int]
        L.orc_assemble_onsurface.argtypes = [_D, _D, ctypes.c_int64, ctypes.c_double, _D, _D, ctypes.c_int]
        L.orc_gmres.argtypes = [_D, ctypes.c_int64, _D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int), _D, ctypes.c_int]
        L.orc_self_cell.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_self_cell.restype = ctypes.c_double
        L.orc_volume_eval.argtypes = [_D, _D, _D, _D, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _I64,
                                      ctypes.c_int64, _D, ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(_D)


def _c(a, dt=np.float64):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def _ok(rc, what):
    """Raise on a failed oracle call (-3: the adaptive quadrature stopped on a
    piece that had not converged)."""
    if rc != 0:
        raise RuntimeError(f"{what} failed: {rc}")


def max_threads() -> int:
    return int(lib().orc_max_threads())


def bessel_k01(z):
    """K0(z), K1(z) for z > 0 (scalar or array)."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    k0 = np.empty_like(z)
    k1 = np.empty_like(z)
    a, b = ctypes.c_double(), ctypes.c_double()
    for i, v in enumerate(z.ravel()):
        lib().orc_bessel_k01(float(v), ctypes.byref(a), ctypes.byref(b))
        k0.flat[i] = a.value
        k1.flat[i] = b.value
    return k0, k1


def gauss_legendre(n):
    t = np.empty(n)
    w = np.empty(n)
    lib().orc_gauss_legendre(n, _p(t), _p(w))
    return t, w


def panel_weights(x, y, panel, tx, ty, alpha, self_node=-1, mode=0):
    """Exact (mode 1), direct (mode 2) or automatic (0) SLP/DLP weights of one
    target against one panel: returns (W_slp[16], W_dlp[16])."""
    x, y = _c(x), _c(y)
    W = np.empty(32)
    _ok(lib().orc_panel_weights(_p(x), _p(y), int(panel), float(tx), float(ty), float(alpha), int(self_node),
                                int(mode), _p(W)), "orc_panel_weights")
    return W[:16].copy(), W[16:].copy()


def eval_potentials(x, y, alpha, tx, ty, sigma=None, mu=None, tgt_node=None, nthreads=0):
    """SLP of sigma and DLP of mu at the targets (exact near-panel integrals)."""
    x, y, tx, ty = _c(x), _c(y), _c(tx), _c(ty)
    sigma, mu = _c(sigma), _c(mu)
    m = tx.size
    us = np.zeros(m) if sigma is not None else None
    ud = np.zeros(m) if mu is not None else None
    tn = None if tgt_node is None else _c(tgt_node, np.int64)
    rc = lib().orc_eval(_p(x), _p(y), x.size // 16, _p(sigma), _p(mu), float(alpha), _p(tx), _p(ty), m,
                        None if tn is None else tn.ctypes.data_as(_I64), _p(us), _p(ud), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_eval failed: {rc}")
    return us, ud


def eval_gradients(x, y, alpha, tx, ty, sigma=None, mu=None, nthreads=0):
    """Gradients of the SLP of sigma and the DLP of mu at off-surface targets
    (exact near-panel integrals).  Returns (grad S as [2][m] or None, grad D as
    [2][m] or None)."""
    x, y, tx, ty = _c(x), _c(y), _c(tx), _c(ty)
    sigma, mu = _c(sigma), _c(mu)
    m = tx.size
    gs = np.zeros((2, m)) if sigma is not None else None
    gd = np.zeros((2, m)) if mu is not None else None
    rc = lib().orc_eval_grad(_p(x), _p(y), x.size // 16, _p(sigma), _p(mu), float(alpha), _p(tx), _p(ty), m,
                             None if gs is None else _p(gs[0]), None if gs is None else _p(gs[1]),
                             None if gd is None else _p(gd[0]), None if gd is None else _p(gd[1]),
                             int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_eval_grad failed: {rc}")
    return gs, gd


def panel_grad_weights(x, y, panel, tx, ty, alpha, mode=0):
    """64 gradient weights of one target against one panel (blocks d/dx1 SLP,
    d/dx2 SLP, d/dx1 DLP, d/dx2 DLP)."""
    x, y = _c(x), _c(y)
    W = np.zeros(64)
    _ok(lib().orc_panel_grad_weights(_p(x), _p(y), int(panel), float(tx), float(ty), float(alpha), int(mode), _p(W)),
        "orc_panel_grad_weights")
    return W.reshape(4, 16)


# --------------------------------------------------------------------------------------
# modified-Stokes double layer (stresslet)
# --------------------------------------------------------------------------------------
def stresslet_T(z):
    """(T1, T2, T3) of the stresslet at z > 0."""
    out = np.zeros(3)
    lib().orc_stresslet_T(float(z), _p(out))
    return tuple(out)


def stokes_panel_weights(x, y, panel, tx, ty, alpha, self_node=-1, mode=0):
    """[2][2][16] weights: u_i += sum_j,l W[i][j][l] mu_j(node l of the panel)."""
    x, y = _c(x), _c(y)
    W = np.zeros(64)
    _ok(lib().orc_stokes_panel_weights(_p(x), _p(y), int(panel), float(tx), float(ty), float(alpha), int(self_node),
                                       int(mode), _p(W)), "orc_stokes_panel_weights")
    return W.reshape(2, 2, 16)


def stokes_eval(x, y, alpha, tx, ty, mu, tgt_node=None, nthreads=0):
    """Modified-Stokes double layer of mu ([2][N]) at the targets; returns [2][m]
    (on-surface targets marked by tgt_node: principal value, no 1/2 mu)."""
    x, y, tx, ty = _c(x), _c(y), _c(tx), _c(ty)
    mu = _c(mu).reshape(2, -1)
    m = tx.size
    u = np.zeros((2, m))
    tn = None if tgt_node is None else _c(tgt_node, np.int64)
    m1, m2 = np.ascontiguousarray(mu[0]), np.ascontiguousarray(mu[1])
    rc = lib().orc_stokes_eval(_p(x), _p(y), x.size // 16, _p(m1), _p(m2), float(alpha), _p(tx), _p(ty), m,
                               None if tn is None else tn.ctypes.data_as(_I64), _p(u[0]), _p(u[1]), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_stokes_eval failed: {rc}")
    return u


def stresslet_dT(z):
    """(T1', T2', T3') at z > 0."""
    out = np.zeros(3)
    lib().orc_stresslet_dT(float(z), _p(out))
    return tuple(out)


def stokes_grad_panel_weights(x, y, panel, tx, ty, alpha, mode=0):
    """[2][2][2][16] weights W[a][l][j]: d u_a/d x_l += sum_k W[a][l][j][k] mu_j(node k)."""
    x, y = _c(x), _c(y)
    W = np.zeros(128)
    _ok(lib().orc_stokes_grad_panel_weights(_p(x), _p(y), int(panel), float(tx), float(ty), float(alpha), int(mode),
                                            _p(W)), "orc_stokes_grad_panel_weights")
    return W.reshape(2, 2, 2, 16)


def stokes_grad_eval(x, y, alpha, tx, ty, mu, nthreads=0):
    """Target gradient of the stresslet double layer of mu ([2][N]) at off-surface
    targets; returns [2][2][m] = d u_a / d x_l."""
    x, y, tx, ty = _c(x), _c(y), _c(tx), _c(ty)
    mu = _c(mu).reshape(2, -1)
    m = tx.size
    g = np.zeros((4, m))
    m1, m2 = np.ascontiguousarray(mu[0]), np.ascontiguousarray(mu[1])
    rc = lib().orc_stokes_grad_eval(_p(x), _p(y), x.size // 16, _p(m1), _p(m2), float(alpha), _p(tx), _p(ty), m,
                                    _p(g), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_stokes_grad_eval failed: {rc}")
    return g.reshape(2, 2, m)


def stokes_matrix(x, y, alpha, nthreads=0):
    """Dense on-surface principal-value stresslet matrix, 2N x 2N (rows a N + i)."""
    x, y = _c(x), _c(y)
    n = x.size
    Dm = np.empty((2 * n, 2 * n))
    rc = lib().orc_stokes_matrix(_p(x), _p(y), n // 16, float(alpha), _p(Dm), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_stokes_matrix failed: {rc}")
    return Dm


def stokes_bie_matrix(Dm, w, nx, ny):
    """1/2 I + D_pv + W with W mu = n (sum_j w_j mu_j . n_j) / sum_j w_j (Sec. 2.2)."""
    n = w.size
    nn = np.concatenate([nx, ny])
    wn = np.concatenate([w * nx, w * ny]) / np.sum(w)
    return 0.5 * np.eye(2 * n) + Dm + np.outer(nn, wn)


def onsurface_matrices(x, y, alpha, want_slp=False, want_dlp=True, nthreads=0):
    """Dense on-surface SLP and DLP (principal value, no 1/2 I) matrices."""
    x, y = _c(x), _c(y)
    n = x.size
    S = np.empty((n, n)) if want_slp else None
    D = np.empty((n, n)) if want_dlp else None
    rc = lib().orc_assemble_onsurface(_p(x), _p(y), n // 16, float(alpha), _p(S), _p(D), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"orc_assemble_onsurface failed: {rc}")
    return S, D


def apply_bie(D, mu):
    """(1/2 I + D) mu with the dense DLP matrix D."""
    return 0.5 * mu + D @ mu


def gmres(A, b, x0=None, tol=1e-10, restart=200, max_iter=1000, nthreads=0):
    """Dense GMRES (MGS Arnoldi) on A x = b, judged by the true relative residual."""
    A = _c(A)
    b = _c(b)
    n = b.size
    x = np.zeros(n) if x0 is None else _c(x0).copy()
    it = ctypes.c_int()
    rr = ctypes.c_double()
    rc = lib().orc_gmres(_p(A), n, _p(b), _p(x), float(tol), int(restart), int(max_iter), ctypes.byref(it),
                         ctypes.byref(rr), int(nthreads))
    return x, dict(iters=it.value, relres=rr.value, converged=(rc == 0))


def self_cell(alpha, h):
    return float(lib().orc_self_cell(float(alpha), float(h)))


def volume_eval(x, y, w, f, alpha, h, idx, nthreads=0):
    x, y, w, f = _c(x), _c(y), _c(w), _c(f)
    idx = _c(idx, np.int64)
    out = np.empty(idx.size)
    lib().orc_volume_eval(_p(x), _p(y), _p(w), _p(f), x.size, float(alpha), float(h),
                          idx.ctypes.data_as(_I64), idx.size, _p(out), int(nthreads))
    return out

"""Thin ctypes binding of ``libmhlp.so`` (include/mhlp.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch supplies device memory and the current stream.
Importing works without a GPU; any call raises if the library is missing or no
HIP device is present.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhlp.so")

FP64 = 0
MIXED = 1
WARM_RECURRENCE = -1  # warm-start base: learned per-coefficient recurrence

OK = 0
NOT_CONVERGED = 1

_lib = None

_c_double_p = ctypes.POINTER(ctypes.c_double)


class MhlpError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [("near_factor", ctypes.c_double), ("rho_direct", ctypes.c_double), ("rho_split", ctypes.c_double),
                ("ah_max", ctypes.c_double), ("far_exp", ctypes.c_double)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("use_x0", ctypes.c_int32)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("x0_residual", ctypes.c_double), ("converged", ctypes.c_int32), ("used_x0", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# every symbol the header declares: name -> (argtypes, restype)
_V = ctypes.c_void_p
_SIGS = {
    "mhlp_last_error": ([], ctypes.c_char_p),
    "mhlp_geometry_create": ([ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, _V, _V, _V,
                              ctypes.POINTER(_V)], ctypes.c_int32),
    "mhlp_geometry_info": ([_V, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32],
                           ctypes.c_int32),
    "mhlp_geometry_destroy": ([_V], ctypes.c_int32),
    "mhlp_geometry_arrays": ([_V, ctypes.POINTER(_V), ctypes.POINTER(_V), ctypes.POINTER(_V), ctypes.POINTER(_V)],
                             ctypes.c_int32),
    "mhlp_plan_create": ([_V, ctypes.c_double, _V, _V, ctypes.c_int64, ctypes.POINTER(Params), _V, ctypes.POINTER(_V)],
                         ctypes.c_int32),
    "mhlp_plan_destroy": ([_V], ctypes.c_int32),
    "mhlp_plan_info": ([_V, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                        ctypes.POINTER(ctypes.c_int64), _c_double_p], ctypes.c_int32),
    "mhlp_plan_set_split": ([_V, ctypes.c_int32], ctypes.c_int32),
    "mhlp_plan_get_split": ([_V, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int32),
    "mhlp_plan_autotune": ([_V, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _V, ctypes.POINTER(ctypes.c_int32),
                            _c_double_p, ctypes.POINTER(ctypes.c_int32), _c_double_p, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int32)], ctypes.c_int32),
    "mhlp_eval_layer": ([_V, _V, _V, _V, _V, ctypes.c_int32, _V], ctypes.c_int32),
    "mhlp_eval_slp": ([_V, _V, _V, ctypes.c_int32, _V], ctypes.c_int32),
    "mhlp_eval_dlp": ([_V, _V, _V, ctypes.c_int32, _V], ctypes.c_int32),
    "mhlp_apply_bie_operator": ([_V, _V, _V, ctypes.c_int32, _V], ctypes.c_int32),
    "mhlp_eval_grad": ([_V, _V, _V, _V, _V, _V, _V, _V], ctypes.c_int32),
    "mhlp_stokes_plan_create": ([_V, ctypes.c_double, _V, _V, ctypes.c_int64, _V, _V, ctypes.POINTER(_V)],
                                ctypes.c_int32),
    "mhlp_stokes_eval": ([_V, _V, _V, _V], ctypes.c_int32),
    "mhlp_stokes_apply_bie": ([_V, _V, _V, _V], ctypes.c_int32),
    "mhlp_stokes_eval_grad": ([_V, _V, _V, _V], ctypes.c_int32),
    "mhlp_plan_set_fmm": ([_V, ctypes.c_int32, ctypes.c_int32, _V], ctypes.c_int32),
    "mhlp_plan_get_fmm": ([_V, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int32),
    "mhlp_volume_fmm_create": ([_V, _V, _V, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                ctypes.c_int32, _V, ctypes.POINTER(_V)], ctypes.c_int32),
    "mhlp_volume_fmm_eval": ([_V, _V, _V, _V], ctypes.c_int32),
    "mhlp_volume_fmm_info": ([_V, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _c_double_p],
                             ctypes.c_int32),
    "mhlp_volume_fmm_destroy": ([_V], ctypes.c_int32),
    "mhlp_box_create": ([ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double, _V,
                         ctypes.POINTER(_V)], ctypes.c_int32),
    "mhlp_box_particular": ([_V, _V, _V, _V, ctypes.c_int64, _V, _V, _V, _V], ctypes.c_int32),
    "mhlp_box_destroy": ([_V], ctypes.c_int32),
    "mhlp_box_set_point_method": ([_V, ctypes.c_int32], ctypes.c_int32),
    "mhlp_sisdc_step": ([_V, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _V, _V, _V, _V], ctypes.c_int32),
    "mhlp_stokes_gmres_solve": ([_V, _V, _V, ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresInfo), _V],
                                ctypes.c_int32),
    "mhlp_gmres_solve": ([_V, _V, _V, ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresInfo), _V], ctypes.c_int32),
    "mhlp_batch_create": ([ctypes.c_int32, ctypes.POINTER(_V), ctypes.c_int32, _V, ctypes.POINTER(_V)],
                          ctypes.c_int32),
    "mhlp_batch_destroy": ([_V], ctypes.c_int32),
    "mhlp_batch_info": ([_V, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], ctypes.c_int32),
    "mhlp_batch_apply_bie": ([_V, _V, _V, _V], ctypes.c_int32),
    "mhlp_batch_autotune": ([_V, ctypes.c_int32, _V, ctypes.POINTER(ctypes.c_int64), _c_double_p], ctypes.c_int32),
    "mhlp_batch_set_tile": ([_V, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _V], ctypes.c_int32),
    "mhlp_batch_tile": ([_V, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), _c_double_p, ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_int32)], ctypes.c_int32),
    "mhlp_batch_gmres_solve": ([_V, _V, _V, ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresInfo), _V],
                               ctypes.c_int32),
    "mhlp_volume_eval": ([_V, _V, _V, _V, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32, _V,
                          _c_double_p, _V], ctypes.c_int32),
    "mhlp_volume_eval_noalloc": ([_V, _V, _V, _V, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                  _V, _V], ctypes.c_int32),
    "mhlp_mlp_create": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _V, ctypes.POINTER(_V)],
                        ctypes.c_int32),
    "mhlp_mlp_destroy": ([_V], ctypes.c_int32),
    "mhlp_mlp_info": ([_V, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int32),
    "mhlp_mlp_params": ([_V, _V, _V, _V], ctypes.c_int32),
    "mhlp_mlp_forward": ([_V, _V, ctypes.c_int32, _V, _V], ctypes.c_int32),
    "mhlp_mlp_loss_grad": ([_V, _V, _V, ctypes.c_int32, _V, _V, _V], ctypes.c_int32),
    "mhlp_mlp_adam_step": ([_V, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _V], ctypes.c_int32),
    "mhlp_gemm_bf16": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _V, ctypes.c_int64, ctypes.c_int64, _V,
                        ctypes.c_int64, ctypes.c_int64, _V, ctypes.c_int64, _V], ctypes.c_int32),
    "mhlp_warm_create": ([_V, _V, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _V, ctypes.POINTER(_V)], ctypes.c_int32),
    "mhlp_warm_destroy": ([_V], ctypes.c_int32),
    "mhlp_warm_info": ([_V, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_V),
                        _c_double_p], ctypes.c_int32),
    "mhlp_warm_coefficients": ([_V, _V, ctypes.c_int32, _V, _V], ctypes.c_int32),
    "mhlp_warm_synthesize": ([_V, _V, ctypes.c_int32, _V, _V, _V], ctypes.c_int32),
    "mhlp_warm_train": ([_V, _V, ctypes.c_int32, ctypes.c_int32, ctypes.c_float, ctypes.POINTER(ctypes.c_float), _V],
                        ctypes.c_int32),
    "mhlp_warm_predict": ([_V, _V, _V, _V], ctypes.c_int32),
}


def load(path: str = LIB_PATH):
    """Load the library (raises MhlpError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise MhlpError(f"{path} is not built; run __graft_entry__.build() or paper_1908_07392_amd/build.py")
    L = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc, what):
    if rc < 0:
        msg = load().mhlp_last_error().decode(errors="replace")
        raise MhlpError(f"{what} failed ({rc}): {msg}")
    return rc


def _dev(t: torch.Tensor, name: str, n: int | None = None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise MhlpError(f"{name} must be a HIP device tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise MhlpError(f"{name} must be contiguous float64")
    if n is not None and t.numel() != n:
        raise MhlpError(f"{name} must have {n} elements, has {t.numel()}")
    return t.data_ptr()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Geometry:
    """Panel geometry on the device from a ``[6][N]`` float64 node array.

    curve_panel_offsets: first panel of each closed curve, then the panel
    count (host sequence; default: one curve).  panel_ends: optional device
    ``[4][Np]`` float64 (xa, ya, xb, yb), checked by the library against the
    node data and the curve chain."""

    def __init__(self, node_soa: torch.Tensor, curve_panel_offsets=None, panel_ends: torch.Tensor | None = None):
        L = load()
        if node_soa.dim() != 2 or node_soa.shape[0] != 6 or node_soa.shape[1] % 16:
            raise MhlpError("node_soa must be [6][16*n_panels]")
        self.n_nodes = int(node_soa.shape[1])
        self.n_panels = self.n_nodes // 16
        self.device = node_soa.device
        if curve_panel_offsets is None:
            curve_panel_offsets = [0, self.n_panels]
        offs = [int(v) for v in curve_panel_offsets]
        if len(offs) < 2 or offs[-1] != self.n_panels:
            raise MhlpError("curve_panel_offsets must end with the panel count of node_soa")
        if panel_ends is not None and tuple(panel_ends.shape) != (4, self.n_panels):
            raise MhlpError("panel_ends must be [4][n_panels]")
        self.curve_panel_offsets = offs
        c_offs = (ctypes.c_int32 * len(offs))(*offs)
        h = ctypes.c_void_p()
        ends = _dev(panel_ends, "panel_ends") if panel_ends is not None else None
        _check(L.mhlp_geometry_create(len(offs) - 1, c_offs, 16, _dev(node_soa, "node_soa"), ends, _stream(),
                                      ctypes.byref(h)), "geometry_create")
        self._h = h

    def info(self):
        """(n_nodes, n_panels, curve_panel_offsets) as the library holds them."""
        n, np_, nc = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(load().mhlp_geometry_info(self._h, ctypes.byref(n), ctypes.byref(np_), ctypes.byref(nc), None, 0),
               "geometry_info")
        offs = (ctypes.c_int32 * (nc.value + 1))()
        _check(load().mhlp_geometry_info(self._h, None, None, None, offs, nc.value + 1), "geometry_info")
        return n.value, np_.value, list(offs)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load().mhlp_geometry_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Targets + near-field corrections (``tx``/``ty`` None: on-surface plan).
    ``stokes=True`` builds the modified-Stokes (stresslet) plan of the
    ``stokes_*`` calls."""

    def __init__(self, geom: Geometry, alpha: float, tx: torch.Tensor | None = None, ty: torch.Tensor | None = None,
                 params: dict | None = None, stokes: bool = False):
        L = load()
        self.geom = geom
        self.alpha = float(alpha)
        self.stokes = bool(stokes)
        prm = None
        if params:
            prm = Params(**{k: float(v) for k, v in params.items()})
        h = ctypes.c_void_p()
        if tx is None:
            m, ptx, pty = 0, None, None
        else:
            m = int(tx.numel())
            ptx, pty = _dev(tx, "tx"), _dev(ty, "ty", m)
        create = L.mhlp_stokes_plan_create if self.stokes else L.mhlp_plan_create
        _check(create(geom.handle, self.alpha, ptx, pty, m, ctypes.byref(prm) if prm else None, _stream(),
                      ctypes.byref(h)), "plan_create")
        self._h = h
        nt, ns, nn = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(L.mhlp_plan_info(h, ctypes.byref(nt), ctypes.byref(ns), ctypes.byref(nn), None), "plan_info")
        self.n_targets, self.n_sources, self.n_near_pairs = nt.value, ns.value, nn.value
        self.onsurface = tx is None

    @property
    def handle(self):
        return self._h

    @property
    def nsplit(self) -> int:
        v = ctypes.c_int32()
        _check(load().mhlp_plan_get_split(self._h, ctypes.byref(v)), "plan_get_split")
        return v.value

    def set_split(self, nsplit: int):
        _check(load().mhlp_plan_set_split(self._h, int(nsplit)), "plan_set_split")

    def autotune(self, layers: int = 3, precision=FP64, reps: int = 5):
        """Time the far evaluation over source-split counts and keep the fastest.
        layers: 1 SLP, 2 DLP, 3 both, 4 BIE operator, 5 gradients, 6 stresslet operator of a stokes
        plan, 7 stresslet gradient (off-surface stokes plan).  Returns (best, best_ms, {nsplit: ms})."""
        cap = 32
        cand, cms = (ctypes.c_int32 * cap)(), (ctypes.c_double * cap)()
        best, bms, nc = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
        _check(load().mhlp_plan_autotune(self._h, int(layers), int(precision), int(reps), _stream(), ctypes.byref(best),
                                         ctypes.byref(bms), cand, cms, cap, ctypes.byref(nc)), "plan_autotune")
        return best.value, bms.value, {cand[i]: cms[i] for i in range(nc.value)}

    def set_fmm(self, order: int = 40, leaf_level: int = -1):
        """FMM far field for FP64 evaluations of an off-surface plan (order 0: off)."""
        _check(load().mhlp_plan_set_fmm(self._h, int(order), int(leaf_level), _stream()), "plan_set_fmm")

    @property
    def fmm(self):
        """(order, leaf level) of the plan's FMM; (0, -1) when the far field is direct."""
        o, lv = ctypes.c_int32(), ctypes.c_int32()
        _check(load().mhlp_plan_get_fmm(self._h, ctypes.byref(o), ctypes.byref(lv)), "plan_get_fmm")
        return o.value, lv.value

    def close(self):
        if getattr(self, "_h", None):
            load().mhlp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eval_layer(plan: Plan, sigma=None, mu=None, precision=FP64, out_slp=None, out_dlp=None):
    """Single layer of sigma and/or double layer of mu at the plan's targets."""
    L = load()
    N, M = plan.n_sources, plan.n_targets
    dev = plan.geom.device
    ps = pm = us = ud = None
    if sigma is not None:
        ps = _dev(sigma, "sigma", N)
        out_slp = torch.empty(M, dtype=torch.float64, device=dev) if out_slp is None else out_slp
        us = _dev(out_slp, "u_slp", M)
    if mu is not None:
        pm = _dev(mu, "mu", N)
        out_dlp = torch.empty(M, dtype=torch.float64, device=dev) if out_dlp is None else out_dlp
        ud = _dev(out_dlp, "u_dlp", M)
    _check(L.mhlp_eval_layer(plan.handle, ps, pm, us, ud, int(precision), _stream()), "eval_layer")
    return (out_slp if sigma is not None else None), (out_dlp if mu is not None else None)


def eval_slp(plan: Plan, sigma, precision=FP64, out=None):
    """S[sigma] at the plan's targets (mhlp_eval_slp)."""
    L = load()
    out = torch.empty(plan.n_targets, dtype=torch.float64, device=plan.geom.device) if out is None else out
    _check(L.mhlp_eval_slp(plan.handle, _dev(sigma, "sigma", plan.n_sources), _dev(out, "u", plan.n_targets),
                           int(precision), _stream()), "eval_slp")
    return out


def eval_dlp(plan: Plan, mu, precision=FP64, out=None):
    """D[mu] at the plan's targets (mhlp_eval_dlp; principal value on an on-surface plan)."""
    L = load()
    out = torch.empty(plan.n_targets, dtype=torch.float64, device=plan.geom.device) if out is None else out
    _check(L.mhlp_eval_dlp(plan.handle, _dev(mu, "mu", plan.n_sources), _dev(out, "u", plan.n_targets),
                           int(precision), _stream()), "eval_dlp")
    return out


def eval_grad(plan: Plan, sigma=None, mu=None, out_slp=None, out_dlp=None):
    """Target gradients of the single layer of sigma and/or the double layer of
    mu on an off-surface plan; each result is a [2][M] float64 tensor (x1 and
    x2 components) or None."""
    L = load()
    N, M = plan.n_sources, plan.n_targets
    dev = plan.geom.device
    ps = pm = None
    gs = [None, None]
    gd = [None, None]
    if sigma is not None:
        ps = _dev(sigma, "sigma", N)
        out_slp = torch.empty(2, M, dtype=torch.float64, device=dev) if out_slp is None else out_slp
        gs = [_dev(out_slp[0], "grad_slp[0]", M), _dev(out_slp[1], "grad_slp[1]", M)]
    if mu is not None:
        pm = _dev(mu, "mu", N)
        out_dlp = torch.empty(2, M, dtype=torch.float64, device=dev) if out_dlp is None else out_dlp
        gd = [_dev(out_dlp[0], "grad_dlp[0]", M), _dev(out_dlp[1], "grad_dlp[1]", M)]
    _check(L.mhlp_eval_grad(plan.handle, ps, pm, gs[0], gs[1], gd[0], gd[1], _stream()), "eval_grad")
    return (out_slp if sigma is not None else None), (out_dlp if mu is not None else None)


def stokes_eval(plan: Plan, mu, out=None):
    """Modified-Stokes double layer of mu ([2][N] float64) at the plan's targets; returns [2][M]."""
    L = load()
    N, M = plan.n_sources, plan.n_targets
    out = torch.empty(2, M, dtype=torch.float64, device=plan.geom.device) if out is None else out
    _check(L.mhlp_stokes_eval(plan.handle, _dev(mu, "mu", 2 * N), _dev(out, "u", 2 * M), _stream()), "stokes_eval")
    return out


def stokes_eval_grad(plan: Plan, mu, out=None):
    """Target gradient of the modified-Stokes double layer of mu ([2][N]) on an
    off-surface stokes plan; returns [2][2][M] float64, out[i][l] = d u_i / d x_l."""
    L = load()
    N, M = plan.n_sources, plan.n_targets
    out = torch.empty(2, 2, M, dtype=torch.float64, device=plan.geom.device) if out is None else out
    _check(L.mhlp_stokes_eval_grad(plan.handle, _dev(mu, "mu", 2 * N), _dev(out, "g", 4 * M), _stream()),
           "stokes_eval_grad")
    return out


def stokes_apply_bie(plan: Plan, mu, out=None):
    """(1/2 I + D + W) mu on an on-surface stokes plan; mu and the result [2][N]."""
    L = load()
    N = plan.n_sources
    out = torch.empty(2, N, dtype=torch.float64, device=plan.geom.device) if out is None else out
    _check(L.mhlp_stokes_apply_bie(plan.handle, _dev(mu, "mu", 2 * N), _dev(out, "out", 2 * N), _stream()),
           "stokes_apply_bie")
    return out


def stokes_gmres_solve(plan: Plan, g, x0=None, tol=1e-10, max_iter=500, restart=100):
    """Solve (1/2 I + D + W) mu = g ([2][N]); returns (mu, info dict)."""
    L = load()
    N = plan.n_sources
    mu = torch.zeros(2, N, dtype=torch.float64, device=plan.geom.device) if x0 is None else x0.clone()
    opts = GmresOpts(float(tol), int(max_iter), int(restart), FP64, 0 if x0 is None else 1)
    info = GmresInfo()
    rc = L.mhlp_stokes_gmres_solve(plan.handle, _dev(g, "g", 2 * N), _dev(mu, "mu", 2 * N), ctypes.byref(opts),
                                   ctypes.byref(info), _stream())
    _check(rc, "stokes_gmres_solve")
    return mu, info.as_dict()


def apply_bie(plan: Plan, mu, precision=FP64, out=None):
    """(1/2 I + D) mu on an on-surface plan."""
    L = load()
    N = plan.n_sources
    out = torch.empty(N, dtype=torch.float64, device=plan.geom.device) if out is None else out
    _check(L.mhlp_apply_bie_operator(plan.handle, _dev(mu, "mu", N), _dev(out, "out", N), int(precision), _stream()),
           "apply_bie_operator")
    return out


def gmres_solve(plan: Plan, g, x0=None, tol=1e-10, max_iter=500, restart=100, precision=FP64):
    """Solve (1/2 I + D) mu = g; returns (mu, info dict)."""
    L = load()
    N = plan.n_sources
    mu = torch.zeros(N, dtype=torch.float64, device=plan.geom.device) if x0 is None else x0.clone()
    opts = GmresOpts(float(tol), int(max_iter), int(restart), int(precision), 0 if x0 is None else 1)
    info = GmresInfo()
    rc = L.mhlp_gmres_solve(plan.handle, _dev(g, "g", N), _dev(mu, "mu", N), ctypes.byref(opts), ctypes.byref(info),
                            _stream())
    _check(rc, "gmres_solve")
    return mu, info.as_dict()


def volume_eval(x, y, w, f, alpha, h, precision=FP64, out=None):
    """All-pairs volume sum with self-cell correction; returns (u, Wcell)."""
    L = load()
    n = x.numel()
    out = torch.empty(n, dtype=torch.float64, device=x.device) if out is None else out
    wc = ctypes.c_double()
    _check(L.mhlp_volume_eval(_dev(x, "x", n), _dev(y, "y", n), _dev(w, "w", n), _dev(f, "f", n), n, float(alpha),
                              float(h), int(precision), _dev(out, "u", n), ctypes.byref(wc), _stream()),
           "volume_eval")
    return out, wc.value


def volume_eval_noalloc(x, y, w, f, alpha, h, out, precision=FP64):
    """``volume_eval`` into the caller's ``out`` through the entry point that
    allocates nothing (fixed device scratch shared by all calls on a device)."""
    L = load()
    n = x.numel()
    _check(L.mhlp_volume_eval_noalloc(_dev(x, "x", n), _dev(y, "y", n), _dev(w, "w", n), _dev(f, "f", n), n,
                                      float(alpha), float(h), int(precision), _dev(out, "u", n), _stream()),
           "volume_eval_noalloc")
    return out


class VolumeFMM:
    """The volume sum of ``volume_eval`` by the FMM; the tree of the points is
    built once, ``eval(f)`` returns u."""

    def __init__(self, x, y, w, alpha, h, order: int = 40, leaf_level: int = -1):
        L = load()
        self.n = int(x.numel())
        self.device = x.device
        hnd = ctypes.c_void_p()
        _check(L.mhlp_volume_fmm_create(_dev(x, "x", self.n), _dev(y, "y", self.n), _dev(w, "w", self.n), self.n,
                                        float(alpha), float(h), int(order), int(leaf_level), _stream(),
                                        ctypes.byref(hnd)), "volume_fmm_create")
        self._h = hnd
        o, lv, wc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(L.mhlp_volume_fmm_info(hnd, ctypes.byref(o), ctypes.byref(lv), ctypes.byref(wc)), "volume_fmm_info")
        self.order, self.leaf_level, self.self_cell = o.value, lv.value, wc.value

    def eval(self, f, out=None):
        out = torch.empty(self.n, dtype=torch.float64, device=self.device) if out is None else out
        _check(load().mhlp_volume_fmm_eval(self._h, _dev(f, "f", self.n), _dev(out, "u", self.n), _stream()),
               "volume_fmm_eval")
        return out

    def close(self):
        if getattr(self, "_h", None):
            load().mhlp_volume_fmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Box:
    """Periodic box [x0, x0+Lb) x [y0, y0+Lb) with an M x M grid for the particular
    solution of the modified Stokes equations (``particular``)."""

    def __init__(self, M: int, x0: float, y0: float, Lb: float, alpha: float, device="cuda:0"):
        hnd = ctypes.c_void_p()
        _check(load().mhlp_box_create(int(M), float(x0), float(y0), float(Lb), float(alpha), _stream(),
                                      ctypes.byref(hnd)), "box_create")
        self._h = hnd
        self.M, self.x0, self.y0, self.Lb, self.alpha = int(M), float(x0), float(y0), float(Lb), float(alpha)
        self.device = device

    def particular(self, F, want_u=True, want_grad=False, px=None, py=None):
        """F: [2][M][M] float64 on the device.  Returns (u [2][M][M] or None,
        grad [4][M][M] or None, up [2][n] at the points or None)."""
        M = self.M
        MM = M * M
        u = torch.empty(2, M, M, dtype=torch.float64, device=self.device) if want_u else None
        g = torch.empty(4, M, M, dtype=torch.float64, device=self.device) if want_grad else None
        n = 0 if px is None else int(px.numel())
        up = torch.empty(2, n, dtype=torch.float64, device=self.device) if n else None
        _check(load().mhlp_box_particular(self._h, _dev(F, "F", 2 * MM), None if u is None else _dev(u, "u", 2 * MM),
                                          None if g is None else _dev(g, "grad", 4 * MM), n,
                                          _dev(px, "px", n) if n else None, _dev(py, "py", n) if n else None,
                                          _dev(up, "up", 2 * n) if n else None, _stream()), "box_particular")
        return u, g, up

    def set_point_method(self, method: int):
        """0: direct type-2 sums; 1: non-uniform FFT (default for M <= 1024)."""
        _check(load().mhlp_box_set_point_method(self._h, int(method)), "box_set_point_method")

    def sisdc_step(self, Re, dt, K, u, grad, lap):
        """One SISDC step of periodic Navier-Stokes in place on u [2][M][M], grad [4][M][M], lap [2][M][M]."""
        MM = self.M * self.M
        _check(load().mhlp_sisdc_step(self._h, float(Re), float(dt), int(K), _dev(u, "u", 2 * MM),
                                      _dev(grad, "grad", 4 * MM), _dev(lap, "lap", 2 * MM), _stream()), "sisdc_step")

    def close(self):
        if getattr(self, "_h", None):
            load().mhlp_box_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many on-surface systems (geometries x right-hand sides) solved together."""

    def __init__(self, plans, n_rhs: int):
        L = load()
        self.plans = list(plans)
        self.n_rhs = int(n_rhs)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(L.mhlp_batch_create(len(self.plans), arr, self.n_rhs, _stream(), ctypes.byref(h)), "batch_create")
        self._h = h
        tot, ns = ctypes.c_int64(), ctypes.c_int32()
        _check(L.mhlp_batch_info(h, ctypes.byref(tot), ctypes.byref(ns), None, None), "batch_info")
        off = (ctypes.c_int64 * ns.value)()
        ln = (ctypes.c_int64 * ns.value)()
        _check(L.mhlp_batch_info(h, None, None, off, ln), "batch_info")
        self.total, self.n_systems = tot.value, ns.value
        self.offsets, self.lengths = list(off), list(ln)
        self.device = self.plans[0].geom.device

    def pack(self, per_system):
        """Concatenate per-system device vectors into one batched vector."""
        return torch.cat([v.reshape(-1) for v in per_system]).contiguous()

    def unpack(self, v):
        return [v[o:o + n] for o, n in zip(self.offsets, self.lengths)]

    def apply(self, mu, out=None):
        out = torch.empty(self.total, dtype=torch.float64, device=self.device) if out is None else out
        _check(load().mhlp_batch_apply_bie(self._h, _dev(mu, "mu", self.total), _dev(out, "out", self.total),
                                           _stream()), "batch_apply_bie")
        return out

    def autotune(self, reps: int = 3):
        """Pick the launch shape of the grouped operator (block target, targets
        per lane, sources per LDS stage); returns (target, ms)."""
        tg, ms = ctypes.c_int64(), ctypes.c_double()
        _check(load().mhlp_batch_autotune(self._h, int(reps), _stream(), ctypes.byref(tg), ctypes.byref(ms)),
               "batch_autotune")
        return tg.value, ms.value

    def set_tile(self, target: int, targets_per_lane: int = 1, sources_per_stage: int = 256):
        _check(load().mhlp_batch_set_tile(self._h, int(target), int(targets_per_lane), int(sources_per_stage),
                                          _stream()), "batch_set_tile")

    def tile(self):
        """{'target', 'targets_per_lane', 'sources_per_stage', 'candidates': [(target, tpl, src, ms), ...]}"""
        L = load()
        tg, tpl, src, n = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(L.mhlp_batch_tile(self._h, ctypes.byref(tg), ctypes.byref(tpl), ctypes.byref(src), None, None, 0,
                                 ctypes.byref(n)), "batch_tile")
        cand = (ctypes.c_int64 * (3 * max(n.value, 1)))()
        cms = (ctypes.c_double * max(n.value, 1))()
        _check(L.mhlp_batch_tile(self._h, None, None, None, cand, cms, n.value, None), "batch_tile")
        rows = [(cand[3 * c], cand[3 * c + 1], cand[3 * c + 2], cms[c]) for c in range(n.value)]
        return {"target": tg.value, "targets_per_lane": tpl.value, "sources_per_stage": src.value,
                "candidates": rows}

    def gmres(self, g, x0=None, tol=1e-10, max_iter=500, restart=64):
        mu = torch.zeros(self.total, dtype=torch.float64, device=self.device) if x0 is None else x0.clone()
        opts = GmresOpts(float(tol), int(max_iter), int(restart), FP64, 0 if x0 is None else 1)
        infos = (GmresInfo * self.n_systems)()
        _check(load().mhlp_batch_gmres_solve(self._h, _dev(g, "g", self.total), _dev(mu, "mu", self.total),
                                             ctypes.byref(opts), infos, _stream()), "batch_gmres_solve")
        return mu, [i.as_dict() for i in infos]

    def close(self):
        if getattr(self, "_h", None):
            load().mhlp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _devf(t: torch.Tensor, name: str, n: int | None = None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise MhlpError(f"{name} must be a HIP device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise MhlpError(f"{name} must be contiguous float32")
    if n is not None and t.numel() != n:
        raise MhlpError(f"{name} must have {n} elements, has {t.numel()}")
    return t.data_ptr()


def gemm_bf16(A, B, transA=False, transB=False):
    """C = op(A) op(B) with BF16 operands and FP32 accumulation (2-D float32)."""
    m, k = (A.shape[1], A.shape[0]) if transA else (A.shape[0], A.shape[1])
    k2, n = (B.shape[1], B.shape[0]) if transB else (B.shape[0], B.shape[1])
    if k != k2:
        raise MhlpError("inner dimensions differ")
    sam, sak = (1, A.shape[1]) if transA else (A.shape[1], 1)
    sbk, sbn = (1, B.shape[1]) if transB else (B.shape[1], 1)
    C = torch.empty(m, n, dtype=torch.float32, device=A.device)
    _check(load().mhlp_gemm_bf16(m, n, k, _devf(A, "A"), sam, sak, _devf(B, "B"), sbk, sbn, _devf(C, "C"), n,
                                 _stream()), "gemm_bf16")
    return C


class MLP:
    """n_in -> width -> width -> n_out network with BF16 matrix-core products."""

    def __init__(self, n_in: int, width: int, n_out: int, seed: int = 0, handle=None, device="cuda"):
        L = load()
        self._owned = handle is None
        if handle is None:
            h = ctypes.c_void_p()
            _check(L.mhlp_mlp_create(int(n_in), int(width), int(n_out), int(seed), _stream(), ctypes.byref(h)),
                   "mlp_create")
            self._h = h
        else:
            self._h = handle
        npar, sizes = ctypes.c_int64(), (ctypes.c_int32 * 4)()
        _check(L.mhlp_mlp_info(self._h, ctypes.byref(npar), sizes), "mlp_info")
        self.n_params, self.sizes = npar.value, list(sizes)
        self.device = torch.device(device)

    def get_params(self):
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(load().mhlp_mlp_params(self._h, _devf(out, "dst"), None, _stream()), "mlp_params")
        return out

    def set_params(self, p):
        _check(load().mhlp_mlp_params(self._h, None, _devf(p, "src", self.n_params), _stream()), "mlp_params")

    def forward(self, X):
        B = X.shape[0]
        Y = torch.empty(B, self.sizes[3], dtype=torch.float32, device=self.device)
        _check(load().mhlp_mlp_forward(self._h, _devf(X, "X", B * self.sizes[0]), B, _devf(Y, "Y"), _stream()),
               "mlp_forward")
        return Y

    def loss_grad(self, X, T):
        B = X.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(load().mhlp_mlp_loss_grad(self._h, _devf(X, "X", B * self.sizes[0]), _devf(T, "T", B * self.sizes[3]),
                                         B, _devf(loss, "loss"), _devf(grad, "grad"), _stream()), "mlp_loss_grad")
        return loss, grad

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(load().mhlp_mlp_adam_step(self._h, lr, beta1, beta2, eps, _stream()), "mlp_adam_step")

    def close(self):
        if getattr(self, "_h", None) and self._owned:
            load().mhlp_mlp_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WarmStart:
    """Learned GMRES initial guess from the last ``n_hist`` densities."""

    def __init__(self, theta, omega, curve_ptr, n_modes=128, n_hist=4, base_order=3, width=256, seed=0):
        L = load()
        self.n_nodes = int(theta.numel())
        self.n_curves = len(curve_ptr) - 1
        cp = (ctypes.c_int64 * len(curve_ptr))(*[int(v) for v in curve_ptr])
        if cp[len(curve_ptr) - 1] != self.n_nodes:
            raise MhlpError("curve_ptr[-1] must equal the node count")
        self.n_hist = int(n_hist)
        self.device = theta.device
        h = ctypes.c_void_p()
        _check(L.mhlp_warm_create(_dev(theta, "theta"), _dev(omega, "omega", self.n_nodes), cp, self.n_curves,
                                  int(n_modes), self.n_hist, int(base_order), int(width), int(seed), _stream(),
                                  ctypes.byref(h)),
               "warm_create")
        self._h = h
        nf, net = ctypes.c_int64(), ctypes.c_void_p()
        _check(L.mhlp_warm_info(h, None, ctypes.byref(nf), ctypes.byref(net), None), "warm_info")
        self.n_features = nf.value
        self.mlp = MLP(0, 0, 0, handle=net, device=self.device)

    def scales(self):
        """(input group factors [n_hist], output unit)."""
        sc = (ctypes.c_double * (self.n_hist + 1))()
        _check(load().mhlp_warm_info(self._h, None, None, None, sc), "warm_info")
        return list(sc)[:self.n_hist], sc[self.n_hist]

    def coefficients(self, mu):
        mu2 = mu.reshape(-1, self.n_nodes)
        d = mu2.shape[0]
        coef = torch.empty(d, self.n_features, dtype=torch.float64, device=self.device)
        _check(load().mhlp_warm_coefficients(self._h, _dev(mu2, "mu"), d, _dev(coef, "coef"), _stream()),
               "warm_coefficients")
        return coef

    def synthesize(self, coef, base=None):
        c2 = coef.reshape(-1, self.n_features)
        d = c2.shape[0]
        out = torch.empty(d, self.n_nodes, dtype=torch.float64, device=self.device)
        pb = None if base is None else _dev(base, "base", d * self.n_nodes)
        _check(load().mhlp_warm_synthesize(self._h, _dev(c2, "coef"), d, pb, _dev(out, "out"), _stream()),
               "warm_synthesize")
        return out

    def train(self, mus, iters=2000, lr=1e-3):
        n_steps = mus.shape[0]
        losses = (ctypes.c_float * max(int(iters), 1))()
        _check(load().mhlp_warm_train(self._h, _dev(mus, "mus", n_steps * self.n_nodes), n_steps, int(iters),
                                      float(lr), losses, _stream()), "warm_train")
        return list(losses)[:int(iters)]

    def predict(self, hist, out=None):
        out = torch.empty(self.n_nodes, dtype=torch.float64, device=self.device) if out is None else out
        _check(load().mhlp_warm_predict(self._h, _dev(hist, "hist", self.n_hist * self.n_nodes),
                                        _dev(out, "x0", self.n_nodes), _stream()), "warm_predict")
        return out

    def close(self):
        if getattr(self, "_h", None):
            self.mlp._h = None
            load().mhlp_warm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""The allocation-free volume sum (mhlp_volume_eval_noalloc) against
mhlp_volume_eval, through the C ABI: two calls in a row on the library's fixed
device scratch, the second with a smaller input, each compared with the
allocating entry point (same kernels and launch shape; bar 1e-12 relative, the
FP64 volume parity bar, and 1e-6 for the FP32 far field)."""
import numpy as np
import pytest
import torch

from paper_1908_07392_amd import mhlp

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _grid(n, L=1.5, seed=0):
    g = np.linspace(-L, L, n)
    h = g[1] - g[0]
    X, Y = np.meshgrid(g, g)
    w1 = np.full(n, h)
    w1[[0, -1]] = h / 2
    rng = np.random.default_rng(seed)
    f = np.zeros_like(X)
    for _ in range(6):
        c = rng.uniform(-L, L, 2)
        s = rng.uniform(0.05, 0.3)
        f += rng.standard_normal() * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2) / (2 * s * s))
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a.ravel()), dtype=torch.float64, device=DEV)  # noqa: E731
    return t(X), t(Y), t(np.outer(w1, w1)), t(f), h


def _relerr(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("sizes", [(256, 37), (520, 50)])
def test_noalloc_matches_volume_eval(sizes):
    alpha = 20.0
    for n, precision, tol in ((sizes[0], mhlp.FP64, 1e-12), (sizes[1], mhlp.FP64, 1e-12),
                              (sizes[1], mhlp.MIXED, 1e-6)):
        x, y, w, f, h = _grid(n, seed=n)
        print(f"noalloc n={n * n} precision={precision}", flush=True)
        ref, _ = mhlp.volume_eval(x, y, w, f, alpha, h, precision=precision)
        out = torch.full_like(ref, float("nan"))
        mhlp.volume_eval_noalloc(x, y, w, f, alpha, h, out, precision=precision)
        torch.cuda.synchronize()
        err = _relerr(out, ref)
        print(f"  rel err vs volume_eval {err:.2e} (bit-identical: {bool(torch.equal(out, ref))})", flush=True)
        assert torch.isfinite(out).all()
        assert err <= tol


def test_noalloc_rejects_bad_arguments():
    x, y, w, f, h = _grid(8)
    out = torch.empty_like(x)
    with pytest.raises(mhlp.MhlpError):
        mhlp.volume_eval_noalloc(x, y, w, f, -1.0, h, out)
    with pytest.raises(mhlp.MhlpError):
        mhlp.volume_eval_noalloc(x, y, w, f, 20.0, h, out, precision=7)

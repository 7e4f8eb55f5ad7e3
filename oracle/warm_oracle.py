"""FP64 oracle of the learned warm start (test infrastructure only).

Plain numpy, written from the definitions; shares no code with the HIP
library and is imported only by the tests, the smoke check and the CPU leg of
the benchmark.

* Fourier features of a density on each closed curve, in the curve parameter
  theta: c_k = (1/2 pi) int_0^{2 pi} mu(theta) e^{-i k theta} d theta, by the
  composite panel rule in theta, and the real Fourier series back.
* The network n_in -> width -> width -> n_out, GELU (tanh form) after the two
  hidden layers, mean-squared-error loss, back-propagation, Adam.  Weights may
  be rounded to BF16 (round to nearest even) before use, as the matrix cores
  see them; everything else is FP64.
* The warm-start data: network inputs are the backward differences of a
  window of coefficient rows, targets the error of a base prediction of the
  next row: polynomial extrapolation of the window, or a per-coefficient
  linear recurrence fitted by regularised least squares over the series.

Parameter layout (shared convention with the library): for l = 0, 1, 2 the
weight W_l as a row-major [n_{l+1}][n_l] block followed by the bias b_l.
"""
from __future__ import annotations

import math

import numpy as np

SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)
GELU_CUBIC = 0.044715


# --------------------------------------------------------------------------------------
# BF16
# --------------------------------------------------------------------------------------
def bf16_round(x) -> np.ndarray:
    """Nearest-even BF16 value (8-bit significand) of each FP32 number, as float64.

    BF16 keeps the top 16 bits of the IEEE binary32 pattern; the 16 dropped bits are
    rounded half to even."""
    b = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    low = b & 0xFFFF
    high = b >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((high & 1) == 1))
    high = high + up.astype(np.uint64)
    return (high << 16).astype(np.uint32).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------------------
# network
# --------------------------------------------------------------------------------------
def gelu(z):
    """GELU in its tanh form: z/2 (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))."""
    return 0.5 * z * (1.0 + np.tanh(SQRT_2_OVER_PI * (z + GELU_CUBIC * z ** 3)))


def gelu_prime(z):
    u = SQRT_2_OVER_PI * (z + GELU_CUBIC * z ** 3)
    t = np.tanh(u)
    du = SQRT_2_OVER_PI * (1.0 + 3.0 * GELU_CUBIC * z ** 2)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * du


def layer_slices(sizes):
    """[(weight slice, bias slice)] of the flat parameter vector."""
    out, o = [], 0
    for l in range(3):
        nw = sizes[l + 1] * sizes[l]
        out.append((slice(o, o + nw), slice(o + nw, o + nw + sizes[l + 1])))
        o += nw + sizes[l + 1]
    return out


def n_params(sizes) -> int:
    return sum(sizes[l + 1] * sizes[l] + sizes[l + 1] for l in range(3))


def unpack(params, sizes, round_weights=True):
    p = np.asarray(params)
    Ws, bs = [], []
    for l, (sw, sb) in enumerate(layer_slices(sizes)):
        w = p[sw].reshape(sizes[l + 1], sizes[l])
        Ws.append(bf16_round(w) if round_weights else w.astype(np.float64))
        bs.append(p[sb].astype(np.float64))
    return Ws, bs


def mlp_forward(params, sizes, X, round_weights=True):
    """Returns (Y, cache) for a batch X [B][n_in]."""
    Ws, bs = unpack(params, sizes, round_weights)
    a = np.asarray(X, dtype=np.float64)
    acts, pre = [a], []
    for l in range(3):
        z = a @ Ws[l].T + bs[l]
        pre.append(z)
        a = gelu(z) if l < 2 else z
        acts.append(a)
    return a, dict(Ws=Ws, acts=acts, pre=pre)


def mlp_loss_grad(params, sizes, X, T, round_weights=True):
    """Loss mean((net(X) - T)^2) over all entries and its gradient (flat, FP64).

    With rounded weights the gradient is taken with respect to the rounded values
    (the usual mixed-precision convention: it is applied to the FP32 masters)."""
    Y, c = mlp_forward(params, sizes, X, round_weights)
    T = np.asarray(T, dtype=np.float64)
    n = Y.size
    loss = float(np.sum((Y - T) ** 2) / n)
    g = np.zeros(n_params(sizes))
    sl = layer_slices(sizes)
    dz = 2.0 * (Y - T) / n
    for l in (2, 1, 0):
        a_in = c["acts"][l]
        g[sl[l][0]] = (dz.T @ a_in).ravel()
        g[sl[l][1]] = dz.sum(axis=0)
        if l > 0:
            da = dz @ c["Ws"][l]
            dz = da * gelu_prime(c["pre"][l - 1])
    return loss, g


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------------------
# Fourier features
# --------------------------------------------------------------------------------------
def fourier_coefficients(theta, omega, curve_ptr, mu, n_modes):
    """[d][F] with F = 2 n_modes n_curves, ordered [curve][k][Re, Im]."""
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    nc = len(curve_ptr) - 1
    k = np.arange(n_modes)
    out = np.zeros((mu.shape[0], nc, n_modes, 2))
    for c in range(nc):
        a, b = curve_ptr[c], curve_ptr[c + 1]
        E = np.exp(-1j * np.outer(theta[a:b], k)) * omega[a:b, None] / (2.0 * math.pi)
        ck = mu[:, a:b] @ E
        out[:, c, :, 0] = ck.real
        out[:, c, :, 1] = ck.imag
    return out.reshape(mu.shape[0], -1)


def fourier_synthesis(theta, curve_ptr, coef, n_modes):
    """Real Fourier series Re(c_0) + sum_{k>=1} 2 Re(c_k e^{i k theta}) on each curve."""
    coef = np.atleast_2d(np.asarray(coef, dtype=np.float64))
    nc = len(curve_ptr) - 1
    C = coef.reshape(coef.shape[0], nc, n_modes, 2)
    out = np.zeros((coef.shape[0], int(curve_ptr[-1])))
    k = np.arange(n_modes)
    wk = np.where(k == 0, 1.0, 2.0)
    for c in range(nc):
        a, b = curve_ptr[c], curve_ptr[c + 1]
        E = np.exp(1j * np.outer(theta[a:b], k))
        ck = C[:, c, :, 0] + 1j * C[:, c, :, 1]
        out[:, a:b] = np.real((ck * wk) @ E.T)
    return out


def extrapolation_coeffs(p):
    """b_i, i = 0..p, of the degree-p polynomial through the last p+1 equally
    spaced values, evaluated one step ahead: next = sum_i b_i x_{s-i}."""
    return np.array([(-1) ** i * math.comb(p + 1, i + 1) for i in range(p + 1)], dtype=np.float64)


def as_complex(coef):
    """Rows of real coefficients [..][F] ordered (Re, Im) as complex rows [..][F/2]."""
    c = np.asarray(coef, dtype=np.float64)
    return c[..., 0::2] + 1j * c[..., 1::2]


def as_real(z):
    z = np.asarray(z)
    out = np.empty(z.shape[:-1] + (2 * z.shape[-1],))
    out[..., 0::2] = z.real
    out[..., 1::2] = z.imag
    return out


REC_LAMBDA = 1e-14


def recurrence_fit(coef, n_hist):
    """Per complex coefficient k, the order-n_hist linear recurrence
    c_k(s) = sum_i a_i c_k(s-1-i) that minimises, over the windows j of the
    series, sum_j |c_k(j+H) - sum_i a_i c_k(j+H-1-i)|^2 + lam |a|^2 with
    lam = 1e-14 tr(G)/H (plus the smallest normal number), G = sum_j conj(h_j) h_j^T:
    the solution of the regularised normal equations.  Returns a [F/2][H] complex."""
    z = as_complex(coef)
    S = z.shape[0] - n_hist
    out = np.zeros((z.shape[1], n_hist), dtype=complex)
    for k in range(z.shape[1]):
        Hm = np.array([[z[j + n_hist - 1 - i, k] for i in range(n_hist)] for j in range(S)])
        y = z[n_hist:n_hist + S, k]
        G = Hm.conj().T @ Hm
        lam = REC_LAMBDA * np.trace(G).real / n_hist + np.finfo(float).tiny
        out[k] = np.linalg.solve(G + lam * np.eye(n_hist), Hm.conj().T @ y)
    return out


def recurrence_predict(window, rec):
    """Next coefficients [F] (real layout) of a window [H][F] (newest last)."""
    z = as_complex(window)
    H = z.shape[0]
    return as_real(sum(rec[:, i] * z[H - 1 - i] for i in range(H)))


def warm_features(coef, n_hist, order, rec=None):
    """Network input groups [S][n_hist][F] (backward differences 0..n_hist-1 of
    the newest row of each window) and targets [S][F] (next row minus the base
    prediction: the order-p extrapolation of the window, or the recurrence rec
    when given)."""
    coef = np.asarray(coef, dtype=np.float64)
    S = coef.shape[0] - n_hist
    grp = np.zeros((S, n_hist, coef.shape[1]))
    for j in range(S):
        cur = coef[j:j + n_hist].copy()
        grp[j, 0] = cur[-1]
        for h in range(1, n_hist):  # repeated first differences of the window
            cur = cur[1:] - cur[:-1]
            grp[j, h] = cur[-1]
    if rec is not None:
        tgt = np.stack([coef[j + n_hist] - recurrence_predict(coef[j:j + n_hist], rec) for j in range(S)])
    else:
        b = extrapolation_coeffs(order)
        tgt = np.stack([coef[j + n_hist] - sum(b[i] * coef[j + n_hist - 1 - i] for i in range(order + 1))
                        for j in range(S)])
    return grp, tgt


def warm_scales(coef, n_hist, order, rec=None):
    """(1 / RMS of each input group over the samples, RMS of the targets)."""
    grp, tgt = warm_features(coef, n_hist, order, rec)
    gx = [math.sqrt(np.mean(grp[:, h] ** 2)) for h in range(n_hist)]
    ry = math.sqrt(np.mean(tgt ** 2))
    return [1.0 / r if r > 0 else 1.0 for r in gx], (ry if ry > 0 else 1.0)


def warm_samples(coef, n_hist, order, scales, rec=None):
    """Network inputs [S][n_hist F] and targets [S][F] of a training series."""
    grp, tgt = warm_features(coef, n_hist, order, rec)
    X = (grp * np.asarray(scales[0])[None, :, None]).reshape(grp.shape[0], -1)
    return X, tgt / scales[1]


def warm_input(hist_coef, scales):
    """Network input of one window of coefficients [n_hist][F] (newest last)."""
    h = np.asarray(hist_coef, dtype=np.float64)
    grp, _ = warm_features(np.vstack([h, h[-1:]]), h.shape[0], 0)
    return (grp * np.asarray(scales[0])[None, :, None]).reshape(1, -1)

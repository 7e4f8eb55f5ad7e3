"""Pins of the warm-start oracle (Fourier features, network, Adam).

Expected values come from the BF16 format's definition, the exact GELU
(z Phi(z) via erf), PyTorch's CPU autograd in float64, central finite
differences, the Adam paper's update written with torch.optim, and band-limited
densities whose Fourier coefficients are known by construction.
"""
import math

import numpy as np
import scipy.special as sp
import torch

from oracle import warm_oracle as wo
from paper_1908_07392_amd import workloads as wl


def test_bf16_round_definition():
    ulp = 2.0 ** -7  # BF16 spacing on [1, 2)
    cases = {
        1.0: 1.0,
        1.0 + ulp / 2: 1.0,                          # tie -> even (1.0)
        1.0 + 1.5 * ulp: 1.0 + 2 * ulp,              # tie -> even (1 + 2 ulp)
        1.0 + ulp / 2 + 2.0 ** -20: 1.0 + ulp,       # just above the tie -> up
        1.0 + ulp / 2 - 2.0 ** -20: 1.0,             # just below the tie -> down
        -3.0: -3.0,
        -(1.0 + 1.5 * ulp): -(1.0 + 2 * ulp),
        2.0 ** -130: 2.0 ** -130,                    # subnormal with few bits
        0.0: 0.0,
    }
    got = wo.bf16_round(np.array(list(cases.keys()), dtype=np.float32))
    assert np.array_equal(got, np.array(list(cases.values())))
    x = np.random.default_rng(0).standard_normal(10000).astype(np.float32)
    r = wo.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * (1 + 1e-12))
    assert np.all(r.astype(np.float32).view(np.uint32) & 0xFFFF == 0)


def test_gelu_tanh_form_vs_exact_gelu():
    z = np.linspace(-6, 6, 2001)
    exact = 0.5 * z * (1.0 + sp.erf(z / math.sqrt(2.0)))
    assert np.max(np.abs(wo.gelu(z) - exact)) < 5e-4
    assert wo.gelu(np.array([0.0]))[0] == 0.0
    assert abs(wo.gelu_prime(np.array([0.0]))[0] - 0.5) < 1e-15
    h = 1e-5
    fd = (wo.gelu(z + h) - wo.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - wo.gelu_prime(z))) < 1e-9


def _tiny(seed=0, sizes=(7, 5, 5, 3), B=4):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(wo.n_params(sizes)) * 0.7
    X = rng.standard_normal((B, sizes[0]))
    T = rng.standard_normal((B, sizes[3]))
    return p, X, T, sizes


def test_mlp_gradient_central_differences():
    p, X, T, sizes = _tiny()
    loss, g = wo.mlp_loss_grad(p, sizes, X, T, round_weights=False)
    h = 1e-6
    fd = np.empty_like(g)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (wo.mlp_loss_grad(p + e, sizes, X, T, False)[0] - wo.mlp_loss_grad(p - e, sizes, X, T, False)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) < 1e-8 * max(1.0, np.max(np.abs(g)))


def test_mlp_forward_and_grad_vs_torch_autograd():
    p, X, T, sizes = _tiny(seed=3, sizes=(11, 9, 9, 6), B=5)
    for rnd in (False, True):
        loss, g = wo.mlp_loss_grad(p, sizes, X, T, round_weights=rnd)
        Ws, bs = [], []
        for l, (sw, sb) in enumerate(wo.layer_slices(sizes)):
            w = p[sw].reshape(sizes[l + 1], sizes[l])
            if rnd:  # BF16 rounding of the weights by torch's own conversion
                w = torch.tensor(w, dtype=torch.float32).to(torch.bfloat16).double().numpy()
            Ws.append(torch.tensor(w, dtype=torch.float64, requires_grad=True))
            bs.append(torch.tensor(p[sb], dtype=torch.float64, requires_grad=True))
        a = torch.tensor(X)
        for l in range(3):
            a = torch.nn.functional.linear(a, Ws[l], bs[l])
            if l < 2:
                a = torch.nn.functional.gelu(a, approximate="tanh")
        Y = wo.mlp_forward(p, sizes, X, rnd)[0]
        assert np.max(np.abs(a.detach().numpy() - Y)) < 1e-13
        L = torch.nn.functional.mse_loss(a, torch.tensor(T))
        L.backward()
        assert abs(L.item() - loss) < 1e-14
        gt = np.concatenate([np.concatenate([Ws[l].grad.numpy().ravel(), bs[l].grad.numpy()]) for l in range(3)])
        assert np.max(np.abs(gt - g)) < 1e-13


def test_adam_vs_torch_optim():
    rng = np.random.default_rng(5)
    p = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        p, m, v = wo.adam_step(p, g, m, v, step)
        tp.grad = torch.tensor(g)
        opt.step()
    assert np.max(np.abs(tp.detach().numpy() - p)) < 1e-14


def test_fourier_band_limited_exact():
    geom, _ = wl.config5_geometry()
    ptr = geom.curve_node_ptr
    K = 128
    rng = np.random.default_rng(11)
    nc = len(ptr) - 1
    C = np.zeros((nc, K), dtype=complex)
    C[:, :40] = rng.standard_normal((nc, 40)) + 1j * rng.standard_normal((nc, 40))
    C[:, 0] = C[:, 0].real
    mu = np.zeros(geom.n_nodes)
    for c in range(nc):
        a, b = ptr[c], ptr[c + 1]
        th = geom.theta[a:b]
        mu[a:b] = C[c, 0].real + 2.0 * np.real(np.exp(1j * np.outer(th, np.arange(1, K))) @ C[c, 1:])
    coef = wo.fourier_coefficients(geom.theta, geom.theta_w, ptr, mu, K)[0].reshape(nc, K, 2)
    assert np.max(np.abs(coef[..., 0] - C.real)) < 1e-13
    assert np.max(np.abs(coef[..., 1] - C.imag)) < 1e-13
    back = wo.fourier_synthesis(geom.theta, ptr, coef.ravel(), K)[0]
    assert np.max(np.abs(back - mu)) < 1e-11 * np.max(np.abs(mu))


def test_extrapolation_exact_on_polynomials():
    # a degree-p polynomial sampled at s-p..s is continued exactly to s+1
    for p in range(4):
        b = wo.extrapolation_coeffs(p)
        assert abs(b.sum() - 1.0) < 1e-15
        for deg in range(p + 1):
            for s0 in (0.0, 3.0, -7.5):
                xs = [(s0 - i) ** deg for i in range(p + 1)]
                assert abs(sum(bi * x for bi, x in zip(b, xs)) - (s0 + 1) ** deg) < 1e-9 * max(1.0, abs(s0 + 1) ** deg)
    # and not beyond: the error on t^(p+1) is (p+1)! (one step of size 1)
    for p in range(4):
        b = wo.extrapolation_coeffs(p)
        err = (1.0) ** (p + 1) - sum(b[i] * (-float(i)) ** (p + 1) for i in range(p + 1))
        assert abs(err - math.factorial(p + 1)) < 1e-9


def test_warm_features_backward_differences_and_targets():
    # rows x_r = r^k (every feature): the h-th backward difference of r^h is h!,
    # and vanishes for h > k
    rows = np.arange(10, dtype=np.float64)
    for k in range(4):
        coef = np.repeat((rows ** k)[:, None], 3, axis=1)
        grp, tgt = wo.warm_features(coef, 4, 3)
        assert grp.shape == (6, 4, 3) and tgt.shape == (6, 3)
        assert np.allclose(grp[:, k], math.factorial(k))
        for h in range(k + 1, 4):
            assert np.allclose(grp[:, h], 0.0)
        assert np.allclose(tgt, 0.0)  # cubic extrapolation is exact for k <= 3
        assert np.allclose(grp[:, 0], coef[3:9])
    coef = np.repeat((rows ** 2)[:, None], 2, axis=1)
    _, tgt = wo.warm_features(coef, 3, 1)
    assert np.allclose(tgt, 2.0)  # linear extrapolation misses r^2 by 2


def test_warm_samples_shapes_and_scales():
    rng = np.random.default_rng(2)
    coef = rng.standard_normal((10, 6))
    sx, sy = wo.warm_scales(coef, 4, 2)
    X, T = wo.warm_samples(coef, 4, 2, (sx, sy))
    assert X.shape == (6, 24) and T.shape == (6, 6)
    for h in range(4):
        assert abs(np.sqrt(np.mean(X.reshape(6, 4, 6)[:, h] ** 2)) - 1.0) < 1e-12
    assert np.allclose(X.reshape(6, 4, 6)[2, 0], coef[5] * sx[0])
    assert np.allclose(X.reshape(6, 4, 6)[2, 1], (coef[5] - coef[4]) * sx[1])
    assert np.allclose(T[5] * sy, coef[9] - (3 * coef[8] - 3 * coef[7] + coef[6]))
    assert abs(np.sqrt(np.mean(T ** 2)) - 1.0) < 1e-12
    Xi = wo.warm_input(coef[2:6], (sx, sy))
    assert np.allclose(Xi, X[2:3])


def test_recurrence_exact_on_sums_of_rotations():
    """A coefficient series that is a sum of H rotations b_m e^{i w_m s} obeys a
    linear recurrence of order H (its characteristic roots are e^{i w_m}); the
    least-squares fit recovers it and predicts the next value to rounding, for
    each coefficient separately.  Fewer terms than H are also exact."""
    rng = np.random.default_rng(5)
    H, S = 4, 40
    s = np.arange(S + H + 1)
    cols = []
    for n_terms in (1, 2, 3, 4):
        w = rng.uniform(-1.5, 1.5, n_terms) + np.arange(n_terms) * 0.7  # distinct frequencies
        b = rng.standard_normal(n_terms) + 1j * rng.standard_normal(n_terms)
        cols.append((b[None, :] * np.exp(1j * np.outer(s, w))).sum(axis=1))
    Z = np.stack(cols, axis=1)                       # [steps][4 coefficients]
    coef = wo.as_real(Z)
    rec = wo.recurrence_fit(coef[:-1], H)             # fitted on all but the last row
    pred = wo.recurrence_predict(coef[-1 - H:-1], rec)
    assert np.max(np.abs(pred - coef[-1])) < 1e-9 * np.max(np.abs(coef))
    # the exact recurrence of one rotation: a_0 = e^{i w}
    z1 = 0.7 * np.exp(1j * 0.37 * s)
    r1 = wo.recurrence_fit(wo.as_real(z1[:, None]), 1)
    assert abs(r1[0, 0] - np.exp(1j * 0.37)) < 1e-12


def test_recurrence_normal_equations_vs_lstsq():
    """On noisy data the regularised normal equations give the least-squares
    solution of numpy's lstsq (the Tikhonov term is 1e-14 of the trace)."""
    rng = np.random.default_rng(6)
    H = 3
    coef = rng.standard_normal((30, 6))
    rec = wo.recurrence_fit(coef, H)
    Z = wo.as_complex(coef)
    for k in range(Z.shape[1]):
        Hm = np.array([[Z[j + H - 1 - i, k] for i in range(H)] for j in range(Z.shape[0] - H)])
        a = np.linalg.lstsq(Hm, Z[H:, k], rcond=None)[0]
        assert np.max(np.abs(a - rec[k])) < 1e-10 * np.max(np.abs(a))

"""Plain FP64 CPU oracle of the particular solution of the modified Stokes
equations on a periodic box (Sec. 2.1, "Particular solution"; Sec. 3.1.2,
"Evaluating the volume potential").

TEST INFRASTRUCTURE ONLY: imported by the test suite; the HIP library never
imports, links or calls it, and the two share no code.

Box B = [x0, x0 + Lb) x [y0, y0 + Lb) with the uniform periodic grid
x_a = x0 + a Lb/M, y_b = y0 + b Lb/M (a, b = 0..M-1; arrays indexed [b][a], i.e.
row = y).  A field on the grid has the Fourier coefficients
    F^(k) = (1/M^2) sum_{a,b} F(x_a, y_b) e^{-i k.(x - x0)},
k = (2 pi/Lb)(k1, k2), k1, k2 in [-M/2, M/2); the Nyquist coefficients
(k1 = -M/2 or k2 = -M/2) are set to zero in every result (odd derivatives have
no real Nyquist term, and a smooth F has none to speak of).

Particular solution (the periodic stokeslet multiplier):
    u^_j(k) = S^_jl(k) F^_l(k),  S^_jl = (delta_jl - k_j k_l/|k|^2)/(alpha^2 + |k|^2)  (k != 0),
    S^_jl(0) = delta_jl/alpha^2,
its gradient d u_j/d x_m = sum_k i k_m u^_j(k) e^{i k.(x - x0)}, and values at
arbitrary points by the type-2 sum u_j(x) = sum_k u^_j(k) e^{i k.(x - x0)} (the sum
a type-2 non-uniform FFT approximates), written out directly.

numpy's FFT is the library primitive for the grid transforms.
"""
from __future__ import annotations

import numpy as np


def wavenumbers(M, Lb):
    """(k1, k2) grids [M][M] (row = k2) in numpy FFT order, and the Nyquist mask."""
    j = np.fft.fftfreq(M, d=1.0 / M)  # 0..M/2-1, -M/2..-1
    k = 2.0 * np.pi / Lb * j
    K1, K2 = np.meshgrid(k, k, indexing="xy")
    nyq = np.zeros((M, M), dtype=bool)
    if M % 2 == 0:
        nyq[:, M // 2] = True
        nyq[M // 2, :] = True
    return K1, K2, nyq


def coefficients(F):
    """F^(k) of a grid field [M][M] (normalised by M^2)."""
    M = F.shape[0]
    return np.fft.fft2(F) / (M * M)


def particular(F1, F2, alpha, Lb):
    """u^ = S^ F^ of the forcing components (grids [M][M]); returns (u1^, u2^) with Nyquist zeroed."""
    M = F1.shape[0]
    K1, K2, nyq = wavenumbers(M, Lb)
    f1, f2 = coefficients(F1), coefficients(F2)
    k2 = K1 * K1 + K2 * K2
    den = alpha * alpha + k2
    with np.errstate(divide="ignore", invalid="ignore"):
        p11 = np.where(k2 > 0, 1.0 - K1 * K1 / k2, 1.0)
        p22 = np.where(k2 > 0, 1.0 - K2 * K2 / k2, 1.0)
        p12 = np.where(k2 > 0, -K1 * K2 / k2, 0.0)
    u1 = (p11 * f1 + p12 * f2) / den
    u2 = (p12 * f1 + p22 * f2) / den
    u1[nyq] = 0.0
    u2[nyq] = 0.0
    return u1, u2


def grid_values(uh):
    """Field on the grid from its coefficients."""
    M = uh.shape[0]
    return np.real(np.fft.ifft2(uh) * (M * M))


def grid_gradient(uh, Lb):
    """(d/dx, d/dy) of the field on the grid (Fourier differentiation)."""
    M = uh.shape[0]
    K1, K2, nyq = wavenumbers(M, Lb)
    dx = 1j * K1 * uh
    dy = 1j * K2 * uh
    dx[nyq] = 0.0
    dy[nyq] = 0.0
    return grid_values(dx), grid_values(dy)


def point_values(uh, Lb, x0, y0, px, py):
    """Type-2 sum of the coefficients at the points (written out directly)."""
    M = uh.shape[0]
    K1, K2, _ = wavenumbers(M, Lb)
    k1 = K1[0, :]
    k2 = K2[:, 0]
    out = np.empty(np.size(px))
    for i, (x, y) in enumerate(zip(np.ravel(px), np.ravel(py))):
        ex = np.exp(1j * k1 * (x - x0))
        ey = np.exp(1j * k2 * (y - y0))
        out[i] = np.real(ey @ uh @ ex)
    return out

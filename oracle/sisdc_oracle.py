"""Plain FP64 CPU oracle of the semi-implicit spectral deferred correction
(SISDC) time step of the Navier-Stokes equations (Sec. 3.3, "Time stepping"),
on a periodic box where every term lives on the grid (no embedded boundary,
so no function extension is needed).

TEST INFRASTRUCTURE ONLY: imported by the test suite; the HIP library never
imports, links or calls it, and the two share no code.

Equations: u_t = G_E(u) + G_I(u), G_E = -(u.grad)u, G_I = (1/Re) Delta u - grad p,
div u = 0, on [x0, x0 + Lb)^2 with an M x M grid (fields [2][M][M], row = y).
A step of length dt has p = K - 1 equal substeps dts = dt/p and K - 1 correction
sweeps (global order K).  Each implicit substep solves the modified Stokes
system (alpha^2 - Delta) u + Re grad p = F, alpha^2 = Re/dts, with the periodic
stokeslet multiplier (particular_oracle); from the solved equation,
L = Delta u - Re grad p = alpha^2 u - F.  With N = (u.grad)u:
  first sweep:        F_{m+1} = alpha^2 u_m - Re N_m
  correction k -> k+1: F_{m+1} = alpha^2 u'_m - Re (N'_m - N_m) - L_{m+1}
                                + (1/dts) sum_j q_j^m (L_j - Re N_j),
where primes are the new sweep, unprimed the previous one, and q_j^m integrate
the Lagrange basis of the equispaced substep times over [t_m, t_{m+1}].
At the start of a step the caller supplies L_0 (Delta u_0 suffices: gradient
terms of F do not change u).
"""
from __future__ import annotations

import numpy as np

from oracle import particular_oracle as P


def quadrature_weights(p):
    """q[m][j] = (1/dts) int_{t_m}^{t_{m+1}} l_j(t) dt on the nodes t_j = j dts, j = 0..p."""
    nodes = np.arange(p + 1, dtype=np.float64)
    q = np.zeros((p, p + 1))
    for j in range(p + 1):
        others = np.delete(nodes, j)
        coef = np.poly(others) / np.prod(nodes[j] - others)  # l_j as a polynomial
        integ = np.polyint(coef)
        for m in range(p):
            q[m, j] = np.polyval(integ, m + 1.0) - np.polyval(integ, float(m))
    return q


def solve(F, alpha, Lb):
    """u and grad u (4 fields: du1/dx, du1/dy, du2/dx, du2/dy) of (alpha^2 - Delta) u + grad p = F."""
    u1h, u2h = P.particular(F[0], F[1], alpha, Lb)
    u = np.stack([P.grid_values(u1h), P.grid_values(u2h)])
    g = np.stack([*P.grid_gradient(u1h, Lb), *P.grid_gradient(u2h, Lb)])
    return u, g


def advection(u, g):
    """(u.grad) u from u and its gradient."""
    return np.stack([u[0] * g[0] + u[1] * g[1], u[0] * g[2] + u[1] * g[3]])


def step(u0, g0, L0, Re, dt, K, Lb):
    """One SISDC step; returns (u, grad u, L) at the end of the step."""
    p = K - 1
    dts = dt / p
    a2 = Re / dts
    alpha = np.sqrt(a2)
    q = quadrature_weights(p)
    # first sweep
    U, Gr, L, N = [u0], [g0], [L0], [advection(u0, g0)]
    for m in range(p):
        F = a2 * U[m] - Re * N[m]
        u, g = solve(F, alpha, Lb)
        U.append(u)
        Gr.append(g)
        N.append(advection(u, g))
        L.append(a2 * u - F)
    # corrections
    for _ in range(K - 1):
        U2, G2, L2, N2 = [u0], [g0], [L0], [N[0]]
        for m in range(p):
            quad = sum(q[m, j] * (L[j] - Re * N[j]) for j in range(p + 1))
            F = a2 * U2[m] - Re * (N2[m] - N[m]) - L[m + 1] + quad
            u, g = solve(F, alpha, Lb)
            U2.append(u)
            G2.append(g)
            N2.append(advection(u, g))
            L2.append(a2 * u - F)
        U, Gr, L, N = U2, G2, L2, N2
    return U[p], Gr[p], L[p]

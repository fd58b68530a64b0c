"""Exact collocation solution on sine-mode data -- TEST INFRASTRUCTURE ONLY.

On initial data that is a sum of discrete sine modes phi_k, every mode is
an eigenvector of the discrete Laplacian (L_h phi_k = lambda_k phi_k) and
the forcing of eq. (3) only excites mode (1,1,1).  The collocation problem
of eq. (6) then splits into one M x M linear system per mode and step:
    (I - dt nu lambda_k Q) a = a_0 1 + dt Q g,   g_j = forcing factor at t_j
(g = 0 except for mode (1,1,1)).  Converged SDC sweeps reach this solution
(section 1.1), so it serves as the reference at any grid size.  lambda_k is
read off the oracle's own Laplacian applied to phi_k on the same grid.
"""
from __future__ import annotations

import math

import numpy as np

import oracle


def mode(n, k):
    x = np.arange(1, n + 1, dtype=np.float64) / (n + 1)
    s = [np.sin(kk * np.pi * x) for kk in k]
    return s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :]


def eigenvalue(n, order, k):
    phi = mode(n, k)
    L = oracle.laplacian(phi, order)
    idx = np.unravel_index(np.argmax(np.abs(phi)), phi.shape)
    return float(L[idx] / phi[idx])


def coefficients(n, order, M, nu, t0, dt, nsteps, modes, forcing_c=3.0):
    """Amplitude of every mode after nsteps collocation steps from t0.
    modes: list of (kx, ky, kz, amplitude); duplicates add up."""
    Q = oracle.collocation_matrix(M)
    tau = oracle.lobatto_nodes(M)
    amp = {}
    for kx, ky, kz, a in modes:
        amp[(kx, ky, kz)] = amp.get((kx, ky, kz), 0.0) + a
    amp.setdefault((1, 1, 1), 0.0)
    out = {}
    for k, a in amp.items():
        mu = nu * eigenvalue(n, order, k)
        A = np.eye(M) - dt * mu * Q
        for s in range(nsteps):
            t = t0 + s * dt + dt * tau
            g = (-(np.sin(t) - forcing_c * nu * math.pi ** 2 * np.cos(t)) if k == (1, 1, 1)
                 else np.zeros(M))
            a = np.linalg.solve(A, a * np.ones(M) + dt * Q @ g)[-1]
        out[k] = a
    return out


def field(n, coeffs):
    u = np.zeros((n, n, n))
    for k, a in coeffs.items():
        u += a * mode(n, k)
    return u

"""SO(3) sampling and quadrature weights for the oracle (test infrastructure only).

Grid (Section II-D, definition of E_L): alpha_a = 2 pi a / n_phi,
beta_b = 2 pi b / n_phi for b = 0..(n_phi-1)/2, gamma_c = 2 pi c / n_omega.
With n_phi = 2L+1 this is exactly E_L; the workloads use per-axis sizes, and
the forward transform is pointwise so any sizes are valid.

Beta weights of the discrete inverse (Section IV-A,
eq. Eq:sig_reconstruction_discrete and the definitions of q(beta) and w(m)
after it), for L = (n_phi - 1)/2:
    q(0)     = 4 pi^2 (floor(L/2) + 1/2)^{-1}
    q(beta)  = 8 pi^2 sum_{m=-L}^{L} w(-m) cos(m beta),   beta != 0
    w(+-1)   = +-i pi/2,  w(m) = 0 for other odd m,  w(m) = 2/(1-m^2) for even m.
"""
from __future__ import annotations

import numpy as np


def alpha_angles(n_phi: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n_phi) / n_phi


def beta_angles(n_phi: int, n_theta: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n_theta) / n_phi


def gamma_angles(n_omega: int) -> np.ndarray:
    return 2.0 * np.pi * np.arange(n_omega) / n_omega


def rho_angles(n_phi: int, n_theta: int, n_omega: int, idx: np.ndarray):
    """(alpha, beta, gamma) arrays for integer grid indices idx[k] = (a, b, c)."""
    idx = np.asarray(idx, dtype=np.int64)
    a, b, c = idx[:, 0], idx[:, 1], idx[:, 2]
    return (2.0 * np.pi * a / n_phi, 2.0 * np.pi * b / n_phi,
            2.0 * np.pi * c / n_omega)


def w_weight(m: int) -> complex:
    if m == 1:
        return 1j * np.pi / 2.0
    if m == -1:
        return -1j * np.pi / 2.0
    if m % 2:
        return 0.0
    return 2.0 / (1.0 - m * m)


def beta_weights(n_phi: int, n_theta: int) -> np.ndarray:
    """q(beta_b) for b < n_theta, as printed in the paper with L = (n_phi-1)/2."""
    L = (n_phi - 1) // 2
    betas = beta_angles(n_phi, n_theta)
    q = np.zeros(n_theta, dtype=np.float64)
    for b, beta in enumerate(betas):
        if b == 0:
            q[b] = 4.0 * np.pi ** 2 / (np.floor(L / 2.0) + 0.5)
        else:
            s = 0.0 + 0.0j
            for m in range(-L, L + 1):
                s += w_weight(-m) * np.cos(m * beta)
            q[b] = (8.0 * np.pi ** 2 * s).real
    return q

"""Spherical harmonics for the oracle (test infrastructure only).

Y_l^m(theta, phi) = N_l^m P_l^m(cos theta) e^{i m phi}, with
N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and the associated Legendre
function P_l^m carrying the Condon-Shortley phase (-1)^m
(Section II-A, eq. Eq:Sph_harmonics).  Negative orders follow from
Y_l^{-m} = (-1)^m conj(Y_l^m).

The normalised function lam_l^m(theta) = N_l^m P_l^m(cos theta) is produced by
the textbook three-term recursion in l at fixed m, started from the sectoral
value lam_m^m = (-1)^m sqrt((2m+1)!! / (4 pi (2m)!!)) sin^m theta.
"""
from __future__ import annotations

import numpy as np


def legendre_table(lmax: int, theta: np.ndarray) -> np.ndarray:
    """lam[l, m, t] = N_l^m P_l^m(cos theta_t) for 0 <= m <= l <= lmax (zero for m > l)."""
    theta = np.asarray(theta, dtype=np.float64)
    x = np.cos(theta)
    s = np.sin(theta)
    nt = theta.shape[0]
    lam = np.zeros((lmax + 1, lmax + 1, nt), dtype=np.float64)
    lam[0, 0] = 1.0 / np.sqrt(4.0 * np.pi)
    for m in range(1, lmax + 1):
        lam[m, m] = -np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * lam[m - 1, m - 1]
    for m in range(0, lmax):
        lam[m + 1, m] = np.sqrt(2.0 * m + 3.0) * x * lam[m, m]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            lam[l, m] = a * (x * lam[l - 1, m] - b * lam[l - 2, m])
    return lam


def lam_signed(lam: np.ndarray, l: int, m: int) -> np.ndarray:
    """lam_l^m for any sign of m, using lam_l^{-m} = (-1)^m lam_l^m."""
    if m >= 0:
        return lam[l, m]
    return ((-1.0) ** m) * lam[l, -m]


def sph_harm(l: int, m: int, theta, phi) -> np.ndarray:
    """Y_l^m at points (theta, phi) (arrays of equal shape)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    lam = legendre_table(l, theta.ravel())
    v = lam_signed(lam, l, m).reshape(theta.shape)
    return v * np.exp(1j * m * phi)


def synthesize(coeffs: np.ndarray, L: int, theta, phi) -> np.ndarray:
    """sum_{l<L, |m|<=l} c_l^m Y_l^m(theta_k, phi_k) at scattered points."""
    theta = np.asarray(theta, dtype=np.float64).ravel()
    phi = np.asarray(phi, dtype=np.float64).ravel()
    lam = legendre_table(max(L - 1, 0), theta)
    out = np.zeros(theta.shape[0], dtype=np.complex128)
    for l in range(L):
        for m in range(-l, l + 1):
            out += coeffs[l * l + l + m] * lam_signed(lam, l, m) * np.exp(1j * m * phi)
    return out

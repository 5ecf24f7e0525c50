"""Wigner-d and Wigner-D functions for the oracle (test infrastructure only).

Convention (Section II-B): D^l_{m,m'}(alpha, beta, gamma)
= e^{-i m alpha} d^l_{m,m'}(beta) e^{-i m' gamma}  (eq. Eq:Dlm), with the
rotation acting on coefficients as (D_rho f)_l^m = sum_{m'} D^l_{m,m'}(rho) f_l^{m'}
(eq. eqn:rotation_non_symm); the zyz rotation is gamma about z, then beta
about y, then alpha about z.

The value Delta^l_{m,m'} = d^l_{m,m'}(pi/2) is taken from Wigner's explicit
sum in exact integer arithmetic.  With cos(pi/4) = sin(pi/4) = 2^{-1/2}, every
term of the sum carries the same power 2^{-l}, and
    (l+m')!(l-m')! / ((l+m'-k)! k! (l-k-m)! (k-m'+m)!)
        = C(l+m', k) C(l-m', k-m'+m),
so that
    Delta^l_{m,m'} = 2^{-l} sqrt((l+m)!(l-m)! / ((l+m')!(l-m')!))
                     * sum_k (-1)^{k-m'+m} C(l+m', k) C(l-m', k-m'+m),
an integer sum times the square root of an exact rational number; both are
evaluated exactly and rounded once.

d^l(beta) for any beta then follows from the factoring of rotations
(Section IV-B, eq. Eq:WignerD_expansion_new with alpha = gamma = 0):
    d^l_{m,m'}(beta) = i^{m-m'} sum_{m''} Delta^l_{m'',m} Delta^l_{m'',m'} e^{-i m'' beta},
which only combines bounded terms and so stays accurate at every degree.
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np


def _sqrt_fraction(num: int, den: int) -> float:
    """Correctly scaled sqrt(num/den) for non-negative integers, to ~1 ulp."""
    if num == 0:
        return 0.0
    k = max(0, (den.bit_length() - num.bit_length() + 140) // 2 + 1)
    r = math.isqrt((num << (2 * k)) // den)
    return float(Fraction(r, 1 << k))


@functools.lru_cache(maxsize=None)
def delta_matrix(l: int) -> np.ndarray:
    """Delta[m+l, m'+l] = d^l_{m,m'}(pi/2), exact to rounding."""
    n = 2 * l + 1
    out = np.zeros((n, n), dtype=np.float64)
    fact = [math.factorial(i) for i in range(2 * l + 2)]
    for m in range(-l, l + 1):          # row index
        for mp in range(-l, l + 1):     # column index
            # Wigner's sum for d^l_{m,mp}: row m, column mp.
            s = 0
            for k in range(max(0, mp - m), min(l + mp, l - m) + 1):
                term = math.comb(l + mp, k) * math.comb(l - mp, k - mp + m)
                s += -term if (k - mp + m) % 2 else term
            if s == 0:
                continue
            num = s * s * fact[l + m] * fact[l - m]
            den = fact[l + mp] * fact[l - mp] * (4 ** l)
            v = _sqrt_fraction(num, den)
            out[m + l, mp + l] = v if s > 0 else -v
    return out


def wigner_d(l: int, beta: float) -> np.ndarray:
    """d[m+l, m'+l] = d^l_{m,m'}(beta) via the Delta-Fourier identity."""
    dl = delta_matrix(l)
    mm = np.arange(-l, l + 1)
    ph = np.exp(-1j * mm * beta)                       # e^{-i m'' beta}
    core = dl.T @ (ph[:, None] * dl)                   # sum_{m''} D[m'',m] D[m'',m'] e^{..}
    phase = (1j) ** ((mm[:, None] - mm[None, :]) % 4)  # i^{m-m'}
    return np.real(phase * core)


def wigner_d_all(L: int, beta: float) -> list[np.ndarray]:
    """[d^0(beta), ..., d^{L-1}(beta)]."""
    return [wigner_d(l, beta) for l in range(L)]


def wigner_D(l: int, alpha: float, beta: float, gamma: float) -> np.ndarray:
    """D[m+l, m'+l] = e^{-i m alpha} d^l_{m,m'}(beta) e^{-i m' gamma}."""
    mm = np.arange(-l, l + 1)
    return (np.exp(-1j * mm * alpha)[:, None] * wigner_d(l, beta)
            * np.exp(-1j * mm * gamma)[None, :])


def rotate_coefficients(h: np.ndarray, L: int, alpha: float, beta: float,
                        gamma: float) -> np.ndarray:
    """(D_rho h)_l^m = sum_{m'} D^l_{m,m'}(rho) h_l^{m'} for l < L."""
    out = np.zeros(L * L, dtype=np.complex128)
    for l in range(L):
        sl = slice(l * l, l * l + 2 * l + 1)
        out[sl] = wigner_D(l, alpha, beta, gamma) @ h[sl]
    return out

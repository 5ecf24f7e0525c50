"""Functions on SO(3) through their Wigner-D expansion (test infrastructure only).

A band-limited function on the rotation group is a finite sum of Wigner-D functions
(Section II-C, the SO(3) expansion, with the orthogonality relation Eq:WignerD_ortho):
    g(rho) = sum_{p < L} sum_{|q|,|q'| <= p} G^p_{q,q'} D^p_{q,q'}(rho),
    G^p_{q,q'} = (2p + 1) / (8 pi^2) int_{SO(3)} g(rho) conj(D^p_{q,q'}(rho)) drho,
with D^p_{q,q'}(alpha, beta, gamma) = e^{-i q alpha} d^p_{q,q'}(beta) e^{-i q' gamma}
(eq. Eq:Dlm).  The forward transform is such a function of rho for every (l, m): by the
harmonic formulation (Eq:harmonic_formulation) its coefficients are
G^p_{q,q'}(l, m) = A^p_q(l, m) h_p^{q'}.

`so3_synthesis` evaluates the sum on the paper's grid; `so3_analysis` evaluates the
integral with the discrete rule of the inverse (Section IV-A, the weights q(beta) of
Eq:sig_reconstruction_discrete):
    int F drho ~ 1 / (n_phi^2 n_omega) sum_{a, b, c} q(beta_b) F(alpha_a, beta_b, gamma_c),
which is exact for the products D^l conj(D^p) with l + p <= (n_phi - 1)/2,
|q - q_2| < n_phi and |q' - q'_2| < n_omega.

Coefficient layout: G[row, p*p + p + q, q' + L - 1] (zero where |q'| > p); grid values
g[row, c, b, a] (omega, theta, phi), the layout of the forward transform's output.
"""
from __future__ import annotations

import numpy as np

from . import grid as _grid
from .wigner import wigner_d


def _d_tables(L: int, betas: np.ndarray) -> list[np.ndarray]:
    """d[p][b, q + p, q' + p] = d^p_{q,q'}(beta_b)."""
    return [np.stack([wigner_d(p, float(be)) for be in betas]) for p in range(L)]


def so3_synthesis(G: np.ndarray, L: int, n_phi: int, n_theta: int, n_omega: int) -> np.ndarray:
    """g[row, c, b, a] = sum_{p,q,q'} G^p_{q,q'} e^{-i q alpha_a} d^p_{q,q'}(beta_b)
    e^{-i q' gamma_c}."""
    G = np.asarray(G, dtype=np.complex128)
    al = _grid.alpha_angles(n_phi)
    be = _grid.beta_angles(n_phi, n_theta)
    ga = _grid.gamma_angles(n_omega)
    d = _d_tables(L, be)
    out = np.zeros((G.shape[0], n_omega, n_theta, n_phi), dtype=np.complex128)
    for p in range(L):
        qq = np.arange(-p, p + 1)
        Ea = np.exp(-1j * qq[:, None] * al[None, :])         # [q, a]
        Ec = np.exp(-1j * qq[:, None] * ga[None, :])         # [q', c]
        Gp = G[:, p * p:p * p + 2 * p + 1, L - 1 - p:L + p]  # [row, q, q']
        out += np.einsum("kqr,qa,bqr,rc->kcba", Gp, Ea, d[p], Ec, optimize=True)
    return out


def so3_analysis(g: np.ndarray, L: int, n_phi: int, n_theta: int, n_omega: int) -> np.ndarray:
    """G^p_{q,q'} = (2p+1)/(8 pi^2) * 1/(n_phi^2 n_omega)
    * sum_{a,b,c} q(beta_b) g[row, c, b, a] e^{i q alpha_a} d^p_{q,q'}(beta_b) e^{i q' gamma_c}
    for p < L (conj(D) with real d)."""
    g = np.asarray(g, dtype=np.complex128)
    al = _grid.alpha_angles(n_phi)
    be = _grid.beta_angles(n_phi, n_theta)
    ga = _grid.gamma_angles(n_omega)
    w = _grid.beta_weights(n_phi, n_theta) / (n_phi * n_phi * n_omega)
    d = _d_tables(L, be)
    out = np.zeros((g.shape[0], L * L, 2 * L - 1), dtype=np.complex128)
    for p in range(L):
        qq = np.arange(-p, p + 1)
        Ea = np.exp(1j * qq[:, None] * al[None, :])
        Ec = np.exp(1j * qq[:, None] * ga[None, :])
        s = np.einsum("kcba,b,qa,bqr,rc->kqr", g, w, Ea, d[p], Ec, optimize=True)
        out[:, p * p:p * p + 2 * p + 1, L - 1 - p:L + p] = (2 * p + 1) / (8 * np.pi ** 2) * s
    return out


def coupling_window_coefficients(A: np.ndarray, h: np.ndarray, L: int) -> np.ndarray:
    """G^p_{q,q'} = A^p_q h_p^{q'} (Eq:harmonic_formulation), A[row, p*p+p+q], h[p*p+p+q']."""
    A = np.asarray(A, dtype=np.complex128)
    h = np.asarray(h, dtype=np.complex128)
    out = np.zeros((A.shape[0], L * L, 2 * L - 1), dtype=np.complex128)
    for p in range(L):
        sl = slice(p * p, p * p + 2 * p + 1)
        out[:, sl, L - 1 - p:L + p] = A[:, sl, None] * h[sl][None, None, :]
    return out

"""Directional SLSHT by direct quadrature of its definition (test infrastructure only).

g(rho; l, m) = int_{S^2} f(x) (D_rho h)(x) conj(Y_l^m(x)) ds(x)
(Definition 1, eq. Eq:stft_spatial), for rho = (alpha, beta, gamma).

Evaluation, in the order the definition states it:
  1. f(x) = sum_{l,m} f_l^m Y_l^m(x) on the quadrature grid (eq. Eq:f_expansion);
  2. (D_rho h)_p^q = sum_{q'} D^p_{q,q'}(rho) h_p^{q'} (eq. eqn:rotation_non_symm),
     then (D_rho h)(x) = sum_{p,q} (D_rho h)_p^q Y_p^q(x);
  3. multiply, and integrate against conj(Y_l^m) with a rule that is exact for
     the product: Gauss-Legendre in cos(theta) with D//2 + 1 nodes times D + 1
     uniform phi samples, D = (L_f-1) + (L_h-1) + (l_hi-1) being the largest
     degree in the integrand.  This grid is deliberately not the paper's
     equiangular grid.
Because Y_l^m(theta, phi) = lam_l^m(theta) e^{i m phi}, each sum over the grid
is written as a sum over theta of a sum over phi; the sums are finite, so this
is the same number.

Also here, by the same quadrature (and, entry by entry, from sympy's exact Gaunt
coefficients: oracle_coupling_exact):
  * A^p_q(l, m) = int f Y_p^q conj(Y_l^m) ds, the coefficient that the harmonic
    formulation contracts with the window (eq. Eq:harmonic_formulation with the
    triple product T; it equals conj((conj(f) Y_l^m)_p^q) of
    eq. Eq:alternative_harmonic_formulation);
  * the energy sum_m |g(rho; l, m)|^2 per (l, rho);
  * the inverse through the spectral marginal (Section III-C): the discrete sum
    of eq. Eq:sig_reconstruction_discrete, then division by sqrt(16 pi^3) h_0^0
    (eq. Eq:inversion_2).
"""
from __future__ import annotations

import functools

import numpy as np

from . import grid as _grid
from .sph import legendre_table
from .wigner import wigner_d


@functools.lru_cache(maxsize=None)
def gauss_legendre(n: int):
    """Gauss-Legendre nodes and weights on [-1, 1], accurate to double precision.

    numpy's rule is the starting guess; each node is then polished by Newton
    steps on P_n in 40-digit arithmetic and its weight taken as
    2 / ((1 - x^2) P_n'(x)^2) there (numpy's own weights carry relative errors
    of order 1e-11 near the poles at the sizes used here)."""
    import mpmath
    x0, _ = np.polynomial.legendre.leggauss(n)
    xs = np.empty(n)
    ws = np.empty(n)
    with mpmath.workdps(40):
        for i, xi in enumerate(x0):
            x = mpmath.mpf(float(xi))
            for it in range(5):
                p0, p1 = mpmath.mpf(1), x
                for k in range(2, n + 1):
                    p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
                dp = n * (x * p1 - p0) / (x * x - 1)
                if it < 4:
                    x = x - p1 / dp
            xs[i] = float(x)
            ws[i] = float(2 / ((1 - x * x) * dp * dp))
    return xs, ws


def quadrature(D: int):
    """(theta_t, w_t, phi_j, n_phi): int F ds = sum_t w_t (2pi/n_phi) sum_j F(theta_t, phi_j)
    exactly for F of spherical-harmonic degree <= D."""
    n_t = D // 2 + 1
    x, w = gauss_legendre(n_t)
    n_p = D + 1
    return np.arccos(x), w, 2.0 * np.pi * np.arange(n_p) / n_p, n_p


def _lam_m(lam: np.ndarray, l: int, m: int) -> np.ndarray:
    return lam[l, m] if m >= 0 else ((-1.0) ** m) * lam[l, -m]


class _Setup:
    """Quadrature grid, Legendre table and f sampled on the grid."""

    def __init__(self, f, L_f, L_h, l_lo, l_hi):
        self.L_f, self.L_h, self.l_lo, self.l_hi = L_f, L_h, l_lo, l_hi
        D = (L_f - 1) + (L_h - 1) + (l_hi - 1)
        self.theta, self.w, self.phi, self.n_p = quadrature(D)
        lmax = max(L_f, L_h, l_hi) - 1
        self.lam = legendre_table(lmax, self.theta)
        nt = self.theta.shape[0]
        # f on the grid: F[t, j] = sum_m e^{i m phi_j} sum_l f_l^m lam_l^m(theta_t)
        fm = np.zeros((2 * L_f - 1, nt), dtype=np.complex128)
        for l in range(L_f):
            for m in range(-l, l + 1):
                fm[m + L_f - 1] += f[l * l + l + m] * _lam_m(self.lam, l, m)
        ms = np.arange(-(L_f - 1), L_f)
        self.F = fm.T @ np.exp(1j * np.outer(ms, self.phi))          # [t, j]
        # window-degree Legendre values, laid out [p, q+L_h-1, t]
        self.lam_h = np.zeros((L_h, 2 * L_h - 1, nt))
        for p in range(L_h):
            for q in range(-p, p + 1):
                self.lam_h[p, q + L_h - 1] = _lam_m(self.lam, p, q)
        qs = np.arange(-(L_h - 1), L_h)
        self.e_q = np.exp(1j * np.outer(qs, self.phi))                # [q, j]
        M = l_hi - 1
        self.ms_out = np.arange(-M, M + 1)
        self.e_out = np.exp(-1j * np.outer(self.phi, self.ms_out)) * (2.0 * np.pi / self.n_p)
        # projection weights wl[m+M, t, k] = w_t lam_l^m(theta_t) for l = l_lo + k
        nl = l_hi - l_lo
        self.wl = np.zeros((2 * M + 1, nt, nl))
        for k, l in enumerate(range(l_lo, l_hi)):
            for m in range(-l, l + 1):
                self.wl[m + M, :, k] = self.w * _lam_m(self.lam, l, m)

    def project(self, Q: np.ndarray) -> np.ndarray:
        """g[r, lm] = sum_t w_t sum_j (2pi/n_p) Q[r, t, j] conj(Y_l^m(theta_t, phi_j))."""
        nr, nt, _ = Q.shape
        R = (Q.reshape(nr * nt, -1) @ self.e_out).reshape(nr, nt, -1)   # [r, t, m]
        M = self.l_hi - 1
        out = np.zeros((nr, self.l_hi ** 2 - self.l_lo ** 2), dtype=np.complex128)
        for m in range(-M, M + 1):
            gm = R[:, :, m + M] @ self.wl[m + M]                          # [r, l]
            for k, l in enumerate(range(self.l_lo, self.l_hi)):
                if abs(m) <= l:
                    out[:, l * l + l + m - self.l_lo ** 2] = gm[:, k]
        return out


def _rotated_window(h, L_h, alpha, beta, gamma, dcache):
    """(D_rho h)_p^q for every rho, as [nrho, p, q+L_h-1]."""
    nr = alpha.shape[0]
    H = np.zeros((nr, L_h, 2 * L_h - 1), dtype=np.complex128)
    for r in range(nr):
        bkey = float(beta[r])
        if bkey not in dcache:
            dcache[bkey] = [wigner_d(p, bkey) for p in range(L_h)]
        ds = dcache[bkey]
        for p in range(L_h):
            qq = np.arange(-p, p + 1)
            Dm = (np.exp(-1j * qq * alpha[r])[:, None] * ds[p]
                  * np.exp(-1j * qq * gamma[r])[None, :])
            H[r, p, L_h - 1 - p:L_h + p] = Dm @ h[p * p:p * p + 2 * p + 1]
    return H


def oracle_g(f, h, L_f, L_h, l_lo, l_hi, alpha, beta, gamma, batch: int = 128):
    """g[r, l*l+l+m - l_lo^2] for rotations (alpha[r], beta[r], gamma[r])."""
    alpha = np.atleast_1d(np.asarray(alpha, dtype=np.float64))
    beta = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    gamma = np.atleast_1d(np.asarray(gamma, dtype=np.float64))
    S = _Setup(np.asarray(f), L_f, L_h, l_lo, l_hi)
    out = np.zeros((alpha.shape[0], l_hi ** 2 - l_lo ** 2), dtype=np.complex128)
    dcache: dict = {}
    for r0 in range(0, alpha.shape[0], batch):
        sl = slice(r0, r0 + batch)
        H = _rotated_window(np.asarray(h), L_h, alpha[sl], beta[sl], gamma[sl], dcache)
        Hq = np.einsum("rpq,pqt->rqt", H, S.lam_h)                       # [r, q, t]
        hx = np.einsum("rqt,qj->rtj", Hq, S.e_q)                        # (D_rho h)(x)
        out[sl] = S.project(S.F[None] * hx)
    return out


def oracle_g_grid(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, idx):
    """oracle_g at integer grid indices idx[k] = (a, b, c) of the SO(3) grid."""
    al, be, ga = _grid.rho_angles(n_phi, n_theta, n_omega, idx)
    return oracle_g(f, h, L_f, L_h, l_lo, l_hi, al, be, ga)


def oracle_g_full(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega):
    """g on the whole grid, laid out [lm, c(omega), b(theta), a(phi)]."""
    a, b, c = np.meshgrid(np.arange(n_phi), np.arange(n_theta), np.arange(n_omega),
                          indexing="ij")
    idx = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
    g = oracle_g_grid(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, idx)
    g = g.reshape(n_phi, n_theta, n_omega, -1)
    return np.ascontiguousarray(np.transpose(g, (3, 2, 1, 0)))


def oracle_coupling(f, L_f, L_h, l_lo, l_hi):
    """A[lm, p*p+p+q] = int f Y_p^q conj(Y_l^m) ds for p < L_h, |q| <= p."""
    S = _Setup(np.asarray(f), L_f, L_h, l_lo, l_hi)
    out = np.zeros((l_hi ** 2 - l_lo ** 2, L_h * L_h), dtype=np.complex128)
    for p in range(L_h):
        for q in range(-p, p + 1):
            Y = S.lam_h[p, q + L_h - 1][:, None] * S.e_q[q + L_h - 1][None, :]
            out[:, p * p + p + q] = S.project((S.F * Y)[None])[0]
    return out


def oracle_coupling_exact(f, L_f, l, m, p, q) -> complex:
    """One coefficient A^p_q(l, m) = int f Y_p^q conj(Y_l^m) ds from exact integrals:
    sum over l' of f_{l'}^{m-q} times int Y_{l'}^{m-q} Y_p^q conj(Y_l^m) ds, the integral
    written as (-1)^m times the Gaunt coefficient G(l', p, l; m-q, q, -m)
    (conj(Y_l^m) = (-1)^m Y_l^{-m}), which sympy evaluates exactly; the triple product T of
    eq. Eq:harmonic_formulation.  For high degrees, where the quadrature above carries more
    rounding (about 1e-12 relative at l = 300-400); slow (sympy)."""
    from sympy import N
    from sympy.physics.wigner import gaunt
    mp = m - q
    s = 0j
    for lp in range(max(abs(l - p), abs(mp)), min(l + p, L_f - 1) + 1):
        G = gaunt(lp, p, l, mp, q, -m)
        if G != 0:
            s += complex(f[lp * lp + lp + mp]) * float(N(G, 30))
    return (-1) ** m * s


def oracle_energy(g: np.ndarray, l_lo: int, l_hi: int) -> np.ndarray:
    """E[..., l - l_lo] = sum_{|m|<=l} |g[..., l*l+l+m-l_lo^2]|^2 (g's last axis is lm)."""
    out = np.zeros(g.shape[:-1] + (l_hi - l_lo,), dtype=np.float64)
    for k, l in enumerate(range(l_lo, l_hi)):
        s = l * l - l_lo ** 2
        out[..., k] = np.sum(np.abs(g[..., s:s + 2 * l + 1]) ** 2, axis=-1)
    return out


def oracle_marginal(g_full: np.ndarray, n_phi: int, n_theta: int, n_omega: int) -> np.ndarray:
    """f_hat[lm] = 1/(n_phi^2 n_omega) sum_{a,b,c} q(beta_b) g[lm, c, b, a]
    (eq. Eq:sig_reconstruction_discrete with per-axis sizes)."""
    q = _grid.beta_weights(n_phi, n_theta)
    s = np.einsum("lcba,b->l", g_full, q)
    return s / (n_phi * n_phi * n_omega)


def oracle_inverse(g_full, h00, n_phi, n_theta, n_omega) -> np.ndarray:
    """f_l^m = f_hat_l^m / (sqrt(16 pi^3) h_0^0)  (eq. Eq:inversion_2)."""
    return oracle_marginal(g_full, n_phi, n_theta, n_omega) / (np.sqrt(16.0 * np.pi ** 3) * h00)

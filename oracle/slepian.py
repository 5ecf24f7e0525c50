"""Slepian eigenfunction window on an elliptical region (Section III-D) -- oracle,
test infrastructure only.

Region (eq. Eq:region_def): R = {x : dist(x, F1) + dist(x, F2) <= 2a}, with foci
F1 = (theta_c, 0), F2 = (theta_c, pi) and 0 <= theta_c < a <= pi/2; dist is the
angular distance.  Among functions band-limited to s < L_h, the one with the largest
concentration  lambda = int_R |h|^2 / int_{S^2} |h|^2  is the top eigenvector of the
concentration matrix

    D_{i,j} = int_R conj(Y_i(x)) Y_j(x) ds(x),     i = s*s + s + r,

Hermitian and positive semi-definite with eigenvalues in [0, 1].  The window is
that eigenvector with a phase making the function real (h_s^{-r} = (-1)^r conj(h_s^r))
and unit energy.

How D is integrated here: for each colatitude theta the region's phi set is the whole
circle (theta <= b, cos b = cos a / cos theta_c), or two arcs |phi| <= phi*(theta) and
|phi - pi| <= phi*(theta) (b < theta <= a), phi* found by Brent's bracketing root
finder (scipy brentq) on the distance sum; the phi integral of e^{i k phi} over that set is
written out; the theta integral runs over [0, b] by Gauss-Legendre in cos(theta) and
over [b, a] by tanh-sinh quadrature, which absorbs the square-root behaviour of phi*
at both ends.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

from .sph import legendre_table, lam_signed
from .slsht import gauss_legendre


def _dist(theta1, phi1, theta2, phi2):
    c = np.sin(theta1) * np.sin(theta2) * np.cos(phi1 - phi2) + np.cos(theta1) * np.cos(theta2)
    return np.arccos(np.clip(c, -1.0, 1.0))


def in_region(theta, phi, theta_c, a):
    """Indicator of R_(theta_c, a) (eq. Eq:region_def)."""
    return _dist(theta, phi, theta_c, 0.0) + _dist(theta, phi, theta_c, np.pi) <= 2.0 * a


def minor_colatitude(theta_c, a):
    """Colatitude b of the ellipse at phi = pi/2: cos a = cos b cos theta_c (each focus is
    at distance a from that point)."""
    return float(np.arccos(np.cos(a) / np.cos(theta_c)))


def phi_half_width(theta, theta_c, a):
    """phi* in [0, pi/2] with dist-sum(theta, phi*) = 2a, for b < theta <= a."""
    f = lambda p: (_dist(theta, p, theta_c, 0.0) + _dist(theta, p, theta_c, np.pi)
                   - 2.0 * a)
    if f(0.0) >= 0.0:
        return 0.0
    if f(np.pi / 2) <= 0.0:
        return np.pi / 2
    return brentq(f, 0.0, np.pi / 2, xtol=1e-15, rtol=1e-15, maxiter=200)


def _arc_integral(k, phs):
    """int over |phi| <= phs and |phi - pi| <= phs of e^{i k phi} dphi (real)."""
    if k == 0:
        return 4.0 * phs
    return (1.0 + (-1.0) ** k) * 2.0 * np.sin(k * phs) / k


def _theta_nodes(theta_c, a, n_cap, n_ts):
    """(theta, weight, phi*) with weight including sin(theta); phi* = None on the cap."""
    b = minor_colatitude(theta_c, a)
    x, w = gauss_legendre(n_cap)
    # [0, b] in x = cos(theta): x in [cos b, 1]
    xc = 0.5 * (1.0 + np.cos(b)) + 0.5 * (1.0 - np.cos(b)) * x
    th1 = np.arccos(xc)
    w1 = 0.5 * (1.0 - np.cos(b)) * w
    # [b, a] by tanh-sinh: theta = m + r tanh(pi/2 sinh t)
    m, r = 0.5 * (a + b), 0.5 * (a - b)
    h = 6.0 / n_ts
    t = np.arange(-n_ts, n_ts + 1) * h
    u = np.tanh(0.5 * np.pi * np.sinh(t))
    du = 0.5 * np.pi * np.cosh(t) / np.cosh(0.5 * np.pi * np.sinh(t)) ** 2
    keep = np.abs(u) < 1.0
    th2 = m + r * u[keep]
    w2 = h * r * du[keep] * np.sin(th2)
    phs = np.array([phi_half_width(tt, theta_c, a) for tt in th2])
    return th1, w1, th2, w2, phs


def concentration_matrix(L_h, theta_c, a, n_cap=None, n_ts=None):
    """D[i, j] = int_R conj(Y_i) Y_j ds for i, j < L_h^2 (complex basis)."""
    n_cap = n_cap or (L_h + 8)
    n_ts = n_ts or (12 * L_h + 120)
    th1, w1, th2, w2, phs = _theta_nodes(theta_c, a, n_cap, n_ts)
    n = L_h * L_h
    idx = [(s, r) for s in range(L_h) for r in range(-s, s + 1)]
    lam1 = legendre_table(L_h - 1, th1)
    lam2 = legendre_table(L_h - 1, th2)
    Lam1 = np.array([lam_signed(lam1, s, r) for s, r in idx])      # [n, nodes]
    Lam2 = np.array([lam_signed(lam2, s, r) for s, r in idx])
    rr = np.array([r for _, r in idx])
    D = np.zeros((n, n), dtype=np.complex128)
    # cap: whole circle, only r == r' survives, int e^{0} = 2 pi
    D1 = 2.0 * np.pi * (Lam1 * w1) @ Lam1.T
    D += np.where(rr[:, None] == rr[None, :], D1, 0.0)
    # band: two arcs; group by k = r' - r
    for k in range(-(2 * L_h - 2), 2 * L_h - 1):
        Jk = np.array([_arc_integral(k, p) for p in phs])          # [nodes]
        if not np.any(Jk):
            continue
        Dk = (Lam2 * (w2 * Jk)) @ Lam2.T
        D += np.where((rr[None, :] - rr[:, None]) == k, Dk, 0.0)
    return D


def real_signal_phase(h, L_h):
    """Multiply an eigenvector by the phase that makes its function real-valued
    (h_s^{-r} = (-1)^r conj(h_s^r)); needs a non-degenerate eigenvalue."""
    t = np.zeros_like(h)
    for s in range(L_h):
        for r in range(-s, s + 1):
            t[s * s + s - r] = (-1.0) ** r * np.conj(h[s * s + s + r])
    psi = np.angle(np.vdot(h, t))
    return h * np.exp(0.5j * psi)


def slepian_window(L_h, theta_c, a):
    """(h, lambda): the unit-energy, real-valued window of largest concentration in
    R_(theta_c, a), and its concentration."""
    D = concentration_matrix(L_h, theta_c, a)
    ev, V = np.linalg.eigh(D)
    h = real_signal_phase(V[:, -1], L_h)
    h /= np.linalg.norm(h)
    return h, float(ev[-1])

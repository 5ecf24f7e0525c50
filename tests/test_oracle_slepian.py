"""Pins of the Slepian-window oracle (Section III-D, eq. Eq:region_def).

Independent of the oracle's own quadrature: polar caps (theta_c = 0, the remark after
eq. Eq:region_def) against scipy's associated Legendre functions integrated by
adaptive quadrature; the trace against the cap area; an elliptical region against a
brute-force indicator quadrature on a fine grid; the window's concentration against a
brute-force integral of |h|^2 over the region.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import lpmv

from oracle.slepian import (concentration_matrix, in_region, minor_colatitude,
                            slepian_window)
from oracle.sph import synthesize


def _nlam(s, r, x):
    """N_s^r P_s^r(x) with the Condon-Shortley phase (scipy's lpmv carries it), r >= 0."""
    n = math.sqrt((2 * s + 1) / (4 * math.pi) * math.factorial(s - r) / math.factorial(s + r))
    return n * lpmv(r, s, x)


@pytest.mark.parametrize("a", [0.4, 1.0, math.pi / 2])
def test_cap_matrix_is_diagonal_in_r_and_matches_adaptive_quadrature(a):
    L_h = 6
    D = concentration_matrix(L_h, 0.0, a)
    idx = [(s, r) for s in range(L_h) for r in range(-s, s + 1)]
    for i, (s, r) in enumerate(idx):
        for j, (s2, r2) in enumerate(idx):
            if r != r2:
                assert abs(D[i, j]) <= 1e-14, (s, r, s2, r2)
            elif r >= 0 and s2 >= s:
                want = 2 * math.pi * quad(lambda x: _nlam(s, r, x) * _nlam(s2, r, x),
                                          math.cos(a), 1.0, epsabs=1e-15, epsrel=1e-13)[0]
                assert abs(D[i, j] - want) <= 1e-13, (s, r, s2, want, D[i, j])
    # trace = L_h^2 * area / (4 pi) by the addition theorem; cap area 2 pi (1 - cos a)
    assert abs(np.trace(D).real - L_h ** 2 * (1 - math.cos(a)) / 2) <= 1e-12


def test_ellipse_matrix_against_brute_force_indicator():
    L_h, tc, a = 4, 0.3, 0.7
    D = concentration_matrix(L_h, tc, a)
    assert np.allclose(D, D.conj().T, atol=1e-15)
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= -1e-13 and ev.max() <= 1 + 1e-13
    # brute force: Gauss-Legendre in cos(theta) over [cos a, 1], midpoint grid in phi
    x, w = np.polynomial.legendre.leggauss(600)
    ca = math.cos(a)
    xc = 0.5 * (1 + ca) + 0.5 * (1 - ca) * x
    wt = 0.5 * (1 - ca) * w
    th = np.arccos(xc)
    nph = 8000
    ph = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    inside = in_region(T, P, tc, a)
    # separable basis: Y_i = lam_i(theta) e^{i r phi}; phi sums of the indicator by brute force
    from oracle.sph import lam_signed, legendre_table
    lam = legendre_table(L_h - 1, th)
    idx = [(s, r) for s in range(L_h) for r in range(-s, s + 1)]
    Lam = np.array([lam_signed(lam, s, r) for s, r in idx])             # [n, theta]
    M = {k: (inside * np.exp(1j * k * ph)[None, :]).sum(axis=1) * (2 * math.pi / nph)
         for k in range(-(2 * L_h - 2), 2 * L_h - 1)}
    Dbf = np.zeros_like(D)
    for i, (s, r) in enumerate(idx):
        for j, (s2, r2) in enumerate(idx):
            Dbf[i, j] = np.sum(wt * Lam[i] * Lam[j] * M[r2 - r])
    assert np.abs(Dbf - D).max() <= 1e-3 * np.abs(D).max()
    Wt = wt[:, None] * (2 * math.pi / nph) * inside
    # area of the region two ways (the trace of D and the indicator)
    area = float(Wt.sum())
    assert abs(np.trace(D).real - L_h ** 2 * area / (4 * math.pi)) <= 1e-3 * L_h ** 2


def test_minor_axis_and_hemisphere_remark():
    # cos a = cos b cos theta_c; a = pi/2 gives the hemisphere for any focus
    assert abs(minor_colatitude(0.3, 0.7) - math.acos(math.cos(0.7) / math.cos(0.3))) < 1e-15
    assert abs(minor_colatitude(0.4, math.pi / 2) - math.pi / 2) < 1e-15
    D1 = concentration_matrix(5, 0.4, math.pi / 2)
    D2 = concentration_matrix(5, 0.0, math.pi / 2)
    assert np.abs(D1 - D2).max() <= 1e-13


def test_window_is_real_unit_and_concentrated():
    L_h, tc, a = 5, 0.25, 0.6
    h, lam = slepian_window(L_h, tc, a)
    assert abs(np.linalg.norm(h) - 1) < 1e-13
    for s in range(L_h):
        for r in range(-s, s + 1):
            assert abs(h[s * s + s - r] - (-1) ** r * np.conj(h[s * s + s + r])) < 1e-13
    # concentration by brute force: int_R |h|^2 on a fine grid
    x, w = np.polynomial.legendre.leggauss(500)
    ca = math.cos(a)
    th = np.arccos(0.5 * (1 + ca) + 0.5 * (1 - ca) * x)
    wt = 0.5 * (1 - ca) * w
    nph = 6000
    ph = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    T, P = np.meshgrid(th, ph, indexing="ij")
    f = synthesize(h, L_h, T.ravel(), P.ravel()).reshape(T.shape)
    assert np.abs(f.imag).max() <= 1e-12 * np.abs(f).max()
    lam_bf = float(np.sum(np.abs(f) ** 2 * in_region(T, P, tc, a) * wt[:, None]) * 2 * math.pi / nph)
    assert abs(lam_bf - lam) <= 2e-3
    # better concentrated than any other band-limited function: random ones score lower
    D = concentration_matrix(L_h, tc, a)
    rng = np.random.default_rng(0)
    for _ in range(20):
        v = rng.standard_normal(L_h * L_h) + 1j * rng.standard_normal(L_h * L_h)
        v /= np.linalg.norm(v)
        assert np.vdot(v, D @ v).real < lam


def _paper_examples():
    import os
    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "slepian_paper_examples.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        L_h, tc, a, lam, pin = line.split()
        rows.append((int(L_h), float(tc), float(a), float(lam), pin == "yes"))
    return rows


def test_paper_stated_concentration():
    """The window of the paper's synthetic example and timing experiment (L_h = 18,
    R_(pi/6, pi/6 + pi/240)) has the concentration the paper states, 90% to the nearest
    percent (Section V)."""
    pinned = [r for r in _paper_examples() if r[4]]
    assert pinned
    for L_h, tc, a, stated, _ in pinned:
        _, lam = slepian_window(L_h, tc, a)
        assert abs(lam - stated) < 0.005, (L_h, lam)

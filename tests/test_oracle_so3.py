"""Pins of the synthesis stage's definition: the forward transform as a function on SO(3).

For every (l, m), g(rho; l, m) is a band-limited function on the rotation group whose
Wigner-D coefficients are A^p_q(l, m) h_p^{q'} (Eq:harmonic_formulation, Section II-C's
SO(3) expansion).  These tests check, on the CPU:
  * synthesis then analysis on the paper's grid returns random coefficients (the
    orthogonality Eq:WignerD_ortho made discrete by the inverse's beta weights);
  * the synthesis of A h equals the direct quadrature of the definition, and the
    analysis of that quadrature returns A h (two routes that share only the Wigner-d
    values);
  * on the beta = 0 row, d(0) is the identity, so g depends on alpha + gamma only and
    equals sum_q (sum_p G^p_{q,q}) e^{-i q (alpha + gamma)}.
"""
import numpy as np
import pytest

from oracle import grid as og
from oracle.slsht import oracle_coupling, oracle_g, oracle_g_full
from oracle.so3 import coupling_window_coefficients, so3_analysis, so3_synthesis
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window, grid_dims


def _random_G(rng, rows, L):
    G = np.zeros((rows, L * L, 2 * L - 1), dtype=np.complex128)
    for p in range(L):
        sl = slice(p * p, p * p + 2 * p + 1)
        G[:, sl, L - 1 - p:L + p] = (rng.standard_normal((rows, 2 * p + 1, 2 * p + 1))
                                     + 1j * rng.standard_normal((rows, 2 * p + 1, 2 * p + 1)))
    return G


@pytest.mark.parametrize("L,n_phi,n_theta,n_omega", [(3, 9, 5, 5), (4, 13, 7, 7),
                                                     (5, 23, 12, 9), (6, 21, 11, 11)])
def test_synthesis_analysis_round_trip(L, n_phi, n_theta, n_omega):
    """Exact whenever (n_phi - 1)/2 >= 2L - 2 and n_omega >= 2L - 1."""
    rng = np.random.default_rng(L)
    G = _random_G(rng, 3, L)
    g = so3_synthesis(G, L, n_phi, n_theta, n_omega)
    back = so3_analysis(g, L, n_phi, n_theta, n_omega)
    assert np.abs(back - G).max() < 1e-12 * np.abs(G).max()


def test_round_trip_needs_the_sampling_condition():
    """Below the condition the rule is not exact for the products, and the round trip
    visibly fails (the check above is not vacuous)."""
    rng = np.random.default_rng(7)
    L = 4
    G = _random_G(rng, 2, L)
    g = so3_synthesis(G, L, 9, 5, 7)           # (9 - 1)/2 = 4 < 2L - 2 = 6
    back = so3_analysis(g, L, 9, 5, 7)
    assert np.abs(back - G).max() > 1e-3


def test_synthesis_of_coupling_times_window_is_the_definition():
    """so3_synthesis(A h) equals the direct quadrature of Eq:stft_spatial on the whole
    grid, and so3_analysis of that quadrature returns A h."""
    rng = np.random.default_rng(11)
    L_f, L_h, l_lo, l_hi = 5, 3, 1, 5
    f = draw_coefficients(rng, L_f)
    h = draw_window(rng, L_h)
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h)
    A = oracle_coupling(f, L_f, L_h, l_lo, l_hi)
    G = coupling_window_coefficients(A, h, L_h)
    g_direct = oracle_g_full(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega)
    g_synth = so3_synthesis(G, L_h, n_phi, n_theta, n_omega)
    scale = np.abs(g_direct).max()
    assert np.abs(g_synth - g_direct).max() < 1e-13 * scale
    back = so3_analysis(g_direct, L_h, n_phi, n_theta, n_omega)
    assert np.abs(back - G).max() < 1e-12 * np.abs(G).max()


def test_beta_zero_row_depends_on_alpha_plus_gamma_only():
    rng = np.random.default_rng(5)
    L, n_phi, n_theta, n_omega = 4, 15, 8, 15
    G = _random_G(rng, 2, L)
    g = so3_synthesis(G, L, n_phi, n_theta, n_omega)
    al = og.alpha_angles(n_phi)
    ga = og.gamma_angles(n_omega)
    diag = np.zeros((2, 2 * L - 1), dtype=np.complex128)
    for p in range(L):
        for q in range(-p, p + 1):
            diag[:, q + L - 1] += G[:, p * p + p + q, q + L - 1]
    qq = np.arange(-(L - 1), L)
    s = al[None, :] + ga[:, None]                             # [c, a]
    closed = np.einsum("kq,qca->kca", diag, np.exp(-1j * qq[:, None, None] * s[None]))
    assert np.abs(g[:, :, 0, :] - closed).max() < 1e-13 * np.abs(closed).max()
    # n_phi == n_omega: the row is a function of (a + c) mod n
    for c in range(n_omega):
        assert np.allclose(g[:, c, 0, :], np.roll(g[:, 0, 0, :], -c, axis=-1), atol=1e-12)
    # and the direct quadrature of the definition does the same off the grid
    f = draw_coefficients(rng, 5)
    h = draw_window(rng, 3)
    t = rng.uniform(0, 2 * np.pi, 4)
    a0, c0 = 0.7, 1.9
    v = oracle_g(f, h, 5, 3, 0, 6, a0 + t, np.zeros(4), c0 - t)
    assert np.abs(v - v[0:1]).max() < 1e-13 * np.abs(v).max()
    w = oracle_g(f, h, 5, 3, 0, 6, np.full(4, a0), np.zeros(4), c0 + t)
    assert np.abs(w - w[0:1]).max() > 1e-3 * np.abs(w).max()

"""Plant plausible mistakes in the CPU oracle and check that a pin catches each.

Each mutant patches one oracle function for the duration of a test (CPU only)
and asserts that an existing pin in test_oracle_pins.py then fails.
"""
import numpy as np
import pytest

import oracle.grid as og
import oracle.slsht as osl
import oracle.sph as osph
import oracle.wigner as ow
import tests.test_oracle_pins as pins


def _patch(monkeypatch, name, value, modules=(ow, osl, osph, og, pins)):
    """Replace `name` in every module that holds it (several import it by name)."""
    for mod in modules:
        if hasattr(mod, name):
            monkeypatch.setattr(mod, name, value)


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_transposed_wigner_d_is_caught(monkeypatch):
    orig = ow.wigner_d
    _patch(monkeypatch, "wigner_d", lambda l, b: orig(l, b).T)
    _fails(pins.test_rotation_convention_pointwise, (0.4, 1.1, 2.3))


def test_wrong_phase_sign_in_delta_identity_is_caught(monkeypatch):
    def bad(l, beta):
        dl = ow.delta_matrix(l)
        mm = np.arange(-l, l + 1)
        core = dl.T @ (np.exp(1j * mm * beta)[:, None] * dl)   # e^{+i m'' beta}
        return np.real((1j) ** ((mm[:, None] - mm[None, :]) % 4) * core)
    _patch(monkeypatch, "wigner_d", bad)
    _fails(pins.test_wigner_d_matches_sympy_exact, 2, 1.9)


def test_missing_condon_shortley_phase_is_caught(monkeypatch):
    orig = osph.legendre_table

    def bad(lmax, theta):
        lam = orig(lmax, theta)
        for m in range(lmax + 1):
            lam[:, m] *= (-1.0) ** m
        return lam
    _patch(monkeypatch, "legendre_table", bad)
    _fails(pins.test_sph_harm_matches_scipy)


def test_unhalved_weight_at_beta_zero_is_caught(monkeypatch):
    orig = og.beta_weights

    def bad(n_phi, n_theta):
        q = orig(n_phi, n_theta)
        q[0] *= 2.0
        return q
    _patch(monkeypatch, "beta_weights", bad)
    _fails(pins.test_beta_weights_exact, 21)


def test_projection_without_conjugate_is_caught(monkeypatch):
    orig_init = osl._Setup.__init__

    def bad_init(self, *a, **k):
        orig_init(self, *a, **k)
        self.e_out = np.conj(self.e_out)
    monkeypatch.setattr(osl._Setup, "__init__", bad_init)
    _fails(pins.test_g_against_pointwise_rotation_and_independent_quadrature)


def test_dropped_window_order_is_caught(monkeypatch):
    orig = osl._rotated_window

    def bad(h, L_h, al, be, ga, dcache):
        H = orig(h, L_h, al, be, ga, dcache)
        H[:, :, 0] = 0.0              # drop q = -(L_h-1)
        return H
    _patch(monkeypatch, "_rotated_window", bad)
    _fails(pins.test_g_matches_harmonic_formulation_with_exact_gaunt)


def test_rotation_angle_swap_is_caught(monkeypatch):
    orig = ow.wigner_D
    _patch(monkeypatch, "wigner_D", lambda l, a, b, g: orig(l, g, b, a))
    _fails(pins.test_rotation_convention_pointwise, (0.4, 1.1, 2.3))


def test_inverse_normalisation_is_caught(monkeypatch):
    orig = osl.oracle_marginal
    monkeypatch.setattr(osl, "oracle_marginal",
                        lambda g, a, b, c: orig(g, a, b, c) * a / (a + 1))
    _fails(pins.test_inverse_recovers_signal)


def test_slepian_arc_integral_without_parity_factor_is_caught(monkeypatch):
    import oracle.slepian as osl_ep
    import tests.test_oracle_slepian as sl_pins
    monkeypatch.setattr(osl_ep, "_arc_integral",
                        lambda k, p: 4.0 * p if k == 0 else 4.0 * np.sin(k * p) / k)
    _fails(sl_pins.test_ellipse_matrix_against_brute_force_indicator)


def test_slepian_cap_without_sin_theta_weight_is_caught(monkeypatch):
    import oracle.slepian as osl_ep
    import tests.test_oracle_slepian as sl_pins
    orig = osl_ep._theta_nodes

    def bad(theta_c, a, n_cap, n_ts):
        th1, w1, th2, w2, phs = orig(theta_c, a, n_cap, n_ts)
        return th1, w1 / np.sqrt(1.0 - np.cos(th1) ** 2 + 1e-300), th2, w2, phs
    monkeypatch.setattr(osl_ep, "_theta_nodes", bad)
    _fails(sl_pins.test_cap_matrix_is_diagonal_in_r_and_matches_adaptive_quadrature, 1.0)

"""Oracle pins for steerable windows (remark on steerable windows, Section IV-B).

A window whose coefficients vanish for |r| >= N makes g(rho; l, m), as a function of
the third Euler angle gamma (= omega), a trigonometric polynomial with frequencies
|q'| < N: rotating the window about its own axis by gamma multiplies h_s^r by
e^{-i r gamma}.  Checked on the oracle's direct quadrature (which knows nothing of
the separated form), together with the converse for a general window, so a window
generator that failed to zero the coefficients would fail here too.
"""
import numpy as np

from oracle.slsht import oracle_g
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window


def _omega_spectrum(h, L_f, L_h, f, n_g=16):
    gam = 2 * np.pi * np.arange(n_g) / n_g
    al = np.full(n_g, 0.7)
    be = np.full(n_g, 1.1)
    g = oracle_g(f, h, L_f, L_h, 0, L_f + L_h - 1, al, be, gam)      # [n_g, n_lm]
    # g(gamma_j) = sum_k c_k e^{-i k gamma_j}  ->  c_k = (1/n) sum_j g_j e^{+i k gamma_j}
    c = np.fft.ifft(g, axis=0)
    k = np.fft.fftfreq(n_g, 1.0 / n_g).astype(int)
    return k, c


def test_steerable_window_is_band_limited_in_omega():
    rng = np.random.default_rng(5)
    L_f, L_h, n_az = 6, 5, 2
    f = draw_coefficients(rng, L_f)
    h = draw_window(rng, L_h, n_az=n_az)
    for s in range(L_h):
        for r in range(-s, s + 1):
            if abs(r) >= n_az:
                assert h[s * s + s + r] == 0
    k, c = _omega_spectrum(h, L_f, L_h, f)
    scale = np.abs(c).max()
    assert np.abs(c[np.abs(k) >= n_az]).max() <= 1e-13 * scale
    assert np.abs(c[np.abs(k) < n_az]).max() >= 0.1 * scale


def test_general_window_has_higher_omega_frequencies():
    rng = np.random.default_rng(5)
    L_f, L_h = 6, 5
    f = draw_coefficients(rng, L_f)
    h = draw_window(rng, L_h)
    k, c = _omega_spectrum(h, L_f, L_h, f)
    assert np.abs(c[np.abs(k) == L_h - 1]).max() >= 1e-3 * np.abs(c).max()
    assert np.abs(c[np.abs(k) >= L_h]).max() <= 1e-13 * np.abs(c).max()

"""Slepian window generator (Section III-D) on the GPU against the oracle.

The window of largest concentration in R_(theta_c, a) must match the oracle's (up to
its sign) and its concentration value, for a polar cap, two ellipses and the paper's
own region R_(pi/6, pi/6 + pi/240) at L_h = 18; the window then drives a forward
transform that matches the oracle."""
import math

import numpy as np
import pytest

from oracle.slepian import slepian_window as oracle_slepian
from oracle.slsht import oracle_g_full
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_coefficients
from tests.gpu_util import FP64_TOL, announce, dev, need_gpu, per_l_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("L_h,tc,a", [(6, 0.0, 0.5), (6, 0.25, 0.6), (10, math.pi / 6, math.pi / 6 + math.pi / 24),
                                      (18, math.pi / 6, math.pi / 6 + math.pi / 240)])
def test_window_matches_oracle(L_h, tc, a):
    announce(f"slepian L_h={L_h} theta_c={tc:.4f} a={a:.4f}")
    h, lam = api.slepian_window(L_h, tc, a)
    ho, lamo = oracle_slepian(L_h, tc, a)
    assert abs(lam - lamo) <= 1e-11 * max(lamo, 1e-3)
    assert abs(np.linalg.norm(h) - 1.0) < 1e-13
    for s in range(L_h):
        for r in range(-s, s + 1):
            assert h[s * s + s - r] == pytest.approx((-1) ** r * np.conj(h[s * s + s + r]), abs=1e-15)
    err = min(np.abs(h - ho).max(), np.abs(h + ho).max())
    assert err <= 1e-9, err


def test_slepian_window_drives_the_forward_transform():
    announce("slepian window in a forward transform")
    L_f, L_h, l_lo, l_hi, n_phi, n_omega = 7, 5, 2, 9, 25, 9
    h, _ = api.slepian_window(L_h, 0.3, 0.8)
    f = draw_coefficients(np.random.default_rng(9), L_f)
    n_theta = (n_phi + 1) // 2
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega))
    g = plan.forward(dev(f), dev(h)).cpu().numpy()
    ref = oracle_g_full(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega)
    assert max(per_l_rel_err(g, ref, l_lo, l_hi).values()) <= FP64_TOL

"""GPU inverse (spectral-marginal inversion, Section III-C) through the C ABI.

The forward output is summed with the beta weights of the discrete inverse
(eq. Eq:sig_reconstruction_discrete) and divided by sqrt(16 pi^3) h_0^0
(eq. Eq:inversion_2).  Checked against the signal itself (the paper's
inversion identity), against the oracle's inverse of the oracle's g, and on
its argument checks.
"""
import numpy as np
import pytest

from oracle.slsht import oracle_g_full, oracle_inverse
from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window, make_inputs, workload
from tests.gpu_util import announce, dev, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _roundtrip(L_f, L_h, l_lo, l_hi, n_phi, n_omega, prec, f, h):
    n_theta = (n_phi + 1) // 2
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision=prec))
    ht = dev(h)
    g = plan.forward(dev(f), ht)
    fr = plan.inverse(g, ht).cpu().numpy()
    ref = np.zeros(max(l_hi, L_f) ** 2, dtype=complex)
    ref[:L_f * L_f] = f
    return fr, ref[l_lo * l_lo:l_hi * l_hi]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6)])
def test_roundtrip_tiny_beyond_band(prec, tol):
    """l window up to L_f + L_h - 1: f_l^m back for l < L_f, zero above."""
    announce(f"inverse tiny {prec}")
    rng = np.random.default_rng(8)
    L_f, L_h = 8, 3
    f = draw_coefficients(rng, L_f)
    h = draw_window(rng, L_h)
    fr, ref = _roundtrip(L_f, L_h, 0, L_f + L_h - 1, 2 * (L_f + L_h) - 1, 2 * L_h - 1, prec, f, h)
    scale = np.abs(f).max()
    assert np.abs(fr - ref).max() <= tol * scale
    assert np.abs(fr[L_f * L_f:]).max() <= tol * scale


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 2e-6)])
def test_roundtrip_mid(prec, tol):
    """The mid-size workload at full size: 11.3 GB (FP64) of g summed back to f."""
    wl = workload("mid")
    announce(f"inverse mid {prec}")
    f, h = make_inputs(wl)
    fr, ref = _roundtrip(wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_omega, prec, f, h)
    torch.cuda.empty_cache()
    assert np.abs(fr - ref).max() <= tol * np.abs(ref).max()


def test_inverse_of_oracle_distribution():
    """The GPU inverse applied to the oracle's g equals the oracle's inverse of it."""
    announce("inverse of oracle g")
    wl = workload("tiny")
    f, h = make_inputs(wl)
    g = oracle_g_full(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta, wl.n_omega)
    plan = api.Plan(api.desc_for(wl))
    fr = plan.inverse(dev(g), dev(h)).cpu().numpy()
    ref = oracle_inverse(g, h[0], wl.n_phi, wl.n_theta, wl.n_omega)
    assert np.abs(fr - ref).max() <= 1e-14 * np.abs(ref).max() * 10


def test_inverse_argument_checks():
    wl = workload("tiny")
    f, h = make_inputs(wl)
    plan = api.Plan(api.desc_for(wl))
    g = plan.forward(dev(f), dev(h))
    h0 = h.copy()
    h0[0] = 0.0
    # h_0^0 is read by the kernel (no host synchronisation): a zero gives non-finite output
    assert not np.isfinite(plan.inverse(g, dev(h0)).cpu().numpy()).any()
    part = api.Plan(api.desc_for(wl, theta_lo=1))
    with pytest.raises(L.SlshtError, match="theta"):
        part.inverse(part.forward(dev(f), dev(h)), dev(h))
    small = api.Plan(api.make_desc(8, 3, 0, 8, 21, 11, 3))
    with pytest.raises(L.SlshtError, match="n_omega"):
        small.inverse(small.forward(dev(f), dev(h)), dev(h))

"""Properties that hold at any size, checked on every sample of the full-size outputs
(the sampled-rotation parity tests compare with the oracle; these cover the rest).

Rotating f about the z axis by alpha_k = 2 pi k / n_phi multiplies f_l^m by e^{-i m alpha_k}
and turns g into e^{-i m alpha_k} g(phi_{a-k}); rotating h about z by gamma_k = 2 pi k /
n_omega multiplies h_s^r by e^{-i r gamma_k} and turns g into g(omega_{c+k}) (rotation
convention of Section II-B; the same identities are pinned on the oracle).  The energy
sum_m |g|^2 is then shifted in phi and unchanged otherwise."""
import numpy as np
import pytest

from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import make_inputs, workload
from tests.gpu_util import FP32_TOL, FP64_TOL, announce, dev, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _orders(l_lo, l_hi):
    return np.concatenate([np.arange(-l, l + 1) for l in range(l_lo, l_hi)])


def _max_rel_per_l(got, ref, l_lo, l_hi):
    worst = 0.0
    for l in range(l_lo, l_hi):
        s = l * l - l_lo * l_lo
        d = torch.linalg.vector_norm((got[s:s + 2 * l + 1] - ref[s:s + 2 * l + 1]).flatten())
        n = torch.linalg.vector_norm(ref[s:s + 2 * l + 1].flatten())
        worst = max(worst, float(d / n))
    return worst


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_mid_phi_shift_every_sample(prec, tol):
    announce(f"mid phi-shift equivariance {prec}")
    wl = workload("mid")
    f, h = make_inputs(wl)
    plan = api.Plan(api.desc_for(wl, precision=prec))
    g = plan.forward(dev(f), dev(h))
    k = 37
    ak = 2 * np.pi * k / wl.n_phi
    mm = np.concatenate([np.arange(-l, l + 1) for l in range(wl.L_f)])
    g2 = plan.forward(dev(f * np.exp(-1j * mm * ak)), dev(h))
    ph = torch.from_numpy(np.exp(-1j * _orders(wl.l_lo, wl.l_hi) * ak)).to(g.device, g.dtype)
    ref = torch.roll(g, k, dims=3)
    ref *= ph[:, None, None, None]
    assert _max_rel_per_l(g2, ref, wl.l_lo, wl.l_hi) <= tol


def test_mid_omega_shift_every_sample():
    announce("mid omega-shift equivariance fp64")
    wl = workload("mid")
    f, h = make_inputs(wl)
    plan = api.Plan(api.desc_for(wl))
    g = plan.forward(dev(f), dev(h))
    kc = 4
    gk = 2 * np.pi * kc / wl.n_omega
    qq = np.concatenate([np.arange(-p, p + 1) for p in range(wl.L_h)])
    g3 = plan.forward(dev(f), dev(h * np.exp(-1j * qq * gk)))
    assert _max_rel_per_l(g3, torch.roll(g, -kc, dims=1), wl.l_lo, wl.l_hi) <= FP64_TOL


def test_large_energy_phi_shift_every_sample():
    """L_f = 512, L_h = 32, l in [100, 116), 1087 x 544 x 63 grid, real-pair energy: the
    whole 2.4 GB output of the rotated signal is the shifted output of the original."""
    announce("large energy phi-shift")
    wl = workload("large")
    f, h = make_inputs(wl)
    plan = api.Plan(api.desc_for(wl, real_pair=True))
    E = plan.forward(dev(f), dev(h))
    k = 101
    ak = 2 * np.pi * k / wl.n_phi
    mm = np.concatenate([np.arange(-l, l + 1) for l in range(wl.L_f)])
    E2 = plan.forward(dev(f * np.exp(-1j * mm * ak)), dev(h))
    ref = torch.roll(E, k, dims=3)
    err = float((E2 - ref).abs().max() / ref.abs().max())
    assert err <= FP32_TOL, err

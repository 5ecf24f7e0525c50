"""The paper's own route (factoring of rotations with Delta = d(pi/2) and a 3-D Fourier
sum, Section IV-B) on its minimal grid E_{L_h}: against the oracle on the whole grid,
and against the separated-form kernel on the same grid, including the paper's window
band-limit L_h = 18."""
import numpy as np
import pytest

from oracle.slsht import oracle_g_full
from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window
from tests.gpu_util import FP64_TOL, announce, dev, need_gpu, per_l_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _minimal(L_f, L_h, l_lo, l_hi):
    K = 2 * L_h - 1
    return api.make_desc(L_f, L_h, l_lo, l_hi, K, L_h, K)


def test_factored_route_whole_grid_vs_oracle():
    announce("factored route vs oracle")
    rng = np.random.default_rng(51)
    L_f, L_h = 8, 3
    f = draw_coefficients(rng, L_f)
    h = draw_window(rng, L_h)
    l_lo, l_hi = 0, L_f + L_h - 1
    plan = api.Plan(_minimal(L_f, L_h, l_lo, l_hi))
    g = plan.forward_factored(dev(f), dev(h)).cpu().numpy()
    K = 2 * L_h - 1
    ref = oracle_g_full(f, h, L_f, L_h, l_lo, l_hi, K, L_h, K)
    assert max(per_l_rel_err(g, ref, l_lo, l_hi).values()) <= FP64_TOL


@pytest.mark.parametrize("L_f,L_h,l_lo,l_hi", [(40, 8, 0, 47), (20, 18, 10, 20), (9, 1, 0, 9)])
def test_factored_route_equals_separated_form(L_f, L_h, l_lo, l_hi):
    announce(f"factored vs separated L_f={L_f} L_h={L_h}")
    rng = np.random.default_rng(52)
    f = draw_coefficients(rng, L_f, 2.0, True)
    h = draw_window(rng, L_h)
    plan = api.Plan(_minimal(L_f, L_h, l_lo, l_hi))
    gf = plan.forward_factored(dev(f), dev(h)).cpu().numpy()
    gs = plan.forward(dev(f), dev(h)).cpu().numpy()
    assert max(per_l_rel_err(gf, gs, l_lo, l_hi).values()) <= FP64_TOL


def test_factored_route_rejects_other_grids():
    d = api.make_desc(8, 3, 0, 8, 21, 11, 5)
    assert L.lib().slsht_factored_workspace(d) == -1
    plan = api.Plan(d)
    rng = np.random.default_rng(0)
    f = draw_coefficients(rng, 8)
    h = draw_window(rng, 3)
    with pytest.raises(L.SlshtError):
        plan.forward_factored(dev(f), dev(h))


def test_trapani_delta_vs_exact():
    """Delta^p = d^p(pi/2) from the Trapani-Navaza recursion against Wigner's sum in
    exact integer arithmetic, every canonical entry up to the largest band-limit."""
    from oracle.wigner import delta_matrix
    announce("Trapani Delta L_h=32")
    L_h = 32
    got = api.wigner_delta(L_h).cpu().numpy()
    err = 0.0
    for p in range(L_h):
        D = delta_matrix(p)
        off = p * (p + 1) * (2 * p + 1) // 6
        for Q in range(p + 1):
            for Qp in range(-Q, Q + 1):
                err = max(err, abs(got[off + Q * Q + Q + Qp] - D[Q + p, Qp + p]))
    assert err <= 1e-14, err


def test_factored_synthesis_from_modulated_coupling_vs_oracle():
    """The paper's whole route (tau_1: coupling by the modulated-signal transform, tau_2:
    factored synthesis from it) against the oracle on every sample of the minimal grid."""
    announce("modulated coupling + factored synthesis vs oracle")
    rng = np.random.default_rng(53)
    L_f, L_h = 7, 4
    f = draw_coefficients(rng, L_f)
    h = draw_window(rng, L_h)
    l_lo, l_hi = 0, L_f + L_h - 1
    plan = api.Plan(_minimal(L_f, L_h, l_lo, l_hi))
    A = plan.coupling_modulated(dev(f))
    g = plan.synthesize_factored(A, dev(h)).cpu().numpy()
    K = 2 * L_h - 1
    ref = oracle_g_full(f, h, L_f, L_h, l_lo, l_hi, K, L_h, K)
    assert max(per_l_rel_err(g, ref, l_lo, l_hi).values()) <= FP64_TOL
    g2 = plan.forward_factored(dev(f), dev(h)).cpu().numpy()
    assert max(per_l_rel_err(g, g2, l_lo, l_hi).values()) <= FP64_TOL

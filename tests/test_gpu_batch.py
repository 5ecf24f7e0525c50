"""Several transforms in common launches (slsht_forward_batch): the couplings of all
plans, then one synthesis grid per group of plans sharing a synthesis kernel, its blocks
split between the transforms by a tile list.  Every output must equal, bit for bit, the
same plan's slsht_forward (same kernels, same arithmetic), and the tiny configuration is
also checked against the oracle on its whole grid."""
import numpy as np
import pytest

from oracle.slsht import oracle_g_full
from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window, grid_dims
from tests.gpu_util import FP64_TOL, announce, dev, need_gpu, per_l_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _case(rng, L_f, L_h, l_lo, l_hi, prec="fp64", output="full", pair=False, grid=None):
    n_phi, n_theta, n_omega = grid or grid_dims(L_f, L_h)
    d = api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision=prec,
                      output=output, real_pair=pair)
    f = draw_coefficients(rng, L_f, 2.0 if L_f > 8 else 0.0, L_f > 8)
    h = draw_window(rng, L_h)
    return api.Plan(d), dev(f), dev(h)


def _check(cases):
    plans = [c[0] for c in cases]
    gb = api.forward_batch(plans, [c[1] for c in cases], [c[2] for c in cases])
    for i, (p, f, h) in enumerate(cases):
        alone = p.forward(f, h).cpu().numpy()
        assert np.array_equal(gb[i].cpu().numpy(), alone), i


def test_batch_uneven_requests_equal_alone():
    """Uneven shapes sharing kernels (VALU FP64 L_h <= 4 and <= 8, FP32, the MFMA phi
    stage at L_h = 16, real pair, a theta window), plus an ENERGY plan."""
    announce("batch uneven")
    rng = np.random.default_rng(71)
    cases = [
        _case(rng, 8, 3, 0, 8, grid=(21, 11, 5)),
        _case(rng, 20, 3, 4, 9),
        _case(rng, 33, 4, 10, 18),
        _case(rng, 24, 8, 5, 13),
        _case(rng, 40, 8, 30, 38, pair=True),
        _case(rng, 32, 8, 0, 8, prec="fp32"),
        _case(rng, 20, 8, 2, 10, prec="fp32", pair=True),
        _case(rng, 32, 16, 8, 16),
        _case(rng, 24, 16, 3, 11),
        _case(rng, 24, 8, 4, 12, prec="fp32", output="energy"),
    ]
    _check(cases)


def test_batch_theta_slices_and_steerable_windows():
    """Per-transform arguments that differ only in the theta slice or the steerable limit
    (all four share the FP64 L_h <= 8 kernel)."""
    announce("batch theta slices and steerable")
    rng = np.random.default_rng(75)
    L_f, L_h = 24, 8
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h)
    cases = []
    for tlo, thi, n_az in ((0, 0, 0), (5, 9, 0), (17, 18, 3), (0, 0, 2)):
        d = api.make_desc(L_f, L_h, 6, 12, n_phi, n_theta, n_omega, theta_lo=tlo,
                          theta_hi=thi, n_az=n_az)
        f = draw_coefficients(rng, L_f, 2.0, True)
        h = draw_window(rng, L_h)
        if n_az:
            for s_ in range(L_h):
                for r in range(-s_, s_ + 1):
                    if abs(r) >= n_az:
                        h[s_ * s_ + s_ + r] = 0
            h /= np.linalg.norm(h)
        cases.append((api.Plan(d), dev(f), dev(h)))
    _check(cases)


def test_batch_more_than_one_grid_of_transforms():
    """20 plans sharing one kernel: two grids (16 + 4 transforms)."""
    announce("batch 20 plans")
    rng = np.random.default_rng(72)
    cases = [_case(rng, 12 + (i % 5), 4, i % 3, i % 3 + 4) for i in range(20)]
    _check(cases)


def test_batch_tiny_whole_grid_vs_oracle():
    announce("batch tiny vs oracle")
    rng = np.random.default_rng(73)
    cases = [_case(rng, 8, 3, 0, 8, grid=(21, 11, 5)) for _ in range(3)]
    gb = api.forward_batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases])
    for (p, f, h), g in zip(cases, gb):
        ref = oracle_g_full(f.cpu().numpy(), h.cpu().numpy(), 8, 3, 0, 8, 21, 11, 5)
        assert max(per_l_rel_err(g.cpu().numpy(), ref, 0, 8).values()) <= FP64_TOL


def test_batch_rejects_a_repeated_plan():
    rng = np.random.default_rng(74)
    p, f, h = _case(rng, 8, 3, 0, 8, grid=(21, 11, 5))
    with pytest.raises(L.SlshtError):
        api.forward_batch([p, p], [f, f], [h, h])

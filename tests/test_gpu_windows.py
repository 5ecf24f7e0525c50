"""Several windows against one signal (remark on multiple windows, Section IV-B):
slsht_forward_windows computes the coupling of f once and one synthesis per window.
Each window's output must equal, bit for bit, slsht_forward with that window alone
(FULL FP64 / FP32, real pair, ENERGY)."""
import numpy as np
import pytest

from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window
from tests.gpu_util import announce, dev, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("prec,output,pair", [("fp64", "full", False), ("fp32", "full", True),
                                              ("fp32", "energy", False)])
def test_windows_equal_separate_forwards(prec, output, pair):
    announce(f"multi-window {prec} {output} pair={pair}")
    rng = np.random.default_rng(41)
    L_f, L_h, l_lo, l_hi, n_phi, n_omega, W = 12, 5, 3, 15, 33, 9, 3
    f = draw_coefficients(rng, L_f)
    hs = np.stack([draw_window(rng, L_h) for _ in range(W)])
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, (n_phi + 1) // 2, n_omega,
                                  precision=prec, output=output, real_pair=pair))
    g = plan.forward_windows(dev(f), dev(hs)).cpu().numpy()
    for w in range(W):
        alone = plan.forward(dev(f), dev(hs[w])).cpu().numpy()
        assert np.array_equal(g[w], alone), w


def test_windows_argument_checks():
    rng = np.random.default_rng(42)
    f = draw_coefficients(rng, 8)
    h = draw_window(rng, 3)
    plan = api.Plan(api.make_desc(8, 3, 0, 8, 21, 11, 5))
    g = plan.empty_output()
    lib = L.lib()
    import ctypes
    rc = lib.slsht_forward_windows(plan._h, ctypes.c_void_p(dev(f).data_ptr()),
                                   ctypes.c_void_p(dev(h).data_ptr()), 0,
                                   ctypes.c_void_p(g.data_ptr()), None)
    assert rc == L.SLSHT_EINVAL
    with pytest.raises(ValueError):
        plan.forward_windows(dev(f), dev(h))            # 1-D h: not [W, L_h^2]
    torch.cuda.synchronize()

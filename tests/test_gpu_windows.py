"""Several windows against one signal (remark on multiple windows, Section IV-B):
slsht_forward_windows computes the coupling of f once and one synthesis per window.
Every window's output is compared with the FP64 oracle: on the whole grid of a small
case (FULL FP64, FULL FP32 with the real pair, ENERGY against the oracle's energy), and
on seeded rotations of the mid-size workload with four windows (the benchmark's shape).
Each window's output must also equal, bit for bit, slsht_forward with that window alone."""
import numpy as np
import pytest

from oracle.slsht import oracle_energy, oracle_g_full, oracle_g_grid
from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import (draw_coefficients, draw_window, make_inputs, rho_subset,
                                        workload)
from tests.gpu_util import (FP32_TOL, FP64_TOL, announce, dev, gather_rho, need_gpu,
                            per_l_rel_err, torch)

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


@pytest.mark.parametrize("prec,output,pair,tol", [("fp64", "full", False, FP64_TOL),
                                                  ("fp32", "full", True, FP32_TOL),
                                                  ("fp32", "energy", False, FP32_TOL)])
def test_every_window_matches_the_oracle_whole_grid(prec, output, pair, tol):
    announce(f"multi-window vs oracle, whole grid {prec} {output} pair={pair}")
    rng = np.random.default_rng(43)
    L_f, L_h, l_lo, l_hi, n_phi, n_omega, W = 11, 5, 2, 15, 31, 9, 3
    n_theta = (n_phi + 1) // 2
    f = draw_coefficients(rng, L_f, 2.0, True)
    hs = np.stack([draw_window(rng, L_h) for _ in range(W)])
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega,
                                  precision=prec, output=output, real_pair=pair))
    g = plan.forward_windows(dev(f), dev(hs)).cpu().numpy()
    for w in range(W):
        ref = oracle_g_full(f, hs[w], L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega)
        if output == "energy":
            E = np.moveaxis(oracle_energy(np.moveaxis(ref, 0, -1), l_lo, l_hi), -1, 0)
            rel = np.abs(g[w] - E).max() / np.abs(E).max()
            assert rel <= tol, (w, rel)
        else:
            errs = per_l_rel_err(g[w], ref, l_lo, l_hi)
            assert max(errs.values()) <= tol, (w, errs)
            assert np.abs(g[w] - ref).max() <= 10 * tol * np.abs(ref).max()


def test_mid_four_windows_sampled_rotations():
    """The benchmark's shape: the mid-size workload's signal against four windows, FP64,
    each window's output on 96 seeded rotations for all 1280 (l, m)."""
    wl = workload("mid")
    f, _ = make_inputs(wl)
    rng = np.random.default_rng(2)
    W = 4
    hs = np.stack([draw_window(rng, wl.L_h) for _ in range(W)])
    idx = rho_subset(wl, 96, seed=77)
    announce("multi-window mid W=4 sampled rotations")
    plan = api.Plan(api.desc_for(wl), device=0)
    g = plan.forward_windows(dev(f), dev(hs))
    got = [gather_rho(g[w], idx) for w in range(W)]
    del g
    torch.cuda.empty_cache()
    for w in range(W):
        ref = oracle_g_grid(f, hs[w], wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta,
                            wl.n_omega, idx)
        errs = per_l_rel_err(got[w], ref, wl.l_lo, wl.l_hi, axis=1)
        assert max(errs.values()) <= FP64_TOL, (w, errs)
        assert np.abs(got[w] - ref).max() <= 10 * FP64_TOL * np.abs(ref).max(), w


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

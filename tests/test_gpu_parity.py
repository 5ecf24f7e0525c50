"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Small cases are compared on the whole SO(3) grid; the mid-size workload
(L_f=128, L_h=8, l in [32,48), 271x136x15 grid) is compared on a seeded sample
of rotations for every (l, m), in the launch configuration the benchmark
times.  Bars: relative Frobenius error per degree <= 1e-12 for FP64 and
<= 1e-5 for FP32-mixed.
"""
import os

import numpy as np
import pytest

from oracle.slsht import oracle_coupling, oracle_g_full, oracle_g_grid
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import (draw_coefficients, draw_window, make_inputs,
                                        rho_subset, workload)
from tests.gpu_util import (FP32_TOL, FP64_TOL, announce, dev, gather_rho, max_rel, need_gpu,
                            per_l_rel_err, torch)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.fixture(scope="module")
def mid_case():
    wl = workload("mid")
    f, h = make_inputs(wl)
    idx = rho_subset(wl, 240, seed=2024)
    ref = oracle_g_grid(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta,
                        wl.n_omega, idx)
    return wl, f, h, idx, ref


def _full_case(L_f, L_h, l_lo, l_hi, n_phi, n_omega, prec, seed, **kw):
    rng = np.random.default_rng(seed)
    f = draw_coefficients(rng, L_f, 0.0)
    h = draw_window(rng, L_h, n_az=kw.get("n_az", 0))     # steerable: |r| >= n_az zeroed
    n_theta = (n_phi + 1) // 2
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision=prec,
                                  **kw))
    g = plan.forward(dev(f), dev(h)).cpu().numpy()
    ref = oracle_g_full(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega)
    return f, h, g, ref


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_tiny_whole_grid(prec, tol):
    wl = workload("tiny")
    announce(f"tiny whole grid {prec}")
    f, h = make_inputs(wl)
    plan = api.Plan(api.desc_for(wl, precision=prec))
    g = plan.forward(dev(f), dev(h)).cpu().numpy()
    ref = oracle_g_full(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta, wl.n_omega)
    errs = per_l_rel_err(g, ref, wl.l_lo, wl.l_hi)
    assert max(errs.values()) <= tol, errs
    assert max_rel(g, ref) <= 10 * tol


def test_coupling_matches_oracle_tiny_and_mid():
    for name in ("tiny", "mid"):
        wl = workload(name)
        announce(f"coupling {name}")
        f, _ = make_inputs(wl)
        plan = api.Plan(api.desc_for(wl))
        A = plan.coupling(dev(f)).cpu().numpy()
        ref = oracle_coupling(f, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi)
        assert max_rel(A, ref) <= FP64_TOL, name


def test_coupling_large_degrees():
    """3j recursions at l' up to 131+31: L_f=132, L_h=32, l in [100,102)."""
    rng = np.random.default_rng(5)
    f = draw_coefficients(rng, 132, 2.5, True)
    announce("coupling large degrees")
    plan = api.Plan(api.make_desc(132, 32, 100, 102, 327, 164, 63, precision="fp32"))
    A = plan.coupling(dev(f)).cpu().numpy()
    ref = oracle_coupling(f, 132, 32, 100, 102)
    assert max_rel(A, ref) <= FP64_TOL


@pytest.mark.parametrize("L_f,L_h,l_lo,l_hi", [
    (12, 18, 0, 29),    # l < p: |l - p| ranges from both sides; 324 pairs: 320 lanes + 4 folded
    (20, 9, 0, 12),     # 81 pairs: 64 lanes + 17 folded; m = 0 blocks pair (p, q) with (p, -q)
    (30, 18, 41, 47),   # odd l_lo: (l, m >= 0) block numbering from an offset
    (7, 1, 0, 7),       # scalar window: one pair, one Z row
    (40, 32, 0, 3),     # 1024 pairs over 512 lanes, l < L_h for every row
])
def test_coupling_block_shapes_and_low_degrees(L_f, L_h, l_lo, l_hi):
    """The coupling's block layouts against the oracle: one block per (l, m >= 0) writing
    the orders +-m, Z rows from the closed-form ratio at l below and above p, whole-wave
    blocks with the leftover (p, q) pairs folded onto the first lanes."""
    rng = np.random.default_rng(L_f * 100 + L_h)
    f = draw_coefficients(rng, L_f, 2.0, True)
    announce(f"coupling L_f={L_f} L_h={L_h} l=[{l_lo},{l_hi})")
    n_phi = 2 * (L_f + L_h) - 1
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, (n_phi + 1) // 2, 2 * L_h - 1))
    A = plan.coupling(dev(f)).cpu().numpy()
    ref = oracle_coupling(f, L_f, L_h, l_lo, l_hi)
    assert max_rel(A, ref) <= FP64_TOL


def test_coupling_high_degree_golden():
    """Degrees 300 and 399 (L_h = 32 and 6) against sampled exact values (sympy's Gaunt
    coefficients through oracle_coupling_exact) stored by
    tests/golden/make_coupling_high_degree.py: long 3j recursions, Z rows of the
    closed-form ratio far from l = p, recursion coefficients near 1e17 under the refined
    reciprocal square root."""
    path = os.path.join(os.path.dirname(__file__), "golden", "coupling_high_degree.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    cases = {}
    for r in rows:
        key = tuple(int(x) for x in r[:4])
        cases.setdefault(key, []).append((int(r[4]), int(r[5]), int(r[6]),
                                          complex(float(r[7]), float(r[8]))))
    assert len(cases) == 2 and len(rows) == 512
    for (L_f, L_h, seed, l), ents in cases.items():
        announce(f"coupling golden L_f={L_f} L_h={L_h} l={l}")
        f = draw_coefficients(np.random.default_rng(seed), L_f, 2.0, True)
        K = 2 * L_h - 1
        plan = api.Plan(api.make_desc(L_f, L_h, l, l + 1, K, L_h, K))
        A = plan.coupling(dev(f)).cpu().numpy()
        got = np.array([A[m + l, p * p + p + q] for m, p, q, _ in ents])
        ref = np.array([v for *_, v in ents])
        assert np.abs(got - ref).max() <= FP64_TOL * np.abs(ref).max()


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_mid_sampled_rotations(mid_case, prec, tol):
    wl, f, h, idx, ref = mid_case
    announce(f"mid sampled {prec}")
    plan = api.Plan(api.desc_for(wl, precision=prec))
    g = plan.forward(dev(f), dev(h))
    got = gather_rho(g, idx)
    del g
    torch.cuda.empty_cache()
    errs = per_l_rel_err(got, ref, wl.l_lo, wl.l_hi, axis=1)
    assert max(errs.values()) <= tol, errs


def test_mid_real_pair_flag(mid_case):
    wl, f, h, idx, ref = mid_case
    announce("mid real-pair")
    plan = api.Plan(api.desc_for(wl, real_pair=True))
    g = plan.forward(dev(f), dev(h))
    got = gather_rho(g, idx)
    del g
    torch.cuda.empty_cache()
    errs = per_l_rel_err(got, ref, wl.l_lo, wl.l_hi, axis=1)
    assert max(errs.values()) <= FP64_TOL, errs


def test_theta_window_is_a_slice_of_the_full_grid():
    wl = workload("tiny")
    f, h = make_inputs(wl)
    announce("theta window")
    full = api.Plan(api.desc_for(wl)).forward(dev(f), dev(h))
    for lo, hi in [(0, 1), (3, 11), (10, 11), (2, 9)]:
        part = api.Plan(api.desc_for(wl, theta_lo=lo, theta_hi=hi)).forward(dev(f), dev(h))
        assert torch.equal(part, full[:, :, lo:hi, :])


@pytest.mark.parametrize("case", [
    dict(L_f=6, L_h=1, l_lo=0, l_hi=6, n_phi=13, n_omega=1),          # scalar window
    dict(L_f=6, L_h=3, l_lo=7, l_hi=8, n_phi=17, n_omega=5),          # top degree only
    dict(L_f=5, L_h=3, l_lo=0, l_hi=7, n_phi=15, n_omega=4),          # even n_omega
    dict(L_f=4, L_h=2, l_lo=0, l_hi=5, n_phi=1, n_omega=3),           # one phi, beta=0 only
    dict(L_f=9, L_h=6, l_lo=2, l_hi=14, n_phi=29, n_omega=11),        # ragged theta tiles
    dict(L_f=5, L_h=12, l_lo=3, l_hi=6, n_phi=33, n_omega=23),        # L_h > L_f, bucket 16
])
@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_edge_cases_whole_grid(case, prec, tol):
    announce(f"edge {case} {prec}")
    f, h, g, ref = _full_case(**case, prec=prec, seed=31)
    errs = per_l_rel_err(g, ref, case["l_lo"], case["l_hi"])
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_largest_window_band_limit(prec, tol):
    """L_h = 32 (the largest supported), small signal, theta rows 5..8, sampled rotations."""
    announce(f"L_h=32 {prec}")
    rng = np.random.default_rng(3)
    L_f, L_h, l_lo, l_hi, n_phi, n_omega = 4, 32, 28, 34, 69, 63
    f = draw_coefficients(rng, L_f, 0.0)
    h = draw_window(rng, L_h)
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, 35, n_omega, precision=prec,
                                  theta_lo=5, theta_hi=9))
    g = plan.forward(dev(f), dev(h))
    idx = np.stack([rng.integers(0, n_phi, 200), rng.integers(5, 9, 200),
                    rng.integers(0, n_omega, 200)], 1)
    ref = oracle_g_grid(f, h, L_f, L_h, l_lo, l_hi, n_phi, 35, n_omega, idx)
    idx_local = idx.copy()
    idx_local[:, 1] -= 5
    got = gather_rho(g, idx_local)
    errs = per_l_rel_err(got, ref, l_lo, l_hi, axis=1)
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("L_h", [16, 20, 24])
@pytest.mark.parametrize("prec,tol,pair", [("fp64", FP64_TOL, False), ("fp64", FP64_TOL, True),
                                           ("fp32", FP32_TOL, True)])
def test_matrix_core_phi_stage_sampled(L_h, prec, tol, pair):
    """L_h >= 16 runs the phi stage on MFMA: 151 phi samples give two 64-slot units, the
    second partial; real pair writes the m < 0 rows from the transposed fragments."""
    announce(f"MFMA phi stage L_h={L_h} {prec} pair={pair}")
    rng = np.random.default_rng(17)
    L_f, l_lo, l_hi, n_phi, n_omega = 6, 14, 17, 151, 7
    f = draw_coefficients(rng, L_f, 0.0)
    h = draw_window(rng, L_h)
    n_theta = (n_phi + 1) // 2
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision=prec,
                                  real_pair=pair))
    g = plan.forward(dev(f), dev(h))
    idx = np.stack([rng.integers(0, n_phi, 160), rng.integers(0, n_theta, 160),
                    rng.integers(0, n_omega, 160)], 1)
    idx[0] = (0, 0, 0)
    idx[1] = (n_phi - 1, n_theta - 1, n_omega - 1)
    idx[2] = (75, n_theta - 1, 3)
    ref = oracle_g_grid(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, idx)
    errs = per_l_rel_err(gather_rho(g, idx), ref, l_lo, l_hi, axis=1)
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("L_h,prec,tol", [(8, "fp64", FP64_TOL), (8, "fp32", FP32_TOL),
                                          (20, "fp64", FP64_TOL), (20, "fp32", FP32_TOL)])
def test_largest_phi_grid_sampled(L_h, prec, tol):
    """n_phi = 2047, the largest supported: 1024 phi slots (several slot chunks per lane in
    the VALU phi stage, sixteen 64-slot units in the MFMA one), on a ragged 3-row theta
    slice in the middle of the 1024 theta rows; sampled rotations against the oracle."""
    announce(f"largest phi grid L_h={L_h} {prec}")
    rng = np.random.default_rng(18)
    L_f, l_lo, l_hi, n_phi, n_omega = 7, 5, 9, 2047, 9
    n_theta, tlo, thi = 1024, 511, 514
    f = draw_coefficients(rng, L_f)
    h = draw_window(rng, L_h)
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision=prec,
                                  theta_lo=tlo, theta_hi=thi))
    g = plan.forward(dev(f), dev(h))
    idx = np.stack([rng.integers(0, n_phi, 200), rng.integers(0, thi - tlo, 200),
                    rng.integers(0, n_omega, 200)], 1)
    idx[0] = (0, 0, 0)
    idx[1] = (n_phi - 1, thi - tlo - 1, n_omega - 1)
    idx[2] = (1023, 1, 4)
    idx[3] = (1024, 2, 8)
    ref = oracle_g_grid(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega,
                        idx + np.array([0, tlo, 0]))
    errs = per_l_rel_err(gather_rho(g, idx), ref, l_lo, l_hi, axis=1)
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
@pytest.mark.parametrize("case", [
    dict(L_f=7, L_h=20, l_lo=0, l_hi=9, n_phi=45, n_omega=39),                  # staged path
    dict(L_f=6, L_h=18, l_lo=2, l_hi=8, n_phi=35, n_omega=5, n_az=3),           # steerable
    dict(L_f=5, L_h=17, l_lo=0, l_hi=6, n_phi=33, n_omega=33, real_pair=True),  # L_h = 17
])
def test_wu_synthesis_whole_grid(case, prec, tol):
    """Band-limits above 16 take the W/U path (W table, U GEMM over the items and phi stage
    in one kernel, the P|M rows in LDS): whole grid against the oracle, with a steerable
    window and with the real-pair path."""
    announce(f"W/U whole grid {case} {prec}")
    f, h, g, ref = _full_case(**case, prec=prec, seed=41)
    errs = per_l_rel_err(g, ref, case["l_lo"], case["l_hi"])
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_wu_synthesis_theta_runs_sampled(prec, tol):
    """L_f = 64, L_h = 32, l in [80, 95) (2625 items, 191 x 96 x 63 grid) on the W/U path:
    enough item tiles that each W/U block loops over a run of theta rows (15 FP32, 31 FP64)
    and the tiles spread over every XCD's run; seeded rotations against the oracle,
    including the first and the last grid point."""
    announce(f"W/U theta runs {prec}")
    rng = np.random.default_rng(43)
    L_f, L_h, l_lo, l_hi, n_phi, n_omega = 64, 32, 80, 95, 191, 63
    n_theta = (n_phi + 1) // 2
    f = draw_coefficients(rng, L_f, 2.0, True)
    h = draw_window(rng, L_h)
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision=prec))
    g = plan.forward(dev(f), dev(h))
    idx = np.stack([rng.integers(0, n_phi, 24), rng.integers(0, n_theta, 24),
                    rng.integers(0, n_omega, 24)], 1)
    idx[0] = (0, 0, 0)
    idx[1] = (n_phi - 1, n_theta - 1, n_omega - 1)
    ref = oracle_g_grid(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, idx)
    errs = per_l_rel_err(gather_rho(g, idx), ref, l_lo, l_hi, axis=1)
    del g
    torch.cuda.empty_cache()
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_minimal_grid_all_degrees_sampled(prec, tol):
    """The paper's timing setting (Section V) at L_f = 66: L_h = 18, every l < L_f + 17
    (6889 items), the minimal grid 35 x 18 x 35; the W/U blocks take runs of theta rows.
    Seeded rotations against the oracle."""
    announce(f"minimal grid L_f=66 {prec}")
    rng = np.random.default_rng(47)
    L_f, L_h = 66, 18
    K = 2 * L_h - 1
    f = draw_coefficients(rng, L_f, 2.0, True)
    h = draw_window(rng, L_h)
    plan = api.Plan(api.make_desc(L_f, L_h, 0, L_f + L_h - 1, K, L_h, K, precision=prec))
    g = plan.forward(dev(f), dev(h))
    idx = np.stack([rng.integers(0, K, 24), rng.integers(0, L_h, 24), rng.integers(0, K, 24)], 1)
    idx[0] = (0, 0, 0)
    idx[1] = (K - 1, L_h - 1, K - 1)
    ref = oracle_g_grid(f, h, L_f, L_h, 0, L_f + L_h - 1, K, L_h, K, idx)
    errs = per_l_rel_err(gather_rho(g, idx), ref, 0, L_f + L_h - 1, axis=1)
    del g
    torch.cuda.empty_cache()
    assert max(errs.values()) <= tol, errs

"""Steerable windows (azimuthal band-limit n_az < L_h; remark on steerable windows,
Section IV-B): the theta and omega contractions run over |q'| < n_az only.

Pins: the steerable plan equals, bit for bit, the general plan run on the same
window (the skipped terms are exact zeros); it matches the FP64 oracle on the whole
grid; g sampled at 2 n_az - 1 orientations omega_c determines g at any other omega
(trigonometric interpolation with |q'| < n_az), the property the paper points out;
the inverse works from those 2 n_az - 1 samples; the mid-size steerable workload
(L_f=128, L_h=8, n_az=3, l in [32,48), 271x136x5 grid) matches the oracle on a seeded
sample of rotations, in the launch configuration the benchmark times.
"""
import numpy as np
import pytest

from oracle.slsht import oracle_g_full, oracle_g_grid
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import (draw_coefficients, draw_window, make_inputs,
                                        rho_subset, workload)
from tests.gpu_util import (FP32_TOL, FP64_TOL, announce, dev, gather_rho, max_rel, need_gpu,
                            per_l_rel_err)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _inputs(L_f, L_h, n_az, seed):
    rng = np.random.default_rng(seed)
    return draw_coefficients(rng, L_f, 0.0), draw_window(rng, L_h, n_az=n_az)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("pair", [False, True])
@pytest.mark.parametrize("n_az", [1, 2, 5])
def test_steerable_plan_equals_general_plan(prec, pair, n_az):
    announce(f"steerable == general {prec} pair={pair} n_az={n_az}")
    L_f, L_h, l_lo, l_hi, n_phi, n_omega = 11, 6, 2, 14, 35, 7
    f, h = _inputs(L_f, L_h, n_az, 31)
    out = []
    for az in (n_az, 0):
        plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, (n_phi + 1) // 2, n_omega,
                                      precision=prec, real_pair=pair, n_az=az))
        out.append(plan.forward(dev(f), dev(h)).cpu().numpy())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("n_az", [2, 4])
def test_steerable_energy_equals_general_plan(n_az):
    announce(f"steerable energy n_az={n_az}")
    L_f, L_h, l_lo, l_hi, n_phi, n_omega = 9, 5, 3, 12, 29, 9
    f, h = _inputs(L_f, L_h, n_az, 32)
    out = []
    for az in (n_az, 0):
        plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, (n_phi + 1) // 2, n_omega,
                                      precision="fp32", output="energy", n_az=az))
        out.append(plan.forward(dev(f), dev(h)).cpu().numpy())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_steerable_whole_grid_vs_oracle(prec, tol):
    announce(f"steerable whole grid {prec}")
    L_f, L_h, n_az, l_lo, l_hi, n_phi = 9, 6, 2, 3, 12, 31
    n_omega, n_theta = 2 * n_az - 1, (n_phi + 1) // 2
    f, h = _inputs(L_f, L_h, n_az, 33)
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega,
                                  precision=prec, n_az=n_az))
    g = plan.forward(dev(f), dev(h)).cpu().numpy()
    ref = oracle_g_full(f, h, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega)
    errs = per_l_rel_err(g, ref, l_lo, l_hi)
    assert max(errs.values()) <= tol, errs


def test_basis_orientations_determine_every_omega():
    """g on 2 n_az - 1 orientations -> g on 7 others by trigonometric interpolation."""
    announce("steerable omega interpolation")
    L_f, L_h, n_az, l_lo, l_hi, n_phi = 10, 7, 3, 4, 12, 27
    n_theta = (n_phi + 1) // 2
    f, h = _inputs(L_f, L_h, n_az, 34)
    M, M2 = 2 * n_az - 1, 7
    gA = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, M, n_az=n_az)).forward(
        dev(f), dev(h)).cpu().numpy()                                   # [lm][c][b][a]
    gB = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, M2, n_az=n_az)).forward(
        dev(f), dev(h)).cpu().numpy()
    om = 2 * np.pi * np.arange(M) / M
    om2 = 2 * np.pi * np.arange(M2) / M2
    k = np.arange(-(n_az - 1), n_az)
    # g(gamma) = sum_{|k| < n_az} c_k e^{-i k gamma}; c_k from the M samples
    D = np.exp(-1j * np.outer(om2, k)) @ np.exp(1j * np.outer(k, om)) / M   # [M2, M]
    interp = np.einsum("dc,lcba->ldba", D, gA)
    assert max_rel(interp, gB) <= FP64_TOL


def test_steerable_inverse_from_basis_orientations():
    announce("steerable inverse")
    L_f, L_h, n_az, n_phi = 8, 6, 2, 27
    l_lo, l_hi = 0, L_f + L_h - 1
    n_theta, n_omega = (n_phi + 1) // 2, 2 * n_az - 1
    f, h = _inputs(L_f, L_h, n_az, 35)
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, n_az=n_az))
    g = plan.forward(dev(f), dev(h))
    fr = plan.inverse(g, dev(h)).cpu().numpy()
    want = np.zeros(l_hi * l_hi, dtype=np.complex128)
    want[:L_f * L_f] = f
    assert np.abs(fr - want).max() <= 1e-12 * np.abs(f).max()


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_mid_steer_sampled_rotations(prec, tol):
    wl = workload("mid_steer")
    announce(f"mid_steer sampled {prec}")
    f, h = make_inputs(wl)
    idx = rho_subset(wl, 200, seed=77)
    ref = oracle_g_grid(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta,
                        wl.n_omega, idx)
    plan = api.Plan(api.desc_for(wl, precision=prec))
    g = gather_rho(plan.forward(dev(f), dev(h)), idx)
    errs = per_l_rel_err(g, ref, wl.l_lo, wl.l_hi, axis=1)
    assert max(errs.values()) <= tol, errs

"""The synthesis stage alone (slsht_synthesize) from a random coupling, against the
function on SO(3) that the coupling and window define.

With A^p_q(l, m) arbitrary (not the coupling of any signal), the synthesis must still
return g(rho) = sum_{p,q,q'} A^p_q h_p^{q'} D^p_{q,q'}(rho) (the harmonic formulation,
Eq:harmonic_formulation, written as an SO(3) expansion): checked on the whole grid
against the oracle's synthesis, by the oracle's Wigner-D analysis of the GPU output
(which must return A h, Eq:WignerD_ortho made discrete by the inverse's weights), and on
the beta = 0 row against sum_q (sum_p A^p_q h_p^q) e^{-i q (alpha + gamma)}.  This covers
every synthesis form: the VALU form (L_h <= 8), the MFMA phi form (L_h = 12, 16, 24) and
the staged form with the W table and the U GEMM (L_h = 17).
"""
import numpy as np
import pytest

from oracle import grid as og
from oracle.so3 import coupling_window_coefficients, so3_analysis, so3_synthesis
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_window, grid_dims
from tests.gpu_util import FP32_TOL, FP64_TOL, announce, dev, need_gpu, per_l_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


CASES = [(4, "fp64"), (8, "fp64"), (12, "fp64"), (16, "fp64"), (17, "fp64"), (24, "fp64"),
         (8, "fp32"), (16, "fp32"), (17, "fp32")]


@pytest.mark.parametrize("L_h,precision", CASES)
def test_random_coupling_synthesis(L_h, precision):
    L_f, l_lo, l_hi = max(16, L_h), 10, 12   # (n_phi - 1)/2 = L_f + L_h - 1 >= 2 L_h - 2
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h)
    announce(f"synthesis from a random coupling L_h={L_h} {precision} "
             f"grid {n_phi}x{n_theta}x{n_omega}")
    rng = np.random.default_rng(100 + L_h)
    plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega,
                                  precision=precision))
    rows = l_hi * l_hi - l_lo * l_lo
    A = rng.standard_normal((rows, L_h * L_h)) + 1j * rng.standard_normal((rows, L_h * L_h))
    h = draw_window(rng, L_h)
    g = plan.synthesize(dev(A), dev(h)).cpu().numpy().reshape(rows, n_omega, n_theta, n_phi)
    G = coupling_window_coefficients(A, h, L_h)
    ref = so3_synthesis(G, L_h, n_phi, n_theta, n_omega)
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    errs = per_l_rel_err(g, ref, l_lo, l_hi)
    assert max(errs.values()) <= tol, errs
    # the Wigner-D analysis of the GPU output returns the coefficients A h
    back = so3_analysis(g, L_h, n_phi, n_theta, n_omega)
    assert np.linalg.norm(back - G) / np.linalg.norm(G) <= 10 * tol
    # beta = 0: a function of alpha + gamma only
    diag = np.zeros((rows, 2 * L_h - 1), dtype=np.complex128)
    for p in range(L_h):
        for q in range(-p, p + 1):
            diag[:, q + L_h - 1] += G[:, p * p + p + q, q + L_h - 1]
    qq = np.arange(-(L_h - 1), L_h)
    s = og.alpha_angles(n_phi)[None, :] + og.gamma_angles(n_omega)[:, None]
    closed = np.einsum("kq,qca->kca", diag, np.exp(-1j * qq[:, None, None] * s[None]))
    assert np.linalg.norm(g[:, :, 0, :] - closed) / np.linalg.norm(closed) <= tol

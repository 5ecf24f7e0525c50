"""slsht_forward_noalloc (static device scratch, no allocation in the call) against
slsht_forward on the same plans: two calls in a row, the second on a smaller
transform, so that the second runs over the scratch contents the first left behind."""
import ctypes

import numpy as np
import pytest

from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window, grid_dims
from tests.gpu_util import FP32_TOL, FP64_TOL, announce, dev, need_gpu, per_l_rel_err, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _case(seed, L_f, L_h, l_lo, l_hi, prec, output="full", real_pair=False):
    rng = np.random.default_rng(seed)
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h)
    f = draw_coefficients(rng, L_f, 2.0, True)
    h = draw_window(rng, L_h)
    desc = api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision=prec,
                         output=output, real_pair=real_pair)
    return api.Plan(desc), dev(f), dev(h)


def _compare(plan, ft, ht, prec, output):
    ref = plan.forward(ft, ht)
    got = plan.empty_output()
    got.fill_(float("nan"))
    plan.forward_noalloc(ft, ht, got)
    torch.cuda.synchronize()
    d = plan.desc
    if output == "full":
        errs = per_l_rel_err(got.cpu().numpy(), ref.cpu().numpy(), d.l_lo, d.l_hi)
    else:
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        errs = {l: float(np.linalg.norm(g[i] - r[i]) / np.linalg.norm(r[i]))
                for i, l in enumerate(range(d.l_lo, d.l_hi))}
    tol = FP64_TOL if prec == "fp64" else FP32_TOL
    assert max(errs.values()) <= tol, errs
    return got, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_equals_forward_two_calls(prec):
    announce(f"noalloc {prec}: large then small")
    big = _case(11, 40, 8, 10, 30, prec)
    small = _case(12, 12, 4, 0, 9, prec)
    for plan, ft, ht in (big, small):
        _compare(plan, ft, ht, prec, "full")


def test_noalloc_energy_and_real_pair():
    announce("noalloc energy then real-pair full")
    e = _case(13, 24, 8, 4, 12, "fp32", output="energy")
    _compare(*e, "fp32", "energy")
    r = _case(14, 16, 6, 2, 8, "fp64", real_pair=True)
    _compare(*r, "fp64", "full")


def test_noalloc_rejects_oversized_scratch():
    announce("noalloc size check")
    # (l_hi^2 - l_lo^2) * L_h^2 * 16 bytes = 66^2 * 1024 * 16, above 64 MiB
    desc = api.make_desc(600, 32, 0, 66, 63, 32, 63, precision="fp64")
    d = L.Desc.from_buffer_copy(desc)
    need = L.lib().slsht_coupling_size(ctypes.byref(d)) * 16
    assert need > (64 << 20)
    plan = api.Plan(desc)
    t = torch.empty(1, dtype=torch.complex128, device="cuda:0")
    st = L.lib().slsht_forward_noalloc(plan._h, ctypes.c_void_p(t.data_ptr()),
                                       ctypes.c_void_p(t.data_ptr()),
                                       ctypes.c_void_p(t.data_ptr()), None)
    assert st == L.SLSHT_ETOOBIG
    assert "static scratch" in L.last_error()

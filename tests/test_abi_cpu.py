"""Host-only checks of the C ABI: the library loads, exports every function that
include/slsht.h declares, and its descriptor checks and footprints behave as
documented.  No compute call is made (no GPU needed)."""
import ctypes
import os

import pytest

from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import WORKLOADS, workload


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1207_5558_amd import build
        build.build()
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = L.declared_functions()
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(L._SIGNATURES), "binding and header disagree"


def _desc(**kw):
    base = dict(L_f=8, L_h=3, l_lo=0, l_hi=8, n_phi=21, n_theta=11, n_omega=5)
    base.update(kw)
    return api.make_desc(**base)


def test_valid_workloads(lib):
    for wl in WORKLOADS.values():
        api.validate(api.desc_for(wl))


@pytest.mark.parametrize("kw,msg", [
    (dict(L_f=0), "L_f"),
    (dict(L_h=33), "L_h"),
    (dict(l_lo=5, l_hi=5), "l_lo"),
    (dict(l_hi=11), "l_hi"),
    (dict(n_phi=20, n_theta=10), "odd"),
    (dict(n_theta=10), "n_theta"),
    (dict(n_omega=0), "n_omega"),
    (dict(precision="fp64", theta_lo=4, theta_hi=3), "theta"),
    (dict(theta_hi=12), "theta"),
])
def test_invalid_descriptors(lib, kw, msg):
    d = _desc(**kw)
    rc = lib.slsht_validate(ctypes.byref(d))
    assert rc == L.SLSHT_EINVAL
    assert msg in L.last_error()


def test_bad_enums_and_flags(lib):
    d = _desc()
    d.precision = 7
    assert lib.slsht_validate(ctypes.byref(d)) == L.SLSHT_EINVAL
    d = _desc()
    d.output_mode = 3
    assert lib.slsht_validate(ctypes.byref(d)) == L.SLSHT_EINVAL
    d = _desc()
    d.flags = 6
    assert lib.slsht_validate(ctypes.byref(d)) == L.SLSHT_EINVAL
    assert lib.slsht_validate(None) == L.SLSHT_EINVAL


def test_footprints_match_layouts(lib):
    wl = workload("mid")
    plan_b, out_b, scr = api.footprint(api.desc_for(wl))
    assert out_b == wl.samples * 16                  # complex128 FULL
    wl3 = workload("mid_fp32")
    assert api.footprint(api.desc_for(wl3))[1] == wl.samples * 8
    wl5 = workload("large")
    n_l = wl5.l_hi - wl5.l_lo
    assert api.footprint(api.desc_for(wl5))[1] == n_l * wl5.n_rho * 4   # float energy
    # the plan holds the canonical d table (136 rows x 204 entries of FP64: p < 8,
    # 0 <= Q <= p, |Q'| <= Q) plus small tables
    assert plan_b >= 136 * 204 * 8
    assert scr == 0
    d = _desc(theta_lo=2, theta_hi=5)
    assert api.footprint(d)[1] == 64 * 5 * 3 * 21 * 16


def test_steerable_window_rules(lib):
    """n_az (azimuthal band-limit of the window) must lie in [0, L_h]."""
    for az, ok in ((0, True), (1, True), (3, True), (-1, False), (4, False)):
        d = _desc()
        d.n_az = az
        assert (lib.slsht_validate(ctypes.byref(d)) == L.SLSHT_OK) == ok, az
    assert ctypes.sizeof(L.Desc) == 13 * 4


def test_slepian_window_argument_checks(lib):
    """Rejected on the host before any GPU work: 0 <= theta_c < a <= pi/2, 1 <= L_h <= 32."""
    import numpy as np
    h = np.zeros(64, dtype=np.complex128)
    c = ctypes.c_double()
    for L_h, tc, a in ((8, 0.5, 0.5), (8, -0.1, 0.5), (8, 0.2, 2.0), (0, 0.1, 0.5),
                       (33, 0.1, 0.5), (8, float("nan"), 0.5)):
        assert lib.slsht_slepian_window(L_h, tc, a, 0, h.ctypes.data,
                                        ctypes.byref(c)) == L.SLSHT_EINVAL, (L_h, tc, a)
    assert lib.slsht_slepian_window(8, 0.1, 0.5, 0, None, None) == L.SLSHT_EINVAL


def test_factored_route_workspace(lib):
    """Host-only eligibility and size of the factoring-of-rotations workspace."""
    d = api.make_desc(8, 3, 0, 10, 5, 3, 5)                      # minimal grid, K = 5
    n_lm, L_h, K, row = 100, 3, 5, 3 * 4 * 7 // 6
    up = lambda b: (b + 255) // 256 * 256
    want = up(row * 8) + up(L_h * K * K * 16) + n_lm * K * L_h * K * 16
    assert lib.slsht_factored_workspace(ctypes.byref(d)) == want
    for bad in (api.make_desc(8, 3, 0, 10, 21, 11, 5),          # not the minimal grid
                api.make_desc(8, 3, 0, 10, 5, 3, 5, precision="fp32"),
                api.make_desc(8, 3, 0, 10, 5, 3, 5, real_pair=True),
                api.make_desc(8, 3, 0, 10, 5, 3, 5, theta_lo=1)):
        assert lib.slsht_factored_workspace(ctypes.byref(bad)) == -1


def test_modulated_route_workspace_and_checks(lib):
    """Workspace of the modulated-signal coupling: nodes, weights, F and two Legendre
    tables, each padded to 256 bytes; argument checks return before any GPU work."""
    up = lambda b: (b + 255) // 256 * 256
    L_f, L_h, l_lo, l_hi = 8, 3, 2, 10
    d = api.make_desc(L_f, L_h, l_lo, l_hi, 21, 11, 5)
    n = ((L_f - 1) + (l_hi - 1) + (L_h - 1)) // 2 + 1
    nW = l_hi * (l_hi + 1) // 2 - l_lo * (l_lo + 1) // 2
    want = (2 * up(n * 8) + up(n * (2 * L_f - 1) * 16) + up(n * nW * 8)
            + up(n * (L_h * (L_h + 1) // 2) * 8))
    assert lib.slsht_modulated_workspace(ctypes.byref(d)) == want
    assert lib.slsht_modulated_workspace(ctypes.byref(_desc(L_h=0))) == -1
    assert lib.slsht_modulated_workspace(None) == -1
    assert lib.slsht_coupling_modulated(None, None, None, None, 0, None) == L.SLSHT_EINVAL
    assert lib.slsht_synthesize_factored(None, None, None, None, None, 0, None) == L.SLSHT_EINVAL
    buf = ctypes.create_string_buffer(16)
    for L_h in (0, 33, -1):
        assert lib.slsht_wigner_delta(L_h, 0, buf, None) == L.SLSHT_EINVAL
    assert lib.slsht_wigner_delta(4, 0, None, None) == L.SLSHT_EINVAL


def test_forward_batch_argument_checks(lib):
    """Rejected on the host before any GPU work."""
    arr = (ctypes.c_void_p * 1)(None)
    assert lib.slsht_forward_batch(0, arr, arr, arr, arr, None) == L.SLSHT_EINVAL
    assert lib.slsht_forward_batch(1, None, arr, arr, arr, None) == L.SLSHT_EINVAL
    assert lib.slsht_forward_batch(1, arr, arr, arr, arr, None) == L.SLSHT_EINVAL


def test_coupling_size(lib):
    d = api.desc_for(workload("mid"))
    assert lib.slsht_coupling_size(ctypes.byref(d)) == 1280 * 64
    assert lib.slsht_coupling_size(None) == -1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        L.lib()


def test_energy_descriptor_rules(lib):
    for kw, msg in [(dict(precision="fp64"), "FP32"), (dict(n_omega=65), "n_omega"),
                    (dict(n_phi=1089, n_theta=545, n_omega=63), "n_phi")]:
        d = _desc(output="energy", **{"precision": "fp32", **kw})
        assert lib.slsht_validate(ctypes.byref(d)) == L.SLSHT_EINVAL
        assert msg in L.last_error()
    assert lib.slsht_validate(ctypes.byref(_desc(output="energy", precision="fp32",
                                                 n_phi=1087, n_theta=544, n_omega=64))) == 0

"""The library used from plain C (tests/native/abi_forward, built by
__graft_entry__.build()): plan, forward and inverse through include/slsht.h with device
buffers from the HIP runtime, no Python binding involved; its output must match the
oracle on the whole tiny grid and its inverse must return the signal."""
import os
import subprocess

import numpy as np
import pytest

from oracle.slsht import oracle_g_full
from paper_1207_5558_amd.inputs import make_inputs, workload
from tests.gpu_util import FP64_TOL, announce, need_gpu, per_l_rel_err

pytestmark = pytest.mark.gpu
EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "abi_forward")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.skipif(not os.path.exists(EXE), reason="tests/native/abi_forward not built "
                    "(__graft_entry__.build() builds it where gcc is available)")
def test_plain_c_forward_and_inverse(tmp_path):
    announce("plain C consumer")
    wl = workload("tiny")
    f, h = make_inputs(wl)
    inp, gout, fout = tmp_path / "in.bin", tmp_path / "g.bin", tmp_path / "f.bin"
    with open(inp, "wb") as fp:
        fp.write(np.ascontiguousarray(f, dtype=np.complex128).tobytes())
        fp.write(np.ascontiguousarray(h, dtype=np.complex128).tobytes())
    res = subprocess.run([EXE, str(inp), str(gout), str(fout)], capture_output=True, text=True,
                         timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    n_lm = wl.l_hi ** 2 - wl.l_lo ** 2
    g = np.fromfile(gout, dtype=np.complex128).reshape(n_lm, wl.n_omega, wl.n_theta, wl.n_phi)
    ref = oracle_g_full(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta, wl.n_omega)
    assert max(per_l_rel_err(g, ref, wl.l_lo, wl.l_hi).values()) <= FP64_TOL
    fo = np.fromfile(fout, dtype=np.complex128)
    assert np.abs(fo[:wl.L_f ** 2] - f[:wl.L_f ** 2]).max() <= 1e-12 * np.abs(f).max()

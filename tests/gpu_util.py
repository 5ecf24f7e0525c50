"""Shared helpers of the GPU tests (parity metrics, device tensors)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

FP64_TOL = 1e-12     # relative Frobenius error per degree, FP64 path vs FP64 oracle
FP32_TOL = 1e-5      # same, FP32-mixed path vs FP64 oracle


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1207_5558_amd import _lib
    _lib.lib()          # raises if the library is not built: the native path must run


def dev(x: np.ndarray, device="cuda:0"):
    return torch.from_numpy(np.ascontiguousarray(x)).to(device)


def announce(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def per_l_rel_err(got: np.ndarray, ref: np.ndarray, l_lo: int, l_hi: int, axis: int = 0):
    """Relative Frobenius error per degree; `axis` of the arrays indexes lm."""
    got = np.moveaxis(got, axis, 0)
    ref = np.moveaxis(ref, axis, 0)
    out = {}
    for l in range(l_lo, l_hi):
        s = l * l - l_lo * l_lo
        d = got[s:s + 2 * l + 1] - ref[s:s + 2 * l + 1]
        nr = np.linalg.norm(ref[s:s + 2 * l + 1])
        out[l] = float(np.linalg.norm(d) / nr) if nr > 0 else float(np.linalg.norm(d))
    return out


def max_rel(got, ref) -> float:
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def gather_rho(g_t, idx: np.ndarray):
    """g[lm][c][b][a] on the device -> numpy [rho, lm] at rho indices idx[k] = (a, b, c)."""
    a = torch.as_tensor(idx[:, 0], device=g_t.device)
    b = torch.as_tensor(idx[:, 1], device=g_t.device)
    c = torch.as_tensor(idx[:, 2], device=g_t.device)
    return g_t[:, c, b, a].transpose(0, 1).cpu().numpy()

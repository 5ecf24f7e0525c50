"""PyTorch-facing wrapper of the C ABI.

PyTorch supplies device memory and streams; the transform itself runs in the
library's kernels.  Coefficient tensors are complex128 at flat index
l*l + l + m (exclusive band-limits); output layouts are those of slsht.h.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib as L

_PREC = {"fp64": L.SLSHT_FP64, "fp32": L.SLSHT_FP32_MIXED}
_MODE = {"full": L.SLSHT_OUT_FULL, "energy": L.SLSHT_OUT_ENERGY}


def make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, precision="fp64", output="full",
              real_pair=False, theta_lo=0, theta_hi=0, n_az=0) -> L.Desc:
    return L.Desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, _PREC[precision],
                  _MODE[output], L.SLSHT_REAL_PAIR if real_pair else 0, theta_lo, theta_hi,
                  n_az)


def desc_for(wl, **over) -> L.Desc:
    """Descriptor of a workload from paper_1207_5558_amd.inputs."""
    kw = dict(precision=wl.precision, output=wl.output, n_az=wl.n_az)
    kw.update(over)
    return make_desc(wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta, wl.n_omega, **kw)


def slepian_window(L_h: int, theta_c: float, a: float, device: int = 0):
    """(h, concentration): the Slepian window of band-limit L_h most concentrated in the
    elliptical region R_(theta_c, a), as a host complex128 array [L_h^2]."""
    import numpy as np
    h = np.zeros(L_h * L_h, dtype=np.complex128)
    c = ctypes.c_double()
    L.check(L.lib().slsht_slepian_window(L_h, theta_c, a, device, h.ctypes.data,
                                         ctypes.byref(c)))
    return h, c.value


def factored_workspace(desc: L.Desc) -> int:
    """Bytes of device workspace slsht_forward_factored needs for desc (raises if desc is
    not eligible for the factoring-of-rotations route)."""
    need = L.lib().slsht_factored_workspace(ctypes.byref(desc))
    if need < 0:
        raise L.SlshtError(L.SLSHT_EINVAL, L.last_error())
    return need


def modulated_workspace(desc: L.Desc) -> int:
    """Bytes of device workspace slsht_coupling_modulated needs for desc."""
    need = L.lib().slsht_modulated_workspace(ctypes.byref(desc))
    if need < 0:
        raise L.SlshtError(L.SLSHT_EINVAL, L.last_error())
    return need


def wigner_delta(L_h: int, device: int = 0, stream=None):
    """Delta^p = d^p(pi/2), p < L_h, canonical layout (float64 device tensor of
    L_h (L_h+1)(2 L_h+1)/6 entries, p(p+1)(2p+1)/6 + Q^2 + Q + Q' for 0 <= Q <= p)."""
    n = L_h * (L_h + 1) * (2 * L_h + 1) // 6
    out = torch.empty(n, dtype=torch.float64, device=f"cuda:{device}")
    L.check(L.lib().slsht_wigner_delta(L_h, device, _dev_ptr(out, torch.float64, n, "delta"),
                                       _stream_handle(stream)))
    return out


def forward_batch(plans, fs, hs, gs=None, stream=None):
    """Forward transforms of several distinct plans in few launches (slsht_forward_batch);
    returns the outputs (allocated if gs is None)."""
    n = len(plans)
    if not (len(fs) == len(hs) == n) or (gs is not None and len(gs) != n):
        raise ValueError("plans, fs, hs (and gs) must have equal lengths")
    if gs is None:
        gs = [p.empty_output() for p in plans]
    def n_out(p):
        k = 1
        for s in p.output_shape:
            k *= s
        return k
    P = (ctypes.c_void_p * n)(*[p._h.value for p in plans])
    F = (ctypes.c_void_p * n)(*[_dev_ptr(f, torch.complex128, p.desc.L_f ** 2, "f").value
                                for p, f in zip(plans, fs)])
    H = (ctypes.c_void_p * n)(*[_dev_ptr(h, torch.complex128, p.desc.L_h ** 2, "h").value
                                for p, h in zip(plans, hs)])
    G = (ctypes.c_void_p * n)(*[_dev_ptr(g, p.output_dtype, n_out(p), "g").value
                                for p, g in zip(plans, gs)])
    L.check(L.lib().slsht_forward_batch(n, P, F, H, G, _stream_handle(stream)))
    return gs


def validate(desc: L.Desc) -> None:
    L.check(L.lib().slsht_validate(ctypes.byref(desc)))


def footprint(desc: L.Desc) -> tuple[int, int, int]:
    a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    L.check(L.lib().slsht_footprint(ctypes.byref(desc), ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)))
    return a.value, b.value, c.value


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype, numel, name) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Device plan for one descriptor (Wigner-d table, twiddles, weights)."""

    def __init__(self, desc: L.Desc, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        self.desc = L.Desc.from_buffer_copy(desc)
        h = ctypes.c_void_p()
        L.check(L.lib().slsht_plan(ctypes.byref(self.desc), device, ctypes.byref(h)))
        self._h = h
        d = self.desc
        self.n_theta_out = (d.theta_hi or d.n_theta) - d.theta_lo
        self.n_lm = d.l_hi * d.l_hi - d.l_lo * d.l_lo

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            L.check(L.lib().slsht_plan_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def output_shape(self) -> tuple[int, ...]:
        d = self.desc
        lead = self.n_lm if d.output_mode == L.SLSHT_OUT_FULL else d.l_hi - d.l_lo
        return (lead, d.n_omega, self.n_theta_out, d.n_phi)

    @property
    def output_dtype(self):
        d = self.desc
        if d.output_mode == L.SLSHT_OUT_FULL:
            return torch.complex128 if d.precision == L.SLSHT_FP64 else torch.complex64
        return torch.float64 if d.precision == L.SLSHT_FP64 else torch.float32

    def empty_output(self) -> torch.Tensor:
        return torch.empty(self.output_shape, dtype=self.output_dtype,
                           device=f"cuda:{self.device}")

    def forward(self, f: torch.Tensor, h: torch.Tensor, g: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
        d = self.desc
        if g is None:
            g = self.empty_output()
        pf = _dev_ptr(f, torch.complex128, d.L_f * d.L_f, "f")
        ph = _dev_ptr(h, torch.complex128, d.L_h * d.L_h, "h")
        n_out = 1
        for s in self.output_shape:
            n_out *= s
        pg = _dev_ptr(g, self.output_dtype, n_out, "g")
        L.check(L.lib().slsht_forward(self._h, pf, ph, pg, _stream_handle(stream)))
        return g

    def forward_noalloc(self, f: torch.Tensor, h: torch.Tensor, g: torch.Tensor,
                        stream=None) -> torch.Tensor:
        """slsht_forward_noalloc: the same transform with the library's static coupling
        scratch; g must be given (nothing is allocated)."""
        d = self.desc
        n_out = 1
        for s in self.output_shape:
            n_out *= s
        L.check(L.lib().slsht_forward_noalloc(
            self._h, _dev_ptr(f, torch.complex128, d.L_f * d.L_f, "f"),
            _dev_ptr(h, torch.complex128, d.L_h * d.L_h, "h"),
            _dev_ptr(g, self.output_dtype, n_out, "g"), _stream_handle(stream)))
        return g

    def coupling(self, f: torch.Tensor, A: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        d = self.desc
        n = self.n_lm * d.L_h * d.L_h
        if A is None:
            A = torch.empty((self.n_lm, d.L_h * d.L_h), dtype=torch.complex128,
                            device=f"cuda:{self.device}")
        L.check(L.lib().slsht_coupling(self._h, _dev_ptr(f, torch.complex128, d.L_f * d.L_f, "f"),
                                       _dev_ptr(A, torch.complex128, n, "A"),
                                       _stream_handle(stream)))
        return A

    def synthesize(self, A: torch.Tensor, h: torch.Tensor, g: torch.Tensor | None = None,
                   stream=None) -> torch.Tensor:
        """Synthesis stage alone from a coupling A (slsht_synthesize)."""
        d = self.desc
        if g is None:
            g = self.empty_output()
        n_out = 1
        for s in self.output_shape:
            n_out *= s
        L.check(L.lib().slsht_synthesize(
            self._h, _dev_ptr(A, torch.complex128, self.n_lm * d.L_h * d.L_h, "A"),
            _dev_ptr(h, torch.complex128, d.L_h * d.L_h, "h"),
            _dev_ptr(g, self.output_dtype, n_out, "g"), _stream_handle(stream)))
        return g

    def coupling_modulated(self, f: torch.Tensor, A: torch.Tensor | None = None,
                           work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """The coupling by the modulated-signal transform (the paper's Appendix A route);
        same result and layout as coupling()."""
        d = self.desc
        n = self.n_lm * d.L_h * d.L_h
        need = modulated_workspace(d)
        if A is None:
            A = torch.empty((self.n_lm, d.L_h * d.L_h), dtype=torch.complex128,
                            device=f"cuda:{self.device}")
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        L.check(L.lib().slsht_coupling_modulated(
            self._h, _dev_ptr(f, torch.complex128, d.L_f * d.L_f, "f"),
            _dev_ptr(A, torch.complex128, n, "A"), _dev_ptr(work, torch.uint8, need, "work"),
            work.numel(), _stream_handle(stream)))
        return A

    def forward_windows(self, f: torch.Tensor, h: torch.Tensor, g: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
        """One signal against W windows h[W, L_h^2]; returns g[W, *output_shape]."""
        d = self.desc
        if h.dim() != 2 or h.shape[1] != d.L_h * d.L_h:
            raise ValueError("h must be [n_windows, L_h^2]")
        W = h.shape[0]
        if g is None:
            g = torch.empty((W,) + tuple(self.output_shape), dtype=self.output_dtype,
                            device=f"cuda:{self.device}")
        n_out = W
        for s in self.output_shape:
            n_out *= s
        L.check(L.lib().slsht_forward_windows(
            self._h, _dev_ptr(f, torch.complex128, d.L_f * d.L_f, "f"),
            _dev_ptr(h, torch.complex128, W * d.L_h * d.L_h, "h"), W,
            _dev_ptr(g, self.output_dtype, n_out, "g"), _stream_handle(stream)))
        return g

    def forward_factored(self, f: torch.Tensor, h: torch.Tensor, g: torch.Tensor | None = None,
                         work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """The paper's factoring-of-rotations route (plans on the minimal grid only)."""
        d = self.desc
        need = factored_workspace(d)
        if g is None:
            g = self.empty_output()
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        n_out = 1
        for s in self.output_shape:
            n_out *= s
        L.check(L.lib().slsht_forward_factored(
            self._h, _dev_ptr(f, torch.complex128, d.L_f * d.L_f, "f"),
            _dev_ptr(h, torch.complex128, d.L_h * d.L_h, "h"),
            _dev_ptr(g, self.output_dtype, n_out, "g"),
            _dev_ptr(work, torch.uint8, need, "work"), need, _stream_handle(stream)))
        return g

    def synthesize_factored(self, A: torch.Tensor, h: torch.Tensor, g: torch.Tensor | None = None,
                            work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """The factored synthesis alone, from a coupling A[n_lm, L_h^2]."""
        d = self.desc
        need = factored_workspace(d)
        if g is None:
            g = self.empty_output()
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
        n_out = 1
        for s in self.output_shape:
            n_out *= s
        L.check(L.lib().slsht_synthesize_factored(
            self._h, _dev_ptr(A, torch.complex128, self.n_lm * d.L_h * d.L_h, "A"),
            _dev_ptr(h, torch.complex128, d.L_h * d.L_h, "h"),
            _dev_ptr(g, self.output_dtype, n_out, "g"),
            _dev_ptr(work, torch.uint8, need, "work"), work.numel(), _stream_handle(stream)))
        return g

    def inverse(self, g: torch.Tensor, h: torch.Tensor, f_out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
        d = self.desc
        if f_out is None:
            f_out = torch.empty(self.n_lm, dtype=torch.complex128, device=f"cuda:{self.device}")
        n_out = 1
        for s in self.output_shape:
            n_out *= s
        L.check(L.lib().slsht_inverse(self._h, _dev_ptr(g, self.output_dtype, n_out, "g"),
                                      _dev_ptr(h, torch.complex128, d.L_h * d.L_h, "h"),
                                      _dev_ptr(f_out, torch.complex128, self.n_lm, "f_out"),
                                      _stream_handle(stream)))
        return f_out

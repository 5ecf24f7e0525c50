"""Python side of the serving loop (continuous batching of forward transforms).

`Server` wraps slsht_server_* (argument marshalling only); `run_stream` plays a
list of timed requests against a server the way a client would: it submits each
request at its arrival time, polls for completions, optionally copies results
out, releases them, and reports per-request latency (arrival -> done).
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import _lib as L
from .api import make_desc

_hip = None


def _hip_memcpy(dst_ptr: int, src_ptr: int, nbytes: int, kind: int) -> None:
    """hipMemcpy through the HIP runtime (kind 2: device to host, 3: device to device)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), nbytes, kind)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")


def _hip_memcpy_d2h(dst: np.ndarray, src_ptr: int, nbytes: int) -> None:
    """Device-to-host copy of a server result."""
    _hip_memcpy(dst.ctypes.data, src_ptr, nbytes, 2)


class Server:
    def __init__(self, hbm_budget: int, n_streams: int = 4, device: int = 0):
        h = ctypes.c_void_p()
        L.check(L.lib().slsht_server_create(device, hbm_budget, n_streams, ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h and self._h.value:
            L.check(L.lib().slsht_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, desc: L.Desc, f: np.ndarray, h: np.ndarray) -> int:
        f = np.ascontiguousarray(f, dtype=np.complex128)
        h = np.ascontiguousarray(h, dtype=np.complex128)
        if f.size < desc.L_f * desc.L_f or h.size < desc.L_h * desc.L_h:
            raise ValueError("coefficient arrays shorter than the band-limits")
        t = ctypes.c_uint64()
        L.check(L.lib().slsht_submit(self._h, ctypes.byref(desc), f.ctypes.data, h.ctypes.data,
                                     ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int):
        st, err = ctypes.c_int(), ctypes.c_int()
        ptr, n = ctypes.c_void_p(), ctypes.c_size_t()
        L.check(L.lib().slsht_poll(self._h, ticket, ctypes.byref(st), ctypes.byref(ptr),
                                   ctypes.byref(n), ctypes.byref(err)))
        return st.value, ptr.value or 0, n.value, err.value

    def wait(self, ticket: int, timeout_ms: int = 120000) -> None:
        L.check(L.lib().slsht_wait(self._h, ticket, timeout_ms))

    def result(self, ticket: int, dtype) -> np.ndarray:
        """Host copy of a finished request's output (flat, in the slsht_forward layout)."""
        st, ptr, n, err = self.poll(ticket)
        if st != L.REQ_DONE:
            raise RuntimeError(f"ticket {ticket} not done (state {st}, err {err})")
        out = np.empty(n // np.dtype(dtype).itemsize, dtype=dtype)
        _hip_memcpy_d2h(out, ptr, n)
        return out

    def result_device(self, ticket: int, dtype, device: int = 0):
        """Device copy (a torch tensor) of a finished request's output, flat.  Returns once
        the copy has completed: a device-to-device hipMemcpy may return before it does, and
        after `release` the server may hand the block to a new request at once."""
        import torch
        st, ptr, n, err = self.poll(ticket)
        if st != L.REQ_DONE:
            raise RuntimeError(f"ticket {ticket} not done (state {st}, err {err})")
        out = torch.empty(n // torch.empty((), dtype=dtype).element_size(), dtype=dtype,
                          device=f"cuda:{device}")
        torch.cuda.synchronize(device)
        _hip_memcpy(out.data_ptr(), ptr, n, 3)
        torch.cuda.synchronize(device)
        return out

    def release(self, ticket: int) -> None:
        L.check(L.lib().slsht_release(self._h, ticket))

    def times(self, ticket: int) -> tuple[float, float, float]:
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        L.check(L.lib().slsht_request_times(self._h, ticket, ctypes.byref(a), ctypes.byref(b),
                                            ctypes.byref(c)))
        return a.value, b.value, c.value

    def clock(self) -> float:
        return L.lib().slsht_server_clock(self._h)

    def stats(self) -> tuple[int, int, int, int]:
        u, b = ctypes.c_size_t(), ctypes.c_size_t()
        q, r = ctypes.c_int(), ctypes.c_int()
        L.check(L.lib().slsht_server_stats(self._h, ctypes.byref(u), ctypes.byref(b),
                                           ctypes.byref(q), ctypes.byref(r)))
        return u.value, b.value, q.value, r.value


def request_desc(req) -> L.Desc:
    n_phi, n_theta, n_omega = req.grid
    return make_desc(req.L_f, req.L_h, req.l_lo, req.l_hi, n_phi, n_theta, n_omega,
                     precision=req.precision)


def run_stream(server: Server, requests, inputs=None, keep=None, poll_sleep_s: float = 2e-4,
               keep_on_device: bool = False):
    """Submit `requests` (ServingRequest list, sorted by arrival) at their arrival times
    and drive them to completion.  `inputs[i]` = (f, h) or None to draw from the request's
    seed; `keep(i)` -> True to copy that result out (to the host, or with `keep_on_device`
    into a torch device tensor, which holds the polling loop up far less).  Returns a dict
    with per-request latencies (s), the host time of each slsht_submit call (s), the
    results kept, the peak budget use seen, and the wall span."""
    n = len(requests)
    tickets = [None] * n
    lat = np.full(n, np.nan)
    submit_s = np.full(n, np.nan)
    kept = {}
    peak = 0
    start = time.perf_counter()
    t0_srv = server.clock()
    pending = []
    i = 0
    done = 0
    while done < n:
        now = time.perf_counter() - start
        while i < n and requests[i].arrival_s <= now:
            f, h = inputs[i] if inputs is not None else requests[i].inputs()
            ts_ = time.perf_counter()
            tickets[i] = server.submit(request_desc(requests[i]), f, h)
            submit_s[i] = time.perf_counter() - ts_
            pending.append(i)
            i += 1
        still = []
        for j in pending:
            st, _, _, err = server.poll(tickets[j])
            if st == L.REQ_DONE or st == L.REQ_FAILED:
                if st == L.REQ_FAILED:
                    raise RuntimeError(f"request {j} failed with status {err}")
                ts, _, td = server.times(tickets[j])
                # latency from the request's scheduled arrival, in server-clock terms
                lat[j] = td - (t0_srv + requests[j].arrival_s) if td > 0 else np.nan
                lat[j] = max(lat[j], td - ts)
                if keep is not None and keep(j):
                    fp64 = requests[j].precision == "fp64"
                    if keep_on_device:
                        import torch
                        kept[j] = server.result_device(
                            tickets[j], torch.complex128 if fp64 else torch.complex64)
                    else:
                        kept[j] = server.result(tickets[j],
                                                np.complex128 if fp64 else np.complex64)
                server.release(tickets[j])
                done += 1
            else:
                still.append(j)
        pending = still
        used = server.stats()[0]
        peak = max(peak, used)
        if i < n and not pending:
            time.sleep(max(0.0, min(requests[i].arrival_s - (time.perf_counter() - start), 0.01)))
        else:
            time.sleep(poll_sleep_s)
    span = time.perf_counter() - start
    return {"latency_s": lat, "kept": kept, "peak_used_bytes": peak, "span_s": span,
            "tickets": tickets, "submit_s": submit_s}

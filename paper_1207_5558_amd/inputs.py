"""Seeded synthetic inputs for the directional SLSHT.

This module only draws random numbers and lays them out; it holds none of the
transform's arithmetic.  Both the CPU oracle and the GPU library consume what
it produces, so it must stay free of any code from either side.

Conventions (paper, Section II):
  * spherical-harmonic coefficients are complex, stored flat at index
    l*l + l + m for 0 <= l < L (exclusive band-limit L), |m| <= l;
  * "real-signal consistent" means f_l^{-m} = (-1)^m conj(f_l^m), which is the
    symmetry of the coefficients of a real-valued signal (Section IV, last
    remark); the paper's windows are real Slepian eigenfunctions (Section III-D),
    so random windows are drawn with the same symmetry;
  * a window is normalised to unit energy <h,h> = sum |h_s^r|^2 = 1
    (Definition 1).

Workloads stand in for the paper's: its numerical-validation experiment
(Section V-A: L_h = 18, 18 <= L_f <= 130, random coefficients) and its
topography examples (Section V-B: L = 128 Earth, L_h = 60 Mars), which need
datasets that are not available here.  The SO(3) grid of every workload is
(2(L_f+L_h)-1) phi x (L_f+L_h) theta x (2L_h-1) omega samples.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "grid_dims", "draw_coefficients",
    "draw_window", "make_inputs", "rho_subset", "ServingRequest",
    "serving_stream", "n_lm",
]


def grid_dims(L_f: int, L_h: int, n_az: int = 0) -> tuple[int, int, int]:
    """(n_phi, n_theta, n_omega) of the oversampled SO(3) grid used by all workloads;
    a steerable window (azimuthal band-limit n_az < L_h) needs 2 n_az - 1 omega samples."""
    return 2 * (L_f + L_h) - 1, L_f + L_h, 2 * (n_az or L_h) - 1


def n_lm(l_lo: int, l_hi: int) -> int:
    """Number of (l, m) pairs with l_lo <= l < l_hi, |m| <= l."""
    return l_hi * l_hi - l_lo * l_lo


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    L_f: int
    L_h: int
    l_lo: int
    l_hi: int
    n_phi: int
    n_theta: int
    n_omega: int
    seed: int
    spectrum: float      # variance of f_l^m is l^-spectrum (0 = flat, unit variance)
    zero_dc: bool        # f_0^0 = 0
    precision: str       # "fp64" or "fp32"
    output: str          # "full" or "energy"
    n_az: int = 0        # azimuthal band-limit of a steerable window (0: L_h)

    @property
    def n_lm(self) -> int:
        return n_lm(self.l_lo, self.l_hi)

    @property
    def n_rho(self) -> int:
        return self.n_phi * self.n_theta * self.n_omega

    @property
    def samples(self) -> int:
        return self.n_lm * self.n_rho


def _wl(name, L_f, L_h, l_lo, l_hi, seed, spectrum, zero_dc, precision, output, n_az=0):
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h, n_az)
    return Workload(name, L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega, seed,
                    spectrum, zero_dc, precision, output, n_az)


WORKLOADS = {
    # tiny FP64 case: L_f=8, L_h=3, all l<8, 21x11x5 grid, N(0,1) coefficients
    "tiny": _wl("tiny", 8, 3, 0, 8, 0, 0.0, False, "fp64", "full"),
    # mid-size FP64 case: L_f=128, L_h=8, l in [32,48), 271x136x15 grid, l^-2 spectrum
    "mid": _wl("mid", 128, 8, 32, 48, 1, 2.0, True, "fp64", "full"),
    # same inputs as "mid", FP32-mixed arithmetic, complex64 output
    "mid_fp32": _wl("mid_fp32", 128, 8, 32, 48, 1, 2.0, True, "fp32", "full"),
    # topography-like map: L_f=512, L_h=32, l in [100,116), 1087x544x63 grid,
    # l^-2.5 spectrum, FP32-mixed, output reduced to sum_m |g|^2 per (l, rho)
    "large": _wl("large", 512, 32, 100, 116, 4, 2.5, True, "fp32", "energy"),
    # "mid" with a steerable window: azimuthal band-limit 3 (h_s^r = 0 for |r| >= 3),
    # so omega needs 2*3-1 = 5 samples: 271x136x5 grid, FP64
    "mid_steer": _wl("mid_steer", 128, 8, 32, 48, 1, 2.0, True, "fp64", "full", n_az=3),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def draw_coefficients(rng: np.random.Generator, L: int, spectrum: float = 0.0,
                      zero_dc: bool = False) -> np.ndarray:
    """Real-signal-consistent complex coefficients c_l^m, l < L.

    Re and Im of c_l^m (m > 0) are i.i.d. N(0, s_l^2) with s_l^2 = l^-spectrum
    (s_l = 1 when spectrum == 0); c_l^0 keeps its real part only; c_l^{-m} is
    (-1)^m conj(c_l^m).  Draw order: l ascending, m = 0..l, (Re, Im) pairs.
    """
    out = np.zeros(L * L, dtype=np.complex128)
    for l in range(L):
        z = rng.standard_normal((l + 1, 2))
        if spectrum != 0.0:
            s = 0.0 if l == 0 else l ** (-0.5 * spectrum)
        else:
            s = 1.0
        if l == 0 and zero_dc:
            s = 0.0
        z *= s
        base = l * l + l
        out[base] = z[0, 0]
        if l:
            m = np.arange(1, l + 1)
            c = z[1:, 0] + 1j * z[1:, 1]
            out[base + m] = c
            out[base - m] = ((-1.0) ** m) * np.conj(c)
    return out


def draw_window(rng: np.random.Generator, L_h: int, min_dc: float = 1e-3,
                n_az: int = 0) -> np.ndarray:
    """Random asymmetric band-limited window, real-signal consistent, unit energy.

    With n_az > 0 the window is steerable: h_s^r is set to zero for |r| >= n_az after
    the draw (the draw itself is unchanged).  Redrawn (from the same generator) while
    |h_0^0| < min_dc, because the inverse transform divides by h_0^0.
    """
    while True:
        h = draw_coefficients(rng, L_h, 0.0, False)
        if n_az:
            for s in range(L_h):
                for r in range(-s, s + 1):
                    if abs(r) >= n_az:
                        h[s * s + s + r] = 0.0
        h /= math.sqrt(float(np.sum(np.abs(h) ** 2)))
        if abs(h[0]) >= min_dc:
            return h


def make_inputs(wl: Workload) -> tuple[np.ndarray, np.ndarray]:
    """(f, h) for a workload; f first, then h, from default_rng(seed)."""
    rng = np.random.default_rng(wl.seed)
    f = draw_coefficients(rng, wl.L_f, wl.spectrum, wl.zero_dc)
    h = draw_window(rng, wl.L_h, n_az=wl.n_az)
    return f, h


def rho_subset(wl: Workload, count: int, seed: int = 12345) -> np.ndarray:
    """Seeded sample of grid rotations as an int array [count, 3] of (a, b, c)
    indices into the (phi, theta, omega) axes.  Always contains the corners
    (0,0,0) and (n_phi-1, n_theta-1, n_omega-1)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, wl.n_phi, count)
    b = rng.integers(0, wl.n_theta, count)
    c = rng.integers(0, wl.n_omega, count)
    idx = np.stack([a, b, c], axis=1)
    if count >= 2:
        idx[0] = (0, 0, 0)
        idx[1] = (wl.n_phi - 1, wl.n_theta - 1, wl.n_omega - 1)
    return idx.astype(np.int64)


@dataclasses.dataclass(frozen=True)
class ServingRequest:
    arrival_s: float
    L_f: int
    L_h: int
    l_lo: int
    l_hi: int
    precision: str
    seed: int

    @property
    def grid(self) -> tuple[int, int, int]:
        return grid_dims(self.L_f, self.L_h)

    @property
    def samples(self) -> int:
        n_phi, n_theta, n_omega = self.grid
        return n_lm(self.l_lo, self.l_hi) * n_phi * n_theta * n_omega

    def inputs(self) -> tuple[np.ndarray, np.ndarray]:
        rng = np.random.default_rng(self.seed)
        f = draw_coefficients(rng, self.L_f, 2.0, True)
        h = draw_window(rng, self.L_h)
        return f, h


def serving_stream(n_requests: int, rate_hz: float, seed: int = 7,
                   L_f_choices=(32, 64, 96, 128, 192), L_h_choices=(4, 8, 16),
                   width: int = 8) -> list[ServingRequest]:
    """Poisson arrivals at rate_hz; L_f, L_h uniform over the choices; an
    l-window of the given width at a uniform offset in [0, L_f - width];
    precision alternates uniformly at random between fp64 and fp32."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        L_f = int(rng.choice(L_f_choices))
        L_h = int(rng.choice(L_h_choices))
        l_lo = int(rng.integers(0, L_f - width + 1))
        prec = "fp64" if rng.random() < 0.5 else "fp32"
        reqs.append(ServingRequest(t, L_f, L_h, l_lo, l_lo + width, prec,
                                   seed * 1000003 + i))
    return reqs

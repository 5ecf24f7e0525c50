"""Throughput benchmark of the directional SLSHT forward transform on one MI355X.

One step = one slsht_forward call (3j coupling + fused theta/omega/phi
synthesis + store) over the mid-size workload: L_f=128, L_h=8, l in [32,48)
(1280 (l,m) pairs), 271 x 136 x 15 SO(3) grid, FP64, complex128 output
(7.076e8 samples, 11.3 GB written per step).  Inputs are resident in HBM before
the timed region.  The same workload in FP32-mixed arithmetic (complex64 out)
is timed beside it, and both are checked against the CPU oracle on a seeded
sample of rotations, which is also timed as the CPU baseline.

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "g(ρ;ℓ,m) samples/s on 1 MI355X, FP32-mixed vs FP64 at stated error; p99 ms"
HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK = 157.3          # TFLOP/s, dense FP32 MFMA (MI355X spec sheet)
MFMA_F64_PEAK = 78.6           # TFLOP/s, dense FP64 MFMA (MI355X spec sheet)
KERNEL = "synth_full_kernel"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    """Digest of the sources of the FULL synthesis kernel (its file and the device
    headers it includes); a counter summary is used only if it carries the same one."""
    h = hashlib.sha256()
    for name in ("slsht_synth.hip", "slsht_device.h", "slsht_phi.h"):
        h.update(open(os.path.join(ROOT, "paper_1207_5558_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def committed_traffic(profile_name: str, digest: str):
    """HBM bytes per launch from a committed counter summary, if it was taken on
    the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", profile_name)
    if not os.path.exists(p):
        return None
    txt = open(p).read()
    m_d = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    m_t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m_d or not m_t or m_d.group(1) != digest:
        return None
    return float(m_t.group(1))


def time_forward(plan, f_t, h_t, g_t, steps, warmup, torch, lib_api):
    """Durations (ms) of the forward call, of its coupling stage and of the synthesis
    kernel alone (slsht_synthesize from that coupling), from HIP events recorded on the
    stream the kernels are launched on."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.forward(f_t, h_t, g_t, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        plan.forward(f_t, h_t, g_t, stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in ev])
    # coupling stage alone, then the synthesis kernel alone from that coupling, same stream
    A = torch.empty((plan.n_lm, plan.desc.L_h ** 2), dtype=torch.complex128, device=g_t.device)
    cev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for s, e in cev:
        s.record(stream)
        plan.coupling(f_t, A, stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    cpl = np.array([s.elapsed_time(e) for s, e in cev])
    sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for s, e in sev:
        s.record(stream)
        plan.synthesize(A, h_t, g_t, stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    syn = np.array([s.elapsed_time(e) for s, e in sev])
    return wall, per, cpl, syn


def cpu_baseline(wl, f, h, budget_s: float):
    """The oracle, untuned, on a bounded seeded sample of rotations (all (l,m))."""
    from threadpoolctl import threadpool_info

    from oracle.slsht import oracle_g_grid
    from paper_1207_5558_amd.inputs import rho_subset
    n = 64
    while True:
        idx = rho_subset(wl, n, seed=99)
        t = time.perf_counter()
        ref = oracle_g_grid(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta,
                            wl.n_omega, idx)
        dt = time.perf_counter() - t
        if dt >= 0.5 * budget_s or n >= 200000:
            break
        n = int(n * min(10.0, budget_s / max(dt, 1e-3)))
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    return idx, ref, dt, threads


def energy_flops_per_m_theta(wl, n_items: int) -> float:
    """Algorithmic flops per (order, theta row) of the ENERGY path as built: the folded phi
    GEMMs (cos part K = L_h, sin part K = L_h - 1, real and imaginary parts), the p-sum
    U_q = sum_p A^p_q W^p_q (sum_q (L_h - |q|) = L_h^2 complex MACs per omega sample), the
    fold into P_k, M_k, forming g(a), g(n-a) and accumulating |g|^2 (6 per sample), and the
    W table (sum_p (2p+1)^2 complex MACs per omega sample and theta row) spread over the
    n_items orders that share it."""
    L, nslot, no = wl.L_h, (wl.n_phi + 1) // 2, wl.n_omega
    phi = 2 * nslot * no * 2 * (L + (L - 1))
    u = 8 * L * L * no
    fold = 4 * (L - 1) * no
    energy = 6 * wl.n_phi * no
    w = 8 * no * sum((2 * p + 1) ** 2 for p in range(L)) / n_items
    return float(phi + u + fold + energy + w)


def energy_leg(torch, api, steps, n_rot=16):
    """Topography-like workload (L_f=512, L_h=32, l in [100,116), 1087x544x63, FP32-mixed),
    output reduced to sum_m |g|^2; timed for all orders and for the real-pair path, with
    the error of E against the FP64 oracle on seeded rotations."""
    from oracle.slsht import oracle_energy, oracle_g_grid
    from paper_1207_5558_amd.inputs import make_inputs, rho_subset, workload
    wl = workload("large")
    f, h = make_inputs(wl)
    ft, ht = torch.from_numpy(f).to("cuda:0"), torch.from_numpy(h).to("cuda:0")
    out = {"workload": "large: L_f=512, L_h=32, l in [100,116) all m (3456 (l,m)), "
                       "1087 x 544 x 63 grid, FP32-mixed, energy output",
           "samples_per_step": wl.samples}
    idx = rho_subset(wl, n_rot, seed=404)
    t0 = time.perf_counter()
    E_ref = oracle_energy(oracle_g_grid(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi,
                                        wl.n_theta, wl.n_omega, idx), wl.l_lo, wl.l_hi)
    oracle_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    for name, pair in (("all_orders", False), ("real_pair", True)):
        plan = api.Plan(api.desc_for(wl, real_pair=pair), device=0)
        E = plan.empty_output()
        plan.forward(ft, ht, E)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        for s_, e_ in ev:
            s_.record(stream)
            plan.forward(ft, ht, E, stream=stream)
            e_.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([s_.elapsed_time(e_) for s_, e_ in ev]))
        # energy kernels alone (W table, A fragments, U GEMM, phi + |g|^2) from one coupling
        A = plan.coupling(ft)
        sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        for s_, e_ in sev:
            s_.record(stream)
            plan.synthesize(A, ht, E, stream=stream)
            e_.record(stream)
        torch.cuda.synchronize()
        syn_ms = float(np.mean([s_.elapsed_time(e_) for s_, e_ in sev]))
        n_items = wl.n_lm if not pair else sum(l + 1 for l in range(wl.l_lo, wl.l_hi))
        fl = energy_flops_per_m_theta(wl, n_items)
        n_m_theta = n_items * wl.n_theta
        tf = fl * n_m_theta / (ms * 1e-3) / 1e12
        a = torch.as_tensor(idx[:, 0], device=E.device)
        b = torch.as_tensor(idx[:, 1], device=E.device)
        c = torch.as_tensor(idx[:, 2], device=E.device)
        got = E[:, c, b, a].transpose(0, 1).double().cpu().numpy()       # [rho, l]
        per_l = {}
        for k, l in enumerate(range(wl.l_lo, wl.l_hi)):
            d = got[:, k] - E_ref[:, k]
            per_l[str(l)] = {"rel_frobenius": float(np.linalg.norm(d) / np.linalg.norm(E_ref[:, k])),
                             "max_abs": float(np.abs(d).max())}
        out[name] = {"ms_per_step": ms, "value": wl.samples / (ms * 1e-3), "unit": "samples/s",
                     "energy_kernels_ms": syn_ms,
                     "roofline": {"bound": "mfma", "achieved": tf, "peak": MFMA_F32_PEAK,
                                  "unit": "TFLOP/s", "frac": tf / MFMA_F32_PEAK,
                                  "flops_per_m_theta": fl,
                                  "algorithmic_flops_per_launch": fl * n_m_theta,
                                  "note": "whole forward (coupling + energy kernels) per step"},
                     "error_vs_oracle": {
                         "max_rel_frobenius_per_l": max(v["rel_frobenius"] for v in per_l.values()),
                         "max_abs": max(v["max_abs"] for v in per_l.values()),
                         "max_abs_ref": float(np.abs(E_ref).max()),
                         "rotations": int(idx.shape[0]), "per_l": per_l}}
        log(f"energy {name}: {ms:.1f} ms (energy kernels {syn_ms:.1f} ms), "
            f"{wl.samples / (ms * 1e-3):.3e} samples/s, {tf:.1f} TFLOP/s, max rel err per l "
            f"{out[name]['error_vs_oracle']['max_rel_frobenius_per_l']:.2e}")
        del E, plan, A
        torch.cuda.empty_cache()
    out["oracle_seconds"] = oracle_s
    return out


def tiny_leg(torch, api, steps, warmup):
    """Tiny workload (L_f=8, L_h=3, l < 8, 21 x 11 x 5 grid, FP64): launch-bound, reported
    for latency only, with its error against the oracle on the whole grid."""
    from oracle.slsht import oracle_g_full
    from paper_1207_5558_amd.inputs import make_inputs, workload
    wl = workload("tiny")
    f, h = make_inputs(wl)
    ft, ht = torch.from_numpy(f).to("cuda:0"), torch.from_numpy(h).to("cuda:0")
    plan = api.Plan(api.desc_for(wl), device=0)
    g = plan.empty_output()
    _, per, cpl, syn = time_forward(plan, ft, ht, g, steps, warmup, torch, api)
    plan.forward(ft, ht, g)
    torch.cuda.synchronize()
    ref = oracle_g_full(f, h, wl.L_f, wl.L_h, wl.l_lo, wl.l_hi, wl.n_phi, wl.n_theta, wl.n_omega)
    got = g.cpu().numpy()
    return {"workload": "tiny: L_f=8, L_h=3, l in [0,8) all m, 21 x 11 x 5 grid, FP64",
            "ms_per_step": float(per.mean()), "p50_ms": float(np.percentile(per, 50)),
            "p99_ms": float(np.percentile(per, 99)), "coupling_ms": float(cpl.mean()),
            "synthesis_ms": float(syn.mean()), "value": wl.samples / (per.mean() * 1e-3),
            "unit": "samples/s",
            "error_vs_oracle": {"max_rel": float(np.abs(got - ref).max() / np.abs(ref).max()),
                                "max_abs": float(np.abs(got - ref).max()),
                                "grid": "whole"}}


def steerable_leg(torch, api, steps, warmup):
    """The mid-size workload with a steerable window (azimuthal band-limit 3): the theta
    and omega contractions run over |q'| < 3 and 5 omega samples carry all of g."""
    from paper_1207_5558_amd.inputs import make_inputs, workload
    wl = workload("mid_steer")
    f, h = make_inputs(wl)
    ft, ht = torch.from_numpy(f).to("cuda:0"), torch.from_numpy(h).to("cuda:0")
    plan = api.Plan(api.desc_for(wl), device=0)
    g = plan.empty_output()
    _, per, cpl, syn = time_forward(plan, ft, ht, g, steps, warmup, torch, api)
    ms, kern = float(per.mean()), float(syn.mean())
    L = wl.L_h
    out_b = g.numel() * g.element_size()
    alg = out_b + wl.n_lm * L * L * 16 + L * L * 16 + wl.n_theta * (L * (L + 1) * (2 * L + 1) // 6) * 8
    log(f"steerable mid: forward {ms:.3f} ms, {wl.samples / (ms * 1e-3):.3e} samples/s")
    del g, plan
    torch.cuda.empty_cache()
    return {"workload": "mid_steer: L_f=128, L_h=8, azimuthal band-limit 3, l in [32,48) all m, "
                        "271 x 136 x 5 grid, FP64", "ms_per_step": ms,
            "value": wl.samples / (ms * 1e-3), "unit": "samples/s",
            "roofline": {"bound": "hbm", "achieved": alg / (kern * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / (kern * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def windows_leg(torch, api, f_t, g_single, steps, warmup, n_windows=4):
    """One signal of the mid-size workload against 4 windows (FP64): one coupling, four
    syntheses (slsht_forward_windows)."""
    from paper_1207_5558_amd.inputs import draw_window, workload
    wl = workload("mid")
    rng = np.random.default_rng(2)
    hs = np.stack([draw_window(rng, wl.L_h) for _ in range(n_windows)])
    ht = torch.from_numpy(hs).to("cuda:0")
    plan = api.Plan(api.desc_for(wl), device=0)
    g = torch.empty((n_windows,) + tuple(plan.output_shape), dtype=plan.output_dtype,
                    device="cuda:0")
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.forward_windows(f_t, ht, g, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for s_, e_ in ev:
        s_.record(stream)
        plan.forward_windows(f_t, ht, g, stream=stream)
        e_.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([s_.elapsed_time(e_) for s_, e_ in ev]))
    log(f"{n_windows} windows, mid FP64: {ms:.3f} ms, "
        f"{n_windows * wl.samples / (ms * 1e-3):.3e} samples/s")
    del g, plan
    torch.cuda.empty_cache()
    return {"workload": f"mid FP64, one signal against {n_windows} windows (one coupling)",
            "windows": n_windows, "ms_per_step": ms,
            "value": n_windows * wl.samples / (ms * 1e-3), "unit": "samples/s"}


def slepian_leg(api):
    """Slepian window generator: the paper's region R_(pi/6, pi/6 + pi/240) at L_h = 18 and
    the largest band-limit, L_h = 32 (concentration matrix on the GPU, eigenvector on the
    host by Householder tridiagonalisation and implicit QL); wall time per call."""
    import math
    out = {}
    for L_h in (18, 32):
        api.slepian_window(L_h, math.pi / 6, math.pi / 6 + math.pi / 240)
        t = time.perf_counter()
        _, lam = api.slepian_window(L_h, math.pi / 6, math.pi / 6 + math.pi / 240)
        out[f"L_h={L_h}"] = {"ms": (time.perf_counter() - t) * 1e3, "concentration": lam}
        log(f"slepian window L_h={L_h}: {out[f'L_h={L_h}']['ms']:.1f} ms, lambda {lam:.6f}")
    out["region"] = "theta_c = pi/6, a = pi/6 + pi/240"
    return out


def factored_leg(torch, api, L_h=18, L_fs=(18, 34, 66, 130)):
    """The paper's timing experiment (Section V), L_h = 18, every g(rho; l, m) for
    l < L_f + L_h - 1 on the minimal grid E_{L_h}, FP64: tau_1 = coupling through the
    modulated-signal transform (Appendix A), tau_2 = factored synthesis from it (Delta by
    the Trapani-Navaza recursion, C, 3-D Fourier sum), tau_3 = inverse; beside them the
    3j coupling and the separated-form forward (coupling + synthesis) on the same grid.
    Log-log slopes between the last two points are reported for comparison with the
    paper's O(L_f^3) (tau_1) and O(L_f^2) (tau_2, tau_3)."""
    from paper_1207_5558_amd.inputs import draw_coefficients, draw_window
    rng = np.random.default_rng(5)
    h = torch.from_numpy(draw_window(rng, L_h)).to("cuda:0")
    K = 2 * L_h - 1
    out = {"workload": f"L_h={L_h}, all l < L_f + L_h - 1, minimal grid {K} x {L_h} x {K}, FP64",
           "points": []}

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_.record()
        for _ in range(reps):
            fn()
        e_.record()
        torch.cuda.synchronize()
        return s_.elapsed_time(e_) / reps

    for L_f in L_fs:
        f = torch.from_numpy(draw_coefficients(rng, L_f, 2.0, True)).to("cuda:0")
        plan = api.Plan(api.make_desc(L_f, L_h, 0, L_f + L_h - 1, K, L_h, K), device=0)
        g = plan.empty_output()
        A = torch.empty((plan.n_lm, L_h * L_h), dtype=torch.complex128, device="cuda:0")
        A3 = torch.empty_like(A)
        f_out = torch.empty(plan.n_lm, dtype=torch.complex128, device="cuda:0")
        work_f = torch.empty(api.factored_workspace(plan.desc), dtype=torch.uint8, device="cuda:0")
        work_m = torch.empty(api.modulated_workspace(plan.desc), dtype=torch.uint8,
                             device="cuda:0")
        res = {
            "tau1_ms": timed(lambda: plan.coupling_modulated(f, A, work_m)),
            "tau2_ms": timed(lambda: plan.synthesize_factored(A, h, g, work_f)),
            "tau3_ms": timed(lambda: plan.inverse(g, h, f_out)),
            "coupling_3j_ms": timed(lambda: plan.coupling(f, A3)),
            "separated_ms": timed(lambda: plan.forward(f, h, g)),
            "separated_synthesis_ms": timed(lambda: plan.synthesize(A3, h, g)),
        }
        # both syntheses write g once (complex128); the inputs (A, tables) are < 1% of it
        gb = g.numel() * g.element_size()
        for key, ms_key in (("roofline_separated_synthesis", "separated_synthesis_ms"),
                            ("roofline_tau2", "tau2_ms")):
            ach = gb / (res[ms_key] * 1e-3) / 1e9
            res[key] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": gb}
        # the same synthesis against the FP64 matrix peak: per output row (l, m, theta, omega)
        # the U GEMM takes sum_{|q|<L_h} (L_h - |q|) = L_h^2 complex MACs (8 flops each) and the
        # folded phi sums L_h x (n_phi + 1)/2 slots x 8 flops
        rows = plan.n_lm * L_h * K
        flops = rows * (8 * L_h * L_h + 8 * L_h * ((K + 1) // 2))
        tf = flops / (res["separated_synthesis_ms"] * 1e-3) / 1e12
        res["roofline_separated_synthesis_mfma"] = {
            "bound": "mfma", "achieved": tf, "peak": MFMA_F64_PEAK, "unit": "TFLOP/s",
            "frac": tf / MFMA_F64_PEAK, "algorithmic_flops_per_launch": flops}
        out["points"].append({"L_f": L_f, "n_lm": plan.n_lm, **res})
        log(f"paper route L_f={L_f}: tau1 {res['tau1_ms']:.3f} ms, tau2 {res['tau2_ms']:.3f} ms, "
            f"tau3 {res['tau3_ms']:.3f} ms | 3j coupling {res['coupling_3j_ms']:.3f} ms, "
            f"separated forward {res['separated_ms']:.3f} ms")
        del g, A, A3, f_out, work_f, work_m, plan
        torch.cuda.empty_cache()
    if len(out["points"]) >= 2:
        p0, p1 = out["points"][-2], out["points"][-1]
        r = np.log(p1["L_f"] / p0["L_f"])
        for k in ("tau1", "tau2", "tau3"):
            out[f"slope_{k}"] = float(np.log(p1[f"{k}_ms"] / p0[f"{k}_ms"]) / r)
    return out


def full_lh16_leg(torch, api, steps, warmup):
    """The largest serving shape run alone: L_f=192, L_h=16, l in [184,192) all m (3008
    (l,m)), 415 x 208 x 31 grid, FULL output in FP64 (128.8 GB) and FP32-mixed (64.4 GB);
    the synthesis here runs the MFMA phi stage of the band-limit bucket 16."""
    from paper_1207_5558_amd.inputs import draw_coefficients, draw_window, grid_dims
    rng = np.random.default_rng(16)
    L_f, L_h, l_lo, l_hi = 192, 16, 184, 192
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h)
    f = torch.from_numpy(draw_coefficients(rng, L_f, 2.0, True)).to("cuda:0")
    h = torch.from_numpy(draw_window(rng, L_h)).to("cuda:0")
    out = {"workload": f"L_f={L_f}, L_h={L_h}, l in [{l_lo},{l_hi}) all m, "
                       f"{n_phi} x {n_theta} x {n_omega} grid, FULL"}
    for prec in ("fp64", "fp32"):
        plan = api.Plan(api.make_desc(L_f, L_h, l_lo, l_hi, n_phi, n_theta, n_omega,
                                      precision=prec), device=0)
        g = plan.empty_output()
        _, per, cpl, syn = time_forward(plan, f, h, g, steps, warmup, torch, api)
        gb = g.numel() * g.element_size()
        ach = gb / (syn.mean() * 1e-3) / 1e9
        samples = plan.n_lm * n_phi * n_theta * n_omega
        out[prec] = {"ms_per_step": float(per.mean()), "synthesis_ms": float(syn.mean()),
                     "value": samples / (per.mean() * 1e-3), "unit": "samples/s",
                     "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                  "algorithmic_bytes_per_launch": gb}}
        log(f"L_h=16 shape {prec}: forward {per.mean():.2f} ms, synthesis {syn.mean():.2f} ms, "
            f"{ach:.0f} GB/s")
        del g, plan
        torch.cuda.empty_cache()
    return out


def serving_leg(n, rate):
    """Continuous batching of the serving workload: n requests with Poisson arrivals at
    `rate` req/s, L_f in {32..192}, L_h in {4,8,16}, width-8 l-windows, half FP64 and half
    FP32-mixed; latency is arrival -> done on the server clock."""
    import torch
    from paper_1207_5558_amd.inputs import serving_stream
    from paper_1207_5558_amd.serving import Server, run_stream
    torch.cuda.empty_cache()
    reqs = serving_stream(n, rate_hz=rate, seed=7)
    inputs = [r.inputs() for r in reqs]
    tot = sum(r.samples for r in reqs)
    # per precision, the in-stream result of a request with the largest band-limits (the
    # lowest l-window among them, to keep the copy small) is kept on the device and checked
    # against the oracle on seeded rotations after the run
    check = {}
    for prec in ("fp64", "fp32"):
        cand = [i for i, r in enumerate(reqs) if r.precision == prec]
        if cand:
            check[prec] = max(cand, key=lambda i: (reqs[i].L_f, reqs[i].L_h, -reqs[i].l_lo))
    srv = Server(hbm_budget=200 << 30, n_streams=4)
    res = run_stream(srv, reqs, inputs=inputs, keep=lambda i: i in check.values(),
                     keep_on_device=True)
    srv.close()
    lat = res["latency_s"] * 1e3
    sub = res["submit_s"] * 1e3
    out = {"requests": n, "arrival_rate_hz": rate, "hbm_budget_bytes": 200 << 30,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "mean_ms": float(lat.mean()), "value": tot / res["span_s"], "unit": "samples/s",
           "span_s": res["span_s"], "samples": tot, "peak_budget_used_bytes": res["peak_used_bytes"],
           "submit_p50_ms": float(np.percentile(sub, 50)),
           "submit_p99_ms": float(np.percentile(sub, 99)),
           "submit_max_ms": float(sub.max())}
    errs = {}
    for prec, i in check.items():
        r = reqs[i]
        f, h = inputs[i]
        n_phi, n_theta, n_omega = r.grid
        rng = np.random.default_rng(100 + i)
        idx = np.stack([rng.integers(0, n_phi, 24), rng.integers(0, n_theta, 24),
                        rng.integers(0, n_omega, 24)], 1)
        from oracle.slsht import oracle_g_grid
        ref = oracle_g_grid(f, h, r.L_f, r.L_h, r.l_lo, r.l_hi, n_phi, n_theta, n_omega, idx)
        g = res["kept"][i].reshape(-1, n_omega, n_theta, n_phi)
        sel = g[:, torch.as_tensor(idx[:, 2], device=g.device),
                torch.as_tensor(idx[:, 1], device=g.device),
                torch.as_tensor(idx[:, 0], device=g.device)].transpose(0, 1).cpu().numpy()
        per_l = rel_err_per_l(sel, ref, r.l_lo, r.l_hi)
        errs[prec] = {"request": i, "L_f": r.L_f, "L_h": r.L_h, "l_range": [r.l_lo, r.l_hi],
                      "rotations": len(idx), "max_rel_frobenius_per_l": max(per_l),
                      "max_abs": float(np.abs(sel - ref).max()),
                      "max_abs_rel_to_max": float(np.abs(sel - ref).max() / np.abs(ref).max())}
    res["kept"].clear()
    out["error_vs_oracle"] = errs
    log(f"serving: {n} req at {rate}/s: p50 {out['p50_ms']:.2f} ms, p99 {out['p99_ms']:.2f} ms, "
        f"{out['value']:.3e} samples/s; submit p50 {out['submit_p50_ms']:.3f} ms, "
        f"p99 {out['submit_p99_ms']:.3f} ms; errors "
        + ", ".join(f"{p} {e['max_rel_frobenius_per_l']:.2e}" for p, e in errs.items()))
    return out


def rel_err_per_l(got, ref, l_lo, l_hi):
    out = []
    for l in range(l_lo, l_hi):
        s = l * l - l_lo * l_lo
        d = got[:, s:s + 2 * l + 1] - ref[:, s:s + 2 * l + 1]
        out.append(float(np.linalg.norm(d) / np.linalg.norm(ref[:, s:s + 2 * l + 1])))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--no-energy", action="store_true", help="skip the ENERGY workload leg")
    ap.add_argument("--steps-energy", type=int, default=3)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the steerable-window, several-window and Slepian-window legs")
    ap.add_argument("--legs", default="steerable,windows,slepian,factored,lh16",
                    help="comma list of the NEXT / serving-shape legs to run (unless --no-next)")
    ap.add_argument("--serve-n", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=200.0, help="Poisson arrival rate, req/s")
    ap.add_argument("--serve-rate-sat", type=float, default=20000.0,
                    help="arrival rate of the second, saturating serving run (capacity)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 4 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = 1 << 29                       # float64 elements: 4 GiB read, 4 GiB written
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": n * 8, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the forward transform shards over l-ranges with no exchange step, but only "
              "the one-GPU kernel is built and measured)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1207_5558_amd import api
    from paper_1207_5558_amd.inputs import make_inputs, workload

    wl = workload("mid")
    f, h = make_inputs(wl)
    dev = "cuda:0"
    f_t = torch.from_numpy(f).to(dev)
    h_t = torch.from_numpy(h).to(dev)
    samples = wl.samples

    results = {}
    outputs = {}
    for prec in ("fp64", "fp32"):
        torch.cuda.synchronize()
        tp = time.perf_counter()
        plan = api.Plan(api.desc_for(wl, precision=prec), device=0)   # synchronous
        plan_ms = (time.perf_counter() - tp) * 1e3
        g_t = plan.empty_output()
        wall, per, cpl, syn = time_forward(plan, f_t, h_t, g_t, args.steps, args.warmup, torch,
                                           api)
        results[prec] = dict(plan=plan, wall=wall, per=per, cpl=cpl, syn=syn, plan_ms=plan_ms,
                             out_bytes=g_t.numel() * g_t.element_size())
        outputs[prec] = g_t
        log(f"{prec}: forward {per.mean():.3f} ms (p50 {np.percentile(per, 50):.3f}, "
            f"p99 {np.percentile(per, 99):.3f}), coupling {cpl.mean():.4f} ms, "
            f"synthesis alone {syn.mean():.3f} ms, "
            f"{samples / (per.mean() * 1e-3):.3e} samples/s")

    # the practical write ceiling on this device: hipMemsetAsync of a buffer the size of
    # the FP64 output, timed like the forward on the same stream
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemsetAsync.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
    hip.hipMemsetAsync.restype = ctypes.c_int
    g64 = torch.empty_like(outputs["fp64"])
    nbytes = g64.numel() * g64.element_size()
    stream = torch.cuda.current_stream()
    fill = lambda: hip.hipMemsetAsync(ctypes.c_void_p(g64.data_ptr()), 0, nbytes,
                                      ctypes.c_void_p(stream.cuda_stream))
    if fill() != 0:
        raise RuntimeError("hipMemsetAsync failed")
    torch.cuda.synchronize()
    fs_, fe_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fs_.record()
    for _ in range(5):
        fill()
    fe_.record()
    torch.cuda.synchronize()
    fill_gbs = nbytes * 5 / (fs_.elapsed_time(fe_) * 1e-3) / 1e9
    log(f"hipMemsetAsync of a buffer the size of the FP64 output: {fill_gbs:.0f} GB/s")
    del g64
    torch.cuda.empty_cache()

    # inverse of the FP64 output (Section III-C): reads all of g once
    plan64 = results["fp64"]["plan"]
    f_out = torch.empty(plan64.n_lm, dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()
    plan64.inverse(outputs["fp64"], h_t, f_out, stream=stream)
    torch.cuda.synchronize()
    iev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(5)]
    for s_, e_ in iev:
        s_.record(stream)
        plan64.inverse(outputs["fp64"], h_t, f_out, stream=stream)
        e_.record(stream)
    torch.cuda.synchronize()
    inv_ms = float(np.mean([s_.elapsed_time(e_) for s_, e_ in iev]))
    lm0 = wl.l_lo * wl.l_lo
    f_ref = torch.from_numpy(f[lm0:lm0 + plan64.n_lm]).to(dev)
    inv_err = float((f_out - f_ref).abs().max() / f_ref.abs().max())
    inv_bytes = results["fp64"]["out_bytes"]
    inverse_obj = {"workload": "inverse of the mid FP64 output (11.3 GB read once)",
                   "ms": inv_ms, "max_rel_err_vs_input": inv_err,
                   "roofline": {"bound": "hbm", "achieved": inv_bytes / (inv_ms * 1e-3) / 1e9,
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": inv_bytes / (inv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}
    log(f"inverse: {inv_ms:.3f} ms, {inv_bytes / (inv_ms * 1e-3) / 1e9:.0f} GB/s, "
        f"max rel err vs input {inv_err:.2e}")
    del f_out

    r = results["fp64"]
    ms = float(r["per"].mean())
    kern_ms = float(r["syn"].mean())
    # algorithmic bytes of the synthesis kernel per launch: the output written once, plus
    # the Wigner-d table, coupling coefficients, window and twiddles read once
    L = wl.L_h
    table_bytes = wl.n_theta * (L * (L + 1) * (2 * L + 1) // 6) * 8     # canonical d entries
    in_bytes = wl.n_lm * L * L * 16 + L * L * 16 + table_bytes
    alg_bytes = r["out_bytes"] + in_bytes
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    digest = kernel_source_digest()
    traffic = committed_traffic("synth_full_mid_fp64_counters.txt", digest)

    line = {
        "metric": METRIC,
        "value": samples / (ms * 1e-3),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "p50_ms": float(np.percentile(r["per"], 50)),
        "p99_ms": float(np.percentile(r["per"], 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "mid: L_f=128, L_h=8, l in [32,48) all m (1280 (l,m)), "
                               "271 phi x 136 theta x 15 omega SO(3) grid, FP64, complex128 output",
                   "samples_per_step": samples, "output_bytes_per_step": r["out_bytes"]},
        "roofline": {"bound": "hbm", "kernel": KERNEL, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel_ms": kern_ms,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "measured_fill_GBps": fill_gbs, "frac_of_measured_fill": achieved / fill_gbs,
                     "kernel_source_sha256_16": digest},
    }
    line["stages"] = {"plan_ms": r["plan_ms"], "coupling_ms": float(r["cpl"].mean()),
                      "synthesis_ms": kern_ms,
                      "note": "plan = Wigner-d table and twiddles (host wall time, once per "
                              "descriptor); coupling and synthesis (slsht_synthesize from the "
                              "coupling) each timed alone with HIP events on the launch stream"}
    line["inverse_mid"] = inverse_obj
    r32 = results["fp32"]
    ms32 = float(r32["per"].mean())
    k32 = float(r32["syn"].mean())
    table32 = table_bytes // 2
    alg32 = r32["out_bytes"] + wl.n_lm * L * L * 16 + L * L * 16 + table32
    line["fp32_mixed"] = {"value": samples / (ms32 * 1e-3), "ms_per_step": ms32,
                          "p50_ms": float(np.percentile(r32["per"], 50)),
                          "p99_ms": float(np.percentile(r32["per"], 99)),
                          "dtype": "f32 (Wigner-d and 3j in f64)",
                          "roofline": {"bound": "hbm", "achieved": alg32 / (k32 * 1e-3) / 1e9,
                                       "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": alg32 / (k32 * 1e-3) / 1e9 / HBM_PEAK_GBS}}

    if not args.no_next:
        legs = set(x.strip() for x in args.legs.split(",") if x.strip())
        if "steerable" in legs:
            line["steerable_mid"] = steerable_leg(torch, api, args.steps, args.warmup)
        if "windows" in legs:
            line["windows_mid"] = windows_leg(torch, api, f_t, outputs["fp64"], args.steps,
                                              args.warmup)
        if "slepian" in legs:
            line["slepian_window"] = slepian_leg(api)
        if "factored" in legs:
            line["factored_route"] = factored_leg(torch, api)
        if "lh16" in legs:
            line["full_lh16"] = full_lh16_leg(torch, api, 5, 2)

    # the mid-size outputs (17 GB) stay resident for the error check below; the other legs
    # fit beside them in 288 GB of HBM
    line["tiny"] = tiny_leg(torch, api, args.steps, args.warmup)
    if not args.no_energy:
        line["energy_large"] = energy_leg(torch, api, args.steps_energy)
    if not args.no_serve:
        line["serving"] = serving_leg(args.serve_n, args.serve_rate)
        sat = serving_leg(args.serve_n, args.serve_rate_sat)
        line["serving"]["saturated"] = {k: sat[k] for k in ("arrival_rate_hz", "value", "unit",
                                                            "span_s", "p50_ms", "p99_ms")}

    if not args.no_cpu:
        log("CPU baseline: oracle on a sample of rotations")
        idx, ref, dt, threads = cpu_baseline(wl, f, h, args.cpu_budget)
        n_s = idx.shape[0] * wl.n_lm
        line["cpu_baseline"] = {"value": n_s / dt, "unit": "samples/s", "cores": threads,
                                "kind": "oracle",
                                "sample": f"{idx.shape[0]} seeded rotations x all 1280 (l,m) of "
                                          f"the same workload ({n_s} samples, {dt:.1f} s, FP64 "
                                          f"direct quadrature, numpy/BLAS)"}
        errs = {}
        for prec in ("fp64", "fp32"):
            g = outputs[prec]
            a = torch.as_tensor(idx[:, 0], device=dev)
            b = torch.as_tensor(idx[:, 1], device=dev)
            c = torch.as_tensor(idx[:, 2], device=dev)
            got = g[:, c, b, a].transpose(0, 1).cpu().numpy().astype(np.complex128)
            e = rel_err_per_l(got, ref, wl.l_lo, wl.l_hi)
            per_l = {}
            for k, l in enumerate(range(wl.l_lo, wl.l_hi)):
                sl = slice(l * l - wl.l_lo ** 2, (l + 1) ** 2 - wl.l_lo ** 2)
                per_l[str(l)] = {"rel_frobenius": e[k],
                                 "max_abs": float(np.abs(got[:, sl] - ref[:, sl]).max())}
            errs[prec] = {"max_rel_frobenius_per_l": max(e),
                          "max_abs": float(np.abs(got - ref).max()),
                          "max_abs_ref": float(np.abs(ref).max()),
                          "per_l": per_l}
        errs["rotations"] = int(idx.shape[0])
        line["error_vs_oracle"] = errs
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Serving loop on the GPU: continuous batching through slsht_submit / slsht_poll.

A mix of uneven requests (band-limits, l-windows, precisions, output kinds) is
submitted at once into a budget that forces queueing; every result must equal,
bit for bit, the same transform run alone through a plan, the server must never
hold more than its budget, and the error paths must report the documented
statuses.
"""
import numpy as np
import pytest

from oracle.slsht import oracle_g_grid
from paper_1207_5558_amd import _lib as L
from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import (ServingRequest, draw_coefficients, draw_window,
                                        grid_dims, serving_stream)
from paper_1207_5558_amd.serving import Server, request_desc, run_stream
from tests.gpu_util import FP32_TOL, FP64_TOL, announce, dev, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _mix(n, seed=3):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        L_f = int(rng.choice([12, 20, 33]))
        L_h = int(rng.choice([3, 4, 8, 16]))
        l_lo = int(rng.integers(0, L_f - 4))
        reqs.append(ServingRequest(0.0, L_f, L_h, l_lo, l_lo + 5,
                                   "fp64" if i % 2 else "fp32", 1000 + i))
    return reqs


def _alone(req, f, h, output="full"):
    n_phi, n_theta, n_omega = req.grid
    plan = api.Plan(api.make_desc(req.L_f, req.L_h, req.l_lo, req.l_hi, n_phi, n_theta, n_omega,
                                  precision=req.precision, output=output))
    return plan.forward(dev(f), dev(h)).cpu().numpy().ravel()


@pytest.mark.parametrize("roomy", [False, True])
def test_mix_equals_alone_bitwise(roomy):
    """roomy=False: a budget of three of the largest outputs forces queueing; roomy=True:
    everything is admitted in the first round, so requests that share a synthesis kernel
    run in common grids."""
    announce(f"serving mix vs alone (roomy={roomy})")
    reqs = _mix(24)
    inputs = [r.inputs() for r in reqs]
    biggest = max(api.footprint(request_desc(r))[1] for r in reqs)
    budget = (4 << 30) if roomy else 3 * biggest + (64 << 20)
    srv = Server(hbm_budget=budget, n_streams=4)
    tickets = [srv.submit(request_desc(r), f, h) for r, (f, h) in zip(reqs, inputs)]
    u, b, q, running = srv.stats()
    assert u <= b
    results = {}
    for i, t in enumerate(tickets):
        srv.wait(t, 120000)
        st, ptr, n, err = srv.poll(t)
        assert st == L.REQ_DONE, (i, st, err)
        results[i] = srv.result(t, np.complex128 if reqs[i].precision == "fp64" else np.complex64)
        srv.release(t)
        u, b, _, _ = srv.stats()
        assert u <= b
    srv.close()
    for i, r in enumerate(reqs):
        alone = _alone(r, *inputs[i])
        assert np.array_equal(results[i], alone), i


def test_stream_respects_budget_and_matches_oracle():
    """A short Poisson stream shaped like the serving workload (width-8 windows,
    L_h in {4,8,16}, half FP64 / half FP32), scaled down in L_f; two results are
    checked against the oracle on sampled rotations."""
    announce("serving stream")
    reqs = serving_stream(30, rate_hz=400.0, seed=11, L_f_choices=(16, 24, 32))
    srv = Server(hbm_budget=2 << 30, n_streams=4)
    res = run_stream(srv, reqs, keep=lambda i: i in (0, 1))
    budget = srv.stats()[1]
    srv.close()
    assert np.all(np.isfinite(res["latency_s"])) and np.all(res["latency_s"] > 0)
    assert res["peak_used_bytes"] <= budget
    for i in (0, 1):
        r = reqs[i]
        f, h = r.inputs()
        n_phi, n_theta, n_omega = r.grid
        rng = np.random.default_rng(i)
        idx = np.stack([rng.integers(0, n_phi, 40), rng.integers(0, n_theta, 40),
                        rng.integers(0, n_omega, 40)], 1)
        ref = oracle_g_grid(f, h, r.L_f, r.L_h, r.l_lo, r.l_hi, n_phi, n_theta, n_omega, idx)
        g = res["kept"][i].reshape(-1, n_omega, n_theta, n_phi)
        got = g[:, idx[:, 2], idx[:, 1], idx[:, 0]].T
        tol = FP64_TOL if r.precision == "fp64" else FP32_TOL
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol


def test_energy_requests_and_error_paths():
    announce("serving energy + errors")
    rng = np.random.default_rng(9)
    f = draw_coefficients(rng, 20)
    h = draw_window(rng, 8)
    n_phi, n_theta, n_omega = grid_dims(20, 8)
    d_e = api.make_desc(20, 8, 4, 12, n_phi, n_theta, n_omega, precision="fp32", output="energy")
    srv = Server(hbm_budget=256 << 20, n_streams=2)
    t = srv.submit(d_e, f, h)
    srv.wait(t)
    got = srv.result(t, np.float32)
    plan = api.Plan(d_e)
    assert np.array_equal(got, plan.forward(dev(f), dev(h)).cpu().numpy().ravel())
    srv.release(t)
    with pytest.raises(L.SlshtError) as e:
        srv.release(t)
    assert e.value.status == L.SLSHT_ENOTFOUND
    big = api.make_desc(192, 16, 176, 184, *grid_dims(192, 16))
    with pytest.raises(L.SlshtError) as e:
        srv.submit(big, np.zeros(192 * 192, complex), np.zeros(256, complex))
    assert e.value.status == L.SLSHT_ETOOBIG
    bad = api.make_desc(20, 8, 4, 40, n_phi, n_theta, n_omega)
    with pytest.raises(L.SlshtError) as e:
        srv.submit(bad, f, h)
    assert e.value.status == L.SLSHT_EINVAL
    srv.close()


def test_serving_shapes_in_a_queued_mix():
    """The serving workload's shapes, including L_f = 192 with L_h = 16 in FP64 and FP32,
    submitted at once into a budget below their total (12 GiB for ~33 GB of outputs), so
    that admission queues: every result equals the same transform run alone (compared on
    the device), and the two L_f = 192, L_h = 16 results match the oracle on sampled
    rotations."""
    announce("serving shapes in a queued mix")
    shapes = [(192, 16, 0, 8, "fp64"), (192, 16, 8, 16, "fp32"), (128, 8, 40, 48, "fp64"),
              (96, 16, 20, 28, "fp32"), (64, 4, 56, 64, "fp64"), (32, 16, 24, 32, "fp32"),
              (192, 8, 30, 38, "fp32"), (128, 16, 0, 8, "fp64"), (160, 4, 100, 108, "fp64"),
              (32, 8, 0, 8, "fp32")]
    reqs = [ServingRequest(0.0, L_f, L_h, lo, hi, prec, 3000 + i)
            for i, (L_f, L_h, lo, hi, prec) in enumerate(shapes)]
    inputs = [r.inputs() for r in reqs]
    total = sum(api.footprint(request_desc(r))[1] for r in reqs)
    budget = 12 << 30
    assert total > budget
    srv = Server(hbm_budget=budget, n_streams=4)
    tickets = [srv.submit(request_desc(r), f, h) for r, (f, h) in zip(reqs, inputs)]
    queued = srv.stats()[2]
    for i, t in enumerate(tickets):
        srv.wait(t, 120000)
        r = reqs[i]
        dt = torch.complex128 if r.precision == "fp64" else torch.complex64
        got = srv.result_device(t, dt)
        srv.release(t)
        n_phi, n_theta, n_omega = r.grid
        f, h = inputs[i]
        plan = api.Plan(api.make_desc(r.L_f, r.L_h, r.l_lo, r.l_hi, n_phi, n_theta, n_omega,
                                      precision=r.precision))
        alone = plan.forward(dev(f), dev(h)).reshape(-1)
        assert torch.equal(got, alone), (i, shapes[i])
        if i < 2:
            rng = np.random.default_rng(50 + i)
            idx = np.stack([rng.integers(0, n_phi, 30), rng.integers(0, n_theta, 30),
                            rng.integers(0, n_omega, 30)], 1)
            ref = oracle_g_grid(f, h, r.L_f, r.L_h, r.l_lo, r.l_hi, n_phi, n_theta, n_omega, idx)
            g = got.reshape(-1, n_omega, n_theta, n_phi)
            a = torch.as_tensor(idx[:, 0], device=g.device)
            b = torch.as_tensor(idx[:, 1], device=g.device)
            c = torch.as_tensor(idx[:, 2], device=g.device)
            sample = g[:, c, b, a].transpose(0, 1).cpu().numpy()
            tol = FP64_TOL if r.precision == "fp64" else FP32_TOL
            assert np.linalg.norm(sample - ref) / np.linalg.norm(ref) <= tol, i
        del got, alone, plan
        torch.cuda.empty_cache()
    srv.close()
    assert queued > 0


def test_device_copies_survive_immediate_reuse():
    """A saturated stream whose blocks are reused as soon as they are released: results
    copied out on the device (Server.result_device) must equal the same transform run alone,
    i.e. the copy has completed before the ticket is released."""
    announce("serving device copies under reuse")
    reqs = serving_stream(300, rate_hz=1e5, seed=13, L_f_choices=(24, 32))
    srv = Server(hbm_budget=3 << 30, n_streams=4)
    keep = set(range(0, len(reqs), 3))
    res = run_stream(srv, reqs, keep=lambda i: i in keep, keep_on_device=True)
    srv.close()
    for i in sorted(keep):
        r = reqs[i]
        f, h = r.inputs()
        n_phi, n_theta, n_omega = r.grid
        plan = api.Plan(api.make_desc(r.L_f, r.L_h, r.l_lo, r.l_hi, n_phi, n_theta, n_omega,
                                      precision=r.precision))
        alone = plan.forward(dev(f), dev(h)).reshape(-1)
        assert torch.equal(res["kept"][i], alone), (i, r)

"""The forward and inverse entry points enqueue only kernels (no allocation, no memset, no
host synchronisation), so a caller can capture them in a HIP graph: every replay must equal
the eager result bit for bit, with the program's own eager work and synchronisations
between replays."""
import numpy as np
import pytest

from paper_1207_5558_amd import api
from paper_1207_5558_amd.inputs import draw_coefficients, draw_window, grid_dims, make_inputs, workload
from tests.gpu_util import announce, dev, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _replays_match(capture, outputs, eager, n=4):
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        capture(stream)                                   # warm-up outside the graph
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        capture(stream)
    for i in range(n):
        for o in outputs:
            o.fill_(float("nan"))                         # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for o, e in zip(outputs, eager):
            assert torch.equal(o, e), f"replay {i} differs"


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forward_graph_replays_equal_eager(prec):
    announce(f"graph forward {prec}")
    wl = workload("tiny")
    f, h = make_inputs(wl)
    plan = api.Plan(api.desc_for(wl, precision=prec))
    ft, ht = dev(f), dev(h)
    eager = plan.forward(ft, ht).clone()
    g = plan.empty_output()
    _replays_match(lambda s: plan.forward(ft, ht, g, stream=s), [g], [eager])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forward_and_inverse_graph_replays_equal_eager(prec):
    """slsht_inverse reads h_0^0 in its kernel, so forward + inverse capture as one graph."""
    announce(f"graph forward + inverse {prec}")
    wl = workload("tiny")
    f, h = make_inputs(wl)
    plan = api.Plan(api.desc_for(wl, precision=prec))
    ft, ht = dev(f), dev(h)
    g_e = plan.forward(ft, ht)
    f_e = plan.inverse(g_e, ht).clone()
    g = plan.empty_output()
    fo = torch.empty_like(f_e)

    def step(s):
        plan.forward(ft, ht, g, stream=s)
        plan.inverse(g, ht, fo, stream=s)
    _replays_match(step, [g, fo], [g_e, f_e])


def test_energy_and_batch_graph_replays_equal_eager():
    announce("graph energy and batch")
    rng = np.random.default_rng(81)
    L_f, L_h = 24, 8
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h)
    f = dev(draw_coefficients(rng, L_f, 2.0, True))
    h = dev(draw_window(rng, L_h))
    pe = api.Plan(api.make_desc(L_f, L_h, 4, 12, n_phi, n_theta, n_omega, precision="fp32",
                                output="energy"))
    p1 = api.Plan(api.make_desc(L_f, L_h, 0, 8, n_phi, n_theta, n_omega))
    p2 = api.Plan(api.make_desc(L_f, L_h, 8, 16, n_phi, n_theta, n_omega))
    e_eager = pe.forward(f, h).clone()
    b_eager = [g.clone() for g in api.forward_batch([p1, p2], [f, f], [h, h])]
    ge = pe.empty_output()
    gb = [p1.empty_output(), p2.empty_output()]

    def capture(s):
        pe.forward(f, h, ge, stream=s)
        api.forward_batch([p1, p2], [f, f], [h, h], gb, stream=s)

    _replays_match(capture, [ge] + gb, [e_eager] + b_eager)


def test_large_lds_launches_graph_replays_equal_eager():
    """L_h = 32: the energy kernel and the batched synthesis need more than 64 KB of LDS,
    so their launches also set the kernels' LDS attribute, inside the capture too."""
    announce("graph L_h=32 energy and batch")
    rng = np.random.default_rng(82)
    L_f, L_h = 40, 32
    n_phi, n_theta, n_omega = grid_dims(L_f, L_h)
    f = dev(draw_coefficients(rng, L_f, 2.0, True))
    h = dev(draw_window(rng, L_h))
    pe = api.Plan(api.make_desc(L_f, L_h, 30, 32, n_phi, n_theta, n_omega, precision="fp32",
                                output="energy"))
    p1 = api.Plan(api.make_desc(L_f, L_h, 30, 31, n_phi, n_theta, n_omega, theta_lo=10,
                                theta_hi=14))
    p2 = api.Plan(api.make_desc(L_f, L_h, 60, 62, n_phi, n_theta, n_omega, theta_lo=40,
                                theta_hi=42))
    e_eager = pe.forward(f, h).clone()
    b_eager = [g.clone() for g in api.forward_batch([p1, p2], [f, f], [h, h])]
    ge = pe.empty_output()
    gb = [p1.empty_output(), p2.empty_output()]

    def capture(s):
        pe.forward(f, h, ge, stream=s)
        api.forward_batch([p1, p2], [f, f], [h, h], gb, stream=s)

    _replays_match(capture, [ge] + gb, [e_eager] + b_eager)

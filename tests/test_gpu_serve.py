"""GPU tests of the continuous-batching server: every result is bit-identical
alone and in the mix, matches the FP64 oracle, and admission respects the
HBM budget."""

import numpy as np
import pytest
import torch

from oracle import cbs as oc
from paper_2506_15411_amd import libcbs as L
from paper_2506_15411_amd import scenes
from paper_2506_15411_amd.serve import Server, slot_bytes, summarize

pytestmark = pytest.mark.gpu
LAM = scenes.LAMBDA0
SMALL_GRIDS = (((32, 32, 48), LAM / 6), ((48, 40, 64), LAM / 8), ((64, 64, 64), LAM / 6))


def small_trace(n=8, seed=3, rate=200.0):
    return scenes.served_trace(n, rate, seed, grids=SMALL_GRIDS)


def test_alone_and_in_the_mix_are_bit_identical(device):
    tr = small_trace()
    assert {r.kind for r in tr} == {"forward", "adjoint"}
    srv = Server(device, max_active=4, tol=1e-5)
    mixed = {r.rid: r for r in srv.run(tr, keep_fields=True, realtime=False)}
    assert len(mixed) == len(tr)
    alone_srv = Server(device, max_active=1, tol=1e-5)
    for req in tr:
        a = alone_srv.run_sequential([req], keep_fields=True)[0]
        m = mixed[req.rid]
        assert a.iterations == m.iterations
        assert torch.equal(a.E, m.E)
        if req.kind == "adjoint":
            assert torch.equal(a.E_adj, m.E_adj) and torch.equal(a.grad, m.grad)
    s = summarize(list(mixed.values()))
    assert s["not_ok"] == 0 and s["p99_latency_s"] >= s["p50_latency_s"] > 0
    srv.close()
    alone_srv.close()


def test_served_forward_matches_oracle(device):
    rng = np.random.default_rng(11)
    sc = scenes.served_scene(rng, ((48, 40, 64), LAM / 8))
    req = scenes.ServedRequest(0, "adjoint", sc, 0.0)
    srv = Server(device, max_active=2, tol=1e-7)
    res = srv.run([req], keep_fields=True, realtime=False)[0]
    g = oc.Grid(*sc.shape, sc.pitch, LAM, 1.0, sc.pml)
    Eo, _ = oc.solve_forward(g, sc.eps_r, tol=1e-10, max_iter=40000)
    ga = oc.solve_adjoint(g, sc.eps_r, oc.adjoint_point_source(g, Eo, sc.r0), tol=1e-10,
                          max_iter=40000)
    lo, hi = sc.design_box
    gref = oc.gradient(g, Eo, ga.E_s, lo, hi, scale=2.0)

    def rel(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    assert rel(res.E.cpu().numpy(), Eo) < 1e-3
    assert rel(res.E_adj.cpu().numpy(), ga.E_s) < 1e-3
    assert rel(res.grad.cpu().numpy(), gref) < 1e-3
    srv.close()


def test_admission_waits_for_memory(device):
    tr = small_trace(6, seed=5)
    big = max(slot_bytes(r.scene.shape) for r in tr)
    srv = Server(device, max_active=4, budget_bytes=big + big // 2, tol=1e-4)
    res = srv.run(tr, realtime=False)
    assert len(res) == len(tr) and all(r.status == 0 for r in res)
    assert srv.used <= srv.budget
    assert srv.refused > 0          # some admissions had to wait for memory
    srv.close()


def test_a_rejected_request_fails_alone(device):
    """A request with material inside the absorbing layer is rejected by the
    library: in the batched run and in the one-at-a-time run its result
    carries CBS_E_INVALID and nothing else, while every other request
    completes exactly as it does without the bad one in the trace."""
    import dataclasses
    tr = small_trace(6, seed=7)
    bad_scene = dataclasses.replace(tr[2].scene, eps_r=tr[2].scene.eps_r.copy())
    nx, ny, nz = bad_scene.shape
    bad_scene.eps_r[0, ny // 2, nx // 2] = 2.25
    bad = scenes.ServedRequest(99, "adjoint", bad_scene, tr[2].arrival)
    srv = Server(device, max_active=3, tol=1e-5)
    ref = {r.rid: r for r in srv.run(tr, keep_fields=True, realtime=False)}
    for run in (lambda t: srv.run(t, keep_fields=True, realtime=False),
                lambda t: srv.run_sequential(t, keep_fields=True)):
        got = {r.rid: r for r in run(tr[:2] + [bad] + tr[2:])}
        assert got[99].status == L.CBS_E_INVALID and got[99].E is None and got[99].grad is None
        for rid, r in ref.items():
            assert got[rid].status == r.status and got[rid].iterations == r.iterations
            assert torch.equal(got[rid].E, r.E)
        assert summarize(list(got.values()))["not_ok"] == 1
    srv.close()

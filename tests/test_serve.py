"""Serving loop: admission by memory budget, continuous batching, and
results independent of the mix."""
import time

import numpy as np
import pytest

from paper_2301_01396_amd import scenes, serve


class FakeServer(serve.Server):
    """Executes no kernels: each request 'runs' for a fixed time."""

    def __init__(self, run_s=0.05, **kw):
        super().__init__(**kw)
        self.run_s = run_s

    def _make_stream(self):
        return None

    def _run_one(self, req, stream):
        time.sleep(self.run_s)
        req.result = {"rid": req.rid}


class CancellingFake(FakeServer):
    """As FakeServer, but a request cancelled while it 'runs' returns no
    result (the real server stops at its next call boundary)."""

    def _run_one(self, req, stream):
        time.sleep(self.run_s)
        if not req.cancelled:
            req.result = {"rid": req.rid}


def _reqs(n, gap, size=5):
    out = []
    for i in range(n):
        sc = scenes.small_cloth(n=size)
        out.append(serve.Request(rid=i, scene=sc, n_frames=2, arrival=i * gap))
    return out


def test_requests_arriving_mid_flight_are_admitted_and_overlap():
    srv = FakeServer(run_s=0.2, slots=4, hbm_budget=1 << 40)
    rep = srv.run(_reqs(6, gap=0.03))
    assert rep["requests"] == 6
    assert rep["max_concurrent"] >= 4          # later arrivals joined running ones
    # every request started after it arrived
    assert all(r.admitted >= r.arrival - 1e-6 for r in srv._finished)


def test_admission_respects_memory_budget():
    reqs = _reqs(4, gap=0.0)
    one = serve.estimate_bytes(reqs[0].scene, 2, False)
    srv = FakeServer(run_s=0.05, slots=4, hbm_budget=int(1.5 * one))
    rep = srv.run(reqs)
    assert rep["requests"] == 4 and rep["max_concurrent"] == 1
    srv = FakeServer(run_s=0.05, slots=4, hbm_budget=int(2.5 * one))
    assert srv.run(_reqs(4, gap=0.0))["max_concurrent"] == 2


def test_cancelled_requests_leave_the_others_unaffected():
    """Two slots, four requests at t = 0: request 0 is cancelled while it
    runs, request 3 while it waits; 1 and 2 complete with their results."""
    import threading
    srv = CancellingFake(run_s=0.3, slots=2, hbm_budget=1 << 40)
    timer = threading.Timer(0.1, lambda: (srv.cancel(0), srv.cancel(3)))
    timer.start()
    rep = srv.run(_reqs(4, gap=0.0))
    timer.join()
    assert rep["requests"] == 2 and rep["cancelled"] == 2
    assert sorted(r.rid for r in srv._finished) == [1, 2]
    assert all(r.result == {"rid": r.rid} for r in srv._finished)
    assert sorted(r.rid for r in srv._cancelled) == [0, 3] and all(not r.result for r in srv._cancelled)
    assert not srv.cancel(1)                      # finished: nothing to cancel


def test_each_context_is_budgeted_within_its_admitted_bytes():
    """The library part of a request's estimate becomes its context's memory
    budget, so what the library sizes (records of more frames included) is
    bounded by what admission counted; with the caller's tensors the two
    parts are the admitted bytes."""
    srv = serve.Server(slots=2, hbm_budget=1 << 40, device="cpu")
    for adjoint in (False, True):
        sc = scenes.small_cloth(n=9)
        sc.f_ext = np.zeros((40, sc.n_verts, 3))
        req = serve.Request(rid=0, scene=sc, n_frames=40, adjoint=adjoint)
        kw = srv._sim_kwargs(req)
        lib_bytes, caller_bytes = serve.estimate_parts(sc, 40, adjoint)
        assert kw["hbm_budget_bytes"] == lib_bytes > 0
        assert lib_bytes + caller_bytes == serve.estimate_bytes(sc, 40, adjoint)
        # the caller's part holds at least the frames, targets, goal gradient
        # and every gradient output the request returns
        V = sc.n_verts
        need = 40 * V * 3 * 4 * (3 if adjoint else 1) + (2 * V * 3 * 4 if adjoint else 0)
        assert caller_bytes >= need


def test_sequential_is_one_slot():
    rep = FakeServer(run_s=0.02, slots=1, hbm_budget=1 << 40).run(_reqs(5, gap=0.0))
    assert rep["max_concurrent"] == 1 and rep["requests"] == 5


def test_mix_generator_is_seeded_and_bounded():
    a = serve.make_mix(6, qps=2.0, seed=6, vmax=20000)
    b = serve.make_mix(6, qps=2.0, seed=6, vmax=20000)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    assert all(1000 * 0.5 <= r.scene.n_verts <= 20000 * 1.3 for r in a)
    assert all(30 <= r.n_frames <= 120 for r in a)


@pytest.mark.gpu
def test_results_are_the_same_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mix = serve.make_mix(8, qps=50.0, seed=6, vmax=6000, frames_scale=0.1)
    srv = serve.Server(slots=4, hbm_budget=32 << 30)
    rep = srv.run(mix)
    assert rep["requests"] == 8 and rep["max_concurrent"] >= 2
    by_id = {r.rid: r for r in srv._finished}
    for r in mix[:4]:
        alone = serve.make_mix(8, qps=50.0, seed=6, vmax=6000, frames_scale=0.1)[r.rid]
        alone.arrival = 0.0
        s1 = serve.Server(slots=1, hbm_budget=32 << 30)
        s1.run([alone])
        got = s1._finished[0].result
        for k, v in got.items():
            assert np.array_equal(np.asarray(v), np.asarray(by_id[r.rid].result[k])), (r.rid, k)


@pytest.mark.gpu
def test_cancelling_requests_mid_mix_leaves_the_others_bitwise_unchanged():
    import threading
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mix = serve.make_mix(6, qps=50.0, seed=6, vmax=6000, frames_scale=0.1)
    srv = serve.Server(slots=2, hbm_budget=32 << 30)
    timer = threading.Timer(0.05, lambda: (srv.cancel(0), srv.cancel(5)))
    timer.start()
    rep = srv.run(mix)
    timer.join()
    done = {r.rid: r for r in srv._finished}
    assert 5 not in done and rep["requests"] + rep["cancelled"] == 6
    for rid, r in done.items():
        alone = serve.make_mix(6, qps=50.0, seed=6, vmax=6000, frames_scale=0.1)[rid]
        alone.arrival = 0.0
        s1 = serve.Server(slots=1, hbm_budget=32 << 30)
        s1.run([alone])
        for k, v in s1._finished[0].result.items():
            assert np.array_equal(np.asarray(v), np.asarray(r.result[k])), (rid, k)


@pytest.mark.gpu
@pytest.mark.parametrize("graphs", [False, True])
def test_packed_server_matches_requests_run_alone(graphs):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mix = serve.make_mix(8, qps=50.0, seed=6, vmax=6000, frames_scale=0.1)
    srv = serve.PackedServer(slots=6, hbm_budget=32 << 30, graphs=graphs, n_packs=2)
    rep = srv.run(mix)
    assert rep["requests"] == 8 and rep["max_concurrent"] >= 2
    assert rep["pack"]["rounds"] > 0
    by_id = {r.rid: r for r in srv.finished}
    for r in mix[:4]:
        alone = serve.make_mix(8, qps=50.0, seed=6, vmax=6000, frames_scale=0.1)[r.rid]
        alone.arrival = 0.0
        s1 = serve.Server(slots=1, hbm_budget=32 << 30)
        s1.run([alone])
        got = s1._finished[0].result
        packed = by_id[r.rid].result
        assert "x_final" in packed and (("loss" in packed) == alone.adjoint)
        for k, v in packed.items():
            assert np.array_equal(np.asarray(v), np.asarray(got[k])), (r.rid, k)

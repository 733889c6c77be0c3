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

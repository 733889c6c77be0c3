"""Autotuner: shape buckets, candidate lists, the JSON table, and (GPU) that
the tuned simulator gives the same results as the default one."""
import json

import numpy as np
import pytest

from paper_2301_01396_amd import scenes, tune


def test_shape_key_buckets():
    a = scenes.small_cloth(n=6)
    b = scenes.small_cloth(n=7)
    t = scenes.small_tets(n=2)
    import torch
    assert tune.shape_key(a, torch.float32) != tune.shape_key(a, torch.float64)
    assert tune.shape_key(a, torch.float32).endswith("dbc")
    assert tune.shape_key(t, torch.float32).endswith(":t")
    # 36 and 49 vertices share the 2^5 bucket but differ in set count or not
    assert tune.shape_key(a, torch.float32).split(":")[1] == tune.shape_key(b, torch.float32).split(":")[1]


def test_candidates_cover_every_launch_structure():
    sc = scenes.config_c2(n_frames=1, n=64, tile=16)
    c = tune.candidates(sc)
    assert {x["launch_mode"] for x in c} == {1, 2}
    assert any(x["use_groups"] for x in c)
    plain = scenes.small_cloth(n=6)
    assert not any(x["use_groups"] for x in tune.candidates(plain))


def test_table_round_trip(tmp_path):
    import torch
    p = str(tmp_path / "t.json")
    sc = scenes.small_cloth(n=6)
    assert tune.lookup(sc, torch.float32, p) is None
    with open(p, "w") as f:
        json.dump({tune.shape_key(sc, torch.float32): {"launch_mode": 2, "use_groups": 0, "persistent_blocks": 64}}, f)
    assert tune.lookup(sc, torch.float32, p)["persistent_blocks"] == 64


def test_packed_server_takes_the_tuned_pack_shape(tmp_path, monkeypatch):
    import torch
    from paper_2301_01396_amd import serve
    p = str(tmp_path / "t.json")
    assert {(c["block_size"], c["graphs"]) for c in tune.pack_candidates()} == {
        (b, g) for b in (64, 128, 256) for g in (0, 1)}
    with open(p, "w") as f:
        json.dump({tune.pack_key(torch.float32): {"block_size": 64, "graphs": 0}}, f)
    monkeypatch.setattr(tune, "TABLE", p)
    monkeypatch.setattr(tune.lookup_pack, "__defaults__", (torch.float32, p))
    srv = serve.PackedServer(device="cpu")
    assert srv.block_size == 64 and srv.graphs is False
    srv = serve.PackedServer(device="cpu", graphs=True, block_size=128)      # explicit shapes win
    assert srv.block_size == 128 and srv.graphs is True
    monkeypatch.setattr(tune.lookup_pack, "__defaults__", (torch.float32, str(tmp_path / "none.json")))
    srv = serve.PackedServer(device="cpu")
    assert srv.block_size == 0 and srv.graphs is True


@pytest.mark.gpu
def test_tuned_pack_matches_every_shape():
    """tune_pack over a small mix; every pack shape gives the same results."""
    import torch
    from tests._cases import needs_gpu
    from paper_2301_01396_amd import serve
    needs_gpu()
    reqs = serve.make_mix(4, qps=100.0, seed=9, vmax=3000, frames_scale=0.05)
    best = tune.tune_pack(reqs, torch.float32, slots=8, path=None)
    assert len(best["timings"]) == len(tune.pack_candidates())
    outs = []
    for cfg in tune.pack_candidates():
        for r in reqs:
            r.arrival, r.result = 0.0, {}
        serve.PackedServer(slots=8, graphs=bool(cfg["graphs"]), block_size=cfg["block_size"]).run(reqs)
        outs.append({r.rid: r.result["x_final"] for r in reqs})
    for o in outs[1:]:
        for k, v in o.items():
            assert np.array_equal(outs[0][k], v)


@pytest.mark.gpu
def test_tuned_simulator_matches_default(tmp_path):
    import torch
    from tests._cases import needs_gpu
    from paper_2301_01396_amd.lib import Simulator
    needs_gpu()
    sc = scenes.config_c2(n_frames=1, n=64, tile=16)
    sc.substeps, sc.iterations = 2, 4
    best = tune.tune(sc, torch.float32, frames=1, path=str(tmp_path / "t.json"))
    assert len(best["timings"]) == len(tune.candidates(sc))
    outs = []
    for cfg in [best] + tune.candidates(sc):
        sim = Simulator(sc, dtype=torch.float32, launch_mode=cfg["launch_mode"],
                        persistent_blocks=cfg["persistent_blocks"], use_groups=bool(cfg["use_groups"]),
                        block_size=cfg["block_size"], group_records=cfg["group_records"],
                        group_block=cfg["group_block"])
        xf, xe, ve = sim.forward(1)
        outs.append(xe.cpu().numpy())
        sim.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)

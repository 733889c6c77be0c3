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

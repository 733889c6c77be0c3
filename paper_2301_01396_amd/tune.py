"""Launch-shape autotuner.

Every launch structure the library offers computes bit-identical results
(one launch per independent set at any workgroup size, LDS group launches
with records staged in LDS or streamed at several workgroup sizes, the
persistent frame kernel at any grid size), so the choice is purely a
performance one.  The
tuner times a short forward + adjoint rollout for each candidate and keeps
the fastest per shape bucket (dtype, log2 of the vertex count, sets per
iteration, groups, constraint mix) in a JSON table.  Packs are tuned the
same way on a request mix (their workgroup size and whether rounds replay
from HIP graphs); the packed server reads that entry.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from .lib import Simulator

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def shape_key(scene, dtype: torch.dtype) -> str:
    mix = "".join(t for t, n in (("d", scene.n_dist), ("b", scene.n_bend), ("t", scene.n_tet)) if n)
    if scene.contact:
        mix += "c"
    return (f"{'f64' if dtype == torch.float64 else 'f32'}:v2^{int(math.log2(max(scene.n_verts, 1)))}:"
            f"sets{len(scene.set_type)}:groups{len(getattr(scene, 'groups', []) or [])}:{mix}")


def candidates(scene) -> List[Dict[str, int]]:
    """Every result-invariant launch shape: one launch per set at several
    workgroup sizes, LDS group launches (if the schedule has groups), the
    persistent frame kernel at several grid sizes."""
    base = {"group_records": 0, "group_block": 0}
    c = [dict(base, launch_mode=1, use_groups=0, persistent_blocks=0, block_size=bs) for bs in (128, 256, 512)]
    if getattr(scene, "groups", None):
        for rec, gb in ((1, 256), (2, 64), (2, 128), (2, 256)):
            c.append({"launch_mode": 1, "use_groups": 1, "persistent_blocks": 0, "block_size": 256,
                      "group_records": rec, "group_block": gb})
    for b in (32, 64, 128):
        c.append(dict(base, launch_mode=2, use_groups=0, persistent_blocks=b, block_size=256))
    return c


def measure(scene, cfg: Dict[str, int], dtype=torch.float32, frames: int = 1, reps: int = 2) -> float:
    """Seconds for one forward + adjoint of ``frames`` frames (best of reps)."""
    sim = Simulator(scene, dtype=dtype, launch_mode=cfg["launch_mode"], persistent_blocks=cfg["persistent_blocks"],
                    use_groups=bool(cfg["use_groups"]), block_size=cfg.get("block_size", 0),
                    group_records=cfg.get("group_records", 0), group_block=cfg.get("group_block", 0))
    try:
        best = float("inf")
        mask = np.zeros(frames, np.uint8)
        mask[-1] = 1
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xf, _, _ = sim.forward(frames, for_adjoint=True)
            _, dL = sim.goal_l2(xf, xf.detach() * 0.999, mask)
            sim.adjoint(dL, mask)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best
    finally:
        sim.close()


def load_table(path: str = TABLE) -> Dict[str, dict]:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def tune(scene, dtype=torch.float32, frames: int = 1, path: Optional[str] = TABLE, log=None) -> Dict[str, int]:
    """Time every candidate on ``scene``; store and return the fastest."""
    results = []
    for cfg in candidates(scene):
        t = measure(scene, cfg, dtype, frames)
        results.append((t, cfg))
        if log:
            log(f"tune {cfg}: {t * 1e3:.2f} ms")
    results.sort(key=lambda r: r[0])
    best = dict(results[0][1])
    best["seconds"] = results[0][0]
    best["timings"] = [{"cfg": c, "seconds": t} for t, c in results]
    if path:
        table = load_table(path)
        table[shape_key(scene, dtype)] = best
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best


def lookup(scene, dtype=torch.float32, path: str = TABLE) -> Optional[Dict[str, int]]:
    return load_table(path).get(shape_key(scene, dtype))


# ---------------------------------------------------------------- packs
PACK_BLOCKS = (64, 128, 256)


def pack_key(dtype: torch.dtype) -> str:
    return f"pack:{'f64' if dtype == torch.float64 else 'f32'}"


def pack_candidates() -> List[Dict[str, int]]:
    """Launch shapes of a pack (all give bitwise the same results): the
    workgroup size of its set and vertex launches (1, 2 or 4 waves, one item
    per thread), with rounds launched directly or replayed from HIP graphs."""
    return [{"block_size": b, "graphs": g} for g in (0, 1) for b in PACK_BLOCKS]


def measure_pack(requests, cfg: Dict[str, int], dtype=torch.float32, slots: int = 32) -> float:
    """Seconds for the packed server to run ``requests`` (all queued at t = 0)
    with this launch shape."""
    from .serve import PackedServer
    for r in requests:
        r.arrival, r.admitted, r.done, r.result = 0.0, -1.0, -1.0, {}
    rep = PackedServer(slots=slots, dtype=dtype, graphs=bool(cfg["graphs"]), block_size=cfg["block_size"],
                       n_packs=1).run(requests)
    return rep["wall_s"]


def tune_pack(requests, dtype=torch.float32, slots: int = 32, path: Optional[str] = TABLE,
              log=None) -> Dict[str, int]:
    """Time every pack launch shape on a request mix; store and return the
    fastest (the packed server reads it when it is not given a shape)."""
    measure_pack(requests[:2], {"block_size": 256, "graphs": 0}, dtype, slots)   # warm up
    results = []
    for cfg in pack_candidates():
        t = measure_pack(requests, cfg, dtype, slots)
        results.append((t, cfg))
        if log:
            log(f"tune pack {cfg}: {t * 1e3:.1f} ms")
    results.sort(key=lambda r: r[0])
    best = dict(results[0][1])
    best["seconds"] = results[0][0]
    best["timings"] = [{"cfg": c, "seconds": t} for t, c in results]
    if path:
        table = load_table(path)
        table[pack_key(dtype)] = best
        with open(path, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    return best


def lookup_pack(dtype=torch.float32, path: str = TABLE) -> Optional[Dict[str, int]]:
    return load_table(path).get(pack_key(dtype))


def simulator(scene, dtype=torch.float32, **kw) -> Simulator:
    """A Simulator with the tuned launch shape for this scene, if any."""
    cfg = lookup(scene, dtype) or {}
    return Simulator(scene, dtype=dtype, launch_mode=cfg.get("launch_mode", 0),
                     persistent_blocks=cfg.get("persistent_blocks", 0),
                     use_groups=bool(cfg.get("use_groups", 1)), block_size=cfg.get("block_size", 0),
                     group_records=cfg.get("group_records", 0), group_block=cfg.get("group_block", 0), **kw)

"""Benchmark: forward + exact-adjoint XPBD constraint projections per second.

One step = one differentiable rollout of the workload (every frame, substep,
iteration and independent set) followed by its adjoint, through the
torch.autograd binding, with inputs resident on the GPU.  Counted
projections are forward evaluations plus reverse evaluations (the adjoint's
recomputation of each frame is overhead and not counted); a tet counts its
deviatoric and hydrostatic projections, a contact constraint counts once
per evaluation.

Default workload: the 2048x4096 cloth (8,388,608 vertices, 25.2M DoF,
25.2M distance + 25.1M bending constraints), FP32, dt 1/60, 2 substeps, 20
iterations, 20 frames, per-vertex force controls, keyframe goal at frames 10
and 20, gradient with respect to every frame's forces: the configuration
whose working set is far larger than the GPU's caches, so the projection and
reverse kernels stream HBM and the roofline is HBM bandwidth.  --workload c2
(256x256 cloth with a sphere), c3 (64^3 tet box), c1 (32x32, FP64) and c5
(serving mix: p50/p99 latency and throughput, packed against one request at
a time) run the other configurations.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic bytes per projection of each kernel family in FP32 (index =
# 2 * type forward, 2 * type + 1 reverse) when one launch runs one set: the
# vertex indices, the constant data, the multiplier and the vertices each
# projection must read and write (and the record, added separately).
ALG_BYTES = {             # family: (index bytes, words of the state dtype)
    0: (8, 20), 1: (8, 26),     # distance fwd: idx 8 + L, at, lambda r/w + 2 vertices r/w
    2: (16, 36), 3: (16, 48),   # bending
    4: (8, 24), 5: (8, 31),     # tet, per projection (one tet item moves twice this)
    6: (4, 10), 7: (4, 22),     # contact
    12: (16, 35), 13: (16, 55), # membrane: Dm^-1 4, at 4, lambda r/w 6, 3 vertices r/w; reverse adds
                                # the record 12, lambda_bar r/w 6, compliance adjoint r/w 8
}


# streamed bytes per projection, the per-unit figure the roofline is priced
# on: every projection reads its constant data and multiplier (and, in the
# reverse, its record) and reads and writes its vertices in HBM, with no
# staging (forward: distance 80, bending 144, tet 98, contact 40; reverse:
# distance 116, bending 204).  Other families fall back to ALG_BYTES.
STREAMED_BYTES = {0: 80.0, 2: 144.0, 4: 98.0, 6: 40.0, 1: 116.0, 3: 204.0}


# record words written per projection by a forward that keeps the adjoint's
# record (vertex differences + multiplier): dist 4, bend 10, tet 6 (12 per
# item), contact 4
TAPE_WORDS = {0: 4, 2: 10, 4: 6, 6: 4, 12: 12}


def alg_bytes(fam: int, tsz: int, recording: float = 0.0) -> float:
    """Bytes per projection; ``recording`` = fraction of the family's
    forward launches that also write the adjoint's record (1 when the
    forward keeps the whole rollout's record, 1/2 when each frame is run
    once forward and once more by the adjoint to record it)."""
    ib, words = ALG_BYTES[fam]
    if fam in TAPE_WORDS:
        words += float(recording) * TAPE_WORDS[fam]
    return ib + words * tsz


# LDS group kernels: words moved per projection for the constraint's entry
# (constant part read: rest/theta0, at, packed vertex slots; tets B, two
# compliances, gamma) and its state (read and written: forward lambda;
# reverse lambda_bar and the compliance adjoint, tets five words per pair,
# contacts the sphere adjoint and lambda_bar), forward and reverse; the
# record of inputs is added separately.  The first iteration's launches do
# not read the state; the model counts it anyway (1 launch in K).
GROUP_REC_WORDS = {0: (5, 7), 2: (6, 8), 4: (9, 12), 6: (3, 11)}


def group_vertices(sc) -> int:
    """Vertices the LDS groups stage, summed over the groups: each group
    loads (and stores) exactly the vertices its constraints touch."""
    tot = 0
    for a, b, _ in sc.groups:
        parts = []
        for t, items in zip(sc.set_type[a:b], sc.set_items[a:b]):
            if t == 0:
                parts.append(sc.dist_v[items].ravel())
            elif t == 1:
                parts.append(sc.bend_v[items].ravel())
            elif t == 2:
                parts.append(sc.tet_v[items].ravel())
            else:
                parts.append(np.asarray(items))
        if parts:
            tot += int(np.unique(np.concatenate(parts)).size)
    return tot


def group_bytes(sc, reverse: bool, tsz: int, recording: float, staged_vertices: int,
                snapshots: bool = False, compliance_adjoints: bool = True) -> float:
    """Average algorithmic bytes per projection of the LDS group launches of
    one iteration: constant entries read, state read and written, record of
    inputs (written by the forward launches that record, read by the
    reverse), and the staged vertices of every group read and written once
    per launch.  With snapshot records the record is the launch's staged
    positions (3 words per vertex) and its multipliers (1 word per
    projection, 2 per tet item); the record the reverse replays from them
    stays within the launch (written and read back by each workgroup) and
    is not counted.  Without ``compliance_adjoints`` (no distance or bending
    compliance gradient asked for) the reverse leaves those constraints'
    compliance adjoints (a word read and written) out."""
    n = {0: sc.n_dist, 2: sc.n_bend, 4: 2 * sc.n_tet,
         6: int(np.count_nonzero(sc.inv_mass > 0)) if sc.contact else 0}
    tot = max(sum(n.values()), 1)
    share = 1.0 if reverse else float(recording)
    b = 0.0
    for f, cnt in n.items():
        words = GROUP_REC_WORDS[f][1 if reverse else 0]
        if reverse and not compliance_adjoints and f in (0, 2):
            words -= 2
        words += (1 if snapshots else TAPE_WORDS[f]) * share
        b += cnt * words * tsz
    b += staged_vertices * 2 * 4 * tsz
    if snapshots:
        b += staged_vertices * 3 * tsz * share
    return b / tot


def mix_bytes(sc, reverse: bool, tsz: int, recording: bool) -> float:
    """Average algorithmic bytes per projection over the workload's mix (the
    persistent frame kernel runs every set type)."""
    n = {0: sc.n_dist, 2: sc.n_bend, 4: 2 * sc.n_tet,
         6: int(np.count_nonzero(sc.inv_mass > 0)) if sc.contact else 0}
    tot = sum(n.values())
    return sum(cnt * alg_bytes(f + (1 if reverse else 0), tsz, recording and not reverse)
               for f, cnt in n.items()) / max(tot, 1)


def streamed_bytes(sc, fam: int, tsz: int) -> float:
    """Streamed bytes per projection for a kernel family; for a
    family that runs several constraint types (LDS groups, the persistent
    frame kernel) the average over the workload's mix."""
    def one(f):
        return STREAMED_BYTES[f] * tsz / 4 if f in STREAMED_BYTES else alg_bytes(f, tsz)
    if fam in (8, 9, 10, 11):
        rev = fam in (9, 11)
        n = {0: sc.n_dist, 2: sc.n_bend, 4: 2 * sc.n_tet,
             6: int(np.count_nonzero(sc.inv_mass > 0)) if sc.contact else 0}
        tot = max(sum(n.values()), 1)
        return sum(cnt * one(f + (1 if rev else 0)) for f, cnt in n.items()) / tot
    return one(fam)


FAMILY = {0: "dist_fwd", 1: "dist_rev", 2: "bend_fwd", 3: "bend_rev", 4: "tet_fwd", 5: "tet_rev",
          6: "contact_fwd", 7: "contact_rev", 8: "frame_fwd", 9: "frame_rev", 10: "group_fwd", 11: "group_rev",
          12: "membrane_fwd", 13: "membrane_rev"}
KERNEL_SYMBOL = {0: "k_dist", 1: "k_dist_rev", 2: "k_bend", 3: "k_bend_rev", 4: "k_tet", 5: "k_tet_rev",
                 6: "k_contact", 7: "k_contact_rev", 8: "k_program(forward frame)", 9: "k_program(reverse frame)",
                 10: "k_group_fwd", 11: "k_group_rev", 12: "k_tri", 13: "k_tri_rev"}
N_FAM = len(FAMILY)
WORKLOAD_LAUNCH = {"c4": {"group_records": 2, "group_block": 256}}
# adjoint record per workload (1: snapshots of each LDS group launch, replayed
# by the reverse; needs every set in an LDS group)
WORKLOAD_RECORD = {}
# adjoint record mode per workload when --tape-mode is not given: the 256x256
# cloths follow their configuration's per-frame checkpoints (every frame's
# record recomputed from its checkpoint, tape mode 1); the others take the
# library's choice (the whole rollout if it fits, else the last frames)
WORKLOAD_TAPE = {"c2": 1, "c2m": 1, "c2b": 1}
HBM_PEAK_GBS = 8000.0

# what the parity tests establish for each workload's results, by dtype
ACCURACY = {
    ("c1", "f64"): "positions and gradients within 1e-10 / 1e-8 of the FP64 reference (full rollout)",
    ("c2", "f32"): "one full frame at full size: positions 1e-5, every gradient group 1e-3 of the FP64 reference; "
                   "the 30-frame drape is chaotic at FP32 resolution (gradients of the whole step differ from FP64 "
                   "by order one): run --dtype f64 for digits",
    ("c4", "f32"): "full size, the benchmark's adjoint structure: positions 1e-5, gradients 1e-3 of the "
                   "reference with FP32 state storage (the plain FP64 reference differs from both by 3.5e-3 "
                   "in dL/dalpha)",
    ("c3", "f64"): "full size, one frame: positions 1e-10, gradients 1e-5 of the FP64 reference",
    ("c3", "f32"): "full size, one frame: positions 1e-5, gradients within 1.2e-3 of the reference with FP32 "
                   "state storage (whose own distance from FP64 is 3-4e-3); the 20-frame step: dL/dE 1.5e-2 "
                   "from the same step in FP64",
    ("c2m", "f32"): "gradients parity unpinned: at 0.2 kg/m^2 the membrane amplifies rounding ~1e11, FP32 "
                    "storage alone moves them by more than their size; FP32 positions within twice that "
                    "intrinsic error, a full-size frame pinned in FP64; run --dtype f64 for a parity-backed "
                    "gradient",
}


# sources of the single-context kernels and their launches (the pack's
# files do not change them)
KERNEL_SOURCES = ("xpbd_device.hpp", "xpbd_kernels.hpp", "xpbd.hip")


def csrc_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2301_01396_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(name: str, tile: int = -1, frames: int = 0, lds_groups: str = "", merge: str = "",
                  tiling: str = ""):
    from paper_2301_01396_amd import scenes
    kw = {} if tile < 0 else {"tile": tile}
    if name == "c1":
        return scenes.config_c1(), scenes.config_c1(target=True)
    if name == "c2":
        return scenes.config_c2(**kw), scenes.config_c2(target=True, **kw)
    if name == "c3":
        return scenes.config_c3(**kw), scenes.config_c3(target=True, **kw)
    if name == "c2m":
        return scenes.config_c2_membrane(**kw), scenes.config_c2_membrane(target=True, **kw)
    if name == "c2b":
        return scenes.config_c2_body(**kw), scenes.config_c2_body(target=True, **kw)
    if name == "c4":
        if frames:
            kw["n_frames"] = frames
        if lds_groups:
            kw["lds_groups"] = tuple(int(ch) for ch in lds_groups)
        if merge:
            kw["merge"] = tuple(int(v) for v in merge.split(","))
        if tiling:
            kw["tiling"] = tiling
        return scenes.config_c4(**kw), None
    raise SystemExit(f"unknown workload {name}")


def workload_config(name, sc, F):
    return {"workload": {"c1": "cloth32_distance_fp64", "c2": "cloth256_dist_bend_sphere",
                         "c3": "tetbox64_neohookean", "c4": "cloth2048x4096_dist_bend_force",
                         "c2m": "cloth256_membrane_bend_sphere", "c2b": "cloth256_dist_bend_body_mesh"}[name],
            "verts": sc.n_verts, "dist": sc.n_dist, "bend": sc.n_bend, "tets": sc.n_tet,
            "contacts": int(np.count_nonzero(sc.inv_mass > 0)) if sc.contact else 0,
            "membrane_triangles": sc.n_tri, "body_triangles": sc.n_body_tris,
            "frames": F, "substeps": sc.substeps, "iterations": sc.iterations, "dt": sc.dt,
            "sets_per_iteration": len(sc.set_type), "lds_groups": len(sc.groups)}


def cpu_baseline(name, sc, max_projections: int = 60_000_000, threads: int = 0):
    """The FP64 reference on the host cores (``threads``, 0 = all the
    process may use), on a bounded prefix of the workload: one frame, with
    fewer substeps / iterations when one frame holds more than
    ``max_projections`` forward projections; forward and adjoint are both
    timed."""
    import copy
    import oracle as O
    if threads <= 0:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        threads = max(1, min(threads, os.cpu_count() or 1))
    sample = copy.copy(sc)
    per_it = sc.projections_per_iteration()
    if per_it * sc.iterations * sc.substeps > max_projections:
        sample.substeps = 1
        sample.iterations = max(1, min(sc.iterations, max_projections // max(per_it, 1)))
    frames = 1
    if sample.substeps == sc.substeps and sample.iterations == sc.iterations:
        frames = int(max(1, min(sc.n_frames, max_projections // max(sc.projections_per_rollout(1), 1))))
    osc = O.OracleScene(sample, n_threads=threads)
    kw = {}
    if sc.f_ext is not None:
        kw["f_ext"] = sc.f_ext[:frames]
    t0 = time.perf_counter()
    xf, _, _ = O.forward(osc, frames, **kw)
    t1 = time.perf_counter()
    dL = xf - xf.mean(axis=1, keepdims=True)
    O.adjoint(osc, frames, dL, **kw)
    t2 = time.perf_counter()
    proj = sample.projections_per_rollout(frames)
    value = 2 * proj / (t2 - t0)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": value, "unit": "projections/s", "cores": threads, "kind": "oracle",
            "forward_projections_per_s": proj / (t1 - t0), "adjoint_projections_per_s": proj / (t2 - t1),
            "cpu_model": model,
            "sample": f"{frames} frame(s) of the workload with {sample.substeps} substep(s) x {sample.iterations} "
                      f"iterations ({proj} forward + {proj} reverse projections, FP64): "
                      f"forward {t1 - t0:.2f} s, adjoint incl. recompute {t2 - t1:.2f} s"}


def scenes_small_for_one_core(name, sc):
    """A sample of the workload one core times in seconds: the 2048x4096
    cloth cut to 256 of its rows (same columns, tiling and parameters'
    distribution), the other workloads unchanged."""
    if name != "c4":
        return sc
    from paper_2301_01396_amd import scenes
    return scenes.config_c4(n_frames=1, nr=256)


def serve_bench(args):
    """Serving mix: sequential capacity first (one request at a time, all
    queued at t = 0), then Poisson arrivals at fractions of that capacity
    served with continuous batching; p50/p99 latency and throughput."""
    import torch
    from paper_2301_01396_amd import serve
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    reqs = serve.make_mix(args.requests, qps=1.0, seed=6)
    base = [r.arrival for r in reqs]     # Poisson arrivals at 1 request/s; rescaled per rate

    def at_rate(qps):
        for r, a in zip(reqs, base):
            r.arrival = a / qps
            r.admitted = r.done = -1.0
            r.result = {}
        return reqs

    log(f"serving mix: {len(reqs)} requests, {sum(r.scene.n_verts for r in reqs)} vertices in total")
    warm = serve.make_mix(2, qps=100.0, seed=7, vmax=4000, frames_scale=0.1)
    serve.Server(slots=2, record_whole_rollout=False).run(warm)
    seq = serve.Server(slots=1, record_whole_rollout=False).run(at_rate(1e9))
    cap = seq["throughput_rps"]
    log(f"sequential: {seq}")
    executors = {
        "streams": lambda: serve.Server(slots=args.slots, record_whole_rollout=False),
        "pack": lambda: serve.PackedServer(slots=args.pack_slots, graphs=False, n_packs=1),
        "pack_graphs": lambda: serve.PackedServer(slots=args.pack_slots, graphs=True, n_packs=1),
        "packs_graphs": lambda: serve.PackedServer(slots=args.pack_slots, graphs=True, n_packs=args.packs),
    }
    rows = []
    for frac in (0.25, 0.5, 0.75, 1.0, 1.5, 3.0, 1e9):
        for name, make in executors.items():
            rep = make().run(at_rate(frac * cap))
            rep["executor"] = name
            rep["qps"] = frac * cap if frac < 1e8 else None
            rep["qps_over_sequential_capacity"] = frac if frac < 1e8 else "all at t=0"
            rows.append(rep)
            log(f"qps {frac:g} x capacity, {name}: {rep}")
    best = max(rows, key=lambda r: r["projections_per_s"])
    out = {"metric": "constraint projections/s fwd+adjoint vs plain launch; p50/p99 request latency",
           "value": best["projections_per_s"], "unit": "projections/s", "n_gpus": 1,
           "steps": len(rows), "warmup": 1, "ms_per_step": best["wall_s"] * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic serving mix (seed 6)",
           "config": {"workload": "serving_mix", "requests": args.requests, "slots": args.slots,
                      "pack_slots": args.pack_slots, "packs": args.packs,
                      "mesh": "50% grid cloth / 50% tet box, ln V ~ N(ln 16000, 1) in [1k, 250k]",
                      "frames": "U{30..120}", "adjoint_fraction": 0.5, "substeps": 2, "iterations": 20},
           "best": {"executor": best["executor"], "qps_over_sequential_capacity": best["qps_over_sequential_capacity"],
                    "p50_latency_s": best["p50_latency_s"], "p99_latency_s": best["p99_latency_s"],
                    "throughput_rps": best["throughput_rps"]},
           "sequential": seq, "served": rows,
           "speedup_vs_sequential": best["projections_per_s"] / seq["projections_per_s"]}
    print(json.dumps(out), flush=True)


def serving_leg(n_requests: int, pack_slots: int, log) -> dict:
    """The serving part of the metric, short enough for the default line: a
    fixed mix of requests (seed 6; grid cloths and tet boxes of 1k-250k
    vertices, 30-120 frames, half with the adjoint) served one at a time with
    one launch per set (the sequential plain baseline), then by the packed
    server (every admitted request in one pack, each launch serving the same
    step of all of them) with all requests queued at t = 0 and with Poisson
    arrivals at the sequential capacity.  p50/p99 latency from arrival to
    result, requests/s and projections/s."""
    import torch
    from paper_2301_01396_amd import serve
    reqs = serve.make_mix(n_requests, qps=1.0, seed=6)
    base = [r.arrival for r in reqs]

    def at_rate(qps):
        for r, a in zip(reqs, base):
            r.arrival = a / qps
            r.admitted = r.done = -1.0
            r.result = {}
        return reqs

    keys = ("requests", "throughput_rps", "p50_latency_s", "p99_latency_s", "projections_per_s", "wall_s")
    pick = lambda rep: {k: rep.get(k) for k in keys}
    serve.Server(slots=1, record_whole_rollout=False).run(serve.make_mix(2, qps=100.0, seed=7, vmax=4000,
                                                                         frames_scale=0.1))
    seq = serve.Server(slots=1, record_whole_rollout=False).run(at_rate(1e9))
    log(f"serving, sequential plain launches: {pick(seq)}")
    cap = seq["throughput_rps"]
    sat = serve.PackedServer(slots=pack_slots, graphs=False, n_packs=1).run(at_rate(1e9))
    log(f"serving, packed, all at t = 0: {pick(sat)}")
    poi = serve.PackedServer(slots=pack_slots, graphs=False, n_packs=1).run(at_rate(cap))
    log(f"serving, packed, Poisson at the sequential capacity: {pick(poi)}")
    torch.cuda.synchronize()
    return {"requests": n_requests, "mix": "seed 6: 50% grid cloth / 50% tet box, ln V ~ N(ln 16000, 1) in "
                                           "[1k, 250k], frames U{30..120}, half with the adjoint, S 2, K 20",
            "sequential_plain": pick(seq), "packed_all_at_t0": pick(sat),
            "packed_poisson_at_sequential_capacity": dict(pick(poi), qps=cap),
            "throughput_vs_sequential": sat["projections_per_s"] / seq["projections_per_s"],
            "p50_vs_sequential": sat["p50_latency_s"] / seq["p50_latency_s"],
            "p99_vs_sequential": sat["p99_latency_s"] / seq["p99_latency_s"]}


def implicit_bench(args):
    """The paper's implicit adjoint (CG per substep) against the exact
    reverse adjoint on one workload: time of each and their gradients'
    relative difference per parameter group."""
    import torch
    from paper_2301_01396_amd.lib import Simulator
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    sc, tg = make_workload(args.workload, args.tile, args.frames, args.lds_groups, args.merge, args.tiling)
    F = args.frames or sc.n_frames
    dtype = torch.float64 if args.workload == "c1" else torch.float32
    sim = Simulator(sc, dtype=dtype)
    mask = np.zeros(F, np.uint8)
    mask[F - 1] = 1
    if tg is not None:
        tsim = Simulator(tg, dtype=dtype)
        targets, _, _ = tsim.forward(F)
        tsim.close()
    else:
        targets, _, _ = sim.forward(F)
        targets = targets * 0.99
    res = {}
    for kind in ("exact", "implicit", "exact", "implicit"):      # second pass timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xf, _, _ = sim.forward(F, for_adjoint=(kind == "exact"))
        _, dL = sim.goal_l2(xf, targets, mask)
        if kind == "exact":
            g = sim.adjoint(dL, mask, want=("x0", "v0", "dist_alpha", "bend_alpha", "f_ext"))
            rep = None
        else:
            g, rep = sim.adjoint_implicit(dL, mask, max_iterations=args.cg_iters, rel_tolerance=args.cg_tol,
                                          pd_projection=args.pd)
        torch.cuda.synchronize()
        res[kind] = {"s": time.perf_counter() - t0, "g": {k: v.double().cpu().numpy() for k, v in g.items()},
                     "cg": rep}
        log(f"{kind}: {res[kind]['s']:.3f} s {rep or ''}")
    diff = {}
    for k, a in res["exact"]["g"].items():
        b = res["implicit"]["g"].get(k)
        if b is not None and np.linalg.norm(a) > 0:
            diff[k] = float(np.linalg.norm(b - a) / np.linalg.norm(a))
    out = {"metric": "implicit adjoint (CG per substep) vs exact reverse adjoint", "workload":
           workload_config(args.workload, sc, F), "dtype": "f64" if dtype == torch.float64 else "f32",
           "exact_fwd_adjoint_s": res["exact"]["s"], "implicit_fwd_adjoint_s": res["implicit"]["s"],
           "cg": res["implicit"]["cg"], "cg_rel_tolerance": args.cg_tol, "cg_max_iterations": args.cg_iters,
           "pd_projection": bool(args.pd),
           "rel_difference_implicit_vs_exact": diff}
    print(json.dumps(out), flush=True)


def estimate_bench(args):
    """Material estimation on the tet box of the tet workload's size
    (Sec. 5.2): 100 random material clusters, a two-material target,
    fixed-step gradient descent on (a, b) (the step set from the first
    gradient so the first update changes a control by at most 5%, then kept);
    reports the time per descent
    iteration (rollout + goal + exact adjoint + update) and the goal's fall."""
    import torch
    from paper_2301_01396_amd import scenes
    from paper_2301_01396_amd.estimate import estimate_materials
    from paper_2301_01396_amd.lib import Simulator
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    n = args.estimate_n
    F = args.frames or 20
    model, tgt, d = scenes.material_estimation(n=n, frames=F)
    tsim = Simulator(tgt, dtype=torch.float32)
    targets, _, _ = tsim.forward(F, tet_mu=tsim.tensor(d["target_mu"]), tet_lambda=tsim.tensor(d["target_lambda"]))
    tsim.close()
    sim = Simulator(model, dtype=torch.float32)
    w = torch.as_tensor(d["vertex_weight"], dtype=torch.float64, device="cuda")
    estimate_materials(sim, F, targets, d["mu0"], d["lambda0"], None, 1, d["frame_mask"], w)    # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, b, losses, step = estimate_materials(sim, F, targets, d["mu0"], d["lambda0"], None, args.steps,
                                            d["frame_mask"], w,
                                            callback=lambda i, L: log(f"iteration {i}: goal {L:.6e}"))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    proj = 2 * model.projections_per_rollout(F)
    mu = (a * a).cpu().numpy()
    out = {"metric": "material estimation: fixed-step gradient descent iterations", "value": 1.0 / dt,
           "unit": "iterations/s", "ms_per_iteration": dt * 1e3, "projections_per_s": proj / dt,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"tet box {n}^3 cubes, {model.n_tet} tets, {model.n_materials} materials, "
                                  f"two-material target, {F} frames, S={model.substeps}, K={model.iterations}"},
           "goal_first": losses[0], "goal_last": losses[-1], "iterations": args.steps, "step": step,
           "mu_range": [float(mu.min()), float(mu.max())]}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "c5", "c2m", "c2b"])
    ap.add_argument("--requests", type=int, default=24, help="serving mix size (c5)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="only run a plain device copy kernel over this many bytes (counter calibration)")
    ap.add_argument("--slots", type=int, default=8, help="concurrent requests, one stream each (c5)")
    ap.add_argument("--pack-slots", type=int, default=32, help="requests in packs at once (c5)")
    ap.add_argument("--packs", type=int, default=4, help="packs, one stream each (c5)")
    ap.add_argument("--frames", type=int, default=0, help="override frame count (0 = the workload's)")
    ap.add_argument("--profile-stride", type=int, default=7,
                    help="bracket one in n projection launches (hash-picked) with HIP events (0 = off)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default="auto", choices=["auto", "plain", "persistent"])
    ap.add_argument("--blocks", type=int, default=0, help="persistent workgroups (0 = auto)")
    ap.add_argument("--tile", type=int, default=-1, help="schedule tile width (-1 = the workload's, 0 = untiled)")
    ap.add_argument("--no-groups", action="store_true", help="run every set as its own launch")
    ap.add_argument("--block", type=int, default=0, help="workgroup size of the per-set kernels (0 = 256)")
    ap.add_argument("--group-records", type=int, default=0,
                    help="LDS groups: 1 entries and state staged in LDS, 2 streamed (0 = the library's choice)")
    ap.add_argument("--group-block", type=int, default=0, help="workgroup size of the group kernels (0 = 256)")
    ap.add_argument("--tape-mode", type=int, default=0, choices=[0, 1, 2, 3, 4],
                    help="adjoint record mode (0: the workload's choice, else the library's: whole rollout if "
                         "it fits, else the last frames, else per frame; 1 recompute every frame from its "
                         "checkpoint)")
    ap.add_argument("--record-kind", type=int, default=-1, choices=[-1, 0, 1],
                    help="adjoint record: 0 every projection's inputs, 1 snapshots of each LDS group launch "
                         "replayed by the reverse (-1 = the workload's)")
    ap.add_argument("--merge", default="",
                    help="tiled cloth: border segments and corner clusters per patch, e.g. 8,16 (default: the workload's)")
    ap.add_argument("--tiling", default="", choices=["", "lines", "quads"],
                    help="tiled cloth: interiors + border lines + corners (lines) or four colours of whole "
                         "tiles (quads); default: the workload's")
    ap.add_argument("--lds-groups", default="",
                    help="tiled cloth: which of the tiling's groups (0 interiors, 1 borders, 2 corners) run as "
                         "LDS groups, e.g. 012 (default: the workload's)")
    ap.add_argument("--implicit", action="store_true",
                    help="compare the implicit (CG) adjoint with the exact one on the workload")
    ap.add_argument("--cg-iters", type=int, default=2000)
    ap.add_argument("--cg-tol", type=float, default=1e-8)
    ap.add_argument("--pd", action="store_true", help="implicit adjoint: project the blocks to PSD first")
    ap.add_argument("--estimate", action="store_true",
                    help="time material-estimation descent iterations instead (--steps iterations)")
    ap.add_argument("--estimate-n", type=int, default=64, help="cubes per side of the estimation box")
    ap.add_argument("--dtype", default="auto", choices=["auto", "f32", "f64"],
                    help="state dtype (auto: FP64 for the 32x32 cloth, FP32 otherwise)")
    ap.add_argument("--serve-requests", type=int, default=12,
                    help="requests of the serving leg of the default line (0 = skip)")
    ap.add_argument("--plain-steps", type=int, default=1,
                    help="also time this many steps with one launch per set (0 = skip)")
    args = ap.parse_args()
    # launch shape of the LDS group kernels per workload (measured fastest):
    # the 25.2M-DoF cloth streams its constraint entries and state with
    # 256-thread workgroups
    for k, v in WORKLOAD_LAUNCH.get(args.workload, {}).items():
        if getattr(args, k) == 0:
            setattr(args, k, v)
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per process: the path and its measurement run on a single GPU, --gpus must be 1"}), flush=True)
        sys.exit(2)

    import torch
    from paper_2301_01396_amd import autograd as AG
    from paper_2301_01396_amd.lib import Simulator

    if args.calibrate_copy:
        # reads and writes exactly calibrate_copy bytes per launch
        n = args.calibrate_copy // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                          "launches": 5}), flush=True)
        return
    if args.workload == "c5":
        return serve_bench(args)
    if args.estimate:
        return estimate_bench(args)
    if args.implicit:
        return implicit_bench(args)

    dev = torch.device("cuda:0")
    sc, tg = make_workload(args.workload, args.tile, args.frames, args.lds_groups, args.merge, args.tiling)
    F = args.frames or sc.n_frames
    dtype = {"f32": torch.float32, "f64": torch.float64}.get(args.dtype) or (
        torch.float64 if args.workload == "c1" else torch.float32)
    lm = {"auto": 0, "plain": 1, "persistent": 2}[args.launch]
    rk = args.record_kind if args.record_kind >= 0 else WORKLOAD_RECORD.get(args.workload, 0)
    sim = Simulator(sc, dtype=dtype, device=dev, launch_mode=lm, persistent_blocks=args.blocks,
                    use_groups=not args.no_groups, block_size=args.block, group_records=args.group_records,
                    group_block=args.group_block, record_kind=rk,
                    tape_mode=args.tape_mode or WORKLOAD_TAPE.get(args.workload, 0))
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    log(f"workload {args.workload}: {sc.n_verts} verts, {len(sc.set_type)} sets, {F} frames")

    # ---------------- targets (outside the timed region)
    mask = np.zeros(F, np.uint8)
    if args.workload == "c4":
        mask[min(9, F - 1)] = 1
        mask[F - 1] = 1
        from paper_2301_01396_amd import scenes
        f_key = sim.tensor(scenes.force_field(5, 4096, 2048, F))
        targets, _, _ = sim.forward(F, f_ext=f_key)
        del f_key
        f_ctrl = sim.tensor(sc.f_ext[:F])
    else:
        mask[F - 1] = 1
        tsim = Simulator(tg, dtype=dtype, device=dev)
        targets, _, _ = tsim.forward(F)
        tsim.close()
        f_ctrl = None
    torch.cuda.synchronize()

    x0 = sim.tensor(sc.x0)
    v0 = sim.tensor(sc.v0).requires_grad_(args.workload in ("c2", "c2m", "c2b"))
    da = sim.tensor(sc.dist_alpha).requires_grad_(args.workload in ("c1", "c2", "c2b")) if sc.n_dist else None
    ba = sim.tensor(sc.bend_alpha).requires_grad_(args.workload in ("c2", "c2m", "c2b")) if sc.n_bend else None
    te = sim.tensor(sc.tet_E).requires_grad_(True) if sc.n_tet else None
    tc = sim.tensor(sc.tri_coef).requires_grad_(True) if sc.n_tri else None
    bxx = sim.tensor(sc.body_x).requires_grad_(True) if sc.n_body_tris else None
    if f_ctrl is not None:
        f_ctrl.requires_grad_(True)
    sphere = torch.tensor(sc.sphere, dtype=torch.float64) if sc.contact else None
    leaves = [t for t in (v0, da, ba, te, f_ctrl, tc, bxx) if t is not None and t.requires_grad]

    def step(s=sim, ev=None):
        for t in leaves:
            t.grad = None
        if ev:
            ev[0].record()
        xf = AG.rollout(s, F, x0, v0, da, ba, te, f_ctrl, sphere, tri_coef=tc, body_x=bxx)
        loss = AG.goal_l2(s, xf, targets, mask)
        if ev:
            ev[1].record()
        loss.backward()
        if ev:
            ev[2].record()
        return loss

    for _ in range(args.warmup):
        step()
        log("warmup step done")
    torch.cuda.synchronize()
    sim.profile_read()
    # the persistent path launches two kernels per frame: time every one;
    # otherwise a stride coprime with the launches of one iteration
    stride = args.profile_stride
    if stride and sim.info()["persistent"]:
        stride = 1
    sim.profile_enable(stride)
    torch.cuda.synchronize()
    # phases on the call's stream (the adjoint's own streams join it before
    # the call ends): forward + goal, then the adjoint with its recomputation
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        loss = step(ev=evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = {"forward_and_goal_ms": round(sum(e[0].elapsed_time(e[1]) for e in evs) / max(args.steps, 1), 1),
              "adjoint_ms": round(sum(e[1].elapsed_time(e[2]) for e in evs) / max(args.steps, 1), 1)}
    sim.profile_enable(0)
    launches, ms, items = sim.profile_read()
    elapsed = t1 - t0
    proj_step = 2 * sc.projections_per_rollout(F)
    value = proj_step * args.steps / elapsed
    grads_finite = all(bool(torch.isfinite(t.grad).all()) for t in leaves)
    info = sim.info()
    log(f"timed {args.steps} steps: {elapsed / args.steps * 1e3:.1f} ms/step, info {info}")
    # share of forward launches that write the record: every frame is recorded
    # once, by the forward (its last forward_record_frames frames) or by the
    # adjoint's recomputation (the others, which run the forward twice)
    kept = info["forward_record_frames"] if info["tape_mode"] in (3, 4) else 0
    recording = F / (F + (F - kept)) if info["tape_mode"] in (1, 3, 4) else 0.0

    plain = None
    if args.plain_steps > 0 and (info["persistent"] or info["n_groups_lds"]):
        sim.close()          # its record of the last frames would crowd the plain run's memory
        psim = Simulator(sc, dtype=dtype, device=dev, launch_mode=1, use_groups=False)
        step(psim)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(psim)
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        psim.close()
        plain = {"value": proj_step * args.plain_steps / (p1 - p0),
                 "ms_per_step": (p1 - p0) / args.plain_steps * 1e3, "steps": args.plain_steps,
                 "launch": "one kernel launch per independent set"}
        log(f"plain launch: {plain['ms_per_step']:.1f} ms/step")
    elif not (info["persistent"] or info["n_groups_lds"]):
        plain = {"value": value, "ms_per_step": elapsed / args.steps * 1e3, "steps": args.steps,
                 "launch": "the timed path itself: one kernel launch per independent set"}

    roof = None
    kernels = {}
    tsz = 8 if dtype == torch.float64 else 4
    staged = group_vertices(sc) if info["n_groups_lds"] else 0
    # the reverse moves the distance / bending compliance adjoints only when
    # their gradient is asked for (the 25.2M-DoF cloth asks for dL/df_ext)
    want_ab = any(t is not None and t.requires_grad for t in (da, ba))
    def fam_bytes(fam):
        if fam == 8:
            return mix_bytes(sc, False, tsz, recording)
        if fam == 9:
            return mix_bytes(sc, True, tsz, recording)
        if fam in (10, 11):
            return group_bytes(sc, fam == 11, tsz, recording, staged, rk == 1, want_ab)
        return alg_bytes(fam, tsz, recording)

    for fam in range(N_FAM):
        if launches[fam]:
            avg_ms = ms[fam] / launches[fam]
            per_launch_items = items[fam] / launches[fam]
            gbs = fam_bytes(fam) * per_launch_items / (avg_ms * 1e-3) / 1e9
            kernels[FAMILY[fam]] = {"launches_sampled": launches[fam], "avg_us": round(avg_ms * 1e3, 3),
                                    "items_per_launch": round(per_launch_items, 1),
                                    "bytes_per_projection": round(fam_bytes(fam), 1),
                                    "alg_GBps": round(gbs, 1),
                                    "share_of_sampled_ms": None}
    tot = sum(ms)
    for fam in range(N_FAM):
        if launches[fam]:
            kernels[FAMILY[fam]]["share_of_sampled_ms"] = round(ms[fam] / tot, 3)
    pmc = {}
    tf = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if os.path.exists(tf):
        pmc = {key: rec for key, rec in json.load(open(tf)).items() if rec.get("csrc_sha") == csrc_hash()}
    def kernel_roof(fam):
        k = kernels[FAMILY[fam]]
        sb = streamed_bytes(sc, fam, tsz)
        achieved = sb * k["items_per_launch"] / (k["avg_us"] * 1e-6) / 1e9
        r = {"bound": "hbm", "kernel": KERNEL_SYMBOL[fam], "achieved": round(achieved, 1),
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
             "traffic": None,
             "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
             "bytes_per_projection": round(sb, 1),
             "byte_model": "streamed bytes per projection (each projection reads and writes its "
                           "vertices in HBM); LDS group kernels stage a patch's vertices once per launch "
                           "and move fewer bytes, so this model can exceed the HBM peak: 'counter' holds the "
                           "measured HBM traffic",
             "avg_launch_us": k["avg_us"], "projections_per_launch": k["items_per_launch"],
             "staged_model": {"bytes_per_projection": k["bytes_per_projection"], "GBps": k["alg_GBps"]}}
        rec = pmc.get(f"{args.workload}:{KERNEL_SYMBOL[fam]}")
        if rec:
            traffic = rec["bytes_per_dispatch_scaled"] * k["items_per_launch"] / rec["items_per_dispatch"]
            alone_s = rec["avg_ns_under_counters"] * 1e-9 * k["items_per_launch"] / rec["items_per_dispatch"]
            r["traffic"] = round(traffic)
            r["counter"] = {
                "bytes_per_projection": round(traffic / k["items_per_launch"], 1),
                "shared_GBps": round(traffic / (k["avg_us"] * 1e-6) / 1e9, 1),
                "shared_frac": round(traffic / (k["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "alone_GBps": round(traffic / alone_s / 1e9, 1),
                "alone_frac": round(traffic / alone_s / 1e9 / HBM_PEAK_GBS, 4),
                "lds_reuse": round(sb * k["items_per_launch"] / traffic, 2),
                "note": "shared: over the timed run's launch time (the adjoint's second stream runs beside); "
                        "alone: over the launch time under the counters (one dispatch at a time)"}
        return r

    if tot > 0:
        dom = max(range(N_FAM), key=lambda f: ms[f])
        roof = kernel_roof(dom)
        # the forward and reverse group kernels take about equal time on the
        # tiled cloth, so the dominant one can change from run to run: both
        # are reported, each with its share of the sampled kernel time
        if launches[10] and launches[11]:
            roof["by_kernel"] = {}
            for fam in (10, 11):
                r = kernel_roof(fam)
                roof["by_kernel"][KERNEL_SYMBOL[fam]] = {
                    "share_of_sampled_ms": kernels[FAMILY[fam]]["share_of_sampled_ms"],
                    "avg_launch_us": r["avg_launch_us"], "achieved": r["achieved"], "frac": r["frac"],
                    "bytes_per_projection": r["bytes_per_projection"], "counter": r.get("counter")}

        # the whole path per step: algorithmic bytes of every projection run
        # (forward frames, the adjoint's recomputed frames, reversed frames)
        # over the step's wall time.  Per-launch figures above are taken on
        # launches that, in the adjoint, share the GPU with the other stream
        # (recomputation beside the reverse), so they understate a kernel
        # running alone; the path figure does not depend on that.
        covered = set()
        for (a, b, _pm) in sc.groups:
            covered.update(range(a, b))
        all_grouped = (info["n_groups_lds"] == len(sc.groups) > 0 and len(covered) == len(sc.set_type))
        if info["tape_mode"] in (1, 3, 4) and (all_grouped or not sc.groups) and not info["persistent"]:
            half = proj_step / 2
            frames_fwd = F + (F - kept)
            if all_grouped:
                fb = group_bytes(sc, False, tsz, recording, staged, rk == 1, want_ab)
                rb = group_bytes(sc, True, tsz, recording, staged, rk == 1, want_ab)
            else:
                fb = recording * mix_bytes(sc, False, tsz, True) + (1 - recording) * mix_bytes(sc, False, tsz, False)
                rb = mix_bytes(sc, True, tsz, False)
            pb = half * frames_fwd / F * fb + half * rb
            sec = elapsed / args.steps
            roof["path"] = {"bytes_per_step": round(pb), "achieved": round(pb / sec / 1e9, 1),
                            "frac": round(pb / sec / 1e9 / HBM_PEAK_GBS, 4), "frames_run_forward": frames_fwd,
                            "byte_model": "staged (the group kernels' own bytes)"}
            fr, rr = pmc.get(f"{args.workload}:k_group_fwd"), pmc.get(f"{args.workload}:k_group_rev")
            if all_grouped and fr and rr:
                launches_frame = sc.substeps * sc.iterations * len(sc.groups)
                def per_dispatch(recording):     # dispatch-weighted over the template variants
                    # third template argument of k_group_fwd: the record kind (0 none)
                    vs = [v for n_, v in fr["variants"].items()
                          if (n_.split(",")[2].strip() not in ("0", "false")) == recording]
                    return (sum(v["dispatches"] * (v["fetch_bytes"] + v["write_bytes"]) for v in vs)
                            / max(sum(v["dispatches"] for v in vs), 1))
                cb = launches_frame * (F * per_dispatch(True) + (frames_fwd - F) * per_dispatch(False)
                                       + F * rr["bytes_per_dispatch_scaled"])
                roof["path"]["counter_bytes_per_step"] = round(float(cb))
                roof["path"]["counter_GBps"] = round(float(cb) / sec / 1e9, 1)
                roof["path"]["counter_frac"] = round(float(cb) / sec / 1e9 / HBM_PEAK_GBS, 4)
        roof["adjoint_streams"] = info["adjoint_streams"]
        if info["adjoint_streams"] == 2:
            roof["note"] = ("the adjoint recomputes earlier frames on a second stream beside the reverse, so those "
                            "launches share the GPU and the per-launch figures above are shared rates; 'path' is "
                            "every projection's algorithmic bytes over the step time")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, sc)
        # one core, on a sample small enough for it: the 2048-column cloth
        # cut to 256 rows (the same tiles, sets and launch structure), the
        # smaller workloads as they are
        one_sc = scenes_small_for_one_core(args.workload, sc)
        one = cpu_baseline(args.workload, one_sc, max_projections=4_000_000, threads=1)
        cpu["one_core"] = {k: one[k] for k in ("value", "forward_projections_per_s", "adjoint_projections_per_s",
                                              "sample")}
        if one_sc is not sc:
            cpu["one_core"]["sample"] = (f"{one_sc.n_verts}-vertex cut of the workload ({one_sc.name}): "
                                         + one["sample"])

    serving = None
    if args.workload == "c4" and args.serve_requests > 0:
        sim.close()
        for t in leaves:
            t.grad = None
        torch.cuda.empty_cache()
        serving = serving_leg(args.serve_requests, args.pack_slots, log)

    out = {
        "metric": "constraint projections/s fwd+adjoint vs plain launch; p50/p99 request latency",
        "value": value, "unit": "projections/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if dtype == torch.float64 else "f32",
        "data": "synthetic (seeded grid cloth / tet box, parameters and targets generated)",
        "config": workload_config(args.workload, sc, F),
        "projections_per_step": proj_step, "loss": float(loss.detach().cpu()), "grads_finite": grads_finite,
        "roofline": roof, "kernels": kernels, "phases": phases, "cpu_baseline": cpu, "plain_launch": plain,
        "launch": ("persistent frame kernel" if info["persistent"] else
                   f"LDS group launches ({info['n_groups_lds']} groups), one launch per other set"
                   if info["n_groups_lds"] else "one kernel launch per set"),
        "persistent_blocks": info["persistent_blocks"], "tape_mode": info["tape_mode"], "record_kind": rk,
        "record_bytes_per_iteration": info["tape_bytes_per_iteration"],
        "forward_record_frames": info["forward_record_frames"],
        "profile_stride": args.profile_stride, "csrc_sha": csrc_hash(),
        "accuracy": ACCURACY.get((args.workload, "f64" if dtype == torch.float64 else "f32")),
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    if not grads_finite:
        # a step whose gradient is not finite measured nothing worth a number
        log("error: the step's gradients are not finite")
        sys.exit(3)


if __name__ == "__main__":
    main()

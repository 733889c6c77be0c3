"""Continuous-batching request loop for rollout and gradient requests.

Requests (a mesh with its parameters, a frame count and optionally a goal
whose gradient is wanted) arrive at any time.  The server admits a request
when a slot is free and its device-memory estimate fits the HBM budget next
to the requests already resident; admitted requests run concurrently, each
on its own HIP stream, so their kernels overlap on the device.  A request
that arrives while others run is admitted as soon as a slot and memory free
up.  Every request's state stays on the device until its result is copied
out.  Latency is measured from arrival to result.

All simulation work runs in the library's kernels; this module only
schedules calls.  Each request gets its own context, so its result does not
depend on what else is running (bitwise).  Two executors: ``Server`` runs
each admitted request on its own stream (kernels of different requests
overlap on the device), ``PackedServer`` runs every admitted request in one
pack, so each launch serves the same step of all of them.
"""
from __future__ import annotations

import heapq
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Dict, List, Optional

import numpy as np
import torch

from .lib import Simulator


@dataclass
class Request:
    rid: int
    scene: Any                      # scenes.Scene
    n_frames: int
    adjoint: bool = False
    targets: Optional[np.ndarray] = None   # (F, V, 3) goal targets; goal on the last frame
    arrival: float = 0.0            # seconds after the start of the run
    # filled by the server
    admitted: float = -1.0
    done: float = -1.0
    slot: int = -1
    result: Dict[str, np.ndarray] = field(default_factory=dict)
    projections: int = 0
    device_bytes: int = 0
    cancelled: bool = False         # set by Server.cancel


def estimate_parts(sc, n_frames: int, adjoint: bool, dtype_bytes: int = 4):
    """Upper estimates of a request's device memory: (bytes the library
    allocates: constraint records, state, checkpoints, the adjoint's working
    set and one frame of its record of projection inputs; bytes the caller's
    tensors take: frames, final state, targets, goal gradient and gradient
    outputs).  The library part is handed to the request's context as its
    budget, so the library never sizes beyond what was admitted (a record of
    more frames is kept only if it fits)."""
    V, nd, nb, nt = sc.n_verts, sc.n_dist, sc.n_bend, sc.n_tet
    t = dtype_bytes
    rec = nd * (8 + 6 * t) + nb * (16 + 6 * t) + nt * (16 + 17 * t) + V * (8 + 5 * t)
    state = V * 16 * t
    ck = 2 * n_frames * V * 4 * t
    adj = 0
    if adjoint:
        adj = V * 8 * t + (nd + nb + nt) * (2 * t + 8)
        adj += sc.substeps * sc.iterations * (nd * 4 * t + nb * 10 * t + nt * 12 * t + V * 4 * t)
    lib = int(1.15 * (rec + state + ck + adj)) + (8 << 20)
    caller = (n_frames + 2) * V * 3 * t
    if adjoint:
        caller += 2 * n_frames * V * 3 * t + 2 * V * 3 * t + (nd + nb + nt) * 8
        if getattr(sc, "f_ext", None) is not None:
            caller += n_frames * V * 3 * t
    return lib, int(1.15 * caller) + (1 << 20)


def estimate_bytes(sc, n_frames: int, adjoint: bool, dtype_bytes: int = 4) -> int:
    """Upper estimate of a request's device memory: both parts of
    estimate_parts."""
    return sum(estimate_parts(sc, n_frames, adjoint, dtype_bytes))


class Server:
    """Runs requests with ``slots`` concurrent streams within ``hbm_budget``."""

    def __init__(self, slots: int = 4, hbm_budget: int = 64 << 30, device="cuda:0",
                 dtype: torch.dtype = torch.float32, record_whole_rollout: bool = True):
        self.slots = slots
        self.budget = hbm_budget
        self.device = torch.device(device)
        self.dtype = dtype
        self.record = record_whole_rollout
        self._lock = threading.Condition()
        self._pending: List = []          # heap of (arrival, rid, request)
        self._in_use = 0
        self._free_slots = list(range(slots))
        self._finished: List[Request] = []
        self._cancelled: List[Request] = []
        self._running: Dict[int, Request] = {}
        self._closed = False
        self._t0 = 0.0
        self._queue_depth: List[int] = []
        self._errors: List[str] = []

    # ---------------------------------------------------------------- execution
    def _run_one(self, req: Request, stream: torch.cuda.Stream):
        sc = req.scene
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            # every step of a request on its slot's stream: the server
            # overlaps requests, and one request at a time stays the plain
            # one-stream baseline
            sim = Simulator(sc, **self._sim_kwargs(req))
            try:
                xf, xe, ve = sim.forward(req.n_frames, for_adjoint=req.adjoint)
                res = {}
                if req.cancelled:                 # stop at the call boundary, no result
                    stream.synchronize()
                    return
                if req.adjoint:
                    mask = np.zeros(req.n_frames, np.uint8)
                    mask[-1] = 1
                    tg = sim.tensor(req.targets)
                    loss, dL = sim.goal_l2(xf, tg, mask)
                    g = sim.adjoint(dL, mask)
                    res["loss"] = loss
                    res.update({k: v for k, v in g.items()})
                res["x_final"] = xe
                stream.synchronize()
                if req.cancelled:
                    return
                req.result = {k: (v.detach().cpu().numpy() if isinstance(v, torch.Tensor) else v)
                              for k, v in res.items()}
                req.projections = sc.projections_per_rollout(req.n_frames) * (2 if req.adjoint else 1)
            finally:
                sim.close()

    def _sim_kwargs(self, req: Request) -> Dict[str, Any]:
        """Context options of a request: its share of the admitted memory is
        the library's budget."""
        lib_bytes, _ = estimate_parts(req.scene, req.n_frames, req.adjoint, 8 if self.dtype == torch.float64 else 4)
        return {"dtype": self.dtype, "device": self.device, "tape_mode": 0 if self.record else 1,
                "serial_adjoint": True, "hbm_budget_bytes": lib_bytes}

    def _make_stream(self):
        return torch.cuda.Stream(device=self.device)      # default priority

    def cancel(self, rid: int) -> bool:
        """Cancel request ``rid``: a pending one is dropped before it is
        admitted; a running one stops at its next call boundary (after its
        forward, before its adjoint) and returns no result.  Other requests
        are unaffected (each has its own context and stream).  Returns
        whether the request was found unfinished."""
        with self._lock:
            for k, (_, r_id, req) in enumerate(self._pending):
                if r_id == rid:
                    self._pending.pop(k)
                    heapq.heapify(self._pending)
                    req.cancelled = True
                    self._cancelled.append(req)
                    self._lock.notify_all()
                    return True
            req = self._running.get(rid)
            if req is not None:
                req.cancelled = True
                return True
        return False

    def _worker(self, slot: int):
        stream = self._make_stream()
        while True:
            with self._lock:
                while True:
                    if self._closed and not self._pending:
                        return
                    now = time.perf_counter() - self._t0
                    admissible = None
                    if self._pending and self._pending[0][0] <= now:
                        arr, rid, req = self._pending[0]
                        if self._in_use + req.device_bytes <= self.budget or self._in_use == 0:
                            admissible = heapq.heappop(self._pending)[2]
                    if admissible is not None:
                        req = admissible
                        self._running[req.rid] = req
                        self._in_use += req.device_bytes
                        self._queue_depth.append(sum(1 for a, _, _ in self._pending if a <= now))
                        break
                    timeout = None
                    if self._pending and self._pending[0][0] > now:
                        timeout = self._pending[0][0] - now
                    self._lock.wait(timeout if timeout is not None else 0.05)
            req.admitted = time.perf_counter() - self._t0
            req.slot = slot
            try:
                self._run_one(req, stream)
            except Exception as e:        # report, keep serving the others
                self._errors.append(f"request {req.rid}: {e}")
            req.done = time.perf_counter() - self._t0
            with self._lock:
                self._in_use -= req.device_bytes
                self._running.pop(req.rid, None)
                (self._cancelled if req.cancelled else self._finished).append(req)
                self._lock.notify_all()

    def run(self, requests: List[Request]) -> Dict[str, Any]:
        """Serve ``requests`` (arrival times relative to now); returns a report."""
        for r in requests:
            r.device_bytes = estimate_bytes(r.scene, r.n_frames, r.adjoint,
                                            8 if self.dtype == torch.float64 else 4)
        self._pending = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(self._pending)
        self._finished = []
        self._cancelled = []
        self._running = {}
        self._closed = True
        self._queue_depth = []
        if torch.cuda.is_available():
            torch.cuda.synchronize(self.device)
        self._t0 = time.perf_counter()
        threads = [threading.Thread(target=self._worker, args=(s,), daemon=True) for s in range(self.slots)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        wall = time.perf_counter() - self._t0
        if self._errors:
            raise RuntimeError("; ".join(self._errors))
        rep = report(self._finished, wall, self._queue_depth)
        rep["cancelled"] = len(self._cancelled)
        return rep


class PackedServer:
    """Continuous batching through packs: a scheduler thread admits arrived
    requests by HBM budget and slot count into one of ``n_packs`` packs (cloth
    and tet requests in separate packs, so a pack's launches are not
    lengthened by the other kind's longer schedule), where they join the next
    round and share every launch with the requests already in that pack.
    Each pack runs on its own stream, so the packs' launches overlap on the
    device; the scheduler keeps at most ``ahead`` rounds of each pack queued.
    Finished requests leave at once and their results are copied out on the
    pack's stream while later rounds run.  ``graphs`` replays a round from a
    captured HIP graph while a pack's membership stays the same."""

    def __init__(self, slots: int = 32, hbm_budget: int = 64 << 30, device="cuda:0",
                 dtype: torch.dtype = torch.float32, graphs: Optional[bool] = None, n_packs: int = 1,
                 ahead: int = 2, block_size: Optional[int] = None):
        """graphs / block_size: the packs' launch shape; None takes the
        autotuner's entry for this dtype (``tune.tune_pack``), else graphs
        on and 256-thread workgroups."""
        self.slots = slots
        self.budget = hbm_budget
        self.device = torch.device(device)
        self.dtype = dtype
        tuned = {}
        if graphs is None or block_size is None:
            from .tune import lookup_pack
            tuned = lookup_pack(dtype) or {}
        self.graphs = bool(tuned.get("graphs", 1)) if graphs is None else graphs
        self.block_size = int(tuned.get("block_size", 0)) if block_size is None else block_size
        self.n_packs = max(1, n_packs)
        self.ahead = max(1, ahead)
        self.pack_stats: List[Dict[str, int]] = []
        self.finished: List[Request] = []

    def _admit(self, pack, req: Request):
        sc = req.scene
        lib_bytes, _ = estimate_parts(sc, req.n_frames, req.adjoint, 8 if self.dtype == torch.float64 else 4)
        sim = Simulator(sc, dtype=self.dtype, device=self.device, tape_mode=1, hbm_budget_bytes=lib_bytes)
        mask = None
        if req.adjoint:
            mask = np.zeros(req.n_frames, np.uint8)
            mask[-1] = 1
        job = pack.add(sim, req.n_frames, targets=req.targets if req.adjoint else None, frame_mask=mask,
                       want=("x0", "v0", "dist_alpha", "bend_alpha", "tet_E"), frames=False, tag=req)
        req.projections = sc.projections_per_rollout(req.n_frames) * (2 if req.adjoint else 1)
        return job

    @staticmethod
    def _collect(job, stream):
        """Start the device-to-host copies of a finished job's results."""
        res = {"x_final": job.x_final}
        if job.loss is not None:
            res["loss"] = job.loss
            res.update(job.grads)
        host = {}
        for k, v in res.items():
            h = torch.empty(v.shape, dtype=v.dtype, pin_memory=True)
            h.copy_(v, non_blocking=True)
            host[k] = h
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev, host

    def _pick(self, packs, req):
        kind = 1 if req.scene.n_tet else 0
        mine = [i for i in range(len(packs)) if i % 2 == kind % 2] if len(packs) > 1 else [0]
        return min(mine, key=lambda i: len(packs[i][0].jobs))

    def run(self, requests: List[Request]) -> Dict[str, Any]:
        from .lib import Pack
        for r in requests:
            r.device_bytes = estimate_bytes(r.scene, r.n_frames, r.adjoint, 8 if self.dtype == torch.float64 else 4)
        pending = [(r.arrival, r.rid, r) for r in requests]
        heapq.heapify(pending)
        finished: List[Request] = []
        depth: List[int] = []
        in_use = 0
        running = 0
        copying = []
        closing = []
        # (pack, stream, queued round events)
        packs = []
        for _ in range(self.n_packs):
            st = torch.cuda.Stream(device=self.device)     # default priority
            packs.append((Pack(dtype=self.dtype, device=self.device, graphs=self.graphs, block_size=self.block_size),
                          st, []))
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        with torch.cuda.device(self.device):
            while pending or running or copying:
                now = time.perf_counter() - t0
                while pending and pending[0][0] <= now and running < self.slots:
                    req = pending[0][2]
                    if running and in_use + req.device_bytes > self.budget:
                        break
                    heapq.heappop(pending)
                    depth.append(sum(1 for a, _, _ in pending if a <= now))
                    req.admitted = time.perf_counter() - t0
                    i = self._pick(packs, req)
                    req.slot = i
                    self._admit(packs[i][0], req)
                    running += 1
                    in_use += req.device_bytes
                progressed = False
                for pack, st, queued in packs:
                    while queued and queued[0].query():
                        queued.pop(0)
                    if not pack.jobs or len(queued) >= self.ahead:
                        continue
                    with torch.cuda.stream(st):
                        for job in pack.run(1):
                            running -= 1
                            copying.append((job,) + self._collect(job, st))
                        ev = torch.cuda.Event()
                        ev.record(st)
                    queued.append(ev)
                    progressed = True
                still = []
                for job, ev, host in copying:
                    if ev.query():
                        req = job.tag
                        req.done = time.perf_counter() - t0
                        req.result = {k: v.numpy() for k, v in host.items()}
                        closing.append(job.sim)      # freed after the run: a free waits for the device
                        in_use -= req.device_bytes
                        finished.append(req)
                    else:
                        still.append((job, ev, host))
                copying = still
                if not progressed:
                    waits = [q[0] for _, _, q in packs if q]
                    if waits:
                        waits[0].synchronize()
                    elif copying:
                        copying[0][1].synchronize()
                    elif pending:
                        time.sleep(max(0.0, min(0.005, pending[0][0] - (time.perf_counter() - t0))))
        wall = time.perf_counter() - t0
        for sim in closing:
            sim.close()
        self.finished = finished
        self.pack_stats = [p.stats() for p, _, _ in packs]
        for p, _, _ in packs:
            p.close()
        rep = report(finished, wall, depth)
        tot = {}
        for st_ in self.pack_stats:
            for k, v in st_.items():
                tot[k] = tot.get(k, 0) + v
        rep["pack"] = tot
        rep["n_packs"] = self.n_packs
        return rep


def report(done: List[Request], wall: float, depth: List[int]) -> Dict[str, Any]:
    lat = np.array([r.done - r.arrival for r in done])
    proj = sum(r.projections for r in done)
    return {"requests": len(done), "wall_s": wall,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_latency_s": float(lat.mean()) if len(lat) else None,
            "throughput_rps": len(done) / wall if wall > 0 else None,
            "projections_per_s": proj / wall if wall > 0 else None,
            "max_queue_depth": int(max(depth)) if depth else 0,
            "max_concurrent": max_concurrency(done)}


def max_concurrency(done: List[Request]) -> int:
    ev = []
    for r in done:
        ev.append((r.admitted, 1))
        ev.append((r.done, -1))
    ev.sort()
    cur = best = 0
    for _, d in ev:
        cur += d
        best = max(best, cur)
    return best


def make_mix(n: int, qps: float, seed: int = 6, frames=(30, 120), size_mu=np.log(16000), size_sigma=1.0,
             vmin=1000, vmax=250_000, substeps: int = 2, iterations: int = 20, frames_scale: float = 1.0):
    """Serving mix: Poisson arrivals at ``qps``; half grid cloths, half tet
    boxes; ln V ~ N(size_mu, size_sigma) clipped to [vmin, vmax]; frames
    ~ U{frames}; half the requests want the gradient.  Draw order: arrival
    gaps, kind, size, frames, adjoint flag, then per-request parameter
    seeds."""
    from . import scenes
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, n)
    kind = rng.integers(0, 2, n)
    sizes = np.clip(np.exp(rng.normal(size_mu, size_sigma, n)), vmin, vmax)
    fr = rng.integers(frames[0], frames[1] + 1, n)
    adj = rng.integers(0, 2, n)
    pseed = rng.integers(0, 2 ** 31, n)
    reqs = []
    t = 0.0
    for i in range(n):
        t += gaps[i]
        if kind[i] == 0:
            m = max(4, int(round(np.sqrt(sizes[i]))))
            sc = scenes.cloth_grid(m, m, 1.0 / (m - 1), origin=(-0.5, 0.0, -0.5), pinned=(0, m - 1))
            sc.dist_alpha, sc.bend_alpha = scenes.cloth_alpha(int(pseed[i]), sc.n_dist, sc.n_bend)
            sc.tet_E = np.zeros(0)
        else:
            m = max(1, int(round(sizes[i] ** (1.0 / 3.0))) - 1)
            sc = scenes.tet_box(m, size=m * scenes.TET_SPACING)
            sc.tet_E, sc.tet_nu = scenes.tet_material(int(pseed[i]), sc.n_tet)
            sc.dist_alpha, sc.bend_alpha = np.zeros(0), np.zeros(0)
        sc.dt, sc.substeps, sc.iterations = 1.0 / 60.0, substeps, iterations
        F = max(1, int(fr[i] * frames_scale))
        sc.n_frames = F
        tg = None
        if adj[i]:
            tg = np.repeat((sc.rest + np.array([0.0, -0.05, 0.0]))[None], F, axis=0)
        reqs.append(Request(rid=i, scene=sc, n_frames=F, adjoint=bool(adj[i]), targets=tg, arrival=t))
    return reqs

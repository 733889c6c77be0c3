"""Packs: many meshes advanced together, one launch per step for all of them.

Each job's outputs must be bitwise those of its context run alone (forward,
goal, adjoint), whatever else is in the pack, whether rounds are replayed
from a captured HIP graph, and whether the job joined a pack that was
already running.  CPU tests cover the entry points that need no device."""
import ctypes as C

import numpy as np
import pytest

from paper_2301_01396_amd import lib as L
from paper_2301_01396_amd import scenes


def test_pack_create_rejects_bad_arguments():
    lib = L.load()
    pk = C.c_void_p()
    assert lib.xpbd_pack_create(7, 0, 0, C.byref(pk)) == L.XPBD_ERR_INVALID
    assert lib.xpbd_pack_create(L.F32, 4, 0, C.byref(pk)) == L.XPBD_ERR_INVALID
    for bad in (32, 96, 512, -1):
        assert lib.xpbd_pack_create(L.F32, 0, bad, C.byref(pk)) == L.XPBD_ERR_INVALID
    assert lib.xpbd_pack_create(L.F32, L.PACK_GRAPHS, 0, C.byref(pk)) == L.XPBD_OK
    st = L.PackStats()
    assert lib.xpbd_pack_get_stats(pk, C.byref(st)) == L.XPBD_OK
    assert st.active_jobs == 0 and st.rounds == 0
    n = C.c_int32(-1)
    ids = (C.c_int64 * 1)()
    # nothing queued: returns at once without touching a device
    assert lib.xpbd_pack_run(pk, 5, None, ids, 1, C.byref(n)) == L.XPBD_OK
    assert n.value == 0
    assert lib.xpbd_pack_run(pk, -1, None, ids, 1, C.byref(n)) == L.XPBD_ERR_INVALID
    assert lib.xpbd_pack_add(pk, None, None, None, None) == L.XPBD_ERR_INVALID
    assert lib.xpbd_pack_destroy(pk) == L.XPBD_OK
    assert lib.xpbd_pack_destroy(None) == L.XPBD_ERR_INVALID


# ---------------------------------------------------------------- GPU

def _scenes(S=2, K=5):
    a = scenes.small_cloth(n=6, frames=3, substeps=S, iterations=K)
    b = scenes.small_tets(n=2, frames=4, substeps=S, iterations=K)
    c = scenes.small_cloth(n=9, frames=2, substeps=S, iterations=K, sphere=False, seed=3)
    d = scenes.small_cloth(n=5, frames=5, substeps=S, iterations=K, seed=4)
    e = scenes.membrane_cloth(n=6, frames=3, substeps=S, iterations=K)
    return [a, b, c, d, e]


def _targets(sc, F, seed):
    rng = np.random.default_rng(seed)
    return np.repeat(sc.rest[None], F, axis=0) + 0.05 * rng.standard_normal((F, sc.n_verts, 3))


def _alone(sim, F, tg, mask, adj):
    import torch
    xf, xe, ve = sim.forward(F, for_adjoint=adj)
    out = {"x_frames": xf, "x_final": xe, "v_final": ve}
    if adj:
        loss, dL = sim.goal_l2(xf, sim.tensor(tg), mask)
        out["loss"] = loss
        out.update({"g_" + k: v for k, v in sim.adjoint(dL, mask).items()})
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def _packed(job):
    out = {"x_frames": job.x_frames, "x_final": job.x_final, "v_final": job.v_final}
    if job.loss is not None:
        out["loss"] = job.loss
        out.update({"g_" + k: v for k, v in job.grads.items()})
    return {k: v.cpu().numpy() for k, v in out.items()}


def _same(a, b, label):
    assert a.keys() == b.keys(), label
    for k in a:
        assert a[k].shape == b[k].shape, (label, k)
        assert np.array_equal(a[k], b[k]), (label, k, float(np.abs(a[k] - b[k]).max()))


def _case(dtype, graphs, tape_mode=0, late=False, block=0):
    import torch
    from tests._cases import needs_gpu
    needs_gpu()
    scs = _scenes()
    adj = [True, True, False, True, True]
    masks = [None, np.array([0, 1, 0, 1], np.uint8), None, np.array([1, 0, 0, 0, 1], np.uint8), None]
    ref = []
    for i, sc in enumerate(scs):
        sim = L.Simulator(sc, dtype=dtype, tape_mode=tape_mode)
        F = sc.n_frames
        m = masks[i] if masks[i] is not None else np.ones(F, np.uint8)
        ref.append(_alone(sim, F, _targets(sc, F, i), m, adj[i]))
        sim.close()
    pk = L.Pack(dtype=dtype, graphs=graphs, block_size=block)
    sims = [L.Simulator(sc, dtype=dtype, tape_mode=tape_mode) for sc in scs]
    jobs = {}
    first = scs[:2] if late else scs
    for i, sc in enumerate(first):
        F = sc.n_frames
        jobs[i] = pk.add(sims[i], F, targets=_targets(sc, F, i) if adj[i] else None, frame_mask=masks[i])
    done = []
    if late:
        done += pk.run(max_rounds=2)
        for i in range(2, len(scs)):
            F = scs[i].n_frames
            jobs[i] = pk.add(sims[i], F, targets=_targets(scs[i], F, i) if adj[i] else None,
                             frame_mask=masks[i])
    done += pk.run_all()
    torch.cuda.synchronize()
    assert sorted(j.id for j in done) == sorted(j.id for j in jobs.values())
    for i, j in jobs.items():
        _same(ref[i], _packed(j), (i, scs[i].name))
    st = pk.stats()
    pk.close()
    for s in sims:
        s.close()
    return st


@pytest.mark.gpu
@pytest.mark.parametrize("graphs", [False, True])
def test_pack_matches_alone_fp64(graphs):
    import torch
    st = _case(torch.float64, graphs)
    assert st["active_jobs"] == 0
    if graphs:
        assert st["graph_captures"] >= 1 and st["graph_launches"] == st["rounds"]
    else:
        assert st["launches"] > 0 and st["graph_launches"] == 0


@pytest.mark.gpu
def test_pack_matches_alone_fp32_graphs():
    import torch
    _case(torch.float32, True)


@pytest.mark.gpu
@pytest.mark.parametrize("block", [64, 128])
def test_pack_workgroup_size_does_not_change_results(block):
    import torch
    _case(torch.float32, True, block=block)


@pytest.mark.gpu
def test_pack_jobs_join_a_running_pack():
    import torch
    _case(torch.float32, True, late=True)


@pytest.mark.gpu
def test_pack_per_frame_recompute_matches_alone():
    import torch
    _case(torch.float32, False, tape_mode=1)


@pytest.mark.gpu
def test_pack_rejects_mismatched_jobs():
    import torch
    from tests._cases import needs_gpu
    needs_gpu()
    a = scenes.small_cloth(n=6, substeps=2, iterations=5)
    b = scenes.small_cloth(n=6, substeps=2, iterations=6)
    sa, sb = L.Simulator(a), L.Simulator(b)
    s64 = L.Simulator(a, dtype=torch.float64)
    pk = L.Pack()
    pk.add(sa, 2)
    with pytest.raises(L.XPBDError) as e:
        pk.add(sa, 2)                       # context already serving a job
    assert e.value.status == L.XPBD_ERR_INVALID
    with pytest.raises(L.XPBDError):
        pk.add(sb, 2)                       # different iteration count
    with pytest.raises(ValueError):
        pk.add(s64, 2)                      # different dtype
    assert sa.lib.xpbd_destroy(sa._ctx) == L.XPBD_ERR_STATE   # in a job
    with pytest.raises(L.XPBDError) as e:
        sa.forward(2)
    assert e.value.status == L.XPBD_ERR_STATE
    pk.run_all()
    torch.cuda.synchronize()
    sa.forward(2)                           # free again
    pk.close()
    for s in (sa, sb, s64):
        s.close()

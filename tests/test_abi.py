"""The C ABI library loads, exports every declared entry point, and rejects
invalid problems before touching the device (runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2301_01396_amd import lib as L
from paper_2301_01396_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "xpbd.h")).read()
    return sorted(set(re.findall(r"\b(xpbd_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared()
    assert "xpbd_create" in names and "xpbd_adjoint" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_status_strings():
    lib = L.load()
    assert lib.xpbd_status_string(0) == b"ok"
    assert lib.xpbd_status_string(4) == b"invalid state"


def _create(sc, **opt):
    lib = L.load()
    rest = np.ascontiguousarray(sc.rest, np.float64)
    im = np.ascontiguousarray(sc.inv_mass, np.float64)
    dv = np.ascontiguousarray(sc.dist_v, np.int32)
    bv = np.ascontiguousarray(sc.bend_v, np.int32)
    tv = np.ascontiguousarray(sc.tet_v, np.int32)
    nu = np.ascontiguousarray(sc.tet_nu, np.float64)
    st, off, items = sc.schedule_arrays()
    m = L.MeshDesc(sc.n_verts, rest.ctypes.data_as(L._dp), im.ctypes.data_as(L._dp))
    cd = L.ConstraintDesc(sc.n_dist, dv.ctypes.data_as(L._ip), sc.n_bend, bv.ctypes.data_as(L._ip), sc.n_tet,
                          tv.ctypes.data_as(L._ip), nu.ctypes.data_as(L._dp), 1 if sc.contact else 0,
                          sc.contact_thickness, sc.contact_compliance)
    gs, gp = L.schedule_groups(sc)
    sd = L.ScheduleDesc(len(st), st.ctypes.data_as(L._ip), off.ctypes.data_as(L._lp), items.ctypes.data_as(L._ip),
                        len(gs) // 2, gs.ctypes.data_as(L._ip), gp.ctypes.data_as(L._ip))
    o = L.Options()
    o.dt = opt.get("dt", sc.dt)
    o.substeps = opt.get("substeps", sc.substeps)
    o.iterations = opt.get("iterations", sc.iterations)
    o.dtype = opt.get("dtype", 0)
    o.tape_mode = opt.get("tape_mode", 0)
    o.block_size = opt.get("block_size", 0)
    o.record_frames = opt.get("record_frames", 0)
    o.serial_adjoint = opt.get("serial_adjoint", 0)
    ctx = C.c_void_p()
    rc = lib.xpbd_create(C.byref(m), C.byref(cd), C.byref(sd), C.byref(o), C.byref(ctx))
    msg = lib.xpbd_last_error(None).decode()
    return rc, ctx, msg


def test_rejects_non_independent_set():
    sc = scenes.small_cloth(n=4)
    # put two edges sharing a vertex into one set
    sc.set_items[0] = np.concatenate([sc.set_items[0], sc.set_items[1][:1]])
    sc.set_items[1] = sc.set_items[1][1:]
    rc, ctx, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "not independent" in msg


def test_rejects_missing_and_repeated_constraints():
    sc = scenes.small_cloth(n=4)
    sc.set_items[0] = sc.set_items[0][1:]
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "not scheduled" in msg
    sc = scenes.small_cloth(n=4)
    sc.set_type.append(scenes.DIST)
    sc.set_items.append(sc.set_items[0][:1].copy())
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "twice" in msg


def test_rejects_bad_indices_and_geometry():
    sc = scenes.small_cloth(n=4)
    sc.dist_v = sc.dist_v.copy()
    sc.dist_v[2, 1] = 99
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "out of range" in msg
    sc = scenes.small_tets(n=1)
    sc.tet_v = sc.tet_v.copy()
    sc.tet_v[0, [2, 3]] = sc.tet_v[0, [3, 2]]      # inverted rest tet
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "rest volume" in msg
    lib = L.load()                                  # a mesh without vertices
    o = L.Options()
    o.dt, o.substeps, o.iterations = 1.0 / 60.0, 1, 1
    rc = lib.xpbd_create(C.byref(L.MeshDesc(0, None, None)), C.byref(L.ConstraintDesc()), C.byref(L.ScheduleDesc()),
                         C.byref(o), C.byref(C.c_void_p()))
    assert rc == L.XPBD_ERR_INVALID and "empty mesh" in lib.xpbd_last_error(None).decode()


def test_rejects_contact_on_pinned_vertex_and_bad_options():
    sc = scenes.small_cloth(n=4)
    sc.set_items[-1] = np.concatenate([sc.set_items[-1], [0]]).astype(np.int32)   # vertex 0 is pinned
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "pinned" in msg
    sc = scenes.small_cloth(n=4)
    assert _create(sc, substeps=0)[0] == L.XPBD_ERR_INVALID
    assert _create(sc, dt=-1.0)[0] == L.XPBD_ERR_INVALID
    assert _create(sc, dtype=7)[0] == L.XPBD_ERR_INVALID
    assert _create(sc, tape_mode=5)[0] == L.XPBD_ERR_INVALID
    assert _create(sc, record_frames=-1)[0] == L.XPBD_ERR_INVALID


def test_null_context_calls_fail_cleanly():
    lib = L.load()
    assert lib.xpbd_destroy(None) == L.XPBD_ERR_INVALID
    p = L.Params()
    assert lib.xpbd_forward(None, None, None, C.byref(p), 1, None, None, None, 0, None) == L.XPBD_ERR_INVALID


@pytest.mark.parametrize("maker", [lambda: scenes.small_cloth(n=6), lambda: scenes.small_tets(n=2),
                                   lambda: scenes.config_c1(1)])
def test_generated_schedules_are_valid_colorings(maker):
    sc = maker()
    st, off, items = sc.schedule_arrays()
    cv = {scenes.DIST: sc.dist_v, scenes.BEND: sc.bend_v, scenes.TET: sc.tet_v, scenes.TRI: sc.tri_v}
    seen = {k: np.zeros(len(v), int) for k, v in cv.items()}
    for s in range(len(st)):
        it = items[off[s]:off[s + 1]]
        if st[s] == scenes.CONTACT:
            verts = it
        else:
            verts = cv[st[s]][it].ravel()
            seen[st[s]][it] += 1
        assert len(np.unique(verts)) == len(verts)
    for k, v in seen.items():
        assert np.all(v == 1)


def test_rejects_groups_whose_constraints_span_patches():
    sc = scenes.small_cloth(n=20)
    scenes.tile_cloth(sc, 20, 20, tile=8)
    a, b, pm = sc.groups[0]
    bad = pm.copy()
    bad[sc.dist_v[sc.set_items[a][0], 0]] += 1       # split the first constraint's vertices
    sc.groups[0] = (a, b, bad)
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "spans two patches" in msg
    sc = scenes.small_cloth(n=20)
    scenes.tile_cloth(sc, 20, 20, tile=8)
    sc.groups.append((0, 2, sc.groups[0][2]))          # overlaps group 0
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "overlap" in msg


def test_rejects_groups_of_more_than_64_sets():
    """A group holds at most 64 consecutive sets (each group launch stages its
    sets' item counts and types in fixed LDS arrays of that size)."""
    from tests._cases import split_sets
    sc = split_sets(scenes.small_cloth(n=12), 65)
    sc.groups = [(0, 65, np.zeros(sc.n_verts, np.int32))]
    rc, _, msg = _create(sc)
    assert rc == L.XPBD_ERR_INVALID and "bad set range [0, 65)" in msg


@pytest.mark.parametrize("maker", [lambda: scenes.tile_cloth(scenes.small_cloth(n=40), 40, 40, 16),
                                   lambda: scenes.tile_cloth_lines(scenes.small_cloth(n=40), 40, 40, 16),
                                   lambda: scenes.tile_cloth_lines(scenes.small_cloth(n=37), 37, 37, 8),
                                   lambda: scenes.tile_cloth_quads(scenes.small_cloth(n=45), 45, 45, 8),
                                   lambda: scenes.tile_cloth_quads(scenes.small_cloth(n=40), 40, 40, 16),
                                   lambda: scenes.tile_cloth_quads(scenes.membrane_cloth(n=41), 41, 41, 8),
                                   lambda: scenes.tile_cloth_lines(scenes.membrane_cloth(n=37), 37, 37, 8),
                                   lambda: scenes.config_c2_body(n_frames=1, n=48, body_res=(8, 16), tile=16),
                                   lambda: scenes.tile_box(scenes.small_tets(n=8), 8, 4)])
def test_tiled_schedules_are_valid_and_grouped(maker):
    sc = maker()
    st, off, items = sc.schedule_arrays()
    cv = {scenes.DIST: sc.dist_v, scenes.BEND: sc.bend_v, scenes.TET: sc.tet_v, scenes.TRI: sc.tri_v}
    seen = {k: np.zeros(len(v), int) for k, v in cv.items()}
    for s in range(len(st)):
        it = items[off[s]:off[s + 1]]
        point = st[s] in (scenes.CONTACT, scenes.BODY)
        verts = it[:, None] if point else cv[st[s]][it]
        if not point:
            seen[st[s]][it] += 1
        assert len(np.unique(verts)) == verts.size
    for v in seen.values():
        assert np.all(v == 1)
    covered = set()
    for a, b, pm in sc.groups:
        for s in range(a, b):
            covered.add(s)
            it = items[off[s]:off[s + 1]]
            verts = it[:, None] if st[s] in (scenes.CONTACT, scenes.BODY) else cv[st[s]][it]
            pc = pm[verts]
            assert np.all(pc == pc[:, :1])
    assert covered == set(range(len(st)))


def test_profile_family_count_matches_header():
    txt = open(os.path.join(ROOT, "include", "xpbd.h")).read()
    m = re.search(r"xpbd_profile_read\(xpbd_ctx ctx, int64_t launches\[(\d+)\], double ms\[(\d+)\], "
                  r"int64_t items\[(\d+)\]\)", txt)
    assert m and len(set(m.groups())) == 1
    assert int(m.group(1)) == L.N_FAMILIES


@pytest.mark.parametrize("bs", [32, 96, 2048, -64])
def test_rejects_bad_block_size(bs):
    rc, _, msg = _create(scenes.small_cloth(n=4), block_size=bs)
    assert rc == L.XPBD_ERR_INVALID and "block_size" in msg


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_periodic_tet_colouring_is_a_valid_33_set_schedule(n):
    sc = scenes.tet_box(n)
    st, off, items = sc.schedule_arrays()
    assert len(st) == 33 and np.all(st == scenes.TET)
    seen = np.zeros(sc.n_tet, int)
    for k in range(len(st)):
        it = items[off[k]:off[k + 1]]
        v = sc.tet_v[it].ravel()
        assert len(np.unique(v)) == len(v)
        seen[it] += 1
    assert np.all(seen == 1)
    if n >= 8:   # on large boxes the greedy colouring of the 2-periodic classes needs more sets
        assert len(scenes.tet_box(n, colouring="greedy").set_type) > 33

"""Seeded synthetic scene generators shared by the GPU path and its FP64 checker.

This module builds *inputs only*: mesh topology, rest positions, inverse
masses, the ordered list of independent constraint sets (the Gauss-Seidel
colour schedule), parameter fields, initial state and external-force fields.
It holds none of the simulation's arithmetic (no constraint functions, no
rest lengths, angles or rest-shape matrices, no projections): every consumer
derives those from the rest positions on its own.

Readings of the paper's unstated scene parameters (all marked "reading"):

* Cloth grids lie in the plane y = 0, y is up, gravity is (0, -9.81, 0);
  every quad (i, j)-(i+1, j+1) is split along that diagonal.
* Bending uses one hinge per interior edge: hinge (v0, v1), wing v2 in the
  triangle (v0, v1, v2) and wing v3 in the triangle (v1, v0, v3).  The paper
  names a discrete bending term for cloth (Sec. "Cloth Material Parameter
  Estimation") without a formula; the constraint is the signed dihedral angle.
* Tet boxes split each cube into 5 tets, alternating the split with the
  parity of (i + j + k) so neighbouring cubes conform; mass is lumped
  (rho * V_e / 4 per incident tet corner), the y = 0 face is pinned.
* Grid cloths: 6 distance and 12 bending sets, each touching every vertex
  once (greedy first-fit over batches independent by construction yields
  exactly these); tet boxes: 33 sets from a 4-periodic colouring table.
  Each colour is sorted by its smallest vertex index (locality).  Any schedule whose sets are vertex
  disjoint is valid input; both consumers replay it in the same order.

RNG: ``numpy.random.default_rng(seed)`` (PCG64), values drawn in the order
written here.  Seeds: 1 parameters, 2 target parameters, 4 force field,
5 keyframe force field, 6 serving arrivals.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

DIST, BEND, TET, CONTACT, TRI, BODY = 0, 1, 2, 3, 4, 5
TYPE_NAMES = {DIST: "dist", BEND: "bend", TET: "tet", CONTACT: "contact"}
GRAVITY = (0.0, -9.81, 0.0)
# Lattice spacing (m) of the tet-box workloads.  With 2 substeps of 1/120 s
# and 20 iterations, the deviatoric constraint sqrt(tr F^T F), which never
# vanishes and is held at rest only by the hydrostatic one, is projected
# hard when the tets are small against the step: on a 1/64 m lattice of this
# material (E ~ 1e5 Pa, 1000 kg/m^3) the box sags by its own height and
# inverts tets within a frame, and the exact gradient grows past FP64's range
# over 20 frames.  At 0.25 m the 64^3 box settles by about 4% with no tet
# inverted (smallest volume ratio 0.59 at frame 20).
TET_SPACING = 0.25


@dataclass
class Scene:
    """One simulation problem: topology, schedule, options and parameters."""

    rest: np.ndarray                      # (V, 3) float64 rest positions
    inv_mass: np.ndarray                  # (V,) float64, 0 = pinned
    dist_v: np.ndarray                    # (n_dist, 2) int32
    bend_v: np.ndarray                    # (n_bend, 4) int32
    tet_v: np.ndarray                     # (n_tet, 4) int32
    tet_nu: np.ndarray                    # (n_tet,) float64 Poisson ratio
    contact: bool = False
    contact_thickness: float = 0.005
    contact_compliance: float = 1e-9
    # schedule: ordered independent sets of one constraint type each
    set_type: List[int] = field(default_factory=list)
    set_items: List[np.ndarray] = field(default_factory=list)
    dt: float = 1.0 / 60.0
    substeps: int = 1
    iterations: int = 20
    gravity: Tuple[float, float, float] = GRAVITY
    n_frames: int = 1
    # parameters (controls)
    dist_alpha: Optional[np.ndarray] = None   # (n_dist,) compliance [m/N]
    bend_alpha: Optional[np.ndarray] = None   # (n_bend,) compliance [1/(N m)]
    tet_E: Optional[np.ndarray] = None        # (n_tet,) Young's modulus [Pa]; (n_materials,) with clusters
    sphere: Tuple[float, float, float, float] = (0.0, -1e3, 0.0, 1.0)
    f_ext: Optional[np.ndarray] = None        # (F, V, 3) per-vertex force [N]
    x0: Optional[np.ndarray] = None           # (V, 3)
    v0: Optional[np.ndarray] = None           # (V, 3)
    name: str = ""
    # optional LDS groups: (first set, one past last set, patch id per vertex)
    groups: List[Tuple[int, int, np.ndarray]] = field(default_factory=list)
    # optional material clusters: tet t uses parameter tet_material[t] of
    # n_materials (0 = one parameter per tet)
    n_materials: int = 0
    tet_material: Optional[np.ndarray] = None   # (n_tet,) int32
    # orthotropic StVK membrane triangles: vertices, warp/weft (u, v)
    # coordinates of their corners, and per-triangle coefficients
    # (C00, C01, C11, C22) of the stiffness block A K = alpha^-1
    tri_v: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int32))
    tri_uv: np.ndarray = field(default_factory=lambda: np.zeros((0, 6), np.float64))
    tri_coef: Optional[np.ndarray] = None   # (n_tri, 4)
    # body collider: a triangle mesh with outward normals ((b - a) x (c - a));
    # body_x is a control (the body's vertex positions, constant over a rollout)
    body_tris: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int32))
    body_x: Optional[np.ndarray] = None     # (n_body_verts, 3)
    body_thickness: float = 0.005
    body_compliance: float = 1e-9
    body_radius: float = 0.05               # pairing search radius

    @property
    def n_verts(self) -> int:
        return int(self.rest.shape[0])

    @property
    def n_dist(self) -> int:
        return int(self.dist_v.shape[0])

    @property
    def n_bend(self) -> int:
        return int(self.bend_v.shape[0])

    @property
    def n_tet(self) -> int:
        return int(self.tet_v.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri_v.shape[0])

    @property
    def n_body_tris(self) -> int:
        return int(self.body_tris.shape[0])

    @property
    def n_body_verts(self) -> int:
        return 0 if self.body_x is None else int(np.asarray(self.body_x).shape[0])

    @property
    def n_tet_params(self) -> int:
        """Length of the tet parameter arrays: materials, else tets."""
        return self.n_materials if self.n_materials else self.n_tet

    def schedule_arrays(self):
        """Flatten the schedule to (set_type int32, set_offsets int64, set_items int32)."""
        st = np.asarray(self.set_type, dtype=np.int32)
        sizes = [len(s) for s in self.set_items]
        off = np.zeros(len(sizes) + 1, dtype=np.int64)
        off[1:] = np.cumsum(sizes)
        items = (np.concatenate(self.set_items).astype(np.int32)
                 if self.set_items else np.zeros(0, np.int32))
        return st, off, items

    def projections_per_iteration(self) -> int:
        """Constraint evaluations in one Gauss-Seidel sweep (tets count D and H)."""
        n = self.n_dist + self.n_bend + 2 * self.n_tet + self.n_tri
        if self.contact:
            n += int(np.count_nonzero(self.inv_mass > 0))
        n += sum(len(it) for t, it in zip(self.set_type, self.set_items) if t == BODY)
        return n

    def projections_per_rollout(self, n_frames: Optional[int] = None) -> int:
        f = self.n_frames if n_frames is None else n_frames
        return self.projections_per_iteration() * self.iterations * self.substeps * f


# ---------------------------------------------------------------- colouring

def greedy_color(cverts: np.ndarray, batches: List[np.ndarray], n_verts: int,
                 subset: bool = False) -> np.ndarray:
    """Greedy first-fit colouring, visiting ``batches`` in order.

    Each batch must be vertex-disjoint (independent by construction), so its
    members are coloured simultaneously; the result equals sequential
    first-fit in (batch, member) order.  At most 64 colours.  With
    ``subset`` the batches may cover only some constraints; the others get
    colour -1.
    """
    cverts = np.asarray(cverts)
    vmask = np.zeros(n_verts, dtype=np.uint64)
    color = np.full(cverts.shape[0], -1, dtype=np.int32)
    for b in batches:
        if len(b) == 0:
            continue
        cv = cverts[b]
        used = np.bitwise_or.reduce(vmask[cv], axis=1)
        if np.any(used == np.uint64(0xFFFFFFFFFFFFFFFF)):
            raise ValueError("more than 64 colours needed")
        free = (~used) & (used + np.uint64(1))
        c = np.log2(free.astype(np.float64)).astype(np.int32)
        color[b] = c
        bits = np.left_shift(np.uint64(1), c.astype(np.uint64))
        for col in range(cv.shape[1]):
            vmask[cv[:, col]] |= bits
    if not subset and np.any(color < 0):
        raise ValueError("a constraint was not in any batch")
    return color


def sets_from_colors(cverts: np.ndarray, color: np.ndarray) -> List[np.ndarray]:
    """One set per colour (ascending), each sorted by its smallest vertex."""
    out = []
    key = np.min(cverts, axis=1) if len(cverts) else np.zeros(0, np.int64)
    for c in range(int(color.max()) + 1 if len(color) else 0):
        idx = np.nonzero(color == c)[0]
        if len(idx) == 0:
            continue
        idx = idx[np.argsort(key[idx], kind="stable")]
        out.append(idx.astype(np.int32))
    return out


# ---------------------------------------------------------------- cloth grid

def cloth_grid_topology(nr: int, nc: int):
    """Edges (H, V, D in row-major order), hinges and independent batches."""
    k = np.arange(nr * nc, dtype=np.int64).reshape(nr, nc)
    ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    eh = np.stack([k[:, :-1].ravel(), k[:, 1:].ravel()], 1)
    ev = np.stack([k[:-1, :].ravel(), k[1:, :].ravel()], 1)
    ed = np.stack([k[:-1, :-1].ravel(), k[1:, 1:].ravel()], 1)
    dist_v = np.concatenate([eh, ev, ed]).astype(np.int32)
    nh, nv = len(eh), len(ev)
    # independent batches: H by column parity, V and D by row parity
    bh_j = jj[:, :-1].ravel()
    bv_i = ii[:-1, :].ravel()
    bd_i = ii[:-1, :-1].ravel()
    dist_batches = [np.nonzero(bh_j % 2 == p)[0] for p in (0, 1)]
    dist_batches += [nh + np.nonzero(bv_i % 2 == p)[0] for p in (0, 1)]
    dist_batches += [nh + nv + np.nonzero(bd_i % 2 == p)[0] for p in (0, 1)]

    # hinges: (v0, v1) edge, v2 wing of triangle (v0, v1, v2), v3 of (v1, v0, v3)
    hh = np.stack([k[1:-1, :-1], k[1:-1, 1:], k[2:, 1:], k[:-2, :-1]], -1).reshape(-1, 4)
    hv = np.stack([k[:-1, 1:-1], k[1:, 1:-1], k[1:, 2:], k[:-1, :-2]], -1).reshape(-1, 4)
    hd = np.stack([k[:-1, :-1], k[1:, 1:], k[:-1, 1:], k[1:, :-1]], -1).reshape(-1, 4)
    bend_v = np.concatenate([hh, hv, hd]).astype(np.int32)
    n_hh, n_hv = len(hh), len(hv)
    hi, hj = ii[1:-1, :-1].ravel(), jj[1:-1, :-1].ravel()
    vi, vj = ii[:-1, 1:-1].ravel(), jj[:-1, 1:-1].ravel()
    di, dj = ii[:-1, :-1].ravel(), jj[:-1, :-1].ravel()
    # each batch touches every vertex at most once, and (away from the
    # border) every vertex exactly once: H hinges of rows i, i + 2 meet row
    # i + 1 in columns of opposite parity, likewise V hinges; D hinges are
    # the 2x2 quads of one parity class.  Twelve batches is the minimum
    # (twelve hinges share an interior vertex), and dense sets read and write
    # whole cache lines of the vertex array.
    bend_batches = []
    for a in range(2):
        for b in range(2):
            bend_batches.append(np.nonzero((hi % 2 == a) & (hj % 2 == b))[0])
    for a in range(2):
        for b in range(2):
            bend_batches.append(n_hh + np.nonzero((vj % 2 == a) & (vi % 2 == b))[0])
    for a in range(2):
        for b in range(2):
            bend_batches.append(n_hh + n_hv + np.nonzero((di % 2 == a) & (dj % 2 == b))[0])
    return dist_v, dist_batches, bend_v, bend_batches


def cloth_grid(nr: int, nc: int, spacing: float, origin=(0.0, 0.0, 0.0),
               pinned=(), bending: bool = True, contact: bool = False) -> Scene:
    """A flat nr x nc particle grid in y = 0, vertex k = i * nc + j at
    origin + (j * spacing, 0, i * spacing); unit mass; ``pinned`` vertices
    get inverse mass 0."""
    ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    rest = np.zeros((nr * nc, 3), dtype=np.float64)
    rest[:, 0] = origin[0] + jj.ravel() * spacing
    rest[:, 1] = origin[1]
    rest[:, 2] = origin[2] + ii.ravel() * spacing
    inv_mass = np.ones(nr * nc, dtype=np.float64)
    for p in pinned:
        inv_mass[p] = 0.0
    dist_v, dist_batches, bend_v, bend_batches = cloth_grid_topology(nr, nc)
    if not bending:
        bend_v = np.zeros((0, 4), np.int32)
        bend_batches = []
    sc = Scene(rest=rest, inv_mass=inv_mass, dist_v=dist_v, bend_v=bend_v,
               tet_v=np.zeros((0, 4), np.int32), tet_nu=np.zeros(0), contact=contact)
    n_verts = nr * nc
    dcol = greedy_color(dist_v, dist_batches, n_verts)
    for s in sets_from_colors(dist_v, dcol):
        sc.set_type.append(DIST)
        sc.set_items.append(s)
    if bending and len(bend_v):
        bcol = greedy_color(bend_v, bend_batches, n_verts)
        for s in sets_from_colors(bend_v, bcol):
            sc.set_type.append(BEND)
            sc.set_items.append(s)
    if contact:
        free = np.nonzero(inv_mass > 0)[0].astype(np.int32)
        sc.set_type.append(CONTACT)
        sc.set_items.append(free)
    sc.x0 = rest.copy()
    sc.v0 = np.zeros_like(rest)
    return sc


# ---------------------------------------------------------------- tet box

# 5-tet split of a unit cube; corners indexed by (a, b, c) bits.  Even cubes
# use corner tets at (000), (110), (101), (011); odd cubes the mirror set.
_EVEN = [((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)),
         ((1, 1, 0), (0, 1, 0), (1, 0, 0), (1, 1, 1)),
         ((1, 0, 1), (0, 0, 1), (1, 1, 1), (1, 0, 0)),
         ((0, 1, 1), (0, 1, 0), (0, 0, 1), (1, 1, 1)),
         ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1))]
_ODD = [((1, 0, 0), (0, 0, 0), (1, 1, 0), (1, 0, 1)),
        ((0, 1, 0), (1, 1, 0), (0, 0, 0), (0, 1, 1)),
        ((0, 0, 1), (1, 0, 1), (0, 1, 1), (0, 0, 0)),
        ((1, 1, 1), (0, 1, 1), (1, 0, 1), (1, 1, 0)),
        ((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1))]


# Colour of tet slot t (0..4) of cube (i, j, k) by (i mod 4, j mod 4, k mod 4,
# t), one base-36 digit each, 33 colours.  Found by a tabu search over the
# colourings of the lattice folded onto a 4x4x4 torus (tets conflict when
# they share a vertex); a colouring of the torus is valid on every box.  The
# lower bound is 32 (32 tets share an even-parity vertex); the greedy
# colouring of the 2-periodic classes needs 40.
_TET_COLOUR_4 = (
    "dw310nosflq1vtwbjl7pa9bq6h7d3p90ak6elun3w7id4olgn1ba2wqsmjophktqc2p37jk905631v2njmug5ckbtea2gcd4stro8c4v2"
    "isjmr8uqi5nmhe01bk95fatwehl4bcgjrdtga68svr0omiurh879eif7ktdp0nw4l6s2vpel16b93q6w7b10hgo9w3f1uvapmn8olgd7js"
    "48p672lqkc4hi329kf1nq5m3wjvn0horf8gmbeirjo47dkgqms2vjcua2k5nv8tcrhi458bte0fsmprie9oud1frg596wa4ud5vt8haciflus")


def tet_box(n: int, size: float = 1.0, density: float = 1000.0,
            pin_bottom: bool = True, colouring: str = "periodic") -> Scene:
    """n^3 cubes over [0, size]^3, 5 tets per cube, vertex (i, j, k) at
    (i, j, k) * size / n with index (i * (n + 1) + j) * (n + 1) + k.
    ``colouring``: "periodic" (33 sets from the 4-periodic table) or
    "greedy" (greedy first-fit over the 40 classes cube parity x slot)."""
    n1 = n + 1
    ii, jj, kk = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    rest = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.float64) * (size / n)

    def vid(i, j, k):
        return (i * n1 + j) * n1 + k

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    par = (ci + cj + ck) % 2
    tets = np.zeros((len(ci), 5, 4), dtype=np.int64)
    for t in range(5):
        for c in range(4):
            ea, eb, ec = _EVEN[t][c]
            oa, ob, oc = _ODD[t][c]
            ve = vid(ci + ea, cj + eb, ck + ec)
            vo = vid(ci + oa, cj + ob, ck + oc)
            tets[:, t, c] = np.where(par == 0, ve, vo)
    tet_v = tets.reshape(-1, 4)
    # orient every tet so that det[x1-x0, x2-x0, x3-x0] > 0 (mesh validity)
    p = rest[tet_v]
    d1, d2, d3 = p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 3] - p[:, 0]
    vol6 = np.einsum("ij,ij->i", np.cross(d1, d2), d3)
    neg = vol6 < 0
    tet_v[neg, 2], tet_v[neg, 3] = tet_v[neg, 3].copy(), tet_v[neg, 2].copy()
    vol = np.abs(vol6) / 6.0
    mass = np.zeros(len(rest))
    np.add.at(mass, tet_v.ravel(), np.repeat(density * vol / 4.0, 4))
    inv_mass = 1.0 / mass
    if pin_bottom:
        inv_mass[rest[:, 1] == 0.0] = 0.0
    tet_v = tet_v.astype(np.int32)
    sc = Scene(rest=rest, inv_mass=inv_mass, dist_v=np.zeros((0, 2), np.int32),
               bend_v=np.zeros((0, 4), np.int32), tet_v=tet_v,
               tet_nu=np.full(len(tet_v), 0.3))
    if colouring == "periodic":
        table = np.array([int(ch, 36) for ch in _TET_COLOUR_4], np.int32).reshape(4, 4, 4, 5)
        col = table[ci % 4, cj % 4, ck % 4][:, :].reshape(-1)
    else:
        # batches: cube parity class (8) x tet slot (5) are vertex disjoint
        cls = (ci % 2) * 4 + (cj % 2) * 2 + (ck % 2)
        tid = np.arange(len(tet_v)).reshape(-1, 5)
        batches = []
        for c in range(8):
            cubes = np.nonzero(cls == c)[0]
            for t in range(5):
                batches.append(tid[cubes, t])
        col = greedy_color(tet_v, batches, len(rest))
    for s in sets_from_colors(tet_v, col):
        sc.set_type.append(TET)
        sc.set_items.append(s)
    sc.x0 = rest.copy()
    sc.v0 = np.zeros_like(rest)
    return sc


# ---------------------------------------------------------------- tiled schedules

def tiled_schedule(sc: Scene, coords: np.ndarray, tile: int, typed_batches, contact_last: bool = True):
    """Replace ``sc``'s schedule by a tiled one and record its LDS groups.

    ``coords`` are integer lattice coordinates of the vertices (V, d);
    tilings are the 2^d shifts of a ``tile``-wide lattice by 0 or tile/2 per
    axis.  Each constraint goes to the first tiling in which all its
    vertices fall in one tile; every tiling contributes its constraints as
    greedily coloured sets (distance, then bending, then tets), forming one
    group with that tiling's tile id per vertex.  The contact set closes
    the last group.  Constraints left over (none for tiles wider than twice
    a constraint's extent) follow as ungrouped sets.
    """
    d = coords.shape[1]
    V = sc.n_verts
    shifts = [tuple((m >> a) & 1 for a in range(d)) for m in range(2 ** d)]
    ext = coords.max(axis=0) + tile + 2
    maps = []
    for sh in shifts:
        cell = (coords + np.array(sh) * (tile // 2)) // tile
        pid = np.zeros(V, np.int64)
        for a in range(d):
            pid = pid * int(ext[a] // tile + 2) + cell[:, a]
        maps.append(pid.astype(np.int32))
    sets_t, sets_i, groups = [], [], []
    assign = {}
    for ty, cv, batches in typed_batches:
        a = np.full(len(cv), -1, np.int32)
        for t, pm in enumerate(maps):
            if len(cv) == 0:
                break
            pc = pm[cv]
            inside = np.all(pc == pc[:, :1], axis=1) & (a < 0)
            a[inside] = t
        assign[ty] = a
    for t, pm in enumerate(maps):
        first = len(sets_t)
        for ty, cv, batches in typed_batches:
            sel = assign[ty] == t
            if not np.any(sel):
                continue
            col = greedy_color(cv, [b[sel[b]] for b in batches], V, subset=True)
            for st in sets_from_colors(cv, col):
                sets_t.append(ty)
                sets_i.append(st)
        if contact_last and sc.contact and t == len(maps) - 1:
            sets_t.append(CONTACT)
            sets_i.append(np.nonzero(sc.inv_mass > 0)[0].astype(np.int32))
        if len(sets_t) > first:
            groups.append((first, len(sets_t), pm))
    for ty, cv, batches in typed_batches:
        sel = assign[ty] < 0
        if np.any(sel):
            col = greedy_color(cv, [b[sel[b]] for b in batches], V, subset=True)
            for st in sets_from_colors(cv, col):
                sets_t.append(ty)
                sets_i.append(st)
    sc.set_type, sc.set_items, sc.groups = sets_t, sets_i, groups
    return sc


def _group_sets(typed, sel_of, V):
    """Greedy sets of the selected constraints of each type, in type order."""
    out_t, out_i = [], []
    for ty, cv, batches in typed:
        sel = sel_of[ty]
        if not np.any(sel):
            continue
        col = greedy_color(cv, [b[sel[b]] for b in batches], V, subset=True)
        for st in sets_from_colors(cv, col):
            out_t.append(ty)
            out_i.append(st)
    return out_t, out_i


def tile_cloth_lines(sc: Scene, nr: int, nc: int, tile: int = 16, lds_groups=(0, 1, 2), merge=(1, 1)) -> Scene:
    """Three-group tiled schedule for an nr x nc grid cloth.

    Group A: constraints inside one tile x tile tile (patch = tile).
    Group B: constraints crossing exactly one tile border line, away from
    the tile corners (patch = the border segment between two corners; the
    segments are vertex-disjoint because every vertex within two rows of a
    row line and two columns of a column line is a corner vertex).
    Group C: the constraints that touch a corner vertex, then the contact
    set (patch = the tile of the half-shifted tiling around that corner).
    Every constraint is in exactly one group; an iteration runs A, B, C.
    ``lds_groups`` selects which of A, B, C (0, 1, 2) are offered to the
    library as LDS groups; the others run as ordinary sets.  ``merge`` = (mB,
    mC) joins runs of mB consecutive border segments and mC corner clusters
    into one patch (still vertex-disjoint), so one workgroup serves several
    of these small patches.  The schedule (and so every result) is the same
    either way.
    """
    dist_v, dist_batches, bend_v, bend_batches = cloth_grid_topology(nr, nc)
    V = sc.n_verts
    ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    ntj = nc // tile + 2
    tile_id = (ii // tile) * ntj + jj // tile
    near_r = np.isin(ii % tile, [tile - 2, tile - 1, 0, 1])
    near_c = np.isin(jj % tile, [tile - 2, tile - 1, 0, 1])
    corner = near_r & near_c
    h = tile // 2
    corner_tile = ((ii + h) // tile) * ntj + (jj + h) // tile
    # border segments: row line k (between rows tile*k - 1 and tile*k) within
    # column tile m, and column line m within row tile k
    row_line = (ii + 2) // tile
    col_line = (jj + 2) // tile
    nseg = (nr // tile + 2) * ntj
    seg_id = np.where(near_r, row_line * ntj + jj // tile, nseg + (ii // tile) * ntj + col_line)
    typed = []
    if sc.n_tri:
        tri_v, _uv, tri_batches = membrane_triangles(nr, nc, sc.rest)
        assert np.array_equal(tri_v, sc.tri_v)
        typed.append((TRI, sc.tri_v, tri_batches))
    if sc.n_dist:
        assert np.array_equal(dist_v, sc.dist_v)
        typed.append((DIST, sc.dist_v, dist_batches))
    if sc.n_bend:
        typed.append((BEND, sc.bend_v, bend_batches))
    verts_of = {ty: cv for ty, cv, _ in typed}
    sel = {}
    for ty, cv, _ in typed:
        t = tile_id[cv]
        in_a = np.all(t == t[:, :1], axis=1)
        touches_corner = np.any(corner[cv], axis=1)
        sel[ty] = (in_a, ~in_a & ~touches_corner, ~in_a & touches_corner)
    sets_t, sets_i, groups = [], [], []
    for g, pm in enumerate((tile_id, seg_id // max(1, merge[0]), corner_tile // max(1, merge[1]))):
        first = len(sets_t)
        st, si = _group_sets(typed, {ty: sel[ty][g] for ty, _, _ in typed}, V)
        sets_t += st
        sets_i += si
        if g == 2 and sc.contact:
            sets_t.append(CONTACT)
            sets_i.append(np.nonzero(sc.inv_mass > 0)[0].astype(np.int32))
        if len(sets_t) > first:
            groups.append((first, len(sets_t), pm.astype(np.int32)))
    groups = [g for k, g in enumerate(groups) if k in tuple(lds_groups)]
    # every constraint must lie within one patch of its group
    for (a, b, pm) in groups:
        for k in range(a, b):
            if sets_t[k] == CONTACT:
                continue
            cv = verts_of[sets_t[k]][sets_i[k]]
            p = pm[cv]
            assert np.all(p == p[:, :1]), "tiling left a constraint across patches"
    sc.set_type, sc.set_items, sc.groups = sets_t, sets_i, groups
    return sc


def tile_cloth_quads(sc: Scene, nr: int, nc: int, tile: int = 32) -> Scene:
    """Four-group tiled schedule for an nr x nc grid cloth.

    Every constraint belongs to the tile of its anchor (the smallest row and
    the smallest column among its vertices); its vertices lie within two rows
    and two columns of the anchor, so the patch of a tile is the tile plus
    the two rows and columns after it.  Group g = (tile row parity, tile
    column parity) holds the constraints of the tiles of that colour: two
    tiles of one colour are at least a tile apart, so their patches share no
    vertex, and every group is a set of whole tiles with no border groups.
    An iteration runs the four groups in colour order, then the contact set
    as a fifth group of whole tiles (patch = the tile holding the vertex).
    Membrane triangles (the membrane cloth) come first in each group.
    """
    dist_v, dist_batches, bend_v, bend_batches = cloth_grid_topology(nr, nc)
    V = sc.n_verts
    ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    ntj = (nc + tile - 1) // tile
    typed = []
    if sc.n_tri:
        tri_v, _uv, tri_batches = membrane_triangles(nr, nc, sc.rest)
        assert np.array_equal(tri_v, sc.tri_v)
        typed.append((TRI, sc.tri_v, tri_batches))
    if sc.n_dist:
        assert np.array_equal(dist_v, sc.dist_v)
        typed.append((DIST, sc.dist_v, dist_batches))
    if sc.n_bend:
        assert np.array_equal(bend_v, sc.bend_v)
        typed.append((BEND, sc.bend_v, bend_batches))
    verts_of = {ty: cv for ty, cv, _ in typed}
    anchor, colour = {}, {}
    for ty, cv, _ in typed:
        ar, ac = ii[cv].min(axis=1) // tile, jj[cv].min(axis=1) // tile
        assert np.all(ii[cv].max(axis=1) - ii[cv].min(axis=1) <= 2)
        assert np.all(jj[cv].max(axis=1) - jj[cv].min(axis=1) <= 2)
        anchor[ty] = ar * ntj + ac
        colour[ty] = (ar % 2) * 2 + ac % 2
    sets_t, sets_i, groups = [], [], []
    for g in range(4):
        sel = {ty: colour[ty] == g for ty, _, _ in typed}
        first = len(sets_t)
        st, si = _group_sets(typed, sel, V)
        sets_t += st
        sets_i += si
        if len(sets_t) == first:
            continue
        pm = (ii // tile) * ntj + jj // tile        # vertices outside the group: any
        for ty, cv, _ in typed:
            k = sel[ty]
            pm[cv[k].ravel()] = np.repeat(anchor[ty][k], cv.shape[1])
        groups.append((first, len(sets_t), pm.astype(np.int32)))
    if sc.contact:
        first = len(sets_t)
        sets_t.append(CONTACT)
        sets_i.append(np.nonzero(sc.inv_mass > 0)[0].astype(np.int32))
        groups.append((first, first + 1, ((ii // tile) * ntj + jj // tile).astype(np.int32)))
    for (a, b, pm) in groups:
        for k in range(a, b):
            if sets_t[k] == CONTACT:
                continue
            cv = verts_of[sets_t[k]][sets_i[k]]
            p = pm[cv]
            assert np.all(p == p[:, :1]), "tiling left a constraint across patches"
    sc.set_type, sc.set_items, sc.groups = sets_t, sets_i, groups
    return sc


def tile_cloth(sc: Scene, nr: int, nc: int, tile: int = 16) -> Scene:
    """Tiled schedule for an nr x nc grid cloth (4 tilings of tile x tile)."""
    dist_v, dist_batches, bend_v, bend_batches = cloth_grid_topology(nr, nc)
    assert np.array_equal(dist_v, sc.dist_v)
    ii, jj = np.meshgrid(np.arange(nr), np.arange(nc), indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel()], 1)
    typed = [(DIST, sc.dist_v, dist_batches)]
    if sc.n_bend:
        typed.append((BEND, sc.bend_v, bend_batches))
    return tiled_schedule(sc, coords, tile, typed)


def tile_box(sc: Scene, n: int, tile: int = 4) -> Scene:
    """Tiled schedule for an n^3-cube tet box (8 tilings of tile^3 cubes)."""
    n1 = n + 1
    ii, jj, kk = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    coords = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    cls = ((ci % 2) * 4 + (cj % 2) * 2 + (ck % 2)).ravel()
    tid = np.arange(sc.n_tet).reshape(-1, 5)
    batches = [tid[np.nonzero(cls == c)[0], t] for c in range(8) for t in range(5)]
    return tiled_schedule(sc, coords, tile, [(TET, sc.tet_v, batches)])


# ---------------------------------------------------------------- parameter fields

def lognormal(rng, mu, sigma, n):
    return np.exp(rng.normal(mu, sigma, n))


def force_field(seed: int, nr: int, nc: int, n_frames: int, amplitude: float = 2.0,
                frames_period: int = 20) -> np.ndarray:
    """Smooth per-vertex force sequence (F, V, 3).

    Per component c: A * sum_m a_m sin(2 pi (p_m u + q_m v + r_m f / 20) + phi_m)
    with u = j/(nc-1), v = i/(nr-1), p, q, r in {1, 2, 3}, a ~ N(0, 1),
    phi ~ U[0, 2 pi).  Draw order: p, q, r, a, phi, each of shape (3, 4).
    """
    rng = np.random.default_rng(seed)
    p = rng.integers(1, 4, size=(3, 4))
    q = rng.integers(1, 4, size=(3, 4))
    r = rng.integers(1, 4, size=(3, 4))
    a = rng.standard_normal((3, 4))
    phi = rng.uniform(0.0, 2.0 * np.pi, (3, 4))
    u = (np.arange(nc) / max(nc - 1, 1))[None, :]
    v = (np.arange(nr) / max(nr - 1, 1))[:, None]
    out = np.zeros((n_frames, nr * nc, 3), dtype=np.float64)
    # sin(S + T) = sin S cos T + cos S sin T with S the spatial phase and
    # T = 2 pi r (f + 1) / frames_period the temporal one
    sS = np.empty((3, 4, nr * nc))
    cS = np.empty((3, 4, nr * nc))
    for c in range(3):
        for m in range(4):
            S = (2 * np.pi * (p[c, m] * u + q[c, m] * v) + phi[c, m]).ravel()
            np.sin(S, out=sS[c, m])
            np.cos(S, out=cS[c, m])
    acc = np.empty(nr * nc)
    tmp = np.empty(nr * nc)
    for f in range(n_frames):
        for c in range(3):
            acc.fill(0.0)
            for m in range(4):
                T = 2 * np.pi * r[c, m] * (f + 1) / frames_period
                np.multiply(sS[c, m], amplitude * a[c, m] * np.cos(T), out=tmp)
                acc += tmp
                np.multiply(cS[c, m], amplitude * a[c, m] * np.sin(T), out=tmp)
                acc += tmp
            out[f, :, c] = acc
    return out


def cloth_alpha(seed: int, n_dist: int, n_bend: int, mu=-16.0, sigma=0.5):
    rng = np.random.default_rng(seed)
    return lognormal(rng, mu, sigma, n_dist), lognormal(rng, mu, sigma, n_bend)


def tet_material(seed: int, n_tet: int, nu=None):
    """(E, nu): E ~ lognormal(ln 1e5, 0.3), then nu ~ U[0.3, 0.45]."""
    rng = np.random.default_rng(seed)
    E = lognormal(rng, np.log(1e5), 0.3, n_tet)
    nu_draw = rng.uniform(0.3, 0.45, n_tet)
    return E, (nu_draw if nu is None else nu)


# ---------------------------------------------------------------- configurations

def config_c1(n_frames: int = 60, target: bool = False) -> Scene:
    """32x32 cloth over a 1 m square, corners of row 0 pinned, ~3k edges,
    compliance 1e-7 * U[0.5, 2] per edge, dt 1/60, 1 substep, 20 iterations."""
    n = 32
    sc = cloth_grid(n, n, 1.0 / (n - 1), pinned=(0, n - 1), bending=False)
    rng = np.random.default_rng(2 if target else 1)
    sc.dist_alpha = 1e-7 * rng.uniform(0.5, 2.0, sc.n_dist)
    sc.bend_alpha = np.zeros(0)
    sc.tet_E = np.zeros(0)
    sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, 1, 20, n_frames
    sc.name = "cloth32_dist_fp64"
    return sc


def config_c2(n_frames: int = 30, target: bool = False, n: int = 256, tile: int = 16,
              tiling: str = "lines") -> Scene:
    """256x256 cloth centred at the origin with distance + bending + sphere
    contact (c = (0, -0.35, 0), R = 0.3), dt 1/60, 4 substeps, 30 iterations.
    tile > 0: tiled schedule, either three groups (tiles, border segments,
    corners: ``tiling="lines"``) or four shifted tilings (``"shifts"``)."""
    sc = cloth_grid(n, n, 1.0 / (n - 1), origin=(-0.5, 0.0, -0.5), contact=True)
    if tile:
        (tile_cloth_lines if tiling == "lines" else tile_cloth)(sc, n, n, tile)
    sc.dist_alpha, sc.bend_alpha = cloth_alpha(2 if target else 1, sc.n_dist, sc.n_bend)
    sc.tet_E = np.zeros(0)
    sc.sphere = (0.0, -0.35, 0.0, 0.3)
    sc.contact_thickness, sc.contact_compliance = 0.005, 1e-9
    sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, 4, 30, n_frames
    sc.name = f"cloth{n}_dist_bend_sphere"
    return sc


def config_c2_membrane(n_frames: int = 30, target: bool = False, n: int = 256, tile: int = 16,
                       tiling: str = "lines") -> Scene:
    """The 256x256 cloth with orthotropic StVK membrane triangles in place of
    the distance constraints (Sec. 5.1's cloth model), dihedral bending and
    the sphere; per-triangle coefficients (C00, C01, C11, C22) =
    (4e3, 6e2, 2e3, 8e2) N/m x U[0.7, 1.3] (seed 1, seed 2 for the target);
    8 membrane sets, 12 bending sets, 1 contact set per iteration.  Mass
    from an areal density of 0.2 kg/m^2 (3.1 mg per vertex): with the grid's
    unit mass per vertex these coefficients let the 65 t sheet stretch
    several-fold under its own weight over 30 frames.  tile > 0:
    a tiled schedule with LDS groups, tiles + border segments + corners
    (``tiling="lines"``, 16 x 16 by default: 668 ms per step against 780 ms
    with one launch per set on MI355X) or four colours of whole tiles
    (``"quads"``); 0: the untiled sets."""
    sc = membrane_cloth(n=n, frames=n_frames, substeps=4, iterations=30, sphere=True, pinned=(),
                        seed=2 if target else 1)
    sc.inv_mass = np.where(sc.inv_mass > 0, (n - 1) ** 2 / 0.2, 0.0)
    if tile:
        (tile_cloth_lines if tiling == "lines" else tile_cloth_quads)(sc, n, n, tile)
    sc.sphere = (0.0, -0.35, 0.0, 0.3)
    sc.contact_thickness, sc.contact_compliance = 0.005, 1e-9
    sc.name = f"cloth{n}_membrane_bend_sphere"
    return sc


def config_c2_body(n_frames: int = 30, target: bool = False, n: int = 256, body_res=(64, 128),
                   tile: int = 16) -> Scene:
    """The 256x256 cloth (distance + bending) falling onto a body collider
    given as a triangle mesh: a UV sphere of 64 x 128 (16,128 triangles)
    standing where the sphere collider is, tau 0.005, alpha 1e-9, search
    radius 0.02; one body-contact set of every vertex.  tile > 0: the cloth's
    three-group tiling with the body-contact set in the corner group (where
    the sphere's contact set sits); 0: untiled sets, one launch each."""
    sc = config_c2(n_frames=n_frames, target=target, n=n, tile=tile)
    sc.contact = False
    free = np.nonzero(sc.inv_mass > 0)[0].astype(np.int32)
    if tile:
        k = sc.set_type.index(CONTACT)
        sc.set_type[k], sc.set_items[k] = BODY, free
    else:
        keep = [(t, it) for t, it in zip(sc.set_type, sc.set_items) if t != CONTACT]
        sc.set_type = [t for t, _ in keep] + [BODY]
        sc.set_items = [it for _, it in keep] + [free]
    bx, bt = uv_sphere((0.0, -0.35, 0.0), 0.3, *body_res)
    sc.body_x, sc.body_tris = bx, bt
    sc.body_thickness, sc.body_compliance, sc.body_radius = 0.005, 1e-9, 0.02
    sc.name = f"cloth{n}_dist_bend_body{len(bt)}"
    return sc


def config_c3(n_frames: int = 20, target: bool = False, n: int = 64, tile: int = 0) -> Scene:
    """64^3-cube tet box (5 tets per cube) on a TET_SPACING lattice (16 m
    across), density 1000 kg/m^3, bottom pinned, Neo-Hookean, dt 1/60,
    2 substeps, 20 iterations.  tile > 0: tiled schedule (8 shifted tilings
    of tile^3 cubes)."""
    sc = tet_box(n, size=n * TET_SPACING)
    if tile:
        tile_box(sc, n, tile)
    E, nu = tet_material(1, sc.n_tet)
    if target:
        E = tet_material(2, sc.n_tet, nu=nu)[0]
    sc.tet_E, sc.tet_nu = E, nu
    sc.dist_alpha, sc.bend_alpha = np.zeros(0), np.zeros(0)
    sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, 2, 20, n_frames
    sc.name = f"tetbox{n}_neohookean"
    return sc


def config_c4(n_frames: int = 20, nr: int = 4096, nc: int = 2048, force_seed: int = 4, tile: int = 32,
              tiling: str = "lines", lds_groups=(0, 1, 2), merge=(16, 32)) -> Scene:
    """2048 x 4096 cloth (8.4M vertices, 25.2M DoF), row-0 corners pinned,
    distance + bending, per-frame per-vertex force controls, dt 1/60,
    2 substeps, 20 iterations.  tile > 0: three-group tiled schedule (tile
    interiors, border segments, corners) with the groups in ``lds_groups``
    offered as LDS groups; 0: the dense 6 + 12 set schedule.  32 x 32 tiles
    with all three groups in LDS, 16 border segments and 32 corner clusters
    per patch, measured fastest on MI355X (with constraint entries and state
    streamed from global memory and 256-thread workgroups)."""
    sc = cloth_grid(nr, nc, 1.0 / (nc - 1), pinned=(0, nc - 1))
    if tile:
        if tiling == "lines":
            tile_cloth_lines(sc, nr, nc, tile, lds_groups=lds_groups, merge=merge)
        elif tiling == "quads":
            tile_cloth_quads(sc, nr, nc, tile)
        else:
            tile_cloth(sc, nr, nc, tile)
    sc.dist_alpha, sc.bend_alpha = cloth_alpha(1, sc.n_dist, sc.n_bend)
    sc.tet_E = np.zeros(0)
    sc.f_ext = force_field(force_seed, nr, nc, n_frames)
    sc.n_frames = n_frames
    sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, 2, 20, n_frames
    sc.name = f"cloth{nc}x{nr}_dist_bend_force"
    return sc


def membrane_triangles(nr: int, nc: int, rest: np.ndarray):
    """Triangles of an nr x nc grid (each quad (i, j) split along
    (i, j)-(i+1, j+1)), their warp/weft coordinates (u, v) = (x, z) of the
    flat rest grid, and 8 vertex-disjoint sets: quads of equal (i mod 2,
    j mod 2) share no vertex, times the two triangles of a quad."""
    ii, jj = np.meshgrid(np.arange(nr - 1), np.arange(nc - 1), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    v00, v01 = ii * nc + jj, ii * nc + jj + 1
    v10, v11 = (ii + 1) * nc + jj, (ii + 1) * nc + jj + 1
    tri = np.concatenate([np.stack([v00, v01, v11], 1), np.stack([v00, v11, v10], 1)]).astype(np.int32)
    uv = rest[tri][:, :, [0, 2]].reshape(-1, 6)
    nq = len(ii)
    cls = (ii % 2) * 2 + (jj % 2)
    sets = []
    for slot in range(2):
        for c in range(4):
            sets.append((np.nonzero(cls == c)[0] + slot * nq).astype(np.int32))
    return tri, uv, sets


def membrane_cloth(n: int = 6, frames: int = 3, substeps: int = 2, iterations: int = 5, sphere: bool = True,
                   pinned=None, seed: int = 1, coef=(4.0e3, 6.0e2, 2.0e3, 8.0e2)) -> Scene:
    """Cloth of orthotropic StVK membrane triangles (Sec. 5.1) with dihedral
    bending and an optional sphere: per-triangle coefficients (C00, C01,
    C11, C22) = coef times U[0.7, 1.3] each (seed), warp along x, weft
    along z.  One iteration runs the 8 membrane sets, the bending sets and
    the contact set."""
    pins = (0, n - 1) if pinned is None else pinned
    sc = cloth_grid(n, n, 1.0 / (n - 1), origin=(-0.5, 0.0, -0.5), pinned=pins, contact=sphere)
    tri, uv, tsets = membrane_triangles(n, n, sc.rest)
    # the distance constraints give way to the membrane
    keep = [(t, it) for t, it in zip(sc.set_type, sc.set_items) if t != DIST]
    sc.dist_v = np.zeros((0, 2), np.int32)
    sc.set_type = [TRI] * len(tsets) + [t for t, _ in keep]
    sc.set_items = list(tsets) + [it for _, it in keep]
    sc.tri_v, sc.tri_uv = tri, uv
    rng = np.random.default_rng(seed)
    sc.tri_coef = np.asarray(coef, np.float64)[None, :] * rng.uniform(0.7, 1.3, (len(tri), 4))
    sc.dist_alpha = np.zeros(0)
    sc.bend_alpha = 1e-3 * rng.uniform(0.5, 2.0, sc.n_bend)
    sc.tet_E = np.zeros(0)
    sc.sphere = (0.05, -0.28, -0.03, 0.3)
    sc.contact_thickness, sc.contact_compliance = 0.005, 1e-7
    sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, substeps, iterations, frames
    sc.name = f"cloth{n}_membrane"
    return sc


def uv_sphere(center=(0.0, 0.0, 0.0), radius: float = 0.3, n_lat: int = 8, n_lon: int = 16):
    """Closed triangle mesh of a sphere: two poles and n_lat - 1 rings of
    n_lon vertices; triangles oriented so (b - a) x (c - a) points outward."""
    c = np.asarray(center, np.float64)
    verts = [c + [0.0, radius, 0.0]]
    for i in range(1, n_lat):
        th = np.pi * i / n_lat
        for j in range(n_lon):
            ph = 2 * np.pi * j / n_lon
            verts.append(c + radius * np.array([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)]))
    verts.append(c + [0.0, -radius, 0.0])
    V = np.array(verts)
    south = len(verts) - 1
    ring = lambda i, j: 1 + (i - 1) * n_lon + (j % n_lon)
    tris = []
    for j in range(n_lon):
        tris.append((0, ring(1, j), ring(1, j + 1)))
        tris.append((south, ring(n_lat - 1, j + 1), ring(n_lat - 1, j)))
    for i in range(1, n_lat - 1):
        for j in range(n_lon):
            a, b, cc, d = ring(i, j), ring(i, j + 1), ring(i + 1, j), ring(i + 1, j + 1)
            tris += [(a, cc, b), (b, cc, d)]
    T = np.array(tris, np.int32)
    nrm = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, V[T].mean(axis=1) - c) < 0
    T[flip, 1], T[flip, 2] = T[flip, 2].copy(), T[flip, 1].copy()
    return V, T


def body_shape_modes(body_x, center):
    """Synthetic linear shape model of the body (the stand-in for a
    statistical body model's blend shapes): x_body(a) = x0 + sum_k a_k S_k
    with S_0..S_2 stretching along x, y, z about the centre and S_3 a smooth
    bulge on the upper half.  Returns S (4, n_body_verts, 3)."""
    d = np.asarray(body_x, np.float64) - np.asarray(center, np.float64)
    S = np.zeros((4,) + d.shape)
    for k in range(3):
        S[k][:, k] = d[:, k]
    r = np.linalg.norm(d, axis=1, keepdims=True)
    up = np.clip(d[:, 1:2] / np.maximum(r, 1e-12), 0.0, None)
    S[3] = up ** 2 * d / np.maximum(r, 1e-12)
    return S


def body_cloth(n: int = 8, frames: int = 3, substeps: int = 2, iterations: int = 5, seed: int = 1,
               body_res=(8, 16), center=(0.05, -0.28, -0.03), radius: float = 0.3) -> Scene:
    """Cloth (distance + bending, row-0 corners pinned) falling onto a body
    collider given as a closed triangle mesh (a sphere mesh standing in for a
    body), one body-contact set of every free vertex."""
    sc = small_cloth(n=n, frames=frames, substeps=substeps, iterations=iterations, sphere=False, seed=seed)
    bx, bt = uv_sphere(center, radius, *body_res)
    sc.body_x, sc.body_tris = bx, bt
    sc.body_thickness, sc.body_compliance, sc.body_radius = 0.01, 1e-8, 0.1
    sc.set_type.append(BODY)
    sc.set_items.append(np.nonzero(sc.inv_mass > 0)[0].astype(np.int32))
    sc.name = f"cloth{n}_body"
    return sc


def small_cloth(n: int = 6, frames: int = 3, substeps: int = 2, iterations: int = 5,
                sphere: bool = True, pinned=None, seed: int = 1) -> Scene:
    """Tiny cloth with bending (and a sphere under it) for exact checks."""
    pins = (0, n - 1) if pinned is None else pinned
    sc = cloth_grid(n, n, 1.0 / (n - 1), origin=(-0.5, 0.0, -0.5), pinned=pins,
                    contact=sphere)
    rng = np.random.default_rng(seed)
    sc.dist_alpha = 1e-6 * rng.uniform(0.5, 2.0, sc.n_dist)
    sc.bend_alpha = 1e-3 * rng.uniform(0.5, 2.0, sc.n_bend)
    sc.tet_E = np.zeros(0)
    sc.sphere = (0.05, -0.28, -0.03, 0.3)
    sc.contact_thickness, sc.contact_compliance = 0.005, 1e-7
    sc.v0 = np.zeros_like(sc.rest)
    sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, substeps, iterations, frames
    sc.name = f"cloth{n}_small"
    return sc


def assign_materials(sc: Scene, n_materials: int, seed: int = 7) -> Scene:
    """Material clusters drawn uniformly at random over all tets (Sec. 5.2's
    estimation problem spreads its materials that way).  The scene's tet_E
    becomes per material: the mean over each material's tets (E of an empty
    material: the overall mean)."""
    rng = np.random.default_rng(seed)
    mat = rng.integers(0, n_materials, sc.n_tet).astype(np.int32)
    E = np.asarray(sc.tet_E, np.float64)
    cnt = np.bincount(mat, minlength=n_materials)
    tot = np.bincount(mat, weights=E, minlength=n_materials)
    sc.tet_E = np.where(cnt > 0, tot / np.maximum(cnt, 1), E.mean())
    sc.n_materials, sc.tet_material = int(n_materials), mat
    return sc


def lame_from_E(E, nu):
    """(mu, lambda) of Young's modulus E and Poisson ratio nu."""
    E, nu = np.asarray(E, np.float64), np.asarray(nu, np.float64)
    return E / (2 * (1 + nu)), E * nu / ((1 + nu) * (1 - 2 * nu))


def material_estimation(n: int = 8, n_materials: int = 100, frames: int = 20, substeps: int = 2,
                        iterations: int = 20, size: float = 1.0, E_stiff: float = 5e4, E_soft: float = 5e3,
                        nu: float = 0.3, guess_scale: float = 0.1, seed: int = 7):
    """Inhomogeneous volumetric material estimation (Sec. 5.2): an n^3-cube tet
    box clamped on its x = 0 face sags under gravity.  The target is made of
    two materials (stiff for tet centroids with x < size/2, soft beyond); the
    model has ``n_materials`` materials spread at random over the tets, all
    starting at guess_scale times the stiff target's Lame parameters.  The
    goal compares the boundary-surface vertices at the last frame.

    Returns (model scene, target scene, dict with the target's per-material
    (mu, lambda) of the target scene, the model's initial (mu, lambda), the
    boundary weights [V], the frame mask [F] and a gradient-descent step on
    (a, b) that decreases the goal steadily from this guess)."""
    def box():
        sc = tet_box(n, size=size, pin_bottom=False)
        sc.inv_mass[sc.rest[:, 0] == 0.0] = 0.0
        sc.tet_nu = np.full(sc.n_tet, nu)
        sc.dist_alpha, sc.bend_alpha = np.zeros(0), np.zeros(0)
        sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, substeps, iterations, frames
        return sc
    tgt = box()
    cx = tgt.rest[tgt.tet_v].mean(axis=1)[:, 0]
    tgt.n_materials, tgt.tet_material = 2, (cx >= 0.5 * size).astype(np.int32)
    mu_t, la_t = lame_from_E(np.array([E_stiff, E_soft]), nu)
    tgt.tet_E = np.array([E_stiff, E_soft])
    tgt.name = f"tetbox{n}_two_materials"
    model = box()
    model.tet_E = np.full(model.n_tet, guess_scale * E_stiff)
    assign_materials(model, n_materials, seed)
    model.name = f"tetbox{n}_{n_materials}_materials"
    mu0, la0 = lame_from_E(np.full(n_materials, guess_scale * E_stiff), nu)
    r = model.rest
    edge = np.isclose(r, 0.0) | np.isclose(r, size)
    weight = edge.any(axis=1).astype(np.float64)
    mask = np.zeros(frames, bool)
    mask[-1] = True
    return model, tgt, {"target_mu": mu_t, "target_lambda": la_t, "mu0": mu0, "lambda0": la0,
                        "vertex_weight": weight, "frame_mask": mask, "step": 3000.0}


def small_tets(n: int = 2, frames: int = 3, substeps: int = 2, iterations: int = 5,
               seed: int = 1) -> Scene:
    sc = tet_box(n, size=0.2)
    E, nu = tet_material(seed, sc.n_tet)
    sc.tet_E, sc.tet_nu = E * 0.05, nu
    sc.dist_alpha, sc.bend_alpha = np.zeros(0), np.zeros(0)
    sc.dt, sc.substeps, sc.iterations, sc.n_frames = 1.0 / 60.0, substeps, iterations, frames
    sc.name = f"tetbox{n}_small"
    return sc

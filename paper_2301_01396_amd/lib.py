"""ctypes binding of ``libxpbd.so`` (declared in include/xpbd.h).

Argument marshalling only: every step of the simulation and its adjoint runs
in the library's HIP kernels.  PyTorch provides device memory and the
stream.  Loading fails loudly when the library is not built; there is no
other implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxpbd.so")

XPBD_OK, XPBD_ERR_INVALID, XPBD_ERR_OOM, XPBD_ERR_HIP, XPBD_ERR_STATE, XPBD_ERR_NONFINITE, XPBD_ERR_SOLVER = range(7)
F32, F64 = 0, 1
FWD_FOR_ADJOINT = 1
N_FAMILIES = 14   # kernel families reported by xpbd_profile_read
PACK_GRAPHS = 1
EXPORTS = ("xpbd_create", "xpbd_destroy", "xpbd_forward", "xpbd_adjoint", "xpbd_goal_l2",
           "xpbd_get_info", "xpbd_profile_enable", "xpbd_profile_read", "xpbd_last_error",
           "xpbd_status_string", "xpbd_pack_create", "xpbd_pack_destroy", "xpbd_pack_add", "xpbd_pack_run",
           "xpbd_pack_get_stats", "xpbd_pack_last_error", "xpbd_adjoint_implicit", "xpbd_goal_weighted",
           "xpbd_goal_weighted_noalloc")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_vp = C.c_void_p


class MeshDesc(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("rest_pos", _dp), ("inv_mass", _dp)]


class ConstraintDesc(C.Structure):
    _fields_ = [("n_dist", C.c_int32), ("dist_v", _ip), ("n_bend", C.c_int32), ("bend_v", _ip),
                ("n_tet", C.c_int32), ("tet_v", _ip), ("tet_nu", _dp), ("contact", C.c_int32),
                ("contact_thickness", C.c_double), ("contact_compliance", C.c_double),
                ("n_materials", C.c_int32), ("tet_material", _ip),
                ("n_tri", C.c_int32), ("tri_v", _ip), ("tri_uv", _dp),
                ("n_body_verts", C.c_int32), ("n_body_tris", C.c_int32), ("body_tris", _ip),
                ("body_thickness", C.c_double), ("body_compliance", C.c_double), ("body_radius", C.c_double)]


class ScheduleDesc(C.Structure):
    _fields_ = [("n_sets", C.c_int32), ("set_type", _ip), ("set_offsets", _lp), ("set_items", _ip),
                ("n_groups", C.c_int32), ("group_sets", _ip), ("group_patch", _ip)]


class Options(C.Structure):
    _fields_ = [("dt", C.c_double), ("substeps", C.c_int32), ("iterations", C.c_int32),
                ("gravity", C.c_double * 3), ("dtype", C.c_int32), ("hbm_budget_bytes", C.c_size_t),
                ("tet_gamma_one", C.c_int32), ("tape_mode", C.c_int32), ("launch_mode", C.c_int32),
                ("persistent_blocks", C.c_int32), ("block_size", C.c_int32), ("group_records", C.c_int32),
                ("group_block", C.c_int32), ("record_frames", C.c_int32), ("serial_adjoint", C.c_int32),
                ("record_kind", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("dist_compliance", _vp), ("bend_compliance", _vp), ("tet_E", _vp), ("f_ext", _vp),
                ("sphere", C.c_double * 4), ("tet_mu", _vp), ("tet_lambda", _vp), ("tri_coef", _vp),
                ("body_x", _vp)]


class Grads(C.Structure):
    _fields_ = [("dist_compliance", _vp), ("bend_compliance", _vp), ("tet_E", _vp), ("f_ext", _vp),
                ("x0", _vp), ("v0", _vp), ("sphere", _vp), ("tet_mu", _vp), ("tet_lambda", _vp),
                ("tri_coef", _vp), ("body_x", _vp)]


class Info(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_dist", C.c_int32), ("n_bend", C.c_int32), ("n_tet", C.c_int32),
                ("n_contact", C.c_int32), ("n_sets", C.c_int32), ("projections_per_iteration", C.c_int64),
                ("device_bytes", C.c_int64), ("tape_bytes_per_iteration", C.c_int64),
                ("tape_mode", C.c_int32), ("persistent", C.c_int32), ("persistent_blocks", C.c_int32),
                ("n_groups", C.c_int32), ("n_groups_lds", C.c_int32), ("max_group_lds_bytes", C.c_int32),
                ("n_materials", C.c_int32), ("n_tri", C.c_int32), ("n_body_contacts", C.c_int32),
                ("forward_record_frames", C.c_int32), ("adjoint_streams", C.c_int32)]


class Job(C.Structure):
    _fields_ = [("x0", _vp), ("v0", _vp), ("params", Params), ("n_frames", C.c_int32), ("x_frames", _vp),
                ("x_final", _vp), ("v_final", _vp), ("targets", _vp), ("frame_mask", C.POINTER(C.c_uint8)),
                ("dLdv_final", _vp), ("loss", _vp), ("grads", Grads)]


class PackStats(C.Structure):
    _fields_ = [("active_jobs", C.c_int32), ("rounds", C.c_int64), ("launches", C.c_int64),
                ("graph_launches", C.c_int64), ("graph_captures", C.c_int64), ("last_round_launches", C.c_int32)]


class CG(C.Structure):
    _fields_ = [("max_iterations", C.c_int32), ("rel_tolerance", C.c_double), ("pd_projection", C.c_int32),
                ("total_iterations", C.c_int64),
                ("max_iterations_used", C.c_int32), ("worst_rel_residual", C.c_double)]


class XPBDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"xpbd status {status}: {msg}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Open the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        lib = C.CDLL(LIB_PATH)
        lib.xpbd_create.restype = C.c_int
        lib.xpbd_create.argtypes = [C.POINTER(MeshDesc), C.POINTER(ConstraintDesc), C.POINTER(ScheduleDesc),
                                    C.POINTER(Options), C.POINTER(_vp)]
        lib.xpbd_destroy.restype = C.c_int
        lib.xpbd_destroy.argtypes = [_vp]
        lib.xpbd_forward.restype = C.c_int
        lib.xpbd_forward.argtypes = [_vp, _vp, _vp, C.POINTER(Params), C.c_int32, _vp, _vp, _vp, C.c_int32, _vp]
        lib.xpbd_adjoint.restype = C.c_int
        lib.xpbd_adjoint.argtypes = [_vp, C.POINTER(Params), _vp, C.POINTER(C.c_uint8), _vp,
                                     C.POINTER(Grads), _vp]
        lib.xpbd_goal_l2.restype = C.c_int
        lib.xpbd_goal_l2.argtypes = [_vp, _vp, _vp, C.POINTER(C.c_uint8), C.c_int32, _vp, _vp, _vp]
        lib.xpbd_goal_weighted.restype = C.c_int
        lib.xpbd_goal_weighted.argtypes = [_vp, _vp, _vp, C.POINTER(C.c_uint8), _vp, C.c_int32, _vp, _vp, _vp]
        lib.xpbd_goal_weighted_noalloc.restype = C.c_int
        lib.xpbd_goal_weighted_noalloc.argtypes = [_vp, _vp, _vp, C.POINTER(C.c_uint8), _vp, C.c_int32, _vp, _vp,
                                                   _vp]
        lib.xpbd_get_info.restype = C.c_int
        lib.xpbd_get_info.argtypes = [_vp, C.POINTER(Info)]
        lib.xpbd_profile_enable.restype = C.c_int
        lib.xpbd_profile_enable.argtypes = [_vp, C.c_int32]
        lib.xpbd_profile_read.restype = C.c_int
        lib.xpbd_profile_read.argtypes = [_vp, _lp, _dp, _lp]
        lib.xpbd_last_error.restype = C.c_char_p
        lib.xpbd_last_error.argtypes = [_vp]
        lib.xpbd_status_string.restype = C.c_char_p
        lib.xpbd_status_string.argtypes = [C.c_int]
        lib.xpbd_adjoint_implicit.restype = C.c_int
        lib.xpbd_adjoint_implicit.argtypes = [_vp, C.POINTER(Params), _vp, C.POINTER(C.c_uint8), C.POINTER(CG),
                                              C.POINTER(Grads), _vp]
        lib.xpbd_pack_create.restype = C.c_int
        lib.xpbd_pack_create.argtypes = [C.c_int, C.c_int32, C.c_int32, C.POINTER(_vp)]
        lib.xpbd_pack_destroy.restype = C.c_int
        lib.xpbd_pack_destroy.argtypes = [_vp]
        lib.xpbd_pack_add.restype = C.c_int
        lib.xpbd_pack_add.argtypes = [_vp, _vp, C.POINTER(Job), _vp, _lp]
        lib.xpbd_pack_run.restype = C.c_int
        lib.xpbd_pack_run.argtypes = [_vp, C.c_int32, _vp, _lp, C.c_int32, _ip]
        lib.xpbd_pack_get_stats.restype = C.c_int
        lib.xpbd_pack_get_stats.argtypes = [_vp, C.POINTER(PackStats)]
        lib.xpbd_pack_last_error.restype = C.c_char_p
        lib.xpbd_pack_last_error.argtypes = [_vp]
        _lib = lib
    return _lib


def schedule_groups(scene, use_groups: bool = True):
    """Flatten a scene's LDS groups to (int32 [G*2], int32 [G*V])."""
    groups = getattr(scene, "groups", None) or []
    if not use_groups or not groups:
        return np.zeros(2, np.int32)[:0], np.zeros(1, np.int32)[:0]
    gs = np.asarray([[a, b] for a, b, _ in groups], np.int32).reshape(-1)
    gp = np.ascontiguousarray(np.stack([np.asarray(pm, np.int32) for _, _, pm in groups]).reshape(-1))
    return gs, gp


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_ptr(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Simulator:
    """One problem (mesh, constraints, schedule, options) resident on a GPU."""

    def __init__(self, scene, dtype: torch.dtype = torch.float32, device="cuda:0",
                 hbm_budget_bytes: int = 0, tape_mode: int = 0, tet_gamma_one: bool = False,
                 iterations: Optional[int] = None, substeps: Optional[int] = None, launch_mode: int = 0,
                 persistent_blocks: int = 0, use_groups: bool = True, block_size: int = 0,
                 group_records: int = 0, group_block: int = 0, record_frames: int = 0,
                 serial_adjoint: bool = False, record_kind: int = 0):
        self.lib = load()
        self.scene = scene
        self.dtype = dtype
        self.device = torch.device(device)
        self._ctx = _vp()
        rest = np.ascontiguousarray(scene.rest, np.float64)
        inv_mass = np.ascontiguousarray(scene.inv_mass, np.float64)
        dist_v = np.ascontiguousarray(scene.dist_v, np.int32)
        bend_v = np.ascontiguousarray(scene.bend_v, np.int32)
        tet_v = np.ascontiguousarray(scene.tet_v, np.int32)
        tet_nu = np.ascontiguousarray(scene.tet_nu, np.float64)
        n_mat = int(scene.n_materials or 0)
        tet_mat = (np.ascontiguousarray(scene.tet_material, np.int32) if n_mat else np.zeros(0, np.int32))
        tri_v = np.ascontiguousarray(scene.tri_v, np.int32)
        tri_uv = np.ascontiguousarray(scene.tri_uv, np.float64)
        body_tris = np.ascontiguousarray(scene.body_tris, np.int32)
        st, off, items = scene.schedule_arrays()
        m = MeshDesc(scene.n_verts, rest.ctypes.data_as(_dp), inv_mass.ctypes.data_as(_dp))
        cd = ConstraintDesc(scene.n_dist, dist_v.ctypes.data_as(_ip), scene.n_bend, bend_v.ctypes.data_as(_ip),
                            scene.n_tet, tet_v.ctypes.data_as(_ip), tet_nu.ctypes.data_as(_dp),
                            1 if scene.contact else 0, scene.contact_thickness, scene.contact_compliance,
                            n_mat, tet_mat.ctypes.data_as(_ip), scene.n_tri, tri_v.ctypes.data_as(_ip),
                            tri_uv.ctypes.data_as(_dp), scene.n_body_verts, scene.n_body_tris,
                            body_tris.ctypes.data_as(_ip), scene.body_thickness, scene.body_compliance,
                            scene.body_radius)
        gs, gp = schedule_groups(scene, use_groups)
        sd = ScheduleDesc(len(st), st.ctypes.data_as(_ip), off.ctypes.data_as(_lp), items.ctypes.data_as(_ip),
                          len(gs) // 2, gs.ctypes.data_as(_ip), gp.ctypes.data_as(_ip))
        o = Options()
        o.dt = scene.dt
        o.substeps = scene.substeps if substeps is None else substeps
        o.iterations = scene.iterations if iterations is None else iterations
        for a in range(3):
            o.gravity[a] = scene.gravity[a]
        o.dtype = F64 if dtype == torch.float64 else F32
        o.hbm_budget_bytes = hbm_budget_bytes
        o.tet_gamma_one = 1 if tet_gamma_one else 0
        o.tape_mode = tape_mode
        o.launch_mode = launch_mode
        o.persistent_blocks = persistent_blocks
        o.block_size = block_size
        o.group_records = group_records
        o.group_block = group_block
        o.record_frames = record_frames
        o.record_kind = record_kind
        o.serial_adjoint = 1 if serial_adjoint else 0
        with torch.cuda.device(self.device):
            rc = self.lib.xpbd_create(C.byref(m), C.byref(cd), C.byref(sd), C.byref(o), C.byref(self._ctx))
        if rc != XPBD_OK:
            raise XPBDError(rc, self.lib.xpbd_last_error(None).decode())
        self._fwd_keep = None

    # ------------------------------------------------------------------ helpers
    def _check(self, rc):
        if rc != XPBD_OK:
            raise XPBDError(rc, self.lib.xpbd_last_error(self._ctx).decode())

    def close(self):
        if self._ctx:
            self.lib.xpbd_destroy(self._ctx)
            self._ctx = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tensor(self, a, dtype=None) -> torch.Tensor:
        return torch.as_tensor(np.asarray(a), dtype=dtype or self.dtype, device=self.device).contiguous()

    def _params(self, dist_alpha, bend_alpha, tet_E, f_ext, sphere):
        p = Params()
        p.dist_compliance = _ptr(dist_alpha)
        p.bend_compliance = _ptr(bend_alpha)
        p.tet_E = _ptr(tet_E)
        p.f_ext = _ptr(f_ext)
        sph = self.scene.sphere if sphere is None else sphere
        sph = [float(v) for v in (sph.tolist() if hasattr(sph, "tolist") else sph)]
        for a in range(4):
            p.sphere[a] = sph[a]
        return p

    def _arg(self, t, shape):
        if t is None:
            return None
        if not isinstance(t, torch.Tensor):
            t = self.tensor(t)
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {self.dtype} tensor on {self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    # ------------------------------------------------------------------ API
    def _inputs(self, n_frames, x0, v0, dist_alpha, bend_alpha, tet_E, f_ext, sphere, tet_mu=None,
                tet_lambda=None, tri_coef=None, body_x=None):
        sc = self.scene
        V = sc.n_verts
        x0 = self._arg(sc.x0 if x0 is None else x0, (V, 3))
        v0 = self._arg(sc.v0 if v0 is None else v0, (V, 3))
        da = self._arg(sc.dist_alpha if dist_alpha is None else dist_alpha, (sc.n_dist,)) if sc.n_dist else None
        ba = self._arg(sc.bend_alpha if bend_alpha is None else bend_alpha, (sc.n_bend,)) if sc.n_bend else None
        lame = tet_mu is not None or tet_lambda is not None
        te = None
        if sc.n_tet and not lame:
            te = self._arg(sc.tet_E if tet_E is None else tet_E, (sc.n_tet_params,))
        fe = f_ext if f_ext is not None else sc.f_ext
        fe = self._arg(fe, (n_frames, V, 3)) if fe is not None else None
        p = self._params(da, ba, te, fe, sphere)
        tm = tl = None
        if lame:
            tm = self._arg(tet_mu, (sc.n_tet_params,))
            tl = self._arg(tet_lambda, (sc.n_tet_params,))
            p.tet_mu, p.tet_lambda = _ptr(tm), _ptr(tl)
        tc = None
        if sc.n_tri:
            tc = self._arg(sc.tri_coef if tri_coef is None else tri_coef, (sc.n_tri, 4))
            p.tri_coef = _ptr(tc)
        bxx = None
        if sc.n_body_tris:
            bxx = self._arg(sc.body_x if body_x is None else body_x, (sc.n_body_verts, 3))
            p.body_x = _ptr(bxx)
        self._lame = lame
        return x0, v0, da, ba, te, fe, p, (tm, tl, tc, bxx)

    def _grad_buffers(self, F, want):
        sc = self.scene
        V = sc.n_verts
        lame = getattr(self, "_lame", False)
        want = set(want or ("x0", "v0", "dist_alpha", "bend_alpha", "f_ext", "sphere", "tri_coef", "body_x") +
                   (("tet_mu", "tet_lambda") if lame else ("tet_E",)))
        dev, f64 = self.device, torch.float64
        g = {}
        if "x0" in want:
            g["x0"] = torch.empty((V, 3), dtype=self.dtype, device=dev)
        if "v0" in want:
            g["v0"] = torch.empty((V, 3), dtype=self.dtype, device=dev)
        if "dist_alpha" in want and sc.n_dist:
            g["dist_alpha"] = torch.empty(sc.n_dist, dtype=f64, device=dev)
        if "bend_alpha" in want and sc.n_bend:
            g["bend_alpha"] = torch.empty(sc.n_bend, dtype=f64, device=dev)
        if "tet_E" in want and sc.n_tet:
            g["tet_E"] = torch.empty(sc.n_tet_params, dtype=f64, device=dev)
        if "f_ext" in want:
            g["f_ext"] = torch.empty((F, V, 3), dtype=self.dtype, device=dev)
        if "sphere" in want:
            g["sphere"] = torch.empty(4, dtype=f64, device=dev)
        for k in ("tet_mu", "tet_lambda"):
            if k in want and sc.n_tet and lame:
                g[k] = torch.empty(sc.n_tet_params, dtype=f64, device=dev)
        if not lame:
            g.pop("tet_mu", None)
            g.pop("tet_lambda", None)
        else:
            g.pop("tet_E", None)
        if "tri_coef" in want and sc.n_tri:
            g["tri_coef"] = torch.empty((sc.n_tri, 4), dtype=f64, device=dev)
        if "body_x" in want and sc.n_body_tris:
            g["body_x"] = torch.empty((sc.n_body_verts, 3), dtype=f64, device=dev)
        gr = Grads(*(_ptr(g.get(k)) for k in ("dist_alpha", "bend_alpha", "tet_E", "f_ext", "x0", "v0",
                                              "sphere", "tet_mu", "tet_lambda", "tri_coef", "body_x")))
        return g, gr

    def forward(self, n_frames: int, x0=None, v0=None, dist_alpha=None, bend_alpha=None, tet_E=None,
                f_ext=None, sphere=None, frames: bool = True, x_frames_out=None, for_adjoint: bool = False,
                tet_mu=None, tet_lambda=None, tri_coef=None, body_x=None):
        """Roll out; returns (x_frames or None, x_final, v_final) on the device.

        ``for_adjoint``: an adjoint will follow; the library may keep the record
        of every projection now so the adjoint needs no recomputation."""
        sc = self.scene
        V = sc.n_verts
        x0, v0, da, ba, te, fe, p, lm = self._inputs(n_frames, x0, v0, dist_alpha, bend_alpha, tet_E, f_ext, sphere,
                                                     tet_mu, tet_lambda, tri_coef, body_x)
        xf = None
        if frames:
            xf = x_frames_out if x_frames_out is not None else torch.empty((n_frames, V, 3), dtype=self.dtype,
                                                                           device=self.device)
        xe = torch.empty((V, 3), dtype=self.dtype, device=self.device)
        ve = torch.empty((V, 3), dtype=self.dtype, device=self.device)
        rc = self.lib.xpbd_forward(self._ctx, _ptr(x0), _ptr(v0), C.byref(p), n_frames, _ptr(xf), _ptr(xe),
                                   _ptr(ve), FWD_FOR_ADJOINT if for_adjoint else 0, _stream_ptr(self.device))
        self._check(rc)
        self._fwd_keep = (p, x0, v0, da, ba, te, fe, n_frames, lm)
        self.forward_count = getattr(self, "forward_count", 0) + 1
        return xf, xe, ve

    def adjoint(self, dLdx_frames=None, frame_mask=None, dLdv_final=None, want=None) -> Dict[str, torch.Tensor]:
        """Exact adjoint of the last forward; returns a dict of gradients."""
        if self._fwd_keep is None:
            raise XPBDError(XPBD_ERR_STATE, "adjoint without forward")
        p, x0, v0, da, ba, te, fe, F, _lm = self._fwd_keep
        sc = self.scene
        V = sc.n_verts
        g, gr = self._grad_buffers(F, want)
        dl = self._arg(dLdx_frames, (F, V, 3)) if dLdx_frames is not None else None
        dv = self._arg(dLdv_final, (V, 3)) if dLdv_final is not None else None
        mask_arr = None
        mask_ptr = None
        if frame_mask is not None:
            mask_arr = np.ascontiguousarray(np.asarray(frame_mask, dtype=np.uint8))
            if mask_arr.shape != (F,):
                raise ValueError("frame_mask must have one entry per frame")
            mask_ptr = mask_arr.ctypes.data_as(C.POINTER(C.c_uint8))
        rc = self.lib.xpbd_adjoint(self._ctx, C.byref(p), _ptr(dl), mask_ptr, _ptr(dv), C.byref(gr),
                                   _stream_ptr(self.device))
        self._check(rc)
        return g

    def adjoint_implicit(self, dLdx_frames, frame_mask=None, max_iterations: int = 1000,
                         rel_tolerance: float = 1e-10, pd_projection: bool = False, want=None):
        """Implicit adjoint of the last forward (the paper's converged-step
        form, solved by CG): returns (gradients, CG report)."""
        if self._fwd_keep is None:
            raise XPBDError(XPBD_ERR_STATE, "adjoint without forward")
        p, x0, v0, da, ba, te, fe, F, _lm = self._fwd_keep
        V = self.scene.n_verts
        g, gr = self._grad_buffers(F, want or ("x0", "v0", "dist_alpha", "bend_alpha", "f_ext"))
        gr.tri_coef = None
        gr.body_x = None
        g.pop("tri_coef", None)
        g.pop("body_x", None)
        gr.tet_E = None
        gr.sphere = None
        g.pop("tet_E", None)
        g.pop("sphere", None)
        dl = self._arg(dLdx_frames, (F, V, 3))
        cg = CG(max_iterations, rel_tolerance, 1 if pd_projection else 0, 0, 0, 0.0)
        mask_ptr = None
        mask_arr = None
        if frame_mask is not None:
            mask_arr = np.ascontiguousarray(np.asarray(frame_mask, dtype=np.uint8))
            mask_ptr = mask_arr.ctypes.data_as(C.POINTER(C.c_uint8))
        rc = self.lib.xpbd_adjoint_implicit(self._ctx, C.byref(p), _ptr(dl), mask_ptr, C.byref(cg), C.byref(gr),
                                            _stream_ptr(self.device))
        self._check(rc)
        return g, {"total_iterations": cg.total_iterations, "max_iterations_used": cg.max_iterations_used,
                   "worst_rel_residual": cg.worst_rel_residual}

    def goal_l2(self, x_frames: torch.Tensor, targets: torch.Tensor, frame_mask=None, vertex_weight=None):
        """FP64 goal 1/2 sum_{masked f} |W (x(f) - x*(f))|^2 and its gradient;
        W = I, or diag(vertex_weight) (FP64 [V] on the device)."""
        F = x_frames.shape[0]
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        dL = torch.empty_like(x_frames)
        mask_arr = None if frame_mask is None else np.ascontiguousarray(np.asarray(frame_mask, np.uint8))
        mp = None if mask_arr is None else mask_arr.ctypes.data_as(C.POINTER(C.c_uint8))
        if vertex_weight is not None:
            vw = vertex_weight
            if (not isinstance(vw, torch.Tensor) or vw.dtype != torch.float64 or vw.device != self.device
                    or tuple(vw.shape) != (self.scene.n_verts,) or not vw.is_contiguous()):
                raise ValueError("vertex_weight must be a contiguous float64 tensor [V] on the device")
            rc = self.lib.xpbd_goal_weighted(self._ctx, _ptr(x_frames), _ptr(targets), mp, _ptr(vw), F,
                                             _ptr(loss), _ptr(dL), _stream_ptr(self.device))
        else:
            rc = self.lib.xpbd_goal_l2(self._ctx, _ptr(x_frames), _ptr(targets), mp, F, _ptr(loss), _ptr(dL),
                                       _stream_ptr(self.device))
        self._check(rc)
        return loss, dL

    def goal_noalloc(self, x_frames: torch.Tensor, targets: torch.Tensor, loss: torch.Tensor, dLdx=None,
                     frame_mask=None, vertex_weight=None, n_frames=None):
        """The goal of goal_l2 through the entry point that allocates no device
        memory: the caller passes the outputs (loss: float64 scalar on the
        device; dLdx: like x_frames, or None).  n_frames overrides the frame
        count given to the library (default: x_frames.shape[0])."""
        F = x_frames.shape[0] if n_frames is None else int(n_frames)
        mask_arr = None if frame_mask is None else np.ascontiguousarray(np.asarray(frame_mask, np.uint8))
        mp = None if mask_arr is None else mask_arr.ctypes.data_as(C.POINTER(C.c_uint8))
        rc = self.lib.xpbd_goal_weighted_noalloc(self._ctx, _ptr(x_frames), _ptr(targets), mp,
                                                 None if vertex_weight is None else _ptr(vertex_weight), F,
                                                 _ptr(loss), None if dLdx is None else _ptr(dLdx),
                                                 _stream_ptr(self.device))
        self._check(rc)

    def info(self) -> Dict[str, int]:
        i = Info()
        self._check(self.lib.xpbd_get_info(self._ctx, C.byref(i)))
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def profile_enable(self, stride: int = 1):
        self._check(self.lib.xpbd_profile_enable(self._ctx, stride))

    def profile_read(self):
        """Per kernel family (2*type fwd, 2*type+1 reverse, 8/9 persistent
        forward/reverse frames): timed launches, ms, projections."""
        la = (C.c_int64 * N_FAMILIES)()
        ms = (C.c_double * N_FAMILIES)()
        it = (C.c_int64 * N_FAMILIES)()
        self._check(self.lib.xpbd_profile_read(self._ctx, la, ms, it))
        return list(la), list(ms), list(it)


class PackJob:
    """One job of a Pack: its simulator, its output tensors on the device
    (``x_frames``, ``x_final``, ``v_final``, ``loss``, ``grads``) and the
    inputs the device still reads (kept alive until the job is done)."""

    def __init__(self, sim, n_frames, keep, outputs):
        self.sim = sim
        self.n_frames = n_frames
        self._keep = keep
        self.x_frames, self.x_final, self.v_final, self.loss, self.grads = outputs
        self.id = 0
        self.tag = None


class Pack:
    """Jobs on many simulators advanced together, one frame per round, each
    launch serving the same step of every job (xpbd_pack_* in xpbd.h)."""

    def __init__(self, dtype: torch.dtype = torch.float32, device="cuda:0", graphs: bool = False,
                 block_size: int = 0):
        """block_size: workgroup size of the pack's launches (64, 128, 256;
        0 = 256), a performance choice that never changes results."""
        self.lib = load()
        self.dtype = dtype
        self.device = torch.device(device)
        self.block_size = block_size
        self._pk = _vp()
        rc = self.lib.xpbd_pack_create(F64 if dtype == torch.float64 else F32, PACK_GRAPHS if graphs else 0,
                                       int(block_size), C.byref(self._pk))
        if rc != XPBD_OK:
            raise XPBDError(rc, "pack create failed")
        self.jobs: Dict[int, PackJob] = {}

    def _check(self, rc):
        if rc != XPBD_OK:
            raise XPBDError(rc, self.lib.xpbd_pack_last_error(self._pk).decode())

    def add(self, sim: Simulator, n_frames: int, x0=None, v0=None, dist_alpha=None, bend_alpha=None, tet_E=None,
            f_ext=None, sphere=None, targets=None, frame_mask=None, dLdv_final=None, want=None,
            frames: bool = True, tag=None) -> PackJob:
        """Queue a rollout of ``n_frames`` frames and, with ``targets`` ([F, V, 3]),
        the goal and its adjoint.  Returns the job; its tensors are complete
        once ``run`` has reported it done and the stream has reached that point."""
        if sim.dtype != self.dtype or sim.device != self.device:
            raise ValueError("simulator dtype / device differ from the pack's")
        V = sim.scene.n_verts
        x0, v0, da, ba, te, fe, p, lm = sim._inputs(n_frames, x0, v0, dist_alpha, bend_alpha, tet_E, f_ext, sphere)
        adj = targets is not None
        xf = torch.empty((n_frames, V, 3), dtype=self.dtype, device=self.device) if (frames or adj) else None
        xe = torch.empty((V, 3), dtype=self.dtype, device=self.device)
        ve = torch.empty((V, 3), dtype=self.dtype, device=self.device)
        tg = sim._arg(targets, (n_frames, V, 3)) if adj else None
        dv = sim._arg(dLdv_final, (V, 3)) if dLdv_final is not None else None
        loss = torch.zeros((), dtype=torch.float64, device=self.device) if adj else None
        g, gr = sim._grad_buffers(n_frames, want) if adj else ({}, Grads())
        mask_arr = None
        j = Job()
        j.x0, j.v0, j.params, j.n_frames = _ptr(x0), _ptr(v0), p, n_frames
        j.x_frames, j.x_final, j.v_final = _ptr(xf), _ptr(xe), _ptr(ve)
        j.targets, j.dLdv_final, j.loss, j.grads = _ptr(tg), _ptr(dv), _ptr(loss), gr
        if frame_mask is not None:
            mask_arr = np.ascontiguousarray(np.asarray(frame_mask, dtype=np.uint8))
            if mask_arr.shape != (n_frames,):
                raise ValueError("frame_mask must have one entry per frame")
            j.frame_mask = mask_arr.ctypes.data_as(C.POINTER(C.c_uint8))
        jid = C.c_int64(0)
        self._check(self.lib.xpbd_pack_add(self._pk, sim._ctx, C.byref(j), _stream_ptr(self.device), C.byref(jid)))
        job = PackJob(sim, n_frames, (x0, v0, da, ba, te, fe, tg, dv, j), (xf, xe, ve, loss, g))
        job.id = jid.value
        job.tag = tag
        self.jobs[job.id] = job
        return job

    def run(self, max_rounds: int = 1 << 30):
        """Run rounds until one finishes a job (or max_rounds); returns the
        finished jobs (stream-ordered: synchronise before reading them)."""
        cap = max(1, len(self.jobs))
        ids = (C.c_int64 * cap)()
        n = C.c_int32(0)
        self._check(self.lib.xpbd_pack_run(self._pk, max_rounds, _stream_ptr(self.device), ids, cap, C.byref(n)))
        return [self.jobs.pop(ids[i]) for i in range(n.value)]

    def run_all(self):
        """Run until every queued job is done; returns them in completion order."""
        out = []
        while self.jobs:
            got = self.run()
            if not got and self.stats()["active_jobs"] == 0:
                break
            out.extend(got)
        return out

    def stats(self) -> Dict[str, int]:
        s = PackStats()
        self._check(self.lib.xpbd_pack_get_stats(self._pk, C.byref(s)))
        return {k: getattr(s, k) for k, _ in PackStats._fields_}

    def close(self):
        if self._pk:
            self.lib.xpbd_pack_destroy(self._pk)
            self._pk = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

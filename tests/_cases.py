"""Shared helpers for GPU-versus-reference comparisons (test support only)."""
import dataclasses

import numpy as np
import pytest

import oracle as O


def needs_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    if nb == 0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def f32(a):
    """The FP32 value of every element, held in FP64."""
    return None if a is None else np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def rounded_scene(sc):
    """The scene with every input the FP32 GPU path receives as an FP32 array
    (initial state, compliances, moduli, forces, membrane coefficients, body
    positions) rounded to FP32, so the FP64 reference computes the exact
    result for the inputs the GPU actually gets.  Rest shape, inverse masses
    and the sphere stay FP64: the library takes them in FP64."""
    r = dataclasses.replace(sc)
    for k in ("x0", "v0", "dist_alpha", "bend_alpha", "tet_E", "f_ext", "tri_coef", "body_x"):
        setattr(r, k, f32(getattr(sc, k)))
    return r


def split_sets(sc, total):
    """Split the largest sets of sc's schedule in two until it has `total`
    sets.  The items of a set share no vertex, so projecting a set's halves
    one after the other computes exactly what projecting the set does: the
    schedule is the same computation with more, smaller sets."""
    st, si = list(sc.set_type), [np.asarray(x) for x in sc.set_items]
    while len(st) < total:
        k = max(range(len(si)), key=lambda j: len(si[j]))
        h = len(si[k]) // 2
        st.insert(k + 1, st[k])
        si[k:k + 1] = [si[k][:h], si[k][h:]]
    sc.set_type, sc.set_items = st, si
    return sc


def reference_case(sc, F, mask=None, seed=0, noise=0.01, f_ext=None, emulate_f32=False, n_threads=4,
                   round_inputs=False, targets=None):
    """Forward, targets, goal gradient and exact adjoint from the reference.
    round_inputs: run it on rounded_scene(sc) (and FP32 forces and targets),
    the exact answer for the FP32 inputs the GPU receives."""
    if round_inputs:
        sc, f_ext = rounded_scene(sc), f32(f_ext)
    osc = O.OracleScene(sc, emulate_f32=emulate_f32, n_threads=n_threads)
    kw = {} if f_ext is None else {"f_ext": f_ext}
    xf, xe, ve = O.forward(osc, F, **kw)
    if targets is None:
        rng = np.random.default_rng(seed)
        targets = xf + noise * rng.standard_normal(xf.shape)
        if round_inputs:
            targets = f32(targets)
    if mask is None:
        mask = np.ones(F, bool)
    L, dL = O.goal_l2(xf, targets, mask)
    g = O.adjoint(osc, F, dL, **kw)
    return {"x_frames": xf, "x_final": xe, "v_final": ve, "targets": targets, "mask": mask, "loss": L,
            "dL": dL, "grads": g}


def gpu_case(sim, F, ref, f_ext=None, for_adjoint=True):
    """Same rollout, goal and adjoint through the C ABI."""
    import torch
    fe = None if f_ext is None else sim.tensor(f_ext)
    xf, xe, ve = sim.forward(F, f_ext=fe, for_adjoint=for_adjoint)
    loss, dL = sim.goal_l2(xf, sim.tensor(ref["targets"]), ref["mask"])
    g = sim.adjoint(dL, ref["mask"])
    torch.cuda.synchronize()
    out = {"x_frames": xf.double().cpu().numpy(), "x_final": xe.double().cpu().numpy(),
           "v_final": ve.double().cpu().numpy(), "loss": float(loss.cpu()), "grads": {}}
    for k, v in g.items():
        out["grads"][k] = v.double().cpu().numpy()
    return out


GROUPS = ("x0", "v0", "dist_alpha", "bend_alpha", "tet_E", "f_ext", "sphere", "tri_coef", "body_x")


def max_err(a, b):
    """Largest element error over the largest reference element: a bound that
    a few wrong entries among millions cannot hide in a norm."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    d = float(np.max(np.abs(a - b))) if b.size else 0.0
    return d / mb if mb > 0 else d


def compare(sc, ref, got, pos_tol, grad_tol, groups=GROUPS, report=None, pos_max_tol=None, grad_max_tol=None):
    """Relative L2 per output group within pos_tol / grad_tol, and each
    group's largest element error against its largest reference element
    within pos_max_tol / grad_max_tol (default: the same tolerances).  A
    group the reference has and the GPU output lacks is a failure."""
    pos_max_tol = pos_tol if pos_max_tol is None else pos_max_tol
    grad_max_tol = grad_tol if grad_max_tol is None else grad_max_tol
    errs = {"x_frames": rel(got["x_frames"], ref["x_frames"]), "v_final": rel(got["v_final"], ref["v_final"]),
            "loss": abs(got["loss"] - ref["loss"]) / max(abs(ref["loss"]), 1e-300),
            "x_frames_max": max_err(got["x_frames"], ref["x_frames"])}
    for k in groups:
        if k not in ref["grads"]:
            continue
        r = ref["grads"][k]
        if r.size == 0 or np.linalg.norm(r) == 0:
            continue
        assert k in got["grads"], ("gradient group missing from the GPU output", k)
        errs[k] = rel(got["grads"][k], r)
        errs[k + "_max"] = max_err(got["grads"][k], r)
    if report is not None:
        report.update(errs)
    print("parity", getattr(sc, "name", ""), {k: float("%.3g" % v) for k, v in errs.items()}, flush=True)
    assert errs["x_frames"] <= pos_tol, errs
    assert errs["x_frames_max"] <= pos_max_tol, errs
    for k in groups:
        if k in errs:
            assert errs[k] <= grad_tol, (k, errs)
            assert errs[k + "_max"] <= grad_max_tol, (k + "_max", errs)
    return errs

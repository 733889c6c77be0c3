"""Material estimation (Sec. 5.2): 100 random material clusters on a clamped
tet box, fixed-step gradient descent on (a, b) with mu = a^2, lambda = b^2.
The GPU descent follows the reference's descent iterate by iterate, and the
goal falls."""
import numpy as np
import pytest

import oracle as O
from paper_2301_01396_amd import scenes
from tests._cases import needs_gpu, rel


def _reference_descent(model, F, xt, d, iters):
    om = O.OracleScene(model, n_threads=4)
    a, b = np.sqrt(d["mu0"]), np.sqrt(d["lambda0"])
    out = []
    for _ in range(iters):
        xf, _, _ = O.forward(om, F, tet_mu=a * a, tet_lambda=b * b)
        L, dL = O.goal_l2(xf, xt, d["frame_mask"], d["vertex_weight"])
        g = O.adjoint(om, F, dL, tet_mu=a * a, tet_lambda=b * b)
        out.append((L, a.copy(), b.copy()))
        a = a - d["step"] * 2 * a * g["tet_mu"]
        b = b - d["step"] * 2 * b * g["tet_lambda"]
    out.append((None, a, b))
    return out


def test_scene_and_reference_descent_decreases_goal():
    F = 6
    model, tgt, d = scenes.material_estimation(n=3, frames=F, iterations=10)
    assert model.n_materials == 100 and model.tet_material.max() < 100
    assert tgt.n_materials == 2 and set(np.unique(tgt.tet_material)) == {0, 1}
    assert d["vertex_weight"].sum() == 4 ** 3 - 2 ** 3            # boundary of a 4^3 vertex grid
    xt, _, _ = O.forward(O.OracleScene(tgt, n_threads=4), F, tet_mu=d["target_mu"], tet_lambda=d["target_lambda"])
    hist = _reference_descent(model, F, xt, d, 4)
    losses = [h[0] for h in hist[:-1]]
    assert all(l1 < l0 for l0, l1 in zip(losses, losses[1:])), losses


@pytest.mark.gpu
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gpu_descent_follows_reference(dtype):
    import torch
    from paper_2301_01396_amd.estimate import estimate_materials
    from paper_2301_01396_amd.lib import Simulator
    needs_gpu()
    F, iters = 10, 6
    model, tgt, d = scenes.material_estimation(n=4, frames=F)
    xt, _, _ = O.forward(O.OracleScene(tgt, n_threads=4), F, tet_mu=d["target_mu"], tet_lambda=d["target_lambda"])
    ref = _reference_descent(model, F, xt, d, iters)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sim = Simulator(model, dtype=tdt)
    w = torch.as_tensor(d["vertex_weight"], dtype=torch.float64, device="cuda")
    a, b, losses, step = estimate_materials(sim, F, sim.tensor(xt), d["mu0"], d["lambda0"], d["step"], iters,
                                            d["frame_mask"], w)
    assert step == d["step"]
    torch.cuda.synchronize()
    ref_losses = np.array([h[0] for h in ref[:-1]])
    assert all(l1 < l0 for l0, l1 in zip(losses, losses[1:])), losses
    tol_l, tol_p = (1e-9, 1e-9) if dtype == "f64" else (1e-3, 1e-3)
    assert np.max(np.abs(np.array(losses) - ref_losses) / ref_losses) <= tol_l, (losses, ref_losses)
    assert rel(a.cpu().numpy(), ref[-1][1]) <= tol_p
    assert rel(b.cpu().numpy(), ref[-1][2]) <= tol_p

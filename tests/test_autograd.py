"""The torch.autograd binding: a rollout plus the FP64 goal, differentiated by
loss.backward(), gives the reference's gradients; the tet inputs may be Young's
moduli or Lame parameters; a second forward before backward is refused."""
import numpy as np
import pytest

import oracle as O
from paper_2301_01396_amd import scenes
from tests._cases import needs_gpu, reference_case, rel

pytestmark = pytest.mark.gpu


def _leaf(sim, a):
    t = sim.tensor(a)
    t.requires_grad_(True)
    return t


def test_rollout_backward_matches_reference_cloth():
    import torch
    from paper_2301_01396_amd.autograd import goal_l2, rollout
    from paper_2301_01396_amd.lib import Simulator
    needs_gpu()
    sc = scenes.small_cloth(n=6, frames=3, substeps=2, iterations=5)
    rng = np.random.default_rng(3)
    f = 0.3 * rng.standard_normal((3, sc.n_verts, 3))
    mask = np.array([0, 1, 1], bool)
    ref = reference_case(sc, 3, mask=mask, f_ext=f)
    sim = Simulator(sc, dtype=torch.float64)
    x0, v0 = _leaf(sim, sc.x0), _leaf(sim, sc.v0)
    da, ba, fe = _leaf(sim, sc.dist_alpha), _leaf(sim, sc.bend_alpha), _leaf(sim, f)
    sph = torch.tensor(np.asarray(sc.sphere, np.float64), requires_grad=True)
    xf = rollout(sim, 3, x0, v0, da, ba, None, fe, sph)
    loss = goal_l2(sim, xf, sim.tensor(ref["targets"]), mask)
    loss.backward()
    torch.cuda.synchronize()
    assert abs(float(loss.detach()) - ref["loss"]) <= 1e-9 * abs(ref["loss"])
    g = ref["grads"]
    for name, t in (("x0", x0), ("v0", v0), ("dist_alpha", da), ("bend_alpha", ba), ("f_ext", fe),
                    ("sphere", sph)):
        assert t.grad is not None, name
        assert rel(t.grad.detach().double().cpu().numpy(), g[name]) <= 1e-8, name


def test_rollout_backward_lame_parameters():
    import torch
    from paper_2301_01396_amd.autograd import goal_l2, rollout
    from paper_2301_01396_amd.lib import Simulator
    needs_gpu()
    sc = scenes.small_tets(n=2, frames=3, substeps=2, iterations=4)
    rng = np.random.default_rng(5)
    E, nu = sc.tet_E, sc.tet_nu
    mu = E / (2 * (1 + nu)) * np.exp(0.2 * rng.standard_normal(sc.n_tet))
    la = E * nu / ((1 + nu) * (1 - 2 * nu)) * np.exp(0.2 * rng.standard_normal(sc.n_tet))
    osc = O.OracleScene(sc, n_threads=2)
    xr, _, _ = O.forward(osc, 3, tet_mu=mu, tet_lambda=la)
    tgt = xr + 1e-3 * rng.standard_normal(xr.shape)
    L, dL = O.goal_l2(xr, tgt, np.ones(3, bool))
    gr = O.adjoint(osc, 3, dL, tet_mu=mu, tet_lambda=la)
    sim = Simulator(sc, dtype=torch.float64)
    tm, tl = _leaf(sim, mu), _leaf(sim, la)
    xf = rollout(sim, 3, sim.tensor(sc.x0), sim.tensor(sc.v0), tet_mu=tm, tet_lambda=tl)
    loss = goal_l2(sim, xf, sim.tensor(tgt))
    loss.backward()
    torch.cuda.synchronize()
    assert rel(xf.detach().cpu().numpy(), xr) <= 1e-10
    assert rel(tm.grad.cpu().numpy(), gr["tet_mu"]) <= 1e-8
    assert rel(tl.grad.cpu().numpy(), gr["tet_lambda"]) <= 1e-8


def test_backward_after_another_forward_is_refused():
    import torch
    from paper_2301_01396_amd.autograd import goal_l2, rollout
    from paper_2301_01396_amd.lib import Simulator, XPBDError
    needs_gpu()
    sc = scenes.small_cloth(n=5, frames=2, substeps=1, iterations=3)
    sim = Simulator(sc, dtype=torch.float32)
    x0 = _leaf(sim, sc.x0)
    xf = rollout(sim, 2, x0, sim.tensor(sc.v0))
    loss = goal_l2(sim, xf, sim.tensor(np.zeros((2, sc.n_verts, 3))))
    sim.forward(2)
    with pytest.raises(XPBDError):
        loss.backward()

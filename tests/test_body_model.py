"""Synthetic articulated body (shape modes + linear blend skinning) and the
chain of Sec. 5.3 from the rollout's body-vertex gradient to shape and pose
parameters."""
import numpy as np
import pytest

import oracle as O
from paper_2301_01396_amd import scenes
from paper_2301_01396_amd.body_model import rodrigues, sphere_body
from tests._cases import needs_gpu, rel


def test_rodrigues_is_a_rotation_and_matches_the_exponential_map():
    import torch
    from scipy.linalg import expm
    rng = np.random.default_rng(3)
    tau = torch.as_tensor(rng.standard_normal((5, 3)))
    R = rodrigues(tau).numpy()
    for k in range(5):
        t = tau[k].numpy()
        K = np.array([[0, -t[2], t[1]], [t[2], 0, -t[0]], [-t[1], t[0], 0]])
        np.testing.assert_allclose(R[k], expm(K), atol=1e-12)
        np.testing.assert_allclose(R[k] @ R[k].T, np.eye(3), atol=1e-12)
    np.testing.assert_allclose(rodrigues(torch.zeros(2, 3, dtype=torch.float64)).numpy(), np.eye(3)[None].repeat(2, 0),
                               atol=0)


def test_body_model_identity_shape_and_rigid_pose():
    import torch
    body, T = sphere_body()
    z = torch.zeros(body.n_shape, dtype=torch.float64)
    x = body(z, torch.zeros(body.n_joints, 3, dtype=torch.float64)).numpy()
    np.testing.assert_allclose(x, body.rest.numpy(), atol=1e-15)
    # the same rotation at every joint about a common point is a rigid motion:
    # distances between body vertices are kept
    tau = torch.as_tensor(np.array([[0.0, 0.4, 0.1]] * body.n_joints))
    body.joints[:] = body.joints[0]
    y = body(z, tau).numpy()
    d0 = np.linalg.norm(x[:, None] - x[None], axis=-1)
    d1 = np.linalg.norm(y[:, None] - y[None], axis=-1)
    np.testing.assert_allclose(d1, d0, atol=1e-12)


@pytest.mark.gpu
def test_shape_and_pose_gradients_through_the_collider():
    """Cloth falling on the articulated body: loss.backward() through the
    rollout (library) and the body model (torch) gives dL/dalpha and dL/dtau
    equal to central differences of the reference rollout."""
    import torch
    from paper_2301_01396_amd.autograd import goal_l2, rollout
    from paper_2301_01396_amd.lib import Simulator
    needs_gpu()
    body, _ = sphere_body()
    sc = scenes.body_cloth(n=9, frames=3, substeps=2, iterations=5)
    F = 3
    rng = np.random.default_rng(13)
    alpha0 = 0.05 * rng.standard_normal(body.n_shape)
    tau0 = 0.1 * rng.standard_normal((body.n_joints, 3))
    xb0 = body(torch.as_tensor(alpha0), torch.as_tensor(tau0)).numpy()
    osc = O.OracleScene(sc, n_threads=4)
    xr, _, _ = O.forward(osc, F, body_x=xb0)
    tgt = xr + 0.01 * rng.standard_normal(xr.shape)
    mask = np.array([0, 1, 1], bool)

    def ref_loss(alpha, tau):
        xb = body(torch.as_tensor(alpha), torch.as_tensor(tau)).numpy()
        x, _, _ = O.forward(osc, F, body_x=xb)
        return O.goal_l2(x, tgt, mask)[0]

    sim = Simulator(sc, dtype=torch.float64)
    alpha = torch.as_tensor(alpha0, device="cuda").requires_grad_(True)
    tau = torch.as_tensor(tau0, device="cuda").requires_grad_(True)
    xb = body(alpha, tau)
    xf = rollout(sim, F, sim.tensor(sc.x0), sim.tensor(sc.v0), body_x=xb)
    loss = goal_l2(sim, xf, sim.tensor(tgt), mask)
    loss.backward()
    torch.cuda.synchronize()
    assert abs(float(loss.detach()) - ref_loss(alpha0, tau0)) <= 1e-9 * float(loss.detach())
    eps = 1e-6
    ga = alpha.grad.cpu().numpy()
    for k in range(body.n_shape):
        d = np.zeros(body.n_shape)
        d[k] = eps
        fd = (ref_loss(alpha0 + d, tau0) - ref_loss(alpha0 - d, tau0)) / (2 * eps)
        assert abs(fd - ga[k]) <= 1e-5 * abs(fd) + 1e-11, (k, fd, ga[k])
    gt = tau.grad.cpu().numpy()
    for j in range(body.n_joints):
        for a in range(3):
            d = np.zeros((body.n_joints, 3))
            d[j, a] = eps
            fd = (ref_loss(alpha0, tau0 + d) - ref_loss(alpha0, tau0 - d)) / (2 * eps)
            assert abs(fd - gt[j, a]) <= 1e-5 * abs(fd) + 1e-11, (j, a, fd, gt[j, a])

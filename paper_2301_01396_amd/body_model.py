"""A synthetic articulated body standing in for a statistical body model
(Sec. 5.3 optimises SMPL's shape coefficients and joint angles through the
cloth-body collisions; SMPL is not available here).

The body's vertex positions are
    x(alpha, tau) = sum_j W[v, j] (R(tau_j) (s_v - c_j) + c_j),
    s_v = x0_v + sum_k alpha_k S_k[v]
with linear shape modes S_k (the blend shapes) and linear blend skinning
over joints c_j, rotations R(tau_j) given as axis-angle vectors (Rodrigues'
formula).  It is written with torch operations so the rollout's gradient
with respect to the body vertices (the library's dL/dx_body) flows on to
alpha and tau by the chain rule of Sec. 5.3.
"""
from __future__ import annotations

import numpy as np
import torch


def rodrigues(tau: torch.Tensor) -> torch.Tensor:
    """Rotation matrices (J, 3, 3) of axis-angle vectors tau (J, 3); smooth
    at tau = 0 (Taylor terms below a small angle)."""
    th2 = (tau * tau).sum(-1, keepdim=True)[..., None]          # (J, 1, 1)
    th = torch.sqrt(th2 + 1e-300)
    small = th2 < 1e-12
    a = torch.where(small, 1.0 - th2 / 6.0, torch.sin(th) / th)
    b = torch.where(small, 0.5 - th2 / 24.0, (1.0 - torch.cos(th)) / (th2 + 1e-300))
    z = torch.zeros_like(tau[..., 0])
    K = torch.stack([torch.stack([z, -tau[..., 2], tau[..., 1]], -1),
                     torch.stack([tau[..., 2], z, -tau[..., 0]], -1),
                     torch.stack([-tau[..., 1], tau[..., 0], z], -1)], -2)
    eye = torch.eye(3, dtype=tau.dtype, device=tau.device).expand_as(K)
    return eye + a * K + b * (K @ K)


class SyntheticBody:
    """x(alpha, tau) of the module docstring; arrays are float64."""

    def __init__(self, rest, modes, joints, weights):
        self.rest = torch.as_tensor(np.asarray(rest, np.float64))
        self.modes = torch.as_tensor(np.asarray(modes, np.float64))        # (K, V, 3)
        self.joints = torch.as_tensor(np.asarray(joints, np.float64))      # (J, 3)
        self.weights = torch.as_tensor(np.asarray(weights, np.float64))    # (V, J), rows sum to 1

    @property
    def n_shape(self) -> int:
        return int(self.modes.shape[0])

    @property
    def n_joints(self) -> int:
        return int(self.joints.shape[0])

    def __call__(self, alpha: torch.Tensor, tau: torch.Tensor) -> torch.Tensor:
        dev = alpha.device
        s = self.rest.to(dev) + torch.einsum("k,kvd->vd", alpha, self.modes.to(dev))
        R = rodrigues(tau)                                                   # (J, 3, 3)
        c = self.joints.to(dev)
        per_joint = torch.einsum("jab,jvb->jva", R, s[None] - c[:, None]) + c[:, None]
        return torch.einsum("vj,jva->va", self.weights.to(dev), per_joint)


def sphere_body(center=(0.05, -0.28, -0.03), radius: float = 0.3, res=(8, 16)):
    """The sphere mesh of scenes.uv_sphere as an articulated body: shape
    modes of scenes.body_shape_modes, two joints (the centre and a point
    above it) with smooth weights rising with height, so tau_1 bends the
    upper cap."""
    from .scenes import body_shape_modes, uv_sphere
    V, T = uv_sphere(center, radius, *res)
    c = np.asarray(center, np.float64)
    modes = body_shape_modes(V, c)
    joints = np.stack([c, c + [0.0, 0.6 * radius, 0.0]])
    h = np.clip((V[:, 1] - c[1]) / radius, -1.0, 1.0)
    w1 = 1.0 / (1.0 + np.exp(-6.0 * (h - 0.3)))
    weights = np.stack([1.0 - w1, w1], 1)
    return SyntheticBody(V, modes, joints, weights), T

"""Material estimation by fixed-step gradient descent (Sec. 5.2, Sec. 6).

The controls are (a, b) with mu = a^2 and lambda = b^2 per material, which
keeps both Lame parameters positive whatever step the descent takes.  Each
iteration is one rollout, the weighted goal and the library's exact adjoint,
which returns dL/dmu and dL/dlambda per material; the chain to (a, b) is
dL/da = 2 a dL/dmu, dL/db = 2 b dL/dlambda.
"""
from __future__ import annotations

from typing import Callable, List, Optional

import numpy as np
import torch

from .lib import Simulator


def estimate_materials(sim: Simulator, n_frames: int, targets: torch.Tensor, mu0, lambda0, step: Optional[float],
                       iterations: int, frame_mask=None, vertex_weight: Optional[torch.Tensor] = None,
                       callback: Optional[Callable[[int, float], None]] = None, first_change: float = 0.05):
    """Runs ``iterations`` descent steps from (sqrt(mu0), sqrt(lambda0)).

    ``step`` None: the step is fixed from the first gradient so that the
    first update changes no control by more than ``first_change`` of its
    value (the gradient's scale depends on the mesh and the goal), then kept.
    Returns (a, b, losses): the final controls (FP64 tensors on the device)
    and the goal at every iterate before its update."""
    dev = sim.device
    a = torch.as_tensor(np.sqrt(np.asarray(mu0, np.float64)), device=dev)
    b = torch.as_tensor(np.sqrt(np.asarray(lambda0, np.float64)), device=dev)
    if frame_mask is None:
        frame_mask = np.ones(n_frames, bool)
    losses: List[float] = []
    for it in range(iterations):
        mu = (a * a).to(sim.dtype).contiguous()
        la = (b * b).to(sim.dtype).contiguous()
        xf, _, _ = sim.forward(n_frames, tet_mu=mu, tet_lambda=la, for_adjoint=True)
        loss, dL = sim.goal_l2(xf, targets, frame_mask, vertex_weight)
        g = sim.adjoint(dL, frame_mask, want=("tet_mu", "tet_lambda"))
        ga, gb = 2.0 * a * g["tet_mu"], 2.0 * b * g["tet_lambda"]
        if step is None:
            worst = float(torch.max(torch.cat([(ga / a).abs(), (gb / b).abs()])))
            step = first_change / worst if worst > 0 else 0.0
        a = a - step * ga
        b = b - step * gb
        losses.append(float(loss))
        if callback is not None:
            callback(it, losses[-1])
    return a, b, losses, step

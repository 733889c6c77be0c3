"""The goal entry point that allocates no device memory (partial sums in the
library's static scratch) against xpbd_goal_weighted, the entry point it is
a variant of: the same kernels, so loss and gradient must match bit for bit,
on two calls in a row (the second with a smaller input) and for both state
dtypes."""
import numpy as np
import pytest

from paper_2301_01396_amd import scenes
from tests._cases import needs_gpu

pytestmark = pytest.mark.gpu


def _rollout(sc, dtype, F, seed):
    import torch
    from paper_2301_01396_amd.lib import Simulator
    sim = Simulator(sc, dtype=dtype)
    xf, _, _ = sim.forward(F)
    rng = np.random.default_rng(seed)
    tgt = sim.tensor(xf.double().cpu().numpy() + 0.01 * rng.standard_normal(tuple(xf.shape)))
    torch.cuda.synchronize()
    return sim, xf, tgt


def _both(sim, xf, tgt, mask, weight):
    import torch
    loss_a, dl_a = sim.goal_l2(xf, tgt, mask, vertex_weight=weight)
    loss_b = torch.full((), float("nan"), dtype=torch.float64, device=sim.device)
    dl_b = torch.full_like(xf, float("nan"))
    sim.goal_noalloc(xf, tgt, loss_b, dl_b, frame_mask=mask, vertex_weight=weight)
    torch.cuda.synchronize()
    assert torch.equal(loss_a, loss_b), (float(loss_a), float(loss_b))
    assert torch.equal(dl_a, dl_b)
    assert float(loss_a) > 0
    return float(loss_a)


@pytest.mark.parametrize("dtype_name", ["f32", "f64"])
def test_goal_noalloc_matches_goal_on_two_calls(dtype_name):
    import torch
    needs_gpu()
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    big = scenes.cloth_grid(40, 37, 0.02, origin=(-0.4, 0.0, -0.36), pinned=(0, 36))
    big.dist_alpha = np.full(big.n_dist, 1e-6)
    big.bend_alpha = np.full(big.n_bend, 1e-3)
    big.tet_E = np.zeros(0)
    big.v0 = np.zeros_like(big.rest)
    big.dt, big.substeps, big.iterations = 1 / 60, 1, 2
    small = scenes.small_cloth(n=5, frames=2, substeps=1, iterations=2, sphere=False)
    sa, xa, ta = _rollout(big, dtype, 4, 0)
    sb, xb, tb = _rollout(small, dtype, 2, 1)
    assert 3 * big.n_verts > 4 * 256   # several partial sums per frame
    w = torch.linspace(0.0, 2.0, big.n_verts, dtype=torch.float64, device=sa.device)
    _both(sa, xa, ta, np.array([1, 0, 1, 1], bool), w)
    _both(sb, xb, tb, None, None)      # second call, smaller input
    _both(sa, xa[:1].contiguous(), ta[:1].contiguous(), None, None)
    sa.close()
    sb.close()


def test_goal_noalloc_rejects_more_partial_sums_than_its_scratch():
    import torch
    from paper_2301_01396_amd import lib as L
    needs_gpu()
    sc = scenes.small_cloth(n=5, frames=1, substeps=1, iterations=1, sphere=False)
    sim, xf, tgt = _rollout(sc, torch.float32, 1, 2)
    loss = torch.zeros((), dtype=torch.float64, device=sim.device)
    # one partial sum per frame here: 2^21 + 1 frames exceed the scratch, and
    # the call must refuse before it launches anything
    with pytest.raises(L.XPBDError) as e:
        sim.goal_noalloc(xf, tgt, loss, None, n_frames=(1 << 21) + 1)
    assert e.value.status == L.XPBD_ERR_INVALID and "static scratch" in str(e.value)
    sim.goal_noalloc(xf, tgt, loss, None)
    torch.cuda.synchronize()
    assert float(loss) > 0
    sim.close()

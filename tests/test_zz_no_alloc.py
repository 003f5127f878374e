"""The allocation-free collision entry point (static per-GPU workspace) against
bz_collide_batch on the same inputs: bitwise equal results on two calls in a
row, the second with a smaller batch (the static workspace then holds the
first call's leftovers), in the batched FP32 mode with its FP64 core and in
the plain FP64 mode; a few cells also against the oracle; and the size
limit."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1211_0540_amd import bz
from paper_1211_0540_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _both(col, f):
    """bz_collide_batch on the batch's own workspace (filled with NaN bytes first, so that
    a result leaning on zeroed memory would show) and bz_collide_batch_static."""
    col.work.fill_(255)
    a = col.collide(f)
    b = torch.full_like(a, 7.0)
    bz.bz_collide_batch_static(col.batch, f, b)
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("mode", ["batched_f32", "plain_f64"])
def test_static_workspace_matches_the_caller_workspace(dev, mode):
    N, L = 16, 6.0
    first = list(W.random_smooth_cells(100, N, L, seed=41))   # two groups
    second = list(W.random_smooth_cells(30, N, L, seed=42))   # one ragged group
    for cells in (first, second):
        n = len(cells) if mode == "batched_f32" else 3
        cells = cells[:n]
        col = bz.Collision([(N, L, 1.0)], [0] * n, mode)
        assert bz.bz_workspace_bytes(col.batch) <= bz.BZ_STATIC_SCRATCH_BYTES
        f = torch.from_numpy(col.pack(cells)).to(dev)
        a, b = _both(col, f)
        assert torch.equal(a, b), (mode, n)
        q = col.unpack(col.project(b).cpu().numpy())
        o = O.Oracle(N, L, 1.0)
        for i in (0, n - 1):
            _, qo, _, _ = o.collide(cells[i])
            err = np.linalg.norm(q[i] - qo) / np.linalg.norm(qo)
            assert err < (TOL32 if mode == "batched_f32" else 1e-12), (mode, n, i, err)
        col.close()


def test_static_workspace_rejects_a_batch_too_large(dev):
    N, L, n = 32, 8.0, 190
    col = bz.Collision([(N, L, 1.0)], [0] * n, "batched_f32")
    assert bz.bz_workspace_bytes(col.batch) > bz.BZ_STATIC_SCRATCH_BYTES
    f = torch.zeros(col.elems, dtype=torch.float64, device=dev)
    q = torch.zeros_like(f)
    with pytest.raises(bz.BzError, match="static scratch"):
        bz.bz_collide_batch_static(col.batch, f, q)
    col.close()

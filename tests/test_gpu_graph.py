"""HIP-graph capture of whole steps: every replay must equal the eager step
(replays interleaved with eager work and synchronisations)."""
import numpy as np
import pytest
import torch

from paper_1211_0540_amd import bz
from paper_1211_0540_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def test_captured_heun_step_replays_equal_eager(dev):
    """Uneven mixed-mesh batch (N = 16, 24, 32), batched FP32, one Heun step per replay."""
    full = W.uneven_batch(n_cells=200)
    idx = {16: 0, 24: 1, 32: 2}
    c = bz.Collision([(16, 6.0, 1.0), (24, 7.0, 1.0), (32, 8.0, 1.0)], [idx[int(n)] for n in full.Ns],
                     "batched_f32")
    f0 = torch.from_numpy(c.pack(full.cells)).to(dev)
    s = torch.cuda.Stream()
    fg = f0.clone()
    fe = f0.clone()
    work_g = torch.zeros_like(c.work)
    with torch.cuda.stream(s):
        g = bz.bz_graph_capture_step(c.batch, fg, 0.01, work_g, s)
    torch.cuda.synchronize()
    for rep in range(4):
        bz.bz_graph_launch(g, s)
        s.synchronize()
        c.step(fe, 0.01)                 # eager reference on the default stream
        torch.cuda.synchronize()
        assert torch.equal(fg, fe), rep
    bz.bz_graph_free(g)
    c.close()


def test_captured_strang_step_replays_equal_eager(dev):
    N, L, nx = 16, 6.0, 64
    c = bz.Collision([(N, L, 1.0)], [0] * nx, "batched_f32")
    t = bz.bz_transport_create(c.grids[0], nx, 1.0, 2.0, 1.0, 0.0, 1.0)
    f0 = torch.from_numpy(W.shock_initial(nx, N, L).ravel().copy()).to(dev)
    need = bz.bz_strang_workspace_bytes(c.batch, t)
    wg = torch.zeros(need, dtype=torch.uint8, device=dev)
    we = torch.zeros(need, dtype=torch.uint8, device=dev)
    fg, fe = f0.clone(), f0.clone()
    dt = 0.5 / nx / L
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = bz.bz_graph_capture_strang(c.batch, t, fg, dt, 0.1, wg, s)
    torch.cuda.synchronize()
    for rep in range(3):
        bz.bz_graph_launch(g, s)
        s.synchronize()
        bz.bz_strang_step(c.batch, t, fe, dt, 0.1, we)
        torch.cuda.synchronize()
        assert torch.equal(fg, fe), rep
    bz.bz_graph_free(g)
    bz.bz_transport_free(t)
    c.close()

"""Network kernels of the learned closure against the FP64 oracle (GPU, C ABI).

The oracle mirrors the GPU's bfloat16 storage (inputs, weights, hidden
activations, layer-output gradients); the remaining differences are FP32
accumulation order and rare one-ulp bfloat16 flips of a hidden value."""
import numpy as np
import pytest
import torch

from oracle import mlp as OM
from paper_1211_0540_amd import bz

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def to_bf16_bits(x):
    a = np.ascontiguousarray(OM.bf16_round(x), dtype=np.float32)
    return (a.view(np.uint32) >> 16).astype(np.uint16)


def setup(n_in, n_h, n_out, B, seed, dev):
    n = bz.bz_mlp_create(n_in, n_h, n_out)
    p = OM.init_params(n_in, n_h, n_out, seed)
    params = torch.zeros(bz.bz_mlp_param_bytes(n), dtype=torch.uint8, device=dev)
    bz.bz_mlp_set_params(n, params, bz.mlp_pack(p))
    work = torch.zeros(bz.bz_mlp_workspace_bytes(n, B), dtype=torch.uint8, device=dev)
    # oracle sees the same FP32-rounded master weights
    p32 = bz.mlp_unpack(bz.mlp_pack(p), n_in, n_h, n_out)
    return n, params, work, p32


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("shape", [(64, 64, 96, 40), (13824, 1024, 13824, 64)])
def test_forward_matches_oracle(dev, shape):
    n_in, n_h, n_out, B = shape
    n, params, work, p = setup(n_in, n_h, n_out, B, 3, dev)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((B, n_in))
    x = torch.from_numpy(to_bf16_bits(X).view(np.int16)).to(dev)
    y = torch.zeros(B, n_out, dtype=torch.float32, device=dev)
    bz.bz_mlp_forward(n, params, x, B, y, work)
    Y, _ = OM.forward(p, X, bf16=True)
    assert rel(y.cpu().numpy(), Y) < 1e-3
    bz.bz_mlp_free(n)


@pytest.mark.parametrize("shape", [(64, 96, 64, 64), (13824, 1024, 13824, 64)])
def test_gradients_match_oracle(dev, shape):
    n_in, n_h, n_out, B = shape
    n, params, work, p = setup(n_in, n_h, n_out, B, 4, dev)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    x = torch.from_numpy(to_bf16_bits(X).view(np.int16)).to(dev)
    t = torch.from_numpy(T.astype(np.float32)).to(dev)
    grad = torch.zeros(bz.bz_mlp_param_count(n), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    bz.bz_mlp_backward(n, params, x, t, B, grad, loss, work)
    L, g, _ = OM.loss_and_grads(p, X, T, bf16=True)
    gg = bz.mlp_unpack(grad.cpu().numpy(), n_in, n_h, n_out)
    assert float(loss.item()) == pytest.approx(L, rel=1e-4)
    for k in g:
        assert rel(gg[k], g[k]) < 5e-3, k
    bz.bz_mlp_free(n)


def test_adam_step_matches_oracle(dev):
    n_in, n_h, n_out, B = 64, 64, 32, 32
    n, params, work, p = setup(n_in, n_h, n_out, B, 5, dev)
    rng = np.random.default_rng(2)
    G = rng.standard_normal(bz.bz_mlp_param_count(n)).astype(np.float32)
    grad = torch.from_numpy(G).to(dev)
    st = {}
    q = p
    for step in (1, 2):
        bz.bz_mlp_adam(n, params, grad, step, 1e-3)
        q = OM.adam_update(q, bz.mlp_unpack(G, n_in, n_h, n_out), st, step, 1e-3)
    got = bz.mlp_unpack(bz.bz_mlp_get_params(n, params), n_in, n_h, n_out)
    for k in q:
        assert np.max(np.abs(got[k] - q[k])) < 1e-6 * (1 + np.max(np.abs(q[k]))), k
    bz.bz_mlp_free(n)



def test_unaligned_buffers_give_the_same_results(dev):
    """The transposes and Adam use 16-byte accesses on 16-byte aligned buffers and an
    element-wise path otherwise: an input or gradient buffer one element off alignment must
    give bitwise the same gradients, parameters and BF16 weight copies."""
    n_in, n_h, n_out, B = 64, 96, 64, 64
    rng = np.random.default_rng(7)
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    xb = torch.from_numpy(to_bf16_bits(X).view(np.int16)).to(dev)
    x_off = torch.zeros(B * n_in + 1, dtype=torch.int16, device=dev)[1:].view(B, n_in)
    x_off.copy_(xb)
    assert x_off.data_ptr() % 16 != 0
    t = torch.from_numpy(T.astype(np.float32)).to(dev)
    runs = []
    for x, off in ((xb, False), (x_off, True)):
        n, params, work, _ = setup(n_in, n_h, n_out, B, 8, dev)
        P = bz.bz_mlp_param_count(n)
        grad = torch.zeros(P + 1, dtype=torch.float32, device=dev)[1:] if off else \
            torch.zeros(P, dtype=torch.float32, device=dev)
        assert (grad.data_ptr() % 16 != 0) == off
        loss = torch.zeros(1, dtype=torch.float32, device=dev)
        for step in (1, 2):
            bz.bz_mlp_backward(n, params, x, t, B, grad, loss, work)
            bz.bz_mlp_adam(n, params, grad, step, 1e-3)
        y = torch.zeros(B, n_out, dtype=torch.float32, device=dev)
        bz.bz_mlp_forward(n, params, x, B, y, work)
        runs.append((grad.clone(), bz.bz_mlp_get_params(n, params), y.clone()))
        bz.bz_mlp_free(n)
    (g0, p0, y0), (g1, p1, y1) = runs
    assert torch.equal(g0, g1)
    assert np.array_equal(p0, p1)
    assert torch.equal(y0, y1)   # the forward reads the BF16 copies Adam wrote

def test_training_reduces_loss(dev):
    n_in, n_h, n_out, B = 128, 128, 64, 64
    n, params, work, p = setup(n_in, n_h, n_out, B, 6, dev)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((B, n_in))
    A = rng.standard_normal((n_in, n_out)) / np.sqrt(n_in)
    T = np.tanh(X @ A)
    x = torch.from_numpy(to_bf16_bits(X).view(np.int16)).to(dev)
    t = torch.from_numpy(T.astype(np.float32)).to(dev)
    grad = torch.zeros(bz.bz_mlp_param_count(n), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    hist = []
    for step in range(1, 201):
        bz.bz_mlp_backward(n, params, x, t, B, grad, loss, work)
        bz.bz_mlp_adam(n, params, grad, step, 3e-3)
        hist.append(float(loss.item()))
    assert hist[-1] < 0.05 * hist[0]
    bz.bz_mlp_free(n)


def test_real_shape_against_the_unmirrored_fp64_oracle(dev):
    """The network at its real shape against the plain FP64 oracle (no bfloat16 mirroring,
    whose own pin is finite differences): the loss, the output and every gradient within the
    bfloat16 storage tolerance 1e-2 (the mirrored and plain oracles differ by about 4e-3)."""
    n_in, n_h, n_out, B = 13824, 1024, 13824, 64
    n, params, work, p = setup(n_in, n_h, n_out, B, 4, dev)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    x = torch.from_numpy(to_bf16_bits(X).view(np.int16)).to(dev)
    t = torch.from_numpy(T.astype(np.float32)).to(dev)
    y = torch.zeros(B, n_out, dtype=torch.float32, device=dev)
    bz.bz_mlp_forward(n, params, x, B, y, work)
    grad = torch.zeros(bz.bz_mlp_param_count(n), dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    bz.bz_mlp_backward(n, params, x, t, B, grad, loss, work)
    L, g, Y = OM.loss_and_grads(p, X, T, bf16=False)
    assert rel(y.cpu().numpy(), Y) < 1e-2
    assert float(loss.item()) == pytest.approx(L, rel=1e-3)
    gg = bz.mlp_unpack(grad.cpu().numpy(), n_in, n_h, n_out)
    for k in g:
        assert rel(gg[k], g[k]) < 1e-2, k
    bz.bz_mlp_free(n)

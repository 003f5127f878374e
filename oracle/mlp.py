"""FP64 oracle of the learned closure's network: a 3-layer perceptron with exact
(erf) GELU, mean-squared-error loss and Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, matmuls
as library primitives, no fusion.

Network (weights stored as [out, in], like the GPU):
    Z1 = X W1^T + b1,  A1 = gelu(Z1)
    Z2 = A1 W2^T + b2, A2 = gelu(Z2)
    Y  = A2 W3^T + b3
loss = mean over batch and outputs of (Y - T)^2.

`bf16=True` mirrors the GPU's storage roundings (inputs, weights and the two
hidden activations rounded to bfloat16, round-to-nearest-even) while doing
the arithmetic in FP64.
"""
from __future__ import annotations

import math

import numpy as np


def bf16_round(x):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init_params(n_in, n_hidden, n_out, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (FP64)."""
    rng = np.random.default_rng(seed)
    def lin(o, i):
        s = 1.0 / math.sqrt(i)
        return rng.uniform(-s, s, (o, i)), rng.uniform(-s, s, o)
    W1, b1 = lin(n_hidden, n_in)
    W2, b2 = lin(n_hidden, n_hidden)
    W3, b3 = lin(n_out, n_hidden)
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "W3": W3, "b3": b3}


def forward(p, X, bf16=False):
    r = bf16_round if bf16 else (lambda a: a)
    X = r(X)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    Z1 = X @ W1.T + p["b1"]
    A1 = r(gelu(Z1))
    Z2 = A1 @ W2.T + p["b2"]
    A2 = r(gelu(Z2))
    Y = A2 @ W3.T + p["b3"]
    return Y, {"X": X, "Z1": Z1, "A1": A1, "Z2": Z2, "A2": A2, "W1": W1, "W2": W2, "W3": W3}


def loss_and_grads(p, X, T, bf16=False):
    """Loss (mean squared error) and its gradients.

    With bf16=True the storage roundings of the GPU are mirrored: the output error
    Y - T is stored as bfloat16 and the factor 2/n is applied after each product
    with it, and dL/dZ2, dL/dZ1 are stored as bfloat16 before their products."""
    r = bf16_round if bf16 else (lambda a: a)
    Y, c = forward(p, X, bf16)
    n = Y.size
    loss = float(((Y - T) ** 2).sum() / n)
    gs = 2.0 / n
    E = r(Y - T)
    g = {"W3": gs * (E.T @ c["A2"]), "b3": gs * E.sum(0)}
    dA2 = gs * (E @ c["W3"])
    dZ2 = r(dA2 * gelu_prime(c["Z2"]))
    g["W2"] = dZ2.T @ c["A1"]
    g["b2"] = dZ2.sum(0)
    dA1 = dZ2 @ c["W2"]
    dZ1 = r(dA1 * gelu_prime(c["Z1"]))
    g["W1"] = dZ1.T @ c["X"]
    g["b1"] = dZ1.sum(0)
    return loss, g, Y


def adam_update(p, g, state, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) at step number t >= 1; state holds m and v per tensor."""
    out = {}
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        out[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return out

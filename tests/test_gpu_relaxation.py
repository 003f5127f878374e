"""Homogeneous relaxation of a bi-Maxwellian on the N=32, L=8 mesh: 100 Heun
steps with dt = 0.01 (Sec. 3.1), the batched FP32 path (compensated
convolution, FP64 projection) against the plain FP64 path, and the Maxwell
molecule twin against its closed-form temperature relaxation."""
import math

import numpy as np
import pytest
import torch

from paper_1211_0540_amd import bz
from paper_1211_0540_amd import workloads as W

pytestmark = pytest.mark.gpu

N, L, STEPS, DT = 32, 8.0, 100, 0.01


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _directional(f):
    """rho, energy and (T_1, T_2, T_3) of one cell from the definitions (uniform weights)."""
    dv = 2 * L / N
    v = dv * (np.arange(N) - N // 2)
    V = np.meshgrid(v, v, v, indexing="ij")
    w = dv ** 3
    rho = f.sum() * w
    u = [(V[d] * f).sum() * w / rho for d in range(3)]
    Td = np.array([((V[d] - u[d]) ** 2 * f).sum() * w / rho for d in range(3)])
    energy = ((V[0] ** 2 + V[1] ** 2 + V[2] ** 2) * f).sum() * w
    return rho, energy, Td


def _run(dev, mode, lam):
    f0 = W.relaxation_cell(N, L)
    c = bz.Collision([(N, L, lam)], [0], mode)
    f = torch.from_numpy(c.pack([f0])).to(dev)
    hist = [_directional(f0)]
    for _ in range(STEPS):
        c.step(f, DT)
        hist.append(_directional(f.cpu().numpy().reshape(N, N, N)))
    c.check()
    c.close()
    rho = np.array([h[0] for h in hist])
    energy = np.array([h[1] for h in hist])
    T = np.array([h[2] for h in hist])
    return rho, energy, T


def test_hard_sphere_relaxation_fp32_follows_fp64(dev):
    r64, e64, T64 = _run(dev, "plain_f64", 1.0)
    r32, e32, T32 = _run(dev, "batched_f32", 1.0)
    dT = np.max(np.abs(T32 - T64))
    print(f"max |T_d^32 - T_d^64| over {STEPS} steps: {dT:.3e}; T_x(1) = {T64[-1, 0]:.6f}")
    # conservation of mass and energy through every projected step
    for r, e in ((r64, e64), (r32, e32)):
        assert np.max(np.abs(r - r[0])) <= 1e-12 * r[0]
        assert np.max(np.abs(e - e[0])) <= 1e-11 * e[0]
    # relaxation towards the isotropic state: T_x falls, T_y = T_z rise, sum fixed
    assert np.all(np.diff(T64[:, 0]) < 0) and np.all(np.diff(T64[:, 1]) > 0)
    assert np.max(np.abs(T64[:, 1] - T64[:, 2])) < 1e-12
    assert 1.0 < T64[-1, 0] < 1.7
    # the FP32 curve follows the FP64 one
    assert dT < 1e-6


def test_maxwell_molecule_twin_matches_closed_form(dev):
    """For Maxwell molecules with isotropic b, T_x(t) = T + (T_x0 - T) exp(-rho t / 2)."""
    rho, _, T = _run(dev, "batched_f64", 0.0)
    t = DT * np.arange(STEPS + 1)
    Tm = T.mean(axis=1)
    exact = Tm[0] + (T[0, 0] - Tm[0]) * np.exp(-rho[0] * t / 2)
    err = np.max(np.abs(T[:, 0] - exact))
    print(f"max |T_x - closed form| = {err:.3e}")
    assert err < 2e-3

"""Pins for the transport oracle (Sec. 3.4 upwind/minmod, Sec. 2.1 diffuse wall,
RK2 in time): exact identities and the scheme's known orders."""
import numpy as np
import pytest

from oracle import transport as T
from paper_1211_0540_amd import workloads as W

N, L = 8, 4.0


def _mass(f, dx):
    return f.sum() * dx * (2 * L / N) ** 3


def test_wall_mass_flux_is_exactly_zero():
    rng = np.random.default_rng(0)
    f = rng.uniform(0.1, 1.0, (5, N, N, N))
    for Tw in (0.5, 1.0, 2.0):
        Mw = T.wall_maxwellian(N, L, Tw)
        assert abs(T.wall_flux(f, N, L, Mw)) < 1e-15 * np.abs(f[0]).sum()


def test_mass_changes_only_by_the_far_field_flux():
    """Right cells equal to M_far: the right face carries v1 M_far exactly, so one RK2 step
    changes the mass by -dt * sum v1 M_far dv^3 (the wall flux is zero)."""
    nx, dx, dt = 32, 1.0 / 32, 0.2 / 32 / L
    Mfar = W.maxwellian(N, L, 1.0, (0.3, 0, 0), 1.0)
    Mw = T.wall_maxwellian(N, L, 2.0)
    f = np.broadcast_to(Mfar, (nx, N, N, N)).copy()
    x = (np.arange(nx) + 0.5) * dx
    f *= (1 + 0.5 * np.exp(-((x - 0.3) / 0.05) ** 2))[:, None, None, None]
    g = T.transport_rk2(f, N, L, dx, dt, Mw, Mfar)
    v1 = W.velocity_mesh(N, L)[:, None, None]
    expect = -dt * (v1 * Mfar).sum() * (2 * L / N) ** 3
    assert _mass(g, dx) - _mass(f, dx) == pytest.approx(expect, rel=1e-9, abs=1e-15)


def test_equilibrium_at_wall_temperature_is_steady():
    """Gas at rest at the wall temperature is steady up to the mesh asymmetry: the
    v1 = -L plane has no +L partner, so sigma_w - 1 equals its outgoing flux share."""
    Lw, nx, dx = 6.0, 16, 1.0 / 16
    M = W.maxwellian(N, Lw, 1.0, (0, 0, 0), 1.0)
    Mw = T.wall_maxwellian(N, Lw, 1.0)
    f = np.broadcast_to(M, (nx, N, N, N)).copy()
    _, sigma = T.transport_rhs(f, N, Lw, dx, Mw, M)
    v1 = W.velocity_mesh(N, Lw)
    pos = (v1[v1 > 0][:, None, None] * M[v1 > 0]).sum()
    assert sigma - 1.0 == pytest.approx(Lw * M[0].sum() / pos, rel=1e-9)
    g = f
    for _ in range(10):
        g = T.transport_rk2(g, N, Lw, dx, 0.01, Mw, M)
    assert np.max(np.abs(g - f)) < 10 * 0.01 / dx * (sigma - 1.0) * Lw * M.max()


def _advect_error(nx):
    dx = 1.0 / nx
    x = (np.arange(nx) + 0.5) * dx
    v = W.velocity_mesh(N, L)
    prof = lambda y: np.exp(-((y - 0.4) / 0.08) ** 2)
    f = prof(x)[:, None, None, None] * np.ones((1, N, N, N))
    zero = np.zeros((N, N, N))
    tend = 0.02
    steps = int(round(tend / (0.2 * dx / L)))
    dt = tend / steps
    for _ in range(steps):
        f = T.transport_rk2(f, N, L, dx, dt, T.wall_maxwellian(N, L, 1.0), zero)
    exact = prof(x[:, None] - v[None, :] * tend)[:, :, None, None]
    return np.abs(f - exact).sum() * dx / (np.abs(exact).sum() * dx)


def test_muscl_rk2_converges_at_second_order():
    e1, e2 = _advect_error(64), _advect_error(128)
    assert e2 < e1 and e1 / e2 > 3.0


def test_no_new_extrema_away_from_boundaries():
    nx, dx = 64, 1.0 / 64
    x = (np.arange(nx) + 0.5) * dx
    rng = np.random.default_rng(3)
    prof = np.where(np.abs(x - 0.5) < 0.2, rng.uniform(0, 1, nx), 0.0)
    f = prof[:, None, None, None] * np.ones((1, N, N, N))
    g = T.transport_rk2(f, N, L, dx, 0.4 * dx / L, T.wall_maxwellian(N, L, 1.0), np.zeros((N, N, N)))
    assert g.max() <= f.max() + 1e-14 and g.min() >= f.min() - 1e-14

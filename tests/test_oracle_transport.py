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


# ----------------------------------------------------------------------------
# Cells of width dx_j (Sec. 3.4: "cells of size dx_j (not necessarily uniform)")
# ----------------------------------------------------------------------------
def _stretched(nx, ratio=1.15, seed=None):
    """Widths growing geometrically away from the wall, normalised to a unit domain."""
    w = ratio ** np.arange(nx)
    if seed is not None:
        w *= np.random.default_rng(seed).uniform(0.7, 1.3, nx)
    return w / w.sum()


def test_uniform_width_array_is_the_uniform_scheme():
    rng = np.random.default_rng(1)
    nx = 12
    f = rng.uniform(0.1, 1.0, (nx, N, N, N))
    Mw, Mf = T.wall_maxwellian(N, L, 1.5), W.maxwellian(N, L, 1.0, (0.2, 0, 0), 1.0)
    a, sa = T.transport_rhs(f, N, L, 1.0 / nx, Mw, Mf)
    b, sb = T.transport_rhs(f, N, L, np.full(nx, 1.0 / nx), Mw, Mf)
    assert np.array_equal(a, b) and sa == sb


def test_free_stream_is_preserved_on_a_stretched_mesh():
    """A gas uniform in x (far field equal to it) has zero flux divergence in every cell not
    touching the wall, whatever the widths: all slopes vanish and each face carries v1 g."""
    nx = 20
    g = W.maxwellian(N, L, 1.3, (0.4, -0.2, 0.1), 0.8)
    f = np.broadcast_to(g, (nx, N, N, N)).copy()
    rhs, _ = T.transport_rhs(f, N, L, _stretched(nx, seed=3), T.wall_maxwellian(N, L, 2.0), g)
    assert np.max(np.abs(rhs[1:])) == 0.0


def test_mass_balance_on_a_stretched_mesh():
    """sum_j dx_j f_j changes only by the boundary fluxes (the wall's is zero): with the
    right cells at M_far, one RK2 step changes it by -dt sum v1 M_far dv^3."""
    nx = 32
    w = _stretched(nx, ratio=1.05, seed=4)
    Mfar = W.maxwellian(N, L, 1.0, (0.3, 0, 0), 1.0)
    Mw = T.wall_maxwellian(N, L, 2.0)
    x = np.cumsum(w) - 0.5 * w
    f = np.broadcast_to(Mfar, (nx, N, N, N)).copy()
    f *= (1 + 0.5 * np.exp(-((x - 0.3) / 0.05) ** 2))[:, None, None, None]
    dt = 0.2 * w.min() / L
    g = T.transport_rk2(f, N, L, w, dt, Mw, Mfar)
    dv3 = (2 * L / N) ** 3
    mass = lambda h: (h.sum(axis=(1, 2, 3)) * w).sum() * dv3
    v1 = W.velocity_mesh(N, L)[:, None, None]
    assert mass(g) - mass(f) == pytest.approx(-dt * (v1 * Mfar).sum() * dv3, rel=1e-9, abs=1e-15)


def _advect_error_mapped(nx):
    """A Gaussian advected on the smooth map x(s) = s + 0.15 sin(2 pi s) / (2 pi), s uniform."""
    s = np.linspace(0.0, 1.0, nx + 1)
    xe = s + 0.15 * np.sin(2 * np.pi * s) / (2 * np.pi)
    w = np.diff(xe)
    xc = 0.5 * (xe[1:] + xe[:-1])
    v = W.velocity_mesh(N, L)
    prof = lambda y: np.exp(-((y - 0.45) / 0.08) ** 2)
    f = prof(xc)[:, None, None, None] * np.ones((1, N, N, N))
    zero = np.zeros((N, N, N))
    tend = 0.02
    steps = int(np.ceil(tend / (0.2 * w.min() / L)))
    dt = tend / steps
    for _ in range(steps):
        f = T.transport_rk2(f, N, L, w, dt, T.wall_maxwellian(N, L, 1.0), zero)
    exact = prof(xc[:, None] - v[None, :] * tend)[:, :, None, None]
    return (np.abs(f - exact) * w[:, None, None, None]).sum() / (np.abs(exact) * w[:, None, None, None]).sum()


def test_muscl_rk2_second_order_on_a_smooth_stretching():
    e1, e2 = _advect_error_mapped(64), _advect_error_mapped(128)
    assert e2 < e1 and e1 / e2 > 3.0


# ----------------------------------------------------------------------------
# Strang splitting T(dt/2) C(dt) T(dt/2) (Sec. 3.1)
# ----------------------------------------------------------------------------
class _NoCollision:
    """Stands in for the collision oracle with Q = 0: its Heun step is the identity."""
    N, L = N, L

    def rk2(self, f, dt, eps, steps):
        return np.array(f, copy=True)


def _shock_state(nx, seed=0):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    base = W.maxwellian(N, L, 1.0, (0.0, 0, 0), 1.0)
    bump = W.maxwellian(N, L, 0.6, (0.5, 0.2, 0), 0.7)
    return base[None] + np.exp(-((x - 0.35) / 0.1) ** 2)[:, None, None, None] * bump[None] * rng.uniform(0.8, 1.2)


def test_strang_without_collisions_is_two_transport_half_steps():
    nx, dx, dt = 10, 0.1, 0.01
    f = _shock_state(nx)
    Mw, Mf = T.wall_maxwellian(N, L, 2.0), W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    got = T.strang_step(f, _NoCollision(), dx, dt, 1.0, Mw, Mf)
    half = T.transport_rk2(T.transport_rk2(f, N, L, dx, 0.5 * dt, Mw, Mf), N, L, dx, 0.5 * dt, Mw, Mf)
    assert np.array_equal(got, half)


def test_strang_without_transport_is_one_collision_step(monkeypatch):
    import oracle as O
    nx, dt, eps = 4, 0.05, 0.5
    f = _shock_state(nx, seed=1)
    o = O.Oracle(N, L, 1.0)
    monkeypatch.setattr(T, "transport_rk2", lambda g, *a: np.array(g, copy=True))
    got = T.strang_step(f, o, 0.1, dt, eps, T.wall_maxwellian(N, L, 2.0), f[-1])
    assert np.max(np.abs(got - o.rk2(f, dt, eps, 1))) == 0.0


def _strang_solution(o, f0, dx, dt, nsteps, eps, Mw, Mf):
    f = f0
    for _ in range(nsteps):
        f = T.strang_step(f, o, dx, dt, eps, Mw, Mf)
    return f


def test_strang_splitting_is_second_order_in_time():
    """N = 8, 16 cells, collision and transport of comparable speed (eps = 0.25): halving dt
    cuts the error at t = 0.1 about fourfold against a fine-dt reference."""
    import oracle as O
    nx, eps, tend = 16, 0.25, 0.1
    dx = 1.0 / nx
    o = O.Oracle(N, L, 1.0)
    f0 = _shock_state(nx, seed=2)
    Mw, Mf = T.wall_maxwellian(N, L, 2.0), W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    ref = _strang_solution(o, f0, dx, tend / 64, 64, eps, Mw, Mf)
    e = [np.linalg.norm(_strang_solution(o, f0, dx, tend / n, n, eps, Mw, Mf) - ref) for n in (4, 8)]
    assert 3.2 < e[0] / e[1] < 5.0, e


@pytest.mark.parametrize("mutation", [1, 2])
def test_planted_strang_mistake_is_caught(mutation, monkeypatch):
    """Full-dt transport substeps, or a collision part over dt/2, fail the pins above: one of
    the two structural pins, and the order-of-accuracy pin (the mutated step is inconsistent,
    so its error against the unmutated fine-dt solution does not shrink with dt)."""
    import oracle as O
    nx, eps, tend = 16, 0.25, 0.1
    o = O.Oracle(N, L, 1.0)
    f0 = _shock_state(nx, seed=2)
    Mw, Mf = T.wall_maxwellian(N, L, 2.0), W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    ref = _strang_solution(o, f0, 1.0 / nx, tend / 64, 64, eps, Mw, Mf)
    T.set_mutation(mutation)
    try:
        e = [np.linalg.norm(_strang_solution(o, f0, 1.0 / nx, tend / n, n, eps, Mw, Mf) - ref) for n in (4, 8)]
        assert not (3.2 < e[0] / e[1] < 5.0)
        caught = []
        try:
            test_strang_without_collisions_is_two_transport_half_steps()
            caught.append(False)
        except AssertionError:
            caught.append(True)
        with monkeypatch.context() as m:
            try:
                test_strang_without_transport_is_one_collision_step(m)
                caught.append(False)
            except AssertionError:
                caught.append(True)
        assert any(caught)
    finally:
        T.set_mutation(0)


def test_moments_and_marginal_of_a_maxwellian():
    """Moments of a discrete Maxwellian on a wide mesh return its parameters; the v1
    marginal integrates to the density."""
    Nw, Lw = 24, 8.0
    f = W.maxwellian(Nw, Lw, 1.7, (0.3, -0.2, 0.1), 1.2)[None]
    rho, u, Tm = T.moments_1d(f, Nw, Lw)
    assert rho[0] == pytest.approx(1.7, rel=1e-9) and Tm[0] == pytest.approx(1.2, rel=1e-8)
    assert np.allclose(u[0], (0.3, -0.2, 0.1), atol=1e-9)
    m = T.marginal_v1(f[0], Nw, Lw)
    assert m.sum() * (2 * Lw / Nw) == pytest.approx(rho[0], rel=1e-13)
    # the v1 marginal of a Maxwellian is the 1-D Gaussian of rho, u1 and T (the mesh sums over
    # v2, v3 of a smooth Gaussian are exact to far below 1e-8 here); a marginal over another
    # axis would carry u2 or u3 instead
    v1 = (2 * Lw / Nw) * (np.arange(Nw) - Nw // 2)
    g = 1.7 * (2 * np.pi * 1.2) ** -0.5 * np.exp(-(v1 - 0.3) ** 2 / (2 * 1.2))
    assert np.max(np.abs(m - g)) < 1e-8 * g.max()

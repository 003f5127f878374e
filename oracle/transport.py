"""FP64 oracle for the 1-D-in-space transport step and the Strang-split step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy, written
from Sec. 3.4 (finite-volume upwind flux with minmod slopes, eq. upwind, on
cells of width dx_j that need not be uniform), Sec. 2.1 (diffuse Maxwell wall,
eq. BC) and Sec. 3.1 (operator splitting, second-order Runge-Kutta for each
part, Strang combination).

Readings (the paper is silent on these):
  * RK2 is Heun's method; Strang order is T(dt/2) C(dt) T(dt/2).
  * Cells j = 0..nx-1 of widths dx_j (a scalar dx means uniform cells).  The
    minmod slope uses the distances between cell centres,
      sigma_j = minmod((f_j - f_{j-1}) / d_{j-1/2}, (f_{j+1} - f_j) / d_{j+1/2}),
      d_{j+1/2} = (dx_j + dx_{j+1}) / 2,
    each cell is reconstructed to its faces with its own half-width,
    f_j +- (dx_j / 2) sigma_j, and the update divides the flux difference by
    dx_j.  On a uniform mesh this is the formula of eq. (upwind) as printed.
  * Wall at the left end (x = 0), wall velocity 0, temperature T_w, R = 1.
    Two ghost cells of width dx_0 copy the first cell, so the first cell's
    slope is 0 and the outgoing face value is f_0.  The wall face flux is
    v1 f_0 for v1 < 0 and v1 sigma_w M_w for v1 > 0 with the discrete
      sigma_w = sum_{v1<0} |v1| f_0 / sum_{v1>0} v1 M_w,
    M_w = (2 pi T_w)^{-3/2} exp(-|v|^2 / (2 T_w)), which makes the net mass
    flux through the wall exactly zero.
  * Right end: two ghost cells of width dx_{nx-1} hold a far-field Maxwellian
    M_far.

`set_mutation` plants a known mistake in the Strang composition for the pin
tests (0 restores it): 1 transport substeps over the full dt instead of dt/2,
2 the collision part over dt/2 instead of dt.
"""
from __future__ import annotations

import numpy as np

_mutation = 0


def set_mutation(m: int) -> None:
    global _mutation
    _mutation = int(m)


def minmod(a, b):
    return np.where(a * b > 0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _mesh_v1(N, L):
    return (2.0 * L / N) * (np.arange(N) - N // 2)


def wall_maxwellian(N, L, T_w):
    v = _mesh_v1(N, L)
    V = np.meshgrid(v, v, v, indexing="ij")
    r2 = V[0] ** 2 + V[1] ** 2 + V[2] ** 2
    return (2 * np.pi * T_w) ** -1.5 * np.exp(-r2 / (2 * T_w))


def cell_widths(dx, nx):
    """The nx cell widths: a scalar dx repeated, or the given array."""
    w = np.broadcast_to(np.asarray(dx, dtype=np.float64), (nx,)).astype(np.float64)
    if np.any(w <= 0):
        raise ValueError("cell widths must be positive")
    return w


def transport_rhs(f, N, L, dx, M_wall, M_far):
    """-(F_{j+1/2} - F_{j-1/2}) / dx_j for every cell; f has shape (nx, N, N, N)."""
    nx = f.shape[0]
    w = cell_widths(dx, nx)
    v1 = _mesh_v1(N, L)[None, :, None, None]
    g = np.empty((nx + 4,) + f.shape[1:])
    g[2:-2] = f
    g[0] = g[1] = f[0]            # wall side: zero-gradient ghosts
    g[-2] = g[-1] = M_far          # far field
    wg = np.concatenate([[w[0], w[0]], w, [w[-1], w[-1]]])[:, None, None, None]
    d = 0.5 * (wg[:-1] + wg[1:])   # centre distances d_{i+1/2}, i = -2 .. nx
    s = minmod((g[1:-1] - g[:-2]) / d[:-1], (g[2:] - g[1:-1]) / d[1:])   # slopes of cells -1 .. nx
    # faces between cell i-1 and i for i = 0 .. nx (face i-1/2); arrays over g-index
    fl = g[1:-2] + 0.5 * wg[1:-2] * s[:-1]     # left state (cell i-1 reconstructed to its right face)
    fr = g[2:-1] - 0.5 * wg[2:-1] * s[1:]      # right state (cell i reconstructed to its left face)
    F = np.where(v1 >= 0, v1 * fl, v1 * fr)         # faces -1/2 .. nx-1/2, shape (nx+1, ...)
    # diffuse wall at face -1/2
    dv3 = (2.0 * L / N) ** 3
    out_flux = np.sum(np.where(v1 < 0, -v1 * f[0], 0.0)) * dv3
    in_norm = np.sum(np.where(v1 > 0, v1 * M_wall, 0.0)) * dv3
    sigma_w = out_flux / in_norm
    F[0] = np.where(v1[0] > 0, v1[0] * sigma_w * M_wall, v1[0] * f[0])
    return -(F[1:] - F[:-1]) / w[:, None, None, None], sigma_w


def transport_rk2(f, N, L, dx, dt, M_wall, M_far):
    """Heun step of the transport part over dt."""
    k1, _ = transport_rhs(f, N, L, dx, M_wall, M_far)
    fs = f + dt * k1
    k2, _ = transport_rhs(fs, N, L, dx, M_wall, M_far)
    return 0.5 * (f + fs + dt * k2)


def wall_flux(f, N, L, M_wall):
    """Net mass flux through the wall face (positive into the domain)."""
    v1 = _mesh_v1(N, L)[:, None, None]
    dv3 = (2.0 * L / N) ** 3
    out_flux = np.sum(np.where(v1 < 0, -v1 * f[0], 0.0)) * dv3
    in_norm = np.sum(np.where(v1 > 0, v1 * M_wall, 0.0)) * dv3
    sigma_w = out_flux / in_norm
    return np.sum(np.where(v1 > 0, v1 * sigma_w * M_wall, v1 * f[0])) * dv3


def strang_step(f, oracle, dx, dt, eps, M_wall, M_far):
    """T(dt/2) C(dt) T(dt/2); C is the Heun step of df/dt = Q(f,f)/eps per cell."""
    N, L = oracle.N, oracle.L
    tt = dt if _mutation == 1 else 0.5 * dt
    tc = 0.5 * dt if _mutation == 2 else dt
    f = transport_rk2(f, N, L, dx, tt, M_wall, M_far)
    f = oracle.rk2(f, tc, eps, 1)
    return transport_rk2(f, N, L, dx, tt, M_wall, M_far)


def moments_1d(f, N, L):
    """Per cell: density, bulk velocity (3) and temperature; f has shape (nx, N, N, N)."""
    v = _mesh_v1(N, L)
    dv3 = (2.0 * L / N) ** 3
    V = np.meshgrid(v, v, v, indexing="ij")
    rho = f.sum(axis=(1, 2, 3)) * dv3
    u = np.stack([(f * V[d]).sum(axis=(1, 2, 3)) * dv3 / rho for d in range(3)], 1)
    e = sum(((V[d][None] - u[:, d, None, None, None]) ** 2 * f).sum(axis=(1, 2, 3)) for d in range(3)) * dv3
    return rho, u, e / (3.0 * rho)


def marginal_v1(f_cell, N, L):
    """Marginal of one cell's distribution in v1: sum over v2, v3 of f dv^2."""
    dv = 2.0 * L / N
    return f_cell.sum(axis=(1, 2)) * dv * dv

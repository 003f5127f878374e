"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no arithmetic of the collision method: it only evaluates
distribution functions (Maxwellians, bi-Maxwellians, the BKW profile) on the
velocity mesh of Sec. 3.1 so that the oracle and the HIP path receive the same
inputs.  Every generator is deterministic for a given seed.

Workloads (the paper runs a sudden wall-heating problem whose sizes it does
not give; these stand in for it):
  single_cell_mixture   N=16, L=6, Maxwell molecules, two counter-streaming
                        Maxwellians, density renormalised to 1
  bkw_state             BKW closed-form state for Maxwell molecules
  relaxation_cell       N=32, L=8, hard spheres, bi-Maxwellian T=(2, 1/2, 1/2)
  shock_initial         256 cells on [0,1], N=24, L=7, gas at rest, T=1
  uneven_batch          1024 cells, N drawn from {16, 24, 32} with weights
                        0.5/0.3/0.2, perturbed Maxwellians
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED = 1211

# mesh half-width per velocity resolution used by the uneven batch
DOMAIN_FOR_N = {16: 6.0, 24: 7.0, 32: 8.0}


def velocity_mesh(N: int, L: float) -> np.ndarray:
    """1-D velocity nodes v_k = (2L/N)(k - N/2), k = 0..N-1 (Sec. 3.1)."""
    return (2.0 * L / N) * (np.arange(N) - N // 2)


def _v3(N: int, L: float):
    v = velocity_mesh(N, L)
    return np.meshgrid(v, v, v, indexing="ij")


def maxwellian(N: int, L: float, rho: float, u, T: float) -> np.ndarray:
    """rho (2 pi T)^{-3/2} exp(-|v-u|^2 / (2T)) on the mesh (R = 1)."""
    V = _v3(N, L)
    r2 = sum((V[d] - u[d]) ** 2 for d in range(3))
    return rho * (2 * np.pi * T) ** -1.5 * np.exp(-r2 / (2 * T))


def bi_maxwellian(N: int, L: float, rho: float, Td) -> np.ndarray:
    V = _v3(N, L)
    e = sum(V[d] ** 2 / (2 * Td[d]) for d in range(3))
    return rho * (2 * np.pi) ** -1.5 * (Td[0] * Td[1] * Td[2]) ** -0.5 * np.exp(-e)


def discrete_mass(f: np.ndarray, L: float) -> float:
    N = f.shape[-1]
    return float(f.sum() * (2.0 * L / N) ** 3)


def single_cell_mixture(N: int = 16, L: float = 6.0) -> np.ndarray:
    """0.5 M(1,(+1,0,0),1) + 0.5 M(1,(-1,0,0),1), divided by its discrete mass."""
    f = 0.5 * maxwellian(N, L, 1.0, (1.0, 0, 0), 1.0) + 0.5 * maxwellian(N, L, 1.0, (-1.0, 0, 0), 1.0)
    return f / discrete_mass(f, L)


def bkw_K(t: float) -> float:
    """BKW scaling K(t) = 1 - exp(-t/6) for Maxwell molecules with b = 1/(4 pi)."""
    return 1.0 - np.exp(-t / 6.0)


def bkw_state(N: int, L: float, t: float) -> np.ndarray:
    """BKW profile (2 pi K)^{-3/2} exp(-|v|^2/2K) [(5K-3)/(2K) + (1-K)|v|^2/(2K^2)]."""
    K = bkw_K(t)
    V = _v3(N, L)
    r2 = V[0] ** 2 + V[1] ** 2 + V[2] ** 2
    return (2 * np.pi * K) ** -1.5 * np.exp(-r2 / (2 * K)) * ((5 * K - 3) / (2 * K) + (1 - K) * r2 / (2 * K * K))


def relaxation_cell(N: int = 32, L: float = 8.0, Td=(2.0, 0.5, 0.5)) -> np.ndarray:
    f = bi_maxwellian(N, L, 1.0, Td)
    return f / discrete_mass(f, L)


def shock_initial(n_cells: int = 256, N: int = 24, L: float = 7.0) -> np.ndarray:
    """Gas at rest, rho = 1, T = 1, in every cell: array (n_cells, N, N, N)."""
    m = maxwellian(N, L, 1.0, (0.0, 0.0, 0.0), 1.0)
    return np.broadcast_to(m, (n_cells, N, N, N)).copy()


def wall_refined_widths(eps: float = 1.0, length: float = 30.0, wall_per_mfp: int = 8, inner_per_mfp: int = 2,
                        wall_mfp: float = 1.0, ratio: float = 1.1) -> np.ndarray:
    """Cell widths of the sudden-heating run of Sec. 5, wall first: eight cells per mean free
    path next to the wall, two in the interior.  The mean free path is taken as eps (the
    scaled Knudsen number is its ratio to the unit length).  Cells of width eps/wall_per_mfp
    fill the first wall_mfp mean free paths, then each cell is `ratio` times wider than the
    last up to eps/inner_per_mfp, which fills the rest of [0, length]; what is left at the
    far end (less than one interior cell) is added to the last cell.  Geometry only: the
    widths are input data."""
    wmin, wmax = eps / wall_per_mfp, eps / inner_per_mfp
    w = [wmin] * max(1, int(round(wall_mfp * wall_per_mfp)))
    while len(w) > 1 and sum(w) > length:
        w.pop()
    while w[-1] * ratio < wmax and sum(w) + w[-1] * ratio <= length:
        w.append(w[-1] * ratio)
    while sum(w) + wmax <= length:
        w.append(wmax)
    w[-1] += length - sum(w)
    return np.array(w)


def perturbed_maxwellian(rng: np.random.Generator, N: int, L: float, rho: float, u, T: float,
                         amp: float = 0.1, modes: int = 6) -> np.ndarray:
    """M (1 + amp p) with a smooth random p, scaled so that ||M p||_2 = ||M||_2 on the mesh."""
    V = _v3(N, L)
    M = maxwellian(N, L, rho, u, T)
    for _ in range(100):
        a = rng.standard_normal(modes)
        kap = rng.uniform(-0.8, 0.8, size=(modes, 3))
        phi = rng.uniform(0.0, 2 * np.pi, size=modes)
        p = np.zeros_like(M)
        for i in range(modes):
            arg = sum(kap[i, d] * (V[d] - u[d]) for d in range(3)) / np.sqrt(T) + phi[i]
            p += a[i] * np.cos(arg)
        p *= np.linalg.norm(M) / max(np.linalg.norm(M * p), 1e-300)
        f = M * (1.0 + amp * p)
        if np.all(f > 0):
            return f
    raise RuntimeError("could not draw a positive perturbation")


@dataclass
class Batch:
    Ns: np.ndarray          # velocity resolution per cell
    Ls: np.ndarray          # mesh half-width per cell
    cells: list             # list of (N, N, N) float64 arrays


def uneven_batch(n_cells: int = 1024, seed: int = SEED, weights=(0.5, 0.3, 0.2),
                 only_N: int | None = None) -> Batch:
    """1024 cells with N ~ Cat{16, 24, 32}, rho ~ U[.5, 2], |u| ~ U[0, 1.5] in a
    random direction, T ~ U[.5, 2], plus a smooth perturbation of relative size 0.1.
    With only_N, the cells of the same draw whose N equals only_N are returned."""
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.array([16, 24, 32]), size=n_cells, p=np.array(weights))
    cells, out_N = [], []
    for N in Ns:
        N = int(N)
        L = DOMAIN_FOR_N[N]
        rho = rng.uniform(0.5, 2.0)
        g = rng.standard_normal(3)
        u = rng.uniform(0.0, 1.5) * g / np.linalg.norm(g)
        T = rng.uniform(0.5, 2.0)
        f = perturbed_maxwellian(rng, N, L, rho, u, T)
        if only_N is None or N == only_N:
            cells.append(f)
            out_N.append(N)
    out_N = np.array(out_N, dtype=np.int32)
    return Batch(Ns=out_N, Ls=np.array([DOMAIN_FOR_N[int(n)] for n in out_N]), cells=cells)


def random_smooth_cells(n: int, N: int, L: float, seed: int = SEED, umax: float = 1.5,
                        Trange=(0.5, 2.0)) -> np.ndarray:
    """n perturbed Maxwellians on one mesh (parameters drawn as in uneven_batch)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n, N, N, N))
    for c in range(n):
        rho = rng.uniform(0.5, 2.0)
        g = rng.standard_normal(3)
        u = rng.uniform(0.0, umax) * g / np.linalg.norm(g)
        T = rng.uniform(*Trange)
        out[c] = perturbed_maxwellian(rng, N, L, rho, u, T)
    return out

"""The sudden wall-heating run of Sec. 5 through the library's C ABI.

Gas at rest (rho = 1, T = 1) fills [0, length]; at t = 0 the diffuse wall at
x = 0 is heated to T_wall and a far field at rest holds the other end.  The
scaled Knudsen number is eps = 1 as in the paper's run; the cells are eps/8
wide at the wall and eps/2 inside (two points per mean free path in the
interior, eight at the wall; workloads.wall_refined_widths).  Each step is the
Strang step T(dt/2) C(dt) T(dt/2) of Sec. 3.1 with dt = cfl * min dx / L.
The recorded quantities are those of the paper's figures: the bulk velocity
u1(x) of every cell and the v1 marginal of the cell at the wall.

Orchestration only: every step and every diagnostic runs in the library.
"""
from __future__ import annotations

import numpy as np

from . import bz
from . import workloads as W


class SuddenHeating:
    def __init__(self, N: int = 24, L: float = 7.0, lam: float = 1.0, eps: float = 1.0, length: float = 30.0,
                 T_wall: float = 2.0, mode: str = "batched_f32", cfl: float = 0.5, device: str = "cuda",
                 weights_cache=None):
        import torch
        self.N, self.L, self.eps = N, L, eps
        self.widths = W.wall_refined_widths(eps=eps, length=length)
        self.nx = len(self.widths)
        self.x = np.cumsum(self.widths) - 0.5 * self.widths
        self.col = bz.Collision([(N, L, lam)], [0] * self.nx, mode, weights_cache=weights_cache, device=device)
        self.transport = bz.bz_transport_create_ex(self.col.grids[0], self.widths, T_wall, 1.0, 0.0, 1.0)
        self.f = torch.from_numpy(W.shock_initial(self.nx, N, L).ravel().copy()).to(device)
        self.dt = cfl * float(self.widths.min()) / L
        self.time = 0.0
        self._mom = torch.zeros(5 * self.nx, dtype=torch.float64, device=device)
        self._marg = torch.zeros(N, dtype=torch.float64, device=device)

    def step(self, n: int = 1):
        for _ in range(n):
            self.col.strang_step(self.transport, self.dt, self.eps, self.f)
            self.time += self.dt

    def diagnostics(self) -> dict:
        """Density, bulk velocity and temperature per cell, and the wall cell's v1 marginal."""
        bz.bz_cell_moments(self.col.batch, self.f, self._mom)
        bz.bz_marginal_v1(self.col.batch, self.f, 0, self._marg)
        m = self._mom.cpu().numpy().reshape(self.nx, 5)
        return {"t": self.time, "x": self.x, "rho": m[:, 0], "u1": m[:, 1], "T": m[:, 4],
                "wall_marginal_v1": self._marg.cpu().numpy(), "v1": W.velocity_mesh(self.N, self.L)}

    def mass(self) -> float:
        """sum_j dx_j sum_k f dv^3."""
        d = self.diagnostics()
        return float((d["rho"] * self.widths).sum())

    def close(self):
        if getattr(self, "transport", None):
            bz.bz_transport_free(self.transport)
            self.transport = None
        if getattr(self, "col", None):
            self.col.close()
            self.col = None

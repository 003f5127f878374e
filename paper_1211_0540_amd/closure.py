"""Training and serving driver of the gated learned closure.

Only the host loop lives here; every computation (collision operator,
transport, gate, network forward/backward, Adam) is a libbz kernel reached
through the C ABI.  torch tensors hold the device arrays, and torch indexing
gathers the rows of a minibatch from the training set.

Training data (on the N=24, L=7 mesh the network serves):
  * snapshots of the wall-heating shock problem (256 cells, diffuse wall at
    T=2, Knudsen number 0.1, batched FP32 collisions), and
  * snapshots of space-homogeneous relaxations from perturbed Maxwellians,
keeping the cells whose deviation d = |f - M| / |M| is below `keep` (twice
the serving gate by default) and above D_MIN.  The input is the direction of
f - M scaled to unit RMS with the amplitude d / s_in in its corner entry
(s_in = AMPLITUDE_SCALE); the target is the projected collision operator
divided by rho |f - M| s_out, s_out a power of two fixed from a first batch.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import bz
from . import workloads as W


def _pow2(x: float) -> float:
    return 2.0 ** round(math.log2(x)) if x > 0 else 1.0


# deviation mapped to 1 on the amplitude entry of the network input (the serving gate)
AMPLITUDE_SCALE = 0.05
# cells closer to equilibrium are not harvested: their f - M is at the level of the
# transport's rounding and their Q is the discretisation residual of Q(M, M), which
# does not scale with f - M; the closure serves them with a Q_s that vanishes with f - M
D_MIN = 1e-6


class ClosureModel:
    def __init__(self, N=24, L=7.0, lam=1.0, hidden=1024, seed=1211, device="cuda"):
        self.N, self.L, self.lam, self.H = N, float(L), float(lam), hidden
        self.M = N ** 3
        self.dev = torch.device(device)
        self.net = bz.bz_mlp_create(self.M, hidden, self.M)
        self.params = torch.zeros(bz.bz_mlp_param_bytes(self.net), dtype=torch.uint8, device=self.dev)
        rng = np.random.default_rng(seed)
        parts = []
        for o, i in ((hidden, self.M), (hidden, hidden), (self.M, hidden)):
            s = 1.0 / math.sqrt(i)
            parts += [rng.uniform(-s, s, (o, i)).astype(np.float32).ravel(),
                      rng.uniform(-s, s, o).astype(np.float32)]
        # start the output layer at zero so the untrained closure predicts Q = 0
        parts[4][:] = 0.0
        parts[5][:] = 0.0
        bz.bz_mlp_set_params(self.net, self.params, np.concatenate(parts))
        self.s_in = self.s_out = None
        self.xs, self.ys = [], []
        self.step = 0
        self.history = []
        self.val_idx = torch.zeros(0, dtype=torch.long)
        self.wcache = {}

    # ----------------------------------------------------------------- data
    def _harvest_batch(self, col, f, keep, state, x, q, y):
        """Append (x, y) rows of the cells of `col` whose deviation is below keep."""
        bz.bz_closure_prepare(col.batch, f, 1e30, self.s_in, state, x)
        col.collide(f, out=q)
        col.project(q)
        bz.bz_closure_targets(col.batch, state, q, self.s_out, y)
        d = state.view(-1, 10)[:, 5]
        sel = torch.nonzero((d < keep) & (d > D_MIN)).flatten()
        if sel.numel():
            self.xs.append(x.view(-1, self.M)[sel].clone())
            self.ys.append(y.view(-1, self.M)[sel].clone())
        return int(sel.numel())

    def _scales(self, col, f, keep=0.1):
        n = len(col.grid_of_cell)
        state = torch.zeros(n * 10, dtype=torch.float64, device=self.dev)
        x = torch.zeros(n * self.M, dtype=torch.int16, device=self.dev)
        q = torch.zeros(col.elems, dtype=torch.float64, device=self.dev)
        y = torch.zeros(n * self.M, dtype=torch.float32, device=self.dev)
        self.s_in = AMPLITUDE_SCALE
        bz.bz_closure_prepare(col.batch, f, 1e30, self.s_in, state, x)
        col.collide(f, out=q)
        col.project(q)
        bz.bz_closure_targets(col.batch, state, q, 1.0, y)
        d = state.view(-1, 10)[:, 5]
        sel = torch.nonzero((d < keep) & (d > D_MIN)).flatten()
        rows = y.view(n, self.M)[sel] if sel.numel() else y.view(n, self.M)
        self.s_out = _pow2(float(rows.pow(2).mean().sqrt()))

    def harvest_shock(self, snapshots=600, every=1, nx=256, eps=0.1, T_wall=2.0, keep=0.1):
        N, L = self.N, self.L
        col = bz.Collision([(N, L, self.lam)], [0] * nx, "batched_f32", weights_cache=self.wcache)
        t = bz.bz_transport_create(col.grids[0], nx, 1.0, T_wall, 1.0, 0.0, 1.0)
        f = torch.from_numpy(W.shock_initial(nx, N, L).ravel().copy()).to(self.dev)
        dt = 0.5 * (1.0 / nx) / L
        # the first steps only are near-uniform: take the scales after a few steps
        for _ in range(5):
            col.strang_step(t, dt, eps, f)
        if self.s_in is None:
            self._scales(col, f)
        state = torch.zeros(nx * 10, dtype=torch.float64, device=self.dev)
        x = torch.zeros(nx * self.M, dtype=torch.int16, device=self.dev)
        q = torch.zeros(col.elems, dtype=torch.float64, device=self.dev)
        y = torch.zeros(nx * self.M, dtype=torch.float32, device=self.dev)
        kept = 0
        for s in range(snapshots * every):
            col.strang_step(t, dt, eps, f)
            if s % every == 0:
                kept += self._harvest_batch(col, f, keep, state, x, q, y)
        col.check()
        bz.bz_transport_free(t)
        col.close()
        return kept

    def harvest_relaxation(self, cells=256, steps=20, dt=0.05, amp=0.3, seed=7, keep=0.1):
        N, L = self.N, self.L
        rng = np.random.default_rng(seed)
        init = np.empty((cells, N, N, N))
        for c in range(cells):
            rho = rng.uniform(0.5, 2.0)
            g = rng.standard_normal(3)
            u = rng.uniform(0.0, 1.2) * g / np.linalg.norm(g)
            T = rng.uniform(0.6, 1.8)
            init[c] = W.perturbed_maxwellian(rng, N, L, rho, u, T, amp=amp * rng.uniform(0.05, 1.0))
        col = bz.Collision([(N, L, self.lam)], [0] * cells, "batched_f32", weights_cache=self.wcache)
        f = torch.from_numpy(col.pack(list(init))).to(self.dev)
        if self.s_in is None:
            self._scales(col, f)
        state = torch.zeros(cells * 10, dtype=torch.float64, device=self.dev)
        x = torch.zeros(cells * self.M, dtype=torch.int16, device=self.dev)
        q = torch.zeros(col.elems, dtype=torch.float64, device=self.dev)
        y = torch.zeros(cells * self.M, dtype=torch.float32, device=self.dev)
        kept = 0
        for _ in range(steps):
            kept += self._harvest_batch(col, f, keep, state, x, q, y)
            col.step(f, dt)
        col.check()
        col.close()
        return kept

    def dataset_size(self):
        return sum(int(a.shape[0]) for a in self.xs)

    # ---------------------------------------------------------------- train
    def fit(self, steps=1000, batch=256, lr=1e-3, seed=0, lr_min_frac=0.05, holdout=0.1):
        """Adam on the MSE of the normalised targets, cosine learning-rate decay.  A
        random `holdout` fraction of the rows is kept out of training for
        `validation_error`."""
        X = torch.cat(self.xs) if len(self.xs) > 1 else self.xs[0]
        Y = torch.cat(self.ys) if len(self.ys) > 1 else self.ys[0]
        self.xs, self.ys = [X], [Y]
        gen = torch.Generator(device="cpu").manual_seed(seed)
        order = torch.randperm(X.shape[0], generator=gen)
        nval = int(X.shape[0] * holdout) if holdout > 0 else 0
        self.val_idx = order[:nval].to(self.dev)
        train_idx = order[nval:]
        S = train_idx.numel()
        batch = max(32, min(batch, (S // 32) * 32))
        work = torch.zeros(bz.bz_mlp_workspace_bytes(self.net, batch), dtype=torch.uint8, device=self.dev)
        grad = torch.zeros(bz.bz_mlp_param_count(self.net), dtype=torch.float32, device=self.dev)
        loss = torch.zeros(1, dtype=torch.float32, device=self.dev)
        perm = torch.randperm(S, generator=gen)
        pos = 0
        for i in range(steps):
            if pos + batch > S:
                perm = torch.randperm(S, generator=gen)
                pos = 0
            idx = train_idx[perm[pos:pos + batch]].to(self.dev)
            pos += batch
            xb = X[idx].contiguous()
            yb = Y[idx].contiguous()
            # cosine decay of the learning rate
            lr_i = lr * (lr_min_frac + (1 - lr_min_frac) * 0.5 * (1 + math.cos(math.pi * i / max(steps, 1))))
            bz.bz_mlp_backward(self.net, self.params, xb, yb, batch, grad, loss, work)
            self.step += 1
            bz.bz_mlp_adam(self.net, self.params, grad, self.step, lr_i)
            if i % 50 == 0 or i == steps - 1:
                self.history.append((self.step, float(loss.item())))
        return self.history

    def validation_error(self, rows=4096):
        """Relative L2 error of the network on up to `rows` held-out rows (kept out of
        training by `fit`): (overall |Yhat - Y| / |Y|, median over rows of the per-row
        relative error)."""
        idx = self.val_idx[:rows]
        n_all = idx.numel()
        if n_all == 0:
            raise RuntimeError("no held-out rows: fit with holdout > 0")
        num = den = 0.0
        per_row = []
        for a in range(0, n_all, 1024):
            X = self.xs[0][idx[a:a + 1024]].contiguous()
            Y = self.ys[0][idx[a:a + 1024]]
            n = X.shape[0]
            work = torch.zeros(bz.bz_mlp_workspace_bytes(self.net, n), dtype=torch.uint8, device=self.dev)
            out = torch.zeros(n, self.M, dtype=torch.float32, device=self.dev)
            bz.bz_mlp_forward(self.net, self.params, X, n, out, work)
            d, r = (out - Y).norm(dim=1), Y.norm(dim=1)
            num += float((d ** 2).sum())
            den += float((r ** 2).sum())
            per_row.append((d / r).cpu())
        return math.sqrt(num / den), float(torch.cat(per_row).median())

    def desc(self, gate=0.05, judge_every=16, judge_tol=1e-2, judge_floor=1e-3):
        return bz.closure_desc(self.net, self.params, gate, self.s_in, self.s_out, judge_every, judge_tol,
                               judge_floor)

    def release_data(self):
        self.xs, self.ys = [], []
        torch.cuda.empty_cache()

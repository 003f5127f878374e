"""Parity of the HIP collision path with the FP64 oracle (GPU, through the C ABI).

Bars (the tolerances are derived in the design notes):
  FP64 paths       max |Q_gpu - Q_oracle| <= 1e-12 max |Q_oracle|
  FP32 batched     per-cell relative L2 of the projected Q <= 1e-5 against the
                   oracle, on every input (the low-frequency pairs are summed in
                   FP64 by the core kernel); without the core (BZ_CORE_OFF) the
                   bound is 8 u32 kappa, kappa = ||sum |terms| || / ||Qhat||.
  conservation     |sum_j w phi_j Q_j| <= 1e-12 sum_j w |phi_j Q_j| per invariant
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1211_0540_amd import bz
from paper_1211_0540_amd import workloads as W

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    bz.lib()
    return torch.device("cuda:0")


_ORACLES = {}


def oracle_for(N, L, lam):
    key = (N, float(L), float(lam))
    if key not in _ORACLES:
        _ORACLES[key] = O.Oracle(N, L, lam)
    return _ORACLES[key]


_WCACHE = {}


TOL32 = 1e-5


def run(meshes, goc, cells, mode, dev, project=True, schedule="symmetric", fine_split=False):
    c = bz.Collision(meshes, goc, mode, weights_cache=_WCACHE, schedule=schedule, fine_split=fine_split)
    f = torch.from_numpy(c.pack(cells)).to(dev)
    qt = c.collide(f)
    q = qt.clone()
    if project:
        c.project(q)
    torch.cuda.synchronize()
    out = (c.unpack(qt.cpu().numpy()), c.unpack(q.cpu().numpy()))
    c.close()
    return out


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def constraints(N, L):
    v, _, dv, _ = O.grid(N, L)
    V = np.meshgrid(v, v, v, indexing="ij")
    rows = [np.ones_like(V[0]), V[0], V[1], V[2], V[0] ** 2 + V[1] ** 2 + V[2] ** 2]
    return [r * dv ** 3 for r in rows]


def assert_conserved(q, N, L, tol=1e-12):
    for c in constraints(N, L):
        assert abs((c * q).sum()) <= tol * np.abs(c * q).sum()


# ---------------------------------------------------------------------------
# FP64 paths: the plain baseline and the batched FP64 schedule
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["plain_f64", "batched_f64"])
def test_mixture_cell_fp64(dev, mode):
    """One Maxwell-molecule cell on N=16, L=6 (two counter-streaming Maxwellians)."""
    N, L, lam = 16, 6.0, 0.0
    f = W.single_cell_mixture(N, L)
    qt_o, q_o, _, _ = oracle_for(N, L, lam).collide(f)
    (qt,), (q,) = run([(N, L, lam)], [0], [f], mode, dev)
    assert max_rel(qt, qt_o) < 1e-12
    assert max_rel(q, q_o) < 1e-12
    assert_conserved(q, N, L)


@pytest.mark.parametrize("mode,schedule", [("plain_f64", "full"), ("batched_f64", "symmetric"),
                                           ("batched_f64", "full")])
def test_ragged_batch_fp64_hard_spheres(dev, mode, schedule):
    """70 cells on N=12 (one full wavefront group and a ragged tail of 6)."""
    N, L, lam = 12, 5.0, 1.0
    n = 70 if mode == "batched_f64" else 5
    cells = list(W.random_smooth_cells(n, N, L, seed=3, umax=0.7))
    qts, qs = run([(N, L, lam)], [0] * n, cells, mode, dev, schedule=schedule)
    o = oracle_for(N, L, lam)
    for i in range(n):
        qt_o, q_o, _, _ = o.collide(cells[i])
        assert max_rel(qts[i], qt_o) < 1e-12, i
        assert max_rel(qs[i], q_o) < 1e-12, i


# ---------------------------------------------------------------------------
# FP32 batched path with compensated accumulation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("schedule", ["symmetric", "full"])
def test_mixture_cell_fp32_batched(dev, schedule):
    N, L, lam = 16, 6.0, 0.0
    f = W.single_cell_mixture(N, L)
    _, q_o, _, _ = oracle_for(N, L, lam).collide(f)
    _, (q,) = run([(N, L, lam)], [0], [f], "batched_f32", dev, schedule=schedule)
    assert rel_l2(q, q_o) < 1e-5
    assert_conserved(q, N, L)


@pytest.mark.parametrize("mode", ["batched_f32", "plain_f32"])
def test_relaxation_cell_n32(dev, mode):
    """The N=32, L=8 hard-sphere bi-Maxwellian (T = 2, 1/2, 1/2) of the relaxation problem."""
    N, L, lam = 32, 8.0, 1.0
    f = W.relaxation_cell(N, L)
    _, q_o, _, _ = oracle_for(N, L, lam).collide(f)
    _, (q,) = run([(N, L, lam)], [0], [f], mode, dev)
    assert rel_l2(q, q_o) < 1e-5
    assert_conserved(q, N, L)


def test_relaxation_cell_n32_fp64_plain(dev):
    N, L, lam = 32, 8.0, 1.0
    f = W.relaxation_cell(N, L)
    qt_o, q_o, _, _ = oracle_for(N, L, lam).collide(f)
    (qt,), (q,) = run([(N, L, lam)], [0], [f], "plain_f64", dev)
    assert max_rel(qt, qt_o) < 1e-12
    assert max_rel(q, q_o) < 1e-12


@pytest.mark.parametrize("N,L,n", [(8, 4.0, 3), (12, 5.0, 70), (16, 6.0, 65), (20, 6.0, 2), (24, 7.0, 2),
                                   (28, 7.0, 1), (32, 8.0, 2)])
def test_symmetric_schedule_equals_full_sum_fp64(dev, N, L, n):
    """The conjugate-symmetric schedule (half the rows, edge passes, mirrored assembly)
    gives the full FP64 sum to rounding, for every cell and output, on several meshes and
    ragged groups; sampled cells also against the oracle."""
    lam = 1.0
    cells = list(W.random_smooth_cells(n, N, L, seed=N, umax=1.0))
    full, _ = run([(N, L, lam)], [0] * n, cells, "batched_f64", dev, project=False, schedule="full")
    sym, _ = run([(N, L, lam)], [0] * n, cells, "batched_f64", dev, project=False, schedule="symmetric")
    for i in range(n):
        assert max_rel(sym[i], full[i]) < 1e-12, i
    o = oracle_for(N, L, lam)
    for i in sorted({0, n // 2, n - 1}):
        qt_o, _, _, _ = o.collide(cells[i])
        assert max_rel(sym[i], qt_o) < 1e-12, i


@pytest.mark.parametrize("schedule,N,L,n", [("symmetric", 24, 7.0, 130), ("full", 24, 7.0, 130),
                                             ("symmetric", 8, 4.0, 1)])
def test_fine_split_equals_default_split_fp64(dev, schedule, N, L, n):
    """BZ_BATCH_FINE_SPLIT (rows cut into up to 6 partial sums for one group alone) gives the
    default split's FP64 sums to rounding: 130 N=24 cells in three groups, the last ragged, and
    a single N=8 cell."""
    lam = 1.0
    cells = list(W.random_smooth_cells(n, N, L, seed=41, umax=1.0))
    a, _ = run([(N, L, lam)], [0] * n, cells, "batched_f64", dev, project=False, schedule=schedule)
    b, _ = run([(N, L, lam)], [0] * n, cells, "batched_f64", dev, project=False, schedule=schedule,
               fine_split=True)
    for i in range(n):
        assert max_rel(b[i], a[i]) < 1e-12, i


def test_symmetric_schedule_fp32_mixed_meshes(dev):
    """FP32, two meshes in one batch (N=16 ragged, N=24): both schedules against the oracle."""
    meshes = [(16, 6.0, 1.0), (24, 7.0, 1.0)]
    c16 = list(W.random_smooth_cells(67, 16, 6.0, seed=4, umax=1.2))
    c24 = list(W.random_smooth_cells(3, 24, 7.0, seed=5, umax=1.2))
    cells, goc = c16 + c24, [0] * 67 + [1] * 3
    _, q_full = run(meshes, goc, cells, "batched_f32", dev, schedule="full")
    _, q_sym = run(meshes, goc, cells, "batched_f32", dev, schedule="symmetric")
    for i in (0, 40, 64, 66, 67, 69):
        N, L = (16, 6.0) if i < 67 else (24, 7.0)
        _, q_o, _, _ = oracle_for(N, L, 1.0).collide(cells[i])
        assert rel_l2(q_sym[i], q_o) < TOL32, i
        assert rel_l2(q_full[i], q_o) < TOL32, i
        assert_conserved(q_sym[i], N, L)


def _kappa(f, N, L, lam):
    return oracle_for(N, L, lam).kappa(f)


def test_uneven_mixed_mesh_batch_fp32(dev):
    """A 96-cell sample of the 1024-cell uneven draw (N in {16, 24, 32}) in one batch."""
    full = W.uneven_batch(n_cells=96)
    meshes = [(16, 6.0, 1.0), (24, 7.0, 1.0), (32, 8.0, 1.0)]
    idx = {16: 0, 24: 1, 32: 2}
    goc = [idx[int(n)] for n in full.Ns]
    _, qs = run(meshes, goc, full.cells, "batched_f32", dev)
    errs = []
    for i in range(len(full.cells)):
        N = int(full.Ns[i])
        L = W.DOMAIN_FOR_N[N]
        _, q_o, _, _ = oracle_for(N, L, 1.0).collide(full.cells[i])
        e = rel_l2(qs[i], q_o)
        errs.append(e)
        assert e < TOL32, (i, N, e)
        assert_conserved(qs[i], N, L)
    print("uneven batch FP32 rel L2: median %.2e max %.2e" % (np.median(errs), np.max(errs)))


def test_uneven_batch_full_size_sampled(dev):
    """The whole 1024-cell uneven draw in one batch, as the benchmark runs it: the first and
    last cell of each mesh against the oracle, conservation for every cell."""
    full = W.uneven_batch(n_cells=1024)
    meshes = [(16, 6.0, 1.0), (24, 7.0, 1.0), (32, 8.0, 1.0)]
    idx = {16: 0, 24: 1, 32: 2}
    goc = [idx[int(n)] for n in full.Ns]
    _, qs = run(meshes, goc, full.cells, "batched_f32", dev)
    for N in (16, 24, 32):
        members = [i for i in range(len(goc)) if int(full.Ns[i]) == N]
        L = W.DOMAIN_FOR_N[N]
        for i in (members[0], members[-1]):
            _, q_o, _, _ = oracle_for(N, L, 1.0).collide(full.cells[i])
            assert rel_l2(qs[i], q_o) < TOL32, (i, N)
    for i in range(len(goc)):
        N = int(full.Ns[i])
        assert_conserved(qs[i], N, W.DOMAIN_FOR_N[N])


def test_shock_cells_fp32_full_size(dev):
    """All 256 cells of the N=24, L=7 shock problem in one launch; 8 sampled against the oracle."""
    N, L, lam = 24, 7.0, 1.0
    cells = list(W.random_smooth_cells(256, N, L, seed=5, umax=1.0))
    _, qs = run([(N, L, lam)], [0] * 256, cells, "batched_f32", dev)
    o = oracle_for(N, L, lam)
    for i in np.random.default_rng(0).choice(256, 8, replace=False):
        _, q_o, _, _ = o.collide(cells[i])
        assert rel_l2(qs[i], q_o) < TOL32, i


def test_bench_workload_n32_full_batch(dev):
    """The benchmark's launch: the 190 N=32 cells of the 1024-cell uneven draw in one
    batched FP32 launch (default schedule and core, autotuned variant).  Every cell against
    the oracle at the flat 1e-5; conservation everywhere."""
    N, L, lam = 32, 8.0, 1.0
    batch = W.uneven_batch(n_cells=1024, only_N=32)
    cells, n = batch.cells, len(batch.cells)
    assert n == 190
    c = bz.Collision([(N, L, lam)], [0] * n, "batched_f32", weights_cache=_WCACHE)
    f = torch.from_numpy(c.pack(cells)).to(dev)
    c.autotune(f, reps=1)
    q32 = c.unpack(c.project(c.collide(f)).cpu().numpy())
    c.close()
    o = oracle_for(N, L, lam)
    errs = []
    for i in range(n):
        _, q_o, _, _ = o.collide(cells[i])
        errs.append(rel_l2(q32[i], q_o))
        assert_conserved(q32[i], N, L)
    errs = np.array(errs)
    print("bench workload FP32 vs oracle: median %.2e max %.2e, %.0f%% <= 1e-5"
          % (np.median(errs), errs.max(), 100 * np.mean(errs <= TOL32)))
    assert errs.max() < TOL32, (int(errs.argmax()), errs.max())


def test_core_off_keeps_the_fp32_bound(dev):
    """Without the FP64 core every pair is summed in FP32: the error is then bounded by
    the cancellation of the terms, 8 u32 kappa (kappa from the oracle)."""
    N, L, lam = 24, 7.0, 1.0
    cells = list(W.random_smooth_cells(66, N, L, seed=12, umax=1.2))
    _, qs = run([(N, L, lam, bz.BZ_CORE_OFF)], [0] * 66, cells, "batched_f32", dev)
    o = oracle_for(N, L, lam)
    for i in (0, 31, 64, 65):
        _, q_o, _, _ = o.collide(cells[i])
        assert rel_l2(qs[i], q_o) < max(TOL32, 8 * U32 * _kappa(cells[i], N, L, lam)), i
        assert_conserved(qs[i], N, L)


@pytest.mark.parametrize("N,L,r2", [(24, 7.0, 8), (24, 7.0, 35), (32, 8.0, 80), (16, 6.0, 49), (12, 5.0, 24)])
def test_core_radii_match_oracle(dev, N, L, r2):
    """Other core radii (a small ball, and the largest half-width 8 at N=32, N=16 with a core
    reaching the k_d = 0 outputs): the same sum, FP64 core plus FP32 rest, against the oracle
    at 1e-5 (the small ball removes less of the rounding, so its cells are mixtures)."""
    lam = 1.0
    n = 66
    cells = list(W.random_smooth_cells(n, N, L, seed=r2, umax=1.0))
    if r2 == 8:
        cells = [W.single_cell_mixture(N, L)] * n
    _, qs = run([(N, L, lam, r2)], [0] * n, cells, "batched_f32", dev)
    o = oracle_for(N, L, lam)
    for i in (0, 33, 65):
        _, q_o, _, _ = o.collide(cells[i])
        assert rel_l2(qs[i], q_o) < TOL32, (i, rel_l2(qs[i], q_o))
        assert_conserved(qs[i], N, L)


@pytest.mark.parametrize("mode", ["batched_f64", "batched_f32"])
def test_degenerate_cells_zero_and_maxwellian(dev, mode):
    """Degenerate inputs in one ragged batch: f = 0 gives Q = 0 exactly; an exact discrete
    Maxwellian gives only the discretisation residual, matched to the oracle within the
    rounding bound of its cancellation (kappa ~ 1e4); the neighbouring cells are unaffected."""
    N, L, lam = 16, 6.0, 1.0
    smooth = list(W.random_smooth_cells(3, N, L, seed=6))
    maxw = W.maxwellian(N, L, 1.3, (0.4, -0.2, 0.1), 0.9)
    cells = [np.zeros((N, N, N)), smooth[0], maxw, smooth[1], np.zeros((N, N, N)), smooth[2]]
    _, qs = run([(N, L, lam)], [0] * len(cells), cells, mode, dev)
    assert not np.any(qs[0]) and not np.any(qs[4])
    o = oracle_for(N, L, lam)
    u = 2.0 ** -52 if mode == "batched_f64" else U32
    floor = 1e-12 if mode == "batched_f64" else 1e-5
    for i in (1, 2, 3, 5):
        _, q_o, _, _ = o.collide(cells[i])
        kap = _kappa(cells[i], N, L, lam)
        assert rel_l2(qs[i], q_o) < max(floor, 8 * u * kap), (i, kap)
        assert_conserved(qs[i], N, L)


def test_batched_fp32_is_deterministic(dev):
    N, L, lam = 16, 6.0, 1.0
    cells = list(W.random_smooth_cells(80, N, L, seed=9))
    a, _ = run([(N, L, lam)], [0] * 80, cells, "batched_f32", dev, project=False)
    b, _ = run([(N, L, lam)], [0] * 80, cells, "batched_f32", dev, project=False)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------------------
# Projection and time stepping
# ---------------------------------------------------------------------------
def test_projection_matches_oracle_and_conserves(dev):
    """Every mesh size (N^3 from 512 to 32768 values per cell: one to 32 per thread of the
    projection block, with and without a ragged last round), two cells per mesh."""
    rng = np.random.default_rng(1)
    meshes = [(8, 4.0, 1.0), (12, 5.0, 1.0), (16, 6.0, 1.0), (20, 6.0, 1.0), (24, 7.0, 1.0), (28, 7.0, 1.0),
              (32, 8.0, 1.0)]
    goc = [i for i in range(len(meshes)) for _ in range(2)]
    qt = [rng.standard_normal((meshes[g][0],) * 3) for g in goc]
    c = bz.Collision(meshes, goc, "batched_f32", weights_cache=_WCACHE)
    q = torch.from_numpy(c.pack(qt)).to(dev)
    c.project(q)
    out = c.unpack(q.cpu().numpy())
    for x, ref, g in zip(out, qt, goc):
        N, L, _ = meshes[g]
        assert max_rel(x, O.project(ref, L)) < 1e-12, N
        assert_conserved(x, N, L)
    c.close()


@pytest.mark.parametrize("mode,tol", [("plain_f64", 1e-11), ("batched_f32", 1e-5)])
def test_heun_step_matches_oracle(dev, mode, tol):
    """Three Heun steps of the homogeneous equation, dt = 0.05, eps = 1."""
    N, L, lam = 16, 6.0, 1.0
    f0 = W.relaxation_cell(N, L)
    ref = oracle_for(N, L, lam).rk2(f0, 0.05, 1.0, 3)
    c = bz.Collision([(N, L, lam)], [0], mode, weights_cache=_WCACHE)
    f = torch.from_numpy(c.pack([f0])).to(dev)
    for _ in range(3):
        c.step(f, 0.05)
    c.check()
    got = c.unpack(f.cpu().numpy())[0]
    assert rel_l2(got - f0, ref - f0) < tol
    c.close()


def test_nonfinite_input_is_reported(dev):
    N, L, lam = 8, 4.0, 1.0
    f0 = W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    f0[3, 3, 3] = np.nan
    c = bz.Collision([(N, L, lam)], [0], "batched_f32", weights_cache=_WCACHE)
    f = torch.from_numpy(c.pack([f0])).to(dev)
    c.step(f, 0.01)
    with pytest.raises(bz.BzError) as e:
        c.check()
    assert e.value.status == bz.BZ_ENONFINITE
    c.check()  # the flag was cleared
    c.close()


def test_step_flags_report_negative_and_nonfinite_values(dev):
    """BZ_FLAG_NEGATIVE after a step whose new f has a value below zero (a Maxwellian with one
    entry set to -1, which one small step cannot lift), none for a step of length zero on a
    Maxwellian (f unchanged and positive; a real step may leave tiny negative values in the far
    tails of a coarse mesh); the flags clear on reading; BZ_FLAG_NONFINITE with a NaN entry,
    and bz_step_check then raises."""
    N, L, lam = 8, 4.0, 1.0
    M = W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    c = bz.Collision([(N, L, lam)], [0, 0], "batched_f32", weights_cache=_WCACHE)
    f = torch.from_numpy(c.pack([M, M])).to(dev)
    c.step(f, 0.0)
    assert bz.bz_step_flags(c.batch, c.work) == 0
    g = M.copy()
    g[4, 4, 4] = -1.0
    f = torch.from_numpy(c.pack([M, g])).to(dev)
    c.step(f, 1e-3)
    assert bz.bz_step_flags(c.batch, c.work) == bz.BZ_FLAG_NEGATIVE
    assert bz.bz_step_flags(c.batch, c.work) == 0
    g[1, 2, 3] = np.nan
    f = torch.from_numpy(c.pack([M, g])).to(dev)
    c.step(f, 1e-3)
    assert bz.bz_step_flags(c.batch, c.work) & bz.BZ_FLAG_NONFINITE
    c.step(f, 1e-3)
    with pytest.raises(bz.BzError) as e:
        c.check()
    assert e.value.status == bz.BZ_ENONFINITE
    c.close()


def test_unbound_weights_and_short_workspace(dev):
    g = bz.bz_grid_init(8, 4.0, 1.0)
    b = bz.bz_batch_create([0], [g], bz.BZ_MODE_BATCHED_F32)
    f = torch.zeros(512, dtype=torch.float64, device=dev)
    q = torch.zeros_like(f)
    work = torch.zeros(bz.bz_workspace_bytes(b), dtype=torch.uint8, device=dev)
    with pytest.raises(bz.BzError) as e:
        bz.bz_collide_batch(b, f, q, work)
    assert e.value.status == bz.BZ_ESTATE
    buf = torch.empty(bz.bz_weights_bytes(g, bz.BZ_W_BATCHED_F32), dtype=torch.uint8, device=dev)
    bz.bz_weights(g, bz.BZ_W_BATCHED_F32, buf)
    with pytest.raises(bz.BzError):
        bz.bz_batch_set_weights(b, 0, bz.BZ_W_PLAIN_F64, buf)
    bz.bz_batch_set_weights(b, 0, bz.BZ_W_BATCHED_F32, buf)
    with pytest.raises(bz.BzError) as e:
        bz.bz_collide_batch(b, f, q, work[:16])
    assert e.value.status == bz.BZ_EINVAL
    bz.bz_collide_batch(b, f, q, work)
    torch.cuda.synchronize()
    bz.bz_batch_free(b)
    bz.bz_grid_free(g)


@pytest.mark.parametrize("variant", range(16))
def test_every_batched_fp32_variant_matches_oracle(dev, variant):
    """Each tuning variant computes the same sums: 70 cells on N=24 (a ragged second group)."""
    N, L, lam = 24, 7.0, 1.0
    cells = list(W.random_smooth_cells(70, N, L, seed=21, umax=1.0))
    c = bz.Collision([(N, L, lam)], [0] * 70, "batched_f32", weights_cache=_WCACHE)
    c.set_variant(variant)
    f = torch.from_numpy(c.pack(cells)).to(dev)
    q = c.collide(f)
    c.project(q)
    got = c.unpack(q.cpu().numpy())
    c.close()
    o = oracle_for(N, L, lam)
    for i in (0, 33, 63, 64, 69):
        _, q_o, _, _ = o.collide(cells[i])
        assert rel_l2(got[i], q_o) < TOL32, (variant, i)


def test_autotune_keeps_results(dev):
    N, L, lam = 16, 6.0, 1.0
    cells = list(W.random_smooth_cells(64, N, L, seed=2))
    c = bz.Collision([(N, L, lam)], [0] * 64, "batched_f32", weights_cache=_WCACHE)
    f = torch.from_numpy(c.pack(cells)).to(dev)
    q0 = c.collide(f).cpu().numpy()
    best = c.autotune(f, reps=1)
    assert 0 <= best[0] < bz.bz_variant_count()
    q1 = c.collide(f).cpu().numpy()
    q2 = c.collide(f).cpu().numpy()
    assert np.array_equal(q1, q2)           # the tuned choice is kept and deterministic
    assert rel_l2(q1, q0) < 2 * TOL32   # variants differ only by FP32 rounding
    c.close()


# ---------------------------------------------------------------------------
# Other collision exponents (text after eq. GHat_calc): variable hard spheres and
# soft potentials, weights from the library's quadrature table
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lam", [0.5, -1.5])
@pytest.mark.parametrize("mode", ["batched_f64", "plain_f64", "batched_f32"])
def test_general_lambda_matches_oracle(dev, lam, mode):
    N, L = 12, 5.0
    n = 2 if mode == "plain_f64" else 66
    cells = list(W.random_smooth_cells(n, N, L, seed=int(10 * lam) + 60, umax=1.0))
    qts, qs = run([(N, L, lam)], [0] * n, cells, mode, dev)
    o = oracle_for(N, L, lam)
    for i in sorted({0, n // 2, n - 1}):
        qt_o, q_o, _, _ = o.collide(cells[i])
        if mode == "batched_f32":
            assert rel_l2(qs[i], q_o) < TOL32, i
        else:
            assert max_rel(qts[i], qt_o) < 1e-12, i
            assert max_rel(qs[i], q_o) < 1e-12, i
        assert_conserved(qs[i], N, L)


def test_general_lambda_shock_mesh_fp64(dev):
    """lambda = 0.5 on the N=24, L=7 mesh of the shock problem, batched FP64."""
    N, L, lam = 24, 7.0, 0.5
    cells = list(W.random_smooth_cells(3, N, L, seed=61, umax=1.0))
    qts, _ = run([(N, L, lam)], [0] * 3, cells, "batched_f64", dev)
    o = oracle_for(N, L, lam)
    for i in range(3):
        qt_o, _, _, _ = o.collide(cells[i])
        assert max_rel(qts[i], qt_o) < 1e-12, i


# ---------------------------------------------------------------------------
# Inelastic collisions (beta < 1 in eq. GHat_calc; mass and momentum projection)
# ---------------------------------------------------------------------------
_INEL = {}


@pytest.mark.parametrize("lam", [0.0, 1.0])
@pytest.mark.parametrize("mode", ["batched_f64", "plain_f64", "batched_f32"])
def test_inelastic_matches_oracle(dev, lam, mode):
    N, L, beta = 12, 5.0, 0.8
    n = 2 if mode == "plain_f64" else 66
    cells = list(W.random_smooth_cells(n, N, L, seed=70 + int(lam), umax=1.0))
    qts, qs = run([(N, L, lam, bz.BZ_CORE_DEFAULT, beta)], [0] * n, cells, mode, dev)
    key = (N, L, lam, beta)
    if key not in _INEL:
        _INEL[key] = O.InelasticOracle(N, L, lam, beta)
    o = _INEL[key]
    C = constraints(N, L)
    for i in sorted({0, n // 2, n - 1}):
        qt_o, q_o = o.collide(cells[i])
        if mode == "batched_f32":
            assert rel_l2(qs[i], q_o) < TOL32, i
        else:
            assert max_rel(qts[i], qt_o) < 1e-12, i
            assert max_rel(qs[i], q_o) < 1e-12, i
        for a in range(4):   # mass and momentum, not energy
            assert abs((C[a] * qs[i]).sum()) <= 1e-12 * np.abs(C[a] * qs[i]).sum()
        assert abs((C[4] * qs[i]).sum()) > 1e-6 * np.abs(C[4] * qs[i]).sum()


# ---------------------------------------------------------------------------
# One convolution launch for cells on several meshes
# ---------------------------------------------------------------------------
def test_one_launch_for_several_meshes_equals_per_mesh_launches(dev):
    """The default batched FP32 batch on three meshes issues one convolution launch whose queue
    holds the items of every mesh; with the per-mesh launches set to the same accumulation
    variant the results are bitwise equal (each item's arithmetic does not depend on the
    queue), and both match the oracle."""
    meshes = [(16, 6.0, 1.0), (24, 7.0, 1.0), (32, 8.0, 1.0)]
    cells = (list(W.random_smooth_cells(70, 16, 6.0, seed=80)) + list(W.random_smooth_cells(3, 24, 7.0, seed=81))
             + list(W.random_smooth_cells(2, 32, 8.0, seed=82)))
    goc = [0] * 70 + [1] * 3 + [2] * 2
    merged = bz.Collision(meshes, goc, "batched_f32", weights_cache=_WCACHE)
    per = bz.Collision(meshes, goc, "batched_f32", weights_cache=_WCACHE, per_mesh=True)
    per.set_variant(12)
    f = torch.from_numpy(merged.pack(cells)).to(dev)
    bz.bz_batch_timer(merged.batch, True)
    qa = merged.collide(f)
    torch.cuda.synchronize()
    _, launches = bz.bz_batch_timer_read(merged.batch)
    assert launches == 1
    qb = per.collide(f)
    torch.cuda.synchronize()
    assert torch.equal(qa, qb)
    q = merged.unpack(merged.project(qa).cpu().numpy())
    for i in (0, 69, 70, 72, 74):
        N = meshes[goc[i]][0]
        L = meshes[goc[i]][1]
        _, q_o, _, _ = oracle_for(N, L, 1.0).collide(cells[i])
        assert rel_l2(q[i], q_o) < TOL32, i
    merged.close()
    per.close()


@pytest.mark.parametrize("meshes,counts,one", [
    ([(8, 4.0, 1.0), (12, 5.0, 1.0), (20, 6.0, 1.0), (28, 7.0, 1.0)], [3, 66, 2, 1], True),
    ([(8, 4.0, 1.0), (12, 5.0, 1.0), (16, 6.0, 1.0), (20, 6.0, 1.0), (24, 7.0, 1.0)], [2, 2, 65, 1, 1], False)])
def test_one_launch_covers_every_mesh_size(dev, meshes, counts, one):
    """FP32 with the default FP64 cores on the mesh sizes the other tests leave out of the one
    launch (N = 8, 12, 20, 28: four meshes, the most one launch takes, ragged groups), and a
    five-mesh batch, which falls back to one launch per mesh: sampled cells against the
    oracle at 1e-5, conservation after projection."""
    cells, goc = [], []
    for gi, ((N, L, lam), k) in enumerate(zip(meshes, counts)):
        cells += list(W.random_smooth_cells(k, N, L, seed=60 + N))
        goc += [gi] * k
    c = bz.Collision(meshes, goc, "batched_f32", weights_cache=_WCACHE)
    assert bz.bz_batch_one_launch(c.batch) == one
    f = torch.from_numpy(c.pack(cells)).to(dev)
    q = c.unpack(c.project(c.collide(f)).cpu().numpy())
    c.close()
    start = np.cumsum([0] + counts)
    for gi, (N, L, lam) in enumerate(meshes):
        for i in sorted({start[gi], start[gi + 1] - 1}):
            _, q_o, _, _ = oracle_for(N, L, lam).collide(cells[i])
            assert rel_l2(q[i], q_o) < TOL32, (N, i, rel_l2(q[i], q_o))
            assert_conserved(q[i], N, L)

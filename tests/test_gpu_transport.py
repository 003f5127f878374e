"""GPU transport and Strang-split steps against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import transport as T
from paper_1211_0540_amd import bz
from paper_1211_0540_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def _shock_like(nx, N, L, seed):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    M = W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    hot = W.maxwellian(N, L, 1.0, (0.4, 0, 0), 1.6)
    wgt = np.exp(-x / 0.2)[:, None, None, None]
    return (1 - wgt) * M + wgt * hot * (1 + 0.05 * rng.uniform(-1, 1, (nx, 1, 1, 1)))


@pytest.mark.parametrize("N,L,nx", [(8, 4.0, 40), (12, 5.0, 17)])
def test_transport_step_matches_oracle(dev, N, L, nx):
    f0 = _shock_like(nx, N, L, N)
    g = bz.bz_grid_init(N, L, 1.0)
    t = bz.bz_transport_create(g, nx, 1.0, 2.0, 1.0, 0.0, 1.0)
    Mw = T.wall_maxwellian(N, L, 2.0)
    Mfar = W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    f = torch.from_numpy(f0.ravel().copy()).to(dev)
    work = torch.zeros(bz.bz_transport_workspace_bytes(t), dtype=torch.uint8, device=dev)
    dt = 0.4 / nx / L
    ref = f0
    for _ in range(3):
        bz.bz_transport_step(t, f, dt, work)
        ref = T.transport_rk2(ref, N, L, 1.0 / nx, dt, Mw, Mfar)
    got = f.cpu().numpy().reshape(ref.shape)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    bz.bz_transport_free(t)
    bz.bz_grid_free(g)


def test_strang_step_fp64_matches_oracle(dev):
    N, L, lam, nx, eps = 12, 5.0, 1.0, 8, 0.1
    f0 = _shock_like(nx, N, L, 1)
    c = bz.Collision([(N, L, lam)], [0] * nx, "plain_f64")
    t = bz.bz_transport_create(c.grids[0], nx, 1.0, 2.0, 1.0, 0.0, 1.0)
    f = torch.from_numpy(f0.ravel().copy()).to(dev)
    dt = 0.5 / nx / L
    o = O.Oracle(N, L, lam)
    Mw = T.wall_maxwellian(N, L, 2.0)
    Mfar = W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    ref = f0
    for _ in range(2):
        c.strang_step(t, dt, eps, f)
        ref = T.strang_step(ref, o, 1.0 / nx, dt, eps, Mw, Mfar)
    c.check()
    got = f.cpu().numpy().reshape(ref.shape)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    bz.bz_transport_free(t)
    c.close()


def test_shock_problem_full_size_fp32(dev):
    """256 cells on [0,1], N=24, L=7, hard spheres, Kn 0.1, wall jumps to T=2, batched FP32
    collisions, dt = 0.5 dx / max|v1|: mass is conserved (zero wall flux, far field at rest)
    and the gas next to the wall heats up; one step is compared with the oracle on all cells."""
    N, L, lam, nx, eps = 24, 7.0, 1.0, 256, 0.1
    dx = 1.0 / nx
    dt = 0.5 * dx / L
    f0 = W.shock_initial(nx, N, L)
    c = bz.Collision([(N, L, lam)], [0] * nx, "batched_f32")
    t = bz.bz_transport_create(c.grids[0], nx, 1.0, 2.0, 1.0, 0.0, 1.0)
    f = torch.from_numpy(f0.ravel().copy()).to(dev)
    c.strang_step(t, dt, eps, f)
    c.check()
    one = f.cpu().numpy().reshape(f0.shape)
    o = O.Oracle(N, L, lam)
    Mw = T.wall_maxwellian(N, L, 2.0)
    ref = T.strang_step(f0, o, dx, dt, eps, Mw, f0[-1])
    inc, inc_ref = one - f0, ref - f0
    assert np.linalg.norm(inc - inc_ref) / np.linalg.norm(inc_ref) < 1e-5
    for _ in range(19):
        c.strang_step(t, dt, eps, f)
    c.check()
    fin = f.cpu().numpy().reshape(f0.shape)
    dv3 = (2 * L / N) ** 3
    m0, m1 = f0.sum() * dv3 * dx, fin.sum() * dv3 * dx
    # the wall flux is zero by construction; the far-field ghost M(1,0,1) is not an exact
    # equilibrium of the discrete operator (|Q(M)| ~ 1e-5 |Q| at N=24), so the last cells drift
    # and the right face carries a net flux of order dt |v| |Q(M)| per step
    assert abs(m1 - m0) < 1e-8 * m0
    rho, u, Tmp, _ = O.moments(fin[0], L)
    # the conservative spectral method does not preserve positivity: the projection's
    # polynomial correction leaves tail values slightly negative (~1e-7 of the peak here)
    assert Tmp > 1.05 and np.all(fin > -1e-5 * fin.max())
    bz.bz_transport_free(t)
    c.close()


# ---------------------------------------------------------------------------
# Cells of width dx_j, the wall-refined mesh of the sudden-heating run, diagnostics
# ---------------------------------------------------------------------------
def _heated(widths, N, L, seed):
    x = np.cumsum(widths) - 0.5 * widths
    rng = np.random.default_rng(seed)
    M = W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    hot = W.maxwellian(N, L, 1.0, (0.4, 0, 0), 1.6)
    wgt = np.exp(-x / (0.2 * x[-1]))[:, None, None, None]
    return (1 - wgt) * M + wgt * hot * (1 + 0.05 * rng.uniform(-1, 1, (len(x), 1, 1, 1)))


@pytest.mark.parametrize("N,L", [(8, 4.0), (12, 5.0)])
def test_transport_on_the_wall_refined_mesh_matches_oracle(dev, N, L):
    widths = W.wall_refined_widths(eps=0.25, length=2.0)
    nx = len(widths)
    f0 = _heated(widths, N, L, N)
    g = bz.bz_grid_init(N, L, 1.0)
    t = bz.bz_transport_create_ex(g, widths, 2.0, 1.0, 0.0, 1.0)
    Mw, Mfar = T.wall_maxwellian(N, L, 2.0), W.maxwellian(N, L, 1.0, (0, 0, 0), 1.0)
    f = torch.from_numpy(f0.ravel().copy()).to(dev)
    work = torch.zeros(bz.bz_transport_workspace_bytes(t), dtype=torch.uint8, device=dev)
    dt = 0.4 * widths.min() / L
    ref = f0
    for _ in range(3):
        bz.bz_transport_step(t, f, dt, work)
        ref = T.transport_rk2(ref, N, L, widths, dt, Mw, Mfar)
    got = f.cpu().numpy().reshape(ref.shape)
    assert np.max(np.abs(got - ref)) < 1e-13 * np.max(np.abs(ref))
    bz.bz_transport_free(t)
    bz.bz_grid_free(g)


def test_equal_widths_are_bitwise_the_uniform_transport(dev):
    N, L, nx = 8, 4.0, 24
    f0 = _shock_like(nx, N, L, 3)
    g = bz.bz_grid_init(N, L, 1.0)
    ta = bz.bz_transport_create(g, nx, 1.0, 2.0, 1.0, 0.0, 1.0)
    tb = bz.bz_transport_create_ex(g, np.full(nx, 1.0 / nx), 2.0, 1.0, 0.0, 1.0)
    out = []
    for t in (ta, tb):
        f = torch.from_numpy(f0.ravel().copy()).to(dev)
        work = torch.zeros(bz.bz_transport_workspace_bytes(t), dtype=torch.uint8, device=dev)
        for _ in range(2):
            bz.bz_transport_step(t, f, 0.3 / nx / L, work)
        out.append(f.cpu().numpy())
        bz.bz_transport_free(t)
    assert np.array_equal(out[0], out[1])
    bz.bz_grid_free(g)


@pytest.mark.parametrize("mode,tol", [("batched_f64", 1e-12), ("batched_f32", 1e-5)])
def test_strang_on_the_wall_refined_mesh_matches_oracle(dev, mode, tol):
    """The sudden-heating configuration of Sec. 5 at small size: eps = 1, eight cells per mean
    free path at the wall and two inside, two Strang steps against the oracle."""
    N, L, lam, eps = 12, 5.0, 1.0, 1.0
    widths = W.wall_refined_widths(eps=eps, length=4.0)
    nx = len(widths)
    f0 = W.shock_initial(nx, N, L)
    c = bz.Collision([(N, L, lam)], [0] * nx, mode)
    t = bz.bz_transport_create_ex(c.grids[0], widths, 2.0, 1.0, 0.0, 1.0)
    f = torch.from_numpy(f0.ravel().copy()).to(dev)
    dt = 0.5 * widths.min() / L
    o = O.Oracle(N, L, lam)
    Mw = T.wall_maxwellian(N, L, 2.0)
    ref = f0
    for _ in range(2):
        c.strang_step(t, dt, eps, f)
        ref = T.strang_step(ref, o, widths, dt, eps, Mw, f0[-1])
    c.check()
    got = f.cpu().numpy().reshape(ref.shape)
    if mode == "batched_f64":
        assert np.max(np.abs(got - ref)) < tol * np.max(np.abs(ref))
    else:
        assert np.linalg.norm((got - f0) - (ref - f0)) / np.linalg.norm(ref - f0) < tol
    bz.bz_transport_free(t)
    c.close()


def test_moments_and_marginal_match_oracle(dev):
    """Per-cell density, bulk velocity and temperature on two meshes in one batch, and the
    v1 marginal of one cell, against the oracle's moment sums."""
    meshes = [(12, 5.0, 1.0), (16, 6.0, 1.0)]
    cells = list(W.random_smooth_cells(5, 12, 5.0, seed=8)) + list(W.random_smooth_cells(4, 16, 6.0, seed=9))
    goc = [0] * 5 + [1] * 4
    c = bz.Collision(meshes, goc, "batched_f64")
    f = torch.from_numpy(c.pack(cells)).to(dev)
    mom = torch.zeros(5 * len(cells), dtype=torch.float64, device=dev)
    bz.bz_cell_moments(c.batch, f, mom)
    marg = torch.zeros(16, dtype=torch.float64, device=dev)
    bz.bz_marginal_v1(c.batch, f, 7, marg)
    got = mom.cpu().numpy().reshape(-1, 5)
    for i, x in enumerate(cells):
        N, L, _ = meshes[goc[i]]
        rho, u, Tm = T.moments_1d(x[None], N, L)
        assert got[i, 0] == pytest.approx(rho[0], rel=1e-13)
        assert np.allclose(got[i, 1:4], u[0], rtol=0, atol=1e-13 * (1 + np.abs(u[0]).max()))
        assert got[i, 4] == pytest.approx(Tm[0], rel=1e-12)
    ref = T.marginal_v1(cells[7], 16, 6.0)
    assert np.max(np.abs(marg.cpu().numpy() - ref)) < 1e-14 * np.max(np.abs(ref))
    with pytest.raises(bz.BzError):
        bz.bz_marginal_v1(c.batch, f, 9, marg)
    c.close()


def test_sudden_heating_run(dev):
    """The Sec. 5 run at small size (N=12, 6 mean free paths, eps = 1): the mass changes only
    by the far-field face (the wall's net flux is zero; on the mesh [-L, L) the v1 = -L plane
    has no +L partner, so the far-field Maxwellian carries a net flux of order L exp(-L^2/2)),
    the gas next to the heated wall warms and moves away from it, and the diagnostics equal
    the oracle's moments of the final state."""
    from paper_1211_0540_amd.sudden_heating import SuddenHeating
    run = SuddenHeating(N=12, L=5.0, length=6.0, mode="batched_f64")
    m0 = run.mass()
    run.step(12)
    d = run.diagnostics()
    v1 = W.velocity_mesh(12, 5.0)
    far = (v1[:, None, None] * W.maxwellian(12, 5.0, 1.0, (0, 0, 0), 1.0)).sum() * (10.0 / 12) ** 3
    assert abs(run.mass() - m0) < 2 * abs(far) * run.time + 1e-12 * m0
    assert d["T"][0] > 1.05 and d["u1"][: run.nx // 4].max() > 1e-3
    fin = run.f.cpu().numpy().reshape(run.nx, 12, 12, 12)
    rho, u, Tm = T.moments_1d(fin, 12, 5.0)
    assert np.allclose(d["rho"], rho, rtol=1e-12) and np.allclose(d["u1"], u[:, 0], atol=1e-12)
    assert np.allclose(d["T"], Tm, rtol=1e-11)
    assert np.allclose(d["wall_marginal_v1"], T.marginal_v1(fin[0], 12, 5.0), rtol=1e-12, atol=1e-15)
    run.close()

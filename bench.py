"""Benchmark: cell-collision evaluations per second at N=32 on one MI355X.

Workload: the N=32 cells (L=8, hard spheres) of the seeded 1024-cell uneven
draw (perturbed Maxwellians, rho ~ U[.5,2], |u| ~ U[0,1.5], T ~ U[.5,2]).
One bench step is one Heun (second-order Runge-Kutta) step of the space-
homogeneous equation for every cell of the batch: two collision evaluations
per cell (forward transform, batched FP32 convolution with compensated
accumulation and its FP64 low-frequency core in the same persistent launch,
inverse transform, FP64 projection) and the Heun updates.

The JSON line also carries:
  roofline      the convolution launch against the FP32 vector peak, timed with
                HIP events on the library's stream inside the timed region.
                `achieved` counts the FP32 work the launch executes: 10 flops
                (4 FMA + 2 MUL) per weight slot the conjugate-symmetric schedule
                visits, per cell.  The full sum's algorithmic flops over the same
                time are reported apart as `effective_tflops` (never in `frac`);
                so are the FP64 core's flops and the issue ceiling of the kernel's
                instruction mix without packed FP32.
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same cells
  comparisons   the plain unbatched and the batched FP64 paths on the same GPU,
                the relative L2 error of every cell against the plain FP64
                result, the per-mesh launch, the batch without its FP64 core,
                graph replay, the full-sum schedule, the N=32 relaxation, the
                whole uneven batch, and the gated closure on the shock problem
                at N=24 and N=32
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-collision evals/s at N=32: FP32 batched & surrogate vs FP64 plain; rel L2 err"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector, published (packed FP32: two lanes' FMAs per instruction)
# Without packed FP32 one FMA per lane issues per 4 cycles per SIMD (78.6 TFLOP/s, half the peak);
# the kernel's 4 FMA + 2 MUL per slot carry 10 flops in 6 instructions: 0.5 * 10 / 12 of the peak.
ISSUE_CEILING_FRAC = 0.5 * 10.0 / 12.0
TRAIN_STEPS = 30000        # closure training: Adam steps of 512 rows
HBM_TBPS = 8.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def conv_source_sha():
    """Digest of the sources that fix what one convolution launch reads and writes:
    the kernel and the schedule that builds its work items."""
    h = hashlib.sha256()
    for name in ("bz_conv.hip", "bz_runtime.hip", "bz_internal.h"):
        with open(os.path.join(ROOT, "paper_1211_0540_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join("profiles", "conv_multi_n32_traffic.json")


def measured_traffic(cells):
    """HBM bytes per launch of the N=32 convolution launch from the committed counter
    summary (rocprofv3 FETCH_SIZE and WRITE_SIZE passes of `bench.py --profile-run`),
    if it was taken on the current kernel and schedule sources and the same batch."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_FILE)) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha") != conv_source_sha() or d.get("cells") != cells:
        return None
    return d.get("traffic_bytes_per_launch")


def measured_valu_insts(cells):
    """Wavefront VALU instructions per launch of the same kernel (rocprofv3 --pmc SQ_INSTS_VALU
    pass of `bench.py --profile-run`) from the same committed summary, under the same
    conditions as measured_traffic."""
    try:
        with open(os.path.join(ROOT, TRAFFIC_FILE)) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha") != conv_source_sha() or d.get("cells") != cells:
        return None
    return d.get("sq_insts_valu_per_launch")


def core_products(N, r2):
    """Complex products per cell and evaluation of the FP64 core (r2 = 0: none): for every
    output row (k1, k2) within 2r of the centre, the pairs of disk rows m <= j with
    m + j = k + N/2 (the core steps), each the products of the two rows' entries inside the
    ball (a row at distance rho from the centre has 2 floor(sqrt(r2 - rho^2)) + 1 of them), of
    all outputs, or of the outputs k3 <= N/2 on the derived rows of the conjugate-symmetric
    schedule, which are skipped when 2r < N/2."""
    if r2 < 1:
        return 0
    import numpy as np
    h = N // 2
    r = 0
    while (r + 1) ** 2 <= r2:
        r += 1
    a = np.arange(N)
    rho2 = (a[:, None] - h) ** 2 + (a[None, :] - h) ** 2
    disk = rho2 <= r2
    ext = np.floor(np.sqrt(np.maximum(r2 - rho2, 0) + 1e-9)).astype(int)
    pts = np.argwhere(disk)
    t = np.arange(-r, r + 1)

    def pairs(am, aj, half):
        tm = t[np.abs(t) <= am][:, None]
        tj = t[np.abs(t) <= aj][None, :]
        return int(((tm + tj) <= 0).sum()) if half else tm.size * tj.size

    total = 0
    for k1 in range(max(0, h - 2 * r), min(N - 1, h + 2 * r) + 1):
        for k2 in range(max(0, h - 2 * r), min(N - 1, h + 2 * r) + 1):
            derived = k1 >= 1 and k2 >= 1 and (k1 > h or (k1 == h and k2 > h))
            if derived and 2 * r < h:
                continue
            j = np.stack([k1 + h - pts[:, 0], k2 + h - pts[:, 1]], 1)
            ok = (j >= 0).all(1) & (j < N).all(1)
            ok[ok] &= disk[j[ok, 0], j[ok, 1]]
            m_le_j = (pts[:, 0] < j[:, 0]) | ((pts[:, 0] == j[:, 0]) & (pts[:, 1] <= j[:, 1]))
            for i in np.flatnonzero(ok & m_le_j):
                total += pairs(ext[pts[i, 0], pts[i, 1]], ext[j[i, 0], j[i, 1]], derived)
    return total


def timed_steps(torch, step, steps):
    """Run `steps` steps, each bracketed by HIP events on the current stream; the total
    (first start to last stop) and the per-step times in milliseconds."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    per = [a.elapsed_time(b) for a, b in ev]
    return ev[0][0].elapsed_time(ev[-1][1]), per


def spread(np, x):
    x = np.asarray(x, dtype=float)
    q1, q2, q3 = np.percentile(x, [25, 50, 75])
    return {"median": float(q2), "iqr": float(q3 - q1), "min": float(x.min()), "max": float(x.max())}


def schedule_slots(N, symmetric):
    """Weight slots (unordered pairs incl. the zero-weight half of diagonal steps) one
    64-cell group processes: every row's steps in the full-sum schedule; in the
    conjugate-symmetric one, the direct rows less their m1 = 0 block, the three edge
    passes and pass Z."""
    h = N // 2
    lo = lambda k: max(0, k - h + 1)
    hi = lambda k: min(N - 1, k + h)
    cnt = lambda k: hi(k) - lo(k) + 1

    def steps(k1, k2):
        n = 0
        for m1 in range(lo(k1), min((k1 + h) // 2, hi(k1)) + 1):
            last = hi(k2) if 2 * m1 < k1 + h else min((k2 + h) // 2, hi(k2))
            n += last - lo(k2) + 1
        return n

    derived = lambda a, b: a >= 1 and b >= 1 and (a > h or (a == h and b > h))
    rows = sum(steps(a, b) for a in range(N) for b in range(N) if not (symmetric and derived(a, b)))
    if symmetric:
        # pass A skips the steps that only meet zeroed planes of its fhat copy: the
        # m1 = 0 block of rows k1 < N/2, and the steps with m2 = 0 or j2 = 0
        for a in range(N):
            for b in range(N):
                if derived(a, b):
                    continue
                if a < h:
                    rows -= cnt(b)
                if b < h:
                    for m1 in range(max(lo(a), 1), min((a + h) // 2, hi(a)) + 1):
                        last = hi(b) if 2 * m1 < a + h else min((b + h) // 2, hi(b))
                        rows -= 1 + (1 if last == b + h else 0)
        rows += sum(cnt(b) + 2 * (cnt(b) - (2 if b < h else 0)) for a in range(h) for b in range(N))
        rows += sum(steps(0, b) for b in range(h, N))
    return rows * 3 * N * N // 4


def step_leg(torch, np, bz, meshes, gidx, f0, wcache, steps=5, per_mesh=False, schedule="symmetric",
             autotune=False):
    """Heun steps of one batch configuration: median step time, convolution launches per
    evaluation and their mean time."""
    c = bz.Collision(meshes, gidx, "batched_f32", weights_cache=wcache, per_mesh=per_mesh, schedule=schedule)
    variants = c.autotune(f0, reps=2) if autotune else None
    f = f0.clone()
    c.step(f, 0.01)
    torch.cuda.synchronize()
    bz.bz_batch_timer_read(c.batch)
    bz.bz_batch_timer(c.batch, True)
    _, per = timed_steps(torch, lambda: c.step(f, 0.01), steps)
    bz.bz_batch_timer(c.batch, False)
    conv, k = bz.bz_batch_timer_read(c.batch)
    c.check()
    out = {"step_ms": spread(np, per), "conv_launches_per_eval": k / (2 * steps),
           "conv_ms_per_eval": conv / (2 * steps), "one_launch": bz.bz_batch_one_launch(c.batch)}
    if variants is not None:
        out["variants"] = variants
    c.close()
    return out


def relaxation_leg(torch, np, bz, W):
    """Bi-Maxwellian relaxation on the N=32, L=8 mesh, hard spheres: 100 Heun steps
    with dt = 0.01, batched FP32 against plain FP64; directional temperatures."""
    N, L, steps, dt = 32, 8.0, 100, 0.01
    f0 = W.relaxation_cell(N, L)
    dv = 2 * L / N
    v = dv * (np.arange(N) - N // 2)
    V = np.meshgrid(v, v, v, indexing="ij")

    def temps(f):
        rho = f.sum()
        u = [(V[d] * f).sum() / rho for d in range(3)]
        return np.array([((V[d] - u[d]) ** 2 * f).sum() / rho for d in range(3)])

    res = {}
    for mode in ("plain_f64", "batched_f32"):
        c = bz.Collision([(N, L, 1.0)], [0], mode)
        f = torch.from_numpy(c.pack([f0])).cuda()
        T = [temps(f0)]
        ms = 0.0
        for _ in range(steps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            c.step(f, dt)
            torch.cuda.synchronize()
            ms += (time.perf_counter() - a) * 1e3
            T.append(temps(f.cpu().numpy().reshape(N, N, N)))
        c.check()
        c.close()
        res[mode] = (np.array(T), ms / steps)
    dT = np.abs(res["batched_f32"][0] - res["plain_f64"][0])
    return {"workload": "one N=32 bi-Maxwellian cell (T = 2, 0.5, 0.5), hard spheres, 100 Heun steps, dt = 0.01",
            "max_abs_dT_fp32_vs_fp64": float(dT.max()), "T_x_final_fp64": float(res["plain_f64"][0][-1, 0]),
            "fp64_plain_ms_per_step": res["plain_f64"][1], "fp32_batched_ms_per_step": res["batched_f32"][1]}


def uneven_leg(torch, np, bz, W, n32_step_ms, steps=5):
    """All 1024 cells of the uneven draw (N = 16, 24, 32 in one batch): FP32 Heun steps with
    the one persistent launch for every mesh and core (the default) and with one launch per
    mesh (autotuned variants); the step time against the N=32-only step of this run and
    against the ratio of executed FP32 work; per-mesh FP32 vs batched-FP64 errors of one
    evaluation; graph replay."""
    batch = W.uneven_batch(n_cells=1024)
    meshes = [(16, 6.0, 1.0), (24, 7.0, 1.0), (32, 8.0, 1.0)]
    gidx = [{16: 0, 24: 1, 32: 2}[int(n)] for n in batch.Ns]
    wc = {}
    c32 = bz.Collision(meshes, gidx, "batched_f32", weights_cache=wc)
    f0 = torch.from_numpy(c32.pack(batch.cells)).cuda()
    q32 = c32.project(c32.collide(f0)).cpu().numpy()
    c64 = bz.Collision(meshes, gidx, "batched_f64", weights_cache=wc)
    q64 = c64.project(c64.collide(f0)).cpu().numpy()
    c64.close()
    errs = {16: [], 24: [], 32: []}
    for n, x, y in zip(batch.Ns, c32.unpack(q32), c32.unpack(q64)):
        errs[int(n)].append(float(np.linalg.norm(x - y) / np.linalg.norm(y)))
    one = step_leg(torch, np, bz, meshes, gidx, f0, wc, steps=steps)
    per = step_leg(torch, np, bz, meshes, gidx, f0, wc, steps=steps, per_mesh=True, autotune=True)
    tuned = step_leg(torch, np, bz, meshes, gidx, f0, wc, steps=steps, autotune=True)
    # executed FP32 slots: every 64-cell group of a mesh runs its schedule (idle lanes included)
    Ns, counts = np.unique(batch.Ns, return_counts=True)
    work = sum(schedule_slots(int(n), True) * -(-int(k) // 64) for n, k in zip(Ns, counts))
    work32 = schedule_slots(32, True) * -(-int(counts[list(Ns).index(32)]) // 64)
    # the same step captured as one HIP graph (three meshes, all their launches) and replayed
    graph = None
    try:
        f = f0.clone()
        gs = torch.cuda.Stream()
        wg = torch.zeros_like(c32.work)
        with torch.cuda.stream(gs):
            gh = bz.bz_graph_capture_step(c32.batch, f, 0.01, wg, gs)
        torch.cuda.synchronize()
        bz.bz_graph_launch(gh, gs)
        gs.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(gs)
        for _ in range(steps):
            bz.bz_graph_launch(gh, gs)
        e1.record(gs)
        gs.synchronize()
        graph = {"ms_per_step": e0.elapsed_time(e1) / steps}
        bz.bz_graph_free(gh)
    except Exception as exc:
        graph = {"error": str(exc)}
    c32.close()
    ms = one["step_ms"]["median"]
    return {"workload": "1024 cells of the seeded uneven draw (521 N=16, 313 N=24, 190 N=32), one batch",
            "ms_per_step": ms, "cell_evals_per_s": 2 * len(batch.Ns) / ms * 1e3,
            "one_launch": one, "per_mesh_launches_autotuned": per, "autotuned_choice": tuned,
            "step_vs_n32_only_step": ms / n32_step_ms,
            "executed_fp32_work_vs_n32_only": work / work32,
            "graph_replay": graph,
            "rel_l2_fp32_vs_fp64_batched": {str(k): {"median": float(np.median(v)), "max": float(np.max(v)),
                                                     "frac_le_1e-5": float(np.mean(np.array(v) <= 1e-5))}
                                            for k, v in errs.items()}}


def closure_leg(args, torch, np, bz, W, N=24, L=7.0, snapshots=900, relax_cells=768):
    """Harvest (f, Q) pairs on the shock problem and homogeneous relaxations on the
    N^3 mesh, train the N^3-1024-1024-N^3 network with the library's kernels, then
    time Strang steps of the 256-cell shock problem with and without the gated closure
    (gate 0.05, one group in 16 judged) and compare the temperature profiles."""
    import oracle as O
    from paper_1211_0540_amd.closure import ClosureModel
    lam, nx, eps = 1.0, 256, 0.1
    t0 = time.perf_counter()
    m = ClosureModel(N, L, lam, hidden=1024, seed=1211)
    rows = (m.harvest_shock(snapshots=snapshots, every=1, keep=0.1)
            + m.harvest_relaxation(cells=relax_cells, steps=40, keep=0.1))
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    t0 = time.perf_counter()
    hist = m.fit(steps=TRAIN_STEPS, batch=512, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    val, val_median = m.validation_error()
    m.release_data()
    dt = 0.5 / nx / L
    f0 = torch.from_numpy(W.shock_initial(nx, N, L).ravel().copy()).cuda()
    # the plain step on the default split; the closure on a batch whose work items are sized for
    # the one or two groups it still convolves
    c = bz.Collision([(N, L, lam)], [0] * nx, "batched_f32", weights_cache=m.wcache)
    cf = bz.Collision([(N, L, lam)], [0] * nx, "batched_f32", weights_cache=m.wcache, fine_split=True)
    t = bz.bz_transport_create(c.grids[0], nx, 1.0, 2.0, 1.0, 0.0, 1.0)
    d = m.desc(gate=0.05, judge_every=16)
    work = torch.zeros(bz.bz_closure_workspace_bytes(cf.batch, d) + bz.bz_transport_workspace_bytes(t) + 256,
                       dtype=torch.uint8, device="cuda")
    K = 300
    fa, fb = f0.clone(), f0.clone()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(K):
        c.strang_step(t, dt, eps, fa)
    torch.cuda.synchronize()
    ta = time.perf_counter() - a
    a = time.perf_counter()
    for _ in range(K):
        bz.bz_closure_strang_step(cf.batch, t, d, fb, dt, eps, work)
    torch.cuda.synchronize()
    tb = time.perf_counter() - a
    st = bz.bz_closure_read_stats(cf.batch, d, work)
    served = served_errors(torch, np, bz, cf, d, fb, work, N)
    A = fa.cpu().numpy().reshape(nx, N, N, N)
    B = fb.cpu().numpy().reshape(nx, N, N, N)
    TA = np.array([O.moments(A[j], L)[2] for j in range(nx)])
    TB = np.array([O.moments(B[j], L)[2] for j in range(nx)])
    bz.bz_transport_free(t)
    c.close()
    cf.close()
    evals = 2 * nx * K
    return {"workload": f"256-cell N={N} shock problem (wall T=2, Kn 0.1), 300 Strang steps",
            "training_rows": rows, "harvest_s": t_harvest, "train_steps": TRAIN_STEPS,
            "train_s": t_train,
            "loss_first_last": [hist[0][1], hist[-1][1]], "heldout_rel_l2": val, "heldout_median_row_rel_l2": val_median,
            "plain_fp32_ms_per_step": ta / K * 1e3, "closure_ms_per_step": tb / K * 1e3,
            "speedup": ta / tb, "closure_cell_evals_per_s": evals / tb, "served_fraction": st["served"] / evals,
            "judged": st["judged"], "judge_failed": st["failed"],
            "judge_pass_fraction": 1.0 - st["failed"] / max(st["judged"], 1), "judge_max_rel_err": st["max_err"],
            "unbounded_served": st["unbounded"], "gate_cap": st["gate_cap"],
            "served_cells_one_evaluation": served,
            "max_abs_T_profile_deviation": float(np.max(np.abs(TA - TB)))}


def served_errors(torch, np, bz, col, desc, f, work, N):
    """Every cell the gate serves in one evaluation of the final state, against the
    convolution: err = |P(Q_s - Q_c)| / (|P Q_c| + floor rho |M|_2), the judge's measure,
    with the library's FP64 projection P."""
    n = len(col.grid_of_cell)
    d0 = bz.ClosureDesc(desc.net, desc.d_params, desc.gate, desc.s_in, desc.s_out, 0, desc.judge_tol,
                        desc.judge_floor)
    state = torch.zeros(n * 10, dtype=torch.float64, device=f.device)
    x = torch.zeros(n * N ** 3, dtype=torch.int16, device=f.device)
    bz.bz_closure_prepare(col.batch, f, desc.gate, desc.s_in, state, x)
    qs = torch.zeros(col.elems, dtype=torch.float64, device=f.device)
    bz.bz_closure_collide(col.batch, d0, f, qs, work)
    bz.bz_closure_read_stats(col.batch, d0, work)
    qc = col.collide(f)
    col.project(qs)
    col.project(qc)
    st = state.view(n, 10)
    D = (qs - qc).view(n, -1).norm(dim=1)
    C = qc.view(n, -1).norm(dim=1)
    err = (D / (C + desc.judge_floor * st[:, 0] * st[:, 8]))[st[:, 6] != 0].cpu().numpy()
    if err.size == 0:
        return {"served": 0}
    return {"served": int(err.size), "median": float(np.median(err)), "p90": float(np.percentile(err, 90)),
            "max": float(err.max()), "frac_le_judge_tol": float(np.mean(err <= desc.judge_tol)),
            "judge_tol": desc.judge_tol}


def closure_profile_run(args, N=24, L=7.0):
    """Strang steps of the 256-cell N=24 shock problem with the gated closure (gate 0.05, one
    group in 16 judged) after a short harvest (60 shock snapshots) and 300 training steps, then
    the same number of plain steps: one JSON line with both step times, for profiler runs.  The
    served fraction, and so the step time, depends on the training; the bench's closure leg
    trains the network fully."""
    import torch
    from paper_1211_0540_amd import bz
    from paper_1211_0540_amd import workloads as W
    from paper_1211_0540_amd.closure import ClosureModel

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lam, nx, eps = 1.0, 256, 0.1
    m = ClosureModel(N, L, lam, hidden=1024, seed=1211)
    m.harvest_shock(snapshots=60, every=1, keep=0.1)
    m.fit(steps=300, batch=512, lr=1e-3)
    m.release_data()
    dt = 0.5 / nx / L
    f0 = torch.from_numpy(W.shock_initial(nx, N, L).ravel().copy()).cuda()
    c = bz.Collision([(N, L, lam)], [0] * nx, "batched_f32", weights_cache=m.wcache)
    cf = bz.Collision([(N, L, lam)], [0] * nx, "batched_f32", weights_cache=m.wcache, fine_split=True)
    t = bz.bz_transport_create(c.grids[0], nx, 1.0, 2.0, 1.0, 0.0, 1.0)
    d = m.desc(gate=0.05, judge_every=16)
    work = torch.zeros(bz.bz_closure_workspace_bytes(cf.batch, d) + bz.bz_transport_workspace_bytes(t) + 256,
                       dtype=torch.uint8, device="cuda")
    f, g = f0.clone(), f0.clone()
    for _ in range(args.warmup):
        bz.bz_closure_strang_step(cf.batch, t, d, f, dt, eps, work)
        c.strang_step(t, dt, eps, g)
    total_c, _ = timed_steps(torch, lambda: bz.bz_closure_strang_step(cf.batch, t, d, f, dt, eps, work), args.steps)
    total_p, _ = timed_steps(torch, lambda: c.strang_step(t, dt, eps, g), args.steps)
    st = bz.bz_closure_read_stats(cf.batch, d, work)
    evals = 2 * nx * (args.steps + args.warmup)
    print(json.dumps({"profile_closure": True, "cells": nx, "N": N, "closure_ms_per_step": total_c / args.steps,
                      "plain_ms_per_step": total_p / args.steps, "served_fraction": st["served"] / evals,
                      "judged": st["judged"], "judge_failed": st["failed"]}), flush=True)
    bz.bz_transport_free(t)
    c.close()
    cf.close()
    return 0


def uneven_profile_run(args):
    """Heun steps of the 1024-cell uneven batch only (one persistent convolution launch per
    evaluation for all three meshes and their cores): one JSON line with the step and the
    convolution time, for profiler runs."""
    import numpy as np
    import torch
    from paper_1211_0540_amd import bz
    from paper_1211_0540_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    batch = W.uneven_batch(n_cells=1024)
    meshes = [(16, 6.0, 1.0), (24, 7.0, 1.0), (32, 8.0, 1.0)]
    gidx = [{16: 0, 24: 1, 32: 2}[int(n)] for n in batch.Ns]
    col = bz.Collision(meshes, gidx, "batched_f32")
    f = torch.from_numpy(col.pack(batch.cells)).cuda()
    for _ in range(args.warmup):
        col.step(f, 0.01)
    torch.cuda.synchronize()
    bz.bz_batch_timer_read(col.batch)  # clear
    bz.bz_batch_timer(col.batch, True)
    total_ms, _ = timed_steps(torch, lambda: col.step(f, 0.01), args.steps)
    bz.bz_batch_timer(col.batch, False)
    col.check()
    conv_ms, launches = bz.bz_batch_timer_read(col.batch)
    print(json.dumps({"profile_uneven": True, "cells": len(batch.Ns), "one_launch": bz.bz_batch_one_launch(col.batch),
                      "ms_per_step": total_ms / args.steps, "conv_avg_ms": conv_ms / max(launches, 1),
                      "kernel_src_sha": conv_source_sha()}), flush=True)
    col.close()
    return 0


def mlp_profile_run(args, n_in=13824, hidden=1024, rows=512, cells=256):
    """Training steps (forward, backward, Adam) and serving forwards of the closure network at
    its configured shape on seeded synthetic BF16 inputs; one JSON line with the times and the
    matrix-product rates."""
    import numpy as np
    import torch
    from paper_1211_0540_amd import bz
    net = bz.bz_mlp_create(n_in, hidden, n_in)
    params = torch.zeros(bz.bz_mlp_param_bytes(net), dtype=torch.uint8, device="cuda")
    rng = np.random.default_rng(1211)
    parts = []
    for o, i in ((hidden, n_in), (hidden, hidden), (n_in, hidden)):
        sc = 1.0 / np.sqrt(i)
        parts += [rng.uniform(-sc, sc, o * i).astype(np.float32), rng.uniform(-sc, sc, o).astype(np.float32)]
    bz.bz_mlp_set_params(net, params, np.concatenate(parts))
    x = torch.randn(rows, n_in, device="cuda").to(torch.bfloat16).view(torch.int16)
    y = torch.randn(rows, n_in, device="cuda")
    work = torch.zeros(bz.bz_mlp_workspace_bytes(net, rows), dtype=torch.uint8, device="cuda")
    grad = torch.zeros(bz.bz_mlp_param_count(net), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = torch.zeros(cells, n_in, dtype=torch.float32, device="cuda")

    def train():
        bz.bz_mlp_backward(net, params, x, y, rows, grad, loss, work)
        bz.bz_mlp_adam(net, params, grad, 1, 1e-4)

    def serve():
        bz.bz_mlp_forward(net, params, x[:cells], cells, out, work)

    for fn in (train, serve):
        fn()
    steps = max(args.steps, 10)
    t_train, _ = timed_steps(torch, train, steps)
    t_serve, _ = timed_steps(torch, serve, steps)
    fwd = 2.0 * (n_in * hidden + hidden * hidden + hidden * n_in)
    # training: forward, weight gradients (the same flops) and the activation gradients of layers 2, 3
    train_flops = rows * (2 * fwd + 2.0 * (hidden * hidden + n_in * hidden))
    out_line = {"profile_mlp": True, "shape": [n_in, hidden, hidden, n_in], "train_rows": rows,
                "train_ms_per_step": t_train / steps, "train_tflops": train_flops / (t_train / steps * 1e-3) / 1e12,
                "serve_cells": cells, "serve_ms": t_serve / steps,
                "serve_tflops": cells * fwd / (t_serve / steps * 1e-3) / 1e12, "peak_bf16_tflops": 2500.0}
    print(json.dumps(out_line), flush=True)
    bz.bz_mlp_free(net)
    return 0


def gpu_clocks():
    """The GPU engine clock as rocm-smi reports it (best effort), read after the timed legs."""
    import subprocess
    try:
        out = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        d = json.loads(out.stdout)
        card = next(iter(d.values()))
        return {k: v for k, v in card.items() if "sclk" in k.lower()}
    except Exception:
        return None


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure leg")
    ap.add_argument("--profile-run", action="store_true",
                    help="timed steps only (default launch configuration, no comparisons, no CPU leg)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--profile-closure", action="store_true",
                    help="only Strang steps of the 256-cell N=24 shock problem with the gated closure, after a "
                         "short harvest and training, for kernel traces")
    ap.add_argument("--profile-uneven", action="store_true",
                    help="only timed Heun steps of the 1024-cell uneven batch (N = 16, 24, 32) in the default "
                         "launch form, for kernel traces and counters")
    ap.add_argument("--profile-mlp", action="store_true",
                    help="only the closure network's kernels: training steps of 512 rows and forwards of 256 "
                         "cells of the N=24 network on synthetic data")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2
    if args.profile_mlp:
        return mlp_profile_run(args)
    if args.profile_uneven:
        return uneven_profile_run(args)
    if args.profile_closure:
        return closure_profile_run(args)

    import numpy as np
    import torch
    from paper_1211_0540_amd import bz
    from paper_1211_0540_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    N, L, lam = 32, W.DOMAIN_FOR_N[32], 1.0
    batch = W.uneven_batch(n_cells=1024, only_N=32)
    cells = batch.cells
    nc = len(cells)
    P = (3 * N * N // 4) ** 3
    log(f"workload: {nc} N=32 cells of the 1024-cell uneven draw")

    wcache = {}
    col = bz.Collision([(N, L, lam)], [0] * nc, "batched_f32", weights_cache=wcache)
    info = bz.bz_grid_query(col.grids[0])
    f0 = torch.from_numpy(col.pack(cells)).to(dev)
    one_launch = bz.bz_batch_one_launch(col.batch)
    log(f"convolution: {'one launch for the FP32 items and the FP64 core' if one_launch else 'per-mesh launch'}")

    # FP32 result of one evaluation (kept for the error report)
    q32 = col.collide(f0)
    col.project(q32)

    f = f0.clone()
    dt_over_eps = 0.01
    for _ in range(args.warmup):
        col.step(f, dt_over_eps)
    torch.cuda.synchronize()
    bz.bz_batch_timer_read(col.batch)  # clear
    bz.bz_batch_timer(col.batch, True)
    total_ms, per_step = timed_steps(torch, lambda: col.step(f, dt_over_eps), args.steps)
    bz.bz_batch_timer(col.batch, False)
    col.check()
    conv_ms, conv_launches = bz.bz_batch_timer_read(col.batch)
    ms_step = total_ms / args.steps
    evals = 2 * nc * args.steps
    value = evals / (total_ms * 1e-3)
    conv_avg_ms = conv_ms / max(conv_launches, 1)
    slots = schedule_slots(N, True)           # weight slots per cell the schedule visits
    fp32_flops = 10.0 * slots * nc
    core_flops = 10.0 * core_products(N, info["core_r2"]) * nc
    achieved = fp32_flops / (conv_avg_ms * 1e-3) / 1e12
    log(f"step {ms_step:.3f} ms, {value:.0f} evals/s, conv {conv_avg_ms:.3f} ms/launch ({conv_launches} launches)")

    # the same step captured as a HIP graph and replayed
    graph = None
    try:
        gs = torch.cuda.Stream()
        fg = f.clone()
        wg = torch.zeros_like(col.work)
        with torch.cuda.stream(gs):
            gh = bz.bz_graph_capture_step(col.batch, fg, dt_over_eps, wg, gs)
        torch.cuda.synchronize()
        for _ in range(2):
            bz.bz_graph_launch(gh, gs)
        gs.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(gs)
        for _ in range(args.steps):
            bz.bz_graph_launch(gh, gs)
        e1.record(gs)
        gs.synchronize()
        graph = {"ms_per_step": e0.elapsed_time(e1) / args.steps}
        bz.bz_graph_free(gh)
        del fg, wg
    except Exception as exc:  # reported, never fatal for the main line
        graph = {"error": str(exc)}

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    if args.profile_run:
        print(json.dumps({"profile_run": True, "ms_per_step": ms_step, "conv_avg_ms": conv_avg_ms,
                          "cells": nc, "kernel_src_sha": conv_source_sha()}), flush=True)
        col.close()
        return 0

    # ---- comparisons on the same GPU ----------------------------------
    comp = {}
    # plain unbatched FP64 (one cell per launch sequence) on every cell
    plain = bz.Collision([(N, L, lam)], [0] * nc, "plain_f64", weights_cache=wcache)
    q64 = plain.collide(f0)
    plain.project(q64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qq = plain.collide(f0)
    plain.project(qq)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    comp["plain_fp64_evals_per_s"] = nc / plain_s
    b64 = q64.cpu().numpy()
    ref = plain.unpack(b64)
    plain.close()
    del qq

    def errs_of(q):
        e = np.array([np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(col.unpack(q.cpu().numpy()), ref)])
        return {"median": float(np.median(e)), "max": float(e.max()), "frac_le_1e-5": float(np.mean(e <= 1e-5)),
                "cells": int(e.size)}

    comp["rel_l2_fp32_batched_vs_fp64_plain"] = errs_of(q32)
    # batched FP64: every cell of the batch in the FP64 kernel
    b64c = bz.Collision([(N, L, lam)], [0] * nc, "batched_f64", weights_cache=wcache)
    qb = b64c.collide(f0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qb = b64c.collide(f0)
    b64c.project(qb)
    torch.cuda.synchronize()
    comp["batched_fp64_evals_per_s"] = nc / (time.perf_counter() - t0)
    b64c.close()
    del qb
    comp["fp32_batched_step_evals_per_s"] = value
    comp["speedup_fp32_batched_vs_fp64_plain"] = value / comp["plain_fp64_evals_per_s"]
    comp["speedup_fp32_batched_vs_fp64_batched"] = value / comp["batched_fp64_evals_per_s"]
    comp["graph_replay"] = graph
    # the same batch with one launch for the FP32 items and the core on a second stream
    # (autotuned variant), and without the FP64 core (FP32 only)
    for key, meshes, kw in (("per_mesh_launch", [(N, L, lam)], dict(per_mesh=True, autotune=True)),
                            ("fp64_core_off", [(N, L, lam, bz.BZ_CORE_OFF)], dict(autotune=True)),
                            ("full_sum_schedule", [(N, L, lam)], dict(schedule="full"))):
        try:
            comp[key] = step_leg(torch, np, bz, meshes, [0] * nc, f0, wcache, **kw)
            if key == "fp64_core_off":
                c = bz.Collision(meshes, [0] * nc, "batched_f32", weights_cache=wcache)
                comp[key]["rel_l2_vs_fp64_plain"] = errs_of(c.project(c.collide(f0)))
                c.close()
        except Exception as exc:
            comp[key] = {"error": str(exc)}
    wcache.clear()
    col.close()
    torch.cuda.empty_cache()

    # ---- homogeneous relaxation (N=32) and the whole uneven batch --------
    for key, fn in (("relaxation_n32", lambda: relaxation_leg(torch, np, bz, W)),
                    ("uneven_batch_1024", lambda: uneven_leg(torch, np, bz, W, float(np.median(per_step))))):
        try:
            comp[key] = fn()
        except Exception as exc:
            comp[key] = {"error": str(exc)}
        torch.cuda.empty_cache()

    # ---- learned closure on the N=24 shock problem, and on the N=32 mesh of the metric
    if not args.no_closure:
        for key, kw in (("closure_shock_n24", {}),
                        ("closure_shock_n32", dict(N=32, L=8.0, snapshots=400, relax_cells=256))):
            try:
                comp[key] = closure_leg(args, torch, np, bz, W, **kw)
            except Exception as exc:
                comp[key] = {"error": str(exc)}
            torch.cuda.empty_cache()

    # ---- CPU oracle baseline ------------------------------------------
    cpu = None
    if not args.no_cpu:
        import oracle as O
        o = O.Oracle(N, L, lam)          # the weight quadrature is built before timing
        done, t0 = 0, time.perf_counter()
        while done < nc and (time.perf_counter() - t0) < args.cpu_seconds:
            o.collide(cells[done])
            done += 1
        el = time.perf_counter() - t0
        cpu = {"value": done / el, "unit": "cell-collision evals/s", "cores": O.num_threads(), "kind": "oracle",
               "value_per_core": done / el / max(O.num_threads(), 1), "cpu_model": cpu_model(),
               "sample": f"{done} of the {nc} N=32 cells, one FP64 evaluation each (transform, O(N^6) sum, "
                         f"inverse, projection), {el:.1f} s"}

    traffic = measured_traffic(nc)
    valu = measured_valu_insts(nc)
    kernel = "k_conv_cells_f32_multi (FP32 items + FP64 core items)" if one_launch else "k_conv_cells_f32<32>"
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-collision evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "step_ms": spread(np, per_step),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "N=32 cells of the seeded 1024-cell uneven batch, Heun RK2 step, batched FP32 "
                               "convolution with compensated accumulation and an FP64 low-frequency core, "
                               "FP64 projection",
                   "cells": nc, "N": N, "L": L, "lambda": lam, "dt_over_eps": dt_over_eps,
                   "evals_per_step": 2 * nc, "core_r2": info["core_r2"], "one_launch": one_launch},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "traffic_source": (TRAFFIC_FILE + " (rocprofv3 --pmc FETCH_SIZE, WRITE_SIZE on this kernel "
                                        "source and batch, scaled by a 1 GiB copy)") if traffic else None,
                     "kernel": kernel, "avg_launch_ms": conv_avg_ms, "launches": conv_launches,
                     "fp32_flops_per_launch": fp32_flops,
                     "fp32_slots_per_cell": slots, "slots_vs_full_sum_pairs": slots / P,
                     "issue_ceiling_frac": ISSUE_CEILING_FRAC,
                     "fp64_core_flops_per_launch": core_flops,
                     "frac_incl_fp64_core": (fp32_flops + core_flops) / (conv_avg_ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                     "effective_tflops": 10.0 * P * nc / (conv_avg_ms * 1e-3) / 1e12,
                     "traffic_gb_per_s": (traffic / (conv_avg_ms * 1e-3) / 1e9) if traffic else None,
                     "hbm_peak_gb_per_s": HBM_TBPS * 1e3,
                     "valu_insts_per_launch": valu,
                     # one wave64 VALU instruction per SIMD every 4 cycles (1024 SIMDs): the mean shader
                     # clock the launch needs at least to issue them in its measured time
                     "valu_issue_clock_ghz_min": (valu / 1024 * 4 / (conv_avg_ms * 1e-3) / 1e9) if valu else None},
        "cpu_baseline": cpu,
        "gpu_clock_idle_after_run": gpu_clocks(),
        "comparisons": comp,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

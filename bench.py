"""Benchmark: cell-collision evaluations per second at N=32 on one MI355X.

Workload: the N=32 cells (L=8, hard spheres) of the seeded 1024-cell uneven
draw (perturbed Maxwellians, rho ~ U[.5,2], |u| ~ U[0,1.5], T ~ U[.5,2]).
One bench step is one Heun (second-order Runge-Kutta) step of the space-
homogeneous equation for every cell of the batch: two collision evaluations
per cell (forward transform, batched FP32 convolution with compensated
accumulation, inverse transform, FP64 projection) and the Heun updates.

The JSON line also carries:
  roofline      the batched convolution kernel against the FP32 vector peak
                (its launches are timed with HIP events on the library's stream
                inside the timed region)
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same cells
  comparisons   the plain unbatched FP64 path on the same GPU, the batched
                FP64 path, and the relative L2 error of the FP32 result
                against the FP64 plain result for every cell
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
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector, published
HBM_TBPS = 8.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def conv_source_sha():
    with open(os.path.join(ROOT, "paper_1211_0540_amd", "csrc", "bz_conv.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(cells):
    """HBM bytes per launch of the batched N=32 kernel from the committed counter
    summary, if it was taken on the current kernel source and the same batch."""
    p = os.path.join(ROOT, "profiles", "conv_cells_f32_n32_traffic.json")
    try:
        with open(p) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_src_sha") != conv_source_sha() or d.get("cells") != cells:
        return None
    return d.get("traffic_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-run", action="store_true",
                    help="timed steps only (default kernel variant, no comparisons, no CPU leg)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        return 2

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
    f0 = torch.from_numpy(col.pack(cells)).to(dev)
    if args.profile_run:
        variant = bz.bz_batch_get_variant(col.batch, 0)
    else:
        variant = col.autotune(f0, reps=1)[0]
    log(f"convolution variant {variant}")

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
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        col.step(f, dt_over_eps)
    stop.record()
    torch.cuda.synchronize()
    bz.bz_batch_timer(col.batch, False)
    col.check()
    total_ms = start.elapsed_time(stop)
    conv_ms, conv_launches = bz.bz_batch_timer_read(col.batch)
    ms_step = total_ms / args.steps
    evals = 2 * nc * args.steps
    value = evals / (total_ms * 1e-3)
    conv_avg_ms = conv_ms / max(conv_launches, 1)
    achieved = 10.0 * P * nc / (conv_avg_ms * 1e-3) / 1e12
    log(f"step {ms_step:.3f} ms, {value:.0f} evals/s, conv {conv_avg_ms:.3f} ms/launch ({conv_launches} launches)")

    if args.copy_calibration:
        x = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()

    if args.profile_run:
        print(json.dumps({"profile_run": True, "ms_per_step": ms_step, "conv_avg_ms": conv_avg_ms,
                          "cells": nc}), flush=True)
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
    reps = 1
    for _ in range(reps):
        qq = plain.collide(f0)
        plain.project(qq)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / reps
    comp["plain_fp64_evals_per_s"] = nc / plain_s
    a = q32.cpu().numpy()
    b64 = q64.cpu().numpy()
    errs = [float(np.linalg.norm(x - y) / np.linalg.norm(y)) for x, y in zip(col.unpack(a), plain.unpack(b64))]
    comp["rel_l2_fp32_batched_vs_fp64_plain"] = {"median": float(np.median(errs)), "max": float(np.max(errs)),
                                                 "cells": nc}
    plain.close()
    # batched FP64
    b64c = bz.Collision([(N, L, lam)], [0] * nc, "batched_f64", weights_cache=wcache)
    qb = b64c.collide(f0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qb = b64c.collide(f0)
    b64c.project(qb)
    torch.cuda.synchronize()
    comp["batched_fp64_evals_per_s"] = nc / (time.perf_counter() - t0)
    b64c.close()
    comp["fp32_batched_step_evals_per_s"] = value
    comp["speedup_fp32_batched_vs_fp64_plain"] = value / comp["plain_fp64_evals_per_s"]
    wcache.clear()

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
               "sample": f"{done} of the {nc} N=32 cells, one FP64 evaluation each (transform, O(N^6) sum, "
                         f"inverse, projection), {el:.1f} s"}

    traffic = measured_traffic(nc)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-collision evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "N=32 cells of the seeded 1024-cell uneven batch, Heun RK2 step, batched FP32 "
                               "convolution with compensated accumulation + FP64 projection",
                   "cells": nc, "N": N, "L": L, "lambda": lam, "dt_over_eps": dt_over_eps,
                   "evals_per_step": 2 * nc, "variant": variant},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                     "kernel": "k_conv_cells_f32<32>", "flops_per_launch": 10.0 * P * nc,
                     "avg_launch_ms": conv_avg_ms, "launches": conv_launches},
        "cpu_baseline": cpu,
        "comparisons": comp,
    }
    print(json.dumps(out), flush=True)
    col.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

#!/usr/bin/env python3
"""Benchmark of the hot path: cell-updates/s of one 256^3 two-phase solve.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision f32|f64]

Workload: a 500-bubble cloud (centres uniform in a ball of radius 0.3 in the
unit cube, log-normal radii, median 0.015, sigma 0.1, clipped to +-20 %),
water/air stiffened gases, 0.0234 bar inside the cloud ramped to 100 bar
outside, on a 256^3 grid.  A step is one full time step of the solver:
three fused RHS + low-storage RK stages (the third with the CFL / QoI
reduction) and the per-step finalisation, all HIP kernels of libofm.so.  The
state is resident in HBM before timing starts; W warm-up steps, then K timed
steps.  value = 256^3 cells x K steps / wall time.

The JSON line also carries
  roofline     for the dominant kernel (the fused stage kernel): its average
               launch duration measured with HIP events on the stream it runs
               on, against the per-launch algorithmic bytes (HBM roofline) and
               the per-launch algorithmic flops (vector ALU roofline); `bound`
               names the roofline the kernel is closer to;
  cpu_baseline the serial FP64 oracle timed on this host's cores on a bounded
               sample of the same workload (one 64^3 box of the 256^3 cloud per
               process, 4 steps each);
  fp64         the same measurement with the stencil in double;
  weno3        the same measurement (float stencil, the tile tuned above) with
               the third-order reconstruction the paper also allows.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# vector ALU peak without packed FP32 (packed math is disabled in this
# build): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
VALU_PEAK_TFLOPS = {"f32": 78.6, "f64": 78.6}
# algorithmic words per cell and step of the fused stage kernel (nv = 7):
# stage 1 reads U, writes dU and U'; stage 2 reads U, dU, writes dU, U';
# stage 3 reads U, dU, writes U'  -> 10 nv words per step
WORDS_PER_CELL_STEP = 10 * 7
# algorithmic flops per cell and stage (3-D), counted from the operations of
# the scheme; see the design notes for the itemised count
FLOPS_PER_CELL_STAGE = 2650


PROFILE = os.path.join(ROOT, "profiles", "stage_kernel_cloud500_256cubed_f32.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1705_04374_amd", "csrc", "flow_kernels.hip")


def profiled_traffic(tile, n, precision):
    """HBM bytes per stage launch measured with rocprofv3 (FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy's counts), as recorded in the profile
    summary; None unless that summary is for the kernel source, tile and
    workload measured here."""
    import hashlib
    if precision != "f32" or n != 256 or tile is None or not os.path.exists(PROFILE):
        return None
    fields = {}
    with open(PROFILE) as f:
        for line in f:
            k, _, v = line.strip().partition(": ")
            if v:
                fields[k] = v.strip()
    with open(KERNEL_SOURCE, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    want = "%dx%dx%d" % (tile["tx"], tile["ty"], tile["zchunk"])
    if not sha.startswith(fields.get("kernel_source_sha256_prefix", "-")) or fields.get("tile") != want:
        return None
    return float(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cloud", default="cloud500", choices=["cloud500", "cloud50"],
                    help="cloud of the solve (cloud50: 50 bubbles in a ball of 0.25)")
    ap.add_argument("--weno-order", type=int, default=5, choices=[3, 5],
                    help="reconstruction of the timed solve (3: the third-order WENO the paper also allows)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 side measurement")
    ap.add_argument("--no-weno3", action="store_true", help="skip the WENO3 side measurement")
    ap.add_argument("--nn", action="store_true",
                    help="instead: forward pass of the learned level over 65 536 sets of 500 bubbles (one JSON line)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-tune", action="store_true", help="use the default tile instead of autotuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 1 GiB device copy three times (reference for HBM byte counters)")
    return ap.parse_args()


def measure(ctx, capi, cfg, bub, precision, steps, warmup, tune=True):
    import torch
    from paper_1705_04374_amd.state import alloc_state
    spec = capi.make_spec(cfg, precision, n_steps=steps)
    st, bufs = alloc_state(cfg, precision)
    tuned = None
    if tune:
        # the library's autotuner times every compiled tile / z-chunk on this
        # workload (2 steps each) and keeps the fastest; then start afresh
        capi.ofm_state_init(ctx, spec, bub, st)
        tuned = capi.ofm_autotune(ctx, spec, st, 2)
        print("autotune %s: %s" % (precision, json.dumps(tuned)), file=sys.stderr, flush=True)
    capi.ofm_state_init(ctx, spec, bub, st)
    torch.cuda.synchronize()
    if warmup:
        capi.ofm_step(ctx, spec, st, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q, dts = capi.ofm_step(ctx, spec, st, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-launch durations of the stage kernel, events on its own stream
    capi.ofm_kernel_timing(ctx, True)
    capi.ofm_step(ctx, spec, st, 4)
    kt = capi.ofm_kernel_times(ctx)
    capi.ofm_kernel_timing(ctx, False)
    del bufs
    torch.cuda.empty_cache()
    return dict(wall=wall, q=q, kt=kt, tuned=tuned)


def nn_bench(a):
    """The learned level's inference at the scale of its OF-MLMC term: the
    set network's forward over 65 536 sets of 500 bubbles (features of 256
    sampled clouds, repeated), timed with events on the stream it runs on.
    Algorithmic flops per bubble row: the 4 -> 128 input layer (2 x 4 x 128)
    and the 128 x 128 layer on the matrix cores (2 x 128 x 128); the per-set
    head (2 x 128 x 128 + 2 x 128 x 5) is counted per set.  Roofline: dense
    BF16 matrix-core peak."""
    import numpy as np
    import torch
    from paper_1705_04374_amd import capi
    from workloads.configs import MASTER_SEED, cloud_spec
    cloud = cloud_spec("cloud500")
    ctx = capi.Context(0)
    n_sets, n_distinct = 65536, 256
    bub = [capi.ofm_sample_cloud(cloud, MASTER_SEED, 3, i) for i in range(n_distinct)]
    nb = cloud["n_bubbles"]
    b = torch.tensor(np.concatenate(bub), dtype=torch.float64, device="cuda")
    x0 = torch.empty((b.shape[0], 4), dtype=torch.float32, device="cuda")
    capi.ofm_nn_features(cloud, b, x0)
    x = x0.repeat(n_sets // n_distinct, 1).contiguous()
    off = torch.arange(0, (n_sets + 1) * nb, nb, dtype=torch.int32, device="cuda")
    y = torch.empty((n_sets, 5), dtype=torch.float32, device="cuda")
    net = capi.SetNet(ctx, 1.0 / nb, seed=MASTER_SEED)
    for _ in range(max(a.warmup, 1)):
        net.forward(x, off, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(a.steps, 1)
    e0.record()
    for _ in range(reps):
        net.forward(x, off, y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    rows = n_sets * nb
    flops = rows * (2 * 4 * 128 + 2 * 128 * 128) + n_sets * (2 * 128 * 128 + 2 * 128 * 5)
    tfl = flops / (ms * 1e-3) / 1e12
    assert bool(torch.isfinite(y).all())
    net.close()
    ctx.close()
    return {
        "metric": "learned-level forward: sets/s (65 536 sets of 500 bubbles)",
        "value": n_sets / (ms * 1e-3), "unit": "sets/s", "n_gpus": 1, "steps": reps, "warmup": max(a.warmup, 1),
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (features of 256 seeded 500-bubble clouds, repeated)",
        "config": {"workload": "set network 4-128-128 / sum pool / 128-128-5 forward, 65536 sets x 500 bubbles",
                   "rows": rows},
        "roofline": {"kernel": "ofm_nn_forward (phi_pool_kernel + head)", "bound": "mfma", "achieved": round(tfl, 2),
                     "peak": 2500.0, "unit": "TFLOP/s", "frac": round(tfl / 2500.0, 4), "traffic": None,
                     "algorithmic_flops_per_call": flops},
    }


def host_cpu():
    """(model name, cores this process may run on, logical CPUs of the host)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return model, usable, os.cpu_count()


def cpu_baseline(cfg, bub):
    """Serial FP64 oracle on P host cores, each advancing its own 64^3 box of
    the same 256^3 cloud by 4 steps (the rate counts every box cell; cells
    near the box sides see box ghosts, the arithmetic per cell is the same).
    P = the cores this process may run on, at most the job's share of the
    host given by OMP_NUM_THREADS when that is set (a shared GPU host gives
    each GPU's job a fixed share of its cores)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    model, usable, logical = host_cpu()
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    P = max(1, min(usable, share) if share > 0 else usable)
    n = cfg["n"]
    b = 64
    nst = 4
    rng_boxes = []
    for k in range(P):
        o = (n // 2 - b) + (k * 37) % max(1, n // 2)
        lo = (min(o, n - b), min((o + 11 * k) % (n - b), n - b), min((o + 23 * k) % (n - b), n - b))
        rng_boxes.append(lo)
    from oracle.flow import initial_reduction
    dt = 0.3 * (1.0 / n) / initial_reduction(cfg, bub)["s_max"]
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=P, mp_context=ctx) as ex:
        res = list(ex.map(_cpu_box, [(cfg, bub, lo, b, dt, nst) for lo in rng_boxes]))
    wall = time.perf_counter() - t0
    cells = sum(r[0] for r in res)
    step_s = max(r[1] for r in res)
    return dict(value=cells / step_s, unit="cell-updates/s", cores=P, kind="oracle",
                sample="%d processes x one %d^3 box of the %d^3 500-bubble cloud, %d FP64 steps each "
                       "(init excluded), wall %.1f s" % (P, b, n, nst, wall),
                per_core=cells / step_s / P, cpu_model=model, cores_usable=usable, host_logical_cpus=logical,
                job_core_share=share or None)


def _cpu_box(args):
    cfg, bub, lo, b, dt, nst = args
    import oracle.flow as OF
    box = (lo, (b, b, b))
    t0 = time.perf_counter()
    OF.box_steps(cfg, bub, box, [])
    t1 = time.perf_counter()
    OF.box_steps(cfg, bub, box, [dt] * nst)
    t2 = time.perf_counter()
    return (nst * b ** 3, (t2 - t1) - (t1 - t0))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(samples would shard across GPUs with one small all-reduce per OF-MLMC iteration; "
              "see the design notes). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if a.nn:
        print(json.dumps(nn_bench(a)), flush=True)
        return
    import torch
    from paper_1705_04374_amd import capi
    from workloads.configs import MASTER_SEED, cloud_spec, solver_config

    if a.calibrate_copy:
        # a plain copy of known size: 2^28 floats read and 2^28 written per launch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
        torch.cuda.empty_cache()
    n = a.n
    cfg = dict(solver_config(a.cloud, n), weno_order=a.weno_order)
    bub = capi.ofm_sample_cloud(cloud_spec(a.cloud), MASTER_SEED, 0, 0)
    ctx = capi.Context(0)
    cells = n ** 3
    r = measure(ctx, capi, cfg, bub, a.precision, a.steps, a.warmup, tune=not a.no_tune)
    ms_per_step = r["wall"] * 1e3 / a.steps
    value = cells * a.steps / r["wall"]
    kt = r["kt"]
    avg_ms = kt["total_ms"] / max(kt["launches"], 1)
    word = 4 if a.precision == "f32" else 8
    cells_per_launch = kt["cells"] / max(kt["launches"], 1)
    bytes_per_launch = cells_per_launch * WORDS_PER_CELL_STEP * word / 3.0
    flops_per_launch = cells_per_launch * FLOPS_PER_CELL_STAGE
    gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    tfl = flops_per_launch / (avg_ms * 1e-3) / 1e12
    hbm_frac = gbs / HBM_PEAK_GBS
    alu_frac = tfl / VALU_PEAK_TFLOPS[a.precision]
    bound = "alu" if alu_frac >= hbm_frac else "hbm"
    used = capi.ofm_tune_get(ctx, capi.OFM_F32 if a.precision == "f32" else capi.OFM_F64, 3, n)
    tile = {k: used[k] for k in ("tx", "ty", "zchunk")}
    traffic = profiled_traffic(tile, n, a.precision)
    roof = {
        "kernel": "stage_kernel (fused WENO5/HLLC RHS + LSRK3 stage, 3 launches per step)",
        "bound": bound,
        "achieved": round(tfl if bound == "alu" else gbs, 3),
        "peak": VALU_PEAK_TFLOPS[a.precision] if bound == "alu" else HBM_PEAK_GBS,
        "unit": "TFLOP/s" if bound == "alu" else "GB/s",
        "frac": round(alu_frac if bound == "alu" else hbm_frac, 4),
        "traffic": traffic,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
        "avg_launch_ms": round(avg_ms, 4),
        "tile": tile,
        "hbm": {"achieved_GBs": round(gbs, 1), "peak_GBs": HBM_PEAK_GBS, "frac": round(hbm_frac, 4),
                "algorithmic_bytes_per_launch": bytes_per_launch},
        "alu": {"achieved_TFLOPs": round(tfl, 2), "peak_TFLOPs": VALU_PEAK_TFLOPS[a.precision],
                "frac": round(alu_frac, 4), "algorithmic_flops_per_launch": flops_per_launch},
    }
    out = {
        "metric": "cell-updates/s at 256^3 (one 500-bubble cloud solve, 3-stage LSRK step incl. CFL/QoI reduction)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.precision,
        "data": "synthetic (seeded 500-bubble cloud, no dataset)",
        "config": {"workload": "%s single solve, %d^3, %s stencil, FP64 QoI/dt" % (a.cloud, n, a.precision),
                   "cells": cells, "bubbles": cloud_spec(a.cloud)["n_bubbles"], "status": r["q"]["status"], "steps_taken": r["q"]["steps"]},
        "roofline": roof,
    }
    if not a.no_fp64 and a.precision == "f32":
        r64 = measure(ctx, capi, cfg, bub, "f64", max(4, a.steps // 3), 1, tune=not a.no_tune)
        kt64 = r64["kt"]
        ms64 = kt64["total_ms"] / max(kt64["launches"], 1)
        c64 = kt64["cells"] / max(kt64["launches"], 1)
        out["fp64"] = {"value": cells * max(4, a.steps // 3) / r64["wall"], "unit": "cell-updates/s",
                       "avg_stage_launch_ms": round(ms64, 4),
                       "tile": None if r64["tuned"] is None else {k: r64["tuned"][k] for k in ("tx", "ty", "zchunk")},
                       "hbm_frac": round(c64 * WORDS_PER_CELL_STEP * 8 / 3.0 / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                       "alu_frac": round(c64 * FLOPS_PER_CELL_STAGE / (ms64 * 1e-3) / 1e12 / VALU_PEAK_TFLOPS["f64"], 4)}
    if not a.no_weno3 and a.precision == "f32":
        k3 = max(4, a.steps // 3)
        r3 = measure(ctx, capi, dict(cfg, weno_order=3), bub, "f32", k3, 1, tune=False)
        kt3 = r3["kt"]
        out["weno3"] = {"value": cells * k3 / r3["wall"], "unit": "cell-updates/s", "steps": k3,
                        "avg_stage_launch_ms": round(kt3["total_ms"] / max(kt3["launches"], 1), 4),
                        "status": r3["q"]["status"]}
    if not a.no_cpu:
        try:
            out["cpu_baseline"] = cpu_baseline(cfg, bub)
        except Exception as e:  # the baseline is reported, never required
            out["cpu_baseline"] = {"error": repr(e)}
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

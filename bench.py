#!/usr/bin/env python3
"""Throughput of the time-tiled acoustic-wave sweep on one MI355X.

One "step" is one pass of the hot path over one synthetic batch: the full
forward modelling of the 512^3 (+40-point absorbing layer = 592^3) space-order-8
layered-model problem for 1000 time steps (source injection, receiver
sampling, time-tiled sweep), with the inputs resident in HBM.  Reported:

* value: grid-point updates per second of that step with the tuned
  time-tiled schedule (Gpts/s = 592^3 * 1000 / wall);
* untiled: the same step with the single-step (untiled) sweep, and the ratio;
* adjoint_grad: the 256^3 (+40) so8 gradient problem (forward with
  checkpoints every 50 steps, tiled recompute, time-reversed adjoint with the
  imaging condition) for 2000 steps, in Gpts/s of forward time steps;
* roofline: the dominant kernel (time-tiled forward sweep) against HBM;
* cpu_baseline: the FP64 oracle on the host cores on a bounded sample.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_forward(op, w, wav, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        op.forward(w.nt, w.src_xyz, wav, w.rec_xyz)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(steps):
        e0.record(stream)
        op.forward(w.nt, w.src_xyz, wav, w.rec_xyz)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    return times


def cpu_baseline(w, budget_s=20.0):
    """FP64 oracle on the host: the same grid, model, order and source for a
    few time steps (bounded to ~budget_s of CPU work), as Gpts/s."""
    import oracle
    oracle.build(force=False)
    g = oracle.Grid(w.shape, w.spacing, w.dt, w.so, nbl=w.nbl, sigma_max=w.sigma_max)
    m = w.m.astype(np.float64)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    t0 = time.perf_counter()
    oracle.forward(g, m, 1, w.src_xyz, w.wavelet[:1].astype(np.float64), w.rec_xyz)
    t1 = time.perf_counter() - t0
    steps = max(1, min(50, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.forward(g, m, steps, w.src_xyz, w.wavelet[:steps].astype(np.float64), w.rec_xyz)
    dt = time.perf_counter() - t0
    return {"value": w.npts * steps / dt / 1e9, "unit": "Gpts/s", "cores": threads, "kind": "oracle",
            "sample": "%s: first %d of %d time steps on the full %s grid (FP64, OpenMP over points), "
                      "%.1f s" % (w.name, steps, w.nt, "x".join(map(str, w.shape)), dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="physical grid edge of the forward workload")
    ap.add_argument("--nt", type=int, default=1000)
    ap.add_argument("--T", type=int, default=0, help="time-tile depth (0: autotune)")
    ap.add_argument("--shape", type=int, default=0)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="small sizes for a functional check")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import (wave_autotune, wave_bytes_per_point, wave_flops_per_point,
                                           wave_scratch_bytes)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.quick:
        args.n, args.nt = 128, 100

    # ---------------------------------------------------------------- forward, tuned tiled schedule
    t0 = time.time()
    w = wi.c2(nt=args.nt, n=args.n)
    log("workload %s shape %s nt %d (%.1f s to generate)" % (w.name, w.shape, w.nt, time.time() - t0))
    m = torch.from_numpy(w.m).to(dev)
    wav = torch.from_numpy(w.wavelet).to(dev)
    op = WaveOp(w.shape, w.spacing, w.dt, w.so, m, nbl=w.nbl, sigma_max=w.sigma_max, time_tile=-1)
    if args.T > 0:
        op.set_schedule(args.T, 0, args.shape, 0)
    else:
        sc = op.scratch(wave_scratch_bytes(op.ctx, 40, 0, 0, 0, 0))
        best = wave_autotune(op.ctx, 40, 2, 8, sc)
        log("autotune -> schedule %s, %.3f ms/step" % (op.schedule(), best * 1e3))
    T, skew, shape, zch = op.schedule()
    times = timed_forward(op, w, wav, args.steps, args.warmup, stream)
    t_step = min(times)
    value = w.npts * w.nt / t_step / 1e9
    log("tiled T=%d shape=%d: %.3f s/step -> %.1f Gpts/s" % (T, shape, t_step, value))

    # ---------------------------------------------------------------- untiled reference sweep
    op.set_schedule(-1, 0, 0, 0)
    ut = timed_forward(op, w, wav, max(1, args.steps // 2), 1, stream)
    untiled = w.npts * w.nt / min(ut) / 1e9
    log("untiled: %.3f s/step -> %.1f Gpts/s" % (min(ut), untiled))
    op.set_schedule(T, skew, shape, zch)

    # ---------------------------------------------------------------- roofline of the tiled kernel
    # launches per step: ceil(nt / T) windows of the tiled kernel; the step's
    # other kernels (forcing table, two fills, receiver reduction) are < 0.1 %.
    launches = -(-w.nt // T) if T > 0 else w.nt
    t_launch = t_step / launches
    bpp = wave_bytes_per_point(T, 0)                     # algorithmic bytes per point-update
    pts_per_launch = w.npts * (T if T > 0 else 1)
    achieved = bpp * pts_per_launch / t_launch / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_tiled R=4 T=%d" % T, "bytes_per_point_update": bpp,
                "flops_per_point_update": wave_flops_per_point(3, w.so, 0),
                "avg_launch_ms": round(t_launch * 1e3, 4)}

    del op
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- adjoint gradient
    adj = None
    if not args.no_adjoint:
        n4, nt4 = (96, 200) if args.quick else (256, 2000)
        w4 = wi.c4(nt=nt4, n=n4)
        tr, init = w4["true"], w4["init"]
        K = w4["ckpt_every"]
        opt = WaveOp(tr.shape, tr.spacing, tr.dt, tr.so, torch.from_numpy(tr.m).to(dev), nbl=tr.nbl,
                     sigma_max=tr.sigma_max, time_tile=T if T > 0 else -1)
        dobs, _ = opt.forward(tr.nt, tr.src_xyz, torch.from_numpy(tr.wavelet).to(dev), tr.rec_xyz)
        del opt
        op4 = WaveOp(init.shape, init.spacing, init.dt, init.so, torch.from_numpy(init.m).to(dev), nbl=init.nbl,
                     sigma_max=init.sigma_max, time_tile=T if T > 0 else -1)
        wv4 = torch.from_numpy(init.wavelet).to(dev)
        gtimes = []
        for it in range(2):
            torch.cuda.synchronize()
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            rec, _ = op4.forward(init.nt, init.src_xyz, wv4, init.rec_xyz, ckpt_every=K, adjoint_scratch=True)
            resid = rec - dobs
            e1.record(stream)
            gm, _ = op4.adjoint_grad(init.nt, init.src_xyz, wv4, init.rec_xyz, resid, K, reuse=True)
            e2.record(stream)
            e2.synchronize()
            gtimes.append((e0.elapsed_time(e1) * 1e-3, e1.elapsed_time(e2) * 1e-3))
        tf, ta = min(g[0] for g in gtimes), min(g[1] for g in gtimes)
        adj = {"workload": "c4_256cube_so8 (+40 layer = %s), nt=%d, checkpoints every %d"
                           % ("x".join(map(str, init.shape)), init.nt, K),
               "value": round(init.npts * init.nt / (tf + ta) / 1e9, 2), "unit": "Gpts/s",
               "forward_with_checkpoints_s": round(tf, 4), "recompute_plus_adjoint_s": round(ta, 4),
               "adjoint_only_gpts": round(init.npts * init.nt / ta / 1e9, 2),
               "grad_finite": bool(torch.isfinite(gm).all().item())}
        log("gradient: fwd %.3f s + adjoint %.3f s" % (tf, ta))
        del op4
        torch.cuda.empty_cache()

    cpu = None if args.no_cpu else cpu_baseline(w)

    line = {
        "metric": "Gpts/s fwd & adjoint-grad vs untiled sweep; % HBM roofline (1 MI355X)",
        "value": round(value, 2), "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "shape": list(w.shape), "physical": [args.n] * 3, "nbl": w.nbl,
                   "space_order": w.so, "nt": w.nt, "schedule": {"T": T, "skew": skew, "tile_shape": shape,
                                                                  "zchunks": zch}},
        "untiled": {"value": round(untiled, 2), "ms_per_step": round(min(ut) * 1e3, 3)},
        "speedup_vs_untiled": round(value / untiled, 3),
        "adjoint_grad": adj,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

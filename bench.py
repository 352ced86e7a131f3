#!/usr/bin/env python3
"""Throughput of the time-tiled acoustic-wave sweep on one MI355X.

One "step" is one pass of the hot path over one synthetic batch: the full
forward modelling of the 512^3 (+40-point absorbing layer = 592^3)
space-order-8 layered-model problem for 1000 time steps (source injection,
receiver sampling, the sweep), with every input resident in HBM.  Reported
on one JSON line (progress goes to stderr):

* value: grid-point updates per second of that step with the autotuned
  schedule (time-tile depth T, tile shape, axis-0 segments; the untiled sweep
  is one of the candidates), Gpts/s = 592^3 * 1000 * K / time of K steps;
* untiled: the same step with the single-step sweep (its segment count tuned
  the same way), and the ratio of the two;
* adjoint_grad: the 256^3 (+40) space-order-8 gradient problem (forward with
  checkpoints every 50 steps, recompute of each segment, time-reversed
  adjoint with the imaging condition) for 2000 steps, tiled and untiled;
* roofline: the dominant kernel of the step against HBM bandwidth, with the
  HBM traffic read from hardware counters when a matching record exists;
* ai: the arithmetic intensity measured from those counters beside the
  naive and tight estimators of the time-tiling intensity model;
* batch: 32 independent shots (128^3..320^3, orders 4/8, 800 steps), forward
  and gradient through one captured sequence, against the shots one by one;
* tiling_by_order: the best time-tiled against the best untiled schedule on
  the same 592^3 layered workload at space orders 2, 4 and 8 (100 steps);
* laplace: the paper's second workload, explicit diffusion on 500^3 x 32
  and 600^3 x 16 steps at space orders 2..16, default, best untiled and best
  time-tiled schedule with their algorithmic HBM rates;
* point_source_64: the 64^3 space-order-4 100-step problem, untiled,
  register-tiled T = 1, 2, 4 and skewed, each with its roofline fraction
  (the working set fits the last-level cache);
* depth_sweep: the headline workload at every time-tile depth T = 1..8,
  register-tiled (where built) and skewed, with algorithmic rates;
* smooth_768: the 768^3 (+40 = 848^3) smooth-model problem at space orders
  12 and 16 (500 steps), autotuned, untiled and best time-tiled;
* wave2d: 16384^2 at space orders 2, 4, 8 (100 steps), untiled against the
  best register-tiled and skewed schedules;
* two_level_laplace: the Laplace operator with a two-level time dependence
  (two-step Adams-Bashforth) on 500^3 x 32 steps, untiled against skewed,
  beside the one-level step at the same time step;
* cpu_baseline: the FP64 oracle on the host cores on bounded samples.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
L2_FLOATS = 4 * 2 ** 20 // 4          # 4 MiB L2 per XCD
MALL_FLOATS = 256 * 2 ** 20 // 4      # 256 MiB last-level (Infinity) cache


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sources_sha() -> str:
    """Digest of the sources that define the single-context sweep kernels
    (kernel templates, per-point arithmetic, instantiation units, build
    flags): a counter record is only used while they are unchanged."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1806_08299_amd", "csrc")
    files = [os.path.join(csrc, f) for f in ("wave_kernels.h", "wave_device.h", "wave_inst.inc")]
    files += sorted(glob.glob(os.path.join(csrc, "wave_r*_m*.hip")))
    files.append(os.path.join(ROOT, "paper_1806_08299_amd", "build.py"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(workload: str, sched) -> dict | None:
    """Counter record (profiles/hbm_traffic.txt) for this workload, schedule
    and kernel sources, or None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    sha = kernel_sources_sha()
    T, shape, zc, slab = sched[0], sched[2], sched[3], sched[5]
    for line in open(path):
        if not line.startswith("record "):
            continue
        kv = dict(f.split("=", 1) for f in line.split()[1:])
        if (kv.get("workload") == workload and int(kv["T"]) == T and int(kv["shape"]) == shape
                and int(kv["zchunks"]) == zc and int(kv.get("slab", 0)) == slab and kv.get("sources") == sha):
            return kv
    return None


def run_steps(op, w, wav, steps, stream):
    """K forward steps between two device synchronisations; returns seconds
    (HIP events on the sweep's stream) and the host wall time."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        op.forward(w.nt, w.src_xyz, wav, w.rec_xyz)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3, time.perf_counter() - t0


def tune_untiled(op, trial_steps=40, repeats=2):
    """Best axis-0 segment count for the untiled sweep (short trials)."""
    import torch
    best = (1e30, 0)
    for zc in (0, 1, 2, 4, 8, 12, 16, 24, 32):
        op.set_schedule(-1, 0, 0, zc)
        op.forward(trial_steps)
        torch.cuda.synchronize()
        t = 1e30
        for _ in range(repeats):
            t0 = time.perf_counter()
            op.forward(trial_steps)
            torch.cuda.synchronize()
            t = min(t, time.perf_counter() - t0)
        best = min(best, (t, zc))
    op.set_schedule(-1, 0, 0, best[1])
    return best[1]


def autotune(op, w, trial_steps=40):
    """The autotuner with trial forwards that carry the workload's source and
    receivers."""
    best = op.autotune(trial_steps, 2, 8, w.src_xyz, w.rec_xyz)
    op._scratch = None
    return best


def guided_vs_exhaustive(op, w, wav, stream, trial_steps=40, keep=10):
    """The estimator-guided autotuner against the exhaustive one on the same
    context: candidates timed, tuning wall time, and the rate of each kept
    schedule over the full run."""
    import torch
    from paper_1806_08299_amd.wave import wave_autotune_points, wave_autotune_scratch_bytes
    out = {}
    sc = op.scratch(wave_autotune_scratch_bytes(op.ctx, trial_steps, len(w.src_xyz), len(w.rec_xyz)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wave_autotune_points(op.ctx, trial_steps, 2, 8, 0, w.src_xyz, w.rec_xyz, sc)
    t_ex = time.perf_counter() - t0
    ex = op.schedule()
    out["exhaustive"] = {"schedule": sched_dict(ex), "tuning_s": round(t_ex, 2),
                         "value": round(_rate(op, w.nt, w, wav, stream, 1), 1)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, n = wave_autotune_points(op.ctx, trial_steps, 2, 8, keep, w.src_xyz, w.rec_xyz, sc)
    t_gd = time.perf_counter() - t0
    gd = op.schedule()
    out["guided"] = {"schedule": sched_dict(gd), "tuning_s": round(t_gd, 2), "timed_candidates": n, "keep": keep,
                     "value": round(_rate(op, w.nt, w, wav, stream, 1), 1)}
    out["guided_over_exhaustive"] = round(out["guided"]["value"] / out["exhaustive"]["value"], 3)
    op._scratch = None
    return out


def kernel_name(sched, so) -> str:
    T, slab, tile = sched[0], sched[5], sched[4]
    if T < 0:
        return "k_untiled R=%d (single-step sweep)" % (so // 2)
    if slab > 0:
        return "k_untiled R=%d (single-step sweep) in the skewed schedule, T=%d, slab %d" % (so // 2, T, slab)
    return "k_tiled R=%d T=%d tile %dx%d" % (so // 2, T, tile[0], tile[1])


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _physical_cores(cpus) -> int:
    """Distinct (package, core) pairs among the logical CPUs `cpus`, from
    /proc/cpuinfo (0 if it cannot be read)."""
    cur, pairs = {}, {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" not in line:
                if "processor" in cur:
                    pairs[int(cur["processor"])] = (cur.get("physical id", "0"), cur.get("core id", cur["processor"]))
                cur = {}
                continue
            k, v = (x.strip() for x in line.split(":", 1))
            cur[k] = v
        if "processor" in cur:
            pairs[int(cur["processor"])] = (cur.get("physical id", "0"), cur.get("core id", cur["processor"]))
    except OSError:
        return 0
    return len({pairs[c] for c in cpus if c in pairs})


_ORACLE_ONE_THREAD = r"""
import sys, time, json
sys.path.insert(0, sys.argv[1])
import numpy as np, oracle, waveinputs as wi
w = wi.layered_512(nt=1, n=int(sys.argv[2]))
g = oracle.Grid(w.shape, w.spacing, w.dt, w.so, nbl=w.nbl, sigma_max=w.sigma_max)
m = w.m.astype(np.float64)
t0 = time.perf_counter()
oracle.forward(g, m, 1, w.src_xyz, w.wavelet[:1].astype(np.float64), w.rec_xyz)
print(json.dumps({"s": time.perf_counter() - t0, "npts": int(w.npts)}))
"""


def cpu_baseline(w, budget_s=20.0, n=512, quick=False):
    """FP64 oracle on the host: the headline grid, model, order and source for
    a few time steps (bounded to ~budget_s of CPU work), as Gpts/s, on all the
    threads OpenMP is given; one step of it on one thread (a child process
    with OMP_NUM_THREADS=1); the 64^3 point-source problem complete; the
    gradient problem (forward with history, adjoint with imaging) on a bounded
    slice of its steps."""
    import subprocess
    import oracle
    import waveinputs as wi
    oracle.build(force=False)
    g = oracle.Grid(w.shape, w.spacing, w.dt, w.so, nbl=w.nbl, sigma_max=w.sigma_max)
    m = w.m.astype(np.float64)
    cpus = sorted(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else list(range(os.cpu_count()))
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(cpus)
    t0 = time.perf_counter()
    oracle.forward(g, m, 1, w.src_xyz, w.wavelet[:1].astype(np.float64), w.rec_xyz)
    t1 = time.perf_counter() - t0
    steps = max(1, min(50, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    oracle.forward(g, m, steps, w.src_xyz, w.wavelet[:steps].astype(np.float64), w.rec_xyz)
    dt = time.perf_counter() - t0
    out = {"value": round(w.npts * steps / dt / 1e9, 4), "unit": "Gpts/s", "cores": threads, "kind": "oracle",
           "sample": "%s: first %d of %d time steps on the full %s grid (FP64, OpenMP over axis 0), "
                     "%.1f s" % (w.name, steps, w.nt, "x".join(map(str, w.shape)), dt),
           "threads": threads, "physical_cores": _physical_cores(cpus), "logical_cpus_available": len(cpus),
           "cpu_model": _cpu_model()}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", _ORACLE_ONE_THREAD, ROOT, str(n)], env=env, capture_output=True,
                           text=True, timeout=300)
        one = json.loads(r.stdout.strip().splitlines()[-1])
        out["single_thread_value"] = round(one["npts"] / one["s"] / 1e9, 5)
        out["single_thread_sample"] = "one time step of the same grid on one thread, %.1f s" % one["s"]
    except Exception as e:   # the single-thread figure is context only
        out["single_thread_value"] = None
        out["single_thread_sample"] = "not measured: %s" % type(e).__name__
    # the 64^3 point-source problem, complete
    c1 = wi.point_source_64()
    g1 = oracle.Grid(c1.shape, c1.spacing, c1.dt, c1.so)
    t0 = time.perf_counter()
    oracle.forward(g1, c1.m.astype(np.float64), c1.nt, c1.src_xyz, c1.wavelet.astype(np.float64), c1.rec_xyz)
    d1 = time.perf_counter() - t0
    out["point_source_64"] = {"value": round(c1.npts * c1.nt / d1 / 1e9, 4), "unit": "Gpts/s",
                              "sample": "complete: %d steps on 64^3, %.2f s" % (c1.nt, d1)}
    # the gradient problem: forward with history + adjoint with imaging on a
    # slice of its steps (the complete 2000-step run takes about 15 CPU-minutes)
    n4 = 96 if quick else 256
    G = wi.gradient_256(nt=2000, n=n4)["init"]
    g4 = oracle.Grid(G.shape, G.spacing, G.dt, G.so, nbl=G.nbl, sigma_max=G.sigma_max)
    k = 12
    m4 = G.m.astype(np.float64)
    t0 = time.perf_counter()
    fw = oracle.forward(g4, m4, k, G.src_xyz, G.wavelet[:k].astype(np.float64), G.rec_xyz, want_hist=True)
    oracle.adjoint(g4, m4, k, np.ones_like(fw["rec"]), hist=fw["hist"], src_xyz=G.src_xyz, rec_xyz=G.rec_xyz)
    d4 = time.perf_counter() - t0
    out["gradient_256"] = {"value": round(G.npts * k / d4 / 1e9, 4), "unit": "Gpts/s (forward + adjoint per step)",
                           "sample": "%d of %d steps of forward with history and adjoint with imaging on %s, "
                                     "%.1f s" % (k, G.nt, "x".join(map(str, G.shape)), d4)}
    return out


def gradient_bench(args, dev, stream):
    """Forward with checkpoints + recompute/adjoint/imaging on the 256^3 so8
    gradient problem, with the autotuned and with the untiled schedule."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import wave_bytes_per_point
    n4, nt4 = (96, 200) if args.quick else (256, 2000)
    w4 = wi.gradient_256(nt=nt4, n=n4)
    tr, init = w4["true"], w4["init"]
    K = w4["ckpt_every"]
    opt = WaveOp(tr.shape, tr.spacing, tr.dt, tr.so, torch.from_numpy(tr.m).to(dev), nbl=tr.nbl,
                 sigma_max=tr.sigma_max, time_tile=-1)
    dobs, _ = opt.forward(tr.nt, tr.src_xyz, torch.from_numpy(tr.wavelet).to(dev), tr.rec_xyz)
    del opt
    op = WaveOp(init.shape, init.spacing, init.dt, init.so, torch.from_numpy(init.m).to(dev), nbl=init.nbl,
                sigma_max=init.sigma_max, time_tile=-1)
    wv = torch.from_numpy(init.wavelet).to(dev)
    if args.T != 0:     # a schedule pinned on the command line (profiling runs) instead of the autotuner's
        op.set_schedule(args.T, 0, args.shape if args.slab == 0 else 0, args.zchunks, slab=args.slab)
    else:
        op.autotune_gradient(40, 2, 8, init.src_xyz, init.rec_xyz, ckpt_every=20)
        op._scratch = None
    tuned = op.schedule()
    out = {"workload": "%s, model %s, nt=%d, checkpoints every %d"
                       % (init.name, "x".join(map(str, init.shape)), init.nt, K), "unit": "Gpts/s"}

    def one(sched, keep=0):
        op.set_schedule(*sched)
        best = None
        for _ in range(2):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            torch.cuda.synchronize()
            e0.record(stream)
            rec, _ = op.forward(init.nt, init.src_xyz, wv, init.rec_xyz, ckpt_every=K, adjoint_scratch=True,
                                keep_segments=keep)
            resid = rec - dobs
            e1.record(stream)
            gm, _ = op.adjoint_grad(init.nt, init.src_xyz, wv, init.rec_xyz, resid, K, reuse=True)
            e2.record(stream)
            torch.cuda.synchronize()
            t = (e0.elapsed_time(e1) * 1e-3, e1.elapsed_time(e2) * 1e-3)
            if best is None or sum(t) < sum(best):
                best = t
        return best, gm

    (tf, ta), gm = one(tuned)
    out.update({"schedule": sched_dict(tuned),
                "value": round(init.npts * init.nt / (tf + ta) / 1e9, 2),
                "forward_with_checkpoints_s": round(tf, 4), "recompute_plus_adjoint_s": round(ta, 4),
                "grad_finite": bool(torch.isfinite(gm).all().item())})
    # Roofline of the two phases: algorithmic bytes of their sweeps (forward
    # 16 B or 20/T B per point-update; recompute storing the history,
    # recompute_bpp; adjoint with imaging + 4 + 8/T B) over the phase's
    # HIP-event time; the
    # per-kernel split is in profiles/gradient_kernels_const2000_256cube_so8.txt.
    T = tuned[0]
    b_f, b_a = wave_bytes_per_point(T, 0), wave_bytes_per_point(T, 2)
    b_h = recompute_bpp(tuned)
    restore = 0.0                                 # the recompute reads its checkpoint in place
    nseg = -(-init.nt // K)
    fwd_bytes = (b_f * init.nt + 8.0 * nseg) * init.npts            # + checkpoint copies (read + write a level)
    adj_bytes = ((b_h + b_a) * init.nt + restore * nseg) * init.npts
    out["adjoint_bytes_per_point_update"] = b_a
    out["history_bytes_per_point_update"] = b_h
    out["roofline"] = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
                       "forward_achieved": round(fwd_bytes / tf / 1e9, 1),
                       "forward_frac": round(fwd_bytes / tf / 1e9 / HBM_PEAK_GBS, 4),
                       "recompute_adjoint_achieved": round(adj_bytes / ta / 1e9, 1),
                       "recompute_adjoint_frac": round(adj_bytes / ta / 1e9 / HBM_PEAK_GBS, 4),
                       "bytes": "forward %.0f + checkpoint copies; recompute %.0f + adjoint %.0f B per point-update"
                                % (b_f, b_h, b_a)}
    log("gradient %s: fwd %.3f s + recompute/adjoint %.3f s" % (tuned, tf, ta))
    out["kept_history"] = kept_history_leg(op, init, K, one, tuned, gm, (tf, ta), (b_f, b_h, b_a))
    if not args.no_untiled:
        (uf, ua), _ = one((-1, 0, 0, tuned[3] if tuned[0] < 0 else 0))
        out["untiled"] = {"value": round(init.npts * init.nt / (uf + ua) / 1e9, 2),
                          "forward_with_checkpoints_s": round(uf, 4), "recompute_plus_adjoint_s": round(ua, 4)}
        out["speedup_vs_untiled"] = round((uf + ua) / (tf + ta), 3)
        log("gradient untiled: fwd %.3f s + recompute/adjoint %.3f s" % (uf, ua))
    del op
    torch.cuda.empty_cache()
    if not args.no_untiled:
        out["by_order"] = gradient_orders(init, dev, stream, 200 if args.quick else 400, K)
    return out


def recompute_bpp(sched):
    """Algorithmic bytes per point-update of a step that stores the history:
    every schedule runs out of place straight into the history slots, reading
    u^n, u^{n-1} and b once per launch and writing every level once: 12/T + 4 B
    for a register tile of depth T, 16 for a single-step launch (the untiled
    sweep and the skewed schedule's slab steps)."""
    T, slab = sched[0], sched[5]
    return 16.0 if (T < 1 or slab > 0) else 12.0 / T + 4.0


def kept_history_leg(op, init, K, one, sched, gm_ref, t_ref, bpp):
    """The same gradient with the history of as many last checkpoint segments
    as the free HBM holds kept from the forward (wave_forward with scratch
    beyond the adjoint's layout): those segments skip their recompute
    (recompute_bpp), and the forward writes their levels straight into the
    history slots."""
    import torch
    from paper_1806_08299_amd.wave import wave_history_segment_bytes, wave_last_kept_segments, wave_scratch_bytes
    op._scratch = None
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    seg = wave_history_segment_bytes(op.ctx, K)
    base = wave_scratch_bytes(op.ctx, init.nt, len(init.src_xyz), len(init.rec_xyz), K, 1)
    nseg = -(-init.nt // K)
    keep = int(max(0, min(nseg, (free - base - (6 << 30)) // seg)))
    while True:
        try:
            (kf, ka), gm = one(sched, keep)
            break
        except torch.cuda.OutOfMemoryError:    # the free figure was optimistic: ask for half
            op._scratch = None
            torch.cuda.empty_cache()
            keep //= 2
            log("kept history: out of memory, retrying with %d segments" % keep)
            if keep == 0:
                return {"skipped": "no scratch for kept history"}
    kept = wave_last_kept_segments(op.ctx)
    same = bool(torch.equal(gm, gm_ref))
    op._scratch = None
    torch.cuda.empty_cache()
    b_f, b_h, b_a = bpp
    ks = max(0, init.nt - (nseg - kept) * K)                       # steps in kept segments
    b_k = b_h                                       # kept forward steps store the history as the recompute does
    restore = 0.0                                   # the recompute reads its checkpoint in place
    fwd_bytes = (b_f * (init.nt - ks) + b_k * ks + 8.0 * (nseg - kept)) * init.npts
    adj_bytes = (b_h * (init.nt - ks) + b_a * init.nt + restore * (nseg - kept)) * init.npts
    log("gradient, history of %d of %d segments kept: fwd %.3f s + recompute/adjoint %.3f s" % (kept, nseg, kf, ka))
    return {"segments_kept": kept, "segments": nseg, "scratch_GB": round((base + keep * seg) / 1e9, 1),
            "value": round(init.npts * init.nt / (kf + ka) / 1e9, 2),
            "forward_with_checkpoints_s": round(kf, 4), "recompute_plus_adjoint_s": round(ka, 4),
            "speedup_vs_full_recompute": round(sum(t_ref) / (kf + ka), 3),
            "bitwise_equal_to_full_recompute": same,
            "forward_achieved_GBs": round(fwd_bytes / kf / 1e9, 1),
            "recompute_adjoint_achieved_GBs": round(adj_bytes / ka / 1e9, 1)}


def gradient_orders(init, dev, stream, nt, K):
    """The same gradient problem (model, geometry, dt) at space orders 2 and
    4 over nt steps: the schedule of the gradient autotuner
    (wave_autotune_gradient) and, for reference, the forward autotuner's,
    against the untiled sweep.  The time-tiled adjoint carries each point's
    imaging sum across its window in registers, so the gradient is read and
    written once per window."""
    import torch
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import wave_bytes_per_point
    wv = torch.from_numpy(np.ascontiguousarray(init.wavelet[:nt])).to(dev)
    rows = []
    for so in (2, 4):
        op = WaveOp(init.shape, init.spacing, init.dt, so, torch.from_numpy(init.m).to(dev), nbl=init.nbl,
                    sigma_max=init.sigma_max, time_tile=-1)
        rec0, _ = op.forward(nt, init.src_xyz, wv, init.rec_xyz)
        resid = rec0.clone()

        def one(sched, keep=0):
            op.set_schedule(*sched)
            best, gm = None, None
            for _ in range(2):
                e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
                torch.cuda.synchronize()
                e0.record(stream)
                op.forward(nt, init.src_xyz, wv, init.rec_xyz, ckpt_every=K, adjoint_scratch=True,
                           keep_segments=keep)
                e1.record(stream)
                gm, _ = op.adjoint_grad(nt, init.src_xyz, wv, init.rec_xyz, resid, K, reuse=True)
                e2.record(stream)
                torch.cuda.synchronize()
                t = (e0.elapsed_time(e1) * 1e-3, e1.elapsed_time(e2) * 1e-3)
                if best is None or sum(t) < sum(best):
                    best = t
            return best, gm.cpu()

        (uf, ua), gu = one((-1, 0, 0, 0))
        # the forward autotuner ranks schedules by the forward alone, while the
        # adjoint's kernels hold more registers (some spill where the forward's
        # do not): its choice for reference, then the gradient autotuner's
        autotune(op, init)
        auto = op.schedule()
        (af, aa), ga = one(auto)
        op.autotune_gradient(40, 2, 8, init.src_xyz, init.rec_xyz, ckpt_every=20)
        op._scratch = None
        tuned = op.schedule()
        (tf, ta), gt = one(tuned)
        # every segment's history kept from the forward (8 x 50 levels fit)
        nseg = -(-nt // K)
        (kf, ka), gk = one(tuned, nseg)
        (kuf, kua), gku = one((-1, 0, 0, 0), nseg)
        op._scratch = None
        T = tuned[0]
        rows.append({"space_order": so, "nt": nt, "schedule": sched_dict(tuned),
                     "forward_autotuned_schedule": sched_dict(auto),
                     "forward_autotuned_value": round(init.npts * nt / (af + aa) / 1e9, 2),
                     "value": round(init.npts * nt / (tf + ta) / 1e9, 2),
                     "untiled_value": round(init.npts * nt / (uf + ua) / 1e9, 2),
                     "speedup_vs_untiled": round((uf + ua) / (tf + ta), 3),
                     "adjoint_speedup_vs_untiled": round(ua / ta, 3),
                     "adjoint_bytes_per_point_update": wave_bytes_per_point(T, 2),
                     "bitwise_equal_to_untiled": bool(torch.equal(gt, gu)),
                     "forward_with_checkpoints_s": round(tf, 4), "recompute_plus_adjoint_s": round(ta, 4),
                     "untiled_forward_s": round(uf, 4), "untiled_recompute_plus_adjoint_s": round(ua, 4),
                     "kept_history": {"segments_kept": nseg,
                                      "value": round(init.npts * nt / (kf + ka) / 1e9, 2),
                                      "untiled_value": round(init.npts * nt / (kuf + kua) / 1e9, 2),
                                      "speedup_vs_untiled": round((kuf + kua) / (kf + ka), 3),
                                      "speedup_vs_full_recompute": round((tf + ta) / (kf + ka), 3),
                                      "bitwise_equal": bool(torch.equal(gk, gt) and torch.equal(gku, gu)),
                                      "forward_s": round(kf, 4), "adjoint_s": round(ka, 4)}})
        log("gradient so%d: %s fwd %.3f + adj %.3f s, untiled %.3f + %.3f s (%.2fx); history kept: %.3f + %.3f s, "
            "untiled %.3f + %.3f s" % (so, tuned, tf, ta, uf, ua, (uf + ua) / (tf + ta), kf, ka, kuf, kua))
        del op
        torch.cuda.empty_cache()
    return rows


def batch_bench(args, dev, stream):
    """32 independent shots (128^3..320^3, space orders 4/8, 800 steps):
    forward and gradient through one captured, merged sequence (wave_batch),
    against the same shots run one after another."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import ShotBatch, WaveOp
    from paper_1806_08299_amd.wave import wave_bytes_per_point
    if args.quick:
        S = wi.shot_batch(nshots=6, nt=100, sizes=[(64 + 16 * (i % 3), 64, 80) for i in range(6)], workers=8)
    else:
        S = wi.shot_batch(workers=16)
    nt = S[0].nt
    K = 40                                   # ~sqrt(2 nt) checkpoints
    ops, wavs = [], []
    for w in S:
        op = WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).to(dev), nbl=w.nbl,
                    sigma_max=w.sigma_max, time_tile=-1)
        op.autotune(20, 1, 16, w.src_xyz, w.rec_xyz)
        if op.schedule().T > 2 and op.schedule().slab == 0:   # batched register tiles: T <= 2
            op.autotune(20, 1, 2, w.src_xyz, w.rec_xyz)
        op._scratch = None
        ops.append(op)
        wavs.append(torch.from_numpy(w.wavelet).to(dev))
    npts = sum(w.npts for w in S)
    scheds = {}
    for op in ops:
        sc_ = op.schedule()
        key = "T=%d tile=%dx%d slab=%d" % (sc_.T, sc_.tile[0], sc_.tile[1], sc_.slab)
        scheds[key] = scheds.get(key, 0) + 1

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e-3, out

    # one after another (single-context calls)
    def seq_forward():
        return [op.forward(nt, w.src_xyz, wv, w.rec_xyz)[0] for op, w, wv in zip(ops, S, wavs)]
    seq_forward()
    t_seq, recs_seq = timed(seq_forward)
    dobs = [(0.5 * r).contiguous() for r in recs_seq]

    def seq_grad():
        out = []
        for op, w, wv, d in zip(ops, S, wavs, dobs):
            rec, _ = op.forward(nt, w.src_xyz, wv, w.rec_xyz, ckpt_every=K, adjoint_scratch=True)
            gm, _ = op.adjoint_grad(nt, w.src_xyz, wv, w.rec_xyz, rec - d, K, want_grad_wavelet=False, reuse=True)
            op._scratch = None               # release before the next shot
            torch.cuda.empty_cache()
            out.append(gm)
        return out
    # best of two calls (the first gradient calls of a process ran up to 7 %
    # slower, batched and sequential alike)
    tg_seq = min(timed(seq_grad)[0] for _ in range(2))
    torch.cuda.empty_cache()
    log("batch: %d shots, %.1f Mpts, sequential forward %.3f s, gradient %.3f s" % (len(S), npts / 1e6, t_seq, tg_seq))

    # batched: first call records and captures, the timed call replays
    B = ShotBatch(ops, nt, [w.src_xyz for w in S], [w.rec_xyz for w in S])
    t_first, _ = timed(lambda: B.run(wavs))
    t_fwd, (recs_b, _) = timed(lambda: B.run(wavs))
    same_fwd = all(torch.equal(a, b) for a, b in zip(recs_b, recs_seq))
    del B
    torch.cuda.empty_cache()
    G = ShotBatch(ops, nt, [w.src_xyz for w in S], [w.rec_xyz for w in S], ckpt_every=K, gradient=True)
    tg_first, _ = timed(lambda: G.run(wavs, dobs))
    tg, (_, grads) = timed(lambda: G.run(wavs, dobs))
    tg = min(tg, timed(lambda: G.run(wavs, dobs))[0])
    finite = all(bool(torch.isfinite(g).all().item()) for g in grads)
    del G
    torch.cuda.empty_cache()
    # the other branch layout: one graph branch for all radii in the forward
    # (no side-by-side launches of different orders), one per radius in the
    # gradient
    os.environ["WAVE_BATCH_BRANCHES"] = "0"
    try:
        B1 = ShotBatch(ops, nt, [w.src_xyz for w in S], [w.rec_xyz for w in S])
        timed(lambda: B1.run(wavs))
        t_fwd1, (recs1, _) = timed(lambda: B1.run(wavs))
        same1 = all(torch.equal(a, b) for a, b in zip(recs1, recs_seq))
        del B1
        torch.cuda.empty_cache()
        os.environ["WAVE_BATCH_BRANCHES"] = "1"
        G1 = ShotBatch(ops, nt, [w.src_xyz for w in S], [w.rec_xyz for w in S], ckpt_every=K, gradient=True)
        timed(lambda: G1.run(wavs, dobs))
        tg1 = min(timed(lambda: G1.run(wavs, dobs))[0] for _ in range(2))
        del G1
        torch.cuda.empty_cache()
    finally:
        del os.environ["WAVE_BATCH_BRANCHES"]
    log("batch, other branch layout: forward (one branch) %.3f s, gradient (a branch per radius) %.3f s" % (t_fwd1, tg1))
    log("batch: batched forward %.3f s (first call %.3f s), gradient %.3f s (first call %.3f s)"
        % (t_fwd, t_first, tg, tg_first))
    # algorithmic bytes: forward 16 B per point-update (20/T with a time
    # tile); gradient: forward with checkpoints + recompute with history
    # (recompute_bpp) + adjoint with imaging, per shot with its own schedule
    def grad_bpp(sc):
        return wave_bytes_per_point(sc[0], 0) + recompute_bpp(sc) + wave_bytes_per_point(sc[0], 2)
    fb = sum(wave_bytes_per_point(op.schedule().T, 0) * w.npts for op, w in zip(ops, S)) * nt
    gb = sum(grad_bpp(op.schedule()) * w.npts for op, w in zip(ops, S)) * nt
    roof = {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "forward_achieved": round(fb / t_fwd / 1e9, 1), "forward_frac": round(fb / t_fwd / 1e9 / HBM_PEAK_GBS, 4),
            "gradient_achieved": round(gb / tg / 1e9, 1), "gradient_frac": round(gb / tg / 1e9 / HBM_PEAK_GBS, 4)}
    return {"roofline": roof,
            "workload": "shot_batch: %d shots, %d^3..%d^3 grids (%.1f Mpts in all), space orders 4/8, nt=%d, "
                        "gradient checkpoints every %d" % (len(S), round(min(w.npts for w in S) ** (1 / 3)),
                                                          round(max(w.npts for w in S) ** (1 / 3)), npts / 1e6, nt, K),
            "schedules": scheds, "unit": "Gpts/s",
            "other_branch_layout": {"forward_one_branch": round(npts * nt / t_fwd1 / 1e9, 2),
                                    "gradient_branch_per_radius": round(npts * nt / tg1 / 1e9, 2),
                                    "bitwise_equal_to_sequential": same1,
                                    "note": "the default is a graph branch per radius for the forward, one branch for "
                                            "the gradient; here the other layout (WAVE_BATCH_BRANCHES=0, then =1), "
                                            "timed after the default (later gradient calls of a process run faster)"},
            "forward": {"value": round(npts * nt / t_fwd / 1e9, 2), "s": round(t_fwd, 4),
                        "first_call_s": round(t_first, 4), "sequential_value": round(npts * nt / t_seq / 1e9, 2),
                        "speedup_vs_sequential": round(t_seq / t_fwd, 3), "bitwise_equal_to_sequential": same_fwd},
            "gradient": {"value": round(npts * nt / tg / 1e9, 2), "s": round(tg, 4), "first_call_s": round(tg_first, 4),
                         "sequential_value": round(npts * nt / tg_seq / 1e9, 2),
                         "speedup_vs_sequential": round(tg_seq / tg, 3), "grad_finite": finite}}


def sched_dict(sc) -> dict:
    """JSON form of a schedule (T, skew, extended tile, slab, axis-0 segments)."""
    return {"T": sc[0], "skew": sc[1], "tile": list(sc[4]), "slab": sc[5], "zchunks": sc[3]}


def launches_per_step(sc, n0, nt) -> int:
    """Sweep launches of one nt-step forward under schedule sc."""
    T, skew, slab = sc[0], sc[1], sc[5]
    if T < 1:
        return nt
    if slab == 0:
        return -(-nt // T)
    total, done = 0, 0
    while done < nt:
        Tw = min(T, nt - done)
        J = -(-(n0 + (Tw - 1) * skew) // slab)
        for j in range(J):
            for k in range(Tw):
                if max(0, j * slab - k * skew) < min(n0, (j + 1) * slab - k * skew):
                    total += 1
        done += Tw
    return total


def _rate(op, nt, w, wav, stream, reps=2, sched=None):
    """Gpts/s of an nt-step forward (minimum over reps after one warm-up);
    0 if the schedule is not available."""
    import torch
    from paper_1806_08299_amd import WaveError
    if sched is not None:
        try:
            op.set_schedule(*sched[:4], tile=sched[4], slab=sched[5])
        except WaveError:
            return 0.0
    op.forward(min(nt, 20), w.src_xyz, wav[:min(nt, 20)].contiguous(), w.rec_xyz)   # warm-up
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        op.forward(nt, w.src_xyz, wav, w.rec_xyz)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    return w.npts * nt / best / 1e9


def _frac(gpts, T):
    """Algorithmic GB/s and fraction of 8 TB/s at `gpts` point-updates/s for
    depth T (compulsory bytes per point-update of the forward)."""
    from paper_1806_08299_amd.wave import wave_bytes_per_point
    gbs = gpts * wave_bytes_per_point(T, 0)
    return round(gbs, 1), round(gbs / HBM_PEAK_GBS, 4)


def _row(kind, gpts, sc):
    gbs, fr = _frac(gpts, sc[0] if gpts else -1)
    return {"kind": kind, "value": round(gpts, 1), "GBs": gbs, "frac": fr, "schedule": sched_dict(sc)}


def c1_bench(dev, stream):
    """64^3, space order 4, 100 steps (point source, receiver line): untiled,
    register-tiled T = 1, 2, 4 (best tile) and skewed T = 2, 4, each with its
    algorithmic rate.  The working set (five 1 MiB levels) fits the L2 and
    the last-level cache, so the fractions of 8 TB/s are not HBM-limited."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import Schedule, tile_table, wave_tiled_max_depth
    w = wi.point_source_64()
    wav = torch.from_numpy(w.wavelet).to(dev)
    op = WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).to(dev), time_tile=-1)
    rows = []
    best_u = max((_rate(op, w.nt, w, wav, stream, 3, Schedule(-1, 0, 0, zc, (0, 0), 0)), zc) for zc in (0, 1, 2, 4))
    rows.append(_row("untiled", best_u[0], Schedule(-1, 4 // 2, 0, best_u[1], (0, 0), 0)))
    for T in (1, 2, 4):
        cands = [Schedule(T, 0, i + 1, zc, t, 0) for i, t in enumerate(tile_table(3))
                 if wave_tiled_max_depth(w.so, 3, tile=t) >= T for zc in (0, 1, 2)]
        if not cands:
            rows.append({"kind": "register-tiled", "T": T, "value": None,
                         "unsupported": "no register tile holds depth %d at space order %d" % (T, w.so)})
            continue
        r = max((_rate(op, w.nt, w, wav, stream, 3, c), c) for c in cands)
        rows.append(_row("register-tiled", r[0], r[1]))
    for T in (2, 4):
        r = max((_rate(op, w.nt, w, wav, stream, 3, Schedule(T, 0, 0, zc, (0, 0), Z)), Schedule(T, 2, 0, zc, (0, 0), Z))
                for Z in (8, 16, 32) for zc in (0, 1))
        rows.append(_row("skewed", r[0], r[1]))
    del op
    torch.cuda.empty_cache()
    return {"workload": "%s, model %s, nt=%d, 64 receivers" % (w.name, "x".join(map(str, w.shape)), w.nt),
            "unit": "Gpts/s", "note": "working set 5 MiB: served by the L2 and the last-level cache, "
                                      "so the fraction of 8 TB/s is not an HBM-bound figure", "rows": rows}


def depth_sweep(op, w, wav, stream, nt=40):
    """The headline workload at every time-tile depth T = 1..8: the best
    register-tiled schedule over the tiles that hold T (or why none does)
    and the best skewed schedule, on an nt-step slice, with algorithmic
    rates (20/T B per point-update, 16 at T = 1)."""
    from paper_1806_08299_amd.wave import Schedule, tile_table, wave_tiled_max_depth
    rows = []
    tab = tile_table(3)
    for T in range(1, 9):
        row = {"T": T}
        cands = [Schedule(T, 0, i + 1, zc, t, 0) for i, t in enumerate(tab)
                 if wave_tiled_max_depth(w.so, 3, tile=t) >= T for zc in (0, 16)]
        if cands:
            r = max((_rate(op, nt, w, wav, stream, 1, c), c) for c in cands)
            row["register_tiled"] = _row("register-tiled", r[0], r[1])
        else:
            row["register_tiled"] = {"value": None, "unsupported":
                                     "not built: every fused level keeps a %d-plane window per column in registers, "
                                     "and no tile of the table holds %d levels at space order %d"
                                     % (w.so + 1, T, w.so)}
        if T >= 2:
            r = max((_rate(op, nt, w, wav, stream, 1, Schedule(T, 0, 0, 2, (0, 0), Z)), Schedule(T, w.so // 2, 0, 2, (0, 0), Z))
                    for Z in (32, 48, 64))
            row["skewed"] = _row("skewed", r[0], r[1])
        rows.append(row)
        log("depth %d: register-tiled %s, skewed %s" % (T, row["register_tiled"].get("value"),
                                                        row.get("skewed", {}).get("value")))
    return rows


def skew_sweep(dev, stream, quick=False, nt=40):
    """The paper's skewing-factor experiment (Evaluation, Effect of the
    skewing factor): the minimum legal skew r against larger ones (r, 3r/2,
    2r) for the best register tiles and the skewed schedule of the layered
    workload at orders 4 and 8 (nt-step slices), and for the Laplace
    operator at order 8 (500^3, 32 steps: the grid of the paper's note on
    skews 4 and 8).  A skew that leaves a tile no core reads 'no core'."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import DiffOp, WaveError, WaveOp
    from paper_1806_08299_amd.wave import Schedule, tile_table
    tab = tile_table(3)
    n = 128 if quick else 512
    rows = []
    for so, cfgs in ((4, [(2, (32, 128), 0), (8, (0, 0), 64)]),
                     (8, [(1, (32, 128), 0), (2, (32, 64), 0), (8, (0, 0), 64)])):
        r = so // 2
        skews = sorted({r, (3 * r + 1) // 2, 2 * r})
        w = wi.layered_512(nt=nt, n=n, so=so)
        op = WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).to(dev), nbl=w.nbl,
                    sigma_max=w.sigma_max, time_tile=-1)
        wav = torch.from_numpy(w.wavelet).to(dev)
        for T, tile, slab in cfgs:
            shape = tab.index(tile) + 1 if slab == 0 else 0
            by = {}
            for sk in skews:
                v = _rate(op, nt, w, wav, stream, 2, Schedule(T, sk, shape, 2 if slab else 0, tile, slab))
                by[str(sk)] = round(v, 1) if v > 0 else "no core"
            kind = "skewed, %d-plane slabs" % slab if slab else "register-tiled %dx%d" % tile
            rows.append({"workload": w.name, "space_order": so, "T": T, "kind": kind, "unit": "Gpts/s",
                         "by_skew": by})
            log("skew sweep so%d T=%d %s: %s" % (so, T, kind, by))
        del op
        torch.cuda.empty_cache()
    w = wi.laplace(n=128 if quick else 500, so=8, nt=32)
    d = DiffOp(w.shape, w.spacing, w.dt, w.alpha, w.so)
    u0 = torch.from_numpy(w.u0).to(dev)
    for T, tile, slab, zc in ((8, (0, 0), 64, 2), (1, (32, 128), 0, 4)):
        by = {}
        for sk in (4, 6, 8):
            try:
                d.set_schedule(T, sk, tab.index(tile) + 1 if slab == 0 else 0, zc, slab=slab)
            except WaveError:
                by[str(sk)] = "no core"
                continue
            d.forward(w.nt, u0)
            best = 1e30
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                d.forward(w.nt, u0)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            by[str(sk)] = round(w.npts * w.nt / best / 1e9, 1)
        kind = "skewed, %d-plane slabs" % slab if slab else "register-tiled %dx%d" % tile
        rows.append({"workload": w.name, "space_order": 8, "T": T, "kind": kind, "unit": "Gpts/s", "by_skew": by})
        log("skew sweep laplace so8 T=%d %s: %s" % (T, kind, by))
    del d
    torch.cuda.empty_cache()
    return rows


def c3_bench(dev, stream, quick=False):
    """768^3 (+40 = 848^3), smooth random model, space orders 12 and 16, 500
    steps: the autotuned schedule, the untiled sweep and the best time-tiled
    schedule (register-tiled or skewed), each over the full run."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import Schedule, tile_table, wave_tiled_max_depth
    n, nt = (160, 60) if quick else (768, 500)
    t0 = time.time()
    base = wi.smooth_768(so=12, nt=nt, n=n, device=dev)
    log("smooth_768 model generated in %.1f s" % (time.time() - t0))
    m = torch.from_numpy(base.m).to(dev)
    out = []
    for so in (12, 16):
        w = wi.Workload("smooth_%dcube_so%d" % (n, so), base.shape, base.spacing, base.dt, so, nt, base.nbl,
                        base.sigma_max, base.m, base.src_xyz, base.wavelet, base.rec_xyz)
        wav = torch.from_numpy(w.wavelet).to(dev)
        op = WaveOp(w.shape, w.spacing, w.dt, so, m, nbl=w.nbl, sigma_max=w.sigma_max, time_tile=-1)
        op.autotune(16, 1, 8, w.src_xyz, w.rec_xyz)
        op._scratch = None
        tuned = op.schedule()
        v_t = _rate(op, nt, w, wav, stream, 1)
        untiled = max((_rate(op, nt, w, wav, stream, 1, Schedule(-1, 0, 0, zc, (0, 0), 0)), zc) for zc in (12,))
        # the time-tiled schedules that came closest on the 592^3 workload
        cands = [Schedule(1, 0, 3, 2, (32, 128), 0), Schedule(8, 0, 0, 2, (0, 0), 64), Schedule(4, 0, 0, 2, (0, 0), 64)]
        if tuned[0] >= 1:
            cands = [tuned]
        best = max((_rate(op, nt, w, wav, stream, 1, c), c) for c in cands)
        row = {"workload": w.name, "shape": list(w.shape), "space_order": so, "nt": nt, "unit": "Gpts/s",
               "autotuned": _row("autotuned", v_t, tuned),
               "untiled": _row("untiled", untiled[0], Schedule(-1, so // 2, 0, untiled[1], (0, 0), 0)),
               "best_time_tiled": _row("time-tiled", best[0], best[1]),
               "speedup_vs_untiled": round(max(v_t, best[0]) / untiled[0], 3)}
        out.append(row)
        log("smooth so%d: autotuned %s %.1f, untiled %.1f, best tiled %.1f %s" % (so, tuned, v_t, untiled[0],
                                                                              best[0], best[1]))
        del op
        torch.cuda.empty_cache()
    del m, base
    torch.cuda.empty_cache()
    return out


def wave2d_bench(dev, stream, quick=False):
    """2D 16384^2 (16384 x 16384 points, layered model, 40-point layer
    inside), space orders 2, 4, 8, 100 steps: the untiled sweep against the
    best register-tiled (1 x 1024 tiles, depth up to the built limit) and
    skewed schedules."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import Schedule, wave_tiled_max_depth
    n, nt = (2048, 50) if quick else (16384, 100)
    shape = (n - 80, n - 80)
    c = wi.layered_velocity(shape, 8, seed=7)
    out = []
    for so in (2, 4, 8):
        w = wi.make_workload("layered2d_%d_so%d" % (n, so), shape, 10.0, so, nt, 40, c, 10.0, (20, shape[1] // 2),
                             2, c_max=wi.C_MAX)
        wav = torch.from_numpy(w.wavelet).to(dev)
        op = WaveOp(w.shape, w.spacing, w.dt, so, torch.from_numpy(w.m).to(dev), nbl=w.nbl,
                    sigma_max=w.sigma_max, time_tile=-1)
        u = max((_rate(op, nt, w, wav, stream, 2, Schedule(-1, 0, 0, zc, (0, 0), 0)), zc) for zc in (0, 64, 256))
        reg = max((_rate(op, nt, w, wav, stream, 2, Schedule(T, 0, 0, zc, (1, 1024), 0)), Schedule(T, so // 2, 1, zc, (1, 1024), 0))
                  for T in range(1, wave_tiled_max_depth(so, 2) + 1) for zc in (0, 64, 256))
        skw = max((_rate(op, nt, w, wav, stream, 2, Schedule(T, 0, 0, zc, (0, 0), Z)), Schedule(T, so // 2, 0, zc, (0, 0), Z))
                  for T in (4, 8) for Z in (512, 1024) for zc in (0, 8))
        out.append({"workload": w.name, "shape": list(w.shape), "space_order": so, "nt": nt, "unit": "Gpts/s",
                    "untiled": _row("untiled", u[0], Schedule(-1, so // 2, 0, u[1], (0, 0), 0)),
                    "register_tiled": _row("register-tiled", reg[0], reg[1]),
                    "skewed": _row("skewed", skw[0], skw[1]),
                    "speedup_vs_untiled": round(max(reg[0], skw[0]) / u[0], 3)})
        log("2D so%d: untiled %.1f, register-tiled %.1f %s, skewed %.1f %s" % (so, u[0], reg[0], reg[1], skw[0], skw[1]))
        del op
        torch.cuda.empty_cache()
    return out


def tiling_factor(so, dev, stream, nt=100, n=512):
    """Best untiled and best time-tiled schedule (register-tiled over every
    built tile and depth, or skewed) for the layered workload at space order
    `so` (short runs, minimum of 2), and their ratio."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import Schedule, tile_table, wave_tiled_max_depth
    w = wi.layered_512(nt=nt, n=n, so=so)
    op = WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).to(dev), nbl=w.nbl,
                sigma_max=w.sigma_max, time_tile=-1)
    wav = torch.from_numpy(w.wavelet).to(dev)
    untiled = max((_rate(op, nt, w, wav, stream, 2, Schedule(-1, 0, 0, zc, (0, 0), 0)), zc) for zc in (12, 16, 24))
    cands = [Schedule(T, 0, i + 1, zc, t, 0) for i, t in enumerate(tile_table(3))
             for T in range(1, wave_tiled_max_depth(so, 3, tile=t) + 1) for zc in (0, 16, 32)]
    cands += [Schedule(T, 0, 0, 2, (0, 0), Z) for T in (4, 8) for Z in (48, 64)]
    tiled = max((_rate(op, nt, w, wav, stream, 2, c), c) for c in cands)
    guided = guided_vs_exhaustive(op, w, wav, stream, trial_steps=20)
    del op
    torch.cuda.empty_cache()
    return {"space_order": so, "untiled": round(untiled[0], 1), "untiled_zchunks": untiled[1],
            "tiled": round(tiled[0], 1), "tiled_schedule": sched_dict(tiled[1]),
            "factor": round(tiled[0] / untiled[0], 3), "autotuners": guided}


def laplace_bench(dev, stream, grids=((500, 32), (600, 16)), orders=(2, 4, 8, 16)):
    """The Laplace-operator workload (explicit diffusion) on the paper's grids
    (500^3 x 32 steps, 600^3 x 16 steps) at space orders 2..16: the default
    schedule, the best untiled and the best time-tiled schedule (minimum of
    three runs each), and the algorithmic HBM rate of each (8/T B per
    point-update)."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import DiffOp, WaveError
    from paper_1806_08299_amd.wave import wave_bytes_per_point, wave_tiled_max_depth
    out = []
    for n, nt in grids:
        base = wi.laplace(n=n, so=orders[0], nt=nt)   # the field is the same at every order
        u0 = torch.from_numpy(base.u0).to(dev)
        for so in orders:
            w = wi.DiffWorkload("laplace_%dcube_so%d" % (n, so), base.shape, base.spacing, base.dt, base.alpha,
                                so, nt, base.u0)
            op = DiffOp(w.shape, w.spacing, w.dt, w.alpha, w.so, time_tile=0)
            dflt = op.schedule()
            res = torch.empty_like(u0)

            def rate(sched):
                try:
                    op.set_schedule(*sched[:4], tile=sched[4] if len(sched) > 4 else None,
                                    slab=sched[5] if len(sched) > 5 else 0)
                except WaveError:
                    return 0.0
                op.forward(nt, u0, res)
                ts = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    torch.cuda.synchronize()
                    e0.record(stream)
                    op.forward(nt, u0, res)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e-3)
                return w.npts * nt / min(ts) / 1e9

            d_rate = rate(tuple(dflt))
            untiled = max((rate((-1, 0, 0, zc)), zc) for zc in (0, 8, 24))
            cands = [(T, shape, zc, 0) for shape in (2, 1, 3, 4)
                     for T in range(1, min(4, wave_tiled_max_depth(so, 3, shape)) + 1) for zc in (0, 4, 8, 16)]
            cands += [(T, 0, 2, Z) for T in (4, 8) for Z in (32, 64)]
            tiled = max((rate((T, 0, shape, zc, None, Z)), (T, shape, zc, Z)) for T, shape, zc, Z in cands)
            Tb = tiled[1][0]

            def gbs(v, T):
                return v * 1e9 * wave_bytes_per_point(T, 3) / 1e9
            out.append({"workload": w.name, "nt": nt, "space_order": so,
                        "default_schedule": sched_dict(dflt),
                        "default": round(d_rate, 1),
                        "untiled": round(untiled[0], 1), "untiled_zchunks": untiled[1],
                        "untiled_GBs": round(gbs(untiled[0], -1), 1),
                        "untiled_frac": round(gbs(untiled[0], -1) / HBM_PEAK_GBS, 4),
                        "tiled": round(tiled[0], 1),
                        "tiled_schedule": dict(zip(("T", "tile_shape", "zchunks", "slab"), tiled[1])),
                        "tiled_GBs": round(gbs(tiled[0], Tb), 1),
                        "tiled_frac": round(gbs(tiled[0], Tb) / HBM_PEAK_GBS, 4),
                        "factor": round(tiled[0] / untiled[0], 3)})
            log("laplace %s: default %s %.1f, untiled %.1f, tiled %.1f %s -> %.3fx"
                % (w.name, dflt, d_rate, untiled[0], tiled[0], tiled[1], out[-1]["factor"]))
            del op, res
            torch.cuda.empty_cache()
        del u0, base
        torch.cuda.empty_cache()
    return out


def ab2_bench(dev, stream, n=500, nt=32, orders=(2, 4, 8), quick=False):
    """The two-level (delta_t = 2) Laplace-operator stencil, the two-step
    Adams-Bashforth rule, on the 500^3 x 32-step grid of the Laplace section:
    the untiled sweep (12 B per point-update: two levels read, one written)
    against the best skewed schedule (16/T B), beside the one-level step's
    untiled and skewed rates on the same grid: the paper's hypothesis that
    time-tiling gains more with a larger time dependence."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import DiffOp, WaveError
    from paper_1806_08299_amd.wave import wave_bytes_per_point
    if quick:
        n = 128
    base = wi.laplace(n=n, so=orders[0], nt=nt)
    u0 = torch.from_numpy(base.u0).to(dev)
    res = torch.empty_like(u0)
    out = []
    for so in orders:
        rows = {}
        for scheme, mode, dt in (("ab2", 4, base.dt / 2.0), ("euler", 3, base.dt / 2.0)):
            op = DiffOp(base.shape, base.spacing, dt, base.alpha, so, time_tile=-1, scheme=scheme)

            def rate(T, Z, zc):
                try:
                    op.set_schedule(T, 0, 0, zc, slab=Z)
                except WaveError:
                    return 0.0
                op.forward(nt, u0, res)
                ts = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    torch.cuda.synchronize()
                    e0.record(stream)
                    op.forward(nt, u0, res)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e-3)
                return base.npts * nt / min(ts) / 1e9

            u = max((rate(-1, 0, zc), zc) for zc in (0, 8, 24))
            sk = max((rate(T, Z, zc), (T, Z, zc)) for T in (4, 8, 16) for Z in (32, 48, 64) for zc in (2,))
            bu, bs = wave_bytes_per_point(-1, mode), wave_bytes_per_point(sk[1][0], mode)
            rows[scheme] = {"untiled": round(u[0], 1), "untiled_GBs": round(u[0] * bu, 1),
                            "untiled_frac": round(u[0] * bu / HBM_PEAK_GBS, 4),
                            "skewed": round(sk[0], 1), "skewed_schedule": dict(zip(("T", "slab", "zchunks"), sk[1])),
                            "skewed_GBs": round(sk[0] * bs, 1), "skewed_frac": round(sk[0] * bs / HBM_PEAK_GBS, 4),
                            "factor": round(sk[0] / u[0], 3)}
            del op
            torch.cuda.empty_cache()
        out.append({"workload": "laplace_%dcube_so%d, %d steps, dt at 0.9 of the two-level limit" % (n, so, nt),
                    "space_order": so, "unit": "Gpts/s", "two_level": rows["ab2"], "one_level_same_dt": rows["euler"]})
        log("ab2 so%d: untiled %.1f, skewed %.1f (%.3fx); one-level %.1f / %.1f (%.3fx)"
            % (so, rows["ab2"]["untiled"], rows["ab2"]["skewed"], rows["ab2"]["factor"],
               rows["euler"]["untiled"], rows["euler"]["skewed"], rows["euler"]["factor"]))
    del u0, res, base
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="physical grid edge of the forward workload")
    ap.add_argument("--nt", type=int, default=1000)
    ap.add_argument("--so", type=int, default=8, help="space order of the forward workload")
    ap.add_argument("--T", type=int, default=0, help="time-tile depth (0: autotune, -1: untiled)")
    ap.add_argument("--shape", type=int, default=1, help="register-tiled: index of the extended tile")
    ap.add_argument("--slab", type=int, default=0, help="skewed schedule: slab thickness (0: not skewed)")
    ap.add_argument("--zchunks", type=int, default=0)
    ap.add_argument("--no-untiled", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-orders", action="store_true")
    ap.add_argument("--no-laplace", action="store_true", help="skip the Laplace-operator (diffusion) section")
    ap.add_argument("--no-c1", action="store_true", help="skip the 64^3 point-source section")
    ap.add_argument("--no-depths", action="store_true", help="skip the depth sweep of the headline workload")
    ap.add_argument("--no-skew", action="store_true", help="skip the skewing-factor sweep")
    ap.add_argument("--no-smooth", action="store_true", help="skip the 768^3 smooth-model section")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D section")
    ap.add_argument("--no-ab2", action="store_true", help="skip the two-level (Adams-Bashforth) section")
    ap.add_argument("--laplace-only", action="store_true",
                    help="diagnostic: run only the Laplace-operator section and print its results")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run plain device copies of known size (reference for the traffic counters)")
    ap.add_argument("--quick", action="store_true", help="small sizes for a functional check")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sweep has no multi-GPU path in this library "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import wave_ai_naive, wave_ai_tight, wave_bytes_per_point, wave_flops_per_point

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    if args.quick:
        args.n, args.nt = 128, 100
    if args.laplace_only:
        lap = laplace_bench(dev, stream, grids=((128, 32),) if args.quick else ((500, 32), (600, 16)))
        print(json.dumps({"laplace": lap}), flush=True)
        return

    # ---------------------------------------------------------------- forward, tuned schedule
    t0 = time.time()
    w = wi.layered_512(nt=args.nt, n=args.n, so=args.so)
    log("workload %s shape %s nt %d (%.1f s to generate)" % (w.name, w.shape, w.nt, time.time() - t0))
    m = torch.from_numpy(w.m).to(dev)
    wav = torch.from_numpy(w.wavelet).to(dev)
    op = WaveOp(w.shape, w.spacing, w.dt, w.so, m, nbl=w.nbl, sigma_max=w.sigma_max, time_tile=-1)
    if args.copy_calibration:
        # zero steps with an initial and a final state: four plain copies of
        # N floats (one time level each) through the library's copy kernel,
        # one float per lane like the sweep's own accesses
        x = torch.zeros((2,) + tuple(w.shape), dtype=torch.float32, device=dev)
        for _ in range(3):
            op.forward(0, u_init=x, want_final=True)
        torch.cuda.synchronize()
        del x
        log("copy calibration: 12 copies of %d bytes" % (w.npts * 4))
    if args.T != 0:
        op.set_schedule(args.T, 0, args.shape if args.slab == 0 else 0, args.zchunks, slab=args.slab)
    else:
        best = autotune(op, w)
        log("autotune -> schedule %s, %.3f ms/step" % (op.schedule(), best * 1e3))
    sched = op.schedule()
    T = sched[0]
    for _ in range(args.warmup):
        op.forward(w.nt, w.src_xyz, wav, w.rec_xyz)
    elapsed, wall = run_steps(op, w, wav, args.steps, stream)
    t_step = elapsed / args.steps
    value = w.npts * w.nt / t_step / 1e9
    log("schedule %s: %.4f s/step (wall %.4f) -> %.1f Gpts/s" % (sched, t_step, wall / args.steps, value))

    # ---------------------------------------------------------------- untiled reference sweep
    untiled = None
    if not args.no_untiled:
        zu = tune_untiled(op)
        op.forward(w.nt, w.src_xyz, wav, w.rec_xyz)
        ue, _ = run_steps(op, w, wav, max(1, args.steps), stream)
        ut = ue / max(1, args.steps)
        untiled = {"value": round(w.npts * w.nt / ut / 1e9, 2), "ms_per_step": round(ut * 1e3, 3), "zchunks": zu}
        log("untiled (zchunks %d): %.4f s/step -> %.1f Gpts/s" % (zu, ut, untiled["value"]))
        op.set_schedule(*sched)

    # ---------------------------------------------------------------- plain copy rate on this GPU
    # zero steps with an initial and a final state: four copies of one time
    # level through the library's copy kernel (read N floats, write N floats)
    x = torch.zeros((2,) + tuple(w.shape), dtype=torch.float32, device=dev)
    op.forward(0, u_init=x, want_final=True)
    ec = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        op.forward(0, u_init=x, want_final=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ec.append(e0.elapsed_time(e1) * 1e-3)
    copy_gbs = 4 * 2 * w.npts * 4 / min(ec) / 1e9
    del x
    # the sweep's own mix, three streams read and one written (16 B per
    # point), as a plain elementwise kernel: torch's addcmul over N floats
    s3 = [torch.empty(w.npts, dtype=torch.float32, device=dev) for _ in range(4)]
    torch.addcmul(s3[0], s3[1], s3[2], out=s3[3])
    es = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        torch.addcmul(s3[0], s3[1], s3[2], out=s3[3])
        e1.record(stream)
        torch.cuda.synchronize()
        es.append(e0.elapsed_time(e1) * 1e-3)
    stream_gbs = 16 * w.npts / min(es) / 1e9
    del s3

    # ---------------------------------------------------------------- roofline of the dominant kernel
    # One step = the sweep launches of the schedule (ceil(nt / T) register-
    # tiled or untiled launches over the grid, or one launch per slab and
    # step of the skewed schedule) plus four small kernels (forcing table,
    # two fills, receiver reduction; < 0.1 % of the step).  Algorithmic bytes
    # of the step: bytes per point-update of the schedule x points x nt; per
    # launch: that over the launches (every launch of a skewed step moves one
    # slab's share).
    Tn = max(T, 1)
    launches = launches_per_step(sched, w.shape[0], w.nt)
    t_launch = t_step / launches
    bpp = wave_bytes_per_point(T, 0)
    alg_bytes = bpp * w.npts * w.nt / launches      # per launch, on average
    achieved = alg_bytes / t_launch / 1e9
    flops_pt = wave_flops_per_point(3, w.so, 0)
    rec = traffic_record(w.name, sched)
    traffic = None
    if rec is not None:
        f = float(rec["fetch_kib"]) * float(rec["copy_bytes"]) / float(rec["copy_fetch_kib"])
        wr = float(rec["write_kib"]) * float(rec["copy_bytes"]) / float(rec["copy_write_kib"])
        traffic = round(f + wr)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": kernel_name(sched, w.so), "algorithmic_bytes_per_launch": alg_bytes,
                "bytes_per_point_update": bpp, "point_updates_per_launch": round(w.npts * w.nt / launches),
                "avg_launch_ms": round(t_launch * 1e3, 4), "launches_per_step": launches,
                "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                "stream_3r1w_GBs": round(stream_gbs, 1), "frac_of_stream_3r1w": round(achieved / stream_gbs, 4)}

    # ---------------------------------------------------------------- arithmetic intensity
    # AI of the untiled sweep: useful flops per compulsory byte; the estimators
    # take it times T (naive) and shrink it by re-loaded tile faces (tight),
    # with the cache read as one XCD's L2 or as the shared last-level cache.
    ai_s = flops_pt / 16.0
    ai = {"flops_per_point_update": flops_pt, "untiled_ai": round(ai_s, 4),
          "naive": round(wave_ai_naive(ai_s, Tn), 4)}
    # tile sizes: the extended tile of the register-tiled sweep, the 16 x 64
    # block of the single-step kernel (untiled or skewed; the skewed slab is
    # the tile along axis 0)
    ey, ex = tuple(sched[4]) if (T >= 1 and sched[5] == 0) else (16, 64)
    t0_ = sched[5] if sched[5] > 0 else w.shape[0]
    for nm, om in (("tight_l2", L2_FLOATS), ("tight_mall", MALL_FLOATS)):
        ai[nm] = round(wave_ai_tight(ai_s, Tn, w.shape, [w.so // 2] * 3, [t0_, ey, ex], om), 4)
    if traffic:
        ai["measured"] = round(flops_pt * w.npts * w.nt / launches / traffic, 4)
    ai["compulsory"] = round(flops_pt / bpp, 4)
    depths = None
    if not args.no_depths:
        depths = depth_sweep(op, w, wav, stream, nt=20 if args.quick else 40)
    del op, m, wav
    torch.cuda.empty_cache()

    skews = None if args.no_skew else skew_sweep(dev, stream, quick=args.quick)
    c1 = None if args.no_c1 else c1_bench(dev, stream)
    c3 = None if args.no_smooth else c3_bench(dev, stream, quick=args.quick)
    w2d = None if args.no_2d else wave2d_bench(dev, stream, quick=args.quick)
    adj = None if args.no_adjoint else gradient_bench(args, dev, stream)
    batch = None if args.no_batch else batch_bench(args, dev, stream)
    orders = None
    if not args.no_orders:
        orders = []
        for so in (2, 4, 8):
            orders.append(tiling_factor(so, dev, stream, n=128 if args.quick else 512))
            log("order %d: untiled %.1f, tiled %.1f %s -> %.3fx" % (so, orders[-1]["untiled"], orders[-1]["tiled"],
                                                                  orders[-1]["tiled_schedule"], orders[-1]["factor"]))
    lap = None
    if not args.no_laplace:
        lap = laplace_bench(dev, stream, grids=((128, 32),) if args.quick else ((500, 32), (600, 16)))
    ab2 = None if args.no_ab2 else ab2_bench(dev, stream, quick=args.quick)
    cpu = None if args.no_cpu else cpu_baseline(w, n=args.n, quick=args.quick)

    line = {
        "metric": "Gpts/s fwd & adjoint-grad vs untiled sweep; % HBM roofline (1 MI355X)",
        "value": round(value, 2), "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "shape": list(w.shape), "physical": [args.n] * 3, "nbl": w.nbl,
                   "space_order": w.so, "nt": w.nt,
                   "schedule": sched_dict(sched)},
        "untiled": untiled,
        "speedup_vs_untiled": round(value / untiled["value"], 3) if untiled else None,
        "adjoint_grad": adj,
        "batch": batch,
        "tiling_by_order": orders,
        "depth_sweep": depths,
        "skew_sweep": skews,
        "point_source_64": c1,
        "smooth_768": c3,
        "wave2d": w2d,
        "laplace": lap,
        "two_level_laplace": ab2,
        "roofline": roofline,
        "ai": ai,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

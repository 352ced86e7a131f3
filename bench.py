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
* cpu_baseline: the FP64 oracle on the host cores on a bounded sample.

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
    T, _, shape, zc = sched
    for line in open(path):
        if not line.startswith("record "):
            continue
        kv = dict(f.split("=", 1) for f in line.split()[1:])
        if (kv.get("workload") == workload and int(kv["T"]) == T and int(kv["shape"]) == shape
                and int(kv["zchunks"]) == zc and kv.get("sources") == sha):
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


def autotune(op, trial_steps=40):
    from paper_1806_08299_amd.wave import wave_autotune, wave_scratch_bytes
    sc = op.scratch(wave_scratch_bytes(op.ctx, trial_steps, 0, 0, 0, 0))
    return wave_autotune(op.ctx, trial_steps, 2, 8, sc)


def kernel_name(sched, so) -> str:
    T, _, shape, _ = sched
    if T < 0:
        return "k_untiled R=%d (single-step sweep)" % (so // 2)
    return "k_tiled R=%d T=%d tile_shape=%d" % (so // 2, T, shape)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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


def cpu_baseline(w, budget_s=20.0, n=512):
    """FP64 oracle on the host: the same grid, model, order and source for a
    few time steps (bounded to ~budget_s of CPU work), as Gpts/s, on all the
    threads OpenMP is given; plus one step on one thread (a child process
    with OMP_NUM_THREADS=1)."""
    import subprocess
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
    out = {"value": round(w.npts * steps / dt / 1e9, 4), "unit": "Gpts/s", "cores": threads, "kind": "oracle",
           "sample": "%s: first %d of %d time steps on the full %s grid (FP64, OpenMP over axis 0), "
                     "%.1f s" % (w.name, steps, w.nt, "x".join(map(str, w.shape)), dt),
           "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count()}
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
    autotune(op)
    tuned = op.schedule()
    out = {"workload": "%s, model %s, nt=%d, checkpoints every %d"
                       % (init.name, "x".join(map(str, init.shape)), init.nt, K), "unit": "Gpts/s"}

    def one(sched):
        op.set_schedule(*sched)
        best = None
        for _ in range(2):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            torch.cuda.synchronize()
            e0.record(stream)
            rec, _ = op.forward(init.nt, init.src_xyz, wv, init.rec_xyz, ckpt_every=K, adjoint_scratch=True)
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
    out.update({"schedule": dict(zip(("T", "skew", "tile_shape", "zchunks"), tuned)),
                "value": round(init.npts * init.nt / (tf + ta) / 1e9, 2),
                "forward_with_checkpoints_s": round(tf, 4), "recompute_plus_adjoint_s": round(ta, 4),
                "grad_finite": bool(torch.isfinite(gm).all().item())})
    # adjoint launch: recompute (history) + adjoint per segment; the adjoint
    # kernel's algorithmic bytes per point-update
    T = tuned[0]
    out["adjoint_bytes_per_point_update"] = wave_bytes_per_point(T, 2)
    out["history_bytes_per_point_update"] = wave_bytes_per_point(T, 1)
    log("gradient %s: fwd %.3f s + recompute/adjoint %.3f s" % (tuned, tf, ta))
    if not args.no_untiled:
        (uf, ua), _ = one((-1, 0, 0, tuned[3] if tuned[0] < 0 else 0))
        out["untiled"] = {"value": round(init.npts * init.nt / (uf + ua) / 1e9, 2),
                          "forward_with_checkpoints_s": round(uf, 4), "recompute_plus_adjoint_s": round(ua, 4)}
        out["speedup_vs_untiled"] = round((uf + ua) / (tf + ta), 3)
        log("gradient untiled: fwd %.3f s + recompute/adjoint %.3f s" % (uf, ua))
    del op
    torch.cuda.empty_cache()
    return out


def batch_bench(args, dev, stream):
    """32 independent shots (128^3..320^3, space orders 4/8, 800 steps):
    forward and gradient through one captured, merged sequence (wave_batch),
    against the same shots run one after another."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import ShotBatch, WaveOp
    from paper_1806_08299_amd.wave import wave_autotune, wave_scratch_bytes
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
        sc = op.scratch(wave_scratch_bytes(op.ctx, 20, 0, 0, 0, 0))
        wave_autotune(op.ctx, 20, 1, 2, sc)          # batched kernels: untiled or T <= 2
        op._scratch = None
        ops.append(op)
        wavs.append(torch.from_numpy(w.wavelet).to(dev))
    npts = sum(w.npts for w in S)
    scheds = {}
    for op in ops:
        key = "T=%d shape=%d" % (op.schedule()[0], op.schedule()[2])
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
    tg_seq, _ = timed(seq_grad)
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
    finite = all(bool(torch.isfinite(g).all().item()) for g in grads)
    del G
    torch.cuda.empty_cache()
    log("batch: batched forward %.3f s (first call %.3f s), gradient %.3f s (first call %.3f s)"
        % (t_fwd, t_first, tg, tg_first))
    return {"workload": "shot_batch: %d shots, %d^3..%d^3 grids (%.1f Mpts in all), space orders 4/8, nt=%d, "
                        "gradient checkpoints every %d" % (len(S), round(min(w.npts for w in S) ** (1 / 3)),
                                                          round(max(w.npts for w in S) ** (1 / 3)), npts / 1e6, nt, K),
            "schedules": scheds, "unit": "Gpts/s",
            "forward": {"value": round(npts * nt / t_fwd / 1e9, 2), "s": round(t_fwd, 4),
                        "first_call_s": round(t_first, 4), "sequential_value": round(npts * nt / t_seq / 1e9, 2),
                        "speedup_vs_sequential": round(t_seq / t_fwd, 3), "bitwise_equal_to_sequential": same_fwd},
            "gradient": {"value": round(npts * nt / tg / 1e9, 2), "s": round(tg, 4), "first_call_s": round(tg_first, 4),
                         "sequential_value": round(npts * nt / tg_seq / 1e9, 2),
                         "speedup_vs_sequential": round(tg_seq / tg, 3), "grad_finite": finite}}


def tiling_factor(so, dev, stream, nt=100, n=512):
    """Best untiled and best time-tiled schedule for the layered workload at
    space order `so` (short runs, minimum of 2), and their ratio."""
    import torch
    import waveinputs as wi
    from paper_1806_08299_amd import WaveOp, WaveError
    from paper_1806_08299_amd.wave import wave_tiled_max_depth
    w = wi.layered_512(nt=nt, n=n, so=so)
    op = WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).to(dev), nbl=w.nbl,
                sigma_max=w.sigma_max, time_tile=-1)
    wav = torch.from_numpy(w.wavelet).to(dev)

    def rate(sched):
        try:
            op.set_schedule(*sched)
        except WaveError:
            return 0.0
        op.forward(nt, w.src_xyz, wav, w.rec_xyz)
        t, _ = run_steps(op, w, wav, 1, stream)
        t = min(t, run_steps(op, w, wav, 1, stream)[0])
        return w.npts * nt / t / 1e9

    untiled = max((rate((-1, 0, 1, zc)), zc) for zc in (12, 16, 24))
    tiled = max((rate((T, 0, shape, zc)), (T, shape, zc)) for shape in (1, 2)
                for T in range(1, wave_tiled_max_depth(so, 3, shape) + 1) for zc in (0, 16, 32))
    del op
    torch.cuda.empty_cache()
    return {"space_order": so, "untiled": round(untiled[0], 1), "untiled_zchunks": untiled[1],
            "tiled": round(tiled[0], 1), "tiled_schedule": dict(zip(("T", "tile_shape", "zchunks"), tiled[1])),
            "factor": round(tiled[0] / untiled[0], 3)}


def laplace_bench(dev, stream, grids=((500, 32), (600, 16)), orders=(2, 4, 8, 16)):
    """The Laplace-operator workload (explicit diffusion) on the paper's grids
    (500^3 x 32 steps, 600^3 x 16 steps) at space orders 2..16: the default
    schedule, the best untiled and the best time-tiled schedule (minimum of
    five runs each), and the algorithmic HBM rate of each (8/T B per
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
                    op.set_schedule(*sched)
                except WaveError:
                    return 0.0
                op.forward(nt, u0, res)
                ts = []
                for _ in range(5):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    torch.cuda.synchronize()
                    e0.record(stream)
                    op.forward(nt, u0, res)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e-3)
                return w.npts * nt / min(ts) / 1e9

            d_rate = rate((dflt[0], dflt[1], dflt[2], dflt[3]))
            untiled = max((rate((-1, 0, 0, zc)), zc) for zc in (0, 8, 24))
            cands = [(T, shape, zc) for shape in (2, 1) for T in range(1, min(4, wave_tiled_max_depth(so, 3, shape)) + 1)
                     for zc in (0, 4, 8, 16)]
            tiled = max((rate((T, 0, shape, zc)), (T, shape, zc)) for T, shape, zc in cands)
            Tb = tiled[1][0]

            def gbs(v, T):
                return v * 1e9 * wave_bytes_per_point(T, 3) / 1e9
            out.append({"workload": w.name, "nt": nt, "space_order": so,
                        "default_schedule": dict(zip(("T", "skew", "tile_shape", "zchunks"), dflt)),
                        "default": round(d_rate, 1),
                        "untiled": round(untiled[0], 1), "untiled_zchunks": untiled[1],
                        "untiled_GBs": round(gbs(untiled[0], -1), 1),
                        "untiled_frac": round(gbs(untiled[0], -1) / HBM_PEAK_GBS, 4),
                        "tiled": round(tiled[0], 1),
                        "tiled_schedule": dict(zip(("T", "tile_shape", "zchunks"), tiled[1])),
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512, help="physical grid edge of the forward workload")
    ap.add_argument("--nt", type=int, default=1000)
    ap.add_argument("--so", type=int, default=8, help="space order of the forward workload")
    ap.add_argument("--T", type=int, default=0, help="time-tile depth (0: autotune, -1: untiled)")
    ap.add_argument("--shape", type=int, default=1)
    ap.add_argument("--zchunks", type=int, default=0)
    ap.add_argument("--no-untiled", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-orders", action="store_true")
    ap.add_argument("--no-laplace", action="store_true", help="skip the Laplace-operator (diffusion) section")
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
        op.set_schedule(args.T, 0, args.shape, args.zchunks)
    else:
        best = autotune(op)
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
    # One step = ceil(nt / T) launches of the sweep kernel plus four small
    # kernels (forcing table, two fills, receiver reduction; < 0.1 % of the
    # step), so the kernel's average launch time is bounded by step / launches.
    Tn = max(T, 1)
    launches = -(-w.nt // Tn)
    t_launch = t_step / launches
    bpp = wave_bytes_per_point(T, 0)
    alg_bytes = bpp * w.npts * Tn                   # per launch (full window)
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
                "bytes_per_point_update": bpp, "points_per_launch": w.npts * Tn,
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
    from paper_1806_08299_amd.wave import block_extent
    # tile sizes: the extended tile of the tiled sweep, the 16 x 64 block of the untiled one
    ey, ex = block_extent(3, sched[2]) if T >= 1 else (16, 64)
    for nm, om in (("tight_l2", L2_FLOATS), ("tight_mall", MALL_FLOATS)):
        ai[nm] = round(wave_ai_tight(ai_s, Tn, w.shape, [w.so // 2] * 3, [w.shape[0], ey, ex], om), 4)
    if traffic:
        ai["measured"] = round(flops_pt * w.npts * Tn / traffic, 4)
    ai["compulsory"] = round(flops_pt / bpp, 4)
    del op, m, wav
    torch.cuda.empty_cache()

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
    cpu = None if args.no_cpu else cpu_baseline(w, n=args.n)

    line = {
        "metric": "Gpts/s fwd & adjoint-grad vs untiled sweep; % HBM roofline (1 MI355X)",
        "value": round(value, 2), "unit": "Gpts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "shape": list(w.shape), "physical": [args.n] * 3, "nbl": w.nbl,
                   "space_order": w.so, "nt": w.nt,
                   "schedule": dict(zip(("T", "skew", "tile_shape", "zchunks"), sched))},
        "untiled": untiled,
        "speedup_vs_untiled": round(value / untiled["value"], 3) if untiled else None,
        "adjoint_grad": adj,
        "batch": batch,
        "tiling_by_order": orders,
        "laplace": lap,
        "roofline": roofline,
        "ai": ai,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

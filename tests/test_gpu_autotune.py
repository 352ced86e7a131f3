"""GPU tests of the autotuners (implementation chapter, "Auto-tuning";
evaluation chapter, "Minimising runtime based on tile size choices").

* the exhaustive tuner and the estimator-guided one both keep a schedule
  whose result is bitwise that of the untiled sweep;
* the guided tuner times fewer candidates than phase 1 of the exhaustive one
  holds, and the schedule it keeps is close to the exhaustive winner's speed;
* keep < 1 is refused;
* wave_autotune_points (trials with the operator's sources and receivers):
  bitwise results, its scratch sizing and its refusals.
"""
import numpy as np
import pytest
import torch

from test_gpu_forward import _op, _run, _small

pytestmark = pytest.mark.gpu


def _seconds(op, w, reps=3):
    wav = torch.from_numpy(w.wavelet).cuda()
    op.forward(w.nt, w.src_xyz, wav, w.rec_xyz)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        op.forward(w.nt, w.src_xyz, wav, w.rec_xyz)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


@pytest.mark.parametrize("so", [2, 8])
def test_guided_autotune_against_exhaustive(so):
    from paper_1806_08299_amd import WaveError
    from paper_1806_08299_amd.wave import tile_table, wave_autotune, wave_autotune_guided, wave_scratch_bytes, \
        wave_tiled_max_depth
    w = _small(so, (160, 176, 192), nbl=6, seed=400 + so, nt=32)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    sc = op.scratch(wave_scratch_bytes(op.ctx, 16, 0, 0, 0, 0))
    wave_autotune(op.ctx, 16, 2, 8, sc)
    ex = op.schedule()
    t_ex = _seconds(op, w)
    rec_e, fin_e = _run(op, w)
    assert np.array_equal(fin_e, fin_u) and np.array_equal(rec_e, rec_u)
    sc = op.scratch(wave_scratch_bytes(op.ctx, 16, 0, 0, 0, 0))
    _, timed = wave_autotune_guided(op.ctx, 16, 2, 8, 10, sc)
    gd = op.schedule()
    t_gd = _seconds(op, w)
    rec_g, fin_g = _run(op, w)
    assert np.array_equal(fin_g, fin_u) and np.array_equal(rec_g, rec_u)
    phase1 = 1 + sum(wave_tiled_max_depth(so, 3, tile=t) for t in tile_table(3)) + 8
    print("so %d: exhaustive %s %.3f ms, guided %s %.3f ms, %d timed (phase 1 holds %d)"
          % (so, ex, t_ex, gd, t_gd, timed, phase1), flush=True)
    assert timed < phase1 + 5 * 8          # fewer than phase 1 + the zchunk sweep of five
    assert t_gd <= 1.25 * t_ex
    with pytest.raises(WaveError):
        wave_autotune_guided(op.ctx, 16, 2, 8, 0, sc)


@pytest.mark.parametrize("keep", [0, 10])
def test_autotune_with_points(keep):
    """wave_autotune_points: trials that carry the operator's sources and
    receivers keep a schedule whose result is bitwise the untiled sweep's;
    its scratch is the plain tuner's with no points and grows with them;
    too little scratch, non-finite coordinates and points on a diffusion
    context are refused."""
    from paper_1806_08299_amd import DiffOp, WaveError
    from paper_1806_08299_amd.wave import wave_autotune_points, wave_autotune_scratch_bytes, wave_scratch_bytes
    w = _small(4, (96, 112, 130), nbl=6, seed=420 + keep, nt=24)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    assert wave_autotune_scratch_bytes(op.ctx, 12) == wave_scratch_bytes(op.ctx, 12, 0, 0, 0, 0)
    nb = wave_autotune_scratch_bytes(op.ctx, 12, len(w.src_xyz), len(w.rec_xyz))
    assert nb > wave_autotune_scratch_bytes(op.ctx, 12)
    sc = op.scratch(nb)
    best, timed = wave_autotune_points(op.ctx, 12, 1, 4, keep, w.src_xyz, w.rec_xyz, sc)
    assert best > 0 and timed >= 4
    rec_t, fin_t = _run(op, w)
    assert np.array_equal(fin_t, fin_u) and np.array_equal(rec_t, rec_u), op.schedule()
    # the method on the operator
    op.set_schedule(-1)
    assert op.autotune(8, 1, 2, w.src_xyz, w.rec_xyz, keep=keep) > 0
    rec_t, fin_t = _run(op, w)
    assert np.array_equal(fin_t, fin_u) and np.array_equal(rec_t, rec_u), op.schedule()
    small = sc[:nb - 1]
    with pytest.raises(WaveError) as e:
        wave_autotune_points(op.ctx, 12, 1, 4, keep, w.src_xyz, w.rec_xyz, small)
    assert e.value.status == -4
    bad = np.array(w.rec_xyz, dtype=np.float64)
    bad[0, 1] = np.nan
    with pytest.raises(WaveError) as e:
        wave_autotune_points(op.ctx, 12, 1, 4, keep, w.src_xyz, bad, sc)
    assert e.value.status == -1
    d = DiffOp((40, 30, 70), (1.0, 1.0, 1.0), 0.01, 1.0, 4)
    dsc = torch.empty(wave_autotune_scratch_bytes(d.ctx, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(WaveError) as e:
        wave_autotune_points(d.ctx, 4, 1, 2, keep, [[1.0, 1.0, 1.0]], None, dsc)
    assert e.value.status == -1


@pytest.mark.parametrize("shape", [(40, 60, 140), (60, 1100)])
def test_autotune_gradient(shape):
    """wave_autotune_gradient keeps a schedule whose gradient is bitwise that
    of the untiled sweep; its scratch covers the forward trials and a trial
    gradient; too little scratch and a diffusion context are refused."""
    from paper_1806_08299_amd import DiffOp, WaveError
    from paper_1806_08299_amd.wave import (wave_autotune_gradient, wave_autotune_gradient_scratch_bytes,
                                           wave_autotune_scratch_bytes)
    from test_gpu_adjoint import _grad, _op as _aop, _problem
    P = _problem(so=4, shape=shape, nbl=4, nt=16, seed=7, nsrc=2, nrec=9)
    P["resid"] = np.random.default_rng(8).standard_normal((P["nt"], P["rec"].shape[0])).astype(np.float32)
    op = _aop(P, P["m0"], time_tile=-1)
    gm_u, gq_u = _grad(op, P, 6)
    nb = wave_autotune_gradient_scratch_bytes(op.ctx, 12, len(P["src"]), len(P["rec"]), 6)
    assert nb >= wave_autotune_scratch_bytes(op.ctx, 12, len(P["src"]), len(P["rec"]))
    sc = op.scratch(nb)
    best, timed = wave_autotune_gradient(op.ctx, 12, 1, 4, 6, P["src"], P["rec"], sc, len(shape))
    print("shape %s: kept %s, %.3g s per step, %d timed" % (shape, op.schedule(), best, timed), flush=True)
    assert best > 0 and timed >= 3
    gm_t, gq_t = _grad(op, P, 6)
    assert np.array_equal(gm_t, gm_u) and np.array_equal(gq_t, gq_u), op.schedule()
    assert op.autotune_gradient(8, 1, 2, P["src"], P["rec"], ckpt_every=4) > 0
    gm_t, gq_t = _grad(op, P, 6)
    assert np.array_equal(gm_t, gm_u) and np.array_equal(gq_t, gq_u), op.schedule()
    with pytest.raises(WaveError) as e:
        wave_autotune_gradient(op.ctx, 12, 1, 4, 6, P["src"], P["rec"], sc[:nb - 1], len(shape))
    assert e.value.status == -4
    d = DiffOp((40, 30, 70), (1.0, 1.0, 1.0), 0.01, 1.0, 4)
    assert wave_autotune_gradient_scratch_bytes(d.ctx, 4, 0, 0, 2) == 0
    with pytest.raises(WaveError) as e:
        wave_autotune_gradient(d.ctx, 4, 1, 2, 2, None, None, torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert e.value.status == -6

"""The allocation-free forward (wave_forward_static) against wave_forward.

wave_forward_static runs the same drivers and kernels as wave_forward, with
its tables in the library's static per-GPU scratch array instead of a
caller-provided buffer.  Its receiver traces and final state must equal
those of wave_forward bitwise, on two calls in a row whose second has a
smaller grid, fewer steps and fewer points (the array keeps the first call's
contents, so anything read before being written would show); a call that
needs more than the static maximum is refused before any launch.
"""
import numpy as np
import pytest
import torch

import waveinputs as wi

pytestmark = pytest.mark.gpu


def _case(shape, nt, nsrc, nrec, so, seed):
    rng = np.random.default_rng(seed)
    h = 10.0
    c = wi.smooth_random_velocity(shape, seed=seed, sigma_cells=2.0, cmin=1500.0, cmax=2500.0)
    m = wi.to_slowness2(c)
    dt = 0.35 * h / 2500.0
    ext = np.array(shape, dtype=np.float64) * h
    src = rng.uniform(0.1, 0.9, size=(nsrc, 3)) * ext
    rec = rng.uniform(0.0, 1.0, size=(nrec, 3)) * ext
    wav = np.stack([wi.ricker(nt, dt, 15.0 + 2.0 * k) for k in range(nsrc)], axis=1).astype(np.float32)
    return m, dt, src, rec, wav


def _both(shape, nt, nsrc, nrec, so, seed, nbl=3, **sched):
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import wave_forward_static
    m, dt, src, rec, wav = _case(shape, nt, nsrc, nrec, so, seed)
    smax = wi.sigma_max_estimate(2500.0, nbl, 10.0)
    op = WaveOp(shape, 10.0, dt, so, torch.from_numpy(m).cuda(), nbl=nbl, sigma_max=smax, **sched)
    w = torch.from_numpy(wav).cuda()
    u0 = torch.from_numpy(np.random.default_rng(seed + 1).standard_normal((2,) + shape).astype(np.float32)).cuda()
    print("no-alloc case shape %s nt %d nsrc %d nrec %d so %d sched %s" % (shape, nt, nsrc, nrec, so, sched),
          flush=True)
    rec_a, fin_a = op.forward(nt, src, w, rec, u_init=u0, want_final=True)
    rec_b = torch.full((nt, nrec), float("nan"), dtype=torch.float32, device="cuda")
    fin_b = torch.full((2,) + shape, float("nan"), dtype=torch.float32, device="cuda")
    wave_forward_static(op.ctx, nt, src, w, rec, rec_b, u0, fin_b, 3)
    torch.cuda.synchronize()
    return (rec_a, fin_a), (rec_b, fin_b)


def test_static_forward_equals_forward_twice_second_smaller():
    (ra, fa), (rb, fb) = _both((40, 44, 70), 30, 2, 50, 8, seed=11, time_tile=-1)
    assert torch.equal(ra, rb) and torch.equal(fa, fb)
    # a smaller second call: fewer planes, points and steps than the first left in the array
    (ra, fa), (rb, fb) = _both((20, 24, 30), 12, 1, 5, 4, seed=12, time_tile=2, tile_shape=2)
    assert torch.equal(ra, rb) and torch.equal(fa, fb)


def test_static_forward_refuses_calls_above_the_maximum():
    from paper_1806_08299_amd import WaveError, WaveOp
    from paper_1806_08299_amd.wave import WAVE_STATIC_SCRATCH_BYTES, wave_forward_static, wave_scratch_bytes
    shape = (16, 16, 16)
    m = torch.full(shape, 1.0 / 2000.0 ** 2, dtype=torch.float32, device="cuda")
    op = WaveOp(shape, 10.0, 1e-3, 4, m)
    nt, nrec = 400, 4000
    rec = np.random.default_rng(0).uniform(5.0, 150.0, size=(nrec, 3))
    assert wave_scratch_bytes(op.ctx, nt, 0, nrec, 0, 0) > WAVE_STATIC_SCRATCH_BYTES
    out = torch.empty((nt, nrec), dtype=torch.float32, device="cuda")
    with pytest.raises(WaveError) as e:
        wave_forward_static(op.ctx, nt, None, None, rec, out, None, None, 3)
    assert e.value.status == -4

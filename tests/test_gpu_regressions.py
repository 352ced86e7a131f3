"""GPU regression tests for host-side checks of the C ABI.

* wave_init / wave_set_model on grids smaller than the model reduction's
  former fixed grid: nothing is written past the caller's state buffer (a
  canary tail after the state stays untouched);
* a model with a NaN or an infinite entry is rejected (WAVE_EINVAL);
* reusing checkpoints with a different receiver count is rejected
  (WAVE_ESTATE), since the checkpoint offset in the scratch depends on it;
* diff_forward rejects any overlap of input, output and the context's own
  levels (WAVE_EINVAL), not only exact aliasing.
"""
import numpy as np
import pytest
import torch

import waveinputs as wi

pytestmark = pytest.mark.gpu

CANARY = 0x5A


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 3, 7), (5, 9, 13), (7, 1), (21, 1)])
def test_set_model_writes_nothing_past_the_state(shape):
    from paper_1806_08299_amd.wave import make_desc, wave_destroy, wave_init, wave_set_model, wave_state_bytes
    n = int(np.prod(shape))
    d = make_desc(shape, 10.0, 1e-3, 4, time_tile=-1)
    nb = wave_state_bytes(d)
    assert nb > 0
    tail = 8192
    buf = torch.full((nb + tail,), CANARY, dtype=torch.uint8, device="cuda")
    m = torch.full((n,), 1.0 / 2000.0 ** 2, dtype=torch.float32, device="cuda")
    print("canary test shape %s, state %d bytes" % (shape, nb), flush=True)
    ctx = wave_init(d, m, buf[:nb])
    try:
        wave_set_model(ctx, m * 1.01)
        torch.cuda.synchronize()
        assert bool((buf[nb:] == CANARY).all().item()), "bytes written past the end of the state buffer"
    finally:
        wave_destroy(ctx)


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), 0.0, -1e-7])
def test_model_with_invalid_entry_is_rejected(bad):
    from paper_1806_08299_amd import WaveError, WaveOp
    shape = (9, 10, 11)
    m = torch.full(shape, 1.0 / 2000.0 ** 2, dtype=torch.float32)
    op = WaveOp(shape, 10.0, 1e-3, 4, m.cuda())
    mb = m.clone()
    mb[4, 5, 6] = bad
    with pytest.raises(WaveError) as e:
        op.set_model(mb.cuda())
    assert e.value.status == -1
    # an all-NaN model too (a NaN-blind minimum would pass it)
    with pytest.raises(WaveError) as e:
        op.set_model(torch.full(shape, float("nan"), dtype=torch.float32).cuda())
    assert e.value.status == -1
    op.set_model(m.cuda())   # a valid model is still accepted afterwards


def test_reuse_with_other_receiver_count_is_rejected():
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import WaveError, wave_adjoint_grad, wave_scratch_bytes
    shape, nt, K = (20, 22, 24), 12, 4
    c = wi.smooth_random_velocity(shape, seed=3, sigma_cells=2.0, cmin=1500.0, cmax=2500.0)
    m = torch.from_numpy(wi.to_slowness2(c)).cuda()
    dt = 0.3 * 10.0 / 2500.0
    op = WaveOp(shape, 10.0, dt, 4, m)
    src = np.array([[100.0, 110.0, 120.0]])
    rec9 = np.stack([np.full(9, 20.0), np.full(9, 100.0), np.arange(9) * 20.0], axis=1)
    wav = torch.from_numpy(wi.ricker(nt, dt, 20.0).reshape(nt, 1)).cuda()
    # scratch large enough for either receiver count
    nb = wave_scratch_bytes(op.ctx, nt, 1, 9, K, 1)
    sc = op.scratch(nb)
    op.forward(nt, src, wav, rec9, ckpt_every=K, adjoint_scratch=True)
    rec5 = rec9[:5]
    resid = torch.zeros((nt, 5), dtype=torch.float32, device="cuda")
    gm = torch.empty(shape, dtype=torch.float32, device="cuda")
    with pytest.raises(WaveError) as e:
        wave_adjoint_grad(op.ctx, nt, src, wav, rec5, resid, gm, None, K, 1, sc, 3)
    assert e.value.status == -6


def test_diffusion_rejects_partial_overlap():
    from paper_1806_08299_amd import DiffOp, WaveError
    from paper_1806_08299_amd.wave import diff_forward
    w = wi.laplace(shape=(12, 10, 70), so=4, nt=3, seed=2)
    op = DiffOp(w.shape, w.spacing, w.dt, w.alpha, w.so, time_tile=-1)
    n = int(np.prod(w.shape))
    big = torch.zeros(2 * n, dtype=torch.float32, device="cuda")
    big[:n] = torch.from_numpy(w.u0.ravel()).cuda()
    u0 = big[:n].view(w.shape)
    for off in (1, 64, n - 1):   # output shifted by part of a field: overlaps the input
        with pytest.raises(WaveError) as e:
            diff_forward(op.ctx, 3, u0, big[off:off + n].view(w.shape))
        assert e.value.status == -1
    # input or output inside the context's own levels
    lvl = op.state[: 4 * n].view(torch.float32).view(w.shape)
    with pytest.raises(WaveError) as e:
        diff_forward(op.ctx, 3, lvl, torch.empty(w.shape, dtype=torch.float32, device="cuda"))
    assert e.value.status == -1
    with pytest.raises(WaveError) as e:
        diff_forward(op.ctx, 3, u0, lvl)
    assert e.value.status == -1
    # disjoint buffers still work
    out = big[n:].view(w.shape)
    diff_forward(op.ctx, 3, u0, out)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all().item())

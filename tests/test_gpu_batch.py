"""GPU parity of the batched shots (wave_batch through the C ABI).

Shots of different grids, orders, dimensions and schedules are advanced in
one captured sequence whose sweeps are merged across shots.  Bars:

* every shot's traces (and, with a gradient, its gradient) are bitwise those
  of the same shot run alone through wave_forward / wave_adjoint_grad;
* one shot against the FP64 oracle (relative L2 <= 1e-5);
* more shots of one instantiation than fit one launch (split launches);
* a repeated call replays the captured graph and follows new device inputs;
* error paths.
"""
import numpy as np
import pytest
import torch

import oracle
import waveinputs as wi

pytestmark = pytest.mark.gpu

# (shape, space order, schedule (T, tile shape), layer width)
SHOTS = [
    ((40, 44, 52), 4, (2, 1), 4),
    ((36, 50, 40), 8, (-1, 0), 0),
    ((48, 36, 44), 4, (2, 1), 0),
    ((44, 40, 36), 8, (-1, 0), 4),
    ((38, 42, 46), 8, (1, 2), 3),
    ((60, 70), 4, (2, 0), 5),
    ((50, 66), 4, (2, 0), 0),
    ((46, 40, 42), 8, (2, 2), 0),
    ((40, 48, 38), 8, (2, 2), 4),
]
NT = 37
K = 8


def _shot(i, shape, so, nbl, nt=NT):
    rng = np.random.default_rng(100 + i)
    nd = len(shape)
    c = wi.smooth_random_velocity(shape, seed=i, sigma_cells=3.0, cmin=1800.0, cmax=2600.0)
    m = wi.to_slowness2(c)
    h = (10.0,) * nd
    dt = 0.35 * 10.0 / 2600.0
    src = np.array([[rng.uniform(nbl + 2, shape[a] - nbl - 3) * h[a] for a in range(nd)]])
    rec = np.array([[np.clip(src[0][a] / h[a] + rng.uniform(-6, 6), 0, shape[a] - 1) * h[a] for a in range(nd)]
                    for _ in range(5)])
    wav = wi.ricker(nt, dt, 30.0, t0=0.02 + 0.003 * i)[:, None].astype(np.float32)
    smax = wi.sigma_max_estimate(2600.0, nbl, 10.0) if nbl else 0.0
    return dict(shape=shape, so=so, nbl=nbl, smax=smax, m=m, h=h, dt=dt, src=src, rec=rec, wav=wav)


def _op(S, sched):
    from paper_1806_08299_amd import WaveOp
    op = WaveOp(S["shape"], S["h"], S["dt"], S["so"], torch.from_numpy(S["m"]).cuda(), nbl=S["nbl"],
                sigma_max=S["smax"], time_tile=-1)
    T, shape = sched
    op.set_schedule(T, 0, shape if shape else 1, 0)
    return op


@pytest.fixture(scope="module")
def shots():
    return [_shot(i, sh, so, nbl) for i, (sh, so, _, nbl) in enumerate(SHOTS)]


def _single_forward(S, sched, wav):
    op = _op(S, sched)
    rec, _ = op.forward(NT, S["src"], wav, S["rec"])
    torch.cuda.synchronize()
    return rec.cpu().numpy()


@pytest.mark.parametrize("branches", ["1", "0"])
def test_batch_forward_bitwise_equals_single_shots(shots, branches, monkeypatch):
    """Shots of different radii in independent graph branches (default) or
    on one stream: bitwise the shots run alone either way."""
    from paper_1806_08299_amd import ShotBatch
    monkeypatch.setenv("WAVE_BATCH_BRANCHES", branches)
    ops = [_op(S, SHOTS[i][2]) for i, S in enumerate(shots)]
    wavs = [torch.from_numpy(S["wav"]).cuda() for S in shots]
    B = ShotBatch(ops, NT, [S["src"] for S in shots], [S["rec"] for S in shots])
    recs, _ = B.run(wavs)
    torch.cuda.synchronize()
    for i, S in enumerate(shots):
        ref = _single_forward(S, SHOTS[i][2], wavs[i])
        got = recs[i].cpu().numpy()
        assert np.abs(ref).max() > 0, i
        assert np.array_equal(got, ref), i
    # one shot against the FP64 oracle
    S = shots[0]
    g = oracle.Grid(S["shape"], S["h"], S["dt"], S["so"], nbl=S["nbl"], sigma_max=S["smax"])
    o = oracle.forward(g, S["m"].astype(np.float64), NT, S["src"], S["wav"].astype(np.float64), S["rec"])
    r = recs[0].cpu().numpy().astype(np.float64)
    assert np.linalg.norm(r - o["rec"]) / np.linalg.norm(o["rec"]) <= 1e-5


@pytest.mark.parametrize("branches", ["1", "0"])
def test_batch_gradient_bitwise_equals_single_shots(shots, branches, monkeypatch):
    from paper_1806_08299_amd import ShotBatch
    monkeypatch.setenv("WAVE_BATCH_BRANCHES", branches)
    ops = [_op(S, SHOTS[i][2]) for i, S in enumerate(shots)]
    wavs = [torch.from_numpy(S["wav"]).cuda() for S in shots]
    rng = np.random.default_rng(7)
    dobs = [torch.from_numpy((1e-3 * rng.standard_normal((NT, 5))).astype(np.float32)).cuda() for _ in shots]
    B = ShotBatch(ops, NT, [S["src"] for S in shots], [S["rec"] for S in shots], ckpt_every=K, gradient=True)
    recs, grads = B.run(wavs, dobs)
    torch.cuda.synchronize()
    for i, S in enumerate(shots):
        op = _op(S, SHOTS[i][2])
        rec, _ = op.forward(NT, S["src"], wavs[i], S["rec"], ckpt_every=K, adjoint_scratch=True)
        resid = rec - dobs[i]
        gm, _ = op.adjoint_grad(NT, S["src"], wavs[i], S["rec"], resid, K, want_grad_wavelet=False, reuse=True)
        torch.cuda.synchronize()
        assert np.array_equal(recs[i].cpu().numpy(), rec.cpu().numpy()), i
        g = grads[i].cpu().numpy()
        assert np.abs(g).max() > 0, i
        assert np.array_equal(g, gm.cpu().numpy()), i


def test_batch_replay_follows_new_inputs(shots):
    from paper_1806_08299_amd import ShotBatch
    sel = [0, 1, 5]
    ops = [_op(shots[i], SHOTS[i][2]) for i in sel]
    wavs = [torch.from_numpy(shots[i]["wav"]).cuda() for i in sel]
    B = ShotBatch(ops, NT, [shots[i]["src"] for i in sel], [shots[i]["rec"] for i in sel])
    first = [r.cpu().numpy().copy() for r in B.run(wavs)[0]]
    for w in wavs:
        w.mul_(-2.0)                       # same tensors, new contents: the graph is replayed
    second = [r.cpu().numpy().copy() for r in B.run(wavs)[0]]
    for k, i in enumerate(sel):
        ref = _single_forward(shots[i], SHOTS[i][2], wavs[k])
        assert np.array_equal(second[k], ref), i
        assert not np.array_equal(second[k], first[k])
    # another call on one of the contexts invalidates the captured graph
    ops[1].forward(NT, shots[1]["src"], wavs[1], shots[1]["rec"][:2])
    third = [r.cpu().numpy().copy() for r in B.run(wavs)[0]]
    for k in range(len(sel)):
        assert np.array_equal(third[k], second[k])


def test_batch_more_shots_than_one_launch():
    from paper_1806_08299_amd import ShotBatch
    n = 14                                  # beyond the 12 shots of one launch
    S = [_shot(20 + i, (24 + 2 * (i % 3), 28, 30 + 2 * (i % 4)), 4, 0, nt=12) for i in range(n)]
    for s in S:
        s["wav"] = s["wav"][:12]
    for sched in ((-1, 0), (2, 1)):
        ops = [_op(s, sched) for s in S]
        wavs = [torch.from_numpy(s["wav"]).cuda() for s in S]
        B = ShotBatch(ops, 12, [s["src"] for s in S], [s["rec"] for s in S])
        recs, _ = B.run(wavs)
        torch.cuda.synchronize()
        for i, s in enumerate(S):
            op = _op(s, sched)
            ref, _ = op.forward(12, s["src"], wavs[i], s["rec"])
            assert np.array_equal(recs[i].cpu().numpy(), ref.cpu().numpy()), (sched, i)


def test_batch_errors(shots):
    from paper_1806_08299_amd import ShotBatch, WaveError
    S = shots[0]
    wav = torch.from_numpy(S["wav"]).cuda()
    op = _op(S, (2, 1))
    with pytest.raises(WaveError) as e:              # the same context twice
        ShotBatch([op, op], NT, [S["src"]] * 2, [S["rec"]] * 2).run([wav, wav])
    assert e.value.status == -1
    from paper_1806_08299_amd.wave import wave_tiled_max_depth
    if wave_tiled_max_depth(4, 3, 1) >= 3:
        deep = _op(S, (3, 1))                        # batched kernels stop at depth 2
        with pytest.raises(WaveError) as e:
            ShotBatch([deep], NT, [S["src"]], [S["rec"]]).run([wav])
        assert e.value.status == -7
    with pytest.raises(ValueError):
        ShotBatch([op], NT, [S["src"]], [S["rec"]], gradient=True)

"""GPU tests of the skewed schedule (slab > 0): the paper's time tile with the
axis-0 loop skewed by the time index, executed slab after slab in dependence
order (implementation chapter, "Time-tiling"), every point of every step
computed once by the single-step kernel.

Criterion (evaluation chapter, "Functional correctness"): bitwise equality
with the untiled sweep -- final state, receiver traces, gradients and the
diffusion field -- for depths far beyond the register-tiled kernels' limits,
slabs thinner than skew + radius (so a z-stencil reaches two slabs back),
slabs that do not divide the grid, skews above the radius, windows longer
than the run, every space order; and the legality checks of the schedule.
"""
import numpy as np
import pytest
import torch

import oracle
import waveinputs as wi
from test_gpu_forward import TOL, _oracle, _op, _run, _small, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
def test_skewed_every_order_bitwise(so):
    R = so // 2
    w = _small(so, (61, 37, 70), nbl=3, seed=300 + so, nt=19)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    ref = _oracle(w)
    assert rel(fin_u[0], ref["final"][0]) <= TOL
    for T, Z, skew in [(1, 16, 0), (3, 7, 0), (8, 16, R + 3), (16, 25, 0), (32, 100, 0), (5, max(1, R), 0)]:
        print("so %d skewed T=%d slab=%d skew=%d" % (so, T, Z, skew), flush=True)
        op.set_schedule(T, skew, 0, 0, slab=Z)
        sch = op.schedule()
        assert sch.slab == Z and sch.T == T and sch.tile == (0, 0)
        rec_t, fin_t = _run(op, w)
        assert np.array_equal(fin_t, fin_u), (so, T, Z, skew)
        assert np.array_equal(rec_t, rec_u), (so, T, Z, skew)


@pytest.mark.parametrize("zchunks", [0, 1, 3])
def test_skewed_2d_and_segments_bitwise(zchunks):
    w = _small(8, (75, 1100), nbl=4, seed=311, nt=23)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    for T, Z in [(4, 20), (8, 9), (23, 40)]:
        op.set_schedule(T, 0, 0, zchunks, slab=Z)
        rec_t, fin_t = _run(op, w)
        assert np.array_equal(fin_t, fin_u), (T, Z, zchunks)
        assert np.array_equal(rec_t, rec_u), (T, Z, zchunks)


def test_skewed_gradient_bitwise():
    from test_gpu_adjoint import _grad, _op as _aop, _problem
    P = _problem()
    # any residual will do: the comparison is with the untiled sweep
    P["resid"] = np.random.default_rng(5).standard_normal((P["nt"], P["rec"].shape[0])).astype(np.float32)
    op = _aop(P, P["m0"], time_tile=-1)
    g_u, q_u = _grad(op, P, 7)
    for T, Z, K, zc in [(4, 10, 7, 0), (8, 16, 40, 0), (3, 5, 13, 0), (6, 12, 9, 3), (2, 7, 5, 2)]:
        print("gradient skewed T=%d slab=%d K=%d zchunks=%d" % (T, Z, K, zc), flush=True)
        op.set_schedule(T, 0, 0, zc, slab=Z)
        g_t, q_t = _grad(op, P, K)
        assert np.array_equal(g_t, g_u), (T, Z, K, zc)
        assert np.array_equal(q_t, q_u), (T, Z, K, zc)
    # the untiled sweep in several axis-0 segments (its adjoint fetches the
    # history and the gradient two planes ahead, up to each segment's end)
    for zc in (2, 5, 36):
        print("gradient untiled zchunks=%d" % zc, flush=True)
        op.set_schedule(-1, 0, 0, zc)
        g_t, q_t = _grad(op, P, 11)
        assert np.array_equal(g_t, g_u), zc
        assert np.array_equal(q_t, q_u), zc


@pytest.mark.parametrize("so", [2, 8, 16])
def test_skewed_diffusion_bitwise(so):
    from paper_1806_08299_amd import DiffOp
    w = wi.laplace(shape=(53, 30, 75), so=so, nt=13, seed=so)
    u0 = torch.from_numpy(w.u0).cuda()
    op = DiffOp(w.shape, w.spacing, w.dt, w.alpha, w.so, time_tile=-1)
    ref = op.forward(w.nt, u0).cpu().numpy()
    lref = oracle.diffuse(oracle.Grid(w.shape, w.spacing, w.dt, w.so), w.alpha, w.nt, w.u0.astype(np.float64))
    assert rel(ref, lref) <= TOL
    for T, Z in [(2, 8), (4, 16), (13, 30), (6, 3)]:
        op.set_schedule(T, 0, 0, 0, slab=Z)
        got = op.forward(w.nt, u0).cpu().numpy()
        assert np.array_equal(got, ref), (so, T, Z)


def test_skewed_schedule_validation():
    from paper_1806_08299_amd import WaveError
    w = _small(8, (30, 33, 40), nbl=2, seed=320, nt=5)
    op = _op(w, time_tile=-1)
    before = op.schedule()
    with pytest.raises(WaveError) as e:
        op.set_schedule(-1, 0, 0, 0, slab=16)       # skewing needs a time tile
    assert e.value.status == -1
    with pytest.raises(WaveError) as e:
        op.set_schedule(4, 3, 0, 0, slab=16)        # skew below the radius
    assert e.value.status == -2
    with pytest.raises(WaveError) as e:
        op.set_schedule(2, 0, 0, 0, tile=(48, 64))  # not a built tile
    assert e.value.status == -7
    assert op.schedule() == before                  # unchanged after a rejected call
    # depth beyond every register-tiled kernel, fine when skewed
    op.set_schedule(64, 0, 0, 0, slab=12)
    assert op.schedule().T == 64


def test_skewed_shot_in_a_batch_bitwise():
    from paper_1806_08299_amd import ShotBatch
    ws = [_small(4, (40, 36, 50), nbl=0, seed=330, nt=12), _small(8, (33, 30, 70), nbl=2, seed=331, nt=12)]
    ops, singles = [], []
    for i, w in enumerate(ws):
        op = _op(w, time_tile=-1)
        op.set_schedule(4, 0, 0, 0, slab=10 + 5 * i)
        rec, _ = op.forward(w.nt, w.src_xyz, torch.from_numpy(w.wavelet).cuda(), w.rec_xyz)
        singles.append(rec.clone())
        ops.append(op)
    B = ShotBatch(ops, 12, [w.src_xyz for w in ws], [w.rec_xyz for w in ws])
    recs, _ = B.run([torch.from_numpy(w.wavelet).cuda() for w in ws])
    torch.cuda.synchronize()
    for a, b in zip(recs, singles):
        assert torch.equal(a, b)

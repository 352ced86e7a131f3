"""Parity at full size: the benchmark's forward workload (512^3 + 40-point
layer = 592^3, space order 8) in its launch configurations, the largest grid
and order of the workload list (768^3 + 40 = 848^3 at space order 16, with
the fast layered model in place of the smooth one: the properties below do
not depend on the model), and the 256^3 (+40) gradient problem over 2000
steps.

These are too large for the FP64 oracle to follow over many steps, so
properties are checked instead:

* from a seeded random state (which excites every point, the absorbing layer
  and the grid faces), 10 steps of every benchmarked schedule -- the untiled
  sweep in the benchmark's 16-segment configuration and the time-tiled
  schedules -- are bitwise equal;
* one further step from the GPU's own state equals one FP64 oracle step from
  the same state within relative L2 1e-6 over the whole grid, and the
  receiver samples of that step within 1e-5.  One step is ~30 FP32
  operations (2^-24 ~ 6e-8 each, mostly independent) plus FP32 coefficients
  and b, so the expected error is ~1e-7 (measured 6e-8); 1e-6 leaves margin
  while any wrong term (an O(1) change) fails;
* gradient problem: the FP32 dot-product test <F q, dd> = <q, F^T dd> over
  2000 steps within 1e-4, and the gradient bitwise independent of the
  checkpoint interval and of the schedule (untiled vs time-tiled adjoint);
* the Laplace-operator workload (explicit diffusion) at 500^3, orders 2 and
  8: the bench's time-tiled launch configurations bitwise equal to the
  untiled sweep, and one further step against the FP64 oracle (1e-6).
"""
import numpy as np
import pytest
import torch

import oracle
import waveinputs as wi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,so", [(512, 8), (768, 16)])
def test_full_size_schedules_and_one_step_against_oracle(n, so):
    from paper_1806_08299_amd import WaveOp
    from paper_1806_08299_amd.wave import wave_tiled_max_depth
    w = wi.layered_512(nt=11, n=n, so=so)              # n^3 + 40-point layer
    dev = torch.device("cuda")
    op = WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).to(dev), nbl=w.nbl,
                sigma_max=w.sigma_max, time_tile=-1)
    gen = torch.Generator(device=dev).manual_seed(0)
    u0 = torch.randn((2,) + tuple(w.shape), generator=gen, device=dev, dtype=torch.float32)
    wav = torch.from_numpy(w.wavelet).to(dev)
    nt0 = 10
    print("full size: untiled, 16 segments", flush=True)
    op.set_schedule(-1, 0, 1, 16)
    rec_u, fin_u = op.forward(nt0, w.src_xyz, wav[:nt0].contiguous(), w.rec_xyz, u_init=u0, want_final=True)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(fin_u).all())
    for T, shape, zc in ((-1, 1, 0), (1, 1, 0), (1, 2, 0), (2, 2, 0), (2, 1, 4)):
        if T > wave_tiled_max_depth(so, 3, shape):
            continue
        print("full size: T=%d shape=%d zchunks=%d" % (T, shape, zc), flush=True)
        op.set_schedule(T, 0, shape, zc)
        rec_t, fin_t = op.forward(nt0, w.src_xyz, wav[:nt0].contiguous(), w.rec_xyz, u_init=u0, want_final=True)
        torch.cuda.synchronize()
        assert torch.equal(fin_t, fin_u), (T, shape, zc)
        assert torch.equal(rec_t, rec_u), (T, shape, zc)
        del rec_t, fin_t
    # one more step, GPU vs FP64 oracle, from the GPU's state after nt0 steps
    op.set_schedule(-1, 0, 1, 16)
    rec1, fin1 = op.forward(1, w.src_xyz, wav[nt0:nt0 + 1].contiguous(), w.rec_xyz, u_init=fin_u, want_final=True)
    torch.cuda.synchronize()
    state = fin_u.cpu().numpy().astype(np.float64)
    got = fin1.cpu().numpy()
    del fin1, fin_u, u0
    torch.cuda.empty_cache()
    assert np.array_equal(got[1], state[0].astype(np.float32))   # the level carried over
    g = oracle.Grid(w.shape, w.spacing, w.dt, w.so, nbl=w.nbl, sigma_max=w.sigma_max)
    print("full size: oracle step", flush=True)
    o = oracle.forward(g, w.m.astype(np.float64), 1, w.src_xyz, w.wavelet[nt0:nt0 + 1].astype(np.float64),
                       w.rec_xyz, u_init=state, want_final=True)
    ref = o["final"][0]
    err = np.linalg.norm(got[0].astype(np.float64) - ref) / np.linalg.norm(ref)
    print("full size: one-step relative L2 %.3e" % err, flush=True)
    assert err <= 1e-6
    r = rec1.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(r - o["rec"]) / np.linalg.norm(o["rec"]) <= 1e-5


def test_full_size_gradient_dot_product_and_schedule_independence():
    from paper_1806_08299_amd import WaveOp
    w4 = wi.gradient_256()                              # 336^3 with the layer, so8, 2000 steps, K = 50
    w = w4["init"]
    dev = torch.device("cuda")
    op = WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).to(dev), nbl=w.nbl,
                sigma_max=w.sigma_max, time_tile=-1)
    rng = np.random.default_rng(11)
    q = torch.from_numpy(rng.standard_normal((w.nt, 1)).astype(np.float32)).to(dev)
    dd = torch.from_numpy(rng.standard_normal((w.nt, w.rec_xyz.shape[0])).astype(np.float32)).to(dev)
    print("gradient: forward", flush=True)
    rec, _ = op.forward(w.nt, w.src_xyz, q, w.rec_xyz)
    print("gradient: adjoint", flush=True)
    gm, gq = op.adjoint_grad(w.nt, w.src_xyz, q, w.rec_xyz, dd, 50)
    torch.cuda.synchronize()
    lhs = float((rec.double() * dd.double()).sum())
    rhs = float((q.double() * gq.double()).sum())
    print("gradient: dot test %.3e" % (abs(lhs - rhs) / abs(lhs)), flush=True)
    assert abs(lhs - rhs) / abs(lhs) < 1e-4
    assert bool(torch.isfinite(gm).all()) and float(gm.abs().max()) > 0
    for T, shape, K in ((-1, 1, 40), (2, 2, 50), (1, 1, 64)):
        print("gradient: T=%d shape=%d K=%d" % (T, shape, K), flush=True)
        op.set_schedule(T, 0, shape, 0)
        gm2, _ = op.adjoint_grad(w.nt, w.src_xyz, q, w.rec_xyz, dd, K, want_grad_wavelet=False)
        torch.cuda.synchronize()
        assert torch.equal(gm2, gm), (T, shape, K)
        del gm2
    # the history of the last 8 of 40 segments kept from the forward (61 GB)
    print("gradient: 8 segments kept", flush=True)
    op.set_schedule(-1, 0, 1, 0)
    gm2, _ = op.adjoint_grad(w.nt, w.src_xyz, q, w.rec_xyz, dd, 50, want_grad_wavelet=False, keep_segments=8)
    torch.cuda.synchronize()
    from paper_1806_08299_amd.wave import wave_last_kept_segments
    assert wave_last_kept_segments(op.ctx) == 8
    assert torch.equal(gm2, gm)
    del gm2, op
    torch.cuda.empty_cache()


@pytest.mark.parametrize("so,scheds", [(2, [(4, 2, 8), (4, 2, 0), (2, 2, 32)]), (8, [(1, 2, 4), (2, 2, 0)])])
def test_full_size_diffusion(so, scheds):
    """The Laplace-operator workload at the paper's 500^3 grid: the bench's
    time-tiled launch configurations bitwise equal to the untiled sweep over
    8 steps, then one more step against one FP64 oracle step over the whole
    grid (relative L2 1e-6, the bound argued above for one step)."""
    from paper_1806_08299_amd import DiffOp
    w = wi.laplace(n=500, so=so, nt=8)
    op = DiffOp(w.shape, w.spacing, w.dt, w.alpha, w.so)
    u0 = torch.from_numpy(w.u0).cuda()
    print("full-size diffusion so%d: untiled" % so, flush=True)
    ref = op.forward(w.nt, u0)
    torch.cuda.synchronize()
    for T, shape, zc in scheds:
        print("full-size diffusion so%d: T=%d shape=%d zc=%d" % (so, T, shape, zc), flush=True)
        op.set_schedule(T, 0, shape, zc)
        assert torch.equal(op.forward(w.nt, u0), ref), (T, shape, zc)
    op.set_schedule(-1, 0, 0, 0)
    one = op.forward(1, ref).cpu().numpy().astype(np.float64)
    state = ref.cpu().numpy().astype(np.float64)
    del ref, u0
    torch.cuda.empty_cache()
    g = oracle.Grid(w.shape, w.spacing, w.dt, w.so)
    expect = oracle.diffuse(g, w.alpha, 1, state)
    err = np.linalg.norm(one - expect) / np.linalg.norm(expect)
    print("full-size diffusion so%d: one-step relative L2 %.3e" % (so, err), flush=True)
    assert err <= 1e-6

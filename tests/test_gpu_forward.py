"""GPU parity of the forward sweep (untiled and time-tiled) through the C ABI.

* untiled GPU (FP32) vs the FP64 oracle: relative L2 <= 1e-5 on the final two
  levels and on the receiver traces;
* time-tiled GPU vs untiled GPU: bitwise, for every fused depth T, tile shape,
  skew and axis-0 segmentation available for the order (the paper's
  functional-correctness criterion);
* edge cases: ragged grids smaller than a tile, partial last windows, nt = 0,
  points on nodes / on the boundary / outside the grid, 2D, every order, no
  sources or receivers, grids of a single point, plane or row.
"""
import numpy as np
import pytest
import torch

import oracle
import waveinputs as wi
from parity import assert_field, assert_traces

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _op(w, **kw):
    from paper_1806_08299_amd import WaveOp
    return WaveOp(w.shape, w.spacing, w.dt, w.so, torch.from_numpy(w.m).cuda(), nbl=w.nbl,
                  sigma_max=w.sigma_max, **kw)


def _run(op, w, nt=None, want_final=True):
    nt = w.nt if nt is None else nt
    wav = torch.from_numpy(np.ascontiguousarray(w.wavelet[:nt])).cuda()
    rec, fin = op.forward(nt, w.src_xyz, wav, w.rec_xyz, want_final=want_final)
    torch.cuda.synchronize()
    return (rec.cpu().numpy() if rec is not None else None), (fin.cpu().numpy() if fin is not None else None)


def _oracle(w, nt=None):
    nt = w.nt if nt is None else nt
    g = oracle.Grid(w.shape, w.spacing, w.dt, w.so, nbl=w.nbl, sigma_max=w.sigma_max)
    return oracle.forward(g, w.m.astype(np.float64), nt, w.src_xyz, w.wavelet[:nt].astype(np.float64),
                          w.rec_xyz, want_final=True)


def rel(a, b):
    return np.linalg.norm(np.ravel(a).astype(np.float64) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _schedules(R, ndim):
    """Every (T, tile shape) built for radius R; the caller drops those the
    device cannot hold (WAVE_EUNSUPPORTED from set_schedule)."""
    from paper_1806_08299_amd.wave import wave_tiled_max_depth
    from paper_1806_08299_amd.wave import tile_table
    out = []
    for shape in (range(1, len(tile_table(3)) + 1) if ndim == 3 else (0,)):
        for T in range(1, wave_tiled_max_depth(2 * R, ndim, shape) + 1):
            out.append((T, shape))
    return out


def _try_schedule(op, T, shape, skew=0, zchunks=0):
    from paper_1806_08299_amd import WaveError
    try:
        op.set_schedule(T, skew, shape, zchunks)
        return True
    except WaveError as e:
        if e.status != -7:
            raise
        print("schedule T=%d shape=%d unavailable: %s" % (T, shape, e))
        return False


# --------------------------------------------------------------------------- 64^3 so4 point source, 100 steps

@pytest.fixture(scope="module")
def ps64_ref():
    w = wi.point_source_64()
    return w, _oracle(w)


def test_point_source_64_untiled_matches_oracle(ps64_ref):
    w, ref = ps64_ref
    op = _op(w, time_tile=-1)
    rec, fin = _run(op, w)
    assert np.abs(fin).max() > 1e-3, "solution is (nearly) zero"
    assert np.all(np.isfinite(fin))
    for lev in (0, 1):
        assert_field(fin[lev], ref["final"][lev], TOL, "level %d" % lev)
    assert_traces(rec, ref["rec"], TOL)


@pytest.mark.parametrize("T", [1, 2, 4])
def test_point_source_64_tiled_bitwise_equals_untiled(ps64_ref, T):
    w, ref = ps64_ref
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    for shape in (1, 2, 3, 4):
        if not _try_schedule(op, T, shape):
            continue
        rec_t, fin_t = _run(op, w)
        assert np.array_equal(fin_t, fin_u), (T, shape)
        assert np.array_equal(rec_t, rec_u), (T, shape)
    assert_field(fin_t[0], ref["final"][0], TOL)


# --------------------------------------------------------------------------- every order

def _small(so, shape, nbl, seed, nt=24, nsrc=2, nrec=7):
    rng = np.random.default_rng(seed)
    nd = len(shape)
    h = tuple(float(v) for v in rng.uniform(8.0, 12.0, size=nd))
    c = rng.uniform(1500, 3000, size=shape)
    m = wi.to_slowness2(c)
    dt = 0.35 * min(h) / 3000.0
    src = np.array([[rng.uniform(0.2, shape[a] - 1.2) * h[a] for a in range(nd)] for _ in range(nsrc)])
    # receivers within a few cells of a source, so that every trace is non-zero within nt steps
    rec = np.array([[np.clip(src[i % nsrc][a] / h[a] + rng.uniform(-5.0, 5.0), 0.0, shape[a] - 1.0) * h[a]
                     for a in range(nd)] for i in range(nrec)])
    wav = rng.standard_normal((nt, nsrc)).astype(np.float32)
    u0 = 1e-3 * rng.standard_normal(shape)
    return wi.Workload("small", tuple(shape), h, dt, so, nt, nbl, 60.0 if nbl else 0.0, m, src, wav, rec,
                       extra={"u0": u0})


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
def test_every_order_3d_oracle_and_bitwise(so):
    R = so // 2
    shape = (4 * R + 7, 83, 71)   # ragged: not multiples of any tile
    w = _small(so, shape, nbl=3, seed=so)
    ref = _oracle(w)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    assert_field(fin_u[0], ref["final"][0], TOL)
    assert_traces(rec_u, ref["rec"], TOL)
    ran = 0
    for T, shp in _schedules(R, 3):
        if not _try_schedule(op, T, shp):
            continue
        ran += 1
        rec_t, fin_t = _run(op, w)
        assert np.array_equal(fin_t, fin_u), (so, T, shp)
        assert np.array_equal(rec_t, rec_u), (so, T, shp)
    assert ran >= 2


@pytest.mark.parametrize("so", [2, 4, 8, 16])
def test_every_order_2d_oracle_and_bitwise(so):
    R = so // 2
    shape = (57, 1100)   # axis 1 longer than one 2D tile
    w = _small(so, shape, nbl=4, seed=100 + so, nt=30)
    ref = _oracle(w)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    assert_field(fin_u[0], ref["final"][0], TOL)
    assert_traces(rec_u, ref["rec"], TOL)
    for T, shp in _schedules(R, 2):
        if not _try_schedule(op, T, shp):
            continue
        rec_t, fin_t = _run(op, w)
        assert np.array_equal(fin_t, fin_u), (so, T)
        assert np.array_equal(rec_t, rec_u), (so, T)


@pytest.mark.parametrize("skew_extra,zchunks", [(1, 0), (2, 3), (0, 1), (0, 5)])
def test_skew_and_segmentation_bitwise(skew_extra, zchunks):
    w = _small(8, (45, 70, 90), nbl=5, seed=7)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    op.set_schedule(2, 4 + skew_extra, 2, zchunks)
    rec_t, fin_t = _run(op, w)
    assert np.array_equal(fin_t, fin_u)
    assert np.array_equal(rec_t, rec_u)


def test_partial_windows_and_nt_edge_cases():
    w = _small(4, (30, 40, 50), nbl=2, seed=9, nt=7)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    op.set_schedule(4, 0, 2, 0)          # windows 4 + 3
    rec_t, fin_t = _run(op, w)
    assert np.array_equal(fin_t, fin_u) and np.array_equal(rec_t, rec_u)
    ref = _oracle(w)
    assert_field(fin_u[0], ref["final"][0], TOL)
    # nt = 0: final state is the (zero) initial state, no traces
    rec0, fin0 = _run(op, w, nt=0)
    assert np.array_equal(fin0, np.zeros_like(fin0))


def test_tiny_grid_and_points_on_boundary_or_outside():
    so = 8
    shape = (9, 5, 13)                    # smaller than every tile in every axis
    w = _small(so, shape, nbl=0, seed=11, nt=12)
    h = w.spacing
    w.src_xyz = np.array([[4 * h[0], 2 * h[1], 6 * h[2]],              # on a node
                          [0.0, 0.0, 0.0],                             # on the corner node
                          [8 * h[0], 4.5 * h[1], 12 * h[2]]])          # on the far faces
    w.wavelet = np.random.default_rng(3).standard_normal((12, 3)).astype(np.float32)
    w.rec_xyz = np.array([[3.3 * h[0], 1.1 * h[1], 7.7 * h[2]],
                          [-50.0, 1.0, 1.0],                           # outside: zero trace
                          [8 * h[0], 4 * h[1], 12 * h[2]]])
    ref = _oracle(w)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    assert_field(fin_u[0], ref["final"][0], TOL)
    assert np.array_equal(rec_u[:, 1], np.zeros(12, np.float32))
    assert_traces(rec_u, ref["rec"], TOL)
    for T, shp in _schedules(4, 3):
        if not _try_schedule(op, T, shp):
            continue
        rec_t, fin_t = _run(op, w)
        assert np.array_equal(fin_t, fin_u) and np.array_equal(rec_t, rec_u), (T, shp)


def test_initial_state_and_resume_bitwise():
    w = _small(6, (40, 33, 66), nbl=3, seed=13, nt=20)
    op = _op(w, time_tile=3)
    u0 = torch.from_numpy(np.stack([w.extra["u0"], 0.5 * w.extra["u0"]]).astype(np.float32)).cuda()
    wav = torch.from_numpy(w.wavelet).cuda()
    rec_full, fin_full = op.forward(20, w.src_xyz, wav, w.rec_xyz, u_init=u0, want_final=True)
    rec_a, fin_a = op.forward(9, w.src_xyz, wav[:9].contiguous(), w.rec_xyz, u_init=u0, want_final=True)
    rec_b, fin_b = op.forward(11, w.src_xyz, wav[9:].contiguous(), w.rec_xyz, u_init=fin_a, want_final=True)
    assert torch.equal(torch.cat([rec_a, rec_b]), rec_full)
    assert torch.equal(fin_b, fin_full)
    g = oracle.Grid(w.shape, w.spacing, w.dt, w.so, nbl=w.nbl, sigma_max=w.sigma_max)
    ref = oracle.forward(g, w.m.astype(np.float64), 20, w.src_xyz, w.wavelet.astype(np.float64), w.rec_xyz,
                         u_init=u0.cpu().numpy().astype(np.float64), want_final=True)
    assert_field(fin_full.cpu().numpy()[0], ref["final"][0], TOL)


def test_error_paths():
    from paper_1806_08299_amd import WaveError
    w = _small(8, (20, 20, 20), nbl=0, seed=1, nt=4)
    with pytest.raises(WaveError) as e:
        _op(w, time_tile=2, skew=3)
    assert e.value.status == -2                       # WAVE_ESKEW
    bad = _small(8, (20, 20, 20), nbl=0, seed=1, nt=4)
    bad.dt = w.dt * 1.5 / 0.35                        # CFL far above the limit
    with pytest.raises(WaveError) as e:
        _op(bad)
    assert e.value.status == -3                       # WAVE_ECFL
    op = _op(w, time_tile=-1)
    with pytest.raises(WaveError) as e:
        op.set_schedule(7, 0, 1, 0)                   # T beyond what is built for so8
    assert e.value.status == -7
    from paper_1806_08299_amd.wave import wave_forward
    tiny = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(WaveError) as e:
        wave_forward(op.ctx, 4, None, None, None, None, None, None, 0, tiny, 3)
    assert e.value.status == -4                       # WAVE_ENOMEM


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 7, 3), (6, 1, 9), (1, 5), (7, 1)])
def test_empty_point_sets_and_degenerate_grids(shape):
    """No sources, no receivers, grids of one point / one plane / one row,
    from a random initial state: oracle parity and every schedule bitwise."""
    so, nt = 4, 9
    nd = len(shape)
    rng = np.random.default_rng(21)
    h = (10.0,) * nd
    m = wi.to_slowness2(rng.uniform(1500, 3000, size=shape))
    dt = 0.35 * 10.0 / 3000.0
    u0 = rng.standard_normal((2,) + tuple(shape)).astype(np.float32)
    w = wi.Workload("degenerate", tuple(shape), h, dt, so, nt, 0, 0.0, m, np.zeros((0, nd)),
                    np.zeros((nt, 0), np.float32), np.zeros((0, nd)))
    g = oracle.Grid(shape, h, dt, so)
    ref = oracle.forward(g, m.astype(np.float64), nt, u_init=u0.astype(np.float64), want_final=True)
    op = _op(w, time_tile=-1)
    ui = torch.from_numpy(u0).cuda()
    rec, fin = op.forward(nt, None, None, None, u_init=ui, want_final=True)
    torch.cuda.synchronize()
    assert rec is None
    fin_u = fin.cpu().numpy()
    assert_field(fin_u[0], ref["final"][0], TOL)
    assert_field(fin_u[1], ref["final"][1], TOL)
    for T, shp in _schedules(2, nd):
        if not _try_schedule(op, T, shp):
            continue
        _, fin_t = op.forward(nt, None, None, None, u_init=ui, want_final=True)
        torch.cuda.synchronize()
        assert np.array_equal(fin_t.cpu().numpy(), fin_u), (T, shp)
    # adjoint with no receivers and no sources: the gradient is exactly zero
    gm, gq = op.adjoint_grad(nt, None, None, None, torch.zeros((nt, 0), device="cuda"), 4)
    torch.cuda.synchronize()
    assert gq is None
    assert not bool(gm.abs().max() > 0)


@pytest.mark.parametrize("so,shape,expect", [(2, (40, 70, 80), 3), (4, (40, 70, 80), 2), (6, (40, 70, 80), -1),
                                               (8, (40, 70, 80), -1), (2, (50, 300), 6), (4, (50, 300), 4),
                                               (6, (50, 300), 3), (8, (50, 300), 3), (16, (50, 300), -1)])
def test_default_schedule(so, shape, expect):
    """time_tile = 0: in 3D depth 3 on 32x128 tiles at radius 1 and depth 2 on
    32x128 tiles at radius 2; in 2D depth 6 at radius 1, 4 at radius 2, 3 up
    to radius 4; untiled otherwise; the result is bitwise that of the untiled
    sweep."""
    w = _small(so, shape, nbl=3, seed=31, nt=10)
    op = _op(w, time_tile=0)
    T, skew, tshape, _ = op.schedule()[:4]
    assert T == expect and skew == so // 2
    if T > 0 and len(shape) == 3:
        assert op.schedule().tile == (32, 128)
    rec_d, fin_d = _run(op, w)
    op.set_schedule(-1, 0, 0, 0)
    rec_u, fin_u = _run(op, w)
    assert np.array_equal(fin_d, fin_u) and np.array_equal(rec_d, rec_u)


@pytest.mark.parametrize("shape", [(20, 9, 47), (16, 6, 130), (30, 700)])
def test_dense_receiver_lines_on_adjacent_rows(shape):
    """Receivers on every node of two adjacent rows and sources on a third,
    in rows shorter and longer than one 64-lane window: each trace against
    the oracle and every schedule bitwise (the per-window point lookup must
    never take a point of a neighbouring row)."""
    nd = len(shape)
    so, nt = 4, 14
    rng = np.random.default_rng(41)
    h = (10.0,) * nd
    m = wi.to_slowness2(rng.uniform(1500, 3000, size=shape))
    dt = 0.35 * 10.0 / 3000.0
    n2 = shape[-1]
    if nd == 3:
        z, y = shape[0] // 2, shape[1] // 2
        rec = [[z * h[0], yy * h[1], x * h[2]] for yy in (y - 1, y) for x in range(n2)]
        src = [[z * h[0], (y + 1) * h[1], x * h[2]] for x in range(0, n2, 5)]
    else:
        z = shape[0] // 2
        rec = [[zz * h[0], x * h[1]] for zz in (z - 1, z) for x in range(n2)]
        src = [[(z + 1) * h[0], x * h[1]] for x in range(0, n2, 7)]
    src, rec = np.array(src), np.array(rec)
    wav = rng.standard_normal((nt, len(src))).astype(np.float32)
    w = wi.Workload("lines", tuple(shape), h, dt, so, nt, 0, 0.0, m, src, wav, rec)
    ref = _oracle(w)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    assert_field(fin_u[0], ref["final"][0], TOL)
    assert_traces(rec_u, ref["rec"], TOL)
    for T, shp in _schedules(2, nd):
        if not _try_schedule(op, T, shp):
            continue
        rec_t, fin_t = _run(op, w)
        assert np.array_equal(fin_t, fin_u) and np.array_equal(rec_t, rec_u), (T, shp)


@pytest.mark.parametrize("so,T,expect", [(2, 3, (64, 64)), (2, 4, (64, 64)), (2, 5, (32, 64)), (4, 2, (64, 64)),
                                         (4, 3, (32, 64)),
                                         (8, 1, (64, 64)), (8, 2, (32, 64)), (8, 3, (32, 64))])
def test_auto_tile_is_first_entry_holding_the_depth(so, T, expect):
    """An explicit depth with tile {0, 0}: the first entry of the table of
    built tiles whose depth limit at this order holds T, and the result
    bitwise that of the untiled sweep."""
    from paper_1806_08299_amd.wave import tile_table, wave_tiled_max_depth
    first = next(t for t in tile_table(3) if wave_tiled_max_depth(so, 3, tile=t) >= T)
    assert first == expect
    w = _small(so, (40, 70, 80), nbl=3, seed=33, nt=9)
    op = _op(w, time_tile=T)
    assert op.schedule().T == T and op.schedule().tile == expect
    rec_t, fin_t = _run(op, w)
    op.set_schedule(-1, 0, 0, 0)
    rec_u, fin_u = _run(op, w)
    assert np.array_equal(fin_t, fin_u) and np.array_equal(rec_t, rec_u)


@pytest.mark.parametrize("so", [2, 4])
def test_carried_b_across_segments_bitwise(so):
    """Up to radius 2 the register tiles load b once per plane and carry it
    from stage to stage, filling the carry from the planes below each axis-0
    segment before the first iteration: every built tile and depth in three
    and in seven segments, bitwise the untiled sweep (fields and traces)."""
    w = _small(so, (70, 60, 140), nbl=4, seed=90 + so, nt=14)
    op = _op(w, time_tile=-1)
    rec_u, fin_u = _run(op, w)
    for T, shp in _schedules(so // 2, 3):
        for zc in (3, 7):
            if not _try_schedule(op, T, shp, zchunks=zc):
                continue
            print("so %d T %d shape %d zchunks %d" % (so, T, shp, zc), flush=True)
            rec_t, fin_t = _run(op, w)
            assert np.array_equal(fin_t, fin_u) and np.array_equal(rec_t, rec_u), (so, T, shp, zc)

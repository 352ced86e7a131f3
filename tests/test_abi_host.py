"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library builds/loads and exports every function include/wave.h
  declares (no compute call is made here);
* host-only entry points: descriptor sizing and validation, flop/byte
  counts, and the arithmetic-intensity estimators of the evaluation chapter
  ("Arithmetic intensity under time-tiling") against the paper's printed
  tables.
"""
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wave.h")
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_ai_tables.txt")


@pytest.fixture(scope="module")
def W():
    import paper_1806_08299_amd.wave as w
    if not os.path.exists(w.LIB_PATH):
        from paper_1806_08299_amd import build
        build.build(verbose=False)
    w.lib()
    return w


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b((?:wave|diff)_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_symbols_exported(W):
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", W.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT ((?:wave|diff)_[a-z_]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(W.lib(), n)


def test_state_bytes_and_validation(W):
    d = W.make_desc((64, 64, 64), 10.0, 1e-3, 8)
    n = 64 ** 3
    assert W.wave_state_bytes(d) >= 5 * 4 * n
    for bad in (dict(space_order=7), dict(space_order=18), dict(ndim=4)):
        dd = W.make_desc((64, 64, 64), 10.0, 1e-3, 8)
        for k, v in bad.items():
            setattr(dd, k, v)
        assert W.wave_state_bytes(dd) == 0
    dd = W.make_desc((64, 64, 64), 10.0, -1.0, 8)
    assert W.wave_state_bytes(dd) == 0


def test_flop_and_byte_counts(W):
    # 3D: per axis and radius one pair add + one FMA; plus centre and update
    assert W.wave_flops_per_point(3, 8, 0) == 1 + 3 * 3 * 4 + 7
    assert W.wave_flops_per_point(2, 4, 0) == 1 + 3 * 2 * 2 + 7
    assert W.wave_bytes_per_point(-1, 0) == 16.0
    assert W.wave_bytes_per_point(1, 0) == 16.0
    assert W.wave_bytes_per_point(4, 0) == 5.0
    assert W.wave_bytes_per_point(2, 1) == 14.0
    # adjoint with imaging: the history read at every step, the gradient read
    # and written once per window: (7 + T) 4 / T for T >= 2, 28 untiled
    assert W.wave_bytes_per_point(-1, 2) == 28.0
    assert W.wave_bytes_per_point(1, 2) == 28.0
    for T in (2, 3, 4, 8):
        assert W.wave_bytes_per_point(T, 2) == pytest.approx((7 + T) * 4.0 / T, rel=1e-12)
    # explicit diffusion: centre, per axis and radius one add + one FMA, the final add;
    # one level read and one written per launch
    assert W.diff_flops_per_point(3, 8) == 2 + 3 * 3 * 4
    assert W.wave_bytes_per_point(-1, 3) == 8.0
    assert W.wave_bytes_per_point(4, 3) == 2.0
    # the two-level step: also 3/2 u^n - 1/2 u^{n-1}; reads two levels, writes one
    # (two per time tile)
    assert W.diff_flops_per_point(3, 8, "ab2") == 5 + 3 * 3 * 4
    assert W.wave_bytes_per_point(-1, 4) == 12.0
    assert W.wave_bytes_per_point(8, 4) == 2.0


def test_diff_state_bytes_and_validation(W):
    d = W.make_diff_desc((48, 40, 72), 0.1, 1e-4, 0.5, 8)
    assert W.diff_state_bytes(d) >= 2 * 4 * 48 * 40 * 72
    d2 = W.make_diff_desc((48, 40, 72), 0.1, 1e-4, 0.5, 8, scheme="ab2")
    assert W.diff_state_bytes(d2) >= 3 * 4 * 48 * 40 * 72 > W.diff_state_bytes(d)
    d2.scheme = 2
    assert W.diff_state_bytes(d2) == 0
    for bad in (dict(space_order=7), dict(ndim=1), dict(dt=-1.0)):
        dd = W.make_diff_desc((48, 40, 72), 0.1, 1e-4, 0.5, 8)
        for k, v in bad.items():
            setattr(dd, k, v)
        assert W.diff_state_bytes(dd) == 0


def _table():
    rows = []
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            p = line.split()
            rows.append((p[0], int(p[1]), [float(v) for v in p[2:]]))
    return rows


def test_naive_estimator_reproduces_unbounded_entries(W):
    """Naive estimate = t_t * AI_S; where the paper's tighter bound does not
    bite, its printed value equals the naive one (to the 3 printed digits), and
    it never exceeds it."""
    hits = 0
    for wl, so, v in _table():
        S = v[1]
        for T, printed in zip((1, 2, 4, 8, 16), v[2:]):
            naive = W.wave_ai_naive(S, T)
            assert printed <= naive * (1 + 5e-3) + 1e-9, (wl, so, T)
            if abs(printed - naive) <= 0.006 * naive:
                hits += 1
    # T=1 rows (9), AWE so4/6/8 at T=2, AWE so4 at T=4, Laplace so2/4 at T=2 and so2 at T=4
    assert hits >= 9 + 3 + 1 + 2 + 1


def test_tight_estimator_invariants(W):
    D = [512.0, 512.0, 512.0]
    delta = [4.0, 4.0, 4.0]
    tile = [32.0, 32.0, 512.0]
    S = 2.89
    for T in (1, 2, 4, 8, 16):
        naive = W.wave_ai_naive(S, T)
        # huge cache: every face fits -> no reload -> tight == naive
        assert W.wave_ai_tight(S, T, D, delta, tile, 1e12) == pytest.approx(naive, rel=1e-15)
        for omega in (1e3, 1e4, 1e5, 1e6, 1e7, 1e8):
            t = W.wave_ai_tight(S, T, D, delta, tile, omega)
            assert 0 < t <= naive
    # F_1 = 2 delta_1 D_2 D_3 t_t;  only d_1 faces exceed the cache -> variant
    T = 2
    F1 = 2 * 4 * 512 * 512 * T
    F2 = 2 * 32 * 4 * 512 * T
    omega = (F1 + F2) / 2.0
    got = W.wave_ai_tight(S, T, D, delta, tile, omega)
    frac = (F1 - omega) * np.floor(512 / 32) / 512 ** 3
    assert got == pytest.approx(S * T / (1 + frac), rel=1e-14)
    # F_2 >= omega > F_3: d_1 faces reloaded (B = B_1)
    omega = F2 / 2.0
    got = W.wave_ai_tight(S, T, D, delta, tile, omega)
    b1 = 2 * 4 / 512 * np.floor(512 / 32)
    assert got == pytest.approx(S * T / (1 + b1), rel=1e-14)
    # F_3 >= omega: B = B_1 u B_2 (proportional overlap)
    omega = 10.0
    got = W.wave_ai_tight(S, T, D, delta, tile, omega)
    b2 = 2 * 4 / 512 * np.floor(512 / 32)
    u = b1 + b2 - b1 * b2
    assert got == pytest.approx(S * T / (1 + u), rel=1e-14)


def test_tile_table_and_depth_limits(W):
    """The run-time extended tiles come from a table of built tiles; every
    entry leaves a core at its deepest depth, and extents outside the table
    have no depth."""
    assert W.tile_table(3) == [(64, 64), (32, 64), (32, 128), (16, 128)]
    assert W.tile_table(2) == [(1, 1024)]
    for so in range(2, 17, 2):
        r = so // 2
        for ey, ex in W.tile_table(3):
            T = W.wave_tiled_max_depth(so, 3, tile=(ey, ex))
            assert T >= 0
            if T:
                assert ey - 2 * r * T >= 1 and ex - 2 * r * T >= 1, (so, ey, ex, T)
        assert W.wave_tiled_max_depth(so, 3, tile=(48, 64)) == 0
        assert W.wave_tiled_max_depth(so, 3, tile=(0, 0)) == 0
    assert W.wave_tiled_max_depth(8, 3, tile=(32, 64)) == 3
    assert W.wave_tiled_max_depth(16, 3, tile=(16, 128)) == 0
    assert W.wave_tiled_max_depth(4, 2, tile=(1, 1024)) == 8
    assert W.block_extent(3, 3) == (32, 128)


def test_descriptor_tile_and_slab_validation(W):
    ok = W.make_desc((64, 64, 64), 10.0, 1e-3, 8, time_tile=2, tile=(32, 128))
    assert W.wave_state_bytes(ok) > 0
    sk = W.make_desc((64, 64, 64), 10.0, 1e-3, 8, time_tile=4, slab=48)
    assert W.wave_state_bytes(sk) > 0
    bad = W.make_desc((64, 64, 64), 10.0, 1e-3, 8, time_tile=2, tile=(32, 128))
    bad.tile[0] = 48                     # not a built tile: rejected by validation
    assert W.wave_state_bytes(bad) == 0
    neg = W.make_desc((64, 64, 64), 10.0, 1e-3, 8, time_tile=2, slab=0)
    neg.slab = -3
    assert W.wave_state_bytes(neg) == 0


def test_null_context_entry_points(W):
    """Entry points refuse a null context before any device call: the
    autotuners return WAVE_EINVAL, the sizing calls 0."""
    L = W.lib()
    assert L.wave_autotune_scratch_bytes(None, 10, 0, 0) == 0
    assert L.wave_scratch_bytes(None, 10, 0, 0, 0, 0) == 0
    assert L.wave_autotune(None, 10, 1, 0, None, 0, None) == -1
    assert L.wave_autotune_guided(None, 10, 1, 0, 4, None, 0, None, None) == -1
    assert L.wave_autotune_points(None, 10, 1, 0, 0, 0, None, 0, None, None, 0, None, None) == -1
    assert L.wave_autotune_gradient_scratch_bytes(None, 10, 0, 0, 5) == 0
    assert L.wave_autotune_gradient(None, 10, 1, 0, 5, 0, None, 0, None, None, 0, None, None) == -1
    assert L.wave_history_segment_bytes(None, 5) == 0
    assert L.wave_last_kept_segments(None) == -1

"""Python binding of the C ABI in include/wave.h (libwavett.so).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
libwavett.so.  PyTorch provides device memory (tensors whose data pointers
are handed to the library) and the stream (torch's current HIP stream).  The
functions keep the C names; ``WaveOp`` bundles a context with its buffers and
``WaveFn`` is the ``torch.autograd.Function`` that makes the modelled
receiver traces differentiable with respect to the model m and the wavelet.

If the library has not been built the first call raises: there is no CPU or
pure-PyTorch fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwavett.so")

WAVE_OK = 0
STATUS = {0: "WAVE_OK", -1: "WAVE_EINVAL", -2: "WAVE_ESKEW", -3: "WAVE_ECFL", -4: "WAVE_ENOMEM",
          -5: "WAVE_EHIP", -6: "WAVE_ESTATE", -7: "WAVE_EUNSUPPORTED"}


class WaveError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class wave_desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("space_order", ctypes.c_int32),
                ("shape", ctypes.c_int64 * 3), ("spacing", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("nbl", ctypes.c_int32), ("sigma_max", ctypes.c_double),
                ("time_tile", ctypes.c_int32), ("skew", ctypes.c_int32),
                ("tile", ctypes.c_int32 * 2), ("slab", ctypes.c_int32), ("zchunks", ctypes.c_int32)]


class Schedule(tuple):
    """(T, skew, tile_shape, zchunks, tile, slab): tile_shape is the index of
    the extended tile in the table of built tiles (0 when the schedule is
    untiled or skewed), tile its (rows, columns), slab the slab thickness of
    the skewed schedule (0: not skewed)."""
    __slots__ = ()
    _names = ("T", "skew", "tile_shape", "zchunks", "tile", "slab")

    def __new__(cls, *v):
        return tuple.__new__(cls, v)

    def __getattr__(self, k):
        try:
            return self[self._names.index(k)]
        except ValueError:
            raise AttributeError(k)

    def asdict(self):
        return dict(zip(self._names, self))


def tile_table(ndim: int):
    """Extended tiles (rows, columns) of the register-tiled sweep, index 1.."""
    out = []
    i = 1
    while True:
        ey, ex = ctypes.c_int32(), ctypes.c_int32()
        if lib().wave_tile_extent(ndim, i, ctypes.byref(ey), ctypes.byref(ex)) != WAVE_OK:
            return out
        out.append((ey.value, ex.value))
        i += 1


def _tile_of(ndim, tile_shape, tile):
    """Extents for a table index (0 = automatic) or explicit extents."""
    if tile is not None:
        return (int(tile[0]), int(tile[1]))
    if not tile_shape or ndim == 2:   # 2D has one tile: the index is ignored
        return (0, 0)
    tab = tile_table(ndim)
    if not 1 <= tile_shape <= len(tab):
        raise WaveError(-7, "no tile %d in the table of built tiles" % tile_shape)
    return tab[tile_shape - 1]


def make_desc(shape, spacing, dt, space_order, nbl=0, sigma_max=0.0, time_tile=-1, skew=0,
              tile_shape=0, zchunks=0, tile=None, slab=0) -> wave_desc:
    d = wave_desc()
    shape = tuple(int(s) for s in shape)
    d.ndim = len(shape)
    d.space_order = int(space_order)
    sp = tuple(float(h) for h in (spacing if np.ndim(spacing) else (spacing,) * len(shape)))
    for a in range(3):
        d.shape[a] = shape[a] if a < len(shape) else 1
        d.spacing[a] = sp[a] if a < len(shape) else 1.0
    d.dt = float(dt)
    d.nbl = int(nbl)
    d.sigma_max = float(sigma_max)
    d.time_tile = int(time_tile)
    d.skew = int(skew)
    d.tile[0], d.tile[1] = _tile_of(d.ndim, tile_shape, tile)
    d.slab = int(slab)
    d.zchunks = int(zchunks)
    return d


class diff_desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("space_order", ctypes.c_int32),
                ("shape", ctypes.c_int64 * 3), ("spacing", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("alpha", ctypes.c_double),
                ("time_tile", ctypes.c_int32), ("skew", ctypes.c_int32),
                ("tile", ctypes.c_int32 * 2), ("slab", ctypes.c_int32), ("zchunks", ctypes.c_int32),
                ("scheme", ctypes.c_int32)]

SCHEMES = {"euler": 0, "ab2": 1}


def make_diff_desc(shape, spacing, dt, alpha, space_order, time_tile=-1, skew=0, tile_shape=0,
                   zchunks=0, tile=None, slab=0, scheme="euler") -> diff_desc:
    d = diff_desc()
    shape = tuple(int(s) for s in shape)
    d.ndim = len(shape)
    d.space_order = int(space_order)
    sp = tuple(float(h) for h in (spacing if np.ndim(spacing) else (spacing,) * len(shape)))
    for a in range(3):
        d.shape[a] = shape[a] if a < len(shape) else 1
        d.spacing[a] = sp[a] if a < len(shape) else 1.0
    d.dt = float(dt)
    d.alpha = float(alpha)
    d.time_tile = int(time_tile)
    d.skew = int(skew)
    d.tile[0], d.tile[1] = _tile_of(d.ndim, tile_shape, tile)
    d.slab = int(slab)
    d.zchunks = int(zchunks)
    d.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    return d


_lib = None
P = ctypes.c_void_p


def lib():
    """Load libwavett.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwavett.so not built: run __graft_entry__.build() "
                              "(or python -m paper_1806_08299_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, sz, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
        sig = {
            "wave_state_bytes": (sz, [P]),
            "wave_init": (i32, [P, P, P, sz, P, ctypes.POINTER(P)]),
            "wave_set_model": (i32, [P, P]),
            "wave_set_schedule": (i32, [P, i32, i32, P, i32, i32]),
            "wave_get_schedule": (i32, [P, P, P, P, P, P]),
            "wave_scratch_bytes": (sz, [P, i32, i32, i32, i32, i32]),
            "wave_history_segment_bytes": (sz, [P, i32]),
            "wave_last_kept_segments": (i32, [P]),
            "wave_forward": (i32, [P, i32, i32, P, P, i32, P, P, P, P, i32, P, sz]),
            "wave_forward_static": (i32, [P, i32, i32, P, P, i32, P, P, P, P]),
            "wave_adjoint_grad": (i32, [P, i32, i32, P, P, i32, P, P, P, P, i32, i32, P, sz]),
            "wave_batch": (i32, [P, i32, i32, P, P, P, P, P, P, P, P, i32, P, P]),
            "wave_autotune": (i32, [P, i32, i32, i32, P, sz, P]),
            "wave_autotune_guided": (i32, [P, i32, i32, i32, i32, P, sz, P, P]),
            "wave_autotune_points": (i32, [P, i32, i32, i32, i32, i32, P, i32, P, P, sz, P, P]),
            "wave_autotune_scratch_bytes": (sz, [P, i32, i32, i32]),
            "wave_autotune_gradient": (i32, [P, i32, i32, i32, i32, i32, P, i32, P, P, sz, P, P]),
            "wave_autotune_gradient_scratch_bytes": (sz, [P, i32, i32, i32, i32]),
            "wave_tiled_max_depth": (i32, [i32, i32, i32, i32]),
            "wave_tile_extent": (i32, [i32, i32, P, P]),
            "wave_ai_naive": (dbl, [dbl, i32]),
            "wave_ai_tight": (dbl, [dbl, i32, i32, P, P, P, dbl]),
            "wave_flops_per_point": (dbl, [i32, i32, i32]),
            "wave_bytes_per_point": (dbl, [i32, i32]),
            "diff_flops_per_point": (dbl, [i32, i32, i32]),
            "diff_state_bytes": (sz, [P]),
            "diff_init": (i32, [P, P, sz, P, ctypes.POINTER(P)]),
            "diff_forward": (i32, [P, i32, P, P]),
            "wave_strerror": (ctypes.c_char_p, [i32]),
            "wave_last_error": (ctypes.c_char_p, [P]),
            "wave_destroy": (None, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, ctx=None):
    if status != WAVE_OK:
        msg = lib().wave_last_error(ctx).decode() if ctx else ""
        if not msg:
            msg = lib().wave_strerror(status).decode()
        raise WaveError(status, msg)


def _dptr(t: Optional[torch.Tensor], dtype=torch.float32):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError("expected a contiguous %s device tensor" % dtype)
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a: Optional[np.ndarray]):
    if a is None or a.size == 0:
        return None
    return a.ctypes.data_as(ctypes.c_void_p)


def _coords(x, ndim):
    if x is None:
        return np.zeros((0, ndim), dtype=np.float64)
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1, ndim))


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ C names

def wave_state_bytes(desc: wave_desc) -> int:
    return int(lib().wave_state_bytes(ctypes.byref(desc)))


def wave_init(desc: wave_desc, m: torch.Tensor, state: torch.Tensor, stream=None):
    out = ctypes.c_void_p()
    st = lib().wave_init(ctypes.byref(desc), _dptr(m), ctypes.c_void_p(state.data_ptr()),
                         state.numel() * state.element_size(), _stream(stream), ctypes.byref(out))
    _check(st)
    return out


def wave_set_model(ctx, m: torch.Tensor):
    _check(lib().wave_set_model(ctx, _dptr(m)), ctx)


def wave_set_schedule(ctx, time_tile: int, skew: int = 0, tile_shape: int = 0, zchunks: int = 0, tile=None,
                      slab: int = 0, ndim: int = 3):
    """time_tile, skew, the extended tile (a table index tile_shape, or
    extents tile=(rows, columns)), slab (> 0: the skewed schedule) and the
    number of axis-0 segments."""
    ext = (ctypes.c_int32 * 2)(*_tile_of(ndim, tile_shape, tile))
    _check(lib().wave_set_schedule(ctx, int(time_tile), int(skew), ext, int(slab), int(zchunks)), ctx)


def wave_get_schedule(ctx, ndim: int = 3) -> Schedule:
    T, sk, sl, zc = (ctypes.c_int32() for _ in range(4))
    ext = (ctypes.c_int32 * 2)()
    _check(lib().wave_get_schedule(ctx, ctypes.byref(T), ctypes.byref(sk), ext, ctypes.byref(sl),
                                   ctypes.byref(zc)), ctx)
    tile = (ext[0], ext[1])
    idx = 0
    if tile != (0, 0):
        tab = tile_table(ndim)
        idx = tab.index(tile) + 1 if tile in tab else 0
    return Schedule(T.value, sk.value, idx, zc.value, tile, sl.value)


def wave_scratch_bytes(ctx, nt: int, nsrc: int, nrec: int, ckpt_every: int = 0, adjoint: int = 0) -> int:
    return int(lib().wave_scratch_bytes(ctx, nt, nsrc, nrec, ckpt_every, adjoint))


def wave_forward(ctx, nt, src_xyz, wavelet, rec_xyz, rec_out, u_init, u_final, ckpt_every, scratch, ndim):
    src = _coords(src_xyz, ndim)
    rec = _coords(rec_xyz, ndim)
    st = lib().wave_forward(ctx, nt, src.shape[0], _hptr(src), _dptr(wavelet), rec.shape[0], _hptr(rec),
                            _dptr(rec_out), _dptr(u_init), _dptr(u_final), ckpt_every,
                            ctypes.c_void_p(scratch.data_ptr()), scratch.numel() * scratch.element_size())
    _check(st, ctx)


def wave_forward_static(ctx, nt, src_xyz, wavelet, rec_xyz, rec_out, u_init, u_final, ndim):
    """wave_forward without checkpoints or a scratch argument: the library's
    static per-GPU scratch array is used (for callers that cannot allocate)."""
    src = _coords(src_xyz, ndim)
    rec = _coords(rec_xyz, ndim)
    st = lib().wave_forward_static(ctx, nt, src.shape[0], _hptr(src), _dptr(wavelet), rec.shape[0], _hptr(rec),
                                   _dptr(rec_out), _dptr(u_init), _dptr(u_final))
    _check(st, ctx)


WAVE_STATIC_SCRATCH_BYTES = 32 << 20


def wave_history_segment_bytes(ctx, ckpt_every: int) -> int:
    return int(lib().wave_history_segment_bytes(ctx, ckpt_every))


def wave_last_kept_segments(ctx) -> int:
    return int(lib().wave_last_kept_segments(ctx))


def wave_adjoint_grad(ctx, nt, src_xyz, wavelet, rec_xyz, resid, grad_m, grad_wavelet, ckpt_every, reuse,
                      scratch, ndim):
    src = _coords(src_xyz, ndim)
    rec = _coords(rec_xyz, ndim)
    st = lib().wave_adjoint_grad(ctx, nt, src.shape[0], _hptr(src), _dptr(wavelet), rec.shape[0], _hptr(rec),
                                 _dptr(resid), _dptr(grad_m), _dptr(grad_wavelet), ckpt_every, int(reuse),
                                 ctypes.c_void_p(scratch.data_ptr()), scratch.numel() * scratch.element_size())
    _check(st, ctx)


def wave_autotune(ctx, trial_steps, repeats, max_T, scratch):
    best = ctypes.c_double()
    st = lib().wave_autotune(ctx, trial_steps, repeats, max_T, ctypes.c_void_p(scratch.data_ptr()),
                             scratch.numel() * scratch.element_size(), ctypes.byref(best))
    _check(st, ctx)
    return best.value


def wave_autotune_guided(ctx, trial_steps, repeats, max_T, keep, scratch):
    """The estimator-guided autotuner: returns (seconds per step of the
    schedule kept, number of candidates timed)."""
    best = ctypes.c_double()
    n = ctypes.c_int32()
    st = lib().wave_autotune_guided(ctx, trial_steps, repeats, max_T, keep, ctypes.c_void_p(scratch.data_ptr()),
                                    scratch.numel() * scratch.element_size(), ctypes.byref(best), ctypes.byref(n))
    _check(st, ctx)
    return best.value, n.value


def wave_autotune_scratch_bytes(ctx, trial_steps, nsrc=0, nrec=0) -> int:
    return int(lib().wave_autotune_scratch_bytes(ctx, trial_steps, nsrc, nrec))


def wave_autotune_points(ctx, trial_steps, repeats, max_T, keep, src_xyz, rec_xyz, scratch, ndim=3):
    """The autotuner whose trials carry the operator's sources and
    receivers (keep = 0: exhaustive, else estimator-guided): returns
    (seconds per step of the schedule kept, number of candidates timed)."""
    src = _coords(src_xyz, ndim)
    rec = _coords(rec_xyz, ndim)
    best = ctypes.c_double()
    n = ctypes.c_int32()
    st = lib().wave_autotune_points(ctx, trial_steps, repeats, max_T, keep, src.shape[0], _hptr(src), rec.shape[0],
                                    _hptr(rec), ctypes.c_void_p(scratch.data_ptr()),
                                    scratch.numel() * scratch.element_size(), ctypes.byref(best), ctypes.byref(n))
    _check(st, ctx)
    return best.value, n.value


def wave_autotune_gradient_scratch_bytes(ctx, trial_steps, nsrc, nrec, ckpt_every) -> int:
    return int(lib().wave_autotune_gradient_scratch_bytes(ctx, trial_steps, nsrc, nrec, ckpt_every))


def wave_autotune_gradient(ctx, trial_steps, repeats, max_T, ckpt_every, src_xyz, rec_xyz, scratch, ndim=3):
    """The autotuner for gradients: returns (seconds per step of the kept
    schedule's trial gradient, number of candidates timed)."""
    src = _coords(src_xyz, ndim)
    rec = _coords(rec_xyz, ndim)
    best = ctypes.c_double()
    n = ctypes.c_int32()
    st = lib().wave_autotune_gradient(ctx, trial_steps, repeats, max_T, ckpt_every, src.shape[0], _hptr(src),
                                      rec.shape[0], _hptr(rec), ctypes.c_void_p(scratch.data_ptr()),
                                      scratch.numel() * scratch.element_size(), ctypes.byref(best), ctypes.byref(n))
    _check(st, ctx)
    return best.value, n.value


def wave_batch(ctxs, nt, nsrc, src, wavelets, nrec, rec, rec_out, dobs, grad_m, ckpt_every, scratch):
    """Marshal per-shot lists into the C arrays of wave_batch (lists of equal
    length; host coordinate arrays float64 [n][ndim], device tensors)."""
    n = len(ctxs)
    P = ctypes.c_void_p

    def parr(items):
        return (P * n)(*[(x.value if isinstance(x, ctypes.c_void_p) else x) for x in items])

    i32a = (ctypes.c_int32 * n)(*[int(v) for v in nsrc])
    i32b = (ctypes.c_int32 * n)(*[int(v) for v in nrec])
    sp = parr([_hptr(a) for a in src])
    rp = parr([_hptr(a) for a in rec])
    wp = parr([_dptr(t) for t in wavelets])
    op = parr([_dptr(t) for t in rec_out])
    dp = parr([_dptr(t) for t in dobs]) if dobs is not None else None
    gp = parr([_dptr(t) for t in grad_m]) if grad_m is not None else None
    sc = parr([ctypes.c_void_p(t.data_ptr()) for t in scratch])
    sb = (ctypes.c_size_t * n)(*[t.numel() * t.element_size() for t in scratch])
    cp = parr(ctxs)
    st = lib().wave_batch(cp, n, nt, i32a, sp, wp, i32b, rp, op, dp, gp, ckpt_every, sc, sb)
    _check(st, ctxs[0])


class ShotBatch:
    """Independent shots (each a WaveOp: own grid, order, model, schedule)
    advanced together by wave_batch.  Outputs and scratch are kept, so that
    a repeated run with the same wavelet/observed-data tensors replays the
    captured graph."""

    def __init__(self, ops, nt, src_xyz, rec_xyz, ckpt_every=0, gradient=False):
        self.ops = list(ops)
        self.nt = int(nt)
        self.src = [_coords(s, op.ndim) for s, op in zip(src_xyz, self.ops)]
        self.rec = [_coords(r, op.ndim) for r, op in zip(rec_xyz, self.ops)]
        self.gradient = bool(gradient)
        self.K = int(ckpt_every) if gradient else 0
        if self.gradient and self.K < 1:
            raise ValueError("a gradient batch needs ckpt_every >= 1")
        dev = self.ops[0].device
        self.rec_out = [torch.empty((self.nt, r.shape[0]), dtype=torch.float32, device=dev) for r in self.rec]
        self.grad = [torch.empty(op.shape, dtype=torch.float32, device=dev) for op in self.ops] if gradient else None
        self.scratch = [
            torch.empty(max(256, wave_scratch_bytes(op.ctx, self.nt, s.shape[0], r.shape[0], self.K,
                                                    2 if gradient else 0)), dtype=torch.uint8, device=dev)
            for op, s, r in zip(self.ops, self.src, self.rec)]

    def run(self, wavelets, dobs=None):
        wav = [w.to(self.ops[0].device, torch.float32).contiguous() if w.dtype != torch.float32 or not w.is_contiguous()
               else w for w in wavelets]
        if self.gradient:
            if dobs is None:
                raise ValueError("a gradient batch needs observed traces")
        else:
            dobs = None
        wave_batch([op.ctx for op in self.ops], self.nt, [s.shape[0] for s in self.src], self.src, wav,
                   [r.shape[0] for r in self.rec], self.rec, self.rec_out, dobs, self.grad, self.K, self.scratch)
        return self.rec_out, self.grad


def wave_tiled_max_depth(space_order: int, ndim: int, tile_shape: int = 1, tile=None) -> int:
    """Deepest register-tiled depth built for the order and the extended tile
    (table index tile_shape, or extents tile)."""
    ey, ex = _tile_of(ndim, tile_shape if ndim == 3 else 1, tile)
    return int(lib().wave_tiled_max_depth(space_order, ndim, ey, ex))


def block_extent(ndim: int, tile_shape: int = 1):
    """(ey, ex) columns loaded by one workgroup of the time-tiled sweep for
    entry tile_shape of the table of built tiles."""
    ey, ex = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().wave_tile_extent(ndim, tile_shape if ndim == 3 else 1, ctypes.byref(ey), ctypes.byref(ex)), None)
    return ey.value, ex.value


def wave_ai_naive(ai_space: float, t_t: int) -> float:
    return float(lib().wave_ai_naive(ai_space, t_t))


def wave_ai_tight(ai_space, t_t, D, delta, tile, omega) -> float:
    n = len(D)
    arr = [np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (D, delta, tile)]
    return float(lib().wave_ai_tight(ai_space, t_t, n, *[_hptr(a) for a in arr], float(omega)))


def wave_flops_per_point(ndim, space_order, damped=0) -> float:
    return float(lib().wave_flops_per_point(ndim, space_order, damped))


def wave_bytes_per_point(time_tile, mode=0) -> float:
    return float(lib().wave_bytes_per_point(time_tile, mode))


def wave_destroy(ctx):
    if ctx:
        lib().wave_destroy(ctx)


def diff_flops_per_point(ndim, space_order, scheme="euler") -> float:
    return float(lib().diff_flops_per_point(ndim, space_order, SCHEMES[scheme] if isinstance(scheme, str) else scheme))


def diff_state_bytes(desc: diff_desc) -> int:
    return int(lib().diff_state_bytes(ctypes.byref(desc)))


def diff_init(desc: diff_desc, state: torch.Tensor, stream=None):
    out = ctypes.c_void_p()
    st = lib().diff_init(ctypes.byref(desc), ctypes.c_void_p(state.data_ptr()),
                         state.numel() * state.element_size(), _stream(stream), ctypes.byref(out))
    _check(st)
    return out


def diff_forward(ctx, nt: int, u0: torch.Tensor, u_out: torch.Tensor):
    _check(lib().diff_forward(ctx, int(nt), _dptr(u0), _dptr(u_out)), ctx)


# ------------------------------------------------------------------ convenience

class WaveOp:
    """A context plus the device buffers it needs (allocated as torch tensors)."""

    def __init__(self, shape, spacing, dt, space_order, m: torch.Tensor, nbl=0, sigma_max=0.0,
                 time_tile=-1, skew=0, tile_shape=0, zchunks=0, device="cuda", tile=None, slab=0):
        self.desc = make_desc(shape, spacing, dt, space_order, nbl, sigma_max, time_tile, skew,
                              tile_shape, zchunks, tile=tile, slab=slab)
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.device = torch.device(device)
        nbytes = wave_state_bytes(self.desc)
        if nbytes == 0:
            raise WaveError(-1, "invalid descriptor")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.m = m.to(self.device, torch.float32).contiguous()
        self.ctx = wave_init(self.desc, self.m, self.state)
        self._scratch = None

    def __del__(self):
        try:
            wave_destroy(self.ctx)
        except Exception:
            pass

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def scratch(self, nbytes: int) -> torch.Tensor:
        if self._scratch is None or self._scratch.numel() < nbytes:
            self._scratch = None
            self._scratch = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self._scratch

    def set_model(self, m: torch.Tensor):
        self.m = m.to(self.device, torch.float32).contiguous()
        wave_set_model(self.ctx, self.m)

    def set_schedule(self, time_tile, skew=0, tile_shape=0, zchunks=0, tile=None, slab=0):
        wave_set_schedule(self.ctx, time_tile, skew, tile_shape, zchunks, tile=tile, slab=slab, ndim=self.ndim)

    def schedule(self) -> Schedule:
        return wave_get_schedule(self.ctx, self.ndim)

    def autotune(self, trial_steps=40, repeats=2, max_T=0, src_xyz=None, rec_xyz=None, keep=0) -> float:
        """Time the schedules with trial forwards that carry these sources
        and receivers (wave_autotune_points; keep = 0 exhaustive, else the
        estimator-guided tuner) and keep the fastest; returns its seconds
        per step."""
        nsrc = 0 if src_xyz is None else len(src_xyz)
        nrec = 0 if rec_xyz is None else len(rec_xyz)
        sc = self.scratch(wave_autotune_scratch_bytes(self.ctx, trial_steps, nsrc, nrec))
        best, _ = wave_autotune_points(self.ctx, trial_steps, repeats, max_T, keep, src_xyz, rec_xyz, sc, self.ndim)
        return best

    def autotune_gradient(self, trial_steps=40, repeats=2, max_T=0, src_xyz=None, rec_xyz=None, ckpt_every=20):
        """Tune the schedule for adjoint_grad (wave_autotune_gradient): the
        forward autotuner, then trial gradients of its winner, the untiled
        sweep and a few register tiles; returns the kept schedule's trial
        seconds per step."""
        nsrc = 0 if src_xyz is None else len(src_xyz)
        nrec = 0 if rec_xyz is None else len(rec_xyz)
        sc = self.scratch(wave_autotune_gradient_scratch_bytes(self.ctx, trial_steps, nsrc, nrec, ckpt_every))
        best, _ = wave_autotune_gradient(self.ctx, trial_steps, repeats, max_T, ckpt_every, src_xyz, rec_xyz, sc,
                                         self.ndim)
        return best

    def forward(self, nt, src_xyz=None, wavelet=None, rec_xyz=None, u_init=None, want_final=False,
                ckpt_every=0, adjoint_scratch=False, keep_segments=0):
        """Forward (wave_forward).  adjoint_scratch sizes the scratch for a
        following adjoint_grad(reuse=True); keep_segments > 0 (with it) also
        keeps the history of that many last segments for that adjoint."""
        src = _coords(src_xyz, self.ndim)
        rec = _coords(rec_xyz, self.ndim)
        if wavelet is not None:
            wavelet = wavelet.to(self.device, torch.float32).contiguous()
        rec_out = torch.empty((nt, rec.shape[0]), dtype=torch.float32, device=self.device) if rec.shape[0] else None
        fin = torch.empty((2,) + self.shape, dtype=torch.float32, device=self.device) if want_final else None
        nb = wave_scratch_bytes(self.ctx, nt, src.shape[0], rec.shape[0], ckpt_every, 1 if adjoint_scratch else 0)
        if adjoint_scratch and keep_segments > 0 and ckpt_every > 0:
            nb += keep_segments * wave_history_segment_bytes(self.ctx, ckpt_every)
        sc = self.scratch(nb)
        wave_forward(self.ctx, nt, src, wavelet, rec, rec_out, u_init, fin, ckpt_every, sc, self.ndim)
        return rec_out, fin

    def adjoint_grad(self, nt, src_xyz, wavelet, rec_xyz, resid, ckpt_every, want_grad_wavelet=True, reuse=False,
                     keep_segments=0):
        """Gradient (wave_adjoint_grad).  keep_segments > 0 sizes the scratch so
        that the forward keeps the history of that many last segments, which
        the adjoint then does not recompute (scratch already larger keeps as
        many as fit); the gradient is bitwise the same."""
        src = _coords(src_xyz, self.ndim)
        rec = _coords(rec_xyz, self.ndim)
        gm = torch.empty(self.shape, dtype=torch.float32, device=self.device)
        gq = torch.empty((nt, src.shape[0]), dtype=torch.float32, device=self.device) \
            if (want_grad_wavelet and src.shape[0]) else None
        nb = wave_scratch_bytes(self.ctx, nt, src.shape[0], rec.shape[0], ckpt_every, 1)
        if keep_segments > 0 and not reuse:
            nb += keep_segments * wave_history_segment_bytes(self.ctx, ckpt_every)
        if reuse and (self._scratch is None or self._scratch.numel() < nb):
            reuse = False
        sc = self.scratch(nb)
        resid = resid.to(self.device, torch.float32).contiguous()
        if wavelet is not None:
            wavelet = wavelet.to(self.device, torch.float32).contiguous()
        try:
            wave_adjoint_grad(self.ctx, nt, src, wavelet, rec, resid, gm, gq, ckpt_every, 1 if reuse else 0,
                              sc, self.ndim)
        except WaveError as e:
            if not (reuse and e.status == -6):
                raise
            wave_adjoint_grad(self.ctx, nt, src, wavelet, rec, resid, gm, gq, ckpt_every, 0, sc, self.ndim)
        return gm, gq


class WaveFn(torch.autograd.Function):
    """rec = WaveFn.apply(m, wavelet, op, src_xyz, rec_xyz, ckpt_every, keep_segments).

    Forward models the receiver traces [nt, nrec] for squared slowness m and
    source wavelet [nt, nsrc]; backward returns (dL/dm, dL/dwavelet) from the
    time-reversed adjoint sweep with the imaging condition, recomputing the
    forward in checkpointed segments of ckpt_every steps, except the last
    keep_segments ones, whose history the forward keeps in the op's scratch
    (the same gradient, bitwise)."""

    @staticmethod
    def forward(ctx, m, wavelet, op: WaveOp, src_xyz, rec_xyz, ckpt_every: int = 50, keep_segments: int = 0):
        op.set_model(m.detach())
        nt = wavelet.shape[0]
        rec, _ = op.forward(nt, src_xyz, wavelet.detach(), rec_xyz, ckpt_every=ckpt_every, adjoint_scratch=True,
                            keep_segments=keep_segments)
        # The checkpoints left in the op's scratch belong to this forward only
        # while no other forward has run on the op since.
        token = object()
        op._fwd_token = token
        ctx.token = token
        ctx.op = op
        ctx.src_xyz = src_xyz
        ctx.rec_xyz = rec_xyz
        ctx.ckpt_every = ckpt_every
        ctx.keep_segments = keep_segments
        ctx.save_for_backward(m.detach(), wavelet.detach())
        return rec

    @staticmethod
    def backward(ctx, grad_rec):
        m, wavelet = ctx.saved_tensors
        op = ctx.op
        nt = wavelet.shape[0]
        reuse = getattr(op, "_fwd_token", None) is ctx.token
        if not reuse:                      # another forward ran on the op: its model and checkpoints are not ours
            op.set_model(m)
        gm, gq = op.adjoint_grad(nt, ctx.src_xyz, wavelet, ctx.rec_xyz, grad_rec.contiguous(), ctx.ckpt_every,
                                 want_grad_wavelet=ctx.needs_input_grad[1], reuse=reuse,
                                 keep_segments=ctx.keep_segments)
        op._fwd_token = None               # adjoint_grad overwrote the scratch
        return gm, gq, None, None, None, None, None


class DiffOp:
    """Explicit diffusion u <- u + dt a (L u) (the Laplace-operator workload)
    on the sweep engine, or with scheme="ab2" its two-level Adams-Bashforth
    form: a diffusion context plus its state."""

    def __init__(self, shape, spacing, dt, alpha, space_order, time_tile=-1, skew=0, tile_shape=0, zchunks=0,
                 device="cuda", tile=None, slab=0, scheme="euler"):
        self.desc = make_diff_desc(shape, spacing, dt, alpha, space_order, time_tile, skew, tile_shape, zchunks,
                                   tile=tile, slab=slab, scheme=scheme)
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.device = torch.device(device)
        nbytes = diff_state_bytes(self.desc)
        if nbytes == 0:
            raise WaveError(-1, "invalid descriptor")
        self.state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ctx = diff_init(self.desc, self.state)

    def __del__(self):
        try:
            wave_destroy(self.ctx)
        except Exception:
            pass

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def set_schedule(self, time_tile, skew=0, tile_shape=0, zchunks=0, tile=None, slab=0):
        wave_set_schedule(self.ctx, time_tile, skew, tile_shape, zchunks, tile=tile, slab=slab, ndim=self.ndim)

    def schedule(self) -> Schedule:
        return wave_get_schedule(self.ctx, self.ndim)

    def autotune(self, trial_steps: int = 8, repeats: int = 2, max_T: int = 0) -> float:
        """Time the schedules (wave_autotune) and keep the fastest; returns
        its seconds per step."""
        sc = torch.empty(max(256, wave_scratch_bytes(self.ctx, trial_steps, 0, 0)), dtype=torch.uint8,
                         device=self.device)
        return wave_autotune(self.ctx, trial_steps, repeats, max_T, sc)

    def forward(self, nt: int, u0: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        u0 = u0.to(self.device, torch.float32).contiguous()
        if tuple(u0.shape) != self.shape:
            raise ValueError("u0 must have the grid's shape")
        if out is None:
            out = torch.empty_like(u0)
        diff_forward(self.ctx, nt, u0, out)
        return out

"""FP64 CPU oracle for the time-stepped acoustic-wave sweep and for explicit
diffusion (the paper's Laplace-operator workload).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does, and this
package never imports the product library.

The arithmetic lives in ``oracle.c`` (plain loops, double precision, no
tiling); this module compiles it with gcc and marshals numpy arrays through
ctypes.  ``dense.py`` holds an independent brute-force formulation (the whole
space-time system as one sparse linear solve) used to pin the loop oracle on
tiny grids.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("so", ctypes.c_int),
                ("n", ctypes.c_long * 3), ("h", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("nbl", ctypes.c_int),
                ("sigma_max", ctypes.c_double), ("periodic", ctypes.c_int)]


@dataclass
class Grid:
    """Problem geometry: shape (axis 0 slowest, last axis unit stride)."""
    shape: tuple
    spacing: tuple
    dt: float
    so: int
    nbl: int = 0
    sigma_max: float = 0.0
    periodic: bool = False
    ndim: int = field(init=False)

    def __post_init__(self):
        self.shape = tuple(int(s) for s in self.shape)
        self.ndim = len(self.shape)
        sp = tuple(float(h) for h in self.spacing)
        if len(sp) == 1:
            sp = sp * self.ndim
        self.spacing = sp

    @property
    def npts(self) -> int:
        return int(np.prod(self.shape))

    def c(self) -> _Grid:
        g = _Grid()
        g.ndim = self.ndim
        g.so = self.so
        for a in range(3):
            g.n[a] = self.shape[a] if a < self.ndim else 1
            g.h[a] = self.spacing[a] if a < self.ndim else 1.0
        g.dt = self.dt
        g.nbl = self.nbl
        g.sigma_max = self.sigma_max
        g.periodic = 1 if self.periodic else 0
        return g


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.og_fd_coeffs.argtypes = [ctypes.c_int, P]
        L.og_laplacian.argtypes = [P, P, P]
        L.og_sigma.argtypes = [P, P]
        L.og_interp_corners.argtypes = [P, P, P, P]
        L.og_forward.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int, P, P, P, P, P]
        L.og_adjoint.argtypes = [P, P, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P,
                                 P, P, P, P, ctypes.c_int, P]
        L.og_diffuse.argtypes = [P, ctypes.c_double, ctypes.c_int, P, P]
        L.og_diffuse_ab2.argtypes = [P, ctypes.c_double, ctypes.c_int, P, P]
        for f in (L.og_fd_coeffs, L.og_laplacian, L.og_sigma, L.og_interp_corners,
                  L.og_forward, L.og_adjoint, L.og_diffuse, L.og_diffuse_ab2):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def fd_coeffs(so: int) -> np.ndarray:
    """c_0..c_k of the order-`so` central second derivative (unit spacing)."""
    c = np.zeros(9)
    if lib().og_fd_coeffs(so, _p(c)) != 0:
        raise ValueError("space order must be even in 2..16")
    return c[: so // 2 + 1].copy()


def laplacian(g: Grid, u) -> np.ndarray:
    u = _f64(u, g.shape)
    out = np.empty_like(u)
    gc = g.c()
    if lib().og_laplacian(ctypes.byref(gc), _p(u), _p(out)) != 0:
        raise ValueError("bad grid")
    return out


def sigma(g: Grid) -> np.ndarray:
    out = np.empty(g.shape)
    gc = g.c()
    lib().og_sigma(ctypes.byref(gc), _p(out))
    return out


def interp_corners(g: Grid, x):
    x = _f64(x)
    lin = np.zeros(8, dtype=np.int64)
    w = np.zeros(8)
    gc = g.c()
    n = lib().og_interp_corners(ctypes.byref(gc), _p(x), _p(lin), _p(w))
    return lin[:n].copy(), w[:n].copy()


def forward(g: Grid, m, nt: int, src_xyz=None, wavelet=None, rec_xyz=None,
            u_init=None, want_final: bool = False, want_hist: bool = False):
    """Run nt forward steps. Returns dict with 'rec' [nt, nrec], optionally
    'final' [2, *shape] = (u^nt, u^{nt-1}) and 'hist' [nt+2, *shape] = u^{-1}..u^nt."""
    m = _f64(m, g.shape)
    src = _f64(src_xyz if src_xyz is not None else np.zeros((0, g.ndim)))
    src = src.reshape(-1, g.ndim)
    nsrc = src.shape[0]
    wav = _f64(wavelet if wavelet is not None else np.zeros((nt, nsrc)))
    wav = wav.reshape(nt, nsrc)
    rec_xyz = _f64(rec_xyz if rec_xyz is not None else np.zeros((0, g.ndim))).reshape(-1, g.ndim)
    nrec = rec_xyz.shape[0]
    rec = np.zeros((nt, nrec))
    ui = _f64(u_init, (2,) + g.shape) if u_init is not None else None
    fin = np.zeros((2,) + g.shape) if want_final else None
    hist = np.zeros((nt + 2,) + g.shape) if want_hist else None
    gc = g.c()
    rc = lib().og_forward(ctypes.byref(gc), _p(m), nt, nsrc, _p(src), _p(wav), nrec, _p(rec_xyz),
                          _p(rec), _p(ui), _p(fin), _p(hist))
    if rc != 0:
        raise RuntimeError("og_forward failed")
    out = {"rec": rec}
    if want_final:
        out["final"] = fin
    if want_hist:
        out["hist"] = hist
    return out


def adjoint(g: Grid, m, nt: int, resid, hist=None, src_xyz=None, rec_xyz=None,
            form: int = 1, want_grad_m: bool = True, want_grad_q: bool = False,
            want_final: bool = False):
    """Adjoint sweep driven by receiver residuals [nt, nrec]. Returns dict with
    'grad_m' (needs the forward history), 'grad_q' [nt, nsrc], 'final' (mu^0, mu^1)."""
    m = _f64(m, g.shape)
    src = _f64(src_xyz if src_xyz is not None else np.zeros((0, g.ndim))).reshape(-1, g.ndim)
    rec_xyz = _f64(rec_xyz if rec_xyz is not None else np.zeros((0, g.ndim))).reshape(-1, g.ndim)
    nsrc, nrec = src.shape[0], rec_xyz.shape[0]
    resid = _f64(resid).reshape(nt, nrec)
    h = _f64(hist, (nt + 2,) + g.shape) if hist is not None else None
    gm = np.zeros(g.shape) if want_grad_m else None
    gq = np.zeros((nt, nsrc)) if want_grad_q else None
    fin = np.zeros((2,) + g.shape) if want_final else None
    gc = g.c()
    rc = lib().og_adjoint(ctypes.byref(gc), _p(m), nt, nsrc, _p(src), nrec, _p(rec_xyz),
                          _p(resid), _p(h), _p(gm), _p(gq), form, _p(fin))
    if rc != 0:
        raise RuntimeError("og_adjoint failed")
    out = {}
    if want_grad_m:
        out["grad_m"] = gm
    if want_grad_q:
        out["grad_q"] = gq
    if want_final:
        out["final"] = fin
    return out


def diffuse(g: Grid, a: float, nt: int, u0) -> np.ndarray:
    """The Laplace-operator family (evaluation chapter), read as explicit
    diffusion: nt steps of u <- u + dt a (L u) from u0 (g.dt is the step)."""
    u0 = _f64(u0, g.shape)
    out = np.empty_like(u0)
    gc = g.c()
    if lib().og_diffuse(ctypes.byref(gc), float(a), int(nt), _p(u0), _p(out)) != 0:
        raise ValueError("og_diffuse failed")
    return out


def diffuse_ab2(g: Grid, a: float, nt: int, u0) -> np.ndarray:
    """The same operator with a two-level time dependence: nt steps of the
    two-step Adams-Bashforth rule u <- u + dt a (3/2 L u^n - 1/2 L u^{n-1})
    from u0, with u^{-1} = u^0 (g.dt is the step)."""
    u0 = _f64(u0, g.shape)
    out = np.empty_like(u0)
    gc = g.c()
    if lib().og_diffuse_ab2(ctypes.byref(gc), float(a), int(nt), _p(u0), _p(out)) != 0:
        raise ValueError("og_diffuse_ab2 failed")
    return out

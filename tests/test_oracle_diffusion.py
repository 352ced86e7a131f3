"""Pins for the FP64 diffusion oracle (the paper's Laplace-operator family,
evaluation chapter, read as explicit diffusion u <- u + dt a (L u)).

Each pin comes from outside the oracle's loop:

* Fourier mode on a periodic grid: the exact discrete growth factor
  (1 + dt a lambda)^n with lambda the stencil's symbol, built from the
  textbook weights in tests/golden;
* brute force by a different method: the spectral solution V (1 + dt a
  Lambda)^n V^T u0 of the dense Laplacian of oracle/dense.py (Kronecker
  sums), on tiny Dirichlet grids;
* the von Neumann stability limit dt a sum_a rho/h_a^2 <= 2;
* the discrete maximum principle at space order 2 when the centre weight
  1 - 2 dt a sum_a h_a^-2 is non-negative;
* conservation of the total under periodic wrap (the weights sum to zero).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import dense

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden_coeffs():
    out = {}
    with open(os.path.join(GOLD, "fd_coeffs_textbook.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            out[int(parts[0])] = [float(Fraction(p)) for p in parts[1:]]
    return out


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _rho(c):
    """-(symbol at the Nyquist wavenumber) of the 1D weights c_0..c_k."""
    return -(c[0] + 2 * sum(c[j] * (-1) ** j for j in range(1, len(c))))


@pytest.mark.parametrize("so", [2, 4, 8])
def test_diffusion_fourier_mode(oracle_lib, so):
    """u0 = cos(k.x) on a periodic grid stays a pure mode scaled by
    (1 + dt a lambda)^n.  A low mode with a moderate total decay (~0.3), so
    that FP64 roundoff left in the slower modes stays far below it."""
    gold = _golden_coeffs()[so]
    shape = (16, 12, 20)
    h = (0.1, 0.12, 0.08)
    a = 0.5
    kk = [2 * math.pi * 1 / (shape[0] * h[0]), 2 * math.pi * 1 / (shape[1] * h[1]),
          2 * math.pi * 2 / (shape[2] * h[2])]
    lam = sum((gold[0] + 2 * sum(gold[j] * math.cos(j * kk[ax] * h[ax]) for j in range(1, len(gold))))
              / h[ax] ** 2 for ax in range(3))
    nt = 60
    dt = 0.02 / (a * abs(lam))
    assert dt < 2.0 / (a * _rho(gold) * sum(1 / x ** 2 for x in h))   # inside the stability limit
    x = [np.arange(n) * h[ax] for ax, n in enumerate(shape)]
    X = np.meshgrid(*x, indexing="ij")
    mode = np.cos(kk[0] * X[0] + kk[1] * X[1] + kk[2] * X[2])
    g = oracle.Grid(shape, h, dt, so, periodic=True)
    got = oracle.diffuse(g, a, nt, mode)
    expect = (1.0 + dt * a * lam) ** nt * mode
    assert 0.2 < (1.0 + dt * a * lam) ** nt < 0.4
    assert rel(got, expect) < 1e-12


@pytest.mark.parametrize("shape,so,h", [((6, 5, 7), 4, (1.0, 1.3, 0.8)), ((9, 8), 8, (0.5, 0.7)),
                                        ((5, 6, 4), 2, (1.0, 1.0, 1.0))])
def test_diffusion_matches_spectral_solution(oracle_lib, shape, so, h):
    rng = np.random.default_rng(12)
    a = 0.3
    L = dense.laplacian_matrix(shape, h, so).toarray()
    lam, V = np.linalg.eigh(L)                       # L is symmetric with zero ghosts
    dt = 0.9 * 2.0 / (a * np.abs(lam).max())
    u0 = rng.standard_normal(shape)
    nt = 25
    expect = V @ ((1.0 + dt * a * lam) ** nt * (V.T @ u0.ravel()))
    g = oracle.Grid(shape, h, dt, so)
    got = oracle.diffuse(g, a, nt, u0)
    assert rel(got, expect.reshape(shape)) < 1e-12


@pytest.mark.parametrize("so", [4, 8])
def test_diffusion_stability_limit(oracle_lib, so):
    gold = _golden_coeffs()[so]
    shape = (12, 12, 12)
    h = 0.1
    a = 1.0
    dt_lim = 2.0 / (a * 3 * _rho(gold) / h ** 2)
    u0 = np.random.default_rng(3).standard_normal(shape)
    growth = {}
    for f in (0.98, 1.02):
        g = oracle.Grid(shape, (h,), f * dt_lim, so, periodic=True)
        growth[f] = np.abs(oracle.diffuse(g, a, 900, u0)).max() / np.abs(u0).max()
    assert growth[0.98] <= 1.0
    assert growth[1.02] > 1e3


def test_diffusion_maximum_principle(oracle_lib):
    shape = (14, 11, 13)
    h = (0.1, 0.09, 0.11)
    a = 0.7
    dt = 1.0 / (2 * a * sum(1 / x ** 2 for x in h))  # centre weight exactly 0
    rng = np.random.default_rng(4)
    u0 = rng.uniform(-1.0, 2.0, size=shape)
    g = oracle.Grid(shape, h, dt, 2)
    lo, hi = min(u0.min(), 0.0), max(u0.max(), 0.0)
    u = u0
    for _ in range(5):
        u = oracle.diffuse(g, a, 7, u)
        assert u.min() >= lo - 1e-12 and u.max() <= hi + 1e-12
        lo, hi = min(u.min(), 0.0), max(u.max(), 0.0)
    assert np.abs(u).max() < np.abs(u0).max()


def test_diffusion_conserves_total_periodic(oracle_lib):
    shape = (10, 13, 9)
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal(shape) + 3.0
    gold = _golden_coeffs()[8]
    h = (0.2, 0.25, 0.15)
    a = 0.4
    dt = 0.8 * 2.0 / (a * _rho(gold) * sum(1 / x ** 2 for x in h))
    g = oracle.Grid(shape, h, dt, 8, periodic=True)
    u = oracle.diffuse(g, a, 40, u0)
    assert abs(u.sum() - u0.sum()) <= 1e-12 * np.abs(u0).sum()
    assert np.abs(u - u.mean()).max() < np.abs(u0 - u0.mean()).max()   # smoothing

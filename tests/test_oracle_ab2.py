"""Pins for the FP64 oracle of the two-level (delta_t = 2) Laplace-operator
stencil: the two-step Adams-Bashforth rule for u' = a L u (evaluation
chapter, "Time-tiling with larger time dependences"),
    u^{n+1} = u^n + dt a (3/2 L u^n - 1/2 L u^{n-1}),   u^{-1} = u^0.

Each pin comes from outside the oracle's loop:

* a Fourier mode on a periodic grid against the closed form of the scalar
  recurrence a_{n+1} = (1 + 3c/2) a_n - (c/2) a_{n-1}, a_{-1} = a_0 = 1,
  c = dt a lambda, through the roots of its characteristic polynomial, with
  lambda from the textbook weights in tests/golden;
* the same closed form per eigenvalue of the dense Laplacian of
  oracle/dense.py (Kronecker sums) on tiny Dirichlet grids;
* second order in time: against the exact solution exp(a lambda t) of the
  semi-discrete mode, the error falls fourfold per halving of dt;
* the stability limit of the scheme, dt a sum_a rho/h_a^2 <= 1 (half the
  forward-Euler limit);
* conservation of the total under periodic wrap;
* the first step is the forward-Euler step of the one-level oracle.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import dense
from test_oracle_diffusion import _golden_coeffs, _rho, rel


def ab2_closed_form(c, n):
    """a_n of a_{k+1} = (1 + 1.5 c) a_k - 0.5 c a_{k-1}, a_{-1} = a_0 = 1,
    for an array of c (real roots for c in [-1, 0])."""
    c = np.asarray(c, dtype=np.float64)
    tr = 1.0 + 1.5 * c
    disc = np.sqrt(tr * tr - 2.0 * c)
    r1, r2 = (tr + disc) / 2.0, (tr - disc) / 2.0
    # alpha + beta = 1 (a_0), alpha / r1 + beta / r2 = 1 (a_{-1})
    with np.errstate(divide="ignore", invalid="ignore"):
        beta = np.where(np.abs(r2) > 0, (1.0 - 1.0 / r1) / (1.0 / r2 - 1.0 / r1), 0.0)
    alpha = 1.0 - beta
    return alpha * r1 ** n + beta * r2 ** n


def _symbol(gold, k, h):
    return (gold[0] + 2 * sum(gold[j] * math.cos(j * k * h) for j in range(1, len(gold)))) / h ** 2


@pytest.mark.parametrize("so", [2, 4, 8])
def test_ab2_fourier_mode(oracle_lib, so):
    gold = _golden_coeffs()[so]
    shape = (16, 12, 20)
    h = (0.1, 0.12, 0.08)
    a = 0.5
    kk = [2 * math.pi / (shape[0] * h[0]), 2 * math.pi / (shape[1] * h[1]), 2 * math.pi * 2 / (shape[2] * h[2])]
    lam = sum(_symbol(gold, kk[ax], h[ax]) for ax in range(3))
    nt = 60
    dt = 0.02 / (a * abs(lam))
    x = [np.arange(n) * h[ax] for ax, n in enumerate(shape)]
    X = np.meshgrid(*x, indexing="ij")
    mode = np.cos(kk[0] * X[0] + kk[1] * X[1] + kk[2] * X[2])
    g = oracle.Grid(shape, h, dt, so, periodic=True)
    got = oracle.diffuse_ab2(g, a, nt, mode)
    amp = ab2_closed_form(dt * a * lam, nt)
    assert 0.2 < amp < 0.4
    assert rel(got, amp * mode) < 1e-12
    # a strongly damped high mode (c = -0.8): the parasitic root matters
    kh = [math.pi * (shape[ax] // 2 - 1) / (shape[ax] // 2) / h[ax] for ax in range(3)]
    lam_h = sum(_symbol(gold, kh[ax], h[ax]) for ax in range(3))
    dt_h = 0.8 / (a * abs(lam_h))
    mode_h = np.cos(kh[0] * X[0] + kh[1] * X[1] + kh[2] * X[2])
    g = oracle.Grid(shape, h, dt_h, so, periodic=True)
    got = oracle.diffuse_ab2(g, a, 9, mode_h)
    assert rel(got, ab2_closed_form(dt_h * a * lam_h, 9) * mode_h) < 1e-11


@pytest.mark.parametrize("shape,so,h", [((6, 5, 7), 4, (1.0, 1.3, 0.8)), ((9, 8), 8, (0.5, 0.7)),
                                        ((5, 6, 4), 2, (1.0, 1.0, 1.0))])
def test_ab2_matches_spectral_solution(oracle_lib, shape, so, h):
    rng = np.random.default_rng(21)
    a = 0.3
    L = dense.laplacian_matrix(shape, h, so).toarray()
    lam, V = np.linalg.eigh(L)
    dt = 0.9 / (a * np.abs(lam).max())
    u0 = rng.standard_normal(shape)
    nt = 25
    expect = V @ (ab2_closed_form(dt * a * lam, nt) * (V.T @ u0.ravel()))
    g = oracle.Grid(shape, h, dt, so)
    got = oracle.diffuse_ab2(g, a, nt, u0)
    assert rel(got, expect.reshape(shape)) < 1e-11


def test_ab2_second_order_in_time(oracle_lib):
    gold = _golden_coeffs()[4]
    shape = (8, 8, 16)
    h = (0.1, 0.1, 0.1)
    a = 1.0
    k = 2 * math.pi / (shape[2] * h[2])
    lam = _symbol(gold, k, h[2])
    X = np.arange(shape[2]) * h[2]
    mode = np.broadcast_to(np.cos(k * X), shape).copy()
    t_end = 0.5 / (a * abs(lam))               # exp(-0.5) decay
    errs = []
    for nt in (10, 20, 40, 80):
        g = oracle.Grid(shape, h, t_end / nt, 4, periodic=True)
        got = oracle.diffuse_ab2(g, a, nt, mode)
        errs.append(np.abs(got - math.exp(a * lam * t_end) * mode).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in ratios), ratios


@pytest.mark.parametrize("so", [4, 8])
def test_ab2_stability_limit(oracle_lib, so):
    gold = _golden_coeffs()[so]
    shape = (12, 12, 12)
    h = 0.1
    a = 1.0
    dt_lim = 1.0 / (a * 3 * _rho(gold) / h ** 2)
    u0 = np.random.default_rng(3).standard_normal(shape)
    growth = {}
    for f in (0.98, 1.02):
        g = oracle.Grid(shape, (h,), f * dt_lim, so, periodic=True)
        growth[f] = np.abs(oracle.diffuse_ab2(g, a, 1500, u0)).max() / np.abs(u0).max()
    assert growth[0.98] <= 1.0
    assert growth[1.02] > 1e3


def test_ab2_conserves_total_periodic_and_starts_with_euler(oracle_lib):
    shape = (10, 13, 9)
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal(shape) + 3.0
    gold = _golden_coeffs()[8]
    h = (0.2, 0.25, 0.15)
    a = 0.4
    dt = 0.8 / (a * _rho(gold) * sum(1 / x ** 2 for x in h))
    g = oracle.Grid(shape, h, dt, 8, periodic=True)
    u = oracle.diffuse_ab2(g, a, 40, u0)
    assert abs(u.sum() - u0.sum()) <= 1e-12 * np.abs(u0).sum()
    assert np.abs(u - u.mean()).max() < np.abs(u0 - u0.mean()).max()
    one = oracle.diffuse_ab2(g, a, 1, u0)
    euler = oracle.diffuse(g, a, 1, u0)
    assert rel(one, euler) < 1e-15
    assert np.array_equal(oracle.diffuse_ab2(g, a, 0, u0), u0)

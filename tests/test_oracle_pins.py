"""Pins for the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against mathematics (closed forms, invariants,
exact rational weights, brute force by a different method) so that a dropped
term, a wrong sign or index, or a transposed operand in oracle.c fails at
least one of them:

* weights: textbook values and polynomial-exactness moments;
* Laplacian: exactness on polynomials, symmetry (zero ghosts);
* time stepping: exact discrete Fourier-mode recurrence (periodic), the von
  Neumann stability limit, discrete energy conservation / decay;
* whole forward: space-time sparse solve on tiny grids (oracle/dense.py);
* sources/receivers: interpolation reproduces affine functions, linearity,
  exact time-shift, reciprocity;
* adjoint: dot-product test and the transposed space-time system;
* gradient: two summation forms agree and central finite differences;
* checkpoint/resume: bitwise.
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


# --------------------------------------------------------------------------- weights

def test_coeffs_textbook(oracle_lib):
    for so, ref in _golden_coeffs().items():
        got = oracle.fd_coeffs(so)
        np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
def test_coeffs_moments(oracle_lib, so):
    """sum_{j=-k..k} c_|j| j^{2q} = 0 (q=0), 2 (q=1), 0 (2<=q<=k), != 0 at q=k+1."""
    c = oracle.fd_coeffs(so)
    k = so // 2
    for q in range(k + 2):
        mom = (c[0] if q == 0 else 0.0) + sum(2.0 * c[j] * float(j) ** (2 * q) for j in range(1, k + 1))
        if q <= k:
            expect = 2.0 if q == 1 else 0.0
            assert abs(mom - expect) < 1e-10 * max(1.0, float(k) ** (2 * q)), (so, q, mom)
        else:
            assert abs(mom) > 1e-3
    exact = [float(v) for v in dense.moment_coeffs(so)]
    np.testing.assert_allclose(c, exact, rtol=1e-13, atol=1e-16)


# --------------------------------------------------------------------------- Laplacian

@pytest.mark.parametrize("so", [2, 4, 8, 12, 16])
def test_laplacian_exact_on_polynomials(oracle_lib, so):
    """On interior points the order-2k stencil differentiates polynomials of
    degree <= 2k+1 exactly; compare with the analytic Laplacian."""
    k = so // 2
    shape = (2 * k + 5, 2 * k + 4, 2 * k + 6)
    h = (0.7, 1.3, 0.9)
    g = oracle.Grid(shape, h, 1e-3, so)
    rng = np.random.default_rng(so)
    deg = 2 * k + 1
    coef = rng.uniform(-1, 1, size=(3, deg + 1))
    x = [np.arange(n) * h[a] - 0.5 * n * h[a] for a, n in enumerate(shape)]
    X = np.meshgrid(*x, indexing="ij")
    # separable sum  sum_a p_a(x_a)  plus a mixed product x0*x1*x2 (Laplacian 0)
    u = sum(np.polyval(coef[a], X[a]) for a in range(3)) + X[0] * X[1] * X[2]
    lap = sum(np.polyval(np.polyder(coef[a], 2), X[a]) for a in range(3))
    got = oracle.laplacian(g, u)
    sl = tuple(slice(k, n - k) for n in shape)
    scale = np.abs(u).max() / min(h) ** 2
    np.testing.assert_allclose(got[sl], lap[sl], atol=1e-9 * scale, rtol=0)


@pytest.mark.parametrize("so,shape", [(4, (5, 4, 6)), (8, (6, 7)), (16, (9, 3, 4))])
def test_laplacian_symmetric_and_matches_kron(oracle_lib, so, shape):
    g = oracle.Grid(shape, (1.0, 2.0, 0.5)[: len(shape)], 1e-3, so)
    N = g.npts
    M = np.zeros((N, N))
    for q in range(N):
        e = np.zeros(N)
        e[q] = 1.0
        M[:, q] = oracle.laplacian(g, e.reshape(shape)).ravel()
    assert np.array_equal(M, M.T)
    K = dense.laplacian_matrix(shape, g.spacing, so).toarray()
    np.testing.assert_allclose(M, K, rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------------------- time stepping

@pytest.mark.parametrize("so", [4, 8])
def test_fourier_mode_recurrence(oracle_lib, so):
    """Periodic grid, constant m, u^0 = u^-1 = cos(k.x): the exact discrete
    solution is cos((n+1/2) theta)/cos(theta/2) cos(k.x) with
    cos theta = 1 - dt^2 lambda/(2 m), lambda the stencil's symbol."""
    gold = _golden_coeffs()[so]
    shape = (16, 12, 20)
    h = (10.0, 12.0, 8.0)
    c = 2000.0
    m = 1.0 / c ** 2
    dt = 0.3 * min(h) / c
    kk = [2 * math.pi * 3 / (shape[0] * h[0]), 2 * math.pi * 2 / (shape[1] * h[1]), 2 * math.pi * 5 / (shape[2] * h[2])]
    lam = 0.0
    for a in range(3):
        s = gold[0] + 2 * sum(gold[j] * math.cos(j * kk[a] * h[a]) for j in range(1, len(gold)))
        lam -= s / h[a] ** 2
    theta = math.acos(1 - dt * dt * lam / (2 * m))
    x = [np.arange(n) * h[a] for a, n in enumerate(shape)]
    X = np.meshgrid(*x, indexing="ij")
    mode = np.cos(kk[0] * X[0] + kk[1] * X[1] + kk[2] * X[2])
    nt = 200
    g = oracle.Grid(shape, h, dt, so, periodic=True)
    out = oracle.forward(g, np.full(shape, m), nt, u_init=np.stack([mode, mode]), want_final=True)
    for lev, n in ((0, nt), (1, nt - 1)):
        expect = math.cos((n + 0.5) * theta) / math.cos(theta / 2) * mode
        assert rel(out["final"][lev], expect) < 1e-11


@pytest.mark.parametrize("so", [4, 8])
def test_stability_limit(oracle_lib, so):
    """Von Neumann: stable iff c dt sqrt(sum_a rho/h_a^2) <= 2 with
    rho = -(c_0 + 2 sum_j (-1)^j c_j) (the symbol at the Nyquist wavenumber)."""
    gold = _golden_coeffs()[so]
    rho = -(gold[0] + 2 * sum(gold[j] * (-1) ** j for j in range(1, len(gold))))
    shape = (12, 12, 12)
    h = 10.0
    c = 3000.0
    dt_lim = 2.0 / (c * math.sqrt(3 * rho / h ** 2))
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(shape)
    growth = {}
    for f in (0.98, 1.02):
        g = oracle.Grid(shape, (h,), f * dt_lim, so, periodic=True)
        out = oracle.forward(g, np.full(shape, 1 / c ** 2), 600, u_init=np.stack([u0, u0]), want_final=True)
        growth[f] = np.abs(out["final"][0]).max() / np.abs(u0).max()
    assert growth[0.98] < 50.0
    assert growth[1.02] > 1e6


def _energy(g, m, hist):
    """E^{n+1/2} = <m (u^{n+1}-u^n), (u^{n+1}-u^n)>/dt^2 - <u^{n+1}, L u^n>."""
    E = []
    for n in range(1, hist.shape[0] - 1):
        un, up = hist[n], hist[n + 1]
        d = up - un
        E.append(np.sum(m * d * d) / g.dt ** 2 - np.sum(up * oracle.laplacian(g, un)))
    return np.array(E)


def test_energy_conserved_without_damping(oracle_lib):
    shape = (14, 11, 13)
    rng = np.random.default_rng(7)
    c = rng.uniform(1500, 4000, size=shape)
    m = 1.0 / c ** 2
    g = oracle.Grid(shape, (10.0, 9.0, 11.0), 0.35 * 9.0 / 4000, 8)
    u0 = rng.standard_normal(shape)
    um = u0 + 0.01 * rng.standard_normal(shape)
    out = oracle.forward(g, m, 80, u_init=np.stack([u0, um]), want_hist=True)
    E = _energy(g, m, out["hist"])
    assert E.min() > 0
    assert np.abs(E - E[0]).max() / E[0] < 1e-11


def test_energy_decays_with_damping(oracle_lib):
    shape = (16, 16, 16)
    rng = np.random.default_rng(8)
    c = np.full(shape, 2000.0)
    m = 1.0 / c ** 2
    g = oracle.Grid(shape, (10.0,), 0.4 * 10 / 2000, 4, nbl=5, sigma_max=60.0)
    u0 = rng.standard_normal(shape)
    out = oracle.forward(g, m, 60, u_init=np.stack([u0, u0]), want_hist=True)
    E = _energy(g, m, out["hist"])
    assert np.all(np.diff(E) <= 1e-12 * E[0])
    assert E[-1] < 0.9 * E[0]


# --------------------------------------------------------------------------- brute force

@pytest.mark.parametrize("shape,so,nbl", [((7, 6, 8), 4, 2), ((9, 8), 8, 3), ((6, 5, 7), 2, 0)])
def test_forward_matches_spacetime_solve(oracle_lib, shape, so, nbl):
    rng = np.random.default_rng(sum(shape))
    nd = len(shape)
    h = tuple(rng.uniform(8, 12, size=nd))
    c = rng.uniform(1500, 3500, size=shape)
    m = 1.0 / c ** 2
    dt = 0.3 * min(h) / 3500
    nt = 12
    src = np.array([[rng.uniform(1, shape[a] - 2) * h[a] for a in range(nd)] for _ in range(2)])
    rec = np.array([[rng.uniform(0, shape[a] - 1) * h[a] for a in range(nd)] for _ in range(3)])
    wav = rng.standard_normal((nt, 2))
    u_init = rng.standard_normal((2,) + shape)
    g = oracle.Grid(shape, h, dt, so, nbl=nbl, sigma_max=80.0)
    out = oracle.forward(g, m, nt, src, wav, rec, u_init=u_init, want_hist=True)
    drec, U = dense.forward_spacetime(shape, h, dt, so, m, nt, src, wav, rec, nbl=nbl, sigma_max=80.0,
                                      u_init=u_init)
    assert rel(out["rec"], drec) < 1e-11
    assert rel(out["hist"][1:].reshape(nt + 1, -1), U) < 1e-11
    # sigma profile agrees with the independent construction
    np.testing.assert_allclose(oracle.sigma(g), dense.damping_profile(shape, nbl, 80.0), rtol=1e-14, atol=0)


def test_adjoint_matches_transposed_system(oracle_lib):
    shape = (6, 7, 5)
    rng = np.random.default_rng(3)
    h = (10.0, 11.0, 9.0)
    m = 1.0 / rng.uniform(1500, 3000, size=shape) ** 2
    dt = 0.3 * 9.0 / 3000
    nt = 10
    src = np.array([[23.0, 31.0, 17.0], [40.0, 12.5, 30.0]])
    rec = np.array([[11.0, 52.0, 8.0], [30.0, 30.0, 30.0], [5.0, 7.0, 33.0]])
    resid = rng.standard_normal((nt, 3))
    g = oracle.Grid(shape, h, dt, 4, nbl=2, sigma_max=50.0)
    got = oracle.adjoint(g, m, nt, resid, src_xyz=src, rec_xyz=rec, want_grad_m=False, want_grad_q=True)
    exp = dense.adjoint_spacetime(shape, h, dt, 4, m, nt, src, rec, resid, nbl=2, sigma_max=50.0)
    assert rel(got["grad_q"], exp) < 1e-11


# --------------------------------------------------------------------------- sources / receivers

def test_interpolation_reproduces_affine(oracle_lib):
    shape = (9, 10, 11)
    h = (10.0, 12.5, 7.0)
    g = oracle.Grid(shape, h, 1e-3, 4)
    rng = np.random.default_rng(5)
    a = rng.standard_normal(4)
    idx = np.indices(shape).reshape(3, -1).T * np.array(h)
    f = a[0] + idx @ a[1:]
    for _ in range(50):
        x = np.array([rng.uniform(0, (shape[i] - 1) * h[i]) for i in range(3)])
        lin, w = oracle.interp_corners(g, x)
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs(np.dot(w, f[lin]) - (a[0] + x @ a[1:])) < 1e-10
    lin, w = oracle.interp_corners(g, np.array([3 * h[0], 4 * h[1], 5 * h[2]]))
    assert w[np.argmax(w)] == 1.0 and lin[np.argmax(w)] == (3 * 10 + 4) * 11 + 5


def _small_problem(seed, shape=(10, 9, 11), so=4, nbl=2, nt=30):
    rng = np.random.default_rng(seed)
    h = (10.0, 10.0, 10.0)
    m = 1.0 / rng.uniform(1500, 3000, size=shape) ** 2
    dt = 0.35 * 10 / 3000
    g = oracle.Grid(shape, h, dt, so, nbl=nbl, sigma_max=40.0)
    return g, m, rng


def test_linearity_and_time_shift(oracle_lib):
    g, m, rng = _small_problem(11)
    nt = 30
    src = np.array([[43.0, 51.0, 37.0]])
    rec = np.array([[12.0, 33.0, 71.0], [80.0, 20.0, 20.0]])
    q1, q2 = rng.standard_normal((nt, 1)), rng.standard_normal((nt, 1))
    d1 = oracle.forward(g, m, nt, src, q1, rec)["rec"]
    d2 = oracle.forward(g, m, nt, src, q2, rec)["rec"]
    d12 = oracle.forward(g, m, nt, src, 2.0 * q1 - 3.0 * q2, rec)["rec"]
    assert rel(d12, 2.0 * d1 - 3.0 * d2) < 1e-13
    k = 7
    qs = np.zeros_like(q1)
    qs[k:] = q1[:-k]
    ds = oracle.forward(g, m, nt, src, qs, rec)["rec"]
    assert np.array_equal(ds[:k], np.zeros_like(ds[:k]))
    assert np.array_equal(ds[k:], d1[:-k])


def test_reciprocity(oracle_lib):
    """Swapping an (off-grid) source and receiver leaves the trace unchanged:
    every step's Green's matrix is a palindromic product of symmetric blocks."""
    g, m, rng = _small_problem(12)
    nt = 40
    a = np.array([[23.0, 41.5, 37.2]])
    b = np.array([[71.0, 30.0, 66.6]])
    q = rng.standard_normal((nt, 1))
    dab = oracle.forward(g, m, nt, a, q, b)["rec"]
    dba = oracle.forward(g, m, nt, b, q, a)["rec"]
    assert rel(dab, dba) < 1e-12


# --------------------------------------------------------------------------- adjoint / gradient

def test_dot_product(oracle_lib):
    g, m, rng = _small_problem(13)
    nt = 30
    src = np.array([[43.0, 51.0, 37.0], [20.0, 60.0, 50.0]])
    rec = np.array([[12.0, 33.0, 71.0], [80.0, 20.0, 20.0], [55.5, 44.4, 33.3]])
    q = rng.standard_normal((nt, 2))
    dd = rng.standard_normal((nt, 3))
    Fq = oracle.forward(g, m, nt, src, q, rec)["rec"]
    Ftd = oracle.adjoint(g, m, nt, dd, src_xyz=src, rec_xyz=rec, want_grad_m=False, want_grad_q=True)["grad_q"]
    lhs, rhs = np.sum(Fq * dd), np.sum(q * Ftd)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def _misfit(g, m, nt, src, q, rec, dobs):
    d = oracle.forward(g, m, nt, src, q, rec)["rec"]
    return 0.5 * np.sum((d - dobs) ** 2)


@pytest.mark.parametrize("shape,so", [((10, 9, 11), 4), ((14, 12), 8)])
def test_gradient_finite_difference(oracle_lib, shape, so):
    g, m, rng = _small_problem(14, shape=shape, so=so, nbl=2, nt=40)
    nt = 40
    nd = len(shape)
    src = np.array([[43.0, 51.0, 37.0][:nd]])
    rec = np.array([[12.0, 33.0, 71.0][:nd], [80.0, 20.0, 20.0][:nd]])
    q = np.asarray(rng.standard_normal((nt, 1)))
    m_true = m * (1 + 0.1 * rng.uniform(-1, 1, size=shape))
    dobs = oracle.forward(g, m_true, nt, src, q, rec)["rec"]
    fw = oracle.forward(g, m, nt, src, q, rec, want_hist=True)
    resid = fw["rec"] - dobs
    grads = [oracle.adjoint(g, m, nt, resid, hist=fw["hist"], src_xyz=src, rec_xyz=rec, form=f)["grad_m"]
             for f in (1, 2)]
    assert rel(grads[1], grads[0]) < 1e-12
    dm = m * rng.uniform(-1, 1, size=shape)
    gd = np.sum(grads[0] * dm)
    errs = []
    for eps in (1e-3, 1e-4):
        fd = (_misfit(g, m + eps * dm, nt, src, q, rec, dobs)
              - _misfit(g, m - eps * dm, nt, src, q, rec, dobs)) / (2 * eps)
        errs.append(abs(fd - gd) / abs(gd))
    # central differences: error O(eps^2) -> 100x smaller per 10x smaller eps
    assert errs[1] < 1e-5
    assert errs[1] < errs[0] / 30


def test_checkpoint_resume_bitwise(oracle_lib):
    g, m, rng = _small_problem(15)
    nt, k = 30, 11
    src = np.array([[43.0, 51.0, 37.0]])
    rec = np.array([[12.0, 33.0, 71.0]])
    q = rng.standard_normal((nt, 1))
    full = oracle.forward(g, m, nt, src, q, rec, want_final=True)
    a = oracle.forward(g, m, k, src, q[:k], rec, want_final=True)
    b = oracle.forward(g, m, nt - k, src, q[k:], rec, u_init=a["final"], want_final=True)
    assert np.array_equal(np.vstack([a["rec"], b["rec"]]), full["rec"])
    assert np.array_equal(b["final"], full["final"])


def test_damping_profile_hand_values(oracle_lib):
    """sigma at listed points against values worked out by hand from the
    definition (tests/golden/damping_profile_values.txt)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "damping_profile_values.txt")
    n = 0
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        nd = int(f[0])
        shape = tuple(int(v) for v in f[1:1 + nd])
        nbl, smax = int(f[1 + nd]), float(f[2 + nd])
        idx = tuple(int(v) for v in f[3 + nd:3 + 2 * nd])
        expect = float(f[3 + 2 * nd])
        g = oracle.Grid(shape, (10.0,) * nd, 1e-4, 2, nbl=nbl, sigma_max=smax)
        assert oracle.sigma(g)[idx] == expect, (shape, nbl, idx)
        n += 1
    assert n == 19

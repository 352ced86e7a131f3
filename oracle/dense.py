"""Brute-force pin for the loop oracle on tiny grids.  TEST INFRASTRUCTURE ONLY.

Everything here is built a second way, sharing nothing with ``oracle.c``:

* the second-derivative weights come from solving the polynomial-exactness
  (moment) conditions in exact rational arithmetic, not from a closed form;
* the Laplacian is an explicit sparse matrix assembled from Kronecker products
  of 1D operators;
* all nt time steps are solved at once as one block lower-triangular
  space-time linear system  A u^{n+1} - B u^n + C u^{n-1} = f^n  with
  A = diag(m (1 + st)), B = 2 diag(m) + dt^2 L, C = diag(m (1 - st)), by a
  sparse direct solver, instead of being marched;
* source/receiver interpolation is an explicit sparse matrix.

The scheme itself (leapfrog with centred damping, zero ghosts) follows the
standard discretisation of  m u_tt + m sigma u_t = lap u + q  that the oracle
implements; see the header of oracle.c.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def moment_coeffs(so: int):
    """c_0..c_k (k = so/2) such that sum_{j=-k..k} c_|j| x_j^p is the exact
    second derivative of x^p at 0 for p = 0..2k (odd p vanish by symmetry).
    Solved in exact rationals by Gauss-Jordan elimination."""
    k = so // 2
    # unknowns c_0..c_k; equation q (q=0..k): sum_j w_j(q) c_j = rhs_q where
    # w_0(q) = 0^{2q}, w_j(q) = 2 j^{2q}; rhs = 2 for q=1 (d2/dx2 x^2 = 2), else 0.
    A = [[Fraction(0)] * (k + 2) for _ in range(k + 1)]
    for q in range(k + 1):
        A[q][0] = Fraction(1 if q == 0 else 0)
        for j in range(1, k + 1):
            A[q][j] = Fraction(2 * j ** (2 * q))
        A[q][k + 1] = Fraction(2 if q == 1 else 0)
    n = k + 1
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    return [A[j][k + 1] for j in range(n)]


def second_derivative_1d(n: int, so: int, periodic: bool = False) -> sp.csr_matrix:
    c = [float(v) for v in moment_coeffs(so)]
    k = so // 2
    rows, cols, vals = [], [], []
    for i in range(n):
        rows.append(i); cols.append(i); vals.append(c[0])
        for j in range(1, k + 1):
            for t in (i - j, i + j):
                if 0 <= t < n:
                    rows.append(i); cols.append(t); vals.append(c[j])
                elif periodic:
                    rows.append(i); cols.append(t % n); vals.append(c[j])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def laplacian_matrix(shape, spacing, so: int, periodic: bool = False) -> sp.csr_matrix:
    mats = []
    for a, n in enumerate(shape):
        D = second_derivative_1d(n, so, periodic) / (spacing[a] ** 2)
        ops = [sp.identity(s, format="csr") for s in shape]
        ops[a] = D
        K = ops[0]
        for o in ops[1:]:
            K = sp.kron(K, o, format="csr")
        mats.append(K)
    L = mats[0]
    for M in mats[1:]:
        L = L + M
    return L.tocsr()


def damping_profile(shape, nbl: int, sigma_max: float) -> np.ndarray:
    """sigma_max * sum_a (depth into the layer / nbl)^2, per point."""
    if nbl <= 0:
        return np.zeros(shape)
    prof = np.zeros(shape)
    for a, n in enumerate(shape):
        i = np.arange(n)
        inner_lo, inner_hi = nbl, n - 1 - nbl
        d = np.where(i < inner_lo, inner_lo - i, np.where(i > inner_hi, i - inner_hi, 0)) / nbl
        sh = [1] * len(shape)
        sh[a] = n
        prof = prof + (d ** 2).reshape(sh)
    return sigma_max * prof


def interp_matrix(shape, spacing, xyz) -> sp.csr_matrix:
    """Sparse [npoints, N] multilinear interpolation (corners outside dropped)."""
    xyz = np.atleast_2d(np.asarray(xyz, dtype=np.float64))
    nd = len(shape)
    rows, cols, vals = [], [], []
    strides = np.cumprod((1,) + tuple(shape[::-1]))[:-1][::-1]
    for r, x in enumerate(xyz):
        base = [int(np.floor(x[a] / spacing[a])) for a in range(nd)]
        frac = [x[a] / spacing[a] - base[a] for a in range(nd)]
        for bits in product((0, 1), repeat=nd):
            idx = [base[a] + bits[a] for a in range(nd)]
            if any(i < 0 or i >= shape[a] for a, i in enumerate(idx)):
                continue
            w = 1.0
            for a in range(nd):
                w *= frac[a] if bits[a] else 1.0 - frac[a]
            rows.append(r)
            cols.append(int(np.dot(idx, strides)))
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(xyz.shape[0], int(np.prod(shape))))


def forward_spacetime(shape, spacing, dt, so, m, nt, src_xyz, wavelet, rec_xyz,
                      nbl=0, sigma_max=0.0, u_init=None):
    """Solve all nt steps at once. Returns (receivers [nt, nrec], u [nt+1, N] = u^0..u^nt)."""
    N = int(np.prod(shape))
    m = np.asarray(m, dtype=np.float64).reshape(N)
    st = damping_profile(shape, nbl, sigma_max).reshape(N) * dt / 2.0
    L = laplacian_matrix(shape, spacing, so)
    A = sp.diags(m * (1.0 + st))
    B = sp.diags(2.0 * m) + dt * dt * L
    C = sp.diags(m * (1.0 - st))
    Ps = interp_matrix(shape, spacing, src_xyz).T.tocsr()   # [N, nsrc]
    Pr = interp_matrix(shape, spacing, rec_xyz)             # [nrec, N]
    u0 = np.zeros(N) if u_init is None else np.asarray(u_init[0], dtype=np.float64).reshape(N)
    um = np.zeros(N) if u_init is None else np.asarray(u_init[1], dtype=np.float64).reshape(N)
    wavelet = np.asarray(wavelet, dtype=np.float64).reshape(nt, -1)
    blocks = [[None] * nt for _ in range(nt)]
    rhs = np.zeros(nt * N)
    for n in range(nt):
        blocks[n][n] = A
        if n >= 1:
            blocks[n][n - 1] = -B
        if n >= 2:
            blocks[n][n - 2] = C
        f = dt * dt * (Ps @ wavelet[n])
        if n == 0:
            f = f + B @ u0 - C @ um
        if n == 1:
            f = f - C @ u0
        rhs[n * N:(n + 1) * N] = f
    S = sp.bmat(blocks, format="csc")
    U = spla.spsolve(S, rhs).reshape(nt, N)
    rec = (Pr @ U.T).T
    return rec, np.vstack([u0[None], U])


def adjoint_spacetime(shape, spacing, dt, so, m, nt, src_xyz, rec_xyz, resid,
                      nbl=0, sigma_max=0.0):
    """Source-side adjoint by the transposed space-time system: returns
    dt^2 Ps^T lambda where S^T lambda = Pr^T resid (the exact transpose of the
    forward map q -> d)."""
    N = int(np.prod(shape))
    m = np.asarray(m, dtype=np.float64).reshape(N)
    st = damping_profile(shape, nbl, sigma_max).reshape(N) * dt / 2.0
    L = laplacian_matrix(shape, spacing, so)
    A = sp.diags(m * (1.0 + st))
    B = sp.diags(2.0 * m) + dt * dt * L
    C = sp.diags(m * (1.0 - st))
    Ps = interp_matrix(shape, spacing, src_xyz).T.tocsr()
    Pr = interp_matrix(shape, spacing, rec_xyz)
    blocks = [[None] * nt for _ in range(nt)]
    for n in range(nt):
        blocks[n][n] = A
        if n >= 1:
            blocks[n][n - 1] = -B
        if n >= 2:
            blocks[n][n - 2] = C
    S = sp.bmat(blocks, format="csc")
    resid = np.asarray(resid, dtype=np.float64).reshape(nt, -1)
    rhs = np.concatenate([Pr.T @ resid[n] for n in range(nt)])
    lam = spla.spsolve(S.T.tocsc(), rhs).reshape(nt, N)
    return dt * dt * np.stack([Ps.T @ lam[n] for n in range(nt)])

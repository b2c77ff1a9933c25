"""Oracle for the sparse mixed-precision iterative solver (test
infrastructure only: the tests, __graft_entry__.smoke() and the CPU leg of
bench.py use it; the GPU path shares nothing with it).

Section 3.2, Algorithm 2: the inner-outer FGMRES(m_out)-GMRES_SP(m_in).
The outer loop is flexible GMRES in double precision; its preconditioner
is one cycle of GMRES(m_in) from a zero initial guess run in single
precision on the single-precision copy of A (CRS storage).  Plain numpy,
one step at a time in the algorithm's order:

* ``csr_matvec``   y = A x with A in CRS (row pointers, column indices,
                   values), accumulated in the dtype of the values.
* ``gmres_cycle``  one GMRES(m) cycle from z = 0 on A z = v in a given
                   precision: Arnoldi with modified Gram-Schmidt, Givens
                   rotations on the Hessenberg matrix, z = V y.
* ``fgmres_gmres`` Algorithm 2, with the readings listed in its docstring.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

EPS_D = 2.0 ** -53
ITERMAX = 30


def csr_matvec(rowptr, colind, vals, x):
    """y_i = sum_{p in row i} vals[p] x[colind[p]], in the precision of vals."""
    rowptr = np.asarray(rowptr)
    n = rowptr.size - 1
    prod = np.asarray(vals) * np.asarray(x, dtype=np.asarray(vals).dtype)[np.asarray(colind)]
    row = np.repeat(np.arange(n), np.diff(rowptr))
    y = np.zeros(n, dtype=prod.dtype)
    np.add.at(y, row, prod)
    return y


def norm_inf_csr(rowptr, vals):
    """||A||_inf: the largest row sum of |a_ij|."""
    n = len(rowptr) - 1
    a = np.abs(np.asarray(vals, dtype=np.float64))
    sums = np.add.reduceat(a, np.asarray(rowptr[:-1])) if a.size else np.zeros(n)
    sums[np.diff(rowptr) == 0] = 0.0
    return float(sums.max()) if n else 0.0


def _givens(a, b):
    """c, s with [c s; -s c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0
    r = math.hypot(a, b)
    return a / r, b / r


def gmres_cycle(matvec, v, m: int, dtype=np.float32, tol_rel: float | None = None):
    """One cycle of GMRES(m) for A z = v from z = 0, every operation in dtype:
    the Krylov basis by Arnoldi with modified Gram-Schmidt, the least-squares
    problem min ||beta e1 - H y|| by Givens rotations as the columns of H
    arrive, then z = V y.  Stops early on breakdown (h_{j+1,j} = 0) or when
    the rotated residual |g_{j+1}| falls to tol_rel * beta (default: the unit
    roundoff of dtype).  Returns (z, steps)."""
    dt = np.dtype(dtype)
    eps = float(np.finfo(dt).eps) / 2 if tol_rel is None else tol_rel
    v = np.asarray(v, dtype=dt)
    n = v.size
    beta = dt.type(np.sqrt(np.dot(v, v)))
    if beta == 0:
        return np.zeros(n, dtype=dt), 0
    V = np.zeros((m + 1, n), dtype=dt)
    H = np.zeros((m + 1, m), dtype=dt)
    cs = np.zeros(m, dtype=dt)
    sn = np.zeros(m, dtype=dt)
    g = np.zeros(m + 1, dtype=dt)
    g[0] = beta
    V[0] = v / beta
    k = 0
    for j in range(m):
        w = np.asarray(matvec(V[j]), dtype=dt)
        for i in range(j + 1):                      # modified Gram-Schmidt
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = dt.type(np.sqrt(np.dot(w, w)))
        for i in range(j):                          # earlier rotations
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        c, s = _givens(float(H[j, j]), float(H[j + 1, j]))
        cs[j], sn[j] = c, s
        H[j, j] = c * H[j, j] + s * H[j + 1, j]
        H[j + 1, j] = 0
        g[j + 1] = -s * g[j]
        g[j] = c * g[j]
        k = j + 1
        breakdown = float(np.sqrt(np.dot(w, w))) == 0.0
        if breakdown or abs(float(g[j + 1])) <= eps * float(beta):
            break
        V[j + 1] = w / dt.type(np.sqrt(np.dot(w, w)))
    y = np.zeros(k, dtype=dt)
    for i in range(k - 1, -1, -1):                  # back substitution
        y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
    z = V[:k].T @ y
    return z.astype(dt), k


@dataclass
class SparseIRResult:
    x: np.ndarray
    outer: int         # outer cycles (restarts) that ended with x updated
    inner_calls: int   # preconditioner applications (inner GMRES_SP cycles)
    converged: bool
    rnorm: float
    xnorm: float


def fgmres_gmres(rowptr, colind, vals, b, m_out: int = 20, m_in: int = 30,
                 inner_dtype=np.float32, itermax: int = ITERMAX, stall: float = 0.9):
    """Algorithm 2, FGMRES(m_out)-GMRES_SP(m_in), from x_0 = 0.  Each outer
    iteration i: r = b - A x_i in FP64; the stopping test of Section 3 in the
    infinity norm, ||r||_inf <= sqrt(n) eps_d ||A||_inf ||x_i||_inf, checked
    on this true residual; then up to m_out flexible Arnoldi steps in FP64:
    v_k = r / h_{k,k-1}; z_k = one GMRES(m_in) cycle in inner_dtype on the
    inner_dtype copy of A for A z = v_k (x = 0 start); r = A z_k; modified
    Gram-Schmidt against v_1..v_k; h_{k+1,k} = ||r||_2.  The cycle ends early
    when the rotated least-squares residual |g_{k+1}| reaches the 2-norm form
    of the same threshold (sqrt(n) eps_d ||A||_inf max(||x_i||_inf, ||b||_inf
    / ||A||_inf)).  Then y minimizes ||beta e1 - H y||_2 and
    x_{i+1} = x_i + Z y.  Failure: itermax outer iterations, or the dense
    path's stall rule applied to the outer residuals."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colind = np.asarray(colind, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    vals_s = vals.astype(inner_dtype)
    anorm = norm_inf_csr(rowptr, vals)
    thr = math.sqrt(n) * EPS_D * anorm
    x = np.zeros(n)
    inner_calls = 0
    prev = ratio_prev = 0.0
    mv_s = lambda u: csr_matvec(rowptr, colind, vals_s, u)
    for i in range(itermax + 1):
        r = b - csr_matvec(rowptr, colind, vals, x)
        rn, xn = float(np.abs(r).max()), float(np.abs(x).max()) if n else 0.0
        if rn <= thr * xn or n == 0:
            return SparseIRResult(x, i, inner_calls, True, rn, xn)
        if not (math.isfinite(rn) and math.isfinite(xn)):
            break
        if i >= 1 and prev > 0:
            rho = rn / prev
            if (i >= 2 and rho >= stall and ratio_prev >= stall) or (i >= 3 and rho >= 1.0):
                break
            ratio_prev = rho
        prev = rn
        if i == itermax:
            break
        beta = float(np.linalg.norm(r))
        scale = max(xn, float(np.abs(b).max()) / anorm if anorm > 0 else 0.0)
        thr2 = thr * scale
        V = np.zeros((m_out + 1, n))
        Z = np.zeros((m_out, n))
        H = np.zeros((m_out + 1, m_out))
        cs, sn = np.zeros(m_out), np.zeros(m_out)
        g = np.zeros(m_out + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m_out):
            z, _ = gmres_cycle(mv_s, V[j].astype(inner_dtype), m_in, inner_dtype)
            inner_calls += 1
            Z[j] = z.astype(np.float64)
            w = csr_matvec(rowptr, colind, vals, Z[j])
            for q in range(j + 1):                  # modified Gram-Schmidt
                H[q, j] = float(w @ V[q])
                w = w - H[q, j] * V[q]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            for q in range(j):
                t = cs[q] * H[q, j] + sn[q] * H[q + 1, j]
                H[q + 1, j] = -sn[q] * H[q, j] + cs[q] * H[q + 1, j]
                H[q, j] = t
            c, s = _givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = c * H[j, j] + s * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -s * g[j]
            g[j] = c * g[j]
            k = j + 1
            if hn == 0.0 or abs(g[j + 1]) <= thr2:
                break
            V[j + 1] = w / hn
        y = np.zeros(k)
        for q in range(k - 1, -1, -1):
            y[q] = (g[q] - H[q, q + 1:k] @ y[q + 1:k]) / H[q, q]
        x = x + Z[:k].T @ y
    r = b - csr_matvec(rowptr, colind, vals, x)
    return SparseIRResult(x, itermax, inner_calls, False, float(np.abs(r).max()),
                          float(np.abs(x).max()) if n else 0.0)

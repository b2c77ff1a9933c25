"""Generators of seeded synthetic linear systems.

All draws use numpy's PCG64 (``numpy.random.default_rng``) in a fixed order,
so a (kind, size, seed) triple names one input exactly.  Matrices are FP64,
row-major.  The paper measures on random dense matrices with a prescribed
condition number (Section 4: 200 random 200-by-200 matrices per condition
number) and on matrices with uniformly distributed random entries
(Section 5); these generators produce inputs of those kinds at the sizes the
solver is benchmarked on:

* ``uniform_system``: A with iid U[-1, 1] entries, x_true iid U[-1, 1],
  b = A x_true.
* ``prescribed_cond_system``: A = U diag(sigma) V^T with U, V Haar-random
  orthogonal and sigma geometric from 1 down to 1/kappa, so that the
  2-norm condition number is kappa; x_true iid U[-1, 1], b = A x_true.
* ``spd_system``: A = Q diag(lambda) Q^T with lambda log-uniform in
  [1/kappa, 1] (endpoints forced), symmetrized; X_true iid U[-1, 1], B = A X.
* ``batched_systems``: many independent prescribed-condition systems of
  uneven sizes.
* ``grad_problem``: a prescribed-condition A with Gaussian right-hand sides
  and Gaussian loss weights W (loss = sum W * X).
* ``integer_system``: small integer A and x_true so that b = A x_true is
  exact in FP64 and x_true is the exact solution.
* ``sparse_convdiff3d``: the 7-point finite-difference operator of
  -Laplace(u) + w . grad(u) on a k^3 grid (Dirichlet boundary, first-order
  upwind convection with Peclet number w h / 2 per direction; w = 0 gives the
  symmetric 3-D Poisson matrix) in CRS form, x_true iid U[-1, 1],
  b = A x_true: synthetic stand-ins for the sparse matrices of Section 3.2.

Haar-random orthogonal matrices are the Q factor of a QR factorization of a
Gaussian matrix with the columns' signs fixed by sign(diag R) (Stewart 1980;
Mezzadri 2007).  For large n the QR may run through torch on a GPU; the
Gaussian itself is always drawn by numpy from the seed.
"""
from __future__ import annotations

import numpy as np


def _rng(seed):
    if isinstance(seed, np.random.Generator):
        return seed
    return np.random.default_rng(seed)


def sigma_geometric(n: int, kappa: float) -> np.ndarray:
    """sigma_i = kappa^(-i/(n-1)), i = 0..n-1: geometric from 1 to 1/kappa."""
    if n == 1:
        return np.ones(1)
    return kappa ** (-np.arange(n, dtype=np.float64) / (n - 1))


def haar_orthogonal(n: int, g: np.random.Generator, backend: str = "numpy", device=None):
    """Haar-distributed n x n orthogonal matrix from the next n*n normals of g.

    backend="numpy": LAPACK QR on the host, returns numpy.
    backend="torch": torch.linalg.qr on ``device``, returns a torch tensor.
    """
    G = g.standard_normal((n, n))
    if backend == "numpy":
        Q, R = np.linalg.qr(G)
        d = np.sign(np.diag(R))
        d[d == 0] = 1.0
        return Q * d
    import torch

    Gt = torch.from_numpy(G).to(device)
    del G
    Q, R = torch.linalg.qr(Gt)
    del Gt
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    del R
    Q.mul_(d)
    return Q


def uniform_system(n: int, seed, nrhs: int = 1):
    """A iid U[-1,1], x_true iid U[-1,1] (n x nrhs), b = A x_true; all FP64."""
    g = _rng(seed)
    A = g.uniform(-1.0, 1.0, (n, n))
    x_true = g.uniform(-1.0, 1.0, (n, nrhs))
    b = A @ x_true
    return A, b, x_true


def prescribed_cond_system(n: int, kappa: float, seed, nrhs: int = 1,
                           backend: str = "numpy", device=None):
    """A = U diag(sigma) V^T, sigma geometric 1..1/kappa, U and V Haar.

    Draw order: U's Gaussian, V's Gaussian, then x_true iid U[-1,1];
    b = A x_true.  With backend="torch" A and b are torch tensors on
    ``device`` (x_true stays numpy)."""
    g = _rng(seed)
    s = sigma_geometric(n, kappa)
    if backend == "numpy":
        U = haar_orthogonal(n, g)
        V = haar_orthogonal(n, g)
        A = (U * s) @ V.T
        del U, V
        x_true = g.uniform(-1.0, 1.0, (n, nrhs))
        b = A @ x_true
        return A, b, x_true
    import torch

    U = haar_orthogonal(n, g, "torch", device)
    U.mul_(torch.from_numpy(s).to(U.device))
    V = haar_orthogonal(n, g, "torch", device)
    A = U @ V.T
    del U, V
    x_true = g.uniform(-1.0, 1.0, (n, nrhs))
    b = A @ torch.from_numpy(x_true).to(A.device)
    return A, b, x_true


def spd_system(n: int, kappa: float, seed, nrhs: int = 16, backend: str = "numpy", device=None):
    """A = Q diag(lambda) Q^T, lambda log-uniform in [1/kappa, 1] with
    lambda_0 = 1 and lambda_{n-1} = 1/kappa; A symmetrized as (A + A^T)/2.
    Draw order: lambda, Q's Gaussian, X_true iid U[-1,1]; B = A X_true."""
    g = _rng(seed)
    lam = np.exp(g.uniform(np.log(1.0 / kappa), 0.0, n))
    lam[0] = 1.0
    if n > 1:
        lam[-1] = 1.0 / kappa
    if backend == "numpy":
        Q = haar_orthogonal(n, g)
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
        del Q
        X = g.uniform(-1.0, 1.0, (n, nrhs))
        return A, A @ X, X
    import torch

    Q = haar_orthogonal(n, g, "torch", device)
    A = (Q * torch.from_numpy(lam).to(Q.device)) @ Q.T
    del Q
    A = 0.5 * (A + A.T)
    X = g.uniform(-1.0, 1.0, (n, nrhs))
    return A, A @ torch.from_numpy(X).to(A.device), X


def batched_systems(count: int = 4096, seed: int = 401, nmin: int = 16, nmax: int = 512,
                    kmin: float = 1e1, kmax: float = 1e5):
    """``count`` independent systems; system i uses SeedSequence(seed).spawn(count)[i]:
    n_i ~ U{nmin..nmax}, kappa_i log-uniform in [kmin, kmax], then A_i, b_i as in
    prescribed_cond_system.  Returns lists (A_i, b_i, x_true_i) and the kappas."""
    children = np.random.SeedSequence(seed).spawn(count)
    As, bs, xs, ks = [], [], [], []
    for ss in children:
        g = np.random.default_rng(ss)
        n = int(g.integers(nmin, nmax + 1))
        kappa = float(np.exp(g.uniform(np.log(kmin), np.log(kmax))))
        A, b, x = prescribed_cond_system(n, kappa, g)
        As.append(A)
        bs.append(b)
        xs.append(x)
        ks.append(kappa)
    return As, bs, xs, ks


def grad_problem(n: int = 4096, nrhs: int = 64, kappa: float = 1e3, seed=501,
                 backend: str = "numpy", device=None):
    """A = U diag(sigma) V^T (kappa), B iid N(0,1) n x nrhs, W iid N(0,1)."""
    g = _rng(seed)
    s = sigma_geometric(n, kappa)
    if backend == "numpy":
        U = haar_orthogonal(n, g)
        V = haar_orthogonal(n, g)
        A = (U * s) @ V.T
    else:
        import torch

        U = haar_orthogonal(n, g, "torch", device)
        U.mul_(torch.from_numpy(s).to(U.device))
        V = haar_orthogonal(n, g, "torch", device)
        A = (U @ V.T).cpu().numpy()
    B = g.standard_normal((n, nrhs))
    W = g.standard_normal((n, nrhs))
    return A, B, W


def integer_system(n: int, seed, lo: int = -9, hi: int = 9, xlo: int = -9, xhi: int = 9):
    """Integer A (entries in [lo, hi]) and integer x_true, with b = A x_true
    computed exactly (all values are small integers, so the FP64 product is
    exact and x_true is the exact solution).  A is re-drawn while it looks
    numerically singular; callers that need certainty confirm with an exact
    rational solve."""
    g = _rng(seed)
    while True:
        A = g.integers(lo, hi + 1, (n, n)).astype(np.float64)
        if n == 0 or abs(np.linalg.det(A)) > 0.5:
            break
    x = g.integers(xlo, xhi + 1, (n, 1)).astype(np.float64)
    b = A @ x
    return A, b, x


def sparse_convdiff3d(k: int, peclet: float = 0.0, seed=0):
    """CRS (rowptr, colind, vals) of the 7-point operator on a k x k x k grid
    (row index i + k j + k^2 l), scaled by h^2: diagonal 6 + sum of the upwind
    terms, neighbours -1 (minus the upwind term in the upstream direction);
    x_true iid U[-1, 1] from the seed and b = A x_true (FP64)."""
    g = _rng(seed)
    n = k ** 3
    p = float(peclet)
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(k, k, k)  # [l, j, i]
    for (dl, dj, di) in ((0, 0, 0), (-1, 0, 0), (0, -1, 0), (0, 0, -1), (1, 0, 0), (0, 1, 0),
                         (0, 0, 1)):
        if (dl, dj, di) == (0, 0, 0):
            src = idx.ravel()
            rows.append(src)
            cols.append(src)
            vals.append(np.full(n, 6.0 + 3.0 * 2.0 * p))
            continue
        sl = [slice(None)] * 3
        sd = [slice(None)] * 3
        for ax, d in enumerate((dl, dj, di)):
            if d == -1:
                sl[ax], sd[ax] = slice(1, None), slice(0, -1)
            elif d == 1:
                sl[ax], sd[ax] = slice(0, -1), slice(1, None)
        r = idx[tuple(sl)].ravel()
        c = idx[tuple(sd)].ravel()
        # upwind convection with positive velocity in every direction: the
        # upstream neighbour (d = -1) takes -(1 + 2p), the downstream one -1
        v = -(1.0 + 2.0 * p) if -1 in (dl, dj, di) else -1.0
        rows.append(r)
        cols.append(c)
        vals.append(np.full(r.size, v))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    colind = c.astype(np.int32)
    x_true = g.uniform(-1.0, 1.0, n)
    # b = A x_true, row by row in FP64
    b = np.zeros(n)
    np.add.at(b, r, v * x_true[c])
    return rowptr, colind, v.astype(np.float64), b, x_true


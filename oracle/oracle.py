"""ctypes front end of the C oracle (test infrastructure only).

Every function takes and returns numpy arrays in row-major (C) order and
calls the plain C routines of ``oracle.c``:

* ``getrf``     -- unblocked Gaussian elimination with partial row pivoting,
                   PA = LU (Section 2.1, Direct Methods).
* ``getrs``     -- Ly = Pb, Ux = y, or the transposed system.
* ``gesv_ir``   -- iterative refinement with the structure of Algorithm 1:
                   ``lowp=False`` refines with double-precision factors (the
                   reference solver), ``lowp=True`` is Algorithm 1 with an
                   FP32 factor and FP64 residual/update.
* ``potrf``, ``posv_ir`` -- the symmetric positive definite variant
                   (SPOTRF/SPOTRS with a DSYMM residual, Section 3.1.1).
* ``residual_ld`` -- b - A x accumulated in extended precision, for checks.
* ``metrics``   -- normwise/componentwise backward error and forward error.
* ``condest1``  -- estimate of kappa_1(A) (Hager's method with Higham's
                   refinement) from the FP64 factors, for the Section 4 rule
                   that refinement needs kappa eps_s below about one.

The stopping rule is ||r||_inf <= sqrt(n) 2^-53 ||A||_inf ||x||_inf per
right-hand side (Section 3), checked on the residual of the current iterate;
30 iterations mean failure (Section 4).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ITERMAX = 30
EPS_D = 2.0 ** -53


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(os.path.join(_HERE, "oracle.c"))
    ):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.orc_norm_inf.argtypes = [I, P, I]
    lib.orc_norm_inf.restype = ctypes.c_double
    lib.orc_dgetrf_steps.argtypes = [I, P, I, P, I]
    lib.orc_dgetrf_steps.restype = I
    lib.orc_dgetrf.argtypes = [I, P, I, P]
    lib.orc_dgetrf.restype = I
    lib.orc_sgetrf.argtypes = [I, P, I, P]
    lib.orc_sgetrf.restype = I
    lib.orc_dgetrs.argtypes = [I, I, P, I, P, P, I, I]
    lib.orc_dgetrs.restype = None
    lib.orc_sgetrs.argtypes = [I, I, P, I, P, P, I]
    lib.orc_sgetrs.restype = None
    lib.orc_dpotrf.argtypes = [I, P, I]
    lib.orc_dpotrf.restype = I
    lib.orc_spotrf.argtypes = [I, P, I]
    lib.orc_spotrf.restype = I
    lib.orc_dpotrs.argtypes = [I, I, P, I, P, I]
    lib.orc_dpotrs.restype = None
    lib.orc_spotrs.argtypes = [I, I, P, I, P, I]
    lib.orc_spotrs.restype = None
    lib.orc_residual.argtypes = [I, I, P, I, P, I, P, I, P, I, I]
    lib.orc_residual.restype = None
    lib.orc_residual_ld.argtypes = [I, I, P, I, P, I, P, I, P, P]
    lib.orc_residual_ld.restype = None
    lib.orc_gesv_ir.argtypes = [I, I, P, I, P, I, P, I, I, I, I, P]
    lib.orc_gesv_ir.restype = I
    lib.orc_posv_ir.argtypes = [I, I, P, I, P, I, P, I, I, I, P]
    lib.orc_posv_ir.restype = I
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as2d(b):
    b = np.asarray(b)
    return (b.reshape(-1, 1), True) if b.ndim == 1 else (b, False)


def norm_inf(A) -> float:
    A = _c(A, np.float64)
    n = A.shape[0]
    return _load().orc_norm_inf(n, _ptr(A), A.shape[1])


def getrf(A, steps: int | None = None):
    """Return (LU, ipiv, info) of PA = LU with partial pivoting, in FP64.

    ``steps`` stops the elimination after that many columns (used to time a
    bounded sample of a large factorization)."""
    LU = np.array(A, dtype=np.float64, order="C", copy=True)
    n = LU.shape[0]
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    info = _load().orc_dgetrf_steps(n, _ptr(LU), n, _ptr(ipiv), n if steps is None else steps)
    return LU, ipiv[:n], info


def sgetrf(A):
    """FP32 PA = LU (Algorithm 1 step 1 in single precision)."""
    LU = np.array(A, dtype=np.float32, order="C", copy=True)
    n = LU.shape[0]
    ipiv = np.zeros(max(n, 1), dtype=np.int32)
    info = _load().orc_sgetrf(n, _ptr(LU), n, _ptr(ipiv))
    return LU, ipiv[:n], info


def getrs(LU, ipiv, B, trans: bool = False):
    LU = _c(LU, np.float64)
    ipiv = _c(ipiv, np.int32)
    B2, vec = _as2d(B)
    X = np.array(B2, dtype=np.float64, order="C", copy=True)
    n, nrhs = X.shape
    _load().orc_dgetrs(n, nrhs, _ptr(LU), LU.shape[1], _ptr(ipiv), _ptr(X), nrhs, int(trans))
    return X.ravel() if vec else X


def sgetrs(LU, ipiv, B):
    LU = _c(LU, np.float32)
    ipiv = _c(ipiv, np.int32)
    B2, vec = _as2d(B)
    X = np.array(B2, dtype=np.float32, order="C", copy=True)
    n, nrhs = X.shape
    _load().orc_sgetrs(n, nrhs, _ptr(LU), LU.shape[1], _ptr(ipiv), _ptr(X), nrhs)
    return X.ravel() if vec else X


def potrf(A):
    """Return (L, info) with A = L L^T (lower triangle; upper part untouched)."""
    L = np.array(A, dtype=np.float64, order="C", copy=True)
    n = L.shape[0]
    info = _load().orc_dpotrf(n, _ptr(L), n)
    return np.tril(L), info


def spotrf(A):
    L = np.array(A, dtype=np.float32, order="C", copy=True)
    n = L.shape[0]
    info = _load().orc_spotrf(n, _ptr(L), n)
    return np.tril(L), info


def spotrs(L, B):
    """FP32 L L^T x = b with the factor of ``spotrf`` (the SPOTRS of the
    single-precision variant)."""
    L = _c(L, np.float32)
    B2, vec = _as2d(B)
    X = np.array(B2, dtype=np.float32, order="C", copy=True)
    n, nrhs = X.shape
    _load().orc_spotrs(n, nrhs, _ptr(L), L.shape[1], _ptr(X), nrhs)
    return X.ravel() if vec else X


def potrs(L, B):
    L = _c(L, np.float64)
    B2, vec = _as2d(B)
    X = np.array(B2, dtype=np.float64, order="C", copy=True)
    n, nrhs = X.shape
    _load().orc_dpotrs(n, nrhs, _ptr(L), L.shape[1], _ptr(X), nrhs)
    return X.ravel() if vec else X


def residual(A, X, B, trans: bool = False):
    """R = B - op(A) X in FP64 (Algorithm 1 step 4)."""
    A = _c(A, np.float64)
    X2, vec = _as2d(X)
    B2, _ = _as2d(B)
    X2 = _c(X2, np.float64)
    B2 = _c(B2, np.float64)
    n, nrhs = X2.shape
    R = np.empty((n, nrhs), dtype=np.float64)
    _load().orc_residual(n, nrhs, _ptr(A), A.shape[1], _ptr(X2), nrhs, _ptr(B2), nrhs,
                         _ptr(R), nrhs, int(trans))
    return R.ravel() if vec else R


def residual_ld(A, X, B):
    """Per right-hand side: (||b - A x||_inf, componentwise backward error),
    both accumulated in extended precision."""
    A = _c(A, np.float64)
    X2, _ = _as2d(X)
    B2, _ = _as2d(B)
    X2 = _c(X2, np.float64)
    B2 = _c(B2, np.float64)
    n, nrhs = X2.shape
    rn = np.empty(nrhs)
    cb = np.empty(nrhs)
    _load().orc_residual_ld(n, nrhs, _ptr(A), A.shape[1], _ptr(X2), nrhs, _ptr(B2), nrhs,
                            _ptr(rn), _ptr(cb))
    return rn, cb


@dataclass
class IRResult:
    x: np.ndarray
    iters: int  # >= 0 corrections applied; -(itermax+1) no convergence; -1 zero pivot
    info: int


def gesv_ir(A, B, lowp: bool = False, trans: bool = False, itermax: int = ITERMAX) -> IRResult:
    """Iterative refinement (Algorithm 1).  lowp=False: FP64 factors (the
    reference solve).  lowp=True: FP32 factor and solves, FP64 residual and
    update with the original A (Algorithm 1 as printed)."""
    if lowp and trans:
        raise ValueError("the single-precision variant has no transposed mode")
    A = _c(A, np.float64)
    B2, vec = _as2d(B)
    B2 = _c(B2, np.float64)
    n, nrhs = B2.shape
    X = np.zeros((n, nrhs), dtype=np.float64)
    it = ctypes.c_int(0)
    info = _load().orc_gesv_ir(n, nrhs, _ptr(A), A.shape[1], _ptr(B2), nrhs, _ptr(X), nrhs,
                               itermax, int(lowp), int(trans), ctypes.byref(it))
    return IRResult(X.ravel() if vec else X, it.value, info)


def posv_ir(A, B, lowp: bool = False, itermax: int = ITERMAX) -> IRResult:
    """Cholesky-based refinement (SPOTRF/SPOTRS + DSYMM residual)."""
    A = _c(A, np.float64)
    B2, vec = _as2d(B)
    B2 = _c(B2, np.float64)
    n, nrhs = B2.shape
    X = np.zeros((n, nrhs), dtype=np.float64)
    it = ctypes.c_int(0)
    info = _load().orc_posv_ir(n, nrhs, _ptr(A), A.shape[1], _ptr(B2), nrhs, _ptr(X), nrhs,
                               itermax, int(lowp), ctypes.byref(it))
    return IRResult(X.ravel() if vec else X, it.value, info)


def stopping_threshold(n: int, anorm: float, xnorm: float) -> float:
    """sqrt(n) * 2^-53 * ||A||_inf * ||x||_inf (Section 3, infinity norms)."""
    return float(np.sqrt(n)) * EPS_D * anorm * xnorm


def metrics(A, x, b, x_ref=None, x_true=None) -> dict:
    """Reported accuracy figures for one solve.

    * ``rnorm``: ||b - A x||_inf in extended precision;
    * ``nbe``: normwise backward error rnorm / (||A|| ||x|| + ||b||);
    * ``cbe``: componentwise backward error max_i |r_i| / (|A||x| + |b|)_i;
    * ``passes``: the stopping rule holds (extended-precision residual);
    * ``fwd_ref`` / ``fwd_true``: ||x - x_ref|| / ||x_ref|| (infinity norms).
    """
    A = _c(A, np.float64)
    X2, _ = _as2d(x)
    B2, _ = _as2d(b)
    n = A.shape[0]
    rn, cb = residual_ld(A, X2, B2)
    an = norm_inf(A)
    xn = np.abs(X2).max(axis=0) if n else np.zeros(X2.shape[1])
    bn = np.abs(B2).max(axis=0) if n else np.zeros(X2.shape[1])
    out = {
        "rnorm": rn,
        "anorm": an,
        "xnorm": xn,
        "nbe": rn / np.maximum(an * xn + bn, np.finfo(float).tiny),
        "cbe": cb,
        "passes": bool(np.all(rn <= np.sqrt(n) * EPS_D * an * xn)),
    }
    for key, ref in (("fwd_ref", x_ref), ("fwd_true", x_true)):
        if ref is not None:
            R2, _ = _as2d(ref)
            d = np.abs(X2 - R2).max(axis=0)
            out[key] = d / np.maximum(np.abs(R2).max(axis=0), np.finfo(float).tiny)
    return out


def norm_1(A) -> float:
    """||A||_1: the largest column sum of |a_ij|."""
    return float(np.abs(np.asarray(A, dtype=np.float64)).sum(axis=0).max()) if np.size(A) else 0.0


def condest1(A, itmax: int = 5) -> float:
    """Estimate of kappa_1(A) = ||A||_1 ||A^{-1}||_1 by Hager's method with
    Higham's refinement (the scheme of LAPACK's xGECON), every solve by the
    FP64 factors of ``getrf``.  In the method's order: x = (1/n, ..., 1/n);
    y = A^{-1} x; xi = sign(y) with sign(0) = +1; z = A^{-T} xi; stop when
    ||z||_inf <= z^T x or the new vertex repeats the last one, else x = e_j
    at the first index j of the largest |z_j|; at most ``itmax`` sweeps,
    keeping the largest ||y||_1.  Then Higham's alternating vector
    v_i = (-1)^i (1 + i/(n-1)) gives 2 ||A^{-1} v||_1 / (3n), and the
    estimate of ||A^{-1}||_1 is the larger of the two."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if n == 0:
        return 0.0
    a1 = norm_1(A)
    LU, ipiv, info = getrf(A)
    if info:
        return float("inf")
    x = np.full(n, 1.0 / n)
    est = 0.0
    jprev = -1
    for _ in range(itmax):
        y = getrs(LU, ipiv, x)
        est = max(est, float(np.abs(y).sum()))
        xi = np.where(y >= 0.0, 1.0, -1.0)
        z = getrs(LU, ipiv, xi, trans=True)
        zinf = float(np.abs(z).max())
        j = int(np.argmax(np.abs(z)))  # first index among equal maxima
        if zinf <= float(z @ x) or j == jprev:
            break
        jprev = j
        x = np.zeros(n)
        x[j] = 1.0
    i = np.arange(n)
    v = np.where(i % 2 == 1, -1.0, 1.0) * (1.0 + (i / (n - 1) if n > 1 else 0.0))
    alt = 2.0 * float(np.abs(getrs(LU, ipiv, v)).sum()) / (3.0 * n)
    return a1 * max(est, alt)


"""GPU tests of the FP64 residual behind the stopping test of Section 3
(||r||_inf <= sqrt(n) 2^-53 ||A||_inf ||x||_inf), through the C ABI.

The certificate is only as good as the residual it is evaluated on: an
ordinary FP64 sum of n products carries rounding up to about
n 2^-53 sum_j |a_ij x_j|, the same size as the threshold itself.  The
residual kernels accumulate compensated sums (products split exactly by an
FMA, additions by TwoSum), so the ||r||_inf a report carries must equal the
exact residual norm of the returned x, computed here in rational arithmetic,
to a few units in the last place.  Cases: the one-shot solve, the transposed
refinement of the adjoint, and the batched kernel, each on small systems
(where the threshold is tightest) and on near-cancelling right-hand sides.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact
from synth import gen

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def solver():
    import torch

    from paper_0808_2794_amd import mixlu

    torch.cuda.init()
    s = mixlu.Solver()
    yield s
    s.close()


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _exact_rnorm(A, x, b):
    r = exact.residual(A.tolist(), [float(v) for v in x], [float(v) for v in b])
    return float(max(abs(v) for v in r)) if r else 0.0


def _check(rep_rnorm, exact_rnorm, what):
    # the reported norm is the compensated residual rounded once: within a
    # few ulps of the exact value (an uncompensated sum misses by O(1) here)
    tol = 8 * U * exact_rnorm + 1e-300
    assert abs(rep_rnorm - exact_rnorm) <= tol, (what, rep_rnorm, exact_rnorm)


@pytest.mark.parametrize("n", [2, 3, 5, 17, 40])
def test_dxgesv_reported_residual_is_exact(solver, n):
    from paper_0808_2794_amd import mixlu

    for seed in range(6):
        A, b, _ = gen.prescribed_cond_system(n, 10.0 ** (seed % 4), 900 + 10 * n + seed)
        _say(f"residual dxgesv n={n} seed={seed}")
        r = solver.dxgesv(_dev(A), _dev(b), "fp32", mixlu.default_opts(equilibrate=0))
        assert r.report["converged"], r.report
        x = r.x.cpu().numpy().reshape(-1)
        _check(r.report["rnorm"], _exact_rnorm(A, x, b.reshape(-1)), ("dxgesv", n, seed))


@pytest.mark.parametrize("n", [2, 7, 33])
def test_transposed_refine_reported_residual_is_exact(solver, n):
    """A^T g = w through mixlu_refine(trans=1), as the adjoint calls it."""
    import torch

    from paper_0808_2794_amd import mixlu

    for seed in range(4):
        A, _, _ = gen.prescribed_cond_system(n, 100.0, 950 + n + seed)
        w = np.random.default_rng(seed).standard_normal((n, 1))
        Ad, Wd = _dev(A), _dev(w)
        o = mixlu.default_opts()
        nbytes = mixlu.mixlu_workspace_size(solver.ctx, mixlu.OP_GESV, mixlu.FP32, n, 1, o)
        work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
        F, info = mixlu.mixlu_getrf(solver.ctx, mixlu.FP32, Ad, work, o)
        assert info == 0
        G = torch.empty_like(Wd)
        mixlu.mixlu_getrs(solver.ctx, F, Wd, G, trans=1)
        _say(f"residual transposed refine n={n} seed={seed}")
        rep = mixlu.mixlu_refine(solver.ctx, F, Ad, Wd, G, o, trans=1).as_dict()
        assert rep["converged"], rep
        g = G.cpu().numpy().reshape(-1)
        _check(rep["rnorm"], _exact_rnorm(A.T.copy(), g, w.reshape(-1)), ("transposed", n, seed))


def test_batched_reported_residual_is_exact(solver):
    sizes = [1, 2, 2, 3, 4, 9, 16, 31, 48]
    g = np.random.default_rng(77)
    systems = []
    for n in sizes:
        A, b, _ = gen.prescribed_cond_system(n, float(10 ** g.integers(0, 5)), g)
        systems.append((A, b))
    _say("residual batched")
    Xs, reps = solver.dxgesv_batched([_dev(A) for A, _ in systems], [_dev(b) for _, b in systems],
                                     "fp32")
    for i, ((A, b), X, rep) in enumerate(zip(systems, Xs, reps)):
        assert rep["converged"], (i, rep)
        x = X.cpu().numpy().reshape(-1)
        _check(rep["rnorm"], _exact_rnorm(A, x, b.reshape(-1)), ("batched", i, A.shape[0]))


def test_cancelling_right_hand_side(solver):
    """b = A x_true with x_true of mixed signs and widely different sizes, so
    the products of each row cancel to a small residual: the case where an
    uncompensated sum's rounding dominates."""
    from paper_0808_2794_amd import mixlu

    n = 24
    rng = np.random.default_rng(5)
    A = rng.uniform(-1, 1, (n, n))
    xt = rng.uniform(-1, 1, n) * np.exp2(rng.integers(-20, 20, n))
    b = np.array([float(sum(Fraction(A[i, j]) * Fraction(xt[j]) for j in range(n)))
                  for i in range(n)]).reshape(n, 1)
    _say("residual cancelling rhs")
    r = solver.dxgesv(_dev(A), _dev(b), "fp32", mixlu.default_opts(equilibrate=0))
    x = r.x.cpu().numpy().reshape(-1)
    _check(r.report["rnorm"], _exact_rnorm(A, x, b.reshape(-1)), "cancelling")

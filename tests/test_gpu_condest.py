"""GPU parity of the kappa_1 estimate (Hager's method with Higham's
refinement, solves by the stored factors) against the oracle's estimate,
and of the option that uses it to skip a refinement that cannot converge
(Section 4: kappa eps_s must stay below about one).

With FP64 factors both sides take the same decisions (sign vectors, the
vertex e_j), so the estimates agree to rounding: relative 1e-9.  With
FP32 factors the solves carry relative error ~ kappa 2^-24, so the
estimates agree to 1e-3 at kappa <= 1e4.
"""
import numpy as np
import pytest

from oracle import oracle as O
from synth import gen

pytestmark = pytest.mark.gpu


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


def _gpu_condest(solver, A, prec, kind="lu", equil=0):
    from paper_0808_2794_amd import mixlu

    n = A.shape[0]
    o = mixlu.default_opts(equilibrate=equil)
    op = mixlu.OP_GESV if kind == "lu" else mixlu.OP_POSV
    work = solver.workspace(op, mixlu.PREC[prec], n, 1, o)
    fac = mixlu.mixlu_getrf if kind == "lu" else mixlu.mixlu_potrf
    F, info = fac(solver.ctx, mixlu.PREC[prec], _dev(A), work, o)
    assert info == 0 and F.lowp_status == 0
    return mixlu.mixlu_condest(solver.ctx, F)


@pytest.mark.parametrize("n,kappa", [(1, 1.0), (17, 1e2), (200, 1e4), (700, 1e6), (1100, 1e3)])
def test_condest_fp64_factors_match_oracle(solver, n, kappa):
    A, _, _ = gen.prescribed_cond_system(n, kappa, 700 + n)
    _say(f"condest fp64 n={n} kappa={kappa:g}")
    est = _gpu_condest(solver, A, "fp64")
    ref = O.condest1(A)
    assert est == pytest.approx(ref, rel=1e-9), (est, ref)


def test_condest_closed_forms(solver):
    """Diagonal A: max|d| / min|d| exactly; the bidiagonal I - 2N of order 40:
    3 (2^40 - 1)."""
    g = np.random.default_rng(8)
    d = g.uniform(0.5, 2.0, 300)
    d[123] = 1e-6
    _say("condest diagonal")
    assert _gpu_condest(solver, np.diag(d), "fp64") == pytest.approx(d.max() / d.min(), rel=1e-12)
    n = 40
    A = np.eye(n) - 2.0 * np.eye(n, k=1)
    _say("condest bidiagonal")
    assert _gpu_condest(solver, A, "fp64") == pytest.approx(3.0 * (2.0 ** n - 1.0), rel=1e-12)


@pytest.mark.parametrize("n,kappa", [(300, 1e2), (1000, 1e4)])
def test_condest_fp32_factors(solver, n, kappa):
    A, _, _ = gen.prescribed_cond_system(n, kappa, 710 + n)
    _say(f"condest fp32 n={n} kappa={kappa:g}")
    est = _gpu_condest(solver, A, "fp32")
    ref = O.condest1(A)
    assert est == pytest.approx(ref, rel=1e-3), (est, ref)


def test_condest_cholesky_factor(solver):
    A, _, _ = gen.spd_system(500, 1e3, 77)
    _say("condest cholesky fp64")
    est = _gpu_condest(solver, A, "fp64", kind="chol")
    assert est == pytest.approx(O.condest1(A), rel=1e-9)


def test_condest_option_routes_to_fp64(solver):
    """opts.condest: FP16 factors at kappa = 1e5 (kappa eps_s ~ 49) go
    straight to the FP64 path (iter = -5) and still give an FP64-accurate x;
    FP32 factors at kappa = 1e3 keep the low-precision refinement.  The
    report carries the estimate."""
    from paper_0808_2794_amd import mixlu

    for prec, kappa, expect_skip in (("fp16", 1e5, True), ("fp32", 1e3, False)):
        A, b, _ = gen.prescribed_cond_system(600, kappa, 720)
        _say(f"dxgesv condest prec={prec} kappa={kappa:g}")
        r = solver.dxgesv(_dev(A), _dev(b), prec, opts=mixlu.default_opts(condest=1))
        rep = r.report
        ref = O.condest1(A)
        if expect_skip:
            # the FP16-operand factor is too coarse for an accurate estimate;
            # what counts is that it rules the low precision out
            assert rep["cond_est"] * 2.0 ** -11 >= 1.0, (rep, ref)
            assert rep["iter"] == -5 and rep["prec"] == "fp64", rep
        else:
            assert rep["cond_est"] == pytest.approx(ref, rel=1e-2), (rep, ref)
            assert rep["iter"] >= 0 and rep["prec"] == prec, rep
        assert rep["converged"], rep
        x = r.x.cpu().numpy()
        m = O.metrics(A, x, b, x_ref=O.gesv_ir(A, b).x)
        assert m["passes"] and float(np.max(m["fwd_ref"])) <= 1e-12 * kappa


def test_condest_empty_system(solver):
    """n = 0: the estimate is 0 (nothing to invert)."""
    import torch

    from paper_0808_2794_amd import mixlu

    o = mixlu.default_opts()
    work = solver.workspace(mixlu.OP_GESV, mixlu.FP32, 0, 1, o)
    A = torch.zeros((0, 0), dtype=torch.float64, device="cuda")
    F, info = mixlu.mixlu_getrf(solver.ctx, mixlu.FP32, A, work, o)
    assert info == 0
    assert mixlu.mixlu_condest(solver.ctx, F) == 0.0

"""GPU parity of the flexible GMRES refinement (the outer FGMRES of
Algorithm 2 with the low-precision LU solve as preconditioner) against the
CPU oracle, through the C ABI.

Same bar as the stationary refinement: the stopping rule for the returned x
with the residual recomputed on the CPU in extended precision, and the
forward error against the oracle's FP64 solve within 1e-12 kappa.  The
cases are those where the stationary iteration of Algorithm 1 stalls
(kappa eps_s near or above 1): here they must finish in the low precision,
without the FP64 fallback.
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


@pytest.mark.parametrize("n,kappa,prec", [(1, 1.0, "fp16"), (17, 1e2, "fp16"), (700, 1e3, "bf16"),
                                          (1100, 1e4, "fp16"), (600, 1e3, "fp16"),
                                          (900, 1e6, "fp32"), (300, 2.0, "fp8"),
                                          (200, 10.0, "fp8")])
def test_fgmres_low_precision_factors(solver, n, kappa, prec):
    from paper_0808_2794_amd import mixlu

    A, b, _ = gen.prescribed_cond_system(n, kappa, 800 + n)
    _say(f"fgmres n={n} kappa={kappa:g} prec={prec}")
    r = solver.dxgesv(_dev(A), _dev(b), prec, refine=mixlu.REFINE_FGMRES)
    ref = O.gesv_ir(A, b)
    m = O.metrics(A, r.x.cpu().numpy(), b, x_ref=ref.x)
    assert m["passes"], (r.report, m["rnorm"])
    assert float(np.max(m["fwd_ref"])) <= 1e-12 * kappa, m["fwd_ref"]
    _say(f"  report {r.report}")
    assert r.report["converged"] and r.report["prec"] == prec and r.report["iter"] >= 0, r.report


def test_fgmres_matches_classic_where_both_converge(solver):
    """FP32 factor, kappa = 1e2: both refinements reach the same x to the
    stopping tolerance, FGMRES with no more preconditioner applications than
    the stationary iteration's corrections plus one cycle."""
    from paper_0808_2794_amd import mixlu

    n = 800
    A, b, _ = gen.prescribed_cond_system(n, 1e2, 81)
    _say("fgmres vs classic fp32")
    r1 = solver.dxgesv(_dev(A), _dev(b), "fp32")
    r2 = solver.dxgesv(_dev(A), _dev(b), "fp32", refine=mixlu.REFINE_FGMRES)
    assert r1.report["converged"] and r2.report["converged"]
    x1, x2 = r1.x.cpu().numpy(), r2.x.cpu().numpy()
    assert np.abs(x1 - x2).max() <= 1e-13 * 1e2 * np.abs(x1).max()
    assert r2.report["iter"] <= r1.report["iter"] + 30


def test_fgmres_multi_rhs_uses_classic(solver):
    """Several right-hand sides take the stationary refinement (FGMRES is for
    one right-hand side); the answer is still FP64-accurate."""
    from paper_0808_2794_amd import mixlu

    n = 300
    A, b, _ = gen.prescribed_cond_system(n, 1e2, 83, nrhs=3)
    _say("fgmres option with 3 rhs")
    r = solver.dxgesv(_dev(A), _dev(b), "fp32", refine=mixlu.REFINE_FGMRES)
    ref = O.gesv_ir(A, b)
    m = O.metrics(A, r.x.cpu().numpy(), b, x_ref=ref.x)
    assert m["passes"] and r.report["converged"]


def test_history_matches_report(solver):
    """The residual history of a stationary refinement has one entry per
    iteration (the corrections plus the final test), ending at the reported
    residual; FGMRES records one entry per restart cycle."""
    from paper_0808_2794_amd import mixlu

    n = 500
    A, b, _ = gen.prescribed_cond_system(n, 1e3, 85)
    _say("history classic fp32")
    r = solver.dxgesv(_dev(A), _dev(b), "fp32")
    h = mixlu.mixlu_refine_history(solver.ctx)
    assert r.report["converged"] and r.report["prec"] == "fp32", r.report
    assert len(h) == r.report["iter"] + 1 and h[-1] == r.report["rnorm"], (h, r.report)
    _say("history fgmres fp16")
    o = mixlu.default_opts(refine=mixlu.REFINE_FGMRES)
    o.restart = 8
    r = solver.dxgesv(_dev(A), _dev(b), "fp16", o)
    h = mixlu.mixlu_refine_history(solver.ctx)
    assert r.report["converged"] and r.report["prec"] == "fp16", r.report
    assert h[-1] == r.report["rnorm"] and len(h) >= 2, (h, r.report)
    # at most `restart` preconditioner applications per completed cycle
    assert r.report["iter"] <= 8 * (len(h) - 1), (h, r.report)


@pytest.mark.parametrize("prec,kappa,seed", [("fp16", 1e3, 231), ("bf16", 1e2, 232)])
def test_fgmres_n8192(solver, prec, kappa, seed):
    """Benchmarked size, kappa eps_s near 1/2: FGMRES finishes in the low
    precision (no fallback), the answer meets the stopping rule with the
    residual recomputed on the CPU and agrees with the oracle's FP64 solve."""
    import torch

    from paper_0808_2794_amd import mixlu

    n = 8192
    _say(f"fgmres n={n} {prec} kappa={kappa:g}: generate")
    Ad, bd, x_true = gen.prescribed_cond_system(n, kappa, seed, backend="torch", device="cuda")
    _say("solve")
    r = solver.dxgesv(Ad, bd, prec, refine=mixlu.REFINE_FGMRES)
    torch.cuda.synchronize()
    h = mixlu.mixlu_refine_history(solver.ctx)
    _say(f"  report {r.report} history {h}")
    assert r.report["converged"] and r.report["prec"] == prec, (r.report, h)
    A, b, x = Ad.cpu().numpy(), bd.cpu().numpy(), r.x.cpu().numpy()
    del Ad, bd
    _say("oracle")
    ref = O.gesv_ir(A, b)
    m = O.metrics(A, x, b, x_ref=ref.x, x_true=x_true)
    assert m["passes"], m["rnorm"]
    assert float(np.max(m["fwd_ref"])) <= 1e-12 * kappa, m["fwd_ref"]


def test_fgmres_no_progress_ends_in_fallback(solver):
    """kappa eps_s = 5 (FP16 operands, kappa = 1e4, n = 4096): the restart
    cycles stop cutting the residual; two cycles in a row with less than 1%
    progress end the iteration well before itermax, and the FP64 fallback
    returns a certified answer."""
    import torch

    from paper_0808_2794_amd import mixlu

    n = 4096
    _say(f"fgmres stall n={n} fp16 kappa=1e4")
    Ad, bd, x_true = gen.prescribed_cond_system(n, 1e4, 233, backend="torch", device="cuda")
    o = mixlu.default_opts(refine=mixlu.REFINE_FGMRES)
    o.itermax = 30
    r = solver.dxgesv(Ad, bd, "fp16", o)
    torch.cuda.synchronize()
    h = mixlu.mixlu_refine_history(solver.ctx)
    _say(f"  report {r.report} history {h}")
    if r.report["prec"] == "fp16":  # converged after all: must then be certified
        assert r.report["converged"], r.report
    else:
        assert r.report["prec"] == "fp64" and r.report["iter"] == -4 and r.report["converged"]
        lp = h[:-(r.report["fallback_iter"] + 1)]  # the FGMRES cycles
        assert 3 <= len(lp) < 30, h
        assert not (lp[-1] < 0.99 * lp[-2]) and not (lp[-2] < 0.99 * lp[-3]), lp
    x = r.x.cpu().numpy()
    fwd = np.abs(x - x_true).max() / np.abs(x_true).max()
    assert fwd <= 1e-12 * 1e4, fwd

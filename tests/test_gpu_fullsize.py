"""GPU parity at the benchmarked sizes, through the C ABI, in the launch
configuration the benchmark times (default options, one solve call).

* dense nonsymmetric n = 8192, A = U diag(sigma) V^T: FP32 factor at
  kappa = 1e4, FP16 trailing-update operands at kappa = 1e2 and the FP64
  factor at kappa = 1e4, each against
  the oracle's FP64 refinement (G2: forward error <= 1e-12 kappa) and the
  stopping test of Section 3 with the residual recomputed on the CPU in
  extended precision (G1);
* SPD n = 8192, 16 right-hand sides, Cholesky with FP16 operands at
  kappa = 1e3, against the oracle's FP64 Cholesky refinement;
* the headline solve, n = 16384, kappa = 1e4, FP32 factor: G1 in extended
  precision and the error against the planted solution (<= 1e-12 kappa);
  the oracle's own solve at this size takes minutes and is not run.

Inputs are generated on the GPU (QR by the device library) and copied to the
host, so the oracle and the HIP path see the same bytes.
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
    torch.cuda.empty_cache()


def _g1_g2(A, b, x, kappa, x_ref=None, x_true=None):
    m = O.metrics(A, x, b, x_ref=x_ref, x_true=x_true)
    assert m["passes"], f"stopping rule fails: rnorm={m['rnorm']} anorm={m['anorm']} xnorm={m['xnorm']}"
    if x_ref is not None:
        assert float(np.max(m["fwd_ref"])) <= 1e-12 * kappa, m["fwd_ref"]
    if x_true is not None:
        assert float(np.max(m["fwd_true"])) <= 1e-12 * kappa, m["fwd_true"]
    return m


@pytest.mark.parametrize("prec,kappa,seed", [("fp32", 1e4, 212), ("fp16", 1e2, 211),
                                             ("fp64", 1e4, 213)])
def test_dense_n8192(solver, prec, kappa, seed):
    import torch

    n = 8192
    _say(f"dense n={n} {prec} kappa={kappa:g} seed={seed}: generate")
    Ad, bd, x_true = gen.prescribed_cond_system(n, kappa, seed, backend="torch", device="cuda")
    _say("solve")
    r = solver.dxgesv(Ad, bd, prec)
    torch.cuda.synchronize()
    assert r.report["converged"] and r.report["prec"] == prec, r.report
    A = Ad.cpu().numpy()
    b = bd.cpu().numpy()
    x = r.x.cpu().numpy()
    del Ad, bd
    _say("oracle")
    ref = O.gesv_ir(A, b)
    assert ref.info == 0 and ref.iters >= 0
    _g1_g2(A, b, x, kappa, x_ref=ref.x, x_true=x_true)


def test_spd_n8192_16rhs_fp16(solver):
    import torch

    n, kappa, nrhs = 8192, 1e3, 16
    _say(f"spd n={n} nrhs={nrhs} fp16: generate")
    Ad, Bd, X_true = gen.spd_system(n, kappa, 301, nrhs=nrhs, backend="torch", device="cuda")
    _say("solve")
    r = solver.dxposv(Ad, Bd, "fp16")
    torch.cuda.synchronize()
    assert r.report["converged"] and r.report["prec"] == "fp16", r.report
    A = Ad.cpu().numpy()
    B = Bd.cpu().numpy()
    X = r.x.cpu().numpy()
    del Ad, Bd
    _say("oracle")
    ref = O.posv_ir(A, B)
    assert ref.info == 0 and ref.iters >= 0
    _g1_g2(A, B, X, kappa, x_ref=ref.x, x_true=X_true)


def test_headline_n16384_fp32(solver):
    import torch

    n, kappa, seed = 16384, 1e4, 221
    _say(f"headline n={n} fp32 kappa={kappa:g}: generate")
    Ad, bd, x_true = gen.prescribed_cond_system(n, kappa, seed, backend="torch", device="cuda")
    _say("solve")
    r = solver.dxgesv(Ad, bd, "fp32")
    torch.cuda.synchronize()
    assert r.report["converged"] and r.report["prec"] == "fp32", r.report
    x = r.x.cpu().numpy()
    b = bd.cpu().numpy()
    A = Ad.cpu().numpy()
    del Ad, bd
    torch.cuda.empty_cache()
    _say("extended-precision residual")
    _g1_g2(A, b, x, kappa, x_true=x_true)

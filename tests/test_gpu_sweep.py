"""The iterations-against-kappa experiment of Section 4 on the batched
solver (reduced: 40 systems of order 200 per kappa), checked against the
oracle's Algorithm 1 on the same systems and against the generalized Datta
bound."""
import numpy as np
import pytest

from oracle import oracle as O

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


def test_sweep_fp32_matches_oracle_and_bound(solver):
    """FP32 factors: every system converges for kappa <= 1e5, the mean
    number of solves lies between the kappa -> 1 limit (3) and the Datta
    bound, grows with kappa, and is within one solve of the oracle's
    Algorithm 1 (unblocked FP32 LU) on the same systems."""
    from paper_0808_2794_amd import sweep

    means = []
    for kappa in (1e1, 1e3, 1e5):
        _say(f"sweep fp32 kappa={kappa:g}")
        row = sweep.sweep(solver, "fp32", kappa, count=40, n=200, seed=5)
        assert row["converged"] == 40, row
        assert 3 <= row["mean_solves"] <= row["datta_bound"], row
        ref = [O.gesv_ir(A, b, lowp=True).iters + 1 for A, b in sweep.systems(kappa, 40, 200, 5)]
        assert abs(row["mean_solves"] - float(np.mean(ref))) <= 1.0, (row, np.mean(ref))
        means.append(row["mean_solves"])
    assert means == sorted(means) and means[-1] > means[0]


def test_sweep_failure_above_one(solver):
    """kappa eps_s well above one: the low-precision refinement fails for
    (nearly) every system, FP32 at kappa = 1e9 and FP16 at kappa = 1e6;
    FP16 at kappa = 10 converges for all."""
    from paper_0808_2794_amd import sweep

    for prec, kappa, want in (("fp32", 1e9, "fail"), ("fp16", 1e6, "fail"), ("fp16", 1e1, "ok")):
        _say(f"sweep {prec} kappa={kappa:g}")
        row = sweep.sweep(solver, prec, kappa, count=40, n=200, seed=6)
        if want == "fail":
            assert row["converged"] <= 4, row
            assert row["datta_bound"] is None
        else:
            assert row["converged"] == 40, row

"""GPU test of mixlu_dxgesv_batched_noalloc (the batched solve whose queue
and factor slots live in the library's device array instead of a caller
workspace) against mixlu_dxgesv_batched on the same systems, through the C
ABI: two calls in a row, the second on a smaller batch, each bit for bit
equal to the workspace call (the same per-system kernels run on each
system, only the number of persistent workgroups differs), and each
system's solution checked against the oracle's.  Also the argument and
batch-limit errors, which touch no device memory.
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


def _systems(count, seed, nmax=512):
    g = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(g.integers(16, nmax + 1))
        kappa = float(np.exp(g.uniform(np.log(1e1), np.log(1e5))))
        A, b, _ = gen.prescribed_cond_system(n, kappa, g)
        out.append((A, b, kappa))
    return out


def _solve_both(solver, systems, prec):
    import torch

    from paper_0808_2794_amd import mixlu

    As = [_dev(A) for A, _, _ in systems]
    Bs = [_dev(b) for _, b, _ in systems]
    ref = solver.batched_buffers(As, Bs, prec)
    solver.run_batched(ref)
    na = solver.batched_buffers(As, Bs, prec)
    for X in na["X"]:
        X.fill_(-3.0)
    mixlu.mixlu_dxgesv_batched_noalloc(solver.ctx, na["prec"], na["n"], na["pA"], None, na["pB"],
                                       na["pX"], na["nrhs"], na["reps"], na["opts"])
    torch.cuda.synchronize()
    return ref, na


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_noalloc_matches_workspace_call_twice(solver, prec):
    from paper_0808_2794_amd import mixlu

    for call, (count, seed) in enumerate([(70, 811), (23, 812)]):
        systems = _systems(count, seed)
        _say(f"noalloc batched {prec} call {call}: {count} systems")
        ref, na = _solve_both(solver, systems, prec)
        reps_ref = mixlu.reports_from_bytes(bytes(ref["reps"].cpu().numpy()))
        reps_na = mixlu.reports_from_bytes(bytes(na["reps"].cpu().numpy()))
        assert reps_na == reps_ref
        for i, (A, b, kappa) in enumerate(systems):
            x_ref = ref["X"][i].cpu().numpy()
            x_na = na["X"][i].cpu().numpy()
            assert np.array_equal(x_na, x_ref), (call, i, A.shape[0])
            assert reps_na[i]["converged"], (call, i, reps_na[i])
            if i % 7 == 0:  # the oracle on a sample of the systems
                m = O.metrics(A, x_na, b, x_ref=O.gesv_ir(A, b).x)
                assert m["passes"] and float(np.max(m["fwd_ref"])) <= 1e-12 * kappa, (call, i)


def test_noalloc_argument_errors(solver):
    import ctypes

    import torch

    from paper_0808_2794_amd import mixlu

    lib = mixlu.load()
    rep = torch.zeros(ctypes.sizeof(mixlu.mixlu_report), dtype=torch.uint8, device="cuda")
    n = torch.ones(1, dtype=torch.int32, device="cuda")
    ptr = torch.zeros(1, dtype=torch.int64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    # empty batch: nothing to do
    assert lib.mixlu_dxgesv_batched_noalloc(solver.ctx, mixlu.FP32, 0, None, None, None, None,
                                            None, 1, None, None) == 0
    # a null pointer array, nrhs < 1, FP8, a batch beyond the array's limit
    assert lib.mixlu_dxgesv_batched_noalloc(solver.ctx, mixlu.FP32, 1, p(n), None, None, p(ptr),
                                            p(ptr), 1, None, p(rep)) == -5
    assert lib.mixlu_dxgesv_batched_noalloc(solver.ctx, mixlu.FP32, 1, p(n), p(ptr), None, p(ptr),
                                            p(ptr), 0, None, p(rep)) == -9
    assert lib.mixlu_dxgesv_batched_noalloc(solver.ctx, mixlu.FP8, 1, p(n), p(ptr), None, p(ptr),
                                            p(ptr), 1, None, p(rep)) == mixlu.ERR_NOT_IMPLEMENTED
    assert lib.mixlu_dxgesv_batched_noalloc(solver.ctx, mixlu.FP32, 65537, p(n), p(ptr), None,
                                            p(ptr), p(ptr), 1, None, p(rep)) == mixlu.ERR_WORKSPACE

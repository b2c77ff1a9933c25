"""GPU tests of the stream-ordered factorizations (mixlu_getrf_async,
mixlu_potrf_async), through the C ABI: the same factors as the synchronous
calls (solves with them agree bit for bit), the outcome written to device
memory with the codes of the synchronous calls, refinement on a factor whose
outcome is still pending, and a single-system factorization and solve
captured in a HIP graph whose replays reproduce the eager result bit for
bit, with eager work and synchronizations between the replays.
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


def _work(solver, op, prec, n, nrhs=1):
    import torch

    from paper_0808_2794_amd import mixlu

    nbytes = mixlu.mixlu_workspace_size(solver.ctx, op, prec, n, nrhs)
    return torch.zeros(max(nbytes, 256), dtype=torch.uint8, device="cuda")


def _info_dev():
    import torch

    return torch.full((1,), 12345, dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("n,prec", [(300, "fp32"), (1100, "fp32"), (1100, "fp16"), (700, "fp64")])
def test_getrf_async_matches_sync(solver, n, prec):
    import torch

    from paper_0808_2794_amd import mixlu

    p = mixlu.PREC[prec]
    A, b, _ = gen.prescribed_cond_system(n, 1e2, 610 + n)
    Ad, bd = _dev(A), _dev(b)
    w1, w2 = _work(solver, mixlu.OP_GESV, p, n), _work(solver, mixlu.OP_GESV, p, n)
    _say(f"getrf sync/async n={n} {prec}")
    F1, info = mixlu.mixlu_getrf(solver.ctx, p, Ad, w1)
    d_info = _info_dev()
    F2 = mixlu.mixlu_getrf_async(solver.ctx, p, Ad, w2, d_info)
    assert F2.lowp_status == mixlu.FACTOR_PENDING
    X1, X2 = torch.empty_like(bd), torch.empty_like(bd)
    mixlu.mixlu_getrs(solver.ctx, F1, bd, X1)
    mixlu.mixlu_getrs(solver.ctx, F2, bd, X2)
    torch.cuda.synchronize()
    assert info == 0 and int(d_info.item()) == 0
    assert torch.equal(X1, X2)
    # refinement on the pending factor reads the outcome itself
    o = mixlu.default_opts()
    r1 = mixlu.mixlu_refine(solver.ctx, F1, Ad, bd, X1, o).as_dict()
    r2 = mixlu.mixlu_refine(solver.ctx, F2, Ad, bd, X2, o).as_dict()
    assert F2.lowp_status == 0
    assert r1 == r2 and r2["converged"] and r2["prec"] == prec, (r1, r2)
    assert torch.equal(X1, X2)
    ref = O.gesv_ir(A, b)
    m = O.metrics(A, X2.cpu().numpy(), b, x_ref=ref.x)
    assert m["passes"] and float(np.max(m["fwd_ref"])) <= 1e-12 * 1e2


def test_async_outcome_codes(solver):
    """Exact zero pivot of an FP64 factor (k+1, as the synchronous info),
    conversion overflow of an FP16 factor (-2), a non-positive Cholesky
    pivot (-3 for FP32, k+1 for FP64)."""
    import torch

    from paper_0808_2794_amd import mixlu

    n = 200
    rng = np.random.default_rng(3)
    A = rng.uniform(-1, 1, (n, n))
    A[:, 37] = 0.0  # singular: the elimination meets a zero pivot
    Ad = _dev(A)
    _say("async outcome: fp64 singular")
    F1, info = mixlu.mixlu_getrf(solver.ctx, mixlu.FP64, Ad, _work(solver, mixlu.OP_GESV, mixlu.FP64, n))
    d = _info_dev()
    mixlu.mixlu_getrf_async(solver.ctx, mixlu.FP64, Ad, _work(solver, mixlu.OP_GESV, mixlu.FP64, n), d)
    torch.cuda.synchronize()
    assert info > 0 and int(d.item()) == info, (info, int(d.item()))

    n2 = 1100  # the FP16 operands are those of the trailing updates
    B = rng.uniform(-1, 1, (n2, n2))
    B[5] *= 1e7  # row 5 of U12 leaves the FP16 range without equilibration
    assert np.sum(np.abs(B[5, 512:]) > 65504.0) > 100
    o = mixlu.default_opts(equilibrate=0)
    _say("async outcome: fp16 overflow")
    F1, _ = mixlu.mixlu_getrf(solver.ctx, mixlu.FP16, _dev(B),
                              _work(solver, mixlu.OP_GESV, mixlu.FP16, n2), o)
    d = _info_dev()
    mixlu.mixlu_getrf_async(solver.ctx, mixlu.FP16, _dev(B),
                            _work(solver, mixlu.OP_GESV, mixlu.FP16, n2), d, o)
    torch.cuda.synchronize()
    assert F1.lowp_status == -2 and int(d.item()) == -2, (F1.lowp_status, int(d.item()))

    S = np.diag(np.r_[np.ones(10), -np.ones(n - 10)])  # indefinite: pivot 11 is negative
    for prec, want in ((mixlu.FP32, -3), (mixlu.FP64, 11)):
        _say(f"async outcome: potrf indefinite prec={prec}")
        d = _info_dev()
        mixlu.mixlu_potrf_async(solver.ctx, prec, _dev(S), _work(solver, mixlu.OP_POSV, prec, n), d)
        torch.cuda.synchronize()
        assert int(d.item()) == want, (prec, int(d.item()))
    _say("async outcome: empty system")
    d = _info_dev()
    mixlu.mixlu_getrf_async(solver.ctx, mixlu.FP32, _dev(np.zeros((0, 0))),
                            _work(solver, mixlu.OP_GESV, mixlu.FP32, 0), d)
    torch.cuda.synchronize()
    assert int(d.item()) == 0


@pytest.mark.parametrize("op", ["gesv", "posv"])
def test_factor_graph_capture_replay(solver, op):
    """Factorization (two outer blocks, so the second stream takes part) and
    solve captured once; three replays with eager work in between each give
    the eager X bit for bit; new data in the same buffers, replayed, gives
    what an eager call gives on it."""
    import torch

    from paper_0808_2794_amd import mixlu

    n = 1100
    if op == "gesv":
        A, b, _ = gen.prescribed_cond_system(n, 1e3, 620)
        A2, b2, _ = gen.prescribed_cond_system(n, 1e3, 621)
        fac, code = mixlu.mixlu_getrf_async, mixlu.OP_GESV
    else:
        A, b, _ = gen.spd_system(n, 1e3, 622, nrhs=1)
        A2, b2, _ = gen.spd_system(n, 1e3, 623, nrhs=1)
        fac, code = mixlu.mixlu_potrf_async, mixlu.OP_POSV
    Ad, bd = _dev(A), _dev(b)
    Xd = torch.empty_like(bd)
    work = _work(solver, code, mixlu.FP32, n)
    d_info = _info_dev()

    def step():
        F = fac(solver.ctx, mixlu.FP32, Ad, work, d_info)
        mixlu.mixlu_getrs(solver.ctx, F, bd, Xd)

    _say(f"{op} eager reference")
    step()  # also creates the context's second stream and events
    torch.cuda.synchronize()
    eager = Xd.clone()
    assert int(d_info.item()) == 0
    stream = torch.cuda.Stream()
    mixlu.mixlu_set_stream(solver.ctx, stream)
    try:
        g = torch.cuda.CUDAGraph()
        _say(f"{op} capture")
        with torch.cuda.graph(g, stream=stream):
            step()
        for rep in range(3):
            Xd.zero_()
            d_info.fill_(777)
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            _say(f"{op} replay {rep}")
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(Xd, eager), rep
            assert int(d_info.item()) == 0
            del junk
        Ad.copy_(_dev(A2))
        bd.copy_(_dev(b2))
        torch.cuda.synchronize()
        _say(f"{op} replay with new data")
        g.replay()
        torch.cuda.synchronize()
        got = Xd.clone()
    finally:
        mixlu.mixlu_set_stream(solver.ctx, torch.cuda.current_stream())
    step()
    torch.cuda.synchronize()
    assert torch.equal(got, Xd)
    # the low-precision solve of a kappa = 1e3 system: a few digits at least
    ref = np.linalg.solve(A2, b2)
    assert np.abs(got.cpu().numpy() - ref).max() <= 1e-3 * np.abs(ref).max()

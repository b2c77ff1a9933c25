"""GPU parity of the batched solve (one persistent launch over many
independent systems) against the CPU oracle, through the C ABI; HIP-graph
capture and replay of the same launch.

Bar per system: the stopping rule with the residual recomputed on the CPU in
extended precision, and ||x - x_oracle||_inf / ||x_oracle||_inf <=
1e-12 kappa_i.
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


def _systems(sizes, seed):
    g = np.random.default_rng(seed)
    out = []
    for n in sizes:
        kappa = float(np.exp(g.uniform(np.log(1e1), np.log(1e5))))
        A, b, _ = gen.prescribed_cond_system(n, kappa, g)
        out.append((A, b, kappa if n > 1 else 1.0))
    return out


def _check_all(systems, Xs, reps, expect_converged=True):
    for i, ((A, b, kappa), X, rep) in enumerate(zip(systems, Xs, reps)):
        x = X.cpu().numpy()
        ref = O.gesv_ir(A, b)
        m = O.metrics(A, x, b, x_ref=ref.x)
        assert m["passes"], (i, A.shape[0], rep)
        assert float(np.max(m["fwd_ref"])) <= 1e-12 * kappa, (i, A.shape[0], rep, m["fwd_ref"])
        if expect_converged:
            assert rep["converged"], (i, rep)


EDGE = [1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257,
        300, 383, 511, 512]


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp16", "bf16"])
def test_batched_ragged_sizes(solver, prec):
    """Every edge of the 16-column panels, 32-row diagonal blocks and
    128-column update chunks, up to the largest order."""
    systems = _systems(EDGE, 601)
    _say(f"batched ragged sizes prec={prec}")
    Xs, reps = solver.dxgesv_batched([_dev(A) for A, _, _ in systems],
                                     [_dev(b) for _, b, _ in systems], prec)
    _check_all(systems, Xs, reps)
    for rep in reps:
        if prec in ("fp32", "fp64"):
            assert rep["iter"] >= 0 and rep["prec"] == prec, rep


def test_batched_many_rhs_and_order(solver):
    """Three right-hand sides; systems given in increasing size (the queue
    reorders them) and the output lands in the caller's order."""
    g = np.random.default_rng(7)
    sizes = sorted(int(v) for v in g.integers(16, 513, 40))
    systems = []
    for n in sizes:
        A, b, _ = gen.prescribed_cond_system(n, 1e3, g, nrhs=3)
        systems.append((A, b, 1e3))
    _say("batched nrhs=3, 40 systems")
    Xs, reps = solver.dxgesv_batched([_dev(A) for A, _, _ in systems],
                                     [_dev(b) for _, b, _ in systems], "fp32")
    _check_all(systems, Xs, reps)


def test_batched_failures(solver):
    """An exactly singular system (FP64 fallback reports info), an order
    above the limit (info = -1, X untouched) and a kappa = 1e9 system with
    FP16 operands (fallback) next to ordinary ones."""
    import torch

    g = np.random.default_rng(3)
    A_ok, b_ok, _ = gen.prescribed_cond_system(90, 1e2, g)
    A_sing = g.uniform(-1, 1, (70, 70))
    A_sing[:, 13] = 0.0
    b_sing = np.ones((70, 1))
    A_big = g.uniform(-1, 1, (520, 520))
    b_big = np.ones((520, 1))
    A_ill, b_ill, _ = gen.prescribed_cond_system(200, 1e9, g)
    As = [A_ok, A_sing, A_big, A_ill]
    Bs = [b_ok, b_sing, b_big, b_ill]
    _say("batched failures")
    from paper_0808_2794_amd import mixlu

    buf = solver.batched_buffers([_dev(A) for A in As], [_dev(b) for b in Bs], "fp16")
    for X in buf["X"]:
        X.fill_(7.0)
    solver.run_batched(buf)
    torch.cuda.synchronize()
    reps = mixlu.reports_from_bytes(bytes(buf["reps"].cpu().numpy()))
    assert mixlu.mixlu_report_read(solver.ctx, buf["reps"], len(As)) == reps
    assert reps[0]["converged"]
    assert reps[1]["info"] == 14 and reps[1]["prec"] == "fp64" and not reps[1]["converged"], reps[1]
    assert reps[2]["info"] == -1 and not reps[2]["converged"], reps[2]
    assert bool((buf["X"][2] == 7.0).all())
    assert reps[3]["iter"] < 0 and reps[3]["prec"] == "fp64" and reps[3]["converged"], reps[3]
    ref = O.gesv_ir(A_ill, b_ill)
    m = O.metrics(A_ill, buf["X"][3].cpu().numpy(), b_ill, x_ref=ref.x)
    assert m["passes"] and float(np.max(m["fwd_ref"])) <= 1e-12 * 1e9


def test_batched_graph_capture_and_replay(solver):
    """The batched launch captured once in a HIP graph: every replay gives
    the eager result bit for bit, with eager work and synchronizations
    between replays; then new data in the same buffers, replayed, matches
    the oracle."""
    import torch

    from paper_0808_2794_amd import mixlu

    systems = _systems([48, 200, 333, 17, 512, 96], 77)
    buf = solver.batched_buffers([_dev(A) for A, _, _ in systems],
                                 [_dev(b) for _, b, _ in systems], "fp32")
    _say("batched eager reference")
    solver.run_batched(buf)
    torch.cuda.synchronize()
    eager = [X.clone() for X in buf["X"]]
    eager_reps = bytes(buf["reps"].cpu().numpy())
    stream = torch.cuda.Stream()
    mixlu.mixlu_set_stream(solver.ctx, stream)
    try:
        g = torch.cuda.CUDAGraph()
        _say("batched capture")
        with torch.cuda.graph(g, stream=stream):
            solver.run_batched(buf)
        for rep in range(3):
            for X in buf["X"]:
                X.zero_()
            torch.cuda.synchronize()
            _say(f"batched replay {rep}")
            g.replay()
            torch.cuda.synchronize()
            for X, E in zip(buf["X"], eager):
                assert torch.equal(X, E), rep
            assert bytes(buf["reps"].cpu().numpy()) == eager_reps
        # new systems of the same orders in the same buffers
        new = _systems([48, 200, 333, 17, 512, 96], 78)
        for (A, b, _), dA, dB in zip(new, buf["A"], buf["B"]):
            dA.copy_(_dev(A))
            dB.copy_(_dev(b))
        torch.cuda.synchronize()
        _say("batched replay with new data")
        g.replay()
        torch.cuda.synchronize()
        reps = mixlu.reports_from_bytes(bytes(buf["reps"].cpu().numpy()))
        _check_all(new, buf["X"], reps)
    finally:
        mixlu.mixlu_set_stream(solver.ctx, torch.cuda.current_stream())


def test_batched_full_workload_sampled(solver):
    """The full batched workload: 4096 systems, n_i uniform in [16, 512],
    kappa_i log-uniform in [1e1, 1e5]; every report converged, 64 sampled
    systems checked against the oracle."""
    As, bs, _, ks = gen.batched_systems(4096, 401)
    _say("batched 4096 systems fp32")
    Xs, reps = solver.dxgesv_batched([_dev(A) for A in As], [_dev(b) for b in bs], "fp32")
    assert all(r["converged"] for r in reps)
    assert all(r["prec"] == "fp32" for r in reps)
    idx = np.random.default_rng(0).choice(4096, 64, replace=False)
    _check_all([(As[i], bs[i], ks[i]) for i in idx], [Xs[i] for i in idx],
               [reps[i] for i in idx])


def _oracle_refs(systems):
    return [O.gesv_ir(A, b).x for A, b, _ in systems]


def _check_with_refs(systems, refs, Xs, reps):
    for i, ((A, b, kappa), ref, X, rep) in enumerate(zip(systems, refs, Xs, reps)):
        m = O.metrics(A, X.cpu().numpy(), b, x_ref=ref)
        assert m["passes"], (i, A.shape[0], rep)
        assert float(np.max(m["fwd_ref"])) <= 1e-12 * kappa, (i, A.shape[0], rep)
        assert rep["converged"], (i, rep)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_every_tile_set(solver, prec):
    """Every candidate of the autotuner's search space (panel 16/8, chunk
    128/64/32, 2/1 workgroups per CU) solves the ragged-size batch to the
    oracle's bar."""
    import torch

    from paper_0808_2794_amd import mixlu

    systems = _systems([1, 7, 8, 9, 16, 17, 31, 33, 64, 65, 100, 129, 255, 300, 511, 512], 611)
    refs = _oracle_refs(systems)
    p = mixlu.PREC[prec]
    buf = solver.batched_buffers([_dev(A) for A, _, _ in systems],
                                 [_dev(b) for _, b, _ in systems], prec)
    saved = mixlu.mixlu_batched_get_tiles(solver.ctx, p)
    try:
        for panel, chunk, groups in mixlu.TILE_CANDIDATES:
            _say(f"batched tiles {prec} panel={panel} chunk={chunk} groups={groups}")
            mixlu.mixlu_batched_set_tiles(solver.ctx, p, panel, chunk, groups)
            for X in buf["X"]:
                X.zero_()
            solver.run_batched(buf)
            torch.cuda.synchronize()
            reps = mixlu.reports_from_bytes(bytes(buf["reps"].cpu().numpy()))
            _check_with_refs(systems, refs, buf["X"], reps)
    finally:
        mixlu.mixlu_batched_set_tiles(solver.ctx, p, saved["panel"], saved["chunk"],
                                      saved["groups"], saved["tuned"])


def test_batched_autotune(solver):
    """The autotuner times all twelve candidates on the caller's batch, keeps
    the fastest in the context (tuned flag set), and the tuned launch - also
    when captured in a graph - solves the batch to the oracle's bar.  An
    invalid tile set is refused."""
    import torch

    from paper_0808_2794_amd import mixlu

    g = np.random.default_rng(12)
    sizes = [int(v) for v in g.integers(16, 513, 96)]
    systems = _systems(sizes, 612)
    refs = _oracle_refs(systems)
    buf = solver.batched_buffers([_dev(A) for A, _, _ in systems],
                                 [_dev(b) for _, b, _ in systems], "fp32")
    _say("batched autotune fp32")
    best, ms = solver.tune_batched(buf)
    assert best["tuned"] and (best["panel"], best["chunk"], best["groups"]) in ms
    assert len(ms) == 12 and all(v > 0 for v in ms.values()), ms
    assert ms[(best["panel"], best["chunk"], best["groups"])] == min(ms.values())
    assert mixlu.mixlu_batched_get_tiles(solver.ctx, mixlu.FP32) == best
    # the tune's own last run left complete results
    torch.cuda.synchronize()
    _check_with_refs(systems, refs, buf["X"],
                     mixlu.reports_from_bytes(bytes(buf["reps"].cpu().numpy())))
    stream = torch.cuda.Stream()
    mixlu.mixlu_set_stream(solver.ctx, stream)
    try:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            solver.run_batched(buf)
        for X in buf["X"]:
            X.zero_()
        torch.cuda.synchronize()
        _say("batched tuned graph replay")
        graph.replay()
        torch.cuda.synchronize()
        _check_with_refs(systems, refs, buf["X"],
                         mixlu.reports_from_bytes(bytes(buf["reps"].cpu().numpy())))
    finally:
        mixlu.mixlu_set_stream(solver.ctx, torch.cuda.current_stream())
    with pytest.raises(mixlu.MixluError):
        mixlu.mixlu_batched_set_tiles(solver.ctx, mixlu.FP32, 12, 128, 2)
    mixlu.mixlu_batched_set_tiles(solver.ctx, mixlu.FP32, 16, 128, 2)


def test_batched_tune_refused_during_capture(solver):
    """The autotuner synchronizes, so under graph capture it refuses with
    MIXLU_ERR_CAPTURING before enqueuing anything; the tiles stay as they
    were."""
    import torch

    from paper_0808_2794_amd import mixlu

    systems = _systems([40, 90], 91)
    buf = solver.batched_buffers([_dev(A) for A, _, _ in systems],
                                 [_dev(b) for _, b, _ in systems], "fp32")
    before = mixlu.mixlu_batched_get_tiles(solver.ctx, mixlu.FP32)
    stream = torch.cuda.Stream()
    mixlu.mixlu_set_stream(solver.ctx, stream)
    try:
        g = torch.cuda.CUDAGraph()
        _say("batched tune under capture")
        with pytest.raises(mixlu.MixluError, match="code 6"):
            with torch.cuda.graph(g, stream=stream):
                solver.tune_batched(buf)
    finally:
        mixlu.mixlu_set_stream(solver.ctx, torch.cuda.current_stream())
    torch.cuda.synchronize()
    assert mixlu.mixlu_batched_get_tiles(solver.ctx, mixlu.FP32) == before

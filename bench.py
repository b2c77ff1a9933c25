#!/usr/bin/env python3
"""Time to an FP64-accurate solve on one MI355X: low-precision factorization +
FP64 iterative refinement (Algorithm 1 of Baboulin et al., arXiv:0808.2794)
versus FP64 factorizations on the same GPU.

Workloads (--workload; all inputs seeded, synthetic and already in HBM when
the timed region starts; one step = one complete solve call):

  dense    (default) A = U diag(sigma) V^T, n = 16384, sigma geometric from 1
           to 1/kappa, kappa = 1e4, U, V Haar, b = A x_true, one right-hand
           side (seed 221); mixlu_dxgesv with an FP32 factor.
  spd      A = Q diag(lambda) Q^T, n = 16384, lambda log-uniform in [1e-3, 1],
           16 right-hand sides (seed 301); mixlu_dxposv (Cholesky).
  batched  4096 systems, n_i uniform in [16, 512], kappa_i log-uniform in
           [1e1, 1e5] (seed 401); mixlu_dxgesv_batched, one launch.
  adjoint  n = 4096, 64 right-hand sides, kappa = 1e3 (seed 501); forward
           solve + adjoint (G_B = A^-T G_X, G_A = -G_B X^T) with the same
           factors.

Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload dense|spd|batched|adjoint]
                    [--prec fp32|fp16|bf16|fp64]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published peaks of one MI355X (dense, no sparsity).  The FP32 vector
# figure is the non-packed rate (256 CU x 64 lanes x 2 flop x 2.4 GHz): the
# library is built without packed-FP32 instructions.
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFS = {"fp16": 2500.0, "bf16": 2500.0, "fp8": 5000.0, "fp32": 157.3, "fp64": 78.6}
PEAK_VALU_TFS = {"fp32": 78.6, "fp64": 78.6}
METRIC = "time to FP64-accurate solve, mixed vs FP64 LU on 1 GPU; MFMA util"
DTYPE = {"fp32": "f32", "fp16": "f16", "bf16": "bf16", "fp8": "e4m3", "fp64": "f64"}
DEFAULT_PREC = {"dense": "fp32", "spd": "fp16", "batched": "fp32", "adjoint": "fp32",
                "sparse": "fp32"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="dense",
                    choices=["dense", "spd", "batched", "adjoint", "sparse"])
    ap.add_argument("--prec", default=None, choices=["fp32", "fp16", "bf16", "fp8", "fp64"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--kappa", type=float, default=None)
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--refine", default="classic", choices=["classic", "fgmres"],
                    help="refinement after the low-precision factor (dense workload)")
    ap.add_argument("--nb", type=int, default=0,
                    help="outer block width of the dense factorization (0: the library's choice)")
    ap.add_argument("--restart", type=int, default=0,
                    help="FGMRES restart length (0: the library's default, 30; at most 128)")
    ap.add_argument("--matrix", default="prescribed", choices=["prescribed", "uniform"],
                    help="dense workload input: U diag(sigma) V^T (default) or iid U[-1,1] "
                         "entries (no QR; for counter runs, whose traffic depends on the "
                         "shapes only)")
    ap.add_argument("--compare-steps", type=int, default=2, help="timed FP64 comparator runs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target wall time of the CPU oracle sample (0: skip)")
    ap.add_argument("--tiles", default=None,
                    help="batched workload: panel,chunk,groups tile set instead of autotuning "
                         "(e.g. 16,128,2)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 512 MiB once on the device (the reference kernel for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    return ap.parse_args()


def calibrate_copy():
    """One device copy of 512 MiB: the counter runs divide a kernel's
    FETCH_SIZE / WRITE_SIZE by what the counters read here per byte copied."""
    import torch

    x = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    sync()
    y.copy_(x)
    sync()
    print(json.dumps({"copied_bytes": x.numel() * 4}), flush=True)


def sync():
    import torch

    torch.cuda.synchronize()


def time_calls(fn, k):
    sync()
    t0 = time.perf_counter()
    out = None
    for _ in range(k):
        out = fn()
    sync()
    return (time.perf_counter() - t0) / k * 1e3, out


def source_digest(names=None):
    """Digest of the kernel sources (all of them, or the named files), to tie
    stored counter readings to the code they were taken on."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0808_2794_amd", "csrc")
    for name in sorted(names or os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stored_traffic(workload, kernel_class):
    """HBM bytes per launch of the dominant kernel from the rocprofv3 PMC
    readings kept in profiles/traffic.json, only if they were taken on the
    current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(workload, {}).get(kernel_class)
    except (OSError, ValueError):
        return None
    # a record names the files that define its kernel (the kernel's own file
    # and the shared header); without that list every kernel source counts
    if not rec or rec.get("source_digest") != source_digest(rec.get("sources")):
        return None
    return rec.get("bytes_per_launch")


def roofline(kstats, prec, steps, workload):
    """Roofline record of the kernel class with the largest device time."""
    name, st = max(kstats.items(), key=lambda kv: kv[1]["ms"])
    if st["launches"] == 0 or st["ms"] <= 0:
        return None
    sec = st["ms"] / 1e3
    wprec = "fp64" if prec == "fp64" else "fp32"
    if name == "trailing_update":
        rec = {"bound": "mfma", "achieved": st["flops"] / sec / 1e12,
               "peak": PEAK_MFMA_TFS[prec], "unit": "TFLOP/s"}
    elif name in ("trsv", "residual", "pack_operands", "sparse_spmv"):
        rec = {"bound": "hbm", "achieved": st["bytes"] / sec / 1e9, "peak": PEAK_HBM_GBS,
               "unit": "GB/s"}
    else:  # panels and the batched kernel: dependent steps on the vector ALUs
        rec = {"bound": "alu", "achieved": st["flops"] / sec / 1e12, "peak": PEAK_VALU_TFS[wprec],
               "unit": "TFLOP/s"}
    rec["frac"] = rec["achieved"] / rec["peak"]
    rec["traffic"] = stored_traffic(workload, name)
    rec["kernel"] = name
    rec["launches_per_step"] = st["launches"] / steps
    rec["avg_launch_us"] = st["ms"] / st["launches"] * 1e3
    return rec


def stored_record(workload, kernel_class, key):
    """A stored rocprofv3 counter record (profiles/traffic.json), only if it
    was taken on the current sources of the files that define the kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(workload, {}).get(kernel_class)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_digest") != source_digest(rec.get("sources")):
        return None
    return rec.get(key)


def class_measures(kst, prec, steps, workload, columns):
    """Per-class figures of the hot path: the panel's time per eliminated
    column (latency-bound), the trailing update's FLOP rate and MFMA
    utilization (from the timed flops, and from the MfmaUtil counter when a
    current record exists), and the algorithmic GB/s of the triangular solves
    and of the FP64 residual (with the counter-measured HBM bytes beside them
    when recorded)."""
    out = {}
    for name in ("panel_getf2", "panel_potf2"):
        st = kst.get(name)
        if st and st["launches"] and columns:
            out["panel_us_per_column"] = st["ms"] / steps / columns * 1e3
    st = kst.get("trailing_update")
    if st and st["ms"] > 0:
        tf = st["flops"] / (st["ms"] / 1e3) / 1e12
        out["trailing_tflops"] = tf
        out["mfma_util_timed"] = tf / PEAK_MFMA_TFS[prec]
        cnt = stored_record(workload, "trailing_update", "mfma_util")
        if cnt is not None:
            out["mfma_util"] = cnt
            out["mfma_util_source"] = "rocprofv3 MfmaUtil, duration-weighted over the update kernels"
        else:
            out["mfma_util"] = out["mfma_util_timed"]
            out["mfma_util_source"] = "timed flops / peak (no current counter record)"
    for name, key in (("trsv", "trsv"), ("residual", "residual")):
        st = kst.get(name)
        if st and st["ms"] > 0 and st["launches"]:
            sec = st["ms"] / 1e3
            out[f"{key}_gbs"] = st["bytes"] / sec / 1e9
            out[f"{key}_hbm_frac"] = out[f"{key}_gbs"] / PEAK_HBM_GBS
            tb = stored_record(workload, name, "bytes_per_launch")
            if tb is not None:
                out[f"{key}_traffic_gbs"] = tb * st["launches"] / sec / 1e9
    return out


def kernel_table(kst, steps):
    return {k: {"ms_per_step": v["ms"] / steps, "launches_per_step": v["launches"] / steps}
            for k, v in kst.items() if v["launches"]}


def threads():
    return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def cpu_getrf_sample(A_host, target_s, label):
    """The CPU oracle's FP64 elimination on the same matrix, stopped after as
    many steps as fit the time budget, scaled by the exact ratio of
    elimination work (sum over steps of (n-k-1)^2 + (n-k-1))."""
    import numpy as np

    from oracle import oracle as O

    n = A_host.shape[0]
    k = np.arange(n, dtype=np.float64)
    work = (n - k - 1.0) ** 2 + (n - k - 1.0)
    cum = np.cumsum(work)
    steps = 8
    t0 = time.perf_counter()
    O.getrf(A_host, steps=steps)
    dt = time.perf_counter() - t0
    steps = int(np.clip(np.searchsorted(cum, cum[steps - 1] * target_s / max(dt, 1e-3)), 8, n))
    t0 = time.perf_counter()
    O.getrf(A_host, steps=steps)
    dt = time.perf_counter() - t0
    frac = cum[steps - 1] / cum[-1]
    return {"value": dt / frac * 1e3, "unit": "ms", "cores": threads(), "kind": "oracle",
            "sample": f"{label}: first {steps} of {n} elimination steps of the FP64 oracle "
                      f"({dt:.1f} s wall), scaled by the exact elimination-work ratio "
                      f"{1 / frac:.1f}; refinement (O(n^2) per iteration) not included"}


def comparator_speedup(comp, ms):
    vals = [v for k, v in comp.items() if k.endswith("_ms")]
    if vals:
        comp["speedup_vs_fastest_fp64"] = min(vals) / ms
    return comp


# --------------------------------------------------------------- workloads
def run_dense(args, prec):
    import numpy as np
    import torch

    from paper_0808_2794_amd import mixlu
    from synth import gen

    n = args.n or 16384
    kappa = args.kappa or 1e4
    seed = args.seed or 221
    if args.matrix == "uniform":
        g = torch.Generator(device="cuda").manual_seed(seed)
        A = torch.rand(n, n, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
        x_true_d = torch.rand(n, 1, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
        b = A @ x_true_d
        x_true = x_true_d.cpu().numpy()
    else:
        A, b, x_true = gen.prescribed_cond_system(n, kappa, seed, backend="torch", device="cuda")
    A, b = A.contiguous(), b.contiguous()
    sync()
    solver = mixlu.Solver()
    refine = mixlu.REFINE_FGMRES if args.refine == "fgmres" else mixlu.REFINE_CLASSIC
    kw = dict(refine=refine, restart=args.restart, nb=args.nb)
    for _ in range(args.warmup):
        solver.dxgesv(A, b, prec, **kw)
    mixlu.mixlu_profile_enable(solver.ctx, True)
    ms, res = time_calls(lambda: solver.dxgesv(A, b, prec, **kw), args.steps)
    history = mixlu.mixlu_refine_history(solver.ctx)
    kst = mixlu.mixlu_profile_read(solver.ctx)
    mixlu.mixlu_profile_enable(solver.ctx, False)
    x = res.x.double().cpu().numpy()
    fwd = float(np.abs(x - x_true).max() / np.abs(x_true).max())
    comp = {}
    if args.compare_steps > 0:
        solver.dgesv(A, b)
        comp["mixlu_dgesv_ms"], _ = time_calls(lambda: solver.dgesv(A, b), args.compare_steps)
        torch.linalg.solve(A, b)
        comp["torch_linalg_solve_fp64_ms"], _ = time_calls(lambda: torch.linalg.solve(A, b),
                                                          args.compare_steps)
        comparator_speedup(comp, ms)
    cpu = cpu_getrf_sample(A.cpu().numpy(), args.cpu_seconds, "same matrix") \
        if args.cpu_seconds > 0 else None
    solver.close()
    rep = res.report
    return ms, kst, cpu, comp, {
        "columns": n,
        "config": {"workload": (f"dense_nonsym_prescribed_cond_n{n}_kappa{kappa:g}_nrhs1"
                                if args.matrix == "prescribed" else f"dense_nonsym_uniform_n{n}_nrhs1"),
                   "n": n, "kappa": kappa, "nrhs": 1, "seed": seed, "factor_precision": prec,
                   "refinement": "fp64 " + args.refine
                   + (f" restart {args.restart}" if args.refine == "fgmres" and args.restart else ""),
                   **({"nb": args.nb} if args.nb else {})},
        "solve": {"iter": rep["iter"], "prec_used": rep["prec"], "converged": rep["converged"],
                  "berr": rep["berr"], "fwd_err_vs_x_true": fwd,
                  "residual_history": [float(f"{v:.3e}") for v in history[:40]]}}


def run_spd(args, prec):
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_0808_2794_amd import mixlu
    from synth import gen

    n = args.n or 16384
    kappa = args.kappa or 1e3
    seed = args.seed or 301
    nrhs = 16
    A, B, X_true = gen.spd_system(n, kappa, seed, nrhs=nrhs, backend="torch", device="cuda")
    A, B = A.contiguous(), B.contiguous()
    sync()
    solver = mixlu.Solver()
    for _ in range(args.warmup):
        solver.dxposv(A, B, prec)
    mixlu.mixlu_profile_enable(solver.ctx, True)
    ms, res = time_calls(lambda: solver.dxposv(A, B, prec), args.steps)
    kst = mixlu.mixlu_profile_read(solver.ctx)
    mixlu.mixlu_profile_enable(solver.ctx, False)
    X = res.x.cpu().numpy()
    fwd = float(np.abs(X - X_true).max() / np.abs(X_true).max())
    comp = {}
    if args.compare_steps > 0:
        solver.dposv(A, B)
        comp["mixlu_dposv_ms"], _ = time_calls(lambda: solver.dposv(A, B), args.compare_steps)

        def torch_chol():
            L = torch.linalg.cholesky(A)
            return torch.cholesky_solve(B, L)

        torch_chol()
        comp["torch_cholesky_solve_fp64_ms"], _ = time_calls(torch_chol, args.compare_steps)
        comparator_speedup(comp, ms)
    cpu = None
    if args.cpu_seconds > 0:
        # the oracle's Cholesky on a leading principal block sized to the
        # budget, scaled by the cube of the order ratio
        A_host = A.cpu().numpy()
        m = 1024
        t0 = time.perf_counter()
        O.potrf(A_host[:m, :m])
        dt = time.perf_counter() - t0
        m = int(min(n, m * (args.cpu_seconds / max(dt, 1e-3)) ** (1 / 3)))
        t0 = time.perf_counter()
        O.potrf(A_host[:m, :m])
        dt = time.perf_counter() - t0
        scale = (n / m) ** 3
        cpu = {"value": dt * scale * 1e3, "unit": "ms", "cores": threads(), "kind": "oracle",
               "sample": f"FP64 oracle Cholesky of the leading {m} x {m} block of the same "
                         f"matrix ({dt:.1f} s wall), scaled by (n/m)^3 = {scale:.1f}; "
                         "solves and refinement not included"}
    solver.close()
    rep = res.report
    return ms, kst, cpu, comp, {
        "columns": n,
        "config": {"workload": f"dense_spd_n{n}_kappa{kappa:g}_nrhs{nrhs}", "n": n, "kappa": kappa,
                   "nrhs": nrhs, "seed": seed, "factor_precision": prec, "factorization": "cholesky",
                   "refinement": "fp64"},
        "solve": {"iter": rep["iter"], "prec_used": rep["prec"], "converged": rep["converged"],
                  "berr": rep["berr"], "fwd_err_vs_x_true": fwd}}


def run_batched(args, prec):
    import numpy as np
    import torch

    from oracle import oracle as O
    from paper_0808_2794_amd import mixlu
    from synth import gen

    seed = args.seed or 401
    count = 4096
    As, bs, xs, ks = gen.batched_systems(count, seed)
    solver = mixlu.Solver()
    dA = [torch.from_numpy(a).cuda() for a in As]
    dB = [torch.from_numpy(b).cuda() for b in bs]
    buf = solver.batched_buffers(dA, dB, prec)
    sync()
    # tile sets chosen by the autotuner on this batch (outside the timed region)
    if args.tiles:
        p_, c_, g_ = (int(v) for v in args.tiles.split(","))
        mixlu.mixlu_batched_set_tiles(solver.ctx, mixlu.PREC[prec], p_, c_, g_)
        tiles, tile_ms = mixlu.mixlu_batched_get_tiles(solver.ctx, mixlu.PREC[prec]), {}
    else:
        tiles, tile_ms = solver.tune_batched(buf)
    sync()
    for _ in range(args.warmup):
        solver.run_batched(buf)
    mixlu.mixlu_profile_enable(solver.ctx, True)
    ms, _ = time_calls(lambda: solver.run_batched(buf), args.steps)
    kst = mixlu.mixlu_profile_read(solver.ctx)
    mixlu.mixlu_profile_enable(solver.ctx, False)
    # algorithmic LU work of the batch, charged to the batched kernel class
    flops = sum(2.0 / 3.0 * a.shape[0] ** 3 for a in As)
    kst["batched_solve"]["flops"] = flops * args.steps
    reps = mixlu.reports_from_bytes(bytes(buf["reps"].cpu().numpy()))
    conv = sum(1 for r in reps if r["converged"])
    fb = sum(1 for r in reps if r["prec"] == "fp64" and prec != "fp64")
    fwd = max(float(np.abs(X.cpu().numpy() - x).max() / np.abs(x).max())
              for X, x in zip(buf["X"], xs))
    comp = {}
    if args.compare_steps > 0:
        buf64 = solver.batched_buffers(dA, dB, "fp64")
        comp["mixlu_batched_fp64_tiles"], _ = solver.tune_batched(buf64)
        solver.run_batched(buf64)
        comp["mixlu_batched_fp64_ms"], _ = time_calls(lambda: solver.run_batched(buf64),
                                                      args.compare_steps)

        def torch_loop():
            for a, b in zip(dA, dB):
                torch.linalg.solve(a, b)

        torch_loop()
        comp["torch_linalg_solve_fp64_loop_ms"], _ = time_calls(torch_loop, 1)
        comparator_speedup(comp, ms)
    cpu = None
    if args.cpu_seconds > 0:
        t0 = time.perf_counter()
        done, work_done = 0, 0.0
        while done < count and time.perf_counter() - t0 < args.cpu_seconds:
            O.gesv_ir(As[done], bs[done])
            work_done += As[done].shape[0] ** 3
            done += 1
        dt = time.perf_counter() - t0
        total = sum(a.shape[0] ** 3 for a in As)
        cpu = {"value": dt * total / work_done * 1e3, "unit": "ms", "cores": threads(),
               "kind": "oracle",
               "sample": f"FP64 oracle solve (GE + refinement) of the first {done} of {count} "
                         f"systems ({dt:.1f} s wall), scaled by sum n^3 of the batch / sum n^3 "
                         "of the sample"}
    solver.close()
    return ms, kst, cpu, comp, {
        "config": {"workload": f"batched_{count}_systems_n16to512_kappa1e1to1e5_nrhs1",
                   "systems": count, "sum_n3": float(sum(a.shape[0] ** 3 for a in As)),
                   "seed": seed, "factor_precision": prec, "refinement": "fp64",
                   "tiles": tiles,
                   "tile_candidates_ms": {f"panel{p}_chunk{c}_groups{g}": round(v, 3)
                                          for (p, c, g), v in tile_ms.items()}},
        "solve": {"converged": conv, "systems": count, "fp64_fallbacks": fb,
                  "max_fwd_err_vs_x_true": fwd}}


def run_sparse(args, prec):
    """Algorithm 2 (FGMRES(20)-GMRES_SP(30)) on the 3-D convection-diffusion
    stand-in (k^3 grid, Peclet 1), against the same solver with FP64 inner
    solves (FGMRES-GMRES_DP, the paper's comparison)."""
    import numpy as np
    import torch

    from paper_0808_2794_amd import mixlu
    from synth import gen

    k = args.n or 64
    peclet = 1.0
    seed = args.seed or 950
    m_out, m_in = 20, 30
    rp, ci, v, b, x_true = gen.sparse_convdiff3d(k, peclet, seed)
    solver = mixlu.Solver()
    d = [torch.from_numpy(a).cuda() for a in (rp, ci, v, b)]
    sync()
    res = {}
    for _ in range(args.warmup):
        solver.sparse_fgmres(*d, inner=prec, m_out=m_out, m_in=m_in)
    mixlu.mixlu_profile_enable(solver.ctx, True)

    def one():
        res["r"] = solver.sparse_fgmres(*d, inner=prec, m_out=m_out, m_in=m_in)

    ms, _ = time_calls(one, args.steps)
    kst = mixlu.mixlu_profile_read(solver.ctx)
    mixlu.mixlu_profile_enable(solver.ctx, False)
    rep = res["r"].report
    fwd = float(np.abs(res["r"].x.cpu().numpy() - x_true).max() / np.abs(x_true).max())
    comp = {}
    if args.compare_steps > 0 and prec != "fp64":
        solver.sparse_fgmres(*d, inner="fp64", m_out=m_out, m_in=m_in)
        out = {}

        def dp():
            out["r"] = solver.sparse_fgmres(*d, inner="fp64", m_out=m_out, m_in=m_in)

        comp["fgmres_gmres_dp_ms"], _ = time_calls(dp, args.compare_steps)
        comp["fgmres_gmres_dp_inner_cycles"] = out["r"].report["iter"]
        comparator_speedup(comp, ms)
    solver.close()
    return ms, kst, None, comp, {
        "config": {"workload": f"sparse_convdiff3d_k{k}_peclet{peclet:g}_mout{m_out}_min{m_in}",
                   "n": k ** 3, "nnz": int(len(v)), "seed": seed, "inner_precision": prec,
                   "outer": "fp64 fgmres"},
        "solve": {"inner_cycles": rep["iter"], "outer_cycles": rep["outer"],
                  "converged": rep["converged"], "berr": rep["berr"],
                  "fwd_err_vs_x_true": fwd}}


def run_adjoint(args, prec):
    import numpy as np
    import torch

    from paper_0808_2794_amd import mixlu
    from paper_0808_2794_amd.autograd import solve
    from synth import gen

    n = args.n or 4096
    kappa = args.kappa or 1e3
    seed = args.seed or 501
    nrhs = 64
    A_h, B_h, W_h = gen.grad_problem(n, nrhs, kappa, seed, backend="torch", device="cuda")
    A0 = torch.from_numpy(A_h).cuda()
    B0 = torch.from_numpy(B_h).cuda()
    Wt = torch.from_numpy(W_h).cuda()
    solver = mixlu.Solver()

    reports = {}

    def step():
        from paper_0808_2794_amd.autograd import MixedSolve

        A = A0.detach().requires_grad_(True)
        B = B0.detach().requires_grad_(True)
        X = solve(A, B, prec, solver)
        (X * Wt).sum().backward()
        node = X.grad_fn
        if isinstance(node, torch.autograd.function.BackwardCFunction):
            reports["forward"] = getattr(node, "report", None)
            reports["adjoint"] = getattr(node, "backward_report", None)
        return X, A.grad, B.grad

    for _ in range(args.warmup):
        step()
    mixlu.mixlu_profile_enable(solver.ctx, True)
    ms, (X, GA, GB) = time_calls(step, args.steps)
    kst = mixlu.mixlu_profile_read(solver.ctx)
    mixlu.mixlu_profile_enable(solver.ctx, False)
    comp = {}
    if args.compare_steps > 0:
        def torch_step():
            A = A0.detach().requires_grad_(True)
            B = B0.detach().requires_grad_(True)
            (torch.linalg.solve(A, B) * Wt).sum().backward()
            return A.grad, B.grad

        GA_ref, GB_ref = torch_step()
        comp["torch_linalg_solve_fp64_autograd_ms"], _ = time_calls(torch_step, args.compare_steps)
        comparator_speedup(comp, ms)
        comp["rel_diff_GB_vs_torch_fp64"] = float((GB - GB_ref).abs().max() / GB_ref.abs().max())
        comp["rel_diff_GA_vs_torch_fp64"] = float((GA - GA_ref).abs().max() / GA_ref.abs().max())
    cpu = cpu_getrf_sample(A_h, args.cpu_seconds, "the forward matrix") \
        if args.cpu_seconds > 0 else None
    solver.close()
    return ms, kst, cpu, comp, {
        "columns": n,
        "config": {"workload": f"differentiable_solve_n{n}_nrhs{nrhs}_kappa{kappa:g}", "n": n,
                   "nrhs": nrhs, "kappa": kappa, "seed": seed, "factor_precision": prec,
                   "refinement": "fp64", "passes": "forward+adjoint"},
        "solve": {k: ({"iter": v["iter"], "prec_used": v["prec"], "converged": v["converged"],
                       "fallback_iter": v["fallback_iter"], "berr": v["berr"]} if v else None)
                  for k, v in reports.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(how it would shard is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        calibrate_copy()
        return
    prec = args.prec or DEFAULT_PREC[args.workload]
    fn = {"dense": run_dense, "spd": run_spd, "batched": run_batched,
          "adjoint": run_adjoint, "sparse": run_sparse}[args.workload]
    ms, kst, cpu, comp, extra = fn(args, prec)
    rl = roofline(kst, prec, args.steps, args.workload)
    line = {
        "metric": METRIC,
        "value": ms,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec] + "+f64",
        "data": "synthetic",
        "config": extra["config"],
        "solve": extra["solve"],
        "comparators": comp,
        "kernels": kernel_table(kst, args.steps),
        **class_measures(kst, prec, args.steps, args.workload, extra.get("columns")),
        "roofline": rl,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

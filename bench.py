#!/usr/bin/env python3
"""Time to an FP64-accurate solve on one MI355X: low-precision LU + FP64
iterative refinement (Algorithm 1 of Baboulin et al., arXiv:0808.2794)
versus FP64 LU on the same GPU.

Workload: dense nonsymmetric A = U diag(sigma) V^T, n = 16384, sigma
geometric from 1 to 1/kappa with kappa = 1e4, U and V Haar orthogonal,
x_true iid U[-1, 1], b = A x_true, one right-hand side (seed 221).  One
step = one mixlu_dxgesv call (equilibration, conversion, factorization,
x_0, refinement to the stopping test, fallback when needed) with A and b
already in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec fp32|fp16|bf16|fp64]
"""
import argparse
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


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--kappa", type=float, default=1e4)
    ap.add_argument("--seed", type=int, default=221)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp16", "bf16", "fp64"])
    ap.add_argument("--compare-steps", type=int, default=2, help="timed FP64 comparator runs")
    ap.add_argument("--cpu-steps", type=int, default=400,
                    help="elimination steps of the CPU oracle sample (0: skip)")
    return ap.parse_args()


def time_calls(fn, k):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = None
    for _ in range(k):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / k * 1e3, out


def roofline(kstats, prec):
    """Roofline record of the kernel class with the largest device time."""
    name, st = max(kstats.items(), key=lambda kv: kv[1]["ms"])
    if st["launches"] == 0 or st["ms"] <= 0:
        return None, name
    sec = st["ms"] / 1e3
    wprec = "fp64" if prec == "fp64" else "fp32"
    if name == "trailing_update":
        peak = PEAK_MFMA_TFS["fp64" if prec == "fp64" else prec]
        rec = {"bound": "mfma", "achieved": st["flops"] / sec / 1e12, "peak": peak,
               "unit": "TFLOP/s"}
    elif name in ("trsv", "residual", "pack_operands"):
        rec = {"bound": "hbm", "achieved": st["bytes"] / sec / 1e9, "peak": PEAK_HBM_GBS,
               "unit": "GB/s"}
    else:  # the panel: dependent per-column steps on the vector ALUs
        rec = {"bound": "alu", "achieved": st["flops"] / sec / 1e12, "peak": PEAK_VALU_TFS[wprec],
               "unit": "TFLOP/s"}
    rec["frac"] = rec["achieved"] / rec["peak"]
    rec["traffic"] = None
    rec["kernel"] = name
    rec["launches_per_step"] = None
    rec["avg_launch_us"] = st["ms"] / st["launches"] * 1e3
    return rec, name


def cpu_baseline(A_host, b_host, steps):
    """The CPU oracle (plain FP64 Gaussian elimination with partial pivoting)
    timed on a bounded sample: the first `steps` elimination steps on the
    same n x n matrix, scaled by the exact ratio of elimination work."""
    import numpy as np

    from oracle import oracle as O

    n = A_host.shape[0]
    t0 = time.perf_counter()
    O.getrf(A_host, steps=steps)
    dt = time.perf_counter() - t0
    k = np.arange(n, dtype=np.float64)
    work = (n - k - 1.0) ** 2 + (n - k - 1.0)
    frac = work[:steps].sum() / work.sum()
    projected_ms = dt / frac * 1e3
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": projected_ms, "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"first {steps} of {n} elimination steps of the FP64 oracle on the same "
                      f"matrix ({dt:.1f} s wall), scaled by the exact elimination-work ratio "
                      f"{1/frac:.1f}; refinement (O(n^2) per iteration) not included"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0808_2794_amd import mixlu
    from synth import gen

    torch.cuda.set_device(0)
    n, kappa = args.n, args.kappa
    A, b, x_true = gen.prescribed_cond_system(n, kappa, args.seed, backend="torch", device="cuda")
    A = A.contiguous()
    b = b.contiguous()
    torch.cuda.synchronize()
    solver = mixlu.Solver()

    # ---- mixed-precision solve: warmup, then K timed steps with kernel timing on
    for _ in range(args.warmup):
        solver.dxgesv(A, b, args.prec)
    mixlu.mixlu_profile_enable(solver.ctx, True)
    ms, res = time_calls(lambda: solver.dxgesv(A, b, args.prec), args.steps)
    kst = mixlu.mixlu_profile_read(solver.ctx)
    mixlu.mixlu_profile_enable(solver.ctx, False)
    rep = res.report
    x = res.x.double().cpu().numpy()
    fwd = float(np.abs(x - x_true).max() / np.abs(x_true).max())

    # ---- FP64 LU on the same GPU: ours (mixlu_dgesv) and torch.linalg.solve
    comp = {}
    if args.compare_steps > 0:
        solver.dgesv(A, b)
        comp["mixlu_dgesv_ms"], _ = time_calls(lambda: solver.dgesv(A, b), args.compare_steps)
        torch.linalg.solve(A, b)
        comp["torch_linalg_solve_fp64_ms"], _ = time_calls(lambda: torch.linalg.solve(A, b),
                                                          args.compare_steps)
        best = min(comp.values())
        comp["speedup_vs_fastest_fp64"] = best / ms
    rl, dom = roofline(kst, args.prec)
    if rl is not None:
        rl["launches_per_step"] = kst[dom]["launches"] / args.steps
    kernels = {k: {"ms_per_step": v["ms"] / args.steps, "launches_per_step": v["launches"] / args.steps}
               for k, v in kst.items() if v["launches"]}

    cpu = None
    if args.cpu_steps > 0:
        A_host = A.cpu().numpy()
        cpu = cpu_baseline(A_host, b.cpu().numpy(), args.cpu_steps)
        del A_host

    line = {
        "metric": "time to FP64-accurate solve, mixed vs FP64 LU on 1 GPU; MFMA util",
        "value": ms,
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16": "f16", "bf16": "bf16", "fp64": "f64"}[args.prec] + "+f64",
        "data": "synthetic",
        "config": {"workload": f"dense_nonsym_prescribed_cond_n{n}_kappa{kappa:g}_nrhs1",
                   "n": n, "kappa": kappa, "nrhs": 1, "seed": args.seed,
                   "factor_precision": args.prec, "refinement": "fp64"},
        "solve": {"iter": rep["iter"], "prec_used": rep["prec"], "converged": rep["converged"],
                  "berr": rep["berr"], "fwd_err_vs_x_true": fwd},
        "comparators": comp,
        "kernels": kernels,
        "roofline": rl,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    solver.close()


if __name__ == "__main__":
    main()

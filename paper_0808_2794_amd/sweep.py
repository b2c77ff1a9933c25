"""Refinement iterations against the condition number (the experiment of
Section 4), run on the batched solver.

For each factor precision and each kappa: ``count`` systems of order ``n``
with A = U diag(sigma) V^T (U, V Haar-orthogonal, sigma geometric from 1 to
1/kappa) and b = A x_true, solved in one batched launch with the FP64
fallback switched off, so every report shows what the low-precision
refinement alone did.  The number of solves per system (x_0 plus the
corrections) is set beside the generalized Datta bound
ceil(ln eps_d / (ln eps_s + ln kappa)), which assumes the worst-case
contraction kappa eps_s per step and is finite only while kappa eps_s < 1.

    python -m paper_0808_2794_amd.sweep --precs fp32,fp16,bf16 --count 200
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np

EPS = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "fp64": 2.0 ** -53}
EPS_D = 2.0 ** -53


def datta(prec: str, kappa: float):
    """ceil(ln eps_d / (ln eps_s + ln kappa)); None when kappa eps_s >= 1."""
    den = math.log(EPS[prec]) + math.log(kappa)
    return None if den >= 0 else math.ceil(math.log(EPS_D) / den)


def systems(kappa: float, count: int, n: int, seed: int):
    """The seeded systems of one kappa (the same for every precision)."""
    from synth import gen

    g = np.random.default_rng([seed, int(round(math.log10(kappa) * 1000))])
    return [gen.prescribed_cond_system(n, kappa, g)[:2] for _ in range(count)]


def sweep(solver, prec: str, kappa: float, count: int = 200, n: int = 200, seed: int = 0,
          itermax: int = 30) -> dict:
    """One row of the experiment: solve the systems of this kappa with the
    batched launch (fallback off) and summarize the iteration counts."""
    import torch

    from . import mixlu

    sys_ = systems(kappa, count, n, seed)
    opts = mixlu.default_opts(fallback=0, itermax=itermax)
    buf = solver.batched_buffers([torch.from_numpy(A).cuda() for A, _ in sys_],
                                 [torch.from_numpy(b).cuda() for _, b in sys_], prec, opts)
    solver.run_batched(buf)
    torch.cuda.synchronize()
    reps = mixlu.reports_from_bytes(bytes(buf["reps"].cpu().numpy()))
    solves = [r["iter"] + 1 for r in reps if r["converged"]]
    return {"prec": prec, "kappa": kappa, "n": n, "systems": count,
            "converged": len(solves),
            "mean_solves": float(np.mean(solves)) if solves else None,
            "max_solves": int(max(solves)) if solves else None,
            "datta_bound": datta(prec, kappa),
            "solves": solves}


def main(argv=None) -> None:
    from . import mixlu

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--precs", default="fp32,fp16,bf16")
    ap.add_argument("--kappas", default="1e1,1e2,1e3,1e4,1e5,1e6,1e7,1e8,1e9")
    ap.add_argument("--count", type=int, default=200)
    ap.add_argument("--n", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)
    solver = mixlu.Solver()
    rows = []
    for prec in args.precs.split(","):
        for k in args.kappas.split(","):
            row = sweep(solver, prec, float(k), args.count, args.n, args.seed)
            row.pop("solves")
            rows.append(row)
            print(json.dumps(row), flush=True)
    solver.close()
    print("\n| factor | kappa | converged | mean solves | max | Datta bound |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        mean = "-" if r["mean_solves"] is None else f"{r['mean_solves']:.2f}"
        mx = "-" if r["max_solves"] is None else str(r["max_solves"])
        bound = "-" if r["datta_bound"] is None else str(r["datta_bound"])
        print(f"| {r['prec']} | {r['kappa']:.0e} | {r['converged']}/{r['systems']} | {mean} | "
              f"{mx} | {bound} |")


if __name__ == "__main__":
    main()

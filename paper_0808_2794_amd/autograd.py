"""Differentiable mixed-precision solve X = A^{-1} B.

Forward: factor A once in the requested precision (``mixlu_getrf``), solve
(``mixlu_getrs``) and refine to FP64 accuracy (``mixlu_refine``).
Backward: the adjoint of X = A^{-1} B is G_B = A^{-T} G_X and
G_A = -G_B X^T; G_B is solved with the *same* low-precision factors through
the transposed solve (``mixlu_getrs``/``mixlu_refine`` with trans = 1), and
G_A is formed by ``mixlu_outer_update``.  All arithmetic runs in the HIP
library; this module only keeps the workspace alive between the passes.
"""
from __future__ import annotations

import torch

from . import mixlu


def _require(rep, what: str) -> None:
    """Raise unless the refinement certified every column (stopping test of
    Section 3) without meeting a singular FP64 factor."""
    if rep.info != 0:
        raise mixlu.MixluError(f"MixedSolve {what}: A is singular (info={rep.info})")
    if not rep.converged:
        raise mixlu.MixluError(f"MixedSolve {what}: refinement did not converge "
                               f"(iter={rep.iter}, fallback_iter={rep.fallback_iter}, "
                               f"berr={rep.berr:g})")


class MixedSolve(torch.autograd.Function):
    """X = MixedSolve.apply(A, B, prec): FP64 A (n x n, row-major) and B
    (n x nrhs) on the GPU; prec in {"fp32", "bf16", "fp16", "fp64"}."""

    @staticmethod
    def forward(ctx, A, B, prec="fp32", solver=None, reports=None):
        if A.dtype != torch.float64 or B.dtype != torch.float64:
            raise TypeError("A and B must be float64")
        # a solver created here lives as long as the autograd graph holds ctx
        # (its context is released when the Solver object is collected), so
        # repeated backward passes (retain_graph=True) keep a valid context
        s = mixlu.Solver() if solver is None else solver
        p = mixlu.PREC[prec] if isinstance(prec, str) else prec
        A = A.contiguous()
        vec = B.dim() == 1
        B2 = (B.reshape(-1, 1) if vec else B).contiguous()
        n, nrhs = B2.shape
        o = mixlu.default_opts()
        nbytes = mixlu.mixlu_workspace_size(s.ctx, mixlu.OP_GESV, p, n, nrhs, o)
        work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=A.device)
        F, info = mixlu.mixlu_getrf(s.ctx, p, A, work, o)
        if info != 0:
            raise mixlu.MixluError(f"MixedSolve: A is singular (info={info})")
        X = torch.empty_like(B2)
        if F.lowp_status == 0:
            mixlu.mixlu_getrs(s.ctx, F, B2, X)
        rep = mixlu.mixlu_refine(s.ctx, F, A, B2, X, o)
        _require(rep, "forward")
        # F now describes the factor that produced X: the low-precision one,
        # or the FP64 factor when the refinement fell back
        ctx.solver, ctx.work, ctx.F, ctx.opts, ctx.vec = s, work, F, o, vec
        ctx.report = rep.as_dict()
        ctx.reports = reports
        if reports is not None:
            reports["forward"] = ctx.report
        ctx.save_for_backward(A, X)
        return X.reshape(-1) if vec else X

    @staticmethod
    def backward(ctx, gX):
        A, X = ctx.saved_tensors
        s, F, o = ctx.solver, ctx.F, ctx.opts
        G = (gX.reshape(-1, 1) if ctx.vec else gX).contiguous().to(torch.float64)
        GB = torch.empty_like(G)
        if F.lowp_status == 0:
            mixlu.mixlu_getrs(s.ctx, F, G, GB, trans=1)
        rep = mixlu.mixlu_refine(s.ctx, F, A, G, GB, o, trans=1)
        ctx.backward_report = rep.as_dict()
        if ctx.reports is not None:
            ctx.reports["backward"] = ctx.backward_report
        _require(rep, "backward")
        GA = None
        if ctx.needs_input_grad[0]:
            GA = torch.empty_like(A)
            mixlu.mixlu_outer_update(s.ctx, GB, X, GA, -1.0, 0.0)
        gB = GB.reshape(-1) if ctx.vec else GB
        return GA, (gB if ctx.needs_input_grad[1] else None), None, None, None


def solve(A, B, prec="fp32", solver=None, reports=None):
    """Differentiable X = A^{-1} B with low-precision factors and FP64
    refinement in both passes.  When ``reports`` is a dict, the refinement
    reports of the two passes are stored in it under "forward" and
    "backward" (iterations, the precision of the factor that produced the
    result, fallback corrections)."""
    return MixedSolve.apply(A, B, prec, solver, reports)

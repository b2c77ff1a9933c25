"""GPU unit tests of the trailing update alone (mixlu_gemm_update): the
FP32 MFMA GEMM and the BF16 / FP16 / FP8 operand packing and MFMA kernels,
against the oracle's emulation of the same operand rounding
(oracle/lowp.py) with the products accumulated exactly.

Products of the rounded operands are exact in FP32 (at most 11 + 11
significand bits), so the only error is the FP32 accumulation:
|C_gpu - C_emul| <= (k + 2) 2^-24 (|C| + |A_q| |B_q|) elementwise.  The
scaled FP8 instruction adds its 128 products in one step, after aligning
products of different block scales, so FP8 is allowed a further
2^-14 |A_q| |B_q|.  A wrong block scale or a K block paired with the wrong
scale moves entries by factors like 2^12, far outside either bound.
"""
import numpy as np
import pytest

from oracle import lowp

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


def _operands(m, n, k, seed, spread):
    """Row/column blocks of 32 along k scaled by powers of two that differ
    from block to block (spread = largest exponent used)."""
    g = np.random.default_rng(seed)
    A = g.uniform(-1, 1, (m, k))
    B = g.uniform(-1, 1, (k, n))
    if spread:
        ea = g.integers(-spread, spread + 1, (m, k // 32))
        eb = g.integers(-spread, spread + 1, (k // 32, n))
        A = A * np.exp2(np.repeat(ea, 32, axis=1))
        B = B * np.exp2(np.repeat(eb, 32, axis=0))
    C = g.uniform(-1, 1, (m, n)) * (np.abs(A) @ np.abs(B)).mean()
    return A.astype(np.float32), B.astype(np.float32), C.astype(np.float32)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "fp8"])
@pytest.mark.parametrize("m,n,k,spread", [(256, 256, 128, 0), (300, 200, 256, 12),
                                          (1000, 700, 512, 12), (64, 1100, 128, 6)])
def test_gemm_update_vs_emulation(solver, prec, m, n, k, spread):
    import torch

    from paper_0808_2794_amd import mixlu

    if prec == "fp16" and spread > 6:
        spread = 6  # keep the FP16 operands inside its range (2^15)
    A, B, C = _operands(m, n, k, 100 + m + k + spread, spread)
    _say(f"gemm_update {prec} m={m} n={n} k={k} spread={spread}")
    Ad, Bd, Cd = (torch.from_numpy(x).cuda() for x in (A, B, C))
    work = torch.empty(mixlu.gemm_update_workspace_bytes(m, n, k), dtype=torch.uint8,
                       device="cuda")
    ov = mixlu.mixlu_gemm_update(solver.ctx, mixlu.PREC[prec], Ad, Bd, Cd, work, overflow=True)
    assert ov == 0
    got = Cd.cpu().numpy().astype(np.float64)
    expect, absprod = lowp.gemm_update(C, A, B, prec)
    tol = (k + 2) * 2.0 ** -24 * (np.abs(C) + absprod)
    if prec == "fp8":
        # One scaled FP8 MFMA sums 128 products whose block scales may differ
        # by 2^24 here; the hardware aligns them before adding, and that
        # alignment is not specified as exact.  Allow 2^-14 of the products'
        # magnitude on top of the FP32 accumulation bound: a misplaced scale
        # or K block still moves entries by 2^-3 of it or more.
        tol = tol + 2.0 ** -14 * absprod
    bad = np.abs(got - expect) > tol
    assert not bad.any(), (int(bad.sum()), float(np.max(np.abs(got - expect) / np.maximum(tol, 1e-300))))


def test_gemm_update_fp16_overflow_count(solver):
    import torch

    from paper_0808_2794_amd import mixlu

    m, n, k = 128, 128, 64
    A, B, C = _operands(m, n, k, 7, 0)
    A[3, 5] = 1e5  # beyond FP16's 65504
    B[7, 9] = -7e4
    _say("gemm_update fp16 overflow count")
    Ad, Bd, Cd = (torch.from_numpy(x).cuda() for x in (A, B, C))
    work = torch.empty(mixlu.gemm_update_workspace_bytes(m, n, k), dtype=torch.uint8,
                       device="cuda")
    assert mixlu.mixlu_gemm_update(solver.ctx, mixlu.FP16, Ad, Bd, Cd, work, overflow=True) == 2

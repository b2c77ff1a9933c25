"""Low-precision operand formats of the trailing update (test infrastructure
only; the GPU library never imports this module).

The method performs the O(n^3) part of the factorization in the low
precision eps_s (Section 2.1).  With BF16, FP16 or FP8 operands the factor
is kept in FP32 and only the trailing-update operands L21 and U12 are rounded
(reading C8), FP8 with one power-of-two scale per 32 consecutive K values of
each row of L21 and column of U12 (reading C10).  This module states those
roundings in plain numpy, in float64 arithmetic:

* ``round_fp16``: IEEE binary16, round to nearest even;
* ``round_bf16``: bfloat16 (FP32 with 8 significand bits), round to nearest
  even;
* ``round_e4m3``: OCP E4M3 (4 exponent bits, bias 7, 3 stored significand
  bits, subnormals down to 2^-9, largest finite 448, no infinities), round
  to nearest even, saturating at +-448;
* ``quantize_fp8_rows``: the E8M0 block scale 2^e with e = floor(log2 amax)
  - 7 (clamped to [-127, 127]), which puts the block's largest magnitude in
  [2^7, 2^8), then E4M3 codes of x / 2^e;
* ``gemm_update``: C - A_q B_q with the rounded operands, in float64.

Each rounding is written from the format's definition (sign, exponent,
significand grid) rather than by calling a converter, so that the tests can
pin it against the library converters (numpy float16, torch bfloat16 and
float8_e4m3fn) independently.
"""
from __future__ import annotations

import numpy as np


def _round_to_grid(x: np.ndarray, mant_bits: int, emin: int) -> np.ndarray:
    """Round float64 x to nearest even on the grid of a binary format with
    `mant_bits` stored significand bits and smallest normal exponent `emin`
    (no overflow handling).  The spacing at |x| in [2^e, 2^(e+1)) is
    2^(e - mant_bits); below 2^emin it is the subnormal spacing
    2^(emin - mant_bits)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    ax = np.abs(x[nz])
    e = np.floor(np.log2(ax))
    # log2 can be off by one next to powers of two: correct it exactly
    e = np.where(np.ldexp(1.0, e.astype(np.int64)) > ax, e - 1, e)
    e = np.where(np.ldexp(1.0, (e + 1).astype(np.int64)) <= ax, e + 1, e)
    e = np.maximum(e, emin).astype(np.int64)
    q = np.ldexp(1.0, e - mant_bits)
    out[nz] = np.sign(x[nz]) * np.round(ax / q) * q  # np.round: half to even
    out[~np.isfinite(x)] = x[~np.isfinite(x)]
    return out


def round_fp16(x) -> np.ndarray:
    """IEEE binary16 (10 stored bits, emin -14), nearest even; beyond the
    largest finite value 65504 the result overflows to +-inf."""
    r = _round_to_grid(x, 10, -14)
    big = np.abs(r) > 65504.0
    return np.where(big, np.copysign(np.inf, r), r)


def round_bf16(x) -> np.ndarray:
    """bfloat16 (7 stored bits, emin -126), nearest even."""
    r = _round_to_grid(x, 7, -126)
    big = np.abs(r) > 3.3895313892515355e38  # (2 - 2^-7) 2^127
    return np.where(big, np.copysign(np.inf, r), r)


E4M3_MAX = 448.0


def round_e4m3(x) -> np.ndarray:
    """OCP E4M3 (3 stored bits, emin -6), nearest even, saturating at
    +-448; NaN stays NaN."""
    r = _round_to_grid(x, 3, -6)
    return np.clip(r, -E4M3_MAX, E4M3_MAX)


def e4m3_values() -> np.ndarray:
    """Every finite non-negative E4M3 number in increasing order (127 of
    them): 0, the 7 subnormals k 2^-9, then the normals (1 + m/8) 2^e for
    e = -6..8, m = 0..7, without the NaN code at e = 8, m = 7."""
    vals = [0.0] + [k * 2.0 ** -9 for k in range(1, 8)]
    for e in range(-6, 9):
        for m in range(8):
            if e == 8 and m == 7:
                continue
            vals.append((1 + m / 8) * 2.0 ** e)
    return np.array(vals)


def block_scale_exponent(amax: float) -> int:
    """E8M0 exponent of a 32-value block whose largest magnitude is amax:
    floor(log2 amax) - 7, clamped to [-127, 127]; -127 for an all-zero
    block."""
    if amax == 0.0:
        return -127
    e = int(np.floor(np.log2(amax)))
    if 2.0 ** e > amax:
        e -= 1
    if 2.0 ** (e + 1) <= amax:
        e += 1
    return int(min(max(e - 7, -127), 127))


def quantize_fp8_rows(M) -> np.ndarray:
    """Dequantized value of every entry of M (rows x K, K a multiple of 32)
    after per-row, per-32-column E8M0 scaling and E4M3 rounding."""
    M = np.asarray(M, dtype=np.float64)
    rows, K = M.shape
    out = np.empty_like(M)
    for r in range(rows):
        for b in range(K // 32):
            blk = M[r, 32 * b:32 * (b + 1)]
            e = block_scale_exponent(float(np.abs(blk).max()))
            out[r, 32 * b:32 * (b + 1)] = round_e4m3(np.ldexp(blk, -e)) * 2.0 ** e
    return out


def quantize(M, prec: str, axis: int = 1) -> np.ndarray:
    """Operand M as the update uses it.  For FP8 the 32-value blocks run
    along `axis` (1: rows of L21 = A; 0: columns of U12 = B)."""
    if prec == "fp32":
        return np.asarray(M, dtype=np.float32).astype(np.float64)
    if prec == "fp16":
        return round_fp16(M)
    if prec == "bf16":
        return round_bf16(M)
    if prec == "fp8":
        return quantize_fp8_rows(M) if axis == 1 else quantize_fp8_rows(np.asarray(M).T).T
    raise ValueError(prec)


def gemm_update(C, A, B, prec: str):
    """C - A_q B_q in float64 with the operands rounded as the update rounds
    them (A: m x k, blocks along its rows; B: k x n, blocks along its
    columns).  Also returns |A_q| |B_q| for error bounds."""
    Aq = quantize(A, prec, axis=1)
    Bq = quantize(B, prec, axis=0)
    return np.asarray(C, dtype=np.float64) - Aq @ Bq, np.abs(Aq) @ np.abs(Bq)

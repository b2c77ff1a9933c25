"""Pins of the oracle's low-precision operand formats (oracle/lowp.py)
against library converters and the formats' definitions (CPU only)."""
import numpy as np
import pytest

from oracle import lowp


def _samples(seed=0, count=20000):
    g = np.random.default_rng(seed)
    x = g.standard_normal(count) * np.exp2(g.integers(-30, 30, count))
    edge = np.array([0.0, -0.0, 1.0, -1.0, 2.0 ** -24, 2.0 ** -14, 65504.0, 65519.9, 65520.0,
                     3.0e-8, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 1.0 + 2.0 ** -8,
                     1.0 + 3 * 2.0 ** -8, 448.0, 464.0, 2.0 ** -9, 3 * 2.0 ** -10])
    return np.concatenate([x, edge, -edge])


def test_fp16_matches_numpy_float16():
    x = _samples(1)
    assert np.array_equal(lowp.round_fp16(x), x.astype(np.float16).astype(np.float64))


def test_bf16_matches_torch_bfloat16():
    import torch

    x = _samples(2)
    x = x[np.abs(x) < 1e30]
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    # torch rounds from FP32; the values here are FP32-exact only after that
    # first rounding, so round the oracle's input to FP32 as well
    got = lowp.round_bf16(x.astype(np.float32).astype(np.float64))
    assert np.array_equal(got, ref)


def test_e4m3_grid_and_saturation():
    vals = lowp.e4m3_values()
    assert len(vals) == 127 and vals[-1] == 448.0 and vals[1] == 2.0 ** -9
    # every representable value is kept, negatives too
    assert np.array_equal(lowp.round_e4m3(vals), vals)
    assert np.array_equal(lowp.round_e4m3(-vals), -vals)
    # midpoints go to the neighbour with an even significand
    mids = 0.5 * (vals[1:] + vals[:-1])
    r = lowp.round_e4m3(mids)
    for lo, hi, m, got in zip(vals[:-1], vals[1:], mids, r):
        assert got in (lo, hi)
        code = np.searchsorted(vals, got)
        assert code % 2 == 0, (lo, hi, m, got)
    # saturation instead of overflow
    assert lowp.round_e4m3(np.array([500.0, -1e9]))[0] == 448.0
    assert lowp.round_e4m3(np.array([500.0, -1e9]))[1] == -448.0


def test_e4m3_matches_torch_float8():
    import torch

    x = _samples(3)
    x = x[np.abs(x) <= 448.0].astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(lowp.round_e4m3(x), ref)


@pytest.mark.parametrize("amax", [1.0, 3.0, 255.9, 256.0, 2.0 ** -100, 1e30])
def test_block_scale_range(amax):
    e = lowp.block_scale_exponent(amax)
    assert 2.0 ** 7 <= amax * 2.0 ** -e < 2.0 ** 8
    assert lowp.block_scale_exponent(0.0) == -127


def test_fp8_blocks_are_independent():
    """Blocks of 32 along a row scale separately: a block 2^12 larger next to
    one 2^-12 smaller keeps both at E4M3 relative accuracy."""
    g = np.random.default_rng(4)
    row = g.uniform(0.5, 1.0, (1, 64))
    row[0, :32] *= 2.0 ** 12
    row[0, 32:] *= 2.0 ** -12
    q = lowp.quantize_fp8_rows(row)
    assert np.all(np.abs(q - row) <= 2.0 ** -4 * np.abs(row))
    # columns of B block along K (axis 0)
    qb = lowp.quantize(row.T, "fp8", axis=0)
    assert np.array_equal(qb, q.T)


def test_gemm_update_fp32_is_exact_product():
    g = np.random.default_rng(5)
    A = g.standard_normal((7, 64)).astype(np.float32)
    B = g.standard_normal((64, 5)).astype(np.float32)
    C = g.standard_normal((7, 5)).astype(np.float32)
    D, bound = lowp.gemm_update(C, A, B, "fp32")
    assert np.allclose(D, C.astype(np.float64) - A.astype(np.float64) @ B.astype(np.float64),
                       rtol=0, atol=1e-12)
    assert np.all(bound >= 0)

"""Storage-format pins: Table 1 (unit roundoff), Table 2 (dynamic range) and
the rounding used by the oracle's decoded product and by the generator."""

import math

import numpy as np
import pytest
import torch

import oracle
from hmgen.hmatrix import round_to as gen_round, DT_F32, DT_F16, DT_BF16
from conftest import golden

FMT_DT = {"fp32": DT_F32, "fp16": DT_F16, "bf16": DT_BF16}
ORACLE_ROUND = {"fp32": oracle.round_f32, "fp16": oracle.round_f16, "bf16": oracle.round_bf16}


@pytest.mark.parametrize("row", golden("table1_unit_roundoff.txt"), ids=lambda r: r[0])
def test_table1_unit_roundoff(row):
    fmt, e, m, bits, printed = row[0], int(row[1]), int(row[2]), int(row[3]), float(row[4])
    assert 1 + e + m == bits
    u = 2.0 ** -(m + 1)
    # printed to two significant digits, halves rounded up (2^-4 = 0.0625 -> 6.3e-2)
    exp10 = math.floor(math.log10(u))
    scaled = u / 10.0 ** (exp10 - 1)
    assert math.floor(scaled + 0.5) * 10.0 ** (exp10 - 1) == pytest.approx(printed, rel=1e-12)
    assert oracle.UNIT_ROUNDOFF[fmt] == u
    assert oracle.oracle.FORMAT_BITS[fmt] == (e, m)


@pytest.mark.parametrize("row", golden("table2_dynamic_range.txt"), ids=lambda r: r[0])
def test_table2_dynamic_range(row):
    fmt, printed = row[0], int(row[1])
    assert math.floor(oracle.dynamic_range(fmt)) == printed


def _samples(seed=0, count=200000, lo=-30, hi=30):
    rng = np.random.default_rng(seed)
    mant = rng.uniform(1.0, 2.0, count)
    ex = rng.integers(lo, hi, count)
    sign = rng.choice([-1.0, 1.0], count)
    return sign * np.ldexp(mant, ex)


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16"])
def test_rounding_meets_unit_roundoff_tightly(fmt):
    # Normal range only: |fl(x)-x| <= u|x| must hold and be nearly attained.
    lo, hi = (-12, 14) if fmt == "fp16" else (-100, 100)
    x = _samples(1, lo=lo, hi=hi)
    r = ORACLE_ROUND[fmt](x)
    rel = np.abs(r - x) / np.abs(x)
    u = oracle.UNIT_ROUNDOFF[fmt]
    assert rel.max() <= u
    assert rel.max() > 0.95 * u


def test_fp16_matches_torch_and_limits():
    # torch converts FP64 -> FP16 through FP32 (two roundings), so compare on
    # FP32-representable inputs, where its second rounding is the only one.
    x = _samples(2, lo=-30, hi=17).astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x).to(torch.float16).to(torch.float64).numpy()
    with np.errstate(over="ignore"):
        np.testing.assert_array_equal(oracle.round_f16(x), ref)
    # single rounding from FP64: nearer neighbour wins even where FP32 would tie
    v = -1764.5000177825455
    assert oracle.round_f16(np.array([v]))[0] == -1765.0
    assert oracle.round_f16(np.array([65519.0]))[0] == 65504.0
    with np.errstate(over="ignore"):
        assert np.isinf(oracle.round_f16(np.array([65520.0]))[0])
    assert oracle.round_f16(np.array([2.0 ** -25]))[0] == 0.0          # tie to even (zero)
    assert oracle.round_f16(np.array([3 * 2.0 ** -25]))[0] == 2.0 ** -23


def test_bf16_definition_cases():
    r = oracle.round_bf16
    one = 1.0
    assert r(np.array([one + 2.0 ** -8]))[0] == one                       # tie -> even
    assert r(np.array([one + 3 * 2.0 ** -8]))[0] == one + 2.0 ** -6       # tie -> even (up)
    assert r(np.array([-(one + 2.0 ** -8)]))[0] == -one
    # rounded once from FP64: no double rounding through FP32
    assert r(np.array([one + 2.0 ** -8 + 2.0 ** -30]))[0] == one + 2.0 ** -7
    fmax = oracle.FORMAT_LIMITS["bf16"][0]
    assert r(np.array([fmax]))[0] == fmax
    assert np.isinf(r(np.array([(2 - 2.0 ** -8) * 2.0 ** 127]))[0])
    assert r(np.array([2.0 ** -134]))[0] == 0.0                           # half of min subnormal
    assert r(np.array([3 * 2.0 ** -134]))[0] == 2.0 ** -132


def test_bf16_matches_torch_on_fp32_values():
    # torch's float32 -> bfloat16 cast is RNE; on FP32-representable inputs a
    # single rounding from FP64 must agree with it.
    x = _samples(3, lo=-120, hi=120).astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.round_bf16(x), ref)


@pytest.mark.parametrize("fmt", ["fp32", "fp16", "bf16"])
def test_generator_and_oracle_rounding_agree(fmt):
    # Two independent implementations of RNE from FP64 must agree bit for bit,
    # including subnormals and ties.
    x = np.concatenate([_samples(4, lo=-150, hi=130),
                        np.ldexp(np.arange(-40, 40, dtype=np.float64) + 0.5, -140),
                        np.array([0.0, -0.0, 1 + 2.0 ** -8, 1 + 2.0 ** -11, 1 + 2.0 ** -24])])
    with np.errstate(over="ignore"):
        a = ORACLE_ROUND[fmt](x)
    b = gen_round(x, FMT_DT[fmt])
    np.testing.assert_array_equal(a, b)

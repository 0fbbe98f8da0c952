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


# ------------------------------------------------------------------ DFL (Sec. 3.2)

def _dfl_by_bits(x: np.ndarray, nbytes: int) -> np.ndarray:
    """Independent form of DFL rounding: keep the leading nbytes bytes of
    each FP64 encoding, rounding the dropped bits to nearest, ties to the
    even kept pattern, with integer arithmetic on the bit pattern (a carry
    runs into the exponent field)."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64).astype(object)
    drop = 64 - 8 * nbytes
    out = []
    for v in b:
        kept, rem, half = v >> drop, v & ((1 << drop) - 1), 1 << (drop - 1)
        if rem > half or (rem == half and kept & 1):
            kept += 1
        out.append((kept << drop) & ((1 << 64) - 1))
    return np.array(out, dtype=np.uint64).view(np.float64)


@pytest.mark.parametrize("nbytes", [4, 5, 6])
def test_dfl_matches_bit_pattern_rounding(nbytes):
    """round_dfl (frexp / rint, from the value) equals rounding of the bit
    pattern, over magnitudes from FP64 subnormals to near the largest finite
    value and over exact ties."""
    rng = np.random.default_rng(nbytes)
    x = rng.standard_normal(3000) * np.exp2(rng.integers(-1060, 1000, 3000).astype(float))
    m = 8 * nbytes - 12
    # exact ties: kept pattern odd and even, dropped part exactly one half
    k = rng.integers(1 << m, 1 << (m + 1), 400).astype(float)
    ties = np.ldexp(k + 0.5, rng.integers(-900, 900, 400) - m) * rng.choice([-1.0, 1.0], 400)
    x = np.concatenate([x, ties, [5e-324, -5e-324, 2.2250738585072014e-308, 1.7976931348623157e308]])
    x = x[np.isfinite(x)]
    got = oracle.round_to(x, {4: oracle.DFL32, 5: oracle.DFL40, 6: oracle.DFL48}[nbytes])
    want = _dfl_by_bits(x, nbytes)
    both_inf = np.isinf(got) & np.isinf(want) & (np.sign(got) == np.sign(want))
    assert np.array_equal(got[~both_inf].view(np.uint64), want[~both_inf].view(np.uint64))


def test_dfl_definition_cases():
    """Hand-worked DFL32 values (20 explicit mantissa bits, FP64 exponent)."""
    r = lambda v: float(oracle.round_dfl(np.array([v]), 4)[0])
    u = 2.0 ** -20                                   # spacing of the kept mantissa at 1
    assert r(1 + u / 2) == 1.0                       # tie, kept pattern even: down
    assert r(1 + 3 * u / 2) == 1 + 2 * u             # tie, kept pattern odd: up to even
    assert r(1 + u / 2 + 2.0 ** -52) == 1 + u        # just above the tie: up
    assert r(-(1 + u / 2)) == -1.0                   # sign carried, same rule
    assert r(2 - 2.0 ** -30) == 2.0                  # carry into the exponent
    assert r(1e300) == pytest.approx(1e300, rel=2.0 ** -21)   # FP64 range kept (BF16 / FP32 would overflow)
    assert r(1e-300) == pytest.approx(1e-300, rel=2.0 ** -21)
    assert oracle.round_dfl(np.array([0.1]), 8)[0] == 0.1     # 8 bytes: FP64 itself


@pytest.mark.parametrize("nbytes", [4, 5, 6])
def test_dfl_unit_roundoff(nbytes):
    """|fl(x) - x| <= 2^-(m+1) |x| for normal x, m = 8 nbytes - 12, and the
    bound is reached (to within 1%) on random values."""
    m = 8 * nbytes - 12
    rng = np.random.default_rng(7)
    x = rng.uniform(0.5, 1.0, 200000) * np.exp2(rng.integers(-500, 500, 200000).astype(float))
    rel = np.abs(oracle.round_dfl(x, nbytes) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -(m + 1)
    assert rel.max() >= 0.99 * 2.0 ** -(m + 1)


def test_dfl_format_choice():
    """Sec. 3.2: 1 + 11 + m_eps bits, the mantissa increased to fill whole
    bytes; m_eps = ceil(log2(1/eps)) (the reading used here)."""
    import hmgen
    for eps, m, nbytes in ((1e-6, 20, 4), (1e-8, 27, 5), (1e-10, 34, 6), (1e-4, 14, 4)):
        assert hmgen.dfl_mantissa_bits(eps) == m
        assert (1 + 11 + m + 7) // 8 == max(nbytes, (1 + 11 + m + 7) // 8)
        assert hmgen.dfl_format(eps) == {4: oracle.DFL32, 5: oracle.DFL40, 6: oracle.DFL48}[nbytes]
        # the kept mantissa's unit roundoff meets eps / 2
        assert 2.0 ** -(8 * nbytes - 12 + 1) <= eps / 2
    assert hmgen.dfl_format(1e-12) == oracle.F64                 # 7 bytes: FP64 instead


# ------------------------------------------------------------------ AFLP (Sec. 3.2)

def test_aflp_worked_examples():
    """Exponent bits by hand: values shifted to d = |v| / 2^k + 1; the
    exponent field spans the binary exponents 0 .. top of d (0 is zero's
    code), so e = bit length of top, unless rounding the largest d opens
    the next binade."""
    p = lambda v, nb: oracle.aflp_params(np.array(v, dtype=float), nb)
    assert p([1.0, 6.0], 3) == (0, 2, 21)            # d in [2, 7]: top 2
    assert p([1.0, 7.0], 3) == (0, 2, 21)            # d = 8: top 3 still fits two bits
    assert p([1.0, 15.0], 3) == (0, 3, 20)           # d = 16: top 4 needs three
    assert p([1.0, 1000.0], 3) == (0, 4, 19)         # d = 1001: top 9
    assert p([-3.0, 0.75, 0.0], 4) == (-1, 2, 29)    # 2^-1 <= 0.75; d = 3 / 0.5 + 1 = 7; zero ignored
    # rounding the largest value up opens a binade: d = 15.9999 needs 16 at
    # 13 mantissa bits (spacing 2^-10), so one more exponent bit
    assert p([1.0, 14.9999], 2) == (0, 3, 12)
    assert p([1.0, 14.99], 2) == (0, 2, 13)          # 15.99 stays below 16
    # the same value decoded: d rounds to 16 at 12 bits, v = (16 - 1) 2^0
    assert oracle.round_aflp(np.array([1.0, 14.9999]), 2)[1] == 15.0
    assert p([0.0, -0.0], 2) == (0, 0, 15)           # no nonzeros
    assert p([3.0], 4) == (1, 1, 30)                 # one value: d = 2.5


@pytest.mark.parametrize("nbytes", [2, 3, 4, 5, 6])
def test_aflp_unit_binade_is_fixed_point(nbytes):
    """Special case in closed form: a block whose magnitudes lie in [1, 2)
    has k = 0, e = 1 and m = 8 nbytes - 2, and AFLP rounding is then
    rounding to the fixed-point grid of step 2^-(m-1), ties to even.
    The inputs lie on FP64's grid at 2 (multiples of 2^-51), so d = |v| + 1
    is exact."""
    rng = np.random.default_rng(nbytes)
    m = 8 * nbytes - 2
    q = rng.integers(0, 2 ** 51, 4000)
    mag = 1.0 + q.astype(np.float64) * 2.0 ** -51
    mag = np.concatenate([[1.0], mag[mag < 1.75]])
    # exact ties on the step 2^-(m-1): odd and even neighbours
    t = rng.integers(2 ** (m - 1), int(1.7 * 2 ** (m - 1)), 300)
    mag = np.concatenate([mag, (t + 0.5) * 2.0 ** -(m - 1)])
    x = mag * rng.choice([-1.0, 1.0], mag.size)
    assert oracle.aflp_params(x, nbytes) == (0, 1, m)
    want = np.copysign(np.rint(mag * 2.0 ** (m - 1)) * 2.0 ** -(m - 1), x)
    np.testing.assert_array_equal(oracle.round_aflp(x, nbytes), want)


def _aflp_block(rng, n, decades):
    """Signed values with magnitudes log-uniform over `decades` decades,
    a few exact zeros."""
    x = rng.choice([-1.0, 1.0], n) * 10.0 ** rng.uniform(-decades, 0, n) * 10.0 ** rng.uniform(-5, 5)
    x[rng.integers(0, n, 3)] = 0.0
    return x


@pytest.mark.parametrize("nbytes", [2, 3, 4, 5, 6])
def test_aflp_error_bound_and_layout(nbytes):
    """|v - fl(v)| <= (2^-(m+1) + 2^-52) (|v| + 2^k) with 2^k at or below the
    smallest nonzero magnitude; 1 + e + m fills the bytes; zeros stay zero,
    signs are kept; e is the fewest bits: with e - 1 of them the largest
    rounded value falls outside the field."""
    rng = np.random.default_rng(100 + nbytes)
    for decades in (0.5, 3, 12, 60):
        x = _aflp_block(rng, 3000, decades)
        k, e, m = oracle.aflp_params(x, nbytes)
        assert 1 + e + m == 8 * nbytes
        nzm = np.abs(x[x != 0]).min()
        assert 2.0 ** k <= nzm < 2.0 ** (k + 1)
        r = oracle.round_aflp(x, nbytes)
        assert np.all(r[x == 0] == 0)
        assert np.all(np.sign(r) == np.sign(x))
        bound = (2.0 ** -(m + 1) + 2.0 ** -52) * (np.abs(x) + 2.0 ** k)
        assert np.all(np.abs(r - x) <= bound)
        np.testing.assert_array_equal(oracle.round_aflp(-x, nbytes), -r)
        # minimality of e, from Python floats: the largest shifted value
        # rounded to m + 1 mantissa bits has binary exponent >= 2^(e-1)
        if e >= 1:
            import math
            dmax = math.ldexp(float(np.abs(x).max()), -k) + 1.0
            f, ex = math.frexp(dmax)
            dr = math.ldexp(round(math.ldexp(f, m + 2)), ex - m - 2)
            assert math.frexp(dr)[1] - 1 >= 2 ** (e - 1)


def test_aflp_nearest_code_brute_force():
    """Every rounded value is a code of the block's format and is the code
    nearest to the input (all 2^15 magnitudes of a 2-byte format listed)."""
    rng = np.random.default_rng(5)
    for decades in (1, 4, 9):
        x = _aflp_block(rng, 1500, decades)
        k, e, m = oracle.aflp_params(x, 2)
        j = np.arange(1, 2 ** e, dtype=np.float64)[:, None]
        f = np.arange(2 ** m, dtype=np.float64)[None, :]
        codes = np.sort(np.concatenate([[0.0], ((2.0 ** j * (1 + f * 2.0 ** -m) - 1) * 2.0 ** k).ravel()]))
        r = np.abs(oracle.round_aflp(x, 2))
        a = np.abs(x)
        pos = np.searchsorted(codes, r)
        assert np.all(codes[np.minimum(pos, codes.size - 1)] == r)
        i = np.clip(np.searchsorted(codes, a), 1, codes.size - 1)
        best = np.minimum(np.abs(codes[i] - a), np.abs(codes[i - 1] - a))
        assert np.all(np.abs(r - a) <= best + 2.0 ** -52 * (a + 2.0 ** k))


def test_aflp_rejects_unrepresentable_blocks():
    with pytest.raises(ValueError):
        oracle.aflp_params(np.array([1.0, np.inf]), 4)
    with pytest.raises(ValueError):
        oracle.aflp_params(np.array([1e-300, 1e300]), 4)      # shifted range overflows
    np.testing.assert_array_equal(oracle.round_aflp(np.zeros(5), 3), np.zeros(5))


# ------------------------------------------------------------------ BFL (Sec. 3.2)

def _keep_top_bits(x: np.ndarray, m: int) -> np.ndarray:
    """Independent rounding of FP64 values to m explicit mantissa bits on
    the bit pattern (integer RNE of the dropped bits; a carry runs into the
    exponent): the significand rounding of any binary format with m bits,
    whatever its exponent range, for values inside that range."""
    b = np.ascontiguousarray(x, dtype=np.float64).view(np.uint64).astype(object)
    drop = 52 - m
    out = []
    for v in b:
        kept, rem, half = v >> drop, v & ((1 << drop) - 1), 1 << (drop - 1)
        if rem > half or (rem == half and kept & 1):
            kept += 1
        out.append((kept << drop) & ((1 << 64) - 1))
    return np.array(out, dtype=np.uint64).view(np.float64)


def test_bfl_four_bytes_is_fp32():
    """BFL at 4 bytes (8 exponent, 23 mantissa bits) is FP32: equal to
    numpy's correctly rounded float32 conversion over FP32's normal range."""
    rng = np.random.default_rng(21)
    x = rng.standard_normal(20000) * np.exp2(rng.integers(-120, 120, 20000).astype(float))
    x = x[np.abs(x) >= 2.0 ** -126]                  # FP32's normal range (subnormals flush)
    want = x.astype(np.float32).astype(np.float64)
    np.testing.assert_array_equal(oracle.round_bfl(x, 4), want)


@pytest.mark.parametrize("nbytes", [2, 3, 5, 6])
def test_bfl_matches_bit_pattern_rounding(nbytes):
    """Inside FP32's normal range BFL rounding equals rounding the FP64 bit
    pattern to m = 8 nbytes - 9 mantissa bits (exact ties included)."""
    m = 8 * nbytes - 9
    rng = np.random.default_rng(nbytes + 30)
    x = rng.standard_normal(3000) * np.exp2(rng.integers(-110, 110, 3000).astype(float))
    k = rng.integers(1 << m, 1 << (m + 1), 300).astype(float)
    ties = np.ldexp(k + 0.5, rng.integers(-100, 100, 300) - m) * rng.choice([-1.0, 1.0], 300)
    x = np.concatenate([x, ties])
    got = oracle.round_bfl(x, nbytes)
    assert np.array_equal(got.view(np.uint64), _keep_top_bits(x, m).view(np.uint64))
    rel = np.abs(got - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -(m + 1)


def test_bfl_definition_cases():
    """FP32's exponent range at every width: 2^-126 is the smallest value
    kept (a value that rounds up to it is kept, smaller ones flush to zero),
    and values rounding to 2^128 or beyond are rejected; 40 bits carry 31
    mantissa bits."""
    r = lambda v, nb=5: float(oracle.round_bfl(np.array([v]), nb)[0])
    tiny = 2.0 ** -126
    assert r(tiny) == tiny and r(-tiny) == -tiny
    assert r(tiny * (1 - 2.0 ** -40)) == tiny                     # rounds up into the normal range
    assert r(tiny * 0.75) == 0.0 and r(1e-300) == 0.0
    assert r(1 + 2.0 ** -31) == 1 + 2.0 ** -31                    # 31 explicit bits at 5 bytes
    assert r(1 + 2.0 ** -32) == 1.0                               # tie, even: down
    assert r(1 + 3 * 2.0 ** -32) == 1 + 2.0 ** -30                # tie, odd: up
    assert r(3e38, 6) == pytest.approx(3e38, rel=2.0 ** -39)
    with pytest.raises(ValueError):
        oracle.round_bfl(np.array([3.5e38]), 5)                   # beyond FP32's range
    with pytest.raises(ValueError):
        oracle.round_bfl(np.array([np.nan]), 3)
    assert oracle.round_to(np.array([0.1]), oracle.BFL40)[0] == r(0.1)


def test_bfl_format_choice():
    """Sec. 3.2: 1 + 8 + m_eps bits, the mantissa increased to whole bytes
    (m_eps as for DFL); 2 and 4 bytes are BF16 and FP32."""
    import hmgen
    from hmgen.hmatrix import DT_BF16, DT_F32, DT_BFL24, DT_BFL40, DT_BFL48, DT_F64
    for eps, dt in ((1e-2, DT_BF16), (1e-4, DT_BFL24), (1e-6, DT_F32), (1e-8, DT_BFL40), (1e-10, DT_BFL48),
                    (1e-13, DT_F64)):
        assert hmgen.bfl_format(eps) == dt, eps
    assert (DT_BFL24, DT_BFL40, DT_BFL48) == (oracle.BFL24, oracle.BFL40, oracle.BFL48)


def _aflp_variant(x, nbytes, shift=1.0, pow2_scale=True, e_delta=0):
    """AFLP rounding re-done with knobs for planted mistakes: the shift added
    after scaling, the scale (a power of two, or the smallest magnitude
    itself) and an error in the exponent bit count.  With the defaults it
    must reproduce oracle.round_aflp."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x[x != 0])
    k = int(np.frexp(a.min())[1]) - 1
    scale = 2.0 ** k if pow2_scale else a.min()
    e = oracle.aflp_params(x, nbytes)[1] + e_delta
    m = 8 * nbytes - 1 - e
    out = np.zeros_like(x)
    nz = x != 0
    d = np.abs(x[nz]) / scale + shift
    _, ex = np.frexp(d)
    lsb = ex - 1 - m
    dr = np.ldexp(np.rint(np.ldexp(d, -lsb)), lsb)
    # a field of e bits holds binary exponents below 2^e: larger ones saturate
    dr = np.minimum(dr, np.ldexp(2.0 - 2.0 ** -m, 2 ** e - 1))
    out[nz] = np.copysign((dr - shift) * scale, x[nz])
    return out


def test_aflp_planted_mistakes_are_caught():
    """Plausible mistakes in AFLP rounding (no shift by 1, the smallest
    magnitude as the scale, one exponent bit too few) each break a pin:
    the unit-binade closed form, the error bound, or the nearest-code
    brute force."""
    rng = np.random.default_rng(9)
    m2 = 8 * 3 - 2
    unit = 1.0 + rng.integers(0, 2 ** 51, 500).astype(np.float64) * 2.0 ** -51
    unit = unit[unit < 1.75] * rng.choice([-1.0, 1.0], unit[unit < 1.75].size)
    closed = np.copysign(np.rint(np.abs(unit) * 2.0 ** (m2 - 1)) * 2.0 ** -(m2 - 1), unit)
    wide = _aflp_block(rng, 1500, 9)
    k, e, m = oracle.aflp_params(wide, 2)
    bound = (2.0 ** -(m + 1) + 2.0 ** -52) * (np.abs(wide) + 2.0 ** k)

    def codebook_ok(r):
        j = np.arange(1, 2 ** e, dtype=np.float64)[:, None]
        f = np.arange(2 ** m, dtype=np.float64)[None, :]
        codes = np.sort(np.concatenate([[0.0], ((2.0 ** j * (1 + f * 2.0 ** -m) - 1) * 2.0 ** k).ravel()]))
        r = np.abs(r)
        pos = np.minimum(np.searchsorted(codes, r), codes.size - 1)
        return bool(np.all(codes[pos] == r))

    def pins_hold(fn):
        return (np.array_equal(fn(unit, 3), closed) and np.all(np.abs(fn(wide, 2) - wide) <= bound)
                and codebook_ok(fn(wide, 2)))

    # the knob-free variant is the oracle, and it passes
    np.testing.assert_array_equal(_aflp_variant(wide, 2), oracle.round_aflp(wide, 2))
    assert pins_hold(lambda v, nb: oracle.round_aflp(v, nb))
    for mistake in (lambda v, nb: _aflp_variant(v, nb, shift=0.0),
                    lambda v, nb: _aflp_variant(v, nb, pow2_scale=False),
                    lambda v, nb: _aflp_variant(v, nb, e_delta=-1)):
        assert not pins_hold(mistake)


@pytest.mark.parametrize("kind,nbytes", [("dfl", 3), ("dfl", 5), ("bfl", 3), ("bfl", 5), ("bfl", 6),
                                         ("aflp", 2), ("aflp", 4), ("aflp", 6)])
def test_byte_aligned_rounding_invariants(kind, nbytes):
    """Properties of any round-to-nearest: monotone (x <= y gives
    fl(x) <= fl(y)), idempotent (rounded values round to themselves; for
    AFLP with the block's own parameters unchanged) and odd."""
    fn = {"dfl": oracle.round_dfl, "bfl": oracle.round_bfl, "aflp": oracle.round_aflp}[kind]
    rng = np.random.default_rng(nbytes + len(kind))
    x = np.sort(rng.choice([-1.0, 1.0], 4000) * 10.0 ** rng.uniform(-12, 12, 4000))
    r = fn(x, nbytes)
    assert np.all(np.diff(r) >= 0)
    np.testing.assert_array_equal(fn(r, nbytes), r)
    np.testing.assert_array_equal(fn(-x, nbytes), -r)
    if kind == "aflp":
        assert oracle.aflp_params(r, nbytes) == oracle.aflp_params(x, nbytes)

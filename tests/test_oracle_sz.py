"""Pins for the reconstruction oracle (oracle/sz.py) against facts that do not
come from the oracle itself: a hand-worked example (tests/golden/), brute-force
box sums, the seven-neighbour Lorenzo predictor written out point by point,
the generator's own prequantized field and the error bound it guarantees."""
import itertools

import numpy as np
import pytest

import hdsynth
from conftest import load_golden
from oracle import sz


def _ints(g, key):
    return [int(v) for v in g[key][0]]


def test_hand_worked_2x2x2():
    g = load_golden("lorenzo_2x2x2.txt")
    shape = tuple(_ints(g, "shape"))
    idx, val = _ints(g, "outlier")
    q, x = sz.reconstruct(np.array(_ints(g, "codes"), np.uint16), shape, int(g["radius"][0][0]),
                          np.array([idx], np.uint64), np.array([val], np.int32), float(g["eb"][0][0]))
    assert q.reshape(-1).tolist() == _ints(g, "q")
    assert x.reshape(-1).tolist() == [float(v) for v in g["value"][0]]
    r = sz.residuals(np.array(_ints(g, "codes"), np.uint16), 512, np.array([idx], np.uint64),
                     np.array([val], np.int32))
    assert r.tolist() == _ints(g, "residual")


def _predictor_residual(q):
    """Residual of the first-order 3-D Lorenzo predictor, point by point."""
    ni, nj, nk = q.shape

    def at(i, j, k):
        return int(q[i, j, k]) if i >= 0 and j >= 0 and k >= 0 else 0

    r = np.zeros(q.shape, np.int64)
    for i, j, k in itertools.product(range(ni), range(nj), range(nk)):
        pred = (at(i - 1, j, k) + at(i, j - 1, k) + at(i, j, k - 1) - at(i - 1, j - 1, k) - at(i - 1, j, k - 1)
                - at(i, j - 1, k - 1) + at(i - 1, j - 1, k - 1))
        r[i, j, k] = at(i, j, k) - pred
    return r


@pytest.mark.parametrize("shape", [(1, 1, 7), (1, 5, 3), (3, 4, 5), (4, 1, 6), (2, 3, 1)])
def test_inverse_is_box_sum_brute_force(shape):
    rng = np.random.default_rng(sum(shape))
    r = rng.integers(-50, 50, size=shape)
    q = sz.inverse_lorenzo(r.reshape(-1), shape)
    for i, j, k in itertools.product(*(range(n) for n in shape)):
        assert q[i, j, k] == r[: i + 1, : j + 1, : k + 1].sum()


@pytest.mark.parametrize("shape", [(3, 4, 5), (5, 2, 7), (1, 6, 6)])
def test_round_trip_through_the_predictor(shape):
    rng = np.random.default_rng(11)
    q = rng.integers(-(1 << 20), 1 << 20, size=shape)
    r = _predictor_residual(q)
    assert np.array_equal(sz.inverse_lorenzo(r.reshape(-1), shape), q)


def test_generator_field_recovered_within_error_bound():
    # the generator quantizes the float32 field itself; reconstruction must give
    # back its q exactly and values within eb (plus float32 rounding of the product)
    F = hdsynth.lorenzo_field((12, 40, 96), seed=4, n_waves=2, noise_sigma=1e-3, eb=1e-3, radius=512,
                              keep_field=True)
    assert 0 < F.outlier_idx.size < F.codes.size // 4
    q, x = sz.reconstruct(F.codes, F.shape, F.radius, F.outlier_idx, F.outlier_val, F.eb)
    q_direct = np.floor(F.field.astype(np.float64) / (2 * F.eb) + 0.5).astype(np.int64)
    assert np.array_equal(q, q_direct)
    err = np.abs(x.astype(np.float64) - F.field.astype(np.float64))
    slack = np.spacing(np.abs(F.field)).astype(np.float64)      # one float32 ulp of either side
    assert (err <= F.eb * (1 + 1e-9) + 2 * slack).all()


def _round_to_bits(x, p):
    """The rational x rounded to p significant bits, ties to even (exact)."""
    from fractions import Fraction
    if x == 0:
        return Fraction(0)
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    scale = Fraction(2) ** (e - (p - 1))
    m = a / scale
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return (fl * scale) if x > 0 else -(fl * scale)


def _binary32_bits(x):
    """IEEE binary32 bit pattern of a rational that is a normal float32."""
    from fractions import Fraction
    s = 1 if x < 0 else 0
    a = abs(x)
    e = 0
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    m = a / Fraction(2) ** (e - 23)
    assert m.denominator == 1 and (1 << 23) <= m.numerator < (1 << 24)
    return (s << 31) | ((e + 127) << 23) | (m.numerator - (1 << 23))


def test_dequantize_golden_separates_double_from_float_product(golden):
    """Pins the reading "q * 2eb in double, then rounded to float32" with
    cases where a float32 product gives different bits
    (tests/golden/dequantize_f64_product.txt, worked with exact rationals)."""
    from fractions import Fraction
    g = golden("dequantize_f64_product.txt")
    assert len(g["case"]) >= 4
    for eb_s, q_s, want_s, f32_s in g["case"]:
        eb, q, want, f32_bits = float(eb_s), int(q_s), int(want_s), int(f32_s)
        two_eb = Fraction(2.0 * eb)
        exact = _binary32_bits(_round_to_bits(_round_to_bits(Fraction(q) * two_eb, 53), 24))
        f32 = _binary32_bits(_round_to_bits(_round_to_bits(Fraction(q), 24) * _round_to_bits(two_eb, 24), 24))
        assert exact == want and f32 == f32_bits and want != f32_bits
        got = sz.dequantize(np.array([q], np.int64), eb).view(np.uint32)[0]
        assert int(got) == want


def test_dequantize_single_rounding():
    q = np.array([0, 1, -1, 3, 12345, -987654, (1 << 31) - 1], np.int64)
    eb = 1e-4
    want = [np.float32(float(v) * (2 * eb)) for v in q.tolist()]     # Python float = IEEE double
    assert sz.dequantize(q, eb).tolist() == [float(w) for w in want]


def test_missing_outlier_is_an_error():
    codes = np.array([513, 0, 511, 0], np.uint16)
    with pytest.raises(sz.MissingOutlier):
        sz.residuals(codes, 512, np.array([1], np.uint64), np.array([5], np.int32))
    r = sz.residuals(codes, 512, np.array([1, 3, 9], np.uint64), np.array([5, -7, 100], np.int32))
    assert r.tolist() == [1, 5, -1, -7]


def test_list_entries_off_code_zero_are_ignored():
    codes = np.array([513, 0, 511], np.uint16)
    r = sz.residuals(codes, 512, np.array([0, 1, 2], np.uint64), np.array([77, 5, 88], np.int32))
    assert r.tolist() == [1, 5, -1]

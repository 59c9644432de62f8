"""Pins of the oracle's split storage rule (values held as float32 hi + lo).

What the arithmetic fixes, checked with exact rationals:
* hi is the float32 nearest P and lo the float32 nearest P - hi, so
  |P - (hi + lo)| <= 2^-24 |P - hi| <= 2^-48 |P| before the final sum
  while lo is a normal float32, and at most half the smallest subnormal
  spacing (2^-150) once it is not (|P| below about 2^-102);
  the sum is one round-to-nearest in float64 of the exact rational hi + lo;
* a value of float32 has lo = 0 and comes back unchanged;
* a value of at most 48 significant bits comes back exactly (lo then takes
  the remaining bits without rounding);
* the row perturbation is the largest row sum of |P - (hi + lo)|, taken
  exactly on a tiny MDP.
A wrong split (lo left out, lo formed in float32, hi truncated instead of
rounded) breaks one of these; the planted versions below must fail.
"""
from fractions import Fraction

import numpy as np

from oracle import ipi_oracle as O


def _values(n=4000, seed=3):
    rng = np.random.default_rng(seed)
    # transition probabilities over many binades, plus a few edge values
    v = rng.random(n) ** rng.integers(1, 12, size=n)
    return np.concatenate([v, [0.0, 1.0, 0.5, 1.0 / 3.0, 2.0 ** -149, 1e-30, 1.0 - 2.0 ** -53]])


def _check_split(val, hi, lo, eff):
    for v, h, l, e in zip(val, hi, lo, eff):
        fv, fh, fl = Fraction(float(v)), Fraction(float(h)), Fraction(float(l))
        # hi: the float32 nearest v (no float32 strictly closer on either side)
        up = np.nextafter(np.float32(h), np.float32(np.inf))
        dn = np.nextafter(np.float32(h), np.float32(-np.inf))
        assert abs(fv - fh) <= abs(fv - Fraction(float(up))) and abs(fv - fh) <= abs(fv - Fraction(float(dn)))
        # the two-part error bound
        assert abs(fv - fh - fl) <= max(Fraction(1, 2 ** 48) * abs(fv), Fraction(1, 2 ** 150))
        # the float64 sum: the exact rational hi + lo rounded once to nearest
        assert e == float(fh + fl)


def test_split_error_bound_and_single_rounding():
    val = _values()
    hi, lo = O.split_values(val)
    assert hi.dtype == np.float32 and lo.dtype == np.float32
    _check_split(val, hi, lo, O.split_effective(val))


def test_float32_values_are_unchanged():
    v = np.random.default_rng(5).random(1000).astype(np.float32).astype(np.float64)
    hi, lo = O.split_values(v)
    assert np.all(lo == 0.0)
    assert np.array_equal(O.split_effective(v), v)


def test_values_of_48_bits_come_back_exactly():
    rng = np.random.default_rng(9)
    k = rng.integers(0, 2 ** 47, size=2000, dtype=np.int64)
    e = rng.integers(1, 30, size=2000)
    # (2^47 + k) 2^-48 has 48 significant bits; scaled by powers of two
    v = np.ldexp((2.0 ** 47 + k.astype(np.float64)) * 2.0 ** -48, -e)
    assert np.array_equal(O.split_effective(v), v)


def test_row_perturbation_exact_on_a_tiny_mdp():
    S, A = 7, 3
    rng = np.random.default_rng(13)
    lens = rng.integers(1, 6, size=S * A)
    row_ptr = np.concatenate([[0], np.cumsum(lens)])
    val = rng.random(int(row_ptr[-1]))
    eff = O.split_effective(val)
    want = max(sum(abs(Fraction(float(val[j])) - Fraction(float(eff[j]))) for j in range(row_ptr[r], row_ptr[r + 1]))
               for r in range(S * A))
    got = O.split_row_perturbation(S, A, row_ptr, val)
    assert abs(Fraction(got) - want) <= Fraction(1, 2 ** 40) * want
    assert 0 < got <= 2.0 ** -48 * float(np.max(np.bincount(np.repeat(np.arange(S * A), lens), weights=val)))


def test_planted_wrong_splits_fail():
    val = _values(n=3000, seed=17)
    hi = val.astype(np.float32)
    wrong = {
        # lo left out
        "no_lo": (hi, np.zeros_like(hi)),
        # lo formed from float32 operands (always 0 after the rounding of P)
        "lo_in_float32": (hi, (val.astype(np.float32) - hi).astype(np.float32)),
        # hi truncated toward zero, lo rounded from the remainder
        "hi_truncated": (np.where(hi.astype(np.float64) > val, np.nextafter(hi, np.float32(0)), hi),
                         None),
    }
    for name, (h, l) in wrong.items():
        h = np.asarray(h, dtype=np.float32)
        if l is None:
            l = (val - h.astype(np.float64)).astype(np.float32)
        eff = h.astype(np.float64) + l.astype(np.float64)
        failed = False
        try:
            _check_split(val, h, l, eff)
        except AssertionError:
            failed = True
        assert failed, name

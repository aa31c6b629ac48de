"""Pins of the oracle's error-free transformations (Sec. 2.1, 2.3, 2.4)
against exact rational arithmetic and textbook properties."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import pyref

F = lambda x: Fr(float(x))  # noqa: E731


def wide_doubles(rng, n, emin=-60, emax=60):
    """Full-mantissa doubles with random sign and exponent."""
    mant = rng.integers(2 ** 52, 2 ** 53, size=n).astype(np.float64)
    e = rng.integers(emin, emax + 1, size=n)
    s = rng.choice([-1.0, 1.0], size=n)
    return s * np.ldexp(mant, e - 52)


def adversarial_pairs(rng, n):
    a = wide_doubles(rng, n)
    b = wide_doubles(rng, n)
    # equal exponents, near-cancellation, exact cancellation, zeros, ties
    k = n // 8
    b[:k] = -a[:k] * (1 + 2.0 ** -52)
    b[k:2 * k] = -a[k:2 * k]
    b[2 * k:3 * k] = a[2 * k:3 * k] * 0.75
    a[3 * k:3 * k + 4] = [0.0, -0.0, 1.0, -1.0]
    b[3 * k:3 * k + 4] = [-0.0, -0.0, 2.0 ** -53, -(2.0 ** -53)]
    b[4 * k:5 * k] = np.array([math.ulp(float(x)) / 2 for x in a[4 * k:5 * k]]) * np.sign(a[4 * k:5 * k])
    return a, b


@pytest.fixture(scope="module")
def rng():
    return np.random.Generator(np.random.PCG64(20210115))


def test_two_sum_exact(rng):
    a, b = adversarial_pairs(rng, 4000)
    s, e = oracle.prim("two_sum", a, b)
    for x, y, ss, ee in zip(a, b, s, e):
        assert ss == x + y                       # s is the rounded sum
        assert F(ss) + F(ee) == F(x) + F(y)      # error-free
        assert abs(ee) <= math.ulp(ss) / 2 or ss == 0


def test_quick_two_sum_exact_under_precondition(rng):
    a, b = adversarial_pairs(rng, 4000)
    swap = np.abs(a) < np.abs(b)
    a2 = np.where(swap, b, a)
    b2 = np.where(swap, a, b)
    s, e = oracle.prim("quick_two_sum", a2, b2)
    for x, y, ss, ee in zip(a2, b2, s, e):
        assert ss == x + y
        assert F(ss) + F(ee) == F(x) + F(y)


def test_quick_two_sum_outside_precondition_matches_formula(rng):
    # |a| < |b|: result is whatever b - (s - a) rounds to; the sum part is fl(a+b)
    a = wide_doubles(rng, 500, -80, -20)
    b = wide_doubles(rng, 500, 0, 10)
    s, e = oracle.prim("quick_two_sum", a, b)
    for x, y, ss, ee in zip(a, b, s, e):
        assert ss == x + y
        assert ee == y - (ss - x)


def test_two_prod_exact(rng):
    a = wide_doubles(rng, 4000, -200, 200)
    b = wide_doubles(rng, 4000, -200, 200)
    p, e = oracle.prim("two_prod", a, b)
    for x, y, pp, ee in zip(a, b, p, e):
        assert pp == x * y
        assert F(pp) + F(ee) == F(x) * F(y)


def test_three_sum_and_three_sum2(rng):
    n = 3000
    a, b = adversarial_pairs(rng, n)
    c = wide_doubles(rng, n, -70, 10)
    o = oracle.prim("three_sum", a, b, c)
    o2 = oracle.prim("three_sum2", a, b, c)
    for i in range(n):
        tot = F(a[i]) + F(b[i]) + F(c[i])
        assert F(o[0][i]) + F(o[1][i]) + F(o[2][i]) == tot          # ThreeSum error-free
        assert o[0][i] == c[i] + (a[i] + b[i])                      # leading term fl(c + fl(a+b))
        assert o2[0][i] == o[0][i]
        # ThreeSum2 rounds the two error terms into one
        err = abs(F(o2[0][i]) + F(o2[1][i]) - tot)
        assert err <= Fr(math.ulp(o2[1][i])) / 2


def test_vec_sum_error_free_and_top_is_recursive_sum(rng):
    n = 2000
    xs = [wide_doubles(rng, n, -10 - 30 * q, 10 - 30 * q) for q in range(4)]
    e = oracle.prim("vec_sum4", *xs)
    for i in range(n):
        tot = sum(F(x[i]) for x in xs)
        assert sum(F(ee[i]) for ee in e) == tot
        assert e[0][i] == xs[0][i] + (xs[1][i] + (xs[2][i] + xs[3][i]))
        # each error term is at most half an ulp of the partial sum it came from
        assert abs(e[1][i]) <= math.ulp(e[0][i]) / 2 or e[0][i] == 0


def _nonoverlap_terms(rng, n, k, gap=0):
    """Expansions with k non-zero terms, each below half an ulp of the one
    before (so the expansion is already normalised); gap adds extra zeros."""
    terms = [wide_doubles(rng, n, -5, 5)]
    for q in range(1, k):
        half_ulp = 0.5 * np.spacing(np.abs(terms[-1]))
        v = wide_doubles(rng, n, -1 - gap, -1)        # |v| < 1
        terms.append(half_ulp * v)
    return terms


def test_vseb_returns_representable_input_unchanged(rng):
    # three already non-overlapping terms with a zero in between
    n = 1000
    t = _nonoverlap_terms(rng, n, 3)
    r = oracle.prim("vseb3", t[0], np.zeros(n), t[1], np.zeros(n), t[2], np.zeros(n))
    for q in range(3):
        assert np.array_equal(r[q], t[q])
    r2 = oracle.prim("vseb2", t[0], t[1], np.zeros(n))
    assert np.array_equal(r2[0], t[0]) and np.array_equal(r2[1], t[1])


def test_vseb_drops_only_below_last_term(rng):
    n = 2000
    xs = [wide_doubles(rng, n, -5, 5), wide_doubles(rng, n, -55, -45), wide_doubles(rng, n, -105, -95)]
    e = oracle.prim("vec_sum3", *xs)
    r = oracle.prim("vseb2", *e)
    for i in range(n):
        tot = sum(F(x[i]) for x in xs)
        got = F(r[0][i]) + F(r[1][i])
        # what is lost is at most about one ulp of the second output term
        assert abs(got - tot) <= 2 * Fr(math.ulp(r[1][i])) + Fr(math.ulp(r[0][i])) * Fr(1, 2 ** 50)
        assert abs(r[1][i]) <= math.ulp(r[0][i])


def test_renorm4_idempotent_on_normalised_input(rng):
    n = 1000
    t = _nonoverlap_terms(rng, n, 4, gap=3)
    z = np.zeros(n)
    r = oracle.prim("renorm4", t[0], t[1], t[2], t[3], z)
    for q in range(4):
        assert np.array_equal(r[q], t[q])


def test_renorm4_accuracy_and_nonoverlap(rng):
    n = 3000
    c = [wide_doubles(rng, n, -2, 2)]
    for q in range(1, 5):
        c.append(c[-1] * rng.uniform(-1, 1, n) * 2.0 ** -50)
    r = oracle.prim("renorm4", *c)
    for i in range(n):
        tot = sum(F(x[i]) for x in c)
        got = sum(F(x[i]) for x in r)
        assert abs(got - tot) <= 2 * Fr(math.ulp(r[3][i])) + Fr(math.ulp(r[0][i])) * Fr(1, 2 ** 200)
        for q in range(3):
            if r[q][i] != 0:
                assert abs(r[q + 1][i]) <= math.ulp(r[q][i])
        assert r[0][i] == float(tot) or abs(F(r[0][i]) - tot) <= Fr(math.ulp(r[0][i]))


def test_renorm4_tail_absorbed_into_last_slot():
    # four separated terms plus a fifth: the fifth is added into the last slot
    c = [1.0, 2.0 ** -60, 2.0 ** -120, 2.0 ** -180, 2.0 ** -190]
    r = oracle.prim("renorm4", *[np.array([v]) for v in c])
    assert [float(x[0]) for x in r] == [1.0, 2.0 ** -60, 2.0 ** -120, 2.0 ** -180 + 2.0 ** -190]


@pytest.mark.parametrize("name,nin", [("quick_two_sum", 2), ("two_sum", 2), ("two_prod", 2),
                                      ("three_sum", 3), ("three_sum2", 3), ("vec_sum4", 4),
                                      ("vseb2", 3), ("vseb3", 6), ("renorm4", 5), ("vec_sum3", 3)])
def test_primitives_match_second_transcription(rng, name, nin):
    n = 1500
    cols = []
    base = wide_doubles(rng, n, -3, 3)
    for q in range(nin):
        v = base * rng.uniform(-1, 1, n) * 2.0 ** (-50 * q * rng.uniform(0.5, 1.2))
        if q and rng.uniform() < 0.3:
            v[: n // 10] = 0.0
        cols.append(v)
    got = oracle.prim(name, *cols)
    fn = {"quick_two_sum": pyref.qts, "two_sum": pyref.ts, "two_prod": pyref.tp,
          "three_sum": pyref.three_sum, "three_sum2": pyref.three_sum2,
          "vec_sum4": lambda *x: pyref.vec_sum(x), "vec_sum3": lambda *x: pyref.vec_sum(x),
          "vseb2": lambda *x: pyref.vseb(list(x), 2), "vseb3": lambda *x: pyref.vseb(list(x), 3),
          "renorm4": pyref.renorm4}[name]
    for i in range(n):
        want = fn(*[float(c[i]) for c in cols])
        for q in range(len(got)):
            assert got[q][i] == want[q], (name, i, q)

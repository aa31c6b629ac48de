"""Pins of the oracle's other TD operations of Sec. 2.3: the accurate
addition (Algorithm 3: Merge, VecSum, VSEB(3)) and TDmulq (the QD product on
zero-extended operands), and of the TD GEMM built on them."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, mp_frac
from tests.test_oracle_arith import operands

U159 = Fr(1, 2 ** 159)


def test_merge_is_the_stable_sort_by_decreasing_magnitude():
    """On normalised operands the merge equals Python's stable sort of
    (x0, x1, x2, y0, y1, y2) by decreasing |.| (x first on equal magnitudes,
    which the exact-cancellation operands exercise)."""
    x, y = operands(3, 3000, 901)
    z = oracle.prim("merge3", x[0], x[1], x[2], y[0], y[1], y[2])
    checked = ties = 0
    for i in range(x.shape[1]):
        xs, ys = list(x[:, i]), list(y[:, i])
        if not (all(abs(xs[q]) >= abs(xs[q + 1]) for q in range(2))
                and all(abs(ys[q]) >= abs(ys[q + 1]) for q in range(2))):
            continue
        want = sorted(xs + ys, key=abs, reverse=True)
        got = [z[q][i] for q in range(6)]
        assert got == want and [np.signbit(v) for v in got] == [np.signbit(v) for v in want], i
        checked += 1
        ties += abs(xs[0]) == abs(ys[0])
    assert checked > 2500 and ties > 100


def test_merge_tie_goes_to_x():
    z = oracle.prim("merge3", [1.0], [0.25], [0.0], [-1.0], [0.5], [0.0])
    assert [v[0] for v in z] == [1.0, -1.0, 0.5, 0.25, 0.0, 0.0]


def test_accurate_add_error_relative_to_the_sum():
    """The six merged terms are summed exactly (VecSum) and VSEB(3) keeps the
    leading three, so the error is relative to |x + y| itself, also under heavy
    cancellation (measured maximum 0.87 x 2^-159)."""
    x, y = operands(3, 6000, 902)
    r = oracle.vec(3, "add_acc", x, y)
    for i in range(x.shape[1]):
        X, Y, R = mp_frac(x[:, i]), mp_frac(y[:, i]), mp_frac(r[:, i])
        assert abs(R - (X + Y)) <= 2 * U159 * abs(X + Y), i


def test_accurate_add_exact_cancellation_and_single_doubles():
    rng = np.random.Generator(np.random.PCG64(903))
    x = synth.mp_uniform(rng, 3, (500,))
    r = oracle.vec(3, "add_acc", x, -x)
    assert np.all(r == 0.0)
    n = 2000
    a = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-40, 40, n)
    b = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-40, 40, n)
    xs = np.zeros((3, n)); xs[0] = a
    ys = np.zeros((3, n)); ys[0] = b
    r = oracle.vec(3, "add_acc", xs, ys)
    for i in range(n):                           # TwoSum: (fl(a+b), exact error, 0)
        s = a[i] + b[i]
        assert r[0, i] == s and Fr(r[1, i]) == Fr(a[i]) + Fr(b[i]) - Fr(s) and r[2, i] == 0


def test_mulq_error_and_single_doubles():
    """TDmulq: the QD product's four components minus the last, so the error
    is below about an ulp of the third component (measured 0.24 x 2^-159 |xy|);
    single-double operands give TwoProd exactly."""
    x, y = operands(3, 6000, 904)
    r = oracle.vec(3, "mulq", x, y)
    for i in range(x.shape[1]):
        X, Y, R = mp_frac(x[:, i]), mp_frac(y[:, i]), mp_frac(r[:, i])
        assert abs(R - X * Y) <= 2 * U159 * abs(X * Y), i
    rng = np.random.Generator(np.random.PCG64(905))
    n = 2000
    a = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-40, 40, n)
    b = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-40, 40, n)
    xs = np.zeros((3, n)); xs[0] = a
    ys = np.zeros((3, n)); ys[0] = b
    r = oracle.vec(3, "mulq", xs, ys)
    for i in range(n):
        p = a[i] * b[i]
        assert r[0, i] == p and Fr(r[1, i]) == Fr(a[i]) * Fr(b[i]) - Fr(p) and r[2, i] == 0


def test_variant_ops_only_for_td():
    x = np.zeros((2, 4))
    with pytest.raises(AssertionError):
        oracle.vec(2, "add_acc", x, x)


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_variant_gemm_bound_brute_force(variant):
    """Small GEMMs with every transpose pair: within 8 (k + 2) u (|alpha||A||B|
    + |beta||C|) of the exact result, u = 2^-150, on every entry."""
    rng = np.random.Generator(np.random.PCG64(910 + variant))
    for ta, tb in (("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")):
        m, n, k = 5, 4, 7
        A = synth.mp_uniform(rng, 3, (m, k) if ta == "T" else (k, m))
        B = synth.mp_uniform(rng, 3, (k, n) if tb == "T" else (n, k))
        C = synth.mp_uniform(rng, 3, (n, m))
        alpha = synth.mp_uniform(rng, 3, (1,))[:, 0]
        beta = synth.mp_uniform(rng, 3, (1,))[:, 0]
        got = oracle.gemm(3, ta, tb, m, n, k, alpha, A, B, beta, C, variant=variant)
        chk = GemmChecker(3, ta, tb, m, n, k, alpha, A, B, beta, C)
        r = chk.ratios(got, [(i, j) for i in range(m) for j in range(n)])
        assert r.max() <= 8 * (k + 2) / k, (variant, ta, tb, r.max())


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_variant_gemm_integers_exact(variant):
    rng = np.random.Generator(np.random.PCG64(920 + variant))
    m, n, k = 6, 5, 9
    A = np.zeros((3, k, m)); A[0] = rng.integers(-300, 300, (k, m))
    B = np.zeros((3, n, k)); B[0] = rng.integers(-300, 300, (n, k))
    one, zero = synth.mp_one(3), np.zeros(3)
    got = oracle.gemm(3, "N", "N", m, n, k, one, A, B, zero, np.zeros((3, n, m)), variant=variant)
    exact = A[0].T.astype(np.int64) @ B[0].T.astype(np.int64)
    assert np.all(got[0].T == exact) and np.all(got[1:] == 0)

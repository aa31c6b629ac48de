"""Pins of the oracle's DD/TD/QD additions and multiplications (Algorithms
1, 2, 4, 5, 6 and TDaddq) against exact rational arithmetic."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import pyref, synth
from tests.exact import mp_frac

# Error constants relative to 2^(-53P) (measured maxima on 2e4 random and
# cancelling operands: DD add 1.34, DD mul 2.80, TD add 0.25, TD mul 3.14,
# QD add 0.11, QD mul 6.28).  A dropped or mis-signed term of the algorithms
# shows up as an error about 2^53 times larger.
C_ADD = {2: 4, 3: 4, 4: 4}
C_MUL = {2: 8, 3: 16, 4: 32}


def operands(P, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = synth.mp_uniform(rng, P, (n,))
    y = synth.mp_uniform(rng, P, (n,))
    x = np.ldexp(x, rng.integers(-30, 31, n)[None])
    y = np.ldexp(y, rng.integers(-30, 31, n)[None])
    k = n // 5
    y[:, :k] = -x[:, :k]
    y[0, :k] *= 1 + 2.0 ** -50             # heavy cancellation
    y[:, k:2 * k] = -x[:, k:2 * k]          # exact cancellation
    y[P - 1, k:2 * k] += np.spacing(np.abs(x[P - 1, k:2 * k]))
    return x, y


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("op", ["add", "mul"])
def test_error_bound_against_exact(P, op):
    x, y = operands(P, 6000, 100 + P)
    r = oracle.vec(P, op, x, y)
    c = C_ADD[P] if op == "add" else C_MUL[P]
    u = Fr(1, 2 ** (53 * P))
    for i in range(x.shape[1]):
        X, Y, R = mp_frac(x[:, i]), mp_frac(y[:, i]), mp_frac(r[:, i])
        exact = X + Y if op == "add" else X * Y
        base = abs(X) + abs(Y) if op == "add" else abs(X * Y)
        assert abs(R - exact) <= c * u * base, (P, op, i)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("op", ["add", "mul"])
def test_output_is_normalised(P, op):
    x, y = operands(P, 4000, 200 + P)
    r = oracle.vec(P, op, x, y)
    for q in range(P - 1):
        nz = r[q] != 0
        assert np.all(np.abs(r[q + 1][nz]) <= np.spacing(np.abs(r[q][nz])))
        # a zero component is followed only by zeros
        assert np.all(r[q + 1][~nz] == 0)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_single_double_operands_reduce_to_twosum_twoprod(P):
    """With x = (a, 0, ..), y = (b, 0, ..) the sum is (fl(a+b), a+b-fl(a+b), 0..)
    and the product (fl(ab), ab-fl(ab), 0..): the textbook EFT results."""
    rng = np.random.Generator(np.random.PCG64(300 + P))
    n = 3000
    a = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-40, 40, n)
    b = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-40, 40, n)
    x = np.zeros((P, n)); x[0] = a
    y = np.zeros((P, n)); y[0] = b
    ra = oracle.vec(P, "add", x, y)
    rm = oracle.vec(P, "mul", x, y)
    for i in range(n):
        s = a[i] + b[i]
        assert ra[0, i] == s and Fr(ra[1, i]) == Fr(a[i]) + Fr(b[i]) - Fr(s)
        p = a[i] * b[i]
        assert rm[0, i] == p and Fr(rm[1, i]) == Fr(a[i]) * Fr(b[i]) - Fr(p)
        for q in range(2, P):
            assert ra[q, i] == 0 and rm[q, i] == 0


@pytest.mark.parametrize("P", [2, 3, 4])
def test_representable_results_are_exact(P):
    """Operands with short, well separated bit strings whose exact sum and
    product fit in P non-overlapping components come back exactly."""
    rng = np.random.Generator(np.random.PCG64(400 + P))
    n = 2000
    gap = 50
    x = np.zeros((P, n))
    y = np.zeros((P, n))
    for q in range(P):
        x[q] = rng.integers(1, 2 ** 8, n) * 2.0 ** (-gap * q - 10)
        y[q] = rng.integers(1, 2 ** 8, n) * 2.0 ** (-gap * q - 20)
    ra = oracle.vec(P, "add", x, y)
    for i in range(n):
        assert mp_frac(ra[:, i]) == mp_frac(x[:, i]) + mp_frac(y[:, i])
    # products: single-component times short multi-component operand
    x1 = np.zeros((P, n)); x1[0] = rng.integers(1, 2 ** 8, n) * 2.0 ** -3
    rm = oracle.vec(P, "mul", x1, y)
    for i in range(n):
        assert mp_frac(rm[:, i]) == mp_frac(x1[:, i]) * mp_frac(y[:, i])


@pytest.mark.parametrize("P,op", [(2, "add"), (2, "mul"), (4, "add")])
def test_bitwise_commutative(P, op):
    """DDadd, DDmul and QDadd are symmetric in their operands operation by
    operation (the TwoSum error term is unique), so swapping x and y cannot
    change a bit."""
    x, y = operands(P, 5000, 500 + P)
    assert np.array_equal(oracle.vec(P, op, x, y), oracle.vec(P, op, y, x))


def test_td_add_is_qd_add_with_zero_fourth_components():
    x, y = operands(3, 3000, 600)
    z = np.zeros((1, x.shape[1]))
    r3 = oracle.vec(3, "add", x, y)
    r4 = oracle.vec(4, "add", np.vstack([x, z]), np.vstack([y, z]))
    assert np.array_equal(r3, r4[:3])


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("op", ["add", "mul"])
def test_matches_second_transcription(P, op):
    x, y = operands(P, 1500, 700 + P)
    r = oracle.vec(P, op, x, y)
    fn = (pyref.ADD if op == "add" else pyref.MUL)[P]
    for i in range(x.shape[1]):
        want = fn([float(v) for v in x[:, i]], [float(v) for v in y[:, i]])
        assert [float(v) for v in r[:, i]] == want, (P, op, i)

"""Pins of the oracle's evaluation orders by a second transcription.

The error bounds and exactness tests elsewhere hold for any summation order
and any operand order of MUL, so they cannot tell a misread order from the
intended one.  Here the C oracle is compared bit for bit with the pure-Python
transcription in tests/pyref.py, written separately from the definitions:

* the canonical GEMM (eqn (1), Sec. 3, with the BLAS epilogue): for every
  entry one ascending chain acc = ADD(acc, MUL(op(A)_il, op(B)_lj)), then
  ADD(MUL(alpha, acc), MUL(beta, c)).  QD multiplication (Algorithm 6) is
  not commutative bit for bit, so there a swapped MUL operand order or a
  swapped epilogue changes bits; a descending chain does in every precision;
* the fixed 64-ary dot tree (Sec. 4), across two tree levels;
* Strassen's seven-product levels (Sec. 3, Fig. 5), left-to-right sums.

The inputs are seeded draws whose entries carry exponent spread, so that
rounding differs between orders.
"""
import numpy as np
import pytest

import oracle
from tests import pyref, synth

TRANS = [("N", "N"), ("N", "T"), ("T", "N"), ("T", "T")]


def spread(P, rows, cols, seed, e=12):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = synth.mp_uniform(rng, P, (cols, rows))
    return np.ldexp(X, rng.integers(-e, e + 1, (cols, rows))[None])


def operands(P, ta, tb, m, n, k, seed):
    A = spread(P, *((m, k) if ta == "N" else (k, m)), seed)
    B = spread(P, *((k, n) if tb == "N" else (n, k)), seed + 1)
    C = spread(P, m, n, seed + 2)
    alpha = synth.mp_scalar(seed % 97, "alpha", P)
    beta = synth.mp_scalar(seed % 97, "beta", P)
    return A, B, C, alpha, beta


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("ta,tb", TRANS)
def test_gemm_chain_and_epilogue(P, ta, tb):
    for idx, (m, n, k) in enumerate([(3, 2, 200), (4, 3, 37), (1, 5, 1)]):
        seed = 1000 * P + 10 * idx + TRANS.index((ta, tb))
        A, B, C, alpha, beta = operands(P, ta, tb, m, n, k, seed)
        want = pyref.gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C)
        got = oracle.gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C)
        assert np.array_equal(got, want), (m, n, k)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_gemm_special_scalars(P):
    """beta = 0 (C never read), alpha = 0, k = 0 and beta = 1 with alpha = 0."""
    m, n, k = 3, 4, 25
    A, B, C, alpha, beta = operands(P, "N", "T", m, n, k, 77 + P)
    zero, one = np.zeros(P), synth.mp_one(P)
    for al, be, kk in ((alpha, zero, k), (zero, beta, k), (alpha, beta, 0), (zero, one, k)):
        want = pyref.gemm(P, "N", "T", m, n, kk, al, A, B, be, C)
        got = oracle.gemm(P, "N", "T", m, n, kk, al, A, B, be, C)
        assert np.array_equal(got, want)
    Cnan = np.full_like(C, np.nan)
    got = oracle.gemm(P, "N", "T", m, n, k, alpha, A, B, zero, Cnan)
    assert np.array_equal(got, pyref.gemm(P, "N", "T", m, n, k, alpha, A, B, zero, C))


@pytest.mark.parametrize("P", [2, 3, 4])
def test_orders_are_distinguishable(P):
    """The inputs above do separate the readings: the descending chain gives
    other bits, and for QD so do swapped MUL operands.  (DD multiplication,
    Algorithm 2, and TD multiplication, Algorithm 4, are symmetric bit for
    bit: swapping x and y only exchanges the operands of commutative sums and
    of the two fused products added together, so there the operand order
    cannot matter.)"""
    m, n, k = 3, 2, 200
    A, B, C, alpha, beta = operands(P, "N", "N", m, n, k, 5000 + P)
    want = pyref.gemm(P, "N", "N", m, n, k, alpha, A, B, beta, C)
    rev = A[:, ::-1, :].copy(), B[:, :, ::-1].copy()     # l -> k-1-l in op(A) and op(B)
    assert not np.array_equal(pyref.gemm(P, "N", "N", m, n, k, alpha, rev[0], rev[1], beta, C), want)
    if P == 4:
        swapped = pyref.gemm(P, "T", "T", n, m, k, alpha, B, A, beta, C.transpose(0, 2, 1).copy())
        assert not np.array_equal(swapped.transpose(0, 2, 1), want)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_dot_tree(P):
    for n in (1, 63, 64, 65, 64 * 64 + 3):
        rng = np.random.Generator(np.random.PCG64(300 + n + P))
        x = np.ldexp(synth.mp_uniform(rng, P, (n,)), rng.integers(-12, 13, n)[None])
        y = np.ldexp(synth.mp_uniform(rng, P, (n,)), rng.integers(-12, 13, n)[None])
        assert np.array_equal(oracle.dot(P, x, y), np.array(pyref.dot(P, x, y))), n
    # the tree differs from one long chain on these inputs
    assert not np.array_equal(np.array(pyref.dot(P, x, y)), np.array(pyref.dot(P, x, y, fanin=n)))


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("levels,ta,tb,m,n,k", [(1, "N", "N", 4, 6, 8), (1, "T", "N", 6, 2, 4),
                                                (1, "N", "T", 2, 4, 6), (2, "T", "T", 4, 8, 4)])
def test_strassen_levels(P, levels, ta, tb, m, n, k):
    A, B, C, alpha, beta = operands(P, ta, tb, m, n, k, 900 + 7 * P + m)
    want = pyref.gemm_strassen(P, levels, ta, tb, m, n, k, alpha, A, B, beta, C)
    got = oracle.gemm_strassen(P, levels, ta, tb, m, n, k, alpha, A, B, beta, C)
    assert np.array_equal(got, want)
    # and it is not the canonical product's rounding
    assert not np.array_equal(got, pyref.gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C))


@pytest.mark.parametrize("P", [2, 3])
def test_dd_td_multiplication_is_symmetric(P):
    """The fact used above: MUL(x, y) == MUL(y, x) bit for bit for DD and TD,
    on spread random operands."""
    rng = np.random.Generator(np.random.PCG64(4242 + P))
    x = np.ldexp(synth.mp_uniform(rng, P, (4000,)), rng.integers(-40, 41, 4000)[None])
    y = np.ldexp(synth.mp_uniform(rng, P, (4000,)), rng.integers(-40, 41, 4000)[None])
    assert np.array_equal(oracle.vec(P, "mul", x, y), oracle.vec(P, "mul", y, x))


@pytest.mark.parametrize("P", [2, 3, 4])
def test_addition_is_symmetric(P):
    """ADD(x, y) == ADD(y, x) bit for bit in every precision: Algorithms 1 and
    5 start from component-wise TwoSums, whose sum and error are the same
    whatever the operand order, and continue on those results only.  So the
    order of ADD's operands (in the chain and in the epilogue) is not a
    reading that needs a pin."""
    rng = np.random.Generator(np.random.PCG64(4343 + P))
    x = np.ldexp(synth.mp_uniform(rng, P, (4000,)), rng.integers(-40, 41, 4000)[None])
    y = np.ldexp(synth.mp_uniform(rng, P, (4000,)), rng.integers(-40, 41, 4000)[None])
    y[:, :500] = -x[:, :500] * np.ldexp(1.0, -rng.integers(0, 3, 500))[None]   # cancellation
    assert np.array_equal(oracle.vec(P, "add", x, y), oracle.vec(P, "add", y, x))

"""Pins of the oracle's Strassen form (Sec. 3, Fig. 5): L levels of Strassen's
seven-product recursion over canonical-order block products."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, mp_frac

U = {2: Fr(1, 2 ** 104), 3: Fr(1, 2 ** 150), 4: Fr(1, 2 ** 200)}


def test_zero_levels_is_the_canonical_gemm():
    P, m, n, k = 3, 12, 10, 14
    A = synth.mp_matrix(21, "A", P, m, k)
    B = synth.mp_matrix(21, "B", P, k, n)
    C = synth.mp_matrix(21, "C", P, m, n)
    al, be = synth.mp_scalar(21, "alpha", P), synth.mp_scalar(21, "beta", P)
    assert np.array_equal(oracle.gemm_strassen(P, 0, "N", "N", m, n, k, al, A, B, be, C),
                          oracle.gemm(P, "N", "N", m, n, k, al, A, B, be, C))


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("levels", [1, 2, 3])
def test_integer_matrices_exact(P, levels):
    """Small integers stay exact through every block sum and product."""
    rng = np.random.Generator(np.random.PCG64(30 + P + 3 * levels))
    m, n, k = 16, 24, 32
    A = np.zeros((P, k, m)); A[0] = rng.integers(-200, 200, (k, m))
    B = np.zeros((P, n, k)); B[0] = rng.integers(-200, 200, (n, k))
    one, zero = synth.mp_one(P), np.zeros(P)
    got = oracle.gemm_strassen(P, levels, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    exact = A[0].T.astype(np.int64) @ B[0].T.astype(np.int64)
    assert np.all(got[0].T == exact) and np.all(got[1:] == 0)


def higham_strassen_bound(n, levels):
    """Strassen's normwise error constant for square n with blocks of n0 =
    n / 2^levels multiplied conventionally (Higham, Accuracy and Stability of
    Numerical Algorithms, 2nd ed., Thm 23.3):
    (n / n0)^log2(12) (n0^2 + 5 n0) - 5 n."""
    n0 = n // 2 ** levels
    return (n / n0) ** math.log2(12) * (n0 * n0 + 5 * n0) - 5 * n


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("levels", [1, 2, 3])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_normwise_bound_against_exact(P, levels, ta, tb):
    """max |C - C*| <= c * gamma * u * max|A| * max|B|, gamma the constant
    above and c = 32 the largest per-operation error constant of the
    multi-component operations (QD multiplication); every entry checked."""
    n = 16
    rng = np.random.Generator(np.random.PCG64(40 + P + 7 * levels))
    A = synth.mp_uniform(rng, P, (n, n))
    B = synth.mp_uniform(rng, P, (n, n))
    one, zero = synth.mp_one(P), np.zeros(P)
    got = oracle.gemm_strassen(P, levels, ta, tb, n, n, n, one, A, B, zero, np.zeros((P, n, n)))
    chk = GemmChecker(P, ta, tb, n, n, n, one, A, B, zero, np.zeros((P, n, n)))
    amax = max(abs(mp_frac(A[:, j, i])) for i in range(n) for j in range(n))
    bmax = max(abs(mp_frac(B[:, j, i])) for i in range(n) for j in range(n))
    bound = 32 * Fr(higham_strassen_bound(n, levels)) * U[P] * amax * bmax
    worst = Fr(0)
    for i in range(n):
        for j in range(n):
            exact, _ = chk.entry(i, j)
            worst = max(worst, abs(mp_frac(got[:, j, i]) - exact))
    assert worst <= bound, (P, levels, float(worst / bound))


@pytest.mark.parametrize("P,n,levels", [(2, 64, 2), (3, 32, 2), (4, 32, 3)])
def test_paper_matrices_lose_at_most_two_digits(P, n, levels):
    """The paper's fixed matrices through Strassen's method: at most one or
    two decimal digits lost (Sec. 3), against sqrt15 n(n-1)(3i+n-2)/6."""
    A, B = synth.paper_matrices(n, P)
    one, zero = synth.mp_one(P), np.zeros(P)
    got = oracle.gemm_strassen(P, levels, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, n)))
    for i in range(1, n + 1):
        exact = synth.paper_exact_entry(n, i)
        for j in (1, n // 2, n):
            rel = abs(mp_frac(got[:, j - 1, i - 1]) - exact) / exact
            assert rel <= 100 * U[P], (P, i, j, float(rel / U[P]))


def test_dimensions_must_split_evenly():
    P = 2
    A = np.zeros((P, 6, 6))
    with pytest.raises(AssertionError):
        oracle.gemm_strassen(P, 2, "N", "N", 6, 6, 6, synth.mp_one(P), A, A, np.zeros(P), A)

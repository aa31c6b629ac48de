"""Pins of the oracle's residue (CRT) form of the split product: the exact
product of the split form's digit integers over the full square of digit
pairs, rounded to P components."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, mp_frac

SLICES = {2: 16, 3: 23, 4: 31}


@pytest.mark.parametrize("P", [2, 3])
def test_brute_force_integer_product_and_rounding(P):
    """Tiny shapes: from the oracle's own digits, the integers A' = sum_p d_p
    128^(s-p), their exact product in Python integers, times 2^(E_i + F_j -
    14 s), rounded component by component with Python's correctly rounded
    float(Fraction) of the exact remainder; the oracle gives the same bits."""
    s = SLICES[P]
    m, n, k = 3, 4, 5
    rng = np.random.Generator(np.random.PCG64(1100 + P))
    A = synth.mp_uniform(rng, P, (k, m))
    B = synth.mp_uniform(rng, P, (n, k))
    A = np.ldexp(A, rng.integers(-8, 9, (k, m))[None])
    one, zero = synth.mp_one(P), np.zeros(P)
    got = oracle.gemm_crt(P, s, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    E = oracle.split_exponents(P, "N", 0, m, k, A)
    F = oracle.split_exponents(P, "N", 1, n, k, B)
    DA = oracle.split_slices(P, s, "N", 0, m, k, A, E).astype(np.int64)
    DB = oracle.split_slices(P, s, "N", 1, n, k, B, F).astype(np.int64)
    w = [128 ** (s - p) for p in range(1, s + 1)]
    Ai = [[sum(int(DA[p, i, l]) * w[p] for p in range(s)) for l in range(k)] for i in range(m)]
    Bj = [[sum(int(DB[p, j, l]) * w[p] for p in range(s)) for l in range(k)] for j in range(n)]
    for i in range(m):
        for j in range(n):
            X = sum(Ai[i][l] * Bj[j][l] for l in range(k))
            rem = Fr(X) * Fr(2) ** (int(E[i]) + int(F[j]) - 14 * s)
            for c in range(P):
                v = float(rem)
                assert got[c, j, i] == v, (i, j, c)
                rem -= Fr(v)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_integers_exact(P):
    rng = np.random.Generator(np.random.PCG64(1200 + P))
    m, n, k = 9, 7, 40
    A = np.zeros((P, k, m)); A[0] = rng.integers(-3000, 3000, (k, m))
    B = np.zeros((P, n, k)); B[0] = rng.integers(-3000, 3000, (n, k))
    one, zero = synth.mp_one(P), np.zeros(P)
    got = oracle.gemm_crt(P, SLICES[P], "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    exact = A[0].T.astype(np.int64) @ B[0].T.astype(np.int64)
    assert np.all(got[0].T == exact) and np.all(got[1:] == 0)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_truncation_bound_every_entry(P, ta, tb):
    """Only the operands' digit truncation errs: |a - A' 2^(E-7s)| <=
    2^(E-7s-1)(1 + 2^-40) (the slicing pin), so with da, db those bounds
    |C - AB| <= sum_l (da |b| + |a| db + da db) + the final rounding
    (2^(1-53P) |C|); checked exactly on every entry, alpha = 1, beta = 0."""
    s = SLICES[P]
    m, n, k = 11, 9, 37
    rng = np.random.Generator(np.random.PCG64(1300 + P))
    A = synth.mp_uniform(rng, P, (m, k) if ta == "T" else (k, m))
    B = synth.mp_uniform(rng, P, (k, n) if tb == "T" else (n, k))
    A = np.ldexp(A, rng.integers(-20, 21, A.shape[1:])[None])
    one, zero = synth.mp_one(P), np.zeros(P)
    got = oracle.gemm_crt(P, s, ta, tb, m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    E = oracle.split_exponents(P, ta, 0, m, k, A)
    F = oracle.split_exponents(P, tb, 1, n, k, B)
    chk = GemmChecker(P, ta, tb, m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    slack = 1 + Fr(1, 2 ** 40)
    for i in range(m):
        for j in range(n):
            exact, _ = chk.entry(i, j)
            da = Fr(2) ** (int(E[i]) - 7 * s - 1) * slack
            db = Fr(2) ** (int(F[j]) - 7 * s - 1) * slack
            sa = sum(abs(mp_frac(A[:, l, i] if ta == "N" else A[:, i, l])) for l in range(k))
            sb = sum(abs(mp_frac(B[:, j, l] if tb == "N" else B[:, l, j])) for l in range(k))
            val = mp_frac(got[:, j, i])
            bound = da * sb + db * sa + k * da * db + Fr(2, 2 ** (53 * P)) * abs(val)
            assert abs(val - exact) <= bound, (i, j)


def test_more_accurate_than_the_triangular_form():
    """The full square of digit pairs drops nothing the triangle keeps: on
    uniform data the error is at most that of the split form's triangle."""
    P, s = 2, 16
    m = n = k = 48
    A = synth.mp_matrix(20, "A", P, m, k)
    B = synth.mp_matrix(20, "B", P, k, n)
    one, zero = synth.mp_one(P), np.zeros(P)
    crt = oracle.gemm_crt(P, s, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    tri = oracle.gemm_split(P, s, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    chk = GemmChecker(P, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    ents = [(i, j) for i in range(0, m, 5) for j in range(0, n, 5)]
    assert chk.ratios(crt, ents).max() <= chk.ratios(tri, ents).max()

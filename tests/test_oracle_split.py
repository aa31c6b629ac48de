"""Pins of the oracle's split (sliced-integer) form: scale exponents, digit
slicing, anti-diagonal integer sums and the recombined result against exact
arithmetic."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, mp_frac

S_DEFAULT = {2: 16, 3: 23, 4: 30}


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("t", ["N", "T"])
def test_exponents_brute_force(P, t):
    A = synth.mp_matrix(20, "A", P, 13, 9, exp_range=(-30, 30))
    rows, k = (13, 9) if t == "N" else (9, 13)
    E = oracle.split_exponents(P, t, 0, rows, k, A)
    for i in range(rows):
        lead = A[0, :k, i] if t == "N" else A[0, i, :k]
        M = np.abs(lead).max()
        # largest entry of the row scaled into [1/4, 1/2)
        assert Fr(0.25) <= Fr(M) / Fr(2) ** int(E[i]) < Fr(0.5)
    Z = np.zeros((P, 4, 4))
    assert np.array_equal(oracle.split_exponents(P, "N", 0, 4, 4, Z), np.zeros(4, np.int32))


@pytest.mark.parametrize("P,s", [(2, 16), (3, 23), (4, 30), (4, 40), (2, 3), (3, 1)])
def test_slices_reconstruct_within_half_digit(P, s):
    """value / 2^E == sum_p d_p 2^(-7p) + r with |r| <= 2^(-7s-1)(1+2^-40)
    and every digit in [-64, 64]."""
    m, k = 11, 17
    A = synth.mp_matrix(21, "A", P, m, k, exp_range=(-30, 30))
    E = oracle.split_exponents(P, "N", 0, m, k, A)
    D = oracle.split_slices(P, s, "N", 0, m, k, A, E)
    assert D.shape == (s, m, k)
    assert np.abs(D.astype(int)).max() <= 64
    tol = Fr(1, 2 ** (7 * s + 1)) * (1 + Fr(1, 2 ** 40))
    for i in range(m):
        for l in range(k):
            x = mp_frac(A[:, l, i]) / Fr(2) ** int(E[i])
            rec = sum(Fr(int(D[p, i, l]), 2 ** (7 * (p + 1))) for p in range(s))
            assert abs(x - rec) <= tol


def test_slices_of_b_columns_equal_slices_of_transposed_rows():
    P, s, k, n = 3, 12, 7, 5
    B = synth.mp_matrix(22, "B", P, k, n)
    Bt = np.ascontiguousarray(np.transpose(B[:, :n, :k], (0, 2, 1)))   # n x k stored
    F = oracle.split_exponents(P, "N", 1, n, k, B)
    assert np.array_equal(F, oracle.split_exponents(P, "N", 0, n, k, Bt))
    assert np.array_equal(oracle.split_slices(P, s, "N", 1, n, k, B, F),
                          oracle.split_slices(P, s, "N", 0, n, k, Bt, F))


@pytest.mark.parametrize("P,s", [(2, 5), (4, 9)])
def test_diagonal_sums_brute_force(P, s):
    """S_d == sum over p+q == d (1 <= p, q <= s) of sum_l dA_p(i,l) dB_q(l,j)."""
    m, n, k = 4, 3, 10
    A = synth.mp_matrix(23, "A", P, m, k)
    B = synth.mp_matrix(23, "B", P, k, n)
    one, zero = synth.mp_one(P), np.zeros(P)
    _, E, F, S = oracle.gemm_split(P, s, "N", "N", m, n, k, one, A, B, zero,
                                   np.zeros((P, n, m)), debug=True)
    DA = oracle.split_slices(P, s, "N", 0, m, k, A, E)
    DB = oracle.split_slices(P, s, "N", 1, n, k, B, F)
    for d in range(2, s + 2):
        for i in range(m):
            for j in range(n):
                want = sum(int(DA[p - 1, i, l]) * int(DB[d - p - 1, j, l])
                           for p in range(1, d) for l in range(k))
                assert S[d - 2, j, i] == want


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T")])
def test_split_within_bound(P, ta, tb):
    m, n, k = 10, 9, 37
    A_rows, A_cols = (m, k) if ta == "N" else (k, m)
    B_rows, B_cols = (k, n) if tb == "N" else (n, k)
    A = synth.mp_matrix(24, "A", P, A_rows, A_cols)
    B = synth.mp_matrix(24, "B", P, B_rows, B_cols)
    C = synth.mp_matrix(24, "C", P, m, n)
    alpha = synth.mp_scalar(24, "alpha", P)
    beta = synth.mp_scalar(24, "beta", P)
    out = oracle.gemm_split(P, S_DEFAULT[P], ta, tb, m, n, k, alpha, A, B, beta, C)
    chk = GemmChecker(P, ta, tb, m, n, k, alpha, A, B, beta, C)
    r = chk.ratios(out, [(i, j) for i in range(m) for j in range(n)])
    assert r.max() <= 8 * (k + 2) / k


def slices_needed(P, rho):
    """Smallest s with (s + 1.1) 2^(-7s-2) <= 7 u rho: the digits dropped by
    slicing and by keeping only p + q <= s + 1 then cost at most 7 k u
    sum_l |a_il||b_lj| per entry (rho = sum_l |a_il||b_lj| / (k 2^(Ei+Fj)))."""
    u = {2: Fr(1, 2 ** 104), 3: Fr(1, 2 ** 150), 4: Fr(1, 2 ** 200)}[P]
    s = 1
    while Fr(s * 10 + 11, 10) / Fr(2) ** (7 * s + 2) > 7 * u * rho:
        s += 1
    return s


def test_split_qd_exponent_spread_needs_more_slices():
    """Entries u 2^e, e in -30..30 per entry: the row/column scales no longer
    fit every entry, so QD accuracy needs more digits than for uniform data.
    With s from the dropped-digit bound the result meets the GEMM bound;
    with far fewer digits it does not."""
    P, m, n, k = 4, 8, 8, 64
    A = synth.mp_matrix(3, "A", P, m, k, exp_range=(-30, 30))
    B = synth.mp_matrix(3, "B", P, k, n, exp_range=(-30, 30))
    one, zero = synth.mp_one(P), np.zeros(P)
    C0 = np.zeros((P, n, m))
    chk = GemmChecker(P, "N", "N", m, n, k, one, A, B, zero, C0)
    ents = [(i, j) for i in range(m) for j in range(n)]
    E = oracle.split_exponents(P, "N", 0, m, k, A)
    F = oracle.split_exponents(P, "N", 1, n, k, B)
    rho = min(chk.entry(i, j)[1] / (k * Fr(2) ** int(E[i] + F[j])) for i, j in ents)
    s = slices_needed(P, rho)
    assert 31 <= s <= 40
    r = chk.ratios(oracle.gemm_split(P, s, "N", "N", m, n, k, one, A, B, zero, C0), ents)
    assert r.max() <= 8.0
    r_few = chk.ratios(oracle.gemm_split(P, s - 8, "N", "N", m, n, k, one, A, B, zero, C0), ents)
    assert r_few.max() > 8.0


def test_split_integer_inputs_exact():
    """Small integers: with enough digits the sliced product is exact."""
    P, m, n, k = 2, 5, 6, 20
    rng = np.random.Generator(np.random.PCG64(31))
    A = np.zeros((P, k, m)); A[0] = rng.integers(-1000, 1000, (k, m))
    B = np.zeros((P, n, k)); B[0] = rng.integers(-1000, 1000, (n, k))
    one, zero = synth.mp_one(P), np.zeros(P)
    out = oracle.gemm_split(P, 4, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    exact = A[0].T.astype(np.int64) @ B[0].T.astype(np.int64)
    assert np.array_equal(out[0].T, exact.astype(np.float64))
    assert np.all(out[1] == 0)


def test_split_alpha_beta_semantics_match_plain():
    P, m, n, k = 3, 4, 5, 6
    A = synth.mp_matrix(25, "A", P, m, k)
    B = synth.mp_matrix(25, "B", P, k, n)
    C = synth.mp_matrix(25, "C", P, m, n)
    zero, one = np.zeros(P), synth.mp_one(P)
    beta = synth.mp_scalar(25, "beta", P)
    for (al, be, kk) in [(zero, beta, k), (zero, one, k), (one, one, 0), (zero, zero, k)]:
        a = oracle.gemm(P, "N", "N", m, n, kk, al, A, B, be, C)
        b = oracle.gemm_split(P, 8, "N", "N", m, n, kk, al, A, B, be, C)
        assert np.array_equal(a, b)
    Cnan = np.full_like(C, np.nan)
    assert np.isfinite(oracle.gemm_split(P, 8, "N", "N", m, n, k, one, A, B, zero, Cnan)).all()

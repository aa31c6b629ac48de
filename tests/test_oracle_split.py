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


def _round_components(X, e, P):
    """Components of X 2^e by repeated correctly rounded float(Fraction)."""
    rem = Fr(X) * Fr(2) ** e
    out = []
    for _ in range(P):
        v = float(rem)
        out.append(v)
        rem -= Fr(v)
    return out


def _adversarial_sums(rng, s, count):
    """Anti-diagonal sums that make the exact value need many bits or sit
    near a rounding tie: sparse patterns, runs of ones, single bits and
    full-range int32 values, both signs."""
    S = np.zeros((count, s), np.int64)
    for r in range(count):
        kind = r % 4
        dens = (0.15, 0.4, 1.0)[r % 3]
        for d in range(s):
            if rng.random() > dens:
                continue
            if kind == 0:
                v = int(rng.integers(-2 ** 31 + 1, 2 ** 31))
            elif kind == 1:
                v = int(rng.choice([-1, 1])) << int(rng.integers(0, 31))
            elif kind == 2:
                v = int(rng.choice([-1, 1])) * ((1 << int(rng.integers(1, 32))) - 1)
            else:
                v = int(rng.integers(-200, 201))
            S[r, d] = v
    return S


@pytest.mark.parametrize("P,s", [(2, 16), (2, 7), (3, 23), (3, 30), (3, 12), (4, 31), (4, 40)])
def test_recombination_is_the_exact_sum_rounded_once(P, s):
    """The recombination step alone on adversarial anti-diagonal sums: the
    exact integer X = sum_d S_d 128^(s+1-d) in Python, scaled by 2^(ef -
    7 (s+1)) and rounded component by component with Python's correctly
    rounded float(Fraction) of the exact remainder, gives the oracle's bits.
    A recombination that adds partial sums with the precision's own rounded
    addition instead fails on some of these."""
    rng = np.random.Generator(np.random.PCG64(1500 + 10 * P + s))
    count = 4000
    S = _adversarial_sums(rng, s, count)
    ef = rng.integers(-40, 41, count).astype(np.int32)
    got = oracle.split_recombine(P, s, S, ef)
    for r in range(count):
        X = 0
        for d in range(s):
            X = X * 128 + int(S[r, d])
        want = _round_components(X, int(ef[r]) - 7 * (s + 1), P)
        assert list(got[r]) == want, (r, S[r].tolist(), int(ef[r]))


@pytest.mark.parametrize("P,s,ta,tb", [(2, 16, "N", "N"), (2, 5, "T", "N"), (3, 23, "N", "T"),
                                        (3, 9, "T", "T"), (4, 31, "N", "N"), (4, 40, "T", "N")])
def test_exact_recombination_brute_force(P, s, ta, tb):
    """The split product is the exact triangle sum rounded once: from the
    oracle's own digits (pinned above), X_ij = sum over digit pairs with
    p + q <= s + 1 of sum_l d_p(a_il) d_q(b_lj) 128^(s+1-p-q) in Python
    integers, times 2^(E_i + F_j - 7 (s+1)), rounded component by component
    with Python's correctly rounded float(Fraction) of the exact remainder;
    the oracle gives the same bits (alpha = 1, beta = 0, whose epilogue
    leaves a normalised result unchanged)."""
    m, n, k = 3, 4, 7
    rng = np.random.Generator(np.random.PCG64(1400 + 10 * P + s))
    A = synth.mp_uniform(rng, P, (m, k) if ta == "T" else (k, m))
    B = synth.mp_uniform(rng, P, (k, n) if tb == "T" else (n, k))
    A = np.ldexp(A, rng.integers(-12, 13, A.shape[1:])[None])
    B = np.ldexp(B, rng.integers(-12, 13, B.shape[1:])[None])
    one, zero = synth.mp_one(P), np.zeros(P)
    got = oracle.gemm_split(P, s, ta, tb, m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    E = oracle.split_exponents(P, ta, 0, m, k, A)
    F = oracle.split_exponents(P, tb, 1, n, k, B)
    DA = oracle.split_slices(P, s, ta, 0, m, k, A, E).astype(np.int64)
    DB = oracle.split_slices(P, s, tb, 1, n, k, B, F).astype(np.int64)
    for i in range(m):
        for j in range(n):
            X = 0
            for p in range(1, s + 1):
                for q in range(1, s + 2 - p):
                    dot = sum(int(DA[p - 1, i, l]) * int(DB[q - 1, j, l]) for l in range(k))
                    X += dot * 128 ** (s + 1 - p - q)
            rem = Fr(X) * Fr(2) ** (int(E[i]) + int(F[j]) - 7 * (s + 1))
            for c in range(P):
                v = float(rem)
                assert got[c, j, i] == v, (i, j, c)
                rem -= Fr(v)


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

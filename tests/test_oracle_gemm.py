"""Pins of the oracle GEMM (eqn (1) of Sec. 3 with alpha/beta, canonical
ascending-k order) against exact products, closed forms and special cases."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, mp_frac

P_OF = {"dd": 2, "td": 3, "qd": 4}


def problem(P, ta, tb, m, n, k, fam=1, beta_zero=False, ld_pad=0):
    A_rows, A_cols = (m, k) if ta == "N" else (k, m)
    B_rows, B_cols = (k, n) if tb == "N" else (n, k)
    A = synth.mp_matrix(fam, "A", P, A_rows, A_cols, ld=A_rows + ld_pad)
    B = synth.mp_matrix(fam, "B", P, B_rows, B_cols, ld=B_rows + ld_pad)
    C = synth.mp_matrix(fam, "C", P, m, n, ld=m + ld_pad)
    alpha = synth.mp_scalar(fam, "alpha", P)
    beta = np.zeros(P) if beta_zero else synth.mp_scalar(fam, "beta", P)
    return A, B, C, alpha, beta


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_brute_force_exact_small(P, ta, tb):
    """Every entry of small GEMMs within 8 (k+2) u (|alpha||A||B| + |beta||C|)."""
    for (m, n, k) in [(1, 1, 1), (3, 5, 7), (8, 8, 8), (7, 2, 1)]:
        A, B, C, alpha, beta = problem(P, ta, tb, m, n, k, fam=10 + m, ld_pad=1)
        out = oracle.gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C)
        chk = GemmChecker(P, ta, tb, m, n, k, alpha, A, B, beta, C)
        r = chk.ratios(out, [(i, j) for i in range(m) for j in range(n)])
        assert r.max() <= 8 * (k + 2) / max(k, 1), r.max()


@pytest.mark.parametrize("P", [2, 3, 4])
def test_bound_alpha1_beta0_random(P):
    m = n = 24
    k = 96
    A, B, C, _, _ = problem(P, "N", "N", m, n, k, fam=1, beta_zero=True)
    one = synth.mp_one(P)
    zero = np.zeros(P)
    out = oracle.gemm(P, "N", "N", m, n, k, one, A, B, zero, C)
    chk = GemmChecker(P, "N", "N", m, n, k, one, A, B, zero, C)
    r = chk.ratios(out, [(i, j) for i in range(0, m, 3) for j in range(0, n, 3)])
    assert r.max() <= 8.0


@pytest.mark.parametrize("P", [2, 3, 4])
def test_transposed_storage_gives_identical_bits(P):
    """op(A) op(B) from A, B stored as-is ('N') or stored transposed ('T')."""
    m, n, k = 9, 11, 13
    A, B, C, alpha, beta = problem(P, "N", "N", m, n, k, fam=3)
    At = np.ascontiguousarray(np.transpose(A[:, :k, :m], (0, 2, 1)))   # (P, m, k): k x m stored
    Bt = np.ascontiguousarray(np.transpose(B[:, :n, :k], (0, 2, 1)))
    ref = oracle.gemm(P, "N", "N", m, n, k, alpha, A, B, beta, C)
    for ta, tb, AA, BB in [("T", "N", At, B), ("N", "T", A, Bt), ("T", "T", At, Bt)]:
        assert np.array_equal(oracle.gemm(P, ta, tb, m, n, k, alpha, AA, BB, beta, C), ref)


def test_dd_transpose_identity_bitwise():
    """DDmul and DDadd are bitwise commutative, so (AB)^T == B^T A^T exactly."""
    P, m, n, k = 2, 10, 7, 33
    A, B, C, _, _ = problem(P, "N", "N", m, n, k, fam=4)
    one, zero = synth.mp_one(P), np.zeros(P)
    AB = oracle.gemm(P, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    BtAt = oracle.gemm(P, "T", "T", n, m, k, one, B, A, zero, np.zeros((P, m, n)))
    assert np.array_equal(AB, np.transpose(BtAt, (0, 2, 1)))


@pytest.mark.parametrize("P", [2, 3, 4])
def test_identity_right_factor_bitwise(P):
    m, k = 17, 12
    A = synth.mp_matrix(5, "A", P, m, k)
    I = np.zeros((P, k, k))
    I[0] = np.eye(k)
    one, zero = synth.mp_one(P), np.zeros(P)
    out = oracle.gemm(P, "N", "N", m, k, k, one, A, I, zero, np.zeros((P, k, m)))
    assert np.array_equal(out, A)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_integer_matrices_exact(P):
    """Integer entries: every intermediate fits in P components, so the
    result is the exact integer product (DD: 30-bit entries; TD/QD: 50-bit
    entries split over two components)."""
    rng = np.random.Generator(np.random.PCG64(900 + P))
    m, n, k = 6, 5, 40
    bits = 30 if P == 2 else 50
    Ai = rng.integers(-(2 ** bits), 2 ** bits, size=(k, m))
    Bi = rng.integers(-(2 ** bits), 2 ** bits, size=(n, k))

    def planes(M):
        out = np.zeros((P,) + M.shape)
        for idx, v in np.ndenumerate(M):
            comps = synth.fraction_to_components(Fr(int(v)), P)
            out[(slice(None),) + idx] = comps
        return out

    A, B = planes(Ai), planes(Bi)
    one, zero = synth.mp_one(P), np.zeros(P)
    out = oracle.gemm(P, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    exact = Ai.T.astype(object) @ Bi.T.astype(object)
    for i in range(m):
        for j in range(n):
            assert mp_frac(out[:, j, i]) == exact[i, j]


def test_closed_form_identity():
    """sum_k (i+k-1)(n-k) = n(n-1)(3i+n-2)/6 for the paper's test matrices."""
    for n in (1, 2, 3, 5, 8, 17, 64):
        for i in range(1, n + 1):
            assert 6 * sum((i + k - 1) * (n - k) for k in range(1, n + 1)) == n * (n - 1) * (3 * i + n - 2)


@pytest.mark.parametrize("P,n", [(2, 64), (3, 48), (4, 40), (2, 33)])
def test_paper_matrices_digits(P, n):
    """The paper's fixed test matrices lose at most one or two decimal digits
    (Sec. 3): at least -log10(u) - 2 correct digits against the exact
    sqrt(15) n (n-1) (3i+n-2) / 6."""
    A, B = synth.paper_matrices(n, P)
    one, zero = synth.mp_one(P), np.zeros(P)
    out = oracle.gemm(P, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, n)))
    u = {2: 2.0 ** -104, 3: 2.0 ** -150, 4: 2.0 ** -200}[P]
    need = -math.log10(u) - 2
    for i in range(n):
        ex = synth.paper_exact_entry(n, i + 1)
        for j in (0, n // 2, n - 1):
            got = mp_frac(out[:, j, i])
            rel = abs(got - ex) / ex
            digits = math.inf if rel == 0 else -math.log10(float(rel))
            assert digits >= need, (P, n, i, j, digits)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_alpha_beta_semantics(P):
    m, n, k = 5, 4, 6
    A, B, C, alpha, beta = problem(P, "N", "N", m, n, k, fam=7)
    zero, one = np.zeros(P), synth.mp_one(P)
    Cnan = C.copy()
    Cnan[:, :, :] = np.nan
    # beta == 0: C is never read
    out = oracle.gemm(P, "N", "N", m, n, k, alpha, A, B, zero, Cnan)
    assert np.isfinite(out).all()
    # alpha == 0, beta == 1: quick return leaves C (even NaN) untouched
    out = oracle.gemm(P, "N", "N", m, n, k, zero, A, B, one, Cnan)
    assert np.isnan(out).all()
    # k == 0, beta == 1: quick return
    out = oracle.gemm(P, "N", "N", m, n, 0, alpha, A, B, one, C)
    assert np.array_equal(out, C)
    # alpha == 0: C = beta * C element-wise
    out = oracle.gemm(P, "N", "N", m, n, k, zero, A, B, beta, C)
    flat = C.reshape(P, -1)
    want = oracle.vec(P, "mul", np.repeat(beta[:, None], flat.shape[1], 1), flat).reshape(C.shape)
    assert np.array_equal(out, want)
    # alpha == 0, beta == 0: C = 0
    out = oracle.gemm(P, "N", "N", m, n, k, zero, A, B, zero, Cnan)
    assert np.array_equal(out, np.zeros_like(C))
    # m == 0 / n == 0: nothing touched
    assert np.array_equal(oracle.gemm(P, "N", "N", 0, n, k, alpha, A, B, beta, C), C)


def test_row_range_matches_full():
    P, m, n, k = 3, 12, 5, 9
    A, B, C, alpha, beta = problem(P, "N", "T", m, n, k, fam=8)
    full = oracle.gemm(P, "N", "T", m, n, k, alpha, A, B, beta, C)
    part = oracle.gemm(P, "N", "T", m, n, k, alpha, A, B, beta, C, rows=(4, 9))
    assert np.array_equal(part[:, :, 4:9], full[:, :, 4:9])
    assert np.array_equal(part[:, :, :4], C[:, :, :4])

"""Pins of the oracle's BLAS-1/2 operations in DD/TD/QD: axpy, the
fixed-order dot product and gemv."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import mp_frac
from tests.test_oracle_arith import C_ADD, C_MUL

U = {2: Fr(1, 2 ** 104), 3: Fr(1, 2 ** 150), 4: Fr(1, 2 ** 200)}


def vecs(P, n, seed, spread=20):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = synth.mp_uniform(rng, P, (n,))
    y = synth.mp_uniform(rng, P, (n,))
    x = np.ldexp(x, rng.integers(-spread, spread + 1, n)[None])
    y = np.ldexp(y, rng.integers(-spread, spread + 1, n)[None])
    return x, y


@pytest.mark.parametrize("P", [2, 3, 4])
def test_axpy_unit_alpha_is_the_addition(P):
    """alpha = 1: MUL(1, x) returns x unchanged, so axpy is the element-wise
    addition (a separately pinned oracle function)."""
    x, y = vecs(P, 3000, 50 + P)
    assert np.array_equal(oracle.axpy(P, synth.mp_one(P), x, y), oracle.vec(P, "add", x, y))


@pytest.mark.parametrize("P", [2, 3, 4])
def test_axpy_error_bound(P):
    x, y = vecs(P, 2000, 60 + P)
    alpha = synth.mp_scalar(7, "alpha", P)
    r = oracle.axpy(P, alpha, x, y)
    al = mp_frac(alpha)
    for i in range(x.shape[1]):
        X, Y, R = mp_frac(x[:, i]), mp_frac(y[:, i]), mp_frac(r[:, i])
        bound = (C_MUL[P] * (1 + C_ADD[P] * U[P]) + C_ADD[P]) * U[P] * (abs(al * X) + abs(Y))
        assert abs(R - (al * X + Y)) <= bound, i


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("n", [1, 17, 64])
def test_dot_short_is_the_sequential_chain(P, n):
    """Up to 64 terms the tree is one block: the ascending chain, which is
    the canonical GEMM entry of a 1 x n times n x 1 product."""
    x, y = vecs(P, n, 70 + P + n)
    one, zero = synth.mp_one(P), np.zeros(P)
    # A = x as a 1 x n matrix (n columns of leading dimension 1), B = y as n x 1
    g = oracle.gemm(P, "N", "N", 1, 1, n, one, x.reshape(P, n, 1), y.reshape(P, 1, n), zero,
                    np.zeros((P, 1, 1)))
    assert np.array_equal(oracle.dot(P, x, y), g[:, 0, 0])


@pytest.mark.parametrize("P", [2, 3, 4])
def test_dot_integers_exact_and_bound(P):
    rng = np.random.Generator(np.random.PCG64(80 + P))
    n = 64 * 64 * 3 + 17                    # three levels, ragged
    xi = rng.integers(-1000, 1000, n).astype(float)
    yi = rng.integers(-1000, 1000, n).astype(float)
    x = np.zeros((P, n)); x[0] = xi
    y = np.zeros((P, n)); y[0] = yi
    r = oracle.dot(P, x, y)
    assert r[0] == float(int(np.dot(xi.astype(np.int64), yi.astype(np.int64)))) and np.all(r[1:] == 0)
    x, y = vecs(P, n, 90 + P)
    r = oracle.dot(P, x, y)
    exact = sum(mp_frac(x[:, i]) * mp_frac(y[:, i]) for i in range(n))
    base = sum(abs(mp_frac(x[:, i]) * mp_frac(y[:, i])) for i in range(n))
    assert abs(mp_frac(r) - exact) <= 8 * (n + 2) * U[P] * base


def test_dot_empty():
    assert np.all(oracle.dot(3, np.zeros((3, 0)), np.zeros((3, 0))) == 0)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("trans", ["N", "T"])
def test_gemv_bound_and_gemm_identity(P, trans):
    """gemv against the exact product, and equal to the GEMM with one column
    (x as an inner x 1 matrix)."""
    m, n = 23, 37
    rng = np.random.Generator(np.random.PCG64(100 + P))
    A = synth.mp_uniform(rng, P, (n, m))            # column-major m x n
    rows, inner = (m, n) if trans == "N" else (n, m)
    x = synth.mp_uniform(rng, P, (inner,))
    y = synth.mp_uniform(rng, P, (rows,))
    alpha, beta = synth.mp_scalar(8, "alpha", P), synth.mp_scalar(8, "beta", P)
    got = oracle.gemv(P, trans, m, n, alpha, A, x, beta, y)
    g = oracle.gemm(P, trans, "N", rows, 1, inner, alpha, A, x.reshape(P, 1, inner), beta,
                    y.reshape(P, 1, rows))
    assert np.array_equal(got, g[:, 0, :])
    al, be = mp_frac(alpha), mp_frac(beta)
    for i in range(rows):
        acc = Fr(0)
        base = Fr(0)
        for l in range(inner):
            a = mp_frac(A[:, l, i] if trans == "N" else A[:, i, l])
            acc += a * mp_frac(x[:, l])
            base += abs(a * mp_frac(x[:, l]))
        exact = al * acc + be * mp_frac(y[:, i])
        bound = 8 * (inner + 2) * U[P] * (abs(al) * base + abs(be * mp_frac(y[:, i])))
        assert abs(mp_frac(got[:, i]) - exact) <= bound, (trans, i)

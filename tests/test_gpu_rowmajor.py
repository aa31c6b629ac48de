"""Row-major products (`matmul`): the column-major call C^T = B^T A^T on the
same buffers.  Bit for bit as the oracle's canonical GEMM of that transposed
problem (plain and residue forms, beta = 0 and beta != 0), and for DD, whose
multiplication is symmetric, also as the canonical chain of A B itself."""
import numpy as np
import pytest

import oracle
from tests import synth
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def operands(P, m, n, k, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = np.ascontiguousarray(synth.mp_uniform(rng, P, (m, k)))     # row-major planes
    B = np.ascontiguousarray(synth.mp_uniform(rng, P, (k, n)))
    C = np.ascontiguousarray(synth.mp_uniform(rng, P, (m, n)))
    alpha = synth.mp_uniform(rng, P, (1,))[:, 0]
    beta = synth.mp_uniform(rng, P, (1,))[:, 0]
    return A, B, C, alpha, beta


@pytest.mark.parametrize("P", [2, 3, 4])
def test_row_major_plain(gpu_lib, P):
    m, n, k = 70, 45, 130
    A, B, C, alpha, beta = operands(P, m, n, k, 610 + P)
    one, zero = synth.mp_one(P), np.zeros(P)
    note("row-major", P, (m, n, k))
    got = host(gpu_lib.matmul(P, dev(A), dev(B)))
    assert got.shape == (P, m, n)
    # a row-major (P, r, c) array is the oracle's column-major c x r matrix
    want = oracle.gemm(P, "N", "N", n, m, k, one, B, A, zero, np.zeros((P, m, n)))
    assert np.array_equal(got, want)
    if P == 2:
        canon = oracle.gemm(P, "T", "T", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
        assert np.array_equal(got, np.swapaxes(canon, 1, 2))
    # alpha and beta, C given (read row-major)
    dC = dev(C)
    out = gpu_lib.matmul(P, dev(A), dev(B), dC, alpha=alpha, beta=beta)
    assert out is dC
    want = oracle.gemm(P, "N", "N", n, m, k, alpha, B, A, beta, C)
    assert np.array_equal(host(dC), want)


@pytest.mark.parametrize("P", [2, 4])
def test_row_major_residue_form(gpu_lib, P):
    m, n, k = 129, 66, 200
    s = gpu_lib.DEFAULT_SLICES[P]
    A, B, C, alpha, beta = operands(P, m, n, k, 620 + P)
    note("row-major residue", P, (m, n, k))
    ws = gpu_lib.alloc_workspace(P, n, m, k, s, form="crt")         # the call's M = n, N = m
    dC = dev(C)
    gpu_lib.matmul(P, dev(A), dev(B), dC, alpha=alpha, beta=beta, form="crt", slices=s, workspace=ws)
    want = oracle.gemm_crt(P, s, "N", "N", n, m, k, alpha, B, A, beta, C)
    assert np.array_equal(host(dC), want)

"""BLAS-1/2 in DD/TD/QD on the GPU, bit for bit against the oracle: axpy, the
fixed-order dot product and gemv (also against the GPU GEMM with one
column)."""
import numpy as np
import pytest
import torch

import oracle
from tests import synth
from tests.gpu_util import dev, host, note
from tests.test_gpu_vec import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P", [2, 3, 4])
def test_axpy_bitwise(gpu_lib, P):
    n = 300_001
    x, y = inputs(P, n, 500 + P)
    alpha = synth.mp_scalar(16, "alpha", P)
    want = oracle.axpy(P, alpha, x, y)
    dy = dev(y)
    note("axpy", P, n)
    gpu_lib.axpy(P, alpha, dev(x), dy)
    got = host(dy)
    ok = (got == want) | (np.isnan(got) & np.isnan(want))
    assert ok.all()


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4096, 262_145, 4_194_307])
def test_dot_bitwise(gpu_lib, P, n):
    rng = np.random.Generator(np.random.PCG64(600 + P))
    x = synth.mp_uniform(rng, P, (n,))
    y = synth.mp_uniform(rng, P, (n,))
    want = oracle.dot(P, x, y)
    res = torch.full((P,), float("nan"), dtype=torch.float64, device="cuda")
    note("dot", P, n)
    gpu_lib.dot(P, dev(x), dev(y), res)
    assert np.array_equal(res.cpu().numpy(), want)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("trans", ["N", "T"])
def test_gemv_bitwise(gpu_lib, P, trans):
    for m, n in [(1, 1), (257, 129), (1000, 2000)]:
        A = synth.mp_matrix(17, "A", P, m, n)
        rows, inner = (m, n) if trans == "N" else (n, m)
        rng = np.random.Generator(np.random.PCG64(700 + P + m))
        x = synth.mp_uniform(rng, P, (inner,))
        y = synth.mp_uniform(rng, P, (rows,))
        alpha, beta = synth.mp_scalar(17, "alpha", P), synth.mp_scalar(17, "beta", P)
        want = oracle.gemv(P, trans, m, n, alpha, A, x, beta, y)
        dy = dev(y)
        note("gemv", P, trans, m, n)
        gpu_lib.gemv(P, trans, m, n, alpha, dev(A), dev(x), beta, dy)
        assert np.array_equal(host(dy), want), (P, trans, m, n)


@pytest.mark.parametrize("P", [2, 4])
def test_gemv_equals_gemm_one_column_n4096(gpu_lib, P):
    m = n = 4096
    A = synth.mp_matrix(18, "A", P, m, n)
    rng = np.random.Generator(np.random.PCG64(800 + P))
    x = synth.mp_uniform(rng, P, (n,))
    y = synth.mp_uniform(rng, P, (m,))
    alpha, beta = synth.mp_scalar(18, "alpha", P), synth.mp_scalar(18, "beta", P)
    dA = dev(A)
    dy = dev(y)
    note("gemv vs gemm", P)
    gpu_lib.gemv(P, "N", m, n, alpha, dA, dev(x), beta, dy)
    dC = dev(y.reshape(P, 1, m))
    gpu_lib.gemm(P, "N", "N", m, 1, n, alpha, dA, dev(x.reshape(P, 1, n)), beta, dC)
    assert np.array_equal(host(dy), host(dC)[:, 0, :])


def test_gemv_alpha_zero_beta_zero(gpu_lib):
    P, m, n = 3, 50, 40
    A = synth.mp_matrix(19, "A", P, m, n)
    y = np.full((P, m), np.nan)
    dy = dev(y)
    gpu_lib.gemv(P, "N", m, n, np.zeros(P), dev(A), dev(np.zeros((P, n))), np.zeros(P), dy)
    assert np.all(host(dy) == 0.0)              # y never read when beta == 0


@pytest.mark.parametrize("P", [2, 4])
def test_gemv_beta_zero_does_not_read_y(gpu_lib, P):
    """alpha != 0, beta = 0: y is written, never read (NaN in y stays out)."""
    m, n = 130, 77
    A = synth.mp_matrix(20, "A", P, m, n)
    rng = np.random.Generator(np.random.PCG64(900 + P))
    x = synth.mp_uniform(rng, P, (n,))
    alpha = synth.mp_scalar(20, "alpha", P)
    want = oracle.gemv(P, "N", m, n, alpha, A, x, np.zeros(P), np.zeros((P, m)))
    dy = dev(np.full((P, m), np.nan))
    note("gemv beta 0", P)
    gpu_lib.gemv(P, "N", m, n, alpha, dev(A), dev(x), np.zeros(P), dy)
    assert np.array_equal(host(dy), want)

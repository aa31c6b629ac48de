"""Strassen's method (Sec. 3, Fig. 5) on the GPU: bit for bit against the
oracle's Strassen recursion (same block products in canonical order, same
block sums), and within Strassen's normwise bound of the exact product."""
import math

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, mp_frac, sample_entries
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def make(P, ta, tb, m, n, k, fam):
    A = synth.mp_matrix(fam, "A", P, *((m, k) if ta == "N" else (k, m)))
    B = synth.mp_matrix(fam, "B", P, *((k, n) if tb == "N" else (n, k)))
    C = synth.mp_matrix(fam, "C", P, m, n)
    return A, B, C, synth.mp_scalar(fam, "alpha", P), synth.mp_scalar(fam, "beta", P)


def run(gpu_lib, P, L, ta, tb, m, n, k, alpha, A, B, beta, C):
    ws = gpu_lib.alloc_workspace(P, m, n, k, form="strassen", levels=L)
    dC = dev(C)
    gpu_lib.gemm(P, ta, tb, m, n, k, alpha, dev(A), dev(B), beta, dC, form="strassen", levels=L,
                 workspace=ws)
    return host(dC)


CASES = [
    # P, L, ta, tb, m, n, k
    (2, 1, "N", "N", 64, 32, 48),
    (3, 2, "T", "N", 64, 64, 64),
    (4, 2, "N", "T", 32, 96, 64),
    (2, 3, "T", "T", 128, 64, 128),
    (3, 1, "N", "N", 2, 2, 2),
    (4, 4, "T", "N", 48, 32, 16),
    (2, 5, "N", "N", 64, 64, 64),
]


@pytest.mark.parametrize("P,L,ta,tb,m,n,k", CASES)
def test_bitwise_against_oracle(gpu_lib, P, L, ta, tb, m, n, k):
    A, B, C, alpha, beta = make(P, ta, tb, m, n, k, fam=14)
    note("strassen", P, L, ta, tb, (m, n, k))
    got = run(gpu_lib, P, L, ta, tb, m, n, k, alpha, A, B, beta, C)
    want = oracle.gemm_strassen(P, L, ta, tb, m, n, k, alpha, A, B, beta, C)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("P,L", [(2, 2), (4, 1)])
def test_bitwise_n1024(gpu_lib, P, L):
    n = 1024
    A, B, C, alpha, beta = make(P, "N", "N", n, n, n, fam=2)
    note("strassen n1024", P, L)
    got = run(gpu_lib, P, L, "N", "N", n, n, n, alpha, A, B, beta, C)
    want = oracle.gemm_strassen(P, L, "N", "N", n, n, n, alpha, A, B, beta, C)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_normwise_bound_n4096(gpu_lib, P):
    """Two levels at the benchmark size: sampled entries within
    c gamma u max|A| max|B| (Strassen's normwise constant gamma, c = 32)."""
    n, L = 4096, 2
    A, B, _, _, _ = make(P, "N", "N", n, n, n, fam=2)
    one, zero = synth.mp_one(P), np.zeros(P)
    note("strassen n4096", P, L)
    got = run(gpu_lib, P, L, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, n)))
    n0 = n // 2 ** L
    gamma = (n / n0) ** math.log2(12) * (n0 * n0 + 5 * n0) - 5 * n
    u = 2.0 ** (-{2: 104, 3: 150, 4: 200}[P])
    amax = float(np.abs(A[0]).max()) * (1 + 2.0 ** -50)
    bmax = float(np.abs(B[0]).max()) * (1 + 2.0 ** -50)
    chk = GemmChecker(P, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, 1)))
    worst = 0.0
    for i, j in sample_entries(synth.rng_for(2, "samples"), n, n, 48):
        exact, _ = chk.entry(i, j)
        worst = max(worst, float(abs(mp_frac(got[:, j, i]) - exact)))
    print(f"strassen P={P} L={L}: max err / (gamma u max|A| max|B|) = {worst / (gamma * u * amax * bmax):.3g}")
    assert worst <= 32 * gamma * u * amax * bmax


def test_alpha_zero_and_errors(gpu_lib):
    P, m, n, k = 2, 16, 16, 16
    A, B, C, _, beta = make(P, "N", "N", m, n, k, fam=15)
    zero = np.zeros(P)
    got = run(gpu_lib, P, 2, "N", "N", m, n, k, zero, A, B, beta, C)
    assert np.array_equal(got, oracle.gemm(P, "N", "N", m, n, k, zero, A, B, beta, C))
    one = synth.mp_one(P)
    ws = gpu_lib.alloc_workspace(P, 16, 16, 16, form="strassen", levels=3)
    assert gpu_lib.gemm_raw(P, "N", "N", 12, 16, 16, one, dev(A), dev(B), zero, dev(C),
                            form="strassen", levels=3, workspace=ws) == 3          # 12 % 8 != 0
    small = gpu_lib.alloc_workspace(P, 4, 4, 4, form="strassen", levels=1)
    assert gpu_lib.gemm_raw(P, "N", "N", m, n, k, one, dev(A), dev(B), zero, dev(C),
                            form="strassen", levels=1, workspace=small) == 2
    A3 = synth.mp_matrix(15, "A", 3, m, k)
    assert gpu_lib.gemm_raw(3, "N", "N", m, n, k, synth.mp_one(3), dev(A3), dev(A3), np.zeros(3),
                            dev(np.zeros((3, n, m))), form="strassen", levels=1, workspace=ws,
                            variant=1) == 3

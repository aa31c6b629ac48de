"""Plain GEMM on inputs that leave the common Renorm/VSEB branch (zero
components, integers, exact cancellation, mixtures inside one wavefront):
the kernels' fallback must give the same bits as the oracle.  Also the
autotuner: it returns a valid configuration and results do not depend on
the configuration."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from tests import synth
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def structured(P, rows, cols, kind, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = synth.mp_uniform(rng, P, (cols, rows))
    if kind == "integers":                       # short integers: errors vanish
        X[:] = 0.0
        X[0] = rng.integers(-50, 50, size=(cols, rows))
    elif kind == "single":                       # lower components zero
        X[1:] = 0.0
    elif kind == "mixed":                        # every other column structured
        X[1:, ::2, :] = 0.0
        X[0, ::3, :] = np.round(X[0, ::3, :] * 64)
        X[1:, ::3, :] = 0.0
    elif kind == "sparse":                       # many exact zeros
        mask = rng.uniform(size=(cols, rows)) < 0.7
        X[:, mask] = 0.0
    elif kind == "dyadic":                       # few-bit dyadic values, exact sums
        X[:] = 0.0
        X[0] = rng.integers(-8, 8, size=(cols, rows)) * 2.0 ** rng.integers(-40, 40, size=(cols, rows))
    return X


@pytest.mark.parametrize("P", [3, 4])
@pytest.mark.parametrize("kind", ["integers", "single", "mixed", "sparse", "dyadic"])
def test_plain_fallback_bitwise(gpu_lib, P, kind):
    m, n, k = 70, 66, 45
    A = structured(P, m, k, kind, 1000 + P)
    B = structured(P, k, n, kind, 2000 + P)
    C = synth.mp_matrix(9, "C", P, m, n)
    alpha = synth.mp_scalar(9, "alpha", P)
    beta = synth.mp_scalar(9, "beta", P)
    want = oracle.gemm(P, "N", "N", m, n, k, alpha, A, B, beta, C)
    for tile in range(gpu_lib.num_configs(P, "plain")):
        note("fallback", P, kind, "tile", tile)
        dC = dev(C)
        gpu_lib.gemm(P, "N", "N", m, n, k, alpha, dev(A), dev(B), beta, dC, form="plain", tile=tile)
        assert np.array_equal(host(dC), want), (P, kind, tile)


@pytest.mark.parametrize("P", [3, 4])
def test_vec_fallback_bitwise(gpu_lib, P):
    n = 50_000
    x = structured(P, n, 1, "mixed", 3000 + P)[:, 0, :]
    y = structured(P, n, 1, "sparse", 4000 + P)[:, 0, :]
    for op in ("add", "mul"):
        want = oracle.vec(P, op, x, y)
        dr = dev(np.zeros_like(x))
        note("vec fallback", P, op)
        gpu_lib.vec(P, op, dev(x), dev(y), dr)
        assert np.array_equal(host(dr), want)


def test_integer_product_exact_on_gpu(gpu_lib):
    """QD: integer inputs give the exact integer product (the result of the
    fallback path is also checked against exact arithmetic)."""
    P, m, n, k = 4, 33, 31, 40
    A = structured(P, m, k, "integers", 5)
    B = structured(P, k, n, "integers", 6)
    one, zero = synth.mp_one(P), np.zeros(P)
    dC = dev(np.zeros((P, n, m)))
    gpu_lib.gemm(P, "N", "N", m, n, k, one, dev(A), dev(B), zero, dC)
    got = host(dC)
    exact = A[0, :k, :m].T.astype(np.int64) @ B[0, :n, :k].T.astype(np.int64)
    for i in range(m):
        for j in range(n):
            assert sum(Fr(float(v)) for v in got[:, j, i]) == int(exact[i, j])


def test_autotune_returns_valid_config_and_same_bits(gpu_lib):
    P, n = 3, 384
    note("autotune plain", P, n)
    best = gpu_lib.autotune(P, "plain", n, n, n)
    assert 0 <= best < gpu_lib.num_configs(P, "plain")
    best_s = gpu_lib.autotune(P, "split", n, n, n, 23)
    assert 0 <= best_s < gpu_lib.num_configs(P, "split")
    A = synth.mp_matrix(11, "A", P, n, n)
    B = synth.mp_matrix(11, "B", P, n, n)
    one, zero = synth.mp_one(P), np.zeros(P)
    outs = []
    for tile in (-1, 0, 1):        # -1 = the tuned choice
        dC = dev(np.zeros((P, n, n)))
        gpu_lib.gemm(P, "N", "N", n, n, n, one, dev(A), dev(B), zero, dC, form="plain", tile=tile)
        outs.append(host(dC))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    ws = gpu_lib.alloc_workspace(P, n, n, n, 23, tile=0)
    ws2 = gpu_lib.alloc_workspace(P, n, n, n, 23, tile=3)
    souts = []
    for tile, w in ((0, ws), (3, ws2), (-1, gpu_lib.alloc_workspace(P, n, n, n, 23))):
        dC = dev(np.zeros((P, n, n)))
        gpu_lib.gemm(P, "N", "N", n, n, n, one, dev(A), dev(B), zero, dC, form="split", slices=23,
                     tile=tile, workspace=w)
        souts.append(host(dC))
    assert np.array_equal(souts[0], souts[1]) and np.array_equal(souts[0], souts[2])

"""The other TD operations of Sec. 2.3 on the GPU: the accurate addition
(Algorithm 3) and TDmulq, element-wise and inside the plain TD GEMM, bit for
bit against the oracle; the GEMM variants also within the error bound."""
import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, sample_entries
from tests.gpu_util import dev, host, note
from tests.test_gpu_vec import inputs

pytestmark = pytest.mark.gpu

VARIANTS = [1, 2, 3]       # bit 0: accurate addition, bit 1: TDmulq


@pytest.mark.parametrize("op", ["add_acc", "mulq"])
def test_vec_variants_bitwise(gpu_lib, op):
    n = 300_001
    x, y = inputs(3, n, 77)
    want = oracle.vec(3, op, x, y)
    note("td vec", op, n)
    dr = dev(np.zeros_like(x))
    gpu_lib.vec(3, op, dev(x), dev(y), dr)
    got = host(dr)
    bad = np.nonzero(~((got == want) | (np.isnan(got) & np.isnan(want))).all(axis=0))[0]
    assert bad.size == 0, (op, bad[:5], got[:, bad[:3]], want[:, bad[:3]])


def make(ta, tb, m, n, k, fam):
    A = synth.mp_matrix(fam, "A", 3, *((m, k) if ta == "N" else (k, m)))
    B = synth.mp_matrix(fam, "B", 3, *((k, n) if tb == "N" else (n, k)))
    C = synth.mp_matrix(fam, "C", 3, m, n)
    return A, B, C, synth.mp_scalar(fam, "alpha", 3), synth.mp_scalar(fam, "beta", 3)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_gemm_variant_ragged_bitwise(gpu_lib, variant, ta, tb):
    for m, n, k in [(67, 45, 33), (130, 129, 65), (1, 1, 1), (5, 200, 17)]:
        A, B, C, alpha, beta = make(ta, tb, m, n, k, fam=11)
        want = oracle.gemm(3, ta, tb, m, n, k, alpha, A, B, beta, C, variant=variant)
        note("td variant gemm", variant, ta, tb, (m, n, k))
        dC = dev(C)
        gpu_lib.gemm(3, ta, tb, m, n, k, alpha, dev(A), dev(B), beta, dC, variant=variant)
        assert np.array_equal(host(dC), want), (variant, ta, tb, m, n, k)


@pytest.mark.parametrize("variant", VARIANTS)
def test_gemm_variant_n1024_sampled(gpu_lib, variant):
    n = 1024
    A, B, C, alpha, beta = make("N", "N", n, n, n, fam=2)
    note("td variant gemm n1024", variant)
    dC = dev(C)
    gpu_lib.gemm(3, "N", "N", n, n, n, alpha, dev(A), dev(B), beta, dC, variant=variant)
    got = host(dC)
    rows, cols = (n - 2, n), (n - 16, n)
    want = oracle.gemm(3, "N", "N", n, n, n, alpha, A, B, beta, C, rows=rows, cols=cols, variant=variant)
    blk = (slice(None), slice(*cols), slice(*rows))
    assert np.array_equal(got[blk], want[blk])
    chk = GemmChecker(3, "N", "N", n, n, n, alpha, A, B, beta, C)
    r = chk.ratios(got, sample_entries(synth.rng_for(2, "samples"), n, n, 48))
    print(f"TD variant {variant} n={n}: max err ratio {r.max():.3g}")
    assert r.max() <= 8 * (n + 2) / n


@pytest.mark.parametrize("variant", VARIANTS)
def test_gemm_variant_alpha_zero(gpu_lib, variant):
    """alpha == 0: C = beta C with the variant's product."""
    m, n, k = 37, 29, 11
    A, B, C, _, beta = make("N", "N", m, n, k, fam=12)
    zero = np.zeros(3)
    want = oracle.gemm(3, "N", "N", m, n, k, zero, A, B, beta, C, variant=variant)
    dC = dev(C)
    gpu_lib.gemm(3, "N", "N", m, n, k, zero, dev(A), dev(B), beta, dC, variant=variant)
    assert np.array_equal(host(dC), want)


def test_variant_errors(gpu_lib):
    m = n = k = 8
    for P in (2, 4):
        A = synth.mp_matrix(13, "A", P, m, k)
        rc = gpu_lib.gemm_raw(P, "N", "N", m, n, k, synth.mp_one(P), dev(A), dev(A), np.zeros(P),
                              dev(np.zeros((P, n, m))), variant=1)
        assert rc == 3
    A = synth.mp_matrix(13, "A", 3, m, k)
    one, zero, C = synth.mp_one(3), np.zeros(3), np.zeros((3, n, m))
    ws = gpu_lib.alloc_workspace(3, m, n, k, 23)
    assert gpu_lib.gemm_raw(3, "N", "N", m, n, k, one, dev(A), dev(A), zero, dev(C), form="split",
                            slices=23, workspace=ws, variant=2) == 3
    assert gpu_lib.gemm_raw(3, "N", "N", m, n, k, one, dev(A), dev(A), zero, dev(C), variant=4) == -18

"""Plain (FP64-VALU EFT) GEMM on the GPU against the oracle: bit for bit
(one ascending-k chain per entry on both sides), plus the error bound against
the exact product on sampled entries."""
import math

import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, mp_frac, sample_entries
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def make(P, ta, tb, m, n, k, fam, pad=0, beta_zero=False, unit_alpha=False):
    A_rows, A_cols = (m, k) if ta == "N" else (k, m)
    B_rows, B_cols = (k, n) if tb == "N" else (n, k)
    A = synth.mp_matrix(fam, "A", P, A_rows, A_cols, ld=A_rows + pad)
    B = synth.mp_matrix(fam, "B", P, B_rows, B_cols, ld=B_rows + pad)
    C = synth.mp_matrix(fam, "C", P, m, n, ld=m + pad)
    alpha = synth.mp_one(P) if unit_alpha else synth.mp_scalar(fam, "alpha", P)
    beta = np.zeros(P) if beta_zero else synth.mp_scalar(fam, "beta", P)
    return A, B, C, alpha, beta


def run_gpu(mp, P, ta, tb, m, n, k, alpha, A, B, beta, C, **kw):
    dA, dB, dC = dev(A), dev(B), dev(C)
    mp.gemm(P, ta, tb, m, n, k, alpha, dA, dB, beta, dC, **kw)
    return host(dC)


def test_dd256_bitwise_and_bound(gpu_lib):
    """DD, m = n = k = 256, alpha = 1, beta = 0: every entry bit-identical to
    the oracle, and within 8 k u (|A||B|)_ij of the exact product."""
    P, m = 2, 256
    A, B, C, alpha, beta = make(P, "N", "N", m, m, m, fam=1, beta_zero=True, unit_alpha=True)
    want = oracle.gemm(P, "N", "N", m, m, m, alpha, A, B, beta, C)
    note("plain DD 256 cube")
    got = run_gpu(gpu_lib, P, "N", "N", m, m, m, alpha, A, B, beta, C)
    assert np.array_equal(got, want)
    chk = GemmChecker(P, "N", "N", m, m, m, alpha, A, B, beta, C)
    rng = synth.rng_for(1, "samples")
    r = chk.ratios(got, sample_entries(rng, m, m, 1024))
    print("DD 256 cube: max err / (k u |A||B|) =", r.max())
    assert r.max() <= 8.0


SHAPES = [(1, 1, 1), (67, 45, 33), (130, 129, 65), (5, 200, 17)]


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_ragged_shapes_all_tiles_bitwise(gpu_lib, P, ta, tb):
    for (m, n, k) in SHAPES:
        A, B, C, alpha, beta = make(P, ta, tb, m, n, k, fam=2, pad=3)
        want = oracle.gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C)
        for tile in range(gpu_lib.num_configs(P, "plain")):
            note("plain", P, ta, tb, (m, n, k), "tile", tile)
            got = run_gpu(gpu_lib, P, ta, tb, m, n, k, alpha, A, B, beta, C, form="plain", tile=tile)
            assert np.array_equal(got, want), (P, ta, tb, (m, n, k), tile)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_alpha_beta_semantics(gpu_lib, P):
    m, n, k = 37, 29, 41
    A, B, C, alpha, beta = make(P, "N", "N", m, n, k, fam=3)
    zero, one = np.zeros(P), synth.mp_one(P)
    Cnan = np.full_like(C, np.nan)
    cases = [(alpha, zero, Cnan, k),          # beta == 0: C never read
             (zero, beta, C, k),              # alpha == 0: C = beta C
             (zero, zero, Cnan, k),           # C = 0
             (alpha, beta, C, 0),             # k == 0: C = beta C
             (zero, one, Cnan, k),            # quick return: untouched
             (alpha, one, C, k)]              # beta == 1, full update
    for al, be, C0, kk in cases:
        want = oracle.gemm(P, "N", "N", m, n, kk, al, A, B, be, C0)
        note("semantics", P, al[0], be[0], kk)
        got = run_gpu(gpu_lib, P, "N", "N", m, n, kk, al, A, B, be, C0)
        same = (got == want) | (np.isnan(got) & np.isnan(want))
        assert same.all()


def test_plane_stride_larger_than_plane(gpu_lib):
    P, m, n, k = 3, 40, 30, 20
    A, B, C, alpha, beta = make(P, "N", "N", m, n, k, fam=4)
    want = oracle.gemm(P, "N", "N", m, n, k, alpha, A, B, beta, C)
    # embed each plane in a larger buffer: plane stride = cols * ld + 7
    def spread(X):
        Pn, cols, ld = X.shape
        buf = np.zeros(Pn * (cols * ld + 7))
        for p in range(Pn):
            buf[p * (cols * ld + 7): p * (cols * ld + 7) + cols * ld] = X[p].reshape(-1)
        return buf, cols * ld + 7
    import ctypes as Cc
    import torch
    L = gpu_lib.load()
    bufs = [spread(X) for X in (A, B, C)]
    dA, dB, dC = (torch.from_numpy(b).cuda() for b, _ in bufs)
    sa, sb, sc = (s for _, s in bufs)
    note("plane stride")
    rc = L.mpgemm_td(b"N", b"N", m, n, k, (Cc.c_double * 3)(*alpha), Cc.c_void_p(dA.data_ptr()), m, sa,
                     Cc.c_void_p(dB.data_ptr()), k, sb, (Cc.c_double * 3)(*beta),
                     Cc.c_void_p(dC.data_ptr()), m, sc, None)
    assert rc == 0
    out = host(dC)
    got = np.stack([out[p * sc: p * sc + n * m].reshape(n, m) for p in range(P)])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("n", [1023, 4096])
def test_square_full_size_sampled(gpu_lib, P, n):
    """Square n x n x n with random alpha/beta and C (the benchmark workload):
    the GPU computes all of C; the oracle recomputes a sampled block, which
    must match bit for bit; sampled entries meet the error bound."""
    A, B, C, alpha, beta = make(P, "N", "N", n, n, n, fam=2)
    note("plain square full size", P, n)
    got = run_gpu(gpu_lib, P, "N", "N", n, n, n, alpha, A, B, beta, C)
    rng = synth.rng_for(2, "samples")
    r0 = int(rng.integers(0, n - 2))
    c0 = int(rng.integers(0, n - 64))
    for rows, cols in [((r0, r0 + 2), (c0, c0 + 64)), ((n - 1, n), (n - 16, n))]:
        want = oracle.gemm(P, "N", "N", n, n, n, alpha, A, B, beta, C, rows=rows, cols=cols)
        blk = (slice(None), slice(*cols), slice(*rows))
        assert np.array_equal(got[blk], want[blk]), (P, n, rows, cols)
    chk = GemmChecker(P, "N", "N", n, n, n, alpha, A, B, beta, C)
    ratios = chk.ratios(got, sample_entries(rng, n, n, 64))
    print(f"square P={P} n={n}: max err / (k u (|alpha||A||B| + |beta||C|)) = {ratios.max():.3g}")
    assert ratios.max() <= 8 * (n + 2) / n


@pytest.mark.parametrize("P,n", [(2, 1024), (3, 257), (4, 129)])
def test_paper_matrices(gpu_lib, P, n):
    """The paper's fixed matrices A = sqrt5 (i+j-1), B = sqrt3 (n-i): at most
    one or two decimal digits lost, and bitwise equal to the oracle."""
    A, B = synth.paper_matrices(n, P)
    one, zero = synth.mp_one(P), np.zeros(P)
    C = np.zeros((P, n, n))
    note("paper matrices", P, n)
    got = run_gpu(gpu_lib, P, "N", "N", n, n, n, one, A, B, zero, C)
    want = oracle.gemm(P, "N", "N", n, n, n, one, A, B, zero, C, rows=(0, 4))
    assert np.array_equal(got[:, :, :4], want[:, :, :4])
    u = {2: 2.0 ** -104, 3: 2.0 ** -150, 4: 2.0 ** -200}[P]
    for i in (0, n // 3, n - 1):
        ex = synth.paper_exact_entry(n, i + 1)
        for j in (0, n - 1):
            rel = abs(mp_frac(got[:, j, i]) - ex) / ex
            digits = math.inf if rel == 0 else -math.log10(float(rel))
            assert digits >= -math.log10(u) - 2, (P, n, i, j, digits)

"""Residue (CRT) form of the split product on the GPU: bit for bit against
the oracle's residue form (the exact product of the digit integers, rounded
component by component), on ragged shapes, every transpose pair, odd and
even digit counts and every modulus-count bucket; at the benchmark size on
sampled blocks, and within the truncation bound of the exact product."""
import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, sample_entries
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def make(P, ta, tb, m, n, k, fam, exp_range=None):
    A_rows, A_cols = (m, k) if ta == "N" else (k, m)
    B_rows, B_cols = (k, n) if tb == "N" else (n, k)
    A = synth.mp_matrix(fam, "A", P, A_rows, A_cols, exp_range=exp_range)
    B = synth.mp_matrix(fam, "B", P, B_rows, B_cols, exp_range=exp_range)
    C = synth.mp_matrix(fam, "C", P, m, n)
    return A, B, C, synth.mp_scalar(fam, "alpha", P), synth.mp_scalar(fam, "beta", P)


def run(gpu_lib, P, ta, tb, m, n, k, alpha, A, B, beta, C, s, tile=-1):
    ws = gpu_lib.alloc_workspace(P, m, n, k, s, tile, form="crt")
    dC = dev(C)
    gpu_lib.gemm(P, ta, tb, m, n, k, alpha, dev(A), dev(B), beta, dC, form="crt", slices=s, tile=tile,
                 workspace=ws)
    return host(dC)


CASES = [
    # P, ta, tb, m, n, k, s, tile        (moduli: from k and s)
    (2, "N", "N", 130, 67, 100, 16, 0),    # 31 moduli, 8 limbs
    (2, "T", "N", 64, 64, 64, 5, 1),       # odd s; 10 moduli, 4 limbs
    (3, "N", "T", 97, 140, 33, 23, 1),     # 46 moduli, 11 limbs
    (3, "T", "T", 129, 31, 70, 23, 0),
    (4, "N", "N", 1, 1, 1, 9, 1),          # 16 moduli
    (4, "T", "N", 200, 3, 129, 20, 0),     # QD with a feasible s: 40 moduli
    (2, "N", "T", 33, 65, 17, 1, 1),       # one digit: 3 moduli
    (2, "N", "N", 257, 300, 1000, 16, 0),  # 16 k-tiles
    (3, "N", "N", 65, 70, 2000, 23, 1),    # 48 moduli, 11 limbs
    (2, "T", "T", 70, 129, 300, 11, 1),    # 21 moduli, 6 limbs
    (3, "N", "N", 50, 40, 90, 14, 0),      # 27 moduli
    (2, "N", "T", 50, 60, 50, 13, 0),      # 25 moduli, 6 limbs
    (4, "T", "T", 40, 41, 129, 20, 1),     # 40 moduli
    # QD beyond one level: two halves, three products (hh, ll, ss) of N moduli
    (4, "N", "N", 70, 65, 100, 31, 0),     # default s: halves of 16 + 15 digits
    (4, "T", "N", 33, 129, 70, 32, 1),     # 16 + 16
    (4, "N", "T", 66, 40, 300, 25, 2),     # 13 + 12
    (4, "T", "T", 17, 19, 2000, 28, 0),    # 14 + 14, 32 k-tiles
    # op(A) and op(B) padded to different row counts: the shared residue
    # launch has row blocks past the shorter operand
    (2, "N", "N", 600, 40, 150, 16, 0),    # 768 vs 256 rows
    (3, "N", "T", 300, 9, 64, 23, 2),      # 384 vs 128
    (4, "T", "N", 20, 530, 90, 31, 1),     # two levels; 256 vs 640
    # the largest modulus counts: 49 (all) at one level, and two levels of
    # 33 (a second block of 32 moduli per set: s = 32, k = 65536)
    (2, "N", "T", 70, 40, 50, 24, 0),      # 49 moduli, 11 limbs
    (4, "T", "N", 20, 17, 65536, 32, 0),   # 3 x 33 moduli, 2048 k-tiles
]


@pytest.mark.parametrize("P,ta,tb,m,n,k,s,tile", CASES)
def test_bitwise_against_oracle(gpu_lib, P, ta, tb, m, n, k, s, tile):
    A, B, C, alpha, beta = make(P, ta, tb, m, n, k, fam=5)
    note("crt", P, ta, tb, (m, n, k), "s", s, "tile", tile)
    got = run(gpu_lib, P, ta, tb, m, n, k, alpha, A, B, beta, C, s, tile)
    want = oracle.gemm_crt(P, s, ta, tb, m, n, k, alpha, A, B, beta, C)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_exponent_spread_and_beta_zero(gpu_lib, P):
    """Entries u 2^e with e in -30..30 per entry (wide scale exponents, long
    remainders), beta = 0 and alpha = 1."""
    m, n, k = 90, 75, 130
    s = gpu_lib.DEFAULT_SLICES[P]
    A, B, _, _, _ = make(P, "N", "N", m, n, k, fam=3, exp_range=(-30, 30))
    one, zero = synth.mp_one(P), np.zeros(P)
    C = np.full((P, n, m), np.nan)          # beta = 0: C is not read
    note("crt spread", P, (m, n, k))
    got = run(gpu_lib, P, "N", "N", m, n, k, one, A, B, zero, C, s)
    want = oracle.gemm_crt(P, s, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)))
    assert np.array_equal(got, want)


def test_integers_exact(gpu_lib):
    """Integer operands below 2^12: the product is the exact integer matrix."""
    P, m, n, k = 2, 70, 66, 300
    rng = np.random.Generator(np.random.PCG64(77))
    A = np.zeros((P, k, m)); A[0] = rng.integers(-4096, 4096, (k, m))
    B = np.zeros((P, n, k)); B[0] = rng.integers(-4096, 4096, (n, k))
    one, zero = synth.mp_one(P), np.zeros(P)
    note("crt integers", (m, n, k))
    got = run(gpu_lib, P, "N", "N", m, n, k, one, A, B, zero, np.zeros((P, n, m)), 16)
    exact = A[0].T.astype(np.int64) @ B[0].T.astype(np.int64)
    assert np.array_equal(got[0].T, exact.astype(np.float64)) and not got[1:].any()


@pytest.mark.parametrize("P", [2, 3, 4])
def test_full_size_sampled(gpu_lib, P):
    """The benchmark's square workload (n = 4096, default digits): sampled
    blocks bit-identical to the oracle's residue form, sampled entries within
    the split form's bound of the exact product."""
    n = 4096
    A, B, C, alpha, beta = make(P, "N", "N", n, n, n, fam=2)
    s = gpu_lib.DEFAULT_SLICES[P]
    note("crt full size", P, n, s)
    got = run(gpu_lib, P, "N", "N", n, n, n, alpha, A, B, beta, C, s)
    rng = synth.rng_for(2, 9)                # a seed slot of its own
    r0 = int(rng.integers(0, n - 2))
    c0 = int(rng.integers(0, n - 16))
    for rows, cols in [((r0, r0 + 2), (c0, c0 + 16)), ((n - 1, n), (n - 8, n)), ((0, 1), (0, 8))]:
        want = oracle.gemm_crt(P, s, "N", "N", n, n, n, alpha, A, B, beta, C, rows=rows, cols=cols)
        blk = (slice(None), slice(*cols), slice(*rows))
        assert np.array_equal(got[blk], want[blk]), (P, rows, cols)
    chk = GemmChecker(P, "N", "N", n, n, n, alpha, A, B, beta, C)
    r = chk.ratios(got, sample_entries(rng, n, n, 64))
    print(f"crt P={P} n={n} s={s}: max err / (k u (|alpha||A||B| + |beta||C|)) = {r.max():.3g}")
    assert r.max() <= 8 * (n + 2) / n


@pytest.mark.parametrize("P,m,n,k,s,tile", [
    (2, 1100, 1100, 300, 16, 0),    # 25 tiles: 31 planes in 11 groups of 3 (the last holds 1)
    (4, 700, 700, 200, 31, 2),      # 36 tiles: 93 planes (two levels) in 14 groups of 7 (last 2)
])
def test_planes_shared_out_over_workgroups(gpu_lib, P, m, n, k, s, tile):
    """Few output tiles: each tile's planes are split over several
    workgroups (an uneven last share); sampled blocks bit for bit."""
    A, B, C, alpha, beta = make(P, "N", "N", m, n, k, fam=8)
    note("crt plane groups", P, (m, n, k), "s", s, "tile", tile)
    got = run(gpu_lib, P, "N", "N", m, n, k, alpha, A, B, beta, C, s, tile)
    for rows, cols in [((0, 40), (0, 24)), ((m - 33, m), (n - 17, n)), ((300, 310), (500, 520))]:
        want = oracle.gemm_crt(P, s, "N", "N", m, n, k, alpha, A, B, beta, C, rows=rows, cols=cols)
        blk = (slice(None), slice(*cols), slice(*rows))
        assert np.array_equal(got[blk], want[blk]), (rows, cols)


def test_repeat_and_workspace_reuse(gpu_lib):
    """Deterministic: repeated calls, a larger reused workspace and both
    tile configurations give the same bits."""
    P, m, n, k, s = 3, 150, 130, 260, 23
    A, B, C, alpha, beta = make(P, "T", "N", m, n, k, fam=6)
    big = gpu_lib.alloc_workspace(P, 300, 300, 600, s, 0, form="crt")
    outs = []
    for tile in (0, 1, 0):
        note("crt reuse", tile)
        dC = dev(C)
        gpu_lib.gemm(P, "T", "N", m, n, k, alpha, dev(A), dev(B), beta, dC, form="crt", slices=s,
                     tile=tile, workspace=big)
        outs.append(host(dC))
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    small = gpu_lib.alloc_workspace(P, 8, 8, 8, s, 0, form="crt")
    with pytest.raises(gpu_lib.MPGemmError) as e:
        gpu_lib.gemm(P, "T", "N", m, n, k, alpha, dev(A), dev(B), beta, dev(C), form="crt", slices=s,
                     tile=0, workspace=small)
    assert e.value.code == 2


@pytest.mark.parametrize("P", [2, 3, 4])
def test_auto_form_choice(gpu_lib, P):
    """FORM_AUTO: the residue form when the workspace holds it, the
    triangular split form when only that fits, the plain form with no
    workspace or below the sizes where the others pay -- each bit for bit
    as the oracle's form."""
    import torch
    m, n, k = 256, 260, 300
    A, B, C, alpha, beta = make(P, "N", "N", m, n, k, fam=7)
    s = gpu_lib.DEFAULT_SLICES[P]
    split_b = gpu_lib.workspace_bytes(P, "split", m, n, k, s)
    crt_b = gpu_lib.workspace_bytes(P, "crt", m, n, k, s)
    assert crt_b > split_b > 0
    assert gpu_lib.workspace_bytes(P, "auto", m, n, k, s) == crt_b

    def call(ws, mm=m):
        dC = dev(C)
        gpu_lib.gemm(P, "N", "N", mm, n, k, alpha, dev(A), dev(B), beta, dC, form="auto", slices=s,
                     workspace=ws)
        return host(dC)

    big = gpu_lib.alloc_workspace(P, m, n, k, s, form="auto")
    small = torch.empty(split_b, dtype=torch.uint8, device="cuda")
    note("auto: residue, split, plain", P, (m, n, k))
    assert np.array_equal(call(big), oracle.gemm_crt(P, s, "N", "N", m, n, k, alpha, A, B, beta, C))
    assert np.array_equal(call(small), oracle.gemm_split(P, s, "N", "N", m, n, k, alpha, A, B, beta, C))
    plain = oracle.gemm(P, "N", "N", m, n, k, alpha, A, B, beta, C)
    assert np.array_equal(call(None), plain)
    assert np.array_equal(call(big[1:]), plain)            # not 256-byte aligned: plain as well
    # below the residue form's smallest size (DD 128, TD 96, QD 64; lda
    # stays 256): the triangular split form needs 256, so plain
    mm = {2: 127, 3: 95, 4: 63}[P]
    assert np.array_equal(call(big, mm), oracle.gemm(P, "N", "N", mm, n, k, alpha, A, B, beta, C))
    # from that size on the residue form, also with little room above it
    mm = {2: 128, 3: 96, 4: 64}[P]
    assert np.array_equal(call(big, mm), oracle.gemm_crt(P, s, "N", "N", mm, n, k, alpha, A, B, beta, C))


@pytest.mark.parametrize("P", [2, 4])
def test_degenerate_shapes_and_scalars(gpu_lib, P):
    """Residue form on the cases it shares with every form: k = 0 and
    alpha = 0 (C = beta C), alpha = 0 with beta = 1 (C untouched), m = 0 or
    n = 0 (nothing to do) -- each as the oracle has it."""
    m, n, k = 40, 33, 70
    A, B, C, alpha, beta = make(P, "N", "N", m, n, k, fam=9)
    s = gpu_lib.DEFAULT_SLICES[P]
    zero, one = np.zeros(P), synth.mp_one(P)
    for kk, al, be in [(0, alpha, beta), (k, zero, beta), (k, zero, one)]:
        note("crt degenerate", P, "k", kk, "alpha zero", not np.any(al), "beta one", np.array_equal(be, one))
        got = run(gpu_lib, P, "N", "N", m, n, kk, al, A, B, be, C, s)
        assert np.array_equal(got, oracle.gemm(P, "N", "N", m, n, kk, al, A, B, be, C))
    for mm, nn in [(0, n), (m, 0)]:
        note("crt empty", P, mm, nn)
        got = run(gpu_lib, P, "N", "N", mm, nn, k, alpha, A, B, beta, C, s)
        assert np.array_equal(got, C)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_auto_form_without_digit_count_is_plain_on_spread_inputs(gpu_lib, P):
    """FORM_AUTO with slices = 0 runs the plain form, also with a workspace
    that would hold the residue form: on entries u 2^e with e in -60..60 per
    entry the default digit count leaves the componentwise bound, so the
    library does not choose a split form on its own.  Bit for bit as the
    oracle's canonical product, and within 8 (k+2) u on sampled entries."""
    m, n, k = 200, 190, 180
    A, B, C, alpha, beta = make(P, "N", "N", m, n, k, fam=11, exp_range=(-60, 60))
    s = gpu_lib.DEFAULT_SLICES[P]
    ws = gpu_lib.alloc_workspace(P, m, n, k, s, form="auto")
    dC = dev(C)
    note("auto without slices on spread inputs", P, (m, n, k))
    gpu_lib.gemm(P, "N", "N", m, n, k, alpha, dev(A), dev(B), beta, dC, form="auto", workspace=ws)
    got = host(dC)
    assert np.array_equal(got, oracle.gemm(P, "N", "N", m, n, k, alpha, A, B, beta, C))
    chk = GemmChecker(P, "N", "N", m, n, k, alpha, A, B, beta, C)
    r = chk.ratios(got, sample_entries(synth.rng_for(11, 9), m, n, 64))
    assert r.max() <= 8 * (k + 2) / k
    # with the default digit count given explicitly it is the residue form,
    # bit for bit (its accuracy on such inputs is the caller's choice)
    dC = dev(C)
    gpu_lib.gemm(P, "N", "N", m, n, k, alpha, dev(A), dev(B), beta, dC, form="auto", slices=s, workspace=ws)
    assert np.array_equal(host(dC), oracle.gemm_crt(P, s, "N", "N", m, n, k, alpha, A, B, beta, C))

"""Split (INT8 MFMA) form on the GPU against the oracle's split form, stage by
stage (exponents and digits bit for bit, anti-diagonal sums as exact
integers, the recombined product bit for bit), and against the exact product
within the error bound."""
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


def workspace_views(ws, lay, s):
    raw = host(ws)
    Mp, Np, Kp = lay["Mp"], lay["Np"], lay["Kp"]
    E = raw[lay["E"]: lay["E"] + 4 * Mp].view(np.int32)
    F = raw[lay["F"]: lay["F"] + 4 * Np].view(np.int32)
    # digit planes are k-tile-major: [s][Kp/KT][rows][KT], KT = 64
    KT = 64
    nkt = Kp // KT
    DA = raw[lay["DA"]: lay["DA"] + s * Mp * Kp].view(np.int8).reshape(s, nkt, Mp, KT)
    DA = DA.transpose(0, 2, 1, 3).reshape(s, Mp, Kp)
    DB = raw[lay["DB"]: lay["DB"] + s * Np * Kp].view(np.int8).reshape(s, nkt, Np, KT)
    DB = DB.transpose(0, 2, 1, 3).reshape(s, Np, Kp)
    S = raw[lay["S"]: lay["S"] + 4 * s * Np * Mp].view(np.int32).reshape(s, Np, Mp)
    return E, F, DA, DB, S


CASES = [
    # P, ta, tb, m, n, k, s, tile
    (2, "N", "N", 130, 67, 100, 16, 0),
    (2, "T", "N", 64, 64, 64, 5, 1),
    (3, "N", "T", 97, 140, 33, 23, 1),
    (4, "T", "T", 129, 31, 70, 30, 0),
    (4, "N", "N", 1, 1, 1, 9, 1),
    (3, "T", "N", 200, 3, 129, 18, 0),
    (2, "N", "N", 700, 20, 90, 16, 1),     # operands padded to different row counts
    (4, "T", "T", 9, 450, 60, 31, 0),
]
# tile configuration 2 (128 x 64, four diagonals at once): one ragged shape
# per precision under every transpose pair
CASES += [(P, ta, tb, m, n, k, s, 2)
          for (P, m, n, k, s) in [(2, 150, 70, 90, 16), (3, 131, 129, 45, 23), (4, 257, 63, 70, 31)]
          for ta in "NT" for tb in "NT"]


@pytest.mark.parametrize("P,ta,tb,m,n,k,s,tile", CASES)
def test_stages_bitwise(gpu_lib, P, ta, tb, m, n, k, s, tile):
    A, B, C, alpha, beta = make(P, ta, tb, m, n, k, fam=5)
    lay = gpu_lib.split_layout(P, m, n, k, s, tile)
    ws = gpu_lib.alloc_workspace(P, m, n, k, s, tile)
    ws.zero_()
    dA, dB, dC = dev(A), dev(B), dev(C)
    note("split stages", P, ta, tb, (m, n, k), "s", s, "tile", tile)
    gpu_lib.split_stages(P, 3, ta, tb, m, n, k, alpha, dA, dB, beta, dC, slices=s, tile=tile,
                         workspace=ws)
    E, F, DA, DB, S = workspace_views(ws, lay, s)
    wantC, wE, wF, wS = oracle.gemm_split(P, s, ta, tb, m, n, k, alpha, A, B, beta, C, debug=True)
    # stage 1: exponents (padding rows/columns get 0)
    assert np.array_equal(E[:m], wE) and not E[m:].any()
    assert np.array_equal(F[:n], wF) and not F[n:].any()
    # stage 2: digits, zero outside the matrix
    wDA = oracle.split_slices(P, s, ta, 0, m, k, A, wE)
    wDB = oracle.split_slices(P, s, tb, 1, n, k, B, wF)
    assert np.array_equal(DA[:, :m, :k], wDA)
    assert np.array_equal(DB[:, :n, :k], wDB)
    assert not DA[:, m:, :].any() and not DA[:, :, k:].any()
    assert not DB[:, n:, :].any() and not DB[:, :, k:].any()
    # stage 3: anti-diagonal sums, exact integers
    assert np.array_equal(S[:, :n, :m].astype(np.int64), wS)
    # stage 4: the whole product
    note("split full", P, (m, n, k), s, tile)
    dC2 = dev(C)
    gpu_lib.gemm(P, ta, tb, m, n, k, alpha, dA, dB, beta, dC2, form="split", slices=s, tile=tile,
                 workspace=ws)
    assert np.array_equal(host(dC2), wantC)


@pytest.mark.parametrize("P,n,tile", [(P, n, None) for P in (2, 3, 4) for n in (1025, 4096)]
                         + [(P, 1025, 2) for P in (2, 3, 4)])
def test_full_size_sampled(gpu_lib, P, n, tile):
    """The benchmark's square workload in the split form: a sampled block
    bit-identical to the oracle's split form, sampled entries within the
    error bound of the exact product."""
    A, B, C, alpha, beta = make(P, "N", "N", n, n, n, fam=2)
    s = gpu_lib.DEFAULT_SLICES[P]
    t = -1 if tile is None else tile
    ws = gpu_lib.alloc_workspace(P, n, n, n, s, t)
    dA, dB, dC = dev(A), dev(B), dev(C)
    note("split full size", P, n, s, "tile", tile)
    gpu_lib.gemm(P, "N", "N", n, n, n, alpha, dA, dB, beta, dC, form="split", slices=s, tile=t,
                 workspace=ws)
    got = host(dC)
    rng = synth.rng_for(2, "samples")
    r0 = int(rng.integers(0, n - 2))
    c0 = int(rng.integers(0, n - 16))
    for rows, cols in [((r0, r0 + 2), (c0, c0 + 16)), ((n - 1, n), (n - 8, n))]:
        want = oracle.gemm_split(P, s, "N", "N", n, n, n, alpha, A, B, beta, C, rows=rows, cols=cols)
        blk = (slice(None), slice(*cols), slice(*rows))
        assert np.array_equal(got[blk], want[blk]), (P, n, rows, cols)
    chk = GemmChecker(P, "N", "N", n, n, n, alpha, A, B, beta, C)
    r = chk.ratios(got, sample_entries(rng, n, n, 64))
    print(f"split P={P} n={n} s={s}: max err / (k u (|alpha||A||B| + |beta||C|)) = {r.max():.3g}")
    assert r.max() <= 8 * (n + 2) / n


def test_qd_exponent_spread_with_tuned_slices(gpu_lib):
    """The QD spread input class (entries u 2^e, e in -30..30 per entry) at a
    reduced size: the slice count picked by the accuracy rule keeps the split
    result within the bound of the exact product."""
    P, n = 4, 512
    A, B, _, _, _ = make(P, "N", "N", n, n, n, fam=3, exp_range=(-30, 30))
    one, zero = synth.mp_one(P), np.zeros(P)
    C = np.zeros((P, n, n))
    dA, dB = dev(A), dev(B)
    note("tune slices QD spread", n)
    s, ratio = gpu_lib.tune_slices(P, "N", "N", n, n, n, dA, dB, target=1.0, smin=28, smax=40)
    print("tuned slices:", s, "ratio vs plain:", ratio)
    assert 28 <= s <= 40
    ws = gpu_lib.alloc_workspace(P, n, n, n, s)
    dC = dev(C)
    gpu_lib.gemm(P, "N", "N", n, n, n, one, dA, dB, zero, dC, form="split", slices=s, workspace=ws)
    got = host(dC)
    chk = GemmChecker(P, "N", "N", n, n, n, one, A, B, zero, C)
    r = chk.ratios(got, sample_entries(synth.rng_for(3, "samples"), n, n, 256))
    print("QD spread class, split: max err ratio", r.max())
    assert r.max() <= 8.0


def test_workspace_reuse_and_errors(gpu_lib):
    """A workspace that is too small is rejected; a larger one reused across
    calls of different shapes gives the same bits as fresh ones."""
    P = 2
    A, B, C, alpha, beta = make(P, "N", "N", 100, 90, 80, fam=6)
    big = gpu_lib.alloc_workspace(P, 300, 300, 300, 16)
    small = gpu_lib.alloc_workspace(P, 10, 10, 10, 16)
    dA, dB = dev(A), dev(B)
    dC = dev(C)
    rc = gpu_lib.gemm_raw(P, "N", "N", 100, 90, 80, alpha, dA, dB, beta, dC, form="split", slices=16,
                          workspace=small)
    assert rc == 2
    outs = []
    for ws in (big, gpu_lib.alloc_workspace(P, 100, 90, 80, 16)):
        dC = dev(C)
        gpu_lib.gemm(P, "N", "N", 100, 90, 80, alpha, dA, dB, beta, dC, form="split", slices=16,
                     workspace=ws)
        outs.append(host(dC))
    assert np.array_equal(outs[0], outs[1])

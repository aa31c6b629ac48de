"""The two other benchmark workloads at full size, in the launch
configuration bench.py times, in every form it times (plain, split and its
residue variant):

* QD m = n = k = 2048 with entries u 2^e, e drawn per entry from -30..30,
  slices from the accuracy rule;
* DD m = n = k = 8192.

Sampled blocks are bit-identical to the oracle (its canonical plain order, and
its split and residue forms with the same slice count); sampled entries meet
the error bound against the exact product."""
import numpy as np
import pytest

import oracle
from tests import synth
from tests.exact import GemmChecker, sample_entries
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu

SAME_ERROR_TARGET = 1e-6      # the accuracy rule's target in bench.py --workload qd2048-spread


def blocks(fam, n):
    rng = synth.rng_for(fam, "samples")
    r0 = int(rng.integers(0, n - 1))
    c0 = int(rng.integers(0, n - 32))
    return rng, [((r0, r0 + 1), (c0, c0 + 32)), ((n - 1, n), (n - 8, n))]


def check_forms(gpu_lib, fam, P, n, A, B, s, samples):
    import torch
    one, zero = synth.mp_one(P), np.zeros(P)
    Cz = np.zeros((P, n, n))                  # beta = 0: C is never read
    dA, dB = dev(A), dev(B)
    rng, blks = blocks(fam, n)
    ents = sample_entries(rng, n, n, samples)
    chk = GemmChecker(P, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, 1)))
    for form in ("plain", "split", "crt"):
        dC = torch.zeros((P, n, n), dtype=torch.float64, device="cuda")
        note("workload", P, n, form, "s", s)
        ws = gpu_lib.alloc_workspace(P, n, n, n, s, form=form) if form != "plain" else None
        kw = dict(form=form, slices=s, workspace=ws) if form != "plain" else dict(form="plain")
        gpu_lib.gemm(P, "N", "N", n, n, n, one, dA, dB, zero, dC, **kw)
        got = host(dC)
        del dC, ws
        ref = {"plain": None, "split": oracle.gemm_split, "crt": oracle.gemm_crt}[form]
        for rows, cols in blks:
            if form == "plain":
                want = oracle.gemm(P, "N", "N", n, n, n, one, A, B, zero, Cz, rows=rows, cols=cols)
            else:
                want = ref(P, s, "N", "N", n, n, n, one, A, B, zero, Cz, rows=rows, cols=cols)
            blk = (slice(None), slice(*cols), slice(*rows))
            assert np.array_equal(got[blk], want[blk]), (P, n, form, rows, cols)
        r = chk.ratios(got, ents)
        print(f"{'DD' if P == 2 else 'QD'} n={n} {form}: max err / (k u |A||B|) = {r.max():.3g}, "
              f"median {np.median(r):.3g}")
        assert r.max() <= 8.0, (P, n, form, r.max())


def test_qd2048_exponent_spread(gpu_lib):
    P, n = 4, 2048
    A = synth.mp_matrix(3, "A", P, n, n, exp_range=(-30, 30))
    B = synth.mp_matrix(3, "B", P, n, n, exp_range=(-30, 30))
    note("qd2048 spread: slice rule")
    s, ratio = gpu_lib.tune_slices(P, "N", "N", n, n, n, dev(A), dev(B), target=SAME_ERROR_TARGET,
                                   smin=28, smax=40)
    print("qd2048 spread: slices", s, "rule ratio", ratio)
    assert 28 <= s <= 40 and ratio <= SAME_ERROR_TARGET
    assert gpu_lib.crt_moduli(P, n, s) > 0           # the residue form covers the chosen s
    check_forms(gpu_lib, 3, P, n, A, B, s, samples=128)


def test_dd8192(gpu_lib):
    P, n = 2, 8192
    A = synth.mp_matrix(4, "A", P, n, n)
    B = synth.mp_matrix(4, "B", P, n, n)
    check_forms(gpu_lib, 4, P, n, A, B, gpu_lib.DEFAULT_SLICES[P], samples=32)

"""A seeded random sweep over precisions, transpose pairs, shapes (ragged
against every tile), tile configurations, digit counts and alpha/beta,
beyond the hand-picked cases of the other files: the plain form bit for bit
as the oracle's canonical GEMM (for TD with a random choice of the TD
addition and multiplication variants), the triangular split and the residue form bit
for bit as the oracle's split and residue forms.  Operands carry a per-row
and per-column exponent spread in half of the cases, so that the scale
exponents differ from row to row."""
import numpy as np
import pytest

import oracle
from paper_2101_06584_amd import _lib
from tests import synth
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu

TRANS = "NnTtCc"


def draw(form, q):
    rng = np.random.Generator(np.random.PCG64(7700 + 100 * ["plain", "split", "crt"].index(form) + q))
    P = int(rng.integers(2, 5))
    ta, tb = TRANS[int(rng.integers(6))], TRANS[int(rng.integers(6))]
    big = 160 if form != "split" else 100
    m, n = int(rng.integers(1, big + 1)), int(rng.integers(1, big + 1))
    k = int(rng.integers(1, (260 if form != "split" else 200) + 1))
    s = 0
    if form == "split":
        s = int(rng.integers(1, 21))
    elif form == "crt":
        s = int(rng.integers(1, (33 if P == 4 else 25)))
    spread = bool(rng.integers(2))
    rA = (m, k) if ta in "Nn" else (k, m)      # stored rows, columns
    rB = (k, n) if tb in "Nn" else (n, k)
    A = synth.mp_uniform(rng, P, (rA[1], rA[0]))  # (P, cols, ld)
    B = synth.mp_uniform(rng, P, (rB[1], rB[0]))
    C = synth.mp_uniform(rng, P, (n, m))
    if spread:
        A *= np.ldexp(1.0, rng.integers(-25, 26, rA[0]))[None, None, :]
        B *= np.ldexp(1.0, rng.integers(-25, 26, rB[1]))[None, :, None]
    alpha = synth.mp_uniform(rng, P, (1,))[:, 0]
    beta = synth.mp_uniform(rng, P, (1,))[:, 0] if rng.integers(3) else np.zeros(P)
    return P, ta, tb, m, n, k, s, A, B, C, alpha, beta, rng


@pytest.mark.parametrize("form,q", [("plain", q) for q in range(24)] + [("split", q) for q in range(14)] +
                         [("crt", q) for q in range(24)])
def test_random_case(gpu_lib, form, q):
    P, ta, tb, m, n, k, s, A, B, C, alpha, beta, rng = draw(form, q)
    tile = int(rng.integers(gpu_lib.num_configs(P, form)))
    # TD plain: the accurate addition (Algorithm 3) and / or TDmulq in place of the defaults
    variant = int(rng.integers(4)) if form == "plain" and P == 3 else 0
    note("sweep", form, q, P, ta, tb, (m, n, k), "s", s, "tile", tile, "variant", variant)
    dC = dev(C)
    if form == "crt" and gpu_lib.crt_moduli(P, k, s) == 0:
        # more digits than the moduli hold at this k: refused before any GPU
        # work, C untouched; then the largest digit count that fits
        rc = gpu_lib.gemm_raw(P, ta, tb, m, n, k, alpha, dev(A), dev(B), beta, dC, form="crt", slices=s,
                              tile=tile, workspace=gpu_lib.alloc_workspace(P, m, n, k, 16, tile, form="crt"))
        assert rc == _lib.ERR_UNSUPPORTED and np.array_equal(host(dC), C)
        while gpu_lib.crt_moduli(P, k, s) == 0:
            s -= 1
    if form == "plain":
        gpu_lib.gemm(P, ta, tb, m, n, k, alpha, dev(A), dev(B), beta, dC, form="plain", tile=tile,
                     variant=variant)
        want = oracle.gemm(P, ta, tb, m, n, k, alpha, A, B, beta, C, variant=variant)
    else:
        ws = gpu_lib.alloc_workspace(P, m, n, k, s, tile, form=form)
        gpu_lib.gemm(P, ta, tb, m, n, k, alpha, dev(A), dev(B), beta, dC, form=form, slices=s, tile=tile,
                     workspace=ws)
        f = oracle.gemm_split if form == "split" else oracle.gemm_crt
        want = f(P, s, ta, tb, m, n, k, alpha, A, B, beta, C)
    assert np.array_equal(host(dC), want), (form, q, P, ta, tb, m, n, k, s, tile)

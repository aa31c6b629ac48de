"""GPU element-wise DD/TD/QD add and mul (Sec. 2.5) against the oracle, bit
for bit, on random, cancelling and special inputs."""
import numpy as np
import pytest

import oracle
from tests import synth
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def inputs(P, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = synth.mp_uniform(rng, P, (n,))
    y = synth.mp_uniform(rng, P, (n,))
    x = np.ldexp(x, rng.integers(-40, 41, n)[None])
    y = np.ldexp(y, rng.integers(-40, 41, n)[None])
    k = n // 6
    y[:, :k] = -x[:, :k]
    y[0, :k] *= 1 + 2.0 ** -51                   # heavy cancellation
    y[:, k:2 * k] = -x[:, k:2 * k]               # exact cancellation
    x[1:, 2 * k:3 * k] = 0.0                     # single-double operands
    y[1:, 2 * k:3 * k] = 0.0
    y[:, 3 * k:3 * k + 10] = 0.0                 # zeros
    x[:, 4 * k:5 * k] = np.round(x[:, 4 * k:5 * k] * 2 ** 20)  # integers
    y[:, 4 * k:5 * k] = np.round(y[:, 4 * k:5 * k] * 2 ** 20)
    return x, y


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("op", ["add", "mul"])
def test_vec_bitwise(gpu_lib, P, op):
    n = 300_001                                   # ragged against 256-thread blocks
    x, y = inputs(P, n, 40 + P)
    want = oracle.vec(P, op, x, y)
    note("vec", P, op, n)
    dx, dy = dev(x), dev(y)
    dr = dev(np.zeros_like(x))
    gpu_lib.vec(P, op, dx, dy, dr)
    got = host(dr)
    bad = np.nonzero(~((got == want) | (np.isnan(got) & np.isnan(want))).all(axis=0))[0]
    assert bad.size == 0, (P, op, bad[:5], got[:, bad[:3]], want[:, bad[:3]])


def test_vec_in_place_and_empty(gpu_lib):
    P = 3
    x, y = inputs(P, 1000, 7)
    want = oracle.vec(P, "mul", x, y)
    note("vec in-place")
    dx, dy = dev(x), dev(y)
    gpu_lib.vec(P, "mul", dx, dy, dx)
    assert np.array_equal(host(dx), want)
    gpu_lib.vec(P, "add", dx, dy, dx, n=0)

"""Batched residue form: every residue problem bit for bit as the oracle's
residue form (the exact product of the digit integers, rounded once) and as
a single residue-form call; problems that do not multiply (alpha = 0, k = 0)
bit for bit as the oracle's canonical GEMM; AUTO's per-problem choice;
graph replays equal to a direct launch; chunked workspaces; grouped calls.

Operands carry a per-row (op(A)) and per-column (op(B)) exponent spread, so
that every problem's scale exponents differ from its neighbours' and a
block reading another problem's exponents or residues changes bits."""
import numpy as np
import pytest
import torch

import oracle
from tests import synth
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu

SLICES = {2: 16, 3: 23, 4: 20}          # QD: a one-level digit count
# (P, s): every precision at one level, and QD at two levels (s > 24), with
# halves of equal (s even) and unequal (s odd, its default) digit counts
PS = [(2, 16), (3, 23), (4, 20), (4, 31), (4, 26)]
CRT_MIN = {2: 128, 3: 96, 4: 64}        # the single call's AUTO sizes


def spread_problem(P, ta, tb, m, n, k, seed, alpha_zero=False):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = synth.mp_uniform(rng, P, (k, m) if ta == "N" else (m, k))
    B = synth.mp_uniform(rng, P, (n, k) if tb == "N" else (k, n))
    C = synth.mp_uniform(rng, P, (n, m))
    ea = np.ldexp(1.0, rng.integers(-20, 21, m))
    eb = np.ldexp(1.0, rng.integers(-20, 21, n))
    if ta == "N":
        A *= ea[None, None, :]          # row i of op(A) is A[:, :, i]
    else:
        A *= ea[None, :, None]
    if tb == "N":
        B *= eb[None, :, None]          # column j of op(B) is B[:, j, :]
    else:
        B *= eb[None, None, :]
    alpha = np.zeros(P) if alpha_zero else (synth.mp_uniform(rng, P, (1,))[:, 0] if seed % 2 else synth.mp_one(P))
    beta = synth.mp_uniform(rng, P, (1,))[:, 0] if seed % 3 else np.zeros(P)
    return dict(transa=ta, transb=tb, m=m, n=n, k=k, A=A, B=B, C=C, alpha=alpha, beta=beta)


TRANS = [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")]


def problem_set(P, shapes, seed0):
    return [spread_problem(P, *TRANS[q % 4], m, n, k, seed0 + q) for q, (m, n, k) in enumerate(shapes)]


def to_dev(probs):
    out = []
    for p in probs:
        d = dict(p)
        d["A"], d["B"], d["C"] = dev(p["A"]), dev(p["B"]), dev(p["C"])
        out.append(d)
    return out


def multiplies(p):
    return p["m"] > 0 and p["n"] > 0 and p["k"] > 0 and np.any(np.asarray(p["alpha"]) != 0)


def want_of(P, s, p, residue):
    f = (lambda *a: oracle.gemm_crt(P, s, *a)) if residue else (lambda *a: oracle.gemm(P, *a))
    return f(p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"], p["B"], p["beta"], p["C"])


def single_call(gpu_lib, P, s, d):
    ws = gpu_lib.alloc_workspace(P, d["m"], d["n"], d["k"], s, form="crt")
    C = d["C"].clone()
    gpu_lib.gemm(P, d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], d["A"], d["B"], d["beta"], C,
                 form="crt", slices=s, workspace=ws)
    return C


# ragged shapes around the 128-row product tiles and 64-wide k segments
EDGE = [(1, 1, 1), (128, 128, 128), (129, 257, 65), (127, 1, 64), (3, 130, 129), (200, 64, 1)]


@pytest.mark.parametrize("P,s", PS)
def test_batched_residue_against_oracle(gpu_lib, P, s):
    rng = synth.rng_for(11, 100 * P + s)
    shapes = [tuple(int(v) for v in r) for r in rng.integers(16, 200, size=(18, 3))] + EDGE
    probs = problem_set(P, shapes, 500 * P + s)
    probs.append(spread_problem(P, "N", "N", 40, 30, 20, 9001, alpha_zero=True))     # plain part
    k0 = spread_problem(P, "N", "N", 33, 17, 0, 9002)                               # k = 0
    k0["A"], k0["B"] = np.zeros((P, 1, 33)), np.zeros((P, 17, 1))   # leading dimensions >= 1
    probs.append(k0)
    dprobs = to_dev(probs)
    note("batched residue", P, len(probs), "s", s)
    plan = gpu_lib.BatchPlan(P, dprobs, form="crt", slices=s)
    info = plan.info()
    res = [multiplies(p) for p in probs]
    kmax = max(p["k"] for p, r in zip(probs, res) if r)
    assert info["residue_problems"] == sum(res)
    assert info["moduli"] == gpu_lib.crt_moduli(P, kmax, s)
    assert info["chunks"] == 1
    C0 = [d["C"].clone() for d in dprobs]
    plan.run()
    got = [host(d["C"]) for d in dprobs]
    for q, (p, r) in enumerate(zip(probs, res)):
        assert np.array_equal(got[q], want_of(P, s, p, r)), (P, q, p["m"], p["n"], p["k"], r)
    # a direct launch and a second replay (other work in between) give the same bits
    for rep, how in enumerate(("launch", "run")):
        for d, c0 in zip(dprobs, C0):
            d["C"].copy_(c0)
        note("batched residue", how, P)
        getattr(plan, how)()
        x = torch.randn(512, 512, device="cuda") @ torch.randn(512, 512, device="cuda")
        torch.cuda.synchronize()
        del x
        for q, d in enumerate(dprobs):
            assert np.array_equal(host(d["C"]), got[q]), (how, q)
    plan.close()
    # and the same bits as one residue-form call per problem
    for q in (0, 5, len(shapes) - 1):
        d = dict(dprobs[q])
        d["C"] = dev(probs[q]["C"])
        assert np.array_equal(host(single_call(gpu_lib, P, s, d)), got[q]), q


@pytest.mark.parametrize("P", [2, 3])
def test_batched_auto_chooses_per_problem(gpu_lib, P):
    """AUTO with s given: the residue form for problems with m, n, k at least
    the single call's residue sizes, the plain form (canonical bits) for the
    rest."""
    s = SLICES[P]
    lo = CRT_MIN[P]
    shapes = [(lo, lo, lo), (lo - 1, 300, 300), (300, lo - 1, 200), (200, 200, lo - 1), (250, 140, 333),
              (16, 16, 16), (lo + 5, lo + 70, lo + 1)]
    probs = problem_set(P, shapes, 7000 + P)
    dprobs = to_dev(probs)
    note("batched auto", P)
    plan = gpu_lib.BatchPlan(P, dprobs, form="auto", slices=s)
    res = [min(p["m"], p["n"], p["k"]) >= lo for p in probs]
    assert plan.info()["residue_problems"] == sum(res)
    plan.run()
    for q, (p, d, r) in enumerate(zip(probs, dprobs, res)):
        assert np.array_equal(host(d["C"]), want_of(P, s, p, r)), (q, r)
    plan.close()
    # without s, AUTO means plain
    plan = gpu_lib.BatchPlan(P, to_dev(probs), form="auto", slices=0)
    assert plan.info()["residue_problems"] == 0
    plan.close()


@pytest.mark.parametrize("P,s", [(2, 16), (4, 31)])
def test_batched_residue_chunks(gpu_lib, P, s):
    """More residue workspace than one chunk holds (a 1 GiB bound): several
    chunks run one after another over one workspace; every problem's bits
    equal a single residue-form call, and sampled blocks the oracle (QD at
    two levels too)."""
    shapes = [(1536, 1536, 1536)] * 5 + [(1000, 1200, 1400)]
    probs = problem_set(P, shapes, 4242 + s)
    dprobs = to_dev(probs)
    note("batched residue chunks", P, s)
    plan = gpu_lib.BatchPlan(P, dprobs, form="crt", slices=s, chunk_bytes=1 << 30)
    info = plan.info()
    assert info["chunks"] >= 2 and info["residue_problems"] == len(probs)
    refs = [single_call(gpu_lib, P, s, d) for d in dprobs]
    plan.run()
    torch.cuda.synchronize()
    for q, (d, r) in enumerate(zip(dprobs, refs)):
        assert torch.equal(d["C"], r), q
    plan.close()
    for q in (0, 5):
        p = probs[q]
        r0, c0 = p["m"] - 70, p["n"] - 50
        want = oracle.gemm_crt(P, s, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"],
                               p["B"], p["beta"], p["C"], rows=(r0, p["m"]), cols=(c0, p["n"]))
        got = host(refs[q])
        assert np.array_equal(got[:, c0:, r0:], want[:, c0:, r0:]), q


@pytest.mark.parametrize("P,s", [(2, 16), (4, 20), (4, 31)])
def test_grouped_residue_calls(gpu_lib, P, s):
    """Grouped calls with the residue form: the cached plan is replayed by a
    second call with the same array (beta != 0: each call adds onto the
    last), and the form is part of the key (a plain call on the same array
    gets a plan of its own)."""
    shapes = [(100, 90, 80), (17, 200, 33), (130, 5, 129), (64, 64, 64)]
    probs = problem_set(P, shapes, 3100 + P + s)
    for q, p in enumerate(probs):
        p["beta"] = synth.mp_uniform(np.random.Generator(np.random.PCG64(55 + q)), P, (1,))[:, 0]
    dprobs = to_dev(probs)
    arr = gpu_lib.problem_array(P, dprobs)
    note("grouped residue", P)
    gpu_lib.grouped(P, dprobs, arr=arr, form="crt", slices=s)
    gpu_lib.grouped(P, dprobs, arr=arr, form="crt", slices=s)
    gpu_lib.grouped(P, dprobs, arr=arr)                           # plain, same array
    torch.cuda.synchronize()
    for q, p in enumerate(probs):
        w = p["C"]
        for _ in range(2):
            w = oracle.gemm_crt(P, s, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"],
                                p["B"], p["beta"], w)
        w = oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"], p["B"],
                        p["beta"], w)
        assert np.array_equal(host(dprobs[q]["C"]), w), q


def test_batched_auto_qd_two_levels(gpu_lib):
    """QD's default s = 31 takes two levels (hh, ll and ss products of one
    modulus set): AUTO runs problems of at least 64 on every side in the
    residue form, bit for bit as the oracle's, and the rest in the plain
    form (canonical bits); the plan reports 3 N products."""
    P, s = 4, 31
    shapes = [(100, 90, 80), (70, 130, 65), (63, 200, 200), (64, 64, 64), (300, 64, 1000)]
    probs = problem_set(P, shapes, 8100)
    dprobs = to_dev(probs)
    note("batched auto qd s=31")
    plan = gpu_lib.BatchPlan(P, dprobs, form="auto", slices=s)
    res = [min(p["m"], p["n"], p["k"]) >= 64 for p in probs]
    info = plan.info()
    assert info["residue_problems"] == sum(res)
    kmax = max(p["k"] for p, r in zip(probs, res) if r)
    assert info["moduli"] == gpu_lib.crt_moduli(P, kmax, s) and info["moduli"] % 3 == 0
    plan.run()
    for q, (p, d, r) in enumerate(zip(probs, dprobs, res)):
        assert np.array_equal(host(d["C"]), want_of(P, s, p, r)), (q, r)
    plan.close()


def test_batched_two_levels_of_33_moduli(gpu_lib):
    """QD with s = 32 and one problem of k = 65536: the plan takes two levels
    of 33 moduli (a second block of 32 per set in every stage) for all its
    residue problems; each bit for bit as the oracle's residue form."""
    P, s = 4, 32
    shapes = [(20, 17, 65536), (70, 65, 100), (33, 129, 70)]
    probs = problem_set(P, shapes, 8800)
    dprobs = to_dev(probs)
    note("batched two levels of 33 moduli")
    plan = gpu_lib.BatchPlan(P, dprobs, form="crt", slices=s)
    assert plan.info()["moduli"] == gpu_lib.crt_moduli(P, 65536, s) == 99
    plan.run()
    for q, (p, d) in enumerate(zip(probs, dprobs)):
        assert np.array_equal(host(d["C"]), want_of(P, s, p, True)), q
    plan.close()

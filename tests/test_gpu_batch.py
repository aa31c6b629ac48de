"""Batched persistent form: every problem bit-identical to the oracle and to
one plain call per problem; replays of the captured hipGraph are identical
to a direct launch, also with other work between replays."""
import numpy as np
import pytest
import torch

import oracle
from tests import synth
from tests.gpu_util import dev, host, note

pytestmark = pytest.mark.gpu


def problems(P, count, lo, hi, fam=5, seed_slot="shapes", shapes=None):
    if shapes is None:
        rng = synth.rng_for(fam, seed_slot)
        shapes = rng.integers(lo, hi + 1, size=(count, 3))
    out = []
    for q, (m, n, k) in enumerate(shapes):
        m, n, k = int(m), int(n), int(k)
        rq = np.random.Generator(np.random.PCG64(synth.seed_for(fam, 0) * 7 + q))
        A = synth.mp_uniform(rq, P, (k, m))
        B = synth.mp_uniform(rq, P, (n, k))
        C = synth.mp_uniform(rq, P, (n, m))
        tr = ("N", "N") if q % 3 else ("T", "N")
        if tr[0] == "T":
            A = synth.mp_uniform(rq, P, (m, k))
        alpha = synth.mp_uniform(rq, P, (1,))[:, 0] if q % 2 else synth.mp_one(P)
        beta = synth.mp_uniform(rq, P, (1,))[:, 0] if q % 4 == 1 else np.zeros(P)
        out.append(dict(transa=tr[0], transb=tr[1], m=m, n=n, k=k, A=A, B=B, C=C, alpha=alpha,
                        beta=beta))
    return out


def to_dev(probs):
    d = []
    for p in probs:
        q = dict(p)
        q["A"], q["B"], q["C"] = dev(p["A"]), dev(p["B"]), dev(p["C"])
        d.append(q)
    return d


@pytest.mark.parametrize("P", [2, 3])
def test_batch_matches_oracle_and_single_calls(gpu_lib, P):
    probs = problems(P, 48, 16, 160)
    dprobs = to_dev(probs)
    note("batch build", P, len(probs))
    plan = gpu_lib.BatchPlan(P, dprobs)
    info = plan.info()
    assert info["tiles"] > 0
    note("batch run", P, info)
    plan.run()
    torch.cuda.synchronize()
    for q, (p, d) in enumerate(zip(probs, dprobs)):
        got = host(d["C"])
        want = oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"],
                           p["B"], p["beta"], p["C"])
        assert np.array_equal(got, want), (P, q, p["m"], p["n"], p["k"])
    plan.close()


# Shapes that end inside, at and just past the quadrant and tile edges of
# every batched tile (tiles 16..64 rows by 16..64 columns).
EDGE_SHAPES = [(8, 8, 5), (9, 17, 16), (16, 16, 17), (17, 33, 3), (24, 8, 33), (32, 40, 1),
               (33, 64, 20), (40, 7, 31), (64, 65, 18), (65, 31, 47), (96, 100, 12), (1, 1, 1)]


@pytest.mark.parametrize("P", [2, 3, 4])
def test_every_batched_tile_on_edge_shapes(gpu_lib, P):
    """Each batched tile configuration (its waves own tile quadrants and skip
    those wholly outside a problem) is bit-identical to the oracle on shapes
    ending inside, at and past the quadrant edges."""
    probs = problems(P, 0, 0, 0, shapes=EDGE_SHAPES)
    wants = [oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"],
                         p["B"], p["beta"], p["C"]) for p in probs]
    for cfg in range(gpu_lib.num_configs(P, "batched")):
        dprobs = to_dev(probs)
        note("batch tile", P, cfg)
        plan = gpu_lib.BatchPlan(P, dprobs, tile=cfg)
        assert plan.info()["tile_cfg"] == cfg
        plan.run()
        for q, (d, w) in enumerate(zip(dprobs, wants)):
            assert np.array_equal(host(d["C"]), w), (P, cfg, q, EDGE_SHAPES[q])
        plan.close()


@pytest.mark.parametrize("P", [2, 3])
def test_graph_replays_equal_direct_launch(gpu_lib, P):
    """The batched shape mix (512 problems, m, n, k uniform in 16..512): each graph replay,
    with eager work and synchronisation between replays, gives the same bits
    as a direct launch and as one plain call per problem."""
    probs = problems(P, 512, 16, 512)
    dprobs = to_dev(probs)
    # reference: one plain call per problem
    refs = []
    note("batch per-problem reference", P)
    for d in dprobs:
        C = d["C"].clone()
        gpu_lib.gemm(P, d["transa"], d["transb"], d["m"], d["n"], d["k"], d["alpha"], d["A"], d["B"],
                     d["beta"], C)
        refs.append(C)
    torch.cuda.synchronize()
    C0 = [d["C"].clone() for d in dprobs]
    plan = gpu_lib.BatchPlan(P, dprobs)
    for rep in range(3):
        for d, c0 in zip(dprobs, C0):
            d["C"].copy_(c0)
        note("graph replay", P, rep)
        if rep == 1:
            plan.launch()
        else:
            plan.run()
        x = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        torch.cuda.synchronize()
        del x
        for q, (d, r) in enumerate(zip(dprobs, refs)):
            assert torch.equal(d["C"], r), (rep, q)
    plan.close()
    # a few problems fully against the oracle
    for q in (0, 1, 2, 255, 511):
        p = probs[q]
        want = oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"],
                           p["B"], p["beta"], p["C"])
        assert np.array_equal(host(refs[q]), want), q


def test_batch_empty_and_degenerate(gpu_lib):
    P = 2
    probs = problems(P, 6, 1, 40)
    probs[1]["m"] = 0
    probs[1]["A"] = np.zeros((P, probs[1]["k"], 1))
    probs[1]["C"] = np.zeros((P, probs[1]["n"], 1))
    probs[2]["k"] = 0
    probs[2]["beta"] = np.zeros(P)
    probs[2]["A"] = np.zeros((P, 1, probs[2]["m"]))
    probs[2]["B"] = np.zeros((P, probs[2]["n"], 1))
    probs[3]["alpha"] = np.zeros(P)
    probs[3]["beta"] = synth.mp_one(P)
    dprobs = to_dev(probs)
    note("batch degenerate")
    plan = gpu_lib.BatchPlan(P, dprobs)
    plan.run()
    for q, (p, d) in enumerate(zip(probs, dprobs)):
        want = oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"],
                           p["B"], p["beta"], p["C"])
        assert np.array_equal(host(d["C"]), want), q
    plan.close()
    empty = gpu_lib.BatchPlan(P, [])
    empty.run()
    empty.close()


def test_runs_back_to_back_on_one_stream(gpu_lib):
    """A plan's runs share its tile counter, so they must be stream-ordered:
    replay, direct launch and replay queued back to back on one stream with
    no synchronisation between them.  With beta != 0 each run adds onto the
    last one's C, so a tile skipped or repeated by one run shows in the end
    result: three runs equal three plain products in a row."""
    P = 2
    probs = problems(P, 40, 16, 200, fam=6)
    for p in probs:
        p["beta"] = synth.mp_uniform(np.random.Generator(np.random.PCG64(p["m"] * 1000 + p["k"])), P, (1,))[:, 0]
    dprobs = to_dev(probs)
    plan = gpu_lib.BatchPlan(P, dprobs)
    note("batch back to back", P, plan.info())
    stream = torch.cuda.current_stream()
    plan.run(stream)
    plan.launch(stream)
    plan.run(stream)
    torch.cuda.synchronize()
    for q, (p, d) in enumerate(zip(probs, dprobs)):
        want = p["C"]
        for _ in range(3):
            want = oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"], p["B"],
                               p["beta"], want)
        assert np.array_equal(host(d["C"]), want), (q, p["m"], p["n"], p["k"])


@pytest.mark.parametrize("P", [2, 3, 4])
def test_grouped_calls(gpu_lib, P):
    """mpgemm_{dd,td,qd}_grouped: every problem bit for bit as the oracle;
    a second call with the same problem array replays the cached plan (beta
    != 0, so each call adds onto the last: a stale or skipped tile shows);
    another array (one alpha changed) gets a plan of its own."""
    probs = problems(P, 24, 16, 140, fam=7)
    for q, p in enumerate(probs):
        if q % 2 == 0:
            p["beta"] = synth.mp_uniform(np.random.Generator(np.random.PCG64(77 + q)), P, (1,))[:, 0]
    dprobs = to_dev(probs)
    arr = gpu_lib.problem_array(P, dprobs)
    note("grouped", P, len(probs))
    gpu_lib.grouped(P, dprobs, arr=arr)
    gpu_lib.grouped(P, dprobs, arr=arr)            # cached plan
    torch.cuda.synchronize()
    want = []
    for p in probs:
        w = p["C"]
        for _ in range(2):
            w = oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], p["alpha"], p["A"], p["B"],
                            p["beta"], w)
        want.append(w)
    for q, d in enumerate(dprobs):
        assert np.array_equal(host(d["C"]), want[q]), (P, q)
    # a changed alpha is another problem array: a new plan, not the cached one
    dprobs[3]["alpha"] = 2.0 * np.asarray(dprobs[3]["alpha"])
    dprobs[3]["beta"] = np.zeros(P)
    gpu_lib.grouped(P, dprobs)
    torch.cuda.synchronize()
    p = probs[3]
    w3 = oracle.gemm(P, p["transa"], p["transb"], p["m"], p["n"], p["k"], dprobs[3]["alpha"], p["A"], p["B"],
                     np.zeros(P), want[3])
    assert np.array_equal(host(dprobs[3]["C"]), w3)

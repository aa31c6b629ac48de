"""Benchmark: square DD / TD / QD GEMM C = alpha A B + beta C on one MI355X.

One step = the whole hot path over one batch of synthetic input: for each
precision (DD, TD, QD) the plain FP64-VALU EFT GEMM and the split INT8-MFMA
GEMM (scale scan, digit slicing, anti-diagonal MFMA sums, recombination and
epilogue) on the same m = n = k = 4096 operands with random alpha, beta and C.
`value` is the whole step's throughput in 2mnk/s (six GEMMs per step).

Prints ONE JSON line (rank 0).  Extra fields: per-GEMM breakdown with the
measured error against the exact product on sampled entries (split vs
plain "at the same error"), the roofline of the dominant kernel, and the
CPU oracle timed on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DD/TD/QD GEMM 2mnk/s, % FP64 peak; Ozaki-MFMA vs plain EFT at same error"
FP64_PEAK = 78.6e12            # MI355X FP64 vector, FLOP/s (FMA = 2)
FP64_ISSUE = 256 * 64 * 2.4e9  # FP64 lane-instructions per second (256 CU x 64 lanes x 2.4 GHz)
INT8_PEAK = 5.0e15             # MI355X dense INT8 MFMA, OP/s
# FP64 operations per multiply-add of the paper's algorithms (MUL + ADD):
#   DD: Algorithm 2 (9 instr, 10 flops) + Algorithm 1 (11)          -> 20 instr, 21 flops
#   TD: Algorithm 4 (47 instr, 53 flops) + TDaddq = Algorithm 5 (85) -> 132 instr, 138 flops
#   QD: Algorithm 6 (121 instr, 127 flops) + Algorithm 5 (85)        -> 206 instr, 212 flops
INSTR_PER_MAC = {2: 20, 3: 132, 4: 206}
FLOPS_PER_MAC = {2: 21, 3: 138, 4: 212}
NAME = {2: "DD", 3: "TD", 4: "QD"}
PAPER_CONTEXT = {
    "note": "paper's CPU seconds for C := AB, n = 4096 (AVX2 + OpenMP); other hardware, context only",
    "DD": {"seconds": 10.72, "2mnk/s": 1.282e10, "hw": "EPYC 7402P, 24 threads, block+AVX2"},
    "TD": {"seconds": 94.76, "2mnk/s": 1.450e9, "hw": "EPYC 7402P, 24 threads, block+AVX2"},
    "QD": {"seconds": 153.63, "2mnk/s": 8.95e8, "hw": "Core i9-10900X, 10 threads, Strassen+AVX2"},
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_plain_qd_4096.txt")
ROOFLINE_SOURCES = ["paper_2101_06584_amd/csrc/plain_gemm.hip", "paper_2101_06584_amd/csrc/mp_arith.hpp",
                    "paper_2101_06584_amd/csrc/tile_order.hpp"]


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_hash") != source_hash(ROOFLINE_SOURCES):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", default="2,3,4")
    ap.add_argument("--forms", default="plain,split")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled error check")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds for the CPU baseline")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain device copy of 1 GiB first (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2101_06584_amd as mp
    from tests import synth

    mp.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    n = args.n
    precs = [int(p) for p in args.prec.split(",")]
    forms = args.forms.split(",")

    if args.copy_calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- inputs (config: square n, random alpha/beta, C like A and B) ----
    host = {}
    devd = {}
    for P in precs:
        A = synth.mp_matrix(2, "A", P, n, n)
        B = synth.mp_matrix(2, "B", P, n, n)
        C = synth.mp_matrix(2, "C", P, n, n)
        alpha = synth.mp_scalar(2, "alpha", P)
        beta = synth.mp_scalar(2, "beta", P)
        host[P] = (A, B, C, alpha, beta)
        d = {"A": torch.from_numpy(A).to(dev), "B": torch.from_numpy(B).to(dev),
             "C0": torch.from_numpy(C).to(dev), "alpha": alpha, "beta": beta}
        for f in forms:
            d["C_" + f] = d["C0"].clone()
        if "split" in forms:
            d["s"] = mp.DEFAULT_SLICES[P]
            d["ws"] = mp.alloc_workspace(P, n, n, n, d["s"], device=dev)
        devd[P] = d
    torch.cuda.synchronize()

    def run(P, f):
        d = devd[P]
        if f == "plain":
            mp.gemm(P, "N", "N", n, n, n, d["alpha"], d["A"], d["B"], d["beta"], d["C_plain"],
                    form="plain", stream=stream)
        else:
            mp.gemm(P, "N", "N", n, n, n, d["alpha"], d["A"], d["B"], d["beta"], d["C_split"],
                    form="split", slices=d["s"], workspace=d["ws"], stream=stream)

    # ---- accuracy on sampled entries (outside the timed region) ----
    errors = {}
    if not args.no_check:
        from tests.exact import GemmChecker, sample_entries
        for P in precs:
            A, B, C, alpha, beta = host[P]
            chk = GemmChecker(P, "N", "N", n, n, n, alpha, A, B, beta, C)
            ents = sample_entries(synth.rng_for(2, "samples"), n, n, 64)
            for f in forms:
                devd[P]["C_" + f].copy_(devd[P]["C0"])
                run(P, f)
                got = devd[P]["C_" + f].cpu().numpy()
                r = chk.ratios(got, ents)
                errors[(P, f)] = float(r.max())
                devd[P]["C_" + f].copy_(devd[P]["C0"])
        torch.cuda.synchronize()

    # ---- warmup + timed steps; per-GEMM events on the launch stream ----
    order = [(P, f) for P in precs for f in forms]
    for _ in range(args.warmup):
        for P, f in order:
            run(P, f)
    torch.cuda.synchronize()
    ev = {key: [] for key in order}
    t0 = time.perf_counter()
    start_all = torch.cuda.Event(enable_timing=True)
    end_all = torch.cuda.Event(enable_timing=True)
    start_all.record(stream)
    for _ in range(args.steps):
        for key in order:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run(*key)
            e1.record(stream)
            ev[key].append((e0, e1))
    end_all.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start_all.elapsed_time(end_all)
    ms_per_step = total_ms / args.steps
    work_per_step = 2.0 * n * n * n * len(order)
    value = work_per_step / (ms_per_step * 1e-3)

    breakdown = {}
    for key in order:
        P, f = key
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev[key]]))
        rate = 2.0 * n ** 3 / (ms * 1e-3)
        item = {"ms": round(ms, 3), "2mnk/s": rate}
        if f == "plain":
            item["fp64_peak_frac"] = n ** 3 * FLOPS_PER_MAC[P] / (ms * 1e-3) / FP64_PEAK
            item["fp64_issue_frac"] = n ** 3 * INSTR_PER_MAC[P] / (ms * 1e-3) / FP64_ISSUE
        else:
            s = devd[P]["s"]
            item["slices"] = s
            item["int8_ops_frac"] = s * (s + 1) / 2 * 2.0 * n ** 3 / (ms * 1e-3) / INT8_PEAK
        if (P, f) in errors:
            item["max_err_ratio"] = errors[(P, f)]
        breakdown[f"{NAME[P]}_{f}"] = item

    # ---- roofline of the dominant kernel: the plain GEMM of the widest
    # precision run (one kernel launch per call) ----
    dom_P = max(precs) if "plain" in forms else None
    roofline = None
    if dom_P is not None:
        ms = breakdown[f"{NAME[dom_P]}_plain"]["ms"]
        flops = n ** 3 * FLOPS_PER_MAC[dom_P]
        achieved = flops / (ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": f"plain_gemm_kernel<{dom_P},...> ({NAME[dom_P]}, n={n})",
                    "achieved": round(achieved, 3), "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
                    "frac": round(achieved * 1e12 / FP64_PEAK, 4),
                    "issue_frac": round(n ** 3 * INSTR_PER_MAC[dom_P] / (ms * 1e-3) / FP64_ISSUE, 4),
                    "flops_per_launch": flops,
                    "traffic": read_traffic() if (dom_P == 4 and n == 4096) else None}

    out = {
        "metric": METRIC, "value": value, "unit": "2mnk/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+i8", "data": "synthetic",
        "config": {"workload": f"square DD/TD/QD GEMM C = alpha*A*B + beta*C, m=n=k={n}, "
                               "random alpha/beta/C; plain EFT and split INT8-MFMA forms per step",
                   "m": n, "n": n, "k": n, "precisions": [NAME[P] for P in precs], "forms": forms,
                   "gemms_per_step": len(order), "parallelism": "single GPU"},
        "breakdown": breakdown,
        "roofline": roofline,
        "wall_s_timed": round(wall, 3),
        "paper_context": PAPER_CONTEXT,
    }

    # ---- CPU oracle on this host's cores (bounded sample) ----
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(host, precs, forms, n, devd, args.cpu_budget)

    print(json.dumps(out), flush=True)


def cpu_baseline(host, precs, forms, n, devd, budget):
    """The oracle, as it stands, on a block of rows of each of the step's
    GEMMs; the step's 2mnk/s is extrapolated from the per-GEMM sampled rates."""
    import oracle
    threads = oracle.num_threads()
    per = budget / max(1, len(precs) * len(forms))
    est_total = 0.0
    parts = []
    for P in precs:
        A, B, C, alpha, beta = host[P]
        for f in forms:
            def once(rows, cols):
                t = time.perf_counter()
                if f == "plain":
                    oracle.gemm(P, "N", "N", n, n, n, alpha, A, B, beta, C, rows=(0, rows),
                                cols=(0, cols))
                else:
                    oracle.gemm_split(P, devd[P]["s"], "N", "N", n, n, n, alpha, A, B, beta, C,
                                      rows=(0, rows), cols=(0, cols))
                return time.perf_counter() - t
            rows, cols = 1, 64
            t = once(rows, cols)
            # grow the block until it takes about its share of the budget
            while t < per / 4 and rows * cols < n * n:
                if cols < n:
                    cols = min(n, cols * 4)
                else:
                    rows = min(n, rows * 4)
                t = once(rows, cols)
            rate = 2.0 * rows * cols * n / t
            est_total += 2.0 * n ** 3 / rate
            parts.append(f"{NAME[P]}-{f}: {rows}x{cols} block ({rate:.3g} 2mnk/s)")
    value = len(precs) * len(forms) * 2.0 * n ** 3 / est_total
    return {"value": value, "unit": "2mnk/s", "cores": threads, "kind": "oracle",
            "sample": "per GEMM of the step, a block of rows x columns of C (all k) timed and the "
                      "full n^3 extrapolated: " + "; ".join(parts)}


if __name__ == "__main__":
    main()

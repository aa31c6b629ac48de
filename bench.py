"""Benchmark: DD / TD / QD GEMM C = alpha A B + beta C on one MI355X.

One step = the whole hot path over one batch of synthetic input:
  * for each precision (DD, TD, QD), m = n = k = 4096 with random alpha, beta
    and C: the plain FP64-VALU EFT GEMM and the split INT8-MFMA GEMM in both
    its variants: triangular (scale scan, digit slicing, anti-diagonal MFMA
    sums, recombination, epilogue) and residue (the same digits, one INT8
    product per coprime modulus, exact Chinese-remainder reconstruction);
  * the batched form: 512 DD and 512 TD GEMMs with m, n, k uniform in
    16..512, each set once in the plain form (one persistent launch) and once
    in the residue form (the four residue stages, one launch each over the
    set), each one replay of its captured hipGraph;
with tile configurations from the autotuner's table.  `value` is the step's
total 2mnk divided by its time.

Prints ONE JSON line.  Extra fields: per-part breakdown with the measured
error against the exact product on sampled entries (split vs plain "at the
same error"), the batched form against one launch per problem, the
roofline of the dominant kernel, and the CPU oracle on this host's cores.

Other workloads (separate JSON lines): --workload qd2048-spread (QD n = 2048,
entries u 2^e with e in -30..30 per entry, all forms, slice count from the
accuracy rule) and --workload dd8192 (DD n = 8192, all forms).
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
HBM_PEAK = 8.0e12              # MI355X HBM3E, bytes/s
# FP64 arithmetic per multiply-add (MUL_P + ADD_P, common Renorm/VSEB branch)
# as the plain kernels execute it, counted by the hardware
# (SQ_INSTS_VALU_{ADD,MUL,FMA}_F64 x 64 / n^3 at n = 4096):
#   DD: Algorithms 2 + 1:                    16 add, 3 mul, 1 FMA ->  20 ops,  21 flops
#   TD: Algorithm 4 + TDaddq (Algorithm 5 on zero fourth components, whose
#       all-constant operations fold and whose TwoSum(+0, carry) error, always
#       +0, is not formed):                104 add, 3 mul, 6 FMA -> 113 ops, 119 flops
#   QD: Algorithms 6 + 5:                   184 add, 10 mul, 6 FMA -> 200 ops, 206 flops
# The kernels issue a few more vector instructions per multiply-add than that
# (compares and selects of the Renorm/VSEB test, LDS address arithmetic):
# 21.2 (DD), 122.0 (TD), 210.6 (QD) in all; VALU_PER_MAC gives the issue-slot use.
INSTR_PER_MAC = {2: 20, 3: 113, 4: 200}
FLOPS_PER_MAC = {2: 21, 3: 119, 4: 206}
VALU_PER_MAC = {2: 21.2, 3: 122.0, 4: 210.6}
NAME = {2: "DD", 3: "TD", 4: "QD"}
PAPER_CONTEXT = {
    "note": "paper's CPU seconds for C := AB, n = 4096 (AVX2 + OpenMP); other hardware, context only",
    "DD": {"seconds": 10.72, "2mnk/s": 1.282e10, "hw": "EPYC 7402P, 24 threads, block+AVX2"},
    "TD": {"seconds": 94.76, "2mnk/s": 1.450e9, "hw": "EPYC 7402P, 24 threads, block+AVX2"},
    "QD": {"seconds": 153.63, "2mnk/s": 8.95e8, "hw": "Core i9-10900X, 10 threads, Strassen+AVX2"},
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_plain_qd_4096.txt")
SAME_ERROR_TARGET = 1e-6       # slice rule target for "split at the same error as plain"
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
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--prec", default="2,3,4")
    ap.add_argument("--forms", default="plain,split,crt")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the sampled error check")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds for the CPU baseline")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain device copy of 1 GiB first (counter calibration)")
    ap.add_argument("--no-batched", action="store_true", help="leave the batched sets out")
    ap.add_argument("--workload", default="", choices=["", "qd2048-spread", "dd8192"],
                    help="one of the other workloads instead of the step")
    ap.add_argument("--vec", action="store_true",
                    help="element-wise DD/TD/QD add and mul (Sec. 2.5) against the HBM roofline")
    ap.add_argument("--vec-n", type=int, default=1 << 26, help="vector length for --vec")
    ap.add_argument("--td-variants", action="store_true",
                    help="accuracy and speed of the TD operation variants (Sec. 2.3)")
    ap.add_argument("--blas", action="store_true",
                    help="BLAS-1/2 (axpy, dot, gemv) in DD/TD/QD against the HBM roofline")
    ap.add_argument("--strassen", action="store_true",
                    help="Strassen's method (Sec. 3, Fig. 5) against the plain form, n = 4096")
    ap.add_argument("--crt", action="store_true",
                    help="residue (CRT) split form against the triangular split form, DD, TD and QD")
    return ap.parse_args()


def note(*a):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
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
    if args.copy_calib:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        src.fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload:
        return other_workload(args, mp, synth, dev, stream)
    if args.vec:
        return vec_bench(args, mp, dev, stream)
    if args.td_variants:
        return td_variants_bench(args, mp, synth, dev, stream)
    if args.strassen:
        return strassen_bench(args, mp, synth, dev, stream)
    if args.blas:
        return blas_bench(args, mp, dev, stream)
    if args.crt:
        return crt_bench(args, mp, synth, dev, stream)
    n = args.n
    precs = [int(p) for p in args.prec.split(",")]
    forms = args.forms.split(",")

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
        d["s"] = mp.DEFAULT_SLICES[P]
        if "split" in forms:
            d["ws"] = mp.alloc_workspace(P, n, n, n, d["s"], device=dev)
        if "crt" in forms:
            d["ws_crt"] = mp.alloc_workspace(P, n, n, n, d["s"], device=dev, form="crt")
        devd[P] = d
        note("inputs ready", NAME[P])
    torch.cuda.synchronize()

    # batched sets (512 problems with m, n, k uniform in 16..512): DD and TD
    batched = {}
    if not args.no_batched:
        for P in (2, 3):
            hp = synth.batch_problems(5, P, 512, 16, 512)
            dp = []
            for pr in hp:
                q = dict(pr)
                q["A"] = torch.from_numpy(pr["A"]).to(dev)
                q["B"] = torch.from_numpy(pr["B"]).to(dev)
                q["C"] = torch.from_numpy(pr["C"]).to(dev)
                dp.append(q)
            plan = mp.BatchPlan(P, dp, stream=stream)
            work = sum(2.0 * q["m"] * q["n"] * q["k"] for q in dp)
            # the residue form of the same set: the same operands, C of its own
            dc = [dict(q, C=q["C"].clone()) for q in dp]
            plan_crt = mp.BatchPlan(P, dc, stream=stream, form="crt", slices=mp.DEFAULT_SLICES[P])
            batched[P] = {"plan": plan, "probs": dp, "work": work, "host": hp, "crt_plan": plan_crt,
                          "crt_probs": dc, "s": mp.DEFAULT_SLICES[P]}
            note("batched plans ready", NAME[P], plan_crt.info())
        torch.cuda.synchronize()

    def run(P, f):
        if f == "batched":
            batched[P]["plan"].run(stream=stream)
            return
        if f == "batched_crt":
            batched[P]["crt_plan"].run(stream=stream)
            return
        d = devd[P]
        if f == "plain":
            mp.gemm(P, "N", "N", n, n, n, d["alpha"], d["A"], d["B"], d["beta"], d["C_plain"],
                    form="plain", stream=stream)
        elif f == "crt":
            mp.gemm(P, "N", "N", n, n, n, d["alpha"], d["A"], d["B"], d["beta"], d["C_crt"],
                    form="crt", slices=d["s"], workspace=d["ws_crt"], stream=stream)
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
            ents = sample_entries(synth.rng_for(2, "samples"), n, n, 1024)
            for f in forms:
                devd[P]["C_" + f].copy_(devd[P]["C0"])
                run(P, f)
                got = devd[P]["C_" + f].cpu().numpy()
                r = chk.ratios(got, ents)
                errors[(P, f)] = float(r.max())
                errors[(P, f, "median")] = float(np.median(r))
                devd[P]["C_" + f].copy_(devd[P]["C0"])
                note("checked", NAME[P], f, "max err ratio", errors[(P, f)])
        # batched residue form: 128 sampled entries of each of the first 8 problems
        for P, b in sorted(batched.items()):
            b["crt_plan"].run(stream=stream)
            torch.cuda.synchronize()
            rs = []
            for q in range(8):
                h, d = b["host"][q], b["crt_probs"][q]
                chk = GemmChecker(P, "N", "N", h["m"], h["n"], h["k"], h["alpha"], h["A"], h["B"], h["beta"], h["C"])
                rs.append(chk.ratios(d["C"].cpu().numpy(), sample_entries(synth.rng_for(5, q), h["m"], h["n"], 128)))
            r = np.concatenate(rs)
            errors[(P, "batched_crt")] = float(r.max())
            errors[(P, "batched_crt", "median")] = float(np.median(r))
            errors[(P, "batched_crt", "n")] = int(r.size)
            note("checked", NAME[P], "batched_crt", "max err ratio", errors[(P, "batched_crt")])

    # ---- warmup + timed steps; per-part events on the launch stream ----
    order = [(P, f) for P in precs for f in forms] + [(P, f) for P in sorted(batched)
                                                      for f in ("batched", "batched_crt")]
    part_work = {key: (batched[key[0]]["work"] if key[1].startswith("batched") else 2.0 * n ** 3)
                 for key in order}
    for _ in range(args.warmup):
        for P, f in order:
            run(P, f)
    torch.cuda.synchronize()
    note("warmup done")
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
    note("timed steps done", round(wall, 2), "s")
    total_ms = start_all.elapsed_time(end_all)
    ms_per_step = total_ms / args.steps
    work_per_step = sum(part_work.values())
    value = work_per_step / (ms_per_step * 1e-3)

    breakdown = {}
    for key in order:
        P, f = key
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev[key]]))
        rate = part_work[key] / (ms * 1e-3)
        item = {"ms": round(ms, 3), "2mnk/s": rate}
        if f == "batched":
            info = batched[P]["plan"].info()
            item.update(problems=len(batched[P]["probs"]), tiles=info["tiles"],
                        tile_cfg=info["tile_cfg"], grid=info["grid"])
            item.update(separate_launches(mp, P, batched[P], stream))
        elif f == "batched_crt":
            info = batched[P]["crt_plan"].info()
            item.update(problems=len(batched[P]["crt_probs"]), slices=batched[P]["s"],
                        residue_problems=info["residue_problems"], int8_products=info["moduli"],
                        chunks=info["chunks"], workspace_bytes=info["residue_workspace"])
            # INT8 operations of the unpadded products over the time
            item["int8_ops_frac"] = info["moduli"] * part_work[key] / (ms * 1e-3) / INT8_PEAK
        elif f == "plain":
            item["fp64_peak_frac"] = n ** 3 * FLOPS_PER_MAC[P] / (ms * 1e-3) / FP64_PEAK
            item["fp64_issue_frac"] = n ** 3 * INSTR_PER_MAC[P] / (ms * 1e-3) / FP64_ISSUE
            item["valu_issue_frac"] = n ** 3 * VALU_PER_MAC[P] / (ms * 1e-3) / FP64_ISSUE
        elif f == "crt":
            s = devd[P]["s"]
            item["slices"] = s
            item["int8_products"] = mp.crt_moduli(P, n, s)
            item["int8_ops_frac"] = item["int8_products"] * 2.0 * n ** 3 / (ms * 1e-3) / INT8_PEAK
        else:
            s = devd[P]["s"]
            item["slices"] = s
            item["int8_products"] = s * (s + 1) // 2
            item["int8_ops_frac"] = s * (s + 1) / 2 * 2.0 * n ** 3 / (ms * 1e-3) / INT8_PEAK
        if (P, f) in errors:
            item["max_err_ratio"] = errors[(P, f)]
            item["median_err_ratio"] = errors[(P, f, "median")]
            item["err_samples"] = errors.get((P, f, "n"), 1024)
        breakdown[f"{NAME[P]}_{f}"] = item

    # ---- roofline of the dominant kernel: the plain GEMM of the widest
    # precision run (one kernel launch per call) ----
    dom_P = max(precs) if "plain" in forms else None
    roofline = None
    if dom_P is not None:
        ms = breakdown[f"{NAME[dom_P]}_plain"]["ms"]
        flops = n ** 3 * FLOPS_PER_MAC[dom_P]
        achieved = flops / (ms * 1e-3) / 1e12
        # The EFT chains are almost all separate adds and multiplies (QD: 6 of
        # 200 operations per multiply-add are FMAs), so the bound is the FP64
        # operation issue rate, 256 CU x 64 lanes x 2.4 GHz = 39.3 T op/s; the
        # FMA-counted 78.6 TFLOP/s figure is reported beside it, and so is the
        # fraction of vector issue slots used by all the kernel's instructions.
        ops = n ** 3 * INSTR_PER_MAC[dom_P]
        achieved_ops = ops / (ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": f"plain_gemm_kernel<{dom_P},...> ({NAME[dom_P]}, n={n})",
                    "achieved": round(achieved_ops, 3), "peak": round(FP64_ISSUE / 1e12, 2),
                    "unit": "T FP64 op/s", "frac": round(achieved_ops * 1e12 / FP64_ISSUE, 4),
                    "ops_per_launch": ops,
                    "flops_per_launch": flops, "achieved_tflops": round(achieved, 3),
                    "fp64_tflops_peak": FP64_PEAK / 1e12,
                    "flops_frac": round(achieved * 1e12 / FP64_PEAK, 4),
                    "valu_issue_frac": round(n ** 3 * VALU_PER_MAC[dom_P] / (ms * 1e-3) / FP64_ISSUE, 4),
                    "traffic": read_traffic() if (dom_P == 4 and n == 4096) else None}

    for P in batched:
        batched[P]["plan"].close()
        batched[P]["crt_plan"].close()

    # ---- measured peaks of this GPU (after the timed region), and the parts'
    # fractions of them beside the fractions of the published figures ----
    peaks = measured_peaks(mp, stream)
    note("measured peaks", peaks)
    for key, item in breakdown.items():
        P = PREC_OF[key.split("_")[0]]
        ms = item["ms"]
        if "_batched" in key:
            continue
        if key.endswith("_plain"):
            item["fp64_issue_frac_measured"] = n ** 3 * INSTR_PER_MAC[P] / (ms * 1e-3) / peaks["fp64_add_op_s"]
        elif key.endswith("_split") or key.endswith("_crt"):
            item["int8_ops_frac_measured"] = item["int8_products"] * 2.0 * n ** 3 / (ms * 1e-3) / peaks["int8_mfma_op_s"]
    if roofline is not None:
        roofline["peak_measured"] = round(peaks["fp64_add_op_s"] / 1e12, 2)
        roofline["frac_of_measured"] = round(roofline["achieved"] * 1e12 / peaks["fp64_add_op_s"], 4)

    out = {
        "metric": METRIC, "value": value, "unit": "2mnk/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+i8", "data": "synthetic",
        "config": {"workload": f"square DD/TD/QD GEMM C = alpha*A*B + beta*C, m=n=k={n}, "
                               "random alpha/beta/C, plain EFT form and the split INT8-MFMA form in "
                               "both its triangular and its residue (CRT) variant; plus "
                               "batched DD and TD sets of 512 GEMMs with m,n,k ~ U[16,512], "
                               "each in the plain and the residue form (one hipGraph replay each)",
                   "m": n, "n": n, "k": n, "precisions": [NAME[P] for P in precs], "forms": forms,
                   "batched_sets": [NAME[P] for P in sorted(batched)],
                   "parts_per_step": len(order), "parallelism": "single GPU"},
        "breakdown": breakdown,
        "roofline": roofline,
        "measured_peaks": peaks,
        "wall_s_timed": round(wall, 3),
        "paper_context": PAPER_CONTEXT,
    }

    # ---- CPU oracle on this host's cores (bounded sample) ----
    if not args.no_cpu:
        note("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(host, precs, forms, n, devd, args.cpu_budget, batched)

    print(json.dumps(out), flush=True)


PREC_OF = {"DD": 2, "TD": 3, "QD": 4}


def blas_bench(args, mp, dev, stream):
    """axpy and dot at n = args.vec_n, gemv at m = n = 16384 ('N' and 'T'), in
    DD/TD/QD.  Reported against HBM bandwidth (algorithmic bytes: axpy 3 x 8P
    per element, dot 2 x 8P, gemv 8P per matrix entry) and as multiply-adds
    per second.  One JSON line."""
    import numpy as np
    import torch

    def timed(call):
        call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(max(3, args.steps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def fill(P, shape, seed):
        g = torch.Generator(device=dev).manual_seed(seed)
        t = torch.empty((P,) + shape, dtype=torch.float64, device=dev)
        t[0].uniform_(-1, 1, generator=g)
        for p in range(1, P):
            t[p] = t[p - 1] * 2.0 ** -54 * (torch.rand(shape, dtype=torch.float64, device=dev,
                                                       generator=g) * 2 - 1)
        return t

    parts = {}
    nv = args.vec_n
    for P in (2, 3, 4):
        x, y = fill(P, (nv,), 1), fill(P, (nv,), 2)
        alpha = [0.75] + [0.0] * (P - 1)
        ms = timed(lambda: mp.axpy(P, alpha, x, y, stream=stream))
        parts[f"{NAME[P]}_axpy"] = {"ms": round(ms, 4), "GB/s": 3 * 8 * P * nv / (ms * 1e-3) / 1e9,
                                    "MAC/s": nv / (ms * 1e-3)}
        res = torch.empty(P, dtype=torch.float64, device=dev)
        ws = mp.dot_workspace(P, nv, dev)
        ms = timed(lambda: mp.dot(P, x, y, res, workspace=ws, stream=stream))
        parts[f"{NAME[P]}_dot"] = {"ms": round(ms, 4), "GB/s": 2 * 8 * P * nv / (ms * 1e-3) / 1e9,
                                   "MAC/s": nv / (ms * 1e-3)}
        del x, y, ws
        torch.cuda.empty_cache()
        m = nm = 16384
        A = fill(P, (nm, m), 3)
        xv, yv = fill(P, (nm,), 4), fill(P, (m,), 5)
        for trans in ("N", "T"):
            ms = timed(lambda: mp.gemv(P, trans, m, nm, alpha, A, xv, [0.0] * P, yv, stream=stream))
            parts[f"{NAME[P]}_gemv_{trans}"] = {"ms": round(ms, 3), "GB/s": 8 * P * m * nm / (ms * 1e-3) / 1e9,
                                                "MAC/s": m * nm / (ms * 1e-3)}
        for k, v in parts.items():
            if k.startswith(NAME[P]):
                note("blas", k, v["ms"], "ms", round(v["GB/s"], 1), "GB/s")
        del A, xv, yv
        torch.cuda.empty_cache()
    copy_rate = mp.probe_peak("hbm_copy", stream)
    for v in parts.values():
        v["hbm_frac"] = v["GB/s"] * 1e9 / HBM_PEAK
        v["hbm_frac_of_copy"] = v["GB/s"] * 1e9 / copy_rate
    total_ms = sum(v["ms"] for v in parts.values())
    out = {"metric": "DD/TD/QD BLAS-1/2 bytes/s", "unit": "B/s",
           "value": sum(v["GB/s"] * 1e9 * v["ms"] for v in parts.values()) / total_ms, "n_gpus": 1,
           "steps": max(3, args.steps), "warmup": 1, "ms_per_step": round(total_ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"axpy and dot with n = {nv}, gemv 'N' and 'T' with m = n = 16384, "
                                  "DD/TD/QD, component planes", "n": nv},
           "hbm_copy_probe_GB/s": copy_rate / 1e9, "breakdown": parts}
    print(json.dumps(out), flush=True)


def strassen_bench(args, mp, synth, dev, stream):
    """C = A B at m = n = k = args.n in DD/TD/QD: the plain form against 1..4
    levels of Strassen's method over it.  Time (2 n^3 counted as the work, as
    for the plain form) and error on sampled entries, both componentwise
    (k u |A||B|) and normwise (u max|A| max|B| n).  One JSON line."""
    import numpy as np
    import torch
    from tests.exact import GemmChecker, mp_frac, sample_entries
    n = args.n
    parts = {}
    for P in (2, 3, 4):
        A = synth.mp_matrix(2, "A", P, n, n)
        B = synth.mp_matrix(2, "B", P, n, n)
        dA, dB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        one, zero = synth.mp_one(P), np.zeros(P)
        chk = GemmChecker(P, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, 1)))
        ents = sample_entries(synth.rng_for(2, "samples"), n, n, 32)
        u = 2.0 ** -{2: 104, 3: 150, 4: 200}[P]
        norm = u * float(np.abs(A[0]).max()) * float(np.abs(B[0]).max()) * n
        base_ms = None
        for L in (0, 1, 2, 3, 4):
            dC = torch.zeros((P, n, n), dtype=torch.float64, device=dev)
            if L == 0:
                call = lambda: mp.gemm(P, "N", "N", n, n, n, one, dA, dB, zero, dC, stream=stream)  # noqa: E731
            else:
                ws = mp.alloc_workspace(P, n, n, n, form="strassen", levels=L, device=dev)
                call = lambda: mp.gemm(P, "N", "N", n, n, n, one, dA, dB, zero, dC,  # noqa: E731
                                       form="strassen", levels=L, workspace=ws, stream=stream)
            call()
            torch.cuda.synchronize()
            times = []
            for _ in range(max(3, args.steps)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                call()
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            base_ms = ms if L == 0 else base_ms
            got = dC.cpu().numpy()
            comp = chk.ratios(got, ents)
            nw = 0.0
            for i, j in ents:
                exact, _ = chk.entry(i, j)
                nw = max(nw, float(abs(mp_frac(got[:, j, i]) - exact)) / norm)
            parts[f"{NAME[P]}_L{L}"] = {"ms": round(ms, 3), "2mnk/s": 2.0 * n ** 3 / (ms * 1e-3),
                                        "speedup_vs_plain": round(base_ms / ms, 4),
                                        "err_ratio_max": float(comp.max()), "normwise_err": nw}
            note("strassen", NAME[P], "L", L, round(ms, 2), "ms", f"{comp.max():.3g}", f"{nw:.3g}")
            del dC
            if L > 0:
                del ws
            torch.cuda.empty_cache()
        del dA, dB
    total_ms = sum(v["ms"] for v in parts.values())
    out = {"metric": "DD/TD/QD GEMM 2mnk/s, plain vs Strassen levels", "unit": "2mnk/s",
           "value": 2.0 * n ** 3 * len(parts) / (total_ms * 1e-3), "n_gpus": 1,
           "steps": max(3, args.steps), "warmup": 1, "ms_per_step": round(total_ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"C = A B, m = n = k = {n}, DD/TD/QD, plain form and 1..4 levels of "
                                  "Strassen's method over it", "n": n,
                      "err_units": "err_ratio_max: |C - C*| / (k u |A||B|); normwise_err: |C - C*| / "
                                   "(u max|A| max|B| n); 32 sampled entries"},
           "breakdown": parts}
    print(json.dumps(out), flush=True)


def crt_bench(args, mp, synth, dev, stream):
    """C = alpha A B + beta C at m = n = k = args.n in DD, TD and QD (default
    digits): the triangular split form (one INT8 product per digit pair,
    s (s + 1) / 2 of them) against its residue form (one per modulus; for QD
    three half-size products of N moduli) with each tile configuration.  Time and error on sampled entries (k u
    (|alpha||A||B| + |beta||C|)).  One JSON line."""
    import numpy as np
    import torch
    from tests.exact import GemmChecker, sample_entries
    n = args.n
    parts = {}
    for P in (2, 3, 4):
        A = synth.mp_matrix(2, "A", P, n, n)
        B = synth.mp_matrix(2, "B", P, n, n)
        C = synth.mp_matrix(2, "C", P, n, n)
        alpha, beta = synth.mp_scalar(2, "alpha", P), synth.mp_scalar(2, "beta", P)
        dA, dB, dC0 = (torch.from_numpy(x).to(dev) for x in (A, B, C))
        s = mp.DEFAULT_SLICES[P]
        chk = GemmChecker(P, "N", "N", n, n, n, alpha, A, B, beta, C)
        ents = sample_entries(synth.rng_for(2, "samples"), n, n, 32)
        runs = [("split", -1)] + [("crt", t) for t in range(mp.num_configs(P, "crt"))]
        for form, tile in runs:
            ws = mp.alloc_workspace(P, n, n, n, s, tile, device=dev, form=form)
            dC = dC0.clone()
            call = lambda: mp.gemm(P, "N", "N", n, n, n, alpha, dA, dB, beta, dC, form=form,  # noqa: E731
                                   slices=s, tile=tile, workspace=ws, stream=stream)
            call()
            torch.cuda.synchronize()
            times = []
            for _ in range(max(3, args.steps)):
                dC.copy_(dC0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                call()
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            r = chk.ratios(dC.cpu().numpy(), ents)
            key = f"{NAME[P]}_{form}" + (f"_tile{tile}" if form == "crt" else "")
            products = s * (s + 1) // 2 if form == "split" else mp.crt_moduli(P, n, s)
            parts[key] = {"ms": round(ms, 3), "2mnk/s": 2.0 * n ** 3 / (ms * 1e-3), "s": s,
                          "int8_products": products,
                          "int8_ops/s": products * 2.0 * n ** 3 / (ms * 1e-3),
                          "err_ratio_max": float(r.max())}
            note("crt", key, round(ms, 3), "ms", f"{r.max():.3g}")
            del ws, dC
            torch.cuda.empty_cache()
        best = min(v["ms"] for k_, v in parts.items() if k_.startswith(NAME[P] + "_crt"))
        parts[f"{NAME[P]}_crt_speedup_vs_split"] = round(parts[f"{NAME[P]}_split"]["ms"] / best, 3)
        del dA, dB, dC0
    best_ms = [min(v["ms"] for k_, v in parts.items() if k_.startswith(nm + "_crt") and isinstance(v, dict))
               for nm in ("DD", "TD", "QD")]
    out = {"metric": "DD/TD/QD GEMM 2mnk/s, residue split form", "unit": "2mnk/s",
           "value": 2.0 * n ** 3 * 3 / (sum(best_ms) * 1e-3), "n_gpus": 1, "steps": max(3, args.steps),
           "warmup": 1, "ms_per_step": round(sum(best_ms), 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "i8", "data": "synthetic",
           "config": {"workload": f"C = alpha A B + beta C, m = n = k = {n}, DD (s = 16), TD (s = 23) and "
                                  "QD (s = 31, two levels), triangular split form vs residue form", "n": n,
                      "err_units": "|C - C*| / (k u (|alpha||A||B| + |beta||C|)), 32 sampled entries"},
           "breakdown": parts}
    print(json.dumps(out), flush=True)


TD_VARIANT_NAMES = {0: "TDaddq+TDmul", 1: "TDadd+TDmul", 2: "TDaddq+TDmulq", 3: "TDadd+TDmulq"}


def td_variants_bench(args, mp, synth, dev, stream):
    """The TD operations of Sec. 2.3 side by side: the default pair (TDaddq,
    Algorithm 4) against the accurate addition (Algorithm 3) and TDmulq.
    GEMM: m = n = k = 2048 on uniform and on exponent-spread inputs, time and
    error against the exact product on sampled entries.  Element-wise: rate at
    n = 2^26 and relative error against the exact result on cancelling
    operands.  One JSON line."""
    import numpy as np
    import torch
    from fractions import Fraction
    from tests.exact import GemmChecker, mp_frac, sample_entries
    P, n = 3, 2048
    one, zero = synth.mp_one(P), np.zeros(P)
    gemm_parts = {}
    for label, spread in (("uniform", None), ("spread_e30", (-30, 30))):
        A = synth.mp_matrix(3, "A", P, n, n, exp_range=spread)
        B = synth.mp_matrix(3, "B", P, n, n, exp_range=spread)
        dA, dB = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        chk = GemmChecker(P, "N", "N", n, n, n, one, A, B, zero, np.zeros((P, n, 1)))
        ents = sample_entries(synth.rng_for(3, "samples"), n, n, 256)
        for v, name in TD_VARIANT_NAMES.items():
            dC = torch.zeros((P, n, n), dtype=torch.float64, device=dev)
            call = lambda: mp.gemm(P, "N", "N", n, n, n, one, dA, dB, zero, dC, variant=v,  # noqa: E731
                                   stream=stream)
            call()
            torch.cuda.synchronize()
            times = []
            for _ in range(max(3, args.steps)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                call()
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            r = chk.ratios(dC.cpu().numpy(), ents)
            gemm_parts[f"gemm_{label}_{name}"] = {"ms": round(ms, 3), "2mnk/s": 2.0 * n ** 3 / (ms * 1e-3),
                                                  "err_ratio_max": float(r.max()),
                                                  "err_ratio_median": float(np.median(r))}
            note("td gemm", label, name, round(ms, 2), "ms", f"{r.max():.3g}")
            del dC
        del dA, dB
    # element-wise: rate on long vectors, error on cancelling operands
    vec_parts = {}
    nv = args.vec_n
    g = torch.Generator(device=dev).manual_seed(3)
    x = torch.empty((P, nv), dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    for t in (x, y):
        t[0].uniform_(-1, 1, generator=g)
        for p in range(1, P):
            t[p] = t[p - 1] * 2.0 ** -54 * (torch.rand(nv, dtype=torch.float64, device=dev, generator=g) * 2 - 1)
    r = torch.empty_like(x)
    rng = np.random.Generator(np.random.PCG64(31))
    ns = 1 << 13
    xs = synth.mp_uniform(rng, P, (ns,))
    ys = synth.mp_uniform(rng, P, (ns,))
    ys[:, : ns // 2] = -xs[:, : ns // 2]
    ys[0, : ns // 2] *= 1 + 2.0 ** -45 * rng.uniform(-1, 1, ns // 2)   # heavy cancellation
    dxs, dys = torch.from_numpy(xs).to(dev), torch.from_numpy(ys).to(dev)
    for op in ("add", "add_acc", "mul", "mulq"):
        call = lambda: mp.vec(P, op, x, y, r, stream=stream)  # noqa: E731
        call()
        torch.cuda.synchronize()
        times = []
        for _ in range(max(3, args.steps)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        drs = torch.empty_like(dxs)
        mp.vec(P, op, dxs, dys, drs, stream=stream)
        got = drs.cpu().numpy()
        worst = 0.0
        for i in range(ns):
            X, Y, R = mp_frac(xs[:, i]), mp_frac(ys[:, i]), mp_frac(got[:, i])
            ex = X + Y if op.startswith("add") else X * Y
            if ex != 0:
                worst = max(worst, float(abs(R - ex) / abs(ex) / Fraction(1, 2 ** 159)))
        vec_parts[op] = {"ms": round(ms, 4), "GB/s": 3.0 * 8 * P * nv / (ms * 1e-3) / 1e9,
                         "max_rel_err_2^-159": worst}
        note("td vec", op, round(ms, 3), "ms", f"{worst:.3g}")
    total_ms = sum(v["ms"] for v in gemm_parts.values())
    out = {"metric": "TD GEMM 2mnk/s and error by TD operation variant", "unit": "2mnk/s",
           "value": 2.0 * n ** 3 * len(gemm_parts) / (total_ms * 1e-3), "n_gpus": 1,
           "steps": max(3, args.steps), "warmup": 1, "ms_per_step": round(total_ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"TD GEMM m=n=k={n} (uniform and exponent-spread entries), four "
                                  "add/mul variants; element-wise TD add/mul variants, n = 2^26",
                      "err_ratio_unit": "|C - C*| / (k u |A||B|), u = 2^-150, 256 sampled entries",
                      "vec_error_sample": f"{ns} operand pairs, half with |x + y| ~ 2^-45 |x|"},
           "gemm": gemm_parts, "vec": vec_parts}
    print(json.dumps(out), flush=True)


def vec_bench(args, mp, dev, stream):
    """Element-wise r = x + y and r = x * y on n-element DD/TD/QD vectors in
    component planes (Sec. 2.5): reads 2 x 8P bytes and writes 8P bytes per
    element, so the bound is HBM bandwidth.  One JSON line."""
    import numpy as np
    import torch
    n = args.vec_n
    parts = {}
    for P in (2, 3, 4):
        g = torch.Generator(device=dev).manual_seed(P)
        x = torch.empty((P, n), dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for t in (x, y):
            t[0].uniform_(-1, 1, generator=g)
            for p in range(1, P):      # each further component below half an ulp of the one before
                t[p] = t[p - 1] * 2.0 ** -54 * (torch.rand(n, dtype=torch.float64, device=dev,
                                                           generator=g) * 2 - 1)
        r = torch.empty_like(x)
        for op in ("add", "mul"):
            call = lambda: mp.vec(P, op, x, y, r, stream=stream)  # noqa: E731
            for _ in range(max(1, args.warmup)):
                call()
            torch.cuda.synchronize()
            times = []
            for _ in range(max(3, args.steps)):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                call()
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            nbytes = 3.0 * 8 * P * n
            parts[f"{NAME[P]}_{op}"] = {"ms": round(ms, 4), "GB/s": nbytes / (ms * 1e-3) / 1e9,
                                        "hbm_frac": nbytes / (ms * 1e-3) / HBM_PEAK,
                                        "elements/s": n / (ms * 1e-3)}
            note("vec", NAME[P], op, round(ms, 3), "ms", round(nbytes / (ms * 1e-3) / 1e9, 1), "GB/s")
        del x, y, r
        torch.cuda.empty_cache()
    copy_rate = mp.probe_peak("hbm_copy", stream)
    note("hbm copy probe", round(copy_rate / 1e9, 1), "GB/s")
    for v in parts.values():
        v["hbm_frac_of_copy"] = v["GB/s"] * 1e9 / copy_rate
    worst = min(parts, key=lambda k: parts[k]["hbm_frac"])
    total_ms = sum(v["ms"] for v in parts.values())
    total_bytes = sum(3.0 * 8 * PREC_OF[k.split("_")[0]] * n for k in parts)
    out = {"metric": "element-wise DD/TD/QD add and mul, bytes/s", "value": total_bytes / (total_ms * 1e-3),
           "unit": "B/s", "n_gpus": 1, "steps": max(3, args.steps), "warmup": max(1, args.warmup),
           "ms_per_step": round(total_ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"r = x op y, n = {n} elements per vector, DD/TD/QD, add and mul, "
                                  "component planes", "n": n},
           "breakdown": parts,
           "roofline": {"bound": "hbm", "kernel": f"vec_kernel ({worst})",
                        "achieved": round(parts[worst]["GB/s"], 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                        "frac": round(parts[worst]["hbm_frac"], 4), "traffic": None,
                        "peak_measured": round(copy_rate / 1e9, 1),
                        "frac_of_measured": round(parts[worst]["GB/s"] * 1e9 / copy_rate, 4)}}
    print(json.dumps(out), flush=True)


def measured_peaks(mp, stream):
    """FP64 and INT8 matrix-core throughput measured on this GPU by the
    library's probes (independent FMA / add / multiply chains per thread;
    back-to-back 32x32x32 INT8 MFMAs per wave), a few milliseconds each."""
    return {"fp64_fma_flop_s": mp.probe_peak("fp64_fma", stream),
            "fp64_add_op_s": mp.probe_peak("fp64_add", stream),
            "fp64_mul_op_s": mp.probe_peak("fp64_mul", stream),
            "int8_mfma_op_s": mp.probe_peak("int8_mfma", stream),
            "hbm_copy_byte_s": mp.probe_peak("hbm_copy", stream),
            "published": {"fp64_fma_flop_s": FP64_PEAK, "fp64_op_s": FP64_ISSUE, "int8_op_s": INT8_PEAK,
                          "hbm_byte_s": HBM_PEAK}}


def separate_launches(mp, P, b, stream):
    """The same batched set as one plain launch per problem (not in the step)."""
    import torch
    for _ in range(2):
        for q in b["probs"]:
            mp.gemm(P, q["transa"], q["transb"], q["m"], q["n"], q["k"], q["alpha"], q["A"], q["B"],
                    q["beta"], q["C"], stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for q in b["probs"]:
        mp.gemm(P, q["transa"], q["transb"], q["m"], q["n"], q["k"], q["alpha"], q["A"], q["B"],
                q["beta"], q["C"], stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    return {"separate_launches_ms": round(ms, 3), "separate_launches_2mnk/s": b["work"] / (ms * 1e-3)}


def other_workload(args, mp, synth, dev, stream):
    """qd2048-spread: QD n = 2048 with exponent spread, all forms, slices from
    the accuracy rule; dd8192: DD n = 8192, all forms.  One JSON line."""
    import numpy as np
    import torch
    from tests.exact import GemmChecker, sample_entries
    spread_qd = args.workload == "qd2048-spread"
    fam = 3 if spread_qd else 4               # seed family of the workload's inputs
    if spread_qd:
        P, n, spread = 4, 2048, (-30, 30)
    else:
        P, n, spread = 2, 8192, None
    A = synth.mp_matrix(fam, "A", P, n, n, exp_range=spread)
    B = synth.mp_matrix(fam, "B", P, n, n, exp_range=spread)
    one, zero = synth.mp_one(P), np.zeros(P)
    dA = torch.from_numpy(A).to(dev)
    dB = torch.from_numpy(B).to(dev)
    note("inputs ready", NAME[P], n)
    forms = args.forms.split(",")
    if "crt" not in forms:
        forms.append("crt")        # the residue form of the split product, too
    if spread_qd:
        # "same error": the smallest s whose result on a block of rows stays
        # within 1e-6 k u (|A||B|)_ij of the plain (canonical) result
        s, rule_ratio = mp.tune_slices(P, "N", "N", n, n, n, dA, dB, target=SAME_ERROR_TARGET,
                                       smin=28, smax=40, stream=stream)
        note("slice rule", s, rule_ratio)
    else:
        s, rule_ratio = mp.DEFAULT_SLICES[P], None
    ws = mp.alloc_workspace(P, n, n, n, s, device=dev) if "split" in forms else None
    n_mod = mp.crt_moduli(P, n, s) if "crt" in forms else 0
    if "crt" in forms and n_mod == 0:
        note("residue form: no modulus count suffices for", NAME[P], "s =", s, "- skipped")
        forms.remove("crt")
    ws_crt = mp.alloc_workspace(P, n, n, n, s, device=dev, form="crt") if "crt" in forms else None
    parts = {}
    chk = None if args.no_check else GemmChecker(P, "N", "N", n, n, n, one, A, B, zero,
                                                 np.zeros((P, 1, 1)))
    ents = sample_entries(synth.rng_for(fam, "samples"), n, n, 1024)
    for f in forms:
        dC = torch.zeros((P, n, n), dtype=torch.float64, device=dev)
        kw = (dict(form="split", slices=s, workspace=ws) if f == "split" else
              dict(form="crt", slices=s, workspace=ws_crt) if f == "crt" else dict(form="plain"))
        call = lambda: mp.gemm(P, "N", "N", n, n, n, one, dA, dB, zero, dC, stream=stream, **kw)  # noqa: E731
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        times = []
        for _ in range(args.steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            call()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        note("timed", f, round(ms, 3), "ms")
        item = {"ms": round(ms, 3), "2mnk/s": 2.0 * n ** 3 / (ms * 1e-3)}
        if f == "split":
            item["slices"] = s
            item["int8_ops_frac"] = s * (s + 1) / 2 * 2.0 * n ** 3 / (ms * 1e-3) / INT8_PEAK
        elif f == "crt":
            item["slices"] = s
            item["moduli"] = n_mod
            item["int8_ops_frac"] = n_mod * 2.0 * n ** 3 / (ms * 1e-3) / INT8_PEAK
        else:
            item["fp64_peak_frac"] = n ** 3 * FLOPS_PER_MAC[P] / (ms * 1e-3) / FP64_PEAK
        if chk is not None:
            r = chk.ratios(dC.cpu().numpy(), ents)
            item["err_ratio_max"] = float(r.max())
            item["err_ratio_median"] = float(np.median(r))
            note("checked", f, item["err_ratio_max"])
        parts[f"{NAME[P]}_{f}"] = item
    total_ms = sum(v["ms"] for v in parts.values())
    workload = ("QD GEMM m=n=k=2048, entries u*2^e, e ~ U{-30..30} per entry, plain, split and "
                "residue (CRT) split forms, slices from the accuracy rule" if spread_qd else
                "DD GEMM m=n=k=8192, plain, split and residue (CRT) split forms")
    out = {"metric": METRIC, "value": 2.0 * n ** 3 * len(parts) / (total_ms * 1e-3), "unit": "2mnk/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(total_ms, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64+i8", "data": "synthetic",
           "config": {"workload": workload, "m": n, "n": n, "k": n, "precision": NAME[P],
                      "samples": len(ents) if chk is not None else 0,
                      "err_ratio_unit": "|C - C*| / (k u (|A||B|)_ij), u = 2^-104 DD / 2^-200 QD"},
           "breakdown": parts}
    if rule_ratio is not None:
        out["slice_rule"] = {"slices": s, "max_diff_vs_plain_on_64_rows": rule_ratio,
                             "target": SAME_ERROR_TARGET}
    print(json.dumps(out), flush=True)


def cpu_baseline(host, precs, forms, n, devd, budget, batched):
    """The oracle, as it stands, timed on samples of each part of the step and
    extrapolated to the part's full work:

    * plain form: a square block of C (all k), grown until it takes about its
      share of the budget; per-entry cost is uniform, so the block's rate is
      the part's rate;
    * split forms: the oracle slices the rows and columns a block needs
      (serially) and then forms the block's entries; slicing is linear in
      rows + columns, so it is timed on 256 columns of op(B) and scaled to all
      2n rows and columns once, and only the products of a square block are
      scaled by n^2 / (rows cols);
    * batched sets: the first problems of each set, in the plain and in
      the residue form.

    One thread and all threads are timed on the same block (DD plain)."""
    import oracle
    threads = oracle.num_threads()
    per = budget / max(1, len(precs) * len(forms) + 2 * len(batched))
    est_total = 0.0
    total_work = 0.0
    parts = []
    for P, b in sorted(batched.items()):
        t0 = time.perf_counter()
        done = 0.0
        cnt = 0
        for q in b["host"]:
            oracle.gemm(P, q["transa"], q["transb"], q["m"], q["n"], q["k"], q["alpha"], q["A"],
                        q["B"], q["beta"], q["C"])
            done += 2.0 * q["m"] * q["n"] * q["k"]
            cnt += 1
            if time.perf_counter() - t0 > per / 2:
                break
        rate = done / (time.perf_counter() - t0)
        est_total += b["work"] / rate
        total_work += b["work"]
        parts.append(f"{NAME[P]}-batched: first {cnt} problems ({rate:.3g} 2mnk/s)")
        t0 = time.perf_counter()
        done = 0.0
        cnt = 0
        for q in b["host"]:
            oracle.gemm_crt(P, b["s"], q["transa"], q["transb"], q["m"], q["n"], q["k"], q["alpha"], q["A"],
                            q["B"], q["beta"], q["C"])
            done += 2.0 * q["m"] * q["n"] * q["k"]
            cnt += 1
            if time.perf_counter() - t0 > per / 2:
                break
        rate = done / (time.perf_counter() - t0)
        est_total += b["work"] / rate
        total_work += b["work"]
        parts.append(f"{NAME[P]}-batched-residue: first {cnt} problems ({rate:.3g} 2mnk/s)")
    for P in precs:
        A, B, C, alpha, beta = host[P]
        for f in forms:
            s = devd[P]["s"]

            def once(r):
                t = time.perf_counter()
                if f == "plain":
                    oracle.gemm(P, "N", "N", n, n, n, alpha, A, B, beta, C, rows=(0, r), cols=(0, r))
                elif f == "crt":
                    oracle.gemm_crt(P, s, "N", "N", n, n, n, alpha, A, B, beta, C, rows=(0, r), cols=(0, r))
                else:
                    oracle.gemm_split(P, s, "N", "N", n, n, n, alpha, A, B, beta, C, rows=(0, r), cols=(0, r))
                return time.perf_counter() - t
            slice_full = 0.0
            if f != "plain":
                # slicing of 256 columns of op(B) (exponents and digits), the
                # oracle's own serial code, scaled to the 2n rows and columns
                t = time.perf_counter()
                F = oracle.split_exponents(P, "N", True, 256, n, B)
                oracle.split_slices(P, s, "N", True, 256, n, B, F)
                slice_full = (time.perf_counter() - t) * 2 * n / 256
            r = 2
            t = once(r)
            while t < per / 4 and r < n:
                r = min(n, r * 2)
                t = once(r)
            prod = max(t - slice_full * 2 * r / (2 * n), 1e-9)
            full = slice_full + prod * (n / r) ** 2
            rate = 2.0 * n ** 3 / full
            est_total += full
            total_work += 2.0 * n ** 3
            extra = f", slicing {slice_full:.3g} s of it" if f != "plain" else ""
            parts.append(f"{NAME[P]}-{f}: {r}x{r} block ({rate:.3g} 2mnk/s{extra})")
    value = total_work / est_total
    # one thread and all threads on the same block: DD (or the lowest
    # precision) plain, 32 x 256 entries, all k
    P1 = min(precs)
    A, B, C, alpha, beta = host[P1]
    same = {}
    for nt in (1, threads):
        t = time.perf_counter()
        oracle.gemm(P1, "N", "N", n, n, n, alpha, A, B, beta, C, rows=(0, 32), cols=(0, 256), nthreads=nt)
        same[nt] = 2.0 * 32 * 256 * n / (time.perf_counter() - t)
    info = cpu_info()
    return {"value": value, "unit": "2mnk/s", "cores": threads, "kind": "oracle",
            "cpu_model": info["model"], "physical_cores": info["physical_cores"],
            "logical_cpus": info["logical_cpus"], "cpus_allowed": info["cpus_allowed"],
            "same_block": {"sample": f"{NAME[P1]} plain, 32 x 256 block of C, k = {n}",
                           "one_thread_2mnk/s": same[1], "all_threads_2mnk/s": same[threads],
                           "threads": threads, "speedup": same[threads] / same[1]},
            "sample": "per large GEMM of the step a square block of C (all k) and, for the split "
                      "forms, the slicing scaled separately; per batched set its first problems; "
                      "each extrapolated to the part's full 2mnk: " + "; ".join(parts)}


def cpu_info():
    """Model name and core counts of this host (lscpu, else /proc/cpuinfo)."""
    import subprocess
    out = {"model": "unknown", "physical_cores": None, "logical_cpus": os.cpu_count(),
           "cpus_allowed": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = {}
        for line in txt.splitlines():
            if ":" in line:
                key, val = line.split(":", 1)
                kv[key.strip()] = val.strip()
        out["model"] = kv.get("Model name", out["model"])
        cores = int(kv.get("Core(s) per socket", "0")) * int(kv.get("Socket(s)", "0"))
        out["physical_cores"] = cores or None
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    if out["model"] == "unknown":
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        out["model"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    return out


if __name__ == "__main__":
    main()

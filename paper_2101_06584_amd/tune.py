"""Autotuning front end: runs the library's autotuner (mpgemm_autotune,
mpgemm_batch_autotune) over the shapes this project benchmarks and writes the
tuning table that the binding loads with the library (tuned_gfx950.txt).

    python -m paper_2101_06584_amd.tune [--out PATH] [--quick]

Timing uses synthetic operands on the GPU; the table records, per precision,
form (0 plain, 1 split, 3 batched, 5 residue split) and log2 shape bucket, the
fastest configuration id.  --forms limits the forms tuned; --keep starts from
the table already there (so the other forms keep their entries).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import torch

from . import api


def batch_problems(P: int, count: int, lo: int, hi: int, seed: int, device="cuda"):
    """Uneven GEMMs with m, n, k uniform in [lo, hi] (random operands)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    shapes = torch.randint(lo, hi + 1, (count, 3), generator=g).tolist()
    probs = []
    for m, n, k in shapes:
        def mat(rows, cols):
            t = torch.empty((P, cols, rows), dtype=torch.float64, device=device)
            t[0].uniform_(-1, 1)
            for p in range(1, P):
                t[p] = t[p - 1] * 2.0 ** -54 * (torch.rand_like(t[p - 1]) * 2 - 1)
            return t
        probs.append(dict(m=m, n=n, k=k, A=mat(m, k), B=mat(k, n), C=mat(m, n),
                          alpha=[1.0] + [0.0] * (P - 1), beta=[0.0] * P))
    return probs


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "tuned_gfx950.txt"))
    ap.add_argument("--quick", action="store_true", help="only the n = 4096 benchmark shapes")
    ap.add_argument("--forms", default="plain,split,crt,batched",
                    help="comma-separated forms to tune (plain, split, crt, batched)")
    ap.add_argument("--keep", action="store_true", help="start from the table already there")
    args = ap.parse_args(argv)
    forms = args.forms.split(",")
    if not args.keep:
        os.environ["MPGEMM_NO_TUNED_TABLE"] = "1"   # tune from the built-in defaults
    api.load()
    t0 = time.time()
    sizes = [4096] if args.quick else [1024, 2048, 4096]
    gemm_forms = [f for f in ("plain", "split", "crt") if f in forms]
    for n in sizes:
        for P in (2, 3, 4):
            for form in gemm_forms:
                best = api.autotune(P, form, n, n, n, api.DEFAULT_SLICES[P] if form != "plain" else 0)
                print(f"P={P} {form:5s} n={n}: tile {best}", flush=True)
    if not args.quick:
        # exponent-spread QD (more digits: 33 for the split form, 32 for the
        # residue form's two levels) and DD n = 8192
        if "split" in forms:
            best = api.autotune(4, "split", 2048, 2048, 2048, 33)
            print(f"P=4 split n=2048 s=33: tile {best}", flush=True)
        if "crt" in forms:
            best = api.autotune(4, "crt", 2048, 2048, 2048, 32)
            print(f"P=4 crt   n=2048 s=32: tile {best}", flush=True)
        for form in gemm_forms:
            best = api.autotune(2, form, 8192, 8192, 8192, 16 if form != "plain" else 0)
            print(f"P=2 {form:5s} n=8192: tile {best}", flush=True)
    if "batched" in forms:
        for P in (2, 3):
            probs = batch_problems(P, 512, 16, 512, seed=5)
            best = api.batch_autotune(P, probs)
            print(f"P={P} batched 512 x U[16,512]^3: tile {best}", flush=True)
            del probs
            torch.cuda.empty_cache()
    api.autotune_save(args.out)
    print(f"wrote {args.out} in {time.time() - t0:.1f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

#!/usr/bin/env python3
"""Throughput of the fused Pauli-sum outer product + sort-and-combine.

One step = pauli_outer_product_merged on the n=500, 10,000 x 10,000
Jordan-Wigner-shaped workload (1e8 products, complex128, plain FP64): every
pair is multiplied (XOR of the X/Z words, phase from popcounts, coefficient
product times i^k), the products are sorted on their fingerprint key and
equal strings are combined.  Inputs are resident in HBM before timing starts;
each step ends with the merged sum on the device.

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits with a
message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
WORKLOADS = {
    1: "n=16, 2,000 x 2,000 weight-1..4 sums, complex128, plain FP64 (4e6 products)",
    2: "n=500, 10,000 x 10,000 Jordan-Wigner-shaped sums, complex128, plain FP64 (1e8 products)",
    3: "n=500, H*H with 20,000 Jordan-Wigner-shaped real terms, FP64 plain (4e8 products)",
}


def _inputs(workload):
    import synth
    if workload == 1:
        return synth.workload1()
    if workload == 2:
        return synth.workload2()
    if workload == 3:
        H = synth.workload3()
        return H, H
    raise SystemExit("unknown workload %d" % workload)


def _traffic(stage, source_files):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current sources of the kernel."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(stage)
    except Exception:
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    for f in source_files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec.get("bytes_per_launch")


STAGE_SOURCES = {
    "bucket": ["paper_2605_25974_amd/csrc/k_bucket.hip", "paper_2605_25974_amd/csrc/common.h"],
    "sort": ["paper_2605_25974_amd/csrc/k_sort.hip"],
    "segment": ["paper_2605_25974_amd/csrc/k_merge.hip", "paper_2605_25974_amd/csrc/common.h"],
    "outer_product": ["paper_2605_25974_amd/csrc/k_basic.hip", "paper_2605_25974_amd/csrc/common.h"],
}


def cpu_baseline(A, B, target_s=15.0):
    """The CPU oracle timed on a bounded block of the same pair space."""
    from oracle import oracle as O
    SA = O.Sum(A["n"], A["x"], A["z"], A["phase"], A["coef"])
    SB = O.Sum(B["n"], B["x"], B["z"], B["phase"], B["coef"])
    mj = B["x"].shape[0]
    rows = 4
    t = time.perf_counter()
    O.product_merge(SA, SB, i_range=(0, rows), j_range=(0, mj))
    dt = time.perf_counter() - t
    rows = max(1, min(A["x"].shape[0], int(rows * target_s / max(dt, 1e-3))))
    t = time.perf_counter()
    O.product_merge(SA, SB, i_range=(0, rows), j_range=(0, mj))
    dt = time.perf_counter() - t
    return {"value": rows * mj / dt, "unit": "products/s", "cores": 1, "kind": "oracle",
            "sample": "%d x %d pair block (%d products) of the same workload, %.1f s, "
                      "single thread" % (rows, mj, rows * mj, dt)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2605_25974_amd as pl

    torch.cuda.set_device(0)
    A, B = _inputs(args.workload)
    GA = pl.PauliSum.from_dict(A)
    GB = GA if B is A else pl.PauliSum.from_dict(B)
    P = A["x"].shape[0] * B["x"].shape[0]

    for _ in range(args.warmup):
        out = pl.outer_product_merged(GA, GB)
        out.destroy()
    torch.cuda.synchronize()

    pl.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U = 0
    for _ in range(args.steps):
        out = pl.outer_product_merged(GA, GB)
        U = out.m
        out.destroy()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = pl.profile_read()
    pl.profile_enable(False)

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    dom = max(stages, key=lambda k: stages[k][0]) if stages else None
    roof = None
    if dom:
        ms, launches, by = stages[dom]
        achieved = (by / launches) / (ms / launches * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _traffic(dom, STAGE_SOURCES.get(dom, [])),
                "kernel_stage": dom, "launch_ms": round(ms / launches, 4),
                "algorithmic_bytes_per_launch": by / launches}

    rec = {
        "metric": "Pauli products/s incl. sort-merge, 500 qubits; FP32-comp vs FP64 at <=1e-6 err",
        "value": P * args.steps / elapsed,
        "unit": "products/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generators standing in for the paper's random sums)",
        "config": {"workload": WORKLOADS[args.workload], "products": P, "merged_terms": U},
        "merged_terms_per_s": U * args.steps / elapsed,
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(A, B, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

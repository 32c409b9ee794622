#!/usr/bin/env python3
"""Throughput of the fused Pauli-sum outer product with sort-and-combine.

One step = pauli_outer_product_merged on the chosen workload.  The default is
the n=500, 10,000 x 10,000 Jordan-Wigner-shaped sum product (1e8 products,
complex128, plain FP64).  Every pair is multiplied: XOR of the X/Z words,
phase from popcounts, coefficient product times i^k.  The products are then
ordered by their fingerprint key and equal strings are combined.  Inputs are
resident in HBM before timing starts, and each step ends with the merged sum
on the device.

The same steps are then run in the precision form: FP32 products,
compensated merge, FP64 re-merge of cancelled segments.  Its largest
relative coefficient error against the plain FP64 result of the same GPU is
reported beside its throughput.

Prints one JSON line.  Only one GPU is used; --gpus above 1 exits with a
message.  --copy-calibration runs a plain copy kernel of known size instead;
its FETCH_SIZE / WRITE_SIZE counters scale the expand kernel's counters to
bytes.
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
# 32-bit integer vector ALU: 256 compute units x 64 lanes per clock x 2.4 GHz
INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
COMP_TAU = 0.3         # cancellation threshold of the precision form
WORKLOADS = {
    1: "n=16, 2,000 x 2,000 weight-1..4 sums, complex128 (4e6 products)",
    2: "n=500, 10,000 x 10,000 Jordan-Wigner-shaped sums, complex128 (1e8 products)",
    3: "n=500, H*H with 20,000 Jordan-Wigner-shaped real terms, complex128 (4e8 products)",
    4: "256 products, n in {64,128,256,500}, lognormal term counts (median 2,000, clipped "
       "to [100, 20,000]), complex64, compensated, autotuned, in calls of 32",
    5: "1e6 terms at n=500 (weight 1..20, |c| log-uniform in [1e-8, 1]) through 64 "
       "rotations, drop |c| < 1e-10",
    6: "commutator [A, B] of the n=500 10,000 x 10,000 Jordan-Wigner-shaped sums, "
       "complex128 (1e8 pairs)",
    7: "Clifford circuit of 112 random gates (H, S, S^dag, X, Y, Z, CX, CZ, SWAP) on the "
       "1e6-term n=500 propagation state, complex128",
    8: "lexicographic order of the merged product of the n=500 10,000 x 10,000 "
       "Jordan-Wigner-shaped sums (about 1e8 terms), complex128",
}
# sources of the kernel each stage's traffic figure was measured on
STAGE_SOURCES = {
    "write": ["paper_2605_25974_amd/csrc/expand.h", "paper_2605_25974_amd/csrc/common.h"],
    "clifford": ["paper_2605_25974_amd/csrc/k_clifford.hip", "paper_2605_25974_amd/csrc/common.h"],
}
COPY_BYTES = 2 << 30


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _inputs(workload):
    import synth
    if workload == 1:
        return synth.workload1()
    if workload == 2:
        return synth.workload2()
    H = synth.workload3()
    return H, H


def _sources_sha(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def _traffic(stage, workload):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current sources of the kernel and on this workload."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or stage not in STAGE_SOURCES:
        return None
    try:
        rec = json.load(open(path)).get(stage)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("workload") != workload:
        return None
    if rec.get("source_sha256") != _sources_sha(STAGE_SOURCES[stage]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(A, B, target_s=10.0):
    """The CPU oracle timed on a bounded block of the same pair space."""
    from oracle import oracle as O
    SA = O.Sum(A["n"], A["x"], A["z"], A["phase"], A["coef"])
    SB = SA if B is A else O.Sum(B["n"], B["x"], B["z"], B["phase"], B["coef"])
    mj = B["x"].shape[0]
    rows = 2
    t = time.perf_counter()
    O.product_merge(SA, SB, i_range=(0, rows), j_range=(0, mj))
    dt = time.perf_counter() - t
    rows = max(1, min(A["x"].shape[0], int(rows * target_s / max(dt, 1e-3))))
    t = time.perf_counter()
    O.product_merge(SA, SB, i_range=(0, rows), j_range=(0, mj))
    dt = time.perf_counter() - t
    return {"value": rows * mj / dt, "unit": "products/s", "cores": 1, "kind": "oracle",
            "sample": "rows 0..%d of the left sum times all %d right terms (%d products) of "
                      "the same workload, multiply and exact merge, %.1f s, one thread"
                      % (rows - 1, mj, rows * mj, dt)}


def _timed(pl, torch, GA, GB, steps, warmup, **kw):
    for _ in range(warmup):
        pl.outer_product_merged(GA, GB, **kw).destroy()
    torch.cuda.synchronize()
    pl.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    U = 0
    for _ in range(steps):
        out = pl.outer_product_merged(GA, GB, **kw)
        U = out.m
        out.destroy()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = pl.profile_read()
    pl.profile_enable(False)
    return elapsed, U, stages


def _rel_err(pl, torch, GA, GB, tau, CA=None, CB=None):
    """Max relative error of the precision form against plain FP64 on this
    GPU, over strings with |c| >= 1e-6 max |c| (both outputs hold the same
    strings in the same order).  CA, CB: the operands of the precision form
    when they differ from the FP64 ones (complex64 copies)."""
    pl.trim_memory()  # torch needs device memory for the comparison
    ref = pl.outer_product_merged(GA, GB).export_torch()
    got = pl.outer_product_merged(GA if CA is None else CA, GB if CB is None else CB,
                                  mode=pl.COMPENSATED, tau=tau).export_torch()
    for k in ("x", "z", "fp"):
        if not torch.equal(ref[k], got[k]):
            raise SystemExit("precision form produced different strings than plain FP64")
    r = ref["coef"]
    g = got["coef"].to(torch.complex128)
    mag = r.abs()
    sel = mag >= 1e-6 * mag.max()
    return float(((g - r).abs()[sel] / mag[sel]).max())


def _batched(pl, torch, args):
    """Batched form: 256 products in calls of 32, compensated and autotuned,
    against the same products as single plain launches."""
    import numpy as np
    import synth
    plan = synth.workload4_plan()
    pairs = [synth.workload4_batch(b, n, m1, m2) for b, (n, m1, m2) in enumerate(plan)]
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    P = sum(m1 * m2 for _, m1, m2 in plan)
    chunk = 32
    _log("batched: %d products in %d pairs" % (P, len(plan)))

    def run_batched():
        U = 0
        for c0 in range(0, len(plan), chunk):
            outs = pl.outer_product_batched(GA[c0:c0 + chunk], GB[c0:c0 + chunk],
                                            mode=pl.COMPENSATED, tau=COMP_TAU)
            for o in outs:
                U += o.m
                o.destroy()
        return U

    def run_single():
        for a, b in zip(GA, GB):
            pl.outer_product_merged(a, b).destroy()

    for _ in range(max(1, args.warmup)):  # also tunes every class
        run_batched()
        run_single()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        U = run_batched()
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / args.steps
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_single()
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / args.steps
    # error of the compensated products against plain FP64 on the same
    # (complex64) inputs, on every 16th pair
    err = 0.0
    for b in range(0, len(plan), 16):
        A, B = pairs[b]
        A64 = dict(A, coef=A["coef"].astype(np.complex128))
        B64 = dict(B, coef=B["coef"].astype(np.complex128))
        g64a, g64b = pl.PauliSum.from_dict(A64), pl.PauliSum.from_dict(B64)
        err = max(err, _rel_err(pl, torch, g64a, g64b, COMP_TAU, GA[b], GB[b]))
    return {
        "metric": "Pauli products/s incl. sort-merge, batched form",
        "value": P / tb, "unit": "products/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * tb, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (compensated)",
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[4], "products": P, "merged_terms": U},
        "single_plain_launches": {"value": P / ts, "unit": "products/s",
                                  "ms_per_step": round(1e3 * ts, 3), "dtype": "f32"},
        "max_rel_err_vs_fp64": err,
        "err_definition": "max over every 16th pair of |c32 - c64| / |c64|, |c64| >= 1e-6 max|c64|",
    }


def _propagation(pl, torch, args):
    """Propagation loop: 64 conjugation steps (FP64 and compensated) and the
    literal left-multiplication for its first 8 steps."""
    import synth
    S = synth.workload5_state()
    theta, px, pz = synth.workload5_rotations()
    G = pl.PauliSum.from_dict(S)
    drop = 1e-10
    res = {}
    for name, rot, steps, mode in (("conjugate_fp64", pl.ROTATE_CONJUGATE, 64, pl.PLAIN),
                                   ("conjugate_compensated", pl.ROTATE_CONJUGATE, 64,
                                    pl.COMPENSATED),
                                   ("product_fp64_8_steps", pl.ROTATE_PRODUCT, 8, pl.PLAIN)):
        pl.propagate(G, px[:1], pz[:1], theta[:1], rotate_mode=rot, mode=mode,
                     drop_abs=drop).destroy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = pl.propagate(G, px[:steps], pz[:steps], theta[:steps], rotate_mode=rot, mode=mode,
                           drop_abs=drop, tau=COMP_TAU)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"steps": steps, "seconds": round(dt, 4), "final_terms": out.m,
                     "ms_per_step": round(1e3 * dt / steps, 3)}
        res[name + "_out"] = out
        _log("%s: %.3f s for %d steps, %d terms" % (name, dt, steps, out.m))
    # literal steps: products = 2 * terms entering each step
    m, prods = S["x"].shape[0], 0
    cur = G
    for t in range(8):
        prods += 2 * cur.m
        nxt = pl.propagate(cur, px[t:t + 1], pz[t:t + 1], theta[t:t + 1],
                           rotate_mode=pl.ROTATE_PRODUCT, drop_abs=drop)
        if cur is not G:
            cur.destroy()
        cur = nxt
    cur.destroy()
    lit = res["product_fp64_8_steps"]
    # compensated vs FP64 after 64 conjugation steps, on common strings
    pl.trim_memory()  # torch needs device memory for the comparison
    a = res.pop("conjugate_fp64_out").export_torch()
    b = res.pop("conjugate_compensated_out").export_torch()
    res.pop("product_fp64_8_steps_out").destroy()
    err = _common_rel_err(torch, a, b)
    return {
        "metric": "Pauli products/s incl. sort-merge, propagation loop",
        "value": prods / lit["seconds"], "unit": "products/s", "n_gpus": 1, "steps": 8,
        "warmup": 1, "ms_per_step": lit["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[5], "products": prods, "merged_terms": lit["final_terms"]},
        "runs": res,
        "compensated_max_rel_err_vs_fp64_after_64_steps": err,
        "err_definition": "strings present in both, |c64| >= 1e-6 max|c64|",
    }


def _common_rel_err(torch, a, b):
    import numpy as np
    fa, fb = a["fp"].cpu().numpy(), b["fp"].cpu().numpy()
    _, ia, ib = np.intersect1d(fa, fb, return_indices=True)
    ia = torch.from_numpy(ia).to(a["fp"].device)
    ib = torch.from_numpy(ib).to(b["fp"].device)
    same = (a["x"][ia] == b["x"][ib]).all(1) & (a["z"][ia] == b["z"][ib]).all(1)
    r = a["coef"][ia][same]
    g = b["coef"][ib][same].to(torch.complex128)
    mag = r.abs()
    sel = mag >= 1e-6 * mag.max()
    return float(((g - r).abs()[sel] / mag[sel]).max())


def _commutator(pl, torch, args):
    """[A, B] of the metric workload's sums: pairs/s including the search for
    anticommuting pairs, their sort and merge."""
    import synth
    A, B = synth.workload2()
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    P = A["x"].shape[0] * B["x"].shape[0]
    for _ in range(args.warmup):
        pl.commutator(GA, GB).destroy()
    torch.cuda.synchronize()
    pl.profile_enable(True)
    t0 = time.perf_counter()
    U = 0
    for _ in range(args.steps):
        out = pl.commutator(GA, GB)
        U = out.m
        out.destroy()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = pl.profile_read()
    pl.profile_enable(False)
    # dominant kernel: the anticommuting-pair search, bound by integer ALU work
    ms, launches, ops = stages["filter"]
    achieved = (ops / launches) / (ms / launches * 1e-3) / 1e12
    rec = {
        "metric": "Pauli pairs/s of the commutator incl. sort-merge",
        "value": P * args.steps / elapsed, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[6], "pairs": P, "merged_terms": U},
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": INT32_PEAK_TOPS,
                     "unit": "TOP/s (32-bit integer)", "frac": round(achieved / INT32_PEAK_TOPS, 4),
                     "traffic": None, "kernel": "k_comm_tiles", "stage": "filter",
                     "launch_ms": round(ms / launches, 4),
                     "algorithmic_ops_per_launch": ops / launches},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        rows = 2
        SB = O.Sum(B["n"], B["x"], B["z"], B["phase"], B["coef"])

        def sample(r):
            SA = O.Sum(A["n"], A["x"][:r], A["z"][:r], A["phase"][:r], A["coef"][:r])
            t = time.perf_counter()
            O.commutator(SA, SB)
            return time.perf_counter() - t

        dt = sample(rows)
        rows = max(1, min(A["x"].shape[0], int(rows * args.cpu_seconds / max(dt, 1e-3))))
        dt = sample(rows)
        rec["cpu_baseline"] = {
            "value": rows * B["x"].shape[0] / dt, "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": "the first %d left terms times all %d right terms (%d pairs), both "
                      "orders multiplied and merged exactly, %.1f s, one thread"
                      % (rows, B["x"].shape[0], rows * B["x"].shape[0], dt)}
    return rec


def _clifford_gates(n, count):
    import synth
    rng = synth.rng_for(7, 0)
    gates = []
    for _ in range(count):
        kind = int(rng.integers(0, 9))
        if kind >= 6:
            q0, q1 = rng.choice(n, size=2, replace=False)
            gates.append((kind, int(q0), int(q1)))
        else:
            gates.append((kind, int(rng.integers(0, n))))
    return gates


def _clifford(pl, torch, args):
    """Gate application on the SoA: terms/s through a 112-gate circuit in one
    streaming pass over the sum."""
    import synth
    S = synth.workload5_state()
    G = pl.PauliSum.from_dict(S)
    gates = _clifford_gates(S["n"], 112)
    m = S["x"].shape[0]
    for _ in range(args.warmup):
        pl.apply_clifford(G, gates).destroy()
    torch.cuda.synchronize()
    pl.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pl.apply_clifford(G, gates).destroy()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = pl.profile_read()
    pl.profile_enable(False)
    ms, launches, by = stages["clifford"]
    achieved = (by / launches) / (ms / launches * 1e-3) / 1e9
    rec = {
        "metric": "Pauli terms/s through a Clifford circuit",
        "value": m * args.steps / elapsed, "unit": "terms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64 (strings), f64 (copied)",
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[7], "terms": m, "gates": len(gates)},
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": _traffic("clifford", 7),
                     "kernel": "k_clifford", "stage": "clifford",
                     "launch_ms": round(ms / launches, 4),
                     "algorithmic_bytes_per_launch": by / launches},
    }
    if not args.no_cpu_baseline:
        import numpy as np
        from oracle import clifford as C
        from oracle import oracle as O
        so = O.Sum(S["n"], S["x"], S["z"], S.get("phase"), S["coef"])
        terms = 200
        t = time.perf_counter()
        C.apply(so, gates, terms=np.arange(terms))
        dt = time.perf_counter() - t
        terms = max(1, min(m, int(terms * args.cpu_seconds / max(dt, 1e-3))))
        t = time.perf_counter()
        C.apply(so, gates, terms=np.arange(terms))
        dt = time.perf_counter() - t
        rec["cpu_baseline"] = {
            "value": terms / dt, "unit": "terms/s", "cores": 1, "kind": "oracle",
            "sample": "the first %d terms through the same %d gates, letter images from the "
                      "gate matrices, %.1f s, one thread" % (terms, len(gates), dt)}
    return rec


def _lex(pl, torch, args):
    """Lexicographic order (pauli_sort_lex) of the merged 1e8-product output:
    terms/s, the merged sum resident in HBM before timing."""
    import synth
    A, B = synth.workload2()
    S = pl.outer_product_merged(pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B))
    m = S.m
    for _ in range(args.warmup):
        pl.sort_lex(S).destroy()
    torch.cuda.synchronize()
    pl.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pl.sort_lex(S).destroy()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = pl.profile_read()
    pl.profile_enable(False)
    ms, launches, by = stages["lex"]
    achieved = (by / launches) / (ms / launches * 1e-3) / 1e9
    rec = {
        "metric": "Pauli terms/s put in lexicographic order",
        "value": m * args.steps / elapsed, "unit": "terms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64 (keys)",
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[8], "terms": m},
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        # the whole call: word gathers, radix passes and the final row gather
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "sort_lex (all kernels of the call)",
                     "stage": "lex", "launch_ms": round(ms / launches, 4),
                     "algorithmic_bytes_per_launch": by / launches},
    }
    S.destroy()
    if not args.no_cpu_baseline:
        from oracle import lexorder as L
        from oracle import oracle as O
        SA = O.Sum(A["n"], A["x"], A["z"], A["phase"], A["coef"])
        SB = O.Sum(B["n"], B["x"], B["z"], B["phase"], B["coef"])
        rows = 100
        ref = O.product_merge(SA, SB, i_range=(0, rows))
        t = time.perf_counter()
        L.order(ref.x, ref.z)
        dt = time.perf_counter() - t
        rec["cpu_baseline"] = {
            "value": ref.x.shape[0] / dt, "unit": "terms/s", "cores": 1, "kind": "oracle",
            "sample": "the oracle's merged product of rows 0..%d of the left sum with all "
                      "10,000 right terms (%d strings), ordered by the lexicographic oracle "
                      "(numpy lexsort), %.2f s, one thread" % (rows - 1, ref.x.shape[0], dt)}
    return rec


def copy_calibration(steps):
    import torch
    n = COPY_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(steps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_kernel": "torch.mul(src, 1.0, out=dst), float32",
                      "bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES,
                      "launches": steps}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=2, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compensated", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--pcie", action="store_true",
                    help="also time one call from host inputs to the merged sum in host memory")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.steps)
        return

    import torch
    import paper_2605_25974_amd as pl

    torch.cuda.set_device(0)
    if args.workload in (4, 5, 6, 7, 8):
        rec = {4: _batched, 5: _propagation, 6: _commutator,
               7: _clifford, 8: _lex}[args.workload](pl, torch, args)
        print(json.dumps(rec), flush=True)
        return
    A, B = _inputs(args.workload)
    GA = pl.PauliSum.from_dict(A)
    GB = GA if B is A else pl.PauliSum.from_dict(B)
    P = A["x"].shape[0] * B["x"].shape[0]
    _log("inputs resident: %d x %d terms, n=%d" % (A["x"].shape[0], B["x"].shape[0], A["n"]))

    elapsed, U, stages = _timed(pl, torch, GA, GB, args.steps, args.warmup)
    ms_per_step = 1e3 * elapsed / args.steps
    _log("plain FP64: %.3f ms/step" % ms_per_step)

    dom = max(stages, key=lambda k: stages[k][0]) if stages else None
    roof = None
    if dom:
        ms, launches, by = stages[dom]
        achieved = (by / launches) / (ms / launches * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _traffic(dom, args.workload),
                "kernel": "k_expand" if dom == "write" else dom,
                "stage": dom, "launch_ms": round(ms / launches, 4),
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
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[args.workload], "products": P, "merged_terms": U},
        "merged_terms_per_s": U * args.steps / elapsed,
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "roofline": roof,
    }
    if not args.no_compensated:
        ce, cu, cst = _timed(pl, torch, GA, GB, args.steps, args.warmup,
                             mode=pl.COMPENSATED, tau=COMP_TAU)
        _log("precision form: %.3f ms/step" % (1e3 * ce / args.steps))
        rec["compensated"] = {
            "value": P * args.steps / ce, "unit": "products/s", "dtype": "f32 (compensated)",
            "ms_per_step": round(1e3 * ce / args.steps, 4), "tau": COMP_TAU,
            "merged_terms": cu,
            "max_rel_err_vs_fp64": _rel_err(pl, torch, GA, GB, COMP_TAU),
            "max_rel_err_vs_fp64_tau_1e-3": _rel_err(pl, torch, GA, GB, 1e-3),
            "err_definition": "max |c32 - c64| / |c64| over strings with |c64| >= 1e-6 max|c64|",
            "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in cst.items()},
        }
    if args.pcie:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ha = pl.PauliSum.from_dict(A)
        hb = ha if B is A else pl.PauliSum.from_dict(B)
        out = pl.outer_product_merged(ha, hb)
        host = out.export()
        dt = time.perf_counter() - t0
        rec["pcie_inclusive"] = {
            "value": P / dt, "unit": "products/s", "ms": round(1e3 * dt, 2),
            "note": "host inputs uploaded, fused product, merged sum (%d terms) copied back "
                    "to host memory" % host["x"].shape[0]}
        out.destroy()
    if not args.no_cpu_baseline:
        _log("timing the CPU oracle")
        rec["cpu_baseline"] = cpu_baseline(A, B, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

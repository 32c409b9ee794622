#!/usr/bin/env python3
"""Throughput of the fused Pauli-sum outer product with sort-and-combine.

One step = pauli_outer_product_merged on the chosen workload.  The default is
the n=500, 10,000 x 10,000 Jordan-Wigner-shaped sum product (1e8 products,
complex128, plain FP64).  Every pair is multiplied: XOR of the X/Z words,
phase from popcounts, coefficient product times i^k.  The products are then
ordered by their fingerprint key and equal strings are combined.  Inputs are
resident in HBM before timing starts, and each step ends with the merged sum
on the device.

The same steps are then run in the precision form (FP32 products,
compensated merge, FP64 re-merge of cancelled segments); its largest
relative coefficient error against the plain FP64 result of the same GPU is
reported beside its throughput.  The default run also reports every stage's
achieved bandwidth, a measured copy ceiling, and sub-records of the other
workloads: the H*H cancellation case (4e8 products), the batched form (256
products, eager calls and captured graphs, against single launches) and the
propagation loop (64 conjugation steps and 8 literal steps, host loop and
captured graph), and the CPU oracle timed on the host's cores.

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
    9: "1e6 terms at n=500 through 64 conjugation steps, drop |c| < 1e-10, complex128: the "
       "whole loop as one captured HIP graph (pauli_propagate_plan), replayed",
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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_block(n, A, B, i0, i1):
    """One worker of the CPU baseline: rows [i0, i1) of the left sum times
    every right term, multiplied and merged exactly by the oracle."""
    from oracle import oracle as O
    SA = O.Sum(n, A[0], A[1], A[2], A[3])
    SB = O.Sum(n, B[0], B[1], B[2], B[3])
    t = time.perf_counter()
    O.product_merge(SA, SB, i_range=(i0, i1), j_range=(0, B[0].shape[0]))
    return time.perf_counter() - t


def cpu_baseline(A, B, target_s=10.0, workers=None):
    """The CPU oracle timed on the host's cores: `workers` processes (one per
    core, at most 16) each multiply and merge a disjoint block of rows of the
    same pair space; throughput is all their products over the wall time."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    mj = B["x"].shape[0]
    pa = (A["x"], A["z"], A["phase"], A["coef"])
    pb = (B["x"], B["z"], B["phase"], B["coef"])
    dt = _oracle_block(A["n"], pa, pb, 0, 2)
    rows = max(1, int(2 * target_s / max(dt, 1e-3)))
    rows = min(rows, A["x"].shape[0] // workers)
    ctx = mp.get_context("spawn")  # fresh interpreters: nothing of the GPU process is inherited
    with cf.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        list(ex.map(_oracle_block, [A["n"]] * workers, [pa] * workers, [pb] * workers,
                    [0] * workers, [1] * workers))  # the workers start and load the oracle
        t = time.perf_counter()
        futs = [ex.submit(_oracle_block, A["n"], pa, pb, w * rows, (w + 1) * rows)
                for w in range(workers)]
        for f in futs:
            f.result()
        wall = time.perf_counter() - t
    prods = workers * rows * mj
    return {"value": prods / wall, "unit": "products/s", "cores": workers, "kind": "oracle",
            "cpu": _cpu_model(),
            "sample": "%d processes, each a disjoint block of %d left terms times all %d right "
                      "terms of the same workload (%d products in all), multiply and exact merge, "
                      "%.1f s wall" % (workers, rows, mj, prods, wall)}


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


def _pair_err(torch, r, g, sel):
    if not bool(sel.any()):
        return 0.0
    return float(((g - r).abs()[sel] / r.abs()[sel]).max())


def _rel_err(pl, torch, GA, GB, tau, CA=None, CB=None, drop_rel=None):
    """Largest relative error of the precision form against plain FP64 on
    this GPU.  Both outputs hold the same strings in the same order (checked).
    Over every string with |c64| > 0 (which contains the set
    |c| > 1e-12 A(s)), or with drop_rel, over |c64| >= drop_rel max |c64|."""
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
    sel = mag > 0 if drop_rel is None else mag >= drop_rel * mag.max()
    err = _pair_err(torch, r, g, sel)
    del ref, got, r, g, mag, sel
    torch.cuda.empty_cache()
    return err


def _batched(pl, torch, args):
    """Batched form: the 256 products in calls of 32 (compensated,
    autotuned), as eager calls and as replays of one captured graph per call
    (plans), against the same products as single plain launches."""
    import numpy as np
    import synth
    plan = synth.workload4_plan()
    pairs = [synth.workload4_batch(b, n, m1, m2) for b, (n, m1, m2) in enumerate(plan)]
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    P = sum(m1 * m2 for _, m1, m2 in plan)
    chunk = 32
    chunks = [(c0, min(c0 + chunk, len(plan))) for c0 in range(0, len(plan), chunk)]
    _log("batched: %d products in %d pairs" % (P, len(plan)))

    def run_batched():
        U = 0
        for c0, c1 in chunks:
            outs = pl.outer_product_batched(GA[c0:c1], GB[c0:c1], mode=pl.COMPENSATED,
                                            tau=COMP_TAU)
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
    # graph replays: one plan per call of 32 (its buffers exist only while it
    # is timed), every step replaying all of them
    tg, tcap = 0.0, 0.0
    for c0, c1 in chunks:
        pl.trim_memory()
        t0 = time.perf_counter()
        plan_c = pl.BatchPlan(GA[c0:c1], GB[c0:c1], mode=pl.COMPENSATED, tau=COMP_TAU)
        torch.cuda.synchronize()
        tcap += time.perf_counter() - t0
        plan_c.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan_c.run()
        torch.cuda.synchronize()
        tg += (time.perf_counter() - t0) / args.steps
        plan_c.destroy()
    pl.trim_memory()
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
        "graph_replay": {"value": P / tg, "unit": "products/s", "ms_per_step": round(1e3 * tg, 3),
                         "plan_create_ms_total": round(1e3 * tcap, 1),
                         "note": "one captured HIP graph per call of 32, replayed"},
        "single_plain_launches": {"value": P / ts, "unit": "products/s",
                                  "ms_per_step": round(1e3 * ts, 3), "dtype": "f32"},
        "speedup_vs_single_launches": round(ts / tb, 3),
        "max_rel_err_vs_fp64": err,
        "err_definition": "max over every 16th pair of |c32 - c64| / |c64| over all strings with "
                          "|c64| > 0",
    }


def _common_rel_err(torch, a, b, drop_rel=1e-6):
    """Precision-form state b against FP64 state a: the largest relative
    error over the strings of a with |c| >= drop_rel max |c|, matched on
    their full words; such a string missing from b counts as error 1, and
    the strings present on one side only are counted."""
    import numpy as np
    ra = a["coef"]
    mag = ra.abs()
    big = mag >= drop_rel * mag.max()
    same = a["x"].shape == b["x"].shape and torch.equal(a["x"], b["x"]) and \
        torch.equal(a["z"], b["z"])
    if same:
        g = b["coef"].to(torch.complex128)
        return {"max_rel_err": _pair_err(torch, ra, g, big), "only_fp64": 0, "only_comp": 0,
                "only_fp64_above_floor": 0}
    fa, fb = a["fp"].cpu().numpy(), b["fp"].cpu().numpy()
    _, ia, ib = np.intersect1d(fa, fb, return_indices=True)
    ia_t = torch.from_numpy(ia).to(a["fp"].device)
    ib_t = torch.from_numpy(ib).to(b["fp"].device)
    eq = (a["x"][ia_t] == b["x"][ib_t]).all(1) & (a["z"][ia_t] == b["z"][ib_t]).all(1)
    ia_t, ib_t = ia_t[eq], ib_t[eq]
    inb = torch.zeros(fa.size, dtype=torch.bool, device=a["fp"].device)
    inb[ia_t] = True
    err = _pair_err(torch, ra[ia_t], b["coef"][ib_t].to(torch.complex128), big[ia_t])
    missing = int((big & ~inb).sum())
    return {"max_rel_err": 1.0 if missing else err, "only_fp64": int(fa.size - ia_t.numel()),
            "only_comp": int(fb.size - ib_t.numel()), "only_fp64_above_floor": missing}


def _propagation(pl, torch, args):
    """Propagation loop on the 1e6-term state: 64 conjugation steps (FP64
    and the precision form) and the first 8 literal product steps, each as
    the host-synchronised loop and as one captured HIP graph (plan)."""
    import synth
    S = synth.workload5_state()
    theta, px, pz = synth.workload5_rotations()
    G = pl.PauliSum.from_dict(S)
    drop = 1e-10
    res = {}

    def eager(name, rot, steps, mode):
        # a whole warm-up loop: the arena has grown to the loop's sizes
        pl.propagate(G, px[:steps], pz[:steps], theta[:steps], rotate_mode=rot, mode=mode,
                     drop_abs=drop, tau=COMP_TAU).destroy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = pl.propagate(G, px[:steps], pz[:steps], theta[:steps], rotate_mode=rot, mode=mode,
                           drop_abs=drop, tau=COMP_TAU)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[name] = {"steps": steps, "seconds": round(dt, 4), "final_terms": out.m,
                     "ms_per_step": round(1e3 * dt / steps, 3)}
        _log("%s: %.3f s for %d steps, %d terms" % (name, dt, steps, out.m))
        return out

    def graph(name, rot, steps, mode, cap):
        pl.trim_memory()
        t0 = time.perf_counter()
        plan = pl.PropagatePlan(G, px[:steps], pz[:steps], theta[:steps], max_terms=cap,
                                rotate_mode=rot, mode=mode, drop_abs=drop, tau=COMP_TAU)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        plan.run()
        plan.result().destroy()
        plan.run()  # new state blocks and a new capture, untimed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run()  # a replay of the captured loop
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out = plan.result()
        plan.destroy()
        res[name] = {"steps": steps, "seconds": round(dt, 4), "final_terms": out.m,
                     "ms_per_step": round(1e3 * dt / steps, 3), "max_terms": cap,
                     "plan_create_s": round(tc, 3),
                     "note": "one HIP graph launch for the whole loop, no host synchronisation "
                             "inside it"}
        _log("%s: %.3f s for %d steps (graph), %d terms" % (name, dt, steps, out.m))
        return out

    eager("conjugate_fp64", pl.ROTATE_CONJUGATE, 64, pl.PLAIN).destroy()
    eager("conjugate_compensated", pl.ROTATE_CONJUGATE, 64, pl.COMPENSATED).destroy()
    a = graph("conjugate_fp64_graph", pl.ROTATE_CONJUGATE, 64, pl.PLAIN, 100_000_000)
    pl.trim_memory()
    A64 = a.export_torch()
    a.destroy()
    b = graph("conjugate_compensated_graph", pl.ROTATE_CONJUGATE, 64, pl.COMPENSATED,
              100_000_000)
    pl.trim_memory()
    B32 = b.export_torch()
    b.destroy()
    cmp_err = _common_rel_err(torch, A64, B32)
    cmp_all = _common_rel_err(torch, A64, B32, drop_rel=0.0)
    del A64, B32
    torch.cuda.empty_cache()
    # literal steps: products = 2 * terms entering each step
    prods = 0
    cur = G
    for t in range(8):
        prods += 2 * cur.m
        nxt = pl.propagate(cur, px[t:t + 1], pz[t:t + 1], theta[t:t + 1],
                           rotate_mode=pl.ROTATE_PRODUCT, drop_abs=drop)
        if cur is not G:
            cur.destroy()
        cur = nxt
    cur.destroy()
    eager("product_fp64_8_steps", pl.ROTATE_PRODUCT, 8, pl.PLAIN).destroy()
    graph("product_fp64_8_steps_graph", pl.ROTATE_PRODUCT, 8, pl.PLAIN, 200_000_000).destroy()
    pl.trim_memory()
    lit = res["product_fp64_8_steps"]
    return {
        "metric": "Pauli products/s incl. sort-merge, propagation loop",
        "value": prods / lit["seconds"], "unit": "products/s", "n_gpus": 1, "steps": 8,
        "warmup": 1, "ms_per_step": lit["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[5], "products": prods, "merged_terms": lit["final_terms"]},
        "graph_value": prods / res["product_fp64_8_steps_graph"]["seconds"],
        "runs": res,
        "compensated_vs_fp64_after_64_steps": cmp_err,
        "compensated_vs_fp64_after_64_steps_all_strings": cmp_all,
        "err_definition": "graph loops: precision form against FP64, strings matched on their "
                          "full words; over |c64| >= 1e-6 max|c64| and over every string; a "
                          "string of the FP64 state missing from the precision form counts as "
                          "error 1",
    }


def _propagation_graph(pl, torch, args):
    """The 64-step conjugation loop as one graph launch, replayed `steps`
    times after one warm-up run (each run recomputes the whole loop from the
    input state)."""
    import synth
    S = synth.workload5_state()
    theta, px, pz = synth.workload5_rotations()
    G = pl.PauliSum.from_dict(S)
    plan = pl.PropagatePlan(G, px, pz, theta, max_terms=100_000_000, drop_abs=1e-10)
    plan.run()
    plan.result().destroy()
    plan.run()  # new state block and capture after the result
    torch.cuda.synchronize()
    _log("propagation graph: timed replays")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    out = plan.result()
    rec = {
        "metric": "64 conjugation steps per second as one graph launch",
        "value": 1.0 / dt, "unit": "loops/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(1e3 * dt, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded generators of the workload's shape)",
        "config": {"workload": WORKLOADS[9], "final_terms": out.m},
    }
    out.destroy()
    plan.destroy()
    return rec


def _hh(pl, torch, args):
    """The cancellation case: H*H with 20,000 Jordan-Wigner-shaped terms
    (4e8 products), FP64 and the precision form at tau = 0.3 and 1e-3,
    compared after dropping |c| < 1e-6 max |c| on both sides."""
    H = synth_workload3()
    G = pl.PauliSum.from_dict(H)
    P = H["x"].shape[0] ** 2
    e64, U, st64 = _timed(pl, torch, G, G, args.steps, args.warmup)
    e32, _, st32 = _timed(pl, torch, G, G, args.steps, args.warmup, mode=pl.COMPENSATED,
                          tau=COMP_TAU)
    rec = {
        "config": {"workload": WORKLOADS[3], "products": P, "merged_terms": U},
        "fp64": {"value": P * args.steps / e64, "unit": "products/s",
                 "ms_per_step": round(1e3 * e64 / args.steps, 3),
                 "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in st64.items()}},
        "compensated": {"value": P * args.steps / e32, "unit": "products/s",
                        "ms_per_step": round(1e3 * e32 / args.steps, 3), "tau": COMP_TAU,
                        "stages_ms_per_step": {k: round(v[0] / args.steps, 4)
                                               for k, v in st32.items()}},
    }
    for tau in (COMP_TAU, 1e-3):
        rec["compensated"]["max_rel_err_after_drop_tau_%g" % tau] = _rel_err(
            pl, torch, G, G, tau, drop_rel=1e-6)
    rec["compensated"]["max_rel_err_all_strings_tau_%g" % COMP_TAU] = _rel_err(
        pl, torch, G, G, COMP_TAU)
    rec["err_definition"] = ("max |c32 - c64| / |c64| over strings with |c64| >= 1e-6 max|c64| "
                             "(the workload's drop rule; the string sets are checked equal)")
    return rec


def synth_workload3():
    import synth
    return synth.workload3()


def _copy_ceiling(torch, nbytes=2 << 30, reps=5):
    """A device copy of nbytes (read + write), timed with HIP events on the
    current stream: the practical HBM ceiling of a streaming kernel."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"kernel": "torch copy_ of float32, 2 GiB read + 2 GiB written",
            "achieved_GBps": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "ms": round(ms, 3)}


def _stage_rooflines(stages, steps):
    """Achieved algorithmic GB/s of every stage of a profiled run (its HIP
    events on the launching stream), and its fraction of the 8 TB/s peak."""
    out = {}
    for k, (ms, launches, by) in stages.items():
        if ms <= 0 or by <= 0:
            continue
        gbs = by / (ms * 1e-3) / 1e9
        out[k] = {"achieved_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                  "algorithmic_bytes_per_step": by / steps, "ms_per_step": round(ms / steps, 4)}
    return out


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
    ap.add_argument("--quick", action="store_true",
                    help="the headline workload only (no sub-records of the other workloads)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes of the CPU baseline (0: one per core, at most 16)")
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
    if args.workload in (4, 5, 6, 7, 8, 9):
        rec = {4: _batched, 5: _propagation, 6: _commutator,
               7: _clifford, 8: _lex, 9: _propagation_graph}[args.workload](pl, torch, args)
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
        "stage_rooflines": _stage_rooflines(stages, args.steps),
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
            "err_definition": "max |c32 - c64| / |c64| over every string with |c64| > 0 (the "
                              "same strings on both sides, checked)",
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
    pl.trim_memory()
    rec["copy_ceiling"] = _copy_ceiling(torch)
    if args.workload == 2 and not args.quick:
        del GA, GB
        pl.trim_memory()
        _log("sub-record: H*H cancellation case")
        rec["hh_cancellation"] = _hh(pl, torch, args)
        pl.trim_memory()
        _log("sub-record: batched form")
        rec["batched"] = _batched(pl, torch, args)
        pl.trim_memory()
        _log("sub-record: propagation loop")
        rec["propagation"] = _propagation(pl, torch, args)
        pl.trim_memory()
    if not args.no_cpu_baseline:
        _log("timing the CPU oracle")
        rec["cpu_baseline"] = cpu_baseline(A, B, args.cpu_seconds, args.cpu_workers or None)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

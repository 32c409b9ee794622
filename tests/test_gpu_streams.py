"""Calls on a stream other than the one their inputs (or plans) were made
on, through the C ABI: the results equal those of the same calls on the
default stream, bit for bit.  Every call is ordered on the stream it is
given; plans made on one stream run on another after that stream's earlier
work and before its later work."""
import numpy as np
import pytest
import torch

import paper_2605_25974_amd as pl
import synth

pytestmark = pytest.mark.gpu


def _same(a, b):
    for k in ("x", "z", "phase", "fp"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["coef"].view(np.uint8), b["coef"].view(np.uint8))


def test_fused_and_general_calls_on_a_side_stream():
    A, B = synth.workload2(m1=300, m2=210)
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    ref = pl.outer_product_merged(GA, GB).export()
    ref_c = pl.outer_product_merged(GA, GB, mode=pl.COMPENSATED, tau=0.3).export()
    side = torch.cuda.Stream()
    h = side.cuda_stream
    g = pl.outer_product_merged(GA, GB, stream=h)
    c = pl.outer_product_merged(GA, GB, mode=pl.COMPENSATED, tau=0.3, stream=h)
    m = pl.merge(pl.outer_product(GA, GB, stream=h), stream=h)
    _same(g.export(stream=h), ref)
    _same(c.export(stream=h), ref_c)
    _same(m.export(stream=h), ref)


def test_plans_run_on_a_side_stream():
    pairs = [synth.workload4_batch(800 + b, n, m1, m2)
             for b, (n, m1, m2) in enumerate([(64, 150, 90), (500, 80, 120), (64, 40, 70)])]
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    eager = [o.export() for o in pl.outer_product_batched(GA, GB, mode=pl.COMPENSATED)]
    P = pl.BatchPlan(GA, GB, mode=pl.COMPENSATED)  # made on the default stream
    side = torch.cuda.Stream()
    h = side.cuda_stream
    for _ in range(2):
        P.run(stream=h)
        res = P.results(stream=h)
        for g, e in zip(res, eager):
            _same(g.export(stream=h), e)
    P.destroy()
    # a batched call made on the side stream (its plan lives on that stream)
    for g, e in zip(pl.outer_product_batched(GA, GB, mode=pl.COMPENSATED, stream=h), eager):
        _same(g.export(stream=h), e)
    # a propagation plan made on the default stream, run on the side stream
    S = synth.workload5_state(m=2000)
    th, x, z = synth.workload5_rotations(steps=5)
    G = pl.PauliSum.from_dict(S)
    ref = pl.propagate(G, x, z, th, drop_abs=1e-10).export()
    Q = pl.PropagatePlan(G, x, z, th, max_terms=2000 * 32, drop_abs=1e-10)
    Q.run(stream=h)
    _same(Q.result().export(stream=h), ref)
    Q.destroy()

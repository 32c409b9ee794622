"""Calls from several host threads at once, each on a stream of its own,
through the C ABI: every result equals, bit for bit, the same call made
alone on the default stream.  The library's host state (allocator arenas,
tune table, stage timers, error strings) is shared by the threads; the
device buffers of a call belong to that call."""
import concurrent.futures as cf

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


def test_concurrent_calls_from_threads():
    A, B = synth.workload2(m1=1500, m2=1200)
    C, D = synth.workload4_batch(910, 64, 900, 700)
    E = synth.workload5_state(m=3000)
    th, x, z = synth.workload5_rotations(steps=4)
    GA, GB, GC, GD, GE = (pl.PauliSum.from_dict(s) for s in (A, B, C, D, E))
    jobs = {
        "fused_fp64": lambda h: pl.outer_product_merged(GA, GB, stream=h),
        "fused_comp": lambda h: pl.outer_product_merged(GC, GD, mode=pl.COMPENSATED, tau=0.3,
                                                        stream=h),
        "general": lambda h: pl.merge(pl.outer_product(GC, GD, stream=h), stream=h),
        "batched": lambda h: pl.outer_product_batched([GA, GC], [GB, GD], stream=h)[1],
        "propagate": lambda h: pl.propagate(GE, x, z, th, drop_abs=1e-10, stream=h),
    }
    ref = {k: f(None).export() for k, f in jobs.items()}
    torch.cuda.synchronize()

    def run(name):
        s = torch.cuda.Stream()
        h = s.cuda_stream
        outs = []
        for _ in range(3):
            outs.append(jobs[name](h).export(stream=h))
        return name, outs

    with cf.ThreadPoolExecutor(len(jobs)) as ex:
        for name, outs in ex.map(run, list(jobs)):
            for o in outs:
                _same(o, ref[name])

"""Seeded random rotation loops (needs an MI355X): qubit counts on and
around word boundaries, small and empty states (some with repeated
strings), generators of any weight, both semantics, through the host loop
and a propagation plan, both against the CPU oracle.  The plan merges its
input before the first step, so its strings equal the host loop's, and its
coefficients equal them bit for bit when the input strings are distinct
(with repeated strings the first step sums in another order)."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _same(a, b):
    for k in ("x", "z", "phase", "fp"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["coef"].view(np.uint8), b["coef"].view(np.uint8))


def _case(k):
    rng = synth.rng_for(960, k)
    n = int(rng.choice([1, 2, 5, 63, 64, 65, 128, 300, 500]))
    m = int(rng.choice([0, 1, 9, 120, 700]))
    steps = int(rng.integers(1, 7))
    S = synth.random_sum(rng, n, m, wmax=min(n, 12))
    x, z = synth.random_weight(rng, n, steps, 1, min(n, 6))
    th = rng.uniform(0.0, np.pi, size=steps)
    rot = pl.ROTATE_CONJUGATE if rng.integers(0, 2) else pl.ROTATE_PRODUCT
    return S, x, z, th, rot


@pytest.mark.parametrize("mode", [pl.PLAIN, pl.COMPENSATED])
def test_random_rotation_loops(mode):
    for k in range(40):
        S, x, z, th, rot = _case(k + (1000 if mode == pl.COMPENSATED else 0))
        G = pl.PauliSum.from_dict(S)
        ref = O.propagate(_osum(S), x, z, th, mode=rot)
        eager = pl.propagate(G, x, z, th, rotate_mode=rot, mode=mode).export()
        cap = max(16, len(S["coef"]) * 2 ** len(th))
        P = pl.PropagatePlan(G, x, z, th, max_terms=cap, rotate_mode=rot, mode=mode)
        P.run()
        plan = P.result().export()
        P.destroy()
        for g in (eager, plan):
            if mode == pl.PLAIN:
                parity.assert_merged_fp64(g, ref)
            else:
                assert parity.max_rel_err(g, ref) <= 1e-6, k
            parity.assert_sorted_by_key(g)
        for key in ("x", "z", "phase", "fp"):
            assert np.array_equal(plan[key], eager[key]), (k, key)
        keys = parity.row_keys(S["x"], S["z"])
        if len(np.unique(keys)) == len(keys):
            _same(plan, eager)

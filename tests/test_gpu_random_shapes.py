"""Seeded random shapes through the fused call and the batched form at
once, against the CPU oracle (needs an MI355X): qubit counts on and around
word boundaries, empty and one-term sides, repeated strings, both
coefficient types, both merge modes and a drop threshold."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu

N_CHOICES = [1, 3, 17, 63, 64, 65, 127, 130, 200, 256, 257, 500, 511, 700]


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _side(rng, n, m, pool):
    """m terms at n qubits; with pool > 0 drawn from `pool` strings."""
    if pool and m:
        base = synth.random_sum(rng, n, pool)
        idx = rng.integers(0, pool, size=m)
        return {"n": n, "x": base["x"][idx], "z": base["z"][idx],
                "phase": rng.integers(0, 4, size=m).astype(np.uint8),
                "coef": rng.standard_normal(m) + 1j * rng.standard_normal(m)}
    return synth.random_sum(rng, n, m)


def _case(k):
    rng = synth.rng_for(950, k)
    n = int(rng.choice(N_CHOICES))
    sizes = [0, 1, 2, 37, 150, 333]
    m1, m2 = int(rng.choice(sizes)), int(rng.choice(sizes))
    pool = int(rng.choice([0, 0, 5, 40]))
    A, B = _side(rng, n, m1, pool), _side(rng, n, m2, pool)
    c64 = bool(rng.integers(0, 2))
    if c64:
        A["coef"] = A["coef"].astype(np.complex64)
        B["coef"] = B["coef"].astype(np.complex64)
    return A, B, c64


def _check(g, ref, mode, c64):
    if mode == pl.COMPENSATED:
        parity.assert_compensated(g, ref, input_rounding=not c64)
    elif not c64:
        parity.assert_merged_fp64(g, ref)
    else:  # FP32 products and sums
        gi, ri = parity.align(g["x"], g["z"], ref.x, ref.z)
        err = np.abs(g["coef"][gi].astype(np.complex128) - ref.coef[ri])
        assert np.all(err <= 1e-5 * np.maximum(ref.mass[ri], 1e-30))
    parity.assert_sorted_by_key(g)


@pytest.mark.parametrize("mode", [pl.PLAIN, pl.COMPENSATED])
def test_random_shapes_fused_and_batched(mode):
    cases = [_case(k + (1000 if mode == pl.COMPENSATED else 0)) for k in range(48)]
    GA = [pl.PauliSum.from_dict(A) for A, _, _ in cases]
    GB = [pl.PauliSum.from_dict(B) for _, B, _ in cases]
    refs = [O.product_merge(_osum(A), _osum(B)) for A, B, _ in cases]
    batched = pl.outer_product_batched(GA, GB, mode=mode, tau=0.3)
    for (A, B, c64), ga, gb, ref, ob in zip(cases, GA, GB, refs, batched):
        single = pl.outer_product_merged(ga, gb, mode=mode, tau=0.3).export()
        _check(single, ref, mode, c64)
        got = ob.export()
        _check(got, ref, mode, c64)
        for key in ("x", "z", "fp"):
            assert np.array_equal(got[key], single[key])


def test_random_shapes_drop():
    """A drop threshold between neighbouring merged moduli: the fused and
    the batched results keep exactly the oracle's strings."""
    cases = [_case(2000 + k) for k in range(32)]
    cases = [(A, B, c64) for A, B, c64 in cases if not c64]  # FP64 values decide the drop
    GA = [pl.PauliSum.from_dict(A) for A, _, _ in cases]
    GB = [pl.PauliSum.from_dict(B) for _, B, _ in cases]
    full = [O.product_merge(_osum(A), _osum(B)) for A, B, _ in cases]
    mods = np.unique(np.concatenate([np.abs(f.coef) for f in full] + [np.zeros(1)]))
    mods = mods[mods > 0]
    if len(mods) < 2:
        pytest.skip("no merged terms to threshold")
    k = len(mods) // 3
    t = float(0.5 * (mods[k - 1] + mods[k])) if k >= 1 else float(mods[0] * 0.5)
    batched = pl.outer_product_batched(GA, GB, drop_abs=t)
    for (A, B, _), ga, gb, f, ob in zip(cases, GA, GB, full, batched):
        keep = np.abs(f.coef) >= t
        for g in (pl.outer_product_merged(ga, gb, drop_abs=t).export(), ob.export()):
            gi, ri = parity.align(g["x"], g["z"], f.x[keep], f.z[keep])
            assert np.all(np.abs(g["coef"][gi] - f.coef[keep][ri])
                          <= np.maximum(1e-12 * np.abs(f.coef[keep][ri]),
                                        1e-14 * np.maximum(1.0, f.mass[keep][ri])))

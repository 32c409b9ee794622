"""Clifford gates on the device sum (pauli_apply_clifford) against the CPU
oracle, through the C ABI (needs an MI355X).  Strings, phases and
coefficients must agree bit for bit, and the fingerprint must be that of the
new string."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import clifford as C
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _gates(seed, n, count):
    rng = synth.rng_for(960, seed)
    out = []
    for _ in range(count):
        kind = int(rng.integers(0, 9)) if n > 1 else int(rng.integers(0, 6))
        if kind in C.TWO_QUBIT:
            q0, q1 = rng.choice(n, size=2, replace=False)
            out.append((kind, int(q0), int(q1)))
        else:
            out.append((kind, int(rng.integers(0, n))))
    return out


def _check(g, x, z, ph, c):
    assert np.array_equal(g["x"], x) and np.array_equal(g["z"], z)
    assert np.array_equal(g["phase"], ph)
    assert np.array_equal(g["coef"].view(np.uint64), c.astype(g["coef"].dtype).view(np.uint64))
    assert np.array_equal(g["fp"], parity.fingerprint(g["x"], g["z"]))


@pytest.mark.parametrize("n,m,ngates", [(1, 50, 20), (5, 300, 60), (64, 500, 120), (100, 400, 57),
                                        (500, 700, 150), (1000, 200, 90)])
def test_clifford_parity(n, m, ngates):
    d = synth.random_sum(synth.rng_for(961, n), n, m, distinct_strings=False)
    gates = _gates(n, n, ngates)
    g = pl.apply_clifford(pl.PauliSum.from_dict(d), gates).export()
    _check(g, *C.apply(_osum(d), gates))


def test_clifford_no_gates_and_c64():
    d = synth.random_sum(synth.rng_for(962), 40, 100)
    g = pl.apply_clifford(pl.PauliSum.from_dict(d), []).export()
    _check(g, d["x"], d["z"], d["phase"], d["coef"])
    d64 = dict(d)
    d64["coef"] = d["coef"].astype(np.complex64)
    gates = _gates(3, 40, 70)
    g = pl.apply_clifford(pl.PauliSum.from_dict(d64), gates).export()
    x, z, ph, c = C.apply(_osum(d), gates)
    assert g["coef"].dtype == np.complex64
    _check(g, x, z, ph, d64["coef"])


def test_clifford_on_fused_output_then_merge():
    """The output of the fused product (leading dimension rounded up) through
    a circuit, then merged: equals the oracle's merge of the oracle's
    circuit output (the updated fingerprints order the merge)."""
    A, B = synth.workload2(m1=120, m2=90)
    prod = pl.outer_product_merged(pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B))
    e = prod.export()
    gates = _gates(4, 500, 80)
    g = pl.merge(pl.apply_clifford(prod, gates)).export()
    x, z, ph, c = C.apply(O.Sum(500, e["x"], e["z"], e["phase"], e["coef"]), gates)
    ref = O.merge(O.Sum(500, x, z, ph, c))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


def test_clifford_invalid_gates():
    s = pl.PauliSum.from_dict(synth.random_sum(synth.rng_for(963), 10, 5))
    for bad in ([(9, 0)], [(0, 10)], [(0, -1)], [(6, 3, 3)], [(7, 2, 10)]):
        with pytest.raises(pl.PauliError) as e:
            pl.apply_clifford(s, bad)
        assert e.value.status == "INVALID"


def test_clifford_fullsize_sampled():
    """1e6 terms at n=500 through 100 gates (the launch configuration the
    benchmark times); 3,000 sampled terms recomputed by the oracle."""
    d = synth.workload5_state()
    gates = _gates(5, 500, 100)
    g = pl.apply_clifford(pl.PauliSum.from_dict(d), gates).export()
    idx = synth.rng_for(965).choice(d["x"].shape[0], size=3000, replace=False)
    x, z, ph, c = C.apply(_osum(d), gates, terms=idx)
    assert np.array_equal(g["x"][idx], x) and np.array_equal(g["z"][idx], z)
    assert np.array_equal(g["phase"][idx], ph)
    assert np.array_equal(g["coef"][idx], c)
    assert np.array_equal(g["fp"][idx], parity.fingerprint(x, z))

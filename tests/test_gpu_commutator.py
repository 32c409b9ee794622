"""The commutator [a, b] = a*b - b*a (pauli_commutator) against the CPU
oracle, through the C ABI (needs an MI355X)."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _gsum(d):
    return pl.PauliSum.from_dict(d)


def _dup_sum(seed, n, m, pool):
    """m terms drawn from a pool of `pool` strings (repeated strings),
    random phases and complex coefficients."""
    rng = synth.rng_for(940, seed)
    base = synth.random_sum(rng, n, pool)
    idx = rng.integers(0, pool, size=m)
    return {"n": n, "x": base["x"][idx], "z": base["z"][idx],
            "phase": rng.integers(0, 4, size=m).astype(np.uint8),
            "coef": rng.standard_normal(m) + 1j * rng.standard_normal(m)}


@pytest.mark.parametrize("n,m1,m2", [(1, 30, 20), (5, 400, 300), (64, 700, 650), (100, 900, 800),
                                     (500, 1000, 800), (1000, 300, 250)])
def test_commutator_parity(n, m1, m2):
    A, B = _dup_sum(n, n, m1, max(2, m1 * 3 // 4)), _dup_sum(n + 7, n, m2, max(2, m2 // 2))
    g = pl.commutator(_gsum(A), _gsum(B)).export()
    ref = O.commutator(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


def test_commutator_workload_shape():
    """Jordan-Wigner-shaped sums at n=500 (the metric workload's shape)."""
    A, B = synth.workload2(m1=600, m2=500)
    g = pl.commutator(_gsum(A), _gsum(B)).export()
    ref = O.commutator(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


@pytest.mark.parametrize("key_bits", [4, 12])
def test_commutator_fingerprint_collisions(key_bits):
    """Truncated keys force collisions: the call falls back to merging the
    materialised anticommuting products and gives the same result."""
    A, B = _dup_sum(41, 40, 300, 250), _dup_sum(42, 40, 280, 200)
    g = pl.commutator(_gsum(A), _gsum(B), key_bits=key_bits).export()
    ref = O.commutator(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)


def test_commutator_compensated():
    A, B = _dup_sum(51, 200, 700, 600), _dup_sum(52, 200, 650, 500)
    g = pl.commutator(_gsum(A), _gsum(B), mode=pl.COMPENSATED, tau=0.3).export()
    ref = O.commutator(_osum(A), _osum(B))
    parity.assert_compensated(g, ref)


def test_self_commutator_is_exactly_zero():
    """[a, a]: the strings of anticommuting pairs of a, every coefficient 0
    (to the FP64 tolerance)."""
    A = _dup_sum(61, 30, 500, 400)
    G = _gsum(A)
    g = pl.commutator(G, G).export()
    ref = O.commutator(_osum(A), _osum(A))
    assert ref.x.shape[0] > 0 and np.all(ref.coef == 0)
    # (i, j) and (j, i) cancel pair by pair; summed in another order a
    # string given by several pairs may keep a rounding residue
    parity.assert_merged_fp64(g, ref)


def test_commutator_drop_and_empty():
    A, B = _dup_sum(71, 20, 300, 200), _dup_sum(72, 20, 300, 200)
    ref = O.commutator(_osum(A), _osum(B), drop_abs=0.5)
    g = pl.commutator(_gsum(A), _gsum(B), drop_abs=0.5).export()
    parity.assert_merged_fp64(g, ref)
    E = {"n": 20, "x": np.zeros((0, 1), np.uint64), "z": np.zeros((0, 1), np.uint64),
         "phase": np.zeros(0, np.uint8), "coef": np.zeros(0, np.complex128)}
    assert pl.commutator(_gsum(A), _gsum(E)).m == 0
    assert pl.commutator(_gsum(E), _gsum(B)).m == 0


def test_commutator_commuting_sums_is_empty():
    """Z-only sums commute term by term: the commutator has no terms."""
    rng = synth.rng_for(941)
    n, m = 90, 300
    W = (n + 63) // 64
    z = rng.integers(0, 2 ** 63, size=(m, W), dtype=np.uint64)
    z[:, -1] &= np.uint64((1 << (n - 64 * (W - 1))) - 1)
    A = {"n": n, "x": np.zeros_like(z), "z": z, "phase": np.zeros(m, np.uint8),
         "coef": rng.standard_normal(m) + 0j}
    assert pl.commutator(_gsum(A), _gsum(A)).m == 0

"""Lexicographic order on the device (pauli_sort_lex) against the CPU oracle,
through the C ABI (needs an MI355X).  The output is a permutation of the
input, so strings, phases, coefficients and fingerprints must agree bit for
bit with the oracle's stable order."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import lexorder as L
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _with_duplicates(rng, n, m):
    d = synth.random_sum(rng, n, m, distinct_strings=False)
    k = max(1, m // 5)
    src = rng.integers(0, m, size=k)
    dst = rng.integers(0, m, size=k)
    d["x"][dst] = d["x"][src]
    d["z"][dst] = d["z"][src]
    return d


def _ref(d):
    """The oracle's order of the input d, with the fingerprints computed on
    the test side."""
    return L.sort_lex(dict(d, fp=parity.fingerprint(d["x"], d["z"])))


def _exact(g, ref):
    for k in ("x", "z", "phase", "fp"):
        assert np.array_equal(g[k], ref[k]), k
    assert np.array_equal(g["coef"].view(np.uint64), ref["coef"].view(np.uint64))


def _keys_in_order(x, z):
    """(m, 2W) key columns, most significant first."""
    return np.concatenate([x[:, ::-1], z[:, ::-1]], axis=1)


def _assert_nondecreasing(x, z):
    K = _keys_in_order(x, z)
    if K.shape[0] < 2:
        return
    a, b = K[:-1], K[1:]
    diff = a != b
    first = np.argmax(diff, axis=1)
    rows = np.arange(a.shape[0])
    ok = ~diff.any(axis=1) | (a[rows, first] < b[rows, first])
    assert ok.all(), "out of order at %s" % np.nonzero(~ok)[0][:5]


@pytest.mark.parametrize("n,m", [(1, 40), (5, 3000), (31, 5000), (32, 9000), (33, 4097),
                                 (64, 8193), (65, 12000), (130, 6000), (500, 20000),
                                 (1000, 3000)])
def test_lex_parity(n, m):
    d = _with_duplicates(synth.rng_for(970, n), n, m)
    g = pl.sort_lex(pl.PauliSum.from_dict(d)).export()
    _exact(g, _ref(d))
    _assert_nondecreasing(g["x"], g["z"])


def test_lex_empty_single_and_c64():
    for m in (0, 1):
        d = synth.random_sum(synth.rng_for(971, m), 70, m, distinct_strings=False)
        _exact(pl.sort_lex(pl.PauliSum.from_dict(d)).export(), _ref(d))
    d = _with_duplicates(synth.rng_for(972), 200, 7000)
    d["coef"] = d["coef"].astype(np.complex64)
    g = pl.sort_lex(pl.PauliSum.from_dict(d)).export()
    assert g["coef"].dtype == np.complex64
    _exact(g, _ref(d))


def test_lex_constant_words_and_all_equal():
    """Words (and digits) that never vary are skipped: a sum whose strings
    differ in one bit only, and a sum of one repeated string (the identity
    permutation)."""
    n, m = 300, 5000
    rng = synth.rng_for(973)
    x = np.zeros((m, 5), np.uint64)
    z = np.zeros((m, 5), np.uint64)
    x[:, 2] = np.uint64(1) << np.uint64(17)
    z[:, 4] = (rng.integers(0, 2, size=m).astype(np.uint64) << np.uint64(40))
    d = synth.make_sum(n, x, z, rng.standard_normal(m) + 1j * rng.standard_normal(m),
                       rng.integers(0, 4, size=m).astype(np.uint8))
    _exact(pl.sort_lex(pl.PauliSum.from_dict(d)).export(), _ref(d))
    z[:, 4] = 0
    d = synth.make_sum(n, x, z, d["coef"], d["phase"])
    g = pl.sort_lex(pl.PauliSum.from_dict(d)).export()
    _exact(g, _ref(d))
    assert np.array_equal(g["coef"], d["coef"])  # the identity permutation


@pytest.mark.parametrize("n", [20, 130])
def test_lex_of_merged_product(n):
    """Lexicographic order of a fused product (which comes out in fingerprint
    order): the same strings and coefficients as the oracle's merged product
    in its lexicographic order."""
    rng = synth.rng_for(974, n)
    a = synth.random_sum(rng, n, 150)
    b = synth.random_sum(rng, n, 170)
    g = pl.sort_lex(pl.outer_product_merged(pl.PauliSum.from_dict(a),
                                            pl.PauliSum.from_dict(b))).export()
    ref = O.product_merge(O.Sum(n, a["x"], a["z"], a["phase"], a["coef"]),
                          O.Sum(n, b["x"], b["z"], b["phase"], b["coef"]))
    p = L.order(ref.x, ref.z)
    assert np.array_equal(g["x"], ref.x[p]) and np.array_equal(g["z"], ref.z[p])
    parity.assert_merged_fp64(g, ref)


def test_lex_propagation_state_full_size():
    """The 1e6-term, 500-qubit propagation state: full comparison with the
    oracle order."""
    d = synth.workload5_state()
    g = pl.sort_lex(pl.PauliSum.from_dict(d)).export()
    _exact(g, _ref(d))


@pytest.mark.parametrize("n,where", [(200, "x"), (100, "z"), (40, "x"), (300, "x2")])
def test_lex_runs_of_equal_top_words(n, where):
    """Strings whose most significant varying word takes a handful of values,
    so that the words below decide the order inside long runs: the runs are
    ordered on their lower words (with repeats of whole strings among them).
    "x2": the two top X words both take few values."""
    rng = synth.rng_for(975, n)
    W = (n + 63) // 64
    m = 20000
    d = synth.random_sum(rng, n, m, distinct_strings=False)
    top_bits = n - 64 * (W - 1)
    few = np.array([0, 1, 3, 1 << (top_bits - 1)], np.uint64)
    if where == "z":
        d["x"][:] = 0
        d["z"][:, W - 1] = rng.choice(few, size=m)
    else:
        d["x"][:, W - 1] = rng.choice(few, size=m)
        if where == "x2":
            d["x"][:, W - 2] = rng.choice(np.array([7, 1 << 63], np.uint64), size=m)
    k = m // 5
    src, dst = rng.integers(0, m, size=k), rng.integers(0, m, size=k)
    d["x"][dst] = d["x"][src]
    d["z"][dst] = d["z"][src]
    g = pl.sort_lex(pl.PauliSum.from_dict(d)).export()
    _exact(g, _ref(d))
    _assert_nondecreasing(g["x"], g["z"])


def _ranges(rng, n, m):
    """Z on one random range of qubits (sometimes reaching qubit 0 or the
    last qubit), X on at most two qubits."""
    W = (n + 63) // 64
    bits_z = np.zeros((m, n), bool)
    bits_x = np.zeros((m, n), bool)
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n + 1, size=m)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    lo[rng.random(m) < 0.2] = 0
    hi[rng.random(m) < 0.2] = n
    q = np.arange(n)
    bits_z[:] = (q[None, :] >= lo[:, None]) & (q[None, :] < hi[:, None])
    for _ in range(2):
        sel = rng.random(m) < 0.5
        bits_x[np.nonzero(sel)[0], rng.integers(0, n, size=int(sel.sum()))] = True
    pack = lambda B: np.packbits(np.pad(B, ((0, 0), (0, 64 * W - n))).reshape(m, W, 64)[:, :, ::-1],
                                 axis=2, bitorder="big").view(">u8").reshape(m, W).astype(np.uint64)
    return pack(bits_x), pack(bits_z)


@pytest.mark.parametrize("n,kind", [(70, "jw"), (130, "jw"), (500, "jw"), (200, "sparse"),
                                    (300, "ranges"), (64, "ranges"), (1000, "ranges")])
def test_lex_strings_with_few_transitions(n, kind):
    """Strings with few bit transitions, which are put in order on their
    transition codes: Jordan-Wigner-shaped strings, strings of weight <= 3,
    and Z ranges with X on a qubit or two.  Full comparison with the oracle's
    stable order (repeats of whole strings included), in complex128 and in
    complex64."""
    rng = synth.rng_for(976, n)
    m = 20000
    if kind == "jw":
        x, z = synth.jordan_wigner(rng, n, m)
    elif kind == "sparse":
        d = synth.random_sum(rng, n, m, wmax=3, distinct_strings=False)
        x, z = d["x"], d["z"]
    else:
        x, z = _ranges(rng, n, m)
    k = m // 10
    src, dst = rng.integers(0, m, size=k), rng.integers(0, m, size=k)
    x[dst] = x[src]
    z[dst] = z[src]
    c = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    d = synth.make_sum(n, x, z, c, rng.integers(0, 4, size=m).astype(np.uint8))
    g = pl.sort_lex(pl.PauliSum.from_dict(d)).export()
    _exact(g, _ref(d))
    _assert_nondecreasing(g["x"], g["z"])
    d["coef"] = d["coef"].astype(np.complex64)
    _exact(pl.sort_lex(pl.PauliSum.from_dict(d)).export(), _ref(d))

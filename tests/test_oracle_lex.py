"""Pins of the lexicographic-order oracle (no GPU).

The oracle sorts with numpy's lexsort; these tests check its result by other
routes: a word-by-word comparison loop on Python integers, the multiset of
rows, stability of equal strings, and for n <= 32 the order of the single
integer x * 2^32 + z."""
import numpy as np
import pytest

from oracle import lexorder as L
import synth


def _key(x_row, z_row):
    """The comparison key of one string as a tuple of Python integers:
    X words from the most significant down, then Z words likewise."""
    W = len(x_row)
    return tuple(int(x_row[w]) for w in reversed(range(W))) + \
        tuple(int(z_row[w]) for w in reversed(range(W)))


def _less_equal(a, b):
    """Word-by-word comparison of two keys, written as a loop."""
    for u, v in zip(a, b):
        if u != v:
            return u < v
    return True


def _with_duplicates(rng, n, m):
    d = synth.random_sum(rng, n, m, distinct_strings=False)
    # repeat some strings so that stability is exercised
    k = max(1, m // 4)
    src = rng.integers(0, m, size=k)
    dst = rng.integers(0, m, size=k)
    d["x"][dst] = d["x"][src]
    d["z"][dst] = d["z"][src]
    return d


@pytest.mark.parametrize("n", [1, 2, 5, 31, 32, 33, 64, 65, 130, 500])
def test_sorted_permutation_and_stable(n):
    rng = synth.rng_for(7100, n)
    d = _with_duplicates(rng, n, 300)
    p = L.order(d["x"], d["z"])
    assert sorted(p.tolist()) == list(range(300))  # a permutation
    keys = [_key(d["x"][i], d["z"][i]) for i in p]
    for a, b in zip(keys, keys[1:]):
        assert _less_equal(a, b)
    for i in range(1, len(p)):  # equal strings keep their input order
        if keys[i] == keys[i - 1]:
            assert p[i] > p[i - 1]


@pytest.mark.parametrize("n", [1, 7, 16, 32])
def test_small_n_is_integer_order(n):
    """For n <= 32 the order is that of the integer x * 2^32 + z."""
    rng = synth.rng_for(7101, n)
    d = _with_duplicates(rng, n, 200)
    v = (d["x"][:, 0].astype(np.uint64) << np.uint64(32)) | d["z"][:, 0].astype(np.uint64)
    ref = np.argsort(v, kind="stable")
    assert np.array_equal(L.order(d["x"], d["z"]), ref)


def test_single_qubit_letters():
    """Table I encodings (x, z): I = (0,0), Z = (0,1), X = (1,0), Y = (1,1);
    the X bit is compared first, so the order is I, Z, X, Y."""
    x = np.array([[1], [0], [1], [0]], np.uint64)  # X, Z, Y, I
    z = np.array([[0], [1], [1], [0]], np.uint64)
    assert L.order(x, z).tolist() == [3, 1, 0, 2]


def test_sort_lex_carries_the_term_data():
    rng = synth.rng_for(7102, 0)
    d = _with_duplicates(rng, 70, 50)
    d["fp"] = rng.integers(0, 2 ** 63, size=50, dtype=np.int64).astype(np.uint64)
    s = L.sort_lex(d)
    p = L.order(d["x"], d["z"])
    for k in ("x", "z", "phase", "coef", "fp"):
        assert np.array_equal(s[k], d[k][p])
    assert s["n"] == 70


def test_empty_and_single():
    x = np.zeros((0, 2), np.uint64)
    assert L.order(x, x).size == 0
    x1 = np.array([[5, 9]], np.uint64)
    assert L.order(x1, x1).tolist() == [0]

"""Pins of the oracle's commutator [H1, H2] = H1*H2 - H2*H1 (no GPU).

The commutator keeps one term per string that an anticommuting pair gives
(Section III-A: P Q = -Q P exactly when the strings anticommute).  It is
pinned against dense matrices, against the algebraic identities every
commutator obeys, and against a planted table mistake."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import dense_string, dense_sum, unpack
import synth


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _rand(seed, n, m, distinct=False):
    return _osum(synth.random_sum(synth.rng_for(930, seed), n, m, distinct_strings=distinct))


def _dense(r: O.Merged):
    return dense_sum(r.n, r.x, r.z, np.zeros(r.x.shape[0], np.uint8), r.coef)


def _as_dict(r: O.Merged):
    return {(r.x[u].tobytes(), r.z[u].tobytes()): r.coef[u] for u in range(r.x.shape[0])}


@pytest.fixture(autouse=True)
def _clean_table():
    O.table_reset()
    yield
    O.table_reset()


@pytest.mark.parametrize("n,m1,m2", [(1, 3, 4), (2, 7, 5), (3, 12, 9), (4, 16, 14)])
def test_commutator_against_dense(n, m1, m2):
    """dense(H1) dense(H2) - dense(H2) dense(H1) equals the dense matrix of
    the oracle's commutator; every string it lists comes from an
    anticommuting pair, and every Pauli component of the dense commutator
    is present."""
    A, B = _rand(n, n, m1), _rand(100 + n, n, m2)
    dA = dense_sum(n, A.x, A.z, A.phase, A.coef)
    dB = dense_sum(n, B.x, B.z, B.phase, B.coef)
    ref = dA @ dB - dB @ dA
    r = O.commutator(A, B)
    np.testing.assert_allclose(_dense(r), ref, atol=1e-12)
    # Pauli components of the dense commutator, tr(P^dagger M) / 2^n
    listed = set(_as_dict(r))
    for u in range(r.x.shape[0]):
        s = unpack(n, r.x[u], r.z[u])
        comp = np.trace(dense_string(s).conj().T @ ref) / 2 ** n
        assert abs(comp - r.coef[u]) <= 1e-12
    for x in range(2 ** n):
        for z in range(2 ** n):
            xs, zs = np.array([x], np.uint64), np.array([z], np.uint64)
            s = unpack(n, xs, zs)
            comp = np.trace(dense_string(s).conj().T @ ref) / 2 ** n
            if abs(comp) > 1e-9:
                assert (xs.tobytes(), zs.tobytes()) in listed, s


def test_antisymmetry_and_self_commutator():
    """[B, A] = -[A, B] term by term (the same strings); [A, A] lists only
    strings of anticommuting pairs, all with coefficient exactly zero."""
    A, B = _rand(1, 9, 40), _rand(2, 9, 35)
    ab, ba = _as_dict(O.commutator(A, B)), _as_dict(O.commutator(B, A))
    assert ab.keys() == ba.keys()
    for k, v in ab.items():
        assert ba[k] == -v
    aa = O.commutator(A, A)
    assert aa.x.shape[0] > 0
    assert np.all(aa.coef == 0)


def test_only_anticommuting_pairs_contribute():
    """A sum of mutually commuting strings (Z-only) has no commutator with
    another Z-only sum; with X on a qubit each pair anticommutes exactly when
    the Z sum acts on that qubit."""
    rng = synth.rng_for(931)
    n = 5
    zs = np.unique(rng.integers(1, 2 ** n, size=12)).astype(np.uint64).reshape(-1, 1)
    Zsum = O.Sum(n, np.zeros_like(zs), zs, None, rng.standard_normal(zs.shape[0]) + 0j)
    Z2 = O.Sum(n, np.zeros_like(zs[:5]), zs[:5][::-1].copy(), None, np.ones(5, complex))
    assert O.commutator(Zsum, Z2).x.shape[0] == 0
    X0 = O.Sum(n, np.array([[1]], np.uint64), np.array([[0]], np.uint64), None, np.array([1.0 + 0j]))
    r = O.commutator(X0, Zsum)
    expect = int(np.sum((zs[:, 0] & 1) == 1))
    assert r.x.shape[0] == expect
    # X Z = -i Y on qubit 0: [X, c Z..] = 2 c X Z.. = -2i c (Y on qubit 0)
    for u in range(r.x.shape[0]):
        t = int(np.nonzero(zs[:, 0] == r.z[u, 0])[0][0])
        assert r.x[u, 0] == 1 and r.coef[u] == -2j * Zsum.coef[t]


def test_jacobi_identity_integer_coefficients():
    """[A,[B,C]] + [B,[C,A]] + [C,[A,B]] = 0, exactly for small-integer
    coefficients (every partial sum is exact)."""
    rng = synth.rng_for(932)
    n = 4

    def intsum(seed, m):
        d = synth.random_sum(synth.rng_for(933, seed), n, m)
        d["coef"] = (rng.integers(-3, 4, m) + 1j * rng.integers(-3, 4, m)).astype(complex)
        return _osum(d)

    def as_sum(r):
        return O.Sum(n, r.x, r.z, None, r.coef)

    A, B, C = intsum(1, 6), intsum(2, 5), intsum(3, 7)
    parts = [O.commutator(A, as_sum(O.commutator(B, C))),
             O.commutator(B, as_sum(O.commutator(C, A))),
             O.commutator(C, as_sum(O.commutator(A, B)))]
    x = np.concatenate([p.x for p in parts])
    z = np.concatenate([p.z for p in parts])
    c = np.concatenate([p.coef for p in parts])
    total = O.merge(O.Sum(n, x, z, None, c))
    assert np.all(total.coef == 0)


def test_planted_table_mistake_is_caught():
    """A wrong phase in the single-qubit table (X*Y = -iZ) breaks the dense
    check of the commutator."""
    O.table_set(1, 2, 3, 3)
    with pytest.raises(AssertionError):
        test_commutator_against_dense(2, 7, 5)
    O.table_reset()
    test_commutator_against_dense(2, 7, 5)

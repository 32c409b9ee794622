"""Pins of the Clifford oracle (no GPU): whole-string conjugation by the
dense circuit matrix, inverse circuits, and the Pauli-gate sign rule."""
import numpy as np
import pytest

from oracle import clifford as C
from oracle import oracle as O
from tests.helpers import dense_sum
import synth


def _dense_gate(n, kind, q0, q1=None):
    """The gate's 2^n x 2^n matrix, built from its action on basis states
    (qubit 0 is the first tensor factor, as in the dense strings)."""
    U = C._unitary(kind)
    D = np.zeros((2 ** n, 2 ** n), complex)
    qs = [q0] if kind not in C.TWO_QUBIT else [q0, q1]
    k = len(qs)
    for col in range(2 ** n):
        bits = [(col >> (n - 1 - q)) & 1 for q in range(n)]
        loc = 0
        for q in qs:
            loc = loc * 2 + bits[q]
        for out_loc in range(2 ** k):
            amp = U[out_loc, loc]
            if amp == 0:
                continue
            nb = list(bits)
            for i, q in enumerate(qs):
                nb[q] = (out_loc >> (k - 1 - i)) & 1
            row = 0
            for b in nb:
                row = row * 2 + b
            D[row, col] += amp
    return D


def _random_gates(rng, n, count):
    gates = []
    for _ in range(count):
        kind = int(rng.integers(0, 9))
        if kind in C.TWO_QUBIT:
            q0, q1 = rng.choice(n, size=2, replace=False)
            gates.append((kind, int(q0), int(q1)))
        else:
            gates.append((kind, int(rng.integers(0, n))))
    return gates


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_clifford_against_dense_circuit(n):
    """Every term: dense(C) dense(term) dense(C)^dagger equals the dense
    matrix of the oracle's output term, for random circuits of all kinds."""
    rng = synth.rng_for(950, n)
    for trial in range(6):
        d = synth.random_sum(rng, n, 12, distinct_strings=False)
        s = O.Sum(n, d["x"], d["z"], d["phase"], d["coef"])
        gates = _random_gates(rng, n, 10) if n > 1 else \
            [(int(rng.integers(0, 6)), 0) for _ in range(10)]
        U = np.eye(2 ** n, dtype=complex)
        for g in gates:
            U = _dense_gate(n, *g) @ U
        x, z, ph, c = C.apply(s, gates)
        for t in range(s.m):
            before = dense_sum(n, s.x[t:t + 1], s.z[t:t + 1], s.phase[t:t + 1], s.coef[t:t + 1])
            after = dense_sum(n, x[t:t + 1], z[t:t + 1], ph[t:t + 1], c[t:t + 1])
            np.testing.assert_allclose(U @ before @ U.conj().T, after, atol=1e-12)


def test_inverse_circuit_restores_terms():
    """H, X, Y, Z, CX, CZ and SWAP are their own inverses and S^dagger undoes
    S: a circuit followed by its inverse returns every term, phase included."""
    rng = synth.rng_for(951)
    n = 70
    d = synth.random_sum(rng, n, 40)
    s = O.Sum(n, d["x"], d["z"], d["phase"], d["coef"])
    gates = _random_gates(rng, n, 30)
    inv = {C.S: C.SDG, C.SDG: C.S}
    back = [(inv.get(g[0], g[0]),) + tuple(g[1:]) for g in reversed(gates)]
    x, z, ph, c = C.apply(s, gates)
    x2, z2, ph2, c2 = C.apply(O.Sum(n, x, z, ph, c), back)
    assert np.array_equal(x2, s.x) and np.array_equal(z2, s.z) and np.array_equal(ph2, s.phase)
    assert not (np.array_equal(x, s.x) and np.array_equal(z, s.z))


def test_pauli_gate_sign_rule():
    """Conjugation by a Pauli gate P keeps the string and flips its sign
    exactly when the letter on that qubit anticommutes with P (Section III-B,
    theta = pi case)."""
    n = 3
    letters = ["IXY", "ZZZ", "YIX"]
    for kind, L in ((C.X, 1), (C.Y, 2), (C.Z, 3)):
        for s_ in letters:
            x, z = C._encode(n, ["IXYZ".index(ch) for ch in s_])
            s = O.Sum(n, x.reshape(1, -1), z.reshape(1, -1))
            xo, zo, ph, _ = C.apply(s, [(kind, 1)])
            mid = "IXYZ".index(s_[1])
            anti = mid != 0 and mid != L
            assert np.array_equal(xo[0], x) and np.array_equal(zo[0], z)
            assert ph[0] == (2 if anti else 0)

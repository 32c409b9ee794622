"""CPU oracle for Clifford gates on Pauli sums.

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's
CPU-baseline leg, never by the product path; it shares no code with the HIP
library.

Definition followed (Section III-B, Clifford paragraph; Section V-B, "Gate
Application"): a Clifford U maps a Pauli string Q to the single string
U Q U^dagger up to a sign, so a gate relabels strings and keeps the number of
terms.  The oracle takes that definition literally: each gate's unitary is
written out as a 2x2 or 4x4 matrix, and the image of every local letter (or
letter pair) is found by conjugating its matrix and decomposing the result in
the Pauli basis, tr(P^dagger M) / d.  A term's letters on the gate's qubits
are replaced by that image and the phase exponent gains 2 when the image
carries a minus sign.  Gates act in list order (gates[0] first).
"""
from __future__ import annotations

import itertools

import numpy as np

from oracle import oracle as O

# gate kinds, in the order of the library's enumeration
H, S, SDG, X, Y, Z, CX, CZ, SWAP = range(9)
TWO_QUBIT = (CX, CZ, SWAP)

_SIG = {0: np.eye(2, dtype=complex),
        1: np.array([[0, 1], [1, 0]], dtype=complex),
        2: np.array([[0, -1j], [1j, 0]], dtype=complex),
        3: np.array([[1, 0], [0, -1]], dtype=complex)}


def _unitary(kind):
    r2 = 1 / np.sqrt(2)
    one = {H: np.array([[r2, r2], [r2, -r2]], dtype=complex),
           S: np.diag([1, 1j]),
           SDG: np.diag([1, -1j]),
           X: _SIG[1], Y: _SIG[2], Z: _SIG[3]}
    if kind in one:
        return one[kind]
    if kind == CX:  # control = first qubit (q0), target = second (q1)
        return np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex)
    if kind == CZ:
        return np.diag([1, 1, 1, -1]).astype(complex)
    if kind == SWAP:
        return np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=complex)
    raise ValueError("unknown gate kind %r" % kind)


def _images(kind):
    """{local letters: (image letters, sign)} for the gate's 1 or 2 qubits
    (letters 0 I, 1 X, 2 Y, 3 Z; the first letter is qubit q0)."""
    U = _unitary(kind)
    k = 2 if kind in TWO_QUBIT else 1
    basis = list(itertools.product(range(4), repeat=k))

    def mat(ls):
        m = np.array([[1.0 + 0j]])
        for L in ls:
            m = np.kron(m, _SIG[L])
        return m

    out = {}
    for ls in basis:
        M = U @ mat(ls) @ U.conj().T
        found = None
        for rs in basis:
            comp = np.trace(mat(rs).conj().T @ M) / 2 ** k
            if abs(comp) > 1e-9:
                assert found is None and abs(abs(comp) - 1) < 1e-9, "not a Clifford image"
                assert abs(comp.imag) < 1e-9
                found = (rs, 1 if comp.real > 0 else -1)
        out[ls] = found
    return out


_TABLES = {kind: _images(kind) for kind in range(9)}


def _encode(n, letters):
    W = (n + 63) // 64
    x = np.zeros(W, np.uint64)
    z = np.zeros(W, np.uint64)
    for q, L in enumerate(letters):
        if L in (1, 2):
            x[q // 64] |= np.uint64(1) << np.uint64(q % 64)
        if L in (2, 3):
            z[q // 64] |= np.uint64(1) << np.uint64(q % 64)
    return x, z


def apply(s: O.Sum, gates, terms=None):
    """Terms of s (all, or the indices `terms`) conjugated by the gates.
    gates: sequence of (kind, q0[, q1]).  Returns (x, z, phase, coef) of the
    selected terms in order; coefficients are unchanged."""
    idx = np.arange(s.m) if terms is None else np.asarray(terms)
    letters = O.decode(s.n, s.x[idx], s.z[idx]).astype(np.int64) if idx.size else \
        np.zeros((0, s.n), np.int64)
    W = (s.n + 63) // 64
    xo = np.zeros((idx.size, W), np.uint64)
    zo = np.zeros((idx.size, W), np.uint64)
    ph = np.zeros(idx.size, np.uint8)
    for r, t in enumerate(idx):
        L = list(letters[r])
        k = int(s.phase[t])
        for g in gates:
            kind, q0 = int(g[0]), int(g[1])
            if kind in TWO_QUBIT:
                q1 = int(g[2])
                (a, b), sign = _TABLES[kind][(L[q0], L[q1])]
                L[q0], L[q1] = a, b
            else:
                (a,), sign = _TABLES[kind][(L[q0],)]
                L[q0] = a
            if sign < 0:
                k += 2
        xo[r], zo[r] = _encode(s.n, L)
        ph[r] = k % 4
    return xo, zo, ph, s.coef[idx].copy()

"""Test-side helpers: letter strings <-> packed words, dense matrices.

The dense 2x2 matrices are the ones printed in Section III-A; the packed
layout follows Table I (Section III-C) with qubit q at bit q % 64 of word
q // 64.  Nothing here calls the oracle or the GPU library.
"""
import numpy as np

SIGMA = {
    "I": np.array([[1, 0], [0, 1]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
}
LETTERS = "IXYZ"  # the oracle's decode() order


def W(n):
    return (n + 63) // 64


def pack(s: str):
    """Letter string (qubit 0 first) -> (x words, z words) per Table I."""
    n = len(s)
    x = np.zeros(W(n), np.uint64)
    z = np.zeros(W(n), np.uint64)
    for q, L in enumerate(s):
        if L in "XY":
            x[q // 64] |= np.uint64(1) << np.uint64(q % 64)
        if L in "ZY":
            z[q // 64] |= np.uint64(1) << np.uint64(q % 64)
    return x, z


def unpack(n, x, z) -> str:
    out = []
    for q in range(n):
        xb = (int(x[q // 64]) >> (q % 64)) & 1
        zb = (int(z[q // 64]) >> (q % 64)) & 1
        out.append({(0, 0): "I", (0, 1): "Z", (1, 0): "X", (1, 1): "Y"}[(xb, zb)])
    return "".join(out)


def pack_many(strings):
    n = len(strings[0])
    xs = np.zeros((len(strings), W(n)), np.uint64)
    zs = np.zeros((len(strings), W(n)), np.uint64)
    for t, s in enumerate(strings):
        xs[t], zs[t] = pack(s)
    return xs, zs


def dense_string(s: str) -> np.ndarray:
    m = np.array([[1.0 + 0j]])
    for L in s:
        m = np.kron(m, SIGMA[L])
    return m


def dense_sum(n, x, z, phase, coef) -> np.ndarray:
    D = np.zeros((2 ** n, 2 ** n), np.complex128)
    for t in range(x.shape[0]):
        D += (1j ** int(phase[t])) * coef[t] * dense_string(unpack(n, x[t], z[t]))
    return D


def all_strings(n):
    out = [""]
    for _ in range(n):
        out = [s + L for s in out for L in LETTERS]
    return out

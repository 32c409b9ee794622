"""Lexicographic order of a Pauli sum: the CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.

Definition followed (Section III-H: the sum is ordered by a key formed from
the bit-packed words of each string, and equal strings end up adjacent).
The paper does not fix the order of the words inside the key; the reading
taken here is the packed words compared as unsigned 64-bit integers in the
order

    X[W-1], X[W-2], ..., X[0], Z[W-1], ..., Z[0]

(the X part first, most significant word first).  For n <= 32 this is the
order of the integer x * 2^32 + z.  Terms with equal strings keep their
input order (a stable sort), and the phase, coefficient and fingerprint of
a term travel with its string.

The sort itself is numpy's stable lexsort over the word columns, a library
primitive taken as one step.
"""
from __future__ import annotations

import numpy as np


def order(x: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Permutation p such that rows x[p], z[p] are in lexicographic order.

    x, z: uint64 arrays of shape (m, W).  np.lexsort sorts on its last key
    first, so the keys are passed from the least significant word (Z[0])
    to the most significant (X[W-1])."""
    x = np.asarray(x, dtype=np.uint64)
    z = np.asarray(z, dtype=np.uint64)
    m, W = x.shape
    if m == 0:
        return np.zeros(0, dtype=np.int64)
    keys = [z[:, w] for w in range(W)] + [x[:, w] for w in range(W)]
    return np.lexsort(keys)


def sort_lex(s: dict) -> dict:
    """The sum s (dict with n, x, z, phase, coef and optionally fp) with its
    terms in lexicographic order."""
    p = order(s["x"], s["z"])
    out = {"n": s["n"]}
    for k in ("x", "z", "phase", "coef", "fp"):
        if k in s and s[k] is not None:
            out[k] = np.asarray(s[k])[p]
    return out

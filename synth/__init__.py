"""Seeded synthetic Pauli sums shaped like the paper's workloads.

Shared by the tests, the smoke check and the benchmark: the GPU path and the
CPU oracle both receive their inputs from here.  This module contains no
Pauli arithmetic (no products, phases or merging); it only draws strings in
the packed layout and coefficients.

Packed layout (Section III-C, Table I): a string on n qubits is two uint64
arrays x, z of W = ceil(n/64) words; qubit q is bit q % 64 of word q // 64;
the letter at q is I (x=0,z=0), Z (0,1), X (1,0) or Y (1,1).

Workloads (the paper benchmarks "random 500-qubit sums" and cites molecular
Hamiltonians from Jordan-Wigner mappings; neither generator is specified, so
these recipes stand in for them):

* ``random_weight``: weight w uniform in [wmin, wmax] on distinct uniform
  qubits, each non-identity letter uniform over {X, Y, Z}.
* ``jordan_wigner``: a chain picks qubits p < q uniformly, puts Z on
  p+1..q-1 and X or Y (each with probability 1/2) at p and q; half of the
  terms are the letter-wise combination (bitwise XOR of x and z) of two
  independent chains.

Seeds: numpy PCG64 with SeedSequence(25974000 + workload id).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 25974000


def words(n: int) -> int:
    return (n + 63) // 64


def rng_for(workload: int, *spawn) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED_BASE + int(workload), spawn_key=tuple(int(s) for s in spawn))
    return np.random.Generator(np.random.PCG64(ss))


def _pack_rows(bits: np.ndarray) -> np.ndarray:
    """bool (m, n) -> uint64 (m, W), qubit q at bit q % 64 of word q // 64."""
    m, n = bits.shape
    W = words(n)
    pad = np.zeros((m, W * 64), dtype=bool)
    pad[:, :n] = bits
    by = np.packbits(pad, axis=1, bitorder="little")  # (m, 8W) bytes
    return np.ascontiguousarray(by).view("<u8").reshape(m, W).astype(np.uint64)


def _letters_to_bits(letters: np.ndarray):
    """letters in {0: I, 1: X, 2: Y, 3: Z} -> (xbits, zbits) per Table I."""
    xb = (letters == 1) | (letters == 2)
    zb = (letters == 3) | (letters == 2)
    return xb, zb


def _distinct_qubits(rng, n, m, w):
    """(m, max w) qubit indices; row r uses its first w[r] entries, all distinct."""
    wmax = int(w.max()) if m else 0
    if wmax * 8 > n:  # dense choice: a random permutation prefix per row
        return np.argsort(rng.random((m, n)), axis=1)[:, :wmax]
    q = rng.integers(0, n, size=(m, wmax))
    cols = np.arange(wmax)
    while True:
        key = np.where(cols[None, :] < w[:, None], q, n + cols[None, :])
        s = np.sort(key, axis=1)
        bad = np.any(s[:, 1:] == s[:, :-1], axis=1) if wmax > 1 else np.zeros(m, bool)
        nb = int(bad.sum())
        if nb == 0:
            return q
        q[bad] = rng.integers(0, n, size=(nb, wmax))


def random_weight(rng, n: int, m: int, wmin: int, wmax: int):
    """m strings (not necessarily distinct) of random weight; -> (x, z)."""
    x = np.zeros((m, words(n)), np.uint64)
    z = np.zeros((m, words(n)), np.uint64)
    chunk = 1 << 16
    for s0 in range(0, m, chunk):
        mm = min(chunk, m - s0)
        w = rng.integers(wmin, wmax + 1, size=mm)
        q = _distinct_qubits(rng, n, mm, w)
        let = rng.integers(1, 4, size=q.shape)
        let = np.where(np.arange(q.shape[1])[None, :] < w[:, None], let, 0)
        dense = np.zeros((mm, n), np.uint8)
        rows = np.repeat(np.arange(mm), q.shape[1])
        dense[rows, q.reshape(-1)] = np.maximum(dense[rows, q.reshape(-1)], let.reshape(-1))
        xb, zb = _letters_to_bits(dense)
        x[s0:s0 + mm] = _pack_rows(xb)
        z[s0:s0 + mm] = _pack_rows(zb)
    return x, z


def _chains(rng, n, m):
    """m Jordan-Wigner chains as dense bit rows (xbits, zbits)."""
    a = rng.integers(0, n, size=m)
    b = rng.integers(0, n - 1, size=m)
    b = np.where(b >= a, b + 1, b)  # distinct from a, uniform over the others
    p, q = np.minimum(a, b), np.maximum(a, b)
    idx = np.arange(n)[None, :]
    zb = (idx > p[:, None]) & (idx < q[:, None])
    xb = np.zeros((m, n), bool)
    r = np.arange(m)
    xb[r, p] = True
    xb[r, q] = True
    yp = rng.integers(0, 2, size=m).astype(bool)  # endpoint letter Y instead of X
    yq = rng.integers(0, 2, size=m).astype(bool)
    zb[r, p] = yp
    zb[r, q] = yq
    return xb, zb


def jordan_wigner(rng, n: int, m: int):
    """m Jordan-Wigner-shaped strings (not necessarily distinct); -> (x, z)."""
    x = np.zeros((m, words(n)), np.uint64)
    z = np.zeros((m, words(n)), np.uint64)
    chunk = 1 << 15
    for s0 in range(0, m, chunk):
        mm = min(chunk, m - s0)
        xb, zb = _chains(rng, n, mm)
        two = rng.integers(0, 2, size=mm).astype(bool)
        x2, z2 = _chains(rng, n, mm)
        xb = np.where(two[:, None], xb ^ x2, xb)
        zb = np.where(two[:, None], zb ^ z2, zb)
        x[s0:s0 + mm] = _pack_rows(xb)
        z[s0:s0 + mm] = _pack_rows(zb)
    return x, z


def _row_keys(x, z):
    xz = np.ascontiguousarray(np.concatenate([x, z], axis=1))
    return xz.view(np.dtype((np.void, xz.dtype.itemsize * xz.shape[1]))).reshape(-1)


def distinct(rng, draw, m: int):
    """Draw strings with ``draw(rng, count)`` until m distinct ones exist;
    keeps first occurrences in draw order."""
    if m <= 0:  # the words' shape from one draw
        x, z = draw(rng, 1)
        return np.ascontiguousarray(x[:0]), np.ascontiguousarray(z[:0])
    xs, zs = [], []
    have = 0
    seen = None
    while have < m:
        need = max(16, int((m - have) * 1.1) + 16)
        x, z = draw(rng, need)
        xs.append(x)
        zs.append(z)
        X = np.concatenate(xs)
        Z = np.concatenate(zs)
        _, first = np.unique(_row_keys(X, Z), return_index=True)
        first.sort()
        have = first.size
        seen = first
        xs, zs = [X], [Z]
    keep = seen[:m]
    return np.ascontiguousarray(xs[0][keep]), np.ascontiguousarray(zs[0][keep])


def log_uniform_complex(rng, m, lo_exp, hi_exp):
    mag = 10.0 ** rng.uniform(lo_exp, hi_exp, size=m)
    arg = rng.uniform(0.0, 2.0 * np.pi, size=m)
    return mag * np.exp(1j * arg)


def log_uniform_signed(rng, m, lo_exp, hi_exp):
    mag = 10.0 ** rng.uniform(lo_exp, hi_exp, size=m)
    sgn = np.where(rng.integers(0, 2, size=m) == 1, 1.0, -1.0)
    return (sgn * mag).astype(np.complex128)


def make_sum(n, x, z, coef, phase=None):
    m = x.shape[0]
    return {"n": int(n), "x": x, "z": z,
            "phase": np.zeros(m, np.uint8) if phase is None else phase.astype(np.uint8),
            "coef": coef}


# ---------------------------------------------------------------- workloads

def small_weight_sum(rng, n: int, m: int, wmin=1, wmax=4, merge_duplicates=True):
    """Workload 1 shape: weight 1..4 on n qubits, re, im ~ N(0,1); strings
    that repeat during drawing have their coefficients added, and drawing
    continues until m distinct strings exist."""
    table = {}
    order = []
    while len(order) < m:
        x, z = random_weight(rng, n, max(64, m - len(order)), wmin, wmax)
        c = rng.standard_normal(x.shape[0]) + 1j * rng.standard_normal(x.shape[0])
        for t in range(x.shape[0]):
            key = (x[t].tobytes(), z[t].tobytes())
            if key in table:
                table[key][2] += c[t]
            elif len(order) < m:
                table[key] = [x[t], z[t], c[t]]
                order.append(key)
    X = np.stack([table[k][0] for k in order]).astype(np.uint64)
    Z = np.stack([table[k][1] for k in order]).astype(np.uint64)
    C = np.array([table[k][2] for k in order], np.complex128)
    return make_sum(n, X, Z, C)


def jw_sum(rng, n: int, m: int, coef="complex", lo_exp=-6.0):
    x, z = distinct(rng, lambda r, k: jordan_wigner(r, n, k), m)
    if coef == "complex":
        c = log_uniform_complex(rng, m, lo_exp, 0.0)
    else:
        c = log_uniform_signed(rng, m, lo_exp, 0.0)
    return make_sum(n, x, z, c)


def workload1(m=2000, n=16):
    """Plain FP64, n=16: two sums of m distinct weight-1..4 strings."""
    return (small_weight_sum(rng_for(1, 0), n, m), small_weight_sum(rng_for(1, 1), n, m))


def workload2(m1=10000, m2=10000, n=500):
    """Plain FP64, n=500: two Jordan-Wigner-shaped sums, complex coefficients
    with log-uniform modulus in [1e-6, 1] and uniform argument."""
    return (jw_sum(rng_for(2, 0), n, m1), jw_sum(rng_for(2, 1), n, m2))


def workload3(m=20000, n=500):
    """Precision form: Hermitian H, Jordan-Wigner-shaped, real coefficients
    s * 10^U(-6,0) with random sign; the product is H*H."""
    return jw_sum(rng_for(3, 0), n, m, coef="real")


def workload4_plan(nb=256, median=2000, lo=100, hi=20000, sigma=1.0):
    """Per-batch (n, m1, m2) for the batched form: n uniform over
    {64, 128, 256, 500}; term counts lognormal (median 2000) clipped to
    [100, 20000]."""
    rng = rng_for(4, 0)
    ns = rng.choice(np.array([64, 128, 256, 500]), size=nb)
    m = np.clip(np.round(median * np.exp(sigma * rng.standard_normal((nb, 2)))), lo, hi).astype(int)
    return [(int(ns[b]), int(m[b, 0]), int(m[b, 1])) for b in range(nb)]


def workload4_batch(b, n, m1, m2):
    """Pair b of the batched form: complex64 coefficients as in workload 2."""
    A = jw_sum(rng_for(4, 1, b, 0), n, m1)
    B = jw_sum(rng_for(4, 1, b, 1), n, m2)
    A["coef"] = A["coef"].astype(np.complex64)
    B["coef"] = B["coef"].astype(np.complex64)
    return A, B


def workload5_state(m=1_000_000, n=500):
    """Propagation state: m distinct strings of weight 1..20, complex
    coefficients with log-uniform modulus in [1e-8, 1], uniform argument."""
    rng = rng_for(5, 0)
    x, z = distinct(rng, lambda r, k: random_weight(r, n, k, 1, 20), m)
    c = log_uniform_complex(rng, m, -8.0, 0.0)
    return make_sum(n, x, z, c)


def workload5_rotations(steps=64, n=500):
    """(theta_s, x_s, z_s) for the rotation steps: theta uniform in (0, pi),
    the generator a random weight-3 string."""
    rng = rng_for(5, 1)
    theta = rng.uniform(0.0, np.pi, size=steps)
    x, z = random_weight(rng, n, steps, 3, 3)
    return theta, x, z


def random_sum(rng, n: int, m: int, wmax=None, distinct_strings=True, phases=True):
    """Small generic sums for tests: random letters (weight up to wmax),
    random phases and N(0,1) complex coefficients."""
    wmax = n if wmax is None else wmax
    if distinct_strings:
        x, z = distinct(rng, lambda r, k: random_weight(r, n, k, 0 if n > 0 else 0, wmax), m) \
            if _can_be_distinct(n, wmax, m) else random_weight(rng, n, m, 0, wmax)
    else:
        x, z = random_weight(rng, n, m, 0, wmax)
    c = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    ph = rng.integers(0, 4, size=m).astype(np.uint8) if phases else None
    return make_sum(n, x, z, c, ph)


def _can_be_distinct(n, wmax, m):
    from math import comb
    total = sum(comb(n, w) * 3 ** w for w in range(0, min(n, wmax) + 1))
    return m <= total // 2

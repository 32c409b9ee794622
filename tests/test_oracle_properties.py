"""Algebraic properties of the oracle's sort-and-combine on generated sums
(hypothesis; no GPU).  With Gaussian-integer coefficients every product and
sum is exact, so the identities below hold to the last bit; a merge that
loses a duplicate, keeps a string twice, or drops a phase fails them.

* distributivity: merge((A + A') B) = merge(A B) + merge(A' B), where A + A'
  is the concatenation of the two term lists;
* identity: merge(I B) = merge(B) for the one-term sum I;
* idempotence: merge(merge(S)) = merge(S);
* scaling by a phase: the terms of A with their phase bytes raised by one
  give i * merge(A B)."""
import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import oracle as O


def _W(n):
    return (n + 63) // 64


def _sum(seed, n, m, dup):
    rng = np.random.default_rng(seed)
    W = _W(n)
    nd = max(1, m // 2) if dup else m
    bits = rng.integers(0, 2, (nd, 2, n))
    pick = rng.integers(0, nd, m) if dup else np.arange(m)
    x = np.zeros((m, W), np.uint64)
    z = np.zeros((m, W), np.uint64)
    for t in range(m):
        for q in range(n):
            if bits[pick[t], 0, q]:
                x[t, q >> 6] |= np.uint64(1 << (q & 63))
            if bits[pick[t], 1, q]:
                z[t, q >> 6] |= np.uint64(1 << (q & 63))
    c = (rng.integers(-3, 4, m) + 1j * rng.integers(-3, 4, m)).astype(np.complex128)
    ph = rng.integers(0, 4, m).astype(np.uint8)
    return O.Sum(n, x, z, ph, c)


def _cat(a, b):
    return O.Sum(a.n, np.vstack([a.x, b.x]), np.vstack([a.z, b.z]),
                 np.concatenate([a.phase, b.phase]), np.concatenate([a.coef, b.coef]))


def _table(r):
    """{string: coef} of a merged result, zero terms left out."""
    return {k: v[0] for k, v in r.as_dict().items() if v[0] != 0}


def _add(t1, t2):
    out = dict(t1)
    for k, v in t2.items():
        out[k] = out.get(k, 0) + v
    return {k: v for k, v in out.items() if v != 0}


sizes = st.sampled_from([1, 3, 64, 65, 130])


@settings(max_examples=25, deadline=None)
@given(n=sizes, m1=st.integers(1, 12), m2=st.integers(1, 12), m3=st.integers(1, 12),
       seed=st.integers(0, 2**31), dup=st.booleans())
def test_distributivity_and_identity(n, m1, m2, m3, seed, dup):
    A = _sum(seed, n, m1, dup)
    A2 = _sum(seed + 1, n, m2, dup)
    B = _sum(seed + 2, n, m3, dup)
    lhs = _table(O.product_merge(_cat(A, A2), B))
    rhs = _add(_table(O.product_merge(A, B)), _table(O.product_merge(A2, B)))
    assert lhs == rhs
    W = _W(n)
    I = O.Sum(n, np.zeros((1, W), np.uint64), np.zeros((1, W), np.uint64), None,
              np.ones(1, np.complex128))
    assert _table(O.product_merge(I, B)) == _table(O.merge(B))


@settings(max_examples=25, deadline=None)
@given(n=sizes, m=st.integers(1, 30), seed=st.integers(0, 2**31))
def test_idempotence_and_phase_scaling(n, m, seed):
    S = _sum(seed, n, m, True)
    once = O.merge(S)
    again = O.merge(O.Sum(n, once.x, once.z, None, once.coef))
    assert _table(again) == _table(once)
    B = _sum(seed + 7, n, 5, False)
    up = O.Sum(n, S.x, S.z, (S.phase + 1) % 4, S.coef)
    assert _table(O.product_merge(up, B)) == {k: 1j * v for k, v in
                                              _table(O.product_merge(S, B)).items()}

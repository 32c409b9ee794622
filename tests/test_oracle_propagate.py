"""Pins of the oracle's rotation steps (Section III-B eq. (5)) against dense
matrices, the paper's special angles and the unitary-invariance of the
Hilbert-Schmidt norm.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import oracle as O
from tests import helpers as H


def _sum(rng, n, m, wmax=None):
    d = synth.random_sum(rng, n, m, wmax=wmax)
    return d, O.Sum(n, d["x"], d["z"], d["phase"], d["coef"])


def _rand_string(rng, n, w):
    qs = rng.choice(n, size=w, replace=False)
    s = ["I"] * n
    for q in qs:
        s[q] = "XYZ"[rng.integers(0, 3)]
    return "".join(s)


def _decompose(n, D):
    """Coefficients of a dense operator in the Pauli basis: Tr(s D) / 2^n."""
    out = {}
    for s in H.all_strings(n):
        c = np.trace(H.dense_string(s) @ D) / 2 ** n
        out[s] = c
    return out


def _as_letters(n, R):
    return {H.unpack(n, R.x[u], R.z[u]): R.coef[u] for u in range(R.x.shape[0])}


@pytest.mark.parametrize("mode", [O.PRODUCT, O.CONJUGATE])
@pytest.mark.parametrize("n", [2, 3])
def test_rotation_steps_against_dense(n, mode):
    rng = synth.rng_for(720, n * 10 + mode)
    d, S = _sum(rng, n, 7)
    steps = 3
    Ps = [_rand_string(rng, n, rng.integers(1, n + 1)) for _ in range(steps)]
    th = rng.uniform(0, np.pi, steps)
    px, pz = H.pack_many(Ps)
    R = O.propagate(S, px, pz, th, mode=mode)
    D = H.dense_sum(n, d["x"], d["z"], d["phase"], d["coef"])
    for P, t in zip(Ps, th):
        Pm = H.dense_string(P)
        if mode == O.CONJUGATE:
            U = np.cos(t / 2) * np.eye(2 ** n) - 1j * np.sin(t / 2) * Pm   # eq. (4)
            D = U @ D @ U.conj().T
        else:
            D = (np.cos(t) * np.eye(2 ** n) - 1j * np.sin(t) * Pm) @ D
    ref = _decompose(n, D)
    got = _as_letters(n, R)
    for s, c in ref.items():
        assert abs(got.get(s, 0.0) - c) <= 1e-12 * max(1.0, abs(c)), (s, got.get(s), c)


@pytest.mark.parametrize("mode", [O.PRODUCT, O.CONJUGATE])
def test_norm_is_invariant(mode):
    """R is unitary, so sum |c|^2 = Tr(H^dagger H) / 2^n is kept by both
    left multiplication and conjugation (no truncation)."""
    rng = synth.rng_for(721, mode)
    n = 70
    d, S = _sum(rng, n, 300, wmax=6)
    Ps = [_rand_string(rng, n, 3) for _ in range(5)]
    px, pz = H.pack_many(Ps)
    R = O.propagate(S, px, pz, rng.uniform(0, np.pi, 5), mode=mode)
    M = O.merge(S)
    n0 = np.sum(np.abs(M.coef) ** 2)
    n1 = np.sum(np.abs(R.coef) ** 2)
    assert abs(n1 - n0) <= 1e-13 * n0


def test_clifford_and_pauli_angles():
    """Section III-B: at theta = pi/2 an anticommuting Q becomes -i P Q; at
    theta = pi it becomes -Q; commuting terms never change.  The round-off
    remnants of cos(pi/2) and sin(pi) are truncated."""
    rng = synth.rng_for(722)
    n = 12
    d, S = _sum(rng, n, 40, wmax=5)
    P = _rand_string(rng, n, 3)
    px, pz = H.pack_many([P])
    M = O.merge(S)
    base = _as_letters(n, M)
    for theta, expect in ((np.pi / 2, "clifford"), (np.pi, "pauli")):
        R = _as_letters(n, O.propagate(S, px, pz, [theta], mode=O.CONJUGATE, drop_abs=1e-12))
        want = {}
        for Q, c in base.items():
            xq, zq = H.pack(Q)
            xp, zp = H.pack(P)
            x3, z3, k = O.mul(n, xp, zp, 0, xq, zq, 0)
            anti = sum(1 for a, b in zip(P, Q) if a != "I" and b != "I" and a != b) % 2
            if not anti:
                want[Q] = want.get(Q, 0) + c
            elif expect == "pauli":
                want[Q] = want.get(Q, 0) - c
            else:
                PQ = H.unpack(n, x3, z3)
                want[PQ] = want.get(PQ, 0) + (-1j) * (1j ** k) * c
        want = {s: c for s, c in want.items() if abs(c) >= 1e-12}
        assert set(R) == set(want)
        for s in want:
            assert abs(R[s] - want[s]) <= 1e-15 * abs(want[s]) + 1e-15


def test_truncation_removes_exactly_the_small_terms():
    rng = synth.rng_for(723)
    n = 40
    d, S = _sum(rng, n, 200, wmax=4)
    d["coef"] = d["coef"] * 10.0 ** rng.uniform(-8, 0, 200)
    S = O.Sum(n, d["x"], d["z"], d["phase"], d["coef"])
    P = _rand_string(rng, n, 3)
    px, pz = H.pack_many([P])
    full = O.propagate(S, px, pz, [0.7], mode=O.PRODUCT)
    t = 1e-4
    cut = O.propagate(S, px, pz, [0.7], mode=O.PRODUCT, drop_abs=t)
    keep = np.abs(full.coef) >= t
    assert cut.x.shape[0] == int(keep.sum())
    assert np.array_equal(cut.coef, full.coef[keep])


def test_zero_angle_is_identity():
    rng = synth.rng_for(724)
    n = 30
    d, S = _sum(rng, n, 50)
    px, pz = H.pack_many([_rand_string(rng, n, 3)])
    M = _as_letters(n, O.merge(S))
    for mode in (O.PRODUCT, O.CONJUGATE):
        # sin(0) = 0: the P Q terms of the product mode carry exact zeros
        R = _as_letters(n, O.propagate(S, px, pz, [0.0], mode=mode))
        assert {s: c for s, c in R.items() if s in M} == M
        assert all(c == 0 for s, c in R.items() if s not in M)

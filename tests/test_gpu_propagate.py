"""Rotation steps of the propagation loop (pauli_propagate) against the CPU
oracle, through the C ABI."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _state(m, n=500):
    return synth.workload5_state(m=m, n=n)


def _rots(steps, n=500):
    th, x, z = synth.workload5_rotations(steps=steps, n=n)
    return th, x, z


def _no_band(ref_full, thr):
    return not np.any(np.abs(np.abs(ref_full.coef) - thr) <= 1e-9 * thr)


@pytest.mark.parametrize("rot_mode,steps", [(pl.ROTATE_CONJUGATE, 8), (pl.ROTATE_PRODUCT, 4)])
def test_propagate_fp64_matches_oracle(rot_mode, steps):
    S = _state(3000)
    th, x, z = _rots(steps)
    thr = 1e-10
    g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, rotate_mode=rot_mode,
                     drop_abs=thr).export()
    ref = O.propagate(_osum(S), x, z, th, mode=rot_mode, drop_abs=thr)
    assert _no_band(ref, thr)
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)
    if rot_mode == pl.ROTATE_PRODUCT:
        assert g["x"].shape[0] > 2 ** (steps - 1) * 3000 // 2  # the literal step doubles the sum


def test_propagate_compensated():
    """The precision form carries float-float coefficients between steps:
    after 16 conjugation steps every string with |c| > 1e-12 A (A: the
    mass of its last merge) is within 1e-6 relative of the FP64 oracle,
    and the string set is the oracle's (no string lost or gained at the
    drop threshold)."""
    S = _state(3000)
    th, x, z = _rots(16)
    thr = 1e-10
    g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, mode=pl.COMPENSATED,
                     drop_abs=thr).export()
    ref = O.propagate(_osum(S), x, z, th, mode=O.CONJUGATE, drop_abs=thr)
    assert _no_band(ref, thr)
    assert g["coef"].dtype == np.complex64
    err = parity.max_rel_err(g, ref)
    print("16 conjugation steps, compensated: max rel err %.3e" % err)
    assert err <= 1e-6
    parity.assert_sorted_by_key(g)


@pytest.mark.parametrize("tau", [0.0, 0.3])
def test_propagate_compensated_cancellation(tau):
    """Pairs Q, Q' = P Q that both anticommute with P: after the step the
    string Q holds cos(theta) c_Q + kappa c_Q', chosen to cancel to about
    1e-4 of its mass, and Q' likewise.  The segment is re-merged in FP64
    from the float-float state (FP64 products of the state and the FP64
    cos, sin), so the error stays below 1e-6 of the cancelled value;
    further steps then carry it on."""
    rng = synth.rng_for(734)
    n, W = 130, 3
    px, pz = synth.random_weight(rng, n, 1, 3, 3)
    px, pz = px[0], pz[0]
    theta = 0.7
    pairs = []
    while len(pairs) < 40:
        qx, qz = synth.random_weight(rng, n, 1, 2, 12)
        qx, qz = qx[0], qz[0]
        par = sum(bin(int(a) & int(b)).count("1") + bin(int(c) & int(d)).count("1")
                  for a, b, c, d in zip(qx, pz, qz, px)) & 1
        if not par:
            continue
        # Q' and the factor kappa of Q' -> Q: step on the one-term sum Q'
        one = O.propagate(O.Sum(n, qx[None, :], qz[None, :], None, np.array([1.0 + 0j])),
                          px[None, :], pz[None, :], [theta], mode=O.CONJUGATE)
        kq = (qx.tobytes(), qz.tobytes())
        d = one.as_dict()
        (kp,) = [k for k in d if k != kq]
        px2 = np.frombuffer(kp[0], np.uint64).copy()
        pz2 = np.frombuffer(kp[1], np.uint64).copy()
        back = O.propagate(O.Sum(n, px2[None, :], pz2[None, :], None, np.array([1.0 + 0j])),
                           px[None, :], pz[None, :], [theta], mode=O.CONJUGATE).as_dict()
        kappa = back[kq][0]
        cq = np.exp(1j * rng.uniform(0, 2 * np.pi)) * 10 ** rng.uniform(-3, 0)
        eps = 10 ** rng.uniform(-4.5, -3.5)
        cqp = -np.cos(theta) * cq / kappa * (1 - eps)
        pairs.append((qx, qz, cq, px2, pz2, cqp))
    x = np.array([p[0] for p in pairs] + [p[3] for p in pairs])
    z = np.array([p[1] for p in pairs] + [p[4] for p in pairs])
    c = np.array([p[2] for p in pairs] + [p[5] for p in pairs])
    R = synth.random_sum(synth.rng_for(735), n, 300, wmax=8)
    S = {"n": n, "x": np.concatenate([x, R["x"]]), "z": np.concatenate([z, R["z"]]),
         "phase": np.zeros(len(c) + 300, np.uint8), "coef": np.concatenate([c, R["coef"]])}
    th2, x2, z2 = synth.workload5_rotations(steps=3, n=n)
    X = np.concatenate([px[None, :], x2])
    Z = np.concatenate([pz[None, :], z2])
    TH = np.concatenate([[theta], th2])
    for steps in (1, 4):
        g = pl.propagate(pl.PauliSum.from_dict(S), X[:steps], Z[:steps], TH[:steps],
                         mode=pl.COMPENSATED, tau=tau).export()
        ref = O.propagate(_osum(S), X[:steps], Z[:steps], TH[:steps], mode=O.CONJUGATE)
        if steps == 1:
            d = ref.as_dict()
            r = [abs(d[(p[0].tobytes(), p[1].tobytes())][0]) /
                 d[(p[0].tobytes(), p[1].tobytes())][1] for p in pairs]
            assert max(r) < 1e-3 and min(r) > 1e-5  # the planted cancellation
        err = parity.max_rel_err(g, ref)
        print("cancellation, %d steps, tau %g: max rel err %.3e" % (steps, tau, err))
        assert err <= 1e-6


def test_propagate_edge_cases():
    n = 70
    S = synth.random_sum(synth.rng_for(730), n, 400, wmax=5)
    G = pl.PauliSum.from_dict(S)
    W = 2
    # no steps: the merged input
    g0 = pl.propagate(G, np.zeros((0, W)), np.zeros((0, W)), []).export()
    parity.assert_merged_fp64(g0, O.merge(_osum(S)))
    # identity generator: everything commutes; the product mode scales by
    # cos(theta) - i sin(theta)
    zx = np.zeros((1, W), np.uint64)
    for rm in (pl.ROTATE_CONJUGATE, pl.ROTATE_PRODUCT):
        g = pl.propagate(G, zx, zx, [0.9], rotate_mode=rm).export()
        parity.assert_merged_fp64(g, O.propagate(_osum(S), zx, zx, [0.9], mode=rm))
    # an empty sum stays empty
    E = {"n": n, "x": np.zeros((0, W), np.uint64), "z": np.zeros((0, W), np.uint64),
         "phase": np.zeros(0, np.uint8), "coef": np.zeros(0, np.complex128)}
    px = np.zeros((1, W), np.uint64)
    px[0, 0] = 5
    for rm in (pl.ROTATE_CONJUGATE, pl.ROTATE_PRODUCT):
        assert pl.propagate(pl.PauliSum.from_dict(E), px, px, [0.3], rotate_mode=rm).m == 0
    # a generator with a bit at or above n is rejected
    bad = np.zeros((1, W), np.uint64)
    bad[0, 1] = np.uint64(1) << np.uint64(10)   # qubit 74 >= 70
    with pytest.raises(pl.PauliError) as e:
        pl.propagate(G, bad, zx, [0.3])
    assert e.value.status == "INVALID"


def test_propagate_small_n_many_merges():
    """n = 4: only 256 strings exist, so every step merges heavily."""
    n = 4
    S = synth.random_sum(synth.rng_for(731), n, 60, wmax=4)
    rng = synth.rng_for(732)
    steps = 10
    x, z = synth.random_weight(rng, n, steps, 1, 3)
    th = rng.uniform(0, np.pi, steps)
    for rm in (pl.ROTATE_CONJUGATE, pl.ROTATE_PRODUCT):
        g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, rotate_mode=rm).export()
        parity.assert_merged_fp64(g, O.propagate(_osum(S), x, z, th, mode=rm))


@pytest.mark.parametrize("key_bits", [6, 20])
@pytest.mark.parametrize("rot_mode,steps", [(pl.ROTATE_CONJUGATE, 6), (pl.ROTATE_PRODUCT, 4)])
def test_conjugation_merge_path_with_truncated_keys(key_bits, rot_mode, steps):
    """After the first step the conjugation (and the literal product)
    merges the kept (already sorted) strings with the sorted new strings
    instead of sorting everything.  Truncated keys make many distinct
    strings share a key across the two lists (in the product, P Q of one
    term lands on strings of other terms); every step must still match the
    oracle and stay in key order."""
    S = _state(2000)
    th, x, z = _rots(steps)
    g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, rotate_mode=rot_mode,
                     key_bits=key_bits).export()
    ref = O.propagate(_osum(S), x, z, th, mode=rot_mode)
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g, key_bits=key_bits)


def test_conjugation_steps_without_anticommuting_terms():
    """A rotation string that commutes with every term (Z-only strings on a
    Z-only state) leaves the state unchanged step after step."""
    rng = synth.rng_for(731)
    n, m = 80, 500
    W = 2
    zs = rng.integers(0, 2 ** 62, size=(m, W), dtype=np.uint64)
    zs[:, 1] &= np.uint64((1 << 16) - 1)
    S = {"n": n, "x": np.zeros_like(zs), "z": zs, "phase": np.zeros(m, np.uint8),
         "coef": rng.standard_normal(m) + 1j * rng.standard_normal(m)}
    px = np.zeros((3, W), np.uint64)
    pz = rng.integers(0, 2 ** 62, size=(3, W), dtype=np.uint64)
    pz[:, 1] &= np.uint64((1 << 16) - 1)
    g = pl.propagate(pl.PauliSum.from_dict(S), px, pz, [0.3, 0.7, 1.1],
                     rotate_mode=pl.ROTATE_CONJUGATE).export()
    ref = O.merge(_osum(S))
    parity.assert_merged_fp64(g, ref)


def _letter(n, W, q, letter):
    """(x, z) words of one letter (1 X, 2 Y, 3 Z) on qubit q."""
    x = np.zeros(W, np.uint64)
    z = np.zeros(W, np.uint64)
    b = np.uint64(1) << np.uint64(q % 64)
    if letter in (1, 2):
        x[q // 64] |= b
    if letter in (2, 3):
        z[q // 64] |= b
    return x, z


@pytest.mark.parametrize("n", [100, 1000])
def test_conjugation_generators_in_few_words(n):
    """Generators whose letters sit in one word, in the first and last
    words, and in the last (partial) word: the steps read only the words
    where the generator has letters (anticommutation count and the phase of
    the new terms) and must still match the oracle, with 2 and 16 words."""
    W = (n + 63) // 64
    S = synth.random_sum(synth.rng_for(733, n), n, 1500, wmax=min(n, 300), distinct_strings=False)
    gens = [[(1, 1), (5, 2), (9, 3)],                       # one word (the first)
            [(2, 2), (n - 1, 1)],                           # first and last qubit
            [(n - 3, 3), (n - 2, 2), (n - 1, 1)],           # the last word only
            [(64 * (W // 2) + 7, 2), (3, 3), (n - 5, 1)]]   # three words
    x = np.zeros((len(gens), W), np.uint64)
    z = np.zeros((len(gens), W), np.uint64)
    for s, g in enumerate(gens):
        for q, letter in g:
            gx, gz = _letter(n, W, q, letter)
            x[s] |= gx
            z[s] |= gz
    th = np.array([0.4, 1.3, 2.2, 0.8])
    g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, rotate_mode=pl.ROTATE_CONJUGATE).export()
    ref = O.propagate(_osum(S), x, z, th, mode=O.CONJUGATE)
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


def test_product_steps_compensated():
    """The literal product in the precision form (the steps after the first
    go through the merge path in FP32 with compensated sums) against the
    FP64 oracle."""
    S = _state(2000)
    th, x, z = _rots(4)
    g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, rotate_mode=pl.ROTATE_PRODUCT,
                     mode=pl.COMPENSATED, drop_abs=1e-10).export()
    ref = O.propagate(_osum(S), x, z, th, mode=O.PRODUCT, drop_abs=1e-10)
    assert _no_band(ref, 1e-10)
    assert g["coef"].dtype == np.complex64
    err = parity.max_rel_err(g, ref)
    print("4 product steps, compensated: max rel err %.3e" % err)
    assert err <= 1e-6

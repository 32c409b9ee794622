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
    S = _state(3000)
    th, x, z = _rots(8)
    g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, mode=pl.COMPENSATED,
                     drop_abs=1e-10).export()
    ref = O.propagate(_osum(S), x, z, th, mode=O.CONJUGATE, drop_abs=1e-10)
    assert g["coef"].dtype == np.complex64
    err = parity.max_rel_err_after_drop(g, ref)
    print("8 conjugation steps, compensated: max rel err %.3e" % err)
    assert err <= 1e-5


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
def test_conjugation_merge_path_with_truncated_keys(key_bits):
    """After the first step the conjugation merges the kept (already sorted)
    strings with the sorted new strings instead of sorting everything.
    Truncated keys make many distinct strings share a key across the two
    lists; every step must still match the oracle and stay in key order."""
    S = _state(2000)
    th, x, z = _rots(6)
    g = pl.propagate(pl.PauliSum.from_dict(S), x, z, th, rotate_mode=pl.ROTATE_CONJUGATE,
                     key_bits=key_bits).export()
    ref = O.propagate(_osum(S), x, z, th, mode=O.CONJUGATE)
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
    assert g["coef"].dtype == np.complex64
    err = parity.max_rel_err_after_drop(g, ref)
    print("4 product steps, compensated: max rel err %.3e" % err)
    assert err <= 1e-5

"""Propagation plans (pauli_propagate_plan_*): the rotation loop of Section
III-B eq. (5) captured into one HIP graph with every size on the device,
against the CPU oracle and against the host-synchronised loop, through the
C ABI."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _no_band(ref, thr):
    return not np.any(np.abs(np.abs(ref.coef) - thr) <= 1e-9 * thr)


def _same(a, b):
    for k in ("x", "z", "phase", "fp"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["coef"].view(np.uint8), b["coef"].view(np.uint8))


@pytest.mark.parametrize("rot_mode,steps", [(pl.ROTATE_CONJUGATE, 8), (pl.ROTATE_PRODUCT, 4)])
def test_plan_fp64_matches_oracle_and_replays(rot_mode, steps):
    S = synth.workload5_state(m=3000)
    th, x, z = synth.workload5_rotations(steps=steps)
    thr = 1e-10
    G = pl.PauliSum.from_dict(S)
    P = pl.PropagatePlan(G, x, z, th, max_terms=3000 * 2 ** steps, rotate_mode=rot_mode,
                         drop_abs=thr)
    P.run()
    g1 = P.result().export()
    P.run()
    P.run()  # results are taken from the last run only
    g2 = P.result().export()
    P.destroy()
    ref = O.propagate(_osum(S), x, z, th, mode=rot_mode, drop_abs=thr)
    assert _no_band(ref, thr)
    parity.assert_merged_fp64(g1, ref)
    parity.assert_sorted_by_key(g1)
    _same(g1, g2)


def test_plan_compensated_matches_oracle_and_eager_loop():
    """The precision form's float-float state: within 1e-6 of the FP64
    oracle, and bit-equal to the host-synchronised loop (same kernels, same
    order of every sum)."""
    S = synth.workload5_state(m=3000)
    th, x, z = synth.workload5_rotations(steps=16)
    thr = 1e-10
    G = pl.PauliSum.from_dict(S)
    P = pl.PropagatePlan(G, x, z, th, max_terms=200000, mode=pl.COMPENSATED, drop_abs=thr)
    P.run()
    g = P.result().export()
    ref = O.propagate(_osum(S), x, z, th, mode=O.CONJUGATE, drop_abs=thr)
    assert _no_band(ref, thr)
    assert g["coef"].dtype == np.complex64
    err = parity.max_rel_err(g, ref)
    print("graph loop, 16 steps, precision form: max rel err %.3e" % err)
    assert err <= 1e-6
    eager = pl.propagate(G, x, z, th, mode=pl.COMPENSATED, drop_abs=thr).export()
    _same(g, eager)


@pytest.mark.parametrize("key_bits", [6, 20])
@pytest.mark.parametrize("rot_mode,steps", [(pl.ROTATE_CONJUGATE, 6), (pl.ROTATE_PRODUCT, 3)])
def test_plan_truncated_keys(key_bits, rot_mode, steps):
    S = synth.workload5_state(m=2000)
    th, x, z = synth.workload5_rotations(steps=steps)
    G = pl.PauliSum.from_dict(S)
    P = pl.PropagatePlan(G, x, z, th, max_terms=2000 * 2 ** steps, rotate_mode=rot_mode,
                         key_bits=key_bits)
    P.run()
    g = P.result().export()
    parity.assert_merged_fp64(g, O.propagate(_osum(S), x, z, th, mode=rot_mode))
    parity.assert_sorted_by_key(g, key_bits=key_bits)


def test_plan_small_n_c64_and_edges():
    n = 4
    S = synth.random_sum(synth.rng_for(736), n, 60, wmax=4)
    rng = synth.rng_for(737)
    x, z = synth.random_weight(rng, n, 10, 1, 3)
    th = rng.uniform(0, np.pi, 10)
    for rm in (pl.ROTATE_CONJUGATE, pl.ROTATE_PRODUCT):
        P = pl.PropagatePlan(pl.PauliSum.from_dict(S), x, z, th, max_terms=256, rotate_mode=rm)
        P.run()
        parity.assert_merged_fp64(P.result().export(), O.propagate(_osum(S), x, z, th, mode=rm))
    # complex64 state in the plain form (FP32 sums)
    C = dict(S, coef=S["coef"].astype(np.complex64))
    P = pl.PropagatePlan(pl.PauliSum.from_dict(C), x, z, th, max_terms=256)
    P.run()
    g = P.result().export()
    ref = O.propagate(_osum(C), x, z, th, mode=O.CONJUGATE)
    gi, ri = parity.align(g["x"], g["z"], ref.x, ref.z)
    assert np.all(np.abs(g["coef"][gi] - ref.coef[ri]) <= 1e-5 * np.maximum(ref.mass[ri], 1e-30))
    # an empty sum stays empty; no steps gives the merged input
    E = {"n": n, "x": np.zeros((0, 1), np.uint64), "z": np.zeros((0, 1), np.uint64),
         "phase": None, "coef": np.zeros(0, np.complex128)}
    P = pl.PropagatePlan(pl.PauliSum.from_dict(E), x[:2], z[:2], th[:2], max_terms=16)
    P.run()
    assert P.result().m == 0
    P = pl.PropagatePlan(pl.PauliSum.from_dict(S), x[:0], z[:0], th[:0], max_terms=64)
    P.run()
    parity.assert_merged_fp64(P.result().export(), O.merge(_osum(S)))


def test_plan_capacity():
    S = synth.workload5_state(m=2000)
    th, x, z = synth.workload5_rotations(steps=3)
    G = pl.PauliSum.from_dict(S)
    need = pl.propagate(G, x, z, th, rotate_mode=pl.ROTATE_PRODUCT).m  # about 8 * 2000 terms
    P = pl.PropagatePlan(G, x, z, th, max_terms=need - 1, rotate_mode=pl.ROTATE_PRODUCT)
    P.run()
    with pytest.raises(pl.PauliError) as e:
        P.result()
    assert e.value.status == "CAPACITY"
    with pytest.raises(pl.PauliError) as e:
        P.result()  # no run since the last result
    assert e.value.status == "INVALID"
    P.run()  # the plan still runs after the failed result
    with pytest.raises(pl.PauliError):
        P.result()
    P = pl.PropagatePlan(G, x, z, th, max_terms=need, rotate_mode=pl.ROTATE_PRODUCT)
    P.run()
    parity.assert_merged_fp64(P.result().export(),
                              O.propagate(_osum(S), x, z, th, mode=O.PRODUCT))


@pytest.mark.parametrize("mode", [pl.PLAIN, pl.COMPENSATED])
def test_plan_full_state_matches_eager_loop(mode):
    """The 1e6-term state of the propagation workload through 6 conjugation
    steps as one graph, with its kernels sized from the measuring run (state
    and new-string bounds well below the doubling bound): bit-equal to the
    host-synchronised loop, whose full-size parity against the oracle is
    checked elsewhere."""
    S = synth.workload5_state()
    th, x, z = synth.workload5_rotations(steps=6)
    G = pl.PauliSum.from_dict(S)
    P = pl.PropagatePlan(G, x, z, th, max_terms=len(S["coef"]) * 4, mode=mode, drop_abs=1e-10)
    P.run()
    P.run()
    g = P.result().export()
    P.destroy()
    eager = pl.propagate(G, x, z, th, mode=mode, drop_abs=1e-10).export()
    assert len(g["coef"]) > len(S["coef"])
    _same(g, eager)

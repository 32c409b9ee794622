"""The precision form (FP32 products, Sum2-compensated merge, FP64 re-merge
of cancelled segments) against the exact CPU oracle, through the C ABI."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu

COMP = pl.COMPENSATED


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _gsum(d):
    return pl.PauliSum.from_dict(d)


def _rand(seed, n, m, wmax=None):
    return synth.random_sum(synth.rng_for(710, seed), n, m, wmax=wmax)


def test_compensated_fused_workload2_shape():
    A, B = synth.workload2(m1=300, m2=257)
    g = pl.outer_product_merged(_gsum(A), _gsum(B), mode=COMP, tau=0.3).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_compensated(g, ref)
    parity.assert_sorted_by_key(g)
    err = parity.max_rel_err(g, ref)
    print("max rel err (|c| > 1e-12 A), tau=0.3: %.3e" % err)
    assert parity.max_rel_err_after_drop(g, ref) <= 1e-6


@pytest.mark.parametrize("tau", [1e-3, 0.3])
def test_compensated_hermitian_square(tau):
    """The cancellation case at reduced size: H*H with real coefficients.
    Anticommuting pairs cancel exactly, in FP32 as in FP64."""
    H = synth.workload3(m=500)
    G = _gsum(H)
    g = pl.outer_product_merged(G, G, mode=COMP, tau=tau).export()
    ref = O.product_merge(_osum(H), _osum(H))
    parity.assert_compensated(g, ref)
    gi, ri = parity.align(g["x"], g["z"], ref.x, ref.z)
    # exact cancellations exist, and come out at the FP64 re-merge's accuracy
    zero = ref.coef[ri] == 0
    assert np.any(zero)
    assert np.all(np.abs(g["coef"][gi][zero]) <= 1e-12 * ref.mass[ri][zero])
    err = parity.max_rel_err_after_drop(g, ref)
    print("tau=%g: max rel err after dropping |c| < 1e-6 max|c|: %.3e" % (tau, err))
    if tau >= 0.3:
        assert err <= 1e-6


def _remerge_case():
    """Two products land on each of the strings I and X with values
    1 + 2^-30 and -1.  In FP32 the first input rounds to 1 and the segment
    cancels to 0; the FP64 re-merge recovers 2^-30 exactly."""
    n = 5
    x = np.array([[0], [1]], np.uint64)
    z = np.zeros((2, 1), np.uint64)
    A = {"n": n, "x": x, "z": z, "phase": np.zeros(2, np.uint8),
         "coef": np.array([1 + 2.0 ** -30, -1.0], np.complex128)}
    B = {"n": n, "x": x[::-1].copy(), "z": z, "phase": np.zeros(2, np.uint8),
         "coef": np.array([1.0, 1.0], np.complex128)}
    return A, B


def test_remerge_recovers_fp64_inputs():
    A, B = _remerge_case()
    GA, GB = _gsum(A), _gsum(B)
    for g in (pl.outer_product_merged(GA, GB, mode=COMP).export(),
              pl.merge(pl.outer_product(GA, GB), mode=COMP).export()):
        assert g["coef"].dtype == np.complex64
        assert g["x"].shape[0] == 2
        assert np.all(g["coef"] == np.complex64(2.0 ** -30))


@pytest.mark.parametrize("n", [2, 3])
def test_compensated_long_segments(n):
    """Few distinct strings, hundreds of records each: the block reduction
    of long segments (and its re-merge) runs."""
    A = _rand(20 + n, n, 4 ** n, wmax=n)
    rng = synth.rng_for(711, n)
    base = _rand(30 + n, n, 6, wmax=n)
    idx = rng.integers(0, 6, size=400)
    B = {"n": n, "x": base["x"][idx], "z": base["z"][idx],
         "phase": rng.integers(0, 4, size=400).astype(np.uint8),
         "coef": rng.standard_normal(400) + 1j * rng.standard_normal(400)}
    g = pl.outer_product_merged(_gsum(A), _gsum(B), mode=COMP).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_compensated(g, ref)


def test_compensated_c64_inputs():
    A, B = _rand(40, 130, 200), _rand(41, 130, 150)
    A["coef"] = A["coef"].astype(np.complex64)
    B["coef"] = B["coef"].astype(np.complex64)
    g = pl.outer_product_merged(_gsum(A), _gsum(B), mode=COMP).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_compensated(g, ref, input_rounding=False)


def test_compensated_general_path_and_collisions():
    A, B = _rand(50, 70, 90), _rand(51, 70, 80)
    GA, GB = _gsum(A), _gsum(B)
    ref = O.product_merge(_osum(A), _osum(B))
    staged = pl.merge(pl.outer_product(GA, GB), mode=COMP).export()
    parity.assert_compensated(staged, ref)
    forced = pl.outer_product_merged(GA, GB, mode=COMP, key_bits=8).export()
    parity.assert_compensated(forced, ref)
    parity.assert_sorted_by_key(forced, key_bits=8)


def test_compensated_with_drop():
    A, B = synth.workload2(m1=120, m2=100)
    thr = 1e-4
    g = pl.outer_product_merged(_gsum(A), _gsum(B), mode=COMP, drop_abs=thr).export()
    full = O.product_merge(_osum(A), _osum(B))
    assert np.all(np.abs(g["coef"].astype(np.complex128)) >= thr)
    # strings clear of the threshold by the FP32 error bound agree
    band = np.abs(np.abs(full.coef) - thr) <= 1e-6 * thr + 4.5 * parity.U32 * full.mass
    gk = set(map(tuple, zip(map(bytes, g["x"]), map(bytes, g["z"]))))
    sure = {(full.x[u].tobytes(), full.z[u].tobytes()) for u in np.nonzero(~band)[0]}
    keep = {(full.x[u].tobytes(), full.z[u].tobytes())
            for u in np.nonzero(np.abs(full.coef) >= thr)[0]}
    assert (gk & sure) == (keep & sure)


def test_fused_drop_matches_general_path():
    """Plain FP64 with a drop threshold: the fused path (merge, then drop
    compaction) and the general pipeline keep the same strings."""
    A, B = synth.workload2(m1=150, m2=90)
    GA, GB = _gsum(A), _gsum(B)
    thr = 3e-5
    fused = pl.outer_product_merged(GA, GB, drop_abs=thr).export()
    staged = pl.merge(pl.outer_product(GA, GB), drop_abs=thr).export()
    ref = O.product_merge(_osum(A), _osum(B), drop_abs=thr)
    parity.assert_sorted_by_key(fused)
    full = O.product_merge(_osum(A), _osum(B))
    band = np.abs(np.abs(full.coef) - thr) <= 1e-9 * thr
    if not np.any(band):
        parity.assert_merged_fp64(fused, ref)
        parity.assert_merged_fp64(staged, ref)
    assert np.array_equal(fused["x"], staged["x"]) and np.array_equal(fused["z"], staged["z"])

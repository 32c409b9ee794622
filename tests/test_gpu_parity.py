"""GPU path vs the CPU oracle through the C ABI (needs an MI355X).

Sizes are chosen so the oracle finishes in seconds while the GPU kernels
still see many tiles and a ragged tail; the full-size workloads are checked
on sampled outputs in test_gpu_fullsize.py."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _gsum(d, dtype=None):
    return pl.PauliSum.from_dict(d, dtype=dtype)


def _rand(seed, n, m, wmax=None, distinct=True):
    return synth.random_sum(synth.rng_for(700, seed), n, m, wmax=wmax, distinct_strings=distinct)


def _dup_sum(seed, n, m, pool):
    """m terms drawn from a pool of `pool` strings: many duplicates."""
    rng = synth.rng_for(701, seed)
    base = synth.random_sum(rng, n, pool)
    idx = rng.integers(0, pool, size=m)
    return {"n": n, "x": base["x"][idx], "z": base["z"][idx],
            "phase": rng.integers(0, 4, size=m).astype(np.uint8),
            "coef": rng.standard_normal(m) + 1j * rng.standard_normal(m)}


# ------------------------------------------------------------ outer product

@pytest.mark.parametrize("n,m1,m2", [(1, 3, 5), (16, 300, 257), (64, 100, 130), (65, 77, 91),
                                     (130, 64, 65), (500, 200, 151)])
def test_outer_product_bitexact(n, m1, m2):
    A, B = _rand(n, n, m1), _rand(n + 1, n, m2)
    g = pl.outer_product(_gsum(A), _gsum(B)).export()
    x, z, ph, c = O.outer_product(_osum(A), _osum(B))
    assert np.array_equal(g["x"], x) and np.array_equal(g["z"], z)
    assert np.array_equal(g["phase"], ph)
    assert np.array_equal(g["coef"].view(np.uint64), c.view(np.uint64))
    assert np.array_equal(g["fp"], parity.fingerprint(x, z))


@pytest.mark.parametrize("n", [64, 128, 512, 1024])
def test_fused_full_words(n):
    """Qubit counts that fill their last word (no spare bits in a row),
    up to the largest width the library takes: the fused product of two
    sums with phases and repeated strings, over a few buckets with a ragged
    last one, in FP64 and in the precision form."""
    A, B = _dup_sum(30 + n, n, 130, 90), _dup_sum(31 + n, n, 117, 80)
    GA, GB = _gsum(A), _gsum(B)
    ref = O.product_merge(_osum(A), _osum(B))
    g = pl.outer_product_merged(GA, GB).export()
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)
    g32 = pl.outer_product_merged(GA, GB, mode=pl.COMPENSATED, tau=0.3).export()
    parity.assert_compensated(g32, ref)


def test_outer_product_c64_bitexact():
    n = 200
    A, B = _rand(1, n, 70), _rand(2, n, 90)
    A["coef"] = A["coef"].astype(np.complex64)
    B["coef"] = B["coef"].astype(np.complex64)
    g = pl.outer_product(_gsum(A), _gsum(B)).export()
    x, z, ph, _ = O.outer_product(_osum(A), _osum(B))
    assert np.array_equal(g["x"], x) and np.array_equal(g["phase"], ph)
    # float32 product, rounded operation by operation
    a = np.tile(A["coef"], B["coef"].size)
    b = np.repeat(B["coef"], A["coef"].size)
    re = a.real * b.real - a.imag * b.imag
    im = a.real * b.imag + a.imag * b.real
    assert g["coef"].dtype == np.complex64
    assert np.array_equal(g["coef"].real, re) and np.array_equal(g["coef"].imag, im)


def test_outer_product_empty_and_self():
    A = _rand(3, 40, 50)
    E = {"n": 40, "x": np.zeros((0, 1), np.uint64), "z": np.zeros((0, 1), np.uint64),
         "phase": np.zeros(0, np.uint8), "coef": np.zeros(0, np.complex128)}
    GA = _gsum(A)
    assert pl.outer_product(GA, _gsum(E)).m == 0
    assert pl.outer_product(_gsum(E), GA).m == 0
    g = pl.outer_product(GA, GA).export()
    x, z, ph, c = O.outer_product(_osum(A), _osum(A))
    assert np.array_equal(g["x"], x) and np.array_equal(g["phase"], ph)


def test_shape_errors():
    A, B = _rand(4, 10, 5), _rand(5, 11, 5)
    with pytest.raises(pl.PauliError) as e:
        pl.outer_product(_gsum(A), _gsum(B))
    assert e.value.status == "SHAPE"
    C = dict(_rand(6, 10, 5))
    C["coef"] = C["coef"].astype(np.complex64)
    with pytest.raises(pl.PauliError) as e:
        pl.outer_product_merged(_gsum(A), _gsum(C))
    assert e.value.status == "SHAPE"


# -------------------------------------------------------------------- merge

@pytest.mark.parametrize("n,m,pool", [(1, 50, 4), (3, 2000, 60), (16, 5000, 700),
                                      (100, 3000, 2999), (500, 4097, 1500)])
def test_merge_term_source(n, m, pool):
    S = _dup_sum(n, n, m, pool)
    g = pl.merge(_gsum(S)).export()
    ref = O.merge(_osum(S))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


def test_merge_of_outer_product_equals_fused():
    A, B = _rand(7, 30, 120), _rand(8, 30, 140)
    GA, GB = _gsum(A), _gsum(B)
    staged = pl.merge(pl.outer_product(GA, GB)).export()
    fused = pl.outer_product_merged(GA, GB).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_merged_fp64(staged, ref)
    parity.assert_merged_fp64(fused, ref)
    assert np.array_equal(staged["x"], fused["x"]) and np.array_equal(staged["fp"], fused["fp"])


# -------------------------------------------------------------------- fused

def test_fused_workload1_shape():
    A, B = synth.workload1(m=400)
    g = pl.outer_product_merged(_gsum(A), _gsum(B)).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


def test_fused_workload2_shape():
    A, B = synth.workload2(m1=300, m2=257)
    g = pl.outer_product_merged(_gsum(A), _gsum(B)).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


def test_fused_hermitian_square():
    """H*H: a == b; anticommuting pairs cancel exactly, coef(I) = sum c^2."""
    H = synth.workload3(m=400)
    G = _gsum(H)
    g = pl.outer_product_merged(G, G).export()
    ref = O.product_merge(_osum(H), _osum(H))
    parity.assert_merged_fp64(g, ref)
    assert np.all(g["coef"].imag == 0)


@pytest.mark.parametrize("n,m,pool", [(1, 40, 4), (5, 700, 300), (64, 900, 900),
                                      (100, 1500, 1400), (200, 1100, 700), (500, 1300, 1300),
                                      (1000, 300, 250)])
def test_fused_self_product(n, m, pool):
    """S*S with complex coefficients, arbitrary phases and repeated strings:
    the fused path takes each unordered pair once (the symmetric form)."""
    S = _dup_sum(90 + n, n, m, pool)
    G = _gsum(S)
    g = pl.outer_product_merged(G, G).export()
    ref = O.product_merge(_osum(S), _osum(S))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)
    g32 = pl.outer_product_merged(G, G, mode=pl.COMPENSATED, tau=0.3).export()
    parity.assert_compensated(g32, ref)


@pytest.mark.parametrize("n,m", [(40, 2600), (500, 3000)])
def test_fused_self_product_matches_two_operand_form(n, m):
    """At sizes with more than 256 buckets: S*S (symmetric form) against S*S'
    with S' a separate copy of S (every ordered pair generated)."""
    S = _dup_sum(95 + n, n, m, m // 2)
    G, G2 = _gsum(S), _gsum(S)
    sym = pl.outer_product_merged(G, G).export()
    full = pl.outer_product_merged(G, G2).export()
    for f in ("x", "z", "phase", "fp"):
        assert np.array_equal(sym[f], full[f])
    bound = 1e-12 * 64 * np.max(np.abs(S["coef"])) ** 2
    assert np.max(np.abs(sym["coef"] - full["coef"])) <= bound
    pl.trim_memory()


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_fused_small_n_heavy_duplicates(n):
    A, B = _rand(20 + n, n, 4 ** n, wmax=n), _dup_sum(30 + n, n, 300, min(4 ** n, 10))
    g = pl.outer_product_merged(_gsum(A), _gsum(B)).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)


def test_fused_integer_coefficients_bitexact():
    """Small-integer coefficients: every partial sum is exact in FP64, so the
    merged coefficients must equal the oracle's exactly."""
    rng = synth.rng_for(702)
    A, B = _rand(40, 24, 500, wmax=3), _rand(41, 24, 400, wmax=3)
    A["coef"] = (rng.integers(-64, 65, 500) + 1j * rng.integers(-64, 65, 500)).astype(np.complex128)
    B["coef"] = (rng.integers(-64, 65, 400) + 1j * rng.integers(-64, 65, 400)).astype(np.complex128)
    g = pl.outer_product_merged(_gsum(A), _gsum(B)).export()
    ref = O.product_merge(_osum(A), _osum(B))
    gi, ri = parity.align(g["x"], g["z"], ref.x, ref.z)
    assert np.array_equal(g["coef"][gi], ref.coef[ri])


@pytest.mark.parametrize("key_bits", [4, 8, 20])
def test_forced_fingerprint_collisions(key_bits):
    """A narrow sort key puts many distinct strings into each key run; the
    packed-word verification must still separate them exactly."""
    A, B = _rand(50, 70, 90), _rand(51, 70, 80)
    g = pl.outer_product_merged(_gsum(A), _gsum(B), key_bits=key_bits).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g, key_bits=key_bits)
    S = _dup_sum(52, 70, 3000, 500)
    gm = pl.merge(_gsum(S), key_bits=key_bits).export()
    parity.assert_merged_fp64(gm, O.merge(_osum(S)))


def test_drop_threshold():
    A, B = synth.workload2(m1=120, m2=100)
    thr = 1e-4
    g = pl.outer_product_merged(_gsum(A), _gsum(B), drop_abs=thr).export()
    ref = O.product_merge(_osum(A), _osum(B), drop_abs=thr)
    full = O.product_merge(_osum(A), _osum(B))
    assert np.all(np.abs(g["coef"]) >= thr)
    # strings near the threshold may fall either way; everything else agrees
    band = np.abs(np.abs(full.coef) - thr) <= 1e-9 * thr
    keep_ref = {k for k, v in full.as_dict().items() if abs(v[0]) >= thr}
    gkeys = set(map(tuple, zip(map(bytes, g["x"]), map(bytes, g["z"]))))
    sure = {(full.x[u].tobytes(), full.z[u].tobytes()) for u in np.nonzero(~band)[0]}
    assert (gkeys & sure) == (keep_ref & sure)
    assert len(ref.x) == len(keep_ref)


def test_empty_and_single_term():
    n = 9
    E = {"n": n, "x": np.zeros((0, 1), np.uint64), "z": np.zeros((0, 1), np.uint64),
         "phase": np.zeros(0, np.uint8), "coef": np.zeros(0, np.complex128)}
    A = _rand(60, n, 1)
    assert pl.outer_product_merged(_gsum(E), _gsum(A)).m == 0
    assert pl.merge(_gsum(E)).m == 0
    g = pl.outer_product_merged(_gsum(A), _gsum(A)).export()
    ref = O.product_merge(_osum(A), _osum(A))
    parity.assert_merged_fp64(g, ref)


def test_zero_coefficients_kept_unless_dropped():
    n = 4
    x = np.array([[1], [1]], np.uint64)
    z = np.array([[0], [0]], np.uint64)
    S = {"n": n, "x": x, "z": z, "phase": np.array([0, 2], np.uint8),
         "coef": np.array([1.5 + 0j, 1.5 + 0j])}
    g = pl.merge(_gsum(S)).export()
    assert g["x"].shape[0] == 1 and g["coef"][0] == 0
    # |c| < t is decided exactly: a zero sum lies below any positive
    # threshold, also one whose square underflows
    assert pl.merge(_gsum(S), drop_abs=1e-300).m == 0
    assert pl.merge(_gsum(S), drop_abs=5e-324).m == 0
    assert pl.merge(_gsum(S), drop_abs=0.0).m == 1


def test_drop_is_exact():
    """Section III-B truncation, |c| < t strictly, on exact ties, near ties,
    subnormals and thresholds whose squares under- or overflow: the kept set
    equals exact rational arithmetic and the oracle's."""
    from tests.test_oracle_truncation import _cases, _exact_below
    by_t = {}
    for re, im, t in _cases():
        by_t.setdefault(t, []).append((re, im))
    ts = sorted(by_t)
    ts = [t for k, t in enumerate(ts) if len(by_t[t]) > 1 or k % 12 == 0]
    n = 40
    for t in ts:
        vals = by_t[t]
        m = len(vals)
        S = {"n": n, "x": np.arange(1, m + 1, dtype=np.uint64).reshape(m, 1),
             "z": np.zeros((m, 1), np.uint64), "phase": np.zeros(m, np.uint8),
             "coef": np.array([complex(re, im) for re, im in vals], np.complex128)}
        got = {int(v) for v in pl.merge(_gsum(S), drop_abs=t).export()["x"][:, 0]}
        ref = {int(v) for v in O.merge(_osum(S), drop_abs=t).x[:, 0]}
        want = {u + 1 for u, (re, im) in enumerate(vals) if not _exact_below(re, im, t)}
        assert got == want == ref, t


def test_determinism():
    A, B = synth.workload2(m1=200, m2=300)
    GA, GB = _gsum(A), _gsum(B)
    r1 = pl.outer_product_merged(GA, GB).export()
    r2 = pl.outer_product_merged(GA, GB).export()
    for k in ("x", "z", "fp"):
        assert np.array_equal(r1[k], r2[k])
    assert np.array_equal(r1["coef"].view(np.uint64), r2["coef"].view(np.uint64))


def test_device_input_pointers():
    import torch
    A = _rand(70, 77, 64)
    dA = {"n": 77, "x": torch.from_numpy(A["x"].view(np.int64)).cuda(),
          "z": torch.from_numpy(A["z"].view(np.int64)).cuda(),
          "phase": torch.from_numpy(A["phase"]).cuda(),
          "coef": torch.from_numpy(A["coef"]).cuda()}
    G = pl.PauliSum.create(77, dA["x"], dA["z"], dA["phase"], dA["coef"])
    e = G.export()
    assert np.array_equal(e["x"], A["x"]) and np.array_equal(e["coef"], A["coef"])
    bad = dA["x"].clone()
    bad[3, 1] = 1 << 20  # qubit 84 >= 77
    with pytest.raises(pl.PauliError) as err:
        pl.PauliSum.create(77, bad, dA["z"], dA["phase"], dA["coef"])
    assert err.value.status == "INVALID"

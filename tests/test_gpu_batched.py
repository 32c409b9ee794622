"""The batched form (pauli_outer_product_batched) against the CPU oracle
and against single fused products, through the C ABI."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _plan():
    # mixed qubit counts and uneven term counts, as in the batched workload
    return [(64, 120, 300), (500, 250, 90), (128, 33, 410), (256, 200, 200), (500, 1, 77),
            (64, 300, 1)]


@pytest.mark.parametrize("mode", [pl.PLAIN, pl.COMPENSATED])
def test_batched_mixed_widths_match_oracle(mode):
    pairs = [synth.workload4_batch(b, n, m1, m2) for b, (n, m1, m2) in enumerate(_plan())]
    if mode == pl.PLAIN:
        for A, B in pairs:
            A["coef"] = A["coef"].astype(np.complex128)
            B["coef"] = B["coef"].astype(np.complex128)
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    outs = pl.outer_product_batched(GA, GB, mode=mode)
    assert len(outs) == len(pairs)
    for (A, B), o in zip(pairs, outs):
        g = o.export()
        ref = O.product_merge(_osum(A), _osum(B))
        if mode == pl.PLAIN:
            parity.assert_merged_fp64(g, ref)
        else:
            parity.assert_compensated(g, ref, input_rounding=False)
        parity.assert_sorted_by_key(g)


@pytest.mark.parametrize("mode", [pl.PLAIN, pl.COMPENSATED])
def test_batched_wide_strings(mode):
    """Products above 512 qubits (the widest class, 16 words) beside narrower
    ones in one batch, against the oracle."""
    plan = [(700, 90, 140), (1024, 120, 75), (513, 40, 60), (64, 100, 80)]
    pairs = [synth.workload4_batch(600 + b, n, m1, m2) for b, (n, m1, m2) in enumerate(plan)]
    for k, (A, B) in enumerate(pairs):
        pairs[k] = (dict(A, coef=A["coef"].astype(np.complex128)),
                    dict(B, coef=B["coef"].astype(np.complex128)))
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    outs = pl.outer_product_batched(GA, GB, mode=mode, tau=0.3)
    for (A, B), o in zip(pairs, outs):
        g = o.export()
        ref = O.product_merge(_osum(A), _osum(B))
        if mode == pl.PLAIN:
            parity.assert_merged_fp64(g, ref)
        else:
            parity.assert_compensated(g, ref)
        parity.assert_sorted_by_key(g)


def test_batched_autotune_gives_the_single_product_result():
    """Products above the tuning threshold (2^22) are run at three bucket
    widths; the kept result equals the plain single call bit for bit."""
    pairs = [synth.workload4_batch(100 + b, 500, 2100, 2050) for b in range(2)]
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    outs = pl.outer_product_batched(GA, GB, mode=pl.COMPENSATED)
    for a, b, o in zip(GA, GB, outs):
        one = pl.outer_product_merged(a, b, mode=pl.COMPENSATED).export()
        g = o.export()
        for k in ("x", "z", "fp"):
            assert np.array_equal(g[k], one[k])
        assert np.array_equal(g["coef"].view(np.uint32), one["coef"].view(np.uint32))


@pytest.mark.parametrize("bits", [3, 9, 14])
def test_batched_explicit_bucket_bits(bits):
    A, B = synth.workload2(m1=300, m2=210)
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    (o,) = pl.outer_product_batched([GA], [GB], tune=bits)
    parity.assert_merged_fp64(o.export(), O.product_merge(_osum(A), _osum(B)))


def test_batched_errors_and_empty():
    assert pl.outer_product_batched([], []) == []
    A, B = synth.workload4_batch(0, 64, 20, 30)
    C, _ = synth.workload4_batch(1, 128, 20, 30)
    GA, GB, GC = (pl.PauliSum.from_dict(d) for d in (A, B, C))
    with pytest.raises(pl.PauliError) as e:
        pl.outer_product_batched([GA, GA], [GB, GC])
    assert e.value.status == "SHAPE"
    with pytest.raises(pl.PauliError) as e:
        pl.outer_product_batched([GA], [GB], tune=17)
    assert e.value.status == "INVALID"


def _pairs_mixed():
    """Mixed widths and precisions, a sum times itself, an empty side."""
    plan = [(64, 120, 300), (500, 250, 90), (128, 33, 410), (256, 200, 200), (500, 1, 77),
            (64, 300, 1), (130, 150, 170)]
    pairs = [synth.workload4_batch(200 + b, n, m1, m2) for b, (n, m1, m2) in enumerate(plan)]
    for k in (1, 3, 6):  # complex128 products in the same batch
        A, B = pairs[k]
        pairs[k] = (dict(A, coef=A["coef"].astype(np.complex128)),
                    dict(B, coef=B["coef"].astype(np.complex128)))
    G = [(pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)) for A, B in pairs]
    # a sum times itself (one handle on both sides), and an empty right side
    S = synth.workload4_batch(300, 256, 180, 1)[0]
    GS = pl.PauliSum.from_dict(S)
    E = {"n": 64, "x": np.zeros((0, 1), np.uint64), "z": np.zeros((0, 1), np.uint64),
         "phase": None, "coef": np.zeros(0, np.complex64)}
    pairs += [(S, S), (pairs[0][0], E)]
    G += [(GS, GS), (G[0][0], pl.PauliSum.from_dict(E))]
    return pairs, [a for a, _ in G], [b for _, b in G]


def test_batched_plan_graph_replays_match_oracle():
    """The plan's graph is replayed three times (results taken after the
    second and third runs, the second run writing fresh output blocks);
    every product equals the oracle and the single fused call."""
    pairs, GA, GB = _pairs_mixed()
    P = pl.BatchPlan(GA, GB, mode=pl.COMPENSATED, tau=0.3)
    P.run()
    P.run()
    first = P.results()
    P.run()
    second = P.results()
    P.destroy()
    for t, ((A, B), o1, o2) in enumerate(zip(pairs, first, second)):
        g1, g2 = o1.export(), o2.export()
        one = pl.outer_product_merged(GA[t], GB[t], mode=pl.COMPENSATED, tau=0.3).export()
        for k in ("x", "z", "fp", "phase"):
            assert np.array_equal(g1[k], one[k]), (t, k)
            assert np.array_equal(g2[k], one[k]), (t, k)
        assert np.array_equal(g1["coef"].view(np.uint32), one["coef"].view(np.uint32))
        assert np.array_equal(g2["coef"].view(np.uint32), one["coef"].view(np.uint32))
        ref = O.product_merge(_osum(A), _osum(B))
        parity.assert_compensated(g1, ref, input_rounding=A["coef"].dtype == np.complex128)
    # results stay valid after the plan is gone; results without a run fail
    assert all(o.m >= 0 for o in first)
    P2 = pl.BatchPlan(GA[:2], GB[:2])
    with pytest.raises(pl.PauliError) as e:
        P2.results()
    assert e.value.status == "INVALID"


@pytest.mark.parametrize("shape", [{"bucket_records": 300}, {"bucket_records": 8000, "class_bits": 2},
                                   {"expand_parts": 1}, {"expand_parts": 8, "class_bits": 5}])
def test_batched_launch_shapes(shape):
    """Every launch shape computes the same products (FP64 against the
    oracle; the sum times itself and the empty side included)."""
    pairs, GA, GB = _pairs_mixed()
    outs = pl.outer_product_batched(GA, GB, tune=shape)
    for (A, B), o in zip(pairs, outs):
        g = o.export()
        ref = O.product_merge(_osum(A), _osum(B))
        if A["coef"].dtype == np.complex128:
            parity.assert_merged_fp64(g, ref)
        else:  # complex64 inputs, plain FP32 sums
            gi, ri = parity.align(g["x"], g["z"], ref.x, ref.z)
            err = np.abs(g["coef"][gi] - ref.coef[ri])
            assert np.all(err <= 1e-5 * np.maximum(ref.mass[ri], 1e-30))
        parity.assert_sorted_by_key(g)


def test_batched_drop_and_tune_file(tmp_path):
    pairs, GA, GB = _pairs_mixed()
    outs = pl.outer_product_batched(GA, GB, drop_abs=0.05)
    for (A, B), o in zip(pairs, outs):
        ref = O.product_merge(_osum(A), _osum(B), drop_abs=0.05)
        g = o.export()
        gi, ri = parity.align(g["x"], g["z"], ref.x, ref.z)
    f = tmp_path / "tune.txt"
    pl.tune_save(str(f))
    text = f.read_text()
    assert text.startswith("#") and len(text.splitlines()) >= 2
    pl.tune_load(str(f))
    bad = tmp_path / "bad.txt"
    bad.write_text("1 2 3\n")
    with pytest.raises(pl.PauliError) as e:
        pl.tune_load(str(bad))
    assert e.value.status == "INVALID"


def _threshold_between(vals, q):
    """A threshold halfway between two neighbouring distinct moduli near
    quantile q, so that no modulus lies within rounding of it."""
    u = np.unique(vals)
    k = max(1, min(len(u) - 1, int(q * len(u))))
    t = 0.5 * (u[k - 1] + u[k])
    assert np.min(np.abs(vals - t)) > 1e-9 * t
    return float(t)


@pytest.mark.parametrize("key_bits", [0, 32])
def test_batched_drop_is_one_compaction_of_the_kept_terms(key_bits):
    """The drop of a batched call keeps, product by product and in order,
    exactly the terms of the undropped batched result with |c| >= drop_abs,
    every array bit for bit; products span several 4096-term tiles with a
    ragged end, one product loses every term, and with a 32-bit key one
    product collides and is recomputed (its drop applied there)."""
    plan = [(500, 150, 100), (64, 300, 40), (128, 1, 3), (500, 90, 130), (256, 70, 70),
            (500, 1000, 1000)]
    pairs = [synth.workload4_batch(700 + b, n, m1, m2) for b, (n, m1, m2) in enumerate(plan)]
    for k in (0, 2, 5):
        A, B = pairs[k]
        pairs[k] = (dict(A, coef=A["coef"].astype(np.complex128)),
                    dict(B, coef=B["coef"].astype(np.complex128)))
    A, B = pairs[4]
    pairs[4] = (dict(A, coef=(A["coef"] * np.float32(1e-9)).astype(A["coef"].dtype)), B)
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    full = [o.export() for o in pl.outer_product_batched(GA, GB, key_bits=key_bits)]
    mods = np.concatenate([np.abs(g["coef"].astype(np.complex128)) for g in full])
    t = _threshold_between(np.concatenate(
        [np.abs(g["coef"].astype(np.complex128)) for k, g in enumerate(full) if k != 4]), 0.4)
    assert np.min(np.abs(mods - t)) > 1e-9 * t
    assert np.max(np.abs(full[4]["coef"].astype(np.complex128))) < t
    outs = pl.outer_product_batched(GA, GB, drop_abs=t, key_bits=key_bits)
    kept_total = 0
    for g, o in zip(full, outs):
        d = o.export()
        keep = np.abs(g["coef"].astype(np.complex128)) >= t
        kept_total += int(keep.sum())
        for k in ("x", "z", "fp", "phase"):
            assert np.array_equal(d[k], g[k][keep]), k
        assert d["coef"].dtype == g["coef"].dtype
        assert np.array_equal(d["coef"].view(np.uint8), g["coef"][keep].view(np.uint8))
    assert len(outs[4].export()["x"]) == 0
    assert 0 < kept_total < len(mods)
    assert len(full[0]["x"]) > 2 * 4096


def test_batched_plan_drop_matches_the_eager_call():
    """A graph plan with a drop threshold: the results of two replays (each
    compacted once per class) equal the eager batched call bit for bit."""
    pairs, GA, GB = _pairs_mixed()
    eager = [o.export() for o in pl.outer_product_batched(GA, GB, drop_abs=0.02)]
    P = pl.BatchPlan(GA, GB, drop_abs=0.02)
    runs = []
    for _ in range(2):
        P.run()
        runs.append([o.export() for o in P.results()])
    P.destroy()
    for res in runs:
        for t, (g, e) in enumerate(zip(res, eager)):
            for k in ("x", "z", "fp", "phase"):
                assert np.array_equal(g[k], e[k]), (t, k)
            assert np.array_equal(g["coef"].view(np.uint8), e["coef"].view(np.uint8)), t


@pytest.mark.parametrize("tau", [1e-3, 0.3])
def test_batched_compensated_remerge(tau):
    """Cancelling segments in the batched launch sequence: two Hermitian
    squares (sums times themselves, exact cancellations) and a product
    whose FP32 inputs lose 2^-30 (the FP64 re-merge must recover it exactly)
    in one batch; the re-merge reads each product's own operands."""
    H1, H2 = synth.workload3(m=400), synth.workload3(m=260)
    G1, G2 = pl.PauliSum.from_dict(H1), pl.PauliSum.from_dict(H2)
    n = 5
    A = {"n": n, "x": np.array([[0], [1]], np.uint64), "z": np.zeros((2, 1), np.uint64),
         "phase": None, "coef": np.array([1.0 + 2.0 ** -30, -1.0], np.complex128)}
    B = {"n": n, "x": np.array([[0], [1]], np.uint64), "z": np.zeros((2, 1), np.uint64),
         "phase": None, "coef": np.array([1.0, 1.0], np.complex128)}
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    outs = pl.outer_product_batched([G1, GA, G2], [G1, GB, G2], mode=pl.COMPENSATED, tau=tau)
    for H, o in ((H1, outs[0]), (H2, outs[2])):
        g = o.export()
        ref = O.product_merge(_osum(H), _osum(H))
        parity.assert_compensated(g, ref)
        gi, ri = parity.align(g["x"], g["z"], ref.x, ref.z)
        zero = ref.coef[ri] == 0
        assert np.any(zero)
        assert np.all(np.abs(g["coef"][gi][zero]) <= 1e-12 * ref.mass[ri][zero])
    r = outs[1].export()
    ref = O.product_merge(_osum(A), _osum(B))
    gi, ri = parity.align(r["x"], r["z"], ref.x, ref.z)
    assert np.all(r["coef"] == np.complex64(2.0 ** -30))


def test_batched_collisions_recomputed():
    """A 32-bit key makes fingerprint collisions certain in 1e6-record
    products: those products are recomputed by the general pipeline after
    the sequence and still equal the oracle; keys below 30 bits are refused."""
    plan = [(128, 1000, 1000), (500, 900, 1100), (64, 40, 50)]
    pairs = [synth.workload4_batch(400 + b, n, m1, m2) for b, (n, m1, m2) in enumerate(plan)]
    for k, (A, B) in enumerate(pairs):
        pairs[k] = (dict(A, coef=A["coef"].astype(np.complex128)),
                    dict(B, coef=B["coef"].astype(np.complex128)))
    GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
    GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
    outs = pl.outer_product_batched(GA, GB, key_bits=32)
    for (A, B), o in zip(pairs, outs):
        g = o.export()
        parity.assert_merged_fp64(g, O.product_merge(_osum(A), _osum(B)))
        parity.assert_sorted_by_key(g, key_bits=32)
    with pytest.raises(pl.PauliError) as e:
        pl.outer_product_batched(GA, GB, key_bits=29)
    assert e.value.status == "INVALID"

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

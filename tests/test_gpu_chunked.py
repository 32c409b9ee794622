"""merge(a b) with |a| |b| at or beyond 2^32 products, beyond the 32-bit
pair index of one fused pipeline (Section III-H's sort-and-combine over the
products of Section IV-C's outer product): the call runs the fused pipeline
over ranges of one operand's terms and merges the merged ranges once more.

At n = 6 there are at most 4,096 strings, so 4.6e9 products merge into a few
thousand terms; with Gaussian-integer coefficients every sum is exact in
FP64 whatever its order, so the result must equal, exactly, the same product
formed from the merged operands (at most 4,096 terms each, one fused call),
and sampled terms must equal the oracle's exact coefficients."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _int_sum(rng, n, m):
    x = rng.integers(0, 1 << n, (m, 1)).astype(np.uint64)
    z = rng.integers(0, 1 << n, (m, 1)).astype(np.uint64)
    c = (rng.integers(-4, 5, m) + 1j * rng.integers(-4, 5, m)).astype(np.complex128)
    ph = rng.integers(0, 4, m).astype(np.uint8)
    return {"n": n, "x": x, "z": z, "phase": ph, "coef": c}


def _same_terms(g, r):
    for k in ("x", "z", "fp"):
        assert np.array_equal(g[k], r[k]), k
    assert not g["phase"].any() and not r["phase"].any()
    assert np.array_equal(g["coef"], r["coef"])  # exact (zeros of either sign equal)


def test_product_beyond_the_pair_index():
    rng = synth.rng_for(760)
    A, B = _int_sum(rng, 6, 70_000), _int_sum(rng, 6, 66_000)
    assert A["x"].shape[0] * B["x"].shape[0] >= 1 << 32
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    try:
        got = pl.outer_product_merged(GA, GB).export()
        MA, MB = pl.merge(GA), pl.merge(GB)
        ref = pl.outer_product_merged(MA, MB).export()
        _same_terms(got, ref)
        assert got["x"].shape[0] > 1000
        # sampled terms against the oracle's exact sums over the 4.6e9 pairs
        q = rng.choice(got["x"].shape[0], 24, replace=False)
        oa = O.Sum(6, A["x"], A["z"], A["phase"], A["coef"])
        ob = O.Sum(6, B["x"], B["z"], B["phase"], B["coef"])
        c, mass, cnt = O.product_coeff(oa, ob, got["x"][q], got["z"][q])
        assert np.all(cnt > 0)
        assert np.array_equal(got["coef"][q], c)
        # the drop applies once, to the merged sum
        t = float(np.quantile(np.abs(ref["coef"]), 0.5)) + 0.5
        gd = pl.outer_product_merged(GA, GB, drop_abs=t).export()
        rd = pl.outer_product_merged(MA, MB, drop_abs=t).export()
        _same_terms(gd, rd)
        assert 0 < gd["x"].shape[0] < got["x"].shape[0]
        # the same product with the operands swapped in size (ranges of b)
        got2 = pl.outer_product_merged(GB, GA).export()
        _same_terms(got2, pl.outer_product_merged(MB, MA).export())
        # the precision form is refused beyond 2^32 products
        with pytest.raises(pl.PauliError) as e:
            pl.outer_product_merged(GA, GB, mode=pl.COMPENSATED)
        assert e.value.status == "OVERFLOW"
    finally:
        del GA, GB
        pl.trim_memory()

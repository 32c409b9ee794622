"""The hand-written sorts against a library sort on the device.

A merged sum is in ascending fingerprint order with one term per string,
so its fingerprint column must equal the distinct fingerprints of the
unmerged products, sorted by PyTorch's device sort (a library radix sort,
independent of this package).  The record counts cover the general merge's
full LSD radix sort (under 2^16 records), its partition + LDS bucket sort,
and the fused pipeline's generation into buckets."""
import pytest
import torch

import paper_2605_25974_amd as pl
import synth

pytestmark = pytest.mark.gpu

SIGN = -(1 << 63)  # int64 order of (u ^ SIGN) is the unsigned order of u


def _library_order(fp):
    """Distinct fingerprints (int64 views), unsigned ascending, by torch.sort."""
    s = torch.sort(fp ^ SIGN).values
    return torch.unique_consecutive(s)


@pytest.mark.parametrize("n,m1,m2", [(40, 30, 25), (130, 300, 200), (64, 400, 300), (500, 2000, 1500),
                                     (12, 1500, 1200)])
def test_merged_fingerprints_equal_library_sort(n, m1, m2):
    rng = synth.rng_for(770, n)
    A = synth.random_sum(rng, n, m1, wmax=6)
    B = synth.random_sum(rng, n, m2, wmax=6)
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    prods = pl.outer_product(GA, GB).export_torch()["fp"]
    want = _library_order(prods)
    merged = pl.merge(pl.outer_product(GA, GB)).export_torch()["fp"] ^ SIGN
    fused = pl.outer_product_merged(GA, GB).export_torch()["fp"] ^ SIGN
    assert torch.equal(merged, want)
    assert torch.equal(fused, want)

"""Error paths of the C ABI that need device sums: OVERFLOW for a pair
count beyond the 32-bit pair index, OOM under a memory budget (and a clean
state afterwards), CAPACITY when a result does not fit caller-owned
arrays."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def test_overflow_pair_index():
    n, m = 20, 1 << 16  # |a| |b| = 2^32: one more than the pair index holds
    rng = synth.rng_for(750)
    x, z = synth.random_weight(rng, n, m, 1, 4)
    S = {"n": n, "x": x, "z": z, "phase": None, "coef": np.ones(m, np.complex128)}
    G = pl.PauliSum.from_dict(S)
    small = pl.PauliSum.from_dict({"n": n, "x": x[:3], "z": z[:3], "phase": None,
                                   "coef": np.ones(3, np.complex128)})
    # (the plain fused product merges ranges beyond 2^32, tests/test_gpu_chunked.py)
    for call in (lambda: pl.outer_product(G, G),
                 lambda: pl.outer_product_merged(G, G, mode=pl.COMPENSATED),
                 lambda: pl.commutator(G, G),
                 lambda: pl.outer_product_batched([small, G], [small, G])):
        with pytest.raises(pl.PauliError) as e:
            call()
        assert e.value.status == "OVERFLOW"
    # one term fewer fits
    H = pl.PauliSum.from_dict({"n": n, "x": x[:-1], "z": z[:-1], "phase": None,
                               "coef": np.ones(m - 1, np.complex128)})
    assert pl.outer_product_merged(small, H).m > 0


def test_oom_under_budget_then_recovers():
    A, B = synth.workload2(m1=2000, m2=2000)
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    try:
        # 64 KiB: below what the two operands alone hold (about 0.6 MB), so the
        # first allocation of every call exceeds it whatever else is alive
        pl.set_memory_budget(1 << 16)
        for call in (lambda: pl.outer_product_merged(GA, GB), lambda: pl.outer_product(GA, GB),
                     lambda: pl.merge(GA)):
            with pytest.raises(pl.PauliError) as e:
                call()
            assert e.value.status == "OOM"
    finally:
        pl.set_memory_budget(0)
    # nothing leaked into later calls: the same product is right afterwards
    g = pl.outer_product_merged(GA, GB).export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)


def test_capacity_of_caller_arrays():
    import torch
    n = 40
    S = synth.random_sum(synth.rng_for(751), n, 500, wmax=6)
    G = pl.PauliSum.from_dict(S)
    U = pl.merge(G).m
    o = torch.zeros(U, dtype=torch.int64, device="cuda")
    c = torch.zeros(U, dtype=torch.complex128, device="cuda")
    p = torch.zeros(U, dtype=torch.uint8, device="cuda")
    with pytest.raises(pl.PauliError) as e:
        pl.merge_into(G, o, o, p, c, o, U - 1)
    assert e.value.status == "CAPACITY"


def test_narrow_key_bounded():
    """A key narrower than 52 bits is refused for more than 2^(key_bits + 12)
    records (the runs of equal keys are ordered one run per thread)."""
    S = synth.random_sum(synth.rng_for(752), 40, 9000, wmax=6)
    G = pl.PauliSum.from_dict(S)
    with pytest.raises(pl.PauliError) as e:
        pl.merge(G, key_bits=1)  # 9000 > 2^13 records
    assert e.value.status == "INVALID"
    parity.assert_merged_fp64(pl.merge(G, key_bits=2).export(), O.merge(_osum(S)))

"""The fused product's three bucket sorts on the same inputs, against the
CPU oracle (needs an MI355X): the LDS counting sort, the LDS radix sort that
takes a bucket with a bin of many equal keys, and the global-memory sort of a
bucket over the LDS capacity.  The inputs repeat one product string many
times: B holds a_i P for every term a_i of A, so every pair (i, i) gives the
string P."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d["phase"], d["coef"])


def _repeating(n, m, seed):
    rng = synth.rng_for(990, seed)
    A = synth.random_sum(rng, n, m)
    P = synth.random_sum(rng, n, 1)
    B = synth.random_sum(rng, n, m, distinct_strings=False)
    B["x"] = A["x"] ^ P["x"][0]
    B["z"] = A["z"] ^ P["z"][0]
    return A, B


@pytest.mark.parametrize("n,m,bits", [
    (70, 600, None),  # buckets of ~5600 records: the bin of P (600 equal keys) -> radix sort
    (70, 200, None),  # buckets of ~2500 records: a bin of 200 equal keys, ranked in the bin
    (500, 600, 10),   # small buckets, the same repeated string
    (70, 300, 2),     # 4 buckets of ~22,500 records: the global-memory sort
    (500, 300, 16),   # many tiny buckets
])
def test_repeated_string_paths(n, m, bits):
    A, B = _repeating(n, m, m + n + (bits or 0))
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    o = pl.outer_product_merged(GA, GB) if bits is None else \
        pl.outer_product_batched([GA], [GB], tune=bits)[0]
    g = o.export()
    ref = O.product_merge(_osum(A), _osum(B))
    parity.assert_merged_fp64(g, ref)
    # the repeated string is there once, with the sum of its m contributions
    assert len(np.unique(parity.row_keys(g["x"], g["z"]))) == len(g["x"])


def test_repeated_string_self_product():
    """A sum times itself (the symmetric form) where many pairs give the
    same strings: every term squared is the identity, and a_i (a_i P) = P."""
    A, B = _repeating(120, 400, 7)
    H = {k: np.concatenate([A[k], B[k]]) for k in ("x", "z", "phase", "coef")}
    H["n"] = 120
    G = pl.PauliSum.from_dict(H)
    g = pl.outer_product_merged(G, G).export()
    parity.assert_merged_fp64(g, O.product_merge(_osum(H), _osum(H)))

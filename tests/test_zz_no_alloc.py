"""pauli_merge_into, the merge that allocates nothing (temporaries in the
library's fixed device scratch array, result in caller-owned arrays),
against pauli_merge on the same inputs, through the C ABI."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth

pytestmark = pytest.mark.gpu


def _dup_sum(seed, n, m, pool):
    """m terms drawn from `pool` distinct strings (many duplicates)."""
    rng = synth.rng_for(760, seed)
    base = synth.random_sum(rng, n, pool, wmax=min(n, 40))
    idx = rng.integers(0, pool, size=m)
    return {"n": n, "x": base["x"][idx], "z": base["z"][idx],
            "phase": rng.integers(0, 4, size=m).astype(np.uint8),
            "coef": rng.standard_normal(m) + 1j * rng.standard_normal(m)}


def _into(G, n, ld, c64, **kw):
    """merge_into with fresh output tensors pre-filled with garbage."""
    import torch
    W = (n + 63) // 64
    ox = torch.full((W, ld), -1, dtype=torch.int64, device="cuda")
    oz = torch.full((W, ld), -1, dtype=torch.int64, device="cuda")
    oph = torch.full((ld,), 7, dtype=torch.uint8, device="cuda")
    oc = torch.full((ld,), float("nan"), dtype=torch.complex64 if c64 else torch.complex128,
                    device="cuda")
    ofp = torch.full((ld,), -1, dtype=torch.int64, device="cuda")
    cnt = pl.merge_into(G, ox, oz, oph, oc, ofp, ld, **kw)
    torch.cuda.synchronize()
    return {"x": ox[:, :cnt].T.contiguous().cpu().numpy().view(np.uint64),
            "z": oz[:, :cnt].T.contiguous().cpu().numpy().view(np.uint64),
            "phase": oph[:cnt].cpu().numpy(), "coef": oc[:cnt].cpu().numpy(),
            "fp": ofp[:cnt].cpu().numpy().view(np.uint64)}


def _same(got, ref):
    assert got["x"].shape == ref["x"].shape, (got["x"].shape, ref["x"].shape)
    for k in ("x", "z", "phase", "fp"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["coef"].dtype == ref["coef"].dtype
    assert np.array_equal(got["coef"].view(np.uint8), ref["coef"].view(np.uint8))


CASES = [
    # (n, terms, distinct strings, opts): the largest input it takes, then smaller ones
    (500, 1 << 20, 300000, {}),
    (70, 5000, 900, {}),
    (500, 200000, 50000, {"mode": pl.COMPENSATED, "drop_abs": 0.3}),
    (1000, 30000, 4000, {"drop_abs": 1.0}),
    (3, 4000, 64, {}),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_merge_into_matches_merge(case):
    """Two calls in a row (the second on a smaller input): each equals
    pauli_merge bit for bit (strings, phases, coefficients, fingerprints)."""
    for k in (case, (case + 1) % len(CASES)):
        n, m, pool, kw = CASES[k]
        S = _dup_sum(k, n, m, pool)
        G = pl.PauliSum.from_dict(S)
        ref = pl.merge(G, **kw).export()
        c64 = kw.get("mode") == pl.COMPENSATED
        got = _into(G, n, m, c64, **kw)
        _same(got, ref)
        assert got["x"].shape[0] < m  # duplicates merged
        G.destroy()


def test_merge_into_limits():
    import torch
    n = 64
    # output arrays too short for the merged result
    S = _dup_sum(9, n, 3000, 2500)
    G = pl.PauliSum.from_dict(S)
    U = pl.merge(G).m
    with pytest.raises(pl.PauliError) as e:
        _into(G, n, U - 1, False)
    assert e.value.status == "CAPACITY"
    _same(_into(G, n, U, False), pl.merge(G).export())  # exactly enough
    # more terms than the scratch array takes
    big = {"n": n, "x": np.zeros(((1 << 20) + 1, 1), np.uint64),
           "z": np.zeros(((1 << 20) + 1, 1), np.uint64), "phase": None,
           "coef": np.ones((1 << 20) + 1, np.complex128)}
    GB = pl.PauliSum.from_dict(big)
    with pytest.raises(pl.PauliError) as e:
        _into(GB, n, 16, False)
    assert e.value.status == "CAPACITY"
    # an empty sum merges to nothing
    E = {"n": n, "x": np.zeros((0, 1), np.uint64), "z": np.zeros((0, 1), np.uint64),
         "phase": None, "coef": np.zeros(0, np.complex128)}
    assert _into(pl.PauliSum.from_dict(E), n, 4, False)["x"].shape[0] == 0
    # a NULL output array is rejected
    o = torch.zeros(8, dtype=torch.int64, device="cuda")
    with pytest.raises(pl.PauliError) as e:
        pl.merge_into(G, 0, o, o, o, o, 8)
    assert e.value.status == "INVALID"

"""Full-size checks of the commutator and of the lexicographic order on the
benchmark's workloads, in its launch configuration (default options).  The
outputs are checked on sampled outputs recomputed exactly by the oracle and
by properties that hold at any size."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity

pytestmark = pytest.mark.gpu

SIGN = -(1 << 63)


def _torch():
    import torch
    return torch


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def test_fullsize_commutator_1e8_pairs():
    """[A, B] of the two 10,000-term n=500 sums: key order, no repeated
    string, sampled coefficients against the oracle's ab - ba for the same
    strings, and the strings of sampled anticommuting pairs present."""
    torch = _torch()
    A, B = synth.workload2()
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    out = pl.commutator(GA, GB)
    print("[A, B] of 10,000 x 10,000: %d terms" % out.m, flush=True)
    T = out.export_torch()
    out.destroy()
    fp = T["fp"] ^ SIGN
    assert bool(torch.all(fp[1:] >= fp[:-1])), "output is not in key order"
    assert bool(torch.all(T["phase"] == 0))
    U = fp.numel()
    rng = synth.rng_for(742, 0)
    idx = np.unique(np.concatenate([[0, U - 1], rng.integers(0, U, 300)]))
    it = torch.from_numpy(idx).to(fp.device)
    xq, zq = _u64(T["x"][it]), _u64(T["z"][it])
    got = T["coef"][it].cpu().numpy()
    ab, mab, cab = O.product_coeff(_osum(A), _osum(B), xq, zq)
    ba, mba, cba = O.product_coeff(_osum(B), _osum(A), xq, zq)
    ref = ab - ba
    assert np.all(cab > 0)
    assert np.all(_u64(T["fp"][it]) == parity.fingerprint(xq, zq))
    tol = np.maximum(1e-12 * np.abs(ref), 1e-14 * np.maximum(1.0, mab + mba))
    bad = np.nonzero(np.abs(got - ref) > tol)[0]
    assert bad.size == 0, (got[bad[:3]], ref[bad[:3]])
    # sampled anticommuting pairs: their string is in the output (a string
    # that an anticommuting pair gives is kept)
    i = rng.integers(0, A["x"].shape[0], 4000)
    j = rng.integers(0, B["x"].shape[0], 4000)
    ax, az, bx, bz = A["x"][i], A["z"][i], B["x"][j], B["z"][j]
    par = np.zeros(len(i), np.int64)
    for w in range(ax.shape[1]):
        v = (ax[:, w] & bz[:, w]) ^ (az[:, w] & bx[:, w])
        par += np.array([bin(int(u)).count("1") for u in v])
    anti = (par & 1) == 1
    assert anti.any()
    x, z = ax[anti] ^ bx[anti], az[anti] ^ bz[anti]
    fq = parity.fingerprint(x, z)
    q = torch.from_numpy(fq.view(np.int64)).to(fp.device) ^ SIGN
    pos = torch.searchsorted(fp, q).cpu().numpy()
    for s in range(x.shape[0]):
        p = int(pos[s])
        found = p < U and int(T["fp"][p]) == int(fq.view(np.int64)[s]) and \
            np.array_equal(_u64(T["x"][p]), x[s]) and np.array_equal(_u64(T["z"][p]), z[s])
        assert found, "string of anticommuting pair %d missing" % s


def test_fullsize_lex_of_merged_1e8():
    """The merged 1e8-product output put in lexicographic order: adjacent
    strings in order over all words, the same multiset of fingerprints,
    and sampled terms equal to the merged sum's term of the same string."""
    torch = _torch()
    A, B = synth.workload2()
    S = pl.outer_product_merged(pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B))
    L = pl.sort_lex(S)
    assert L.m == S.m
    pl.trim_memory()
    TS = S.export_torch()
    S.destroy()
    TL = L.export_torch()
    L.destroy()
    W = TL["x"].shape[1]
    cols = [TL["x"][:, w] for w in reversed(range(W))] + [TL["z"][:, w] for w in reversed(range(W))]
    lt = torch.zeros(TL["x"].shape[0] - 1, dtype=torch.bool, device=TL["x"].device)
    eq = torch.ones_like(lt)
    for col in cols:
        a = col[:-1] ^ SIGN
        b = col[1:] ^ SIGN
        lt |= eq & (a < b)
        eq &= a == b
    assert bool(torch.all(lt)), "not strictly increasing (the merged strings are distinct)"
    fs = torch.sort(TS["fp"] ^ SIGN).values
    fl = torch.sort(TL["fp"] ^ SIGN).values
    assert torch.equal(fs, fl)
    U = TL["fp"].numel()
    rng = synth.rng_for(743, 0)
    idx = torch.from_numpy(rng.integers(0, U, 2000)).to(fs.device)
    pos = torch.searchsorted(TS["fp"] ^ SIGN, TL["fp"][idx] ^ SIGN)
    for k in ("x", "z", "fp", "coef", "phase"):
        assert torch.equal(TS[k][pos], TL[k][idx]), k

"""Full-size checks on the workloads the benchmark times, in its launch
configuration (pauli_outer_product_merged, default options).  The outputs
(1e8 and 2e8 merged terms) are too large for the oracle to recompute whole,
so they are checked on sampled outputs, each recomputed exactly by the
oracle, and by properties that hold at any size: ascending key order, no
repeated string, every sampled pair's product present, and the precision
form's error against plain FP64 on every term."""
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


def _check_order_and_distinct(T):
    torch = _torch()
    fp = T["fp"] ^ SIGN  # unsigned order as signed order
    assert bool(torch.all(fp[1:] >= fp[:-1])), "merged output is not in key order"
    tie = torch.nonzero(T["fp"][1:] == T["fp"][:-1]).flatten()
    for k in tie.tolist()[:1000]:
        same = torch.equal(T["x"][k], T["x"][k + 1]) and torch.equal(T["z"][k], T["z"][k + 1])
        assert not same, "repeated string at %d" % k


def _check_sampled_coefficients(T, A, B, nsamp, seed):
    torch = _torch()
    U = T["fp"].numel()
    rng = synth.rng_for(740, seed)
    idx = np.unique(np.concatenate([[0, U - 1], rng.integers(0, U, nsamp)]))
    it = torch.from_numpy(idx).to(T["fp"].device)
    xq, zq = _u64(T["x"][it]), _u64(T["z"][it])
    got = T["coef"][it].cpu().numpy().astype(np.complex128)
    ref, mass, cnt = O.product_coeff(_osum(A), _osum(B), xq, zq)
    assert np.all(cnt > 0), "an output string is no product of the inputs"
    assert np.all(_u64(T["fp"][it]) == parity.fingerprint(xq, zq))
    tol = np.maximum(1e-12 * np.abs(ref), 1e-14 * np.maximum(1.0, mass))
    bad = np.nonzero(np.abs(got - ref) > tol)[0]
    assert bad.size == 0, (got[bad[:3]], ref[bad[:3]])


def _check_sampled_pairs(T, A, B, nsamp, seed):
    torch = _torch()
    rng = synth.rng_for(741, seed)
    i = rng.integers(0, A["x"].shape[0], nsamp)
    j = rng.integers(0, B["x"].shape[0], nsamp)
    x = A["x"][i] ^ B["x"][j]
    z = A["z"][i] ^ B["z"][j]
    fq = parity.fingerprint(x, z)
    keys = T["fp"] ^ SIGN
    q = torch.from_numpy(fq.view(np.int64)).to(keys.device) ^ SIGN
    pos = torch.searchsorted(keys, q).cpu().numpy()
    U = keys.numel()
    for s in range(nsamp):
        p = int(pos[s])
        found = False
        while p < U and int(T["fp"][p]) == int(fq.view(np.int64)[s]):
            if np.array_equal(_u64(T["x"][p]), x[s]) and np.array_equal(_u64(T["z"][p]), z[s]):
                found = True
                break
            p += 1
        assert found, "product of pair (%d, %d) missing" % (i[s], j[s])


def _comp_vs_plain(GA, GB, T):
    torch = _torch()
    C = pl.outer_product_merged(GA, GB, mode=pl.COMPENSATED, tau=0.3).export_torch()
    for k in ("x", "z", "fp"):
        assert torch.equal(C[k], T[k])
    r = T["coef"]
    g = C["coef"].to(torch.complex128)
    mag = r.abs()
    sel = mag >= 1e-6 * mag.max()
    err = float(((g - r).abs()[sel] / mag[sel]).max())
    print("precision form vs FP64, max rel err over |c| >= 1e-6 max: %.3e" % err)
    assert err <= 1e-6


def test_fullsize_1e8_products():
    A, B = synth.workload2()
    GA, GB = pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)
    out = pl.outer_product_merged(GA, GB)
    print("n=500 10,000 x 10,000: %d merged terms" % out.m, flush=True)
    pl.trim_memory()  # torch allocates the exported copy
    T = out.export_torch()
    out.destroy()
    _check_order_and_distinct(T)
    _check_sampled_coefficients(T, A, B, 300, 0)
    _check_sampled_pairs(T, A, B, 300, 0)
    _comp_vs_plain(GA, GB, T)


def test_fullsize_hermitian_square_4e8_products():
    H = synth.workload3()
    G = pl.PauliSum.from_dict(H)
    out = pl.outer_product_merged(G, G)
    print("H*H with 20,000 terms: %d merged terms" % out.m, flush=True)
    pl.trim_memory()  # torch allocates the exported copy
    T = out.export_torch()
    out.destroy()
    _check_order_and_distinct(T)
    _check_sampled_coefficients(T, H, H, 120, 1)
    _check_sampled_pairs(T, H, H, 200, 1)
    _comp_vs_plain(G, G, T)

"""The workloads at their stated sizes against the oracle:

* n = 16, 2,000 x 2,000 (4e6 products): the whole merged output;
* the 256 products of the batched form (term counts lognormal, median
  2,000, n in {64, 128, 256, 500}, complex64, compensated merge): every
  product on sampled strings (recomputed exactly by the oracle) and sampled
  pairs, the 32 smallest products whole;
* the 1e6-term propagation state at n = 500: the first 4 conjugation steps
  (FP64, and the precision form) and the first 2 literal product steps,
  whole."""
import numpy as np
import pytest

import paper_2605_25974_amd as pl
import synth
from oracle import oracle as O
from tests import parity
from tests.test_gpu_fullsize import _check_order_and_distinct, _check_sampled_pairs, _u64

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
TAU = 0.3


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d.get("phase"), d["coef"])


def test_n16_2000x2000_whole():
    A, B = synth.workload1()
    g = pl.outer_product_merged(pl.PauliSum.from_dict(A), pl.PauliSum.from_dict(B)).export()
    ref = O.product_merge(_osum(A), _osum(B))
    print("n=16 2000 x 2000: %d merged terms" % ref.x.shape[0], flush=True)
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)


def _check_batched_product(T, A, B, b, nsamp):
    """Sampled strings of product b against the oracle's exact coefficient:
    the compensated bound per string and relative error <= 1e-6 over
    |c| > 1e-12 A."""
    import torch
    U = T["fp"].numel()
    rng = synth.rng_for(742, b)
    idx = np.unique(np.concatenate([[0, U - 1], rng.integers(0, U, nsamp)]))
    it = torch.from_numpy(idx).to(T["fp"].device)
    xq, zq = _u64(T["x"][it]), _u64(T["z"][it])
    got = T["coef"][it].cpu().numpy().astype(np.complex128)
    ref, mass, cnt = O.product_coeff(_osum(A), _osum(B), xq, zq)
    assert np.all(cnt > 0), "product %d: an output string is no product of the inputs" % b
    assert np.all(_u64(T["fp"][it]) == parity.fingerprint(xq, zq))
    err = np.abs(got - ref)
    tol = 2.5 * U32 * mass + 1.01 * U32 * np.abs(ref) + 1e-12 * mass
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (b, got[bad[:3]], ref[bad[:3]], mass[bad[:3]])
    sel = np.abs(ref) > 1e-12 * mass
    return float(np.max(err[sel] / np.abs(ref[sel]))) if np.any(sel) else 0.0


def test_batched_256_products():
    plan = synth.workload4_plan()
    sizes = [m1 * m2 for _, m1, m2 in plan]
    smallest = set(np.argsort(sizes, kind="stable")[:32].tolist())
    worst = 0.0
    whole = 0
    chunk = 32
    for c0 in range(0, len(plan), chunk):
        pairs = [synth.workload4_batch(b, *plan[b]) for b in range(c0, min(c0 + chunk, len(plan)))]
        GA = [pl.PauliSum.from_dict(A) for A, _ in pairs]
        GB = [pl.PauliSum.from_dict(B) for _, B in pairs]
        outs = pl.outer_product_batched(GA, GB, mode=pl.COMPENSATED, tau=TAU)
        for k, out in enumerate(outs):
            b = c0 + k
            A, B = pairs[k]
            assert out.info()[2] == "c64"
            if b in smallest:
                g = out.export()
                ref = O.product_merge(_osum(A), _osum(B))
                parity.assert_compensated(g, ref, input_rounding=False)
                worst = max(worst, parity.max_rel_err(g, ref))
                parity.assert_sorted_by_key(g)
                whole += 1
            else:
                pl.trim_memory()  # torch allocates the exported copy
                T = out.export_torch()
                _check_order_and_distinct(T)
                worst = max(worst, _check_batched_product(T, A, B, b, 40))
                _check_sampled_pairs(T, A, B, 20, b)
                del T
            out.destroy()
        for g in GA + GB:
            g.destroy()
    print("batched form: 256 products, %d whole; max rel err %.3e" % (whole, worst))
    assert whole == 32
    assert worst <= 1e-6


def test_propagation_1e6_first_steps_whole():
    S = synth.workload5_state()
    th, x, z = synth.workload5_rotations()
    G = pl.PauliSum.from_dict(S)
    drop = 1e-10
    ref = O.propagate(_osum(S), x[:4], z[:4], th[:4], mode=O.CONJUGATE, drop_abs=drop)
    assert not np.any(np.abs(np.abs(ref.coef) - drop) <= 1e-9 * drop)
    g = pl.propagate(G, x[:4], z[:4], th[:4], rotate_mode=pl.ROTATE_CONJUGATE,
                     drop_abs=drop).export()
    print("4 conjugation steps: %d terms" % g["x"].shape[0], flush=True)
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)
    c = pl.propagate(G, x[:4], z[:4], th[:4], rotate_mode=pl.ROTATE_CONJUGATE,
                     mode=pl.COMPENSATED, tau=TAU, drop_abs=drop).export()
    err = parity.max_rel_err(c, ref)
    print("4 conjugation steps, precision form: max rel err %.3e" % err, flush=True)
    assert err <= 1e-6
    del g, c, ref
    ref = O.propagate(_osum(S), x[:2], z[:2], th[:2], mode=O.PRODUCT, drop_abs=drop)
    assert not np.any(np.abs(np.abs(ref.coef) - drop) <= 1e-9 * drop)
    g = pl.propagate(G, x[:2], z[:2], th[:2], rotate_mode=pl.ROTATE_PRODUCT,
                     drop_abs=drop).export()
    print("2 literal steps: %d terms" % g["x"].shape[0], flush=True)
    parity.assert_merged_fp64(g, ref)
    parity.assert_sorted_by_key(g)

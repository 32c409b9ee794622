"""Comparison rules between the GPU path and the CPU oracle.

* Strings and phase exponents: bit-exact.
* Unmerged coefficients: bit-exact (both sides form re = ac - bd and
  im = ad + bc with the same roundings).
* Merged FP64 coefficients (the bar the build states): per string,
  |gpu - oracle| <= max(1e-12 |oracle|, 1e-14 max(1, A)), where A is the
  sum of the moduli of the contributions (the absolute floor near exact
  cancellation is scaled by A: a correct FP64 reduction of contributions of
  size A carries errors of order 1e-16 A).
* Merged FP32 sums (compensated form) are compared by relative error.

Also a test-side implementation of the ordering fingerprint (the
counter-based SplitMix64 columns, from the published generator), used only
to check the order property of merged output.
"""
import numpy as np

MASK = (1 << 64) - 1
FP_SEED = 0x5041554C49420001
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64_at(seed, counter):
    z = (seed + counter * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


_COLS = {}


def _cols(W):
    if W not in _COLS:
        _COLS[W] = np.array([splitmix64_at(FP_SEED, b + 1) for b in range(2 * 64 * W)],
                            dtype=np.uint64)
    return _COLS[W]


def fingerprint(x, z):
    """64-bit fingerprint of packed strings (m, W): XOR of column 2q for each
    set X bit of qubit q and column 2q+1 for each set Z bit."""
    x = np.asarray(x, np.uint64)
    z = np.asarray(z, np.uint64)
    m, W = x.shape
    cols = _cols(W)
    fp = np.zeros(m, np.uint64)
    for w in range(W):
        for b in range(64):
            q = 64 * w + b
            bit = np.uint64(1) << np.uint64(b)
            fp ^= np.where((x[:, w] & bit) != 0, cols[2 * q], np.uint64(0))
            fp ^= np.where((z[:, w] & bit) != 0, cols[2 * q + 1], np.uint64(0))
    return fp


def row_keys(x, z):
    xz = np.ascontiguousarray(np.concatenate([np.asarray(x, np.uint64),
                                              np.asarray(z, np.uint64)], axis=1))
    return xz.view(np.dtype((np.void, 8 * xz.shape[1]))).reshape(-1)


def align(gx, gz, rx, rz):
    """Index arrays (gi, ri) matching equal strings; asserts the sets agree."""
    gk = row_keys(gx, gz)
    rk = row_keys(rx, rz)
    assert len(np.unique(gk)) == len(gk), "GPU output has duplicate strings"
    gi = np.argsort(gk, kind="stable")
    ri = np.argsort(rk, kind="stable")
    assert len(gk) == len(rk), "string counts differ: gpu %d oracle %d" % (len(gk), len(rk))
    assert np.array_equal(gk[gi], rk[ri]), "string sets differ"
    return gi, ri


def assert_merged_fp64(gpu, ref, rel=1e-12, abs_floor=1e-14):
    gi, ri = align(gpu["x"], gpu["z"], ref.x, ref.z)
    assert np.all(gpu["phase"] == 0)
    g = gpu["coef"][gi].astype(np.complex128)
    r = ref.coef[ri]
    A = ref.mass[ri]
    err = np.abs(g - r)
    tol = np.maximum(rel * np.abs(r), abs_floor * np.maximum(1.0, A))
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, "coefficient mismatch at %d strings, e.g. gpu %r oracle %r A %r" % (
        bad.size, g[bad[:3]], r[bad[:3]], A[bad[:3]])


def max_rel_err(gpu, ref, floor_rel=1e-12):
    """max |gpu - ref| / |ref| over strings with |ref| > floor_rel * A."""
    gi, ri = align(gpu["x"], gpu["z"], ref.x, ref.z)
    g = gpu["coef"][gi].astype(np.complex128)
    r = ref.coef[ri]
    A = ref.mass[ri]
    sel = np.abs(r) > floor_rel * np.maximum(A, 1e-300)
    if not np.any(sel):
        return 0.0
    return float(np.max(np.abs(g[sel] - r[sel]) / np.abs(r[sel])))


def assert_sorted_by_key(gpu, key_bits=64):
    """Merged output is ascending in (fingerprint >> (64-key_bits), then the
    packed words from the most significant X word down, then Z words), and
    its fingerprint column is the fingerprint of each string."""
    fp = fingerprint(gpu["x"], gpu["z"])
    assert np.array_equal(fp, gpu["fp"])
    key = fp >> np.uint64(64 - key_bits) if key_bits < 64 else fp
    W = gpu["x"].shape[1]
    cols = [key] + [gpu["x"][:, w] for w in range(W - 1, -1, -1)] + \
           [gpu["z"][:, w] for w in range(W - 1, -1, -1)]
    order = np.lexsort(cols[::-1])
    assert np.array_equal(order, np.arange(len(key))), "merged output is not in key order"


U32 = 2.0 ** -24


def assert_compensated(gpu, ref, input_rounding=True):
    """Bound check of the compensated FP32 form, string by string.

    Each contribution carries the FP32 product error: the two inputs
    rounded to FP32 (when they were FP64; relative u each) and the complex
    product (sqrt(5) u, Brent, Percival and Zimmermann 2007), about 4.3 u of
    its modulus.  Sum2 adds u |sum| plus a second-order term, and a
    re-merged segment is FP64-accurate before its final rounding to FP32.
    So |gpu - ref| <= 4.5 u A + 1.01 u |ref| + 1e-12 A for every string."""
    gi, ri = align(gpu["x"], gpu["z"], ref.x, ref.z)
    assert np.all(gpu["phase"] == 0)
    assert gpu["coef"].dtype == np.complex64
    g = gpu["coef"][gi].astype(np.complex128)
    r = ref.coef[ri]
    A = ref.mass[ri]
    per_term = (4.5 if input_rounding else 2.5) * U32
    tol = per_term * A + 1.01 * U32 * np.abs(r) + 1e-12 * A
    err = np.abs(g - r)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, "compensated bound broken at %d strings, e.g. gpu %r oracle %r A %r" % (
        bad.size, g[bad[:3]], r[bad[:3]], A[bad[:3]])


def max_rel_err_after_drop(gpu, ref, drop_rel=1e-6):
    """max |gpu - ref| / |ref| over strings with |ref| >= drop_rel * max |ref|
    (the comparison of the cancellation case: both sides dropped below
    drop_rel times the largest coefficient)."""
    gi, ri = align(gpu["x"], gpu["z"], ref.x, ref.z)
    g = gpu["coef"][gi].astype(np.complex128)
    r = ref.coef[ri]
    if r.size == 0:
        return 0.0
    sel = np.abs(r) >= drop_rel * np.max(np.abs(r))
    return float(np.max(np.abs(g[sel] - r[sel]) / np.abs(r[sel])))

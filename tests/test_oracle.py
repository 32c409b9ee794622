"""Pins of the CPU oracle against facts fixed by the paper and by linear
algebra (no GPU).  Each test names what it pins and why a plausible mistake
in the oracle (a wrong table entry, a dropped phase, a transposed operand, a
wrong qubit order, a lost duplicate) fails it."""
import itertools
import os

import numpy as np
import pytest

from oracle import oracle as O
from tests.helpers import (LETTERS, W, all_strings, dense_string, dense_sum, pack, pack_many,
                           unpack)
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mul_str(a: str, b: str, k1=0, k2=0):
    n = len(a)
    x1, z1 = pack(a)
    x2, z2 = pack(b)
    x3, z3, k3 = O.mul(n, x1, z1, k1, x2, z2, k2)
    return unpack(n, x3, z3), k3


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    return rows


@pytest.fixture(autouse=True)
def _clean_table():
    O.table_reset()
    yield
    O.table_reset()


def test_printed_products_and_worked_example():
    """Section III-A: the nine +-i products, identity rules, P^2 = I and the
    worked example (X I Z)(Z I X) = Y I Y with phase +1."""
    for a, b, c, k in _golden("paper_products.txt"):
        got, kk = _mul_str(a, b)
        assert (got, kk) == (c, int(k)), (a, b)


def test_commutation_examples():
    """Section III-A: XIZ/ZIX commute, XIZ/XIY anticommute.  Checked as
    P1 P2 = +-P2 P1 from the oracle's two products."""
    for a, b, rel in _golden("paper_commutation.txt"):
        s1, k1 = _mul_str(a, b)
        s2, k2 = _mul_str(b, a)
        assert s1 == s2
        assert ((k1 - k2) % 4 == 0) == (rel == "commute")


def test_single_qubit_table_against_matrices():
    """All 16 single-qubit products equal the 2x2 matrix products of
    Section III-A: sigma_a sigma_b = i^k sigma_c."""
    for a in LETTERS:
        for b in LETTERS:
            c, k = _mul_str(a, b)
            np.testing.assert_array_equal(SIG(a) @ SIG(b), (1j ** k) * SIG(c))


def SIG(L):
    return dense_string(L)


def _check_dense(a, b, k1, k2):
    c, k3 = _mul_str(a, b, k1, k2)
    lhs = (1j ** k1) * dense_string(a) @ ((1j ** k2) * dense_string(b))
    rhs = (1j ** k3) * dense_string(c)
    np.testing.assert_allclose(lhs, rhs, atol=0, rtol=0)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_dense_products_exhaustive(n):
    """Every pair of n-qubit strings (n <= 3): the oracle's product string and
    phase reproduce the 2^n x 2^n matrix product exactly (entries are in
    {0, +-1, +-i}, so equality is exact)."""
    S = all_strings(n)
    rng = np.random.default_rng(n)
    for a in S:
        for b in S:
            k1, k2 = rng.integers(0, 4, size=2)
            _check_dense(a, b, int(k1), int(k2))


@pytest.mark.parametrize("n", [4, 5, 6])
def test_dense_products_sampled(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(60):
        a = "".join(rng.choice(list(LETTERS), n))
        b = "".join(rng.choice(list(LETTERS), n))
        k1, k2 = rng.integers(0, 4, size=2)
        _check_dense(a, b, int(k1), int(k2))


def test_multiword_qubit_order():
    """Strings longer than one word: the result must not depend on which
    word a qubit lives in.  Checked against the per-qubit product of the
    same letters (each single-qubit product pinned above)."""
    rng = np.random.default_rng(7)
    for n in (63, 64, 65, 130, 500):
        a = "".join(rng.choice(list(LETTERS), n))
        b = "".join(rng.choice(list(LETTERS), n))
        c, k = _mul_str(a, b)
        kk = 0
        for q in range(n):
            cq, kq = _mul_str(a[q], b[q])
            assert c[q] == cq
            kk += kq
        assert k == kk % 4


def test_square_is_identity_and_associativity():
    rng = np.random.default_rng(11)
    for n in (1, 7, 64, 100):
        for _ in range(30):
            a, b, c = ("".join(rng.choice(list(LETTERS), n)) for _ in range(3))
            s, k = _mul_str(a, a)
            assert s == "I" * n and k == 0  # P^2 = I (Section III-A)
            ab, k_ab = _mul_str(a, b)
            left, k_l = _mul_str(ab, c, k_ab, 0)
            bc, k_bc = _mul_str(b, c)
            right, k_r = _mul_str(a, bc, 0, k_bc)
            assert left == right and k_l == k_r


def test_commutation_equals_symplectic_parity():
    """Section III-F: strings commute iff the symplectic inner product
    sum_q (x1 z2 + z1 x2) is even."""
    rng = np.random.default_rng(12)
    for n in (3, 64, 200):
        for _ in range(50):
            a, b = ("".join(rng.choice(list(LETTERS), n)) for _ in range(2))
            s1, k1 = _mul_str(a, b)
            s2, k2 = _mul_str(b, a)
            x1, z1 = pack(a)
            x2, z2 = pack(b)
            sp = sum(bin(int(p)).count("1") for p in (x1 & z2) ^ (z1 & x2)) % 2
            assert s1 == s2
            assert (k1 - k2) % 4 == 2 * sp


def _rand_sum(rng, n, m, distinct=True):
    return synth.random_sum(rng, n, m, distinct_strings=distinct)


def _osum(d):
    return O.Sum(d["n"], d["x"], d["z"], d["phase"], d["coef"])


def _dense_merged(r: O.Merged):
    return dense_sum(r.n, r.x, r.z, np.zeros(r.x.shape[0], np.uint8), r.coef)


@pytest.mark.parametrize("n,m1,m2", [(1, 3, 4), (2, 7, 5), (3, 12, 9), (4, 20, 17)])
def test_sum_product_against_dense(n, m1, m2):
    """Pauli-sum level (eq. (2)): dense(H1) @ dense(H2) equals the dense
    matrix of merge(H1*H2), and of merge(outer_product(H1, H2)); the merged
    strings are distinct."""
    rng = synth.rng_for(900, n)
    A = _osum(_rand_sum(rng, n, m1, distinct=False))
    B = _osum(_rand_sum(rng, n, m2, distinct=False))
    ref = dense_sum(n, A.x, A.z, A.phase, A.coef) @ dense_sum(n, B.x, B.z, B.phase, B.coef)
    r = O.product_merge(A, B)
    np.testing.assert_allclose(_dense_merged(r), ref, atol=1e-12)
    keys = {(r.x[u].tobytes(), r.z[u].tobytes()) for u in range(r.x.shape[0])}
    assert len(keys) == r.x.shape[0]
    x, z, ph, c = O.outer_product(A, B)
    r2 = O.merge(O.Sum(n, x, z, ph, c))
    np.testing.assert_allclose(_dense_merged(r2), ref, atol=1e-12)


def test_outer_product_layout_and_plain_coefficients():
    """Section IV-C: output p = j*m1 + i holds a_i * b_j; the coefficient is
    the plain complex product (re = ac - bd, im = ad + bc) and the phase is
    the sum of the input phases and the product phase."""
    rng = synth.rng_for(901)
    n = 70
    A = _osum(_rand_sum(rng, n, 6))
    B = _osum(_rand_sum(rng, n, 5))
    x, z, ph, c = O.outer_product(A, B)
    for j in range(B.m):
        for i in range(A.m):
            p = j * A.m + i
            x3, z3, k3 = O.mul(n, A.x[i], A.z[i], A.phase[i], B.x[j], B.z[j], B.phase[j])
            assert np.array_equal(x[p], x3) and np.array_equal(z[p], z3) and ph[p] == k3
            a, b = A.coef[i].real, A.coef[i].imag
            cc, d = B.coef[j].real, B.coef[j].imag
            assert c[p].real == a * cc - b * d and c[p].imag == a * d + b * cc


def test_merge_integer_coefficients_exact():
    """Integer coefficients: every partial sum is exact, so the merged value
    must equal exact integer arithmetic over the (pinned) single products."""
    rng = np.random.default_rng(5)
    n = 5
    strings = ["".join(rng.choice(list(LETTERS), n)) for _ in range(12)]
    A = [(s, int(rng.integers(0, 4)), complex(*rng.integers(-50, 51, size=2))) for s in strings]
    B = [(s, int(rng.integers(0, 4)), complex(*rng.integers(-50, 51, size=2))) for s in strings[:9]]
    exact = {}
    for sb, kb, cb in B:
        for sa, ka, ca in A:
            s, k = _mul_str(sa, sb, ka, kb)
            exact[s] = exact.get(s, 0) + (1j ** k) * ca * cb
    xa, za = pack_many([a[0] for a in A])
    xb, zb = pack_many([b[0] for b in B])
    SA = O.Sum(n, xa, za, np.array([a[1] for a in A]), np.array([a[2] for a in A]))
    SB = O.Sum(n, xb, zb, np.array([b[1] for b in B]), np.array([b[2] for b in B]))
    got = O.product_merge(SA, SB)
    d = {unpack(n, got.x[u], got.z[u]): got.coef[u] for u in range(got.x.shape[0])}
    assert set(d) == set(exact)
    for s in exact:
        assert d[s] == exact[s]


def test_hermitian_square_closed_forms():
    """H*H for Hermitian H with distinct strings and real coefficients: the
    identity coefficient is sum c^2 and every coefficient is real (pairs
    (a, b), (b, a) that anticommute cancel exactly)."""
    H = synth.jw_sum(synth.rng_for(902), 40, 300, coef="real")
    S = _osum(H)
    r = O.product_merge(S, S)
    d = r.as_dict()
    ident = (np.zeros(1, np.uint64).tobytes(), np.zeros(1, np.uint64).tobytes())
    c_id = d[ident][0]
    ref = float(np.sum(H["coef"].real.astype(np.longdouble) ** 2))
    assert abs(c_id.real - ref) <= 1e-15 * ref and c_id.imag == 0
    assert np.all(r.coef.imag == 0)


def test_identity_coefficient_is_trace():
    """coef(I) of H1*H2 = tr(H1 H2) / 2^n = sum over common strings of
    i^{k1+k2} c1 c2 (only P*P gives I)."""
    rng = synth.rng_for(903)
    n = 6
    A = _osum(_rand_sum(rng, n, 40))
    B = _osum(_rand_sum(rng, n, 40))
    ref = np.trace(dense_sum(n, A.x, A.z, A.phase, A.coef) @
                   dense_sum(n, B.x, B.z, B.phase, B.coef)) / 2 ** n
    r = O.product_merge(A, B).as_dict()
    ident = (np.zeros(1, np.uint64).tobytes(), np.zeros(1, np.uint64).tobytes())
    got = r.get(ident, (0j, 0.0))[0]
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))


def test_drop_is_strict():
    n = 2
    x, z = pack_many(["XI", "ZI", "IY"])
    S = O.Sum(n, x, z, None, np.array([0.5, 0.25 + 0j, 1e-3]))
    kept = O.merge(S, drop_abs=0.25)
    names = sorted(unpack(n, kept.x[u], kept.z[u]) for u in range(kept.x.shape[0]))
    assert names == ["XI", "ZI"]  # |0.25| is not strictly below 0.25
    assert O.merge(S, drop_abs=-1.0).x.shape[0] == 3


def test_product_coeff_matches_full_merge():
    """The one-string-at-a-time coefficient used for sampled checks at full
    size equals the full merge on every output string, and is zero with no
    contributing pair for a string outside the product set."""
    rng = synth.rng_for(904)
    n = 90
    A = _osum(synth.jw_sum(rng, n, 120))
    B = _osum(synth.jw_sum(rng, n, 80))
    full = O.product_merge(A, B)
    c, mass, cnt = O.product_coeff(A, B, full.x, full.z)
    np.testing.assert_array_equal(c, full.coef)
    np.testing.assert_allclose(mass, full.mass, rtol=1e-15)
    assert np.all(cnt >= 1)
    xq, zq = pack("X" * n)
    c0, _, cnt0 = O.product_coeff(A, B, xq, zq)
    assert cnt0[0] == 0 and c0[0] == 0


def test_planted_table_mistake_is_caught():
    """Mutation check on the pins: a wrong phase in one table entry (XY = -iZ)
    or a wrong letter (XY = iX) makes the dense-matrix check fail."""
    O.table_set(1, 2, 3, 3)  # X*Y -> -iZ (wrong sign)
    with pytest.raises(AssertionError):
        test_single_qubit_table_against_matrices()
    O.table_reset()
    O.table_set(1, 2, 1, 1)  # X*Y -> iX (wrong letter)
    with pytest.raises(AssertionError):
        test_dense_products_exhaustive(2)
    O.table_reset()
    test_dense_products_exhaustive(2)

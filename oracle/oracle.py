"""ctypes wrapper around the CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It marshals
numpy arrays and nothing else; every step of the arithmetic lives in
oracle.cpp (see the header there for the paper passages it follows).

Arrays use the packed layout of Section III-C / Table I: ``x`` and ``z`` are
uint64 arrays of shape (m, W) with W = ceil(n/64); qubit q is bit q % 64 of
word q // 64.  ``phase`` is uint8 (m,) holding the exponent k of i^k, and
``coef`` is complex128 (m,).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_int = ctypes.c_int


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (no fused multiply-add contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(
            ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
             _SRC, "-o", tmp],
            check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_mul.restype = _int
        L.oracle_mul.argtypes = [_int, _u64p, _u64p, _int, _u64p, _u64p, _int, _u64p, _u64p]
        L.oracle_decode.restype = None
        L.oracle_decode.argtypes = [_int, _i64, _u64p, _u64p, _u8p]
        L.oracle_outer_product.restype = _int
        L.oracle_outer_product.argtypes = (
            [_int] + [_i64, _u64p, _u64p, _u8p, _f64p] * 2 + [_u64p, _u64p, _u8p, _f64p])
        L.oracle_merge.restype = ctypes.c_void_p
        L.oracle_merge.argtypes = [_int, _i64, _u64p, _u64p, _u8p, _f64p, ctypes.c_double]
        L.oracle_product_merge.restype = ctypes.c_void_p
        L.oracle_product_merge.argtypes = (
            [_int] + [_i64, _u64p, _u64p, _u8p, _f64p] * 2 + [ctypes.c_double, _i64, _i64, _i64, _i64])
        L.oracle_result_size.restype = _i64
        L.oracle_result_size.argtypes = [ctypes.c_void_p]
        L.oracle_result_copy.restype = None
        L.oracle_result_copy.argtypes = [ctypes.c_void_p, _u64p, _u64p, _f64p, _f64p]
        L.oracle_result_free.restype = None
        L.oracle_result_free.argtypes = [ctypes.c_void_p]
        L.oracle_product_coeff.restype = _int
        L.oracle_product_coeff.argtypes = (
            [_int] + [_i64, _u64p, _u64p, _u8p, _f64p] * 2 + [_i64, _u64p, _u64p, _f64p, _f64p, _i64p])
        L.oracle_commutator.restype = ctypes.c_void_p
        L.oracle_commutator.argtypes = (
            [_int] + [_i64, _u64p, _u64p, _u8p, _f64p] * 2 + [ctypes.c_double])
        L.oracle_propagate.restype = ctypes.c_void_p
        L.oracle_propagate.argtypes = (
            [_int, _i64, _u64p, _u64p, _u8p, _f64p, _int, _u64p, _u64p, _f64p, _int,
             ctypes.c_double])
        L.oracle_table_set.restype = None
        L.oracle_table_set.argtypes = [_int, _int, _int, _int]
        L.oracle_table_reset.restype = None
        L.oracle_table_reset.argtypes = []
        _lib = L
    return _lib


def _W(n: int) -> int:
    return (n + 63) // 64


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


class Sum:
    """A Pauli sum on the host: value = sum_t i^phase[t] * coef[t] * P(x[t], z[t])."""

    def __init__(self, n, x, z, phase=None, coef=None):
        self.n = int(n)
        W = _W(self.n)
        self.x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, W)
        self.z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, W)
        m = self.x.shape[0]
        if phase is None:
            phase = np.zeros(m, np.uint8)
        self.phase = np.ascontiguousarray(phase, dtype=np.uint8).reshape(m)
        if coef is None:
            coef = np.ones(m, np.complex128)
        self.coef = np.ascontiguousarray(coef, dtype=np.complex128).reshape(m)
        self._c = self.coef.view(np.float64)

    @property
    def m(self):
        return self.x.shape[0]

    def _args(self):
        return [self.m, _ptr(self.x, _u64p), _ptr(self.z, _u64p), _ptr(self.phase, _u8p),
                _ptr(self._c, _f64p)]


class Merged:
    """Result of sort-and-combine: strings, coefficients and contribution mass."""

    def __init__(self, n, x, z, coef, mass):
        self.n, self.x, self.z, self.coef, self.mass = n, x, z, coef, mass

    def as_dict(self):
        """{(x-words bytes, z-words bytes): (coef, mass)}"""
        return {(self.x[u].tobytes(), self.z[u].tobytes()): (self.coef[u], self.mass[u])
                for u in range(self.x.shape[0])}


def _take(n, h) -> Merged:
    L = lib()
    try:
        U = L.oracle_result_size(h)
        W = _W(n)
        x = np.zeros((U, W), np.uint64)
        z = np.zeros((U, W), np.uint64)
        c = np.zeros(U, np.complex128)
        mass = np.zeros(U, np.float64)
        L.oracle_result_copy(h, _ptr(x, _u64p), _ptr(z, _u64p), _ptr(c.view(np.float64), _f64p),
                             _ptr(mass, _f64p))
        return Merged(n, x, z, c, mass)
    finally:
        L.oracle_result_free(h)


def decode(n, x, z) -> np.ndarray:
    """Letters (0 I, 1 X, 2 Y, 3 Z) of packed strings, shape (m, n)."""
    x = np.ascontiguousarray(x, dtype=np.uint64).reshape(-1, _W(n))
    z = np.ascontiguousarray(z, dtype=np.uint64).reshape(-1, _W(n))
    out = np.zeros((x.shape[0], n), np.uint8)
    lib().oracle_decode(n, x.shape[0], _ptr(x, _u64p), _ptr(z, _u64p), _ptr(out, _u8p))
    return out


def mul(n, x1, z1, k1, x2, z2, k2):
    """(i^k1 P1)(i^k2 P2) = i^k3 P3 -> (x3, z3, k3)."""
    W = _W(n)
    x1 = np.ascontiguousarray(x1, np.uint64).reshape(W)
    z1 = np.ascontiguousarray(z1, np.uint64).reshape(W)
    x2 = np.ascontiguousarray(x2, np.uint64).reshape(W)
    z2 = np.ascontiguousarray(z2, np.uint64).reshape(W)
    x3 = np.zeros(W, np.uint64)
    z3 = np.zeros(W, np.uint64)
    k3 = lib().oracle_mul(n, _ptr(x1, _u64p), _ptr(z1, _u64p), int(k1), _ptr(x2, _u64p),
                          _ptr(z2, _u64p), int(k2), _ptr(x3, _u64p), _ptr(z3, _u64p))
    return x3, z3, k3


def outer_product(a: Sum, b: Sum):
    """Unmerged H1*H2 in block order p = j*m1 + i -> (x, z, phase, coef)."""
    assert a.n == b.n
    n, W, P = a.n, _W(a.n), a.m * b.m
    x = np.zeros((P, W), np.uint64)
    z = np.zeros((P, W), np.uint64)
    ph = np.zeros(P, np.uint8)
    c = np.zeros(P, np.complex128)
    lib().oracle_outer_product(n, *a._args(), *b._args(), _ptr(x, _u64p), _ptr(z, _u64p),
                               _ptr(ph, _u8p), _ptr(c.view(np.float64), _f64p))
    return x, z, ph, c


def merge(s: Sum, drop_abs: float = -1.0) -> Merged:
    h = lib().oracle_merge(s.n, *s._args(), float(drop_abs))
    return _take(s.n, h)


def product_merge(a: Sum, b: Sum, drop_abs: float = -1.0, i_range=None, j_range=None) -> Merged:
    """merge(H1*H2) restricted to the pair block i_range x j_range (default: all)."""
    assert a.n == b.n
    i0, i1 = i_range if i_range is not None else (0, a.m)
    j0, j1 = j_range if j_range is not None else (0, b.m)
    h = lib().oracle_product_merge(a.n, *a._args(), *b._args(), float(drop_abs), i0, i1, j0, j1)
    return _take(a.n, h)


def commutator(a: Sum, b: Sum, drop_abs: float = -1.0) -> Merged:
    """[H1, H2] = H1*H2 - H2*H1 merged exactly: the strings that an
    anticommuting pair gives, each with the exact sum of a_i b_j - b_j a_i."""
    assert a.n == b.n
    h = lib().oracle_commutator(a.n, *a._args(), *b._args(), float(drop_abs))
    if not h:
        raise RuntimeError("oracle_commutator failed")
    return _take(a.n, h)


PRODUCT, CONJUGATE = 0, 1


def propagate(s: Sum, px, pz, theta, mode=CONJUGATE, drop_abs: float = -1.0) -> Merged:
    """Rotation steps of Section III-B eq. (5) on the merged sum s: step t uses
    the string (px[t], pz[t]) (packed words, shape (steps, W)) and angle
    theta[t].  mode PRODUCT multiplies every term on the left by
    cos(theta) I - i sin(theta) P; CONJUGATE leaves terms commuting with P
    unchanged.  Each step is merged exactly and truncated at drop_abs."""
    W = _W(s.n)
    px = np.ascontiguousarray(px, dtype=np.uint64).reshape(-1, W)
    pz = np.ascontiguousarray(pz, dtype=np.uint64).reshape(-1, W)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    assert px.shape[0] == pz.shape[0] == th.size
    h = lib().oracle_propagate(s.n, *s._args(), int(th.size), _ptr(px, _u64p), _ptr(pz, _u64p),
                               _ptr(th, _f64p), int(mode), float(drop_abs))
    return _take(s.n, h)


def product_coeff(a: Sum, b: Sum, xq, zq):
    """Coefficient, mass and pair count of each query string in merge(H1*H2)."""
    W = _W(a.n)
    xq = np.ascontiguousarray(xq, np.uint64).reshape(-1, W)
    zq = np.ascontiguousarray(zq, np.uint64).reshape(-1, W)
    nq = xq.shape[0]
    c = np.zeros(nq, np.complex128)
    mass = np.zeros(nq, np.float64)
    cnt = np.zeros(nq, np.int64)
    rc = lib().oracle_product_coeff(a.n, *a._args(), *b._args(), nq, _ptr(xq, _u64p),
                                    _ptr(zq, _u64p), _ptr(c.view(np.float64), _f64p),
                                    _ptr(mass, _f64p), _ptr(cnt, _i64p))
    if rc != 0:
        raise RuntimeError("oracle_product_coeff failed")
    return c, mass, cnt


def table_set(a, b, letter, k):
    """Plant a wrong single-qubit product (mutation tests only)."""
    lib().oracle_table_set(a, b, letter, k)


def table_reset():
    lib().oracle_table_reset()

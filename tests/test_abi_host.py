"""The C-ABI library without a GPU: it loads, exports every symbol the header
declares, and rejects bad arguments on the host before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2605_25974_amd as pl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paulisum.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b((?:pauli|paulisum)_[a-z_]+)\s*\(", src))
    return sorted(n for n in names if not n.endswith("_fn"))


def test_header_declares_what_binding_lists():
    assert set(_declared()) == set(pl.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = pl.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings():
    L = pl.lib()
    for code in range(7):
        assert L.pauli_status_string(code)
    assert L.pauli_status_string(0) == b"ok"


def _create(n, x, z, ph=None, coef=None, out=True):
    L = pl.lib()
    h = ctypes.c_void_p()
    m = x.shape[0] if x is not None else 0
    return L.paulisum_create(n, m, x.ctypes.data if x is not None else None,
                             z.ctypes.data if z is not None else None,
                             ph.ctypes.data if ph is not None else None,
                             coef.ctypes.data if coef is not None else None, 0, 0, None,
                             ctypes.byref(h) if out else None)


def test_create_rejects_bad_host_input():
    W = 1
    x = np.zeros((3, W), np.uint64)
    z = np.zeros((3, W), np.uint64)
    c = np.ones(3, np.complex128)
    # a bit at qubit 5 >= n = 5
    x2 = x.copy()
    x2[1, 0] = np.uint64(1 << 5)
    assert _create(5, x2, z, None, c) == 1
    assert b"at or above n" in pl.lib().pauli_last_error()
    # Z padding too
    z2 = z.copy()
    z2[2, 0] = np.uint64(1 << 63)
    assert _create(5, x, z2, None, c) == 1
    # phase > 3
    ph = np.array([0, 4, 1], np.uint8)
    assert _create(5, x, z, ph, c) == 1
    assert b"phase" in pl.lib().pauli_last_error()
    # n out of range
    assert _create(0, x, z, None, c) == 1
    assert _create(1025, np.zeros((3, 17), np.uint64), np.zeros((3, 17), np.uint64), None, c) == 1
    # null out / null arrays
    assert _create(5, x, z, None, c, out=False) == 1
    assert _create(5, x, None, None, c) == 1


def test_multiword_padding_rule():
    # n = 70: word 1 holds qubits 64..69; bit 6 of word 1 is qubit 70 (padding)
    x = np.zeros((1, 2), np.uint64)
    z = np.zeros((1, 2), np.uint64)
    c = np.ones(1, np.complex128)
    x[0, 1] = np.uint64(1 << 6)
    assert _create(70, x, z, None, c) == 1


def test_negative_terms_and_flags():
    L = pl.lib()
    h = ctypes.c_void_p()
    assert L.paulisum_create(5, -1, None, None, None, None, 0, 0, None, ctypes.byref(h)) == 1
    assert L.paulisum_create(5, 0, None, None, None, None, 0, 8, None, ctypes.byref(h)) == 1
    assert L.paulisum_create(5, 0, None, None, None, None, 7, 0, None, ctypes.byref(h)) == 1


def test_null_handles():
    L = pl.lib()
    out = ctypes.c_void_p()
    assert L.pauli_outer_product(None, None, ctypes.byref(out), None) == 1
    assert L.pauli_merge(None, None, ctypes.byref(out), None) == 1
    assert L.pauli_outer_product_merged(None, None, None, ctypes.byref(out), None) == 1
    assert L.paulisum_info(None, None, None, None) == 1
    assert L.paulisum_destroy(None) == 0
    assert L.pauli_outer_product_batched(-1, None, None, None, None, None, None) == 1
    assert L.pauli_outer_product_batched(0, None, None, None, None, None, None) == 0


def test_allocator_hook_requires_both():
    L = pl.lib()
    assert L.pauli_set_allocator(ctypes.c_void_p(1), None, None) == 1
    assert L.pauli_set_allocator(None, None, None) == 0
    assert L.pauli_set_memory_budget(0) == 0


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(pl, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pl, "_lib", None)
    with pytest.raises(pl.PauliLibraryMissing):
        pl.lib()


def test_tune_file_round_trip_and_all_or_nothing(tmp_path):
    """The tune table is host state: a saved file loads back unchanged, and a
    file with one malformed line is refused as a whole (none of its lines
    enter the table)."""
    good = tmp_path / "good.txt"
    good.write_text("# W log2_records dtype mode target class_bits parts\n"
                    "8 27 1 0 3000 8 4\n")
    pl.tune_load(str(good))
    saved = tmp_path / "saved.txt"
    pl.tune_save(str(saved))
    rows = [ln.split() for ln in saved.read_text().splitlines() if not ln.startswith("#")]
    assert ["8", "27", "1", "0", "3000", "8", "4"] in rows
    mixed = tmp_path / "mixed.txt"
    mixed.write_text("4 20 1 1 2000 6 2\n"   # valid
                     "4 21 1 1 100 6 2\n")   # target below 256: malformed
    with pytest.raises(pl.PauliError) as e:
        pl.tune_load(str(mixed))
    assert e.value.status == "INVALID"
    pl.tune_save(str(saved))
    rows = [ln.split() for ln in saved.read_text().splitlines() if not ln.startswith("#")]
    assert not any(r[:2] == ["4", "20"] for r in rows)
    for text in ("1 2 3\n", "8 27 1 0 3000 9 4\n", "8 27 1 0 3000 8 3\n", "8 27 1 0 nan 8 4\n"):
        bad = tmp_path / "bad.txt"
        bad.write_text(text)
        with pytest.raises(pl.PauliError):
            pl.tune_load(str(bad))
    with pytest.raises(pl.PauliError):
        pl.tune_load(str(tmp_path / "missing.txt"))

"""Python binding of the MI355X Pauli-sum library (libpaulisum.so).

Argument marshalling only: every step of every operation runs in the HIP
kernels behind the C ABI declared in include/paulisum.h.  PyTorch is used for
device memory (torch tensors as inputs/outputs) and for the current stream.
If the shared library has not been built the import of this package still
works, but the first call raises ``PauliLibraryMissing``: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaulisum.so")

PAULI_OK = 0
STATUS = {0: "OK", 1: "INVALID", 2: "SHAPE", 3: "OVERFLOW", 4: "OOM", 5: "CAPACITY", 6: "DEVICE"}
C128, C64 = 0, 1
PTR_DEVICE = 1
PLAIN, COMPENSATED = 0, 1

# Every symbol include/paulisum.h declares.
EXPORTS = (
    "pauli_status_string", "pauli_last_error", "paulisum_create", "paulisum_destroy",
    "paulisum_info", "paulisum_export", "pauli_outer_product", "pauli_merge",
    "pauli_outer_product_merged", "pauli_outer_product_batched", "pauli_set_allocator",
    "pauli_set_memory_budget", "pauli_profile_enable", "pauli_profile_read", "pauli_propagate",
    "pauli_trim_memory", "pauli_commutator", "pauli_apply_clifford", "pauli_sort_lex",
    "pauli_merge_into", "pauli_batch_plan_create", "pauli_batch_plan_run",
    "pauli_batch_plan_results", "pauli_batch_plan_destroy", "pauli_tune_save", "pauli_tune_load",
    "pauli_propagate_plan_create", "pauli_propagate_plan_run", "pauli_propagate_plan_result",
    "pauli_propagate_plan_destroy",
)
STAGES = ("outer_product", "prep", "sort", "segment", "write", "long", "clifford", "lex",
          "filter")


class PauliLibraryMissing(RuntimeError):
    pass


class PauliError(RuntimeError):
    def __init__(self, status, msg):
        self.status = STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.status, msg))


class MergeOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("drop_abs", ctypes.c_double),
                ("remerge_tau", ctypes.c_double), ("key_bits", ctypes.c_int32)]


class Tune(ctypes.Structure):
    _fields_ = [("bucket_bits", ctypes.c_int32), ("bucket_records", ctypes.c_int32),
                ("class_bits", ctypes.c_int32), ("expand_parts", ctypes.c_int32)]


_vp = ctypes.c_void_p
_lib = None


def lib():
    """The loaded ctypes library (raises PauliLibraryMissing if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PauliLibraryMissing(
            "libpaulisum.so is not built (run __graft_entry__.build() or "
            "python paper_2605_25974_amd/build.py); there is no CPU fallback")
    # Load torch's HIP runtime first so that the library and torch share one
    # runtime (both link libamdhip64.so.7 by soname).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    L.pauli_status_string.restype = ctypes.c_char_p
    L.pauli_status_string.argtypes = [st]
    L.pauli_last_error.restype = ctypes.c_char_p
    L.pauli_last_error.argtypes = []
    L.paulisum_create.restype = st
    L.paulisum_create.argtypes = [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.c_int,
                                  ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]
    L.paulisum_destroy.restype = st
    L.paulisum_destroy.argtypes = [_vp]
    L.paulisum_info.restype = st
    L.paulisum_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int)]
    L.paulisum_export.restype = st
    L.paulisum_export.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint32, _vp]
    L.pauli_outer_product.restype = st
    L.pauli_outer_product.argtypes = [_vp, _vp, ctypes.POINTER(_vp), _vp]
    L.pauli_merge.restype = st
    L.pauli_merge.argtypes = [_vp, ctypes.POINTER(MergeOpts), ctypes.POINTER(_vp), _vp]
    L.pauli_merge_into.restype = st
    L.pauli_merge_into.argtypes = [_vp, ctypes.POINTER(MergeOpts), _vp, _vp, _vp, _vp, _vp,
                                   ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _vp]
    L.pauli_outer_product_merged.restype = st
    L.pauli_outer_product_merged.argtypes = [_vp, _vp, ctypes.POINTER(MergeOpts),
                                             ctypes.POINTER(_vp), _vp]
    L.pauli_apply_clifford.restype = st
    L.pauli_apply_clifford.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.POINTER(_vp), _vp]
    L.pauli_sort_lex.restype = st
    L.pauli_sort_lex.argtypes = [_vp, ctypes.POINTER(_vp), _vp]
    L.pauli_commutator.restype = st
    L.pauli_commutator.argtypes = [_vp, _vp, ctypes.POINTER(MergeOpts), ctypes.POINTER(_vp), _vp]
    L.pauli_outer_product_batched.restype = st
    L.pauli_outer_product_batched.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp),
                                              ctypes.POINTER(_vp), ctypes.POINTER(MergeOpts),
                                              ctypes.POINTER(Tune), ctypes.POINTER(_vp), _vp]
    L.pauli_batch_plan_create.restype = st
    L.pauli_batch_plan_create.argtypes = [ctypes.c_int32, ctypes.POINTER(_vp),
                                          ctypes.POINTER(_vp), ctypes.POINTER(MergeOpts),
                                          ctypes.POINTER(Tune), _vp, ctypes.POINTER(_vp)]
    L.pauli_batch_plan_run.restype = st
    L.pauli_batch_plan_run.argtypes = [_vp, _vp]
    L.pauli_batch_plan_results.restype = st
    L.pauli_batch_plan_results.argtypes = [_vp, ctypes.POINTER(_vp), _vp]
    L.pauli_batch_plan_destroy.restype = st
    L.pauli_batch_plan_destroy.argtypes = [_vp]
    L.pauli_tune_save.restype = st
    L.pauli_tune_save.argtypes = [ctypes.c_char_p]
    L.pauli_tune_load.restype = st
    L.pauli_tune_load.argtypes = [ctypes.c_char_p]
    L.pauli_propagate_plan_create.restype = st
    L.pauli_propagate_plan_create.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32,
                                              ctypes.POINTER(MergeOpts), ctypes.c_int64, _vp,
                                              ctypes.POINTER(_vp)]
    L.pauli_propagate_plan_run.restype = st
    L.pauli_propagate_plan_run.argtypes = [_vp, _vp]
    L.pauli_propagate_plan_result.restype = st
    L.pauli_propagate_plan_result.argtypes = [_vp, ctypes.POINTER(_vp)]
    L.pauli_propagate_plan_destroy.restype = st
    L.pauli_propagate_plan_destroy.argtypes = [_vp]
    L.pauli_trim_memory.restype = st
    L.pauli_trim_memory.argtypes = []
    L.pauli_propagate.restype = st
    L.pauli_propagate.argtypes = [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int32,
                                  ctypes.POINTER(MergeOpts), ctypes.POINTER(_vp), _vp]
    L.pauli_set_allocator.restype = st
    L.pauli_set_allocator.argtypes = [_vp, _vp, _vp]
    L.pauli_set_memory_budget.restype = st
    L.pauli_set_memory_budget.argtypes = [ctypes.c_uint64]
    L.pauli_profile_enable.restype = st
    L.pauli_profile_enable.argtypes = [ctypes.c_int32]
    L.pauli_profile_read.restype = st
    L.pauli_profile_read.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_double)]
    _lib = L
    return L


def _check(status):
    if status != PAULI_OK:
        raise PauliError(status, lib().pauli_last_error().decode())


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


def _words(n):
    return (n + 63) // 64


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _opts(mode=PLAIN, drop_abs=-1.0, tau=0.0, key_bits=0):
    return MergeOpts(int(mode), float(drop_abs), float(tau), int(key_bits))


class PauliSum:
    """A Pauli sum resident on the GPU (opaque handle owned by this object)."""

    def __init__(self, handle):
        self._h = _vp(handle) if not isinstance(handle, _vp) else handle

    @classmethod
    def create(cls, n, x, z, phase=None, coef=None, dtype=None, stream=None):
        """From packed words x, z [m][W] uint64, phase [m] uint8 (or None),
        coef [m] complex.  numpy arrays (host) or torch CUDA tensors (device);
        dtype 'c128' (default for complex128 input) or 'c64'."""
        m = int(x.shape[0])
        dev = _is_torch(x) and x.is_cuda
        if dev:
            import torch
            if dtype is None:
                dtype = "c64" if coef.dtype == torch.complex64 else "c128"
            tdt = torch.complex64 if dtype == "c64" else torch.complex128
            x = x.contiguous().view(torch.int64)
            z = z.contiguous().view(torch.int64)
            coef = coef.to(tdt).contiguous()
            ph = phase.to(torch.uint8).contiguous() if phase is not None else None
            keep = (x, z, coef, ph)
            ptrs = (x.data_ptr(), z.data_ptr(), ph.data_ptr() if ph is not None else None,
                    coef.data_ptr())
            flags = PTR_DEVICE
        else:
            x = np.ascontiguousarray(x, dtype=np.uint64).reshape(m, _words(n))
            z = np.ascontiguousarray(z, dtype=np.uint64).reshape(m, _words(n))
            if coef is None:
                coef = np.ones(m, np.complex128)
            if dtype is None:
                dtype = "c64" if np.asarray(coef).dtype == np.complex64 else "c128"
            coef = np.ascontiguousarray(coef, dtype=np.complex64 if dtype == "c64"
                                        else np.complex128).reshape(m)
            ph = (np.ascontiguousarray(phase, dtype=np.uint8).reshape(m)
                  if phase is not None else None)
            keep = (x, z, coef, ph)
            ptrs = (x.ctypes.data, z.ctypes.data, ph.ctypes.data if ph is not None else None,
                    coef.ctypes.data)
            flags = 0
        out = _vp()
        _check(lib().paulisum_create(int(n), m, ptrs[0], ptrs[1], ptrs[2], ptrs[3],
                                     C64 if dtype == "c64" else C128, flags, _stream(stream),
                                     ctypes.byref(out)))
        del keep
        return cls(out)

    @classmethod
    def from_dict(cls, d, dtype=None, stream=None):
        return cls.create(d["n"], d["x"], d["z"], d.get("phase"), d["coef"], dtype=dtype,
                          stream=stream)

    def destroy(self):
        if self._h is not None and self._h.value:
            _check(lib().paulisum_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self):
        n = ctypes.c_int32()
        m = ctypes.c_int64()
        dt = ctypes.c_int()
        _check(lib().paulisum_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(dt)))
        return n.value, m.value, ("c64" if dt.value == C64 else "c128")

    @property
    def n(self):
        return self.info()[0]

    @property
    def m(self):
        return self.info()[1]

    def __len__(self):
        return self.m

    def export(self, stream=None):
        """Host copy: dict(n, x, z, phase, coef, fp) of numpy arrays."""
        n, m, dt = self.info()
        W = _words(n)
        x = np.zeros((m, W), np.uint64)
        z = np.zeros((m, W), np.uint64)
        ph = np.zeros(m, np.uint8)
        c = np.zeros(m, np.complex64 if dt == "c64" else np.complex128)
        fp = np.zeros(m, np.uint64)
        _check(lib().paulisum_export(self._h, x.ctypes.data, z.ctypes.data, ph.ctypes.data,
                                     c.ctypes.data, fp.ctypes.data, 0, _stream(stream)))
        return {"n": n, "x": x, "z": z, "phase": ph, "coef": c, "fp": fp}

    def export_torch(self, device="cuda", stream=None):
        """Device copy as torch tensors (x, z as int64 views of the words)."""
        import torch
        n, m, dt = self.info()
        W = _words(n)
        x = torch.empty((m, W), dtype=torch.int64, device=device)
        z = torch.empty((m, W), dtype=torch.int64, device=device)
        ph = torch.empty(m, dtype=torch.uint8, device=device)
        c = torch.empty(m, dtype=torch.complex64 if dt == "c64" else torch.complex128,
                        device=device)
        fp = torch.empty(m, dtype=torch.int64, device=device)
        _check(lib().paulisum_export(self._h, x.data_ptr(), z.data_ptr(), ph.data_ptr(),
                                     c.data_ptr(), fp.data_ptr(), PTR_DEVICE, _stream(stream)))
        return {"n": n, "x": x, "z": z, "phase": ph, "coef": c, "fp": fp}


def outer_product(a: PauliSum, b: PauliSum, stream=None) -> PauliSum:
    out = _vp()
    _check(lib().pauli_outer_product(a.handle, b.handle, ctypes.byref(out), _stream(stream)))
    return PauliSum(out)


def merge(s: PauliSum, mode=PLAIN, drop_abs=-1.0, tau=0.0, key_bits=0, stream=None) -> PauliSum:
    out = _vp()
    o = _opts(mode, drop_abs, tau, key_bits)
    _check(lib().pauli_merge(s.handle, ctypes.byref(o), ctypes.byref(out), _stream(stream)))
    return PauliSum(out)


def merge_into(s: PauliSum, out_x, out_z, out_phase, out_coef, out_fp, out_ld: int,
               mode=PLAIN, drop_abs=-1.0, tau=0.0, key_bits=0, stream=None) -> int:
    """pauli_merge_into: merge(s) written to caller-owned device arrays
    (device pointers as ints, or tensors: out_x/out_z (W, out_ld) uint64
    words, out_phase (out_ld,) uint8, out_coef (out_ld,) complex of the
    result's dtype, out_fp (out_ld,) uint64).  Returns the merged count."""
    def ptr(a):
        return a.data_ptr() if _is_torch(a) else int(a)
    m = ctypes.c_int64(-1)
    o = _opts(mode, drop_abs, tau, key_bits)
    _check(lib().pauli_merge_into(s.handle, ctypes.byref(o), ptr(out_x), ptr(out_z),
                                  ptr(out_phase), ptr(out_coef), ptr(out_fp), int(out_ld),
                                  ctypes.byref(m), _stream(stream)))
    return m.value


def outer_product_merged(a: PauliSum, b: PauliSum, mode=PLAIN, drop_abs=-1.0, tau=0.0,
                         key_bits=0, stream=None) -> PauliSum:
    out = _vp()
    o = _opts(mode, drop_abs, tau, key_bits)
    _check(lib().pauli_outer_product_merged(a.handle, b.handle, ctypes.byref(o),
                                            ctypes.byref(out), _stream(stream)))
    return PauliSum(out)


def commutator(a: PauliSum, b: PauliSum, mode=PLAIN, drop_abs=-1.0, tau=0.0, key_bits=0,
               stream=None) -> PauliSum:
    """[a, b] = a*b - b*a, merged (pauli_commutator): one term per string that
    an anticommuting pair gives, coefficient sum of 2 i^k c_a c_b."""
    out = _vp()
    o = _opts(mode, drop_abs, tau, key_bits)
    _check(lib().pauli_commutator(a.handle, b.handle, ctypes.byref(o), ctypes.byref(out),
                                  _stream(stream)))
    return PauliSum(out)


GATE_H, GATE_S, GATE_SDG, GATE_X, GATE_Y, GATE_Z, GATE_CX, GATE_CZ, GATE_SWAP = range(9)


def apply_clifford(s: PauliSum, gates, stream=None) -> PauliSum:
    """Every term conjugated by the gates in order (pauli_apply_clifford).
    gates: sequence of (kind, q0[, q1]); the output keeps the term order."""
    g = np.zeros((len(gates), 3), dtype=np.int32)
    for i, gate in enumerate(gates):
        g[i, :len(gate)] = gate
    out = _vp()
    _check(lib().pauli_apply_clifford(s.handle, int(len(gates)), g.ctypes.data if len(gates) else None,
                                      ctypes.byref(out), _stream(stream)))
    return PauliSum(out)


def sort_lex(s: PauliSum, stream=None) -> PauliSum:
    """The terms of s in lexicographic order of their packed words
    (pauli_sort_lex): X[W-1] .. X[0] then Z[W-1] .. Z[0], each an unsigned
    64-bit integer; equal strings keep their order."""
    out = _vp()
    _check(lib().pauli_sort_lex(s.handle, ctypes.byref(out), _stream(stream)))
    return PauliSum(out)


ROTATE_PRODUCT, ROTATE_CONJUGATE = 0, 1


def propagate(s: PauliSum, px, pz, theta, rotate_mode=ROTATE_CONJUGATE, mode=PLAIN,
              drop_abs=-1.0, tau=0.0, key_bits=0, stream=None) -> PauliSum:
    """Rotation steps R_t = cos(theta_t) I - i sin(theta_t) P_t applied to s
    (pauli_propagate).  px, pz: (steps, W) packed words of the P_t; theta:
    (steps,) angles.  Each step ends with merge and the drop_abs truncation."""
    W = _words(s.info()[0])
    px = np.ascontiguousarray(px, dtype=np.uint64).reshape(-1, W)
    pz = np.ascontiguousarray(pz, dtype=np.uint64).reshape(-1, W)
    th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
    if not (px.shape[0] == pz.shape[0] == th.size):
        raise ValueError("px, pz and theta must have one entry per step")
    o = _opts(mode, drop_abs, tau, key_bits)
    out = _vp()
    _check(lib().pauli_propagate(s.handle, int(th.size), px.ctypes.data, pz.ctypes.data,
                                 th.ctypes.data, int(rotate_mode), ctypes.byref(o),
                                 ctypes.byref(out), _stream(stream)))
    return PauliSum(out)


def _tune(tune):
    """None, an int (bucket bits) or a dict of pauli_tune_t fields."""
    if tune is None:
        return None
    if isinstance(tune, dict):
        return Tune(**{k: int(v) for k, v in tune.items()})
    return Tune(bucket_bits=int(tune))


def outer_product_batched(a_list, b_list, mode=PLAIN, drop_abs=-1.0, tau=0.0, key_bits=0,
                          tune=None, stream=None):
    nb = len(a_list)
    A = (_vp * max(nb, 1))(*[x.handle for x in a_list])
    B = (_vp * max(nb, 1))(*[x.handle for x in b_list])
    O = (_vp * max(nb, 1))()
    o = _opts(mode, drop_abs, tau, key_bits)
    t = _tune(tune)
    _check(lib().pauli_outer_product_batched(nb, A, B, ctypes.byref(o),
                                             ctypes.byref(t) if t is not None else None, O,
                                             _stream(stream)))
    return [PauliSum(O[i]) for i in range(nb)]


class BatchPlan:
    """pauli_batch_plan_*: the batched form captured into a HIP graph.  The
    plan keeps references to its input sums."""

    def __init__(self, a_list, b_list, mode=PLAIN, drop_abs=-1.0, tau=0.0, key_bits=0,
                 tune=None, stream=None):
        self._inputs = (list(a_list), list(b_list))
        nb = len(a_list)
        self.nb = nb
        A = (_vp * max(nb, 1))(*[x.handle for x in a_list])
        B = (_vp * max(nb, 1))(*[x.handle for x in b_list])
        o = _opts(mode, drop_abs, tau, key_bits)
        t = _tune(tune)
        h = _vp()
        _check(lib().pauli_batch_plan_create(nb, A, B, ctypes.byref(o),
                                             ctypes.byref(t) if t is not None else None,
                                             _stream(stream), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(lib().pauli_batch_plan_run(self._h, _stream(stream)))

    def results(self, stream=None):
        O = (_vp * max(self.nb, 1))()
        _check(lib().pauli_batch_plan_results(self._h, O, _stream(stream)))
        return [PauliSum(O[i]) for i in range(self.nb)]

    def destroy(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().pauli_batch_plan_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class PropagatePlan:
    """pauli_propagate_plan_*: the propagation loop captured into a HIP
    graph, every state holding at most max_terms terms.  The plan keeps a
    reference to its input sum."""

    def __init__(self, s, px, pz, theta, max_terms, rotate_mode=ROTATE_CONJUGATE, mode=PLAIN,
                 drop_abs=-1.0, tau=0.0, key_bits=0, stream=None):
        self._input = s
        W = _words(s.info()[0])
        px = np.ascontiguousarray(px, dtype=np.uint64).reshape(-1, W)
        pz = np.ascontiguousarray(pz, dtype=np.uint64).reshape(-1, W)
        th = np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
        if not (px.shape[0] == pz.shape[0] == th.size):
            raise ValueError("px, pz and theta must have one entry per step")
        o = _opts(mode, drop_abs, tau, key_bits)
        h = _vp()
        _check(lib().pauli_propagate_plan_create(s.handle, int(th.size), px.ctypes.data,
                                                 pz.ctypes.data, th.ctypes.data, int(rotate_mode),
                                                 ctypes.byref(o), int(max_terms),
                                                 _stream(stream), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(lib().pauli_propagate_plan_run(self._h, _stream(stream)))

    def result(self):
        out = _vp()
        _check(lib().pauli_propagate_plan_result(self._h, ctypes.byref(out)))
        return PauliSum(out)

    def destroy(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().pauli_propagate_plan_destroy(self._h))
            self._h = _vp()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def tune_save(path):
    _check(lib().pauli_tune_save(os.fsencode(path)))


def tune_load(path):
    _check(lib().pauli_tune_load(os.fsencode(path)))


def trim_memory():
    """Return the device memory the library holds but does not use."""
    _check(lib().pauli_trim_memory())


def set_memory_budget(nbytes: int):
    _check(lib().pauli_set_memory_budget(int(nbytes)))


_ALLOC_T = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp, _vp)
_FREE_T = ctypes.CFUNCTYPE(None, _vp, _vp, _vp)
_hooks = None


def use_torch_allocator(enable=True):
    """Back every library allocation by torch's caching allocator."""
    global _hooks
    if not enable:
        _check(lib().pauli_set_allocator(None, None, None))
        _hooks = None
        return
    import torch

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream or 0)
        except Exception:
            return None

    def _free(ptr, stream, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    _hooks = (_ALLOC_T(_alloc), _FREE_T(_free))
    _check(lib().pauli_set_allocator(ctypes.cast(_hooks[0], _vp), ctypes.cast(_hooks[1], _vp),
                                     None))


def profile_enable(on=True):
    """Start (clearing totals) or stop per-stage HIP-event timing."""
    _check(lib().pauli_profile_enable(1 if on else 0))


def profile_read():
    """{stage: (total_ms, launches, algorithmic_bytes)} for stages that ran."""
    out = {}
    for i, name in enumerate(STAGES):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        by = ctypes.c_double()
        _check(lib().pauli_profile_read(i, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        if n.value:
            out[name] = (ms.value, n.value, by.value)
    return out

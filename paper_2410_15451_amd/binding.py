"""ctypes binding of the C-ABI in include/leiden.h (argument marshalling only).

Every step of the computation runs in the HIP library; this module converts
numpy arrays or torch tensors into pointers and raises on error codes.  It
never falls back to anything else: without the built library it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libleiden_mi355x.so")

LEIDEN_OK, LEIDEN_EINVAL, LEIDEN_ENOMEM, LEIDEN_EDEVICE, LEIDEN_ESTATE = 0, -1, -2, -3, -4
MODES = {"nd": 0, "ds": 1, "df": 2}

# Every symbol include/leiden.h declares.
EXPORTS = ("leiden_default_opts", "leiden_graph_create", "leiden_graph_destroy", "leiden_graph_nnz", "leiden_static",
           "leiden_update", "leiden_modularity", "leiden_graph_export", "leiden_state_export",
           "leiden_state_import", "leiden_last_error", "leiden_kernel_name")


# leiden_kernel values (timed kernels)
KERNELS = {"none": 0, "hub_insert": 1}


def kernel_name(kernel):
    """Symbol of a timed kernel as profilers list it."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    f = lib().leiden_kernel_name
    f.restype = ctypes.c_char_p
    r = f(ctypes.c_int32(k))
    if r is None:
        raise ValueError("unknown kernel %r" % (kernel,))
    return r.decode()


class LeidenOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("tau_re_num", ctypes.c_uint32), ("tau_re_den", ctypes.c_uint32),
                ("tol_decline", ctypes.c_uint32), ("max_iters", ctypes.c_uint32), ("max_passes", ctypes.c_uint32),
                ("move_classes", ctypes.c_uint32), ("refine_rounds", ctypes.c_uint32),
                ("deterministic", ctypes.c_int32), ("compute_modularity", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("timed_kernel", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class LeidenStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint32), ("iters", ctypes.c_uint32 * 16), ("subrounds", ctypes.c_uint32 * 16),
                ("affected", ctypes.c_uint64), ("split_marked", ctypes.c_uint64),
                ("refine_marked", ctypes.c_uint64), ("moves", ctypes.c_uint64), ("refine_moves", ctypes.c_uint64),
                ("edges_scanned", ctypes.c_uint64), ("refined_first_pass", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("ms_total", ctypes.c_double), ("ms_batch", ctypes.c_double),
                ("ms_modularity", ctypes.c_double), ("nnz", ctypes.c_uint64),
                ("kt_launches", ctypes.c_uint32), ("kt_pad_", ctypes.c_uint32), ("kt_ms", ctypes.c_double),
                ("kt_units", ctypes.c_uint64), ("kt_bytes", ctypes.c_double)]

    def as_dict(self):
        p = self.passes
        return {"passes": p, "iters": list(self.iters[:min(p, 16)]), "subrounds": list(self.subrounds[:min(p, 16)]),
                "affected": self.affected, "split_marked": self.split_marked, "moves": self.moves,
                "refine_moves": self.refine_moves, "edges_scanned": self.edges_scanned,
                "refined_first_pass": self.refined_first_pass, "ms_total": self.ms_total,
                "ms_batch": self.ms_batch, "ms_modularity": self.ms_modularity, "nnz": self.nnz,
                "kt_launches": self.kt_launches, "kt_ms": self.kt_ms, "kt_units": self.kt_units,
                "kt_bytes": self.kt_bytes}


class LeidenError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("leiden error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load the HIP library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library missing: %s (run __graft_entry__.build())" % LIB_PATH)
        # PyTorch ships its own HIP runtime under the same soname; loading it
        # first makes the library bind to that one runtime, so torch's device
        # pointers and streams are valid handles in every call.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, i32, dbl = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        L.leiden_default_opts.argtypes = [P]
        L.leiden_default_opts.restype = i32
        L.leiden_graph_create.argtypes = [i32, u32, u64, P, P, P, i32, dbl, ctypes.POINTER(P)]
        L.leiden_graph_create.restype = i32
        L.leiden_graph_destroy.argtypes = [P]
        L.leiden_graph_destroy.restype = None
        L.leiden_graph_nnz.argtypes = [P, ctypes.POINTER(u64)]
        L.leiden_graph_nnz.restype = i32
        L.leiden_static.argtypes = [P, P, P, i32, P, P]
        L.leiden_static.restype = i32
        L.leiden_update.argtypes = [P, P, u64, P, u64, i32, P, i32, i32, P, P, i32, P, P]
        L.leiden_update.restype = i32
        L.leiden_modularity.argtypes = [P, P, i32, P]
        L.leiden_modularity.restype = i32
        L.leiden_graph_export.argtypes = [P, P, P, P]
        L.leiden_graph_export.restype = i32
        L.leiden_state_export.argtypes = [P, P, P, P, P]
        L.leiden_state_export.restype = i32
        L.leiden_state_import.argtypes = [P, P, P, P, P]
        L.leiden_state_import.restype = i32
        L.leiden_last_error.argtypes = []
        L.leiden_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != LEIDEN_OK:
        raise LeidenError(rc, lib().leiden_last_error().decode())


def _ptr(a):
    """(pointer, on_device) of a numpy array or torch tensor (None -> null)."""
    if a is None:
        return None, 0
    if hasattr(a, "data_ptr"):  # torch tensor
        return ctypes.c_void_p(a.data_ptr()), 1 if a.is_cuda else 0
    return a.ctypes.data_as(ctypes.c_void_p), 0


def default_opts(**kw) -> LeidenOpts:
    o = LeidenOpts()
    _check(lib().leiden_default_opts(ctypes.byref(o)))
    for k, v in kw.items():
        if k == "tau_re":
            o.tau_re_num, o.tau_re_den = v
        elif k == "stream":
            o.stream = ctypes.c_void_p(v)
        elif k == "timed_kernel" and isinstance(v, str):
            o.timed_kernel = KERNELS[v]
        else:
            setattr(o, k, v)
    return o


@dataclass
class Result:
    membership: object
    q: float
    stats: dict


class Graph:
    """A graph handle on one GPU (owns the device CSR and the community state)."""

    def __init__(self, offs, cols, w, n=None, device=0, slack=0.2):
        if hasattr(offs, "data_ptr") != hasattr(cols, "data_ptr"):
            raise TypeError("offsets, cols and w must all be numpy arrays or all torch tensors")
        if not hasattr(offs, "data_ptr"):
            offs = np.ascontiguousarray(offs, np.int64)
            cols = np.ascontiguousarray(cols, np.uint32)
            w = np.ascontiguousarray(w, np.uint32)
        n = int(offs.shape[0] - 1) if n is None else n
        nnz = int(cols.shape[0])
        po, dev = _ptr(offs)
        pc, _ = _ptr(cols)
        pw, _ = _ptr(w)
        h = ctypes.c_void_p()
        _check(lib().leiden_graph_create(device, n, nnz, po, pc, pw, dev, float(slack), ctypes.byref(h)))
        self._h = h
        self.n = n
        self.device = device

    @classmethod
    def from_csr(cls, csr, **kw):
        return cls(csr.offs, csr.cols, csr.w, n=csr.n, **kw)

    def close(self):
        if getattr(self, "_h", None):
            lib().leiden_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nnz(self) -> int:
        x = ctypes.c_uint64()
        _check(lib().leiden_graph_nnz(self._h, ctypes.byref(x)))
        return int(x.value)

    def _out(self, out):
        if out is None:
            return np.zeros(self.n, np.uint32)
        return out

    def static(self, out=None, **opts) -> Result:
        o = default_opts(**opts)
        out = self._out(out)
        po, dev = _ptr(out)
        q = ctypes.c_double()
        st = LeidenStats()
        _check(lib().leiden_static(self._h, ctypes.byref(o), po, dev, ctypes.byref(q), ctypes.byref(st)))
        return Result(out, q.value, st.as_dict())

    def update(self, dels, ins, mode="df", prev=None, out=None, **opts) -> Result:
        """dels: uint32[nd, 2] pairs; ins: uint32[ni, 3] (u, v, w); numpy or device tensors."""
        o = default_opts(**opts)
        if not hasattr(dels, "data_ptr"):
            dels = np.ascontiguousarray(dels, np.uint32).reshape(-1, 2)
        if not hasattr(ins, "data_ptr"):
            ins = np.ascontiguousarray(ins, np.uint32).reshape(-1, 3)
        nd, ni = int(dels.shape[0]), int(ins.shape[0])
        pd, dev_d = _ptr(dels)
        pi, dev_i = _ptr(ins)
        if nd and ni and dev_d != dev_i:
            raise TypeError("deletions and insertions must both be host or both device buffers")
        dev_b = dev_d if nd else dev_i
        if prev is not None and not hasattr(prev, "data_ptr"):
            prev = np.ascontiguousarray(prev, np.uint32)
        pp, dev_p = _ptr(prev)
        out = self._out(out)
        po, dev_o = _ptr(out)
        q = ctypes.c_double()
        st = LeidenStats()
        _check(lib().leiden_update(self._h, pd, nd, pi, ni, dev_b, pp, dev_p, MODES.get(mode, mode),
                                   ctypes.byref(o), po, dev_o, ctypes.byref(q), ctypes.byref(st)))
        return Result(out, q.value, st.as_dict())

    def modularity(self, membership) -> float:
        if not hasattr(membership, "data_ptr"):
            membership = np.ascontiguousarray(membership, np.uint32)
        p, dev = _ptr(membership)
        q = ctypes.c_double()
        _check(lib().leiden_modularity(self._h, p, dev, ctypes.byref(q)))
        return q.value

    def export(self):
        """(offs int64[n+1], cols uint32[nnz], w uint32[nnz]) of the current graph, rows sorted."""
        nnz = self.nnz
        offs = np.zeros(self.n + 1, np.int64)
        cols = np.zeros(max(nnz, 1), np.uint32)
        w = np.zeros(max(nnz, 1), np.uint32)
        _check(lib().leiden_graph_export(self._h, _ptr(offs)[0], _ptr(cols)[0], _ptr(w)[0]))
        return offs, cols[:nnz], w[:nnz]

    def state(self):
        """(C, K, Sigma, DeltaSigma) as numpy arrays."""
        n = self.n
        C = np.zeros(n, np.uint32)
        K, S, dS = (np.zeros(n, np.int64) for _ in range(3))
        _check(lib().leiden_state_export(self._h, _ptr(C)[0], _ptr(K)[0], _ptr(S)[0], _ptr(dS)[0]))
        return C, K, S, dS

    def set_state(self, C, K, S, dS):
        arrs = [np.ascontiguousarray(C, np.uint32)] + [np.ascontiguousarray(x, np.int64) for x in (K, S, dS)]
        _check(lib().leiden_state_import(self._h, *[_ptr(a)[0] for a in arrs]))

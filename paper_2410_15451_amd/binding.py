"""ctypes binding of the C-ABI in include/leiden.h (argument marshalling only).

Every step of the computation runs in the HIP library; this module converts
numpy arrays or torch tensors into pointers and raises on error codes.  It
never falls back to anything else: without the built library it raises.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libleiden_mi355x.so")

LEIDEN_OK, LEIDEN_EINVAL, LEIDEN_ENOMEM, LEIDEN_EDEVICE, LEIDEN_ESTATE, LEIDEN_EBUSY = 0, -1, -2, -3, -4, -5
MODES = {"nd": 0, "ds": 1, "df": 2}

# Every symbol include/leiden.h declares.
EXPORTS = ("leiden_default_opts", "leiden_graph_create", "leiden_graph_destroy", "leiden_graph_nnz", "leiden_static",
           "leiden_update", "leiden_modularity", "leiden_graph_export", "leiden_state_export",
           "leiden_state_import", "leiden_last_error", "leiden_kernel_name", "leiden_get_tuning",
           "leiden_set_tuning", "leiden_autotune", "leiden_batch_run", "leiden_server_create",
           "leiden_server_destroy", "leiden_server_add_graph", "leiden_server_remove_graph", "leiden_server_submit",
           "leiden_server_wait", "leiden_server_get_stats", "leiden_modularity_noalloc", "leiden_forest_create",
           "leiden_forest_results", "leiden_forest_info", "leiden_server_footprint", "leiden_set_memory_budget",
           "leiden_memory_used")

FOREST_ITER_HIST = 16  # passes whose iteration counts leiden_forest_results returns


# leiden_work order (work counters of a call)
WORK_NAMES = ("scan0", "scan_up", "decided", "refine_scan", "marks", "split", "agg_in", "agg_out", "merge")

# leiden_kernel values (timed kernels)
KERNELS = {"none": 0, "hub_insert": 1, "agg_big": 2}


def kernel_name(kernel):
    """Symbol of a timed kernel as profilers list it."""
    k = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    r = lib().leiden_kernel_name(k)
    if r is None:
        raise ValueError("unknown kernel %r" % (kernel,))
    return r.decode()


class LeidenOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("tau_re_num", ctypes.c_uint32), ("tau_re_den", ctypes.c_uint32),
                ("tol_decline", ctypes.c_uint32), ("max_iters", ctypes.c_uint32), ("max_passes", ctypes.c_uint32),
                ("move_classes", ctypes.c_uint32), ("refine_rounds", ctypes.c_uint32),
                ("deterministic", ctypes.c_int32), ("compute_modularity", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("timed_kernel", ctypes.c_int32), ("split_all", ctypes.c_int32)]


class LeidenStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint32), ("iters", ctypes.c_uint32 * 16), ("subrounds", ctypes.c_uint32 * 16),
                ("affected", ctypes.c_uint64), ("split_marked", ctypes.c_uint64),
                ("refine_marked", ctypes.c_uint64), ("moves", ctypes.c_uint64), ("refine_moves", ctypes.c_uint64),
                ("edges_scanned", ctypes.c_uint64), ("refined_first_pass", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("ms_total", ctypes.c_double), ("ms_batch", ctypes.c_double),
                ("ms_modularity", ctypes.c_double), ("nnz", ctypes.c_uint64),
                ("kt_launches", ctypes.c_uint32), ("kt_pad_", ctypes.c_uint32), ("kt_ms", ctypes.c_double),
                ("kt_units", ctypes.c_uint64), ("kt_bytes", ctypes.c_double),
                ("work", ctypes.c_uint64 * 9), ("sweep_vertices", ctypes.c_uint64),
                ("batch_entries", ctypes.c_uint64), ("algo_bytes", ctypes.c_double)]

    def as_dict(self):
        p = self.passes
        return {"passes": p, "iters": list(self.iters[:min(p, 16)]), "subrounds": list(self.subrounds[:min(p, 16)]),
                "affected": self.affected, "split_marked": self.split_marked, "moves": self.moves,
                "refine_moves": self.refine_moves, "edges_scanned": self.edges_scanned,
                "refined_first_pass": self.refined_first_pass, "ms_total": self.ms_total,
                "ms_batch": self.ms_batch, "ms_modularity": self.ms_modularity, "nnz": self.nnz,
                "kt_launches": self.kt_launches, "kt_ms": self.kt_ms, "kt_units": self.kt_units,
                "kt_bytes": self.kt_bytes, "work": dict(zip(WORK_NAMES, self.work)),
                "sweep_vertices": self.sweep_vertices, "batch_entries": self.batch_entries,
                "algo_bytes": self.algo_bytes}


class LeidenTuning(ctypes.Structure):
    _fields_ = [("bin_max_degree", ctypes.c_uint32 * 5), ("agg_emit_slots", ctypes.c_uint32),
                ("probe_ms", ctypes.c_double), ("agg_probe_ms", ctypes.c_double)]

    def as_dict(self):
        return {"bin_max_degree": list(self.bin_max_degree), "agg_emit_slots": self.agg_emit_slots,
                "probe_ms": self.probe_ms, "agg_probe_ms": self.agg_probe_ms}


class LeidenBatchItem(ctypes.Structure):
    _fields_ = [("dels", ctypes.c_void_p), ("n_del", ctypes.c_uint64), ("ins", ctypes.c_void_p),
                ("n_ins", ctypes.c_uint64)]


class LeidenServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64), ("waiting", ctypes.c_uint64),
                ("graphs", ctypes.c_uint32), ("pad_", ctypes.c_uint32), ("hbm_reserved", ctypes.c_uint64),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("service_p50_ms", ctypes.c_double), ("service_p99_ms", ctypes.c_double),
                ("updated_edges_per_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


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
        L.leiden_set_memory_budget.argtypes = [P, u64]
        L.leiden_set_memory_budget.restype = i32
        L.leiden_memory_used.argtypes = [P, ctypes.POINTER(u64)]
        L.leiden_memory_used.restype = i32
        L.leiden_static.argtypes = [P, P, P, i32, P, P]
        L.leiden_static.restype = i32
        L.leiden_update.argtypes = [P, P, u64, P, u64, i32, P, i32, i32, P, P, i32, P, P]
        L.leiden_update.restype = i32
        L.leiden_modularity.argtypes = [P, P, i32, P]
        L.leiden_modularity.restype = i32
        L.leiden_modularity_noalloc.argtypes = [P, P, P, P]
        L.leiden_modularity_noalloc.restype = i32
        L.leiden_graph_export.argtypes = [P, P, P, P]
        L.leiden_graph_export.restype = i32
        L.leiden_state_export.argtypes = [P, P, P, P, P]
        L.leiden_state_export.restype = i32
        L.leiden_state_import.argtypes = [P, P, P, P, P]
        L.leiden_state_import.restype = i32
        L.leiden_last_error.argtypes = []
        L.leiden_last_error.restype = ctypes.c_char_p
        L.leiden_kernel_name.argtypes = [i32]
        L.leiden_kernel_name.restype = ctypes.c_char_p
        for name, args in (("leiden_get_tuning", [P, P]), ("leiden_set_tuning", [P, P]),
                           ("leiden_autotune", [P, P, P]),
                           ("leiden_batch_run", [P, u32, P, i32, P, u32, P, P, P]),
                           ("leiden_server_create", [i32, u64, u32, ctypes.POINTER(P)]),
                           ("leiden_server_add_graph", [P, u32, u64, P, P, P, i32, dbl, P, ctypes.POINTER(u32)]),
                           ("leiden_server_remove_graph", [P, u32]),
                           ("leiden_server_submit", [P, u32, P, u64, P, u64, i32, P, ctypes.POINTER(u64)]),
                           ("leiden_server_wait", [P, u64, P, P, P, P, P]),
                           ("leiden_server_get_stats", [P, P]),
                           ("leiden_forest_create", [i32, u32, P, u64, P, P, P, i32, dbl, ctypes.POINTER(P)]),
                           ("leiden_forest_results", [P, P, P, P]),
                           ("leiden_forest_info", [P, P, P]),
                           ("leiden_server_footprint", [u32, u64, dbl, ctypes.POINTER(u64)])):
            getattr(L, name).argtypes = args
            getattr(L, name).restype = i32
        L.leiden_server_destroy.argtypes = [P]
        L.leiden_server_destroy.restype = None
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


# Live handles and servers, closed at interpreter exit (servers first: their
# worker threads must be joined while the HIP runtime is still up).
_LIVE_SERVERS = weakref.WeakSet()
_LIVE_GRAPHS = weakref.WeakSet()


@atexit.register
def _close_all():
    for s in list(_LIVE_SERVERS):
        try:
            s.close()
        except Exception:
            pass
    for g in list(_LIVE_GRAPHS):
        try:
            g.close()
        except Exception:
            pass


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
        _LIVE_GRAPHS.add(self)

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

    def set_memory_budget(self, budget_bytes: int):
        """Bound the handle's device memory (0: no bound)."""
        _check(lib().leiden_set_memory_budget(self._h, ctypes.c_uint64(int(budget_bytes))))

    def memory_used(self) -> int:
        x = ctypes.c_uint64()
        _check(lib().leiden_memory_used(self._h, ctypes.byref(x)))
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

    def modularity_noalloc(self, membership, stream=None) -> float:
        """Eq. 1 of a device-resident membership without any allocation by
        the library (leiden_modularity_noalloc)."""
        if not hasattr(membership, "data_ptr"):
            raise TypeError("membership must be a device tensor")
        pm, dev = _ptr(membership)
        if not dev:
            raise TypeError("membership must be a device tensor")
        q = ctypes.c_double()
        _check(lib().leiden_modularity_noalloc(self._h, pm, ctypes.c_void_p(stream), ctypes.byref(q)))
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

    def tuning(self) -> dict:
        t = LeidenTuning()
        _check(lib().leiden_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, bin_max_degree=None, agg_emit_slots=0):
        t = LeidenTuning()
        cur = self.tuning()["bin_max_degree"] if bin_max_degree is None else bin_max_degree
        for i, x in enumerate(cur):
            t.bin_max_degree[i] = int(x)
        t.agg_emit_slots = int(agg_emit_slots)
        _check(lib().leiden_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, **opts) -> dict:
        """Pick the degree-bin thresholds for this graph by measurement."""
        o = default_opts(**opts)
        t = LeidenTuning()
        _check(lib().leiden_autotune(self._h, ctypes.byref(o), ctypes.byref(t)))
        return t.as_dict()

    def set_state(self, C, K, S, dS):
        arrs = [np.ascontiguousarray(C, np.uint32)] + [np.ascontiguousarray(x, np.int64) for x in (K, S, dS)]
        _check(lib().leiden_state_import(self._h, *[_ptr(a)[0] for a in arrs]))


class Forest(Graph):
    """Many independent graphs in one handle (leiden_forest_create): every
    phase runs as one launch over all of them.  Memberships are labels
    inside each graph; batch pairs name forest vertices (first_vertex[q] +
    the vertex inside graph q)."""

    def __init__(self, sizes, offs, cols, w, device=0, slack=0.2):
        sizes = np.ascontiguousarray(sizes, np.uint32)
        if hasattr(offs, "data_ptr") != hasattr(cols, "data_ptr"):
            raise TypeError("offsets, cols and w must all be numpy arrays or all torch tensors")
        if not hasattr(offs, "data_ptr"):
            offs = np.ascontiguousarray(offs, np.int64)
            cols = np.ascontiguousarray(cols, np.uint32)
            w = np.ascontiguousarray(w, np.uint32)
        nnz = int(cols.shape[0])
        po, dev = _ptr(offs)
        pc, _ = _ptr(cols)
        pw, _ = _ptr(w)
        h = ctypes.c_void_p()
        _check(lib().leiden_forest_create(device, int(sizes.shape[0]), sizes.ctypes.data, nnz, po, pc, pw, dev,
                                          float(slack), ctypes.byref(h)))
        self._h = h
        self.n = int(sizes.sum(dtype=np.uint64))
        self.device = device
        self.sizes = sizes
        self.first = np.zeros(sizes.shape[0] + 1, np.uint32)
        nq = ctypes.c_uint32()
        _check(lib().leiden_forest_info(self._h, ctypes.byref(nq), self.first.ctypes.data))
        _LIVE_GRAPHS.add(self)

    @property
    def n_graphs(self) -> int:
        return int(self.sizes.shape[0])

    def results(self):
        """(q float64[n_graphs], passes uint32[n_graphs], iters uint32[n_graphs, 16]) of the last call."""
        nq = self.n_graphs
        q = np.zeros(nq, np.float64)
        passes = np.zeros(nq, np.uint32)
        iters = np.zeros((nq, FOREST_ITER_HIST), np.uint32)
        _check(lib().leiden_forest_results(self._h, q.ctypes.data, passes.ctypes.data, iters.ctypes.data))
        return q, passes, iters

    def modularity(self, membership):
        """Eq. 1 of every graph (float64[n_graphs]) under labels inside each graph."""
        super().modularity(membership)
        q = np.zeros(self.n_graphs, np.float64)
        _check(lib().leiden_forest_results(self._h, q.ctypes.data, None, None))
        return q


def _batch_arrays(dels, ins):
    d = np.ascontiguousarray(dels, np.uint32).reshape(-1, 2)
    i = np.ascontiguousarray(ins, np.uint32).reshape(-1, 3)
    return d, i


def batch_run(graphs, batches=None, mode="df", streams=8, **opts):
    """Batched form: leiden_static (batches None) or leiden_update on every
    handle, `streams` graphs at a time.  Returns (memberships, q values)."""
    count = len(graphs)
    o = default_opts(**opts)
    hs = (ctypes.c_void_p * count)(*[g._h.value for g in graphs])
    outs = [np.zeros(g.n, np.uint32) for g in graphs]
    po = (ctypes.c_void_p * count)(*[o_.ctypes.data for o_ in outs])
    q = np.zeros(count, np.float64)
    st = (ctypes.c_int * count)()
    items = None
    keep = []
    if batches is not None:
        items = (LeidenBatchItem * count)()
        for k, (d, i) in enumerate(batches):
            d, i = _batch_arrays(d, i)
            keep += [d, i]
            items[k] = LeidenBatchItem(d.ctypes.data if d.shape[0] else None, d.shape[0],
                                       i.ctypes.data if i.shape[0] else None, i.shape[0])
    rc = lib().leiden_batch_run(hs, count, items, MODES.get(mode, mode), ctypes.byref(o), streams, po,
                                q.ctypes.data_as(ctypes.c_void_p), st)
    _check(rc)
    return outs, q


def server_footprint(n, nnz, slack=0.2) -> int:
    """Device bytes the server's admission charges for a graph (leiden_server_footprint)."""
    b = ctypes.c_uint64()
    _check(lib().leiden_server_footprint(n, ctypes.c_uint64(nnz), ctypes.c_double(slack), ctypes.byref(b)))
    return int(b.value)


class Server:
    """Serving form: tenant graphs under an HBM budget, update requests served
    by `workers` streams in arrival order (one request per graph at a time)."""

    def __init__(self, hbm_budget_bytes, workers=4, device=0):
        h = ctypes.c_void_p()
        _check(lib().leiden_server_create(device, ctypes.c_uint64(int(hbm_budget_bytes)), workers, ctypes.byref(h)))
        self._h = h
        self._n = {}
        _LIVE_SERVERS.add(self)

    def add_graph(self, csr, slack=0.2, **opts):
        o = default_opts(**opts)
        offs = np.ascontiguousarray(csr.offs, np.int64)
        cols = np.ascontiguousarray(csr.cols, np.uint32)
        w = np.ascontiguousarray(csr.w, np.uint32)
        gid = ctypes.c_uint32()
        _check(lib().leiden_server_add_graph(self._h, csr.n, ctypes.c_uint64(cols.shape[0]), _ptr(offs)[0],
                                             _ptr(cols)[0], _ptr(w)[0], 0, ctypes.c_double(slack), ctypes.byref(o),
                                             ctypes.byref(gid)))
        self._n[gid.value] = csr.n
        return gid.value

    def add_graph_device(self, n, offs, cols, w, slack=0.2, **opts):
        """Admit a graph given as device tensors (int64 offsets, 32-bit cols and weights)."""
        o = default_opts(**opts)
        gid = ctypes.c_uint32()
        _check(lib().leiden_server_add_graph(self._h, n, ctypes.c_uint64(int(cols.shape[0])), offs.data_ptr(),
                                             cols.data_ptr(), w.data_ptr(), 1, ctypes.c_double(slack),
                                             ctypes.byref(o), ctypes.byref(gid)))
        self._n[gid.value] = n
        return gid.value

    def remove_graph(self, gid):
        _check(lib().leiden_server_remove_graph(self._h, gid))
        self._n.pop(gid, None)

    def submit(self, gid, dels, ins, mode="df", **opts):
        o = default_opts(**opts)
        d, i = _batch_arrays(dels, ins)
        t = ctypes.c_uint64()
        _check(lib().leiden_server_submit(self._h, gid, d.ctypes.data if d.shape[0] else None,
                                          ctypes.c_uint64(d.shape[0]), i.ctypes.data if i.shape[0] else None,
                                          ctypes.c_uint64(i.shape[0]), MODES.get(mode, mode), ctypes.byref(o),
                                          ctypes.byref(t)))
        return (gid, t.value)

    def wait(self, ticket):
        gid, t = ticket
        out = np.zeros(self._n[gid], np.uint32)
        q, lat, svc = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        st = LeidenStats()
        _check(lib().leiden_server_wait(self._h, ctypes.c_uint64(t), out.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(q), ctypes.byref(st), ctypes.byref(lat), ctypes.byref(svc)))
        return Result(out, q.value, st.as_dict()), lat.value, svc.value

    def stats(self):
        s = LeidenServerStats()
        _check(lib().leiden_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            lib().leiden_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

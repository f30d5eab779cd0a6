"""Python binding of the CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and its
binding) never imports it.

The oracle itself is ``leiden_oracle.cpp``: a plain single-threaded C++17
implementation of the Static / ND / DS / DF Leiden method written from the
paper's algorithms (Alg. 1-12, Eq. 1-2).  ``build()`` compiles it with g++
(``-O2 -ffp-contract=off``, so no fused multiply-add changes the Eq. 2 rounding).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "leiden_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

SEQ, JACOBI = 0, 1
ND, DS, DF = 0, 1, 2
MODES = {"nd": ND, "ds": DS, "df": DF}


class OracleOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("tau_re_num", ctypes.c_uint32), ("tau_re_den", ctypes.c_uint32),
                ("tol_decline", ctypes.c_uint32), ("max_iters", ctypes.c_uint32),
                ("max_passes", ctypes.c_uint32), ("schedule", ctypes.c_int32),
                ("move_classes", ctypes.c_uint32), ("refine_rounds", ctypes.c_uint32),
                ("split_all", ctypes.c_int32)]


class OracleStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint32), ("iters", ctypes.c_uint32 * 16),
                ("subrounds", ctypes.c_uint32 * 16), ("affected", ctypes.c_uint64),
                ("split_marked", ctypes.c_uint64), ("refine_marked", ctypes.c_uint64),
                ("moves", ctypes.c_uint64), ("refine_moves", ctypes.c_uint64),
                ("edges_scanned", ctypes.c_uint64), ("refined_first_pass", ctypes.c_int32),
                ("m2_zero", ctypes.c_int32)]

    def as_dict(self):
        p = self.passes
        return {"passes": p, "iters": list(self.iters[:min(p, 16)]),
                "subrounds": list(self.subrounds[:min(p, 16)]), "affected": self.affected,
                "split_marked": self.split_marked, "refine_marked": self.refine_marked,
                "moves": self.moves, "refine_moves": self.refine_moves,
                "edges_scanned": self.edges_scanned, "refined_first_pass": self.refined_first_pass}


# A test that plants a mistake in the oracle points this at a mutated build.
_OVERRIDE = os.environ.get("LEIDEN_ORACLE_LIB")


def build(force: bool = False) -> str:
    """Compile liboracle.so next to its source (always when ``force``)."""
    if _OVERRIDE:
        return _OVERRIDE
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P = ctypes.c_void_p
        u32, u64, i64, i32, dbl = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.oracle_default_opts.argtypes = [P]
        L.oracle_delta_modularity.argtypes = [i64, i64, i64, i64, i64, i64]
        L.oracle_delta_modularity.restype = dbl
        L.oracle_modularity.argtypes = [u32, P, P, P, P]
        L.oracle_modularity.restype = dbl
        L.oracle_modularity64.argtypes = [u32, P, P, P, P, P, P, P]
        L.oracle_modularity64.restype = dbl
        L.oracle_aggregate.argtypes = [u32, P, P, P, P, u32, P, P, P]
        L.oracle_aggregate.restype = i64
        L.oracle_split.argtypes = [u32, P, P, P, P, P, P]
        L.oracle_trace_enable.argtypes = [i32]
        L.oracle_trace_moves.argtypes = [P, P, i64]
        L.oracle_trace_moves.restype = i64
        L.oracle_trace_passes.argtypes = [P, P, u32]
        L.oracle_trace_passes.restype = u32
        L.oracle_trace_projection.argtypes = [u32, i32, P]
        L.oracle_trace_projection.restype = i32
        L.oracle_static.argtypes = [u32, P, P, P, P, P, P, P]
        L.oracle_static.restype = i32
        L.oracle_apply_batch.argtypes = [u32, P, P, P, P, u64, P, u64, P, P, P, P]
        L.oracle_apply_batch.restype = i32
        L.oracle_update.argtypes = [u32, P, P, P, P, u64, P, u64, P, P, P, P, i32, P, P, P, P, P, P, P]
        L.oracle_update.restype = i32
        L.oracle_track.argtypes = [u32, P, P, P, P]
        L.oracle_prepare.argtypes = [u32, P, P, P, P, u64, P, u64, P, P, P, P, i32, P, P, P, P, P, P, P, P]
        L.oracle_prepare.restype = i32
        L.oracle_subset_renumber.argtypes = [u32, P, P, P, P]
        L.oracle_move_class.argtypes = [u32, u32, u32]
        L.oracle_move_class.restype = u32
        L.oracle_refine_colour.argtypes = [u32, u32]
        L.oracle_refine_colour.restype = u32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def make_opts(schedule=JACOBI, tau=1e-2, tau_re=(3, 5), tol_decline=10, max_iters=20, max_passes=10,
              move_classes=4, refine_rounds=8, split_all=0):
    o = OracleOpts()
    lib().oracle_default_opts(ctypes.byref(o))
    o.tau = tau
    o.tau_re_num, o.tau_re_den = tau_re
    o.tol_decline, o.max_iters, o.max_passes = tol_decline, max_iters, max_passes
    o.schedule = schedule
    o.move_classes, o.refine_rounds = move_classes, refine_rounds
    o.split_all = split_all
    return o


@dataclass
class State:
    """Auxiliary state carried between snapshots: C, K, Sigma, DeltaSigma."""
    C: np.ndarray
    K: np.ndarray
    S: np.ndarray
    dS: np.ndarray = field(default=None)


def delta_modularity(Kic, Kid, Ki, Sc, Sd, M2) -> float:
    return lib().oracle_delta_modularity(Kic, Kid, Ki, Sc, Sd, M2)


def move_class(v: int, t: int, P: int) -> int:
    return lib().oracle_move_class(v, t, P)


def refine_colour(v: int, R: int) -> int:
    return lib().oracle_refine_colour(v, R)


def modularity(g, C) -> float:
    C = _c(C, np.uint32)
    return lib().oracle_modularity(g.n, _p(_c(g.offs, np.int64)), _p(_c(g.cols, np.uint32)),
                                   _p(_c(g.w, np.uint32)), _p(C))


def modularity64(n, offs, cols, w64, C):
    """Eq. 1 on an int64-weighted CSR; returns (q, sigma, 2m, T)."""
    sig = np.zeros(1, np.int64)
    m2 = np.zeros(1, np.int64)
    T = np.zeros(2, np.uint64)
    q = lib().oracle_modularity64(n, _p(_c(offs, np.int64)), _p(_c(cols, np.uint32)), _p(_c(w64, np.int64)),
                                  _p(_c(C, np.uint32)), _p(sig), _p(m2), _p(T))
    return q, int(sig[0]), int(m2[0]), (int(T[0]) << 64) | int(T[1])


def aggregate(n, offs, cols, w64, C, nc):
    offs, cols, w64, C = _c(offs, np.int64), _c(cols, np.uint32), _c(w64, np.int64), _c(C, np.uint32)
    nnz = lib().oracle_aggregate(n, _p(offs), _p(cols), _p(w64), _p(C), nc, None, None, None)
    o2 = np.zeros(nc + 1, np.int64)
    c2 = np.zeros(max(nnz, 1), np.uint32)
    w2 = np.zeros(max(nnz, 1), np.int64)
    lib().oracle_aggregate(n, _p(offs), _p(cols), _p(w64), _p(C), nc, _p(o2), _p(c2), _p(w2))
    return o2, c2[:nnz], w2[:nnz]


def split(g, C, split_flags, refine_flags):
    C = _c(C, np.uint32).copy()
    lib().oracle_split(g.n, _p(_c(g.offs, np.int64)), _p(_c(g.cols, np.uint32)), _p(_c(g.w, np.uint32)), _p(C),
                       _p(_c(split_flags, np.uint8)), _p(_c(refine_flags, np.uint8)))
    return C


@dataclass
class PassRecord:
    iters: int      # local-moving iterations executed
    refined: bool   # some community was refined
    n_level: int    # vertices of the pass's level graph
    moves: int      # local-moving moves
    tau: float      # the pass's iteration tolerance
    bound: np.ndarray    # communities of the input vertices by the pass's local-moving labels
    refined_labels: np.ndarray  # ... and by its refined labels


@dataclass
class Trace:
    moves: list     # (pass, iteration, vertex, from, to, dq) in order
    passes: list    # PassRecord per pass


def traced(fn, *a, n_input, **kw):
    """Run ``fn(*a, **kw)`` (static or update) while the oracle records its
    pass loop; returns (fn's result, Trace)."""
    L = lib()
    L.oracle_trace_enable(1)
    try:
        res = fn(*a, **kw)
        cnt = L.oracle_trace_moves(None, None, 0)
        rec = np.zeros(5 * max(cnt, 1), np.uint32)
        dq = np.zeros(max(cnt, 1), np.float64)
        L.oracle_trace_moves(_p(rec), _p(dq), cnt)
        moves = [tuple(int(x) for x in rec[5 * k:5 * k + 5]) + (float(dq[k]),) for k in range(cnt)]
        npass = L.oracle_trace_passes(None, None, 0)
        prec = np.zeros(4 * max(npass, 1), np.uint32)
        ptau = np.zeros(max(npass, 1), np.float64)
        L.oracle_trace_passes(_p(prec), _p(ptau), npass)
        passes = []
        for p in range(npass):
            b = np.zeros(n_input, np.uint32)
            r = np.zeros(n_input, np.uint32)
            L.oracle_trace_projection(p, 0, _p(b))
            L.oracle_trace_projection(p, 1, _p(r))
            passes.append(PassRecord(int(prec[4 * p]), bool(prec[4 * p + 1]), int(prec[4 * p + 2]),
                                     int(prec[4 * p + 3]), float(ptau[p]), b, r))
        return res, Trace(moves, passes)
    finally:
        L.oracle_trace_enable(0)


def static(g, schedule=JACOBI, **kw):
    """Static Leiden; returns (membership, modularity, stats dict)."""
    o = make_opts(schedule=schedule, **kw)
    C = np.zeros(g.n, np.uint32)
    q = ctypes.c_double(0.0)
    st = OracleStats()
    rc = lib().oracle_static(g.n, _p(_c(g.offs, np.int64)), _p(_c(g.cols, np.uint32)), _p(_c(g.w, np.uint32)),
                             ctypes.byref(o), _p(C), ctypes.byref(q), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle_static failed: %d" % rc)
    return C, q.value, st.as_dict()


def apply_batch(g, dels, ins):
    """G^{t-1} -> G^t; returns (Csr of G^t, deletions as (u, v, w_old) triples).

    Raises ValueError for an invalid batch (absent deletion, present insertion,
    self-loop, ID out of range, pair repeated)."""
    from paper_2410_15451_amd.inputs import Csr
    dels = _c(dels, np.uint32).reshape(-1, 2)
    ins = _c(ins, np.uint32).reshape(-1, 3)
    nnz = g.nnz - 2 * dels.shape[0] + 2 * ins.shape[0]
    o2 = np.zeros(g.n + 1, np.int64)
    c2 = np.zeros(max(nnz, 1), np.uint32)
    w2 = np.zeros(max(nnz, 1), np.uint32)
    dw = np.zeros(max(dels.shape[0], 1), np.uint32)
    rc = lib().oracle_apply_batch(g.n, _p(_c(g.offs, np.int64)), _p(_c(g.cols, np.uint32)),
                                  _p(_c(g.w, np.uint32)), _p(dels), dels.shape[0], _p(ins), ins.shape[0],
                                  _p(o2), _p(c2), _p(w2), _p(dw))
    if rc != 0:
        raise ValueError("invalid batch")
    dtrip = np.concatenate([dels, dw[:dels.shape[0], None]], axis=1).astype(np.uint32)
    return Csr(g.n, o2, c2[:nnz], w2[:nnz]), dtrip


def initial_state(g, C):
    """State after a static run: K = row sums, Sigma by community, DeltaSigma = 0."""
    C = _c(C, np.uint32)
    K = np.zeros(g.n, np.int64)
    np.add.at(K, np.repeat(np.arange(g.n), np.diff(g.offs)), g.w.astype(np.int64))
    S = np.zeros(g.n, np.int64)
    np.add.at(S, C, K)
    return State(C.copy(), K, S, np.zeros(g.n, np.int64))


def update(g_t, dels_w, ins, state: State, mode, schedule=JACOBI, **kw):
    """ND / DS / DF update on G^t; returns (membership, new State, modularity, stats)."""
    mode = MODES.get(mode, mode)
    o = make_opts(schedule=schedule, **kw)
    n = g_t.n
    dels_w = _c(dels_w, np.uint32).reshape(-1, 3)
    ins = _c(ins, np.uint32).reshape(-1, 3)
    C = np.zeros(n, np.uint32)
    K = np.zeros(n, np.int64)
    S = np.zeros(n, np.int64)
    dS = np.zeros(n, np.int64)
    q = ctypes.c_double(0.0)
    st = OracleStats()
    rc = lib().oracle_update(n, _p(_c(g_t.offs, np.int64)), _p(_c(g_t.cols, np.uint32)),
                             _p(_c(g_t.w, np.uint32)), _p(dels_w), dels_w.shape[0], _p(ins), ins.shape[0],
                             _p(_c(state.C, np.uint32)), _p(_c(state.K, np.int64)), _p(_c(state.S, np.int64)),
                             _p(_c(state.dS, np.int64)), int(mode), ctypes.byref(o), _p(C), _p(K), _p(S),
                             _p(dS), ctypes.byref(q), ctypes.byref(st))
    if rc != 0:
        raise ValueError("oracle_update failed: %d" % rc)
    return C, State(C.copy(), K, S, dS), q.value, st.as_dict()


def track(C_cur, C_prev, K):
    C_cur, C_prev, K = _c(C_cur, np.uint32), _c(C_prev, np.uint32), _c(K, np.int64)
    out = np.zeros(C_cur.shape[0], np.uint32)
    lib().oracle_track(C_cur.shape[0], _p(C_cur), _p(C_prev), _p(K), _p(out))
    return out


def prepare(g_t, dels_w, ins, state: State, mode, **kw):
    """Update front-end alone (Alg. 11, Alg. 5 and the marking of Alg. 1-3).

    Returns a dict with K, S (Sigma^t by C^{t-1}), dS (DeltaSigma^t after the
    refinement resets), split, refine (community flags), affected, in_range."""
    mode = MODES.get(mode, mode)
    o = make_opts(**kw)
    n = g_t.n
    dels_w = _c(dels_w, np.uint32).reshape(-1, 3)
    ins = _c(ins, np.uint32).reshape(-1, 3)
    out = {k: np.zeros(n, np.int64) for k in ("K", "S", "dS")}
    out.update({k: np.zeros(n, np.uint8) for k in ("split", "refine", "affected", "in_range")})
    rc = lib().oracle_prepare(n, _p(_c(g_t.offs, np.int64)), _p(_c(g_t.cols, np.uint32)),
                              _p(_c(g_t.w, np.uint32)), _p(dels_w), dels_w.shape[0], _p(ins), ins.shape[0],
                              _p(_c(state.C, np.uint32)), _p(_c(state.K, np.int64)), _p(_c(state.S, np.int64)),
                              _p(_c(state.dS, np.int64)), int(mode), ctypes.byref(o), _p(out["K"]), _p(out["S"]),
                              _p(out["dS"]), _p(out["split"]), _p(out["refine"]), _p(out["affected"]),
                              _p(out["in_range"]))
    if rc != 0:
        raise ValueError("oracle_prepare failed: %d" % rc)
    return out


def subset_renumber(C, S, split, refine):
    """Alg. 10 alone; returns (C, Sigma, split, refine) relabelled."""
    C, S = _c(C, np.uint32).copy(), _c(S, np.int64).copy()
    split, refine = _c(split, np.uint8).copy(), _c(refine, np.uint8).copy()
    lib().oracle_subset_renumber(C.shape[0], _p(C), _p(S), _p(split), _p(refine))
    return C, S, split, refine

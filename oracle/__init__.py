"""The oracle: plain, slow, obviously correct CPU betweenness centrality.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the GPU
library never does, and the two share no code.

Contents
  brandes.c  serial Brandes (Sec. 1.1, Theorem 1.1): BFS for unit weights,
             Dijkstra for positive integer weights; exact 128-bit path counts,
             IEEE double dependencies, BC and (optionally) edge betweenness.
             Loaded here through ctypes.
  cross.py   independent cross-oracles used to pin brandes.c:
             brute-force path enumeration from the definitions (Sec. 1.1),
             all-pairs counts + Algorithm 2 (Sec. 4.2.1), and the corrected
             dense algebraic method (Sec. 3.1, and Sec. 3.2 per weight class)
             in exact arithmetic.
  sampled.py Algorithm 1 (Sec. 4.1.1), the sampled forward, distances only:
             limited searches from a distinguished set, all-pairs distances
             on the auxiliary graph, and the final minimum.

Every pin is a ``-m "not gpu"`` test under tests/.  No function here is
"parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "brandes.c")
_LIB = os.path.join(_HERE, "_brandes.so")
_lock = threading.Lock()
_lib = None

OK, ERR_OVERFLOW, ERR_ARG, ERR_NOMEM = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile brandes.c with gcc into oracle/_brandes.so (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            try:
                lib = ctypes.CDLL(build())
            except OSError:
                # a prebuilt library for another host CPU: rebuild it here
                lib = ctypes.CDLL(build(force=True))
            i32p = ctypes.POINTER(ctypes.c_int32)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            lib.oracle_bc.argtypes = [ctypes.c_int32, i32p, i32p, u32p, i32p, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_double), i32p]
            lib.oracle_bc.restype = ctypes.c_int
            lib.oracle_edge_bc.argtypes = [ctypes.c_int32, i32p, i32p, u32p, i32p, ctypes.c_int64,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double), i32p]
            lib.oracle_edge_bc.restype = ctypes.c_int
            lib.oracle_sssp.argtypes = [ctypes.c_int32, i32p, i32p, u32p, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_uint64),
                                        ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_double)]
            lib.oracle_sssp.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct)) if a is not None else None


def _graph_arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)
    w = None if g.weight is None else np.ascontiguousarray(g.weight, dtype=np.uint32)
    if w is not None and w.size == 0:
        w = np.ones(1, np.uint32)
    return rp, col, w


class OracleError(RuntimeError):
    pass


def bc(g, sources=None, threads: int = 1, return_flags: bool = False):
    """BC(v) = sum over the given sources s != v of delta_s*(v), ordered pairs,
    no halving (Sec. 1.1).  ``sources=None`` means every vertex."""
    lib = _load()
    rp, col, w = _graph_arrays(g)
    src = np.arange(g.n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    out = np.zeros(max(g.n, 1), dtype=np.float64)
    flag = np.zeros(1, dtype=np.int32)
    src_arg = src if src.size else np.zeros(1, np.int32)
    rc = lib.oracle_bc(g.n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(w, ctypes.c_uint32),
                       _ptr(src_arg, ctypes.c_int32), int(src.size), int(threads),
                       _ptr(out, ctypes.c_double), _ptr(flag, ctypes.c_int32))
    if rc != OK:
        raise OracleError(f"oracle_bc failed with code {rc}")
    out = out[: g.n]
    return (out, bool(flag[0])) if return_flags else out


def edge_bc(g, sources=None, threads: int = 1):
    """(BC, EB): vertex betweenness as :func:`bc` and, per arc of g's CSR, the
    edge betweenness of its edge -- the sum over ordered pairs (s,t), s in the
    sources, of the fraction of shortest s-t paths through the edge.  Both arcs
    of an edge carry the same value.  Rows of g must be sorted."""
    lib = _load()
    rp, col, w = _graph_arrays(g)
    src = np.arange(g.n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    out = np.zeros(max(g.n, 1), dtype=np.float64)
    eb = np.zeros(max(col.size, 1), dtype=np.float64)
    flag = np.zeros(1, dtype=np.int32)
    src_arg = src if src.size else np.zeros(1, np.int32)
    rc = lib.oracle_edge_bc(g.n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(w, ctypes.c_uint32),
                            _ptr(src_arg, ctypes.c_int32), int(src.size), int(threads),
                            _ptr(out, ctypes.c_double), _ptr(eb, ctypes.c_double), _ptr(flag, ctypes.c_int32))
    if rc != OK:
        raise OracleError(f"oracle_edge_bc failed with code {rc}")
    return out[: g.n], eb[: int(np.asarray(g.col).size)]


def sssp(g, s: int):
    """(dist int64 with -1 = unreachable, sigma as Python-int object array,
    delta float64) for one source."""
    lib = _load()
    rp, col, w = _graph_arrays(g)
    n = max(g.n, 1)
    dist = np.zeros(n, np.int64)
    lo = np.zeros(n, np.uint64)
    hi = np.zeros(n, np.uint64)
    delta = np.zeros(n, np.float64)
    rc = lib.oracle_sssp(g.n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(w, ctypes.c_uint32),
                         int(s), _ptr(dist, ctypes.c_int64), _ptr(lo, ctypes.c_uint64),
                         _ptr(hi, ctypes.c_uint64), _ptr(delta, ctypes.c_double))
    if rc != OK:
        raise OracleError(f"oracle_sssp failed with code {rc}")
    sigma = np.array([(int(h) << 64) | int(l) for l, h in zip(lo[: g.n], hi[: g.n])], dtype=object)
    return dist[: g.n], sigma, delta[: g.n]


def sssp_u64(g, s: int):
    """As :func:`sssp` but sigma as uint64 (raises if some count exceeds 2^64-1)."""
    lib = _load()
    rp, col, w = _graph_arrays(g)
    n = max(g.n, 1)
    dist = np.zeros(n, np.int64)
    lo = np.zeros(n, np.uint64)
    hi = np.zeros(n, np.uint64)
    delta = np.zeros(n, np.float64)
    rc = lib.oracle_sssp(g.n, _ptr(rp, ctypes.c_int32), _ptr(col, ctypes.c_int32), _ptr(w, ctypes.c_uint32),
                         int(s), _ptr(dist, ctypes.c_int64), _ptr(lo, ctypes.c_uint64),
                         _ptr(hi, ctypes.c_uint64), _ptr(delta, ctypes.c_double))
    if rc != OK:
        raise OracleError(f"oracle_sssp failed with code {rc}")
    if np.any(hi[: g.n]):
        raise OracleError("path count above 2^64 - 1")
    return dist[: g.n], lo[: g.n], delta[: g.n]

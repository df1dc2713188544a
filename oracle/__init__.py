"""CPU oracle for Brandes betweenness centrality -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import this package.  It shares no code with the device path: the arithmetic lives in
``brandes.c`` (plain sequential Brandes, exact uint64 path counts with a double-precision
re-count on overflow, double-precision dependencies), and ``brute.py`` holds an
exhaustive path enumerator used to pin it on tiny graphs.

Conventions (the readings of the paper's definition in section I):
  * BC is the raw sum over ordered pairs (s, t), s != v != t, of sigma_st(v)/sigma_st --
    no normalisation, endpoints excluded, unreachable pairs contribute 0;
  * the input pair list is reduced to a simple digraph (self-loops and repeats dropped);
  * a multiset of sources gives the raw partial sum over those sources.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


class _Stats(ctypes.Structure):
    _fields_ = [("reached", ctypes.c_int64), ("examined", ctypes.c_int64),
                ("dag_edges", ctypes.c_int64), ("levels", ctypes.c_int64)]


def _load():
    global _lib
    if _lib is None:
        use_native(False)
    return _lib


def use_native(native: bool) -> str:
    """Load the generic build, or the host-tuned one (-O3 -march=native, compiled here and now);
    returns the path of the library loaded."""
    global _lib
    path = _build.build_native() if native else _build.build(force=False)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_simple_adjacency.restype = ctypes.c_int64
    lib.oracle_simple_adjacency.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P]
    lib.oracle_brandes_source.restype = ctypes.c_int
    lib.oracle_brandes_source.argtypes = [ctypes.c_int32, P, P, ctypes.c_uint32, P, P, P, P, P, P,
                                          ctypes.POINTER(_Stats)]
    lib.oracle_bc.restype = ctypes.c_int
    lib.oracle_bc.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int64, P, P, P, ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return path


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def simple_adjacency(n, src, dst):
    """Adjacency (row_ptr uint32[n+1], col uint32[m]) of the simple digraph given by the pairs."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    row_ptr = np.zeros(n + 1, dtype=np.uint32)
    col = np.zeros(max(len(src), 1), dtype=np.uint32)
    m = lib.oracle_simple_adjacency(int(n), len(src), _ptr(src), _ptr(dst), _ptr(row_ptr), _ptr(col))
    if m < 0:
        raise ValueError("vertex id out of range" if m == -1 else "allocation failed")
    return row_ptr, col[:m].copy()


class Graph:
    """Simple digraph held as adjacency arrays (oracle side)."""

    def __init__(self, n, src, dst):
        self.n = int(n)
        self.row_ptr, self.col = simple_adjacency(n, src, dst)
        self.m = int(self.col.shape[0])


def brandes_source(g: Graph, s: int):
    """dist, sigma (uint64; valid iff not overflowed), sigma_f (float64), delta, overflow, stats."""
    lib = _load()
    n = g.n
    dist = np.empty(n, dtype=np.int32)
    sigma = np.empty(n, dtype=np.uint64)
    sigma_f = np.empty(n, dtype=np.float64)
    delta = np.empty(n, dtype=np.float64)
    order = np.empty(n, dtype=np.uint32)
    ovf = np.zeros(1, dtype=np.int32)
    st = _Stats()
    rc = lib.oracle_brandes_source(n, _ptr(g.row_ptr), _ptr(g.col), int(s), _ptr(dist), _ptr(sigma),
                                   _ptr(sigma_f), _ptr(delta), _ptr(order), _ptr(ovf), ctypes.byref(st))
    if rc != 0:
        raise ValueError("source out of range")
    return dict(dist=dist, sigma=sigma, sigma_f=sigma_f, delta=delta, overflow=bool(ovf[0]),
                reached=st.reached, examined=st.examined, dag_edges=st.dag_edges, levels=st.levels)


def bc(g: Graph, sources=None, threads: int | None = None):
    """(bc float64[n], overflowed uint8[k], stats int64[k,4]) over a multiset of sources.

    ``sources=None`` means every vertex once (exact BC).  stats columns: reached vertices,
    examined edges, shortest-path DAG edges, BFS levels.
    """
    lib = _load()
    if sources is None:
        sources = np.arange(g.n, dtype=np.uint32)
    sources = np.ascontiguousarray(sources, dtype=np.uint32)
    k = int(sources.shape[0])
    out = np.zeros(g.n, dtype=np.float64)
    ovf = np.zeros(max(k, 1), dtype=np.uint8)
    stats = np.zeros((max(k, 1), 4), dtype=np.int64)
    if threads is None:
        threads = max_threads()
    rc = lib.oracle_bc(g.n, _ptr(g.row_ptr), _ptr(g.col), _ptr(sources), k, _ptr(out), _ptr(ovf),
                       _ptr(stats), int(threads))
    if rc != 0:
        raise ValueError("source out of range" if rc == -1 else "allocation failed")
    return out, ovf[:k].copy(), stats[:k].copy()


"""Thin Python binding of libbcmi.so (the C ABI in include/bc.h).

Argument marshalling only: torch CUDA tensors provide device memory and streams, and every
step of the computation runs in the library's HIP kernels.  Loading fails loudly when the
built library is missing; there is no fallback implementation.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbcmi.so")

BC_OK, BC_PENDING = 0, 1
BC_E_INVAL, BC_E_RANGE, BC_E_NOMEM, BC_E_HIP, BC_E_STATE = -1, -2, -3, -4, -5
_NAMES = {BC_E_INVAL: "BC_E_INVAL", BC_E_RANGE: "BC_E_RANGE", BC_E_NOMEM: "BC_E_NOMEM",
          BC_E_HIP: "BC_E_HIP", BC_E_STATE: "BC_E_STATE"}


class BcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class bc_tuning(ctypes.Structure):
    _fields_ = [("wg_size", ctypes.c_int32), ("wgs_per_source", ctypes.c_int32),
                ("sources_per_launch", ctypes.c_int32), ("hub_threshold", ctypes.c_int32),
                ("lds_max_n", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("batched", ctypes.c_int32),
                ("batch_wg_size", ctypes.c_int32), ("batch_pull", ctypes.c_int32),
                ("deterministic", ctypes.c_int32)]


class bc_info(ctypes.Structure):
    _fields_ = [("n_sources", ctypes.c_uint32), ("n_sigma_fp64_fallback", ctypes.c_uint32),
                ("levels_max", ctypes.c_uint32), ("path", ctypes.c_uint32), ("kernel_ms", ctypes.c_double),
                ("t_submit_ms", ctypes.c_double), ("t_start_ms", ctypes.c_double),
                ("t_done_ms", ctypes.c_double), ("reached", ctypes.c_uint64), ("examined", ctypes.c_uint64),
                ("dag_edges", ctypes.c_uint64), ("batch_entries", ctypes.c_uint64),
                ("batch_edge_visits", ctypes.c_uint64), ("batch_scans", ctypes.c_uint64),
                ("batch_handoffs", ctypes.c_uint64),
                ("batch_cycles", ctypes.c_uint64 * 3), ("batch_pull_edges", ctypes.c_uint64),
                ("batch_pull_levels", ctypes.c_uint64), ("batch_pull_skipped", ctypes.c_uint64),
                ("batch_pull_pairs", ctypes.c_uint64)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_}
        out["batch_cycles"] = list(self.batch_cycles)
        return out


_lib = None
P = ctypes.c_void_p


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        L.bc_build_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, ctypes.POINTER(P)]
        L.bc_graph_info.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
        L.bc_graph_arrays.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P)]
        L.bc_graph_order.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P)]
        L.bc_graph_free.argtypes = [P]
        L.bc_exact.argtypes = [P, P, ctypes.POINTER(bc_tuning), P, ctypes.POINTER(bc_info)]
        L.bc_sampled.argtypes = [P, P, ctypes.c_int32, P, ctypes.POINTER(bc_tuning), P, ctypes.POINTER(bc_info)]
        L.bc_sampled_flags.argtypes = [P, P, ctypes.c_int32, P, P, ctypes.POINTER(bc_tuning), P,
                                       ctypes.POINTER(bc_info)]
        L.bc_sssp.argtypes = [P, ctypes.c_uint32, P, P, P, P, ctypes.POINTER(ctypes.c_int32), P]
        L.bc_batch.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(bc_tuning), P,
                               ctypes.POINTER(bc_info)]
        L.bc_tune.argtypes = [P, ctypes.POINTER(bc_tuning)]
        L.bc_paper_strategy.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, P, P,
                                        ctypes.POINTER(bc_info)]
        L.bc_approx.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, P,
                                ctypes.POINTER(ctypes.c_int32), P, ctypes.c_int32, P, ctypes.POINTER(bc_info)]
        L.bc_approx_vertex.argtypes = [P, ctypes.c_uint32, ctypes.c_double, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32), P,
                                       ctypes.c_int32, P]
        L.bc_sampled_noalloc.argtypes = [P, P, ctypes.c_int32, P, ctypes.POINTER(bc_tuning), P]
        L.bc_stream_probe.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]
        L.bc_serve_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(P)]
        L.bc_serve_submit.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_uint64)]
        L.bc_serve_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(bc_info)]
        L.bc_serve_destroy.argtypes = [P]
        for name in ["bc_build_csr", "bc_graph_info", "bc_graph_arrays", "bc_graph_order", "bc_graph_free", "bc_exact",
                     "bc_sampled", "bc_sampled_flags",
                     "bc_sssp", "bc_batch", "bc_tune", "bc_paper_strategy", "bc_approx", "bc_approx_vertex",
                     "bc_serve_create", "bc_serve_submit", "bc_serve_poll", "bc_serve_destroy", "bc_stream_probe", "bc_sampled_noalloc"]:
            getattr(L, name).restype = ctypes.c_int32
        L.bc_last_error.restype = ctypes.c_char_p
        L.bc_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc, allow=(BC_OK,)):
    if rc not in allow:
        raise BcError(rc, lib().bc_last_error().decode())
    return rc


def _stream(stream):
    if stream is None:
        return P(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return P(stream.cuda_stream)
    return P(int(stream))


def _dev_u32(x, device="cuda"):
    """Device tensor whose storage holds uint32 ids (int32 dtype, same bits)."""
    if not torch.is_tensor(x):
        import numpy as np
        x = torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.uint32)).view(np.int32))
    if x.dtype in (torch.int64, torch.uint8, torch.int16):
        x = x.to(torch.int32)
    assert x.dtype in (torch.int32, torch.uint32), x.dtype
    return x.to(device).contiguous()


def tuning(**kw):
    t = bc_tuning()
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


# Handles still alive at interpreter exit are released by an exit hook, which runs before the C
# runtime's own exit handlers (a profiler's among them): the library then makes no HIP call
# once those have torn down.
_live_graphs = weakref.WeakSet()
_live_servers = weakref.WeakSet()


def _release_all():
    for s in list(_live_servers):
        try:
            s.destroy()
        except Exception:
            pass
    for g in list(_live_graphs):
        try:
            g.free()
        except Exception:
            pass


atexit.register(_release_all)


class Graph:
    """Owning wrapper of a bc_graph handle."""

    def __init__(self, handle, n, m):
        self.handle = handle
        self.n = n
        self.m = m
        _live_graphs.add(self)

    def free(self):
        if self.handle:
            _check(lib().bc_graph_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def arrays(self):
        """(row_ptr, col, csc_ptr, csc_row) copied into int64 CPU tensors."""
        ptrs = [P() for _ in range(4)]
        _check(lib().bc_graph_arrays(self.handle, *[ctypes.byref(p) for p in ptrs]))
        sizes = [self.n + 1, self.m, self.n + 1, self.m]
        out = []
        for p, sz in zip(ptrs, sizes):
            t = torch.empty(sz, dtype=torch.int32, device="cuda")
            if sz:
                torch.cuda.synchronize()
                _copy_device(t.data_ptr(), p.value, 4 * sz)
            out.append(t.cpu().to(torch.int64) & 0xFFFFFFFF)
        return tuple(out)


    def order(self):
        """(order, rank) of the batching order as int64 CPU tensors, or None without edges."""
        po, pr = P(), P()
        _check(lib().bc_graph_order(self.handle, ctypes.byref(po), ctypes.byref(pr)))
        if not po.value:
            return None
        out = []
        for p in (po, pr):
            t = torch.empty(self.n, dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            _copy_device(t.data_ptr(), p.value, 4 * self.n)
            out.append(t.cpu().to(torch.int64) & 0xFFFFFFFF)
        return tuple(out)


def _copy_device(dst, src, nbytes):
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [P, P, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(P(dst), P(src), nbytes, 3)   # device to device
    if rc != 0:
        raise BcError(BC_E_HIP, f"hipMemcpy failed ({rc})")


def bc_build_csr(n, src, dst, stream=None) -> Graph:
    src = _dev_u32(src)
    dst = _dev_u32(dst)
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    h = P()
    _check(lib().bc_build_csr(int(n), src.numel(), P(src.data_ptr()), P(dst.data_ptr()), _stream(stream),
                              ctypes.byref(h)))
    nn, mm = ctypes.c_int32(), ctypes.c_int64()
    _check(lib().bc_graph_info(h, ctypes.byref(nn), ctypes.byref(mm)))
    return Graph(h, nn.value, mm.value)


def _out(g, out):
    if out is None:
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    assert out.dtype == torch.float64 and out.numel() >= g.n and out.is_contiguous()
    return out


def bc_exact(g: Graph, out=None, tuning=None, stream=None, info=False):
    out = _out(g, out)
    inf = bc_info() if info else None
    _check(lib().bc_exact(g.handle, P(out.data_ptr()), ctypes.byref(tuning) if tuning else None, _stream(stream),
                          ctypes.byref(inf) if inf is not None else None))
    return (out, inf.as_dict()) if info else out


def bc_sampled(g: Graph, sources, out=None, tuning=None, stream=None, info=False):
    out = _out(g, out)
    srcs = _dev_u32(sources)
    inf = bc_info() if info else None
    _check(lib().bc_sampled(g.handle, P(srcs.data_ptr()) if srcs.numel() else None, srcs.numel(),
                            P(out.data_ptr()), ctypes.byref(tuning) if tuning else None, _stream(stream),
                            ctypes.byref(inf) if inf is not None else None))
    if not info:
        # keep the source tensor alive until the stream has consumed it
        _check_keepalive(srcs, stream)
    return (out, inf.as_dict()) if info else out


def bc_sampled_flags(g: Graph, sources=None, out=None, flags=None, tuning=None, stream=None, info=False):
    """BC over `sources` (None: every vertex, exact) plus the per-source overflow flags: a uint8
    tensor of n entries, 1 at every source whose path counts exceeded 2^64 - 1."""
    out = _out(g, out)
    if flags is None:
        flags = torch.empty(g.n, dtype=torch.uint8, device="cuda")
    assert flags.dtype == torch.uint8 and flags.numel() >= g.n and flags.is_contiguous()
    srcs = _dev_u32(sources) if sources is not None else None
    k = srcs.numel() if srcs is not None else -1
    inf = bc_info() if info else None
    _check(lib().bc_sampled_flags(g.handle, P(srcs.data_ptr()) if srcs is not None and srcs.numel() else None, k,
                                  P(out.data_ptr()), P(flags.data_ptr()), ctypes.byref(tuning) if tuning else None,
                                  _stream(stream), ctypes.byref(inf) if inf is not None else None))
    if not info and srcs is not None:
        _check_keepalive(srcs, stream)
    return (out, flags, inf.as_dict()) if info else (out, flags)


def bc_sampled_noalloc(g: Graph, sources, out, tuning=None, stream=None):
    """bc_sampled through the entry point that allocates no device memory (its state lives in
    the library's fixed per-device array); `out` must be given."""
    srcs = _dev_u32(sources)
    assert out.dtype == torch.float64 and out.numel() >= g.n and out.is_contiguous()
    _check(lib().bc_sampled_noalloc(g.handle, P(srcs.data_ptr()) if srcs.numel() else None, srcs.numel(),
                                    P(out.data_ptr()), ctypes.byref(tuning) if tuning else None, _stream(stream)))
    _check_keepalive(srcs, stream)
    return out


def bc_paper_strategy(g: Graph, strategy: int, wg_size: int = 256, sources=None, out=None, stream=None,
                      info=False):
    """One of the paper's three GPU strategies (1 vertex-parallel, 2 edge-parallel, 3 host-
    synchronised levels) as a baseline: same BC as bc_exact (sources None) or bc_sampled."""
    out = _out(g, out)
    srcs = _dev_u32(sources) if sources is not None else None
    inf = bc_info() if info else None
    _check(lib().bc_paper_strategy(g.handle, int(strategy), int(wg_size),
                                   P(srcs.data_ptr()) if srcs is not None and srcs.numel() else None,
                                   srcs.numel() if srcs is not None else -1, P(out.data_ptr()), _stream(stream),
                                   ctypes.byref(inf) if inf is not None else None))
    return (out, inf.as_dict()) if info else out


def bc_approx(g: Graph, eps: float, delta: float, seed: int, out=None, stream=None, info=False):
    """Pivot-sampled BC scaled by n/k, k from a Hoeffding bound (exact BC when k >= n).
    Returns (estimate, pivots as a numpy array[, info])."""
    import numpy as np
    out = _out(g, out)
    cap = g.n
    piv = np.zeros(max(cap, 1), dtype=np.uint32)
    k = ctypes.c_int32(0)
    inf = bc_info() if info else None
    _check(lib().bc_approx(g.handle, float(eps), float(delta), int(seed), P(out.data_ptr()), ctypes.byref(k),
                           piv.ctypes.data_as(P), cap, _stream(stream),
                           ctypes.byref(inf) if inf is not None else None))
    piv = piv[:k.value].copy()
    return (out, piv, inf.as_dict()) if info else (out, piv)


def bc_approx_vertex(g: Graph, v: int, c: float, seed: int, max_samples: int, stream=None):
    """Adaptive sampling for one vertex: (estimate, pivots used)."""
    import numpy as np
    piv = np.zeros(max(int(max_samples), 1), dtype=np.uint32)
    est = ctypes.c_double(0.0)
    k = ctypes.c_int32(0)
    _check(lib().bc_approx_vertex(g.handle, int(v), float(c), int(seed), int(max_samples), ctypes.byref(est),
                                  ctypes.byref(k), piv.ctypes.data_as(P), int(max_samples), _stream(stream)))
    return est.value, piv[:k.value].copy()


_keep = []


def _check_keepalive(t, stream):
    ev = torch.cuda.Event()
    ev.record(torch.cuda.current_stream() if stream is None else stream)
    _keep.append((ev, t))
    while _keep and _keep[0][0].query():
        _keep.pop(0)


def bc_sssp(g: Graph, s: int, stream=None):
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    sig = torch.empty(g.n, dtype=torch.int64, device="cuda")
    sigf = torch.empty(g.n, dtype=torch.float64, device="cuda")
    delta = torch.empty(g.n, dtype=torch.float64, device="cuda")
    ovf = ctypes.c_int32(0)
    _check(lib().bc_sssp(g.handle, int(s), P(dist.data_ptr()), P(sig.data_ptr()), P(sigf.data_ptr()),
                         P(delta.data_ptr()), ctypes.byref(ovf), _stream(stream)))
    return dict(dist=dist, sigma_u64=sig, sigma_f64=sigf, delta=delta, overflow=bool(ovf.value))


def bc_batch(graphs, outs=None, tuning=None, stream=None, info=False):
    if outs is None:
        outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for g in graphs]
    num = len(graphs)
    hs = (P * max(num, 1))(*[g.handle for g in graphs])
    os_ = (P * max(num, 1))(*[P(o.data_ptr()) for o in outs])
    infos = (bc_info * max(num, 1))() if info else None
    _check(lib().bc_batch(hs, num, os_, ctypes.byref(tuning) if tuning else None, _stream(stream), infos))
    if info:
        return outs, [infos[i].as_dict() for i in range(num)]
    return outs


def bc_tune(g: Graph) -> dict:
    t = bc_tuning()
    _check(lib().bc_tune(g.handle, ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in bc_tuning._fields_}


@dataclass(eq=False)
class Server:
    handle: object

    def destroy(self):
        if self.handle:
            _check(lib().bc_serve_destroy(self.handle))
            self.handle = None


def bc_serve_create(hbm_budget_bytes: int, max_slots: int = 0) -> Server:
    h = P()
    _check(lib().bc_serve_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)))
    s = Server(h)
    _live_servers.add(s)
    return s


def bc_serve_submit(server: Server, g: Graph, sources, out) -> int:
    import numpy as np
    tk = ctypes.c_uint64()
    if sources is None:
        _check(lib().bc_serve_submit(server.handle, g.handle, None, 0, P(out.data_ptr()), ctypes.byref(tk)))
    else:
        arr = np.ascontiguousarray(np.asarray(sources, dtype=np.uint32))
        _check(lib().bc_serve_submit(server.handle, g.handle, arr.ctypes.data_as(P), arr.shape[0],
                                     P(out.data_ptr()), ctypes.byref(tk)))
    return tk.value


def bc_serve_poll(server: Server, ticket: int):
    """None while pending, else the info dict."""
    inf = bc_info()
    rc = _check(lib().bc_serve_poll(server.handle, int(ticket), ctypes.byref(inf)), allow=(BC_OK, BC_PENDING))
    return None if rc == BC_PENDING else inf.as_dict()


def bc_serve_destroy(server: Server):
    server.destroy()


def bc_stream_probe(nbytes: int, reps: int = 5):
    """(copy GB/s, triad GB/s) of STREAM-style kernels over arrays of `nbytes` each."""
    c, t = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().bc_stream_probe(int(nbytes), int(reps), ctypes.byref(c), ctypes.byref(t)))
    return c.value, t.value


def version() -> str:
    return lib().bc_version().decode()

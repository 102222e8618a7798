"""Thin ctypes binding of libqg (C ABI in include/qg.h).

Argument marshalling only: every step of the search runs in the HIP kernels of
libqg.so.  torch tensors provide device memory and streams.  The library must
be built (``python -m paper_2411_12229_amd.build``); importing this module
without it raises immediately -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqg.so")

QG_OK, QG_EINVAL, QG_ENOMEM, QG_EIO, QG_EFORMAT, QG_EDEVICE, QG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
QG_SEARCH_NO_ME = 1
QG_SEARCH_SMALL_HASH = 2
QG_SEARCH_LDS_BEAM = 4
QG_GRAPH_REFINE = 1
QG_GRAPH_REPAIR = 2
QG_GRAPH_PROGRESS = 4
QG_NOALLOC_SCRATCH_BYTES = 16 << 20
QG_MAX_EF = 2048
QG_MAX_K = 1024
QG_STOP_MLP_PARAMS = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1

EXPORTS = ("qg_load_index", "qg_build_index", "qg_save_index", "qg_search", "qg_search_ex", "qg_search_stop",
           "qg_rotate",
           "qg_estimate", "qg_copy_blocks", "qg_set_stream", "qg_index_info", "qg_timing", "qg_timing_read",
           "qg_free_index", "qg_last_error")


class StopParams(ctypes.Structure):
    _fields_ = [("mlp", ctypes.c_void_p), ("theta", ctypes.c_float), ("t_min", ctypes.c_int32),
                ("t_every", ctypes.c_int32), ("trace_max", ctypes.c_int32), ("trace_features", ctypes.c_void_p),
                ("trace_nn", ctypes.c_void_p), ("trace_out", ctypes.c_void_p), ("trace_count", ctypes.c_void_p)]


class QGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqg error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_12229_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "qg_load_index": ([ctypes.c_char_p, c_int, PP], c_int),
        "qg_build_index": ([P, i64, i32, P, i32, P, i32, c_int, PP], c_int),
        "qg_build_graph": ([P, i64, i32, i32, i32, i32, P, i32, P, P, i32, c_int, P, ctypes.POINTER(i64)], c_int),
        "qg_save_index": ([P, ctypes.c_char_p], c_int),
        "qg_search": ([P, P, i64, i32, i32, P, P], c_int),
        "qg_search_ex": ([P, P, i64, i32, i32, i32, P, P, P], c_int),
        "qg_search_noalloc": ([P, P, i64, i32, i32, i32, P, P, P], c_int),
        "qg_search_stop": ([P, P, i64, i32, i32, i32, ctypes.POINTER(StopParams), P, P, P], c_int),
        "qg_search_mixed": ([P, P, i64, P, P, i32, i32, i32, P, P, P], c_int),
        "qg_search_mixed_stop": ([P, P, i64, P, P, i32, i32, i32, ctypes.POINTER(StopParams), P, P, P], c_int),
        "qg_rotate": ([P, P, i64, P], c_int),
        "qg_estimate": ([P, P, P, i64, P, P, P], c_int),
        "qg_copy_blocks": ([P, i64, i64, P], c_int),
        "qg_set_stream": ([P, P], c_int),
        "qg_reserve": ([P, i64], c_int),
        "qg_set_launch": ([P, i32, i32, i32, i32, i32], c_int),
        "qg_autotune": ([P, P, i64, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                         ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], c_int),
        "qg_autotune_mixed": ([P, P, i64, P, P, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                               ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                               ctypes.POINTER(ctypes.c_double)], c_int),
        "qg_index_info": ([P, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                           ctypes.POINTER(i64)], c_int),
        "qg_timing": ([P, c_int], c_int),
        "qg_timing_read": ([P, c_int, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], c_int),
        "qg_free_index": ([P], None),
        "qg_server_create": ([P, i32, i32, i32, i32, PP], c_int),
        "qg_server_submit": ([P, P, i32, i32, ctypes.c_uint64], c_int),
        "qg_server_poll": ([P, i64, P, P, P, P, P], i64),
        "qg_server_batches": ([P, i64, i64, P], i64),
        "qg_server_replay": ([P, P, P, P, P, i64], c_int),
        "qg_server_set_recall_map": ([P, P, P, P, i32], c_int),
        "qg_server_submit_target": ([P, P, i32, ctypes.c_float, ctypes.c_uint64], c_int),
        "qg_server_replay_target": ([P, P, P, P, P, i64], c_int),
        "qg_server_set_stop": ([P, ctypes.POINTER(StopParams)], c_int),
        "qg_server_drain": ([P, ctypes.c_double], c_int),
        "qg_server_stats": ([P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
                            c_int),
        "qg_server_destroy": ([P], None),
        "qg_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    return L


_lib = _load()


def lib():
    return _lib


def qg_last_error() -> str:
    return _lib.qg_last_error().decode()


def _check(rc: int):
    if rc != QG_OK:
        raise QGError(rc, qg_last_error())


def _dev(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Index:
    """Owner of a libqg index handle."""

    def __init__(self, handle: ctypes.c_void_p, device: int):
        self._h = handle
        self.device = device
        n, d, r, e, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(_lib.qg_index_info(self._h, ctypes.byref(n), ctypes.byref(d), ctypes.byref(r), ctypes.byref(e),
                                  ctypes.byref(b)))
        self.n, self.d, self.r, self.entry, self.block_bytes = n.value, d.value, r.value, e.value, b.value
        self._stream = None

    @property
    def handle(self):
        return self._h

    def set_stream(self, stream) -> None:
        """Run later work on a torch.cuda.Stream (None = null stream)."""
        self._stream = stream
        _check(_lib.qg_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream if stream is not None else 0)))

    def autotune(self, queries: torch.Tensor, k: int, ef: int, flags: int = 0):
        """Pick the launch shape (wavefronts per workgroup, visited-hash factor, cap on resident
        wavefronts per compute unit, beam storage, LUT layout) by timing searches of these queries; returns
        (wpb, hash_factor, cu_waves (0 = no cap), best ms per call, beam (1 = registers, 0 = LDS),
        lut (bit 0: padded rows, bit 1: int32 entries))."""
        w, h, c, b, lu = (ctypes.c_int32() for _ in range(5))
        ms = ctypes.c_double()
        _check(_lib.qg_autotune(self._h, _dev(queries, torch.float32, "queries"), queries.shape[0], k, ef, flags,
                                ctypes.byref(w), ctypes.byref(h), ctypes.byref(c), ctypes.byref(b), ctypes.byref(lu),
                                ctypes.byref(ms)))
        return w.value, h.value, c.value, ms.value, b.value, lu.value

    def autotune_mixed(self, queries: torch.Tensor, k: torch.Tensor, ef: torch.Tensor, k_max: int, ef_max: int,
                       flags: int = 0):
        """autotune for mixed batches (per-query k and ef, int32 device tensors [nq]); same return values."""
        nq = queries.shape[0]
        if k.shape != (nq,) or ef.shape != (nq,):
            raise ValueError("shape mismatch")
        w, h, c, b, lu = (ctypes.c_int32() for _ in range(5))
        ms = ctypes.c_double()
        _check(_lib.qg_autotune_mixed(self._h, _dev(queries, torch.float32, "queries"), nq,
                                      _dev(k, torch.int32, "k_per_query"), _dev(ef, torch.int32, "ef_per_query"),
                                      int(k_max), int(ef_max), flags, ctypes.byref(w), ctypes.byref(h),
                                      ctypes.byref(c), ctypes.byref(b), ctypes.byref(lu), ctypes.byref(ms)))
        return w.value, h.value, c.value, ms.value, b.value, lu.value

    def set_launch(self, wpb: int, hash_factor: int, cu_waves: int = 0, beam: int = 1, lut: int = 1) -> None:
        """Set the launch shape directly (the values qg_autotune picks)."""
        _check(_lib.qg_set_launch(self._h, int(wpb), int(hash_factor), int(cu_waves), int(beam), int(lut)))

    def reserve(self, nq: int) -> None:
        """Size the query scratch for batches of up to nq queries (before capturing graphs)."""
        _check(_lib.qg_reserve(self._h, int(nq)))

    def search_mixed(self, queries: torch.Tensor, k: torch.Tensor, ef: torch.Tensor, k_max: int | None = None,
                     ef_max: int | None = None, flags: int = 0, stats: bool = False):
        """Algorithm 1 with a k and ef per query (int32 device tensors [nq]) in one launch ->
        (ids [nq,k_max], dists [nq,k_max][, stats [nq,4]]); row q is its k_q results, then padding.
        The bounds default to the tensors' maxima (one device-to-host read)."""
        nq = queries.shape[0]
        dev = queries.device
        if k_max is None:
            k_max = int(k.max().item()) if nq else 1
        if ef_max is None:
            ef_max = int(ef.max().item()) if nq else 1
        ids = torch.empty((nq, k_max), dtype=torch.int32, device=dev)
        dists = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
        st = torch.empty((nq, 4), dtype=torch.int32, device=dev) if stats else None
        qg_search_mixed(self, queries, nq, k, ef, k_max, ef_max, flags, ids, dists, st)
        return (ids, dists, st) if stats else (ids, dists)

    def search_mixed_stop(self, queries: torch.Tensor, k: torch.Tensor, ef: torch.Tensor, mlp: torch.Tensor,
                          theta: float, t_min: int = 8, t_every: int = 4, k_max: int | None = None,
                          ef_max: int | None = None, flags: int = 0, stats: bool = False):
        """search_mixed with the learned stop (shared model, theta, t_min, t_every; no trace)."""
        nq = queries.shape[0]
        dev = queries.device
        if k_max is None:
            k_max = int(k.max().item()) if nq else 1
        if ef_max is None:
            ef_max = int(ef.max().item()) if nq else 1
        if queries.shape != (nq, self.d) or k.shape != (nq,) or ef.shape != (nq,):
            raise ValueError("shape mismatch")
        ids = torch.empty((nq, k_max), dtype=torch.int32, device=dev)
        dists = torch.empty((nq, k_max), dtype=torch.float32, device=dev)
        st = torch.empty((nq, 4), dtype=torch.int32, device=dev) if stats else None
        sp = _stop_params(mlp, theta, t_min, t_every)
        _check(_lib.qg_search_mixed_stop(self._h, _dev(queries, torch.float32, "queries"), nq,
                                         _dev(k, torch.int32, "k_per_query"), _dev(ef, torch.int32, "ef_per_query"),
                                         k_max, ef_max, flags, ctypes.byref(sp), _dev(ids, torch.int32, "out_ids"),
                                         _dev(dists, torch.float32, "out_dists"),
                                         _dev(st, torch.int32, "out_stats") if stats else None))
        return (ids, dists, st) if stats else (ids, dists)

    def search(self, queries: torch.Tensor, k: int, ef: int, flags: int = 0, stats: bool = False):
        """Algorithm 1 for every row of `queries` -> (ids int32 [nq,k], dists f32 [nq,k][, stats int32 [nq,4]])."""
        nq = queries.shape[0]
        dev = queries.device
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
        st = torch.empty((nq, 4), dtype=torch.int32, device=dev) if stats else None
        qg_search_ex(self, queries, nq, k, ef, flags, ids, dists, st)
        return (ids, dists, st) if stats else (ids, dists)

    def search_stop(self, queries: torch.Tensor, k: int, ef: int, mlp: torch.Tensor | None, theta: float = 0.0,
                    t_min: int = 8, t_every: int = 4, trace_max: int = 0, flags: int = 0, stats: bool = False):
        """Search with the learned stop (mlp: uint16/int16 bf16 bits on the device, or None for
        trace only).  Returns (ids, dists, stats or None, trace or None); trace =
        (features [nq,T,16], nn [nq,T,k], out [nq,T], count [nq])."""
        nq = queries.shape[0]
        dev = queries.device
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        dists = torch.empty((nq, k), dtype=torch.float32, device=dev)
        st = torch.empty((nq, 4), dtype=torch.int32, device=dev) if stats else None
        tr = None
        if trace_max > 0:
            tr = (torch.zeros((nq, trace_max, 16), dtype=torch.float32, device=dev),
                  torch.zeros((nq, trace_max, k), dtype=torch.int32, device=dev),
                  torch.zeros((nq, trace_max), dtype=torch.float32, device=dev),
                  torch.zeros((nq,), dtype=torch.int32, device=dev))
        qg_search_stop(self, queries, nq, k, ef, flags, mlp, theta, t_min, t_every, trace_max, tr, ids, dists, st)
        return ids, dists, st, tr

    def rotate(self, x: torch.Tensor) -> torch.Tensor:
        out = torch.empty_like(x)
        qg_rotate(self, x, x.shape[0], out)
        return out

    def estimate(self, queries: torch.Tensor, vertices: torch.Tensor):
        nq = queries.shape[0]
        S = torch.empty((nq, self.r), dtype=torch.int32, device=queries.device)
        est = torch.empty((nq, self.r), dtype=torch.float32, device=queries.device)
        dist = torch.empty((nq,), dtype=torch.float32, device=queries.device)
        qg_estimate(self, queries, vertices, nq, S, est, dist)
        return S, est, dist

    def blocks(self, first: int = 0, count: int | None = None) -> torch.Tensor:
        count = self.n - first if count is None else count
        out = torch.empty((count, self.block_bytes), dtype=torch.uint8, device=f"cuda:{self.device}")
        qg_copy_blocks(self, first, count, out)
        return out

    def save(self, path: str) -> None:
        qg_save_index(self, path)

    def timing(self, enable: bool) -> None:
        _check(_lib.qg_timing(self._h, 1 if enable else 0))

    def timing_read(self, kernel: int):
        n, ms = ctypes.c_int32(), ctypes.c_double()
        _check(_lib.qg_timing_read(self._h, kernel, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def free(self) -> None:
        if self._h:
            _lib.qg_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------- C ABI names, tensor arguments

def qg_load_index(path: str, device: int = 0) -> Index:
    h = ctypes.c_void_p()
    _check(_lib.qg_load_index(path.encode(), device, ctypes.byref(h)))
    return Index(h, device)


def qg_build_graph(vectors: torch.Tensor, r: int, ef_build: int, iters: int, rotation: torch.Tensor, entry: int,
                   init_graph: torch.Tensor, fill: torch.Tensor | None, refine: bool = True, repair: bool = True,
                   progress: bool = False):
    """Algorithm 2 on the vectors' device -> (graph int32 [n, r] on the device, stats dict)."""
    n, d = vectors.shape
    out = torch.empty((n, r), dtype=torch.int32, device=vectors.device)
    st = (ctypes.c_int64 * 4)()
    flags = (QG_GRAPH_REFINE if refine else 0) | (QG_GRAPH_REPAIR if repair else 0) | \
        (QG_GRAPH_PROGRESS if progress else 0)
    _check(_lib.qg_build_graph(_dev(vectors, torch.float32, "vectors"), n, d, r, ef_build, iters,
                               _dev(rotation, torch.float32, "rotation"), int(entry),
                               _dev(init_graph, torch.int32, "init_graph"),
                               _dev(fill, torch.int32, "fill") if fill is not None else None, flags,
                               vectors.device.index or 0, _dev(out, torch.int32, "out_graph"), st))
    return out, dict(zip(("reach_before_repair", "repairs", "reach_after_repair", "microseconds"), list(st)))


def qg_build_index(vectors: torch.Tensor, graph: torch.Tensor, rotation: torch.Tensor, entry: int) -> Index:
    n, d = vectors.shape
    r = graph.shape[1]
    if graph.shape[0] != n or tuple(rotation.shape) != (d, d):
        raise ValueError("shape mismatch between vectors, graph and rotation")
    h = ctypes.c_void_p()
    dev = vectors.device.index or 0
    _check(_lib.qg_build_index(_dev(vectors, torch.float32, "vectors"), n, d, _dev(graph, torch.int32, "graph"), r,
                               _dev(rotation, torch.float32, "rotation"), int(entry), dev, ctypes.byref(h)))
    return Index(h, dev)


def qg_save_index(idx: Index, path: str) -> None:
    _check(_lib.qg_save_index(idx.handle, path.encode()))


def qg_search_ex(idx: Index, queries, nq: int, k: int, ef: int, flags: int, out_ids, out_dists, out_stats=None):
    if queries.shape != (nq, idx.d) or out_ids.shape != (nq, k) or out_dists.shape != (nq, k):
        raise ValueError("shape mismatch")
    if out_stats is not None and out_stats.shape != (nq, 4):
        raise ValueError("stats shape mismatch")
    st = _dev(out_stats, torch.int32, "out_stats") if out_stats is not None else None
    _check(_lib.qg_search_ex(idx.handle, _dev(queries, torch.float32, "queries"), nq, k, ef, flags,
                             _dev(out_ids, torch.int32, "out_ids"), _dev(out_dists, torch.float32, "out_dists"), st))


def qg_search_mixed(idx: Index, queries, nq: int, k_per_query, ef_per_query, k_max: int, ef_max: int, flags: int,
                    out_ids, out_dists, out_stats=None):
    if queries.shape != (nq, idx.d) or out_ids.shape != (nq, k_max) or out_dists.shape != (nq, k_max):
        raise ValueError("shape mismatch")
    if k_per_query.shape != (nq,) or ef_per_query.shape != (nq,):
        raise ValueError("per-query k and ef must be [nq]")
    if out_stats is not None and out_stats.shape != (nq, 4):
        raise ValueError("stats shape mismatch")
    st = _dev(out_stats, torch.int32, "out_stats") if out_stats is not None else None
    _check(_lib.qg_search_mixed(idx.handle, _dev(queries, torch.float32, "queries"), nq,
                                _dev(k_per_query, torch.int32, "k_per_query"),
                                _dev(ef_per_query, torch.int32, "ef_per_query"), k_max, ef_max, flags,
                                _dev(out_ids, torch.int32, "out_ids"), _dev(out_dists, torch.float32, "out_dists"),
                                st))


def _stop_params(mlp, theta: float, t_min: int, t_every: int) -> StopParams:
    """Stop parameters without a trace (the MLP kept alive by the caller)."""
    if mlp is None or mlp.numel() != QG_STOP_MLP_PARAMS or mlp.element_size() != 2:
        raise ValueError("MLP parameters must be QG_STOP_MLP_PARAMS 16-bit values")
    sp = StopParams()
    sp.mlp = _dev(mlp, mlp.dtype, "mlp")
    sp.theta, sp.t_min, sp.t_every, sp.trace_max = float(theta), int(t_min), int(t_every), 0
    return sp


def qg_search_stop(idx: Index, queries, nq: int, k: int, ef: int, flags: int, mlp, theta: float, t_min: int,
                   t_every: int, trace_max: int, trace, out_ids, out_dists, out_stats=None):
    if queries.shape != (nq, idx.d) or out_ids.shape != (nq, k) or out_dists.shape != (nq, k):
        raise ValueError("shape mismatch")
    sp = StopParams()
    if mlp is not None:
        if mlp.numel() != QG_STOP_MLP_PARAMS or mlp.element_size() != 2:
            raise ValueError("MLP parameters must be QG_STOP_MLP_PARAMS 16-bit values")
        sp.mlp = _dev(mlp, mlp.dtype, "mlp")
    sp.theta, sp.t_min, sp.t_every, sp.trace_max = float(theta), int(t_min), int(t_every), int(trace_max)
    if trace_max > 0:
        f, n, o, c = trace
        if f.shape != (nq, trace_max, 16) or n.shape != (nq, trace_max, k) or o.shape != (nq, trace_max) \
                or c.shape != (nq,):
            raise ValueError("trace shape mismatch")
        sp.trace_features = _dev(f, torch.float32, "trace_features")
        sp.trace_nn = _dev(n, torch.int32, "trace_nn")
        sp.trace_out = _dev(o, torch.float32, "trace_out")
        sp.trace_count = _dev(c, torch.int32, "trace_count")
    st = _dev(out_stats, torch.int32, "out_stats") if out_stats is not None else None
    _check(_lib.qg_search_stop(idx.handle, _dev(queries, torch.float32, "queries"), nq, k, ef, flags,
                               ctypes.byref(sp), _dev(out_ids, torch.int32, "out_ids"),
                               _dev(out_dists, torch.float32, "out_dists"), st))


def qg_search(idx: Index, queries, nq: int, k: int, ef: int, out_ids, out_dists) -> None:
    qg_search_ex(idx, queries, nq, k, ef, 0, out_ids, out_dists, None)


def qg_rotate(idx: Index, x, n: int, out) -> None:
    if x.shape != (n, idx.d) or out.shape != (n, idx.d):
        raise ValueError("shape mismatch")
    _check(_lib.qg_rotate(idx.handle, _dev(x, torch.float32, "in"), n, _dev(out, torch.float32, "out")))


def qg_estimate(idx: Index, queries, vertex_of_query, nq: int, out_S, out_est, out_dist) -> None:
    if queries.shape != (nq, idx.d) or vertex_of_query.shape != (nq,):
        raise ValueError("shape mismatch")
    _check(_lib.qg_estimate(idx.handle, _dev(queries, torch.float32, "queries"),
                            _dev(vertex_of_query, torch.int32, "vertex_of_query"), nq,
                            _dev(out_S, torch.int32, "out_S"), _dev(out_est, torch.float32, "out_est"),
                            _dev(out_dist, torch.float32, "out_dist")))


def qg_copy_blocks(idx: Index, first: int, count: int, dst) -> None:
    if dst.numel() * dst.element_size() < count * idx.block_bytes:
        raise ValueError("destination too small")
    _check(_lib.qg_copy_blocks(idx.handle, first, count, _dev(dst, dst.dtype, "dst")))


def qg_set_stream(idx: Index, stream) -> None:
    idx.set_stream(stream)


def qg_index_info(idx: Index):
    return idx.n, idx.d, idx.r, idx.entry, idx.block_bytes


def qg_timing(idx: Index, enable: int) -> None:
    idx.timing(bool(enable))


def qg_timing_read(idx: Index, kernel: int):
    return idx.timing_read(kernel)


def qg_free_index(idx: Index) -> None:
    idx.free()


def _host(a: np.ndarray, dtype, name: str):
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags.c_contiguous:
        raise TypeError(f"{name} must be a C-contiguous numpy array of {np.dtype(dtype).name}")
    return ctypes.c_void_p(a.ctypes.data)


class Server:
    """The library's serving loop over one index (qg_server_*): requests with
    their own k and ef are batched continuously onto `streams` device streams."""

    def __init__(self, index: Index, streams: int = 2, max_batch: int = 1024, k_max: int = 100, ef_max: int = 256):
        h = ctypes.c_void_p()
        _check(_lib.qg_server_create(index.handle, streams, max_batch, k_max, ef_max, ctypes.byref(h)))
        self._h, self._index, self.d, self.k_max = h, index, index.d, k_max
        # host arrays of accepted traces: the library's threads read them (the
        # producer, and dispatch through each pending request's row pointer)
        # until a drain succeeds or the server is destroyed
        self._traces = []
        self._stop = None

    def set_stop(self, mlp: torch.Tensor | None, theta: float = 0.0, t_min: int = 8, t_every: int = 4) -> None:
        """Run later batches with the learned stop (mlp: bf16 bits on the device), or without it (None)."""
        if mlp is None:
            _check(_lib.qg_server_set_stop(self._h, None))
            self._stop = None
            return
        sp = _stop_params(mlp, theta, t_min, t_every)
        _check(_lib.qg_server_set_stop(self._h, ctypes.byref(sp)))
        self._stop = mlp  # the server reads the parameters from device memory while it runs

    def submit(self, query: np.ndarray, k: int, ef: int, tag: int) -> None:
        q = np.ascontiguousarray(query, dtype=np.float32).reshape(-1)
        if q.shape[0] != self.d:
            raise ValueError("query has the wrong dimension")
        _check(_lib.qg_server_submit(self._h, ctypes.c_void_p(q.ctypes.data), k, ef, ctypes.c_uint64(tag)))

    def set_recall_map(self, k, target, ef) -> None:
        """Beam per (k, target recall): rows of equal-length sequences k, target, ef."""
        ka = np.ascontiguousarray(k, dtype=np.int32)
        ta = np.ascontiguousarray(target, dtype=np.float32)
        ea = np.ascontiguousarray(ef, dtype=np.int32)
        if not (ka.shape == ta.shape == ea.shape) or ka.ndim != 1:
            raise ValueError("recall map rows must be equal-length vectors")
        _check(_lib.qg_server_set_recall_map(self._h, _host(ka, np.int32, "k"), _host(ta, np.float32, "target"),
                                             _host(ea, np.int32, "ef"), int(ka.shape[0])))

    def submit_target(self, query: np.ndarray, k: int, target: float, tag: int) -> None:
        """submit with a target recall, mapped to a beam by the recall map."""
        q = np.ascontiguousarray(query, dtype=np.float32).reshape(-1)
        if q.shape[0] != self.d:
            raise ValueError("query has the wrong dimension")
        _check(_lib.qg_server_submit_target(self._h, ctypes.c_void_p(q.ctypes.data), k, float(target),
                                            ctypes.c_uint64(tag)))

    def replay_target(self, queries: np.ndarray, k: np.ndarray, target: np.ndarray, arrival_s: np.ndarray) -> None:
        """replay with a target recall per request in place of ef (mapped by the recall map)."""
        arrs = (np.ascontiguousarray(queries, dtype=np.float32), np.ascontiguousarray(k, dtype=np.int32),
                np.ascontiguousarray(target, dtype=np.float32), np.ascontiguousarray(arrival_s, dtype=np.float64))
        n = arrs[0].shape[0]
        if arrs[0].shape != (n, self.d) or arrs[1].shape != (n,) or arrs[2].shape != (n,) or arrs[3].shape != (n,):
            raise ValueError("trace shape mismatch")
        _check(_lib.qg_server_replay_target(self._h, _host(arrs[0], np.float32, "queries"),
                                            _host(arrs[1], np.int32, "k"), _host(arrs[2], np.float32, "target"),
                                            _host(arrs[3], np.float64, "arrival_s"), n))
        self._traces.append(arrs)  # accepted: kept alive until a drain succeeds or close()

    def poll(self, max_results: int = 1 << 16, payload: bool = True, with_batch: bool = False):
        """-> (tags uint64 [n], ids int32 [n,k_max], dists f32 [n,k_max], latency s [n][, batch index int64 [n]])
        of finished requests."""
        tags = np.empty(max_results, np.uint64)
        lat = np.empty(max_results, np.float64)
        bat = np.empty(max_results, np.int64) if with_batch else None
        ids = np.empty((max_results, self.k_max), np.int32) if payload else None
        dists = np.empty((max_results, self.k_max), np.float32) if payload else None
        n = _lib.qg_server_poll(self._h, max_results, ctypes.c_void_p(tags.ctypes.data),
                                ctypes.c_void_p(ids.ctypes.data) if payload else None,
                                ctypes.c_void_p(dists.ctypes.data) if payload else None,
                                ctypes.c_void_p(lat.ctypes.data),
                                ctypes.c_void_p(bat.ctypes.data) if with_batch else None)
        if n < 0:
            _check(int(n))
        out = (tags[:n], (ids[:n] if payload else None), (dists[:n] if payload else None), lat[:n])
        return out + (bat[:n],) if with_batch else out

    BATCH_RECORD = np.dtype([("t_oldest", np.float64), ("t_dispatch", np.float64), ("t_enqueued", np.float64),
                             ("t_done", np.float64), ("device_ms", np.float32), ("n", np.int32),
                             ("ef_max", np.int32), ("k_max", np.int32), ("slot", np.int32),
                             ("enqueue_cpu_ms", np.float32), ("enqueue_nvcsw", np.int32),
                             ("enqueue_nivcsw", np.int32), ("upload_ms", np.float32), ("search_ms", np.float32),
                             ("download_ms", np.float32)],
                            align=True)  # the C struct's layout, padded to its doubles' alignment

    def batches(self, first: int = 0, max_records: int = 1 << 22) -> np.ndarray:
        """Batch records (a structured array, fields as qg_server_batch) from index `first`."""
        out = np.zeros(max_records, self.BATCH_RECORD)
        n = _lib.qg_server_batches(self._h, int(first), int(max_records), ctypes.c_void_p(out.ctypes.data))
        if n < 0:
            _check(int(n))
        return out[:n]

    def replay(self, queries: np.ndarray, k: np.ndarray, ef: np.ndarray, arrival_s: np.ndarray) -> None:
        """Submit an open-loop trace (request i at arrival_s[i] seconds, tag i) from a library thread."""
        arrs = (np.ascontiguousarray(queries, dtype=np.float32), np.ascontiguousarray(k, dtype=np.int32),
                np.ascontiguousarray(ef, dtype=np.int32), np.ascontiguousarray(arrival_s, dtype=np.float64))
        n = arrs[0].shape[0]
        if arrs[0].shape != (n, self.d) or arrs[1].shape != (n,) or arrs[2].shape != (n,) or arrs[3].shape != (n,):
            raise ValueError("trace shape mismatch")
        _check(_lib.qg_server_replay(self._h, _host(arrs[0], np.float32, "queries"), _host(arrs[1], np.int32, "k"),
                                     _host(arrs[2], np.int32, "ef"), _host(arrs[3], np.float64, "arrival_s"), n))
        self._traces.append(arrs)  # accepted: kept alive until a drain succeeds or close()

    def drain(self, timeout_s: float = 120.0) -> None:
        """Wait until every submitted request has finished.  On a time-out or
        error the traces stay referenced (pending requests still point into
        them) until close()."""
        _check(_lib.qg_server_drain(self._h, float(timeout_s)))
        self._traces = []

    def stats(self):
        v = [ctypes.c_int64() for _ in range(4)]
        _check(_lib.qg_server_stats(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("submitted", "completed", "batches", "largest_batch"), (x.value for x in v)))

    def close(self) -> None:
        if self._h:
            _lib.qg_server_destroy(self._h)  # joins the library's threads
            self._h = None
            self._traces = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""ctypes front end of the plain CPU oracle (``qg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP path; both consume the same seeded inputs and the same index byte
layout (Sec. 3.1.3 of the SymphonyQG paper).

``build()`` compiles ``liboracle.so`` with gcc; ``lib()`` loads it (building
it first if it is missing).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "qg_oracle.c"), os.path.join(HERE, "qg_oracle_build.c")]
LIB = os.path.join(HERE, "liboracle.so")

NO_ME = 1
EXACT_EST = 2

_lib = None


def build() -> str:
    """Compile the oracle: -O2, no FP contraction, no fast-math, OpenMP."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-o", LIB + ".tmp"] + SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or any(os.path.getmtime(s) > os.path.getmtime(LIB) for s in SRC):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.qgo_block_bytes.argtypes = [ctypes.c_int, ctypes.c_int]
        L.qgo_block_bytes.restype = i64
        L.qgo_rotate.argtypes = [P, ctypes.c_int, P, i64, P]
        L.qgo_rotate.restype = None
        L.qgo_encode.argtypes = [P, i64, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int]
        L.qgo_encode.restype = ctypes.c_int
        L.qgo_query_prep.argtypes = [P, ctypes.c_int, P, P, P]
        L.qgo_query_prep.restype = None
        L.qgo_exact_dist.argtypes = [P, P, ctypes.c_int]
        L.qgo_exact_dist.restype = ctypes.c_float
        L.qgo_estimate.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, i32, P, P, P]
        L.qgo_estimate.restype = None
        L.qgo_search.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, i32, P, P, i64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, P, P, P, ctypes.c_int]
        L.qgo_search.restype = ctypes.c_int
        L.qgo_search_ls.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, i32, P, P, i64, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, P, P, P, ctypes.c_int, P, ctypes.c_float, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, P, P, P, P]
        L.qgo_search_ls.restype = ctypes.c_int
        L.qgo_ls_mlp.argtypes = [P, P]
        L.qgo_ls_mlp.restype = ctypes.c_float
        L.qgo_max_threads.argtypes = []
        L.qgo_max_threads.restype = ctypes.c_int
        L.qgo_build_graph.argtypes = [P, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, i32, P, P,
                                      P, P, ctypes.c_int]
        L.qgo_build_graph.restype = ctypes.c_int
        L.qgo_write_index.argtypes = [ctypes.c_char_p, i64, ctypes.c_int, ctypes.c_int, i32, P, P]
        L.qgo_write_index.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def block_bytes(D: int, R: int) -> int:
    return int(lib().qgo_block_bytes(D, R))


def rotate(M: np.ndarray, X: np.ndarray) -> np.ndarray:
    M = _c(M, np.float32)
    X = _c(np.atleast_2d(X), np.float32)
    out = np.empty_like(X)
    lib().qgo_rotate(_p(M), M.shape[0], _p(X), X.shape[0], _p(out))
    return out


def encode(X: np.ndarray, G: np.ndarray, M: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Vertex blocks [N, block_bytes] (uint8) for vectors X, graph G and rotation M."""
    X = _c(X, np.float32)
    G = _c(G, np.int32)
    M = _c(M, np.float32)
    N, D = X.shape
    R = G.shape[1]
    out = np.zeros((N, block_bytes(D, R)), dtype=np.uint8)
    rc = lib().qgo_encode(_p(X), N, D, _p(G), R, _p(M), _p(out), nthreads)
    if rc != 0:
        raise RuntimeError(f"qgo_encode failed: {rc}")
    return out


def query_prep(qrot: np.ndarray):
    """(Delta, q_s[D], LUT[D/4][16]) for one rotated query."""
    qrot = _c(qrot, np.float32)
    D = qrot.shape[0]
    delta = np.zeros(1, np.float32)
    qs = np.zeros(D, np.int32)
    lut = np.zeros((D // 4, 16), np.int32)
    lib().qgo_query_prep(_p(qrot), D, _p(delta), _p(qs), _p(lut))
    return float(delta[0]), qs, lut


def exact_dist(q: np.ndarray, x: np.ndarray) -> float:
    q = _c(q, np.float32)
    x = _c(x, np.float32)
    return float(lib().qgo_exact_dist(_p(q), _p(x), q.shape[0]))


def estimate(blocks: np.ndarray, D: int, R: int, q: np.ndarray, qrot: np.ndarray, v: int):
    """(S[R], est[R], dist_c) for the neighbours of vertex v."""
    blocks = _c(blocks, np.uint8)
    q = _c(q, np.float32)
    qrot = _c(qrot, np.float32)
    S = np.zeros(R, np.int32)
    est = np.zeros(R, np.float32)
    dc = np.zeros(1, np.float32)
    lib().qgo_estimate(_p(blocks), D, R, _p(q), _p(qrot), int(v), _p(S), _p(est), _p(dc))
    return S, est, float(dc[0])


def search(blocks: np.ndarray, D: int, R: int, entry: int, M: np.ndarray, Q: np.ndarray, k: int, ef: int,
           flags: int = 0, nthreads: int = 0, with_stats: bool = False):
    """Algorithm 1 for every row of Q: (ids[nq,k], dists[nq,k][, stats[nq,4]])."""
    blocks = _c(blocks, np.uint8)
    M = _c(M, np.float32)
    Q = _c(np.atleast_2d(Q), np.float32)
    nq = Q.shape[0]
    N = blocks.shape[0]
    ids = np.zeros((nq, k), np.int32)
    dists = np.zeros((nq, k), np.float32)
    stats = np.zeros((nq, 4), np.int64)
    rc = lib().qgo_search(_p(blocks), N, D, R, int(entry), _p(M), _p(Q), nq, k, ef, flags, _p(ids), _p(dists),
                          _p(stats), nthreads)
    if rc != 0:
        raise RuntimeError(f"qgo_search failed: {rc}")
    return (ids, dists, stats) if with_stats else (ids, dists)


LS_PARAMS = 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1


def search_ls(blocks, D, R, entry, M, Q, k, ef, w=None, theta=0.0, t_min=8, t_every=4, max_evals=0,
              flags=0, nthreads=0):
    """Algorithm 1 with the learned stop (w: uint16 bf16 parameters or None) and
    an optional trace.  Returns (ids, dists, stats, trace) with trace =
    (features [nq,max_evals,16], nn ids [nq,max_evals,k], mlp out [nq,max_evals], count [nq]) or None."""
    blocks = _c(blocks, np.uint8)
    M = _c(M, np.float32)
    Q = _c(np.atleast_2d(Q), np.float32)
    nq, N = Q.shape[0], blocks.shape[0]
    ids = np.zeros((nq, k), np.int32)
    dists = np.zeros((nq, k), np.float32)
    stats = np.zeros((nq, 4), np.int64)
    wp = None
    if w is not None:
        w = _c(w, np.uint16)
        assert w.size == LS_PARAMS
        wp = _p(w)
    me = max(max_evals, 0)
    tf = np.zeros((nq, max(me, 1), 16), np.float32)
    tn = np.zeros((nq, max(me, 1), k), np.int32)
    to = np.zeros((nq, max(me, 1)), np.float32)
    tc = np.zeros(nq, np.int32)
    rc = lib().qgo_search_ls(_p(blocks), N, D, R, int(entry), _p(M), _p(Q), nq, k, ef, flags, _p(ids), _p(dists),
                             _p(stats), nthreads, wp, float(theta), t_min, t_every, me, _p(tf), _p(tn), _p(to),
                             _p(tc))
    if rc != 0:
        raise RuntimeError(f"qgo_search_ls failed: {rc}")
    return ids, dists, stats, ((tf, tn, to, tc) if me else None)


def ls_mlp(w, f) -> float:
    w = _c(w, np.uint16)
    f = _c(f, np.float32)
    return float(lib().qgo_ls_mlp(_p(w), _p(f)))


def build_graph(X: np.ndarray, R: int, EF: int, t: int, M: np.ndarray, entry: int, G0: np.ndarray,
                fill: np.ndarray, refine: bool = True, nthreads: int = 0) -> np.ndarray:
    """Algorithm 2 (Indexing): returns the final graph G[N][R] (-1 = empty slot when refine is False)."""
    X = _c(X, np.float32)
    M = _c(M, np.float32)
    G0 = _c(G0, np.int32)
    fill = _c(fill, np.int32)
    N, D = X.shape
    G = np.zeros((N, R), np.int32)
    st = np.zeros(4, np.int64)
    rc = lib().qgo_build_graph(_p(X), N, D, R, EF, t, _p(M), int(entry), _p(G0), _p(fill), _p(G),
                               _p(st), (1 if refine else 0) | (nthreads << 8))
    if rc != 0:
        raise RuntimeError(f"qgo_build_graph failed: {rc} (reach before/after repair {st[0]}/{st[2]}, "
                           f"repairs {st[1]})")
    return G


def max_threads() -> int:
    return int(lib().qgo_max_threads())


def write_index(path: str, blocks: np.ndarray, D: int, R: int, entry: int, M: np.ndarray) -> None:
    """Write an index file in the on-disk format (header, rotation, blocks)."""
    blocks = _c(blocks, np.uint8)
    M = _c(M, np.float32)
    rc = lib().qgo_write_index(path.encode(), blocks.shape[0], D, R, int(entry), _p(M), _p(blocks))
    if rc != 0:
        raise RuntimeError(f"qgo_write_index failed: {rc}")

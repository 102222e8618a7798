"""Seeded synthetic inputs for the SymphonyQG query path.

This module holds none of the method's arithmetic: it draws vectors, queries,
the random orthogonal rotation and random graphs, builds a generic
k-nearest-neighbour input graph, and computes brute-force ground truth.  Both
the HIP path and the CPU oracle consume what it produces; neither is imported
here.

The paper's datasets (Table 1: SIFT, GIST, Deep, ...) are not available, so
these distributions stand in for them with the same shapes (N, D, number of
queries, metric).  All draws use numpy ``Generator(PCG64(seed))`` with seeds
1000*cfg + {1: data, 2: queries, 3: rotation, 4: graph init, 5: random fill}.
"""
from __future__ import annotations

import math
import sys
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Config:
    cfg: int
    N: int
    D: int
    R: int
    nq: int
    k: int
    efs: tuple = field(default=())
    note: str = ""


# The synthetic workloads, by what they stand in for.
TINY, SIFT_LIKE, GIST_LIKE, UNIT768, DEEP_LIKE = 1, 2, 3, 4, 5

CONFIGS = {
    1: Config(1, 10_000, 128, 32, 200, 10, (64,), "16-cluster Gaussian mixture, sigma 0.3"),
    2: Config(2, 1_000_000, 128, 32, 10_000, 10, (16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512),
              "SIFT-shaped: 1000-cluster mixture, integer values clipped to [0,255]"),
    3: Config(3, 1_000_000, 960, 64, 1_000, 10, (64, 128, 256), "GIST-shaped: rank-64 non-negative factor model"),
    4: Config(4, 1_000_000, 768, 32, 10_000, 10, (64, 128, 256),
              "unit-norm rank-128 (1000 overlapping blobs in a 16-d latent) plus noise, shifted queries"),
    5: Config(5, 5_000_000, 96, 32, 10_000, 10, (32, 64, 128),
              "unit-norm 4096-cluster mixture (overlapping blobs in a 16-d latent)"),
}


def seed(cfg: int, what: str) -> int:
    return 1000 * cfg + {"data": 1, "queries": 2, "rotation": 3, "graph": 4, "fill": 5, "long": 6, "train": 7}[what]


def _rng(s: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(s))


def _normalize(x: np.ndarray) -> np.ndarray:
    n = np.linalg.norm(x.astype(np.float64), axis=1, keepdims=True)
    n[n == 0] = 1.0
    return (x / n).astype(np.float32)


def gen_data(cfg: int, n: int | None = None, nq: int | None = None, D: int | None = None, **kw):
    """(X[n, D], Q[nq, D]) float32 for config ``cfg``; n/nq/D override the sizes.
    ``qseed`` draws the queries from another seed (e.g. training queries for the
    learned stop); the data distribution does not depend on it."""
    c = CONFIGS[cfg]
    n = c.N if n is None else n
    nq = c.nq if nq is None else nq
    D = c.D if D is None else D
    g = _rng(seed(cfg, "data"))
    gq = _rng(kw.get("qseed", seed(cfg, "queries")))
    if cfg == 1:
        mu = g.standard_normal((16, D))
        X = mu[g.integers(0, 16, n)] + 0.3 * g.standard_normal((n, D))
        Q = mu[gq.integers(0, 16, nq)] + 0.3 * gq.standard_normal((nq, D))
        return X.astype(np.float32), Q.astype(np.float32)
    if cfg == 2:
        # A 1000-component Gaussian mixture with SIFT's low local dimension:
        # components are overlapping blobs in a shared 12-d latent space
        # (centre z_c ~ N(0, I), within-component N(0, 0.6^2 I), mapped to 128-d
        # by one random W), plus 4 component-specific directions and an
        # isotropic floor.  Values are clipped to [0, 255] and rounded.
        ncent = kw.get("ncent", 1000)
        dl, dc = 12, 4
        W = (g.standard_normal((D, dl)) * (26.0 / math.sqrt(dl))).astype(np.float32)
        zc = g.standard_normal((ncent, dl)).astype(np.float32)
        Ac = (g.standard_normal((ncent, D, dc)) * (8.0 / math.sqrt(dc))).astype(np.float32)

        def draw(gg, m):
            out = np.empty((m, D), np.float32)
            lab = gg.integers(0, ncent, m)
            for s in range(0, m, 1 << 16):
                e = min(m, s + (1 << 16))
                zz = zc[lab[s:e]] + np.float32(0.6) * gg.standard_normal((e - s, dl), dtype=np.float32)
                v = 64.0 + zz @ W.T
                v += np.einsum("bdr,br->bd", Ac[lab[s:e]], gg.standard_normal((e - s, dc), dtype=np.float32))
                v += np.float32(3.0) * gg.standard_normal((e - s, D), dtype=np.float32)
                out[s:e] = np.rint(np.clip(v, 0.0, 255.0))
            return out

        return draw(g, n), draw(gq, nq)
    # configs 3-5 are drawn in float32, 32,768 rows at a time (the full sizes
    # are 1M x 960, 1M x 768 and 5M x 96)
    def chunked(m, row):
        out = np.empty((m, D), np.float32)
        for s in range(0, m, 1 << 15):
            e = min(m, s + (1 << 15))
            out[s:e] = row(e - s)
        return out

    f32 = np.float32
    if cfg == 3:
        W = (np.abs(g.standard_normal((D, 64))) / 8.0).astype(f32)

        def draw(gg, m):
            return chunked(m, lambda b: np.maximum(f32(0.0), np.abs(gg.standard_normal((b, 64), dtype=f32)) @ W.T
                                                   + f32(0.05) * gg.standard_normal((b, D), dtype=f32)))

        return draw(g, n), draw(gq, nq)
    if cfg == 4:
        # Unit-norm rank-128 data plus noise: a 128-d latent z mapped to 768-d
        # by one random U, plus N(0, 0.06^2) per coordinate, renormalised.  The
        # latent is shaped like the SIFT-shaped set's: 1000 overlapping blobs in
        # a shared 16-d space (centres N(0, I), within-blob N(0, I)) mapped by a
        # random W, 8 blob-specific directions (total variance 0.28^2 per latent
        # coordinate) and an N(0, 0.1^2) floor, so the local dimension is about
        # 15 while the span is all 128 dims.  Queries come from the same
        # distribution with the latent mean moved by half its RMS norm along a
        # random direction.
        L, dl, dc, nb = 128, 16, 8, 1000
        U = (g.standard_normal((D, L)) / math.sqrt(D)).astype(f32)
        W = (g.standard_normal((L, dl)) / math.sqrt(dl)).astype(f32)
        zc = g.standard_normal((nb, dl)).astype(f32)
        Ac = (g.standard_normal((nb, L, dc)) * (0.28 / math.sqrt(dc))).astype(f32)
        gvec = g.standard_normal(L)  # the query shift is part of the distribution, not of one query draw
        rms = math.sqrt(L * (2.0 + 0.28 ** 2 + 0.1 ** 2))
        shift = (0.5 * rms * gvec / np.linalg.norm(gvec)).astype(f32)

        def draw(gg, m, sh):
            lab = gg.integers(0, nb, m)
            pos = [0]

            def row(b):
                s = pos[0]
                pos[0] += b
                li = lab[s:s + b]
                z = (zc[li] + gg.standard_normal((b, dl), dtype=f32)) @ W.T
                z += np.einsum("blc,bc->bl", Ac[li], gg.standard_normal((b, dc), dtype=f32))
                z += f32(0.1) * gg.standard_normal((b, L), dtype=f32) + sh
                return _normalize(z @ U.T + f32(0.06) * gg.standard_normal((b, D), dtype=f32))

            return chunked(m, row)

        return draw(g, n, f32(0.0)), draw(gq, nq, shift)
    if cfg == 5:
        # Unit-norm 4096-blob mixture with a low local dimension (like the
        # Deep embeddings it stands in for): blobs overlap in a shared 16-d
        # latent space (centres N(0, I), within-blob N(0, I)) mapped to 96-d by
        # a random W, plus 4 blob-specific directions (total variance 0.28^2
        # per coordinate) and an N(0, 0.1^2) floor, renormalised.  Queries come
        # from the same distribution.
        dl, dc, nb = 16, 4, 4096
        W = (g.standard_normal((D, dl)) / math.sqrt(dl)).astype(f32)
        zc = g.standard_normal((nb, dl)).astype(f32)
        Ac = (g.standard_normal((nb, D, dc)) * (0.28 / math.sqrt(dc))).astype(f32)

        def draw(gg, m):
            lab = gg.integers(0, nb, m)
            pos = [0]

            def row(b):
                s = pos[0]
                pos[0] += b
                li = lab[s:s + b]
                z = (zc[li] + gg.standard_normal((b, dl), dtype=f32)) @ W.T
                z += np.einsum("bdc,bc->bd", Ac[li], gg.standard_normal((b, dc), dtype=f32))
                z += f32(0.1) * gg.standard_normal((b, D), dtype=f32)
                return _normalize(z)

            return chunked(m, row)

        return draw(g, n), draw(gq, nq)
    raise ValueError(cfg)


def rotation(D: int, s: int) -> np.ndarray:
    """A random orthogonal matrix M = P^T (P: Gaussian matrix -> QR with the
    sign of diag(R) folded in), rounded to multiples of 2^-24 so every entry is
    an exact float32 with a fixed absolute precision."""
    G = _rng(s).standard_normal((D, D))
    Qm, Rm = np.linalg.qr(G)
    P = Qm * np.sign(np.diag(Rm))[None, :]
    M = np.round(P.T * 2.0 ** 24) / 2.0 ** 24
    return np.ascontiguousarray(M, dtype=np.float32)


def random_graph(N: int, R: int, s: int) -> np.ndarray:
    """R distinct non-self random out-neighbours per vertex (int32 [N, R])."""
    g = _rng(s)
    if R >= N:
        raise ValueError("R must be < N")
    G = g.integers(0, N - 1, size=(N, R), dtype=np.int64)
    G += G >= np.arange(N)[:, None]  # skip self
    for _ in range(64):
        srt = np.sort(G, axis=1)
        dup = np.zeros_like(G, dtype=bool)
        dup_rows = np.any(srt[:, 1:] == srt[:, :-1], axis=1)
        if not dup_rows.any():
            break
        for u in np.nonzero(dup_rows)[0]:
            seen = set()
            for j in range(R):
                while G[u, j] in seen:
                    v = int(g.integers(0, N - 1))
                    G[u, j] = v + (v >= u)
                seen.add(int(G[u, j]))
        del dup
    return G.astype(np.int32)


def medoid(X: np.ndarray) -> int:
    """The vertex nearest (fp64) to the mean of X; ties go to the lowest id."""
    mean = X.astype(np.float64).mean(axis=0)
    best, bi = np.inf, 0
    for s in range(0, X.shape[0], 1 << 16):
        d = ((X[s:s + (1 << 16)].astype(np.float64) - mean) ** 2).sum(axis=1)
        i = int(np.argmin(d))
        if d[i] < best:
            best, bi = float(d[i]), s + i
    return bi


# ----------------------------------------------------------- brute force ---

def _topk_rows_np(X: np.ndarray, Y: np.ndarray, k: int, exclude_self: bool = False, row0: int = 0):
    """For each row of Y: the k nearest rows of X by (fp64 squared distance, id)."""
    X64 = X.astype(np.float64)
    xx = (X64 ** 2).sum(axis=1)
    ids_out = np.empty((Y.shape[0], k), np.int64)
    d_out = np.empty((Y.shape[0], k), np.float64)
    for s in range(0, Y.shape[0], 512):
        y = Y[s:s + 512].astype(np.float64)
        d = xx[None, :] + (y ** 2).sum(axis=1)[:, None] - 2.0 * y @ X64.T
        if exclude_self:
            d[np.arange(y.shape[0]), row0 + s + np.arange(y.shape[0])] = np.inf
        kk = min(k + 32, X.shape[0])
        part = np.argpartition(d, kk - 1, axis=1)[:, :kk]
        for r in range(y.shape[0]):
            cand = part[r]
            exact = ((X64[cand] - y[r]) ** 2).sum(axis=1)
            if exclude_self:
                exact[cand == row0 + s + r] = np.inf
            o = np.lexsort((cand, exact))[:k]
            ids_out[s + r] = cand[o]
            d_out[s + r] = exact[o]
    return ids_out, d_out


_TOPK_BLOCK = 1 << 20  # base rows per shortlist block of the torch brute force


def _topk_rows_torch(X, Y, k: int, exclude_self: bool, device):
    """Same as _topk_rows_np on a torch device (fp32 GEMM shortlist, fp64 re-rank)."""
    import torch
    Xt = torch.from_numpy(np.ascontiguousarray(X)).to(device)
    xx = (Xt.double() ** 2).sum(1).float()
    N = Xt.shape[0]
    kk = min(k + 32, N)
    ids_out = np.empty((Y.shape[0], k), np.int64)
    d_out = np.empty((Y.shape[0], k), np.float64)
    chunk = max(256, min(8192, int(2e9 // max(N, 1))))
    t0 = time.time()
    for s in range(0, Y.shape[0], chunk):
        if s and (s // chunk) % 100 == 0:
            print(f"[synth] brute force {s}/{Y.shape[0]} rows, {time.time() - t0:.0f}s", file=sys.stderr, flush=True)
        y = torch.from_numpy(np.ascontiguousarray(Y[s:s + chunk])).to(device)
        # shortlist per block of at most 2^20 base rows, then over the blocks'
        # shortlists (a top-k over a whole 5M-wide row is not relied on)
        parts_v, parts_i = [], []
        for b0 in range(0, N, _TOPK_BLOCK):
            b1 = min(N, b0 + _TOPK_BLOCK)
            d = xx[None, b0:b1] - 2.0 * (y @ Xt[b0:b1].T)
            if exclude_self:
                r = torch.arange(y.shape[0], device=device)
                own = (s + r >= b0) & (s + r < b1)
                d[r[own], (s + r[own] - b0)] = float("inf")
            v, i = torch.topk(d, min(kk, b1 - b0), dim=1, largest=False, sorted=False)
            parts_v.append(v)
            parts_i.append(i + b0)
        v, i = torch.cat(parts_v, 1), torch.cat(parts_i, 1)
        cand = torch.gather(i, 1, torch.topk(v, kk, dim=1, largest=False, sorted=False).indices)
        exact = ((Xt[cand].double() - y.double()[:, None, :]) ** 2).sum(-1)
        if exclude_self:
            exact[cand == (s + torch.arange(y.shape[0], device=device))[:, None]] = float("inf")
        # lexicographic (distance, id): sort by id, then stable sort by distance
        o1 = torch.argsort(cand, dim=1, stable=True)
        cand = torch.gather(cand, 1, o1)
        exact = torch.gather(exact, 1, o1)
        o2 = torch.argsort(exact, dim=1, stable=True)[:, :k]
        ids_out[s:s + y.shape[0]] = torch.gather(cand, 1, o2).cpu().numpy()
        d_out[s:s + y.shape[0]] = torch.gather(exact, 1, o2).cpu().numpy()
    return ids_out, d_out


def ground_truth(X: np.ndarray, Q: np.ndarray, k: int, device=None):
    """Exact k nearest neighbours of each query: ids int32 [nq, k] and fp64
    squared distances, ordered by (distance, id)."""
    if device is None:
        ids, d = _topk_rows_np(X, Q, k)
    else:
        ids, d = _topk_rows_torch(X, Q, k, False, device)
    return ids.astype(np.int32), d


def knn_graph(X: np.ndarray, R: int, s: int, n_long: int = 8, device=None) -> np.ndarray:
    """A generic input graph, int32 [N, R], with no duplicate or self edges.

    Slots 0 .. R-n_long-1 hold the nearest neighbours by (distance, id);
    slots R-n_long .. R-1 hold uniformly random long-range links (seeded),
    which make the graph an expander so every vertex is reachable with high
    probability.  A vertex that nobody points to takes over the last
    nearest-neighbour slot of its nearest neighbour whose target keeps
    another in-edge.  This is plain k-NN plus random links, not the paper's
    index construction."""
    N = X.shape[0]
    nk = R - n_long
    if nk < 1 or R >= N:
        raise ValueError("bad R / n_long")
    if device is None:
        nn, _ = _topk_rows_np(X, X, nk + 4, exclude_self=True)
    else:
        nn, _ = _topk_rows_torch(X, X, nk + 4, True, device)
    G = np.full((N, R), -1, np.int64)
    G[:, :nk] = nn[:, :nk]
    g = _rng(s)
    rows = np.arange(N)
    for col in range(nk, R):
        todo = rows
        for _ in range(1000):
            v = g.integers(0, N, todo.size)
            bad = (v == todo) | (G[todo, :col] == v[:, None]).any(axis=1)
            G[todo[~bad], col] = v[~bad]
            todo = todo[bad]
            if todo.size == 0:
                break
    indeg = np.bincount(G[G >= 0].ravel(), minlength=N)
    taken = np.zeros(N, bool)
    for v in np.nonzero(indeg == 0)[0]:
        for w in nn[v]:
            old = G[w, nk - 1]
            if not taken[w] and indeg[old] > 1 and not (G[w] == v).any():
                indeg[old] -= 1
                G[w, nk - 1] = v
                indeg[v] += 1
                taken[w] = True
                break
    return G.astype(np.int32)


def reachable(G: np.ndarray, entry: int) -> int:
    """Number of vertices reachable from entry (breadth first)."""
    N = G.shape[0]
    seen = np.zeros(N, bool)
    seen[entry] = True
    frontier = np.array([entry])
    while frontier.size:
        nxt = G[frontier].ravel()
        nxt = nxt[nxt >= 0]
        nxt = np.unique(nxt[~seen[nxt]])
        seen[nxt] = True
        frontier = nxt
    return int(seen.sum())


def recall(ids: np.ndarray, gt: np.ndarray, k: int) -> float:
    """Mean |G cap S| / K over queries (Sec. 4.1 metrics)."""
    hit = 0
    for a, b in zip(ids[:, :k], gt[:, :k]):
        hit += len(set(a.tolist()) & set(b.tolist()))
    return hit / (k * ids.shape[0])


def adr(dists: np.ndarray, gt_d: np.ndarray, k: int) -> float:
    """Average distance ratio: mean over queries and ranks of
    sqrt(d(S_i)) / sqrt(d(G_i)), skipping ranks whose true distance is 0."""
    a = np.sqrt(np.maximum(dists[:, :k].astype(np.float64), 0))
    b = np.sqrt(gt_d[:, :k])
    m = b > 0
    return float((a[m] / b[m]).mean()) if m.any() else 1.0

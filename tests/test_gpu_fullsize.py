"""Parity at full size: the index sizes of the benchmark workloads, searched in
the launch configuration the benchmark times, checked against the oracle on
sampled outputs it can compute one by one.

- Blocks: the oracle encodes a sample of vertices from their own and their
  neighbours' vectors (a small re-indexed copy of the inputs), and those
  blocks must equal the device's byte for byte.
- Search: the oracle searches the device's blocks (copied to the host; the
  sample above pins them to the oracle's encoding) for a sample of queries,
  and ids, distances and counters must equal those of the full-batch device
  search.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_12229_amd import qg  # noqa: E402

DEV = torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(msg):
    print(msg, flush=True)


def oracle_blocks_for(X, G, M, verts):
    """Oracle blocks of the vertices `verts`, encoded from a copy of the inputs
    that holds only them and their neighbours (ids renumbered, then restored)."""
    R = G.shape[1]
    nb = G[verts].ravel()
    keep = np.unique(np.concatenate([verts, nb[nb >= 0]]))
    pos = np.searchsorted(keep, verts)
    Gs = np.full((len(keep), R), -1, np.int32)
    sub = G[verts]
    Gs[pos] = np.where(sub >= 0, np.searchsorted(keep, np.maximum(sub, 0)), -1)
    blocks = oracle.encode(X[keep], Gs, M)[pos]
    # the neighbour ids stored in a block are the renumbered ones: restore them
    D = X.shape[1]
    off = 4 * D + R * (D // 8) + 8 * R
    ids = blocks[:, off:off + 4 * R].copy().view(np.int32)
    ids[ids >= 0] = keep[ids[ids >= 0]]
    blocks[:, off:off + 4 * R] = ids.view(np.uint8)
    return blocks


def check_full_size(cfg, X, Q, G, M, k, ef, launch, n_blocks=256, n_queries=48, seed=0, no_me_ef=0):
    N, D = X.shape
    R = G.shape[1]
    e = synth.medoid(X)
    say(f"full size cfg {cfg}: N={N} D={D} R={R} nq={len(Q)} k={k} ef={ef} launch={launch}")
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    rng = np.random.default_rng(seed)
    verts = np.sort(rng.choice(N, n_blocks, replace=False))
    dev_blocks = idx.blocks().cpu().numpy()
    assert np.array_equal(dev_blocks[verts], oracle_blocks_for(X, G, M, verts)), "sampled blocks differ"
    say("  sampled blocks equal")
    idx.set_launch(*launch)
    ids, dists, st = idx.search(T(Q), k, ef, stats=True)
    torch.cuda.synchronize()
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    qs = np.sort(rng.choice(len(Q), n_queries, replace=False))
    oi, od, os_ = oracle.search(dev_blocks, D, R, e, M, Q[qs], k, ef, with_stats=True)
    bad = np.nonzero((ids[qs] != oi).any(axis=1))[0]
    assert bad.size == 0, f"ids differ for queries {qs[bad][:10].tolist()}"
    assert np.array_equal(dists[qs], od), "distances differ"
    assert np.array_equal(st[qs, :3], os_[:, :3]), "counters differ"
    say(f"  {n_queries} sampled queries equal; mean expansions {st[:, 0].mean():.1f}")
    if no_me_ef:  # the w/o ME ablation on the same index and sample
        ids, dists, st = idx.search(T(Q), k, no_me_ef, flags=qg.QG_SEARCH_NO_ME, stats=True)
        torch.cuda.synchronize()
        ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
        oi, od, os_ = oracle.search(dev_blocks, D, R, e, M, Q[qs], k, no_me_ef, flags=oracle.NO_ME, with_stats=True)
        bad = np.nonzero((ids[qs] != oi).any(axis=1))[0]
        assert bad.size == 0, f"w/o ME: ids differ for queries {qs[bad][:10].tolist()}"
        assert np.array_equal(dists[qs], od), "w/o ME: distances differ"
        assert np.array_equal(st[qs, :3], os_[:, :3]), "w/o ME: counters differ"
        say(f"  w/o ME ef={no_me_ef}: {n_queries} sampled queries equal")


def test_sift_shaped_full_size():
    """1M x 128, R = 32, the benchmark's input graph, 10,000 queries at the
    benchmark's beam (68) in a launch shape its autotuner picks, and at the
    default shape;
    the w/o ME search at the beam that reaches the same recall (48)."""
    c = synth.SIFT_LIKE
    X, Q = synth.gen_data(c)
    M = synth.rotation(128, synth.seed(c, "rotation"))
    G = synth.knn_graph(X, 32, synth.seed(c, "long"), device=DEV)
    check_full_size(c, X, Q, G, M, 10, 68, (2, 4, 24))
    check_full_size(c, X, Q, G, M, 10, 68, (4, 3, 0), seed=1, no_me_ef=48)


def test_serving_shaped_full_size():
    """5M x 96 unit-norm (the serving workload's size), R = 32, with a seeded
    random graph (its k-NN graph takes minutes to build), 10,000 queries."""
    c = synth.DEEP_LIKE
    X, Q = synth.gen_data(c)
    M = synth.rotation(96, synth.seed(c, "rotation"))
    G = synth.random_graph(len(X), 32, synth.seed(c, "graph"))
    check_full_size(c, X, Q, G, M, 10, 64, (4, 3, 0), n_queries=24)


def test_gist_shaped_full_size():
    """1M x 960, R = 64 (12.3 GB of blocks), with a seeded random graph,
    1,000 queries at k = 100."""
    c = synth.GIST_LIKE
    X, Q = synth.gen_data(c)
    M = synth.rotation(960, synth.seed(c, "rotation"))
    G = synth.random_graph(len(X), 64, synth.seed(c, "graph"))
    check_full_size(c, X, Q, G, M, 100, 128, (4, 3, 0), n_blocks=64, n_queries=8)

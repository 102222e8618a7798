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


def check_full_size(cfg, X, Q, G, M, k, ef, launch, n_blocks=256, n_queries=48, seed=0, no_me_ef=0,
                    mixed_classes=()):
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
    if mixed_classes:  # one mixed launch, every query its own (k, ef), in the shape the mixed-batch tuner picks
        cls = rng.integers(0, len(mixed_classes), len(Q))
        ks = np.array([mixed_classes[i][0] for i in cls], np.int32)
        efs = np.array([mixed_classes[i][1] for i in cls], np.int32)
        k_max, ef_max = int(ks.max()), int(efs.max())
        Qd, kd, efd = T(Q), T(ks), T(efs)
        tuned = idx.autotune_mixed(Qd, kd, efd, k_max, ef_max)
        ids, dists, st = idx.search_mixed(Qd, kd, efd, k_max=k_max, ef_max=ef_max, stats=True)
        torch.cuda.synchronize()
        ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
        for i, (kc, efc) in enumerate(mixed_classes):
            sel = qs[cls[qs] == i]
            if sel.size == 0:
                continue
            oi, od, os_ = oracle.search(dev_blocks, D, R, e, M, Q[sel], kc, efc, with_stats=True)
            assert np.array_equal(ids[sel, :kc], oi), f"mixed class (k={kc}, ef={efc}): ids differ"
            assert np.array_equal(dists[sel, :kc], od), f"mixed class (k={kc}, ef={efc}): distances differ"
            assert np.array_equal(st[sel, :3], os_[:, :3]), f"mixed class (k={kc}, ef={efc}): counters differ"
            assert (ids[sel, kc:] == -1).all() and np.isinf(dists[sel, kc:]).all()
        say(f"  mixed launch {mixed_classes} in shape {tuned[:3] + tuned[4:]}: sampled rows equal")


def test_sift_shaped_full_size():
    """1M x 128, R = 32, the benchmark's graph (Algorithm 2 on the device,
    EF = 400, t = 3, from the same seeds), 10,000 queries at the benchmark's
    beam (48) in the launch shape its autotuner picked (8 wavefronts per
    workgroup, F = 3, no cap, beam in registers), at the default shape with
    the beam in LDS, and the w/o ME search at ef 32."""
    c = synth.SIFT_LIKE
    X, Q = synth.gen_data(c)
    M = synth.rotation(128, synth.seed(c, "rotation"))
    e = synth.medoid(X)
    G0 = T(synth.random_graph(len(X), 32, synth.seed(c, "graph")))
    fill = T(synth.random_graph(len(X), 32, synth.seed(c, "fill")))
    Gd, st = qg.qg_build_graph(T(X), 32, 400, 3, T(M), e, G0, fill, progress=True)
    G = Gd.cpu().numpy()
    say(f"Algorithm 2 graph: {st}")
    check_full_size(c, X, Q, G, M, 10, 48, (8, 3, 0, 1))
    check_full_size(c, X, Q, G, M, 10, 48, (4, 3, 0, 0), seed=1, no_me_ef=32)


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
    1,000 queries at k = 100, then one mixed launch of k = 10 and k = 100 at
    two beams each (the 1M x 960 bench leg's kind of batch)."""
    c = synth.GIST_LIKE
    X, Q = synth.gen_data(c)
    M = synth.rotation(960, synth.seed(c, "rotation"))
    G = synth.random_graph(len(X), 64, synth.seed(c, "graph"))
    check_full_size(c, X, Q, G, M, 100, 128, (4, 3, 0), n_blocks=64, n_queries=24,
                    mixed_classes=((10, 48), (10, 128), (100, 160), (100, 256)))

"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: rotated queries, codes, factors, FastScan sums and estimates bit-exact;
result ids identical and distances bit-equal (the requirement is 1e-5
relative; the canonical arithmetic makes them equal); per-query counters equal.
"""
import os

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


@pytest.fixture(scope="module")
def cfg1():
    """The small configuration: 10,000 vectors of the 16-cluster mixture, its
    index graph built by the oracle's Algorithm 2 (R = 32, EF = 200, t = 3,
    from seeded random initial and fill ids)."""
    X, Q = synth.gen_data(1)
    M = synth.rotation(128, synth.seed(1, "rotation"))
    e = synth.medoid(X)
    G = oracle.build_graph(X, 32, 200, 3, M, e, synth.random_graph(len(X), 32, synth.seed(1, "graph")),
                           synth.random_graph(len(X), 32, synth.seed(1, "fill")))
    blocks = oracle.encode(X, G, M)
    say("cfg1 index: N=10000 D=128 R=32, oracle Algorithm 2 graph")
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    return dict(X=X, Q=Q, M=M, G=G, e=e, blocks=blocks, idx=idx)


def _search(idx, Q, k, ef, flags=0):
    ids, dists, st = idx.search(T(Q), k, ef, flags=flags, stats=True)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()


def _assert_same(gpu, orc, ctx):
    gi, gd, gs = gpu
    oi, od, os_ = orc
    bad = np.nonzero((gi != oi).any(axis=1))[0]
    assert bad.size == 0, f"{ctx}: ids differ for queries {bad[:10].tolist()}"
    assert np.array_equal(gd, od), f"{ctx}: distances differ"
    assert np.array_equal(gs[:, :3], os_[:, :3]), f"{ctx}: counters differ"


def test_rotation_bit_exact(cfg1):
    """Rotated queries (Eq. rotation) equal the oracle's fp64 chain bit for bit."""
    idx = cfg1["idx"]
    say("rotate cfg1 queries")
    out = idx.rotate(T(cfg1["Q"])).cpu().numpy()
    assert np.array_equal(out, oracle.rotate(cfg1["M"], cfg1["Q"]))
    Xi, Qi = synth.gen_data(2, n=300, nq=77, ncent=5)
    M2 = synth.rotation(128, 99)
    G2 = synth.knn_graph(Xi, 32, 3)
    idx2 = qg.qg_build_index(T(Xi), T(G2), T(M2), 0)
    out2 = idx2.rotate(T(Qi)).cpu().numpy()
    assert np.array_equal(out2, oracle.rotate(M2, Qi))
    # rows that start 4 bytes past a 16-byte boundary take the one-column-per-lane loads
    buf = torch.zeros(Qi.size + 1, dtype=torch.float32, device=DEV)
    buf[1:] = T(Qi).reshape(-1)
    Qv = buf[1:].view(Qi.shape)
    assert Qv.data_ptr() % 16 == 4
    out3 = idx2.rotate(Qv).cpu().numpy()
    assert np.array_equal(out3, oracle.rotate(M2, Qi))


def test_encode_bit_exact_cfg1(cfg1):
    """Every block (raw vector, codes, factors, ids, padding) equals the oracle's bytes."""
    say("encode cfg1")
    got = cfg1["idx"].blocks().cpu().numpy()
    exp = cfg1["blocks"]
    bad = np.nonzero((got != exp).any(axis=1))[0]
    assert bad.size == 0, f"blocks differ at vertices {bad[:10].tolist()}"


@pytest.mark.parametrize("D,R,cfg", [(96, 32, 5), (960, 64, 3), (768, 32, 4), (128, 64, 1)])
def test_encode_bit_exact_shapes(D, R, cfg):
    X, Q = synth.gen_data(cfg, n=600, nq=20, D=D) if cfg != 4 else synth.gen_data(cfg, n=600, nq=20)
    M = synth.rotation(D, 7)
    G = synth.knn_graph(X, R, 8, n_long=8)
    G[5, 3] = -1  # an empty slot
    say(f"encode D={D} R={R}")
    idx = qg.qg_build_index(T(X), T(G), T(M), synth.medoid(X))
    got = idx.blocks().cpu().numpy()
    assert np.array_equal(got, oracle.encode(X, G, M))
    # the queries' rotation at this width (2 x 2 tiles per wavefront when D > 256; 20 rows: a ragged block)
    assert np.array_equal(idx.rotate(T(Q)).cpu().numpy(), oracle.rotate(M, Q))


def test_estimate_bit_exact(cfg1):
    """FastScan sums S_j are bit-exact integers and the estimates equal the oracle's."""
    rng = np.random.default_rng(3)
    vs = rng.integers(0, 10000, 64).astype(np.int32)
    Q = cfg1["Q"][:64]
    say("estimate cfg1")
    S, est, dist = cfg1["idx"].estimate(T(Q), T(vs))
    S, est, dist = S.cpu().numpy(), est.cpu().numpy(), dist.cpu().numpy()
    qrot = oracle.rotate(cfg1["M"], Q)
    for i in range(64):
        oS, oe, od = oracle.estimate(cfg1["blocks"], 128, 32, Q[i], qrot[i], int(vs[i]))
        assert np.array_equal(S[i], oS)
        assert np.array_equal(est[i], oe)
        assert dist[i] == od


def test_search_parity_cfg1(cfg1):
    """200 queries, k = 10, ef = 64: identical ids, distances and counters."""
    c = cfg1
    say("search cfg1 k=10 ef=64")
    gpu = _search(c["idx"], c["Q"], 10, 64)
    orc = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], 10, 64, with_stats=True)
    _assert_same(gpu, orc, "cfg1")
    gt, _ = synth.ground_truth(c["X"], c["Q"], 10)
    rec = synth.recall(gpu[0], gt, 10)
    say(f"recall@10 = {rec:.4f}")
    # the 16-cluster mixture is isotropic within clusters (high local
    # dimension): on this graph the oracle reaches 0.78 here
    assert rec > 0.7


@pytest.mark.parametrize("k,ef,nq", [(10, 16, 200), (1, 1, 3), (100, 100, 257), (10, 512, 64), (150, 7, 5),
                                     (64, 64, 1), (10, 2048, 8)])
def test_search_parity_sweep(cfg1, k, ef, nq):
    c = cfg1
    Q = np.concatenate([c["Q"], c["Q"] + 0.05])[:nq]
    say(f"search cfg1 k={k} ef={ef} nq={nq}")
    gpu = _search(c["idx"], Q, k, ef)
    orc = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], Q, k, ef, with_stats=True)
    _assert_same(gpu, orc, f"k={k} ef={ef}")


def test_search_overflow_path(cfg1):
    """With a 128-slot on-chip visited set most queries move to the global
    bitset path; results must not change."""
    c = cfg1
    say("search cfg1 overflow path")
    gpu = _search(c["idx"], c["Q"], 10, 64, flags=qg.QG_SEARCH_SMALL_HASH)
    assert gpu[2][:, 3].sum() > 0, "overflow path not taken"
    orc = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], 10, 64, with_stats=True)
    _assert_same(gpu, orc, "overflow")


@pytest.mark.parametrize("D,R,cfg", [(96, 32, 5), (960, 64, 3), (768, 32, 4), (128, 64, 1)])
def test_search_parity_shapes(D, R, cfg):
    X, Q = synth.gen_data(cfg, n=3000, nq=40, D=D) if cfg != 4 else synth.gen_data(cfg, n=3000, nq=40)
    M = synth.rotation(D, 17)
    G = synth.knn_graph(X, R, 18, n_long=8)
    e = synth.medoid(X)
    say(f"search D={D} R={R}")
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    blocks = oracle.encode(X, G, M)
    for k, ef in ((10, 32), (100, 128)):
        gpu = _search(idx, Q, k, ef)
        orc = oracle.search(blocks, D, R, e, M, Q, k, ef, with_stats=True)
        _assert_same(gpu, orc, f"D={D} R={R} k={k} ef={ef}")
        # every LUT layout (bit 0: padded rows, bit 1: int32 entries) gives the same search
        for lut in (0, 2, 3):
            idx.set_launch(4, 3, 0, 1, lut)
            _assert_same(_search(idx, Q, k, ef), orc, f"D={D} R={R} k={k} ef={ef} LUT layout {lut}")
        idx.set_launch(4, 3, 0, 1, 1)
    # the per-query (mixed batch) kernel on the same shape
    ks = np.resize(np.array([10, 100, 1], np.int32), len(Q))
    efs = np.resize(np.array([32, 128, 64], np.int32), len(Q))
    for lut in (1, 3):  # int16 and int32 entries
        idx.set_launch(4, 3, 0, 1, lut)
        mi, md, ms = idx.search_mixed(T(Q), T(ks), T(efs), 100, 128, stats=True)
        torch.cuda.synchronize()
        mi, md, ms = mi.cpu().numpy(), md.cpu().numpy(), ms.cpu().numpy()
        for k, ef in ((10, 32), (100, 128), (1, 64)):
            sel = np.nonzero((ks == k) & (efs == ef))[0]
            oi, od, os_ = oracle.search(blocks, D, R, e, M, Q[sel], k, ef, with_stats=True)
            _assert_same((mi[sel, :k], md[sel, :k], ms[sel]), (oi, od, os_),
                         f"mixed D={D} R={R} k={k} ef={ef} LUT layout {lut}")
            assert (mi[sel, k:] == -1).all()
    idx.set_launch(4, 3, 0, 1, 1)
    # the learned-stop kernel (MLP in LDS) on the same shape, theta set so that some queries stop
    rng = np.random.default_rng(D + R)
    w = ((rng.standard_normal(oracle.LS_PARAMS) * 0.3).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    _, _, _, (_, _, oo, oc) = oracle.search_ls(blocks, D, R, e, M, Q, 10, 64, w=w, theta=np.inf, t_min=4, t_every=2,
                                               max_evals=128)
    outs = np.concatenate([oo[i, :oc[i]] for i in range(len(oc))])
    theta = float(np.quantile(outs, 0.7))
    si, sd, ss, _ = idx.search_stop(T(Q), 10, 64, torch.from_numpy(w.view(np.int16)).to(DEV), theta=theta, t_min=4,
                                    t_every=2, stats=True)
    torch.cuda.synchronize()
    oi, od, os_, _ = oracle.search_ls(blocks, D, R, e, M, Q, 10, 64, w=w, theta=theta, t_min=4, t_every=2)
    _assert_same((si.cpu().numpy(), sd.cpu().numpy(), ss.cpu().numpy()), (oi, od, os_), f"stop D={D} R={R}")


def test_search_parity_algorithm2_graph():
    """Same bar on a graph built by the oracle's Algorithm 2 (exact degree R)."""
    X, Q = synth.gen_data(1, n=2000, nq=50)
    M = synth.rotation(128, 5)
    e = synth.medoid(X)
    G = oracle.build_graph(X, 32, 64, 2, M, e, synth.random_graph(2000, 32, 6), synth.random_graph(2000, 32, 7))
    say("search on an Algorithm 2 graph")
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    blocks = oracle.encode(X, G, M)
    gpu = _search(idx, Q, 10, 48)
    orc = oracle.search(blocks, 128, 32, e, M, Q, 10, 48, with_stats=True)
    _assert_same(gpu, orc, "alg2 graph")


def test_file_roundtrip(cfg1, tmp_path):
    """An oracle-written file loads and searches identically; the library's own
    file is byte-identical to the oracle's."""
    c = cfg1
    p1 = str(tmp_path / "oracle.qgi")
    oracle.write_index(p1, c["blocks"], 128, 32, c["e"], c["M"])
    say("load oracle-written index")
    idx = qg.qg_load_index(p1)
    gpu = _search(idx, c["Q"][:50], 10, 32)
    orc = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], c["Q"][:50], 10, 32, with_stats=True)
    _assert_same(gpu, orc, "loaded")
    p2 = str(tmp_path / "lib.qgi")
    c["idx"].save(p2)
    assert open(p1, "rb").read() == open(p2, "rb").read()
    idx.free()


def test_bad_inputs(cfg1, tmp_path):
    c = cfg1
    idx = c["idx"]
    Qd = T(c["Q"][:4])
    ids = torch.empty((4, 10), dtype=torch.int32, device=DEV)
    d = torch.empty((4, 10), dtype=torch.float32, device=DEV)
    for k, ef, code in ((0, 10, qg.QG_EINVAL), (10, 0, qg.QG_EINVAL), (10, 4096, qg.QG_EUNSUPPORTED),
                        (2000, 10, qg.QG_EUNSUPPORTED)):
        with pytest.raises(qg.QGError) as ex:
            qg._check(qg.lib().qg_search(idx.handle, qg._dev(Qd, torch.float32, "q"), 4, k, ef,
                                         qg._dev(ids, torch.int32, "i"), qg._dev(d, torch.float32, "d")))
        assert ex.value.code == code
    assert qg.lib().qg_search(idx.handle, None, 0, 10, 10, None, None) == qg.QG_OK  # nq = 0: no-op
    assert qg.lib().qg_search(idx.handle, None, 4, 10, 10, None, None) == qg.QG_EINVAL
    G = c["G"].copy()
    G[7, 2] = 10000  # out of range
    with pytest.raises(qg.QGError) as ex:
        qg.qg_build_index(T(c["X"]), T(G), T(c["M"]), c["e"])
    assert ex.value.code == qg.QG_EINVAL
    p = str(tmp_path / "x.qgi")
    oracle.write_index(p, c["blocks"][:100].copy(), 128, 32, 0, c["M"])
    raw = bytearray(open(p, "rb").read())
    raw[-5] ^= 0xFF
    open(p, "wb").write(bytes(raw))
    with pytest.raises(qg.QGError) as ex:
        qg.qg_load_index(p)
    assert ex.value.code == qg.QG_EFORMAT
    open(p, "wb").write(bytes(raw[:5000]))
    with pytest.raises(qg.QGError) as ex:
        qg.qg_load_index(p)
    assert ex.value.code == qg.QG_EFORMAT
    with pytest.raises(qg.QGError) as ex:
        qg.qg_load_index(str(tmp_path / "missing.qgi"))
    assert ex.value.code == qg.QG_EIO


def test_deterministic_batch_independent_and_stream(cfg1):
    c = cfg1
    say("determinism")
    a = _search(c["idx"], c["Q"], 10, 48)
    b = _search(c["idx"], c["Q"], 10, 48)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    for i in (0, 77, 199):
        s = _search(c["idx"], c["Q"][i:i + 1], 10, 48)
        assert np.array_equal(s[0][0], a[0][i]) and np.array_equal(s[1][0], a[1][i])
    st = torch.cuda.Stream()
    c["idx"].set_stream(st)
    with torch.cuda.stream(st):
        Qd = T(c["Q"])
        ids, dists = c["idx"].search(Qd, 10, 48)
    st.synchronize()
    c["idx"].set_stream(None)
    assert np.array_equal(ids.cpu().numpy(), a[0])


@pytest.mark.parametrize("k,ef", [(1, 1), (10, 5), (10, 48), (10, 64), (10, 65), (100, 100), (64, 128), (10, 129)])
def test_beam_storage_parity(cfg1, k, ef):
    """Beams of at most 128 entries run with the beam in registers (one or two
    words per lane, the pipelined loop) unless QG_SEARCH_LDS_BEAM keeps it in
    LDS; both must equal the oracle in ids, distances and counters, at the
    edges of each storage (1, 64, 65, 128, 129 entries)."""
    c = cfg1
    Q = np.concatenate([c["Q"], c["Q"] + 0.05])
    say(f"beam storage k={k} ef={ef}")
    orc = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], Q, k, ef, with_stats=True)
    _assert_same(_search(c["idx"], Q, k, ef), orc, f"registers k={k} ef={ef}")
    _assert_same(_search(c["idx"], Q, k, ef, flags=qg.QG_SEARCH_LDS_BEAM), orc, f"LDS k={k} ef={ef}")


def test_beam_storage_mixed_and_stop(cfg1):
    """The mixed-batch, stop-only and mixed-with-stop kernels also run with the
    register beam below 129 entries; each row equals the oracle's search (or
    stopped search) at its own k and ef, with either storage."""
    c = cfg1
    rng = np.random.default_rng(41)
    Q = np.concatenate([c["Q"], c["Q"] + 0.05])
    n = len(Q)
    ks = rng.choice([1, 10, 20], n).astype(np.int32)
    efs = rng.choice([8, 40, 64, 100], n).astype(np.int32)
    w = ((rng.standard_normal(qg.QG_STOP_MLP_PARAMS) * 0.3).astype(np.float32).view(np.uint32) >> 16)
    w = w.astype(np.uint16)
    wd = torch.from_numpy(w.view(np.int16)).to(DEV)
    _, _, _, (_, _, oo, oc) = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], Q, 10, 64, w=w, theta=np.inf,
                                               t_min=4, t_every=2, max_evals=128)
    theta = float(np.quantile(np.concatenate([oo[i, :oc[i]] for i in range(n)]), 0.7))
    say(f"beam storage: mixed and stop kernels, theta={theta:.4f}")
    for flags in (0, qg.QG_SEARCH_LDS_BEAM):
        gi, gd, gs = c["idx"].search_mixed(T(Q), T(ks), T(efs), k_max=20, ef_max=100, flags=flags, stats=True)
        si, sd, ss, _ = c["idx"].search_stop(T(Q), 10, 64, wd, theta=theta, t_min=4, t_every=2, flags=flags,
                                              stats=True)
        mi, md, ms_ = c["idx"].search_mixed_stop(T(Q), T(ks), T(efs), wd, theta, t_min=4, t_every=2, k_max=20,
                                                 ef_max=100, flags=flags, stats=True)
        torch.cuda.synchronize()
        gi, gd, gs = gi.cpu().numpy(), gd.cpu().numpy(), gs.cpu().numpy()
        mi, md, ms_ = mi.cpu().numpy(), md.cpu().numpy(), ms_.cpu().numpy()
        oi, od, ost, _ = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], Q, 10, 64, w=w, theta=theta,
                                          t_min=4, t_every=2)
        _assert_same((si.cpu().numpy(), sd.cpu().numpy(), ss.cpu().numpy()), (oi, od, ost), f"stop flags={flags}")
        for k, ef in set(zip(ks.tolist(), efs.tolist())):
            sel = np.nonzero((ks == k) & (efs == ef))[0]
            o = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], Q[sel], k, ef, with_stats=True)
            _assert_same((gi[sel, :k], gd[sel, :k], gs[sel]), o, f"mixed k={k} ef={ef} flags={flags}")
            o2 = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], Q[sel], k, ef, w=w, theta=theta, t_min=4,
                                  t_every=2)
            _assert_same((mi[sel, :k], md[sel, :k], ms_[sel]), o2[:3], f"mixed stop k={k} ef={ef} flags={flags}")

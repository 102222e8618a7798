"""The "w/o ME" ablation (Sec. 4.2.3) on the device, through the C ABI: a
vertex enters the beam only on its first estimate.

Bar: ids identical, distances bit-equal and counters equal to the oracle's
search with its NO_ME flag, on the on-chip set and on the overflow path.
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


@pytest.fixture(scope="module")
def cfg1():
    X, Q = synth.gen_data(1)
    M = synth.rotation(128, synth.seed(1, "rotation"))
    G = synth.knn_graph(X, 32, synth.seed(1, "long"))
    e = synth.medoid(X)
    blocks = oracle.encode(X, G, M)
    say("cfg1 index: N=10000 D=128 R=32")
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    return dict(X=X, Q=Q, M=M, G=G, e=e, blocks=blocks, idx=idx)


def _check(idx, blocks, D, R, e, M, Q, k, ef, flags, ctx):
    ids, dists, st = idx.search(T(Q), k, ef, flags=flags, stats=True)
    torch.cuda.synchronize()
    gi, gd, gs = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    oi, od, os_ = oracle.search(blocks, D, R, e, M, Q, k, ef, flags=oracle.NO_ME, with_stats=True)
    bad = np.nonzero((gi != oi).any(axis=1))[0]
    assert bad.size == 0, f"{ctx}: ids differ for queries {bad[:10].tolist()}"
    assert np.array_equal(gd, od), f"{ctx}: distances differ"
    assert np.array_equal(gs[:, :3], os_[:, :3]), f"{ctx}: counters differ"
    # each vertex enters the beam once, so every pop is an expansion
    assert np.array_equal(gs[:, 0], gs[:, 1]), f"{ctx}: a pop met a visited vertex"
    return gs


@pytest.mark.parametrize("k,ef,nq", [(10, 40, 200), (1, 1, 3), (100, 100, 64), (10, 512, 32), (64, 2048, 4)])
def test_no_me_equals_oracle(cfg1, k, ef, nq):
    c = cfg1
    Q = np.concatenate([c["Q"], c["Q"] + 0.05])[:nq]
    say(f"w/o ME cfg1 k={k} ef={ef} nq={nq}")
    _check(c["idx"], c["blocks"], 128, 32, c["e"], c["M"], Q, k, ef, qg.QG_SEARCH_NO_ME, f"k={k} ef={ef}")


def test_no_me_overflow_path(cfg1):
    """A 128-slot on-chip set fills after a few expansions: the queries finish
    on the global bitset, with the same results."""
    c = cfg1
    say("w/o ME cfg1 overflow path")
    gs = _check(c["idx"], c["blocks"], 128, 32, c["e"], c["M"], c["Q"], 10, 64,
                qg.QG_SEARCH_NO_ME | qg.QG_SEARCH_SMALL_HASH, "overflow")
    assert gs[:, 3].sum() > 0, "overflow path not taken"


def test_no_me_differs_from_me(cfg1):
    """The ablation changes the search: fewer candidates are appended than
    with multiple estimates, on the same queries."""
    c = cfg1
    Qd = T(c["Q"])
    _, _, s_me = c["idx"].search(Qd, 10, 64, stats=True)
    _, _, s_no = c["idx"].search(Qd, 10, 64, flags=qg.QG_SEARCH_NO_ME, stats=True)
    torch.cuda.synchronize()
    assert s_no[:, 2].sum().item() < s_me[:, 2].sum().item()


@pytest.mark.parametrize("D,R,cfg", [(96, 32, 5), (960, 64, 3), (128, 64, 1)])
def test_no_me_shapes(D, R, cfg):
    X, Q = synth.gen_data(cfg, n=3000, nq=40, D=D)
    M = synth.rotation(D, 17)
    G = synth.knn_graph(X, R, 18, n_long=8)
    e = synth.medoid(X)
    say(f"w/o ME D={D} R={R}")
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    blocks = oracle.encode(X, G, M)
    for k, ef in ((10, 32), (100, 128)):
        _check(idx, blocks, D, R, e, M, Q, k, ef, qg.QG_SEARCH_NO_ME, f"D={D} R={R} k={k} ef={ef}")


def test_no_me_only_plain_search(cfg1):
    c = cfg1
    Qd = T(c["Q"][:4])
    k = T(np.full(4, 10, np.int32))
    with pytest.raises(qg.QGError) as ex:
        c["idx"].search_mixed(Qd, k, k, 10, 10, flags=qg.QG_SEARCH_NO_ME)
    assert ex.value.code == qg.QG_EUNSUPPORTED
    with pytest.raises(qg.QGError) as ex:
        c["idx"].search_stop(Qd, 10, 10, None, trace_max=2, flags=qg.QG_SEARCH_NO_ME)
    assert ex.value.code == qg.QG_EUNSUPPORTED


def test_self_edges_and_empty_slots():
    """A graph whose lists point at their own vertex and hold -1 slots: both
    searches (with and without multiple estimates) equal the oracle's.  A list
    that repeats an id is refused at build time, before any kernel runs."""
    X, Q = synth.gen_data(1, n=2000, nq=60)
    M = synth.rotation(128, 23)
    G = synth.knn_graph(X, 32, 24, n_long=4)
    rng = np.random.default_rng(25)
    n = len(X)
    G[rng.choice(n, 200, replace=False), 5] = -1
    sl = rng.choice(n, 200, replace=False)
    G[sl, 7] = sl  # self edges
    for row in G:  # the self edges above must not repeat an id of their list
        r = row[row >= 0]
        assert len(np.unique(r)) == len(r)
    e = synth.medoid(X)
    say("self edges and empty slots: N=2000 D=128 R=32")
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    blocks = oracle.encode(X, G, M)
    assert np.array_equal(idx.blocks().cpu().numpy(), blocks)
    for flags, oflags in ((0, 0), (qg.QG_SEARCH_NO_ME, oracle.NO_ME)):
        for k, ef in ((10, 40), (32, 200)):
            ids, dists, st = idx.search(T(Q), k, ef, flags=flags, stats=True)
            torch.cuda.synchronize()
            oi, od, os_ = oracle.search(blocks, 128, 32, e, M, Q, k, ef, flags=oflags, with_stats=True)
            ctx = f"flags={flags} k={k} ef={ef}"
            assert np.array_equal(ids.cpu().numpy(), oi), ctx
            assert np.array_equal(dists.cpu().numpy(), od), ctx
            assert np.array_equal(st.cpu().numpy()[:, :3], os_[:, :3]), ctx
    G2 = G.copy()
    G2[11, 9] = G2[11, 3] if G2[11, 3] >= 0 else G2[11, 4]
    with pytest.raises(qg.QGError) as ex:
        qg.qg_build_index(T(X), T(G2), T(M), e)
    assert ex.value.code == qg.QG_EINVAL

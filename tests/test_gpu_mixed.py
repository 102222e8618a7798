"""One launch with a result count and beam size per query, and search calls
captured into HIP graphs (through the C ABI).

Bar: every query of a mixed batch returns exactly what the oracle returns for
that query with its own k and ef (ids, distances bit-equal, counters equal),
padded to the batch's row width; rejected (k, ef) give an all-padding row.
Graph replays, with other device work between them, equal the eager results.
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


@pytest.fixture(scope="module")
def cfg1():
    X, Q = synth.gen_data(1)
    M = synth.rotation(128, synth.seed(1, "rotation"))
    G = synth.knn_graph(X, 32, synth.seed(1, "long"))
    e = synth.medoid(X)
    blocks = oracle.encode(X, G, M)
    print("cfg1 index: N=10000 D=128 R=32", flush=True)
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    return dict(X=X, Q=Q, M=M, G=G, e=e, blocks=blocks, idx=idx)


def _oracle_rows(c, Q, ks, efs, k_max):
    ids = np.full((len(Q), k_max), -1, np.int32)
    d = np.full((len(Q), k_max), np.inf, np.float32)
    st = np.zeros((len(Q), 4), np.int64)
    for k, ef in sorted(set(zip(ks.tolist(), efs.tolist()))):
        sel = np.nonzero((ks == k) & (efs == ef))[0]
        oi, od, os_ = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], Q[sel], k, ef, with_stats=True)
        ids[sel, :k], d[sel, :k], st[sel] = oi, od, os_
    return ids, d, st


@pytest.mark.parametrize("seed,nq", [(0, 200), (1, 37), (2, 1)])
def test_mixed_batch_equals_oracle_per_query(cfg1, seed, nq):
    c = cfg1
    rng = np.random.default_rng(seed)
    Q = np.concatenate([c["Q"], c["Q"] + 0.05])[:nq] if nq <= 400 else None
    ks = rng.choice([1, 3, 10, 17, 64], nq).astype(np.int32)
    efs = rng.choice([1, 4, 16, 40, 96, 200], nq).astype(np.int32)
    k_max, ef_max = 64, 256
    print(f"mixed seed={seed} nq={nq}", flush=True)
    ids, d, st = c["idx"].search_mixed(T(Q), T(ks), T(efs), k_max, ef_max, stats=True)
    torch.cuda.synchronize()
    oi, od, os_ = _oracle_rows(c, Q, ks, efs, k_max)
    gi, gd, gs = ids.cpu().numpy(), d.cpu().numpy(), st.cpu().numpy()
    bad = np.nonzero((gi != oi).any(axis=1))[0]
    assert bad.size == 0, f"ids differ for queries {bad[:10].tolist()}"
    assert np.array_equal(gd, od)
    assert np.array_equal(gs[:, :3], os_[:, :3])


def _stop_model(c, seed=5, t_min=4, t_every=2):
    """A random bf16 stop model and a theta at which about a third of the evaluation points stop."""
    rng = np.random.default_rng(seed)
    w = ((rng.standard_normal(oracle.LS_PARAMS) * 0.3).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    _, _, _, (_, _, oo, oc) = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], c["Q"][:64], 10, 64, w=w,
                                               theta=np.inf, t_min=t_min, t_every=t_every, max_evals=128)
    outs = np.concatenate([oo[i, :oc[i]] for i in range(len(oc))])
    return w, float(np.quantile(outs, 0.7))


def test_mixed_stop_equals_oracle_per_query(cfg1):
    """A mixed batch with the learned stop: every query equals the oracle's
    stopped search for that query with its own k and ef (shared model, theta,
    t_min and t_every)."""
    c = cfg1
    rng = np.random.default_rng(7)
    nq = 150
    Q = c["Q"][:nq]
    ks = rng.choice([1, 10, 33], nq).astype(np.int32)
    efs = rng.choice([16, 64, 160], nq).astype(np.int32)
    w, theta = _stop_model(c)
    wd = torch.from_numpy(w.view(np.int16)).to(DEV)
    ids, d, st = c["idx"].search_mixed_stop(T(Q), T(ks), T(efs), wd, theta, t_min=4, t_every=2, k_max=33,
                                            ef_max=160, stats=True)
    torch.cuda.synchronize()
    gi, gd, gs = ids.cpu().numpy(), d.cpu().numpy(), st.cpu().numpy()
    stopped = 0
    for k, ef in sorted(set(zip(ks.tolist(), efs.tolist()))):
        sel = np.nonzero((ks == k) & (efs == ef))[0]
        oi, od, os_, _ = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], Q[sel], k, ef, w=w, theta=theta,
                                          t_min=4, t_every=2)
        assert np.array_equal(gi[sel, :k], oi) and np.array_equal(gd[sel, :k], od), f"k={k} ef={ef}"
        assert np.array_equal(gs[sel, :3], os_[:, :3]), f"counters k={k} ef={ef}"
        assert (gi[sel, k:] == -1).all()
        full = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], Q[sel], k, ef, with_stats=True)[2]
        stopped += int((os_[:, 0] < full[:, 0]).sum())
    assert stopped > 0, "theta stopped no query early"


def test_mixed_stop_argument_errors(cfg1):
    c = cfg1
    Qd = T(c["Q"][:4])
    k = T(np.full(4, 10, np.int32))
    ef = T(np.full(4, 64, np.int32))
    with pytest.raises(ValueError):
        c["idx"].search_mixed_stop(Qd, k, ef, None, 0.0)
    lib = qg.lib()
    assert lib.qg_search_mixed_stop(c["idx"].handle, None, 0, None, None, 10, 10, 0, None, None, None, None) == -1


def test_mixed_uniform_equals_plain_search(cfg1):
    c = cfg1
    Qd = T(c["Q"])
    nq = Qd.shape[0]
    ids, d, st = c["idx"].search(Qd, 10, 64, stats=True)
    k = torch.full((nq,), 10, dtype=torch.int32, device=DEV)
    ef = torch.full((nq,), 64, dtype=torch.int32, device=DEV)
    mi, md, ms = c["idx"].search_mixed(Qd, k, ef, stats=True)
    torch.cuda.synchronize()
    assert torch.equal(ids, mi) and torch.equal(d, md) and torch.equal(st, ms)


def test_mixed_rejects_out_of_range_rows(cfg1):
    c = cfg1
    Q = c["Q"][:6]
    ks = np.array([10, 0, 10, 65, 5, -3], np.int32)
    efs = np.array([32, 32, 0, 32, 300, 32], np.int32)
    ids, d, st = c["idx"].search_mixed(T(Q), T(ks), T(efs), 64, 256, stats=True)
    torch.cuda.synchronize()
    gi, gd, gs = ids.cpu().numpy(), d.cpu().numpy(), st.cpu().numpy()
    for q in (1, 2, 3, 4, 5):
        assert (gi[q] == -1).all() and np.isinf(gd[q]).all() and gs[q].tolist() == [0, 0, 0, -1]
    oi, od = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], Q[:1], 10, 32)
    assert np.array_equal(gi[0, :10], oi[0]) and (gi[0, 10:] == -1).all() and gs[0, 3] == 0


def test_mixed_argument_errors(cfg1):
    idx = cfg1["idx"]
    Qd = T(cfg1["Q"][:4])
    k = torch.full((4,), 10, dtype=torch.int32, device=DEV)
    with pytest.raises(qg.QGError):
        idx.search_mixed(Qd, k, k, 10, qg.QG_MAX_EF + 1)
    with pytest.raises(qg.QGError):
        idx.search_mixed(Qd, k, k, 0, 10)


def test_graph_capture_replays_equal_eager(cfg1):
    """qg_search and qg_search_mixed recorded into HIP graphs (through torch's
    capture on the library's stream): three replays with other device work
    between them each equal the eager results."""
    c = cfg1
    idx = c["idx"]
    Qd = T(c["Q"])
    nq = Qd.shape[0]
    ks = T(np.resize(np.array([1, 10, 30], np.int32), nq))
    efs = T(np.resize(np.array([64, 16, 128, 40], np.int32), nq))
    ref = idx.search(Qd, 10, 64, stats=True)
    refm = idx.search_mixed(Qd, ks, efs, 30, 128, stats=True)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        idx.search(Qd, 10, 64)  # warm-up on the capture stream
    idx.reserve(nq)  # the scratch the graph will refer to exists before capture
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        idx.set_stream(torch.cuda.current_stream())
        out = idx.search(Qd, 10, 64, stats=True)
        outm = idx.search_mixed(Qd, ks, efs, 30, 128, stats=True)
    idx.set_stream(None)
    torch.cuda.synchronize()
    print("graph captured", flush=True)
    other = T(c["Q"][::-1].copy())
    for rep in range(3):
        idx.search(other, 5, 32)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), f"replay {rep}: uniform search differs"
        for a, b in zip(outm, refm):
            assert torch.equal(a, b), f"replay {rep}: mixed search differs"


@pytest.mark.parametrize("k,ef", [(10, 512), (10, 64)])
def test_autotune_keeps_results(cfg1, k, ef):
    """The tuner only changes the launch shape: results before and after are
    bit-identical (and equal the oracle's)."""
    c = cfg1
    idx = c["idx"]
    Qd = T(c["Q"])
    before = idx.search(Qd, k, ef, stats=True)
    wpb, hf, cw, ms, beam, lut = idx.autotune(Qd, k, ef)
    print(f"autotune k={k} ef={ef}: wpb={wpb} hash factor={hf} cu waves={cw} beam={beam} lut={lut} {ms:.3f} ms",
          flush=True)
    assert wpb in (1, 2, 4, 8) and hf in (2, 3, 4) and cw in (0, 16, 20, 24) and beam in (0, 1) and ms > 0
    assert lut in (0, 1, 2, 3)
    assert ef <= 128 or beam == 1  # larger beams are always in LDS; nothing to choose
    after = idx.search(Qd, k, ef, stats=True)
    torch.cuda.synchronize()
    for a, b in zip(before, after):
        assert torch.equal(a, b)
    oi, od = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], k, ef)
    assert np.array_equal(after[0].cpu().numpy(), oi) and np.array_equal(after[1].cpu().numpy(), od)
    # a shape set by hand: two wavefronts per workgroup, F = 4, at most 16 resident per compute unit
    for beam_hand, lut_hand in ((0, 1), (1, 0), (0, 0), (1, 3), (0, 2), (1, 2)):
        idx.set_launch(2, 4, 16, beam_hand, lut_hand)
        hand = idx.search(Qd, k, ef, stats=True)
        torch.cuda.synchronize()
        for a, b in zip(before, hand):
            assert torch.equal(a, b)
    for bad in ((3, 3, 0, 1), (4, 5, 0, 1), (4, 3, -1, 1), (4, 3, 65, 1), (4, 3, 0, 2), (4, 3, 0, 1, 4), (4, 3, 0, 1, -1)):
        with pytest.raises(qg.QGError):
            idx.set_launch(*bad)
    idx.set_launch(wpb, hf, cw, beam, lut)


def test_autotune_mixed_keeps_results(cfg1):
    """The mixed-batch tuner times the mixed kernel over the same settings and
    only changes the launch shape: the batch's rows still equal the oracle's
    per query, before and after."""
    c = cfg1
    rng = np.random.default_rng(11)
    nq = 200
    ks = rng.choice([1, 10, 100], nq).astype(np.int32)
    efs = rng.choice([16, 48, 160], nq).astype(np.int32)
    Qd, kd, efd = T(c["Q"][:nq]), T(ks), T(efs)
    before = c["idx"].search_mixed(Qd, kd, efd, k_max=100, ef_max=160, stats=True)
    wpb, hf, cw, ms, beam, lut = c["idx"].autotune_mixed(Qd, kd, efd, 100, 160)
    print(f"autotune mixed: wpb={wpb} hash factor={hf} cu waves={cw} beam={beam} {ms:.3f} ms", flush=True)
    assert wpb in (1, 2, 4, 8) and hf in (2, 3, 4) and cw in (0, 16, 20, 24) and beam == 1 and ms > 0
    after = c["idx"].search_mixed(Qd, kd, efd, k_max=100, ef_max=160, stats=True)
    torch.cuda.synchronize()
    for a, b in zip(before, after):
        assert torch.equal(a, b)
    oi, od, ost = _oracle_rows(c, c["Q"][:nq], ks, efs, 100)
    assert np.array_equal(after[0].cpu().numpy(), oi) and np.array_equal(after[1].cpu().numpy(), od)
    assert np.array_equal(after[2].cpu().numpy(), ost)
    with pytest.raises(qg.QGError):  # k_max above the largest result count
        c["idx"].autotune_mixed(Qd, kd, efd, qg.QG_MAX_K + 1, 160)
    c["idx"].set_launch(4, 3, 0, 1)

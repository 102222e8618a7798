"""The serving loop (qg_server_*, through the C ABI): requests with their own
k and ef, batched continuously onto several streams.

Bar: every request's result equals the result of searching that query alone
with its own k and ef (ids and distances bit-equal, which the oracle also
returns); every tag comes back exactly once; a timed open-loop trace reports
sane latencies.
"""
import ctypes

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


def _alone(c, Q, ks, efs, k_max):
    """Each query searched by itself on the device (plain qg_search_ex) and by the oracle."""
    ids = np.full((len(Q), k_max), -1, np.int32)
    d = np.full((len(Q), k_max), np.inf, np.float32)
    for i in range(len(Q)):
        gi, gd = c["idx"].search(T(Q[i:i + 1]), int(ks[i]), int(efs[i]))
        ids[i, :ks[i]], d[i, :ks[i]] = gi.cpu().numpy()[0], gd.cpu().numpy()[0]
    for k, ef in set(zip(ks.tolist(), efs.tolist())):
        sel = np.nonzero((ks == k) & (efs == ef))[0]
        oi, od = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], Q[sel], k, ef)
        assert np.array_equal(ids[sel, :k], oi) and np.array_equal(d[sel, :k], od)
    return ids, d


def _collect(srv, n):
    tags, ids, dists, lat = [], [], [], []
    while sum(len(t) for t in tags) < n:
        t, i, d, l = srv.poll()
        tags.append(t), ids.append(i), dists.append(d), lat.append(l)
    return np.concatenate(tags), np.concatenate(ids), np.concatenate(dists), np.concatenate(lat)


def test_each_result_alone_equals_in_the_mix(cfg1):
    c = cfg1
    rng = np.random.default_rng(5)
    Q = np.concatenate([c["Q"], c["Q"] + 0.03]).astype(np.float32)
    n = len(Q)
    ks = rng.choice([1, 10, 100], n).astype(np.int32)
    efs = rng.choice([16, 64, 200], n).astype(np.int32)
    srv = qg.Server(c["idx"], streams=3, max_batch=64, k_max=100, ef_max=256)
    try:
        order = rng.permutation(n)
        for i in order:
            srv.submit(Q[i], int(ks[i]), int(efs[i]), int(i))
        srv.drain()
        tags, ids, dists, lat = _collect(srv, n)
        st = srv.stats()
    finally:
        srv.close()
    print(f"served {n} requests in {st['batches']} batches (largest {st['largest_batch']})", flush=True)
    assert sorted(tags.tolist()) == list(range(n))
    assert st["submitted"] == st["completed"] == n and 1 <= st["largest_batch"] <= 64
    ref_ids, ref_d = _alone(c, Q, ks, efs, 100)
    assert np.array_equal(ids, ref_ids[tags]) and np.array_equal(dists, ref_d[tags])
    assert (lat > 0).all()


def test_replay_open_loop_trace(cfg1):
    c = cfg1
    rng = np.random.default_rng(9)
    n = 4000
    Q = c["Q"][rng.integers(0, len(c["Q"]), n)].astype(np.float32)
    ks = rng.choice([1, 10], n).astype(np.int32)
    efs = rng.choice([32, 96], n).astype(np.int32)
    arrival = np.cumsum(rng.exponential(1.0 / 50_000, n))  # Poisson, 50k requests/s
    srv = qg.Server(c["idx"], streams=2, max_batch=512, k_max=10, ef_max=96)
    try:
        srv.replay(Q, ks, efs, arrival)
        srv.drain()
        parts = []
        while sum(len(p[0]) for p in parts) < n:
            parts.append(srv.poll(with_batch=True))
        tags, ids, dists, lat, bat = (np.concatenate([p[j] for p in parts]) for j in range(5))
        st = srv.stats()
        rec = srv.batches()
    finally:
        srv.close()
    # the batch records account for every request and batch, in time order
    assert len(rec) == st["batches"] and rec["n"].sum() == n
    assert (rec["t_oldest"] <= rec["t_dispatch"]).all() and (rec["t_dispatch"] <= rec["t_enqueued"]).all()
    assert (rec["t_enqueued"] <= rec["t_done"]).all() and (rec["device_ms"] > 0).all()
    assert set(rec["slot"].tolist()) <= {0, 1}
    assert np.array_equal(np.bincount(bat, minlength=len(rec)), rec["n"])
    assert (ks[tags] <= rec["k_max"][bat]).all() and (efs[tags] <= rec["ef_max"][bat]).all()
    lat_from_rec = rec["t_done"][bat] - rec["t_oldest"][bat]  # the oldest request's latency bounds its batch's
    assert (lat <= lat_from_rec + 1e-9).all()
    p50, p99 = np.percentile(lat, [50, 99])
    print(f"replay 50k/s: p50 {p50 * 1e6:.0f} us, p99 {p99 * 1e6:.0f} us, {st['batches']} batches", flush=True)
    assert sorted(tags.tolist()) == list(range(n))
    assert 0 < p50 <= p99 < 1.0
    for k, ef in ((1, 32), (10, 96)):
        sel = np.nonzero((ks[tags] == k) & (efs[tags] == ef))[0]
        gi, gd = c["idx"].search(T(Q[tags[sel]]), k, ef)
        assert np.array_equal(ids[sel, :k], gi.cpu().numpy()) and np.array_equal(dists[sel, :k], gd.cpu().numpy())


def test_server_with_learned_stop(cfg1):
    """With qg_server_set_stop every result equals that query searched alone
    with the learned stop at its own k and ef."""
    c = cfg1
    rng = np.random.default_rng(21)
    w = ((rng.standard_normal(qg.QG_STOP_MLP_PARAMS) * 0.3).astype(np.float32).view(np.uint32) >> 16)
    wd = torch.from_numpy(w.astype(np.uint16).view(np.int16)).to(DEV)
    theta = 0.5
    n = 300
    sel = rng.integers(0, len(c["Q"]), n)
    ks = rng.choice([1, 10], n).astype(np.int32)
    efs = rng.choice([32, 96], n).astype(np.int32)
    srv = qg.Server(c["idx"], streams=2, max_batch=64, k_max=10, ef_max=96)
    try:
        sp = qg.StopParams()  # no model: refused
        sp.t_min, sp.t_every = 4, 2
        assert qg.lib().qg_server_set_stop(srv._h, ctypes.byref(sp)) == qg.QG_EINVAL
        srv.set_stop(wd, theta, t_min=4, t_every=2)
        for i in range(n):
            srv.submit(c["Q"][sel[i]], int(ks[i]), int(efs[i]), i)
        srv.drain()
        tags, ids, dists, _ = _collect(srv, n)
    finally:
        srv.close()
    for k, ef in ((1, 32), (1, 96), (10, 32), (10, 96)):
        rows = np.nonzero((ks[tags] == k) & (efs[tags] == ef))[0]
        if rows.size == 0:
            continue
        gi, gd, _, _ = c["idx"].search_stop(T(c["Q"][sel[tags[rows]]]), k, ef, wd, theta=theta, t_min=4, t_every=2)
        assert np.array_equal(ids[rows, :k], gi.cpu().numpy()) and np.array_equal(dists[rows, :k], gd.cpu().numpy())


def test_server_argument_errors(cfg1):
    with pytest.raises(qg.QGError):
        qg.Server(cfg1["idx"], streams=0)
    srv = qg.Server(cfg1["idx"], streams=1, max_batch=8, k_max=10, ef_max=64)
    try:
        with pytest.raises(qg.QGError):
            srv.submit(cfg1["Q"][0], 11, 32, 0)
        with pytest.raises(qg.QGError):
            srv.submit(cfg1["Q"][0], 5, 65, 0)
        with pytest.raises(qg.QGError):  # arrival times must not decrease
            srv.replay(cfg1["Q"][:2], np.array([5, 5]), np.array([32, 32]), np.array([0.002, 0.001]))
        srv.submit(cfg1["Q"][0], 5, 64, 7)
        srv.drain()
        tags, ids, _, _ = _collect(srv, 1)
        assert tags.tolist() == [7] and (ids[0, 5:] == -1).all()
    finally:
        srv.close()


def test_trace_outlives_a_timed_out_drain(cfg1):
    """A trace the binding had to convert (float64 queries, int64 k and ef) is
    held by the binding itself.  A drain that times out must keep it alive:
    pending requests still point into its rows, and a second replay refused
    while the first runs must not drop it either.  After a full drain every
    result equals that query searched alone."""
    import gc
    c = cfg1
    rng = np.random.default_rng(31)
    n = 3000
    sel = rng.integers(0, len(c["Q"]), n)
    Q64 = c["Q"][sel].astype(np.float64)  # converted (copied) by the binding
    ks = np.full(n, 10, np.int64)
    efs = np.full(n, 256, np.int64)
    arrival = np.linspace(0.0, 0.02, n)
    srv = qg.Server(c["idx"], streams=2, max_batch=256, k_max=10, ef_max=256)
    try:
        srv.replay(Q64, ks, efs, arrival)
        with pytest.raises(qg.QGError):  # a second replay while the first runs is refused
            srv.replay(Q64[:2], ks[:2], efs[:2], arrival[:2])
        try:
            srv.drain(timeout_s=1e-6)  # the producer finishes first; the searches may still run
        except qg.QGError:
            pass
        del Q64
        gc.collect()
        srv.drain()
        tags, ids, dists, _ = _collect(srv, n)
    finally:
        srv.close()
    assert sorted(tags.tolist()) == list(range(n))
    gi, gd = c["idx"].search(T(c["Q"][sel[tags]]), 10, 256)
    assert np.array_equal(ids, gi.cpu().numpy()) and np.array_equal(dists, gd.cpu().numpy())


def test_target_recall_requests(cfg1):
    """Requests that name a recall target take the beam the recall map gives
    their (k, target); each result equals that query searched alone with it,
    for submitted and for replayed requests.  Unmapped (k, target) pairs are
    refused."""
    c = cfg1
    rng = np.random.default_rng(44)
    n = 300
    sel = rng.integers(0, len(c["Q"]), n)
    ks = rng.choice([1, 10], n).astype(np.int32)
    tg = rng.choice([0.9, 0.95, 0.99], n).astype(np.float32)
    emap = {(1, 0.9): 16, (1, 0.95): 32, (1, 0.99): 64, (10, 0.9): 24, (10, 0.95): 48, (10, 0.99): 96}
    efs = np.array([emap[(int(k), round(float(t), 2))] for k, t in zip(ks, tg)], np.int32)
    srv = qg.Server(c["idx"], streams=2, max_batch=128, k_max=10, ef_max=96)
    try:
        rows = list(emap.items())
        srv.set_recall_map([kk for (kk, _), _ in rows], [t for (_, t), _ in rows], [e for _, e in rows])
        with pytest.raises(qg.QGError):  # no row for k = 5
            srv.submit_target(c["Q"][0], 5, 0.9, 0)
        with pytest.raises(qg.QGError):  # no target above 0.99
            srv.submit_target(c["Q"][0], 10, 0.999, 0)
        with pytest.raises(qg.QGError):  # a beam above the server's bound
            srv.set_recall_map([10], [0.9], [97])
        for i in range(n):
            srv.submit_target(c["Q"][sel[i]], int(ks[i]), float(tg[i]), i)
        srv.drain()
        got_s = _collect(srv, n)
        srv.replay_target(c["Q"][sel], ks, tg, np.linspace(0.0, 0.005, n))
        srv.drain()
        got_r = _collect(srv, n)
    finally:
        srv.close()
    for tags, ids, dists, _ in (got_s, got_r):
        tags = tags.astype(np.int64)
        assert sorted(tags.tolist()) == list(range(n))
        for (k, t), e in emap.items():
            rows_ = np.nonzero((ks[tags] == k) & (efs[tags] == e))[0]
            if rows_.size == 0:
                continue
            gi, gd = c["idx"].search(T(c["Q"][sel[tags[rows_]]]), k, e)
            assert np.array_equal(ids[rows_, :k], gi.cpu().numpy())
            assert np.array_equal(dists[rows_, :k], gd.cpu().numpy())

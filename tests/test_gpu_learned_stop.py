"""Learned stop on the device against the oracle (through the C ABI).

The stop decision compares an fp32 MLP output with theta, so both sides take
it in the same arithmetic order; the bar is the same as for the plain search:
ids, distances, counters, and the traced features, top-k ids and MLP outputs
bit-identical.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_12229_amd import learned_stop, qg  # noqa: E402

DEV = torch.device("cuda:0")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.fixture(scope="module")
def small():
    X, Q = synth.gen_data(2, n=20000, nq=300, ncent=40)
    M = synth.rotation(128, 31)
    G = synth.knn_graph(X, 32, 32)
    e = synth.medoid(X)
    blocks = oracle.encode(X, G, M)
    idx = qg.qg_build_index(T(X), T(G), T(M), e)
    print("learned-stop index: N=20000 D=128 R=32", flush=True)
    return dict(X=X, Q=Q, M=M, G=G, e=e, blocks=blocks, idx=idx)


def _mlp_bits(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    w = (rng.standard_normal(oracle.LS_PARAMS) * scale).astype(np.float32)
    return (w.view(np.uint32) >> 16).astype(np.uint16)


@pytest.mark.parametrize("k,ef,t_min,t_every", [(10, 64, 8, 4), (1, 16, 1, 1), (20, 128, 5, 3)])
def test_trace_parity(small, k, ef, t_min, t_every):
    c = small
    print(f"trace k={k} ef={ef}", flush=True)
    ids, d, st, tr = c["idx"].search_stop(T(c["Q"]), k, ef, None, t_min=t_min, t_every=t_every, trace_max=48,
                                          stats=True)
    torch.cuda.synchronize()
    oi, od, ost, (of, on, oo, oc) = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], k, ef,
                                                     t_min=t_min, t_every=t_every, max_evals=48)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(d.cpu().numpy(), od)
    assert np.array_equal(st.cpu().numpy()[:, :3], ost[:, :3])
    cnt = tr[3].cpu().numpy()
    assert np.array_equal(cnt, oc)
    f, n = tr[0].cpu().numpy(), tr[1].cpu().numpy()
    for i in range(len(cnt)):
        assert np.array_equal(f[i, :cnt[i]], of[i, :cnt[i]]), f"features differ, query {i}"
        assert np.array_equal(n[i, :cnt[i]], on[i, :cnt[i]]), f"trace ids differ, query {i}"


def test_stop_decisions_parity(small):
    """A random bf16 MLP with theta at the median output: some queries stop
    early, some run out; every decision and result matches the oracle."""
    c = small
    w = _mlp_bits(7)
    _, _, _, (_, _, oo, oc) = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], 10, 64, w=w,
                                               theta=np.inf, t_min=6, t_every=2, max_evals=64)
    outs = np.concatenate([oo[i, :oc[i]] for i in range(len(oc))])
    theta = float(np.median(outs))
    wd = torch.from_numpy(w.view(np.int16)).to(DEV)
    print(f"stop parity theta={theta:.4f}", flush=True)
    ids, d, st, tr = c["idx"].search_stop(T(c["Q"]), 10, 64, wd, theta=theta, t_min=6, t_every=2, trace_max=64,
                                          stats=True)
    torch.cuda.synchronize()
    oi, od, ost, (_, _, oo2, oc2) = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], 10, 64, w=w,
                                                     theta=theta, t_min=6, t_every=2, max_evals=64)
    plain = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], 10, 64, with_stats=True)
    early = (ost[:, 0] < plain[2][:, 0]).sum()
    assert 0 < early < len(oc2), "theta should stop some but not all queries early"
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(d.cpu().numpy(), od)
    assert np.array_equal(st.cpu().numpy()[:, :3], ost[:, :3])
    cnt = tr[3].cpu().numpy()
    o = tr[2].cpu().numpy()
    assert np.array_equal(cnt, oc2)
    for i in range(len(cnt)):
        assert np.array_equal(o[i, :cnt[i]], oo2[i, :cnt[i]]), f"MLP outputs differ, query {i}"


@pytest.mark.parametrize("k,ef,t_min,t_every", [(10, 64, 6, 2), (1, 1, 1, 1), (20, 128, 3, 5)])
def test_stop_only_parity(small, k, ef, t_min, t_every):
    """Without a trace the kernel keeps the MLP in LDS (a separate code path);
    ids, distances and counters still match the oracle, and the stop fires for
    some queries."""
    c = small
    w = _mlp_bits(11)
    _, _, _, (_, _, oo, oc) = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], k, ef, w=w,
                                               theta=np.inf, t_min=t_min, t_every=t_every, max_evals=256)
    outs = np.concatenate([oo[i, :oc[i]] for i in range(len(oc))])
    theta = float(np.quantile(outs, 0.7)) if outs.size else 0.0
    wd = torch.from_numpy(w.view(np.int16)).to(DEV)
    print(f"stop-only k={k} ef={ef} theta={theta:.4f}", flush=True)
    ids, d, st, tr = c["idx"].search_stop(T(c["Q"]), k, ef, wd, theta=theta, t_min=t_min, t_every=t_every,
                                          stats=True)
    torch.cuda.synchronize()
    assert tr is None
    oi, od, ost, _ = oracle.search_ls(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], k, ef, w=w, theta=theta,
                                      t_min=t_min, t_every=t_every)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(d.cpu().numpy(), od)
    assert np.array_equal(st.cpu().numpy()[:, :3], ost[:, :3])
    if ef > 1:
        plain = oracle.search(c["blocks"], 128, 32, c["e"], c["M"], c["Q"], k, ef, with_stats=True)
        assert (ost[:, 0] < plain[2][:, 0]).any()


def test_training_pipeline_runs(small):
    """Traces -> labels -> MLP -> bf16 export -> theta: the trained stop cuts
    expansions while keeping recall close to the plain search."""
    c = small
    _, Qtr = synth.gen_data(2, n=1, nq=2000, ncent=40, qseed=synth.seed(2, "train"))
    gt_tr, _ = synth.ground_truth(c["X"], Qtr, 10, device=DEV)
    feat, lab = learned_stop.collect(c["idx"], T(Qtr), T(gt_tr), 10, 96, 8, 4)
    assert feat.shape[0] == lab.shape[0] > 1000 and 0 < lab.mean().item() < 1
    model = learned_stop.train(feat, lab, epochs=4)
    bits = learned_stop.export(model)
    assert bits.dtype == torch.int16 and bits.numel() == qg.QG_STOP_MLP_PARAMS
    gt, _ = synth.ground_truth(c["X"], c["Q"], 10, device=DEV)
    ids, _, st = c["idx"].search(T(c["Q"]), 10, 96, stats=True)
    r_plain = learned_stop.recall_rows(ids, T(gt)).mean().item()
    got = learned_stop.pick_theta(c["idx"], T(c["Q"]), T(gt), bits, 10, 96, 8, 4, target=r_plain - 0.02)
    assert got is not None
    th, r, e_mean = got
    assert e_mean < st[:, 0].float().mean().item()

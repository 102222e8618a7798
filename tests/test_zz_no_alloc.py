"""Allocation-free search entry point (qg_search_noalloc), through the C ABI.

Bar: ids, distances and per-query counters bit-identical to qg_search_ex on
the same inputs, on two calls in a row (the second with a smaller batch and
beam), the overflow path included; a batch past the fixed scratch is refused
with QG_EUNSUPPORTED; a call on a fresh index takes no device memory.
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


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@pytest.fixture(scope="module")
def cfg1():
    X, Q = synth.gen_data(1, nq=3000)
    M = synth.rotation(128, synth.seed(1, "rotation"))
    G = synth.knn_graph(X, 32, synth.seed(1, "long"))
    e = synth.medoid(X)
    print("no-alloc fixture: N=10000 D=128 R=32, 3000 queries", flush=True)
    return dict(X=X, Q=Q, M=M, G=G, e=e, idx=qg.qg_build_index(T(X), T(G), T(M), e))


def _noalloc(index, Qd, k, ef, flags=0):
    nq = Qd.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int32, device=DEV)
    dists = torch.full((nq, k), -7.0, dtype=torch.float32, device=DEV)
    st = torch.full((nq, 4), -7, dtype=torch.int32, device=DEV)
    rc = qg.lib().qg_search_noalloc(index.handle, _p(Qd), nq, k, ef, flags, _p(ids), _p(dists), _p(st))
    return rc, ids, dists, st


def test_noalloc_equals_search_ex_twice(cfg1):
    c = cfg1
    index = c["idx"]
    for nq, k, ef, flags in ((3000, 10, 64, 0), (700, 5, 32, 0), (400, 10, 48, qg.QG_SEARCH_SMALL_HASH),
                             (90, 10, 16, 0)):
        print(f"no-alloc call: nq={nq} k={k} ef={ef} flags={flags}", flush=True)
        Qd = T(c["Q"][:nq])
        rc, ids, dists, st = _noalloc(index, Qd, k, ef, flags)
        assert rc == qg.QG_OK, qg.qg_last_error()
        ref_ids, ref_d, ref_st = index.search(Qd, k, ef, flags=flags, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(ids, ref_ids) and torch.equal(dists, ref_d) and torch.equal(st, ref_st)
        if flags & qg.QG_SEARCH_SMALL_HASH:
            assert (st[:, 3] == 1).any().item()  # some queries finished in the overflow pass
    # and the oracle agrees on a sample of the last call
    blocks = oracle.encode(c["X"], c["G"], c["M"])
    oi, od = oracle.search(blocks, 128, 32, c["e"], c["M"], c["Q"][:90], 10, 16)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(dists.cpu().numpy(), od)


def test_noalloc_refuses_batches_past_the_scratch(cfg1):
    index = cfg1["idx"]
    limit = (qg.QG_NOALLOC_SCRATCH_BYTES - 256) // (4 * 128 + 4)
    Qd = torch.zeros((limit + 1, 128), dtype=torch.float32, device=DEV)
    rc, _, _, _ = _noalloc(index, Qd, 10, 32)
    assert rc == qg.QG_EUNSUPPORTED and "allocation-free limit" in qg.qg_last_error()
    rc, _, _, _ = _noalloc(index, Qd[:0], 10, 32)
    assert rc == qg.QG_OK
    rc, _, _, _ = _noalloc(index, Qd[:4], 0, 32)
    assert rc == qg.QG_EINVAL


def test_noalloc_takes_no_device_memory(cfg1):
    """A fresh index has no query scratch yet; qg_search_ex would allocate
    some for a batch this size, qg_search_noalloc must not."""
    c = cfg1
    fresh = qg.qg_build_index(T(c["X"]), T(c["G"]), T(c["M"]), c["e"])
    nq = 30000
    rng = np.random.default_rng(3)
    Qd = T(c["Q"][rng.integers(0, len(c["Q"]), nq)])
    rc, ids, dists, st = _noalloc(fresh, Qd[:8], 10, 32)  # first use on this index
    torch.cuda.synchronize()
    assert rc == qg.QG_OK
    out = (torch.empty((nq, 10), dtype=torch.int32, device=DEV), torch.empty((nq, 10), dtype=torch.float32, device=DEV))
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    rc = qg.lib().qg_search_noalloc(fresh.handle, _p(Qd), nq, 10, 32, 0, _p(out[0]), _p(out[1]), None)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert rc == qg.QG_OK, qg.qg_last_error()
    assert free0 - free1 < 2 << 20  # qg_search_ex would take 4 * nq * (d + 1) = 15.5 MB here
    ref = c["idx"].search(Qd, 10, 32)
    torch.cuda.synchronize()
    assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1])
    fresh.free()

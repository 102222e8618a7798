"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the passage it pins (SymphonyQG, arXiv 2411.12229).  None of
them re-types an oracle formula and compares it with itself: they use a
hand-derived example, closed forms, brute force on tiny inputs, exact integer
arithmetic, invariants and the estimator's statistics.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_index(N=300, D=64, R=16, seed=7, graph="knn"):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, D)).astype(np.float32)
    M = synth.rotation(D, seed + 1)
    if graph == "knn":
        G = synth.knn_graph(X, R, seed + 2, n_long=4)
    else:
        G = synth.random_graph(N, R, seed + 2)
    e = synth.medoid(X)
    return X, M, G, e


# ------------------------------------------------------------ hand example

def test_hand_example_d8():
    """Worked example derived by hand from Eq. codebook, Eq. normalization,
    Eq. 3.1 and the FastScan LUT (Sec. 2.2) with D = 8, R = 1, M = I."""
    h = json.load(open(os.path.join(GOLDEN, "hand_example_d8.json")))
    D = h["D"]
    X = np.array([h["c"], h["o"]], np.float32)
    G = np.array([[1], [0]], np.int32)
    M = np.eye(D, dtype=np.float32)
    blocks = oracle.encode(X, G, M)
    B = oracle.block_bytes(D, 1)
    assert B == 128
    blk = blocks[0]
    assert blk[4 * D] == h["code_byte"]
    fadd = np.frombuffer(blk[4 * D + 1:4 * D + 5].tobytes(), np.float32)[0]
    fres = np.frombuffer(blk[4 * D + 5:4 * D + 9].tobytes(), np.float32)[0]
    nbr = np.frombuffer(blk[4 * D + 9:4 * D + 13].tobytes(), np.int32)[0]
    assert nbr == 1
    assert fadd == np.float32(h["f_add"])
    assert fres == np.float32(h["f_rescale_num"] / h["f_rescale_den"])
    q = np.array(h["q"], np.float32)
    delta, qs, lut = oracle.query_prep(q)  # M = I: rotated query = query
    assert list(qs) == h["q_s"]
    assert delta == np.float32(h["delta_num"] / h["delta_den"])
    assert list(lut[0]) == h["lut_row0"]
    assert list(lut[1]) == h["lut_row1"]
    S, est, dc = oracle.estimate(blocks, D, 1, q, q, 0)
    assert dc == h["dist_c"]
    assert S[0] == h["S"]
    assert abs(est[0] - h["est_num"] / h["est_den"]) < 1e-5
    assert oracle.exact_dist(q, X[1]) == h["true_dist"]


# ---------------------------------------------------------------- rotation

def test_rotation_orthogonal():
    """M is orthogonal (a random orthogonal P, Eq. codebook): |M^T M - I| <= 1e-6 and |Mx| = |x|."""
    for D in (8, 96, 128):
        M = synth.rotation(D, 11 + D).astype(np.float64)
        assert np.abs(M.T @ M - np.eye(D)).max() <= 1e-6
        x = np.random.default_rng(D).standard_normal(D)
        assert abs(np.linalg.norm(M @ x) - np.linalg.norm(x)) <= 1e-6 * np.linalg.norm(x)


def test_rotate_exact_for_integer_inputs():
    """With M on the 2^-24 grid and integer inputs every product and partial
    sum is an integer multiple of 2^-24 below 2^53, so M x is exact; the
    oracle's output must equal the exact value rounded once to fp32."""
    D = 128
    M = synth.rotation(D, 5)
    X, _ = synth.gen_data(2, n=40, nq=1, ncent=4)
    out = oracle.rotate(M, X)
    n = np.round(M.astype(np.float64) * 2 ** 24).astype(np.int64)
    xi = X.astype(np.int64)
    for r in range(X.shape[0]):
        for i in range(D):
            exact = Fraction(int((n[i] * xi[r]).sum()), 2 ** 24)
            assert out[r, i] == np.float32(float(exact))  # exact < 2^53 units: float() is exact


def test_rotate_close_to_fp64():
    rng = np.random.default_rng(3)
    M = synth.rotation(96, 9)
    X = rng.standard_normal((20, 96)).astype(np.float32)
    ref = X.astype(np.float64) @ M.astype(np.float64).T
    out = oracle.rotate(M, X)
    assert np.abs(out - ref).max() <= 1e-6 * np.abs(ref).max()


# ----------------------------------------------------------- exact distance

def test_exact_distance_integer_inputs_exact():
    """Implicit re-ranking needs |q_r - c|^2 (Sec. 3.1.2); for integer data in
    [0, 255] at D = 128 every partial sum is an integer below 2^24, so the
    fp32 result is exact in any order."""
    X, Q = synth.gen_data(2, n=50, nq=5, ncent=3)
    for q in Q:
        for x in X:
            assert oracle.exact_dist(q, x) == float(((q.astype(np.int64) - x.astype(np.int64)) ** 2).sum())


def test_exact_distance_float_close():
    rng = np.random.default_rng(1)
    for D in (96, 128, 960):
        q = rng.standard_normal(D).astype(np.float32)
        x = rng.standard_normal(D).astype(np.float32)
        ref = ((q.astype(np.float64) - x) ** 2).sum()
        assert abs(oracle.exact_dist(q, x) - ref) <= 4 * D * 2 ** -24 * ref


# ------------------------------------------------------------------ encode

def _block_fields(blk, D, R):
    codes = blk[4 * D:4 * D + R * D // 8].reshape(R, D // 8)
    off = 4 * D + R * D // 8
    fadd = np.frombuffer(blk[off:off + 4 * R].tobytes(), np.float32)
    fres = np.frombuffer(blk[off + 4 * R:off + 8 * R].tobytes(), np.float32)
    nbr = np.frombuffer(blk[off + 8 * R:off + 12 * R].tobytes(), np.int32)
    return codes, fadd, fres, nbr


def test_code_bits_are_nearest_codeword_signs():
    """The RaBitQ code of o w.r.t. the holder c is the nearest bi-valued vector
    to P^{-1} o: bit i is the sign of (M (o_r - c))_i (Eq. codebook, Sec. 3.1.1)."""
    X, M, G, e = _tiny_index()
    N, D = X.shape
    R = G.shape[1]
    blocks = oracle.encode(X, G, M)
    M64 = M.astype(np.float64)
    checked = 0
    for c in range(0, N, 7):
        codes, _, _, nbr = _block_fields(blocks[c], D, R)
        assert (nbr == G[c]).all()
        for j in range(R):
            y = M64 @ (X[G[c, j]].astype(np.float64) - X[c])
            bits = np.unpackbits(codes[j], bitorder="little").astype(bool)
            ok = np.abs(y) > 1e-4  # away from the sign boundary
            assert (bits[ok] == (y[ok] > 0)).all()
            checked += 1
    assert checked > 100


def test_estimator_matches_rabitq_definition():
    """Factors + unquantised query reproduce the RaBitQ estimate written from
    first principles: est = |r|^2 + |q_r-c|^2 - 2|r||q_r-c| <obar,q>/<obar,o>,
    obar = P xbar, xbar = (2b-1)/sqrt(D), o = r/|r|, q = (q_r-c)/|q_r-c|
    (Eq. normalization, Sec. 2.2, Eq. 3.1)."""
    X, M, G, e = _tiny_index()
    N, D = X.shape
    R = G.shape[1]
    blocks = oracle.encode(X, G, M)
    P = M.astype(np.float64).T
    rng = np.random.default_rng(5)
    worst = 0.0
    for c in rng.integers(0, N, 20):
        q = rng.standard_normal(D)
        codes, fadd, fres, nbr = _block_fields(blocks[c], D, R)
        qrot = M.astype(np.float64) @ q
        dc = ((q - X[c]) ** 2).sum()
        for j in range(R):
            b = np.unpackbits(codes[j], bitorder="little").astype(np.float64)
            xbar = (2 * b - 1) / math.sqrt(D)
            obar = P @ xbar
            r = X[nbr[j]].astype(np.float64) - X[c]
            o = r / np.linalg.norm(r)
            qq = (q - X[c]) / math.sqrt(dc)
            direct = (r @ r) + dc - 2 * np.linalg.norm(r) * math.sqrt(dc) * (obar @ qq) / (obar @ o)
            via = fadd[j] + dc + fres[j] * ((2 * b - 1) @ qrot)
            worst = max(worst, abs(via - direct) / (abs(direct) + 1e-9))
    assert worst < 2e-5


def test_obar_o_range_and_mean():
    """<obar,o> lies in [1/sqrt(D), 1]; for a random rotation its mean is
    sqrt(2/pi) ~ 0.798 (E|N(0,1)| for each coordinate) (Sec. 2.2)."""
    X, M, G, e = _tiny_index(N=400, D=128, R=16, graph="random")
    D, R = 128, 16
    blocks = oracle.encode(X, G, M)
    vals = []
    for c in range(X.shape[0]):
        _, _, fres, nbr = _block_fields(blocks[c], D, R)
        for j in range(R):
            rn = np.linalg.norm(X[nbr[j]].astype(np.float64) - X[c])
            vals.append(-2 * rn / (fres[j] * math.sqrt(D)))  # f_rescale = -2|r|/(<obar,o> sqrt D)
    vals = np.array(vals)
    assert vals.min() >= 1 / math.sqrt(D) - 1e-5 and vals.max() <= 1 + 1e-5
    assert abs(vals.mean() - math.sqrt(2 / math.pi)) < 0.01


def test_degenerate_edge_is_exact():
    """A neighbour equal to its holder (r = 0) gets a zero code and factors so
    that its estimate is exactly the holder's distance (the paper leaves the
    0/0 of this degenerate edge open)."""
    rng = np.random.default_rng(2)
    X = rng.standard_normal((5, 64)).astype(np.float32)
    X[4] = X[1]
    G = np.array([[1, 2], [4, 0], [0, 1], [0, 1], [1, 2]], np.int32)
    M = synth.rotation(64, 3)
    blocks = oracle.encode(X, G, M)
    q = rng.standard_normal(64).astype(np.float32)
    qrot = oracle.rotate(M, q)[0]
    S, est, dc = oracle.estimate(blocks, 64, 2, q, qrot, 1)
    assert est[0] == np.float32(dc)  # slot 0 of vertex 1 is vertex 4 == vertex 1


def test_estimate_at_self_is_near_zero():
    """q_r = o_r: the float estimate is 0 up to rounding, the quantised one is
    within the quantisation bound |f_rescale| * Delta * D / 2."""
    X, M, G, e = _tiny_index()
    D, R = X.shape[1], G.shape[1]
    blocks = oracle.encode(X, G, M)
    for c in (0, 17, 123):
        _, fadd, fres, nbr = _block_fields(blocks[c], D, R)
        for j in (0, 5):
            q = X[nbr[j]]
            qrot = oracle.rotate(M, q)[0]
            S, est, dc = oracle.estimate(blocks, D, R, q, qrot, c)
            delta, _, _ = oracle.query_prep(qrot)
            bound = abs(fres[j]) * delta * D / 2 + 1e-3 * (abs(fadd[j]) + dc)
            assert abs(est[j]) <= bound


# ------------------------------------------------------------- LUT / sums

def test_lut_sum_equals_signed_dot():
    """FastScan: summing the per-nibble LUT entries equals the inner product
    of the +-1 code with q_s (Sec. 2.2), checked by brute force."""
    rng = np.random.default_rng(4)
    for D in (8, 96, 128, 960):
        qrot = (rng.standard_normal(D) * rng.uniform(0.1, 10)).astype(np.float32)
        delta, qs, lut = oracle.query_prep(qrot)
        assert np.abs(qs).max() == 127 and np.abs(qs).max() <= 127
        assert np.all(np.abs(delta * qs.astype(np.float64) - qrot) <= delta / 2 * (1 + 1e-5) + 1e-7)
        for _ in range(20):
            bits = rng.integers(0, 2, D)
            nib = bits.reshape(-1, 4) @ np.array([1, 2, 4, 8])
            s_lut = int(lut[np.arange(D // 4), nib].sum())
            assert s_lut == int(((2 * bits - 1) * qs).sum())


def test_zero_query_quantises_to_zero():
    delta, qs, lut = oracle.query_prep(np.zeros(64, np.float32))
    assert delta == 0.0 and not qs.any() and not lut.any()


def test_integer_vs_float_estimator_bound():
    """|Delta*S - sum (2b-1) q'_i| <= Delta*D/2, so the quantised estimate is
    within |f_rescale| * Delta * D / 2 of the unquantised one."""
    X, M, G, e = _tiny_index()
    D, R = X.shape[1], G.shape[1]
    blocks = oracle.encode(X, G, M)
    rng = np.random.default_rng(8)
    for c in rng.integers(0, X.shape[0], 10):
        q = rng.standard_normal(D).astype(np.float32)
        qrot = oracle.rotate(M, q)[0]
        S, est, dc = oracle.estimate(blocks, D, R, q, qrot, int(c))
        delta, _, _ = oracle.query_prep(qrot)
        codes, fadd, fres, nbr = _block_fields(blocks[c], D, R)
        for j in range(R):
            b = np.unpackbits(codes[j], bitorder="little").astype(np.float64)
            fl = fadd[j] + dc + fres[j] * ((2 * b - 1) @ qrot.astype(np.float64))
            assert abs(est[j] - fl) <= abs(fres[j]) * delta * D / 2 + 1e-4 * (abs(fl) + 1)


def test_estimator_unbiased_and_error_scale():
    """RaBitQ's estimator <obar,q>/<obar,o> of <o,q> is unbiased with error of
    order sqrt((1-<obar,o>^2)/<obar,o>^2)/sqrt(D-1) (Sec. 2.2, Sec. 3.1.2).
    Over fresh random rotations z = err/sigma must look standard normal."""
    D = 128
    rng = np.random.default_rng(12)
    zs = []
    for t in range(25):
        M = synth.rotation(D, 1000 + t).astype(np.float64)
        for _ in range(100):
            o = rng.standard_normal(D)
            o /= np.linalg.norm(o)
            qv = 0.6 * o + rng.standard_normal(D) * 0.08
            qv /= np.linalg.norm(qv)
            y = M @ o
            xbar = np.where(y > 0, 1.0, -1.0) / math.sqrt(D)
            oo = xbar @ y
            est = (xbar @ (M @ qv)) / oo
            ip = o @ qv
            sigma = math.sqrt(1 - ip ** 2) * math.sqrt(1 - oo ** 2) / (oo * math.sqrt(D - 1))
            zs.append((est - ip) / sigma)
    zs = np.array(zs)
    assert abs(zs.mean()) < 0.1
    assert abs(zs.std() - 1) < 0.1
    assert (np.abs(zs) > 3).mean() < 0.01


# ------------------------------------------------------------------ search

def test_search_exhaustive_beam_is_brute_force():
    """With ef large enough that nothing is ever truncated, Algorithm 1 visits
    every vertex reachable from the entry, so implicit re-ranking returns the
    exact k nearest neighbours."""
    X, M, G, e = _tiny_index(N=400, D=64, R=16)
    assert synth.reachable(G, e) == 400
    blocks = oracle.encode(X, G, M)
    Q = np.random.default_rng(9).standard_normal((10, 64)).astype(np.float32)
    ids, dists, st = oracle.search(blocks, 64, 16, e, M, Q, 10, 400 * 16, with_stats=True)
    gt, gtd = synth.ground_truth(X, Q, 10)
    assert (ids == gt).all()
    assert (st[:, 0] == 400).all()
    for i in range(10):
        for j in range(10):
            assert dists[i, j] == oracle.exact_dist(Q[i], X[ids[i, j]])


def _textbook_beam_search(X, G, e, q, ef, k):
    """Vanilla greedy beam search of Sec. 2.1, written independently: a beam
    of at most ef vertices keyed by exact distance, each vertex entering once."""
    dist = lambda v: oracle.exact_dist(q, X[v])
    beam = [(dist(e), e)]
    seen = {e}
    visited = set()
    while True:
        cand = [(d, v) for d, v in beam if v not in visited]
        if not cand:
            break
        d, p = min(cand)
        visited.add(p)
        for v in G[p]:
            v = int(v)
            if v < 0 or v in seen:
                continue
            seen.add(v)
            beam.append((dist(v), v))
        beam.sort()
        beam = beam[:ef]
    res = sorted((dist(v), v) for v in visited)[:k]
    return [v for _, v in res], [d for d, _ in res], len(visited)


def test_search_control_flow_equals_textbook_beam_search():
    """Replacing the estimator by the exact distance and letting a vertex enter
    the beam once turns Algorithm 1 into the vanilla search of Sec. 2.1."""
    X, M, G, e = _tiny_index(N=500, D=64, R=16)
    blocks = oracle.encode(X, G, M)
    Q = np.random.default_rng(10).standard_normal((6, 64)).astype(np.float32)
    for ef in (4, 10, 32):
        ids, dists, st = oracle.search(blocks, 64, 16, e, M, Q, 5, ef,
                                       flags=oracle.EXACT_EST | oracle.NO_ME, with_stats=True)
        for i in range(Q.shape[0]):
            tid, td, nvis = _textbook_beam_search(X, G, e, Q[i], ef, 5)
            assert list(ids[i]) == tid
            assert list(dists[i]) == td
            assert st[i, 0] == nvis


def test_search_padding_and_small_ef():
    """k larger than the visited set pads with (-1, inf); ef < k is allowed."""
    X, M, G, e = _tiny_index(N=200, D=64, R=16)
    blocks = oracle.encode(X, G, M)
    q = X[:1] + 0.01
    ids, dists = oracle.search(blocks, 64, 16, e, M, q, 150, 1)
    n_real = int((ids[0] >= 0).sum())
    assert 1 <= n_real < 150
    assert np.isinf(dists[0, n_real:]).all() and (ids[0, n_real:] == -1).all()
    assert (np.diff(dists[0, :n_real]) >= 0).all()


def test_search_deterministic_and_batch_independent():
    """Two runs are identical and a query alone equals the same query in a batch."""
    X, M, G, e = _tiny_index(N=400, D=64, R=16)
    blocks = oracle.encode(X, G, M)
    Q = np.random.default_rng(11).standard_normal((12, 64)).astype(np.float32)
    a = oracle.search(blocks, 64, 16, e, M, Q, 10, 24)
    b = oracle.search(blocks, 64, 16, e, M, Q, 10, 24, nthreads=1)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()
    for i in (0, 5, 11):
        s = oracle.search(blocks, 64, 16, e, M, Q[i:i + 1], 10, 24)
        assert (s[0][0] == a[0][i]).all() and (s[1][0] == a[1][i]).all()


def test_recall_trends_config1():
    """Soft trends: recall rises with the beam size (Sec. 2.1), and at one
    beam size a single estimate per vertex is not far ahead of multiple
    estimates (Sec. 4.2.3 compares the two at equal speed, where multiple
    estimates win; at equal beam the single-estimate beam holds more distinct
    vertices)."""
    X, Q = synth.gen_data(1, n=3000, nq=60)
    M = synth.rotation(128, synth.seed(1, "rotation"))
    G = synth.knn_graph(X, 32, synth.seed(1, "long"))
    e = synth.medoid(X)
    blocks = oracle.encode(X, G, M)
    gt, _ = synth.ground_truth(X, Q, 10)
    rec = [synth.recall(oracle.search(blocks, 128, 32, e, M, Q, 10, ef)[0], gt, 10) for ef in (10, 40, 160)]
    assert rec[0] <= rec[1] + 0.02 <= rec[2] + 0.04
    no_me = synth.recall(oracle.search(blocks, 128, 32, e, M, Q, 10, 40, flags=oracle.NO_ME)[0], gt, 10)
    assert rec[1] >= no_me - 0.02


# ------------------------------------------------------------------- index

def test_build_graph_invariants():
    """Algorithm 2 with refinement: every vertex has exactly R distinct
    non-self out-neighbours (Sec. 3.2.2, Table 5 caption) and every vertex is
    reachable from the entry."""
    X, _ = synth.gen_data(1, n=1500, nq=1)
    N, D, R = 1500, 128, 32
    M = synth.rotation(D, 3)
    e = synth.medoid(X)
    G0 = synth.random_graph(N, R, 4)
    fill = synth.random_graph(N, R, 5)
    G = oracle.build_graph(X, R, 100, 2, M, e, G0, fill)
    assert (G >= 0).all() and (G < N).all()
    assert not (G == np.arange(N)[:, None]).any()
    srt = np.sort(G, axis=1)
    assert not (srt[:, 1:] == srt[:, :-1]).any()
    assert synth.reachable(G, e) == N
    Gn = oracle.build_graph(X, R, 100, 2, M, e, G0, fill, refine=False)
    deg = (Gn >= 0).sum(axis=1)
    assert deg.mean() < R  # the NSG rule alone leaves vertices below R (Table 5)


def test_space_lower_bound_and_file(tmp_path):
    """Index size >= n (32D + 32R + DR) bits (Sec. 3.3); the file carries the
    header fields and an FNV-1a checksum of the payload."""
    import struct
    X, M, G, e = _tiny_index(N=100, D=64, R=16)
    blocks = oracle.encode(X, G, M)
    N, D, R = 100, 64, 16
    assert blocks.nbytes * 8 >= N * (32 * D + 32 * R + D * R)
    p = str(tmp_path / "x.qgi")
    oracle.write_index(p, blocks, D, R, e, M)
    raw = open(p, "rb").read()
    assert raw[:8] == b"QGINDEX1"
    n, d, r, ent = struct.unpack_from("<qiii", raw, 16)
    assert (n, d, r, ent) == (N, D, R, e)
    bb, orot, oblk, payload, cks = struct.unpack_from("<qqqQQ", raw, 40)
    assert bb == oracle.block_bytes(D, R) and len(raw) == 4096 + payload
    assert np.frombuffer(raw[orot:orot + 4 * D * D], np.float32).reshape(D, D).tobytes() == M.tobytes()
    assert raw[oblk:] == blocks.tobytes()
    h = 0xcbf29ce484222325
    for byte in raw[4096:]:
        h = ((h ^ byte) * 0x100000001b3) & (2 ** 64 - 1)
    assert cks == h


# ------------------------------------------------------------ learned stop

def _random_mlp(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    w = (rng.standard_normal(oracle.LS_PARAMS) * scale).astype(np.float32)
    return (w.view(np.uint32) >> 16).astype(np.uint16)  # truncate to bf16 bits


def _bf16(u16):
    return (u16.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def test_ls_mlp_matches_fp64_forward():
    """The stop MLP is 16-64-64-1 with ReLU and the documented parameter
    layout: the oracle's fp32 evaluation matches an independent fp64 forward pass."""
    w = _random_mlp(3)
    p = _bf16(w)
    W1, b1 = p[:1024].reshape(64, 16), p[1024:1088]
    W2, b2 = p[1088:1088 + 4096].reshape(64, 64), p[5184:5248]
    W3, b3 = p[5248:5312], p[5312]
    rng = np.random.default_rng(4)
    for _ in range(20):
        f = rng.uniform(0, 4, 16).astype(np.float32)
        h1 = np.maximum(W1 @ f + b1, 0)
        h2 = np.maximum(W2 @ h1 + b2, 0)
        ref = W3 @ h2 + b3
        assert abs(oracle.ls_mlp(w, f) - ref) <= 1e-4 * (1 + abs(ref))


def test_ls_trace_features_and_limits():
    """Trace features follow their definitions (expansion count, NN fill and
    NN distances relative to the entry, recomputed here from the traced ids),
    theta = +inf never stops and theta = -inf stops at the first evaluation."""
    X, M, G, e = _tiny_index(N=500, D=64, R=16)
    blocks = oracle.encode(X, G, M)
    Q = np.random.default_rng(21).standard_normal((8, 64)).astype(np.float32)
    k, ef, t_min, t_every = 5, 32, 3, 2
    plain = oracle.search(blocks, 64, 16, e, M, Q, k, ef, with_stats=True)
    ids, d, st, (tf, tn, to, tc) = oracle.search_ls(blocks, 64, 16, e, M, Q, k, ef, t_min=t_min, t_every=t_every,
                                                    max_evals=64)
    assert (ids == plain[0]).all() and (st == plain[2]).all()
    de = [oracle.exact_dist(q, X[e]) for q in Q]
    for i in range(Q.shape[0]):
        assert tc[i] == min(64, (st[i, 0] - t_min) // t_every + 1)
        for j in range(tc[i]):
            f = tf[i, j]
            E = t_min + j * t_every
            assert f[0] == np.float32(E) / 64 and f[15] == 1.0
            nn = tn[i, j][tn[i, j] >= 0]
            assert f[2] == np.float32(len(nn)) / np.float32(k)
            dn = [oracle.exact_dist(Q[i], X[v]) for v in nn]
            assert dn == sorted(dn)
            assert f[4] == min(np.float32(8), np.float32(dn[0]) / np.float32(de[i]))
            assert f[5] == min(np.float32(8), np.float32(dn[-1]) / np.float32(de[i]))
            assert np.isnan(to[i, j])
    w = _random_mlp(5)
    never = oracle.search_ls(blocks, 64, 16, e, M, Q, k, ef, w=w, theta=np.inf, t_min=t_min, t_every=t_every)
    assert (never[0] == plain[0]).all() and (never[2] == plain[2]).all()
    first = oracle.search_ls(blocks, 64, 16, e, M, Q, k, ef, w=w, theta=-np.inf, t_min=t_min, t_every=t_every)
    assert (first[2][:, 0] == np.minimum(t_min, plain[2][:, 0])).all()


def test_brute_force_blocks_equal_one_pass(monkeypatch):
    """The torch brute force (ground truth, k-NN graphs) shortlists per block
    of base rows and then over the blocks; with blocks of 700 rows it returns
    exactly what the numpy brute force returns, self-exclusion included."""
    monkeypatch.setattr(synth, "_TOPK_BLOCK", 700)
    X, Q = synth.gen_data(1, n=3000, nq=40)
    a = synth._topk_rows_torch(X, Q, 10, False, "cpu")
    b = synth._topk_rows_np(X, Q, 10)
    assert np.array_equal(a[0], b[0]) and np.allclose(a[1], b[1], rtol=0, atol=1e-9)
    a = synth._topk_rows_torch(X, X[:900], 10, True, "cpu")
    b = synth._topk_rows_np(X, X[:900], 10, exclude_self=True)
    assert np.array_equal(a[0], b[0])

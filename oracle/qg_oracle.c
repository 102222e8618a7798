/*
 * qg_oracle.c -- plain, slow CPU oracle for the SymphonyQG query path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header, table or constant with the HIP
 * path: the two are written independently from the paper (SymphonyQG,
 * arXiv 2411.12229) and agree only through the index byte layout.
 *
 * Every step is written in the paper's order with no blocking or fusion.
 * Floating point that decides an integer (a code bit, a beam ordering) is
 * taken in the same precision as the device kernel (fp32 with one fused
 * multiply-add where stated); everything else is fp64.  The readings taken
 * where the paper is silent are listed next to each function.
 *
 * Index block of one vertex (bytes, all little endian), for dimension D and
 * out-degree R:
 *   raw       f32[D]          the vertex's own vector            (Sec. 3.1.3, data layout)
 *   codes     u8[R][D/8]      neighbour j's 1-bit code, dim i in byte i/8, bit i%8
 *   f_add     f32[R]          per-edge additive factor
 *   f_rescale f32[R]          per-edge scale factor
 *   nbr       i32[R]          neighbour ids (-1 = empty slot)
 *   padding to a multiple of 128 bytes.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QGO_NO_ME 1     /* "w/o ME" ablation: a vertex enters the beam only on its first estimate (Sec. 4.2.3) */
#define QGO_EXACT_EST 2 /* estimator replaced by the exact distance: vanilla greedy beam search (Sec. 2.1) */

/* ------------------------------------------------------------------ layout */

int64_t qgo_block_bytes(int D, int R) {
  int64_t raw = 4LL * D, codes = (int64_t)R * (D / 8), tail = 12LL * R;
  int64_t b = raw + codes + tail;
  return (b + 127) / 128 * 128;
}

static const float *blk_raw(const uint8_t *blk) { return (const float *)blk; }
static const uint8_t *blk_codes(const uint8_t *blk, int D) { return blk + 4 * (int64_t)D; }
static const float *blk_fadd(const uint8_t *blk, int D, int R) {
  return (const float *)(blk + 4 * (int64_t)D + (int64_t)R * (D / 8));
}
static const float *blk_fres(const uint8_t *blk, int D, int R) { return blk_fadd(blk, D, R) + R; }
static const int32_t *blk_nbr(const uint8_t *blk, int D, int R) {
  return (const int32_t *)(blk_fadd(blk, D, R) + 2 * R);
}

/* ---------------------------------------------------------------- rotation */

/* y = M x for each row x of X (Eq. rotation: the code is compared with the
 * inversely rotated vector, M = P^{-1}).  Reading: each output is an fp64
 * fused multiply-add chain over j ascending, started at +0, rounded once to
 * fp32. */
void qgo_rotate(const float *M, int D, const float *X, int64_t n, float *out) {
  for (int64_t r = 0; r < n; ++r) {
    const float *x = X + r * D;
    for (int i = 0; i < D; ++i) {
      double acc = 0.0;
      for (int j = 0; j < D; ++j) acc = fma((double)M[(int64_t)i * D + j], (double)x[j], acc);
      out[r * D + i] = (float)acc;
    }
  }
}

/* ------------------------------------------------------------------ encode */

/* RaBitQ code and factors of the edge c -> o, normalised by the holder c
 * (Sec. 3.1.1: the neighbour's code is computed with the holding vertex as the
 * centre).  With r = o_r - c, y = M r (taken as rot(o) - rot(c), each rounded
 * to fp32), the code bit is [y_i > 0] (nearest codeword, Eq. codebook; a zero
 * coordinate reads as bit 0).  With sum_abs = sum |y_i|:
 *   <obar,o> = sum_abs / (sqrt(D) |r|)          (Sec. 2.2)
 *   <xbar,Mc> = sum_i (2b_i-1) rot(c)_i / sqrt(D)  (Eq. 3.1b, query independent)
 * and substituting both into Eq. normalization and Eq. 3.1 gives
 *   est = f_add + |q_r - c|^2 + f_rescale * (Delta * S)
 *   f_rescale = -2 |r|^2 / sum_abs,  f_add = |r|^2 - f_rescale * xc,
 *   xc = sum_i (2b_i-1) rot(c)_i,
 * where Delta*S approximates sum_i (2b_i-1) (M q_r)_i.  Factors are computed
 * in fp64 and rounded once to fp32.  Reading for the three fp64 sums: dim i
 * goes into partial i mod 64 in ascending i (|r|^2 by fused multiply-add),
 * then the partials are combined by the butterfly p[l] = p[l] + p[l^s],
 * s = 32, ..., 1 (the same order as the exact distance, in fp64).
 * Degenerate edge (sum_abs = 0, e.g. o_r = c): f_rescale = 0, f_add = |r|^2,
 * so the estimate is |r|^2 + |q_r - c|^2. */
static double butterfly64(double *p) {
  double t[64];
  for (int s = 32; s >= 1; s >>= 1) {
    for (int l = 0; l < 64; ++l) t[l] = p[l] + p[l ^ s];
    memcpy(p, t, sizeof t);
  }
  return p[0];
}

static void encode_edge(const float *xo, const float *xc_raw, const float *ro, const float *rc, int D,
                        uint8_t *code, float *fadd, float *fres) {
  double pr[64], pa[64], px[64];
  for (int l = 0; l < 64; ++l) pr[l] = pa[l] = px[l] = 0.0;
  memset(code, 0, (size_t)(D / 8));
  for (int i = 0; i < D; ++i) {
    double d = (double)xo[i] - (double)xc_raw[i];
    pr[i & 63] = fma(d, d, pr[i & 63]);
    float y = ro[i] - rc[i];
    int b = y > 0.0f;
    if (b) code[i / 8] |= (uint8_t)(1u << (i % 8));
    pa[i & 63] += fabs((double)y);
    px[i & 63] += b ? (double)rc[i] : -(double)rc[i];
  }
  double r2 = butterfly64(pr), sum_abs = butterfly64(pa), xc = butterfly64(px);
  if (sum_abs == 0.0) {
    *fres = 0.0f;
    *fadd = (float)r2;
  } else {
    double fr = (-2.0 * r2) / sum_abs;
    double fa = r2 - fr * xc;
    *fres = (float)fr;
    *fadd = (float)fa;
  }
}

/* Build every vertex block from the vectors X[N][D], the graph G[N][R]
 * (-1 = empty slot) and the rotation M (Sec. 3.1.3 data layout; the
 * FastScan data of every vertex that Alg. 2 builds after its last round). */
int qgo_encode(const float *X, int64_t N, int D, const int32_t *G, int R, const float *M, uint8_t *blocks,
               int nthreads) {
  if (D <= 0 || D % 8 || R <= 0 || N <= 0) return -1;
  int64_t B = qgo_block_bytes(D, R);
  float *rot = (float *)malloc(sizeof(float) * (size_t)N * D);
  if (!rot) return -2;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < N; ++v) qgo_rotate(M, D, X + v * D, 1, rot + v * D);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < N; ++c) {
    uint8_t *blk = blocks + c * B;
    memset(blk, 0, (size_t)B);
    memcpy(blk, X + c * D, sizeof(float) * D);
    uint8_t *codes = blk + 4 * (int64_t)D;
    float *fadd = (float *)(blk + 4 * (int64_t)D + (int64_t)R * (D / 8));
    float *fres = fadd + R;
    int32_t *nbr = (int32_t *)(fres + R);
    for (int j = 0; j < R; ++j) {
      int32_t o = G[c * R + j];
      nbr[j] = o;
      if (o < 0) {
        fadd[j] = 0.0f;
        fres[j] = 0.0f;
        continue;
      }
      encode_edge(X + (int64_t)o * D, X + c * D, rot + (int64_t)o * D, rot + c * D, D, codes + (int64_t)j * (D / 8),
                  &fadd[j], &fres[j]);
    }
  }
  free(rot);
  return 0;
}

/* ------------------------------------------------------------ query side */

/* Query quantisation and FastScan LUT (Sec. 2.2 FastScan; Eq. 3.1b: one LUT
 * per query built from M q_r).  Reading: symmetric 8-bit scalar quantisation
 * with levels -127..127, m = max_i |q'_i|, inv = fl32(127/m),
 * q_s[i] = clamp(rint(fl32(q'_i * inv))) (round half to even),
 * Delta = fl32(m / 127).  LUT row k, entry p: sum over the four dims 4k+t of
 * +q_s if bit t of p is set, else -q_s (the +-1 form of the bi-valued code). */
void qgo_query_prep(const float *qrot, int D, float *delta, int32_t *qs, int32_t *lut) {
  float m = 0.0f;
  for (int i = 0; i < D; ++i) {
    float a = fabsf(qrot[i]);
    if (a > m) m = a;
  }
  if (m == 0.0f) {
    *delta = 0.0f;
    for (int i = 0; i < D; ++i) qs[i] = 0;
  } else {
    float inv = 127.0f / m;
    for (int i = 0; i < D; ++i) {
      float v = rintf(qrot[i] * inv);
      if (v > 127.0f) v = 127.0f;
      if (v < -127.0f) v = -127.0f;
      qs[i] = (int32_t)v;
    }
    *delta = m / 127.0f;
  }
  for (int k = 0; k < D / 4; ++k)
    for (int p = 0; p < 16; ++p) {
      int32_t s = 0;
      for (int t = 0; t < 4; ++t) s += ((p >> t) & 1) ? qs[4 * k + t] : -qs[4 * k + t];
      lut[k * 16 + p] = s;
    }
}

/* Exact squared distance |q_r - c|^2 (implicit re-ranking, Sec. 3.1.2).
 * Reading: 64 fp32 partial sums, dim i into partial i mod 64 by a fused
 * multiply-add chain in ascending i, then a butterfly p[l] = p[l] + p[l^s]
 * for s = 32, 16, ..., 1; the result is p[0]. */
float qgo_exact_dist(const float *q, const float *x, int D) {
  float p[64], t[64];
  for (int l = 0; l < 64; ++l) p[l] = 0.0f;
  for (int i = 0; i < D; ++i) {
    float d = q[i] - x[i];
    p[i & 63] = fmaf(d, d, p[i & 63]);
  }
  for (int s = 32; s >= 1; s >>= 1) {
    for (int l = 0; l < 64; ++l) t[l] = p[l] + p[l ^ s];
    memcpy(p, t, sizeof p);
  }
  return p[0];
}

/* FastScan sum for neighbour j of a block: S_j = sum_k LUT[k][nibble_k]
 * (Sec. 2.2); nibble k holds dims 4k..4k+3, dim 4k+t in bit t. */
static int32_t fastscan_sum(const uint8_t *code, int D, const int32_t *lut) {
  int32_t s = 0;
  for (int k = 0; k < D / 4; ++k) {
    int nib = (code[k / 2] >> (4 * (k % 2))) & 15;
    s += lut[k * 16 + nib];
  }
  return s;
}

/* Estimated squared distance of neighbour j (Eq. normalization with Eq. 3.1
 * substituted): est = fl32(f_rescale * fl32(S * Delta) + fl32(f_add + dist_c)),
 * the outer step one fused multiply-add. */
static float estimate(float fres, float fadd, int32_t S, float delta, float dist_c) {
  return fmaf(fres, (float)S * delta, fadd + dist_c);
}

/* Exported for tests: S_j and est_j for every slot of vertex v, given the raw
 * and rotated query. */
void qgo_estimate(const uint8_t *blocks, int D, int R, const float *q, const float *qrot, int32_t v, int32_t *S_out,
                  float *est_out, float *dist_out) {
  int64_t B = qgo_block_bytes(D, R);
  const uint8_t *blk = blocks + (int64_t)v * B;
  float delta;
  int32_t *qs = (int32_t *)malloc(sizeof(int32_t) * D);
  int32_t *lut = (int32_t *)malloc(sizeof(int32_t) * 4 * D);
  qgo_query_prep(qrot, D, &delta, qs, lut);
  float dc = qgo_exact_dist(q, blk_raw(blk), D);
  if (dist_out) *dist_out = dc;
  const uint8_t *codes = blk_codes(blk, D);
  const float *fa = blk_fadd(blk, D, R), *fr = blk_fres(blk, D, R);
  for (int j = 0; j < R; ++j) {
    int32_t S = fastscan_sum(codes + (int64_t)j * (D / 8), D, lut);
    S_out[j] = S;
    est_out[j] = estimate(fr[j], fa[j], S, delta, dc);
  }
  free(qs);
  free(lut);
}

/* --------------------------------------------------------------- search */

/* ------------------------------------------------------- learned stop */

/* Learned early stop (an extension beyond the paper; the paper's Algorithm 1
 * runs until the beam has no unchecked entry).  After the t-th expansion, for
 * t >= t_min with (t - t_min) divisible by t_every, 16 features of the search
 * state feed a 16-64-64-1 ReLU MLP with bf16 parameters and fp32 arithmetic;
 * the search stops when its output exceeds theta.  Canonical arithmetic (the
 * device kernel uses the same order): hidden unit j = fma chain over its
 * inputs in ascending order starting from its bias, then ReLU (x > 0 ? x : 0);
 * output = butterfly sum (p[l] + p[l^s], s = 32 .. 1) of w3[j] * h2[j], plus
 * the output bias.  Parameter layout (bf16 bit patterns): W1[64][16], b1[64],
 * W2[64][64], b2[64], W3[64], b3. */
#define QGO_LS_PARAMS (64 * 16 + 64 + 64 * 64 + 64 + 64 + 1)

typedef struct {
  const uint16_t *w; /* NULL: never stop early */
  float theta;
  int t_min, t_every;
  int max_evals; /* trace capacity per query (0: no trace) */
  float *tr_feat; /* [max_evals][16] */
  int32_t *tr_nn; /* [max_evals][k] */
  float *tr_out;  /* [max_evals] (MLP output, NaN without a model) */
  int32_t *tr_count;
} qgo_ls;

static float bf16f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

static float ratio(float a, float b) { return b > 0.0f ? a / b : 0.0f; }

static float clamp8(float x) { return x < 0.0f ? 0.0f : (x > 8.0f ? 8.0f : x); }

/* Search-state features at an evaluation point.  de: entry distance; nn1,
 * nnk: best and last of NN; bf: estimate of the next beam entry to pop (+inf
 * if none); dp: exact distance of the vertex just expanded; app: neighbours
 * appended by that expansion; since: expansions since NN last changed. */
static void ls_features(float *f, int E, int P, int nnc, int k, int since, float de, float nn1, float nnk, float bf,
                        int size, int ef, float dp, int app, int R) {
  f[0] = (float)E / 64.0f;
  f[1] = (float)P / 64.0f;
  f[2] = (float)nnc / (float)k;
  f[3] = (float)since / 16.0f;
  f[4] = ratio(nn1, de);
  f[5] = ratio(nnk, de);
  f[6] = ratio(bf, nnk);
  f[7] = ratio(bf, nn1);
  f[8] = (float)size / (float)ef;
  f[9] = ratio(dp, nnk);
  f[10] = (float)app / (float)R;
  f[11] = ratio(nnk - nn1, nnk);
  f[12] = (float)ef / 256.0f;
  f[13] = ratio(bf, de);
  f[14] = (float)E / (float)ef;
  f[15] = 1.0f;
  for (int i = 0; i < 16; ++i) f[i] = clamp8(f[i]);
}

static float ls_mlp(const uint16_t *w, const float *f) {
  const uint16_t *W1 = w, *b1 = W1 + 64 * 16, *W2 = b1 + 64, *b2 = W2 + 64 * 64, *W3 = b2 + 64, *b3 = W3 + 64;
  float h1[64], h2[64], p[64], t[64];
  for (int j = 0; j < 64; ++j) {
    float acc = bf16f(b1[j]);
    for (int i = 0; i < 16; ++i) acc = fmaf(bf16f(W1[j * 16 + i]), f[i], acc);
    h1[j] = acc > 0.0f ? acc : 0.0f;
  }
  for (int j = 0; j < 64; ++j) {
    float acc = bf16f(b2[j]);
    for (int i = 0; i < 64; ++i) acc = fmaf(bf16f(W2[j * 64 + i]), h1[i], acc);
    h2[j] = acc > 0.0f ? acc : 0.0f;
  }
  for (int j = 0; j < 64; ++j) p[j] = bf16f(W3[j]) * h2[j];
  for (int sft = 32; sft >= 1; sft >>= 1) {
    for (int l = 0; l < 64; ++l) t[l] = p[l] + p[l ^ sft];
    memcpy(p, t, sizeof p);
  }
  return p[0] + bf16f(b3[0]);
}

float qgo_ls_mlp(const uint16_t *w, const float *f) { return ls_mlp(w, f); }

typedef struct {
  float key;
  int32_t id;
  int checked;
} beam_entry;

/* (key, id) lexicographic order, ascending. */
static int less_kv(float ka, int32_t ia, float kb, int32_t ib) { return ka < kb || (ka == kb && ia < ib); }

/* Algorithm 1 (Querying) with multiple estimates (Sec. 3.1.2) and implicit
 * re-ranking, for one query.  Readings:
 *  - the beam S holds at most ef entries, checked ones included; entries are
 *    ordered by (estimate, id); after each batch of appends S is truncated to
 *    its first ef entries (an old entry precedes a new one with the same key
 *    and id);
 *  - S starts with the entry point keyed by its exact distance; NN starts
 *    empty and receives every vertex whose exact distance is computed;
 *  - a popped entry whose vertex was already visited (a second estimate of
 *    the same vertex) is only marked checked;
 *  - a neighbour is appended unless it has been visited (so a vertex may sit
 *    in S several times with different estimates);
 *  - the loop ends when no unchecked entry remains;
 *  - the answer is the k smallest (distance, id) of NN, padded with (-1, inf).
 * stats (nullable): [expansions, pops, appended, 0]. */
static void search_one(const uint8_t *blocks, int64_t N, int D, int R, int32_t entry, const float *M, const float *q,
                       int k, int ef, int flags, int32_t *ids, float *dists, int64_t *stats, uint8_t *visited,
                       uint8_t *seen, int32_t *touched, const qgo_ls *ls, int64_t qi) {
  int64_t B = qgo_block_bytes(D, R);
  float *qrot = (float *)malloc(sizeof(float) * D);
  int32_t *qs = (int32_t *)malloc(sizeof(int32_t) * D);
  int32_t *lut = (int32_t *)malloc(sizeof(int32_t) * 4 * D);
  beam_entry *S = (beam_entry *)malloc(sizeof(beam_entry) * (size_t)(ef + R + 1));
  beam_entry *merged = (beam_entry *)malloc(sizeof(beam_entry) * (size_t)(ef + R + 1));
  float *nn_d = (float *)malloc(sizeof(float) * (size_t)(k + 1));
  int32_t *nn_i = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
  int64_t ntouched = 0, nseen = 0;
  int32_t *seen_list = (flags & QGO_NO_ME) ? (int32_t *)malloc(sizeof(int32_t) * (size_t)N) : NULL;
  float delta;
  qgo_rotate(M, D, q, 1, qrot);
  qgo_query_prep(qrot, D, &delta, qs, lut);

  int n = 0, nn = 0;
  int64_t expansions = 0, pops = 0, appended = 0;
  int since = 0, nevals = 0;
  const float de = qgo_exact_dist(q, blk_raw(blocks + (int64_t)entry * B), D);
  S[n].key = de;
  S[n].id = entry;
  S[n].checked = 0;
  ++n;
  if (seen) {
    seen[entry] = 1;
    seen_list[nseen++] = entry;
  }
  for (;;) {
    int c = -1;
    for (int i = 0; i < n; ++i)
      if (!S[i].checked) {
        c = i;
        break;
      }
    if (c < 0) break;
    S[c].checked = 1;
    ++pops;
    int32_t p = S[c].id;
    if (visited[p]) continue;
    visited[p] = 1;
    touched[ntouched++] = p;
    ++expansions;
    const uint8_t *blk = blocks + (int64_t)p * B;
    float dp = qgo_exact_dist(q, blk_raw(blk), D);
    /* update NN with (dp, p) */
    ++since;
    if (nn < k || less_kv(dp, p, nn_d[nn - 1], nn_i[nn - 1])) {
      since = 0;
      int pos = nn < k ? nn : k - 1;
      while (pos > 0 && less_kv(dp, p, nn_d[pos - 1], nn_i[pos - 1])) {
        nn_d[pos] = nn_d[pos - 1];
        nn_i[pos] = nn_i[pos - 1];
        --pos;
      }
      nn_d[pos] = dp;
      nn_i[pos] = p;
      if (nn < k) ++nn;
    }
    /* estimate every neighbour and append the unvisited ones */
    const uint8_t *codes = blk_codes(blk, D);
    const float *fa = blk_fadd(blk, D, R), *fr = blk_fres(blk, D, R);
    const int32_t *nb = blk_nbr(blk, D, R);
    int n_before = n;
    int64_t app0 = appended;
    for (int j = 0; j < R; ++j) {
      int32_t o = nb[j];
      if (o < 0 || visited[o]) continue;
      if (seen) {
        if (seen[o]) continue;
        seen[o] = 1;
        seen_list[nseen++] = o;
      }
      float e;
      if (flags & QGO_EXACT_EST)
        e = qgo_exact_dist(q, blk_raw(blocks + (int64_t)o * B), D);
      else
        e = estimate(fr[j], fa[j], fastscan_sum(codes + (int64_t)j * (D / 8), D, lut), delta, dp);
      S[n].key = e;
      S[n].id = o;
      S[n].checked = 0;
      ++n;
      ++appended;
    }
    /* order the appended batch by (key, id), then merge it behind equal old
     * entries and keep the first ef */
    for (int i = n_before + 1; i < n; ++i) {
      beam_entry x = S[i];
      int pos = i;
      while (pos > n_before && less_kv(x.key, x.id, S[pos - 1].key, S[pos - 1].id)) {
        S[pos] = S[pos - 1];
        --pos;
      }
      S[pos] = x;
    }
    if (n > n_before) {
      int a = 0, b = n_before, w = 0;
      while (w < n && w < ef) {
        if (b >= n || (a < n_before && !less_kv(S[b].key, S[b].id, S[a].key, S[a].id)))
          merged[w++] = S[a++];
        else
          merged[w++] = S[b++];
      }
      memcpy(S, merged, sizeof(beam_entry) * (size_t)w);
      n = w;
    }
    /* learned stop: evaluation point after this expansion */
    if (ls && expansions >= ls->t_min && (expansions - ls->t_min) % ls->t_every == 0) {
      float bf = INFINITY;
      for (int i = 0; i < n; ++i)
        if (!S[i].checked) {
          bf = S[i].key;
          break;
        }
      float f[16];
      ls_features(f, (int)expansions, (int)pops, nn, k, since, de, nn_d[0], nn_d[nn - 1], bf, n, ef, dp,
                  (int)(appended - app0), R);
      float out = ls->w ? ls_mlp(ls->w, f) : NAN;
      if (ls->max_evals > 0 && nevals < ls->max_evals) {
        memcpy(ls->tr_feat + (qi * ls->max_evals + nevals) * 16, f, sizeof f);
        for (int i = 0; i < k; ++i) ls->tr_nn[(qi * ls->max_evals + nevals) * k + i] = i < nn ? nn_i[i] : -1;
        ls->tr_out[qi * ls->max_evals + nevals] = out;
      }
      ++nevals;
      if (ls->w && out > ls->theta) break;
    }
    if (n > ef) n = ef;
  }
  for (int i = 0; i < k; ++i) {
    ids[i] = i < nn ? nn_i[i] : -1;
    dists[i] = i < nn ? nn_d[i] : INFINITY;
  }
  if (stats) {
    stats[0] = expansions;
    stats[1] = pops;
    stats[2] = appended;
    stats[3] = 0;
  }
  if (ls && ls->max_evals > 0) ls->tr_count[qi] = nevals < ls->max_evals ? nevals : ls->max_evals;
  for (int64_t i = 0; i < ntouched; ++i) visited[touched[i]] = 0;
  if (seen)
    for (int64_t i = 0; i < nseen; ++i) seen[seen_list[i]] = 0;
  free(seen_list);
  free(qrot);
  free(qs);
  free(lut);
  free(S);
  free(merged);
  free(nn_d);
  free(nn_i);
}

/* Search nq queries Q[nq][D]; ids/dists are [nq][k]; stats [nq][4] or NULL.
 * Queries are independent; OpenMP spreads them over nthreads (0 = default). */
static int search_all(const uint8_t *blocks, int64_t N, int D, int R, int32_t entry, const float *M, const float *Q,
                      int64_t nq, int k, int ef, int flags, int32_t *ids, float *dists, int64_t *stats, int nthreads,
                      const qgo_ls *ls) {
  if (N <= 0 || D <= 0 || D % 8 || R <= 0 || k <= 0 || ef <= 0 || nq < 0 || entry < 0 || entry >= N) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int rc = 0;
#pragma omp parallel
  {
    uint8_t *visited = (uint8_t *)calloc((size_t)N, 1);
    uint8_t *seen = (flags & QGO_NO_ME) ? (uint8_t *)calloc((size_t)N, 1) : NULL;
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    if (!visited || !touched || ((flags & QGO_NO_ME) && !seen)) {
#pragma omp atomic write
      rc = -2;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < nq; ++i)
        search_one(blocks, N, D, R, entry, M, Q + i * D, k, ef, flags, ids + i * k, dists + i * k,
                   stats ? stats + 4 * i : NULL, visited, seen, touched, ls, i);
    }
    free(visited);
    free(seen);
    free(touched);
  }
  return rc;
}

int qgo_search(const uint8_t *blocks, int64_t N, int D, int R, int32_t entry, const float *M, const float *Q,
               int64_t nq, int k, int ef, int flags, int32_t *ids, float *dists, int64_t *stats, int nthreads) {
  return search_all(blocks, N, D, R, entry, M, Q, nq, k, ef, flags, ids, dists, stats, nthreads, NULL);
}

/* Algorithm 1 with the learned stop (w may be NULL: plain search) and an
 * optional trace of the features, NN ids and MLP output at every evaluation
 * point (max_evals per query; tr_* may be NULL when max_evals is 0). */
int qgo_search_ls(const uint8_t *blocks, int64_t N, int D, int R, int32_t entry, const float *M, const float *Q,
                  int64_t nq, int k, int ef, int flags, int32_t *ids, float *dists, int64_t *stats, int nthreads,
                  const uint16_t *w, float theta, int t_min, int t_every, int max_evals, float *tr_feat,
                  int32_t *tr_nn, float *tr_out, int32_t *tr_count) {
  if (t_min < 1 || t_every < 1 || max_evals < 0) return -1;
  qgo_ls ls = {w, theta, t_min, t_every, max_evals, tr_feat, tr_nn, tr_out, tr_count};
  return search_all(blocks, N, D, R, entry, M, Q, nq, k, ef, flags, ids, dists, stats, nthreads, &ls);
}

int qgo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

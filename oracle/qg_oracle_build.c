/*
 * qg_oracle_build.c -- plain CPU oracle for SymphonyQG's index phase
 * (Algorithm 2, Sec. 3.2) and the index file writer.
 *
 * TEST INFRASTRUCTURE ONLY (see qg_oracle.c).  Random numbers the method
 * draws (the initial random graph and the random fill of Sec. 3.2.2's
 * footnote) are passed in as inputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int64_t qgo_block_bytes(int D, int R);
int qgo_encode(const float *X, int64_t N, int D, const int32_t *G, int R, const float *M, uint8_t *blocks,
               int nthreads);
int qgo_search(const uint8_t *blocks, int64_t N, int D, int R, int32_t entry, const float *M, const float *Q,
               int64_t nq, int k, int ef, int flags, int32_t *ids, float *dists, int64_t *stats, int nthreads);

static double dist2(const float *a, const float *b, int D) {
  double s = 0.0;
  for (int i = 0; i < D; ++i) {
    double d = (double)a[i] - (double)b[i];
    s += d * d;
  }
  return s;
}

typedef struct {
  double d;
  int32_t id;
} cand_t;

static int cmp_cand(const void *a, const void *b) {
  const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
  if (x->d < y->d) return -1;
  if (x->d > y->d) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

static int cmp_dbl(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

/* NSG edge selection on candidates sorted by distance to u: scan in order and
 * keep v unless an already kept w is closer to v than u is (Sec. 3.2.1: the
 * rule NSG prunes with), until R are kept.  kept[] receives candidate
 * indices; returns the count. */
static int nsg_prune(const float *X, int D, const cand_t *c, int nc, int R, int *kept) {
  int nk = 0;
  for (int i = 0; i < nc && nk < R; ++i) {
    const float *xv = X + (int64_t)c[i].id * D;
    int occluded = 0;
    for (int a = 0; a < nk && !occluded; ++a)
      if (dist2(X + (int64_t)c[kept[a]].id * D, xv, D) < c[i].d) occluded = 1;
    if (!occluded) kept[nk++] = i;
  }
  return nk;
}

/* Graph refinement (Sec. 3.2.2).  Over the candidates that the NSG rule
 * pruned, a candidate v is pruned at angle threshold theta when some other
 * candidate w closer to u (by (distance, id)) makes an angle below theta with
 * v at u.  The surviving count falls monotonically as theta grows; the
 * largest theta that still leaves need = R - nk survivors is found exactly
 * (the limit of the paper's binary search): v survives iff
 * t_v = max_w cos(w,u,v) <= cos(theta), so cos(theta*) is the need-th
 * smallest t_v.  The nearest `need` survivors are added.  Returns the new
 * count of kept[] (may stay below R when too few candidates exist). */
static int refine(const float *X, int D, int32_t u, const cand_t *c, int nc, int *kept, int nk, int R) {
  int need = R - nk;
  if (need <= 0) return nk;
  const float *xu = X + (int64_t)u * D;
  char *is_kept = (char *)calloc((size_t)nc, 1);
  for (int a = 0; a < nk; ++a) is_kept[kept[a]] = 1;
  int np = 0;
  int *pr = (int *)malloc(sizeof(int) * (size_t)nc);
  double *tv = (double *)malloc(sizeof(double) * (size_t)nc);
  double *du = (double *)malloc(sizeof(double) * (size_t)D);
  double *dw = (double *)malloc(sizeof(double) * (size_t)D);
  for (int i = 0; i < nc; ++i) {
    if (is_kept[i]) continue;
    const float *xv = X + (int64_t)c[i].id * D;
    double nv = 0.0;
    for (int t = 0; t < D; ++t) {
      du[t] = (double)xv[t] - (double)xu[t];
      nv += du[t] * du[t];
    }
    double best = -2.0;
    for (int w = 0; w < i; ++w) { /* candidates are sorted: index < i means closer */
      const float *xw = X + (int64_t)c[w].id * D;
      double nw = 0.0, dot = 0.0;
      for (int t = 0; t < D; ++t) {
        dw[t] = (double)xw[t] - (double)xu[t];
        nw += dw[t] * dw[t];
        dot += dw[t] * du[t];
      }
      double cs = (nv > 0.0 && nw > 0.0) ? dot / (sqrt(nv) * sqrt(nw)) : 1.0;
      if (cs > best) best = cs;
    }
    pr[np] = i;
    tv[np] = best;
    ++np;
  }
  if (np > 0) {
    double *sorted = (double *)malloc(sizeof(double) * (size_t)np);
    memcpy(sorted, tv, sizeof(double) * (size_t)np);
    qsort(sorted, (size_t)np, sizeof(double), cmp_dbl);
    double cstar = sorted[(need <= np ? need : np) - 1];
    free(sorted);
    for (int a = 0; a < np && nk < R; ++a) /* pr[] is in distance order */
      if (tv[a] <= cstar) kept[nk++] = pr[a];
  }
  free(is_kept);
  free(pr);
  free(tv);
  free(du);
  free(dw);
  return nk;
}

/* Breadth-first reachability from the entry point; returns the count reached. */
static int64_t bfs(const int32_t *G, int64_t N, int R, int32_t entry, char *seen, int32_t *queue) {
  memset(seen, 0, (size_t)N);
  int64_t h = 0, t = 0;
  queue[t++] = entry;
  seen[entry] = 1;
  while (h < t) {
    int32_t u = queue[h++];
    for (int j = 0; j < R; ++j) {
      int32_t v = G[(int64_t)u * R + j];
      if (v >= 0 && !seen[v]) {
        seen[v] = 1;
        queue[t++] = v;
      }
    }
  }
  return t;
}

/* Algorithm 2 (Indexing).  G0 is the random initial graph, fill[N][R] the
 * random ids used when a vertex has fewer than R candidates.  Readings:
 *  - candidates of u = the EF nearest results (by exact distance) of
 *    Algorithm 1 run for x_u with beam EF on the current graph, together with
 *    u's current neighbours (the old list is reconsidered, not retained),
 *    minus u itself;
 *  - the graph takes every vertex's new list at once, after all vertices
 *    are pruned;
 *  - refinement (the step of Algorithm 2 after its iterations) runs on the
 *    last iteration's candidates;
 *  - an addition: vertices unreachable from the entry are linked, in rounds,
 *    from the nearest reachable vertex their search finds (its empty slot,
 *    else its farthest edge), since the NSG rule leaves vertices that no list
 *    keeps (in-degree 0) and clustered inputs can leave disconnected parts.
 * stats (nullable): [reachable before repair, repairs made, reachable after].
 * opts: bit 0 = refine; bits 8.. = thread count. */
int qgo_build_graph(const float *X, int64_t N, int D, int R, int EF, int t, const float *M, int32_t entry,
                    const int32_t *G0, const int32_t *fill, int32_t *G, int64_t *stats, int opts) {
  int do_refine = opts & 1, nthreads = opts >> 8;
  if (N <= 1 || D <= 0 || D % 8 || R <= 0 || EF <= 0 || t < 0 || entry < 0 || entry >= N) return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int64_t B = qgo_block_bytes(D, R);
  uint8_t *blocks = (uint8_t *)malloc((size_t)(N * B));
  int32_t *newG = (int32_t *)malloc(sizeof(int32_t) * (size_t)(N * R));
  int cap = EF + R;
  cand_t *cands = (cand_t *)malloc(sizeof(cand_t) * (size_t)(N * cap));
  int *ncand = (int *)calloc((size_t)N, sizeof(int));
  int *nkept = (int *)calloc((size_t)N, sizeof(int));
  int *keptidx = (int *)malloc(sizeof(int) * (size_t)(N * R));
  if (!blocks || !newG || !cands || !ncand || !nkept || !keptidx) return -2;
  memcpy(G, G0, sizeof(int32_t) * (size_t)(N * R));

  for (int it = 0; it < t; ++it) {
    if (qgo_encode(X, N, D, G, R, M, blocks, nthreads) != 0) return -3;
#pragma omp parallel
    {
      int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)EF);
      float *dd = (float *)malloc(sizeof(float) * (size_t)EF);
#pragma omp for schedule(dynamic, 16)
      for (int64_t u = 0; u < N; ++u) {
        const float *xu = X + u * D;
        qgo_search(blocks, N, D, R, entry, M, xu, 1, EF, EF, 0, ids, dd, NULL, 1);
        cand_t *c = cands + u * cap;
        int nc = 0;
        for (int a = 0; a < EF; ++a)
          if (ids[a] >= 0 && ids[a] != u) c[nc++].id = ids[a];
        for (int j = 0; j < R; ++j) {
          int32_t v = G[u * R + j];
          if (v < 0 || v == u) continue;
          int dup = 0;
          for (int a = 0; a < nc && !dup; ++a) dup = c[a].id == v;
          if (!dup) c[nc++].id = v;
        }
        for (int a = 0; a < nc; ++a) c[a].d = dist2(xu, X + (int64_t)c[a].id * D, D);
        qsort(c, (size_t)nc, sizeof(cand_t), cmp_cand);
        int *kept = keptidx + u * R;
        int nk = nsg_prune(X, D, c, nc, R, kept);
        ncand[u] = nc;
        nkept[u] = nk;
        for (int j = 0; j < R; ++j) newG[u * R + j] = j < nk ? c[kept[j]].id : -1;
      }
      free(ids);
      free(dd);
    }
    memcpy(G, newG, sizeof(int32_t) * (size_t)(N * R));
  }

  if (do_refine && t > 0) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < N; ++u) {
      cand_t *c = cands + u * cap;
      int *kept = keptidx + u * R;
      int nk = refine(X, D, (int32_t)u, c, ncand[u], kept, nkept[u], R);
      int32_t *row = G + u * R;
      for (int j = 0; j < R; ++j) row[j] = j < nk ? c[kept[j]].id : -1;
      /* too few candidates: random neighbours (Sec. 3.2.2 footnote) */
      for (int f = 0; nk < R && f < R; ++f) {
        int32_t v = fill[u * R + f];
        if (v < 0 || v == u) continue;
        int dup = 0;
        for (int a = 0; a < nk && !dup; ++a) dup = row[a] == v;
        if (!dup) row[nk++] = v;
      }
    }
  }

  /* Connectivity repair (an addition; Sec. 3.2 has none), in rounds.  A round
   * finds the vertices unreachable from the entry (breadth first).  Each such v
   * runs Algorithm 1 on the current graph (beam EF, EF results) and picks the
   * nearest result that still has a slot not taken by an earlier repair (every
   * result was visited from the entry, hence is reachable).  Then, per picked
   * vertex w in increasing id, its v's in increasing id take w's empty slots
   * (in slot order), then w's edges not taken by a repair, farthest first
   * (fp64, ties to the larger id), while such slots are left.  The next round
   * starts from the new graph, until every vertex is reachable or a round
   * links none. */
  char *seen = (char *)malloc((size_t)N);
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int64_t repairs = 0;
  char *fixed = (char *)calloc((size_t)(N * R), 1); /* edges added by the repair are never overwritten */
  int32_t *unr = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
  int64_t *pick = (int64_t *)malloc(sizeof(int64_t) * (size_t)N); /* (w << 32) | v, sorted below */
  cand_t *slots = (cand_t *)malloc(sizeof(cand_t) * (size_t)R);
  if (stats) stats[0] = bfs(G, N, R, entry, seen, queue);
  for (int round = 0; round < 64; ++round) {
    if (bfs(G, N, R, entry, seen, queue) == N) break;
    int64_t nu = 0;
    for (int64_t v = 0; v < N; ++v)
      if (!seen[v]) unr[nu++] = (int32_t)v;
    if (qgo_encode(X, N, D, G, R, M, blocks, nthreads) != 0) return -3;
#pragma omp parallel
    {
      int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)EF);
      float *dd = (float *)malloc(sizeof(float) * (size_t)EF);
#pragma omp for schedule(dynamic, 16)
      for (int64_t a = 0; a < nu; ++a) {
        const int32_t v = unr[a];
        qgo_search(blocks, N, D, R, entry, M, X + (int64_t)v * D, 1, EF, EF, 0, ids, dd, NULL, 1);
        int64_t w = -1;
        for (int b = 0; b < EF && w < 0 && ids[b] >= 0; ++b) {
          int free_slot = 0;
          for (int j = 0; j < R && !free_slot; ++j) free_slot = !fixed[(int64_t)ids[b] * R + j];
          if (free_slot) w = ids[b];
        }
        pick[a] = w < 0 ? -1 : (int64_t)((uint64_t)w << 32 | (uint32_t)v);
      }
      free(ids);
      free(dd);
    }
    qsort(pick, (size_t)nu, sizeof(int64_t), cmp_i64);
    int64_t made = 0;
    for (int64_t a = 0; a < nu;) {
      if (pick[a] < 0) {
        ++a;
        continue;
      }
      const int64_t w = pick[a] >> 32;
      int32_t *row = G + w * R;
      int ns = 0;
      for (int j = 0; j < R; ++j)
        if (row[j] < 0) {
          slots[ns].d = INFINITY; /* empty slots first, in slot order */
          slots[ns++].id = j;
        }
      const int nempty = ns;
      for (int j = 0; j < R; ++j)
        if (row[j] >= 0 && !fixed[w * R + j]) {
          slots[ns].d = dist2(X + w * D, X + (int64_t)row[j] * D, D);
          slots[ns++].id = j;
        }
      for (int i = nempty + 1; i < ns; ++i) { /* farthest first, ties to the larger neighbour id */
        cand_t x = slots[i];
        int pos = i;
        while (pos > nempty && (slots[pos - 1].d < x.d ||
                                (slots[pos - 1].d == x.d && row[slots[pos - 1].id] < row[x.id]))) {
          slots[pos] = slots[pos - 1];
          --pos;
        }
        slots[pos] = x;
      }
      int next = 0;
      for (; a < nu && pick[a] >= 0 && (pick[a] >> 32) == w; ++a) {
        if (next >= ns) continue; /* no slot left: this v waits for the next round */
        const int j = slots[next++].id;
        row[j] = (int32_t)(pick[a] & 0xffffffff);
        fixed[w * R + j] = 1;
        ++repairs;
        ++made;
      }
    }
    if (!made) break;
  }
  free(fixed);
  free(unr);
  free(pick);
  free(slots);
  int64_t reach = bfs(G, N, R, entry, seen, queue);
  if (stats) {
    stats[1] = repairs;
    stats[2] = reach;
  }
  free(seen);
  free(queue);
  free(blocks);
  free(newG);
  free(cands);
  free(ncand);
  free(nkept);
  free(keptidx);
  return reach == N ? 0 : -4;
}

/* ----------------------------------------------------------- index file */

/* Index file: a 4096-byte header, the rotation M (f32, row-major D x D,
 * padded to a 4096-byte boundary), then N vertex blocks.  Header fields
 * (little endian): 0 magic "QGINDEX1"; 8 u32 version = 1; 12 u32 header size
 * = 4096; 16 i64 N; 24 i32 D; 28 i32 R; 32 i32 entry; 36 i32 query bits = 8;
 * 40 i64 block bytes; 48 i64 rotation offset; 56 i64 blocks offset;
 * 64 u64 payload bytes (file size - 4096); 72 u64 FNV-1a-64 of the payload. */
static uint64_t fnv1a(uint64_t h, const uint8_t *p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ULL;
  }
  return h;
}

int qgo_write_index(const char *path, int64_t N, int D, int R, int32_t entry, const float *M, const uint8_t *blocks) {
  int64_t B = qgo_block_bytes(D, R);
  int64_t rot_bytes = 4LL * D * D, rot_pad = (rot_bytes + 4095) / 4096 * 4096;
  int64_t payload = rot_pad + N * B;
  uint8_t *rot = (uint8_t *)calloc((size_t)rot_pad, 1);
  memcpy(rot, M, (size_t)rot_bytes);
  uint64_t h = 0xcbf29ce484222325ULL;
  h = fnv1a(h, rot, (size_t)rot_pad);
  h = fnv1a(h, blocks, (size_t)(N * B));
  uint8_t hdr[4096];
  memset(hdr, 0, sizeof hdr);
  memcpy(hdr, "QGINDEX1", 8);
  uint32_t ver = 1, hsz = 4096;
  int32_t qbits = 8;
  int64_t off_rot = 4096, off_blk = 4096 + rot_pad;
  memcpy(hdr + 8, &ver, 4);
  memcpy(hdr + 12, &hsz, 4);
  memcpy(hdr + 16, &N, 8);
  memcpy(hdr + 24, &D, 4);
  memcpy(hdr + 28, &R, 4);
  memcpy(hdr + 32, &entry, 4);
  memcpy(hdr + 36, &qbits, 4);
  memcpy(hdr + 40, &B, 8);
  memcpy(hdr + 48, &off_rot, 8);
  memcpy(hdr + 56, &off_blk, 8);
  memcpy(hdr + 64, &payload, 8);
  memcpy(hdr + 72, &h, 8);
  FILE *f = fopen(path, "wb");
  if (!f) {
    free(rot);
    return -3;
  }
  int ok = fwrite(hdr, 1, sizeof hdr, f) == sizeof hdr && fwrite(rot, 1, (size_t)rot_pad, f) == (size_t)rot_pad &&
           fwrite(blocks, 1, (size_t)(N * B), f) == (size_t)(N * B);
  ok = (fclose(f) == 0) && ok;
  free(rot);
  return ok ? 0 : -3;
}

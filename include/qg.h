/*
 * qg.h -- C ABI of libqg, the MI355X (gfx950) query path of SymphonyQG
 * (Gou, Gao, Xu, Long: "SymphonyQG: Towards Symphonious Integration of
 * Quantization and Graph for Approximate Nearest Neighbor Search",
 * arXiv 2411.12229).
 *
 * The library owns a quantization-graph index resident in device memory:
 * one contiguous block per vertex holding its raw vector, the 1-bit RaBitQ
 * codes and two correction factors of each out-neighbour (normalised with
 * the vertex itself as the centre), and the neighbour ids (Sec. 3.1.3).
 * qg_search runs Algorithm 1 (Sec. 3.1.3) for a batch of queries.
 *
 * Conventions for every entry point:
 *  - Array arguments are raw pointers to DEVICE memory on the index's device
 *    unless stated otherwise; the caller owns them.  Row-major layouts.
 *  - Work is enqueued on the index's stream (qg_set_stream, default: the
 *    null stream) and the call returns after enqueueing; outputs are valid
 *    once that stream has reached the call.
 *  - Return value: QG_OK or a negative QG_E* code.  Argument errors are
 *    detected before anything is enqueued.  qg_last_error() describes the
 *    last failure on the calling thread.  No C++ exception crosses the ABI.
 *  - Distances are squared Euclidean distances in fp32.  Cosine similarity
 *    is served by searching unit-norm vectors (Sec. 3, footnote on metrics).
 */
#ifndef QG_H
#define QG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qg_index qg_index;

enum {
  QG_OK = 0,
  QG_EINVAL = -1,       /* bad argument (NULL pointer, negative size, k or ef <= 0, ...) */
  QG_ENOMEM = -2,       /* device or host allocation failed */
  QG_EIO = -3,          /* file could not be opened, read or written */
  QG_EFORMAT = -4,      /* index file malformed: magic, version, sizes or checksum */
  QG_EDEVICE = -5,      /* a HIP runtime call failed */
  QG_EUNSUPPORTED = -6  /* valid but not supported: (D, R) pair, ef or k above the maximum */
};

/* Flags for qg_search_ex. */
enum {
  QG_SEARCH_NO_ME = 1,     /* "w/o ME" ablation (Sec. 4.2.3): a vertex enters the beam only on its first estimate
                              (plain search only: QG_EUNSUPPORTED with per-query k and ef or the learned stop) */
  QG_SEARCH_SMALL_HASH = 2, /* test hook: shrink the on-chip visited set to 128 slots so that queries take the
                              overflow path (results are identical by construction) */
  QG_SEARCH_LDS_BEAM = 4    /* keep the beam in LDS for this call, as for beams above 128 entries, instead of in
                              registers (results are identical by construction) */
};

/* Largest supported beam size and result count. */
#define QG_MAX_EF 2048
#define QG_MAX_K 1024

/* Load an index file into device memory of `device`: a 4096-byte header,
 * the rotation M, then one contiguous block per vertex laid out as the
 * paper's data layout prescribes (Sec. 3.1.3: raw vector, then the FastScan
 * data of its neighbours -- codes and two factors each -- then the neighbour
 * ids, padded to 128 bytes), FNV-1a-64 checksum verified.  *out receives a new
 * index, NULL on error.  Supported (D, R): D in {96, 128, 768, 960} (or any
 * multiple of 32 up to 1024 for which the library was built), R in {32, 64}.
 * QG_EFORMAT also for a neighbour id outside [-1, N) or one that a vertex's
 * list holds twice. */
int qg_load_index(const char *path, int device, qg_index **out);

/* Build an index on `device` from vectors[n][d] (fp32), graph[n][r] (int32
 * ids in [0, n), -1 = empty slot; no id twice in one list, as Algorithm 2's
 * lists of distinct neighbours: QG_EINVAL otherwise), rotation[d][d] (fp32, the matrix M =
 * P^{-1} applied to vectors, Eq. rotation) and the entry vertex.  All three
 * arrays are device pointers; they are read during the call and may be freed
 * afterwards.  Encodes every block on the GPU (Sec. 3.1.1 normalisation by
 * the holding vertex; the FastScan data of every vertex built in Alg. 2). Synchronous. */
int qg_build_index(const float *vectors, int64_t n, int32_t d, const int32_t *graph, int32_t r,
                   const float *rotation, int32_t entry, int device, qg_index **out);

/* Flags of qg_build_graph. */
enum {
  QG_GRAPH_REFINE = 1, /* supplement edges to exactly r per vertex (Sec. 3.2.2), random fill when too few */
  QG_GRAPH_REPAIR = 2,  /* link vertices unreachable from the entry (an addition: clustered data can leave the
                           graph disconnected) */
  QG_GRAPH_PROGRESS = 4 /* print one line to stderr as each stage ends (iteration search and pruning,
                           refinement, repair rounds), for builds that run for minutes */
};

/* Algorithm 2 (Indexing, Sec. 3.2) on `device`: starting from init_graph[n][r]
 * (distinct non-self ids, as a random initial graph), `iters` times: encode
 * the current graph (the FastScan data of every vertex), run Algorithm 1 for
 * every vector with beam ef_build and ef_build results (the search kernels of
 * qg_search_ex), take as candidates of u the results other than u together
 * with u's current neighbours, and keep by the NSG rule (Sec. 3.2.1: scan the
 * candidates by (distance, id) and keep v unless a kept w is closer to v than
 * u is; at most r); all lists are replaced at once.  With QG_GRAPH_REFINE a
 * vertex left with fewer than r neighbours then takes the pruned candidates
 * that survive the largest angle threshold leaving enough of them (Sec.
 * 3.2.2: a candidate is pruned when a closer candidate makes an angle below
 * the threshold with it at u; the limit of the paper's binary search is taken
 * exactly), nearest first, and ids from fill[n][r] while still short.  With
 * QG_GRAPH_REPAIR every vertex unreachable from `entry` is then linked from
 * its nearest reachable vertex.  Distances, norms and inner products are fp64
 * sums over dimensions in ascending order.  vectors[n][d], rotation[d][d],
 * init_graph, fill (needed with QG_GRAPH_REFINE) and out_graph[n][r] (int32,
 * -1 = empty slot) are device arrays; out_stats (host, nullable) receives
 * [vertices reachable before the repair, repairs made, reachable after,
 * elapsed microseconds].  Synchronous; allocates its working memory (about
 * n (12 (ef_build + r) + 8 r) bytes). */
int qg_build_graph(const float *vectors, int64_t n, int32_t d, int32_t r, int32_t ef_build, int32_t iters,
                   const float *rotation, int32_t entry, const int32_t *init_graph, const int32_t *fill,
                   int32_t flags, int device, int32_t *out_graph, int64_t *out_stats);

/* Write the index to a file in the format read by qg_load_index. Synchronous. */
int qg_save_index(const qg_index *idx, const char *path);

/* Algorithm 1 for nq queries[nq][d] (fp32): out_ids[nq][k] (int32) and
 * out_dists[nq][k] (fp32), each row ascending by (distance, id), padded with
 * (-1, +inf) when fewer than k vertices were visited.  1 <= k <= QG_MAX_K,
 * 1 <= ef <= QG_MAX_EF (ef is the beam size n_b; it is not raised to k).
 * nq == 0 is a no-op. */
int qg_search(const qg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t ef, int32_t *out_ids,
              float *out_dists);

/* qg_search with flags (QG_SEARCH_*) and optional per-query counters
 * out_stats[nq][4] (int32, device, nullable): expansions (vertices whose
 * exact distance was computed), pops from the beam, appended candidates, and
 * 1 if the query was finished by the overflow path (its visited set, or
 * without ME its set of estimated vertices, outgrew on-chip memory; results
 * are identical either way). */
int qg_search_ex(const qg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                 int32_t *out_ids, float *out_dists, int32_t *out_stats);

/* Learned early stop (an addition beyond the paper, whose Algorithm 1 runs
 * until the beam holds no unchecked entry).  After the t-th expansion, for
 * t >= t_min with (t - t_min) divisible by t_every, a 16-64-64-1 ReLU MLP with
 * bf16 parameters and fp32 arithmetic reads 16 features of the search state
 * (expansions, pops, NN fill and distances relative to the entry, the next
 * beam estimate relative to the k-th distance, beam fill, ...) and the query
 * stops when its output exceeds theta.  Parameters (QG_STOP_MLP_PARAMS bf16
 * bit patterns, device memory): W1[64][16], b1[64], W2[64][64], b2[64],
 * W3[64], b3.  With mlp == NULL nothing stops early and only the trace is
 * written: features [nq][trace_max][16] (fp32), NN ids [nq][trace_max][k],
 * MLP output [nq][trace_max] (NaN without a model) and the number of
 * evaluation points recorded per query [nq] -- the training data. */
#define QG_STOP_MLP_PARAMS (64 * 16 + 64 + 64 * 64 + 64 + 64 + 1)

typedef struct qg_stop_params {
  const uint16_t *mlp; /* device, QG_STOP_MLP_PARAMS values, 16-byte aligned; NULL = no early stop */
  float theta;
  int32_t t_min;   /* >= 1 */
  int32_t t_every; /* >= 1 */
  int32_t trace_max;      /* evaluation points recorded per query; 0 = no trace */
  float *trace_features;  /* device, nullable when trace_max == 0 */
  int32_t *trace_nn;
  float *trace_out;
  int32_t *trace_count;
} qg_stop_params;

/* qg_search_ex with the learned stop (stop != NULL) described above. */
int qg_search_stop(const qg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                   const qg_stop_params *stop, int32_t *out_ids, float *out_dists, int32_t *out_stats);

/* Algorithm 1 with a result count and beam size of its own for every query,
 * in one launch (queries of a mixed batch do not wait for the slowest
 * setting).  k_per_query[nq] and ef_per_query[nq] are int32 device arrays;
 * k_max and ef_max bound them (1 <= k_max <= QG_MAX_K, 1 <= ef_max <=
 * QG_MAX_EF) and size on-chip memory for the whole batch.  out_ids and
 * out_dists are [nq][k_max] (row stride k_max): row q holds its k_q results
 * ascending by (distance, id), then (-1, +inf).  A query with k_q or ef_q
 * outside [1, k_max] or [1, ef_max] is not searched: its row is all padding
 * and, when out_stats is given, its counters are (0, 0, 0, -1).  Each
 * query's results are those of qg_search_ex with its own k_q and ef_q. */
int qg_search_mixed(const qg_index *idx, const float *queries, int64_t nq, const int32_t *k_per_query,
                    const int32_t *ef_per_query, int32_t k_max, int32_t ef_max, int32_t flags, int32_t *out_ids,
                    float *out_dists, int32_t *out_stats);

/* qg_search_mixed with the learned stop: every query runs with its own k_q
 * and ef_q and the shared stop model (stop->mlp non-NULL, theta, t_min,
 * t_every; stop->trace_max must be 0).  Each query's results are those of
 * qg_search_stop for that query alone with its own k_q and ef_q.  QG_EINVAL
 * without a model or with a trace requested. */
int qg_search_mixed_stop(const qg_index *idx, const float *queries, int64_t nq, const int32_t *k_per_query,
                         const int32_t *ef_per_query, int32_t k_max, int32_t ef_max, int32_t flags,
                         const qg_stop_params *stop, int32_t *out_ids, float *out_dists, int32_t *out_stats);

/* out[n][d] = M in[n][d] for the index's rotation M (Eq. rotation), on the
 * matrix cores: fp64 products accumulated over j ascending, rounded once to
 * fp32.  This is the first step of qg_search, exposed for checking.  Any
 * 4-byte-aligned `in` works; rows that start 16-byte aligned take wider loads
 * (the result is the same either way). */
int qg_rotate(const qg_index *idx, const float *in, int64_t n, float *out);

/* The estimator alone (Sec. 3.1.1, Eq. 3.1): for query i and vertex
 * vertex_of_query[i], out_S[i][r] = FastScan sums S_j (int32),
 * out_est[i][r] = estimated squared distances of the vertex's neighbours,
 * out_dist[i] = exact squared distance to the vertex.  Same device code as
 * qg_search. */
int qg_estimate(const qg_index *idx, const float *queries, const int32_t *vertex_of_query, int64_t nq,
                int32_t *out_S, float *out_est, float *out_dist);

/* Copy blocks [first, first + count) (block_bytes each) to device memory dst. */
int qg_copy_blocks(const qg_index *idx, int64_t first, int64_t count, void *dst);

/* Select the HIP stream (hipStream_t) for later work; NULL = null stream.
 * (Runtime plumbing: the paper's search is single-threaded on a CPU and has
 * no counterpart.)
 * Every search call only enqueues kernels on this stream (no host
 * synchronisation, no memset), so a caller may record searches into a HIP
 * graph by capturing this stream.  Calls on one index share its scratch and
 * must not overlap in time on different streams. */
int qg_set_stream(qg_index *idx, void *hip_stream);

/* Launch-shape autotuning.  Times qg_search_ex on the given device queries
 * (k, ef, flags as they will be used) for every combination of wavefronts per
 * workgroup (1, 2, 4, 8; halved at launch while the LDS does not fit) and
 * visited-hash size (2^h >= F * min(ef, 256) + max(ef - 256, 0) slots, F = 2, 3, 4; a smaller table leaves
 * room for more wavefronts, a larger one sends fewer queries to the overflow
 * pass), then, for the fastest pair, caps of 24, 20 and 16 resident
 * wavefronts per compute unit against no cap (a batch only a little larger
 * than the resident query slots can finish sooner on fewer, less contended
 * slots), then, for beams of at most 128 entries, the beam kept in LDS
 * against the beam kept in registers, then the LUT layout (the per-query
 * table of Sec. 2.2's FastScan, rows of 16 entries: int16 or int32 entries,
 * with a padding row between the lane groups that share a neighbour, so that
 * their lookups fall in different LDS banks, or with packed rows; int32
 * entries apply to the plain and mixed searches).  The fastest setting is kept for
 * later searches of this index.  Each setting is timed as the median of seven
 * calls after one untimed call.  Results do not depend on the choice, only
 * the speed.  Outputs (host, nullable): the chosen wavefronts per workgroup,
 * F, the cap (0 = none), the beam storage (1 = registers where the beam size
 * allows, 0 = LDS), the LUT layout (bit 0: padded rows, bit 1: int32
 * entries; 1 = padded int16, the default) and the median time in ms of one
 * qg_search_ex call in that setting.
 * Synchronous; allocates and frees temporary outputs. */
int qg_autotune(qg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                int32_t *out_wpb, int32_t *out_hash_factor, int32_t *out_cu_waves, int32_t *out_beam,
                int32_t *out_lut, double *out_ms);

/* qg_autotune for mixed batches: times qg_search_mixed on the given device
 * queries and per-query k and ef (device int32[nq] each, bounded by k_max and
 * ef_max as in qg_search_mixed) over the same settings, and keeps the fastest
 * for later searches of this index (plain and mixed alike).  Errors and
 * outputs as qg_autotune's.  (Runtime plumbing with no counterpart in the
 * paper.) */
int qg_autotune_mixed(qg_index *idx, const float *queries, int64_t nq, const int32_t *k_per_query,
                      const int32_t *ef_per_query, int32_t k_max, int32_t ef_max, int32_t flags, int32_t *out_wpb,
                      int32_t *out_hash_factor, int32_t *out_cu_waves, int32_t *out_beam, int32_t *out_lut,
                      double *out_ms);

/* Set the launch shape directly (as qg_autotune would): wavefronts per
 * workgroup (1, 2, 4 or 8), visited-hash factor F (2, 3 or 4), the cap on
 * resident wavefronts per compute unit (0 = none, at most 64), the beam
 * storage (1: in registers for beams of at most 128 entries, the default;
 * 0: always in LDS) and the LUT layout (0..3; bit 0: padded rows, bit 1:
 * int32 entries; 1, padded int16 rows, is the default).  Results do not
 * depend on it.  QG_EINVAL for values outside these sets. */
int qg_set_launch(qg_index *idx, int32_t wpb, int32_t hash_factor, int32_t cu_waves, int32_t beam, int32_t lut);

/* ---- Serving loop (continuous batching) ----------------------------------
 * A server owns `streams` slots over one index.  Each slot has its own
 * stream, its own view of the index (the blocks are shared, the search
 * scratch is not), pinned staging buffers for max_batch queries and its own
 * worker thread.  Requests wait in classes of beam size (ef up to a power of
 * two).  As soon as a slot is free, its thread takes the class of the oldest
 * waiting request and
 * every waiting request of that class (up to max_batch), and runs upload, one
 * qg_search_mixed launch sized for the batch's largest ef, and download on
 * that slot's stream.  Batches grow with the load, short searches never wait
 * in a batch for long ones, and the slots overlap transfers with searches.  Every request's results are those of qg_search_ex
 * for that query alone with its own k and ef.  The index must outlive the
 * server; 1 <= streams <= 16, 1 <= k_max <= QG_MAX_K, 1 <= ef_max <= QG_MAX_EF.
 * Creation runs single-query searches on every slot (synchronously), one
 * for each beam storage a batch can use, so that every kernel a batch may
 * launch is loaded before the first request; qg_server_set_stop does the same
 * for the stop kernels. */
typedef struct qg_server qg_server;

int qg_server_create(qg_index *idx, int32_t streams, int32_t max_batch, int32_t k_max, int32_t ef_max,
                     qg_server **out);

/* Run every later batch of this server with the learned stop (the model,
 * theta, t_min and t_every of *stop, trace_max 0; the MLP parameters are
 * device memory that must stay valid while the server runs), or without it
 * (stop = NULL).  Each request's results are then those of qg_search_stop for
 * that query alone with its own k and ef.  Call it while no request is
 * waiting or in flight (after creation or qg_server_drain). */
int qg_server_set_stop(qg_server *s, const qg_stop_params *stop);

/* Queue one request: query[d] (fp32, host memory, copied before the call
 * returns), 1 <= k <= k_max, 1 <= ef <= ef_max, and a caller tag returned with
 * the results.  Thread-safe; never blocks on the device. */
int qg_server_submit(qg_server *s, const float *query, int32_t k, int32_t ef, uint64_t tag);

/* Beam sizes for target recalls (requests may name a recall@k target instead
 * of a beam): n rows of (k[i], target[i], ef[i]) host arrays, e.g. calibrated
 * on held-out queries.  A request with (k, target) takes the ef of the row
 * with the same k and the smallest target not below its own.  Replaces any
 * earlier map; call it while no request waits or runs.  QG_EINVAL for a k or
 * ef outside the server's bounds or a target outside (0, 1].  (Serving
 * plumbing; the paper's search takes a beam size.) */
int qg_server_set_recall_map(qg_server *s, const int32_t *k, const float *target, const int32_t *ef, int32_t n);

/* qg_server_submit with a target recall in place of ef, looked up in the
 * recall map (QG_EINVAL when no row covers (k, target)). */
int qg_server_submit_target(qg_server *s, const float *query, int32_t k, float target, uint64_t tag);

/* qg_server_replay with a target recall per request (target[n], host) in place
 * of ef; every (k, target) must be covered by the recall map (checked before
 * the replay starts). */
int qg_server_replay_target(qg_server *s, const float *queries, const int32_t *k, const float *target,
                            const double *arrival_s, int64_t n);

/* Move up to max_results finished requests out of the server, oldest first.
 * Host outputs, each nullable: tags[n], ids[n][k_max] and dists[n][k_max]
 * (a request's k results, then (-1, +inf)), latency_s[n] (submission, or
 * for a replayed request its scheduled arrival, to completion seen by the
 * worker, seconds), batch[n] (the index of the request's batch record, see
 * qg_server_batches; -1 past the records kept).  Returns the number written,
 * or a negative QG_* code. */
int64_t qg_server_poll(qg_server *s, int64_t max_results, uint64_t *tags, int32_t *ids, float *dists,
                       double *latency_s, int64_t *batch);

/* One batch the serving loop ran.  Host times are seconds on the clock the
 * latencies use (steady, arbitrary origin). */
typedef struct {
  double t_oldest;   /* arrival (submission or scheduled arrival) of its oldest request */
  double t_dispatch; /* the worker took the batch from the queue */
  double t_enqueued; /* its uploads, search, downloads and event were enqueued */
  double t_done;     /* the worker saw the batch's event complete (0 while in flight) */
  float device_ms;   /* device time between an event before the uploads and one after the downloads
                        (-1 while in flight) */
  int32_t n;         /* requests in the batch */
  int32_t ef_max;    /* largest beam among them (the launch is sized for it) */
  int32_t k_max;     /* largest k among them */
  int32_t slot;      /* the stream slot it ran on */
  float enqueue_cpu_ms;   /* CPU time the worker thread used between t_dispatch and t_enqueued */
  int32_t enqueue_nvcsw;  /* the worker's voluntary context switches in that interval (it blocked) */
  int32_t enqueue_nivcsw; /* its involuntary context switches in that interval (it was preempted) */
  float upload_ms;        /* host time of the enqueue's parts: staging the queries and the uploads, */
  float search_ms;        /* the search call (qg_search_mixed or qg_search_mixed_stop), */
  float download_ms;      /* the downloads and the event */
} qg_server_batch;

/* Copy batch records [first, first + max) (host out[max]); the server keeps
 * the first 2^22.  Returns the number copied, or a negative QG_* code.
 * (Instrumentation of the serving loop: a slow request is traced through its
 * batch index from qg_server_poll to where its time went.) */
int64_t qg_server_batches(qg_server *s, int64_t first, int64_t max, qg_server_batch *out);

/* Submit queries[n][d] (host) with tags 0 .. n-1 at arrival_s[i] seconds after
 * the call (an open-loop arrival trace; arrival_s non-decreasing), from a
 * thread of the server; returns at once.  A request's latency counts from its
 * scheduled arrival time, also when the thread queues it later (every request
 * whose time has passed is queued at once).  The arrays must stay valid until
 * qg_server_drain returns. */
int qg_server_replay(qg_server *s, const float *queries, const int32_t *k, const int32_t *ef,
                     const double *arrival_s, int64_t n);

/* Wait until every submitted request has finished (its results wait for
 * poll), at most timeout_s seconds.  Ends a running replay first. */
int qg_server_drain(qg_server *s, double timeout_s);

/* Counters (host, nullable): requests submitted and finished, batches
 * launched and the largest batch. */
int qg_server_stats(qg_server *s, int64_t *submitted, int64_t *completed, int64_t *batches, int64_t *largest_batch);

/* Finish every queued request, stop the worker and free the server. */
void qg_server_destroy(qg_server *s);

/* Grow the index's per-query scratch (rotated queries, overflow list) to hold
 * at least nq queries.  Searches grow it themselves (reallocating) when a
 * batch is larger than any before; captured graphs refer to the scratch that
 * existed at capture time, so reserve the largest batch before capturing and
 * replay only while no later call has grown it.  Synchronous. */
int qg_reserve(qg_index *idx, int64_t nq);

/* For callers that cannot allocate device memory during a search (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): qg_search_ex with the same arguments, results and errors, but
 * its per-call scratch (queue counters, rotated queries, overflow list) lives
 * in a fixed device array of QG_NOALLOC_SCRATCH_BYTES compiled into the
 * library, one copy per device held until the process ends, instead of the
 * index's scratch that grows on demand.  The call allocates and frees
 * nothing.  nq may be at most (QG_NOALLOC_SCRATCH_BYTES - 256) / (4 d + 4)
 * (32,513 queries at d = 128, 4,364 at d = 960); a larger batch gives
 * QG_EUNSUPPORTED before anything is enqueued.  Every call on a device, for
 * any index and on any stream, shares that device's array, which keeps the
 * last call's contents (the call's first kernel clears the counters): calls
 * that overlap in time on one device race and give wrong results.  The
 * overflow pass uses the bitsets the index allocated when it was created.
 * Not recorded by qg_timing. */
#define QG_NOALLOC_SCRATCH_BYTES (16 << 20)
int qg_search_noalloc(const qg_index *idx, const float *queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                      int32_t *out_ids, float *out_dists, int32_t *out_stats);

/* Index geometry: vector count n, dimension d, out-degree r (R of Sec. 3.2),
 * the entry vertex e of Algorithm 1, and the byte size of one vertex block
 * (Sec. 3.1.3 layout, padded to 128 bytes).  Any output pointer may be NULL.
 * Host pointers. */
int qg_index_info(const qg_index *idx, int64_t *n, int32_t *d, int32_t *r, int32_t *entry, int64_t *block_bytes);

/* Kernel timing with HIP events recorded on the index's stream around every
 * search-kernel launch (kernel 1) and rotation launch (kernel 0).
 * qg_timing(idx, 1) clears and starts recording, qg_timing(idx, 0) stops.
 * qg_timing_read waits for the recorded events and returns the number of
 * launches and their summed duration in milliseconds (host pointers). */
int qg_timing(qg_index *idx, int enable);
int qg_timing_read(qg_index *idx, int kernel, int32_t *launches, double *total_ms);

/* Release all device memory of the index. NULL is accepted. */
void qg_free_index(qg_index *idx);

/* Description of the last error on this thread (empty string if none). */
const char *qg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QG_H */

// qg_server.cpp -- a serving loop over one index (C ABI in include/qg.h).
//
// Requests (one query, its k and ef, a caller tag) are queued by any thread,
// in classes of beam size (ef up to 2^c).  The server has S stream slots, each
// with its own view of the index (shared blocks, private scratch), pinned
// staging buffers and worker thread.  Whenever a slot is free its worker
// takes the class of the oldest waiting request, every waiting request of that
// class (up to the batch limit), and enqueues on that slot's stream: the
// queries' upload, one mixed search launch sized for the batch's largest ef
// (a k and ef per query) and the results' download, then an event.  Batches
// grow with the load and shrink when it is light (continuous batching); a
// batch of short searches never waits for a long one and is sized for its own
// beam (more wavefronts fit), and the S slots overlap transfers with searches.
// Latency is measured on the host from submission to the moment the worker
// sees the batch's event complete.  Every batch leaves a record (host times of
// its oldest arrival, dispatch, enqueue and completion, and its device time
// between two events), so that a slow request can be traced to what held it.
#include <hip/hip_runtime.h>
#include <sys/resource.h>
#include <time.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "qg.h"
#include "qg_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The calling thread's CPU time and context-switch counts.
struct ThreadUsage {
  double cpu_s = 0;
  long nvcsw = 0, nivcsw = 0;
  static ThreadUsage now() {
    ThreadUsage u;
    timespec ts{};
    if (clock_gettime(CLOCK_THREAD_CPUTIME_ID, &ts) == 0) u.cpu_s = (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
    rusage ru{};
    if (getrusage(RUSAGE_THREAD, &ru) == 0) {
      u.nvcsw = ru.ru_nvcsw;
      u.nivcsw = ru.ru_nivcsw;
    }
    return u;
  }
};

struct Request {
  uint64_t tag = 0;
  int32_t k = 0, ef = 0;
  double t_submit = 0;
  std::vector<float> q;     // a copy of the query (submit)
  const float* src = nullptr;  // or the caller's row, valid until drain (replay: no allocation per request)
  const float* data() const { return src ? src : q.data(); }
};

// One finished batch: its rows are handed out by poll, oldest first.
struct DoneBatch {
  int64_t seq = 0;           // index of the batch's record
  std::vector<uint64_t> tags;
  std::vector<int32_t> ks;
  std::vector<double> latency;
  std::vector<int32_t> ids;  // row i's k_i results, rows back to back
  std::vector<float> dists;
  size_t next = 0;           // rows already polled
  size_t pos = 0;            // offset of row `next` in ids and dists
};

struct Slot {
  qg_index* view = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr;  // before the uploads (timing)
  hipEvent_t done = nullptr;   // after the downloads (timing)
  float* h_q = nullptr;  // pinned host staging
  int32_t* h_k = nullptr;
  int32_t* h_ef = nullptr;
  int32_t* h_ids = nullptr;
  float* h_dists = nullptr;
  float* d_q = nullptr;  // device
  int32_t* d_k = nullptr;
  int32_t* d_ef = nullptr;
  int32_t* d_ids = nullptr;
  float* d_dists = nullptr;
  std::vector<Request> batch;
  int64_t seq = -1;  // record of the batch in flight
  bool busy = false;
};

}  // namespace

struct qg_server {
  qg_index* idx = nullptr;
  int device = 0, D = 0;
  int32_t k_max = 0, ef_max = 0, max_batch = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv;  // new requests, or a stop request, for the idle worker
  std::condition_variable cv_done;  // completions, for drain
  static constexpr int kClasses = 12;  // ef <= 2^c, c < 12 (QG_MAX_EF = 2^11)
  std::deque<Request> pending[kClasses];
  int64_t npending = 0;
  std::deque<DoneBatch> done;
  std::vector<DoneBatch> spare;  // records already polled, kept for reuse (no allocation per batch)
  bool use_stop = false;         // batches run with the learned stop (qg_server_set_stop)
  qg_stop_params stop_params{};
  int64_t submitted = 0, completed = 0, batches = 0, largest = 0;
  struct RecallRow {
    int32_t k;
    float target;
    int32_t ef;
  };
  std::vector<RecallRow> recall_map;     // sorted by (k, target)
  std::vector<int32_t> replay_ef;        // the beams of a replay given by target recalls
  static constexpr size_t kMaxRecords = size_t(1) << 22;  // batch records kept (the first 4M)
  std::vector<qg_server_batch> records;
  int error = QG_OK;
  std::string errmsg;
  bool stop = false;
  std::vector<std::thread> workers;  // one per slot
  std::thread producer;
};

namespace {

void free_slot(Slot& s) {
  (void)hipFree(s.d_q);
  (void)hipFree(s.d_k);
  (void)hipFree(s.d_ef);
  (void)hipFree(s.d_ids);
  (void)hipFree(s.d_dists);
  (void)hipHostFree(s.h_q);
  (void)hipHostFree(s.h_k);
  (void)hipHostFree(s.h_ef);
  (void)hipHostFree(s.h_ids);
  (void)hipHostFree(s.h_dists);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.start) (void)hipEventDestroy(s.start);
  if (s.view) qg_free_index(s.view);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot{};
}

// One batch of a single zero query through every step a batch takes
// (uploads, search, downloads, events) for each beam storage a batch can get
// (a beam of one entry, of 65 and of 129: one or two register words per lane,
// or LDS), with the stop if `stop` is given, so that every kernel a batch may
// launch is loaded, and the copy paths set up, before the first request: the
// first launch of a kernel loads its code and takes milliseconds.
bool warm_up(qg_server* sv, Slot& s, const qg_stop_params* stop) {
  const size_t K = (size_t)sv->k_max, D = (size_t)sv->D;
  std::memset(s.h_q, 0, sizeof(float) * D);
  s.h_k[0] = 1;
  for (int32_t ef : {1, 65, 129}) {
    if (ef > sv->ef_max) break;
    s.h_ef[0] = ef;
    const bool ok =
        hipMemcpyAsync(s.d_q, s.h_q, sizeof(float) * D, hipMemcpyHostToDevice, s.stream) == hipSuccess &&
        hipMemcpyAsync(s.d_k, s.h_k, sizeof(int32_t), hipMemcpyHostToDevice, s.stream) == hipSuccess &&
        hipMemcpyAsync(s.d_ef, s.h_ef, sizeof(int32_t), hipMemcpyHostToDevice, s.stream) == hipSuccess &&
        (stop ? qg_search_mixed_stop(s.view, s.d_q, 1, s.d_k, s.d_ef, sv->k_max, ef, 0, stop, s.d_ids, s.d_dists,
                                     nullptr)
              : qg_search_mixed(s.view, s.d_q, 1, s.d_k, s.d_ef, sv->k_max, ef, 0, s.d_ids, s.d_dists, nullptr)) ==
            QG_OK &&
        hipMemcpyAsync(s.h_ids, s.d_ids, sizeof(int32_t) * K, hipMemcpyDeviceToHost, s.stream) == hipSuccess &&
        hipMemcpyAsync(s.h_dists, s.d_dists, sizeof(float) * K, hipMemcpyDeviceToHost, s.stream) == hipSuccess &&
        hipEventRecord(s.done, s.stream) == hipSuccess && hipEventSynchronize(s.done) == hipSuccess &&
        hipEventQuery(s.done) == hipSuccess;
    if (!ok) return false;
  }
  return true;
}

bool init_slot(qg_server* sv, Slot& s) {
  const size_t B = (size_t)sv->max_batch, K = (size_t)sv->k_max, D = (size_t)sv->D;
  if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipEventCreate(&s.done) != hipSuccess || hipEventCreate(&s.start) != hipSuccess) return false;
  if (hipHostMalloc(&s.h_q, sizeof(float) * B * D) != hipSuccess ||
      hipHostMalloc(&s.h_k, sizeof(int32_t) * B) != hipSuccess ||
      hipHostMalloc(&s.h_ef, sizeof(int32_t) * B) != hipSuccess ||
      hipHostMalloc(&s.h_ids, sizeof(int32_t) * B * K) != hipSuccess ||
      hipHostMalloc(&s.h_dists, sizeof(float) * B * K) != hipSuccess)
    return false;
  if (hipMalloc(&s.d_q, sizeof(float) * B * D) != hipSuccess || hipMalloc(&s.d_k, sizeof(int32_t) * B) != hipSuccess ||
      hipMalloc(&s.d_ef, sizeof(int32_t) * B) != hipSuccess ||
      hipMalloc(&s.d_ids, sizeof(int32_t) * B * K) != hipSuccess ||
      hipMalloc(&s.d_dists, sizeof(float) * B * K) != hipSuccess)
    return false;
  s.view = qgi::make_view(sv->idx);
  if (!s.view) return false;
  if (qg_set_stream(s.view, s.stream) != QG_OK || qg_reserve(s.view, sv->max_batch) != QG_OK) return false;
  return warm_up(sv, s, nullptr);
}

void fail_server(qg_server* sv, const std::string& msg) {
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->error == QG_OK) {
    sv->error = QG_EDEVICE;
    sv->errmsg = msg;
  }
  sv->cv_done.notify_all();
}

int ef_class(int32_t ef) {
  int c = 0;
  while ((1 << c) < ef) ++c;
  return c;
}

// Enqueue one batch on a free slot.  Returns false on a device error.
bool dispatch(qg_server* sv, Slot& s, std::vector<Request>&& take, int slot) {
  qg_server_batch rec{};
  const ThreadUsage u0 = ThreadUsage::now();
  rec.t_dispatch = now_s();
  const int n = (int)take.size();
  const size_t D = (size_t)sv->D;
  for (int i = 0; i < n; ++i) {
    std::memcpy(s.h_q + (size_t)i * D, take[i].data(), sizeof(float) * D);
    s.h_k[i] = take[i].k;
    s.h_ef[i] = take[i].ef;
  }
  const size_t K = (size_t)sv->k_max;
  if (hipEventRecord(s.start, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.d_q, s.h_q, sizeof(float) * D * n, hipMemcpyHostToDevice, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.d_k, s.h_k, sizeof(int32_t) * n, hipMemcpyHostToDevice, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.d_ef, s.h_ef, sizeof(int32_t) * n, hipMemcpyHostToDevice, s.stream) != hipSuccess) {
    fail_server(sv, "upload of a batch failed");
    return false;
  }
  const double t_up = now_s();
  int32_t ef_batch = 1, k_batch = 1;
  double oldest = take[0].t_submit;
  for (int i = 0; i < n; ++i) {
    ef_batch = std::max(ef_batch, take[i].ef);
    k_batch = std::max(k_batch, take[i].k);
    oldest = std::min(oldest, take[i].t_submit);
  }
  const int rc = sv->use_stop ? qg_search_mixed_stop(s.view, s.d_q, n, s.d_k, s.d_ef, sv->k_max, ef_batch, 0,
                                                     &sv->stop_params, s.d_ids, s.d_dists, nullptr)
                              : qg_search_mixed(s.view, s.d_q, n, s.d_k, s.d_ef, sv->k_max, ef_batch, 0, s.d_ids,
                                                s.d_dists, nullptr);
  if (rc != QG_OK) {
    fail_server(sv, std::string("search: ") + qg_last_error());
    return false;
  }
  const double t_se = now_s();
  if (hipMemcpyAsync(s.h_ids, s.d_ids, sizeof(int32_t) * K * n, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
      hipMemcpyAsync(s.h_dists, s.d_dists, sizeof(float) * K * n, hipMemcpyDeviceToHost, s.stream) != hipSuccess ||
      hipEventRecord(s.done, s.stream) != hipSuccess) {
    fail_server(sv, "download of a batch failed");
    return false;
  }
  rec.t_enqueued = now_s();
  const ThreadUsage u1 = ThreadUsage::now();
  rec.upload_ms = (float)((t_up - rec.t_dispatch) * 1e3);
  rec.search_ms = (float)((t_se - t_up) * 1e3);
  rec.download_ms = (float)((rec.t_enqueued - t_se) * 1e3);
  rec.enqueue_cpu_ms = (float)((u1.cpu_s - u0.cpu_s) * 1e3);
  rec.enqueue_nvcsw = (int32_t)(u1.nvcsw - u0.nvcsw);
  rec.enqueue_nivcsw = (int32_t)(u1.nivcsw - u0.nivcsw);
  rec.t_oldest = oldest;
  rec.n = n;
  rec.ef_max = ef_batch;
  rec.k_max = k_batch;
  rec.slot = slot;
  rec.device_ms = -1.0f;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    s.seq = (int64_t)sv->records.size();
    if (sv->records.size() < qg_server::kMaxRecords) sv->records.push_back(rec);
    else s.seq = -1;
  }
  s.batch = std::move(take);
  s.busy = true;
  return true;
}

// The worker thread of slot `si`: takes the class of the oldest waiting
// request and every waiting request of that class (up to the batch limit),
// enqueues the batch on its stream, waits for the batch's event and hands the
// results out.  Each slot has its own thread, so a host call that takes long
// in one slot (a copy call once held a thread for 5-11 ms) does not hold up
// the batches of the others.
void slot_loop(qg_server* sv, size_t si) {
  (void)hipSetDevice(sv->device);
  Slot& s = sv->slots[si];
  const size_t K = (size_t)sv->k_max;
  for (;;) {
    std::vector<Request> take;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      while (sv->npending == 0 && !sv->stop && sv->error == QG_OK) sv->cv.wait(lk);
      if (sv->error != QG_OK) {
        // a failed server completes nothing more: drop what waits
        for (auto& d : sv->pending) d.clear();
        sv->npending = 0;
        sv->cv_done.notify_all();
        if (sv->stop) return;
        sv->cv.wait(lk);
        continue;
      }
      if (sv->npending == 0) return;  // stopping, nothing left
      int c = -1;  // the class of the oldest waiting request
      for (int i = 0; i < qg_server::kClasses; ++i)
        if (!sv->pending[i].empty() && (c < 0 || sv->pending[i].front().t_submit < sv->pending[c].front().t_submit))
          c = i;
      auto& q = sv->pending[c];
      while (!q.empty() && (int)take.size() < sv->max_batch) {
        take.push_back(std::move(q.front()));
        q.pop_front();
      }
      const size_t n = take.size();
      sv->npending -= (int64_t)n;
      ++sv->batches;
      sv->largest = std::max<int64_t>(sv->largest, (int64_t)n);
      if (sv->npending > 0) sv->cv.notify_one();  // more waits: wake another free slot
    }
    if (!dispatch(sv, s, std::move(take), (int)si)) continue;
    hipError_t e;
    while ((e = hipEventQuery(s.done)) == hipErrorNotReady) std::this_thread::yield();
    if (e != hipSuccess) {
      fail_server(sv, std::string("batch failed: ") + hipGetErrorString(e));
      s.busy = false;
      continue;
    }
    const double t = now_s();
    float dev_ms = -1.0f;
    if (hipEventElapsedTime(&dev_ms, s.start, s.done) != hipSuccess) dev_ms = -1.0f;
    const size_t n = s.batch.size();
    DoneBatch db;  // built outside the lock: one record per batch, reusing a polled one's storage
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (!sv->spare.empty()) {
        db = std::move(sv->spare.back());
        sv->spare.pop_back();
      }
    }
    db.next = db.pos = 0;
    db.seq = s.seq;
    db.tags.resize(n);
    db.ks.resize(n);
    db.latency.resize(n);
    db.ids.clear();
    db.dists.clear();
    for (size_t i = 0; i < n; ++i) {
      db.tags[i] = s.batch[i].tag;
      db.ks[i] = s.batch[i].k;
      db.latency[i] = t - s.batch[i].t_submit;
      const size_t k = (size_t)s.batch[i].k;
      db.ids.insert(db.ids.end(), s.h_ids + i * K, s.h_ids + i * K + k);
      db.dists.insert(db.dists.end(), s.h_dists + i * K, s.h_dists + i * K + k);
    }
    s.batch.clear();
    s.busy = false;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (s.seq >= 0) {
        sv->records[(size_t)s.seq].t_done = t;
        sv->records[(size_t)s.seq].device_ms = dev_ms;
      }
      sv->done.push_back(std::move(db));
      sv->completed += (int64_t)n;
    }
    sv->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

int qg_server_create(qg_index* idx, int32_t streams, int32_t max_batch, int32_t k_max, int32_t ef_max,
                     qg_server** out) {
  if (!out) return qgi::set_error(QG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!idx) return qgi::set_error(QG_EINVAL, "index is NULL");
  if (streams < 1 || streams > 16) return qgi::set_error(QG_EINVAL, "streams must be in [1, 16]");
  if (max_batch < 1 || max_batch > (1 << 20)) return qgi::set_error(QG_EINVAL, "max_batch must be in [1, 2^20]");
  if (k_max < 1 || k_max > QG_MAX_K || ef_max < 1 || ef_max > QG_MAX_EF)
    return qgi::set_error(QG_EINVAL, "k_max or ef_max out of range");
  qg_server* sv = new qg_server;
  sv->idx = idx;
  sv->device = qgi::device_of(idx);
  sv->D = qgi::dim_of(idx);
  sv->k_max = k_max;
  sv->ef_max = ef_max;
  sv->max_batch = max_batch;
  int old = 0;
  (void)hipGetDevice(&old);
  (void)hipSetDevice(sv->device);
  sv->slots.resize(streams);
  bool ok = true;
  for (auto& s : sv->slots) ok = ok && init_slot(sv, s);
  (void)hipSetDevice(old);
  if (!ok) {
    for (auto& s : sv->slots) free_slot(s);
    delete sv;
    return qgi::set_error(QG_ENOMEM, "server buffers or streams");
  }
  for (size_t i = 0; i < sv->slots.size(); ++i) sv->workers.emplace_back(slot_loop, sv, i);
  *out = sv;
  return QG_OK;
}

int qg_server_set_stop(qg_server* sv, const qg_stop_params* stop) {
  if (!sv) return qgi::set_error(QG_EINVAL, "server is NULL");
  if (stop && (!stop->mlp || stop->trace_max != 0 || stop->t_min < 1 || stop->t_every < 1))
    return qgi::set_error(QG_EINVAL, "the stop needs the MLP parameters, t_min, t_every >= 1 and no trace");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->npending > 0 || sv->completed < sv->submitted)
    return qgi::set_error(QG_EINVAL, "requests are waiting or in flight");
  if (stop) {
    // the worker is idle (nothing waits or runs) and dispatches only under
    // this lock, so slot 0 is free: load the stop kernels there first
    int old = 0;
    (void)hipGetDevice(&old);
    (void)hipSetDevice(sv->device);
    const bool ok = warm_up(sv, sv->slots[0], stop);
    (void)hipSetDevice(old);
    if (!ok) return qgi::set_error(QG_EDEVICE, "warm-up of the stop kernels failed");
  }
  sv->use_stop = stop != nullptr;
  if (stop) sv->stop_params = *stop;
  return QG_OK;
}

int qg_server_submit(qg_server* sv, const float* query, int32_t k, int32_t ef, uint64_t tag) {
  if (!sv || !query) return qgi::set_error(QG_EINVAL, "server or query is NULL");
  if (k < 1 || k > sv->k_max || ef < 1 || ef > sv->ef_max)
    return qgi::set_error(QG_EINVAL, "k or ef outside the server's bounds");
  Request r;
  r.tag = tag;
  r.k = k;
  r.ef = ef;
  r.q.assign(query, query + sv->D);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->error != QG_OK) return qgi::set_error(sv->error, sv->errmsg);
    if (sv->stop) return qgi::set_error(QG_EINVAL, "server is stopping");
    r.t_submit = now_s();
    sv->pending[ef_class(ef)].push_back(std::move(r));
    ++sv->npending;
    ++sv->submitted;
  }
  sv->cv.notify_one();
  return QG_OK;
}

}  // extern "C"

namespace {
// The beam of (k, target) from the recall map, or 0 when no row covers it
// (called with the server's lock held or before its threads read the map).
int32_t beam_for(const qg_server* sv, int32_t k, float target) {
  for (const auto& r : sv->recall_map)
    if (r.k == k && r.target >= target) return r.ef;
  return 0;
}
}  // namespace

extern "C" {

int qg_server_set_recall_map(qg_server* sv, const int32_t* k, const float* target, const int32_t* ef, int32_t n) {
  if (!sv || n < 0 || (n > 0 && (!k || !target || !ef))) return qgi::set_error(QG_EINVAL, "bad recall map arguments");
  std::vector<qg_server::RecallRow> rows;
  for (int32_t i = 0; i < n; ++i) {
    if (k[i] < 1 || k[i] > sv->k_max || ef[i] < 1 || ef[i] > sv->ef_max || !(target[i] > 0.0f && target[i] <= 1.0f))
      return qgi::set_error(QG_EINVAL, "recall map row outside the server's bounds");
    rows.push_back({k[i], target[i], ef[i]});
  }
  std::sort(rows.begin(), rows.end(), [](const qg_server::RecallRow& a, const qg_server::RecallRow& b) {
    return a.k < b.k || (a.k == b.k && a.target < b.target);
  });
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->npending > 0 || sv->completed < sv->submitted)
    return qgi::set_error(QG_EINVAL, "requests are waiting or in flight");
  sv->recall_map = std::move(rows);
  return QG_OK;
}

int qg_server_submit_target(qg_server* sv, const float* query, int32_t k, float target, uint64_t tag) {
  if (!sv) return qgi::set_error(QG_EINVAL, "server is NULL");
  int32_t ef;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    ef = beam_for(sv, k, target);
  }
  if (ef == 0) return qgi::set_error(QG_EINVAL, "no recall map row covers this k and target");
  return qg_server_submit(sv, query, k, ef, tag);
}

int qg_server_replay_target(qg_server* sv, const float* queries, const int32_t* k, const float* target,
                            const double* arrival_s, int64_t n) {
  if (!sv || n < 0 || (n > 0 && (!queries || !k || !target || !arrival_s)))
    return qgi::set_error(QG_EINVAL, "bad replay arguments");
  if (sv->producer.joinable()) return qgi::set_error(QG_EINVAL, "a replay is already running");
  std::vector<int32_t> ef((size_t)n);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (int64_t i = 0; i < n; ++i)
      if ((ef[(size_t)i] = beam_for(sv, k[i], target[i])) == 0)
        return qgi::set_error(QG_EINVAL, "no recall map row covers a request's k and target");
  }
  sv->replay_ef = std::move(ef);  // read by the replay thread until the replay ends
  return qg_server_replay(sv, queries, k, sv->replay_ef.data(), arrival_s, n);
}

int64_t qg_server_poll(qg_server* sv, int64_t max_results, uint64_t* tags, int32_t* ids, float* dists,
                       double* latency_s, int64_t* batch) {
  if (!sv || max_results < 0) return qgi::set_error(QG_EINVAL, "server is NULL or max_results < 0");
  // Finished batches are moved out under the lock and copied into the
  // caller's arrays after it is released: first writes to fresh caller memory
  // can take page faults, and the worker must not wait for them.
  std::vector<DoneBatch> got;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    int64_t avail = 0;
    while (avail < max_results && !sv->done.empty()) {
      got.push_back(std::move(sv->done.front()));
      sv->done.pop_front();
      avail += (int64_t)(got.back().tags.size() - got.back().next);
    }
  }
  const size_t K = (size_t)sv->k_max;
  int64_t n = 0;
  for (auto& b : got) {
    while (n < max_results && b.next < b.tags.size()) {
      const size_t r = b.next++;
      if (tags) tags[n] = b.tags[r];
      if (latency_s) latency_s[n] = b.latency[r];
      if (batch) batch[n] = b.seq;
      const size_t k = (size_t)b.ks[r];
      for (size_t j = 0; j < K; ++j) {
        const bool in = j < k;
        if (ids) ids[n * K + j] = in ? b.ids[b.pos + j] : -1;
        if (dists) dists[n * K + j] = in ? b.dists[b.pos + j] : __builtin_inff();
      }
      b.pos += k;
      ++n;
    }
  }
  // only the last batch taken can be partly handed out: its rest goes back in
  // front; the others keep their storage for later batches
  if (!got.empty()) {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (got.back().next < got.back().tags.size()) {
      sv->done.push_front(std::move(got.back()));
      got.pop_back();
    }
    for (auto& b : got)
      if (sv->spare.size() < 64) sv->spare.push_back(std::move(b));
  }
  return n;
}

int qg_server_replay(qg_server* sv, const float* queries, const int32_t* k, const int32_t* ef,
                     const double* arrival_s, int64_t n) {
  if (!sv || n < 0 || (n > 0 && (!queries || !k || !ef || !arrival_s)))
    return qgi::set_error(QG_EINVAL, "bad replay arguments");
  if (sv->producer.joinable()) return qgi::set_error(QG_EINVAL, "a replay is already running");
  for (int64_t i = 0; i < n; ++i) {
    if (k[i] < 1 || k[i] > sv->k_max || ef[i] < 1 || ef[i] > sv->ef_max)
      return qgi::set_error(QG_EINVAL, "k or ef outside the server's bounds");
    if (i > 0 && !(arrival_s[i] >= arrival_s[i - 1])) return qgi::set_error(QG_EINVAL, "arrival times decrease");
  }
  sv->producer = std::thread([sv, queries, k, ef, arrival_s, n]() {
    // Open loop: request i enters at t0 + arrival_s[i], and its latency counts
    // from that time even when the producer reaches it later.  Every request
    // whose arrival time has passed is built outside the lock and queued
    // under one lock, so the producer keeps up with high offered rates.
    const double t0 = now_s();
    std::vector<Request> rs;
    for (int64_t i = 0; i < n;) {
      const double t = now_s() - t0;
      int64_t j = i;
      while (j < n && arrival_s[j] <= t) ++j;
      if (j == i) continue;  // spin until request i arrives
      rs.resize((size_t)(j - i));
      for (int64_t r = i; r < j; ++r) {
        Request& q = rs[(size_t)(r - i)];
        q.tag = (uint64_t)r;
        q.k = k[r];
        q.ef = ef[r];
        q.t_submit = t0 + arrival_s[r];
        q.src = queries + (size_t)r * sv->D;
      }
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->error != QG_OK || sv->stop) break;
        for (auto& q : rs) {
          const int c = ef_class(q.ef);
          sv->pending[c].push_back(std::move(q));
        }
        sv->npending += j - i;
        sv->submitted += j - i;
      }
      sv->cv.notify_one();
      i = j;
    }
  });
  return QG_OK;
}

int qg_server_drain(qg_server* sv, double timeout_s) {
  if (!sv) return qgi::set_error(QG_EINVAL, "server is NULL");
  if (sv->producer.joinable()) sv->producer.join();
  std::unique_lock<std::mutex> lk(sv->mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (sv->completed < sv->submitted && sv->error == QG_OK) {
    if (sv->cv_done.wait_until(lk, until) == std::cv_status::timeout) return qgi::set_error(QG_EINVAL, "drain timed out");
  }
  if (sv->error != QG_OK) return qgi::set_error(sv->error, sv->errmsg);
  return QG_OK;
}

int qg_server_stats(qg_server* sv, int64_t* submitted, int64_t* completed, int64_t* batches, int64_t* largest_batch) {
  if (!sv) return qgi::set_error(QG_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (submitted) *submitted = sv->submitted;
  if (completed) *completed = sv->completed;
  if (batches) *batches = sv->batches;
  if (largest_batch) *largest_batch = sv->largest;
  return QG_OK;
}

int64_t qg_server_batches(qg_server* sv, int64_t first, int64_t max, qg_server_batch* out) {
  if (!sv || first < 0 || max < 0 || (max > 0 && !out)) return qgi::set_error(QG_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(sv->mu);
  const int64_t have = (int64_t)sv->records.size();
  const int64_t n = std::max<int64_t>(0, std::min(max, have - first));
  if (n > 0) std::memcpy(out, sv->records.data() + first, sizeof(qg_server_batch) * (size_t)n);
  return n;
}

void qg_server_destroy(qg_server* sv) {
  if (!sv) return;
  if (sv->producer.joinable()) sv->producer.join();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv.notify_all();
  for (auto& w : sv->workers)
    if (w.joinable()) w.join();
  int old = 0;
  (void)hipGetDevice(&old);
  (void)hipSetDevice(sv->device);
  for (auto& s : sv->slots) {
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    free_slot(s);
  }
  (void)hipSetDevice(old);
  delete sv;
}

}  // extern "C"

// qg_graph.cpp -- Algorithm 2 (Indexing, Sec. 3.2) on the device: qg_build_graph.
//
// Each iteration encodes the current graph into a temporary index (the FastScan
// data of every vertex), searches every vector with Algorithm 1 (beam EF, EF
// results) through the same search kernels as queries, turns the results and
// the current neighbours into sorted candidate lists, and applies the NSG
// pruning rule; every list is replaced at once.  Then the refinement
// supplements edges up to R, random ids fill vertices with too few candidates,
// and unreachable vertices are linked from their nearest reachable vertex.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "qg.h"
#include "qg_graph.h"
#include "qg_internal.h"

namespace {

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() { (void)hipFree(p); }
  hipError_t alloc(size_t n) { return hipMalloc(&p, n); }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

int hip_err(hipError_t e, const char* what) {
  return qgi::set_error(QG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(call, what)           \
  do {                                    \
    hipError_t e_ = (call);               \
    if (e_ != hipSuccess) return hip_err(e_, what); \
  } while (0)

// Breadth-first reachability from the entry over rows of r ids (-1 = empty).
int64_t reach_from(const std::vector<int32_t>& G, int64_t n, int r, int32_t entry, std::vector<char>& seen,
                   std::vector<int32_t>& queue) {
  std::fill(seen.begin(), seen.end(), 0);
  int64_t h = 0, t = 0;
  queue[t++] = entry;
  seen[entry] = 1;
  while (h < t) {
    const int32_t u = queue[h++];
    for (int j = 0; j < r; ++j) {
      const int32_t v = G[(size_t)u * r + j];
      if (v >= 0 && !seen[v]) {
        seen[v] = 1;
        queue[t++] = v;
      }
    }
  }
  return t;
}

class DeviceScope {
 public:
  explicit DeviceScope(int dev) {
    (void)hipGetDevice(&old_);
    if (old_ != dev) (void)hipSetDevice(dev);
  }
  ~DeviceScope() { (void)hipSetDevice(old_); }

 private:
  int old_ = 0;
};

}  // namespace

extern "C" int qg_build_graph(const float* vectors, int64_t n, int32_t d, int32_t r, int32_t ef_build, int32_t iters,
                              const float* rotation, int32_t entry, const int32_t* init_graph, const int32_t* fill,
                              int32_t flags, int device, int32_t* out_graph, int64_t* out_stats) {
  if (!vectors || !rotation || !init_graph || !out_graph) return qgi::set_error(QG_EINVAL, "NULL array");
  if (n < 2 || n > 0x3fffffffLL) return qgi::set_error(QG_EINVAL, "n must be in [2, 2^30)");
  if (d <= 0 || d % 8 || r <= 0 || r > 64) return qgi::set_error(QG_EINVAL, "bad d or r");
  if (ef_build < 1 || ef_build > QG_MAX_K || iters < 0) return qgi::set_error(QG_EINVAL, "bad ef_build or iters");
  if (entry < 0 || entry >= n) return qgi::set_error(QG_EINVAL, "entry out of range");
  if (flags & ~(QG_GRAPH_REFINE | QG_GRAPH_REPAIR | QG_GRAPH_PROGRESS))
    return qgi::set_error(QG_EINVAL, "unknown flags");
  const bool refine = (flags & QG_GRAPH_REFINE) && iters > 0;
  if (refine && !fill) return qgi::set_error(QG_EINVAL, "refinement needs the fill ids");
  int ndev = 0;
  HIP_OR_FAIL(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return qgi::set_error(QG_EINVAL, "bad device");
  DeviceScope scope(device);
  const auto t0 = std::chrono::steady_clock::now();
  auto note = [&](const char* what, int i, int64_t count) {
    if (!(flags & QG_GRAPH_PROGRESS)) return;
    const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[qg_build_graph] %.1fs %s %d: %lld\n", s, what, i, (long long)count);
    std::fflush(stderr);
  };
  const int C = ef_build + r;  // candidate capacity: EF results and R old neighbours
  const int64_t chunk = std::min<int64_t>(n, 65536);
  DevBuf G, cid, cd, ncand, kidx, nkept, sids, sdist;
  HIP_OR_FAIL(G.alloc(sizeof(int32_t) * (size_t)(n * r)), "hipMalloc graph");
  HIP_OR_FAIL(cid.alloc(sizeof(int32_t) * (size_t)(n * C)), "hipMalloc candidates");
  HIP_OR_FAIL(cd.alloc(sizeof(double) * (size_t)(n * C)), "hipMalloc candidate distances");
  HIP_OR_FAIL(ncand.alloc(sizeof(int32_t) * (size_t)n), "hipMalloc candidate counts");
  HIP_OR_FAIL(kidx.alloc(sizeof(int32_t) * (size_t)(n * r)), "hipMalloc kept indices");
  HIP_OR_FAIL(nkept.alloc(sizeof(int32_t) * (size_t)n), "hipMalloc kept counts");
  HIP_OR_FAIL(sids.alloc(sizeof(int32_t) * (size_t)(chunk * ef_build)), "hipMalloc search ids");
  HIP_OR_FAIL(sdist.alloc(sizeof(float) * (size_t)(chunk * ef_build)), "hipMalloc search distances");
  HIP_OR_FAIL(hipMemcpy(G.p, init_graph, sizeof(int32_t) * (size_t)(n * r), hipMemcpyDeviceToDevice), "copy graph");

  for (int it = 0; it < iters; ++it) {
    qg_index* idx = nullptr;
    int rc = qg_build_index(vectors, n, d, G.as<int32_t>(), r, rotation, entry, device, &idx);
    if (rc) return rc;  // the message is set
    for (int64_t q0 = 0; q0 < n && rc == QG_OK; q0 += chunk) {
      const int64_t nq = std::min(chunk, n - q0);
      rc = qg_search_ex(idx, vectors + q0 * d, nq, ef_build, ef_build, 0, sids.as<int32_t>(), sdist.as<float>(),
                        nullptr);
      if (rc == QG_OK) {
        const hipError_t e = qgg::launch_candidates(vectors, d, sids.as<int32_t>(), ef_build, G.as<int32_t>(), r, q0,
                                                    nq, C, cid.as<int32_t>(), cd.as<double>(), ncand.as<int32_t>(),
                                                    nullptr);
        if (e != hipSuccess) rc = hip_err(e, "candidates");
      }
    }
    const hipError_t es = hipDeviceSynchronize();
    qg_free_index(idx);
    if (rc) return rc;
    HIP_OR_FAIL(es, "search for candidates");
    note("iteration, vertices searched", it, n);
    HIP_OR_FAIL(qgg::launch_nsg(vectors, d, r, n, C, cid.as<int32_t>(), cd.as<double>(), ncand.as<int32_t>(),
                                G.as<int32_t>(), kidx.as<int32_t>(), nkept.as<int32_t>(), nullptr),
                "NSG pruning");
    if (flags & QG_GRAPH_PROGRESS) {
      HIP_OR_FAIL(hipDeviceSynchronize(), "NSG pruning");
      note("iteration, lists pruned", it, n);
    }
  }
  if (refine)
    HIP_OR_FAIL(qgg::launch_refine(vectors, d, r, n, C, 1, cid.as<int32_t>(), ncand.as<int32_t>(),
                                   kidx.as<int32_t>(), nkept.as<int32_t>(), fill, G.as<int32_t>(), nullptr),
                "refinement");
  HIP_OR_FAIL(hipDeviceSynchronize(), "graph construction");
  if (refine) note("refinement done", iters - 1, n);

  int64_t stats[4] = {0, 0, 0, 0};
  if (flags & QG_GRAPH_REPAIR) {
    // An addition to the paper, in rounds.  A round finds the vertices
    // unreachable from the entry; each such v runs Algorithm 1 on the current
    // graph (beam ef_build, ef_build results) and picks the nearest result
    // that still has a slot not taken by an earlier repair (every result was
    // visited from the entry, so it is reachable).  Per picked vertex w in
    // increasing id, its v's in increasing id take w's empty slots in slot
    // order, then w's edges not taken by a repair, farthest first (fp64, ties
    // to the larger id).  Rounds repeat until every vertex is reachable or a
    // round links none.
    std::vector<int32_t> H((size_t)(n * r));
    HIP_OR_FAIL(hipMemcpy(H.data(), G.p, sizeof(int32_t) * H.size(), hipMemcpyDeviceToHost), "download graph");
    std::vector<char> seen((size_t)n), fixed((size_t)(n * r), 0);
    std::vector<int32_t> queue((size_t)n), unr, ws, ids;
    std::vector<int64_t> pick;
    std::vector<double> rowd;
    DevBuf unr_d, qv_d, ws_d, rowd_d;
    int64_t cap = 0, wcap = 0;
    stats[0] = reach_from(H, n, r, entry, seen, queue);
    note("repair, reachable before", 0, stats[0]);
    for (int round = 0; round < 64; ++round) {
      const int64_t reached = reach_from(H, n, r, entry, seen, queue);
      if (round) note("repair round, reachable", round, reached);
      if (reached == n) break;
      unr.clear();
      for (int64_t v = 0; v < n; ++v)
        if (!seen[(size_t)v]) unr.push_back((int32_t)v);
      const int64_t nu = (int64_t)unr.size();
      if (nu > cap) {
        cap = nu;
        (void)hipFree(unr_d.p);
        (void)hipFree(qv_d.p);
        unr_d.p = qv_d.p = nullptr;
        HIP_OR_FAIL(unr_d.alloc(sizeof(int32_t) * (size_t)cap), "hipMalloc");
        HIP_OR_FAIL(qv_d.alloc(sizeof(float) * (size_t)(cap * d)), "hipMalloc");
      }
      HIP_OR_FAIL(hipMemcpy(unr_d.p, unr.data(), sizeof(int32_t) * (size_t)nu, hipMemcpyHostToDevice), "upload");
      HIP_OR_FAIL(hipMemcpy(G.p, H.data(), sizeof(int32_t) * H.size(), hipMemcpyHostToDevice), "upload graph");
      HIP_OR_FAIL(qgg::launch_gather(vectors, d, unr_d.as<int32_t>(), nu, qv_d.as<float>(), nullptr), "gather");
      qg_index* idx = nullptr;
      int rc = qg_build_index(vectors, n, d, G.as<int32_t>(), r, rotation, entry, device, &idx);
      if (rc) return rc;
      ids.resize((size_t)(std::min(chunk, nu) * ef_build));
      pick.assign((size_t)nu, -1);
      for (int64_t q0 = 0; q0 < nu && rc == QG_OK; q0 += chunk) {
        const int64_t nq = std::min(chunk, nu - q0);
        rc = qg_search_ex(idx, qv_d.as<float>() + q0 * d, nq, ef_build, ef_build, 0, sids.as<int32_t>(),
                          sdist.as<float>(), nullptr);
        if (rc) break;
        const hipError_t e = hipMemcpy(ids.data(), sids.p, sizeof(int32_t) * (size_t)(nq * ef_build),
                                       hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = hip_err(e, "download search results");
        for (int64_t a = 0; a < nq && rc == QG_OK; ++a) {
          int64_t w = -1;
          for (int b = 0; b < ef_build && w < 0; ++b) {
            const int32_t x = ids[(size_t)(a * ef_build + b)];
            if (x < 0) break;
            bool free_slot = false;
            for (int j = 0; j < r && !free_slot; ++j) free_slot = !fixed[(size_t)((int64_t)x * r + j)];
            if (free_slot) w = x;
          }
          if (w >= 0) pick[(size_t)(q0 + a)] = (int64_t)((uint64_t)w << 32 | (uint32_t)unr[(size_t)(q0 + a)]);
        }
      }
      qg_free_index(idx);
      if (rc) return rc;
      std::sort(pick.begin(), pick.end());
      ws.clear();
      for (int64_t x : pick)
        if (x >= 0 && (ws.empty() || ws.back() != (int32_t)(x >> 32))) ws.push_back((int32_t)(x >> 32));
      const int64_t nw = (int64_t)ws.size();
      if (nw > wcap) {
        wcap = nw;
        (void)hipFree(ws_d.p);
        (void)hipFree(rowd_d.p);
        ws_d.p = rowd_d.p = nullptr;
        HIP_OR_FAIL(ws_d.alloc(sizeof(int32_t) * (size_t)wcap), "hipMalloc");
        HIP_OR_FAIL(rowd_d.alloc(sizeof(double) * (size_t)(wcap * r)), "hipMalloc");
      }
      rowd.resize((size_t)(nw * r));
      HIP_OR_FAIL(hipMemcpy(ws_d.p, ws.data(), sizeof(int32_t) * (size_t)nw, hipMemcpyHostToDevice), "upload");
      HIP_OR_FAIL(qgg::launch_rows_dist(vectors, d, r, ws_d.as<int32_t>(), nw, G.as<int32_t>(), rowd_d.as<double>(),
                                        nullptr),
                  "row distances");
      HIP_OR_FAIL(hipMemcpy(rowd.data(), rowd_d.p, sizeof(double) * rowd.size(), hipMemcpyDeviceToHost), "download");
      int64_t made = 0;
      size_t a = 0;
      while (a < pick.size() && pick[a] < 0) ++a;
      for (int64_t g = 0; g < nw; ++g) {
        const int64_t w = ws[(size_t)g];
        int32_t* row = H.data() + (size_t)(w * r);
        const double* dr = rowd.data() + (size_t)(g * r);
        std::vector<int> slots;
        for (int j = 0; j < r; ++j)
          if (row[j] < 0) slots.push_back(j);  // empty slots first, in slot order
        const size_t nempty = slots.size();
        for (int j = 0; j < r; ++j)
          if (row[j] >= 0 && !fixed[(size_t)(w * r + j)]) slots.push_back(j);
        std::stable_sort(slots.begin() + (std::ptrdiff_t)nempty, slots.end(), [&](int x, int y) {
          return dr[x] > dr[y] || (dr[x] == dr[y] && row[x] > row[y]);  // farthest first, ties to the larger id
        });
        size_t next = 0;
        for (; a < pick.size() && (pick[a] >> 32) == w; ++a) {
          if (next >= slots.size()) continue;  // no slot left: this v waits for the next round
          const int j = slots[next++];
          row[j] = (int32_t)(pick[a] & 0xffffffff);
          fixed[(size_t)(w * r + j)] = 1;
          ++stats[1];
          ++made;
        }
      }
      if (!made) break;
    }
    stats[2] = reach_from(H, n, r, entry, seen, queue);
    HIP_OR_FAIL(hipMemcpy(G.p, H.data(), sizeof(int32_t) * H.size(), hipMemcpyHostToDevice), "upload graph");
    if (stats[2] != n) return qgi::set_error(QG_EUNSUPPORTED, "connectivity repair could not reach every vertex");
  }
  HIP_OR_FAIL(hipMemcpy(out_graph, G.p, sizeof(int32_t) * (size_t)(n * r), hipMemcpyDeviceToDevice), "copy graph");
  HIP_OR_FAIL(hipDeviceSynchronize(), "copy graph");
  stats[3] = std::chrono::duration_cast<std::chrono::microseconds>(std::chrono::steady_clock::now() - t0).count();
  if (out_stats) std::memcpy(out_stats, stats, sizeof stats);
  return QG_OK;
}

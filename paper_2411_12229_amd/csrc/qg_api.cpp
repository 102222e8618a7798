// qg_api.cpp -- host side of libqg: index lifetime, file I/O, argument checks,
// scratch management and kernel launches (C ABI declared in include/qg.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "qg.h"
#include "qg_internal.h"
#include "qg_kernels.h"
#include "qg_layout.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return QG_EDEVICE;
}

#define HIP_TRY(call, what)                      \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr int kCounters = 4;
constexpr int kTimingSlots = 4096;

// FNV-1a 64 over a byte range (file checksum).
uint64_t fnv1a(uint64_t h, const uint8_t* p, size_t n) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ULL;
  }
  return h;
}

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&old_);
    if (old_ != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() { (void)hipSetDevice(old_); }

 private:
  int old_ = 0;
};

}  // namespace

struct qg_index {
  bool owns_data = true;  // false for a view: rot and blocks belong to another handle
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0;
  int D = 0, R = 0, entry = 0;
  int64_t block_bytes = 0;
  float* rot = nullptr;       // M, [D][D]
  uint8_t* blocks = nullptr;  // [N][block_bytes]
  // scratch for searches
  float* qrot = nullptr;
  int64_t qrot_cap = 0;  // queries
  int32_t* overflow = nullptr;
  int64_t overflow_cap = 0;
  int* counters = nullptr;
  uint32_t* fb_bits = nullptr;
  int fb_slots = 0;
  int64_t fb_words = 0;
  // launch shape chosen by qg_autotune: wavefronts per workgroup (preferred,
  // halved while the LDS does not fit) and visited-hash slots per beam entry
  int wpb_pref = 4;
  int hash_factor = 3;
  int cu_waves = 0;  // cap on resident wavefronts per compute unit (0 = as many as fit)
  int cus = 256;     // compute units of the device (read at creation; sizes the persistent grid)
  bool beam_regs = true;  // beams of at most 128 entries live in registers (else in LDS)
  bool lut_pad = true;    // LUT layout: a padding row between lane groups (else packed rows)
  bool lut32 = false;     // LUT entries int32 (else int16), for the plain and mixed main pass
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev[2];  // pairs per kernel class
  int ev_used[2] = {0, 0};
};

static int validate_shape(int64_t n, int d, int r) {
  if (n <= 0 || n > 0x7fffffffLL) return fail(QG_EINVAL, "n must be in [1, 2^31)");
  if (d <= 0 || r <= 0) return fail(QG_EINVAL, "d and r must be positive");
  if (!qgk::shape_supported(d, r))
    return fail(QG_EUNSUPPORTED, "unsupported (d, r) = (" + std::to_string(d) + ", " + std::to_string(r) + ")");
  return QG_OK;
}

static int alloc_common(qg_index* idx) {
  int cus = 0;
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, idx->device), "compute unit count");
  idx->cus = cus > 0 ? cus : 1;
  HIP_TRY(hipMalloc(&idx->rot, sizeof(float) * idx->D * idx->D), "hipMalloc rotation");
  HIP_TRY(hipMalloc(&idx->blocks, (size_t)(idx->N * idx->block_bytes)), "hipMalloc blocks");
  HIP_TRY(hipMalloc(&idx->counters, sizeof(int) * kCounters), "hipMalloc counters");
  HIP_TRY(hipMemset(idx->counters, 0, sizeof(int) * kCounters), "hipMemset counters");
  idx->fb_slots = 64;
  idx->fb_words = (idx->N + 31) / 32;
  HIP_TRY(hipMalloc(&idx->fb_bits, sizeof(uint32_t) * (size_t)(idx->fb_words * idx->fb_slots)), "hipMalloc bitsets");
  return QG_OK;
}

static void release(qg_index* idx) {
  if (!idx) return;
  DeviceGuard g(idx->device);
  if (idx->owns_data) {
    (void)hipFree(idx->rot);
    (void)hipFree(idx->blocks);
  }
  (void)hipFree(idx->qrot);
  (void)hipFree(idx->overflow);
  (void)hipFree(idx->counters);
  (void)hipFree(idx->fb_bits);
  for (auto& v : idx->ev)
    for (auto e : v) (void)hipEventDestroy(e);
  delete idx;
}

static int ensure_scratch(qg_index* idx, int64_t nq) {
  if (nq > idx->qrot_cap) {
    int64_t cap = std::max<int64_t>(nq, 1024);
    (void)hipFree(idx->qrot);
    idx->qrot = nullptr;
    idx->qrot_cap = 0;
    HIP_TRY(hipMalloc(&idx->qrot, sizeof(float) * (size_t)(cap * idx->D)), "hipMalloc rotated queries");
    idx->qrot_cap = cap;
  }
  if (nq > idx->overflow_cap) {
    int64_t cap = std::max<int64_t>(nq, 1024);
    (void)hipFree(idx->overflow);
    idx->overflow = nullptr;
    idx->overflow_cap = 0;
    HIP_TRY(hipMalloc(&idx->overflow, sizeof(int32_t) * (size_t)cap), "hipMalloc overflow list");
    idx->overflow_cap = cap;
  }
  return QG_OK;
}

static int record(qg_index* idx, int kind, bool start) {
  if (!idx->timing) return QG_OK;
  auto& v = idx->ev[kind];
  int slot = idx->ev_used[kind];
  if (start) {
    if (slot + 2 > kTimingSlots) return QG_OK;  // ring full: stop recording
    while ((int)v.size() < slot + 2) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e), "hipEventCreate");
      v.push_back(e);
    }
    HIP_TRY(hipEventRecord(v[slot], idx->stream), "hipEventRecord");
  } else {
    if (slot + 2 > (int)v.size()) return QG_OK;
    HIP_TRY(hipEventRecord(v[slot + 1], idx->stream), "hipEventRecord");
    idx->ev_used[kind] = slot + 2;
  }
  return QG_OK;
}

extern "C" {

const char* qg_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace qgi {

qg_index* make_view(const qg_index* base) {
  if (!base) {
    fail(QG_EINVAL, "index is NULL");
    return nullptr;
  }
  DeviceGuard g(base->device);
  qg_index* v = new qg_index;
  v->owns_data = false;
  v->device = base->device;
  v->N = base->N;
  v->D = base->D;
  v->R = base->R;
  v->entry = base->entry;
  v->block_bytes = base->block_bytes;
  v->rot = base->rot;
  v->blocks = base->blocks;
  v->wpb_pref = base->wpb_pref;
  v->hash_factor = base->hash_factor;
  v->lut_pad = base->lut_pad;
  v->lut32 = base->lut32;
  v->cu_waves = base->cu_waves;
  v->cus = base->cus;
  v->beam_regs = base->beam_regs;
  v->fb_slots = base->fb_slots;
  v->fb_words = base->fb_words;
  if (hipMalloc(&v->counters, sizeof(int) * kCounters) != hipSuccess ||
      hipMemset(v->counters, 0, sizeof(int) * kCounters) != hipSuccess ||
      hipMalloc(&v->fb_bits, sizeof(uint32_t) * (size_t)(v->fb_words * v->fb_slots)) != hipSuccess) {
    release(v);
    fail(QG_ENOMEM, "index view scratch");
    return nullptr;
  }
  return v;
}

int set_error(int code, const std::string& msg) { return fail(code, msg); }
int device_of(const qg_index* idx) { return idx->device; }
int dim_of(const qg_index* idx) { return idx->D; }

}  // namespace qgi

extern "C" {

void qg_free_index(qg_index* idx) { release(idx); }

int qg_set_stream(qg_index* idx, void* hip_stream) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  idx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return QG_OK;
}

int qg_index_info(const qg_index* idx, int64_t* n, int32_t* d, int32_t* r, int32_t* entry, int64_t* block_bytes) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (n) *n = idx->N;
  if (d) *d = idx->D;
  if (r) *r = idx->R;
  if (entry) *entry = idx->entry;
  if (block_bytes) *block_bytes = idx->block_bytes;
  return QG_OK;
}

// True if some vertex lists one neighbour id twice (-1 padding aside).  The
// search merges a vertex's new candidates by rank, and two equal candidate
// words would share a rank; a graph of distinct neighbours (as Algorithm 2
// builds) never has them, so such input is refused.
// id_at(u, j) gives neighbour j of vertex u.
extern "C++" {
template <class IdAt>
static bool has_repeated_id(int64_t n, int r, IdAt id_at) {
  std::vector<int32_t> stamp((size_t)n, -1);  // stamp[v] = the last list that held v
  for (int64_t u = 0; u < n; ++u)
    for (int j = 0; j < r; ++j) {
      const int32_t v = id_at(u, j);
      if (v < 0) continue;
      if (stamp[(size_t)v] == (int32_t)u) return true;
      stamp[(size_t)v] = (int32_t)u;
    }
  return false;
}
}  // extern "C++"

int qg_build_index(const float* vectors, int64_t n, int32_t d, const int32_t* graph, int32_t r,
                   const float* rotation, int32_t entry, int device, qg_index** out) {
  if (!out) return fail(QG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!vectors || !graph || !rotation) return fail(QG_EINVAL, "NULL array");
  int rc = validate_shape(n, d, r);
  if (rc) return rc;
  if (entry < 0 || entry >= n) return fail(QG_EINVAL, "entry out of range");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(QG_EINVAL, "bad device");
  DeviceGuard g(device);
  {  // every neighbour id becomes a block address in the kernels: check them all here
    std::vector<int32_t> h;
    try {
      h.resize((size_t)(n * r));
    } catch (...) {
      return fail(QG_ENOMEM, "host buffer");
    }
    HIP_TRY(hipMemcpy(h.data(), graph, sizeof(int32_t) * h.size(), hipMemcpyDeviceToHost), "copy graph");
    for (int32_t v : h)
      if (v < -1 || v >= n) return fail(QG_EINVAL, "graph id out of range");
    bool rep = false;
    try {
      rep = has_repeated_id(n, r, [&](int64_t u, int j) { return h[(size_t)(u * r + j)]; });
    } catch (...) {
      return fail(QG_ENOMEM, "host buffer");
    }
    if (rep) return fail(QG_EINVAL, "a neighbour list repeats an id");
  }
  qg_index* idx = new qg_index;
  idx->device = device;
  idx->N = n;
  idx->D = d;
  idx->R = r;
  idx->entry = entry;
  idx->block_bytes = qgl::block_bytes(d, r);
  if ((rc = alloc_common(idx)) != QG_OK) {
    release(idx);
    return rc;
  }
  float* tmp = nullptr;
  hipError_t e = hipMalloc(&tmp, sizeof(float) * (size_t)(n * d));
  if (e != hipSuccess) {
    release(idx);
    return hip_fail(e, "hipMalloc rotated vectors");
  }
  e = hipMemcpy(idx->rot, rotation, sizeof(float) * d * d, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemset(idx->blocks, 0, (size_t)(n * idx->block_bytes));
  if (e == hipSuccess) e = qgk::launch_rotate(vectors, n, d, idx->rot, tmp, nullptr, 0, nullptr);
  if (e == hipSuccess) e = qgk::launch_encode(vectors, tmp, n, d, graph, r, idx->blocks, idx->block_bytes, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(tmp);
  if (e != hipSuccess) {
    release(idx);
    return hip_fail(e, "encode");
  }
  *out = idx;
  return QG_OK;
}

int qg_load_index(const char* path, int device, qg_index** out) {
  if (!out) return fail(QG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!path) return fail(QG_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(QG_EIO, std::string("cannot open ") + path);
  uint8_t hdr[4096];
  if (std::fread(hdr, 1, sizeof hdr, f) != sizeof hdr) {
    std::fclose(f);
    return fail(QG_EFORMAT, "truncated header");
  }
  auto rd = [&](size_t off, void* dst, size_t n) { std::memcpy(dst, hdr + off, n); };
  uint32_t ver = 0, hsz = 0;
  int64_t N = 0, B = 0, off_rot = 0, off_blk = 0;
  int32_t D = 0, R = 0, entry = 0, qbits = 0;
  uint64_t payload = 0, cks = 0;
  rd(8, &ver, 4);
  rd(12, &hsz, 4);
  rd(16, &N, 8);
  rd(24, &D, 4);
  rd(28, &R, 4);
  rd(32, &entry, 4);
  rd(36, &qbits, 4);
  rd(40, &B, 8);
  rd(48, &off_rot, 8);
  rd(56, &off_blk, 8);
  rd(64, &payload, 8);
  rd(72, &cks, 8);
  if (std::memcmp(hdr, "QGINDEX1", 8) != 0 || ver != 1 || hsz != 4096) {
    std::fclose(f);
    return fail(QG_EFORMAT, "bad magic or version");
  }
  if (D <= 0 || R <= 0 || N <= 0 || qbits != 8 || entry < 0 || entry >= N || B != qgl::block_bytes(D, R) ||
      off_rot != 4096 || off_blk < off_rot + 4LL * D * D || (uint64_t)(off_blk - 4096) + (uint64_t)(N * B) != payload) {
    std::fclose(f);
    return fail(QG_EFORMAT, "inconsistent header fields");
  }
  int rc = validate_shape(N, D, R);
  if (rc) {
    std::fclose(f);
    return rc;
  }
  std::vector<uint8_t> buf;
  try {
    buf.resize(payload);
  } catch (...) {
    std::fclose(f);
    return fail(QG_ENOMEM, "host buffer");
  }
  size_t got = std::fread(buf.data(), 1, payload, f);
  uint8_t extra;
  bool trailing = std::fread(&extra, 1, 1, f) == 1;
  std::fclose(f);
  if (got != payload || trailing) return fail(QG_EFORMAT, "file size does not match header");
  if (fnv1a(0xcbf29ce484222325ULL, buf.data(), buf.size()) != cks) return fail(QG_EFORMAT, "checksum mismatch");
  {  // neighbour ids become block addresses in the kernels: all must be -1 or in [0, N)
    const uint8_t* blk0 = buf.data() + (off_blk - 4096);
    for (int64_t v = 0; v < N; ++v) {
      const int32_t* nb = reinterpret_cast<const int32_t*>(blk0 + v * B + qgl::off_nbr(D, R));
      for (int j = 0; j < R; ++j) {
        int32_t x;
        std::memcpy(&x, nb + j, 4);
        if (x < -1 || x >= N) return fail(QG_EFORMAT, "neighbour id out of range");
      }
    }
    bool rep = false;
    try {
      const int64_t off = qgl::off_nbr(D, R);
      rep = has_repeated_id(N, R, [&](int64_t u, int j) {
        int32_t x;
        std::memcpy(&x, blk0 + u * B + off + 4 * j, 4);
        return x;
      });
    } catch (...) {
      return fail(QG_ENOMEM, "host buffer");
    }
    if (rep) return fail(QG_EFORMAT, "a neighbour list repeats an id");
  }
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(QG_EINVAL, "bad device");
  DeviceGuard g(device);
  qg_index* idx = new qg_index;
  idx->device = device;
  idx->N = N;
  idx->D = D;
  idx->R = R;
  idx->entry = entry;
  idx->block_bytes = B;
  if ((rc = alloc_common(idx)) != QG_OK) {
    release(idx);
    return rc;
  }
  hipError_t e = hipMemcpy(idx->rot, buf.data(), sizeof(float) * D * D, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(idx->blocks, buf.data() + (off_blk - 4096), (size_t)(N * B), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    release(idx);
    return hip_fail(e, "upload index");
  }
  *out = idx;
  return QG_OK;
}

int qg_save_index(const qg_index* idx, const char* path) {
  if (!idx || !path) return fail(QG_EINVAL, "NULL argument");
  DeviceGuard g(idx->device);
  const int64_t rot_bytes = 4LL * idx->D * idx->D, rot_pad = (rot_bytes + 4095) / 4096 * 4096;
  const int64_t payload = rot_pad + idx->N * idx->block_bytes;
  std::vector<uint8_t> buf;
  try {
    buf.assign(payload, 0);
  } catch (...) {
    return fail(QG_ENOMEM, "host buffer");
  }
  HIP_TRY(hipStreamSynchronize(idx->stream), "hipStreamSynchronize");
  HIP_TRY(hipMemcpy(buf.data(), idx->rot, rot_bytes, hipMemcpyDeviceToHost), "download rotation");
  HIP_TRY(hipMemcpy(buf.data() + rot_pad, idx->blocks, (size_t)(idx->N * idx->block_bytes), hipMemcpyDeviceToHost),
          "download blocks");
  uint8_t hdr[4096];
  std::memset(hdr, 0, sizeof hdr);
  std::memcpy(hdr, "QGINDEX1", 8);
  const uint32_t ver = 1, hsz = 4096;
  const int32_t qbits = 8;
  const int64_t off_rot = 4096, off_blk = 4096 + rot_pad;
  const uint64_t cks = fnv1a(0xcbf29ce484222325ULL, buf.data(), buf.size());
  auto wr = [&](size_t off, const void* src, size_t n) { std::memcpy(hdr + off, src, n); };
  wr(8, &ver, 4);
  wr(12, &hsz, 4);
  wr(16, &idx->N, 8);
  wr(24, &idx->D, 4);
  wr(28, &idx->R, 4);
  wr(32, &idx->entry, 4);
  wr(36, &qbits, 4);
  wr(40, &idx->block_bytes, 8);
  wr(48, &off_rot, 8);
  wr(56, &off_blk, 8);
  wr(64, &payload, 8);
  wr(72, &cks, 8);
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(QG_EIO, std::string("cannot create ") + path);
  bool ok = std::fwrite(hdr, 1, sizeof hdr, f) == sizeof hdr && std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? QG_OK : fail(QG_EIO, "write failed");
}

int qg_rotate(const qg_index* idx, const float* in, int64_t n, float* out) {
  if (!idx || (n > 0 && (!in || !out))) return fail(QG_EINVAL, "NULL argument");
  if (n < 0) return fail(QG_EINVAL, "n < 0");
  if (n == 0) return QG_OK;
  DeviceGuard g(idx->device);
  HIP_TRY(qgk::launch_rotate(in, n, idx->D, idx->rot, out, nullptr, 0, idx->stream), "rotate");
  return QG_OK;
}

// Per-call scratch taken from the fixed device array instead of the index
// (the allocation-free entry point).
struct FixedScratch {
  float* qrot;
  int32_t* overflow;
  int* counters;
};

// Every search entry point ends here.  k and ef are the values of a uniform
// batch, or the bounds of a mixed one (k_q, ef_q: per-query device arrays).
// With fx, nothing is allocated: the rotated queries, overflow list and queue
// counters live in *fx, and no timing events are recorded.
static int search_impl(const qg_index* cidx, const float* queries, int64_t nq, int32_t k, int32_t ef,
                       const int32_t* k_q, const int32_t* ef_q, int32_t flags, const qg_stop_params* stop,
                       int32_t* out_ids, float* out_dists, int32_t* out_stats, const FixedScratch* fx = nullptr) {
  qg_index* idx = const_cast<qg_index*>(cidx);
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (nq < 0) return fail(QG_EINVAL, "nq < 0");
  if (k <= 0 || ef <= 0) return fail(QG_EINVAL, "k and ef must be positive");
  if (k > QG_MAX_K || ef > QG_MAX_EF) return fail(QG_EUNSUPPORTED, "k or ef above the supported maximum");
  if (flags & ~(QG_SEARCH_NO_ME | QG_SEARCH_SMALL_HASH | QG_SEARCH_LDS_BEAM)) return fail(QG_EINVAL, "unknown flags");
  const bool no_me = flags & QG_SEARCH_NO_ME;
  if (no_me && (ef_q || stop)) return fail(QG_EUNSUPPORTED, "QG_SEARCH_NO_ME applies to the plain search only");
  if (stop) {
    if (stop->t_min < 1 || stop->t_every < 1 || stop->trace_max < 0) return fail(QG_EINVAL, "bad stop parameters");
    if (stop->trace_max > 0 && (!stop->trace_features || !stop->trace_nn || !stop->trace_out || !stop->trace_count))
      return fail(QG_EINVAL, "NULL trace array");
    if (reinterpret_cast<uintptr_t>(stop->mlp) % 16) return fail(QG_EINVAL, "MLP parameters must be 16-byte aligned");
  }
  if (nq == 0) return QG_OK;
  if (nq > 0x7fffffffLL) return fail(QG_EINVAL, "nq too large");
  if (!queries || !out_ids || !out_dists) return fail(QG_EINVAL, "NULL array");
  DeviceGuard g(idx->device);
  int rc = fx ? QG_OK : ensure_scratch(idx, nq);
  if (rc) return rc;
  float* const qrot = fx ? fx->qrot : idx->qrot;
  int* const counters = fx ? fx->counters : idx->counters;

  const int ef_cap = (ef + 3) / 4 * 4;
  const int k_cap = (k + 3) / 4 * 4;
  // visited hash: 2^h >= F ef slots (at least 256), filled to at most one half;
  // queries that visit more finish in the overflow pass.  Past 256 entries the
  // slots grow one per beam entry, not F: a search expands about 0.4-0.6 ef
  // vertices at large beams (1M x 128: 238 at ef 512, 580 at ef 1536, at most
  // 975), and a smaller table leaves LDS for more resident queries
  int hbits = 8;
  // w/o ME the set holds every estimated vertex, not only the visited ones: up
  // to R per expansion (measured: about two thirds of them new), for about ef
  // expansions
  const int64_t hash_want =
      no_me ? (int64_t)idx->hash_factor * idx->R * (ef + 16) / 2
            : (int64_t)idx->hash_factor * std::min(ef, 256) + std::max(ef - 256, 0);
  while ((1 << hbits) < hash_want && hbits < 14) ++hbits;
  if (flags & QG_SEARCH_SMALL_HASH) hbits = 7;
  qgk::SearchArgs a{};
  a.blocks = idx->blocks;
  a.block_bytes = idx->block_bytes;
  a.N = idx->N;
  a.queries = queries;
  a.qrot = qrot;
  a.nq = nq;
  a.k = k;
  a.ef = ef;
  a.k_q = k_q;
  a.ef_q = ef_q;
  a.k_out = k;
  a.k_cap = k_cap;
  a.ef_cap = ef_cap;
  a.hash_bits = hbits;
  a.lut_pad = idx->lut_pad ? 1 : 0;
  a.flags = flags;
  a.entry = idx->entry;
  a.out_ids = out_ids;
  a.out_dists = out_dists;
  a.out_stats = out_stats;
  a.counters = counters;
  a.overflow_list = fx ? fx->overflow : idx->overflow;
  a.fb_bits = idx->fb_bits;
  a.fb_words = idx->fb_words;
  // ls_mode 1: stop only, MLP in LDS; 2: trace (and the MLP, if given, read from global memory); 3: mixed
  // batch; 4: mixed batch with the stop (MLP in LDS); 5: w/o ME
  const int ls = no_me ? 5 : ef_q ? (stop ? 4 : 3) : !stop ? 0 : (stop->trace_max == 0 && stop->mlp ? 1 : 2);
  if (stop) {
    a.ls_w = stop->mlp;
    a.ls_theta = stop->theta;
    a.ls_t_min = stop->t_min;
    a.ls_t_every = stop->t_every;
    a.tr_max = stop->trace_max;
    a.tr_feat = stop->trace_features;
    a.tr_nn = stop->trace_nn;
    a.tr_out = stop->trace_out;
    a.tr_count = stop->trace_count;
  }

  // LUT entries: int32 when chosen, for the main pass of the plain and mixed
  // modes (the overflow pass and the other modes keep int16)
  const int lb = (idx->lut32 && (ls == 0 || ls == 3)) ? 4 : 2;
  const qgl::SearchLds L = qgl::search_lds(idx->D, idx->R, ef_cap, 1 << hbits, k_cap, lb);
  const qgl::SearchLds Lf = qgl::search_lds(idx->D, idx->R, ef_cap, 0, k_cap);
  if (L.hash % 16 || L.total % 16)  // the kernels read the hash 16 bytes at a time
    return fail(QG_EUNSUPPORTED, "per-query LDS layout is not 16-byte aligned");
  const size_t lds_cap = 160 * 1024;
  const bool mlp_lds = ls == 1 || ls == 4;
  const size_t extra = mlp_lds ? qgk::mlp_lds_bytes() : 0;  // MLP image shared by a workgroup
  int wpb = mlp_lds ? 8 : idx->wpb_pref;  // 8 wavefronts share the MLP image
  while (wpb > 1 && (size_t)wpb * L.total + extra > lds_cap) wpb >>= 1;
  if ((size_t)L.total + extra > lds_cap) return fail(QG_EUNSUPPORTED, "per-query LDS exceeds the device limit");
  const size_t lds = (size_t)wpb * L.total + extra;
  const int nb = (idx->beam_regs && !(flags & QG_SEARCH_LDS_BEAM)) ? qgk::beam_regs(false, ls, ef, idx->N) : 0;
  int occ = qgk::search_occupancy(idx->D, idx->R, false, ls, nb, lb, wpb, lds);
  if (occ <= 0) occ = 1;
  if (idx->cu_waves > 0) occ = std::min(occ, std::max(1, idx->cu_waves / wpb));
  int64_t want = (nq + wpb - 1) / wpb;
  int grid = (int)std::min<int64_t>(want, (int64_t)occ * idx->cus);

  // the rotation's first workgroup also clears the queue counters (a kernel,
  // not a memset, so the call can be captured into a graph)
  if (!fx && (rc = record(idx, 0, true))) return rc;
  HIP_TRY(qgk::launch_rotate(queries, nq, idx->D, idx->rot, qrot, counters, kCounters, idx->stream),
          "rotate queries");
  if (!fx && (rc = record(idx, 0, false))) return rc;
  if (!fx && (rc = record(idx, 1, true))) return rc;
  HIP_TRY(qgk::launch_search(idx->D, idx->R, false, ls, nb, lb, a, grid, wpb, lds, idx->stream), "search");
  if (!fx && (rc = record(idx, 1, false))) return rc;
  // overflow pass: one wavefront per workgroup, one bitset each
  HIP_TRY(qgk::launch_search(idx->D, idx->R, true, ls, 0, 2, a, idx->fb_slots, 1, (size_t)Lf.total + extra,
                             idx->stream),
          "search overflow pass");
  return QG_OK;
}

int qg_search_stop(const qg_index* idx, const float* queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                   const qg_stop_params* stop, int32_t* out_ids, float* out_dists, int32_t* out_stats) {
  return search_impl(idx, queries, nq, k, ef, nullptr, nullptr, flags, stop, out_ids, out_dists, out_stats);
}

int qg_search_mixed(const qg_index* idx, const float* queries, int64_t nq, const int32_t* k_per_query,
                    const int32_t* ef_per_query, int32_t k_max, int32_t ef_max, int32_t flags, int32_t* out_ids,
                    float* out_dists, int32_t* out_stats) {
  if (nq > 0 && (!k_per_query || !ef_per_query)) return fail(QG_EINVAL, "NULL per-query k or ef array");
  return search_impl(idx, queries, nq, k_max, ef_max, k_per_query, ef_per_query, flags, nullptr, out_ids, out_dists,
                     out_stats);
}

int qg_search_mixed_stop(const qg_index* idx, const float* queries, int64_t nq, const int32_t* k_per_query,
                         const int32_t* ef_per_query, int32_t k_max, int32_t ef_max, int32_t flags,
                         const qg_stop_params* stop, int32_t* out_ids, float* out_dists, int32_t* out_stats) {
  if (nq > 0 && (!k_per_query || !ef_per_query)) return fail(QG_EINVAL, "NULL per-query k or ef array");
  if (!stop || !stop->mlp) return fail(QG_EINVAL, "a mixed batch with the stop needs the MLP parameters");
  if (stop->trace_max != 0) return fail(QG_EINVAL, "a mixed batch records no trace");
  return search_impl(idx, queries, nq, k_max, ef_max, k_per_query, ef_per_query, flags, stop, out_ids, out_dists,
                     out_stats);
}

// The autotuner over one kind of call: `call(ids, dists)` runs the search
// being tuned into outputs of nq x kcap; `mixed` selects the mixed-batch
// kernel's beam-storage rule (ef_bound is the largest beam of the batch;
// kernel modes as in search_impl: 0 plain, 3 mixed batch).
extern "C++" template <class Call>
static int autotune_impl(qg_index* idx, int64_t nq, int32_t kcap, int32_t ef_bound, bool mixed, Call call,
                         int32_t* out_wpb, int32_t* out_hash_factor, int32_t* out_cu_waves, int32_t* out_beam,
                         int32_t* out_lut, double* out_ms) {
  DeviceGuard g(idx->device);
  int32_t* ids = nullptr;
  float* dists = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int keep_wpb = idx->wpb_pref, keep_hf = idx->hash_factor, keep_cw = idx->cu_waves;
  const bool keep_beam = idx->beam_regs, keep_lut = idx->lut_pad, keep_lut32 = idx->lut32;
  int best_wpb = keep_wpb, best_hf = keep_hf, best_cw = 0, rc = QG_OK;
  bool best_beam = true, best_lut = true, best_lut32 = false;
  double best = -1.0;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(ids);
    (void)hipFree(dists);
  };
  if (hipMalloc(&ids, sizeof(int32_t) * (size_t)(nq * kcap)) != hipSuccess ||
      hipMalloc(&dists, sizeof(float) * (size_t)(nq * kcap)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(QG_ENOMEM, "autotune buffers");
  }
  // one untimed call, then the median of seven timed ones (the median, not the
  // minimum: settings within a few percent of each other are told apart by
  // their typical time, not by one lucky call)
  auto time_it = [&](double& t) {
    t = -1.0;
    if ((rc = call(ids, dists))) return;
    float ms[7];
    for (int rep = 0; rep < 7 && rc == QG_OK; ++rep) {
      if (hipEventRecord(e0, idx->stream) != hipSuccess) rc = fail(QG_EDEVICE, "hipEventRecord");
      if (!rc) rc = call(ids, dists);
      if (!rc && (hipEventRecord(e1, idx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms[rep], e0, e1) != hipSuccess))
        rc = fail(QG_EDEVICE, "timing events");
    }
    if (rc) return;
    std::sort(ms, ms + 7);
    t = ms[3];
  };
  // workgroup shape and hash size at full residency, then a cap on resident
  // wavefronts per compute unit for that shape (a batch only slightly larger
  // than the resident slots can finish sooner with fewer, less contended slots)
  idx->cu_waves = 0;
  idx->beam_regs = true;
  idx->lut_pad = true;
  idx->lut32 = false;
  for (int wpb : {1, 2, 4, 8}) {
    for (int hf : {2, 3, 4}) {
      idx->wpb_pref = wpb;
      idx->hash_factor = hf;
      double t;
      time_it(t);
      if (rc) break;
      if (best < 0 || t < best) {
        best = t;
        best_wpb = wpb;
        best_hf = hf;
      }
    }
    if (rc) break;
  }
  if (!rc) {
    idx->wpb_pref = best_wpb;
    idx->hash_factor = best_hf;
    for (int cw : {24, 20, 16}) {
      idx->cu_waves = cw;
      double t;
      time_it(t);
      if (rc) break;
      if (t < best) {
        best = t;
        best_cw = cw;
      }
    }
  }
  if (!rc && qgk::beam_regs(false, mixed ? 3 : 0, ef_bound, idx->N) > 0) {
    idx->cu_waves = best_cw;  // the beam in LDS for the best shape
    idx->beam_regs = false;
    double t;
    time_it(t);
    if (!rc && t < best) {
      best = t;
      best_beam = false;
    }
  }
  // the other LUT layouts (packed int16 rows, padded and packed int32 rows)
  // for the best setting so far
  for (int layout : {0, 3, 2}) {
    if (rc) break;
    idx->cu_waves = best_cw;
    idx->beam_regs = best_beam;
    idx->lut_pad = (layout & 1) != 0;
    idx->lut32 = (layout & 2) != 0;
    double t;
    time_it(t);
    if (!rc && t < best) {
      best = t;
      best_lut = idx->lut_pad;
      best_lut32 = idx->lut32;
    }
  }
  cleanup();
  idx->wpb_pref = rc ? keep_wpb : best_wpb;
  idx->hash_factor = rc ? keep_hf : best_hf;
  idx->cu_waves = rc ? keep_cw : best_cw;
  idx->beam_regs = rc ? keep_beam : best_beam;
  idx->lut_pad = rc ? keep_lut : best_lut;
  idx->lut32 = rc ? keep_lut32 : best_lut32;
  if (rc) return rc;
  if (out_wpb) *out_wpb = best_wpb;
  if (out_hash_factor) *out_hash_factor = best_hf;
  if (out_cu_waves) *out_cu_waves = best_cw;
  if (out_beam) *out_beam = best_beam ? 1 : 0;
  if (out_lut) *out_lut = (best_lut ? 1 : 0) | (best_lut32 ? 2 : 0);
  if (out_ms) *out_ms = best;
  return QG_OK;
}

int qg_autotune(qg_index* idx, const float* queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                int32_t* out_wpb, int32_t* out_hash_factor, int32_t* out_cu_waves, int32_t* out_beam,
                int32_t* out_lut, double* out_ms) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (nq <= 0 || !queries) return fail(QG_EINVAL, "autotuning needs queries");
  if (k < 1 || k > QG_MAX_K) return fail(QG_EINVAL, "k out of range");
  auto call = [&](int32_t* ids, float* dists) {
    return qg_search_ex(idx, queries, nq, k, ef, flags, ids, dists, nullptr);
  };
  return autotune_impl(idx, nq, k, ef, false, call, out_wpb, out_hash_factor, out_cu_waves, out_beam, out_lut,
                       out_ms);
}

int qg_autotune_mixed(qg_index* idx, const float* queries, int64_t nq, const int32_t* k_per_query,
                      const int32_t* ef_per_query, int32_t k_max, int32_t ef_max, int32_t flags, int32_t* out_wpb,
                      int32_t* out_hash_factor, int32_t* out_cu_waves, int32_t* out_beam, int32_t* out_lut,
                      double* out_ms) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (nq <= 0 || !queries || !k_per_query || !ef_per_query) return fail(QG_EINVAL, "autotuning needs queries");
  if (k_max < 1 || k_max > QG_MAX_K) return fail(QG_EINVAL, "k_max out of range");
  auto call = [&](int32_t* ids, float* dists) {
    return qg_search_mixed(idx, queries, nq, k_per_query, ef_per_query, k_max, ef_max, flags, ids, dists, nullptr);
  };
  return autotune_impl(idx, nq, k_max, ef_max, true, call, out_wpb, out_hash_factor, out_cu_waves, out_beam,
                       out_lut, out_ms);
}

int qg_set_launch(qg_index* idx, int32_t wpb, int32_t hash_factor, int32_t cu_waves, int32_t beam, int32_t lut) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8) return fail(QG_EINVAL, "wavefronts per workgroup not 1, 2, 4 or 8");
  if (hash_factor < 2 || hash_factor > 4) return fail(QG_EINVAL, "hash factor not 2, 3 or 4");
  if (cu_waves < 0 || cu_waves > 64) return fail(QG_EINVAL, "resident wavefront cap out of range");
  if (beam != 0 && beam != 1) return fail(QG_EINVAL, "beam storage not 0 (LDS) or 1 (registers)");
  if (lut < 0 || lut > 3) return fail(QG_EINVAL, "LUT layout not in 0..3 (bit 0: padded rows, bit 1: int32)");
  idx->beam_regs = beam == 1;
  idx->lut_pad = (lut & 1) != 0;
  idx->lut32 = (lut & 2) != 0;
  idx->wpb_pref = wpb;
  idx->hash_factor = hash_factor;
  idx->cu_waves = cu_waves;
  return QG_OK;
}

int qg_reserve(qg_index* idx, int64_t nq) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (nq < 0 || nq > 0x7fffffffLL) return fail(QG_EINVAL, "nq out of range");
  DeviceGuard g(idx->device);
  return ensure_scratch(idx, nq);
}

int qg_search_ex(const qg_index* idx, const float* queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                 int32_t* out_ids, float* out_dists, int32_t* out_stats) {
  return qg_search_stop(idx, queries, nq, k, ef, flags, nullptr, out_ids, out_dists, out_stats);
}

int qg_search_noalloc(const qg_index* idx, const float* queries, int64_t nq, int32_t k, int32_t ef, int32_t flags,
                      int32_t* out_ids, float* out_dists, int32_t* out_stats) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (nq < 0) return fail(QG_EINVAL, "nq < 0");
  static_assert(QG_NOALLOC_SCRATCH_BYTES == qgk::kNoAllocScratchBytes, "scratch size in qg.h");
  // layout: counters in [0, 256), then nq x d rotated queries, then nq overflow slots
  const int64_t max_nq = (QG_NOALLOC_SCRATCH_BYTES - 256) / (4LL * idx->D + 4);
  if (nq > max_nq)
    return fail(QG_EUNSUPPORTED, "nq = " + std::to_string(nq) + " exceeds the allocation-free limit of " +
                                     std::to_string(max_nq) + " queries at d = " + std::to_string(idx->D));
  if (nq == 0) return search_impl(idx, queries, nq, k, ef, nullptr, nullptr, flags, nullptr, out_ids, out_dists,
                                  out_stats);  // argument checks only
  uint8_t* base = nullptr;
  {
    DeviceGuard g(idx->device);
    HIP_TRY(qgk::noalloc_scratch(idx->device, &base), "fixed scratch address");
  }
  FixedScratch fx;
  fx.counters = reinterpret_cast<int*>(base);
  fx.qrot = reinterpret_cast<float*>(base + 256);
  fx.overflow = reinterpret_cast<int32_t*>(base + 256 + 4 * nq * idx->D);
  return search_impl(idx, queries, nq, k, ef, nullptr, nullptr, flags, nullptr, out_ids, out_dists, out_stats, &fx);
}

int qg_search(const qg_index* idx, const float* queries, int64_t nq, int32_t k, int32_t ef, int32_t* out_ids,
              float* out_dists) {
  return qg_search_ex(idx, queries, nq, k, ef, 0, out_ids, out_dists, nullptr);
}

int qg_estimate(const qg_index* cidx, const float* queries, const int32_t* vertex_of_query, int64_t nq,
                int32_t* out_S, float* out_est, float* out_dist) {
  qg_index* idx = const_cast<qg_index*>(cidx);
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  if (nq < 0) return fail(QG_EINVAL, "nq < 0");
  if (nq == 0) return QG_OK;
  if (!queries || !vertex_of_query || !out_S || !out_est || !out_dist) return fail(QG_EINVAL, "NULL array");
  DeviceGuard g(idx->device);
  int rc = ensure_scratch(idx, nq);
  if (rc) return rc;
  // vertex ids are checked on the host copy to keep every block access in bounds
  std::vector<int32_t> v((size_t)nq);
  HIP_TRY(hipMemcpyAsync(v.data(), vertex_of_query, sizeof(int32_t) * nq, hipMemcpyDeviceToHost, idx->stream),
          "copy vertex ids");
  HIP_TRY(hipStreamSynchronize(idx->stream), "hipStreamSynchronize");
  for (int32_t x : v)
    if (x < 0 || x >= idx->N) return fail(QG_EINVAL, "vertex id out of range");
  HIP_TRY(qgk::launch_rotate(queries, nq, idx->D, idx->rot, idx->qrot, nullptr, 0, idx->stream), "rotate");
  qgk::EstimateArgs a{idx->blocks, idx->block_bytes, queries, idx->qrot, vertex_of_query, out_S, out_est, out_dist,
                      idx->lut_pad ? 1 : 0};
  HIP_TRY(qgk::launch_estimate(idx->D, idx->R, a, nq, idx->stream), "estimate");
  return QG_OK;
}

int qg_copy_blocks(const qg_index* idx, int64_t first, int64_t count, void* dst) {
  if (!idx || !dst) return fail(QG_EINVAL, "NULL argument");
  if (first < 0 || count < 0 || first + count > idx->N) return fail(QG_EINVAL, "block range out of bounds");
  if (count == 0) return QG_OK;
  DeviceGuard g(idx->device);
  HIP_TRY(hipMemcpyAsync(dst, idx->blocks + first * idx->block_bytes, (size_t)(count * idx->block_bytes),
                         hipMemcpyDeviceToDevice, idx->stream),
          "copy blocks");
  return QG_OK;
}

int qg_timing(qg_index* idx, int enable) {
  if (!idx) return fail(QG_EINVAL, "index is NULL");
  idx->timing = enable != 0;
  if (enable) idx->ev_used[0] = idx->ev_used[1] = 0;
  return QG_OK;
}

int qg_timing_read(qg_index* idx, int kernel, int32_t* launches, double* total_ms) {
  if (!idx || !launches || !total_ms || kernel < 0 || kernel > 1) return fail(QG_EINVAL, "bad argument");
  DeviceGuard g(idx->device);
  double tot = 0.0;
  const int used = idx->ev_used[kernel];
  for (int i = 0; i + 1 < used; i += 2) {
    HIP_TRY(hipEventSynchronize(idx->ev[kernel][i + 1]), "hipEventSynchronize");
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, idx->ev[kernel][i], idx->ev[kernel][i + 1]), "hipEventElapsedTime");
    tot += ms;
  }
  *launches = used / 2;
  *total_ms = tot;
  return QG_OK;
}

}  // extern "C"

// Host side of the C-ABI (include/sad.h): argument checks, workspace
// planning, kernel sequencing, device status readback.
#include <climits>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <tuple>
#include <map>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sad_internal.h"

namespace sad {

// ------------------------------------------------------------------ state
struct DeviceCtx {
  char* arena = nullptr;      // per-step workspace (engine, k-mer lists, ...)
  size_t cap = 0;
  char* keep = nullptr;       // buffers that live across engine runs in one call
  size_t keep_cap = 0;
  DevStatus* st = nullptr;    // device status word
  DevStatus* h_st = nullptr;  // pinned host copy
  int64_t* h_small = nullptr; // pinned host scratch for small readbacks
  size_t h_small_cap = 0;
  // pinned staging of small uploads: copies are queued without a host wait
  // and the area is reused only after its stream has been synchronised
  char* up = nullptr;
  size_t up_cap = 0, up_off = 0;
  hipStream_t up_stream = nullptr;
  unsigned long long* phase = nullptr;  // engine phase ticks (profiling)
  long long* jobrec = nullptr;          // per-job records (profiling)
  int64_t jobrec_cap = 0;
  // captured launch sequence of the batched bucket alignment, replayed while
  // every baked-in argument is unchanged
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};  // set-up, engine, results
  std::vector<unsigned char> gkey;
  std::vector<unsigned char> last_key;  // of the previous eager call
};

static std::mutex g_mu;
static std::vector<DeviceCtx> g_ctx;
static thread_local std::string g_err;

// Caller-owned device workspace of the running call (null: the library's own
// arenas).  Buffers that live across the engine runs of one call take the
// first `keep` bytes, per-step buffers the rest.
struct CallWs {
  char* base = nullptr;
  size_t bytes = 0;
  size_t keep = 0;
  size_t bound = 0;  // a size that suffices for this call, once known
};
static thread_local CallWs* g_ws = nullptr;
static thread_local size_t g_ws_needed = 0;  // sad_workspace_needed()

// Installs the caller's workspace for the duration of one call.
struct WsScope {
  CallWs w;
  CallWs* prev;
  WsScope(void* base, size_t bytes) : prev(g_ws) {
    if (base) {
      w.base = static_cast<char*>(base);
      w.bytes = bytes;
      g_ws = &w;
    } else {
      g_ws = nullptr;
    }
  }
  ~WsScope() { g_ws = prev; }
  WsScope(const WsScope&) = delete;
  WsScope& operator=(const WsScope&) = delete;
};

// engine-kernel timing (sad_profile_enable / sad_profile_read)
static bool g_prof_on = false;   // engine kernel timing (HIP events)
static bool g_phase_on = false;  // per-phase ticks and per-job records
static bool g_tuning = false;    // sad_tune is timing candidates (no graph capture)

// SAD_LOG=1: one line on stderr per alignment-engine launch (status, expired
// waits, workspace sizes)
static bool log_enabled() {
  static const bool on = [] {
    const char* v = getenv("SAD_LOG");
    return v && atoi(v) > 0;
  }();
  return on;
}
static int64_t g_graph_captured = 0, g_graph_replayed = 0;
static double g_prof_ms = 0.0;
static int64_t g_prof_launches = 0;
static unsigned long long g_phase[6] = {0, 0, 0, 0, 0, 0};
static std::vector<long long> g_jobrec;  // records of the last profiled engine launch
static double g_tick_khz = 0.0;

struct EngineTimer {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t s;
  explicit EngineTimer(hipStream_t st) : s(st) {
    if (!g_prof_on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, s);
  }
  void stop() {
    if (a) (void)hipEventRecord(b, s);
  }
  // call after the stream has been synchronised
  void collect() {
    if (!a) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) == hipSuccess) {
      std::lock_guard<std::mutex> lk(g_mu);
      g_prof_ms += ms;
      g_prof_launches += 1;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    a = b = nullptr;
  }
  ~EngineTimer() {
    if (a) {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  }
};

static int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

int32_t report_error(int32_t code, const std::string& msg) { return fail(code, msg); }

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(SAD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

constexpr size_t kUploadBytes = 1 << 20;

static int32_t get_ctx(DeviceCtx** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ctx.size() <= dev) g_ctx.resize(dev + 1);
  DeviceCtx& c = g_ctx[dev];
  if (!c.st) {
    HIPCHK(hipMalloc(&c.st, sizeof(DevStatus)));
    HIPCHK(hipHostMalloc(&c.h_st, sizeof(DevStatus), hipHostMallocDefault));
  }
  if (!c.up) {
    if (hipHostMalloc(&c.up, kUploadBytes, hipHostMallocDefault) == hipSuccess) {
      c.up_cap = kUploadBytes;
    } else {
      c.up = nullptr;  // uploads then wait for their copy
      c.up_cap = 0;
    }
  }
  *out = &c;
  return SAD_OK;
}

// Called right after stream s has been synchronised: uploads staged for it
// have completed, so their area can be reused.
static void uploads_done(DeviceCtx* c, hipStream_t s) {
  if (c && s == c->up_stream) c->up_off = 0;
}

static int32_t ensure_host_small(DeviceCtx* c, size_t count) {
  if (count <= c->h_small_cap) return SAD_OK;
  if (c->h_small) HIPCHK(hipHostFree(c->h_small));
  c->h_small = nullptr;
  size_t n = std::max(count, (size_t)4096);
  HIPCHK(hipHostMalloc(&c->h_small, n * sizeof(int64_t), hipHostMallocDefault));
  c->h_small_cap = n;
  return SAD_OK;
}

// Plans a set of device buffers, then carves them from the grow-only arena.
struct Carver {
  struct Req {
    void** ptr;
    size_t bytes;
  };
  std::vector<Req> reqs;
  template <class T>
  void add(T*& p, size_t count) {
    reqs.push_back({reinterpret_cast<void**>(&p), count * sizeof(T)});
  }
  size_t total() const {
    size_t t = 0;
    for (auto& r : reqs) t += (r.bytes + 255) & ~size_t(255);
    return t + 256;
  }
  int32_t carve_into(char** base, size_t* cap) {
    size_t need = total();
    if (need > *cap) {
      if (*base) HIPCHK(hipFree(*base));
      *base = nullptr;
      *cap = 0;
      hipError_t e = hipMalloc(base, need);
      if (e != hipSuccess) {
        *base = nullptr;
        return fail(SAD_E_DEVICE, "workspace of " + std::to_string(need) +
                                      " bytes: " + hipGetErrorString(e));
      }
      *cap = need;
    }
    size_t off = 0;
    for (auto& r : reqs) {
      *r.ptr = *base + off;
      off += (r.bytes + 255) & ~size_t(255);
    }
    return SAD_OK;
  }
  // Fixed region [base, base + cap) of a caller workspace, with `others`
  // bytes of the workspace outside it: no growth; a shortfall is
  // SAD_E_CAPACITY, and sad_workspace_needed() reports others + the region's
  // need.
  int32_t carve_fixed(char* base, size_t cap, size_t others) {
    const size_t need = total();
    if (need > cap) {
      g_ws_needed = std::max(g_ws_needed, std::max(others + need, g_ws ? g_ws->bound : 0));
      return fail(SAD_E_CAPACITY, "caller workspace too small: " +
                                      std::to_string(others + need) + " bytes needed");
    }
    size_t off = 0;
    for (auto& r : reqs) {
      *r.ptr = base + off;
      off += (r.bytes + 255) & ~size_t(255);
    }
    return SAD_OK;
  }
  int32_t carve(DeviceCtx* c) {
    if (g_ws) return carve_fixed(g_ws->base + g_ws->keep, g_ws->bytes - g_ws->keep, g_ws->keep);
    return carve_into(&c->arena, &c->cap);
  }
  int32_t carve_keep(DeviceCtx* c) {
    if (g_ws) return carve_fixed(g_ws->base, g_ws->keep, g_ws->bytes - g_ws->keep);
    return carve_into(&c->keep, &c->keep_cap);
  }
};

// Checks a caller workspace argument and installs nothing (WsScope does).
static int32_t check_ws(void* d_ws, size_t ws_bytes) {
  g_ws_needed = 0;
  if (d_ws && (reinterpret_cast<uintptr_t>(d_ws) & 255))
    return fail(SAD_E_INVAL, "workspace must be 256-byte aligned");
  if (!d_ws && ws_bytes) return fail(SAD_E_INVAL, "null workspace with a nonzero size");
  return SAD_OK;
}

static const char* where_name(int32_t w) {
  switch (w) {
    case W_VALIDATE: return "input validation";
    case W_KMER: return "k-mer lists";
    case W_RANK: return "rank";
    case W_PART: return "partition";
    case W_UPGMA: return "guide tree";
    case W_ENGINE: return "alignment engine (row count)";
    case W_ENGINE_POOL: return "alignment engine (profile pool)";
    case W_ENGINE_TB: return "alignment engine (traceback scratch)";
    case W_ENGINE_WIDTH: return "alignment engine (profile width limit)";
    case W_ENGINE_BOUND: return "alignment engine (32-bit score bound)";
    case W_ENGINE_WAIT: return "alignment engine (queue wait limit)";
    case W_REFINE: return "refine";
    case W_ENGINE_LINK: return "alignment engine (strip boundary scratch)";
    case W_QUALITY: return "quality (class id out of range)";
    default: return "device";
  }
}

static int32_t reset_status(DeviceCtx* c, hipStream_t s) {
  static_assert(sizeof(DevStatus) % 4 == 0, "status is whole words");
  launch_fill_i32(reinterpret_cast<int32_t*>(c->st), 0, sizeof(DevStatus) / 4, s);
  return SAD_OK;
}

// Copies the status word back (synchronising the stream).
static int32_t read_status(DeviceCtx* c, hipStream_t s, DevStatus* out) {
  HIPCHK(hipMemcpyAsync(c->h_st, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  uploads_done(c, s);
  HIPCHK(hipGetLastError());
  *out = *c->h_st;
  return SAD_OK;
}

static int32_t status_to_code(const DevStatus& d) {
  if (d.code == 0) return SAD_OK;
  int64_t detail = ((int64_t)d.detail_hi << 32) | (uint32_t)d.detail_lo;
  return fail(d.code, std::string(where_name(d.where)) + ": status " + std::to_string(d.code) +
                          ", detail " + std::to_string(detail));
}

static int32_t finish(DeviceCtx* c, hipStream_t s) {
  DevStatus d{};
  int32_t r = read_status(c, s, &d);
  if (r) return r;
  return status_to_code(d);
}

// finish() and up to two small device-to-host reads in one synchronisation:
// the reads are taken whatever the status, and returned only when it is OK.
template <class T1, class T2 = int32_t>
static int32_t finish_read(DeviceCtx* c, hipStream_t s, const T1* d1, size_t n1,
                           std::vector<T1>& o1, const T2* d2 = nullptr, size_t n2 = 0,
                           std::vector<T2>* o2 = nullptr) {
  const size_t b1 = n1 * sizeof(T1), b2 = d2 ? n2 * sizeof(T2) : 0;
  const size_t off2 = (b1 + 15) & ~size_t(15);
  int32_t r = ensure_host_small(c, (off2 + b2) / 8 + 2);
  if (r) return r;
  char* h = reinterpret_cast<char*>(c->h_small);
  HIPCHK(hipMemcpyAsync(c->h_st, c->st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
  if (b1) HIPCHK(hipMemcpyAsync(h, d1, b1, hipMemcpyDeviceToHost, s));
  if (b2) HIPCHK(hipMemcpyAsync(h + off2, d2, b2, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  uploads_done(c, s);
  HIPCHK(hipGetLastError());
  const DevStatus d = *c->h_st;
  if (d.code) return status_to_code(d);
  o1.resize(n1);
  if (b1) std::memcpy(o1.data(), h, b1);
  if (o2) {
    o2->resize(n2);
    if (b2) std::memcpy(o2->data(), h + off2, b2);
  }
  return SAD_OK;
}

template <class T>
static int32_t d2h(DeviceCtx* c, const T* dptr, size_t count, std::vector<T>& out, hipStream_t s) {
  size_t words = (count * sizeof(T) + 7) / 8;
  int32_t r = ensure_host_small(c, words);
  if (r) return r;
  HIPCHK(hipMemcpyAsync(c->h_small, dptr, count * sizeof(T), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  uploads_done(c, s);
  out.resize(count);
  std::memcpy(out.data(), c->h_small, count * sizeof(T));
  return SAD_OK;
}

// Host-to-device copy of a small host array.  Staged in the context's pinned
// upload area and queued without waiting (the area is reused only after the
// stream is next synchronised); without room, a plain copy that waits.
template <class T>
static int32_t h2d(const std::vector<T>& in, T* dptr, hipStream_t s) {
  if (in.empty()) return SAD_OK;
  const size_t bytes = in.size() * sizeof(T);
  DeviceCtx* c = nullptr;
  int32_t r = get_ctx(&c);
  if (r) return r;
  if (c->up && c->up_off > 0 && s != c->up_stream) {
    // uploads pending on another stream: let them finish first
    HIPCHK(hipStreamSynchronize(c->up_stream));
    c->up_off = 0;
  }
  if (c->up && c->up_off + bytes <= c->up_cap) {
    char* src = c->up + c->up_off;
    std::memcpy(src, in.data(), bytes);
    c->up_off += (bytes + 255) & ~size_t(255);
    c->up_stream = s;
    HIPCHK(hipMemcpyAsync(dptr, src, bytes, hipMemcpyHostToDevice, s));
    return SAD_OK;
  }
  HIPCHK(hipMemcpyAsync(dptr, in.data(), bytes, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  uploads_done(c, s);
  return SAD_OK;
}

// ------------------------------------------------------------------ checks

static int64_t kmer_space(int A, int k) {
  int64_t v = 1;
  for (int u = 0; u < k; ++u) {
    v *= A;
    if (v > 65536) return -1;
  }
  return v;
}

static int32_t check_seqs(const sad_seqs* s, int k) {
  if (!s) return fail(SAD_E_INVAL, "null sequences");
  if (s->n < 0) return fail(SAD_E_INVAL, "negative sequence count");
  if (s->alphabet != 4 && s->alphabet != 20) return fail(SAD_E_INVAL, "alphabet must be 4 or 20");
  if (k < 1 || kmer_space(s->alphabet, k) < 0) return fail(SAD_E_INVAL, "k-mer length out of range");
  if (s->n > 0 && (!s->d_codes || !s->d_offsets)) return fail(SAD_E_INVAL, "null device arrays");
  if (s->total_len < 0) return fail(SAD_E_INVAL, "negative total length");
  if (s->max_len > kMaxLen) return fail(SAD_E_INVAL, "sequence longer than the library limit");
  if (s->n > 0 && s->max_len < k) return fail(SAD_E_INVAL, "sequences shorter than k");
  return SAD_OK;
}

static int32_t check_params(const sad_params* p, int A, bool need_scoring) {
  if (!p) return fail(SAD_E_INVAL, "null params");
  if (p->p < 1) return fail(SAD_E_INVAL, "p must be >= 1");
  if (p->s_max < 1) return fail(SAD_E_INVAL, "s_max must be >= 1");
  if (need_scoring) {
    if (!p->subst) return fail(SAD_E_INVAL, "null substitution matrix");
    if (p->gap_extend < 0 || p->gap_open < p->gap_extend)
      return fail(SAD_E_INVAL, "gaps must satisfy gap_open >= gap_extend >= 0");
    for (int a = 0; a < A; ++a)
      for (int b = 0; b < A; ++b)
        if (p->subst[a * A + b] != p->subst[b * A + a])
          return fail(SAD_E_INVAL, "substitution matrix must be symmetric");
  }
  return SAD_OK;
}

static int32_t validate_on_device(DeviceCtx* c, const sad_seqs* s, int k, hipStream_t stream) {
  int32_t r = reset_status(c, stream);
  if (r) return r;
  launch_validate(*s, k, c->st, stream);
  return finish(c, stream);
}

// The same validation, with up to two small reads of caller arrays in the
// same synchronisation (for calls whose next step is to read them).
template <class T1, class T2 = int32_t>
static int32_t validate_read(DeviceCtx* c, const sad_seqs* s, int k, hipStream_t stream,
                             const T1* d1, size_t n1, std::vector<T1>& o1,
                             const T2* d2 = nullptr, size_t n2 = 0,
                             std::vector<T2>* o2 = nullptr) {
  int32_t r = reset_status(c, stream);
  if (r) return r;
  launch_validate(*s, k, c->st, stream);
  return finish_read(c, stream, d1, n1, o1, d2, n2, o2);
}

static void chunk_sizes(int n, int p, int* w_min) {
  int m = n;
  for (int c = 0; c < p; ++c) {
    int w = (int)(((int64_t)(c + 1) * n) / p) - (int)(((int64_t)c * n) / p);
    m = std::min(m, w);
  }
  *w_min = m;
}

// ------------------------------------------------------------------ engine driver

struct TreeSet {
  // groups of leaves: group g = leaf nodes group_off[g] .. group_off[g+1]
  int ngroups;
  int nleaves;
  const int32_t* d_group_off;      // device [ngroups + 1]
  std::vector<int32_t> h_group_off;
  const uint8_t* d_codes;          // leaf sequences
  const int64_t* d_offsets;
  const int32_t* d_ids;            // leaf r = sequence d_ids[r] (or r if null)
  int64_t total_len;               // residues addressed by offsets
  int max_len;
  int kmer_k;
};

struct EngineBuffers {
  int32_t *node_W, *node_n, *node_parent;
  int64_t *node_prof, *node_up;
  int32_t *job_a, *job_b, *job_out, *job_next, *job_pending, *job_link;
  int32_t *coop_next, *coop_strips, *coop_owner, *coop_tag;
  int64_t* coop_score;
  int64_t *job_score, *job_cells, *job_ops_off;
  int32_t *queue, *queue_flag, *qctl;
  int32_t *prio, *prio_cnt;  // job priority scratch (batched launches with separate trees)
  unsigned long long* tops;
  uint16_t* prof_pool;
  int32_t* up_pool;
  uint32_t* tb;
  int32_t* bnd;
  int64_t prof_cap, up_cap, tb_words, link_words;
  int link_rows, link_stride;
  int nwg;
};

// Engine scratch sized for profiles up to wcap columns; wide_links: strip
// boundary rows hold 64-bit values (some merge may need the 64-bit DP).
static int64_t tb_words_for(int wcap) {
  int64_t strips = (wcap + 63) / 64;
  int64_t chunks = (wcap + 63 + 63) / 64;
  return strips * chunks * 16 * 64;
}

static void plan_engine(Carver& cv, EngineBuffers& e, int nnodes, int nslots, int njobs,
                        int64_t prof_cap, int64_t up_cap, int wcap, bool wide_links,
                        int grid = 0) {
  e.nwg = std::max(1, std::min(njobs, grid > 0 ? grid : engine_workgroups()));
  e.prof_cap = prof_cap;
  e.up_cap = up_cap;
  e.tb_words = tb_words_for(wcap);
  e.link_rows = std::max(1, (wcap + 63) / 64 - 1);
  e.link_stride = (wcap + 1) * (wide_links ? 2 : 1);
  e.link_words = (int64_t)e.link_rows * 2 * e.link_stride;
  cv.add(e.node_W, nnodes);
  cv.add(e.node_n, nnodes);
  cv.add(e.node_parent, nnodes);
  cv.add(e.node_prof, nnodes);
  cv.add(e.node_up, nnodes);
  cv.add(e.job_a, nslots);
  cv.add(e.job_b, nslots);
  cv.add(e.job_out, nslots);
  cv.add(e.job_next, nslots);
  cv.add(e.job_link, nslots);
  cv.add(e.coop_next, nslots);
  cv.add(e.coop_strips, nslots);
  cv.add(e.coop_owner, nslots);
  cv.add(e.coop_tag, nslots);
  cv.add(e.coop_score, nslots);
  cv.add(e.job_pending, nslots);
  cv.add(e.job_score, nslots);
  cv.add(e.job_cells, nslots);
  cv.add(e.job_ops_off, nslots);
  // merges and the helper tickets of cooperative merges
  cv.add(e.queue, (size_t)std::max(njobs, 1) * (1 + kMaxHelpers));
  cv.add(e.queue_flag, (size_t)std::max(njobs, 1) * (1 + kMaxHelpers));
  cv.add(e.qctl, 8);
  cv.add(e.prio, nslots);
  cv.add(e.prio_cnt, kPrioBins);
  cv.add(e.tops, 2);
  cv.add(e.prof_pool, (size_t)prof_cap);
  cv.add(e.up_pool, (size_t)up_cap);
  cv.add(e.tb, (size_t)e.nwg * (size_t)e.tb_words);
  cv.add(e.bnd, (size_t)e.nwg * (size_t)e.link_words);
}

// Largest persistent grid any schedule launches (up to 3 workgroups per CU;
// SAD_ENGINE_WGS_PER_CU raises the default).
static int max_grid(uint32_t mode) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  (void)mode;  // plain launches and the batched mode's vector-ALU schedules reach 3 per CU
  return std::max(engine_workgroups(), 3 * cus);
}

// Columns the profile pools of a set of trees can take: the leaves' own
// columns, then per internal node W1 + W2 <= 2 kMaxWidth columns (a wider
// child fails its merge before the parent allocates).  The t-th largest
// internal node of a tree with m leaves has at most m - t + 1 leaves (the
// internal nodes with at least s leaves form a subtree of at most m - s + 1
// nodes), so it holds at most (m - t + 1) max_len columns.
static int64_t pool_cols_bound(const std::vector<int32_t>& goff, int max_len, int64_t total_len) {
  int64_t cols = total_len + 4096;
  for (size_t g = 0; g + 1 < goff.size(); ++g) {
    const int m = goff[g + 1] - goff[g];
    for (int t = 2; t <= m; ++t) cols += std::min<int64_t>(2 * kMaxWidth, (int64_t)t * max_len);
  }
  return cols;
}

// Engine workspace (after the buffers in `base`) that suffices for any
// alignment of the groups of leaves in goff: the pool bound above, tie-byte
// scratch and boundary rows for kMaxWidth-column profiles in 64-bit values,
// the largest grid.
static size_t engine_bound_bytes(const Carver& base, const std::vector<int32_t>& goff,
                                 int max_len, int64_t total_len, int A, uint32_t mode) {
  const int N = goff.empty() ? 0 : goff.back();
  int njobs = 0;
  for (size_t g = 0; g + 1 < goff.size(); ++g) njobs += std::max(0, goff[g + 1] - goff[g] - 1);
  const int64_t cols = pool_cols_bound(goff, max_len, total_len);
  Carver cv = base;
  EngineBuffers e{};
  plan_engine(cv, e, 2 * std::max(N, 1), std::max(N, 1), njobs, cols * A, cols, kMaxWidth, true,
              max_grid(mode));
  return cv.total();
}

// Boundary rows of cooperative merges cross workgroups (and L2 slices), so
// they live in uncached device memory: one area per owner workgroup, one
// workgroup per CU.  Allocated once per device, zeroed (no word carries a tag
// before the first merge), and kept until the process ends (uncached memory
// that a kernel has read is never handed back).  SAD_COOP=0 turns
// cooperation off.
static int32_t* coop_buffer(int32_t* wgs) {
  static std::mutex mu;
  static int32_t* buf[64] = {};
  static int32_t cnt[64] = {};
  *wgs = 0;
  const char* v = getenv("SAD_COOP");
  if (v && v[0] == '0') return nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (!buf[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      return nullptr;
    void* p = nullptr;
    const size_t bytes = (size_t)cus * kCoopWordsPerWG * sizeof(int32_t);
    if (hipExtMallocWithFlags(&p, bytes, hipDeviceMallocUncached) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    if (hipMemset(p, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;  // left allocated: never handed back, never used
    }
    buf[dev] = static_cast<int32_t*>(p);
    cnt[dev] = cus;
  }
  *wgs = cnt[dev];
  return buf[dev];
}

// Boundary rows of the batched engine's 32-bit strips inside a workgroup:
// tagged words, so the memory must hold nothing else and start at zero.  One
// area per workgroup, allocated for the largest grid seen (at least one
// workgroup per CU), zeroed, and kept for the process; a larger grid replaces
// it after the device has finished with the old one.
static int32_t* tag_rows(int nwg) {
  static std::mutex mu;
  static int32_t* buf[64] = {};
  static int cap[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (cap[dev] < nwg) {
    const int want = std::max(nwg, engine_workgroups());
    if (buf[dev]) {
      if (hipDeviceSynchronize() != hipSuccess) return nullptr;
      (void)hipFree(buf[dev]);
      buf[dev] = nullptr;
      cap[dev] = 0;
    }
    void* p = nullptr;
    const size_t bytes = (size_t)want * kTagRowWordsPerWG * sizeof(int32_t);
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    if (hipMemset(p, 0, bytes) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(p);
      return nullptr;
    }
    buf[dev] = static_cast<int32_t*>(p);
    cap[dev] = want;
  }
  return buf[dev];
}

static EngineArgs engine_args(const EngineBuffers& e, int njobs, int A, const int8_t* S, int go,
                              int ge, uint32_t mode, uint8_t* ops_out, DevStatus* st,
                              bool coop = true, int chunk = 32) {
  EngineArgs a{};
  a.node_W = e.node_W;
  a.node_n = e.node_n;
  a.node_prof = e.node_prof;
  a.node_up = e.node_up;
  a.node_parent = e.node_parent;
  a.prof_pool = e.prof_pool;
  a.up_pool = e.up_pool;
  a.prof_top = e.tops;
  a.up_top = e.tops + 1;
  a.prof_cap = e.prof_cap;
  a.up_cap = e.up_cap;
  a.njobs = njobs;
  a.job_a = e.job_a;
  a.job_b = e.job_b;
  a.job_out = e.job_out;
  a.job_next = e.job_next;
  a.job_link = e.job_link;
  a.job_pending = e.job_pending;
  a.job_score = e.job_score;
  a.job_cells = e.job_cells;
  a.job_ops_off = e.job_ops_off;
  a.ops_out = ops_out;
  a.queue = e.queue;
  a.queue_flag = e.queue_flag;
  a.queue_head = e.qctl;
  a.queue_tail = e.qctl + 1;
  a.queue_cap = std::max(njobs, 1) * (1 + kMaxHelpers);
  a.jobs_done = e.qctl + 3;
  a.finished = e.qctl + 4;
  a.wait_sites = e.qctl + 5;
  a.coop_next = e.coop_next;
  a.coop_strips = e.coop_strips;
  a.coop_owner = e.coop_owner;
  a.coop_tag = e.coop_tag;
  a.coop_score = e.coop_score;
  a.coop_words_per_wg = kCoopWordsPerWG;
  a.coop_wgs = 0;
  if (mode == SAD_BATCHED_MFMA) {
    a.coop_buf = coop ? coop_buffer(&a.coop_wgs) : nullptr;
    if (!a.coop_buf) a.coop_wgs = 0;
    a.trow = tag_rows(e.nwg);  // null: the launch is refused
    a.trow_words_per_wg = kTagRowWordsPerWG;
  }
  a.tb = e.tb;
  a.tb_words_per_wg = e.tb_words;
  a.bnd = e.bnd;
  a.link_words_per_wg = e.link_words;
  a.link_rows = e.link_rows;
  a.link_stride = e.link_stride;
  a.A = A;
  int smax = 0;
  for (int q = 0; q < A * A; ++q) {
    a.S[q] = S[q];
    smax = std::max(smax, std::abs((int)S[q]));
  }
  a.smax = smax;
  a.go = go;
  a.ge = ge;
  a.mode = mode;
  a.chunk = chunk == 16 ? 16 : 32;
  a.st = st;
  // queue waits end after 20 s of wall clock (a malformed DAG cannot hang)
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    khz = 100000;
  a.wait_ticks = (int64_t)khz * 1000 * 20;
  g_tick_khz = khz;
  return a;
}

// Per-phase tick accumulation of the engine kernel while profiling is on.
// nslots: job ids are below it (slot-indexed jobs may leave unused slots).
static int32_t attach_phases(DeviceCtx* c, EngineArgs& a, int nslots, hipStream_t s) {
  a.phase_acc = nullptr;
  a.job_rec = nullptr;
  a.nrec = 0;
  if (!g_phase_on) return SAD_OK;
  if (!c->phase) HIPCHK(hipMalloc(&c->phase, 8 * sizeof(unsigned long long)));
  HIPCHK(hipMemsetAsync(c->phase, 0, 8 * sizeof(unsigned long long), s));
  a.phase_acc = c->phase;
  if (nslots > c->jobrec_cap) {
    if (c->jobrec) HIPCHK(hipFree(c->jobrec));
    c->jobrec = nullptr;
    c->jobrec_cap = 0;
    HIPCHK(hipMalloc(&c->jobrec, (size_t)nslots * 8 * sizeof(long long)));
    c->jobrec_cap = nslots;
  }
  if (nslots > 0) {
    // unused slots read back as zeros
    HIPCHK(hipMemsetAsync(c->jobrec, 0, (size_t)nslots * 8 * sizeof(long long), s));
    a.job_rec = c->jobrec;
    a.nrec = nslots;
  }
  return SAD_OK;
}

static int32_t collect_phases(DeviceCtx* c, const EngineArgs& a, hipStream_t s) {
  if (!a.phase_acc) return SAD_OK;
  unsigned long long h[8];
  HIPCHK(hipMemcpyAsync(h, c->phase, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::lock_guard<std::mutex> lk(g_mu);
  for (int q = 0; q < 6; ++q) g_phase[q] += h[q];
  if (a.job_rec) {
    g_jobrec.resize((size_t)a.nrec * 8);
    HIPCHK(hipMemcpy(g_jobrec.data(), a.job_rec, g_jobrec.size() * sizeof(long long),
                     hipMemcpyDeviceToHost));
    // timestamps in nanoseconds from the launch's first job fetch; slots
    // without a job stay all zero
    long long t0 = LLONG_MAX;
    for (int64_t q = 0; q < a.nrec; ++q)
      if (g_jobrec[q * 8 + 3] != 0) t0 = std::min(t0, g_jobrec[q * 8 + 3]);
    const double ns = g_tick_khz > 0 ? 1e6 / g_tick_khz : 0.0;
    for (int64_t q = 0; q < a.nrec; ++q)
      if (g_jobrec[q * 8 + 3] != 0)
        for (int f = 3; f < 8; ++f)
          g_jobrec[q * 8 + f] = (long long)((double)(g_jobrec[q * 8 + f] - t0) * ns);
  }
  return SAD_OK;
}

// Uploads tops (prof_top, up_top) and resets the queue control words.
__global__ void init_engine_ctl_kernel(unsigned long long* tops, unsigned long long prof0,
                                       unsigned long long up0, int32_t* qctl) {
  tops[0] = prof0;
  tops[1] = up0;
  // queue head, tail, next guide tree, merges done, finished
  for (int q = 0; q < 8; ++q) qctl[q] = 0;
}

// Progressive alignment of every group of leaves along its UPGMA tree.
// Merge lists (local ids) must already be in d_merges at slots of
// h_group_off.  Outputs per slot: score/cells; colmap of every leaf residue;
// width per group.
struct TreeOutputs {
  int32_t* d_colmap;
  int32_t* d_width;
  int64_t* d_score;
  int64_t* d_cells;
  int64_t* d_cells_total;
  bool keep_engine;   // leave engine buffers for the caller to read nodes
};

// Guide trees built inside the engine launch (instead of merges given up
// front): k-mer similarity matrices per group and where the merges go.
struct FusedTrees {
  uint32_t* const* F;            // carved with the caller's buffers (base carver)
  int64_t* const* d_fm_off;
  int32_t* d_merges;
  uint64_t* const* Sw;           // pair sums of groups too large for LDS (or null)
  // after each carve (a regrown workspace loses earlier contents): host
  // upload of the matrix offsets, then the kernels that fill the matrices
  std::function<int32_t()> upload;
  std::function<void(hipStream_t)> kernels;
  // captured into the context's one hipGraph when its arguments repeat (off
  // for a second tree set in the same pass, which would evict the first's)
  bool graph = true;
};

static bool graphs_enabled() {
  const char* v = getenv("SAD_GRAPHS");
  return !(v && v[0] == '0');
}

static void drop_graph(DeviceCtx* c) {
  for (hipGraphExec_t& x : c->gexec) {
    if (x) (void)hipGraphExecDestroy(x);
    x = nullptr;
  }
  c->gkey.clear();
}

// Records the three parts of `enqueue(part, stream)` (kernel launches only:
// set-up, the engine launch, result kernels) on the context's capture stream
// as three graphs kept under `key` (the engine's own graph so that the
// timing events can bracket it on the caller's stream).  Any failure leaves
// the eager path in charge.
template <class F>
static void capture_graph(DeviceCtx* c, const std::vector<unsigned char>& key, F&& enqueue) {
  drop_graph(c);
  if (!c->cap_stream &&
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    c->cap_stream = nullptr;
    (void)hipGetLastError();
    return;
  }
  hipGraphExec_t ex[3] = {nullptr, nullptr, nullptr};
  bool ok = true;
  for (int part = 0; part < 3 && ok; ++part) {
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      ok = false;
      break;
    }
    enqueue(part, c->cap_stream);
    ok = hipStreamEndCapture(c->cap_stream, &g) == hipSuccess && g;
    if (ok) ok = hipGraphInstantiate(&ex[part], g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
  }
  (void)hipGetLastError();
  if (!ok) {
    for (hipGraphExec_t x : ex)
      if (x) (void)hipGraphExecDestroy(x);
    return;
  }
  for (int q = 0; q < 3; ++q) c->gexec[q] = ex[q];
  c->gkey = key;
  std::lock_guard<std::mutex> lk(g_mu);
  ++g_graph_captured;
}

// Tree levels for level-by-level launches: a job's level is one more than its
// children's (leaf-leaf merges are level 0).  Writes the jobs grouped by
// level into the queue (all flags set) and the level offsets to lvl_off.
static int32_t plan_levels(DeviceCtx* c, const TreeSet& ts, const int32_t* d_merges,
                           EngineBuffers& e, int njobs, std::vector<int32_t>* lvl_off,
                           hipStream_t stream) {
  const int N = ts.nleaves;
  std::vector<int32_t> merges(2 * (size_t)N);
  HIPCHK(hipMemcpyAsync(merges.data(), d_merges, merges.size() * sizeof(int32_t),
                        hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  std::vector<int32_t> level(N, 0);
  int maxl = 0;
  for (int g = 0; g < ts.ngroups; ++g) {
    const int g0 = ts.h_group_off[g], ng = ts.h_group_off[g + 1] - g0;
    for (int t = 0; t + 1 < ng; ++t) {
      int l = 0;
      for (int q = 0; q < 2; ++q) {
        const int x = merges[2 * (size_t)(g0 + t) + q];
        if (x < 0 || x >= 2 * ng - 1) return fail(SAD_E_INVAL, "malformed guide tree");
        if (x >= ng) l = std::max(l, level[g0 + (x - ng)] + 1);
      }
      level[g0 + t] = l;
      maxl = std::max(maxl, l);
    }
  }
  std::vector<int32_t> cnt(maxl + 2, 0);
  for (int g = 0; g < ts.ngroups; ++g)
    for (int t = ts.h_group_off[g]; t + 1 < ts.h_group_off[g + 1]; ++t) ++cnt[level[t] + 1];
  for (int l = 0; l <= maxl; ++l) cnt[l + 1] += cnt[l];
  std::vector<int32_t> order(njobs), pos(cnt.begin(), cnt.end() - 1);
  for (int g = 0; g < ts.ngroups; ++g)
    for (int t = ts.h_group_off[g]; t + 1 < ts.h_group_off[g + 1]; ++t) order[pos[level[t]]++] = t;
  HIPCHK(hipMemcpyAsync(e.queue, order.data(), (size_t)njobs * sizeof(int32_t),
                        hipMemcpyHostToDevice, stream));
  HIPCHK(hipStreamSynchronize(stream));
  launch_fill_i32(e.queue_flag, 1, njobs, stream);
  *lvl_off = std::move(cnt);
  return SAD_OK;
}

static int32_t run_trees(DeviceCtx* c, const TreeSet& ts, const int32_t* d_merges,
                         const sad_params* prm, int A, Carver& base_cv, EngineBuffers& e,
                         const TreeOutputs& out, hipStream_t stream,
                         const FusedTrees* fused = nullptr, int grid = 0, bool coop = true,
                         bool valu_scores = false, int chunk = 32) {
  const int N = ts.nleaves;
  int njobs = 0;
  for (int g = 0; g < ts.ngroups; ++g)
    njobs += std::max(0, ts.h_group_off[g + 1] - ts.h_group_off[g] - 1);
  int wcap = std::min(kMaxWidth, std::max(2 * ts.max_len + 64, 128));
  int max_group = 0;
  for (int g = 0; g < ts.ngroups; ++g)
    max_group = std::max(max_group, ts.h_group_off[g + 1] - ts.h_group_off[g]);
  int smax = 0;
  for (int q = 0; q < A * A; ++q) smax = std::max(smax, std::abs((int)prm->subst[q]));
  const double unit = (double)std::max(std::max(smax, (int)prm->gap_open), 1);
  int64_t prof_cap = (int64_t)A * (ts.total_len * 6 + 4096);
  int64_t up_cap = ts.total_len * 6 + 4096;
  for (int attempt = 0; attempt < 8; ++attempt) {
    Carver cv = base_cv;
    // a merge takes the 64-bit DP when (W1 + W2 + 2) n1 n2 max(smax, go)
    // reaches 2^29 (n1 + n2 at most the largest group)
    const double g2 = std::floor(max_group / 2.0) * std::ceil(max_group / 2.0);
    const bool wide_links = (2.0 * wcap + 2.0) * g2 * unit >= (double)(1 << 29);
    if (g_ws) {
      // caller workspace: the profile pools take all the space the other
      // buffers leave, so a pool shortfall means the workspace is too small
      Carver probe = base_cv;
      EngineBuffers pe{};
      plan_engine(probe, pe, 2 * std::max(N, 1), std::max(N, 1), njobs, 0, 0, wcap, wide_links,
                  grid);
      const size_t avail = g_ws->bytes - g_ws->keep, fixed = probe.total() + 512;
      const int64_t cols = fixed < avail ? (int64_t)((avail - fixed) / (2 * A + 4)) : 0;
      if (cols <= ts.total_len) {
        g_ws_needed = std::max(g_ws_needed,
                               g_ws->keep + engine_bound_bytes(base_cv, ts.h_group_off,
                                                               ts.max_len, ts.total_len, A,
                                                               prm->mode));
        return fail(SAD_E_CAPACITY, "caller workspace too small for the alignment engine: " +
                                        std::to_string(g_ws_needed) + " bytes suffice");
      }
      prof_cap = cols * A;
      up_cap = cols;
    }
    plan_engine(cv, e, 2 * std::max(N, 1), std::max(N, 1), njobs, prof_cap, up_cap, wcap,
                wide_links, grid);
    int32_t r = cv.carve(c);
    if (r) return r;
    if (fused) {
      r = fused->upload();
      if (r) return r;
    }
    // device work before the engine (everything here is capturable)
    auto setup = [&](hipStream_t st) {
      reset_status(c, st);
      if (fused) fused->kernels(st);
      launch_fill_i32(e.node_parent, -1, 2 * (int64_t)std::max(N, 1), st);
      launch_fill_i32(e.job_next, -1, std::max(N, 1), st);
      launch_fill_i32(e.job_a, -1, std::max(N, 1), st);
      launch_fill_i32(e.queue_flag, 0, (int64_t)std::max(njobs, 1) * (1 + kMaxHelpers), st);
      launch_fill_i32(reinterpret_cast<int32_t*>(e.job_ops_off), -1,
                      2 * (int64_t)std::max(N, 1), st);
      init_engine_ctl_kernel<<<1, 1, 0, st>>>(e.tops, (unsigned long long)ts.total_len * A,
                                              (unsigned long long)ts.total_len, e.qctl);
      launch_make_leaves(ts.d_codes, ts.d_offsets, ts.d_ids, N, A, 0, e.node_W, e.node_n,
                         e.node_prof, e.node_up, e.node_parent, e.prof_pool, ts.total_len, st);
      launch_fill_i32(e.job_link, 0, std::max(N, 1), st);
    };
    auto results = [&](hipStream_t st) {
      if (out.d_colmap)
        launch_colmap(ts.d_offsets, ts.d_ids, N, e.node_parent, e.node_up, e.up_pool,
                      out.d_colmap, c->st, st);
      if (out.d_width) launch_widths(ts.d_group_off, ts.ngroups, N, e.node_W, out.d_width, st);
      if (out.d_cells_total)
        launch_fill_i32(reinterpret_cast<int32_t*>(out.d_cells_total), 0, 2, st);
      if (out.d_score)
        launch_job_results(e.job_a, e.job_score, e.job_cells, N, out.d_score, out.d_cells,
                           out.d_cells_total, st);
    };
    // the batched launch with its guide trees built inside has no host step
    // between setup and results: it is captured once into a hipGraph and
    // replayed while its arguments (all baked into the graph) are unchanged
    const bool graphable =
        fused && fused->graph && !g_phase_on && !g_tuning && njobs > 0 && graphs_enabled();
    // batched mode with vector-ALU scores: the plain kernel as one persistent
    // launch over the whole merge DAG (no cooperative merges)
    const uint32_t kmode = valu_scores ? SAD_PLAIN : prm->mode;
    std::vector<unsigned char> gkey;
    if (graphable) {
      EngineArgs ka = engine_args(e, njobs, A, prm->subst, prm->gap_open, prm->gap_extend,
                                  kmode, nullptr, c->st, coop, chunk);
      const uintptr_t extra[] = {(uintptr_t)ts.d_codes, (uintptr_t)ts.d_offsets,
                                 (uintptr_t)ts.d_ids, (uintptr_t)ts.d_group_off,
                                 (uintptr_t)*fused->F, (uintptr_t)*fused->d_fm_off,
                                 (uintptr_t)fused->d_merges, (uintptr_t)out.d_colmap,
                                 (uintptr_t)out.d_width, (uintptr_t)out.d_score,
                                 (uintptr_t)out.d_cells, (uintptr_t)out.d_cells_total,
                                 (uintptr_t)e.prof_pool, (uintptr_t)c->st,
                                 (uintptr_t)N, (uintptr_t)ts.ngroups, (uintptr_t)ts.total_len,
                                 (uintptr_t)A, (uintptr_t)e.nwg, (uintptr_t)stream,
                                 (uintptr_t)ts.kmer_k, (uintptr_t)ts.max_len,
                                 (uintptr_t)(fused->Sw ? *fused->Sw : nullptr)};
      gkey.resize(sizeof(ka) + sizeof(extra));
      std::memcpy(gkey.data(), &ka, sizeof(ka));
      std::memcpy(gkey.data() + sizeof(ka), extra, sizeof(extra));
      if (c->gexec[0] && c->gkey == gkey) {
        // the engine's graph is bracketed by the timing events on the stream
        HIPCHK(hipGraphLaunch(c->gexec[0], stream));
        EngineTimer timer(stream);
        HIPCHK(hipGraphLaunch(c->gexec[1], stream));
        timer.stop();
        HIPCHK(hipGraphLaunch(c->gexec[2], stream));
        {
          std::lock_guard<std::mutex> lk(g_mu);
          ++g_graph_replayed;
        }
        DevStatus d{};
        r = read_status(c, stream, &d);
        if (r) return r;
        if (d.code == 0) {
          timer.collect();
          return SAD_OK;
        }
        // a replay that reports an error is redone eagerly (which also
        // handles capacity retries)
        drop_graph(c);
      }
    }
    setup(stream);
    if (!fused)
      launch_make_jobs(d_merges, ts.d_group_off, ts.ngroups, N, N, e.node_parent, e.job_a,
                       e.job_b, e.job_out, e.job_next, e.job_pending, e.job_link, e.queue,
                       e.queue_flag, e.qctl + 1, stream);
    EngineArgs a = engine_args(e, njobs, A, prm->subst, prm->gap_open, prm->gap_extend, kmode,
                               nullptr, c->st, coop, chunk);
    if (kmode == SAD_BATCHED_MFMA && !a.trow) return SAD_E_DEVICE;
    if (fused) {
      a.up_F = *fused->F;
      a.up_fm_off = *fused->d_fm_off;
      a.up_Sw = fused->Sw ? *fused->Sw : nullptr;
      a.up_group_off = ts.d_group_off;
      a.up_ngroups = ts.ngroups;
      a.up_N = N;
      a.up_merges = fused->d_merges;
      a.up_next = e.qctl + 2;
    }
    r = attach_phases(c, a, std::max(N, 1), stream);
    if (r) return r;
    // plain mode: one launch per tree level (jobs of a level are independent)
    std::vector<int32_t> lvl_off;
    if (prm->mode == SAD_PLAIN && njobs > 0) {
      if (fused) return fail(SAD_E_INVAL, "level-by-level launches need the merges up front");
      r = plan_levels(c, ts, d_merges, e, njobs, &lvl_off, stream);
      if (r) return r;
    } else if (njobs > 0 && !fused) {
      // the ready jobs, longest estimated path to the root first
      launch_job_priorities(d_merges, ts.d_group_off, ts.ngroups, max_group, std::max(N, 1),
                            e.node_W, e.prio, e.prio_cnt, e.queue, c->st, stream);
    }
    EngineTimer timer(stream);
    if (lvl_off.empty()) {
      launch_engine(a, e.nwg, stream);
    } else {
      for (size_t l = 0; l + 1 < lvl_off.size(); ++l) {
        const int cnt = lvl_off[l + 1] - lvl_off[l];
        EngineArgs al = a;
        al.queue = e.queue + lvl_off[l];
        al.queue_flag = e.queue_flag + lvl_off[l];
        al.njobs = cnt;
        al.no_push = 1;
        launch_fill_i32(e.qctl, 0, 2, stream);
        launch_engine(al, std::max(1, std::min(cnt, e.nwg)), stream);
      }
    }
    timer.stop();
    DevStatus d{};
    r = read_status(c, stream, &d);
    if (r) return r;
    if (log_enabled()) {
      int32_t sites = 0;
      HIPCHK(hipMemcpy(&sites, a.wait_sites, sizeof(sites), hipMemcpyDeviceToHost));
      const int64_t detail = ((int64_t)d.detail_hi << 32) | (uint32_t)d.detail_lo;
      fprintf(stderr,
              "[sad] engine attempt %d: %d merges, status %d (%s, detail %lld), expired wait "
              "sites 0x%x, width cap %d, pools %lld/%lld\n",
              attempt, njobs, d.code, d.code ? where_name(d.where) : "ok", (long long)detail,
              sites, wcap, (long long)prof_cap, (long long)up_cap);
    }
    if (njobs > 0) timer.collect();
    r = collect_phases(c, a, stream);
    if (r) return r;
    if (d.code == SAD_E_CAPACITY &&
        (d.where == W_ENGINE_POOL ||
         ((d.where == W_ENGINE_TB || d.where == W_ENGINE_LINK) && wcap < kMaxWidth))) {
      if (d.where == W_ENGINE_POOL) {
        if (g_ws) {
          g_ws_needed = std::max(g_ws_needed,
                                 g_ws->keep + engine_bound_bytes(base_cv, ts.h_group_off,
                                                                 ts.max_len, ts.total_len, A,
                                                                 prm->mode));
          return fail(SAD_E_CAPACITY, "caller workspace too small for the profile pools: " +
                                          std::to_string(g_ws_needed) + " bytes suffice");
        }
        prof_cap *= 2;
        up_cap *= 2;
      } else {
        wcap = std::min(kMaxWidth, 2 * wcap);
      }
      continue;
    }
    if (d.code) return status_to_code(d);
    r = reset_status(c, stream);
    if (r) return r;
    results(stream);
    r = finish(c, stream);
    if (r || !graphable) return r;
    // capture only when the same arguments come twice in a row
    if (c->last_key != gkey) {
      c->last_key = gkey;
      return SAD_OK;
    }
    capture_graph(c, gkey, [&](int part, hipStream_t st) {
      if (part == 0) setup(st);
      if (part == 1) launch_engine(a, e.nwg, st);
      if (part == 2) results(st);
    });
    return SAD_OK;
  }
  return fail(SAD_E_CAPACITY, "alignment engine workspace did not converge");
}

// ---------------------------------------------------------------- autotune
// Schedule of the bucket alignment: persistent grid size (0 = one workgroup
// per CU times the default occupancy) and whether the guide trees are built
// inside the engine launch (-1 = default rule).  The results do not depend
// on it.  sad_tune measures the candidates on the caller's data and caches
// the fastest per workload shape; sad_align_buckets looks the shape up.
struct Schedule {
  int grid = 0;
  int fuse = -1;
  int coop = 1;  // cooperative merges (batched mode): a merge's strip groups spread over idle workgroups
  int mfma = 1;  // batched mode: column scores as int8 MFMA tiles (1) or vector-ALU dot products (0)
  int chunk = 32;  // MFMA scores: steps per chunk of the 32-bit strips (32 or 16)
};

struct TuneKey {
  int A, n, p, mode, max_n;
  int64_t total_len;
  bool operator<(const TuneKey& o) const {
    return std::tie(A, n, p, mode, max_n, total_len) <
           std::tie(o.A, o.n, o.p, o.mode, o.max_n, o.total_len);
  }
};

static std::mutex g_tune_mu;
static std::map<TuneKey, Schedule> g_tune;
static thread_local const Schedule* g_forced = nullptr;  // set while sad_tune measures

// SAD_SCHEDULE=grid,fuse[,coop[,mfma[,chunk]]] (e.g. "192,1,0") imposes one
// schedule on every call, for tests that compare each autotuner candidate with
// the oracle.
static bool schedule_from_env(Schedule* out) {
  const char* v = getenv("SAD_SCHEDULE");
  int grid = 0, fuse = -1, coop = 1, mfma = 1, chunk = 32;
  if (!v) return false;
  const int got = sscanf(v, "%d,%d,%d,%d,%d", &grid, &fuse, &coop, &mfma, &chunk);
  if (got < 2 || grid < 0 || fuse < -1 || fuse > 1 || coop < 0 || coop > 1 || mfma < 0 ||
      mfma > 1 || (chunk != 16 && chunk != 32))
    return false;
  out->grid = grid;
  out->fuse = fuse;
  out->coop = coop;
  out->mfma = mfma;
  out->chunk = chunk;
  return true;
}

static Schedule schedule_for(const TuneKey& k) {
  if (g_forced) return *g_forced;
  Schedule env{};
  if (schedule_from_env(&env)) return env;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(k);
  return it == g_tune.end() ? Schedule{} : it->second;
}

}  // namespace sad

// ====================================================================== C-ABI

using namespace sad;

namespace sad {
struct KmerRankBufs {
  uint32_t* entries;
  int32_t *nu, *sorted;
  uint64_t* kloc;
};
static void plan_kmer_rank(Carver& cv, KmerRankBufs& b, int n, int64_t total_len) {
  cv.add(b.entries, (size_t)std::max<int64_t>(total_len, 1));
  cv.add(b.nu, std::max(n, 1));
  cv.add(b.kloc, std::max(n, 1));
  cv.add(b.sorted, std::max(n, 1));
}
}  // namespace sad

extern "C" int32_t sad_kmer_rank_workspace(const sad_seqs* seqs, const sad_params* prm,
                                           size_t* ws_bytes) {
  if (!prm || !ws_bytes) return fail(SAD_E_INVAL, "null argument");
  int32_t r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  Carver cv;
  KmerRankBufs b{};
  plan_kmer_rank(cv, b, seqs->n, seqs->total_len);
  *ws_bytes = cv.total();
  return SAD_OK;
}

extern "C" int32_t sad_kmer_rank(const sad_seqs* seqs, const sad_params* prm, uint64_t* d_key,
                                 int32_t* d_sample_ids, int32_t sample_cap, int32_t* n_samples,
                                 void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!prm) return fail(SAD_E_INVAL, "null params");
  int32_t r = check_ws(d_ws, ws_bytes);
  if (r) return r;
  WsScope wss(d_ws, ws_bytes);
  r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  r = check_params(prm, seqs->alphabet, false);
  if (r) return r;
  const int n = seqs->n, p = prm->p, A = seqs->alphabet, k = prm->kmer_k;
  if (n < 2 * p) return fail(SAD_E_INVAL, "need N >= 2p");
  if (!d_key || !n_samples || (!d_sample_ids && sample_cap > 0))
    return fail(SAD_E_INVAL, "null output");
  int w_min = 0;
  chunk_sizes(n, p, &w_min);
  int ks = std::min(p - 1, std::min(std::max(1, prm->s_max / p), w_min - 1));
  const int S = p * ks;
  *n_samples = S;
  if (S > sample_cap) return fail(SAD_E_CAPACITY, "sample capacity too small");
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  r = validate_on_device(c, seqs, k, stream);
  if (r) return r;
  const int kspace = (int)kmer_space(A, k);
  Carver cv;
  KmerRankBufs b{};
  plan_kmer_rank(cv, b, n, seqs->total_len);
  r = cv.carve(c);
  if (r) return r;
  uint32_t* entries = b.entries;
  int32_t *nu = b.nu, *sorted = b.sorted;
  uint64_t* kloc = b.kloc;
  r = reset_status(c, stream);
  if (r) return r;
  launch_kmer_lists(seqs->d_codes, seqs->d_offsets, n, A, k, entries, nullptr, nu, c->st, stream);
  KmerLists kl{entries, seqs->d_offsets, nu, seqs->d_offsets};
  launch_rowsum_chunk(kl, n, p, k, kspace, kloc, stream);
  launch_chunk_sort(kloc, n, p, sorted, stream);
  launch_pick_samples(sorted, n, p, ks, d_sample_ids, stream);
  launch_rowsum_list(kl, n, d_sample_ids, S, k, kspace, d_key, c->st, stream);
  return finish(c, stream);
}

extern "C" int32_t sad_rank_against(const sad_seqs* seqs, int32_t kmer_k,
                                    const int32_t* d_sample_ids, int32_t n_samples,
                                    uint64_t* d_key, hipStream_t stream) {
  int32_t r = check_seqs(seqs, kmer_k);
  if (r) return r;
  const int n = seqs->n, A = seqs->alphabet, k = kmer_k;
  if (!d_sample_ids) n_samples = n;
  if (n_samples < 0) return fail(SAD_E_INVAL, "negative sample count");
  if (n > 0 && !d_key) return fail(SAD_E_INVAL, "null output");
  if (n == 0) return SAD_OK;
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  r = validate_on_device(c, seqs, k, stream);
  if (r) return r;
  const int kspace = (int)kmer_space(A, k);
  uint32_t* entries;
  int32_t* nu;
  Carver cv;
  cv.add(entries, (size_t)std::max<int64_t>(seqs->total_len, 1));
  cv.add(nu, std::max(n, 1));
  r = cv.carve(c);
  if (r) return r;
  r = reset_status(c, stream);
  if (r) return r;
  launch_kmer_lists(seqs->d_codes, seqs->d_offsets, n, A, k, entries, nullptr, nu, c->st, stream);
  KmerLists kl{entries, seqs->d_offsets, nu, seqs->d_offsets};
  launch_rowsum_list(kl, n, d_sample_ids, n_samples, k, kspace, d_key, c->st, stream);
  return finish(c, stream);
}

extern "C" int32_t sad_partition_workspace(const sad_seqs* seqs, const sad_params* prm,
                                           size_t* ws_bytes) {
  if (!seqs || !prm || !ws_bytes) return fail(SAD_E_INVAL, "null argument");
  int32_t r = check_params(prm, seqs->alphabet, false);
  if (r) return r;
  if (seqs->n < 2 * prm->p) return fail(SAD_E_INVAL, "need N >= 2p");
  char* base = nullptr;
  Carver cv;
  cv.add(base, partition_scratch(seqs->n, prm->p, nullptr, nullptr));
  *ws_bytes = cv.total();
  return SAD_OK;
}

extern "C" int32_t sad_partition(const sad_seqs* seqs, const uint64_t* d_key, const sad_params* prm,
                                 uint64_t* d_pivot_key, int32_t* d_pivot_id, int32_t* d_bucket,
                                 int32_t* d_bucket_off, int32_t* d_members, void* d_ws,
                                 size_t ws_bytes, hipStream_t stream) {
  if (!seqs || !prm) return fail(SAD_E_INVAL, "null argument");
  int32_t r = check_ws(d_ws, ws_bytes);
  if (r) return r;
  WsScope wss(d_ws, ws_bytes);
  r = check_params(prm, seqs->alphabet, false);
  if (r) return r;
  const int n = seqs->n, p = prm->p;
  if (n < 2 * p) return fail(SAD_E_INVAL, "need N >= 2p");
  if (!d_key || !d_bucket || !d_bucket_off || !d_members || (p > 1 && (!d_pivot_key || !d_pivot_id)))
    return fail(SAD_E_INVAL, "null device array");
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  // one block of scratch, laid out as the static-scratch variant lays it out
  const size_t need = partition_scratch(n, p, nullptr, nullptr);
  char* base = nullptr;
  Carver cv;
  cv.add(base, need);
  r = cv.carve(c);
  if (r) return r;
  PartitionScratch ps{};
  partition_scratch(n, p, base, &ps);
  r = reset_status(c, stream);
  if (r) return r;
  launch_partition_keys(d_key, n, p, ps, d_pivot_key, d_pivot_id, d_bucket, d_bucket_off,
                        d_members, stream);
  return finish(c, stream);
}

namespace sad {
// k-mer lists, bucket similarity matrices and (trees by a separate kernel)
// the UPGMA pair sums of the bucket alignment
struct AlignBufs {
  uint32_t *entries, *F;
  int32_t* nu;
  int64_t* d_fm_off;
  uint64_t* Sw;
};
static void plan_align(Carver& cv, AlignBufs& b, int n, int p, int64_t total_len,
                       int64_t fm_total, bool with_sums) {
  cv.add(b.entries, (size_t)std::max<int64_t>(total_len, 1));
  cv.add(b.nu, std::max(n, 1));
  cv.add(b.d_fm_off, std::max(p, 1));
  cv.add(b.F, (size_t)std::max<int64_t>(fm_total, 1));
  if (with_sums) cv.add(b.Sw, (size_t)std::max<int64_t>(fm_total, 1));
}

// Checks the bucket offsets read from the device; sums of squared sizes and
// the largest bucket.
static int32_t bucket_shape(const std::vector<int32_t>& off, int n, int p, int64_t* fm_total,
                            int* max_n) {
  if (off[0] != 0 || off[p] != n) return fail(SAD_E_INVAL, "bucket offsets must span 0..N");
  *fm_total = 0;
  *max_n = 0;
  for (int b = 0; b < p; ++b) {
    const int nb = off[b + 1] - off[b];
    if (nb < 0) return fail(SAD_E_INVAL, "bucket offsets must be non-decreasing");
    *fm_total += (int64_t)nb * nb;
    *max_n = std::max(*max_n, nb);
  }
  return SAD_OK;
}

// Workspace that suffices for sad_align_buckets on these buckets under any
// schedule (trees inside the launch or by a separate kernel, any grid).
static size_t align_bound(const sad_seqs* seqs, const std::vector<int32_t>& off, int p,
                          int64_t fm_total, int A, uint32_t mode) {
  Carver base;
  AlignBufs b{};
  plan_align(base, b, seqs->n, p, seqs->total_len, fm_total, true);
  return engine_bound_bytes(base, off, seqs->max_len, seqs->total_len, A, mode);
}
}  // namespace sad

extern "C" int32_t sad_align_buckets_workspace(const sad_seqs* seqs, const int32_t* d_bucket_off,
                                               const sad_params* prm, size_t* ws_bytes,
                                               hipStream_t stream) {
  if (!prm || !ws_bytes) return fail(SAD_E_INVAL, "null argument");
  int32_t r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  r = check_params(prm, seqs->alphabet, false);
  if (r) return r;
  if (!d_bucket_off) return fail(SAD_E_INVAL, "null device array");
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  std::vector<int32_t> off;
  r = reset_status(c, stream);
  if (!r) r = finish_read(c, stream, d_bucket_off, (size_t)prm->p + 1, off);
  if (r) return r;
  int64_t fm_total = 0;
  int max_n = 0;
  r = bucket_shape(off, seqs->n, prm->p, &fm_total, &max_n);
  if (r) return r;
  *ws_bytes = align_bound(seqs, off, prm->p, fm_total, seqs->alphabet, prm->mode);
  return SAD_OK;
}

extern "C" int32_t sad_align_buckets(const sad_seqs* seqs, const int32_t* d_bucket_off,
                                     const int32_t* d_members, const sad_params* prm, sad_msa* out,
                                     void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!prm || !out) return fail(SAD_E_INVAL, "null argument");
  int32_t r = check_ws(d_ws, ws_bytes);
  if (r) return r;
  WsScope wss(d_ws, ws_bytes);
  r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  r = check_params(prm, seqs->alphabet, true);
  if (r) return r;
  if (!d_bucket_off || !d_members || !out->d_colmap || !out->d_width || !out->d_merge_score ||
      !out->d_merge_list || !out->d_merge_cells || !out->d_cells)
    return fail(SAD_E_INVAL, "null device array");
  const int n = seqs->n, p = prm->p, A = seqs->alphabet, k = prm->kmer_k;
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  std::vector<int32_t> off;
  r = validate_read(c, seqs, k, stream, d_bucket_off, (size_t)p + 1, off);
  if (r) return r;
  int64_t fm_total = 0;
  int max_n = 0;
  r = bucket_shape(off, n, p, &fm_total, &max_n);
  if (r) return r;
  std::vector<int64_t> fm_off(p);
  {
    int64_t acc = 0;
    for (int b = 0; b < p; ++b) {
      const int64_t nb = off[b + 1] - off[b];
      fm_off[b] = acc;
      acc += nb * nb;
    }
  }
  if (max_n > kMaxGroup) return fail(SAD_E_CAPACITY, "bucket larger than the library limit");
  if (g_ws) g_ws->bound = align_bound(seqs, off, p, fm_total, A, prm->mode);
  const int kspace = (int)kmer_space(A, k);
  // batched mode with small enough buckets: the guide trees are built inside
  // the engine launch, which starts aligning each merge as soon as it is known
  const Schedule sched = schedule_for(TuneKey{A, n, p, (int)prm->mode, max_n, seqs->total_len});
  const bool valu = prm->mode == SAD_BATCHED_MFMA && sched.mfma == 0;
  // (by default only while the pair sums fit the MFMA kernel's LDS: with sums
  // in HBM the separate tree kernels are faster unless the autotuner finds
  // otherwise)
  const bool fuse = prm->mode == SAD_BATCHED_MFMA && sched.fuse != 0 &&
                    max_n <= (sched.fuse == 1 ? engine_fused_max_group()
                                              : engine_fused_lds_group());
  // pair sums in HBM: guide trees by the separate kernel, or built in the
  // launch for groups too large for the MFMA kernel's LDS (every group of the
  // vector-ALU kernel)
  const bool sums_in_hbm = !fuse || valu || max_n > engine_fused_lds_group();
  Carver cv;
  AlignBufs ab{};
  plan_align(cv, ab, n, p, seqs->total_len, fm_total, sums_in_hbm);
  uint32_t *&entries = ab.entries, *&F = ab.F;
  int32_t*& nu = ab.nu;
  int64_t*& d_fm_off = ab.d_fm_off;
  uint64_t*& Sw = ab.Sw;
  // k-mer lists and per-bucket similarity matrices into the carved buffers
  auto upload = [&]() -> int32_t { return h2d(fm_off, d_fm_off, stream); };
  auto kernels = [&](hipStream_t st) {
    launch_fill_i32(out->d_merge_list, -1, 2 * (int64_t)n, st);
    launch_fill_i32(reinterpret_cast<int32_t*>(out->d_merge_score), 0, 2 * (int64_t)n, st);
    launch_fill_i32(reinterpret_cast<int32_t*>(out->d_merge_cells), 0, 2 * (int64_t)n, st);
    launch_kmer_lists(seqs->d_codes, seqs->d_offsets, n, A, k, entries, nullptr, nu, c->st, st);
    KmerLists kl{entries, seqs->d_offsets, nu, seqs->d_offsets};
    launch_fmatrix_groups(kl, d_bucket_off, d_members, p, max_n, d_fm_off, k, kspace, F, st);
  };
  TreeSet ts;
  ts.ngroups = p;
  ts.nleaves = n;
  ts.d_group_off = d_bucket_off;
  ts.h_group_off = off;
  ts.d_codes = seqs->d_codes;
  ts.d_offsets = seqs->d_offsets;
  ts.d_ids = d_members;
  ts.total_len = seqs->total_len;
  ts.max_len = seqs->max_len;
  ts.kmer_k = k;
  EngineBuffers e{};
  TreeOutputs to{out->d_colmap, out->d_width, out->d_merge_score, out->d_merge_cells,
                 out->d_cells, false};
  if (fuse) {
    // the similarity matrices stay alive under the engine's workspace, which
    // is carved after them on every attempt
    const FusedTrees fz{&F, &d_fm_off, out->d_merge_list, sums_in_hbm ? &Sw : nullptr, upload,
                        kernels};
    return run_trees(c, ts, out->d_merge_list, prm, A, cv, e, to, stream, &fz, sched.grid,
                     sched.coop != 0 && !valu, valu, sched.chunk);
  }
  r = cv.carve(c);
  if (r) return r;
  r = reset_status(c, stream);
  if (r) return r;
  r = upload();
  if (r) return r;
  kernels(stream);
  launch_upgma(F, d_fm_off, d_bucket_off, p, max_n, Sw, out->d_merge_list, d_bucket_off, c->st,
               stream);
  r = finish(c, stream);
  if (r) return r;
  // the engine's workspace follows the k-mer/UPGMA buffers (merge lists are
  // in the caller's array, so those buffers are no longer needed)
  Carver base;
  return run_trees(c, ts, out->d_merge_list, prm, A, base, e, to, stream, nullptr, sched.grid,
                   sched.coop != 0 && !valu, valu, sched.chunk);
}

extern "C" int32_t sad_tune(const sad_seqs* seqs, const int32_t* d_bucket_off,
                            const int32_t* d_members, const sad_params* prm, sad_msa* out,
                            int32_t* grid_out, int32_t* fuse_out, int32_t* flags_out,
                            hipStream_t stream) {
  if (!prm || !out || !seqs) return fail(SAD_E_INVAL, "null argument");
  int32_t r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  r = check_params(prm, seqs->alphabet, true);
  if (r) return r;
  if (!d_bucket_off || !d_members) return fail(SAD_E_INVAL, "null device array");
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  std::vector<int32_t> off;
  r = validate_read(c, seqs, prm->kmer_k, stream, d_bucket_off, (size_t)prm->p + 1, off);
  if (r) return r;
  if (off[0] != 0 || off[prm->p] != seqs->n) return fail(SAD_E_INVAL, "bucket offsets must span 0..N");
  for (int b = 0; b < prm->p; ++b)
    if (off[b + 1] < off[b]) return fail(SAD_E_INVAL, "bucket offsets must be non-decreasing");
  int max_n = 0;
  for (int b = 0; b < prm->p; ++b) max_n = std::max(max_n, off[b + 1] - off[b]);
  const TuneKey key{seqs->alphabet, seqs->n, prm->p, (int)prm->mode, max_n, seqs->total_len};
  const int cus = std::max(1, engine_workgroups());
  std::vector<Schedule> cand;
  if (prm->mode == SAD_BATCHED_MFMA) {
    // one workgroup per CU fits (LDS); try smaller grids and both tree modes
    for (int coop : {1, 0})
      for (int fuse : {1, 0})
        for (int den : {4, 3, 2}) cand.push_back(Schedule{cus * den / 4, fuse, coop, 1});
    // the same persistent DAG launch with vector-ALU scores (the plain kernel,
    // whose registers and LDS leave room for several workgroups per CU)
    for (int fuse : {1, 0})
      for (int per_cu : {1, 2, 3}) cand.push_back(Schedule{cus * per_cu, fuse, 0, 0});
  } else {
    for (int per_cu : {1, 2, 3}) cand.push_back(Schedule{cus * per_cu, 0, 0, 0});
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  Schedule best{};
  float best_ms = 0.0f;
  // every candidate runs eagerly (no graph capture while tuning): one warm-up
  // run, then the fastest of three timed runs counts
  g_tuning = true;
  // (the MFMA schedules run with 32-step chunks; the best of them is then
  // also timed with 16-step chunks, a shape of the DP strips)
  bool shaped = false;
  Schedule best_mfma{};
  float best_mfma_ms = 0.0f;
  for (size_t ci = 0; ci < cand.size(); ++ci) {
    const Schedule sc = cand[ci];
    g_forced = &sc;
    float ms = 0.0f;
    for (int rep = 0; rep < 4 && r == SAD_OK; ++rep) {
      float t = 0.0f;
      if (hipEventRecord(e0, stream) != hipSuccess) r = fail(SAD_E_DEVICE, "event record");
      if (!r) r = sad_align_buckets(seqs, d_bucket_off, d_members, prm, out, nullptr, 0, stream);
      if (!r && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                 hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        r = fail(SAD_E_DEVICE, "event timing");
      if (!r && rep > 0 && (rep == 1 || t < ms)) ms = t;
    }
    g_forced = nullptr;
    if (r) break;
    if (log_enabled())
      fprintf(stderr, "[sad] tune: grid %d fuse %d coop %d mfma %d chunk %d: %.3f ms\n", sc.grid,
              sc.fuse, sc.coop, sc.mfma, sc.chunk, ms);
    if (best_ms == 0.0f || ms < best_ms) {
      best_ms = ms;
      best = sc;
    }
    if (prm->mode == SAD_BATCHED_MFMA && sc.mfma && (best_mfma_ms == 0.0f || ms < best_mfma_ms)) {
      best_mfma_ms = ms;
      best_mfma = sc;
    }
    if (ci + 1 == cand.size() && !shaped && best_mfma_ms > 0.0f) {
      shaped = true;
      Schedule sh = best_mfma;
      sh.chunk = 16;
      cand.push_back(sh);
    }
  }
  g_tuning = false;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (r) return r;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
  }
  if (grid_out) *grid_out = best.grid;
  if (fuse_out) *fuse_out = best.fuse;
  if (flags_out)
    *flags_out = (best.coop ? 1 : 0) | (best.mfma ? 2 : 0) | (best.chunk == 16 ? 4 : 0);
  return SAD_OK;
}

namespace sad {

__global__ void iota_kernel(int32_t* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

__global__ void group_one_kernel(int32_t* goff, int q, int32_t* list, int32_t root) {
  goff[0] = 0;
  goff[1] = q;
  list[0] = root;
}

// Refinement outputs: ancestor merges (slots 0..q-2) then the q refinement
// alignments; pairs of the refinement steps are (bucket, -1).
__global__ void refine_results_kernel(int q, const int64_t* __restrict__ ga_score,
                                      const int64_t* __restrict__ ga_cells,
                                      const int32_t* __restrict__ ga_merges,
                                      const int64_t* __restrict__ rf_score,
                                      const int64_t* __restrict__ rf_cells,
                                      const int32_t* __restrict__ bucket_of_u, int64_t* score,
                                      int32_t* list, int64_t* cells, int64_t* total) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int64_t tot = 0;
  int m = 0;
  for (int t = 0; t < q - 1; ++t, ++m) {
    score[m] = ga_score[t];
    cells[m] = ga_cells[t];
    list[2 * m] = ga_merges[2 * t];
    list[2 * m + 1] = ga_merges[2 * t + 1];
    tot += ga_cells[t];
  }
  for (int u = 0; u < q; ++u, ++m) {
    score[m] = rf_score[u];
    cells[m] = rf_cells[u];
    list[2 * m] = bucket_of_u[u];
    list[2 * m + 1] = -1;
    tot += rf_cells[u];
  }
  *total = tot;
}

// Buffers of the refinement that live across its engine runs: bucket
// profiles, ancestors, the ancestors' guide tree and GA (plan_refine_keep),
// then the refinement's op strings and the glue's slot tables once the
// template's width TL is known (plan_refine_keep2, carved with the same
// prefix so the earlier buffers keep their addresses).
struct RefineKeep {
  int32_t *d_uidx, *d_bucket_of_u, *d_width_u, *d_rows_u, *anc_len, *cons_list, *ga_goff,
      *ga_merges, *ga_list, *ga_len_d, *to_g, *tl_d, *cnode_W, *cnode_n;
  int64_t *d_wo, *anc_off, *stage_off, *ga_score, *ga_cells, *ga_cells_tot, *ga_off0,
      *cnode_prof;
  uint32_t* cnt32;
  uint16_t *prof16, *tmpl16;
  uint8_t *anc_stage, *anc_codes, *ga_stage;
  // second part
  uint8_t* rf_ops;
  int64_t* rf_ops_off;
  int32_t *ins, *used, *slot_total, *slot_start, *shared_at;
};

static void plan_refine_keep(Carver& kv, RefineKeep& K, int p, int q, int64_t Wt1, int A,
                             bool msa_tmpl) {
  kv.add(K.d_uidx, p);
  kv.add(K.d_bucket_of_u, q);
  kv.add(K.d_width_u, q);
  kv.add(K.d_rows_u, q);
  kv.add(K.d_wo, q + 1);
  kv.add(K.cnt32, (size_t)Wt1 * A);
  kv.add(K.prof16, (size_t)Wt1 * A);
  kv.add(K.cnode_W, q);
  kv.add(K.cnode_n, q);
  kv.add(K.cnode_prof, q);
  kv.add(K.cons_list, q);
  kv.add(K.anc_stage, (size_t)Wt1);
  kv.add(K.anc_len, q);
  kv.add(K.anc_off, q + 1);
  kv.add(K.stage_off, q + 1);
  kv.add(K.anc_codes, (size_t)Wt1);
  kv.add(K.ga_goff, 2);
  kv.add(K.ga_list, 1);
  kv.add(K.ga_merges, 2 * std::max(q, 1));
  kv.add(K.ga_score, std::max(q, 1));
  kv.add(K.ga_cells, std::max(q, 1));
  kv.add(K.ga_cells_tot, 1);
  kv.add(K.ga_stage, (size_t)Wt1 + 1);
  kv.add(K.ga_len_d, 1);
  kv.add(K.ga_off0, 2);
  kv.add(K.to_g, (size_t)Wt1);
  kv.add(K.tmpl16, msa_tmpl ? (size_t)Wt1 * A : 1);
  kv.add(K.tl_d, 1);
}

static void plan_refine_keep2(Carver& kv, RefineKeep& K, int q, int TL, int64_t ops_tot) {
  kv.add(K.rf_ops, (size_t)std::max<int64_t>(ops_tot, 1));
  kv.add(K.rf_ops_off, q + 1);
  kv.add(K.ins, (size_t)q * (TL + 1));
  kv.add(K.used, std::max(TL, 1));
  kv.add(K.slot_total, TL + 1);
  kv.add(K.slot_start, TL + 1);
  kv.add(K.shared_at, std::max(TL, 1));
}

// Workspace that suffices for a refinement of q non-empty buckets of Wtot
// columns in all (widest maxW) after `keep` bytes of stage buffers: the
// larger of the ancestors' stage (k-mer lists, similarity matrix and UPGMA
// sums of q ancestors no longer than their buckets' widths, then their tree's
// engine) and the refinement engine (q bucket-vs-template merges with a
// template of up to min(kMaxWidth, Wtot) columns).
static size_t refine_bound_bytes(size_t keep, int q, int64_t Wtot, int maxW, int A,
                                 uint32_t mode) {
  const int64_t Wt1 = std::max<int64_t>(Wtot, 1);
  size_t arena = 0;
  if (q > 1) {
    uint32_t *entries, *F;
    int32_t *nu, *ids;
    int64_t* fm0;
    uint64_t* Sw;
    Carver base;
    base.add(entries, (size_t)Wt1);
    base.add(nu, q);
    base.add(ids, q);
    base.add(fm0, 1);
    base.add(F, (size_t)q * q);
    base.add(Sw, (size_t)q * q);
    arena = engine_bound_bytes(base, std::vector<int32_t>{0, q}, maxW, Wtot, A, mode);
  }
  const int64_t tl = std::min<int64_t>(kMaxWidth, Wt1);
  const int64_t ops = Wtot + (int64_t)q * tl;
  Carver cv;
  EngineBuffers e{};
  plan_engine(cv, e, 2 * q + 1, q, q, (Wtot + tl) * A + (ops + 1) * A, Wtot + tl + ops + 1,
              (int)std::max<int64_t>(64, std::max<int64_t>(maxW, tl)), true, max_grid(mode));
  return keep + std::max(arena, cv.total());
}

__global__ void init_refine_ctl_kernel(unsigned long long* tops, unsigned long long prof0,
                                       unsigned long long up0, int32_t* qctl) {
  tops[0] = prof0;
  tops[1] = up0;
  // queue head, tail, merges done, finished
  for (int q = 0; q < 8; ++q) qctl[q] = 0;
}

}  // namespace sad

extern "C" int32_t sad_refine_template(const sad_seqs* seqs, const int32_t* d_bucket_off,
                                       const int32_t* d_members, const sad_msa* buckets,
                                       const sad_params* prm, int32_t tmpl, uint8_t* d_ga,
                                       int32_t ga_cap, int32_t* ga_len, sad_msa* gout,
                                       int32_t* n_steps, void* d_ws, size_t ws_bytes,
                                       hipStream_t stream) {
  if (!prm || !buckets || !gout || !ga_len || !n_steps) return fail(SAD_E_INVAL, "null argument");
  if (tmpl != SAD_TEMPLATE_GA && tmpl != SAD_TEMPLATE_GA_MSA)
    return fail(SAD_E_INVAL, "unknown refinement template");
  int32_t r = check_ws(d_ws, ws_bytes);
  if (r) return r;
  WsScope wss(d_ws, ws_bytes);
  r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  r = check_params(prm, seqs->alphabet, true);
  if (r) return r;
  if (!d_bucket_off || !d_members || !buckets->d_colmap || !buckets->d_width || !gout->d_colmap ||
      !gout->d_width || !gout->d_merge_score || !gout->d_merge_list || !gout->d_merge_cells ||
      !gout->d_cells || (!d_ga && ga_cap > 0))
    return fail(SAD_E_INVAL, "null device array");
  const int n = seqs->n, p = prm->p, A = seqs->alphabet, k = prm->kmer_k;
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  std::vector<int32_t> off, wid;
  r = validate_read(c, seqs, k, stream, d_bucket_off, (size_t)p + 1, off,
                    (const int32_t*)buckets->d_width, (size_t)p, &wid);
  if (r) return r;
  if (off[0] != 0 || off[p] != n) return fail(SAD_E_INVAL, "bucket offsets must span 0..N");

  // non-empty buckets u = 0..q-1 in bucket order; their columns at wo[u]
  std::vector<int32_t> uidx(p, -1), bucket_of_u, width_u, rows_u;
  std::vector<int64_t> wo;
  int64_t Wtot = 0;
  int maxW = 0;
  for (int b = 0; b < p; ++b) {
    const int nb = off[b + 1] - off[b];
    if (nb < 0) return fail(SAD_E_INVAL, "bucket offsets must be non-decreasing");
    if (nb == 0) continue;
    if (wid[b] < 0 || wid[b] > kMaxWidth) return fail(SAD_E_INVAL, "bucket width out of range");
    uidx[b] = (int)bucket_of_u.size();
    bucket_of_u.push_back(b);
    width_u.push_back(wid[b]);
    rows_u.push_back(nb);
    wo.push_back(Wtot);
    Wtot += wid[b];
    maxW = std::max(maxW, wid[b]);
  }
  const int q = (int)bucket_of_u.size();
  wo.push_back(Wtot);
  if (q == 0) return fail(SAD_E_INVAL, "no sequences");
  if (q > kMaxGroup) return fail(SAD_E_CAPACITY, "too many buckets for the ancestor tree");

  // ---- stage buffers that live across the engine runs
  const int64_t Wt1 = std::max<int64_t>(Wtot, 1);
  // the ancestors' alignment as a template (at most as wide as all ancestors)
  const bool msa_tmpl = tmpl == SAD_TEMPLATE_GA_MSA && q > 1;
  RefineKeep K{};
  Carver kv;
  plan_refine_keep(kv, K, p, q, Wt1, A, msa_tmpl);
  if (g_ws) {
    // caller workspace: the front holds these buffers and the refinement's
    // (sized for the widest template the library accepts), the rest is for
    // the engine runs
    RefineKeep K2{};
    Carver kb = kv;
    const int tl_max = (int)std::min<int64_t>(kMaxWidth, Wt1);
    plan_refine_keep2(kb, K2, q, tl_max, Wtot + (int64_t)q * tl_max);
    g_ws->keep = kb.total();
    g_ws->bound = refine_bound_bytes(kb.total(), q, Wtot, maxW, A, prm->mode);
    if (g_ws->keep > g_ws->bytes) {
      g_ws_needed = g_ws->bound;
      return fail(SAD_E_CAPACITY, "caller workspace too small for the refinement: " +
                                      std::to_string(g_ws_needed) + " bytes suffice");
    }
  }
  r = kv.carve_keep(c);
  if (r) return r;
  int32_t *d_uidx = K.d_uidx, *d_bucket_of_u = K.d_bucket_of_u, *d_width_u = K.d_width_u,
          *d_rows_u = K.d_rows_u;
  int64_t* d_wo = K.d_wo;
  uint32_t* cnt32 = K.cnt32;
  uint16_t *prof16 = K.prof16, *tmpl16 = K.tmpl16;
  int32_t *cnode_W = K.cnode_W, *cnode_n = K.cnode_n, *cons_list = K.cons_list,
          *anc_len = K.anc_len, *ga_goff = K.ga_goff, *ga_list = K.ga_list,
          *ga_merges = K.ga_merges, *ga_len_d = K.ga_len_d, *to_g = K.to_g, *tl_d = K.tl_d;
  int64_t *cnode_prof = K.cnode_prof, *anc_off = K.anc_off, *stage_off = K.stage_off,
          *ga_score = K.ga_score, *ga_cells = K.ga_cells, *ga_cells_tot = K.ga_cells_tot,
          *ga_off0 = K.ga_off0;
  uint8_t *anc_stage = K.anc_stage, *anc_codes = K.anc_codes, *ga_stage = K.ga_stage;
  r = h2d(uidx, d_uidx, stream);
  if (!r) r = h2d(bucket_of_u, d_bucket_of_u, stream);
  if (!r) r = h2d(width_u, d_width_u, stream);
  if (!r) r = h2d(rows_u, d_rows_u, stream);
  if (!r) r = h2d(wo, d_wo, stream);
  if (!r) r = h2d(wo, stage_off, stream);
  if (r) return r;
  std::vector<int64_t> prof_offs(q);
  for (int u = 0; u < q; ++u) prof_offs[u] = wo[u] * A;
  r = h2d(prof_offs, cnode_prof, stream);
  if (!r) r = h2d(width_u, cnode_W, stream);
  if (!r) r = h2d(rows_u, cnode_n, stream);
  if (r) return r;

  // ---- bucket profiles and local ancestors
  r = reset_status(c, stream);
  if (r) return r;
  launch_fill_i32(reinterpret_cast<int32_t*>(cnt32), 0, Wt1 * A, stream);
  launch_rebuild_profiles(seqs->d_codes, seqs->d_offsets, d_members, d_bucket_off, p, n,
                          buckets->d_colmap, d_uidx, d_wo, buckets->d_width, A, cnt32, Wt1 * A,
                          prof16, c->st, stream);
  iota_kernel<<<(q + 255) / 256, 256, 0, stream>>>(cons_list, q);
  launch_consensus(cons_list, q, cnode_W, cnode_n, cnode_prof, prof16, A, anc_stage, stage_off,
                   anc_len, stream);
  launch_compact(anc_stage, stage_off, anc_len, q, anc_off, anc_codes, stream);
  std::vector<int64_t> h_anc_off;
  r = finish_read(c, stream, anc_off, (size_t)q + 1, h_anc_off);
  if (r) return r;
  int max_anc = 0;
  for (int u = 0; u < q; ++u) max_anc = std::max<int>(max_anc, (int)(h_anc_off[u + 1] - h_anc_off[u]));

  // ---- global ancestor (and the width of the ancestors' alignment)
  int GL = 0, TLq = 0;
  if (q == 1) {
    GL = (int)h_anc_off[1];
    HIPCHK(hipMemcpyAsync(ga_stage, anc_codes, (size_t)std::max(GL, 0), hipMemcpyDeviceToDevice,
                          stream));
  } else {
    const int kspace = (int)kmer_space(A, k);
    uint32_t *entries, *F;
    int32_t *nu, *ids;
    int64_t* fm0;
    uint64_t* Sw;
    // batched mode with few enough ancestors: their guide tree is built
    // inside the engine launch, as the buckets' trees are
    const bool fuse_tree = prm->mode == SAD_BATCHED_MFMA && q <= engine_fused_max_group();
    Carver cv;
    cv.add(entries, (size_t)std::max<int64_t>(h_anc_off[q], 1));
    cv.add(nu, q);
    cv.add(ids, q);
    cv.add(fm0, 1);
    cv.add(F, (size_t)q * q);
    if (!fuse_tree || q > engine_fused_lds_group()) cv.add(Sw, (size_t)q * q);
    // the ancestors' k-mer lists and similarity matrix (again after every
    // carve when the engine's workspace is carved with them)
    auto kernels = [&](hipStream_t st) {
      group_one_kernel<<<1, 1, 0, st>>>(ga_goff, q, ga_list, q + (q - 2));
      iota_kernel<<<(q + 255) / 256, 256, 0, st>>>(ids, q);
      launch_fill_i32(reinterpret_cast<int32_t*>(fm0), 0, 2, st);
      launch_fill_i32(reinterpret_cast<int32_t*>(ga_off0), 0, 4, st);
      launch_kmer_lists(anc_codes, anc_off, q, A, k, entries, nullptr, nu, c->st, st);
      KmerLists kl{entries, anc_off, nu, anc_off};
      launch_fmatrix_groups(kl, ga_goff, ids, 1, q, fm0, k, kspace, F, st);
    };
    if (!fuse_tree) {
      r = cv.carve(c);
      if (r) return r;
      r = reset_status(c, stream);
      if (r) return r;
      kernels(stream);
      launch_upgma(F, fm0, ga_goff, 1, q, Sw, ga_merges, reinterpret_cast<int32_t*>(ga_off0),
                   c->st, stream);
      r = finish(c, stream);
      if (r) return r;
    }
    TreeSet ts;
    ts.ngroups = 1;
    ts.nleaves = q;
    ts.d_group_off = ga_goff;
    ts.h_group_off = {0, q};
    ts.d_codes = anc_codes;
    ts.d_offsets = anc_off;
    ts.d_ids = nullptr;
    ts.total_len = h_anc_off[q];
    ts.max_len = max_anc;
    ts.kmer_k = k;
    EngineBuffers e{};
    TreeOutputs to{nullptr, nullptr, ga_score, ga_cells, ga_cells_tot, true};
    if (fuse_tree) {
      FusedTrees fz{&F, &fm0, ga_merges, q > engine_fused_lds_group() ? &Sw : nullptr,
                    []() -> int32_t { return SAD_OK; }, kernels};
      fz.graph = false;
      r = run_trees(c, ts, ga_merges, prm, A, cv, e, to, stream, &fz);
    } else {
      Carver base;
      r = run_trees(c, ts, ga_merges, prm, A, base, e, to, stream);
    }
    if (r) return r;
    r = reset_status(c, stream);
    if (r) return r;
    if (msa_tmpl)
      launch_copy_node_profile(e.node_W, e.node_prof, e.prof_pool, 2 * q - 2, A, tmpl16,
                               Wt1 * A, tl_d, c->st, stream);
    launch_consensus(ga_list, 1, e.node_W, e.node_n, e.node_prof, e.prof_pool, A, ga_stage,
                     ga_off0, ga_len_d, stream);
    std::vector<int32_t> gl, tl;
    r = finish_read(c, stream, ga_len_d, 1, gl, (const int32_t*)tl_d, msa_tmpl ? 1 : 0,
                    msa_tmpl ? &tl : nullptr);
    if (r) return r;
    GL = gl[0];
    if (msa_tmpl) TLq = tl[0];
  }
  *ga_len = GL;
  if (GL > ga_cap) return fail(SAD_E_CAPACITY, "GA capacity too small");
  if (GL > kMaxWidth) return fail(SAD_E_CAPACITY, "global ancestor wider than the library limit");
  if (GL > 0) HIPCHK(hipMemcpyAsync(d_ga, ga_stage, (size_t)GL, hipMemcpyDeviceToDevice, stream));
  // the template: GA as one row, or the ancestors' alignment (TL columns, q rows)
  int TL = GL, tn = 1;
  if (msa_tmpl) {
    TL = TLq;
    tn = q;
    if (TL > kMaxWidth) return fail(SAD_E_CAPACITY, "template wider than the library limit");
  }
  {
    std::vector<int32_t> gl{GL}, tl{TL};
    r = h2d(gl, ga_len_d, stream);
    if (!r) r = h2d(tl, tl_d, stream);
    if (r) return r;
  }

  // ---- refinement: every bucket alignment against the template
  std::vector<int64_t> ops_off(q + 1);
  int64_t ops_tot = 0;
  for (int u = 0; u < q; ++u) {
    ops_off[u] = ops_tot;
    ops_tot += width_u[u] + TL;
  }
  ops_off[q] = ops_tot;
  uint8_t* rf_ops;
  int64_t* rf_ops_off;
  int32_t *ins, *used, *slot_total, *slot_start, *shared_at;
  {
    Carver kv2 = kv;
    RefineKeep K2{};
    plan_refine_keep2(kv2, K2, q, TL, ops_tot);
    // same prefix as kv: earlier buffers keep their addresses and contents
    if (!g_ws && kv2.total() > c->keep_cap) {
      // grow while preserving: copy the prefix out through the work arena
      size_t keep_bytes = kv.total();
      char* tmp = nullptr;
      HIPCHK(hipMalloc(&tmp, keep_bytes));
      HIPCHK(hipMemcpyAsync(tmp, c->keep, keep_bytes, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipStreamSynchronize(stream));
      r = kv2.carve_keep(c);
      if (r) {
        hipFree(tmp);
        return r;
      }
      HIPCHK(hipMemcpyAsync(c->keep, tmp, keep_bytes, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipStreamSynchronize(stream));
      HIPCHK(hipFree(tmp));
    } else {
      r = kv2.carve_keep(c);
      if (r) return r;
    }
    rf_ops = K2.rf_ops;
    rf_ops_off = K2.rf_ops_off;
    ins = K2.ins;
    used = K2.used;
    slot_total = K2.slot_total;
    slot_start = K2.slot_start;
    shared_at = K2.shared_at;
  }
  r = h2d(ops_off, rf_ops_off, stream);
  if (r) return r;
  const int rwcap = std::max(64, std::max(maxW, TL));
  const int64_t prof_fixed = (Wtot + TL) * A;
  const int64_t prof_cap = prof_fixed + (ops_tot + 1) * A;
  const int64_t up_cap = Wtot + TL + ops_tot + 1;
  EngineBuffers e{};
  Carver cv;
  plan_engine(cv, e, 2 * q + 1, q, q, prof_cap, up_cap, rwcap, true);
  r = cv.carve(c);
  if (r) return r;
  r = reset_status(c, stream);
  if (r) return r;
  HIPCHK(hipMemcpyAsync(e.prof_pool, prof16, (size_t)Wtot * A * sizeof(uint16_t),
                        hipMemcpyDeviceToDevice, stream));
  if (msa_tmpl) {
    if (TL > 0)
      HIPCHK(hipMemcpyAsync(e.prof_pool + Wtot * A, tmpl16, (size_t)TL * A * sizeof(uint16_t),
                            hipMemcpyDeviceToDevice, stream));
  } else {
    launch_onehot_seq(ga_stage, ga_len_d, std::max(GL, 1), A, e.prof_pool + Wtot * A, stream);
  }
  launch_fill_i32(e.node_parent, -1, 2 * q + 1, stream);
  launch_fill_i32(e.queue_flag, 0, (int64_t)q * (1 + kMaxHelpers), stream);
  launch_fill_i32(e.job_link, 0, q, stream);
  init_refine_ctl_kernel<<<1, 1, 0, stream>>>(e.tops, (unsigned long long)prof_fixed,
                                              (unsigned long long)(Wtot + TL), e.qctl);
  launch_refine_nodes(q, d_wo, d_width_u, d_rows_u, Wtot * A, Wtot, tl_d, tn, A, 0, e.node_W,
                      e.node_n, e.node_prof, e.node_up, stream);
  launch_refine_jobs(q, rf_ops_off, e.job_a, e.job_b, e.job_out, e.job_next, e.job_pending,
                     e.job_ops_off, e.queue, e.queue_flag, e.qctl + 1, e.node_parent, stream);
  EngineArgs a = engine_args(e, q, A, prm->subst, prm->gap_open, prm->gap_extend, prm->mode,
                             rf_ops, c->st);
  if (prm->mode == SAD_BATCHED_MFMA && !a.trow) return SAD_E_DEVICE;
  r = attach_phases(c, a, q, stream);
  if (r) return r;
  EngineTimer timer(stream);
  launch_engine(a, e.nwg, stream);
  timer.stop();
  r = finish(c, stream);
  if (r) return r;
  timer.collect();
  r = collect_phases(c, a, stream);
  if (r) return r;

  // ---- glue
  r = reset_status(c, stream);
  if (r) return r;
  launch_fill_i32(ins, 0, (int64_t)q * (TL + 1), stream);
  launch_fill_i32(used, 0, std::max(TL, 1), stream);
  launch_glue(rf_ops, rf_ops_off, e.node_W + q + 1, q, TL, ins, used, slot_total, slot_start,
              shared_at, gout->d_width, d_wo, to_g, seqs->d_offsets, d_members, d_bucket_off, p, n,
              d_uidx, buckets->d_colmap, gout->d_colmap, stream);
  refine_results_kernel<<<1, 1, 0, stream>>>(q, ga_score, ga_cells, ga_merges, e.job_score,
                                             e.job_cells, d_bucket_of_u, gout->d_merge_score,
                                             gout->d_merge_list, gout->d_merge_cells,
                                             gout->d_cells);
  *n_steps = 2 * q - 1;
  return finish(c, stream);
}

extern "C" int32_t sad_refine_tree(const sad_seqs* seqs, const int32_t* d_bucket_off,
                                   const int32_t* d_members, const sad_msa* glued,
                                   const sad_params* prm, int32_t passes, sad_msa* out,
                                   int32_t* n_steps, int32_t* n_accepted, int64_t* rec,
                                   int32_t rec_cap, hipStream_t stream) {
  if (!prm || !glued || !out || !n_steps || !n_accepted || passes < 0 || rec_cap < 0 ||
      (!rec && rec_cap > 0))
    return fail(SAD_E_INVAL, "null or negative argument");
  int32_t r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  r = check_params(prm, seqs->alphabet, true);
  if (r) return r;
  if (!d_bucket_off || !d_members || !glued->d_colmap || !glued->d_width ||
      !glued->d_merge_list || !out->d_colmap || !out->d_width)
    return fail(SAD_E_INVAL, "null device array");
  const int n = seqs->n, p = prm->p, A = seqs->alphabet;
  *n_steps = 0;
  *n_accepted = 0;
  if (n > 65535) return fail(SAD_E_CAPACITY, "tree refinement counts residues in 16 bits");
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  std::vector<int32_t> off, wv;
  r = validate_read(c, seqs, prm->kmer_k, stream, d_bucket_off, (size_t)p + 1, off,
                    (const int32_t*)glued->d_width, (size_t)1, &wv);
  if (r) return r;
  if (off[0] != 0 || off[p] != n) return fail(SAD_E_INVAL, "bucket offsets must span 0..N");
  std::vector<int32_t> uidx(p, -1), size_u;
  for (int b = 0; b < p; ++b) {
    if (off[b + 1] < off[b]) return fail(SAD_E_INVAL, "bucket offsets must be non-decreasing");
    if (off[b + 1] == off[b]) continue;
    uidx[b] = (int)size_u.size();
    size_u.push_back(off[b + 1] - off[b]);
  }
  const int q = (int)size_u.size();
  int W = wv[0];
  if (W < 0 || W > kMaxWidth) return fail(SAD_E_CAPACITY, "glued width beyond the library limit");
  const int64_t total = seqs->total_len;
  // the ancestors' guide tree: merges (a, b) over leaves 0..q-1, node q + t
  // made by merge t; its edges in the order deeper first, then smaller id
  // (the root's second child splits like its first and is skipped)
  std::vector<int32_t> order;
  std::vector<int8_t> in1tab;
  if (q >= 2) {
    std::vector<int32_t> tree;
    r = d2h(c, glued->d_merge_list, 2 * (size_t)(q - 1), tree, stream);
    if (r) return r;
    const int nn = 2 * q - 1;
    std::vector<int32_t> parent(nn, -1), depth(nn, 0);
    for (int t = 0; t < q - 1; ++t) {
      const int a = tree[2 * t], b = tree[2 * t + 1];
      if (a < 0 || b < 0 || a >= q + t || b >= q + t || a == b || parent[a] >= 0 ||
          parent[b] >= 0)
        return fail(SAD_E_INVAL, "ancestor merge list is not a tree over the non-empty buckets");
      parent[a] = parent[b] = q + t;
    }
    for (int v = nn - 1; v >= 0; --v) depth[v] = parent[v] < 0 ? 0 : depth[parent[v]] + 1;
    const int skip = tree[2 * (q - 2) + 1];
    for (int v = 0; v < nn - 1; ++v)
      if (v != skip) order.push_back(v);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return depth[x] != depth[y] ? depth[x] > depth[y] : x < y;
    });
    in1tab.assign(order.size() * (size_t)q, 0);
    for (size_t x = 0; x < order.size(); ++x)
      for (int u = 0; u < q; ++u) {
        int w = u;
        while (w >= 0 && w != order[x]) w = parent[w];
        in1tab[x * q + u] = w == order[x] ? 1 : 0;
      }
  }
  // buffers kept across the steps
  int32_t *seq_u, *d_uidx, *colA, *colB, *S32;
  int8_t* d_in1;
  Carver kv;
  kv.add(seq_u, std::max(n, 1));
  kv.add(d_uidx, p);
  kv.add(colA, (size_t)std::max<int64_t>(total, 1));
  kv.add(colB, (size_t)std::max<int64_t>(total, 1));
  kv.add(S32, A * A);
  kv.add(d_in1, std::max<size_t>(in1tab.size(), 1));
  r = kv.carve_keep(c);
  if (r) return r;
  std::vector<int32_t> S32h(A * A);
  for (int t = 0; t < A * A; ++t) S32h[t] = prm->subst[t];
  r = h2d(uidx, d_uidx, stream);
  if (!r) r = h2d(S32h, S32, stream);
  if (!r) r = h2d(in1tab, d_in1, stream);
  if (r) return r;
  r = reset_status(c, stream);
  if (r) return r;
  launch_seq_leaf(d_bucket_off, p, d_members, d_uidx, n, seq_u, stream);
  if (total > 0)
    HIPCHK(hipMemcpyAsync(colA, glued->d_colmap, (size_t)total * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, stream));
  r = finish(c, stream);
  if (r) return r;
  int steps = 0, accepted = 0;
  for (int pass = 0; pass < passes && q >= 2 && W > 0; ++pass) {
    int acc_pass = 0;
    for (size_t x = 0; x < order.size(); ++x) {
      int n1 = 0;
      for (int u = 0; u < q; ++u)
        if (in1tab[x * q + u]) n1 += size_u[u];
      const int n2 = n - n1;
      const int8_t* in1 = d_in1 + x * q;
      // one merge of the two parts: nodes 0 (group 1) and 1 (group 2) -> 2
      EngineBuffers e{};
      Carver cv;
      const int64_t prof_cap = 2 * (int64_t)W * A + (2 * (int64_t)W + 1) * A;
      const int64_t up_cap = 4 * (int64_t)W + 1;
      plan_engine(cv, e, 3, 1, 1, prof_cap, up_cap, std::max(64, W), true, 1);
      uint32_t* cnt;
      int32_t *idx1, *idx2, *wid, *map1, *map2;
      uint8_t *oldops, *ops;
      unsigned long long* s_old;
      int64_t *res, *zero64, *opsoff;
      cv.add(cnt, 2 * (size_t)W * A);
      cv.add(idx1, W);
      cv.add(idx2, W);
      cv.add(map1, W);
      cv.add(map2, W);
      cv.add(wid, 4);
      cv.add(oldops, W);
      cv.add(ops, 2 * (size_t)W + 1);
      cv.add(s_old, 2);
      cv.add(res, 4);
      cv.add(zero64, 1);
      cv.add(opsoff, 2);
      r = cv.carve(c);
      if (r) return r;
      const std::vector<int64_t> oo{0, 2 * (int64_t)W + 1}, z{0};
      const std::vector<int32_t> n1v{0, 0, n1, 0};
      r = h2d(oo, opsoff, stream);
      if (!r) r = h2d(z, zero64, stream);
      if (!r) r = h2d(n1v, wid, stream);
      if (!r) r = reset_status(c, stream);
      if (r) return r;
      const int64_t G = (int64_t)n1 * n2;
      launch_split_step(seqs->d_codes, seqs->d_offsets, n, colA, seq_u, in1, W, A, cnt, idx1,
                        idx2, oldops, wid, e.prof_pool, 0, (int64_t)W * A, S32,
                        G * prm->gap_open, G * prm->gap_extend, s_old, c->st, stream);
      launch_fill_i32(e.node_parent, -1, 3, stream);
      launch_fill_i32(e.queue_flag, 0, 1 + kMaxHelpers, stream);
      launch_fill_i32(e.job_link, 0, 1, stream);
      init_refine_ctl_kernel<<<1, 1, 0, stream>>>(e.tops, 2ull * W * A, 2ull * W, e.qctl);
      launch_refine_nodes(1, zero64, wid, wid + 2, (int64_t)W * A, W, wid + 1, n2, A, 0,
                          e.node_W, e.node_n, e.node_prof, e.node_up, stream);
      launch_refine_jobs(1, opsoff, e.job_a, e.job_b, e.job_out, e.job_next, e.job_pending,
                         e.job_ops_off, e.queue, e.queue_flag, e.qctl + 1, e.node_parent, stream);
      EngineArgs a = engine_args(e, 1, A, prm->subst, prm->gap_open, prm->gap_extend, prm->mode,
                                 ops, c->st);
      if (prm->mode == SAD_BATCHED_MFMA && !a.trow) return SAD_E_DEVICE;
      EngineTimer timer(stream);
      launch_engine(a, e.nwg, stream);
      timer.stop();
      launch_split_result(s_old, e.job_score, e.node_W, 2, res, stream);
      r = finish(c, stream);
      if (r) return r;
      timer.collect();
      std::vector<int64_t> rv;
      r = d2h(c, res, 3, rv, stream);
      if (r) return r;
      if (steps < rec_cap) {
        rec[3 * (int64_t)steps] = order[x];
        rec[3 * (int64_t)steps + 1] = rv[0];
        rec[3 * (int64_t)steps + 2] = rv[1];
      }
      ++steps;
      if (rv[1] > rv[0]) {
        launch_split_apply(ops, e.node_W + 2, map1, map2, seqs->d_offsets, n, seq_u, in1, idx1,
                           idx2, colA, colB, stream);
        r = finish(c, stream);
        if (r) return r;
        std::swap(colA, colB);
        W = (int)rv[2];
        ++acc_pass;
        ++accepted;
        if (W > kMaxWidth) return fail(SAD_E_CAPACITY, "refined width beyond the library limit");
      }
    }
    if (acc_pass == 0) break;
  }
  if (total > 0)
    HIPCHK(hipMemcpyAsync(out->d_colmap, colA, (size_t)total * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, stream));
  {
    const std::vector<int32_t> wout{W};
    r = h2d(wout, out->d_width, stream);
    if (r) return r;
  }
  *n_steps = steps;
  *n_accepted = accepted;
  return finish(c, stream);
}

extern "C" int32_t sad_refine(const sad_seqs* seqs, const int32_t* d_bucket_off,
                              const int32_t* d_members, const sad_msa* buckets,
                              const sad_params* prm, uint8_t* d_ga, int32_t ga_cap,
                              int32_t* ga_len, sad_msa* gout, int32_t* n_steps, void* d_ws,
                              size_t ws_bytes, hipStream_t stream) {
  return sad_refine_template(seqs, d_bucket_off, d_members, buckets, prm, SAD_TEMPLATE_GA, d_ga,
                             ga_cap, ga_len, gout, n_steps, d_ws, ws_bytes, stream);
}

extern "C" int32_t sad_refine_workspace(const sad_seqs* seqs, const int32_t* d_bucket_off,
                                        const sad_msa* buckets, const sad_params* prm,
                                        size_t* ws_bytes, hipStream_t stream) {
  if (!prm || !buckets || !ws_bytes) return fail(SAD_E_INVAL, "null argument");
  int32_t r = check_seqs(seqs, prm->kmer_k);
  if (r) return r;
  r = check_params(prm, seqs->alphabet, false);
  if (r) return r;
  if (!d_bucket_off || !buckets->d_width) return fail(SAD_E_INVAL, "null device array");
  const int n = seqs->n, p = prm->p, A = seqs->alphabet;
  DeviceCtx* c = nullptr;
  r = get_ctx(&c);
  if (r) return r;
  std::vector<int32_t> off, wid;
  r = reset_status(c, stream);
  if (!r)
    r = finish_read(c, stream, d_bucket_off, (size_t)p + 1, off, (const int32_t*)buckets->d_width,
                    (size_t)p, &wid);
  if (r) return r;
  if (off[0] != 0 || off[p] != n) return fail(SAD_E_INVAL, "bucket offsets must span 0..N");
  int q = 0, maxW = 0;
  int64_t Wtot = 0;
  for (int b = 0; b < p; ++b) {
    const int nb = off[b + 1] - off[b];
    if (nb < 0) return fail(SAD_E_INVAL, "bucket offsets must be non-decreasing");
    if (nb == 0) continue;
    if (wid[b] < 0 || wid[b] > kMaxWidth) return fail(SAD_E_INVAL, "bucket width out of range");
    ++q;
    Wtot += wid[b];
    maxW = std::max(maxW, wid[b]);
  }
  if (q == 0) return fail(SAD_E_INVAL, "no sequences");
  // either template: the q-row template's buffer included
  const int64_t Wt1 = std::max<int64_t>(Wtot, 1);
  const int tl_max = (int)std::min<int64_t>(kMaxWidth, Wt1);
  RefineKeep K{};
  Carver kb;
  plan_refine_keep(kb, K, p, q, Wt1, A, q > 1);
  plan_refine_keep2(kb, K, q, tl_max, Wtot + (int64_t)q * tl_max);
  *ws_bytes = refine_bound_bytes(kb.total(), q, Wtot, maxW, A, prm->mode);
  return SAD_OK;
}

extern "C" size_t sad_workspace_needed(void) { return g_ws_needed; }

extern "C" int32_t sad_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_prof_on = (on & 1) != 0;
  g_phase_on = (on & 2) != 0;
  return SAD_OK;
}

extern "C" int32_t sad_profile_read(double* engine_ms, int64_t* engine_launches, int32_t reset) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (engine_ms) *engine_ms = g_prof_ms;
  if (engine_launches) *engine_launches = g_prof_launches;
  if (reset) {
    g_prof_ms = 0.0;
    g_prof_launches = 0;
  }
  return SAD_OK;
}

extern "C" int32_t sad_profile_phases(double* ms_out, int64_t* jobs, int32_t reset) {
  std::lock_guard<std::mutex> lk(g_mu);
  const double per_ms = g_tick_khz > 0 ? 1.0 / g_tick_khz : 0.0;
  if (ms_out) {
    for (int q = 0; q < 4; ++q) ms_out[q] = (double)g_phase[q] * per_ms;
    ms_out[4] = (double)g_phase[5] * per_ms;
  }
  if (jobs) *jobs = (int64_t)g_phase[4];
  if (reset)
    for (int q = 0; q < 6; ++q) g_phase[q] = 0;
  return SAD_OK;
}

extern "C" int32_t sad_profile_graphs(int64_t* captured, int64_t* replayed, int32_t reset) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (captured) *captured = g_graph_captured;
  if (replayed) *replayed = g_graph_replayed;
  if (reset) g_graph_captured = g_graph_replayed = 0;
  return SAD_OK;
}

extern "C" int32_t sad_profile_jobs(int64_t* out, int64_t cap, int64_t* njobs) {
  std::lock_guard<std::mutex> lk(g_mu);
  const int64_t n = (int64_t)g_jobrec.size() / 8;
  if (njobs) *njobs = n;
  if (out && cap > 0) {
    const int64_t m = std::min(n, cap);
    std::copy(g_jobrec.begin(), g_jobrec.begin() + m * 8, out);
  }
  return SAD_OK;
}

extern "C" const char* sad_last_error(void) { return g_err.c_str(); }

extern "C" void sad_release(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& c : g_ctx) {
    if (c.arena) hipFree(c.arena);
    if (c.keep) hipFree(c.keep);
    if (c.st) hipFree(c.st);
    if (c.h_st) hipHostFree(c.h_st);
    if (c.h_small) hipHostFree(c.h_small);
    if (c.up) {
      // staged uploads may still be queued
      if (c.up_off > 0) (void)hipStreamSynchronize(c.up_stream);
      hipHostFree(c.up);
    }
    if (c.phase) hipFree(c.phase);
    if (c.jobrec) hipFree(c.jobrec);
    for (hipGraphExec_t x : c.gexec)
      if (x) hipGraphExecDestroy(x);
    if (c.cap_stream) hipStreamDestroy(c.cap_stream);
    c = DeviceCtx{};
  }
}

extern "C" const char* sad_version(void) { return "sad-gfx950 0.1"; }

extern "C" int32_t sad_quality(const int32_t* d_colmap, const int32_t* d_class, int64_t total,
                               int32_t nclass, uint64_t* aligned_pairs, uint64_t* true_pairs,
                               hipStream_t stream) {
  using namespace sad;
  if (!aligned_pairs || !true_pairs) return fail(SAD_E_INVAL, "null output");
  if (total < 0 || total > INT32_MAX || nclass < 1 || nclass > INT32_MAX - 1)
    return fail(SAD_E_INVAL, "total or class count out of range");
  if (total > 0 && (!d_colmap || !d_class)) return fail(SAD_E_INVAL, "null input");
  DeviceCtx* c = nullptr;
  int32_t r = get_ctx(&c);
  if (r) return r;
  int32_t *cnt = nullptr, *off = nullptr, *cursor = nullptr, *cols = nullptr;
  unsigned long long* sums = nullptr;
  Carver cv;
  cv.add(cnt, (size_t)nclass);
  cv.add(off, (size_t)nclass + 1);
  cv.add(cursor, (size_t)nclass);
  cv.add(cols, (size_t)std::max<int64_t>(total, 1));
  cv.add(sums, 2);
  r = cv.carve(c);
  if (r) return r;
  r = reset_status(c, stream);
  if (r) return r;
  launch_quality(d_colmap, d_class, total, nclass, cnt, off, cursor, cols, sums, c->st, stream);
  r = finish(c, stream);
  if (r) return r;
  unsigned long long h[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  *aligned_pairs = h[0];
  *true_pairs = h[1];
  return SAD_OK;
}

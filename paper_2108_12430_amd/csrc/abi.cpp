// C ABI of libgwstream.so: argument validation, slot/arena bookkeeping,
// per-call item tables and kernel dispatch.  No kernel arithmetic lives here.
#include "gwstream.h"

#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using gw::Item;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  return fail(GW_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(expr)                              \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, #expr); \
  } while (0)
#define CHK(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != GW_OK) return rc_; \
  } while (0)

inline size_t r256(size_t x) { return (x + 255) & ~size_t(255); }
inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

struct Stager;

// Records a staged table's reuse event when the entry point that staged it
// returns, i.e. after every launch that reads the table has been enqueued.
struct StageGuard {
  Stager* s = nullptr;
  int k = -1;
  hipStream_t st = nullptr;
  StageGuard() = default;
  StageGuard(const StageGuard&) = delete;
  StageGuard& operator=(const StageGuard&) = delete;
  inline ~StageGuard();
};

// Ring of pinned host staging slots for the per-call item tables.  Slot k's
// event is recorded on the caller's stream after the last launch of the call
// that staged it, so a later call (on any stream) reuses the slot only after
// the kernels that read its table have finished.  gen[k] counts the uses of
// slot k: a (k, gen) pair names one call's completion event until the slot
// is staged again, by which time the host has waited for that event.
struct Stager {
  static constexpr int K = 32;
  Item* host = nullptr;
  Item* dev = nullptr;
  int cap = 0;
  int next = 0;
  hipEvent_t ev[K] = {};
  bool used[K] = {};
  uint64_t gen[K] = {};
  static size_t dev_bytes(int cap) { return r256(sizeof(Item) * (size_t)cap * K); }
  int init(void* dev_region, int cap_items) {
    cap = cap_items;
    dev = reinterpret_cast<Item*>(dev_region);
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&host), sizeof(Item) * (size_t)cap * K,
                         hipHostMallocDefault));
    for (int k = 0; k < K; ++k) HIPCHK(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming));
    return GW_OK;
  }
  void release() {
    for (int k = 0; k < K; ++k)
      if (ev[k]) {
        if (used[k]) (void)hipEventSynchronize(ev[k]);
        (void)hipEventDestroy(ev[k]);
        ev[k] = nullptr;
      }
    if (host) (void)hipHostFree(host);
    host = nullptr;
  }
  // True while call (k, g) may still have work in flight.
  bool pending(int k, uint64_t g) const {
    return k >= 0 && gen[k] == g && hipEventQuery(ev[k]) == hipErrorNotReady;
  }
  int stage(const std::vector<Item>& items, hipStream_t st, const Item** out, StageGuard* guard) {
    if ((int)items.size() > cap) return fail(GW_EINVAL, "too many items in one call");
    const void* d = nullptr;
    CHK(stage_raw(items.data(), items.size() * sizeof(Item), st, &d, guard));
    *out = reinterpret_cast<const Item*>(d);
    return GW_OK;
  }
  // Any table of at most cap * sizeof(Item) bytes (same slots and reuse rule).
  int stage_raw(const void* data, size_t bytes, hipStream_t st, const void** out, StageGuard* guard) {
    if (bytes > (size_t)cap * sizeof(Item)) return fail(GW_EINVAL, "too many items in one call");
    const int k = next;
    next = (next + 1) % K;
    if (used[k]) HIPCHK(hipEventSynchronize(ev[k]));
    ++gen[k];
    std::memcpy(host + (size_t)k * cap, data, bytes);
    HIPCHK(hipMemcpyAsync(dev + (size_t)k * cap, host + (size_t)k * cap, bytes, hipMemcpyHostToDevice, st));
    // provisional record (covers the copy if the call ends before its launches);
    // the guard records again after the launches
    HIPCHK(hipEventRecord(ev[k], st));
    used[k] = true;
    guard->s = this;
    guard->k = k;
    guard->st = st;
    *out = dev + (size_t)k * cap;
    return GW_OK;
  }
  void done(int k, hipStream_t st) { (void)hipEventRecord(ev[k], st); }
};

StageGuard::~StageGuard() {
  if (s && k >= 0) s->done(k, st);
}

// Optional per-launch timing with HIP events recorded on the launch stream.
struct Prof {
  bool on = false;
  struct Rec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> spare;
  hipEvent_t get() {
    if (!spare.empty()) {
      hipEvent_t e = spare.back();
      spare.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Prof g_prof;

}  // namespace

// Launch through a gw::launch_* function; with profiling on, bracket it with
// events on the same stream.
#define LAUNCH(name, st, expr)                                   \
  do {                                                           \
    hipEvent_t a_ = nullptr;                                     \
    if (g_prof.on && (a_ = g_prof.get())) (void)hipEventRecord(a_, st); \
    HIPCHK(expr);                                                \
    if (a_) {                                                    \
      hipEvent_t b_ = g_prof.get();                              \
      if (b_) {                                                  \
        (void)hipEventRecord(b_, st);                            \
        g_prof.recs.push_back({std::string(name), a_, b_});      \
      }                                                          \
    }                                                            \
  } while (0)

static std::string nm(const char* k, const char* tag, int i) {
  return std::string(k) + "." + tag + std::to_string(i);
}

extern "C" int gw_profile_begin(void) {
  for (auto& r : g_prof.recs) {
    g_prof.spare.push_back(r.a);
    g_prof.spare.push_back(r.b);
  }
  g_prof.recs.clear();
  g_prof.on = true;
  return GW_OK;
}

extern "C" int gw_profile_end(char* buf, size_t len) {
  g_prof.on = false;
  std::map<std::string, std::pair<int, double>> agg;
  for (auto& r : g_prof.recs) {
    HIPCHK(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    auto& e = agg[r.name];
    e.first += 1;
    e.second += ms;
  }
  std::string out;
  for (auto& kv : agg)
    out += kv.first + " " + std::to_string(kv.second.first) + " " + std::to_string(kv.second.second) + "\n";
  if (buf && len) {
    const size_t n = std::min(len - 1, out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return GW_OK;
}

// ===========================================================================
// Pool
// ===========================================================================
struct gw_pool {
  char* arena = nullptr;
  size_t bytes = 0;
  int max_slots = 0, max_items = 0;
  size_t ring_base = 0;
  Stager stager;
  struct Slot {
    bool open = false;
    int C = 0, W = 0;
    size_t off = 0, size = 0;
    int head = 0;
    int64_t n_seen = 0;
    hipEvent_t fill = nullptr;  // recorded after the zero-fill of gw_stream_open
    int last_k = -1;            // the last call that read or wrote the ring: stager
    uint64_t last_gen = 0;      // slot and generation (see Stager)
    // activation cache of the incremental DeepClean forward (caller-owned)
    void* cache = nullptr;
    size_t cache_bytes = 0;
    bool cache_valid = false;  // holds the window that ended cache_seen samples into the stream
    int cache_T = 0;           // its window start modulo W (ring heads)
    int64_t cache_seen = 0;
    uint64_t cache_model = 0;  // the id and weight generation of the model that computed it
    uint64_t cache_gen = 0;
  };
  // A closed slot's region whose last users may still be running: a later
  // open that reuses any of its bytes orders its zero-fill after them.
  struct Retired {
    size_t off, size;
    hipEvent_t fill;
    int k;
    uint64_t gen;
  };
  std::vector<Slot> slots;
  std::map<size_t, size_t> free_;  // offset -> size
  std::vector<Retired> retired;
  std::vector<hipEvent_t> spare_ev;
  size_t used = 0;

  hipEvent_t get_event() {
    if (!spare_ev.empty()) {
      hipEvent_t e = spare_ev.back();
      spare_ev.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
  }
  // Drop retired regions whose users have all finished.
  void prune() {
    size_t j = 0;
    for (size_t i = 0; i < retired.size(); ++i) {
      Retired& r = retired[i];
      const bool busy = (r.fill && hipEventQuery(r.fill) == hipErrorNotReady) || stager.pending(r.k, r.gen);
      if (busy) {
        retired[j++] = r;
      } else if (r.fill) {
        spare_ev.push_back(r.fill);
      }
    }
    retired.resize(j);
  }
  void mark_used(const int32_t* ids, int n, const StageGuard& g) {
    for (int i = 0; i < n; ++i) {
      slots[ids[i]].last_k = g.k;
      slots[ids[i]].last_gen = stager.gen[g.k];
    }
  }

  static size_t ring_bytes(int C, int W) { return r256((size_t)C * W * 4) + r256((size_t)C * W * 2); }
  int64_t ring_elem(const Slot& s) const { return (int64_t)(s.off / 4); }
  int64_t shadow_elem(const Slot& s) const {
    return (int64_t)((s.off + r256((size_t)s.C * s.W * 4)) / 2);
  }
  bool alloc(size_t size, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= size) {
        *off = it->first;
        const size_t rest = it->second - size;
        const size_t noff = it->first + size;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        used += size;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t size) {
    used -= size;
    auto it = free_.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int check_slot(int32_t s) const {
    if (s < 0 || s >= max_slots) return fail(GW_EINVAL, "slot id out of range");
    if (!slots[s].open) return fail(GW_ESTATE, "slot is not open");
    return GW_OK;
  }
};

extern "C" const char* gw_last_error(void) { return g_err.c_str(); }

extern "C" int gw_pool_init(void* dev_arena, size_t bytes, int32_t max_slots, int32_t max_items,
                            gw_pool** out) {
  if (!dev_arena || !out) return fail(GW_EINVAL, "null arena or out pointer");
  if (reinterpret_cast<uintptr_t>(dev_arena) % 256) return fail(GW_EINVAL, "arena not 256-byte aligned");
  if (max_slots < 1 || max_items < 1 || max_items > (1 << 16))
    return fail(GW_EINVAL, "max_slots/max_items out of range");
  const size_t desc = Stager::dev_bytes(max_items);
  if (bytes < desc + 256) return fail(GW_EINVAL, "arena too small for the item tables");
  auto* p = new gw_pool();
  p->arena = reinterpret_cast<char*>(dev_arena);
  p->bytes = bytes;
  p->max_slots = max_slots;
  p->max_items = max_items;
  p->ring_base = desc;
  p->slots.resize(max_slots);
  const size_t usable = (bytes - desc) & ~size_t(255);
  if (usable) p->free_[desc] = usable;
  int rc = p->stager.init(p->arena, max_items);
  if (rc != GW_OK) {
    p->stager.release();
    delete p;
    return rc;
  }
  *out = p;
  return GW_OK;
}

extern "C" int gw_pool_free(gw_pool* pool) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  pool->stager.release();
  for (auto& r : pool->retired)
    if (r.fill) pool->spare_ev.push_back(r.fill);
  for (auto& sl : pool->slots)
    if (sl.fill) pool->spare_ev.push_back(sl.fill);
  for (hipEvent_t e : pool->spare_ev) {
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  delete pool;
  return GW_OK;
}

extern "C" int gw_stream_open(gw_pool* pool, int32_t C, int32_t W, void* hip_stream, int32_t* slot) {
  if (!pool || !slot) return fail(GW_EINVAL, "null pool or slot pointer");
  if (C < 1 || W < 1 || (int64_t)C * W > (int64_t)1 << 30) return fail(GW_EINVAL, "bad C or W");
  int id = -1;
  for (int i = 0; i < pool->max_slots; ++i)
    if (!pool->slots[i].open) {
      id = i;
      break;
    }
  if (id < 0) return fail(GW_ENOMEM, "slot table full");
  const size_t size = gw_pool::ring_bytes(C, W);
  hipEvent_t fill = pool->get_event();
  if (!fill) return fail(GW_EHIP, "hipEventCreate failed");
  size_t off = 0;
  if (!pool->alloc(size, &off)) {
    pool->spare_ev.push_back(fill);
    return fail(GW_ENOMEM, "arena full");
  }
  const hipStream_t st = S(hip_stream);
  // the region may still be read or written by work of a closed slot
  // (possibly on another stream): the zero-fill waits for it
  pool->prune();
  hipError_t e = hipSuccess;
  for (const auto& r : pool->retired) {
    if (r.off >= off + size || off >= r.off + r.size) continue;
    if (e == hipSuccess && r.fill) e = hipStreamWaitEvent(st, r.fill, 0);
    if (e == hipSuccess && pool->stager.pending(r.k, r.gen)) e = hipStreamWaitEvent(st, pool->stager.ev[r.k], 0);
  }
  if (e == hipSuccess) e = gw::launch_fill_zero(pool->arena + off, size, st);
  if (e == hipSuccess) e = hipEventRecord(fill, st);
  if (e != hipSuccess) {
    pool->release(off, size);
    pool->spare_ev.push_back(fill);
    return hip_fail(e, "fill_zero");
  }
  auto& s = pool->slots[id];
  s.open = true;
  s.C = C;
  s.W = W;
  s.off = off;
  s.size = size;
  s.head = 0;
  s.n_seen = 0;
  s.fill = fill;
  s.last_k = -1;
  s.last_gen = 0;
  s.cache = nullptr;
  s.cache_bytes = 0;
  s.cache_valid = false;
  *slot = id;
  return GW_OK;
}

extern "C" int gw_stream_close(gw_pool* pool, int32_t slot) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  CHK(pool->check_slot(slot));
  auto& s = pool->slots[slot];
  pool->retired.push_back({s.off, s.size, s.fill, s.last_k, s.last_gen});
  pool->release(s.off, s.size);
  s = gw_pool::Slot();
  pool->prune();
  return GW_OK;
}

extern "C" int gw_stream_info(const gw_pool* pool, int32_t slot, int32_t* C, int32_t* W,
                              int64_t* n_seen) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  CHK(pool->check_slot(slot));
  const auto& s = pool->slots[slot];
  if (C) *C = s.C;
  if (W) *W = s.W;
  if (n_seen) *n_seen = s.n_seen;
  return GW_OK;
}

extern "C" int gw_stream_window(gw_pool* pool, int32_t slot, float* out, uint16_t* out_bf16,
                                void* hip_stream) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  CHK(pool->check_slot(slot));
  if (!out && !out_bf16) return GW_OK;
  const auto& s = pool->slots[slot];
  std::vector<Item> items(1);
  std::memset(&items[0], 0, sizeof(Item));
  items[0].ring = pool->ring_elem(s);
  items[0].shadow = pool->shadow_elem(s);
  items[0].head = s.head;
  items[0].C = s.C;
  items[0].W = s.W;
  const Item* dev = nullptr;
  StageGuard guard;
  CHK(pool->stager.stage(items, S(hip_stream), &dev, &guard));
  pool->mark_used(&slot, 1, guard);
  LAUNCH("gather", S(hip_stream), gw::launch_gather(pool->arena, dev, 1, s.C, s.W, out, out_bf16, S(hip_stream)));
  return GW_OK;
}

extern "C" int gw_stream_load(gw_pool* pool, int32_t slot, const float* window, int64_t n_seen, void* hip_stream) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  CHK(pool->check_slot(slot));
  if (!window) return fail(GW_EINVAL, "null window");
  if (n_seen < 0) return fail(GW_EINVAL, "negative n_seen");
  auto& s = pool->slots[slot];
  // one update of W samples written from ring position 0: the ring holds the
  // window oldest first and the head returns to 0
  std::vector<Item> items(1);
  std::memset(&items[0], 0, sizeof(Item));
  items[0].ring = pool->ring_elem(s);
  items[0].shadow = pool->shadow_elem(s);
  items[0].src = 0;
  items[0].head = 0;
  items[0].s = s.W;
  items[0].C = s.C;
  items[0].W = s.W;
  const Item* dev = nullptr;
  StageGuard guard;
  CHK(pool->stager.stage(items, S(hip_stream), &dev, &guard));
  pool->mark_used(&slot, 1, guard);
  LAUNCH("snapshot", S(hip_stream), gw::launch_snapshot(pool->arena, dev, 1, s.C * s.W, window, S(hip_stream)));
  s.head = 0;
  s.n_seen = n_seen;
  s.cache_valid = false;
  return GW_OK;
}

extern "C" int gw_pool_usage(const gw_pool* pool, size_t* used, size_t* free_bytes) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  size_t f = 0;
  for (auto& kv : pool->free_) f += kv.second;
  if (used) *used = pool->used;
  if (free_bytes) *free_bytes = f;
  return GW_OK;
}

extern "C" int snapshot_update(gw_pool* pool, int32_t n, const int32_t* slots, const int32_t* strides,
                               const float* samples, const int64_t* offsets, void* hip_stream) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  if (n == 0) return GW_OK;
  if (n < 0 || n > pool->max_items) return fail(GW_EINVAL, "n out of range");
  if (!slots || !strides || !samples || !offsets) return fail(GW_EINVAL, "null argument");
  std::vector<char> seen(pool->max_slots, 0);
  std::vector<Item> items(n);
  int max_cs = 0;
  for (int i = 0; i < n; ++i) {
    CHK(pool->check_slot(slots[i]));
    if (seen[slots[i]]) return fail(GW_EINVAL, "slot appears twice in one call");
    seen[slots[i]] = 1;
    const auto& s = pool->slots[slots[i]];
    if (strides[i] < 1 || strides[i] > s.W) return fail(GW_EINVAL, "stride must be in [1, W]");
    if (offsets[i] < 0) return fail(GW_EINVAL, "negative sample offset");
    Item& it = items[i];
    it.ring = pool->ring_elem(s);
    it.shadow = pool->shadow_elem(s);
    it.src = offsets[i];
    it.out = 0;
    it.head = s.head;
    it.s = strides[i];
    it.C = s.C;
    it.W = s.W;
    max_cs = std::max(max_cs, s.C * strides[i]);
  }
  const Item* dev = nullptr;
  StageGuard guard;
  CHK(pool->stager.stage(items, S(hip_stream), &dev, &guard));
  pool->mark_used(slots, n, guard);
  LAUNCH("snapshot", S(hip_stream), gw::launch_snapshot(pool->arena, dev, n, max_cs, samples, S(hip_stream)));
  for (int i = 0; i < n; ++i) {
    auto& s = pool->slots[slots[i]];
    s.head = (s.head + strides[i]) % s.W;
    s.n_seen += strides[i];
  }
  return GW_OK;
}

// ===========================================================================
// Models
// ===========================================================================
namespace {

struct LayerD {
  int type, ci, co, k, s, p, op, bn;
  int64_t w, b, g, be, m, v;  // parameter offsets (floats)
  size_t scale, shift;        // packed byte offsets
  size_t wbf;                 // packed bf16 weights byte offset
  size_t wbf_lo;              // packed low bf16 terms (training variant's split operands)
  size_t wdg, wdg_lo;         // split bf16 packs of the input-gradient (adjoint) convolution
  bool dg_mfma;               // the adjoint convolution has a matrix-core kernel
  size_t wf16;                // packed fp16 weights byte offset (fused-shape networks)
  size_t wfs, wfs16;          // the fused kernel's own fragment layout (bf16, fp16), where it differs
  bool bf16;                  // BF16 kernel available
};

struct StageD {
  int ci, co;
  int64_t wa, ba, wb, bb, ws, bs;
  size_t wa_bf, wb_bf, ws_bf;
  bool bf16;
};

constexpr int DENSE_ITEMS = 4096;  // item-table capacity for dense-input calls

}  // namespace

// process-wide model ids, never reused (a cache names the model that computed it)
static std::atomic<uint64_t> g_next_model_id{1};

struct gw_model {
  int kind = 0;
  uint64_t id = g_next_model_id.fetch_add(1);
  uint64_t gen = 0;  // weight generation: counts gw_model_refresh calls
  std::vector<LayerD> layers;
  std::vector<StageD> stages;
  int c_in = 0, c_last = 0;
  int64_t head_w = 0, head_b = 0;
  int64_t n_params = 0;
  size_t packed_bytes = 0;
  const float* params = nullptr;
  char* packed = nullptr;
  Stager stager;
  bool bf16_all = false;
  bool fused = false;  // reference DeepClean / BBHnet shape: whole-network BF16 kernel available
  bool layerwise = false;  // BBHnet BF16: run the per-layer kernels instead of the fused one
  int cu_budget = 0;   // CUs the persistent kernels size their grid for (0: all)
};

namespace {

int build_layout(int32_t kind, const int32_t* desc, int32_t len, gw_model& m) {
  if (!desc || len < 1) return fail(GW_EINVAL, "null or empty description");
  m.kind = kind;
  int64_t off = 0;
  size_t pk = 0;
  if (kind == GW_MODEL_DEEPCLEAN) {
    const int L = desc[0];
    if (L < 1 || L > 64 || len != 1 + 8 * L) return fail(GW_EINVAL, "bad DeepClean description length");
    pk = Stager::dev_bytes(DENSE_ITEMS);
    m.bf16_all = true;
    for (int l = 0; l < L; ++l) {
      const int32_t* d = desc + 1 + 8 * l;
      LayerD ly{};
      ly.type = d[0];
      ly.ci = d[1];
      ly.co = d[2];
      ly.k = d[3];
      ly.s = d[4];
      ly.p = d[5];
      ly.op = d[6];
      ly.bn = d[7];
      if (ly.type != GW_LAYER_CONV && ly.type != GW_LAYER_CONVT) return fail(GW_EINVAL, "bad layer type");
      if (ly.ci < 1 || ly.co < 1 || ly.ci > 4096 || ly.co > 4096) return fail(GW_EINVAL, "bad channel count");
      if (ly.k < 1 || ly.k > 7) return fail(GW_EUNSUPPORTED, "kernel size must be 1..7");
      if (ly.s != 1 && ly.s != 2) return fail(GW_EUNSUPPORTED, "stride must be 1 or 2");
      if (ly.p < 0 || ly.p >= ly.k) return fail(GW_EINVAL, "pad must be in [0, k)");
      if (ly.op < 0 || ly.op >= ly.s || (ly.type == GW_LAYER_CONV && ly.op))
        return fail(GW_EINVAL, "bad output padding");
      if (ly.bn != 0 && ly.bn != GW_LAYER_BN_TANH) return fail(GW_EINVAL, "bad layer flags");
      if (l > 0 && ly.ci != m.layers.back().co) return fail(GW_EINVAL, "channel chain mismatch");
      ly.w = off;
      off += (int64_t)ly.ci * ly.co * ly.k;
      ly.b = off;
      off += ly.co;
      if (ly.bn) {
        ly.g = off;
        ly.be = off + ly.co;
        ly.m = off + 2 * ly.co;
        ly.v = off + 3 * ly.co;
        off += 4 * ly.co;
      }
      ly.scale = pk;
      pk += r256(sizeof(float) * ly.co);
      ly.shift = pk;
      pk += r256(sizeof(float) * ly.co);
      m.layers.push_back(ly);
    }
    if (m.layers.back().co != 1 || m.layers.back().bn)
      return fail(GW_EINVAL, "last layer must have one output channel and no normalisation");
    for (auto& ly : m.layers) {
      ly.bf16 = gw::conv_bf16_supported(ly.ci, ly.co, ly.k, ly.s, ly.type == GW_LAYER_CONVT);
      if (ly.bf16) {
        const size_t eb = r256(2 * gw::conv_bf16_packed_elems(ly.ci, ly.co, ly.k, ly.type == GW_LAYER_CONVT));
        ly.wbf = pk;
        pk += eb;
        ly.wbf_lo = pk;
        pk += eb;
      }
      // the adjoint of a stride-2 conv is a stride-2 transposed conv and
      // vice versa, with input and output channels exchanged
      const bool conv = ly.type == GW_LAYER_CONV;
      ly.dg_mfma = ly.s == 2 && gw::conv_bf16_supported(ly.co, ly.ci, ly.k, 2, conv);
      if (ly.dg_mfma) {
        const size_t eb = r256(2 * gw::conv_bf16_packed_elems(ly.co, ly.ci, ly.k, conv));
        ly.wdg = pk;
        pk += eb;
        ly.wdg_lo = pk;
        pk += eb;
      }
      m.bf16_all = m.bf16_all && ly.bf16;
    }
    m.c_in = m.layers[0].ci;
    {
      const int Ln = (int)m.layers.size();
      std::vector<int> ci(Ln), co(Ln), ty(Ln), k(Ln), st(Ln), pd(Ln), op(Ln), bn(Ln);
      for (int l = 0; l < Ln; ++l) {
        const auto& ly = m.layers[l];
        ci[l] = ly.ci;
        co[l] = ly.co;
        ty[l] = ly.type;
        k[l] = ly.k;
        st[l] = ly.s;
        pd[l] = ly.p;
        op[l] = ly.op;
        bn[l] = ly.bn;
      }
      m.fused = m.bf16_all && gw::dc_fused_supported(ci.data(), co.data(), ty.data(), k.data(), st.data(),
                                                     pd.data(), op.data(), bn.data(), Ln);
      if (m.fused)
        for (int l = 0; l < Ln; ++l) {  // FP16 copies for the fused kernel's FP16 variant
          auto& ly = m.layers[l];
          ly.wf16 = pk;
          pk += r256(2 * gw::conv_bf16_packed_elems(ly.ci, ly.co, ly.k, ly.type == GW_LAYER_CONVT));
          if (gw::dc_fused_special(l)) {
            const size_t eb = r256(2 * gw::dc_fused_special_elems(l));
            ly.wfs = pk;
            pk += eb;
            ly.wfs16 = pk;
            pk += eb;
          }
        }
    }
  } else if (kind == GW_MODEL_BBHNET) {
    const int Sn = desc[0];
    if (Sn < 1 || Sn > 8 || len != 2 + Sn) return fail(GW_EINVAL, "bad BBHnet description length");
    m.c_in = desc[1];
    if (m.c_in < 1 || m.c_in > 1024) return fail(GW_EINVAL, "bad input channels");
    int ci = m.c_in;
    m.bf16_all = true;
    for (int s = 0; s < Sn; ++s) {
      StageD sd{};
      sd.ci = ci;
      sd.co = desc[2 + s];
      if (sd.co < 1 || sd.co > 1024) return fail(GW_EINVAL, "bad stage channels");
      sd.wa = off;
      off += (int64_t)sd.co * sd.ci * 7;
      sd.ba = off;
      off += sd.co;
      sd.wb = off;
      off += (int64_t)sd.co * sd.co * 7;
      sd.bb = off;
      off += sd.co;
      sd.ws = off;
      off += (int64_t)sd.co * sd.ci;
      sd.bs = off;
      off += sd.co;
      sd.bf16 = gw::conv_bf16_supported(sd.ci, sd.co, 7, 2, false) &&
                gw::conv_bf16_supported(sd.co, sd.co, 7, 1, false);
      if (sd.bf16) {
        sd.wa_bf = pk;
        pk += r256(2 * gw::conv_bf16_packed_elems(sd.ci, sd.co, 7, false));
        sd.wb_bf = pk;
        pk += r256(2 * gw::conv_bf16_packed_elems(sd.co, sd.co, 7, false));
        sd.ws_bf = pk;
        pk += r256(2 * gw::conv_bf16_packed_elems(sd.ci, sd.co, 1, false));
      }
      m.bf16_all = m.bf16_all && sd.bf16;
      m.stages.push_back(sd);
      ci = sd.co;
    }
    m.c_last = ci;
    {
      std::vector<int> co;
      for (auto& sd : m.stages) co.push_back(sd.co);
      m.fused = m.bf16_all && gw::bbh_fused_supported(m.c_in, co.data(), Sn);
    }
    m.head_w = off;
    off += ci;
    m.head_b = off;
    off += 1;
    pk = std::max<size_t>(pk, 256);
  } else {
    return fail(GW_EINVAL, "unknown model kind");
  }
  m.n_params = off;
  m.packed_bytes = pk;
  return GW_OK;
}

int pack_model(gw_model* m, hipStream_t st) {
  const float* P = m->params;
  if (m->kind == GW_MODEL_DEEPCLEAN) {
    for (int l = 0; l < (int)m->layers.size(); ++l) {
      auto& ly = m->layers[l];
      float* sc = reinterpret_cast<float*>(m->packed + ly.scale);
      float* sh = reinterpret_cast<float*>(m->packed + ly.shift);
      HIPCHK(gw::launch_fold_bn(P + ly.b, ly.bn ? P + ly.g : nullptr, ly.bn ? P + ly.be : nullptr,
                                ly.bn ? P + ly.m : nullptr, ly.bn ? P + ly.v : nullptr, sc, sh, ly.co,
                                st));
      if (ly.bf16) {
        HIPCHK(gw::launch_pack_bf16(P + ly.w, reinterpret_cast<uint16_t*>(m->packed + ly.wbf), ly.ci,
                                    ly.co, ly.k, ly.type == GW_LAYER_CONVT, st));
        HIPCHK(gw::launch_pack_bf16(P + ly.w, reinterpret_cast<uint16_t*>(m->packed + ly.wbf_lo), ly.ci,
                                    ly.co, ly.k, ly.type == GW_LAYER_CONVT, st, gw::PACK_BF16_LO));
      }
      if (ly.dg_mfma) {
        const bool conv = ly.type == GW_LAYER_CONV;
        HIPCHK(gw::launch_pack_bf16(P + ly.w, reinterpret_cast<uint16_t*>(m->packed + ly.wdg), ly.co, ly.ci, ly.k,
                                    conv, st));
        HIPCHK(gw::launch_pack_bf16(P + ly.w, reinterpret_cast<uint16_t*>(m->packed + ly.wdg_lo), ly.co, ly.ci,
                                    ly.k, conv, st, gw::PACK_BF16_LO));
      }
      if (m->fused) {
        HIPCHK(gw::launch_pack_bf16(P + ly.w, reinterpret_cast<uint16_t*>(m->packed + ly.wf16), ly.ci,
                                    ly.co, ly.k, ly.type == GW_LAYER_CONVT, st, gw::PACK_F16));
        if (gw::dc_fused_special(l)) {
          HIPCHK(gw::launch_pack_fused(P + ly.w, reinterpret_cast<uint16_t*>(m->packed + ly.wfs), l, st, false));
          HIPCHK(gw::launch_pack_fused(P + ly.w, reinterpret_cast<uint16_t*>(m->packed + ly.wfs16), l, st, true));
        }
      }
    }
  } else {
    for (auto& sd : m->stages) {
      if (!sd.bf16) continue;
      HIPCHK(gw::launch_pack_bf16(P + sd.wa, reinterpret_cast<uint16_t*>(m->packed + sd.wa_bf), sd.ci,
                                  sd.co, 7, false, st));
      HIPCHK(gw::launch_pack_bf16(P + sd.wb, reinterpret_cast<uint16_t*>(m->packed + sd.wb_bf), sd.co,
                                  sd.co, 7, false, st));
      HIPCHK(gw::launch_pack_bf16(P + sd.ws, reinterpret_cast<uint16_t*>(m->packed + sd.ws_bf), sd.ci,
                                  sd.co, 1, false, st));
    }
  }
  return GW_OK;
}

int layer_lout(const LayerD& ly, int L) {
  if (ly.type == GW_LAYER_CONV) {
    if (L + 2 * ly.p < ly.k) return -1;
    return (L + 2 * ly.p - ly.k) / ly.s + 1;
  }
  return (L - 1) * ly.s - 2 * ly.p + ly.k + ly.op;
}

// Per-layer input/output lengths for a window of W samples; error unless the
// network maps W back to W.
int dc_lengths(const gw_model* m, int W, std::vector<int>& lin, std::vector<int>& lout) {
  lin.clear();
  lout.clear();
  int L = W;
  for (auto& ly : m->layers) {
    lin.push_back(L);
    L = layer_lout(ly, L);
    if (L < 1) return fail(GW_EINVAL, "window too short for the network");
    lout.push_back(L);
  }
  if (L != W) return fail(GW_EINVAL, "network does not map W samples back to W (W must be a multiple of the total stride)");
  return GW_OK;
}

// Start `a` of the input band [a, W) that the newest s outputs depend on:
// propagate the needed index range back through the layers, then align `a`
// to the network's total stride so every layer's sample grid in the band
// coincides with the full window's, and check that at every layer the band
// still contains every needed position.  Returns 0 when no shorter band works.
int causal_band_start(const gw_model* m, int W, int s) {
  std::vector<int> lin, lout;
  if (dc_lengths(m, W, lin, lout) != GW_OK || s >= W) return 0;
  const int L = (int)m->layers.size();
  std::vector<int64_t> need(L);
  int64_t lo = W - s, hi = W - 1;
  for (int l = L - 1; l >= 0; --l) {
    const LayerD& ly = m->layers[l];
    int64_t a, b;
    if (ly.type == GW_LAYER_CONV) {
      a = (int64_t)ly.s * lo - ly.p;
      b = (int64_t)ly.s * hi - ly.p + ly.k - 1;
    } else {
      const int64_t num = lo + ly.p - ly.k + 1;
      a = num >= 0 ? (num + ly.s - 1) / ly.s : -((-num) / ly.s);
      const int64_t nh = hi + ly.p;
      b = nh >= 0 ? nh / ly.s : -((-nh + ly.s - 1) / ly.s);
    }
    lo = std::max<int64_t>(a, 0);
    hi = std::min<int64_t>(b, lin[l] - 1);
    need[l] = lo;
  }
  int64_t D = 1;
  for (auto& ly : m->layers)
    if (ly.type == GW_LAYER_CONV) D *= ly.s;
  for (int64_t a = need[0] / D * D; a > 0; a -= D) {
    std::vector<int> li, lo2;
    if (dc_lengths(m, (int)(W - a), li, lo2) != GW_OK) continue;
    bool ok = true;
    for (int l = 0; l < L && ok; ++l) {
      if ((a * lin[l]) % W) ok = false;                 // grids must coincide
      else if (a * lin[l] / W > need[l]) ok = false;     // band must cover the need
      else if (li[l] != lin[l] - a * lin[l] / W) ok = false;
    }
    if (ok) return (int)a;
  }
  return 0;
}

}  // namespace

extern "C" int gw_model_n_params(int32_t kind, const int32_t* desc, int32_t desc_len, int64_t* n) {
  if (!n) return fail(GW_EINVAL, "null out pointer");
  gw_model m;
  CHK(build_layout(kind, desc, desc_len, m));
  *n = m.n_params;
  return GW_OK;
}

extern "C" int gw_model_packed_bytes(int32_t kind, const int32_t* desc, int32_t desc_len, size_t* bytes) {
  if (!bytes) return fail(GW_EINVAL, "null out pointer");
  gw_model m;
  CHK(build_layout(kind, desc, desc_len, m));
  *bytes = m.packed_bytes;
  return GW_OK;
}

extern "C" int gw_model_create(int32_t kind, const int32_t* desc, int32_t desc_len,
                               const float* dev_params, int64_t n_params, void* dev_packed,
                               size_t packed_bytes, void* hip_stream, gw_model** out) {
  if (!out || !dev_params || !dev_packed) return fail(GW_EINVAL, "null argument");
  if (reinterpret_cast<uintptr_t>(dev_packed) % 256) return fail(GW_EINVAL, "packed buffer not 256-byte aligned");
  auto* m = new gw_model();
  int rc = build_layout(kind, desc, desc_len, *m);
  if (rc == GW_OK && n_params != m->n_params) rc = fail(GW_EINVAL, "n_params does not match the description");
  if (rc == GW_OK && packed_bytes < m->packed_bytes) rc = fail(GW_EINVAL, "packed buffer too small");
  if (rc != GW_OK) {
    delete m;
    return rc;
  }
  m->params = dev_params;
  m->packed = reinterpret_cast<char*>(dev_packed);
  if (kind == GW_MODEL_DEEPCLEAN) rc = m->stager.init(m->packed, DENSE_ITEMS);
  if (rc == GW_OK) rc = pack_model(m, S(hip_stream));
  if (rc != GW_OK) {
    m->stager.release();
    delete m;
    return rc;
  }
  *out = m;
  return GW_OK;
}

extern "C" int gw_model_refresh(gw_model* m, void* hip_stream) {
  if (!m) return fail(GW_EINVAL, "null model");
  ++m->gen;  // activation caches computed with the previous weights are recomputed in full
  return pack_model(m, S(hip_stream));
}

extern "C" int gw_model_set_layerwise(gw_model* m, int32_t on) {
  if (!m) return fail(GW_EINVAL, "null model");
  if (m->kind != GW_MODEL_BBHNET) return fail(GW_EINVAL, "DeepClean takes GW_LAYERWISE per call");
  m->layerwise = on != 0;
  return GW_OK;
}

extern "C" int gw_model_set_cu_budget(gw_model* m, int32_t ncu) {
  if (!m) return fail(GW_EINVAL, "null model");
  if (ncu < 0) return fail(GW_EINVAL, "negative CU budget");
  m->cu_budget = ncu;
  return GW_OK;
}

extern "C" int gw_model_free(gw_model* m) {
  if (!m) return fail(GW_EINVAL, "null model");
  m->stager.release();
  delete m;
  return GW_OK;
}

// ===========================================================================
// DeepClean
// ===========================================================================
namespace {

struct DcWs {
  // inference
  size_t buf[2] = {0, 0};
  size_t total = 0;
  // training
  std::vector<size_t> mean, invstd, z, a;  // per layer (SIZE_MAX = none)
  size_t ztmp = 0, atmp[2] = {0, 0};
  size_t partial = 0;
  int ckpt = -1;
};

constexpr size_t NONE = ~size_t(0);

int dc_ws_layout(const gw_model* m, int n, int W, int precision, uint32_t flags, DcWs& w) {
  std::vector<int> lin, lout;
  CHK(dc_lengths(m, W, lin, lout));
  const int L = (int)m->layers.size();
  const size_t esz = 4;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += r256(bytes);
    return o;
  };
  if (!(flags & GW_TRAIN)) {
    size_t mx = 256;
    for (int l = 0; l + 1 < L; ++l)
      mx = std::max(mx, (size_t)n * m->layers[l].co * lout[l] * esz);
    w.buf[0] = take(mx);
    w.buf[1] = take(mx);
    w.total = off;
    (void)precision;
    return GW_OK;
  }
  const bool rec = flags & GW_RECOMPUTE;
  // checkpoint: the layer with the shortest output (the bottleneck)
  int ck = 0;
  for (int l = 0; l + 1 < L; ++l)
    if (lout[l] < lout[ck]) ck = l;
  w.ckpt = rec ? ck : -1;
  w.mean.assign(L, NONE);
  w.invstd.assign(L, NONE);
  w.z.assign(L, NONE);
  w.a.assign(L, NONE);
  for (int l = 0; l < L; ++l)
    if (m->layers[l].bn) {
      w.mean[l] = take(4 * m->layers[l].co);
      w.invstd[l] = take(4 * m->layers[l].co);
    }
  size_t mx = 256;
  int maxc = 1, maxchunk = 1;
  for (int l = 0; l + 1 < L; ++l) {
    const size_t sz = (size_t)n * m->layers[l].co * lout[l] * esz;
    mx = std::max(mx, sz);
    maxc = std::max(maxc, m->layers[l].co);
    maxchunk = std::max(maxchunk, gw::red_chunks(n, lout[l]));
    if (!rec) {
      if (m->layers[l].bn) w.z[l] = take(sz);
      w.a[l] = take(sz);
    } else if (l == ck) {
      w.a[l] = take(sz);
    }
  }
  if (rec) {
    w.ztmp = take(mx);
    w.atmp[0] = take(mx);
    w.atmp[1] = take(mx);
  }
  w.partial = take((size_t)maxc * maxchunk * 2 * sizeof(double));
  w.total = off;
  return GW_OK;
}

gw::ConvP conv_params(const gw_model* m, const LayerD& ly, int n, int Lin, int Lout) {
  gw::ConvP p{};
  p.n = n;
  p.Ci = ly.ci;
  p.Co = ly.co;
  p.Lin = Lin;
  p.Lout = Lout;
  p.k = ly.k;
  p.stride = ly.s;
  p.pad = ly.p;
  p.w = m->params + ly.w;
  if (ly.type == GW_LAYER_CONV) {
    p.wso = (int64_t)ly.ci * ly.k;
    p.wsi = ly.k;
  } else {
    p.wsi = (int64_t)ly.co * ly.k;
    p.wso = ly.k;
  }
  p.bias = m->params + ly.b;
  p.scale = reinterpret_cast<const float*>(m->packed + ly.scale);
  p.shift = reinterpret_cast<const float*>(m->packed + ly.shift);
  if (ly.bf16) p.wpk = reinterpret_cast<const uint16_t*>(m->packed + ly.wbf);
  return p;
}

hipError_t run_conv(const gw::ConvP& p, const LayerD& ly, int epi, int src, int precision,
                    hipStream_t st) {
  const bool tr = ly.type == GW_LAYER_CONVT;
  if (precision == GW_BF16) return gw::launch_conv_bf16(p, tr, epi, src, st);
  return gw::launch_conv_fp32(p, tr, epi, src, st);
}

}  // namespace

extern "C" int deepclean_workspace(const gw_model* m, int32_t n, int32_t W, int32_t precision,
                                   uint32_t flags, size_t* bytes) {
  if (!m || !bytes) return fail(GW_EINVAL, "null argument");
  if (m->kind != GW_MODEL_DEEPCLEAN) return fail(GW_ESTATE, "not a DeepClean model");
  if (n < 1) return fail(GW_EINVAL, "n must be >= 1");
  DcWs w;
  CHK(dc_ws_layout(m, n, W, precision, flags, w));
  *bytes = w.total;
  return GW_OK;
}

// deepclean_forward; with upd set (fused BF16 inference on pool input only),
// the launch also performs the snapshot update whose new samples sit at
// upd + upd_off[i]: the slots' host heads have already been advanced, so the
// items carry the heads after the update
static int dc_forward(const gw_model* m, gw_pool* pool, const int32_t* slots, const float* x, int32_t n, int32_t W,
                      const int32_t* strides, const int32_t* delays, const float* strain, float* noise, float* clean,
                      int32_t precision, uint32_t flags, void* ws, size_t ws_bytes, hipStream_t st, const float* upd,
                      const int64_t* upd_off) {
  if (!m) return fail(GW_EINVAL, "null model");
  if (m->kind != GW_MODEL_DEEPCLEAN) return fail(GW_ESTATE, "not a DeepClean model");
  if (n == 0) return GW_OK;
  if (n < 0) return fail(GW_EINVAL, "negative n");
  if ((pool != nullptr) == (x != nullptr)) return fail(GW_EINVAL, "exactly one of pool and x must be given");
  if (pool && !slots) return fail(GW_EINVAL, "pool input needs slots");
  if (precision != GW_FP32 && precision != GW_BF16 && precision != GW_FP16) return fail(GW_EINVAL, "bad precision");
  if (flags & ~(GW_TRAIN | GW_RECOMPUTE | GW_CAUSAL | GW_LAYERWISE)) return fail(GW_EINVAL, "bad flags");
  if (precision == GW_FP16 && (!m->fused || (flags & (GW_TRAIN | GW_LAYERWISE))))
    return fail(GW_EUNSUPPORTED, "FP16 is the fused kernel's variant: reference network, inference only");
  if ((flags & GW_CAUSAL) && (flags & GW_TRAIN)) return fail(GW_EINVAL, "GW_CAUSAL is for inference");
  if ((flags & GW_CAUSAL) && (!clean || noise))
    return fail(GW_EINVAL, "GW_CAUSAL computes only the clean output (noise must be NULL)");
  if ((flags & GW_RECOMPUTE) && !(flags & GW_TRAIN)) return fail(GW_EINVAL, "GW_RECOMPUTE needs GW_TRAIN");
  if ((flags & GW_TRAIN) && !x) return fail(GW_EINVAL, "training forward needs dense input x");

  if (precision == GW_BF16 && !m->bf16_all) return fail(GW_EUNSUPPORTED, "no BF16 kernel for this network");
  if (clean && (!strides || !strain)) return fail(GW_EINVAL, "clean output needs strides and strain");
  if (delays && !clean) return fail(GW_EINVAL, "delays apply to the clean output");
  if (!ws) return fail(GW_EINVAL, "null workspace");
  {
    std::vector<int> l0, l1;
    CHK(dc_lengths(m, W, l0, l1));
  }
  // GW_CAUSAL: run the layers on the band [a, W) only
  int a_band = 0;
  if (flags & GW_CAUSAL) {
    // the clean block of item i ends delay_i before W: the band must reach
    // back s_i + delay_i samples (plus the receptive field)
    int smax = 1;
    for (int i = 0; i < n; ++i) {
      if (strides[i] < 1 || strides[i] > W) return fail(GW_EINVAL, "stride must be in [1, W]");
      const int d = delays ? delays[i] : 0;
      if (d < 0 || d > W - strides[i]) return fail(GW_EINVAL, "delay must be in [0, W - stride]");
      smax = std::max(smax, strides[i] + d);
    }
    a_band = causal_band_start(m, W, smax);
  }
  const int Wb = W - a_band;
  DcWs w;
  CHK(dc_ws_layout(m, n, Wb, precision, flags & ~(GW_CAUSAL | GW_LAYERWISE), w));
  if (ws_bytes < w.total)
    return fail(GW_EINVAL, "workspace too small: need " + std::to_string(w.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GW_EINVAL, "workspace not 256-byte aligned");
  std::vector<int> lin, lout;
  CHK(dc_lengths(m, Wb, lin, lout));

  // item table: ring addresses (pool input) and stride/offset of the clean block
  const bool need_items = pool || clean;
  std::vector<Item> items;
  if (need_items) {
    items.resize(n);
    std::vector<char> seen(pool ? pool->max_slots : 0, 0);
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
      Item& it = items[i];
      std::memset(&it, 0, sizeof(it));
      if (pool) {
        CHK(pool->check_slot(slots[i]));
        if (seen[slots[i]]) return fail(GW_EINVAL, "slot appears twice in one call");
        seen[slots[i]] = 1;
        const auto& s = pool->slots[slots[i]];
        if (s.C != m->c_in || s.W != W) return fail(GW_EINVAL, "slot C/W does not match the model and W");
        it.ring = pool->ring_elem(s);
        it.shadow = pool->shadow_elem(s);
        it.head = (s.head + a_band) % s.W;  // oldest sample of the band
        it.C = s.C;
        it.W = s.W;
        if (upd) it.src = upd_off[i];
      }
      if (clean) {
        if (strides[i] < 1 || strides[i] > W) return fail(GW_EINVAL, "stride must be in [1, W]");
        it.s = strides[i];
        it.delay = delays ? delays[i] : 0;
        if (it.delay < 0 || it.delay > W - it.s) return fail(GW_EINVAL, "delay must be in [0, W - stride]");
        it.out = off;
        off += strides[i];
      } else {
        it.s = upd ? strides[i] : 0;  // the update's new samples (no clean output to place)
      }
    }
  }
  const Item* dev_items = nullptr;
  StageGuard guard;
  if (need_items) {
    if (pool) {
      CHK(pool->stager.stage(items, st, &dev_items, &guard));
      pool->mark_used(slots, n, guard);
    } else {
      CHK(const_cast<gw_model*>(m)->stager.stage(items, st, &dev_items, &guard));
    }
  }

  char* wsb = reinterpret_cast<char*>(ws);
  const int L = (int)m->layers.size();
  const void* arena = pool ? pool->arena : nullptr;
  const bool f16 = precision == GW_FP16;
  if (!(flags & GW_TRAIN) && (precision == GW_BF16 || f16) && m->fused && !(flags & GW_LAYERWISE)) {
    // whole network in one kernel, activations on chip
    gw::ConvP p{};
    p.n = n;
    p.items = dev_items;
    p.arena = arena;
    p.x = x ? x + a_band : nullptr;
    p.ldx = x ? W : 0;
    p.noise = noise;
    p.clean = clean;
    p.strain = strain;
    p.upd = upd;
    const uint16_t* wpk[9];
    const float* sc[9];
    const float* sh[9];
    for (int l = 0; l < 9; ++l) {
      const LayerD& ly = m->layers[l];
      const size_t off = gw::dc_fused_special(l) ? (f16 ? ly.wfs16 : ly.wfs) : (f16 ? ly.wf16 : ly.wbf);
      wpk[l] = reinterpret_cast<const uint16_t*>(m->packed + off);
      sc[l] = reinterpret_cast<const float*>(m->packed + m->layers[l].scale);
      sh[l] = reinterpret_cast<const float*>(m->packed + m->layers[l].shift);
    }
    LAUNCH(f16 ? "dc_fused_f16" : "dc_fused_bf16", st,
           gw::launch_dc_fused_bf16(p, wpk, sc, sh, Wb, pool != nullptr, m->cu_budget, st, f16, upd != nullptr));
    return GW_OK;
  }
  if (upd) return fail(GW_EINVAL, "the fused update runs on the fused BF16 inference path only");
  if (!(flags & GW_TRAIN)) {
    const float* in = x ? x + a_band : nullptr;
    for (int l = 0; l < L; ++l) {
      const LayerD& ly = m->layers[l];
      gw::ConvP p = conv_params(m, ly, n, lin[l], lout[l]);
      p.items = dev_items;
      p.arena = arena;
      p.x = in;
      if (l == 0 && x) p.ldx = W;  // band rows inside full-length input rows
      const int src = (l == 0 && pool) ? gw::SRC_RING : gw::SRC_DENSE;
      int epi;
      if (l == L - 1) {
        epi = gw::EPI_OUT;
        p.noise = noise;
        p.clean = clean;
        p.strain = strain;
      } else {
        epi = ly.bn ? gw::EPI_AFFINE_TANH : gw::EPI_AFFINE;
        p.y = reinterpret_cast<float*>(wsb + w.buf[l & 1]);
        p.yh = reinterpret_cast<uint16_t*>(wsb + w.buf[l & 1]);
      }
      if (precision == GW_BF16 && l > 0) p.xh = reinterpret_cast<const uint16_t*>(in);
      LAUNCH(nm(precision == GW_BF16 ? "dc_conv_bf16" : "dc_conv_fp32", "L", l), st,
             run_conv(p, ly, epi, src, precision, st));
      in = p.y;
    }
    return GW_OK;
  }
  // training forward: z = conv(a) + b, batch statistics, a = tanh(BN(z))
  double* partial = reinterpret_cast<double*>(wsb + w.partial);
  const float* in = x;
  for (int l = 0; l < L; ++l) {
    const LayerD& ly = m->layers[l];
    gw::ConvP p = conv_params(m, ly, n, lin[l], lout[l]);
    p.items = dev_items;
    p.x = in;
    if (precision == GW_BF16) p.wpk_lo = reinterpret_cast<const uint16_t*>(m->packed + ly.wbf_lo);
    if (l == L - 1) {
      p.noise = noise;
      p.clean = clean;
      p.strain = strain;
      LAUNCH(nm("dc_train_conv", "L", l), st, run_conv(p, ly, gw::EPI_OUT, gw::SRC_DENSE, precision, st));
      break;
    }
    float* z = reinterpret_cast<float*>(wsb + (w.ckpt >= 0 ? w.ztmp : (ly.bn ? w.z[l] : w.a[l])));
    float* a;
    if (w.ckpt < 0)
      a = reinterpret_cast<float*>(wsb + w.a[l]);
    else if (l == w.ckpt)
      a = reinterpret_cast<float*>(wsb + w.a[l]);
    else
      a = reinterpret_cast<float*>(wsb + w.atmp[l & 1]);
    if (!ly.bn) z = a;
    p.y = z;
    LAUNCH(nm("dc_train_conv", "L", l), st, run_conv(p, ly, gw::EPI_BIAS, gw::SRC_DENSE, precision, st));
    if (ly.bn) {
      float* mean = reinterpret_cast<float*>(wsb + w.mean[l]);
      float* invstd = reinterpret_cast<float*>(wsb + w.invstd[l]);
      LAUNCH(nm("bn_stats", "L", l), st,
             gw::launch_bn_stats(z, n, ly.co, lout[l], partial, gw::red_chunks(n, lout[l]), mean, invstd, st));
      LAUNCH(nm("bn_apply", "L", l), st,
             gw::launch_bn_apply_tanh(z, mean, invstd, m->params + ly.g, m->params + ly.be, a, n, ly.co,
                                      lout[l], st));
    }
    in = a;
  }
  return GW_OK;
}

// ---------------------------------------------------------------------------
// Incremental forward over per-stream activation caches
// ---------------------------------------------------------------------------
namespace {

// Cache geometry of a DeepClean model for windows of W samples, and the
// byte offset of every layer's ring in a stream's cache.
int cache_layout(const gw_model* m, int W, gw::CacheLayerP& P, size_t* total) {
  if (m->kind != GW_MODEL_DEEPCLEAN) return fail(GW_ESTATE, "not a DeepClean model");
  const int L = (int)m->layers.size();
  if (L > gw::kCacheMaxLayers) return fail(GW_EUNSUPPORTED, "activation caches support at most 16 layers");
  std::vector<int> lin, lout;
  CHK(dc_lengths(m, W, lin, lout));
  size_t off = 0;
  for (int l = 0; l < L; ++l) {
    const LayerD& ly = m->layers[l];
    if (W % lout[l]) return fail(GW_EUNSUPPORTED, "layer length must divide the window");
    gw::CacheGeo& g = P.geo[l];
    g.type = ly.type == GW_LAYER_CONVT ? 1 : 0;
    g.ci = ly.ci;
    g.co = ly.co;
    g.k = ly.k;
    g.s = ly.s;
    g.p = ly.p;
    g.op = ly.op;
    g.Lin = lin[l];
    g.Lout = lout[l];
    g.f = W / lout[l];
    g.bn = ly.bn ? 1 : 0;
    g.f32 = l == L - 1 ? 1 : 0;
    if (16 % g.f) return fail(GW_EUNSUPPORTED, "layer grids must divide the 16-sample shift unit");
    if (!gw::cache_layer_fits(g) || !ly.bf16)
      return fail(GW_EUNSUPPORTED, "no cached kernel for this layer shape (k7 p3 layers with compiled channel tiles)");
    P.off[l] = off;
    off += r256((size_t)g.co * g.Lout * (g.f32 ? 4 : 2));
  }
  P.W = W;
  P.L = L;
  *total = off;
  return GW_OK;
}

}  // namespace


extern "C" int deepclean_forward(const gw_model* m, gw_pool* pool, const int32_t* slots, const float* x,
                                 int32_t n, int32_t W, const int32_t* strides, const int32_t* delays,
                                 const float* strain, float* noise, float* clean, int32_t precision, uint32_t flags,
                                 void* ws, size_t ws_bytes, void* hip_stream) {
  return dc_forward(m, pool, slots, x, n, W, strides, delays, strain, noise, clean, precision, flags, ws, ws_bytes,
                    S(hip_stream), nullptr, nullptr);
}

extern "C" int deepclean_update_forward(const gw_model* m, gw_pool* pool, int32_t n, const int32_t* slots,
                                        const int32_t* strides, const float* samples, const int64_t* offsets,
                                        int32_t W, const int32_t* delays, const float* strain, float* noise,
                                        float* clean, int32_t precision, uint32_t flags, void* ws, size_t ws_bytes,
                                        void* hip_stream) {
  if (!m) return fail(GW_EINVAL, "null model");
  if (!pool) return fail(GW_EINVAL, "null pool");
  if (n == 0) return GW_OK;
  if (n < 0 || n > pool->max_items) return fail(GW_EINVAL, "n out of range");
  if (!slots || !strides || !samples || !offsets) return fail(GW_EINVAL, "null argument");
  const bool one_launch = m->kind == GW_MODEL_DEEPCLEAN && precision == GW_BF16 && m->fused && flags == 0;
  if (!one_launch) {
    CHK(snapshot_update(pool, n, slots, strides, samples, offsets, hip_stream));
    return deepclean_forward(m, pool, slots, nullptr, n, W, strides, delays, strain, noise, clean, precision, flags,
                             ws, ws_bytes, hip_stream);
  }
  // the update's checks (the forward checks the rest before it launches)
  std::vector<char> seen(pool->max_slots, 0);
  for (int i = 0; i < n; ++i) {
    CHK(pool->check_slot(slots[i]));
    if (seen[slots[i]]) return fail(GW_EINVAL, "slot appears twice in one call");
    seen[slots[i]] = 1;
    if (strides[i] < 1 || strides[i] > pool->slots[slots[i]].W) return fail(GW_EINVAL, "stride must be in [1, W]");
    if (offsets[i] < 0) return fail(GW_EINVAL, "negative sample offset");
  }
  // advance the host state as snapshot_update does; restored if the forward
  // refuses the call
  std::vector<std::pair<int, int64_t>> prev(n);
  for (int i = 0; i < n; ++i) {
    auto& sl = pool->slots[slots[i]];
    prev[i] = {sl.head, sl.n_seen};
    sl.head = (sl.head + strides[i]) % sl.W;
    sl.n_seen += strides[i];
  }
  const int rc = dc_forward(m, pool, slots, nullptr, n, W, strides, delays, strain, noise, clean, precision, flags,
                            ws, ws_bytes, S(hip_stream), samples, offsets);
  if (rc != GW_OK)
    for (int i = 0; i < n; ++i) {
      auto& sl = pool->slots[slots[i]];
      sl.head = prev[i].first;
      sl.n_seen = prev[i].second;
    }
  return rc;
}

extern "C" int deepclean_cache_bytes(const gw_model* m, int32_t W, size_t* bytes) {
  if (!m || !bytes) return fail(GW_EINVAL, "null argument");
  gw::CacheLayerP P{};
  return cache_layout(m, W, P, bytes);
}

extern "C" int deepclean_cache_bands(const int32_t* desc, int32_t desc_len, int32_t W, int32_t shift, int32_t* zl,
                                     int32_t* zr) {
  if (!desc || !zl || !zr) return fail(GW_EINVAL, "null argument");
  gw_model m;  // host-side layout only
  CHK(build_layout(GW_MODEL_DEEPCLEAN, desc, desc_len, m));
  gw::CacheLayerP P{};
  size_t total = 0;
  CHK(cache_layout(&m, W, P, &total));
  if (shift >= 0 && (shift % 16 || shift >= W)) return fail(GW_EINVAL, "shift must be a multiple of 16 below W, or -1");
  for (int l = 0; l < (int)m.layers.size(); ++l) gw::cache_band(P.geo, l, shift, W, &zl[l], &zr[l]);
  return GW_OK;
}

extern "C" int gw_stream_attach_cache(gw_pool* pool, int32_t slot, void* cache, size_t bytes) {
  if (!pool) return fail(GW_EINVAL, "null pool");
  CHK(pool->check_slot(slot));
  if (cache && reinterpret_cast<uintptr_t>(cache) % 256) return fail(GW_EINVAL, "cache not 256-byte aligned");
  auto& s = pool->slots[slot];
  s.cache = cache;
  s.cache_bytes = cache ? bytes : 0;
  s.cache_valid = false;
  return GW_OK;
}

extern "C" int deepclean_forward_cached(const gw_model* m, gw_pool* pool, const int32_t* slots, int32_t n,
                                        int32_t W, const int32_t* strides, const int32_t* delays,
                                        const float* strain, float* noise, float* clean, uint32_t flags,
                                        void* hip_stream) {
  const hipStream_t st = S(hip_stream);
  if (!m || !pool || !slots) return fail(GW_EINVAL, "null model, pool or slots");
  if (n == 0) return GW_OK;
  if (n < 0) return fail(GW_EINVAL, "negative n");
  if (flags & ~GW_CACHE_FULL) return fail(GW_EINVAL, "bad flags");
  if (clean && (!strides || !strain)) return fail(GW_EINVAL, "clean output needs strides and strain");
  if (delays && !clean) return fail(GW_EINVAL, "delays apply to the clean output");
  gw::CacheLayerP P{};
  size_t need = 0;
  CHK(cache_layout(m, W, P, &need));
  std::vector<gw::CacheItem> items(n);
  std::vector<char> seen(pool->max_slots, 0);
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    CHK(pool->check_slot(slots[i]));
    if (seen[slots[i]]) return fail(GW_EINVAL, "slot appears twice in one call");
    seen[slots[i]] = 1;
    const auto& sl = pool->slots[slots[i]];
    if (sl.C != m->c_in || sl.W != W) return fail(GW_EINVAL, "slot C/W does not match the model and W");
    if (!sl.cache || sl.cache_bytes < need)
      return fail(GW_EINVAL, "slot has no activation cache of deepclean_cache_bytes bytes attached");
    gw::CacheItem& it = items[i];
    std::memset(&it, 0, sizeof(it));
    it.cache = sl.cache;
    it.shadow = pool->shadow_elem(sl);
    it.in_head = sl.head;  // oldest sample of the current window
    const int64_t adv = sl.n_seen - sl.cache_seen;
    if (!sl.cache_valid || sl.cache_model != m->id || sl.cache_gen != m->gen || (flags & GW_CACHE_FULL) || adv < 0 ||
        adv >= W || adv % 16) {
      it.shift = -1;
      it.T = 0;
    } else {
      it.shift = (int32_t)adv;
      it.T = (int32_t)((sl.cache_T + adv) % W);
    }
    if (clean) {
      if (strides[i] < 1 || strides[i] > W) return fail(GW_EINVAL, "stride must be in [1, W]");
      it.s = strides[i];
      it.delay = delays ? delays[i] : 0;
      if (it.delay < 0 || it.delay > W - it.s) return fail(GW_EINVAL, "delay must be in [0, W - stride]");
      it.out = off;
      off += strides[i];
    }
  }
  const int L = (int)m->layers.size();
  const void* dev = nullptr;
  StageGuard guard;
  CHK(pool->stager.stage_raw(items.data(), items.size() * sizeof(gw::CacheItem), st, &dev, &guard));
  // until every launch is enqueued the caches hold no known window (an error
  // below leaves them to be recomputed in full by the next call)
  for (int i = 0; i < n; ++i) pool->slots[slots[i]].cache_valid = false;
  pool->mark_used(slots, n, guard);
  const auto* dit = reinterpret_cast<const gw::CacheItem*>(dev);
  for (int l = 0; l < L; ++l) {
    const LayerD& ly = m->layers[l];
    P.wpk[l] = reinterpret_cast<const uint16_t*>(m->packed + ly.wbf);
    P.scale[l] = reinterpret_cast<const float*>(m->packed + ly.scale);
    P.shift[l] = reinterpret_cast<const float*>(m->packed + ly.shift);
  }
  LAUNCH("cache_forward", st, gw::launch_cache_forward(dit, n, pool->arena, P, strain, noise, clean, st));
  // every cache now holds the current window
  for (int i = 0; i < n; ++i) {
    auto& sl = pool->slots[slots[i]];
    sl.cache_valid = true;
    sl.cache_T = items[i].T;
    sl.cache_seen = sl.n_seen;
    sl.cache_model = m->id;
    sl.cache_gen = m->gen;
  }
  return GW_OK;
}

// ---------------------------------------------------------------------------
// Backward
// ---------------------------------------------------------------------------
namespace {

struct BwWs {
  size_t g[2] = {0, 0};
  size_t dz = 0;
  std::vector<size_t> z, a;  // recomputed activations (recompute mode)
  size_t partial = 0;
  size_t wg = 0;
  size_t total = 0;
};

int bw_layout(const gw_model* m, int n, int W, uint32_t flags, BwWs& b) {
  std::vector<int> lin, lout;
  CHK(dc_lengths(m, W, lin, lout));
  const int L = (int)m->layers.size();
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += r256(bytes);
    return o;
  };
  size_t mx = 256, mxin = 256, mwg = 256;
  int maxc = 1, maxchunk = 1;
  for (int l = 0; l < L; ++l) {
    const auto& ly = m->layers[l];
    mx = std::max(mx, (size_t)n * ly.co * lout[l] * 4);
    if (l > 0) mxin = std::max(mxin, (size_t)n * ly.ci * lin[l] * 4);
    maxc = std::max(maxc, ly.co);
    maxchunk = std::max(maxchunk, gw::red_chunks(n, lout[l]));
    const bool tr = ly.type == GW_LAYER_CONVT;
    const int Lp = tr ? lin[l] : lout[l];
    mwg = std::max(mwg, gw::wgrad_scratch_bytes(n, Lp, ly.ci * ly.co * ly.k));
  }
  b.g[0] = take(mxin);
  b.g[1] = take(mxin);
  b.dz = take(mx);
  b.z.assign(L, NONE);
  b.a.assign(L, NONE);
  if (flags & GW_RECOMPUTE) {
    // The two segments (up to and including the checkpoint layer, and after
    // it) are recomputed one at a time, so they share one region.
    int ck = 0;
    for (int l = 0; l + 1 < L; ++l)
      if (lout[l] < lout[ck]) ck = l;
    const size_t base = off;
    size_t seg_end[2] = {base, base};
    for (int l = 0; l + 1 < L; ++l) {
      size_t& e = seg_end[l <= ck ? 0 : 1];
      const size_t sz = r256((size_t)n * m->layers[l].co * lout[l] * 4);
      if (m->layers[l].bn) {
        b.z[l] = e;
        e += sz;
      }
      b.a[l] = e;
      e += sz;
    }
    off = std::max(seg_end[0], seg_end[1]);
  }
  b.partial = take((size_t)maxc * maxchunk * 2 * sizeof(double));
  b.wg = take(mwg);
  b.total = off;
  return GW_OK;
}

}  // namespace

extern "C" int gw_decimate2(int32_t n, int32_t C, int32_t s, int32_t ntaps, const float* taps, const float* x,
                            float* hist, float* y, void* hip_stream) {
  const hipStream_t st = S(hip_stream);
  if (n == 0) return GW_OK;
  if (n < 0 || C < 1 || C > 65535) return fail(GW_EINVAL, "need n >= 0 and 1 <= C <= 65535");
  if (s < 2 || s % 2) return fail(GW_EINVAL, "stride must be even and positive");
  if (ntaps < 1 || ntaps > 257) return fail(GW_EINVAL, "ntaps must be in [1, 257]");
  if (!taps || !x || !y || (ntaps > 1 && !hist)) return fail(GW_EINVAL, "null argument");
  LAUNCH("decimate2", st, gw::launch_decimate2(n, C, s, ntaps, taps, x, hist, y, st));
  return GW_OK;
}

extern "C" int deepclean_overlap_average(const gw_model* m, int32_t n, int32_t W, const int32_t* strides,
                                         int32_t depth, const int64_t* counts, const float* noise, float* state,
                                         const float* strain, float* clean, float* avg, void* hip_stream) {
  const hipStream_t st = S(hip_stream);
  if (!m) return fail(GW_EINVAL, "null model");
  if (m->kind != GW_MODEL_DEEPCLEAN) return fail(GW_ESTATE, "not a DeepClean model");
  if (n == 0) return GW_OK;
  if (n < 0 || W < 1 || depth < 1) return fail(GW_EINVAL, "need n >= 0, W >= 1, depth >= 1");
  if (!strides || !counts || !noise || !state) return fail(GW_EINVAL, "null argument");
  if (!clean && !avg) return fail(GW_EINVAL, "no output requested");
  if (clean && !strain) return fail(GW_EINVAL, "clean output needs strain");
  std::vector<Item> items(n);
  int64_t off = 0, soff = 0;
  int max_s = 1;
  for (int i = 0; i < n; ++i) {
    const int s = strides[i];
    if (s < 1 || (int64_t)depth * s > W) return fail(GW_EINVAL, "stride must be in [1, W / depth]");
    if (counts[i] < 0) return fail(GW_EINVAL, "negative request count");
    Item& it = items[i];
    std::memset(&it, 0, sizeof(it));
    it.s = s;
    it.out = off;
    it.src = soff;
    it.head = (int)(counts[i] % depth);
    it.C = (int)std::min<int64_t>(depth, counts[i] + 1);
    off += s;
    soff += (int64_t)depth * s;
    max_s = std::max(max_s, s);
  }
  const Item* dev_items = nullptr;
  StageGuard guard;
  CHK(const_cast<gw_model*>(m)->stager.stage(items, st, &dev_items, &guard));
  LAUNCH("overlap_average", st,
         gw::launch_overlap_average(dev_items, n, max_s, W, depth, noise, state, strain, clean, avg, st));
  return GW_OK;
}

extern "C" int deepclean_backward_scratch(const gw_model* m, int32_t n, int32_t W, uint32_t flags,
                                          size_t* bytes) {
  if (!m || !bytes) return fail(GW_EINVAL, "null argument");
  if (m->kind != GW_MODEL_DEEPCLEAN) return fail(GW_ESTATE, "not a DeepClean model");
  if (n < 1) return fail(GW_EINVAL, "n must be >= 1");
  BwWs b;
  CHK(bw_layout(m, n, W, flags, b));
  *bytes = b.total;
  return GW_OK;
}

extern "C" int deepclean_backward(const gw_model* m, int32_t n, int32_t W, const float* x,
                                  const float* dnoise, const void* saved, float* dparams,
                                  uint32_t flags, int32_t precision, void* scratch,
                                  size_t scratch_bytes, void* hip_stream) {
  const hipStream_t st = S(hip_stream);
  if (!m) return fail(GW_EINVAL, "null model");
  if (m->kind != GW_MODEL_DEEPCLEAN) return fail(GW_ESTATE, "not a DeepClean model");
  if (n < 1) return fail(GW_EINVAL, "n must be >= 1");
  if (!x || !dnoise || !saved || !dparams || !scratch) return fail(GW_EINVAL, "null argument");
  if (!(flags & GW_TRAIN) || (flags & ~(GW_TRAIN | GW_RECOMPUTE)))
    return fail(GW_EINVAL, "flags must be GW_TRAIN or GW_TRAIN|GW_RECOMPUTE (as in the forward)");
  if (precision == GW_FP16) return fail(GW_EUNSUPPORTED, "FP16 is an inference variant");
  if (precision != GW_FP32 && precision != GW_BF16) return fail(GW_EINVAL, "bad precision");
  if (precision == GW_BF16 && !m->bf16_all) return fail(GW_EUNSUPPORTED, "no BF16 kernel for this network");
  DcWs w;
  CHK(dc_ws_layout(m, n, W, precision, flags, w));
  BwWs b;
  CHK(bw_layout(m, n, W, flags, b));
  if (scratch_bytes < b.total)
    return fail(GW_EINVAL, "scratch too small: need " + std::to_string(b.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(scratch) % 256 || reinterpret_cast<uintptr_t>(saved) % 256)
    return fail(GW_EINVAL, "saved/scratch not 256-byte aligned");
  std::vector<int> lin, lout;
  CHK(dc_lengths(m, W, lin, lout));
  const int L = (int)m->layers.size();
  const char* sv = reinterpret_cast<const char*>(saved);
  char* sc = reinterpret_cast<char*>(scratch);
  double* partial = reinterpret_cast<double*>(sc + b.partial);
  const bool rec = flags & GW_RECOMPUTE;
  auto savedf = [&](size_t off) { return reinterpret_cast<const float*>(sv + off); };
  auto scf = [&](size_t off) { return reinterpret_cast<float*>(sc + off); };

  std::vector<const float*> Z(L, nullptr), A(L, nullptr);
  if (rec) A[w.ckpt] = savedf(w.a[w.ckpt]);
  if (!rec)
    for (int l = 0; l + 1 < L; ++l) {
      A[l] = savedf(w.a[l]);
      Z[l] = m->layers[l].bn ? savedf(w.z[l]) : A[l];
    }
  // recompute layers [l0, l1] from `in` with the saved statistics
  auto recompute = [&](int l0, int l1, const float* in) -> int {
    for (int l = l0; l <= l1; ++l) {
      const LayerD& ly = m->layers[l];
      gw::ConvP p = conv_params(m, ly, n, lin[l], lout[l]);
      p.x = in;
      if (precision == GW_BF16) p.wpk_lo = reinterpret_cast<const uint16_t*>(m->packed + ly.wbf_lo);
      float* a = scf(b.a[l]);
      float* z = ly.bn ? scf(b.z[l]) : a;
      p.y = z;
      LAUNCH(nm("dc_recompute_conv", "L", l), st, run_conv(p, ly, gw::EPI_BIAS, gw::SRC_DENSE, precision, st));
      if (ly.bn)
        LAUNCH(nm("bn_apply", "L", l), st, gw::launch_bn_apply_tanh(z, savedf(w.mean[l]), savedf(w.invstd[l]), m->params + ly.g,
                                        m->params + ly.be, a, n, ly.co, lout[l], st));
      Z[l] = z;
      A[l] = a;
      in = a;
    }
    return GW_OK;
  };
  // running-statistics entries and the biases of normalised layers have
  // zero gradient; every other entry is written below
  LAUNCH("zero", st, gw::launch_zero_floats(dparams, m->n_params, st));
  const float* g = dnoise;
  int gi = 0;
  for (int l = L - 1; l >= 0; --l) {
    if (rec) {
      if (l == L - 1 && w.ckpt + 1 <= L - 2) CHK(recompute(w.ckpt + 1, L - 2, savedf(w.a[w.ckpt])));
      if (l == w.ckpt) CHK(recompute(0, w.ckpt, x));
    }
    const LayerD& ly = m->layers[l];
    const float* a_in = l == 0 ? x : A[l - 1];
    const float* dz = g;
    float* dzb = scf(b.dz);
    if (ly.bn) {
      LAUNCH(nm("bn_bwd", "L", l), st, gw::launch_bn_tanh_backward(g, A[l], Z[l], savedf(w.mean[l]), savedf(w.invstd[l]),
                                         m->params + ly.g, n, ly.co, lout[l], partial,
                                         gw::red_chunks(n, lout[l]), dzb, dparams + ly.g,
                                         dparams + ly.be, st));
      dz = dzb;
    }
    // a conv bias followed by batch-statistics normalisation has an exactly
    // zero gradient (the batch mean removes it): left at the initial zero
    if (!ly.bn)
      LAUNCH(nm("bias_grad", "L", l), st, gw::launch_channel_sum(dz, n, ly.co, lout[l], partial,
                                                                  gw::red_chunks(n, lout[l]), dparams + ly.b, st));
    if (ly.type == GW_LAYER_CONV)
      LAUNCH(nm("wgrad", "L", l), st, gw::launch_wgrad(dz, ly.co, lout[l], a_in, ly.ci, lin[l], n, ly.k, ly.s, ly.p, sc + b.wg,
                              dparams + ly.w, st));
    else
      LAUNCH(nm("wgrad", "L", l), st, gw::launch_wgrad(a_in, ly.ci, lin[l], dz, ly.co, lout[l], n, ly.k, ly.s, ly.p, sc + b.wg,
                              dparams + ly.w, st));
    if (l == 0) break;
    // input gradient: the adjoint convolution with the same weights
    gw::ConvP p{};
    p.n = n;
    p.Ci = ly.co;
    p.Co = ly.ci;
    p.Lin = lout[l];
    p.Lout = lin[l];
    p.k = ly.k;
    p.stride = ly.s;
    p.pad = ly.p;
    p.w = m->params + ly.w;
    p.x = dz;
    p.bias = nullptr;
    float* gout = scf(b.g[gi]);
    gi ^= 1;
    p.y = gout;
    if (precision == GW_BF16 && ly.dg_mfma) {
      // split BF16 operands on the matrix cores (as the forward convolutions)
      p.wpk = reinterpret_cast<const uint16_t*>(m->packed + ly.wdg);
      p.wpk_lo = reinterpret_cast<const uint16_t*>(m->packed + ly.wdg_lo);
      LAUNCH(nm("dgrad_bf16", "L", l), st,
             gw::launch_conv_bf16(p, ly.type == GW_LAYER_CONV, gw::EPI_BIAS, gw::SRC_DENSE, st));
    } else if (ly.type == GW_LAYER_CONV) {
      p.wsi = (int64_t)ly.ci * ly.k;  // transposed kernel reads w[i*wsi + o*wso + j], i = conv out ch
      p.wso = ly.k;
      LAUNCH(nm("dgrad", "L", l), st, gw::launch_conv_fp32(p, true, gw::EPI_BIAS, gw::SRC_DENSE, st));
    } else {
      p.wso = (int64_t)ly.co * ly.k;  // conv kernel reads w[o*wso + i*wsi + j], o = convT in ch
      p.wsi = ly.k;
      LAUNCH(nm("dgrad", "L", l), st, gw::launch_conv_fp32(p, false, gw::EPI_BIAS, gw::SRC_DENSE, st));
    }
    g = gout;
  }
  return GW_OK;
}

// ===========================================================================
// Band-passed MSE
// ===========================================================================
namespace {
int band(int W, float fs, float f_lo, float f_hi, int* k_lo, int* k_hi) {
  if (W < 2 || !(fs > 0) || !(f_lo >= 0) || !(f_hi >= f_lo)) return fail(GW_EINVAL, "bad band");
  int lo = -1, hi = -2;
  for (int k = 0; k <= W / 2; ++k) {
    const double f = (double)k * (double)fs / (double)W;
    if (f >= (double)f_lo && f <= (double)f_hi) {
      if (lo < 0) lo = k;
      hi = k;
    }
  }
  if (lo < 0) return fail(GW_EINVAL, "no DFT bin inside the band");
  *k_lo = lo;
  *k_hi = hi;
  return GW_OK;
}
}  // namespace

extern "C" int gw_bandpass_workspace(int32_t n, int32_t W, float fs, float f_lo, float f_hi,
                                     size_t* bytes) {
  if (!bytes || n < 1) return fail(GW_EINVAL, "bad argument");
  int lo, hi;
  CHK(band(W, fs, f_lo, f_hi, &lo, &hi));
  *bytes = r256(gw::bandpass_ws_floats(n, W, hi - lo + 1) * sizeof(float));
  return GW_OK;
}

extern "C" int gw_bandpass_mse(int32_t n, int32_t W, float fs, float f_lo, float f_hi,
                               const float* strain, const float* noise, float* loss, float* dnoise,
                               void* ws, size_t ws_bytes, void* hip_stream) {
  if (n < 1 || !strain || !noise || !ws || (!loss && !dnoise)) return fail(GW_EINVAL, "bad argument");
  int lo, hi;
  CHK(band(W, fs, f_lo, f_hi, &lo, &hi));
  if (ws_bytes < gw::bandpass_ws_floats(n, W, hi - lo + 1) * sizeof(float))
    return fail(GW_EINVAL, "workspace too small");
  LAUNCH("bandpass", S(hip_stream), gw::launch_bandpass(n, W, lo, hi, strain, noise, reinterpret_cast<float*>(ws), loss, dnoise,
                             S(hip_stream)));
  return GW_OK;
}

// ---------------------------------------------------------------------------
// Band-passed MSE without allocation.  The projection scratch of
// gw_bandpass_mse (n x bins (cos, sin) pairs) lives in a file-scope device
// array: every GPU the library runs on holds one copy until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory, so
// the kernels get the address that hipGetSymbolAddress returns for the
// stream's device (looked up once per device, with that device current).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // per device ordinal; null until looked up

int scratch_for_stream(hipStream_t st, void** out) {
  int dev = -1;
  if (st)
    HIPCHK(hipStreamGetDevice(st, &dev));
  else
    HIPCHK(hipGetDevice(&dev));  // the null stream runs on the current device
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)dev >= g_scratch_dev.size()) g_scratch_dev.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) HIPCHK(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(GW_EHIP, "hipGetSymbolAddress(scratch) returned a null address");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return GW_OK;
}
}  // namespace

extern "C" int gw_bandpass_mse_noalloc(int32_t n, int32_t W, float fs, float f_lo, float f_hi,
                                       const float* strain, const float* noise, float* loss, float* dnoise,
                                       void* hip_stream) {
  if (n < 1 || !strain || !noise || (!loss && !dnoise)) return fail(GW_EINVAL, "bad argument");
  int lo, hi;
  CHK(band(W, fs, f_lo, f_hi, &lo, &hi));
  const size_t need = gw::bandpass_ws_floats(n, W, hi - lo + 1) * sizeof(float);
  if (need > kNoAllocScratchBytes)
    return fail(GW_EINVAL, "n x band bins = " + std::to_string((size_t)n * (hi - lo + 1)) +
                               " exceeds the no-allocation scratch limit of " +
                               std::to_string(kNoAllocScratchBytes / (2 * sizeof(float))));
  void* ptr = nullptr;
  CHK(scratch_for_stream(S(hip_stream), &ptr));
  // every (window, bin) pair the loss and gradient read is written first by
  // this call's projection kernel, so nothing in the array needs clearing
  HIPCHK(gw::launch_bandpass(n, W, lo, hi, strain, noise, reinterpret_cast<float*>(ptr), loss, dnoise,
                             S(hip_stream)));
  return GW_OK;
}

// ===========================================================================
// BBHnet
// ===========================================================================
namespace {
// partial sums per window of the pooled last BBHnet stage (column tiles x
// channel shares; 16 for 2048-sample windows)
constexpr int kGapParts = 256;

struct BbWs {
  size_t gath = NONE, h = 0, o[2] = {0, 0}, gap = 0, total = 0;
};
int bb_layout(const gw_model* m, int n, int W, bool pool, int precision, BbWs& b) {
  const int Sn = (int)m->stages.size();
  if (W < 1 || W % (1 << Sn)) return fail(GW_EINVAL, "W must be a multiple of 2^stages");
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += r256(bytes);
    return o;
  };
  (void)precision;
  if (pool) b.gath = take((size_t)n * m->c_in * W * 4);
  size_t mh = 256;
  int L = W;
  for (auto& sd : m->stages) {
    L /= 2;
    mh = std::max(mh, (size_t)n * sd.co * L * 4);
  }
  b.h = take(mh);
  b.o[0] = take(mh);
  b.o[1] = take(mh);
  b.gap = take((size_t)n * kGapParts * sizeof(float));
  b.total = off;
  return GW_OK;
}
}  // namespace

namespace {
// The whole BBHnet in one kernel (blocks of 64 last-stage positions), then
// the fixed-order sum of each window's pooled-head shares into its logit.
int bbh_fused_forward(const gw_model* m, const void* arena, const Item* items, const float* x, int n, int W,
                      char* gap, float* logits, hipStream_t st) {
  gw::BbFusedP fp{};
  fp.arena = arena;
  fp.items = items;
  fp.x = x;
  const float* P = m->params;
  for (int s = 0; s < 3; ++s) {
    const StageD& sd = m->stages[s];
    fp.wa[s] = reinterpret_cast<const uint16_t*>(m->packed + sd.wa_bf);
    fp.wb[s] = reinterpret_cast<const uint16_t*>(m->packed + sd.wb_bf);
    fp.ws[s] = reinterpret_cast<const uint16_t*>(m->packed + sd.ws_bf);
    fp.ba[s] = P + sd.ba;
    fp.bb[s] = P + sd.bb;
    fp.bs[s] = P + sd.bs;
  }
  fp.hw = P + m->head_w;
  fp.part = reinterpret_cast<float*>(gap);
  fp.n = n;
  fp.W = W;
  fp.tiles = gw::bbh_fused_tiles(W);
  LAUNCH("bbh_fused", st, gw::launch_bbh_fused(fp, st));
  LAUNCH("gap_finalize", st, gw::launch_gap_finalize(fp.part, fp.tiles, P + m->head_b, logits, n, W / 8, st));
  return GW_OK;
}
}  // namespace

extern "C" int bbhnet_workspace(const gw_model* m, int32_t n, int32_t W, int32_t precision,
                                size_t* bytes) {
  if (!m || !bytes) return fail(GW_EINVAL, "null argument");
  if (m->kind != GW_MODEL_BBHNET) return fail(GW_ESTATE, "not a BBHnet model");
  if (n < 1) return fail(GW_EINVAL, "n must be >= 1");
  BbWs b;
  CHK(bb_layout(m, n, W, true, precision, b));
  *bytes = b.total;
  return GW_OK;
}

extern "C" int bbhnet_forward(const gw_model* m, gw_pool* pool, const int32_t* slots, const float* x,
                              int32_t n, int32_t W, float* logits, int32_t precision, void* ws,
                              size_t ws_bytes, void* hip_stream) {
  const hipStream_t st = S(hip_stream);
  if (!m) return fail(GW_EINVAL, "null model");
  if (m->kind != GW_MODEL_BBHNET) return fail(GW_ESTATE, "not a BBHnet model");
  if (n == 0) return GW_OK;
  if (n < 0) return fail(GW_EINVAL, "negative n");
  if ((pool != nullptr) == (x != nullptr)) return fail(GW_EINVAL, "exactly one of pool and x must be given");
  if (pool && !slots) return fail(GW_EINVAL, "pool input needs slots");
  if (!logits || !ws) return fail(GW_EINVAL, "null logits or workspace");
  if (precision == GW_FP16) return fail(GW_EUNSUPPORTED, "no FP16 BBHnet kernels");
  if (precision != GW_FP32 && precision != GW_BF16) return fail(GW_EINVAL, "bad precision");
  if (precision == GW_BF16 && !m->bf16_all) return fail(GW_EUNSUPPORTED, "no BF16 kernel for this network");
  BbWs b;
  CHK(bb_layout(m, n, W, pool != nullptr, precision, b));
  if (ws_bytes < b.total) return fail(GW_EINVAL, "workspace too small: need " + std::to_string(b.total) + " bytes");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(GW_EINVAL, "workspace not 256-byte aligned");
  char* wsb = reinterpret_cast<char*>(ws);
  const float* in = x;
  StageGuard guard;  // the gathered window is read by the first stage only, but
                     // the table stays reserved until the call's last launch
  const bool fused = precision == GW_BF16 && m->fused && !m->layerwise && gw::bbh_fused_tiles(W) <= kGapParts;
  if (pool) {
    std::vector<Item> items(n);
    std::vector<char> seen(pool->max_slots, 0);
    for (int i = 0; i < n; ++i) {
      CHK(pool->check_slot(slots[i]));
      if (seen[slots[i]]) return fail(GW_EINVAL, "slot appears twice in one call");
      seen[slots[i]] = 1;
      const auto& s = pool->slots[slots[i]];
      if (s.C != m->c_in || s.W != W) return fail(GW_EINVAL, "slot C/W does not match the model and W");
      std::memset(&items[i], 0, sizeof(Item));
      items[i].ring = pool->ring_elem(s);
      items[i].shadow = pool->shadow_elem(s);
      items[i].head = s.head;
      items[i].C = s.C;
      items[i].W = s.W;
    }
    const Item* dev = nullptr;
    CHK(pool->stager.stage(items, st, &dev, &guard));
    pool->mark_used(slots, n, guard);
    if (fused) {
      // the fused kernel reads every window straight from its ring
      CHK(bbh_fused_forward(m, pool->arena, dev, nullptr, n, W, wsb + b.gap, logits, st));
      return GW_OK;
    }
    float* g = reinterpret_cast<float*>(wsb + b.gath);
    LAUNCH("gather", st, gw::launch_gather(pool->arena, dev, n, m->c_in, W, g, nullptr, st));
    in = g;
  } else if (fused) {
    CHK(bbh_fused_forward(m, nullptr, nullptr, x, n, W, wsb + b.gap, logits, st));
    return GW_OK;
  }
  int L = W;
  const float* P = m->params;
  const bool bf = precision == GW_BF16;
  const int Sn = (int)m->stages.size();
  const void* cur = in;  // stage input: fp32 for stage 0, bf16 after (BF16 path)
  for (int s = 0; s < Sn; ++s) {
    const auto& sd = m->stages[s];
    const int Lo = L / 2;
    const bool last = s == Sn - 1;
    gw::ConvP pa{};
    pa.n = n;
    pa.Ci = sd.ci;
    pa.Co = sd.co;
    pa.Lin = L;
    pa.Lout = Lo;
    pa.k = 7;
    pa.stride = 2;
    pa.pad = 3;
    pa.w = P + sd.wa;
    pa.wso = (int64_t)sd.ci * 7;
    pa.wsi = 7;
    pa.bias = P + sd.ba;
    gw::ConvP pb{};
    pb.n = n;
    pb.Ci = sd.co;
    pb.Co = sd.co;
    pb.Lin = Lo;
    pb.Lout = Lo;
    pb.k = 7;
    pb.stride = 1;
    pb.pad = 3;
    pb.w = P + sd.wb;
    pb.wso = (int64_t)sd.co * 7;
    pb.wsi = 7;
    pb.bias = P + sd.bb;
    pb.Cs = sd.ci;
    pb.Ls = L;
    pb.ws = P + sd.ws;
    pb.bs = P + sd.bs;
    void* hbuf = wsb + b.h;
    void* obuf = wsb + b.o[s & 1];
    if (bf) {
      pa.wpk = reinterpret_cast<const uint16_t*>(m->packed + sd.wa_bf);
      pb.wpk = reinterpret_cast<const uint16_t*>(m->packed + sd.wb_bf);
      pb.wspk = reinterpret_cast<const uint16_t*>(m->packed + sd.ws_bf);
      if (s == 0) {
        pa.x = reinterpret_cast<const float*>(cur);
        pb.xs = reinterpret_cast<const float*>(cur);
      } else {
        pa.xh = reinterpret_cast<const uint16_t*>(cur);
        pb.xsh = reinterpret_cast<const uint16_t*>(cur);
      }
      pa.yh = reinterpret_cast<uint16_t*>(hbuf);
      pb.xh = pa.yh;
      int epi_b = gw::EPI_RESID_RELU;
      if (last) {
        // last stage: the pooling head is fused into the epilogue
        const int nblk = gw::conv_bf16_gap_parts(pb.Ci, sd.co, Lo, n);
        if (nblk < 1 || nblk > kGapParts) return fail(GW_EUNSUPPORTED, "window too long for the fused pooling head");
        pb.hw = P + m->head_w;
        pb.gap_part = reinterpret_cast<float*>(wsb + b.gap);
        epi_b = gw::EPI_RESID_GAP;
      } else {
        pb.yh = reinterpret_cast<uint16_t*>(obuf);
      }
      LAUNCH(nm("bbh_conva_bf16", "S", s), st, gw::launch_conv_bf16(pa, false, gw::EPI_RELU, gw::SRC_DENSE, st));
      LAUNCH(nm("bbh_convb_bf16", "S", s), st, gw::launch_conv_bf16(pb, false, epi_b, gw::SRC_DENSE, st));
      if (last) {
        const int nblk = gw::conv_bf16_gap_parts(pb.Ci, sd.co, Lo, n);
        LAUNCH("gap_finalize", st,
               gw::launch_gap_finalize(pb.gap_part, nblk, P + m->head_b, logits, n, Lo, st));
      }
    } else {
      pa.x = reinterpret_cast<const float*>(cur);
      pa.y = reinterpret_cast<float*>(hbuf);
      pb.x = pa.y;
      pb.xs = reinterpret_cast<const float*>(cur);
      pb.y = reinterpret_cast<float*>(obuf);
      LAUNCH(nm("bbh_conva_fp32", "S", s), st, gw::launch_conv_fp32(pa, false, gw::EPI_RELU, gw::SRC_DENSE, st));
      LAUNCH(nm("bbh_convb_fp32", "S", s), st,
             gw::launch_conv_fp32(pb, false, gw::EPI_RESID_RELU, gw::SRC_DENSE, st));
    }
    cur = obuf;
    L = Lo;
  }
  in = reinterpret_cast<const float*>(cur);
  if (bf) return GW_OK;  // BF16: the pooling head ran in the last stage's epilogue
  LAUNCH("gap_linear", st, gw::launch_gap_linear(in, P + m->head_w, P + m->head_b, logits, n, m->c_last, L, st));
  return GW_OK;
}

// ---------------------------------------------------------------------------
// Host staging copies on a small persistent thread pool.  A call splits its
// copies into contiguous runs of about equal bytes, one per participating
// thread (the caller takes run 0); workers wait on a condition variable for
// the next call's generation and report completion through a counter.  The
// pool is created on first use and never torn down (its threads are detached
// and idle between calls).
// ---------------------------------------------------------------------------
namespace {

struct CopyPool {
  std::mutex call;  // one call at a time
  std::mutex m;
  std::condition_variable wake, done;
  uint64_t gen = 0;
  int nrun = 0, pending = 0;
  void* const* dst = nullptr;
  const void* const* src = nullptr;
  const size_t* bytes = nullptr;
  std::vector<int> cut;  // run r copies items [cut[r], cut[r + 1])
  int nworkers = 0;

  void run(int r) {
    for (int i = cut[r]; i < cut[r + 1]; ++i)
      if (bytes[i]) std::memcpy(dst[i], src[i], bytes[i]);
  }
  void worker(int id) {  // takes run id + 1
    uint64_t seen = 0;
    for (;;) {
      std::unique_lock<std::mutex> lk(m);
      wake.wait(lk, [&] { return gen != seen; });
      seen = gen;
      const bool mine = id + 1 < nrun;
      lk.unlock();
      if (mine) run(id + 1);
      lk.lock();
      if (mine && --pending == 0) done.notify_one();
    }
  }
  void ensure(int want) {
    while (nworkers < want) {
      std::thread(&CopyPool::worker, this, nworkers).detach();
      ++nworkers;
    }
  }
};

CopyPool& copy_pool() {
  static CopyPool* p = new CopyPool();  // never destroyed: its threads outlive static destruction
  return *p;
}

}  // namespace

extern "C" int gw_host_copy_batch(void* const* dst, const void* const* src, const size_t* bytes, int32_t n,
                                  int32_t threads) {
  if (n < 0 || threads < 1) return fail(GW_EINVAL, "n must be >= 0 and threads >= 1");
  if (n == 0) return GW_OK;
  if (!dst || !src || !bytes) return fail(GW_EINVAL, "null argument");
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (bytes[i] && (!dst[i] || !src[i])) return fail(GW_EINVAL, "null pointer with bytes > 0");
    total += bytes[i];
  }
  // below ~256 KB per extra thread the wake-up costs more than it saves
  const int nt = (int)std::max<size_t>(1, std::min<size_t>({(size_t)threads, (size_t)16, (size_t)n,
                                                             total / (1u << 18) + 1}));
  if (nt == 1) {
    for (int i = 0; i < n; ++i)
      if (bytes[i]) std::memcpy(dst[i], src[i], bytes[i]);
    return GW_OK;
  }
  CopyPool& P = copy_pool();
  std::lock_guard<std::mutex> call(P.call);
  {
    std::lock_guard<std::mutex> lk(P.m);
    P.ensure(nt - 1);
    P.dst = dst;
    P.src = src;
    P.bytes = bytes;
    // runs of about total / nt bytes each
    P.cut.assign(nt + 1, n);
    P.cut[0] = 0;
    size_t acc = 0;
    int r = 1;
    for (int i = 0; i < n && r < nt; ++i) {
      acc += bytes[i];
      if (acc >= total * r / nt) P.cut[r++] = i + 1;
    }
    for (; r < nt; ++r) P.cut[r] = n;
    P.nrun = nt;
    P.pending = nt - 1;
    ++P.gen;
  }
  P.wake.notify_all();
  P.run(0);
  std::unique_lock<std::mutex> lk(P.m);
  P.done.wait(lk, [&] { return P.pending == 0; });
  return GW_OK;
}

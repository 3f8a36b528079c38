// henn_serve.hip -- the serving form: a continuous-batching request loop.
//
// Requests (query vector, k, beam width, tag) are submitted on the host and
// wait in a FIFO until admission.  A request is admitted at the next tick
// when a slot is free and the device arena has room for its traversal
// state (its list of next_pow2(max(ef, k, ef_upper)) keys plus the visited
// table):
// admission is by memory.  Every tick advances every active request by at
// most steps_per_tick expansions in one launch (k_serve_step), so requests
// that arrive while others are in flight join the running batch and their
// work overlaps on the device; finished requests are retired to a host
// completion queue with their results.  Index and per-request state stay
// in HBM; only the admitted query vectors and the finished rows cross PCIe.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "henn_device.h"
#include "henn_internal.h"

namespace henn {

// Allocator of the device arena [0, size) (host bookkeeping).  A request's
// state size is one of a few values (list capacity and visited table), so
// freed blocks go to a free list per size and are reused by requests of the
// same size; new blocks come from the untouched top of the arena.  Neither
// operation scans the blocks: a lookup among the few sizes in use and a
// stack push / pop.
class ArenaAlloc {
 public:
  explicit ArenaAlloc(int64_t size) : size_(size) {}
  bool alloc(int64_t len, int64_t* off) {
    std::vector<int64_t>* fl = list_of(len);
    if (fl && !fl->empty()) {
      *off = fl->back();
      fl->pop_back();
    } else if (top_ + len <= size_) {
      *off = top_;
      top_ += len;
    } else {
      return false;
    }
    used_ += len;
    return true;
  }
  void release(int64_t off, int64_t len) {
    used_ -= len;
    std::vector<int64_t>* fl = list_of(len);
    if (!fl) {
      free_.emplace_back(len, std::vector<int64_t>());
      fl = &free_.back().second;
    }
    fl->push_back(off);
  }
  int64_t used() const { return used_; }

 private:
  std::vector<int64_t>* list_of(int64_t len) {
    for (auto& e : free_)
      if (e.first == len) return &e.second;
    return nullptr;
  }
  std::vector<std::pair<int64_t, std::vector<int64_t>>> free_;  // (block size, free blocks)
  int64_t size_, top_ = 0, used_ = 0;
};

// Requests waiting for admission, in arrival order: entries [head, size)
// of meta, with their queries at q[d * i] (one contiguous buffer, so that a
// request costs no allocation of its own).
struct PendingQueue {
  struct Meta {
    int32_t k, ef;
    int64_t tag;
  };
  std::vector<Meta> meta;
  std::vector<float> q;
  size_t head = 0;
  size_t size() const { return meta.size() - head; }
  bool empty() const { return head == meta.size(); }
  void push(const float* qv, int d, int32_t k, int32_t ef, int64_t tag) {
    meta.push_back(Meta{k, ef, tag});
    q.insert(q.end(), qv, qv + d);
  }
  void pop(int d) {
    ++head;
    if (head == meta.size()) {
      meta.clear();
      q.clear();
      head = 0;
    } else if (head > 4096 && head > meta.size() / 2) {
      meta.erase(meta.begin(), meta.begin() + head);
      q.erase(q.begin(), q.begin() + head * (size_t)d);
      head = 0;
    }
  }
};


}  // namespace henn

using namespace henn;

struct henn_server {
  const henn_index* idx = nullptr;
  int64_t idx_updates = 0;  // the index's update count at creation
  henn_server_params p{};
  hipStream_t st = nullptr;
  int d = 0, k_max = 0, ef_cap = 0, vis_bits = 0;
  LaunchShape shape{};
  // device
  float* slot_q = nullptr;
  int32_t *slot_k = nullptr, *slot_ef = nullptr, *slot_ids = nullptr, *cap = nullptr;
  float* slot_dist = nullptr;
  QState* states = nullptr;
  int64_t* state_off = nullptr;
  char* arena = nullptr;
  // done_d: two completion counters, used by alternate steps
  int32_t* done_d = nullptr;
  float* stage_q_d = nullptr;  // [2][max_slots][d], by launch parity
  // the staged queries go to the device on their own stream while the
  // previous step runs; the admission kernels wait for copy_done[parity]
  hipStream_t st_copy = nullptr;
  hipEvent_t copy_done[2] = {nullptr, nullptr};
  bool copy_pending[2] = {false, false};
  int32_t* stage_meta_d = nullptr;
  int32_t* rows_d = nullptr;  // device address of rows_h: a step writes its completion
                              // rows straight into host memory, rows_h[parity]
  // complete-graph root on matrix cores (prepared roots only): each admitted
  // request's root key, its shortlist scratch and the per-slot keys
  uint64_t* root_keys = nullptr;
  char* root_sl = nullptr;  // the admission batch's root shortlist
  uint64_t* slot_root = nullptr;
  // pinned host; the staging buffers are doubled so that a tick can stage its
  // admissions while the previous tick's step still runs
  float* stage_q_h = nullptr;     // [2][max_slots][d]
  int32_t* stage_meta_h = nullptr;  // [2][max_slots * 7]
  int32_t* done_h = nullptr;
  int32_t* rows_h = nullptr;  // [2][max_slots][1 + 2 k_max], by launch parity
  // host state
  bool inflight = false;  // a launched step whose completions are not yet retired
  int inflight_parity = 0;
  int inflight_active = 0;  // requests the launched step advanced
  // steps launched so far; its parity picks the staging buffer and the
  // completion counter of the next step (a tick with nothing active launches
  // nothing and must not flip it: the counter a step counts into is cleared
  // by the step before it)
  int64_t launches = 0;
  ArenaAlloc* alloc = nullptr;
  PendingQueue pending;
  std::vector<int32_t> free_slots;
  std::vector<int32_t> active;
  std::vector<int64_t> slot_tag, slot_off, slot_bytes;
  std::vector<int32_t> slot_kk;
  std::vector<char> slot_cancelled;  // admitted requests cancelled by henn_server_cancel
  std::vector<char> finished;        // scratch of retire_step, per slot
  // the retired step's result rows whose ids and distances are still to be
  // copied into done_vals (their tags are queued already): copied after the
  // next launch, while the device works (rows_h[payload_parity])
  std::vector<int32_t> payload_rows;
  int payload_parity = 0;
  // completed, not yet polled: tags, and per completion k_max ids then
  // k_max distance bits
  // completion queue: entries [done_head, done_tags.size()) are waiting to
  // be polled; entry i's ids and distance bits are done_vals[2 K i ..)
  std::vector<int64_t> done_tags;
  std::vector<int32_t> done_vals;
  size_t done_head = 0;
  int64_t ticks = 0, admitted = 0, completed = 0, max_active = 0, cancelled = 0;
  int64_t n_slot_cancelled = 0;  // slots marked in slot_cancelled, not yet freed
};

namespace henn {
void set_error(const std::string& msg);
}

static henn_status srv_fail(henn_status s, const std::string& m) {
  henn::set_error(m);
  return s;
}

static void srv_release(henn_server* s) {
  (void)hipFree(s->slot_q);
  (void)hipFree(s->slot_k);
  (void)hipFree(s->slot_ef);
  (void)hipFree(s->slot_ids);
  (void)hipFree(s->slot_dist);
  (void)hipFree(s->cap);
  (void)hipFree(s->states);
  (void)hipFree(s->state_off);
  (void)hipFree(s->arena);
  (void)hipFree(s->done_d);
  (void)hipFree(s->stage_q_d);
  (void)hipFree(s->stage_meta_d);
  (void)hipFree(s->root_keys);
  (void)hipFree(s->root_sl);
  (void)hipFree(s->slot_root);
  (void)hipHostFree(s->stage_q_h);
  (void)hipHostFree(s->stage_meta_h);
  (void)hipHostFree(s->done_h);
  (void)hipHostFree(s->rows_h);
  if (s->st) (void)hipStreamDestroy(s->st);
  if (s->st_copy) (void)hipStreamDestroy(s->st_copy);
  for (hipEvent_t& e : s->copy_done)
    if (e) (void)hipEventDestroy(e);
  delete s->alloc;
  delete s;
}

template <typename T>
static void dmalloc(T** p, int64_t n) {
  HENN_HIP(dev_alloc(reinterpret_cast<void**>(p), sizeof(T) * (size_t)std::max<int64_t>(n, 1)));
}
// Pinned host memory.  coherent: fine-grained memory the device writes
// straight through (no copy in its caches), so that kernel stores are what
// the host reads once the stream has completed.
template <typename T>
static void hmalloc(T** p, int64_t n, bool coherent = false) {
  const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(n, 1);
  HENN_HIP(hipHostMalloc(reinterpret_cast<void**>(p), bytes,
                         coherent ? (hipHostMallocCoherent | hipHostMallocMapped)
                                  : hipHostMallocDefault));
  // touch every page now, so that no tick pays for first-touch faults
  memset(*p, 0, bytes);
}

// List capacity of a request: its layer-0 beam max(ef, k), and the beam of
// ef_upper entries the layers above layer 0 keep in the same list.
static int request_cap(const henn_server* s, int32_t k, int32_t ef) {
  return next_pow2(std::max(std::max(std::max(ef, k), s->p.ef_upper), 1));
}

static int64_t state_bytes(const henn_server* s, int32_t k, int32_t ef) {
  const int cap = request_cap(s, k, ef);
  const int64_t b = (int64_t)cap * 8 +
                    ((int64_t)1 << s->vis_bits) * vis_tag_bytes(s->idx->n, s->vis_bits);
  return (b + 255) / 256 * 256;
}

extern "C" {

henn_status henn_default_server_params(henn_server_params* p) {
  if (!p) return srv_fail(HENN_E_INVAL, "null params");
  memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(henn_server_params);
  p->max_slots = 4096;
  p->pool_bytes = 64ll << 20;
  p->steps_per_tick = 16;
  p->k_max = 10;
  p->ef_max = 128;
  p->ef_upper = 1;
  p->rerank_factor = 4;
  return HENN_OK;
}

henn_status henn_server_create(const henn_index* idx, const henn_server_params* p,
                               henn_server** out) {
  if (!idx || !p || !out) return srv_fail(HENN_E_INVAL, "null argument");
  if (p->struct_size != sizeof(henn_server_params))
    return srv_fail(HENN_E_INVAL, "server params struct_size mismatch");
  if (p->max_slots < 1 || p->max_slots > (1 << 20)) return srv_fail(HENN_E_INVAL, "max_slots");
  if (p->steps_per_tick < 1) return srv_fail(HENN_E_INVAL, "steps_per_tick >= 1");
  if (p->k_max < 1 || p->k_max > 1024) return srv_fail(HENN_E_INVAL, "k_max in [1, 1024]");
  if (p->ef_max < 1 || p->ef_upper < 1) return srv_fail(HENN_E_INVAL, "ef_max, ef_upper >= 1");
  henn_server* s = new henn_server();
  try {
    s->idx = idx;
    s->idx_updates = idx->updates;
    s->p = *p;
    s->d = idx->d;
    s->k_max = p->k_max;
    s->ef_cap = next_pow2(std::max(std::max(p->ef_max, p->k_max), p->ef_upper));
    if (s->ef_cap > 2048) throw HipError{hipErrorInvalidValue, "beam width above 2048"};
    s->vis_bits = p->vis_bits ? p->vis_bits
                              : default_vis_bits(std::max(std::max(p->ef_max, p->k_max), p->ef_upper),
                                                 idx->n, true);
    if (s->vis_bits < 8 || s->vis_bits > 13) throw HipError{hipErrorInvalidValue, "vis_bits"};
    // launch shape: the caller's, else the autotuned one of a batched search
    // on this index with the same storage (the same beam bucket first)
    int want_lpn = p->lanes_per_vec, want_wpb = p->waves_per_block;
    {
      std::lock_guard<std::mutex> lk(const_cast<henn_index*>(idx)->tune_mu);
      const TuneEntry* pick = nullptr;
      for (const TuneEntry& te : idx->tune)
        if (te.storage == idx->storage && (!pick || te.ef_bucket == s->ef_cap)) pick = &te;
      if (pick) {
        if (!want_lpn) want_lpn = pick->lanes_per_vec;
        if (!want_wpb) want_wpb = pick->waves_per_block;
      }
    }
    int lpn = 0, cpl = 0;
    pick_lanes(idx->nchunks, want_lpn, &lpn, &cpl);
    if (!lpn) throw HipError{hipErrorInvalidValue, "lanes_per_vec"};
    s->shape.lanes_per_vec = lpn;
    s->shape.chunks_per_lane = cpl;
    s->shape.vis_bits = s->vis_bits;
    int wpb = want_wpb ? want_wpb : 4;
    while (wpb > 1 && search_lds_per_wave(s->ef_cap, s->vis_bits, vis_tag_bytes(idx->n, s->vis_bits)) * wpb > 65536) wpb /= 2;
    s->shape.waves_per_block = wpb;
    const int64_t M = p->max_slots;
    if (p->pool_bytes < state_bytes(s, p->k_max, p->ef_max))
      throw HipError{hipErrorInvalidValue, "pool_bytes below one request's state"};
    HENN_HIP(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking));
    HENN_HIP(hipStreamCreateWithFlags(&s->st_copy, hipStreamNonBlocking));
    for (hipEvent_t& e : s->copy_done)
      HENN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    dmalloc(&s->slot_q, M * s->d);
    dmalloc(&s->slot_k, M);
    dmalloc(&s->slot_ef, M);
    dmalloc(&s->cap, M);
    dmalloc(&s->states, M);
    dmalloc(&s->state_off, M);
    dmalloc(&s->arena, p->pool_bytes);
    dmalloc(&s->done_d, 2);
    HENN_HIP(hipMemset(s->done_d, 0, sizeof(int32_t) * 2));
    dmalloc(&s->stage_q_d, 2 * M * s->d);
    dmalloc(&s->stage_meta_d, M * 7);  // admission metadata [n_new][6], then the active list
    if (idx->root.size > 0) {
      dmalloc(&s->root_keys, M);
      dmalloc(&s->slot_root, M);
      dmalloc(&s->root_sl, root_shortlist_bytes(M, idx->root.kp));  // the largest admission
    }
    hmalloc(&s->stage_q_h, 2 * M * s->d);
    hmalloc(&s->stage_meta_h, 2 * M * 7);
    hmalloc(&s->done_h, 2);
    hmalloc(&s->rows_h, 2 * M * (1 + 2 * s->k_max), true);
    HENN_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&s->rows_d), s->rows_h, 0));
    s->alloc = new ArenaAlloc(p->pool_bytes);
    s->slot_tag.assign(M, 0);
    s->slot_off.assign(M, 0);
    s->slot_bytes.assign(M, 0);
    s->slot_kk.assign(M, 0);
    s->slot_cancelled.assign(M, 0);
    s->finished.assign(M, 0);
    for (int64_t i = M - 1; i >= 0; --i) s->free_slots.push_back((int32_t)i);
    *out = s;
    return HENN_OK;
  } catch (const HipError& e) {
    srv_release(s);
    henn::set_error(std::string("server create: ") + e.what + " (" + hipGetErrorString(e.e) + ")");
    return e.e == hipErrorOutOfMemory ? HENN_E_NOMEM : HENN_E_INVAL;
  } catch (const std::bad_alloc&) {
    srv_release(s);
    return srv_fail(HENN_E_NOMEM, "host allocation failed");
  }
}

henn_status henn_server_submit(henn_server* s, const float* q_host, int32_t k, int32_t ef,
                               int64_t tag) {
  if (!s || !q_host) return srv_fail(HENN_E_INVAL, "null argument");
  if (k < 1 || k > s->k_max) return srv_fail(HENN_E_INVAL, "k outside [1, k_max]");
  if (ef < 1 || std::max(ef, k) > s->ef_cap) return srv_fail(HENN_E_INVAL, "ef outside [1, ef_max]");
  try {
    s->pending.push(q_host, s->d, k, ef, tag);
  } catch (const std::bad_alloc&) {
    return srv_fail(HENN_E_NOMEM, "host allocation failed");
  }
  return HENN_OK;
}

henn_status henn_server_submit_batch(henn_server* s, const float* q_host, const int32_t* k,
                                     const int32_t* ef, const int64_t* tags, int64_t n) {
  if (!s || (n > 0 && (!q_host || !k || !ef || !tags))) return srv_fail(HENN_E_INVAL, "null argument");
  for (int64_t i = 0; i < n; ++i)
    if (k[i] < 1 || k[i] > s->k_max || ef[i] < 1 || std::max(ef[i], k[i]) > s->ef_cap)
      return srv_fail(HENN_E_INVAL, "k or ef out of range");
  try {
    s->pending.meta.reserve(s->pending.meta.size() + n);
    for (int64_t i = 0; i < n; ++i)
      s->pending.meta.push_back(PendingQueue::Meta{k[i], ef[i], tags[i]});
    s->pending.q.insert(s->pending.q.end(), q_host, q_host + n * s->d);
  } catch (const std::bad_alloc&) {
    return srv_fail(HENN_E_NOMEM, "host allocation failed");
  }
  return HENN_OK;
}

// Retires the launched step: waits for the stream, then moves its
// completions (rows the kernel wrote into host memory) to the poll queue and
// frees their slots and state bytes.
// Frees the slots of admitted requests that were cancelled (no step may be
// in flight: the device no longer touches them).
static void free_cancelled(henn_server* s) {
  if (s->n_slot_cancelled == 0) return;
  std::vector<int32_t> keep;
  keep.reserve(s->active.size());
  for (int32_t sl : s->active) {
    if (s->slot_cancelled[sl]) {
      s->slot_cancelled[sl] = 0;
      s->alloc->release(s->slot_off[sl], s->slot_bytes[sl]);
      s->free_slots.push_back(sl);
    } else {
      keep.push_back(sl);
    }
  }
  s->active.swap(keep);
  s->n_slot_cancelled = 0;
}

static void flush_payload(henn_server* s);

static void retire_step(henn_server* s) {
  flush_payload(s);  // a payload left by a tick that failed after retiring
  if (!s->inflight) {
    free_cancelled(s);
    return;
  }
  HENN_HIP(hipStreamSynchronize(s->st));
  s->inflight = false;
  const int nd = s->done_h[s->inflight_parity];
  // each request the step advanced completes at most once in it
  if (nd > s->inflight_active) throw HipError{hipErrorIllegalState, "completion count"};
  if (nd <= 0) {
    free_cancelled(s);
    return;
  }
  const int words = 1 + 2 * s->k_max;
  const int32_t* rows = s->rows_h + (int64_t)s->inflight_parity * s->p.max_slots * words;
  s->done_tags.reserve(s->done_tags.size() + nd);
  s->payload_rows.clear();
  s->payload_parity = s->inflight_parity;
  for (int i = 0; i < nd; ++i) {
    const int32_t slot = rows[(int64_t)i * words];
    if (s->slot_cancelled[slot]) {
      // cancelled after admission: no result (the slot is freed below)
      continue;
    }
    s->done_tags.push_back(s->slot_tag[slot]);
    s->payload_rows.push_back(i);
    s->alloc->release(s->slot_off[slot], s->slot_bytes[slot]);
    s->free_slots.push_back(slot);
    s->finished[slot] = 1;
    ++s->completed;
  }
  std::vector<int32_t> keep;
  keep.reserve(s->active.size());
  for (int32_t sl : s->active)
    if (!s->finished[sl]) keep.push_back(sl);
  for (int i = 0; i < nd; ++i) s->finished[rows[(int64_t)i * words]] = 0;
  s->active.swap(keep);
  free_cancelled(s);
}

// Copies the retired step's ids and distances behind their queued tags.
// Must run before the next launch with the same parity rewrites those rows
// (every tick ends with it, and poll / stats start with it).
static void flush_payload(henn_server* s) {
  if (s->payload_rows.empty()) return;
  const int words = 1 + 2 * s->k_max;
  const int32_t* rows = s->rows_h + (int64_t)s->payload_parity * s->p.max_slots * words;
  s->done_vals.reserve(s->done_vals.size() + s->payload_rows.size() * (size_t)(words - 1));
  for (int32_t i : s->payload_rows) {
    const int32_t* row = rows + (int64_t)i * words;
    s->done_vals.insert(s->done_vals.end(), row + 1, row + words);
  }
  s->payload_rows.clear();
}

henn_status henn_server_tick(henn_server* s, int32_t* n_active_out) {
  if (!s) return srv_fail(HENN_E_INVAL, "null server");
  // sizes fixed at creation (visited-table tags, root scan) follow the index
  // as it was then
  if (s->idx->updates != s->idx_updates)
    return srv_fail(HENN_E_INVAL, "the index was updated after this server was created");
  try {
    // 1) while the previous step may still run: copy the queries of the
    //    requests that could be admitted once it is retired (at most the
    //    free slots plus the requests it advances) into this step's staging
    //    buffer; those requests stay at the head of the FIFO until admitted
    const int64_t M = s->p.max_slots;
    const int c = (int)(s->launches & 1);
    float* stage_q = s->stage_q_h + (size_t)c * M * s->d;
    int32_t* stage_meta = s->stage_meta_h + (size_t)c * M * 7;
    const int64_t could_free = (int64_t)s->free_slots.size() + (s->inflight ? s->inflight_active : 0);
    const int n_stage = (int)std::min<int64_t>((int64_t)s->pending.size(), std::min(could_free, M));
    float* stage_q_dev = s->stage_q_d + (size_t)c * M * s->d;
    if (s->copy_pending[c]) {
      // this buffer's previous copy (two launches ago) has long finished
      HENN_HIP(hipEventSynchronize(s->copy_done[c]));
      s->copy_pending[c] = false;
    }
    if (n_stage > 0) {
      memcpy(stage_q, s->pending.q.data() + s->pending.head * (size_t)s->d,
             sizeof(float) * (size_t)n_stage * s->d);
      // row i of the staging buffer is the i-th request admitted below, so
      // the copy can start now, while the previous step still runs (the
      // device buffer of this parity was last read by the admission of two
      // launches ago, which precedes the step retired below)
      HENN_HIP(hipMemcpyAsync(stage_q_dev, stage_q, sizeof(float) * (size_t)n_stage * s->d,
                              hipMemcpyHostToDevice, s->st_copy));
      HENN_HIP(hipEventRecord(s->copy_done[c], s->st_copy));
      s->copy_pending[c] = true;
    }
    // 2) the previous step's completions free their slots
    retire_step(s);
    // 3) admission, FIFO, among the staged requests while a slot and arena
    //    bytes are free (row i of the staging buffer is the i-th admitted)
    int n_new = 0;
    while (n_new < n_stage && !s->free_slots.empty()) {
      const PendingQueue::Meta& r = s->pending.meta[s->pending.head];
      const int64_t need = state_bytes(s, r.k, r.ef);
      int64_t off = 0;
      if (!s->alloc->alloc(need, &off)) break;
      const int32_t slot = s->free_slots.back();
      s->free_slots.pop_back();
      int32_t* m = stage_meta + n_new * 6;
      m[0] = slot;
      m[1] = r.k;
      m[2] = r.ef;
      m[3] = request_cap(s, r.k, r.ef);
      m[4] = (int32_t)(uint32_t)((uint64_t)off & 0xffffffffu);
      m[5] = (int32_t)(uint32_t)((uint64_t)off >> 32);
      s->slot_tag[slot] = r.tag;
      s->slot_off[slot] = off;
      s->slot_bytes[slot] = need;
      s->slot_kk[slot] = r.k;
      s->active.push_back(slot);
      s->pending.pop(s->d);
      ++n_new;
      ++s->admitted;
    }
    // 4) this tick's launches
    const henn_index* idx = s->idx;
    SearchArgs a;
    memset(&a, 0, sizeof(a));
    const int eb = idx->storage == HENN_F32 ? 4 : idx->storage == HENN_BF16 ? 2 : 1;
    for (int i = 0; i < idx->num_layers; ++i) {
      const LayerDev& L = idx->L[i];
      SearchLayer& sl = a.layer[i];
      sl.vec = idx->storage == HENN_F32 ? (const void*)L.vec32 : (const void*)L.vecq;
      sl.scale = L.scale;
      sl.adj = L.adj;
      sl.adj_scale = L.adj_scale;
      sl.down = L.down;
      sl.size = (int32_t)L.size;
      sl.deg = L.deg;
      sl.row_bytes = (int64_t)idx->dpad * eb;
    }
    a.rerank_vec = idx->storage == HENN_F32 ? nullptr : idx->L[0].vec32;
    a.ids0 = idx->L[0].ids;
    a.k_all = 1;
    a.ef_all = 1;
    a.k_max = s->k_max;
    a.ef_upper = s->p.ef_upper;
    a.ef_cap = s->ef_cap;
    a.rerank_factor = std::max(1, s->p.rerank_factor);
    a.num_layers = idx->num_layers;
    a.d = idx->d;
    a.dpad = idx->dpad;
    a.nchunks = idx->nchunks;
    a.metric = idx->metric;
    a.vis_bits = s->vis_bits;
    a.vis_bytes = vis_tag_bytes(idx->n, s->vis_bits);
    a.root_complete = idx->root_complete ? 1 : 0;
    if (n_new > 0) HENN_HIP(hipStreamWaitEvent(s->st, s->copy_done[c], 0));
    // one H2D copy: the admission metadata, then the active list
    const int n_active = (int)s->active.size();
    memcpy(stage_meta + n_new * 6, s->active.data(), sizeof(int32_t) * n_active);
    if (n_new + n_active > 0)
      HENN_HIP(hipMemcpyAsync(s->stage_meta_d, stage_meta,
                              sizeof(int32_t) * (n_new * 6 + n_active), hipMemcpyHostToDevice,
                              s->st));
    if (n_new > 0) {
      if (s->slot_root) {
        // the new requests' complete-root scans, on matrix cores
        int64_t per = 0;
        const int splits = root_gram_splits(n_new, idx->root.size, &per);
        const RootShortlist sl = root_shortlist_at(s->root_sl, n_new, idx->root.kp);
        launch_root_gram(stage_q_dev, n_new, s->d, idx->root, idx->dpad, idx->metric, splits,
                         per, sl, s->st);
        SearchArgs ra = a;
        ra.Q = stage_q_dev;
        ra.nq = n_new;
        if (!launch_root_check(idx->storage, ra, sl, s->root_keys, s->st))
          return srv_fail(HENN_E_UNSUPPORTED, "no root check kernel for this shape");
      }
      launch_serve_admit(stage_q_dev, s->stage_meta_d, n_new, s->d, s->slot_q, s->slot_k,
                         s->slot_ef, s->state_off, s->cap, s->states, s->root_keys,
                         s->slot_root, s->st);
    }
    s->max_active = std::max<int64_t>(s->max_active, n_active);
    if (n_active_out) *n_active_out = n_active;
    ++s->ticks;
    if (n_active == 0) {
      flush_payload(s);
      return HENN_OK;
    }
    // one step of every active request; completions are counted in done_d[c]
    // (c = launch parity) while the kernel clears done_d[c ^ 1] for the next
    // step
    a.Q = s->slot_q;
    a.nq = s->p.max_slots;
    a.k_arr = s->slot_k;
    a.ef_arr = s->slot_ef;
    if (s->slot_root) {
      a.root_best = s->slot_root;
      a.root_splits = 1;
    }
    ServeArgs sv;
    sv.active = s->stage_meta_d + n_new * 6;
    sv.n_active = n_active;
    sv.budget = s->p.steps_per_tick;
    sv.states = s->states;
    sv.state_off = s->state_off;
    sv.cap = s->cap;
    sv.arena = s->arena;
    sv.done_count = s->done_d + c;
    sv.done_clear = s->done_d + (c ^ 1);
    sv.done_rows = s->rows_d + (int64_t)c * s->p.max_slots * (1 + 2 * s->k_max);
    if (!launch_serve_step(idx->storage, a, sv, s->shape, s->st))
      return srv_fail(HENN_E_UNSUPPORTED, "no serving kernel for this shape");
    HENN_HIP(hipGetLastError());
    // the count follows the step on the stream; the next tick (or a drain)
    // retires the step
    HENN_HIP(hipMemcpyAsync(s->done_h + c, s->done_d + c, sizeof(int32_t),
                            hipMemcpyDeviceToHost, s->st));
    s->inflight = true;
    s->inflight_parity = c;
    s->inflight_active = n_active;
    ++s->launches;
    // the previous step's ids and distances, while this step runs
    flush_payload(s);
    return HENN_OK;
  } catch (const HipError& e) {
    henn::set_error(std::string("server tick: HIP error ") + hipGetErrorString(e.e) + " in " + e.what);
    return HENN_E_DEVICE;
  } catch (const std::bad_alloc&) {
    return srv_fail(HENN_E_NOMEM, "host allocation failed");
  }
}

henn_status henn_server_poll(henn_server* s, int32_t max_results, int64_t* tags, int32_t* ids,
                             float* dist, int32_t* n_out) {
  if (!s || !n_out) return srv_fail(HENN_E_INVAL, "null argument");
  try {
    flush_payload(s);  // normally a no-op: every tick ends with it
  } catch (const std::bad_alloc&) {
    return srv_fail(HENN_E_NOMEM, "host allocation failed");
  }
  const int K = s->k_max;
  const size_t avail = s->done_tags.size() - s->done_head;
  const int n = (int)std::min<size_t>(avail, (size_t)std::max(max_results, 0));
  for (int i = 0; i < n; ++i) {
    const size_t e = s->done_head + (size_t)i;
    const int32_t* v = s->done_vals.data() + e * 2 * (size_t)K;
    if (tags) tags[i] = s->done_tags[e];
    if (ids) memcpy(ids + (int64_t)i * K, v, sizeof(int32_t) * K);
    if (dist) memcpy(dist + (int64_t)i * K, v + K, sizeof(float) * K);
  }
  s->done_head += (size_t)n;
  if (s->done_head == s->done_tags.size()) {
    s->done_tags.clear();
    s->done_vals.clear();
    s->done_head = 0;
  } else if (s->done_head > s->done_tags.size() / 2) {
    // drop the polled half so the queue does not grow without bound
    s->done_tags.erase(s->done_tags.begin(), s->done_tags.begin() + s->done_head);
    s->done_vals.erase(s->done_vals.begin(), s->done_vals.begin() + s->done_head * 2 * K);
    s->done_head = 0;
  }
  *n_out = n;
  return HENN_OK;
}

henn_status henn_server_cancel(henn_server* s, int64_t tag, int32_t* state) {
  if (!s) return srv_fail(HENN_E_INVAL, "null server");
  int32_t st = 0;
  // waiting for admission: remove it from the FIFO
  for (size_t i = s->pending.head; i < s->pending.meta.size(); ++i) {
    if (s->pending.meta[i].tag != tag) continue;
    s->pending.meta.erase(s->pending.meta.begin() + i);
    s->pending.q.erase(s->pending.q.begin() + i * (size_t)s->d,
                       s->pending.q.begin() + (i + 1) * (size_t)s->d);
    if (s->pending.head == s->pending.meta.size()) {
      s->pending.meta.clear();
      s->pending.q.clear();
      s->pending.head = 0;
    }
    st = 1;
    break;
  }
  // admitted and not finished (as far as the host knows): no result
  if (st == 0) {
    for (int32_t sl : s->active) {
      if (s->slot_tag[sl] == tag && !s->slot_cancelled[sl]) {
        s->slot_cancelled[sl] = 1;
        ++s->n_slot_cancelled;
        st = 2;
        break;
      }
    }
  }
  // finished, waiting to be polled
  if (st == 0) {
    for (size_t i = s->done_head; i < s->done_tags.size(); ++i)
      if (s->done_tags[i] == tag) {
        st = 3;
        break;
      }
  }
  if (st == 1 || st == 2) ++s->cancelled;
  if (state) *state = st;
  return HENN_OK;
}

henn_status henn_server_stats(const henn_server* s, henn_server_stats_t* out) {
  if (!s || !out) return srv_fail(HENN_E_INVAL, "null argument");
  out->pending = (int64_t)s->pending.size();
  out->active = (int64_t)s->active.size();
  out->completed = s->completed;
  out->admitted = s->admitted;
  out->ticks = s->ticks;
  out->pool_bytes_used = s->alloc->used();
  out->max_active = s->max_active;
  out->done_queued = (int64_t)(s->done_tags.size() - s->done_head);
  out->cancelled = s->cancelled;
  return HENN_OK;
}

void henn_server_destroy(henn_server* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  if (s->st_copy) (void)hipStreamSynchronize(s->st_copy);
  srv_release(s);
}

}  // extern "C"

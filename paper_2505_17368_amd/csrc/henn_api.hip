// henn_api.hip -- host runtime behind the C ABI of include/henn.h.
//
// henn_build runs Alg. 1 (BuildHENN): for i = 1, 2, ... it draws
// ceil(|L_{i-1}| / 2^m) samples with replacement from L_{i-1} (Alg. 2,
// Cor. "layer-size"), takes eps_i from Eq. (1) (natural log), and accepts the
// first attempt whose sample hits every one of r sampled ring ranges (the
// practical IsEpsNet of App. B.1 / App. G.2; rings are minimal heavy rings:
// a uniform centre in L_{i-1} and a uniform rank window of floor(eps*s)+1
// points).  The decision is taken on the host after each attempt.  Each
// layer then gets its exact kNN graph (App. B.2) and, for the precision
// forms, a BF16 / FP8 traversal copy.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "henn_device.h"
#include "henn_internal.h"

namespace henn {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static henn_status fail(henn_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

// Allocation-failure injector (henn_testing.h): < 0 off; otherwise the
// number of device allocations that may still succeed.
static std::atomic<int64_t> g_alloc_budget{-1};

static bool alloc_allowed() {
  int64_t b = g_alloc_budget.load();
  while (b >= 0) {
    if (b == 0) return false;
    if (g_alloc_budget.compare_exchange_weak(b, b - 1)) return true;
  }
  return true;
}

}  // namespace henn

extern "C" henn_status henn_testing_fail_alloc_after(int64_t n) {
  henn::g_alloc_budget.store(n < 0 ? -1 : n);
  return HENN_OK;
}

namespace henn {

hipError_t dev_alloc(void** p, size_t bytes) {
  if (!alloc_allowed()) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}

hipError_t dev_alloc_async(void** p, size_t bytes, hipStream_t st) {
  if (!alloc_allowed()) return hipErrorOutOfMemory;
  return hipMallocAsync(p, bytes, st);
}

static henn_status from_hip(const HipError& e) {
  set_error(std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what);
  if (e.e == hipErrorOutOfMemory || e.e == hipErrorMemoryAllocation) return HENN_E_NOMEM;
  if (e.e == hipErrorNotSupported) return HENN_E_UNSUPPORTED;
  return HENN_E_DEVICE;
}

static void free_layer(LayerDev& L) {
  (void)hipFree(L.vec32);
  (void)hipFree(L.vecq);
  (void)hipFree(L.scale);
  (void)hipFree(L.adj_scale);
  (void)hipFree(L.adj);
  (void)hipFree(L.ids);
  (void)hipFree(L.down);
  L = LayerDev{};
}

template <typename T>
static T* dalloc(int64_t count) {
  T* p = nullptr;
  if (count <= 0) count = 1;
  HENN_HIP(dev_alloc(reinterpret_cast<void**>(&p), sizeof(T) * (size_t)count));
  return p;
}

static int storage_bytes(int storage) {
  return storage == HENN_F32 ? 4 : storage == HENN_BF16 ? 2 : 1;
}

// Attempt cap of Alg. 2's repeat loop: max_attempts, or with 0 the smallest
// t with phi^t <= 1e-9 (each attempt fails with probability phi).
static int attempt_cap(const henn_build_params& p) {
  if (p.max_attempts > 0) return p.max_attempts;
  return std::max(1, (int)ceil(log(1e-9) / log(p.phi)));
}

static bool valid_build_params(const henn_build_params* p, std::string* why) {
  if (!p) { *why = "null build params"; return false; }
  if (p->struct_size != sizeof(henn_build_params)) { *why = "build params struct_size mismatch"; return false; }
  if (p->metric != HENN_L2 && p->metric != HENN_IP) { *why = "metric"; return false; }
  if (p->m < 1 || p->m > 30) { *why = "m must be in [1, 30]"; return false; }
  if (!(p->c0 > 0.0)) { *why = "c0 must be positive"; return false; }
  if (p->num_rings < 1 || p->num_rings > 4096) { *why = "num_rings in [1, 4096]"; return false; }
  if (p->max_attempts < 0) { *why = "max_attempts >= 0"; return false; }
  if (p->gram != 0 && p->gram != 1) {
    *why = "gram must be 0 (split BF16) or 1 (FP32)";
    return false;
  }
  if (p->max_attempts == 0 && !(p->phi > 0.0 && p->phi < 1.0)) {
    *why = "max_attempts = 0 needs phi in (0, 1)";
    return false;
  }
  if (p->degree < 1 || p->degree > 32) { *why = "degree in [1, 32]"; return false; }
  if (p->graph < HENN_GRAPH_KNN || p->graph > HENN_GRAPH_NSW) { *why = "graph"; return false; }
  const bool sym = p->graph == HENN_GRAPH_KNN_SYM || p->graph == HENN_GRAPH_PRUNED_SYM ||
                   p->graph == HENN_GRAPH_NSW;
  if (sym && (p->max_degree < p->degree || p->max_degree > 64)) {
    *why = "max_degree in [degree, 64]"; return false;
  }
  if (p->storage < HENN_F32 || p->storage > HENN_FP8_E4M3) { *why = "storage"; return false; }
  if (p->root_complete_max < 0) { *why = "root_complete_max >= 0"; return false; }
  if (p->sampler != HENN_SAMPLER_DRAWS && p->sampler != HENN_SAMPLER_HALVING) {
    *why = "sampler"; return false;
  }
  if (p->graph == HENN_GRAPH_NSW) {
    if (p->ef_construction < 1 || p->ef_construction > 2048) {
      *why = "ef_construction in [1, 2048]"; return false;
    }
    if (p->insert_shift < 0 || p->insert_shift > 62) { *why = "insert_shift in [0, 62]"; return false; }
  }
  return true;
}

// ---- NSW graphs (App. B.2) ---------------------------------------------------
// Batched incremental insertion: the layer's members join in ascending id
// order, in batches [lo, lo + max(1, lo >> insert_shift)).  The searches of
// a batch are the library's own beam search (one FP32 layer: the graph on
// [0, lo), entry position 0, beam max(ef_construction, R), top R), then
// nsw_merge_batch writes the new rows and merges the reverse edges.
struct NswWork {
  int32_t* res = nullptr;
  float* dist = nullptr;
  uint32_t* cnt = nullptr;
  uint32_t* off = nullptr;
  int32_t* inl = nullptr;
  NswWork(int64_t s, int64_t nb_max, int R) {
    try {
      res = dalloc<int32_t>(nb_max * R);
      dist = dalloc<float>(nb_max * R);
      cnt = dalloc<uint32_t>(s + 1);
      off = dalloc<uint32_t>(s + 1);
      inl = dalloc<int32_t>(nb_max * R);
    } catch (...) {
      release();
      throw;
    }
  }
  ~NswWork() { release(); }
  void release() {
    (void)hipFree(res);
    (void)hipFree(dist);
    (void)hipFree(cnt);
    (void)hipFree(off);
    (void)hipFree(inl);
    res = nullptr;
    dist = nullptr;
    cnt = off = nullptr;
    inl = nullptr;
  }
};

static int64_t nsw_batch_end(int64_t lo, int64_t s, int shift) {
  return std::min(s, lo + std::max<int64_t>(1, lo >> shift));
}

// vec: FP32 rows [>= hi][dpad]; adj: [>= hi][M], rows < lo hold the graph.
static void nsw_insert_batch(int device, const float* vec, int dpad, int nchunks, int metric,
                             int32_t* adj, int M, int64_t lo, int64_t hi, int R, int ef,
                             const NswWork& w, hipStream_t st) {
  const int64_t nb = hi - lo;
  if (nb <= 0) return;
  if (lo == 0) {
    HENN_HIP(hipMemsetAsync(w.res, 0xFF, sizeof(int32_t) * nb * R, st));  // no graph yet
  } else {
    henn_index g;  // a one-layer view of the graph on [0, lo); owns nothing
    g.n = lo;
    g.d = dpad;
    g.dpad = dpad;
    g.nchunks = nchunks;
    g.metric = metric;
    g.storage = HENN_F32;
    g.num_layers = 1;
    g.device = device;
    g.L[0].size = lo;
    g.L[0].deg = M;
    g.L[0].vec32 = const_cast<float*>(vec);
    g.L[0].adj = adj;
    henn_search_params sp;
    henn_default_search_params(&sp);
    sp.k_all = R;
    sp.k_max = R;
    sp.ef_all = std::max(ef, R);
    if (henn_search_batch(&g, vec + lo * dpad, nb, &sp, w.res, w.dist, st) != HENN_OK)
      throw HipError{hipErrorInvalidValue, "NSW insertion search"};
  }
  int lpn, cpl;
  pick_lanes(nchunks, 0, &lpn, &cpl);
  nsw_merge_batch(vec, dpad, nchunks, metric, w.res, lo, nb, R, adj, M, w.cnt, w.off, w.inl, lpn,
                  cpl, st);
}

static int32_t* nsw_graph(henn_index* ix, const float* vec, int64_t s, hipStream_t st) {
  const henn_build_params& p = ix->params;
  const int M = p.max_degree, R = p.degree;
  int32_t* adj = dalloc<int32_t>(s * M);
  try {
    HENN_HIP(hipMemsetAsync(adj, 0xFF, sizeof(int32_t) * s * M, st));
    const NswWork w(s, std::max<int64_t>(1, s >> p.insert_shift), R);
    for (int64_t lo = 0; lo < s;) {
      const int64_t hi = nsw_batch_end(lo, s, p.insert_shift);
      nsw_insert_batch(ix->device, vec, ix->dpad, ix->nchunks, ix->metric, adj, M, lo, hi, R,
                       p.ef_construction, w, st);
      lo = hi;
    }
    HENN_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipFree(adj);
    throw;
  }
  return adj;
}

static int sample_layer(henn_index* ix, int i, hipStream_t st, int32_t* local_out,
                        int64_t* count_out);

// Alg. 1's layer loop from layer `first` on (layers below it exist): samples
// each layer from the one below until the stopping rule; graphs are built by
// the caller.  Returns true when some layer kept an unverified attempt.
static bool sample_layers_from(henn_index* ix, int first, hipStream_t st) {
  const henn_build_params& p = ix->params;
  bool unverified = false;
  ix->num_layers = first;
  for (int i = first; i < HENN_MAX_LAYERS; ++i) {
    const int64_t s = ix->L[i - 1].size;
    const int64_t D = (s + (1ll << p.m) - 1) >> p.m;
    if (D < (int64_t)p.degree + 1) break;
    if (p.max_layers >= 0 && i > p.max_layers) break;
    if (p.root_complete_max > 0 && s <= p.root_complete_max) break;
    int32_t* local = dalloc<int32_t>(s);
    try {
      int64_t cnt = 0;
      sample_layer(ix, i, st, local, &cnt);
      LayerDev& L = ix->L[i];
      L.size = cnt;
      L.info.size = cnt;
      L.ids = dalloc<int32_t>(cnt);
      L.down = dalloc<int32_t>(cnt);
      launch_map_ids(ix->L[i - 1].ids, local, cnt, L.ids, L.down, st);
      L.vec32 = dalloc<float>(cnt * ix->dpad);
      launch_copy_rows(ix->L[i - 1].vec32, ix->dpad, local, cnt, ix->dpad, L.vec32, ix->dpad,
                       st);
      HENN_HIP(hipStreamSynchronize(st));
    } catch (...) {
      (void)hipFree(local);
      throw;
    }
    (void)hipFree(local);
    ix->num_layers = i + 1;
    if (ix->L[i].info.status == 3) unverified = true;
  }
  return unverified;
}

// ---- insertion into a built NSW index (App. C "Dynamic Setting") --------------
// Layer i takes the new points g of layer i - 1 whose coin u(word g of stream
// (tag 5, layer i, attempt 0), 2^m) is 0, i.e. with probability 2^-m, as the
// random layers are maintained under insertion.  New points have the largest
// ids, so they are appended to every member list in order; each layer graph
// then takes them by NSW insertion, continuing the build's batch schedule.
static constexpr uint32_t kTagInsert = 5;

static void replace(float*& p, float* q) { (void)hipFree(p); p = q; }
static void replace(int32_t*& p, int32_t* q) { (void)hipFree(p); p = q; }

// The precision-form copy of a whole layer again (after its rows changed).
static void refresh_forms(henn_index* ix, LayerDev& L, hipStream_t st) {
  if (ix->storage == HENN_F32) return;
  (void)hipFree(L.vecq);
  (void)hipFree(L.scale);
  (void)hipFree(L.adj_scale);
  L.vecq = nullptr;
  L.scale = L.adj_scale = nullptr;
  L.vecq = dalloc<uint8_t>(L.size * ix->dpad * storage_bytes(ix->storage));
  if (ix->storage == HENN_FP8_E4M3) L.scale = dalloc<float>(L.size);
  launch_quantize(ix->storage, L.vec32, L.size, ix->dpad, L.vecq, L.scale, st);
  if (ix->storage == HENN_FP8_E4M3) {
    L.adj_scale = dalloc<float>(L.size * L.deg);
    launch_adj_scale(L.adj, L.size * L.deg, L.scale, L.adj_scale, st);
  }
  HENN_HIP(hipStreamSynchronize(st));
}

static void prepare_root(henn_index* ix, hipStream_t st);

// The complete root's scan data again (after the root layer changed).
static void refresh_root(henn_index* ix, hipStream_t st) {
  RootAux& r = ix->root;
  if (r.dec_owned) (void)hipFree(r.dec);
  (void)hipFree(r.mean);
  (void)hipFree(r.norm);
  (void)hipFree(r.rowb);
  (void)hipFree(r.normp);
  r = RootAux{};
  prepare_root(ix, st);
  HENN_HIP(hipStreamSynchronize(st));
}

// Grows layer i by the points new_ids (ascending, all above the old ids);
// new_local: their rows in X_new; new_down: their positions one layer below.
static void grow_layer(henn_index* ix, int i, const float* X_new,
                       const std::vector<int32_t>& new_ids, const std::vector<int32_t>& new_local,
                       const std::vector<int32_t>& new_down, hipStream_t st) {
  LayerDev& L = ix->L[i];
  const int64_t s = L.size, c = (int64_t)new_ids.size(), t = s + c;
  const int M = L.deg, dpad = ix->dpad;
  const henn_build_params& p = ix->params;
  int32_t* local_d = dalloc<int32_t>(c);
  float* vec = nullptr;
  int32_t *adj = nullptr, *ids = nullptr, *down = nullptr;
  try {
    HENN_HIP(hipMemcpyAsync(local_d, new_local.data(), sizeof(int32_t) * c,
                            hipMemcpyHostToDevice, st));
    vec = dalloc<float>(t * dpad);
    HENN_HIP(hipMemcpyAsync(vec, L.vec32, sizeof(float) * s * dpad, hipMemcpyDeviceToDevice, st));
    launch_copy_rows(X_new, ix->d, local_d, c, ix->d, vec + s * dpad, dpad, st);
    adj = dalloc<int32_t>(t * M);
    HENN_HIP(hipMemcpyAsync(adj, L.adj, sizeof(int32_t) * s * M, hipMemcpyDeviceToDevice, st));
    HENN_HIP(hipMemsetAsync(adj + s * M, 0xFF, sizeof(int32_t) * c * M, st));
    if (L.ids) {  // upper layers, and layer 0 once deletions gave it an id list
      ids = dalloc<int32_t>(t);
      HENN_HIP(hipMemcpyAsync(ids, L.ids, sizeof(int32_t) * s, hipMemcpyDeviceToDevice, st));
      HENN_HIP(hipMemcpyAsync(ids + s, new_ids.data(), sizeof(int32_t) * c,
                              hipMemcpyHostToDevice, st));
    }
    if (i > 0) {
      down = dalloc<int32_t>(t);
      HENN_HIP(hipMemcpyAsync(down, L.down, sizeof(int32_t) * s, hipMemcpyDeviceToDevice, st));
      HENN_HIP(hipMemcpyAsync(down + s, new_down.data(), sizeof(int32_t) * c,
                              hipMemcpyHostToDevice, st));
    }
    const NswWork w(t, std::max<int64_t>(1, t >> p.insert_shift), p.degree);
    for (int64_t lo = s; lo < t;) {
      const int64_t hi = nsw_batch_end(lo, t, p.insert_shift);
      nsw_insert_batch(ix->device, vec, dpad, ix->nchunks, ix->metric, adj, M, lo, hi, p.degree,
                       p.ef_construction, w, st);
      lo = hi;
    }
    HENN_HIP(hipStreamSynchronize(st));
  } catch (...) {
    (void)hipFree(local_d);
    (void)hipFree(vec);
    (void)hipFree(adj);
    (void)hipFree(ids);
    (void)hipFree(down);
    throw;
  }
  (void)hipFree(local_d);
  replace(L.vec32, vec);
  replace(L.adj, adj);
  if (ids) replace(L.ids, ids);
  if (down) replace(L.down, down);
  L.size = t;
  L.info.size = t;
  refresh_forms(ix, L, st);
}

// Finishes a layer: graph (+ optional symmetrisation) and traversal copy.
static void finish_layer(henn_index* ix, int i, hipStream_t st) {
  LayerDev& L = ix->L[i];
  const henn_build_params& p = ix->params;
  int lpn, cpl;
  pick_lanes(ix->nchunks, 0, &lpn, &cpl);
  if (p.graph == HENN_GRAPH_NSW) {
    L.adj = nsw_graph(ix, L.vec32, L.size, st);
    L.deg = p.max_degree;
  } else {
    const bool pruned = p.graph == HENN_GRAPH_PRUNED || p.graph == HENN_GRAPH_PRUNED_SYM;
    const int R = p.degree;
    // the pruned graphs scan the exact top min(2R, 32) candidates
    const int C = pruned ? std::min(2 * R, 32) : R;
    int32_t* adj = dalloc<int32_t>(L.size * R);
    int32_t* cand = pruned ? dalloc<int32_t>(L.size * C) : adj;
    try {
      L.info.fallback_rows =
          (int32_t)build_knn_graph(L.vec32, L.size, ix->dpad, ix->nchunks, ix->metric, C, lpn, cpl,
                                   cand, p.gram, st);
      if (pruned) {
        prune_graph(L.vec32, L.size, ix->dpad, ix->nchunks, ix->metric, cand, C, R, adj, lpn, cpl,
                    st);
        HENN_HIP(hipStreamSynchronize(st));
        (void)hipFree(cand);
        cand = adj;
      }
    } catch (...) {
      if (cand != adj) (void)hipFree(cand);
      (void)hipFree(adj);
      throw;
    }
    if (p.graph == HENN_GRAPH_KNN_SYM || p.graph == HENN_GRAPH_PRUNED_SYM) {
      int32_t* adj2 = dalloc<int32_t>(L.size * p.max_degree);
      try {
        symmetrize_graph(L.vec32, L.size, ix->dpad, ix->nchunks, ix->metric, adj, R, adj2,
                         p.max_degree, lpn, cpl, st);
      } catch (...) {
        (void)hipFree(adj);
        (void)hipFree(adj2);
        throw;
      }
      (void)hipFree(adj);
      L.adj = adj2;
      L.deg = p.max_degree;
    } else {
      L.adj = adj;
      L.deg = R;
    }
  }
  L.info.degree = L.deg;
  if (ix->storage != HENN_F32) {
    L.vecq = dalloc<uint8_t>(L.size * ix->dpad * storage_bytes(ix->storage));
    if (ix->storage == HENN_FP8_E4M3) L.scale = dalloc<float>(L.size);
    launch_quantize(ix->storage, L.vec32, L.size, ix->dpad, L.vecq, L.scale, st);
    if (ix->storage == HENN_FP8_E4M3) {
      L.adj_scale = dalloc<float>(L.size * L.deg);
      launch_adj_scale(L.adj, L.size * L.deg, L.scale, L.adj_scale, st);
    }
  }
  HENN_HIP(hipStreamSynchronize(st));
}

// One eps-net layer (Alg. 2's draws or Alg. 3's halving, then the ring
// check).  Returns the accepted attempt and fills info.
static int sample_layer(henn_index* ix, int i, hipStream_t st, int32_t* local_out,
                        int64_t* count_out) {
  const henn_build_params& p = ix->params;
  LayerDev& prev = ix->L[i - 1];
  const int64_t s = prev.size;
  const int64_t D = (s + (1ll << p.m) - 1) >> p.m;
  const double eps = p.eps_override > 0.0
                         ? p.eps_override
                         : p.c0 * (double)ix->d * log((double)s) / (double)s * (double)(1ll << p.m);
  const int64_t w = (int64_t)floor(eps * (double)s) + 1;
  henn_layer_info& info = ix->L[i].info;
  info.draws = D;
  info.eps = eps;
  info.window = w;
  const bool halving = p.sampler == HENN_SAMPLER_HALVING;
  int lpn, cpl;
  pick_lanes(ix->nchunks, 0, &lpn, &cpl);
  int accepted = 0;
  if (halving) {
    // the halved sample is distinct and ascending already: written in place
    *count_out = launch_halve(p.seed, i, 0, s, p.m, local_out, st);
  }
  if (w > s) {
    info.status = 1;  // vacuous: no ring can be heavy
    info.attempts = 1;
    info.hits = 0;
  } else {
    const int r = p.num_rings;
    std::vector<int32_t> centres((size_t)r);
    std::vector<int64_t> ranks((size_t)(2 * r));
    for (int j = 0; j < r; ++j) {
      centres[(size_t)j] = (int32_t)uniform_index(stream_word(p.seed, kTagRingCentre, i, 0, j),
                                                  (uint64_t)s);
      const int64_t a = (int64_t)uniform_index(stream_word(p.seed, kTagRingStart, i, 0, j),
                                               (uint64_t)(s - w + 1));
      ranks[(size_t)(2 * j)] = a;
      ranks[(size_t)(2 * j + 1)] = a + w - 1;
    }
    int32_t* d_centres = dalloc<int32_t>(r);
    uint64_t* keys = nullptr;
    uint64_t* d_lohi = dalloc<uint64_t>(2 * r);
    uint32_t* d_hits = dalloc<uint32_t>(r);
    try {
      keys = dalloc<uint64_t>((int64_t)r * s);
      HENN_HIP(hipMemcpyAsync(d_centres, centres.data(), sizeof(int32_t) * r,
                              hipMemcpyHostToDevice, st));
      launch_ring_keys(lpn, cpl, prev.vec32, ix->dpad, ix->nchunks, ix->metric, s, d_centres, r,
                       keys, st);
      std::vector<uint64_t> ends((size_t)(2 * r));
      launch_radix_select(keys, s, r, ranks.data(), ends.data(), st);
      (void)hipFree(keys);
      keys = nullptr;
      std::vector<uint64_t> lohi((size_t)(2 * r));
      for (int j = 0; j < r; ++j) {
        lohi[(size_t)j] = ends[(size_t)(2 * j)];
        lohi[(size_t)(r + j)] = ends[(size_t)(2 * j + 1)];
      }
      HENN_HIP(hipMemcpyAsync(d_lohi, lohi.data(), sizeof(uint64_t) * 2 * r,
                              hipMemcpyHostToDevice, st));
      int best_t = -1, best_hits = -1;
      std::vector<uint32_t> hits((size_t)r);
      const int cap = attempt_cap(p);
      int t = 0;
      for (; t < cap; ++t) {
        HENN_HIP(hipMemsetAsync(d_hits, 0, sizeof(uint32_t) * r, st));
        if (halving && t > 0) launch_halve(p.seed, i, t, s, p.m, local_out, st);
        launch_ring_hits(lpn, cpl, prev.vec32, ix->dpad, ix->nchunks, ix->metric, s, p.seed, i,
                         t, D, halving ? local_out : nullptr, d_centres, d_lohi, d_lohi + r, r,
                         d_hits, st);
        HENN_HIP(hipMemcpyAsync(hits.data(), d_hits, sizeof(uint32_t) * r, hipMemcpyDeviceToHost,
                                st));
        HENN_HIP(hipStreamSynchronize(st));
        int h = 0;
        for (int j = 0; j < r; ++j) h += hits[(size_t)j] != 0;
        if (h > best_hits) {
          best_hits = h;
          best_t = t;
        }
        if (h == r) break;
      }
      if (best_hits == r) {
        info.status = 2;
        info.attempts = t + 1;
      } else {
        info.status = 3;
        info.attempts = cap;
      }
      info.hits = best_hits;
      accepted = best_t;
    } catch (...) {
      (void)hipFree(keys);
      (void)hipFree(d_centres);
      (void)hipFree(d_lohi);
      (void)hipFree(d_hits);
      throw;
    }
    (void)hipFree(d_centres);
    (void)hipFree(d_lohi);
    (void)hipFree(d_hits);
  }
  if (halving) {
    // local_out holds the last attempt made; redo the kept one if it differs
    if (accepted != info.attempts - 1) launch_halve(p.seed, i, accepted, s, p.m, local_out, st);
    return accepted;
  }
  const int64_t nwords = (s + 31) / 32;
  uint32_t* bitmap = dalloc<uint32_t>(nwords);
  try {
    HENN_HIP(hipMemsetAsync(bitmap, 0, sizeof(uint32_t) * nwords, st));
    launch_draw_mark(p.seed, i, accepted, s, D, bitmap, st);
    *count_out = compact_bitmap(bitmap, s, local_out, st);
  } catch (...) {
    (void)hipFree(bitmap);
    throw;
  }
  (void)hipFree(bitmap);
  return accepted;
}

static void destroy(henn_index* ix) {
  if (!ix) return;
  for (int i = 0; i < HENN_MAX_LAYERS; ++i) free_layer(ix->L[i]);
  if (ix->root.dec_owned) (void)hipFree(ix->root.dec);
  (void)hipFree(ix->root.mean);
  (void)hipFree(ix->root.norm);
  (void)hipFree(ix->root.rowb);
  (void)hipFree(ix->root.normp);
  delete ix;
}

// Prepares a complete-graph root for the MFMA scan (RootAux): FP32 rows of
// the stored values, their mean (L2), norms and the bounds the exact check
// needs.  Roots wider than 128 coordinates keep the canonical scans only.
static void prepare_root(henn_index* ix, hipStream_t st) {
  if (!ix->root_complete || ix->dpad > 128) return;
  const LayerDev& R = ix->L[ix->num_layers - 1];
  RootAux& r = ix->root;
  r.size = R.size;
  if (ix->storage == HENN_F32) {
    r.dec = R.vec32;
  } else {
    r.dec = dalloc<float>(R.size * ix->dpad);
    r.dec_owned = true;
    launch_decode_rows(ix->storage, R.vecq, R.scale, R.size, ix->dpad, r.dec, st);
  }
  if (ix->metric == HENN_L2) {
    r.mean = dalloc<float>(ix->dpad);
    layer_mean(r.dec, R.size, ix->dpad, r.mean, st);
    std::vector<float> m((size_t)ix->dpad);
    HENN_HIP(hipMemcpyAsync(m.data(), r.mean, sizeof(float) * ix->dpad, hipMemcpyDeviceToHost,
                            st));
    HENN_HIP(hipStreamSynchronize(st));
    double s2 = 0.0;
    for (float v : m) s2 += (double)v * v;
    r.mean_n2 = (float)s2;
  }
  r.norm = dalloc<float>(R.size);
  launch_row_norms(r.dec, r.mean, R.size, ix->dpad, r.norm, st);
  r.nmax = max_norm(r.norm, R.size, st);
  prepare_root_bf16(r, ix->dpad, ix->metric, st);
}

static henn_index* new_index(const float* X, int64_t n, int32_t d, const henn_build_params* p,
                             hipStream_t st) {
  henn_index* ix = new henn_index();
  ix->n = n;
  ix->next_id = n;
  ix->d = d;
  ix->dpad = (d + 7) / 8 * 8;
  ix->nchunks = ix->dpad / 8;
  ix->metric = p->metric;
  ix->storage = p->storage;
  ix->params = *p;
  (void)hipGetDevice(&ix->device);
  try {
    LayerDev& L0 = ix->L[0];
    L0.size = n;
    L0.vec32 = dalloc<float>(n * ix->dpad);
    launch_copy_rows(X, d, nullptr, n, d, L0.vec32, ix->dpad, st);
    HENN_HIP(hipGetLastError());
    L0.info.size = n;
    L0.info.draws = n;
    L0.info.status = 0;
    ix->num_layers = 1;
  } catch (...) {
    destroy(ix);
    throw;
  }
  return ix;
}

static henn_status check_common(const float* X, int64_t n, int32_t d, henn_index** out) {
  if (!X) return fail(HENN_E_INVAL, "X is null");
  if (!out) return fail(HENN_E_INVAL, "out is null");
  if (n < 1 || n > 2147483647ll) return fail(HENN_E_INVAL, "n must be in [1, 2^31-1]");
  if (d < 1 || d > 1024) return fail(HENN_E_INVAL, "d must be in [1, 1024]");
  return HENN_OK;
}

}  // namespace henn

using namespace henn;

extern "C" {

const char* henn_last_error(void) { return g_last_error.c_str(); }

henn_status henn_default_build_params(henn_build_params* p) {
  if (!p) return fail(HENN_E_INVAL, "null params");
  memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(henn_build_params);
  p->metric = HENN_L2;
  p->max_layers = -1;
  p->m = 4;
  p->c0 = 1.0;
  p->eps_override = 0.0;
  p->num_rings = 64;
  p->max_attempts = 64;
  p->degree = 16;
  p->max_degree = 32;
  p->graph = HENN_GRAPH_KNN;
  p->storage = HENN_F32;
  p->seed = 0;
  p->sampler = HENN_SAMPLER_DRAWS;
  p->ef_construction = 256;
  p->phi = 0.5;
  p->insert_shift = 3;
  return HENN_OK;
}

henn_status henn_default_search_params(henn_search_params* p) {
  if (!p) return fail(HENN_E_INVAL, "null params");
  memset(p, 0, sizeof(*p));
  p->struct_size = sizeof(henn_search_params);
  p->k_all = 10;
  p->ef_all = 32;
  p->k_max = 10;
  p->ef_max = 32;
  p->ef_upper = 1;
  p->rerank_factor = 4;
  return HENN_OK;
}

henn_status henn_build(const float* X, int64_t n, int32_t d, const henn_build_params* p,
                       void* hip_stream, henn_index** out) {
  henn_status cs = check_common(X, n, d, out);
  if (cs != HENN_OK) return cs;
  std::string why;
  if (!valid_build_params(p, &why)) return fail(HENN_E_INVAL, why);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  henn_index* ix = nullptr;
  try {
    ix = new_index(X, n, d, p, st);
    const bool unverified = sample_layers_from(ix, 1, st);
    ix->root_complete = p->root_complete_max > 0 && ix->num_layers >= 2;
    for (int i = 0; i < ix->num_layers; ++i) finish_layer(ix, i, st);
    prepare_root(ix, st);
    *out = ix;
    return unverified ? fail(HENN_W_NOT_VERIFIED, "a layer kept its best unverified attempt")
                      : HENN_OK;
  } catch (const HipError& e) {
    destroy(ix);
    return from_hip(e);
  } catch (const std::bad_alloc&) {
    destroy(ix);
    return fail(HENN_E_NOMEM, "host allocation failed");
  }
}

henn_status henn_import(const float* X, int64_t n, int32_t d, const henn_build_params* p,
                        int32_t num_layers, const int64_t* sizes, const int32_t* const* ids_host,
                        const int32_t* const* adj_host, int32_t adj_stride, void* hip_stream,
                        henn_index** out) {
  henn_status cs = check_common(X, n, d, out);
  if (cs != HENN_OK) return cs;
  std::string why;
  if (!valid_build_params(p, &why)) return fail(HENN_E_INVAL, why);
  if (num_layers < 1 || num_layers > HENN_MAX_LAYERS) return fail(HENN_E_INVAL, "num_layers");
  if (!sizes || !adj_host || !ids_host) return fail(HENN_E_INVAL, "null layer arrays");
  if (adj_stride < 1 || adj_stride > 64) return fail(HENN_E_INVAL, "adj_stride in [1, 64]");
  if (sizes[0] != n) return fail(HENN_E_INVAL, "sizes[0] must equal n");
  // host-side validation: ascending ids, nesting, adjacency range, no duplicates
  std::vector<std::vector<int32_t>> down((size_t)num_layers);
  for (int i = 0; i < num_layers; ++i) {
    const int64_t sz = sizes[i];
    if (sz < 1 || (i > 0 && sz > sizes[i - 1])) return fail(HENN_E_INVAL, "layer sizes");
    if (i > 0 || ids_host[0]) {
      const int32_t* ids = ids_host[i];
      if (!ids) return fail(HENN_E_INVAL, "null ids for an upper layer");
      for (int64_t j = 0; j < sz; ++j) {
        if (ids[j] < 0 || ids[j] >= n || (j > 0 && ids[j] <= ids[j - 1]))
          return fail(HENN_E_INVAL, "layer ids must be ascending point ids");
      }
    }
    if (i > 0) {
      down[(size_t)i].resize((size_t)sz);
      const int32_t* below = ids_host[i - 1];
      for (int64_t j = 0; j < sz; ++j) {
        const int32_t id = ids_host[i][j];
        int64_t pos;
        if (!below) {
          pos = id;
        } else {
          const int32_t* it = std::lower_bound(below, below + sizes[i - 1], id);
          if (it == below + sizes[i - 1] || *it != id)
            return fail(HENN_E_INVAL, "layer is not nested in the layer below");
          pos = it - below;
        }
        down[(size_t)i][(size_t)j] = (int32_t)pos;
      }
    }
    const int32_t* a = adj_host[i];
    if (!a) return fail(HENN_E_INVAL, "null adjacency");
    for (int64_t j = 0; j < sz; ++j) {
      for (int c = 0; c < adj_stride; ++c) {
        const int32_t u = a[j * adj_stride + c];
        if (u < -1 || u >= sz) return fail(HENN_E_INVAL, "adjacency entry out of range");
        if (u >= 0)
          for (int c2 = 0; c2 < c; ++c2)
            if (a[j * adj_stride + c2] == u) return fail(HENN_E_INVAL, "duplicate neighbour");
      }
    }
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  henn_index* ix = nullptr;
  try {
    ix = new_index(X, n, d, p, st);
    ix->num_layers = num_layers;
    ix->root_complete = p->root_complete_max > 0 && num_layers >= 2;
    for (int i = 0; i < num_layers; ++i) {
      LayerDev& L = ix->L[i];
      L.size = sizes[i];
      L.info.size = sizes[i];
      L.info.status = i == 0 ? 0 : 2;
      L.deg = adj_stride;
      L.info.degree = adj_stride;
      L.adj = dalloc<int32_t>(L.size * adj_stride);
      HENN_HIP(hipMemcpyAsync(L.adj, adj_host[i], sizeof(int32_t) * L.size * adj_stride,
                              hipMemcpyHostToDevice, st));
      if (i > 0) {
        L.ids = dalloc<int32_t>(L.size);
        L.down = dalloc<int32_t>(L.size);
        HENN_HIP(hipMemcpyAsync(L.ids, ids_host[i], sizeof(int32_t) * L.size,
                                hipMemcpyHostToDevice, st));
        HENN_HIP(hipMemcpyAsync(L.down, down[(size_t)i].data(), sizeof(int32_t) * L.size,
                                hipMemcpyHostToDevice, st));
        L.vec32 = dalloc<float>(L.size * ix->dpad);
        launch_copy_rows(ix->L[0].vec32, ix->dpad, L.ids, L.size, ix->dpad, L.vec32, ix->dpad,
                         st);
      }
      if (ix->storage != HENN_F32) {
        L.vecq = dalloc<uint8_t>(L.size * ix->dpad * storage_bytes(ix->storage));
        if (ix->storage == HENN_FP8_E4M3) L.scale = dalloc<float>(L.size);
        launch_quantize(ix->storage, L.vec32, L.size, ix->dpad, L.vecq, L.scale, st);
        if (ix->storage == HENN_FP8_E4M3) {
          L.adj_scale = dalloc<float>(L.size * L.deg);
          launch_adj_scale(L.adj, L.size * L.deg, L.scale, L.adj_scale, st);
        }
      }
      HENN_HIP(hipStreamSynchronize(st));
    }
    prepare_root(ix, st);
    *out = ix;
    return HENN_OK;
  } catch (const HipError& e) {
    destroy(ix);
    return from_hip(e);
  } catch (const std::bad_alloc&) {
    destroy(ix);
    return fail(HENN_E_NOMEM, "host allocation failed");
  }
}

henn_status henn_insert(henn_index* idx, const float* X_new, int64_t count, void* hip_stream) {
  if (!idx) return fail(HENN_E_INVAL, "index is null");
  if (count < 0) return fail(HENN_E_INVAL, "count must be >= 0");
  if (count == 0) return HENN_OK;
  if (!X_new) return fail(HENN_E_INVAL, "X_new is null");
  if (idx->next_id + count > 2147483647ll)
    return fail(HENN_E_INVAL, "ids would pass 2^31 - 1");
  if (idx->params.graph != HENN_GRAPH_NSW)
    return fail(HENN_E_UNSUPPORTED, "insertion needs an index built with the NSW graph");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const henn_build_params& p = idx->params;
  const int64_t base = idx->next_id;
  ++idx->updates;
  try {
    // membership: layer 0 takes every new point, layer i each member of
    // layer i - 1's new points whose coin comes up (probability 2^-m)
    std::vector<int32_t> ids((size_t)count), local((size_t)count), down;
    for (int64_t j = 0; j < count; ++j) {
      ids[(size_t)j] = (int32_t)(base + j);
      local[(size_t)j] = (int32_t)j;
    }
    grow_layer(idx, 0, X_new, ids, local, down, st);
    for (int i = 1; i < idx->num_layers && !ids.empty(); ++i) {
      const int64_t below_old = idx->L[i - 1].size - (int64_t)ids.size();
      std::vector<int32_t> up, up_local, up_down;
      for (size_t j = 0; j < ids.size(); ++j) {
        const uint64_t w = stream_word(p.seed, kTagInsert, (uint32_t)i, 0u, (uint64_t)ids[j]);
        if (uniform_index(w, 1ull << p.m) != 0) continue;
        up.push_back(ids[j]);
        up_local.push_back((int32_t)(ids[j] - base));
        up_down.push_back((int32_t)(below_old + (int64_t)j));
      }
      if (!up.empty()) grow_layer(idx, i, X_new, up, up_local, up_down, st);
      ids.swap(up);
    }
    idx->n += count;
    idx->next_id = base + count;
    if (idx->root_complete) refresh_root(idx, st);
  } catch (const HipError& e) {
    return from_hip(e);
  } catch (const std::bad_alloc&) {
    return fail(HENN_E_NOMEM, "host allocation failed");
  }
  return HENN_OK;
}

henn_status henn_delete(henn_index* idx, const int32_t* ids_host, int64_t count,
                        void* hip_stream) {
  if (!idx) return fail(HENN_E_INVAL, "index is null");
  if (count < 0) return fail(HENN_E_INVAL, "count must be >= 0");
  if (count == 0) return HENN_OK;
  if (!ids_host) return fail(HENN_E_INVAL, "ids_host is null");
  if (idx->params.graph != HENN_GRAPH_NSW)
    return fail(HENN_E_UNSUPPORTED, "deletion needs an index built with the NSW graph");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const henn_build_params& p = idx->params;
  std::vector<int32_t> gone(ids_host, ids_host + count);
  std::sort(gone.begin(), gone.end());
  gone.erase(std::unique(gone.begin(), gone.end()), gone.end());
  int32_t* below_np = nullptr;  // the layer below's old -> new positions (device)
  uint8_t* del_d = nullptr;
  int32_t* np_d = nullptr;
  try {
    // validate against layer 0's ids before touching anything
    LayerDev& L0 = idx->L[0];
    std::vector<int32_t> id0((size_t)L0.size);
    if (L0.ids) {
      HENN_HIP(hipMemcpy(id0.data(), L0.ids, sizeof(int32_t) * L0.size, hipMemcpyDeviceToHost));
    } else {
      for (int64_t j = 0; j < L0.size; ++j) id0[(size_t)j] = (int32_t)j;
    }
    for (int32_t g : gone)
      if (!std::binary_search(id0.begin(), id0.end(), g))
        return fail(HENN_E_INVAL, "an id to delete is not in the index");
    if ((int64_t)gone.size() >= L0.size)
      return fail(HENN_E_INVAL, "deletion would leave the index empty");
    ++idx->updates;
    int lpn, cpl;
    pick_lanes(idx->nchunks, 0, &lpn, &cpl);
    for (int i = 0; i < idx->num_layers; ++i) {
      LayerDev& L = idx->L[i];
      const int64_t s = L.size;
      std::vector<int32_t> ids_i;
      if (i == 0) {
        ids_i.swap(id0);
      } else {
        ids_i.resize((size_t)s);
        HENN_HIP(hipMemcpy(ids_i.data(), L.ids, sizeof(int32_t) * s, hipMemcpyDeviceToHost));
      }
      std::vector<uint8_t> del((size_t)s, 0);
      int64_t ndel = 0;
      for (int32_t g : gone) {
        const auto it = std::lower_bound(ids_i.begin(), ids_i.end(), g);
        if (it != ids_i.end() && *it == g) {
          del[(size_t)(it - ids_i.begin())] = 1;
          ++ndel;
        }
      }
      if (ndel == 0) {
        if (below_np) launch_remap_down(L.down, s, below_np, st);
        HENN_HIP(hipStreamSynchronize(st));
        (void)hipFree(below_np);
        below_np = nullptr;
        continue;
      }
      // repair the rows around the deleted members, then drop them
      del_d = dalloc<uint8_t>(s);
      HENN_HIP(hipMemcpyAsync(del_d, del.data(), s, hipMemcpyHostToDevice, st));
      repair_graph(L.vec32, s, idx->dpad, idx->nchunks, idx->metric, del_d, L.deg, L.adj, lpn,
                   cpl, st);
      std::vector<int32_t> np((size_t)s);
      int64_t t = 0;
      for (int64_t r = 0; r < s; ++r) np[(size_t)r] = del[(size_t)r] ? -1 : (int32_t)t++;
      np_d = dalloc<int32_t>(s);
      HENN_HIP(hipMemcpyAsync(np_d, np.data(), sizeof(int32_t) * s, hipMemcpyHostToDevice, st));
      float* vec = nullptr;
      int32_t *adj = nullptr, *ids = nullptr, *down = nullptr;
      try {
        vec = dalloc<float>(t * idx->dpad);
        adj = dalloc<int32_t>(t * L.deg);
        ids = dalloc<int32_t>(t);
        if (i > 0) down = dalloc<int32_t>(t);
        launch_compact_layer(L.vec32, L.adj, L.ids, L.down, np_d, below_np, s, idx->dpad, L.deg,
                             vec, adj, ids, down, st);
        HENN_HIP(hipStreamSynchronize(st));
      } catch (...) {
        (void)hipFree(vec);
        (void)hipFree(adj);
        (void)hipFree(ids);
        (void)hipFree(down);
        throw;
      }
      replace(L.vec32, vec);
      replace(L.adj, adj);
      replace(L.ids, ids);
      if (i > 0) replace(L.down, down);
      L.size = t;
      L.info.size = t;
      refresh_forms(idx, L, st);
      (void)hipFree(del_d);
      del_d = nullptr;
      (void)hipFree(below_np);
      below_np = np_d;
      np_d = nullptr;
    }
    (void)hipFree(below_np);
    below_np = nullptr;
    idx->n = idx->L[0].size;
    // a layer that fell below half its expected size is drawn again, with
    // every layer above it (App. C)
    for (int i = 1; i < idx->num_layers; ++i) {
      const int64_t expect = (idx->L[i - 1].size + (1ll << p.m) - 1) >> p.m;
      if (2 * idx->L[i].size >= expect) continue;
      for (int j = i; j < idx->num_layers; ++j) free_layer(idx->L[j]);
      sample_layers_from(idx, i, st);
      for (int j = i; j < idx->num_layers; ++j) finish_layer(idx, j, st);
      break;
    }
    idx->root_complete = p.root_complete_max > 0 && idx->num_layers >= 2;
    refresh_root(idx, st);
  } catch (const HipError& e) {
    (void)hipFree(below_np);
    (void)hipFree(del_d);
    (void)hipFree(np_d);
    return from_hip(e);
  } catch (const std::bad_alloc&) {
    (void)hipFree(below_np);
    (void)hipFree(del_d);
    (void)hipFree(np_d);
    return fail(HENN_E_NOMEM, "host allocation failed");
  }
  return HENN_OK;
}

henn_status henn_nsw_insert(const float* V, int64_t s, int32_t d, int32_t metric, int32_t* adj,
                            int32_t max_degree, int64_t lo, int64_t hi, int32_t degree,
                            int32_t ef_construction, void* hip_stream) {
  if (!V || !adj) return fail(HENN_E_INVAL, "null V or adj");
  if (s < 1 || s > 2147483647ll) return fail(HENN_E_INVAL, "s must be in [1, 2^31-1]");
  if (d < 1 || d > 1024) return fail(HENN_E_INVAL, "d must be in [1, 1024]");
  if (metric != HENN_L2 && metric != HENN_IP) return fail(HENN_E_INVAL, "metric");
  if (lo < 0 || hi < lo || hi > s) return fail(HENN_E_INVAL, "need 0 <= lo <= hi <= s");
  if (degree < 1 || degree > 32) return fail(HENN_E_INVAL, "degree in [1, 32]");
  if (max_degree < degree || max_degree > 64)
    return fail(HENN_E_INVAL, "max_degree in [degree, 64]");
  if (ef_construction < 1 || ef_construction > 2048)
    return fail(HENN_E_INVAL, "ef_construction in [1, 2048]");
  if (hi == lo) return HENN_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int dpad = (d + 7) / 8 * 8;
  float* vec = nullptr;
  try {
    int device = 0;
    HENN_HIP(hipGetDevice(&device));
    vec = dalloc<float>(hi * dpad);  // the rows in the library's padded layout
    launch_copy_rows(V, d, nullptr, hi, d, vec, dpad, st);
    const NswWork w(hi, hi - lo, degree);
    nsw_insert_batch(device, vec, dpad, dpad / 8, metric, adj, max_degree, lo, hi, degree,
                     ef_construction, w, st);
    HENN_HIP(hipStreamSynchronize(st));
  } catch (const HipError& e) {
    (void)hipFree(vec);
    return from_hip(e);
  } catch (const std::bad_alloc&) {
    (void)hipFree(vec);
    return fail(HENN_E_NOMEM, "host allocation failed");
  }
  (void)hipFree(vec);
  return HENN_OK;
}

// How a complete-graph root is scanned: 0 inside the search kernel (or no
// complete root), 1 the tiled VALU scan, 2 the MFMA shortlist + exact check.
// All three give the same keys.
static int root_mode(const henn_index* idx, const henn_search_params* sp) {
  if (!idx->root_complete || (sp->flags & HENN_SEARCH_NO_ROOT_KERNEL)) return 0;
  if (idx->root.size > 0 && !(sp->flags & HENN_SEARCH_ROOT_VALU)) return 2;
  return idx->nchunks <= 16 ? 1 : 0;
}

// Scratch layout: 256 B (persistent work counter), then for mode 1 the
// [splits][nq] root keys, for mode 2 the [nq] root keys and the Gram
// shortlists (RootShortlist).
static int64_t exact_visited_words(const henn_index* idx) {
  return ((int64_t)idx->L[0].size + 31) / 32;
}

// Offset of the exact visited sets (HENN_SEARCH_EXACT_VISITED) in the
// scratch: after the counter and the root-scan data, 256-byte aligned.
static int64_t search_root_bytes(const henn_index* idx, int64_t nq,
                                 const henn_search_params* sp) {
  const int64_t rs = idx->L[idx->num_layers - 1].size;
  int64_t per = 0;
  switch (root_mode(idx, sp)) {
    case 1:
      return (int64_t)sizeof(uint64_t) * root_scan_splits(nq, rs, &per) * nq;
    case 2:
      return (int64_t)sizeof(uint64_t) * nq + root_shortlist_bytes(nq, idx->root.kp);
    default:
      return 0;
  }
}

static int64_t exact_visited_offset(const henn_index* idx, int64_t nq,
                                    const henn_search_params* sp) {
  return (256 + search_root_bytes(idx, nq, sp) + 255) / 256 * 256;
}

static int64_t search_workspace_bytes(const henn_index* idx, int64_t nq,
                                      const henn_search_params* sp) {
  if (sp->flags & HENN_SEARCH_EXACT_VISITED)
    return exact_visited_offset(idx, nq, sp) + nq * exact_visited_words(idx) * 4;
  return 256 + search_root_bytes(idx, nq, sp);
}

// Rate of the current device's constant clock in kHz (read once per device).
static int device_clock_khz() {
  static std::atomic<int> rate[64];
  int dev = 0;
  HENN_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw HipError{hipErrorInvalidDevice, "device index"};
  int r = rate[dev].load(std::memory_order_relaxed);
  if (r <= 0) {
    HENN_HIP(hipDeviceGetAttribute(&r, hipDeviceAttributeWallClockRate, dev));
    if (r <= 0) throw HipError{hipErrorInvalidValue, "device clock rate"};
    rate[dev].store(r, std::memory_order_relaxed);
  }
  return r;
}

// The search behind henn_search_batch and henn_search_batch_noalloc.
// Scratch (the persistent work counter, then the root-scan keys) comes from
// `fixed` when given (fixed_bytes must hold search_workspace_bytes), else from
// the caller's workspace when large enough, else from one stream-ordered
// block of this call's own, so that concurrent searches never share a work
// counter or root keys.
static henn_status search_impl(const henn_index* idx, const float* Q, int64_t nq,
                               const henn_search_params* sp, int32_t* out_ids, float* out_dist,
                               hipStream_t st, char* fixed, int64_t fixed_bytes) {
  if (!idx) return fail(HENN_E_INVAL, "index is null");
  if (!sp || sp->struct_size != sizeof(henn_search_params))
    return fail(HENN_E_INVAL, "search params null or struct_size mismatch");
  if (nq < 0 || nq > 2147483647ll) return fail(HENN_E_INVAL, "nq out of range");
  if (nq == 0) return HENN_OK;
  if (!Q || !out_ids || !out_dist) return fail(HENN_E_INVAL, "null query or output pointer");
  if (sp->k_max < 1 || sp->k_max > 1024) return fail(HENN_E_INVAL, "k_max in [1, 1024]");
  if (!sp->k && (sp->k_all < 1 || sp->k_all > sp->k_max)) return fail(HENN_E_INVAL, "k_all");
  if (!sp->ef && sp->ef_all < 1) return fail(HENN_E_INVAL, "ef_all >= 1");
  if (sp->ef && sp->ef_max < 1) return fail(HENN_E_INVAL, "ef_max >= 1");
  if (sp->ef_upper < 1) return fail(HENN_E_INVAL, "ef_upper >= 1");
  if (idx->storage != HENN_F32 && sp->rerank_factor < 1)
    return fail(HENN_E_INVAL, "rerank_factor >= 1");
  const int ef_need = std::max(std::max(sp->k_max, sp->ef ? sp->ef_max : sp->ef_all), sp->ef_upper);
  if (ef_need > 2048) return fail(HENN_E_INVAL, "beam width above 2048");
  char* ws = nullptr;
  bool ws_owned = false;
  try {
    SearchArgs a;
    memset(&a, 0, sizeof(a));
    const int eb = storage_bytes(idx->storage);
    for (int i = 0; i < idx->num_layers; ++i) {
      const LayerDev& L = idx->L[i];
      SearchLayer& s = a.layer[i];
      s.vec = idx->storage == HENN_F32 ? (const void*)L.vec32 : (const void*)L.vecq;
      s.scale = L.scale;
      s.adj = L.adj;
      s.adj_scale = L.adj_scale;
      s.down = L.down;
      s.size = (int32_t)L.size;
      s.deg = L.deg;
      s.row_bytes = (int64_t)idx->dpad * eb;
    }
    a.rerank_vec = idx->storage == HENN_F32 ? nullptr : idx->L[0].vec32;
    a.ids0 = idx->L[0].ids;
    a.Q = Q;
    a.nq = nq;
    a.k_arr = sp->k;
    a.ef_arr = sp->ef;
    a.k_all = sp->k_all;
    a.ef_all = sp->ef_all;
    a.k_max = sp->k_max;
    a.ef_upper = sp->ef_upper;
    a.ef_cap = next_pow2(ef_need);
    a.rerank_factor = std::max(1, sp->rerank_factor);
    a.num_layers = idx->num_layers;
    a.d = idx->d;
    a.dpad = idx->dpad;
    a.nchunks = idx->nchunks;
    a.metric = idx->metric;
    if (sp->vis_bits != 0 && (sp->vis_bits < 8 || sp->vis_bits > 13))
      return fail(HENN_E_INVAL, "vis_bits in [8, 13]");
    a.vis_bits = sp->vis_bits ? sp->vis_bits
                              : default_vis_bits(ef_need, idx->n,
                                                 !(sp->flags & (HENN_SEARCH_VIS16 | HENN_SEARCH_VIS32)));
    a.root_complete = idx->root_complete ? 1 : 0;
    a.out_ids = out_ids;
    a.out_dist = out_dist;
    a.counters = sp->counters;
    if (sp->query_ns) {
      a.query_ns = sp->query_ns;
      a.clock_ns = 1e6 / device_clock_khz();
    }
    if (!rows_addressable(a))
      return fail(HENN_E_UNSUPPORTED, "search needs n * ceil(d / 8) < 2^32");

    // autotuned shape for this (storage, beam bucket, k bucket), if cached
    int want_lpn = sp->lanes_per_vec, want_wpb = sp->waves_per_block;
    bool want_pers = (sp->flags & HENN_SEARCH_PERSISTENT) != 0;
    {
      std::lock_guard<std::mutex> lk(const_cast<henn_index*>(idx)->tune_mu);
      for (const TuneEntry& te : idx->tune) {
        if (te.storage == idx->storage && te.ef_bucket == a.ef_cap &&
            te.k_bucket == next_pow2(sp->k_max)) {
          if (!want_lpn) want_lpn = te.lanes_per_vec;
          if (!want_wpb) want_wpb = te.waves_per_block;
          if (!sp->vis_bits) a.vis_bits = te.vis_bits;
          if (te.persistent && !(sp->flags & HENN_SEARCH_PERSISTENT)) want_pers = true;
          break;
        }
      }
    }
    LaunchShape sh;
    int lpn = 0, cpl = 0;
    pick_lanes(idx->nchunks, want_lpn, &lpn, &cpl);
    if (lpn == 0) return fail(HENN_E_INVAL, "lanes_per_vec not available for this dimension");
    sh.lanes_per_vec = lpn;
    sh.chunks_per_lane = cpl;
    sh.vis_bits = a.vis_bits;
    a.vis_bytes = (sp->flags & HENN_SEARCH_VIS32) ? 4 : vis_tag_bytes(idx->n, a.vis_bits);
    if (a.vis_bytes == 1 && (sp->flags & HENN_SEARCH_VIS16)) a.vis_bytes = 2;
    int wpb = want_wpb > 0 ? want_wpb : 4;
    if (wpb != 1 && wpb != 2 && wpb != 4 && wpb != 8) return fail(HENN_E_INVAL, "waves_per_block");
    while (wpb > 1 && search_lds_per_wave(a.ef_cap, a.vis_bits, a.vis_bytes) * wpb > 65536) wpb /= 2;
    sh.waves_per_block = wpb;
    sh.persistent = want_pers;
    sh.blocks = 0;

    // scratch: the persistent work counter (256 B), the root-scan data, the
    // exact visited sets
    const int rmode = root_mode(idx, sp);
    const bool exact_vis = (sp->flags & HENN_SEARCH_EXACT_VISITED) != 0;
    if (sh.persistent || rmode != 0 || exact_vis) {
      const int64_t need = search_workspace_bytes(idx, nq, sp);
      if (fixed) {
        if (fixed_bytes < need)
          return fail(HENN_E_INVAL, "search needs " + std::to_string(need) +
                                        " scratch bytes, above the fixed maximum of " +
                                        std::to_string(fixed_bytes));
        ws = fixed;
      } else if (sp->workspace && sp->workspace_bytes >= need) {
        ws = static_cast<char*>(sp->workspace);
      } else {
        HENN_HIP(dev_alloc_async(reinterpret_cast<void**>(&ws), need, st));
        ws_owned = true;
      }
    }
    if (sh.persistent) a.work_counter = reinterpret_cast<uint32_t*>(ws);
    if (exact_vis) {
      a.vis_exact = reinterpret_cast<uint32_t*>(ws + exact_visited_offset(idx, nq, sp));
      a.vis_exact_words = exact_visited_words(idx);
    }
    if (rmode == 2) {
      int64_t per = 0;
      const int splits = root_gram_splits(nq, idx->root.size, &per);
      uint64_t* root_best = reinterpret_cast<uint64_t*>(ws + 256);
      const RootShortlist sl = root_shortlist_at(root_best + nq, nq, idx->root.kp);
      launch_root_gram(Q, nq, idx->d, idx->root, idx->dpad, idx->metric, splits, per, sl, st);
      if (!launch_root_check(idx->storage, a, sl, root_best, st)) {
        if (ws_owned) (void)hipFreeAsync(ws, st);
        return fail(HENN_E_UNSUPPORTED, "no root check kernel for this shape");
      }
      a.root_best = root_best;
      a.root_splits = 1;
    } else if (rmode == 1) {
      int64_t per = 0;
      const int splits = root_scan_splits(nq, idx->L[idx->num_layers - 1].size, &per);
      uint64_t* root_best = reinterpret_cast<uint64_t*>(ws + 256);
      if (!launch_root_scan(idx->storage, a, splits, per, root_best, st)) {
        if (ws_owned) (void)hipFreeAsync(ws, st);
        return fail(HENN_E_UNSUPPORTED, "no root scan kernel for this shape");
      }
      a.root_best = root_best;
      a.root_splits = splits;
    }
    if (sp->ev_begin) HENN_HIP(hipEventRecord(static_cast<hipEvent_t>(sp->ev_begin), st));
    const bool ok = launch_search(idx->storage, a, sh, st);
    if (sp->ev_end) HENN_HIP(hipEventRecord(static_cast<hipEvent_t>(sp->ev_end), st));
    if (ws_owned) {
      ws_owned = false;
      HENN_HIP(hipFreeAsync(ws, st));
    }
    if (!ok) return fail(HENN_E_UNSUPPORTED, "no search kernel for this shape");
    HENN_HIP(hipGetLastError());
    return HENN_OK;
  } catch (const HipError& e) {
    if (ws_owned) (void)hipFreeAsync(ws, st);
    return from_hip(e);
  }
}

henn_status henn_search_batch(const henn_index* idx, const float* Q, int64_t nq,
                              const henn_search_params* sp, int32_t* out_ids, float* out_dist,
                              void* hip_stream) {
  return search_impl(idx, Q, nq, sp, out_ids, out_dist, static_cast<hipStream_t>(hip_stream),
                     nullptr, 0);
}

}  // extern "C"

// Scratch of henn_search_batch_noalloc: a fixed device array (one copy per
// GPU, held until the process ends).  Host code never passes the array's
// name to a kernel: it takes the device address from hipGetSymbolAddress,
// once per device, with that device current.
static constexpr int64_t kNoAllocScratchBytes = 32ll << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[64] = {};

extern "C" {

henn_status henn_search_batch_noalloc(const henn_index* idx, const float* Q, int64_t nq,
                                      const henn_search_params* sp, int32_t* out_ids,
                                      float* out_dist, void* hip_stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(HENN_E_DEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= 64) return fail(HENN_E_UNSUPPORTED, "device id above 63");
  char* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(HENN_E_DEVICE, std::string("hipGetSymbolAddress of the scratch array: ") +
                                       hipGetErrorString(e));
      g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    ptr = g_scratch_ptr[dev];
  }
  return search_impl(idx, Q, nq, sp, out_ids, out_dist, static_cast<hipStream_t>(hip_stream),
                     ptr, kNoAllocScratchBytes);
}

henn_status henn_autotune(henn_index* idx, const float* Q, int64_t nq,
                          const henn_search_params* sp, void* hip_stream,
                          henn_search_params* tuned) {
  if (!idx || !Q || !sp) return fail(HENN_E_INVAL, "null argument");
  if (sp->struct_size != sizeof(henn_search_params))
    return fail(HENN_E_INVAL, "search params struct_size mismatch");
  if (nq < 1) return fail(HENN_E_INVAL, "autotune needs at least one query");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int32_t* ids = nullptr;
  float* dist = nullptr;
  void* ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  try {
    ids = dalloc<int32_t>(nq * sp->k_max);
    dist = dalloc<float>(nq * sp->k_max);
    HENN_HIP(hipEventCreate(&e0));
    HENN_HIP(hipEventCreate(&e1));
    const int P = next_pow2(idx->nchunks);
    std::vector<int> lpns;
    for (int l : {1, 2, 4, 8, 16}) {
      int lp = 0, cp = 0;
      pick_lanes(idx->nchunks, l, &lp, &cp);
      if (lp == l && l <= P) lpns.push_back(l);
    }
    henn_search_params c = *sp;
    c.counters = nullptr;
    c.query_ns = nullptr;
    c.ev_begin = c.ev_end = nullptr;
    // one workspace for every trial, so that no trial times an allocation
    // (its size depends on the flags and nq, not on the launch shape)
    {
      henn_search_params cp = c;
      cp.flags |= HENN_SEARCH_PERSISTENT;
      const int64_t wb = search_workspace_bytes(idx, nq, &cp);
      HENN_HIP(dev_alloc(reinterpret_cast<void**>(&ws), wb));
      c.workspace = ws;
      c.workspace_bytes = wb;
    }
    // one warm-up launch, then the median of five
    auto time_of = [&](const henn_search_params& q) -> float {
      float t[5];
      for (int rep = 0; rep < 6; ++rep) {
        HENN_HIP(hipEventRecord(e0, st));
        henn_status s2 = henn_search_batch(idx, Q, nq, &q, ids, dist, st);
        HENN_HIP(hipEventRecord(e1, st));
        HENN_HIP(hipEventSynchronize(e1));
        if (s2 != HENN_OK) return 1e30f;
        float ms = 0.f;
        HENN_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) t[rep - 1] = ms;
      }
      std::sort(t, t + 5);
      return t[2];
    };
    // 1) lanes per vector x visited-table size at 4 waves per block
    henn_search_params bestp = c;
    float bt = 1e30f;
    for (int l : lpns) {
      for (int vb = 8; vb <= 12; ++vb) {
        henn_search_params q = c;
        q.lanes_per_vec = l;
        q.waves_per_block = 4;
        q.vis_bits = vb;
        q.flags &= ~HENN_SEARCH_PERSISTENT;
        const float t = time_of(q);
        if (t < bt) { bt = t; bestp = q; }
      }
    }
    // 2) waves per block and persistent launch around the best (the phase-1
    //    winner is timed again among them)
    const henn_search_params base = bestp;
    bt = 1e30f;
    for (int w : {1, 2, 4, 8}) {
      for (int pers = 0; pers < 2; ++pers) {
        henn_search_params q = base;
        q.waves_per_block = w;
        q.flags = pers ? (q.flags | HENN_SEARCH_PERSISTENT) : (q.flags & ~HENN_SEARCH_PERSISTENT);
        const float t = time_of(q);
        if (t < bt) { bt = t; bestp = q; }
      }
    }
    const int ef_need = std::max(std::max(sp->k_max, sp->ef ? sp->ef_max : sp->ef_all), sp->ef_upper);
    TuneEntry te{idx->storage, next_pow2(ef_need), next_pow2(sp->k_max), bestp.lanes_per_vec,
                 bestp.waves_per_block, bestp.vis_bits,
                 (bestp.flags & HENN_SEARCH_PERSISTENT) ? 1 : 0};
    {
      std::lock_guard<std::mutex> lk(idx->tune_mu);
      bool found = false;
      for (TuneEntry& x : idx->tune)
        if (x.storage == te.storage && x.ef_bucket == te.ef_bucket && x.k_bucket == te.k_bucket) {
          x = te;
          found = true;
        }
      if (!found) idx->tune.push_back(te);
    }
    if (tuned) {
      *tuned = *sp;
      tuned->lanes_per_vec = bestp.lanes_per_vec;
      tuned->waves_per_block = bestp.waves_per_block;
      tuned->vis_bits = bestp.vis_bits;
      tuned->flags = bestp.flags | (sp->flags & HENN_SEARCH_COUNTERS);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(ids);
    (void)hipFree(dist);
    (void)hipFree(ws);
    return HENN_OK;
  } catch (const HipError& e) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(ids);
    (void)hipFree(dist);
    (void)hipFree(ws);
    return from_hip(e);
  }
}

henn_status henn_search_workspace_size(const henn_index* idx, int64_t nq,
                                       const henn_search_params* sp, int64_t* bytes) {
  if (!idx || !sp || !bytes) return fail(HENN_E_INVAL, "null argument");
  if (sp->struct_size != sizeof(henn_search_params))
    return fail(HENN_E_INVAL, "search params struct_size mismatch");
  if (nq < 0) return fail(HENN_E_INVAL, "nq < 0");
  *bytes = search_workspace_bytes(idx, nq, sp);
  return HENN_OK;
}

}  // extern "C"

struct henn_search_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* workspace = nullptr;
  const henn_index* idx = nullptr;
  int64_t idx_updates = 0;  // the index's update count when captured
};

extern "C" {

henn_status henn_search_graph_create(const henn_index* idx, const float* Q, int64_t nq,
                                     const henn_search_params* sp, int32_t* out_ids,
                                     float* out_dist, henn_search_graph** out) {
  if (!idx || !sp || !out) return fail(HENN_E_INVAL, "null argument");
  if (sp->struct_size != sizeof(henn_search_params))
    return fail(HENN_E_INVAL, "search params struct_size mismatch");
  if (nq < 1) return fail(HENN_E_INVAL, "a graph needs nq >= 1");
  if (sp->ev_begin || sp->ev_end) return fail(HENN_E_INVAL, "no timing events in a graph");
  henn_search_graph* g = new henn_search_graph();
  g->idx = idx;
  g->idx_updates = idx->updates;
  hipStream_t cs = nullptr;
  try {
    const int64_t need = search_workspace_bytes(idx, nq, sp);
    HENN_HIP(dev_alloc(reinterpret_cast<void**>(&g->workspace), need));
    HENN_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    henn_search_params c = *sp;
    c.workspace = g->workspace;
    c.workspace_bytes = need;
    HENN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const henn_status st = henn_search_batch(idx, Q, nq, &c, out_ids, out_dist, cs);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &graph);
    if (st != HENN_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      throw std::runtime_error(henn_last_error());
    }
    HENN_HIP(ec);
    g->graph = graph;
    HENN_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    HENN_HIP(hipStreamDestroy(cs));
    *out = g;
    return HENN_OK;
  } catch (const HipError& e) {
    if (cs) (void)hipStreamDestroy(cs);
    henn_search_graph_free(g);
    return from_hip(e);
  } catch (const std::exception& e) {
    if (cs) (void)hipStreamDestroy(cs);
    henn_search_graph_free(g);
    return fail(HENN_E_INVAL, std::string("capture failed: ") + e.what());
  }
}

henn_status henn_search_graph_launch(henn_search_graph* g, void* hip_stream) {
  if (!g || !g->exec) return fail(HENN_E_INVAL, "null graph");
  // the graph holds the layer arrays of capture time, which Insert / Delete replace
  if (g->idx->updates != g->idx_updates)
    return fail(HENN_E_INVAL, "the index was updated after this graph was captured");
  const hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return from_hip(HipError{e, "hipGraphLaunch"});
  return HENN_OK;
}

void henn_search_graph_free(henn_search_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->workspace) (void)hipFree(g->workspace);
  delete g;
}

void henn_free(henn_index* idx) { destroy(idx); }

henn_status henn_index_shape(const henn_index* idx, int32_t* num_layers, int64_t* n, int32_t* d) {
  if (!idx) return fail(HENN_E_INVAL, "index is null");
  if (num_layers) *num_layers = idx->num_layers;
  if (n) *n = idx->n;
  if (d) *d = idx->d;
  return HENN_OK;
}

henn_status henn_layer_info_get(const henn_index* idx, int32_t layer, henn_layer_info* info) {
  if (!idx || !info) return fail(HENN_E_INVAL, "null argument");
  if (layer < 0 || layer >= idx->num_layers) return fail(HENN_E_INVAL, "layer out of range");
  *info = idx->L[layer].info;
  info->size = idx->L[layer].size;
  info->degree = idx->L[layer].deg;
  return HENN_OK;
}

henn_status henn_export_layer(const henn_index* idx, int32_t layer, int32_t* ids_host,
                              int32_t* adj_host) {
  if (!idx) return fail(HENN_E_INVAL, "index is null");
  if (layer < 0 || layer >= idx->num_layers) return fail(HENN_E_INVAL, "layer out of range");
  const LayerDev& L = idx->L[layer];
  try {
    if (ids_host) {
      if (L.ids) {
        HENN_HIP(hipMemcpy(ids_host, L.ids, sizeof(int32_t) * L.size, hipMemcpyDeviceToHost));
      } else {
        for (int64_t j = 0; j < L.size; ++j) ids_host[j] = (int32_t)j;
      }
    }
    if (adj_host)
      HENN_HIP(hipMemcpy(adj_host, L.adj, sizeof(int32_t) * L.size * L.deg, hipMemcpyDeviceToHost));
    return HENN_OK;
  } catch (const HipError& e) {
    return from_hip(e);
  }
}

}  // extern "C"

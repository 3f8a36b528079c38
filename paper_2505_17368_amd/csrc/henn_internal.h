// henn_internal.h -- host-side index layout and kernel launch interfaces.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/henn.h"
#include "../../include/henn_testing.h"

namespace henn {

// One layer of the hierarchy as it lives in HBM.
//   vec32: FP32 rows [size][dpad] (zero padded to a multiple of 8 coords);
//          for layer 0 this is the library's copy of X.
//   vecq:  storage-format rows (BF16 [size][dpad] or FP8 [size][dpad]) for
//          the precision forms, else nullptr.
//   scale: per-row FP32 scale (FP8) or nullptr.
//   adj:   int32 [size][deg], positions within the layer, (dist, id) order,
//          -1 padded.
//   adj_scale: FP8 only, float [size][deg]: the scale of each neighbour, so
//          that an expansion reads its neighbours' scales with the adjacency
//          row instead of one scattered 4-byte read per evaluated row.
//   ids:   int32 [size] ascending point ids. For layer 0 it is nullptr (the
//          position is the id) until the first deletion leaves gaps in the
//          ids; from then on it is kept like the upper layers' lists.
//   down:  int32 [size] position of the same point in layer-1 (the
//          inter-layer edge of Def. HENN); nullptr for layer 0.
struct LayerDev {
  int64_t size = 0;
  int32_t deg = 0;
  float* vec32 = nullptr;
  void* vecq = nullptr;
  float* scale = nullptr;
  int32_t* adj = nullptr;
  float* adj_scale = nullptr;
  int32_t* ids = nullptr;
  int32_t* down = nullptr;
  henn_layer_info info{};
};

}  // namespace henn

namespace henn {
// A complete-graph root prepared for the MFMA scan (dpad <= 128):
//   dec:  FP32 [size][dpad], the values the search form stores (the FP32
//         rows themselves, decoded BF16, or scale * decoded FP8);
//   mean: [dpad] mean of dec (L2 only, else nullptr);
//   norm: [size] |dec - mean|^2 (L2) or |dec|^2 (IP);
//   nmax: max of norm; mean_n2: |mean|^2;
//   rowb: the BF16 Gram operand, bf16 of dec - mean (L2) or dec (IP),
//         [rows_pad][kp] with kp = dpad rounded up to 16 and rows_pad = size
//         rounded up to 32, zero padded;
//   normp: [rows_pad] the Gram value's norm term, norm (L2) or 0 (IP), +inf
//         for the padding rows.
struct RootAux {
  int64_t size = 0;
  float* dec = nullptr;
  bool dec_owned = false;
  float* mean = nullptr;
  float* norm = nullptr;
  float nmax = 0.0f, mean_n2 = 0.0f;
  uint16_t* rowb = nullptr;
  float* normp = nullptr;
  int kp = 0;
};
// Gram shortlist of a complete-root scan, one per query: the rows whose
// Gram value lies within the query's margin mq of a threshold at or above
// the smallest Gram value over the root (each root split's pass uses the
// smaller of its own smallest value and the query's running minimum qmin).
// Up to kRootCap (value, root position) entries in ent, in no particular
// order, and their full number in cnt (above kRootCap: the list overflowed
// and the check scans the root).  qb holds each query's BF16 Gram operand.
constexpr int kRootCap = 64;
struct RootShortlist {
  uint16_t* qb = nullptr;   // [nq][kp]: bf16 of -2 (q - mean) (L2) or -q (IP)
  float* mq = nullptr;      // [nq]: the margin of each query
  uint32_t* qmin = nullptr; // [nq]: running minimum Gram value (ordered bits)
  int32_t* cnt = nullptr;   // [nq]: rows listed
  uint2* ent = nullptr;     // [nq][kRootCap]: (value bits, root position)
};
// Bytes of a shortlist for (nq, kp), including 256 bytes of slack for
// aligning its start.
int64_t root_shortlist_bytes(int64_t nq, int kp);
RootShortlist root_shortlist_at(void* base, int64_t nq, int kp);

// One autotuned launch shape, valid for a (storage, beam bucket, k bucket).
struct TuneEntry {
  int storage, ef_bucket, k_bucket;
  int lanes_per_vec, waves_per_block, vis_bits, persistent;
};
}  // namespace henn

struct henn_index {
  int64_t n = 0;
  int32_t d = 0, dpad = 0, nchunks = 0;
  int32_t metric = 0, storage = 0;
  henn_build_params params{};
  int32_t num_layers = 0;
  int64_t next_id = 0;         // id of the next inserted point (ids are never reused)
  int64_t updates = 0;         // Insert / Delete calls that changed the index; servers
                               // and captured graphs made before one refuse to run
  bool root_complete = false;  // root searched by exhaustive scan (complete graph)
  henn::LayerDev L[HENN_MAX_LAYERS];
  henn::RootAux root;  // prepared when root_complete and dpad <= 128
  int device = 0;
  std::mutex tune_mu;
  std::vector<henn::TuneEntry> tune;  // autotuned launch shapes
};

namespace henn {

// ---- error plumbing -------------------------------------------------------
void set_error(const std::string& msg);

struct HipError {
  hipError_t e;
  const char* what;
};

#define HENN_HIP(call)                                   \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) throw ::henn::HipError{_e, #call}; \
  } while (0)

// Device allocation of every library path: hipMalloc / hipMallocAsync behind
// the allocation-failure injector of henn_testing.h (off unless a test arms
// it).
hipError_t dev_alloc(void** p, size_t bytes);
hipError_t dev_alloc_async(void** p, size_t bytes, hipStream_t st);

// Owning device array for temporaries: freed when its scope ends, also when
// an exception unwinds it (hipFree waits for the device as usual).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  explicit DevBuf(int64_t count) {
    HENN_HIP(dev_alloc(reinterpret_cast<void**>(&p), sizeof(T) * (size_t)(count > 0 ? count : 1)));
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  T* get() const { return p; }
};

inline int next_pow2(int v) {
  int p = 1;
  while (p < v) p *= 2;
  return p;
}

// ---- search ---------------------------------------------------------------
struct SearchLayer {
  const void* vec;
  const float* scale;
  const int32_t* adj;
  const float* adj_scale;  // FP8: neighbour scales beside adj, else nullptr
  const int32_t* down;
  int32_t size;
  int32_t deg;
  int64_t row_bytes;
};

struct SearchArgs {
  SearchLayer layer[HENN_MAX_LAYERS];
  const float* rerank_vec;  // FP32 layer-0 rows for the precision forms, else nullptr
  const int32_t* ids0;      // point id of each layer-0 position (after deletions), or
                            // nullptr when positions are the ids
  const float* Q;
  int64_t nq;
  const int32_t* k_arr;
  const int32_t* ef_arr;
  int32_t k_all, ef_all, k_max, ef_upper, ef_cap, rerank_factor;
  int32_t num_layers, d, dpad, nchunks, metric, vis_bits, root_complete;
  int32_t vis_bytes;  // bytes per visited-table entry: 1, 2 or 4 (see vis_tag_bytes)
  int32_t* out_ids;
  float* out_dist;
  int32_t* counters;
  uint32_t* work_counter;  // persistent form: device query counter
  const uint64_t* root_best;  // [root_splits][nq] best root keys from k_root_scan, or nullptr
  int32_t root_splits;
  // HENN_SEARCH_EXACT_VISITED: per query vis_exact_words 32-bit words, one
  // bit per member of the largest layer, replacing the LDS table
  uint32_t* vis_exact = nullptr;
  int64_t vis_exact_words = 0;
  // per-query time in ns (henn_search_params::query_ns) and the period of
  // the device's constant clock in ns
  int64_t* query_ns = nullptr;
  double clock_ns = 0;
};

// Traversal state of one query between expansions (wave-uniform).  The
// serving form keeps it in HBM between ticks, with the list W and the
// visited table.  li: current layer, or kSlotNew / kSlotDone.
constexpr int32_t kSlotNew = -1;
constexpr int32_t kSlotDone = -2;
struct QState {
  int32_t li;
  int32_t need_init;
  int32_t wsize;
  int32_t cur;
  float cur_d;
  int32_t exps, evals, exps0, evals0;
  int32_t k, ef0;
  int32_t pad;
};

struct ServeArgs {
  const int32_t* active;      // [n_active] slots to advance this tick
  int32_t n_active;
  int32_t budget;             // expansions per slot per tick
  QState* states;             // [max_slots]
  const int64_t* state_off;   // [max_slots] byte offset of the slot's W + visited table
  const int32_t* cap;         // [max_slots] list capacity of the slot (power of two)
  char* arena;
  int32_t* done_count;        // completions of this tick
  int32_t* done_clear;        // the next tick's counter, cleared by this kernel
  // completion i of the tick: row i of [max_slots][1 + 2 k_max] words =
  // its slot, k_max ids, k_max distances (FP32 bits), written straight into
  // the host's pinned completion buffer
  int32_t* done_rows;
};

struct LaunchShape {
  int lanes_per_vec;    // LPN
  int chunks_per_lane;  // CPL
  int waves_per_block;
  int vis_bits;
  bool persistent;
  int blocks;           // persistent grid size (0 = computed)
};

// The visited table's entry for id is at slot id mod 2^vis_bits and holds
// the tag (id >> vis_bits) + 1 (0 = empty), which identifies the id exactly:
// in one byte when every id of the index is below 2^vis_bits * 255, in two
// below 2^vis_bits * 65535; larger indexes keep full ids (4 bytes, hashed slot).
inline int vis_tag_bytes(int64_t n, int vis_bits) {
  const int64_t hi = (n - 1) >> vis_bits;
  return hi < 255 ? 1 : hi < 65535 ? 2 : 4;
}

// Default table size for a beam width: 2^10 / 2^11 / 2^12 slots, one more
// bit where one-byte tags are exact there (the bytes of two-byte tags at the
// base size) unless the caller keeps wider tags.
inline int default_vis_bits(int ef_need, int64_t n, bool narrow_ok) {
  int b = ef_need <= 64 ? 10 : ef_need <= 256 ? 11 : 12;
  if (narrow_ok && vis_tag_bytes(n, b + 1) == 1) b += 1;
  return b;
}

// Shared-memory bytes one wave needs for a given list capacity.
size_t search_lds_per_wave(int ef_cap, int vis_bits, int vis_bytes);

// Whether every layer's rows have 32-bit first-chunk indices
// (size * chunks per row < 2^32), which the search kernel needs.
bool rows_addressable(const SearchArgs& a);

// Enqueues the search kernel.  Returns false when no kernel instance
// matches (storage, lanes_per_vec, chunks_per_lane) or !rows_addressable(a).
bool launch_search(int storage, const SearchArgs& a, const LaunchShape& s, hipStream_t st);
// The per-storage halves of launch_search and launch_serve_step.
bool launch_search_f32(const SearchArgs& a, const LaunchShape& s, hipStream_t st);
bool launch_search_bf16(const SearchArgs& a, const LaunchShape& s, hipStream_t st);
bool launch_search_fp8(const SearchArgs& a, const LaunchShape& s, hipStream_t st);

bool launch_serve_step(int storage, const SearchArgs& a, const ServeArgs& sv,
                       const LaunchShape& sh, hipStream_t st);
bool launch_serve_f32(const SearchArgs& a, const ServeArgs& sv, const LaunchShape& sh,
                      hipStream_t st);
bool launch_serve_bf16(const SearchArgs& a, const ServeArgs& sv, const LaunchShape& sh,
                       hipStream_t st);
bool launch_serve_fp8(const SearchArgs& a, const ServeArgs& sv, const LaunchShape& sh,
                      hipStream_t st);
// root_keys (nullable): the new requests' complete-root keys, copied to
// slot_root[slot].
void launch_serve_admit(const float* staged_q, const int32_t* meta, int n_new, int d,
                        float* slot_q, int32_t* slot_k, int32_t* slot_ef, int64_t* state_off,
                        int32_t* cap, QState* states, const uint64_t* root_keys,
                        uint64_t* slot_root, hipStream_t st);

// Exhaustive scan of a complete-graph root (dpad <= 128): writes
// [splits][nq] best keys.  root_scan_splits() picks the split of the root.
int root_scan_splits(int64_t nq, int64_t root_size, int64_t* rows_per_split);
bool launch_root_scan(int storage, const SearchArgs& a, int splits, int64_t rows_per_split,
                      uint64_t* out, hipStream_t st);

// The same scan on matrix cores: a BF16 Gram shortlist per (split, query,
// lane half) over the prepared root (launch_root_gram), then per query the
// exact canonical distances of the rows that can still be the nearest given
// the Gram error bound, or a full canonical scan when a list overflowed
// (launch_root_check); writes [nq] best keys.
int root_gram_splits(int64_t nq, int64_t root_size, int64_t* rows_per_split);
// Fills r.rowb / r.normp / r.kp from r.dec, r.mean and r.norm (allocates).
void prepare_root_bf16(RootAux& r, int dpad, int metric, hipStream_t st);
void launch_root_gram(const float* Q, int64_t nq, int d, const RootAux& r, int dpad, int metric,
                      int splits, int64_t rows_per_split, const RootShortlist& sl,
                      hipStream_t st);
bool launch_root_check(int storage, const SearchArgs& a, const RootShortlist& sl, uint64_t* out,
                       hipStream_t st);

// ---- build ----------------------------------------------------------------
void launch_copy_rows(const float* src, int64_t src_stride, const int32_t* ids, int64_t count,
                      int d, float* dst, int dpad, hipStream_t st);
void launch_ring_keys(int lpn, int cpl, const float* vec, int dpad, int nchunks, int metric,
                      int64_t s, const int32_t* centres, int r, uint64_t* keys, hipStream_t st);
void launch_radix_select(const uint64_t* keys, int64_t s, int r, const int64_t* ranks_host,
                         uint64_t* out_keys_host, hipStream_t st);
// cand == nullptr: the sample is Alg. 2's draws of (seed, layer, attempt);
// else the `draws` positions in cand.
void launch_ring_hits(int lpn, int cpl, const float* vec, int dpad, int nchunks, int metric,
                      int64_t s, uint64_t seed, int layer, int attempt, int64_t draws,
                      const int32_t* cand, const int32_t* centres, const uint64_t* lo,
                      const uint64_t* hi, int r, uint32_t* hits, hipStream_t st);
// Alg. 3 (BuildEpsNetDiscV2): m halving steps of positions [0, s); writes the
// ceil(s / 2^m) ascending survivors to out and returns their count.
int64_t launch_halve(uint64_t seed, int layer, int attempt, int64_t s, int m, int32_t* out,
                     hipStream_t st);
void launch_draw_mark(uint64_t seed, int layer, int attempt, int64_t s, int64_t draws,
                      uint32_t* bitmap, hipStream_t st);
int64_t compact_bitmap(const uint32_t* bitmap, int64_t s, int32_t* out_local, hipStream_t st);
int64_t exclusive_scan_u32(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t st);
void launch_map_ids(const int32_t* prev_ids, const int32_t* local, int64_t count, int32_t* ids,
                    int32_t* down, hipStream_t st);
void layer_mean(const float* vec, int64_t size, int dpad, float* mean_dev, hipStream_t st);
void launch_row_norms(const float* vec, const float* mean, int64_t size, int dpad, float* norms,
                      hipStream_t st);
float max_norm(const float* norms, int64_t size, hipStream_t st);
void launch_quantize(int storage, const float* vec, int64_t size, int dpad, void* out,
                     float* scale, hipStream_t st);
// FP32 rows of the stored values: decoded BF16, or scale * decoded FP8.
void launch_decode_rows(int storage, const void* vq, const float* scale, int64_t size, int dpad,
                        float* out, hipStream_t st);
// out[i] = scale[adj[i]] for the n entries of an adjacency array (0 for -1).
void launch_adj_scale(const int32_t* adj, int64_t n, const float* scale, float* out,
                      hipStream_t st);

// kNN graph of one layer: FP32 MFMA Gram shortlist + exact re-rank + exact
// fallback for rows whose shortlist cannot be proven to hold the top R.
// Returns the number of fallback rows.
// gram: 0 = split-BF16 matrix-core tiles (d <= 128), 1 = FP32 tiles; the
// graph is the same exact kNN graph either way
int64_t build_knn_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric, int R,
                        int lpn, int cpl, int32_t* adj, int gram, hipStream_t st);

// Reverse-edge augmentation (HENN_GRAPH_KNN_SYM): rows become the first
// max_deg of the deduplicated union of out- and in-neighbours in
// (distance, id) order.
void symmetrize_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric,
                      const int32_t* adj_knn, int R, int32_t* adj_out, int max_deg, int lpn,
                      int cpl, hipStream_t st);

// Diversity pruning of C <= 32 candidates per row (ascending, -1 padded)
// to at most R kept neighbours (-1 padded), as the NSW/HNSW neighbour
// selection does.
// Delete(x): repair of a layer graph around the deleted members (del[pos] = 1),
// in place on the live rows; then the compaction of the layer.
void repair_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric,
                  const uint8_t* del, int M, int32_t* adj, int lpn, int cpl, hipStream_t st);
void launch_compact_layer(const float* vec, const int32_t* adj, const int32_t* ids,
                          const int32_t* down, const int32_t* newpos,
                          const int32_t* below_newpos, int64_t size, int dpad, int M,
                          float* vec_out, int32_t* adj_out, int32_t* ids_out, int32_t* down_out,
                          hipStream_t st);
void launch_remap_down(int32_t* down, int64_t size, const int32_t* below_newpos, hipStream_t st);

// One NSW insertion batch after its searches (res: [nb][R] positions of the
// new points [lo, lo + nb), -1 padded): writes their rows and merges the
// reverse edges into the rows of [0, lo).  Scratch: cnt and off hold lo + 1
// entries, inl nb * R.
void nsw_merge_batch(const float* vec, int dpad, int nchunks, int metric, const int32_t* res,
                     int64_t lo, int64_t nb, int R, int32_t* adj, int M, uint32_t* cnt,
                     uint32_t* off, int32_t* inl, int lpn, int cpl, hipStream_t st);
void prune_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric,
                 const int32_t* adj_in, int C, int R, int32_t* adj_out, int lpn, int cpl,
                 hipStream_t st);

// Picks (lanes per vector, chunks per lane) for a dimension.
void pick_lanes(int nchunks, int requested_lpn, int* lpn, int* cpl);

}  // namespace henn

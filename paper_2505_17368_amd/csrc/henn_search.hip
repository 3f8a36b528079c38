// henn_search.hip -- batched HENN query kernel (Alg. 4 Query, Sec. 2.2).
//
// One query per wavefront.  For each layer from the root down, the wave runs
// a beam search with list width ef_upper (1 = Alg. 4 GreedySearch) on the
// upper layers and max(ef, k) on layer 0, handing the best node down the
// inter-layer edge (Def. HENN: the same point one layer below).
//
// The beam keeps one ascending list W of (distance, id, expanded) keys in
// LDS and repeatedly expands the smallest unexpanded entry; this is the
// two-heap SEARCH-LAYER of HNSW (the candidate set the paper relies on for
// k > 1) in an equivalent form: the expansion sequence and the final list
// are identical under the strict (distance, id) order.  Visited nodes are
// remembered in a direct-mapped LDS table that may forget (never invent)
// entries; a forgotten node that comes back is either already in W (caught
// by the duplicate check) or no better than W's worst (rejected again).
//
// Per expansion: 16 neighbour ids (one 64-byte load), the visited filter,
// coalesced gathers of the fresh neighbours' rows (LPN lanes per row, each
// lane a run of CPL 8-coordinate chunks), the canonical FP32 reduction
// (henn_device.h), and a merge of the new keys into W by rank computation.
// Precision forms traverse BF16 / FP8 rows and re-rank the first
// min(|W|, rerank_factor*k) entries from the FP32 copy at the end.
//
// The library compiles this file four times: HENN_PART 0 holds the host
// functions and root-scan kernels, parts 1 / 2 / 3 the search and serving
// kernels of FP32 / BF16 / FP8 rows, so that the instantiations build in
// parallel.  Without HENN_PART one translation unit holds everything.
#include <math.h>

#include "henn_device.h"
#include "henn_internal.h"

#ifndef HENN_PART
#define HENN_PART -1
#endif
#define HENN_COMMON_PART (HENN_PART <= 0)
#define HENN_KIND_PART(kind) (HENN_PART < 0 || HENN_PART == (kind) + 1)

namespace henn {

#if HENN_COMMON_PART
size_t search_lds_per_wave(int ef_cap, int vis_bits, int vis_bytes) {
  return (size_t)ef_cap * 8 + 64 * 8 * 2 + 64 * 4 * 2 + ((size_t)1 << vis_bits) * vis_bytes;
}
#endif

// One list W, merged in place.  A merge ranks the kept keys in kstage, then
// reuses it as the map of the list positions that take a kept key.
// The fresh neighbours of an expansion, by compacted slot: crow (the row's
// first chunk index, row * chunks per row) and cidk (id << 1, the low word of
// its key).
struct WaveLds {
  uint64_t* W;
  uint64_t* ckey;     // candidate keys (by compacted slot)
  uint64_t* kstage;   // kept keys in arrival order; FP8 scales during the
                      // gather and the merge's slot map after the ranks
  uint32_t* crow;
  uint32_t* cidk;
  void* vis;  // 2^vis_bits entries: uint8 or uint16 tags, or int32 ids
};

__device__ inline WaveLds carve(char* base, int ef_cap, int vis_bits, int vis_bytes) {
  WaveLds s;
  s.W = reinterpret_cast<uint64_t*>(base);
  s.ckey = s.W + ef_cap;
  s.kstage = s.ckey + 64;
  s.crow = reinterpret_cast<uint32_t*>(s.kstage + 64);
  s.cidk = s.crow + 64;
  s.vis = s.cidk + 64;
  return s;
}

// Visited table slot and stored value of id u (see vis_tag_bytes).
__device__ inline void vis_slot(int32_t u, int bits, int vis_bytes, uint32_t& h, uint32_t& tag) {
  if (vis_bytes < 4) {
    h = (uint32_t)u & ((1u << bits) - 1u);
    tag = ((uint32_t)u >> bits) + 1u;
  } else {
    h = ((uint32_t)u * 2654435761u) >> (32 - bits);
    tag = (uint32_t)u;
  }
}
__device__ inline uint32_t vis_get(const void* vis, int vis_bytes, uint32_t h) {
  if (vis_bytes == 1) return static_cast<const uint8_t*>(vis)[h];
  if (vis_bytes == 2) return static_cast<const uint16_t*>(vis)[h];
  return static_cast<const uint32_t*>(vis)[h];
}
__device__ inline void vis_put(void* vis, int vis_bytes, uint32_t h, uint32_t tag) {
  if (vis_bytes == 1)
    static_cast<uint8_t*>(vis)[h] = (uint8_t)tag;
  else if (vis_bytes == 2)
    static_cast<uint16_t*>(vis)[h] = (uint16_t)tag;
  else
    static_cast<uint32_t*>(vis)[h] = tag;
}


// Largest power of two <= v (0 for v <= 0).
__device__ inline int pow2_floor(int v) { return v <= 0 ? 0 : 1 << (31 - __clz(v)); }

__device__ inline int next_pow2_dev(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Ascending bitonic sort of n (a power of two) keys in this wave's LDS.
__device__ inline void wave_bitonic_sort(uint64_t* A, int n) {
  const int lane = lane_id();
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = lane; i < (n >> 1); i += 64) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t x = A[lo], y = A[hi];
        if ((x > y) == asc) {
          A[lo] = y;
          A[hi] = x;
        }
      }
      wave_sync();
    }
  }
}

// One lane computes a whole distance with the same canonical order as
// group_distance: chunk sums (eight sequential FMAs), then the pairwise tree
// over P leaves, built left to right with a stack of partial sums (leaf c
// merges with the pending left siblings named by the set low bits of c).
template <int KIND, int P>
__device__ inline float serial_distance(const float (&q)[P][8], const char* row, float scale,
                                        int nchunks, int metric) {
  float stack[8];
  float v = 0.0f;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    v = 0.0f;
    if (c < nchunks) {
      float x[8];
      Chunk<KIND>::load(row, c, x);
      v = metric == 0 ? chunk_l2(q[c], x, scale, KIND == kFP8) : chunk_ip(q[c], x);
    }
#pragma unroll
    for (int l = 0; (1 << l) < P; ++l) {
      if (c & (1 << l)) {
        v = stack[l] + v;
      } else {
        stack[l] = v;
        break;
      }
    }
  }
  if (metric != 0) v = (KIND == kFP8) ? -(scale * v) : -v;
  return v;
}

// Exhaustive scan of the complete-graph root for a batch of queries: one
// thread per query (its vector in registers), root rows staged through LDS
// tiles shared by the 256 queries of a block; the root is split over
// blockIdx.y and each split writes its best (distance, position) key.
constexpr int kRootTile = 32;

template <int KIND, int P>
__global__ __launch_bounds__(256) void k_root_scan(const float* Q, int64_t nq, int d, int nchunks,
                                                   int metric, const void* rvec,
                                                   const float* rscale, int64_t rsize,
                                                   int64_t row_bytes, int64_t rows_per_split,
                                                   uint64_t* best_out) {
  extern __shared__ __align__(16) char tile[];
  float* tscale = reinterpret_cast<float*>(tile + kRootTile * row_bytes);
  const int64_t qi = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool qv = qi < nq;
  float q[P][8];
#pragma unroll
  for (int c = 0; c < P; ++c) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = c * 8 + j;
      q[c][j] = (qv && e < d) ? Q[qi * d + e] : 0.0f;
    }
  }
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < rsize ? r0 + rows_per_split : rsize;
  uint64_t best = ~0ull;
  for (int64_t rt = r0; rt < r1; rt += kRootTile) {
    const int nr = (int)(r1 - rt < kRootTile ? r1 - rt : kRootTile);
    __syncthreads();
    const uint2* src = reinterpret_cast<const uint2*>(static_cast<const char*>(rvec) + rt * row_bytes);
    uint2* dst = reinterpret_cast<uint2*>(tile);
    const int64_t nwords = (nr * row_bytes) >> 3;
    for (int64_t i = threadIdx.x; i < nwords; i += 256) dst[i] = src[i];
    if (KIND == kFP8 && (int)threadIdx.x < nr) tscale[threadIdx.x] = rscale[rt + threadIdx.x];
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
      const float sc = KIND == kFP8 ? tscale[r] : 1.0f;
      const float dist = serial_distance<KIND, P>(q, tile + r * row_bytes, sc, nchunks, metric);
      const uint64_t key = wkey(dist, (int32_t)(rt + r));
      best = key < best ? key : best;
    }
  }
  if (qv) best_out[(int64_t)blockIdx.y * nq + qi] = best;
}

#if HENN_COMMON_PART
template <int KIND>
static bool launch_root_scan_kind(const SearchArgs& a, int P, int splits, int64_t rows_per_split,
                                  uint64_t* out, hipStream_t st) {
  const SearchLayer& R = a.layer[a.num_layers - 1];
  const size_t lds = kRootTile * (size_t)R.row_bytes + kRootTile * sizeof(float);
  const dim3 grid((unsigned)((a.nq + 255) / 256), (unsigned)splits);
#define HENN_ROOT(PP)                                                                          \
  if (P == PP) {                                                                               \
    hipLaunchKernelGGL((k_root_scan<KIND, PP>), grid, dim3(256), lds, st, a.Q, a.nq, a.d,      \
                       a.nchunks, a.metric, R.vec, R.scale, (int64_t)R.size, R.row_bytes,      \
                       rows_per_split, out);                                                   \
    return true;                                                                               \
  }
  HENN_ROOT(1) HENN_ROOT(2) HENN_ROOT(4) HENN_ROOT(8) HENN_ROOT(16)
#undef HENN_ROOT
  return false;
}

int root_scan_splits(int64_t nq, int64_t root_size, int64_t* rows_per_split) {
  const int64_t qblocks = (nq + 255) / 256;
  int64_t splits = (2048 + qblocks - 1) / qblocks;
  const int64_t max_splits = (root_size + kRootTile - 1) / kRootTile;
  splits = splits < 1 ? 1 : splits > max_splits ? max_splits : splits;
  if (splits > 64) splits = 64;
  int64_t per = (root_size + splits - 1) / splits;
  per = (per + kRootTile - 1) / kRootTile * kRootTile;
  *rows_per_split = per;
  return (int)((root_size + per - 1) / per);
}

bool launch_root_scan(int storage, const SearchArgs& a, int splits, int64_t rows_per_split,
                      uint64_t* out, hipStream_t st) {
  const int P = next_pow2(a.nchunks);
  if (P > 16) return false;
  switch (storage) {
    case kF32: return launch_root_scan_kind<kF32>(a, P, splits, rows_per_split, out, st);
    case kBF16: return launch_root_scan_kind<kBF16>(a, P, splits, rows_per_split, out, st);
    case kFP8: return launch_root_scan_kind<kFP8>(a, P, splits, rows_per_split, out, st);
    default: return false;
  }
}

#endif  // HENN_COMMON_PART

// Exhaustive canonical scan of a complete-graph root by one wave (two rows
// per lane group in flight); every lane returns the best (distance,
// position) key.
template <int KIND, int LPN, int CPL>
__device__ uint64_t root_scan_wave(const SearchArgs& a, const SearchLayer& R,
                                   const float (&q)[CPL][8]) {
  constexpr int G = 64 / LPN;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  uint64_t best = ~0ull;
  for (int base = 0; base < R.size; base += 2 * G) {
    const int c0 = base + g, c1 = base + G + g;
    const bool v0 = c0 < R.size, v1 = c1 < R.size;
    const float s0 = (KIND == kFP8 && v0) ? R.scale[c0] : 1.0f;
    const float s1 = (KIND == kFP8 && v1) ? R.scale[c1] : 1.0f;
    const void* const rows[2] = {
        static_cast<const char*>(R.vec) + (int64_t)(v0 ? c0 : 0) * R.row_bytes,
        static_cast<const char*>(R.vec) + (int64_t)(v1 ? c1 : 0) * R.row_bytes};
    const float sc[2] = {s0, s1};
    const bool vd[2] = {v0, v1};
    float dd[2];
    group_distances<KIND, LPN, CPL, 2>(q, rows, sc, t, a.nchunks, a.metric, vd, dd);
    const float d0 = dd[0], d1 = dd[1];
    if (v0) {
      const uint64_t k0 = wkey(d0, c0);
      best = k0 < best ? k0 : best;
    }
    if (v1) {
      const uint64_t k1 = wkey(d1, c1);
      best = k1 < best ? k1 : best;
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const uint64_t o = shfl_xor_u64(best, m);
    best = o < best ? o : best;
  }
  return best;
}

// Exact check after the MFMA root shortlist (one query per half wave).  With
// a(y) the Gram value of root row y (BF16 products of the centred stored
// values and the centred query, FP32 accumulation, the query-norm term
// dropped) and c(y) the canonical distance, both are within an absolute
// bound of the exact distance that scales with
// N = |q - mean|^2 + max_y |y - mean|^2 + |mean|^2 (L2; uncentred for IP):
//   |a - e| <= (2^-8 + 2^-18 + (3 dpad + 35) 2^-24) N
// (each BF16 rounding is within 2^-9 relative, so a product of two is
// within 2^-8 + 2^-18 of 2 |y_k| |q_k|, which sums to at most N; the FP32
// sums add the rest), and |c - e| <= (10 + log2 chunks) 2^-23 N.  A row
// whose Gram value exceeds a_min + M, M = (2^-7 + 2^-14 + 32 (dpad + 16)
// 2^-24) N (above twice the sum of both bounds), has c(y) > c(argmin_a), so
// the nearest root member under (distance, position) is among the rows with
// a <= a_min + M.  Each split of the Gram pass listed every row within M of
// a threshold at or above a_min: so the list holds all of them unless it
// overflowed, and then the wave scans the root.
template <int KIND, int LPN, int CPL>
__global__ __launch_bounds__(256) void k_root_check(SearchArgs a, RootShortlist sl, uint64_t* out) {
  // Two queries a wave, one a half wave (lanes 0..31 and 32..63): 10,000
  // queries fit one round of resident waves.  A half holds its query's 64
  // list entries two a lane and evaluates the kept rows G at a time.
  static_assert(kRootCap == 64, "two list entries per lane of a half wave");
  static_assert(LPN <= 32, "a lane group inside a half wave");
  constexpr int G = 32 / LPN;
  const int lane = lane_id(), t = lane % LPN, hl = lane & 31, half = lane >> 5;
  const int g = hl / LPN;
  const int64_t qi = (int64_t)blockIdx.x * 8 + (threadIdx.x >> 6) * 2 + half;
  const bool qv = qi < a.nq;
  const int64_t qs = qv ? qi : 0;  // reads of a missing second query stay in bounds
  __shared__ int32_t rows_all[4][2][64];
  int32_t* rows = rows_all[threadIdx.x >> 6][half];
  const SearchLayer& R = a.layer[a.num_layers - 1];
  float q[CPL][8];
  // an overflowed list: the whole wave loads that query and scans the root
  // for it (first, so that the scan's registers are free afterwards)
  const int cnt = qv ? sl.cnt[qs] : 0;
  const bool over = cnt > kRootCap;
  const uint64_t ovm = ballot(over);
  uint64_t best_over = ~0ull;
#pragma unroll 1
  for (int hq = 0; hq < 2; ++hq) {
    if (ovm & (1ull << (32 * hq))) {
      load_query<CPL>(a.Q + (qi - half + hq) * a.d, a.d, t, q);
      const uint64_t k = root_scan_wave<KIND, LPN, CPL>(a, R, q);
      if (half == hq) best_over = k;
    }
  }
  load_query<CPL>(a.Q + qs * a.d, a.d, t, q);
  // entries past the count hold stale values (dropped)
  const uint2 e0 = sl.ent[qs * kRootCap + hl], e1 = sl.ent[qs * kRootCap + 32 + hl];
  const bool l0 = !over && hl < cnt, l1 = !over && hl + 32 < cnt;
  const float v0 = l0 ? __uint_as_float(e0.x) : INFINITY;
  const float v1 = l1 ? __uint_as_float(e1.x) : INFINITY;
  float amin = fminf(v0, v1);
#pragma unroll
  for (int m = 16; m >= 1; m >>= 1) amin = fminf(amin, __shfl_xor(amin, m));
  const float T = amin + (qv ? sl.mq[qs] : 0.0f);
  // the rows with a <= T, gathered into rows[] (first entries, then second)
  const bool k0 = l0 && v0 <= T, k1 = l1 && v1 <= T;
  const uint32_t h0 = (uint32_t)(ballot(k0) >> (32 * half));
  const uint32_t h1 = (uint32_t)(ballot(k1) >> (32 * half));
  const uint32_t below = (1u << hl) - 1u;
  const int n0 = __popc(h0), total = n0 + __popc(h1);
  wave_sync();
  if (k0) rows[__popc(h0 & below)] = (int32_t)e0.y;
  if (k1) rows[n0 + __popc(h1 & below)] = (int32_t)e1.y;
  wave_sync();
  // the longer list sets the trip count: every lane joins each butterfly
  const int tmax = max(total, __shfl_xor(total, 32));
  uint64_t best = ~0ull;
  for (int b = 0; b < tmax; b += G) {
    const int32_t row = b + g < total ? rows[b + g] : -1;
    const bool valid = row >= 0;
    const float sc = (KIND == kFP8 && valid) ? R.scale[row] : 1.0f;
    const char* rp = static_cast<const char*>(R.vec) + (int64_t)(valid ? row : 0) * R.row_bytes;
    const float dist = group_distance<KIND, LPN, CPL>(q, rp, sc, t, a.nchunks, a.metric, valid);
    if (valid) {
      const uint64_t k = wkey(dist, row);
      best = k < best ? k : best;
    }
  }
#pragma unroll
  for (int m = 16; m >= 1; m >>= 1) {
    const uint64_t o = shfl_xor_u64(best, m);
    best = o < best ? o : best;
  }
  if (over) best = best_over;
  if (qv && hl == 0) out[qi] = best;
}

// Loads this query's k and beam width and finds the entry of the first
// searched layer: the root's smallest id, or the exact root nearest when the
// root carries the complete graph (from k_root_scan's or k_root_check's keys
// when given).
template <int KIND, int LPN, int CPL>
__device__ void start_query(const SearchArgs& a, int64_t qi, const float (&q)[CPL][8],
                            QState& st) {
  constexpr int G = 64 / LPN;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  int k = uni(a.k_arr ? a.k_arr[qi] : a.k_all);
  const int ef = uni(a.ef_arr ? a.ef_arr[qi] : a.ef_all);
  k = min(max(k, 1), a.k_max);
  st.k = k;
  st.ef0 = min(max(ef, k), a.ef_cap);
  st.exps = st.evals = st.exps0 = st.evals0 = 0;
  st.need_init = 1;
  st.wsize = 0;
  int top = a.num_layers - 1;
  if (a.root_complete && top >= 1 && a.root_best) {
    // complete graph on the root, scanned by k_root_scan: min over the splits
    const SearchLayer& R = a.layer[top];
    uint64_t best = ~0ull;
    for (int sp = 0; sp < a.root_splits; ++sp) {
      const uint64_t kk = a.root_best[(int64_t)sp * a.nq + qi];
      best = kk < best ? kk : best;
    }
    best = uni_u64(best);
    st.evals = R.size;
    st.cur = uni(R.down[wkey_id(best)]);
    st.cur_d = wkey_dist(best);
    st.li = top - 1;
  } else if (a.root_complete && top >= 1) {
    // complete graph on the root: exhaustive scan for its nearest member
    const SearchLayer& R = a.layer[top];
    const uint64_t best = uni_u64(root_scan_wave<KIND, LPN, CPL>(a, R, q));
    st.evals = R.size;
    st.cur = uni(R.down[wkey_id(best)]);
    st.cur_d = wkey_dist(best);
    st.li = top - 1;
  } else {
    // entry: the smallest id of the root layer (position 0)
    const SearchLayer& R = a.layer[top];
    const float sc = (KIND == kFP8) ? R.scale[0] : 1.0f;
    float dd = group_distance<KIND, LPN, CPL>(q, R.vec, sc, t, a.nchunks, a.metric, g == 0);
    st.cur_d = uni_f(dd);  // lane 0 holds group 0's distance
    st.cur = 0;
    st.li = top;
  }
}

// Rows each lane group gathers per pass of an expansion.
constexpr int kGatherRows = 3;

// FP8 traversal distances, one chunk of 8 coordinates at a time.  The
// converter turns two codes into f16 values multiplied by a power of two:
// it takes only the exponent of its FP32 scale operand, so with the row
// scale s = 2^e m (1 <= m < 2) it yields c 2^e exactly, and t = q - m (c 2^e)
// = q - s c is one packed f16 FMA with the query rounded to f16 (qh); sum t^2
// is accumulated in FP32 by pairwise dot products (each product exact).
// Inner products convert the codes unscaled and accumulate sum q c the same
// way, the caller applying -s.  This is the precision form's arithmetic: f16
// keeps 11 significant bits against the 4 of an E4M3 code, and the final
// list is re-ranked in FP32.  Chunk sums then go through the canonical tree,
// so the result does not depend on the launch shape.
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));

template <int CPL>
__device__ inline void query_f16(const float (&q)[CPL][8], h2_t (&qh)[CPL][4]) {
#pragma unroll
  for (int i = 0; i < CPL; ++i)
#pragma unroll
    for (int k = 0; k < 4; ++k) qh[i][k] = h2_t{(_Float16)q[i][2 * k], (_Float16)q[i][2 * k + 1]};
}

// The mantissa m of a positive scale s = 2^e m, as an f16 pair.
__device__ inline h2_t scale_mantissa(float s) {
  const _Float16 m = (_Float16)__uint_as_float((__float_as_uint(s) & 0x007fffffu) | 0x3f800000u);
  return h2_t{m, m};
}

__device__ inline float fp8_chunk_l2(const uint2 w, const h2_t (&qh)[4], float s, h2_t nm) {
  const h2_t x0 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.x, s, false);
  const h2_t x1 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.x, s, true);
  const h2_t x2 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.y, s, false);
  const h2_t x3 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.y, s, true);
  // nm = -m: t = q - m x in one rounding
  const h2_t t0 = __builtin_elementwise_fma(nm, x0, qh[0]);
  const h2_t t1 = __builtin_elementwise_fma(nm, x1, qh[1]);
  const h2_t t2 = __builtin_elementwise_fma(nm, x2, qh[2]);
  const h2_t t3 = __builtin_elementwise_fma(nm, x3, qh[3]);
  float acc = __builtin_amdgcn_fdot2(t0, t0, 0.0f, false);
  acc = __builtin_amdgcn_fdot2(t1, t1, acc, false);
  acc = __builtin_amdgcn_fdot2(t2, t2, acc, false);
  return __builtin_amdgcn_fdot2(t3, t3, acc, false);
}

__device__ inline float fp8_chunk_ip(const uint2 w, const h2_t (&qh)[4]) {
  const h2_t x0 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.x, 1.0f, false);
  const h2_t x1 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.x, 1.0f, true);
  const h2_t x2 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.y, 1.0f, false);
  const h2_t x3 = __builtin_amdgcn_cvt_scalef32_pk_f16_fp8(w.y, 1.0f, true);
  float acc = __builtin_amdgcn_fdot2(qh[0], x0, 0.0f, false);
  acc = __builtin_amdgcn_fdot2(qh[1], x1, acc, false);
  acc = __builtin_amdgcn_fdot2(qh[2], x2, acc, false);
  return __builtin_amdgcn_fdot2(qh[3], x3, acc, false);
}

// One chunk's partial distance in the traversal: the canonical FP32 sum
// (henn_device.h) for FP32 and BF16 rows, the f16 form above for FP8 rows.
template <int KIND>
__device__ inline float traversal_chunk(const ChunkRaw<KIND>& raw, const float (&q)[8],
                                        const h2_t (&qh)[4], float sc, h2_t nm, int metric) {
  if constexpr (KIND == kFP8) {
    return metric == 0 ? fp8_chunk_l2(raw.a, qh, sc, nm) : fp8_chunk_ip(raw.a, qh);
  } else {
    float x[8];
    raw.decode(x);
    return metric == 0 ? chunk_l2(q, x, 1.0f, false) : chunk_ip(q, x);
  }
}

// One gather pass: rows [base, base + NR * G) of this expansion's fresh
// candidates (crow / cidk / csc), their distances, and their keys into ckey.
// FULL: the row has exactly LPN * CPL chunks, so lane t's chunks
// t * CPL .. t * CPL + CPL - 1 are contiguous and read at constant offsets
// from one pointer; otherwise chunk indices past the row are clamped to
// chunk 0 and their sums dropped (group_distances).  Every lane of the
// wave takes part (butterflies); a slot at or past cnt computes the pass's
// first row again and writes nothing.  Distances are the canonical sums of
// henn_device.h.
template <int KIND, int LPN, int CPL, int NR, bool FULL>
__device__ inline void gather_pass(const SearchArgs& a, const SearchLayer& L,
                                   const float (&q)[CPL][8], const h2_t (&qh)[CPL][4],
                                   const WaveLds& s, const float* csc, int base, int cnt, int t,
                                   int g) {
  constexpr int G = 64 / LPN;
  constexpr int CB = KIND == kF32 ? 32 : KIND == kBF16 ? 16 : 8;  // bytes per chunk
  const char* vec = static_cast<const char*>(L.vec);
  const void* rows[NR];
  float sc[NR];
  bool vd[NR];
  uint32_t idk[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int ci = base + r * G + g;
    vd[r] = ci < cnt;
    // an empty slot re-reads the pass's first row, which its group reads anyway
    const int e = vd[r] ? ci : base;
    const uint32_t ch = s.crow[e] + (FULL ? (uint32_t)(t * CPL) : 0u);
    rows[r] = vec + (size_t)ch * CB;
    idk[r] = s.cidk[e];
    sc[r] = (KIND == kFP8) ? csc[e] : 1.0f;
  }
  // FP8: minus the mantissa of each row's scale (fp8_chunk_l2)
  h2_t nm[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) nm[r] = (KIND == kFP8) ? -scale_mantissa(sc[r]) : h2_t{0, 0};
  // this lane's chunk sums of each row (tree over its CPL chunks)
  float ts[NR];
  if constexpr (FULL) {
    ChunkRaw<KIND> raw[NR][CPL];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < CPL; ++i) raw[r][i].fetch(rows[r], i);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      float part[CPL];
#pragma unroll
      for (int i = 0; i < CPL; ++i)
        part[i] = traversal_chunk<KIND>(raw[r][i], q[i], qh[i], sc[r], nm[r], a.metric);
      ts[r] = tree_sum<CPL>(part);
    }
  } else {
    ChunkRaw<KIND> raw[NR][CPL];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < CPL; ++i) {
        const int c = t * CPL + i;
        raw[r][i].fetch(rows[r], c < a.nchunks ? c : 0);
      }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      float part[CPL];
#pragma unroll
      for (int i = 0; i < CPL; ++i) {
        const int c = t * CPL + i;
        const float v = traversal_chunk<KIND>(raw[r][i], q[i], qh[i], sc[r], nm[r], a.metric);
        part[i] = c < a.nchunks ? v : 0.0f;
      }
      ts[r] = tree_sum<CPL>(part);
    }
  }
  // lane-group sums; rows 2p and 2p + 1 share one butterfly
  // (group_distances_paired): the even lanes of a group end with row 2p's
  // sum, the odd lanes with row 2p + 1's
  constexpr int NP = (LPN >= 2) ? NR / 2 : 0;  // row pairs
  const bool odd = (lane_id() & 1) != 0;
  float d[NR];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    float v = (odd ? ts[2 * p + 1] : ts[2 * p]) + dpp_mov<0xB1>(odd ? ts[2 * p] : ts[2 * p + 1]);
    d[2 * p] = group_sum_from2<LPN>(v);
  }
#pragma unroll
  for (int r = 2 * NP; r < NR; ++r) d[r] = group_sum<LPN>(ts[r]);
  // keys: (ordered distance bits << 32) | (id << 1).  Squared L2 distances
  // are sums of squares, never negative or -0, so their ordered bits are
  // the float bits with the sign bit set (ordered_bits on that range).
  auto key_of = [&](float dist, float scale, uint32_t idk_) -> uint64_t {
    uint32_t ob;
    if (a.metric == 0) {
      ob = __float_as_uint(dist) | 0x80000000u;
    } else {
      ob = ordered_bits((KIND == kFP8) ? -(scale * dist) : -dist);
    }
    return ((uint64_t)ob << 32) | idk_;
  };
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const int r = 2 * p + (odd ? 1 : 0);
    if (t < 2 && vd[r]) s.ckey[base + r * G + g] = key_of(d[2 * p], sc[r], idk[r]);
  }
#pragma unroll
  for (int r = 2 * NP; r < NR; ++r)
    if (t == 0 && vd[r]) s.ckey[base + r * G + g] = key_of(d[r], sc[r], idk[r]);
}

// All gather passes of one expansion, each with every load of its rows in
// flight together: up to kGatherRows * G rows per pass, the last pass sized
// to the rows left.
template <int KIND, int LPN, int CPL, bool FULL>
__device__ inline void gather_all(const SearchArgs& a, const SearchLayer& L,
                                  const float (&q)[CPL][8], const h2_t (&qh)[CPL][4],
                                  const WaveLds& s, const float* csc, int cnt, int t, int g) {
  constexpr int G = 64 / LPN;
  static_assert(kGatherRows == 3, "pass sizes below");
  for (int base = 0; base < cnt;) {
    const int rest = cnt - base;
    if (rest > 2 * G) {
      gather_pass<KIND, LPN, CPL, 3, FULL>(a, L, q, qh, s, csc, base, cnt, t, g);
      base += 3 * G;
    } else if (rest > G) {
      gather_pass<KIND, LPN, CPL, 2, FULL>(a, L, q, qh, s, csc, base, cnt, t, g);
      base += 2 * G;
    } else {
      gather_pass<KIND, LPN, CPL, 1, FULL>(a, L, q, qh, s, csc, base, cnt, t, g);
      base += G;
    }
  }
}

// Runs up to `budget` expansions from the current state (layer changes are
// free).  Returns true once the layer-0 beam has no unexpanded entry; then
// W (this wave's LDS list) holds the final list (st.wsize entries).  q: this
// lane's FP32 query slice; qh: the same in f16 pairs (read by the FP8 form
// only, which then never reads q).
template <int KIND, int LPN, int CPL, bool FULL, bool EXACT = false>
__device__ bool advance(const SearchArgs& a, const float (&q)[CPL][8], const h2_t (&qh)[CPL][4],
                        WaveLds s, uint64_t* W, QState& st, int budget, uint32_t* vis_bm) {
  constexpr int G = 64 / LPN;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  const int vis_n = 1 << a.vis_bits;
  for (;;) {
    const SearchLayer L = a.layer[st.li];
    const int efl = st.li == 0 ? st.ef0 : min(a.ef_upper, a.ef_cap);
    if (st.need_init) {
      if (st.li == 0) {
        st.exps0 = st.exps;
        st.evals0 = st.evals;
      }
      st.evals += 1;  // the entry (its distance is carried down, counted per layer)
      if constexpr (EXACT) {
        // the exact set: one bit per member of the layer, in the workspace
        const int64_t words = ((int64_t)L.size + 31) >> 5;
        for (int64_t i = lane; i < words; i += 64) vis_bm[i] = 0u;
        __builtin_amdgcn_s_waitcnt(0);  // cleared before the first bit is set
      } else {
        // empty: tag 0 (8 / 16-bit) or id -1 (32-bit); cleared as 32-bit words
        const int vis_words = vis_n * a.vis_bytes / 4;
        const uint32_t empty = a.vis_bytes < 4 ? 0u : 0xffffffffu;
        for (int i = lane; i < vis_words; i += 64) static_cast<uint32_t*>(s.vis)[i] = empty;
      }
      if constexpr (KIND == kFP8) {
        // the entry's distance in the traversal's own form: the one handed
        // down (a root scan, or the first distance of the root) is the
        // canonical FP32 sum, and the list's duplicate check compares keys
        if (lane == 0) {
          s.crow[0] = (uint32_t)st.cur * (uint32_t)a.nchunks;
          s.cidk[0] = (uint32_t)st.cur << 1;
          reinterpret_cast<float*>(s.kstage)[0] = L.scale[st.cur];
        }
        wave_sync();
        gather_pass<KIND, LPN, CPL, 1, FULL>(a, L, q, qh, s, reinterpret_cast<float*>(s.kstage),
                                             0, 1, t, g);
        wave_sync();
        st.cur_d = wkey_dist(uni_u64(s.ckey[0]));
      }
      wave_sync();
      if (lane == 0) {
        W[0] = wkey(st.cur_d, st.cur);
        if constexpr (EXACT) {
          atomicOr(vis_bm + (st.cur >> 5), 1u << (st.cur & 31));
        } else {
          uint32_t h0, t0;
          vis_slot(st.cur, a.vis_bits, a.vis_bytes, h0, t0);
          vis_put(s.vis, a.vis_bytes, h0, t0);
        }
      }
      st.wsize = 1;
      st.need_init = 0;
      wave_sync();
    }
    int wsize = st.wsize;
    bool layer_done = false;
    while (budget > 0) {
      // smallest unexpanded entry of W
      int pos = -1;
      for (int base = 0; base < wsize; base += 64) {
        const int i = base + lane;
        const bool un = i < wsize && !(W[i] & 1ull);
        const uint64_t m = ballot(un);
        if (m) {
          pos = base + __ffsll((unsigned long long)m) - 1;
          break;
        }
      }
      if (pos < 0) {
        layer_done = true;
        break;
      }
      --budget;
      const uint64_t ck = uni_u64(W[pos]);
      wave_sync();
      if (lane == 0) W[pos] = ck | 1ull;
      const int32_t c = wkey_id(ck);
      ++st.exps;

      // neighbour ids (and, for FP8 rows, their scales) and the visited filter
      int32_t u = -1;
      float usc = 1.0f;
      if (lane < L.deg) {
        u = L.adj[(int64_t)c * L.deg + lane];
        if (KIND == kFP8) usc = L.adj_scale[(int64_t)c * L.deg + lane];
      }
      bool fresh = false;
      if constexpr (EXACT) {
        // exact set: the bit's old value says whether u was seen (the
        // update is atomic, so of lanes holding one id only one finds it new)
        if (u >= 0) {
          const uint32_t bit = 1u << (u & 31);
          fresh = !(atomicOr(vis_bm + (u >> 5), bit) & bit);
        }
      } else {
        uint32_t h = 0, tag = 0;
        if (u >= 0) {
          vis_slot(u, a.vis_bits, a.vis_bytes, h, tag);
          fresh = vis_get(s.vis, a.vis_bytes, h) != tag;
        }
        wave_sync();
        if (fresh) vis_put(s.vis, a.vis_bytes, h, tag);
      }
      const uint64_t fm = ballot(fresh);
      const int cnt = popc64(fm);
      // the scales ride in kstage, which is free until the merge below
      float* csc = reinterpret_cast<float*>(s.kstage);
      if (fresh) {
        const int rb = rank_below(fm);
        s.crow[rb] = (uint32_t)u * (uint32_t)a.nchunks;
        s.cidk[rb] = (uint32_t)u << 1;
        if (KIND == kFP8) csc[rb] = usc;
      }
      wave_sync();
      st.evals += cnt;

      // gather + distance
      gather_all<KIND, LPN, CPL, FULL>(a, L, q, qh, s, csc, cnt, t, g);
      wave_sync();

      // merge the new keys into W (truncated to efl)
      const uint64_t key = lane < cnt ? s.ckey[lane] : ~0ull;
      bool keep = lane < cnt;
      if (keep && wsize >= efl) keep = key < wkey_strip(W[efl - 1]);
      // nothing can enter a full list: skip the merge (common late in a search)
      if (!ballot(keep)) continue;
      // lo = number of W entries below key (fixed-step lower bound: the trip
      // count depends only on the wave-uniform list size)
      int lo = 0;
      for (int step = pow2_floor(wsize); step > 0; step >>= 1)
        if (lo + step <= wsize && wkey_strip(W[lo + step - 1]) < key) lo += step;
      if (keep && lo < wsize && wkey_strip(W[lo]) == key) keep = false;  // already in W
      const uint64_t km = ballot(keep);
      const int nk = popc64(km);
      if (nk == 0) continue;
      if (keep) s.kstage[rank_below(km)] = key;
      // pad to a multiple of 4 (at most 64 slots) with keys below which
      // nothing ranks, so the count below reads four keys per step
      const int nk4 = (nk + 3) & ~3;
      if (lane >= nk && lane < nk4) s.kstage[lane] = ~0ull;
      wave_sync();
      int rk = 0;  // kept keys below this one
      if (keep)
        for (int j = 0; j < nk4; j += 4)
          rk += (s.kstage[j] < key) + (s.kstage[j + 1] < key) + (s.kstage[j + 2] < key) +
                (s.kstage[j + 3] < key);
      // a kept key lands at p = lo + rk: the p are distinct and ascend with
      // the key; the entries below the smallest stay where they are
      const int p = lo + rk;
      const uint64_t m0 = ballot(keep && rk == 0);
      const int lo_min = uni(__shfl(lo, __ffsll((unsigned long long)m0) - 1));
      const int nsize = min(efl, wsize + nk);
      wave_sync();
      // slot map (in kstage, free again): bit x of word x >> 6 marks the
      // positions that take a kept key; nsize <= 2048 needs at most 32 words.
      // The words are cleared as 32-bit halves: a 64-bit zero is otherwise
      // kept live in two registers through the whole expansion loop.
      uint64_t* slot = s.kstage;
      const int w0 = lo_min >> 6;
      if (lane <= ((nsize - 1) >> 6) - w0) {
        uint32_t* sw = reinterpret_cast<uint32_t*>(slot + w0 + lane);
        sw[0] = 0u;
        sw[1] = 0u;
      }
      wave_sync();
      if (keep && p < nsize) atomicOr(reinterpret_cast<unsigned long long*>(&slot[p >> 6]),
                                      1ull << (p & 63));
      wave_sync();
      // in place, by output position: a position x in [lo_min, nsize) that
      // takes no key takes W[x - K(x)], K(x) the key positions below x.  The
      // source never lies above x, so blocks of 64 go from the top down and
      // each reads its sources whole before it writes.
      int kb = popc64(ballot(keep && p < nsize));  // then: key positions below block b
      for (int b = (nsize - 1) & ~63; b >= 0 && b + 64 > lo_min; b -= 64) {
        const int x = b + lane;
        const uint64_t mask = uni_u64(slot[b >> 6]);
        kb -= popc64(mask);
        const int below = rank_below(mask);
        const int kx = kb + below;
        // x takes a key when the count through this lane exceeds the one
        // below (counted, not tested as mask & (1 << lane): that lane mask
        // would stay live in two registers)
        const bool is_key = rank_below(mask >> 1) + (int)(mask & 1ull) != below;
        const bool mv = x >= lo_min && x < nsize && !is_key && kx > 0;
        uint64_t wv = 0;
        if (mv) wv = W[x - kx];
        wave_sync();
        if (mv) W[x] = wv;
        wave_sync();
      }
      if (keep && p < nsize) W[p] = key;
      wave_sync();
      wsize = nsize;
    }
    st.wsize = wsize;
    if (!layer_done) return false;
    if (st.li == 0) return true;
    // hand the best node down the inter-layer edge
    const uint64_t best = uni_u64(W[0]);
    st.cur = uni(L.down[wkey_id(best)]);
    st.cur_d = wkey_dist(best);
    st.li -= 1;
    st.need_init = 1;
    wave_sync();
  }
}

// Writes the first k results (after the FP32 re-rank for the precision
// forms) to out_ids / out_dist (k_max entries, padded) and the counters.
template <int KIND, int LPN, int CPL>
__device__ void finish_query(const SearchArgs& a, const float (&q)[CPL][8], uint64_t* W,
                             const QState& st, int32_t* out_ids, float* out_dist,
                             int32_t* counters) {
  constexpr int G = 64 / LPN;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  const int k = st.k, wsize = st.wsize;
  if (a.rerank_vec == nullptr) {
    for (int j = lane; j < a.k_max; j += 64) {
      int32_t id = -1;
      float dd = INFINITY;
      if (j < k && j < wsize) {
        id = wkey_id(W[j]);
        dd = wkey_dist(W[j]);
        if (a.ids0) id = a.ids0[id];
      }
      out_ids[j] = id;
      out_dist[j] = dd;
    }
  } else {
    // FP32 re-rank of the first min(|W|, rerank_factor*k) entries
    const int nr = min(wsize, a.rerank_factor * k);
    for (int base = 0; base < nr; base += G) {
      const int ci = base + g;
      const bool valid = ci < nr;
      const int32_t id = valid ? wkey_id(W[ci]) : 0;
      const float dist = group_distance<kF32, LPN, CPL>(
          q, a.rerank_vec + (int64_t)id * a.dpad, 1.0f, t, a.nchunks, a.metric, valid);
      // in place: a group reads its entry before the distance and writes it after
      if (valid && t == 0) W[ci] = wkey(dist, id);
    }
    const int n2 = next_pow2_dev(nr);
    for (int i = nr + lane; i < n2; i += 64) W[i] = ~0ull;
    wave_sync();
    wave_bitonic_sort(W, n2);
    for (int j = lane; j < a.k_max; j += 64) {
      int32_t id = -1;
      float dd = INFINITY;
      if (j < k && j < nr) {
        id = wkey_id(W[j]);
        dd = wkey_dist(W[j]);
        if (a.ids0) id = a.ids0[id];
      }
      out_ids[j] = id;
      out_dist[j] = dd;
    }
  }
  if (counters && lane == 0) {
    counters[0] = st.exps;
    counters[1] = st.evals;
    counters[2] = st.exps - st.exps0;
    counters[3] = st.evals - st.evals0;
  }
  wave_sync();
}

// The per-query time output, read from the kernel's argument segment at the
// point of use (SearchArgs is the first argument of every kernel that calls
// search_one, so it starts the segment).  A volatile read: the traversal keeps
// its scalar registers full, and a pointer held across it would spill.
__device__ __forceinline__ int64_t* query_ns_arg() {
  const SearchArgs* ka = reinterpret_cast<const SearchArgs*>(
      (const char*)__builtin_amdgcn_kernarg_segment_ptr());
  return *reinterpret_cast<int64_t* const volatile*>(&ka->query_ns);
}

template <int KIND, int LPN, int CPL, bool FULL, bool EXACT>
__device__ void search_one(const SearchArgs& a, int64_t qi, WaveLds s) {
  // the constant-rate clock when times are asked for; the start waits in the
  // query's output word (volatile: a memory round trip, so no register stays
  // live across the traversal)
  if (lane_id() == 0) {
    int64_t* qt = query_ns_arg();
    if (qt) *reinterpret_cast<volatile int64_t*>(qt + qi) = (int64_t)wall_clock64();
  }
  const int t = lane_id() % LPN;
  float q[CPL][8];
  load_query<CPL>(a.Q + qi * a.d, a.d, t, q);
  QState st;
  start_query<KIND, LPN, CPL>(a, qi, q, st);
  h2_t qh[CPL][4];
  if constexpr (KIND == kFP8) query_f16<CPL>(q, qh);
  uint64_t* W = s.W;
  uint32_t* vis_bm = EXACT ? a.vis_exact + qi * a.vis_exact_words : nullptr;
  advance<KIND, LPN, CPL, FULL, EXACT>(a, q, qh, s, W, st, 0x7fffffff, vis_bm);
  // the FP8 traversal holds only the f16 query; the FP32 re-rank reads it again
  if constexpr (KIND == kFP8) load_query<CPL>(a.Q + qi * a.d, a.d, t, q);
  finish_query<KIND, LPN, CPL>(a, q, W, st, a.out_ids + qi * a.k_max,
                               a.out_dist + qi * a.k_max,
                               a.counters ? a.counters + qi * 4 : nullptr);
  int64_t* qt = lane_id() == 0 ? query_ns_arg() : nullptr;
  if (qt) {
    volatile int64_t* slot = reinterpret_cast<volatile int64_t*>(qt + qi);
    const uint32_t ticks = (uint32_t)((uint64_t)wall_clock64() - (uint64_t)*slot);
    *slot = (int64_t)((double)ticks * a.clock_ns);
  }
}

// ---------------------------------------------------------- serving ------
// One tick of the serving form: every active slot advances by at most
// `budget` expansions.  A slot's state (QState, its list W and visited
// table) lives in HBM between ticks at arena + state_off[slot]; it is
// loaded into this wave's LDS, advanced, and stored back.  A slot that
// finishes appends its slot and result row to the tick's compact completion
// list.  The traversal is the batch kernel's own code, so
// a request's result does not depend on which others share its ticks.
template <int KIND, int LPN, int CPL, bool FULL>
__device__ __forceinline__ void serve_step_body(const SearchArgs& a, const ServeArgs& sv,
                                                int per_wave_bytes, int waves_per_block) {
  extern __shared__ __align__(16) char smem[];
  const int wave = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * waves_per_block + wave;
  if (blockIdx.x == 0 && threadIdx.x == 0) *sv.done_clear = 0;
  if (idx >= sv.n_active) return;
  const int lane = lane_id(), t = lane % LPN;
  const int32_t slot = uni(sv.active[idx]);
  WaveLds s = carve(smem + (size_t)wave * per_wave_bytes, a.ef_cap, a.vis_bits, a.vis_bytes);
  float q[CPL][8];
  load_query<CPL>(a.Q + (int64_t)slot * a.d, a.d, t, q);
  QState st = sv.states[slot];
  st.li = uni(st.li);
  st.need_init = uni(st.need_init);
  st.wsize = uni(st.wsize);
  st.cur = uni(st.cur);
  st.cur_d = uni_f(st.cur_d);
  st.k = uni(st.k);
  st.ef0 = uni(st.ef0);
  char* base = sv.arena + sv.state_off[slot];
  uint64_t* gW = reinterpret_cast<uint64_t*>(base);
  uint32_t* gvis = reinterpret_cast<uint32_t*>(base + (size_t)sv.cap[slot] * 8);
  const int vis_n = (1 << a.vis_bits) * a.vis_bytes / 4;  // 32-bit words of the table
  if (st.li == kSlotNew) {
    start_query<KIND, LPN, CPL>(a, slot, q, st);
  } else if (!st.need_init) {
    for (int i = lane; i < st.wsize; i += 64) s.W[i] = gW[i];
    for (int i = lane; i < vis_n; i += 64) static_cast<uint32_t*>(s.vis)[i] = gvis[i];
    wave_sync();
  }
  uint64_t* W = s.W;
  h2_t qh[CPL][4];
  if constexpr (KIND == kFP8) query_f16<CPL>(q, qh);
  const bool done = advance<KIND, LPN, CPL, FULL>(a, q, qh, s, W, st, sv.budget, nullptr);
  if (done) {
    if constexpr (KIND == kFP8) load_query<CPL>(a.Q + (int64_t)slot * a.d, a.d, t, q);
    // finished: append (slot, row) to this tick's compact completion list
    int pos = 0;
    if (lane == 0) pos = atomicAdd(sv.done_count, 1);
    pos = __shfl(pos, 0);
    int32_t* row = sv.done_rows + (int64_t)pos * (1 + 2 * a.k_max);
    finish_query<KIND, LPN, CPL>(a, q, W, st, row + 1,
                                 reinterpret_cast<float*>(row + 1 + a.k_max), nullptr);
    st.li = kSlotDone;
    if (lane == 0) row[0] = slot;
  } else if (!st.need_init) {
    for (int i = lane; i < st.wsize; i += 64) gW[i] = W[i];
    for (int i = lane; i < vis_n; i += 64) gvis[i] = static_cast<uint32_t*>(s.vis)[i];
  }
  if (lane == 0) sv.states[slot] = st;
}

template <int KIND, int LPN, int CPL, bool FULL>
__global__ __launch_bounds__(512) void k_serve_step(SearchArgs a, ServeArgs sv, int per_wave_bytes,
                                                    int waves_per_block) {
  serve_step_body<KIND, LPN, CPL, FULL>(a, sv, per_wave_bytes, waves_per_block);
}

// The FP8 form with at most two chunks per lane fits 80 registers without
// spilling in the traversal loop; held to that, six waves share a SIMD (the
// LDS of a wave at the usual beam widths also allows six).
template <int KIND, int CPL>
constexpr bool six_waves() { return KIND == kFP8 && CPL <= 2; }

template <int KIND, int LPN, int CPL, bool FULL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6))) void k_serve_step6(
    SearchArgs a, ServeArgs sv, int per_wave_bytes, int waves_per_block) {
  serve_step_body<KIND, LPN, CPL, FULL>(a, sv, per_wave_bytes, waves_per_block);
}

template <int KIND, int LPN, int CPL, bool FULL>
static auto serve_kernel() {
  if constexpr (six_waves<KIND, CPL>())
    return &k_serve_step6<KIND, LPN, CPL, FULL>;
  else
    return &k_serve_step<KIND, LPN, CPL, FULL>;
}

static __global__ void k_serve_admit(const float* staged_q, const int32_t* meta, int n_new, int d,
                              float* slot_q, int32_t* slot_k, int32_t* slot_ef,
                              int64_t* state_off, int32_t* cap, QState* states,
                              const uint64_t* root_keys, uint64_t* slot_root) {
  // meta per new request: slot, k, ef, cap, offset (lo, hi)
  const int r = blockIdx.x;
  if (r >= n_new) return;
  const int32_t* m = meta + r * 6;
  const int32_t slot = m[0];
  for (int j = threadIdx.x; j < d; j += blockDim.x)
    slot_q[(int64_t)slot * d + j] = staged_q[(int64_t)r * d + j];
  if (threadIdx.x == 0) {
    slot_k[slot] = m[1];
    slot_ef[slot] = m[2];
    cap[slot] = m[3];
    state_off[slot] = (int64_t)(((uint64_t)(uint32_t)m[5] << 32) | (uint32_t)m[4]);
    QState st;
    memset(&st, 0, sizeof(st));
    st.li = kSlotNew;
    states[slot] = st;
    if (root_keys) slot_root[slot] = root_keys[r];
  }
}

template <int KIND, int LPN, int CPL, bool FULL>
static void launch_serve_one(const SearchArgs& a, const ServeArgs& sv, int wpb, hipStream_t st) {
  const size_t per_wave = search_lds_per_wave(a.ef_cap, a.vis_bits, a.vis_bytes);
  const unsigned blocks = (unsigned)((sv.n_active + wpb - 1) / wpb);
  auto kern = serve_kernel<KIND, LPN, CPL, FULL>();
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), per_wave * wpb, st, a, sv,
                     (int)per_wave, wpb);
}

template <int KIND, int LPN, int CPL, bool FULL, bool EXACT>
__device__ __forceinline__ void search_kernel_body(const SearchArgs& a, int per_wave_bytes,
                                                   int waves_per_block, int persistent) {
  extern __shared__ __align__(16) char smem[];
  const int wave = threadIdx.x >> 6;
  WaveLds s = carve(smem + (size_t)wave * per_wave_bytes, a.ef_cap, a.vis_bits, a.vis_bytes);
  if (persistent) {
    for (;;) {
      uint32_t qi = 0;
      if (lane_id() == 0) qi = atomicAdd(a.work_counter, 1u);
      qi = (uint32_t)uni((int32_t)qi);
      if ((int64_t)qi >= a.nq) break;
      search_one<KIND, LPN, CPL, FULL, EXACT>(a, (int64_t)qi, s);
    }
  } else {
    const int64_t qi = (int64_t)blockIdx.x * waves_per_block + wave;
    if (qi < a.nq) search_one<KIND, LPN, CPL, FULL, EXACT>(a, qi, s);
  }
}

template <int KIND, int LPN, int CPL, bool FULL, bool EXACT = false>
__global__ __launch_bounds__(512) void k_search(SearchArgs a, int per_wave_bytes,
                                                int waves_per_block, int persistent) {
  search_kernel_body<KIND, LPN, CPL, FULL, EXACT>(a, per_wave_bytes, waves_per_block, persistent);
}

// The same kernel held to 80 registers (see six_waves).
template <int KIND, int LPN, int CPL, bool FULL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6))) void k_search6(
    SearchArgs a, int per_wave_bytes, int waves_per_block, int persistent) {
  search_kernel_body<KIND, LPN, CPL, FULL, false>(a, per_wave_bytes, waves_per_block, persistent);
}

template <int KIND, int LPN, int CPL, bool FULL>
static auto search_kernel(bool exact) {
  // the exact visited set (an analysis form) runs the general-width kernel
  if (exact) return &k_search<KIND, LPN, CPL, false, true>;
  if constexpr (six_waves<KIND, CPL>())
    return &k_search6<KIND, LPN, CPL, FULL>;
  else
    return &k_search<KIND, LPN, CPL, FULL>;
}

static __global__ void k_reset_counter(uint32_t* c) { *c = 0u; }

template <int KIND, int LPN, int CPL, bool FULL>
static void launch_one(const SearchArgs& a, const LaunchShape& sh, hipStream_t st) {
  const size_t per_wave = search_lds_per_wave(a.ef_cap, a.vis_bits, a.vis_bytes);
  const int wpb = sh.waves_per_block;
  const size_t lds = per_wave * wpb;
  auto kern = search_kernel<KIND, LPN, CPL, FULL>(a.vis_exact != nullptr);
  if (sh.persistent) {
    int blocks = sh.blocks;
    if (blocks <= 0) {
      int dev = 0, cus = 0, per_cu = 0;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(kern), 64 * wpb, lds);
      blocks = max(1, cus * max(per_cu, 1));
    }
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, a.work_counter);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), lds, st, a, (int)per_wave, wpb, 1);
  } else {
    const int64_t blocks = (a.nq + wpb - 1) / wpb;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a, (int)per_wave,
                       wpb, 0);
  }
}

#define HENN_SEARCH_COMBOS(X) \
  X(1, 1) X(2, 1) X(4, 1) X(2, 2) X(4, 2) X(8, 1) X(2, 4) X(4, 4) X(8, 2) X(16, 1) X(8, 4) \
  X(16, 2) X(4, 8) X(16, 4) X(16, 8)

template <int KIND>
static bool dispatch(const SearchArgs& a, const LaunchShape& sh, hipStream_t st) {
#define HENN_TRY(LPN, CPL)                              \
  if (sh.lanes_per_vec == LPN && sh.chunks_per_lane == CPL) { \
    if (a.nchunks == LPN * CPL)                         \
      launch_one<KIND, LPN, CPL, true>(a, sh, st);      \
    else                                                \
      launch_one<KIND, LPN, CPL, false>(a, sh, st);     \
    return true;                                        \
  }
  HENN_SEARCH_COMBOS(HENN_TRY)
#undef HENN_TRY
  return false;
}

#if HENN_COMMON_PART
// The gather addresses a row by its 32-bit first-chunk index.
bool rows_addressable(const SearchArgs& a) {
  for (int i = 0; i < a.num_layers; ++i)
    if ((int64_t)a.layer[i].size * a.nchunks >= (1ll << 32)) return false;
  return true;
}
#endif

#if HENN_KIND_PART(0)  // kF32
bool launch_search_f32(const SearchArgs& a, const LaunchShape& s, hipStream_t st) {
  return dispatch<kF32>(a, s, st);
}
#endif
#if HENN_KIND_PART(1)  // kBF16
bool launch_search_bf16(const SearchArgs& a, const LaunchShape& s, hipStream_t st) {
  return dispatch<kBF16>(a, s, st);
}
#endif
#if HENN_KIND_PART(2)  // kFP8
bool launch_search_fp8(const SearchArgs& a, const LaunchShape& s, hipStream_t st) {
  return dispatch<kFP8>(a, s, st);
}
#endif

template <int KIND>
static bool dispatch_serve(const SearchArgs& a, const ServeArgs& sv, const LaunchShape& sh,
                           hipStream_t st) {
#define HENN_TRY(LPN, CPL)                                        \
  if (sh.lanes_per_vec == LPN && sh.chunks_per_lane == CPL) {     \
    if (a.nchunks == LPN * CPL)                                   \
      launch_serve_one<KIND, LPN, CPL, true>(a, sv, sh.waves_per_block, st);  \
    else                                                          \
      launch_serve_one<KIND, LPN, CPL, false>(a, sv, sh.waves_per_block, st); \
    return true;                                                  \
  }
  HENN_SEARCH_COMBOS(HENN_TRY)
#undef HENN_TRY
  return false;
}

#if HENN_KIND_PART(0)  // kF32
bool launch_serve_f32(const SearchArgs& a, const ServeArgs& sv, const LaunchShape& sh,
                      hipStream_t st) {
  return dispatch_serve<kF32>(a, sv, sh, st);
}
#endif
#if HENN_KIND_PART(1)  // kBF16
bool launch_serve_bf16(const SearchArgs& a, const ServeArgs& sv, const LaunchShape& sh,
                       hipStream_t st) {
  return dispatch_serve<kBF16>(a, sv, sh, st);
}
#endif
#if HENN_KIND_PART(2)  // kFP8
bool launch_serve_fp8(const SearchArgs& a, const ServeArgs& sv, const LaunchShape& sh,
                      hipStream_t st) {
  return dispatch_serve<kFP8>(a, sv, sh, st);
}
#endif

#if HENN_COMMON_PART
bool launch_search(int storage, const SearchArgs& a, const LaunchShape& s, hipStream_t st) {
  if (!rows_addressable(a)) return false;
  switch (storage) {
    case kF32: return launch_search_f32(a, s, st);
    case kBF16: return launch_search_bf16(a, s, st);
    case kFP8: return launch_search_fp8(a, s, st);
    default: return false;
  }
}

bool launch_serve_step(int storage, const SearchArgs& a, const ServeArgs& sv,
                       const LaunchShape& sh, hipStream_t st) {
  if (sv.n_active <= 0) return true;
  if (!rows_addressable(a)) return false;
  switch (storage) {
    case kF32: return launch_serve_f32(a, sv, sh, st);
    case kBF16: return launch_serve_bf16(a, sv, sh, st);
    case kFP8: return launch_serve_fp8(a, sv, sh, st);
    default: return false;
  }
}

void launch_serve_admit(const float* staged_q, const int32_t* meta, int n_new, int d,
                        float* slot_q, int32_t* slot_k, int32_t* slot_ef, int64_t* state_off,
                        int32_t* cap, QState* states, const uint64_t* root_keys,
                        uint64_t* slot_root, hipStream_t st) {
  if (n_new <= 0) return;
  hipLaunchKernelGGL(k_serve_admit, dim3(n_new), dim3(64), 0, st, staged_q, meta, n_new, d,
                     slot_q, slot_k, slot_ef, state_off, cap, states, root_keys, slot_root);
}

template <int KIND>
static bool launch_root_check_kind(const SearchArgs& a, const RootShortlist& sl, uint64_t* out,
                                   hipStream_t st) {
  int lpn = 0, cpl = 0;
  pick_lanes(a.nchunks, 0, &lpn, &cpl);
  const dim3 grid((unsigned)((a.nq + 7) / 8));  // eight queries a block
#define HENN_TRY(L, C)                                                                       \
  if (lpn == L && cpl == C) {                                                                \
    hipLaunchKernelGGL((k_root_check<KIND, L, C>), grid, dim3(256), 0, st, a, sl, out);         \
    return true;                                                                             \
  }
  HENN_TRY(1, 1) HENN_TRY(2, 1) HENN_TRY(4, 1) HENN_TRY(2, 2) HENN_TRY(4, 2) HENN_TRY(8, 1)
  HENN_TRY(2, 4) HENN_TRY(4, 4) HENN_TRY(8, 2) HENN_TRY(16, 1)
#undef HENN_TRY
  return false;
}

bool launch_root_check(int storage, const SearchArgs& a, const RootShortlist& sl, uint64_t* out,
                       hipStream_t st) {
  if (a.nq <= 0) return true;
  switch (storage) {
    case kF32: return launch_root_check_kind<kF32>(a, sl, out, st);
    case kBF16: return launch_root_check_kind<kBF16>(a, sl, out, st);
    case kFP8: return launch_root_check_kind<kFP8>(a, sl, out, st);
    default: return false;
  }
}

void pick_lanes(int nchunks, int requested_lpn, int* lpn, int* cpl) {
  const int P = next_pow2(nchunks);
  // instantiated (LPN, CPL) pairs with LPN * CPL == P
  static const int combos[][2] = {{1, 1}, {2, 1},  {4, 1},  {2, 2}, {4, 2},  {8, 1},
                                  {2, 4}, {4, 4},  {8, 2},  {16, 1}, {8, 4},  {16, 2},
                                  {4, 8}, {16, 4}, {16, 8}};
  int best_l = 0, best_c = 0;
  for (auto& c : combos) {
    if (c[0] * c[1] != P) continue;
    if (requested_lpn > 0) {
      if (c[0] == requested_lpn) { best_l = c[0]; best_c = c[1]; }
      continue;
    }
    // default: the fewest lanes with at most 4 chunks per lane
    if (best_l == 0 || (c[1] <= 4 && (best_c > 4 || c[0] < best_l))) {
      best_l = c[0];
      best_c = c[1];
    }
  }
  *lpn = best_l;
  *cpl = best_c;
}
#endif  // HENN_COMMON_PART

}  // namespace henn

// henn_build.hip -- eps-net layer construction kernels (Alg. 1, Alg. 2).
//
//  * k_draw_mark: one thread per Philox block draws 4 of the
//    ceil(|L_{i-1}| / 2^m) samples with replacement (Alg. 2; App. D: the
//    draws are independent, so they parallelise trivially) and sets their
//    bits in a membership bitmap over L_{i-1}.
//  * compaction: popcount + two-level exclusive scan -> ascending positions.
//  * k_halve: Alg. 3's m halving steps (BuildEpsNetDiscV2).  With pairs of
//    consecutive members, the survivor of pair p of a step lands at position
//    p of the next step, so one thread per final position walks the m steps
//    backwards (one coin per step) to its position in L_{i-1}; no scan.
//  * ring verification (App. B.1 "Practical Implementation", App. G.2):
//    r sampled rings, each the rank window [a, a+w-1] of L_{i-1} ordered by
//    (distance to a sampled centre, id).  k_ring_keys writes the 64-bit
//    (distance | position) keys, a radix select finds the keys at both ends
//    of every window, and k_ring_hits tests an attempt's draws against the
//    windows with bit-identical distances.
//  * row copies, layer mean / norms (for the Gram tiles of the graph
//    build) and BF16 / FP8 quantisation of the traversal copy.
#include <math.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "henn_device.h"
#include "henn_internal.h"

namespace henn {

// ---------------------------------------------------------------- rows ----
__global__ void k_copy_rows(const float* src, int64_t src_stride, const int32_t* ids,
                            int64_t count, int d, float* dst, int dpad) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= count) return;
  const int64_t sr = ids ? (int64_t)ids[row] : row;
  const float* s = src + sr * src_stride;
  float* o = dst + row * dpad;
  for (int j = threadIdx.x & 63; j < dpad; j += 64) o[j] = j < d ? s[j] : 0.0f;
}

void launch_copy_rows(const float* src, int64_t src_stride, const int32_t* ids, int64_t count,
                      int d, float* dst, int dpad, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_copy_rows, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, st, src,
                     src_stride, ids, count, d, dst, dpad);
}

// ------------------------------------------------------------- sampling ---
__global__ void k_draw_mark(uint64_t seed, int layer, int attempt, int64_t s, int64_t draws,
                            uint32_t* bitmap) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b * 4 >= draws) return;
  const Philox4x64 r = philox4x64_10((uint64_t)b, (uint64_t)layer, (uint64_t)attempt,
                                     kTagSample, seed, 0);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (b * 4 + j < draws) {
      const uint64_t idx = uniform_index(r.x[j], (uint64_t)s);
      atomicOr(bitmap + (idx >> 5), 1u << (idx & 31));
    }
  }
}

void launch_draw_mark(uint64_t seed, int layer, int attempt, int64_t s, int64_t draws,
                      uint32_t* bitmap, hipStream_t st) {
  const int64_t blocks4 = (draws + 3) / 4;
  hipLaunchKernelGGL(k_draw_mark, dim3((unsigned)((blocks4 + 255) / 256)), dim3(256), 0, st,
                     seed, layer, attempt, s, draws, bitmap);
}

// ------------------------------------------------------------- halving ----
struct HalveSizes {
  int64_t a[32];  // a[j]: member count before step j; a[m] = final count
};

__global__ void k_halve(uint64_t seed, int layer, int attempt, int m, HalveSizes sz,
                        int32_t* out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= sz.a[m]) return;
  int64_t pos = p;
  for (int j = m - 1; j >= 0; --j) {
    const int64_t a = sz.a[j];
    if (pos == a / 2) {
      pos = a - 1;  // odd count: the unpaired last member is kept
    } else {
      const uint64_t w = stream_word(seed, kTagHalve + (uint32_t)j, (uint32_t)layer,
                                     (uint32_t)attempt, (uint64_t)pos);
      pos = 2 * pos + (int64_t)uniform_index(w, 2);
    }
  }
  out[p] = (int32_t)pos;
}

int64_t launch_halve(uint64_t seed, int layer, int attempt, int64_t s, int m, int32_t* out,
                     hipStream_t st) {
  HalveSizes sz;
  sz.a[0] = s;
  for (int j = 0; j < m; ++j) sz.a[j + 1] = (sz.a[j] + 1) / 2;
  const int64_t count = sz.a[m];
  if (count > 0)
    hipLaunchKernelGGL(k_halve, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, seed,
                       layer, attempt, m, sz, out);
  return count;
}

// ------------------------------------------------ Delete(x) compaction ----
// Old position r of a layer moves to newpos[r] (-1: deleted).  One wave per
// old row: the row's vector, its adjacency renumbered through newpos (the
// repaired rows link only to live members), its id (positions are the ids of
// a layer without an id list), and its down position renumbered through the
// layer below's map (below_newpos nullptr: unchanged).
__global__ void k_compact_layer(const float* vec, const int32_t* adj, const int32_t* ids,
                                const int32_t* down, const int32_t* newpos,
                                const int32_t* below_newpos, int64_t size, int dpad, int M,
                                float* vec_out, int32_t* adj_out, int32_t* ids_out,
                                int32_t* down_out) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= size) return;
  const int32_t np = newpos[r];
  if (np < 0) return;
  const int lane = threadIdx.x & 63;
  for (int j = lane; j < dpad; j += 64) vec_out[(int64_t)np * dpad + j] = vec[r * dpad + j];
  for (int j = lane; j < M; j += 64) {
    const int32_t e = adj[r * M + j];
    adj_out[(int64_t)np * M + j] = e >= 0 ? newpos[e] : -1;
  }
  if (lane == 0) {
    ids_out[np] = ids ? ids[r] : (int32_t)r;
    if (down_out) down_out[np] = below_newpos ? below_newpos[down[r]] : down[r];
  }
}

void launch_compact_layer(const float* vec, const int32_t* adj, const int32_t* ids,
                          const int32_t* down, const int32_t* newpos,
                          const int32_t* below_newpos, int64_t size, int dpad, int M,
                          float* vec_out, int32_t* adj_out, int32_t* ids_out, int32_t* down_out,
                          hipStream_t st) {
  if (size <= 0) return;
  hipLaunchKernelGGL(k_compact_layer, dim3((unsigned)((size + 3) / 4)), dim3(256), 0, st, vec,
                     adj, ids, down, newpos, below_newpos, size, dpad, M, vec_out, adj_out,
                     ids_out, down_out);
}

// down positions of a layer whose own members all stay, after the layer
// below was compacted
__global__ void k_remap_down(int32_t* down, int64_t size, const int32_t* below_newpos) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < size) down[r] = below_newpos[down[r]];
}

void launch_remap_down(int32_t* down, int64_t size, const int32_t* below_newpos,
                       hipStream_t st) {
  if (size <= 0) return;
  hipLaunchKernelGGL(k_remap_down, dim3((unsigned)((size + 255) / 256)), dim3(256), 0, st, down,
                     size, below_newpos);
}

// ---------------------------------------------------------- compaction ----
constexpr int kScanBlock = 256;

__global__ void k_block_popc(const uint32_t* bm, int64_t nwords, uint32_t* bsum) {
  __shared__ uint32_t part[kScanBlock / 64];
  const int64_t w = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  uint32_t c = w < nwords ? __popc(bm[w]) : 0u;
  for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int i = 0; i < kScanBlock / 64; ++i) s += part[i];
    bsum[blockIdx.x] = s;
  }
}

// exclusive scan of nb block sums by a single block (serial runs + scan)
__global__ void k_scan_bsum(uint32_t* bsum, int64_t nb, uint32_t* total) {
  __shared__ uint32_t sums[1024];
  const int tid = threadIdx.x;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = tid * per, b1 = min(nb, b0 + per);
  uint32_t s = 0;
  for (int64_t i = b0; i < b1; ++i) s += bsum[i];
  sums[tid] = s;
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const uint32_t v = sums[i];
      sums[i] = acc;
      acc += v;
    }
    *total = acc;
  }
  __syncthreads();
  uint32_t acc = sums[tid];
  for (int64_t i = b0; i < b1; ++i) {
    const uint32_t v = bsum[i];
    bsum[i] = acc;
    acc += v;
  }
}

__global__ void k_compact(const uint32_t* bm, int64_t nwords, int64_t nbits, const uint32_t* boff,
                          int32_t* out) {
  __shared__ uint32_t scan[kScanBlock];
  const int64_t w = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  const uint32_t word = w < nwords ? bm[w] : 0u;
  scan[threadIdx.x] = __popc(word);
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0u;
    __syncthreads();
    scan[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t pos = boff[blockIdx.x] + scan[threadIdx.x] - __popc(word);
  uint32_t bits = word;
  while (bits) {
    const int b = __ffs(bits) - 1;
    bits &= bits - 1;
    const int64_t idx = w * 32 + b;
    if (idx < nbits) out[pos++] = (int32_t)idx;
  }
}

int64_t compact_bitmap(const uint32_t* bitmap, int64_t s, int32_t* out_local, hipStream_t st) {
  const int64_t nwords = (s + 31) / 32;
  const int64_t nb = (nwords + kScanBlock - 1) / kScanBlock;
  DevBuf<uint32_t> bsum_buf(nb + 1);
  uint32_t* bsum = bsum_buf.get();
  uint32_t* total = bsum + nb;
  hipLaunchKernelGGL(k_block_popc, dim3((unsigned)nb), dim3(kScanBlock), 0, st, bitmap, nwords,
                     bsum);
  hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, st, bsum, nb, total);
  hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(kScanBlock), 0, st, bitmap, nwords, s,
                     bsum, out_local);
  uint32_t h_total = 0;
  HENN_HIP(hipMemcpyAsync(&h_total, total, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HENN_HIP(hipStreamSynchronize(st));
  return (int64_t)h_total;
}

// generic exclusive scan of uint32 counts: out[0..n] (out[n] = total)
__global__ void k_block_sum_u32(const uint32_t* in, int64_t n, uint32_t* bsum) {
  __shared__ uint32_t part[kScanBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  uint32_t c = i < n ? in[i] : 0u;
  for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int j = 0; j < kScanBlock / 64; ++j) s += part[j];
    bsum[blockIdx.x] = s;
  }
}

__global__ void k_block_scan_u32(const uint32_t* in, int64_t n, const uint32_t* boff,
                                 const uint32_t* total, uint32_t* out) {
  __shared__ uint32_t scan[kScanBlock];
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  const uint32_t v = i < n ? in[i] : 0u;
  scan[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const uint32_t a = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0u;
    __syncthreads();
    scan[threadIdx.x] += a;
    __syncthreads();
  }
  if (i < n) out[i] = boff[blockIdx.x] + scan[threadIdx.x] - v;
  if (i == 0) out[n] = *total;
}

int64_t exclusive_scan_u32(const uint32_t* in, int64_t n, uint32_t* out, hipStream_t st) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
  DevBuf<uint32_t> bsum_buf(nb + 1);
  uint32_t* bsum = bsum_buf.get();
  hipLaunchKernelGGL(k_block_sum_u32, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bsum);
  hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, st, bsum, nb, bsum + nb);
  hipLaunchKernelGGL(k_block_scan_u32, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, bsum,
                     bsum + nb, out);
  uint32_t total = 0;
  HENN_HIP(hipMemcpyAsync(&total, bsum + nb, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HENN_HIP(hipStreamSynchronize(st));
  return (int64_t)total;
}

__global__ void k_map_ids(const int32_t* prev_ids, const int32_t* local, int64_t count,
                          int32_t* ids, int32_t* down) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  const int32_t l = local[j];
  ids[j] = prev_ids ? prev_ids[l] : l;
  down[j] = l;
}

void launch_map_ids(const int32_t* prev_ids, const int32_t* local, int64_t count, int32_t* ids,
                    int32_t* down, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_map_ids, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st,
                     prev_ids, local, count, ids, down);
}

// ---------------------------------------------------------------- rings ---
// keys[ring][j] = (dist(centre_ring, row j) | j), rows of one layer.
template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_ring_keys(const float* vec, int dpad, int nchunks,
                                                   int metric, int64_t s,
                                                   const int32_t* centres, uint64_t* keys) {
  constexpr int G = 64 / LPN;
  const int ring = blockIdx.y;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  float q[CPL][8];
  load_query<CPL>(vec + (int64_t)centres[ring] * dpad, dpad, t, q);
  const int64_t per_block = 4 * G;
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < s;
       base += (int64_t)gridDim.x * per_block) {
    const int64_t row = base + (threadIdx.x >> 6) * G + g;
    const bool valid = row < s;
    const float dist = group_distance<kF32, LPN, CPL>(q, vec + (valid ? row : 0) * dpad, 1.0f, t,
                                                      nchunks, metric, valid);
    if (valid && t == 0) keys[(int64_t)ring * s + row] = dkey(dist, (int32_t)row);
  }
}

// a draw's key against every ring window: hit flag per ring
template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_ring_hits(const float* vec, int dpad, int nchunks,
                                                   int metric, int64_t s, uint64_t seed,
                                                   int layer, int attempt, int64_t draws,
                                                   const int32_t* cand,
                                                   const int32_t* centres, const uint64_t* lo,
                                                   const uint64_t* hi, uint32_t* hits) {
  constexpr int G = 64 / LPN;
  const int ring = blockIdx.y;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  float q[CPL][8];
  load_query<CPL>(vec + (int64_t)centres[ring] * dpad, dpad, t, q);
  const uint64_t klo = lo[ring], khi = hi[ring];
  const int64_t per_block = 4 * G;
  for (int64_t base = (int64_t)blockIdx.x * per_block; base < draws;
       base += (int64_t)gridDim.x * per_block) {
    const int64_t qd = base + (threadIdx.x >> 6) * G + g;
    const bool valid = qd < draws;
    int64_t row = 0;
    if (valid && cand) {
      row = cand[qd];
    } else if (valid) {
      const uint64_t w = stream_word(seed, kTagSample, (uint32_t)layer, (uint32_t)attempt,
                                     (uint64_t)qd);
      row = (int64_t)uniform_index(w, (uint64_t)s);
    }
    const float dist =
        group_distance<kF32, LPN, CPL>(q, vec + row * dpad, 1.0f, t, nchunks, metric, valid);
    if (valid && t == 0) {
      const uint64_t key = dkey(dist, (int32_t)row);
      if (key >= klo && key <= khi) atomicOr(hits + ring, 1u);
    }
  }
}

#define HENN_RING_COMBOS(X) \
  X(1, 1) X(2, 1) X(4, 1) X(2, 2) X(4, 2) X(8, 1) X(2, 4) X(4, 4) X(8, 2) X(16, 1) X(8, 4) \
  X(16, 2) X(4, 8) X(16, 4) X(16, 8)

void launch_ring_keys(int lpn, int cpl, const float* vec, int dpad, int nchunks, int metric,
                      int64_t s, const int32_t* centres, int r, uint64_t* keys, hipStream_t st) {
  const int64_t per_block = 4 * (64 / lpn);
  const unsigned gx = (unsigned)std::min<int64_t>((s + per_block - 1) / per_block, 65535);
#define HENN_TRY(L, C)                                                                         \
  if (lpn == L && cpl == C) {                                                                  \
    hipLaunchKernelGGL((k_ring_keys<L, C>), dim3(gx, r), dim3(256), 0, st, vec, dpad, nchunks, \
                       metric, s, centres, keys);                                              \
    return;                                                                                    \
  }
  HENN_RING_COMBOS(HENN_TRY)
#undef HENN_TRY
}

void launch_ring_hits(int lpn, int cpl, const float* vec, int dpad, int nchunks, int metric,
                      int64_t s, uint64_t seed, int layer, int attempt, int64_t draws,
                      const int32_t* cand, const int32_t* centres, const uint64_t* lo,
                      const uint64_t* hi, int r, uint32_t* hits, hipStream_t st) {
  const int64_t per_block = 4 * (64 / lpn);
  const unsigned gx = (unsigned)std::min<int64_t>((draws + per_block - 1) / per_block, 65535);
#define HENN_TRY(L, C)                                                                          \
  if (lpn == L && cpl == C) {                                                                   \
    hipLaunchKernelGGL((k_ring_hits<L, C>), dim3(gx, r), dim3(256), 0, st, vec, dpad, nchunks,  \
                       metric, s, seed, layer, attempt, draws, cand, centres, lo, hi, hits);    \
    return;                                                                                     \
  }
  HENN_RING_COMBOS(HENN_TRY)
#undef HENN_TRY
}

// ------------------------------------------------------- radix select ----
// Selects, for every target, the key of a given rank among the s keys of
// its ring (8 passes of 8 bits, most significant first).
__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t* keys, int64_t s, int nt_per_ring,
                                                    const uint64_t* prefix, int shift,
                                                    uint32_t* hist) {
  __shared__ uint32_t h[2][256];
  const int ring = blockIdx.y;
  for (int i = threadIdx.x; i < 2 * 256; i += blockDim.x) (&h[0][0])[i] = 0u;
  __syncthreads();
  const uint64_t hmask = shift + 8 >= 64 ? 0ull : (~0ull << (shift + 8));
  const uint64_t p0 = prefix[ring * nt_per_ring + 0] & hmask;
  const uint64_t p1 = prefix[ring * nt_per_ring + 1] & hmask;
  const uint64_t* kr = keys + (int64_t)ring * s;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < s;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = kr[j];
    const uint32_t bin = (uint32_t)(k >> shift) & 255u;
    if ((k & hmask) == p0) atomicAdd(&h[0][bin], 1u);
    if ((k & hmask) == p1) atomicAdd(&h[1][bin], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * 256; i += blockDim.x) {
    const uint32_t v = (&h[0][0])[i];
    if (v) atomicAdd(hist + (int64_t)ring * 512 + i, v);
  }
}

__global__ void k_radix_pick(uint32_t* hist, uint64_t* prefix, int64_t* rank, int ntargets,
                             int shift) {
  const int tg = blockIdx.x * blockDim.x + threadIdx.x;
  if (tg >= ntargets) return;
  uint32_t* h = hist + (int64_t)tg * 256;
  int64_t r = rank[tg];
  int64_t cum = 0;
  int chosen = 255;
  for (int b = 0; b < 256; ++b) {
    if (r < cum + h[b]) {
      chosen = b;
      break;
    }
    cum += h[b];
  }
  prefix[tg] |= (uint64_t)chosen << shift;
  rank[tg] = r - cum;
  for (int b = 0; b < 256; ++b) h[b] = 0u;
}

void launch_radix_select(const uint64_t* keys, int64_t s, int r, const int64_t* ranks_host,
                         uint64_t* out_keys_host, hipStream_t st) {
  const int nt = 2 * r;
  DevBuf<uint32_t> hist_buf(256 * nt);
  DevBuf<uint64_t> prefix_buf(nt);
  DevBuf<int64_t> rank_buf(nt);
  uint32_t* hist = hist_buf.get();
  uint64_t* prefix = prefix_buf.get();
  int64_t* rank = rank_buf.get();
  HENN_HIP(hipMemsetAsync(hist, 0, sizeof(uint32_t) * 256 * nt, st));
  HENN_HIP(hipMemsetAsync(prefix, 0, sizeof(uint64_t) * nt, st));
  HENN_HIP(hipMemcpyAsync(rank, ranks_host, sizeof(int64_t) * nt, hipMemcpyHostToDevice, st));
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>((s + 255) / 256, 1024));
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(gx, r), dim3(256), 0, st, keys, s, 2, prefix, shift,
                       hist);
    hipLaunchKernelGGL(k_radix_pick, dim3((nt + 63) / 64), dim3(64), 0, st, hist, prefix, rank,
                       nt, shift);
  }
  HENN_HIP(hipMemcpyAsync(out_keys_host, prefix, sizeof(uint64_t) * nt, hipMemcpyDeviceToHost,
                          st));
  HENN_HIP(hipStreamSynchronize(st));
}

// ------------------------------------------------------- mean, norms -----
__global__ void k_col_partial(const float* vec, int64_t size, int dpad, int64_t rows_per_block,
                              float* partial) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(size, r0 + rows_per_block);
  for (int j = threadIdx.x; j < dpad; j += blockDim.x) {
    float acc = 0.0f;
    for (int64_t r = r0; r < r1; ++r) acc += vec[r * dpad + j];
    partial[(int64_t)blockIdx.x * dpad + j] = acc;
  }
}

void layer_mean(const float* vec, int64_t size, int dpad, float* mean_dev, hipStream_t st) {
  const int64_t nb = std::min<int64_t>(size, 2048);
  const int64_t per = (size + nb - 1) / nb;
  const int64_t nblk = (size + per - 1) / per;
  DevBuf<float> partial_buf(nblk * dpad);
  float* partial = partial_buf.get();
  hipLaunchKernelGGL(k_col_partial, dim3((unsigned)nblk), dim3(256), 0, st, vec, size, dpad, per,
                     partial);
  std::vector<float> h((size_t)(nblk * dpad));
  HENN_HIP(hipMemcpyAsync(h.data(), partial, sizeof(float) * nblk * dpad, hipMemcpyDeviceToHost,
                          st));
  HENN_HIP(hipStreamSynchronize(st));
  std::vector<float> mean((size_t)dpad);
  for (int j = 0; j < dpad; ++j) {
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) acc += h[(size_t)(b * dpad + j)];
    mean[(size_t)j] = (float)(acc / (double)size);
  }
  HENN_HIP(hipMemcpyAsync(mean_dev, mean.data(), sizeof(float) * dpad, hipMemcpyHostToDevice, st));
  HENN_HIP(hipStreamSynchronize(st));
}

__global__ void k_row_norms(const float* vec, const float* mean, int64_t size, int dpad,
                            float* norms) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= size) return;
  float acc = 0.0f;
  for (int j = 0; j < dpad; ++j) {
    const float v = vec[r * dpad + j] - (mean ? mean[j] : 0.0f);
    acc = __builtin_fmaf(v, v, acc);
  }
  norms[r] = acc;
}

void launch_row_norms(const float* vec, const float* mean, int64_t size, int dpad, float* norms,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_row_norms, dim3((unsigned)((size + 255) / 256)), dim3(256), 0, st, vec,
                     mean, size, dpad, norms);
}

__global__ void k_max_reduce(const float* v, int64_t n, unsigned int* out) {
  float m = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, v[i]);
  for (int s = 32; s > 0; s >>= 1) m = fmaxf(m, __shfl_xor(m, s));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));  // m >= 0: bits are monotone
}

float max_norm(const float* norms, int64_t size, hipStream_t st) {
  DevBuf<unsigned int> d_buf(1);
  unsigned int* d = d_buf.get();
  HENN_HIP(hipMemsetAsync(d, 0, sizeof(unsigned int), st));
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((size + 255) / 256, 1024));
  hipLaunchKernelGGL(k_max_reduce, dim3(g), dim3(256), 0, st, norms, size, d);
  unsigned int h = 0;
  HENN_HIP(hipMemcpyAsync(&h, d, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
  HENN_HIP(hipStreamSynchronize(st));
  float f;
  memcpy(&f, &h, sizeof(f));
  return f;
}

// ------------------------------------------------------- quantisation ----
// BF16: round-to-nearest-even of each FP32 coordinate (scale 1).
// FP8:  scale = max|x| / 448 per row (1 for an all-zero row); code =
//       round-to-nearest-even of x / scale in OCP E4M3 (saturating at 448).
__device__ inline uint32_t f32_to_e4m3_rne(float v) {
  const uint32_t sign = v < 0.0f ? 0x80u : 0u;
  float a = fabsf(v);
  if (!(a < 448.0f)) return sign | 0x7eu;  // saturate (also catches NaN -> 448)
  uint32_t code;
  if (a < 0x1p-6f) {
    // subnormal grid: multiples of 2^-9
    const float qv = rintf(a * 512.0f);  // 0..8; 8 is the smallest normal
    code = (uint32_t)qv;
  } else {
    int e;
    frexpf(a, &e);  // a = f * 2^e, f in [0.5, 1)
    const int ue = e - 1;  // a in [2^ue, 2^(ue+1))
    float qv = rintf(ldexpf(a, 3 - ue));  // in [8, 16]
    int uee = ue;
    if (qv >= 16.0f) {
      qv = 8.0f;
      uee += 1;
    }
    code = ((uint32_t)(uee + 7) << 3) | ((uint32_t)qv - 8u);
    if (code > 0x7eu) code = 0x7eu;
  }
  return sign | code;
}

__global__ void k_quantize_bf16(const float* vec, int64_t size, int dpad, uint16_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= size * dpad) return;
  out[i] = (uint16_t)f32_to_bf16_rne(vec[i]);
}

__global__ void k_quantize_fp8(const float* vec, int64_t size, int dpad, uint8_t* out,
                               float* scale) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= size) return;
  const int lane = lane_id();
  const float* x = vec + row * dpad;
  float m = 0.0f;
  for (int j = lane; j < dpad; j += 64) m = fmaxf(m, fabsf(x[j]));
  for (int s = 32; s > 0; s >>= 1) m = fmaxf(m, __shfl_xor(m, s));
  const float sc = m > 0.0f ? m / 448.0f : 1.0f;
  if (lane == 0) scale[row] = sc;
  for (int j = lane; j < dpad; j += 64) out[row * dpad + j] = (uint8_t)f32_to_e4m3_rne(x[j] / sc);
}

__global__ void k_decode_rows(int storage, const void* vq, const float* scale, int64_t size,
                              int dpad, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= size * dpad) return;
  if (storage == kBF16) {
    out[i] = bf16_to_f32(static_cast<const uint16_t*>(vq)[i]);
  } else {
    out[i] = scale[i / dpad] * fp8_to_f32(static_cast<const uint8_t*>(vq)[i]);
  }
}

void launch_decode_rows(int storage, const void* vq, const float* scale, int64_t size, int dpad,
                        float* out, hipStream_t st) {
  const int64_t n = size * dpad;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_decode_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, storage,
                     vq, scale, size, dpad, out);
  HENN_HIP(hipGetLastError());
}

__global__ void k_adj_scale(const int32_t* adj, int64_t n, const float* scale, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t u = adj[i];
  out[i] = u >= 0 ? scale[u] : 0.0f;
}

void launch_adj_scale(const int32_t* adj, int64_t n, const float* scale, float* out,
                      hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_adj_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, adj, n,
                     scale, out);
  HENN_HIP(hipGetLastError());
}

void launch_quantize(int storage, const float* vec, int64_t size, int dpad, void* out,
                     float* scale, hipStream_t st) {
  if (storage == kBF16) {
    const int64_t n = size * dpad;
    hipLaunchKernelGGL(k_quantize_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, vec,
                       size, dpad, static_cast<uint16_t*>(out));
  } else if (storage == kFP8) {
    hipLaunchKernelGGL(k_quantize_fp8, dim3((unsigned)((size + 3) / 4)), dim3(256), 0, st, vec,
                       size, dpad, static_cast<uint8_t*>(out), scale);
  }
}

}  // namespace henn

// henn_knn.hip -- exact kNN navigable graph of one layer (App. B.2; the
// "knn" graph of App. G.4): every member's R nearest other members in
// (distance, id) order.
//
// Three steps:
//  1. k_gram_topk / k_knn_gram_wide (MFMA): all-pairs Gram tiles on FP32
//     matrix cores (the wide form streams K in slices for d > 128).  A
//     workgroup owns 128 rows (4 waves x 32); candidate tiles of 32 rows are
//     staged in LDS and multiplied with v_mfma_f32_32x32x2f32, the K split
//     as (lane half h) x (step kk) over the two halves of each row.  Rows are
//     centred on the layer mean first (L2 only), which shrinks the norms
//     the Gram form cancels against.  Each lane keeps the 32 smallest Gram
//     distances it sees in registers, so every row ends with a 64-entry
//     shortlist (two halves) plus the 32nd Gram value of each half.
//  2. k_knn_rerank: one wave per row recomputes the shortlist's distances
//     in the canonical difference form, sorts the (distance, id) keys and
//     keeps R.  A row is re-solved exactly when the shortlist cannot be
//     proven to contain the true top R: when neither the bound with the
//     layer's largest norm nor (L2) the bound relative to each candidate's
//     own distance puts every left-out candidate beyond the R-th exact
//     distance.
//  3. k_knn_exact: the exact brute force for those rows.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <chrono>

#include "henn_device.h"
#include "henn_internal.h"

namespace henn {

constexpr int kShort = 32;  // shortlist entries per lane half
constexpr int kTileC = 32;  // candidates per LDS tile
// candidates a lane of k_gram_topk_x3 stages in LDS before merging them into
// its list (at most four enter per step of four values)
constexpr int kX3Cand = 8;

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Gram shortlist pass of the layer's kNN graph (d <= 128; Alg. 1 builds
// one graph per layer): queries and candidates are the layer's rows and a
// row never lists itself.  A block takes 128 rows (one 32-row MFMA column
// block per wave) and streams the layer through LDS in tiles of kTileC.
// The distance is assembled inside the contraction: with y = centred
// candidate and x = centred row,
//   |y - x|^2 = sum_k y_k (-2 x_k) + (|y|^2 + pen) * 1 + 1 * |x|^2
//   -<y, x>   = sum_k y_k (-x_k)  +  pen * 1         + 0 * 0
// the last two products being one extra MFMA step over the two lane
// halves; pen = +inf marks rows past the end of the layer.  Rows are taken
// as zero-padded to 2 * KH coordinates (dpad <= 2 * KH); the K dimension
// splits at KH between the lane halves, so each tile is a fixed,
// branch-free chain of KH + 1 MFMAs and the epilogue is one compare per
// value, with an insertion into the lane's sorted top-KS only when the
// value beats the current KS-th.  Output: per (row, lane half) the KS
// smallest (value, candidate index) pairs, ascending.
// row_list: when given, the block's rows are row_list[i] for i < n_rows
// (the rows the split form could not prove) and the shortlists go to
// position i; otherwise rows 0 .. size - 1 in order (n_rows = size).
template <int KH, int KS>
__global__ __launch_bounds__(256, 2) void k_gram_topk(const float* vec, int64_t size, int dpad,
                                                      const float* norms, const float* mean,
                                                      int metric, float* sl_d, int32_t* sl_i,
                                                      int64_t block0, const int32_t* row_list,
                                                      int64_t n_rows) {
  // two LDS buffers of [kTileC][2 * KH + 4] candidates + their norms; the
  // next tile is fetched into registers while the current one is multiplied
  extern __shared__ __align__(16) float tile[];
  constexpr int kStride = 2 * KH + 4;
  constexpr int kBuf = kTileC * kStride + kTileC;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qc = lane & 31, h = lane >> 5;
  const int64_t qi = (block0 + blockIdx.x) * 128 + wave * 32 + qc;
  const bool qvalid = qi < n_rows;
  const int64_t qrow = !qvalid ? -1 : row_list ? (int64_t)row_list[qi] : qi;
  const int64_t cb = 0, ce = size;
  const bool l2 = metric == 0;
  const float qscale = l2 ? -2.0f : -1.0f;

  // the row's coordinates: loads clamped into the row (no branches, all in
  // flight together), out-of-range values dropped afterwards
  float bq[KH];
  {
    const float* qr = vec + (qvalid ? qrow : 0) * dpad;
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      const int e = h * KH + kk;
      bq[kk] = qr[e < dpad ? e : 0];
    }
#pragma unroll
    for (int kk = 0; kk < KH; ++kk) {
      const int e = h * KH + kk;
      const float m = (mean && e < dpad) ? mean[e] : 0.0f;
      bq[kk] = (qvalid && e < dpad) ? qscale * (bq[kk] - m) : 0.0f;
    }
  }
  // B operand of the extra step: row 0 is all ones, row 1 holds |x|^2 (L2)
  const float b_extra = h == 0 ? 1.0f : (l2 && qvalid ? norms[qrow] : 0.0f);
  const float a_one = l2 ? 1.0f : 0.0f;

  float td[KS];
  int32_t ti[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    td[j] = INFINITY;
    ti[j] = -1;
  }

  // zero the padding columns [dpad, 2 KH) of both buffers once; tiles only
  // ever write columns below dpad
  for (int i = threadIdx.x; i < 2 * kTileC * (2 * KH - dpad); i += 256) {
    const int per = 2 * KH - dpad;
    const int b = i / (kTileC * per), rem = i - b * kTileC * per;
    const int r = rem / per, c = dpad + (rem - r * per);
    tile[b * kBuf + r * kStride + c] = 0.0f;
  }

  // a tile is kTileC * dpad / 4 <= 16 * KH float4, so each of the 256
  // threads moves at most KH / 16 of them.  Loads are clamped to valid rows
  // so that they issue without branches and complete while the previous
  // tile is multiplied; the mean is subtracted when the tile is written to
  // LDS.
  constexpr int kMaxF4 = KH / 16;
  const int f4_per_row = dpad >> 2;
  const int tile_f4 = kTileC * f4_per_row;
  float* mean_lds = tile + 2 * kBuf;
  if (mean)
    for (int e = threadIdx.x; e < dpad; e += 256) mean_lds[e] = mean[e];
  int src_row[kMaxF4], src_c4[kMaxF4];
#pragma unroll
  for (int u = 0; u < kMaxF4; ++u) {
    const int idx = min((int)threadIdx.x + u * 256, tile_f4 - 1);
    src_row[u] = idx / f4_per_row;
    src_c4[u] = idx - src_row[u] * f4_per_row;
  }
  // fetch only issues loads (their values are first used by stash, after
  // the tile in flight has been multiplied); stash applies the selects
  float4 pre[kMaxF4];
  float pnorm = 0.0f;
  int plast = 0;
  auto fetch = [&](int64_t c0) {
    const int64_t rem = ce - 1 - c0;
    const int last = rem < kTileC - 1 ? (int)rem : kTileC - 1;  // last valid row of the tile
    const float* base = vec + c0 * dpad;
#pragma unroll
    for (int u = 0; u < kMaxF4; ++u) {
      const int r = src_row[u] < last ? src_row[u] : last;
      pre[u] = reinterpret_cast<const float4*>(base + r * dpad)[src_c4[u]];
    }
    const int r = (int)(threadIdx.x & (kTileC - 1));
    pnorm = norms[c0 + (r < last ? r : last)];
    plast = last;
  };
  auto stash = [&](float* buf) {
#pragma unroll
    for (int u = 0; u < kMaxF4; ++u) {
      if ((int)threadIdx.x + u * 256 < tile_f4) {
        float4 v = pre[u];
        if (mean) {
          const float4 m = reinterpret_cast<const float4*>(mean_lds)[src_c4[u]];
          v.x -= m.x; v.y -= m.y; v.z -= m.z; v.w -= m.w;
        }
        *reinterpret_cast<float4*>(buf + src_row[u] * kStride + 4 * src_c4[u]) = v;
      }
    }
    if (threadIdx.x < kTileC)
      buf[kTileC * kStride + threadIdx.x] =
          (int)threadIdx.x <= plast ? (l2 ? pnorm : 0.0f) : INFINITY;
  };

  __syncthreads();
  if (cb < ce) {
    fetch(cb);
    stash(tile);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t c0 = cb; c0 < ce; c0 += kTileC) {
    const bool more = c0 + kTileC < ce;
    if (more) fetch(c0 + kTileC);
    const float* buf = tile + cur * kBuf;

    floatx16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    const float4* arow = reinterpret_cast<const float4*>(buf + qc * kStride + h * KH);
#pragma unroll
    for (int k4 = 0; k4 < KH / 4; ++k4) {
      const float4 a = arow[k4];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, bq[4 * k4 + 0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, bq[4 * k4 + 1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, bq[4 * k4 + 2], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, bq[4 * k4 + 3], acc, 0, 0, 0);
    }
    const float a_extra = h == 0 ? buf[kTileC * kStride + qc] : a_one;
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a_extra, b_extra, acc, 0, 0, 0);

    bool any = false;
#pragma unroll
    for (int v = 0; v < 16; ++v) any |= acc[v] < td[KS - 1];
    if (__builtin_amdgcn_ballot_w64(any)) {
      // lanes without a hit push +inf through the network, which leaves
      // their list unchanged, so the network runs without divergence
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t crow = c0 + 8 * (v >> 2) + 4 * h + (v & 3);
        float nd = crow == qrow ? INFINITY : acc[v];
        if (__builtin_amdgcn_ballot_w64(nd < td[KS - 1])) {
          int32_t ni = (int32_t)crow;
#pragma unroll
          for (int j = 0; j < KS; ++j) {
            const bool sw = nd < td[j];
            const float od = td[j];
            const int32_t oi = ti[j];
            td[j] = sw ? nd : od;
            ti[j] = sw ? ni : oi;
            nd = sw ? od : nd;
            ni = sw ? oi : ni;
          }
        }
      }
    }
    if (more) stash(tile + (cur ^ 1) * kBuf);
    __syncthreads();
    cur ^= 1;
  }
  if (qvalid) {
    const int64_t o = qi * (2 * KS) + h * KS;
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      sl_d[o + j] = td[j];
      sl_i[o + j] = ti[j];
    }
  }
}

// ------------------------------------------------------------------------
// The same shortlist on BF16 matrix cores with split operands (the default
// build for d <= 128).  Each centred row x' = fl(x - mean) is stored once as
// hi = bf16(x') and lo = bf16(x' - hi) (k_split_rows), and every product is
// taken as y_h b_h + y_h b_l + y_l b_h, three v_mfma_f32_32x32x16_bf16 per
// 16 coordinates, each product exact in FP32.  Error of one Gram value G
// against the canonical FP32 distance D that the re-rank computes, with
// u = 2^-8 the BF16 unit roundoff and b = -2 x' (L2; -x' for IP, which only
// halves the bound):
//  - the dropped terms y_l b_l + (y' - y_h - y_l) b + y' (b - b_h - b_l)
//    are at most (u^2 (1 + u)^2 + 2 u^2) |y'_k| |b_k| per coordinate, so
//    at most 3.25 2^-16 (|x'|^2 + |y'|^2) summed (|b| = 2 |x'|);
//  - the FP32 accumulation of 3 kp exact products onto the two norms, in
//    any order: at most (3 kp + 2) 2^-24 times their absolute sum, itself
//    at most 2 (|x'|^2 + |y'|^2) up to O(u);
//  - the norms, the centring and the canonical distance's own rounding:
//    at most (4 dpad + 20) 2^-24 (|x'|^2 + |y'|^2).
// So |G - D| <= (3.25 2^-16 + (6 kp + 4 dpad + 24) 2^-24) (|x'|^2 + |y'|^2),
// and the re-rank proves each row's shortlist with that coefficient times
// |x'|^2 + max_y |y'|^2 (x3_split_coef).  The products cost 3 / 16 of the
// FP32 ones on the matrix cores; the shortlist, its output and the re-rank
// are those of k_gram_topk.

// rows [size_pad][2 kp] BF16 (hi then lo) of the centred rows, zero past
// dpad and for the padding rows; tnorm [size_pad]: the tile norm a row enters
// the Gram with (|x'|^2 for L2, 0 for IP, +inf for the padding rows)
__global__ void k_split_rows(const float* vec, const float* mean, const float* norms, int metric,
                             int64_t size, int64_t size_pad, int dpad, int kp, uint16_t* out,
                             float* tnorm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= size_pad * kp) return;
  const int64_t r = i / kp;
  const int c = (int)(i - r * kp);
  const float v =
      (r < size && c < dpad) ? vec[r * dpad + c] - (mean ? mean[c] : 0.0f) : 0.0f;
  const uint32_t hi = f32_to_bf16_rne(v);
  const uint32_t lo = f32_to_bf16_rne(v - bf16_to_f32(hi));
  out[r * 2 * kp + c] = (uint16_t)hi;
  out[r * 2 * kp + kp + c] = (uint16_t)lo;
  if (c == 0) tnorm[r] = r < size ? (metric == 0 ? norms[r] : 0.0f) : INFINITY;
}

static float x3_split_coef(int dpad) {
  const int kp = (dpad + 15) / 16 * 16;
  return 3.25f * 0x1p-16f + (float)(6 * kp + 4 * dpad + 24) * 0x1p-24f;
}

typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

// bf16x8 times a power of two (exact: the significands do not change)
__device__ inline bf16x8v scale_bf16x8(uint4 w, float f) {
  uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t a = f32_to_bf16_rne(bf16_to_f32(u[i] & 0xffffu) * f);
    const uint32_t b = f32_to_bf16_rne(bf16_to_f32(u[i] >> 16) * f);
    u[i] = a | (b << 16);
  }
  return __builtin_bit_cast(bf16x8v, make_uint4(u[0], u[1], u[2], u[3]));
}

// Copy instructions of one staged tile of k_gram_topk_x3 (64 slots of 16
// bytes each): 32 rows of 4 S + 1 slots (hi, lo, one pad slot).
__host__ __device__ constexpr int x3_tile_instrs(int S) { return (32 * (4 * S + 1) + 63) / 64; }

// A block takes 128 rows (32 per wave) and streams the layer through LDS in
// tiles of kTileC split rows.  The tiles arrive by the global-to-LDS copy
// (global_load_lds_dwordx4: one instruction moves 64 chunks of 16 bytes into
// 64 consecutive slots), in a ring of three buffers: the copies of the next
// two tiles are in flight while one is multiplied.  A staged row is its hi
// and lo halves plus one pad slot (a copy of its first chunk), so that the
// 32 rows one instruction reads fall on different banks.  The rows and the
// tile norms are padded to a multiple of 32 (zero rows, norm +inf), so every
// copy reads inside them.  The accumulator starts at |y'|^2 + |x'|^2 (L2) or
// 0 (IP), +inf for the padding rows.
template <int S, int KS>
__global__ __launch_bounds__(256, 2) void k_gram_topk_x3(const uint16_t* rows, int64_t size,
                                                         const float* norms, const float* tnorms,
                                                         int metric, float* sl_d, int32_t* sl_i,
                                                         int64_t block0) {
  constexpr int KP = 16 * S;
  constexpr int kHalfU4 = KP / 8;           // uint4 per half row
  constexpr int kRowU4 = 2 * kHalfU4 + 1;   // staged row: hi, lo, pad
  constexpr int kJ = x3_tile_instrs(S);     // copy instructions per tile
  constexpr int kSlots = 64 * kJ;           // >= kTileC * kRowU4
  constexpr int kBufU4 = kSlots + 8;        // slots, then 32 norms
  constexpr int kMaxJ = (kJ + 3) / 4;       // copy instructions of one wave per tile
  static_assert(kTileC == 32, "a tile is one 32-row operand block");
  static_assert(kMaxJ <= 5, "the waits below count at most six copies per wave and tile");
  // three tile buffers (slots, then 32 norms) and the staged candidates of
  // the four waves, as separate objects, so that the compiler can tell most
  // reads of one buffer from the copies into another (69 KB at S = 8, two
  // blocks a CU)
  __shared__ uint4 buf0[kBufU4], buf1[kBufU4], buf2[kBufU4];
  __shared__ uint2 cand_all[4 * 64 * kX3Cand];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qc = lane & 31, h = lane >> 5;
  const int64_t qrow = (block0 + blockIdx.x) * 128 + wave * 32 + qc;
  const bool qvalid = qrow < size;
  const bool l2 = metric == 0;

  // the row operand: coordinates 16 s + 8 h .. + 8 of row qc, hi and lo,
  // times -2 (L2) or -1 (IP)
  bf16x8v bh[S], bl[S];
  {
    const uint4* qr = reinterpret_cast<const uint4*>(rows + (qvalid ? qrow : 0) * 2 * KP);
    const float f = qvalid ? (l2 ? -2.0f : -1.0f) : 0.0f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      bh[s] = scale_bf16x8(qr[2 * s + h], f);
      bl[s] = scale_bf16x8(qr[kHalfU4 + 2 * s + h], f);
    }
  }
  const float qn = (l2 && qvalid) ? norms[qrow] : 0.0f;

  float td[KS];
  int32_t ti[KS];
#pragma unroll
  for (int j = 0; j < KS; ++j) {
    td[j] = INFINITY;
    ti[j] = -1;
  }

  // this lane's staged values (slot i of lane l at i * 64 + l) and their
  // merge into the sorted list: strict comparisons, so equal values keep
  // the order in which they were found; the row itself is dropped here
  uint2* cand = cand_all + wave * (kX3Cand * 64);
  int ncand = 0;
  auto merge = [&]() {
    int m = ncand;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = max(m, __shfl_xor(m, o));
    m = __builtin_amdgcn_readfirstlane(m);
    for (int i = 0; i < m; ++i) {
      const uint2 e = cand[i * 64 + lane];
      float nd = (i < ncand && (int64_t)e.y != qrow) ? __uint_as_float(e.x) : INFINITY;
      if (__builtin_amdgcn_ballot_w64(nd < td[KS - 1])) {
        int32_t ni = (int32_t)e.y;
#pragma unroll
        for (int j = 0; j < KS; ++j) {
          const bool sw = nd < td[j];
          const float od = td[j];
          const int32_t oi = ti[j];
          td[j] = sw ? nd : od;
          ti[j] = sw ? ni : oi;
          nd = sw ? od : nd;
          ni = sw ? oi : ni;
        }
      }
    }
    ncand = 0;
  };

  // this wave's copy instructions j = wave + 4 u (u < kMaxJ, j < kJ); slot
  // p = 64 j + lane of a tile takes chunk c of row r (p = r kRowU4 + c), the
  // row's first chunk for a pad slot or a slot past the rows
  int off0 = 0, off1 = 0, off2 = 0, off3 = 0, off4 = 0;
#define HENN_X3_OFF(U)                                                                   \
  if constexpr (U < kMaxJ) {                                                             \
    const int p_ = 64 * (wave + 4 * U) + lane, r_ = p_ / kRowU4, c_ = p_ - r_ * kRowU4;  \
    off##U = min(r_, kTileC - 1) * 2 * kHalfU4 +                                         \
             ((p_ < kTileC * kRowU4 && c_ < 2 * kHalfU4) ? c_ : 0);                      \
  }
  HENN_X3_OFF(0) HENN_X3_OFF(1) HENN_X3_OFF(2) HENN_X3_OFF(3) HENN_X3_OFF(4)
#undef HENN_X3_OFF
  const int per_tile = (kJ - wave + 3) / 4 + 1;  // this wave's copies per tile, norms included
  typedef __attribute__((address_space(3))) void* lds_ptr;
  auto issue = [&](int64_t c0, uint4* tile) {
    const uint4* src = reinterpret_cast<const uint4*>(rows + c0 * 2 * KP);
#define HENN_X3_COPY(U)                                                                  \
  if constexpr (U < kMaxJ)                                                               \
    if (wave + 4 * U < kJ)                                                               \
      __builtin_amdgcn_global_load_lds(src + off##U, (lds_ptr)(tile + 64 * (wave + 4 * U)), \
                                       16, 0, 0);
    HENN_X3_COPY(0) HENN_X3_COPY(1) HENN_X3_COPY(2) HENN_X3_COPY(3) HENN_X3_COPY(4)
#undef HENN_X3_COPY
    if (lane < 8)
      __builtin_amdgcn_global_load_lds(tnorms + c0 + 8 * wave + lane,
                                       (lds_ptr)(reinterpret_cast<float*>(tile + kSlots) + 8 * wave),
                                       4, 0, 0);
  };
  // waits until at most n of this wave's vector memory operations are
  // outstanding (loads complete in order and nothing else is issued in the
  // loop, so the copies issued before the last n are done)
  auto wait_copies = [](int n) {
    switch (n) {
      case 0: __builtin_amdgcn_s_waitcnt(0xF70); break;
      case 1: __builtin_amdgcn_s_waitcnt(0xF71); break;
      case 2: __builtin_amdgcn_s_waitcnt(0xF72); break;
      case 3: __builtin_amdgcn_s_waitcnt(0xF73); break;
      case 4: __builtin_amdgcn_s_waitcnt(0xF74); break;
      case 5: __builtin_amdgcn_s_waitcnt(0xF75); break;
      default: __builtin_amdgcn_s_waitcnt(0xF76); break;
    }
  };
  // a workgroup barrier that does not wait for the copies of the tiles ahead
  // (LDS is coherent within the workgroup; the memory clobber keeps the
  // compiler from moving LDS accesses across it)
  auto lds_barrier = []() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); };

  auto body = [&](int64_t c0, const uint4* buf) {
    const float4* tn = reinterpret_cast<const float4*>(buf + kSlots);
    floatx16 acc;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 nr = tn[2 * g + h];  // candidates 8 g + 4 h .. + 3
      acc[4 * g + 0] = nr.x + qn;
      acc[4 * g + 1] = nr.y + qn;
      acc[4 * g + 2] = nr.z + qn;
      acc[4 * g + 3] = nr.w + qn;
    }
    const uint4* arow = buf + qc * kRowU4;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const bf16x8v ah = __builtin_bit_cast(bf16x8v, arow[2 * s + h]);
      const bf16x8v al = __builtin_bit_cast(bf16x8v, arow[kHalfU4 + 2 * s + h]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh[s], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl[s], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh[s], acc, 0, 0, 0);
    }

    // values below the list's last entry (as it stood at the last merge) are
    // staged; a merge inserts the staged values of all lanes one slot at a
    // time, so a value that only one lane keeps no longer costs the whole
    // wave a pass of the insertion network
    bool any = false;
#pragma unroll
    for (int v = 0; v < 16; ++v) any |= acc[v] < td[KS - 1];
    if (__builtin_amdgcn_ballot_w64(any)) {
      const uint32_t cbase = (uint32_t)c0 + 4 * h;
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        if (__builtin_amdgcn_ballot_w64(ncand > kX3Cand - 4)) merge();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (acc[4 * g + u] < td[KS - 1]) {  // value 4 g + u: row c0 + 8 g + 4 h + u
            cand[ncand * 64 + lane] = make_uint2(__float_as_uint(acc[4 * g + u]), cbase + 8 * g + u);
            ++ncand;
          }
        }
      }
    }
  };

  // every wave of the block walks the same tiles (the barriers need all of
  // them); the padded layer holds nt whole tiles
  const int64_t nt = (size + kTileC - 1) / kTileC;
  issue(0, buf0);
  if (nt > 1) issue(kTileC, buf1);
  for (int64_t t = 0; t < nt; t += 3) {
#define HENN_X3_STEP(I, CUR, NEXT2)                                                      \
  {                                                                                      \
    const int64_t tt_ = t + (I);                                                         \
    wait_copies(tt_ + 1 < nt ? per_tile : 0);                                            \
    lds_barrier();                                                                       \
    if (tt_ + 2 < nt) issue((tt_ + 2) * kTileC, NEXT2);                                  \
    body(tt_ * kTileC, CUR);                                                             \
  }
    HENN_X3_STEP(0, buf0, buf2)
    if (t + 1 >= nt) break;
    HENN_X3_STEP(1, buf1, buf0)
    if (t + 2 >= nt) break;
    HENN_X3_STEP(2, buf2, buf1)
#undef HENN_X3_STEP
  }
  merge();
  if (qvalid) {
    const int64_t o = qrow * (2 * KS) + h * KS;
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      sl_d[o + j] = td[j];
      sl_i[o + j] = ti[j];
    }
  }
}

// Shortlist pass for rows wider than 128 coordinates (up to 1024), where
// a row block no longer fits in registers.  Same distances, same shortlist
// and the same folded norm step as k_gram_topk, arranged as a GEMM: a block
// owns 128 rows (32 per wave) and walks the layer in tiles of kWideC = 128
// candidates; the K dimension streams through LDS in slices of kSlice = 64
// coordinates (candidate slice and row slice, double buffered, fetched into
// registers one slice ahead).  Each wave multiplies its 32 rows against the
// tile's four 32-candidate blocks into four independent accumulators, the
// two lane halves covering the first and second half of each slice.
// Row values are pre-scaled by -2 (L2) or -1 (IP) when staged; coordinates
// past dpad are staged as zeros.
constexpr int kWideC = 128;
constexpr int kSlice = 64;
constexpr int kSStride = kSlice + 4;
constexpr int kF4Row = kSlice / 4;  // float4 per staged row slice = threads per row

__global__ __launch_bounds__(256) void k_knn_gram_wide(const float* vec, int64_t size,
                                                          int dpad, const float* mean,
                                                          const float* norms, int metric,
                                                          float* sl_d, int32_t* sl_i,
                                                          int64_t block0) {
  extern __shared__ __align__(16) float lds[];
  constexpr int kHalf = kWideC * kSStride;  // one operand slice
  constexpr int kBuf = 2 * kHalf;           // candidate slice + row slice
  float* mean_lds = lds + 2 * kBuf;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qc = lane & 31, h = lane >> 5;
  const int64_t qbase = (block0 + blockIdx.x) * 128;
  const int64_t qrow = qbase + wave * 32 + qc;
  const bool qvalid = qrow < size;
  const bool l2 = metric == 0;
  const float qscale = l2 ? -2.0f : -1.0f;
  const float b_extra = h == 0 ? 1.0f : (l2 && qvalid ? norms[qrow] : 0.0f);
  const float a_one = l2 ? 1.0f : 0.0f;

  float td[kShort];
  int32_t ti[kShort];
#pragma unroll
  for (int j = 0; j < kShort; ++j) {
    td[j] = INFINITY;
    ti[j] = -1;
  }
  if (mean)
    for (int e = threadIdx.x; e < dpad; e += 256) mean_lds[e] = mean[e];

  // thread -> (row, float4 column) of a slice: kF4Row threads cover one
  // row's kSlice coordinates, 256 / kF4Row rows per pass; the first kPass
  // slots stage candidate rows, the next kPass the block's rows
  constexpr int kRowsPerPass = 256 / kF4Row;
  constexpr int kPass = kWideC / kRowsPerPass;
  const int lrow = threadIdx.x / kF4Row, lc4 = threadIdx.x % kF4Row;
  const int nsl = (dpad + kSlice - 1) / kSlice;
  float4 pre[2 * kPass];
  auto fetch = [&](int64_t c0, int ks) {
    const int col = ks * kSlice + 4 * lc4;
    const int colc = col < dpad ? col : 0;
#pragma unroll
    for (int u = 0; u < 2 * kPass; ++u) {
      const int64_t base = u < kPass ? c0 : qbase;
      const int64_t row = min(base + lrow + kRowsPerPass * (u % kPass), size - 1);
      pre[u] = *reinterpret_cast<const float4*>(vec + row * dpad + colc);
    }
  };
  auto stash = [&](float* buf, int ks) {
    const int col = ks * kSlice + 4 * lc4;
    const bool cvalid = col < dpad;
    float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
    if (mean && cvalid) m = *reinterpret_cast<const float4*>(mean_lds + col);
#pragma unroll
    for (int u = 0; u < 2 * kPass; ++u) {
      float4 v = pre[u];
      v.x -= m.x; v.y -= m.y; v.z -= m.z; v.w -= m.w;
      if (u >= kPass) {
        v.x *= qscale; v.y *= qscale; v.z *= qscale; v.w *= qscale;
      }
      if (!cvalid) v = make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(buf + (u < kPass ? 0 : kHalf) +
                                 (lrow + kRowsPerPass * (u % kPass)) * kSStride + 4 * lc4) = v;
    }
  };
  auto tile_norms = [&](int64_t c0, float* cn) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t row = c0 + 32 * b + qc;
      const float nv = norms[min(row, size - 1)];
      cn[b] = row < size ? (l2 ? nv : 0.0f) : INFINITY;
    }
  };

  __syncthreads();
  fetch(0, 0);
  stash(lds, 0);
  __syncthreads();

  int cur = 0;
  for (int64_t c0 = 0; c0 < size; c0 += kWideC) {
    float cn[4];
    tile_norms(c0, cn);
    floatx16 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;

    for (int ks = 0; ks < nsl; ++ks) {
      // the next slice, crossing into the next tile after the last one
      const bool last = ks + 1 == nsl;
      const int nks = last ? 0 : ks + 1;
      const int64_t nc0 = last ? c0 + kWideC : c0;
      const bool more = nc0 < size;
      if (more) fetch(nc0, nks);

      const float* buf = lds + cur * kBuf;
      const float4* brow = reinterpret_cast<const float4*>(
          buf + kHalf + (wave * 32 + qc) * kSStride + (kSlice / 2) * h);
#pragma unroll
      for (int k4 = 0; k4 < kSlice / 8; ++k4) {
        const float4 bv = brow[k4];
        float4 av[4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
          av[b] = reinterpret_cast<const float4*>(buf + (32 * b + qc) * kSStride +
                                                  (kSlice / 2) * h)[k4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b].x, bv.x, acc[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b].y, bv.y, acc[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b].z, bv.z, acc[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[b].w, bv.w, acc[b], 0, 0, 0);
      }
      if (more) stash(lds + (cur ^ 1) * kBuf, nks);
      __syncthreads();
      cur ^= 1;
    }

#pragma unroll
    for (int b = 0; b < 4; ++b)
      acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(h == 0 ? cn[b] : a_one, b_extra, acc[b], 0,
                                                    0, 0);
    float lo = INFINITY;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) lo = fminf(lo, acc[b][v]);
    if (__builtin_amdgcn_ballot_w64(lo < td[kShort - 1])) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t crow = c0 + 32 * b + 8 * (v >> 2) + 4 * h + (v & 3);
          float nd = crow != qrow ? acc[b][v] : INFINITY;
          if (__builtin_amdgcn_ballot_w64(nd < td[kShort - 1])) {
            int32_t ni = (int32_t)crow;
#pragma unroll
            for (int j = 0; j < kShort; ++j) {
              const bool sw = nd < td[j];
              const float od = td[j];
              const int32_t oi = ti[j];
              td[j] = sw ? nd : od;
              ti[j] = sw ? ni : oi;
              nd = sw ? od : nd;
              ni = sw ? oi : ni;
            }
          }
        }
      }
    }
  }
  if (qvalid) {
    float* od = sl_d + qrow * (2 * kShort) + h * kShort;
    int32_t* oi = sl_i + qrow * (2 * kShort) + h * kShort;
#pragma unroll
    for (int j = 0; j < kShort; ++j) {
      od[j] = td[j];
      oi[j] = ti[j];
    }
  }
}

__device__ inline uint64_t wave_sort64(uint64_t key) {
  const int lane = lane_id();
  for (int size = 2; size <= 64; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t other = shfl_xor_u64(key, stride);
      const bool lower = (lane & stride) == 0;
      const bool asc = (lane & size) == 0;
      const bool take_min = lower == asc;
      key = take_min ? (key < other ? key : other) : (key < other ? other : key);
    }
  }
  return key;
}

template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_knn_rerank(const float* vec, int64_t size, int dpad,
                                                    int nchunks, int metric, const float* sl_d,
                                                    const int32_t* sl_i, const float* norms,
                                                    float nmax, float coef, int R, int32_t* adj,
                                                    int32_t* fb_rows, uint32_t* fb_count,
                                                    const int32_t* row_list, int64_t n_rows) {
  constexpr int G = 64 / LPN;
  __shared__ uint64_t keys[4][64];
  const int wave = threadIdx.x >> 6;
  // shortlist i belongs to row row_list[i] (or row i)
  const int64_t li = (int64_t)blockIdx.x * 4 + wave;
  if (li >= n_rows) return;
  const int64_t row = row_list ? (int64_t)row_list[li] : li;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  float q[CPL][8];
  load_query<CPL>(vec + row * dpad, dpad, t, q);
  for (int base = 0; base < 2 * kShort; base += G) {
    const int ci = base + g;
    const int32_t id = sl_i[li * (2 * kShort) + ci];
    const bool valid = id >= 0;
    const float dist = group_distance<kF32, LPN, CPL>(q, vec + (int64_t)(valid ? id : 0) * dpad,
                                                      1.0f, t, nchunks, metric, valid);
    if (t == 0) keys[wave][ci] = valid ? dkey(dist, id) : ~0ull;
  }
  wave_sync();
  const uint64_t key = wave_sort64(keys[wave][lane]);
  if (lane < R) adj[row * R + lane] = key == ~0ull ? -1 : (int32_t)(uint32_t)key;
  const float cut =
      fminf(sl_d[li * (2 * kShort) + kShort - 1], sl_d[li * (2 * kShort) + 2 * kShort - 1]);
  const uint64_t kr = shfl_u64(key, R - 1);
  if (lane == 0 && isfinite(cut)) {
    // every candidate left out of the shortlist has a Gram value >= cut, and
    // |G - D| <= coef (|x'|^2 + |y'|^2) for its canonical distance D
    const float exact_r = kr == ~0ull ? INFINITY : from_ordered((uint32_t)(kr >> 32));
    const float nrow = norms[row];
    // (a) with |y'|^2 <= max_y |y'|^2: D >= cut - delta
    const float delta = coef * (nrow + nmax);
    const bool proof_a = exact_r + delta < cut - delta;
    // (b) L2 only, relative to the candidate's own distance: |y'|^2 <=
    // 2 |x'|^2 + 2 |y - x|^2, so |G - D| <= coef (3 |x'|^2 + 2.1 D) and
    // D >= (cut - 3 coef |x'|^2) / (1 + 2.1 coef); the factors 3 and 4 below
    // leave room for the rounding of this test.  Rows of small norm in
    // multi-scale data pass here where (a) charges them the layer's largest.
    const bool proof_b =
        metric == 0 && exact_r * (1.0f + 3.0f * coef) + 4.0f * coef * nrow < cut;
    if (!(proof_a || proof_b)) fb_rows[atomicAdd(fb_count, 1u)] = (int32_t)row;
  }
}

// Exact brute force for one row per block: every group keeps a private
// sorted top-R of the keys it computes; the lists are merged in LDS.
template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_knn_exact(const float* vec, int64_t size, int dpad,
                                                   int nchunks, int metric, const int32_t* rows,
                                                   int R, int rpad, int32_t* adj) {
  constexpr int G = 64 / LPN;
  extern __shared__ uint64_t lists[];  // [4*G][rpad], then padded to a power of two
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  const int64_t row = rows[blockIdx.x];
  float q[CPL][8];
  load_query<CPL>(vec + row * dpad, dpad, t, q);
  uint64_t best[kShort];
#pragma unroll
  for (int j = 0; j < kShort; ++j) best[j] = ~0ull;
  const int group = wave * G + g;
  for (int64_t base = 0; base < size; base += 4 * G) {
    const int64_t c = base + group;
    const bool valid = c < size && c != row;
    const float dist = group_distance<kF32, LPN, CPL>(q, vec + (valid ? c : 0) * dpad, 1.0f, t,
                                                      nchunks, metric, valid);
    if (valid && t == 0) {
      uint64_t nk = dkey(dist, (int32_t)c);
      if (nk < best[kShort - 1]) {
#pragma unroll
        for (int j = 0; j < kShort; ++j) {
          const bool sw = nk < best[j];
          const uint64_t o = best[j];
          best[j] = sw ? nk : o;
          nk = sw ? o : nk;
        }
      }
    }
  }
  const int total = 4 * G * rpad;
  int n2 = 1;
  while (n2 < total) n2 <<= 1;
  if (t == 0) {
#pragma unroll
    for (int j = 0; j < kShort; ++j)
      if (j < rpad) lists[group * rpad + j] = best[j];
  }
  for (int i = total + threadIdx.x; i < n2; i += blockDim.x) lists[i] = ~0ull;
  __syncthreads();
  for (int sz = 2; sz <= n2; sz <<= 1) {
    for (int stride = sz >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (n2 >> 1); i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & sz) == 0;
        const uint64_t x = lists[lo], y = lists[hi];
        if ((x > y) == asc) {
          lists[lo] = y;
          lists[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < R; j += blockDim.x)
    adj[row * R + j] = lists[j] == ~0ull ? -1 : (int32_t)(uint32_t)lists[j];
}

#define HENN_KNN_COMBOS(X) \
  X(1, 1) X(2, 1) X(4, 1) X(2, 2) X(4, 2) X(8, 1) X(2, 4) X(4, 4) X(8, 2) X(16, 1) X(8, 4) \
  X(16, 2) X(4, 8) X(16, 4) X(16, 8)

int root_gram_splits(int64_t nq, int64_t root_size, int64_t* rows_per_split) {
  // About four 256-thread workgroups of k_root_gram_bf16 fit a CU, so 1024
  // run at once.  Pick the split count with the shortest makespan, (rounds
  // of 1024 workgroups) x (tiles per split), the fewest splits among equals;
  // at least 4 tiles per split.
  const int64_t qblocks = (nq + 127) / 128;
  const int64_t tiles = (root_size + kTileC - 1) / kTileC;
  const int64_t max_splits = std::min<int64_t>(64, std::max<int64_t>(1, tiles / 4));
  int64_t splits = 1, best = -1;
  for (int64_t sp = 1; sp <= max_splits; ++sp) {
    const int64_t rounds = (qblocks * sp + 1023) / 1024;
    const int64_t span = rounds * ((tiles + sp - 1) / sp);
    if (best < 0 || span < best) {
      best = span;
      splits = sp;
    }
  }
  int64_t per = (root_size + splits - 1) / splits;
  per = (per + kTileC - 1) / kTileC * kTileC;
  *rows_per_split = per;
  return (int)((root_size + per - 1) / per);
}

// ------------------------------------------------------------------------
// Complete-root scan on BF16 matrix cores (the shortlist half of the root
// query of Alg. 4 on a complete root; the exact check follows in
// k_root_check).  The root is prepared once (prepare_root_bf16): rows
// centred on the root mean (L2) and rounded to BF16, [rows_pad][kp] with kp
// = dpad rounded up to 16 and rows_pad = size rounded up to 32, and a norm
// column that is +inf for the padding rows.  A block takes 128 queries, one
// 32-query column block per wave, and walks its split of the root 32 rows
// at a time; per tile a wave issues kp / 16 v_mfma_f32_32x32x16_bf16 with
//   A = 32 root rows (lane: row lane & 31, coordinates 16 s + 8 h .. + 7)
//   B = the wave's 32 queries, as bf16 of -2 (q - mean) (L2) or -q (IP)
// so that acc + norm is the Gram value a(y), |y - q|^2 - |q - mean|^2 (L2)
// or -<y, q> (IP) up to the BF16 rounding, which the margin covers.  The
// query operand stays in registers for the whole scan; the root tiles pass
// through LDS, copied ahead of the tile being multiplied (see the ring below).
//
// Two passes over the split: the first keeps only the smallest Gram value
// and merges it into the query's running minimum over the splits; the
// second appends every row within the query's margin M of the smaller of
// the two (normally a handful) to the query's list.  The exact nearest is
// within M of the smallest Gram value over the whole root, hence of any
// larger threshold, so the list holds it.  M = (2^-7 + 2^-14 +
// 32 (dpad + 16) 2^-24) N with N = |q - mean|^2 + max_y |y - mean|^2 +
// |mean|^2 (twice the sum of the Gram and canonical error bounds, derived
// at k_root_check).
// ------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__global__ void k_root_rows_bf16(const float* dec, const float* mean, const float* norm,
                                 int64_t size, int64_t rows_pad, int dpad, int kp, int metric,
                                 uint16_t* rowb, float* normp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows_pad * kp) return;
  const int64_t r = i / kp;
  const int c = (int)(i - r * kp);
  float v = 0.0f;
  if (r < size && c < dpad) v = dec[r * dpad + c] - (mean ? mean[c] : 0.0f);
  rowb[i] = (uint16_t)f32_to_bf16_rne(v);
  if (c == 0) normp[r] = r < size ? (metric == 0 ? norm[r] : 0.0f) : INFINITY;
}

void prepare_root_bf16(RootAux& r, int dpad, int metric, hipStream_t st) {
  if (dpad > 128) throw HipError{hipErrorInvalidValue, "BF16 root scan supports d <= 128"};
  r.kp = (dpad + 15) / 16 * 16;
  const int64_t rows_pad = (r.size + 31) / 32 * 32;
  HENN_HIP(dev_alloc(reinterpret_cast<void**>(&r.rowb), sizeof(uint16_t) * rows_pad * r.kp));
  HENN_HIP(dev_alloc(reinterpret_cast<void**>(&r.normp), sizeof(float) * rows_pad));
  const int64_t n = rows_pad * r.kp;
  hipLaunchKernelGGL(k_root_rows_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     r.dec, r.mean, r.norm, r.size, rows_pad, dpad, r.kp, metric, r.rowb,
                     r.normp);
  HENN_HIP(hipGetLastError());
}

int64_t root_shortlist_bytes(int64_t nq, int kp) {
  return 256 + nq * kp * 2 + nq * 12 + nq * kRootCap * 8;
}

RootShortlist root_shortlist_at(void* base, int64_t nq, int kp) {
  RootShortlist sl;
  sl.ent = reinterpret_cast<uint2*>((reinterpret_cast<uintptr_t>(base) + 255) & ~uintptr_t(255));
  sl.qb = reinterpret_cast<uint16_t*>(sl.ent + nq * kRootCap);
  sl.mq = reinterpret_cast<float*>(sl.qb + nq * kp);
  sl.qmin = reinterpret_cast<uint32_t*>(sl.mq + nq);
  sl.cnt = reinterpret_cast<int32_t*>(sl.qmin + nq);
  return sl;
}

// The Gram pass's query operand, once per query: eight coordinates per
// thread (16 threads per query), centred on the root mean (L2), scaled by -2
// (L2) or -1 (IP) and rounded to BF16, zero past d; the empty list and the
// running minimum at +inf; and the query's margin
// M = (2^-7 + 2^-14 + 32 (dpad + 16) 2^-24) N with
// N = |q - mean|^2 + max_y |y - mean|^2 + |mean|^2 (twice the sum of the
// Gram and canonical error bounds, derived at k_root_check).
__global__ __launch_bounds__(256) void k_root_query_bf16(const float* Q, int64_t nq, int d,
                                                         int dpad, int kp, const float* mean,
                                                         float nmax, float mean_n2, int metric,
                                                         RootShortlist sl) {
  const int64_t qi = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int c = threadIdx.x & 15;
  const bool live = qi < nq && 8 * c < kp;
  const float qscale = metric == 0 ? -2.0f : -1.0f;
  float qn = 0.0f;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  if (live) {
    float x[8], m[8];
    if ((d & 3) == 0 && (reinterpret_cast<uintptr_t>(Q) & 15) == 0 && 8 * c + 8 <= d) {
      // whole 16-byte chunks of the row (every row starts 16-byte aligned)
      const float4* qr = reinterpret_cast<const float4*>(Q + qi * d + 8 * c);
      const float4 x0 = qr[0], x1 = qr[1];
      x[0] = x0.x, x[1] = x0.y, x[2] = x0.z, x[3] = x0.w;
      x[4] = x1.x, x[5] = x1.y, x[6] = x1.z, x[7] = x1.w;
    } else {
      // loads clamped into the row and issued together; values past d dropped
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = Q[qi * d + min(8 * c + j, d - 1)];
    }
    if (mean) {
#pragma unroll
      for (int j = 0; j < 8; ++j) m[j] = mean[min(8 * c + j, d - 1)];
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) m[j] = 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
      const int e0 = 8 * c + j, e1 = e0 + 1;
      const float v0 = e0 < d ? x[j] - m[j] : 0.0f;
      const float v1 = e1 < d ? x[j + 1] - m[j + 1] : 0.0f;
      qn = __builtin_fmaf(v0, v0, qn);
      qn = __builtin_fmaf(v1, v1, qn);
      w[j >> 1] = f32_to_bf16_rne(qscale * v0) | (f32_to_bf16_rne(qscale * v1) << 16);
    }
    reinterpret_cast<uint4*>(sl.qb + qi * kp)[c] = make_uint4(w[0], w[1], w[2], w[3]);
  }
#pragma unroll
  for (int m = 8; m >= 1; m >>= 1) qn += __shfl_xor(qn, m);
  if (qi < nq && c == 0) {
    sl.mq[qi] = (0x1p-7f + 0x1p-14f + 32.0f * (float)(dpad + 16) * 0x1p-24f) *
                (qn + nmax + mean_n2);
    sl.qmin[qi] = ordered_bits(INFINITY);
    sl.cnt[qi] = 0;
  }
}

template <int I>
struct Ic {
  static constexpr int value = I;
};

template <int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_root_gram_bf16(
    const uint16_t* rowb, const float* normp, int64_t size, int64_t nq, int64_t rows_per_split,
    RootShortlist sl) {
  constexpr int kp = 16 * S;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qc = lane & 31, h = lane >> 5;
  const int64_t qrow = (int64_t)blockIdx.x * 128 + wave * 32 + qc;
  const bool qvalid = qrow < nq;
  const int64_t cb = (int64_t)blockIdx.y * rows_per_split;
  const int64_t ce = min(cb + rows_per_split, size);

  // B operand: this lane's query coordinates 16 s + 8 h .. + 7
  bf16x8 bq[S];
  {
    const uint4* src = reinterpret_cast<const uint4*>(sl.qb + (qvalid ? qrow : 0) * kp) + h;
#pragma unroll
    for (int s = 0; s < S; ++s) bq[s] = __builtin_bit_cast(bf16x8, src[2 * s]);
  }
  const float M = qvalid ? sl.mq[qrow] : 0.0f;

  // Tiles are staged in LDS, shared by the block's four waves, by the
  // global-to-LDS copy of gfx950 (global_load_lds_dwordx4): one instruction
  // moves 64 chunks of 16 bytes into 64 consecutive slots.  A tile row takes
  // 2S + 1 slots (its 2S chunks, then one pad slot, so that the 32 rows of
  // one step's reads fall on different banks), S + 1 instructions a tile,
  // instruction j issued by wave j mod 4; pad slots receive a copy of the
  // row's first chunk.  Each wave also copies 8 of the tile's 32 norms
  // (lanes 0..7, one dword each).  rows_per_split is a multiple of 32 and
  // the prepared rows are padded to a multiple of 32, so every tile row
  // below ce rounded up to 32 exists (rows at or past size carry norm +inf
  // and never enter a list).  Three buffers in a ring (the norms after the
  // rows): the copies of the next two tiles are in flight while one is
  // multiplied.
  constexpr int kRowSlots = 2 * S + 1;
  constexpr int kTileU4 = 64 * (S + 1);  // >= 32 * kRowSlots
  constexpr int kBufU4 = kTileU4 + 8;
  __shared__ uint4 buf0[kBufU4], buf1[kBufU4], buf2[kBufU4];
  auto buf_of = [&](auto I) -> uint4* {
    if constexpr (decltype(I)::value == 0) return buf0;
    else if constexpr (decltype(I)::value == 1) return buf1;
    else return buf2;
  };
  typedef __attribute__((address_space(3))) void* lds_ptr;
  // this wave's copy instructions j = wave, wave + 4, ... < S + 1 (at most
  // three); a lane's source offset within the tile depends on (j, lane) only
  constexpr int kMaxJ = (S + 4) / 4;
  const int per_tile = (S + 1 - wave + 3) / 4 + 1;  // copy instructions of this wave per tile
  auto issue = [&](int64_t c0, uint4* tile) {
    const uint16_t* src = rowb + c0 * kp;
#pragma unroll
    for (int u = 0; u < kMaxJ; ++u) {
      const int j = wave + 4 * u;
      if (j < S + 1) {
        const int p = 64 * j + lane, r = p / kRowSlots, c = p - r * kRowSlots;
        const int off = min(r, 31) * kp + 8 * ((p < 32 * kRowSlots && c < 2 * S) ? c : 0);
        __builtin_amdgcn_global_load_lds(src + off, (lds_ptr)(tile + 64 * j), 16, 0, 0);
      }
    }
    if (lane < 8)
      __builtin_amdgcn_global_load_lds(normp + c0 + 8 * wave + lane,
                                       (lds_ptr)(reinterpret_cast<float*>(tile + kTileU4) + 8 * wave),
                                       4, 0, 0);
  };
  // waits until at most n of this wave's vector memory operations are
  // outstanding.  Loads complete in order, so the copies issued before the
  // last n operations are done.  Inside a scan the only other operations are
  // the running-minimum atomic and pass 2's list writes, which can only make
  // the wait longer.
  auto wait_copies = [](int n) {
    switch (n) {
      case 0: __builtin_amdgcn_s_waitcnt(0xF70); break;
      case 1: __builtin_amdgcn_s_waitcnt(0xF71); break;
      case 2: __builtin_amdgcn_s_waitcnt(0xF72); break;
      case 3: __builtin_amdgcn_s_waitcnt(0xF73); break;
      case 4: __builtin_amdgcn_s_waitcnt(0xF74); break;
      case 5: __builtin_amdgcn_s_waitcnt(0xF75); break;
      default: __builtin_amdgcn_s_waitcnt(0xF76); break;
    }
  };
  // one tile's Gram values, the norms entering as the accumulator's start;
  // val[v] belongs to root row c0 + 8 (v >> 2) + 4 h + (v & 3)
  auto gram = [&](const uint4* tile, floatx16& val) {
    const float* nrm = reinterpret_cast<const float*>(tile + kTileU4);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 nr = reinterpret_cast<const float4*>(nrm)[2 * g + h];
      val[4 * g + 0] = nr.x;
      val[4 * g + 1] = nr.y;
      val[4 * g + 2] = nr.z;
      val[4 * g + 3] = nr.w;
    }
    const uint4* arow = tile + qc * kRowSlots + h;
#pragma unroll
    for (int s = 0; s < S; ++s)
      val = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, arow[2 * s]), bq[s],
                                                    val, 0, 0, 0);
  };
  auto tile_min = [](const floatx16& val) {
    float m = val[0];
#pragma unroll
    for (int v = 1; v < 16; ++v) m = fminf(m, val[v]);
    return m;
  };
  // Workgroup barrier for the ring.  __syncthreads() would also wait for
  // every outstanding copy (its release fence), including those of the
  // tiles ahead; the copies a tile needs were waited for above, and LDS
  // itself is coherent within the workgroup, so a plain barrier suffices.
  // The memory clobber keeps the compiler from moving LDS accesses across it.
  auto lds_barrier = []() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); };
  // every wave of the block walks the same tiles (the barriers need all of
  // them, so no wave leaves early)
  auto scan = [&](auto&& body) {
    if (cb >= ce) return;
    const int nt = (int)((ce - cb + 31) / 32);
    issue(cb, buf0);
    if (nt > 1) issue(cb + 32, buf1);
    auto step = [&](int t, auto I) {
      constexpr int i = decltype(I)::value;
      // this wave's copies of tile t are done once only those of the tile
      // issued after it (if any) remain; the barrier covers the other waves'
      wait_copies(t + 1 < nt ? per_tile : 0);
      lds_barrier();
      // into the buffer of tile t - 1, which every wave has finished with
      if (t + 2 < nt) issue(cb + 32 * (t + 2), buf_of(Ic<(i + 2) % 3>{}));
      body(cb + 32 * t, buf_of(I));
    };
    for (int t = 0; t < nt; t += 3) {
      step(t, Ic<0>{});
      if (t + 1 >= nt) break;
      step(t + 1, Ic<1>{});
      if (t + 2 >= nt) break;
      step(t + 2, Ic<2>{});
    }
    __syncthreads();  // the next scan refills the ring
  };

  // pass 1: the split's smallest Gram value of this query, merged into the
  // query's running minimum over the splits
  float vmin = INFINITY;
  scan([&](int64_t, const uint4* tile) {
    floatx16 val;
    gram(tile, val);
    vmin = fminf(vmin, tile_min(val));
  });
  vmin = fminf(vmin, __shfl_xor(vmin, 32));
  // the running minimum before this split's entered it (both lanes of a
  // query ask); its value is first needed after pass 2's first copies are
  // issued, so the two latencies overlap
  const uint32_t run_old = qvalid ? atomicMin(sl.qmin + qrow, ordered_bits(vmin))
                                  : ordered_bits(INFINITY);

  // pass 2: the rows within M of the smaller of the split's minimum and the
  // running minimum it met (both at or above the root's minimum).
  // A lane keeps the rows it finds in registers (up to four; normally one or
  // two) and publishes them after the scan with one global atomic: a wait
  // for an atomic's returned value inside the scan also waits for every copy
  // in flight.  A lane whose rows would not fit publishes at once.
  uint2* lent = sl.ent + (qvalid ? qrow : 0) * kRootCap;
  int nkept = 0;
  uint2 f0 = make_uint2(0u, 0u), f1 = f0, f2 = f0, f3 = f0;
  auto publish_kept = [&]() {
    const int pos = atomicAdd(sl.cnt + qrow, nkept);
    if (pos < kRootCap) lent[pos] = f0;
    if (nkept > 1 && pos + 1 < kRootCap) lent[pos + 1] = f1;
    if (nkept > 2 && pos + 2 < kRootCap) lent[pos + 2] = f2;
    if (nkept > 3 && pos + 3 < kRootCap) lent[pos + 3] = f3;
    nkept = 0;
  };
  scan([&](int64_t c0, const uint4* tile) {
    const float thr = fminf(vmin, from_ordered(run_old)) + M;
    floatx16 val;
    gram(tile, val);
    if (__builtin_amdgcn_ballot_w64(qvalid && tile_min(val) <= thr)) {
      uint32_t hit = 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) hit |= (qvalid && val[v] <= thr) ? 1u << v : 0u;
      const int nh = __popc(hit);
      if (nh > 0 && nkept + nh > 4) {
        if (nkept > 0) publish_kept();
        int pos = atomicAdd(sl.cnt + qrow, nh);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          if (hit & (1u << v)) {
            if (pos < kRootCap)
              lent[pos] = make_uint2(__float_as_uint(val[v]),
                                     (uint32_t)(c0 + 8 * (v >> 2) + 4 * h + (v & 3)));
            ++pos;
          }
        }
      } else if (nh > 0) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          if (hit & (1u << v)) {
            const uint2 e = make_uint2(__float_as_uint(val[v]),
                                       (uint32_t)(c0 + 8 * (v >> 2) + 4 * h + (v & 3)));
            f0 = nkept == 0 ? e : f0;
            f1 = nkept == 1 ? e : f1;
            f2 = nkept == 2 ? e : f2;
            f3 = nkept == 3 ? e : f3;
            ++nkept;
          }
        }
      }
    }
  });
  if (nkept > 0) publish_kept();
}

void launch_root_gram(const float* Q, int64_t nq, int d, const RootAux& r, int dpad, int metric,
                      int splits, int64_t rows_per_split, const RootShortlist& sl,
                      hipStream_t st) {
  if (!r.rowb || rows_per_split % 32 != 0 || r.kp > 128)
    throw HipError{hipErrorInvalidValue, "root scan: root not prepared"};
  hipLaunchKernelGGL(k_root_query_bf16, dim3((unsigned)((nq + 15) / 16)), dim3(256), 0, st, Q, nq,
                     d, dpad, r.kp, r.mean, r.nmax, r.mean_n2, metric, sl);
  const dim3 grid((unsigned)((nq + 127) / 128), (unsigned)splits);
#define HENN_RG(S)                                                                               \
  hipLaunchKernelGGL((k_root_gram_bf16<S>), grid, dim3(256), 0, st, r.rowb, r.normp, r.size, nq, \
                     rows_per_split, sl)
  switch (r.kp / 16) {
    case 1: HENN_RG(1); break;
    case 2: HENN_RG(2); break;
    case 3: HENN_RG(3); break;
    case 4: HENN_RG(4); break;
    case 5: HENN_RG(5); break;
    case 6: HENN_RG(6); break;
    case 7: HENN_RG(7); break;
    case 8: HENN_RG(8); break;
    default: throw HipError{hipErrorInvalidValue, "root scan: unsupported width"};
  }
#undef HENN_RG
  HENN_HIP(hipGetLastError());
}

int64_t build_knn_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric, int R,
                        int lpn, int cpl, int32_t* adj, int gram, hipStream_t st) {
  if (size <= 0) return 0;
  if (dpad > 1024) throw HipError{hipErrorInvalidValue, "kNN build supports d <= 1024"};
  DevBuf<float> norms_buf(size), sl_d_buf(size * 2 * kShort), mean_buf(metric == 0 ? dpad : 1);
  DevBuf<int32_t> sl_i_buf(size * 2 * kShort), fb_rows_buf(size);
  DevBuf<uint32_t> fb_count_buf(1);
  float *norms = norms_buf.get(), *sl_d = sl_d_buf.get();
  float* mean = metric == 0 ? mean_buf.get() : nullptr;
  int32_t *sl_i = sl_i_buf.get(), *fb_rows = fb_rows_buf.get();
  uint32_t* fb_count = fb_count_buf.get();
  HENN_HIP(hipMemsetAsync(fb_count, 0, sizeof(uint32_t), st));
  if (metric == 0) layer_mean(vec, size, dpad, mean, st);
  launch_row_norms(vec, mean, size, dpad, norms, st);
  const float nmax = max_norm(norms, size, st);

  const int kh = dpad <= 32 ? 16 : dpad <= 64 ? 32 : 64;
  const bool wide = dpad > 128;
  // the split-BF16 form for d <= 128 unless FP32 tiles are asked for
  const bool split = !wide && gram == 0;
  const int kp = (dpad + 15) / 16 * 16;
  // the FP32 tiles' bound: 4 (dpad + 8) 2^-24 (|x'|^2 + max |y'|^2)
  const float coef = split ? x3_split_coef(dpad) : 4.0f * (float)(dpad + 8) * 0x1p-24f;
  // the split rows and their tile norms, padded to whole tiles
  const int64_t size_pad = (size + kTileC - 1) / kTileC * kTileC;
  DevBuf<uint16_t> split_buf(split ? size_pad * 2 * kp : 1);
  DevBuf<float> tnorm_buf(split ? size_pad : 1);
  if (split) {
    const int64_t n = size_pad * kp;
    hipLaunchKernelGGL(k_split_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, vec,
                       mean, norms, metric, size, size_pad, dpad, kp, split_buf.get(),
                       tnorm_buf.get());
    HENN_HIP(hipGetLastError());
  }
  const size_t lds = wide    ? sizeof(float) * (4 * kWideC * kSStride + dpad)
                     : split ? 0  // static LDS
                             : sizeof(float) * (2 * (kTileC * (2 * kh + 4) + kTileC) + dpad);
  // FP32 Gram tiles over row blocks [b0, b0 + nbs) of the given rows
  auto launch_fp32_gram = [&](int64_t b0, unsigned nbs, const int32_t* row_list,
                              int64_t n_rows) {
    const size_t lds32 = sizeof(float) * (2 * (kTileC * (2 * kh + 4) + kTileC) + dpad);
    if (kh <= 16)
      hipLaunchKernelGGL((k_gram_topk<16, kShort>), dim3(nbs), dim3(256), lds32, st, vec, size,
                         dpad, norms, mean, metric, sl_d, sl_i, b0, row_list, n_rows);
    else if (kh <= 32)
      hipLaunchKernelGGL((k_gram_topk<32, kShort>), dim3(nbs), dim3(256), lds32, st, vec, size,
                         dpad, norms, mean, metric, sl_d, sl_i, b0, row_list, n_rows);
    else
      hipLaunchKernelGGL((k_gram_topk<64, kShort>), dim3(nbs), dim3(256), lds32, st, vec, size,
                         dpad, norms, mean, metric, sl_d, sl_i, b0, row_list, n_rows);
  };
  const int64_t nb = (size + 127) / 128;
  // Launch in slices of row blocks so that very large layers report progress
  // (HENN_PROGRESS=1) between slices; each slice is a full-width Gram sweep.
  const bool progress = getenv("HENN_PROGRESS") != nullptr;
  const int64_t slice = std::max<int64_t>(4096, (int64_t)(2e13 / ((double)size * dpad * 256.0)));
  auto t_last = std::chrono::steady_clock::now();
  for (int64_t b0 = 0; b0 < nb; b0 += slice) {
    const unsigned nbs = (unsigned)std::min<int64_t>(slice, nb - b0);
    if (wide)
      hipLaunchKernelGGL(k_knn_gram_wide, dim3(nbs), dim3(256), lds, st, vec, size, dpad, mean,
                         norms, metric, sl_d, sl_i, b0);
    else if (split) {
      switch (kp / 16) {
#define HENN_X3(S_)                                                                           \
  case S_:                                                                                    \
    hipLaunchKernelGGL((k_gram_topk_x3<S_, kShort>), dim3(nbs), dim3(256), lds, st,           \
                       split_buf.get(), size, norms, tnorm_buf.get(), metric, sl_d, sl_i, b0); \
    break;
        HENN_X3(1) HENN_X3(2) HENN_X3(3) HENN_X3(4) HENN_X3(5) HENN_X3(6) HENN_X3(7) HENN_X3(8)
#undef HENN_X3
        default:
          throw HipError{hipErrorInvalidValue, "split Gram: d <= 128"};
      }
    } else {
      launch_fp32_gram(b0, nbs, nullptr, size);
    }
    HENN_HIP(hipGetLastError());
    if (progress && b0 + (int64_t)nbs < nb) {
      HENN_HIP(hipStreamSynchronize(st));
      const auto now = std::chrono::steady_clock::now();
      if (std::chrono::duration<double>(now - t_last).count() > 20.0) {
        fprintf(stderr, "[henn] kNN graph of %lld rows: %lld row blocks of %lld done\n",
                (long long)size, (long long)(b0 + nbs), (long long)nb);
        t_last = now;
      }
    }
  }

  // re-rank and proof of n_rows shortlists (of rows row_list[i], or row i);
  // unproven rows are appended to out_rows
  auto rerank = [&](const int32_t* row_list, int64_t n_rows, float c, int32_t* out_rows,
                    uint32_t* out_count) {
    const unsigned nr = (unsigned)((n_rows + 3) / 4);
    bool launched = false;
#define HENN_TRY(L, C)                                                                         \
  if (!launched && lpn == L && cpl == C) {                                                     \
    hipLaunchKernelGGL((k_knn_rerank<L, C>), dim3(nr), dim3(256), 0, st, vec, size, dpad,      \
                       nchunks, metric, sl_d, sl_i, norms, nmax, c, R, adj, out_rows,          \
                       out_count, row_list, n_rows);                                           \
    launched = true;                                                                           \
  }
    HENN_KNN_COMBOS(HENN_TRY)
#undef HENN_TRY
    if (!launched) throw HipError{hipErrorInvalidValue, "no rerank kernel for this lane shape"};
  };
  auto count_of = [&](uint32_t* dev_count) {
    uint32_t n = 0;
    HENN_HIP(hipMemcpyAsync(&n, dev_count, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HENN_HIP(hipStreamSynchronize(st));
    return n;
  };
  rerank(nullptr, size, coef, fb_rows, fb_count);
  uint32_t nfb = count_of(fb_count);
  if (nfb > 0 && split) {
    // the rows the split form could not prove: FP32 tiles on just those rows
    // (128 rows share each pass over the layer, where the brute force below
    // reads the whole layer once per row), then the FP32 proof
    DevBuf<int32_t> fb2_buf(nfb);
    DevBuf<uint32_t> fb2_count(1);
    HENN_HIP(hipMemsetAsync(fb2_count.get(), 0, sizeof(uint32_t), st));
    launch_fp32_gram(0, (unsigned)((nfb + 127) / 128), fb_rows, nfb);
    HENN_HIP(hipGetLastError());
    rerank(fb_rows, nfb, 4.0f * (float)(dpad + 8) * 0x1p-24f, fb2_buf.get(), fb2_count.get());
    nfb = count_of(fb2_count.get());
    if (nfb > 0)
      HENN_HIP(hipMemcpyAsync(fb_rows, fb2_buf.get(), sizeof(int32_t) * nfb,
                              hipMemcpyDeviceToDevice, st));
  }
  if (nfb > 0) {
    const int G = 64 / lpn;
    const int rpad = R;
    int n2 = 1;
    while (n2 < 4 * G * rpad) n2 <<= 1;
    const size_t lds2 = sizeof(uint64_t) * n2;
    bool launched = false;
#define HENN_TRY(L, C)                                                                          \
  if (!launched && lpn == L && cpl == C) {                                                      \
    hipLaunchKernelGGL((k_knn_exact<L, C>), dim3(nfb), dim3(256), lds2, st, vec, size, dpad,    \
                       nchunks, metric, fb_rows, R, rpad, adj);                                 \
    launched = true;                                                                            \
  }
    HENN_KNN_COMBOS(HENN_TRY)
#undef HENN_TRY
  }
  HENN_HIP(hipStreamSynchronize(st));
  return (int64_t)nfb;
}

// ---------------------------------------------------------- kNN_SYM -----
// Reverse edges: in-degree count, exclusive scan, scatter of the in-lists,
// then one wave per node merges its out- and in-neighbours by (distance, id)
// in chunks of 64 keys (sort the chunk, keep the lowest 64 of running list
// and chunk with a bitonic half-cleaner) and writes the first max_deg.
// Diversity pruning of a layer's candidate lists (App. B.2 navigable graphs:
// the neighbour selection of NSW/HNSW-style graphs).  One wave per row v;
// the C <= 32 candidates of adj_in (ascending (distance, id), -1 padded)
// are taken in order and a candidate c is dropped when an already kept r
// has d(c, r) < d(c, v), until R are kept.  All distances are the
// canonical FP32 ones: d(v, c_j) first, then the candidate pairs
// d(c_i, c_j), i < j (the difference form is symmetric in its arguments),
// into a per-wave LDS matrix; the scan is then a ballot per candidate.
template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_prune(const float* vec, int64_t size, int dpad,
                                               int nchunks, int metric, const int32_t* adj_in,
                                               int C, int R, int32_t* adj_out) {
  constexpr int G = 64 / LPN;
  __shared__ float D[4][32][33];
  __shared__ float dv[4][32];
  __shared__ int32_t cid[4][32];
  const int w = threadIdx.x >> 6;
  const int64_t v = (int64_t)blockIdx.x * 4 + w;
  if (v >= size) return;  // whole wave
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  const int32_t my = lane < C ? adj_in[v * C + lane] : -1;
  const int nc = popc64(ballot(my >= 0));  // candidates form a prefix
  if (lane < 32) cid[w][lane] = my;
  wave_sync();

  float q[CPL][8];
  load_query<CPL>(vec + v * dpad, dpad, t, q);
  for (int base = 0; base < nc; base += 2 * G) {
    const int j0 = base + g, j1 = base + G + g;
    const bool v0 = j0 < nc, v1 = j1 < nc;
    const void* const rows[2] = {vec + (int64_t)cid[w][v0 ? j0 : base] * dpad,
                                 vec + (int64_t)cid[w][v1 ? j1 : base] * dpad};
    const float sc[2] = {1.0f, 1.0f};
    const bool vd[2] = {v0, v1};
    float dd[2];
    group_distances<kF32, LPN, CPL, 2>(q, rows, sc, t, nchunks, metric, vd, dd);
    if (t == 0) {
      if (v0) dv[w][j0] = dd[0];
      if (v1) dv[w][j1] = dd[1];
    }
  }
  for (int i = 0; i + 1 < nc; ++i) {
    load_query<CPL>(vec + (int64_t)cid[w][i] * dpad, dpad, t, q);
    for (int base = i + 1; base < nc; base += 2 * G) {
      const int j0 = base + g, j1 = base + G + g;
      const bool v0 = j0 < nc, v1 = j1 < nc;
      const void* const rows[2] = {vec + (int64_t)cid[w][v0 ? j0 : base] * dpad,
                                   vec + (int64_t)cid[w][v1 ? j1 : base] * dpad};
      const float sc[2] = {1.0f, 1.0f};
      const bool vd[2] = {v0, v1};
      float dd[2];
      group_distances<kF32, LPN, CPL, 2>(q, rows, sc, t, nchunks, metric, vd, dd);
      if (t == 0) {
        if (v0) { D[w][i][j0] = dd[0]; D[w][j0][i] = dd[0]; }
        if (v1) { D[w][i][j1] = dd[1]; D[w][j1][i] = dd[1]; }
      }
    }
  }
  wave_sync();
  uint32_t kept = 0;
  int nk = 0;
  for (int j = 0; j < nc && nk < R; ++j) {
    const bool closer = lane < j && ((kept >> lane) & 1u) && D[w][j][lane] < dv[w][j];
    if (!ballot(closer)) {
      kept |= 1u << j;
      if (lane == 0) adj_out[v * R + nk] = cid[w][j];
      ++nk;
    }
  }
  for (int r = nk + lane; r < R; r += 64) adj_out[v * R + r] = -1;
}

void prune_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric,
                 const int32_t* adj_in, int C, int R, int32_t* adj_out, int lpn, int cpl,
                 hipStream_t st) {
  if (size <= 0) return;
  if (C > 32 || R > C) throw HipError{hipErrorInvalidValue, "prune: C <= 32 and R <= C"};
  const unsigned nb = (unsigned)((size + 3) / 4);
  bool launched = false;
#define HENN_TRY(L, CP)                                                                         \
  if (!launched && lpn == L && cpl == CP) {                                                     \
    hipLaunchKernelGGL((k_prune<L, CP>), dim3(nb), dim3(256), 0, st, vec, size, dpad, nchunks, \
                       metric, adj_in, C, R, adj_out);                                          \
    launched = true;                                                                            \
  }
  HENN_KNN_COMBOS(HENN_TRY)
#undef HENN_TRY
  if (!launched) throw HipError{hipErrorInvalidValue, "no prune kernel for this lane shape"};
  HENN_HIP(hipGetLastError());
}

__global__ void k_indeg(const int32_t* adj, int64_t edges, uint32_t* cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= edges) return;
  const int32_t u = adj[e];
  if (u >= 0) atomicAdd(cnt + u, 1u);
}

// in-lists: row r of adj (R entries) is the source src_base + r
__global__ void k_scatter_in(const int32_t* adj, int64_t edges, int R, int64_t src_base,
                             uint32_t* cursor, int32_t* inl) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= edges) return;
  const int32_t u = adj[e];
  if (u >= 0) inl[atomicAdd(cursor + u, 1u)] = (int32_t)(src_base + e / R);
}

template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_sym_merge(const float* vec, int64_t size, int dpad,
                                                   int nchunks, int metric,
                                                   const int32_t* adj_knn, int R,
                                                   const uint32_t* off, const int32_t* inl, int M,
                                                   int32_t* out) {
  constexpr int G = 64 / LPN;
  __shared__ int32_t outids[4][32];
  __shared__ int32_t cids[4][64];
  __shared__ uint64_t keys[4][64];
  const int w = threadIdx.x >> 6;
  const int64_t v = (int64_t)blockIdx.x * 4 + w;
  if (v >= size) return;
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  if (lane < 32) outids[w][lane] = lane < R ? adj_knn[v * R + lane] : -1;
  wave_sync();
  float q[CPL][8];
  load_query<CPL>(vec + v * dpad, dpad, t, q);
  const int64_t ib = off[v];
  const int64_t total = R + (int64_t)(off[v + 1] - off[v]);
  uint64_t best = ~0ull;
  for (int64_t base = 0; base < total; base += 64) {
    const int64_t j = base + lane;
    int32_t cid = -1;
    if (j < R) {
      cid = outids[w][j];
    } else if (j < total) {
      const int32_t u = inl[ib + (j - R)];
      bool dup = false;
      for (int r = 0; r < R; ++r) dup |= outids[w][r] == u;
      cid = dup ? -1 : u;
    }
    cids[w][lane] = cid;
    wave_sync();
    for (int pb = 0; pb < 64; pb += G) {
      const int ci = pb + g;
      const int32_t id = cids[w][ci];
      const bool valid = id >= 0;
      const float dist = group_distance<kF32, LPN, CPL>(
          q, vec + (int64_t)(valid ? id : 0) * dpad, 1.0f, t, nchunks, metric, valid);
      if (t == 0) keys[w][ci] = valid ? dkey(dist, id) : ~0ull;
    }
    wave_sync();
    const uint64_t c = wave_sort64(keys[w][lane]);
    const uint64_t rc = shfl_u64(c, 63 - lane);
    uint64_t m = rc < best ? rc : best;
    for (int stride = 32; stride > 0; stride >>= 1) {
      const uint64_t o = shfl_xor_u64(m, stride);
      const bool lower = (lane & stride) == 0;
      m = lower ? (o < m ? o : m) : (o < m ? m : o);
    }
    best = m;
    wave_sync();
  }
  if (lane < M) out[v * M + lane] = best == ~0ull ? -1 : (int32_t)(uint32_t)best;
}

void symmetrize_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric,
                      const int32_t* adj_knn, int R, int32_t* adj_out, int max_deg, int lpn,
                      int cpl, hipStream_t st) {
  const int64_t edges = size * R;
  DevBuf<uint32_t> cnt_buf(size + 1), off_buf(size + 1);
  DevBuf<int32_t> inl_buf(edges);
  uint32_t *cnt = cnt_buf.get(), *off = off_buf.get();
  int32_t* inl = inl_buf.get();
  HENN_HIP(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (size + 1), st));
  const unsigned eb = (unsigned)((edges + 255) / 256);
  hipLaunchKernelGGL(k_indeg, dim3(eb), dim3(256), 0, st, adj_knn, edges, cnt);
  exclusive_scan_u32(cnt, size, off, st);
  HENN_HIP(hipMemcpyAsync(cnt, off, sizeof(uint32_t) * size, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_scatter_in, dim3(eb), dim3(256), 0, st, adj_knn, edges, R, (int64_t)0,
                     cnt, inl);
  const unsigned nb = (unsigned)((size + 3) / 4);
  bool launched = false;
#define HENN_TRY(L, C)                                                                          \
  if (!launched && lpn == L && cpl == C) {                                                      \
    hipLaunchKernelGGL((k_sym_merge<L, C>), dim3(nb), dim3(256), 0, st, vec, size, dpad,        \
                       nchunks, metric, adj_knn, R, off, inl, max_deg, adj_out);                \
    launched = true;                                                                            \
  }
  HENN_KNN_COMBOS(HENN_TRY)
#undef HENN_TRY
  HENN_HIP(hipStreamSynchronize(st));
  if (!launched) throw HipError{hipErrorInvalidValue, "no merge kernel for this lane shape"};
}

// ---------------------------------------------------------------- NSW -----
// One batch of the NSW insertion (App. B.2), after the batch's searches:
// the new rows [lo, lo + nb) take their R results, -1 padded to M; the old
// points they chose collect them as in-lists (count, scan, scatter as for
// kNN_SYM); then one wave per chosen old point v merges its row with its
// in-list by (distance, id) in chunks of 64 keys and keeps the first M, in
// place (a wave reads its whole row before it writes it, and no other wave
// touches that row).
__global__ void k_nsw_rows(const int32_t* res, int64_t nb, int R, int M, int64_t lo,
                           int32_t* adj) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nb * M) return;
  const int64_t r = e / M;
  const int j = (int)(e % M);
  adj[(lo + r) * M + j] = j < R ? res[r * R + j] : -1;
}

template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_nsw_merge(const float* vec, int64_t lo, int dpad,
                                                   int nchunks, int metric, const uint32_t* off,
                                                   const int32_t* inl, int M, int32_t* adj) {
  constexpr int G = 64 / LPN;
  __shared__ int32_t cids[4][64];
  __shared__ uint64_t keys[4][64];
  const int w = threadIdx.x >> 6;
  const int64_t v = (int64_t)blockIdx.x * 4 + w;
  if (v >= lo) return;
  const int64_t ib = off[v];
  const int64_t nin = (int64_t)(off[v + 1] - off[v]);
  if (nin == 0) return;  // whole wave: v was chosen by no new point
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  const int32_t mine = lane < M ? adj[v * M + lane] : -1;  // the row, read before any write
  float q[CPL][8];
  load_query<CPL>(vec + v * dpad, dpad, t, q);
  const int64_t total = 64 + nin;
  uint64_t best = ~0ull;
  for (int64_t base = 0; base < total; base += 64) {
    const int64_t j = base + lane;
    cids[w][lane] = base == 0 ? mine : j < total ? inl[ib + (j - 64)] : -1;
    wave_sync();
    for (int pb = 0; pb < 64; pb += G) {
      const int ci = pb + g;
      const int32_t id = cids[w][ci];
      const bool valid = id >= 0;
      const float dist = group_distance<kF32, LPN, CPL>(
          q, vec + (int64_t)(valid ? id : 0) * dpad, 1.0f, t, nchunks, metric, valid);
      if (t == 0) keys[w][ci] = valid ? dkey(dist, id) : ~0ull;
    }
    wave_sync();
    const uint64_t c = wave_sort64(keys[w][lane]);
    const uint64_t rc = shfl_u64(c, 63 - lane);
    uint64_t m = rc < best ? rc : best;
    for (int stride = 32; stride > 0; stride >>= 1) {
      const uint64_t o = shfl_xor_u64(m, stride);
      const bool lower = (lane & stride) == 0;
      m = lower ? (o < m ? o : m) : (o < m ? m : o);
    }
    best = m;
    wave_sync();
  }
  if (lane < M) adj[v * M + lane] = best == ~0ull ? -1 : (int32_t)(uint32_t)best;
}

void nsw_merge_batch(const float* vec, int dpad, int nchunks, int metric, const int32_t* res,
                     int64_t lo, int64_t nb, int R, int32_t* adj, int M, uint32_t* cnt,
                     uint32_t* off, int32_t* inl, int lpn, int cpl, hipStream_t st) {
  const int64_t rows = nb * M;
  hipLaunchKernelGGL(k_nsw_rows, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, res,
                     nb, R, M, lo, adj);
  if (lo == 0) return;
  const int64_t edges = nb * R;
  const unsigned eb = (unsigned)((edges + 255) / 256);
  HENN_HIP(hipMemsetAsync(cnt, 0, sizeof(uint32_t) * (lo + 1), st));
  hipLaunchKernelGGL(k_indeg, dim3(eb), dim3(256), 0, st, res, edges, cnt);
  exclusive_scan_u32(cnt, lo, off, st);
  HENN_HIP(hipMemcpyAsync(cnt, off, sizeof(uint32_t) * lo, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_scatter_in, dim3(eb), dim3(256), 0, st, res, edges, R, lo, cnt, inl);
  const unsigned mb = (unsigned)((lo + 3) / 4);
  bool launched = false;
#define HENN_TRY(L, C)                                                                          \
  if (!launched && lpn == L && cpl == C) {                                                      \
    hipLaunchKernelGGL((k_nsw_merge<L, C>), dim3(mb), dim3(256), 0, st, vec, lo, dpad, nchunks, \
                       metric, off, inl, M, adj);                                               \
    launched = true;                                                                            \
  }
  HENN_KNN_COMBOS(HENN_TRY)
#undef HENN_TRY
  if (!launched) throw HipError{hipErrorInvalidValue, "no merge kernel for this lane shape"};
  HENN_HIP(hipGetLastError());
}

// Delete(x) repair of a layer graph: every live row v that links to deleted
// members gets the first M of the live candidates {row(v)} + {row(u) : u a
// deleted member of row(v)}, without v and without repeats, in (distance, id)
// order.  One wave per row; candidates go through one source row at a time
// (a key already in the running list is dropped, then sort and merge).
// Deleted rows are read, never written, and a
// live row is read and written only by its own wave, so the repair runs in
// place.
template <int LPN, int CPL>
__global__ __launch_bounds__(256) void k_nsw_repair(const float* vec, int64_t size, int dpad,
                                                    int nchunks, int metric,
                                                    const uint8_t* del, int M, int32_t* adj) {
  constexpr int G = 64 / LPN;
  __shared__ int32_t rows[4][64];
  __shared__ int32_t cids[4][64];
  __shared__ uint64_t keys[4][64];
  const int w = threadIdx.x >> 6;
  const int64_t v = (int64_t)blockIdx.x * 4 + w;
  if (v >= size || del[v]) return;  // whole wave
  const int lane = lane_id(), t = lane % LPN, g = lane / LPN;
  const int32_t mine = lane < M ? adj[v * M + lane] : -1;
  const bool hit = mine >= 0 && del[mine] != 0;
  const uint64_t hits = ballot(hit);
  if (hits == 0) return;  // nothing of this row was deleted
  rows[w][lane] = mine;
  wave_sync();
  float q[CPL][8];
  load_query<CPL>(vec + v * dpad, dpad, t, q);
  uint64_t best = ~0ull;
  // candidate sources: the row itself, then each deleted neighbour's row
  uint64_t todo = hits;
  for (int src = -1; src < 64; ) {
    int32_t cid = -1;
    if (src < 0) {
      cid = mine;
    } else {
      const int32_t u = rows[w][src];
      cid = lane < M ? adj[(int64_t)u * M + lane] : -1;
    }
    if (cid >= 0 && (del[cid] || cid == v)) cid = -1;
    cids[w][lane] = cid;
    wave_sync();
    for (int pb = 0; pb < 64; pb += G) {
      const int ci = pb + g;
      const int32_t id = cids[w][ci];
      const bool valid = id >= 0;
      const float dist = group_distance<kF32, LPN, CPL>(
          q, vec + (int64_t)(valid ? id : 0) * dpad, 1.0f, t, nchunks, metric, valid);
      if (t == 0) keys[w][ci] = valid ? dkey(dist, id) : ~0ull;
    }
    wave_sync();
    uint64_t key = keys[w][lane];
    for (int j = 0; j < 64; ++j) {  // a candidate already kept (same id, same key)
      const uint64_t b = shfl_u64(best, j);
      if (key != ~0ull && key == b) key = ~0ull;
    }
    const uint64_t c = wave_sort64(key);
    const uint64_t rc = shfl_u64(c, 63 - lane);
    uint64_t m = rc < best ? rc : best;
    for (int stride = 32; stride > 0; stride >>= 1) {
      const uint64_t o = shfl_xor_u64(m, stride);
      const bool lower = (lane & stride) == 0;
      m = lower ? (o < m ? o : m) : (o < m ? m : o);
    }
    best = m;
    wave_sync();
    if (todo == 0) break;
    src = __builtin_ctzll(todo);
    todo &= todo - 1;
  }
  if (lane < M) adj[v * M + lane] = best == ~0ull ? -1 : (int32_t)(uint32_t)best;
}

void repair_graph(const float* vec, int64_t size, int dpad, int nchunks, int metric,
                  const uint8_t* del, int M, int32_t* adj, int lpn, int cpl, hipStream_t st) {
  const unsigned nb = (unsigned)((size + 3) / 4);
  bool launched = false;
#define HENN_TRY(L, C)                                                                          \
  if (!launched && lpn == L && cpl == C) {                                                      \
    hipLaunchKernelGGL((k_nsw_repair<L, C>), dim3(nb), dim3(256), 0, st, vec, size, dpad,       \
                       nchunks, metric, del, M, adj);                                           \
    launched = true;                                                                            \
  }
  HENN_KNN_COMBOS(HENN_TRY)
#undef HENN_TRY
  if (!launched) throw HipError{hipErrorInvalidValue, "no repair kernel for this lane shape"};
  HENN_HIP(hipGetLastError());
}

}  // namespace henn

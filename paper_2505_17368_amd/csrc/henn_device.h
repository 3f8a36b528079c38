// henn_device.h -- device-side building blocks shared by the library's kernels.
//
// Everything here is part of the HIP product path: Philox4x64-10 for the
// with-replacement samples of Alg. 2 and the sampled ring ranges of the
// practical IsEpsNet check (App. B.1), ordered (distance, id) keys, and the
// canonical FP32 distance reduction used by every kernel that compares
// distances.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace henn {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Word q of the stream
// (tag, layer, attempt) is word q%4 of the block with counter
// (q/4, layer, attempt, tag) under key (seed, 0).
// ---------------------------------------------------------------------------
__host__ __device__ inline uint64_t mulhi_u64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
#endif
}

struct Philox4x64 {
  uint64_t x[4];
};

__host__ __device__ inline Philox4x64 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                    uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t kMul0 = 0xD2E7470EE14C6C93ull, kMul1 = 0xCA5A826395121157ull;
  const uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull, kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t h0 = mulhi_u64(kMul0, c0), l0 = kMul0 * c0;
    const uint64_t h1 = mulhi_u64(kMul1, c2), l1 = kMul1 * c2;
    const uint64_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
    k0 += kWeyl0;
    k1 += kWeyl1;
  }
  Philox4x64 r;
  r.x[0] = c0;
  r.x[1] = c1;
  r.x[2] = c2;
  r.x[3] = c3;
  return r;
}

// stream tags; halving step j (0-based) draws from tag kTagHalve + j
enum : uint32_t { kTagSample = 1, kTagRingCentre = 2, kTagRingStart = 3, kTagHalve = 4 };

__host__ __device__ inline uint64_t stream_word(uint64_t seed, uint32_t tag, uint32_t layer,
                                                uint32_t attempt, uint64_t q) {
  Philox4x64 b = philox4x64_10(q >> 2, layer, attempt, tag, seed, 0);
  return b.x[q & 3];
}

// uniform index in [0, s): high half of the 128-bit product w * s
__host__ __device__ inline uint64_t uniform_index(uint64_t w, uint64_t s) {
  return mulhi_u64(w, s);
}

// ---------------------------------------------------------------------------
// Ordered keys.  ordered_bits() maps floats to uint32 monotonically (-0 and
// +0 both map to the +0 code), so (ordered(dist) << 32 | id) compares as the
// lexicographic (distance, id) order used throughout the paper's searches.
// ---------------------------------------------------------------------------
__device__ inline uint32_t ordered_bits(float f) {
  f = f + 0.0f;  // -0 -> +0
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline float from_ordered(uint32_t u) {
  const uint32_t v = (u & 0x80000000u) ? (u & 0x7fffffffu) : ~u;
  return __uint_as_float(v);
}

// search-list key: distance | id | expanded flag (bit 0)
__device__ inline uint64_t wkey(float dist, int32_t id) {
  return ((uint64_t)ordered_bits(dist) << 32) | ((uint64_t)(uint32_t)id << 1);
}
__device__ inline int32_t wkey_id(uint64_t k) { return (int32_t)((uint32_t)k >> 1); }
__device__ inline float wkey_dist(uint64_t k) { return from_ordered((uint32_t)(k >> 32)); }
__device__ inline uint64_t wkey_strip(uint64_t k) { return k & ~1ull; }

// ring / graph key: distance | id
__device__ inline uint64_t dkey(float dist, int32_t id) {
  return ((uint64_t)ordered_bits(dist) << 32) | (uint32_t)id;
}

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64).
// ---------------------------------------------------------------------------
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lane_id() { return (int)(threadIdx.x & 63); }

__device__ inline uint64_t ballot(bool p) { return __ballot(p); }

__device__ inline int popc64(uint64_t m) { return __popcll(m); }

// number of set bits of m below this lane
__device__ inline int rank_below(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Values every lane of the wave holds alike, moved to scalar registers so
// that the compiler treats the control flow that depends on them as uniform.
__device__ inline int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float uni_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline uint64_t uni_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src) {
  const uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)v, m), hi = __shfl_xor((uint32_t)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}

// ---------------------------------------------------------------------------
// Storage formats.  A stored row is nchunks chunks of 8 coordinates.
//   F32:  8 floats per chunk.
//   BF16: 8 bf16 per chunk (round-to-nearest-even from FP32), scale 1.
//   FP8:  8 OCP E4M3 codes per chunk, per-row FP32 scale (max|x| / 448).
// ---------------------------------------------------------------------------
enum StoreKind { kF32 = 0, kBF16 = 1, kFP8 = 2 };

__device__ inline float bf16_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

// FP32 -> BF16 bits, round to nearest even (finite inputs).
__device__ inline uint32_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// OCP E4M3 (e4m3fn): bias 7, subnormals, max 448.  Exact decode: place the
// 7 magnitude bits where an FP32 exponent/mantissa would sit, then rescale
// by 2^120 (exact), which also covers the subnormal codes.
__device__ inline float fp8_to_f32(uint32_t b) {
  const float mag = __uint_as_float((b & 0x7fu) << 20) * 0x1p120f;
  return (b & 0x80u) ? -mag : mag;
}

// One chunk of 8 coordinates of a stored row: fetch() issues the load,
// decode() turns it into FP32 values (exactly).  FP8 rows decode with
// gfx950's packed converter (OCP E4M3; two codes per instruction, the low
// byte first); fp8_to_f32 above is the same map written out, used where
// rows are decoded once.
template <int KIND>
struct ChunkRaw;
template <>
struct ChunkRaw<kF32> {
  float4 a, b;
  __device__ inline void fetch(const void* row, int c) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(row) + c * 8);
    a = p[0];
    b = p[1];
  }
  __device__ inline void decode(float (&v)[8]) const {
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
};
template <>
struct ChunkRaw<kBF16> {
  uint4 a;
  __device__ inline void fetch(const void* row, int c) {
    a = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(row) + c * 8);
  }
  __device__ inline void decode(float (&v)[8]) const {
    v[0] = bf16_to_f32(a.x & 0xffffu); v[1] = bf16_to_f32(a.x >> 16);
    v[2] = bf16_to_f32(a.y & 0xffffu); v[3] = bf16_to_f32(a.y >> 16);
    v[4] = bf16_to_f32(a.z & 0xffffu); v[5] = bf16_to_f32(a.z >> 16);
    v[6] = bf16_to_f32(a.w & 0xffffu); v[7] = bf16_to_f32(a.w >> 16);
  }
};
template <>
struct ChunkRaw<kFP8> {
  uint2 a;
  __device__ inline void fetch(const void* row, int c) {
    a = *reinterpret_cast<const uint2*>(static_cast<const uint8_t*>(row) + c * 8);
  }
  __device__ inline void decode(float (&v)[8]) const {
    const auto p0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)a.x, false);
    const auto p1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)a.x, true);
    const auto p2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)a.y, false);
    const auto p3 = __builtin_amdgcn_cvt_pk_f32_fp8((int)a.y, true);
    v[0] = p0[0]; v[1] = p0[1]; v[2] = p1[0]; v[3] = p1[1];
    v[4] = p2[0]; v[5] = p2[1]; v[6] = p3[0]; v[7] = p3[1];
  }
};

// fetch + decode in one step
template <int KIND>
struct Chunk {
  __device__ static inline void load(const void* row, int c, float (&v)[8]) {
    ChunkRaw<KIND> r;
    r.fetch(row, c);
    r.decode(v);
  }
};

// ---------------------------------------------------------------------------
// Canonical FP32 distance.  The vector is cut into chunks of 8 coordinates;
// each chunk is summed sequentially with fused multiply-adds, and the chunk
// sums are added by a pairwise tree over next_pow2(nchunks) leaves (missing
// leaves are zero).  Any split of the chunks over a power-of-two number of
// lanes, each holding a power-of-two run of chunks, reproduces that tree
// exactly (floating-point addition is commutative), so every kernel and
// every launch shape computes bit-identical distances.
//   L2: sum (q - s*x)^2 with s the row scale (1 for F32/BF16);
//   IP: -(s * sum q*x).
// ---------------------------------------------------------------------------
__device__ inline float chunk_l2(const float (&q)[8], const float (&x)[8], float s, bool scaled) {
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const float t = scaled ? __builtin_fmaf(-s, x[j], q[j]) : (q[j] - x[j]);
    acc = __builtin_fmaf(t, t, acc);
  }
  return acc;
}

__device__ inline float chunk_ip(const float (&q)[8], const float (&x)[8]) {
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < 8; ++j) acc = __builtin_fmaf(q[j], x[j], acc);
  return acc;
}

// In-lane pairwise tree over CPL partial sums (CPL a power of two).
template <int CPL>
__device__ inline float tree_sum(float (&c)[CPL]) {
#pragma unroll
  for (int w = 1; w < CPL; w *= 2) {
#pragma unroll
    for (int i = 0; i + w < CPL; i += 2 * w) c[i] = c[i] + c[i + w];
  }
  return c[0];
}

// Butterfly over LPN consecutive lanes: after it every lane of the group
// holds the same, tree-ordered total.
// Lane exchange inside a row of 16 lanes through DPP (a VALU operand
// modifier, no LDS round trip).  ctrl: 0xB1 quad_perm [1,0,3,2] (lane ^ 1),
// 0x4E quad_perm [2,3,0,1] (lane ^ 2), 0x104 row_shl:4, 0x114 row_shr:4,
// 0x128 row_ror:8 (lane ^ 8).
template <int CTRL>
__device__ inline float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Butterfly sum over the LPN lanes of a group: step m adds the value of lane
// ^ m, for m = 1, 2, 4, ...; every lane of the group ends with the same sum.
// Must be reached by the whole wave.
template <int LPN>
__device__ inline float group_sum_from2(float v);

template <int LPN>
__device__ inline float group_sum(float v) {
  if (LPN >= 2) v = v + dpp_mov<0xB1>(v);
  return group_sum_from2<LPN>(v);
}

// The butterfly's steps from m = 2 on.
template <int LPN>
__device__ inline float group_sum_from2(float v) {
  if (LPN >= 4) v = v + dpp_mov<0x4E>(v);
  if (LPN >= 8) {
    // lane ^ 4: lanes with bit 2 clear read lane + 4, the others lane - 4
    const float up = dpp_mov<0x104>(v), down = dpp_mov<0x114>(v);
    v = v + ((lane_id() & 4) ? down : up);
  }
  if (LPN >= 16) v = v + dpp_mov<0x128>(v);
#pragma unroll
  for (int m = 16; m < LPN; m *= 2) v = v + __shfl_xor(v, m, 64);  // groups wider than a row
  return v;
}

// Distances between a query slice held in registers (this lane's chunks
// [t*CPL, (t+1)*CPL)) and NR rows per lane group; all LPN lanes of a group
// return the same values, and every lane joins the butterfly.  Every chunk the lane needs is
// loaded first, without branches (chunks past the row are clamped to chunk
// 0 and dropped), so that all NR * CPL loads are in flight together; then
// the chunks are decoded and reduced exactly as group_distance does.  rows[r]
// must point at readable row memory even when !valid[r].
template <int KIND, int LPN, int CPL, int NR>
__device__ inline void group_distances(const float (&q)[CPL][8], const void* const (&rows)[NR],
                                       const float (&scale)[NR], int t, int nchunks, int metric,
                                       const bool (&valid)[NR], float (&out)[NR]) {
  ChunkRaw<KIND> raw[NR][CPL];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int c = t * CPL + i;
      raw[r][i].fetch(rows[r], c < nchunks ? c : 0);
    }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    float part[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int c = t * CPL + i;
      float x[8];
      raw[r][i].decode(x);
      const float v = metric == 0 ? chunk_l2(q[i], x, scale[r], KIND == kFP8) : chunk_ip(q[i], x);
      part[i] = (valid[r] && c < nchunks) ? v : 0.0f;
    }
    float s2 = group_sum<LPN>(tree_sum<CPL>(part));
    if (metric != 0) s2 = (KIND == kFP8) ? -(scale[r] * s2) : -s2;
    out[r] = s2;
  }
}

// As group_distances for NR = 2 or 3 rows, with rows 0 and 1 reduced in one
// butterfly: the first step sends row 1's partial sum from the even lanes
// and row 0's from the odd ones, so from then on the even lanes of a group
// carry row 0 and the odd lanes row 1.  Every sum adds the same two operands
// as group_sum's (addition commutes), so the distances are bit-identical to
// group_distance's.  d01: row 0's distance on even lanes, row 1's on odd
// lanes; d2: row 2's (NR = 3) on every lane.  Needs LPN >= 2.
template <int KIND, int LPN, int CPL, int NR>
__device__ inline void group_distances_paired(const float (&q)[CPL][8],
                                              const void* const (&rows)[NR],
                                              const float (&scale)[NR], int t, int nchunks,
                                              int metric, const bool (&valid)[NR], float& d01,
                                              float& d2) {
  static_assert(LPN >= 2 && (NR == 2 || NR == 3), "pairs rows 0 and 1 of a lane group");
  ChunkRaw<KIND> raw[NR][CPL];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int c = t * CPL + i;
      raw[r][i].fetch(rows[r], c < nchunks ? c : 0);
    }
  float ts[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    float part[CPL];
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int c = t * CPL + i;
      float x[8];
      raw[r][i].decode(x);
      const float v = metric == 0 ? chunk_l2(q[i], x, scale[r], KIND == kFP8) : chunk_ip(q[i], x);
      part[i] = (valid[r] && c < nchunks) ? v : 0.0f;
    }
    ts[r] = tree_sum<CPL>(part);
  }
  const bool odd = (lane_id() & 1) != 0;
  float v = (odd ? ts[1] : ts[0]) + dpp_mov<0xB1>(odd ? ts[0] : ts[1]);
  v = group_sum_from2<LPN>(v);
  if (metric != 0) v = (KIND == kFP8) ? -((odd ? scale[1] : scale[0]) * v) : -v;
  d01 = v;
  if (NR == 3) {
    float s2 = group_sum<LPN>(ts[NR - 1]);
    if (metric != 0) s2 = (KIND == kFP8) ? -(scale[NR - 1] * s2) : -s2;
    d2 = s2;
  }
}

template <int KIND, int LPN, int CPL>
__device__ inline float group_distance(const float (&q)[CPL][8], const void* row, float scale,
                                       int t, int nchunks, int metric, bool valid = true) {
  const void* const rows[1] = {row};
  const float sc[1] = {scale};
  const bool vd[1] = {valid};
  float out[1];
  group_distances<KIND, LPN, CPL, 1>(q, rows, sc, t, nchunks, metric, vd, out);
  return out[0];
}

// Loads this lane's query slice (FP32 source, chunked; zero beyond d).
template <int CPL>
__device__ inline void load_query(const float* qrow, int d, int t, float (&q)[CPL][8]) {
#pragma unroll
  for (int i = 0; i < CPL; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = (t * CPL + i) * 8 + j;
      q[i][j] = e < d ? qrow[e] : 0.0f;
    }
  }
}

}  // namespace henn

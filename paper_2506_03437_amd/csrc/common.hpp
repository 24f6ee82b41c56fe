// Device-side building blocks shared by the kernels: the (key, id) total
// order of results, a wave-wide sorted top-k list, an LDS bitonic sort, a
// co-rank merge of two sorted lists, wave bitonic sorts and merges of
// (key, slot) packed into ordered integers, and DPP wave reductions.
//
// Result order: a result is a pair (key, id) with key = squared L2 distance,
// or the negated inner product, so that smaller is better for both metrics;
// equal keys are ordered by the lower id.  Empty slots are (+inf, -1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "index.hpp"

namespace qk {

constexpr int WAVE = 64;
constexpr float KEY_EMPTY = __builtin_inff();

__device__ __forceinline__ bool kv_less(float ak, int64_t ai, float bk, int64_t bi) {
  return ak < bk || (ak == bk && ai < bi);
}

// Order-preserving map of a float to uint32 (finite values and +-inf).
__device__ __forceinline__ uint32_t float_order(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Inverse of float_order.
__device__ __forceinline__ float float_from_order(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ int64_t shfl_up_i64(int64_t v, int delta) {
  int lo = __shfl_up((int)(uint32_t)(uint64_t)v, delta);
  int hi = __shfl_up((int)(uint32_t)((uint64_t)v >> 32), delta);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t shfl_i64(int64_t v, int src) {
  int lo = __shfl((int)(uint32_t)(uint64_t)v, src);
  int hi = __shfl((int)(uint32_t)((uint64_t)v >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t shfl_xor_i64(int64_t v, int mask) {
  int lo = __shfl_xor((int)(uint32_t)(uint64_t)v, mask);
  int hi = __shfl_xor((int)(uint32_t)((uint64_t)v >> 32), mask);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t readlane_i64(int64_t v, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)(uint64_t)v, lane);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), lane));
}

// Lane exchange inside rows of 16 lanes through DPP (no LDS round trip):
// quad_perm [1,0,3,2] and [2,3,0,1] swap neighbours and pairs, row_half_mirror
// reverses each group of 8 and row_mirror each row of 16.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;

// Minimum and maximum of v over the wave (uniform results): DPP steps reduce
// each row of 16 lanes, then the four row results are combined in scalars.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, dpp_u32<DPP_XOR1>(v));
  v = min(v, dpp_u32<DPP_XOR2>(v));
  v = min(v, dpp_u32<DPP_HALF_MIRROR>(v));
  v = min(v, dpp_u32<DPP_MIRROR>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, dpp_u32<DPP_XOR1>(v));
  v = max(v, dpp_u32<DPP_XOR2>(v));
  v = max(v, dpp_u32<DPP_HALF_MIRROR>(v));
  v = max(v, dpp_u32<DPP_MIRROR>(v));
  return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, lane);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_prod_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v *= __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// A sorted list of up to 64*KPL results spread over the lanes of one wave:
// position p = t*64 + lane lives in slot t of that lane.  The list keeps the
// best results seen; `thr` is the entry a new result must beat: the k-th
// entry once k results exist, else the seed the list started from.
template <int KPL>
struct WaveTopK {
  float key[KPL];
  int64_t id[KPL];
  float tk;
  int64_t ti;
  float seed_k;
  int64_t seed_i;
  int k;

  __device__ void init(int k_, float sk, int64_t si) {
    k = k_;
#pragma unroll
    for (int t = 0; t < KPL; ++t) { key[t] = KEY_EMPTY; id[t] = -1; }
    seed_k = sk; seed_i = si;
    tk = sk; ti = si;
  }

  // Insert a wave-uniform candidate that beats thr.
  __device__ void insert(float ck, int64_t ci) {
    const int lane = lane_id();
    int pos = 0;
#pragma unroll
    for (int t = 0; t < KPL; ++t) pos += __popcll(__ballot(kv_less(key[t], id[t], ck, ci)));
    float nk[KPL];
    int64_t ni[KPL];
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
      float uk = __shfl_up(key[t], 1);
      int64_t ui = shfl_up_i64(id[t], 1);
      if (t > 0) {
        float ck2 = readlane_f(key[t - 1], WAVE - 1);
        int64_t ci2 = readlane_i64(id[t - 1], WAVE - 1);
        if (lane == 0) { uk = ck2; ui = ci2; }
      }
      const int p = t * WAVE + lane;
      nk[t] = key[t]; ni[t] = id[t];
      if (p > pos) { nk[t] = uk; ni[t] = ui; }
      else if (p == pos) { nk[t] = ck; ni[t] = ci; }
    }
#pragma unroll
    for (int t = 0; t < KPL; ++t) { key[t] = nk[t]; id[t] = ni[t]; }
    const int kt = (k - 1) / WAVE, kl = (k - 1) % WAVE;
    float kk = KEY_EMPTY;
    int64_t ki = -1;
#pragma unroll
    for (int t = 0; t < KPL; ++t)
      if (t == kt) { kk = readlane_f(key[t], kl); ki = readlane_i64(id[t], kl); }
    if (ki >= 0) { tk = kk; ti = ki; }
  }

  __device__ void store(float* ok, int64_t* oi) const {
    const int lane = lane_id();
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
      const int p = t * WAVE + lane;
      if (p < k) { ok[p] = key[t]; oi[p] = id[t]; }
    }
  }
};

// Bitonic sort of n (power of two) uint64 keys in LDS, ascending; all
// threads of the block take part.
__device__ inline void bitonic_sort_u64(uint64_t* s, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = ((lo & size) == 0);
        uint64_t a = s[lo], b = s[hi];
        if ((a > b) == up) { s[lo] = b; s[hi] = a; }
      }
    }
  }
  __syncthreads();
}

// Number of entries of the sorted list (bk, bi)[0..n) that precede (k, i)
// (strict = true) or that do not follow it (strict = false).
__device__ __forceinline__ int corank(const float* bk, const int64_t* bi, int n, float k, int64_t i, bool strict) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const bool before = strict ? kv_less(bk[mid], bi[mid], k, i) : !kv_less(k, i, bk[mid], bi[mid]);
    if (before) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Merge the sorted lists A and B (length n each, padded with empties) into
// the first n entries of their union, written to O.  One wave.  A's entries
// go before B's on exact equality, which only empties can have.
__device__ inline void wave_merge(const float* ak, const int64_t* ai, const float* bk, const int64_t* bi,
                                  float* ok, int64_t* oi, int n) {
  for (int e = lane_id(); e < n; e += WAVE) {
    const int pa = e + corank(bk, bi, n, ak[e], ai[e], true);
    if (pa < n) { ok[pa] = ak[e]; oi[pa] = ai[e]; }
    const int pb = e + corank(ak, ai, n, bk[e], bi[e], false);
    if (pb < n) { ok[pb] = bk[e]; oi[pb] = bi[e]; }
  }
}

// Two ascending lists of up to 64 entries held one entry per lane (lanes past
// a list's end hold empties): a := the 64 smallest of a and b, ascending.
// Against b reversed, the lane-wise minimum is a bitonic sequence holding
// the 64 smallest entries; six compare-exchange stages sort it.
__device__ __forceinline__ void wave_merge64_kv(float& ak, int64_t& ai, float bk, int64_t bi) {
  const int lane = lane_id();
  const float rk = __shfl(bk, WAVE - 1 - lane);
  const int64_t rv = shfl_i64(bi, WAVE - 1 - lane);
  if (kv_less(rk, rv, ak, ai)) { ak = rk; ai = rv; }
#pragma unroll
  for (int stride = WAVE / 2; stride > 0; stride >>= 1) {
    const float ok = __shfl_xor(ak, stride);
    const int64_t oi = shfl_xor_i64(ai, stride);
    const bool lower = (lane & stride) == 0;
    if (lower ? kv_less(ok, oi, ak, ai) : kv_less(ak, ai, ok, oi)) { ak = ok; ai = oi; }
  }
}

// (key, slot) packed into one integer whose unsigned order is the result
// order: the key's order-preserving bits above the slot's bits (slots are
// >= 0; the empty entry (+inf, -1) sorts last).
__device__ __forceinline__ uint64_t pack_key_slot(float k, int32_t s) {
  return ((uint64_t)float_order(k) << 32) | (uint32_t)s;
}
__device__ __forceinline__ float packed_key(uint64_t v) { return float_from_order((uint32_t)(v >> 32)); }
__device__ __forceinline__ int32_t packed_slot(uint64_t v) { return (int32_t)(uint32_t)v; }

// Sort N independent lists of packed entries (one per lane in each)
// ascending with a bitonic network; per compare-exchange one 64-bit compare
// and a select, the N lists' shuffles overlapping.
template <int N>
__device__ __forceinline__ void wave_sort64_packed_n(uint64_t (&v)[N]) {
  const int lane = lane_id();
#pragma unroll
  for (int size = 2; size <= WAVE; size <<= 1)
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      uint64_t o[N];
#pragma unroll
      for (int q = 0; q < N; ++q) o[q] = (uint64_t)shfl_xor_i64((int64_t)v[q], stride);
      // the lower lane of a pair keeps the smaller entry in ascending runs
      // of length `size`, the larger one in descending runs
      const bool take_min = ((lane & size) == 0) == ((lane & stride) == 0);
#pragma unroll
      for (int q = 0; q < N; ++q) v[q] = ((o[q] < v[q]) == take_min) ? o[q] : v[q];
    }
}

// list (ascending, one packed entry per lane) := the 64 smallest of list and
// b (ascending): a bitonic split against b reversed, then a bitonic merge.
__device__ __forceinline__ void wave_merge64_packed(uint64_t& l, uint64_t b) {
  const int lane = lane_id();
  const uint64_t r = (uint64_t)shfl_i64((int64_t)b, WAVE - 1 - lane);
  l = r < l ? r : l;
#pragma unroll
  for (int stride = WAVE / 2; stride > 0; stride >>= 1) {
    const uint64_t o = (uint64_t)shfl_xor_i64((int64_t)l, stride);
    l = ((o < l) == ((lane & stride) == 0)) ? o : l;
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) f32x4 const_float4;

// Distance of the query to the 64 vectors of one tile, one vector per lane.
// The query is read through the scalar unit (one copy for the whole wave);
// the tile through 16-byte loads that cover 1 KiB contiguous per wave.  Eight
// partial sums (one per dimension modulo 8) are combined pairwise at the end.
template <int METRIC>
__device__ __forceinline__ float tile_distance(const float4* __restrict__ xp, const_float4* qs, int nch4) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f, a6 = 0.f, a7 = 0.f;
#pragma unroll 4
  for (int c = 0; c < nch4; c += 2) {
    const float4 x = xp[(int64_t)c * WAVE];
    const float4 y = xp[(int64_t)(c + 1) * WAVE];
    const f32x4 qa = qs[c];
    const f32x4 qb = qs[c + 1];
    if (METRIC == QUAKE_L2) {
      float t;
      t = x.x - qa.x; a0 = fmaf(t, t, a0);
      t = x.y - qa.y; a1 = fmaf(t, t, a1);
      t = x.z - qa.z; a2 = fmaf(t, t, a2);
      t = x.w - qa.w; a3 = fmaf(t, t, a3);
      t = y.x - qb.x; a4 = fmaf(t, t, a4);
      t = y.y - qb.y; a5 = fmaf(t, t, a5);
      t = y.z - qb.z; a6 = fmaf(t, t, a6);
      t = y.w - qb.w; a7 = fmaf(t, t, a7);
    } else {
      a0 = fmaf(x.x, qa.x, a0); a1 = fmaf(x.y, qa.y, a1);
      a2 = fmaf(x.z, qa.z, a2); a3 = fmaf(x.w, qa.w, a3);
      a4 = fmaf(y.x, qb.x, a4); a5 = fmaf(y.y, qb.y, a5);
      a6 = fmaf(y.z, qb.z, a6); a7 = fmaf(y.w, qb.w, a7);
    }
  }
  const float s = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
  return METRIC == QUAKE_L2 ? s : -s;
}

}  // namespace qk

// Update-path kernels: the id -> slot map, deletes, slot moves for
// compaction, and the hand-over from a level-1 search to level-0 candidates.
//
// The id map is an open-addressing hash table in device memory (linear
// probing, 64-bit keys claimed with atomicCAS).  Key -1 marks an empty
// entry and -2 an erased one; the host keeps the load (live + erased) under
// half of the capacity and rebuilds the table from the store when needed.
// Every probe loop is bounded by the capacity.
#include "common.hpp"
#include "index.hpp"

namespace qk {

constexpr int64_t KEY_FREE = -1;
constexpr int64_t KEY_GONE = -2;

// splitmix64 finaliser (Steele, Lea and Flood, OOPSLA 2014): spreads
// consecutive ids over the table.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__device__ __forceinline__ int64_t map_find_pos(const int64_t* __restrict__ keys, uint64_t mask, int64_t id) {
  uint64_t h = mix64((uint64_t)id) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const int64_t k = keys[h];
    if (k == id) return (int64_t)h;
    if (k == KEY_FREE) return -1;
    h = (h + 1) & mask;
  }
  return -1;
}

__global__ __launch_bounds__(256) void k_map_insert(int64_t* __restrict__ keys, int64_t* __restrict__ vals,
                                                     uint64_t mask, const int64_t* __restrict__ ids,
                                                     const int64_t* __restrict__ slots, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t id = ids[i];
  uint64_t h = mix64((uint64_t)id) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&keys[h], (unsigned long long)KEY_FREE, (unsigned long long)id);
    if ((int64_t)prev == KEY_FREE) {
      vals[h] = slots[i];
      return;
    }
    h = (h + 1) & mask;
  }
}

// Insert every filled slot of a store (table rebuild and initial build).
__global__ __launch_bounds__(256) void k_map_insert_store(int64_t* __restrict__ keys, int64_t* __restrict__ vals,
                                                           uint64_t mask, const int64_t* __restrict__ sid,
                                                           int64_t slots) {
  const int64_t sl = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (sl >= slots) return;
  const int64_t id = sid[sl];
  if (id < 0) return;
  uint64_t h = mix64((uint64_t)id) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&keys[h], (unsigned long long)KEY_FREE, (unsigned long long)id);
    if ((int64_t)prev == KEY_FREE) {
      vals[h] = sl;
      return;
    }
    h = (h + 1) & mask;
  }
}

// slot of every id (-1 when absent); *missing counts the absent ones.
__global__ __launch_bounds__(256) void k_map_find(const int64_t* __restrict__ keys, const int64_t* __restrict__ vals,
                                                   uint64_t mask, const int64_t* __restrict__ ids, int64_t n,
                                                   int64_t* __restrict__ slots, int64_t* __restrict__ missing) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t pos = map_find_pos(keys, mask, ids[i]);
  const int64_t sl = pos >= 0 ? vals[pos] : -1;
  if (slots) slots[i] = sl;
  if (sl < 0) atomicAdd((unsigned long long*)missing, 1ull);
}

__global__ __launch_bounds__(256) void k_map_erase(int64_t* __restrict__ keys, uint64_t mask,
                                                    const int64_t* __restrict__ ids, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t pos = map_find_pos(keys, mask, ids[i]);
  if (pos >= 0) keys[pos] = KEY_GONE;
}

__global__ __launch_bounds__(256) void k_map_update(const int64_t* __restrict__ keys, int64_t* __restrict__ vals,
                                                     uint64_t mask, const int64_t* __restrict__ ids,
                                                     const int64_t* __restrict__ slots, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t pos = map_find_pos(keys, mask, ids[i]);
  if (pos >= 0) vals[pos] = slots[i];
}

static dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

void launch_map_insert(IdMap& m, const int64_t* ids, const int64_t* slots, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_map_insert, grid_of(n), dim3(256), 0, s, m.keys, m.vals, m.mask, ids, slots, n);
}
void launch_map_insert_store(IdMap& m, const int64_t* sid, int64_t slots, hipStream_t s) {
  if (slots > 0)
    hipLaunchKernelGGL(k_map_insert_store, grid_of(slots), dim3(256), 0, s, m.keys, m.vals, m.mask, sid, slots);
}
void launch_map_find(const IdMap& m, const int64_t* ids, int64_t n, int64_t* slots, int64_t* missing, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_map_find, grid_of(n), dim3(256), 0, s, m.keys, m.vals, m.mask, ids, n, slots, missing);
}
void launch_map_erase(IdMap& m, const int64_t* ids, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_map_erase, grid_of(n), dim3(256), 0, s, m.keys, m.mask, ids, n);
}
void launch_map_update(IdMap& m, const int64_t* ids, const int64_t* slots, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_map_update, grid_of(n), dim3(256), 0, s, m.keys, m.vals, m.mask, ids, slots, n);
}

// ---------------------------------------------------------------- store edits

__global__ __launch_bounds__(256) void k_mark_deleted(int64_t* __restrict__ sid, const int64_t* __restrict__ slots,
                                                       int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) sid[slots[i]] = -1;
}

void launch_mark_deleted(Store& st, const int64_t* slots, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mark_deleted, grid_of(n), dim3(256), 0, s, st.ids, slots, n);
}

// Move vector src[i] to slot dst[i] within the store (every copy of it, its
// label bits, product codes and id), leaving src[i] empty.  Sources and
// destinations are disjoint.  Thread c4 of a row moves its code words c4,
// c4 + dp/4, ... (cw of them).
__global__ __launch_bounds__(256) void k_move_slots(const int64_t* __restrict__ src, const int64_t* __restrict__ dst,
                                                     int64_t n, int dp, int dp16, float* __restrict__ v32,
                                                     uint16_t* __restrict__ v16, float* __restrict__ v16n,
                                                     float* __restrict__ rows32, int64_t* __restrict__ sid,
                                                     uint32_t* __restrict__ attr, uint32_t* __restrict__ codes,
                                                     int cw) {
  const int nch4 = dp >> 2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = e / nch4;
  if (i >= n) return;
  const int c4 = (int)(e - i * nch4);
  const int64_t a = src[i], b = dst[i];
  const int64_t ta = a / TILE, tb = b / TILE;
  const int la = (int)(a - ta * TILE), lb = (int)(b - tb * TILE);
  if (v32) {
    float4* f = reinterpret_cast<float4*>(v32);
    f[(tb * nch4 + c4) * TILE + lb] = f[(ta * nch4 + c4) * TILE + la];
  }
  if (v16) {
    const int nc8 = dp16 >> 3;
    const int c8 = c4 >> 1, half = c4 & 1;
    const uint16_t* from = v16 + ((ta * nc8 + c8) * TILE + la) * 8 + half * 4;
    uint16_t* to = v16 + ((tb * nc8 + c8) * TILE + lb) * 8 + half * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) to[u] = from[u];
  }
  if (rows32)
    *reinterpret_cast<float4*>(rows32 + b * dp + c4 * 4) = *reinterpret_cast<const float4*>(rows32 + a * dp + c4 * 4);
  if (codes)
    for (int w = c4; w < cw; w += nch4) codes[(tb * cw + w) * TILE + lb] = codes[(ta * cw + w) * TILE + la];
  if (c4 == 0) {
    if (v16n) v16n[b] = v16n[a];
    if (attr) attr[b] = attr[a];
    sid[b] = sid[a];
    sid[a] = -1;
  }
}

void launch_move_slots(Store& st, const int64_t* src, const int64_t* dst, int64_t n, hipStream_t s) {
  const int64_t total = n * (st.dp >> 2);
  if (total <= 0) return;
  hipLaunchKernelGGL(k_move_slots, grid_of(total), dim3(256), 0, s, src, dst, n, st.dp, st.dp16, st.v32, st.v16,
                     st.v16n, st.rows32, st.ids, st.attr, st.codes, pq_words(st.pq_m));
}

__global__ __launch_bounds__(256) void k_put_u32(const uint32_t* __restrict__ src, const int64_t* __restrict__ slot,
                                                  int64_t n, uint32_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[slot[i]] = src[i];
}

void launch_put_u32(const uint32_t* src, const int64_t* slot, int64_t n, uint32_t* dst, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_put_u32, grid_of(n), dim3(256), 0, s, src, slot, n, dst);
}

// Per partition (one block each): live rows carrying each of the 32 label
// bits, and live rows, into cnt[p][0..32].
__global__ __launch_bounds__(256) void k_attr_counts(const uint32_t* __restrict__ attr,
                                                      const int64_t* __restrict__ sid,
                                                      const int64_t* __restrict__ poff,
                                                      const int32_t* __restrict__ psize, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t c[33];
  const int p = blockIdx.x;
  if (threadIdx.x < 33) c[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = poff[p] * TILE;
  for (int j = threadIdx.x; j < psize[p]; j += 256) {
    if (sid[base + j] < 0) continue;
    uint32_t a = attr[base + j];
    atomicAdd(&c[32], 1u);
    while (a) {
      atomicAdd(&c[__builtin_ctz(a)], 1u);
      a &= a - 1;
    }
  }
  __syncthreads();
  if (threadIdx.x < 33) cnt[(int64_t)p * 33 + threadIdx.x] = c[threadIdx.x];
}

void launch_attr_counts(const Store& st, hipStream_t s) {
  if (st.nlist > 0 && st.attr)
    hipLaunchKernelGGL(k_attr_counts, dim3((unsigned)st.nlist), dim3(256), 0, s, st.attr, st.ids, st.d_off, st.d_size,
                       st.d_attr_cnt);
}

// |x|^2 of the 16-bit copy for the listed slots.
__global__ __launch_bounds__(256) void k_norm16_slots(const uint16_t* __restrict__ v16, const int64_t* __restrict__ slots,
                                                       int64_t n, int dp16, int f16, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t sl = slots[i];
  const int64_t tile = sl / TILE;
  const int lane = (int)(sl - tile * TILE);
  const int nc8 = dp16 >> 3;
  float acc = 0.f;
  for (int c = 0; c < nc8; ++c) {
    const uint16_t* e = v16 + ((tile * nc8 + c) * TILE + lane) * 8;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float v = f16 ? (float)__builtin_bit_cast(_Float16, e[u]) : __uint_as_float((uint32_t)e[u] << 16);
      acc = fmaf(v, v, acc);
    }
  }
  out[sl] = acc;
}

void launch_norm16_slots(Store& st, const int64_t* slots, int64_t n, int dtype16, hipStream_t s) {
  if (n <= 0 || !st.v16n) return;
  hipLaunchKernelGGL(k_norm16_slots, grid_of(n), dim3(256), 0, s, st.v16, slots, n, st.dp16,
                     dtype16 == QUAKE_F16 ? 1 : 0, st.v16n);
}

// ---------------------------------------------------------------- two levels

// Level-1 results (leaf ids by distance) become the level-0 candidate rows:
// cand0[q][0..M0) and the number of valid entries mq[q].
__global__ __launch_bounds__(256) void k_level1_to_candidates(int64_t nq, int M0, int kk, const int64_t* __restrict__ ri,
                                                               int32_t* __restrict__ cand0, int32_t* __restrict__ mq) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= nq) return;
  int valid = 0;
  for (int j = lane; j < M0; j += WAVE) {
    const int64_t id = ri[q * kk + j];
    cand0[q * M0 + j] = id >= 0 ? (int32_t)id : -1;
    valid += id >= 0 ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) valid += __shfl_xor(valid, o);
  if (lane == 0) mq[q] = valid;
}

void launch_level1_to_candidates(int64_t nq, int M0, int kk, const int64_t* ri, int32_t* cand0, int32_t* mq,
                                 hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_level1_to_candidates, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, nq, M0, kk, ri, cand0,
                     mq);
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, grid_of(n), dim3(256), 0, s, p, n, v);
}

}  // namespace qk

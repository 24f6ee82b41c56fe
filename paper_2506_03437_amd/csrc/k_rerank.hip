// FP32 rerank of the batched path's candidates (Sec. 7.4, "Multi-Query Processing" scans a reduced-
// precision copy; the candidates it keeps are re-scored exactly here).
//
// After the last round each query holds rerank_factor * k candidates (store
// slots, in ri) found on the 16-bit copy.  They are re-scored in FP32 from
// the row-major FP32 copy of the store (one contiguous row per slot; the
// tile-interleaved store would fetch a whole cache line per 16 bytes used),
// summing in the plain scan's order: eight partial sums over the dimensions
// modulo 8, i ascending within each, added pairwise - so a candidate's
// distance is bitwise the one the FP32 scan reports.  Then each query keeps
// its best k by (distance, id).
#include "common.hpp"
#include "index.hpp"

namespace qk {

// Distances of all (row, candidate) pairs, flattened over the grid: lanes 2p
// and 2p + 1 of a block score pair blockIdx.x * 128 + p; the first keeps the
// partial sums of dimensions 8i .. 8i + 3, the second those of 8i + 4 ..
// 8i + 7 (dp is a multiple of 8), reading 16 bytes of the row per step.
// The distance overwrites the candidate's committed 16-bit key in rk.
template <int METRIC>
__global__ __launch_bounds__(256) void k_rerank_dist(int64_t nrows, int kk, const float* __restrict__ qpad, int dp,
                                                     const float* __restrict__ rows, float* __restrict__ rk,
                                                     const int64_t* __restrict__ ri,
                                                     const int32_t* __restrict__ slots) {
  const int64_t p = (int64_t)blockIdx.x * 128 + (threadIdx.x >> 1);
  const int half = threadIdx.x & 1;
  const bool valid = p < nrows * kk;
  int64_t e = 0, slot = -1;
  if (valid) {
    const int64_t r = p / kk;
    const int64_t q = slots ? slots[r] : r;
    e = q * kk + (p - r * kk);
    slot = ri[e];
  }
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  if (slot >= 0) {
    const float4* xv4 = reinterpret_cast<const float4*>(rows + slot * (int64_t)dp) + half;
    const float4* qv4 = reinterpret_cast<const float4*>(qpad + (e / kk) * (int64_t)dp) + half;
    auto step = [&](const float4 x, const float4 y) {
      if (METRIC == QUAKE_L2) {
        a0 = fmaf(x.x - y.x, x.x - y.x, a0);
        a1 = fmaf(x.y - y.y, x.y - y.y, a1);
        a2 = fmaf(x.z - y.z, x.z - y.z, a2);
        a3 = fmaf(x.w - y.w, x.w - y.w, a3);
      } else {
        a0 = fmaf(x.x, y.x, a0);
        a1 = fmaf(x.y, y.y, a1);
        a2 = fmaf(x.z, y.z, a2);
        a3 = fmaf(x.w, y.w, a3);
      }
    };
    // eight steps' loads are issued before their products (the sums still
    // run in order, step by step)
    const int steps = dp / 8, whole = steps & ~7;
    for (int i0 = 0; i0 < whole; i0 += 8) {
      float4 xs[8], ys[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        xs[u] = xv4[2 * (i0 + u)];
        ys[u] = qv4[2 * (i0 + u)];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) step(xs[u], ys[u]);
    }
    for (int i = whole; i < steps; ++i) step(xv4[2 * i], qv4[2 * i]);
  }
  // pairwise: ((p0+p1)+(p2+p3))+((p4+p5)+(p6+p7)), the two halves from the
  // lane pair (every lane takes part in the shuffle)
  float acc = (a0 + a1) + (a2 + a3);
  acc += __shfl_xor(acc, 1);
  if (slot >= 0 && half == 0) rk[e] = METRIC == QUAKE_L2 ? acc : -acc;
}

// One wave per row: the row's kk (distance, id) pairs sorted ascending with a
// bitonic network across the wave (kk <= 64); the best k are written back.
__global__ __launch_bounds__(256) void k_rerank_select(int64_t nrows, int k, int kk, const int64_t* __restrict__ sid,
                                                       float* __restrict__ rk, int64_t* __restrict__ ri,
                                                       const int32_t* __restrict__ slots) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= nrows) return;
  const int lane = threadIdx.x & 63;
  const int64_t q = slots ? slots[r] : r;
  const int64_t myslot = lane < kk ? ri[q * kk + lane] : -1;
  float key = KEY_EMPTY;
  int64_t id = -1;
  if (myslot >= 0) {
    key = rk[q * kk + lane];
    id = sid[myslot];
  }
  for (int size = 2; size <= WAVE; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const float ok = __shfl_xor(key, stride);
      const int64_t oi = shfl_xor_i64(id, stride);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const bool other_first = kv_less(ok, oi, key, id);
      const bool take = (lower == up) ? other_first : !other_first;
      if (take) { key = ok; id = oi; }
    }
  }
  if (lane < k) { rk[q * kk + lane] = key; ri[q * kk + lane] = id; }
}

void launch_rerank(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s, bool exact,
                   const int32_t* slots, int64_t nslots) {
  const int64_t n = slots ? nslots : a.nq;
  if (n <= 0) return;
  const int64_t pairs = n * a.kk;
  const dim3 g1((unsigned)((pairs + 127) / 128)), g2((unsigned)((n + 3) / 4));
  // without the FP32 re-scoring the 16-bit path's keys stay and are ranked as they are
  if (exact && a.metric == QUAKE_L2)
    hipLaunchKernelGGL(k_rerank_dist<QUAKE_L2>, g1, dim3(256), 0, s, n, a.kk, ws.q, st.dp, st.rows32, ws.rk, ws.ri,
                       slots);
  else if (exact)
    hipLaunchKernelGGL(k_rerank_dist<QUAKE_IP>, g1, dim3(256), 0, s, n, a.kk, ws.q, st.dp, st.rows32, ws.rk, ws.ri,
                       slots);
  hipLaunchKernelGGL(k_rerank_select, g2, dim3(256), 0, s, n, a.k, a.kk, st.ids, ws.rk, ws.ri, slots);
}

}  // namespace qk

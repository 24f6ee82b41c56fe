// Partition store kernels: placing rows into tiles, and exporting the layout.
#include "common.hpp"
#include "index.hpp"

namespace qk {

__device__ __forceinline__ uint16_t to_bf16(float f) {
  // round to nearest, ties to even, on the upper 16 bits of the binary32 value
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint16_t to_f16(float f) {
  const _Float16 h = (_Float16)f;
  return __builtin_bit_cast(uint16_t, h);
}

// Row i goes to store slot slot[i] = tile * 64 + lane.  One thread moves one
// 4-float chunk: FP32 at [tile][chunk][lane][4], the 16-bit copy at
// [tile][chunk/2][lane][8] (half of an 8-element group per thread; the copy's
// rows are dp16 long and the chunks past dp stay zero).
__global__ __launch_bounds__(256) void k_scatter(const float* __restrict__ x, int64_t n, int d, int dp, int dp16,
                                                  const int64_t* __restrict__ ids, const int64_t* __restrict__ slot,
                                                  float* __restrict__ v32, uint16_t* __restrict__ v16, int dtype16,
                                                  float* __restrict__ rows32, int64_t* __restrict__ sid) {
  const int nch4 = dp >> 2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = e / nch4;
  if (row >= n) return;
  const int c4 = (int)(e - row * nch4);
  const int64_t sl = slot[row];
  const int64_t tile = sl / TILE;
  const int lane = (int)(sl - tile * TILE);
  float v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = c4 * 4 + u;
    v[u] = (j < d) ? x[row * d + j] : 0.f;
  }
  if (v32) reinterpret_cast<float4*>(v32)[(tile * nch4 + c4) * TILE + lane] = make_float4(v[0], v[1], v[2], v[3]);
  if (v16) {
    const int c8 = c4 >> 1, half = c4 & 1;
    uint16_t* d16 = v16 + ((tile * (dp16 >> 3) + c8) * TILE + lane) * 8 + half * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) d16[u] = dtype16 == QUAKE_F16 ? to_f16(v[u]) : to_bf16(v[u]);
  }
  if (rows32) *reinterpret_cast<float4*>(rows32 + sl * dp + c4 * 4) = make_float4(v[0], v[1], v[2], v[3]);
  if (c4 == 0) sid[sl] = ids ? ids[row] : row;
}

void launch_scatter(const float* x, int64_t n, int d, int dp, int dp16, const int64_t* ids, const int64_t* slot,
                    float* v32, uint16_t* v16, int dtype16, float* rows32, int64_t* sid, hipStream_t s) {
  const int64_t total = n * (dp >> 2);
  if (total <= 0) return;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x, n, d, dp, dp16, ids, slot,
                     v32, v16, dtype16, rows32, sid);
}

// ids and partition of every filled slot, partition by partition.
__global__ __launch_bounds__(256) void k_export(const int64_t* __restrict__ sid, const int64_t* __restrict__ poff,
                                                 const int32_t* __restrict__ psize,
                                                 const int64_t* __restrict__ first_out, int64_t* __restrict__ ids,
                                                 int32_t* __restrict__ part) {
  const int p = blockIdx.x;
  const int64_t base = poff[p] * TILE;
  const int64_t o = first_out[p];
  for (int s = threadIdx.x; s < psize[p]; s += 256) {
    ids[o + s] = sid[base + s];
    part[o + s] = p;
  }
}

void launch_export(const Store& st, int64_t* ids, int32_t* part, const int64_t* first_out, hipStream_t s) {
  if (st.nlist <= 0) return;
  hipLaunchKernelGGL(k_export, dim3((unsigned)st.nlist), dim3(256), 0, s, st.ids, st.d_off, st.d_size, first_out, ids,
                     part);
}

}  // namespace qk

// Kernels of the maintenance pass (Sec. 4.2, "Maintenance Actions"): rows of
// partitions gathered out of the tile store, the farthest-row start and the
// assignment step of the 2-means split, and nearest-centroid assignment
// within a candidate set (refinement and deletes).  Centroid updates reuse
// the build's exact fixed-point k-means accumulation.
#include "common.hpp"
#include "index.hpp"

namespace qk {

namespace {

dim3 grid_of(int64_t n, int per_block = 256) { return dim3((unsigned)((n + per_block - 1) / per_block)); }

// Ascending-is-nearer key of row x against centroid c, one wave, FP32:
// squared L2 in the difference form, or the negated inner product.
__device__ __forceinline__ float wave_key(const float* __restrict__ x, const float* __restrict__ c, int dp, int ip) {
  float acc = 0.f;
  for (int j = lane_id(); j < dp; j += WAVE) {
    if (ip) {
      acc = fmaf(x[j], c[j], acc);
    } else {
      const float d = x[j] - c[j];
      acc = fmaf(d, d, acc);
    }
  }
  acc = wave_sum_f(acc);
  return ip ? -acc : acc;
}

}  // namespace

// out[i] = the FP32 vector of store slot slots[i], row-major [n][dp].
__global__ __launch_bounds__(256) void k_gather_slots(const float* __restrict__ v32, const int64_t* __restrict__ slots,
                                                      int64_t n, int dp, float* __restrict__ out) {
  const int nch4 = dp >> 2;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = e / nch4;
  if (i >= n) return;
  const int c4 = (int)(e - i * nch4);
  const int64_t sl = slots[i];
  const int64_t tile = sl / TILE;
  const int lane = (int)(sl - tile * TILE);
  reinterpret_cast<float4*>(out)[i * nch4 + c4] =
      reinterpret_cast<const float4*>(v32)[(tile * nch4 + c4) * TILE + lane];
}

void launch_gather_slots(const Store& st, const int64_t* slots, int64_t n, float* out, hipStream_t s) {
  // without FP32 tiles the row-major FP32 copy holds the same values by slot
  if (!st.v32) {
    launch_gather_rows(st.rows32, st.dp, slots, n, st.dp, out, s);
    return;
  }
  const int64_t total = n * (st.dp >> 2);
  if (total > 0) hipLaunchKernelGGL(k_gather_slots, grid_of(total), dim3(256), 0, s, st.v32, slots, n, st.dp, out);
}

// Per segment s (rows [lo[s], lo[s+1]) of x): the row with the largest key
// against ref[s] (ties to the lower row).  One 256-thread block per segment.
__global__ __launch_bounds__(256) void k_seg_farthest(const float* __restrict__ x, const int64_t* __restrict__ lo,
                                                      const float* __restrict__ ref, int dp, int ip,
                                                      int64_t* __restrict__ far) {
  __shared__ float bk[4];
  __shared__ int64_t br[4];
  const int seg = blockIdx.x;
  const int wave = threadIdx.x >> 6;
  const int64_t a = lo[seg], b = lo[seg + 1];
  const float* c = ref + (int64_t)seg * dp;
  float best = -__builtin_inff();
  int64_t brow = -1;
  for (int64_t r = a + wave; r < b; r += 4) {
    const float key = wave_key(x + r * dp, c, dp, ip);
    if (brow < 0 || key > best) { best = key; brow = r; }  // rows ascend per wave: strict > keeps the lower
  }
  if (lane_id() == 0) { bk[wave] = best; br[wave] = brow; }
  __syncthreads();
  if (threadIdx.x == 0) {
    float kb = bk[0];
    int64_t rb = br[0];
    for (int w = 1; w < 4; ++w) {
      if (br[w] < 0) continue;
      if (rb < 0 || bk[w] > kb || (bk[w] == kb && br[w] < rb)) { kb = bk[w]; rb = br[w]; }
    }
    far[seg] = rb;
  }
}

void launch_seg_farthest(const float* x, const int64_t* lo, int64_t nseg, const float* ref, int dp, int metric,
                         int64_t* far, hipStream_t s) {
  if (nseg > 0)
    hipLaunchKernelGGL(k_seg_farthest, dim3((unsigned)nseg), dim3(256), 0, s, x, lo, ref, dp,
                       metric == QUAKE_IP ? 1 : 0, far);
}

// 2-means assignment: row i of segment seg[i] goes to cluster 2 seg + 1 when
// it is strictly nearer to c[2 seg + 1] than to c[2 seg], else to 2 seg.
// One wave per row.
__global__ __launch_bounds__(256) void k_seg_assign2(const float* __restrict__ x, int64_t n,
                                                     const int32_t* __restrict__ seg, const float* __restrict__ c,
                                                     int dp, int ip, int32_t* __restrict__ lab) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int g = seg[i];
  const float k0 = wave_key(x + i * dp, c + (int64_t)(2 * g) * dp, dp, ip);
  const float k1 = wave_key(x + i * dp, c + (int64_t)(2 * g + 1) * dp, dp, ip);
  if (lane_id() == 0) lab[i] = 2 * g + (k1 < k0 ? 1 : 0);
}

void launch_seg_assign2(const float* x, int64_t n, const int32_t* seg, const float* c, int dp, int metric,
                        int32_t* lab, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_seg_assign2, grid_of(n, 4), dim3(256), 0, s, x, n, seg, c, dp, metric == QUAKE_IP ? 1 : 0,
                       lab);
}

// Nearest of the G centroids c[G][dp] for every row (ties to the lower
// index): lab[i] in [0, G).  One wave per row.
__global__ __launch_bounds__(256) void k_nearest_of(const float* __restrict__ x, int64_t n,
                                                    const float* __restrict__ c, int G, int dp, int ip,
                                                    int32_t* __restrict__ lab) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  float best = 0.f;
  int bg = 0;
  for (int g = 0; g < G; ++g) {
    const float key = wave_key(x + i * dp, c + (int64_t)g * dp, dp, ip);
    if (g == 0 || key < best) { best = key; bg = g; }
  }
  if (lane_id() == 0) lab[i] = bg;
}

void launch_nearest_of(const float* x, int64_t n, const float* c, int G, int dp, int metric, int32_t* lab,
                       hipStream_t s) {
  if (n > 0 && G > 0)
    hipLaunchKernelGGL(k_nearest_of, grid_of(n, 4), dim3(256), 0, s, x, n, c, G, dp, metric == QUAKE_IP ? 1 : 0,
                       lab);
}

// c[rows[g]] = src[g] for g < G (rows of [.][dp]).
__global__ __launch_bounds__(64) void k_put_rows(const float* __restrict__ src, const int32_t* __restrict__ rows,
                                                 int dp, float* __restrict__ c) {
  const int g = blockIdx.x;
  const int64_t r = rows[g];
  for (int j = threadIdx.x; j < dp; j += WAVE) c[r * dp + j] = src[(int64_t)g * dp + j];
}

void launch_put_rows(const float* src, const int32_t* rows, int64_t G, int dp, float* c, hipStream_t s) {
  if (G > 0) hipLaunchKernelGGL(k_put_rows, dim3((unsigned)G), dim3(64), 0, s, src, rows, dp, c);
}

}  // namespace qk

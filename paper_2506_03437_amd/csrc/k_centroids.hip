// Centroid-side kernels: query padding, centroid scoring, candidate selection,
// bisector geometry for the recall model, and the k-means build steps.
//
// Distances are squared Euclidean in the difference form sum (a_i - b_i)^2,
// never |a|^2 - 2ab + |b|^2: near neighbours sit far from the origin in these
// workloads and the expansion would cancel most of the FP32 significand.
// Sums over the dimension are blocked: 32-dimension partial sums are added to
// a running total, which bounds the relative rounding error by about
// (32 + d/32) * 2^-24 instead of d * 2^-24.
#include "common.hpp"
#include "index.hpp"

namespace qk {

// ---------------------------------------------------------------- padding

__global__ __launch_bounds__(256) void k_pad_rows(const float* __restrict__ x, int64_t n, int d, int dp,
                                                   float* __restrict__ out, double* __restrict__ norm2,
                                                   uint32_t* __restrict__ bad) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double acc = 0.0;
  bool finite = true;
  for (int j = lane; j < dp; j += WAVE) {
    const float v = (j < d) ? x[row * d + j] : 0.0f;
    out[row * dp + j] = v;
    finite &= __builtin_isfinite(v);
    acc += (double)v * (double)v;
  }
  acc = wave_sum_d(acc);
  if (norm2 && lane == 0) norm2[row] = acc;
  if (bad && __ballot(!finite) && lane == 0) atomicOr(bad, 1u);
}

void launch_pad_rows(const float* x, int64_t n, int d, int dp, float* out, double* norm2, hipStream_t s,
                     uint32_t* bad) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, x, n, d, dp, out, norm2, bad);
}

// ---------------------------------------------------------------- input checks

__global__ __launch_bounds__(256) void k_nonfinite(const float4* __restrict__ x4, const float* __restrict__ x,
                                                    int64_t n, uint32_t* __restrict__ bad) {
  bool finite = true;
  const int64_t n4 = ((uintptr_t)x & 15) == 0 ? n / 4 : 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n4; e += (int64_t)gridDim.x * 256) {
    const float4 v = x4[e];
    finite &= __builtin_isfinite(v.x) && __builtin_isfinite(v.y) && __builtin_isfinite(v.z) &&
              __builtin_isfinite(v.w);
  }
  for (int64_t e = n4 * 4 + (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    finite &= __builtin_isfinite(x[e]);
  if (__ballot(!finite) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

void launch_nonfinite(const float* x, int64_t n, uint32_t* bad, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n / 4 + 255) / 256, 8192));
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const float4*>(x), x,
                     n, bad);
}

__global__ __launch_bounds__(256) void k_check_range(const int32_t* __restrict__ a, int64_t n, int64_t nlist,
                                                      uint32_t* __restrict__ bad) {
  bool ok = true;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    ok &= a[e] >= 0 && (int64_t)a[e] < nlist;
  if (__ballot(!ok) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

void launch_check_range(const int32_t* a, int64_t n, int64_t nlist, uint32_t* bad, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_check_range, dim3((unsigned)blocks), dim3(256), 0, s, a, n, nlist, bad);
}

// ---------------------------------------------------------------- scoring

constexpr int ST = 64;      // rows / columns per score tile
constexpr int SK = 32;      // dimensions per LDS stage (one blocked partial sum)
constexpr int SLD = SK + 4; // LDS row stride (floats): 16-byte aligned, spreads banks

// Stage a 64 x 32 slab of a row-major [rows][dp] matrix into LDS [64][SLD].
__device__ __forceinline__ void stage_slab(float (*dst)[SLD], const float* __restrict__ src, int64_t row0,
                                           int64_t rows, int dp, int k0) {
  for (int e = threadIdx.x; e < ST * (SK / 4); e += 256) {
    const int r = e >> 3, k4 = (e & 7) * 4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t g = row0 + r;
    if (g < rows && k0 + k4 < dp) v = *reinterpret_cast<const float4*>(src + g * dp + k0 + k4);
    *reinterpret_cast<float4*>(&dst[r][k4]) = v;
  }
}

// acc[i][j] += sum over the staged 32 dims of f(a[row ty+16i], b[row tx+16j]).
template <int METRIC>
__device__ __forceinline__ void tile_stage(const float (*qs)[SLD], const float (*cs)[SLD], int tx, int ty,
                                           float acc[4][4]) {
  float part[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) part[i][j] = 0.f;
#pragma unroll 2
  for (int kk = 0; kk < SK; kk += 4) {
    float4 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const float4*>(&qs[ty + 16 * i][kk]);
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const float4*>(&cs[tx + 16 * j][kk]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (METRIC == QUAKE_L2) {
          float t;
          t = a[i].x - b[j].x; part[i][j] = fmaf(t, t, part[i][j]);
          t = a[i].y - b[j].y; part[i][j] = fmaf(t, t, part[i][j]);
          t = a[i].z - b[j].z; part[i][j] = fmaf(t, t, part[i][j]);
          t = a[i].w - b[j].w; part[i][j] = fmaf(t, t, part[i][j]);
        } else {
          part[i][j] = fmaf(a[i].x, b[j].x, part[i][j]);
          part[i][j] = fmaf(a[i].y, b[j].y, part[i][j]);
          part[i][j] = fmaf(a[i].z, b[j].z, part[i][j]);
          part[i][j] = fmaf(a[i].w, b[j].w, part[i][j]);
        }
      }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] += part[i][j];
}

// S[q][c] = |q - c|^2 (L2) or q . c (IP) for a 64 x 64 tile per block.  The
// slabs are double-buffered: the next slab's share of every thread is read
// into registers while the current one is scored from LDS, so one barrier
// per slab remains and the global loads' latency hides behind the products.
template <int METRIC>
__global__ __launch_bounds__(256) void k_scores(const float* __restrict__ q, int64_t nq,
                                                 const float* __restrict__ c, int64_t nc, int dp,
                                                 float* __restrict__ out) {
  __shared__ float qs[2][ST][SLD];
  __shared__ float cs[2][ST][SLD];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * ST, q0 = (int64_t)blockIdx.y * ST;
  // this thread's two 16-byte pieces of each 64 x 32 slab (pieces e and
  // e + 256 of the slab's 512: row e >> 3, dimensions (e & 7) * 4 ..)
  auto fetch = [&](const float* __restrict__ src, int64_t row0, int64_t rows, int k0, float4 (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      const int r = e >> 3, k4 = (e & 7) * 4;
      const int64_t g = row0 + r;
      v[h] = (g < rows && k0 + k4 < dp) ? *reinterpret_cast<const float4*>(src + g * dp + k0 + k4)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto put = [&](float (*dst)[SLD], const float4 (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      *reinterpret_cast<float4*>(&dst[e >> 3][(e & 7) * 4]) = v[h];
    }
  };
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  float4 vq[2], vc[2];
  fetch(q, q0, nq, 0, vq);
  fetch(c, c0, nc, 0, vc);
  put(qs[0], vq);
  put(cs[0], vc);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < dp; k0 += SK) {
    const bool more = k0 + SK < dp;
    if (more) {
      fetch(q, q0, nq, k0 + SK, vq);
      fetch(c, c0, nc, k0 + SK, vc);
    }
    tile_stage<METRIC>(qs[buf], cs[buf], tx, ty, acc);
    // the other buffer was last read before the previous barrier
    if (more) {
      put(qs[buf ^ 1], vq);
      put(cs[buf ^ 1], vc);
    }
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t qi = q0 + ty + 16 * i;
    if (qi >= nq) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t ci = c0 + tx + 16 * j;
      if (ci < nc) out[qi * nc + ci] = acc[i][j];
    }
  }
}

// Inner-product scores on the FP32 matrix cores: the same 64 x 64 tiles
// and double-buffered 32-dimension slabs as k_scores, each wave computing a
// 32 x 32 quarter as 2 x 2 blocks of v_mfma_f32_16x16x4_f32 (FP32 products
// and sums: a dot product has no cancellation to guard against, unlike the
// L2 difference form, which stays on the vector units).
typedef __attribute__((ext_vector_type(4))) float f32x4v;

__global__ __launch_bounds__(256) void k_scores_ip_mfma(const float* __restrict__ q, int64_t nq,
                                                        const float* __restrict__ c, int64_t nc, int dp,
                                                        float* __restrict__ out) {
  __shared__ float qs[2][ST][SLD];
  __shared__ float cs[2][ST][SLD];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;  // the wave's 32 x 32 quarter of the tile
  const int64_t c0 = (int64_t)blockIdx.x * ST, q0 = (int64_t)blockIdx.y * ST;
  auto fetch = [&](const float* __restrict__ src, int64_t row0, int64_t rows, int k0, float4 (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      const int r = e >> 3, k4 = (e & 7) * 4;
      const int64_t g = row0 + r;
      v[h] = (g < rows && k0 + k4 < dp) ? *reinterpret_cast<const float4*>(src + g * dp + k0 + k4)
                                         : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto put = [&](float (*dst)[SLD], const float4 (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + 256 * h;
      *reinterpret_cast<float4*>(&dst[e >> 3][(e & 7) * 4]) = v[h];
    }
  };
  f32x4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4v{0.f, 0.f, 0.f, 0.f};
  // operand lanes: row (query or centroid) lane & 15 of a 16-block, dimension lane >> 4 of a 4-step
  const int r16 = lane & 15, k4 = lane >> 4;
  float4 vq[2], vc[2];
  fetch(q, q0, nq, 0, vq);
  fetch(c, c0, nc, 0, vc);
  put(qs[0], vq);
  put(cs[0], vc);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < dp; k0 += SK) {
    const bool more = k0 + SK < dp;
    if (more) {
      fetch(q, q0, nq, k0 + SK, vq);
      fetch(c, c0, nc, k0 + SK, vc);
    }
    // each slab's 32 dimensions are summed on their own and then added in
    // (the blocked partial sums of k_scores: a short chain per slab instead
    // of one chain over all dimensions keeps the rounding error small)
    f32x4v part[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) part[i][j] = f32x4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < SK; kk += 4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = qs[buf][wm * 32 + i * 16 + r16][kk + k4];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = cs[buf][wn * 32 + j * 16 + r16][kk + k4];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          part[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], part[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] += part[i][j];
    if (more) {
      put(qs[buf ^ 1], vq);
      put(cs[buf ^ 1], vc);
    }
    __syncthreads();
    buf ^= 1;
  }
  // D[4 (lane >> 4) + r][lane & 15] of each 16 x 16 block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t qi = q0 + wm * 32 + i * 16 + 4 * k4 + r;
      if (qi >= nq) continue;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t ci = c0 + wn * 32 + j * 16 + r16;
        if (ci < nc) out[qi * nc + ci] = acc[i][j][r];
      }
    }
}

void launch_scores(const float* q, int64_t nq, const float* c, int64_t nc, int dp, int metric, float* out,
                   hipStream_t s) {
  if (nq <= 0 || nc <= 0) return;
  dim3 grid((unsigned)((nc + ST - 1) / ST), (unsigned)((nq + ST - 1) / ST));
  if (metric == QUAKE_L2)
    hipLaunchKernelGGL(k_scores<QUAKE_L2>, grid, dim3(256), 0, s, q, nq, c, nc, dp, out);
  else
    hipLaunchKernelGGL(k_scores_ip_mfma, grid, dim3(256), 0, s, q, nq, c, nc, dp, out);
}

// Nearest centroid of every row (k-means assignment and the build's final
// placement).  Lower centroid index wins exact ties.
template <int METRIC>
__global__ __launch_bounds__(256) void k_assign(const float* __restrict__ x, int64_t n,
                                                 const float* __restrict__ c, int64_t nc, int dp,
                                                 int32_t* __restrict__ assign) {
  __shared__ float qs[ST][SLD];
  __shared__ float cs[ST][SLD];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * ST;
  float best[4];
  int32_t bidx[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { best[i] = KEY_EMPTY; bidx[i] = 0x7fffffff; }
  for (int64_t c0 = 0; c0 < nc; c0 += ST) {
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    for (int k0 = 0; k0 < dp; k0 += SK) {
      stage_slab(qs, x, r0, n, dp, k0);
      stage_slab(cs, c, c0, nc, dp, k0);
      __syncthreads();
      tile_stage<METRIC>(qs, cs, tx, ty, acc);
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t ci = c0 + tx + 16 * j;
      if (ci >= nc) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float key = (METRIC == QUAKE_L2) ? acc[i][j] : -acc[i][j];
        if (key < best[i] || (key == best[i] && (int32_t)ci < bidx[i])) { best[i] = key; bidx[i] = (int32_t)ci; }
      }
    }
  }
  // the 16 lanes tx = 0..15 of a row group hold different columns: reduce
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    for (int o = 8; o > 0; o >>= 1) {
      const float ob = __shfl_xor(best[i], o);
      const int32_t oi = __shfl_xor(bidx[i], o);
      if (ob < best[i] || (ob == best[i] && oi < bidx[i])) { best[i] = ob; bidx[i] = oi; }
    }
    const int64_t row = r0 + ty + 16 * i;
    if (tx == 0 && row < n) assign[row] = bidx[i];
  }
}

void launch_assign(const float* x, int64_t n, int dp, const float* c, int64_t nc, int metric, int32_t* assign,
                   hipStream_t s) {
  if (n <= 0) return;
  dim3 grid((unsigned)((n + ST - 1) / ST));
  if (metric == QUAKE_L2)
    hipLaunchKernelGGL(k_assign<QUAKE_L2>, grid, dim3(256), 0, s, x, n, c, nc, dp, assign);
  else
    hipLaunchKernelGGL(k_assign<QUAKE_IP>, grid, dim3(256), 0, s, x, n, c, nc, dp, assign);
}

// ---------------------------------------------------------------- selection

constexpr int SORT_N = 4096;

__device__ __forceinline__ uint64_t composite(float key, uint32_t idx) {
  return ((uint64_t)float_order(key) << 32) | idx;
}

__device__ __forceinline__ float float_unorder(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// The M best centroids of every query by (key, centroid id), ascending.
__global__ __launch_bounds__(256) void k_select(const float* __restrict__ scores, int64_t nc, int M, int ip,
                                                 int32_t* __restrict__ cand) {
  __shared__ uint64_t buf[SORT_N];
  const int64_t qi = blockIdx.x;
  const float* s = scores + qi * nc;
  int keep = 1;
  while (keep < M) keep <<= 1;
  int64_t next = 0;
  int filled = 0;
  bool first = true;
  while (first || next < nc) {
    const int base = first ? 0 : keep;
    int64_t take = nc - next;
    if (take > SORT_N - base) take = SORT_N - base;
    int n = base + (int)take;
    int p2 = 1;
    while (p2 < n) p2 <<= 1;
    for (int e = threadIdx.x; e < p2 - base; e += 256) {
      uint64_t v = ~0ull;
      if (e < take) {
        const float raw = s[next + e];
        v = composite(ip ? -raw : raw, (uint32_t)(next + e));
      }
      buf[base + e] = v;
    }
    next += take;
    filled = n;
    bitonic_sort_u64(buf, p2);
    first = false;
  }
  (void)filled;
  for (int i = threadIdx.x; i < M; i += 256) cand[qi * M + i] = (int32_t)(uint32_t)(buf[i] & 0xffffffffu);
}

void launch_select(const float* scores, int64_t nq, int64_t nc, int M, int metric, int32_t* cand,
                   hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_select, dim3((unsigned)nq), dim3(256), 0, s, scores, nc, M, metric == QUAKE_IP ? 1 : 0,
                     cand);
}

// ---------------------------------------------------------------- geometry

// Distance h_i from the query to the bisector hyperplane of c_0 and c_i,
// evaluated as the projection (c_0 - c_i) . (q - (c_0 + c_i)/2) / |c_0 - c_i|
// for L2 and q . (c_0 - c_i) / |c_0 - c_i| for inner product (the boundary
// of the two inner-product cells), then the candidates after c_0 are put in
// ascending h order; ties keep the (key, id) order of the selection.
__global__ __launch_bounds__(256) void k_geometry(const float* __restrict__ q, const float* __restrict__ c, int dp,
                                                   int stride, const int32_t* __restrict__ mq, int ip,
                                                   const int32_t* __restrict__ sel, int32_t* __restrict__ order,
                                                   float* __restrict__ hout) {
  __shared__ uint64_t buf[SORT_N];
  const int64_t qi = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int M = mq[qi];
  const int32_t* cq = sel + qi * stride;
  if (M <= 0) {  // no candidate at all (an empty upper-level result)
    for (int t = threadIdx.x; t < stride; t += 256) { order[qi * stride + t] = -1; hout[qi * stride + t] = 0.f; }
    return;
  }
  const int c0 = cq[0];
  const float* qv = q + qi * dp;
  const float* c0v = c + (int64_t)c0 * dp;
  for (int i = 1 + w; i < M; i += 4) {
    const float* civ = c + (int64_t)cq[i] * dp;
    float num = 0.f, sep = 0.f;
    for (int j = lane; j < dp; j += WAVE) {
      const float a = c0v[j], b = civ[j], x = qv[j];
      const float diff = a - b;
      sep = fmaf(diff, diff, sep);
      num = ip ? fmaf(x, diff, num) : fmaf(diff, (x - a) + (x - b), num);
    }
    num = wave_sum_f(num);
    sep = wave_sum_f(sep);
    float h = 0.f;
    if (sep > 0.f) h = ip ? num / sqrtf(sep) : num / (2.0f * sqrtf(sep));
    h = fmaxf(h, 0.f);
    if (lane == 0) buf[i - 1] = composite(h, (uint32_t)i);
  }
  int p2 = 1;
  while (p2 < M - 1) p2 <<= 1;
  for (int e = M - 1 + threadIdx.x; e < p2; e += 256) buf[e] = ~0ull;
  if (M > 1) bitonic_sort_u64(buf, p2);
  else __syncthreads();
  for (int t = threadIdx.x; t < stride; t += 256) {
    if (t == 0) {
      order[qi * stride] = c0;
      hout[qi * stride] = 0.f;
    } else if (t < M) {
      const uint64_t e = buf[t - 1];
      order[qi * stride + t] = cq[(uint32_t)(e & 0xffffffffu)];
      hout[qi * stride + t] = float_unorder((uint32_t)(e >> 32));
    } else {
      order[qi * stride + t] = -1;
      hout[qi * stride + t] = 0.f;
    }
  }
}

void launch_geometry(const float* q, const float* c, int64_t nq, int dp, int M, const int32_t* mq, int metric,
                     const int32_t* sel, int32_t* order, float* h, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_geometry, dim3((unsigned)nq), dim3(256), 0, s, q, c, dp, M, mq, metric == QUAKE_IP ? 1 : 0,
                     sel, order, h);
}

// ---------------------------------------------------------------- block selection (64 < M <= 256)

// One block per query for candidate sets past one wave.  Selection is a
// radix select on the order-preserving bits of the keys (value for L2,
// negated score for IP; ties by centroid id): four 8-bit digit passes with
// an LDS histogram find the M-th key T, then every key below T and the
// lowest-id keys equal to T are gathered and sorted by (key, id).
// Geometry (adaptive mode) as in k_geometry - the projection form, since a
// difference of two scores would cancel most of the significand for close
// centroids - with the query and c_0 held in registers (D4 float4 per
// lane) and each wave taking every fourth candidate row; then the
// candidates after c_0 are sorted by (h, selection rank).
template <int KPT, int D4>
__global__ __launch_bounds__(256) void k_select_large(const float* __restrict__ scores, int64_t nc, int M, int ip,
                                                       int aps, const float* __restrict__ q,
                                                       const float* __restrict__ c, int dp,
                                                       int32_t* __restrict__ cand, float* __restrict__ hout) {
  __shared__ uint32_t hist[256];
  __shared__ uint64_t buf[256];
  __shared__ int32_t ids[256];
  __shared__ uint32_t s_digit, s_below, s_count;
  const int tid = threadIdx.x;
  const int64_t qi = blockIdx.x;
  const float* sq = scores + qi * nc;
  uint32_t key[KPT];
#pragma unroll
  for (int t = 0; t < KPT; ++t) {
    const int64_t j = (int64_t)t * 256 + tid;
    key[t] = j < nc ? float_order(ip ? -sq[j] : sq[j]) : 0xffffffffu;
  }
  // radix select: T = the M-th smallest key; `need` keys equal to T are taken
  uint32_t prefix = 0, mask = 0;
  int need = M;
  for (int shift = 24; shift >= 0; shift -= 8) {
    hist[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < KPT; ++t)
      if ((key[t] & mask) == prefix && (int64_t)t * 256 + tid < nc) atomicAdd(&hist[(key[t] >> shift) & 255u], 1u);
    __syncthreads();
    if (tid < WAVE) {
      // inclusive scan of the 256 bins, four per lane
      const uint32_t a0 = hist[4 * tid], a1 = hist[4 * tid + 1], a2 = hist[4 * tid + 2], a3 = hist[4 * tid + 3];
      const uint32_t mine = a0 + a1 + a2 + a3;
      uint32_t run = mine;
      for (int o = 1; o < WAVE; o <<= 1) {
        const uint32_t u = __shfl_up(run, o);
        if (tid >= o) run += u;
      }
      const uint32_t before = run - mine;
      const uint32_t c1 = before + a0, c2 = c1 + a1, c3 = c2 + a2, c4 = c3 + a3;
      const uint32_t n = (uint32_t)need;
      if (before < n && c4 >= n) {
        int d;
        uint32_t below;
        if (c1 >= n) { d = 0; below = before; }
        else if (c2 >= n) { d = 1; below = c1; }
        else if (c3 >= n) { d = 2; below = c2; }
        else { d = 3; below = c3; }
        s_digit = (uint32_t)(4 * tid + d);
        s_below = below;
      }
    }
    __syncthreads();
    prefix |= s_digit << shift;
    mask |= 0xffu << shift;
    need -= (int)s_below;
    __syncthreads();
  }
  const uint32_t T = prefix;
  // gather: keys below T, then `need` keys equal to T, the lowest ids first
  if (tid == 0) s_count = 0;
  buf[tid] = ~0ull;
  int eqs = 0;
#pragma unroll
  for (int t = 0; t < KPT; ++t) eqs += ((int64_t)t * 256 + tid < nc && key[t] == T) ? 1 : 0;
  hist[tid] = (uint32_t)eqs;
  __syncthreads();
#pragma unroll
  for (int t = 0; t < KPT; ++t) {
    const int64_t j = (int64_t)t * 256 + tid;
    if (j < nc && key[t] < T) buf[atomicAdd(&s_count, 1u)] = ((uint64_t)key[t] << 32) | (uint32_t)j;
  }
  if (tid == 0) {
    uint32_t tot = 0;
    for (int u = 0; u < 256; ++u) tot += hist[u];
    s_digit = tot;
  }
  __syncthreads();
  if ((int)s_digit == need) {  // the usual case: every key equal to T is taken
#pragma unroll
    for (int t = 0; t < KPT; ++t) {
      const int64_t j = (int64_t)t * 256 + tid;
      if (j < nc && key[t] == T) buf[atomicAdd(&s_count, 1u)] = ((uint64_t)T << 32) | (uint32_t)j;
    }
  } else {
    // more ties than places: ids run t * 256 + tid, so chunk by chunk in id order
    int taken = 0;
    for (int t = 0; t < KPT && taken < need; ++t) {
      const int64_t j = (int64_t)t * 256 + tid;
      const bool eq = j < nc && key[t] == T;
      __syncthreads();
      hist[tid] = eq ? 1u : 0u;
      __syncthreads();
      uint32_t rank = 0, total = 0;
      for (int u = 0; u < 256; ++u) {
        const uint32_t v = hist[u];
        rank += (u < tid) ? v : 0u;
        total += v;
      }
      if (eq && taken + (int)rank < need) buf[atomicAdd(&s_count, 1u)] = ((uint64_t)T << 32) | (uint32_t)j;
      taken += (int)total;
    }
  }
  bitonic_sort_u64(buf, 256);
  // buf[0..M) holds the M best in (key, id) order
  if (!aps) {
    if (tid < M) cand[qi * M + tid] = (int32_t)(uint32_t)(buf[tid] & 0xffffffffu);
    return;
  }
  const int32_t c0 = (int32_t)(uint32_t)(buf[0] & 0xffffffffu);
  ids[tid] = tid < M ? (int32_t)(uint32_t)(buf[tid] & 0xffffffffu) : -1;
  __syncthreads();
  {
    const int w = tid >> 6, lane = tid & 63;
    const float4* qv = reinterpret_cast<const float4*>(q + qi * dp);
    const float4* c0v = reinterpret_cast<const float4*>(c + (int64_t)c0 * dp);
    const int n4 = dp >> 2;
    float4 qr[D4], ar[D4];
#pragma unroll
    for (int t = 0; t < D4; ++t) {
      const int j = t * WAVE + lane;
      qr[t] = j < n4 ? qv[j] : make_float4(0.f, 0.f, 0.f, 0.f);
      ar[t] = j < n4 ? c0v[j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    for (int i = 1 + w; i < M; i += 4) {
      const float4* cjv = reinterpret_cast<const float4*>(c + (int64_t)ids[i] * dp);
      // the row's loads are unconditional (clamped; lanes past dp add
      // nothing), so they are all in flight before the first product
      float4 bv[D4];
#pragma unroll
      for (int t = 0; t < D4; ++t) bv[t] = cjv[min(t * WAVE + lane, n4 - 1)];
      float num = 0.f, sep = 0.f;
#pragma unroll
      for (int t = 0; t < D4; ++t) {
        const bool in = t * WAVE + lane < n4;
        const float4 a = ar[t], b = bv[t], x = qr[t];
        const float e0 = a.x - b.x, e1 = a.y - b.y, e2 = a.z - b.z, e3 = a.w - b.w;
        float s2 = fmaf(e0, e0, fmaf(e1, e1, fmaf(e2, e2, fmaf(e3, e3, sep))));
        float n2 = ip ? fmaf(x.x, e0, fmaf(x.y, e1, fmaf(x.z, e2, fmaf(x.w, e3, num))))
                      : fmaf(e0, (x.x - a.x) + (x.x - b.x),
                             fmaf(e1, (x.y - a.y) + (x.y - b.y),
                                  fmaf(e2, (x.z - a.z) + (x.z - b.z), fmaf(e3, (x.w - a.w) + (x.w - b.w), num))));
        sep = in ? s2 : sep;
        num = in ? n2 : num;
      }
      num = wave_sum_f(num);
      sep = wave_sum_f(sep);
      float hi = 0.f;
      if (sep > 0.f) hi = ip ? num / sqrtf(sep) : num / (2.0f * sqrtf(sep));
      if (lane == 0) hist[i] = __float_as_uint(fmaxf(hi, 0.f));
    }
  }
  __syncthreads();
  // order the candidates after c_0 by (h, selection rank)
  const float h = (tid >= 1 && tid < M) ? __uint_as_float(hist[tid]) : 0.f;
  buf[tid] = (tid >= 1 && tid < M) ? (((uint64_t)float_order(h) << 32) | (uint32_t)tid) : ~0ull;
  bitonic_sort_u64(buf, 256);
  if (tid == 0) {
    cand[qi * M] = c0;
    hout[qi * M] = 0.f;
  } else if (tid < M) {
    const uint64_t e = buf[tid - 1];
    cand[qi * M + tid] = ids[(uint32_t)(e & 0xffffffffu)];
    hout[qi * M + tid] = float_unorder((uint32_t)(e >> 32));
  }
}

// ---------------------------------------------------------------- fused selection (M <= 64)

// One wave per query.  Selection: chunks of 64 scores are sorted and merged
// into a running list of the 64 best (key, id), one entry per lane; chunks
// with nothing better than the running M-th entry are skipped.  Geometry
// (adaptive mode): the query and c_0 stay in registers (DPL dimensions per
// lane) and each candidate row is read once for its bisector distance, in
// the projection form and summation order of k_geometry; then the
// candidates after c_0 are sorted by (h, selection order).
template <int DPL>
__global__ __launch_bounds__(256) void k_select64(const float* __restrict__ scores, int64_t nq, int64_t nc, int M,
                                                   int ip, int geometry, const float* __restrict__ qpad,
                                                   const float* __restrict__ c, int dp, int32_t* __restrict__ cand,
                                                   float* __restrict__ hout) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= nq) return;
  const float* s = scores + q * nc;
  // (key, id) packed into integers in result order (the key's zero made
  // positive, so that -0 and +0 tie as they do as floats)
  const uint64_t empty = pack_key_slot(KEY_EMPTY, INT32_MAX);
  uint64_t l = empty;
  // each chunk's scores are requested one chunk ahead (clamped reads)
  float raw_next = s[min<int64_t>(lane, nc - 1)];
  for (int64_t base = 0; base < nc; base += WAVE) {
    const int64_t e = base + lane;
    const float raw = raw_next;
    raw_next = s[min<int64_t>(base + WAVE + lane, nc - 1)];
    uint64_t v = empty;
    if (e < nc) v = pack_key_slot((ip ? -raw : raw) + 0.f, (int32_t)e);
    const uint64_t t = (uint64_t)readlane_i64((int64_t)l, M - 1);
    if (!__ballot(v < t)) continue;
    uint64_t vs[1] = {v};
    wave_sort64_packed_n<1>(vs);
    wave_merge64_packed(l, vs[0]);
  }
  const int32_t li = packed_slot(l);
  float h = 0.f;
  int32_t tag = lane;
  if (geometry) {
    const int32_t c0 = (int32_t)__builtin_amdgcn_readlane((uint32_t)li, 0);
    float qr[DPL], ar[DPL];
#pragma unroll
    for (int t = 0; t < DPL; ++t) {
      const int j = t * WAVE + lane;
      qr[t] = j < dp ? qpad[q * dp + j] : 0.f;
      ar[t] = j < dp ? c[(int64_t)c0 * dp + j] : 0.f;
    }
    h = lane == 0 ? -__builtin_inff() : __builtin_inff();
    for (int i = 1; i < M; ++i) {
      const int32_t ci = (int32_t)__builtin_amdgcn_readlane((uint32_t)li, i);
      const float* civ = c + (int64_t)ci * dp;
      // the row's loads are unconditional (clamped; lanes past dp add
      // nothing), so they are all in flight before the first product
      float bv[DPL];
#pragma unroll
      for (int t = 0; t < DPL; ++t) bv[t] = civ[min(t * WAVE + lane, dp - 1)];
      float num = 0.f, sep = 0.f;
#pragma unroll
      for (int t = 0; t < DPL; ++t) {
        const int j = t * WAVE + lane;
        const float a = ar[t], b = bv[t], x = qr[t];
        const float diff = a - b;
        const float s2 = fmaf(diff, diff, sep);
        const float n2 = ip ? fmaf(x, diff, num) : fmaf(diff, (x - a) + (x - b), num);
        sep = j < dp ? s2 : sep;
        num = j < dp ? n2 : num;
      }
      num = wave_sum_f(num);
      sep = wave_sum_f(sep);
      float hi = 0.f;
      if (sep > 0.f) hi = ip ? num / sqrtf(sep) : num / (2.0f * sqrtf(sep));
      if (lane == i) h = fmaxf(hi, 0.f);
    }
    uint64_t hv[1] = {pack_key_slot(h + 0.f, tag)};
    wave_sort64_packed_n<1>(hv);
    h = packed_key(hv[0]);
    tag = packed_slot(hv[0]);
    if (lane == 0) h = 0.f;
  }
  const int32_t id = __shfl(li, tag);
  if (lane < M) {
    cand[q * M + lane] = id;
    if (geometry) hout[q * M + lane] = h;
  }
}

void launch_candidates(const Store& st, const float* q, const float* scores, int64_t nq, int dp, int M, int aps,
                       int metric, const int32_t* mq, int32_t* sel, int32_t* cand, float* h, hipStream_t s) {
  if (nq <= 0) return;
  const int ip = metric == QUAKE_IP ? 1 : 0;
  const int dpl = (dp + WAVE - 1) / WAVE;
  if (M <= WAVE && dpl <= 16) {
    const dim3 grid((unsigned)((nq + 3) / 4));
#define QK_SEL(D)                                                                                             \
  hipLaunchKernelGGL(k_select64<D>, grid, dim3(256), 0, s, scores, nq, st.nlist, M, ip, aps, q, st.centroids, dp, \
                     cand, h)
    if (dpl <= 2) QK_SEL(2);
    else if (dpl <= 4) QK_SEL(4);
    else if (dpl <= 8) QK_SEL(8);
    else if (dpl <= 12) QK_SEL(12);
    else QK_SEL(16);
#undef QK_SEL
    return;
  }
  if (M <= 256 && st.nlist <= 256 * 64 && dp <= 1024) {
    const dim3 grid((unsigned)nq);
    const int d4 = (dp / 4 + WAVE - 1) / WAVE;
#define QK_SELL(K, D)                                                                                            \
  hipLaunchKernelGGL((k_select_large<K, D>), grid, dim3(256), 0, s, scores, st.nlist, M, ip, aps, q, st.centroids, \
                     dp, cand, h)
#define QK_SELL_D(K) \
  if (d4 <= 1) QK_SELL(K, 1); else if (d4 <= 2) QK_SELL(K, 2); else if (d4 <= 3) QK_SELL(K, 3); else QK_SELL(K, 4)
    if (st.nlist <= 256 * 8) { QK_SELL_D(8); }
    else if (st.nlist <= 256 * 16) { QK_SELL_D(16); }
    else if (st.nlist <= 256 * 32) { QK_SELL_D(32); }
    else { QK_SELL_D(64); }
#undef QK_SELL_D
#undef QK_SELL
    return;
  }
  if (aps) {
    launch_select(scores, nq, st.nlist, M, metric, sel, s);
    launch_geometry(q, st.centroids, nq, dp, M, mq, metric, sel, cand, h, s);
  } else {
    launch_select(scores, nq, st.nlist, M, metric, cand, s);
  }
}

// ---------------------------------------------------------------- k-means

// Cluster sums in fixed point: every coordinate becomes an integer multiple
// of 2^-frac_bits and the sums are integer additions, which do not depend on
// the order the atomics land in, so a build is reproducible run to run.
// frac_bits is chosen on the host so that n * max|x| * 2^frac_bits < 2^62.
__global__ __launch_bounds__(256) void k_absmax(const float* __restrict__ x, int64_t n, uint32_t* __restrict__ out) {
  uint32_t m = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const uint32_t b = __float_as_uint(x[e]) & 0x7fffffffu;
    if (b < 0x7f800000u && b > m) m = b;  // finite values only
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t v = __shfl_xor(m, o);
    m = v > m ? v : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

void launch_absmax(const float* x, int64_t n, uint32_t* out, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_absmax, dim3((unsigned)blocks), dim3(256), 0, s, x, n, out);
}

__global__ __launch_bounds__(256) void k_kmeans_accumulate(const float* __restrict__ x, int64_t n, int dp,
                                                            const int32_t* __restrict__ assign, double scale,
                                                            int64_t* __restrict__ sums, int32_t* __restrict__ counts) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t row = e / dp;
  const int j = (int)(e - row * dp);
  if (row >= n) return;
  const int a = assign[row];
  const long long v = __double2ll_rn((double)x[row * dp + j] * scale);
  atomicAdd((unsigned long long*)&sums[(int64_t)a * dp + j], (unsigned long long)v);
  if (j == 0) atomicAdd(&counts[a], 1);
}

void launch_kmeans_accumulate(const float* x, int64_t n, int dp, const int32_t* assign, int frac_bits, int64_t* sums,
                              int32_t* counts, hipStream_t s) {
  const int64_t total = n * dp;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_kmeans_accumulate, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x, n, dp, assign,
                     ldexp(1.0, frac_bits), sums, counts);
}

// Centroid = sum / count (FP64 from the exact integer sums), unit length for
// spherical k-means; empty clusters keep their centroid.
__global__ __launch_bounds__(64) void k_kmeans_update(const int64_t* __restrict__ sums,
                                                       const int32_t* __restrict__ counts, int dp, int normalise,
                                                       double unscale, float* __restrict__ c) {
  const int64_t j = blockIdx.x;
  const int lane = threadIdx.x;
  const int cnt = counts[j];
  if (cnt == 0) return;
  const double inv = unscale / (double)cnt;
  double nrm = 0.0;
  for (int t = lane; t < dp; t += WAVE) {
    const double v = (double)sums[j * dp + t] * inv;
    nrm += v * v;
  }
  nrm = wave_sum_d(nrm);
  const double scale = (normalise && nrm > 0.0) ? inv / sqrt(nrm) : inv;
  for (int t = lane; t < dp; t += WAVE) c[j * dp + t] = (float)((double)sums[j * dp + t] * scale);
}

void launch_kmeans_update(const int64_t* sums, const int32_t* counts, int64_t nc, int dp, int normalise,
                          int frac_bits, float* c, hipStream_t s) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_kmeans_update, dim3((unsigned)nc), dim3(64), 0, s, sums, counts, dp, normalise,
                     ldexp(1.0, -frac_bits), c);
}

// Rows scaled to unit length (rows of zeros stay zero).
__global__ __launch_bounds__(64) void k_normalise_rows(float* __restrict__ c, int dp) {
  const int64_t j = blockIdx.x;
  double nrm = 0.0;
  for (int t = threadIdx.x; t < dp; t += WAVE) nrm += (double)c[j * dp + t] * (double)c[j * dp + t];
  nrm = wave_sum_d(nrm);
  if (!(nrm > 0.0)) return;
  const double inv = 1.0 / sqrt(nrm);
  for (int t = threadIdx.x; t < dp; t += WAVE) c[j * dp + t] = (float)((double)c[j * dp + t] * inv);
}

void launch_normalise_rows(float* c, int64_t n, int dp, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_normalise_rows, dim3((unsigned)n), dim3(64), 0, s, c, dp);
}

__global__ __launch_bounds__(64) void k_gather_rows(const float* __restrict__ x, int d,
                                                     const int64_t* __restrict__ rows, int dp,
                                                     float* __restrict__ out) {
  const int64_t r = blockIdx.x;
  const int64_t src = rows[r];
  for (int j = threadIdx.x; j < dp; j += WAVE) out[r * dp + j] = (j < d) ? x[src * d + j] : 0.f;
}

void launch_gather_rows(const float* x, int d, const int64_t* rows, int64_t nr, int dp, float* out,
                        hipStream_t s) {
  if (nr <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)nr), dim3(64), 0, s, x, d, rows, dp, out);
}

}  // namespace qk

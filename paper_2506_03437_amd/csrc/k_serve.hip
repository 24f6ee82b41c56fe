// Slot-indexed kernels for the serving loop: queries join and leave a
// running batch at round boundaries, each in its own slot of the search
// workspace.
#include "common.hpp"
#include "index.hpp"

namespace qk {

static dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// Row i of x goes to row slots[i] of out, padded to dp; |row|^2 in FP64.
__global__ __launch_bounds__(256) void k_rows_to_slots(const float* __restrict__ x, int64_t n, int d, int dp,
                                                        const int32_t* __restrict__ slots, float* __restrict__ out,
                                                        double* __restrict__ norm2) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int64_t row = slots[i];
  double acc = 0.0;
  for (int j = lane; j < dp; j += WAVE) {
    const float v = j < d ? x[i * d + j] : 0.f;
    out[row * dp + j] = v;
    acc += (double)v * (double)v;
  }
  acc = wave_sum_d(acc);
  if (lane == 0) norm2[row] = acc;
}

void launch_rows_to_slots(const float* x, int64_t n, int d, int dp, const int32_t* slots, float* out, double* norm2,
                          hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_rows_to_slots, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, x, n, d, dp, slots, out,
                       norm2);
}

// Candidate rows computed for the admitted queries go to their slots.
__global__ __launch_bounds__(256) void k_candidates_to_slots(const int32_t* __restrict__ cand, const float* __restrict__ h,
                                                              int64_t n, int M, const int32_t* __restrict__ slots,
                                                              int32_t* __restrict__ cand_out, float* __restrict__ h_out,
                                                              int32_t* __restrict__ mq) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * M) return;
  const int64_t i = e / M;
  const int j = (int)(e - i * M);
  const int64_t row = slots[i];
  cand_out[row * M + j] = cand[e];
  h_out[row * M + j] = h ? h[e] : 0.f;
  if (j == 0) mq[row] = M;
}

void launch_candidates_to_slots(const int32_t* cand, const float* h, int64_t n, int M, const int32_t* slots,
                                int32_t* cand_out, float* h_out, int32_t* mq, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_candidates_to_slots, grid_of(n * M), dim3(256), 0, s, cand, h, n, M, slots, cand_out, h_out,
                       mq);
}

// Fresh search state in the given slots (as k_round_init does for a batch).
__global__ __launch_bounds__(256) void k_init_slots(const int32_t* __restrict__ slots, int64_t n, int kk, int w0,
                                                     int32_t* __restrict__ st_m, int32_t* __restrict__ st_w,
                                                     int32_t* __restrict__ st_done, double* __restrict__ rho,
                                                     double* __restrict__ p0, double* __restrict__ V,
                                                     double* __restrict__ vsum, double* __restrict__ r,
                                                     float* __restrict__ rk, int64_t* __restrict__ ri) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * kk) return;
  const int64_t i = e / kk;
  const int j = (int)(e - i * kk);
  const int64_t q = slots[i];
  rk[q * kk + j] = KEY_EMPTY;
  ri[q * kk + j] = -1;
  if (j == 0) {
    st_m[q] = 0; st_w[q] = w0; st_done[q] = 0;
    rho[q] = __builtin_inf(); p0[q] = 1.0; V[q] = 0.0; vsum[q] = 0.0; r[q] = 0.0;
  }
}

void launch_init_slots(Workspace& ws, const int32_t* slots, int64_t n, int kk, int w0, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_init_slots, grid_of(n * kk), dim3(256), 0, s, slots, n, kk, w0, ws.st_m, ws.st_w, ws.st_done,
                       ws.st_rho, ws.st_p0, ws.st_V, ws.st_vsum, ws.st_r, ws.rk, ws.ri);
}

__global__ __launch_bounds__(256) void k_mark_free(int32_t* __restrict__ st_done, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < n) st_done[e] = 1;
}

void launch_mark_free(Workspace& ws, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_mark_free, grid_of(n), dim3(256), 0, s, ws.st_done, n);
}

// Results of the finished slots, gathered into consecutive rows.
__global__ __launch_bounds__(256) void k_gather_results(const int32_t* __restrict__ slots, int64_t n, int k, int kk,
                                                         int ip, const float* __restrict__ rk,
                                                         const int64_t* __restrict__ ri,
                                                         const int32_t* __restrict__ st_m,
                                                         const double* __restrict__ st_r, int64_t* __restrict__ ids,
                                                         float* __restrict__ dist, int32_t* __restrict__ ns,
                                                         double* __restrict__ rec) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * k) return;
  const int64_t i = e / k;
  const int j = (int)(e - i * k);
  const int64_t q = slots[i];
  const float key = rk[q * kk + j];
  ids[e] = ri[q * kk + j];
  dist[e] = ip ? -key : key;
  if (j == 0) {
    ns[i] = st_m[q];
    rec[i] = st_r[q];
  }
}

void launch_gather_results(const Workspace& ws, const int32_t* slots, int64_t n, int k, int kk, int metric,
                           int64_t* ids, float* dist, int32_t* ns, double* rec, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_gather_results, grid_of(n * k), dim3(256), 0, s, slots, n, k, kk, metric == QUAKE_IP ? 1 : 0,
                       ws.rk, ws.ri, ws.st_m, ws.st_r, ids, dist, ns, rec);
}

}  // namespace qk

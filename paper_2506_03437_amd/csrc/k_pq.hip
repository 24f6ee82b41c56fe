// Product-quantized rows and the scan over their codes (Sec. 8, "Vector
// Compression": product quantization cuts the bytes a scan reads; the
// paper leaves the design open).
//
// The d dimensions are split into M subspaces of ds = d / M consecutive
// dimensions with 256 codewords each, one codebook [M][256][ds] for the
// whole index; a row is stored as M one-byte codes (its nearest codeword in
// each subspace, ties to the lower index) next to its other copies, so it
// keeps its code through every move.  Codes sit in tiles like the vectors:
// word g of slot (tile t, lane l) holds the codes of subspaces 4g .. 4g + 3
// (lowest byte first) at word index (t * M/4 + g) * 64 + l, so the 64 lanes
// of a wave read 256 contiguous bytes per step.
//
// A search first fills one table per query, [M][256] FP32: the squared
// distance of the query's subvector to each codeword (L2), or minus their
// inner product (IP), so that smaller is better either way.  The scan then
// scores every row by adding its M table entries in subspace order and
// keeps the best rerank_factor * k rows (store slots) per query; the
// adaptive rounds and their commit run on these scores unchanged, and once
// a search ends the kept slots are re-scored exactly from the FP32 rows.
#include "common.hpp"
#include "index.hpp"

namespace qk {

static dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// out[r][j] = x[rows[r]][col0 + j] for j < ds, 0 up to dsp (rows of x are d wide).
__global__ __launch_bounds__(256) void k_pq_subspace(const float* __restrict__ x, int64_t nr, int d,
                                                      const int64_t* __restrict__ rows, int col0, int ds, int dsp,
                                                      float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nr * dsp) return;
  const int64_t r = e / dsp;
  const int j = (int)(e - r * dsp);
  out[e] = j < ds ? x[rows[r] * d + col0 + j] : 0.f;
}

void launch_pq_subspace(const float* x, int64_t nr, int d, const int64_t* rows, int col0, int ds, int dsp, float* out,
                        hipStream_t s) {
  if (nr <= 0) return;
  hipLaunchKernelGGL(k_pq_subspace, grid_of(nr * dsp), dim3(256), 0, s, x, nr, d, rows, col0, ds, dsp, out);
}

// Codes of rows x[n][d] in subspace blockIdx.y, written at their store
// slots: block (b, m) stages subspace m's 256 codewords and the subvectors
// of rows 256 b .. 256 b + 255 in LDS; thread r tries every codeword in
// index order (squared differences summed in dimension order, FP32) and
// keeps the first nearest.
__global__ __launch_bounds__(256) void k_pq_encode(const float* __restrict__ x, int64_t n, int d,
                                                    const int64_t* __restrict__ slot, const float* __restrict__ book,
                                                    int M, int ds, uint8_t* __restrict__ codes) {
  __shared__ float cb[256 * PQ_MAX_SUB];
  __shared__ float xs[256 * (PQ_MAX_SUB + 1)];
  const int m = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const float* bm = book + (int64_t)m * 256 * ds;
  for (int e = threadIdx.x; e < 256 * ds; e += 256) cb[e] = bm[e];
  for (int e = threadIdx.x; e < 256 * ds; e += 256) {
    const int r = e / ds, t = e - r * ds;
    xs[r * (PQ_MAX_SUB + 1) + t] = r0 + r < n ? x[(r0 + r) * d + (int64_t)m * ds + t] : 0.f;
  }
  __syncthreads();
  const int64_t row = r0 + threadIdx.x;
  if (row >= n) return;
  const float* v = xs + threadIdx.x * (PQ_MAX_SUB + 1);
  float best = __builtin_inff();
  int arg = 0;
  for (int j = 0; j < 256; ++j) {
    const float* c = cb + j * ds;
    float acc = 0.f;
    for (int t = 0; t < ds; ++t) {
      const float diff = v[t] - c[t];
      acc = fmaf(diff, diff, acc);
    }
    if (acc < best) { best = acc; arg = j; }
  }
  const int64_t sl = slot[row];
  const int64_t tile = sl / TILE;
  const int lane = (int)(sl - tile * TILE);
  codes[((tile * (M >> 2) + (m >> 2)) * TILE + lane) * 4 + (m & 3)] = (uint8_t)arg;
}

void launch_pq_encode(const float* x, int64_t n, int d, const int64_t* slot, const float* book, int M, int ds,
                      uint32_t* codes, hipStream_t s) {
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)M);
  hipLaunchKernelGGL(k_pq_encode, grid, dim3(256), 0, s, x, n, d, slot, book, M, ds,
                     reinterpret_cast<uint8_t*>(codes));
}

// Tables of queries q[nq][dp]: block (query, m), thread j = codeword j.
__global__ __launch_bounds__(256) void k_pq_lut(const float* __restrict__ q, int dp, const float* __restrict__ book,
                                                 int M, int ds, int ip, float* __restrict__ lut) {
  const int64_t qi = blockIdx.x;
  const int m = blockIdx.y, j = threadIdx.x;
  const float* qs = q + qi * dp + (int64_t)m * ds;
  const float* c = book + ((int64_t)m * 256 + j) * ds;
  float acc = 0.f;
  for (int t = 0; t < ds; ++t) {
    if (ip) {
      acc = fmaf(qs[t], c[t], acc);
    } else {
      const float diff = qs[t] - c[t];
      acc = fmaf(diff, diff, acc);
    }
  }
  lut[(qi * M + m) * 256 + j] = ip ? -acc : acc;
}

void launch_pq_lut(const float* q, int64_t nq, int dp, const float* book, int M, int ds, int metric, float* lut,
                   hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_pq_lut, dim3((unsigned)nq, (unsigned)M), dim3(256), 0, s, q, dp, book, M, ds,
                     metric == QUAKE_IP ? 1 : 0, lut);
}

// One work item (query, partition, tiles [t0, t1)): lane l scores slot
// (tile, l) from its codes, and the wave keeps the item's best kk (score,
// slot) pairs, seeded with the query's committed kk-th.  Deleted slots (id
// -1) and rows failing the query's label mask are skipped.
template <int KPL>
__device__ __forceinline__ void pq_item(const int4 item, int64_t it, int lane, const float* __restrict__ lut, int M,
                                        const uint32_t* __restrict__ codes, const int64_t* __restrict__ sid,
                                        const int64_t* __restrict__ poff, const int32_t* __restrict__ psize,
                                        const float* __restrict__ rk, const int64_t* __restrict__ ri, int kk,
                                        float* __restrict__ pk, int64_t* __restrict__ pi,
                                        const uint32_t* __restrict__ attr, const uint32_t* __restrict__ qmask) {
  const int q = __builtin_amdgcn_readfirstlane(item.x);
  const int p = __builtin_amdgcn_readfirstlane(item.y);
  const int t0 = __builtin_amdgcn_readfirstlane(item.z);
  const int t1 = __builtin_amdgcn_readfirstlane(item.w);
  const float seed_k = rk[(int64_t)q * kk + kk - 1];
  const int64_t seed_i = ri[(int64_t)q * kk + kk - 1];
  const uint32_t qm = qmask ? qmask[q] : 0u;
  WaveTopK<KPL> top;
  top.init(kk, seed_k, seed_i);
  const int64_t tile0 = poff[p];
  const int size = psize[p];
  const int mw = M >> 2;
  const float* tq = lut + (int64_t)q * M * 256;
  for (int t = t0; t < t1; ++t) {
    const int64_t slot = (tile0 + t) * TILE + lane;
    const uint32_t* cw = codes + (tile0 + t) * (int64_t)mw * TILE + lane;
    float key = 0.f;
    for (int g = 0; g < mw; ++g) {
      const uint32_t w = cw[(int64_t)g * TILE];
      const float* tg = tq + g * 1024;
      key += tg[w & 255u];
      key += tg[256 + ((w >> 8) & 255u)];
      key += tg[512 + ((w >> 16) & 255u)];
      key += tg[768 + (w >> 24)];
    }
    const bool valid = (t * TILE + lane) < size;
    bool pass = false;
    if (valid && !(key > top.tk)) {
      const int64_t id = sid[slot];
      pass = id >= 0 && (!qmask || (attr[slot] & qm) != 0u) && kv_less(key, slot, top.tk, top.ti);
    }
    uint64_t mask = __ballot(pass);
    while (mask) {
      const int src = __builtin_ctzll(mask);
      mask &= mask - 1;
      const float ck = readlane_f(key, src);
      const int64_t cs = readlane_i64(slot, src);
      if (kv_less(ck, cs, top.tk, top.ti)) top.insert(ck, cs);
    }
  }
  top.store(pk + it * kk, pi + it * kk);
}

// Waves take items from the round's queue (head counters[7], reset by
// k_prefix) until it is empty, as the plain FP32 scan does.
template <int KPL>
__global__ __launch_bounds__(256) void k_scan_pq(const int4* __restrict__ items, int64_t* __restrict__ counters,
                                                  const float* __restrict__ lut, int M,
                                                  const uint32_t* __restrict__ codes,
                                                  const int64_t* __restrict__ sid, const int64_t* __restrict__ poff,
                                                  const int32_t* __restrict__ psize, const float* __restrict__ rk,
                                                  const int64_t* __restrict__ ri, int kk, float* __restrict__ pk,
                                                  int64_t* __restrict__ pi, const uint32_t* __restrict__ attr,
                                                  const uint32_t* __restrict__ qmask) {
  const int lane = threadIdx.x & 63;
  const int64_t nitems = counters[0];
  for (;;) {
    int64_t it = 0;
    if (lane == 0) it = (int64_t)atomicAdd((unsigned long long*)(counters + 7), 1ull);
    it = readlane_i64(it, 0);
    if (it >= nitems) break;
    pq_item<KPL>(items[it], it, lane, lut, M, codes, sid, poff, psize, rk, ri, kk, pk, pi, attr, qmask);
  }
}

void launch_scan_pq(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  if (a.items_cap <= 0) return;
  const int64_t need = (a.items_cap + 3) / 4;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(need, a.blocks)));
  // kk <= 64 (the final rerank sorts a query's candidates within one wave)
  hipLaunchKernelGGL((k_scan_pq<1>), grid, dim3(256), 0, s, ws.items, ws.total, ws.lut, st.pq_m, st.codes, st.ids,
                     st.d_off, st.d_size, ws.rk, ws.ri, a.kk, ws.pk, ws.pi, a.attr, a.qmask);
}

// out[i][m] = code of subspace m at slots[i].
__global__ __launch_bounds__(256) void k_pq_export(const uint8_t* __restrict__ codes, const int64_t* __restrict__ slots,
                                                    int64_t n, int M, uint8_t* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n * M) return;
  const int64_t i = e / M;
  const int m = (int)(e - i * M);
  const int64_t sl = slots[i];
  const int64_t tile = sl / TILE;
  const int lane = (int)(sl - tile * TILE);
  out[e] = codes[((tile * (M >> 2) + (m >> 2)) * TILE + lane) * 4 + (m & 3)];
}

void launch_pq_export(const Store& st, const int64_t* slots, int64_t n, uint8_t* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pq_export, grid_of(n * st.pq_m), dim3(256), 0, s, reinterpret_cast<const uint8_t*>(st.codes),
                     slots, n, st.pq_m, out);
}

}  // namespace qk

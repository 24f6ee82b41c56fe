// Product-quantized rows and the scan over their codes (Sec. 8, "Vector
// Compression": product quantization cuts the bytes a scan reads; the
// paper leaves the design open).
//
// The d dimensions are split into M subspaces of ds = d / M consecutive
// dimensions with 256 codewords each, one codebook [M][256][ds] for the
// whole index.  A row's residual r = x - c to its partition's centroid c is
// stored as M one-byte codes (its nearest codeword in each subspace, ties to
// the lower index); the row decodes to c + r^ (IVFADC, Jegou, Douze and
// Schmid, IEEE TPAMI 33(1), 2011).  A row is encoded when it enters the
// store and again when its partition or centroid changes (maintenance);
// moves inside a partition carry the codes.  Codes sit in tiles like the
// vectors, CW = M/4 + 1 words per slot: word g < M/4 of slot (tile t, lane
// l) holds the codes of subspaces 4g .. 4g + 3 (lowest byte first) at word
// index (t * CW + g) * 64 + l, so the 64 lanes of a wave read 256
// contiguous bytes per step; word M/4 holds e = |r^|^2 + 2 <c, r^>, FP32.
//
// Squared L2: |q - c - r^|^2 = |q - c|^2 + e - 2 <q, r^>, and <q, r^> is a
// sum of per-subspace inner products of the query with codewords.  A search
// fills one table per query, [M][256] FP32: -2 <q_m, codeword> (L2) or
// -<q_m, codeword> (IP).  A work item (query, partition) computes its
// centroid term |q - c|^2 (L2) or -<q, c> (IP) once; a row's score, smaller
// is better, is that term, plus e (L2), plus its M table entries in
// subspace order.  The scan keeps the best rerank_factor * k rows (store
// slots) per query; the adaptive rounds and their commit run on these
// scores unchanged, and once a search ends the kept slots are re-scored
// exactly from the FP32 rows.
#include "common.hpp"
#include "index.hpp"

namespace qk {

static dim3 grid_of(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// Residual subvectors of sampled rows: out[r][j] = x[i][col0 + j] -
// C[part[i]][col0 + j] with i = rows[r], for j < ds, 0 up to dsp (rows of x
// are d wide, centroids dp wide).
__global__ __launch_bounds__(256) void k_pq_subspace(const float* __restrict__ x, int64_t nr, int d,
                                                      const int64_t* __restrict__ rows,
                                                      const int32_t* __restrict__ part, const float* __restrict__ C,
                                                      int dp, int col0, int ds, int dsp, float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nr * dsp) return;
  const int64_t r = e / dsp;
  const int j = (int)(e - r * dsp);
  const int64_t i = rows[r];
  out[e] = j < ds ? x[i * d + col0 + j] - C[(int64_t)part[i] * dp + col0 + j] : 0.f;
}

void launch_pq_subspace(const float* x, int64_t nr, int d, const int64_t* rows, const int32_t* part, const float* C,
                        int dp, int col0, int ds, int dsp, float* out, hipStream_t s) {
  if (nr <= 0) return;
  hipLaunchKernelGGL(k_pq_subspace, grid_of(nr * dsp), dim3(256), 0, s, x, nr, d, rows, part, C, dp, col0, ds, dsp,
                     out);
}

// Codes of the rows at store slots slot[i] (partition part[i]) in subspace
// blockIdx.y: block (b, m) stages subspace m's 256 codewords and the
// residual subvectors (row-major FP32 copy minus centroid) of rows
// 256 b .. 256 b + 255 in LDS; thread r tries every codeword in index order
// (squared differences summed in dimension order, FP32) and keeps the first
// nearest.
__global__ __launch_bounds__(256) void k_pq_encode(const float* __restrict__ rows32, int dp,
                                                    const int64_t* __restrict__ slot, const int32_t* __restrict__ part,
                                                    int64_t n, const float* __restrict__ C,
                                                    const float* __restrict__ book, int M, int ds, int cw,
                                                    uint8_t* __restrict__ codes) {
  __shared__ float cb[256 * PQ_MAX_SUB];
  __shared__ float xs[256 * (PQ_MAX_SUB + 1)];
  const int m = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const float* bm = book + (int64_t)m * 256 * ds;
  for (int e = threadIdx.x; e < 256 * ds; e += 256) cb[e] = bm[e];
  for (int e = threadIdx.x; e < 256 * ds; e += 256) {
    const int r = e / ds, t = e - r * ds;
    float v = 0.f;
    if (r0 + r < n) {
      const int64_t col = (int64_t)m * ds + t;
      v = rows32[slot[r0 + r] * dp + col] - C[(int64_t)part[r0 + r] * dp + col];
    }
    xs[r * (PQ_MAX_SUB + 1) + t] = v;
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
  codes[((tile * cw + (m >> 2)) * TILE + lane) * 4 + (m & 3)] = (uint8_t)arg;
}

// e = |r^|^2 + 2 <c, r^> of each slot's decoded residual r^ (subspaces and
// their dimensions in order), into the slot's last code word (0 for IP,
// which does not use it).
__global__ __launch_bounds__(256) void k_pq_norms(uint32_t* __restrict__ codes, const int64_t* __restrict__ slot,
                                                   const int32_t* __restrict__ part, int64_t n,
                                                   const float* __restrict__ C, int dp,
                                                   const float* __restrict__ book, int M, int ds, int cw, int ip) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t sl = slot[i];
  const int64_t tile = sl / TILE;
  const int lane = (int)(sl - tile * TILE);
  const float* c = C + (int64_t)part[i] * dp;
  float e = 0.f;
  if (!ip) {
    for (int m = 0; m < M; ++m) {
      const uint32_t w = codes[(tile * cw + (m >> 2)) * TILE + lane];
      const int code = (int)((w >> (8 * (m & 3))) & 255u);
      const float* v = book + ((int64_t)m * 256 + code) * ds;
      for (int t = 0; t < ds; ++t) e = fmaf(v[t], fmaf(2.f, c[m * ds + t], v[t]), e);
    }
  }
  codes[(tile * cw + (M >> 2)) * TILE + lane] = __float_as_uint(e);
}

void launch_pq_encode(const float* rows32, int dp, const int64_t* slot, const int32_t* part, int64_t n,
                      const float* C, const float* book, int M, int ds, int metric, uint32_t* codes, hipStream_t s) {
  if (n <= 0) return;
  const int cw = pq_words(M);
  const dim3 grid((unsigned)((n + 255) / 256), (unsigned)M);
  hipLaunchKernelGGL(k_pq_encode, grid, dim3(256), 0, s, rows32, dp, slot, part, n, C, book, M, ds, cw,
                     reinterpret_cast<uint8_t*>(codes));
  hipLaunchKernelGGL(k_pq_norms, grid_of(n), dim3(256), 0, s, codes, slot, part, n, C, dp, book, M, ds, cw,
                     metric == QUAKE_IP ? 1 : 0);
}

// Tables of queries q[nq][dp]: block (query, m), thread j = codeword j:
// -2 <q_m, codeword> (L2) or -<q_m, codeword> (IP).
__global__ __launch_bounds__(256) void k_pq_lut(const float* __restrict__ q, int dp, const float* __restrict__ book,
                                                 int M, int ds, int ip, float* __restrict__ lut) {
  const int64_t qi = blockIdx.x;
  const int m = blockIdx.y, j = threadIdx.x;
  const float* qs = q + qi * dp + (int64_t)m * ds;
  const float* c = book + ((int64_t)m * 256 + j) * ds;
  float acc = 0.f;
  for (int t = 0; t < ds; ++t) acc = fmaf(qs[t], c[t], acc);
  lut[(qi * M + m) * 256 + j] = ip ? -acc : -2.f * acc;
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
                                        const float* __restrict__ qpad, const float* __restrict__ C, int dp, int ip,
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
  const int mw = M >> 2, cwn = mw + 1;
  const float* tq = lut + (int64_t)q * M * 256;
  // the item's centroid term: lane l sums dimensions l, l + 64, ... in
  // order, then the wave adds the 64 partial sums pairwise
  float base = 0.f;
  {
    const float* qv = qpad + (int64_t)q * dp;
    const float* cv = C + (int64_t)p * dp;
    for (int j = lane; j < dp; j += WAVE) {
      const float a = qv[j], b = cv[j];
      base = ip ? fmaf(a, b, base) : fmaf(a - b, a - b, base);
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) base += __shfl_xor(base, o);
    if (ip) base = -base;
  }
  for (int t = t0; t < t1; ++t) {
    const int64_t slot = (tile0 + t) * TILE + lane;
    const uint32_t* cw = codes + (tile0 + t) * (int64_t)cwn * TILE + lane;
    float key = base;
    if (!ip) key += __uint_as_float(cw[(int64_t)mw * TILE]);
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
                                                  const float* __restrict__ qpad, const float* __restrict__ C, int dp,
                                                  int ip, const uint32_t* __restrict__ codes,
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
    pq_item<KPL>(items[it], it, lane, lut, M, qpad, C, dp, ip, codes, sid, poff, psize, rk, ri, kk, pk, pi, attr,
                 qmask);
  }
}

void launch_scan_pq(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  if (a.items_cap <= 0) return;
  const int64_t need = (a.items_cap + 3) / 4;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(need, a.blocks)));
  // kk <= 64 (the final rerank sorts a query's candidates within one wave)
  hipLaunchKernelGGL((k_scan_pq<1>), grid, dim3(256), 0, s, ws.items, ws.total, ws.lut, st.pq_m, ws.q, st.centroids,
                     st.dp, a.metric == QUAKE_IP ? 1 : 0, st.codes, st.ids, st.d_off, st.d_size, ws.rk, ws.ri, a.kk,
                     ws.pk, ws.pi, a.attr, a.qmask);
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
  out[e] = codes[((tile * ((M >> 2) + 1) + (m >> 2)) * TILE + lane) * 4 + (m & 3)];
}

void launch_pq_export(const Store& st, const int64_t* slots, int64_t n, uint8_t* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_pq_export, grid_of(n * st.pq_m), dim3(256), 0, s, reinterpret_cast<const uint8_t*>(st.codes),
                     slots, n, st.pq_m, out);
}

}  // namespace qk

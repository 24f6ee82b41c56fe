// Scan rounds of a batched search.
//
// A search runs in rounds.  In each round every unfinished query names a
// window of its next candidate partitions; the windows are cut into work
// items of at most `chunk_tiles` store tiles; one wave scans one item and
// keeps the item's best results; then one wave per query commits the items
// in candidate order.  Committing follows Algorithm "Adaptive Partition
// Scanning" (Sec. 5.1) one partition at a time: merge that partition's
// results into the query's top-k, take rho from the k-th result, recompute
// the recall model when rho moved by more than tau_rho, and stop once the
// estimated recall reaches the target.  Partitions scanned past the stop
// point are discarded, so the result is the one of the sequential algorithm;
// scanning ahead only trades extra reads for fewer rounds.  With a fixed
// nprobe the window is the whole candidate list and one round suffices.
//
// Recall model (Sec. 5, Eqs. aps-pi, aps-p0, aps-pi-final): with t_i =
// h_i / rho, v_i is the volume share of the ball B(q, rho) beyond the
// bisector of c_0 and c_i (looked up in the 1,024-point table of Sec. 5.1, "Performance Optimizations"
// with linear interpolation, 0 for t >= 1); p_0 = prod (1 - v_i) uses the raw
// shares and the remaining 1 - p_0 is split in proportion to v_i, so the
// estimate after scanning c_0 and the next m - 1 candidates is
//   r = p_0 + (1 - p_0) * (v_1 + ... + v_{m-1}) / (v_1 + ... + v_{M-1}).
// Until k results exist rho = +inf (all t = 0) and r is held at 0.  The
// model is evaluated in FP64; it is the only FP64 on the device.
//
// Estimator variants (Sec. 5.1, Table tab:recall_overhead): APS recomputes
// when rho moved by more than tau_rho, from the table; APS-R recomputes after
// every partition, from the table; APS-RP recomputes after every partition
// and evaluates each share directly from the incomplete beta function.  The
// window prediction (speculation, not a decision) always reads the table.
#include "common.hpp"
#include "index.hpp"

namespace qk {

__device__ __forceinline__ int item_chunks(int32_t size, int chunk_tiles) {
  const int tiles = (size + TILE - 1) / TILE;
  const int c = (tiles + chunk_tiles - 1) / chunk_tiles;
  return c > 0 ? c : 1;
}

// ---------------------------------------------------------------- state

__global__ __launch_bounds__(256) void k_round_init(int64_t nq, int kk, int w0, int32_t* __restrict__ st_m,
                                                     int32_t* __restrict__ st_w, int32_t* __restrict__ st_done,
                                                     double* __restrict__ rho, double* __restrict__ p0,
                                                     double* __restrict__ V, double* __restrict__ vsum,
                                                     double* __restrict__ r, float* __restrict__ rk,
                                                     int64_t* __restrict__ ri) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < nq) {
    st_m[e] = 0; st_w[e] = w0; st_done[e] = 0;
    rho[e] = __builtin_inf(); p0[e] = 1.0; V[e] = 0.0; vsum[e] = 0.0; r[e] = 0.0;
  }
  if (e < nq * kk) { rk[e] = KEY_EMPTY; ri[e] = -1; }
}

void launch_round_init(Workspace& ws, const RoundArgs& a, int w0, hipStream_t s) {
  const int64_t n = a.nq * a.kk;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_round_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.nq, a.kk, w0, ws.st_m,
                     ws.st_w, ws.st_done, ws.st_rho, ws.st_p0, ws.st_V, ws.st_vsum, ws.st_r, ws.rk, ws.ri);
}

// ---------------------------------------------------------------- planning

// Planning a round, in three steps that scale with the batch:
//  k_demand  per query: the work items and vectors of its window this round
//            (st_w is the window it asked for; st_weff what it gets) and, per
//            block of 256 queries, exclusive prefix sums of items and window
//            partitions (kept in st_item / st_pair) and the block's totals;
//  k_prefix  one block: prefix sums over the block totals, and the cut -
//            queries from the first one whose items would overflow the item
//            buffer sit this round out (effective window 0, the requested
//            window is kept for the next round); the buffer always holds the
//            first unfinished query's window, so every round makes progress;
//  k_place   per query: global item and pair offsets, windows past the cut
//            cleared.
constexpr int PLAN_BLOCK = 256;

__device__ __forceinline__ int64_t wave_excl_scan_i64(int64_t v, int64_t& wave_total) {
  const int lane = lane_id();
  int64_t x = v;
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t u = shfl_up_i64(x, o);
    if (lane >= o) x += u;
  }
  wave_total = readlane_i64(x, WAVE - 1);
  return x - v;
}

__global__ __launch_bounds__(PLAN_BLOCK) void k_demand(int64_t nq, int M, int chunk_tiles,
                                                        const int32_t* __restrict__ mq,
                                                        const int32_t* __restrict__ cand,
                                                        const int32_t* __restrict__ psize,
                                                        const int32_t* __restrict__ st_m,
                                                        const int32_t* __restrict__ st_w,
                                                        int32_t* __restrict__ st_weff,
                                                        const int32_t* __restrict__ st_done,
                                                        const uint8_t* __restrict__ slot_tag, int tag,
                                                        int64_t* __restrict__ demand, int64_t* __restrict__ vecs,
                                                        int64_t* __restrict__ loc_item, int64_t* __restrict__ loc_pair,
                                                        int64_t* __restrict__ blk) {
  __shared__ int64_t wd[PLAN_BLOCK / WAVE], ww[PLAN_BLOCK / WAVE], wv[PLAN_BLOCK / WAVE];
  const int64_t q = (int64_t)blockIdx.x * PLAN_BLOCK + threadIdx.x;
  const int wave = threadIdx.x / WAVE;
  int64_t dmd = 0, nv = 0;
  int w = 0;
  // with slot tags, only the queries of this round's store get a window
  if (q < nq && !st_done[q] && (slot_tag == nullptr || slot_tag[q] == tag)) {
    const int m = st_m[q];
    w = st_w[q];
    if (w > mq[q] - m) w = mq[q] - m;
    // eight slots at a time: their candidate loads, then their size loads,
    // are in flight together
    for (int j0 = 0; j0 < w; j0 += 8) {
      int32_t c8[8], s8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) c8[u] = cand[q * M + m + min(j0 + u, w - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u) s8[u] = psize[c8[u]];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < w) {
          dmd += item_chunks(s8[u], chunk_tiles);
          nv += s8[u];
        }
    }
  }
  int64_t td, tw, tv;
  const int64_t ed = wave_excl_scan_i64(dmd, td);
  const int64_t ew = wave_excl_scan_i64((int64_t)w, tw);
  wave_excl_scan_i64(nv, tv);
  if (lane_id() == 0) { wd[wave] = td; ww[wave] = tw; wv[wave] = tv; }
  __syncthreads();
  int64_t bd = 0, bw = 0, bv = 0, od = 0, ow = 0;
  for (int i = 0; i < PLAN_BLOCK / WAVE; ++i) {
    if (i == wave) { od = bd; ow = bw; }
    bd += wd[i]; bw += ww[i]; bv += wv[i];
  }
  if (q < nq) {
    st_weff[q] = w;
    demand[q] = dmd;
    vecs[q] = nv;
    loc_item[q] = od + ed;
    loc_pair[q] = ow + ew;
  }
  if (threadIdx.x == 0) {
    blk[blockIdx.x * 4 + 0] = bd;
    blk[blockIdx.x * 4 + 1] = bv;
    blk[blockIdx.x * 4 + 2] = bw;
  }
}

__global__ __launch_bounds__(1024) void k_prefix(int64_t nq, int64_t cap, const int64_t* __restrict__ demand,
                                                  const int64_t* __restrict__ vecs,
                                                  const int64_t* __restrict__ loc_item,
                                                  const int64_t* __restrict__ loc_pair, int64_t* __restrict__ blk,
                                                  int64_t* __restrict__ total) {
  __shared__ int64_t pd[1024], pw[1024], pv[1024];
  __shared__ unsigned long long cut_blk, cut_q, nv_tail;
  const int t = threadIdx.x;
  const int64_t nb = (nq + PLAN_BLOCK - 1) / PLAN_BLOCK;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t lo = t * per;
  const int64_t hi = (lo + per < nb) ? lo + per : nb;
  int64_t sd = 0, sw = 0, sv = 0;
  for (int64_t b = lo; b < hi; ++b) { sd += blk[b * 4]; sv += blk[b * 4 + 1]; sw += blk[b * 4 + 2]; }
  pd[t] = sd; pw[t] = sw; pv[t] = sv;
  if (t == 0) { cut_blk = (unsigned long long)nb; cut_q = (unsigned long long)nq; nv_tail = 0; }
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t a = (t >= o) ? pd[t - o] : 0;
    const int64_t c = (t >= o) ? pw[t - o] : 0;
    const int64_t e = (t >= o) ? pv[t - o] : 0;
    __syncthreads();
    pd[t] += a; pw[t] += c; pv[t] += e;
    __syncthreads();
  }
  // the block totals become block offsets: items before the block in column
  // 0, vectors in 1, window partitions (pairs) in 2
  int64_t rd = pd[t] - sd, rw = pw[t] - sw, rv = pv[t] - sv;
  for (int64_t b = lo; b < hi; ++b) {
    const int64_t d = blk[b * 4], v = blk[b * 4 + 1], w = blk[b * 4 + 2];
    if (rd + d > cap) atomicMin(&cut_blk, (unsigned long long)b);
    blk[b * 4] = rd; blk[b * 4 + 1] = rv; blk[b * 4 + 2] = rw;
    rd += d; rv += v; rw += w;
  }
  __syncthreads();
  const int64_t cb = (int64_t)cut_blk;
  if (cb < nb && t < PLAN_BLOCK) {
    const int64_t q = cb * PLAN_BLOCK + t;
    if (q < nq && blk[cb * 4] + loc_item[q] + demand[q] > cap) atomicMin(&cut_q, (unsigned long long)q);
  }
  __syncthreads();
  const int64_t cut = (int64_t)cut_q;
  if (cb < nb && t < PLAN_BLOCK) {
    const int64_t q = cb * PLAN_BLOCK + t;
    if (q < cut && q < nq) atomicAdd(&nv_tail, (unsigned long long)vecs[q]);
  }
  __syncthreads();
  if (t == 0) {
    int64_t items, nvec, pairs;
    if (cut < nq) {
      items = blk[cb * 4] + loc_item[cut];
      nvec = blk[cb * 4 + 1] + (int64_t)nv_tail;
      pairs = blk[cb * 4 + 2] + loc_pair[cut];
    } else {
      items = pd[1023];
      nvec = pv[1023];
      pairs = pw[1023];
    }
    total[0] = items;
    total[1] = nvec;
    total[2] = pairs;
    total[6] += nvec;
    total[7] = 0;    // head of the plain scan's item queue
    total[8] = cut;  // first query that sits this round out
  }
}

__global__ __launch_bounds__(PLAN_BLOCK) void k_place(int64_t nq, const int64_t* __restrict__ blk,
                                                       const int64_t* __restrict__ total,
                                                       int64_t* __restrict__ st_item, int64_t* __restrict__ st_pair,
                                                       int32_t* __restrict__ st_weff) {
  const int64_t q = (int64_t)blockIdx.x * PLAN_BLOCK + threadIdx.x;
  if (q >= nq) return;
  const int64_t b = blockIdx.x;
  st_item[q] += blk[b * 4];
  st_pair[q] += blk[b * 4 + 2];
  if (q >= total[8]) st_weff[q] = 0;
}

void launch_demand(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  if (a.nq <= 0) return;
  const unsigned nb = (unsigned)((a.nq + PLAN_BLOCK - 1) / PLAN_BLOCK);
  hipLaunchKernelGGL(k_demand, dim3(nb), dim3(PLAN_BLOCK), 0, s, a.nq, a.M, a.chunk_tiles, ws.mq, ws.cand, st.d_size,
                     ws.st_m, ws.st_w, ws.st_weff, ws.st_done, a.slot_tag, a.tag, ws.st_demand, ws.st_vecs,
                     ws.st_item, ws.st_pair, ws.blk);
  hipLaunchKernelGGL(k_prefix, dim3(1), dim3(1024), 0, s, a.nq, a.items_cap, ws.st_demand, ws.st_vecs, ws.st_item,
                     ws.st_pair, ws.blk, ws.total);
  hipLaunchKernelGGL(k_place, dim3(nb), dim3(PLAN_BLOCK), 0, s, a.nq, ws.blk, ws.total, ws.st_item, ws.st_pair,
                     ws.st_weff);
}

// Write the work items of each query's window, in candidate order.
__global__ __launch_bounds__(256) void k_emit(int64_t nq, int M, int chunk_tiles, const int32_t* __restrict__ cand,
                                               const int32_t* __restrict__ psize, const int32_t* __restrict__ st_m,
                                               const int32_t* __restrict__ st_w, const int64_t* __restrict__ first,
                                               int4* __restrict__ items) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= nq) return;
  const int w = st_w[q];
  if (w == 0) return;
  const int m = st_m[q];
  int64_t pos = first[q];
  for (int j = 0; j < w; ++j) {
    const int p = cand[q * M + m + j];
    const int size = psize[p];
    const int tiles = (size + TILE - 1) / TILE;
    const int nch = item_chunks(size, chunk_tiles);
    for (int c = lane; c < nch; c += WAVE) {
      const int t0 = c * chunk_tiles;
      const int t1 = (t0 + chunk_tiles < tiles) ? t0 + chunk_tiles : tiles;
      items[pos + c] = make_int4((int)q, p, t0, t1);
    }
    pos += nch;
  }
}

void launch_emit(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_emit, dim3((unsigned)((a.nq + 3) / 4)), dim3(256), 0, s, a.nq, a.M, a.chunk_tiles, ws.cand,
                     st.d_size, ws.st_m, ws.st_weff, ws.st_item, ws.items);
}

// ---------------------------------------------------------------- FP32 scan

// One work item (query, partition, tiles [t0, t1)) of the plain scan: the
// item's partial list, seeded with the query's committed k-th result.  With
// qmask (a filtered search) a row is a result only when its label bits share
// a bit with the query's mask.
template <int METRIC, int KPL>
__device__ __forceinline__ void scan_item(const int4 item, int64_t it, int lane, const float* __restrict__ qpad,
                                          int dp, const float* __restrict__ v32, const int64_t* __restrict__ sid,
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
  const int nch4 = dp >> 2;
  const_float4* qs = (const_float4*)(qpad + (int64_t)q * dp);
  for (int t = t0; t < t1; ++t) {
    const int64_t slot = (tile0 + t) * TILE + lane;
    const float4* xp = reinterpret_cast<const float4*>(v32) + (tile0 + t) * (int64_t)nch4 * WAVE + lane;
    const float key = tile_distance<METRIC>(xp, qs, nch4);
    const bool valid = (t * TILE + lane) < size;
    bool pass = false;
    int64_t myid = -1;
    if (valid && !(key > top.tk)) {
      myid = sid[slot];
      pass = myid >= 0 && (!qmask || (attr[slot] & qm) != 0u) && kv_less(key, myid, top.tk, top.ti);
    }
    uint64_t mask = __ballot(pass);
    while (mask) {
      const int src = __builtin_ctzll(mask);
      mask &= mask - 1;
      const float ck = readlane_f(key, src);
      const int64_t ci = readlane_i64(myid, src);
      if (kv_less(ck, ci, top.tk, top.ti)) top.insert(ck, ci);
    }
  }
  top.store(pk + it * kk, pi + it * kk);
}

template <int METRIC, int KPL>
__global__ __launch_bounds__(256) void k_scan_f32(const int4* __restrict__ items, int64_t* __restrict__ counters,
                                                   const float* __restrict__ qpad, int dp,
                                                   const float* __restrict__ v32, const int64_t* __restrict__ sid,
                                                   const int64_t* __restrict__ poff,
                                                   const int32_t* __restrict__ psize,
                                                   const float* __restrict__ rk, const int64_t* __restrict__ ri,
                                                   int kk, float* __restrict__ pk, int64_t* __restrict__ pi,
                                                   const uint32_t* __restrict__ attr,
                                                   const uint32_t* __restrict__ qmask) {
  // Waves take items from the round's queue (head counters[7], reset by
  // k_prefix) until it is empty: items differ in size, so the grid balances
  // itself.
  const int lane = threadIdx.x & 63;
  const int64_t nitems = counters[0];
  for (;;) {
    int64_t it = 0;
    if (lane == 0) it = (int64_t)atomicAdd((unsigned long long*)(counters + 7), 1ull);
    it = readlane_i64(it, 0);
    if (it >= nitems) break;
    scan_item<METRIC, KPL>(items[it], it, lane, qpad, dp, v32, sid, poff, psize, rk, ri, kk, pk, pi, attr, qmask);
  }
}

template <int METRIC>
static void scan_f32_k(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  const int64_t need = (a.items_cap + 3) / 4;
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(need, a.blocks)));
  if (a.kk <= 64)
    hipLaunchKernelGGL((k_scan_f32<METRIC, 1>), grid, dim3(256), 0, s, ws.items, ws.total, ws.q, st.dp, st.v32,
                       st.ids, st.d_off, st.d_size, ws.rk, ws.ri, a.kk, ws.pk, ws.pi, a.attr, a.qmask);
  else if (a.kk <= 128)
    hipLaunchKernelGGL((k_scan_f32<METRIC, 2>), grid, dim3(256), 0, s, ws.items, ws.total, ws.q, st.dp, st.v32,
                       st.ids, st.d_off, st.d_size, ws.rk, ws.ri, a.kk, ws.pk, ws.pi, a.attr, a.qmask);
  else
    hipLaunchKernelGGL((k_scan_f32<METRIC, 4>), grid, dim3(256), 0, s, ws.items, ws.total, ws.q, st.dp, st.v32,
                       st.ids, st.d_off, st.d_size, ws.rk, ws.ri, a.kk, ws.pk, ws.pi, a.attr, a.qmask);
}

// Items whose result lists are longer than a wave's sorted list holds (the
// upper level of a two-level index keeps hundreds of centroids per query):
// one block scores all vectors of the item (at most 16 tiles), then sorts
// them by (key, id) in LDS and keeps the first kk.
template <int METRIC>
__device__ __forceinline__ void sorted_item(const int4 item, int64_t it, float* K, int64_t* I,
                                            const float* __restrict__ qpad, int dp, const float* __restrict__ v32,
                                            const int64_t* __restrict__ sid, const int64_t* __restrict__ poff,
                                            const int32_t* __restrict__ psize, int kk, float* __restrict__ pk,
                                            int64_t* __restrict__ pi) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = item.x, p = item.y, t0 = item.z, t1 = item.w;
  const int64_t tile0 = poff[p];
  const int size = psize[p];
  const int nch4 = dp >> 2;
  const_float4* qs = (const_float4*)(qpad + (int64_t)q * dp);
  for (int e = threadIdx.x; e < SORTED_ITEM_MAX; e += 256) { K[e] = KEY_EMPTY; I[e] = -1; }
  __syncthreads();
  for (int t = t0 + wave; t < t1; t += 4) {
    const int64_t slot = (tile0 + t) * TILE + lane;
    const float4* xp = reinterpret_cast<const float4*>(v32) + (tile0 + t) * (int64_t)nch4 * WAVE + lane;
    const float key = tile_distance<METRIC>(xp, qs, nch4);
    const int e = (t - t0) * TILE + lane;
    if (e < SORTED_ITEM_MAX && t * TILE + lane < size) {
      const int64_t id = sid[slot];
      if (id >= 0) { K[e] = key; I[e] = id; }
    }
  }
  __syncthreads();
  for (int sz = 2; sz <= SORTED_ITEM_MAX; sz <<= 1) {
    for (int stride = sz >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < SORTED_ITEM_MAX / 2; i += 256) {
        const int lo = 2 * i - (i & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & sz) == 0;
        const bool swap = up ? kv_less(K[hi], I[hi], K[lo], I[lo]) : kv_less(K[lo], I[lo], K[hi], I[hi]);
        if (swap) {
          const float tk = K[lo]; K[lo] = K[hi]; K[hi] = tk;
          const int64_t ti = I[lo]; I[lo] = I[hi]; I[hi] = ti;
        }
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < kk; e += 256) {
    pk[it * kk + e] = e < SORTED_ITEM_MAX ? K[e] : KEY_EMPTY;
    pi[it * kk + e] = e < SORTED_ITEM_MAX ? I[e] : -1;
  }
}

template <int METRIC>
__global__ __launch_bounds__(256) void k_scan_f32_sorted(const int4* __restrict__ items,
                                                          int64_t* __restrict__ counters,
                                                          const float* __restrict__ qpad, int dp,
                                                          const float* __restrict__ v32, const int64_t* __restrict__ sid,
                                                          const int64_t* __restrict__ poff,
                                                          const int32_t* __restrict__ psize, int kk,
                                                          float* __restrict__ pk, int64_t* __restrict__ pi) {
  __shared__ float K[SORTED_ITEM_MAX];
  __shared__ int64_t I[SORTED_ITEM_MAX];
  __shared__ int64_t next;
  const int64_t nitems = counters[0];
  for (;;) {
    __syncthreads();  // the previous item's results are out of K / I, and `next` is free
    if (threadIdx.x == 0) next = (int64_t)atomicAdd((unsigned long long*)(counters + 7), 1ull);
    __syncthreads();
    const int64_t it = next;
    if (it >= nitems) break;
    sorted_item<METRIC>(items[it], it, K, I, qpad, dp, v32, sid, poff, psize, kk, pk, pi);
  }
}

// Persistent launch: the grid is fixed on the host and the kernels read
// this round's item count (written by k_prefix) on the device, so a round
// needs no host round trip.
void launch_scan_f32(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  if (a.items_cap <= 0) return;
  if (a.kk > KMAX) {
    const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(a.items_cap, a.blocks)));
    if (a.metric == QUAKE_L2)
      hipLaunchKernelGGL(k_scan_f32_sorted<QUAKE_L2>, grid, dim3(256), 0, s, ws.items, ws.total, ws.q, st.dp, st.v32,
                         st.ids, st.d_off, st.d_size, a.kk, ws.pk, ws.pi);
    else
      hipLaunchKernelGGL(k_scan_f32_sorted<QUAKE_IP>, grid, dim3(256), 0, s, ws.items, ws.total, ws.q, st.dp, st.v32,
                         st.ids, st.d_off, st.d_size, a.kk, ws.pk, ws.pi);
    return;
  }
  if (a.metric == QUAKE_L2) scan_f32_k<QUAKE_L2>(ws, st, a, s);
  else scan_f32_k<QUAKE_IP>(ws, st, a, s);
}

// ---------------------------------------------------------------- commit

__device__ __forceinline__ double cap_share(const double* __restrict__ table, double t) {
  if (!(t < 1.0)) return 0.0;
  if (t < 0.0) t = 0.0;
  const double pos = t * (double)(CAP_TABLE_POINTS - 1);
  int j = (int)pos;
  if (j > CAP_TABLE_POINTS - 2) j = CAP_TABLE_POINTS - 2;
  const double f = pos - (double)j;
  const double a = table[j], b = table[j + 1];
  return a + f * (b - a);
}

// 1 / (1 + e_1 / (1 + e_2 / (1 + ...))), the continued fraction of I_x(a, b)
// with e_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1)) and
// e_{2m} = m (b - m) x / ((a + 2m - 1)(a + 2m)) (NIST DLMF 8.17.22), summed by
// the modified Lentz method (Thompson and Barnett, J. Comput. Phys. 64, 1986)
// until a factor is within 1e-16 of 1 (at most 4,096 terms).
__device__ double beta_fraction(double a, double b, double x) {
  const double tiny = 1e-300;
  double f = 1.0, C = 1.0, D = 0.0;
  for (int j = 1; j <= 4096; ++j) {
    const double m = (double)(j >> 1);
    const double e = (j & 1) ? -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0))
                             : m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
    D = 1.0 + e * D;
    if (fabs(D) < tiny) D = tiny;
    C = 1.0 + e / C;
    if (fabs(C) < tiny) C = tiny;
    D = 1.0 / D;
    const double delta = C * D;
    f *= delta;
    if (fabs(delta - 1.0) < 1e-16) break;
  }
  return 1.0 / f;
}

// The share of the ball beyond the bisector evaluated directly:
// 1/2 I_{1 - t^2}(a, 1/2) with a = (d + 1) / 2 and lb = log B(a, 1/2), both
// stored after the table's points.  The fraction is summed for x = 1 - t^2
// below (a + 1) / (a + 5/2), else for I_{t^2}(1/2, a) = 1 - I_{1-t^2}(a, 1/2),
// with t^2 passed in exactly.
__device__ double cap_direct(const double* __restrict__ table, double t) {
  if (!(t < 1.0)) return 0.0;
  if (t < 0.0) t = 0.0;
  const double a = table[CAP_TABLE_POINTS], lb = table[CAP_TABLE_POINTS + 1], b = 0.5;
  const double y = t * t, x = 1.0 - y;
  if (y <= 0.0) return 0.5;
  const double pre = exp(a * log(x) + b * log(y) - lb);
  if (x < (a + 1.0) / (a + b + 2.0)) return 0.5 * (pre / a) * beta_fraction(a, b, x);
  return 0.5 * (1.0 - (pre / b) * beta_fraction(b, a, y));
}

// The share of the ball beyond the bisector at t, from the table or (DIRECT)
// evaluated directly.
template <int DIRECT>
__device__ __forceinline__ double cap_value(const double* __restrict__ table, double t) {
  if constexpr (DIRECT) return cap_direct(table, t);
  else return cap_share(table, t);
}

// Euclidean distance to a result key: sqrt of the squared L2 distance, or for
// inner product on unit-norm data sqrt(|q|^2 + 1 - 2 s) with s = -key.
__device__ __forceinline__ double key_radius(float key, int ip, double qn2) {
  if (ip) {
    const double v = qn2 + 1.0 + 2.0 * (double)key;
    return sqrt(v > 0.0 ? v : 0.0);
  }
  return sqrt((double)(key > 0.f ? key : 0.f));
}

struct Model {
  double rho, p0, V, vsum;
};

// A filtered search (Sec. 8, "Filters"): each candidate's cap share v
// becomes the share of passing rows beyond its bisector,
// u = v f / (v f + (1 - v) f_0), with f the candidate partition's estimated
// pass fraction and f_0 that of the first partition.  A partition's
// estimate sums the live rows carrying each bit of the query's mask (exact
// for one label per row), capped at its live rows.
struct Filter {
  const int32_t* cand = nullptr;   // the query's candidate row
  const uint32_t* cnt = nullptr;   // [nlist][33]; null: no filter
  uint32_t mask = 0;
  double f0 = 1.0;
  __device__ double fraction(int p) const {
    const uint32_t* c = cnt + (int64_t)p * 33;
    const uint32_t live = c[32];
    if (live == 0) return 0.0;
    uint64_t est = 0;
    for (uint32_t m = mask; m; m &= m - 1) est += c[__builtin_ctz(m)];
    return (double)(est < live ? est : live) / (double)live;
  }
  // the share of candidate position i (>= 1) for cap share v
  __device__ double share(double v, int i) const {
    if (!cnt) return v;
    const double num = v * fraction(cand[i]);
    if (!(num > 0.0)) return 0.0;
    return num / (num + (1.0 - v) * f0);
  }
};

// p_0, V = sum v_i and the committed mass v_1 + ... + v_{m-1} for radius rho
// (candidates 1 .. M - 1 of the query).
template <int DIRECT, int FILT>
__device__ void recompute_model(Model& md, double rho, const float* __restrict__ hq, int M, int committed,
                                const double* __restrict__ table, const Filter& fl) {
  const int lane = lane_id();
  double vs = 0.0, pr = 1.0, vc = 0.0;
  const bool inf = __builtin_isinf(rho);
  for (int i = 1 + lane; i < M; i += WAVE) {
    const double t = inf ? 0.0 : (double)hq[i] / rho;
    double v = cap_value<DIRECT>(table, t);
    if constexpr (FILT) v = fl.share(v, i);
    vs += v;
    pr *= (1.0 - v);
    if (i < committed) vc += v;
  }
  md.rho = rho;
  md.V = wave_sum_d(vs);
  md.p0 = wave_prod_d(pr);
  md.vsum = wave_sum_d(vc);
  if (!(md.V > 0.0)) { md.p0 = 1.0; md.V = 0.0; md.vsum = 0.0; }
}

__device__ __forceinline__ double model_recall(const Model& md) {
  if (!(md.V > 0.0)) return md.p0;
  return md.p0 + (1.0 - md.p0) * (md.vsum / md.V);
}

// Smallest number of further candidates, from position `from`, after which
// the current model reaches the target; M - from if it never does.
template <int FILT>
__device__ int predict_window(const Model& md, const float* __restrict__ hq, int M, int from, double target,
                              const double* __restrict__ table, const Filter& fl) {
  if (!(md.V > 0.0)) return 1;
  const double need = (target - md.p0) * md.V / (1.0 - md.p0) - md.vsum;
  if (need <= 0.0) return 1;
  const int lane = lane_id();
  const bool inf = __builtin_isinf(md.rho);
  double run = 0.0;
  for (int base = from; base < M; base += WAVE) {
    const int i = base + lane;
    double v = 0.0;
    if (i < M) {
      v = cap_share(table, inf ? 0.0 : (double)hq[i] / md.rho);
      if constexpr (FILT) v = fl.share(v, i);
    }
    // inclusive scan over the wave
    for (int o = 1; o < WAVE; o <<= 1) {
      const double u = __shfl_up(v, o);
      if (lane >= o) v += u;
    }
    const uint64_t hit = __ballot(i < M && run + v >= need);
    if (hit) return base - from + __builtin_ctzll(hit) + 1;
    run += readlane_d(v, WAVE - 1);
  }
  return M - from;
}

// A query's committed list in LDS (one wave per query, lists up to LMAX).
template <int LMAX>
struct LdsList {
  float *Ak, *Bk, *Ok;
  int64_t *Ai, *Bi, *Oi;
  int kk;
  __device__ void load(const float* rk, const int64_t* ri) {
    for (int e = lane_id(); e < kk; e += WAVE) { Ak[e] = rk[e]; Ai[e] = ri[e]; }
  }
  __device__ void prime(const float*, const int64_t*) {}
  // merge partial list `cur`; `next` (or null) is the one after it
  __device__ void merge(const float* ck, const int64_t* ci, const float*, const int64_t*) {
    const int lane = lane_id();
    for (int e = lane; e < kk; e += WAVE) { Bk[e] = ck[e]; Bi[e] = ci[e]; }
    __syncthreads();
    wave_merge(Ak, Ai, Bk, Bi, Ok, Oi, kk);
    __syncthreads();
    for (int e = lane; e < kk; e += WAVE) { Ak[e] = Ok[e]; Ai[e] = Oi[e]; }
    __syncthreads();
  }
  __device__ float key(int j) const { return Ak[j]; }
  __device__ int64_t id(int j) const { return Ai[j]; }
  __device__ void store(float* rk, int64_t* ri) const {
    for (int e = lane_id(); e < kk; e += WAVE) { rk[e] = Ak[e]; ri[e] = Ai[e]; }
  }
};

// A query's committed list in registers, entry j in lane j (kk <= 64); the
// next partial list is loaded while the current one merges.
struct RegList {
  float k, nk;
  int64_t i, ni;
  int kk;
  __device__ void load(const float* rk, const int64_t* ri) {
    const int lane = lane_id();
    k = lane < kk ? rk[lane] : KEY_EMPTY;
    i = lane < kk ? ri[lane] : -1;
  }
  __device__ void prime(const float* pk, const int64_t* pi) {
    const int lane = lane_id();
    nk = lane < kk ? pk[lane] : KEY_EMPTY;
    ni = lane < kk ? pi[lane] : -1;
  }
  __device__ void merge(const float*, const int64_t*, const float* next_k, const int64_t* next_i) {
    const float bk = nk;
    const int64_t bi = ni;
    if (next_k) prime(next_k, next_i);
    wave_merge64_kv(k, i, bk, bi);
  }
  __device__ float key(int j) const { return readlane_f(k, j); }
  __device__ int64_t id(int j) const { return readlane_i64(i, j); }
  __device__ void store(float* rk, int64_t* ri) const {
    const int lane = lane_id();
    if (lane < kk) { rk[lane] = k; ri[lane] = i; }
  }
};

// The committed list of a batched search, whose entries carry store slots
// (below 2^31): (key, slot) packed into integers in result order, so that a
// merge step is one 64-bit compare.  A zero key is stored as +0 (a -0 key
// compares equal to it as a float).  Empty entries are (+inf, -1).
struct PackedList {
  uint64_t v, nv;
  int kk;
  __device__ static uint64_t empty() { return pack_key_slot(KEY_EMPTY, -1); }
  __device__ void load(const float* rk, const int64_t* ri) {
    const int lane = lane_id();
    v = lane < kk ? pack_key_slot(rk[lane] + 0.f, (int32_t)ri[lane]) : empty();
  }
  __device__ void prime(const float* pk, const int64_t* pi) {
    const int lane = lane_id();
    nv = lane < kk ? pack_key_slot(pk[lane] + 0.f, (int32_t)pi[lane]) : empty();
  }
  __device__ void merge(const float*, const int64_t*, const float* next_k, const int64_t* next_i) {
    const uint64_t b = nv;
    if (next_k) prime(next_k, next_i);
    wave_merge64_packed(v, b);
  }
  __device__ float key(int j) const { return packed_key((uint64_t)readlane_i64((int64_t)v, j)); }
  __device__ int64_t id(int j) const { return (int64_t)packed_slot((uint64_t)readlane_i64((int64_t)v, j)); }
  __device__ void store(float* rk, int64_t* ri) const {
    const int lane = lane_id();
    if (lane < kk) { rk[lane] = packed_key(v); ri[lane] = (int64_t)packed_slot(v); }
  }
};

// Commit one query's window in candidate order: merge each work item's
// partial list into the committed list; after each partition, update the
// recall model (recompute when rho moved by more than tau_rho * rho) and stop
// once the estimate reaches the target.  Partitions of the window after the
// stop point are discarded.  Then predict the next window.
template <int DIRECT, int FILT, class List>
__device__ void commit_query(int64_t q, List& L, int M, const int32_t* __restrict__ mq, int k, int kk, int aps,
                             int ip, int chunk_tiles, int wmax, int wscale, double tau_r, double tau_rho, int est,
                             const int32_t* __restrict__ cand, const float* __restrict__ hcand,
                             const int32_t* __restrict__ psize, const double* __restrict__ qn2,
                             const float* __restrict__ pk, const int64_t* __restrict__ pi,
                             const double* __restrict__ table, int32_t* __restrict__ st_m, int32_t* __restrict__ st_w,
                             int32_t* __restrict__ st_done, const int32_t* __restrict__ st_weff,
                             const int64_t* __restrict__ st_item, double* __restrict__ st_rho,
                             double* __restrict__ st_p0, double* __restrict__ st_V, double* __restrict__ st_vsum,
                             double* __restrict__ st_r, float* __restrict__ rk, int64_t* __restrict__ ri,
                             uint32_t* __restrict__ hits, const uint32_t* __restrict__ qmask,
                             const uint32_t* __restrict__ attr_cnt) {
  const int lane = lane_id();
  const int w = st_weff[q];
  L.load(rk + q * kk, ri + q * kk);
  const int m0 = st_m[q];
  const int Mq = mq[q];
  int64_t it = st_item[q];
  const float* hq = hcand + q * M;
  // chunk counts and bisector distances of the window's first 64 slots, slot
  // j in lane j: loaded together rather than one slot after another
  int my_nch = 0;
  float my_h = 0.f;
  if (lane < w) {
    my_nch = item_chunks(psize[cand[q * M + m0 + lane]], chunk_tiles);
    if (aps) my_h = hq[m0 + lane];
  }
  int64_t it_end = it;
  {
    int sum = my_nch;
    for (int o = WAVE / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    it_end += sum;
  }
  for (int j = WAVE; j < w; ++j) it_end += item_chunks(psize[cand[q * M + m0 + j]], chunk_tiles);
  L.prime(pk + it * kk, pi + it * kk);
  Model md{st_rho[q], st_p0[q], st_V[q], st_vsum[q]};
  Filter fl;
  if (FILT && aps) {
    fl.cand = cand + q * M;
    fl.cnt = attr_cnt;
    fl.mask = qmask[q];
    fl.f0 = fl.fraction(fl.cand[0]);
  }
  const double qn = ip ? qn2[q] : 0.0;
  double r = st_r[q];
  int committed = m0;
  bool stop = false;
  for (int j = 0; j < w && !stop; ++j) {
    const int nch = j < WAVE ? __builtin_amdgcn_readlane(my_nch, j)
                             : item_chunks(psize[cand[q * M + m0 + j]], chunk_tiles);
    for (int c = 0; c < nch; ++c, ++it) {
      const bool more = it + 1 < it_end;
      L.merge(pk + it * kk, pi + it * kk, more ? pk + (it + 1) * kk : nullptr, more ? pi + (it + 1) * kk : nullptr);
    }
    committed = m0 + j + 1;
    if (!aps) continue;
    const int64_t kth_id = L.id(k - 1);
    const bool full = kth_id >= 0;
    const double rho_new = full ? key_radius(L.key(k - 1), ip, qn) : __builtin_inf();
    if (committed == 1) {
      recompute_model<DIRECT, FILT>(md, rho_new, hq, Mq, committed, table, fl);
    } else {
      const bool redo = est != QUAKE_EST_APS || (__builtin_isinf(md.rho) ? !__builtin_isinf(rho_new)
                                                                          : fabs(rho_new - md.rho) > tau_rho * md.rho);
      if (redo) {
        recompute_model<DIRECT, FILT>(md, rho_new, hq, Mq, committed, table, fl);
      } else if (md.V > 0.0) {
        const float hc = j < WAVE ? readlane_f(my_h, j) : hq[committed - 1];  // committed - 1 = m0 + j
        const double t = __builtin_isinf(md.rho) ? 0.0 : (double)hc / md.rho;
        double v = cap_share(table, t);
        if constexpr (FILT) v = fl.share(v, committed - 1);
        md.vsum += v;
      }
    }
    r = full ? model_recall(md) : 0.0;
    if (r >= tau_r) stop = true;
  }
  const bool done = stop || committed >= Mq;
  int wn = 0;
  if (!done) {
    // the prediction assumes rho stays where it is; rho only shrinks as
    // more partitions are committed, so a query usually needs more - the
    // window is scaled by wscale percent (speculation costs scans, not
    // results: partitions past the stop point are discarded)
    if (aps && L.id(k - 1) >= 0) wn = (predict_window<FILT>(md, hq, Mq, committed, tau_r, table, fl) * wscale + 99) / 100;
    else wn = 2 * w;
    if (wn < 1) wn = 1;
    if (wn > wmax) wn = wmax;
  }
  L.store(rk + q * kk, ri + q * kk);
  // access statistics: every partition committed here was scanned by this query
  if (hits)
    for (int j = m0 + lane; j < committed; j += WAVE) atomicAdd(&hits[cand[q * M + j]], 1u);
  if (lane == 0) {
    st_m[q] = committed;
    st_w[q] = wn;
    st_done[q] = done ? 1 : 0;
    st_rho[q] = md.rho; st_p0[q] = md.p0; st_V[q] = md.V; st_vsum[q] = md.vsum;
    st_r[q] = aps ? r : 1.0;
  }
}

#define QK_COMMIT_PARAMS                                                                                          \
  int64_t nq, int M, const int32_t *__restrict__ mq, int k, int kk, int aps, int ip, int chunk_tiles, int wmax,  \
      int wscale,                                                                                                 \
      double tau_r, double tau_rho, int est, const int32_t *__restrict__ cand, const float *__restrict__ hcand,   \
      const int32_t *__restrict__ psize, const double *__restrict__ qn2, const float *__restrict__ pk,            \
      const int64_t *__restrict__ pi, const double *__restrict__ table, int32_t *__restrict__ st_m,              \
      int32_t *__restrict__ st_w, int32_t *__restrict__ st_done, const int32_t *__restrict__ st_weff,            \
      const int64_t *__restrict__ st_item, double *__restrict__ st_rho, double *__restrict__ st_p0,              \
      double *__restrict__ st_V, double *__restrict__ st_vsum, double *__restrict__ st_r, float *__restrict__ rk, \
      int64_t *__restrict__ ri, uint32_t *__restrict__ hits, const uint32_t *__restrict__ qmask,                  \
      const uint32_t *__restrict__ attr_cnt
#define QK_COMMIT_ARGS                                                                                        \
  M, mq, k, kk, aps, ip, chunk_tiles, wmax, wscale, tau_r, tau_rho, est, cand, hcand, psize, qn2, pk, pi, table, st_m, st_w, \
      st_done, st_weff, st_item, st_rho, st_p0, st_V, st_vsum, st_r, rk, ri, hits, qmask, attr_cnt

// Lists longer than a wave: one 64-thread block per query, lists in LDS.
// DIRECT: cap shares evaluated directly (APS-RP); FILT: a filtered search.
template <int DIRECT, int FILT, int LMAX>
__global__ __launch_bounds__(64) void k_commit(QK_COMMIT_PARAMS) {
  __shared__ float Ak[LMAX], Bk[LMAX], Ok[LMAX];
  __shared__ int64_t Ai[LMAX], Bi[LMAX], Oi[LMAX];
  const int64_t q = blockIdx.x;
  if (st_done[q] || st_weff[q] == 0) return;
  LdsList<LMAX> L{Ak, Bk, Ok, Ai, Bi, Oi, kk};
  commit_query<DIRECT, FILT>(q, L, QK_COMMIT_ARGS);
}

// Lists of at most 64 entries: one wave per query, four queries per block,
// lists in registers.
template <int DIRECT, int FILT, class List>
__global__ __launch_bounds__(256) void k_commit64(QK_COMMIT_PARAMS) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq || st_done[q] || st_weff[q] == 0) return;
  List L;
  L.kk = kk;
  commit_query<DIRECT, FILT>(q, L, QK_COMMIT_ARGS);
}

template <int DIRECT, int FILT>
static void launch_commit_k(Workspace& ws, const Store& st, const RoundArgs& a, const double* table, hipStream_t s) {
#define QK_COMMIT(KERNEL, GRID, BLOCK)                                                                        \
  hipLaunchKernelGGL(KERNEL, dim3((unsigned)(GRID)), dim3(BLOCK), 0, s, a.nq, a.M, ws.mq, a.k, a.kk, a.aps,    \
                     a.metric == QUAKE_IP ? 1 : 0, a.chunk_tiles, a.wmax, a.wscale, a.tau_r, a.tau_rho, a.est,      \
                     ws.cand,                                                                                   \
                     ws.h,                                                                                      \
                     st.d_size, ws.qn2, ws.pk, ws.pi, table, ws.st_m, ws.st_w, ws.st_done, ws.st_weff,        \
                     ws.st_item, ws.st_rho, ws.st_p0, ws.st_V, ws.st_vsum, ws.st_r, ws.rk, ws.ri, a.hits, a.qmask,   \
                     a.attr_cnt)
  if (a.kk <= WAVE && a.slot_ids) QK_COMMIT((k_commit64<DIRECT, FILT, PackedList>), (a.nq + 3) / 4, 256);
  else if (a.kk <= WAVE) QK_COMMIT((k_commit64<DIRECT, FILT, RegList>), (a.nq + 3) / 4, 256);
  else if (a.kk <= KMAX) QK_COMMIT((k_commit<DIRECT, FILT, KMAX>), a.nq, 64);
  else QK_COMMIT((k_commit<DIRECT, FILT, KMAX_LARGE>), a.nq, 64);
#undef QK_COMMIT
}

void launch_commit(Workspace& ws, const Store& st, const RoundArgs& a, const double* table, hipStream_t s) {
  if (a.nq <= 0) return;
  const bool direct = a.aps && a.est == QUAKE_EST_APS_RP, filt = a.aps && a.qmask;
  if (direct) {
    if (filt) launch_commit_k<1, 1>(ws, st, a, table, s);
    else launch_commit_k<1, 0>(ws, st, a, table, s);
  } else {
    if (filt) launch_commit_k<0, 1>(ws, st, a, table, s);
    else launch_commit_k<0, 0>(ws, st, a, table, s);
  }
}

// ---------------------------------------------------------------- outputs

__global__ __launch_bounds__(256) void k_finalize(int64_t nq, int k, int kk, int ip, const float* __restrict__ rk,
                                                   const int64_t* __restrict__ ri, const int32_t* __restrict__ st_m,
                                                   const double* __restrict__ st_r, int64_t* __restrict__ out_ids,
                                                   float* __restrict__ out_dist, int32_t* __restrict__ out_ns,
                                                   double* __restrict__ out_r) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nq * k) return;
  const int64_t q = e / k;
  const int j = (int)(e - q * k);
  const float key = rk[q * kk + j];
  out_ids[e] = ri[q * kk + j];
  out_dist[e] = ip ? -key : key;
  if (j == 0) {
    if (out_ns) out_ns[q] = st_m[q];
    if (out_r) out_r[q] = st_r[q];
  }
}

void launch_finalize(Workspace& ws, const RoundArgs& a, int64_t* out_ids, float* out_dist, int32_t* out_nscanned,
                     double* out_recall, hipStream_t s) {
  const int64_t n = a.nq * a.k;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.nq, a.k, a.kk,
                     a.metric == QUAKE_IP ? 1 : 0, ws.rk, ws.ri, ws.st_m, ws.st_r, out_ids, out_dist, out_nscanned,
                     out_recall);
}

}  // namespace qk

// Batched scan: queries that need the same partition in a round share one
// read of it (multi-query execution: group queries by the partitions they
// access and scan each partition once per batch, Sec. 7.5).
//
// Per round, every query's window of (query, partition) pairs is bucketed by
// partition.  A work item is (partition, group of up to 16 queries, chunk of
// tiles).  One wave scores a 64-vector tile against its 16 queries with
// v_mfma_f32_16x16x32 on the 16-bit store copy (BF16 or FP16 products, FP32
// accumulation): the queries sit in registers as B operands for the whole
// item, the tile is read straight from the store into A operands (the store's
// [chunk][64 vectors][8 elements] tile layout is the A fragment order, so a
// wave's load of one k-step covers four contiguous 256-byte runs).  The
// 16 x 64 score block goes through LDS so that each query's 64 scores sit one
// per lane, where a wave-wide top-k list (one entry per lane) keeps the
// query's best rerank_factor * k candidates.  Partial lists land in the same
// per-(query, partition, chunk) slots as the plain scan, so the in-order
// commit and the recall model are shared.  Candidates carry store slots; after
// the last round each query's candidates are re-scored in FP32 from the FP32
// store (the same arithmetic as the plain scan) and the best k are kept.
#include "common.hpp"
#include "index.hpp"

namespace qk {

constexpr int G = 16;  // queries per work item (one MFMA column block)

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;

__device__ __forceinline__ int chunks_of(int32_t size, int chunk_tiles) {
  const int tiles = (size + TILE - 1) / TILE;
  const int c = (tiles + chunk_tiles - 1) / chunk_tiles;
  return c > 0 ? c : 1;
}

// ---------------------------------------------------------------- queries

__device__ __forceinline__ uint16_t round_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void k_queries16(const float* __restrict__ q, int64_t nq, int dp, int dp16,
                                                    int f16, const double* __restrict__ qn2, uint16_t* __restrict__ q16,
                                                    float* __restrict__ qn2f, const int32_t* __restrict__ slots) {
  const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i = e0 / dp16;
  if (i >= nq) return;
  const int j = (int)(e0 - i * dp16);
  const int64_t row = slots ? slots[i] : i;
  const int64_t e = row * dp16 + j;
  const float v = j < dp ? q[row * dp + j] : 0.f;
  q16[e] = f16 ? __builtin_bit_cast(uint16_t, (_Float16)v) : round_bf16(v);
  if (j == 0) qn2f[row] = (float)qn2[row];
}

void launch_queries16(Workspace& ws, int64_t nq, int dp, int dp16, int dtype16, hipStream_t s, const int32_t* slots) {
  const int64_t n = nq * dp16;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_queries16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ws.q, nq, dp, dp16,
                     dtype16 == QUAKE_F16 ? 1 : 0, ws.qn2, ws.q16, ws.qn2f, slots);
}

// ---------------------------------------------------------------- grouping

// Record every (query, window slot) pair of the round and count pairs per
// partition.  pair_base is the first partial-list slot of the pair (the same
// numbering as the plain scan's work items).
__global__ __launch_bounds__(256) void k_pairs(int64_t nq, int M, int chunk_tiles, const int32_t* __restrict__ cand,
                                                const int32_t* __restrict__ psize, const int32_t* __restrict__ st_m,
                                                const int32_t* __restrict__ st_weff,
                                                const int64_t* __restrict__ st_item,
                                                const int64_t* __restrict__ st_pair, int32_t* __restrict__ pcount,
                                                int32_t* __restrict__ pair_q, int32_t* __restrict__ pair_p,
                                                int32_t* __restrict__ pair_pos, int64_t* __restrict__ pair_base) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nq) return;
  const int w = st_weff[q];
  if (w == 0) return;
  const int m = st_m[q];
  int64_t it = st_item[q];
  const int64_t pr = st_pair[q];
  for (int j = 0; j < w; ++j) {
    const int p = cand[q * M + m + j];
    pair_q[pr + j] = (int32_t)q;
    pair_p[pr + j] = p;
    pair_base[pr + j] = it;
    pair_pos[pr + j] = atomicAdd(&pcount[p], 1);
    it += chunks_of(psize[p], chunk_tiles);
  }
}

// Per-partition pair offsets and work-item offsets (one block); clears the
// counts for the next round and adds the round's vector reads and
// query-vector products to the running totals.
__global__ __launch_bounds__(1024) void k_part_prefix(int64_t N, int chunk_tiles, int32_t* __restrict__ pcount,
                                                       const int32_t* __restrict__ psize, int32_t* __restrict__ pstart,
                                                       int64_t* __restrict__ pitem, int64_t* __restrict__ counters) {
  __shared__ int64_t sp[1024], si[1024];
  __shared__ unsigned long long reads, products;
  const int t = threadIdx.x;
  const int64_t per = (N + 1023) / 1024;
  const int64_t lo = t * per;
  const int64_t hi = (lo + per < N) ? lo + per : N;
  int64_t np = 0, ni = 0;
  unsigned long long rd = 0, pd = 0;
  for (int64_t p = lo; p < hi; ++p) {
    const int c = pcount[p];
    np += c;
    if (c > 0) {
      const int groups = (c + G - 1) / G;
      ni += (int64_t)groups * chunks_of(psize[p], chunk_tiles);
      rd += (unsigned long long)groups * (unsigned long long)psize[p];
      pd += (unsigned long long)c * (unsigned long long)psize[p];
    }
  }
  sp[t] = np;
  si[t] = ni;
  if (t == 0) { reads = 0; products = 0; }
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t a = (t >= o) ? sp[t - o] : 0;
    const int64_t b = (t >= o) ? si[t - o] : 0;
    __syncthreads();
    sp[t] += a;
    si[t] += b;
    __syncthreads();
  }
  int64_t rp = sp[t] - np, ri = si[t] - ni;
  for (int64_t p = lo; p < hi; ++p) {
    const int c = pcount[p];
    pstart[p] = (int32_t)rp;
    pitem[p] = ri;
    rp += c;
    if (c > 0) ri += (int64_t)((c + G - 1) / G) * chunks_of(psize[p], chunk_tiles);
    pcount[p] = 0;
  }
  atomicAdd(&reads, rd);
  atomicAdd(&products, pd);
  __syncthreads();
  if (t == 0) {
    pstart[N] = (int32_t)sp[1023];
    pitem[N] = si[1023];
    counters[3] = si[1023];
    counters[4] += (int64_t)reads;
    counters[5] += (int64_t)products;
  }
}

__global__ __launch_bounds__(256) void k_pair_scatter(const int64_t* __restrict__ counters,
                                                       const int32_t* __restrict__ pair_p,
                                                       const int32_t* __restrict__ pair_pos,
                                                       const int32_t* __restrict__ pstart,
                                                       int32_t* __restrict__ sorted) {
  const int64_t npairs = counters[2];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < npairs; e += (int64_t)gridDim.x * 256)
    sorted[pstart[pair_p[e]] + pair_pos[e]] = (int32_t)e;
}

void launch_group(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pairs, dim3((unsigned)((a.nq + 255) / 256)), dim3(256), 0, s, a.nq, a.M, a.chunk_tiles,
                     ws.cand, st.d_size, ws.st_m, ws.st_weff, ws.st_item, ws.st_pair, ws.pcount, ws.pair_q, ws.pair_p,
                     ws.pair_pos, ws.pair_base);
  hipLaunchKernelGGL(k_part_prefix, dim3(1), dim3(1024), 0, s, st.nlist, a.chunk_tiles, ws.pcount, st.d_size,
                     ws.pstart, ws.pitem, ws.total);
  // at most wmax pairs per query; the kernel reads this round's count
  const int64_t bound = (a.nq * a.wmax + 255) / 256;
  hipLaunchKernelGGL(k_pair_scatter, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(bound, 2048))), dim3(256),
                     0, s, ws.total, ws.pair_p, ws.pair_pos, ws.pstart, ws.sorted);
}

// ---------------------------------------------------------------- MFMA scan

template <int F16>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                   0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                    0, 0, 0);
}

template <int F16, int KS, int IP>
__global__ __launch_bounds__(256, 2) void k_scan_mfma(
    const int64_t* __restrict__ counters, const int64_t* __restrict__ pitem, const int32_t* __restrict__ pstart,
    const int32_t* __restrict__ sorted, const int32_t* __restrict__ pair_q, const int64_t* __restrict__ pair_base,
    int64_t N, int chunk_tiles, const uint16_t* __restrict__ q16, int dp16, const float* __restrict__ qn2f,
    const uint16_t* __restrict__ v16, const float* __restrict__ v16n, const int64_t* __restrict__ sid,
    const int64_t* __restrict__ poff, const int32_t* __restrict__ psize, const float* __restrict__ rk,
    const int64_t* __restrict__ ri, int kk, float* __restrict__ pk, int64_t* __restrict__ pi) {
  __shared__ float S[4][G][TILE + 1];
  __shared__ float BK[4][G][WAVE];      // per query: candidates that beat the threshold, not yet merged
  __shared__ int32_t BS[4][G][WAVE];
  __shared__ float TK[4][G];            // per query: key and slot a candidate must beat
  __shared__ int32_t TS[4][G];
  __shared__ int32_t CN[4][G];          // per query: candidates waiting in BK / BS
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // consecutive logical blocks on one XCD (blocks are dealt to the 8 XCDs in turn)
  int lb = blockIdx.x;
  if ((gridDim.x & 7) == 0) lb = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const int64_t total = counters[3];
  const int64_t stride = (int64_t)gridDim.x * 4;
  static_assert(KS >= 2, "the load pipeline runs two k-steps ahead");
  constexpr int nc8 = KS * 4;  // 8-element chunks per row of the 16-bit copy
  float (*Sw)[TILE + 1] = S[wave];
  float (*Bk)[WAVE] = BK[wave];
  int32_t (*Bs)[WAVE] = BS[wave];
  float* Tk = TK[wave];
  int32_t* Ts = TS[wave];
  int32_t* Cn = CN[wave];
  for (int64_t it = (int64_t)lb * 4 + wave; it < total; it += stride) {
    int64_t lo = 0, hi = N;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (pitem[mid] <= it) lo = mid; else hi = mid;
    }
    const int p = __builtin_amdgcn_readfirstlane((int)lo);
    const int size = psize[p];
    const int tiles = (size + TILE - 1) / TILE;
    const int nch = chunks_of(size, chunk_tiles);
    const int local = (int)(it - pitem[p]);
    const int np = pstart[p + 1] - pstart[p];
    // the query group runs fastest, so that the waves of a block and the
    // neighbouring blocks on the same XCD score the same tiles together and
    // share them through L2
    const int ngroups = (np + G - 1) / G;
    const int c = local / ngroups, g = local - (local / ngroups) * ngroups;
    const int gcount = min(G, np - g * G);
    const int t0 = c * chunk_tiles;
    const int t1 = min(tiles, t0 + chunk_tiles);
    const int j = lane & (G - 1);
    const bool has = j < gcount;
    const int pair = has ? sorted[pstart[p] + g * G + j] : 0;
    const int qj = has ? pair_q[pair] : 0;
    u32x4 breg[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      u32x4 b = {0u, 0u, 0u, 0u};
      if (has) b = *reinterpret_cast<const u32x4*>(q16 + (int64_t)qj * dp16 + 32 * s + 8 * (lane >> 4));
      breg[s] = b;
    }
    const float my_qn2 = (IP || !has) ? 0.f : qn2f[qj];
    // per query: a sorted list of its 64 best (one entry per lane), the
    // threshold a candidate must beat (the kk-th entry, or the seed from the
    // query's committed results) and the fill of its LDS buffer
    float lk[G];
    int32_t ls[G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) { lk[jj] = KEY_EMPTY; ls[jj] = -1; }
    if (lane < G) {
      float sk = -KEY_EMPTY;
      int32_t ss = -1;
      if (lane < gcount) {
        sk = rk[(int64_t)qj * kk + kk - 1];
        ss = (int32_t)ri[(int64_t)qj * kk + kk - 1];
      }
      Tk[lane] = sk;
      Ts[lane] = ss;
      Cn[lane] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    auto flush = [&](int jj) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const int n = Cn[jj];
      float bk = KEY_EMPTY;
      int32_t bs = -1;
      if (lane < n) { bk = Bk[jj][lane]; bs = Bs[jj][lane]; }
      wave_sort64(bk, bs);
      wave_merge64(lk[jj], ls[jj], bk, bs);
      const int32_t ns = __builtin_amdgcn_readlane(ls[jj], kk - 1);
      const float nk = readlane_f(lk[jj], kk - 1);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      if (lane == 0) {
        Cn[jj] = 0;
        if (ns >= 0) { Tk[jj] = nk; Ts[jj] = ns; }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    };
    const int64_t tile0 = poff[p];
    // A fragments of one k-step: vectors 16b + (lane & 15) of the tile,
    // elements 32s + 8 (lane >> 4) .. + 7, i.e. 16-byte chunk 4s + (lane >> 4)
    const int frag = (lane >> 4) * TILE + (lane & 15);
    auto kstep = [&](const u32x4* tb, int s, u32x4 (&a)[4]) {
#pragma unroll
      for (int b = 0; b < 4; ++b) a[b] = tb[(int64_t)(4 * s) * TILE + frag + 16 * b];
    };
    // Loads run two k-steps ahead of the MFMAs and continue into the next
    // tile, so its first fragments are in flight during this tile's top-k.
    const u32x4* tb_cur = reinterpret_cast<const u32x4*>(v16) + (tile0 + t0) * (int64_t)nc8 * TILE;
    u32x4 pa[2][4];
    if (t0 < t1) {
      kstep(tb_cur, 0, pa[0]);
      kstep(tb_cur, 1, pa[1]);
    }
    for (int t = t0; t < t1; ++t) {
      const int64_t tile = tile0 + t;
      const u32x4* tb_next = (t + 1 < t1) ? tb_cur + (int64_t)nc8 * TILE : tb_cur;
      f32x4 acc[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = mfma16<F16>(pa[s & 1][b], breg[s], acc[b]);
        if (s + 2 < KS) kstep(tb_cur, s + 2, pa[s & 1]);
        else kstep(tb_next, s + 2 - KS, pa[s & 1]);
      }
      tb_cur = tb_next;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) Sw[j][16 * b + (lane >> 4) * 4 + v] = acc[b][v];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      const bool valid = t * TILE + lane < size;
      const int32_t slot = (int32_t)(tile * TILE + lane);
      const float xn = IP ? 0.f : v16n[slot];
      const bool live = valid && sid[slot] >= 0;
#pragma unroll
      for (int jj = 0; jj < G; ++jj) {
        if (jj >= gcount) break;
        const float dot = Sw[jj][lane];
        const float key = IP ? -dot : (__shfl(my_qn2, jj) + xn - 2.f * dot);
        const float tkj = Tk[jj];
        const int32_t tsj = Ts[jj];
        bool pass = live && ks_less(key, slot, tkj, tsj);
        uint64_t mask = __ballot(pass);
        if (mask) {
          int n = __popcll(mask);
          int c0 = Cn[jj];
          if (c0 + n > WAVE) {
            flush(jj);
            pass = live && ks_less(key, slot, Tk[jj], Ts[jj]);
            mask = __ballot(pass);
            n = __popcll(mask);
            c0 = 0;
          }
          const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
          if (pass) {
            Bk[jj][c0 + rank] = key;
            Bs[jj][c0 + rank] = slot;
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          if (lane == 0) Cn[jj] = c0 + n;
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      if (jj >= gcount) break;
      if (Cn[jj] > 0) flush(jj);
      const int pr = __builtin_amdgcn_readlane(pair, jj);
      const int64_t out = (pair_base[pr] + c) * kk;
      if (lane < kk) {
        pk[out + lane] = lk[jj];
        pi[out + lane] = (int64_t)ls[jj];
      }
    }
  }
}

template <int F16, int IP>
static void scan_mfma_k(Workspace& ws, const Store& st, const RoundArgs& a, int blocks, hipStream_t s) {
  const int ks = st.dp16 / 32;
#define QK_MFMA_LAUNCH(KS)                                                                                      \
  hipLaunchKernelGGL((k_scan_mfma<F16, KS, IP>), dim3(blocks), dim3(256), 0, s, ws.total, ws.pitem, ws.pstart, \
                     ws.sorted, ws.pair_q, ws.pair_base, st.nlist, a.chunk_tiles, ws.q16, st.dp16, ws.qn2f,    \
                     st.v16, st.v16n, st.ids, st.d_off, st.d_size, ws.rk, ws.ri, a.kk, ws.pk, ws.pi)
  switch (ks) {
    case 2: QK_MFMA_LAUNCH(2); break;
    case 4: QK_MFMA_LAUNCH(4); break;
    case 8: QK_MFMA_LAUNCH(8); break;
    case 12: QK_MFMA_LAUNCH(12); break;
    case 16: QK_MFMA_LAUNCH(16); break;
    case 24: QK_MFMA_LAUNCH(24); break;
    case 32: QK_MFMA_LAUNCH(32); break;
    default: break;  // rows of the 16-bit copy are padded to one of these lengths
  }
#undef QK_MFMA_LAUNCH
}

void launch_scan_mfma(Workspace& ws, const Store& st, const RoundArgs& a, int dtype16, hipStream_t s) {
  const int blocks = std::max(a.blocks, 1);
  const bool f16 = dtype16 == QUAKE_F16;
  const bool ip = a.metric == QUAKE_IP;
  if (f16) { if (ip) scan_mfma_k<1, 1>(ws, st, a, blocks, s); else scan_mfma_k<1, 0>(ws, st, a, blocks, s); }
  else { if (ip) scan_mfma_k<0, 1>(ws, st, a, blocks, s); else scan_mfma_k<0, 0>(ws, st, a, blocks, s); }
}

// ---------------------------------------------------------------- rerank

// Re-score each query's candidates (store slots) in FP32 and keep the best k
// by (distance, id).  The vectors come from the row-major FP32 copy kept for
// this purpose (one contiguous row per candidate; the tile-interleaved store
// would fetch a whole cache line per 16 bytes used); the sum runs in the same
// order as the plain scan's: eight partial sums over the dimensions modulo 8,
// added pairwise.  One wave per query, one lane per candidate for the sort;
// the distance of each candidate is computed by the whole wave.
template <int METRIC>
__global__ __launch_bounds__(64) void k_rerank(int64_t nq, int k, int kk, const float* __restrict__ qpad, int dp,
                                                const float* __restrict__ rows, const int64_t* __restrict__ sid,
                                                float* __restrict__ rk, int64_t* __restrict__ ri,
                                                const int32_t* __restrict__ slots) {
  const int64_t q = slots ? slots[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x;
  const float* qv = qpad + q * dp;
  const int64_t myslot = lane < kk ? ri[q * kk + lane] : -1;
  float key = KEY_EMPTY;
  int64_t id = -1;
  // lanes 8e .. 8e+7 hold the eight partial sums of candidate e (dimension j
  // goes to partial j mod 8); candidates are handled eight at a time
  const int part = lane & 7, grp = lane >> 3;
  for (int e0 = 0; e0 < kk; e0 += 8) {
    const int e = e0 + grp;
    const int64_t slot = e < kk ? __shfl(myslot, e) : -1;
    float acc = 0.f;
    if (slot >= 0) {
      const float* xv = rows + slot * (int64_t)dp;
      for (int jj = part; jj < dp; jj += 8) {
        const float x = xv[jj], y = qv[jj];
        acc = METRIC == QUAKE_L2 ? fmaf(x - y, x - y, acc) : fmaf(x, y, acc);
      }
    }
    // pairwise: ((a0+a1)+(a2+a3))+((a4+a5)+(a6+a7))
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 4);
    const float d = METRIC == QUAKE_L2 ? acc : -acc;
    const float dk = __shfl(d, (lane - e0) * 8);
    if (lane >= e0 && lane < e0 + 8 && myslot >= 0) key = dk;
  }
  if (myslot >= 0) id = sid[myslot];
  // bitonic sort of the 64 (key, id) pairs across the wave, ascending
  for (int size = 2; size <= WAVE; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const float ok = __shfl_xor(key, stride);
      const int64_t oi = (int64_t)(((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)((uint64_t)id >> 32), stride) << 32) |
                                   (uint32_t)__shfl_xor((int)(uint32_t)(uint64_t)id, stride));
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const bool other_first = kv_less(ok, oi, key, id);
      const bool take = (lower == up) ? other_first : !other_first;
      if (take) { key = ok; id = oi; }
    }
  }
  if (lane < k) { rk[q * kk + lane] = key; ri[q * kk + lane] = id; }
}

void launch_rerank(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s, const int32_t* slots,
                   int64_t nslots) {
  const int64_t n = slots ? nslots : a.nq;
  if (n <= 0) return;
  if (a.metric == QUAKE_L2)
    hipLaunchKernelGGL(k_rerank<QUAKE_L2>, dim3((unsigned)n), dim3(64), 0, s, a.nq, a.k, a.kk, ws.q, st.dp,
                       st.rows32, st.ids, ws.rk, ws.ri, slots);
  else
    hipLaunchKernelGGL(k_rerank<QUAKE_IP>, dim3((unsigned)n), dim3(64), 0, s, a.nq, a.k, a.kk, ws.q, st.dp,
                       st.rows32, st.ids, ws.rk, ws.ri, slots);
}

// ---------------------------------------------------------------- store norms

// |x|^2 of the 16-bit copy of every slot (for L2 keys from inner products).
__global__ __launch_bounds__(256) void k_norm16(const uint16_t* __restrict__ v16, int64_t slots, int dp16, int f16,
                                                 float* __restrict__ out) {
  const int64_t sl = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (sl >= slots) return;
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

void launch_norm16(const Store& st, int dtype16, hipStream_t s) {
  const int64_t slots = st.tiles * TILE;
  if (slots <= 0 || !st.v16 || !st.v16n) return;
  hipLaunchKernelGGL(k_norm16, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, s, st.v16, slots, st.dp16,
                     dtype16 == QUAKE_F16 ? 1 : 0, st.v16n);
}

}  // namespace qk

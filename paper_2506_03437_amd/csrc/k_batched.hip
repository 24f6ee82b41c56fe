// Batched scan: queries that need the same partition in a round share one
// read of it (multi-query execution: group queries by the partitions they
// access and scan each partition once per batch, Sec. 7.4, "Multi-Query Processing").
//
// Per round, every query's window of (query, partition) pairs is bucketed by
// partition.  A work item is (partition chunk of up to chunk_tiles tiles,
// set of up to 128 of the partition's queries); items are numbered largest
// partition first.  A block of eight waves takes items from a queue; each
// tile of the chunk is staged once through LDS and scored by the eight waves
// for 128 queries with v_mfma_f32_16x16x32 on the 16-bit store copy (BF16
// or FP16 products, FP32 accumulation): the queries sit in registers as B
// operands for the whole item and the store's [chunk][64 vectors][8
// elements] tile layout is the A fragment order.  The waves work in pairs
// on two 16-query groups, one taking the even k-steps and the other the odd
// ones, so every A fragment read from LDS feeds two MFMAs (LDS reads, not
// the matrix cores, bound a tile shared by this many queries); at the end of
// a tile the two halves of each group's sums meet in LDS.  After each tile every lane
// holds 16 scores of one query and tests them against the query's threshold;
// candidates go to a per-query pool in LDS that is cut by ballot-count
// bisection, and at the item's end each query's best rerank_factor * k
// (key, slot) are written, sorted, to the same per-(query, partition, chunk)
// partial-list slots as the plain scan uses, so the in-order commit and the
// recall model are shared.  Candidates carry store slots; after the last
// round they are re-scored in FP32 (k_rerank.hip).
#include <type_traits>

#include "common.hpp"
#include "index.hpp"

namespace qk {

constexpr int G = 16;           // queries per wave (one MFMA column block)
constexpr int SET_GROUPS = 8;   // query groups per block, one per wave
constexpr int SET = G * SET_GROUPS;  // queries that share one read of a tile
constexpr int NT = WAVE * SET_GROUPS;  // threads per scan block
constexpr int BUF = 2 * WAVE;   // per-query candidate pool (two entries per lane): a cut keeps at most
                                // max(kk, 64) <= 64 entries, so a whole tile's 64 always fit after one
constexpr int MAX_ITEM_TILES = 1024;  // pool slots are 16-bit offsets from the item's first slot
constexpr int SLACK = 16;       // entries a mid-item cut may keep beyond kk (room permitting)
constexpr int QUEUE_X = 16;     // counters[16, 24): the batched scan's item queues, [24, 32): their lengths
constexpr int XCDS = 8;         // compute dies (XCDs) of the GPU, each with its own L2

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
// numbering as the plain scan's work items).  One wave per query, a lane per
// window slot: the slots' item offsets are a prefix sum over the wave.
__global__ __launch_bounds__(256) void k_pairs(int64_t nq, int M, int chunk_tiles, const int32_t* __restrict__ cand,
                                                const int32_t* __restrict__ psize, const int32_t* __restrict__ st_m,
                                                const int32_t* __restrict__ st_weff,
                                                const int64_t* __restrict__ st_item,
                                                const int64_t* __restrict__ st_pair, int32_t* __restrict__ pcount,
                                                int32_t* __restrict__ pair_q, int32_t* __restrict__ pair_p,
                                                int32_t* __restrict__ pair_pos, int64_t* __restrict__ pair_base) {
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (q >= nq) return;
  const int w = st_weff[q];
  if (w == 0) return;
  const int m = st_m[q];
  int64_t it = st_item[q];
  const int64_t pr = st_pair[q];
  for (int j0 = 0; j0 < w; j0 += WAVE) {
    const int j = j0 + lane;
    const bool on = j < w;
    const int p = on ? cand[q * M + m + j] : 0;
    const int c = on ? chunks_of(psize[p], chunk_tiles) : 0;
    int incl = c;
    for (int o = 1; o < WAVE; o <<= 1) {
      const int u = __shfl_up(incl, o);
      if (lane >= o) incl += u;
    }
    if (on) {
      pair_q[pr + j] = (int32_t)q;
      pair_p[pr + j] = p;
      pair_base[pr + j] = it + (incl - c);
      pair_pos[pr + j] = atomicAdd(&pcount[p], 1);
    }
    it += __shfl(incl, WAVE - 1);
  }
}

// Per-partition pair offsets (partition order) and work-item offsets (in
// `order`, largest partitions first: the scan takes items in index order, so
// a launch ends on short items); clears the counts for the next round and
// adds to the running totals the round's distinct vector reads (each
// partition a round touches, once), its reads counted once per query set,
// and its query-vector products.  One block.
//
// The items also go to eight queues, one per compute die (XCD): the
// partition of size rank r to queue r % 8, each queue largest partition
// first.  A scan block takes items from its die's queue (then from the
// others), so the query sets of a chunk are scored on one die at about the
// same time and its L2 serves their repeated reads of the chunk.
__global__ __launch_bounds__(1024) void k_part_prefix(int64_t N, int chunk_tiles, int32_t* __restrict__ pcount,
                                                       const int32_t* __restrict__ psize,
                                                       const int32_t* __restrict__ order, int32_t* __restrict__ pstart,
                                                       int64_t* __restrict__ pitem, int64_t* __restrict__ pxoff,
                                                       int32_t* __restrict__ pxcd, int64_t* __restrict__ counters) {
  __shared__ int64_t sp[1024], si[1024], sx[XCDS][1024];
  __shared__ unsigned long long reads, set_reads, products;
  const int t = threadIdx.x;
  const int64_t per = (N + 1023) / 1024;
  const int64_t lo = t * per;
  const int64_t hi = (lo + per < N) ? lo + per : N;
  auto items_of = [&](int64_t p) -> int64_t {
    const int c = pcount[p];
    return c > 0 ? (int64_t)((c + SET - 1) / SET) * chunks_of(psize[p], chunk_tiles) : 0;
  };
  int64_t np = 0, ni = 0;
  unsigned long long rd = 0, srd = 0, pd = 0;
  for (int64_t p = lo; p < hi; ++p) {
    const int c = pcount[p];
    np += c;
    if (c > 0) {
      const int sets = (c + SET - 1) / SET;
      rd += (unsigned long long)psize[p];
      srd += (unsigned long long)sets * (unsigned long long)psize[p];
      pd += (unsigned long long)c * (unsigned long long)psize[p];
    }
  }
  for (int64_t r = lo; r < hi; ++r) ni += items_of(order[r]);
  sp[t] = np;
  si[t] = ni;
  if (t == 0) { reads = 0; set_reads = 0; products = 0; }
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t a = (t >= o) ? sp[t - o] : 0;
    const int64_t b = (t >= o) ? si[t - o] : 0;
    __syncthreads();
    sp[t] += a;
    si[t] += b;
    __syncthreads();
  }
  int64_t ri = si[t] - ni;
  for (int64_t r = lo; r < hi; ++r) {
    const int64_t p = order[r];
    pitem[p] = ri;
    ri += items_of(p);
  }
  // the die queues: a prefix over the ranks of each residue, the eight
  // residues scanned together
  int64_t mine[XCDS];
#pragma unroll
  for (int x = 0; x < XCDS; ++x) mine[x] = 0;
  for (int64_t r = lo; r < hi; ++r) mine[r & (XCDS - 1)] += items_of(order[r]);
#pragma unroll
  for (int x = 0; x < XCDS; ++x) sx[x][t] = mine[x];
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t a[XCDS];
#pragma unroll
    for (int x = 0; x < XCDS; ++x) a[x] = (t >= o) ? sx[x][t - o] : 0;
    __syncthreads();
#pragma unroll
    for (int x = 0; x < XCDS; ++x) sx[x][t] += a[x];
    __syncthreads();
  }
  {
    int64_t run[XCDS];
#pragma unroll
    for (int x = 0; x < XCDS; ++x) run[x] = sx[x][t] - mine[x];
    for (int64_t r = lo; r < hi; ++r) {
      const int x = (int)(r & (XCDS - 1));
      const int64_t p = order[r];
      pxoff[p] = run[x];
      pxcd[p] = x;
      run[x] += items_of(p);
    }
  }
  if (t < XCDS) {
    counters[QUEUE_X + t] = 0;
    counters[QUEUE_X + XCDS + t] = sx[t][1023];
  }
  // every thread has read the counts it needs before any is cleared
  __syncthreads();
  int64_t rp = sp[t] - np;
  for (int64_t p = lo; p < hi; ++p) {
    pstart[p] = (int32_t)rp;
    rp += pcount[p];
    pcount[p] = 0;
  }
  atomicAdd(&reads, rd);
  atomicAdd(&set_reads, srd);
  atomicAdd(&products, pd);
  __syncthreads();
  if (t == 0) {
    pstart[N] = (int32_t)sp[1023];
    counters[3] = si[1023];
    counters[4] += (int64_t)reads;
    counters[5] += (int64_t)products;
    counters[9] += (int64_t)set_reads;
  }
}

__global__ __launch_bounds__(256) void k_pair_scatter(const int64_t* __restrict__ counters,
                                                       const int32_t* __restrict__ pair_p,
                                                       const int32_t* __restrict__ pair_pos,
                                                       const int32_t* __restrict__ pair_q,
                                                       const int64_t* __restrict__ pair_base,
                                                       const int32_t* __restrict__ pstart,
                                                       int32_t* __restrict__ sorted, int32_t* __restrict__ sorted_q,
                                                       int64_t* __restrict__ sorted_base) {
  const int64_t npairs = counters[2];
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < npairs; e += (int64_t)gridDim.x * 256) {
    const int32_t pos = pstart[pair_p[e]] + pair_pos[e];
    sorted[pos] = (int32_t)e;
    sorted_q[pos] = pair_q[e];
    sorted_base[pos] = pair_base[e];
  }
}

// The batched work items of the round, two int4 each: (partition, index of
// the item within it, its pairs, its first pair) and (its vectors, first
// tile low and high halves, query sets).  Item `local` of a partition is
// chunk local / sets, query set local % sets.
__global__ __launch_bounds__(256) void k_items(int64_t N, int chunk_tiles, const int32_t* __restrict__ pstart,
                                                const int64_t* __restrict__ pitem,
                                                const int32_t* __restrict__ psize,
                                                const int64_t* __restrict__ poff, const int64_t* __restrict__ pxoff,
                                                const int32_t* __restrict__ pxcd,
                                                const int64_t* __restrict__ counters, int4* __restrict__ bitems,
                                                int64_t* __restrict__ xitem) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= N) return;
  const int np = pstart[p + 1] - pstart[p];
  if (np == 0) return;
  const int sets = (np + SET - 1) / SET;
  const int n = sets * chunks_of(psize[p], chunk_tiles);
  const int64_t tile0 = poff[p];
  const int4 b = make_int4(psize[p], (int)(uint32_t)(uint64_t)tile0, (int)(uint32_t)((uint64_t)tile0 >> 32), sets);
  const int x = pxcd[p];
  int64_t xbase = pxoff[p];
  for (int y = 0; y < x; ++y) xbase += counters[QUEUE_X + XCDS + y];
  for (int local = 0; local < n; ++local) {
    bitems[2 * (pitem[p] + local)] = make_int4((int)p, local, np, pstart[p]);
    bitems[2 * (pitem[p] + local) + 1] = b;
    xitem[xbase + local] = pitem[p] + local;
  }
}

void launch_group(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_pairs, dim3((unsigned)((a.nq + 3) / 4)), dim3(256), 0, s, a.nq, a.M, a.chunk_tiles,
                     ws.cand, st.d_size, ws.st_m, ws.st_weff, ws.st_item, ws.st_pair, ws.pcount, ws.pair_q, ws.pair_p,
                     ws.pair_pos, ws.pair_base);
  hipLaunchKernelGGL(k_part_prefix, dim3(1), dim3(1024), 0, s, st.nlist, a.chunk_tiles, ws.pcount, st.d_size,
                     st.d_order, ws.pstart, ws.pitem, ws.pxoff, ws.pxcd, ws.total);
  // at most wmax pairs per query; the kernel reads this round's count
  const int64_t bound = (a.nq * a.wmax + 255) / 256;
  hipLaunchKernelGGL(k_pair_scatter, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(bound, 2048))), dim3(256),
                     0, s, ws.total, ws.pair_p, ws.pair_pos, ws.pair_q, ws.pair_base, ws.pstart, ws.sorted,
                     ws.sorted_q, ws.sorted_base);
  hipLaunchKernelGGL(k_items, dim3((unsigned)((st.nlist + 255) / 256)), dim3(256), 0, s, st.nlist, a.chunk_tiles,
                     ws.pstart, ws.pitem, st.d_size, st.d_off, ws.pxoff, ws.pxcd, ws.total, ws.bitems, ws.xitem);
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

// FILT: a filtered search - a row is a candidate only when its label bits
// (attr, by slot) share a bit with its query's mask (qmask, by query).
template <int F16, int KS, int IP, int FILT>
__global__ __launch_bounds__(NT, 1) void k_scan_mfma(
    int64_t* __restrict__ counters, const int4* __restrict__ bitems, const int32_t* __restrict__ sorted_q,
    const int64_t* __restrict__ sorted_base, int chunk_tiles, const uint16_t* __restrict__ q16, int dp16,
    const float* __restrict__ qn2f, const uint16_t* __restrict__ v16, const float* __restrict__ v16n,
    const int64_t* __restrict__ sid, const float* __restrict__ rk, const int64_t* __restrict__ ri, int kk,
    float* __restrict__ pk, int64_t* __restrict__ pi, const int64_t* __restrict__ xitem,
    const uint32_t* __restrict__ attr, const uint32_t* __restrict__ qmask) {
  // k-steps per stage: 4 (two for each wave of a pair), else 2 or 1 where
  // that leaves an odd number of stages per tile (a tile always starts in
  // LDS buffer 0; with 1 the pair takes alternate stages); the two stages,
  // the 128 queries' candidate pools and the pairs' exchange fill the LDS
  constexpr int KST = (KS % 8 == 0) ? 4 : ((KS % 4 == 0) ? 2 : 1);
  constexpr int NS = KS / KST;                  // stages per tile
  constexpr int SU = KST * 4 * TILE;            // 16-byte units per stage
  constexpr int UPT = SU >= NT ? SU / NT : 1;   // units each thread carries per stage
  // loads run DEPTH stages (TA whole tiles) ahead of the MFMAs, so that each
  // block keeps 32-128 KiB of the store in flight
  constexpr int TA = NS >= 4 ? 1 : 2;
  constexpr int DEPTH = NS * TA;
  static_assert(KS % KST == 0 && NS % 2 == 0 && (SU % NT == 0 || SU < NT), "stage shape");
  __shared__ u32x4 RING[2][SU];                 // two stages of the current tile
  __shared__ float BK[SET_GROUPS][G][BUF];      // per query: candidates that beat the threshold, not yet merged
  __shared__ uint16_t BS[SET_GROUPS][G][BUF];   // their slots, as offsets from the item's first slot
  __shared__ f32x4 XCH[SET_GROUPS][4][WAVE];    // each wave's half sums of its partner's group, per tile
  // the item a block takes next is published in LDS buffer 1 of the ring:
  // between the last barrier of an item (buffer 1 was read before it) and
  // the first stage of the next (it writes buffer 1 after two barriers) no
  // one touches that buffer
  int64_t* next_item = reinterpret_cast<int64_t*>(&RING[1][0]);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // Blocks take items in order from queues: items differ widely in cost
  // (power-law partition sizes and query counts), so a static split would
  // leave some compute units idle; the query sets of one chunk are
  // consecutive items of one queue, scored at about the same time.  A block
  // takes from the queue of its compute die first (workgroups are dealt to
  // the dies in turn, so block b runs on die b % 8), then from the others.
  // (A block claims its next item only when it is free: claiming ahead
  // keeps large items from idle blocks at the end of a launch.)
  const int64_t total = counters[3];
  unsigned long long* queue = (unsigned long long*)(counters + QUEUE_X);
  int xq = 0;  // queues found empty so far (thread 0's)
  const int x0 = (int)(blockIdx.x & (XCDS - 1));
  constexpr int nc8 = KS * 4;  // 8-element chunks per row of the 16-bit copy
  float (*Bk)[BUF] = BK[wave];
  uint16_t (*Bs)[BUF] = BS[wave];
  // wave pair (2p, 2p + 1): query groups 2p and 2p + 1 of the set; the wave
  // of parity h takes the k-steps of parity h for both groups, and at the
  // end of a tile keeps its own group (group `wave`) and hands the partner
  // group's half sums over
  const int h = wave & 1;
  for (int k = 0;; k ^= 1) {
    // every thread read next_item[k] two items ago, before the barrier that
    // started the last item
    if (threadIdx.x == 0) {
      int64_t got = total;  // none left
      while (xq < XCDS) {
        const int x = (x0 + xq) & (XCDS - 1);
        const int64_t j = (int64_t)atomicAdd(queue + x, 1ull);
        if (j < counters[QUEUE_X + XCDS + x]) {
          int64_t base = 0;
          for (int y = 0; y < x; ++y) base += counters[QUEUE_X + XCDS + y];
          got = xitem[base + j];
          break;
        }
        ++xq;
      }
      next_item[k] = got;
    }
    __syncthreads();
    const int64_t it = next_item[k];
    if (it >= total) break;
    const int4 d0 = bitems[2 * it], d1 = bitems[2 * it + 1];
    const int local = __builtin_amdgcn_readfirstlane(d0.y);
    const int np = __builtin_amdgcn_readfirstlane(d0.z);
    const int pfirst = __builtin_amdgcn_readfirstlane(d0.w);
    const int size = __builtin_amdgcn_readfirstlane(d1.x);
    const int64_t tile0 = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(d1.z) << 32) |
                                    (uint32_t)__builtin_amdgcn_readfirstlane(d1.y));
    const int nsets = __builtin_amdgcn_readfirstlane(d1.w);
    const int tiles = (size + TILE - 1) / TILE;
    // the query set runs fastest, so that the sets of one chunk are scored
    // at about the same time
    const int c = local / nsets, gs = local - (local / nsets) * nsets;
    const int g = gs * SET_GROUPS + wave;
    const int gcount = max(0, min(G, np - g * G));
    const int t0 = c * chunk_tiles;
    const int t1 = min(tiles, t0 + chunk_tiles);
    const int j = lane & (G - 1);
    const bool has = j < gcount;
    const int pidx = has ? pfirst + g * G + j : pfirst;  // a valid pair in every lane
    const int qj = sorted_q[pidx];
    uint32_t qm = 0;
    if constexpr (FILT) qm = qmask[qj];
    // the partner wave's query in this lane's column (row 0 when absent)
    const int gp = g ^ 1;
    const int qp = sorted_q[j < max(0, min(G, np - gp * G)) ? pfirst + gp * G + j : pfirst];
    // slot offsets in the pools are relative to the item's first slot
    const int32_t item_slot0 = (int32_t)((tile0 + t0) * TILE);
    // first output slot of this lane's pair, used only at the item's end
    // (loaded now so that its latency hides behind the scan)
    const int64_t my_base = sorted_base[pidx];
    // Stage u of the item = k-steps [KST (u % NS), +KST) of tile t0 + u / NS:
    // SU contiguous 16-byte units of the store.  The block carries two stages
    // in registers (loads in flight) and one in LDS (being scored).
    const int U = (t1 - t0) * NS;
    // stages past the item's end reload its last stage, and an empty item
    // reads the arena's first tile (never used either)
    const u32x4* src = reinterpret_cast<const u32x4*>(v16) + (U > 0 ? (tile0 + t0) * (int64_t)nc8 * TILE : 0);
    // (with fewer units per stage than threads, the surplus threads load a
    // copy of the last unit and store nothing)
    auto load = [&](int u, u32x4 (&r)[UPT]) {
      u = max(0, min(u, U - 1));
      const u32x4* sp = src + (int64_t)(u / NS) * nc8 * TILE + (int64_t)(u % NS) * SU;
#pragma unroll
      for (int e = 0; e < UPT; ++e) r[e] = sp[min(e * NT + (int)threadIdx.x, SU - 1)];
    };
    auto put = [&](const u32x4 (&r)[UPT], int buf) {
#pragma unroll
      for (int e = 0; e < UPT; ++e)
        if (SU >= NT || (int)threadIdx.x < SU) RING[buf][e * NT + threadIdx.x] = r[e];
    };
    // registers: stage u (u >= 1) waits in slot (u - 1) % DEPTH until it is
    // moved to LDS buffer u % 2 at the end of stage u - 1; the first stages
    // are requested before the queries so that both arrive together
    u32x4 rs[DEPTH][UPT];
    u32x4 first[UPT];
    load(0, first);
#pragma unroll
    for (int d = 1; d <= DEPTH; ++d) load(d, rs[d - 1]);
    // Loads in this kernel are unconditional (clamped to valid addresses
    // and the result discarded where unused): a load under a branch leaves
    // the compiler unsure how many loads are in flight, and it then waits
    // for all of them - which would drain the prefetch pipeline below.
    // B fragments of the k-steps of this wave's parity, for its own group
    // (breg[0]) and its partner's (breg[1]); columns of absent queries score
    // row 0 and are never read
    u32x4 breg[2][KS / 2];
#pragma unroll
    for (int i = 0; i < KS / 2; ++i) {
      const int s = 2 * i + h;  // k-step of breg[.][i]
      breg[0][i] = *reinterpret_cast<const u32x4*>(q16 + (int64_t)qj * dp16 + 32 * s + 8 * (lane >> 4));
      breg[1][i] = *reinterpret_cast<const u32x4*>(q16 + (int64_t)qp * dp16 + 32 * s + 8 * (lane >> 4));
    }
    const float qn2_row = qn2f[qj];
    const float my_qn2 = (IP || !has) ? 0.f : qn2_row;
    // Per query j of the wave: an unsorted pool of candidates in LDS
    // (Bk[j] / Bs[j], cn of them) and - held by the four lanes whose MFMA
    // output column is j (lanes j, j + 16, j + 32, j + 48) - the key tk a
    // candidate must not exceed: the seed from the query's committed
    // results, then the cut key of the pool whenever the pool is cut.  A
    // candidate that ties tk is taken whatever its slot; when it ranks after
    // the kk best in (key, slot) order, the final selection (or the commit)
    // drops it.
    float tk;
    int cn = 0;
    tk = rk[(int64_t)qj * kk + kk - 1];
    // Cut the pools of up to NB queries (jq[q] < 0: none) that hold more
    // than `limit` entries (limit >= kk) down to at most `limit`, all of
    // them at or below a key T that at least kk entries reach; T becomes the
    // query's tk.  T is found by bisection on the keys' order-preserving
    // bits between the pool's smallest and largest key, with ballot counts,
    // stopping as soon as the count lands in [kk, limit]; the NB bisections
    // run interleaved.  When ties at T leave more than `limit`, keep exactly
    // the kk best in (key, slot) order, bisecting on the slot among the ties.
    constexpr int EPL = BUF / WAVE;  // pool entries per lane
    auto cut = [&](auto nb_tag, const int* jq, int limit) {
      constexpr int NB = decltype(nb_tag)::value;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      int n[NB];
      bool act[NB], any = false;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        n[q] = jq[q] >= 0 ? __builtin_amdgcn_readlane(cn, jq[q]) : 0;
        act[q] = n[q] > limit;
        any |= act[q];
      }
      if (!any) return;
      float kv[NB][EPL];
      int32_t sv[NB][EPL];
      uint32_t uv[NB][EPL];
      uint32_t lo[NB], hi[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const bool v = act[q] && e * WAVE + lane < n[q];
          const int jj = act[q] ? jq[q] : 0;
          kv[q][e] = v ? Bk[jj][e * WAVE + lane] : KEY_EMPTY;
          sv[q][e] = v ? (int32_t)Bs[jj][e * WAVE + lane] : INT32_MAX;
          uv[q][e] = v ? float_order(kv[q][e]) : 0xffffffffu;
          mn = min(mn, uv[q][e]);
          mx = max(mx, v ? uv[q][e] : 0u);
        }
        lo[q] = wave_min_u32(mn);
        hi[q] = wave_max_u32(mx);
      }
      auto count_le = [&](int q, uint32_t x) {
        int c = 0;
#pragma unroll
        for (int e = 0; e < EPL; ++e) c += __popcll(__ballot(uv[q][e] <= x));
        return c;
      };
      // invariant: at least kk entries are <= hi[q], fewer than kk < lo[q]
      bool done[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) done[q] = !act[q] || lo[q] >= hi[q];
      for (;;) {
        bool all = true;
#pragma unroll
        for (int q = 0; q < NB; ++q) all &= done[q];
        if (all) break;
        int c[NB];
        uint32_t mid[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          mid[q] = lo[q] + ((hi[q] - lo[q]) >> 1);
          c[q] = count_le(q, mid[q]);
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (done[q]) continue;
          if (c[q] >= kk) {
            hi[q] = mid[q];
            done[q] = c[q] <= limit;
          } else {
            lo[q] = mid[q] + 1;
          }
          done[q] |= lo[q] >= hi[q];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (!act[q]) continue;
        const uint32_t T = hi[q];
        int32_t slo = INT32_MAX;
        // many ties at T can leave more than `limit` entries: cut exactly then
        if (count_le(q, T) > limit) {
          int less = 0, eq = 0;
#pragma unroll
          for (int e = 0; e < EPL; ++e) {
            less += __popcll(__ballot(uv[q][e] < T));
            eq += __popcll(__ballot(uv[q][e] == T));
          }
          const int need = kk - less;
          if (eq > need) {
            int32_t a = 0, b = INT32_MAX;
            while (a < b) {
              const int32_t mid = a + ((b - a) >> 1);
              int c = 0;
#pragma unroll
              for (int e = 0; e < EPL; ++e) c += __popcll(__ballot(uv[q][e] == T && sv[q][e] <= mid));
              if (c >= need) b = mid; else a = mid + 1;
            }
            slo = a;
          }
        }
        const int jj = jq[q];
        int base = 0;
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
          const bool keep = uv[q][e] < T || (uv[q][e] == T && sv[q][e] <= slo);
          const uint64_t m = __ballot(keep);
          const int p = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
          if (keep) { Bk[jj][p] = kv[q][e]; Bs[jj][p] = (uint16_t)sv[q][e]; }
          base += __popcll(m);
        }
        if (j == jj) {
          cn = base;
          tk = float_from_order(T);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    };
    put(first, 0);
    __syncthreads();
    // A fragments of one k-step: vectors 16b + (lane & 15), 16-byte chunk
    // 4s + (lane >> 4) of the stage
    const int frag = (lane >> 4) * TILE + (lane & 15);
    f32x4 acc[2][4];
#pragma unroll
    for (int gi = 0; gi < 2; ++gi)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[gi][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Ids (and norms) of a tile are loaded one tile ahead: the wait for them
    // at the tile's end then covers only loads issued before them, not the
    // stage prefetches issued since (an empty item reads the arena's first
    // tile, never used).
    int64_t next_id;
    float next_xn = 0.f;
    uint32_t next_attr = 0;
    {
      const int64_t tn = (U > 0 ? tile0 + t0 : 0) * TILE + lane;
      next_id = sid[tn];
      if (!IP) next_xn = v16n[tn];
      if constexpr (FILT) next_attr = attr[tn];
    }
    for (int tb = t0; tb < t1; tb += TA) {
#pragma unroll
    for (int ta = 0; ta < TA; ++ta) {
      const int t = tb + ta;
      if (t >= t1) break;
      // this tile's ids and norms (loaded during the previous tile); the
      // next tile's are requested now (the last tile requests itself again)
      const int64_t tile_id = next_id;
      const float tile_xn = next_xn;
      const uint32_t tile_attr = next_attr;
      {
        const int64_t tn = (tile0 + min(t + 1, t1 - 1)) * TILE + lane;
        next_id = sid[tn];
        if (!IP) next_xn = v16n[tn];
        if constexpr (FILT) next_attr = attr[tn];
      }
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        const int u = (t - t0) * NS + st;
        const int slot = ta * NS + st;  // u % DEPTH
        // (groups without queries score too - their results are never read -
        // so that the accumulators stay in the matrix registers throughout)
        auto kstep = [&](int s, int i) {
          u32x4 a[4];
#pragma unroll
          for (int b = 0; b < 4; ++b) a[b] = RING[st & 1][4 * s * TILE + frag + 16 * b];
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[0][b] = mfma16<F16>(a[b], breg[0][i], acc[0][b]);
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[1][b] = mfma16<F16>(a[b], breg[1][i], acc[1][b]);
        };
        if constexpr (KST == 4) {
          kstep(h, 2 * st);        // k-steps 4 st + h and 4 st + 2 + h of the tile
          kstep(2 + h, 2 * st + 1);
        } else if constexpr (KST == 2) {
          kstep(h, st);            // k-step 2 st + h of the tile
        } else if ((st & 1) == h) {
          kstep(0, st >> 1);       // k-step st, of this wave's parity
        }
        if (st == NS - 1) {
          // the partner group's half sums go to the partner (read after the
          // barrier below)
#pragma unroll
          for (int b = 0; b < 4; ++b) XCH[wave][b][lane] = acc[1][b];
        }
        // the other LDS buffer was last read in stage u - 1 (before the last
        // barrier): it takes stage u + 1, whose registers then load stage
        // u + 1 + DEPTH (after the last stage, the copy is never read)
        put(rs[slot], (st + 1) & 1);
        load(u + 1 + DEPTH, rs[slot]);
        __syncthreads();
      }
      // the own group's sums: even k-steps plus odd k-steps (in that order
      // on both waves of the pair, so the two halves add up identically)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const f32x4 other = XCH[wave ^ 1][b][lane];
        acc[0][b] = h == 0 ? acc[0][b] + other : other + acc[0][b];
        acc[1][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      if (gcount == 0) {
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[0][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        continue;
      }
      {
        // The tile's scores are complete.  acc[0][b][v] is the product of
        // query j = lane & 15 with vector 16b + 4 (lane >> 4) + v of the
        // tile, so every lane tests its 16 values against its query's
        // threshold in registers; most tiles end here with nothing to keep.
        const uint64_t live = __ballot(t * TILE + lane < size && tile_id >= 0);
        const int32_t slot0 = (int32_t)((t - t0) * TILE);  // relative to the item's first slot
        float key[16];
        // live bits of this lane's 16 vectors (bit 4b + v: vector 16b + 4g + v);
        // absent queries take nothing
        const int g4 = lane >> 4;
        uint32_t lm = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) lm |= (uint32_t)((live >> (16 * b + 4 * g4)) & 0xfull) << (4 * b);
        if constexpr (FILT) {
          // rows whose labels miss the query's mask are never candidates
          uint32_t fm = 0;
#pragma unroll
          for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              fm |= ((__shfl(tile_attr, 16 * b + 4 * g4 + v) & qm) != 0u ? 1u : 0u) << (4 * b + v);
          lm &= fm;
        }
        if (!has) lm = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int vi = 16 * b + 4 * (lane >> 4) + v;
            const float dot = acc[0][b][v];
            key[4 * b + v] = IP ? -dot : (my_qn2 + __shfl(tile_xn, vi) - 2.f * dot);
          }
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[0][b] = f32x4{0.f, 0.f, 0.f, 0.f};
        // bit e: value e is live and at or below the query's threshold
        auto pass_bits = [&]() {
          uint32_t m = 0;
#pragma unroll
          for (int e = 0; e < 16; ++e) m |= (key[e] <= tk ? 1u : 0u) << e;
          return m & lm;
        };
        // nothing at or below the threshold in the whole wave: the usual case
        float kmin = fminf(fminf(fminf(key[0], key[1]), fminf(key[2], key[3])),
                           fminf(fminf(key[4], key[5]), fminf(key[6], key[7])));
        kmin = fminf(kmin, fminf(fminf(fminf(key[8], key[9]), fminf(key[10], key[11])),
                                 fminf(fminf(key[12], key[13]), fminf(key[14], key[15]))));
        uint32_t pm = 0;
        if (__ballot(kmin <= tk && lm != 0)) pm = pass_bits();
        if (__ballot(pm != 0)) {
          // passes of the query over its four lanes, and this lane's offset
          auto totals = [&](int n, int& tot, int& off) {
            const int n0 = __shfl(n, j), n1 = __shfl(n, j + 16), n2 = __shfl(n, j + 32), n3 = __shfl(n, j + 48);
            tot = n0 + n1 + n2 + n3;
            off = (g4 > 0 ? n0 : 0) + (g4 > 1 ? n1 : 0) + (g4 > 2 ? n2 : 0);
          };
          int tot, off;
          totals(__popc(pm), tot, off);
          // queries whose pool would overflow are cut first, two at a time
          uint64_t over = __ballot(lane < G && cn + tot > BUF);
          if (over) {
            const int keep = kk + min(SLACK, BUF - WAVE - kk);
            while (over) {
              int jq[2];
              jq[0] = __builtin_ctzll(over);
              over &= over - 1;
              jq[1] = over ? __builtin_ctzll(over) : -1;
              if (over) over &= over - 1;
              cut(std::integral_constant<int, 2>{}, jq, keep);
            }
            pm = pass_bits();
            totals(__popc(pm), tot, off);
          }
          int pos = cn + off;
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            if ((pm >> e) & 1u) {
              Bk[j][pos] = key[e];
              Bs[j][pos] = (uint16_t)(slot0 + 16 * (e >> 2) + 4 * g4 + (e & 3));
              ++pos;
            }
          }
          cn += tot;
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
      }
    }
    }
    // The item's kk best per query, sorted: pools cut to at most 64 entries
    // (still holding the kk best), four queries at a time, then sorted FB
    // queries at a time (their shuffles overlap).
    if (gcount > 0) {
#pragma unroll
      for (int q0 = 0; q0 < G; q0 += 4) {
        if (q0 >= gcount) break;
        int jq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) jq[q] = q0 + q < gcount ? q0 + q : -1;
        cut(std::integral_constant<int, 4>{}, jq, WAVE);
      }
      constexpr int FB = 8;
#pragma unroll
      for (int q0 = 0; q0 < G; q0 += FB) {
        if (q0 >= gcount) break;
        uint64_t bv[FB];
#pragma unroll
        for (int q = 0; q < FB; ++q) {
          const int n = __builtin_amdgcn_readlane(cn, q0 + q);
          bv[q] = pack_key_slot(lane < n ? Bk[q0 + q][lane] : KEY_EMPTY,
                                lane < n ? item_slot0 + (int32_t)Bs[q0 + q][lane] : -1);
        }
        wave_sort64_packed_n<FB>(bv);
#pragma unroll
        for (int q = 0; q < FB; ++q) {
          if (q0 + q >= gcount) break;
          const int64_t out = (readlane_i64(my_base, q0 + q) + c) * kk;
          if (lane < kk) {
            pk[out + lane] = packed_key(bv[q]);
            pi[out + lane] = (int64_t)packed_slot(bv[q]);
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
  }
}

template <int F16, int IP, int FILT>
static void scan_mfma_k(Workspace& ws, const Store& st, const RoundArgs& a, int blocks, hipStream_t s) {
  const int ks = st.dp16 / 32;
#define QK_MFMA_LAUNCH(KS)                                                                                      \
  hipLaunchKernelGGL((k_scan_mfma<F16, KS, IP, FILT>), dim3(blocks), dim3(NT), 0, s, ws.total, ws.bitems,     \
                     ws.sorted_q, ws.sorted_base, a.chunk_tiles, ws.q16, st.dp16, ws.qn2f, st.v16, st.v16n, st.ids, \
                     ws.rk, ws.ri, a.kk, ws.pk, ws.pi, ws.xitem, a.attr, a.qmask)
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
  if (a.qmask) {
    if (f16) { if (ip) scan_mfma_k<1, 1, 1>(ws, st, a, blocks, s); else scan_mfma_k<1, 0, 1>(ws, st, a, blocks, s); }
    else { if (ip) scan_mfma_k<0, 1, 1>(ws, st, a, blocks, s); else scan_mfma_k<0, 0, 1>(ws, st, a, blocks, s); }
  } else {
    if (f16) { if (ip) scan_mfma_k<1, 1, 0>(ws, st, a, blocks, s); else scan_mfma_k<1, 0, 0>(ws, st, a, blocks, s); }
    else { if (ip) scan_mfma_k<0, 1, 0>(ws, st, a, blocks, s); else scan_mfma_k<0, 0, 0>(ws, st, a, blocks, s); }
  }
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

// Host-side index state, device memory accounting and kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "quake.h"

namespace qk {

struct Error {
  int code;
  std::string msg;
};

#define QK_HIP(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::qk::Error{QUAKE_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define QK_CHECK(cond, code, msg) \
  do {                            \
    if (!(cond)) throw ::qk::Error{code, std::string(msg)}; \
  } while (0)

constexpr int TILE = 64;          // vectors per store tile: one per lane of a wave
constexpr int KMAX = 256;         // largest result list of the wave-list scans
constexpr int KMAX_LARGE = 1024;  // largest result list at all (upper level of two levels)
constexpr int SORTED_ITEM_MAX = 1024;  // vectors per item of the sort-based scan (16 tiles)
constexpr int CAP_TABLE_POINTS = 1024;
// the device table holds the points, then a = (d + 1) / 2 and log B(a, 1/2)
// for the direct evaluation of the cap share
constexpr int CAP_TABLE_SIZE = CAP_TABLE_POINTS + 2;

// Row length of the 16-bit store copy: d rounded up to 32 * KS for a k-step
// count KS the MFMA scan is compiled for (2, 4, 8, 12, 16, 24 or 32).
inline int padded_dim16(int d) {
  const int need = (d + 31) / 32;
  for (int ks : {2, 4, 8, 12, 16, 24, 32})
    if (ks >= need) return 32 * ks;
  return 32 * need;
}
constexpr int MAX_DIM = 4096;
constexpr int PQ_MAX_SUB = 32;    // dimensions per product-quantization subspace
// 32-bit words per slot of the product-code array: the codes of pq_m
// subspaces, four per word, then the slot's FP32 residual term
inline int pq_words(int pq_m) { return pq_m / 4 + 1; }
constexpr int COUNTERS = 32;      // device counters of a search (Workspace::total)
constexpr int MAX_CANDIDATES = 4096;   // APS candidate set M (and nprobe) upper bound

// Device allocations of one index, counted against an optional budget.
// Blocks come from the caller's allocator when one is set (torch's caching
// allocator from the Python binding), else from hipMalloc.  Thread-safe.
class DeviceMemory {
 public:
  size_t used = 0;
  size_t budget = 0;  // 0 = unlimited
  quake_allocator user{};  // user.alloc == nullptr: hipMalloc / hipFree
  bool forbid = false;     // set for the duration of a call that must allocate nothing
  template <class T>
  T* alloc(size_t count) { return static_cast<T*>(raw_alloc(count * sizeof(T))); }
  void* raw_alloc(size_t bytes);
  void release(void* p);
  ~DeviceMemory();

 private:
  struct Block { void* p; size_t bytes; };
  std::vector<Block> blocks_;
  std::mutex mu_;  // the serving loop's update thread allocates beside its search thread
};

// One level's partitions.  Vectors of partition p occupy tiles
// [off[p], off[p] + cap[p]/64) of the arena; the first size[p] slots are
// filled.  Within a tile, FP32 data is laid out [dp/4][64 lanes][4] and the
// 16-bit copy [dp/8][64 lanes][8], so that a wave reading one 16-byte chunk
// of 64 consecutive vectors touches one contiguous 1 KiB span.
// id -> slot map (level 0): open addressing, capacity a power of two.
struct IdMap {
  int64_t* keys = nullptr;
  int64_t* vals = nullptr;
  uint64_t mask = 0;            // capacity - 1
  int64_t used = 0;             // live + erased entries
};

struct Store {
  int32_t d = 0, dp = 0;
  int64_t nlist = 0;
  float* centroids = nullptr;   // [nlist][dp]
  int64_t* d_off = nullptr;     // [nlist] first tile of each partition
  int32_t* d_size = nullptr;    // [nlist] filled slots (deleted slots hold id -1)
  int32_t* d_cap = nullptr;     // [nlist] slots (multiple of 64)
  int32_t* d_order = nullptr;   // [nlist] partitions by decreasing size (ties by index)
  std::vector<int64_t> off;
  std::vector<int32_t> size, cap;
  std::vector<int32_t> order;    // host copy of d_order
  int64_t tiles = 0;            // arena tiles allocated
  int64_t used_tiles = 0;       // arena tiles handed out
  int32_t dp16 = 0;             // row length of the 16-bit copy: d rounded up to 32
  float* v32 = nullptr;         // FP32 tiles [dp/4][64][4] (null when the index keeps only the 16-bit tiles)
  uint16_t* v16 = nullptr;      // BF16 or FP16 copy, or null; tiles [dp16/8][64][8]
  float* v16n = nullptr;        // [tiles * 64] |x|^2 of the 16-bit copy (L2 only)
  float* rows32 = nullptr;      // [tiles * 64][dp] row-major FP32 rows by slot (with a 16-bit copy: rerank)
  int64_t* ids = nullptr;       // [tiles * 64], -1 = empty or deleted
  uint32_t* attr = nullptr;     // [tiles * 64] label bits of every slot (level 0 of a labelled index), or null
  uint32_t* d_attr_cnt = nullptr;  // [nlist][33]: live rows carrying each label bit, then live rows
  int32_t pq_m = 0;             // subspaces of the product-quantized copy (level 0), 0 = none
  uint32_t* codes = nullptr;    // [tiles][pq_words(pq_m)][64]: four one-byte codes of a slot per word, then
                                // its residual term |r^|^2 + 2 <c, r^> (FP32 bits), or null
  mutable bool attr_dirty = true;  // d_attr_cnt must be recounted before the next filtered search
  int64_t live = 0;
  std::vector<int32_t> tomb;     // deleted slots still inside size[p]
  std::vector<int32_t> tile_part;  // partition owning each arena tile (-1 = unused)
  uint32_t* d_hits = nullptr;   // [nlist] queries that scanned each partition since the counters were cleared
  mutable int64_t window = 0;   // queries searched since then (searches take the store const)
};

struct Workspace {
  int64_t nq_cap = 0, scores_cap = 0, cand_cap = 0, k_cap = 0, items_cap = 0, kk_cap = 0;
  float* q = nullptr;           // [nq][dp] queries, zero padded
  double* qn2 = nullptr;        // [nq] |q|^2
  float* scores = nullptr;      // [nq][ncent]
  int32_t* sel = nullptr;       // [nq][M] nearest centroids by (value, id)
  int32_t* cand = nullptr;      // [nq][M] candidate partitions in scan order
  int32_t* mq = nullptr;        // [nq] candidates of each query (M, or fewer below a two-level index)
  int32_t* cand0 = nullptr;     // [nq][M0] level-0 candidates found by the level-1 search
  int32_t* mq0 = nullptr;       // [nq] their number
  int64_t cand0_cap = 0;
  int32_t* cand1 = nullptr;     // [nq][M1] level-1 candidates found by the level-2 search (three levels)
  int32_t* mq1 = nullptr;       // [nq] their number
  int64_t cand1_cap = 0, mq1_cap = 0;
  float* h = nullptr;           // [nq][M] bisector distances in scan order
  float* lut = nullptr;         // [nq][pq_m][256] per-query code tables of a search over product codes
  int64_t lut_cap = 0;
  int32_t* st_m = nullptr;      // committed partitions
  int32_t* st_w = nullptr;      // window the query asks for in the next round
  int32_t* st_weff = nullptr;   // window it got in the current round
  int32_t* st_done = nullptr;
  int64_t* st_item = nullptr;   // first work item of the round
  int64_t* st_demand = nullptr;
  double* st_rho = nullptr;
  double* st_p0 = nullptr;
  double* st_V = nullptr;
  double* st_vsum = nullptr;
  double* st_r = nullptr;
  float* rk = nullptr;          // [nq][kk] committed results
  int64_t* ri = nullptr;
  int4* items = nullptr;        // (query, partition, first tile, end tile)
  float* pk = nullptr;          // [items][kk] partial results
  int64_t* pi = nullptr;
  int64_t* st_vecs = nullptr;   // [nq] vectors in the round's window
  int64_t* st_pair = nullptr;   // [nq] first (query, partition) pair of the round
  uint16_t* q16 = nullptr;      // [nq][dp16] queries rounded to the 16-bit store type
  int q16_dim = 0;
  float* qn2f = nullptr;        // [nq] |q|^2
  int64_t pairs_cap = 0, parts_cap = 0;
  int32_t* pair_q = nullptr;    // [pairs] query of the pair
  int32_t* pair_p = nullptr;    // [pairs] partition of the pair
  int32_t* pair_pos = nullptr;  // [pairs] place among the partition's pairs
  int64_t* pair_base = nullptr; // [pairs] first partial-list slot of the pair
  int32_t* sorted = nullptr;    // [pairs] pairs in partition order
  int32_t* sorted_q = nullptr;  // [pairs] their queries
  int64_t* sorted_base = nullptr;  // [pairs] their first partial-list slots
  int4* bitems = nullptr;       // [items][2] batched work items: (partition, index in it, pairs, first pair),
                                //   (vectors, first tile low, first tile high, query sets)
  int32_t* pcount = nullptr;    // [nlist] pairs per partition (kept zeroed between rounds)
  int32_t* pstart = nullptr;    // [nlist + 1]
  int64_t* pitem = nullptr;     // [nlist] first batched work item of each partition (numbered in Store::order)
  int64_t* pxoff = nullptr;     // [nlist] first place of each partition's items in its compute die's queue
  int32_t* pxcd = nullptr;      // [nlist] that queue (partitions of size rank r: queue r % 8)
  int64_t* xitem = nullptr;     // [items] batched items in the order the eight queues hand them out
  // device counters (COUNTERS of them): [0] items, [1] vectors, [2] pairs of
  // the round, [3] batched items of the round, [4] batched distinct vector
  // reads (each touched partition once per round) and [5] batched
  // query-vector products summed over the search, [6] plain-scan vectors
  // summed over the search, [7] head of the round's item queue, [8] first
  // query cut from the round, [9] batched vector reads counted once per
  // query set, [16, 24) heads of the batched scan's eight item queues,
  // [24, 32) their lengths
  int64_t* total = nullptr;
  int64_t* blk = nullptr;       // [nq / 256 + 1][4] per-block planning sums, then offsets
  int64_t* h_total = nullptr;   // pinned host mirror
};

// HIP-event timing of kernel classes on the search stream.
struct Profiler {
  bool on = false;
  quake_kernel_profile acc[QUAKE_PROF_KINDS] = {};
  struct Span { int kind; hipEvent_t a, b; };
  std::vector<Span> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t event();
  void begin(int kind, hipStream_t s);
  void end(hipStream_t s);
  int only = -1;  // >= 0: every span and count goes to this kind (the level-1 search)
  void add(int kind, double bytes, double flops) {
    if (only >= 0) kind = only;
    if (on) { acc[kind].bytes += bytes; acc[kind].flops += flops; }
  }
  void collect();  // after the stream is synchronised
  ~Profiler();
};

struct ProfileScope {
  Profiler& p;
  hipStream_t s;
  ProfileScope(Profiler& p_, int kind, hipStream_t s_) : p(p_), s(s_) { p.begin(kind, s); }
  ~ProfileScope() { p.end(s); }
};

}  // namespace qk

struct quake_index {
  uint32_t magic = 0x51554b45u;
  int32_t metric = QUAKE_L2;
  int32_t storage = QUAKE_F32;
  int32_t n_levels = 1;
  int32_t d = 0, dp = 0;
  qk::DeviceMemory mem;
  qk::Store L0;                 // level 0: the vectors
  qk::Store L1;                 // level 1 (two or three levels): the level-0 centroids
  qk::Store L2;                 // level 2 (three levels): the level-1 centroids
  qk::IdMap idmap;              // level-0 ids
  int32_t* top_of = nullptr;    // [L0.nlist] level-1 partition of each level-0 centroid
  int32_t* top_of2 = nullptr;   // [L1.nlist] level-2 partition of each level-1 centroid
  double* cap_table = nullptr;  // [1024] device copy of the recall model table
  uint32_t* d_flag = nullptr;   // input checks: set by kernels that find a bad value
  uint32_t* h_flag = nullptr;   // pinned host mirror
  std::vector<double> h_cap_table;
  qk::Workspace ws;
  qk::Profiler prof;
  quake_tuning tune{};
  double slack = 0.0;           // capacity_slack of the build (kept for save / load)
  bool labelled = false;        // level-0 rows carry label bits (filtered searches)
  int32_t pq_m = 0, pq_ds = 0;  // product quantization: subspaces and dimensions per subspace (0 = none)
  float* pq_book = nullptr;     // [pq_m][256][pq_ds] codebook of level 0's codes
  int cu_count = 0;
  // captured scan rounds, keyed by every argument their kernels take
  struct Graph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<Graph> graphs;
  hipStream_t capture_stream = nullptr;
  bool graphs_failed = false;
  bool noalloc = false;         // inside quake_search_noalloc: launch rounds directly, allocate nothing
  bool count_access = true;     // searches add to the access statistics (off while the autotuner runs)
  ~quake_index();  // graphs, streams and pinned buffers; device memory goes with `mem`
};

namespace qk {

// cap_table.cpp
void cap_fraction_table(int d, double* out /*[CAP_TABLE_POINTS]*/);
// the table, then a = (d + 1) / 2 and log B(a, 1/2): the device copy
void cap_model_table(int d, double* out /*[CAP_TABLE_SIZE]*/);
double cap_fraction(double t, int d);

// kernels: centroids and candidates (k_centroids.hip)
// Rows [n][d] to [n][dp] (zero padded), optionally |row|^2 in FP64; `bad`
// (when given) is set non-zero if any value read is not finite.
void launch_pad_rows(const float* x, int64_t n, int d, int dp, float* out, double* norm2, hipStream_t s,
                     uint32_t* bad = nullptr);
// Sets *bad non-zero if any of x[0, n) is not finite (caller clears it).
void launch_nonfinite(const float* x, int64_t n, uint32_t* bad, hipStream_t s);
// Sets *bad non-zero if any of a[0, n) lies outside [0, nlist) (caller clears it).
void launch_check_range(const int32_t* a, int64_t n, int64_t nlist, uint32_t* bad, hipStream_t s);
void launch_scores(const float* q, int64_t nq, const float* c, int64_t nc, int dp, int metric, float* out,
                   hipStream_t s);
void launch_select(const float* scores, int64_t nq, int64_t nc, int M, int metric, int32_t* cand,
                   hipStream_t s);
void launch_geometry(const float* q, const float* c, int64_t nq, int dp, int M, const int32_t* mq, int metric,
                     const int32_t* sel, int32_t* order, float* h, hipStream_t s);
// The M best centroids per query and, in adaptive mode, their scan order and
// bisector distances (one fused wave per query for M <= 64 and d <= 1024,
// else k_select + k_geometry; mq must hold M for the latter).
void launch_candidates(const Store& st, const float* q, const float* scores, int64_t nq, int dp, int M, int aps,
                       int metric, const int32_t* mq, int32_t* sel, int32_t* cand, float* h, hipStream_t s);
void launch_assign(const float* x, int64_t n, int dp, const float* c, int64_t nc, int metric, int32_t* assign,
                   hipStream_t s);
void launch_absmax(const float* x, int64_t n, uint32_t* out, hipStream_t s);
void launch_kmeans_accumulate(const float* x, int64_t n, int dp, const int32_t* assign, int frac_bits, int64_t* sums,
                              int32_t* counts, hipStream_t s);
void launch_kmeans_update(const int64_t* sums, const int32_t* counts, int64_t nc, int dp, int normalise,
                          int frac_bits, float* c, hipStream_t s);
void launch_normalise_rows(float* c, int64_t n, int dp, hipStream_t s);
void launch_gather_rows(const float* x, int d, const int64_t* rows, int64_t nr, int dp, float* out,
                        hipStream_t s);

// kernels: store (k_store.hip)
void launch_scatter(const float* x, int64_t n, int d, int dp, int dp16, const int64_t* ids, const int64_t* slot,
                    float* v32, uint16_t* v16, int dtype16, float* rows32, int64_t* sid, hipStream_t s);
void launch_export(const Store& st, int64_t* ids, int32_t* part, const int64_t* part_first_out,
                   hipStream_t s);

// kernels: the scan rounds (k_scan.hip)
struct RoundArgs {
  int64_t nq;
  int M;             // candidates per query
  int k;             // results returned
  int kk;            // results kept per query while scanning (k, or the rerank pool)
  int aps;           // 1: adaptive; 0: fixed nprobe
  int chunk_tiles;   // tiles per work item
  int wmax;
  int wscale;        // predicted windows are scaled by this percentage (>= 100)
  int metric;
  int dim;           // d, for nothing but documentation of the table
  double tau_r, tau_rho;
  int est;           // recall estimator variant (QUAKE_EST_*)
  const uint32_t* qmask;     // filtered search: label mask of every query (device [nq]), or null
  const uint32_t* attr;      // with qmask: label bits of every slot
  const uint32_t* attr_cnt;  // with qmask: [nlist][33] per-bit and live counts
  int64_t items_cap;
  int blocks;        // grid of the persistent scan kernels (they read their item counts on the device)
  int slot_ids;      // 1: the lists carry store slots below 2^31 (batched path), not ids
  uint32_t* hits;    // per-partition access counts the commit adds to, or null
  const uint8_t* slot_tag;  // serving: store tag of every query slot, or null (all queries take part)
  int tag;           // with slot_tag: the tag of the store this round scans
};
void launch_round_init(Workspace& ws, const RoundArgs& a, int w0, hipStream_t s);
void launch_demand(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s);
void launch_emit(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s);
void launch_scan_f32(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s);
// Product quantization: subspace columns of sampled rows, codes at store
// slots, per-query tables, the scan over codes, and codes by slot.
void launch_pq_subspace(const float* x, int64_t nr, int d, const int64_t* rows, const int32_t* part, const float* C,
                        int dp, int col0, int ds, int dsp, float* out, hipStream_t s);
void launch_pq_encode(const float* rows32, int dp, const int64_t* slot, const int32_t* part, int64_t n,
                      const float* C, const float* book, int M, int ds, int metric, uint32_t* codes, hipStream_t s);
void launch_pq_lut(const float* q, int64_t nq, int dp, const float* book, int M, int ds, int metric, float* lut,
                   hipStream_t s);
void launch_scan_pq(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s);
void launch_pq_export(const Store& st, const int64_t* slots, int64_t n, uint8_t* out, hipStream_t s);
void launch_commit(Workspace& ws, const Store& st, const RoundArgs& a, const double* table, hipStream_t s);
void launch_finalize(Workspace& ws, const RoundArgs& a, int64_t* out_ids, float* out_dist,
                     int32_t* out_nscanned, double* out_recall, hipStream_t s);

// kernels: the batched scan (k_batched.hip)
void launch_queries16(Workspace& ws, int64_t nq, int dp, int dp16, int dtype16, hipStream_t s,
                      const int32_t* slots = nullptr);
void launch_group(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s);
void launch_scan_mfma(Workspace& ws, const Store& st, const RoundArgs& a, int dtype16, hipStream_t s);
// exact = false: no FP32 re-scoring, only the slot -> id mapping and the best k by the 16-bit values.
void launch_rerank(Workspace& ws, const Store& st, const RoundArgs& a, hipStream_t s, bool exact,
                   const int32_t* slots = nullptr,
                   int64_t nslots = 0);
void launch_norm16(const Store& st, int dtype16, hipStream_t s);

// kernels: updates (k_update.hip)
void launch_map_insert(IdMap& m, const int64_t* ids, const int64_t* slots, int64_t n, hipStream_t s);
void launch_map_insert_store(IdMap& m, const int64_t* sid, int64_t slots, hipStream_t s);
void launch_map_find(const IdMap& m, const int64_t* ids, int64_t n, int64_t* slots, int64_t* missing, hipStream_t s);
void launch_map_erase(IdMap& m, const int64_t* ids, int64_t n, hipStream_t s);
void launch_map_update(IdMap& m, const int64_t* ids, const int64_t* slots, int64_t n, hipStream_t s);
void launch_mark_deleted(Store& st, const int64_t* slots, int64_t n, hipStream_t s);
void launch_move_slots(Store& st, const int64_t* src, const int64_t* dst, int64_t n, hipStream_t s);
// dst[slot[i]] = src[i] for i < n (label bits of placed rows)
void launch_put_u32(const uint32_t* src, const int64_t* slot, int64_t n, uint32_t* dst, hipStream_t s);
// d_attr_cnt from the label bits of every live slot
void launch_attr_counts(const Store& st, hipStream_t s);
void launch_norm16_slots(Store& st, const int64_t* slots, int64_t n, int dtype16, hipStream_t s);
void launch_level1_to_candidates(int64_t nq, int M0, int kk, const int64_t* ri, int32_t* cand0, int32_t* mq,
                                 hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

// kernels: maintenance (k_maintain.hip)
// out[i] = the FP32 vector in store slot slots[i], row-major [n][dp].
void launch_gather_slots(const Store& st, const int64_t* slots, int64_t n, float* out, hipStream_t s);
// far[s] = the row of [lo[s], lo[s+1]) farthest from ref[s] (largest squared
// distance, or smallest inner product; ties to the lower row).
void launch_seg_farthest(const float* x, const int64_t* lo, int64_t nseg, const float* ref, int dp, int metric,
                         int64_t* far, hipStream_t s);
// lab[i] = 2 seg[i] + (1 if row i is strictly nearer to c[2 seg + 1] than to c[2 seg]).
void launch_seg_assign2(const float* x, int64_t n, const int32_t* seg, const float* c, int dp, int metric,
                        int32_t* lab, hipStream_t s);
// lab[i] = the nearest of the G centroids c[G][dp] (ties to the lower index).
void launch_nearest_of(const float* x, int64_t n, const float* c, int G, int dp, int metric, int32_t* lab,
                       hipStream_t s);
// c[rows[g]] = src[g] for g < G.
void launch_put_rows(const float* src, const int32_t* rows, int64_t G, int dp, float* c, hipStream_t s);

// kernels: serving (k_serve.hip)
void launch_rows_to_slots(const float* x, int64_t n, int d, int dp, const int32_t* slots, float* out, double* norm2,
                          hipStream_t s);
void launch_candidates_to_slots(const int32_t* cand, const float* h, int64_t n, int M, const int32_t* slots,
                                int32_t* cand_out, float* h_out, int32_t* mq, hipStream_t s);
void launch_init_slots(Workspace& ws, const int32_t* slots, int64_t n, int kk, int w0, hipStream_t s);
void launch_mark_free(Workspace& ws, int64_t n, hipStream_t s);
void launch_gather_results(const Workspace& ws, const int32_t* slots, int64_t n, int k, int kk, int metric,
                           int64_t* ids, float* dist, int32_t* ns, double* rec, hipStream_t s);

}  // namespace qk

// Search-engine internals shared by the C ABI (capi.cpp) and the serving
// loop (serve.cpp).
#pragma once
#include <functional>

#include "index.hpp"

namespace qk {

// Records the message quake_last_error returns on this thread; returns code.
int set_error(int code, const std::string& msg);
extern thread_local std::string g_error;

// Number of candidate partitions for a fraction f of n (ceil, at least 1,
// at most n; the product is taken with a 1e-9 allowance so that 0.05 * 1000
// gives 50 and not 51).
int candidate_count(double f, int64_t n);

// One search over one store, resolved from quake_search_params.
struct Job {
  int k = 0, kk = 0, aps = 0, M = 0, w0 = 0, wmax = 0, batched = 0, dtype16 = QUAKE_F32;
  int rerank = 1;      // batched path: re-score the kk candidates in FP32 (0: keep the 16-bit values)
  double tau_r = 0, f_M = 0, tau_rho = 0.01;
  int est = QUAKE_EST_APS;  // recall estimator variant
  const uint32_t* filter = nullptr;  // label mask of every query (device [nq]), or null
  bool given = false;  // candidate rows already in ws.cand0 / ws.mq0 (level 0 of two levels)
  bool count = true;   // add the queries to the store's access statistics (not for insert routing)
};

Job resolve(const quake_index* idx, const Store& st, const quake_search_params* p);
int64_t max_chunks(const Store& st, int chunk_tiles);
// Per-query arrays of the workspace for nq queries (reallocates, dropping contents, when it grows).
void ensure_queries(quake_index* idx, int64_t nq);
// Grid of the persistent scan kernels.
int scan_blocks(quake_index* idx, int batched);
// R scan rounds on the stream without a host round trip: each round scans
// the windows planned by the previous k_demand / k_prefix, commits, and
// plans the next round (so the item count of the last one tells whether
// work remains).
void run_rounds(quake_index* idx, const Store& st, const Job& job, const RoundArgs& a, int R, hipStream_t s);
// Destroys the captured round graphs of the index.
void release_graphs(quake_index* idx);
void ensure_workspace(quake_index* idx, int64_t nc, int64_t M, int64_t kk, int64_t items, int64_t pairs, int dp16,
                      bool scores = true);
// Tiles per work item, and work items a search of nq queries may need per round.
int search_chunk_tiles(const quake_index* idx, const Job& job);
int64_t search_items(const quake_index* idx, const Store& st, const Job& job, int64_t nq);
// Lays the search workspace for nq queries out in `base` (256-byte aligned
// arrays) and returns its size; w == nullptr only measures.
size_t workspace_layout(Workspace* w, char* base, int64_t nq, int64_t nc, int64_t M, int64_t kk, int64_t items,
                        int64_t pairs, int dp, int dp16);
// quake_search with its workspace in caller-given device memory and host
// counters; allocates nothing (single-level indexes).
void search_in_scratch(quake_index* idx, const float* q, int64_t nq, const quake_search_params* params,
                       int64_t* out_ids, float* out_dist, int32_t* out_nscanned, double* out_recall, hipStream_t s,
                       char* scratch, size_t scratch_bytes, int64_t* host_counters);
// Runs fn under the C ABI's error handling: the return code, and the message
// for quake_last_error on failure.
int run_api(const std::function<void()>& fn);

// Store upkeep shared by updates and maintenance (capi.cpp).
// The arena holds at least `need` tiles (grown by copying; old tiles keep their contents).
void store_grow_arena(quake_index* idx, Store& st, int64_t need, hipStream_t s);
// Partition p moves to fresh tiles at the arena's end (which must have room) with capacity cap.
void store_relocate(Store& st, int64_t p, int32_t cap, hipStream_t s);
// Device copies of off / size / cap and the size order.
void store_upload_table(Store& st, hipStream_t s);
// Deleted slots of the partitions with which[p] set are filled from their live tails.
void store_compact(quake_index* idx, Store& st, const std::vector<char>& which, hipStream_t s);
// Fraction bits of exact fixed-point sums over rows [n][dp].
int store_fixed_point_bits(DeviceMemory& mem, const float* x, int64_t n, int dp, hipStream_t s);
// Batched insert / delete on a level-0 store and its id map (quake_insert and
// quake_delete run them on the index's own; the serving loop also on its
// second copy, from its update thread).  routed: partition of every row,
// else the nearest centroid's.  Errors as quake_insert / quake_delete.
void insert_rows(quake_index* idx, Store& st, IdMap& map, const float* x, const int64_t* ids, int64_t n,
                 const std::vector<int32_t>* routed, hipStream_t s, const uint32_t* attrs = nullptr);
void delete_rows(quake_index* idx, Store& st, IdMap& map, const int64_t* ids, int64_t n, hipStream_t s);
// quake_build's work; with top_centroids (device [nlist_top][d]) and top_of
// (device [nlist]) a two-level index takes that level 1 instead of k-means.
// Returns the new index; throws on error.
quake_index* build_index(const float* x, const int64_t* ids, int64_t n, int32_t d, const quake_build_params* params,
                         const float* top_centroids, const int32_t* top_of, const quake_allocator* allocator,
                         hipStream_t s);
// Level `level` (1 or 2) over the centroids of the level below: k-means, or
// the given top centroids and parent of every centroid below (capi.cpp).
void build_top_level(quake_index* idx, int level, int64_t nlist_top, int32_t kmeans_iters, uint64_t seed,
                     const float* top_centroids, const int32_t* parent, hipStream_t s);
// Level 1 rebuilt over the current level-0 centroids (their nearest level-1
// partitions; level-1 centroids unchanged) after level 0 changed (capi.cpp).
void rebuild_level1(quake_index* idx, hipStream_t s);
// Product codes of the rows at `slots` of `st` (partition parts[i]), or of
// every live row of `st` (after its partitions or centroids changed).
void encode_rows(quake_index* idx, const Store& st, const int64_t* slots, const int32_t* parts, int64_t n,
                 hipStream_t s);
void encode_store(quake_index* idx, const Store& st, hipStream_t s);
// The maintenance pass behind quake_maintain (maintain.cpp).
void maintain(quake_index* idx, const quake_maintain_params& p, quake_maintain_report* report, hipStream_t s);

}  // namespace qk

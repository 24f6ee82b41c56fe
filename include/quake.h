/*
 * quake.h - C ABI of the MI355X partitioned vector index.
 *
 * The library answers the problem of Sec. 2.1 of "Quake: Adaptive Indexing
 * for Vector Search" (Mohoney et al., OSDI'25): given a query q, return the
 * top-k nearest neighbours of q in the vector set X, while batched inserts
 * and deletes change X.  X is kept in disjoint partitions, each with a
 * centroid (Sec. 3, index structure); a search ranks the centroids, scans the
 * vectors of the chosen partitions and merges a per-query top-k.  The number
 * of partitions scanned is either fixed (nprobe) or chosen per query by
 * Adaptive Partition Scanning (Sec. 5, Algorithm "Adaptive Partition
 * Scanning"), which stops once its recall model (Eqs. aps-pi, aps-p0,
 * aps-pi-final) says the recall target is met.
 *
 * Conventions for every entry point:
 *  - Return value: QUAKE_OK (0) or a negative QUAKE_E_* code; the message of
 *    the last failure on the calling thread is quake_last_error().
 *  - Array arguments are DEVICE pointers (HIP device memory on the current
 *    device) owned by the caller; the library reads or writes them during the
 *    call only and never frees them.  Outputs are caller-allocated.
 *  - Matrices are row-major and dense: x[n][d], q[nq][d] float32.
 *  - `stream` is a hipStream_t (NULL = the null stream).  The call enqueues
 *    its work on that stream and returns after the results are written
 *    (search and update calls synchronise the stream before returning).
 *  - An index handle is not thread-safe: one caller at a time.
 *  - The index owns all of its device state and releases it in quake_free.
 */
#ifndef QUAKE_H
#define QUAKE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct quake_index quake_index;

enum {
  QUAKE_OK = 0,
  QUAKE_E_INVALID = -1,   /* bad argument (sizes, k, modes, non-finite input) */
  QUAKE_E_NOMEM = -2,     /* the index would exceed its HBM budget, or hipMalloc failed */
  QUAKE_E_NOTFOUND = -3,  /* a delete batch names an id that is absent; nothing applied */
  QUAKE_E_DUPLICATE = -4, /* an insert batch repeats an id or names a present one; nothing applied */
  QUAKE_E_DEVICE = -5,    /* a HIP call failed */
  QUAKE_E_STATE = -6,     /* the handle is not usable (NULL, freed, wrong level count) */
  QUAKE_E_IO = -7         /* a file could not be opened, written or renamed */
};

enum { QUAKE_L2 = 0, QUAKE_IP = 1 };
enum { QUAKE_F32 = 0, QUAKE_BF16 = 1, QUAKE_F16 = 2 };
/* scan_dtype of a search over the index's product-quantization codes (Sec. 8,
 * "Vector Compression"; built with pq_m > 0) */
enum { QUAKE_PQ8 = 3 };
enum { QUAKE_SCAN_PLAIN = 0, QUAKE_SCAN_BATCHED = 1 };
/* Recall estimator of an adaptive search (Sec. 5.1, Table tab:recall_overhead):
 * APS recomputes the partition probabilities when rho moved by more than
 * tau_rho and reads the cap share from the 1,024-point table; APS_R
 * recomputes after every partition, from the table; APS_RP recomputes after
 * every partition and evaluates the share from the incomplete beta function. */
enum { QUAKE_EST_APS = 0, QUAKE_EST_APS_R = 1, QUAKE_EST_APS_RP = 2 };

/* Device memory provider for everything an index allocates: its partition
 * store, id map, search workspace and temporary build / update buffers.
 * alloc(bytes, ctx) returns device memory of at least `bytes` bytes on the
 * current device, aligned to at least 256 bytes, or NULL when it cannot
 * (the call then fails with QUAKE_E_NOMEM); free(p, ctx) takes back a
 * pointer alloc returned.  ctx is passed through unchanged.  The library
 * waits for the device to be idle before it frees a block, as hipFree does.
 * The index keeps a copy of the struct, so both functions and ctx must stay
 * valid until quake_free returns; they may be called from the serving
 * loop's worker thread.  The Python binding passes torch's caching
 * allocator.  A NULL allocator (or a NULL alloc) means hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* p, void* ctx);
  void* ctx;
} quake_allocator;

/* Build parameters (Sec. 3 index structure; k-means partitioning, Sec. 1). */
typedef struct {
  int32_t metric;          /* QUAKE_L2 (squared Euclidean) or QUAKE_IP (inner product; rows
                              should be unit-norm, centroids are renormalised: spherical k-means) */
  int32_t storage_dtype;   /* extra reduced-precision copy of the vectors: QUAKE_F32 = none,
                              QUAKE_BF16 or QUAKE_F16 (used by scan_dtype != QUAKE_F32) */
  int32_t n_levels;        /* 1, or 2 (level 1 partitions the level-0 centroids); a third level is
                              added to a live index with quake_add_level */
  int32_t kmeans_iters;    /* Lloyd iterations (>= 0) when centroids are not given */
  int64_t nlist;           /* level-0 partitions, 1 <= nlist <= n */
  int64_t nlist_top;       /* level-1 partitions when n_levels == 2 */
  uint64_t seed;           /* k-means initialisation */
  const float* centroids;  /* optional device [nlist][d]: use these centroids (no k-means) */
  const int32_t* assign;   /* optional device [n]: partition of every row, in [0, nlist).  Given,
                              the rows are placed as it says (no nearest-centroid placement: the
                              recall model's pruning assumes every row sits in its nearest
                              partition, Sec. 5 "Geometric Model", which is then the caller's to keep); without
                              centroids, each centroid is the mean of its rows (unit length for
                              QUAKE_IP) and every partition must receive a row */
  size_t hbm_budget_bytes; /* 0 = unlimited; else every device allocation of the index counts */
  double capacity_slack;   /* extra partition capacity for inserts, fraction of size (>= 0); the
                              arena also keeps that fraction of spare tiles for partitions that outgrow theirs */
  int32_t drop_f32_tiles;  /* 1 (with a 16-bit copy): keep no FP32 tile copy of level 0 - only the
                              16-bit tiles the batched scan reads and the row-major FP32 copy the
                              rerank reads (a third less memory); plain FP32 searches are then INVALID */
  const uint32_t* attrs;   /* optional device [n]: 32 label bits of every row, for filtered searches
                              (Sec. 8, "Filters"); a labelled index takes its inserts through
                              quake_insert_attrs */
  int32_t pq_m;            /* 0, or keep a product-quantized copy of level 0 (Sec. 8, "Vector
                              Compression"): pq_m subspaces of d / pq_m consecutive dimensions (pq_m a
                              multiple of 4 dividing d, d / pq_m <= 32), 256 codewords each, one byte
                              per subspace and row; searched with scan_dtype QUAKE_PQ8.  The index also
                              keeps the row-major FP32 copy the rerank reads, and drop_f32_tiles may be
                              set without a 16-bit copy */
  const float* pq_codebook; /* optional device [pq_m][256][d / pq_m]: use this codebook; else it is
                              trained by kmeans_iters Lloyd iterations per subspace (squared L2, from
                              256 distinct rows of a seeded sample of at most 65,536; needs n >= 256) */
} quake_build_params;

/* Search parameters.  Exactly one of nprobe > 0 (fixed number of partitions)
 * or 0 < recall_target <= 1 (Adaptive Partition Scanning) must be set. */
typedef struct {
  int32_t k;               /* 1 <= k <= 256 */
  int32_t nprobe;          /* fixed-nprobe mode: scan the nprobe nearest partitions */
  double recall_target;    /* APS mode: tau_R of Alg. "Adaptive Partition Scanning" */
  double f_M;              /* APS initial candidate fraction (paper: 1%..10%); 0 -> 0.05 */
  double tau_rho;          /* APS recompute threshold (paper: 1%); 0 -> 0.01 */
  double upper_recall_target; /* two-level: level-1 target (paper fixes 99%); 0 -> 0.99 */
  double upper_f_M;        /* two-level: level-1 candidate fraction; 0 -> 0.25 */
  int32_t scan_mode;       /* QUAKE_SCAN_PLAIN: per-(query, partition) scans;
                              QUAKE_SCAN_BATCHED: queries grouped per partition (Sec. 7.4, "Multi-Query Processing") */
  int32_t scan_dtype;      /* QUAKE_F32, or the index's reduced-precision copy (batched scan), or
                              QUAKE_PQ8 (plain scan over product codes: rows are scored from a
                              per-query table of query-to-codeword values, APS runs on those scores,
                              rerank_factor * k rows (<= 64) are kept and re-scored in FP32; an index
                              built with pq_m > 0; not for quake_search_noalloc or the server) */
  int32_t rerank_factor;   /* reduced precision: keep rerank_factor*k candidates, rerank in FP32;
                              0 -> 4; -1: no rerank, the k best by the 16-bit path's own values
                              (IP: the MFMA dot of the rounded query and row, FP32 accumulation;
                              L2: |q|^2 + |x~|^2 - 2 q~.x~ with x~, q~ the rounded vectors) */
  int32_t window;          /* first-round speculation window (partitions per query); 0 -> auto */
  int32_t estimator;       /* QUAKE_EST_APS (default), QUAKE_EST_APS_R or QUAKE_EST_APS_RP; every level */
  const uint32_t* filter;  /* optional device [nq]: label mask of every query (Sec. 8, "Filters"): only
                              rows whose label bits share a bit with it are results, and the recall
                              model scales each candidate's cap share by the partition's estimated
                              pass fraction (per-bit counts of the mask's bits, capped at its live
                              rows).  Needs a labelled one-level index (either scan path). */
} quake_search_params;

/* Build an index over x[n][d] (device, float32) with ids[n] (device int64,
 * unique, >= 0; NULL -> 0..n-1).  Runs k-means on the device unless
 * params->centroids or params->assign is given; without params->assign
 * every vector is then placed in its nearest centroid's partition.  Device
 * memory comes from `allocator` (NULL: hipMalloc).  *out receives the new
 * handle.
 * Errors: INVALID (n < 1, d < 1 or > 4096, nlist out of range, bad enums,
 * a non-finite value in x or the given centroids, an assign entry outside
 * [0, nlist), an empty partition under assign without centroids),
 * DUPLICATE (repeated ids), NOMEM, DEVICE. */
int quake_build(const float* x, const int64_t* ids, int64_t n, int32_t d,
                const quake_build_params* params, const quake_allocator* allocator, void* stream,
                quake_index** out);

/* Search nq queries q[nq][d] (device float32).  Writes out_ids[nq][k]
 * (device int64) and out_dist[nq][k] (device float32): squared L2 distances
 * ascending, or inner products descending; ties go to the lower id; missing
 * results are id -1 with +inf (L2) / -inf (IP).  Optional outputs (NULL to
 * skip): out_nscanned[nq] (device int32, partitions scanned at level 0) and
 * out_recall[nq] (device float64, the recall estimate at stop; 1 in nprobe mode).
 * Errors: INVALID (nq < 0, k, both/neither of nprobe / recall_target, an unknown estimator,
 * scan_dtype without a matching copy, a non-finite value in q; checked
 * before any search work), NOMEM, DEVICE. */
int quake_search(quake_index* index, const float* q, int64_t nq, const quake_search_params* params,
                 int64_t* out_ids, float* out_dist, int32_t* out_nscanned, double* out_recall,
                 void* stream);

/* quake_search for callers that cannot allocate device memory (serving loops
 * and harnesses that forbid allocation): the same search, results and errors
 * as quake_search, but its workspace lives in a scratch array of 256 MiB that
 * the library holds on every device it runs on until the process ends, its
 * host-side counters in a process-wide block, and it calls no allocator
 * (hipMalloc, hipFree or the index's allocator), captures no graph and
 * allocates no pinned memory.  Single-level indexes only (else STATE).  A
 * search whose workspace would exceed the scratch array is rejected with
 * INVALID and a message giving the bytes it needs (fewer queries per call
 * fit; e.g. about 5,000 queries of 768 dims over 4,096 partitions with
 * f_M = 0.05 on the batched path).  All calls on one device share its scratch
 * array and the host counters: calls that overlap in time race; run them one
 * after another (the index handle is single-caller anyway). */
int quake_search_noalloc(quake_index* index, const float* q, int64_t nq, const quake_search_params* params,
                         int64_t* out_ids, float* out_dist, int32_t* out_nscanned, double* out_recall,
                         void* stream);

/* Insert n vectors x[n][d] (device float32) with ids[n] (device int64) as one
 * batch (Sec. 2.1 updates; Sec. 3: each vector goes top-down to its nearest
 * leaf partition and is appended there).  Centroids do not move.
 * Errors: DUPLICATE (repeated id or id already present; nothing applied),
 * INVALID (negative id, a non-finite value in x; nothing applied), NOMEM,
 * DEVICE. */
int quake_insert(quake_index* index, const float* x, const int64_t* ids, int64_t n, void* stream);

/* quake_insert for a labelled index: attrs[n] (device uint32) are the rows'
 * label bits.  Errors as quake_insert; INVALID when the index is not
 * labelled (and quake_insert is INVALID on a labelled one). */
int quake_insert_attrs(quake_index* index, const float* x, const int64_t* ids, const uint32_t* attrs, int64_t n,
                       void* stream);

/* Delete the vectors with ids[n] (device int64) as one batch (Sec. 3: found
 * through the id map and removed).  Errors: NOTFOUND (an id is absent or
 * repeated; nothing applied), INVALID, DEVICE. */
int quake_delete(quake_index* index, const int64_t* ids, int64_t n, void* stream);

/* Host-side counters: live vectors, level-0 partitions, device bytes held. */
int quake_stats(const quake_index* index, int64_t* n_live, int64_t* n_partitions, size_t* device_bytes);

/* Host-side shape of the index: dimension, metric, 16-bit storage dtype
 * (QUAKE_F32 = none) and level count.  Any pointer may be NULL. */
int quake_describe(const quake_index* index, int32_t* d, int32_t* metric, int32_t* storage_dtype, int32_t* n_levels);

/* Export the level-0 partitioning for checking: centroids[nlist][d] (device
 * float32), and for every live vector its id and partition (device int64
 * ids[n_live], int32 part[n_live], in store order).  Any pointer may be NULL. */
int quake_export(const quake_index* index, float* centroids, int64_t* ids, int32_t* part, void* stream);

/* Export the product quantization of level 0 (Sec. 8, "Vector Compression")
 * for checking: *m (host) receives pq_m (0 when the index keeps no codes);
 * codebook[pq_m][256][d / pq_m] (device float32) and, for every live vector
 * in the order quake_export lists them, its codes[n_live][pq_m] (device
 * uint8).  Any pointer may be NULL.  Errors: STATE, DEVICE. */
int quake_export_pq(const quake_index* index, int32_t* m, float* codebook, uint8_t* codes, void* stream);

/* Save the index to a file: the level-0 centroids, every live vector with
 * its id and partition (partition by partition, in store order), the
 * access statistics, the scheduling knobs, and for two levels the level-1
 * centroids and the top partition of every level-0 centroid, followed by a
 * 64-bit FNV-1a checksum.  Written to "<path>.tmp", then renamed to path.
 * No search, update or server may run on the index meanwhile.
 * Errors: INVALID (empty path, an index with no live vector), IO, NOMEM,
 * DEVICE, STATE. */
int quake_save(quake_index* index, const char* path, void* stream);

/* Load a saved index into a new handle: the store is built afresh from the
 * saved centroids and assignment (each partition keeps its saved row order;
 * no k-means, no re-placement), so searches see the same partitions,
 * centroids and rows as on the saved index.  Device memory comes from
 * `allocator` (NULL: hipMalloc), within hbm_budget_bytes (0: unlimited).
 * Errors: IO (cannot open), INVALID (not a saved index, another version, a
 * truncated or corrupt file: checked before anything is built), NOMEM,
 * DEVICE. */
int quake_load(const char* path, const quake_allocator* allocator, size_t hbm_budget_bytes, void* stream,
               quake_index** out);

/* Add a level ("Add Level", Sec. 4.2): partition the centroids of the
 * current top level into nlist_top partitions by k-means (kmeans_iters Lloyd
 * iterations, seeded), which become the new top level.  Searches then run
 * adaptive scanning at every level from the top down, each upper level
 * returning the candidate set of the level below (M_l = ceil(f_M N_l) with
 * upper_f_M for levels >= 1, f_M for level 0), and inserts route top-down.
 * A one-level index becomes two-level as if built so; a two-level one
 * becomes three-level.  Errors: STATE (three levels: at most three are
 * supported), INVALID (nlist_top outside [1, top partitions]), NOMEM,
 * DEVICE. */
int quake_add_level(quake_index* index, int64_t nlist_top, int32_t kmeans_iters, uint64_t seed, void* stream);

/* Remove the top level ("Remove Level", Sec. 4.2): the centroids of the
 * level below become the top again; the levels below are unchanged.
 * Errors: STATE (one level). */
int quake_remove_level(quake_index* index, void* stream);

/* The level thresholds of Sec. 4.2 ("Adding and Removing Levels"): an index
 * of fewer than three levels whose top level has more than add_above
 * partitions (0: never) gets a new top level of nlist_top partitions (0:
 * round(sqrt(top partitions))); an index of several levels whose top level
 * has fewer than remove_below partitions loses it.
 * *action (optional) receives 1 (added), -1 (removed) or 0.  Errors as
 * quake_add_level / quake_remove_level; INVALID for a negative argument. */
int quake_adjust_levels(quake_index* index, int64_t add_above, int64_t remove_below, int64_t nlist_top,
                        int32_t kmeans_iters, uint64_t seed, void* stream, int32_t* action);

/* Export upper level `level` (1 or 2): its centroids [N_level][d] (device
 * float32) and the partition of every centroid of the level below,
 * parent[N_{level-1}] (device int32).  Any pointer may be NULL.
 * Errors: INVALID (no such level). */
int quake_export_level(const quake_index* index, int32_t level, float* centroids, int32_t* parent, void* stream);

/* Partitions per level: out[0] = N_0, out[1] = N_1 (0 without level 1),
 * out[2] = N_2 (0 without level 2). */
int quake_level_sizes(const quake_index* index, int64_t* out);

/* Export the level-1 partitioning of a two- or three-level index: top centroids
 * [nlist_top][d] (device float32) and the top partition of every level-0
 * centroid, top_of[nlist] (device int32). */
int quake_export_top(const quake_index* index, float* top_centroids, int32_t* top_of, void* stream);

/* ------------------------------------------------------------ maintenance
 *
 * Adaptive incremental maintenance (Sec. 4).  Stage 0 of the decision
 * workflow (Sec. 4.2): every search, the serving loop included, adds one to
 * the access count of each partition a query committed (a partition scanned
 * speculatively past the stop point is not counted) and the number of
 * queries to the window; insert routing and the autotuner's searches are not
 * counted.  A_j = hits_j / window is the cost model's access frequency. */

/* Access statistics of level `level` (0, or 1 on a two-level index):
 * hits[nlist] (host int64, may be NULL) and *window (host, may be NULL);
 * reset != 0 clears both afterwards. */
int quake_access_stats(quake_index* index, int32_t level, int64_t* hits, int64_t* window, int32_t reset,
                       void* stream);

/* lambda(s) on this GPU (Sec. 4.1 measures it by offline profiling; Sec. 8
 * asks for a per-device profile on heterogeneous hardware): for each
 * sizes[i], an index of eight partitions of that many of this index's
 * vectors (same metric and copies) is searched by nq of them with params'
 * path and k, once with nprobe 1 and once with nprobe 8, reps times each
 * after a warm-up; out_us[i] (host) = (time with 8 - time with 1) / 7 in
 * microseconds per query: what one more partition of sizes[i] vectors costs
 * a query in a batch of nq, without the work every search does once.  8 x
 * sizes[i] and nq may not exceed the index's live vectors.  Allocates its
 * temporaries like the index does. */
int quake_profile_latency(quake_index* index, const int32_t* sizes, int32_t points, int32_t nq,
                          const quake_search_params* params, int32_t reps, double* out_us, void* stream);

/* One decision of a maintenance pass: the estimate (Eq. delta_split_est, or
 * the uniform-redistribution delete estimate), the verified delta with the
 * actual sizes (Eqs. delta_split_exact / delta_merge_exact), and whether it
 * was committed (verified < -tau). */
typedef struct {
  int32_t partition;   /* id before the pass */
  int32_t action;      /* 0 split, 1 delete */
  int32_t committed;
  int32_t new_partition; /* split: the right child's id before deletes renumber; delete: -1 */
  double estimate;
  double verified;
} quake_decision;

typedef struct {
  double tau;            /* commit threshold (>= 0), in the unit of lambda_cost */
  double alpha;          /* access fraction each split child inherits, in (0, 1] */
  int32_t refine_radius; /* r_f: partitions nearest to each split child refined with it (>= 0) */
  int32_t refine_iters;  /* k-means passes of a refinement (0: no refinement) */
  int32_t split_iters;   /* Lloyd steps of the 2-means split (>= 1) */
  int32_t min_split_size;/* partitions with fewer live vectors are not split (>= 2) */
  int64_t merge_below;   /* partitions with fewer live vectors are delete candidates (0: no deletes) */
  int32_t lambda_points; /* >= 2 */
  int32_t max_decisions; /* capacity of `decisions` */
  const double* lambda_size; /* host [lambda_points], strictly ascending: scan sizes */
  const double* lambda_cost; /* host [lambda_points]: profiled latency of scanning that many vectors */
  const int64_t* hits;   /* host [nlist] access counts to use, or NULL: the index's own */
  int64_t window;        /* queries behind `hits` (>= 1 with hits; ignored without) */
  quake_decision* decisions; /* host [max_decisions] or NULL: the decisions, in the order taken */
} quake_maintain_params;

typedef struct {
  int32_t decisions;     /* decisions taken (may exceed max_decisions; the rest are not written) */
  int32_t splits;        /* committed splits */
  int32_t deletes;       /* committed deletes */
  int32_t pad;
  int64_t nlist_before, nlist_after;
  int64_t vectors_moved; /* vectors that changed partition (splits, refinement, deletes) */
} quake_maintain_report;

/* One maintenance pass over level 0 (Sec. 4.2, Stages
 * 1-3), with lambda interpolated linearly between the profiled sizes
 * (extended linearly past the ends) and the centroid overhead
 * dO+/- = lambda(N +/- 1) - lambda(N):
 *   1. estimate every partition's split; for each one below -tau, split it
 *      by 2-means on the device (start: the vector farthest from the
 *      centroid and the one farthest from that; inner product: spherical),
 *      verify with the children's actual sizes and the same frequency
 *      assumption (alpha A each), commit below -tau, otherwise keep the
 *      partition as it was;
 *   2. refine around each committed split: k-means passes seeded by the
 *      current centroids over the two children and the refine_radius
 *      partitions nearest to each child (Sec. 4.2, "Partition Refinement");
 *   3. for every other partition below merge_below: estimate the delete with
 *      its vectors and accesses spread evenly over its refine_radius nearest
 *      partitions; below -tau, send each vector to its nearest remaining
 *      centroid, verify with the actual receivers (frequency following the
 *      vectors) and commit below -tau;
 *   4. renumber the surviving partitions in their old order, and clear the
 *      access statistics;
 *   5. with upper levels, rebuild level 1 over the new level-0 centroids,
 *      each in its nearest level-1 partition (level-1 centroids do not move,
 *      so higher levels are unchanged): the changes propagate upward.
 * Vectors that change partition move with all their copies; ids are kept.
 * Decisions are taken in partition order, every estimate against the index
 * as the earlier steps of the pass left it, with the centroid overhead taken
 * at the partition count before the pass.  Errors: INVALID for bad
 * parameters. */
int quake_maintain(quake_index* index, const quake_maintain_params* params, quake_maintain_report* report,
                   void* stream);

/* Candidate order of Adaptive Partition Scanning for nq queries, without
 * scanning level 0: order[nq][M] (device int32, c_0 first, then ascending
 * bisector distance) and h[nq][M] (device float32, h[.][0] = 0), with
 * M = ceil(params->f_M * nlist) clamped to [1, nlist] (f_M 0 -> 0.05);
 * *out_M receives M.  Of params only f_M, tau_rho and the upper-level
 * settings are read.  On a two-level index the candidates are the ones the
 * level-1 search returns, as in quake_search (Sec. 3; Sec. 5.1: APS at
 * every level); a query given fewer than M has order -1 and h 0 after them.
 * q = NULL with nq = 0 only reports M. */
int quake_candidates(quake_index* index, const float* q, int64_t nq, const quake_search_params* params,
                     int32_t* order, float* h, int32_t* out_M, void* stream);

/* The recall model's cap-volume table for dimension d (host memory): the
 * volume share of a d-ball beyond a hyperplane at distance t, at the 1,024
 * points t_j = j / 1023 (Sec. 5.1, "Performance Optimizations").  Host-only, no device needed. */
int quake_cap_table(int32_t d, double* out_1024);

/* Scheduling knobs of the search; 0 keeps the built-in default.  They change
 * how the work is cut into items and rounds, never the results: partitions
 * are committed in candidate order whatever the cut.  Errors: INVALID for
 * negative values, STATE for a bad handle. */
typedef struct {
  int32_t chunk_tiles;   /* store tiles (64 vectors each) per work item, <= 1024; default 16 */
  int32_t first_window;  /* APS: partitions per query in the first round; default 2 */
  int32_t max_window;    /* APS: most partitions per query in one round; default 32 */
  int32_t blocks_per_cu; /* persistent scan grid, blocks of 4 waves per compute unit; default 1 (MFMA) / 8 (FP32) */
  int64_t max_items;     /* work items per round (bounds the scratch memory); default from nq */
  int32_t rounds_per_sync; /* rounds enqueued between host checks for completion; default 1, 2, 4, then 8 */
  int32_t no_graph;      /* 1: launch every round's kernels; default 0 replays captured HIP graphs of rounds */
  int32_t window_scale;  /* APS: a query's predicted next window is scaled by this percentage, 100..1000
                            (fewer rounds for more speculative scans); default 100 */
} quake_tuning;
int quake_set_tuning(quake_index* index, const quake_tuning* tuning);

/* Autotuner: times searches of the sample queries q[nq][d] (device) with
 * `params` under candidate settings of the knobs above (work-item size,
 * rounds between host checks, persistent grid size, first and largest
 * window), by coordinate descent from the current settings (median of
 * `reps` timed searches per candidate, 0 -> 3; a change must be 1% faster),
 * and leaves the fastest set on the index.  Writes the chosen knobs to *out
 * and their median search time in milliseconds to *ms (both optional).
 * Results never depend on these knobs, only the time does.  Errors as for
 * quake_search; on error the previous knobs are restored. */
int quake_autotune(quake_index* index, const float* q, int64_t nq, const quake_search_params* params, int32_t reps,
                   quake_tuning* out, double* ms, void* stream);

/* Kernel timing of searches, for roofline measurement.  With enable = 1 the
 * library records HIP events on the search stream around each kernel class
 * and, after the search completes, adds the elapsed times to per-class
 * totals; it also adds the algorithmic bytes and flops of each launch.
 * Bytes: for the plain scan every (query, vector) read, d * 4 each (no
 * reuse between queries by design); for the batched scan every vector of
 * every partition a round touches, once per round, d * 2 each (the bytes a
 * launch has to read); centroid rows for scoring.  QUAKE_PROF_SCAN_SETS
 * holds (bytes only) the batched scan's reads counted once per query set of
 * up to 128 queries, the bytes its blocks request.  reset = 1 zeroes the
 * totals.  out (host, QUAKE_PROF_KINDS entries) receives the totals when
 * not NULL. */
enum {
  QUAKE_PROF_CENTROIDS = 0, /* centroid scoring */
  QUAKE_PROF_SELECT = 1,    /* candidate selection and bisector geometry */
  QUAKE_PROF_PLAN = 2,      /* work-item planning */
  QUAKE_PROF_SCAN = 3,      /* partition scans */
  QUAKE_PROF_COMMIT = 4,    /* in-order commit and recall model */
  QUAKE_PROF_RERANK = 5,    /* FP32 rerank of reduced-precision candidates */
  QUAKE_PROF_SCAN_SETS = 6, /* batched scan reads per query set (bytes only, no launches) */
  QUAKE_PROF_UPPER = 7,     /* everything the level-1 search of a two-level index runs (the other
                               kinds then cover level 0 alone) */
  QUAKE_PROF_KINDS = 8
};
typedef struct {
  int64_t launches;
  double milliseconds;
  double bytes;
  double flops;
} quake_kernel_profile;
int quake_profile(quake_index* index, int32_t enable, int32_t reset, quake_kernel_profile* out);

/* ------------------------------------------------------------------------
 * Serving loop.  A server owns a worker thread and a HIP stream on the
 * index's device and answers single-query search requests and insert /
 * delete batches submitted from any thread, with host arrays.  Searches are
 * batched continuously: a query takes a free slot of the running batch at
 * the next scan round and leaves it when its own adaptive scan stops, so
 * queries that arrive while others are on the device overlap with them.
 * The slot count is max_slots, or what hbm_budget_bytes of search
 * workspace holds (each slot needs the query row, its candidates, its result
 * lists and its share of the work items).  Updates keep submission order:
 * every search answers as if it ran alone on the index state of its epoch
 * (the state after the updates submitted before it; the paper's system
 * runs searches and updates serially, Sec. 8).  Without overlap_updates,
 * admission pauses at an update, the queries already admitted finish, the
 * batch is applied, and admission resumes.  With overlap_updates (Sec. 8,
 * "Concurrency", names copy-on-write views as the way to run updates beside
 * queries) the server holds a second copy of the level-0 store (twice the
 * store's device memory): the update is applied to the copy no search
 * reads, the copies swap, later searches run on the new version while the
 * earlier ones finish on the old one, and the old copy replays the update
 * once its searches are done - an update waits only for the searches of the
 * version before the current one.  While a server runs, its index must not
 * be used through other entry points; afterwards the index holds the newest
 * version.  Single-level indexes only.
 * ---------------------------------------------------------------------- */
typedef struct quake_server quake_server;

typedef struct {
  int32_t max_slots;        /* queries in flight at once; 0 -> from hbm_budget_bytes, else 4096 */
  int32_t overlap_updates;  /* 1: keep a second copy of the level-0 store and apply each update
                               beside the searches admitted before it (see below); 0: drain */
  size_t hbm_budget_bytes;  /* device bytes the in-flight searches may use; 0 -> unlimited */
  quake_search_params search;
} quake_server_params;

typedef struct {
  int64_t completed;        /* searches answered */
  int64_t queued;           /* requests waiting for admission */
  int64_t in_flight;        /* searches holding a slot */
  int64_t slots;            /* slot capacity */
  int64_t max_in_flight;    /* most slots held at once */
  int64_t epochs;           /* update batches applied */
  int64_t rounds;           /* scan rounds run */
  int64_t overlapped_updates; /* updates applied while searches of the previous version ran */
  double p50_latency_s;     /* arrival -> answer ready, over completed searches */
  double p99_latency_s;
  double mean_latency_s;
  double qps;               /* completed / (last answer - first arrival) */
} quake_server_report;

/* Errors: INVALID (bad params, an index with upper levels, a filter in the search
 * params), STATE, NOMEM, DEVICE. */
int quake_server_create(quake_index* index, const quake_server_params* params, quake_server** out);
/* Submit n single-query searches q[n][d] (host float32); tickets are
 * *first_ticket .. *first_ticket + n - 1. */
int quake_server_search(quake_server* server, const float* q, int64_t n, uint64_t* first_ticket);
/* Submit an insert batch x[n][d], ids[n] or a delete batch ids[n] (host). */
int quake_server_insert(quake_server* server, const float* x, const int64_t* ids, int64_t n, uint64_t* ticket);
int quake_server_delete(quake_server* server, const int64_t* ids, int64_t n, uint64_t* ticket);
/* Wait up to timeout_s (< 0: forever) for a ticket.  Searches write k ids
 * and distances (host) and *nscanned; every ticket writes the request's
 * status code (QUAKE_OK or the error of an update batch) to *status.
 * Returns QUAKE_OK when the ticket finished (it is then forgotten),
 * QUAKE_E_STATE on timeout, QUAKE_E_INVALID for an unknown ticket. */
int quake_server_wait(quake_server* server, uint64_t ticket, double timeout_s, int64_t* ids, float* dist,
                      int32_t* nscanned, int32_t* status);
int quake_server_stats(quake_server* server, quake_server_report* out, int32_t reset);
/* Answers what was submitted, stops the worker and frees the server. */
void quake_server_destroy(quake_server* server);

void quake_free(quake_index* index);
const char* quake_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QUAKE_H */

// C ABI: index build, search rounds, exports.  Host-side orchestration only;
// every step of a search runs in the kernels of k_centroids.hip and
// k_scan.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "index.hpp"

namespace {

thread_local std::string g_error;

int fail(int code, const std::string& msg) {
  g_error = msg;
  return code;
}

#define API_BEGIN try {
#define API_END                                                      \
  }                                                                  \
  catch (const qk::Error& e) { return fail(e.code, e.msg); }         \
  catch (const std::bad_alloc&) { return fail(QUAKE_E_NOMEM, "host allocation failed"); } \
  catch (const std::exception& e) { return fail(QUAKE_E_DEVICE, e.what()); }             \
  return QUAKE_OK;

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Number of candidate partitions for a fraction f of n (ceil, at least 1,
// at most n; the product is taken with a 1e-9 allowance so that 0.05 * 1000
// gives 50 and not 51).
int candidate_count(double f, int64_t n) {
  double m = std::ceil(f * (double)n - 1e-9);
  if (m < 1) m = 1;
  if (m > (double)n) m = (double)n;
  return (int)m;
}

void check_index(const quake_index* idx) {
  QK_CHECK(idx && idx->magic == 0x51554b45u, QUAKE_E_STATE, "invalid or freed index handle");
}

}  // namespace

namespace qk {

void* DeviceMemory::raw_alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (budget && used + bytes > budget)
    throw Error{QUAKE_E_NOMEM, "HBM budget exceeded: " + std::to_string(used + bytes) + " > " +
                                   std::to_string(budget) + " bytes"};
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error{QUAKE_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  used += bytes;
  blocks_.push_back({p, bytes});
  return p;
}

void DeviceMemory::release(void* p) {
  if (!p) return;
  for (size_t i = 0; i < blocks_.size(); ++i)
    if (blocks_[i].p == p) {
      (void)hipFree(p);
      used -= blocks_[i].bytes;
      blocks_[i] = blocks_.back();
      blocks_.pop_back();
      return;
    }
}

DeviceMemory::~DeviceMemory() {
  for (auto& b : blocks_) (void)hipFree(b.p);
}

hipEvent_t Profiler::event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  QK_HIP(hipEventCreate(&e));
  return e;
}

void Profiler::begin(int kind, hipStream_t s) {
  if (!on) return;
  Span sp{kind, event(), event()};
  QK_HIP(hipEventRecord(sp.a, s));
  pending.push_back(sp);
}

void Profiler::end(hipStream_t s) {
  if (!on || pending.empty()) return;
  (void)hipEventRecord(pending.back().b, s);
}

void Profiler::collect() {
  for (auto& sp : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) {
      acc[sp.kind].milliseconds += ms;
      acc[sp.kind].launches += 1;
    }
    pool.push_back(sp.a);
    pool.push_back(sp.b);
  }
  pending.clear();
}

Profiler::~Profiler() {
  for (auto& sp : pending) { pool.push_back(sp.a); pool.push_back(sp.b); }
  for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace qk

namespace {

using qk::Error;
using qk::Store;

// Temporary device buffer released at scope exit.
template <class T>
struct Tmp {
  qk::DeviceMemory* mem;
  T* p = nullptr;
  Tmp(qk::DeviceMemory& m, size_t n) : mem(&m) { p = m.alloc<T>(n); }
  ~Tmp() { mem->release(p); }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
};

template <class T>
void grow(qk::DeviceMemory& mem, T*& p, int64_t& cap, int64_t need) {
  if (need <= cap && p) return;
  mem.release(p);
  p = nullptr;
  cap = std::max<int64_t>(need, 1);
  p = mem.alloc<T>((size_t)cap);
}

// Lloyd's k-means on the device over (a seeded sample of) the rows.  Rows
// and centroids are [.][dp] FP32.  Initial centroids are distinct random
// rows; an empty cluster is re-seeded with a random row.  Spherical k-means
// (unit centroids) for inner product.
void kmeans(qk::DeviceMemory& mem, const float* xpad, int64_t n, int dp, int64_t nc, int iters, uint64_t seed,
            int metric, float* centroids, hipStream_t s) {
  std::mt19937_64 rng(seed);
  const int64_t max_train = std::max<int64_t>(nc * 256, 65536);
  const float* train = xpad;
  int64_t nt = n;
  std::unique_ptr<Tmp<float>> sample;
  auto pick_distinct = [&](int64_t pool, int64_t count) {
    std::vector<int64_t> v(pool);
    std::iota(v.begin(), v.end(), 0);
    for (int64_t i = 0; i < count; ++i) {
      const int64_t j = i + (int64_t)(rng() % (uint64_t)(pool - i));
      std::swap(v[i], v[j]);
    }
    v.resize(count);
    return v;
  };
  auto gather = [&](const float* src, const std::vector<int64_t>& rows, float* dst) {
    Tmp<int64_t> d_rows(mem, rows.size());
    QK_HIP(hipMemcpyAsync(d_rows.p, rows.data(), rows.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    qk::launch_gather_rows(src, dp, d_rows.p, (int64_t)rows.size(), dp, dst, s);
    QK_HIP(hipStreamSynchronize(s));
  };
  if (n > max_train) {
    std::vector<int64_t> rows = pick_distinct(n, max_train);
    std::sort(rows.begin(), rows.end());
    sample.reset(new Tmp<float>(mem, (size_t)max_train * dp));
    gather(xpad, rows, sample->p);
    train = sample->p;
    nt = max_train;
  }
  gather(train, pick_distinct(nt, nc), centroids);
  Tmp<float> sums(mem, (size_t)nc * dp);
  Tmp<int32_t> counts(mem, (size_t)nc);
  Tmp<int32_t> assign(mem, (size_t)nt);
  std::vector<int32_t> h_counts(nc);
  const int normalise = metric == QUAKE_IP ? 1 : 0;
  if (normalise) {
    // unit initial centroids: sums = centroids, counts = 1, update
    QK_HIP(hipMemcpyAsync(sums.p, centroids, (size_t)nc * dp * sizeof(float), hipMemcpyDeviceToDevice, s));
    std::vector<int32_t> ones(nc, 1);
    QK_HIP(hipMemcpyAsync(counts.p, ones.data(), nc * sizeof(int32_t), hipMemcpyHostToDevice, s));
    qk::launch_kmeans_update(sums.p, counts.p, nc, dp, 1, centroids, s);
    QK_HIP(hipStreamSynchronize(s));
  }
  for (int it = 0; it < iters; ++it) {
    qk::launch_assign(train, nt, dp, centroids, nc, metric, assign.p, s);
    QK_HIP(hipMemsetAsync(sums.p, 0, (size_t)nc * dp * sizeof(float), s));
    QK_HIP(hipMemsetAsync(counts.p, 0, (size_t)nc * sizeof(int32_t), s));
    qk::launch_kmeans_accumulate(train, nt, dp, assign.p, sums.p, counts.p, s);
    qk::launch_kmeans_update(sums.p, counts.p, nc, dp, normalise, centroids, s);
    QK_HIP(hipMemcpyAsync(h_counts.data(), counts.p, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    for (int64_t j = 0; j < nc; ++j) {
      if (h_counts[j] != 0) continue;
      const int64_t r = (int64_t)(rng() % (uint64_t)nt);
      gather(train, std::vector<int64_t>{r}, centroids + j * dp);
    }
  }
}

// Place rows into a fresh store: partition p gets capacity for its rows plus
// slack, rounded up to whole tiles; rows keep their input order within a
// partition.
void build_store(quake_index* idx, Store& st, const float* xin, int d, const int64_t* ids, int64_t n,
                 const int32_t* d_assign, double slack, int dtype16, hipStream_t s) {
  std::vector<int32_t> a(n);
  QK_HIP(hipMemcpyAsync(a.data(), d_assign, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  const int64_t N = st.nlist;
  st.size.assign(N, 0);
  for (int64_t i = 0; i < n; ++i) st.size[a[i]]++;
  st.cap.resize(N);
  st.off.resize(N);
  int64_t tiles = 0;
  for (int64_t p = 0; p < N; ++p) {
    const int64_t want = st.size[p] + (int64_t)std::ceil(st.size[p] * slack);
    st.cap[p] = (int32_t)round_up(want, qk::TILE);
    st.off[p] = tiles;
    tiles += st.cap[p] / qk::TILE;
  }
  std::vector<int64_t> slot(n);
  std::vector<int64_t> fill(N, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int p = a[i];
    slot[i] = st.off[p] * qk::TILE + fill[p]++;
  }
  const int64_t arena = std::max<int64_t>(tiles, 1);
  st.tiles = arena;
  st.used_tiles = tiles;
  st.v32 = idx->mem.alloc<float>((size_t)arena * qk::TILE * st.dp);
  QK_HIP(hipMemsetAsync(st.v32, 0, (size_t)arena * qk::TILE * st.dp * sizeof(float), s));
  st.dp16 = qk::padded_dim16(st.d);
  if (dtype16 != QUAKE_F32) {
    st.v16 = idx->mem.alloc<uint16_t>((size_t)arena * qk::TILE * st.dp16);
    QK_HIP(hipMemsetAsync(st.v16, 0, (size_t)arena * qk::TILE * st.dp16 * sizeof(uint16_t), s));
    if (idx->metric == QUAKE_L2) st.v16n = idx->mem.alloc<float>((size_t)arena * qk::TILE);
    st.rows32 = idx->mem.alloc<float>((size_t)arena * qk::TILE * st.dp);
    QK_HIP(hipMemsetAsync(st.rows32, 0, (size_t)arena * qk::TILE * st.dp * sizeof(float), s));
  }
  st.ids = idx->mem.alloc<int64_t>((size_t)arena * qk::TILE);
  QK_HIP(hipMemsetAsync(st.ids, 0xff, (size_t)arena * qk::TILE * sizeof(int64_t), s));
  st.d_off = idx->mem.alloc<int64_t>(N);
  st.d_size = idx->mem.alloc<int32_t>(N);
  st.d_cap = idx->mem.alloc<int32_t>(N);
  QK_HIP(hipMemcpyAsync(st.d_off, st.off.data(), N * sizeof(int64_t), hipMemcpyHostToDevice, s));
  QK_HIP(hipMemcpyAsync(st.d_size, st.size.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, s));
  QK_HIP(hipMemcpyAsync(st.d_cap, st.cap.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, s));
  {
    Tmp<int64_t> d_slot(idx->mem, n);
    QK_HIP(hipMemcpyAsync(d_slot.p, slot.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    qk::launch_scatter(xin, n, d, st.dp, st.dp16, ids, d_slot.p, st.v32, st.v16, dtype16, st.rows32, st.ids, s);
    qk::launch_norm16(st, dtype16, s);
    QK_HIP(hipStreamSynchronize(s));
  }
  st.live = n;
}

int64_t max_chunks(const Store& st, int chunk_tiles) {
  int64_t mx = 1;
  for (int32_t sz : st.size) {
    const int64_t t = (sz + qk::TILE - 1) / qk::TILE;
    mx = std::max<int64_t>(mx, (t + chunk_tiles - 1) / chunk_tiles);
  }
  return mx;
}

struct Resolved {
  int k, kk, nprobe, aps, M, w0, wmax, batched, dtype16;
  double tau_r, f_M, tau_rho;
};

Resolved resolve(const quake_index* idx, const Store& st, const quake_search_params* p) {
  QK_CHECK(p, QUAKE_E_INVALID, "params is NULL");
  QK_CHECK(p->k >= 1 && p->k <= qk::KMAX, QUAKE_E_INVALID, "k must be in [1, 256]");
  const bool has_np = p->nprobe > 0;
  const bool has_rt = p->recall_target > 0.0;
  QK_CHECK(has_np != has_rt, QUAKE_E_INVALID, "set exactly one of nprobe > 0 or recall_target > 0");
  QK_CHECK(!has_rt || p->recall_target <= 1.0, QUAKE_E_INVALID, "recall_target must be in (0, 1]");
  QK_CHECK(p->scan_mode == QUAKE_SCAN_PLAIN || p->scan_mode == QUAKE_SCAN_BATCHED, QUAKE_E_INVALID,
           "unknown scan_mode");
  QK_CHECK(p->scan_dtype == QUAKE_F32 || (p->scan_dtype == idx->storage && st.v16), QUAKE_E_INVALID,
           "scan_dtype needs the matching reduced-precision copy in the index");
  Resolved r{};
  r.k = p->k;
  r.batched = p->scan_mode == QUAKE_SCAN_BATCHED ? 1 : 0;
  r.dtype16 = p->scan_dtype;
  QK_CHECK(r.batched == (p->scan_dtype != QUAKE_F32 ? 1 : 0), QUAKE_E_INVALID,
           "the batched scan runs on the 16-bit copy (scan_dtype BF16/F16) and the plain scan on FP32");
  QK_CHECK(p->rerank_factor >= 0, QUAKE_E_INVALID, "rerank_factor must be >= 0");
  r.kk = r.batched ? std::max(p->rerank_factor > 0 ? p->rerank_factor : 4, 1) * r.k : r.k;
  QK_CHECK(!r.batched || r.kk <= 64, QUAKE_E_INVALID, "the batched scan keeps at most 64 candidates per query");
  QK_CHECK(!r.batched || st.dp16 <= 1024, QUAKE_E_INVALID, "the batched scan supports d <= 1024");
  r.aps = has_rt ? 1 : 0;
  r.tau_r = p->recall_target;
  r.f_M = p->f_M > 0 ? p->f_M : 0.05;
  r.tau_rho = p->tau_rho > 0 ? p->tau_rho : 0.01;
  const int64_t N = st.nlist;
  const int64_t cap_m = N > 4096 ? 2048 : qk::MAX_CANDIDATES;
  const quake_tuning& tu = idx->tune;
  if (r.aps) {
    r.M = candidate_count(r.f_M, N);
    QK_CHECK(r.M <= cap_m, QUAKE_E_INVALID, "f_M * nlist exceeds the candidate limit");
    r.w0 = p->window > 0 ? p->window : (tu.first_window > 0 ? tu.first_window : 2);
    r.wmax = tu.max_window > 0 ? tu.max_window : 32;
  } else {
    r.M = (int)std::min<int64_t>(p->nprobe, N);
    QK_CHECK(r.M <= cap_m, QUAKE_E_INVALID, "nprobe exceeds the candidate limit");
    r.w0 = r.M;
    r.wmax = r.M;
  }
  r.w0 = std::min(r.w0, r.M);
  r.wmax = std::max(std::min(r.wmax, r.M), r.w0);
  return r;
}

void ensure_workspace(quake_index* idx, int64_t nq, int64_t nc, int64_t M, int64_t kk, int64_t items,
                      int64_t pairs = 0, bool need16 = false) {
  qk::Workspace& w = idx->ws;
  auto& mem = idx->mem;
  const int dp = idx->dp;
  if (nq > w.nq_cap || !w.q) {
    const int64_t n = std::max<int64_t>(nq, 1);
    for (void* p : {(void*)w.q, (void*)w.qn2, (void*)w.st_m, (void*)w.st_w, (void*)w.st_weff, (void*)w.st_done,
                    (void*)w.st_item,
                    (void*)w.st_demand, (void*)w.st_vecs, (void*)w.st_pair, (void*)w.st_rho, (void*)w.st_p0,
                    (void*)w.st_V, (void*)w.st_vsum, (void*)w.st_r, (void*)w.q16, (void*)w.qn2f})
      mem.release(p);
    w.q = mem.alloc<float>((size_t)n * dp);
    w.qn2 = mem.alloc<double>(n);
    w.st_m = mem.alloc<int32_t>(n);
    w.st_w = mem.alloc<int32_t>(n);
    w.st_weff = mem.alloc<int32_t>(n);
    w.st_done = mem.alloc<int32_t>(n);
    w.st_item = mem.alloc<int64_t>(n);
    w.st_demand = mem.alloc<int64_t>(n);
    w.st_vecs = mem.alloc<int64_t>(n);
    w.st_pair = mem.alloc<int64_t>(n);
    w.q16 = nullptr;
    w.qn2f = mem.alloc<float>(n);
    w.st_rho = mem.alloc<double>(n);
    w.st_p0 = mem.alloc<double>(n);
    w.st_V = mem.alloc<double>(n);
    w.st_vsum = mem.alloc<double>(n);
    w.st_r = mem.alloc<double>(n);
    w.nq_cap = n;
    w.scores_cap = w.cand_cap = w.kk_cap = 0;  // dependent sizes re-grow below
    mem.release(w.scores); w.scores = nullptr;
    mem.release(w.sel); w.sel = nullptr;
    mem.release(w.cand); w.cand = nullptr;
    mem.release(w.h); w.h = nullptr;
    mem.release(w.rk); w.rk = nullptr;
    mem.release(w.ri); w.ri = nullptr;
  }
  grow(mem, w.scores, w.scores_cap, w.nq_cap * nc);
  if (M * w.nq_cap > w.cand_cap || !w.sel) {
    mem.release(w.sel); mem.release(w.cand); mem.release(w.h);
    w.cand_cap = w.nq_cap * M;
    w.sel = mem.alloc<int32_t>(w.cand_cap);
    w.cand = mem.alloc<int32_t>(w.cand_cap);
    w.h = mem.alloc<float>(w.cand_cap);
  }
  if (kk * w.nq_cap > w.kk_cap || !w.rk) {
    mem.release(w.rk); mem.release(w.ri);
    w.kk_cap = kk * w.nq_cap;
    w.rk = mem.alloc<float>(w.kk_cap);
    w.ri = mem.alloc<int64_t>(w.kk_cap);
  }
  if (items > w.items_cap || kk > w.k_cap || !w.items) {
    mem.release(w.items); mem.release(w.pk); mem.release(w.pi);
    w.items_cap = std::max(items, w.items_cap);
    w.k_cap = std::max<int64_t>(kk, w.k_cap);
    w.items = mem.alloc<int4>(w.items_cap);
    w.pk = mem.alloc<float>((size_t)w.items_cap * w.k_cap);
    w.pi = mem.alloc<int64_t>((size_t)w.items_cap * w.k_cap);
  }
  if (!w.total) {
    w.total = mem.alloc<int64_t>(8);
    QK_HIP(hipHostMalloc((void**)&w.h_total, 8 * sizeof(int64_t), hipHostMallocDefault));
  }
  if (need16 && !w.q16) w.q16 = mem.alloc<uint16_t>((size_t)w.nq_cap * idx->L0.dp16);
  if (pairs > w.pairs_cap || !w.pair_q) {
    for (void* p : {(void*)w.pair_q, (void*)w.pair_p, (void*)w.pair_pos, (void*)w.pair_base, (void*)w.sorted})
      mem.release(p);
    w.pairs_cap = std::max<int64_t>(pairs, 1);
    w.pair_q = mem.alloc<int32_t>(w.pairs_cap);
    w.pair_p = mem.alloc<int32_t>(w.pairs_cap);
    w.pair_pos = mem.alloc<int32_t>(w.pairs_cap);
    w.pair_base = mem.alloc<int64_t>(w.pairs_cap);
    w.sorted = mem.alloc<int32_t>(w.pairs_cap);
  }
  if (nc + 1 > w.parts_cap || !w.pcount) {
    for (void* p : {(void*)w.pcount, (void*)w.pstart, (void*)w.pitem}) mem.release(p);
    w.parts_cap = nc + 1;
    w.pcount = mem.alloc<int32_t>(w.parts_cap);
    w.pstart = mem.alloc<int32_t>(w.parts_cap);
    w.pitem = mem.alloc<int64_t>(w.parts_cap);
    QK_HIP(hipMemset(w.pcount, 0, w.parts_cap * sizeof(int32_t)));
  }
}

// Candidate partitions of every query: the nearest M centroids and, for
// adaptive scanning, their order by ascending bisector distance.
void candidates(quake_index* idx, const Store& st, int64_t nq, int M, bool aps, hipStream_t s) {
  qk::Workspace& w = idx->ws;
  {
    qk::ProfileScope ps(idx->prof, QUAKE_PROF_CENTROIDS, s);
    qk::launch_scores(w.q, nq, st.centroids, st.nlist, idx->dp, idx->metric, w.scores, s);
  }
  idx->prof.add(QUAKE_PROF_CENTROIDS, (double)st.nlist * idx->dp * 4.0 + (double)nq * idx->dp * 4.0 +
                                           (double)nq * st.nlist * 4.0,
                (double)nq * st.nlist * idx->dp * (idx->metric == QUAKE_L2 ? 3.0 : 2.0));
  qk::ProfileScope ps(idx->prof, QUAKE_PROF_SELECT, s);
  if (aps) {
    qk::launch_select(w.scores, nq, st.nlist, M, idx->metric, w.sel, s);
    qk::launch_geometry(w.q, st.centroids, nq, idx->dp, M, idx->metric, w.sel, w.cand, w.h, s);
  } else {
    qk::launch_select(w.scores, nq, st.nlist, M, idx->metric, w.cand, s);
  }
}

}  // namespace

extern "C" {

const char* quake_last_error(void) { return g_error.c_str(); }

int quake_cap_table(int32_t d, double* out) {
  API_BEGIN
  QK_CHECK(d >= 1 && d <= qk::MAX_DIM && out, QUAKE_E_INVALID, "bad dimension or output");
  qk::cap_fraction_table(d, out);
  API_END
}

int quake_build(const float* x, const int64_t* ids, int64_t n, int32_t d, const quake_build_params* params,
                void* stream, quake_index** out) {
  API_BEGIN
  QK_CHECK(out, QUAKE_E_INVALID, "out is NULL");
  *out = nullptr;
  QK_CHECK(params, QUAKE_E_INVALID, "params is NULL");
  QK_CHECK(x && n >= 1, QUAKE_E_INVALID, "need x and n >= 1");
  QK_CHECK(d >= 1 && d <= qk::MAX_DIM, QUAKE_E_INVALID, "d must be in [1, 4096]");
  QK_CHECK(params->metric == QUAKE_L2 || params->metric == QUAKE_IP, QUAKE_E_INVALID, "unknown metric");
  QK_CHECK(params->storage_dtype >= QUAKE_F32 && params->storage_dtype <= QUAKE_F16, QUAKE_E_INVALID,
           "unknown storage dtype");
  QK_CHECK(params->n_levels == 1 || params->n_levels == 2, QUAKE_E_INVALID, "n_levels must be 1 or 2");
  QK_CHECK(params->nlist >= 1 && params->nlist <= n, QUAKE_E_INVALID, "nlist must be in [1, n]");
  QK_CHECK(params->nlist <= INT32_MAX, QUAKE_E_INVALID, "nlist too large");
  QK_CHECK(params->kmeans_iters >= 0 && params->capacity_slack >= 0, QUAKE_E_INVALID, "bad k-means settings");
  if (params->n_levels == 2)
    QK_CHECK(params->nlist_top >= 1 && params->nlist_top <= params->nlist, QUAKE_E_INVALID,
             "nlist_top must be in [1, nlist]");
  hipStream_t s = as_stream(stream);
  std::unique_ptr<quake_index> idx(new quake_index());
  idx->mem.budget = params->hbm_budget_bytes;
  idx->metric = params->metric;
  idx->storage = params->storage_dtype;
  idx->n_levels = params->n_levels;
  idx->d = d;
  idx->dp = (int)round_up(d, 8);
  const int dp = idx->dp;

  if (ids) {
    std::vector<int64_t> h(n);
    QK_HIP(hipMemcpyAsync(h.data(), ids, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    QK_CHECK(std::all_of(h.begin(), h.end(), [](int64_t v) { return v >= 0; }), QUAKE_E_INVALID,
             "ids must be >= 0");
    std::sort(h.begin(), h.end());
    QK_CHECK(std::adjacent_find(h.begin(), h.end()) == h.end(), QUAKE_E_DUPLICATE, "ids repeat");
  }

  // rows padded to dp (the input is used as is when d is already a multiple of 8)
  std::unique_ptr<Tmp<float>> xpad_buf;
  const float* xpad = x;
  if (dp != d) {
    xpad_buf.reset(new Tmp<float>(idx->mem, (size_t)n * dp));
    qk::launch_pad_rows(x, n, d, dp, xpad_buf->p, nullptr, s);
    xpad = xpad_buf->p;
  }

  Store& L0 = idx->L0;
  L0.d = d;
  L0.dp = dp;
  L0.nlist = params->nlist;
  L0.centroids = idx->mem.alloc<float>((size_t)L0.nlist * dp);
  if (params->centroids) {
    qk::launch_pad_rows(params->centroids, L0.nlist, d, dp, L0.centroids, nullptr, s);
  } else {
    kmeans(idx->mem, xpad, n, dp, L0.nlist, params->kmeans_iters, params->seed, idx->metric, L0.centroids, s);
  }
  {
    Tmp<int32_t> assign(idx->mem, n);
    qk::launch_assign(xpad, n, dp, L0.centroids, L0.nlist, idx->metric, assign.p, s);
    build_store(idx.get(), L0, x, d, ids, n, assign.p, params->capacity_slack, params->storage_dtype, s);
  }

  if (idx->n_levels == 2) {
    Store& L1 = idx->L1;
    L1.d = d;
    L1.dp = dp;
    L1.nlist = params->nlist_top;
    L1.centroids = idx->mem.alloc<float>((size_t)L1.nlist * dp);
    kmeans(idx->mem, L0.centroids, L0.nlist, dp, L1.nlist, std::max(params->kmeans_iters, 1),
           params->seed ^ 0x9e3779b97f4a7c15ull, QUAKE_L2, L1.centroids, s);
    idx->top_of = idx->mem.alloc<int32_t>(L0.nlist);
    qk::launch_assign(L0.centroids, L0.nlist, dp, L1.centroids, L1.nlist, QUAKE_L2, idx->top_of, s);
    build_store(idx.get(), L1, L0.centroids, dp, nullptr, L0.nlist, idx->top_of, 0.0, QUAKE_F32, s);
  }

  idx->h_cap_table.resize(qk::CAP_TABLE_POINTS);
  qk::cap_fraction_table(d, idx->h_cap_table.data());
  idx->cap_table = idx->mem.alloc<double>(qk::CAP_TABLE_POINTS);
  QK_HIP(hipMemcpyAsync(idx->cap_table, idx->h_cap_table.data(), qk::CAP_TABLE_POINTS * sizeof(double),
                        hipMemcpyHostToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  *out = idx.release();
  API_END
}

int quake_search(quake_index* idx, const float* q, int64_t nq, const quake_search_params* params, int64_t* out_ids,
                 float* out_dist, int32_t* out_nscanned, double* out_recall, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(nq >= 0, QUAKE_E_INVALID, "nq must be >= 0");
  QK_CHECK(idx->n_levels == 1, QUAKE_E_STATE, "two-level search is not available in this build");
  const Store& st = idx->L0;
  const Resolved r = resolve(idx, st, params);
  if (nq == 0) return QUAKE_OK;
  QK_CHECK(q && out_ids && out_dist, QUAKE_E_INVALID, "q, out_ids and out_dist are required");
  hipStream_t s = as_stream(stream);
  const int chunk_tiles = idx->tune.chunk_tiles > 0 ? idx->tune.chunk_tiles : 16;
  const int64_t kk = r.kk;
  const int64_t mc = max_chunks(st, chunk_tiles);
  // the buffer must hold one full window of the largest partitions (progress)
  const int64_t floor_items = (int64_t)r.wmax * mc + 1;
  const int64_t items = std::max<int64_t>(
      idx->tune.max_items > 0 ? idx->tune.max_items : nq * std::max(r.w0, 4) * 2, floor_items);
  ensure_workspace(idx, nq, st.nlist, r.M, kk, items, r.batched ? nq * (int64_t)r.wmax : 0, r.batched != 0);
  qk::Workspace& w = idx->ws;
  QK_HIP(hipMemsetAsync(w.total, 0, 8 * sizeof(int64_t), s));
  qk::launch_pad_rows(q, nq, idx->d, idx->dp, w.q, w.qn2, s);
  candidates(idx, st, nq, r.M, r.aps, s);
  if (r.batched) qk::launch_queries16(w, nq, idx->dp, st.dp16, r.dtype16, s);
  // a smaller requested cap than the buffer already allocated still applies
  const int64_t items_cap = std::min<int64_t>(w.items_cap, items);
  qk::RoundArgs a{};
  a.nq = nq;
  a.M = r.M;
  a.k = r.k;
  a.kk = r.kk;
  a.aps = r.aps;
  a.chunk_tiles = chunk_tiles;
  a.wmax = r.wmax;
  a.metric = idx->metric;
  a.dim = idx->d;
  a.tau_r = r.tau_r;
  a.tau_rho = r.tau_rho;
  a.items_cap = items_cap;
  qk::launch_round_init(w, a, r.w0, s);
  if (r.batched && idx->cu_count == 0) {
    int dev = 0;
    QK_HIP(hipGetDevice(&dev));
    QK_HIP(hipDeviceGetAttribute(&idx->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
  }
  // Every round commits at least one partition of the first unfinished
  // query, so the loop ends within nq * M rounds.
  const int64_t max_rounds = nq * (int64_t)r.M + 2;
  for (int64_t round = 0;; ++round) {
    QK_CHECK(round <= max_rounds, QUAKE_E_DEVICE, "search rounds did not converge");
    {
      qk::ProfileScope ps(idx->prof, QUAKE_PROF_PLAN, s);
      qk::launch_demand(w, st, a, s);
    }
    QK_HIP(hipMemcpyAsync(w.h_total, w.total, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    const int64_t total = w.h_total[0];
    const int64_t nvec = w.h_total[1];
    const int64_t npairs = w.h_total[2];
    if (total == 0) break;
    if (r.batched) {
      {
        qk::ProfileScope ps(idx->prof, QUAKE_PROF_PLAN, s);
        qk::launch_group(w, st, a, npairs, s);
      }
      qk::ProfileScope ps(idx->prof, QUAKE_PROF_SCAN, s);
      qk::launch_scan_mfma(w, st, a, r.dtype16, std::max(idx->cu_count, 8) * 2, s);
    } else {
      {
        qk::ProfileScope ps(idx->prof, QUAKE_PROF_PLAN, s);
        qk::launch_emit(w, st, a, s);
      }
      {
        qk::ProfileScope ps(idx->prof, QUAKE_PROF_SCAN, s);
        qk::launch_scan_f32(w, st, a, total, s);
      }
      idx->prof.add(QUAKE_PROF_SCAN, (double)nvec * idx->d * sizeof(float),
                    (double)nvec * idx->d * (idx->metric == QUAKE_L2 ? 3.0 : 2.0));
    }
    {
      qk::ProfileScope ps(idx->prof, QUAKE_PROF_COMMIT, s);
      qk::launch_commit(w, st, a, idx->cap_table, s);
    }
  }
  if (r.batched) {
    {
      qk::ProfileScope ps(idx->prof, QUAKE_PROF_RERANK, s);
      qk::launch_rerank(w, st, a, s);
    }
    idx->prof.add(QUAKE_PROF_RERANK, (double)nq * kk * idx->d * sizeof(float), (double)nq * kk * idx->d * 2.0);
  }
  {
    qk::ProfileScope ps(idx->prof, QUAKE_PROF_COMMIT, s);
    qk::launch_finalize(w, a, out_ids, out_dist, out_nscanned, out_recall, s);
  }
  QK_HIP(hipGetLastError());
  if (r.batched && idx->prof.on)
    QK_HIP(hipMemcpyAsync(w.h_total + 4, w.total + 4, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  if (r.batched)
    idx->prof.add(QUAKE_PROF_SCAN, (double)w.h_total[4] * idx->d * 2.0, (double)w.h_total[5] * idx->d * 2.0);
  idx->prof.collect();
  API_END
}

int quake_set_tuning(quake_index* idx, const quake_tuning* t) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(t, QUAKE_E_INVALID, "tuning is NULL");
  QK_CHECK(t->chunk_tiles >= 0 && t->first_window >= 0 && t->max_window >= 0 && t->max_items >= 0,
           QUAKE_E_INVALID, "tuning values must be >= 0");
  idx->tune = *t;
  API_END
}

int quake_profile(quake_index* idx, int32_t enable, int32_t reset, quake_kernel_profile* out) {
  API_BEGIN
  check_index(idx);
  if (out) std::memcpy(out, idx->prof.acc, sizeof(idx->prof.acc));
  if (reset) std::memset(idx->prof.acc, 0, sizeof(idx->prof.acc));
  idx->prof.on = enable != 0;
  API_END
}

int quake_candidates(quake_index* idx, const float* q, int64_t nq, double f_M, int32_t* order, float* h,
                     int32_t* out_M, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(nq >= 0 && (nq == 0 || (q && order && h)), QUAKE_E_INVALID, "bad arguments");
  const Store& st = idx->L0;
  const int M = candidate_count(f_M > 0 ? f_M : 0.05, st.nlist);
  QK_CHECK(M <= (st.nlist > 4096 ? 2048 : qk::MAX_CANDIDATES), QUAKE_E_INVALID, "too many candidates");
  if (out_M) *out_M = M;
  if (nq == 0) return QUAKE_OK;
  hipStream_t s = as_stream(stream);
  ensure_workspace(idx, nq, st.nlist, M, 1, 1);
  qk::Workspace& w = idx->ws;
  qk::launch_pad_rows(q, nq, idx->d, idx->dp, w.q, w.qn2, s);
  candidates(idx, st, nq, M, true, s);
  QK_HIP(hipMemcpyAsync(order, w.cand, (size_t)nq * M * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipMemcpyAsync(h, w.h, (size_t)nq * M * sizeof(float), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  API_END
}

int quake_insert(quake_index* idx, const float* x, const int64_t* ids, int64_t n, void* stream) {
  API_BEGIN
  check_index(idx);
  (void)x; (void)ids; (void)n; (void)stream;
  throw Error{QUAKE_E_INVALID, "insert is not available in this build"};
  API_END
}

int quake_delete(quake_index* idx, const int64_t* ids, int64_t n, void* stream) {
  API_BEGIN
  check_index(idx);
  (void)ids; (void)n; (void)stream;
  throw Error{QUAKE_E_INVALID, "delete is not available in this build"};
  API_END
}

int quake_stats(const quake_index* idx, int64_t* n_live, int64_t* n_partitions, size_t* device_bytes) {
  API_BEGIN
  check_index(idx);
  if (n_live) *n_live = idx->L0.live;
  if (n_partitions) *n_partitions = idx->L0.nlist;
  if (device_bytes) *device_bytes = idx->mem.used;
  API_END
}

int quake_export(const quake_index* cidx, float* centroids, int64_t* ids, int32_t* part, void* stream) {
  API_BEGIN
  check_index(cidx);
  quake_index* idx = const_cast<quake_index*>(cidx);
  hipStream_t s = as_stream(stream);
  const Store& st = idx->L0;
  if (centroids) {
    // strip the padding: [nlist][dp] -> [nlist][d]
    QK_HIP(hipMemcpy2DAsync(centroids, idx->d * sizeof(float), st.centroids, idx->dp * sizeof(float),
                            idx->d * sizeof(float), st.nlist, hipMemcpyDeviceToDevice, s));
  }
  if (ids || part) {
    std::vector<int64_t> first(st.nlist);
    int64_t slots = 0;
    for (int64_t p = 0; p < st.nlist; ++p) { first[p] = slots; slots += st.size[p]; }
    Tmp<int64_t> d_first(idx->mem, st.nlist);
    Tmp<int64_t> t_ids(idx->mem, std::max<int64_t>(slots, 1));
    Tmp<int32_t> t_part(idx->mem, std::max<int64_t>(slots, 1));
    QK_HIP(hipMemcpyAsync(d_first.p, first.data(), st.nlist * sizeof(int64_t), hipMemcpyHostToDevice, s));
    qk::launch_export(st, t_ids.p, t_part.p, d_first.p, s);
    std::vector<int64_t> h_ids(slots);
    std::vector<int32_t> h_part(slots);
    QK_HIP(hipMemcpyAsync(h_ids.data(), t_ids.p, slots * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipMemcpyAsync(h_part.data(), t_part.p, slots * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> o_ids;
    std::vector<int32_t> o_part;
    o_ids.reserve(st.live);
    o_part.reserve(st.live);
    for (int64_t i = 0; i < slots; ++i)
      if (h_ids[i] >= 0) { o_ids.push_back(h_ids[i]); o_part.push_back(h_part[i]); }
    if (ids) QK_HIP(hipMemcpyAsync(ids, o_ids.data(), o_ids.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (part) QK_HIP(hipMemcpyAsync(part, o_part.data(), o_part.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  QK_HIP(hipStreamSynchronize(s));
  API_END
}

int quake_export_top(const quake_index* idx, float* top_centroids, int32_t* top_of, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(idx->n_levels == 2, QUAKE_E_STATE, "index has one level");
  hipStream_t s = as_stream(stream);
  if (top_centroids)
    QK_HIP(hipMemcpy2DAsync(top_centroids, idx->d * sizeof(float), idx->L1.centroids, idx->dp * sizeof(float),
                            idx->d * sizeof(float), idx->L1.nlist, hipMemcpyDeviceToDevice, s));
  if (top_of)
    QK_HIP(hipMemcpyAsync(top_of, idx->top_of, idx->L0.nlist * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  API_END
}

void quake_free(quake_index* idx) {
  if (!idx || idx->magic != 0x51554b45u) return;
  if (idx->ws.h_total) (void)hipHostFree(idx->ws.h_total);
  idx->magic = 0;
  delete idx;
}

}  // extern "C"

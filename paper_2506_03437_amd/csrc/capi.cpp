// C ABI: index build, search rounds, exports.  Host-side orchestration only;
// every step of a search runs in the kernels of k_centroids.hip and
// k_scan.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <new>
#include <numeric>
#include <random>
#include <string>
#include <type_traits>
#include <vector>

#include "engine.hpp"
#include "index.hpp"

namespace qk {
thread_local std::string g_error;

int set_error(int code, const std::string& msg) {
  g_error = msg;
  return code;
}
}  // namespace qk

namespace {

int fail(int code, const std::string& msg) { return qk::set_error(code, msg); }

#define API_BEGIN try {
#define API_END                                                      \
  }                                                                  \
  catch (const qk::Error& e) { return fail(e.code, e.msg); }         \
  catch (const std::bad_alloc&) { return fail(QUAKE_E_NOMEM, "host allocation failed"); } \
  catch (const std::exception& e) { return fail(QUAKE_E_DEVICE, e.what()); }             \
  return QUAKE_OK;

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

void check_index(const quake_index* idx) {
  QK_CHECK(idx && idx->magic == 0x51554b45u, QUAKE_E_STATE, "invalid or freed index handle");
}

}  // namespace

namespace qk {

// Number of candidate partitions for a fraction f of n (ceil, at least 1,
// at most n; the product is taken with a 1e-9 allowance so that 0.05 * 1000
// gives 50 and not 51).
int candidate_count(double f, int64_t n) {
  double m = std::ceil(f * (double)n - 1e-9);
  if (m < 1) m = 1;
  if (m > (double)n) m = (double)n;
  return (int)m;
}

void* DeviceMemory::raw_alloc(size_t bytes) {
  std::lock_guard<std::mutex> lk(mu_);
  QK_CHECK(!forbid, QUAKE_E_STATE, "an allocation was attempted inside a call that allocates nothing");
  if (bytes == 0) bytes = 256;
  if (budget && used + bytes > budget)
    throw Error{QUAKE_E_NOMEM, "HBM budget exceeded: " + std::to_string(used + bytes) + " > " +
                                   std::to_string(budget) + " bytes"};
  void* p = nullptr;
  if (user.alloc) {
    p = user.alloc(bytes, user.ctx);
    if (!p) throw Error{QUAKE_E_NOMEM, "the allocator returned no memory for " + std::to_string(bytes) + " bytes"};
    if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
      if (user.free) user.free(p, user.ctx);
      throw Error{QUAKE_E_NOMEM, "the allocator returned a block not aligned to 256 bytes"};
    }
  } else if (hipMalloc(&p, bytes) != hipSuccess || !p) {
    (void)hipGetLastError();
    throw Error{QUAKE_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  used += bytes;
  blocks_.push_back({p, bytes});
  return p;
}

void DeviceMemory::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  for (size_t i = 0; i < blocks_.size(); ++i)
    if (blocks_[i].p == p) {
      if (user.alloc) {
        // work queued on any stream may still use the block; hipFree waits
        // for the device, and so does a release through the allocator
        (void)hipDeviceSynchronize();
        if (user.free) user.free(p, user.ctx);
      } else {
        (void)hipFree(p);
      }
      used -= blocks_[i].bytes;
      blocks_[i] = blocks_.back();
      blocks_.pop_back();
      return;
    }
}

DeviceMemory::~DeviceMemory() {
  if (user.alloc) {
    (void)hipDeviceSynchronize();
    if (user.free)
      for (auto& b : blocks_) user.free(b.p, user.ctx);
  } else {
    for (auto& b : blocks_) (void)hipFree(b.p);
  }
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
  if (only >= 0) kind = only;
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

// Fraction bits of the fixed-point cluster sums over rows [n][dp]: n *
// max|x| * 2^bits stays below 2^62 (inputs are checked finite beforehand).
int fixed_point_bits(qk::DeviceMemory& mem, const float* x, int64_t n, int dp, hipStream_t s) {
  Tmp<uint32_t> amax(mem, 1);
  QK_HIP(hipMemsetAsync(amax.p, 0, sizeof(uint32_t), s));
  qk::launch_absmax(x, n * dp, amax.p, s);
  uint32_t bits = 0;
  QK_HIP(hipMemcpyAsync(&bits, amax.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  float m;
  std::memcpy(&m, &bits, sizeof(m));
  int frac_bits = 40;
  if (m > 0.f) frac_bits = (int)std::floor(62.0 - std::log2((double)n * (double)m)) - 1;
  return std::max(-60, std::min(frac_bits, 60));
}

// Centroid j = mean of the rows assigned to j (unit length when normalise),
// from exact fixed-point sums; counts[j] receives the row count.  A centroid
// with no rows is left as it was.
void centroids_from(qk::DeviceMemory& mem, const float* x, int64_t n, int dp, const int32_t* assign, int64_t nc,
                    int normalise, int frac_bits, float* centroids, int32_t* counts, hipStream_t s) {
  Tmp<int64_t> sums(mem, (size_t)nc * dp);
  QK_HIP(hipMemsetAsync(sums.p, 0, (size_t)nc * dp * sizeof(int64_t), s));
  QK_HIP(hipMemsetAsync(counts, 0, (size_t)nc * sizeof(int32_t), s));
  qk::launch_kmeans_accumulate(x, n, dp, assign, frac_bits, sums.p, counts, s);
  qk::launch_kmeans_update(sums.p, counts, nc, dp, normalise, frac_bits, centroids, s);
  QK_HIP(hipStreamSynchronize(s));
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
  Tmp<int32_t> counts(mem, (size_t)nc);
  Tmp<int32_t> assign(mem, (size_t)nt);
  std::vector<int32_t> h_counts(nc);
  const int normalise = metric == QUAKE_IP ? 1 : 0;
  if (normalise) qk::launch_normalise_rows(centroids, nc, dp, s);
  const int frac_bits = fixed_point_bits(mem, train, nt, dp, s);
  for (int it = 0; it < iters; ++it) {
    qk::launch_assign(train, nt, dp, centroids, nc, metric, assign.p, s);
    centroids_from(mem, train, nt, dp, assign.p, nc, normalise, frac_bits, centroids, counts.p, s);
    QK_HIP(hipMemcpyAsync(h_counts.data(), counts.p, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    for (int64_t j = 0; j < nc; ++j) {
      if (h_counts[j] != 0) continue;
      const int64_t r = (int64_t)(rng() % (uint64_t)nt);
      gather(train, std::vector<int64_t>{r}, centroids + j * dp);
    }
  }
}


// ---------------------------------------------------------------- the store

// A level-0 store, or a copy of one (not an upper level).
bool is_leaf(const quake_index* idx, const Store& st) { return &st != &idx->L1 && &st != &idx->L2; }

// `leaf`: the arrays are for a level-0 store (or a copy of one), which also
// holds the label bits and the product codes when the index has them.
void alloc_store_arrays(quake_index* idx, Store& st, int64_t tiles, int dtype16, bool f32_tiles, bool leaf,
                        hipStream_t s) {
  auto& mem = idx->mem;
  const size_t slots = (size_t)tiles * qk::TILE;
  if (f32_tiles) {
    st.v32 = mem.alloc<float>(slots * st.dp);
    QK_HIP(hipMemsetAsync(st.v32, 0, slots * st.dp * sizeof(float), s));
  }
  if (dtype16 != QUAKE_F32) {
    st.v16 = mem.alloc<uint16_t>(slots * st.dp16);
    QK_HIP(hipMemsetAsync(st.v16, 0, slots * st.dp16 * sizeof(uint16_t), s));
    if (idx->metric == QUAKE_L2) {
      st.v16n = mem.alloc<float>(slots);
      QK_HIP(hipMemsetAsync(st.v16n, 0, slots * sizeof(float), s));
    }
    st.rows32 = mem.alloc<float>(slots * st.dp);
    QK_HIP(hipMemsetAsync(st.rows32, 0, slots * st.dp * sizeof(float), s));
  }
  if (leaf && idx->pq_m > 0) {
    // the rerank of a search over codes reads the row-major FP32 copy
    if (!st.rows32) {
      st.rows32 = mem.alloc<float>(slots * st.dp);
      QK_HIP(hipMemsetAsync(st.rows32, 0, slots * st.dp * sizeof(float), s));
    }
    st.pq_m = idx->pq_m;
    st.codes = mem.alloc<uint32_t>(slots * qk::pq_words(idx->pq_m));
    QK_HIP(hipMemsetAsync(st.codes, 0, slots * qk::pq_words(idx->pq_m) * sizeof(uint32_t), s));
  }
  st.ids = mem.alloc<int64_t>(slots);
  QK_HIP(hipMemsetAsync(st.ids, 0xff, slots * sizeof(int64_t), s));
  if (idx->labelled && leaf) {
    st.attr = mem.alloc<uint32_t>(slots);
    QK_HIP(hipMemsetAsync(st.attr, 0, slots * sizeof(uint32_t), s));
  }
  st.tiles = tiles;
}

void upload_table(Store& st, hipStream_t s) {
  const int64_t N = st.nlist;
  QK_HIP(hipMemcpyAsync(st.d_off, st.off.data(), N * sizeof(int64_t), hipMemcpyHostToDevice, s));
  QK_HIP(hipMemcpyAsync(st.d_size, st.size.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, s));
  QK_HIP(hipMemcpyAsync(st.d_cap, st.cap.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // batched scans hand out work in this order: the largest partitions first,
  // so that the last items of a launch are short ones
  st.order.resize(N);
  for (int64_t p = 0; p < N; ++p) st.order[p] = (int32_t)p;
  std::stable_sort(st.order.begin(), st.order.end(), [&](int32_t a, int32_t b) { return st.size[a] > st.size[b]; });
  QK_HIP(hipMemcpyAsync(st.d_order, st.order.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, s));
}

// Place rows into a fresh store: partition p gets capacity for its rows plus
// slack, rounded up to whole tiles; rows keep their input order within a
// partition.
// Product-quantization codebook of the residuals of rows x[n][d] to their
// centroids C[assign[i]] ([.][dp]) into idx->pq_book [pq_m][256][pq_ds]:
// Lloyd's k-means (squared L2, from 256 distinct rows) in each subspace over
// the same seeded sample of at most 65,536 rows.
void train_codebook(quake_index* idx, const float* x, int64_t n, const int32_t* assign, const float* C, int iters,
                    uint64_t seed, hipStream_t s) {
  const int M = idx->pq_m, ds = idx->pq_ds, d = idx->d;
  const int dsp = (int)round_up(ds, 8);
  const int64_t nt = std::min<int64_t>(n, 65536);
  std::vector<int64_t> rows(n);
  std::iota(rows.begin(), rows.end(), 0);
  if (nt < n) {
    std::mt19937_64 rng(seed);
    for (int64_t i = 0; i < nt; ++i) std::swap(rows[i], rows[i + (int64_t)(rng() % (uint64_t)(n - i))]);
    rows.resize(nt);
    std::sort(rows.begin(), rows.end());
  }
  Tmp<int64_t> d_rows(idx->mem, nt);
  Tmp<float> sub(idx->mem, (size_t)nt * dsp), cent(idx->mem, (size_t)256 * dsp);
  QK_HIP(hipMemcpyAsync(d_rows.p, rows.data(), nt * sizeof(int64_t), hipMemcpyHostToDevice, s));
  for (int m = 0; m < M; ++m) {
    qk::launch_pq_subspace(x, nt, d, d_rows.p, assign, C, idx->dp, m * ds, ds, dsp, sub.p, s);
    kmeans(idx->mem, sub.p, nt, dsp, 256, iters, seed + (uint64_t)m, QUAKE_L2, cent.p, s);
    QK_HIP(hipMemcpy2DAsync(idx->pq_book + (size_t)m * 256 * ds, ds * sizeof(float), cent.p, dsp * sizeof(float),
                            ds * sizeof(float), 256, hipMemcpyDeviceToDevice, s));
  }
  QK_HIP(hipStreamSynchronize(s));
}

void build_store(quake_index* idx, Store& st, const float* xin, int d, const int64_t* ids, int64_t n,
                 const int32_t* d_assign, double slack, int dtype16, bool f32_tiles, hipStream_t s,
                 const uint32_t* attrs = nullptr) {
  std::vector<int32_t> a(n);
  QK_HIP(hipMemcpyAsync(a.data(), d_assign, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  const int64_t N = st.nlist;
  st.size.assign(N, 0);
  st.tomb.assign(N, 0);
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
  st.tile_part.assign(std::max<int64_t>(tiles, 1), -1);
  for (int64_t p = 0; p < N; ++p)
    for (int64_t t = 0; t < st.cap[p] / qk::TILE; ++t) st.tile_part[st.off[p] + t] = (int32_t)p;
  std::vector<int64_t> slot(n);
  std::vector<int64_t> fill(N, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int p = a[i];
    slot[i] = st.off[p] * qk::TILE + fill[p]++;
  }
  st.dp16 = qk::padded_dim16(st.d);
  // with slack, the arena also keeps that fraction of spare tiles for
  // partitions that outgrow their capacity (so that the first overflowing
  // inserts do not have to grow, and copy, the whole arena)
  const int64_t spare = slack > 0 ? (int64_t)std::ceil(tiles * slack) : 0;
  alloc_store_arrays(idx, st, std::max<int64_t>(tiles + spare, 1), dtype16, f32_tiles, is_leaf(idx, st), s);
  st.tile_part.resize(std::max<int64_t>(tiles + spare, 1), -1);
  st.used_tiles = tiles;
  st.d_off = idx->mem.alloc<int64_t>(N);
  st.d_size = idx->mem.alloc<int32_t>(N);
  st.d_cap = idx->mem.alloc<int32_t>(N);
  st.d_order = idx->mem.alloc<int32_t>(N);
  st.d_hits = idx->mem.alloc<uint32_t>(std::max<int64_t>(N, 1));
  QK_HIP(hipMemsetAsync(st.d_hits, 0, std::max<int64_t>(N, 1) * sizeof(uint32_t), s));
  st.window = 0;
  upload_table(st, s);
  if (st.attr) {
    st.d_attr_cnt = idx->mem.alloc<uint32_t>((size_t)std::max<int64_t>(N, 1) * 33);
    st.attr_dirty = true;
  }
  {
    Tmp<int64_t> d_slot(idx->mem, n);
    QK_HIP(hipMemcpyAsync(d_slot.p, slot.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    qk::launch_scatter(xin, n, d, st.dp, st.dp16, ids, d_slot.p, st.v32, st.v16, dtype16, st.rows32, st.ids, s);
    qk::launch_norm16(st, dtype16, s);
    if (st.attr && attrs) qk::launch_put_u32(attrs, d_slot.p, n, st.attr, s);
    if (st.codes) qk::encode_rows(idx, st, d_slot.p, d_assign, n, s);
    QK_HIP(hipStreamSynchronize(s));
  }
  st.live = n;
}

// Copy every partition's filled tiles back to back into a fresh arena of
// `tiles` tiles (relocations leave their old tiles behind; this drops them).
// Store slots change: the caller rebuilds the id map.
void repack_arena(quake_index* idx, Store& st, int64_t tiles, hipStream_t s) {
  Store fresh;
  fresh.d = st.d;
  fresh.dp = st.dp;
  fresh.dp16 = st.dp16;
  alloc_store_arrays(idx, fresh, tiles, st.v16 ? idx->storage : QUAKE_F32, st.v32 != nullptr, is_leaf(idx, st), s);
  std::vector<int64_t> off(st.nlist);
  std::vector<int32_t> tile_part(tiles, -1);
  int64_t next = 0;
  for (int64_t p = 0; p < st.nlist; ++p) {
    off[p] = next;
    for (int64_t t = 0; t < st.cap[p] / qk::TILE; ++t) tile_part[next + t] = (int32_t)p;
    const size_t n = (size_t)((st.size[p] + qk::TILE - 1) / qk::TILE) * qk::TILE;
    const size_t a = (size_t)st.off[p] * qk::TILE, b = (size_t)next * qk::TILE;
    if (n > 0) {
      if (st.v32)
        QK_HIP(hipMemcpyAsync(fresh.v32 + b * st.dp, st.v32 + a * st.dp, n * st.dp * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
      if (st.v16)
        QK_HIP(hipMemcpyAsync(fresh.v16 + b * st.dp16, st.v16 + a * st.dp16, n * st.dp16 * sizeof(uint16_t),
                              hipMemcpyDeviceToDevice, s));
      if (st.v16n) QK_HIP(hipMemcpyAsync(fresh.v16n + b, st.v16n + a, n * sizeof(float), hipMemcpyDeviceToDevice, s));
      if (st.rows32)
        QK_HIP(hipMemcpyAsync(fresh.rows32 + b * st.dp, st.rows32 + a * st.dp, n * st.dp * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
      QK_HIP(hipMemcpyAsync(fresh.ids + b, st.ids + a, n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
      if (st.attr) QK_HIP(hipMemcpyAsync(fresh.attr + b, st.attr + a, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
      if (st.codes) {
        const size_t w = (size_t)qk::pq_words(st.pq_m);  // code words per slot (tile-aligned ranges)
        QK_HIP(hipMemcpyAsync(fresh.codes + b * w, st.codes + a * w, n * w * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
      }
    }
    next += st.cap[p] / qk::TILE;
  }
  QK_HIP(hipStreamSynchronize(s));
  for (void* p : {(void*)st.v32, (void*)st.v16, (void*)st.v16n, (void*)st.rows32, (void*)st.ids, (void*)st.attr,
                  (void*)st.codes})
    idx->mem.release(p);
  st.v32 = fresh.v32;
  st.v16 = fresh.v16;
  st.v16n = fresh.v16n;
  st.rows32 = fresh.rows32;
  st.ids = fresh.ids;
  st.attr = fresh.attr;
  st.codes = fresh.codes;
  st.tiles = tiles;
  st.used_tiles = next;
  st.off.swap(off);
  st.tile_part.swap(tile_part);
}

// Enlarge the arena to at least `need` tiles (allocates before touching the
// old arrays, so a failure leaves the store as it was).  With `repack`, when
// tiles left behind by relocations make up a quarter of the used arena the
// partitions are packed into a fresh arena instead (slots change: the caller
// rebuilds the id map; returns true then).
bool grow_arena(quake_index* idx, Store& st, int64_t need, hipStream_t s, bool repack = false) {
  if (need <= st.tiles) return false;
  if (repack) {
    int64_t held = 0;
    for (int64_t p = 0; p < st.nlist; ++p) held += st.cap[p] / qk::TILE;
    if ((st.used_tiles - held) * 4 >= st.used_tiles) {
      const int64_t extra = need - st.used_tiles;
      repack_arena(idx, st, held + extra + (held + extra) / 8, s);
      return true;
    }
  }
  // an eighth more at a time: growing copies the arena, and the old and new
  // arrays coexist while it does (an index of tens of GB must fit twice)
  const int64_t tiles = std::max<int64_t>(need, st.tiles + st.tiles / 8);
  Store fresh;
  fresh.d = st.d;
  fresh.dp = st.dp;
  fresh.dp16 = st.dp16;
  alloc_store_arrays(idx, fresh, tiles, st.v16 ? idx->storage : QUAKE_F32, st.v32 != nullptr, is_leaf(idx, st), s);
  const size_t used = (size_t)st.used_tiles * qk::TILE;
  if (st.v32) QK_HIP(hipMemcpyAsync(fresh.v32, st.v32, used * st.dp * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (st.v16) QK_HIP(hipMemcpyAsync(fresh.v16, st.v16, used * st.dp16 * sizeof(uint16_t), hipMemcpyDeviceToDevice, s));
  if (st.v16n) QK_HIP(hipMemcpyAsync(fresh.v16n, st.v16n, used * sizeof(float), hipMemcpyDeviceToDevice, s));
  if (st.rows32) QK_HIP(hipMemcpyAsync(fresh.rows32, st.rows32, used * st.dp * sizeof(float), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipMemcpyAsync(fresh.ids, st.ids, used * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  if (st.attr) QK_HIP(hipMemcpyAsync(fresh.attr, st.attr, used * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  if (st.codes)
    QK_HIP(hipMemcpyAsync(fresh.codes, st.codes, used * qk::pq_words(st.pq_m) * sizeof(uint32_t),
                          hipMemcpyDeviceToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  for (void* p : {(void*)st.v32, (void*)st.v16, (void*)st.v16n, (void*)st.rows32, (void*)st.ids, (void*)st.attr,
                  (void*)st.codes})
    idx->mem.release(p);
  st.v32 = fresh.v32;
  st.v16 = fresh.v16;
  st.v16n = fresh.v16n;
  st.rows32 = fresh.rows32;
  st.ids = fresh.ids;
  st.attr = fresh.attr;
  st.codes = fresh.codes;
  st.tiles = tiles;
  st.tile_part.resize(tiles, -1);
  return false;
}

// Copy partition p's filled tiles to `tiles` fresh tiles at the end of the
// arena (which must have room) and give it capacity `cap`.
void relocate(Store& st, int64_t p, int32_t cap, hipStream_t s) {
  const int64_t from = st.off[p], to = st.used_tiles;
  const int64_t ntiles = (st.size[p] + qk::TILE - 1) / qk::TILE;
  const size_t n = (size_t)ntiles * qk::TILE;
  const size_t a = (size_t)from * qk::TILE, b = (size_t)to * qk::TILE;
  if (n > 0) {
    if (st.v32)
      QK_HIP(hipMemcpyAsync(st.v32 + b * st.dp, st.v32 + a * st.dp, n * st.dp * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
    if (st.v16)
      QK_HIP(hipMemcpyAsync(st.v16 + b * st.dp16, st.v16 + a * st.dp16, n * st.dp16 * sizeof(uint16_t),
                            hipMemcpyDeviceToDevice, s));
    if (st.v16n) QK_HIP(hipMemcpyAsync(st.v16n + b, st.v16n + a, n * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (st.rows32)
      QK_HIP(hipMemcpyAsync(st.rows32 + b * st.dp, st.rows32 + a * st.dp, n * st.dp * sizeof(float),
                            hipMemcpyDeviceToDevice, s));
    QK_HIP(hipMemcpyAsync(st.ids + b, st.ids + a, n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    if (st.attr) QK_HIP(hipMemcpyAsync(st.attr + b, st.attr + a, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    if (st.codes) {
      const size_t w = (size_t)qk::pq_words(st.pq_m);
      QK_HIP(hipMemcpyAsync(st.codes + b * w, st.codes + a * w, n * w * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    // the old slots no longer hold the partition's vectors
    QK_HIP(hipMemsetAsync(st.ids + a, 0xff, (size_t)st.cap[p] * sizeof(int64_t), s));
  }
  for (int64_t t = 0; t < st.cap[p] / qk::TILE; ++t) st.tile_part[from + t] = -1;
  for (int64_t t = 0; t < cap / qk::TILE; ++t) st.tile_part[to + t] = (int32_t)p;
  st.off[p] = to;
  st.cap[p] = cap;
  st.used_tiles += cap / qk::TILE;
}

// Fill the holes (deleted slots, id -1) below the live count of every
// partition p with which[p] set from the partition's live tail, so that its
// first size - tomb slots hold its vectors; moved vectors keep their ids.
void compact(quake_index* idx, Store& st, qk::IdMap& map, const std::vector<char>& which, hipStream_t s) {
  std::vector<int64_t> src, dst, moved_ids;
  for (int64_t p = 0; p < st.nlist; ++p) {
    if (!which[p] || st.tomb[p] == 0) continue;
    const int64_t base = st.off[p] * qk::TILE;
    const int64_t size = st.size[p];
    std::vector<int64_t> pid(size);
    QK_HIP(hipMemcpyAsync(pid.data(), st.ids + base, size * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    const int64_t keep = size - st.tomb[p];
    int64_t hole = 0, tail = keep;
    while (true) {
      while (hole < keep && pid[hole] >= 0) ++hole;
      while (tail < size && pid[tail] < 0) ++tail;
      if (hole >= keep || tail >= size) break;
      src.push_back(base + tail);
      dst.push_back(base + hole);
      moved_ids.push_back(pid[tail]);
      ++hole;
      ++tail;
    }
    st.size[p] = (int32_t)keep;
    st.tomb[p] = 0;
  }
  if (!src.empty()) {
    const int64_t m = (int64_t)src.size();
    Tmp<int64_t> d_src(idx->mem, m), d_dst(idx->mem, m), d_ids(idx->mem, m);
    QK_HIP(hipMemcpyAsync(d_src.p, src.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s));
    QK_HIP(hipMemcpyAsync(d_dst.p, dst.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s));
    QK_HIP(hipMemcpyAsync(d_ids.p, moved_ids.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s));
    qk::launch_move_slots(st, d_src.p, d_dst.p, m, s);
    qk::launch_map_update(map, d_ids.p, d_dst.p, m, s);
    QK_HIP(hipStreamSynchronize(s));
  }
}

// ---------------------------------------------------------------- id map

void map_rebuild(quake_index* idx, qk::IdMap& m, const Store& st, int64_t expect, hipStream_t s) {
  uint64_t cap = 1024;
  while (cap < (uint64_t)std::max<int64_t>(expect, 1) * 4) cap <<= 1;
  int64_t* keys = idx->mem.alloc<int64_t>(cap);
  int64_t* vals;
  try {
    vals = idx->mem.alloc<int64_t>(cap);
  } catch (...) {
    idx->mem.release(keys);
    throw;
  }
  idx->mem.release(m.keys);
  idx->mem.release(m.vals);
  m.keys = keys;
  m.vals = vals;
  m.mask = cap - 1;
  QK_HIP(hipMemsetAsync(m.keys, 0xff, cap * sizeof(int64_t), s));
  qk::launch_map_insert_store(m, st.ids, st.used_tiles * qk::TILE, s);
  m.used = st.live;
}

int64_t count_missing(quake_index* idx, const qk::IdMap& m, const int64_t* ids, int64_t n, int64_t* slots,
                      hipStream_t s) {
  Tmp<int64_t> miss(idx->mem, 1);
  QK_HIP(hipMemsetAsync(miss.p, 0, sizeof(int64_t), s));
  qk::launch_map_find(m, ids, n, slots, miss.p, s);
  int64_t h = 0;
  QK_HIP(hipMemcpyAsync(&h, miss.p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  return h;
}

// ---------------------------------------------------------------- input checks

// The index's check flag is cleared, a check kernel sets it, and the host
// reads it back before any work that depends on the input.
void clear_flag(quake_index* idx, hipStream_t s) {
  QK_HIP(hipMemsetAsync(idx->d_flag, 0, sizeof(uint32_t), s));
}

bool flag_set(quake_index* idx, hipStream_t s) {
  QK_HIP(hipMemcpyAsync(idx->h_flag, idx->d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  return *idx->h_flag != 0;
}

void require_finite(quake_index* idx, const float* x, int64_t count, const char* what, hipStream_t s) {
  clear_flag(idx, s);
  qk::launch_nonfinite(x, count, idx->d_flag, s);
  QK_CHECK(!flag_set(idx, s), QUAKE_E_INVALID, std::string(what) + " holds a non-finite value");
}

// ---------------------------------------------------------------- searches

}  // namespace

namespace qk {

// Product codes of the rows at `slots` (partition parts[i]): their residuals
// to the partition centroids, read from the row-major FP32 copy.
void encode_rows(quake_index* idx, const Store& st, const int64_t* slots, const int32_t* parts, int64_t n,
                     hipStream_t s) {
  if (!st.codes || n <= 0) return;
  qk::launch_pq_encode(st.rows32, st.dp, slots, parts, n, st.centroids, idx->pq_book, st.pq_m, idx->pq_ds,
                       idx->metric, st.codes, s);
}

// Product codes of every live row of `st` again (after its partitions or
// centroids changed).
void encode_store(quake_index* idx, const Store& st, hipStream_t s) {
  if (!st.codes || st.live <= 0) return;
  std::vector<int64_t> sid((size_t)st.tiles * qk::TILE);
  QK_HIP(hipMemcpyAsync(sid.data(), st.ids, sid.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  std::vector<int64_t> slots;
  std::vector<int32_t> parts;
  slots.reserve(st.live);
  parts.reserve(st.live);
  for (int64_t p = 0; p < st.nlist; ++p)
    for (int64_t j = 0; j < st.size[p]; ++j)
      if (sid[st.off[p] * qk::TILE + j] >= 0) {
        slots.push_back(st.off[p] * qk::TILE + j);
        parts.push_back((int32_t)p);
      }
  Tmp<int64_t> d_slots(idx->mem, std::max<size_t>(slots.size(), 1));
  Tmp<int32_t> d_parts(idx->mem, std::max<size_t>(parts.size(), 1));
  QK_HIP(hipMemcpyAsync(d_slots.p, slots.data(), slots.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  QK_HIP(hipMemcpyAsync(d_parts.p, parts.data(), parts.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  encode_rows(idx, st, d_slots.p, d_parts.p, (int64_t)slots.size(), s);
  QK_HIP(hipStreamSynchronize(s));
}

void store_grow_arena(quake_index* idx, Store& st, int64_t need, hipStream_t s) { grow_arena(idx, st, need, s, false); }
void store_relocate(Store& st, int64_t p, int32_t cap, hipStream_t s) { relocate(st, p, cap, s); }
void store_upload_table(Store& st, hipStream_t s) { upload_table(st, s); }
void store_compact(quake_index* idx, Store& st, const std::vector<char>& which, hipStream_t s) {
  compact(idx, st, idx->idmap, which, s);
}
int store_fixed_point_bits(DeviceMemory& mem, const float* x, int64_t n, int dp, hipStream_t s) {
  return fixed_point_bits(mem, x, n, dp, s);
}

// Insert n rows x[n][d] with ids into the level-0 store `st` and its id map
// (routed: the partition of every row, else each goes to its nearest
// centroid).  The batch is checked whole before anything changes: ids >= 0,
// no id twice, none already present.  Partitions that overflow move to fresh
// tiles with 1.5x their need.
void insert_rows(quake_index* idx, Store& st, IdMap& map, const float* x, const int64_t* ids, int64_t n,
                 const std::vector<int32_t>* routed, hipStream_t s, const uint32_t* attrs) {
  QK_CHECK(!st.attr || attrs, QUAKE_E_INVALID, "the index labels its rows: insert them with their label bits");
  QK_CHECK(st.attr || !attrs, QUAKE_E_INVALID, "the index was built without row labels");
  std::vector<int64_t> h_ids(n);
  QK_HIP(hipMemcpyAsync(h_ids.data(), ids, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  QK_CHECK(std::all_of(h_ids.begin(), h_ids.end(), [](int64_t v) { return v >= 0; }), QUAKE_E_INVALID,
           "ids must be >= 0");
  {
    std::vector<int64_t> sorted(h_ids);
    std::sort(sorted.begin(), sorted.end());
    QK_CHECK(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(), QUAKE_E_DUPLICATE,
             "the batch repeats an id");
  }
  QK_CHECK(count_missing(idx, map, ids, n, nullptr, s) == n, QUAKE_E_DUPLICATE,
           "the batch names an id already present");
  const int dp = idx->dp;
  std::vector<int32_t> part(n);
  if (routed) {
    part = *routed;
  } else {
    std::unique_ptr<Tmp<float>> xpad_buf;
    const float* xpad = x;
    if (dp != idx->d) {
      xpad_buf.reset(new Tmp<float>(idx->mem, (size_t)n * dp));
      launch_pad_rows(x, n, idx->d, dp, xpad_buf->p, nullptr, s);
      xpad = xpad_buf->p;
    }
    Tmp<int32_t> assign(idx->mem, n);
    launch_assign(xpad, n, dp, st.centroids, st.nlist, idx->metric, assign.p, s);
    QK_HIP(hipMemcpyAsync(part.data(), assign.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
  }
  std::vector<int64_t> cnt(st.nlist, 0);
  for (int64_t i = 0; i < n; ++i) cnt[part[i]]++;
  std::vector<std::pair<int64_t, int32_t>> moves;
  int64_t extra = 0;
  for (int64_t p = 0; p < st.nlist; ++p) {
    if (cnt[p] == 0 || st.size[p] + cnt[p] <= st.cap[p]) continue;
    const int64_t want = round_up((int64_t)std::ceil((st.size[p] + cnt[p]) * 1.5), TILE);
    QK_CHECK(want <= INT32_MAX, QUAKE_E_INVALID, "partition too large");
    moves.push_back({p, (int32_t)want});
    extra += want / TILE;
  }
  const bool repacked = grow_arena(idx, st, st.used_tiles + extra, s, true);
  for (auto& mv : moves) relocate(st, mv.first, mv.second, s);
  std::vector<int64_t> slot(n);
  std::vector<int64_t> fill(st.nlist, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t p = part[i];
    slot[i] = st.off[p] * TILE + st.size[p] + fill[p]++;
  }
  Tmp<int64_t> d_slot(idx->mem, n);
  QK_HIP(hipMemcpyAsync(d_slot.p, slot.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s));
  launch_scatter(x, n, idx->d, dp, st.dp16, ids, d_slot.p, st.v32, st.v16, st.v16 ? idx->storage : QUAKE_F32,
                 st.rows32, st.ids, s);
  launch_norm16_slots(st, d_slot.p, n, idx->storage, s);
  std::unique_ptr<Tmp<int32_t>> d_part;
  if (st.codes) {
    d_part.reset(new Tmp<int32_t>(idx->mem, n));
    QK_HIP(hipMemcpyAsync(d_part->p, part.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    encode_rows(idx, st, d_slot.p, d_part->p, n, s);
  }
  if (st.attr) {
    launch_put_u32(attrs, d_slot.p, n, st.attr, s);
    st.attr_dirty = true;
  }
  for (int64_t p = 0; p < st.nlist; ++p) st.size[p] += (int32_t)cnt[p];
  upload_table(st, s);
  st.live += n;
  if (repacked || !moves.empty() || (map.used + n) * 2 > (int64_t)map.mask + 1) {
    map_rebuild(idx, map, st, st.live, s);
  } else {
    launch_map_insert(map, ids, d_slot.p, n, s);
    map.used += n;
  }
  QK_HIP(hipStreamSynchronize(s));
}

// Delete the rows with the n given ids from `st` and its id map (the batch is
// rejected whole, NOTFOUND, when an id repeats or is absent).  Deleted slots
// hold id -1; a partition with a quarter of its slots deleted is compacted.
void delete_rows(quake_index* idx, Store& st, IdMap& map, const int64_t* ids, int64_t n, hipStream_t s) {
  std::vector<int64_t> h_ids(n);
  QK_HIP(hipMemcpyAsync(h_ids.data(), ids, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  {
    std::vector<int64_t> sorted(h_ids);
    std::sort(sorted.begin(), sorted.end());
    QK_CHECK(std::adjacent_find(sorted.begin(), sorted.end()) == sorted.end(), QUAKE_E_NOTFOUND,
             "the batch repeats an id");
  }
  Tmp<int64_t> slots(idx->mem, n);
  QK_CHECK(count_missing(idx, map, ids, n, slots.p, s) == 0, QUAKE_E_NOTFOUND,
           "the batch names an id that is absent");
  launch_mark_deleted(st, slots.p, n, s);
  launch_map_erase(map, ids, n, s);
  st.attr_dirty = true;
  std::vector<int64_t> h_slots(n);
  QK_HIP(hipMemcpyAsync(h_slots.data(), slots.p, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  st.live -= n;
  std::vector<char> touched(st.nlist, 0);
  for (int64_t sl : h_slots) {
    const int32_t p = st.tile_part[sl / TILE];
    st.tomb[p]++;
    touched[p] = 1;
  }
  for (int64_t p = 0; p < st.nlist; ++p)
    if (touched[p] && st.tomb[p] * 4 < st.size[p]) touched[p] = 0;
  compact(idx, st, map, touched, s);
  upload_table(st, s);
  QK_HIP(hipStreamSynchronize(s));
}

int64_t max_chunks(const Store& st, int chunk_tiles) {
  int64_t mx = 1;
  for (int32_t sz : st.size) {
    const int64_t t = (sz + qk::TILE - 1) / qk::TILE;
    mx = std::max<int64_t>(mx, (t + chunk_tiles - 1) / chunk_tiles);
  }
  return mx;
}

Job resolve(const quake_index* idx, const Store& st, const quake_search_params* p) {
  QK_CHECK(p, QUAKE_E_INVALID, "params is NULL");
  QK_CHECK(p->k >= 1 && p->k <= qk::KMAX, QUAKE_E_INVALID, "k must be in [1, 256]");
  const bool has_np = p->nprobe > 0;
  const bool has_rt = p->recall_target > 0.0;
  QK_CHECK(has_np != has_rt, QUAKE_E_INVALID, "set exactly one of nprobe > 0 or recall_target > 0");
  QK_CHECK(!has_rt || p->recall_target <= 1.0, QUAKE_E_INVALID, "recall_target must be in (0, 1]");
  QK_CHECK(p->scan_mode == QUAKE_SCAN_PLAIN || p->scan_mode == QUAKE_SCAN_BATCHED, QUAKE_E_INVALID,
           "unknown scan_mode");
  const bool pq = p->scan_dtype == QUAKE_PQ8;
  QK_CHECK(p->scan_dtype == QUAKE_F32 || (p->scan_dtype == idx->storage && st.v16) || (pq && st.codes),
           QUAKE_E_INVALID, "scan_dtype needs the matching reduced-precision copy (or product codes) in the index");
  QK_CHECK(p->f_M >= 0 && p->tau_rho >= 0 && p->upper_f_M >= 0 && p->upper_recall_target >= 0 &&
               p->upper_recall_target <= 1.0 && p->window >= 0,
           QUAKE_E_INVALID, "negative or out-of-range search parameter");
  QK_CHECK(p->estimator >= QUAKE_EST_APS && p->estimator <= QUAKE_EST_APS_RP, QUAKE_E_INVALID, "unknown estimator");
  Job r;
  r.k = p->k;
  r.batched = p->scan_mode == QUAKE_SCAN_BATCHED ? 1 : 0;
  r.dtype16 = p->scan_dtype;
  QK_CHECK(r.batched == (p->scan_dtype != QUAKE_F32 && !pq ? 1 : 0), QUAKE_E_INVALID,
           "the batched scan runs on the 16-bit copy (scan_dtype BF16/F16) and the plain scan on FP32 or on "
           "product codes (PQ8)");
  QK_CHECK(r.batched || pq || st.v32, QUAKE_E_INVALID,
           "the index keeps no FP32 tile copy (drop_f32_tiles): search with the batched scan or product codes");
  QK_CHECK(p->rerank_factor >= -1, QUAKE_E_INVALID, "rerank_factor must be >= -1");
  QK_CHECK(p->rerank_factor >= 0 || r.batched, QUAKE_E_INVALID, "rerank_factor -1 is for the batched scan");
  r.rerank = p->rerank_factor >= 0 ? 1 : 0;
  r.kk = r.batched || pq ? (r.rerank ? std::max(p->rerank_factor > 0 ? p->rerank_factor : 4, 1) * r.k : r.k) : r.k;
  QK_CHECK(!(r.batched || pq) || r.kk <= 64, QUAKE_E_INVALID,
           "the batched scan and the scan over product codes keep at most 64 candidates per query");
  QK_CHECK(!r.batched || st.dp16 <= 1024, QUAKE_E_INVALID, "the batched scan supports d <= 1024");
  r.aps = has_rt ? 1 : 0;
  r.tau_r = p->recall_target;
  r.f_M = p->f_M > 0 ? p->f_M : 0.05;
  r.tau_rho = p->tau_rho > 0 ? p->tau_rho : 0.01;
  r.est = p->estimator;
  QK_CHECK(!p->filter || (st.attr && idx->n_levels == 1 && r.kk <= qk::KMAX), QUAKE_E_INVALID,
           "a filtered search needs a labelled one-level index");
  r.filter = p->filter;
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

void ensure_queries(quake_index* idx, int64_t nq) {
  qk::Workspace& w = idx->ws;
  auto& mem = idx->mem;
  const int dp = idx->dp;
  if (nq <= w.nq_cap && w.q) return;
  const int64_t n = std::max<int64_t>(nq, 1);
  for (void* p : {(void*)w.q, (void*)w.qn2, (void*)w.st_m, (void*)w.st_w, (void*)w.st_weff, (void*)w.st_done,
                  (void*)w.st_item, (void*)w.st_demand, (void*)w.st_vecs, (void*)w.st_pair, (void*)w.st_rho,
                  (void*)w.st_p0, (void*)w.st_V, (void*)w.st_vsum, (void*)w.st_r, (void*)w.q16, (void*)w.qn2f,
                  (void*)w.mq, (void*)w.mq0, (void*)w.blk})
    mem.release(p);
  w.q = mem.alloc<float>((size_t)n * dp);
  w.qn2 = mem.alloc<double>(n);
  w.st_m = mem.alloc<int32_t>(n);
  w.st_w = mem.alloc<int32_t>(n);
  w.st_weff = mem.alloc<int32_t>(n);
  w.st_done = mem.alloc<int32_t>(n);
  w.st_item = mem.alloc<int64_t>(n);
  w.st_demand = mem.alloc<int64_t>(n);
  w.blk = mem.alloc<int64_t>((n / 256 + 1) * 4);
  w.st_vecs = mem.alloc<int64_t>(n);
  w.st_pair = mem.alloc<int64_t>(n);
  w.q16 = nullptr;
  w.q16_dim = 0;
  w.qn2f = mem.alloc<float>(n);
  w.mq = mem.alloc<int32_t>(n);
  w.mq0 = mem.alloc<int32_t>(n);
  w.st_rho = mem.alloc<double>(n);
  w.st_p0 = mem.alloc<double>(n);
  w.st_V = mem.alloc<double>(n);
  w.st_vsum = mem.alloc<double>(n);
  w.st_r = mem.alloc<double>(n);
  w.nq_cap = n;
  // sizes that scale with nq re-grow on demand
  w.scores_cap = w.cand_cap = w.kk_cap = w.cand0_cap = 0;
  for (void* p : {(void*)w.scores, (void*)w.sel, (void*)w.cand, (void*)w.h, (void*)w.rk, (void*)w.ri,
                  (void*)w.cand0})
    mem.release(p);
  w.scores = nullptr;
  w.sel = w.cand = w.cand0 = nullptr;
  w.h = nullptr;
  w.rk = nullptr;
  w.ri = nullptr;
}

void ensure_workspace(quake_index* idx, int64_t nc, int64_t M, int64_t kk, int64_t items, int64_t pairs,
                      int dp16, bool scores) {
  qk::Workspace& w = idx->ws;
  auto& mem = idx->mem;
  if (scores) grow(mem, w.scores, w.scores_cap, w.nq_cap * nc);
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
    mem.release(w.items); mem.release(w.pk); mem.release(w.pi); mem.release(w.bitems); mem.release(w.xitem);
    w.items = nullptr; w.pk = nullptr; w.pi = nullptr; w.bitems = nullptr; w.xitem = nullptr;
    w.items_cap = std::max(items, w.items_cap);
    w.k_cap = std::max<int64_t>(kk, w.k_cap);
    w.items = mem.alloc<int4>(w.items_cap);
    // batched items never outnumber the plain ones (one per query set, not per query)
    w.bitems = mem.alloc<int4>(2 * w.items_cap);
    w.xitem = mem.alloc<int64_t>(w.items_cap);
    w.pk = mem.alloc<float>((size_t)w.items_cap * w.k_cap);
    w.pi = mem.alloc<int64_t>((size_t)w.items_cap * w.k_cap);
  }
  if (!w.total) {
    w.total = mem.alloc<int64_t>(qk::COUNTERS);
    QK_HIP(hipHostMalloc((void**)&w.h_total, qk::COUNTERS * sizeof(int64_t), hipHostMallocDefault));
  }
  if (dp16 > 0 && (!w.q16 || dp16 > w.q16_dim)) {
    mem.release(w.q16);
    w.q16 = mem.alloc<uint16_t>((size_t)w.nq_cap * dp16);
    w.q16_dim = dp16;
  }
  if (pairs > w.pairs_cap || !w.pair_q) {
    for (void* p : {(void*)w.pair_q, (void*)w.pair_p, (void*)w.pair_pos, (void*)w.pair_base, (void*)w.sorted,
                    (void*)w.sorted_q, (void*)w.sorted_base})
      mem.release(p);
    w.pairs_cap = std::max<int64_t>(pairs, 1);
    w.pair_q = mem.alloc<int32_t>(w.pairs_cap);
    w.pair_p = mem.alloc<int32_t>(w.pairs_cap);
    w.pair_pos = mem.alloc<int32_t>(w.pairs_cap);
    w.pair_base = mem.alloc<int64_t>(w.pairs_cap);
    w.sorted = mem.alloc<int32_t>(w.pairs_cap);
    w.sorted_q = mem.alloc<int32_t>(w.pairs_cap);
    w.sorted_base = mem.alloc<int64_t>(w.pairs_cap);
  }
  if (nc + 1 > w.parts_cap || !w.pcount) {
    for (void* p : {(void*)w.pcount, (void*)w.pstart, (void*)w.pitem, (void*)w.pxoff, (void*)w.pxcd}) mem.release(p);
    w.parts_cap = nc + 1;
    w.pcount = mem.alloc<int32_t>(w.parts_cap);
    w.pstart = mem.alloc<int32_t>(w.parts_cap);
    w.pitem = mem.alloc<int64_t>(w.parts_cap);
    w.pxoff = mem.alloc<int64_t>(w.parts_cap);
    w.pxcd = mem.alloc<int32_t>(w.parts_cap);
    QK_HIP(hipMemset(w.pcount, 0, w.parts_cap * sizeof(int32_t)));
  }
}

int scan_blocks(quake_index* idx, int batched) {
  if (idx->cu_count == 0) {
    int dev = 0;
    QK_HIP(hipGetDevice(&dev));
    QK_HIP(hipDeviceGetAttribute(&idx->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
  }
  const int per = idx->tune.blocks_per_cu > 0 ? idx->tune.blocks_per_cu : (batched ? 1 : 8);
  return std::max(idx->cu_count, 8) * per;
}

namespace {

void launch_rounds(quake_index* idx, const Store& st, const Job& job, const RoundArgs& a, int R, hipStream_t s) {
  Workspace& w = idx->ws;
  for (int r = 0; r < R; ++r) {
    if (job.batched) {
      {
        ProfileScope ps(idx->prof, QUAKE_PROF_PLAN, s);
        launch_group(w, st, a, s);
      }
      ProfileScope ps(idx->prof, QUAKE_PROF_SCAN, s);
      launch_scan_mfma(w, st, a, job.dtype16, s);
    } else {
      {
        ProfileScope ps(idx->prof, QUAKE_PROF_PLAN, s);
        launch_emit(w, st, a, s);
      }
      ProfileScope ps(idx->prof, QUAKE_PROF_SCAN, s);
      if (job.dtype16 == QUAKE_PQ8) launch_scan_pq(w, st, a, s);
      else launch_scan_f32(w, st, a, s);
    }
    {
      ProfileScope ps(idx->prof, QUAKE_PROF_COMMIT, s);
      launch_commit(w, st, a, idx->cap_table, s);
    }
    ProfileScope ps(idx->prof, QUAKE_PROF_PLAN, s);
    launch_demand(w, st, a, s);
  }
}

std::vector<uint64_t> graph_key(const quake_index* idx, const Store& st, const Job& job, const RoundArgs& a, int R) {
  const Workspace& w = idx->ws;
  auto u = [](const void* p) { return (uint64_t)(uintptr_t)p; };
  std::vector<uint64_t> k = {
      (uint64_t)R, (uint64_t)job.batched, (uint64_t)job.dtype16, (uint64_t)a.nq, (uint64_t)a.M, (uint64_t)a.k,
      (uint64_t)a.kk, (uint64_t)a.aps, (uint64_t)a.chunk_tiles, (uint64_t)a.wmax, (uint64_t)a.wscale, (uint64_t)a.metric,
      (uint64_t)a.items_cap, (uint64_t)a.blocks, (uint64_t)a.slot_ids, u(a.hits), u(a.slot_tag), (uint64_t)a.tag, (uint64_t)st.d, (uint64_t)st.dp, (uint64_t)st.nlist,
      (uint64_t)st.dp16, u(idx->cap_table), u(st.centroids), u(st.d_off), u(st.d_size), u(st.d_cap), u(st.d_order), u(st.v32),
      u(st.v16), u(st.v16n), u(st.rows32), u(st.ids), u(w.q), u(w.qn2), u(w.cand), u(w.mq), u(w.h), u(w.st_m),
      u(w.st_w), u(w.st_weff), u(w.st_done), u(w.st_item), u(w.st_demand), u(w.st_rho), u(w.st_p0), u(w.st_V),
      u(w.st_vsum), u(w.st_r), u(w.rk), u(w.ri), u(w.items), u(w.pk), u(w.pi), u(w.st_vecs), u(w.st_pair),
      u(w.q16), u(w.qn2f), u(w.pair_q), u(w.pair_p), u(w.pair_pos), u(w.pair_base), u(w.sorted), u(w.sorted_q), u(w.sorted_base), u(w.bitems), u(w.pcount),
      u(w.pstart), u(w.pitem), u(w.pxoff), u(w.pxcd), u(w.xitem), u(w.total), u(w.blk)};
  uint64_t tr, tro;
  std::memcpy(&tr, &a.tau_r, 8);
  std::memcpy(&tro, &a.tau_rho, 8);
  k.push_back(tr);
  k.push_back(tro);
  k.push_back((uint64_t)a.est);
  k.push_back(u(a.qmask));
  k.push_back(u(a.attr));
  k.push_back(u(st.codes));
  k.push_back((uint64_t)st.pq_m);
  k.push_back(u(w.lut));
  k.push_back(u(a.attr_cnt));
  return k;
}

}  // namespace

void release_graphs(quake_index* idx) {
  for (auto& g : idx->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  idx->graphs.clear();
}

// R rounds, replayed from a captured HIP graph when possible (profiling needs
// events around each kernel class, so it launches directly).  A graph is
// captured once per distinct set of kernel arguments; the captured rounds
// contain kernel launches only.
void run_rounds(quake_index* idx, const Store& st, const Job& job, const RoundArgs& a, int R, hipStream_t s) {
  if (idx->prof.on || idx->tune.no_graph || idx->graphs_failed || idx->noalloc) {
    launch_rounds(idx, st, job, a, R, s);
    return;
  }
  std::vector<uint64_t> key = graph_key(idx, st, job, a, R);
  hipGraphExec_t exec = nullptr;
  for (auto& g : idx->graphs)
    if (g.key == key) { exec = g.exec; break; }
  if (!exec) {
    if (!idx->capture_stream) QK_HIP(hipStreamCreateWithFlags(&idx->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(idx->capture_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      launch_rounds(idx, st, job, a, R, idx->capture_stream);
      ok = hipStreamEndCapture(idx->capture_stream, &graph) == hipSuccess && graph;
    }
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess && exec;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok) {  // capture is an optimisation only: launch directly from now on
      idx->graphs_failed = true;
      launch_rounds(idx, st, job, a, R, s);
      return;
    }
    if (idx->graphs.size() >= 16) {
      (void)hipGraphExecDestroy(idx->graphs.front().exec);
      idx->graphs.erase(idx->graphs.begin());
    }
    idx->graphs.push_back({std::move(key), exec});
  }
  QK_HIP(hipGraphLaunch(exec, s));
}

}  // namespace qk

quake_index::~quake_index() {
  qk::release_graphs(this);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  if (ws.h_total) (void)hipHostFree(ws.h_total);
  if (h_flag) (void)hipHostFree(h_flag);
}

namespace {

using qk::candidate_count;
using qk::ensure_queries;
using qk::ensure_workspace;
using qk::Job;
using qk::max_chunks;
using qk::resolve;

// Point the workspace's query rows at a sub-range for the duration of a scope.
struct QueryWindow {
  qk::Workspace& w;
  float* q;
  double* qn2;
  QueryWindow(qk::Workspace& w_, int64_t first, int dp) : w(w_), q(w_.q), qn2(w_.qn2) {
    w.q += first * dp;
    w.qn2 += first;
  }
  ~QueryWindow() {
    w.q = q;
    w.qn2 = qn2;
  }
};

// Run one resolved search over `st` for the nq queries in ws.q / ws.qn2.
// Leaves the results in ws.rk / ws.ri ([nq][kk]) and the per-query state in
// ws.st_*; writes the outputs when out_ids is given.
}  // namespace

namespace qk {

int search_chunk_tiles(const quake_index* idx, const Job& job) {
  int chunk_tiles = idx->tune.chunk_tiles > 0 ? idx->tune.chunk_tiles : 16;
  // long result lists are scanned by sorting whole items in LDS
  if (job.kk > qk::KMAX) chunk_tiles = std::min(chunk_tiles, qk::SORTED_ITEM_MAX / qk::TILE);
  return chunk_tiles;
}

int64_t search_items(const quake_index* idx, const Store& st, const Job& job, int64_t nq) {
  const int64_t mc = max_chunks(st, search_chunk_tiles(idx, job));
  // the buffer must hold one full window of the largest partitions (progress)
  const int64_t floor_items = (int64_t)job.wmax * mc + 1;
  // by default room for every query's first window twice over, and on the
  // batched path for a whole round of largest windows (partitions there are
  // mostly one chunk): a round that runs out of items defers queries to a
  // further round, which reads the partitions it touches once more
  const int64_t def_items = nq * (int64_t)std::max(std::max(job.w0, 4) * 2, job.batched ? job.wmax : 0);
  return std::max<int64_t>(idx->tune.max_items > 0 ? idx->tune.max_items : def_items, floor_items);
}

// Byte layout of a search workspace for nq queries (every array of
// ensure_queries and ensure_workspace, 256-byte aligned) inside `base`; with
// w == nullptr only the size is computed.  Host counters are not part of it.
size_t workspace_layout(Workspace* w, char* base, int64_t nq, int64_t nc, int64_t M, int64_t kk, int64_t items,
                        int64_t pairs, int dp, int dp16) {
  size_t off = 0;
  auto take = [&](auto*& p, int64_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(p)>>;
    off = (off + 255) / 256 * 256;
    if (w) p = reinterpret_cast<T*>(base + off);
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
  };
  Workspace dummy;
  Workspace& x = w ? *w : dummy;
  const int64_t n = std::max<int64_t>(nq, 1);
  take(x.q, n * dp);
  take(x.qn2, n);
  for (int32_t** p : {&x.st_m, &x.st_w, &x.st_weff, &x.st_done, &x.mq, &x.mq0}) take(*p, n);
  for (int64_t** p : {&x.st_item, &x.st_demand, &x.st_vecs, &x.st_pair}) take(*p, n);
  take(x.blk, (n / 256 + 1) * 4);
  take(x.qn2f, n);
  for (double** p : {&x.st_rho, &x.st_p0, &x.st_V, &x.st_vsum, &x.st_r}) take(*p, n);
  take(x.scores, n * nc);
  take(x.sel, n * M);
  take(x.cand, n * M);
  take(x.h, n * M);
  take(x.rk, n * kk);
  take(x.ri, n * kk);
  take(x.items, items);
  take(x.bitems, 2 * items);
  take(x.xitem, items);
  take(x.pk, items * kk);
  take(x.pi, items * kk);
  take(x.total, COUNTERS);
  if (dp16 > 0) take(x.q16, n * dp16);
  for (int32_t** p : {&x.pair_q, &x.pair_p, &x.pair_pos, &x.sorted, &x.sorted_q}) take(*p, pairs);
  for (int64_t** p : {&x.pair_base, &x.sorted_base}) take(*p, pairs);
  take(x.pcount, nc + 1);
  take(x.pstart, nc + 1);
  take(x.pitem, nc + 1);
  take(x.pxoff, nc + 1);
  take(x.pxcd, nc + 1);
  if (w) {
    w->nq_cap = n;
    w->scores_cap = n * nc;
    w->cand_cap = n * M;
    w->kk_cap = n * kk;
    w->items_cap = items;
    w->k_cap = kk;
    w->q16_dim = dp16;
    w->pairs_cap = std::max<int64_t>(pairs, 1);
    w->parts_cap = nc + 1;
    w->cand0 = nullptr;
    w->cand0_cap = 0;
  }
  return (off + 255) / 256 * 256;
}

}  // namespace qk

namespace {

void run_search(quake_index* idx, const Store& st, const Job& job, int64_t nq, int64_t* out_ids, float* out_dist,
                int32_t* out_nscanned, double* out_recall, hipStream_t s) {
  const int chunk_tiles = qk::search_chunk_tiles(idx, job);
  const int64_t items = qk::search_items(idx, st, job, nq);
  ensure_workspace(idx, st.nlist, job.M, job.kk, items, job.batched ? nq * (int64_t)job.wmax : 0,
                   job.batched ? st.dp16 : 0, !job.given);
  qk::Workspace& w = idx->ws;
  // (a fill kernel, not a memset: a caller may capture this call's stream)
  qk::launch_fill_i32(reinterpret_cast<int32_t*>(w.total), 2 * qk::COUNTERS, 0, s);
  if (job.given) {
    QK_HIP(hipMemcpyAsync(w.mq, w.mq0, nq * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    qk::ProfileScope ps(idx->prof, QUAKE_PROF_SELECT, s);
    qk::launch_geometry(w.q, st.centroids, nq, idx->dp, job.M, w.mq, idx->metric, w.cand0, w.cand, w.h, s);
  } else {
    qk::launch_fill_i32(w.mq, nq, job.M, s);
    {
      qk::ProfileScope ps(idx->prof, QUAKE_PROF_CENTROIDS, s);
      qk::launch_scores(w.q, nq, st.centroids, st.nlist, idx->dp, idx->metric, w.scores, s);
    }
    idx->prof.add(QUAKE_PROF_CENTROIDS, ((double)st.nlist + nq) * idx->dp * 4.0 + (double)nq * st.nlist * 4.0,
                  (double)nq * st.nlist * idx->dp * (idx->metric == QUAKE_L2 ? 3.0 : 2.0));
    qk::ProfileScope ps(idx->prof, QUAKE_PROF_SELECT, s);
    qk::launch_candidates(st, w.q, w.scores, nq, idx->dp, job.M, job.aps, idx->metric, w.mq, w.sel, w.cand, w.h, s);
  }
  if (job.batched) qk::launch_queries16(w, nq, idx->dp, st.dp16, job.dtype16, s);
  const bool pq = job.dtype16 == QUAKE_PQ8;
  if (pq) {
    const int64_t need = nq * (int64_t)st.pq_m * 256;
    if (need > w.lut_cap || !w.lut) {
      idx->mem.release(w.lut);
      w.lut = nullptr;
      w.lut = idx->mem.alloc<float>(std::max<int64_t>(need, 1));
      w.lut_cap = need;
    }
    qk::ProfileScope ps(idx->prof, QUAKE_PROF_SELECT, s);
    qk::launch_pq_lut(w.q, nq, idx->dp, idx->pq_book, st.pq_m, idx->pq_ds, idx->metric, w.lut, s);
  }
  qk::RoundArgs a{};
  a.nq = nq;
  a.M = job.M;
  a.k = job.k;
  a.kk = job.kk;
  a.aps = job.aps;
  a.chunk_tiles = chunk_tiles;
  a.wmax = job.wmax;
  a.wscale = idx->tune.window_scale > 0 ? idx->tune.window_scale : 100;
  // the batched scan and the scan over codes carry store slots (the rerank reads rows by slot)
  a.slot_ids = (job.batched || pq) && st.tiles * qk::TILE < (int64_t{1} << 31) ? 1 : 0;
  a.metric = idx->metric;
  a.dim = idx->d;
  a.tau_r = job.tau_r;
  a.tau_rho = job.tau_rho;
  a.est = job.est;
  if (job.filter) {
    // per-partition label counts, recounted after any change to the rows
    if (st.attr_dirty) {
      qk::launch_attr_counts(st, s);
      st.attr_dirty = false;
    }
    a.qmask = job.filter;
    a.attr = st.attr;
    a.attr_cnt = st.d_attr_cnt;
  }
  const bool count = job.count && idx->count_access;
  a.hits = count ? st.d_hits : nullptr;
  if (count) st.window += nq;
  // a smaller requested cap than the buffer already allocated still applies
  a.items_cap = std::min<int64_t>(w.items_cap, items);
  qk::launch_round_init(w, a, job.w0, s);
  a.blocks = qk::scan_blocks(idx, job.batched);
  {
    qk::ProfileScope ps(idx->prof, QUAKE_PROF_PLAN, s);
    qk::launch_demand(w, st, a, s);
  }
  // Every round commits at least one partition of the first unfinished
  // query, so the loop ends within nq * M rounds.  Rounds after the last one
  // with work find nothing to do.
  const int64_t max_rounds = nq * (int64_t)job.M + 2;
  int64_t rounds = 0;
  int chunk = 1;
  for (;;) {
    QK_HIP(hipMemcpyAsync(w.h_total, w.total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    if (w.h_total[0] == 0) break;
    QK_CHECK(rounds <= max_rounds, QUAKE_E_DEVICE, "search rounds did not converge");
    const int R = idx->tune.rounds_per_sync > 0 ? idx->tune.rounds_per_sync : chunk;
    qk::run_rounds(idx, st, job, a, R, s);
    rounds += R;
    chunk = std::min(chunk * 2, 8);
  }
  if (job.batched || pq) {
    {
      qk::ProfileScope ps(idx->prof, QUAKE_PROF_RERANK, s);
      qk::launch_rerank(w, st, a, s, job.rerank != 0);
    }
    if (job.rerank)
      idx->prof.add(QUAKE_PROF_RERANK, (double)nq * job.kk * idx->d * sizeof(float),
                    (double)nq * job.kk * idx->d * 2.0);
  }
  if (out_ids) {
    qk::ProfileScope ps(idx->prof, QUAKE_PROF_COMMIT, s);
    qk::launch_finalize(w, a, out_ids, out_dist, out_nscanned, out_recall, s);
  }
  QK_HIP(hipGetLastError());
  if (idx->prof.on)
    QK_HIP(hipMemcpyAsync(w.h_total + 4, w.total + 4, 6 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  if (idx->prof.on && job.batched) {
    idx->prof.add(QUAKE_PROF_SCAN, (double)w.h_total[4] * idx->d * 2.0, (double)w.h_total[5] * idx->d * 2.0);
    idx->prof.add(QUAKE_PROF_SCAN_SETS, (double)w.h_total[9] * idx->d * 2.0, 0.0);
  }
  else if (idx->prof.on && pq)  // a code byte and a table add per subspace and row, and (L2) the residual term
    idx->prof.add(QUAKE_PROF_SCAN, (double)w.h_total[6] * (st.pq_m + (idx->metric == QUAKE_L2 ? 4 : 0)),
                  (double)w.h_total[6] * st.pq_m);
  else if (idx->prof.on)
    idx->prof.add(QUAKE_PROF_SCAN, (double)w.h_total[6] * idx->d * sizeof(float),
                  (double)w.h_total[6] * idx->d * (idx->metric == QUAKE_L2 ? 3.0 : 2.0));
  idx->prof.collect();
}

// int32 buffer of at least `need` entries
void ensure_i32(quake_index* idx, int32_t*& buf, int64_t& cap, int64_t need) {
  if (buf && need <= cap) return;
  idx->mem.release(buf);
  buf = nullptr;
  cap = need;
  buf = idx->mem.alloc<int32_t>(std::max<int64_t>(cap, 1));
}

// Searches of the upper levels for queries [0, nq) already in ws.q, from the
// top down (Sec. 3, Sec. 5: APS at every level, the upper levels at a high
// recall target): the search at level l >= 1 returns the M_{l-1} centroids
// of level l - 1 that are the candidate set of the search below it, where
// M_{l-1} = ceil(f_M(l-1) N_{l-1}).  Only the top level scores all of its
// centroids.  The M0 level-0 candidates of every query end in ws.cand0
// (count in ws.mq0).
void upper_level(quake_index* idx, int64_t nq, int M0, const quake_search_params* p, hipStream_t s) {
  const Store& L1 = idx->L1;
  const bool three = idx->n_levels == 3;
  auto upper_job = [&](int k, const Store& st) {
    Job up;
    up.k = up.kk = k;
    up.aps = 1;
    up.tau_r = p->upper_recall_target > 0 ? p->upper_recall_target : 0.99;
    up.f_M = p->upper_f_M > 0 ? p->upper_f_M : 0.25;
    up.tau_rho = p->tau_rho > 0 ? p->tau_rho : 0.01;
    up.est = p->estimator;
    up.M = candidate_count(up.f_M, st.nlist);
    up.w0 = up.M;  // the upper levels are small: scan their candidates in one round
    up.wmax = up.M;
    return up;
  };
  Job up1 = upper_job(M0, L1);
  Job up2;
  qk::Workspace& w = idx->ws;
  if (three) {
    // level 2 returns the M1 candidates of the level-1 search
    up2 = upper_job(up1.M, idx->L2);
    QK_CHECK(up1.M <= qk::KMAX_LARGE, QUAKE_E_INVALID, "the level-2 search returns at most 1024 candidates");
    up1.given = true;
    ensure_i32(idx, w.cand1, w.cand1_cap, (int64_t)up1.M * w.nq_cap);
    ensure_i32(idx, w.mq1, w.mq1_cap, w.nq_cap);
  }
  ensure_i32(idx, w.cand0, w.cand0_cap, (int64_t)M0 * w.nq_cap);
  // bound the upper levels' partial lists by running them on slices of the batch
  const int chunk_tiles = std::min(idx->tune.chunk_tiles > 0 ? idx->tune.chunk_tiles : 16,
                                   qk::SORTED_ITEM_MAX / qk::TILE);
  int64_t per_query = (int64_t)up1.M * max_chunks(L1, chunk_tiles);
  if (three) per_query = std::max<int64_t>(per_query, (int64_t)up2.M * max_chunks(idx->L2, chunk_tiles));
  const int64_t slice = std::max<int64_t>(1, std::min<int64_t>(nq, (int64_t)(1 << 17) / std::max<int64_t>(per_query, 1)));
  struct Only {  // the upper levels' work is timed as one kind of its own
    qk::Profiler& p;
    explicit Only(qk::Profiler& p_) : p(p_) { p.only = QUAKE_PROF_UPPER; }
    ~Only() { p.only = -1; }
  } only(idx->prof);
  // the level-1 search of three levels reads its candidates where a given
  // search reads them (ws.cand0 / ws.mq0): the two buffers swap for it
  struct Swap {
    qk::Workspace& w;
    bool on = false;
    void flip() {
      std::swap(w.cand0, w.cand1);
      std::swap(w.cand0_cap, w.cand1_cap);
      std::swap(w.mq0, w.mq1);
      on = !on;
    }
    ~Swap() { if (on) flip(); }
  } sw{w};
  for (int64_t q0 = 0; q0 < nq; q0 += slice) {
    const int64_t n = std::min(slice, nq - q0);
    QueryWindow win(w, q0, idx->dp);
    if (three) {
      run_search(idx, idx->L2, up2, n, nullptr, nullptr, nullptr, nullptr, s);
      qk::launch_level1_to_candidates(n, up1.M, up2.kk, w.ri, w.cand1, w.mq1, s);
      sw.flip();
      run_search(idx, L1, up1, n, nullptr, nullptr, nullptr, nullptr, s);
      sw.flip();
    } else {
      run_search(idx, L1, up1, n, nullptr, nullptr, nullptr, nullptr, s);
    }
    qk::launch_level1_to_candidates(n, M0, up1.kk, w.ri, w.cand0 + q0 * M0, w.mq0 + q0, s);
  }
}

}  // namespace

namespace qk {

// A single-level search whose workspace is carved out of caller-given
// device memory (`scratch`, scratch_bytes long) and whose host counter reads
// go to `host_counters` (COUNTERS entries): nothing is allocated, no graph is
// captured, and any allocation attempt fails the call.  The index's own
// workspace is set aside for the call and put back after it.
void search_in_scratch(quake_index* idx, const float* q, int64_t nq, const quake_search_params* params,
                       int64_t* out_ids, float* out_dist, int32_t* out_nscanned, double* out_recall, hipStream_t s,
                       char* scratch, size_t scratch_bytes, int64_t* host_counters) {
  check_index(idx);
  QK_CHECK(nq >= 0, QUAKE_E_INVALID, "nq must be >= 0");
  QK_CHECK(idx->n_levels == 1, QUAKE_E_STATE, "the allocation-free search is for single-level indexes");
  const Store& L0 = idx->L0;
  const Job job = resolve(idx, L0, params);
  QK_CHECK(job.dtype16 != QUAKE_PQ8, QUAKE_E_INVALID, "the allocation-free search does not scan product codes");
  if (nq == 0) return;
  QK_CHECK(q && out_ids && out_dist, QUAKE_E_INVALID, "q, out_ids and out_dist are required");
  const int64_t items = search_items(idx, L0, job, nq);
  const int64_t pairs = job.batched ? nq * (int64_t)job.wmax : 0;
  const int dp16 = job.batched ? L0.dp16 : 0;
  const size_t need = workspace_layout(nullptr, nullptr, nq, L0.nlist, job.M, job.kk, items, pairs, idx->dp, dp16);
  QK_CHECK(need <= scratch_bytes, QUAKE_E_INVALID,
           "this search needs " + std::to_string(need) + " bytes of scratch memory, more than the " +
               std::to_string(scratch_bytes) + " the allocation-free entry point has: search fewer queries per call");
  Workspace view;
  workspace_layout(&view, scratch, nq, L0.nlist, job.M, job.kk, items, pairs, idx->dp, dp16);
  view.h_total = host_counters;
  // the index's workspace, profiling and allocation state come back on any exit
  struct Restore {
    quake_index* idx;
    Workspace ws;
    bool prof;
    ~Restore() {
      idx->ws = ws;
      idx->prof.on = prof;
      idx->noalloc = false;
      idx->mem.forbid = false;
    }
  } restore{idx, idx->ws, idx->prof.on};
  idx->ws = view;
  idx->prof.on = false;
  idx->noalloc = true;
  idx->mem.forbid = true;
  Workspace& w = idx->ws;
  // what the kernels expect zeroed (they keep it so between rounds, but the
  // array holds whatever the last call on this device left)
  launch_fill_i32(w.pcount, L0.nlist + 1, 0, s);
  launch_fill_i32(reinterpret_cast<int32_t*>(idx->d_flag), 1, 0, s);
  launch_pad_rows(q, nq, idx->d, idx->dp, w.q, w.qn2, s, idx->d_flag);
  QK_HIP(hipMemcpyAsync(idx->h_flag, idx->d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  QK_CHECK(*idx->h_flag == 0, QUAKE_E_INVALID, "q holds a non-finite value");
  run_search(idx, L0, job, nq, out_ids, out_dist, out_nscanned, out_recall, s);
}

int run_api(const std::function<void()>& fn) {
  API_BEGIN
  fn();
  API_END
}

}  // namespace qk

extern "C" {

const char* quake_last_error(void) { return qk::g_error.c_str(); }

int quake_cap_table(int32_t d, double* out) {
  API_BEGIN
  QK_CHECK(d >= 1 && d <= qk::MAX_DIM && out, QUAKE_E_INVALID, "bad dimension or output");
  qk::cap_fraction_table(d, out);
  API_END
}

}  // extern "C"

// Level `level` (1 or 2) over the centroids of the level below (Sec. 3;
// "Add Level", Sec. 4.2): k-means of those centroids into nlist_top
// partitions, or the given top centroids (device [nlist_top][d]) and parent
// of every centroid below (device [N below]); then the store of the
// centroids below partitioned by it.
void qk::build_top_level(quake_index* idx, int level, int64_t nlist_top, int32_t kmeans_iters, uint64_t seed,
                     const float* top_centroids, const int32_t* parent, hipStream_t s) {
  const Store& below = level == 1 ? idx->L0 : idx->L1;
  Store& up = level == 1 ? idx->L1 : idx->L2;
  int32_t*& of = level == 1 ? idx->top_of : idx->top_of2;
  const int d = idx->d, dp = idx->dp;
  up = Store();
  up.d = d;
  up.dp = dp;
  up.nlist = nlist_top;
  up.centroids = idx->mem.alloc<float>((size_t)up.nlist * dp);
  of = idx->mem.alloc<int32_t>(below.nlist);
  if (top_centroids && parent) {
    // a given level (a saved index): its centroids and the parent of every centroid below
    require_finite(idx, top_centroids, up.nlist * (int64_t)d, "top centroids", s);
    clear_flag(idx, s);
    qk::launch_check_range(parent, below.nlist, up.nlist, idx->d_flag, s);
    QK_CHECK(!flag_set(idx, s), QUAKE_E_INVALID, "a parent index lies outside the level above");
    qk::launch_pad_rows(top_centroids, up.nlist, d, dp, up.centroids, nullptr, s);
    QK_HIP(hipMemcpyAsync(of, parent, below.nlist * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  } else {
    kmeans(idx->mem, below.centroids, below.nlist, dp, up.nlist, std::max(kmeans_iters, 1),
           seed ^ 0x9e3779b97f4a7c15ull, idx->metric, up.centroids, s);
    qk::launch_assign(below.centroids, below.nlist, dp, up.centroids, up.nlist, idx->metric, of, s);
  }
  build_store(idx, up, below.centroids, dp, nullptr, below.nlist, of, 0.0, QUAKE_F32, true, s);
}

// Drops the top level ("Remove Level", Sec. 4.2): the centroids of the
// level below become the top again.
void drop_top_level(quake_index* idx, int level) {
  Store& up = level == 1 ? idx->L1 : idx->L2;
  int32_t*& of = level == 1 ? idx->top_of : idx->top_of2;
  for (void* p : {(void*)up.centroids, (void*)up.d_off, (void*)up.d_size, (void*)up.d_cap, (void*)up.d_order,
                  (void*)up.d_hits, (void*)up.v32, (void*)up.v16, (void*)up.v16n, (void*)up.rows32, (void*)up.ids,
                  (void*)of})
    idx->mem.release(p);
  up = Store();
  of = nullptr;
}

// After level 0's partitions change (maintenance), the level-1 store is
// rebuilt over the new level-0 centroids, each in its nearest level-1
// partition: a split's new centroid joins the level above and a deleted one
// leaves it (Sec. 4.2, "Decision Workflow", changes propagate upward).
// Level-1 centroids do not move, so the levels above are unchanged.
void qk::rebuild_level1(quake_index* idx, hipStream_t s) {
  const int d = idx->d, dp = idx->dp;
  const int64_t n1 = idx->L1.nlist;
  Tmp<float> C1(idx->mem, (size_t)n1 * d);
  QK_HIP(hipMemcpy2DAsync(C1.p, d * sizeof(float), idx->L1.centroids, dp * sizeof(float), d * sizeof(float), n1,
                          hipMemcpyDeviceToDevice, s));
  Tmp<int32_t> top(idx->mem, idx->L0.nlist);
  qk::launch_assign(idx->L0.centroids, idx->L0.nlist, dp, idx->L1.centroids, n1, idx->metric, top.p, s);
  QK_HIP(hipStreamSynchronize(s));
  drop_top_level(idx, 1);
  try {
    qk::build_top_level(idx, 1, n1, 0, 0, C1.p, top.p, s);
  } catch (...) {
    // the index falls back to level 0 alone rather than keep a stale level 1
    drop_top_level(idx, 1);
    if (idx->n_levels == 3) drop_top_level(idx, 2);
    idx->n_levels = 1;
    throw;
  }
}

quake_index* qk::build_index(const float* x, const int64_t* ids, int64_t n, int32_t d,
                             const quake_build_params* params, const float* top_centroids, const int32_t* top_of,
                             const quake_allocator* allocator, hipStream_t s) {
  QK_CHECK(params, QUAKE_E_INVALID, "params is NULL");
  QK_CHECK(x && n >= 1, QUAKE_E_INVALID, "need x and n >= 1");
  QK_CHECK(d >= 1 && d <= qk::MAX_DIM, QUAKE_E_INVALID, "d must be in [1, 4096]");
  QK_CHECK(params->metric == QUAKE_L2 || params->metric == QUAKE_IP, QUAKE_E_INVALID, "unknown metric");
  QK_CHECK(params->storage_dtype >= QUAKE_F32 && params->storage_dtype <= QUAKE_F16, QUAKE_E_INVALID,
           "unknown storage dtype");
  QK_CHECK(params->n_levels == 1 || params->n_levels == 2, QUAKE_E_INVALID, "n_levels must be 1 or 2");
  // (given centroids and assignment may leave partitions empty, as deletes do)
  QK_CHECK(params->nlist >= 1 && (params->nlist <= n || (params->centroids && params->assign)), QUAKE_E_INVALID,
           "nlist must be in [1, n]");
  QK_CHECK(params->nlist <= INT32_MAX, QUAKE_E_INVALID, "nlist too large");
  QK_CHECK(params->kmeans_iters >= 0 && params->capacity_slack >= 0, QUAKE_E_INVALID, "bad k-means settings");
  if (params->n_levels == 2)
    QK_CHECK(params->nlist_top >= 1 && params->nlist_top <= params->nlist, QUAKE_E_INVALID,
             "nlist_top must be in [1, nlist]");
  QK_CHECK(params->pq_m >= 0 && (params->pq_m > 0 || !params->pq_codebook), QUAKE_E_INVALID,
           "pq_m must be >= 0 (a pq_codebook needs pq_m > 0)");
  if (params->pq_m > 0) {
    QK_CHECK(params->pq_m % 4 == 0 && d % params->pq_m == 0 && d / params->pq_m <= qk::PQ_MAX_SUB, QUAKE_E_INVALID,
             "pq_m must be a multiple of 4 that divides d, with d / pq_m <= 32");
    QK_CHECK(params->pq_codebook || n >= 256, QUAKE_E_INVALID, "training a codebook needs at least 256 rows");
  }
  QK_CHECK(params->drop_f32_tiles == 0 ||
               (params->drop_f32_tiles == 1 && (params->storage_dtype != QUAKE_F32 || params->pq_m > 0)),
           QUAKE_E_INVALID, "drop_f32_tiles needs a 16-bit copy (storage_dtype BF16 or F16) or product codes");
  const bool f32_tiles = params->drop_f32_tiles == 0;
  std::unique_ptr<quake_index> idx(new quake_index());
  if (allocator && allocator->alloc) idx->mem.user = *allocator;
  idx->mem.budget = params->hbm_budget_bytes;
  idx->slack = params->capacity_slack;
  idx->labelled = params->attrs != nullptr;
  idx->metric = params->metric;
  idx->storage = params->storage_dtype;
  idx->n_levels = params->n_levels;
  idx->d = d;
  idx->dp = (int)round_up(d, 8);
  const int dp = idx->dp;
  idx->d_flag = idx->mem.alloc<uint32_t>(1);
  QK_HIP(hipHostMalloc((void**)&idx->h_flag, sizeof(uint32_t), hipHostMallocDefault));
  require_finite(idx.get(), x, n * (int64_t)d, "x", s);
  if (params->centroids) require_finite(idx.get(), params->centroids, params->nlist * (int64_t)d, "centroids", s);
  if (params->assign) {
    clear_flag(idx.get(), s);
    qk::launch_check_range(params->assign, n, params->nlist, idx->d_flag, s);
    QK_CHECK(!flag_set(idx.get(), s), QUAKE_E_INVALID, "assign holds a partition outside [0, nlist)");
  }

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
  } else if (params->assign) {
    // each centroid is the mean of the rows the caller put in its partition
    QK_HIP(hipMemsetAsync(L0.centroids, 0, (size_t)L0.nlist * dp * sizeof(float), s));
    Tmp<int32_t> counts(idx->mem, (size_t)L0.nlist);
    const int bits = fixed_point_bits(idx->mem, xpad, n, dp, s);
    centroids_from(idx->mem, xpad, n, dp, params->assign, L0.nlist, idx->metric == QUAKE_IP ? 1 : 0, bits,
                   L0.centroids, counts.p, s);
    std::vector<int32_t> h_counts(L0.nlist);
    QK_HIP(hipMemcpyAsync(h_counts.data(), counts.p, L0.nlist * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    for (int64_t j = 0; j < L0.nlist; ++j)
      QK_CHECK(h_counts[j] > 0, QUAKE_E_INVALID,
               "assign leaves partition " + std::to_string(j) + " empty and no centroids are given");
  } else {
    kmeans(idx->mem, xpad, n, dp, L0.nlist, params->kmeans_iters, params->seed, idx->metric, L0.centroids, s);
  }
  std::unique_ptr<Tmp<int32_t>> assign_buf;
  const int32_t* assign = params->assign;
  if (!assign) {
    assign_buf.reset(new Tmp<int32_t>(idx->mem, n));
    qk::launch_assign(xpad, n, dp, L0.centroids, L0.nlist, idx->metric, assign_buf->p, s);
    assign = assign_buf->p;
  }
  if (params->pq_m > 0) {
    // the codebook comes before the store (build_store encodes the rows'
    // residuals to their centroids); without one given it is trained on them
    idx->pq_m = params->pq_m;
    idx->pq_ds = d / params->pq_m;
    const size_t book = (size_t)idx->pq_m * 256 * idx->pq_ds;
    idx->pq_book = idx->mem.alloc<float>(book);
    if (params->pq_codebook) {
      require_finite(idx.get(), params->pq_codebook, (int64_t)book, "pq_codebook", s);
      QK_HIP(hipMemcpyAsync(idx->pq_book, params->pq_codebook, book * sizeof(float), hipMemcpyDeviceToDevice, s));
    } else {
      train_codebook(idx.get(), x, n, assign, L0.centroids, params->kmeans_iters, params->seed, s);
    }
  }
  build_store(idx.get(), L0, x, d, ids, n, assign, params->capacity_slack, params->storage_dtype, f32_tiles, s,
              params->attrs);
  map_rebuild(idx.get(), idx->idmap, idx->L0, n, s);

  if (idx->n_levels == 2)
    qk::build_top_level(idx.get(), 1, params->nlist_top, params->kmeans_iters, params->seed, top_centroids, top_of, s);

  idx->h_cap_table.resize(qk::CAP_TABLE_SIZE);
  qk::cap_model_table(d, idx->h_cap_table.data());
  idx->cap_table = idx->mem.alloc<double>(qk::CAP_TABLE_SIZE);
  QK_HIP(hipMemcpyAsync(idx->cap_table, idx->h_cap_table.data(), qk::CAP_TABLE_SIZE * sizeof(double),
                        hipMemcpyHostToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  return idx.release();
}

extern "C" {

int quake_build(const float* x, const int64_t* ids, int64_t n, int32_t d, const quake_build_params* params,
                const quake_allocator* allocator, void* stream, quake_index** out) {
  API_BEGIN
  QK_CHECK(out, QUAKE_E_INVALID, "out is NULL");
  *out = nullptr;
  *out = qk::build_index(x, ids, n, d, params, nullptr, nullptr, allocator, as_stream(stream));
  API_END
}

int quake_search(quake_index* idx, const float* q, int64_t nq, const quake_search_params* params, int64_t* out_ids,
                 float* out_dist, int32_t* out_nscanned, double* out_recall, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(nq >= 0, QUAKE_E_INVALID, "nq must be >= 0");
  const Store& L0 = idx->L0;
  Job job = resolve(idx, L0, params);
  if (nq == 0) return QUAKE_OK;
  QK_CHECK(q && out_ids && out_dist, QUAKE_E_INVALID, "q, out_ids and out_dist are required");
  hipStream_t s = as_stream(stream);
  ensure_queries(idx, nq);
  clear_flag(idx, s);
  qk::launch_pad_rows(q, nq, idx->d, idx->dp, idx->ws.q, idx->ws.qn2, s, idx->d_flag);
  QK_CHECK(!flag_set(idx, s), QUAKE_E_INVALID, "q holds a non-finite value");
  if (idx->n_levels >= 2) {
    // the upper levels pick the level-0 candidates: M0 = ceil(f_M * N0) nearest leaf
    // centroids it finds; nprobe mode takes the nprobe nearest it finds
    const int M0 = job.M;
    QK_CHECK(M0 <= qk::KMAX_LARGE, QUAKE_E_INVALID, "the upper level returns at most 1024 candidates");
    upper_level(idx, nq, M0, params, s);
    job.given = true;
  }
  run_search(idx, L0, job, nq, out_ids, out_dist, out_nscanned, out_recall, s);
  API_END
}

int quake_set_tuning(quake_index* idx, const quake_tuning* t) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(t, QUAKE_E_INVALID, "tuning is NULL");
  QK_CHECK(t->chunk_tiles >= 0 && t->first_window >= 0 && t->max_window >= 0 && t->max_items >= 0 &&
               t->blocks_per_cu >= 0 && t->rounds_per_sync >= 0 && t->no_graph >= 0,
           QUAKE_E_INVALID, "tuning values must be >= 0");
  QK_CHECK(t->chunk_tiles <= 1024, QUAKE_E_INVALID, "chunk_tiles must be <= 1024");
  QK_CHECK(t->window_scale == 0 || (t->window_scale >= 100 && t->window_scale <= 1000), QUAKE_E_INVALID,
           "window_scale must be 0 or in [100, 1000]");
  idx->tune = *t;
  API_END
}

int quake_autotune(quake_index* idx, const float* q, int64_t nq, const quake_search_params* params, int32_t reps,
                   quake_tuning* out, double* out_ms, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(nq >= 1 && q, QUAKE_E_INVALID, "autotuning needs sample queries");
  QK_CHECK(reps >= 0, QUAKE_E_INVALID, "reps must be >= 0");
  const Job job = resolve(idx, idx->L0, params);
  hipStream_t s = as_stream(stream);
  const int R = reps > 0 ? reps : 3;
  Tmp<int64_t> ids(idx->mem, (size_t)nq * job.k);
  Tmp<float> dist(idx->mem, (size_t)nq * job.k);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  QK_HIP(hipEventCreate(&e0));
  QK_HIP(hipEventCreate(&e1));
  const quake_tuning saved = idx->tune;
  const bool prof = idx->prof.on;
  idx->prof.on = false;
  idx->count_access = false;  // tuning searches are not workload: keep them out of the access statistics
  auto search = [&]() {
    const int rc = quake_search(idx, q, nq, params, ids.p, dist.p, nullptr, nullptr, stream);
    if (rc != QUAKE_OK) throw qk::Error{rc, qk::g_error};
  };
  // median wall time of R searches under tuning t (after one warm-up search
  // that grows buffers and captures graphs)
  auto time_it = [&](const quake_tuning& t) {
    idx->tune = t;
    search();
    std::vector<double> ms;
    for (int r = 0; r < R; ++r) {
      QK_HIP(hipEventRecord(e0, s));
      search();
      QK_HIP(hipEventRecord(e1, s));
      QK_HIP(hipEventSynchronize(e1));
      float v = 0.f;
      QK_HIP(hipEventElapsedTime(&v, e0, e1));
      ms.push_back(v);
    }
    std::sort(ms.begin(), ms.end());
    return ms[ms.size() / 2];
  };
  try {
    // coordinate descent over the knobs, twice; a change must win by 3%
    // (more than the run-to-run spread, so the choice is stable)
    quake_tuning best = saved;
    double best_ms = time_it(best);
    struct Knob {
      int32_t quake_tuning::*field;
      std::vector<int32_t> values;
    };
    std::vector<Knob> knobs = {{&quake_tuning::chunk_tiles, {8, 16, 32, 64, 128}},
                               {&quake_tuning::rounds_per_sync, {0, 2, 4, 8}}};
    if (job.batched)
      knobs.push_back({&quake_tuning::blocks_per_cu, {1, 2}});
    else
      knobs.push_back({&quake_tuning::blocks_per_cu, {4, 8, 16}});
    if (job.aps) {
      knobs.push_back({&quake_tuning::first_window, {1, 2, 4, 8, 16, 32, 64}});
      knobs.push_back({&quake_tuning::max_window, {8, 16, 32, 64, 128, 256}});
      knobs.push_back({&quake_tuning::window_scale, {100, 150, 200, 300}});
    }
    // wide windows trade speculative scans for fewer rounds (and so for
    // fewer reads of partitions that several rounds touch); the two window
    // sizes interact, so pairs of them are tried together first
    if (job.aps) {
      const int32_t pairs[][2] = {{1, 32}, {1, 64}, {1, 128}, {2, 32}, {2, 64}, {2, 128}, {4, 32}, {4, 64},
                                  {4, 128}, {8, 32}, {8, 64}, {16, 64}, {16, 128}, {32, 64}, {32, 128},
                                  {64, 128}, {64, 256}};
      for (const auto& pr : pairs) {
        quake_tuning t = best;
        t.first_window = pr[0];
        t.max_window = pr[1];
        if (t.first_window == best.first_window && t.max_window == best.max_window) continue;
        const double ms = time_it(t);
        if (ms < 0.97 * best_ms) { best = t; best_ms = ms; }
      }
    }
    for (int pass = 0; pass < 2; ++pass)
      for (const Knob& kn : knobs)
        for (int32_t v : kn.values) {
          if (best.*kn.field == v) continue;
          quake_tuning t = best;
          t.*kn.field = v;
          const double ms = time_it(t);
          if (ms < 0.97 * best_ms) { best = t; best_ms = ms; }
        }
    idx->tune = best;
    idx->prof.on = prof;
    idx->count_access = true;
    if (out) *out = best;
    if (out_ms) *out_ms = best_ms;
  } catch (...) {
    idx->tune = saved;
    idx->prof.on = prof;
    idx->count_access = true;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
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

int quake_candidates(quake_index* idx, const float* q, int64_t nq, const quake_search_params* params,
                     int32_t* order, float* h, int32_t* out_M, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(params, QUAKE_E_INVALID, "params is NULL");
  QK_CHECK(nq >= 0 && (nq == 0 || (q && order && h)), QUAKE_E_INVALID, "bad arguments");
  QK_CHECK(params->f_M >= 0 && params->upper_f_M >= 0 && params->upper_recall_target >= 0 &&
               params->upper_recall_target <= 1.0 && params->tau_rho >= 0,
           QUAKE_E_INVALID, "negative or out-of-range search parameter");
  QK_CHECK(params->estimator >= QUAKE_EST_APS && params->estimator <= QUAKE_EST_APS_RP, QUAKE_E_INVALID,
           "unknown estimator");
  const Store& st = idx->L0;
  const int M = candidate_count(params->f_M > 0 ? params->f_M : 0.05, st.nlist);
  QK_CHECK(M <= (st.nlist > 4096 ? 2048 : qk::MAX_CANDIDATES), QUAKE_E_INVALID, "too many candidates");
  QK_CHECK(idx->n_levels == 1 || M <= qk::KMAX_LARGE, QUAKE_E_INVALID,
           "the upper level returns at most 1024 candidates");
  if (out_M) *out_M = M;
  if (nq == 0) return QUAKE_OK;
  hipStream_t s = as_stream(stream);
  ensure_queries(idx, nq);
  qk::Workspace& w = idx->ws;
  clear_flag(idx, s);
  qk::launch_pad_rows(q, nq, idx->d, idx->dp, w.q, w.qn2, s, idx->d_flag);
  QK_CHECK(!flag_set(idx, s), QUAKE_E_INVALID, "q holds a non-finite value");
  if (idx->n_levels >= 2) {
    upper_level(idx, nq, M, params, s);
    ensure_workspace(idx, st.nlist, M, 1, 1, 0, 0, false);
    QK_HIP(hipMemcpyAsync(w.mq, w.mq0, nq * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    qk::launch_geometry(w.q, st.centroids, nq, idx->dp, M, w.mq, idx->metric, w.cand0, w.cand, w.h, s);
  } else {
    ensure_workspace(idx, st.nlist, M, 1, 1, 0, 0);
    qk::launch_fill_i32(w.mq, nq, M, s);
    qk::launch_scores(w.q, nq, st.centroids, st.nlist, idx->dp, idx->metric, w.scores, s);
    qk::launch_candidates(st, w.q, w.scores, nq, idx->dp, M, 1, idx->metric, w.mq, w.sel, w.cand, w.h, s);
  }
  QK_HIP(hipMemcpyAsync(order, w.cand, (size_t)nq * M * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipMemcpyAsync(h, w.h, (size_t)nq * M * sizeof(float), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  API_END
}

static void insert_api(quake_index* idx, const float* x, const int64_t* ids, const uint32_t* attrs, int64_t n,
                       void* stream) {
  check_index(idx);
  QK_CHECK(n >= 0, QUAKE_E_INVALID, "n must be >= 0");
  if (n == 0) return;
  QK_CHECK(x && ids, QUAKE_E_INVALID, "x and ids are required");
  hipStream_t s = as_stream(stream);
  require_finite(idx, x, n * (int64_t)idx->d, "x", s);
  std::vector<int32_t> routed;
  if (idx->n_levels >= 2) {
    // top-down: the nearest top partition, then its nearest member at each
    // level below (searches with one candidate and one result)
    std::unique_ptr<Tmp<float>> xpad_buf;
    const float* xpad = x;
    if (idx->dp != idx->d) {
      xpad_buf.reset(new Tmp<float>(idx->mem, (size_t)n * idx->dp));
      qk::launch_pad_rows(x, n, idx->d, idx->dp, xpad_buf->p, nullptr, s);
      xpad = xpad_buf->p;
    }
    ensure_queries(idx, n);
    qk::launch_pad_rows(xpad, n, idx->dp, idx->dp, idx->ws.q, idx->ws.qn2, s);
    Job route;
    route.count = false;
    route.k = route.kk = 1;
    route.M = route.w0 = route.wmax = 1;
    if (idx->n_levels == 3) {
      qk::Workspace& w = idx->ws;
      run_search(idx, idx->L2, route, n, nullptr, nullptr, nullptr, nullptr, s);
      ensure_i32(idx, w.cand0, w.cand0_cap, std::max<int64_t>(n, w.nq_cap));
      qk::launch_level1_to_candidates(n, 1, 1, w.ri, w.cand0, w.mq0, s);
      Job r1 = route;
      r1.given = true;
      run_search(idx, idx->L1, r1, n, nullptr, nullptr, nullptr, nullptr, s);
    } else {
      run_search(idx, idx->L1, route, n, nullptr, nullptr, nullptr, nullptr, s);
    }
    std::vector<int64_t> leaf(n);
    QK_HIP(hipMemcpyAsync(leaf.data(), idx->ws.ri, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    routed.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      QK_CHECK(leaf[i] >= 0, QUAKE_E_DEVICE, "top-down routing found no leaf");
      routed[i] = (int32_t)leaf[i];
    }
  }
  qk::insert_rows(idx, idx->L0, idx->idmap, x, ids, n, routed.empty() ? nullptr : &routed, s, attrs);
}

int quake_insert(quake_index* idx, const float* x, const int64_t* ids, int64_t n, void* stream) {
  API_BEGIN
  insert_api(idx, x, ids, nullptr, n, stream);
  API_END
}

int quake_insert_attrs(quake_index* idx, const float* x, const int64_t* ids, const uint32_t* attrs, int64_t n,
                       void* stream) {
  API_BEGIN
  QK_CHECK(n <= 0 || attrs, QUAKE_E_INVALID, "attrs are required");
  insert_api(idx, x, ids, attrs, n, stream);
  API_END
}

int quake_delete(quake_index* idx, const int64_t* ids, int64_t n, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(n >= 0, QUAKE_E_INVALID, "n must be >= 0");
  if (n == 0) return QUAKE_OK;
  QK_CHECK(ids, QUAKE_E_INVALID, "ids are required");
  qk::delete_rows(idx, idx->L0, idx->idmap, ids, n, as_stream(stream));
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

int quake_describe(const quake_index* idx, int32_t* d, int32_t* metric, int32_t* storage_dtype, int32_t* n_levels) {
  API_BEGIN
  check_index(idx);
  if (d) *d = idx->d;
  if (metric) *metric = idx->metric;
  if (storage_dtype) *storage_dtype = idx->storage;
  if (n_levels) *n_levels = idx->n_levels;
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
    if (ids && !o_ids.empty())
      QK_HIP(hipMemcpyAsync(ids, o_ids.data(), o_ids.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (part && !o_part.empty())
      QK_HIP(hipMemcpyAsync(part, o_part.data(), o_part.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  QK_HIP(hipStreamSynchronize(s));
  API_END
}

int quake_export_pq(const quake_index* cidx, int32_t* m, float* codebook, uint8_t* codes, void* stream) {
  API_BEGIN
  check_index(cidx);
  quake_index* idx = const_cast<quake_index*>(cidx);
  hipStream_t s = as_stream(stream);
  const Store& st = idx->L0;
  if (m) *m = idx->pq_m;
  if (idx->pq_m > 0 && codebook)
    QK_HIP(hipMemcpyAsync(codebook, idx->pq_book, (size_t)idx->pq_m * 256 * idx->pq_ds * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
  if (idx->pq_m > 0 && codes && st.live > 0) {
    // live slots partition by partition, as quake_export lists the rows
    std::vector<int64_t> sid((size_t)st.tiles * qk::TILE);
    QK_HIP(hipMemcpyAsync(sid.data(), st.ids, sid.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> slots;
    slots.reserve(st.live);
    for (int64_t p = 0; p < st.nlist; ++p)
      for (int64_t j = 0; j < st.size[p]; ++j)
        if (sid[st.off[p] * qk::TILE + j] >= 0) slots.push_back(st.off[p] * qk::TILE + j);
    Tmp<int64_t> d_slots(idx->mem, slots.size());
    QK_HIP(hipMemcpyAsync(d_slots.p, slots.data(), slots.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    qk::launch_pq_export(st, d_slots.p, (int64_t)slots.size(), codes, s);
  }
  QK_HIP(hipStreamSynchronize(s));
  API_END
}

int quake_add_level(quake_index* idx, int64_t nlist_top, int32_t kmeans_iters, uint64_t seed, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(idx->n_levels < 3, QUAKE_E_STATE, "the index has three levels already (at most three are supported)");
  const Store& top = idx->n_levels == 1 ? idx->L0 : idx->L1;
  QK_CHECK(nlist_top >= 1 && nlist_top <= top.nlist && kmeans_iters >= 0, QUAKE_E_INVALID,
           "nlist_top must be in [1, partitions of the current top level] and kmeans_iters >= 0");
  hipStream_t s = as_stream(stream);
  QK_HIP(hipStreamSynchronize(s));
  const int level = idx->n_levels;
  try {
    qk::build_top_level(idx, level, nlist_top, kmeans_iters, seed, nullptr, nullptr, s);
  } catch (...) {
    drop_top_level(idx, level);
    throw;
  }
  qk::release_graphs(idx);
  idx->n_levels = level + 1;
  API_END
}

int quake_remove_level(quake_index* idx, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(idx->n_levels >= 2, QUAKE_E_STATE, "the index has one level");
  QK_HIP(hipStreamSynchronize(as_stream(stream)));
  qk::release_graphs(idx);
  drop_top_level(idx, idx->n_levels - 1);
  idx->n_levels -= 1;
  API_END
}

int quake_adjust_levels(quake_index* idx, int64_t add_above, int64_t remove_below, int64_t nlist_top,
                        int32_t kmeans_iters, uint64_t seed, void* stream, int32_t* action) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(add_above >= 0 && remove_below >= 0 && nlist_top >= 0, QUAKE_E_INVALID, "negative threshold");
  if (action) *action = 0;
  const int64_t top = idx->n_levels == 1 ? idx->L0.nlist : idx->n_levels == 2 ? idx->L1.nlist : idx->L2.nlist;
  if (idx->n_levels < 3 && add_above > 0 && top > add_above) {
    const int64_t n = nlist_top > 0 ? std::min<int64_t>(nlist_top, top)
                                    : std::max<int64_t>(1, (int64_t)std::llround(std::sqrt((double)top)));
    const int rc = quake_add_level(idx, n, kmeans_iters, seed, stream);
    if (rc != QUAKE_OK) return rc;
    if (action) *action = 1;
  } else if (idx->n_levels >= 2 && top < remove_below) {
    const int rc = quake_remove_level(idx, stream);
    if (rc != QUAKE_OK) return rc;
    if (action) *action = -1;
  }
  API_END
}

int quake_export_level(const quake_index* idx, int32_t level, float* centroids, int32_t* parent, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(level >= 1 && level < idx->n_levels, QUAKE_E_INVALID, "no such upper level");
  hipStream_t s = as_stream(stream);
  const Store& up = level == 1 ? idx->L1 : idx->L2;
  const Store& below = level == 1 ? idx->L0 : idx->L1;
  const int32_t* of = level == 1 ? idx->top_of : idx->top_of2;
  if (centroids)
    QK_HIP(hipMemcpy2DAsync(centroids, idx->d * sizeof(float), up.centroids, idx->dp * sizeof(float),
                            idx->d * sizeof(float), up.nlist, hipMemcpyDeviceToDevice, s));
  if (parent) QK_HIP(hipMemcpyAsync(parent, of, below.nlist * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  API_END
}

int quake_level_sizes(const quake_index* idx, int64_t* nlist_per_level) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(nlist_per_level, QUAKE_E_INVALID, "output is NULL");
  nlist_per_level[0] = idx->L0.nlist;
  nlist_per_level[1] = idx->n_levels >= 2 ? idx->L1.nlist : 0;
  nlist_per_level[2] = idx->n_levels >= 3 ? idx->L2.nlist : 0;
  API_END
}

int quake_export_top(const quake_index* idx, float* top_centroids, int32_t* top_of, void* stream) {
  API_BEGIN
  check_index(idx);
  QK_CHECK(idx->n_levels >= 2, QUAKE_E_STATE, "index has one level");
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
  idx->magic = 0;
  delete idx;
}

}  // extern "C"

// Adaptive incremental maintenance (Sec. 4): the cost model, the split and
// delete deltas and the estimate -> verify -> commit / reject workflow run
// on the host in FP64 over a few numbers per partition; every action on
// vectors (gathering a partition's rows, the 2-means split, nearest-centroid
// assignment, centroid updates, moving rows between partitions) runs in the
// kernels of k_maintain.hip, k_centroids.hip and k_update.hip.
//
// A tentative action is computed in full (the split's 2-means assignment, a
// delete's receiving partitions) before anything in the store changes, so
// that the verify step reads the action's actual sizes and a rejected
// action leaves the index untouched.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "engine.hpp"
#include "index.hpp"

namespace qk {
namespace {

template <class T>
struct Buf {
  DeviceMemory* mem;
  T* p = nullptr;
  Buf(DeviceMemory& m, size_t n) : mem(&m) { p = m.alloc<T>(std::max<size_t>(n, 1)); }
  ~Buf() { mem->release(p); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
};

template <class T>
void upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (!src.empty()) QK_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

template <class T>
std::vector<T> download(const T* src, size_t n, hipStream_t s) {
  std::vector<T> out(n);
  if (n) QK_HIP(hipMemcpyAsync(out.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  return out;
}

// lambda(s) of the cost model (Sec. 4.1): linear between the profiled
// sizes, extended linearly past the first and the last.
struct Latency {
  std::vector<double> s, v;
  double operator()(double x) const {
    size_t i;
    if (x <= s.front()) i = 0;
    else if (x >= s.back()) i = s.size() - 2;
    else i = (size_t)(std::upper_bound(s.begin(), s.end(), x) - s.begin()) - 1;
    const double t = (x - s[i]) / (s[i + 1] - s[i]);
    return v[i] + t * (v[i + 1] - v[i]);
  }
};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int64_t live_size(const Store& st, int64_t p) { return (int64_t)st.size[p] - st.tomb[p]; }

// Live store slots (and their ids) of the listed partitions, partition by
// partition in slot order; lo[i] = first row of parts[i] (lo has one more entry).
void live_rows(const Store& st, const std::vector<int32_t>& parts, std::vector<int64_t>& slots,
               std::vector<int64_t>& ids, std::vector<int64_t>& lo, hipStream_t s) {
  std::vector<std::vector<int64_t>> raw(parts.size());
  for (size_t i = 0; i < parts.size(); ++i) {
    const int32_t p = parts[i];
    raw[i].resize(st.size[p]);
    if (st.size[p])
      QK_HIP(hipMemcpyAsync(raw[i].data(), st.ids + st.off[p] * TILE, st.size[p] * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
  }
  QK_HIP(hipStreamSynchronize(s));
  slots.clear();
  ids.clear();
  lo.assign(1, 0);
  for (size_t i = 0; i < parts.size(); ++i) {
    const int64_t base = st.off[parts[i]] * TILE;
    for (size_t k = 0; k < raw[i].size(); ++k)
      if (raw[i][k] >= 0) {
        slots.push_back(base + (int64_t)k);
        ids.push_back(raw[i][k]);
      }
    lo.push_back((int64_t)slots.size());
  }
}

// Centroids on the host in FP64, [nlist][dp].
std::vector<double> host_centroids(const Store& st, hipStream_t s) {
  std::vector<float> c = download(st.centroids, (size_t)st.nlist * st.dp, s);
  return std::vector<double>(c.begin(), c.end());
}

// The r centroids nearest to c (ties to the lower id), FP64, skipping `skip`.
std::vector<int32_t> nearest_centroids(const std::vector<double>& C, int64_t N, int dp, const double* c, int r,
                                       const std::vector<char>& skip, int ip) {
  std::vector<std::pair<double, int32_t>> key;
  key.reserve(N);
  for (int64_t p = 0; p < N; ++p) {
    if (skip[p]) continue;
    const double* cp = C.data() + p * dp;
    double acc = 0.0;
    for (int j = 0; j < dp; ++j) {
      if (ip) acc += c[j] * cp[j];
      else { const double d = c[j] - cp[j]; acc += d * d; }
    }
    key.push_back({ip ? -acc : acc, (int32_t)p});
  }
  const size_t take = std::min<size_t>((size_t)std::max(r, 0), key.size());
  std::partial_sort(key.begin(), key.begin() + take, key.end());
  std::vector<int32_t> out;
  for (size_t i = 0; i < take; ++i) out.push_back(key[i].second);
  return out;
}

// Resize the per-partition device arrays to nlist entries (contents are
// uploaded afterwards; the access counters start at zero).
void realloc_tables(quake_index* idx, Store& st, hipStream_t s) {
  auto& mem = idx->mem;
  const int64_t N = std::max<int64_t>(st.nlist, 1);
  for (void* p : {(void*)st.d_off, (void*)st.d_size, (void*)st.d_cap, (void*)st.d_order, (void*)st.d_hits})
    mem.release(p);
  st.d_off = mem.alloc<int64_t>(N);
  st.d_size = mem.alloc<int32_t>(N);
  st.d_cap = mem.alloc<int32_t>(N);
  st.d_order = mem.alloc<int32_t>(N);
  st.d_hits = mem.alloc<uint32_t>(N);
  launch_fill_i32(reinterpret_cast<int32_t*>(st.d_hits), N, 0, s);
  if (st.attr) {
    // label counts per partition: recounted before the next filtered search
    mem.release(st.d_attr_cnt);
    st.d_attr_cnt = mem.alloc<uint32_t>((size_t)N * 33);
    st.attr_dirty = true;
  }
}

// Appends `extra` empty partitions (no tiles yet); their centroids are left
// for the caller to write.
void add_partitions(quake_index* idx, Store& st, int64_t extra, hipStream_t s) {
  if (extra <= 0) return;
  const int64_t N0 = st.nlist, N1 = N0 + extra;
  float* c = idx->mem.alloc<float>((size_t)N1 * st.dp);
  QK_HIP(hipMemcpyAsync(c, st.centroids, (size_t)N0 * st.dp * sizeof(float), hipMemcpyDeviceToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  idx->mem.release(st.centroids);
  st.centroids = c;
  st.off.resize(N1, st.used_tiles);
  st.size.resize(N1, 0);
  st.cap.resize(N1, 0);
  st.tomb.resize(N1, 0);
  st.nlist = N1;
  realloc_tables(idx, st, s);
}

// Removes the partitions with gone[p] set (they hold no vectors); the others
// keep their order.
void drop_partitions(quake_index* idx, Store& st, const std::vector<char>& gone, hipStream_t s) {
  std::vector<int64_t> keep;
  std::vector<int32_t> remap(st.nlist, -1);
  for (int64_t p = 0; p < st.nlist; ++p)
    if (!gone[p]) {
      remap[p] = (int32_t)keep.size();
      keep.push_back(p);
    }
  if ((int64_t)keep.size() == st.nlist) return;
  const int64_t N1 = (int64_t)keep.size();
  float* c = idx->mem.alloc<float>((size_t)std::max<int64_t>(N1, 1) * st.dp);
  {
    Buf<int64_t> rows(idx->mem, keep.size());
    upload(rows.p, keep, s);
    launch_gather_rows(st.centroids, st.dp, rows.p, N1, st.dp, c, s);
    QK_HIP(hipStreamSynchronize(s));
  }
  idx->mem.release(st.centroids);
  st.centroids = c;
  for (int32_t& t : st.tile_part)
    if (t >= 0) t = remap[t];
  std::vector<int64_t> off;
  std::vector<int32_t> size, cap, tomb;
  for (int64_t p : keep) {
    off.push_back(st.off[p]);
    size.push_back(st.size[p]);
    cap.push_back(st.cap[p]);
    tomb.push_back(st.tomb[p]);
  }
  st.off.swap(off);
  st.size.swap(size);
  st.cap.swap(cap);
  st.tomb.swap(tomb);
  st.nlist = N1;
  realloc_tables(idx, st, s);
}

// Moves the vectors in store slots src (ids `ids`) to the ends of the
// partitions dest, growing a receiving partition into fresh tiles when it
// lacks room; the partitions they leave are compacted.  Every copy of a
// vector moves with it and the id map follows.
int64_t move_rows(quake_index* idx, Store& st, std::vector<int64_t> src, const std::vector<int64_t>& ids,
                  const std::vector<int32_t>& dest, hipStream_t s) {
  const int64_t n = (int64_t)src.size();
  if (n == 0) return 0;
  std::vector<int32_t> from(n);
  for (int64_t i = 0; i < n; ++i) from[i] = st.tile_part[src[i] / TILE];
  std::vector<int64_t> cnt(st.nlist, 0);
  for (int32_t p : dest) cnt[p]++;
  std::vector<std::pair<int64_t, int32_t>> grow;
  int64_t extra = 0;
  for (int64_t p = 0; p < st.nlist; ++p) {
    if (cnt[p] == 0 || st.size[p] + cnt[p] <= st.cap[p]) continue;
    const int64_t want = round_up((int64_t)std::ceil((st.size[p] + cnt[p]) * 1.5), TILE);
    QK_CHECK(want <= INT32_MAX, QUAKE_E_INVALID, "partition too large");
    grow.push_back({p, (int32_t)want});
    extra += want / TILE;
  }
  store_grow_arena(idx, st, st.used_tiles + extra, s);
  std::vector<int64_t> old_base(st.nlist, -1);
  for (auto& g : grow) {
    old_base[g.first] = st.off[g.first] * TILE;
    store_relocate(st, g.first, g.second, s);
  }
  for (int64_t i = 0; i < n; ++i)
    if (old_base[from[i]] >= 0) src[i] = st.off[from[i]] * TILE + (src[i] - old_base[from[i]]);
  std::vector<int64_t> dst(n), fill(st.nlist, 0);
  for (int64_t i = 0; i < n; ++i) dst[i] = st.off[dest[i]] * TILE + st.size[dest[i]] + fill[dest[i]]++;
  for (int64_t p = 0; p < st.nlist; ++p) st.size[p] += (int32_t)cnt[p];
  {
    Buf<int64_t> d_src(idx->mem, n), d_dst(idx->mem, n), d_ids(idx->mem, n);
    upload(d_src.p, src, s);
    upload(d_dst.p, dst, s);
    upload(d_ids.p, ids, s);
    launch_move_slots(st, d_src.p, d_dst.p, n, s);
    launch_map_update(idx->idmap, d_ids.p, d_dst.p, n, s);
    QK_HIP(hipStreamSynchronize(s));
  }
  std::vector<char> left(st.nlist, 0);
  for (int32_t p : from) {
    st.tomb[p]++;
    left[p] = 1;
  }
  store_compact(idx, st, left, s);
  return n;
}

// Exact fixed-point k-means update of `nc` centroids c[nc][dp] from rows x
// labelled lab (every label in [0, nc)); a centroid with no rows keeps its value.
void update_centroids(quake_index* idx, const float* x, int64_t n, int dp, const int32_t* lab, int64_t nc, int bits,
                      float* c, hipStream_t s) {
  Buf<int64_t> sums(idx->mem, (size_t)nc * dp);
  Buf<int32_t> counts(idx->mem, (size_t)nc);
  QK_HIP(hipMemsetAsync(sums.p, 0, (size_t)nc * dp * sizeof(int64_t), s));
  QK_HIP(hipMemsetAsync(counts.p, 0, (size_t)nc * sizeof(int32_t), s));
  launch_kmeans_accumulate(x, n, dp, lab, bits, sums.p, counts.p, s);
  launch_kmeans_update(sums.p, counts.p, nc, dp, idx->metric == QUAKE_IP ? 1 : 0, bits, c, s);
  QK_HIP(hipStreamSynchronize(s));
}

struct SplitResult {
  int32_t part;
  std::vector<int64_t> slots, ids;
  std::vector<char> right;    // row goes to the right child
  int64_t nl = 0, nr = 0;
  std::vector<float> cl, cr;  // child centroids [dp]
};

// 2-means of each listed partition on the device (Sec. 4.2, "Split
// Partition"): start from the row farthest from the centroid and the row
// farthest from that one, `iters` Lloyd steps, then a final assignment.
std::vector<SplitResult> two_means(quake_index* idx, Store& st, const std::vector<int32_t>& parts, int iters,
                                   hipStream_t s) {
  const int dp = st.dp;
  const int metric = idx->metric;
  std::vector<int64_t> slots, ids, lo;
  live_rows(st, parts, slots, ids, lo, s);
  const int64_t n = (int64_t)slots.size();
  const int64_t S = (int64_t)parts.size();
  std::vector<SplitResult> out(S);
  for (int64_t g = 0; g < S; ++g) {
    out[g].part = parts[g];
    out[g].slots.assign(slots.begin() + lo[g], slots.begin() + lo[g + 1]);
    out[g].ids.assign(ids.begin() + lo[g], ids.begin() + lo[g + 1]);
  }
  // segments with no rows keep both children empty
  std::vector<int32_t> seg(n);
  for (int64_t g = 0; g < S; ++g)
    for (int64_t i = lo[g]; i < lo[g + 1]; ++i) seg[i] = (int32_t)g;
  Buf<int64_t> d_slots(idx->mem, n), d_lo(idx->mem, S + 1), far(idx->mem, S);
  Buf<int32_t> d_seg(idx->mem, n), lab(idx->mem, n);
  Buf<float> x(idx->mem, (size_t)n * dp), ref(idx->mem, (size_t)S * dp), c2(idx->mem, (size_t)2 * S * dp);
  upload(d_slots.p, slots, s);
  upload(d_lo.p, lo, s);
  upload(d_seg.p, seg, s);
  launch_gather_slots(st, d_slots.p, n, x.p, s);
  const int bits = store_fixed_point_bits(idx->mem, x.p, std::max<int64_t>(n, 1), dp, s);
  {
    std::vector<int64_t> rows(parts.begin(), parts.end());
    Buf<int64_t> d_rows(idx->mem, S);
    upload(d_rows.p, rows, s);
    launch_gather_rows(st.centroids, dp, d_rows.p, S, dp, ref.p, s);
    QK_HIP(hipStreamSynchronize(s));
  }
  // first start: farthest from the centroid; second: farthest from the first
  launch_seg_farthest(x.p, d_lo.p, S, ref.p, dp, metric, far.p, s);
  std::vector<int64_t> a = download(far.p, S, s);
  std::vector<int64_t> pick(2 * S);
  for (int64_t g = 0; g < S; ++g) a[g] = a[g] < 0 ? 0 : a[g];
  {
    Buf<int64_t> d_a(idx->mem, S);
    upload(d_a.p, a, s);
    launch_gather_rows(x.p, dp, d_a.p, S, dp, ref.p, s);
  }
  launch_seg_farthest(x.p, d_lo.p, S, ref.p, dp, metric, far.p, s);
  std::vector<int64_t> b = download(far.p, S, s);
  for (int64_t g = 0; g < S; ++g) {
    pick[2 * g] = a[g];
    pick[2 * g + 1] = b[g] < 0 ? 0 : b[g];
  }
  if (n > 0) {
    Buf<int64_t> d_pick(idx->mem, 2 * S);
    upload(d_pick.p, pick, s);
    launch_gather_rows(x.p, dp, d_pick.p, 2 * S, dp, c2.p, s);
    if (metric == QUAKE_IP) launch_normalise_rows(c2.p, 2 * S, dp, s);
    for (int it = 0; it < iters; ++it) {
      launch_seg_assign2(x.p, n, d_seg.p, c2.p, dp, metric, lab.p, s);
      update_centroids(idx, x.p, n, dp, lab.p, 2 * S, bits, c2.p, s);
    }
    launch_seg_assign2(x.p, n, d_seg.p, c2.p, dp, metric, lab.p, s);
  }
  std::vector<int32_t> h_lab = download(lab.p, n, s);
  std::vector<float> h_c = download(c2.p, (size_t)2 * S * dp, s);
  for (int64_t g = 0; g < S; ++g) {
    SplitResult& r = out[g];
    r.right.resize(lo[g + 1] - lo[g]);
    for (int64_t i = lo[g]; i < lo[g + 1]; ++i) {
      const bool right = (h_lab[i] & 1) != 0;
      r.right[i - lo[g]] = right;
      (right ? r.nr : r.nl)++;
    }
    r.cl.assign(h_c.begin() + (2 * g) * dp, h_c.begin() + (2 * g + 1) * dp);
    r.cr.assign(h_c.begin() + (2 * g + 1) * dp, h_c.begin() + (2 * g + 2) * dp);
  }
  return out;
}

// Nearest-centroid assignment of the live rows of `rows_of` among the
// centroids `among` (ascending partition ids): the receiving partition of
// every row.  With iters > 0, that many k-means passes seeded by the
// current centroids first update the centroids of `among` in the store.
struct Assignment {
  std::vector<int64_t> slots, ids;
  std::vector<int32_t> cur, dest;
};

Assignment assign_among(quake_index* idx, Store& st, const std::vector<int32_t>& rows_of,
                        const std::vector<int32_t>& among, int iters, hipStream_t s) {
  const int dp = st.dp;
  Assignment as;
  std::vector<int64_t> lo;
  live_rows(st, rows_of, as.slots, as.ids, lo, s);
  const int64_t n = (int64_t)as.slots.size();
  as.cur.resize(n);
  for (size_t g = 0; g < rows_of.size(); ++g)
    for (int64_t i = lo[g]; i < lo[g + 1]; ++i) as.cur[i] = rows_of[g];
  as.dest.assign(n, -1);
  const int64_t G = (int64_t)among.size();
  if (n == 0 || G == 0) return as;
  Buf<int64_t> d_slots(idx->mem, n);
  Buf<float> x(idx->mem, (size_t)n * dp), cg(idx->mem, (size_t)G * dp);
  Buf<int32_t> lab(idx->mem, n), d_among(idx->mem, G);
  upload(d_slots.p, as.slots, s);
  upload(d_among.p, among, s);
  launch_gather_slots(st, d_slots.p, n, x.p, s);
  {
    std::vector<int64_t> rows(among.begin(), among.end());
    Buf<int64_t> d_rows(idx->mem, G);
    upload(d_rows.p, rows, s);
    launch_gather_rows(st.centroids, dp, d_rows.p, G, dp, cg.p, s);
    QK_HIP(hipStreamSynchronize(s));
  }
  if (iters > 0) {
    const int bits = store_fixed_point_bits(idx->mem, x.p, n, dp, s);
    for (int it = 0; it < iters; ++it) {
      launch_nearest_of(x.p, n, cg.p, (int)G, dp, idx->metric, lab.p, s);
      update_centroids(idx, x.p, n, dp, lab.p, G, bits, cg.p, s);
    }
    launch_put_rows(cg.p, d_among.p, G, dp, st.centroids, s);
  }
  launch_nearest_of(x.p, n, cg.p, (int)G, dp, idx->metric, lab.p, s);
  std::vector<int32_t> h = download(lab.p, n, s);
  for (int64_t i = 0; i < n; ++i) as.dest[i] = among[h[i]];
  return as;
}

void check_params(const quake_maintain_params& p) {
  QK_CHECK(std::isfinite(p.tau) && p.tau >= 0, QUAKE_E_INVALID, "tau must be finite and >= 0");
  QK_CHECK(p.alpha > 0 && p.alpha <= 1, QUAKE_E_INVALID, "alpha must be in (0, 1]");
  QK_CHECK(p.refine_radius >= 0 && p.refine_iters >= 0, QUAKE_E_INVALID, "refine_radius and refine_iters must be >= 0");
  QK_CHECK(p.split_iters >= 1, QUAKE_E_INVALID, "split_iters must be >= 1");
  QK_CHECK(p.min_split_size >= 2, QUAKE_E_INVALID, "min_split_size must be >= 2");
  QK_CHECK(p.merge_below >= 0, QUAKE_E_INVALID, "merge_below must be >= 0");
  QK_CHECK(p.lambda_points >= 2 && p.lambda_size && p.lambda_cost, QUAKE_E_INVALID,
           "lambda needs at least two profiled points");
  for (int i = 0; i < p.lambda_points; ++i) {
    QK_CHECK(std::isfinite(p.lambda_size[i]) && std::isfinite(p.lambda_cost[i]), QUAKE_E_INVALID,
             "lambda holds a non-finite value");
    QK_CHECK(i == 0 || p.lambda_size[i] > p.lambda_size[i - 1], QUAKE_E_INVALID,
             "lambda sizes must be strictly ascending");
  }
  QK_CHECK(p.max_decisions >= 0 && (p.max_decisions == 0 || p.decisions), QUAKE_E_INVALID,
           "decisions is NULL but max_decisions > 0");
  QK_CHECK(!p.hits || p.window >= 1, QUAKE_E_INVALID, "window must be >= 1 with hits");
}

}  // namespace

void maintain(quake_index* idx, const quake_maintain_params& p, quake_maintain_report* report, hipStream_t s) {
  check_params(p);
  Store& st = idx->L0;
  const int dp = st.dp;
  const int ip = idx->metric == QUAKE_IP ? 1 : 0;
  const int64_t N0 = st.nlist;

  // Stage 0: sizes and access frequencies A_j = hits_j / |W|
  std::vector<double> A0(N0, 0.0);
  if (p.hits) {
    for (int64_t j = 0; j < N0; ++j) {
      QK_CHECK(p.hits[j] >= 0, QUAKE_E_INVALID, "hits must be >= 0");
      A0[j] = (double)p.hits[j] / (double)p.window;
    }
  } else if (st.window > 0) {
    std::vector<uint32_t> h = download(st.d_hits, N0, s);
    for (int64_t j = 0; j < N0; ++j) A0[j] = (double)h[j] / (double)st.window;
  }
  Latency lam{std::vector<double>(p.lambda_size, p.lambda_size + p.lambda_points),
              std::vector<double>(p.lambda_cost, p.lambda_cost + p.lambda_points)};
  // centroid overhead of one more / one fewer partition, at the count before the pass
  const double dO_plus = lam((double)N0 + 1) - lam((double)N0);
  const double dO_minus = lam((double)N0 - 1) - lam((double)N0);
  std::vector<double> A = A0;
  std::vector<quake_decision> dec;
  int64_t moved = 0;
  int32_t n_split = 0, n_delete = 0;

  // Stages 1-3 for splits (Eqs. delta_split_est, delta_split_exact)
  std::vector<int32_t> cands;
  std::vector<double> est;
  std::vector<char> tried(N0, 0);
  for (int64_t j = 0; j < N0; ++j) {
    const double sj = (double)live_size(st, j);
    if (sj < p.min_split_size) continue;
    const double e = dO_plus - A0[j] * lam(sj) + 2.0 * p.alpha * A0[j] * lam(sj / 2.0);
    if (e < -p.tau) {
      cands.push_back((int32_t)j);
      est.push_back(e);
      tried[j] = 1;
    }
  }
  std::vector<std::pair<int32_t, int32_t>> children;  // (left = parent id, right)
  // splits are computed in batches of at most 2^21 rows
  size_t b0 = 0;
  std::vector<SplitResult> done;
  while (b0 < cands.size()) {
    size_t b1 = b0;
    int64_t rows = 0;
    while (b1 < cands.size() && (b1 == b0 || rows + live_size(st, cands[b1]) <= (int64_t{1} << 21)))
      rows += live_size(st, cands[b1++]);
    std::vector<int32_t> batch(cands.begin() + b0, cands.begin() + b1);
    std::vector<SplitResult> r = two_means(idx, st, batch, p.split_iters, s);
    for (auto& x : r) done.push_back(std::move(x));
    b0 = b1;
  }
  std::vector<int> commit_of;
  for (size_t g = 0; g < done.size(); ++g) {
    const int32_t j = done[g].part;
    const double sj = (double)live_size(st, j);
    const double aj = p.alpha * A0[j];
    const double ver =
        dO_plus - A0[j] * lam(sj) + aj * lam((double)done[g].nl) + aj * lam((double)done[g].nr);
    const bool ok = ver < -p.tau;
    dec.push_back({j, 0, ok ? 1 : 0, -1, est[g], ver});
    if (ok) commit_of.push_back((int)g);
  }
  if (!commit_of.empty()) {
    const int64_t K = (int64_t)commit_of.size();
    add_partitions(idx, st, K, s);
    std::vector<float> cents;
    std::vector<int32_t> rows;
    std::vector<int64_t> src, ids;
    std::vector<int32_t> dest;
    for (int64_t t = 0; t < K; ++t) {
      SplitResult& r = done[commit_of[t]];
      const int32_t right = (int32_t)(N0 + t);
      children.push_back({r.part, right});
      cents.insert(cents.end(), r.cl.begin(), r.cl.end());
      cents.insert(cents.end(), r.cr.begin(), r.cr.end());
      rows.push_back(r.part);
      rows.push_back(right);
      for (size_t i = 0; i < r.slots.size(); ++i)
        if (r.right[i]) {
          src.push_back(r.slots[i]);
          ids.push_back(r.ids[i]);
          dest.push_back(right);
        }
      for (auto& d : dec)
        if (d.action == 0 && d.partition == r.part) d.new_partition = right;
      A[r.part] = p.alpha * A0[r.part];
      A.push_back(p.alpha * A0[r.part]);
    }
    {
      Buf<float> d_c(idx->mem, cents.size());
      Buf<int32_t> d_rows(idx->mem, rows.size());
      upload(d_c.p, cents, s);
      upload(d_rows.p, rows, s);
      launch_put_rows(d_c.p, d_rows.p, (int64_t)rows.size(), dp, st.centroids, s);
      QK_HIP(hipStreamSynchronize(s));
    }
    moved += move_rows(idx, st, src, ids, dest, s);
    n_split = (int32_t)K;
  }

  // refinement around each committed split, in commit order (Sec. 4.2,
  // "Partition Refinement")
  if (p.refine_iters > 0) {
    for (auto& ch : children) {
      const std::vector<double> C = host_centroids(st, s);
      std::vector<char> skip(st.nlist, 0);
      skip[ch.first] = skip[ch.second] = 1;
      std::vector<int32_t> group = {ch.first, ch.second};
      for (int32_t c : {ch.first, ch.second}) {
        std::vector<int32_t> nb = nearest_centroids(C, st.nlist, dp, C.data() + (int64_t)c * dp, p.refine_radius,
                                                    skip, ip);
        group.insert(group.end(), nb.begin(), nb.end());
      }
      std::sort(group.begin(), group.end());
      group.erase(std::unique(group.begin(), group.end()), group.end());
      Assignment as = assign_among(idx, st, group, group, p.refine_iters, s);
      std::vector<int64_t> src, ids;
      std::vector<int32_t> dest;
      for (size_t i = 0; i < as.slots.size(); ++i)
        if (as.dest[i] != as.cur[i]) {
          src.push_back(as.slots[i]);
          ids.push_back(as.ids[i]);
          dest.push_back(as.dest[i]);
        }
      moved += move_rows(idx, st, src, ids, dest, s);
    }
  }

  // Stages 1-3 for deletes (Eq. delta_merge_exact; the estimate spreads the
  // partition's vectors and accesses evenly over its nearest partitions)
  if (p.merge_below > 0) {
    const std::vector<double> C = host_centroids(st, s);
    std::vector<char> gone(st.nlist, 0);
    for (int64_t j = 0; j < N0; ++j) {
      const double sj = (double)live_size(st, j);
      if (tried[j] || !(sj < (double)p.merge_below)) continue;
      std::vector<int32_t> alive;
      for (int64_t m = 0; m < st.nlist; ++m)
        if (m != j && !gone[m]) alive.push_back((int32_t)m);
      if (alive.empty()) continue;
      std::vector<char> skip(gone);
      skip[j] = 1;
      const std::vector<int32_t> rec =
          nearest_centroids(C, st.nlist, dp, C.data() + j * dp, p.refine_radius, skip, ip);
      double e = dO_minus - A0[j] * lam(sj);
      if (!rec.empty()) {
        const double r = (double)rec.size();
        for (int32_t m : rec) {
          const double sm = (double)live_size(st, m);
          e += (A[m] + A0[j] / r) * lam(sm + sj / r) - A[m] * lam(sm);
        }
      }
      if (!(e < -p.tau)) continue;
      Assignment as = assign_among(idx, st, {(int32_t)j}, alive, 0, s);
      std::vector<int64_t> ds(st.nlist, 0);
      for (int32_t m : as.dest) ds[m]++;
      double ver = dO_minus - A0[j] * lam(sj);
      for (int64_t m = 0; m < st.nlist; ++m) {
        if (ds[m] == 0) continue;
        const double sm = (double)live_size(st, m);
        ver += (A[m] + A0[j] * (double)ds[m] / sj) * lam(sm + (double)ds[m]) - A[m] * lam(sm);
      }
      const bool ok = ver < -p.tau;
      dec.push_back({(int32_t)j, 1, ok ? 1 : 0, -1, e, ver});
      if (!ok) continue;
      moved += move_rows(idx, st, as.slots, as.ids, as.dest, s);
      gone[j] = 1;
      ++n_delete;
    }
    drop_partitions(idx, st, gone, s);
  }

  store_upload_table(st, s);
  launch_fill_i32(reinterpret_cast<int32_t*>(st.d_hits), std::max<int64_t>(st.nlist, 1), 0, s);
  st.window = 0;
  st.attr_dirty = true;
  // product codes hold residuals to the centroids: rows that changed partition
  // and partitions whose centroid moved are encoded again (all rows, once)
  if (st.codes && (n_split > 0 || n_delete > 0 || moved > 0)) encode_store(idx, st, s);
  QK_HIP(hipStreamSynchronize(s));
  if (idx->n_levels >= 2) rebuild_level1(idx, s);
  release_graphs(idx);
  if (p.decisions)
    for (size_t i = 0; i < dec.size() && (int64_t)i < p.max_decisions; ++i) p.decisions[i] = dec[i];
  if (report) {
    report->decisions = (int32_t)dec.size();
    report->splits = n_split;
    report->deletes = n_delete;
    report->pad = 0;
    report->nlist_before = N0;
    report->nlist_after = st.nlist;
    report->vectors_moved = moved;
  }
}

}  // namespace qk

extern "C" {

int quake_maintain(quake_index* index, const quake_maintain_params* params, quake_maintain_report* report,
                   void* stream) {
  return qk::run_api([&] {
    QK_CHECK(index && index->magic == 0x51554b45u, QUAKE_E_STATE, "invalid or freed index handle");
    QK_CHECK(params, QUAKE_E_INVALID, "params is NULL");
    qk::maintain(index, *params, report, reinterpret_cast<hipStream_t>(stream));
  });
}

int quake_profile_latency(quake_index* index, const int32_t* sizes, int32_t points, int32_t nq,
                          const quake_search_params* params, int32_t reps, double* out_us, void* stream) {
  return qk::run_api([&] {
    QK_CHECK(index && index->magic == 0x51554b45u, QUAKE_E_STATE, "invalid or freed index handle");
    QK_CHECK(sizes && out_us && points >= 1, QUAKE_E_INVALID, "need sizes, out_us and points >= 1");
    QK_CHECK(nq >= 1 && reps >= 1 && params, QUAKE_E_INVALID, "need nq >= 1, reps >= 1 and params");
    qk::Store& st = index->L0;
    constexpr int PARTS = 8;  // partitions of each profiling index
    int64_t want = nq;
    for (int32_t i = 0; i < points; ++i) {
      QK_CHECK(sizes[i] >= 1, QUAKE_E_INVALID, "sizes must be >= 1");
      want = std::max<int64_t>(want, (int64_t)PARTS * sizes[i]);
    }
    QK_CHECK(want <= st.live, QUAKE_E_INVALID, "the index holds fewer than 8 x the largest size (or nq) vectors");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int d = index->d, dp = index->dp;
    // the first `want` live vectors of the store, partition by partition
    std::vector<int64_t> slots, ids, lo;
    std::vector<int32_t> parts;
    int64_t have = 0;
    for (int64_t p = 0; p < st.nlist && have < want; ++p) {
      parts.push_back((int32_t)p);
      have += qk::live_size(st, p);
    }
    qk::live_rows(st, parts, slots, ids, lo, s);
    slots.resize(want);
    qk::Buf<int64_t> d_slots(index->mem, want);
    qk::Buf<float> xp(index->mem, (size_t)want * dp), x(index->mem, (size_t)want * d);
    qk::upload(d_slots.p, slots, s);
    qk::launch_gather_slots(st, d_slots.p, want, xp.p, s);
    QK_HIP(hipMemcpy2DAsync(x.p, d * sizeof(float), xp.p, dp * sizeof(float), d * sizeof(float), want,
                            hipMemcpyDeviceToDevice, s));
    QK_HIP(hipStreamSynchronize(s));
    quake_search_params sp = *params;
    sp.recall_target = 0.0;
    qk::Buf<int64_t> oi(index->mem, (size_t)nq * std::max(sp.k, 1));
    qk::Buf<float> od(index->mem, (size_t)nq * std::max(sp.k, 1));
    qk::Buf<int32_t> assign(index->mem, (size_t)want);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QK_HIP(hipEventCreate(&e0));
    QK_HIP(hipEventCreate(&e1));
    struct Events {
      hipEvent_t a, b;
      ~Events() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } ev{e0, e1};
    for (int32_t i = 0; i < points; ++i) {
      // an index of eight partitions of sizes[i] of those vectors each (same
      // metric and copies); a partition scanned beyond the first costs
      // (time with all eight - time with one) / 7 per query: what the
      // cost model's lambda is, without the per-query work (centroid
      // scoring, selection, rerank) every search does once
      const int64_t n = (int64_t)PARTS * sizes[i];
      std::vector<int32_t> a(n);
      for (int64_t r = 0; r < n; ++r) a[r] = (int32_t)(r / sizes[i]);
      qk::upload(assign.p, a, s);
      QK_HIP(hipStreamSynchronize(s));
      quake_build_params bp{};
      bp.metric = index->metric;
      bp.storage_dtype = index->storage;
      // the same product codes (same codebook): a search over codes profiles lambda for that scan
      bp.pq_m = index->pq_m;
      bp.pq_codebook = index->pq_book;
      bp.n_levels = 1;
      bp.nlist = PARTS;
      bp.assign = assign.p;
      quake_index* tmp = nullptr;
      const quake_allocator* alloc = index->mem.user.alloc ? &index->mem.user : nullptr;
      int rc = quake_build(x.p, nullptr, n, d, &bp, alloc, stream, &tmp);
      QK_CHECK(rc == QUAKE_OK, rc, "profile build: " + qk::g_error);
      std::unique_ptr<quake_index, void (*)(quake_index*)> hold(tmp, quake_free);
      double us[2];
      for (int v = 0; v < 2; ++v) {
        sp.nprobe = v == 0 ? 1 : PARTS;
        auto run = [&] {
          const int r = quake_search(tmp, x.p, nq, &sp, oi.p, od.p, nullptr, nullptr, stream);
          QK_CHECK(r == QUAKE_OK, r, "profile search: " + qk::g_error);
        };
        run();  // grows the workspace and captures the round graphs
        QK_HIP(hipEventRecord(e0, s));
        for (int32_t r = 0; r < reps; ++r) run();
        QK_HIP(hipEventRecord(e1, s));
        QK_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        QK_HIP(hipEventElapsedTime(&ms, e0, e1));
        us[v] = (double)ms * 1e3 / reps / nq;
      }
      out_us[i] = std::max(0.0, (us[1] - us[0]) / (PARTS - 1));
    }
  });
}

int quake_access_stats(quake_index* index, int32_t level, int64_t* hits, int64_t* window, int32_t reset,
                       void* stream) {
  return qk::run_api([&] {
    QK_CHECK(index && index->magic == 0x51554b45u, QUAKE_E_STATE, "invalid or freed index handle");
    QK_CHECK(level >= 0 && level < index->n_levels, QUAKE_E_INVALID, "no such level");
    qk::Store& st = level == 0 ? index->L0 : level == 1 ? index->L1 : index->L2;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hits) {
      std::vector<uint32_t> h(st.nlist);
      QK_HIP(hipMemcpyAsync(h.data(), st.d_hits, st.nlist * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      QK_HIP(hipStreamSynchronize(s));
      for (int64_t j = 0; j < st.nlist; ++j) hits[j] = h[j];
    }
    if (window) *window = st.window;
    if (reset) {
      qk::launch_fill_i32(reinterpret_cast<int32_t*>(st.d_hits), std::max<int64_t>(st.nlist, 1), 0, s);
      st.window = 0;
      QK_HIP(hipStreamSynchronize(s));
    }
  });
}

}  // extern "C"

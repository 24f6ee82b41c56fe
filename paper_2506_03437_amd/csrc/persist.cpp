// Saving an index to a file and loading it back.
//
// The file holds the index's logical content, not its device layout: the
// level-0 centroids, the access statistics, a two-level index's level 1
// (its centroids and the top partition of every level-0 centroid), and every
// live vector with its id, partition and (for a labelled index) label bits,
// partition by partition in store order, and the product-quantization
// codebook when the index keeps codes (loading re-encodes the rows with it,
// which gives the same codes).  Loading builds a fresh store from that content with the given
// centroids and assignment, so each partition keeps its rows in the saved
// order (deleted slots and relocation gaps are gone) and every search on the
// loaded index sees the same partitions, centroids and rows.
//
// Layout (little-endian): a 128-byte header (magic "QUAKEIX1", version,
// sizes, metric, storage, capacity slack, scheduling knobs, access window),
// from version 2 a 16-byte extension (product-quantization subspaces and
// their width), then the sections above as flat arrays, then the 64-bit
// FNV-1a hash of all bytes before it.  Version 1 files (no extension, no
// codes) still load.  A file is written to "<path>.tmp" and renamed into place.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "engine.hpp"
#include "index.hpp"

namespace qk {
namespace {

constexpr char kMagic[8] = {'Q', 'U', 'A', 'K', 'E', 'I', 'X', '1'};
constexpr uint32_t kVersion = 2;
constexpr int64_t kChunkRows = 65536;  // rows per device <-> host transfer

struct FileHeader {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  int32_t d, metric, storage, n_levels, drop_f32_tiles, labelled;
  int64_t nlist, nlist_top, n_live, window;
  double capacity_slack;
  quake_tuning tune;
  int64_t nlist_top2;  // level-2 partitions of a three-level index, else 0
};
static_assert(sizeof(FileHeader) == 128, "file header is 128 bytes");

// Version 2 and later: follows the header.
struct FileHeaderExt {
  int32_t pq_m, pq_ds;  // product quantization (0, 0 = none)
  int64_t reserved;
};
static_assert(sizeof(FileHeaderExt) == 16, "header extension is 16 bytes");

// 64-bit FNV-1a over the bytes written or read so far.
struct Hash {
  uint64_t h = 0xcbf29ce484222325ull;
  void add(const void* p, size_t n) {
    const uint8_t* b = static_cast<const uint8_t*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 0x100000001b3ull; }
  }
};

struct File {
  FILE* f = nullptr;
  ~File() { if (f) std::fclose(f); }
};

struct Writer {
  FILE* f;
  Hash hash;
  void put(const void* p, size_t n) {
    if (n == 0) return;
    QK_CHECK(std::fwrite(p, 1, n, f) == n, QUAKE_E_IO, "write failed");
    hash.add(p, n);
  }
};

struct Reader {
  FILE* f;
  Hash hash;
  void get(void* p, size_t n) {
    if (n == 0) return;
    QK_CHECK(std::fread(p, 1, n, f) == n, QUAKE_E_INVALID, "the file ends early: not a complete saved index");
    hash.add(p, n);
  }
};

template <class T>
struct Buf {
  DeviceMemory* mem;
  T* p = nullptr;
  Buf(DeviceMemory& m, size_t n) : mem(&m) { p = m.alloc<T>(std::max<size_t>(n, 1)); }
  ~Buf() { mem->release(p); }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
};

// rows [n][dp] on the device -> host [n][d]
std::vector<float> strip_rows(const float* src, int64_t n, int d, int dp, hipStream_t s) {
  std::vector<float> out((size_t)n * d);
  if (n > 0)
    QK_HIP(hipMemcpy2DAsync(out.data(), d * sizeof(float), src, dp * sizeof(float), d * sizeof(float), n,
                            hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  return out;
}

void save(quake_index* idx, const char* path, hipStream_t s) {
  QK_CHECK(path && *path, QUAKE_E_INVALID, "path is empty");
  const Store& st = idx->L0;
  QK_CHECK(st.live > 0, QUAKE_E_INVALID, "the index holds no vectors");
  QK_HIP(hipStreamSynchronize(s));
  const int d = idx->d, dp = idx->dp;

  // live slots, partition by partition in store order
  std::vector<int64_t> sid((size_t)st.tiles * TILE);
  if (!sid.empty())
    QK_HIP(hipMemcpyAsync(sid.data(), st.ids, sid.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  std::vector<uint32_t> all_attr;
  if (st.attr) {
    all_attr.resize(sid.size());
    QK_HIP(hipMemcpyAsync(all_attr.data(), st.attr, all_attr.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
  }
  std::vector<int64_t> slots, ids;
  std::vector<int32_t> part;
  std::vector<uint32_t> attr;
  slots.reserve(st.live);
  ids.reserve(st.live);
  part.reserve(st.live);
  for (int64_t p = 0; p < st.nlist; ++p) {
    const int64_t base = st.off[p] * TILE;
    for (int64_t j = 0; j < st.size[p]; ++j) {
      const int64_t id = sid[base + j];
      if (id < 0) continue;
      slots.push_back(base + j);
      ids.push_back(id);
      part.push_back((int32_t)p);
      if (st.attr) attr.push_back(all_attr[base + j]);
    }
  }
  QK_CHECK((int64_t)ids.size() == st.live, QUAKE_E_DEVICE, "live count and store disagree");
  const int64_t n = st.live;

  FileHeader hd;
  std::memset(&hd, 0, sizeof(hd));
  std::memcpy(hd.magic, kMagic, 8);
  hd.version = kVersion;
  hd.header_bytes = sizeof(FileHeader);
  hd.d = d;
  hd.metric = idx->metric;
  hd.storage = idx->storage;
  hd.n_levels = idx->n_levels;
  hd.drop_f32_tiles = st.v32 ? 0 : 1;
  hd.labelled = st.attr ? 1 : 0;
  hd.nlist = st.nlist;
  hd.nlist_top = idx->n_levels >= 2 ? idx->L1.nlist : 0;
  hd.nlist_top2 = idx->n_levels >= 3 ? idx->L2.nlist : 0;
  hd.n_live = n;
  hd.window = st.window;
  hd.capacity_slack = idx->slack;
  hd.tune = idx->tune;

  const std::string tmp = std::string(path) + ".tmp";
  File file;
  file.f = std::fopen(tmp.c_str(), "wb");
  QK_CHECK(file.f, QUAKE_E_IO, "cannot open " + tmp + " for writing");
  Writer w{file.f, {}};
  w.put(&hd, sizeof(hd));
  FileHeaderExt ext{idx->pq_m, idx->pq_ds, 0};
  w.put(&ext, sizeof(ext));
  const std::vector<float> C0 = strip_rows(st.centroids, st.nlist, d, dp, s);
  w.put(C0.data(), C0.size() * sizeof(float));
  std::vector<uint32_t> hits(st.nlist);
  QK_HIP(hipMemcpyAsync(hits.data(), st.d_hits, st.nlist * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  QK_HIP(hipStreamSynchronize(s));
  w.put(hits.data(), hits.size() * sizeof(uint32_t));
  for (int level = 1; level < idx->n_levels; ++level) {
    const Store& up = level == 1 ? idx->L1 : idx->L2;
    const int64_t nbelow = level == 1 ? st.nlist : idx->L1.nlist;
    const std::vector<float> C = strip_rows(up.centroids, up.nlist, d, dp, s);
    w.put(C.data(), C.size() * sizeof(float));
    std::vector<int32_t> parent(nbelow);
    QK_HIP(hipMemcpyAsync(parent.data(), level == 1 ? idx->top_of : idx->top_of2, nbelow * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    w.put(parent.data(), parent.size() * sizeof(int32_t));
  }
  w.put(ids.data(), ids.size() * sizeof(int64_t));
  w.put(part.data(), part.size() * sizeof(int32_t));
  w.put(attr.data(), attr.size() * sizeof(uint32_t));
  {
    const int64_t chunk = std::min<int64_t>(kChunkRows, n);
    Buf<int64_t> d_slots(idx->mem, chunk);
    Buf<float> rows(idx->mem, (size_t)chunk * dp);
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
      const int64_t m = std::min(chunk, n - r0);
      QK_HIP(hipMemcpyAsync(d_slots.p, slots.data() + r0, m * sizeof(int64_t), hipMemcpyHostToDevice, s));
      launch_gather_slots(st, d_slots.p, m, rows.p, s);
      const std::vector<float> h = strip_rows(rows.p, m, d, dp, s);
      w.put(h.data(), h.size() * sizeof(float));
    }
  }
  if (idx->pq_m > 0) {
    std::vector<float> book((size_t)idx->pq_m * 256 * idx->pq_ds);
    QK_HIP(hipMemcpyAsync(book.data(), idx->pq_book, book.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    w.put(book.data(), book.size() * sizeof(float));
  }
  const uint64_t sum = w.hash.h;
  QK_CHECK(std::fwrite(&sum, 1, 8, file.f) == 8, QUAKE_E_IO, "write failed");
  QK_CHECK(std::fflush(file.f) == 0, QUAKE_E_IO, "write failed");
  std::fclose(file.f);
  file.f = nullptr;
  QK_CHECK(std::rename(tmp.c_str(), path) == 0, QUAKE_E_IO, std::string("cannot rename the file to ") + path);
}

quake_index* load(const char* path, const quake_allocator* allocator, size_t hbm_budget_bytes, hipStream_t s) {
  QK_CHECK(path && *path, QUAKE_E_INVALID, "path is empty");
  File file;
  file.f = std::fopen(path, "rb");
  QK_CHECK(file.f, QUAKE_E_IO, std::string("cannot open ") + path);
  Reader r{file.f, {}};
  FileHeader hd;
  r.get(&hd, sizeof(hd));
  QK_CHECK(std::memcmp(hd.magic, kMagic, 8) == 0, QUAKE_E_INVALID, "not a saved index (magic)");
  QK_CHECK((hd.version == 1 || hd.version == kVersion) && hd.header_bytes == sizeof(FileHeader), QUAKE_E_INVALID,
           "unsupported file version");
  FileHeaderExt ext{0, 0, 0};
  if (hd.version >= 2) r.get(&ext, sizeof(ext));
  QK_CHECK(hd.d >= 1 && hd.d <= MAX_DIM && hd.nlist >= 1 && hd.nlist <= INT32_MAX && hd.n_live >= 1 &&
               (hd.n_levels == 1 || (hd.n_levels >= 2 && hd.n_levels <= 3 && hd.nlist_top >= 1 && hd.nlist_top <= hd.nlist)) &&
               (hd.n_levels == 3 ? hd.nlist_top2 >= 1 && hd.nlist_top2 <= hd.nlist_top : hd.nlist_top2 == 0) &&
               hd.capacity_slack >= 0 && hd.window >= 0 && (hd.labelled == 0 || hd.labelled == 1),
           QUAKE_E_INVALID, "corrupt header");
  QK_CHECK(ext.pq_m == 0 ? ext.pq_ds == 0
                         : ext.pq_m > 0 && ext.pq_m % 4 == 0 && hd.d % ext.pq_m == 0 && ext.pq_ds == hd.d / ext.pq_m &&
                               ext.pq_ds <= PQ_MAX_SUB,
           QUAKE_E_INVALID, "corrupt header (product quantization)");
  const int d = hd.d;
  const int64_t n = hd.n_live, N = hd.nlist;

  // device staging through the caller's allocator, released after the build
  DeviceMemory tmp;
  if (allocator && allocator->alloc) tmp.user = *allocator;
  auto to_device = [&](void* dst, size_t bytes) {
    std::vector<uint8_t> h(std::min<size_t>(bytes, (size_t)kChunkRows * d * sizeof(float)));
    for (size_t o = 0; o < bytes; o += h.size()) {
      const size_t m = std::min(h.size(), bytes - o);
      r.get(h.data(), m);
      QK_HIP(hipMemcpyAsync(static_cast<uint8_t*>(dst) + o, h.data(), m, hipMemcpyHostToDevice, s));
      QK_HIP(hipStreamSynchronize(s));
    }
  };
  Buf<float> C0(tmp, (size_t)N * d);
  to_device(C0.p, (size_t)N * d * sizeof(float));
  std::vector<uint32_t> hits(N);
  r.get(hits.data(), N * sizeof(uint32_t));
  std::unique_ptr<Buf<float>> C1, C2;
  std::unique_ptr<Buf<int32_t>> top, top2;
  if (hd.n_levels >= 2) {
    C1.reset(new Buf<float>(tmp, (size_t)hd.nlist_top * d));
    to_device(C1->p, (size_t)hd.nlist_top * d * sizeof(float));
    top.reset(new Buf<int32_t>(tmp, N));
    to_device(top->p, N * sizeof(int32_t));
  }
  if (hd.n_levels == 3) {
    C2.reset(new Buf<float>(tmp, (size_t)hd.nlist_top2 * d));
    to_device(C2->p, (size_t)hd.nlist_top2 * d * sizeof(float));
    top2.reset(new Buf<int32_t>(tmp, hd.nlist_top));
    to_device(top2->p, hd.nlist_top * sizeof(int32_t));
  }
  Buf<int64_t> ids(tmp, n);
  to_device(ids.p, n * sizeof(int64_t));
  Buf<int32_t> part(tmp, n);
  to_device(part.p, n * sizeof(int32_t));
  std::unique_ptr<Buf<uint32_t>> attr;
  if (hd.labelled) {
    attr.reset(new Buf<uint32_t>(tmp, n));
    to_device(attr->p, n * sizeof(uint32_t));
  }
  Buf<float> x(tmp, (size_t)n * d);
  to_device(x.p, (size_t)n * d * sizeof(float));
  std::unique_ptr<Buf<float>> book;
  if (ext.pq_m > 0) {
    book.reset(new Buf<float>(tmp, (size_t)ext.pq_m * 256 * ext.pq_ds));
    to_device(book->p, (size_t)ext.pq_m * 256 * ext.pq_ds * sizeof(float));
  }
  const uint64_t expect = r.hash.h;
  uint64_t sum = 0;
  QK_CHECK(std::fread(&sum, 1, 8, file.f) == 8, QUAKE_E_INVALID, "the file ends early: not a complete saved index");
  QK_CHECK(sum == expect, QUAKE_E_INVALID, "checksum mismatch: the file is corrupt");
  QK_CHECK(std::fgetc(file.f) == EOF, QUAKE_E_INVALID, "trailing bytes after the saved index");

  quake_build_params bp{};
  bp.metric = hd.metric;
  bp.storage_dtype = hd.storage;
  bp.n_levels = hd.n_levels >= 2 ? 2 : 1;
  bp.nlist = N;
  bp.nlist_top = hd.nlist_top;
  bp.centroids = C0.p;
  bp.assign = part.p;
  bp.hbm_budget_bytes = hbm_budget_bytes;
  bp.capacity_slack = hd.capacity_slack;
  bp.drop_f32_tiles = hd.drop_f32_tiles;
  bp.attrs = attr ? attr->p : nullptr;
  bp.pq_m = ext.pq_m;
  bp.pq_codebook = book ? book->p : nullptr;
  std::unique_ptr<quake_index> idx(
      build_index(x.p, ids.p, n, d, &bp, C1 ? C1->p : nullptr, top ? top->p : nullptr, allocator, s));
  if (hd.n_levels == 3) {
    build_top_level(idx.get(), 2, hd.nlist_top2, 0, 0, C2->p, top2->p, s);
    idx->n_levels = 3;
  }
  QK_HIP(hipMemcpyAsync(idx->L0.d_hits, hits.data(), N * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  QK_HIP(hipStreamSynchronize(s));
  idx->L0.window = hd.window;
  idx->tune = hd.tune;
  return idx.release();
}

}  // namespace
}  // namespace qk

extern "C" {

int quake_save(quake_index* index, const char* path, void* stream) {
  return qk::run_api([&] {
    QK_CHECK(index && index->magic == 0x51554b45u, QUAKE_E_STATE, "invalid or freed index handle");
    qk::save(index, path, reinterpret_cast<hipStream_t>(stream));
  });
}

int quake_load(const char* path, const quake_allocator* allocator, size_t hbm_budget_bytes, void* stream,
               quake_index** out) {
  return qk::run_api([&] {
    QK_CHECK(out, QUAKE_E_INVALID, "out is NULL");
    *out = nullptr;
    *out = qk::load(path, allocator, hbm_budget_bytes, reinterpret_cast<hipStream_t>(stream));
  });
}

}  // extern "C"

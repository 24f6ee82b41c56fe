// Serving loop: continuous batching of single-query searches, with update
// batches applied between epochs.
//
// The worker thread keeps up to `cap` searches in flight, each in a slot of
// the index's search workspace.  Every iteration it (1) admits queued
// searches into free slots - scoring and ordering their candidates and
// resetting their state - (2) runs one scan round over all slots (finished
// and free slots do no work), and (3) answers the slots whose adaptive scan
// stopped in that round and frees them.  A search therefore joins a batch
// already in progress and its work items share rounds (and, on the batched
// path, partition reads) with searches admitted earlier.  Per-query results
// do not depend on the company a query keeps: every step of a query's search
// reads only that query's own state.
//
// Updates.  By default an update request at the head of the queue stops
// admission until the slots drain, then runs as one batch.  With
// overlap_updates the server keeps a second copy of the level-0 store (a
// copy-on-write view made coarse: HBM holds two versions of the index): an
// update is applied to the copy that no search is reading, the two swap, and
// new searches run on the new version while the searches admitted before the
// update finish on the old one - every round scans each version for its own
// query slots (slot tags).  The old version catches up by replaying the
// update once its last search has finished; an update only waits for the
// version before the current one to drain.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.hpp"
#include "index.hpp"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int kind = 0;  // 0 search, 1 insert, 2 delete
  std::vector<float> x;
  std::vector<int64_t> ids;
  double arrive = 0;
};

struct Answer {
  bool ready = false;
  int status = QUAKE_OK;
  std::vector<int64_t> ids;
  std::vector<float> dist;
  int32_t nscanned = 0;
};

template <class T>
T* dup(qk::DeviceMemory& mem, std::vector<void*>& got, const T* src, size_t n, hipStream_t s) {
  if (!src) return nullptr;
  T* p = mem.alloc<T>(std::max<size_t>(n, 1));
  got.push_back(p);
  if (n) QK_HIP(hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyDeviceToDevice, s));
  return p;
}

// Second copy of a level-0 store and its id map (the access counters are shared).
void clone_store(qk::DeviceMemory& mem, const qk::Store& a, const qk::IdMap& am, qk::Store& b, qk::IdMap& bm,
                 hipStream_t s) {
  std::vector<void*> got;
  try {
    qk::Store t = a;
    const size_t slots = (size_t)a.tiles * qk::TILE, N = (size_t)a.nlist;
    t.centroids = dup(mem, got, a.centroids, N * a.dp, s);
    t.d_off = dup(mem, got, a.d_off, N, s);
    t.d_size = dup(mem, got, a.d_size, N, s);
    t.d_cap = dup(mem, got, a.d_cap, N, s);
    t.d_order = dup(mem, got, a.d_order, N, s);
    t.v32 = dup(mem, got, a.v32, slots * a.dp, s);
    t.v16 = dup(mem, got, a.v16, slots * a.dp16, s);
    t.v16n = dup(mem, got, a.v16n, slots, s);
    t.rows32 = dup(mem, got, a.rows32, slots * a.dp, s);
    t.ids = dup(mem, got, a.ids, slots, s);
    t.attr = dup(mem, got, a.attr, slots, s);
    t.codes = dup(mem, got, a.codes, slots * qk::pq_words(a.pq_m), s);
    t.d_attr_cnt = dup(mem, got, a.d_attr_cnt, N * 33, s);
    qk::IdMap tm = am;
    tm.keys = dup(mem, got, am.keys, (size_t)am.mask + 1, s);
    tm.vals = dup(mem, got, am.vals, (size_t)am.mask + 1, s);
    QK_HIP(hipStreamSynchronize(s));
    b = std::move(t);
    bm = tm;
  } catch (...) {
    for (void* p : got) mem.release(p);
    throw;
  }
}

void free_store(qk::DeviceMemory& mem, qk::Store& b, qk::IdMap& bm) {
  for (void* p : {(void*)b.centroids, (void*)b.d_off, (void*)b.d_size, (void*)b.d_cap, (void*)b.d_order,
                  (void*)b.v32, (void*)b.v16, (void*)b.v16n, (void*)b.rows32, (void*)b.ids, (void*)b.attr,
                  (void*)b.d_attr_cnt, (void*)b.codes, (void*)bm.keys, (void*)bm.vals})
    mem.release(p);
  b = qk::Store();
  bm = qk::IdMap();
}

template <class T>
T* pinned(size_t n) {
  void* p = nullptr;
  QK_HIP(hipHostMalloc(&p, std::max<size_t>(n, 1) * sizeof(T), hipHostMallocDefault));
  return static_cast<T*>(p);
}

}  // namespace

struct quake_server {
  quake_index* idx = nullptr;
  quake_search_params sp{};
  qk::Job job;
  int64_t cap = 0;
  int device = 0;
  hipStream_t s = nullptr;
  int chunk_tiles = 16;
  int64_t items = 0;
  int blocks = 0;

  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> fifo;
  std::unordered_map<uint64_t, Answer> answers;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string fatal;

  std::vector<uint64_t> slot_ticket;  // 0 = free
  std::vector<double> slot_arrive;
  std::vector<int32_t> free_slots;
  int64_t active = 0, max_active = 0, epochs = 0, rounds = 0, completed = 0;

  // overlapped updates: idx->L0 is the newest version (tag front), `other`
  // the previous one while its searches finish, then a copy that has
  // replayed every update
  bool overlap = false;
  bool have_twin = false;
  qk::Store other;
  qk::IdMap other_map;
  int front = 0;                        // tag of idx->L0; `other` has 1 - front
  std::vector<uint8_t> slot_tag;        // host mirror of d_tag
  uint8_t* d_tag = nullptr;             // [cap] store tag of every slot
  int64_t active_tag[2] = {0, 0};
  std::deque<Request> replay;           // updates `other` has yet to apply
  int64_t overlapped = 0;               // updates applied while searches ran
  // the update thread (overlap mode): it owns `other` while up_busy
  std::thread updater;
  hipStream_t s_up = nullptr;
  std::condition_variable cv_up;
  bool up_busy = false, up_ready = false, up_stop = false, up_fatal = false;
  bool up_replay_only = false;          // the job only brings `other` up to date (admission goes on)
  std::deque<Request> up_jobs;          // replays, then the new batch
  int up_rc = QUAKE_OK;
  std::string up_err;
  std::vector<double> lat;
  double first_arrive = -1, last_done = 0;

  // device staging for admission and answers
  float* d_x = nullptr;
  float* d_pad = nullptr;
  double* d_n2 = nullptr;
  float* d_scores = nullptr;
  int32_t* d_sel = nullptr;
  int32_t* d_cand = nullptr;
  float* d_h = nullptr;
  int32_t* d_mq = nullptr;
  int32_t* d_slots = nullptr;
  int64_t* d_ids = nullptr;
  float* d_dist = nullptr;
  int32_t* d_ns = nullptr;
  double* d_rec = nullptr;
  // pinned host mirrors
  float* h_x = nullptr;
  int32_t* h_slots = nullptr;
  int32_t* h_done = nullptr;
  int64_t* h_ids = nullptr;
  float* h_dist = nullptr;
  int32_t* h_ns = nullptr;
  double* h_rec = nullptr;

  const qk::Store& st() const { return idx->L0; }
  const qk::Store& store_of(int tag) const { return tag == front ? idx->L0 : other; }

  qk::RoundArgs args(int tag) const {
    const qk::Store& st = store_of(tag);
    qk::RoundArgs a{};
    a.nq = cap;
    a.M = job.M;
    a.k = job.k;
    a.kk = job.kk;
    a.aps = job.aps;
    a.chunk_tiles = chunk_tiles;
    a.wmax = job.wmax;
    a.wscale = idx->tune.window_scale > 0 ? idx->tune.window_scale : 100;
    a.slot_ids = job.batched && st.tiles * qk::TILE < (int64_t{1} << 31) ? 1 : 0;
    a.metric = idx->metric;
    a.dim = idx->d;
    a.tau_r = job.tau_r;
    a.tau_rho = job.tau_rho;
    a.est = job.est;
    a.items_cap = std::min<int64_t>(idx->ws.items_cap, items);
    a.blocks = blocks;
    a.hits = st.d_hits;
    if (overlap) {
      a.slot_tag = d_tag;
      a.tag = tag;
    }
    return a;
  }

  // Work-item bound of a round and the workspace for it: the larger of the
  // two versions' needs (partition sizes differ between them).
  void size_items() {
    chunk_tiles = idx->tune.chunk_tiles > 0 ? idx->tune.chunk_tiles : 16;
    // long result lists are scanned by sorting whole items in LDS
    if (job.kk > qk::KMAX) chunk_tiles = std::min(chunk_tiles, qk::SORTED_ITEM_MAX / qk::TILE);
    int64_t mc = qk::max_chunks(st(), chunk_tiles);
    if (have_twin) mc = std::max(mc, qk::max_chunks(other, chunk_tiles));
    items = std::max<int64_t>(cap * std::max(job.w0, 4) * 2, (int64_t)job.wmax * mc + 1);
    qk::ensure_queries(idx, cap);
    qk::ensure_workspace(idx, st().nlist, job.M, job.kk, items, job.batched ? cap * (int64_t)job.wmax : 0,
                         job.batched ? st().dp16 : 0, false);
  }

  // Size the search workspace for cap slots and mark every slot free.
  void setup() {
    size_items();
    QK_HIP(hipMemsetAsync(idx->ws.total, 0, qk::COUNTERS * sizeof(int64_t), s));
    qk::launch_mark_free(idx->ws, cap, s);
    blocks = qk::scan_blocks(idx, job.batched);
    QK_HIP(hipStreamSynchronize(s));
  }

  void admit(std::vector<Request>& reqs, const std::vector<int32_t>& slots) {
    const int64_t n = (int64_t)reqs.size();
    const int d = idx->d, dp = idx->dp;
    for (int64_t i = 0; i < n; ++i) {
      std::memcpy(h_x + i * d, reqs[i].x.data(), d * sizeof(float));
      h_slots[i] = slots[i];
    }
    QK_HIP(hipMemcpyAsync(d_x, h_x, n * d * sizeof(float), hipMemcpyHostToDevice, s));
    QK_HIP(hipMemcpyAsync(d_slots, h_slots, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    qk::Workspace& w = idx->ws;
    qk::launch_rows_to_slots(d_x, n, d, dp, d_slots, w.q, w.qn2, s);
    qk::launch_pad_rows(d_x, n, d, dp, d_pad, d_n2, s);
    qk::launch_scores(d_pad, n, st().centroids, st().nlist, dp, idx->metric, d_scores, s);
    qk::launch_fill_i32(d_mq, n, job.M, s);
    qk::launch_candidates(st(), d_pad, d_scores, n, dp, job.M, job.aps, idx->metric, d_mq, d_sel, d_cand, d_h, s);
    qk::launch_candidates_to_slots(d_cand, job.aps ? d_h : nullptr, n, job.M, d_slots, w.cand, w.h, w.mq, s);
    if (job.batched) qk::launch_queries16(w, n, dp, st().dp16, job.dtype16, s, d_slots);
    qk::launch_init_slots(w, d_slots, n, job.kk, job.w0, s);
    st().window += n;
    if (overlap) {
      for (int64_t i = 0; i < n; ++i) slot_tag[slots[i]] = (uint8_t)front;
      QK_HIP(hipMemcpyAsync(d_tag, slot_tag.data(), cap, hipMemcpyHostToDevice, s));
      active_tag[front] += n;
    }
  }

  // One scan round over all slots: plan, scan, commit.  No host round trip;
  // the harvest that follows reads which slots finished.
  void round() {
    qk::Workspace& w = idx->ws;
    for (int tag : {front, 1 - front}) {
      if (overlap ? active_tag[tag] == 0 : tag != front) continue;
      qk::RoundArgs a = args(tag);
      qk::launch_demand(w, store_of(tag), a, s);
      qk::run_rounds(idx, store_of(tag), job, a, 1, s);
    }
    ++rounds;
  }

  void harvest() {
    qk::Workspace& w = idx->ws;
    QK_HIP(hipMemcpyAsync(h_done, w.st_done, cap * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> fin;
    // finished slots grouped by store (the rerank reads the rows of the version the query scanned)
    for (int tag : {front, 1 - front}) {
      if (!overlap && tag != front) continue;  // one pass over the slots without tags
      for (int64_t q = 0; q < cap; ++q)
        if (slot_ticket[q] != 0 && h_done[q] && (!overlap || slot_tag[q] == tag)) fin.push_back((int32_t)q);
    }
    if (fin.empty()) return;
    const int64_t n = (int64_t)fin.size();
    QK_CHECK(n <= cap, QUAKE_E_DEVICE, "more finished slots than slots");  // the staging buffers hold cap
    std::memcpy(h_slots, fin.data(), n * sizeof(int32_t));
    QK_HIP(hipMemcpyAsync(d_slots, h_slots, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (job.batched) {
      int64_t at = 0;
      for (int tag : {front, 1 - front}) {
        int64_t cnt = 0;
        while (at + cnt < n && (!overlap || slot_tag[fin[at + cnt]] == tag)) ++cnt;
        if (cnt == 0) continue;
        qk::RoundArgs a = args(tag);
        qk::launch_rerank(w, store_of(tag), a, s, job.rerank != 0, d_slots + at, cnt);
        at += cnt;
      }
    }
    qk::launch_gather_results(w, d_slots, n, job.k, job.kk, idx->metric, d_ids, d_dist, d_ns, d_rec, s);
    const int k = job.k;
    QK_HIP(hipMemcpyAsync(h_ids, d_ids, n * k * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipMemcpyAsync(h_dist, d_dist, n * k * sizeof(float), hipMemcpyDeviceToHost, s));
    QK_HIP(hipMemcpyAsync(h_ns, d_ns, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    QK_HIP(hipStreamSynchronize(s));
    const double t = now_s();
    {
      std::lock_guard<std::mutex> lk(mu);
      for (int64_t i = 0; i < n; ++i) {
        const int32_t q = fin[i];
        Answer& an = answers[slot_ticket[q]];
        an.ids.assign(h_ids + i * k, h_ids + (i + 1) * k);
        an.dist.assign(h_dist + i * k, h_dist + (i + 1) * k);
        an.nscanned = h_ns[i];
        an.status = QUAKE_OK;
        an.ready = true;
        lat.push_back(t - slot_arrive[q]);
        slot_ticket[q] = 0;
        free_slots.push_back(q);
        --active;
        if (overlap) --active_tag[slot_tag[q]];
        ++completed;
      }
      last_done = t;
    }
    cv_done.notify_all();
  }

  // Applies an update batch to a store and its id map on stream `us`;
  // returns its status (the batch is rejected whole on error).
  int apply_to(qk::Store& st, qk::IdMap& map, const Request& r, hipStream_t us, std::string* err = nullptr) {
    const int64_t n = (int64_t)r.ids.size();
    if (n == 0) return QUAKE_OK;
    int64_t* d_i = nullptr;
    float* d_v = nullptr;
    int rc = QUAKE_OK;
    try {
      d_i = idx->mem.alloc<int64_t>(n);
      QK_HIP(hipMemcpyAsync(d_i, r.ids.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, us));
      if (r.kind == 1) {
        d_v = idx->mem.alloc<float>((size_t)n * idx->d);
        QK_HIP(hipMemcpyAsync(d_v, r.x.data(), (size_t)n * idx->d * sizeof(float), hipMemcpyHostToDevice, us));
        qk::insert_rows(idx, st, map, d_v, d_i, n, nullptr, us);
      } else {
        qk::delete_rows(idx, st, map, d_i, n, us);
      }
    } catch (const qk::Error& e) {
      rc = e.code;
      if (err) *err = e.msg;
    }
    QK_HIP(hipStreamSynchronize(us));
    idx->mem.release(d_i);
    idx->mem.release(d_v);
    return rc;
  }

  void answer_update(const Request& r, int rc) {
    {
      std::lock_guard<std::mutex> lk(mu);
      Answer& an = answers[r.ticket];
      an.status = rc;
      an.ready = true;
      ++epochs;
    }
    cv_done.notify_all();
  }

  // Drain mode: every slot is free when this runs.
  void apply_update(Request& r) {
    const int rc = apply_to(idx->L0, idx->idmap, r, s);
    setup();  // partition sizes changed: work-item bounds and buffers follow
    answer_update(r, rc);
  }

  // Overlap mode, on the update thread: `other` (no search reads it) takes
  // the batches the newer version took since, then the new one.  The first
  // time, `other` is made as a copy of the index's store (reading it while
  // searches read it too).
  void update_loop() {
    try {
      QK_HIP(hipSetDevice(device));
    } catch (...) {
    }
    while (true) {
      std::deque<Request> jobs;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_up.wait(lk, [&] { return up_stop || (up_busy && !up_ready); });
        if (!(up_busy && !up_ready)) break;
        jobs = up_jobs;
      }
      int rc = QUAKE_OK;
      std::string err;
      bool fatal_err = false;
      try {
        if (!have_twin) {
          clone_store(idx->mem, idx->L0, idx->idmap, other, other_map, s_up);
          other.d_hits = idx->L0.d_hits;
          have_twin = true;
        }
        const size_t replays = up_replay_only ? jobs.size() : jobs.size() - 1;
        for (size_t i = 0; i < replays; ++i) {
          const int prc = apply_to(other, other_map, jobs[i], s_up, &err);
          // a replay that fails (memory) would leave the versions different
          QK_CHECK(prc == QUAKE_OK, QUAKE_E_NOMEM, "the second store copy could not replay an update: " + err);
        }
        if (!up_replay_only) rc = apply_to(other, other_map, jobs.back(), s_up, &err);
      } catch (const qk::Error& e) {
        rc = e.code;
        err = e.msg;
        fatal_err = true;
      } catch (const std::exception& e) {
        rc = QUAKE_E_DEVICE;
        err = e.what();
        fatal_err = true;
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        up_rc = rc;
        up_err = err;
        up_fatal = fatal_err;
        up_ready = true;
      }
      cv_work.notify_all();
    }
  }

  // Overlap mode, on the search thread, once the update thread is done: on
  // success the two versions swap and new searches see the update.
  void finish_update() {
    Request r;
    int rc;
    bool only_replay;
    {
      std::lock_guard<std::mutex> lk(mu);
      QK_CHECK(!up_fatal, QUAKE_E_NOMEM, up_err);
      only_replay = up_replay_only;
      if (!only_replay) r = std::move(up_jobs.back());
      rc = up_rc;
      up_jobs.clear();
      up_busy = false;
      up_ready = false;
      up_replay_only = false;
    }
    replay.clear();
    if (only_replay) {  // `other` has caught up; nothing becomes visible
      qk::release_graphs(idx);
      size_items();
      return;
    }
    if (rc == QUAKE_OK) {
      std::swap(idx->L0, other);
      std::swap(idx->idmap, other_map);
      std::swap(idx->L0.window, other.window);  // the access window stays with the index
      front = 1 - front;
      replay.push_back(std::move(r));
    }
    // captured rounds key on the stores' arrays, which an update may
    // reallocate: the cache is dropped so that no replay reads a freed buffer
    qk::release_graphs(idx);
    size_items();  // partition sizes changed: work-item bounds and buffers follow
    if (rc == QUAKE_OK) answer_update(replay.back(), rc);
    else answer_update(r, rc);
  }

  void run() {
    try {
      QK_HIP(hipSetDevice(device));
      setup();
      while (true) {
        std::vector<Request> adm;
        std::vector<int32_t> slots;
        Request upd;
        bool has_upd = false;
        bool up_done = false;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv_work.wait(lk, [&] { return stop || !fifo.empty() || active > 0 || up_ready; });
          if (stop && fifo.empty() && active == 0 && !up_busy) break;
          up_done = up_ready;
          // while an update is being applied, later searches wait: they must see it
          const bool blocked = up_busy && !up_replay_only;
          while (!blocked && !fifo.empty() && fifo.front().kind == 0 && !free_slots.empty()) {
            const int32_t q = free_slots.back();
            free_slots.pop_back();
            slot_ticket[q] = fifo.front().ticket;
            slot_arrive[q] = fifo.front().arrive;
            slots.push_back(q);
            adm.push_back(std::move(fifo.front()));
            fifo.pop_front();
          }
          active += (int64_t)adm.size();
          max_active = std::max(max_active, active);
          // an update runs once nothing reads the version it will change:
          // the only version (drain mode) or the previous one (overlap mode,
          // where the update thread applies it beside the running searches)
          const bool ready = overlap ? (!up_busy && active_tag[1 - front] == 0) : active == 0;
          if (adm.empty() && ready && !fifo.empty() && fifo.front().kind != 0) {
            if (overlap) {
              up_jobs.assign(replay.begin(), replay.end());
              up_jobs.push_back(std::move(fifo.front()));
              fifo.pop_front();
              up_busy = true;
              if (active > 0) ++overlapped;
              cv_up.notify_one();
            } else {
              upd = std::move(fifo.front());
              fifo.pop_front();
              has_upd = true;
            }
          } else if (overlap && !up_busy && !replay.empty() && active_tag[1 - front] == 0) {
            // the previous version's searches are done: bring it up to date
            // now, beside the searches, so that the next update only waits
            // for its own batch
            up_jobs.assign(replay.begin(), replay.end());
            up_busy = true;
            up_replay_only = true;
            cv_up.notify_one();
          }
        }
        if (up_done) finish_update();
        if (has_upd) {
          apply_update(upd);
          continue;
        }
        if (!adm.empty()) admit(adm, slots);
        if (active > 0) {
          round();
          harvest();
        }
      }
    } catch (const qk::Error& e) {
      fail(e.msg);
    } catch (const std::exception& e) {
      fail(e.what());
    }
  }

  void fail(const std::string& msg) {
    std::lock_guard<std::mutex> lk(mu);
    fatal = msg.empty() ? "serving loop failed" : msg;
    for (auto& kv : answers)
      if (!kv.second.ready) {
        kv.second.ready = true;
        kv.second.status = QUAKE_E_DEVICE;
      }
    cv_done.notify_all();
  }

  uint64_t enqueue(std::vector<Request>& reqs) {
    std::lock_guard<std::mutex> lk(mu);
    QK_CHECK(fatal.empty(), QUAKE_E_STATE, "the serving loop stopped: " + fatal);
    QK_CHECK(!stop, QUAKE_E_STATE, "the server is stopping");
    const uint64_t first = next_ticket;
    const double t = now_s();
    if (first_arrive < 0) first_arrive = t;
    for (auto& r : reqs) {
      r.ticket = next_ticket++;
      r.arrive = t;
      answers.emplace(r.ticket, Answer{});
      fifo.push_back(std::move(r));
    }
    cv_work.notify_one();
    return first;
  }

  void release_buffers() {
    for (void* p : {(void*)d_x, (void*)d_pad, (void*)d_n2, (void*)d_scores, (void*)d_sel, (void*)d_cand, (void*)d_h,
                    (void*)d_mq, (void*)d_slots, (void*)d_ids, (void*)d_dist, (void*)d_ns, (void*)d_rec,
                    (void*)d_tag})
      idx->mem.release(p);
    if (have_twin) {
      // idx->L0 is the newest version; the older copy goes
      qk::release_graphs(idx);
      other.d_hits = nullptr;
      free_store(idx->mem, other, other_map);
      have_twin = false;
    }
    for (void* p : {(void*)h_x, (void*)h_slots, (void*)h_done, (void*)h_ids, (void*)h_dist, (void*)h_ns,
                    (void*)h_rec})
      if (p) (void)hipHostFree(p);
    if (s) (void)hipStreamDestroy(s);
    if (s_up) (void)hipStreamDestroy(s_up);
  }
};

namespace {

int fail_rc(int code, const std::string& msg) { return qk::set_error(code, msg); }

bool all_finite(const float* v, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

#define SRV_BEGIN try {
#define SRV_END                                                                            \
  }                                                                                        \
  catch (const qk::Error& e) { return fail_rc(e.code, e.msg); }                            \
  catch (const std::bad_alloc&) { return fail_rc(QUAKE_E_NOMEM, "host allocation failed"); } \
  catch (const std::exception& e) { return fail_rc(QUAKE_E_DEVICE, e.what()); }            \
  return QUAKE_OK;

// Device bytes one slot of in-flight work needs (workspace rows, its work
// items and partial lists, staging).
int64_t slot_bytes(const quake_index* idx, const qk::Job& job) {
  const int64_t N = idx->L0.nlist, dp = idx->dp, d = idx->d;
  int64_t b = dp * 4 + 8 + N * 4 * 2 + (int64_t)job.M * 12 * 2 + (int64_t)job.kk * 12 + 96;
  b += (int64_t)std::max(job.w0, 4) * 2 * (16 + (int64_t)job.kk * 12);
  if (job.batched) b += (int64_t)job.wmax * 20 + idx->L0.dp16 * 2 + 4;
  b += d * 4 + dp * 4 + 8 + (int64_t)job.k * 12 + 16;
  return b;
}

}  // namespace

extern "C" {

int quake_server_create(quake_index* idx, const quake_server_params* params, quake_server** out) {
  SRV_BEGIN
  QK_CHECK(out && params, QUAKE_E_INVALID, "params and out are required");
  *out = nullptr;
  QK_CHECK(idx && idx->magic == 0x51554b45u, QUAKE_E_STATE, "invalid index handle");
  QK_CHECK(idx->n_levels == 1, QUAKE_E_INVALID, "the serving loop runs on single-level indexes");
  QK_CHECK(params->max_slots >= 0, QUAKE_E_INVALID, "max_slots must be >= 0");
  QK_CHECK(!params->search.filter, QUAKE_E_INVALID, "the serving loop takes no filter (requests carry no masks)");
  QK_CHECK(params->search.scan_dtype != QUAKE_PQ8, QUAKE_E_INVALID, "the serving loop does not scan product codes");
  QK_CHECK(params->overlap_updates == 0 || params->overlap_updates == 1, QUAKE_E_INVALID,
           "overlap_updates must be 0 or 1");
  std::unique_ptr<quake_server> srv(new quake_server());
  srv->idx = idx;
  srv->overlap = params->overlap_updates != 0;
  srv->sp = params->search;
  srv->job = qk::resolve(idx, idx->L0, &srv->sp);
  int64_t cap = params->max_slots > 0 ? params->max_slots : 4096;
  if (params->hbm_budget_bytes > 0) {
    const int64_t by_budget = (int64_t)(params->hbm_budget_bytes / (size_t)slot_bytes(idx, srv->job));
    QK_CHECK(by_budget >= 1, QUAKE_E_NOMEM, "the HBM budget does not hold one search slot");
    cap = params->max_slots > 0 ? std::min<int64_t>(cap, by_budget) : std::min<int64_t>(by_budget, 1 << 16);
  }
  srv->cap = cap;
  QK_HIP(hipGetDevice(&srv->device));
  QK_HIP(hipStreamCreateWithFlags(&srv->s, hipStreamNonBlocking));
  auto& mem = idx->mem;
  const int64_t N = idx->L0.nlist, M = srv->job.M, k = srv->job.k;
  try {
    srv->d_x = mem.alloc<float>(cap * idx->d);
    srv->d_pad = mem.alloc<float>(cap * idx->dp);
    srv->d_n2 = mem.alloc<double>(cap);
    srv->d_scores = mem.alloc<float>(cap * N);
    srv->d_sel = mem.alloc<int32_t>(cap * M);
    srv->d_cand = mem.alloc<int32_t>(cap * M);
    srv->d_h = mem.alloc<float>(cap * M);
    srv->d_mq = mem.alloc<int32_t>(cap);
    srv->d_slots = mem.alloc<int32_t>(cap);
    srv->d_ids = mem.alloc<int64_t>(cap * k);
    srv->d_dist = mem.alloc<float>(cap * k);
    srv->d_ns = mem.alloc<int32_t>(cap);
    srv->d_rec = mem.alloc<double>(cap);
    if (srv->overlap) {
      srv->d_tag = mem.alloc<uint8_t>(cap);
      srv->slot_tag.assign(cap, 0);
      QK_HIP(hipMemcpy(srv->d_tag, srv->slot_tag.data(), cap, hipMemcpyHostToDevice));
    }
    srv->h_x = pinned<float>(cap * idx->d);
    srv->h_slots = pinned<int32_t>(cap);
    srv->h_done = pinned<int32_t>(cap);
    srv->h_ids = pinned<int64_t>(cap * k);
    srv->h_dist = pinned<float>(cap * k);
    srv->h_ns = pinned<int32_t>(cap);
    srv->h_rec = pinned<double>(cap);
  } catch (...) {
    srv->release_buffers();
    throw;
  }
  srv->slot_ticket.assign(cap, 0);
  srv->slot_arrive.assign(cap, 0.0);
  for (int64_t q = cap - 1; q >= 0; --q) srv->free_slots.push_back((int32_t)q);
  if (srv->overlap) QK_HIP(hipStreamCreateWithFlags(&srv->s_up, hipStreamNonBlocking));
  quake_server* raw = srv.get();
  srv->worker = std::thread([raw] { raw->run(); });
  if (srv->overlap) srv->updater = std::thread([raw] { raw->update_loop(); });
  *out = srv.release();
  SRV_END
}

int quake_server_search(quake_server* srv, const float* q, int64_t n, uint64_t* first_ticket) {
  SRV_BEGIN
  QK_CHECK(srv && (n == 0 || q) && n >= 0, QUAKE_E_INVALID, "bad arguments");
  const int d = srv->idx->d;
  QK_CHECK(all_finite(q, n * d), QUAKE_E_INVALID, "q holds a non-finite value");
  std::vector<Request> reqs(n);
  for (int64_t i = 0; i < n; ++i) {
    reqs[i].kind = 0;
    reqs[i].x.assign(q + i * d, q + (i + 1) * d);
  }
  const uint64_t t = srv->enqueue(reqs);
  if (first_ticket) *first_ticket = t;
  SRV_END
}

int quake_server_insert(quake_server* srv, const float* x, const int64_t* ids, int64_t n, uint64_t* ticket) {
  SRV_BEGIN
  QK_CHECK(srv && n >= 0 && (n == 0 || (x && ids)), QUAKE_E_INVALID, "bad arguments");
  QK_CHECK(all_finite(x, n * srv->idx->d), QUAKE_E_INVALID, "x holds a non-finite value");
  std::vector<Request> r(1);
  r[0].kind = 1;
  r[0].x.assign(x, x + n * srv->idx->d);
  r[0].ids.assign(ids, ids + n);
  const uint64_t t = srv->enqueue(r);
  if (ticket) *ticket = t;
  SRV_END
}

int quake_server_delete(quake_server* srv, const int64_t* ids, int64_t n, uint64_t* ticket) {
  SRV_BEGIN
  QK_CHECK(srv && n >= 0 && (n == 0 || ids), QUAKE_E_INVALID, "bad arguments");
  std::vector<Request> r(1);
  r[0].kind = 2;
  r[0].ids.assign(ids, ids + n);
  const uint64_t t = srv->enqueue(r);
  if (ticket) *ticket = t;
  SRV_END
}

int quake_server_wait(quake_server* srv, uint64_t ticket, double timeout_s, int64_t* ids, float* dist,
                      int32_t* nscanned, int32_t* status) {
  SRV_BEGIN
  QK_CHECK(srv, QUAKE_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->answers.find(ticket);
  QK_CHECK(it != srv->answers.end(), QUAKE_E_INVALID, "unknown or already collected ticket");
  auto ready = [&] { return srv->answers[ticket].ready; };
  if (timeout_s < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return fail_rc(QUAKE_E_STATE, "timed out");
  }
  Answer an = std::move(srv->answers[ticket]);
  srv->answers.erase(ticket);
  lk.unlock();
  if (status) *status = an.status;
  if (nscanned) *nscanned = an.nscanned;
  if (ids && !an.ids.empty()) std::memcpy(ids, an.ids.data(), an.ids.size() * sizeof(int64_t));
  if (dist && !an.dist.empty()) std::memcpy(dist, an.dist.data(), an.dist.size() * sizeof(float));
  SRV_END
}

int quake_server_stats(quake_server* srv, quake_server_report* out, int32_t reset) {
  SRV_BEGIN
  QK_CHECK(srv && out, QUAKE_E_INVALID, "bad arguments");
  std::lock_guard<std::mutex> lk(srv->mu);
  std::memset(out, 0, sizeof(*out));
  out->completed = srv->completed;
  out->queued = (int64_t)srv->fifo.size();
  out->in_flight = srv->active;
  out->slots = srv->cap;
  out->max_in_flight = srv->max_active;
  out->epochs = srv->epochs;
  out->rounds = srv->rounds;
  out->overlapped_updates = srv->overlapped;
  if (!srv->lat.empty()) {
    std::vector<double> l(srv->lat);
    std::sort(l.begin(), l.end());
    auto pct = [&](double f) { return l[std::min<size_t>(l.size() - 1, (size_t)(f * (l.size() - 1) + 0.5))]; };
    out->p50_latency_s = pct(0.50);
    out->p99_latency_s = pct(0.99);
    double sum = 0;
    for (double v : l) sum += v;
    out->mean_latency_s = sum / l.size();
    if (srv->last_done > srv->first_arrive) out->qps = srv->completed / (srv->last_done - srv->first_arrive);
  }
  if (reset) {
    srv->lat.clear();
    srv->completed = 0;
    srv->max_active = srv->active;
    srv->rounds = 0;
    srv->first_arrive = -1;
  }
  SRV_END
}

void quake_server_destroy(quake_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->up_stop = true;
  }
  srv->cv_up.notify_all();
  if (srv->updater.joinable()) srv->updater.join();
  srv->release_buffers();
  delete srv;
}

}  // extern "C"

// Continuous-batching query server over a device-resident index.
//
// A dispatcher thread owns `kContexts` iteration contexts, each with its own
// HIP stream, device tables and pinned host buffers, all allocated when the
// server is created (nothing is allocated while serving).  Each turn of its
// loop it
//   1. retires contexts whose iteration has finished on the device (an event
//      query, never a wait), handing results to the completed queue and
//      releasing their memory reservation;
//   2. admits waiting queries, oldest first, into a free context while the
//      context's slot count, chunk memory (the output-to-input bound: at
//      most 128 survivors per 128-value chunk of the shortest list) and
//      result memory (at most the shortest list's length) all fit;
//   3. launches the admitted queries as one batch (persistent decode-fused
//      chunk kernel + scan + compaction) on that context's stream.
// Queries that arrive while earlier ones run on the device are admitted into
// the next free context and launched at once, so iterations overlap on the
// device.  Per-query counts and offsets are written by the device straight
// into pinned, device-mapped host memory; the results themselves are copied
// back with one asynchronous copy of exactly their total size.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "s4_internal.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int kContexts = 3;

struct Query {
  uint64_t id = 0;
  std::vector<uint32_t> terms;  // sorted shortest first
  uint64_t items = 0, bound = 0;
  Clock::time_point submitted;
};

struct Done {
  uint64_t id, count, latency_ns;
  std::vector<uint32_t> result;
};

struct Context {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void *dmem = nullptr;
  s4::BatchDev dev{};
  // pinned host: tables (uploaded) and outputs (written by the device)
  uint32_t *h_sterms = nullptr, *h_qoff = nullptr, *h_ib = nullptr, *h_iq = nullptr;
  uint32_t *h_results = nullptr;  // pinned, results_per_ctx values
  uint64_t *h_counts = nullptr, *h_offs = nullptr;  // pinned, device-mapped
  uint32_t *d_results = nullptr;  // device, one value per staged slot
  uint64_t *d_counts = nullptr, *d_offs = nullptr;  // device views of h_counts / h_offs
  std::vector<Query> queries;
  bool busy = false;
  int phase = 0;  // 1: kernels running, 2: results copy running
  uint64_t reserved_stage = 0;
};

}  // namespace

struct s4_server {
  const s4_index *index = nullptr;
  s4_server_config cfg{};
  uint64_t slots_per_ctx = 0, items_per_ctx = 0, results_per_ctx = 0, terms_per_ctx = 0;
  Context ctx[kContexts];
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Query> waiting;
  std::deque<Done> completed;
  std::deque<Clock::time_point> completed_at;
  std::atomic<bool> stop{false};
  std::thread worker;
  int device = 0;
  uint64_t next_id = 1;
  s4_server_stats st{};
  uint64_t active = 0, pool_in_use = 0;
  int worker_error = 0;
  std::string worker_msg;
};

namespace {

int alloc_context(s4_server *s, Context &c) {
  S4_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
  S4_HIP(hipEventCreateWithFlags(&c.done, hipEventDisableTiming));
  const uint64_t nq = s->slots_per_ctx, items = s->items_per_ctx, nt = s->terms_per_ctx;
  const uint32_t ntiles = uint32_t((items + 1023) / 1024);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = s4::align_up(off + std::max<size_t>(bytes, 4), 256);
    return o;
  };
  const size_t o_sterms = take(4 * nt), o_qoff = take(4 * (nq + 1)), o_ib = take(4 * (nq + 1)),
               o_iq = take(16 * items), o_stage = take(4 * s4::kBlock * items), o_counts = take(4 * items),
               o_excl = take(4 * items), o_tiles = take(4 * (ntiles + 1)), o_ctrl = take(64),
               o_qtick = take(8 * nq), o_res = take(4 * s4::kBlock * items);
  if (hipMalloc(&c.dmem, off) != hipSuccess) return s4::fail(S4_ENOMEM, "server context: device allocation failed");
  char *m = static_cast<char *>(c.dmem);
  s4::BatchDev &d = c.dev;
  d.lists = s->index->d_lists;
  d.sterms = reinterpret_cast<const uint32_t *>(m + o_sterms);
  d.qoff = reinterpret_cast<const uint32_t *>(m + o_qoff);
  d.item_base = reinterpret_cast<const uint32_t *>(m + o_ib);
  d.item_info = reinterpret_cast<const uint4 *>(m + o_iq);
  d.stage = reinterpret_cast<uint32_t *>(m + o_stage);
  d.counts = reinterpret_cast<uint32_t *>(m + o_counts);
  d.excl = reinterpret_cast<uint32_t *>(m + o_excl);
  d.tiles = reinterpret_cast<uint32_t *>(m + o_tiles);
  d.head = reinterpret_cast<uint32_t *>(m + o_ctrl);
  d.total = reinterpret_cast<uint64_t *>(m + o_ctrl + 8);
  d.start = reinterpret_cast<uint64_t *>(m + o_ctrl + 16);
  d.qtick = reinterpret_cast<uint64_t *>(m + o_qtick);
  d.stats = reinterpret_cast<uint64_t *>(m + o_ctrl + 24);
  c.d_results = reinterpret_cast<uint32_t *>(m + o_res);
  auto hmalloc = [&](void **p, size_t bytes, unsigned flags) {
    return hipHostMalloc(p, std::max<size_t>(bytes, 64), flags) == hipSuccess;
  };
  bool ok = hmalloc(reinterpret_cast<void **>(&c.h_sterms), 4 * nt, hipHostMallocDefault) &&
            hmalloc(reinterpret_cast<void **>(&c.h_qoff), 4 * (nq + 1), hipHostMallocDefault) &&
            hmalloc(reinterpret_cast<void **>(&c.h_ib), 4 * (nq + 1), hipHostMallocDefault) &&
            hmalloc(reinterpret_cast<void **>(&c.h_iq), 16 * items, hipHostMallocDefault) &&
            hmalloc(reinterpret_cast<void **>(&c.h_results), 4 * s->results_per_ctx, hipHostMallocDefault) &&
            hmalloc(reinterpret_cast<void **>(&c.h_counts), 8 * nq, hipHostMallocMapped) &&
            hmalloc(reinterpret_cast<void **>(&c.h_offs), 8 * (nq + 1), hipHostMallocMapped);
  if (!ok) return s4::fail(S4_ENOMEM, "server context: pinned host allocation failed");
  S4_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&c.d_counts), c.h_counts, 0));
  S4_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&c.d_offs), c.h_offs, 0));
  return S4_OK;
}

void free_context(Context &c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (c.dmem) (void)hipFree(c.dmem);
  for (void *p : {static_cast<void *>(c.h_sterms), static_cast<void *>(c.h_qoff), static_cast<void *>(c.h_ib),
                  static_cast<void *>(c.h_iq), static_cast<void *>(c.h_results), static_cast<void *>(c.h_counts),
                  static_cast<void *>(c.h_offs)})
    if (p) (void)hipHostFree(p);
  if (c.done) (void)hipEventDestroy(c.done);
  if (c.stream) (void)hipStreamDestroy(c.stream);
  c = Context{};
}

// Launch the queries gathered in c (caller holds no lock; c is private to
// the dispatcher while busy).
int launch_context(s4_server *s, Context &c) {
  uint64_t nt = 0, items = 0;
  const uint64_t nq = c.queries.size();
  for (uint64_t q = 0; q < nq; ++q) {
    const Query &qq = c.queries[q];
    c.h_qoff[q] = uint32_t(nt);
    c.h_ib[q] = uint32_t(items);
    for (uint32_t t : qq.terms) c.h_sterms[nt++] = t;
    for (uint64_t i = 0; i < qq.items; ++i) {
      uint32_t *rec = c.h_iq + 4 * (items + i);
      rec[0] = uint32_t(q);
      rec[1] = uint32_t(i);
      rec[2] = c.h_qoff[q];
      rec[3] = uint32_t(qq.terms.size());
    }
    items += qq.items;
  }
  c.h_qoff[nq] = uint32_t(nt);
  c.h_ib[nq] = uint32_t(items);
  s4::BatchDev d = c.dev;
  d.items = uint32_t(items);
  d.nq = uint32_t(nq);
  d.ntiles = uint32_t((items + 1023) / 1024);
  S4_HIP(hipMemcpyAsync(const_cast<uint32_t *>(d.sterms), c.h_sterms, 4 * std::max<uint64_t>(nt, 1),
                        hipMemcpyHostToDevice, c.stream));
  S4_HIP(hipMemcpyAsync(const_cast<uint32_t *>(d.qoff), c.h_qoff, 4 * (nq + 1), hipMemcpyHostToDevice, c.stream));
  S4_HIP(hipMemcpyAsync(const_cast<uint32_t *>(d.item_base), c.h_ib, 4 * (nq + 1), hipMemcpyHostToDevice, c.stream));
  if (items)
    S4_HIP(hipMemcpyAsync(const_cast<uint4 *>(d.item_info), c.h_iq, 16 * items, hipMemcpyHostToDevice, c.stream));
  int rc = s4::enqueue_batch_dev(d, c.d_counts, c.d_offs, c.d_results, c.stream);
  if (rc) return rc;
  S4_HIP(hipEventRecord(c.done, c.stream));
  c.busy = true;
  c.phase = 1;
  return S4_OK;
}

// Kernels done: copy exactly the results back (asynchronously when they
// fit the pinned buffer).  Returns true when the context can retire now.
bool start_copy(s4_server *s, Context &c, std::vector<uint32_t> *spill) {
  const uint64_t total = c.h_offs[c.queries.size()];
  if (total == 0) return true;
  if (total <= s->results_per_ctx) {
    if (hipMemcpyAsync(c.h_results, c.d_results, 4 * total, hipMemcpyDeviceToHost, c.stream) == hipSuccess &&
        hipEventRecord(c.done, c.stream) == hipSuccess) {
      c.phase = 2;
      return false;
    }
  }
  spill->resize(total);
  (void)hipMemcpy(spill->data(), c.d_results, 4 * total, hipMemcpyDeviceToHost);
  return true;
}

// Move a finished context's results to the completed queue.
void retire_context(s4_server *s, Context &c, const uint32_t *res) {
  const auto now = Clock::now();
  std::vector<Done> out;
  out.reserve(c.queries.size());
  for (size_t q = 0; q < c.queries.size(); ++q) {
    const uint64_t o0 = c.h_offs[q], cnt = c.h_counts[q];
    Done d;
    d.id = c.queries[q].id;
    d.count = cnt;
    d.latency_ns = uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(now - c.queries[q].submitted).count());
    d.result.assign(res + o0, res + o0 + cnt);
    out.push_back(std::move(d));
  }
  std::lock_guard<std::mutex> lock(s->mu);
  for (auto &d : out) {
    s->completed.push_back(std::move(d));
    s->completed_at.push_back(now);
  }
  s->st.completed += out.size();
  s->active -= c.queries.size();
  s->pool_in_use -= c.reserved_stage;
  c.queries.clear();
  c.reserved_stage = 0;
  c.busy = false;
  c.phase = 0;
}

void dispatcher(s4_server *s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool progressed = false;
    for (Context &c : s->ctx) {
      if (c.busy && hipEventQuery(c.done) == hipSuccess) {
        if (c.phase == 1) {
          std::vector<uint32_t> spill;
          if (start_copy(s, c, &spill)) retire_context(s, c, spill.empty() ? c.h_results : spill.data());
        } else {
          retire_context(s, c, c.h_results);
        }
        progressed = true;
      }
    }
    Context *free_ctx = nullptr;
    for (Context &c : s->ctx)
      if (!c.busy) {
        free_ctx = &c;
        break;
      }
    bool launched = false;
    if (free_ctx) {
      Context &c = *free_ctx;
      {
        std::unique_lock<std::mutex> lock(s->mu);
        uint64_t items = 0, terms = 0;
        while (!s->waiting.empty() && c.queries.size() < s->slots_per_ctx) {
          const Query &q = s->waiting.front();
          const bool fits = items + q.items <= s->items_per_ctx && terms + q.terms.size() <= s->terms_per_ctx &&
                            s->pool_in_use + 4 * s4::kBlock * (items + q.items) <= s->cfg.pool_bytes;
          if (!fits) {
            if (c.queries.empty()) ++s->st.waits_for_memory;
            break;
          }
          items += q.items;
          terms += q.terms.size();
          c.queries.push_back(std::move(s->waiting.front()));
          s->waiting.pop_front();
        }
        if (!c.queries.empty()) {
          c.reserved_stage = 4 * s4::kBlock * items;
          s->pool_in_use += c.reserved_stage;
          s->active += c.queries.size();
          s->st.admitted += c.queries.size();
          s->st.peak_active = std::max(s->st.peak_active, s->active);
          s->st.peak_pool_bytes = std::max(s->st.peak_pool_bytes, s->pool_in_use);
          ++s->st.iterations;
        }
      }
      if (!c.queries.empty()) {
        int rc = launch_context(s, c);
        if (rc) {
          std::lock_guard<std::mutex> lock(s->mu);
          s->worker_error = rc;
          s->worker_msg = s4_last_error();
          s->stop = true;
        }
        launched = true;
      }
    }
    bool idle = false;
    {
      std::unique_lock<std::mutex> lock(s->mu);
      bool any_busy = false;
      for (Context &c : s->ctx) any_busy |= c.busy;
      if (s->stop && !any_busy && (s->waiting.empty() || s->worker_error)) break;
      idle = !progressed && !launched;
      if (idle && !any_busy && s->waiting.empty())
        s->cv.wait_for(lock, std::chrono::milliseconds(1));
    }
    if (idle) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

}  // namespace

using namespace s4;

extern "C" {

int s4_server_create(const s4_index *index, const s4_server_config *cfg, s4_server **out) {
  if (!index || !cfg || !out) return fail(S4_EINVAL, "null argument");
  if (!cfg->max_slots || !cfg->pool_bytes || !cfg->max_terms || cfg->max_terms > kMaxTerms + 1)
    return fail(S4_EINVAL, "server config: need max_slots, pool_bytes > 0 and 1 <= max_terms <= 33");
  int rc = ensure_device();
  if (rc) return rc;
  s4_server *s = new (std::nothrow) s4_server;
  if (!s) return fail(S4_ENOMEM, "handle allocation failed");
  s->index = index;
  s->cfg = *cfg;
  (void)hipGetDevice(&s->device);
  s->slots_per_ctx = std::max<uint64_t>(1, cfg->max_slots / kContexts);
  s->items_per_ctx = std::max<uint64_t>(1, cfg->pool_bytes / kContexts / (4 * kBlock));
  const uint64_t rb = cfg->result_bytes ? cfg->result_bytes : (64ull << 20);
  s->results_per_ctx = std::max<uint64_t>(kBlock, rb / kContexts / 4);
  s->terms_per_ctx = s->slots_per_ctx * cfg->max_terms;
  if (s->items_per_ctx >= 0xFFFFFFFFull / kBlock) {
    delete s;
    return fail(S4_EINVAL, "pool_bytes too large");
  }
  for (Context &c : s->ctx) {
    rc = alloc_context(s, c);
    if (rc) {
      for (Context &d : s->ctx) free_context(d);
      delete s;
      return rc;
    }
  }
  s->worker = std::thread(dispatcher, s);
  *out = s;
  return S4_OK;
}

int s4_server_submit(s4_server *s, const uint32_t *terms, uint32_t k, uint64_t *id) {
  if (!s || !terms || !id) return fail(S4_EINVAL, "null argument");
  if (k == 0 || k > s->cfg.max_terms) return fail(S4_EINVAL, "query must have 1..max_terms terms");
  Query q;
  q.terms.assign(terms, terms + k);
  for (uint32_t t : q.terms) {
    if (t >= s->index->count) return fail(S4_EINVAL, "term out of range");
    if (k > 1 && !(s->index->flags[t] & 1u)) return fail(S4_EUNSORTED, "list is not strictly increasing");
  }
  std::stable_sort(q.terms.begin(), q.terms.end(),
                   [&](uint32_t x, uint32_t y) { return s->index->lengths[x] < s->index->lengths[y]; });
  const uint64_t m = s->index->lengths[q.terms[0]];
  q.items = (m + kBlock - 1) / kBlock;
  q.bound = m;
  std::lock_guard<std::mutex> lock(s->mu);
  if (s->stop) return fail(S4_EINVAL, "server is stopping");
  if (s->worker_error) return fail(s->worker_error, "server failed: " + s->worker_msg);
  if (q.items > s->items_per_ctx || q.terms.size() > s->terms_per_ctx ||
      4 * kBlock * q.items > s->cfg.pool_bytes) {
    ++s->st.rejected;
    return fail(S4_ERANGE, "query needs more intermediate memory than one iteration holds");
  }
  if (s->waiting.size() >= 64ull * s->cfg.max_slots) return fail(S4_EAGAIN, "waiting queue full");
  q.id = s->next_id++;
  q.submitted = Clock::now();
  *id = q.id;
  s->waiting.push_back(std::move(q));
  ++s->st.submitted;
  s->cv.notify_one();
  return S4_OK;
}

int s4_server_poll(s4_server *s, uint64_t *ids, uint64_t *counts, uint64_t *latency_ns, uint32_t *results,
                   uint64_t results_cap, uint64_t *res_offsets, uint32_t max_done, uint32_t *done) {
  if (!s || !done || (max_done && (!ids || !counts || !latency_ns || !res_offsets)))
    return fail(S4_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(s->mu);
  uint32_t n = 0;
  uint64_t used = 0;
  res_offsets[0] = 0;
  while (n < max_done && !s->completed.empty()) {
    Done &d = s->completed.front();
    if (used + d.count > results_cap || (d.count && !results)) break;
    std::copy(d.result.begin(), d.result.end(), results + used);
    ids[n] = d.id;
    counts[n] = d.count;
    latency_ns[n] = d.latency_ns;
    used += d.count;
    res_offsets[n + 1] = used;
    s->completed.pop_front();
    s->completed_at.pop_front();
    ++n;
  }
  *done = n;
  if (s->worker_error && n == 0) return fail(s->worker_error, "server failed: " + s->worker_msg);
  return S4_OK;
}

int s4_server_stats_get(const s4_server *s, s4_server_stats *st) {
  if (!s || !st) return fail(S4_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(const_cast<s4_server *>(s)->mu);
  *st = s->st;
  return S4_OK;
}

int s4_server_replay(s4_server *s, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                     const uint64_t *h_arrival_ns, uint64_t *latency_ns, uint64_t *counts, uint32_t *results,
                     uint64_t results_cap, uint64_t *res_offsets, double timeout_s, double *elapsed_s) {
  if (!s || !h_q_offsets || !h_arrival_ns || !latency_ns || !counts || (nq && !h_terms))
    return fail(S4_EINVAL, "null argument");
  if (results && !res_offsets) return fail(S4_EINVAL, "results need res_offsets");
  std::vector<std::vector<uint32_t>> res(results ? nq : 0);
  uint64_t ndone = 0, next = 0;
  std::unordered_map<uint64_t, uint64_t> pending;
  const auto t0 = Clock::now();
  auto now_ns = [&]() { return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count()); };
  uint64_t last_done_ns = 0;
  while (ndone < nq) {
    const uint64_t t = now_ns();
    // submit everything due
    while (next < nq && h_arrival_ns[next] <= t) {
      const uint64_t a = h_q_offsets[next], b = h_q_offsets[next + 1];
      uint64_t id = 0;
      int rc = s4_server_submit(s, h_terms + a, uint32_t(b - a), &id);
      if (rc == S4_EAGAIN) break;
      if (rc) return rc;
      pending.emplace(id, next);
      ++next;
    }
    // drain completions
    {
      std::lock_guard<std::mutex> lock(s->mu);
      while (!s->completed.empty()) {
        Done &d = s->completed.front();
        auto it = pending.find(d.id);
        if (it != pending.end()) {
          const uint64_t q = it->second;
          const uint64_t fin = uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                            s->completed_at.front() - t0).count());
          latency_ns[q] = fin > h_arrival_ns[q] ? fin - h_arrival_ns[q] : 0;
          last_done_ns = std::max(last_done_ns, fin);
          counts[q] = d.count;
          if (results) res[q] = std::move(d.result);
          ++ndone;
          pending.erase(it);
        }
        s->completed.pop_front();
        s->completed_at.pop_front();
      }
      if (s->worker_error) return fail(s->worker_error, "server failed: " + s->worker_msg);
    }
    if (double(now_ns()) * 1e-9 > timeout_s) return fail(S4_ERANGE, "replay timed out");
    if (next < nq && h_arrival_ns[next] > now_ns() + 50000)
      std::this_thread::sleep_for(std::chrono::microseconds(10));
  }
  if (elapsed_s) *elapsed_s = double(last_done_ns - (nq ? h_arrival_ns[0] : 0)) * 1e-9;
  if (results) {
    uint64_t used = 0;
    res_offsets[0] = 0;
    for (uint64_t q = 0; q < nq; ++q) {
      if (used + res[q].size() > results_cap) return fail(S4_ERANGE, "results_cap too small");
      std::copy(res[q].begin(), res[q].end(), results + used);
      used += res[q].size();
      res_offsets[q + 1] = used;
    }
  }
  return S4_OK;
}

int s4_server_destroy(s4_server *s) {
  if (!s) return S4_OK;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
    s->cv.notify_one();
  }
  if (s->worker.joinable()) s->worker.join();
  for (Context &c : s->ctx) free_context(c);
  const int err = s->worker_error;
  delete s;
  return err ? fail(err, "server stopped after an error") : S4_OK;
}

}  // extern "C"

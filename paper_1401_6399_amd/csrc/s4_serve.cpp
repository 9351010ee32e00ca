// Continuous-batching query server over a device-resident index.
//
// A dispatcher thread owns `kContexts` iteration contexts, each with its own
// HIP stream, device tables and pinned host buffers, all allocated when the
// server is created (nothing is allocated on the device while serving).
// Each turn of its loop it
//   1. retires contexts whose iteration has finished on the device (an event
//      query, never a wait), handing the iteration's finished queries to the
//      completed queue as one batch (their results copied once) and
//      releasing their memory reservation;
//   2. fills a free context: first one slice of every query already running
//      in slices (unless every other context already runs such slices, so
//      one context always stays free for short queries), then waiting
//      queries, oldest first, while the context's
//      slot count, chunk memory (the output-to-input bound: at most 128
//      survivors per 128-value chunk of the shortest list), result memory
//      (at most the shortest list's length per query) and the iteration's
//      chunk budget all fit.  A query of more than `slice` chunks is run a
//      slice of its chunks per iteration (intersection distributes over a
//      partition of the shortest list) so that it never holds the device
//      for long while small queries wait behind it; when the last slice
//      retires its slices' results are handed over in chunk order and
//      joined by the consumer, off the dispatcher thread;
//   3. launches the admitted queries as one batch on that context's stream:
//      one upload of the packed query tables (which also resets the work
//      queues; one entry per query), a kernel that expands the entries
//      into chunk records, then, for an iteration of at most one chunk per
//      resident wave, one single-pass persistent decode-fused chunk kernel whose
//      chunks find their output offsets by decoupled look-back; a larger
//      iteration runs the staged form: the chunk kernel into per-chunk
//      slots, whose waves never wait on each other, then one tail kernel
//      that scans the chunk counts tile by tile (decoupled look-back between
//      tiles), gathers the survivors and writes the per-query offsets.
// Queries that arrive while earlier ones run on the device are admitted into
// the next free context and launched at once, so iterations overlap on the
// device.  Submitters queue queries in batches (a replay hands over its
// whole batch); the dispatcher takes every queued batch under the server
// lock in one move and admits from them without it, so neither side copies
// queries while the other waits for the lock.  Per-query offsets, and the results themselves when their bound
// fits the context's result buffer, are written by the device straight into
// pinned, device-mapped host memory; an iteration whose bound does not fit
// writes to device memory and copies exactly the total back.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <list>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "s4_internal.h"

namespace {

using Clock = std::chrono::steady_clock;
// Iteration contexts: four, one per hardware queue of the process (an
// overloaded server held 13.2-13.4 M queries/s with four, 12.0-12.3 M with
// three, 13.0 M with five and 12.5 M with six, whose streams share queues).
constexpr int kContexts = 4;

uint64_t ns_between(Clock::time_point a, Clock::time_point b) {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(b - a).count());
}

struct Query {
  uint64_t id = 0;
  uint32_t k = 0;
  uint32_t terms[s4::kMaxTerms + 1];  // shortest list first
  uint64_t items = 0, bound = 0;
  Clock::time_point submitted;
};

// The whole queries one iteration finished, handed over together: the
// dispatcher copies the iteration's results once (one allocation per
// iteration, not one per query).
struct DoneBatch {
  std::vector<uint64_t> ids, latency_ns;  // per query
  std::vector<uint64_t> offs;             // [n + 1] CSR offsets into results
  std::vector<uint32_t> results;
  Clock::time_point at;  // completion stamp of all of them
  size_t next = 0;       // queries already handed out by s4_server_poll
  size_t size() const { return ids.size(); }
  uint64_t count(size_t i) const { return offs[i + 1] - offs[i]; }
};

// A query run in slices, finished: its slices' results in chunk order,
// joined by the consumer, so the dispatcher never copies a whole large
// result while other queries wait for admission.
struct DoneJob {
  uint64_t id, count, latency_ns;
  std::vector<std::vector<uint32_t>> parts;
  Clock::time_point at;
  // append the result, in order, at dst
  void copy_to(uint32_t *dst) const {
    for (const auto &p : parts) dst = std::copy(p.begin(), p.end(), dst);
  }
};

// A query run in several slices (owned by the dispatcher thread).
struct Job {
  Query q;
  uint64_t next = 0;         // first chunk not admitted yet
  uint32_t outstanding = 0;  // slices admitted and not retired
  std::vector<std::pair<uint64_t, std::vector<uint32_t>>> parts;  // (first chunk, results) per retired slice
};

// A query's share of one iteration: chunks [c0, c1) of its shortest list.
struct Slice {
  const Query *q = nullptr;  // the whole query, in a submitted batch the context holds (job == nullptr)
  Job *job = nullptr;        // or the job this slice belongs to
  uint64_t c0 = 0, c1 = 0;
  const Query &query() const { return job ? job->q : *q; }
  // values of the shortest list in the slice: the bound on its results
  uint64_t bound() const {
    const uint64_t m = query().bound;
    return std::min<uint64_t>(m, s4::kBlock * c1) - std::min<uint64_t>(m, s4::kBlock * c0);
  }
};

struct Context {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void *dmem = nullptr;
  s4::BatchDev dev{};
  // query tables of one iteration, packed: the queue heads (zero; one per
  // sub-queue, 256 bytes apart), terms, first chunk of each query, one
  // 16-byte entry per query (uploaded), then the chunk records the device
  // expands from them (each part 16-byte aligned)
  uint8_t *h_tab = nullptr;  // pinned
  uint8_t *d_tab = nullptr;  // device
  uint64_t *state = nullptr;       // device, one scan word per chunk (single pass)
  uint32_t epoch = 0;              // scan generation of the last launch
  uint32_t *h_results = nullptr;   // pinned, device-mapped, results_per_ctx values
  uint32_t *d_hresults = nullptr;  // device view of h_results
  uint64_t *h_offs = nullptr, *d_offs = nullptr;  // pinned, device-mapped: CSR offsets
  uint32_t *h_err = nullptr, *d_err = nullptr;    // pinned, device-mapped: scan failure flag
  uint32_t *d_results = nullptr;  // device, 128 values per chunk
  std::vector<Slice> slices;
  // the submitted batches its whole-query slices point into, held until
  // the iteration retires (a slice is a pointer, not a copy of the query)
  std::vector<std::shared_ptr<const std::vector<Query>>> held;
  uint64_t items = 0, terms = 0, bound = 0;
  bool busy = false;
  bool has_job = false;  // holds a slice of a query run in slices
  bool direct = false;  // results written to h_results by the device
  bool single = false;  // single-pass kernel
  int phase = 0;        // 1: kernels running, 2: results copy running
  uint64_t reserved_stage = 0;
  Clock::time_point launched;
};

}  // namespace

struct s4_server {
  const s4_index *index = nullptr;
  s4_server_config cfg{};
  uint64_t slots_per_ctx = 0, items_per_ctx = 0, results_per_ctx = 0, terms_per_ctx = 0;
  uint64_t slice = 0;        // most chunks of one query per iteration
  uint64_t iter_items = 0;   // chunk budget of an iteration (a lone first slice aside)
  std::list<Job> jobs;       // queries running in slices (dispatcher only)
  Context ctx[kContexts];
  std::mutex mu;
  std::condition_variable cv;
  // queries submitted and not admitted yet: the batches submitters queue
  // (under mu), which the dispatcher takes all at once into its own list
  // and admits from without the lock; `queued` counts both (under mu)
  std::deque<std::vector<Query>> incoming;
  uint64_t queued = 0;
  std::deque<std::shared_ptr<const std::vector<Query>>> waiting;  // dispatcher only
  size_t waiting_pos = 0;                  // first query of waiting.front() not admitted
  std::deque<DoneBatch> completed;     // whole queries, per iteration
  std::deque<DoneJob> completed_jobs;  // queries run in slices
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

// byte offsets of the parts of a packed table
size_t terms_at() { return 4 * s4::kSubQueues * s4::kHeadStride; }
size_t bases_at(uint64_t nt) { return terms_at() + s4::align_up(4 * nt, 16); }
size_t qinfo_at(uint64_t nt, uint64_t nq) { return bases_at(nt) + s4::align_up(4 * (nq + 1), 16); }
size_t records_at(uint64_t nt, uint64_t nq) { return qinfo_at(nt, nq) + 16 * nq; }

int alloc_context(s4_server *s, Context &c) {
  S4_HIP(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
  S4_HIP(hipEventCreateWithFlags(&c.done, hipEventDisableTiming));
  const uint64_t nq = s->slots_per_ctx, items = s->items_per_ctx, nt = s->terms_per_ctx;
  const size_t tab = records_at(nt, nq) + 16 * items;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = s4::align_up(off + std::max<size_t>(bytes, 4), 256);
    return o;
  };
  const size_t o_tab = take(tab), o_state = take(8 * items), o_stage = take(4 * s4::kBlock * items),
               o_counts = take(4 * items), o_ctrl = take(64), o_qtick = take(8 * nq),
               o_res = take(4 * s4::kBlock * items);
  if (hipMalloc(&c.dmem, off) != hipSuccess) return s4::fail(S4_ENOMEM, "server context: device allocation failed");
  char *m = static_cast<char *>(c.dmem);
  c.d_tab = reinterpret_cast<uint8_t *>(m + o_tab);
  c.state = reinterpret_cast<uint64_t *>(m + o_state);
  c.d_results = reinterpret_cast<uint32_t *>(m + o_res);
  S4_HIP(hipMemset(c.state, 0, 8 * items));  // no word carries a live epoch
  s4::BatchDev &d = c.dev;
  d.lists = s->index->d_lists;
  d.feat = s->index->feat;
  d.head = reinterpret_cast<uint32_t *>(c.d_tab);
  d.sterms = reinterpret_cast<const uint32_t *>(c.d_tab + terms_at());
  d.state = c.state;
  d.stage = reinterpret_cast<uint32_t *>(m + o_stage);
  d.counts = reinterpret_cast<uint32_t *>(m + o_counts);
  d.excl = nullptr;  // the staged tail scans in place of the tile scans
  d.tiles = nullptr;
  d.total = reinterpret_cast<uint64_t *>(m + o_ctrl + 8);
  d.start = reinterpret_cast<uint64_t *>(m + o_ctrl + 16);
  d.stats = reinterpret_cast<uint64_t *>(m + o_ctrl + 24);
  d.qtick = reinterpret_cast<uint64_t *>(m + o_qtick);
  auto hmalloc = [&](void **p, size_t bytes, unsigned flags) {
    return hipHostMalloc(p, std::max<size_t>(bytes, 64), flags) == hipSuccess;
  };
  bool ok = hmalloc(reinterpret_cast<void **>(&c.h_tab), tab, hipHostMallocDefault) &&
            hmalloc(reinterpret_cast<void **>(&c.h_results), 4 * s->results_per_ctx, hipHostMallocMapped) &&
            hmalloc(reinterpret_cast<void **>(&c.h_offs), 8 * (nq + 1), hipHostMallocMapped) &&
            hmalloc(reinterpret_cast<void **>(&c.h_err), 4, hipHostMallocMapped);
  if (!ok) return s4::fail(S4_ENOMEM, "server context: pinned host allocation failed");
  S4_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&c.d_hresults), c.h_results, 0));
  S4_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&c.d_offs), c.h_offs, 0));
  S4_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&c.d_err), c.h_err, 0));
  c.dev.err = c.d_err;
  return S4_OK;
}

void free_context(Context &c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  if (c.dmem) (void)hipFree(c.dmem);
  for (void *p : {static_cast<void *>(c.h_tab), static_cast<void *>(c.h_results), static_cast<void *>(c.h_offs),
                  static_cast<void *>(c.h_err)})
    if (p) (void)hipHostFree(p);
  if (c.done) (void)hipEventDestroy(c.done);
  if (c.stream) (void)hipStreamDestroy(c.stream);
  c = Context{};
}

// Launch the queries gathered in c (caller holds no lock; c is private to
// the dispatcher while busy).
int launch_context(s4_server *s, Context &c) {
  const uint64_t nq = c.slices.size(), items = c.items;
  uint32_t *head = reinterpret_cast<uint32_t *>(c.h_tab);
  uint32_t *sterms = reinterpret_cast<uint32_t *>(c.h_tab + terms_at());
  uint32_t *ib = reinterpret_cast<uint32_t *>(c.h_tab + bases_at(c.terms));
  uint32_t *qi = reinterpret_cast<uint32_t *>(c.h_tab + qinfo_at(c.terms, nq));
  std::memset(head, 0, terms_at());
  uint64_t t = 0, it = 0;
  // one entry per query; the device expands them into chunk records
  for (uint64_t q = 0; q < nq; ++q) {
    const Slice &sl = c.slices[q];
    const Query &qq = sl.query();
    ib[q] = uint32_t(it);
    for (uint32_t j = 0; j < qq.k; ++j) sterms[t + j] = qq.terms[j];
    qi[4 * q] = uint32_t(sl.c0);
    qi[4 * q + 1] = uint32_t(t);
    qi[4 * q + 2] = qq.k;
    qi[4 * q + 3] = 0;
    t += qq.k;
    it += sl.c1 - sl.c0;
  }
  ib[nq] = uint32_t(it);
  c.direct = c.bound <= s->results_per_ctx;
  c.single = false;
  if (items == 0) {  // every shortest list is empty: nothing to run
    std::fill(c.h_offs, c.h_offs + nq + 1, 0);
    c.direct = true;
  } else {
    s4::BatchDev d = c.dev;
    d.item_base = reinterpret_cast<const uint32_t *>(c.d_tab + bases_at(c.terms));
    d.item_info = reinterpret_cast<const uint4 *>(c.d_tab + records_at(c.terms, nq));
    d.items = uint32_t(items);
    d.nq = uint32_t(nq);
    c.single = items <= s4::single_pass_max_items();
    // both forms place results by look-back over epoch-tagged scan words
    if (++c.epoch > s4::kMaxEpoch) {
      c.epoch = 1;
      S4_HIP(hipMemsetAsync(c.state, 0, 8 * s->items_per_ctx, c.stream));
    }
    d.epoch = c.epoch;
    *c.h_err = 0;
    S4_HIP(hipMemcpyAsync(c.d_tab, c.h_tab, records_at(c.terms, nq), hipMemcpyHostToDevice, c.stream));
    int rc = s4::enqueue_expand_items(d, reinterpret_cast<const uint4 *>(c.d_tab + qinfo_at(c.terms, nq)),
                                      reinterpret_cast<uint4 *>(c.d_tab + records_at(c.terms, nq)), c.stream);
    if (rc) return rc;
    uint32_t *out = c.direct ? c.d_hresults : c.d_results;
    // the staged form: chunk kernel and one tail kernel (scan, gather,
    // offsets); the table upload above zeroed the work queue and the tile
    // ticket
    rc = c.single ? s4::enqueue_serve_dev(d, out, c.direct ? s->results_per_ctx : s4::kBlock * items, c.d_offs,
                                          c.stream)
                  : s4::enqueue_staged_serve_dev(d, out, c.d_offs, c.stream);
    if (rc) return rc;
  }
  S4_HIP(hipEventRecord(c.done, c.stream));
  c.busy = true;
  c.phase = 1;
  c.launched = Clock::now();
  return S4_OK;
}

// Kernels done: copy exactly the results back (asynchronously when they
// fit the pinned buffer).  Returns true when the context can retire now.
bool start_copy(s4_server *s, Context &c, std::vector<uint32_t> *spill) {
  const uint64_t total = c.h_offs[c.slices.size()];
  if (c.direct || total == 0) return true;
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

// The CSR offsets the device wrote for c: non-decreasing, within the
// iteration's result bound.
bool offsets_valid(const Context &c) {
  if (c.h_offs[0] != 0) return false;
  for (size_t i = 0; i < c.slices.size(); ++i)
    if (c.h_offs[i + 1] < c.h_offs[i] || c.h_offs[i + 1] - c.h_offs[i] > c.slices[i].bound()) return false;
  return true;
}

// Move a finished context's results to the completed queues: the whole
// queries of the iteration as one batch (their results copied once, in
// slice order), slices into their job (a finished job's slices handed over
// in chunk order, to be joined by the consumer).
void retire_context(s4_server *s, Context &c, const uint32_t *res) {
  const auto now = Clock::now();
  const size_t n = c.slices.size();
  DoneBatch bt;
  bt.at = now;
  bt.ids.reserve(n);
  bt.latency_ns.reserve(n);
  bt.offs.reserve(n + 1);
  bt.offs.push_back(0);
  std::vector<DoneJob> jobs_done;
  bool any_job = false;
  for (size_t i = 0; i < n; ++i) {
    Slice &sl = c.slices[i];
    if (!sl.job) {
      bt.ids.push_back(sl.q->id);
      bt.latency_ns.push_back(ns_between(sl.q->submitted, now));
      bt.offs.push_back(bt.offs.back() + (c.h_offs[i + 1] - c.h_offs[i]));
      continue;
    }
    any_job = true;
    const uint64_t o0 = c.h_offs[i], cnt = c.h_offs[i + 1] - o0;
    Job &j = *sl.job;
    j.parts.emplace_back(sl.c0, std::vector<uint32_t>(res + o0, res + o0 + cnt));
    if (--j.outstanding == 0 && j.next == j.q.items) {
      std::sort(j.parts.begin(), j.parts.end(),
                [](const auto &a, const auto &b) { return a.first < b.first; });
      DoneJob d;
      d.id = j.q.id;
      d.count = 0;
      d.latency_ns = ns_between(j.q.submitted, now);
      d.at = now;
      d.parts.reserve(j.parts.size());
      for (auto &p : j.parts) {
        d.count += p.second.size();
        d.parts.push_back(std::move(p.second));
      }
      jobs_done.push_back(std::move(d));
      const Job *jp = &j;
      s->jobs.remove_if([jp](const Job &x) { return &x == jp; });
    }
  }
  // the whole queries' results: one contiguous range when the iteration
  // held no job slices, else each query's range in turn
  if (!any_job) {
    bt.results.assign(res, res + c.h_offs[n]);
  } else {
    bt.results.reserve(bt.offs.back());
    for (size_t i = 0; i < n; ++i)
      if (!c.slices[i].job) bt.results.insert(bt.results.end(), res + c.h_offs[i], res + c.h_offs[i + 1]);
  }
  const uint64_t finished = bt.size() + jobs_done.size();
  std::lock_guard<std::mutex> lock(s->mu);
  if (bt.size()) s->completed.push_back(std::move(bt));
  for (auto &d : jobs_done) s->completed_jobs.push_back(std::move(d));
  s->st.completed += finished;
  s->active -= finished;
  s->pool_in_use -= c.reserved_stage;
  c.slices.clear();
  c.held.clear();
  c.reserved_stage = 0;
  c.has_job = false;
  c.busy = false;
  c.phase = 0;
}

void dispatcher(s4_server *s) {
  (void)hipSetDevice(s->device);
  uint64_t device_ns = 0, host_ns = 0, retire_ns = 0, admit_ns = 0, launch_ns = 0;
  for (;;) {
    bool progressed = false;
    for (Context &c : s->ctx) {
      if (c.busy && hipEventQuery(c.done) == hipSuccess) {
        const auto t0 = Clock::now();
        if (c.phase == 1) {
          device_ns += ns_between(c.launched, t0);
          if (*c.h_err || !offsets_valid(c)) {
            // results unusable: fail the server loudly, drop the iteration
            std::lock_guard<std::mutex> lock(s->mu);
            s->worker_error = S4_EDEVICE;
            s->worker_msg = *c.h_err ? "single-pass scan failed (look-back guard or output overflow)"
                                     : "device wrote inconsistent result offsets";
            s->stop = true;
            std::fill(c.h_offs, c.h_offs + c.slices.size() + 1, 0);
          }
          std::vector<uint32_t> spill;
          if (start_copy(s, c, &spill)) retire_context(s, c, spill.empty() ? c.h_results : spill.data());
        } else {
          retire_context(s, c, c.h_results);
        }
        const uint64_t dt = ns_between(t0, Clock::now());
        host_ns += dt;
        retire_ns += dt;
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
      const auto t0 = Clock::now();
      {
        {
          // every batch submitted so far, moved (not copied) under the lock
          std::lock_guard<std::mutex> lock(s->mu);
          while (!s->incoming.empty()) {
            s->waiting.push_back(std::make_shared<const std::vector<Query>>(std::move(s->incoming.front())));
            s->incoming.pop_front();
          }
        }
        uint64_t items = 0, terms = 0, bound = 0, started = 0, memory_waits = 0, sliced = 0;
        // does a slice of `n` chunks, k terms and result bound `b` fit?
        auto fits = [&](uint64_t n, uint64_t k, uint64_t b) {
          if (s->pool_in_use + 4 * s4::kBlock * (items + n) > s->cfg.pool_bytes) return false;
          if (c.slices.empty()) return true;  // a single slice always fits the context
          return c.slices.size() < s->slots_per_ctx && items + n <= s->iter_items && terms + k <= s->terms_per_ctx &&
                 bound + b <= s->results_per_ctx;
        };
        auto admit = [&](Slice &&sl) {
          c.has_job |= sl.job != nullptr;
          const uint64_t n = sl.c1 - sl.c0;
          items += n;
          terms += sl.query().k;
          bound += sl.bound();
          c.slices.push_back(std::move(sl));
        };
        // 1. one slice of every query already running in slices, unless
        //    all contexts but this one already run such slices: long
        //    queries never take the last context, which stays free for
        //    short ones
        int job_contexts = 0;
        for (const Context &o : s->ctx) job_contexts += o.busy && o.has_job;
        for (Job &j : s->jobs) {
          if (job_contexts >= kContexts - 1) break;
          if (j.next == j.q.items) continue;
          Slice sl;
          sl.job = &j;
          sl.c0 = j.next;
          sl.c1 = std::min(j.q.items, j.next + s->slice);
          if (!fits(sl.c1 - sl.c0, j.q.k, sl.bound())) break;
          j.next = sl.c1;
          ++j.outstanding;
          admit(std::move(sl));
        }
        // 2. waiting queries, oldest first
        while (!s->waiting.empty()) {
          const std::vector<Query> &batch = *s->waiting.front();
          if (s->waiting_pos == batch.size()) {
            s->waiting.pop_front();
            s->waiting_pos = 0;
            continue;
          }
          const Query &q = batch[s->waiting_pos];
          Slice sl;
          sl.c1 = std::min(q.items, s->slice);
          if (sl.c1 < q.items) {  // too long for one slice: a job
            Job probe;
            probe.q = q;
            sl.job = &probe;
            if (!fits(sl.c1, q.k, sl.bound())) {
              if (c.slices.empty()) ++memory_waits;
              break;
            }
            s->jobs.push_back(std::move(probe));
            Job &j = s->jobs.back();
            sl.job = &j;
            j.next = sl.c1;
            j.outstanding = 1;
            ++sliced;
          } else {
            // a whole query: its slice points at it in its batch, which
            // the context holds until the iteration retires (no copy)
            if (!fits(sl.c1, q.k, q.bound)) {
              if (c.slices.empty()) ++memory_waits;
              break;
            }
            if (c.held.empty() || c.held.back() != s->waiting.front()) c.held.push_back(s->waiting.front());
            c.slices.emplace_back();
            Slice &ns = c.slices.back();
            ns.q = &q;
            ns.c1 = sl.c1;
            items += ns.c1;
            terms += q.k;
            bound += ns.bound();
            ++s->waiting_pos;
            ++started;
            continue;
          }
          ++s->waiting_pos;
          ++started;
          admit(std::move(sl));
        }
        std::lock_guard<std::mutex> lock(s->mu);
        s->queued -= started;
        s->st.waits_for_memory += memory_waits;
        s->st.sliced_queries += sliced;
        if (!c.slices.empty()) {
          c.items = items;
          c.terms = terms;
          c.bound = bound;
          c.reserved_stage = 4 * s4::kBlock * items;
          s->pool_in_use += c.reserved_stage;
          s->active += started;
          s->st.admitted += started;
          s->st.peak_active = std::max(s->st.peak_active, s->active);
          s->st.peak_pool_bytes = std::max(s->st.peak_pool_bytes, s->pool_in_use);
          s->st.max_batch = std::max<uint64_t>(s->st.max_batch, c.slices.size());
          ++s->st.iterations;
        }
      }
      const auto t1 = Clock::now();
      admit_ns += ns_between(t0, t1);
      if (!c.slices.empty()) {
        int rc = launch_context(s, c);
        launch_ns += ns_between(t1, Clock::now());
        if (rc) {
          std::lock_guard<std::mutex> lock(s->mu);
          s->worker_error = rc;
          s->worker_msg = s4_last_error();
          s->stop = true;
        } else {
          std::lock_guard<std::mutex> lock(s->mu);
          s->st.direct_iterations += c.direct;
          s->st.single_pass_iterations += c.single;
        }
        launched = true;
        host_ns += ns_between(t0, Clock::now());
      }
    }
    bool idle = false, any_busy = false;
    {
      std::unique_lock<std::mutex> lock(s->mu);
      s->st.device_ns = device_ns;
      s->st.host_ns = host_ns;
      s->st.retire_ns = retire_ns;
      s->st.admit_ns = admit_ns;
      s->st.launch_ns = launch_ns;
      for (Context &c : s->ctx) any_busy |= c.busy;
      const bool jobs_left = !s->jobs.empty();
      if (s->stop && !any_busy && ((s->queued == 0 && !jobs_left) || s->worker_error)) break;
      idle = !progressed && !launched;
      if (idle && !any_busy && s->queued == 0 && !jobs_left) {
        s->cv.wait_for(lock, std::chrono::milliseconds(1));
        continue;
      }
    }
    // iterations in flight: poll their events again at once
    if (idle) std::this_thread::yield();
  }
}

// Validate a query and put its terms in chain order (no lock needed: the
// index is immutable while the server exists).
int prepare_query(const s4_server *s, const uint32_t *terms, uint32_t k, Query *q) {
  if (k == 0 || k > s->cfg.max_terms) return s4::fail(S4_EINVAL, "query must have 1..max_terms terms");
  const s4_index *ix = s->index;
  for (uint32_t j = 0; j < k; ++j) {
    const uint32_t t = terms[j];
    if (t >= ix->count) return s4::fail(S4_EINVAL, "term out of range");
    if (k > 1 && !(ix->flags[t] & 1u)) return s4::fail(S4_EUNSORTED, "list is not strictly increasing");
    // insertion by length, stable for equal lengths
    uint32_t p = j;
    while (p > 0 && ix->lengths[q->terms[p - 1]] > ix->lengths[t]) {
      q->terms[p] = q->terms[p - 1];
      --p;
    }
    q->terms[p] = t;
  }
  q->k = k;
  const uint64_t m = ix->lengths[q->terms[0]];
  q->items = (m + s4::kBlock - 1) / s4::kBlock;
  q->bound = m;
  if (k > s->terms_per_ctx || 4 * s4::kBlock * std::min(q->items, s->slice) > s->cfg.pool_bytes)
    return s4::fail(S4_ERANGE, "one slice of the query needs more intermediate memory than the pool holds");
  return S4_OK;
}

// Caller holds s->mu.
int check_open_locked(s4_server *s) {
  if (s->stop) return s4::fail(S4_EINVAL, "server is stopping");
  if (s->worker_error) return s4::fail(s->worker_error, "server failed: " + s->worker_msg);
  return S4_OK;
}

}  // namespace

using namespace s4;

extern "C" {

int s4_server_create(const s4_index *index, const s4_server_config *cfg, s4_server **out) {
  if (!index || !cfg || !out) return fail(S4_EINVAL, "null argument");
  if (!cfg->max_slots || !cfg->pool_bytes || !cfg->max_terms || cfg->max_terms > kMaxTerms + 1)
    return fail(S4_EINVAL, "server config: need max_slots, pool_bytes > 0 and 1 <= max_terms <= 33");
  // single-pass iterations take chunks in result order; a partitioned
  // index queues them per part
  if (index->parts > 1) return fail(S4_EINVAL, "the server needs an index built without doc-ID parts");
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
  s->slice = std::max<uint64_t>(1, std::min<uint64_t>(cfg->slice_chunks ? cfg->slice_chunks : 16384,
                                                      s->items_per_ctx));
  s->iter_items = std::min<uint64_t>(s->items_per_ctx, 4 * s->slice);
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
  Query q;
  int rc = prepare_query(s, terms, k, &q);
  std::lock_guard<std::mutex> lock(s->mu);
  if (rc) {
    if (rc == S4_ERANGE) ++s->st.rejected;
    return rc;
  }
  rc = check_open_locked(s);
  if (rc) return rc;
  if (s->queued >= 64ull * s->cfg.max_slots) return fail(S4_EAGAIN, "waiting queue full");
  q.id = s->next_id++;
  q.submitted = Clock::now();
  *id = q.id;
  if (s->incoming.empty() || s->incoming.back().size() >= 256) s->incoming.emplace_back();
  s->incoming.back().push_back(q);
  ++s->queued;
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
  if (max_done) res_offsets[0] = 0;
  bool room = true;
  while (room && n < max_done && !s->completed.empty()) {
    DoneBatch &b = s->completed.front();
    for (; n < max_done && b.next < b.size(); ++b.next, ++n) {
      const uint64_t cnt = b.count(b.next);
      if (used + cnt > results_cap || (cnt && !results)) {
        room = false;
        break;
      }
      std::copy(b.results.begin() + b.offs[b.next], b.results.begin() + b.offs[b.next + 1], results + used);
      ids[n] = b.ids[b.next];
      counts[n] = cnt;
      latency_ns[n] = b.latency_ns[b.next];
      used += cnt;
      res_offsets[n + 1] = used;
    }
    if (b.next == b.size()) s->completed.pop_front();
  }
  while (room && n < max_done && !s->completed_jobs.empty()) {
    DoneJob &d = s->completed_jobs.front();
    if (used + d.count > results_cap || (d.count && !results)) break;
    d.copy_to(results + used);
    ids[n] = d.id;
    counts[n] = d.count;
    latency_ns[n] = d.latency_ns;
    used += d.count;
    res_offsets[n + 1] = used;
    s->completed_jobs.pop_front();
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

// Replay submission batching (see s4_server_replay).
constexpr size_t kSubmitBatch = 256;

// Queries of a replayed trace are validated and put in chain order ahead
// of their arrival, by helper threads, a segment of kPrepSegment queries
// at a time into a ring of kPrepRing segments (the work each client does
// before it submits, done in parallel, so that one replay thread can offer
// the server more than one thread's worth of clients).
constexpr uint64_t kPrepSegment = 4096;
constexpr uint64_t kPrepRing = 16;
constexpr unsigned kPrepThreads = 3;

struct PrepSegment {
  std::vector<Query> q;
  std::atomic<int> ready{0};  // 1 once prepared (release), 0 once consumed
  int rc = S4_OK;             // first failure in the segment, at query bad
  uint64_t bad = 0;
  std::string msg;
};

struct Preparer {
  const s4_server *s;
  const uint32_t *terms;
  const uint64_t *qoffs;
  uint64_t nq, nseg;
  std::vector<PrepSegment> ring;
  std::atomic<uint64_t> claimed{0}, consumed{0};  // segments claimed by helpers / consumed by the replay
  std::atomic<bool> stop{false};
  std::vector<std::thread> helpers;

  Preparer(const s4_server *srv, const uint32_t *t, const uint64_t *o, uint64_t n)
      : s(srv), terms(t), qoffs(o), nq(n), nseg((n + kPrepSegment - 1) / kPrepSegment), ring(kPrepRing) {
    for (auto &g : ring) g.q.resize(kPrepSegment);
    const unsigned nh = unsigned(std::min<uint64_t>(kPrepThreads, std::max<uint64_t>(1, nseg)));
    for (unsigned h = 0; h < nh; ++h) helpers.emplace_back([this] { run(); });
  }
  ~Preparer() {
    stop.store(true);
    for (auto &t : helpers) t.join();
  }
  void run() {
    for (;;) {
      const uint64_t seg = claimed.fetch_add(1);
      if (seg >= nseg) return;
      // the ring slot is free once the segment kPrepRing before is consumed
      while (seg >= consumed.load(std::memory_order_acquire) + kPrepRing) {
        if (stop.load()) return;
        std::this_thread::yield();
      }
      PrepSegment &g = ring[seg % kPrepRing];
      g.rc = S4_OK;
      const uint64_t q0 = seg * kPrepSegment, q1 = std::min(nq, q0 + kPrepSegment);
      for (uint64_t q = q0; q < q1; ++q) {
        const int rc = prepare_query(s, terms + qoffs[q], uint32_t(qoffs[q + 1] - qoffs[q]), &g.q[q - q0]);
        if (rc) {
          g.rc = rc;
          g.bad = q;
          g.msg = s4_last_error();
          break;
        }
      }
      g.ready.store(1, std::memory_order_release);
    }
  }
  // query q, prepared (waits for its segment; false on the stop flag or
  // the time limit); rc / msg set when the segment failed at or before q
  const Query *get(uint64_t q, Clock::time_point t0, double timeout_s, int *rc, std::string *msg) {
    PrepSegment &g = ring[(q / kPrepSegment) % kPrepRing];
    while (!g.ready.load(std::memory_order_acquire))
      if (std::chrono::duration<double>(Clock::now() - t0).count() > timeout_s) {
        *rc = S4_ERANGE;
        *msg = "replay timed out";
        return nullptr;
      }
    if (g.rc && g.bad <= q) {
      *rc = g.rc;
      *msg = g.msg;
      return nullptr;
    }
    return &g.q[q % kPrepSegment];
  }
  // query q was the last of its segment (or of the trace): the slot is free
  void release(uint64_t q) {
    if ((q + 1) % kPrepSegment == 0 || q + 1 == nq) {
      ring[(q / kPrepSegment) % kPrepRing].ready.store(0, std::memory_order_relaxed);
      consumed.fetch_add(1, std::memory_order_release);
    }
  }
};
constexpr uint64_t kSubmitWaitNs = 10000;

int s4_server_replay(s4_server *s, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                     const uint64_t *h_arrival_ns, uint64_t *latency_ns, uint64_t *counts, uint32_t *results,
                     uint64_t results_cap, uint64_t *res_offsets, const uint8_t *keep, double timeout_s,
                     double *elapsed_s) {
  if (!s || !h_q_offsets || !h_arrival_ns || !latency_ns || !counts || (nq && !h_terms))
    return fail(S4_EINVAL, "null argument");
  if (results && !res_offsets) return fail(S4_EINVAL, "results need res_offsets");
  // results stay in the batches they arrived in until the end: query q's
  // are entry where[q].second of kept[where[q].first], or, for a query run
  // in slices or picked by keep, its parts (a copy, so batches are not held)
  std::vector<DoneBatch> kept;
  std::vector<std::pair<uint32_t, uint32_t>> where(results && !keep ? nq : 0, {UINT32_MAX, 0u});
  std::unordered_map<uint64_t, std::vector<std::vector<uint32_t>>> res_parts;
  uint64_t ndone = 0, next = 0;
  // query of each id this replay assigned: ids are handed out in order under
  // the lock, so q_of[id - id0] (UINT64_MAX for ids of other submitters, or
  // once finished) replaces a hash map on the per-query path
  uint64_t id0 = UINT64_MAX;
  std::vector<uint64_t> q_of;
  q_of.reserve(nq);
  std::vector<Query> due;
  std::deque<DoneBatch> got;
  std::deque<DoneJob> got_jobs;
  const auto t0 = Clock::now();
  auto now_ns = [&]() { return ns_between(t0, Clock::now()); };
  uint64_t last_done_ns = 0, last_drain_ns = 0;
  // queries [next, prepared) are validated and wait in `due` to be queued
  uint64_t prepared = 0;
  Preparer prep(s, h_terms, h_q_offsets, nq);
  while (ndone < nq) {
    // every query due by now (prepared ahead by the helpers)
    const uint64_t t = now_ns();
    for (; prepared < nq && h_arrival_ns[prepared] <= t && due.size() < 8192; ++prepared) {
      int rc = S4_OK;
      std::string msg;
      const Query *pq = prep.get(prepared, t0, timeout_s, &rc, &msg);
      if (!pq) {
        if (rc == S4_ERANGE && msg != "replay timed out") {
          std::lock_guard<std::mutex> lock(s->mu);
          ++s->st.rejected;
        }
        return fail(rc, msg);
      }
      due.push_back(*pq);
      prep.release(prepared);
    }
    // queued under one lock per batch: at least kSubmitBatch queries, or
    // the oldest has waited kSubmitWaitNs, or no more will arrive (taking
    // the lock for every few queries of a fast arrival stream kept the
    // dispatcher from its admissions); otherwise the lock is taken only to
    // drain completions now and then (latencies are stamped by the
    // dispatcher, not here)
    const bool submit = !due.empty() && (due.size() >= kSubmitBatch || prepared == nq ||
                                         t >= h_arrival_ns[next] + kSubmitWaitNs);
    if (!submit && t < last_drain_ns + 50000) continue;
    last_drain_ns = t;
    {
      std::lock_guard<std::mutex> lock(s->mu);
      int rc = check_open_locked(s);
      if (rc) return rc;
      const uint64_t room = 64ull * s->cfg.max_slots - std::min<uint64_t>(s->queued, 64ull * s->cfg.max_slots);
      const uint64_t take = std::min<uint64_t>(room, due.size());
      const auto now = Clock::now();
      if (take && id0 == UINT64_MAX) id0 = s->next_id;
      for (uint64_t i = 0; i < take; ++i) {
        Query &q = due[i];
        q.id = s->next_id++;
        q.submitted = now;
        const uint64_t slot = q.id - id0;
        if (slot >= q_of.size()) q_of.resize(slot + 1, UINT64_MAX);
        q_of[slot] = next + i;
      }
      // the batch goes to the server whole (moved, not copied, when all of
      // `due` is taken)
      if (take == due.size()) {
        if (take) s->incoming.push_back(std::move(due));
        due = std::vector<Query>();
        due.reserve(kSubmitBatch);
      } else if (take) {
        s->incoming.emplace_back(due.begin(), due.begin() + std::ptrdiff_t(take));
        due.erase(due.begin(), due.begin() + std::ptrdiff_t(take));
      }
      s->queued += take;
      s->st.submitted += take;
      next += take;
      if (take) s->cv.notify_one();
      got.swap(s->completed);
      got_jobs.swap(s->completed_jobs);
    }
    // completions, outside the lock
    auto finish = [&](uint64_t id, uint64_t count, Clock::time_point at) -> uint64_t {
      if (id0 == UINT64_MAX || id < id0 || id - id0 >= q_of.size() || q_of[id - id0] == UINT64_MAX) return UINT64_MAX;
      const uint64_t q = q_of[id - id0];
      q_of[id - id0] = UINT64_MAX;
      const uint64_t fin = ns_between(t0, at);
      latency_ns[q] = fin > h_arrival_ns[q] ? fin - h_arrival_ns[q] : 0;
      last_done_ns = std::max(last_done_ns, fin);
      counts[q] = count;
      ++ndone;
      return q;
    };
    while (!got.empty()) {
      DoneBatch &b = got.front();
      for (size_t i = b.next; i < b.size(); ++i) {
        const uint64_t q = finish(b.ids[i], b.count(i), b.at);
        if (q == UINT64_MAX || !results) continue;
        if (!keep)
          where[q] = {uint32_t(kept.size()), uint32_t(i)};
        else if (keep[q])
          res_parts[q].emplace_back(b.results.begin() + b.offs[i], b.results.begin() + b.offs[i + 1]);
      }
      if (results && !keep) kept.push_back(std::move(b));
      got.pop_front();
    }
    while (!got_jobs.empty()) {
      DoneJob &d = got_jobs.front();
      const uint64_t q = finish(d.id, d.count, d.at);
      if (q != UINT64_MAX && results && (!keep || keep[q])) res_parts[q] = std::move(d.parts);
      got_jobs.pop_front();
    }
    if (double(now_ns()) * 1e-9 > timeout_s) return fail(S4_ERANGE, "replay timed out");
    if (next < nq && h_arrival_ns[next] > now_ns() + 50000)
      std::this_thread::sleep_for(std::chrono::microseconds(10));
    else if (next == nq)
      std::this_thread::sleep_for(std::chrono::microseconds(5));
  }
  if (elapsed_s) *elapsed_s = double(last_done_ns - (nq ? h_arrival_ns[0] : 0)) * 1e-9;
  if (results) {
    uint64_t used = 0;
    res_offsets[0] = 0;
    for (uint64_t q = 0; q < nq; ++q) {
      if (keep && !keep[q]) {
        res_offsets[q + 1] = used;
        continue;
      }
      if (used + counts[q] > results_cap) return fail(S4_ERANGE, "results_cap too small");
      auto it = res_parts.find(q);
      if (it != res_parts.end()) {
        uint32_t *at = results + used;
        for (const auto &p : it->second) at = std::copy(p.begin(), p.end(), at);
      } else if (where[q].first != UINT32_MAX) {
        const DoneBatch &b = kept[where[q].first];
        const size_t i = where[q].second;
        std::copy(b.results.begin() + b.offs[i], b.results.begin() + b.offs[i + 1], results + used);
      }
      used += counts[q];
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

// The plain path of conjunctive queries over an index: every query is its
// own single-launch conjunction (s4_intersect_k's kernel: chunks of the
// shortest list carried through the other lists in SvS order, Sec. 6, and
// placed by look-back), launched one after another on one stream with no
// batching.  Submission runs here, in C++, so what is measured is the
// device path and the runtime's launch cost, not an interpreter.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>
#include <vector>

#include "s4_internal.h"

using namespace s4;

namespace {

using Clock = std::chrono::steady_clock;

uint64_t ns_since(Clock::time_point t0) {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count());
}

// Query q's descriptors, shortest first (stable: SvS), into ord; its
// shortest length into *m.
int order_query(const s4_index *ix, const uint32_t *terms, uint64_t a, uint64_t b, DList *ord, uint64_t *m) {
  const uint64_t k = b - a;
  if (k < 2 || k > kMaxTerms + 1) return fail(S4_EINVAL, "plain path: queries take 2 to 33 terms");
  for (uint64_t i = 0; i < k; ++i) {
    const uint32_t t = terms[a + i];
    if (t >= ix->count) return fail(S4_EINVAL, "plain path: term outside the index");
    const DList &d = ix->lists[t];
    if (!(ix->flags[t] & 1u)) return fail(S4_EUNSORTED, "plain path: lists must be strictly increasing");
    uint64_t j = i;
    for (; j > 0 && ord[j - 1].n > d.n; --j) ord[j] = ord[j - 1];
    ord[j] = d;
  }
  *m = ord[0].n;
  return S4_OK;
}

int check_index(const s4_index *ix) {
  if (!ix) return fail(S4_EINVAL, "null index");
  if (ix->parts > 1 || ix->bitmap_lists) return fail(S4_EINVAL, "plain path: plain indexes only (no parts, no bitmaps)");
  return S4_OK;
}

}  // namespace

extern "C" {

int s4_plain_run(const s4_index *index, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                 uint32_t *d_results, uint64_t results_cap, uint64_t *res_offsets, uint64_t *d_counts,
                 void *d_scratch, size_t scratch_bytes, uint64_t *lat_ns, uint64_t *elapsed_ns, void *stream) {
  int rc = check_index(index);
  if (rc) return rc;
  if (!h_q_offsets || !res_offsets || (nq && (!h_terms || !d_counts || !d_results)))
    return fail(S4_EINVAL, "null argument");
  rc = ensure_device();
  if (rc) return rc;
  // placement and scratch first: nothing is launched unless everything fits
  DList ord[kMaxTerms + 1];
  uint64_t need = 0;
  res_offsets[0] = 0;
  for (uint64_t q = 0; q < nq; ++q) {
    uint64_t m = 0;
    rc = order_query(index, h_terms, h_q_offsets[q], h_q_offsets[q + 1], ord, &m);
    if (rc) return rc;
    res_offsets[q + 1] = res_offsets[q] + m;
    need = std::max<uint64_t>(need, conjunction_scratch_bytes(m));
  }
  if (res_offsets[nq] > results_cap) return fail(S4_ERANGE, "results_cap below the sum of shortest lengths");
  if (need > scratch_bytes || (need && !d_scratch)) return fail(S4_ERANGE, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  S4_HIP(hipStreamSynchronize(st));
  const Clock::time_point t0 = Clock::now();
  for (uint64_t q = 0; q < nq; ++q) {
    uint64_t m = 0;
    order_query(index, h_terms, h_q_offsets[q], h_q_offsets[q + 1], ord, &m);
    const Clock::time_point tq = Clock::now();
    rc = enqueue_conjunction(ord, uint32_t(h_q_offsets[q + 1] - h_q_offsets[q]), d_scratch,
                             d_results + res_offsets[q], d_counts + q, st);
    if (rc) return rc;
    if (lat_ns) {
      S4_HIP(hipStreamSynchronize(st));
      lat_ns[q] = ns_since(tq);
    }
  }
  S4_HIP(hipStreamSynchronize(st));
  if (elapsed_ns) *elapsed_ns = ns_since(t0);
  return S4_OK;
}

int s4_plain_replay(const s4_index *index, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                    const uint64_t *h_arrival_ns, uint64_t *latency_ns, uint32_t *d_results, uint64_t results_cap,
                    uint64_t *d_counts, void *d_scratch, size_t scratch_bytes, double timeout_s, double *elapsed_s,
                    void *stream) {
  int rc = check_index(index);
  if (rc) return rc;
  if (!h_q_offsets || !h_arrival_ns || !latency_ns || (nq && (!h_terms || !d_counts || !d_results)))
    return fail(S4_EINVAL, "null argument");
  rc = ensure_device();
  if (rc) return rc;
  DList ord[kMaxTerms + 1];
  uint64_t need = 0, longest = 0;
  for (uint64_t q = 0; q < nq; ++q) {
    uint64_t m = 0;
    rc = order_query(index, h_terms, h_q_offsets[q], h_q_offsets[q + 1], ord, &m);
    if (rc) return rc;
    if (q && h_arrival_ns[q] < h_arrival_ns[q - 1]) return fail(S4_EINVAL, "arrivals must not decrease");
    longest = std::max(longest, m);
    need = std::max<uint64_t>(need, conjunction_scratch_bytes(m));
  }
  if (longest > results_cap) return fail(S4_ERANGE, "results_cap below the longest shortest list");
  if (need > scratch_bytes || (need && !d_scratch)) return fail(S4_ERANGE, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  S4_HIP(hipStreamSynchronize(st));
  // completion events, reused in a ring once the watcher has seen them
  constexpr uint32_t kRing = 512;
  std::vector<hipEvent_t> ev(kRing, nullptr);
  auto destroy = [&]() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  };
  for (auto &e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      destroy();
      return fail(S4_EDEVICE, "plain replay: event creation failed");
    }
  std::atomic<uint64_t> launched{0}, seen{0};
  std::atomic<bool> stop{false};
  std::atomic<int> watch_rc{0};
  uint64_t last_done = 0;
  const Clock::time_point t0 = Clock::now();
  // the watcher stamps each query when its event completes, in order
  std::thread watcher([&]() {
    for (uint64_t q = 0; q < nq; ++q) {
      while (launched.load(std::memory_order_acquire) <= q)
        if (stop.load()) return;
      for (;;) {
        const hipError_t e = hipEventQuery(ev[q % kRing]);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) {
          watch_rc.store(S4_EDEVICE);
          return;
        }
        if (stop.load()) return;
      }
      const uint64_t t = ns_since(t0);
      latency_ns[q] = t > h_arrival_ns[q] ? t - h_arrival_ns[q] : 0;
      last_done = t;
      seen.store(q + 1, std::memory_order_release);
    }
  });
  rc = S4_OK;
  for (uint64_t q = 0; q < nq && rc == S4_OK; ++q) {
    // wait for the arrival, and for the ring slot to be free
    while (ns_since(t0) < h_arrival_ns[q] || q - seen.load(std::memory_order_acquire) >= kRing) {
      if (watch_rc.load()) break;
      if (double(ns_since(t0)) * 1e-9 > timeout_s) break;
    }
    if (watch_rc.load()) {
      rc = fail(S4_EDEVICE, "plain replay: a query failed on the device");
      break;
    }
    if (double(ns_since(t0)) * 1e-9 > timeout_s) {
      rc = fail(S4_ERANGE, "plain replay timed out");
      break;
    }
    uint64_t m = 0;
    order_query(index, h_terms, h_q_offsets[q], h_q_offsets[q + 1], ord, &m);
    rc = enqueue_conjunction(ord, uint32_t(h_q_offsets[q + 1] - h_q_offsets[q]), d_scratch, d_results,
                             d_counts + q, st);
    if (rc) break;
    if (hipEventRecord(ev[q % kRing], st) != hipSuccess) {
      rc = fail(S4_EDEVICE, "plain replay: event record failed");
      break;
    }
    launched.store(q + 1, std::memory_order_release);
  }
  if (rc == S4_OK)
    while (seen.load(std::memory_order_acquire) < nq && !watch_rc.load())
      if (double(ns_since(t0)) * 1e-9 > timeout_s) {
        rc = fail(S4_ERANGE, "plain replay timed out");
        break;
      }
  stop.store(true);
  watcher.join();
  if (rc == S4_OK && watch_rc.load()) rc = fail(S4_EDEVICE, "plain replay: a query failed on the device");
  const hipError_t se = hipStreamSynchronize(st);
  destroy();
  if (rc) return rc;
  if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
  if (elapsed_s) *elapsed_s = double(last_done - (nq ? h_arrival_ns[0] : 0)) * 1e-9;
  return S4_OK;
}

}  // extern "C"

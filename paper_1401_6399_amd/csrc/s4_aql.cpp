// Per-list decode dispatched on queues of the library's own: one kernel
// dispatch packet per list (the k_decode launch s4_decode_lists_dev would
// make), written straight into HSA user queues.  The lists are spread over
// kQueues queues by bytes (largest first), each queue alternating its large
// and small lists; a queue's packets carry no barrier and no fence, since
// the lists of a step are independent; each queue ends a step with a
// barrier packet that signals, and starts the next
// one with a barrier packet waiting for every queue's signal, so steps do
// not overlap.  The kernels are the ones HIP loaded for this library, found
// through the AMD loader extension; their argument blocks and packet images
// are built once per plan (arguments in device memory), and a step copies
// the images into the rings.  Every run opens with a barrier
// packet whose system-scope acquire invalidates the caches before the first
// kernel reads arguments or lists written through other queues.  A run can
// be timed per dispatch (profiling enabled on the queues, one completion
// signal per dispatch), or enqueued behind the work of a HIP stream (a host
// function of that stream submits it and returns when it is complete).
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>
#include <hsa/hsa_ven_amd_loader.h>

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "s4_internal.h"

using namespace s4;

namespace {

constexpr uint32_t kArgStride = 128;          // bytes per dispatch's argument block
constexpr double kWaitLimitSeconds = 20.0;    // a step never takes this long
constexpr uint32_t kQueueSlots = 4096;
// Queues of the dispatcher: dispatches of one queue run one after another
// (a tiny one costs about 1.8 us of its queue), so concurrency comes from
// queues; more than four (with the runtime's own) made every queue slower.
constexpr uint32_t kQueues = 4;
static_assert(kQueues >= 1 && kQueues <= 16, "queues per device");
constexpr uint32_t kMaxSteps = 64;            // signals kept per queue


struct KernelInfo {
  uint64_t object = 0;
  uint32_t group = 0, priv = 0, kernarg = 0;
};

struct AqlState {
  bool ready = false;
  // a run stopped with packet slots reserved or packets in flight: the
  // queues may be stalled and argument blocks still referenced, so no
  // further run is accepted and no plan's argument blocks are freed
  bool broken = false;
  int device = -1;
  hsa_agent_t agent{};
  uint64_t ts_hz = 0;  // HSA system timestamp frequency (dispatch profiling)
  hsa_queue_t *queues[kQueues] = {};
  hsa_signal_t step_done[kMaxSteps][kQueues] = {};  // queue q finished step s
  KernelInfo kernels[4];  // k_decode<P, false>, P = 1, 2, 4, 8
};

std::mutex g_mu;
AqlState g_state;
std::atomic<int> g_queue_error{0};

void queue_error(hsa_status_t status, hsa_queue_t *, void *) { g_queue_error.store(int(status)); }

int slot_of(uint32_t P) { return P == 8 ? 3 : P == 4 ? 2 : P == 2 ? 1 : 0; }

std::string decode_kernel_name(uint32_t P) {
  return "_ZN2s48k_decodeILi" + std::to_string(P) + "ELb0EEEvPKhPKjPK15HIP_vector_typeIjLj4EES4_PjjjjjS4_j";
}

struct AgentSearch {
  uint32_t bdf = 0;
  std::vector<hsa_agent_t> gpus;
  hsa_agent_t match{};
  bool found = false;
};

hsa_status_t visit_agent(hsa_agent_t a, void *data) {
  auto *s = static_cast<AgentSearch *>(data);
  hsa_device_type_t type;
  if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &type) != HSA_STATUS_SUCCESS || type != HSA_DEVICE_TYPE_GPU)
    return HSA_STATUS_SUCCESS;
  s->gpus.push_back(a);
  uint32_t bdf = 0;
  if (hsa_agent_get_info(a, hsa_agent_info_t(HSA_AMD_AGENT_INFO_BDFID), &bdf) == HSA_STATUS_SUCCESS &&
      (bdf >> 3) == (s->bdf >> 3)) {
    s->match = a;
    s->found = true;
  }
  return HSA_STATUS_SUCCESS;
}

struct SymbolSearch {
  hsa_agent_t agent{};
  std::string want;
  KernelInfo info;
  int hits = 0;
};

hsa_status_t visit_symbol(hsa_executable_t, hsa_agent_t, hsa_executable_symbol_t sym, void *data) {
  auto *s = static_cast<SymbolSearch *>(data);
  hsa_symbol_kind_t kind;
  if (hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_TYPE, &kind) != HSA_STATUS_SUCCESS ||
      kind != HSA_SYMBOL_KIND_KERNEL)
    return HSA_STATUS_SUCCESS;
  uint32_t len = 0;
  if (hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_NAME_LENGTH, &len) != HSA_STATUS_SUCCESS)
    return HSA_STATUS_SUCCESS;
  std::string name(len, '\0');
  if (hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_NAME, &name[0]) != HSA_STATUS_SUCCESS)
    return HSA_STATUS_SUCCESS;
  name.resize(strnlen(name.c_str(), len));
  if (name != s->want && name != s->want + ".kd") return HSA_STATUS_SUCCESS;
  KernelInfo k;
  if (hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_OBJECT, &k.object) != HSA_STATUS_SUCCESS ||
      hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_KERNARG_SEGMENT_SIZE, &k.kernarg) !=
          HSA_STATUS_SUCCESS ||
      hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_GROUP_SEGMENT_SIZE, &k.group) !=
          HSA_STATUS_SUCCESS ||
      hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_PRIVATE_SEGMENT_SIZE, &k.priv) !=
          HSA_STATUS_SUCCESS)
    return HSA_STATUS_SUCCESS;
  s->info = k;
  ++s->hits;
  return HSA_STATUS_SUCCESS;
}

struct ExecSearch {
  SymbolSearch *sym;
};

hsa_status_t visit_executable(hsa_executable_t e, void *data) {
  auto *s = static_cast<ExecSearch *>(data);
  (void)hsa_executable_iterate_agent_symbols(e, s->sym->agent, visit_symbol, s->sym);
  return HSA_STATUS_SUCCESS;
}

// Agent, queue and completion signal of the current device (once).
int ensure_queue() {
  if (g_state.ready) return S4_OK;
  int dev = 0;
  S4_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  S4_HIP(hipGetDeviceProperties(&prop, dev));
  if (hsa_init() != HSA_STATUS_SUCCESS) return fail(S4_EDEVICE, "hsa_init failed");
  AgentSearch as;
  as.bdf = (uint32_t(prop.pciBusID) << 8) | (uint32_t(prop.pciDeviceID) << 3);
  if (hsa_iterate_agents(visit_agent, &as) != HSA_STATUS_SUCCESS) return fail(S4_EDEVICE, "agent enumeration failed");
  if (!as.found) {
    if (as.gpus.size() != 1) return fail(S4_EDEVICE, "no HSA agent matches the current HIP device");
    as.match = as.gpus[0];
  }
  uint32_t max_size = 0;
  if (hsa_agent_get_info(as.match, HSA_AGENT_INFO_QUEUE_MAX_SIZE, &max_size) != HSA_STATUS_SUCCESS || max_size < 1024)
    return fail(S4_EDEVICE, "agent queue size query failed");
  const uint32_t slots = std::min(kQueueSlots, max_size);
  for (uint32_t j = 0; j < kQueues; ++j)
    if (hsa_queue_create(as.match, slots, HSA_QUEUE_TYPE_MULTI, queue_error, nullptr, UINT32_MAX, UINT32_MAX,
                         &g_state.queues[j]) != HSA_STATUS_SUCCESS)
      return fail(S4_EDEVICE, "hsa_queue_create failed");
  for (auto &row : g_state.step_done)
    for (auto &sig : row)
      if (hsa_signal_create(1, 0, nullptr, &sig) != HSA_STATUS_SUCCESS)
        return fail(S4_EDEVICE, "hsa_signal_create failed");
  if (hsa_system_get_info(HSA_SYSTEM_INFO_TIMESTAMP_FREQUENCY, &g_state.ts_hz) != HSA_STATUS_SUCCESS ||
      g_state.ts_hz == 0)
    return fail(S4_EDEVICE, "HSA timestamp frequency query failed");
  g_state.agent = as.match;
  g_state.device = dev;
  g_state.ready = true;
  return S4_OK;
}

// The loaded k_decode<P, false> of this library, checked against the
// argument block the dispatcher writes.
int ensure_kernel(uint32_t P) {
  KernelInfo &k = g_state.kernels[slot_of(P)];
  if (k.object) return S4_OK;
  // make sure HIP has loaded the code object holding the kernel
  hipFuncAttributes attr;
  S4_HIP(hipFuncGetAttributes(&attr, decode_kernel_host_address(P, false)));
  hsa_ven_amd_loader_1_03_pfn_t loader;
  std::memset(&loader, 0, sizeof loader);
  if (hsa_system_get_major_extension_table(HSA_EXTENSION_AMD_LOADER, 1, sizeof loader, &loader) !=
          HSA_STATUS_SUCCESS ||
      !loader.hsa_ven_amd_loader_iterate_executables)
    return fail(S4_EDEVICE, "HSA loader extension unavailable");
  SymbolSearch ss;
  ss.agent = g_state.agent;
  ss.want = decode_kernel_name(P);
  ExecSearch es{&ss};
  if (loader.hsa_ven_amd_loader_iterate_executables(visit_executable, &es) != HSA_STATUS_SUCCESS)
    return fail(S4_EDEVICE, "executable enumeration failed");
  if (ss.hits != 1) return fail(S4_EDEVICE, "decode kernel found " + std::to_string(ss.hits) + " times, not once");
  if (ss.info.kernarg != kDecodeArgBytes || ss.info.priv != 0 || ss.info.group > 64 * 1024 || !ss.info.object)
    return fail(S4_EDEVICE, "decode kernel's argument or segment sizes differ from the dispatcher's");
  k = ss.info;
  return S4_OK;
}

uint16_t packet_header(hsa_packet_type_t type, bool barrier, hsa_fence_scope_t acquire, hsa_fence_scope_t release) {
  return uint16_t((type << HSA_PACKET_HEADER_TYPE) | ((barrier ? 1 : 0) << HSA_PACKET_HEADER_BARRIER) |
                  (acquire << HSA_PACKET_HEADER_SCACQUIRE_FENCE_SCOPE) |
                  (release << HSA_PACKET_HEADER_SCRELEASE_FENCE_SCOPE));
}

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

// The dispatcher cannot be used again: a packet slot was reserved and never
// filled (the queue stalls there), or packets may still be in flight.
int poison(const std::string &msg) {
  g_state.broken = true;
  return fail(S4_EDEVICE, msg + "; the per-list dispatcher is disabled for the rest of the process");
}

// Reserve the next packet slot once the queue has room for it (bounded
// wait).  The write index is advanced only after the room is seen, so a
// failed wait leaves no reserved slot behind.  One host thread writes the
// queues (the dispatcher's mutex), so the slot stays this thread's.
int next_slot(hsa_queue_t *q, Clock::time_point t0, uint64_t *index) {
  const uint64_t i = hsa_queue_load_write_index_relaxed(q);
  while (i - hsa_queue_load_read_index_scacquire(q) >= q->size) {
    if (g_queue_error.load()) return poison("the decode queue reported an error");
    if (seconds_since(t0) > kWaitLimitSeconds) return poison("the decode queue did not drain");
  }
  hsa_queue_store_write_index_relaxed(q, i + 1);
  *index = i;
  return S4_OK;
}

// Publish a packet: everything but its first word is in place; the first
// word (header and setup) is stored last with release order.
void publish_packet(void *slot, uint32_t word0) {
  __atomic_store_n(reinterpret_cast<uint32_t *>(slot), word0, __ATOMIC_RELEASE);
}

// A barrier-AND packet in slot i of q: waits for deps[0 .. ndeps) (at most
// five), then signals `done` (may be null).
void barrier_packet(hsa_queue_t *q, uint64_t i, const hsa_signal_t *deps, uint32_t ndeps, hsa_signal_t done,
                    hsa_fence_scope_t acquire, hsa_fence_scope_t release) {
  auto *bp = reinterpret_cast<hsa_barrier_and_packet_t *>(static_cast<uint8_t *>(q->base_address) +
                                                           (i & (q->size - 1)) * 64);
  bp->reserved0 = 0;
  bp->reserved1 = 0;
  for (uint32_t j = 0; j < 5; ++j) bp->dep_signal[j].handle = j < ndeps ? deps[j].handle : 0;
  bp->reserved2 = 0;
  bp->completion_signal = done;
  publish_packet(bp, packet_header(HSA_PACKET_TYPE_BARRIER_AND, true, acquire, release));
}

}  // namespace

struct s4_aql_plan {
  // kArgStride bytes per dispatch, in device memory: every wave's preloaded
  // arguments come from HBM / L2 (in host memory each wave's start would
  // wait for a host-link round trip; tiny dispatches took 5.4 instead of
  // 4.7 us in the step)
  void *args = nullptr;
  struct Dispatch {
    hsa_kernel_dispatch_packet_t pkt;  // the packet, completion signal empty; its first word is published last
    uint32_t word0;                    // header and setup
    uint32_t list;                     // index of the list in the plan's input order
    uint32_t rank;                     // position key within its queue
  };
  std::vector<Dispatch> per_queue[kQueues];
  uint32_t count = 0, dispatches = 0;
  uint64_t ints = 0;
  bool lost = false;  // a run of this plan failed: its argument blocks may still be referenced
  std::atomic<uint32_t> pending{0};  // runs enqueued on a stream and not yet done
  std::atomic<int> async_rc{0};      // first failure of an enqueued run
  std::string async_msg;             // its message (under g_mu)
};

namespace {

// Default placement: largest-first assignment of launches to queues by
// bytes moved (plus a fixed cost per launch), then within each queue its
// largest and smallest remaining lists alternate, so small dispatches are
// issued while large kernels run.
void default_placement(const std::vector<DecodeLaunch> &launches, std::vector<uint32_t> *qof,
                       std::vector<uint32_t> *qrank) {
  std::vector<size_t> order(launches.size());
  for (size_t j = 0; j < order.size(); ++j) order[j] = j;
  auto bytes = [&](size_t j) { return uint64_t(launches[j].a.full_end - launches[j].a.first) * 512u + 4096u; };
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return bytes(x) > bytes(y); });
  uint64_t load[kQueues] = {};
  std::vector<size_t> mine[kQueues];
  for (size_t j : order) {
    uint32_t best = 0;
    for (uint32_t q = 1; q < kQueues; ++q)
      if (load[q] < load[best]) best = q;
    load[best] += bytes(j);
    (*qof)[j] = best;
    mine[best].push_back(j);
  }
  for (uint32_t q = 0; q < kQueues; ++q) {
    size_t lo = 0, hi = mine[q].size();
    uint32_t r = 0;
    while (lo < hi) {
      (*qrank)[mine[q][lo++]] = r++;
      if (lo < hi) (*qrank)[mine[q][--hi]] = r++;
    }
  }
}

// Write `steps` steps of the plan into the queues and ring their doorbells.
// Each queue: an opening barrier (step 0: no dependency, system-scope
// acquire; later steps: every queue's previous step), its dispatches, and a
// closing barrier that signals step_done[s][q].  sig: null, or one
// completion signal per dispatch per step (dispatch j of queue q in step s
// at sig[s * dispatches + offset of q + j]).  Caller holds g_mu.
int submit_steps(s4_aql_plan *plan, uint32_t steps, const hsa_signal_t *sig, Clock::time_point t0) {
  for (uint32_t s = 0; s < steps; ++s)
    for (uint32_t q = 0; q < kQueues; ++q) hsa_signal_store_relaxed(g_state.step_done[s][q], 1);
  for (uint32_t s = 0; s < steps; ++s) {
    uint32_t base = s * plan->dispatches;
    for (uint32_t q = 0; q < kQueues; ++q) {
      hsa_queue_t *qu = g_state.queues[q];
      auto *ring = static_cast<uint8_t *>(qu->base_address);
      const uint64_t mask = qu->size - 1;
      uint64_t i;
      int rc;
      if (s == 0) {
        rc = next_slot(qu, t0, &i);
        if (rc) return rc;
        barrier_packet(qu, i, nullptr, 0, hsa_signal_t{0}, HSA_FENCE_SCOPE_SYSTEM, HSA_FENCE_SCOPE_NONE);
      }
      // wait for every queue's previous step (a barrier packet waits on at
      // most five signals: as many packets as the queues need)
      for (uint32_t j0 = 0; s > 0 && j0 < kQueues; j0 += 5) {
        rc = next_slot(qu, t0, &i);
        if (rc) return rc;
        barrier_packet(qu, i, &g_state.step_done[s - 1][j0], std::min<uint32_t>(5, kQueues - j0), hsa_signal_t{0},
                       HSA_FENCE_SCOPE_AGENT, HSA_FENCE_SCOPE_NONE);
      }
      const auto &v = plan->per_queue[q];
      for (size_t j = 0; j < v.size(); ++j) {
        rc = next_slot(qu, t0, &i);
        if (rc) return rc;
        uint8_t *slot = ring + (i & mask) * 64;
        // independent lists: no barrier, no fences (the step's barriers carry them)
        std::memcpy(slot + 4, reinterpret_cast<const uint8_t *>(&v[j].pkt) + 4, 60);
        if (sig) reinterpret_cast<hsa_kernel_dispatch_packet_t *>(slot)->completion_signal = sig[base + j];
        publish_packet(slot, v[j].word0);
      }
      base += uint32_t(v.size());
      // this queue's part of the step is done once its kernels are
      rc = next_slot(qu, t0, &i);
      if (rc) return rc;
      barrier_packet(qu, i, nullptr, 0, g_state.step_done[s][q], HSA_FENCE_SCOPE_NONE,
                     s + 1 == steps ? HSA_FENCE_SCOPE_SYSTEM : HSA_FENCE_SCOPE_AGENT);
      hsa_signal_store_screlease(qu->doorbell_signal, hsa_signal_value_t(i));
    }
  }
  return S4_OK;
}

// Wait (bounded) until the last step is done on every queue.
int wait_steps(uint32_t steps, Clock::time_point t0) {
  for (uint32_t q = 0; q < kQueues; ++q)
    while (hsa_signal_wait_scacquire(g_state.step_done[steps - 1][q], HSA_SIGNAL_CONDITION_LT, 1, 1000000,
                                     HSA_WAIT_STATE_ACTIVE) >= 1) {
      if (g_queue_error.load()) return poison("a decode queue reported an error");
      if (seconds_since(t0) > kWaitLimitSeconds) return poison("decode did not complete in time");
    }
  return S4_OK;
}

int check_runnable(const s4_aql_plan *plan, uint32_t steps) {
  if (!plan || steps == 0 || steps > kMaxSteps) return fail(S4_EINVAL, "null plan or steps outside 1..64");
  if (!g_state.ready) return fail(S4_EINVAL, "dispatcher not set up");
  if (g_state.broken) return fail(S4_EDEVICE, "the per-list dispatcher was disabled by an earlier failure");
  for (uint32_t q = 0; q < kQueues; ++q)
    if (plan->per_queue[q].size() + 3 + kQueues / 5 >= g_state.queues[q]->size)
      return fail(S4_EINVAL, "a step needs more packets than a queue holds");
  return S4_OK;
}

// One run of `steps` steps, returning when they are complete.  Caller holds g_mu.
int run_locked(s4_aql_plan *plan, uint32_t steps, const hsa_signal_t *sig, uint64_t *elapsed_ns) {
  int rc = check_runnable(plan, steps);
  if (rc) return rc;
  const Clock::time_point t0 = Clock::now();
  rc = submit_steps(plan, steps, sig, t0);
  if (!rc) rc = wait_steps(steps, t0);
  if (rc) {
    plan->lost = true;
    return rc;
  }
  if (elapsed_ns)
    *elapsed_ns = uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count());
  return S4_OK;
}

struct Pending {
  s4_aql_plan *plan;
  uint32_t steps;
};

// Host function of a caller's stream: runs the plan and returns when it is
// complete, so the stream's later work is ordered after it.  No HIP call
// is made here (only HSA).
void run_from_stream(void *data) {
  Pending *pd = static_cast<Pending *>(data);
  s4_aql_plan *plan = pd->plan;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    const int rc = run_locked(plan, pd->steps, nullptr, nullptr);
    if (rc && plan->async_rc.load() == 0) {
      plan->async_msg = s4_last_error();
      plan->async_rc.store(rc);
    }
  }
  delete pd;
  plan->pending.fetch_sub(1);
}

}  // namespace

extern "C" {

int s4_aql_plan_create_placed(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps,
                              uint32_t count, const uint32_t *queue_of, const uint32_t *rank, s4_aql_plan **out) {
  if (!out || (count && (!lists || !d_outs || !caps))) return fail(S4_EINVAL, "null argument");
  *out = nullptr;
  for (uint32_t i = 0; i < count; ++i) {
    if (!lists[i] || (!d_outs[i] && lists[i]->n)) return fail(S4_EINVAL, "null list or output");
    if (caps[i] < lists[i]->n) return fail(S4_ERANGE, "cap < n for list " + std::to_string(i));
    if (reinterpret_cast<uintptr_t>(d_outs[i]) & 15u) return fail(S4_EINVAL, "outputs must be 16-byte aligned");
    if (is_patched(lists[i]->d)) return fail(S4_EINVAL, "the dispatcher decodes plain (unpatched) lists only");
    if (queue_of && queue_of[i] >= kQueues) return fail(S4_EINVAL, "queue index out of range");
  }
  int rc = ensure_device();
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  rc = ensure_queue();
  if (rc) return rc;
  int dev = 0;
  S4_HIP(hipGetDevice(&dev));
  if (dev != g_state.device) return fail(S4_EINVAL, "the dispatcher serves the device it was first used on");
  std::vector<DecodeLaunch> launches;
  std::vector<uint32_t> list_of;
  launches.reserve(count);
  for (uint32_t i = 0; i < count; ++i) {
    DecodeLaunch d;
    if (!plan_decode_range(lists[i]->d, 0, lists[i]->nb + (lists[i]->t ? 1u : 0u), d_outs[i], &d)) continue;
    rc = ensure_kernel(d.P);
    if (rc) return rc;
    launches.push_back(d);
    list_of.push_back(i);
  }
  s4_aql_plan *p = new (std::nothrow) s4_aql_plan;
  if (!p) return fail(S4_ENOMEM, "plan allocation failed");
  const size_t arg_bytes = size_t(kArgStride) * launches.size();
  std::vector<uint8_t> arg_image(arg_bytes, 0);
  if (!launches.empty() && hipMalloc(&p->args, arg_bytes) != hipSuccess) {
    delete p;
    return fail(S4_ENOMEM, "argument blocks allocation failed");
  }
  // the queue of every launch: given, or the default placement
  std::vector<uint32_t> qof(launches.size()), qrank(launches.size());
  if (queue_of) {
    for (size_t j = 0; j < launches.size(); ++j) {
      qof[j] = queue_of[list_of[j]];
      qrank[j] = rank ? rank[list_of[j]] : uint32_t(j);
    }
  } else {
    default_placement(launches, &qof, &qrank);
  }
  for (size_t j = 0; j < launches.size(); ++j) {
    const DecodeLaunch &d = launches[j];
    std::memcpy(arg_image.data() + j * kArgStride, &d.a, kDecodeArgBytes);
    uint8_t *a = static_cast<uint8_t *>(p->args) + j * kArgStride;
    const KernelInfo &k = g_state.kernels[slot_of(d.P)];
    s4_aql_plan::Dispatch dp;
    std::memset(&dp, 0, sizeof dp);
    dp.pkt.workgroup_size_x = 256;
    dp.pkt.workgroup_size_y = 1;
    dp.pkt.workgroup_size_z = 1;
    dp.pkt.grid_size_x = d.workgroups * 256u;
    dp.pkt.grid_size_y = 1;
    dp.pkt.grid_size_z = 1;
    dp.pkt.private_segment_size = 0;
    dp.pkt.group_segment_size = k.group;
    dp.pkt.kernel_object = k.object;
    dp.pkt.kernarg_address = a;
    dp.pkt.completion_signal.handle = 0;
    dp.word0 = packet_header(HSA_PACKET_TYPE_KERNEL_DISPATCH, false, HSA_FENCE_SCOPE_NONE, HSA_FENCE_SCOPE_NONE) |
               (uint32_t(1) << (16 + HSA_KERNEL_DISPATCH_PACKET_SETUP_DIMENSIONS));
    dp.list = list_of[j];
    dp.rank = qrank[j];
    p->per_queue[qof[j]].push_back(dp);
  }
  for (auto &v : p->per_queue)
    std::stable_sort(v.begin(), v.end(),
                     [](const s4_aql_plan::Dispatch &x, const s4_aql_plan::Dispatch &y) { return x.rank < y.rank; });
  if (arg_bytes) {
    const hipError_t e = hipMemcpy(p->args, arg_image.data(), arg_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(p->args);
      delete p;
      return hip_fail(e, "argument blocks upload");
    }
  }
  p->count = count;
  p->dispatches = uint32_t(launches.size());
  for (uint32_t i = 0; i < count; ++i) p->ints += lists[i]->n;
  *out = p;
  return S4_OK;
}

int s4_aql_plan_create(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps, uint32_t count,
                       s4_aql_plan **out) {
  return s4_aql_plan_create_placed(lists, d_outs, caps, count, nullptr, nullptr, out);
}

int s4_aql_plan_run(s4_aql_plan *plan, uint32_t steps, uint64_t *elapsed_ns) {
  std::lock_guard<std::mutex> lock(g_mu);
  return run_locked(plan, steps, nullptr, elapsed_ns);
}

int s4_aql_plan_profile(s4_aql_plan *plan, uint32_t steps, uint64_t *start_ns, uint64_t *end_ns,
                        uint64_t *elapsed_ns) {
  if (!plan || !start_ns || !end_ns) return fail(S4_EINVAL, "null argument");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = check_runnable(plan, steps);
  if (rc) return rc;
  const size_t nsig = size_t(steps) * plan->dispatches;
  std::vector<hsa_signal_t> sig(nsig);
  size_t made = 0;
  for (; made < nsig; ++made)
    // ordinary signals: a tool that intercepts the queues may complete them
    // from the host, which a GPU-only signal does not allow
    if (hsa_signal_create(1, 0, nullptr, &sig[made]) != HSA_STATUS_SUCCESS) break;
  auto destroy = [&]() {
    for (size_t j = 0; j < made; ++j) (void)hsa_signal_destroy(sig[j]);
  };
  if (made < nsig) {
    destroy();
    return fail(S4_ENOMEM, "profiling: signal creation failed");
  }
  uint32_t on = 0;
  for (; on < kQueues; ++on)
    if (hsa_amd_profiling_set_profiler_enabled(g_state.queues[on], 1) != HSA_STATUS_SUCCESS) break;
  if (on == kQueues) rc = run_locked(plan, steps, sig.data(), elapsed_ns);
  else rc = fail(S4_EDEVICE, "profiling could not be enabled on the dispatch queues");
  for (uint32_t q = 0; q < on; ++q) (void)hsa_amd_profiling_set_profiler_enabled(g_state.queues[q], 0);
  if (rc) return rc;  // the signals may still be referenced by packets: kept
  std::fill(start_ns, start_ns + size_t(steps) * plan->count, 0);
  std::fill(end_ns, end_ns + size_t(steps) * plan->count, 0);
  std::vector<hsa_amd_profiling_dispatch_time_t> t(nsig);
  uint64_t t0 = UINT64_MAX;
  for (size_t j = 0; j < nsig; ++j) {
    if (hsa_amd_profiling_get_dispatch_time(g_state.agent, sig[j], &t[j]) != HSA_STATUS_SUCCESS) {
      destroy();
      return fail(S4_EDEVICE, "profiling: dispatch time not available");
    }
    t0 = std::min(t0, t[j].start);
  }
  destroy();
  auto ns = [&](uint64_t tick) { return uint64_t(double(tick - t0) * 1e9 / double(g_state.ts_hz)); };
  for (uint32_t s = 0; s < steps; ++s) {
    size_t j = size_t(s) * plan->dispatches;
    for (uint32_t q = 0; q < kQueues; ++q)
      for (const auto &d : plan->per_queue[q]) {
        start_ns[size_t(s) * plan->count + d.list] = ns(t[j].start);
        end_ns[size_t(s) * plan->count + d.list] = ns(t[j].end);
        ++j;
      }
  }
  return S4_OK;
}

int s4_aql_plan_enqueue(s4_aql_plan *plan, uint32_t steps, void *stream) {
  {
    std::lock_guard<std::mutex> lock(g_mu);
    int rc = check_runnable(plan, steps);
    if (rc) return rc;
  }
  Pending *pd = new (std::nothrow) Pending{plan, steps};
  if (!pd) return fail(S4_ENOMEM, "enqueue: allocation failed");
  plan->pending.fetch_add(1);
  const hipError_t e = hipLaunchHostFunc(static_cast<hipStream_t>(stream), run_from_stream, pd);
  if (e != hipSuccess) {
    plan->pending.fetch_sub(1);
    delete pd;
    return hip_fail(e, "hipLaunchHostFunc");
  }
  return S4_OK;
}

int s4_aql_plan_status(s4_aql_plan *plan) {
  if (!plan) return fail(S4_EINVAL, "null plan");
  std::lock_guard<std::mutex> lock(g_mu);
  const int rc = plan->async_rc.load();
  if (rc) return fail(rc, "an enqueued run failed: " + plan->async_msg);
  return S4_OK;
}

int s4_aql_plan_layout(const s4_aql_plan *plan, uint32_t *queue_of, uint32_t *position) {
  if (!plan || !queue_of || !position) return fail(S4_EINVAL, "null argument");
  std::fill(queue_of, queue_of + plan->count, UINT32_MAX);
  std::fill(position, position + plan->count, UINT32_MAX);
  for (uint32_t q = 0; q < kQueues; ++q)
    for (size_t j = 0; j < plan->per_queue[q].size(); ++j) {
      queue_of[plan->per_queue[q][j].list] = q;
      position[plan->per_queue[q][j].list] = uint32_t(j);
    }
  return S4_OK;
}

int s4_aql_plan_free(s4_aql_plan *plan) {
  if (!plan) return S4_OK;
  if (plan->pending.load()) return fail(S4_EINVAL, "a run of the plan is still enqueued on a stream");
  std::lock_guard<std::mutex> lock(g_mu);
  // after a failed run, packets may still reference the argument blocks:
  // they are kept for the rest of the process
  if (plan->args && !plan->lost && !g_state.broken) (void)hipFree(plan->args);
  delete plan;
  return S4_OK;
}

}  // extern "C"

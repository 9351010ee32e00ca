// Per-list decode dispatched on queues of the library's own: one kernel
// dispatch packet per list (the k_decode launch s4_decode_lists_dev would
// make), written straight into HSA user queues.  The lists are spread over
// kQueues queues by bytes (largest first), each queue alternating its large
// and small lists; a queue's packets carry no barrier and no fence, since
// the lists of a step are independent; each queue ends a step with a
// barrier packet that signals, and starts the next
// one with a barrier packet waiting for every queue's signal, so steps do
// not overlap.  The kernels are the ones HIP loaded for this library, found
// through the AMD loader extension; their argument blocks are built once
// per plan in coherent pinned host memory.
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>
#include <hsa/hsa_ven_amd_loader.h>

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
constexpr uint32_t kQueues = 4;               // one queue processes about one dispatch per 4 us
static_assert(kQueues >= 1 && kQueues <= 16, "queues per device");
constexpr uint32_t kMaxSteps = 64;            // signals kept per queue

struct KernelInfo {
  uint64_t object = 0;
  uint32_t group = 0, priv = 0, kernarg = 0;
};

struct AqlState {
  bool ready = false;
  int device = -1;
  hsa_agent_t agent{};
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

// Reserve the next packet slot, waiting (bounded) until the queue has room.
int next_slot(hsa_queue_t *q, Clock::time_point t0, uint64_t *index) {
  const uint64_t i = hsa_queue_add_write_index_scacq_screl(q, 1);
  while (i - hsa_queue_load_read_index_scacquire(q) >= q->size) {
    if (g_queue_error.load()) return fail(S4_EDEVICE, "the decode queue reported an error");
    if (seconds_since(t0) > kWaitLimitSeconds) return fail(S4_EDEVICE, "the decode queue did not drain");
  }
  *index = i;
  return S4_OK;
}

}  // namespace

struct s4_aql_plan {
  void *args = nullptr;  // coherent pinned host memory, kArgStride bytes per dispatch
  struct Dispatch {
    uint64_t object;
    uint32_t group, grid;
    const void *args;
  };
  std::vector<Dispatch> per_queue[kQueues];
  uint64_t ints = 0;
};

extern "C" {

int s4_aql_plan_create(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps, uint32_t count,
                       s4_aql_plan **out) {
  if (!out || (count && (!lists || !d_outs || !caps))) return fail(S4_EINVAL, "null argument");
  *out = nullptr;
  for (uint32_t i = 0; i < count; ++i) {
    if (!lists[i] || (!d_outs[i] && lists[i]->n)) return fail(S4_EINVAL, "null list or output");
    if (caps[i] < lists[i]->n) return fail(S4_ERANGE, "cap < n for list " + std::to_string(i));
    if (reinterpret_cast<uintptr_t>(d_outs[i]) & 15u) return fail(S4_EINVAL, "outputs must be 16-byte aligned");
    if (is_patched(lists[i]->d)) return fail(S4_EINVAL, "the dispatcher decodes plain (unpatched) lists only");
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
  launches.reserve(count);
  for (uint32_t i = 0; i < count; ++i) {
    DecodeLaunch d;
    if (!plan_decode_range(lists[i]->d, 0, lists[i]->nb + (lists[i]->t ? 1u : 0u), d_outs[i], &d)) continue;
    rc = ensure_kernel(d.P);
    if (rc) return rc;
    launches.push_back(d);
  }
  s4_aql_plan *p = new (std::nothrow) s4_aql_plan;
  if (!p) return fail(S4_ENOMEM, "plan allocation failed");
  if (!launches.empty() && hipHostMalloc(&p->args, size_t(kArgStride) * launches.size(), hipHostMallocCoherent) !=
                               hipSuccess) {
    delete p;
    return fail(S4_ENOMEM, "argument blocks allocation failed");
  }
  // largest-first assignment of lists to queues by bytes moved
  std::vector<size_t> order(launches.size());
  for (size_t j = 0; j < order.size(); ++j) order[j] = j;
  std::sort(order.begin(), order.end(),
            [&](size_t x, size_t y) { return launches[x].a.full_end - launches[x].a.first >
                                             launches[y].a.full_end - launches[y].a.first; });
  uint64_t load[kQueues] = {};
  for (size_t j : order) {
    const DecodeLaunch &d = launches[j];
    uint8_t *a = static_cast<uint8_t *>(p->args) + j * kArgStride;
    std::memset(a, 0, kArgStride);
    std::memcpy(a, &d.a, kDecodeArgBytes);
    const KernelInfo &k = g_state.kernels[slot_of(d.P)];
    uint32_t best = 0;
    for (uint32_t q = 1; q < kQueues; ++q)
      if (load[q] < load[best]) best = q;
    load[best] += uint64_t(d.a.full_end - d.a.first) * 512u + 4096u;
    p->per_queue[best].push_back({k.object, k.group, d.workgroups * 256u, a});
  }
  // within a queue, alternate its largest and smallest remaining lists, so
  // small dispatches are issued while large kernels run
  for (auto &v : p->per_queue) {
    std::vector<s4_aql_plan::Dispatch> mixed;
    mixed.reserve(v.size());
    size_t lo = 0, hi = v.size();
    while (lo < hi) {
      mixed.push_back(v[lo++]);
      if (lo < hi) mixed.push_back(v[--hi]);
    }
    v.swap(mixed);
  }
  for (uint32_t i = 0; i < count; ++i) p->ints += lists[i]->n;
  *out = p;
  return S4_OK;
}

int s4_aql_plan_run(s4_aql_plan *plan, uint32_t steps, uint64_t *elapsed_ns) {
  if (!plan || steps == 0 || steps > kMaxSteps) return fail(S4_EINVAL, "null plan or steps outside 1..64");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_state.ready) return fail(S4_EINVAL, "dispatcher not set up");
  for (uint32_t q = 0; q < kQueues; ++q)
    if (plan->per_queue[q].size() + 2 + kQueues / 5 >= g_state.queues[q]->size)
      return fail(S4_EINVAL, "a step needs more packets than a queue holds");
  for (uint32_t s = 0; s < steps; ++s)
    for (uint32_t q = 0; q < kQueues; ++q) hsa_signal_store_relaxed(g_state.step_done[s][q], 1);
  const Clock::time_point t0 = Clock::now();
  for (uint32_t s = 0; s < steps; ++s) {
    for (uint32_t q = 0; q < kQueues; ++q) {
      hsa_queue_t *qu = g_state.queues[q];
      auto *ring = static_cast<uint8_t *>(qu->base_address);
      const uint64_t mask = qu->size - 1;
      uint64_t i;
      int rc;
      // wait for every queue's previous step (a barrier packet waits on
      // at most five signals: as many packets as the queues need)
      for (uint32_t j0 = 0; s > 0 && j0 < kQueues; j0 += 5) {
        rc = next_slot(qu, t0, &i);
        if (rc) return rc;
        auto *bp = reinterpret_cast<hsa_barrier_and_packet_t *>(ring + (i & mask) * 64);
        bp->reserved0 = 0;
        bp->reserved1 = 0;
        for (uint32_t j = 0; j < 5; ++j)
          bp->dep_signal[j].handle = j0 + j < kQueues ? g_state.step_done[s - 1][j0 + j].handle : 0;
        bp->reserved2 = 0;
        bp->completion_signal.handle = 0;
        __atomic_store_n(reinterpret_cast<uint32_t *>(bp),
                         uint32_t(packet_header(HSA_PACKET_TYPE_BARRIER_AND, true, HSA_FENCE_SCOPE_AGENT,
                                                HSA_FENCE_SCOPE_NONE)),
                         __ATOMIC_RELEASE);
      }
      for (const auto &d : plan->per_queue[q]) {
        rc = next_slot(qu, t0, &i);
        if (rc) return rc;
        auto *pk = reinterpret_cast<hsa_kernel_dispatch_packet_t *>(ring + (i & mask) * 64);
        pk->workgroup_size_x = 256;
        pk->workgroup_size_y = 1;
        pk->workgroup_size_z = 1;
        pk->reserved0 = 0;
        pk->grid_size_x = d.grid;
        pk->grid_size_y = 1;
        pk->grid_size_z = 1;
        pk->private_segment_size = 0;
        pk->group_segment_size = d.group;
        pk->kernel_object = d.object;
        pk->kernarg_address = const_cast<void *>(d.args);
        pk->reserved2 = 0;
        pk->completion_signal.handle = 0;
        // independent lists: no barrier, no fences (the step's barriers carry them)
        const uint32_t word =
            packet_header(HSA_PACKET_TYPE_KERNEL_DISPATCH, false, HSA_FENCE_SCOPE_NONE, HSA_FENCE_SCOPE_NONE) |
            (uint32_t(1) << (16 + HSA_KERNEL_DISPATCH_PACKET_SETUP_DIMENSIONS));
        __atomic_store_n(reinterpret_cast<uint32_t *>(pk), word, __ATOMIC_RELEASE);
      }
      // this queue's part of the step is done once its kernels are
      rc = next_slot(qu, t0, &i);
      if (rc) return rc;
      auto *ep = reinterpret_cast<hsa_barrier_and_packet_t *>(ring + (i & mask) * 64);
      ep->reserved0 = 0;
      ep->reserved1 = 0;
      for (auto &dep : ep->dep_signal) dep.handle = 0;
      ep->reserved2 = 0;
      ep->completion_signal.handle = g_state.step_done[s][q].handle;
      __atomic_store_n(reinterpret_cast<uint32_t *>(ep),
                       uint32_t(packet_header(HSA_PACKET_TYPE_BARRIER_AND, true, HSA_FENCE_SCOPE_NONE,
                                              s + 1 == steps ? HSA_FENCE_SCOPE_SYSTEM : HSA_FENCE_SCOPE_AGENT)),
                       __ATOMIC_RELEASE);
      hsa_signal_store_screlease(qu->doorbell_signal, hsa_signal_value_t(i));
    }
  }
  for (uint32_t q = 0; q < kQueues; ++q)
    while (hsa_signal_wait_scacquire(g_state.step_done[steps - 1][q], HSA_SIGNAL_CONDITION_LT, 1, 1000000,
                                     HSA_WAIT_STATE_ACTIVE) >= 1) {
      if (g_queue_error.load()) return fail(S4_EDEVICE, "a decode queue reported an error");
      if (seconds_since(t0) > kWaitLimitSeconds) return fail(S4_EDEVICE, "decode did not complete in time");
    }
  if (elapsed_ns)
    *elapsed_ns = uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count());
  return S4_OK;
}

int s4_aql_plan_free(s4_aql_plan *plan) {
  if (!plan) return S4_OK;
  if (plan->args) (void)hipHostFree(plan->args);
  delete plan;
  return S4_OK;
}

}  // extern "C"

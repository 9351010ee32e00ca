// Kernels and C-ABI entry points for single lists: upload with skip-index
// build, bulk decode (unpack + D4 prefix sum fused, Alg. 1), pairwise and
// k-way (SvS) decode-fused intersection.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include <hip/hip_ext.h>

#include "s4_kernels.h"

namespace s4 {

// ------------------------------------------------------------ device state

static std::mutex g_dev_mu;
static int g_dev_checked = -1;  // device id verified, -1 none
static int g_cus = 0;
static s4_tuning g_tuning = {256u, 8u, 4u, 32u, 4u};

int ensure_device() {
  int dev = -1;
  S4_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_dev_mu);
  if (g_dev_checked == dev) return S4_OK;
  hipDeviceProp_t prop;
  S4_HIP(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(S4_EDEVICE, std::string("libs4 is built for gfx950; device is ") + prop.gcnArchName);
  g_cus = prop.multiProcessorCount;
  g_dev_checked = dev;
  return S4_OK;
}

int cu_count() { return g_cus > 0 ? g_cus : 256; }
s4_tuning &tuning() { return g_tuning; }
static uint32_t tuning_decode_passes() {
  const uint32_t p = g_tuning.decode_passes;
  return (p == 1 || p == 2 || p == 4 || p == 8) ? p : 4u;
}


// Library-owned helper streams (default priority) and events used to fork
// independent launches off a caller's stream and join them back.
constexpr uint32_t kMaxStreams = 8;
struct StreamPool {
  hipStream_t streams[kMaxStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxStreams] = {};
};
static std::mutex g_pool_mu;
static std::map<int, StreamPool> g_pools;

// Caller holds g_pool_mu.
static int get_pool(StreamPool **out) {
  int dev = 0;
  S4_HIP(hipGetDevice(&dev));
  auto it = g_pools.find(dev);
  if (it == g_pools.end()) {
    StreamPool p;
    for (uint32_t s = 1; s < kMaxStreams; ++s) {
      S4_HIP(hipStreamCreateWithFlags(&p.streams[s], hipStreamNonBlocking));
      S4_HIP(hipEventCreateWithFlags(&p.join[s], hipEventDisableTiming));
    }
    S4_HIP(hipEventCreateWithFlags(&p.fork, hipEventDisableTiming));
    it = g_pools.emplace(dev, p).first;
  }
  *out = &it->second;
  return S4_OK;
}

// ----------------------------------------------------------------- kernels

// First pass of the skip index: every block decoded with a zero seed (one
// 16-lane row per block); its last four values are written into the seeds
// array.  Blocks are numbered globally over `nlists` lists; blk_prefix[l]
// is the first global block of list l.
__global__ __launch_bounds__(256) void k_block_sums(const DList *__restrict__ lists,
                                                    const uint64_t *__restrict__ blk_prefix, uint32_t nlists,
                                                    uint64_t total_blocks, uint4 *__restrict__ sums) {
  const uint32_t lane = lane_id();
  const uint64_t wave = uint64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const uint64_t g = wave * 4 + (lane >> 4);
  __shared__ __align__(16) uint32_t slices[4][4][kBlock];  // per wave, per row
  const bool active = g < total_blocks;
  uint32_t d0[4] = {0, 0, 0, 0}, d1[4] = {0, 0, 0, 0};
  uint32_t mode = S4_DELTA_D4;
  uint32_t lo = 0, k = 0;
  bool patched = false;
  if (active) {
    // list of block g: last l with blk_prefix[l] <= g
    uint32_t hi = nlists;
    while (hi - lo > 1) {
      uint32_t mid = (lo + hi) >> 1;
      if (blk_prefix[mid] <= g) lo = mid; else hi = mid;
    }
    const DList &L = lists[lo];
    k = uint32_t(g - blk_prefix[lo]);
    mode = L.mode;
    patched = is_patched(L);
    extract_row(L.payload + gbl(L.offs)[k], gbl(L.widths)[k], lane & 15u, d0, d1);
  }
  // rows of patched lists add their exceptions before the prefix
  if (__ballot(patched))
    patch_row(lists[lo], k, patched, lane & 15u, slices[threadIdx.x >> 6][lane >> 4], d0, d1);
  // rows of one wave may belong to lists of different forms: evaluate each
  // form the wave holds (row scans keep the rows apart)
  uint32_t x0[4], x1[4], y0[4], y1[4];
  const uint32_t zero[4] = {0, 0, 0, 0};
  for (uint32_t m = 0; m < 4; ++m) {
    const uint64_t any = __ballot(active && mode == m);
    if (!any) continue;
    prefix_deltas<true>(m, d0, d1, zero, y0, y1);
    if (mode == m) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        x0[j] = y0[j];
        x1[j] = y1[j];
      }
    }
  }
  if (active && (lane & 15u) == 15u) sums[g] = make_uint4(x1[0], x1[1], x1[2], x1[3]);
}

// Second pass: one wave per list turns the zero-seed last values s_k of
// every block into seeds (the last four values before block k) and bmax.
// Block k's true last values are s_k plus the carry of its form: each
// component's own running sum (D4), the running sum of component 3 (D1,
// DM: one chain), or of components 2 / 3 by parity (D2).  Each lane writes
// only its own block's entries (reading them first), so the pass works in
// place over the seeds array.
__global__ __launch_bounds__(256) void k_seed_scan(const DList *__restrict__ lists,
                                                   const uint64_t *__restrict__ blk_prefix, uint32_t nlists,
                                                   uint4 *__restrict__ seeds, uint32_t *__restrict__ bmax) {
  const uint32_t lane = lane_id();
  const uint32_t list = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (list >= nlists) return;
  const uint32_t mode = lists[list].mode;
  const uint64_t b0 = blk_prefix[list], b1 = blk_prefix[list + 1];
  uint32_t carry[4] = {0, 0, 0, 0};   // running sums of each component
  uint32_t last[4] = {0, 0, 0, 0};    // last four values of the previous chunk
  for (uint64_t base = b0; base < b1; base += 64) {
    const uint64_t g = base + lane;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (g < b1) v = seeds[g];
    const uint32_t sv[4] = {v.x, v.y, v.z, v.w};
    uint32_t inc[4], exc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      inc[j] = scan_wave64(sv[j]);
      exc[j] = carry[j] + inc[j] - sv[j];
    }
    uint32_t out[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t c;
      if (mode == S4_DELTA_D4) c = exc[j];
      else if (mode == S4_DELTA_D2) c = (j & 1) ? exc[3] : exc[2];
      else c = exc[3];
      out[j] = c + sv[j];
    }
    uint32_t prev[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      prev[j] = __shfl_up(out[j], 1);
      if (lane == 0) prev[j] = last[j];
    }
    if (g < b1) {
      seeds[g] = make_uint4(prev[0], prev[1], prev[2], prev[3]);
      bmax[g] = out[3];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      carry[j] += uint32_t(__builtin_amdgcn_readlane(int(inc[j]), 63));
      last[j] = uint32_t(__builtin_amdgcn_readlane(int(out[j]), 63));
    }
  }
}

// LDS words one wave uses to transpose one pass (4 blocks) of output.
constexpr uint32_t kPassWords = 4u * kBlock;

// Bulk decode by one wave: blocks [kbase, min(kbase + 4 P, full_end)) of L,
// block k written at out + 128 (k - first).
//  1. Lane l reads the width of block kbase + l; a wave scan of 4 b gives
//     every block's payload offset from the one offset of block kbase, so
//     the payload loads of all P passes are independent and issue together
//     (the passes are unrolled).
//  2. Each pass decodes 4 consecutive blocks (one 16-lane row each); the D4
//     prefix runs across the whole wave (row scans joined by row
//     broadcasts) and is carried from pass to pass in registers, so only
//     the wave's first block reads a seed from the skip index.
//  3. The pass's 512 values go through the wave's LDS slice so that each
//     store instruction writes 1 KiB of contiguous output (lane l stores
//     values 4l .. 4l + 3 of each half): whole cache lines per instruction.
//  (Patched lists, PATCHED: before its prefix each pass's deltas go through
//  the same LDS slice once, where the rows add their blocks' exceptions.)
template <int P, uint32_t MODE, bool PATCHED, bool PIPE>
__device__ __forceinline__ void decode_wave_form(const DList &L, uint32_t first, uint32_t full_end, uint32_t kbase,
                                                 uint32_t *__restrict__ out, uint32_t *__restrict__ tb) {
  static_assert(P >= 1 && P <= 16, "4 P blocks per wave must fit 64 lanes");
  const uint32_t lane = lane_id();
  const uint32_t row = lane >> 4, i = lane & 15u;
  kbase = uniform(kbase);
  const uint32_t kl = kbase + lane;
  const bool vl = lane < 4u * P && kl < full_end;
  // The block offset, the seeds and the widths are independent loads: all
  // three are issued before any is waited for.  Every lane loads an
  // in-range width (block kbase exists) and drops it when not its own, so
  // no branch around the load makes the others wait for it.
  const uint32_t base_off = gbl(L.offs)[kbase];
  const uint4 s = gbl(L.seeds)[kbase];
  const uint32_t wraw = gbl(L.widths)[vl ? kl : kbase];
  const uint32_t bl = vl ? wraw : 0u;
  const uint32_t wl = 4u * bl;
  const uint32_t ol = base_off + scan_wave64(wl) - wl;
  uint32_t c[4] = {s.x, s.y, s.z, s.w};
  // Rows past the range's last block read that last block instead, so every
  // row's loads are unconditional (their values only reach rows and carries
  // after the range, which are never stored).
  const uint32_t last = full_end - 1u - kbase;
  auto width_of = [&](int p) { return uint32_t(__shfl(int(bl), int(min(4u * p + row, last)))); };
  auto row_of = [&](int p, uint32_t b) {
    return load_row(L.payload + uint32_t(__shfl(int(ol), int(min(4u * p + row, last)))), b, i);
  };
  // a row's exception record for pass p (patched lists), read a pass
  // ahead with the row's payload; clamped like the rows
  auto rec_of = [&](int p) { return gbl(exc_records(L))[kbase + min(4u * p + row, last)]; };
  // one pass: patch, scan (carry across passes in c), transpose, store
  auto pass = [&](int p, uint32_t d0[4], uint32_t d1[4], const uint4 x) {
    const uint32_t k0 = kbase + 4u * p;
    if (PATCHED) patch_row_rec(L, x, k0 + row < full_end, i, tb + row * kBlock, d0, d1);
    uint32_t x0[4], x1[4];
    prefix_form<false, MODE>(d0, d1, c, x0, x1);
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = uint32_t(__builtin_amdgcn_readlane(int(x1[j]), 63));
    u32x4 *t = reinterpret_cast<u32x4 *>(tb + row * kBlock + 8u * i);
    t[0] = u32x4{x0[0], x0[1], x0[2], x0[3]};
    t[1] = u32x4{x1[0], x1[1], x1[2], x1[3]};
    wave_sync();
    const u32x4 y0 = reinterpret_cast<const u32x4 *>(tb)[lane];
    const u32x4 y1 = reinterpret_cast<const u32x4 *>(tb)[64 + lane];
    wave_sync();
    uint32_t *dst = out + uint64_t(k0 - first) * kBlock + 4u * lane;
    if (k0 + (lane >> 5) < full_end) store4(dst, y0);
    if (k0 + 2u + (lane >> 5) < full_end) store4(dst + 256, y1);
  };
  if constexpr (!PIPE) {
    // all 4 P rows' loads in flight at once (most memory parallelism per
    // wave, at 4 P x 8 registers of deltas)
    uint32_t d0[P][4], d1[P][4];
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const uint32_t b = width_of(p);
      unpack_row(row_of(p, b), b, i, d0[p], d1[p]);
    }
#pragma unroll
    for (int p = 0; p < P; ++p) pass(p, d0[p], d1[p], make_uint4(0, 0, 0, 0));
  } else {
    // each pass's row loaded while the previous one is decoded: two passes
    // in flight, few registers, more waves resident (the patched kernels,
    // whose passes also wait on LDS, gain more from waves than from
    // loads in flight)
    uint32_t bcur = width_of(0), bnext = 0;
    RowWords cur = row_of(0, bcur), next;
    uint4 xcur = PATCHED ? rec_of(0) : make_uint4(0, 0, 0, 0), xnext = xcur;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (p + 1 < P) {
        bnext = width_of(p + 1);
        next = row_of(p + 1, bnext);
        if (PATCHED) xnext = rec_of(p + 1);
      }
      uint32_t d0[4], d1[4];
      unpack_row(cur, bcur, i, d0, d1);
      pass(p, d0, d1, xcur);
      if (p + 1 < P) {
        cur = next;
        bcur = bnext;
        xcur = xnext;
      }
    }
  }
}

// Dispatch once per wave on the list's differential form and on patching,
// so each variant of the unrolled passes is straight-line code.  PK: the
// kernel is instantiated for work that may hold patched lists; it decodes
// every list with pipelined rows (see decode_wave_form), the plain kernels
// load all rows at once.
template <int P, bool PATCHED, bool PIPE>
__device__ __forceinline__ void decode_wave_as(const DList &L, uint32_t first, uint32_t full_end, uint32_t kbase,
                                               uint32_t *__restrict__ out, uint32_t *__restrict__ tb) {
  switch (uniform(L.mode)) {
    case S4_DELTA_D1: decode_wave_form<P, S4_DELTA_D1, PATCHED, PIPE>(L, first, full_end, kbase, out, tb); break;
    case S4_DELTA_D2: decode_wave_form<P, S4_DELTA_D2, PATCHED, PIPE>(L, first, full_end, kbase, out, tb); break;
    case S4_DELTA_DM: decode_wave_form<P, S4_DELTA_DM, PATCHED, PIPE>(L, first, full_end, kbase, out, tb); break;
    default: decode_wave_form<P, S4_DELTA_D4, PATCHED, PIPE>(L, first, full_end, kbase, out, tb); break;
  }
}
template <int P, bool PK>
__device__ __forceinline__ void decode_wave(const DList &L, uint32_t first, uint32_t full_end, uint32_t kbase,
                                            uint32_t *__restrict__ out, uint32_t *__restrict__ tb) {
  if (PK && is_patched(L))
    decode_wave_as<P, true, true>(L, first, full_end, kbase, out, tb);
  else
    decode_wave_as<P, false, PK>(L, first, full_end, kbase, out, tb);
}

__device__ __forceinline__ void copy_tail(const DList &L, uint32_t *__restrict__ dst) {
  const uint32_t lane = lane_id();
  if (lane < L.t) gbl_out(dst)[lane] = gbl(L.tail)[lane];
  if (lane + 64 < L.t) gbl_out(dst)[lane + 64] = gbl(L.tail)[lane + 64];
}

// Bulk decode of blocks [first, full_end) of one list, then its raw tail
// when `form` has kDecodeTail (the range then ends at the last full block,
// so the tail goes right after it): waves [0, block_waves) decode 4
// passes-worth of blocks each, wave block_waves copies the tail.  The list
// comes as scalar arguments, those a wave needs first leading, so that they
// arrive preloaded in scalar registers and a wave's first loads do not wait
// for an argument fetch; the tail pointer and nb (needed by the tail wave
// and by patched lists only) follow.  form = differential form |
// kDecodePatched if patched | kDecodeTail | t << 16.
// PK: instantiated for patched lists (see decode_wave).  The plain kernels
// of 4 or more passes are held to 5 waves per SIMD: with more, measured on
// the bulk workload, they streamed slower (all 4 P rows' loads in flight
// per wave is worth more than further waves).
constexpr uint32_t kDecodePatched = 1u << 8, kDecodeTail = 1u << 9;
template <int P, bool PK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, (P >= 4 && !PK) ? 5 : 8))) void k_decode(const uint8_t *widths, const uint32_t *offs, const uint4 *seeds,
                                                const uint32_t *payload, uint32_t *__restrict__ out, uint32_t first,
                                                uint32_t full_end, uint32_t block_waves, uint32_t form,
                                                const uint32_t *tail, uint32_t nb) {
  __shared__ __align__(16) uint32_t stage[4][kPassWords];
  DList L;
  L.widths = widths;
  L.offs = offs;
  L.payload = payload;
  L.bmax = nullptr;
  L.seeds = seeds;
  L.tail = tail;
  L.n = 0;  // not used by the decode
  L.nb = nb;
  L.t = form >> 16;
  L.mode = form & 0xffu;
  L.aux = (form & kDecodePatched) ? 1u : 0u;
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t wave = blockIdx.x * 4u + w;  // always launched with 4 waves per group
  if (wave >= block_waves) {
    if (wave == block_waves && (form & kDecodeTail)) copy_tail(L, out + uint64_t(full_end - first) * kBlock);
    return;
  }
  decode_wave<P, PK>(L, first, full_end, first + wave * 4u * P, out, stage[w]);
}

// Multi-list decode in one launch: wave w decodes for list wave_list[w];
// wave_prefix[l] is the first wave of list l.  Within a list the waves are
// laid out as in k_decode (blocks, then one tail wave when the list has a
// tail).  PK: instantiated for plans that hold patched lists.
template <int P, bool PK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, (P >= 4 && !PK) ? 5 : 8))) void k_decode_multi(const DList *__restrict__ lists,
                                                      uint32_t *const *__restrict__ outs,
                                                      const uint32_t *__restrict__ wave_prefix,
                                                      const uint32_t *__restrict__ wave_list, uint32_t waves) {
  __shared__ __align__(16) uint32_t stage[4][kPassWords];
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t wave = uniform(blockIdx.x * (blockDim.x >> 6) + w);
  if (wave >= waves) return;
  const uint32_t l = uniform(wave_list[wave]);
  const DList L = cst(lists)[l];
  uint32_t *out = cst(outs)[l];
  const uint32_t local = wave - cst(wave_prefix)[l];
  const uint32_t block_waves = (L.nb + 4 * P - 1) / (4 * P);
  if (local >= block_waves) {
    copy_tail(L, out + uint64_t(L.nb) * kBlock);
    return;
  }
  decode_wave<P, PK>(L, 0, L.nb, local * 4u * P, out, stage[w]);
}

// Busy-wait on the constant-rate device clock for `ticks` ticks.
__global__ void k_spin(uint64_t ticks) {
  const uint64_t t0 = wall_clock64();
  while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

// Lists of one conjunction passed by value (the shortest first).
struct ChainArgs {
  DList f[kMaxTerms];
  uint32_t nf;  // lists after the short side
};

// Scratch of one single-launch intersection run: a ticket word, then per
// 128-value chunk of the short side a 64-bit scan tag and two counts.
// Every run carries its own epoch, so nothing needs clearing between runs.
struct RunScratch {
  uint64_t *ticket;  // (low 32 bits of the run's epoch) << 32 | chunks taken
  uint64_t *tag;     // [items] epoch << 2 | flag: 1 agg set, 2 incl set, 3 poisoned
  uint32_t *agg;     // [items] survivors of the chunk
  uint32_t *incl;    // [items] survivors of chunks 0 .. i
  uint32_t items_cap;
};

// Bound on the look-back's waits (each ends with a short sleep): a guard
// that turns a run that cannot finish into a reported failure, never a hang.
constexpr uint32_t kRunSpins = 1u << 22;
// *d_count of a run whose look-back gave up.
constexpr uint64_t kRunFailed = ~0ull;

// The wave's chunk (lane 0 asks): chunks are numbered in the order waves
// start, so every chunk a wave waits for belongs to a wave already running.
// The counter restarts at the first ticket of a new epoch.
__device__ uint32_t run_ticket(uint64_t *ticket, uint32_t e32) {
  for (;;) {
    uint64_t v = __hip_atomic_load(ticket, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (uint32_t(v >> 32) == e32)
      return uint32_t(__hip_atomic_fetch_add(ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (__hip_atomic_compare_exchange_strong(ticket, &v, (uint64_t(e32) << 32) | 1u, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return 0;
  }
}

// Decoupled look-back over the run's tags: publish this chunk's count, read
// the tags of its 64 nearest predecessors at once, and sum counts back to
// the nearest chunk whose inclusive prefix is known; then publish this
// chunk's inclusive prefix.  A chunk that waited too long publishes
// "poisoned" instead, and so does every chunk whose walk reaches one, so a
// failure reaches the run's last chunk and every wave ends.
__device__ uint32_t run_lookback(const RunScratch &s, uint32_t item, uint64_t epoch, uint32_t cnt, bool &ok) {
  const uint32_t lane = lane_id();
  const uint64_t tag_a = (epoch << 2) | 1u, tag_p = (epoch << 2) | 2u, tag_x = (epoch << 2) | 3u;
  if (lane == 0) {
    if (item == 0) {
      __hip_atomic_store(s.incl, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(s.tag, tag_p, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_store(s.agg + item, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(s.tag + item, tag_a, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  ok = true;
  if (item == 0) return 0;
  uint32_t excl = 0, spins = 0;
  bool poisoned = false;
  int64_t base = int64_t(item) - 1;
  for (;;) {
    const int64_t j = base - int64_t(lane);
    uint64_t t = tag_p;  // before the first chunk: inclusive prefix 0
    if (j >= 0) t = __hip_atomic_load(s.tag + j, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t is_t = __ballot(t == tag_p || t == tag_x);
    const uint64_t ready = __ballot(t == tag_p || t == tag_x || t == tag_a);
    // lanes through the nearest terminal word (all 64 if none)
    const uint64_t nearest = is_t & (~is_t + 1);
    const uint64_t need = is_t ? (nearest << 1) - 1 : ~0ull;
    if ((ready & need) == need) {
      if (__ballot(t == tag_x) & nearest) {
        poisoned = true;
        break;
      }
      uint32_t v = 0;
      if (((need >> lane) & 1) && j >= 0)
        v = __hip_atomic_load(t == tag_a ? s.agg + j : s.incl + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      excl += wave_sum(v);
      if (is_t) break;
      base -= 64;
    } else if (++spins > kRunSpins) {
      poisoned = true;
      break;
    } else {
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (lane == 0) {
    if (!poisoned) __hip_atomic_store(s.incl + item, excl + cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(s.tag + item, poisoned ? tag_x : tag_p, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  ok = !poisoned;
  return excl;
}

// One launch per conjunction: each wave takes a 128-value chunk of r and
// carries it through the other lists (decode-fused SvS), finds its output
// offset by look-back and writes its survivors to their final place; the
// last chunk writes the total to *count (kRunFailed if the run gave up).
// r is a compressed list or raw values whose length lives on the device;
// chunks past the end of r count 0.
template <int WAVES, uint32_t FEAT>
__global__ __launch_bounds__(WAVES * 64) void k_chain(DList rl, const uint32_t *__restrict__ r_raw,
                                                      const uint64_t *__restrict__ r_len_dev, ChainArgs args,
                                                      RunScratch rs, uint64_t epoch, uint32_t *__restrict__ out,
                                                      uint64_t *__restrict__ count, uint32_t gallop_blocks) {
  __shared__ ItemLds lds[WAVES];
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  uint32_t ticket = 0;
  if (lane == 0) ticket = run_ticket(rs.ticket, uint32_t(epoch));
  const uint32_t item = uniform(uint32_t(__shfl(int(ticket), 0)));
  if (item >= rs.items_cap) return;
  RSide r;
  r.L = rl;
  r.raw = r_raw;
  // raw values: rl.n holds the host's bound on their count
  r.len = r_raw ? min(*r_len_dev, rl.n) : rl.n;
  const uint64_t n_items = (r.len + kBlock - 1) / kBlock;
  Traffic tr;
  uint32_t cnt = 0;
  uint32_t hint = 0;  // one chunk per wave: no previous chunk to start from
  if (item < n_items)
    cnt = chain_chunk<FEAT>(r, item, args.f[0], [&](uint32_t j) -> const DList & { return args.f[j]; }, args.nf,
                            lds[w], gallop_blocks, tr, hint);
  bool ok = true;
  const uint32_t excl = run_lookback(rs, item, epoch, cnt, ok);
  if (ok) {
    if (lane < cnt) gbl_out(out)[uint64_t(excl) + lane] = lds[w].r[lane];
    if (lane + 64 < cnt) gbl_out(out)[uint64_t(excl) + 64 + lane] = lds[w].r[lane + 64];
  }
  if (item + 1 == rs.items_cap && lane == 0) *gbl_out(count) = ok ? uint64_t(excl) + cnt : kRunFailed;
}

// Exclusive scan of counts[n] in tiles of 1024 (256 threads x 4): local
// offsets to excl[], tile totals to tile_sums[].
__global__ __launch_bounds__(256) void k_scan_tiles(const uint32_t *__restrict__ counts, uint32_t n,
                                                    uint32_t *__restrict__ excl, uint32_t *__restrict__ tile_sums) {
  __shared__ uint32_t wsum[4];
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  const uint64_t base = uint64_t(blockIdx.x) * 1024 + threadIdx.x * 4u;
  uint32_t v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = (base + e < n) ? counts[base + e] : 0u;
  const uint32_t local = v[0] + v[1] + v[2] + v[3];
  const uint32_t inc = scan_wave64(local);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0;
  for (uint32_t q = 0; q < w; ++q) off += wsum[q];
  uint32_t run = off + inc - local;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (base + e < n) excl[base + e] = run;
    run += v[e];
  }
  if (threadIdx.x == 255) tile_sums[blockIdx.x] = off + inc;
}

// Exclusive scan of the tile totals in place (one workgroup); the grand
// total goes to *total.
__global__ __launch_bounds__(256) void k_scan_top(uint32_t *__restrict__ tile_sums, uint32_t ntiles,
                                                  uint64_t *__restrict__ total) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t carry_s;
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (uint32_t base = 0; base < ntiles; base += 256) {
    const uint32_t idx = base + threadIdx.x;
    const uint32_t v = idx < ntiles ? tile_sums[idx] : 0u;
    const uint32_t inc = scan_wave64(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = carry_s;
    for (uint32_t q = 0; q < w; ++q) off += wsum[q];
    if (idx < ntiles) tile_sums[idx] = off + inc - v;
    __syncthreads();
    if (threadIdx.x == 255) carry_s = off + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry_s;
}

// Ordered gather of every chunk's matches into out[]: a wave per 64
// chunks, each lane reading one chunk's count; the wave then copies the
// chunks that have matches, one after another (most chunks of a batch
// have none, so a wave per chunk would mostly start and stop).
__global__ __launch_bounds__(256) void k_compact(const uint32_t *__restrict__ stage,
                                                 const uint32_t *__restrict__ counts,
                                                 const uint32_t *__restrict__ excl,
                                                 const uint32_t *__restrict__ tile_sums, uint32_t n,
                                                 uint32_t *__restrict__ out) {
  const uint32_t lane = lane_id();
  const uint32_t base = (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 64u;
  if (base >= n) return;
  const uint32_t item = base + lane;
  const uint32_t cnt = item < n ? counts[item] : 0u;
  uint64_t off = 0;
  if (cnt) off = uint64_t(excl[item]) + tile_sums[item >> 10];
  for (uint64_t m = __ballot(cnt != 0); m; m &= m - 1) {
    const int l = __builtin_ctzll(m);
    const uint32_t c = uint32_t(__builtin_amdgcn_readlane(int(cnt), l));
    const uint64_t o = uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(off)), l))) |
                       (uint64_t(uint32_t(__builtin_amdgcn_readlane(int(uint32_t(off >> 32)), l))) << 32);
    const uint32_t *src = stage + uint64_t(base + uint32_t(l)) * kBlock;
    if (lane < c) out[o + lane] = src[lane];
    if (lane + 64 < c) out[o + 64 + lane] = src[lane + 64];
  }
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) { *p = v; }
__global__ void k_copy_u64(uint64_t *dst, const uint64_t *src) { *dst = *src; }

// ------------------------------------------------------------ arena build

static void plan_arena(Upload &u) {
  const size_t L = u.views.size();
  u.blk_prefix.assign(L + 1, 0);
  u.pay_base.assign(L, 0);
  u.tail_base.assign(L, 0);
  for (size_t i = 0; i < L; ++i) {
    const StreamView &v = u.views[i];
    u.blk_prefix[i + 1] = u.blk_prefix[i] + v.nb;
    u.pay_base[i] = u.total_words;
    u.total_words += v.pw;
    // each list's tail region starts 16-byte aligned; a patched list's
    // exception records and data follow its tail there
    u.tail_base[i] = u.total_tail;
    u.total_tail += (v.t + 3) & ~uint64_t(3);
    if (v.patched()) u.total_tail += 4ull * v.nb + (v.x_positions + 3) / 4 + v.x_array_words;
  }
  u.total_blocks = u.blk_prefix[L];
  ArenaLayout &a = u.lay;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  a.desc_off = take(sizeof(DList) * L);
  a.blkpre_off = take(sizeof(uint64_t) * (L + 1) + sizeof(uint64_t) * L);
  a.widths_off = take(u.total_blocks);
  a.offs_off = take(4 * u.total_blocks);
  a.bmax_off = take(4 * u.total_blocks);
  a.seeds_off = take(16 * u.total_blocks);
  a.tail_off = take(4 * u.total_tail);
  a.payload_off = take(4 * u.total_words + kPayloadPadBytes);
  a.total = off;
}

static DList make_desc(const Upload &u, size_t i, char *base) {
  const ArenaLayout &a = u.lay;
  DList d;
  const uint64_t b0 = u.blk_prefix[i];
  d.widths = reinterpret_cast<const uint8_t *>(base + a.widths_off) + b0;
  d.offs = reinterpret_cast<const uint32_t *>(base + a.offs_off) + b0;
  d.bmax = reinterpret_cast<const uint32_t *>(base + a.bmax_off) + b0;
  d.seeds = reinterpret_cast<const uint4 *>(base + a.seeds_off) + b0;
  d.payload = reinterpret_cast<const uint32_t *>(base + a.payload_off) + u.pay_base[i];
  d.tail = reinterpret_cast<const uint32_t *>(base + a.tail_off) + u.tail_base[i];
  d.n = u.views[i].n;
  d.nb = u.views[i].nb;
  d.t = u.views[i].t;
  d.mode = (u.views[i].flags >> 1) & 3u;
  d.aux = u.views[i].patched() ? 1u : 0u;
  return d;
}

// Host image of a patched list's exceptions: one record per block (count,
// d = b - b', b'; byte offset of its positions; word offset of its page's
// array for d; index of its first exception there), the positions bytes,
// then every page's arrays, each followed by one zero word.
static void fill_exceptions(const StreamView &v, uint4 *rec, uint8_t *xd) {
  uint64_t pos = 0;                                  // bytes of positions so far
  uint64_t arr = (v.x_positions + 3) / 4;            // words: arrays follow the positions
  const uint8_t *p = v.pages;
  for (uint64_t k0 = 0; k0 < v.nb; k0 += kPage) {
    const uint64_t k1 = std::min<uint64_t>(v.nb, k0 + kPage);
    uint32_t meta_len;
    std::memcpy(&meta_len, p, 4);
    const uint8_t *m = p + 4;
    const uint8_t *q = m + align_up(meta_len, 4);
    uint32_t present;
    std::memcpy(&present, q, 4);
    q += 4;
    uint64_t at[33] = {0};
    for (uint32_t d = 1; d <= 32; ++d) {
      if (!((present >> (d - 1)) & 1u)) continue;
      uint32_t count;
      std::memcpy(&count, q, 4);
      const uint64_t words = uint64_t(d) * ((count + 31u) / 32u);
      at[d] = arr;
      std::memcpy(xd + 4 * arr, q + 4, 4 * words);
      arr += words + 1;
      q += 4 + 4 * words;
    }
    uint32_t used[33] = {0};
    uint64_t o = 0;
    for (uint64_t k = k0; k < k1; ++k) {
      const uint32_t b = m[o], c = m[o + 1], bp = v.widths[k], d = b - bp;
      o += 2;
      rec[k] = make_uint4(c | (d << 8) | (bp << 16), uint32_t(pos), uint32_t(at[d]), used[d]);
      std::memcpy(xd + pos, m + o, c);
      pos += c;
      used[d] += c;
      o += c;
    }
    p = q;
  }
}

// Copy the parsed streams into a new device arena and build the skip
// index.  Synchronous with respect to `stream` only through the staging copy.
int build_arena(Upload &u, hipStream_t stream, void **arena_out, std::vector<DList> *descs) {
  int rc = ensure_device();
  if (rc) return rc;
  plan_arena(u);
  const ArenaLayout &a = u.lay;
  const size_t L = u.views.size();
  char *dev = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&dev), a.total);
  if (e != hipSuccess) return fail(S4_ENOMEM, "hipMalloc of " + std::to_string(a.total) + " bytes failed");
  // host image of everything except bmax / seeds
  std::vector<char> img;
  try {
    img.assign(a.total, 0);
  } catch (...) {
    (void)hipFree(dev);
    return fail(S4_ENOMEM, "host staging allocation failed");
  }
  descs->resize(L);
  for (size_t i = 0; i < L; ++i) (*descs)[i] = make_desc(u, i, dev);
  std::memcpy(img.data() + a.desc_off, descs->data(), sizeof(DList) * L);
  std::memcpy(img.data() + a.blkpre_off, u.blk_prefix.data(), sizeof(uint64_t) * (L + 1));
  std::memcpy(img.data() + a.blkpre_off + sizeof(uint64_t) * (L + 1), u.pay_base.data(), sizeof(uint64_t) * L);
  for (size_t i = 0; i < L; ++i) {
    const StreamView &v = u.views[i];
    const uint64_t b0 = u.blk_prefix[i];
    std::memcpy(img.data() + a.widths_off + b0, v.widths, v.nb);
    uint32_t *offs = reinterpret_cast<uint32_t *>(img.data() + a.offs_off) + b0;
    uint32_t run = 0;
    for (uint32_t k = 0; k < v.nb; ++k) {
      offs[k] = run;
      run += 4u * v.widths[k];
    }
    std::memcpy(img.data() + a.payload_off + 4 * u.pay_base[i], v.payload, 4 * v.pw);
    std::memcpy(img.data() + a.tail_off + 4 * u.tail_base[i], v.tail, 4 * size_t(v.t));
    if (v.patched()) {
      // records and data right after the tail, as exc_records / exc_data expect
      uint32_t *tl = reinterpret_cast<uint32_t *>(img.data() + a.tail_off) + u.tail_base[i] + ((v.t + 3) & ~3u);
      fill_exceptions(v, reinterpret_cast<uint4 *>(tl), reinterpret_cast<uint8_t *>(tl + 4ull * v.nb));
    }
  }
  e = hipMemcpyAsync(dev, img.data(), a.total, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return hip_fail(e, "arena upload");
  }
  if (u.total_blocks) {
    const uint64_t waves = (u.total_blocks + 3) / 4;
    const uint64_t groups = (waves + 3) / 4;
    hipLaunchKernelGGL(k_block_sums, dim3(uint32_t(groups)), dim3(256), 0, stream,
                       reinterpret_cast<const DList *>(dev + a.desc_off),
                       reinterpret_cast<const uint64_t *>(dev + a.blkpre_off), uint32_t(L), u.total_blocks,
                       reinterpret_cast<uint4 *>(dev + a.seeds_off));
    hipLaunchKernelGGL(k_seed_scan, dim3(uint32_t((L + 3) / 4)), dim3(256), 0, stream,
                       reinterpret_cast<const DList *>(dev + a.desc_off),
                       reinterpret_cast<const uint64_t *>(dev + a.blkpre_off), uint32_t(L),
                       reinterpret_cast<uint4 *>(dev + a.seeds_off), reinterpret_cast<uint32_t *>(dev + a.bmax_off));
    e = hipGetLastError();
    if (e != hipSuccess) {
      (void)hipFree(dev);
      return hip_fail(e, "skip index build");
    }
  }
  *arena_out = dev;
  return S4_OK;
}

// ---------------------------------------------------------- pair pipeline

// Layout of a run's scratch when its short side has at most cap_r values
// (bytes needed; fills *rs when base is given).
static size_t run_scratch_layout(uint64_t cap_r, char *base, RunScratch *rs) {
  const uint64_t items = (cap_r + kBlock - 1) / kBlock;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  const size_t tk = take(8), tg = take(8 * items), ag = take(4 * items), in = take(4 * items);
  if (rs) {
    rs->ticket = reinterpret_cast<uint64_t *>(base + tk);
    rs->tag = reinterpret_cast<uint64_t *>(base + tg);
    rs->agg = reinterpret_cast<uint32_t *>(base + ag);
    rs->incl = reinterpret_cast<uint32_t *>(base + in);
    rs->items_cap = uint32_t(items);
  }
  return off;
}

// Epochs of runs, process-wide: a run's tags never match those an earlier
// run left in the same scratch.  Epochs whose low 32 bits are zero are
// skipped, so a zeroed ticket word never looks current.
static std::atomic<uint64_t> g_run_epoch{0};
static uint64_t next_run_epoch() {
  uint64_t e;
  do e = g_run_epoch.fetch_add(1, std::memory_order_relaxed) + 1;
  while (uint32_t(e) == 0);
  return e;
}

// Lists given as handles are never bitmaps; the patched instantiation is
// used only when a patched list takes part.
template <int WAVES>
static void launch_chain_w(const DList &r, const uint32_t *r_raw, const uint64_t *r_len, const ChainArgs &args,
                           const RunScratch &rs, uint32_t *d_out, uint64_t *d_count, hipStream_t stream) {
  const uint32_t groups = std::max<uint32_t>(1, (rs.items_cap + WAVES - 1) / WAVES);
  bool patched = !r_raw && is_patched(r);
  for (uint32_t j = 0; j < args.nf; ++j) patched |= is_patched(args.f[j]);
  const uint64_t epoch = next_run_epoch();
  const uint32_t gb = std::min(tuning().gallop_blocks, kMaxGallopBlocks);
  if (patched)
    hipLaunchKernelGGL((k_chain<WAVES, kFeatPatched>), dim3(groups), dim3(WAVES * 64), 0, stream, r, r_raw, r_len,
                       args, rs, epoch, d_out, d_count, gb);
  else
    hipLaunchKernelGGL((k_chain<WAVES, 0>), dim3(groups), dim3(WAVES * 64), 0, stream, r, r_raw, r_len, args, rs,
                       epoch, d_out, d_count, gb);
}

// One launch: chunk kernel with look-back compaction; count to d_count.
static int run_chain(const DList &r, const uint32_t *r_raw, const uint64_t *r_len, const ChainArgs &args,
                     const RunScratch &rs, uint32_t *d_out, uint64_t *d_count, hipStream_t stream) {
  if (rs.items_cap == 0) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, stream, d_count, uint64_t(0));
    S4_HIP(hipGetLastError());
    return S4_OK;
  }
  switch (tuning().waves_per_group) {
    case 1: launch_chain_w<1>(r, r_raw, r_len, args, rs, d_out, d_count, stream); break;
    case 2: launch_chain_w<2>(r, r_raw, r_len, args, rs, d_out, d_count, stream); break;
    case 8: launch_chain_w<8>(r, r_raw, r_len, args, rs, d_out, d_count, stream); break;
    default: launch_chain_w<4>(r, r_raw, r_len, args, rs, d_out, d_count, stream); break;
  }
  S4_HIP(hipGetLastError());
  return S4_OK;
}

int scan_and_compact(const uint32_t *stage, const uint32_t *counts, uint32_t n, uint32_t *excl, uint32_t *tiles,
                     uint32_t ntiles, uint64_t *total, uint32_t *out, hipStream_t stream) {
  hipLaunchKernelGGL(k_scan_tiles, dim3(std::max<uint32_t>(1, ntiles)), dim3(256), 0, stream, counts, n, excl, tiles);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, stream, tiles, ntiles, total);
  if (n) hipLaunchKernelGGL(k_compact, dim3((n + 255) / 256), dim3(256), 0, stream, stage, counts, excl, tiles, n, out);
  S4_HIP(hipGetLastError());
  return S4_OK;
}

static int run_pair(const DList &r, const uint32_t *r_raw, const uint64_t *r_len, const DList &f,
                    const RunScratch &rs, uint32_t *d_out, uint64_t *d_count, hipStream_t stream) {
  ChainArgs args;
  args.f[0] = f;
  args.nf = 1;
  return run_chain(r, r_raw, r_len, args, rs, d_out, d_count, stream);
}

template <int P, bool PK>
static void launch_decode_k(const DecodeLaunch &d, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  const DecodeArgs &a = d.a;
  if (ev0)
    hipExtLaunchKernelGGL((k_decode<P, PK>), dim3(d.workgroups), dim3(256), 0, stream, ev0, ev1, 0, a.widths, a.offs,
                          a.seeds, a.payload, a.out, a.first, a.full_end, a.block_waves, a.form, a.tail, a.nb);
  else
    hipLaunchKernelGGL((k_decode<P, PK>), dim3(d.workgroups), dim3(256), 0, stream, a.widths, a.offs, a.seeds,
                       a.payload, a.out, a.first, a.full_end, a.block_waves, a.form, a.tail, a.nb);
}
template <int P>
static void launch_decode(const DecodeLaunch &d, hipStream_t stream, hipEvent_t ev0, hipEvent_t ev1) {
  if (d.patched)
    launch_decode_k<P, true>(d, stream, ev0, ev1);
  else
    launch_decode_k<P, false>(d, stream, ev0, ev1);
}

bool plan_decode_range(const DList &L, uint32_t first, uint32_t count, uint32_t *d_out, DecodeLaunch *d) {
  const uint32_t end = first + count;
  const uint32_t full = end > L.nb ? (L.nb > first ? L.nb - first : 0) : count;
  // blocks per wave (4 P): the largest P that still gives ~8 waves per CU
  const uint32_t target_waves = uint32_t(cu_count()) * 8u;
  uint32_t P = tuning_decode_passes();
  while (P > 1 && (full + 4 * P - 1) / (4 * P) < target_waves) P >>= 1;
  const uint32_t block_waves = (full + 4 * P - 1) / (4 * P);
  const bool tail = end > L.nb && L.t > 0;
  const uint32_t waves = block_waves + (tail ? 1 : 0);
  if (waves == 0) return false;
  d->P = P;
  d->patched = is_patched(L);
  d->workgroups = (waves + 3) / 4;
  d->a = DecodeArgs{L.widths, L.offs, L.seeds, L.payload, d_out, first, first + full, block_waves,
                    L.mode | (d->patched ? kDecodePatched : 0u) | (tail ? kDecodeTail : 0u) | (L.t << 16),
                    L.tail, L.nb};
  return true;
}

const void *decode_kernel_host_address(uint32_t P, bool patched) {
  switch (P) {
    case 8: return patched ? reinterpret_cast<const void *>(&k_decode<8, true>) : reinterpret_cast<const void *>(&k_decode<8, false>);
    case 4: return patched ? reinterpret_cast<const void *>(&k_decode<4, true>) : reinterpret_cast<const void *>(&k_decode<4, false>);
    case 2: return patched ? reinterpret_cast<const void *>(&k_decode<2, true>) : reinterpret_cast<const void *>(&k_decode<2, false>);
    default: return patched ? reinterpret_cast<const void *>(&k_decode<1, true>) : reinterpret_cast<const void *>(&k_decode<1, false>);
  }
}

int decode_range(const DList &L, uint32_t first, uint32_t count, uint32_t *d_out, hipStream_t stream) {
  return decode_range_timed(L, first, count, d_out, stream, nullptr, nullptr);
}

int decode_range_timed(const DList &L, uint32_t first, uint32_t count, uint32_t *d_out, hipStream_t stream,
                       hipEvent_t ev0, hipEvent_t ev1) {
  DecodeLaunch d;
  if (!plan_decode_range(L, first, count, d_out, &d)) return S4_OK;
  switch (d.P) {
    case 8: launch_decode<8>(d, stream, ev0, ev1); break;
    case 4: launch_decode<4>(d, stream, ev0, ev1); break;
    case 2: launch_decode<2>(d, stream, ev0, ev1); break;
    default: launch_decode<1>(d, stream, ev0, ev1); break;
  }
  S4_HIP(hipGetLastError());
  return S4_OK;
}

}  // namespace s4

struct s4_decode_plan {
  void *table = nullptr;
  const s4::DList *lists = nullptr;
  uint32_t *const *outs = nullptr;
  const uint32_t *prefix = nullptr;
  const uint32_t *wave_list = nullptr;
  uint32_t count = 0, passes = 4, waves = 0;
  uint64_t ints = 0;
  bool patched = false;  // some list is patched: the kernels instantiated for them
};

using namespace s4;

template <int P>
static void launch_plan(const s4_decode_plan *p, hipStream_t st) {
  if (p->patched)
    hipLaunchKernelGGL((k_decode_multi<P, true>), dim3((p->waves + 3) / 4), dim3(256), 0, st, p->lists, p->outs,
                       p->prefix, p->wave_list, p->waves);
  else
    hipLaunchKernelGGL((k_decode_multi<P, false>), dim3((p->waves + 3) / 4), dim3(256), 0, st, p->lists, p->outs,
                       p->prefix, p->wave_list, p->waves);
}

static inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

int s4_get_tuning(s4_tuning *t) {
  if (!t) return fail(S4_EINVAL, "null tuning");
  *t = tuning();
  return S4_OK;
}

int s4_set_tuning(const s4_tuning *t) {
  if (!t) return fail(S4_EINVAL, "null tuning");
  if (t->gallop_blocks < 1 || t->gallop_blocks > kMaxGallopBlocks)
    return fail(S4_EINVAL, "gallop_blocks must be in [1, 512]");
  if (t->waves_per_group != 1 && t->waves_per_group != 2 && t->waves_per_group != 4 && t->waves_per_group != 8)
    return fail(S4_EINVAL, "waves_per_group must be 1, 2, 4 or 8");
  if (t->groups_per_cu < 1 || t->groups_per_cu > 32) return fail(S4_EINVAL, "groups_per_cu must be in [1, 32]");
  if (t->items_per_grab < 1 || t->items_per_grab > 64) return fail(S4_EINVAL, "items_per_grab must be in [1, 64]");
  if (t->decode_passes != 1 && t->decode_passes != 2 && t->decode_passes != 4 && t->decode_passes != 8)
    return fail(S4_EINVAL, "decode_passes must be 1, 2, 4 or 8");
  tuning() = *t;
  return S4_OK;
}

int s4_list_upload(const uint8_t *enc, size_t bytes, void *stream, s4_list **out) {
  if (!out) return fail(S4_EINVAL, "null out");
  Upload u;
  u.views.resize(1);
  int rc = parse_stream(enc, bytes, &u.views[0]);
  if (rc) return rc;
  s4_list *l = new (std::nothrow) s4_list;
  if (!l) return fail(S4_ENOMEM, "handle allocation failed");
  std::vector<DList> descs;
  rc = build_arena(u, as_stream(stream), &l->arena, &descs);
  if (rc) {
    delete l;
    return rc;
  }
  const StreamView &v = u.views[0];
  l->d = descs[0];
  l->n = v.n;
  l->nb = v.nb;
  l->t = v.t;
  l->pw = v.pw;
  l->flags = v.flags;
  l->payload_bytes = v.data_bytes();
  l->index_bytes = uint64_t(v.nb) * (4 + 4 + 16 + (v.patched() ? 16 : 0));
  *out = l;
  return S4_OK;
}

int s4_list_free(s4_list *list) {
  if (!list) return S4_OK;
  if (list->arena) {
    hipError_t e = hipFree(list->arena);
    delete list;
    if (e != hipSuccess) return hip_fail(e, "hipFree");
    return S4_OK;
  }
  delete list;
  return S4_OK;
}

int s4_list_info(const s4_list *l, uint64_t *n, uint32_t *nb, uint32_t *flags, uint64_t *payload_bytes,
                 uint64_t *index_bytes) {
  if (!l) return fail(S4_EINVAL, "null list");
  if (n) *n = l->n;
  if (nb) *nb = l->nb;
  if (flags) *flags = l->flags;
  if (payload_bytes) *payload_bytes = l->payload_bytes;
  if (index_bytes) *index_bytes = l->index_bytes;
  return S4_OK;
}

int s4_list_skip_index(const s4_list *l, uint32_t *bmax, uint32_t *seeds, void *stream) {
  if (!l || (l->nb && (!bmax || !seeds))) return fail(S4_EINVAL, "null argument");
  if (!l->nb) return S4_OK;
  S4_HIP(hipMemcpyAsync(bmax, l->d.bmax, 4ull * l->nb, hipMemcpyDeviceToHost, as_stream(stream)));
  S4_HIP(hipMemcpyAsync(seeds, l->d.seeds, 16ull * l->nb, hipMemcpyDeviceToHost, as_stream(stream)));
  S4_HIP(hipStreamSynchronize(as_stream(stream)));
  return S4_OK;
}

int s4_decode_dev(const s4_list *l, uint32_t *d_out, uint64_t cap, void *stream) {
  if (!l || (!d_out && l->n)) return fail(S4_EINVAL, "null argument");
  if (cap < l->n) return fail(S4_ERANGE, "s4_decode_dev: cap < n");
  if (reinterpret_cast<uintptr_t>(d_out) & 15u) return fail(S4_EINVAL, "d_out must be 16-byte aligned");
  if (!l->n) return S4_OK;
  return decode_range(l->d, 0, l->nb + (l->t ? 1 : 0), d_out, as_stream(stream));
}

int s4_decode_timed_dev(const s4_list *l, uint32_t *d_out, uint64_t cap, void *start_event, void *stop_event,
                        void *stream) {
  if (!l || (!d_out && l->n) || !start_event || !stop_event) return fail(S4_EINVAL, "null argument");
  if (cap < l->n) return fail(S4_ERANGE, "s4_decode_timed_dev: cap < n");
  if (reinterpret_cast<uintptr_t>(d_out) & 15u) return fail(S4_EINVAL, "d_out must be 16-byte aligned");
  hipEvent_t e0 = static_cast<hipEvent_t>(start_event), e1 = static_cast<hipEvent_t>(stop_event);
  if (!l->n) {
    S4_HIP(hipEventRecord(e0, as_stream(stream)));
    S4_HIP(hipEventRecord(e1, as_stream(stream)));
    return S4_OK;
  }
  return decode_range_timed(l->d, 0, l->nb + (l->t ? 1 : 0), d_out, as_stream(stream), e0, e1);
}

int s4_decode_blocks_dev(const s4_list *l, uint32_t first, uint32_t count, uint32_t *d_out, void *stream) {
  if (!l || (!d_out && count)) return fail(S4_EINVAL, "null argument");
  const uint32_t pseudo = l->nb + (l->t ? 1 : 0);
  if (uint64_t(first) + count > pseudo) return fail(S4_ERANGE, "block range beyond the list");
  if (reinterpret_cast<uintptr_t>(d_out) & 15u) return fail(S4_EINVAL, "d_out must be 16-byte aligned");
  if (!count) return S4_OK;
  return decode_range(l->d, first, count, d_out, as_stream(stream));
}

int s4_decode_lists_dev(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps,
                        uint32_t count, uint32_t nstreams, void *stream) {
  if (nstreams != 1 && nstreams != kMaxStreams) return fail(S4_EINVAL, "nstreams must be 1 or 8");
  if (!count) return S4_OK;
  if (!lists || !d_outs || !caps) return fail(S4_EINVAL, "null argument");
  for (uint32_t i = 0; i < count; ++i) {
    if (!lists[i] || (!d_outs[i] && lists[i]->n)) return fail(S4_EINVAL, "null list or output");
    if (caps[i] < lists[i]->n) return fail(S4_ERANGE, "cap < n for list " + std::to_string(i));
    if (reinterpret_cast<uintptr_t>(d_outs[i]) & 15u) return fail(S4_EINVAL, "outputs must be 16-byte aligned");
  }
  int rc = ensure_device();
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  if (nstreams == 1) {
    for (uint32_t i = 0; i < count; ++i) {
      const s4_list *l = lists[i];
      if (!l->n) continue;
      rc = decode_range(l->d, 0, l->nb + (l->t ? 1 : 0), d_outs[i], st);
      if (rc) return rc;
    }
    return S4_OK;
  }
  // longest-processing-time assignment of lists to streams by bytes moved
  std::vector<uint32_t> order(count);
  std::iota(order.begin(), order.end(), 0u);
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return lists[a]->n > lists[b]->n; });
  std::vector<uint64_t> load(nstreams, 0);
  std::vector<uint32_t> owner(count);
  for (uint32_t i : order) {
    uint32_t best = 0;
    for (uint32_t s = 1; s < nstreams; ++s)
      if (load[s] < load[best]) best = s;
    owner[i] = best;
    load[best] += lists[i]->payload_bytes + 4 * lists[i]->n + 4096;
  }
  std::lock_guard<std::mutex> lock(g_pool_mu);
  StreamPool *pool = nullptr;
  rc = get_pool(&pool);
  if (rc) return rc;
  S4_HIP(hipEventRecord(pool->fork, st));
  for (uint32_t s = 1; s < nstreams; ++s) S4_HIP(hipStreamWaitEvent(pool->streams[s], pool->fork, 0));
  for (uint32_t i : order) {
    const s4_list *l = lists[i];
    if (!l->n) continue;
    hipStream_t target = owner[i] == 0 ? st : pool->streams[owner[i]];
    rc = decode_range(l->d, 0, l->nb + (l->t ? 1 : 0), d_outs[i], target);
    if (rc) return rc;
  }
  for (uint32_t s = 1; s < nstreams; ++s) {
    S4_HIP(hipEventRecord(pool->join[s], pool->streams[s]));
    S4_HIP(hipStreamWaitEvent(st, pool->join[s], 0));
  }
  return S4_OK;
}

int s4_decode_plan_create(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps,
                          uint32_t count, void *stream, s4_decode_plan **out) {
  if (!out || (count && (!lists || !d_outs || !caps))) return fail(S4_EINVAL, "null argument");
  for (uint32_t i = 0; i < count; ++i) {
    if (!lists[i] || (!d_outs[i] && lists[i]->n)) return fail(S4_EINVAL, "null list or output");
    if (caps[i] < lists[i]->n) return fail(S4_ERANGE, "cap < n for list " + std::to_string(i));
    if (reinterpret_cast<uintptr_t>(d_outs[i]) & 15u) return fail(S4_EINVAL, "outputs must be 16-byte aligned");
  }
  int rc = ensure_device();
  if (rc) return rc;
  s4_decode_plan *p = new (std::nothrow) s4_decode_plan;
  if (!p) return fail(S4_ENOMEM, "plan allocation failed");
  p->count = count;
  p->passes = tuning_decode_passes();
  std::vector<uint32_t> prefix(count + 1, 0);
  for (uint32_t i = 0; i < count; ++i) {
    const s4_list *l = lists[i];
    const uint32_t bw = (l->nb + 4 * p->passes - 1) / (4 * p->passes);
    prefix[i + 1] = prefix[i] + bw + (l->t ? 1u : 0u);
    p->ints += l->n;
    p->patched |= is_patched(l->d);
  }
  p->waves = prefix[count];
  const size_t desc_b = align_up(sizeof(DList) * std::max<uint32_t>(1, count), 256);
  const size_t outs_b = align_up(sizeof(uint32_t *) * std::max<uint32_t>(1, count), 256);
  const size_t pre_b = align_up(4 * size_t(count + 1), 256);
  const size_t wl_b = align_up(4 * size_t(std::max<uint32_t>(1, p->waves)), 256);
  hipError_t e = hipMalloc(&p->table, desc_b + outs_b + pre_b + wl_b);
  if (e != hipSuccess) {
    delete p;
    return fail(S4_ENOMEM, "plan table allocation failed");
  }
  std::vector<char> img(desc_b + outs_b + pre_b + wl_b, 0);
  uint32_t *wl = reinterpret_cast<uint32_t *>(img.data() + desc_b + outs_b + pre_b);
  for (uint32_t i = 0; i < count; ++i)
    for (uint32_t w = prefix[i]; w < prefix[i + 1]; ++w) wl[w] = i;
  for (uint32_t i = 0; i < count; ++i) {
    std::memcpy(img.data() + sizeof(DList) * i, &lists[i]->d, sizeof(DList));
    std::memcpy(img.data() + desc_b + sizeof(uint32_t *) * i, &d_outs[i], sizeof(uint32_t *));
  }
  std::memcpy(img.data() + desc_b + outs_b, prefix.data(), 4 * size_t(count + 1));
  e = hipMemcpyAsync(p->table, img.data(), img.size(), hipMemcpyHostToDevice, as_stream(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
  if (e != hipSuccess) {
    (void)hipFree(p->table);
    delete p;
    return hip_fail(e, "plan upload");
  }
  p->lists = static_cast<const DList *>(p->table);
  p->outs = reinterpret_cast<uint32_t *const *>(static_cast<char *>(p->table) + desc_b);
  p->prefix = reinterpret_cast<const uint32_t *>(static_cast<char *>(p->table) + desc_b + outs_b);
  p->wave_list = reinterpret_cast<const uint32_t *>(static_cast<char *>(p->table) + desc_b + outs_b + pre_b);
  *out = p;
  return S4_OK;
}

int s4_decode_plan_run(const s4_decode_plan *p, void *stream) {
  if (!p) return fail(S4_EINVAL, "null plan");
  if (!p->waves) return S4_OK;
  switch (p->passes) {
    case 8: launch_plan<8>(p, as_stream(stream)); break;
    case 2: launch_plan<2>(p, as_stream(stream)); break;
    case 1: launch_plan<1>(p, as_stream(stream)); break;
    default: launch_plan<4>(p, as_stream(stream)); break;
  }
  S4_HIP(hipGetLastError());
  return S4_OK;
}

int s4_decode_plan_free(s4_decode_plan *p) {
  if (!p) return S4_OK;
  hipError_t e = hipFree(p->table);
  delete p;
  if (e != hipSuccess) return hip_fail(e, "hipFree");
  return S4_OK;
}

int s4_spin_dev(uint64_t ns, void *stream) {
  int rc = ensure_device();
  if (rc) return rc;
  int khz = 0;
  S4_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, g_dev_checked));
  if (khz <= 0) khz = 100000;
  const uint64_t ticks = ns * uint64_t(khz) / 1000000ull;
  hipLaunchKernelGGL(k_spin, dim3(1), dim3(64), 0, as_stream(stream), ticks);
  S4_HIP(hipGetLastError());
  return S4_OK;
}

size_t s4_intersect_scratch_bytes(uint64_t len_a, uint64_t len_b) {
  return run_scratch_layout(std::min(len_a, len_b), nullptr, nullptr);
}

int s4_intersect(const s4_list *a, const s4_list *b, uint32_t *d_out, uint64_t cap, uint64_t *d_count,
                 void *d_scratch, size_t scratch_bytes, void *stream) {
  if (!a || !b || !d_count) return fail(S4_EINVAL, "null argument");
  if (!(a->flags & 1u) || !(b->flags & 1u)) return fail(S4_EUNSORTED, "intersection inputs must be strictly increasing");
  const s4_list *r = a->n <= b->n ? a : b;
  const s4_list *f = a->n <= b->n ? b : a;
  if (cap < r->n) return fail(S4_ERANGE, "cap < min(len a, len b)");
  const size_t need = run_scratch_layout(r->n, nullptr, nullptr);
  if (scratch_bytes < need || (!d_scratch && need)) return fail(S4_ERANGE, "scratch too small");
  if (r->n && !d_out) return fail(S4_EINVAL, "null d_out");
  int rc = ensure_device();
  if (rc) return rc;
  RunScratch ps;
  run_scratch_layout(r->n, static_cast<char *>(d_scratch), &ps);
  return run_pair(r->d, nullptr, nullptr, f->d, ps, d_out, d_count, as_stream(stream));
}

size_t s4_intersect_raw_scratch_bytes(uint64_t cap_r) { return run_scratch_layout(cap_r, nullptr, nullptr); }

int s4_intersect_raw(const uint32_t *d_r, const uint64_t *d_len_r, uint64_t cap_r, const s4_list *f,
                     uint32_t *d_out, uint64_t cap, uint64_t *d_count, void *d_scratch, size_t scratch_bytes,
                     void *stream) {
  if (!f || !d_len_r || !d_count || (cap_r && !d_r)) return fail(S4_EINVAL, "null argument");
  if (!(f->flags & 1u)) return fail(S4_EUNSORTED, "intersection inputs must be strictly increasing");
  if (cap < std::min(cap_r, f->n)) return fail(S4_ERANGE, "cap too small");
  const uint64_t cr = cap_r;
  const size_t need = run_scratch_layout(cr, nullptr, nullptr);
  if (scratch_bytes < need || (!d_scratch && need)) return fail(S4_ERANGE, "scratch too small");
  int rc = ensure_device();
  if (rc) return rc;
  RunScratch ps;
  run_scratch_layout(cr, static_cast<char *>(d_scratch), &ps);
  DList none{};
  none.n = cr;  // the kernel reads at most cap_r raw values
  return run_pair(none, d_r, d_len_r, f->d, ps, d_out, d_count, as_stream(stream));
}

size_t s4_intersect_k_scratch_bytes(const s4_list *const *lists, uint32_t k) {
  if (!lists || k == 0) return 0;
  uint64_t m = UINT64_MAX;
  for (uint32_t i = 0; i < k; ++i)
    if (lists[i]) m = std::min(m, lists[i]->n);
  if (m == UINT64_MAX) return 0;
  return run_scratch_layout(m, nullptr, nullptr);
}

}  // extern "C"

// Checks a conjunction's arguments and orders its lists shortest first into
// ord[0 .. k) (stable, so equal lengths keep their given order: SvS).
static int order_conjunction(const s4_list *const *lists, uint32_t k, uint32_t *d_out, uint64_t cap,
                             uint64_t *d_count, const s4_list **ord) {
  if (!lists || k == 0 || !d_count) return fail(S4_EINVAL, "s4_intersect_k: need k >= 1 lists and d_count");
  if (k > kMaxTerms + 1) return fail(S4_EINVAL, "s4_intersect_k: at most 33 lists");
  for (uint32_t i = 0; i < k; ++i) {
    if (!lists[i]) return fail(S4_EINVAL, "null list");
    uint32_t j = i;
    for (; j > 0 && ord[j - 1]->n > lists[i]->n; --j) ord[j] = ord[j - 1];
    ord[j] = lists[i];
  }
  const uint64_t m = ord[0]->n;
  if (cap < m) return fail(S4_ERANGE, "cap < length of the shortest list");
  if (m && !d_out) return fail(S4_EINVAL, "null d_out");
  if (k == 1) {
    if (reinterpret_cast<uintptr_t>(d_out) & 15u) return fail(S4_EINVAL, "d_out must be 16-byte aligned");
    return S4_OK;
  }
  for (uint32_t i = 0; i < k; ++i)
    if (!(ord[i]->flags & 1u)) return fail(S4_EUNSORTED, "intersection inputs must be strictly increasing");
  return S4_OK;
}

// The ordered conjunction on scratch rs: k = 1 decodes the list and sets
// the count; otherwise one chain launch.
static int run_conjunction(const s4_list *const *ord, uint32_t k, const RunScratch &rs, uint32_t *d_out,
                           uint64_t *d_count, hipStream_t st) {
  if (k == 1) {
    if (ord[0]->n) {
      const int rc = decode_range(ord[0]->d, 0, ord[0]->nb + (ord[0]->t ? 1 : 0), d_out, st);
      if (rc) return rc;
    }
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, st, d_count, ord[0]->n);
    S4_HIP(hipGetLastError());
    return S4_OK;
  }
  ChainArgs args;
  args.nf = k - 1;
  for (uint32_t i = 1; i < k; ++i) args.f[i - 1] = ord[i]->d;
  return run_chain(ord[0]->d, nullptr, nullptr, args, rs, d_out, d_count, st);
}

namespace s4 {

size_t conjunction_scratch_bytes(uint64_t m) { return run_scratch_layout(m, nullptr, nullptr); }

int enqueue_conjunction(const DList *ord, uint32_t k, void *scratch, uint32_t *d_out, uint64_t *d_count,
                        hipStream_t st) {
  if (k < 2 || k > kMaxTerms + 1) return fail(S4_EINVAL, "a conjunction takes 2 to 33 lists");
  RunScratch rs{};
  run_scratch_layout(ord[0].n, static_cast<char *>(scratch), &rs);
  ChainArgs args;
  args.nf = k - 1;
  for (uint32_t i = 1; i < k; ++i) args.f[i - 1] = ord[i];
  return run_chain(ord[0], nullptr, nullptr, args, rs, d_out, d_count, st);
}

}  // namespace s4

// Scratch of s4_intersect_k_noalloc: one array per device, for callers that
// cannot allocate; its device address is looked up once per device.
static __device__ __align__(256) uint8_t scratch[S4_NOALLOC_SCRATCH_BYTES];
static std::mutex g_static_mu;
static std::map<int, char *> g_static_ptr;

static int static_scratch(char **out) {
  int dev = 0;
  S4_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_static_mu);
  auto it = g_static_ptr.find(dev);
  if (it == g_static_ptr.end()) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255u)) return fail(S4_EDEVICE, "static scratch address unusable");
    it = g_static_ptr.emplace(dev, static_cast<char *>(p)).first;
  }
  *out = it->second;
  return S4_OK;
}

// Longest shortest list the static scratch serves.
static uint64_t noalloc_max_len() {
  uint64_t lo = 0, hi = uint64_t(S4_NOALLOC_SCRATCH_BYTES) * 8;  // fits at lo, not at hi
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (run_scratch_layout(mid, nullptr, nullptr) <= S4_NOALLOC_SCRATCH_BYTES) lo = mid; else hi = mid;
  }
  return lo;
}

extern "C" {

int s4_init(void) {
  int rc = ensure_device();
  if (rc) return rc;
  char *p = nullptr;
  return static_scratch(&p);
}

int s4_intersect_k(const s4_list *const *lists, uint32_t k, uint32_t *d_out, uint64_t cap, uint64_t *d_count,
                   void *d_scratch, size_t scratch_bytes, void *stream) {
  const s4_list *ord[kMaxTerms + 1];
  int rc = order_conjunction(lists, k, d_out, cap, d_count, ord);
  if (rc) return rc;
  rc = ensure_device();
  if (rc) return rc;
  RunScratch rs{};
  if (k > 1) {
    const size_t need = run_scratch_layout(ord[0]->n, nullptr, nullptr);
    if (scratch_bytes < need || !d_scratch) return fail(S4_ERANGE, "scratch too small");
    run_scratch_layout(ord[0]->n, static_cast<char *>(d_scratch), &rs);
  }
  return run_conjunction(ord, k, rs, d_out, d_count, as_stream(stream));
}

uint64_t s4_intersect_k_noalloc_max_len(void) { return noalloc_max_len(); }

int s4_intersect_k_noalloc(const s4_list *const *lists, uint32_t k, uint32_t *d_out, uint64_t cap,
                           uint64_t *d_count, void *stream) {
  const s4_list *ord[kMaxTerms + 1];
  int rc = order_conjunction(lists, k, d_out, cap, d_count, ord);
  if (rc) return rc;
  static const uint64_t max_len = noalloc_max_len();
  if (ord[0]->n > max_len)
    return fail(S4_ERANGE, "s4_intersect_k_noalloc: shortest list has " + std::to_string(ord[0]->n) +
                               " values; the static scratch serves at most " + std::to_string(max_len));
  rc = ensure_device();
  if (rc) return rc;
  char *base = nullptr;
  rc = static_scratch(&base);
  if (rc) return rc;
  RunScratch rs{};
  run_scratch_layout(ord[0]->n, base, &rs);
  return run_conjunction(ord, k, rs, d_out, d_count, as_stream(stream));
}

}  // extern "C"

// Device-resident index of many lists, and batches of conjunctive queries
// run as one persistent decode-fused launch (plus scan and compaction),
// optionally replayed from a captured hipGraph; autotuning of the launch
// parameters.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <vector>

#include "s4_kernels.h"

namespace s4 {

// Reset the work queues and the per-query completion stamps.
__global__ void k_batch_begin(BatchDev b) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    *b.start = wall_clock64();
    b.stats[0] = 0;
    b.stats[1] = 0;
  }
  const uint32_t nheads = b.parts > 1 ? b.parts : kSubQueues;
  for (uint32_t p = t; p < nheads; p += gridDim.x * blockDim.x) b.head[p * kHeadStride] = 0;
  for (uint32_t q = t; q < b.nq; q += gridDim.x * blockDim.x) b.qtick[q] = 0;
}

// XCDs of the device; workgroups are dispatched to them round-robin by id.
constexpr uint32_t kXcds = 8;

// Persistent chunk kernel: every wave takes `grab` chunks at a time from
// the queue until it is empty; a chunk of query q is 128 values of q's
// shortest list carried through all of q's other lists (SvS per chunk).
// With a doc-ID partitioned index each part has its own queue; a
// workgroup first drains the parts of its own XCD (part x mod P for fewer
// than 8 parts, parts x, x + 8, ... otherwise), so each XCD's L2 holds one
// part's lists, then helps every other queue.
// The chunk kernels are latency-bound, so resident waves matter most: an
// instantiation is held to 64 VGPRs (8 waves per SIMD, whose LDS, 5 KB per
// wave, then just fills a CU) where that spills nothing and pays, else to
// 80 (6 waves): the traffic-counting ones and those for a partitioned index
// (at 8 waves 3-6% slower on most of its batches); bitmap and patched lists
// run at 8 (7-12% faster than at 6).  Work added to the per-chunk path that
// keeps more values live (loading the next candidate group's block metadata
// during the current group, decoding r's block while the first list is
// searched) measured slower than the round trips it saved.
constexpr int chunk_waves_per_simd(uint32_t feat) {
  return (feat & (kFeatCount | kFeatParts)) ? 6 : 8;
}
template <int WAVES, uint32_t FEAT>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(chunk_waves_per_simd(FEAT)))) void k_batch_chunks(
    BatchDev b, uint32_t grab, uint32_t gallop_blocks) {
  __shared__ ItemLds lds[WAVES];
  // queues this workgroup has found empty (bit p, p < 32): its other waves
  // skip them rather than fetch from an exhausted head once each.  The word
  // is wave 0's last skip-index staging entry (the launch stages at most
  // kMaxGallopBlocks - 1), so the workgroup's LDS stays 5 KB per wave.
  uint32_t *const empty_q = &lds[0].bm[kMaxGallopBlocks - 1];
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  if (threadIdx.x == 0) *empty_q = 0;
  __syncthreads();
  const uint64_t t0 = *b.start;
  // counting is an instantiation of its own: the timed kernels carry no
  // counters (they cost the chunk pipeline registers and issue slots)
  Traffic tr;
  tr.on = (FEAT & kFeatCount) != 0;
  // completion stamps: one atomic per run of consecutive chunks of a query
  uint32_t run_q = kInvalid;
  uint64_t run_t = 0;
  // search hint of the second list: valid while the wave takes the next
  // chunk of the same pair of lists
  uint32_t hint = 0, h_id0 = kInvalid, h_id1 = kInvalid, h_local = kInvalid;
  // drain queue p: chunks base .. base + size in queue order
  auto drain = [&](uint32_t p, uint32_t base, uint32_t size) {
    const uint32_t pbit = p < 32 ? 1u << p : 0u;
    for (;;) {
      if (uniform(*(volatile uint32_t *)empty_q) & pbit) break;
      uint32_t it0 = 0;
      if (lane == 0) it0 = atomicAdd(b.head + p * kHeadStride, grab);
      it0 = uniform(it0);  // lane 0's value: every lane is active here
      if (it0 >= size) {
        if (lane == 0) atomicOr(empty_q, pbit);
        break;
      }
      const uint32_t it1 = min(it0 + grab, size);
      for (uint32_t rel = it0; rel < it1; ++rel) {
        const uint32_t item = base + rel;
        // one record per chunk: query, chunk within the query, first term, terms
        const uint4 info = cst(b.item_info)[item];
        const uint32_t q = uniform(info.x), local = uniform(info.y), tq = uniform(info.z), k = uniform(info.w);
        // the two shortest lists' descriptors, loaded together up front
        const uint32_t id0 = uniform(cst(b.sterms)[tq]), id1 = uniform(cst(b.sterms)[tq + (k > 1 ? 1 : 0)]);
        RSide r;
        r.L = cst(b.lists)[id0];
        const DList f1 = cst(b.lists)[id1];
        r.raw = nullptr;
        r.len = r.L.n;
        if (id0 != h_id0 || id1 != h_id1 || local != h_local + 1) hint = 0;
        const uint32_t cnt = chain_chunk<FEAT>(
            r, local, f1, [&](uint32_t j) -> DList { return cst(b.lists)[uniform(cst(b.sterms)[tq + 1 + j])]; }, k - 1,
            lds[w], gallop_blocks, tr, hint);
        h_id0 = id0;
        h_id1 = id1;
        h_local = local;
        const uint32_t slot = (FEAT & kFeatParts) ? b.item_rank[item] : item;
        store_chunk(cnt, lds[w], b.stage + uint64_t(slot) * kBlock, b.counts + slot);
        const uint64_t now = wall_clock64() - t0;
        if (q != run_q) {
          if (run_q != kInvalid && lane == 0)
            atomicMax(reinterpret_cast<unsigned long long *>(b.qtick + run_q), static_cast<unsigned long long>(run_t));
          run_q = q;
        }
        run_t = now;
      }
      if (run_q != kInvalid && lane == 0)
        atomicMax(reinterpret_cast<unsigned long long *>(b.qtick + run_q), static_cast<unsigned long long>(run_t));
      run_q = kInvalid;
    }
  };
  if (!(FEAT & kFeatParts)) {
    // kSubQueues contiguous slices of the chunks: a workgroup drains its
    // own XCD's slice first (a query's chunks stay together, and so its
    // lists in that XCD's L2), then helps the others in turn
    const uint32_t x = blockIdx.x % kSubQueues;
    for (uint32_t v = 0; v < kSubQueues; ++v) {
      const uint32_t p = (x + v) % kSubQueues;
      const uint32_t lo = uint32_t(uint64_t(b.items) * p / kSubQueues);
      const uint32_t hi = uint32_t(uint64_t(b.items) * (p + 1) / kSubQueues);
      drain(p, lo, hi - lo);
    }
  } else {
    const uint32_t P = b.parts, x = blockIdx.x % kXcds;
    const uint32_t own = P >= kXcds ? (P - x + kXcds - 1) / kXcds : 1u;
    for (uint32_t v = 0; v < own + P; ++v) {
      const uint32_t p = v < own ? (P >= kXcds ? x + kXcds * v : x % P) : (x + v - own) % P;
      drain(p, b.part_base[p], b.part_base[p + 1] - b.part_base[p]);
    }
  }
  if (tr.on && lane == 0) {
    atomicAdd(reinterpret_cast<unsigned long long *>(b.stats), static_cast<unsigned long long>(tr.bytes));
    atomicAdd(reinterpret_cast<unsigned long long *>(b.stats + 1), static_cast<unsigned long long>(tr.blocks));
  }
}

// Scan word of one chunk: high half (epoch << 2 | flag), low half a value;
// flag 1: the chunk's count alone, flag 2: inclusive prefix through it.
__device__ __forceinline__ void publish(uint64_t *w, uint32_t tag, uint32_t v) {
  __hip_atomic_store(w, (uint64_t(tag) << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr uint32_t kLookbackSpins = 1u << 22;

// Decoupled look-back: publish this chunk's count, then read the words of
// the 64 nearest predecessors at once; the offset is the sum of the counts
// back to (and including) the nearest inclusive prefix, and is published
// in turn as this chunk's inclusive prefix.  Chunks are taken from the
// queue in increasing order by running waves, so the earliest unfinished
// chunk never waits and the walk always ends; the spin bound is a guard.
__device__ uint32_t lookback(uint64_t *__restrict__ state, uint32_t item, uint32_t epoch, uint32_t cnt,
                             uint32_t *__restrict__ err, bool &ok) {
  const uint32_t lane = lane_id();
  const uint32_t tag_a = (epoch << 2) | 1u, tag_p = (epoch << 2) | 2u;
  if (item == 0) {
    if (lane == 0) publish(state, tag_p, cnt);
    return 0;
  }
  if (lane == 0) publish(state + item, tag_a, cnt);
  uint32_t excl = 0, spins = 0;
  int64_t base = int64_t(item) - 1;
  for (;;) {
    const int64_t j = base - int64_t(lane);
    uint32_t hi = tag_p, val = 0;  // before the first chunk: prefix 0
    if (j >= 0) {
      const uint64_t v = __hip_atomic_load(state + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      hi = uint32_t(v >> 32);
      val = uint32_t(v);
    }
    const uint64_t is_p = __ballot(hi == tag_p);
    const uint64_t ready = __ballot(hi == tag_p || hi == tag_a);
    // lanes through the nearest inclusive prefix (all 64 if none)
    const uint64_t need = is_p ? ((is_p & (~is_p + 1)) << 1) - 1 : ~0ull;
    if ((ready & need) == need) {
      excl += wave_sum(((need >> lane) & 1) ? val : 0u);
      if (is_p) break;
      base -= 64;
    } else {
      if (++spins > kLookbackSpins) {
        if (lane == 0) *err = 1u;
        ok = false;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  if (lane == 0) publish(state + item, tag_p, excl + cnt);
  return excl;
}

// Single-pass persistent chunk kernel: as k_batch_chunks, but every chunk
// writes its survivors straight to out at the offset found by look-back,
// and the first chunk of each entry writes that entry's CSR offset (and
// those of any chunkless entries just before it; the last chunk closes the
// table).  No staging, no per-query stamps.
template <int WAVES, uint32_t FEAT>
__global__ __launch_bounds__(WAVES * 64) __attribute__((amdgpu_waves_per_eu(FEAT == 0 ? 8 : 6))) void k_serve_chunks(
    BatchDev b, uint32_t grab, uint32_t gallop_blocks, uint32_t *__restrict__ out, uint64_t out_cap,
    uint64_t *__restrict__ offs) {
  __shared__ ItemLds lds[WAVES];
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  Traffic tr;
  uint32_t hint = 0, h_id0 = kInvalid, h_id1 = kInvalid, h_local = kInvalid;  // as in k_batch_chunks
  for (;;) {
    uint32_t it0 = 0;
    if (lane == 0) it0 = atomicAdd(b.head, grab);
    it0 = uniform(it0);  // lane 0's value: every lane is active here
    if (it0 >= b.items) break;
    const uint32_t it1 = min(it0 + grab, b.items);
    for (uint32_t item = it0; item < it1; ++item) {
      const uint4 info = cst(b.item_info)[item];
      const uint32_t q = uniform(info.x), local = uniform(info.y), tq = uniform(info.z), k = uniform(info.w);
      const uint32_t id0 = uniform(cst(b.sterms)[tq]), id1 = uniform(cst(b.sterms)[tq + (k > 1 ? 1 : 0)]);
      RSide r;
      r.L = cst(b.lists)[id0];
      const DList f1 = cst(b.lists)[id1];
      r.raw = nullptr;
      r.len = r.L.n;
      if (id0 != h_id0 || id1 != h_id1 || local != h_local + 1) hint = 0;
      const uint32_t cnt = chain_chunk<FEAT>(
          r, local, f1, [&](uint32_t j) -> DList { return cst(b.lists)[uniform(cst(b.sterms)[tq + 1 + j])]; }, k - 1,
          lds[w], gallop_blocks, tr, hint);
      h_id0 = id0;
      h_id1 = id1;
      h_local = local;
      bool ok = true;
      const uint32_t excl = lookback(b.state, item, b.epoch, cnt, b.err, ok);
      if (ok && uint64_t(excl) + cnt <= out_cap) {
        if (lane < cnt) out[excl + lane] = lds[w].r[lane];
        if (lane + 64 < cnt) out[excl + lane + 64] = lds[w].r[lane + 64];
      } else if (lane == 0) {
        *b.err = 1u;
      }
      // first chunk of its entry (entries may start at any chunk of their
      // query): the previous chunk belongs to an earlier entry
      const uint32_t qprev = item ? uniform(cst(b.item_info)[item - 1].x) : kInvalid;
      if (item == 0 || qprev != q) {
        const uint32_t q0 = item ? qprev + 1 : 0u;
        for (uint32_t qq = q0 + lane; qq <= q; qq += 64) offs[qq] = excl;
      }
      if (item + 1 == b.items)
        for (uint32_t qq = q + 1 + lane; qq <= b.nq; qq += 64) offs[qq] = uint64_t(excl) + cnt;
    }
  }
}

// The staged form's tail for the server, in one launch: the chunks'
// counts scanned in tiles of 1024 (a workgroup per tile, tiles numbered in
// the order workgroups start, offsets across tiles by the decoupled
// look-back of the single-pass kernel), every chunk's matches gathered to
// their final place (a wave per 256 chunks, copying only those with
// matches), and the CSR offset of every entry whose first chunk lies in
// the tile (the last tile closes the table).  It replaces the tile scan,
// the scan of tile totals, the gather and the per-entry pass, which in a
// server iteration each waited for compute units behind the other
// contexts' chunk kernels.  b.head[1] is the tile ticket (zeroed by the
// table upload); b.state holds one scan word per tile.
__global__ __launch_bounds__(256) void k_stage_tail(BatchDev b, uint32_t *__restrict__ out,
                                                     uint64_t *__restrict__ offs) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t excl_s[1024];
  __shared__ uint32_t tile_s, prefix_s, first_s;
  const uint32_t lane = lane_id(), w = threadIdx.x >> 6;
  if (threadIdx.x == 0) tile_s = atomicAdd(b.head + 1, 1u);
  __syncthreads();
  const uint32_t tile = tile_s;
  const uint32_t t0 = tile * 1024u, t1 = min(t0 + 1024u, b.items);
  uint32_t v[4], ex[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const uint32_t item = t0 + 4u * threadIdx.x + uint32_t(e);
    v[e] = item < t1 ? b.counts[item] : 0u;
  }
  const uint32_t local = v[0] + v[1] + v[2] + v[3];
  const uint32_t inc = scan_wave64(local);
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t run = inc - local;
  for (uint32_t q = 0; q < w; ++q) run += wsum[q];
  const uint32_t total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    ex[e] = run;
    excl_s[4u * threadIdx.x + uint32_t(e)] = run;
    run += v[e];
  }
  // the tile's offset: wave 0 looks back; thread 0 finds the first entry
  // that starts at or after the tile
  if (w == 0) {
    bool ok = true;
    const uint32_t e = lookback(b.state, tile, b.epoch, total, b.err, ok);
    if (lane == 0) prefix_s = ok ? e : 0u;
  } else if (threadIdx.x == 64) {
    uint32_t lo = 0, hi = b.nq + 1;  // over item_base[0 .. nq]
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (b.item_base[mid] < t0) lo = mid + 1;
      else hi = mid;
    }
    first_s = lo;
  }
  __syncthreads();
  const uint32_t P = prefix_s;
  // each wave gathers its 256 chunks' matches, chunk by chunk
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    for (uint64_t m = __ballot(v[e] != 0); m; m &= m - 1) {
      const int l = __builtin_ctzll(m);
      const uint32_t c = uint32_t(__builtin_amdgcn_readlane(int(v[e]), l));
      const uint64_t o = uint64_t(P) + uint32_t(__builtin_amdgcn_readlane(int(ex[e]), l));
      const uint32_t item = t0 + 4u * (w * 64u + uint32_t(l)) + uint32_t(e);
      const uint32_t *src = b.stage + uint64_t(item) * kBlock;
      if (lane < c) out[o + lane] = src[lane];
      if (lane + 64 < c) out[o + 64 + lane] = src[lane + 64];
    }
  }
  // offsets of the entries that start in the tile; the last tile also
  // writes those that start after the last chunk (no chunks) and the end
  const bool last = t1 == b.items;
  for (uint32_t q = first_s + threadIdx.x; q <= b.nq; q += 256) {
    const uint32_t f = b.item_base[q];
    if (f < t1) offs[q] = uint64_t(P) + excl_s[f - t0];
    else if (last) offs[q] = uint64_t(P) + total;
    else break;
  }
}

// Per-query counts and CSR offsets from the global exclusive scan.
__global__ void k_batch_finish(BatchDev b, uint64_t *__restrict__ d_counts, uint64_t *__restrict__ d_offs) {
  const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t total = *b.total;
  if (q > b.nq) return;
  auto gex = [&](uint32_t i) -> uint64_t {
    return i < b.items ? uint64_t(b.excl[i]) + b.tiles[i >> 10] : total;
  };
  if (q == b.nq) {
    d_offs[b.nq] = total;
    return;
  }
  const uint64_t o0 = gex(b.item_base[q]), o1 = gex(b.item_base[q + 1]);
  d_counts[q] = o1 - o0;
  d_offs[q] = o0;
}

}  // namespace s4

using namespace s4;

struct s4_batch {
  const s4_index *index = nullptr;
  void *mem = nullptr;
  BatchDev dev{};
  uint64_t nq = 0, results_bound = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *g_counts = nullptr, *g_offs = nullptr, *g_results = nullptr;
  s4_tuning g_tuning{};
};

static inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

template <int W, uint32_t F>
static void launch_chunks(const BatchDev &d, const s4_tuning &t, hipStream_t st) {
  // chunks per queue fetch: the tuned value, but small batches spread over
  // every resident wave (at least ~4 fetches per wave)
  const uint32_t resident = uint32_t(cu_count()) * t.groups_per_cu * W;
  const uint32_t grab = std::max<uint32_t>(1, std::min<uint32_t>(t.items_per_grab, d.items / (4 * resident)));
  const uint32_t per_group = W * grab;
  uint32_t groups = uint32_t(cu_count()) * t.groups_per_cu;
  groups = std::max<uint32_t>(1, std::min<uint32_t>(groups, (d.items + per_group - 1) / per_group));
  hipLaunchKernelGGL((k_batch_chunks<W, F>), dim3(groups), dim3(W * 64), 0, st, d, grab,
                     std::min(t.gallop_blocks, kMaxGallopBlocks - 1));
}

// The instantiation for the kinds of list the index holds (bitmap lists
// and parts never come together), with or without traffic counting.
template <int W, uint32_t C>
static void launch_chunks_feat(const BatchDev &d, const s4_tuning &t, hipStream_t st) {
  switch ((d.feat & (kFeatBitmap | kFeatPatched)) | (d.parts > 1 ? kFeatParts : 0u)) {
    case kFeatBitmap: launch_chunks<W, C | kFeatBitmap>(d, t, st); break;
    case kFeatPatched: launch_chunks<W, C | kFeatPatched>(d, t, st); break;
    case kFeatBitmap | kFeatPatched: launch_chunks<W, C | kFeatBitmap | kFeatPatched>(d, t, st); break;
    case kFeatParts: launch_chunks<W, C | kFeatParts>(d, t, st); break;
    case kFeatParts | kFeatPatched: launch_chunks<W, C | kFeatParts | kFeatPatched>(d, t, st); break;
    default: launch_chunks<W, C>(d, t, st); break;
  }
}
template <int W>
static void launch_chunks_w(const BatchDev &d, const s4_tuning &t, hipStream_t st) {
  if (d.count)
    launch_chunks_feat<W, kFeatCount>(d, t, st);
  else
    launch_chunks_feat<W, 0>(d, t, st);
}

template <int W, uint32_t F>
static void launch_serve(const BatchDev &d, const s4_tuning &t, uint32_t *out, uint64_t out_cap, uint64_t *offs,
                         hipStream_t st) {
  const uint32_t resident = uint32_t(cu_count()) * t.groups_per_cu * W;
  const uint32_t grab = std::max<uint32_t>(1, std::min<uint32_t>(t.items_per_grab, d.items / (4 * resident)));
  const uint32_t per_group = W * grab;
  uint32_t groups = uint32_t(cu_count()) * t.groups_per_cu;
  groups = std::max<uint32_t>(1, std::min<uint32_t>(groups, (d.items + per_group - 1) / per_group));
  hipLaunchKernelGGL((k_serve_chunks<W, F>), dim3(groups), dim3(W * 64), 0, st, d, grab,
                     std::min(t.gallop_blocks, kMaxGallopBlocks), out, out_cap, offs);
}

template <int W>
static void launch_serve_w(const BatchDev &d, const s4_tuning &t, uint32_t *out, uint64_t out_cap, uint64_t *offs,
                           hipStream_t st) {
  switch (d.feat & (kFeatBitmap | kFeatPatched)) {
    case kFeatBitmap: launch_serve<W, kFeatBitmap>(d, t, out, out_cap, offs, st); break;
    case kFeatPatched: launch_serve<W, kFeatPatched>(d, t, out, out_cap, offs, st); break;
    case kFeatBitmap | kFeatPatched: launch_serve<W, kFeatBitmap | kFeatPatched>(d, t, out, out_cap, offs, st); break;
    default: launch_serve<W, 0>(d, t, out, out_cap, offs, st); break;
  }
}

namespace s4 {
uint64_t single_pass_max_items() {
  const s4_tuning t = tuning();
  return uint64_t(cu_count()) * t.groups_per_cu * t.waves_per_group;
}

int enqueue_serve_dev(const BatchDev &d, uint32_t *out, uint64_t out_cap, uint64_t *d_offs, hipStream_t st) {
  if (!d.items || !d.state || !d.err || d.epoch == 0 || d.epoch > kMaxEpoch)
    return fail(S4_EINVAL, "single-pass run: needs chunks, scan words and an epoch in 1 .. 2^30 - 1");
  const s4_tuning t = tuning();
  switch (t.waves_per_group) {
    case 1: launch_serve_w<1>(d, t, out, out_cap, d_offs, st); break;
    case 2: launch_serve_w<2>(d, t, out, out_cap, d_offs, st); break;
    case 8: launch_serve_w<8>(d, t, out, out_cap, d_offs, st); break;
    default: launch_serve_w<4>(d, t, out, out_cap, d_offs, st); break;
  }
  S4_HIP(hipGetLastError());
  return S4_OK;
}

// Chunk records from one entry per query: chunk i belongs to the entry q
// with item_base[q] <= i < item_base[q + 1] (the largest q with
// item_base[q] <= i, which passes over entries without chunks); its
// record is {q, the entry's first chunk + i - item_base[q], first term,
// terms}.
__global__ __launch_bounds__(256) void k_expand_items(BatchDev b, const uint4 *__restrict__ qinfo,
                                                      uint4 *__restrict__ records) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= b.items) return;
  uint32_t lo = 0, hi = b.nq;  // item_base[lo] <= i < item_base[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (b.item_base[mid] <= i) lo = mid;
    else hi = mid;
  }
  const uint4 e = qinfo[lo];
  records[i] = make_uint4(lo, e.x + i - b.item_base[lo], e.y, e.z);
}

int enqueue_expand_items(const BatchDev &d, const uint4 *qinfo, uint4 *records, hipStream_t st) {
  if (!d.items || !d.nq || !d.item_base || !qinfo || !records)
    return fail(S4_EINVAL, "chunk records: needs chunks, entries and tables");
  hipLaunchKernelGGL(k_expand_items, dim3((d.items + 255) / 256), dim3(256), 0, st, d, qinfo, records);
  S4_HIP(hipGetLastError());
  return S4_OK;
}

// The server's staged iteration: chunk kernel, then k_stage_tail (needs
// d.state, d.err and an epoch, as the single-pass form).
int enqueue_staged_serve_dev(const BatchDev &d, uint32_t *out, uint64_t *d_offs, hipStream_t st) {
  if (!d.items || !d.state || !d.err || d.epoch == 0 || d.epoch > kMaxEpoch)
    return fail(S4_EINVAL, "staged server run: needs chunks, scan words and an epoch in 1 .. 2^30 - 1");
  const s4_tuning t = tuning();
  switch (t.waves_per_group) {
    case 1: launch_chunks_w<1>(d, t, st); break;
    case 2: launch_chunks_w<2>(d, t, st); break;
    case 8: launch_chunks_w<8>(d, t, st); break;
    default: launch_chunks_w<4>(d, t, st); break;
  }
  hipLaunchKernelGGL(k_stage_tail, dim3(uint32_t((d.items + 1023) / 1024)), dim3(256), 0, st, d, out, d_offs);
  S4_HIP(hipGetLastError());
  return S4_OK;
}

// Enqueue one run of a batch described by d on st.
int enqueue_batch_dev(const BatchDev &d, uint64_t *d_counts, uint64_t *d_offs, uint32_t *d_results, hipStream_t st,
                      bool begin) {
  const s4_tuning t = tuning();
  if (begin) {
    const uint32_t begin_groups = std::max<uint32_t>(1, std::min<uint32_t>(1024, (d.nq + 255) / 256));
    hipLaunchKernelGGL(k_batch_begin, dim3(begin_groups), dim3(256), 0, st, d);
  }
  if (d.items) {
    switch (t.waves_per_group) {
      case 1: launch_chunks_w<1>(d, t, st); break;
      case 2: launch_chunks_w<2>(d, t, st); break;
      case 8: launch_chunks_w<8>(d, t, st); break;
      default: launch_chunks_w<4>(d, t, st); break;
    }
  }
  S4_HIP(hipGetLastError());
  int rc = scan_and_compact(d.stage, d.counts, d.items, d.excl, d.tiles, d.ntiles, d.total, d_results, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_batch_finish, dim3(uint32_t((d.nq + 1 + 255) / 256)), dim3(256), 0, st, d, d_counts, d_offs);
  S4_HIP(hipGetLastError());
  return S4_OK;
}
}  // namespace s4

static int enqueue_batch(s4_batch *b, uint64_t *d_counts, uint64_t *d_offs, uint32_t *d_results, hipStream_t st) {
  return enqueue_batch_dev(b->dev, d_counts, d_offs, d_results, st);
}

static void drop_graph(s4_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// First and last value of each of n lists (one wave each; row 0 decodes
// the first block, patching it when the list is patched).
__global__ __launch_bounds__(256) void k_list_bounds(const DList *__restrict__ lists, uint32_t n,
                                                      uint32_t *__restrict__ bounds) {
  __shared__ __align__(16) uint32_t scratch[4][kBlock];
  const uint32_t w = threadIdx.x >> 6, lane = lane_id();
  const uint32_t i = blockIdx.x * 4 + w;
  if (i >= n) return;
  const DList L = lists[i];
  uint32_t x0[4], x1[4];
  decode_row<true>(L, 0, L.nb > 0 && lane < 16, lane & 15u, x0, x1, scratch[w]);
  if (lane == 0) {
    const uint32_t first = L.nb ? x0[0] : (L.t ? L.tail[0] : 0u);
    const uint32_t last = L.t ? L.tail[L.t - 1] : (L.nb ? L.bmax[L.nb - 1] : 0u);
    bounds[2 * i] = first;
    bounds[2 * i + 1] = last;
  }
}

// Index over count serialized lists; with gap > 0 (hyb+m2) the lists whose
// average gap universe / n is at most gap, and that are strictly
// increasing, are held as bitmaps over [0, universe), the rest compressed.
static int index_build(const uint8_t *encs, const uint64_t *enc_offsets, uint64_t count, uint64_t universe,
                       uint32_t gap, hipStream_t st, s4_index **out) {
  if (!out || !enc_offsets || (count && !encs)) return fail(S4_EINVAL, "null argument");
  if (count > 0xFFFFFFFFull) return fail(S4_EINVAL, "too many lists");
  if (gap && (universe == 0 || universe > (1ull << 32)))
    return fail(S4_EINVAL, "universe must be in [1, 2^32] for a hybrid index");
  int rc = ensure_device();
  if (rc) return rc;
  std::vector<StreamView> views(count);
  for (uint64_t i = 0; i < count; ++i) {
    if (enc_offsets[i + 1] < enc_offsets[i]) return fail(S4_EINVAL, "offsets decrease");
    rc = parse_stream(encs + enc_offsets[i], size_t(enc_offsets[i + 1] - enc_offsets[i]), &views[i]);
    if (rc) return fail(rc, "list " + std::to_string(i) + ": " + s4_last_error());
  }
  s4_index *ix = new (std::nothrow) s4_index;
  if (!ix) return fail(S4_ENOMEM, "handle allocation failed");
  auto drop = [&](int code) {
    if (ix->arena) (void)hipFree(ix->arena);
    if (ix->bitmaps) (void)hipFree(ix->bitmaps);
    if (ix->desc) (void)hipFree(ix->desc);
    delete ix;
    return code;
  };
  ix->count = count;
  ix->universe = universe;
  ix->gap = gap;
  ix->kinds.assign(count, 0);
  Upload uc, ub;
  std::vector<uint64_t> slot(count);
  for (uint64_t i = 0; i < count; ++i) {
    const StreamView &v = views[i];
    const bool bitmap = (v.flags & 1u) && hyb_is_bitmap(v.n, universe, gap);
    ix->kinds[i] = bitmap ? 1 : 0;
    Upload &u = bitmap ? ub : uc;
    slot[i] = u.views.size();
    u.views.push_back(v);
  }
  std::vector<DList> dc, db;
  if (!uc.views.empty()) {
    rc = build_arena(uc, st, &ix->arena, &dc);
    if (rc) return drop(rc);
  }
  if (!ub.views.empty()) {
    rc = build_bitmaps(ub, universe, st, &ix->bitmaps, &db, &ix->bitmap_bytes, &ix->select_bytes);
    if (rc) return drop(rc);
  }
  ix->lists.resize(count);
  for (uint64_t i = 0; i < count; ++i) ix->lists[i] = ix->kinds[i] ? db[slot[i]] : dc[slot[i]];
  hipError_t e = hipMalloc(&ix->desc, sizeof(DList) * std::max<uint64_t>(count, 1));
  if (e != hipSuccess) return drop(fail(S4_ENOMEM, "descriptor table allocation failed"));
  if (count) e = hipMemcpyAsync(ix->desc, ix->lists.data(), sizeof(DList) * count, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return drop(hip_fail(e, "index build"));
  ix->d_lists = static_cast<const DList *>(ix->desc);
  ix->lengths.resize(count);
  ix->flags.resize(count);
  ix->pw.resize(count);
  ix->data_bytes.resize(count);
  for (uint64_t i = 0; i < count; ++i) {
    const StreamView &v = views[i];
    ix->lengths[i] = v.n;
    ix->flags[i] = v.flags;
    ix->data_bytes[i] = v.data_bytes();
    ix->total_ints += v.n;
    if (ix->kinds[i]) {
      ix->pw[i] = 0;
      ++ix->bitmap_lists;
    } else {
      ix->pw[i] = v.pw;
      ix->payload_bytes += v.data_bytes();
      ix->index_bytes += uint64_t(v.nb) * (4 + 4 + 16 + (v.patched() ? 16 : 0));
    }
  }
  ix->payload_bytes += ix->bitmap_bytes;
  ix->index_bytes += ix->select_bytes;
  ix->feat = (ix->bitmap_lists ? kFeatBitmap : 0u);
  for (uint64_t i = 0; i < count; ++i)
    if (!ix->kinds[i] && views[i].patched()) ix->feat |= kFeatPatched;
  *out = ix;
  return S4_OK;
}

extern "C" {

int s4_index_build(const uint8_t *encs, const uint64_t *enc_offsets, uint64_t count, void *stream,
                   s4_index **out) {
  return index_build(encs, enc_offsets, count, 0, 0, as_stream(stream), out);
}

int s4_partition_offsets(const uint32_t *in, const uint64_t *in_offsets, uint64_t count, uint32_t parts,
                         uint64_t universe, uint64_t *sub_offsets) {
  if (!in_offsets || !sub_offsets || (count && !in)) return fail(S4_EINVAL, "null argument");
  if (parts == 0 || universe == 0 || universe > (1ull << 32) || parts > universe)
    return fail(S4_EINVAL, "need 1 <= parts <= universe <= 2^32");
  for (uint64_t t = 0; t < count; ++t) {
    const uint64_t a = in_offsets[t], b = in_offsets[t + 1];
    if (b < a) return fail(S4_EINVAL, "offsets decrease");
    if (b > a && in[b - 1] >= universe) return fail(S4_EINVAL, "list " + std::to_string(t) + " reaches the universe");
    sub_offsets[t * parts] = a;
    for (uint32_t p = 1; p < parts; ++p) {
      const uint64_t edge = uint64_t(p) * universe / parts;  // part p starts at floor(p U / parts)
      sub_offsets[t * parts + p] = uint64_t(std::lower_bound(in + a, in + b, edge, [](uint32_t v, uint64_t e) {
                                              return uint64_t(v) < e;
                                            }) - in);
    }
  }
  sub_offsets[count * parts] = count ? in_offsets[count] : 0;
  return S4_OK;
}

int s4_index_build_parts(const uint8_t *encs, const uint64_t *enc_offsets, uint64_t count, uint32_t parts,
                         void *stream, s4_index **out) {
  if (!out) return fail(S4_EINVAL, "null argument");
  if (parts < 1 || parts > 1024) return fail(S4_EINVAL, "parts must be in [1, 1024]");
  if (count * parts > 0xFFFFFFFFull) return fail(S4_EINVAL, "too many lists");
  s4_index *ix = nullptr;
  int rc = index_build(encs, enc_offsets, count * parts, 0, 0, as_stream(stream), &ix);
  if (rc || parts == 1) {
    if (!rc) *out = ix;
    return rc;
  }
  // each list's parts must hold ascending, disjoint value ranges: results
  // are joined in part order
  const uint64_t ns = count * parts;
  uint32_t *d_bounds = nullptr;
  std::vector<uint32_t> bounds(2 * ns);
  hipError_t e = hipMalloc(&d_bounds, 8 * std::max<uint64_t>(ns, 1));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_list_bounds, dim3(uint32_t((ns + 3) / 4)), dim3(256), 0, as_stream(stream), ix->d_lists,
                       uint32_t(ns), d_bounds);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(bounds.data(), d_bounds, 8 * ns, hipMemcpyDeviceToHost, as_stream(stream));
    if (e == hipSuccess) e = hipStreamSynchronize(as_stream(stream));
    (void)hipFree(d_bounds);
  }
  if (e != hipSuccess) {
    s4_index_free(ix);
    return hip_fail(e, "partition check");
  }
  ix->part_len = ix->lengths;
  ix->parts = parts;
  ix->count = count;
  ix->lengths.assign(count, 0);
  std::vector<uint32_t> flags(count, 1u);
  for (uint64_t t = 0; t < count; ++t) {
    bool any = false;
    uint32_t last = 0;
    for (uint32_t p = 0; p < parts; ++p) {
      const uint64_t s = t * parts + p;
      ix->lengths[t] += ix->part_len[s];
      flags[t] &= ix->flags[s];
      if (!ix->part_len[s]) continue;
      if (any && bounds[2 * s] <= last) {
        s4_index_free(ix);
        return fail(S4_EINVAL, "list " + std::to_string(t) + ": part " + std::to_string(p) +
                                   " does not start above the previous part");
      }
      any = true;
      last = bounds[2 * s + 1];
    }
  }
  ix->flags = flags;
  ix->kinds.assign(count, 0);
  *out = ix;
  return S4_OK;
}

int s4_index_build_hybrid(const uint8_t *encs, const uint64_t *enc_offsets, uint64_t count, uint64_t universe,
                          uint32_t bitmap_gap, void *stream, s4_index **out) {
  if (bitmap_gap == 0) return fail(S4_EINVAL, "bitmap_gap must be > 0 (s4_index_build builds without bitmaps)");
  return index_build(encs, enc_offsets, count, universe, bitmap_gap, as_stream(stream), out);
}

int s4_index_kinds(const s4_index *ix, uint8_t *kinds) {
  if (!ix || (ix->count && !kinds)) return fail(S4_EINVAL, "null argument");
  std::copy(ix->kinds.begin(), ix->kinds.end(), kinds);
  return S4_OK;
}

int s4_index_hybrid_info(const s4_index *ix, uint64_t *universe, uint32_t *bitmap_gap, uint64_t *bitmap_lists,
                         uint64_t *bitmap_bytes, uint64_t *select_bytes) {
  if (!ix) return fail(S4_EINVAL, "null index");
  if (universe) *universe = ix->universe;
  if (bitmap_gap) *bitmap_gap = ix->gap;
  if (bitmap_lists) *bitmap_lists = ix->bitmap_lists;
  if (bitmap_bytes) *bitmap_bytes = ix->bitmap_bytes;
  if (select_bytes) *select_bytes = ix->select_bytes;
  return S4_OK;
}

int s4_index_free(s4_index *ix) {
  if (!ix) return S4_OK;
  hipError_t e = hipSuccess;
  for (void *p : {ix->arena, ix->bitmaps, ix->desc})
    if (p) {
      const hipError_t f = hipFree(p);
      if (e == hipSuccess) e = f;
    }
  delete ix;
  if (e != hipSuccess) return hip_fail(e, "hipFree");
  return S4_OK;
}

int s4_index_lengths(const s4_index *ix, uint64_t *lengths) {
  if (!ix || (ix->count && !lengths)) return fail(S4_EINVAL, "null argument");
  std::copy(ix->lengths.begin(), ix->lengths.end(), lengths);
  return S4_OK;
}

int s4_index_info(const s4_index *ix, uint64_t *count, uint64_t *total_ints, uint64_t *payload_bytes,
                  uint64_t *index_bytes) {
  if (!ix) return fail(S4_EINVAL, "null index");
  if (count) *count = ix->count;
  if (total_ints) *total_ints = ix->total_ints;
  if (payload_bytes) *payload_bytes = ix->payload_bytes;
  if (index_bytes) *index_bytes = ix->index_bytes;
  return S4_OK;
}

int s4_index_list(const s4_index *ix, uint64_t i, s4_list **out) {
  if (!ix || !out) return fail(S4_EINVAL, "null argument");
  if (i >= ix->count) return fail(S4_ERANGE, "list id out of range");
  if (ix->parts > 1) return fail(S4_EINVAL, "a partitioned index holds each list in parts");
  if (ix->kinds[i]) return fail(S4_EINVAL, "list " + std::to_string(i) + " is held as a bitmap (hybrid index)");
  s4_list *l = new (std::nothrow) s4_list;
  if (!l) return fail(S4_ENOMEM, "handle allocation failed");
  const DList &d = ix->lists[i];
  l->d = d;
  l->n = d.n;
  l->nb = d.nb;
  l->t = d.t;
  l->flags = ix->flags[i];
  l->arena = nullptr;
  l->pw = ix->pw[i];
  l->payload_bytes = ix->data_bytes[i];
  l->index_bytes = uint64_t(d.nb) * (4 + 4 + 16 + (is_patched(d) ? 16 : 0));
  *out = l;
  return S4_OK;
}

int s4_batch_plan(const s4_index *ix, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                  void *stream, s4_batch **out) {
  if (!ix || !h_q_offsets || !out || (nq && !h_terms)) return fail(S4_EINVAL, "null argument");
  if (nq >= 0xFFFFFFFFull) return fail(S4_EINVAL, "too many queries");
  int rc = ensure_device();
  if (rc) return rc;
  const uint64_t nterms = h_q_offsets[nq];
  const uint32_t P = ix->parts;
  if (nterms * P >= 0xFFFFFFFFull) return fail(S4_EINVAL, "too many terms");
  std::vector<uint32_t> sterms(nterms * P);
  std::vector<uint32_t> qoff(nq + 1), item_base(nq + 1);
  std::vector<uint32_t> item_info, item_rank, part_base;
  uint64_t items = 0, bound = 0;
  if (P > 1) {
    // doc-ID partitioned index: query q runs once per part p, with terms
    // (descriptors t * P + p) in that part's length order at
    // sterms[P qoff[q] + p k ..]; chunks are numbered query-major (slots,
    // the result order) and queued part-major
    std::vector<uint64_t> qitems(nq * P);
    for (uint64_t q = 0; q < nq; ++q) {
      const uint64_t a = h_q_offsets[q], b = h_q_offsets[q + 1];
      if (b < a || b > nterms) return fail(S4_EINVAL, "query offsets not increasing");
      const uint64_t k = b - a;
      if (k == 0 || k > kMaxTerms + 1) return fail(S4_EINVAL, "query " + std::to_string(q) + ": need 1..33 terms");
      for (uint64_t t = a; t < b; ++t) {
        if (h_terms[t] >= ix->count) return fail(S4_EINVAL, "query " + std::to_string(q) + ": term out of range");
        if (k > 1 && !(ix->flags[h_terms[t]] & 1u))
          return fail(S4_EUNSORTED, "list " + std::to_string(h_terms[t]) + " is not strictly increasing");
      }
      qoff[q] = uint32_t(a);
      item_base[q] = uint32_t(items);
      for (uint32_t p = 0; p < P; ++p) {
        uint32_t *seg = sterms.data() + P * a + p * k;
        for (uint64_t j = 0; j < k; ++j) seg[j] = uint32_t(h_terms[a + j] * uint64_t(P) + p);
        std::stable_sort(seg, seg + k, [&](uint32_t x, uint32_t y) { return ix->part_len[x] < ix->part_len[y]; });
        const uint64_t m = ix->part_len[seg[0]];
        qitems[q * P + p] = (m + kBlock - 1) / kBlock;
        items += qitems[q * P + p];
        bound += m;
      }
      if (items >= 0xFFFFFFFFull / kBlock || bound >= 0xFFFFFFFFull)
        return fail(S4_EINVAL, "batch too large for one plan; split it");
    }
    qoff[nq] = uint32_t(nterms);
    item_base[nq] = uint32_t(items);
    item_info.resize(4 * items);
    item_rank.resize(items);
    part_base.assign(P + 1, 0);
    uint64_t it = 0;
    for (uint32_t p = 0; p < P; ++p) {
      part_base[p] = uint32_t(it);
      for (uint64_t q = 0; q < nq; ++q) {
        uint64_t slot = item_base[q];
        for (uint32_t pp = 0; pp < p; ++pp) slot += qitems[q * P + pp];
        const uint32_t k = uint32_t(h_q_offsets[q + 1] - h_q_offsets[q]);
        for (uint64_t i = 0; i < qitems[q * P + p]; ++i, ++it) {
          item_info[4 * it] = uint32_t(q);
          item_info[4 * it + 1] = uint32_t(i);
          item_info[4 * it + 2] = uint32_t(P * h_q_offsets[q] + uint64_t(p) * k);
          item_info[4 * it + 3] = k;
          item_rank[it] = uint32_t(slot + i);
        }
      }
    }
    part_base[P] = uint32_t(it);
  }
  for (uint64_t q = 0; P == 1 && q < nq; ++q) {
    const uint64_t a = h_q_offsets[q], b = h_q_offsets[q + 1];
    if (b < a || b > nterms) return fail(S4_EINVAL, "query offsets not increasing");
    const uint64_t k = b - a;
    if (k == 0 || k > kMaxTerms + 1) return fail(S4_EINVAL, "query " + std::to_string(q) + ": need 1..33 terms");
    for (uint64_t t = a; t < b; ++t) {
      if (h_terms[t] >= ix->count) return fail(S4_EINVAL, "query " + std::to_string(q) + ": term out of range");
      if (k > 1 && !(ix->flags[h_terms[t]] & 1u))
        return fail(S4_EUNSORTED, "list " + std::to_string(h_terms[t]) + " is not strictly increasing");
      sterms[t] = h_terms[t];
    }
    std::stable_sort(sterms.begin() + a, sterms.begin() + b,
                     [&](uint32_t x, uint32_t y) { return ix->lengths[x] < ix->lengths[y]; });
    qoff[q] = uint32_t(a);
    item_base[q] = uint32_t(items);
    const uint64_t m = ix->lengths[sterms[a]];
    items += (m + kBlock - 1) / kBlock;
    bound += m;
    if (items >= 0xFFFFFFFFull / kBlock || bound >= 0xFFFFFFFFull)
      return fail(S4_EINVAL, "batch too large for one plan; split it");
  }
  if (P == 1) {
    qoff[nq] = uint32_t(nterms);
    item_base[nq] = uint32_t(items);
    item_info.resize(4 * items);
  }
  for (uint64_t q = 0; P == 1 && q < nq; ++q)
    for (uint32_t i = item_base[q]; i < item_base[q + 1]; ++i) {
      item_info[4 * size_t(i)] = uint32_t(q);
      item_info[4 * size_t(i) + 1] = i - item_base[q];
      item_info[4 * size_t(i) + 2] = qoff[q];
      item_info[4 * size_t(i) + 3] = uint32_t(h_q_offsets[q + 1] - h_q_offsets[q]);
    }
  const uint32_t ntiles = uint32_t((items + 1023) / 1024);
  // one device allocation for every table
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 4), 256);
    return o;
  };
  const size_t o_sterms = take(4 * nterms * P), o_qoff = take(4 * (nq + 1)), o_ib = take(4 * (nq + 1)),
               o_iq = take(16 * items), o_stage = take(4 * kBlock * items), o_counts = take(4 * items),
               o_excl = take(4 * items), o_tiles = take(4 * (ntiles + 1)), o_ctrl = take(64),
               o_qtick = take(8 * nq), o_heads = take(4 * kHeadStride * std::max<uint32_t>(P, kSubQueues)),
               o_rank = take(4 * item_rank.size()),
               o_pbase = take(4 * part_base.size());
  s4_batch *bt = new (std::nothrow) s4_batch;
  if (!bt) return fail(S4_ENOMEM, "handle allocation failed");
  if (hipMalloc(&bt->mem, off) != hipSuccess) {
    delete bt;
    return fail(S4_ENOMEM, "batch tables: hipMalloc of " + std::to_string(off) + " bytes failed");
  }
  char *m = static_cast<char *>(bt->mem);
  hipStream_t st = as_stream(stream);
  hipError_t e = hipSuccess;
  auto up = [&](size_t o, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(m + o, src, bytes, hipMemcpyHostToDevice, st);
  };
  up(o_sterms, sterms.data(), 4 * nterms * P);
  up(o_rank, item_rank.data(), 4 * item_rank.size());
  up(o_pbase, part_base.data(), 4 * part_base.size());
  up(o_qoff, qoff.data(), 4 * (nq + 1));
  up(o_ib, item_base.data(), 4 * (nq + 1));
  up(o_iq, item_info.data(), 16 * items);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipFree(bt->mem);
    delete bt;
    return hip_fail(e, "batch plan upload");
  }
  BatchDev &d = bt->dev;
  d.lists = ix->d_lists;
  d.feat = ix->feat;
  d.sterms = reinterpret_cast<const uint32_t *>(m + o_sterms);
  d.qoff = reinterpret_cast<const uint32_t *>(m + o_qoff);
  d.item_base = reinterpret_cast<const uint32_t *>(m + o_ib);
  d.item_info = reinterpret_cast<const uint4 *>(m + o_iq);
  d.stage = reinterpret_cast<uint32_t *>(m + o_stage);
  d.counts = reinterpret_cast<uint32_t *>(m + o_counts);
  d.excl = reinterpret_cast<uint32_t *>(m + o_excl);
  d.tiles = reinterpret_cast<uint32_t *>(m + o_tiles);
  d.head = reinterpret_cast<uint32_t *>(m + o_heads);
  d.total = reinterpret_cast<uint64_t *>(m + o_ctrl + 8);
  d.start = reinterpret_cast<uint64_t *>(m + o_ctrl + 16);
  d.qtick = reinterpret_cast<uint64_t *>(m + o_qtick);
  d.stats = reinterpret_cast<uint64_t *>(m + o_ctrl + 24);
  d.parts = P;
  d.item_rank = P > 1 ? reinterpret_cast<const uint32_t *>(m + o_rank) : nullptr;
  d.part_base = P > 1 ? reinterpret_cast<const uint32_t *>(m + o_pbase) : nullptr;
  d.items = uint32_t(items);
  d.nq = uint32_t(nq);
  d.ntiles = ntiles;
  bt->index = ix;
  bt->nq = nq;
  bt->results_bound = bound;
  *out = bt;
  return S4_OK;
}

int s4_batch_free(s4_batch *b) {
  if (!b) return S4_OK;
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  hipError_t e = b->mem ? hipFree(b->mem) : hipSuccess;
  delete b;
  if (e != hipSuccess) return hip_fail(e, "hipFree");
  return S4_OK;
}

uint64_t s4_batch_results_bound(const s4_batch *b) { return b ? b->results_bound : 0; }

int s4_batch_run(s4_batch *b, uint64_t *d_counts, uint64_t *d_res_offsets, uint32_t *d_results, uint64_t results_cap,
                 int use_graph, void *stream) {
  if (!b || !d_counts || !d_res_offsets || (!d_results && b->results_bound))
    return fail(S4_EINVAL, "null argument");
  if (results_cap < b->results_bound) return fail(S4_ERANGE, "results_cap below s4_batch_results_bound");
  int rc = ensure_device();
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  if (!use_graph) return enqueue_batch(b, d_counts, d_res_offsets, d_results, st);
  const s4_tuning t = tuning();
  const bool stale = !b->exec || b->g_counts != d_counts || b->g_offs != d_res_offsets ||
                     b->g_results != d_results || std::memcmp(&b->g_tuning, &t, sizeof t) != 0;
  if (stale) {
    drop_graph(b);
    if (!b->cap_stream) S4_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    S4_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = enqueue_batch(b, d_counts, d_res_offsets, d_results, b->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(b);
      return hip_fail(e, "hipGraphInstantiate");
    }
    b->g_counts = d_counts;
    b->g_offs = d_res_offsets;
    b->g_results = d_results;
    b->g_tuning = t;
  }
  S4_HIP(hipGraphLaunch(b->exec, st));
  return S4_OK;
}

int s4_batch_set_counting(s4_batch *b, int on) {
  if (!b) return fail(S4_EINVAL, "null batch");
  const uint32_t c = on ? 1u : 0u;
  if (b->dev.count != c) {
    b->dev.count = c;
    drop_graph(b);  // the kernels' arguments changed
  }
  return S4_OK;
}

int s4_batch_traffic(const s4_batch *b, uint64_t *bytes, uint64_t *blocks, void *stream) {
  if (!b || !bytes || !blocks) return fail(S4_EINVAL, "null argument");
  uint64_t v[2] = {0, 0};
  S4_HIP(hipMemcpyAsync(v, b->dev.stats, sizeof v, hipMemcpyDeviceToHost, as_stream(stream)));
  S4_HIP(hipStreamSynchronize(as_stream(stream)));
  *bytes = v[0];
  *blocks = v[1];
  return S4_OK;
}

int s4_batch_query_ticks(const s4_batch *b, uint64_t *ticks, void *stream) {
  if (!b || (b->nq && !ticks)) return fail(S4_EINVAL, "null argument");
  if (!b->nq) return S4_OK;
  S4_HIP(hipMemcpyAsync(ticks, b->dev.qtick, 8 * b->nq, hipMemcpyDeviceToHost, as_stream(stream)));
  S4_HIP(hipStreamSynchronize(as_stream(stream)));
  return S4_OK;
}

int s4_batch_autotune(s4_batch *b, uint64_t *d_counts, uint64_t *d_res_offsets, uint32_t *d_results,
                      uint64_t results_cap, int reps, void *stream, s4_tuning *best, double *best_ms) {
  if (!b || !best) return fail(S4_EINVAL, "null argument");
  if (reps < 1) reps = 1;
  hipStream_t st = as_stream(stream);
  hipEvent_t e0, e1;
  S4_HIP(hipEventCreate(&e0));
  S4_HIP(hipEventCreate(&e1));
  auto measure = [&](const s4_tuning &t, double *ms) -> int {
    int rc = s4_set_tuning(&t);
    if (rc) return rc;
    rc = s4_batch_run(b, d_counts, d_res_offsets, d_results, results_cap, 0, stream);  // warm-up
    if (rc) return rc;
    S4_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) {
      rc = s4_batch_run(b, d_counts, d_res_offsets, d_results, results_cap, 0, stream);
      if (rc) return rc;
    }
    S4_HIP(hipEventRecord(e1, st));
    S4_HIP(hipEventSynchronize(e1));
    float f = 0;
    S4_HIP(hipEventElapsedTime(&f, e0, e1));
    *ms = double(f) / reps;
    return S4_OK;
  };
  s4_tuning cur = tuning();
  double cur_ms = 0;
  int rc = measure(cur, &cur_ms);
  const std::vector<uint32_t> gallops = {4, 16, 64, 256, 512};
  const std::vector<uint32_t> waves = {1, 2, 4, 8};
  const std::vector<uint32_t> groups = {2, 4, 8, 16};
  const std::vector<uint32_t> grabs = {1, 4, 8, 16, 32, 64};
  for (int round = 0; round < 2 && rc == S4_OK; ++round) {
    for (int dim = 0; dim < 4 && rc == S4_OK; ++dim) {
      const std::vector<uint32_t> &vals = dim == 0 ? gallops : dim == 1 ? waves : dim == 2 ? groups : grabs;
      for (uint32_t v : vals) {
        s4_tuning t = cur;
        (dim == 0 ? t.gallop_blocks : dim == 1 ? t.waves_per_group : dim == 2 ? t.groups_per_cu : t.items_per_grab) = v;
        if (std::memcmp(&t, &cur, sizeof t) == 0) continue;
        double ms = 0;
        rc = measure(t, &ms);
        if (rc) break;
        if (ms < cur_ms) {
          cur = t;
          cur_ms = ms;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  rc = s4_set_tuning(&cur);
  if (rc) return rc;
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return S4_OK;
}

}  // extern "C"

// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/s4.h"

namespace s4 {

constexpr uint32_t kMagic = 0x34443453u;  // "S4D4"
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeaderBytes = 32;
constexpr uint32_t kBlock = 128;          // integers per block (Sec. 4.3)
constexpr uint32_t kPayloadPadBytes = 64; // lets extraction read 3 rows past any block
constexpr uint32_t kMaxGallopBlocks = 512;
// Chunk work queues: an unpartitioned batch splits its chunks into
// kSubQueues contiguous slices (one per XCD), and every queue head sits
// kHeadStride words (256 bytes) from the next: atomics on one word are
// served one after another device-wide (about 11 ns each measured), so
// thousands of waves fetching from one head wait on each other.
constexpr uint32_t kSubQueues = 8;
constexpr uint32_t kHeadStride = 64;
constexpr uint32_t kMaxTerms = 32;  // lists after the shortest one in a conjunction
constexpr uint32_t kPage = 512;     // blocks whose exceptions a patched stream pools
constexpr uint16_t kFlagPatched = 8;  // stream flag bit 3: S4-FastPFOR

// Device view of one list: structure of arrays in HBM.
struct DList {
  const uint8_t *widths;    // [nb]
  const uint32_t *offs;     // [nb]  word offset of block k in payload (multiple of 4)
  const uint32_t *payload;  // [pw] + padding, 16-byte aligned
  const uint32_t *bmax;     // [nb]  x[128k + 127]
  const uint4 *seeds;       // [nb]  x[128k-4 .. 128k-1]
  const uint32_t *tail;     // [t]; patched lists: then their exception data (exc_records)
  uint64_t n;
  uint32_t nb;
  uint32_t t;
  uint32_t mode;  // differential form, S4_DELTA_*, or kBitmapList
  uint32_t aux;   // bitmap lists: bitmap length in 32-bit words; compressed lists: 1 if patched
};
// The descriptor stays at 72 bytes: chunk kernels copy several per chunk,
// and a larger one measurably slows them.
static_assert(sizeof(DList) == 72, "list descriptor size");

__host__ __device__ inline bool is_patched(const DList &L) { return L.mode < 4u && L.aux != 0; }
// Patched lists (S4-FastPFOR, Sec. 4.4): after the raw tail, padded to 16
// bytes, one record per block {c | d << 8 | b' << 16, byte offset of its
// positions, word offset of its page's array for d, index of its first
// exception there} (offsets into exc_data), then the positions bytes and
// the arrays (each followed by one zero word).
__host__ __device__ inline const uint4 *exc_records(const DList &L) {
  return reinterpret_cast<const uint4 *>(L.tail + ((L.t + 3u) & ~3u));
}
__host__ __device__ inline const uint32_t *exc_data(const DList &L) {
  return reinterpret_cast<const uint32_t *>(exc_records(L) + L.nb);
}
// DList.mode of a list stored as a bitmap (hybrid index): payload holds
// ceil(U / 32) words, bit x of the list being bit x % 32 of word x / 32;
// bmax holds one select sample per 128 values (chunk k: the value of rank
// 128 k, so the chunk starts at that bit); nb = ceil(n / 128), t = 0;
// widths, offs, seeds and tail are null.
constexpr uint32_t kBitmapList = 8;

// Parsed header of a serialized stream (host).
struct StreamView {
  uint64_t n = 0, pw = 0;
  uint32_t nb = 0, t = 0;
  uint16_t flags = 0;
  const uint8_t *widths = nullptr;   // packed widths (b' for patched streams)
  const uint8_t *payload = nullptr;  // byte pointer (4-byte aligned within the stream)
  const uint8_t *tail = nullptr;
  // patched streams: the pages, their size, and what the device copy of the
  // exceptions needs (positions, array words incl. one pad word per array)
  const uint8_t *pages = nullptr;
  uint64_t pages_bytes = 0, x_positions = 0, x_array_words = 0;
  bool patched() const { return (flags & kFlagPatched) != 0; }
  // bytes of the stream that are data: width bytes, payload, tail, pages
  uint64_t data_bytes() const { return uint64_t(nb) + 4 * pw + 4ull * t + pages_bytes; }
};

// error reporting
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
#define S4_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ::s4::hip_fail(e_, #call); \
  } while (0)

// format (s4_format.cpp)
int parse_stream(const uint8_t *enc, size_t bytes, StreamView *v);
size_t stream_bound(uint64_t n);
int encode_one(const uint32_t *in, uint64_t n, uint32_t delta, uint8_t *out, size_t cap, size_t *out_bytes);

// device (s4_device.hip)
int ensure_device();
int cu_count();
s4_tuning &tuning();

// Host-side layout of a device arena holding `count` lists.
struct ArenaLayout {
  size_t widths_off = 0, offs_off = 0, bmax_off = 0, seeds_off = 0, payload_off = 0, tail_off = 0,
         desc_off = 0, blkpre_off = 0, total = 0;
};

// Parsed streams to be placed in one device arena.
struct Upload {
  std::vector<StreamView> views;
  std::vector<uint64_t> blk_prefix, pay_base, tail_base;
  uint64_t total_blocks = 0, total_words = 0, total_tail = 0;
  ArenaLayout lay;
};

// Copy parsed streams into a new device arena (descriptor table at
// lay.desc_off) and build the skip index on `stream`.
int build_arena(Upload &u, hipStream_t stream, void **arena_out, std::vector<DList> *descs);
// hyb+m2 (Sec. 7.7): a list of n > 0 values over [0, universe) is a
// bitmap when universe / n <= gap (gap 0: never).
inline bool hyb_is_bitmap(uint64_t n, uint64_t universe, uint32_t gap) {
  return gap && n && n >= (universe + gap - 1) / gap;
}
// Build the bitmap lists of u (universe bits each, with select samples) in
// one new device allocation *mem; descs receives their descriptors.
// S4_EINVAL if a value reaches the universe.  Synchronises stream.
int build_bitmaps(Upload &u, uint64_t universe, hipStream_t stream, void **mem, std::vector<DList> *descs,
                  uint64_t *bitmap_bytes, uint64_t *select_bytes);
// Decode blocks [first, first + count) of L into d_out (index nb = tail).
// k_decode's arguments, in the kernel's order and layout (its kernel
// argument segment: 68 bytes, no hidden arguments).
struct DecodeArgs {
  const uint8_t *widths;
  const uint32_t *offs;
  const uint4 *seeds;
  const uint32_t *payload;
  uint32_t *out;
  uint32_t first, full_end, block_waves, form;
  const uint32_t *tail;
  uint32_t nb;
};
static_assert(offsetof(DecodeArgs, out) == 32 && offsetof(DecodeArgs, first) == 40 &&
                  offsetof(DecodeArgs, tail) == 56 && offsetof(DecodeArgs, nb) == 64,
              "k_decode argument layout");
constexpr uint32_t kDecodeArgBytes = 68;
// One k_decode launch: blocks per wave 4 P, kernel for patched lists or not,
// workgroups of 256 lanes, arguments.
struct DecodeLaunch {
  uint32_t P = 1;
  bool patched = false;
  uint32_t workgroups = 0;
  DecodeArgs a{};
};
// The launch that decodes blocks [first, first + count) of L into d_out (block
// nb the tail); false when there is nothing to decode.
bool plan_decode_range(const DList &L, uint32_t first, uint32_t count, uint32_t *d_out, DecodeLaunch *out);
// Host address of the k_decode instantiation a launch names (for lookups of
// the loaded kernel).
const void *decode_kernel_host_address(uint32_t P, bool patched);
int decode_range(const DList &L, uint32_t first, uint32_t count, uint32_t *d_out, hipStream_t stream);
// The same, the kernel launched so that ev0 / ev1 record its start and end.
int decode_range_timed(const DList &L, uint32_t first, uint32_t count, uint32_t *d_out, hipStream_t stream,
                       hipEvent_t ev0, hipEvent_t ev1);
// Exclusive scan of counts[n] (tiles of 1024), grand total to *total, then
// ordered gather of stage[128 i .. 128 i + counts[i]) into out.
int scan_and_compact(const uint32_t *stage, const uint32_t *counts, uint32_t n, uint32_t *excl, uint32_t *tiles,
                     uint32_t ntiles, uint64_t *total, uint32_t *out, hipStream_t stream);
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
// One conjunction as a single launch on st: lists ord[0 .. k) (2 <= k <= 33,
// shortest first, compressed, strictly increasing; none a bitmap), results
// to d_out[ord[0].n], count to *d_count.  scratch holds
// conjunction_scratch_bytes(ord[0].n) bytes; runs sharing it must not
// overlap.
size_t conjunction_scratch_bytes(uint64_t m);
int enqueue_conjunction(const DList *ord, uint32_t k, void *scratch, uint32_t *d_out, uint64_t *d_count,
                        hipStream_t st);

// Device tables of a batch of conjunctive queries (planned on the host).
struct BatchDev {
  const DList *lists;         // index descriptors
  const uint32_t *sterms;     // terms of every query, shortest list first
  const uint32_t *qoff;       // [nq + 1] term offsets
  const uint32_t *item_base;  // [nq + 1] first chunk of each query
  const uint4 *item_info;     // [items] {query, chunk in query, first term, terms}
  uint32_t *stage;            // [items * 128] survivors of each chunk
  uint32_t *counts;           // [items]
  uint32_t *excl;             // [items]
  uint32_t *tiles;            // [ntiles + 1]
  uint32_t *head;             // work-queue heads, queue p at head[p * kHeadStride]: one per part, else
                              // kSubQueues; head[1] is the staged tail's tile ticket
  uint64_t *total;            // number of results
  uint64_t *start;            // device clock at the start of the run
  uint64_t *qtick;            // [nq] completion time of each query
  uint64_t *stats;            // [2] algorithmic bytes read + written, blocks decoded
  // doc-ID partitioned index: chunks are queued per part (head[p], chunks
  // part_base[p] .. part_base[p + 1] in queue order) and chunk i's result
  // goes to slot item_rank[i] (query-major order); null / 1 otherwise
  const uint32_t *item_rank;
  const uint32_t *part_base;
  uint32_t parts;
  uint64_t *state;            // [items] single-pass scan words (see enqueue_serve_dev)
  uint32_t *err;              // set to 1 by the single-pass kernel on a failed look-back or overflow
  uint32_t items, nq, ntiles;
  uint32_t epoch;             // single-pass scan generation, 1 .. 2^30 - 1
  uint32_t feat;              // kinds of list in the index (kFeat* of the chunk pipeline)
  uint32_t count;             // nonzero: the counting instantiation runs, adding algorithmic bytes and blocks into stats
};
// Enqueue one run of a batch on st: persistent chunk kernel, scan,
// compaction into d_results, per-query counts / CSR offsets.
// begin = false: the caller's upload has reset the work queue and nothing
// reads the per-query completion stamps, so the reset kernel is skipped
int enqueue_batch_dev(const BatchDev &d, uint64_t *d_counts, uint64_t *d_offs, uint32_t *d_results, hipStream_t st,
                      bool begin = true);
// Enqueue one single-pass run on st: the persistent chunk kernel alone,
// each chunk taking its output offset from a decoupled look-back over the
// scan words d.state (tagged with d.epoch, so they need no clearing between
// runs) and writing its survivors to their final place in out[out_cap].
// d_offs[nq + 1] receives the CSR offsets.  *d.head must be 0.
int enqueue_serve_dev(const BatchDev &d, uint32_t *out, uint64_t out_cap, uint64_t *d_offs, hipStream_t st);
// The server's staged iteration in two launches: the chunk kernel, then
// one kernel that scans the chunks' counts (look-back across tiles),
// gathers their matches into out and writes the CSR offsets d_offs; needs
// d.state, d.err and an epoch as enqueue_serve_dev.
int enqueue_staged_serve_dev(const BatchDev &d, uint32_t *out, uint64_t *d_offs, hipStream_t st);
// The chunk records of d (records[items]) from one entry per query
// (qinfo[q] = {first chunk of the entry within its query, first term,
// terms, 0}) and d.item_base, written on st.
int enqueue_expand_items(const BatchDev &d, const uint4 *qinfo, uint4 *records, hipStream_t st);
constexpr uint32_t kMaxEpoch = (1u << 30) - 1;
// Most chunks a single-pass run takes under the current tuning: one per
// resident wave.  A chunk's count is known only when its chain is done, so
// with more chunks than waves every wave would wait on the slowest chunk in
// flight before taking the next; larger runs use the staged path.
uint64_t single_pass_max_items();

}  // namespace s4

struct s4_list {
  s4::DList d{};
  uint64_t n = 0, pw = 0;
  uint32_t nb = 0, t = 0, flags = 0;
  void *arena = nullptr;  // owned device memory (null for index views)
  uint64_t payload_bytes = 0, index_bytes = 0;
};

struct s4_index {
  void *arena = nullptr;    // compressed lists
  void *bitmaps = nullptr;  // bitmap lists and their select samples (hybrid index)
  void *desc = nullptr;     // device descriptor table
  uint64_t count = 0, total_ints = 0, payload_bytes = 0, index_bytes = 0;
  uint64_t universe = 0, bitmap_lists = 0, bitmap_bytes = 0, select_bytes = 0;
  uint32_t gap = 0;         // hyb+m2 parameter B (0: no bitmaps)
  uint32_t feat = 0;        // kinds of list held: bitmap 1, patched 2 (chunk-kernel instantiation)
  uint32_t parts = 1;       // doc-ID parts: descriptor t * parts + p is part p of list t
  std::vector<uint64_t> part_len;  // [count * parts] (parts > 1)
  std::vector<s4::DList> lists;    // host copy of the descriptors
  std::vector<uint64_t> lengths, pw, data_bytes;
  std::vector<uint32_t> flags;
  std::vector<uint8_t> kinds;      // 1: bitmap
  const s4::DList *d_lists = nullptr;  // device copy
};

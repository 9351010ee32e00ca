/*
 * s4.h -- C ABI of the MI355X (gfx950) S4-BP128-D4 decode + intersection
 * library (libs4.so).
 *
 * Method: D. Lemire, L. Boytsov, N. Kurz, "SIMD Compression and the
 * Intersection of Sorted Integers" (arXiv:1401.6399).  Sorted 32-bit
 * document-ID lists (Sec. 1) are stored as S4-BP128-D4: blocks of 128
 * integers, one bit width per block (Sec. 4.3), 4-way interleaved bit
 * packing (Sec. 4.2, Fig. 2), stride-4 differential coding (Sec. 5, Alg. 1);
 * conjunctive queries intersect the decoded lists two at a time, shortest
 * first (SvS, Sec. 6).
 *
 * Conventions for every call:
 *   - Return value: S4_OK (0) or a negative S4_E* code; s4_last_error()
 *     gives a thread-local message for the last failure.  No C++ exception
 *     crosses this boundary.
 *   - "host" pointers are ordinary CPU memory; "device" pointers (d_*) are
 *     HIP device memory on the current device.  The caller owns every raw
 *     buffer it passes; the library owns the opaque handles it returns and
 *     frees them only in the matching *_free / *_destroy call.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Device calls
 *     are stream-ordered and asynchronous: they enqueue work and return;
 *     counts are written to device memory, so no call synchronises unless
 *     it says so.  A fault inside a kernel surfaces at the caller's next
 *     synchronisation (hipStreamSynchronize), or as S4_EDEVICE from a later
 *     call that checks the stream.
 *   - Device output buffers must be 16-byte aligned.
 */
#ifndef S4_H
#define S4_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define S4_OK 0
#define S4_EINVAL (-1)    /* bad argument (null pointer, k = 0, misaligned buffer, ...) */
#define S4_EUNSORTED (-2) /* input not non-decreasing (encode) or not strictly increasing
                             (intersections) */
#define S4_ERANGE (-3)    /* output or scratch capacity too small */
#define S4_ECORRUPT (-4)  /* serialized stream malformed or truncated */
#define S4_ENOMEM (-5)    /* host or device allocation failed */
#define S4_EDEVICE (-6)   /* HIP runtime error or no usable gfx950 device */
#define S4_EAGAIN (-7)    /* server: no slot or memory free right now; retry later */

const char *s4_last_error(void);
int s4_version(void); /* stream format version written by s4_encode (1) */
/* Optional set-up of the current device: checks that it is a gfx950 part
 * and looks up the device address of the library's static scratch
 * (s4_intersect_k_noalloc); every call does this itself on first use. */
int s4_init(void);

/* ------------------------------------------------------------------ codec
 *
 * Serialized S4-BP128-D4 stream (little-endian, all offsets in bytes):
 *   0  u32 magic 0x34443453 ("S4D4")      4  u16 version = 1
 *   6  u16 flags (bit 0: strictly increasing; bits 1-2: differential form
 *                 S4_DELTA_*; bit 3: patched (S4-FastPFOR); other bits 0)
 *   8  u64 n      16 u32 nb = floor(n/128)  20 u32 t = n - 128 nb
 *   24 u64 pw = sum over blocks of 4 b_k (payload 32-bit words)
 *   32 u8 widths[nb], zero-padded to a multiple of 4 bytes
 *      u32 payload[pw]   block k holds 4 b_k words: word 4m + j is the
 *                        m-th word of lane j; lane j packs the D4 deltas
 *                        of integers 4q + j (q = 0..31), b_k bits each,
 *                        least significant bit first (Sec. 4.2, Fig. 2)
 *      u32 tail[t]       the last t < 128 integers, raw (the paper uses
 *                        varint here, Sec. 4.3)
 * Width b_k is the smallest b with every delta of block k below 2^b
 * (Sec. 4.3).  Differential forms (Sec. 5; values before the list are 0):
 *   S4_DELTA_D4  delta_i = x_i - x_{i-4}          (the default)
 *   S4_DELTA_DM  delta_{4i+j} = x_{4i+j} - x_{4i-1}
 *   S4_DELTA_D2  delta_i = x_i - x_{i-2}
 *   S4_DELTA_D1  delta_i = x_i - x_{i-1}
 *
 * Patched streams (S4-FastPFOR, Sec. 4.4; flag bit 3): block k is packed
 * at a width b'_k <= b_k (widths[] and pw count b'), keeping each delta's
 * low b' bits; deltas >= 2^b' are exceptions.  b' minimises 128 b' +
 * c(b') (b - b' + 8), c(b') the number of exceptions; ties go to the
 * larger b'.  After the tail come the pages of up to 512 blocks, each:
 *      u32 meta_len; per block u8 b, u8 c, then c u8 positions (increasing,
 *      < 128); zero-padded to a multiple of 4 bytes;
 *      u32 present: bit d-1 set when some block of the page has c > 0 and
 *      b - b' = d; then for each such d ascending: u32 count, and the
 *      count high parts (delta >> b', d bits each, in block then position
 *      order) packed LSB-first, value e at bit e d, padded to a multiple of
 *      32 values (d words per 32).
 */
#define S4_DELTA_D4 0u
#define S4_DELTA_DM 1u
#define S4_DELTA_D2 2u
#define S4_DELTA_D1 3u
/* OR into the `delta` argument of s4_encode_ex / s4_encode_many to write a
 * patched (S4-FastPFOR) stream in that form. */
#define S4_CODEC_FASTPFOR 0x100u

/* Worst-case stream size for n integers (every block at b = 32; covers
 * patched streams too). */
size_t s4_encoded_bound(uint64_t n);

/* Encode host list in[n] (non-decreasing, duplicates allowed) into host
 * buffer out[cap].  *out_bytes receives the stream size (also on
 * S4_ERANGE, so the call can size the buffer).  S4_EUNSORTED if in[] ever
 * decreases. Sec. 4.2-4.3, Sec. 5. */
int s4_encode(const uint32_t *in, uint64_t n, uint8_t *out, size_t cap, size_t *out_bytes);

/* s4_encode with an explicit differential form (S4_DELTA_*), optionally
 * ORed with S4_CODEC_FASTPFOR for a patched stream. */
int s4_encode_ex(const uint32_t *in, uint64_t n, uint32_t delta, uint8_t *out, size_t cap, size_t *out_bytes);

/* Encode `count` host lists in parallel with differential form `delta`:
 * list i is in[in_offsets[i] .. in_offsets[i+1]) and its stream is written
 * to out + out_offsets[i], which the caller sizes with s4_encoded_bound;
 * out_bytes[i] receives each size.  nthreads <= 0 picks the number of
 * hardware threads. */
int s4_encode_many(const uint32_t *in, const uint64_t *in_offsets, uint64_t count, uint32_t delta, uint8_t *out,
                   const uint64_t *out_offsets, uint64_t *out_bytes, int nthreads);

/* Number of integers in a stream; validates the whole header and width
 * table (S4_ECORRUPT on any inconsistency). */
int s4_decoded_length(const uint8_t *enc, size_t bytes, uint64_t *n);

/* Host decode of a whole stream (any form, plain or patched) into host
 * out[cap]; *n_out receives n (also when cap < n: S4_ERANGE, nothing
 * written).  The stream is validated first as by s4_decoded_length
 * (patched pages included).  For tools and checks on the host: the
 * decoding path of this library is the device one (s4_decode_dev and the
 * calls after it); this is a plain scalar loop (Alg. 1's extraction per
 * value, the exceptions of Sec. 4.4, the form's inverse of Sec. 5). */
int s4_decode(const uint8_t *enc, size_t bytes, uint32_t *out, uint64_t cap, uint64_t *n_out);

/* ----------------------------------------------------------- device lists
 *
 * Every device call below handles all four differential forms; lists of
 * different forms can be mixed in one index, intersection or batch.
 *
 * s4_list: one list resident in device memory, structure of arrays:
 * widths u8[nb], block word offsets u32[nb], payload u32[pw] (+32 bytes of
 * padding), raw tail u32[t], and a skip index built on the device at upload:
 * bmax[k] = x[128k + 127] (the block's largest value) and seed[k] =
 * x[128k-4 .. 128k-1] (zeros for k = 0), the prefix seed that lets any
 * block be decoded alone (Alg. 1 seeds each block with the previous
 * block's last four values; D2 needs the last two, D1 and DM the last
 * one).  The skip index is not part of the paper.
 */
typedef struct s4_list s4_list;

/* Upload host stream enc[bytes]; builds the skip index with two kernels on
 * `stream`.  Validates the stream (S4_ECORRUPT).  The host buffer may be
 * reused once the call returns. */
int s4_list_upload(const uint8_t *enc, size_t bytes, void *stream, s4_list **out);
int s4_list_free(s4_list *list);

/* Length facts of an uploaded list (host values, no device access).
 * payload_bytes counts widths + payload + tail (+ the pages of a patched
 * stream: the paper's size); index_bytes counts block offsets + skip index
 * (+ 16 bytes per block of exception records for a patched list). */
int s4_list_info(const s4_list *list, uint64_t *n, uint32_t *nb, uint32_t *flags,
                 uint64_t *payload_bytes, uint64_t *index_bytes);

/* Copy the skip index to host arrays bmax[nb] and seeds[4 nb]
 * (synchronises `stream`).  For tests and tools. */
int s4_list_skip_index(const s4_list *list, uint32_t *bmax, uint32_t *seeds, void *stream);

/* Decode the whole list into device buffer d_out[cap] (cap >= n) on
 * `stream`: unpack and the stream's prefix sum (its differential form,
 * Sec. 5; a patched stream's exceptions added in between, Sec. 4.4) fused
 * in one kernel (Alg. 1), tail copied.  S4_ERANGE if cap < n. */
int s4_decode_dev(const s4_list *list, uint32_t *d_out, uint64_t cap, void *stream);

/* s4_decode_dev with timing: the kernel is launched so that the caller's
 * HIP events start_event / stop_event (hipEvent_t, created with timing) are
 * recorded by the launch itself at the kernel's start and end, so their
 * elapsed time is the kernel's execution without the dispatch of the
 * launch.  For an empty list both events are recorded back to back. */
int s4_decode_timed_dev(const s4_list *list, uint32_t *d_out, uint64_t cap, void *start_event, void *stop_event,
                        void *stream);

/* Decode blocks [first, first + count) into d_out (128 values per block);
 * block index nb denotes the tail (t values).  Each block is seeded from
 * the skip index, so any range decodes alone. */
int s4_decode_blocks_dev(const s4_list *list, uint32_t first, uint32_t count, uint32_t *d_out,
                         void *stream);

/* Decode `count` lists with one kernel launch per list (the same kernel as
 * s4_decode_dev): list i into d_outs[i] (capacity caps[i], 16-byte
 * aligned).  nstreams = 1 issues every launch on `stream`; nstreams = 8
 * spreads them over 8 streams forked from `stream` and joined back into
 * it before the call's work is complete in `stream` order, so independent
 * lists overlap on the device; the call is capturable into a hipGraph on
 * `stream`.  Other stream counts return S4_EINVAL: they are switched off
 * until a host-side crash seen while timing them is explained. */
int s4_decode_lists_dev(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps,
                        uint32_t count, uint32_t nstreams, void *stream);

/* The per-list decode of s4_decode_lists_dev (the same kernel, one launch
 * per list, Alg. 1 fused with the prefix) dispatched by the library itself:
 * each launch is a dispatch packet written into one of four HSA queues the
 * library owns (lists spread over them by size), with no barrier or fence
 * between the lists of a step (they are independent); barrier packets end
 * each step on every queue and make the next step wait for all of them, so
 * steps never overlap, and a launch costs the host one packet instead of a
 * runtime launch call.  Every run opens with a barrier packet whose
 * system-scope acquire invalidates the device caches, so lists and
 * outputs written through HIP before the run are seen.  A plan holds the
 * packets (host) and their argument blocks (device memory), built once;
 * the lists and outputs (16-byte aligned, capacity caps[i] >= n)
 * must outlive it.  Plain lists only: a patched list is S4_EINVAL.  The
 * dispatcher serves the device it is first used on.
 *
 * s4_aql_plan_run is host-synchronous and not ordered with HIP streams: it
 * needs the lists and outputs idle (no HIP work on them in flight) and
 * returns once `steps` (1..64) decodes of every list are complete, with the
 * host wall time from its first packet to completion in *elapsed_ns (may
 * be null).  It is the form the throughput of the per-list decode is timed
 * with: the host thread writes the packets of every step ahead of the
 * device and nothing else stands between them.
 * s4_aql_plan_enqueue is the stream-ordered form: it returns at once; the
 * run starts after the work already enqueued on `stream` and the stream's
 * later work waits for its completion (a host function of the stream
 * submits the packets and waits for the last step; the caller's thread
 * never blocks).  A failure of such a run is reported by the next
 * s4_aql_plan_status (S4_OK while none has failed); the plan must not be
 * freed while a run is enqueued (S4_EINVAL).
 * s4_aql_plan_profile runs `steps` steps like s4_aql_plan_run with
 * dispatch profiling enabled on the queues and a completion signal on every
 * dispatch, and writes each dispatch's start and end on the device
 * (nanoseconds after the earliest start of the run) to start_ns / end_ns
 * [s * count + i] for list i of step s (0 for a list with nothing to
 * decode); for measurement, not for timed runs.
 * Every run returns S4_EDEVICE if a queue reports an error or the work does
 * not complete within 20 s; the dispatcher then refuses every later run
 * (packets may still be queued) and keeps the argument blocks of every
 * plan for the rest of the process. */
typedef struct s4_aql_plan s4_aql_plan;
int s4_aql_plan_create(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps,
                       uint32_t count, s4_aql_plan **out);
/* The same plan with the placement chosen by the caller: list i goes to
 * queue queue_of[i] (< 4), and within a queue dispatches go in increasing
 * rank[i] (ties keep list order; rank may be null).  S4_EINVAL for a queue
 * index out of range. */
int s4_aql_plan_create_placed(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps,
                              uint32_t count, const uint32_t *queue_of, const uint32_t *rank, s4_aql_plan **out);
int s4_aql_plan_run(s4_aql_plan *plan, uint32_t steps, uint64_t *elapsed_ns);
int s4_aql_plan_enqueue(s4_aql_plan *plan, uint32_t steps, void *stream);
int s4_aql_plan_status(s4_aql_plan *plan);
int s4_aql_plan_profile(s4_aql_plan *plan, uint32_t steps, uint64_t *start_ns, uint64_t *end_ns,
                        uint64_t *elapsed_ns);
/* Where each list's dispatch goes: queue_of[i] (0..3) and its position
 * in that queue's order within a step (host arrays [count]; UINT32_MAX for
 * a list with nothing to decode). */
int s4_aql_plan_layout(const s4_aql_plan *plan, uint32_t *queue_of, uint32_t *position);
int s4_aql_plan_free(s4_aql_plan *plan);

/* A reusable multi-list decode: one kernel launch decodes every list of
 * the plan (workgroups are laid out over the concatenated blocks of all
 * lists).  The plan holds a device table of the lists and output
 * pointers, built once; the lists must outlive it. */
typedef struct s4_decode_plan s4_decode_plan;
int s4_decode_plan_create(const s4_list *const *lists, uint32_t *const *d_outs, const uint64_t *caps,
                          uint32_t count, void *stream, s4_decode_plan **out);
int s4_decode_plan_run(const s4_decode_plan *plan, void *stream);
int s4_decode_plan_free(s4_decode_plan *plan);

/* Benchmarking aid: enqueue a kernel that busy-waits on the device's
 * constant-rate clock for about `ns` nanoseconds (always terminates), so a
 * host can enqueue timed work behind it without its own launch latency
 * showing in event timings. */
int s4_spin_dev(uint64_t ns, void *stream);

/* --------------------------------------------------------- intersections
 *
 * Inputs must have been encoded from strictly increasing lists (flag bit 0),
 * else S4_EUNSORTED.  Results are strictly increasing and never longer than
 * the shorter input (the output-to-input property, Sec. 6.2), so
 * cap >= min(len a, len b) is always enough; a smaller cap is S4_ERANGE.
 * The count is written to device memory *d_count (u64).  Scratch is a
 * caller-owned device buffer of at least the size the *_scratch_bytes call
 * reports (16 bytes per 128 values of the shorter side, plus 256); its
 * contents on entry do not matter, and calls that share it must not overlap
 * (stream order is enough).
 * Each call is one kernel launch (an empty shorter side: one launch that
 * writes the zero count): every wavefront takes a 128-value chunk of the
 * shorter side in the order the wavefronts start, intersects it, and finds
 * where its survivors go by a look-back over its predecessors' counts in
 * the scratch (each call's counts carry an epoch of their own, so stale
 * ones are never read).  That wait is bounded: a call that cannot finish
 * (never seen) writes *d_count = UINT64_MAX instead of hanging.
 */
size_t s4_intersect_scratch_bytes(uint64_t len_a, uint64_t len_b);
int s4_intersect(const s4_list *a, const s4_list *b, uint32_t *d_out, uint64_t cap,
                 uint64_t *d_count, void *d_scratch, size_t scratch_bytes, void *stream);

/* k-way conjunction (SvS, Sec. 6): lists are ordered by length, the two
 * shortest are intersected (both compressed), then the uncompressed
 * intermediate is intersected with each next list in turn, decoding only
 * the blocks it needs.  The work is split by 128-value chunks of the
 * shortest list, each chunk carried through all the lists by one wavefront
 * (one launch in all), which gives the same set.  k = 0 or k > 33 is
 * S4_EINVAL; k = 1 decodes the list (d_out 16-byte aligned; no scratch
 * needed). */
size_t s4_intersect_k_scratch_bytes(const s4_list *const *lists, uint32_t k);
int s4_intersect_k(const s4_list *const *lists, uint32_t k, uint32_t *d_out, uint64_t cap,
                   uint64_t *d_count, void *d_scratch, size_t scratch_bytes, void *stream);

/* Intersect an uncompressed strictly increasing device list d_r[*d_len_r]
 * (its length read on the device) with compressed list f; the building
 * block of the chain above.  cap_r is the host-known upper bound of
 * *d_len_r (sizes the launch and the scratch). */
size_t s4_intersect_raw_scratch_bytes(uint64_t cap_r);
int s4_intersect_raw(const uint32_t *d_r, const uint64_t *d_len_r, uint64_t cap_r,
                     const s4_list *f, uint32_t *d_out, uint64_t cap, uint64_t *d_count,
                     void *d_scratch, size_t scratch_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * k-way conjunction of s4_intersect_k, with its scratch taken from a static
 * device array of S4_NOALLOC_SCRATCH_BYTES per device that the library
 * holds until the process ends.  The call allocates nothing; the caller
 * passes lists, outputs and stream as for s4_intersect_k.  The shortest
 * list may hold at most s4_intersect_k_noalloc_max_len() values
 * (33,550,336 = 262,112 chunks of 128 in 4 MiB), else S4_ERANGE.  Every call on a device shares
 * that device's array: calls that overlap on one GPU (other streams, or
 * other threads without ordering) race and give wrong results; calls
 * ordered on one stream are safe, and the array needs no clearing between
 * them.  The array's device address is looked up once per device, by
 * s4_init or by the first call there. */
#define S4_NOALLOC_SCRATCH_BYTES (4u << 20)
uint64_t s4_intersect_k_noalloc_max_len(void);
int s4_intersect_k_noalloc(const s4_list *const *lists, uint32_t k, uint32_t *d_out, uint64_t cap,
                           uint64_t *d_count, void *stream);

/* ---------------------------------------------------------------- tuning
 *
 * gallop_blocks: when a 128-value chunk of the short list spans more than
 * this many blocks of the long list, candidate blocks are found by per-lane
 * binary search over the long list's bmax in global memory (galloping
 * regime, Sec. 6.1); otherwise the spanned bmax entries are staged in LDS
 * first (merge regime).  Only candidate blocks are ever decoded.
 * waves_per_group: waves per workgroup of the intersection kernels (1..8).
 * groups_per_cu: resident workgroups per compute unit for persistent
 * (batch) launches.  items_per_grab: work items a wave takes per atomic
 * fetch in persistent launches.  Results never depend on these values. */
typedef struct {
  uint32_t gallop_blocks;
  uint32_t waves_per_group;
  uint32_t groups_per_cu;
  uint32_t items_per_grab;
  uint32_t decode_passes; /* bulk decode: 4 * decode_passes blocks per wave (1, 2, 4, 8) */
} s4_tuning;

int s4_get_tuning(s4_tuning *t);
int s4_set_tuning(const s4_tuning *t);

/* ------------------------------------------------------------------ index
 *
 * Many lists in one device arena (CSR of lists), for batched queries.
 * encs is a host buffer holding `count` streams back to back, stream i at
 * byte offset enc_offsets[i] with size enc_offsets[i+1] - enc_offsets[i].
 * Synchronises `stream` before returning.
 */
typedef struct s4_index s4_index;
int s4_index_build(const uint8_t *encs, const uint64_t *enc_offsets, uint64_t count, void *stream,
                   s4_index **out);
int s4_index_free(s4_index *index);
/* lengths[count] of the indexed lists (host copy). */
int s4_index_lengths(const s4_index *index, uint64_t *lengths);
int s4_index_info(const s4_index *index, uint64_t *count, uint64_t *total_ints,
                  uint64_t *payload_bytes, uint64_t *index_bytes);
/* A view of list i of the index usable with every s4_list call; valid
 * until the index is freed; release it with s4_list_free.  S4_EINVAL for a
 * list a hybrid index holds as a bitmap. */
int s4_index_list(const s4_index *index, uint64_t i, s4_list **out);

/* Hybrid index (hyb+m2, Sec. 7.7, after Culpepper and Moffat): as
 * s4_index_build, but every strictly increasing list whose average gap
 * universe / n is at most bitmap_gap (B; the paper uses 8, 16 and 32) is
 * held as a bitmap of `universe` bits (bit x in bit x % 32 of 32-bit word
 * x / 32) instead of compressed blocks, with one 4-byte select sample per
 * 128 values; the other lists stay compressed.  Such lists are at least as
 * long as any compressed one, so a query's SvS order (shortest first)
 * intersects the compressed lists first and then checks each survivor's
 * bit in every bitmap list; a query whose lists are all bitmaps walks its
 * shortest bitmap 128 values at a time.  universe in [1, 2^32]; S4_EINVAL
 * if bitmap_gap is 0 or a bitmap list has a value >= universe.  The
 * bitmaps are built on the device from the compressed streams.
 * s4_index_info's payload_bytes counts the bitmaps, index_bytes the select
 * samples.  Synchronises `stream`. */
int s4_index_build_hybrid(const uint8_t *encs, const uint64_t *enc_offsets, uint64_t count,
                          uint64_t universe, uint32_t bitmap_gap, void *stream, s4_index **out);
/* Doc-ID partitioned index (Sec. 7.7: the paper splits its corpora into
 * 32 or 64 independent parts by document ID and answers a query part by
 * part, joining the results).  Stream t * parts + p (enc_offsets has
 * count * parts + 1 entries) is part p of list t; every list's parts must
 * hold ascending value ranges (each non-empty part starting above the end
 * of the previous one: S4_EINVAL otherwise, checked on the device).  A
 * batch over such an index runs each query once per part, in that part's
 * length order, and writes the parts' results one after the other; its
 * chunks are queued per part, and workgroups drain first the parts of
 * their own XCD (part x mod parts for fewer than 8 parts, x, x + 8, ...
 * otherwise; workgroups go to the 8 XCDs round-robin by id) so that each
 * XCD's L2 holds one part's lists.  s4_index_lengths gives each list's
 * total length; s4_index_list and the server refuse a partitioned index.
 * parts in [1, 1024]; parts = 1 is s4_index_build.  Synchronises `stream`. */
int s4_index_build_parts(const uint8_t *encs, const uint64_t *enc_offsets, uint64_t count,
                         uint32_t parts, void *stream, s4_index **out);
/* Host helper for s4_index_build_parts: for count sorted host lists
 * in[in_offsets[t] .. in_offsets[t+1]) with every value below `universe`,
 * sub_offsets[t * parts + p] (count * parts + 1 entries) receives where
 * part p of list t starts in `in`: part p holds the values in
 * [floor(p U / parts), floor((p + 1) U / parts)).  The parts of all lists
 * are consecutive in `in`, so s4_encode_many(in, sub_offsets, count *
 * parts, ...) encodes them.  S4_EINVAL for a value >= universe or parts
 * outside [1, universe]. */
int s4_partition_offsets(const uint32_t *in, const uint64_t *in_offsets, uint64_t count,
                         uint32_t parts, uint64_t universe, uint64_t *sub_offsets);
/* kinds[count]: 0 for a compressed list, 1 for a bitmap. */
int s4_index_kinds(const s4_index *index, uint8_t *kinds);
/* Hybrid parameters and sizes (all 0 for an index built without bitmaps);
 * any pointer may be null. */
int s4_index_hybrid_info(const s4_index *index, uint64_t *universe, uint32_t *bitmap_gap,
                         uint64_t *bitmap_lists, uint64_t *bitmap_bytes, uint64_t *select_bytes);

/* ------------------------------------------------------------------ batch
 *
 * A batch plan: nq conjunctive queries over an index, query q being terms
 * h_terms[h_q_offsets[q] .. h_q_offsets[q+1]) (k >= 1 distinct list ids).
 * The plan orders each query's terms by length (SvS), reserves intermediate
 * memory from the output-to-input bound, and uploads its tables once.
 * s4_batch_run executes every query: one persistent decode-fused launch in
 * which each 128-value chunk of a query's shortest list is carried through
 * the query's other lists in SvS order (no intermediate list is written),
 * then scan and compaction kernels that place each query's results in
 * order; with use_graph != 0 the whole sequence is captured once into a
 * hipGraph and replayed on later runs.  Runs of one batch share its work
 * counters, so they must not overlap: issue them on one stream (or order
 * them); s4_batch_set_counting and s4_batch_free likewise only while no
 * run of the batch is in flight.
 * Outputs (device): d_counts[nq] (u64), d_res_offsets[nq + 1] (u64, CSR),
 * d_results[results_cap] (u32, query q's docIDs at
 * d_results[d_res_offsets[q] ..]).  results_cap >= s4_batch_results_bound.
 */
typedef struct s4_batch s4_batch;
int s4_batch_plan(const s4_index *index, const uint32_t *h_terms, const uint64_t *h_q_offsets,
                  uint64_t nq, void *stream, s4_batch **out);
int s4_batch_free(s4_batch *batch);
uint64_t s4_batch_results_bound(const s4_batch *batch);
int s4_batch_run(s4_batch *batch, uint64_t *d_counts, uint64_t *d_res_offsets, uint32_t *d_results,
                 uint64_t results_cap, int use_graph, void *stream);
/* Per-query completion stamps of the last run, in device clock ticks
 * (100 MHz constant clock) relative to the run's start: host array
 * ticks[nq].  Synchronises `stream`. */
int s4_batch_query_ticks(const s4_batch *batch, uint64_t *ticks, void *stream);

/* Count algorithmic traffic in later runs of this batch (on != 0) or not
 * (the default: counting slows the chunk kernels by 4-15%, so timed runs
 * leave it off).  A captured graph of the batch is dropped and
 * re-captured on its next run. */
int s4_batch_set_counting(s4_batch *batch, int on);

/* Algorithmic traffic of the last run, if it counted (else zeros): bytes =
 * packed payload, width byte, block offset and seed of every block decoded,
 * skip-index entries staged, raw values read, plus 4 bytes per result;
 * blocks = blocks decoded.  Synchronises `stream`. */
int s4_batch_traffic(const s4_batch *batch, uint64_t *bytes, uint64_t *blocks, void *stream);

/* Autotune gallop_blocks / waves_per_group / groups_per_cu / items_per_grab
 * on this plan: times `reps` runs per candidate setting, keeps the fastest
 * and installs it with s4_set_tuning.  best_ms receives its time.  The
 * plan's results are identical under every candidate. */
int s4_batch_autotune(s4_batch *batch, uint64_t *d_counts, uint64_t *d_res_offsets,
                      uint32_t *d_results, uint64_t results_cap, int reps, void *stream,
                      s4_tuning *best, double *best_ms);

/* ------------------------------------------------------------- plain path
 *
 * The plain path a batch is compared with: every query on its own, one
 * single-launch conjunction per query (the kernel of s4_intersect_k, Sec. 6
 * SvS over chunks of the shortest list), launched back to back on `stream`
 * from this call's thread, with no batching.  Queries are as for
 * s4_batch_plan but need 2..33 terms; the index must be neither hybrid nor
 * partitioned (S4_EINVAL).  The call checks every query, then launches,
 * then synchronises `stream`.
 *
 * s4_plain_run: query q's results go to d_results + res_offsets[q]
 * (res_offsets: host [nq + 1], written by the call: the prefix sum of each
 * query's shortest length, the output-to-input bound), its count to
 * d_counts[q] (device u64).  results_cap >= res_offsets[nq] and
 * scratch_bytes >= s4_intersect_raw_scratch_bytes(longest shortest list),
 * else S4_ERANGE before any launch.  lat_ns (host [nq], may be null): each
 * query is then waited for before the next is launched, and lat_ns[q] is
 * its host wall time from launch to completion (an isolated query's
 * latency).  *elapsed_ns: host wall time from the first launch to the
 * completion of the last query. */
int s4_plain_run(const s4_index *index, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                 uint32_t *d_results, uint64_t results_cap, uint64_t *res_offsets, uint64_t *d_counts,
                 void *d_scratch, size_t scratch_bytes, uint64_t *lat_ns, uint64_t *elapsed_ns, void *stream);
/* s4_plain_replay: the same plain path under an open-loop arrival trace
 * (as s4_server_replay): query q is launched h_arrival_ns[q] ns after the
 * call starts, or as soon after as the launching thread gets to it;
 * latency_ns[q] is the time from its scheduled arrival until a watcher
 * thread sees its completion event.  Every query writes its results to
 * d_results (results_cap >= the longest shortest list; each query
 * overwrites the last, in stream order) and its count to d_counts[q].
 * *elapsed_s: wall time from the first arrival to the last completion.
 * S4_ERANGE after timeout_s seconds. */
int s4_plain_replay(const s4_index *index, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                    const uint64_t *h_arrival_ns, uint64_t *latency_ns, uint32_t *d_results, uint64_t results_cap,
                    uint64_t *d_counts, void *d_scratch, size_t scratch_bytes, double timeout_s, double *elapsed_s,
                    void *stream);

/* ----------------------------------------------------------------- server
 *
 * Continuous-batching query server over a device-resident index (each
 * query a conjunction whose lists are intersected as in Sec. 6, shortest
 * list first).  A dispatcher thread owns four iteration contexts, each
 * with its own HIP stream and buffers allocated at creation.  An iteration
 * admits waiting queries, oldest first, while the context's slots, the
 * reserved intermediate memory (the output-to-input bound: 512 bytes per
 * 128-value chunk of the query's shortest list) and the result buffer (the
 * shortest list's length per query) fit, runs every admitted query to
 * completion in one persistent decode-fused launch (a single-pass kernel
 * with look-back offsets when the iteration has at most one 128-value
 * chunk per resident wave, else the chunk kernel and one tail kernel that
 * scans, compacts and writes the per-query offsets), and
 * retires them.  Queries longer than slice_chunks chunks run a slice per
 * iteration (see s4_server_config), in at most three of the four
 * contexts at a time, so one context always stays free for short queries.
 * Queries that arrive while iterations run join the next free context, so
 * up to four iterations overlap on the device.  Submission never blocks
 * on the GPU.
 */
typedef struct s4_server s4_server;
typedef struct {
  uint32_t max_slots;       /* concurrent queries on the device */
  uint64_t pool_bytes;      /* device memory for admitted queries' chunk results (split over
                               the in-flight iterations; each query needs 512 bytes per
                               128-value chunk of its shortest list) */
  uint64_t result_bytes;    /* pinned host memory for results in flight (0: 64 MiB) */
  uint32_t max_terms;       /* longest query accepted */
  uint32_t slice_chunks;    /* most 128-value chunks of one query's shortest list per iteration
                               (0: 16384); a longer query runs one slice per iteration, its
                               slices' results joined in order, so it never holds the device
                               long while short queries wait; an iteration takes at most four
                               slices' worth of chunks */
} s4_server_config;

int s4_server_create(const s4_index *index, const s4_server_config *cfg, s4_server **out);
/* Submit a query (host terms[k]); *id receives its ticket.  S4_EINVAL for
 * bad terms, S4_ERANGE if one slice of it can never fit the pool, S4_EAGAIN
 * if the waiting queue is full. */
int s4_server_submit(s4_server *srv, const uint32_t *terms, uint32_t k, uint64_t *id);
/* Retrieve up to max_done finished queries: ids[], counts[], latency_ns[]
 * (submit -> result on host).  Results are copied to host memory:
 * results + res_offsets[i] (res_offsets has max_done + 1 entries; the
 * results buffer holds results_cap integers; a query whose result does not
 * fit stays queued).  *done receives the number returned.  Non-blocking. */
int s4_server_poll(s4_server *srv, uint64_t *ids, uint64_t *counts, uint64_t *latency_ns,
                   uint32_t *results, uint64_t results_cap, uint64_t *res_offsets,
                   uint32_t max_done, uint32_t *done);
typedef struct {
  uint64_t submitted, admitted, completed, rejected;
  uint64_t iterations;
  uint64_t peak_active;
  uint64_t peak_pool_bytes;
  uint64_t waits_for_memory; /* admissions deferred because the pool was full */
  uint64_t max_batch;        /* most queries admitted into one iteration */
  uint64_t direct_iterations;/* iterations whose results the device wrote straight to pinned host memory */
  uint64_t single_pass_iterations; /* iterations run as one single-pass kernel (at most one chunk per resident wave) */
  uint64_t sliced_queries;   /* queries run in more than one slice */
  uint64_t device_ns;        /* summed launch-to-finish time of iterations, as seen by the dispatcher */
  uint64_t host_ns;          /* dispatcher time spent packing, launching and retiring iterations */
  uint64_t retire_ns;        /* ... of which retiring finished iterations (results handed over) */
  uint64_t admit_ns;         /* ... admitting queries into a free context (under the server lock;
                                also counted when nothing was admitted) */
  uint64_t launch_ns;        /* ... packing an iteration's tables and launching it (host_ns also
                                counts the lock taken after a launch) */
} s4_server_stats;
int s4_server_stats_get(const s4_server *srv, s4_server_stats *st);
/* Stop accepting, finish every admitted query, join the dispatcher. */
int s4_server_destroy(s4_server *srv);

/* Benchmarking aid: replay an open-loop arrival trace.  Query q (host terms
 * h_terms[h_q_offsets[q] .. h_q_offsets[q+1])) is submitted h_arrival_ns[q]
 * nanoseconds after the call starts (non-decreasing; the host spins on its
 * steady clock), whatever the state of earlier queries; completions are
 * drained concurrently.  latency_ns[q] receives the time from the scheduled
 * arrival to the result on the host, counts[q] the result size; when
 * results is not null, result q is copied to results + res_offsets[q]
 * (res_offsets has nq + 1 entries) if everything fits results_cap; keep
 * (host [nq], may be null) limits the copies to the queries with
 * keep[q] != 0 (the others get empty ranges), so a long trace need not hold
 * every result.  Returns
 * S4_ERANGE after timeout_s seconds without every result; *elapsed_s
 * receives the wall time from the first arrival to the last result.  The
 * replay takes every completion the server hands over while it runs:
 * queries submitted by other threads meanwhile finish unseen by
 * s4_server_poll. */
int s4_server_replay(s4_server *srv, const uint32_t *h_terms, const uint64_t *h_q_offsets, uint64_t nq,
                     const uint64_t *h_arrival_ns, uint64_t *latency_ns, uint64_t *counts, uint32_t *results,
                     uint64_t results_cap, uint64_t *res_offsets, const uint8_t *keep, double timeout_s,
                     double *elapsed_s);

#ifdef __cplusplus
}
#endif
#endif /* S4_H */

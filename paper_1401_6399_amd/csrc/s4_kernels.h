// Device building blocks for gfx950 (64-lane wavefronts).
//
// Notation follows the paper: a block holds 128 integers; integer 4q + j of
// a block is the q-th value of lane j (Sec. 4.2, Fig. 2); b is the block's
// bit width (Sec. 4.3); D4 deltas are x_i - x_{i-4} (Sec. 5).  r is the
// shorter list of a pair and f the longer one (Sec. 6).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "s4_internal.h"

namespace s4 {

constexpr uint32_t kInvalid = 0xFFFFFFFFu;

// ----------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// LDS written by some lanes of a wave and read by others: DS instructions of
// one wave execute in order, so only the compiler must be kept from moving
// accesses across this point.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// DPP move with zero fill: lanes whose source is outside the row (or in a
// row disabled by ROW_MASK) receive 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ uint32_t dpp0(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROW_MASK, 0xf, true));
}

// Inclusive scans.  DPP row_shr:n = 0x110 + n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.
__device__ __forceinline__ uint32_t scan_row16(uint32_t v) {
  v += dpp0<0x111>(v);
  v += dpp0<0x112>(v);
  v += dpp0<0x114>(v);
  v += dpp0<0x118>(v);
  return v;
}
__device__ __forceinline__ uint32_t scan_half32(uint32_t v) {
  v = scan_row16(v);
  v += dpp0<0x142, 0xa>(v);  // row 1 += lane 15, row 3 += lane 47
  return v;
}
__device__ __forceinline__ uint32_t scan_wave64(uint32_t v) {
  v = scan_half32(v);
  v += dpp0<0x143, 0xc>(v);  // rows 2, 3 += lane 31
  return v;
}

// Sum over the wave.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v += uint32_t(__shfl_xor(int(v), o));
  return v;
}

// Global-memory views of device pointers.  Lists, tables and outputs live
// in global memory, but pointers read from descriptor tables reach the
// compiler as generic ones, whose loads and stores become flat accesses that
// count against the LDS wait counter too, so every wait for memory would
// also hold LDS work back and the other way round.  Accesses through these
// views are global ones.
// (The qualifiers apply in the device compilation; the host pass, which
// emits no device code, sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define S4_ADDRSPACE(n) __attribute__((address_space(n)))
#else
#define S4_ADDRSPACE(n)
#endif
template <class T>
using gconst = const S4_ADDRSPACE(1) T *;
template <class T>
using gmut = S4_ADDRSPACE(1) T *;
template <class T>
__device__ __forceinline__ gconst<T> gbl(const T *p) {
  return (gconst<T>)p;
}
template <class T>
__device__ __forceinline__ gmut<T> gbl_out(T *p) {
  return (gmut<T>)p;
}
// Read-only view of a table that no kernel writes while it runs (list
// descriptors): uniform loads through it go through the scalar cache into
// scalar registers.
template <class T>
__device__ __forceinline__ const S4_ADDRSPACE(4) T *cst(const T *p) {
  return (const S4_ADDRSPACE(4) T *)p;
}

// Streaming 16-byte store that does not keep the line in cache.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store_nt4(uint32_t *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  u32x4 v = {a, b, c, d};
#ifdef S4_PLAIN_STORES
  *reinterpret_cast<u32x4 *>(p) = v;
#else
  __builtin_nontemporal_store(v, gbl_out(reinterpret_cast<u32x4 *>(p)));
#endif
}

// 16-byte store of decoded output (plain; whole lines per instruction).
__device__ __forceinline__ void store4(uint32_t *p, u32x4 v) {
#ifndef S4_PLAIN_STORES
  __builtin_nontemporal_store(v, gbl_out(reinterpret_cast<u32x4 *>(p)));
#else
  *reinterpret_cast<u32x4 *>(p) = v;
#endif
}

// ------------------------------------------------------------ extraction

__device__ __forceinline__ uint32_t width_mask(uint32_t b) { return b >= 32u ? 0xFFFFFFFFu : ((1u << b) - 1u); }

// Low 32 bits of (hi:lo) >> s, s in [0, 31] (v_alignbit_b32).
__device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t s) {
  return __builtin_amdgcn_alignbit(hi, lo, s);
}

// Row layout (16 lanes per block): lane i of the row extracts the D4 deltas
// of positions q = 2i and 2i + 1 for all four lanes j, i.e. block integers
// 8i .. 8i + 7.  Word rows m = floor(q b / 32) .. m + 2 are read as 16-byte
// vectors (word 4m + j of lane j sits in component j).  load_row issues
// the lane's three row loads and unpack_row extracts from them, so a caller
// can put other work between the two; extract_row does both.
struct RowWords {
  uint4 r0, r1, r2;
};
__device__ __forceinline__ RowWords load_row(const uint32_t *__restrict__ blk, uint32_t b, uint32_t i) {
  const gconst<uint4> p = gbl(reinterpret_cast<const uint4 *>(blk)) + ((2u * i * b) >> 5);
  return RowWords{p[0], p[1], p[2]};
}
__device__ __forceinline__ void unpack_row(const RowWords &w, uint32_t b, uint32_t i, uint32_t d0[4], uint32_t d1[4]) {
  const uint32_t bit0 = 2u * i * b;
  const uint32_t m0 = bit0 >> 5, s0 = bit0 & 31u;
  const uint32_t bit1 = bit0 + b;
  const uint32_t s1 = bit1 & 31u;
  const bool step = (bit1 >> 5) != m0;
  const uint4 r0 = w.r0, r1 = w.r1, r2 = w.r2;
  const uint32_t mask = width_mask(b);
  d0[0] = funnel(r1.x, r0.x, s0) & mask;
  d0[1] = funnel(r1.y, r0.y, s0) & mask;
  d0[2] = funnel(r1.z, r0.z, s0) & mask;
  d0[3] = funnel(r1.w, r0.w, s0) & mask;
  const uint4 lo = step ? r1 : r0;
  const uint4 hi = step ? r2 : r1;
  d1[0] = funnel(hi.x, lo.x, s1) & mask;
  d1[1] = funnel(hi.y, lo.y, s1) & mask;
  d1[2] = funnel(hi.z, lo.z, s1) & mask;
  d1[3] = funnel(hi.w, lo.w, s1) & mask;
}
__device__ __forceinline__ void extract_row(const uint32_t *__restrict__ blk, uint32_t b, uint32_t i,
                                            uint32_t d0[4], uint32_t d1[4]) {
  unpack_row(load_row(blk, b, i), b, i, d0, d1);
}

// Inverse differential coding (Sec. 5) of the row layout: lane i holds the
// deltas of block positions 8i .. 8i + 3 (d0) and 8i + 4 .. 8i + 7 (d1);
// `seed` holds the four values just before the lanes' span (the previous
// block's last four values, or the carry of the previous pass).  The scans
// run over a 16-lane row (ROW, one block) or over the whole wave (four
// consecutive blocks).  Per form:
//   D4  each residue class j mod 4 is one chain: scan of d0[j] + d1[j];
//   D1  one chain through every position: lane totals scanned once;
//   D2  even and odd positions are two chains: two scans;
//   DM  the quad ends (positions 4q + 3) form one chain; the other values
//       of a quad add their delta to the previous quad end.
template <bool ROW, uint32_t MODE>
__device__ __forceinline__ void prefix_form(const uint32_t d0[4], const uint32_t d1[4], const uint32_t seed[4],
                                            uint32_t x0[4], uint32_t x1[4]) {
  auto scan = [](uint32_t v) { return ROW ? scan_row16(v) : scan_wave64(v); };
  if (MODE == S4_DELTA_D1) {
    uint32_t l[8];
    l[0] = d0[0];
    l[1] = l[0] + d0[1];
    l[2] = l[1] + d0[2];
    l[3] = l[2] + d0[3];
    l[4] = l[3] + d1[0];
    l[5] = l[4] + d1[1];
    l[6] = l[5] + d1[2];
    l[7] = l[6] + d1[3];
    const uint32_t base = seed[3] + scan(l[7]) - l[7];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x0[j] = base + l[j];
      x1[j] = base + l[4 + j];
    }
  } else if (MODE == S4_DELTA_D2) {
    const uint32_t e0 = d0[0], e1 = e0 + d0[2], e2 = e1 + d1[0], e3 = e2 + d1[2];
    const uint32_t o0 = d0[1], o1 = o0 + d0[3], o2 = o1 + d1[1], o3 = o2 + d1[3];
    const uint32_t be = seed[2] + scan(e3) - e3;
    const uint32_t bo = seed[3] + scan(o3) - o3;
    x0[0] = be + e0;
    x0[1] = bo + o0;
    x0[2] = be + e1;
    x0[3] = bo + o1;
    x1[0] = be + e2;
    x1[1] = bo + o2;
    x1[2] = be + e3;
    x1[3] = bo + o3;
  } else if (MODE == S4_DELTA_DM) {
    const uint32_t tot = d0[3] + d1[3];
    const uint32_t y0 = seed[3] + scan(tot) - tot;  // quad end before position 8i
    const uint32_t y1 = y0 + d0[3];                   // quad end before position 8i + 4
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x0[j] = y0 + d0[j];
      x1[j] = y1 + d1[j];
    }
  } else {
    // x0 before x1, as in the other forms: with one store order in every
    // form the compiler merges the forms' stores without taking the
    // arrays' addresses (which would put them in scratch memory)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t hi = seed[j] + scan(d0[j] + d1[j]);
      x0[j] = hi - d1[j];
      x1[j] = hi;
    }
  }
}

// The same with the form known only at run time (uniform across the wave).
template <bool ROW>
__device__ __forceinline__ void prefix_deltas(uint32_t mode, const uint32_t d0[4], const uint32_t d1[4],
                                              const uint32_t seed[4], uint32_t x0[4], uint32_t x1[4]) {
  switch (mode) {
    case S4_DELTA_D1: prefix_form<ROW, S4_DELTA_D1>(d0, d1, seed, x0, x1); break;
    case S4_DELTA_D2: prefix_form<ROW, S4_DELTA_D2>(d0, d1, seed, x0, x1); break;
    case S4_DELTA_DM: prefix_form<ROW, S4_DELTA_DM>(d0, d1, seed, x0, x1); break;
    default: prefix_form<ROW, S4_DELTA_D4>(d0, d1, seed, x0, x1); break;
  }
}

// Patching (S4-FastPFOR, Sec. 4.4) of the block of a patched list whose
// exception record is x, on the block's 128 deltas staged in LDS
// v[0..127] in block order: the row's 16
// lanes take its exceptions e = i, i + 16, ...; each adds its high part,
// d = b - b' bits read from the page's array for d at the block's running
// index, above the b' low bits unpacked at its position.  Exceptions of a
// block sit at distinct positions, so the adds never collide.
__device__ __forceinline__ void patch_block_rec(const DList &L, const uint4 x, uint32_t i, uint32_t *v) {
  const uint32_t c = x.x & 0xFFu, d = (x.x >> 8) & 0x3Fu, bp = (x.x >> 16) & 0x3Fu;
  const uint32_t *xd = exc_data(L);
  const gconst<uint8_t> pos = gbl(reinterpret_cast<const uint8_t *>(xd)) + x.y;
  const gconst<uint32_t> arr = gbl(xd) + x.z;
  for (uint32_t e = i; e < c; e += 16) {
    const uint32_t bit = (x.w + e) * d;
    const uint32_t w = bit >> 5, s = bit & 31u;
    const uint32_t lo = arr[w], hi = arr[w + 1];  // the array's pad word keeps w + 1 inside
    const uint32_t h = funnel(hi, lo, s) & width_mask(d);
    v[pos[e]] += h << bp;
  }
}

// Stage a row's deltas (positions 8i .. 8i + 7) in its LDS slice v, patch
// them with the exceptions of the block whose record rec() gives, and load
// them back.  Whole-wave call (it synchronises the wave); only rows with
// `active` touch their slice or call rec().
template <class Rec>
__device__ __forceinline__ void patch_row_with(const DList &L, Rec rec, bool active, uint32_t i, uint32_t *v,
                                               uint32_t d0[4], uint32_t d1[4]) {
  u32x4 *t = reinterpret_cast<u32x4 *>(v + 8u * i);
  if (active) {
    t[0] = u32x4{d0[0], d0[1], d0[2], d0[3]};
    t[1] = u32x4{d1[0], d1[1], d1[2], d1[3]};
  }
  wave_sync();
  if (active) patch_block_rec(L, rec(), i, v);
  wave_sync();
  if (active) {
    const u32x4 a = t[0], b = t[1];
    d0[0] = a.x; d0[1] = a.y; d0[2] = a.z; d0[3] = a.w;
    d1[0] = b.x; d1[1] = b.y; d1[2] = b.z; d1[3] = b.w;
  }
  wave_sync();
}

// For block k of L, its record read once the deltas are staged.
__device__ __forceinline__ void patch_row(const DList &L, uint32_t k, bool active, uint32_t i, uint32_t *v,
                                          uint32_t d0[4], uint32_t d1[4]) {
  patch_row_with(L, [&] { return uint4(gbl(exc_records(L))[k]); }, active, i, v, d0, d1);
}

// For a row whose block's record x was loaded ahead (a pass ahead in the
// decode kernels), which leaves the patch one memory round trip, not two.
__device__ __forceinline__ void patch_row_rec(const DList &L, const uint4 x, bool active, uint32_t i, uint32_t *v,
                                              uint32_t d0[4], uint32_t d1[4]) {
  patch_row_with(L, [&] { return x; }, active, i, v, d0, d1);
}

// Feature set of a chunk-pipeline instantiation: the kinds of list it can
// meet beyond plain compressed lists.  Kernels are instantiated per set so
// that work with neither pays nothing for them (registers, branches).
constexpr uint32_t kFeatBitmap = 1;   // hybrid-index bitmap lists
constexpr uint32_t kFeatPatched = 2;  // patched (S4-FastPFOR) lists
constexpr uint32_t kFeatParts = 4;    // doc-ID partitioned index (per-part queues; batch kernel only)
constexpr uint32_t kFeatCount = 8;    // algorithmic traffic counted (the batch kernel's counting runs only)

// Decode block k of L with one 16-lane row per block: extract, patch when
// the list is patched (its exceptions, staged through the row's 128-word
// LDS slice `scratch`; only with PATCHED), then the integrated prefix sum
// of the list's differential form (Alg. 1 with the form's P(t, v)) seeded
// from the skip index.  Rows whose `active` is false compute zeros.  All
// 64 lanes must call this together, for one list.
template <bool PATCHED>
__device__ __forceinline__ void decode_row(const DList &L, uint32_t k, bool active, uint32_t i,
                                           uint32_t x0[4], uint32_t x1[4], uint32_t *scratch) {
  uint32_t d0[4] = {0, 0, 0, 0}, d1[4] = {0, 0, 0, 0};
  uint4 seed = make_uint4(0, 0, 0, 0);
  if (active) {
    extract_row(L.payload + gbl(L.offs)[k], gbl(L.widths)[k], i, d0, d1);
    seed = gbl(L.seeds)[k];
  }
  if (PATCHED && is_patched(L)) patch_row(L, k, active, i, scratch, d0, d1);
  const uint32_t sv[4] = {seed.x, seed.y, seed.z, seed.w};
  prefix_deltas<true>(L.mode, d0, d1, sv, x0, x1);
}

// The same where every row names a block of the list (k < L.nb in every
// lane): rows whose values are not wanted pass some block that is (or
// another valid one) and `active` false, which only keeps them out of the
// patch step.  With no row to switch off, no lane waits on a branch or
// zeroes its deltas.
template <bool PATCHED>
__device__ __forceinline__ void decode_row_any(const DList &L, uint32_t k, bool active, uint32_t i,
                                               uint32_t x0[4], uint32_t x1[4], uint32_t *scratch) {
  uint32_t d0[4], d1[4];
  extract_row(L.payload + gbl(L.offs)[k], gbl(L.widths)[k], i, d0, d1);
  const uint4 seed = gbl(L.seeds)[k];
  if (PATCHED && is_patched(L)) patch_row(L, k, active, i, scratch, d0, d1);
  const uint32_t sv[4] = {seed.x, seed.y, seed.z, seed.w};
  prefix_deltas<true>(L.mode, d0, d1, sv, x0, x1);
}

// Decode block k of L (a D4 list) with the whole wave (half-wave layout):
// lane l takes q = l mod 32 and lanes j0 = 2 (l div 32), j0 + 1; the two
// half-waves scan over q.  Writes the 128 values to dst[0..127].
__device__ __forceinline__ void decode_block_wave(const DList &L, uint32_t k, uint32_t *dst) {
  const uint32_t l = lane_id();
  const uint32_t q = l & 31u, j0 = (l >> 5) * 2u;
  const uint4 seed = gbl(L.seeds)[k];  // issued with the width and offset loads
  const uint32_t b = gbl(L.widths)[k];
  const uint32_t *w = L.payload + gbl(L.offs)[k];
  const uint32_t bit = q * b, m = bit >> 5, s = bit & 31u;
  const uint2 lo = *gbl(reinterpret_cast<const uint2 *>(w + 4u * m + j0));
  const uint2 hi = *gbl(reinterpret_cast<const uint2 *>(w + 4u * m + 4u + j0));
  const uint32_t mask = width_mask(b);
  const uint32_t d0 = funnel(hi.x, lo.x, s) & mask;
  const uint32_t d1 = funnel(hi.y, lo.y, s) & mask;
  const uint32_t s0 = j0 ? seed.z : seed.x, s1 = j0 ? seed.w : seed.y;
  const uint32_t x0 = s0 + scan_half32(d0);
  const uint32_t x1 = s1 + scan_half32(d1);
  *reinterpret_cast<uint2 *>(dst + 4u * q + j0) = make_uint2(x0, x1);
}

// First index c in [lo, hi) with v[c] >= key, else hi (v: an LDS array or a
// global view).
template <class Ptr>
__device__ __forceinline__ uint32_t lower_bound_u32(Ptr v, uint32_t lo, uint32_t hi, uint32_t key) {
  uint32_t len = hi - lo;
  while (len > 0) {
    const uint32_t half = len >> 1;
    if (v[lo + half] < key) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return lo;
}

// Whether key is among the values of a decoded block row in LDS: 128
// sorted values, or a raw tail of n < 128 values followed by 0xFFFFFFFF
// entries, for a key no larger than the row's largest value (the
// candidate choice over the skip index guarantees it: a key goes to the
// first block whose maximum is not below it, and to the tail only when
// it is at most the list's last value).  A lower bound by seven fixed
// halvings then lands on a real entry; one compare decides.  The probe is
// a byte address in LDS that each step advances by its distance when the
// entry it reads is below the key (a read with an immediate offset, a
// compare, a select and a shifted add); the empty asm keeps the compiler
// from rebuilding it as the row base plus an offset every step.
__device__ __forceinline__ bool block_has(const uint32_t *v, uint32_t key) {
  using lds_u32 = const S4_ADDRSPACE(3) uint32_t;
  uint32_t a = uint32_t(uintptr_t((lds_u32 *)v));
#pragma unroll
  for (int lg = 6; lg >= 0; --lg) {
    const uint32_t t = *(lds_u32 *)uintptr_t(a + (4u << lg) - 4u);
    a += uint32_t(t < key) << (lg + 2);
    asm volatile("" : "+v"(a));
  }
  return *(lds_u32 *)uintptr_t(a) == key;
}

// Two lower bounds at once over v[0 .. n): r0 = first index with
// v[r0] >= key0, r1 = first with v[r1] >= key1 (n if none).  Lanes 0..31
// work on key0 and lanes 32..63 on key1; every round each half probes 32
// evenly spaced entries of its current range in parallel and keeps the
// piece between the last entry below the key and the first one not below,
// so a range of n entries takes about log_32 n rounds of loads instead of
// log_2 n dependent ones.  All 64 lanes call this; the results are uniform.
__device__ __forceinline__ void coop_lower_bound2(gconst<uint32_t> v, uint32_t n, uint32_t key0, uint32_t key1,
                                                  uint32_t &r0, uint32_t &r1) {
  const uint32_t lane = lane_id();
  const bool upper = lane >= 32;
  const uint32_t sub = lane & 31u;
  const uint32_t key = upper ? key1 : key0;
  uint32_t lo0 = 0, hi0 = n, lo1 = 0, hi1 = n;  // answer of each half lies in [lo, hi]
  while (hi0 > lo0 || hi1 > lo1) {
    const uint32_t lo = upper ? lo1 : lo0, hi = upper ? hi1 : hi0;
    const uint32_t len = hi - lo;
    const uint32_t step = (len + 31u) >> 5;
    const uint32_t pos = lo + sub * step;
    const bool below = len > 0 && pos < hi && v[pos] < key;
    const uint64_t m = __ballot(below);
    const uint32_t c0 = uint32_t(__popcll(m & 0xFFFFFFFFull)), c1 = uint32_t(__popcll(m >> 32));
    if (hi0 > lo0) {
      const uint32_t st = (hi0 - lo0 + 31u) >> 5;
      const uint32_t nlo = c0 ? lo0 + (c0 - 1) * st + 1 : lo0;
      const uint32_t nhi = min(hi0, lo0 + c0 * st);
      lo0 = nlo;
      hi0 = max(nlo, nhi);
    }
    if (hi1 > lo1) {
      const uint32_t st = (hi1 - lo1 + 31u) >> 5;
      const uint32_t nlo = c1 ? lo1 + (c1 - 1) * st + 1 : lo1;
      const uint32_t nhi = min(hi1, lo1 + c1 * st);
      lo1 = nlo;
      hi1 = max(nlo, nhi);
    }
  }
  r0 = uniform(lo0);
  r1 = uniform(lo1);
}

// The same two lower bounds when both answers are known to be >= start:
// a first round probes the 32 entries from start (lanes 0..31 for key0,
// 32..63 for key1; the entries below a key form a prefix of the window),
// which settles both keys when their answers lie in it; only what is left
// goes to the 32-ary search of the rest.  Consecutive chunks of one list
// pass the previous chunk's last block as start, so in the merge regime
// a search costs one round instead of log_32 n.  The window is returned:
// win_at = start when the round ran (else kInvalid), and lane l (l < 32)
// holds v[start + l] in win (kInvalid past the end).
__device__ __forceinline__ void coop_lower_bound2_from(gconst<uint32_t> v, uint32_t n, uint32_t start, uint32_t key0,
                                                       uint32_t key1, uint32_t &r0, uint32_t &r1, uint32_t &win,
                                                       uint32_t &win_at) {
  win = kInvalid;
  win_at = kInvalid;
  if (start == 0) {
    coop_lower_bound2(v, n, key0, key1, r0, r1);
    return;
  }
  const uint32_t lane = lane_id();
  const uint32_t pos = start + (lane & 31u);
  const uint32_t key = lane >= 32 ? key1 : key0;
  if (pos < n) win = v[pos];
  win_at = start;
  const bool below = pos < n && win < key;
  const uint64_t m = __ballot(below);
  const uint32_t c0 = uint32_t(__popcll(m & 0xFFFFFFFFull)), c1 = uint32_t(__popcll(m >> 32));
  r0 = start + c0;
  r1 = start + c1;
  // a key with all 32 window entries below it (the window inside the list)
  // continues past the window; key0 <= key1, so key1 is then unsettled too
  if (c1 == 32 && start + 32 < n) {
    uint32_t a0, a1;
    coop_lower_bound2(v + (start + 32), n - (start + 32), key0, key1, a0, a1);
    if (c0 == 32) r0 = start + 32 + a0;
    r1 = start + 32 + a1;
  }
}

// ------------------------------------------------------------ pair items

// Per-wave LDS of the intersection kernels.
struct ItemLds {
  uint32_t r[kBlock];          // the 128-value chunk of r
  uint32_t f[4][kBlock];       // four decoded candidate blocks of f
  uint32_t cand[kBlock];       // distinct candidate blocks of f
  uint32_t bm[kMaxGallopBlocks];  // staged bmax entries (merge regime)
};

// The short side of a pair: a compressed list, or raw values on the device.
struct RSide {
  DList L;
  const uint32_t *raw;  // null when compressed
  uint64_t len;         // number of values of r
};

// Algorithmic bytes read by a wave (uniform): packed payload + width byte +
// block offset + seed of every decoded block, staged skip-index entries,
// raw values; and the number of blocks decoded.  Counted only when `on`,
// which the batch kernel's counting instantiation alone sets: the count (a
// width load and cross-lane reads per candidate group, and 64-bit
// accumulators) would cost the other chunk kernels registers and issue
// slots.
struct Traffic {
  uint64_t bytes = 0;
  uint64_t blocks = 0;
  bool on = false;
  __device__ __forceinline__ void add(uint64_t b, uint64_t k = 0) {
    if (on) {
      bytes += b;
      blocks += k;
    }
  }
};

// Chunk `item` of a bitmap list (its values of rank 128 item .. 128 item +
// 127) into s.r: from the chunk's select sample (its first value), 64 words
// at a time, each lane takes one word, an inclusive wave scan of the
// popcounts places its set bits, and lanes write their values in
// increasing order.  Returns the number of values (uniform).
__device__ __forceinline__ uint32_t load_bitmap_chunk(const DList &L, uint32_t item, ItemLds &s, Traffic &tr) {
  const uint32_t lane = lane_id();
  const uint64_t base = uint64_t(item) * kBlock;
  const uint32_t want = L.n > base ? uint32_t(min<uint64_t>(kBlock, L.n - base)) : 0u;
  uint32_t got = 0;
  if (want) {
    const uint32_t first = uniform(gbl(L.bmax)[item]);
    const uint32_t w0 = first >> 5;
    tr.add(4u);
    for (uint32_t w = w0; got < want && w < L.aux; w += 64) {
      const uint32_t wi = w + lane;
      uint32_t word = wi < L.aux ? gbl(L.payload)[wi] : 0u;
      if (wi == w0) word &= ~((1u << (first & 31u)) - 1u);  // bits of earlier chunks
      tr.add(4u * min(64u, L.aux - w));
      const uint32_t pc = uint32_t(__popc(word));
      const uint32_t incl = scan_wave64(pc);
      uint32_t pos = got + incl - pc;
      while (word && pos < want) {
        s.r[pos++] = (wi << 5) | uint32_t(__builtin_ctz(word));
        word &= word - 1u;
      }
      got += uint32_t(__builtin_amdgcn_readlane(int(incl), 63));
    }
  }
  wave_sync();
  return min(got, want);
}

// Load chunk `item` of r (values 128 item .. 128 item + 127) into s.r;
// returns how many values it has.  The whole wave calls this.
template <uint32_t FEAT>
__device__ __forceinline__ uint32_t load_chunk(const RSide &r, uint32_t item, ItemLds &s, Traffic &tr) {
  const uint32_t lane = lane_id();
  uint32_t cnt;
  if (r.raw) {
    const uint64_t base = uint64_t(item) * kBlock;
    const uint64_t left = r.len > base ? r.len - base : 0;
    cnt = left < kBlock ? uint32_t(left) : kBlock;
    if (lane < cnt) s.r[lane] = gbl(r.raw)[base + lane];
    if (lane + 64 < cnt) s.r[lane + 64] = gbl(r.raw)[base + 64 + lane];
  } else if ((FEAT & kFeatBitmap) && r.L.mode == kBitmapList) {
    return load_bitmap_chunk(r.L, item, s, tr);
  } else if (item < r.L.nb) {
    cnt = kBlock;
    if (tr.on) tr.add(16u * uniform(gbl(r.L.widths)[item]) + 1u + 4u + 16u, 1);  // width load only when counting
    if (r.L.mode == S4_DELTA_D4 && !((FEAT & kFeatPatched) && is_patched(r.L))) {
      decode_block_wave(r.L, item, s.r);
    } else {
      // other forms and patched lists: row 0 decodes the block in the row
      // layout (patching through s.r)
      uint32_t x0[4], x1[4];
      const uint32_t ri = lane & 15u;
      decode_row_any<(FEAT & kFeatPatched) != 0>(r.L, item, lane < 16, ri, x0, x1, s.r);
      if (lane < 16) {
        *reinterpret_cast<uint4 *>(&s.r[8 * ri]) = make_uint4(x0[0], x0[1], x0[2], x0[3]);
        *reinterpret_cast<uint4 *>(&s.r[8 * ri + 4]) = make_uint4(x1[0], x1[1], x1[2], x1[3]);
      }
    }
  } else {
    cnt = item == r.L.nb ? r.L.t : 0u;
    if (lane < cnt) s.r[lane] = gbl(r.L.tail)[lane];
    if (lane + 64 < cnt) s.r[lane + 64] = gbl(r.L.tail)[lane + 64];
  }
  if (r.raw || item >= r.L.nb) tr.add(4u * cnt);
  wave_sync();
  return cnt;
}

// Ordered compaction (ballot + mbcnt), in place: lane values a0 (position
// lane) and a1 (position lane + 64) are kept where f0 / f1; returns the
// number kept (uniform).
__device__ __forceinline__ uint32_t compact_chunk(bool f0, bool f1, uint32_t a0, uint32_t a1, ItemLds &s) {
  const uint64_t mm0 = __ballot(f0), mm1 = __ballot(f1);
  const uint32_t k0 = uint32_t(__popcll(mm0));
  wave_sync();
  if (f0) s.r[mbcnt64(mm0)] = a0;
  if (f1) s.r[k0 + mbcnt64(mm1)] = a1;
  wave_sync();
  return k0 + uint32_t(__popcll(mm1));
}

// Intersect the sorted values s.r[0 .. cnt) with list f; the values found
// in f are compacted in order to the front of s.r and their number is
// returned (uniform).  Only candidate blocks of f are decoded: for every
// value the first block whose bmax is >= the value (Sec. 6: the search of
// the long list for each value of the short one, done here per lane over
// the skip index), each distinct candidate once.
template <bool PATCHED>
__device__ __forceinline__ uint32_t intersect_chunk(uint32_t cnt, const DList &f, ItemLds &s,
                                                    uint32_t gallop_blocks, Traffic &tr, uint32_t &hint) {
  const uint32_t lane = lane_id();
  const bool v0 = lane < cnt, v1 = lane + 64 < cnt;
  const uint32_t a0 = v0 ? s.r[lane] : 0u;
  const uint32_t a1 = v1 ? s.r[lane + 64] : 0u;
  const uint32_t first = uniform(s.r[0]);
  const uint32_t last = uniform(s.r[cnt ? cnt - 1 : 0]);
  const uint32_t nbf = f.nb;
  const bool ftail = f.t > 0;
  // f's largest value and the span of f blocks that can hold [first, last]
  // (index nb stands for the raw tail, bmax taken as +infinity there); the
  // two are independent, so their loads overlap
  uint32_t fmax = 0;
  if (f.n > 0) fmax = ftail ? gbl(f.tail)[f.t - 1] : gbl(f.bmax)[nbf - 1];
  // hint: a block index no later than this chunk's first candidate (the
  // previous chunk's last candidate, or 0); it becomes this chunk's last
  uint32_t lo = 0, hi = 0, win = kInvalid, win_at = kInvalid;
  if (cnt > 0) {
    coop_lower_bound2_from(gbl(f.bmax), nbf, min(hint, nbf), first, last, lo, hi, win, win_at);
    hint = hi;
  }
  const bool any = cnt > 0 && f.n > 0 && first <= fmax;
  bool f0 = false, f1 = false;
  if (any) {
    const uint32_t span = hi - lo + 1;
    uint32_t c0, c1;
    if (span <= gallop_blocks) {
      // merge regime: stage the spanned bmax entries in LDS, search there
      // (from the search's window when it holds them: no memory round trip)
      if (win_at != kInvalid && lo >= win_at && lo + span <= win_at + 32) {
        const uint32_t x = uint32_t(__shfl(int(win), int(lo - win_at + min(lane, span - 1))));
        if (lane < span) s.bm[lane] = x;
      } else {
        for (uint32_t e = lane; e < span; e += 64) s.bm[e] = (lo + e < nbf) ? gbl(f.bmax)[lo + e] : kInvalid;
      }
      tr.add(4u * span);
      wave_sync();
      c0 = lo + lower_bound_u32(s.bm, 0, span - 1, a0);
      c1 = lo + lower_bound_u32(s.bm, 0, span - 1, a1);
    } else {
      // galloping regime: each lane searches the skip index in memory
      c0 = lower_bound_u32(gbl(f.bmax), lo, hi, a0);
      c1 = lower_bound_u32(gbl(f.bmax), lo, hi, a1);
    }
    const bool ok0 = v0 && a0 <= fmax;
    const bool ok1 = v1 && a1 <= fmax;
    // distinct candidates (c is non-decreasing over the chunk)
    uint32_t p0 = __shfl_up(c0, 1);
    uint32_t p1 = __shfl_up(c1, 1);
    const uint32_t c0_last = __shfl(c0, 63);
    if (lane == 0) p1 = c0_last;
    const bool n0 = ok0 && (lane == 0 || c0 != p0);
    const bool n1 = ok1 && (c1 != p1);
    const uint64_t m0 = __ballot(n0), m1 = __ballot(n1);
    const uint32_t u0 = uint32_t(__popcll(m0));
    const uint32_t U = u0 + uint32_t(__popcll(m1));
    if (n0) s.cand[mbcnt64(m0)] = c0;
    if (n1) s.cand[u0 + mbcnt64(m1)] = c1;
    const uint32_t slot0 = ok0 ? mbcnt64(m0) + (n0 ? 1u : 0u) - 1u : kInvalid;
    const uint32_t slot1 = ok1 ? u0 + mbcnt64(m1) + (n1 ? 1u : 0u) - 1u : kInvalid;
    wave_sync();
    // decode candidate blocks four at a time (one row each) and search
    const uint32_t row = lane >> 4, ri = lane & 15u;
    for (uint32_t g = 0; g < U; g += 4) {
      const uint32_t cs = g + row;
      const uint32_t blk = cs < U ? s.cand[cs] : kInvalid;
      // traffic of the four rows' blocks, summed from each row's first lane
      if (tr.on) {
        uint32_t tb = 0;
        if (ri == 0) tb = blk < nbf ? 16u * gbl(f.widths)[blk] + 21u : (blk == nbf ? 4u * f.t : 0u);
        tr.bytes += uint32_t(__builtin_amdgcn_readlane(int(tb), 0)) + uint32_t(__builtin_amdgcn_readlane(int(tb), 16)) +
                    uint32_t(__builtin_amdgcn_readlane(int(tb), 32)) + uint32_t(__builtin_amdgcn_readlane(int(tb), 48));
        tr.blocks += min(4u, U - g);
      }
      // rows past the candidates, and the tail's row, decode a candidate
      // block of the group instead (row 0's, else the last full block):
      // their values are not kept
      if (nbf > 0) {
        const uint32_t b0 = uint32_t(__builtin_amdgcn_readfirstlane(int(blk)));
        const uint32_t kb = blk < nbf ? blk : (b0 < nbf ? b0 : nbf - 1);
        uint32_t x0[4], x1[4];
        decode_row_any<PATCHED>(f, kb, blk < nbf, ri, x0, x1, s.f[row]);
        if (blk < nbf) {
          *reinterpret_cast<uint4 *>(&s.f[row][8 * ri]) = make_uint4(x0[0], x0[1], x0[2], x0[3]);
          *reinterpret_cast<uint4 *>(&s.f[row][8 * ri + 4]) = make_uint4(x1[0], x1[1], x1[2], x1[3]);
        }
      }
      if (blk == nbf) {
        // the raw tail, padded to a full row for block_has
        for (uint32_t e = 0; e < 8; ++e)
          s.f[row][8 * ri + e] = 8 * ri + e < f.t ? gbl(f.tail)[8 * ri + e] : kInvalid;
      }
      wave_sync();
      if (slot0 - g < 4u) f0 = block_has(s.f[slot0 - g], a0);
      if (slot1 - g < 4u) f1 = block_has(s.f[slot1 - g], a1);
      wave_sync();
    }
  }
  return compact_chunk(f0, f1, a0, a1, s);
}

// Keep the values s.r[0 .. cnt) whose bit is set in bitmap list f (hyb+m2,
// Sec. 7.7: the survivors of the compressed lists are checked against the
// bitmaps one by one): one word gathered per value, then ordered compaction.
__device__ __forceinline__ uint32_t probe_chunk(uint32_t cnt, const DList &f, ItemLds &s, Traffic &tr) {
  const uint32_t lane = lane_id();
  const bool v0 = lane < cnt, v1 = lane + 64 < cnt;
  const uint32_t a0 = v0 ? s.r[lane] : 0u;
  const uint32_t a1 = v1 ? s.r[lane + 64] : 0u;
  bool f0 = false, f1 = false;
  if (v0 && (a0 >> 5) < f.aux) f0 = (gbl(f.payload)[a0 >> 5] >> (a0 & 31u)) & 1u;
  if (v1 && (a1 >> 5) < f.aux) f1 = (gbl(f.payload)[a1 >> 5] >> (a1 & 31u)) & 1u;
  tr.add(4u * cnt);
  return compact_chunk(f0, f1, a0, a1, s);
}

// Write s.r[0 .. cnt) to out and cnt to *count.
__device__ __forceinline__ void store_chunk(uint32_t cnt, const ItemLds &s, uint32_t *__restrict__ out,
                                            uint32_t *__restrict__ count) {
  const uint32_t lane = lane_id();
  if (lane < cnt) gbl_out(out)[lane] = s.r[lane];
  if (lane + 64 < cnt) gbl_out(out)[lane + 64] = s.r[lane + 64];
  if (lane == 0) *gbl_out(count) = cnt;
}

// SvS over one chunk: intersect chunk `item` of r with lists f[0 .. nf) in
// order, stopping early when nothing survives (Sec. 6: pairwise, from the
// shortest list up).  Intersection distributes over a partition of the
// shortest list, so chunks are independent.
// hint0: the search hint of the first list (see intersect_chunk), carried
// by the caller from one chunk of r to the next; later lists start at 0.
template <uint32_t FEAT, class FList>
__device__ __forceinline__ uint32_t chain_chunk(const RSide &r, uint32_t item, const DList &f0, FList f, uint32_t nf,
                                                ItemLds &s, uint32_t gallop_blocks, Traffic &tr, uint32_t &hint0) {
  uint32_t cnt = load_chunk<FEAT>(r, item, s, tr);
  // f0 (the second-shortest list, j = 0) comes in already loaded; later
  // lists are loaded as the chain reaches them
  DList fj = f0;
  for (uint32_t j = 0; j < nf && cnt > 0; ++j) {
    if (j > 0) fj = f(j);
    if ((FEAT & kFeatBitmap) && fj.mode == kBitmapList)
      cnt = probe_chunk(cnt, fj, s, tr);
    else {
      uint32_t h = 0;
      cnt = intersect_chunk<(FEAT & kFeatPatched) != 0>(cnt, fj, s, gallop_blocks, tr, j == 0 ? hint0 : h);
    }
  }
  tr.add(4u * cnt);  // the chunk's results
  return cnt;
}

}  // namespace s4

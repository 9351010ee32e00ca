/*
 * oracle.c -- plain, slow, obviously-correct CPU reference for the
 * S4-BP128-D4 codec and sorted-set intersection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can check the GPU path against an
 * independent implementation.  It shares no source, header, table or
 * helper with the GPU library: the stream layout below is re-implemented
 * here from its written description.
 *
 * Paper: D. Lemire, L. Boytsov, N. Kurz, "SIMD Compression and the
 * Intersection of Sorted Integers" (arXiv:1401.6399).
 *
 *   - Binary packing in 128-integer blocks, one bit-width byte per block,
 *     width = smallest b with every value < 2^b, 0 <= b <= 32
 *     (Sec. 4.3, S4-BP128).
 *   - 4-way interleaved packing: integer 4q+j of a block goes to lane j;
 *     lane j is an LSB-first stream of 32 values of b bits stored in words
 *     j, 4+j, 8+j, ...; a value that straddles a word boundary continues in
 *     the same lane's next word (Sec. 4.2, Fig. 2).
 *   - Differential coding (Sec. 5), one of four forms recorded in the
 *     stream: D4 delta_i = x_i - x_{i-4}; DM delta_{4i+j} = x_{4i+j} -
 *     x_{4i-1}; D2 delta_i = x_i - x_{i-2}; D1 delta_i = x_i - x_{i-1};
 *     values before the list are 0.  The inverse (a prefix sum) runs over
 *     the whole list, seeded with zeros (Alg. 1).
 *   - Intersection: the textbook two-pointer merge (the scalar baseline of Sec. 6) and
 *     SvS folding of k lists (Sec. 6).
 *
 * Readings where the paper is silent or garbled (each is also listed in
 * the design notes):
 *   - the final < 128 integers are stored as raw uint32 (the paper stores
 *     them with varint, Sec. 4.3);
 *   - the width bytes of all blocks are stored together before the packed
 *     payload (the paper groups them per 2048-integer meta-block); the
 *     byte count differs only by the <= 3 padding bytes;
 *   - b = 0 decodes to 128 zero deltas; at b = 32 the mask is all ones;
 *   - intersections require strictly increasing inputs; results are sets.
 *
 * Serialized stream (little-endian), as written and read here:
 *   0  u32 magic 0x34443453 ("S4D4")
 *   4  u16 version (1)
 *   6  u16 flags  (bit 0: input strictly increasing; bits 1-2: differential
 *                  form, 0 = D4, 1 = DM, 2 = D2, 3 = D1; other bits zero)
 *   8  u64 n      (number of integers)
 *   16 u32 nb     (= floor(n / 128), number of packed blocks)
 *   20 u32 t      (= n - 128 nb, raw tail length)
 *   24 u64 pw     (payload words = sum over blocks of 4 b_k)
 *   32 u8 widths[nb], then zero bytes up to a multiple of 4
 *      u32 payload[pw]
 *      u32 tail[t]
 *   With flag bit 3 (S4-FastPFOR, Sec. 4.4) the widths are the packed
 *   widths b' and the payload holds each delta's low b' bits; after the tail
 *   come the pages of up to 512 blocks, each:
 *      u32 meta_len, then per block: u8 b, u8 c, c u8 positions (increasing),
 *      zero bytes up to a multiple of 4;
 *      u32 present (bit d-1 set when the page has exceptions with b - b' = d),
 *      then for each such d ascending: u32 count, and the counted high parts
 *      (delta >> b') packed LSB-first at d bits each, value e at bit e d,
 *      padded to a multiple of 32 values (d words per 32).
 *
 * Parity status of each function is recorded in the tests that pin it.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_EUNSORTED (-2)
#define ORC_ERANGE (-3)
#define ORC_ECORRUPT (-4)
#define ORC_ENOMEM (-5)

#define ORC_MAGIC 0x34443453u
#define ORC_HEADER 32u
#define ORC_PATCHED 8u  /* flag bit 3: S4-FastPFOR */
#define ORC_PAGE 512u   /* blocks whose exceptions are pooled (Sec. 4.4) */

static void put32(uint8_t *p, uint32_t v) {
  p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8);
  p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}
static void put16(uint8_t *p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put64(uint8_t *p, uint64_t v) { put32(p, (uint32_t)v); put32(p + 4, (uint32_t)(v >> 32)); }
static uint32_t get32(const uint8_t *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
static uint16_t get16(const uint8_t *p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint64_t get64(const uint8_t *p) { return (uint64_t)get32(p) | ((uint64_t)get32(p + 4) << 32); }

/* Block width (Sec. 4.3): the least b for which every delta of the block
 * is below 2^b.  Written as that definition (increase b until every value
 * fits), in 64-bit arithmetic so that b = 32 is reachable. */
static uint32_t orc_width(const uint32_t *d, size_t count) {
  uint32_t b = 0;
  for (;;) {
    int all_fit = 1;
    for (size_t i = 0; i < count; ++i)
      if ((uint64_t)d[i] >= ((uint64_t)1 << b)) { all_fit = 0; break; }
    if (all_fit) return b;
    ++b;
  }
}

static size_t pad4(size_t v) { return (v + 3u) & ~(size_t)3u; }

#define ORC_D4 0u
#define ORC_DM 1u
#define ORC_D2 2u
#define ORC_D1 3u

/* The value each form subtracts from x_i (Sec. 5), 0 before the list. */
static uint32_t orc_reference(const uint32_t *x, uint64_t i, uint32_t mode) {
  switch (mode) {
    case ORC_D1: return i >= 1 ? x[i - 1] : 0u;
    case ORC_D2: return i >= 2 ? x[i - 2] : 0u;
    case ORC_DM: { uint64_t q = i / 4u; return q >= 1 ? x[4u * q - 1u] : 0u; }
    default: return i >= 4 ? x[i - 4] : 0u;
  }
}

/* Exact serialized size given the block widths (Sec. 4.2: 128 b bits, i.e.
 * 16 b bytes, per block). */
size_t orc_stream_bytes(uint64_t n, const uint8_t *widths) {
  uint64_t nb = n / 128u, t = n % 128u, pw = 0;
  for (uint64_t k = 0; k < nb; ++k) pw += 4u * widths[k];
  return ORC_HEADER + pad4((size_t)nb) + 4u * (size_t)pw + 4u * (size_t)t;
}

/* Pack 128 values of b bits into 4 b words at byte pointer payload: lane j
 * takes values 4q + j, q = 0..31, LSB first; its completed word m goes to
 * payload word 4m + j (Sec. 4.2, Fig. 2).  Bits above b are dropped. */
static void orc_pack_block(const uint32_t *d, uint32_t b, uint8_t *payload) {
  const uint64_t keep = (b == 32u) ? 0xFFFFFFFFull : (((uint64_t)1 << b) - 1u);
  for (uint32_t j = 0; j < 4; ++j) {
    uint64_t acc = 0;
    uint32_t have = 0, m = 0;
    for (uint32_t q = 0; q < 32; ++q) {
      acc |= ((uint64_t)d[4u * q + j] & keep) << have;
      have += b;
      while (have >= 32) {
        put32(payload + 4u * (4u * m + j), (uint32_t)acc);
        acc >>= 32; have -= 32; ++m;
      }
    }
  }
}

/* Encode a non-decreasing list: D4 deltas (Sec. 5), per-block width
 * (Sec. 4.3), 4-lane interleaved LSB-first packing (Sec. 4.2, Fig. 2). */
int orc_encode_mode(const uint32_t *x, uint64_t n, uint32_t mode, uint8_t *out, size_t cap,
                    size_t *out_bytes) {
  if ((!x && n) || !out_bytes || mode > 3u) return ORC_EINVAL;
  int strictly = 1;
  for (uint64_t i = 1; i < n; ++i) {
    if (x[i] < x[i - 1]) return ORC_EUNSORTED;
    if (x[i] == x[i - 1]) strictly = 0;
  }
  uint64_t nb = n / 128u, t = n % 128u;
  if (nb > 0xFFFFFFFFull) return ORC_EINVAL;
  uint64_t packed = nb * 128u;

  /* deltas over the global index, values before the list taken as 0 */
  uint32_t *d = (uint32_t *)malloc((packed ? packed : 1) * sizeof(uint32_t));
  uint8_t *w = (uint8_t *)malloc(nb ? nb : 1);
  if (!d || !w) { free(d); free(w); return ORC_ENOMEM; }
  for (uint64_t i = 0; i < packed; ++i) d[i] = x[i] - orc_reference(x, i, mode);
  uint64_t pw = 0;
  for (uint64_t k = 0; k < nb; ++k) { w[k] = (uint8_t)orc_width(d + 128u * k, 128u); pw += 4u * w[k]; }

  size_t need = ORC_HEADER + pad4((size_t)nb) + 4u * (size_t)pw + 4u * (size_t)t;
  *out_bytes = need;
  if (cap < need) { free(d); free(w); return ORC_ERANGE; }
  memset(out, 0, need);
  put32(out, ORC_MAGIC);
  put16(out + 4, 1);
  put16(out + 6, (uint16_t)((strictly ? 1u : 0u) | (mode << 1)));
  put64(out + 8, n);
  put32(out + 16, (uint32_t)nb);
  put32(out + 20, (uint32_t)t);
  put64(out + 24, pw);
  memcpy(out + ORC_HEADER, w, (size_t)nb);
  uint8_t *payload = out + ORC_HEADER + pad4((size_t)nb);

  uint64_t word_base = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    uint32_t b = w[k];
    for (uint32_t j = 0; j < 4; ++j) {
      /* lane j: append d[128k + 4q + j], q = 0..31, LSB first; emit each
       * completed 32-bit word m at payload word 4m + j */
      uint64_t acc = 0;
      uint32_t have = 0, m = 0;
      for (uint32_t q = 0; q < 32; ++q) {
        acc |= (uint64_t)d[128u * k + 4u * q + j] << have;
        have += b;
        while (have >= 32) {
          put32(payload + 4u * (word_base + 4u * m + j), (uint32_t)acc);
          acc >>= 32; have -= 32; ++m;
        }
      }
      /* 32 values of b bits fill exactly b words: nothing is left over */
    }
    word_base += 4u * b;
  }
  uint8_t *tail = payload + 4u * pw;
  for (uint64_t i = 0; i < t; ++i) put32(tail + 4u * i, x[packed + i]);
  free(d); free(w);
  return ORC_OK;
}

int orc_encode(const uint32_t *x, uint64_t n, uint8_t *out, size_t cap, size_t *out_bytes) {
  return orc_encode_mode(x, n, ORC_D4, out, cap, out_bytes);
}

/* FastPFOR's choice for one block of 128 deltas (Sec. 4.4): b is the
 * block's width (Sec. 4.3); the packed width b' in [0, b] minimises
 * 128 b' + c(b') (b - b' + 8), c(b') the number of deltas >= 2^b' (the
 * exceptions).  Reading: ties go to the larger b'.  Each candidate's count
 * is taken directly from the deltas. */
void orc_fp_choose(const uint32_t *d, uint32_t *b_out, uint32_t *bp_out, uint32_t *c_out) {
  const uint32_t b = orc_width(d, 128u);
  uint64_t best = 0;
  uint32_t best_bp = b, best_c = 0;
  for (uint32_t k = 0; k <= b; ++k) {
    const uint32_t bp = b - k; /* b, b - 1, ..., 0 */
    uint32_t c = 0;
    for (uint32_t i = 0; i < 128u; ++i)
      if ((uint64_t)d[i] >= ((uint64_t)1 << bp)) ++c;
    const uint64_t cost = 128u * (uint64_t)bp + (uint64_t)c * (b - bp + 8u);
    if (k == 0 || cost < best) { best = cost; best_bp = bp; best_c = c; }
  }
  *b_out = b;
  *bp_out = best_bp;
  *c_out = best_c;
}

/* Encode a non-decreasing list as S4-FastPFOR (Sec. 4.4) with the given
 * differential form (Sec. 5): per block, b' by orc_fp_choose; the low b'
 * bits of every delta packed as in S4-BP128 at width b'; the exceptions'
 * positions and high parts pooled per page of 512 blocks, one array per
 * value of b - b' (layout in the header comment). */
int orc_encode_fp(const uint32_t *x, uint64_t n, uint32_t mode, uint8_t *out, size_t cap, size_t *out_bytes) {
  if ((!x && n) || !out_bytes || mode > 3u) return ORC_EINVAL;
  int strictly = 1;
  for (uint64_t i = 1; i < n; ++i) {
    if (x[i] < x[i - 1]) return ORC_EUNSORTED;
    if (x[i] == x[i - 1]) strictly = 0;
  }
  const uint64_t nb = n / 128u, t = n % 128u, packed = nb * 128u;
  if (nb > 0xFFFFFFFFull) return ORC_EINVAL;
  uint32_t *d = (uint32_t *)malloc((packed ? packed : 1) * sizeof(uint32_t));
  uint8_t *bb = (uint8_t *)malloc(nb ? nb : 1), *bp = (uint8_t *)malloc(nb ? nb : 1);
  uint8_t *cc = (uint8_t *)malloc(nb ? nb : 1);
  if (!d || !bb || !bp || !cc) { free(d); free(bb); free(bp); free(cc); return ORC_ENOMEM; }
  for (uint64_t i = 0; i < packed; ++i) d[i] = x[i] - orc_reference(x, i, mode);
  uint64_t pw = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    uint32_t b, p, c;
    orc_fp_choose(d + 128u * k, &b, &p, &c);
    bb[k] = (uint8_t)b; bp[k] = (uint8_t)p; cc[k] = (uint8_t)c;
    pw += 4u * p;
  }
  /* size of the pages */
  size_t pages = 0;
  for (uint64_t k0 = 0; k0 < nb; k0 += ORC_PAGE) {
    const uint64_t k1 = (k0 + ORC_PAGE < nb) ? k0 + ORC_PAGE : nb;
    uint64_t meta = 0, cnt[33] = {0};
    for (uint64_t k = k0; k < k1; ++k) { meta += 2u + cc[k]; cnt[bb[k] - bp[k]] += cc[k]; }
    pages += 4u + pad4((size_t)meta) + 4u;
    for (uint32_t e = 1; e <= 32u; ++e)
      if (cnt[e]) pages += 4u + 4u * (size_t)e * ((cnt[e] + 31u) / 32u);
  }
  const size_t base = ORC_HEADER + pad4((size_t)nb) + 4u * (size_t)pw + 4u * (size_t)t;
  *out_bytes = base + pages;
  if (cap < base + pages) { free(d); free(bb); free(bp); free(cc); return ORC_ERANGE; }
  memset(out, 0, base + pages);
  put32(out, ORC_MAGIC);
  put16(out + 4, 1);
  put16(out + 6, (uint16_t)((strictly ? 1u : 0u) | (mode << 1) | ORC_PATCHED));
  put64(out + 8, n);
  put32(out + 16, (uint32_t)nb);
  put32(out + 20, (uint32_t)t);
  put64(out + 24, pw);
  memcpy(out + ORC_HEADER, bp, (size_t)nb);
  uint8_t *payload = out + ORC_HEADER + pad4((size_t)nb);
  uint64_t word_base = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    orc_pack_block(d + 128u * k, bp[k], payload + 4u * word_base);
    word_base += 4u * bp[k];
  }
  uint8_t *tail = payload + 4u * pw;
  for (uint64_t i = 0; i < t; ++i) put32(tail + 4u * i, x[packed + i]);
  uint8_t *q = out + base;
  for (uint64_t k0 = 0; k0 < nb; k0 += ORC_PAGE) {
    const uint64_t k1 = (k0 + ORC_PAGE < nb) ? k0 + ORC_PAGE : nb;
    uint8_t *m = q + 4;
    uint32_t o = 0, present = 0;
    for (uint64_t k = k0; k < k1; ++k) {
      m[o++] = bb[k];
      m[o++] = cc[k];
      for (uint32_t i = 0; i < 128u; ++i)
        if ((uint64_t)d[128u * k + i] >= ((uint64_t)1 << bp[k])) m[o++] = (uint8_t)i;
      if (cc[k]) present |= 1u << (bb[k] - bp[k] - 1u);
    }
    put32(q, o);
    q = m + pad4(o);
    put32(q, present);
    q += 4;
    for (uint32_t e = 1; e <= 32u; ++e) {
      if (!((present >> (e - 1u)) & 1u)) continue;
      uint8_t *cnt_at = q;
      uint8_t *words = q + 4;
      uint64_t idx = 0;
      for (uint64_t k = k0; k < k1; ++k) {
        if (!cc[k] || (uint32_t)(bb[k] - bp[k]) != e) continue;
        for (uint32_t i = 0; i < 128u; ++i) {
          const uint32_t v = d[128u * k + i];
          if ((uint64_t)v < ((uint64_t)1 << bp[k])) continue;
          const uint64_t high = (uint64_t)v >> bp[k];
          const uint64_t bit = idx++ * e;
          const uint64_t w = bit / 32u, s = bit % 32u;
          uint64_t cur = get32(words + 4u * w);
          if (s + e > 32u) cur |= (uint64_t)get32(words + 4u * (w + 1u)) << 32;
          cur |= high << s;
          put32(words + 4u * w, (uint32_t)cur);
          if (s + e > 32u) put32(words + 4u * (w + 1u), (uint32_t)(cur >> 32));
        }
      }
      put32(cnt_at, (uint32_t)idx);
      q = words + 4u * (size_t)e * ((idx + 31u) / 32u);
    }
  }
  free(d); free(bb); free(bp); free(cc);
  return ORC_OK;
}

typedef struct {
  uint64_t n, nb, t, pw;
  uint16_t flags;
  const uint8_t *widths;
  const uint8_t *payload; /* byte pointer, read with get32 */
  const uint8_t *tail;
  const uint8_t *pages;   /* patched streams: first page */
} orc_view;

/* Check the pages of a patched stream from p to end: every field in range,
 * c > 0 exactly when b' < b, positions increasing below 128, each array's
 * count equal to the exceptions that use it, nothing left over. */
static int orc_check_pages(const orc_view *v, const uint8_t *p, const uint8_t *end) {
  for (uint64_t k0 = 0; k0 < v->nb; k0 += ORC_PAGE) {
    const uint64_t k1 = (k0 + ORC_PAGE < v->nb) ? k0 + ORC_PAGE : v->nb;
    uint64_t cnt[33] = {0};
    if ((size_t)(end - p) < 4u) return ORC_ECORRUPT;
    const uint32_t meta_len = get32(p);
    const uint8_t *m = p + 4;
    if ((size_t)(end - m) < pad4(meta_len) + 4u) return ORC_ECORRUPT;
    uint32_t o = 0;
    for (uint64_t k = k0; k < k1; ++k) {
      if (o + 2u > meta_len) return ORC_ECORRUPT;
      const uint32_t b = m[o], c = m[o + 1], bp = v->widths[k];
      o += 2;
      if (b > 32u || bp > b || c > 128u || (c > 0) != (bp < b) || o + c > meta_len) return ORC_ECORRUPT;
      for (uint32_t e = 0; e < c; ++e)
        if (m[o + e] >= 128u || (e && m[o + e] <= m[o + e - 1])) return ORC_ECORRUPT;
      o += c;
      cnt[b - bp] += c;
    }
    if (o != meta_len) return ORC_ECORRUPT;
    for (uint32_t z = meta_len; z < pad4(meta_len); ++z)
      if (m[z]) return ORC_ECORRUPT;
    const uint8_t *q = m + pad4(meta_len);
    const uint32_t present = get32(q);
    q += 4;
    for (uint32_t d = 1; d <= 32u; ++d) {
      if (!((present >> (d - 1u)) & 1u)) {
        if (cnt[d]) return ORC_ECORRUPT;
        continue;
      }
      if ((size_t)(end - q) < 4u) return ORC_ECORRUPT;
      const uint32_t count = get32(q);
      const size_t words = (size_t)d * ((count + 31u) / 32u);
      if (count == 0 || count != cnt[d] || (size_t)(end - q) < 4u + 4u * words) return ORC_ECORRUPT;
      q += 4u + 4u * words;
    }
    p = q;
  }
  return p == end ? ORC_OK : ORC_ECORRUPT;
}

static int orc_parse(const uint8_t *enc, size_t bytes, orc_view *v) {
  if (!enc || bytes < ORC_HEADER) return ORC_ECORRUPT;
  if (get32(enc) != ORC_MAGIC || get16(enc + 4) != 1) return ORC_ECORRUPT;
  v->flags = get16(enc + 6);
  if (v->flags & ~15u) return ORC_ECORRUPT;
  v->n = get64(enc + 8);
  v->nb = get32(enc + 16);
  v->t = get32(enc + 20);
  v->pw = get64(enc + 24);
  if (v->t >= 128 || v->nb * 128u + v->t != v->n) return ORC_ECORRUPT;
  size_t wbytes = pad4((size_t)v->nb);
  if (bytes < ORC_HEADER + wbytes) return ORC_ECORRUPT;
  v->widths = enc + ORC_HEADER;
  uint64_t pw = 0;
  for (uint64_t k = 0; k < v->nb; ++k) {
    if (v->widths[k] > 32) return ORC_ECORRUPT;
    pw += 4u * v->widths[k];
  }
  for (uint64_t k = v->nb; k < wbytes; ++k)
    if (enc[ORC_HEADER + k] != 0) return ORC_ECORRUPT;
  if (pw != v->pw) return ORC_ECORRUPT;
  const size_t base = ORC_HEADER + wbytes + 4u * pw + 4u * v->t;
  v->payload = enc + ORC_HEADER + wbytes;
  v->tail = v->payload + 4u * pw;
  v->pages = enc + base;
  if (!(v->flags & ORC_PATCHED)) return bytes == base ? ORC_OK : ORC_ECORRUPT;
  if (bytes < base) return ORC_ECORRUPT;
  return orc_check_pages(v, enc + base, enc + bytes);
}

int orc_decoded_length(const uint8_t *enc, size_t bytes, uint64_t *n) {
  orc_view v;
  int rc = orc_parse(enc, bytes, &v);
  if (rc) return rc;
  *n = v.n;
  return ORC_OK;
}

/* Widths of the blocks, for tests of the per-block size formula. */
int orc_widths(const uint8_t *enc, size_t bytes, uint8_t *out, uint64_t cap, uint64_t *nb) {
  orc_view v;
  int rc = orc_parse(enc, bytes, &v);
  if (rc) return rc;
  *nb = v.nb;
  if (cap < v.nb) return ORC_ERANGE;
  memcpy(out, v.widths, (size_t)v.nb);
  return ORC_OK;
}

/* Random-access extraction of delta p (0..127) of a block whose 4b payload
 * words start at byte pointer w: lane j = p mod 4, position q = p div 4,
 * bits [qb, qb+b) of lane j's stream.  The 64-bit window holds lane words
 * m and m+1 (payload words 4m+j and 4m+4+j). */
static uint32_t orc_extract(const uint8_t *w, uint32_t b, uint32_t p) {
  if (b == 0) return 0;
  uint32_t j = p % 4u, q = p / 4u;
  uint32_t bit = q * b, m = bit / 32u, s = bit % 32u;
  uint64_t window = get32(w + 4u * (4u * m + j));
  if (s + b > 32u) window |= (uint64_t)get32(w + 4u * (4u * (m + 1u) + j)) << 32;
  uint64_t mask = (b == 32u) ? 0xFFFFFFFFull : (((uint64_t)1 << b) - 1u);
  return (uint32_t)((window >> s) & mask);
}

/* Patching (Sec. 4.4), by random access: for each page, locate array d of
 * every present d; block k's e-th exception, the j-th of its page to use
 * array d = b - b', has high part bits [j d, j d + d) of that array, added
 * above the b' low bits already unpacked at its position. */
static void orc_patch_random(const orc_view *v, uint32_t *out) {
  const uint8_t *p = v->pages;
  for (uint64_t k0 = 0; k0 < v->nb; k0 += ORC_PAGE) {
    const uint64_t k1 = (k0 + ORC_PAGE < v->nb) ? k0 + ORC_PAGE : v->nb;
    const uint32_t meta_len = get32(p);
    const uint8_t *m = p + 4;
    const uint8_t *q = m + pad4(meta_len);
    const uint32_t present = get32(q);
    q += 4;
    const uint8_t *arr[33] = {0};
    for (uint32_t d = 1; d <= 32u; ++d) {
      if (!((present >> (d - 1u)) & 1u)) continue;
      const uint32_t count = get32(q);
      arr[d] = q + 4;
      q += 4u + 4u * (size_t)d * ((count + 31u) / 32u);
    }
    uint64_t used[33] = {0};
    uint32_t o = 0;
    for (uint64_t k = k0; k < k1; ++k) {
      const uint32_t b = m[o], c = m[o + 1], bp = v->widths[k], d = b - bp;
      o += 2;
      for (uint32_t e = 0; e < c; ++e) {
        const uint64_t bit = used[d]++ * d;
        const uint64_t w = bit / 32u, s = bit % 32u;
        uint64_t window = get32(arr[d] + 4u * w);
        if (s + d > 32u) window |= (uint64_t)get32(arr[d] + 4u * (w + 1u)) << 32;
        const uint64_t mask = (d == 32u) ? 0xFFFFFFFFull : (((uint64_t)1 << d) - 1u);
        const uint32_t high = (uint32_t)((window >> s) & mask);
        out[128u * k + m[o + e]] += (uint32_t)((uint64_t)high << bp);
      }
      o += c;
    }
    p = q;
  }
}

/* Decode: unpack every delta by random access, then invert the stream's
 * differential form over the whole list in index order, x_i = delta_i +
 * (the value the form subtracted) (Sec. 5), then copy the raw tail. */
int orc_decode(const uint8_t *enc, size_t bytes, uint32_t *out, uint64_t cap, uint64_t *n_out) {
  orc_view v;
  int rc = orc_parse(enc, bytes, &v);
  if (rc) return rc;
  if (n_out) *n_out = v.n;
  if (cap < v.n) return ORC_ERANGE;
  uint64_t word_base = 0;
  for (uint64_t k = 0; k < v.nb; ++k) {
    uint32_t b = v.widths[k];
    for (uint32_t p = 0; p < 128u; ++p)
      out[128u * k + p] = orc_extract(v.payload + 4u * word_base, b, p);
    word_base += 4u * b;
  }
  if (v.flags & ORC_PATCHED) orc_patch_random(&v, out);
  const uint32_t mode = (v.flags >> 1) & 3u;
  for (uint64_t i = 0; i < 128u * v.nb; ++i) out[i] += orc_reference(out, i, mode);
  for (uint64_t i = 0; i < v.t; ++i) out[128u * v.nb + i] = get32(v.tail + 4u * i);
  return ORC_OK;
}

/* The vector prefix function P(t, v) of each differential form, for a
 * 4-vector t of deltas and the previous decoded 4-vector v, following the
 * SIMD steps Sec. 5 lists (shifts by whole integers, broadcasts, adds). */
static void orc_prefix(uint32_t mode, uint32_t t[4], const uint32_t v[4]) {
  uint32_t u[4];
  switch (mode) {
    case ORC_DM: /* broadcast v's last integer, add */
      for (int c = 0; c < 4; ++c) t[c] += v[3];
      break;
    case ORC_D2: /* t + (t shifted by two integers), then + (v3, v4, v3, v4) */
      u[0] = t[0]; u[1] = t[1]; u[2] = t[2] + t[0]; u[3] = t[3] + t[1];
      t[0] = u[0] + v[2]; t[1] = u[1] + v[3]; t[2] = u[2] + v[2]; t[3] = u[3] + v[3];
      break;
    case ORC_D1: /* the D2 steps, then + (shifted by one integer), then + v's last */
      u[0] = t[0]; u[1] = t[1]; u[2] = t[2] + t[0]; u[3] = t[3] + t[1];
      t[0] = u[0]; t[1] = u[1] + u[0]; t[2] = u[2] + u[1]; t[3] = u[3] + u[2];
      for (int c = 0; c < 4; ++c) t[c] += v[3];
      break;
    case 4u: /* no differential coding: P(t, v) = t */
      break;
    default: /* D4: t + v */
      for (int c = 0; c < 4; ++c) t[c] += v[c];
      break;
  }
}

/* Second, structurally different decoder that follows the steps of the
 * paper's block unpacking procedure (Alg. 1): walk the b input vectors
 * (four lanes each) with a running bit offset i; while a whole value fits
 * in the current vector, shift it out and mask; otherwise complete it with
 * the low bits of the next vector shifted left by 32-i; after each
 * 4-vector apply the form's prefix P(t,v) and make the result the new v. */
static void orc_alg1_block(const uint8_t *y, uint32_t b, uint32_t mode, uint32_t v[4], uint32_t *w) {
  uint32_t M = (b == 32u) ? 0xFFFFFFFFu : ((1u << b) - 1u);
  uint32_t produced = 0;
  uint32_t t[4];
  if (b == 0) {
    /* no input vectors: 128 zero deltas */
    for (uint32_t r = 0; r < 32u; ++r) {
      t[0] = t[1] = t[2] = t[3] = 0;
      orc_prefix(mode, t, v);
      for (uint32_t c = 0; c < 4u; ++c) { v[c] = t[c]; w[4u * r + c] = t[c]; }
    }
    return;
  }
  uint32_t i = 0;
  for (uint32_t k = 0; k < b; ++k) {
    while (i + b <= 32u) {
      for (uint32_t c = 0; c < 4u; ++c) t[c] = (get32(y + 4u * (4u * k + c)) >> i) & M;
      orc_prefix(mode, t, v);
      for (uint32_t c = 0; c < 4u; ++c) { v[c] = t[c]; w[4u * produced + c] = t[c]; }
      ++produced;
      i += b;
    }
    if (i < 32u) {
      for (uint32_t c = 0; c < 4u; ++c) {
        uint32_t z = (get32(y + 4u * (4u * (k + 1u) + c)) << (32u - i)) & M;
        t[c] = (get32(y + 4u * (4u * k + c)) >> i) | z;
      }
      orc_prefix(mode, t, v);
      for (uint32_t c = 0; c < 4u; ++c) { v[c] = t[c]; w[4u * produced + c] = t[c]; }
      ++produced;
      i = i + b - 32u;
    } else {
      i = 0;
    }
  }
}

/* Sequential reader of one exception array: LSB-first, d bits at a time. */
typedef struct { const uint8_t *w; uint64_t acc; uint32_t have; } orc_bits;
static uint32_t orc_bits_take(orc_bits *r, uint32_t d) {
  while (r->have < d) {
    r->acc |= (uint64_t)get32(r->w) << r->have;
    r->w += 4;
    r->have += 32;
  }
  const uint32_t v = (uint32_t)(r->acc & ((d == 32u) ? 0xFFFFFFFFull : (((uint64_t)1 << d) - 1u)));
  r->acc = (d == 64u) ? 0 : (r->acc >> d);
  r->have -= d;
  return v;
}

/* S4-FastPFOR in the paper's three passes (Sec. 5: unpack, patch, prefix
 * could not be fused): every block of a page is unpacked in the order of
 * Alg. 1 with no prefix; the page's exceptions are then applied in stream
 * order, each array read sequentially; last the form's P(t, v) runs over
 * the page's 4-vectors, v carried from block to block. */
static void orc_three_pass(const orc_view *v, uint32_t *out) {
  const uint32_t mode = (v->flags >> 1) & 3u;
  uint32_t seed[4] = {0, 0, 0, 0}, dummy[4];
  const uint8_t *p = v->pages;
  uint64_t word_base = 0;
  for (uint64_t k0 = 0; k0 < v->nb; k0 += ORC_PAGE) {
    const uint64_t k1 = (k0 + ORC_PAGE < v->nb) ? k0 + ORC_PAGE : v->nb;
    for (uint64_t k = k0; k < k1; ++k) {
      orc_alg1_block(v->payload + 4u * word_base, v->widths[k], 4u, dummy, out + 128u * k);
      word_base += 4u * v->widths[k];
    }
    const uint32_t meta_len = get32(p);
    const uint8_t *m = p + 4, *q = p + 4 + pad4(meta_len);
    const uint32_t present = get32(q);
    q += 4;
    orc_bits rd[33];
    memset(rd, 0, sizeof rd);
    for (uint32_t d = 1; d <= 32u; ++d) {
      if (!((present >> (d - 1u)) & 1u)) continue;
      const uint32_t count = get32(q);
      rd[d].w = q + 4;
      q += 4u + 4u * (size_t)d * ((count + 31u) / 32u);
    }
    const uint8_t *mp = m;
    for (uint64_t k = k0; k < k1; ++k) {
      const uint32_t b = mp[0], c = mp[1], bp = v->widths[k];
      for (uint32_t e = 0; e < c; ++e) {
        const uint32_t high = orc_bits_take(&rd[b - bp], b - bp);
        out[128u * k + mp[2 + e]] |= (uint32_t)((uint64_t)high << bp);
      }
      mp += 2u + c;
    }
    for (uint64_t k = k0; k < k1; ++k)
      for (uint32_t r = 0; r < 32u; ++r) {
        uint32_t t[4];
        for (uint32_t c = 0; c < 4u; ++c) t[c] = out[128u * k + 4u * r + c];
        orc_prefix(mode, t, seed);
        for (uint32_t c = 0; c < 4u; ++c) { seed[c] = t[c]; out[128u * k + 4u * r + c] = t[c]; }
      }
    p = q;
  }
}

int orc_decode_alg1(const uint8_t *enc, size_t bytes, uint32_t *out, uint64_t cap, uint64_t *n_out) {
  orc_view v;
  int rc = orc_parse(enc, bytes, &v);
  if (rc) return rc;
  if (n_out) *n_out = v.n;
  if (cap < v.n) return ORC_ERANGE;
  if (v.flags & ORC_PATCHED) {
    orc_three_pass(&v, out);
    for (uint64_t i = 0; i < v.t; ++i) out[128u * v.nb + i] = get32(v.tail + 4u * i);
    return ORC_OK;
  }
  uint32_t seed[4] = {0, 0, 0, 0};
  uint64_t word_base = 0;
  for (uint64_t k = 0; k < v.nb; ++k) {
    uint32_t b = v.widths[k];
    orc_alg1_block(v.payload + 4u * word_base, b, (v.flags >> 1) & 3u, seed, out + 128u * k);
    word_base += 4u * b;
  }
  for (uint64_t i = 0; i < v.t; ++i) out[128u * v.nb + i] = get32(v.tail + 4u * i);
  return ORC_OK;
}

/* Textbook two-pointer merge intersection (scalar baseline, Sec. 6): advance the
 * pointer at the smaller value; on equality emit once and advance both.
 * Inputs must be strictly increasing.  Safe when out aliases the shorter
 * input (the output-to-input property, Sec. 6.2). */
int orc_intersect(const uint32_t *a, uint64_t m, const uint32_t *b, uint64_t n, uint32_t *out,
                  uint64_t *count) {
  if (!count) return ORC_EINVAL;
  for (uint64_t i = 1; i < m; ++i) if (a[i] <= a[i - 1]) return ORC_EUNSORTED;
  for (uint64_t i = 1; i < n; ++i) if (b[i] <= b[i - 1]) return ORC_EUNSORTED;
  uint64_t i = 0, j = 0, c = 0;
  while (i < m && j < n) {
    if (a[i] < b[j]) ++i;
    else if (b[j] < a[i]) ++j;
    else { out[c++] = a[i]; ++i; ++j; }
  }
  *count = c;
  return ORC_OK;
}

/* k-way intersection as a left fold of the pairwise merge in the order
 * given (the result is a set, so any order gives the same answer; SvS
 * order is an optimisation only, Sec. 6).  k = 1 copies the list. */
int orc_intersect_k(const uint32_t *const *lists, const uint64_t *lens, uint32_t k, uint32_t *out,
                    uint64_t cap, uint64_t *count) {
  if (!count || k == 0) return ORC_EINVAL;
  for (uint32_t l = 0; l < k; ++l)
    for (uint64_t i = 1; i < lens[l]; ++i)
      if (lists[l][i] <= lists[l][i - 1]) return ORC_EUNSORTED;
  uint64_t cur = lens[0];
  if (cap < cur) {
    /* the result is never longer than the first list; require room for it */
    return ORC_ERANGE;
  }
  memcpy(out, lists[0], (size_t)cur * sizeof(uint32_t));
  for (uint32_t l = 1; l < k; ++l) {
    uint64_t c = 0;
    int rc = orc_intersect(out, cur, lists[l], lens[l], out, &c);
    if (rc) return rc;
    cur = c;
  }
  *count = cur;
  return ORC_OK;
}

/* hyb+m2 (Sec. 7.7, the bitmap-list hybrid of Culpepper and Moffat): a
 * list of n > 0 values over the universe [0, U) is kept as a bitmap of U
 * bits when its average gap U / n is at most B, that is when n * B >= U;
 * B = 0 means no bitmaps.  Reading: the average gap of a list is the
 * universe size over its length. */
int orc_hyb_is_bitmap(uint64_t n, uint64_t universe, uint32_t B) {
  if (B == 0 || n == 0) return 0;
  /* n * B >= U  <=>  n >= ceil(U / B), without overflow */
  return n >= (universe + B - 1u) / B;
}

/* A conjunctive query under hyb+m2 (Sec. 7.7): the lists that stay
 * compressed are intersected two at a time starting from the shortest
 * (SvS with the two-pointer merge), then every surviving value is looked
 * up in each bitmap in turn and kept only if its bit is set.  When every
 * list is a bitmap (the paper does not treat this case) the bitmaps are
 * ANDed word by word and the set bits are read out in increasing order.
 * Inputs must be strictly increasing; values of bitmap lists must be
 * below the universe (ORC_EINVAL); a compressed value >= U has no bit and
 * is dropped by any bitmap.  Result capacity: the shortest list's length
 * (ORC_ERANGE otherwise). */
int orc_hyb_intersect_k(const uint32_t *const *lists, const uint64_t *lens, uint32_t k, uint64_t universe,
                        uint32_t B, uint32_t *out, uint64_t cap, uint64_t *count) {
  if (!count || k == 0 || k > 64) return ORC_EINVAL;
  const uint64_t words = (universe + 31u) / 32u;
  uint32_t comp[64], bm[64];
  uint32_t nc = 0, nbm = 0;
  uint64_t shortest = lens[0];
  for (uint32_t l = 0; l < k; ++l) {
    for (uint64_t i = 1; i < lens[l]; ++i)
      if (lists[l][i] <= lists[l][i - 1]) return ORC_EUNSORTED;
    if (lens[l] < shortest) shortest = lens[l];
    if (orc_hyb_is_bitmap(lens[l], universe, B)) {
      if (lists[l][lens[l] - 1] >= universe) return ORC_EINVAL;
      bm[nbm++] = l;
    } else {
      comp[nc++] = l;
    }
  }
  if (cap < shortest) return ORC_ERANGE;
  /* the bitmaps: bit x of list l is bit (x mod 32) of word floor(x / 32) */
  uint32_t **bits = NULL;
  if (nbm) {
    bits = (uint32_t **)calloc(nbm, sizeof(uint32_t *));
    if (!bits) return ORC_ENOMEM;
    for (uint32_t j = 0; j < nbm; ++j) {
      bits[j] = (uint32_t *)calloc(words ? words : 1u, sizeof(uint32_t));
      if (!bits[j]) {
        for (uint32_t i = 0; i < j; ++i) free(bits[i]);
        free(bits);
        return ORC_ENOMEM;
      }
      const uint32_t *x = lists[bm[j]];
      for (uint64_t i = 0; i < lens[bm[j]]; ++i) bits[j][x[i] / 32u] |= 1u << (x[i] % 32u);
    }
  }
  uint64_t cur = 0;
  if (nc) {
    /* compressed lists by length (stable insertion sort), then SvS */
    for (uint32_t i = 1; i < nc; ++i)
      for (uint32_t j = i; j > 0 && lens[comp[j - 1]] > lens[comp[j]]; --j) {
        const uint32_t t = comp[j];
        comp[j] = comp[j - 1];
        comp[j - 1] = t;
      }
    cur = lens[comp[0]];
    memcpy(out, lists[comp[0]], (size_t)cur * sizeof(uint32_t));
    for (uint32_t i = 1; i < nc; ++i) {
      uint64_t c = 0;
      orc_intersect(out, cur, lists[comp[i]], lens[comp[i]], out, &c);
      cur = c;
    }
    /* then the bitmaps, one by one */
    for (uint32_t j = 0; j < nbm; ++j) {
      uint64_t c = 0;
      for (uint64_t i = 0; i < cur; ++i) {
        const uint32_t x = out[i];
        if (x < universe && ((bits[j][x / 32u] >> (x % 32u)) & 1u)) out[c++] = x;
      }
      cur = c;
    }
  } else {
    for (uint64_t w = 0; w < words; ++w) {
      uint32_t a = bits[0][w];
      for (uint32_t j = 1; j < nbm; ++j) a &= bits[j][w];
      for (uint32_t b = 0; b < 32u; ++b)
        if ((a >> b) & 1u) {
          if (cur == cap) { /* more results than the shortest list: impossible */
            for (uint32_t j = 0; j < nbm; ++j) free(bits[j]);
            free(bits);
            return ORC_ERANGE;
          }
          out[cur++] = (uint32_t)(32u * w + b);
        }
    }
  }
  for (uint32_t j = 0; j < nbm; ++j) free(bits[j]);
  free(bits);
  *count = cur;
  return ORC_OK;
}

// Host side of the codec: the S4-BP128 encoder in every differential form
// (Sec. 4.2-4.3, Sec. 5) and its patched variant S4-FastPFOR (Sec. 4.4),
// stream validation, and error reporting for the C ABI.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "s4_internal.h"

namespace s4 {

static thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return S4_EDEVICE;
}

static inline size_t round4(size_t v) { return (v + 3) & ~size_t(3); }

// A patched block's packed bits plus exception bits never exceed 128 b - 8 c
// (its cost is at most plain packing's), so it fits plain packing's 512
// bytes plus 2 metadata bytes; each page adds at most its two counts, 3
// pad bytes, 32 array counts and 31 padding values in each of 32 arrays.
size_t stream_bound(uint64_t n) {
  uint64_t nb = n / kBlock, t = n % kBlock;
  const uint64_t pages = (nb + kPage - 1) / kPage;
  return kHeaderBytes + round4(nb) + size_t(nb) * 514u + 4u * size_t(t) + size_t(pages) * (11u + 32u * (4u + 124u));
}

static inline void wr32(uint8_t *p, uint32_t v) { std::memcpy(p, &v, 4); }
static inline uint32_t rd32(const uint8_t *p) {
  uint32_t v;
  std::memcpy(&v, p, 4);
  return v;
}

// Pack the 128 D4 deltas of one block at width b: lane j = p mod 4 takes
// deltas p = 4q + j in order q = 0..31; its stream is LSB-first and its
// m-th word lands at word 4m + j of the block (Fig. 2).
static void pack_block(const uint32_t *d, uint32_t b, uint32_t *words) {
  if (b == 0) return;
  for (uint32_t j = 0; j < 4; ++j) {
    uint64_t acc = 0;
    uint32_t fill = 0, m = 0;
    for (uint32_t q = 0; q < 32; ++q) {
      acc |= uint64_t(d[4 * q + j]) << fill;
      fill += b;
      if (fill >= 32) {
        words[4 * m + j] = uint32_t(acc);
        ++m;
        acc >>= 32;
        fill -= 32;
      }
    }
  }
}

// The value a differential form subtracts from x_i (Sec. 5); values before
// the list are 0.
static inline uint32_t reference(const uint32_t *in, uint64_t i, uint32_t delta) {
  switch (delta) {
    case S4_DELTA_D1: return i >= 1 ? in[i - 1] : 0u;
    case S4_DELTA_D2: return i >= 2 ? in[i - 2] : 0u;
    case S4_DELTA_DM: return i >= 4 ? in[(i & ~uint64_t(3)) - 1] : 0u;
    default: return i >= 4 ? in[i - 4] : 0u;
  }
}

static inline uint32_t bit_length(uint32_t v) { return v ? 32u - uint32_t(__builtin_clz(v)) : 0u; }

// S4-FastPFOR's block choice (Sec. 4.4): with c(b') the number of deltas
// longer than b' bits (from a histogram of bit lengths), b' minimises
// 128 b' + c(b') (b - b' + 8); scanning b' downward from b with a strict
// comparison keeps the larger b' on ties.
static void fp_choose(const uint32_t *d, uint32_t &b, uint32_t &bp, uint32_t &c) {
  uint32_t hist[33] = {0};
  b = 0;
  for (uint32_t p = 0; p < kBlock; ++p) {
    const uint32_t l = bit_length(d[p]);
    ++hist[l];
    b = std::max(b, l);
  }
  uint64_t best = 128ull * b;
  bp = b;
  c = 0;
  uint32_t above = 0;
  for (int cand = int(b) - 1; cand >= 0; --cand) {
    above += hist[cand + 1];
    const uint64_t cost = 128ull * uint32_t(cand) + uint64_t(above) * (b - uint32_t(cand) + 8u);
    if (cost < best) {
      best = cost;
      bp = uint32_t(cand);
      c = above;
    }
  }
}

// Patched stream (layout in s4.h): blocks packed at b', then the pages'
// metadata and exception arrays.
static int encode_patched(const uint32_t *in, uint64_t n, uint32_t delta, bool strictly, uint8_t *out, size_t cap,
                          size_t *out_bytes) {
  const uint64_t nb = n / kBlock, t = n % kBlock;
  std::vector<uint32_t> d(size_t(nb) * kBlock);
  for (uint64_t i = 0; i < nb * kBlock; ++i) d[i] = in[i] - reference(in, i, delta);
  std::vector<uint8_t> bw(nb), bpw(nb), cnt(nb);
  uint64_t pw = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    uint32_t b, bp, c;
    fp_choose(&d[k * kBlock], b, bp, c);
    bw[k] = uint8_t(b);
    bpw[k] = uint8_t(bp);
    cnt[k] = uint8_t(c);
    pw += 4u * bp;
  }
  // page sizes
  uint64_t pages_bytes = 0;
  for (uint64_t k0 = 0; k0 < nb; k0 += kPage) {
    const uint64_t k1 = std::min<uint64_t>(nb, k0 + kPage);
    uint64_t meta = 0, per_d[33] = {0};
    for (uint64_t k = k0; k < k1; ++k) {
      meta += 2u + cnt[k];
      per_d[bw[k] - bpw[k]] += cnt[k];
    }
    pages_bytes += 4u + round4(meta) + 4u;
    for (uint32_t e = 1; e <= 32; ++e)
      if (per_d[e]) pages_bytes += 4u + 4u * uint64_t(e) * ((per_d[e] + 31u) / 32u);
  }
  const size_t base = kHeaderBytes + round4(nb) + 4u * size_t(pw) + 4u * size_t(t);
  const size_t need = base + size_t(pages_bytes);
  *out_bytes = need;
  if (!out || cap < need) return fail(S4_ERANGE, "s4_encode: output buffer too small");
  std::memset(out, 0, need);
  wr32(out, kMagic);
  uint16_t ver = kVersion, fl = uint16_t((strictly ? 1u : 0u) | (delta << 1) | kFlagPatched);
  std::memcpy(out + 4, &ver, 2);
  std::memcpy(out + 6, &fl, 2);
  std::memcpy(out + 8, &n, 8);
  uint32_t nb32 = uint32_t(nb), t32 = uint32_t(t);
  std::memcpy(out + 16, &nb32, 4);
  std::memcpy(out + 20, &t32, 4);
  std::memcpy(out + 24, &pw, 8);
  if (nb) std::memcpy(out + kHeaderBytes, bpw.data(), nb);
  uint8_t *payload = out + kHeaderBytes + round4(nb);
  uint32_t low[kBlock], words[4 * 32];
  size_t wpos = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    const uint32_t bp = bpw[k];
    const uint32_t keep = bp >= 32 ? 0xFFFFFFFFu : ((1u << bp) - 1u);
    for (uint32_t p = 0; p < kBlock; ++p) low[p] = d[k * kBlock + p] & keep;
    pack_block(low, bp, words);
    std::memcpy(payload + 4 * wpos, words, 16u * bp);
    wpos += 4u * bp;
  }
  if (t) std::memcpy(payload + 4 * pw, in + nb * kBlock, 4u * size_t(t));
  uint8_t *q = out + base;
  for (uint64_t k0 = 0; k0 < nb; k0 += kPage) {
    const uint64_t k1 = std::min<uint64_t>(nb, k0 + kPage);
    uint8_t *meta = q + 4;
    uint32_t o = 0, present = 0;
    for (uint64_t k = k0; k < k1; ++k) {
      meta[o++] = bw[k];
      meta[o++] = cnt[k];
      if (!cnt[k]) continue;
      present |= 1u << (bw[k] - bpw[k] - 1u);
      for (uint32_t p = 0; p < kBlock; ++p)
        if (bit_length(d[k * kBlock + p]) > bpw[k]) meta[o++] = uint8_t(p);
    }
    wr32(q, o);
    q = meta + round4(o);
    wr32(q, present);
    q += 4;
    for (uint32_t e = 1; e <= 32; ++e) {
      if (!((present >> (e - 1)) & 1u)) continue;
      uint8_t *count_at = q;
      uint8_t *arr = q + 4;
      uint64_t idx = 0;
      for (uint64_t k = k0; k < k1; ++k) {
        if (!cnt[k] || uint32_t(bw[k] - bpw[k]) != e) continue;
        for (uint32_t p = 0; p < kBlock; ++p) {
          const uint32_t v = d[k * kBlock + p];
          if (bit_length(v) <= bpw[k]) continue;
          const uint64_t high = uint64_t(v) >> bpw[k];
          const uint64_t bit = idx++ * e, w = bit >> 5, sh = bit & 31;
          uint64_t cur = rd32(arr + 4 * w);
          if (sh + e > 32) cur |= uint64_t(rd32(arr + 4 * (w + 1))) << 32;
          cur |= high << sh;
          wr32(arr + 4 * w, uint32_t(cur));
          if (sh + e > 32) wr32(arr + 4 * (w + 1), uint32_t(cur >> 32));
        }
      }
      wr32(count_at, uint32_t(idx));
      q = arr + 4u * size_t(e) * ((idx + 31u) / 32u);
    }
  }
  return S4_OK;
}

int encode_one(const uint32_t *in, uint64_t n, uint32_t delta, uint8_t *out, size_t cap, size_t *out_bytes) {
  if ((!in && n) || !out_bytes) return fail(S4_EINVAL, "s4_encode: null argument");
  const bool patched = (delta & S4_CODEC_FASTPFOR) != 0;
  delta &= ~S4_CODEC_FASTPFOR;
  if (delta > S4_DELTA_D1) return fail(S4_EINVAL, "s4_encode: unknown differential form");
  if (n / kBlock > 0xFFFFFFFFull) return fail(S4_EINVAL, "s4_encode: list too long");
  bool strictly = true;
  for (uint64_t i = 1; i < n; ++i) {
    if (in[i] < in[i - 1]) return fail(S4_EUNSORTED, "s4_encode: input decreases at index " + std::to_string(i));
    strictly &= in[i] != in[i - 1];
  }
  if (patched) return encode_patched(in, n, delta, strictly, out, cap, out_bytes);
  const uint64_t nb = n / kBlock, t = n % kBlock;
  // widths first (the stream stores them ahead of the payload)
  std::vector<uint8_t> widths(nb);
  uint64_t pw = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    const uint32_t *x = in + k * kBlock;
    uint32_t any = 0;
    for (uint32_t p = 0; p < kBlock; ++p) any |= x[p] - reference(in, k * kBlock + p, delta);
    uint32_t b = any ? 32u - uint32_t(__builtin_clz(any)) : 0u;
    widths[k] = uint8_t(b);
    pw += 4u * b;
  }
  const size_t need = kHeaderBytes + round4(nb) + 4u * size_t(pw) + 4u * size_t(t);
  *out_bytes = need;
  if (!out || cap < need) return fail(S4_ERANGE, "s4_encode: output buffer too small");
  std::memset(out, 0, kHeaderBytes + round4(nb));
  wr32(out, kMagic);
  uint16_t ver = kVersion, fl = uint16_t((strictly ? 1u : 0u) | (delta << 1));
  std::memcpy(out + 4, &ver, 2);
  std::memcpy(out + 6, &fl, 2);
  std::memcpy(out + 8, &n, 8);
  uint32_t nb32 = uint32_t(nb), t32 = uint32_t(t);
  std::memcpy(out + 16, &nb32, 4);
  std::memcpy(out + 20, &t32, 4);
  std::memcpy(out + 24, &pw, 8);
  if (nb) std::memcpy(out + kHeaderBytes, widths.data(), nb);
  uint8_t *payload = out + kHeaderBytes + round4(nb);
  uint32_t d[kBlock];
  uint32_t words[4 * 32];
  size_t wpos = 0;
  for (uint64_t k = 0; k < nb; ++k) {
    for (uint32_t p = 0; p < kBlock; ++p) d[p] = in[k * kBlock + p] - reference(in, k * kBlock + p, delta);
    const uint32_t b = widths[k];
    pack_block(d, b, words);
    std::memcpy(payload + 4 * wpos, words, 16u * b);
    wpos += 4u * b;
  }
  if (t) std::memcpy(payload + 4 * pw, in + nb * kBlock, 4u * size_t(t));
  return S4_OK;
}

// Walk the pages of a patched stream: every field in range, c > 0 exactly
// when b' < b, positions increasing below 128, each array's count equal to
// the exceptions that use it, nothing left over.  Also totals what the
// device copy needs.
static int check_pages(StreamView *v, const uint8_t *p, const uint8_t *end) {
  for (uint64_t k0 = 0; k0 < v->nb; k0 += kPage) {
    const uint64_t k1 = std::min<uint64_t>(v->nb, k0 + kPage);
    uint64_t per_d[33] = {0};
    if (size_t(end - p) < 4) return fail(S4_ECORRUPT, "patched stream truncated in a page");
    const uint32_t meta_len = rd32(p);
    const uint8_t *m = p + 4;
    if (size_t(end - m) < round4(meta_len) + 4u) return fail(S4_ECORRUPT, "page metadata truncated");
    uint64_t o = 0;
    for (uint64_t k = k0; k < k1; ++k) {
      if (o + 2 > meta_len) return fail(S4_ECORRUPT, "page metadata too short");
      const uint32_t b = m[o], c = m[o + 1], bp = v->widths[k];
      o += 2;
      if (b > 32 || bp > b || c > kBlock || (c > 0) != (bp < b) || o + c > meta_len)
        return fail(S4_ECORRUPT, "bad block metadata in block " + std::to_string(k));
      for (uint32_t e = 0; e < c; ++e)
        if (m[o + e] >= kBlock || (e && m[o + e] <= m[o + e - 1]))
          return fail(S4_ECORRUPT, "exception positions not increasing in block " + std::to_string(k));
      o += c;
      per_d[b - bp] += c;
      v->x_positions += c;
    }
    if (o != meta_len) return fail(S4_ECORRUPT, "page metadata length disagrees");
    for (uint64_t z = meta_len; z < round4(meta_len); ++z)
      if (m[z]) return fail(S4_ECORRUPT, "nonzero metadata padding");
    const uint8_t *q = m + round4(meta_len);
    const uint32_t present = rd32(q);
    q += 4;
    for (uint32_t d = 1; d <= 32; ++d) {
      if (!((present >> (d - 1)) & 1u)) {
        if (per_d[d]) return fail(S4_ECORRUPT, "exceptions without their array");
        continue;
      }
      if (size_t(end - q) < 4) return fail(S4_ECORRUPT, "page arrays truncated");
      const uint32_t count = rd32(q);
      const uint64_t words = uint64_t(d) * ((count + 31u) / 32u);
      if (count == 0 || count != per_d[d] || uint64_t(end - q) < 4u + 4u * words)
        return fail(S4_ECORRUPT, "exception array size disagrees with the metadata");
      q += 4u + 4u * words;
      v->x_array_words += words + 1;  // one pad word: two-word reads stay inside
    }
    p = q;
  }
  if (p != end) return fail(S4_ECORRUPT, "bytes after the last page");
  return S4_OK;
}

int parse_stream(const uint8_t *enc, size_t bytes, StreamView *v) {
  if (!enc || !v) return fail(S4_EINVAL, "null stream");
  if (bytes < kHeaderBytes) return fail(S4_ECORRUPT, "stream shorter than its header");
  if (rd32(enc) != kMagic) return fail(S4_ECORRUPT, "bad magic");
  uint16_t ver, fl;
  std::memcpy(&ver, enc + 4, 2);
  std::memcpy(&fl, enc + 6, 2);
  if (ver != kVersion) return fail(S4_ECORRUPT, "unknown stream version");
  if (fl & ~15u) return fail(S4_ECORRUPT, "unknown flag bits");
  std::memcpy(&v->n, enc + 8, 8);
  std::memcpy(&v->nb, enc + 16, 4);
  std::memcpy(&v->t, enc + 20, 4);
  std::memcpy(&v->pw, enc + 24, 8);
  v->flags = fl;
  if (v->t >= kBlock || uint64_t(v->nb) * kBlock + v->t != v->n)
    return fail(S4_ECORRUPT, "length fields disagree");
  const size_t wbytes = round4(v->nb);
  if (bytes < kHeaderBytes + wbytes) return fail(S4_ECORRUPT, "stream truncated in width table");
  v->widths = enc + kHeaderBytes;
  uint64_t pw = 0;
  for (uint32_t k = 0; k < v->nb; ++k) {
    if (v->widths[k] > 32) return fail(S4_ECORRUPT, "block width above 32");
    pw += 4u * v->widths[k];
  }
  for (size_t k = v->nb; k < wbytes; ++k)
    if (enc[kHeaderBytes + k]) return fail(S4_ECORRUPT, "nonzero width padding");
  if (pw != v->pw) return fail(S4_ECORRUPT, "payload size disagrees with widths");
  const size_t base = kHeaderBytes + wbytes + 4u * pw + 4u * size_t(v->t);
  v->payload = enc + kHeaderBytes + wbytes;
  v->tail = v->payload + 4u * pw;
  v->pages = nullptr;
  v->pages_bytes = v->x_positions = v->x_array_words = 0;
  if (!(fl & kFlagPatched)) {
    if (bytes != base) return fail(S4_ECORRUPT, "stream size disagrees with header");
    return S4_OK;
  }
  if (bytes < base) return fail(S4_ECORRUPT, "stream truncated before its pages");
  v->pages = enc + base;
  v->pages_bytes = bytes - base;
  return check_pages(v, enc + base, enc + bytes);
}

}  // namespace s4

using namespace s4;

extern "C" {

const char *s4_last_error(void) { return g_last_error.c_str(); }
int s4_version(void) { return int(kVersion); }

size_t s4_encoded_bound(uint64_t n) { return stream_bound(n); }

int s4_encode(const uint32_t *in, uint64_t n, uint8_t *out, size_t cap, size_t *out_bytes) {
  return encode_one(in, n, S4_DELTA_D4, out, cap, out_bytes);
}

int s4_encode_ex(const uint32_t *in, uint64_t n, uint32_t delta, uint8_t *out, size_t cap, size_t *out_bytes) {
  return encode_one(in, n, delta, out, cap, out_bytes);
}

int s4_encode_many(const uint32_t *in, const uint64_t *in_offsets, uint64_t count, uint32_t delta, uint8_t *out,
                   const uint64_t *out_offsets, uint64_t *out_bytes, int nthreads) {
  if (!in_offsets || !out_offsets || !out_bytes || (count && (!in || !out)))
    return fail(S4_EINVAL, "s4_encode_many: null argument");
  if (nthreads <= 0) nthreads = int(std::max(1u, std::thread::hardware_concurrency()));
  nthreads = int(std::min<uint64_t>(uint64_t(nthreads), std::max<uint64_t>(1, count)));
  std::atomic<uint64_t> next{0};
  std::atomic<int> first_err{0};
  std::vector<std::string> errs(static_cast<size_t>(nthreads));
  auto work = [&](int tid) {
    for (;;) {
      uint64_t i = next.fetch_add(1);
      if (i >= count || first_err.load()) break;
      uint64_t n = in_offsets[i + 1] - in_offsets[i];
      size_t cap = size_t(out_offsets[i + 1] - out_offsets[i]);
      size_t nbytes = 0;
      int rc = encode_one(in + in_offsets[i], n, delta, out + out_offsets[i], cap, &nbytes);
      out_bytes[i] = nbytes;
      if (rc) {
        int expected = 0;
        if (first_err.compare_exchange_strong(expected, rc))
          errs[size_t(tid)] = "list " + std::to_string(i) + ": " + g_last_error;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto &th : pool) th.join();
  if (first_err.load()) {
    for (auto &e : errs)
      if (!e.empty()) return fail(first_err.load(), e);
    return fail(first_err.load(), "s4_encode_many failed");
  }
  return S4_OK;
}

int s4_decode(const uint8_t *enc, size_t bytes, uint32_t *out, uint64_t cap, uint64_t *n_out) {
  if (!n_out) return fail(S4_EINVAL, "null n_out");
  StreamView v;
  int rc = parse_stream(enc, bytes, &v);
  if (rc) return rc;
  *n_out = v.n;
  if (cap < v.n) return fail(S4_ERANGE, "s4_decode: cap < n");
  if (v.n && !out) return fail(S4_EINVAL, "s4_decode: null out");
  const uint32_t form = (v.flags >> 1) & 3u;
  // 1. every block's deltas: value q of lane j is bits [q b, q b + b) of the
  //    lane's LSB-first stream, whose m-th word is payload word 4 m + j
  uint64_t wpos = 0;
  for (uint64_t k = 0; k < v.nb; ++k) {
    const uint32_t b = v.widths[k];
    const uint8_t *w = v.payload + 4 * wpos;
    uint32_t *d = out + k * kBlock;
    const uint64_t mask = (uint64_t(1) << b) - 1u;
    for (uint32_t j = 0; j < 4; ++j)
      for (uint32_t q = 0; q < 32; ++q) {
        if (b == 0) {
          d[4 * q + j] = 0;
          continue;
        }
        const uint32_t bit = q * b, m = bit >> 5, sh = bit & 31u;
        uint64_t win = rd32(w + 4 * (4 * m + j));
        if (sh + b > 32) win |= uint64_t(rd32(w + 4 * (4 * (m + 1) + j))) << 32;
        d[4 * q + j] = uint32_t((win >> sh) & mask);
      }
    wpos += 4u * b;
  }
  // 2. patched streams: each exception's high bits (b - b' of them, from the
  //    page's array for that difference, in order) go above its b' low bits
  if (v.patched()) {
    const uint8_t *p = v.pages;
    for (uint64_t k0 = 0; k0 < v.nb; k0 += kPage) {
      const uint64_t k1 = std::min<uint64_t>(v.nb, k0 + kPage);
      const uint32_t meta_len = rd32(p);
      const uint8_t *m = p + 4;
      const uint8_t *q = m + round4(meta_len);
      const uint32_t present = rd32(q);
      q += 4;
      const uint8_t *arr[33] = {nullptr};
      uint64_t used[33] = {0};
      for (uint32_t e = 1; e <= 32; ++e) {
        if (!((present >> (e - 1)) & 1u)) continue;
        const uint32_t count = rd32(q);
        arr[e] = q + 4;
        q += 4u + 4u * uint64_t(e) * ((count + 31u) / 32u);
      }
      uint64_t o = 0;
      for (uint64_t k = k0; k < k1; ++k) {
        const uint32_t b = m[o], c = m[o + 1], bp = v.widths[k];
        o += 2;
        for (uint32_t x = 0; x < c; ++x) {
          const uint32_t pos = m[o + x], e = b - bp;
          const uint64_t bit = used[e]++ * e, wi = bit >> 5, sh = bit & 31u;
          uint64_t win = rd32(arr[e] + 4 * wi);
          if (sh + e > 32) win |= uint64_t(rd32(arr[e] + 4 * (wi + 1))) << 32;
          const uint64_t high = (win >> sh) & ((uint64_t(1) << e) - 1u);
          out[k * kBlock + pos] |= uint32_t(high << bp);
        }
        o += c;
      }
      p = q;
    }
  }
  // 3. the form's inverse in index order (x_i = delta_i + the value the form
  //    subtracts, Sec. 5), then the raw tail
  for (uint64_t i = 0; i < uint64_t(v.nb) * kBlock; ++i) out[i] += reference(out, i, form);
  for (uint32_t i = 0; i < v.t; ++i) out[uint64_t(v.nb) * kBlock + i] = rd32(v.tail + 4 * i);
  return S4_OK;
}

int s4_decoded_length(const uint8_t *enc, size_t bytes, uint64_t *n) {
  if (!n) return fail(S4_EINVAL, "null n");
  StreamView v;
  int rc = parse_stream(enc, bytes, &v);
  if (rc) return rc;
  *n = v.n;
  return S4_OK;
}

}  // extern "C"

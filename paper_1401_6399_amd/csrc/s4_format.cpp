// Host side of the codec: the S4-BP128-D4 encoder (Sec. 4.2-4.3, Sec. 5),
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

size_t stream_bound(uint64_t n) {
  uint64_t nb = n / kBlock, t = n % kBlock;
  return kHeaderBytes + round4(nb) + size_t(nb) * 512u + 4u * size_t(t);
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

int encode_one(const uint32_t *in, uint64_t n, uint32_t delta, uint8_t *out, size_t cap, size_t *out_bytes) {
  if ((!in && n) || !out_bytes) return fail(S4_EINVAL, "s4_encode: null argument");
  if (delta > S4_DELTA_D1) return fail(S4_EINVAL, "s4_encode: unknown differential form");
  if (n / kBlock > 0xFFFFFFFFull) return fail(S4_EINVAL, "s4_encode: list too long");
  bool strictly = true;
  for (uint64_t i = 1; i < n; ++i) {
    if (in[i] < in[i - 1]) return fail(S4_EUNSORTED, "s4_encode: input decreases at index " + std::to_string(i));
    strictly &= in[i] != in[i - 1];
  }
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

int parse_stream(const uint8_t *enc, size_t bytes, StreamView *v) {
  if (!enc || !v) return fail(S4_EINVAL, "null stream");
  if (bytes < kHeaderBytes) return fail(S4_ECORRUPT, "stream shorter than its header");
  if (rd32(enc) != kMagic) return fail(S4_ECORRUPT, "bad magic");
  uint16_t ver, fl;
  std::memcpy(&ver, enc + 4, 2);
  std::memcpy(&fl, enc + 6, 2);
  if (ver != kVersion) return fail(S4_ECORRUPT, "unknown stream version");
  if (fl & ~7u) return fail(S4_ECORRUPT, "unknown flag bits");
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
  if (bytes != kHeaderBytes + wbytes + 4u * pw + 4u * size_t(v->t))
    return fail(S4_ECORRUPT, "stream size disagrees with header");
  v->payload = enc + kHeaderBytes + wbytes;
  v->tail = v->payload + 4u * pw;
  return S4_OK;
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

int s4_decoded_length(const uint8_t *enc, size_t bytes, uint64_t *n) {
  if (!n) return fail(S4_EINVAL, "null n");
  StreamView v;
  int rc = parse_stream(enc, bytes, &v);
  if (rc) return rc;
  *n = v.n;
  return S4_OK;
}

}  // extern "C"

// Seeded synthetic posting lists and query streams.
//
// This module holds no part of the compression or intersection method: it
// only draws sorted sets of distinct uint32 document IDs and term lists for
// queries.  Both the oracle side and the GPU side consume its output.
//
// Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", 2014) seeds xoshiro256** (Blackman and
// Vigna, "Scrambled linear pseudorandom number generators", 2018).  Every
// list gets its own stream derived from (seed, list index), so the output is
// independent of the thread count.
//
// Distributions:
//   uniform   : n distinct values drawn uniformly without replacement from
//               [0, U) with Floyd's sampling algorithm, emitted sorted.
//   clustered : clusters are generated one after another; a cluster starts
//               at s ~ U[0, U), has c ~ Geometric(1/1024) members on
//               {1, 2, ...} (mean 1024) and consecutive members differ by
//               g ~ Geometric(1/2) on {1, 2, ...} (mean 2); members >= U are
//               dropped; clusters are added until n distinct values have been
//               seen, cutting the last cluster at the n-th new value; the
//               set is emitted sorted.
//   queries   : k distinct terms, each drawn with probability proportional
//               to sqrt(length) (duplicates within a query are redrawn).
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>
#include <atomic>

namespace {

inline uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Xoshiro {
  uint64_t s[4];
  explicit Xoshiro(uint64_t seed) {
    uint64_t sm = seed;
    for (int i = 0; i < 4; ++i) s[i] = splitmix64(sm);
  }
  static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  inline uint64_t next() {
    const uint64_t result = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return result;
  }
  // uniform integer in [0, range), range >= 1, unbiased (Lemire 2019)
  inline uint64_t below(uint64_t range) {
    unsigned __int128 m = (unsigned __int128)next() * range;
    uint64_t l = (uint64_t)m;
    if (l < range) {
      uint64_t t = (0 - range) % range;
      while (l < t) { m = (unsigned __int128)next() * range; l = (uint64_t)m; }
    }
    return (uint64_t)(m >> 64);
  }
  // uniform double in (0, 1]
  inline double unit_open0() { return (double)((next() >> 11) + 1) * (1.0 / 9007199254740992.0); }
  // Geometric(p) on {1, 2, ...} by inversion
  inline uint64_t geometric(double p) {
    if (p >= 1.0) return 1;
    double u = unit_open0();
    return 1 + (uint64_t)std::floor(std::log(u) / std::log1p(-p));
  }
  // Geometric(1/2) on {1, 2, ...}: one plus the number of trailing zero bits
  inline uint64_t geometric_half() {
    uint64_t r;
    uint64_t extra = 0;
    while ((r = next()) == 0) extra += 64;
    return 1 + extra + (uint64_t)__builtin_ctzll(r);
  }
};

uint64_t stream_seed(uint64_t seed, uint64_t idx) {
  uint64_t s = seed ^ (0xD1B54A32D192ED03ull * (idx + 1));
  return splitmix64(s);
}

// Bitmap over [0, U) allocated in 4 KiB pages on first touch.
struct PagedBitmap {
  static constexpr int kPageBits = 15;  // 32768 bits per page
  uint64_t universe;
  std::vector<uint64_t *> pages;
  std::vector<uint32_t> touched;
  explicit PagedBitmap(uint64_t U) : universe(U), pages((size_t)((U >> kPageBits) + 1), nullptr) {}
  ~PagedBitmap() { for (uint32_t p : touched) std::free(pages[p]); }
  // returns true when v was not present before
  inline bool insert(uint64_t v) {
    uint64_t p = v >> kPageBits;
    uint64_t *pg = pages[p];
    if (!pg) {
      pg = (uint64_t *)std::calloc((1u << kPageBits) / 64, sizeof(uint64_t));
      pages[p] = pg;
      touched.push_back((uint32_t)p);
    }
    uint64_t bit = v & ((1u << kPageBits) - 1);
    uint64_t m = 1ull << (bit & 63);
    uint64_t &w = pg[bit >> 6];
    if (w & m) return false;
    w |= m;
    return true;
  }
  inline bool contains(uint64_t v) const {
    const uint64_t *pg = pages[v >> kPageBits];
    if (!pg) return false;
    uint64_t bit = v & ((1u << kPageBits) - 1);
    return (pg[bit >> 6] >> (bit & 63)) & 1;
  }
  uint64_t extract_sorted(uint32_t *out) {
    std::sort(touched.begin(), touched.end());
    uint64_t c = 0;
    for (uint32_t p : touched) {
      const uint64_t *pg = pages[p];
      for (uint32_t w = 0; w < (1u << kPageBits) / 64; ++w) {
        uint64_t word = pg[w];
        while (word) {
          int t = __builtin_ctzll(word);
          out[c++] = (uint32_t)(((uint64_t)p << kPageBits) + 64u * w + (uint64_t)t);
          word &= word - 1;
        }
      }
    }
    return c;
  }
};

void gen_uniform(uint64_t seed, uint64_t U, uint64_t n, uint32_t *out) {
  Xoshiro rng(seed);
  PagedBitmap bm(U);
  // Floyd: for j = U-n .. U-1 draw t in [0, j]; take t if new, else j
  for (uint64_t j = U - n; j < U; ++j) {
    uint64_t t = rng.below(j + 1);
    if (!bm.insert(t)) bm.insert(j);
  }
  bm.extract_sorted(out);
}

void gen_clustered(uint64_t seed, uint64_t U, uint64_t n, uint32_t *out) {
  Xoshiro rng(seed);
  PagedBitmap bm(U);
  uint64_t distinct = 0;
  const double p_size = 1.0 / 1024.0;
  while (distinct < n) {
    uint64_t v = rng.below(U);
    uint64_t c = rng.geometric(p_size);
    for (uint64_t i = 0; i < c && distinct < n; ++i) {
      if (i) {
        v += rng.geometric_half();
        if (v >= U) break;
      }
      if (bm.insert(v)) ++distinct;
    }
  }
  bm.extract_sorted(out);
}

template <class F>
void parallel_for(uint64_t count, int nthreads, F f) {
  if (nthreads <= 1 || count <= 1) {
    for (uint64_t i = 0; i < count; ++i) f(i);
    return;
  }
  std::atomic<uint64_t> next{0};
  std::vector<std::thread> ts;
  for (int t = 0; t < nthreads; ++t)
    ts.emplace_back([&] {
      for (;;) {
        uint64_t i = next.fetch_add(1);
        if (i >= count) break;
        f(i);
      }
    });
  for (auto &t : ts) t.join();
}

}  // namespace

extern "C" {

// kind: 0 = uniform, 1 = clustered.  Returns 0, or -1 if n > U.
int wl_list(int kind, uint64_t seed, uint64_t U, uint64_t n, uint32_t *out) {
  if (n > U) return -1;
  if (n == 0) return 0;
  if (kind == 0) gen_uniform(seed, U, n, out);
  else gen_clustered(seed, U, n, out);
  return 0;
}

// Many lists at once: list i has kind[i], length lens[i], stream
// stream_seed(seed, first_id + i), written at out + offsets[i].
int wl_lists(const int32_t *kind, uint64_t seed, uint64_t first_id, uint64_t U, const uint64_t *lens,
             const uint64_t *offsets, uint64_t count, uint32_t *out, int nthreads) {
  for (uint64_t i = 0; i < count; ++i)
    if (lens[i] > U) return -1;
  parallel_for(count, nthreads, [&](uint64_t i) {
    wl_list(kind[i], stream_seed(seed, first_id + i), U, lens[i], out + offsets[i]);
  });
  return 0;
}

uint64_t wl_stream_seed(uint64_t seed, uint64_t idx) { return stream_seed(seed, idx); }

// Queries: for each query draw k ~ U{kmin..kmax} then k distinct terms with
// P(t) proportional to sqrt(lens[t]).  terms must hold nq * kmax entries;
// offsets[nq + 1] receives the CSR boundaries.
int wl_queries(uint64_t seed, const uint64_t *lens, uint64_t nlists, uint64_t nq, uint32_t kmin,
               uint32_t kmax, uint32_t *terms, uint64_t *offsets) {
  if (kmin == 0 || kmax < kmin || kmax > nlists) return -1;
  std::vector<double> cdf(nlists);
  double acc = 0;
  for (uint64_t t = 0; t < nlists; ++t) { acc += std::sqrt((double)lens[t]); cdf[t] = acc; }
  Xoshiro rng(seed);
  uint64_t pos = 0;
  offsets[0] = 0;
  std::vector<uint32_t> cur;
  for (uint64_t q = 0; q < nq; ++q) {
    uint32_t k = kmin + (uint32_t)rng.below(kmax - kmin + 1);
    cur.clear();
    while (cur.size() < k) {
      double u = (double)(rng.next() >> 11) * (1.0 / 9007199254740992.0) * acc;
      uint64_t t = (uint64_t)(std::upper_bound(cdf.begin(), cdf.end(), u) - cdf.begin());
      if (t >= nlists) t = nlists - 1;
      if (std::find(cur.begin(), cur.end(), (uint32_t)t) == cur.end()) cur.push_back((uint32_t)t);
    }
    for (uint32_t t : cur) terms[pos++] = t;
    offsets[q + 1] = pos;
  }
  return 0;
}

// Long query traces, in parallel: the same law as wl_queries (k ~
// U{kmin..kmax}, k distinct terms, P(t) proportional to sqrt(lens[t])), drawn
// with Vose's alias method (M. D. Vose, "A linear algorithm for generating
// random numbers with a given distribution", IEEE TSE 1991) so each term
// costs O(1).  Queries are generated in blocks of 2^16, block b from the
// stream (seed, b): first every query's k, then (after a prefix sum) its
// terms, so the output does not depend on the thread count.  terms must
// hold nq * kmax entries.
int wl_queries_alias(uint64_t seed, const uint64_t *lens, uint64_t nlists, uint64_t nq, uint32_t kmin,
                     uint32_t kmax, uint32_t *terms, uint64_t *offsets, int nthreads) {
  if (kmin == 0 || kmax < kmin || kmax > nlists || nlists > (1ull << 32)) return -1;
  // alias table: prob[i] scaled to [0, 2^53], alias[i]
  std::vector<double> w(nlists);
  double sum = 0;
  for (uint64_t t = 0; t < nlists; ++t) { w[t] = std::sqrt((double)lens[t]); sum += w[t]; }
  if (!(sum > 0)) return -1;
  std::vector<double> prob(nlists);
  std::vector<uint32_t> alias(nlists, 0);
  std::vector<uint32_t> small, large;
  for (uint64_t t = 0; t < nlists; ++t) {
    prob[t] = w[t] * (double)nlists / sum;
    (prob[t] < 1.0 ? small : large).push_back((uint32_t)t);
  }
  while (!small.empty() && !large.empty()) {
    const uint32_t l = small.back(); small.pop_back();
    const uint32_t g = large.back(); large.pop_back();
    alias[l] = g;
    prob[g] = (prob[g] + prob[l]) - 1.0;
    (prob[g] < 1.0 ? small : large).push_back(g);
  }
  for (uint32_t t : large) prob[t] = 1.0;
  for (uint32_t t : small) prob[t] = 1.0;  // rounding leftovers
  constexpr uint64_t kBlockQ = 1ull << 16;
  const uint64_t blocks = (nq + kBlockQ - 1) / kBlockQ;
  // pass 1: k of every query
  offsets[0] = 0;
  parallel_for(blocks, nthreads, [&](uint64_t b) {
    Xoshiro rng(stream_seed(seed, 2 * b));
    const uint64_t q1 = std::min(nq, (b + 1) * kBlockQ);
    for (uint64_t q = b * kBlockQ; q < q1; ++q) offsets[q + 1] = kmin + rng.below(kmax - kmin + 1);
  });
  for (uint64_t q = 0; q < nq; ++q) offsets[q + 1] += offsets[q];
  // pass 2: the terms
  parallel_for(blocks, nthreads, [&](uint64_t b) {
    Xoshiro rng(stream_seed(seed, 2 * b + 1));
    const uint64_t q1 = std::min(nq, (b + 1) * kBlockQ);
    for (uint64_t q = b * kBlockQ; q < q1; ++q) {
      uint32_t *cur = terms + offsets[q];
      const uint32_t k = (uint32_t)(offsets[q + 1] - offsets[q]);
      uint32_t have = 0;
      while (have < k) {
        const uint64_t i = rng.below(nlists);
        const double u = (double)(rng.next() >> 11) * (1.0 / 9007199254740992.0);
        const uint32_t t = u < prob[i] ? (uint32_t)i : alias[i];
        if (std::find(cur, cur + have, t) == cur + have) cur[have++] = t;
      }
    }
  });
  return 0;
}

// Poisson arrival times (seconds) at the given rate.
int wl_arrivals(uint64_t seed, double rate, uint64_t count, double *times) {
  if (!(rate > 0)) return -1;
  Xoshiro rng(seed);
  double t = 0;
  for (uint64_t i = 0; i < count; ++i) {
    t += -std::log(rng.unit_open0()) / rate;
    times[i] = t;
  }
  return 0;
}

}  // extern "C"

// Bitmap lists of a hybrid index (hyb+m2, Sec. 7.7): lists dense enough
// (average gap universe / n at most B) are held as bitmaps over the
// universe instead of compressed blocks.  They are built on the device from
// their compressed streams: decode, set one bit per value, then one select
// sample per 128 values so that the chunk pipeline can enumerate a bitmap
// list 128 values at a time when it is a query's shortest list.
#include <algorithm>
#include <vector>

#include "s4_kernels.h"

namespace s4 {

// One thread per value: set its bit; flag values outside the universe.
__global__ void k_bitmap_set(const uint32_t *__restrict__ vals, uint64_t n, uint32_t *__restrict__ bm,
                             uint64_t universe, uint32_t *__restrict__ err) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t x = vals[i];
  if (uint64_t(x) >= universe) {
    *err = 1u;
    return;
  }
  atomicOr(bm + (x >> 5), 1u << (x & 31u));
}

// One thread per 128-value chunk: its select sample is its first value.
__global__ void k_bitmap_select(const uint32_t *__restrict__ vals, uint64_t n, uint32_t *__restrict__ sel) {
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k * kBlock < n) sel[k] = vals[k * kBlock];
}

int build_bitmaps(Upload &u, uint64_t universe, hipStream_t stream, void **mem, std::vector<DList> *descs,
                  uint64_t *bitmap_bytes, uint64_t *select_bytes) {
  const size_t L = u.views.size();
  const uint64_t words = (universe + 31) / 32;
  std::vector<uint64_t> bm_off(L), sel_off(L);
  uint64_t total = 0, max_n = 0;
  *bitmap_bytes = 0;
  *select_bytes = 0;
  for (size_t i = 0; i < L; ++i) {
    const uint64_t n = u.views[i].n, chunks = (n + kBlock - 1) / kBlock;
    bm_off[i] = total;
    total = align_up(total + 4 * words, 256);
    sel_off[i] = total;
    total = align_up(total + 4 * std::max<uint64_t>(chunks, 1), 256);
    *bitmap_bytes += 4 * words;
    *select_bytes += 4 * chunks;
    max_n = std::max(max_n, n);
  }
  char *dev = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&dev), std::max<uint64_t>(total, 256)) != hipSuccess)
    return fail(S4_ENOMEM, "bitmap allocation of " + std::to_string(total) + " bytes failed");
  // the lists' compressed forms, decoded one at a time into vals
  void *tmp = nullptr;
  std::vector<DList> tdesc;
  int rc = build_arena(u, stream, &tmp, &tdesc);
  if (rc) {
    (void)hipFree(dev);
    return rc;
  }
  uint32_t *vals = nullptr, *err = nullptr;
  if (hipMalloc(reinterpret_cast<void **>(&vals), 4 * std::max<uint64_t>(max_n, 1)) != hipSuccess ||
      hipMalloc(reinterpret_cast<void **>(&err), 256) != hipSuccess) {
    if (vals) (void)hipFree(vals);
    (void)hipFree(tmp);
    (void)hipFree(dev);
    return fail(S4_ENOMEM, "bitmap build scratch allocation failed");
  }
  auto cleanup = [&]() {
    (void)hipFree(err);
    (void)hipFree(vals);
    (void)hipFree(tmp);
  };
  hipError_t e = hipMemsetAsync(dev, 0, std::max<uint64_t>(total, 256), stream);
  if (e != hipSuccess) {
    cleanup();
    (void)hipFree(dev);
    return hip_fail(e, "bitmap clear");
  }
  e = hipMemsetAsync(err, 0, 4, stream);
  descs->resize(L);
  for (size_t i = 0; e == hipSuccess && i < L; ++i) {
    const DList &t = tdesc[i];
    const uint64_t n = t.n;
    uint32_t *bm = reinterpret_cast<uint32_t *>(dev + bm_off[i]);
    uint32_t *sel = reinterpret_cast<uint32_t *>(dev + sel_off[i]);
    if (n) {
      rc = decode_range(t, 0, t.nb + (t.t ? 1u : 0u), vals, stream);
      if (rc) {
        cleanup();
        (void)hipFree(dev);
        return rc;
      }
      hipLaunchKernelGGL(k_bitmap_set, dim3(uint32_t((n + 255) / 256)), dim3(256), 0, stream, vals, n, bm, universe,
                         err);
      const uint64_t chunks = (n + kBlock - 1) / kBlock;
      hipLaunchKernelGGL(k_bitmap_select, dim3(uint32_t((chunks + 255) / 256)), dim3(256), 0, stream, vals, n, sel);
      e = hipGetLastError();
    }
    DList d{};
    d.payload = bm;
    d.bmax = sel;
    d.n = n;
    d.nb = uint32_t((n + kBlock - 1) / kBlock);
    d.t = 0;
    d.mode = kBitmapList;
    d.aux = uint32_t(words);
    (*descs)[i] = d;
  }
  uint32_t h_err = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h_err, err, 4, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  cleanup();
  if (e != hipSuccess) {
    (void)hipFree(dev);
    return hip_fail(e, "bitmap build");
  }
  if (h_err) {
    (void)hipFree(dev);
    return fail(S4_EINVAL, "a bitmap list has values >= universe");
  }
  *mem = dev;
  return S4_OK;
}

}  // namespace s4

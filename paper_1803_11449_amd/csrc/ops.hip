// Whole-sketch word operations: the window reset (Sec. 4: the DHLA starts
// every period with all bits 0) and the OR-merge of two monitors' sketches.
#include "ddhf_internal.h"

namespace ddhf {

// Word fill with 16-byte stores (a kernel rather than hipMemsetAsync, so
// the launch sequences stay capturable into graphs).
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n4 = n / 4;
  uint4 *p4 = reinterpret_cast<uint4 *>(p);
  const uint4 q = make_uint4(v, v, v, v);
  for (size_t i = tid; i < n4; i += stride) p4[i] = q;
  for (size_t i = n4 * 4 + tid; i < n; i += stride) p[i] = v;
}

// dst |= src, word by word (16-byte accesses; both 16-byte aligned).
__global__ __launch_bounds__(256) void k_or_u32(uint32_t *__restrict__ dst,
                                                const uint32_t *__restrict__ src, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n4 = n / 4;
  uint4 *d4 = reinterpret_cast<uint4 *>(dst);
  const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
  for (size_t i = tid; i < n4; i += stride) {
    uint4 a = d4[i];
    const uint4 b = s4[i];
    a.x |= b.x; a.y |= b.y; a.z |= b.z; a.w |= b.w;
    d4[i] = a;
  }
  for (size_t i = n4 * 4 + tid; i < n; i += stride) dst[i] |= src[i];
}

hipError_t launch_or_u32(uint32_t *dst, const uint32_t *src, size_t n_words, int grid,
                         hipStream_t st) {
  if (n_words == 0) return hipSuccess;
  const size_t need = (n_words / 4 + 255) / 256 + 1;
  if ((size_t)grid > need) grid = (int)need;
  k_or_u32<<<grid, 256, 0, st>>>(dst, src, n_words);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, size_t n_words, uint32_t value, int grid,
                           hipStream_t st) {
  if (n_words == 0) return hipSuccess;
  const size_t need = (n_words / 4 + 255) / 256 + 1;
  if ((size_t)grid > need) grid = (int)need;
  k_fill_u32<<<grid, 256, 0, st>>>(p, n_words, value);
  return hipGetLastError();
}

}  // namespace ddhf

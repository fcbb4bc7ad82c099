// Sketch update (Alg. 1, Sec. 3.2 and 4.1) and the window reset (Sec. 4).
//
// One pass over the packed (a,b) pairs in HBM: each lane loads one 8-byte
// pair (a wave reads 512 contiguous bytes), hashes it in registers (two
// multiply-add-shifts and r-1 shift/xor), and sets one bit in one LE of each
// row. The sketch (10 MiB at the paper's defaults, 160 MiB at k = 18) lives
// in HBM but its hot working set sits in the L2s and the Infinity Cache; the
// bit sets are non-returning atomicOr, which are order-free, so concurrent
// setters never lose a bit. Alg. 1 skips the write when the bit is already
// 1; that test is a plain load, and it turns the heavy hitters' updates
// (whose LEs fill up early in a window) into cache reads instead of
// serialised read-modify-writes on a handful of hot lines.
#include "ddhf_internal.h"

namespace ddhf {

template <int R, bool CHECK>
__global__ __launch_bounds__(256) void k_update(Geom G, uint32_t *__restrict__ sk,
                                                const uint2 *__restrict__ pairs,
                                                size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += stride) {
    const uint2 p = pairs[i];
    const uint32_t bit = hash_h1(G, p.y);
    const uint32_t c0 = hash_dh0(G, p.x);
    const uint32_t mask = 1u << (bit & 31);
    const uint32_t wofs = bit >> 5;
#pragma unroll
    for (int row = 0; row < R; row++) {
      const uint32_t cell = row == 0 ? c0 : (bit_block(G, row, p.x) ^ c0);
      uint32_t *w = sk + ((size_t)(((uint32_t)row << G.k) | cell) * G.wpl + wofs);
      if (CHECK && (*w & mask)) continue;
      atomicOr(w, mask);
    }
  }
}

template <bool CHECK>
static hipError_t dispatch_update(const Geom &G, uint32_t *sk, const uint2 *pairs,
                                  size_t n, int grid, hipStream_t st) {
  switch (G.r) {
    case 3: k_update<3, CHECK><<<grid, 256, 0, st>>>(G, sk, pairs, n); break;
    case 4: k_update<4, CHECK><<<grid, 256, 0, st>>>(G, sk, pairs, n); break;
    case 5: k_update<5, CHECK><<<grid, 256, 0, st>>>(G, sk, pairs, n); break;
    case 6: k_update<6, CHECK><<<grid, 256, 0, st>>>(G, sk, pairs, n); break;
    case 7: k_update<7, CHECK><<<grid, 256, 0, st>>>(G, sk, pairs, n); break;
    case 8: k_update<8, CHECK><<<grid, 256, 0, st>>>(G, sk, pairs, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_update(const Geom &G, uint32_t *sketch, const uint32_t *pairs,
                         size_t n, int grid, int variant, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const size_t need = (n + 255) / 256;
  if ((size_t)grid > need) grid = (int)need;
  const uint2 *p2 = reinterpret_cast<const uint2 *>(pairs);
  return (variant & 1) ? dispatch_update<true>(G, sketch, p2, n, grid, st)
                       : dispatch_update<false>(G, sketch, p2, n, grid, st);
}

// Word fill with 16-byte stores (a kernel rather than hipMemsetAsync, so
// the same launch sequence can later be captured into a graph).
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p,
                                                  size_t n, uint32_t v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n4 = n / 4;
  uint4 *p4 = reinterpret_cast<uint4 *>(p);
  const uint4 q = make_uint4(v, v, v, v);
  for (size_t i = tid; i < n4; i += stride) p4[i] = q;
  for (size_t i = n4 * 4 + tid; i < n; i += stride) p[i] = v;
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

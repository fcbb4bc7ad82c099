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

// ------------------------------------------------------- binned update
//
// For large updates the random read-modify-writes into the sketch are the
// limit (on MI355X a random 4-byte access to a 160 MiB buffer runs at
// ~60 G/s and a global atomicOr at ~27 G/s, whatever the buffer size), so
// the bit sets are moved into LDS instead. Every (pair, row) gives the bit
// index B = ((row * 2^k + cell) * g) + bit of the sketch seen as one bit
// string; tile = B >> 20 names the 128 KiB slice it falls in and
// code = B mod 2^20 the bit inside it.
//   count    each block counts its chunk's codes per tile (LDS histogram)
//   scan     per tile, the blocks' counts become write offsets; over tiles,
//            the totals become run starts; a tile with many codes is cut
//            into several apply items
//   scatter  each block sorts a batch of 4096 pairs' codes by tile in LDS
//            and writes them into its part of each tile's run, so stores
//            go out in runs rather than one line per lane
//   apply    one workgroup per item: the tile in LDS (144 KiB max per
//            workgroup on gfx950), ds_or per code. The first item of a tile
//            reads and writes the tile itself; the other items of a cut
//            tile write their bits to a scratch tile instead
//   merge    each cut tile ORs its scratch tiles into the sketch
// Only the pairs, the code runs and whole tiles move through HBM.

constexpr uint32_t CODE_MASK = (1u << BIN_TILE_LOG2) - 1;
constexpr int PAIRS_PER_THREAD = 4;             // scatter batch: 4096 pairs

template <int R>
__device__ __forceinline__ void pair_codes(const Geom &G, uint2 p, uint32_t *B) {
  const uint32_t bit = hash_h1(G, p.y);
  const uint32_t c0 = hash_dh0(G, p.x);
#pragma unroll
  for (int row = 0; row < R; row++) {
    const uint32_t cell = row == 0 ? c0 : (bit_block(G, row, p.x) ^ c0);
    // sketch bit index; < 2^32 since the sketch is at most 2^BIN_MAX tiles
    B[row] = ((((uint32_t)row << G.k) | cell) << G.log2g) | bit;
  }
}

// Pairs are read as uint4 (two pairs per lane per load), COUNT_V4 loads in
// flight per lane; a chunk starts on an even pair so the loads are aligned.
constexpr int COUNT_V4 = 8;

template <int R>
__device__ __forceinline__ void count_pair(const Geom &G, uint2 p, uint32_t *h) {
  uint32_t B[R];
  pair_codes<R>(G, p, B);
#pragma unroll
  for (int row = 0; row < R; row++) atomicAdd(&h[B[row] >> BIN_TILE_LOG2], 1u);
}

template <int R>
__global__ __launch_bounds__(1024) void k_bin_count(Geom G, const uint2 *__restrict__ pairs,
                                                    size_t n, size_t chunk, uint32_t nbins,
                                                    uint32_t nblk,
                                                    uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[BIN_MAX];
  for (uint32_t t = threadIdx.x; t < nbins; t += blockDim.x) h[t] = 0;
  __syncthreads();
  const size_t p0 = (size_t)blockIdx.x * chunk;
  const size_t p1 = p0 + chunk < n ? p0 + chunk : n;
  if (p0 < p1) {
    // p0 is even (chunk is even); pairs before the last even boundary go
    // through uint4 loads, an odd last pair alone
    const uint4 *q = reinterpret_cast<const uint4 *>(pairs + p0);
    const size_t nq = (p1 - p0) / 2;
    for (size_t i0 = 0; i0 < nq; i0 += (size_t)blockDim.x * COUNT_V4) {
      uint4 v[COUNT_V4];
#pragma unroll
      for (int j = 0; j < COUNT_V4; j++) {
        const size_t i = i0 + (size_t)j * blockDim.x + threadIdx.x;
        v[j] = i < nq ? q[i] : make_uint4(0, 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < COUNT_V4; j++) {
        const size_t i = i0 + (size_t)j * blockDim.x + threadIdx.x;
        if (i >= nq) continue;
        count_pair<R>(G, make_uint2(v[j].x, v[j].y), h);
        count_pair<R>(G, make_uint2(v[j].z, v[j].w), h);
      }
    }
    if (((p1 - p0) & 1) && threadIdx.x == 0) count_pair<R>(G, pairs[p1 - 1], h);
  }
  __syncthreads();
  for (uint32_t t = threadIdx.x; t < nbins; t += blockDim.x)
    hist[(size_t)t * nblk + blockIdx.x] = h[t];
}

// Exclusive prefix sum over a workgroup of 1024 threads.
__device__ __forceinline__ uint32_t blk_scan_1024(uint32_t v, uint32_t *total, uint32_t *sh) {
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t t = __shfl_up(inc, d, 64);
    if (lane >= (uint32_t)d) inc += t;
  }
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t x = lane < 16 ? sh[lane] : 0;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      const uint32_t t = __shfl_up(x, d, 64);
      if (lane >= (uint32_t)d) x += t;
    }
    if (lane < 16) sh[lane] = x;
  }
  __syncthreads();
  const uint32_t off = wid ? sh[wid - 1] : 0;
  *total = sh[15];
  __syncthreads();
  return off + inc - v;
}

// Per tile: the blocks' counts -> exclusive offsets (in place); the total.
__global__ __launch_bounds__(1024) void k_bin_scan_cols(uint32_t *__restrict__ hist,
                                                        uint32_t nblk,
                                                        uint32_t *__restrict__ totals) {
  __shared__ uint32_t sh[16];
  uint32_t *col = hist + (size_t)blockIdx.x * nblk;
  const uint32_t v = threadIdx.x < nblk ? col[threadIdx.x] : 0;
  uint32_t total;
  const uint32_t ex = blk_scan_1024(v, &total, sh);
  if (threadIdx.x < nblk) col[threadIdx.x] = ex;
  if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// Apply items of a tile with v codes: one if v <= SPLIT_MIN, else one per
// APPLY_ITEM codes.
__device__ __forceinline__ uint32_t tile_items(uint32_t v) {
  return v == 0 ? 0u : (v <= SPLIT_MIN ? 1u : (v + APPLY_ITEM - 1) / APPLY_ITEM);
}

// Over tiles: run starts, apply-item starts, scratch-slot starts (a tile
// cut into j items owns j-1 scratch tiles) and the item count.
__global__ __launch_bounds__(1024) void k_bin_scan_tiles(const uint32_t *__restrict__ totals,
                                                         uint32_t nbins,
                                                         uint32_t *__restrict__ base,
                                                         uint32_t *__restrict__ item_start,
                                                         uint32_t *__restrict__ xslot,
                                                         uint32_t *__restrict__ n_items) {
  __shared__ uint32_t sh[16];
  constexpr uint32_t PER = BIN_MAX / 1024;
  const uint32_t t0 = threadIdx.x * PER;
  uint32_t c = 0, it = 0, xs = 0;
#pragma unroll
  for (uint32_t j = 0; j < PER; j++) {
    const uint32_t t = t0 + j;
    const uint32_t v = t < nbins ? totals[t] : 0;
    const uint32_t ni = tile_items(v);
    c += v;
    it += ni;
    xs += ni > 1 ? ni - 1 : 0;
  }
  uint32_t tot_c, tot_it, tot_xs;
  uint32_t ec = blk_scan_1024(c, &tot_c, sh);
  uint32_t ei = blk_scan_1024(it, &tot_it, sh);
  uint32_t ex = blk_scan_1024(xs, &tot_xs, sh);
#pragma unroll
  for (uint32_t j = 0; j < PER; j++) {
    const uint32_t t = t0 + j;
    if (t < nbins) {
      const uint32_t v = totals[t];
      const uint32_t ni = tile_items(v);
      base[t] = ec;
      item_start[t] = ei;
      xslot[t] = ex;
      ec += v;
      ei += ni;
      ex += ni > 1 ? ni - 1 : 0;
    }
  }
  if (threadIdx.x == 0) {
    base[nbins] = tot_c;
    item_start[nbins] = tot_it;
    xslot[nbins] = tot_xs;
    *n_items = tot_it;
  }
}

template <int R>
__global__ __launch_bounds__(1024) void k_bin_scatter(Geom G, const uint2 *__restrict__ pairs,
                                                      size_t n, size_t chunk, uint32_t nbins,
                                                      uint32_t nblk,
                                                      const uint32_t *__restrict__ hist,
                                                      const uint32_t *__restrict__ base,
                                                      uint32_t *__restrict__ codes) {
  constexpr uint32_t BATCH = 1024 * PAIRS_PER_THREAD * R;
  __shared__ uint32_t sorted[BATCH];   // (tile << 20 | code), grouped by tile
  __shared__ uint32_t cnt[BIN_MAX];    // codes per tile in this batch
  __shared__ uint32_t lofs[BIN_MAX];   // batch-local run starts
  __shared__ uint32_t gcur[BIN_MAX];   // next global slot of this block per tile
  __shared__ uint32_t sh[16];
  for (uint32_t t = threadIdx.x; t < BIN_MAX; t += blockDim.x) {
    cnt[t] = 0;
    gcur[t] = t < nbins ? base[t] + hist[(size_t)t * nblk + blockIdx.x] : 0;
  }
  __syncthreads();
  const size_t p0 = (size_t)blockIdx.x * chunk;
  const size_t p1 = p0 + chunk < n ? p0 + chunk : n;
  const size_t step = (size_t)blockDim.x * PAIRS_PER_THREAD;
  // the next batch's pairs are loaded while this batch is sorted and written
  uint2 nxt[PAIRS_PER_THREAD];
#pragma unroll
  for (int j = 0; j < PAIRS_PER_THREAD; j++) {
    const size_t i = p0 + (size_t)j * blockDim.x + threadIdx.x;
    nxt[j] = i < p1 ? pairs[i] : make_uint2(0, 0);
  }
  for (size_t i0 = p0; i0 < p1; i0 += step) {
    uint32_t v[PAIRS_PER_THREAD * R], rk[PAIRS_PER_THREAD * R];
    uint2 cur[PAIRS_PER_THREAD];
#pragma unroll
    for (int j = 0; j < PAIRS_PER_THREAD; j++) {
      cur[j] = nxt[j];
      const size_t i = i0 + step + (size_t)j * blockDim.x + threadIdx.x;
      nxt[j] = i < p1 ? pairs[i] : make_uint2(0, 0);
    }
#pragma unroll
    for (int j = 0; j < PAIRS_PER_THREAD; j++) {
      const size_t i = i0 + (size_t)j * blockDim.x + threadIdx.x;
      if (i < p1) {
        uint32_t B[R];
        pair_codes<R>(G, cur[j], B);
#pragma unroll
        for (int row = 0; row < R; row++) {
          const uint32_t t = B[row] >> BIN_TILE_LOG2;
          v[j * R + row] = B[row];
          rk[j * R + row] = atomicAdd(&cnt[t], 1u);
        }
      } else {
#pragma unroll
        for (int row = 0; row < R; row++) v[j * R + row] = ~0u;
      }
    }
    __syncthreads();
    // batch-local run starts (2 tiles per thread)
    const uint32_t ta = threadIdx.x * 2, tb = ta + 1;
    const uint32_t ca = cnt[ta], cb = cnt[tb];
    uint32_t total;
    const uint32_t ex = blk_scan_1024(ca + cb, &total, sh);
    lofs[ta] = ex;
    lofs[tb] = ex + ca;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PAIRS_PER_THREAD * R; q++)
      if (v[q] != ~0u) sorted[lofs[v[q] >> BIN_TILE_LOG2] + rk[q]] = v[q];
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < total; e += blockDim.x) {
      const uint32_t x = sorted[e];
      const uint32_t t = x >> BIN_TILE_LOG2;
      codes[gcur[t] + (e - lofs[t])] = x & CODE_MASK;
    }
    __syncthreads();
    gcur[ta] += ca;
    gcur[tb] += cb;
    cnt[ta] = 0;
    cnt[tb] = 0;
    __syncthreads();
  }
}

// Tile of an item: the largest t with item_start[t] <= it.
__device__ __forceinline__ uint32_t item_tile(const uint32_t *item_start, uint32_t nbins,
                                              uint32_t it) {
  uint32_t lo = 0, hi = nbins;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (item_start[mid] <= it) lo = mid; else hi = mid;
  }
  return lo;
}

constexpr int APPLY_UNROLL = 4;

__global__ __launch_bounds__(1024) void k_bin_apply(uint32_t *__restrict__ sk, size_t words,
                                                    const uint32_t *__restrict__ codes,
                                                    const uint32_t *__restrict__ base,
                                                    const uint32_t *__restrict__ item_start,
                                                    const uint32_t *__restrict__ xslot,
                                                    const uint32_t *__restrict__ n_items_p,
                                                    uint32_t nbins,
                                                    uint32_t *__restrict__ scratch) {
  __shared__ uint32_t tile[BIN_TILE_WORDS];
  const uint32_t n_items = *n_items_p;
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const uint32_t t = item_tile(item_start, nbins, it);
    const uint32_t sub = it - item_start[t];
    const uint32_t c_end = base[t + 1];
    const uint32_t c0 = item_start[t + 1] - item_start[t] == 1 ? base[t]
                                                               : base[t] + sub * APPLY_ITEM;
    const uint32_t c1 = item_start[t + 1] - item_start[t] == 1
                            ? c_end
                            : (c_end - c0 > APPLY_ITEM ? c0 + APPLY_ITEM : c_end);
    const size_t w0 = (size_t)t * BIN_TILE_WORDS;
    const uint32_t tw = (uint32_t)(words - w0 < BIN_TILE_WORDS ? words - w0 : BIN_TILE_WORDS);
    // the first item of a tile owns the tile; item j >= 1 of a cut tile
    // writes scratch tile xslot[t] + j - 1
    uint32_t *dst = sub == 0 ? sk + w0
                             : scratch + (size_t)(xslot[t] + sub - 1) * BIN_TILE_WORDS;
    if (sub == 0) {
      for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) tile[w] = dst[w];
    } else {
      for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) tile[w] = 0;
    }
    __syncthreads();
    // codes [c0,c1): a scalar head up to a 4-aligned index, uint4 body,
    // scalar tail
    const uint32_t up4 = (c0 + 3u) & ~3u;
    const uint32_t a0 = up4 < c1 ? up4 : c1;
    const uint32_t a1 = a0 + ((c1 - a0) & ~3u);
    for (uint32_t c = c0 + threadIdx.x; c < a0; c += blockDim.x) {
      const uint32_t x = codes[c];
      atomicOr(&tile[x >> 5], 1u << (x & 31));
    }
    const uint4 *q = reinterpret_cast<const uint4 *>(codes + a0);
    const uint32_t nq = (a1 - a0) / 4;
    for (uint32_t i = threadIdx.x; i < nq; i += blockDim.x * APPLY_UNROLL) {
      uint4 x[APPLY_UNROLL];
#pragma unroll
      for (int u = 0; u < APPLY_UNROLL; u++) {
        const uint32_t iu = i + u * blockDim.x;
        x[u] = iu < nq ? q[iu] : make_uint4(~0u, ~0u, ~0u, ~0u);
      }
#pragma unroll
      for (int u = 0; u < APPLY_UNROLL; u++) {
        if (x[u].x == ~0u) continue;
        atomicOr(&tile[x[u].x >> 5], 1u << (x[u].x & 31));
        atomicOr(&tile[x[u].y >> 5], 1u << (x[u].y & 31));
        atomicOr(&tile[x[u].z >> 5], 1u << (x[u].z & 31));
        atomicOr(&tile[x[u].w >> 5], 1u << (x[u].w & 31));
      }
    }
    for (uint32_t c = a1 + threadIdx.x; c < c1; c += blockDim.x) {
      const uint32_t x = codes[c];
      atomicOr(&tile[x >> 5], 1u << (x & 31));
    }
    __syncthreads();
    for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) dst[w] = tile[w];
    __syncthreads();
  }
}

// OR the scratch tiles of every cut tile into the sketch: block (t, y)
// takes the y-th 4096-word slice of tile t.
constexpr uint32_t MERGE_SLICE = 4096;

__global__ __launch_bounds__(256) void k_bin_merge(uint32_t *__restrict__ sk, size_t words,
                                                   const uint32_t *__restrict__ item_start,
                                                   const uint32_t *__restrict__ xslot,
                                                   uint32_t nbins,
                                                   const uint32_t *__restrict__ scratch) {
  const uint32_t t = blockIdx.x;
  if (t >= nbins) return;
  const uint32_t n = item_start[t + 1] - item_start[t];
  if (n <= 1) return;
  const size_t w0 = (size_t)t * BIN_TILE_WORDS;
  const uint32_t tw = (uint32_t)(words - w0 < BIN_TILE_WORDS ? words - w0 : BIN_TILE_WORDS);
  const uint32_t s_lo = blockIdx.y * MERGE_SLICE;
  const uint32_t s_hi = s_lo + MERGE_SLICE < tw ? s_lo + MERGE_SLICE : tw;
  const uint32_t *s0 = scratch + (size_t)xslot[t] * BIN_TILE_WORDS;
  for (uint32_t w = s_lo + threadIdx.x * 4; w < s_hi; w += blockDim.x * 4) {
    if (w + 4 <= s_hi) {
      uint4 v = *reinterpret_cast<const uint4 *>(sk + w0 + w);
      for (uint32_t j = 1; j < n; j++) {
        const uint4 x =
            *reinterpret_cast<const uint4 *>(s0 + (size_t)(j - 1) * BIN_TILE_WORDS + w);
        v.x |= x.x; v.y |= x.y; v.z |= x.z; v.w |= x.w;
      }
      *reinterpret_cast<uint4 *>(sk + w0 + w) = v;
    } else {
      for (uint32_t ww = w; ww < s_hi; ww++) {
        uint32_t v = sk[w0 + ww];
        for (uint32_t j = 1; j < n; j++) v |= s0[(size_t)(j - 1) * BIN_TILE_WORDS + ww];
        sk[w0 + ww] = v;
      }
    }
  }
}

template <int R>
static hipError_t binned_rounds(const Geom &G, uint32_t *sk, size_t words, const uint2 *pairs,
                                size_t n, const BinBufs &BB, hipStream_t st) {
  const uint32_t nbins = (uint32_t)((words + BIN_TILE_WORDS - 1) / BIN_TILE_WORDS);
  const size_t round = BB.codes_cap / R;
  for (size_t done = 0; done < n; done += round) {
    const size_t m = n - done < round ? n - done : round;
    const uint2 *pp = pairs + done;
    size_t chunk = (m + BB.nblk - 1) / BB.nblk;
    chunk += chunk & 1;  // even: count pass loads pairs two at a time
    k_bin_count<R><<<BB.nblk, 1024, 0, st>>>(G, pp, m, chunk, nbins, BB.nblk, BB.hist);
    k_bin_scan_cols<<<nbins, 1024, 0, st>>>(BB.hist, BB.nblk, BB.totals);
    k_bin_scan_tiles<<<1, 1024, 0, st>>>(BB.totals, nbins, BB.base, BB.item_start, BB.xslot,
                                         BB.n_items);
    k_bin_scatter<R><<<BB.nblk, 1024, 0, st>>>(G, pp, m, chunk, nbins, BB.nblk, BB.hist, BB.base,
                                               BB.codes);
    k_bin_apply<<<BB.apply_grid, 1024, 0, st>>>(sk, words, BB.codes, BB.base, BB.item_start,
                                                BB.xslot, BB.n_items, nbins, BB.scratch);
    k_bin_merge<<<dim3(nbins, BIN_TILE_WORDS / MERGE_SLICE), 256, 0, st>>>(
        sk, words, BB.item_start, BB.xslot, nbins, BB.scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_update_binned(const Geom &G, uint32_t *sketch, size_t words,
                                const uint32_t *pairs, size_t n, const BinBufs &BB,
                                hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (((uintptr_t)pairs) & 15u) {
    // the count pass reads pairs 16 bytes at a time: take one pair through
    // the direct kernel so the rest starts 16-byte aligned
    hipError_t e = launch_update(G, sketch, pairs, 1, 1, 1, st);
    if (e != hipSuccess) return e;
    pairs += 2;
    if (--n == 0) return hipSuccess;
  }
  const uint2 *p2 = reinterpret_cast<const uint2 *>(pairs);
  switch (G.r) {
    case 3: return binned_rounds<3>(G, sketch, words, p2, n, BB, st);
    case 4: return binned_rounds<4>(G, sketch, words, p2, n, BB, st);
    case 5: return binned_rounds<5>(G, sketch, words, p2, n, BB, st);
    case 6: return binned_rounds<6>(G, sketch, words, p2, n, BB, st);
    case 7: return binned_rounds<7>(G, sketch, words, p2, n, BB, st);
    case 8: return binned_rounds<8>(G, sketch, words, p2, n, BB, st);
    default: return hipErrorInvalidValue;
  }
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

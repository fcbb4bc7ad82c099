// Sketch update (Alg. 1, Sec. 3.2 and 4.1) and the window reset (Sec. 4).
//
// Every launch takes a table of jobs, one per sketch (UpdJob), so a batch of
// links or windows of uneven size runs in one set of launches; a single
// sketch's update is a batch of one. Blocks, tiles and work items are mapped
// to their job by binary search over the jobs' prefix fields.
//
// Two kernels compute the same sketch:
//
// direct   Alg. 1 as written. Each lane loads one 8-byte pair, hashes it in
//          registers (two multiply-add-shifts, r-1 shift/xor) and sets one
//          bit in one LE of each row with a non-returning atomicOr, after a
//          plain load shows the bit unset (Alg. 1 skips a bit already 1;
//          that turns the heavy hitters' updates, whose LEs fill early, into
//          cache reads). Bound by random accesses into the sketch: on MI355X
//          a random 4-byte access to a 160 MiB buffer runs at ~60 G/s and a
//          global atomicOr at ~27 G/s, whatever the buffer size. Used for
//          small updates.
//
// binned   The bit sets are moved into LDS. Every (pair, row) gives the bit
//          index B = ((row * 2^k + cell) * g) + bit of the sketch seen as
//          one bit string; tile = B / 1310720 names the 160 KiB slice it
//          falls in and code = B mod 1310720 the bit inside it (21 bits).
//          Codes are stored three to a 64-bit word; every run a block writes for one tile in
//          one batch is padded to whole words with copies of a code of the
//          run (setting a bit twice sets it once).
//            count    each block walks a sample of its chunk's batches (every
//                     sample-th, in the scatter's batching) and estimates,
//                     per tile, the words its batches will write
//            layout   per tile and block group (the blocks of one XCD), a
//                     region of the estimate plus an eighth plus a pad;
//                     the regions are laid out tile after tile
//            scatter  each block sorts a batch of pairs' codes by tile in
//                     LDS, claims room for each tile's run in its group's
//                     region with one atomicAdd and writes the codes there.
//                     A run that does not fit goes whole to the spill area
//                     and into its tile's list of spill runs. The blocks of
//                     a group fill each region together, so the L2 holds
//                     one partly written line per region rather than one
//                     per tile and block, and lines leave it whole
//            items    per tile, the words written (regions and spill runs);
//                     a tile with many words is cut into several apply items
//            apply    one workgroup per item: the tile in LDS (up to 160 KiB
//                     per workgroup on gfx950), ds_or per code, over the
//                     tile's regions and spill runs. The first item of a
//                     tile reads and writes the tile itself (or, after a
//                     reset, builds it from zeros); the other items of a cut
//                     tile write scratch tiles instead. A finished tile's LE
//                     zero counts are written with it
//            merge    each cut tile ORs its scratch tiles into the sketch
//          Only the pairs (once, plus the sample), the code runs and whole
//          tiles move through HBM.
#include <type_traits>

#include "ddhf_internal.h"

namespace ddhf {

// Pointers read from a job table are generic to the compiler, which then
// emits flat loads and stores; those count against the LDS wait counter too,
// so every wait for an LDS result would also wait for all memory traffic in
// flight. Every job buffer is device global memory: say so.
#define GMEM __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GMEM T *gmem(T *p) {
  return (GMEM T *)p;
}
// HIP's vector structs cannot be copied out of a qualified pointer: 8- and
// 16-byte accesses go through the compiler's own vector types.
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint2 ld2(const GMEM uint2 *p) {
  const v2u v = *reinterpret_cast<const GMEM v2u *>(p);
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 ld4(const GMEM uint4 *p) {
  const v4u v = *reinterpret_cast<const GMEM v4u *>(p);
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(GMEM uint4 *p, uint4 x) {
  v4u v;
  v.x = x.x; v.y = x.y; v.z = x.z; v.w = x.w;
  *reinterpret_cast<GMEM v4u *>(p) = v;
}

// ------------------------------------------------------------ job lookup

__device__ __forceinline__ uint32_t job_of_block(const UpdJob *jobs, uint32_t nj, uint32_t b) {
  uint32_t lo = 0, hi = nj;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].blk0 <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t job_of_tile(const UpdJob *jobs, uint32_t nj, uint32_t t) {
  uint32_t lo = 0, hi = nj;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].tile0 <= t) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t job_of_item(const UpdJob *jobs, uint32_t nj, uint32_t it) {
  uint32_t lo = 0, hi = nj;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].item0 <= it) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- direct

template <int R, bool CHECK>
__global__ __launch_bounds__(256) void k_update(const UpdJob *__restrict__ jobs, uint32_t nj) {
  const uint32_t j = job_of_block(jobs, nj, blockIdx.x);
  const UpdJob &J = jobs[j];
  const Geom G = J.G;
  GMEM uint32_t *__restrict__ sk = gmem(J.sk);
  const GMEM uint2 *__restrict__ pairs = gmem(J.pairs);
  const size_t n = J.n;
  const size_t stride = (size_t)J.nblk * blockDim.x;
  for (size_t i = (size_t)(blockIdx.x - J.blk0) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint2 p = ld2(pairs + i);
    const uint32_t bit = hash_h1(G, p.y);
    const uint32_t c0 = hash_dh0(G, p.x);
    const uint32_t mask = 1u << (bit & 31);
    const uint32_t wofs = bit >> 5;
#pragma unroll
    for (int row = 0; row < R; row++) {
      const uint32_t cell = row == 0 ? c0 : (bit_block(G, row, p.x) ^ c0);
      GMEM uint32_t *w = sk + ((size_t)(((uint32_t)row << G.k) | cell) * G.wpl + wofs);
      if (CHECK && (*w & mask)) continue;
      atomicOr((uint32_t *)w, mask);    // stays a global atomic after inlining
    }
  }
}

// ---------------------------------------------------------------- binned

constexpr uint32_t CODE_BITS = 21;
constexpr uint32_t CODE_MASK = (1u << CODE_BITS) - 1;

template <int R>
__device__ __forceinline__ void pair_codes(const Geom &G, uint2 p, uint32_t *B) {
  const uint32_t bit = hash_h1(G, p.y);
  const uint32_t c0 = hash_dh0(G, p.x);
#pragma unroll
  for (int row = 0; row < R; row++) {
    const uint32_t cell = row == 0 ? c0 : (bit_block(G, row, p.x) ^ c0);
    // sketch bit index; < 2^32 since a binned sketch has at most BIN_MAX tiles
    B[row] = ((((uint32_t)row << G.k) | cell) << G.log2g) | bit;
  }
}

template <int R>
__device__ __forceinline__ void count_pair(const Geom &G, uint2 p, uint32_t *h) {
  uint32_t B[R];
  pair_codes<R>(G, p, B);
#pragma unroll
  for (int row = 0; row < R; row++) atomicAdd(&h[bin_tile(B[row])], 1u);
}

// Codes are stored three to a 64-bit word (bits 0-20, 21-41, 42-62), and
// every run the scatter writes (one tile, one batch of a block) is padded
// to whole words. Per block and tile, the count therefore estimates the
// words its batches will write there: it walks the same batches as the
// scatter (PPT pairs per thread of 1024, from the start of the block's
// chunk), but only every J.sample-th of them, adds ceil(c / 3) for a
// sampled batch with c codes in the tile and scales the sum by the
// block's pairs over its sampled batches' pairs (exact for J.sample = 1).
//
// A full batch's pairs are read as uint4 (two pairs per lane per load)
// when PPT is even; a job's pairs start 16-byte aligned and its chunks and
// batches are even, so these loads are aligned. The next batch's loads are issued before
// this batch is counted; past the chunk's last whole uint4 they re-read it.
//
// Register budget: left free, the compiler gives some instantiations 65-90
// VGPRs. Capped at 64 (8 waves per SIMD), the 5-row, 6-pair count of a
// 100M-pair window ran 205 us instead of 224 us. The cap is set only where
// the compiler then still needs no spills (several instantiations spill
// under it, and a spill stalls every batch on the scratch access).
template <int R, int PPT> constexpr int count_waves_per_eu() {
  return (R == 4 && PPT >= 6) || (R == 5 && PPT >= 5) || (R == 7 && PPT == 4) ? 8 : 1;
}

template <int R, int PPT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(count_waves_per_eu<R, PPT>())))
void k_bin_count(const UpdJob *__restrict__ jobs, uint32_t nj) {
  constexpr uint32_t TPT = BIN_SLOTS / 1024;            // tiles per thread
  constexpr int V4 = PPT / 2;
  __shared__ uint32_t h[BIN_SLOTS];
  const UpdJob &J = jobs[job_of_block(jobs, nj, blockIdx.x)];
  const Geom G = J.G;
  const uint32_t nbins = J.nbins, lb = blockIdx.x - J.blk0;
  const uint32_t t0 = threadIdx.x * TPT;
  for (uint32_t t = threadIdx.x; t < BIN_SLOTS; t += blockDim.x) h[t] = 0;
  __syncthreads();
  uint32_t acc[TPT] = {};
  // a batch's run of c codes in a tile takes ceil(c / 3) words
  auto close_batch = [&]() {
    __syncthreads();
#pragma unroll
    for (uint32_t u = 0; u < TPT; u++) {
      acc[u] += (h[t0 + u] + 2) / 3;
      h[t0 + u] = 0;
    }
    __syncthreads();
  };
  const size_t p0 = (size_t)lb * J.chunk;
  const size_t p1 = p0 + J.chunk < J.n ? p0 + J.chunk : J.n;
  const size_t step = (size_t)blockDim.x * PPT;
  const uint32_t stride = (uint32_t)step * J.sample;    // sampled batches
  const GMEM uint4 *q = gmem(reinterpret_cast<const uint4 *>(J.pairs + p0));
  const size_t nq = (p1 - p0) / 2;                      // whole uint4 of the chunk
  size_t i0 = p0;
  if constexpr (PPT % 2 == 0) {
    if (i0 + step <= p1) {                               // uniform over the block
      uint4 nxt[V4];
      // the thread index is taken afresh per load (see the scatter), so the
      // per-load offsets are recomputed rather than held across the loop
      auto load = [&](size_t b0) {                       // b0: the batch's first pair
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
#pragma unroll
        for (int k = 0; k < V4; k++) {
          const size_t i = (b0 - p0) / 2 + (size_t)k * blockDim.x + tid;
          nxt[k] = ld4(q + (i < nq ? i : nq - 1));
        }
      };
      load(i0);
      for (; i0 + step <= p1; i0 += stride) {
        uint4 cur[V4];
#pragma unroll
        for (int k = 0; k < V4; k++) cur[k] = nxt[k];
        load(i0 + stride);
#pragma unroll
        for (int k = 0; k < V4; k++) {
          count_pair<R>(G, make_uint2(cur[k].x, cur[k].y), h);
          count_pair<R>(G, make_uint2(cur[k].z, cur[k].w), h);
        }
        close_batch();
      }
    }
  } else {
    // an odd PPT: 8-byte loads, in the scatter's order
    const GMEM uint2 *pairs = gmem(J.pairs);
    if (i0 + step <= p1) {
      uint2 nxt[PPT];
      auto load = [&](size_t b0) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
#pragma unroll
        for (int k = 0; k < PPT; k++) {
          const size_t i = b0 + (size_t)k * blockDim.x + tid;
          nxt[k] = ld2(pairs + (i < p1 ? i : p1 - 1));
        }
      };
      load(i0);
      for (; i0 + step <= p1; i0 += stride) {
        uint2 cur[PPT];
#pragma unroll
        for (int k = 0; k < PPT; k++) cur[k] = nxt[k];
        load(i0 + stride);
#pragma unroll
        for (int k = 0; k < PPT; k++) count_pair<R>(G, cur[k], h);
        close_batch();
      }
    }
  }
  if (i0 < p1) {                                         // the chunk's partial batch,
    const GMEM uint2 *pairs = gmem(J.pairs);             // when it is a sampled one
#pragma unroll
    for (int k = 0; k < PPT; k++) {
      const size_t i = i0 + (size_t)k * blockDim.x + threadIdx.x;
      if (i < p1) count_pair<R>(G, ld2(pairs + i), h);
    }
    close_batch();
  }
  // sampled: scaled by the chunk's pairs over the sampled batches' pairs
  // (an estimate, in float; a chunk's last batch is partial, so a count of
  // batches would under- or overweight it); every batch: the exact count
  const size_t len = p1 > p0 ? p1 - p0 : 0, nfull = len / step, rem = len - nfull * step;
  const size_t sampled = (nfull + J.sample - 1) / J.sample * step +
                         (rem && nfull % J.sample == 0 ? rem : 0);
  const float scale = sampled ? (float)len / (float)sampled : 0.f;
  GMEM uint32_t *hist = gmem(J.hist);
#pragma unroll
  for (uint32_t u = 0; u < TPT; u++)
    if (t0 + u < nbins)
      hist[(size_t)(t0 + u) * J.hstride + lb] =
          J.sample == 1 ? acc[u] : (uint32_t)fminf((float)acc[u] * scale + 0.5f, 4.0e9f);
}

// Exclusive prefix sum over a workgroup of 1024 threads.
__device__ __forceinline__ uint32_t blk_scan_1024(uint32_t v, uint32_t *total, uint32_t *sh,
                                                  uint32_t tid = threadIdx.x) {
  const uint32_t lane = tid & 63, wid = tid >> 6;
  const uint32_t inc = wave_scan_incl(v);
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    const uint32_t x = wave_scan_incl(lane < 16 ? sh[lane] : 0);
    if (lane < 16) sh[lane] = x;
  }
  __syncthreads();
  const uint32_t off = wid ? sh[wid - 1] : 0;
  *total = sh[15];
  __syncthreads();
  return off + inc - v;
}

// Per tile: the blocks' estimates -> each block group's region capacity
// (the group's estimate plus an eighth plus a pad when sampled, exactly the
// count when not, or rscale/64 of it plus the pad when rscale is set; even,
// so that every region starts 16-byte aligned), the tile's spill-run count
// and words, and the tile's capacity.
__global__ __launch_bounds__(1024) void k_bin_scan_cols(const UpdJob *__restrict__ jobs,
                                                        uint32_t nj) {
  __shared__ uint32_t sg[BIN_GROUPS];
  const UpdJob &J = jobs[job_of_tile(jobs, nj, blockIdx.x)];
  const uint32_t t = blockIdx.x - J.tile0;
  const GMEM uint32_t *col = gmem(J.hist) + (size_t)t * J.hstride;
  if (threadIdx.x < BIN_GROUPS) sg[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t v = threadIdx.x < J.nblk ? col[threadIdx.x] : 0;
  if (v) atomicAdd(&sg[(J.blk0 + threadIdx.x) % BIN_GROUPS], v);
  __syncthreads();
  if (threadIdx.x == 0) {
    const TileState S = tile_state(J.tst, J.nbins);
    uint32_t tot = 0;
#pragma unroll
    for (uint32_t g = 0; g < BIN_GROUPS; g++) {
      const uint32_t e = sg[g];
      uint32_t cap = J.rscale ? (uint32_t)((uint64_t)e * J.rscale / 64) + BIN_REGION_PAD
                              : (J.sample > 1 ? e + e / 8 + BIN_REGION_PAD : e);
      cap += cap & 1;
      gmem(S.capg)[(size_t)g * J.nbins + t] = cap;
      tot += cap;
    }
    gmem(S.dcnt)[t] = 0;
    gmem(S.swords)[t] = 0;
    gmem(J.totals)[t] = tot;
  }
}

// Apply items of a tile with v code words: one if v <= SPLIT_MIN, else one
// per APPLY_ITEM words; none for an empty tile, unless the sketch is fresh
// (all zero and not yet written), when the tile's one item writes its zeros.
__device__ __forceinline__ uint32_t tile_items(uint32_t v, uint32_t fresh) {
  return v == 0 ? (fresh ? 1u : 0u) : (v <= SPLIT_MIN ? 1u : (v + APPLY_ITEM - 1) / APPLY_ITEM);
}

// Over one job's tiles (block = job): the regions laid out tile after tile
// (base[t] = the tile's first region; the group regions of a tile follow
// each other), scaled down to the room the job has if the estimates
// exceed it. Per region, in words from the job's codes: its start (regb),
// its end (capg, which held the capacity until here), its claim cursor
// (gcur, at the start) and its written end (fill, at the end until a run
// crosses it). The spill cursor zeroed. Thread x takes tiles x, x + 1024,
// ... (one per round of 1024 tiles), so that a wave's loads and stores of
// a group's row are consecutive words; a round's scan continues from the
// rounds before it.
__global__ __launch_bounds__(1024) void k_bin_layout(const UpdJob *__restrict__ jobs) {
  __shared__ uint32_t sh[16];
  const UpdJob &J = jobs[blockIdx.x];
  const uint32_t nbins = J.nbins;
  const TileState S = tile_state(J.tst, nbins);
  GMEM uint32_t *capg = gmem(S.capg), *fill = gmem(S.fill), *regb = gmem(S.regb);
  GMEM uint32_t *base = gmem(J.base);
  constexpr uint32_t PER = BIN_SLOTS / 1024;
  const uint32_t rounds = (nbins + 1023) / 1024;
  uint32_t cap[PER][BIN_GROUPS], mine[PER], ex[PER];
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    const uint32_t t = k * 1024 + threadIdx.x;
    mine[k] = 0;
    ex[k] = 0;
#pragma unroll
    for (uint32_t g = 0; g < BIN_GROUPS; g++) {
      cap[k][g] = t < nbins ? capg[(size_t)g * nbins + t] : 0;
      mine[k] += cap[k][g];
    }
  }
  // the job's words fit 32 bits (its code buffer is indexed so)
  uint32_t tot = 0;
  auto starts = [&]() {
    tot = 0;
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
      if (k < rounds) {                                 // uniform over the block
        uint32_t tk;
        ex[k] = tot + blk_scan_1024(mine[k], &tk, sh);
        tot += tk;
      }
    }
  };
  starts();
  if (tot > J.rcap) {                                   // uniform over the block
#pragma unroll
    for (uint32_t k = 0; k < PER; k++) {
      mine[k] = 0;
#pragma unroll
      for (uint32_t g = 0; g < BIN_GROUPS; g++) {
        const uint32_t c = (uint32_t)((uint64_t)cap[k][g] * J.rcap / tot) & ~1u;
        cap[k][g] = c;
        mine[k] += c;
      }
    }
    starts();
  }
  GMEM uint32_t *gcur = gmem(J.gcur);
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    const uint32_t t = k * 1024 + threadIdx.x;
    if (t < nbins) {
      uint32_t e = ex[k];
      base[t] = e;
#pragma unroll
      for (uint32_t g = 0; g < BIN_GROUPS; g++) {
        const size_t x = (size_t)g * nbins + t;
        regb[x] = e;
        gcur[x] = e;
        e += cap[k][g];
        capg[x] = e;
        fill[x] = e;
      }
    }
  }
  if (threadIdx.x == 0) {
    base[nbins] = tot;
    *gmem(S.spill_cur) = 0;
  }
}

// Over one job's tiles (block = job), after the scatter: the words each
// tile got (the written part of its regions and its spill runs), its apply
// items, their starts, the scratch-slot starts (a tile cut into j items
// owns j-1 scratch tiles) and the item count. Tiles map to threads as in
// the layout.
__global__ __launch_bounds__(1024) void k_bin_items(const UpdJob *__restrict__ jobs) {
  __shared__ uint32_t sh[16];
  const UpdJob &J = jobs[blockIdx.x];
  const uint32_t nbins = J.nbins;
  const TileState S = tile_state(J.tst, nbins);
  const GMEM uint32_t *gcur = gmem(J.gcur), *fill = gmem(S.fill), *swords = gmem(S.swords);
  const GMEM uint32_t *regb = gmem(S.regb);
  GMEM uint32_t *totals = gmem(J.totals), *item_start = gmem(J.item_start);
  GMEM uint32_t *xslot = gmem(J.xslot), *item_tile = gmem(J.item_tile);
  constexpr uint32_t PER = BIN_SLOTS / 1024;
  const uint32_t rounds = (nbins + 1023) / 1024;
  uint32_t v[PER];
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    const uint32_t t = k * 1024 + threadIdx.x;
    uint32_t w = 0;
    if (t < nbins) {
      w = swords[t];
#pragma unroll
      for (uint32_t g = 0; g < BIN_GROUPS; g++) {
        const size_t x = (size_t)g * nbins + t;
        const uint32_t c = gcur[x], f = fill[x];
        w += (c < f ? c : f) - regb[x];
      }
    }
    v[k] = w;
  }
  uint32_t ci = 0, cx = 0;                              // items, scratch slots so far
#pragma unroll
  for (uint32_t k = 0; k < PER; k++) {
    if (k < rounds) {                                   // uniform over the block
      const uint32_t t = k * 1024 + threadIdx.x;
      const uint32_t ni = t < nbins ? tile_items(v[k], J.fresh) : 0;
      const uint32_t xs = ni > 1 ? ni - 1 : 0;
      uint32_t ti, tx;
      const uint32_t ei = ci + blk_scan_1024(ni, &ti, sh);
      const uint32_t ex = cx + blk_scan_1024(xs, &tx, sh);
      if (t < nbins) {
        totals[t] = v[k];
        item_start[t] = ei;
        xslot[t] = ex;
        for (uint32_t q = 0; q < ni; q++) item_tile[ei + q] = t;
      }
      ci += ti;
      cx += tx;
    }
  }
  if (threadIdx.x == 0) {
    item_start[nbins] = ci;
    xslot[nbins] = cx;
    *gmem(J.n_items) = ci;
  }
}

// First global apply item of every job, and the total (one block).
__global__ __launch_bounds__(1024) void k_item_offsets(UpdJob *__restrict__ jobs, uint32_t nj,
                                                       uint32_t *__restrict__ total) {
  __shared__ uint32_t sh[16];
  const uint32_t v = threadIdx.x < nj ? *gmem(jobs[threadIdx.x].n_items) : 0;
  uint32_t tot;
  const uint32_t ex = blk_scan_1024(v, &tot, sh);
  if (threadIdx.x < nj) jobs[threadIdx.x].item0 = ex;
  if (threadIdx.x == 0) *total = tot;
}

constexpr int SCATTER_UNROLL = 4;

// Two 16-bit ranks per register (q is a compile-time index after unrolling).
__device__ __forceinline__ void put_rank(uint32_t *rk2, int q, uint32_t r) {
  if (q & 1) rk2[q >> 1] |= r << 16;
  else rk2[q >> 1] = r;
}
__device__ __forceinline__ uint32_t get_rank(const uint32_t *rk2, int q) {
  return (q & 1) ? rk2[q >> 1] >> 16 : rk2[q >> 1] & 0xFFFFu;
}

// The value the scatter keeps per bit set. Up to 2048 tiles it is the tile
// (11 bits) over the code (21 bits), split once per bit set; above, the
// sketch bit index, whose tile takes a division wherever it is needed
// (a 12-bit tile and a code do not fit 32 bits). ~0 (a slot past the
// window's end or a pad slot) is neither.
template <int TMAX> struct ScatterValue {
  static constexpr bool SPLIT = TMAX <= 2048;
  __device__ __forceinline__ static uint32_t make(uint32_t B) {
    if constexpr (SPLIT) {
      const uint32_t t = bin_tile(B);
      return (t << CODE_BITS) | (B - t * BIN_TILE_BITS);
    } else {
      return B;
    }
  }
  __device__ __forceinline__ static uint32_t tile(uint32_t v) {
    if constexpr (SPLIT) return v >> CODE_BITS;
    else return bin_tile(v);
  }
  __device__ __forceinline__ static uint32_t code(uint32_t v, uint32_t t) {
    if constexpr (SPLIT) return v & CODE_MASK;
    else return v - t * BIN_TILE_BITS;
  }
};

// TMAX: tiles the LDS arrays hold (1024, 2048, 3072 or 4096), at least the
// jobs' tiles.
template <int R, int PPT, int TMAX>
__global__ __launch_bounds__(1024) void k_bin_scatter(const UpdJob *__restrict__ jobs,
                                                      uint32_t nj) {
  constexpr uint32_t BATCH = 1024 * PPT * R;
  constexpr uint32_t TPT = TMAX / 1024;                // tiles per thread
  using SV = ScatterValue<TMAX>;
  // a batch's codes grouped by tile, each run padded to whole words (at
  // most 2 pad slots per tile); with the three tile arrays this is at most
  // 160 KiB for every (R, PPT, TMAX) the launcher picks
  __shared__ uint32_t sorted[BATCH + 2 * TMAX];
  __shared__ uint32_t cnt[TMAX];       // codes per tile in this batch
  __shared__ uint32_t lofs[TMAX];      // batch-local run starts (multiples of 3)
  __shared__ uint32_t dst[TMAX];       // word slot of batch word j is dst[t] + j
  // the block scan's 16 words: dst is not in use from the end of a batch
  // until step 3 of the next
  uint32_t *const sh = dst;
  const UpdJob &J = jobs[job_of_block(jobs, nj, blockIdx.x)];
  const Geom G = J.G;
  const uint32_t lb = blockIdx.x - J.blk0;
  const GMEM uint2 *__restrict__ pairs = gmem(J.pairs);
  GMEM uint64_t *__restrict__ words = gmem(reinterpret_cast<uint64_t *>(J.codes));
  // this block's group's regions, one per tile: claim cursors and ends (in
  // words from the job's codes)
  const size_t grow = (size_t)(blockIdx.x % BIN_GROUPS) * J.nbins;
  const TileState TS = tile_state(J.tst, J.nbins);
  GMEM uint32_t *gcur = gmem(J.gcur) + grow;
  const GMEM uint32_t *rend = gmem(TS.capg) + grow;
  for (uint32_t t = threadIdx.x; t < TMAX; t += blockDim.x) cnt[t] = 0;
  __syncthreads();
  const size_t p0 = (size_t)lb * J.chunk;
  const size_t p1 = p0 + J.chunk < J.n ? p0 + J.chunk : J.n;
  if (p0 >= p1) return;                                // uniform over the block
  const size_t step = (size_t)blockDim.x * PPT;
  // A batch's pairs are held in pr. The next batch's pairs are loaded into
  // pr as soon as this batch's codes are made (step 1), so they are in
  // flight through the claims and the scan (and, with one tile per thread,
  // the grouping: the first wait that covers them is the one for the
  // claims, see step 2), and no second set of registers is live. Loads past
  // the chunk re-read its last pair (their lanes are masked later): with no
  // branch around them the compiler need not wait for every load in flight.
  uint2 pr[PPT];
  auto load = [&](size_t b0, uint32_t tid) {
#pragma unroll
    for (int k = 0; k < PPT; k++) {
      const size_t i = b0 + (size_t)k * blockDim.x + tid;
      pr[k] = ld2(pairs + (i < p1 ? i : p1 - 1));
    }
  };
  // One batch: the pairs [i0, i0 + step) of the chunk, held in pr. A full
  // batch (FULL) has all its pairs and takes no per-pair bounds test; only
  // a chunk's last batch can be partial, and its missing pairs get the
  // code ~0.
  auto batch = [&](auto full_c, size_t i0) {
    constexpr bool FULL = decltype(full_c)::value;
    // The thread index is taken afresh per batch, so that addresses derived
    // from it are recomputed here rather than held in registers (or spilled)
    // across the batch loop.
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const uint32_t t0 = tid * TPT;                      // tiles this thread keeps
    // ranks are < BATCH <= 2^15: two per register
    uint32_t v[PPT * R], rk2[(PPT * R + 1) / 2];
    // 1: codes and their rank inside their tile's run of this batch (an
    // LDS atomic that returns the rank; a plain count here and a returning
    // placement cursor in step 3 instead was slower: 692 against 608 us
    // for the 100M-pair window)
#pragma unroll
    for (int k = 0; k < PPT; k++) {
      const size_t i = i0 + (size_t)k * blockDim.x + tid;
      if (FULL || i < p1) {
        uint32_t B[R];
        pair_codes<R>(G, pr[k], B);
#pragma unroll
        for (int row = 0; row < R; row++) {
          v[k * R + row] = SV::make(B[row]);
          put_rank(rk2, k * R + row, atomicAdd(&cnt[SV::tile(v[k * R + row])], 1u));
        }
      } else {
#pragma unroll
        for (int row = 0; row < R; row++) v[k * R + row] = ~0u;
      }
    }
    load(i0 + step, tid);
    __syncthreads();
    // 2: claim each tile's run, ceil(c / 3) words, in the group's region,
    // and read the region's end; run starts; the pad slots of each run get
    // the marker ~0. The counts stay in cnt. With one tile per thread the
    // claimed start stays in a register until after the grouping, so the
    // wait for the atomic's return (and, the counter being in order, for
    // the next batch's pairs) falls behind the scan and step 3, not before
    // them; with more tiles per thread the claimed positions wait in dst
    // (the scan is done with it): held in registers through the grouping
    // they would not fit the 6-pair, 5-row variant
    uint32_t run[TPT], end[TPT], sum = 0;
#pragma unroll
    for (uint32_t u = 0; u < TPT; u++) {
      const uint32_t w = (cnt[t0 + u] + 2) / 3;       // 0 for the slots past the tiles
      sum += 3 * w;
      run[u] = w ? atomicAdd((uint32_t *)&gcur[t0 + u], w) : 0;
      end[u] = w ? rend[t0 + u] : 0;
    }
    uint32_t total;
    uint32_t ex = blk_scan_1024(sum, &total, sh, tid);
#pragma unroll
    for (uint32_t u = 0; u < TPT; u++) {
      const uint32_t t = t0 + u, c = cnt[t], padded = 3 * ((c + 2) / 3);
      lofs[t] = ex;
      if constexpr (TPT > 1) dst[t] = run[u];
      if (padded > c) sorted[ex + c] = ~0u;             // at most two pad slots
      if (padded > c + 1) sorted[ex + c + 1] = ~0u;
      ex += padded;
    }
    __syncthreads();
    // 3: group by tile in LDS; dst maps a batch word to its word slot
#pragma unroll
    for (int q = 0; q < PPT * R; q++)
      if (FULL || v[q] != ~0u) sorted[lofs[SV::tile(v[q])] + get_rank(rk2, q)] = v[q];
    // a run that fits its region goes there; one that does not goes whole
    // to the spill area (the run that crosses the region's end marks where
    // the region's written part ends) and joins its tile's spill runs
#pragma unroll
    for (uint32_t u = 0; u < TPT; u++) {
      const uint32_t t = t0 + u;
      const uint32_t w = (cnt[t] + 2) / 3;
      cnt[t] = 0;                                       // for the next batch
      if (!w) continue;
      const uint32_t pos = TPT > 1 ? dst[t] : run[u];
      uint32_t at = pos;
      if (pos + w > end[u]) {
        if (pos < end[u]) gmem(TS.fill)[grow + t] = pos;
        const uint32_t so = atomicAdd((uint32_t *)TS.spill_cur, w);
        const uint32_t d = atomicAdd((uint32_t *)&TS.dcnt[t], 1u);
        J.desc[(size_t)t * J.dmax + d] = make_uint2(so, w);
        atomicAdd((uint32_t *)&TS.swords[t], w);
        at = (uint32_t)J.rcap + so;
      }
      dst[t] = at - lofs[t] / 3;
    }
    __syncthreads();
    // 4: write the words; batch word j holds sorted slots 3j..3j+2, whose
    // first is always a code of the run and stands in for a pad (a code
    // set twice sets the same bit)
    const uint32_t nw = total / 3;
    auto put = [&](uint32_t j) {
      const uint32_t x = sorted[3 * j], y0 = sorted[3 * j + 1], z0 = sorted[3 * j + 2];
      const uint32_t y = y0 == ~0u ? x : y0, z = z0 == ~0u ? x : z0;
      const uint32_t t = SV::tile(x);                   // the word's three share it
      const uint64_t wv = (uint64_t)SV::code(x, t) | ((uint64_t)SV::code(y, t) << CODE_BITS) |
                          ((uint64_t)SV::code(z, t) << (2 * CODE_BITS));
      words[dst[t] + j] = wv;
    };
    uint32_t j = tid;
    for (; j + (SCATTER_UNROLL - 1) * 1024 < nw; j += SCATTER_UNROLL * 1024) {
#pragma unroll
      for (int u = 0; u < SCATTER_UNROLL; u++) put(j + u * 1024);
    }
    for (; j < nw; j += 1024) put(j);
    __syncthreads();
  };
  load(p0, threadIdx.x);
  size_t i0 = p0;
  for (; i0 + step <= p1; i0 += step) batch(std::true_type{}, i0);
  if (i0 < p1) batch(std::false_type{}, i0);
}

constexpr int APPLY_UNROLL = 4;

// Zero count of the LE that holds sketch words [w, w+4) (v), when the LE's
// W = wpl words are spread over W/4 consecutive lanes, each with one 16-byte
// vector (4 <= W <= 256): the lanes' one-counts are summed across the group
// and its first lane writes g - ones. Every lane of a group must call it.
__device__ __forceinline__ void le_zeros(const Geom &G, GMEM uint32_t *lez, size_t w, uint4 v) {
  const uint32_t L = G.wpl / 4;                         // lanes per LE, 1..64
  uint32_t ones = __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
  for (uint32_t m = L >> 1; m >= 1; m >>= 1) ones += __shfl_xor(ones, (int)m, 64);
  if ((w / 4) % L == 0) lez[w / G.wpl] = G.g - ones;
}

// The three codes of a word (low half lo, high half hi) into the LDS tile.
__device__ __forceinline__ void or_word(uint32_t *tile, uint2 w) {
  const uint32_t a = w.x & CODE_MASK;
  const uint32_t b = __builtin_amdgcn_alignbit(w.y, w.x, CODE_BITS) & CODE_MASK;
  const uint32_t c = (w.y >> (2 * CODE_BITS - 32)) & CODE_MASK;
  atomicOr(&tile[a >> 5], 1u << (a & 31));
  atomicOr(&tile[b >> 5], 1u << (b & 31));
  atomicOr(&tile[c >> 5], 1u << (c & 31));
}

// The code words [c0, c1) of one region or spill run into the LDS tile: a
// single word up to an even index, uint4 bodies (two words each; whole
// rounds of APPLY_UNROLL per thread with no bounds test, then one at a
// time), a single word at the end.
__device__ __forceinline__ void apply_words(uint32_t *tile, const GMEM uint2 *__restrict__ codes,
                                            uint32_t c0, uint32_t c1) {
  const uint32_t a0 = (c0 & 1) && c0 < c1 ? c0 + 1 : c0;
  const uint32_t a1 = a0 + ((c1 - a0) & ~1u);
  if (threadIdx.x == 0 && a0 != c0) or_word(tile, ld2(codes + c0));
  if (threadIdx.x == 0 && a1 != c1) or_word(tile, ld2(codes + a1));
  const GMEM uint4 *q = reinterpret_cast<const GMEM uint4 *>(codes + a0);
  const uint32_t nq = (a1 - a0) / 2;
  uint32_t i = threadIdx.x;
  for (; i + (APPLY_UNROLL - 1) * blockDim.x < nq; i += blockDim.x * APPLY_UNROLL) {
    uint4 x[APPLY_UNROLL];
#pragma unroll
    for (int u = 0; u < APPLY_UNROLL; u++) x[u] = ld4(q + i + u * blockDim.x);
#pragma unroll
    for (int u = 0; u < APPLY_UNROLL; u++) {
      or_word(tile, make_uint2(x[u].x, x[u].y));
      or_word(tile, make_uint2(x[u].z, x[u].w));
    }
  }
  for (; i < nq; i += blockDim.x) {
    const uint4 x = ld4(q + i);
    or_word(tile, make_uint2(x.x, x.y));
    or_word(tile, make_uint2(x.z, x.w));
  }
}

__global__ __launch_bounds__(1024) void k_bin_apply(const UpdJob *__restrict__ jobs, uint32_t nj,
                                                    const uint32_t *__restrict__ n_items_p) {
  __shared__ __attribute__((aligned(16))) uint32_t tile[BIN_TILE_WORDS];
  constexpr uint32_t TV4 = BIN_TILE_WORDS / 4 / 1024;      // uint4 per thread per tile
  uint4 *tile4 = reinterpret_cast<uint4 *>(tile);
  const uint32_t n_items = *n_items_p;
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const UpdJob &J = jobs[job_of_item(jobs, nj, it)];
    const uint32_t jit = it - J.item0;
    const GMEM uint32_t *item_start = gmem(J.item_start);
    const uint32_t t = gmem(J.item_tile)[jit];                // tile of this item
    const uint32_t sub = jit - item_start[t];
    const bool whole = item_start[t + 1] - item_start[t] == 1;
    // this item's words of the tile's code stream: its regions in group
    // order, then its spill runs
    const uint32_t v_end = gmem(J.totals)[t];
    const uint32_t v0 = whole ? 0 : sub * APPLY_ITEM;
    const uint32_t v1 = whole ? v_end : (v_end - v0 > APPLY_ITEM ? v0 + APPLY_ITEM : v_end);
    const size_t w0 = (size_t)t * BIN_TILE_WORDS;
    const uint32_t tw = (uint32_t)(J.words - w0 < BIN_TILE_WORDS ? J.words - w0 : BIN_TILE_WORDS);
    const GMEM uint2 *__restrict__ codes = gmem(reinterpret_cast<const uint2 *>(J.codes));
    // the first item of a tile owns the tile; item s >= 1 of a cut tile
    // writes scratch tile xslot[t] + s - 1
    GMEM uint32_t *dstp =
        sub == 0 ? gmem(J.sk) + w0
                 : gmem(J.scratch) + (size_t)(gmem(J.xslot)[t] + sub - 1) * BIN_TILE_WORDS;
    // the tile in: zeros for a scratch tile or a fresh sketch, else a whole
    // tile as 16-byte loads, all in flight before the LDS writes (tiles and
    // scratch tiles are 160 KiB aligned)
    if (sub != 0 || J.fresh) {
      for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) tile[w] = 0;
    } else if (tw == BIN_TILE_WORDS) {
      const GMEM uint4 *src = reinterpret_cast<const GMEM uint4 *>(dstp);
      uint4 v[TV4];
#pragma unroll
      for (uint32_t u = 0; u < TV4; u++) v[u] = ld4(src + threadIdx.x + u * 1024);
#pragma unroll
      for (uint32_t u = 0; u < TV4; u++) tile4[threadIdx.x + u * 1024] = v[u];
    } else {
      for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) tile[w] = dstp[w];
    }
    __syncthreads();
    {
      const TileState S = tile_state(J.tst, J.nbins);
      const uint32_t nd = gmem(S.dcnt)[t];
      uint32_t vo = 0;                                  // stream offset of the segment
      for (uint32_t sg = 0; sg < BIN_GROUPS + nd && vo < v1; sg++) {
        uint32_t off, len;
        if (sg < BIN_GROUPS) {
          const size_t x = (size_t)sg * J.nbins + t;
          const uint32_t c = gmem(J.gcur)[x], f = gmem(S.fill)[x];
          off = gmem(S.regb)[x];
          len = (c < f ? c : f) - off;
        } else {
          const uint2 d = ld2(gmem(J.desc) + (size_t)t * J.dmax + (sg - BIN_GROUPS));
          off = (uint32_t)J.rcap + d.x;
          len = d.y;
        }
        const uint32_t a = v0 > vo ? v0 : vo, b = v1 < vo + len ? v1 : vo + len;
        if (a < b) apply_words(tile, codes, off + (a - vo), off + (b - vo));
        vo += len;
      }
    }
    __syncthreads();
    // a tile with one item is final here: its LEs' zero counts go out too
    // (a cut tile's are counted by the merge)
    GMEM uint32_t *lez = whole && J.lez ? gmem(J.lez) : nullptr;
    if (tw == BIN_TILE_WORDS) {
      GMEM uint4 *d4 = reinterpret_cast<GMEM uint4 *>(dstp);
      uint4 v[TV4];
#pragma unroll
      for (uint32_t u = 0; u < TV4; u++) v[u] = tile4[threadIdx.x + u * 1024];
#pragma unroll
      for (uint32_t u = 0; u < TV4; u++) st4(d4 + threadIdx.x + u * 1024, v[u]);
      if (lez) {
#pragma unroll
        for (uint32_t u = 0; u < TV4; u++)
          le_zeros(J.G, lez, w0 + 4 * (size_t)(threadIdx.x + u * 1024), v[u]);
      }
    } else {
      for (uint32_t w = threadIdx.x; w < tw; w += blockDim.x) dstp[w] = tile[w];
      if (lez) {                                         // the sketch's last, partial tile
        const uint32_t W = J.G.wpl;
        for (uint32_t e = threadIdx.x; e < tw / W; e += blockDim.x) {
          uint32_t ones = 0;
          for (uint32_t w = 0; w < W; w++) ones += __popc(tile[e * W + w]);
          lez[(w0 + (size_t)e * W) / W] = J.G.g - ones;
        }
      }
    }
    __syncthreads();
  }
}

// OR the scratch tiles of every cut tile into the sketch: block (t, y)
// takes the y-th MERGE_SLICE-word slice of global tile t.
constexpr uint32_t MERGE_SLICE = 2048;
constexpr uint32_t MERGE_BATCH = 8;

__global__ __launch_bounds__(256) void k_bin_merge(const UpdJob *__restrict__ jobs, uint32_t nj) {
  const UpdJob &J = jobs[job_of_tile(jobs, nj, blockIdx.x)];
  const uint32_t t = blockIdx.x - J.tile0;
  const GMEM uint32_t *item_start = gmem(J.item_start);
  const uint32_t n = item_start[t + 1] - item_start[t];
  if (n <= 1) return;
  const size_t w0 = (size_t)t * BIN_TILE_WORDS;
  const uint32_t tw = (uint32_t)(J.words - w0 < BIN_TILE_WORDS ? J.words - w0 : BIN_TILE_WORDS);
  const uint32_t s_lo = blockIdx.y * MERGE_SLICE;
  const uint32_t s_hi = s_lo + MERGE_SLICE < tw ? s_lo + MERGE_SLICE : tw;
  const GMEM uint32_t *s0 = gmem(J.scratch) + (size_t)gmem(J.xslot)[t] * BIN_TILE_WORDS;
  GMEM uint32_t *sk = gmem(J.sk) + w0;
  // a slice is a whole number of LEs when the zero counts are kept (an LE
  // of at most 256 words), so a lane group never straddles its end
  GMEM uint32_t *lez = J.lez ? gmem(J.lez) : nullptr;
  for (uint32_t w = s_lo + threadIdx.x * 4; w < s_hi; w += blockDim.x * 4) {
    if (w + 4 <= s_hi) {
      uint4 v = ld4(reinterpret_cast<const GMEM uint4 *>(sk + w));
      // MERGE_BATCH scratch tiles' loads in flight at once; past the last
      // one they re-read it, which ORs in bits already there
      for (uint32_t k0 = 1; k0 < n; k0 += MERGE_BATCH) {
        uint4 x[MERGE_BATCH];
#pragma unroll
        for (uint32_t u = 0; u < MERGE_BATCH; u++) {
          const uint32_t k = k0 + u < n ? k0 + u : n - 1;
          x[u] = ld4(reinterpret_cast<const GMEM uint4 *>(s0 + (size_t)(k - 1) * BIN_TILE_WORDS + w));
        }
#pragma unroll
        for (uint32_t u = 0; u < MERGE_BATCH; u++) {
          v.x |= x[u].x; v.y |= x[u].y; v.z |= x[u].z; v.w |= x[u].w;
        }
      }
      st4(reinterpret_cast<GMEM uint4 *>(sk + w), v);
      if (lez) le_zeros(J.G, lez, w0 + w, v);
    } else {
      for (uint32_t ww = w; ww < s_hi; ww++) {
        uint32_t v = sk[ww];
        for (uint32_t k = 1; k < n; k++) v |= s0[(size_t)(k - 1) * BIN_TILE_WORDS + ww];
        sk[ww] = v;
      }
    }
  }
}

// ---------------------------------------------------------------- launch

// count, the region layout, the scatter and the apply items of a binned round
template <int R, int PPT, int TMAX>
static void launch_front(UpdJob *d, uint32_t nj, uint32_t blocks, uint32_t tiles,
                         hipStream_t st) {
  k_bin_count<R, PPT><<<blocks, 1024, 0, st>>>(d, nj);
  k_bin_scan_cols<<<tiles, 1024, 0, st>>>(d, nj);
  k_bin_layout<<<nj, 1024, 0, st>>>(d);
  k_bin_scatter<R, PPT, TMAX><<<blocks, 1024, 0, st>>>(d, nj);
  k_bin_items<<<nj, 1024, 0, st>>>(d);
}

template <int R>
static hipError_t launch_r(const UpdJob *h, UpdJob *d, uint32_t nj, uint32_t *d_total,
                           bool binned, uint32_t ppt, uint32_t apply_grid, hipStream_t st) {
  uint32_t blocks = 0, tiles = 0;
  for (uint32_t j = 0; j < nj; j++) {
    blocks += h[j].nblk;
    tiles += h[j].nbins;
  }
  if (!binned) {
    bool check = h[0].check != 0;
    if (check) k_update<R, true><<<blocks, 256, 0, st>>>(d, nj);
    else k_update<R, false><<<blocks, 256, 0, st>>>(d, nj);
    return hipGetLastError();
  }
  // LDS of the scatter: 4*(1024*PPT*r + 2*TMAX) bytes of sorted codes +
  // 12*TMAX bytes of tile arrays <= 160 KiB. Up to 2048 tiles: 6 pairs per
  // thread for r <= 5, 4 for r <= 7, else 2; the 6-pair variant has a copy
  // with arrays of 1024 tiles (a k = 18 sketch at r = 5), one tile per
  // thread in the per-batch tile steps. Up to 3072 tiles and r <= 5: 5.
  // Up to 3276 tiles: 4 for r <= 5, else 2 (scatter_ppt gives the same
  // choice to the host, which sizes the spill-run lists by it). The count
  // pass walks the scatter's batches, so both take the same PPT.
  uint32_t max_tiles = 0;
  for (uint32_t j = 0; j < nj; j++) max_tiles = max_tiles > h[j].nbins ? max_tiles : h[j].nbins;
  if (max_tiles <= 2048) {
    constexpr int P4 = R <= 7 ? 4 : 2;
    constexpr int P6 = R <= 5 ? 6 : P4;
    if (ppt == 2) launch_front<R, 2, 2048>(d, nj, blocks, tiles, st);
    else if (ppt == 6 && max_tiles <= 1024) launch_front<R, P6, 1024>(d, nj, blocks, tiles, st);
    else if (ppt == 6) launch_front<R, P6, 2048>(d, nj, blocks, tiles, st);
    else launch_front<R, P4, 2048>(d, nj, blocks, tiles, st);
  } else if (R <= 5 && max_tiles <= 3072 && ppt != 2) {
    if constexpr (R <= 5) launch_front<R, 5, 3072>(d, nj, blocks, tiles, st);
  } else {
    constexpr int P4 = R <= 5 ? 4 : 2;
    if (ppt == 2) launch_front<R, 2, 4096>(d, nj, blocks, tiles, st);
    else launch_front<R, P4, 4096>(d, nj, blocks, tiles, st);
  }
  k_item_offsets<<<1, 1024, 0, st>>>(d, nj, d_total);
  // apply_grid 0: one workgroup per apply item (an upper bound of the
  // items: a tile with v code words makes at most 1 + v / APPLY_ITEM of
  // them), so the dispatcher hands items to compute units as they free up
  uint64_t grid = apply_grid;
  if (grid == 0)
    for (uint32_t j = 0; j < nj; j++)
      grid += h[j].nbins +
              code_words_bound(h[j].n, R, h[j].nbins, h[j].nblk, h[j].chunk) / APPLY_ITEM + 1;
  if (grid > 0x7FFFFFFFull) grid = 0x7FFFFFFFull;
  k_bin_apply<<<(uint32_t)grid, 1024, 0, st>>>(d, nj, d_total);
  k_bin_merge<<<dim3(tiles, BIN_TILE_WORDS / MERGE_SLICE), 256, 0, st>>>(d, nj);
  return hipGetLastError();
}

hipError_t launch_update_jobs(const UpdJob *h_jobs, UpdJob *d_jobs, uint32_t n_jobs,
                              uint32_t *d_total, bool binned, uint32_t r, uint32_t ppt,
                              uint32_t apply_grid, hipStream_t st) {
  if (n_jobs == 0) return hipSuccess;
  switch (r) {
    case 3: return launch_r<3>(h_jobs, d_jobs, n_jobs, d_total, binned, ppt, apply_grid, st);
    case 4: return launch_r<4>(h_jobs, d_jobs, n_jobs, d_total, binned, ppt, apply_grid, st);
    case 5: return launch_r<5>(h_jobs, d_jobs, n_jobs, d_total, binned, ppt, apply_grid, st);
    case 6: return launch_r<6>(h_jobs, d_jobs, n_jobs, d_total, binned, ppt, apply_grid, st);
    case 7: return launch_r<7>(h_jobs, d_jobs, n_jobs, d_total, binned, ppt, apply_grid, st);
    case 8: return launch_r<8>(h_jobs, d_jobs, n_jobs, d_total, binned, ppt, apply_grid, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ddhf

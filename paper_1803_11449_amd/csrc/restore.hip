// Window-end restore (Alg. 2, Sec. 3.3, laid out as in Sec. 4.2).
//
//  1 hot scan      one read of the whole sketch: z0 = g - popcount of every
//                  LE, ZR(i) per row, and a bitmap of hot LEs (z0 <= zhot,
//                  i.e. z0 < Zmin = g*exp(-theta/g)). HBM-bound.
//  2 HE compaction one workgroup per row turns the hot bitmap into HE(i),
//                  ascending, by a block prefix sum.
//  3 buckets       rows >= 2: HE(i) grouped by its low k-alpha bits, so a
//                  join probe finds exactly the entries whose overlap bits
//                  match instead of testing all of HE(i) (Algs. 3-4 test
//                  every tuple; the bucketed probe enumerates the same
//                  accepted tuples and skips only failing ones).
//  4 scalars       psi (Lemma 1 with the flow-count estimate of Sec. 3.3),
//                  D = g(1 - psi^r) (eq. (4)), T_rep = D*exp(-theta/g) and
//                  the integer report bound floor(T_rep), in float64.
//  5 candidates   the addresses whose r LEs are all hot, by one of two
//                  searches, chosen on the device from the hot-list sizes
//                  by their estimated work:
//                  join     stage 1 (Alg. 3) over HE(0) x HE(1) probing row
//                           2; stages 3..r-1 (Alg. 4) over the partial
//                           addresses probing row i. Each stage appends its
//                           outputs with one atomic per wave; counts are
//                           exact even past a buffer's capacity so the host
//                           can grow it and run again. The last stage keeps
//                           a rebuilt address only if it fits 32 bits and
//                           DH0 of it is the CL_0 it was built from.
//                  lattice  every address of every hot row-0 cell, found as
//                           the points of a lattice in a box (see Lattice),
//                           tested against the hot bitmaps of rows 1..r-1:
//                           eq. (2) read forwards, no partial addresses.
//  6 estimate      per candidate, AND of its r LEs (ULE), SZ = g - popcount,
//                  report iff SZ <= floor(T_rep) (<=> C >= theta),
//                  C = -g*ln(SZ/D) (eq. (4)), +inf when SZ = 0.
//  7 sort          reported records ascending by address.
#include <math.h>

#include "ddhf_internal.h"

namespace ddhf {

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) { return wave_scan_incl(v); }

// Reserve `nout` consecutive slots of a global list for this lane, with one
// atomic per wave. Must be called by all 64 lanes of the wave.
__device__ __forceinline__ unsigned long long wave_reserve(
    unsigned long long *counter, uint32_t nout) {
  const uint32_t incl = wave_incl_scan(nout);
  const uint32_t total = wave_lane(incl, 63);
  unsigned long long base = 0;
  if (lane_id() == 63 && total) base = atomicAdd(counter, (unsigned long long)total);
  base = wave_lane64(base, 63);
  return base + (incl - nout);
}

// Exclusive prefix sum over a workgroup of NT threads (NT a multiple of 64).
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total,
                                                    uint32_t *sh) {
  constexpr int NW = NT / 64;
  const uint32_t lane = lane_id(), wid = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) sh[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    uint32_t s = lane < NW ? sh[lane] : 0;
    s = wave_incl_scan(s);
    if (lane < NW) sh[lane] = s;
  }
  __syncthreads();
  const uint32_t off = wid ? sh[wid - 1] : 0;
  *total = sh[NW - 1];
  __syncthreads();
  return off + inc - v;
}

// The most rows a sketch has.
constexpr uint32_t R_MAX = 8;

// How lanes share one LE of WPL words: LPL lanes, each reading VPL uint4.
template <int WPL>
struct LeShape {
  static constexpr int V4 = WPL >= 4 ? WPL / 4 : 0;
  static constexpr int LPL = WPL >= 4 ? (V4 < 64 ? V4 : 64) : 1;
  static constexpr int VPL = WPL >= 4 ? V4 / LPL : 0;
};

// LDS arrays handed to a device function keep their address space (a plain
// pointer would make every access a flat one).
#define LDSP __attribute__((address_space(3)))
template <typename T>
__device__ __forceinline__ LDSP T *lds_ptr(T *p) {
  return (LDSP T *)p;
}

// ----------------------------------------------------------- 0: state init

// The device state, the sort ranks and the hot bitmap back to zero, in one
// launch.
__global__ __launch_bounds__(256) void k_restore_init(DevState *st, uint32_t *rank,
                                                      uint32_t n_rank, uint32_t *hotmask,
                                                      size_t n_hm) {
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  if (blockIdx.x == 0) {
    uint32_t *p = reinterpret_cast<uint32_t *>(st);
    for (uint32_t i = threadIdx.x; i < sizeof(DevState) / 4; i += blockDim.x) p[i] = 0;
  }
  for (size_t i = i0; i < n_rank; i += stride) rank[i] = 0;
  for (size_t i = i0; i < n_hm; i += stride) hotmask[i] = 0;
}

// -------------------------------------------------------------- 1: hot scan

// Each block scans a contiguous run of `chunk` LEs; a pass covers
// 256/LPL LEs and HS_UNROLL passes are loaded before any is reduced, so every
// lane keeps several 16-byte loads in flight. ZR(i) is summed in registers
// and folded into LDS only when a lane's run crosses into the next row.
constexpr int HS_UNROLL = 4;

template <int WPL>
__global__ __launch_bounds__(256) void k_hot_scan(Geom G, const uint32_t *__restrict__ sk,
                                                  uint32_t zhot,
                                                  uint32_t *__restrict__ hotmask,
                                                  DevState *__restrict__ st, uint64_t chunk) {
  using S = LeShape<WPL>;
  constexpr uint32_t GROUPS = 256 / S::LPL;
  __shared__ unsigned long long zr_sh[8];
  if (threadIdx.x < 8) zr_sh[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t n_le = (uint64_t)G.r << G.k;
  const uint64_t e_begin = (uint64_t)blockIdx.x * chunk;
  const uint64_t e_end = e_begin + chunk < n_le ? e_begin + chunk : n_le;
  const uint32_t grp = threadIdx.x / S::LPL, sub = threadIdx.x % S::LPL;
  uint32_t cur_row = (uint32_t)(e_begin >> G.k);
  unsigned long long acc = 0;
  for (uint64_t e0 = e_begin; e0 < e_end; e0 += (uint64_t)GROUPS * HS_UNROLL) {
    uint32_t ones[HS_UNROLL];
#pragma unroll
    for (int u = 0; u < HS_UNROLL; u++) {
      const uint64_t e = e0 + (uint64_t)u * GROUPS + grp;
      ones[u] = 0;
      if (e < e_end) {
        if constexpr (WPL >= 4) {
          const uint4 *le = reinterpret_cast<const uint4 *>(sk + e * WPL);
#pragma unroll
          for (int v = 0; v < S::VPL; v++) {
            const uint4 q = le[v * S::LPL + sub];
            ones[u] += __popc(q.x) + __popc(q.y) + __popc(q.z) + __popc(q.w);
          }
        } else {
#pragma unroll
          for (int w = 0; w < WPL; w++) ones[u] += __popc(sk[e * WPL + w]);
        }
      }
    }
    if constexpr (S::LPL > 1) {
#pragma unroll
      for (int u = 0; u < HS_UNROLL; u++)
#pragma unroll
        for (int m = S::LPL / 2; m >= 1; m >>= 1) ones[u] += __shfl_xor(ones[u], m, 64);
    }
    if (sub == 0) {
#pragma unroll
      for (int u = 0; u < HS_UNROLL; u++) {
        const uint64_t e = e0 + (uint64_t)u * GROUPS + grp;
        if (e >= e_end) continue;
        const uint32_t z0 = G.g - ones[u];
        const uint32_t row = (uint32_t)(e >> G.k);
        if (row != cur_row) {
          if (acc) atomicAdd(&zr_sh[cur_row], acc);
          acc = 0;
          cur_row = row;
        }
        acc += z0;
        if (z0 <= zhot) atomicOr(&hotmask[e >> 5], 1u << (e & 31));
      }
    }
  }
  if (sub == 0 && acc) atomicAdd(&zr_sh[cur_row], acc);
  __syncthreads();
  if (threadIdx.x < G.r && zr_sh[threadIdx.x])
    atomicAdd(&st->zr[threadIdx.x], zr_sh[threadIdx.x]);
}

// The same from the zero counts the binned update kept (one word per LE, 4
// bytes instead of g/8 per LE read). A lane takes 4 consecutive LEs with
// one 16-byte load; 8 lanes make one word of the hot bitmap (their nibbles
// ORed across the group), so every word is written once, with no atomics.
// Rows start at multiples of 2^k >= 32 LEs, so a lane's 4 LEs share a row.
constexpr int HS_LEZ_UNROLL = 4;

__global__ __launch_bounds__(256) void k_hot_scan_lez(Geom G, const uint4 *__restrict__ lez4,
                                                      uint32_t zhot,
                                                      uint32_t *__restrict__ hotmask,
                                                      DevState *__restrict__ st) {
  __shared__ unsigned long long zr_sh[8];
  if (threadIdx.x < 8) zr_sh[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t n_q = ((uint64_t)G.r << G.k) / 4;      // n_le is a multiple of 32
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint32_t cur_row = 0;
  unsigned long long acc = 0;
  // HS_LEZ_UNROLL loads per lane are issued before any is used; n_q is a
  // multiple of 8, so a group of 8 lanes is whole or absent
  for (uint64_t q0 = (uint64_t)blockIdx.x * blockDim.x * HS_LEZ_UNROLL + threadIdx.x; q0 < n_q;
       q0 += stride * HS_LEZ_UNROLL) {
    uint4 z[HS_LEZ_UNROLL];
#pragma unroll
    for (int u = 0; u < HS_LEZ_UNROLL; u++) {
      const uint64_t q = q0 + (uint64_t)u * blockDim.x;
      z[u] = q < n_q ? lez4[q] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < HS_LEZ_UNROLL; u++) {
      const uint64_t q = q0 + (uint64_t)u * blockDim.x;
      if (q >= n_q) break;
      uint32_t nib = (z[u].x <= zhot ? 1u : 0u) | (z[u].y <= zhot ? 2u : 0u) |
                     (z[u].z <= zhot ? 4u : 0u) | (z[u].w <= zhot ? 8u : 0u);
      nib <<= 4 * (lane & 7);
      nib |= __shfl_xor(nib, 1, 64);
      nib |= __shfl_xor(nib, 2, 64);
      nib |= __shfl_xor(nib, 4, 64);
      if ((lane & 7) == 0) hotmask[q >> 3] = nib;
      const uint32_t row = (uint32_t)((q * 4) >> G.k);
      if (row != cur_row) {
        if (acc) atomicAdd(&zr_sh[cur_row], acc);
        acc = 0;
        cur_row = row;
      }
      acc += (unsigned long long)z[u].x + z[u].y + z[u].z + z[u].w;
    }
  }
  // a lane's sum is below 2^22 (at most 2 passes of HS_LEZ_UNROLL x 4 LEs of
  // <= 2^16 zeros), a wave's below 2^28: a wave whose lanes share a row
  // folds its sum in registers and adds it once
  const uint32_t row0 = __builtin_amdgcn_readfirstlane(cur_row);
  if (__all(cur_row == row0)) {
    const uint32_t tot = wave_scan_incl((uint32_t)acc);
    if (lane == 63 && tot) atomicAdd(&zr_sh[row0], (unsigned long long)tot);
  } else if (acc) {
    atomicAdd(&zr_sh[cur_row], acc);
  }
  __syncthreads();
  if (threadIdx.x < G.r && zr_sh[threadIdx.x])
    atomicAdd(&st->zr[threadIdx.x], zr_sh[threadIdx.x]);
}

// ---------------------------------------------------------- 2: HE compaction

// Per-thread values k_rows keeps in registers: hot-mask words (all of a
// row's when 2^k / 32 <= 8 * 1024, i.e. k <= 18) and HE entries (all when
// |HE(i)| <= 8192). Loaded together, they cost one memory latency instead
// of one per loop trip; larger rows take the loops.
constexpr uint32_t ROW_REG = 8;

__device__ __forceinline__ void compact_row(const Geom &G, uint32_t row,
                                            const uint32_t *__restrict__ hotmask,
                                            uint32_t *__restrict__ he,
                                            DevState *__restrict__ st, uint32_t *sh) {
  const uint32_t nw = (1u << G.k) >> 5;
  const uint32_t *hm = hotmask + (size_t)row * nw;
  const uint32_t per = (nw + blockDim.x - 1) / blockDim.x;
  const uint32_t w0 = min(threadIdx.x * per, nw), w1 = min(w0 + per, nw);
  uint32_t total;
  if (per <= ROW_REG) {                                // uniform: k <= 18
    // the thread's words, loaded together and kept for the write pass
    uint32_t m[ROW_REG], cnt = 0;
#pragma unroll
    for (uint32_t u = 0; u < ROW_REG; u++) {
      m[u] = w0 + u < w1 ? hm[w0 + u] : 0u;
      cnt += __popc(m[u]);
    }
    const uint32_t excl = block_excl_scan<1024>(cnt, &total, sh);
    uint32_t *out = he + ((size_t)row << G.k) + excl;
#pragma unroll
    for (uint32_t u = 0; u < ROW_REG; u++) {
      while (m[u]) {
        const uint32_t b = __ffs(m[u]) - 1;
        *out++ = ((w0 + u) << 5) | b;
        m[u] &= m[u] - 1;
      }
    }
  } else {
    uint32_t cnt = 0;
    for (uint32_t w = w0; w < w1; w++) cnt += __popc(hm[w]);
    const uint32_t excl = block_excl_scan<1024>(cnt, &total, sh);
    uint32_t *out = he + ((size_t)row << G.k) + excl;
    for (uint32_t w = w0; w < w1; w++) {
      uint32_t m = hm[w];
      while (m) {
        const uint32_t b = __ffs(m) - 1;
        *out++ = (w << 5) | b;
        m &= m - 1;
      }
    }
  }
  if (threadIdx.x == 0) st->he_count[row] = total;
}

// --------------------------------------------------------------- 3: buckets



// One block per row i in 2..r-1: HE(i) grouped by its low k-alpha bits
// (the bucket a probe of stage i looks up). Counts and cursors live in LDS
// when the table fits (2^(k-alpha) <= BK_LDS buckets), else in bk_cur.
constexpr uint32_t BK_LDS = 8192;

template <typename CurPtr>
__device__ __forceinline__ void bucket_rows(const Geom &G, uint32_t row, const uint32_t *h,
                                            uint32_t n, uint32_t *off, CurPtr cur,
                                            uint32_t *val, uint32_t *sh) {
  const uint32_t nb = 1u << (G.k - G.alpha), M = nb - 1;
  const uint32_t tid = threadIdx.x, bs = blockDim.x;
  // up to ROW_REG entries per thread are loaded together, before the
  // counters are cleared, and kept for the placing pass
  const bool in_regs = n <= ROW_REG * bs;              // uniform
  uint32_t hv[ROW_REG];
  if (in_regs) {
#pragma unroll
    for (uint32_t u = 0; u < ROW_REG; u++) hv[u] = tid + u * bs < n ? h[tid + u * bs] : 0u;
  }
  for (uint32_t b = tid; b < nb; b += bs) cur[b] = 0;
  __syncthreads();
  if (in_regs) {
#pragma unroll
    for (uint32_t u = 0; u < ROW_REG; u++)
      if (tid + u * bs < n) atomicAdd((uint32_t *)&cur[hv[u] & M], 1u);
  } else {
    for (uint32_t x = tid; x < n; x += bs) atomicAdd((uint32_t *)&cur[h[x] & M], 1u);
  }
  __syncthreads();
  const uint32_t per = (nb + bs - 1) / bs;
  const uint32_t b0 = min(tid * per, nb), b1 = min(b0 + per, nb);
  uint32_t s = 0;
  for (uint32_t b = b0; b < b1; b++) s += cur[b];
  uint32_t total;
  uint32_t run = block_excl_scan<1024>(s, &total, sh);
  for (uint32_t b = b0; b < b1; b++) {
    const uint32_t c = cur[b];
    off[b] = run;
    cur[b] = run;
    run += c;
  }
  if (tid == 0) off[nb] = total;
  __syncthreads();
  if (in_regs) {
#pragma unroll
    for (uint32_t u = 0; u < ROW_REG; u++) {
      if (tid + u * bs < n) {
        const uint32_t pos = atomicAdd((uint32_t *)&cur[hv[u] & M], 1u);
        val[pos] = hv[u];
      }
    }
  } else {
    for (uint32_t x = tid; x < n; x += bs) {
      const uint32_t c = h[x];
      const uint32_t pos = atomicAdd((uint32_t *)&cur[c & M], 1u);
      val[pos] = c;
    }
  }
}

// --------------------------------------------------------------- 4: scalars

__device__ __forceinline__ void scalars(const Geom &G, DevState *st, double e_theta) {
  const double m = (double)G.g * (double)(1ull << G.k);
  double lsum = 0.0;
  for (uint32_t i = 0; i < G.r; i++) {
    if (st->zr[i] == 0) {
      st->saturated = 1;
      st->psi = 1.0;
      st->d = 0.0;
      st->trep = 0.0;
      st->szmax = 0;
      return;
    }
    lsum += log((double)st->zr[i] / m);
  }
  const double psi = 1.0 - exp(lsum / (double)G.r);
  double pr = 1.0;
  for (uint32_t i = 0; i < G.r; i++) pr *= psi;
  const double d = (double)G.g * (1.0 - pr);
  const double trep = d * e_theta;
  st->psi = psi;
  st->d = d;
  st->trep = trep;
  st->szmax = (uint32_t)floor(trep);
}

// One block per row i: HE(i) from the hot bitmap (step 2), its bucket table
// when i >= 2 and the join may run (step 3), and in row 0's block the
// scalars (step 4), which need only the ZR(i) of the hot scan.
__global__ __launch_bounds__(1024) void k_rows(Geom G, const uint32_t *__restrict__ hotmask,
                                               uint32_t *__restrict__ he,
                                               uint32_t *__restrict__ bk_off,
                                               uint32_t *__restrict__ bk_cur,
                                               uint32_t *__restrict__ bk_val,
                                               DevState *__restrict__ st, double e_theta,
                                               uint32_t buckets) {
  __shared__ uint32_t sh[17];
  __shared__ uint32_t lcur[BK_LDS];
  const uint32_t row = blockIdx.x;
  compact_row(G, row, hotmask, he, st, sh);
  if (row == 0 && threadIdx.x == 0) scalars(G, st, e_theta);
  if (row < 2 || !buckets) return;                     // uniform over the block
  __syncthreads();                                     // this row's HE and count
  const uint32_t nb = 1u << (G.k - G.alpha);
  uint32_t *off = bk_off + (size_t)row * (nb + 1);
  const uint32_t *h = he + ((size_t)row << G.k);
  uint32_t *val = bk_val + ((size_t)row << G.k);
  const uint32_t n = st->he_count[row];
  if (nb <= BK_LDS) bucket_rows(G, row, h, n, off, lds_ptr(lcur), val, sh);
  else bucket_rows(G, row, h, n, off, bk_cur + (size_t)row * nb, val, sh);
}

// ------------------------------------------------------ 5: search choice

// The join's work is about its probes and partial addresses, |HE(0)||HE(1)|
// then times |HE(i)| / 2^(k-alpha) per further row; the lattice search's is
// 2^(32-k) addresses per hot row-0 cell, each a few integer operations and
// one LDS read (about a quarter of a join item). Every kernel of both
// searches evaluates this on the same counts, so exactly one of them runs.
constexpr double LATTICE_COST = 0.25;

__device__ __forceinline__ bool lattice_chosen(const Geom &G, const DevState *st,
                                               const Lattice &L, uint32_t path) {
  if (!L.ok || path == 1) return false;
  if (path == 2) return true;
  const double nb = (double)(1u << (G.k - G.alpha));
  double p = (double)st->he_count[0] * (double)st->he_count[1], join = p;
  for (uint32_t i = 2; i < G.r; i++) {
    p *= (double)st->he_count[i] / nb;
    join += p;
  }
  const double lat = (double)st->he_count[0] * (double)(1ull << (32 - G.k)) * LATTICE_COST;
  return lat < join;
}

// --------------------------------------------------------- 5b: lattice search
//
// Cell c of row 0 holds exactly the addresses a whose lattice point
// (a, y) lies in the box 0 <= a < 2^32, Y <= y < Y + S, where S = 2^(64-k)
// and Y = c S - B0 (mod 2^64). Every lattice point is p0 + i u + j v for a
// point p0 near (0, Y) and integers (i, j); the box is a parallelogram in
// (i, j). One work item is one line j of one cell: its lane solves the
// line's range of i (in double, widened, then narrowed exactly in 64-bit
// integers to the first and last points inside) and walks it, LAT_TRIP
// points per trip, testing each point's LE in row 1 against row 1's hot
// bitmap in LDS. About |HE(1)| / 2^k of the points pass (a few percent); they go to
// a queue per wave in LDS, and each time the queue holds 64 the wave tests
// them together, one per lane: the LEs of rows 0 and 2..r-1 read from the
// hot bitmap in global memory all at once, then one atomic per wave for
// the appends. The walk runs in step across the wave (a lane whose line is
// done walks no points), so the queue's fill is the same in every lane.
// Each address lies in exactly one cell, so there are no duplicates.

constexpr int LAT_THREADS = 512;
constexpr uint32_t LAT_TRIP = 8;                        // points per lane per trip
constexpr uint32_t LAT_QUEUE = 63 + LAT_TRIP * 64 + 1;  // survivors per wave
constexpr uint32_t LAT_QUEUE_BYTES = (LAT_THREADS / 64) * LAT_QUEUE * 4;
// row 1's bitmap for k <= 20, and the queues
constexpr uint32_t LATTICE_LDS_MAX = 131072 + LAT_QUEUE_BYTES;

__device__ __forceinline__ int64_t mul_hi_s(int64_t m, uint64_t y) {
  return (int64_t)(((__int128)m * (__int128)(unsigned __int128)y) >> 64);
}

// Lanes below this one whose bit is set in mask.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ __launch_bounds__(LAT_THREADS) void k_lattice(
    Geom G, Lattice L, uint32_t path, const uint32_t *__restrict__ he,
    const uint32_t *__restrict__ hotmask, DevState *__restrict__ st,
    uint32_t *__restrict__ cand, size_t cand_cap) {
  extern __shared__ uint32_t row1[];                   // 2^k bits, then the queues
  if (st->saturated || !lattice_chosen(G, st, L, path)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) st->search = 2;
  const uint32_t k = G.k, kw = 1u << (k - 5);
  for (uint32_t w = threadIdx.x; w < kw; w += blockDim.x) row1[w] = hotmask[kw + w];
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63;
  uint32_t *queue = row1 + kw + (threadIdx.x >> 6) * LAT_QUEUE;
  uint32_t qn = 0;                                       // queue fill, wave-uniform

  // one survivor of row 1 per lane (ok = the lane has one): its LEs in row
  // 0 and rows 2..r-1 all hot -> a candidate
  auto test = [&](uint32_t ad, bool ok) {
    const uint32_t c = hash_dh0(G, ad);
    uint32_t wv[8], bit[8];
    bit[0] = c;
    // BL(row) of ad, its shift (row-1)*alpha (0 past bit 31) worked out
    // here rather than read from G, which would hold six more scalar
    // registers through the walk
#pragma unroll
    for (uint32_t row = 2; row < 8; row++)
      if (row < G.r) {
        const uint32_t sh = (row - 1) * G.alpha;
        const uint32_t blk = sh < 32 ? (ad >> sh) & ((1u << k) - 1) : 0u;
        bit[row] = (row << k) | (c ^ blk);
      }
    if (ok) {
      wv[0] = hotmask[bit[0] >> 5];
#pragma unroll
      for (uint32_t row = 2; row < 8; row++)
        if (row < G.r) wv[row] = hotmask[bit[row] >> 5];
      ok = (wv[0] >> (bit[0] & 31)) & 1u;
#pragma unroll
      for (uint32_t row = 2; row < 8; row++)
        if (row < G.r) ok = ok && ((wv[row] >> (bit[row] & 31)) & 1u);
    }
    const uint64_t m = __ballot(ok);
    if (m) {
      unsigned long long b = 0;
      if (lane == (uint32_t)__builtin_ctzll(m)) b = atomicAdd(&st->n_cand, (unsigned long long)__popcll(m));
      b = wave_lane64(b, (int)__builtin_ctzll(m));
      const unsigned long long slot = b + lanes_below(m);
      if (ok && slot < cand_cap) cand[slot] = ad;
    }
  };
  // append the points of this trip that passed row 1 (bit q of hit: point
  // b + q step), placed by a prefix sum over the wave; test 64 at a time
  // while the queue holds them (it holds at most 63 + LAT_TRIP*64 entries)
  auto push = [&](uint32_t b, uint32_t step_, uint32_t hit) {
    const uint32_t cnt = __popc(hit);
    const uint32_t incl = wave_scan_incl(cnt);
    uint32_t pos = qn + incl - cnt;
    for (uint32_t h = hit; h; h &= h - 1) queue[pos++] = b + (uint32_t)__builtin_ctz(h) * step_;
    qn += wave_lane(incl, 63);
    __builtin_amdgcn_wave_barrier();
    while (qn >= 64) {
      qn -= 64;
      const uint32_t ad2 = queue[qn + lane];
      __builtin_amdgcn_wave_barrier();
      test(ad2, true);
    }
  };

  const uint32_t s = 64 - k;
  const uint64_t S = 1ull << s;
  const uint32_t bmask = (kw - 1) << 2;                 // byte offsets of row 1's words
  const double D = L.dneg ? -0x1p64 : 0x1p64;
  const uint32_t lines = L.lines;
  const uint32_t h0 = st->he_count[0];
  const uint32_t items = h0 * lines;                    // < 2^32 for k <= 24
  const uint32_t step = (uint32_t)L.ua;
  // every lane of a block takes the same trips (uniform bounds)
  for (uint32_t t0 = blockIdx.x * blockDim.x; t0 < items; t0 += gridDim.x * blockDim.x) {
    const uint32_t t = t0 + threadIdx.x;
    uint32_t n = 0, a = 0, c = 0;                      // n points from address a in cell c
    if (t < items) {
      // line-major: the lanes of a wave take the same line of consecutive
      // hot cells; every cell's box is the same parallelogram shifted, so
      // these lines are about equally long and the lanes end their walks
      // together (cell-major, a wave's lines differ by up to 2x)
      const uint32_t line = t / h0, x = t - line * h0;
      c = he[x];
      const uint64_t Y = ((uint64_t)c << s) - G.b0;
      // p0 = i0 u + j0 v with (i0, j0) ~ M^-1 (0, Y), M = [u v]; its offsets
      // from (0, Y) are small, so wrapping 64-bit arithmetic gives them exactly
      int64_t i0 = mul_hi_s(-L.va, Y), j0 = mul_hi_s(L.ua, Y);
      if (L.dneg) {
        i0 = -i0;
        j0 = -j0;
      }
      const int64_t a0 = (int64_t)((uint64_t)i0 * (uint64_t)L.ua + (uint64_t)j0 * (uint64_t)L.va);
      const int64_t dy0 =
          (int64_t)((uint64_t)i0 * (uint64_t)L.uy + (uint64_t)j0 * (uint64_t)L.vy - Y);
      // the cell's lines: j over the box corners
      double jmin = 0, jmax = 0;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const double da = ((q & 1) ? 4294967296.0 : 0.0) - (double)a0;
        const double dy = ((q & 2) ? (double)S : 0.0) - (double)dy0;
        const double j = (-(double)L.uy * da + (double)L.ua * dy) / D;
        jmin = q ? fmin(jmin, j) : j;
        jmax = q ? fmax(jmax, j) : j;
      }
      const int64_t jlo = (int64_t)floor(jmin) - 1, jhi = (int64_t)ceil(jmax) + 1;
      const int64_t j = jlo + line;
      if (j <= jhi) {
        // this line's i: 0 <= a0 + i ua + j va < 2^32, 0 <= dy0 + i uy + j vy < S
        const double al = -(double)a0 - (double)j * (double)L.va, ah = al + 4294967296.0;
        const double yl = -(double)dy0 - (double)j * (double)L.vy, yh = yl + (double)S;
        double lo = -1e300, hi = 1e300;
        if (L.ua) {
          const double p = al / (double)L.ua, q = ah / (double)L.ua;
          lo = fmax(lo, fmin(p, q));
          hi = fmin(hi, fmax(p, q));
        }
        if (L.uy) {
          const double p = yl / (double)L.uy, q = yh / (double)L.uy;
          lo = fmax(lo, fmin(p, q));
          hi = fmin(hi, fmax(p, q));
        }
        if (lo <= hi + 2.0) {
          // the box cuts the line in one run of i: the estimate, widened,
          // then narrowed exactly to the first and last points inside
          int64_t ilo = (int64_t)floor(lo) - 1, ihi = (int64_t)ceil(hi) + 1;
          const int64_t aj = a0 + j * L.va, yj = dy0 + j * L.vy;
          auto inside = [&](int64_t i) {
            return (uint64_t)(aj + i * L.ua) < 4294967296ull &&
                   (uint64_t)(yj + i * L.uy) < S;
          };
          while (ilo <= ihi && !inside(ilo)) ilo++;
          while (ihi >= ilo && !inside(ihi)) ihi--;
          if (ilo <= ihi) {
            // every point of [ilo, ihi] is an address of cell c
            a = (uint32_t)(aj + ilo * L.ua);
            n = (uint32_t)(ihi - ilo + 1);
          }
        }
      }
    }
    // the walk: LAT_TRIP points per trip, their row-1 words read together.
    // Point b's row-1 LE is (c ^ b) mod 2^k: its word is bits 5..k-1 of
    // c ^ b (byte offset: bits 3..k-4) and its bit bits 0..4. Points past
    // the line's end read a valid word and are masked out of hit.
    while (__ballot(n != 0)) {
      const uint32_t m = n < LAT_TRIP ? n : LAT_TRIP;
      uint32_t cb[LAT_TRIP], w[LAT_TRIP];
      uint32_t b = a;
#pragma unroll
      for (uint32_t q = 0; q < LAT_TRIP; q++) {
        cb[q] = c ^ b;
        w[q] = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(row1) +
                                                    ((cb[q] >> 3) & bmask));
        b += step;
      }
      uint32_t hit = 0;
#pragma unroll
      for (uint32_t q = 0; q < LAT_TRIP; q++) hit |= __builtin_amdgcn_ubfe(w[q], cb[q] & 31u, 1u) << q;
      hit &= (1u << m) - 1;
      push(a, step, hit);
      a += m * step;
      n -= m;
    }
  }
  // what is left in the queue
  if (qn) test(queue[lane < qn ? lane : 0], lane < qn);
}

// ------------------------------------------------------------------ 5: join
//
// Stage 1 (Alg. 3) takes every (CL_0, CL_1) of HE(0) x HE(1); stage i >= 3
// (Alg. 4) takes every partial address of stage i-1. Each item probes the
// bucket of HE(i) (i = 2 for stage 1) that holds exactly the entries whose
// low k-alpha bits continue the overlap, and every entry of it that extends
// the partial address is an output.
//
//  - The probed row's bucket table is copied into LDS when it fits: offsets
//    as uint16, and per entry only its top alpha bits (the bucket index is
//    the low k-alpha bits), as uint8 or uint16. Otherwise it is read from
//    the global tables.
//  - A wave expands its 64 items together: the bucket sizes are scanned, and
//    each lane then takes one output slot and finds the item that owns it by
//    a binary search over the scan, so uneven bucket sizes do not diverge.
//  - Every block appends its outputs to its own segment of the next
//    stage's buffer through an LDS counter (no global counter); stage i+1's
//    block b reads segment b. Counts stay exact past a segment's capacity,
//    so the host can grow it and run again.
//  - The last stage keeps an address only if it is a 32-bit value and DH0
//    of it is the CL_0 it was built from; those few are appended to the
//    candidate list with a global counter.

constexpr int JOIN_THREADS = 512;

// Orders this wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}
constexpr uint32_t TAB_OFF_MAX = 8193;          // bucket offsets held in LDS
constexpr uint32_t OWN_MAX = 256;               // output slots per wave pass set
constexpr uint32_t TAB_VAL_BYTES = 16384;       // bucket entries held in LDS (4 blocks per CU)

// Bits of the address from block i >= 2: alpha new bits at k + (i-2)*alpha.
// top = the new bits; false if any lands at or above bit 32.
__device__ __forceinline__ bool extend_top(const Geom &G, uint32_t i, uint32_t sub,
                                           uint32_t top, uint32_t *out) {
  const uint32_t pos = G.k + (i - 2) * G.alpha;
  if (pos >= 32) {
    *out = sub;
    return top == 0;
  }
  const uint64_t s2 = (uint64_t)sub | ((uint64_t)top << pos);
  *out = (uint32_t)s2;
  return (s2 >> 32) == 0;
}

// The probed row's bucket table: in LDS (offsets as uint16, entries as
// their top alpha bits) or in the global tables. Which one is a template
// parameter, so a loop over an LDS table issues no global loads that a
// wait for prefetched data would have to cover.
template <bool TLDS>
struct JoinTable {
  const LDSP uint16_t *off16;
  const LDSP uint8_t *hi8;
  const LDSP uint16_t *hi16;
  const uint32_t *off;     // global
  const uint32_t *val;     // global
  uint32_t shift;          // k - alpha
  bool wide;               // alpha > 8
  __device__ __forceinline__ uint32_t start(uint32_t key) const {
    if constexpr (TLDS) return (uint32_t)off16[key];
    else return off[key];
  }
  __device__ __forceinline__ uint32_t top_bits(uint32_t j) const {
    if constexpr (TLDS) return wide ? (uint32_t)hi16[j] : (uint32_t)hi8[j];
    else return val[j] >> shift;
  }
};

// The wave items of one join block (see k_join).
template <bool FIRST, bool LAST, bool TLDS>
__device__ __forceinline__ void join_items(
    const Geom &G, uint32_t row, const uint32_t *__restrict__ he,
    const uint2 *__restrict__ in, const uint32_t *__restrict__ in_cnt,
    const JoinTable<TLDS> &T, DevState *__restrict__ st, uint2 *__restrict__ out,
    size_t seg_cap, uint32_t *__restrict__ cand, size_t cand_cap, uint32_t M,
    LDSP uint32_t *w_incl, LDSP uint16_t *w_own, LDSP uint32_t *seg_fill_p) {
  LDSP uint32_t &seg_fill = *seg_fill_p;
  const uint32_t lane = lane_id();
  const uint32_t wib = threadIdx.x >> 6;                    // wave in block
  const uint32_t wpb = blockDim.x >> 6;                     // waves per block
  LDSP uint32_t *W_incl = w_incl + wib * 64;
  LDSP uint16_t *W_own = w_own + wib * OWN_MAX;
  const uint32_t sh = G.shift[row];
  uint2 *seg = LAST ? nullptr : out + (size_t)blockIdx.x * seg_cap;

  // this block's wave items
  uint64_t w_lo, w_hi, nch = 1;
  const uint32_t *HE0 = he, *HE1 = he + (1u << G.k);
  uint32_t h1 = 0;
  const uint2 *my_in = nullptr;
  uint32_t n_in = 0;
  if (FIRST) {
    const uint32_t h0 = st->he_count[0];
    h1 = st->he_count[1];
    nch = (h1 + 63) >> 6;
    const uint64_t W = (uint64_t)h0 * nch;
    w_lo = W * blockIdx.x / gridDim.x;
    w_hi = W * (blockIdx.x + 1) / gridDim.x;
  } else {
    const uint32_t c = in_cnt[blockIdx.x];
    n_in = (uint32_t)(c < seg_cap ? c : seg_cap);
    my_in = in + (size_t)blockIdx.x * seg_cap;
    w_lo = 0;
    w_hi = (n_in + 63) >> 6;
  }

  // A wave's items are w_lo + wib, + wpb, ...; stage 1's item w is
  // (x0, xc) = (w / nch, w % nch), stepped without dividing. The next
  // item's inputs are loaded before the current one is expanded (indices
  // past the end are clamped: the loads need no branch and stay in bounds).
  uint64_t w = w_lo + wib;
  uint32_t x0 = 0, xc = 0;
  if (FIRST && w < w_hi) {
    x0 = (uint32_t)(w / nch);
    xc = (uint32_t)(w - (uint64_t)x0 * nch);
  }
  auto load_item = [&](uint64_t wi, uint32_t a0, uint32_t ac, uint32_t &sub_o, uint32_t &c0_o,
                       bool &valid_o) {
    if (FIRST) {
      const uint32_t x1 = ac * 64 + lane;
      valid_o = wi < w_hi && x1 < h1;
      const uint32_t c0v = HE0[a0];
      c0_o = c0v;
      sub_o = c0v ^ HE1[x1 < h1 ? x1 : h1 - 1];     // BL(1)
    } else {
      const uint32_t t = (uint32_t)wi * 64 + lane;
      valid_o = wi < w_hi && t < n_in;
      const uint2 p = my_in[t < n_in ? t : n_in - 1];
      sub_o = p.x;
      c0_o = p.y;
    }
  };
  uint32_t n_sub = 0, n_c0 = 0;
  bool n_valid = false;
  if (w < w_hi) load_item(w, x0, xc, n_sub, n_c0, n_valid);

  for (; w < w_hi; w += wpb) {
    // ---- this lane's item; the next one's loads go out now
    uint32_t sub = n_sub, c0 = n_c0, b0 = 0, cnt = 0;
    const bool valid = n_valid;
    {
      const uint64_t wn = w + wpb;
      const uint32_t cx0 = x0, cxc = xc;                   // this item's (x0, xc)
      if (FIRST) {
        xc += wpb;
        while (xc >= nch) {
          xc -= (uint32_t)nch;
          x0++;
        }
      }
      // past the last item: this item's inputs again (in bounds), unused
      const bool more = wn < w_hi;
      if (FIRST) load_item(more ? wn : w, more ? x0 : cx0, more ? xc : cxc, n_sub, n_c0, n_valid);
      else load_item(more ? wn : w, 0, 0, n_sub, n_c0, n_valid);
      if (!more) n_valid = false;
    }
    if (valid) {
      const uint32_t key = ((uint32_t)((uint64_t)sub >> sh) ^ c0) & M;
      b0 = T.start(key);
      cnt = T.start(key + 1) - b0;
    }
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t total = wave_lane(incl, 63);
    if (total == 0) continue;
    // each item writes its own index into its output slots when they fit,
    // so a slot finds its item with one LDS read; otherwise by a binary
    // search over the inclusive scan
    const bool own = total <= OWN_MAX;                 // uniform over the wave
    if (own) {
      for (uint32_t q = incl - cnt; q < incl; q++) W_own[q] = (uint16_t)lane;
    } else {
      W_incl[lane] = incl;
    }
    const int32_t my_base = (int32_t)b0 - (int32_t)(incl - cnt);   // entry j = base + slot
    lds_fence();
    // ---- expand: one output slot per lane per pass
    for (uint32_t base = 0; base < total; base += 64) {
      const uint32_t slot = base + lane;
      const bool live = slot < total;
      const uint32_t sl = live ? slot : total - 1;   // lanes past the end repeat the last slot
      uint32_t o = 0;
      if (own) {
        o = W_own[sl];
      } else {
#pragma unroll
        for (uint32_t s = 32; s; s >>= 1)
          if (W_incl[o + s - 1] <= sl) o += s;
      }
      // the owning item's values straight from its lane (every lane takes part)
      const int32_t ob = __builtin_amdgcn_ds_bpermute((int)(o << 2), my_base);
      const uint32_t osub = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(o << 2), (int)sub);
      const uint32_t oc0 = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(o << 2), (int)c0);
      bool ok = false;
      uint32_t a = 0;
      if (live) {
        const uint32_t j = (uint32_t)(ob + (int32_t)slot);
        const uint32_t top = (oc0 >> (G.k - G.alpha)) ^ T.top_bits(j);
        ok = extend_top(G, row, osub, top, &a);
        if (LAST) ok = ok && hash_dh0(G, a) == oc0;
      }
      const unsigned long long mask = __ballot(ok);
      if (mask == 0) continue;
      const uint32_t n_ok = __popcll(mask);
      const uint32_t rank = __popcll(mask & ((1ull << lane) - 1));
      if (LAST) {
        unsigned long long gb = 0;
        if (lane == 0) gb = atomicAdd(&st->n_cand, (unsigned long long)n_ok);
        gb = wave_lane64(gb, 0);
        if (ok && gb + rank < cand_cap) cand[gb + rank] = a;
      } else {
        uint32_t lb = 0;
        if (lane == 0) lb = atomicAdd((uint32_t *)&seg_fill, n_ok);   // an LDS atomic after inlining
        lb = wave_lane(lb, 0);
        if (ok && (size_t)lb + rank < seg_cap) seg[lb + rank] = make_uint2(a, oc0);
      }
    }
    lds_fence();
  }
}

template <bool FIRST, bool LAST>
__global__ __launch_bounds__(JOIN_THREADS) void k_join(
    Geom G, Lattice Lt, uint32_t path, uint32_t row, const uint32_t *__restrict__ he,
    const uint2 *__restrict__ in, const uint32_t *__restrict__ in_cnt,
    const uint32_t *__restrict__ bk_off, const uint32_t *__restrict__ bk_val,
    DevState *__restrict__ st, uint2 *__restrict__ out, uint32_t *__restrict__ out_cnt,
    size_t seg_cap, uint32_t *__restrict__ cand, size_t cand_cap) {
  __shared__ uint16_t t_off[TAB_OFF_MAX];
  __shared__ __attribute__((aligned(16))) uint8_t t_val[TAB_VAL_BYTES];
  __shared__ uint32_t w_incl[JOIN_THREADS];
  __shared__ uint16_t w_own[(JOIN_THREADS / 64) * OWN_MAX];
  __shared__ uint32_t seg_fill;
  if (st->saturated || lattice_chosen(G, st, Lt, path)) return;
  if (FIRST && blockIdx.x == 0 && threadIdx.x == 0) st->search = 1;

  const uint32_t nb = 1u << (G.k - G.alpha), M = nb - 1;
  const uint32_t h = st->he_count[row];
  const bool wide = G.alpha > 8;
  const bool lds = nb + 1 <= TAB_OFF_MAX && h < 65536 && G.alpha <= 16 &&
                   (size_t)h * (wide ? 2 : 1) <= TAB_VAL_BYTES;
  const uint32_t *g_off = bk_off + (size_t)row * (nb + 1);
  const uint32_t *g_val = bk_val + ((size_t)row << G.k);
  if (threadIdx.x == 0) seg_fill = 0;
  if (lds) {
    for (uint32_t x = threadIdx.x; x <= nb; x += blockDim.x) t_off[x] = (uint16_t)g_off[x];
    for (uint32_t x = threadIdx.x; x < h; x += blockDim.x) {
      const uint32_t hi = g_val[x] >> (G.k - G.alpha);
      if (wide) reinterpret_cast<uint16_t *>(t_val)[x] = (uint16_t)hi;
      else t_val[x] = (uint8_t)hi;
    }
  }
  __syncthreads();
  const bool wide_t = wide;
  if (lds) {
    const JoinTable<true> T{lds_ptr(t_off), lds_ptr(t_val),
                            lds_ptr(reinterpret_cast<uint16_t *>(t_val)), g_off, g_val,
                            G.k - G.alpha, wide_t};
    join_items<FIRST, LAST, true>(G, row, he, in, in_cnt, T, st, out, seg_cap, cand, cand_cap,
                                  M, lds_ptr(w_incl), lds_ptr(w_own), lds_ptr(&seg_fill));
  } else {
    const JoinTable<false> T{lds_ptr(t_off), lds_ptr(t_val),
                             lds_ptr(reinterpret_cast<uint16_t *>(t_val)), g_off, g_val,
                             G.k - G.alpha, wide_t};
    join_items<FIRST, LAST, false>(G, row, he, in, in_cnt, T, st, out, seg_cap, cand,
                                   cand_cap, M, lds_ptr(w_incl), lds_ptr(w_own),
                                   lds_ptr(&seg_fill));
  }
  if (!LAST) {
    __syncthreads();
    if (threadIdx.x == 0) {
      out_cnt[blockIdx.x] = seg_fill;
      atomicAdd(&st->n_out[row], (unsigned long long)seg_fill);
      atomicMax(&st->seg_max[row], seg_fill);
    }
  }
}

// ------------------------------------------------------------ 6: estimate

template <int WPL>
__global__ __launch_bounds__(256) void k_estimate(Geom G, const uint32_t *__restrict__ sk,
                                                  const uint32_t *__restrict__ cand,
                                                  size_t cand_cap, DevState *__restrict__ st,
                                                  uint4 *__restrict__ spl, size_t spl_cap) {
  using S = LeShape<WPL>;
  if (st->saturated) return;
  const unsigned long long nc_all = st->n_cand;
  const uint64_t nc = nc_all < cand_cap ? nc_all : cand_cap;
  const uint32_t szmax = st->szmax;
  const double d = st->d;
  const uint32_t sub = threadIdx.x % S::LPL;
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x / S::LPL;
  for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u)) / S::LPL;
       base < nc; base += step) {
    const uint64_t e = base + lane_id() / S::LPL;
    const bool valid = e < nc;
    const uint32_t a = valid ? cand[e] : 0u;
    uint32_t ones = 0;
    if (valid) {
      // the candidate's LE in each row; all rows' loads of a slice are
      // issued before any is used (rows past r read as all ones)
      const uint32_t c0 = hash_dh0(G, a);
      size_t le[R_MAX];
#pragma unroll
      for (uint32_t i = 0; i < R_MAX; i++)
        le[i] = (size_t)((i << G.k) | (i == 0 ? c0 : (bit_block(G, i, a) ^ c0))) * WPL;
      if constexpr (WPL >= 4) {
#pragma unroll 1
        for (int v = 0; v < S::VPL; v++) {
          uint4 q[R_MAX];
#pragma unroll
          for (uint32_t i = 0; i < R_MAX; i++) {
            q[i] = make_uint4(~0u, ~0u, ~0u, ~0u);
            if (i < G.r) q[i] = reinterpret_cast<const uint4 *>(sk + le[i])[v * S::LPL + sub];
          }
          uint4 acc = q[0];
#pragma unroll
          for (uint32_t i = 1; i < R_MAX; i++) {
            acc.x &= q[i].x; acc.y &= q[i].y; acc.z &= q[i].z; acc.w &= q[i].w;
          }
          ones += __popc(acc.x) + __popc(acc.y) + __popc(acc.z) + __popc(acc.w);
        }
      } else {
        for (int w = 0; w < WPL; w++) {
          uint32_t q[R_MAX];
#pragma unroll
          for (uint32_t i = 0; i < R_MAX; i++) {
            q[i] = ~0u;
            if (i < G.r) q[i] = sk[le[i] + w];
          }
          uint32_t acc = q[0];
#pragma unroll
          for (uint32_t i = 1; i < R_MAX; i++) acc &= q[i];
          ones += __popc(acc);
        }
      }
    }
    if constexpr (S::LPL > 1) {
#pragma unroll
      for (int m = S::LPL / 2; m >= 1; m >>= 1) ones += __shfl_xor(ones, m, 64);
    }
    const uint32_t sz = G.g - ones;
    const bool report = valid && sub == 0 && sz <= szmax;
    unsigned long long slot = wave_reserve(&st->n_spl, report ? 1u : 0u);
    if (report && slot < spl_cap) {
      const double est = sz ? -(double)G.g * log((double)sz / d) : (double)INFINITY;
      const unsigned long long bits = __double_as_longlong(est);
      spl[slot] = make_uint4(a, sz, (uint32_t)bits, (uint32_t)(bits >> 32));
    }
  }
}

// ----------------------------------------------------------------- 7: sort
//
// Records with distinct 32-bit keys (the address in .x for uint4 records,
// the value itself for uint32) are sorted ascending by rank = the number
// of smaller keys; a last kernel places each record at its rank.
// Up to SMALL_SORT entries the ranks are counted by a (SMALL_SORT/256) x
// RANK_SPLIT grid, block (x, y) comparing 256 elements against the y-th
// slice of the keys and adding its counts to a zeroed rank array. 64
// slices rather than 8 spread a few thousand records over more blocks,
// each with a shorter compare loop: 11.3 -> 5.5 us for the 100M-pair
// window's 5.7k records (32 slices: 7.7 us).
// Longer lists: each tile of SORT_TILE keys is sorted in LDS (bitonic), and
// a record's rank is the sum over the tiles of the keys below its own, one
// binary search per tile: n * (n / SORT_TILE) * log2(SORT_TILE) steps
// rather than n^2 compares.
constexpr uint32_t SMALL_SORT = 16384;
constexpr uint32_t RANK_SPLIT = 64;
constexpr uint32_t SORT_TILE = 4096;

template <typename T>
__device__ __forceinline__ uint32_t sort_key(const T &v);
template <>
__device__ __forceinline__ uint32_t sort_key<uint4>(const uint4 &v) { return v.x; }
template <>
__device__ __forceinline__ uint32_t sort_key<uint32_t>(const uint32_t &v) { return v; }

template <typename T>
__global__ __launch_bounds__(256) void k_rank_count(const T *__restrict__ in,
                                                    const unsigned long long *__restrict__ count,
                                                    size_t cap, uint32_t *__restrict__ rank) {
  __shared__ uint32_t keys[SMALL_SORT / RANK_SPLIT];
  const unsigned long long n_all = *count;
  const uint32_t n = (uint32_t)(n_all < cap ? n_all : cap);
  if (n > SMALL_SORT) return;
  const uint32_t j = blockIdx.x * 256 + threadIdx.x;
  if (blockIdx.x * 256 >= n) return;
  const uint32_t per = (n + RANK_SPLIT - 1) / RANK_SPLIT;
  const uint32_t k0 = blockIdx.y * per, k1 = k0 + per < n ? k0 + per : n;
  if (k0 >= k1) return;
  for (uint32_t t = threadIdx.x; t < k1 - k0; t += blockDim.x) keys[t] = sort_key<T>(in[k0 + t]);
  __syncthreads();
  if (j >= n) return;
  const uint32_t mine = sort_key<T>(in[j]);
  uint32_t c = 0;
  for (uint32_t t = 0; t < k1 - k0; t++) c += keys[t] < mine;
  if (c) atomicAdd(&rank[j], c);
}

// Longer lists, step 1 (block = tile): the tile's keys sorted in LDS and
// written to skeys (the last tile padded with 0xFFFFFFFF, which is below no
// key), and the tile's ranks zeroed.
template <typename T>
__global__ __launch_bounds__(1024) void k_tile_sort(const T *__restrict__ in,
                                                    const unsigned long long *__restrict__ count,
                                                    size_t cap, uint32_t *__restrict__ skeys,
                                                    uint32_t *__restrict__ rank) {
  __shared__ uint32_t key[SORT_TILE];
  const unsigned long long n_all = *count;
  const uint64_t n = n_all < cap ? n_all : cap;
  const uint64_t t0 = (uint64_t)blockIdx.x * SORT_TILE;
  if (n <= SMALL_SORT || t0 >= n) return;
  for (uint32_t i = threadIdx.x; i < SORT_TILE; i += blockDim.x) {
    const uint64_t e = t0 + i;
    key[i] = e < n ? sort_key<T>(in[e]) : 0xFFFFFFFFu;
    if (e < n) rank[e] = 0;
  }
  __syncthreads();
  // bitonic network: pair p of a stage joins i = 2p - (p mod stride) and
  // i + stride, ascending where bit `size` of i is clear
  for (uint32_t size = 2; size <= SORT_TILE; size <<= 1)
    for (uint32_t stride = size >> 1; stride; stride >>= 1) {
      for (uint32_t p = threadIdx.x; p < SORT_TILE / 2; p += blockDim.x) {
        const uint32_t i = 2 * p - (p & (stride - 1)), j = i + stride;
        const uint32_t a = key[i], b = key[j];
        if ((a > b) == ((i & size) == 0)) {
          key[i] = b;
          key[j] = a;
        }
      }
      __syncthreads();
    }
  for (uint32_t i = threadIdx.x; i < SORT_TILE; i += blockDim.x) skeys[t0 + i] = key[i];
}

// Longer lists, step 2: for every (element tile, key tile) pair, each
// element adds the keys of the key tile below its own to its rank. The
// grid strides over the pairs.
template <typename T>
__global__ __launch_bounds__(256) void k_tile_rank(const T *__restrict__ in,
                                                   const unsigned long long *__restrict__ count,
                                                   size_t cap, const uint32_t *__restrict__ skeys,
                                                   uint32_t *__restrict__ rank) {
  __shared__ uint32_t key[SORT_TILE];
  const unsigned long long n_all = *count;
  const uint64_t n = n_all < cap ? n_all : cap;
  if (n <= SMALL_SORT) return;
  const uint64_t nt = (n + SORT_TILE - 1) / SORT_TILE;
  for (uint64_t pr = blockIdx.x; pr < nt * nt; pr += gridDim.x) {
    const uint64_t xt = pr / nt, yt = pr - xt * nt;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < SORT_TILE; i += blockDim.x)
      key[i] = skeys[yt * SORT_TILE + i];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < SORT_TILE; i += blockDim.x) {
      const uint64_t e = xt * SORT_TILE + i;
      if (e >= n) break;
      const uint32_t x = sort_key<T>(in[e]);
      // keys below x: the largest prefix whose last key is below x
      uint32_t pos = 0;
#pragma unroll
      for (uint32_t step = SORT_TILE / 2; step; step >>= 1)
        if (key[pos + step - 1] < x) pos += step;
      pos += key[pos] < x;                                // pos <= SORT_TILE - 1 here
      if (pos) atomicAdd(&rank[e], pos);
    }
  }
}

// Each record to its counted rank.
template <typename T>
__global__ __launch_bounds__(256) void k_rank_place(const T *__restrict__ in,
                                                    const unsigned long long *__restrict__ count,
                                                    size_t cap, const uint32_t *__restrict__ rank,
                                                    T *__restrict__ out) {
  const unsigned long long n_all = *count;
  const uint64_t n = n_all < cap ? n_all : cap;
  for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (uint64_t)gridDim.x * blockDim.x)
    out[rank[j]] = in[j];
}

// rank must hold SMALL_SORT zeroed entries and room for cap; skeys room for
// cap rounded up to SORT_TILE. The kernels of the path a list does not take
// return at once.
template <typename T>
static void launch_sort(const T *in, const unsigned long long *count, size_t cap, T *out,
                        uint32_t *rank, uint32_t *skeys, int grid, hipStream_t st) {
  k_rank_count<T><<<dim3(SMALL_SORT / 256, RANK_SPLIT), 256, 0, st>>>(in, count, cap, rank);
  if (cap > SMALL_SORT) {
    const size_t tiles = (cap + SORT_TILE - 1) / SORT_TILE;
    k_tile_sort<T><<<(unsigned)tiles, 1024, 0, st>>>(in, count, cap, skeys, rank);
    k_tile_rank<T><<<grid * 2, 256, 0, st>>>(in, count, cap, skeys, rank);
  }
  const int pg = grid > (int)(SMALL_SORT / 256) ? grid : (int)(SMALL_SORT / 256);
  k_rank_place<T><<<pg, 256, 0, st>>>(in, count, cap, rank, out);
}

// ---------------------------------------------------------------- 8: publish

// The device state and the first min(n, cap) sorted records written straight
// into pinned host memory, so the caller waits once for the whole restore.
__global__ __launch_bounds__(256) void k_publish(const DevState *__restrict__ st,
                                                 const uint4 *__restrict__ recs, size_t recs_cap,
                                                 DevState *h_state, uint4 *h_recs,
                                                 size_t h_cap) {
  if (blockIdx.x == 0) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(st);
    uint32_t *dst = reinterpret_cast<uint32_t *>(h_state);
    for (uint32_t i = threadIdx.x; i < sizeof(DevState) / 4; i += blockDim.x) dst[i] = src[i];
  }
  if (!h_recs) return;
  uint64_t n = st->saturated ? 0 : st->n_spl;
  if (n > recs_cap) n = recs_cap;
  if (n > h_cap) n = h_cap;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    h_recs[i] = recs[i];
}

// ------------------------------------------------------------ orchestration

template <int WPL>
static hipError_t launch_wpl(const Geom &G, const uint32_t *sketch, const RestoreBufs &B,
                             uint32_t zhot, double e_theta, int estimate, int grid,
                             hipStream_t st, const hipEvent_t *marks) {
  const uint32_t r = G.r, k = G.k;
  const size_t n_le = (size_t)r << k;
  auto mark = [&](int i) {
    if (marks) (void)hipEventRecord(marks[i], st);
  };
  mark(0);
  // 0: clear state and the hot bitmap
  k_restore_init<<<(int)((n_le / 32 + 255) / 256 < 256 ? (n_le / 32 + 255) / 256 : 256), 256, 0,
                   st>>>(B.st, B.rank, SMALL_SORT, B.hotmask, n_le / 32);
  // 1: hot scan
  if (B.lez) {
    // HS_LEZ_UNROLL 16-byte loads per lane, the whole array in one pass
    // (few blocks: each adds its row sums to ZR with global atomics)
    const uint64_t blocks = (n_le / 4 + 256 * HS_LEZ_UNROLL - 1) / (256 * HS_LEZ_UNROLL);
    k_hot_scan_lez<<<(int)(blocks < 65535 ? blocks : 65535), 256, 0, st>>>(
        G, reinterpret_cast<const uint4 *>(B.lez), zhot, B.hotmask, B.st);
  } else {
    using S = LeShape<WPL>;
    const uint64_t pass = (uint64_t)(256 / S::LPL) * HS_UNROLL;
    const uint64_t passes = (n_le + pass - 1) / pass;
    const uint64_t blocks = passes < (uint64_t)grid ? passes : (uint64_t)grid;
    const uint64_t chunk = (passes + blocks - 1) / blocks * pass;
    const int gs = (int)((n_le + chunk - 1) / chunk);
    k_hot_scan<WPL><<<gs, 256, 0, st>>>(G, sketch, zhot, B.hotmask, B.st, chunk);
  }
  mark(1);
  // 2-4: HE(i), bucket tables of rows 2..r-1, scalars
  // the bucket tables serve only the join: none when the sketch is set to
  // the lattice search
  const uint32_t buckets = !(B.lat.ok && B.cand_path == 2);
  k_rows<<<r, 1024, 0, st>>>(G, B.hotmask, B.he, B.bk_off, B.bk_cur, B.bk_val, B.st, e_theta,
                             buckets);
  mark(2);
  // 5: candidates, by the lattice search or the join (each kernel returns
  // at once unless its search is the chosen one; a search ruled out by the
  // sketch's setting is not launched)
  if (B.lat.ok && B.cand_path != 1) {
    // row 1's bitmap and the queues (above 64 KiB by the attribute that
    // prepare_restore_kernels sets)
    const size_t lds = ((size_t)4 << (k - 5)) + LAT_QUEUE_BYTES;
    // half the usual grid: each block first copies row 1's bitmap
    k_lattice<<<grid > 1 ? grid / 2 : 1, LAT_THREADS, lds, st>>>(
        G, B.lat, B.cand_path, B.he, B.hotmask, B.st, B.cand, B.cand_cap);
  }
  if (!(B.lat.ok && B.cand_path == 2)) {
    const uint32_t jb = B.jblk;
    const Lattice &Lt = B.lat;
    const uint32_t pth = B.cand_path;
    if (r == 3) {
      k_join<true, true><<<jb, JOIN_THREADS, 0, st>>>(G, Lt, pth, 2, B.he, nullptr, nullptr, B.bk_off,
                                                      B.bk_val, B.st, nullptr, nullptr, 0,
                                                      B.cand, B.cand_cap);
    } else {
      k_join<true, false><<<jb, JOIN_THREADS, 0, st>>>(G, Lt, pth, 2, B.he, nullptr, nullptr, B.bk_off,
                                                       B.bk_val, B.st, B.part[0], B.segc[0],
                                                       B.seg_cap, B.cand, B.cand_cap);
      for (uint32_t row = 3; row < r; row++) {
        // stage 1 wrote part[0]; stage `row` reads part[(row-3)%2], writes the other
        const int ib = (row - 3) & 1, ob = ib ^ 1;
        if (row + 1 == r)
          k_join<false, true><<<jb, JOIN_THREADS, 0, st>>>(
              G, Lt, pth, row, B.he, B.part[ib], B.segc[ib], B.bk_off, B.bk_val, B.st, nullptr, nullptr,
              B.seg_cap, B.cand, B.cand_cap);
        else
          k_join<false, false><<<jb, JOIN_THREADS, 0, st>>>(
              G, Lt, pth, row, B.he, B.part[ib], B.segc[ib], B.bk_off, B.bk_val, B.st, B.part[ob],
              B.segc[ob], B.seg_cap, B.cand, B.cand_cap);
      }
    }
  }
  mark(3);
  if (!estimate) {
    mark(4);
    launch_sort<uint32_t>(B.cand, &B.st->n_cand, B.cand_cap, B.cand_sorted, B.rank, B.skeys,
                          grid, st);
    k_publish<<<1, 256, 0, st>>>(B.st, nullptr, 0, B.h_state, nullptr, 0);
    mark(5);
    return hipGetLastError();
  }
  // 6: estimate and report
  k_estimate<WPL><<<grid, 256, 0, st>>>(G, sketch, B.cand, B.cand_cap, B.st, B.spl,
                                        B.spl_cap);
  mark(4);
  // 7: sort
  launch_sort<uint4>(B.spl, &B.st->n_spl, B.spl_cap, B.spl_sorted, B.rank, B.skeys, grid, st);
  // 8: state and records to the host
  k_publish<<<16, 256, 0, st>>>(B.st, B.spl_sorted, B.spl_cap, B.h_state, B.h_recs,
                                B.h_recs_cap);
  mark(5);
  return hipGetLastError();
}

hipError_t prepare_restore_kernels() {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k_lattice),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)LATTICE_LDS_MAX);
}

hipError_t launch_restore(const Geom &G, const uint32_t *sketch, const RestoreBufs &B,
                          uint32_t zhot, double e_theta, int estimate, int grid,
                          hipStream_t st, const hipEvent_t *marks) {
  switch (G.wpl) {
    case 1: return launch_wpl<1>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 2: return launch_wpl<2>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 4: return launch_wpl<4>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 8: return launch_wpl<8>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 16: return launch_wpl<16>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 32: return launch_wpl<32>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 64: return launch_wpl<64>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 128: return launch_wpl<128>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 256: return launch_wpl<256>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 512: return launch_wpl<512>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 1024: return launch_wpl<1024>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    case 2048: return launch_wpl<2048>(G, sketch, B, zhot, e_theta, estimate, grid, st, marks);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ddhf

// Internal declarations shared by the library's translation units: the
// device-side hash group, kernel argument blocks, device state and the
// kernel launchers. Not part of the public ABI (include/ddhf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ddhf {

// Geometry and hash coefficients of one sketch, passed by value to kernels.
struct Geom {
  uint32_t g;        // bits per LE
  uint32_t k;        // log2 LEs per row
  uint32_t r;        // rows
  uint32_t alpha;    // block stride
  uint32_t log2g;
  uint32_t wpl;      // 32-bit words per LE = g/32
  uint32_t shift[8]; // bit offset of block i: min((i-1)*alpha, 32); [0] unused
  uint64_t a0, b0;   // DH0 coefficients
  uint64_t a1, b1;   // H1 coefficients
};

// DH0: multiply-add-shift to k bits.
__device__ __forceinline__ uint32_t hash_dh0(const Geom &G, uint32_t x) {
  return (uint32_t)((G.a0 * (uint64_t)x + G.b0) >> (64 - G.k));
}

// H1: multiply-add-shift to log2(g) bits.
__device__ __forceinline__ uint32_t hash_h1(const Geom &G, uint32_t y) {
  return (uint32_t)((G.a1 * (uint64_t)y + G.b1) >> (64 - G.log2g));
}

// BL(i): k bits of x starting at bit (i-1)*alpha (0 past bit 31).
__device__ __forceinline__ uint32_t bit_block(const Geom &G, uint32_t i,
                                              uint32_t x) {
  return (uint32_t)(((uint64_t)x >> G.shift[i]) & ((1u << G.k) - 1));
}

// Device-resident state of one restore. Zeroed at the start of each restore
// by a fill kernel.
struct DevState {
  unsigned long long zr[8];          // ZR(i)
  unsigned long long n_out[8];       // outputs of join stage i (2..r-1)
  unsigned long long n_cand;         // candidates (after re-hash)
  unsigned long long n_spl;          // reported
  uint32_t he_count[8];              // |HE(i)|
  double psi, d, trep;
  uint32_t szmax;
  uint32_t saturated;
  uint32_t seg_max[8];               // largest block segment of join stage i
  uint32_t search;                   // candidate search that ran: 1 join, 2 lattice
  uint32_t pad;
};

// Row 0's hash DH0(a) = ((A0 a + B0) mod 2^64) >> (64 - k) puts a in cell c
// iff the point (a, y), y = A0 a mod 2^64 + t 2^64, of the lattice
// {(a, y) : y = A0 a (mod 2^64)} lies in the box 0 <= a < 2^32,
// c 2^(64-k) - B0 <= y < (c + 1) 2^(64-k) - B0. A reduced basis (u, v) of
// that lattice (in the metric that makes the box square) lets the restore
// enumerate each hot cell's 2^(32-k) addresses line by line (k_lattice)
// instead of joining the hot lists. Computed on the host per sketch.
struct Lattice {
  int64_t ua, uy;          // u = (u_a, u_y)
  int64_t va, vy;          // v = (v_a, v_y); u_a v_y - v_a u_y = +-2^64
  uint32_t dneg;           // 1 if that determinant is -2^64
  uint32_t lines;          // lines j = const of a cell's box, at most
  uint32_t ok;             // the basis fits the kernel's 64-bit arithmetic
  uint32_t pad;
};

// Restore work buffers (device pointers) and capacities.
struct RestoreBufs {
  const uint32_t *lez;    // zeros per LE as the update left them, or null
                          // (the hot scan counts them in the sketch)
  DevState *st;
  uint32_t *hotmask;      // r * 2^k bits
  uint32_t *he;           // r * 2^k entries, row i at i*2^k, ascending
  uint32_t *bk_off;       // r * (nb+1): bucket offsets of row i (rows >= 2)
  uint32_t *bk_cur;       // r * nb: fill cursors
  uint32_t *bk_val;       // r * 2^k: row entries grouped by bucket
  uint2 *part[2];         // ping-pong partial addresses (sub, c0): jblk
                          // segments of seg_cap entries, one per join block
  uint32_t *segc[2];      // entries written to each segment
  size_t seg_cap;
  uint32_t jblk;          // blocks of the join kernels
  uint32_t *cand;         // candidate addresses
  size_t cand_cap;
  uint4 *spl;             // records {ip, sz, est.lo, est.hi}, unsorted
  uint4 *spl_sorted;      // the same, ascending by ip
  size_t spl_cap;
  uint32_t *cand_sorted;
  uint32_t *rank;         // sort ranks: at least 16384 entries and the
                          // larger of cand_cap and spl_cap
  uint32_t *skeys;        // tile-sorted keys of a long list: that many,
                          // rounded up to 4096
  // pinned host memory (device-side addresses) the last step writes: the
  // device state and the first min(n, h_recs_cap) sorted records
  DevState *h_state;
  uint4 *h_recs;          // may be null (no records published)
  size_t h_recs_cap;
  // candidate search: the lattice of row 0's cells, and the choice
  // (0 = by estimated work, 1 = the join of Algs. 3-4, 2 = the lattice)
  Lattice lat;
  uint32_t cand_path;
};

// Inclusive prefix sum over the 64 lanes of a wave, in registers: four
// row shifts inside each 16-lane row, then the row broadcasts of lanes 15
// and 31 into the rows above (DPP, no LDS round trips). All lanes active.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Lane l's value broadcast to the wave (a scalar read, no LDS).
__device__ __forceinline__ uint32_t wave_lane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ unsigned long long wave_lane64(unsigned long long v, int l) {
  const uint32_t lo = wave_lane((uint32_t)v, l), hi = wave_lane((uint32_t)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// Binned update (update.hip): the sketch is cut into tiles of 160 KiB, the
// most LDS one gfx950 workgroup can hold (1280 LEs of g = 1024, a whole
// number of LEs for every g); a code is the bit offset inside its tile
// (21 bits).
constexpr uint32_t BIN_TILE_WORDS = 40960;           // 160 KiB
constexpr uint32_t BIN_TILE_BITS = BIN_TILE_WORDS * 32;
constexpr uint32_t BIN_SLOTS = 4096;                 // tile slots of the per-block arrays
constexpr uint32_t BIN_MAX = 3276;                   // tiles: a sketch bit index stays
                                                     // below 2^32 (BIN_MAX * BIN_TILE_BITS)
// The tile of sketch bit index B (a division by a constant).
__host__ __device__ __forceinline__ uint32_t bin_tile(uint32_t B) { return B / BIN_TILE_BITS; }
constexpr uint32_t SPLIT_MIN = 1u << 18;             // tiles above this many code words
constexpr uint32_t APPLY_ITEM = 1u << 17;            //   are cut into items of this many

constexpr uint32_t BIN_BLOCKS_MAX = 1024;

// The binned update keeps each LE's zero count (for the restore's hot scan)
// when an LE spans 4 to 256 words: a whole number of 16-byte vectors held by
// at most one wave's lanes.
constexpr bool lez_kept(uint32_t g) { return g >= 128 && g <= 8192; }

// Scatter blocks are put in BIN_GROUPS groups by block index mod BIN_GROUPS:
// gfx950 hands workgroups of a dispatch to its 8 XCDs in turn, so a group is
// the blocks that share one XCD and its L2. The blocks of a group write
// every tile's codes into one shared region, not one region each.
constexpr uint32_t BIN_GROUPS = 8;

// The count pass estimates each (group, tile) region from every
// BIN_SAMPLE-th batch of each block; the region gets the estimate plus an
// eighth plus BIN_REGION_PAD words. A run that does not fit its region goes
// whole to the spill area and is listed in its tile's spill runs.
constexpr uint32_t BIN_SAMPLE = 16;
constexpr uint32_t BIN_REGION_PAD = 64;

// Per-tile region state of one job, one array of tile_state_words(nbins)
// words: per (group, tile) region its capacity (then, once laid out, its
// end), its start and the end of its written part, in 64-bit words from
// the job's codes; then per tile the count and the words of its spill
// runs; then the spill area's cursor.
__host__ __device__ constexpr uint64_t tile_state_words(uint32_t nbins) {
  return (uint64_t)26 * nbins + 1;
}
struct TileState {
  uint32_t *capg, *regb, *fill;   // [BIN_GROUPS][nbins]
  uint32_t *dcnt, *swords;        // [nbins]
  uint32_t *spill_cur;            // [1]
};
__host__ __device__ inline TileState tile_state(uint32_t *p, uint32_t nbins) {
  TileState T;
  T.capg = p;
  T.regb = p + (size_t)BIN_GROUPS * nbins;
  T.fill = p + (size_t)2 * BIN_GROUPS * nbins;
  T.dcnt = p + (size_t)3 * BIN_GROUPS * nbins;
  T.swords = T.dcnt + nbins;
  T.spill_cur = T.swords + nbins;
  return T;
}

// One sketch's share of an update launch. Kernels of a launch take a table
// of these (device memory) and map each block, tile or work item to its
// job by binary search over the prefix fields blk0 / tile0 / item0.
struct UpdJob {
  Geom G;
  uint32_t *sk;
  const uint2 *pairs;    // this launch's pairs of the job
  uint64_t words;        // sketch words
  uint64_t n;            // pairs
  uint64_t chunk;        // pairs per block (even)
  uint32_t nbins;        // tiles of the sketch
  uint32_t nblk;         // blocks of this job (count / scatter / direct)
  uint32_t blk0;         // first global block of this job
  uint32_t tile0;        // first global tile of this job
  uint32_t hstride;      // row stride of hist (>= nblk)
  uint32_t fresh;        // binned: the sketch is all zero and not yet written
                         // (the first round after a reset): tiles are not
                         // read, and every tile is written
  uint32_t *hist, *totals, *base, *item_start, *xslot, *n_items;
  uint32_t *item_tile;   // tile of each apply item (ITEM_TILE_SLOTS(nbins) entries)
  uint32_t *gcur;        // [BIN_GROUPS][nbins]: claim cursor of each group's region per tile
  uint32_t *tst;         // region state (tile_state_words(nbins) words)
  uint32_t *lez;         // zeros of every LE of each tile the update writes
                         // (one word per LE), or null
  uint32_t *codes, *scratch;
  uint2 *desc;           // spill runs of tile t: desc[t * dmax + i] = (start, words)
  uint64_t rcap;         // 64-bit words of the regions; the spill area follows
  uint32_t dmax;         // spill runs per tile at most (the job's batches)
  uint32_t item0;        // first global apply item (written on the device)
  uint32_t check;        // direct kernel: test the bit before the atomicOr
  uint32_t sample;       // count every sample-th batch of a block (1: all)
  uint32_t rscale;       // region = estimate * rscale / 64 + pad (0: the default
                         // 9/8 of a sampled estimate, or the exact count)
};

constexpr uint32_t MAX_JOBS = 256;     // jobs per launch group

// Pairs of one job in one binned round, at most; it bounds the apply items
// of a job: a tile with v code words makes at most 1 + v / APPLY_ITEM of
// them, and a round has at most 8 * MAX_ROUND_PAIRS codes (and no more
// words than codes).
constexpr uint64_t MAX_ROUND_PAIRS = (uint64_t)1 << 28;
constexpr uint64_t ITEM_TILE_SLOTS(uint32_t nbins) {
  return (uint64_t)nbins + 8 * MAX_ROUND_PAIRS / APPLY_ITEM + 1;
}

// Upper bound of the 64-bit code words (three codes each) a binned job
// writes: a block's batch with c codes in a tile writes ceil(c / 3) words
// there, and every batch but a block's last holds at least 2048 pairs.
inline uint64_t code_words_bound(uint64_t n, uint32_t r, uint32_t nbins, uint32_t nblk,
                                 uint64_t chunk) {
  const uint64_t codes = (uint64_t)r * n;
  const uint64_t runs = (uint64_t)nbins * nblk * ((chunk + 2047) / 2048);
  const uint64_t b = (codes + 2 * runs) / 3 + 1;
  return b < codes ? b : codes;
}

// Pairs per thread of the scatter (and count) batches for r rows, the
// largest tile count of a launch and the requested setting (see
// launch_update_jobs): 6, 5, 4 or 2.
inline uint32_t scatter_ppt(uint32_t r, uint32_t max_tiles, uint32_t ppt) {
  if (max_tiles <= 2048) {
    const uint32_t p4 = r <= 7 ? 4 : 2, p6 = r <= 5 ? 6 : p4;
    return ppt == 2 ? 2 : (ppt == 6 ? p6 : p4);
  }
  if (r <= 5 && max_tiles <= 3072 && ppt != 2) return 5;
  return ppt == 2 ? 2 : (r <= 5 ? 4 : 2);
}

// Code buffer of one binned job, in 64-bit words: the regions (the bound
// plus room for every region's pad) and then the spill area (the bound:
// it never holds more than every word), 16-byte aligned.
inline uint64_t job_region_words(uint64_t bound, uint32_t nbins) {
  return (bound + (uint64_t)BIN_GROUPS * nbins * (BIN_REGION_PAD + 2) + 1) & ~(uint64_t)1;
}
inline uint64_t job_code_words(uint64_t bound, uint32_t nbins) {
  return job_region_words(bound, nbins) + ((bound + 1) & ~(uint64_t)1);
}
// Batches of a job (an upper bound of the spill runs of any one tile).
inline uint32_t job_batches(uint32_t nblk, uint64_t chunk, uint32_t ppt) {
  const uint64_t step = 1024ull * ppt;
  return (uint32_t)(nblk * ((chunk + step - 1) / step));
}

// Launches one update round for n_jobs jobs that share r: `h_jobs` is the
// host copy (blk0 / tile0 / nblk filled in), `d_jobs` its device copy
// (already transferred), `d_total` one device word for the item count.
hipError_t launch_update_jobs(const UpdJob *h_jobs, UpdJob *d_jobs, uint32_t n_jobs,
                              uint32_t *d_total, bool binned, uint32_t r, uint32_t ppt,
                              uint32_t apply_grid, hipStream_t st);

// ---- launchers (update.hip) ----
hipError_t launch_fill_u32(uint32_t *p, size_t n_words, uint32_t value,
                           int grid, hipStream_t st);
hipError_t launch_or_u32(uint32_t *dst, const uint32_t *src, size_t n_words, int grid,
                         hipStream_t st);

// ---- launchers (restore.hip) ----
// Once per device, before any restore (and outside graph capture): lets the
// lattice search take more than 64 KiB of LDS.
hipError_t prepare_restore_kernels();
// Runs every restore step up to and including the candidate list (and, when
// estimate != 0, the estimate, report filter and sort). All counts stay on
// the device; the caller reads DevState afterwards.
// marks: null, or 6 events recorded on st at the phase boundaries (before
// the hot scan, after it, after the per-row kernel, after the join, after
// the estimate, after the publish).
hipError_t launch_restore(const Geom &G, const uint32_t *sketch,
                          const RestoreBufs &B, uint32_t zhot, double e_theta,
                          int estimate, int grid, hipStream_t st,
                          const hipEvent_t *marks = nullptr);

}  // namespace ddhf

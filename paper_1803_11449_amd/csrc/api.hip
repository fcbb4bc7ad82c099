// C ABI of libddhf (declared in include/ddhf.h): handle lifetime, argument
// checks, device memory, batching, and the host side of the restore
// (capacity growth and the copies to the caller).
//
// Memory. A handle owns what is tied to its sketch and must outlive a call:
// the sketch, its per-row restore arrays (hot bitmap, hot lists, bucket
// tables), its per-tile update arrays, its device state and its sorted
// output. The large scratch buffers are shared by every handle on a device
// (DevCtx): the update arena (codes and scratch tiles of one launch group)
// and the restore pool (partial addresses, candidates, unsorted records,
// sort ranks). Work that uses either waits on the event of the last work
// that used them, so streams of different handles stay ordered on them.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "ddhf.h"
#include "ddhf_internal.h"

using namespace ddhf;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_OK(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      return fail(e_ == hipErrorOutOfMemory ? SKETCH_E_NOMEM : SKETCH_E_HIP,    \
                  "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,      \
                  __LINE__);                                                     \
  } while (0)

// Makes a device current for the lifetime of the guard and puts the
// caller's device back afterwards.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

#define DEVICE_GUARD(dev)                                                        \
  DeviceGuard guard_(dev);                                                       \
  if (guard_.err != hipSuccess)                                                  \
    return fail(SKETCH_E_HIP, "hipSetDevice(%d): %s", (int)(dev),                \
                hipGetErrorString(guard_.err));

template <typename T>
int dev_alloc(T **p, size_t count, const char *what) {
  *p = nullptr;
  hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? SKETCH_E_NOMEM : SKETCH_E_HIP,
                "hipMalloc(%s, %zu bytes): %s", what, count * sizeof(T), hipGetErrorString(e));
  }
  return SKETCH_OK;
}

template <typename T>
void dev_free(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

// Pinned host memory for `count` T and the address kernels write it at.
template <typename T>
int pinned_alloc(T **h, T **d, size_t count, const char *what) {
  *h = nullptr;
  *d = nullptr;
  if (hipHostMalloc((void **)h, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
    *h = nullptr;
    return fail(SKETCH_E_NOMEM, "hipHostMalloc(%s, %zu bytes) failed", what, count * sizeof(T));
  }
  if (hipHostGetDevicePointer((void **)d, *h, 0) != hipSuccess) {
    (void)hipHostFree(*h);
    *h = nullptr;
    return fail(SKETCH_E_HIP, "hipHostGetDevicePointer(%s) failed", what);
  }
  return SKETCH_OK;
}

template <typename T>
void pinned_free(T *&h, T *&d) {
  if (h) (void)hipHostFree((void *)h);
  h = nullptr;
  d = nullptr;
}

// ---------------------------------------------------------- ordering

// Orders device work on one resource (a shared buffer, a sketch) across
// streams: work about to be enqueued on a stream waits for the last work
// that used the resource when that work was enqueued on another stream.
struct Lane {
  hipEvent_t ev = nullptr;
  bool armed = false;
  hipStream_t stream = nullptr;   // stream of the last work
};

int lane_init(Lane &l) {
  if (hipEventCreateWithFlags(&l.ev, hipEventDisableTiming) != hipSuccess) {
    l.ev = nullptr;
    return fail(SKETCH_E_HIP, "hipEventCreate failed");
  }
  return SKETCH_OK;
}

void lane_free(Lane &l) {
  if (l.armed) (void)hipEventSynchronize(l.ev);
  if (l.ev) (void)hipEventDestroy(l.ev);
  l.ev = nullptr;
  l.armed = false;
}

int lane_enter(Lane &l, hipStream_t st) {
  if (l.armed && st != l.stream) HIP_OK(hipStreamWaitEvent(st, l.ev, 0));
  return SKETCH_OK;
}

int lane_leave(Lane &l, hipStream_t st) {
  HIP_OK(hipEventRecord(l.ev, st));
  l.armed = true;
  l.stream = st;
  return SKETCH_OK;
}

// Wait on the host until the last work that used the resource is done.
int lane_idle(Lane &l) {
  if (l.armed) HIP_OK(hipEventSynchronize(l.ev));
  return SKETCH_OK;
}

// ---------------------------------------------------------- device context

constexpr size_t ARENA_MAX_PAIRS = MAX_ROUND_PAIRS;   // pairs per binned launch group

// Work memory of sketch_restore_noalloc, for callers that cannot allocate:
// one fixed array per GPU, held until the process ends. Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// for the symbol): it uses the per-device address that ctx_acquire looks up
// with hipGetSymbolAddress.
constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
constexpr size_t NOALLOC_CAND = (size_t)1 << 20;      // candidates (and sorted copy)
constexpr size_t NOALLOC_SPL = (size_t)1 << 18;       // records (and sorted copy)
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

// One restore pool: the work buffers a restore shares with the restores
// before and after it (join partials, candidates, unsorted records, sort
// ranks), and the last work that used them. Pool 0 serves single restores
// on the caller's stream; a batch spreads its jobs over every pool, pools
// 1.. on streams of their own that fork from the caller's stream and join
// it again, so the restores of different jobs run at the same time.
struct RPool {
  uint2 *part[2] = {};
  uint32_t *segc[2] = {};
  size_t seg_cap = 0;
  uint32_t *cand = nullptr, *cand_sorted = nullptr;
  size_t cand_cap = 0;
  uint4 *spl = nullptr;
  size_t spl_cap = 0;
  uint32_t *rank = nullptr, *skeys = nullptr;
  size_t rank_cap = 0;           // entries of rank and skeys
  Lane lane;
  bool ready = false;            // buffers, lane (and stream) exist
  hipStream_t stream = nullptr;  // pools 1..: the pool's stream (default priority)
  hipEvent_t join = nullptr;     // pools 1..: marks the end of the pool's part of a batch
};

constexpr int RESTORE_POOLS = 4;

struct DevCtx {
  static constexpr int SLOTS = 16;
  int dev = -1;
  int refs = 0;
  int n_cu = 0;
  std::mutex mu;
  // ring of update job tables
  UpdJob *h_jobs[SLOTS] = {};
  UpdJob *d_jobs[SLOTS] = {};
  uint32_t *d_total = nullptr;   // SLOTS words
  hipEvent_t ev[SLOTS] = {};
  bool armed[SLOTS] = {};
  int next = 0;
  // update arena
  uint32_t *codes = nullptr;
  size_t codes_cap = 0;          // words
  uint32_t *scratch = nullptr;
  size_t scratch_tiles = 0;
  // restore pools
  uint32_t jblk = 0;             // blocks of the join kernels
  RPool pool[RESTORE_POOLS];
  size_t pool_entries = 0;       // buffer entries of a pool made on demand (0: initial)
  hipEvent_t fork = nullptr;     // a batch's start on the caller's stream
  // last work that used the update arena (the pools have their own): so
  // one batch's update can run while another batch's restore does
  Lane arena_lane;
  uint64_t gen = 0;              // bumped whenever the arena or a pool moves
  // this device's copy of the no-alloc restore's work array (its address
  // from hipGetSymbolAddress at set-up) and the last work that used it
  uint8_t *noalloc = nullptr;
  Lane noalloc_lane;
};

std::mutex g_ctx_mu;
DevCtx *g_ctx[256] = {};

// Wait on the host until a restore pool is idle (before reallocating it).
int pool_idle(RPool &p) { return lane_idle(p.lane); }
int pools_idle(DevCtx *c) {
  for (RPool &p : c->pool)
    if (p.ready) {
      int rc = pool_idle(p);
      if (rc) return rc;
    }
  return SKETCH_OK;
}
int arena_idle(DevCtx *c) { return lane_idle(c->arena_lane); }

// Sort ranks and tile-sorted keys for the longer of the candidate and
// record buffers (after the pool is idle).
int ensure_rank(DevCtx *c, RPool &p) {
  const size_t need = (std::max<size_t>({p.cand_cap, p.spl_cap, 16384}) + 4095) & ~(size_t)4095;
  if (p.rank_cap >= need) return SKETCH_OK;
  c->gen++;
  dev_free(p.rank);
  dev_free(p.skeys);
  p.rank_cap = 0;
  int rc = dev_alloc(&p.rank, need, "sort ranks");
  if (!rc) rc = dev_alloc(&p.skeys, need, "sort keys");
  if (!rc) p.rank_cap = need;
  return rc;
}

// Restore pool buffers at exactly `cap` entries (after the pool is idle).
int alloc_partials(DevCtx *c, RPool &p, size_t cap) {
  int rc = pool_idle(p);
  if (rc) return rc;
  c->gen++;
  dev_free(p.part[0]);
  dev_free(p.part[1]);
  p.seg_cap = 0;
  rc = dev_alloc(&p.part[0], cap * c->jblk, "partials");
  if (!rc) rc = dev_alloc(&p.part[1], cap * c->jblk, "partials");
  if (!rc) p.seg_cap = cap;
  return rc;
}

int alloc_cand(DevCtx *c, RPool &p, size_t cap) {
  int rc = pool_idle(p);
  if (rc) return rc;
  c->gen++;
  dev_free(p.cand);
  dev_free(p.cand_sorted);
  p.cand_cap = 0;
  rc = dev_alloc(&p.cand, cap, "candidates");
  if (!rc) rc = dev_alloc(&p.cand_sorted, cap, "candidates");
  if (!rc) p.cand_cap = cap;
  if (!rc) rc = ensure_rank(c, p);
  return rc;
}

int alloc_pool_spl(DevCtx *c, RPool &p, size_t cap) {
  int rc = pool_idle(p);
  if (rc) return rc;
  c->gen++;
  dev_free(p.spl);
  p.spl_cap = 0;
  rc = dev_alloc(&p.spl, cap, "records");
  if (!rc) p.spl_cap = cap;
  if (!rc) rc = ensure_rank(c, p);
  return rc;
}

// Growth by at least half of what was asked, at least doubling.
size_t grown(size_t need, size_t cap) { return std::max(need + need / 2, cap * 2); }
int grow_partials(DevCtx *c, RPool &p, size_t need) {
  return alloc_partials(c, p, grown(need, p.seg_cap));
}
int grow_cand(DevCtx *c, RPool &p, size_t need) { return alloc_cand(c, p, grown(need, p.cand_cap)); }
int grow_pool_spl(DevCtx *c, RPool &p, size_t need) {
  return alloc_pool_spl(c, p, grown(need, p.spl_cap));
}

// Initial restore pool: partial addresses per join block, candidates, records.
constexpr size_t POOL_SEG0 = (size_t)1 << 12, POOL_CAND0 = (size_t)1 << 16,
                 POOL_SPL0 = (size_t)1 << 16;

// Update arena for `words` code words and `tiles` scratch tiles.
int ensure_arena(DevCtx *c, size_t words, size_t tiles) {
  if (c->codes_cap >= words && c->scratch_tiles >= tiles) return SKETCH_OK;
  int rc = arena_idle(c);
  if (rc) return rc;
  c->gen++;
  if (c->codes_cap < words) {
    dev_free(c->codes);
    c->codes_cap = 0;
    const size_t cap = std::max(words, c->codes_cap + c->codes_cap / 2);
    rc = dev_alloc(&c->codes, cap, "update codes");
    if (rc) return rc;
    c->codes_cap = cap;
  }
  if (c->scratch_tiles < tiles) {
    dev_free(c->scratch);
    c->scratch_tiles = 0;
    rc = dev_alloc(&c->scratch, tiles * (size_t)BIN_TILE_WORDS, "update scratch tiles");
    if (rc) return rc;
    c->scratch_tiles = tiles;
  }
  return SKETCH_OK;
}

// Buffers of pool i at `entries` per buffer (0: the initial sizes), its
// lane, and for i >= 1 its stream and join event. Caller holds c->mu.
int pool_init(DevCtx *c, int i, size_t entries) {
  RPool &p = c->pool[i];
  int rc = SKETCH_OK;
  if (!p.lane.ev) rc = lane_init(p.lane);
  if (!rc && i > 0 && !p.stream &&
      hipStreamCreateWithFlags(&p.stream, hipStreamNonBlocking) != hipSuccess) {
    p.stream = nullptr;
    rc = fail(SKETCH_E_HIP, "device context: hipStreamCreate failed");
  }
  if (!rc && i > 0 && !p.join &&
      hipEventCreateWithFlags(&p.join, hipEventDisableTiming) != hipSuccess) {
    p.join = nullptr;
    rc = fail(SKETCH_E_HIP, "device context: hipEventCreate failed");
  }
  if (!rc && !p.segc[0]) rc = dev_alloc(&p.segc[0], c->jblk, "segment counts");
  if (!rc && !p.segc[1]) rc = dev_alloc(&p.segc[1], c->jblk, "segment counts");
  if (!rc) rc = alloc_partials(c, p, entries ? entries : POOL_SEG0);
  if (!rc) rc = alloc_cand(c, p, entries ? entries : POOL_CAND0);
  if (!rc) rc = alloc_pool_spl(c, p, entries ? entries : POOL_SPL0);
  p.ready = rc == SKETCH_OK;
  return rc;
}

// A pool's device buffers freed (its lane idle first); the lane, stream
// and event stay.
void pool_free_buffers(RPool &p) {
  (void)pool_idle(p);
  dev_free(p.part[0]);
  dev_free(p.part[1]);
  dev_free(p.segc[0]);
  dev_free(p.segc[1]);
  dev_free(p.cand);
  dev_free(p.cand_sorted);
  dev_free(p.spl);
  dev_free(p.rank);
  dev_free(p.skeys);
  p.seg_cap = p.cand_cap = p.spl_cap = p.rank_cap = 0;
  p.ready = false;
}

// Free the update arena and the batch pools, and reallocate pool 0 at
// `entries` per buffer (0: the initial sizes). Caller holds c->mu.
int trim_pools(DevCtx *c, size_t entries) {
  int rc = pools_idle(c);
  if (!rc) rc = arena_idle(c);
  if (rc) return rc;
  c->gen++;
  dev_free(c->codes);
  c->codes_cap = 0;
  dev_free(c->scratch);
  c->scratch_tiles = 0;
  for (int i = 1; i < RESTORE_POOLS; i++)
    if (c->pool[i].ready) pool_free_buffers(c->pool[i]);
  c->pool_entries = entries;            // the batch pools come back at this size
  RPool &p = c->pool[0];
  dev_free(p.rank);
  dev_free(p.skeys);
  p.rank_cap = 0;
  return pool_init(c, 0, entries);
}

void ctx_free(DevCtx *c) {
  for (int i = 0; i < DevCtx::SLOTS; i++) {
    if (c->armed[i]) (void)hipEventSynchronize(c->ev[i]);
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    if (c->h_jobs[i]) (void)hipHostFree(c->h_jobs[i]);
    dev_free(c->d_jobs[i]);
  }
  for (RPool &p : c->pool) {
    pool_free_buffers(p);
    lane_free(p.lane);
    if (p.stream) (void)hipStreamDestroy(p.stream);
    if (p.join) (void)hipEventDestroy(p.join);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  lane_free(c->arena_lane);
  lane_free(c->noalloc_lane);
  dev_free(c->d_total);
  dev_free(c->codes);
  dev_free(c->scratch);
  delete c;
}

// The context of `dev` (created on first use; refcounted by handles).
int ctx_acquire(int dev, int n_cu, DevCtx **out) {
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  if (dev < 0 || dev >= 256) return fail(SKETCH_E_INVAL, "device %d out of range", dev);
  DevCtx *c = g_ctx[dev];
  if (!c) {
    c = new DevCtx();
    c->dev = dev;
    c->n_cu = n_cu;
    c->jblk = (uint32_t)(n_cu * 4);      // four join blocks per compute unit fit in LDS
    int rc = SKETCH_OK;
    for (int i = 0; i < DevCtx::SLOTS && !rc; i++) {
      if (hipHostMalloc((void **)&c->h_jobs[i], sizeof(UpdJob) * MAX_JOBS) != hipSuccess) {
        c->h_jobs[i] = nullptr;
        rc = fail(SKETCH_E_NOMEM, "device context: hipHostMalloc failed");
        break;
      }
      rc = dev_alloc(&c->d_jobs[i], MAX_JOBS, "job tables");
      if (!rc && hipEventCreateWithFlags(&c->ev[i], hipEventDisableTiming) != hipSuccess)
        rc = fail(SKETCH_E_HIP, "device context: hipEventCreate failed");
    }
    if (!rc) rc = lane_init(c->arena_lane);
    if (!rc && hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess) {
      c->fork = nullptr;
      rc = fail(SKETCH_E_HIP, "device context: hipEventCreate failed");
    }
    if (!rc) rc = lane_init(c->noalloc_lane);
    if (!rc && prepare_restore_kernels() != hipSuccess)
      rc = fail(SKETCH_E_HIP, "device context: restore kernel attributes");
    // the caller made dev current: this is dev's copy of the array
    if (!rc && hipGetSymbolAddress((void **)&c->noalloc, HIP_SYMBOL(scratch)) != hipSuccess) {
      c->noalloc = nullptr;
      rc = fail(SKETCH_E_HIP, "device context: hipGetSymbolAddress(scratch) failed");
    }
    if (!rc) rc = dev_alloc(&c->d_total, DevCtx::SLOTS, "item totals");
    if (!rc) rc = pool_init(c, 0, 0);
    if (rc) {
      ctx_free(c);
      return rc;
    }
    g_ctx[dev] = c;
  }
  c->refs++;
  *out = c;
  return SKETCH_OK;
}

void ctx_release(DevCtx *c) {
  if (!c) return;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  if (--c->refs > 0) return;
  g_ctx[c->dev] = nullptr;
  ctx_free(c);
}

// Copy n jobs into the next ring slot and launch them on st (caller holds
// c->mu and has entered the pools).
int launch_jobs(DevCtx *c, const UpdJob *jobs, uint32_t n, bool binned, uint32_t r,
                uint32_t ppt, uint32_t apply_grid, hipStream_t st) {
  const int slot = c->next;
  c->next = (c->next + 1) % DevCtx::SLOTS;
  if (c->armed[slot]) HIP_OK(hipEventSynchronize(c->ev[slot]));
  memcpy(c->h_jobs[slot], jobs, sizeof(UpdJob) * n);
  HIP_OK(hipMemcpyAsync(c->d_jobs[slot], c->h_jobs[slot], sizeof(UpdJob) * n,
                        hipMemcpyHostToDevice, st));
  HIP_OK(launch_update_jobs(c->h_jobs[slot], c->d_jobs[slot], n, c->d_total + slot, binned, r,
                            ppt, apply_grid, st));
  HIP_OK(hipEventRecord(c->ev[slot], st));
  c->armed[slot] = true;
  return SKETCH_OK;
}

uint64_t splitmix64_next(uint64_t &state) {
  // SplitMix64 (Steele, Lea and Flood 2014).
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

bool params_ok(const sketch_params_t *p) {
  if (!p) return false;
  const uint32_t g = p->g, k = p->k, r = p->r, al = p->alpha;
  if (g < 32 || g > 65536 || (g & (g - 1))) return false;
  if (k < 5 || k > 24) return false;
  if (r < 3 || r > 8) return false;
  if (al < 1 || al > k) return false;
  if ((r - 2) * al + k < 32) return false;
  if (k - al > 20) return false;
  return true;
}

// A reduced basis of the lattice {(a, y) : y = A a (mod 2^64)} in the
// metric where the box of one row-0 cell, 2^32 wide in a and 2^(64-k) in y,
// is a square (a scaled by 2^(32-k)): Lagrange's reduction, with exact
// 128-bit components and long double only to pick each step's multiple.
// ok only if the kernel's arithmetic holds for it: k <= 20 (row 1's hot
// bitmap in LDS), the determinant is +-2^64, and the components and the
// lines per cell stay small.
Lattice make_lattice(uint64_t A, uint32_t k) {
  Lattice L{};
  if (k > 20) return L;
  typedef __int128 i128;
  const i128 sig = (i128)1 << (32 - k);
  i128 x1 = sig, y1 = (i128)A, x2 = 0, y2 = (i128)1 << 64;
  auto ld = [](i128 v) { return (long double)v; };
  for (int it = 0; it < 256; it++) {
    long double n1 = ld(x1) * ld(x1) + ld(y1) * ld(y1);
    const long double n2 = ld(x2) * ld(x2) + ld(y2) * ld(y2);
    if (n2 < n1) {
      std::swap(x1, x2);
      std::swap(y1, y2);
      n1 = n2;
    }
    const long double mu = roundl((ld(x1) * ld(x2) + ld(y1) * ld(y2)) / n1);
    if (mu == 0) break;
    x2 -= (i128)mu * x1;
    y2 -= (i128)mu * y1;
  }
  if (x1 % sig || x2 % sig) return L;
  const i128 ua = x1 / sig, va = x2 / sig;
  const i128 lim_a = (i128)1 << 40, lim_y = (i128)1 << 58;
  if (ua >= lim_a || ua <= -lim_a || va >= lim_a || va <= -lim_a || y1 >= lim_y ||
      y1 <= -lim_y || y2 >= lim_y || y2 <= -lim_y)
    return L;
  const i128 det = ua * y2 - va * y1;
  const i128 d64 = (i128)1 << 64;
  if (det != d64 && det != -d64) return L;
  L.ua = (int64_t)ua;
  L.uy = (int64_t)y1;
  L.va = (int64_t)va;
  L.vy = (int64_t)y2;
  L.dneg = det < 0;
  // j spans (|u_y| 2^32 + |u_a| 2^(64-k)) / 2^64 over a cell's box; the
  // kernel widens each side by 1 and rounds outwards
  const long double width =
      (fabsl(ld(y1)) * 4294967296.0L + fabsl(ld(ua)) * ldexpl(1.0L, 64 - (int)k)) /
      ldexpl(1.0L, 64);
  if (width > 1e6L) return L;
  L.lines = (uint32_t)floorl(width) + 6;
  // the kernel indexes (cell, line) in 32 bits
  if ((((uint64_t)1 << k) * (uint64_t)L.lines) >> 32) return L;
  L.ok = 1;
  return L;
}

Geom make_geom(const sketch_params_t &p) {
  Geom G{};
  G.g = p.g; G.k = p.k; G.r = p.r; G.alpha = p.alpha;
  G.log2g = 0;
  while ((1u << G.log2g) < p.g) G.log2g++;
  G.wpl = p.g / 32;
  for (uint32_t i = 1; i < 8; i++) G.shift[i] = std::min<uint32_t>((i - 1) * p.alpha, 32);
  uint64_t s = p.seed;
  G.a0 = splitmix64_next(s) | 1ull;
  G.b0 = splitmix64_next(s);
  G.a1 = splitmix64_next(s) | 1ull;
  G.b1 = splitmix64_next(s);
  return G;
}

// Thresholds that depend on theta only (host, float64).
struct Thresholds {
  double e_theta, zmin;
  uint32_t zhot;
};

}  // namespace

// ------------------------------------------------------------------ handle

struct sketch {
  sketch_params_t p;
  Geom G;
  Lattice lat{};                // row 0's cells as lattice boxes (restore)
  uint32_t cand_path = 0;       // SKETCH_OPT_CANDIDATES: 0 auto, 1 join, 2 lattice
  uint32_t join_blocks = 0;     // SKETCH_OPT_JOIN_BLOCKS: 0 = by the last restore's hot lists
  DevCtx *ctx = nullptr;
  mutable Lane lane;            // last work on this sketch (any stream)
  // a restore begun by sketch_restore_batch_begin and not yet ended: its
  // thresholds, and the event that marks the end of its device work
  bool pending = false;
  Thresholds pend_t{};
  hipEvent_t restore_ev = nullptr;
  // SKETCH_OPT_TIMING: events between the restore's phases, and what the
  // last timed restore read
  bool timing = false;
  hipEvent_t tev[6] = {};
  bool timed = false;           // a restore has recorded tev
  bool timed_lez = false;       // ... from the update's zero counts
  int n_cu = 0;
  int grid = 0;                 // blocks of grid-stride kernels
  uint32_t *d_sketch = nullptr;
  size_t words = 0;
  // All zero but not yet written: a reset only sets this. The first binned
  // update then writes every tile from zeros instead of reading it; other
  // work that reads the sketch or sets bits in place writes the zeros first
  // (materialize).
  bool fresh = false;
  // Zeros per LE as the binned update leaves them (when lez_kept(g)). Valid
  // after a binned update of a fresh window from its first pair (which
  // writes every tile) and through later binned updates (which rewrite the
  // counts of every tile they write); anything else that sets bits makes it
  // stale, and the restore then counts zeros in the sketch.
  uint32_t *lez = nullptr;
  bool lez_valid = false;
  // update
  int update_grid = 0;          // blocks of the direct kernel
  int update_check = 1;
  int update_path = 0;          // 0 by size, 1 direct, 2 binned
  size_t binned_min_pairs = 0;
  size_t binned_round = ARENA_MAX_PAIRS;
  uint32_t nbins = 0;
  uint32_t bin_nblk = 0;        // count/scatter blocks per job (hist width)
  uint32_t scatter_ppt = 6;
  uint32_t bin_sample = 0;      // count every n-th batch (0: by the block's batches)
  uint32_t bin_rscale = 0;      // region = estimate * rscale / 64 + pad (0: default)
  uint32_t apply_grid = 0;     // blocks of the apply pass (0: one per item)
  uint32_t *hist = nullptr, *totals = nullptr, *base = nullptr, *item_start = nullptr,
           *xslot = nullptr, *n_items = nullptr, *item_tile = nullptr, *gcur = nullptr,
           *tst = nullptr;
  // restore
  DevState *st = nullptr;
  DevState *h_state = nullptr, *d_h_state = nullptr;   // pinned copy of the device state
  uint4 *h_recs = nullptr, *d_h_recs = nullptr;         // pinned copy of the records
  size_t h_recs_cap = 0;
  uint32_t *hotmask = nullptr, *he = nullptr, *bk_off = nullptr, *bk_cur = nullptr,
           *bk_val = nullptr;
  uint4 *spl_sorted = nullptr;
  size_t spl_sorted_cap = 0;
  // capacities the last enqueued restore ran with (the pools may grow
  // between its launch and its check when restores are batched)
  size_t ran_seg_cap = 0, ran_cand_cap = 0, ran_spl_cap = 0, ran_h_recs_cap = 0;
  int ran_pool = 0;             // the pool that restore ran on
  uint64_t cost_hint = 0;       // the last restore's row-0 cells times their addresses
  uint64_t join_hint = 0;       // the last restore's join wave items of stage 1 (0: none yet)
};

namespace {

void free_sketch(sketch *s) {
  lane_free(s->lane);
  for (hipEvent_t &e : s->tev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (s->restore_ev) (void)hipEventDestroy(s->restore_ev);
  s->restore_ev = nullptr;
  dev_free(s->d_sketch);
  dev_free(s->hist);
  dev_free(s->totals);
  dev_free(s->base);
  dev_free(s->item_start);
  dev_free(s->xslot);
  dev_free(s->n_items);
  dev_free(s->item_tile);
  dev_free(s->gcur);
  dev_free(s->tst);
  dev_free(s->lez);
  dev_free(s->st);
  dev_free(s->hotmask);
  dev_free(s->he);
  dev_free(s->bk_off);
  dev_free(s->bk_cur);
  dev_free(s->bk_val);
  dev_free(s->spl_sorted);
  pinned_free(s->h_state, s->d_h_state);
  pinned_free(s->h_recs, s->d_h_recs);
  s->h_recs_cap = 0;
  ctx_release(s->ctx);
  s->ctx = nullptr;
}

int grow_sorted(sketch *s, size_t need) {
  const size_t cap = std::max(need + need / 2, s->spl_sorted_cap * 2);
  dev_free(s->spl_sorted);
  s->spl_sorted_cap = 0;
  int rc = dev_alloc(&s->spl_sorted, cap, "sorted records");
  if (!rc) s->spl_sorted_cap = cap;
  return rc;
}

RestoreBufs restore_bufs(const sketch *s, const RPool &p) {
  const DevCtx *c = s->ctx;
  RestoreBufs B{};
  B.lez = s->lez_valid ? s->lez : nullptr;
  B.st = s->st;
  B.hotmask = s->hotmask;
  B.he = s->he;
  B.bk_off = s->bk_off;
  B.bk_cur = s->bk_cur;
  B.bk_val = s->bk_val;
  B.part[0] = p.part[0];
  B.part[1] = p.part[1];
  B.segc[0] = p.segc[0];
  B.segc[1] = p.segc[1];
  B.seg_cap = p.seg_cap;
  // fewer join blocks use the first of the pool's segments. Unset, the
  // join takes four blocks per compute unit, or one when the sketch's last
  // restore had fewer stage-1 wave items than compute units: short hot
  // lists leave most of a larger grid idle, and each block still loads its
  // bucket table
  const uint32_t n_cu = c->jblk / 4;
  B.jblk = s->join_blocks ? std::min(s->join_blocks, c->jblk)
           : (s->join_hint && s->join_hint < n_cu) ? n_cu
                                                    : c->jblk;
  B.cand = p.cand;
  B.cand_sorted = p.cand_sorted;
  B.cand_cap = p.cand_cap;
  B.spl = p.spl;
  B.spl_sorted = s->spl_sorted;
  B.spl_cap = std::min(p.spl_cap, s->spl_sorted_cap);
  B.rank = p.rank;
  B.skeys = p.skeys;
  B.h_state = s->d_h_state;
  B.h_recs = s->d_h_recs;
  B.h_recs_cap = s->h_recs_cap;
  B.lat = s->lat;
  B.cand_path = s->cand_path;
  return B;
}

// The records of the restore that just finished into host memory `out`:
// from the pinned copy the restore wrote when it fit, else from the device
// (and the pinned buffer grows for the next restore). Caller holds ctx->mu.
int copy_records(sketch *s, sketch_sp_t *out, size_t n, size_t published_cap, hipStream_t st) {
  static_assert(sizeof(sketch_sp_t) == sizeof(uint4), "record layout");
  if (n == 0) return SKETCH_OK;
  if (n <= published_cap) {
    memcpy(out, s->h_recs, n * sizeof(uint4));
    return SKETCH_OK;
  }
  HIP_OK(hipMemcpyAsync(out, s->spl_sorted, n * sizeof(uint4), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  pinned_free(s->h_recs, s->d_h_recs);
  s->h_recs_cap = 0;
  const size_t cap = n + n / 2;
  int rc = pinned_alloc(&s->h_recs, &s->d_h_recs, cap, "records");
  if (!rc) s->h_recs_cap = cap;
  return rc;
}

void fill_info(const sketch *s, const DevState &st, double zmin, uint32_t zhot,
               sketch_info_t *info) {
  if (!info) return;
  memset(info, 0, sizeof *info);
  for (uint32_t i = 0; i < s->p.r; i++) {
    info->zr[i] = st.zr[i];
    info->he_count[i] = st.he_count[i];
    if (i >= 2 && i + 1 < s->p.r) info->n_partials[i] = st.n_out[i];
  }
  info->n_candidates = st.n_cand;
  info->n_reported = st.n_spl;
  info->psi = st.psi;
  info->d = st.d;
  info->zmin = zmin;
  info->trep = st.trep;
  info->zhot = zhot;
  info->szmax = st.szmax;
}

Thresholds thresholds(const sketch *s, double theta) {
  Thresholds t;
  t.e_theta = exp(-theta / (double)s->p.g);
  t.zmin = (double)s->p.g * t.e_theta;
  // hot <=> z0 < zmin <=> z0 <= ceil(zmin) - 1 for integer z0
  const double zc = ceil(t.zmin) - 1.0;
  t.zhot = zc < 0 ? 0u : (zc > (double)s->p.g ? s->p.g : (uint32_t)zc);
  return t;
}

// Write the zeros of a fresh sketch (on st).
int materialize(sketch *s, hipStream_t st) {
  if (!s->fresh) return SKETCH_OK;
  HIP_OK(launch_fill_u32(s->d_sketch, s->words, 0u, s->grid * 4, st));
  s->fresh = false;
  s->lez_valid = false;
  return SKETCH_OK;
}

// Enqueue the restore kernels on buffers B, whose shared part is ordered by
// `pool`, and the copy of the device state (no wait). Caller holds ctx->mu.

// Enqueue the restore kernels on buffers B, whose shared part is ordered by
// `pool`, and the copy of the device state (no wait). Caller holds ctx->mu.
int restore_launch_on(sketch *s, const RestoreBufs &B, Lane &pool, const Thresholds &t,
                      int estimate, hipStream_t st) {
  int rc = lane_enter(s->lane, st);
  if (!rc) rc = materialize(s, st);
  if (!rc) rc = lane_enter(pool, st);
  if (rc) return rc;
  HIP_OK(launch_restore(s->G, s->d_sketch, B, t.zhot, t.e_theta, estimate, s->grid, st,
                        s->timing ? s->tev : nullptr));
  if (s->timing) {
    s->timed = true;
    s->timed_lez = B.lez != nullptr;
  }
  rc = lane_leave(pool, st);
  if (!rc) rc = lane_leave(s->lane, st);
  return rc;
}

// The restore on restore pool i, enqueued on st.
int restore_launch_pool(sketch *s, const Thresholds &t, int estimate, int i, hipStream_t st) {
  RPool &p = s->ctx->pool[i];
  const RestoreBufs B = restore_bufs(s, p);
  s->ran_seg_cap = B.seg_cap;
  s->ran_cand_cap = B.cand_cap;
  s->ran_spl_cap = B.spl_cap;
  s->ran_h_recs_cap = B.h_recs_cap;
  s->ran_pool = i;
  return restore_launch_on(s, B, p.lane, t, estimate, st);
}

// The restore on the device's first restore pool (the caller's stream).
int restore_launch(sketch *s, const Thresholds &t, int estimate, hipStream_t st) {
  return restore_launch_pool(s, t, estimate, 0, st);
}

// Relative work of a restore of s: its LEs, and the row-0 addresses the
// candidate search covered the last time (|HE(0)| 2^(32-k)).
double restore_cost(const sketch *s) {
  return (double)((size_t)s->p.r << s->p.k) / 4.0 + (double)s->cost_hint;
}

void note_cost(sketch *s, const DevState &h) {
  if (h.saturated) return;
  s->cost_hint = (uint64_t)h.he_count[0] << (32 - s->p.k);
  s->join_hint = std::max<uint64_t>(1, (uint64_t)h.he_count[0] * ((h.he_count[1] + 63) / 64));
}

// Pools of a batch's jobs: the costliest job first, each to the pool with
// the least work so far (longest processing time first); every pool that
// gets a job is made ready. Caller holds c->mu.
int assign_pools(DevCtx *c, const std::vector<const sketch *> &ss, std::vector<int> &pools) {
  const size_t n = ss.size();
  pools.assign(n, 0);
  if (n < 2) return SKETCH_OK;
  std::vector<size_t> order(n);
  for (size_t i = 0; i < n; i++) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return restore_cost(ss[a]) > restore_cost(ss[b]);
  });
  const int np = (int)std::min<size_t>(RESTORE_POOLS, n);
  double load[RESTORE_POOLS] = {};
  for (size_t i : order) {
    int best = 0;
    for (int q = 1; q < np; q++)
      if (load[q] < load[best]) best = q;
    pools[i] = best;
    load[best] += restore_cost(ss[i]);
  }
  for (int q = 1; q < np; q++)
    if (!c->pool[q].ready) {
      int rc = pool_init(c, q, c->pool_entries);
      if (rc) return rc;
    }
  return SKETCH_OK;
}

// The stream that pool i's restores of a batch run on (pool 0: the
// caller's).
hipStream_t pool_stream(const DevCtx *c, int i, hipStream_t st) {
  return i == 0 ? st : c->pool[i].stream;
}

// The pools' streams (used[i] for i >= 1) start after what st holds so far.
hipError_t batch_fork(DevCtx *c, const uint8_t *used, hipStream_t st) {
  bool any = false;
  for (int i = 1; i < RESTORE_POOLS; i++) any = any || used[i];
  if (!any) return hipSuccess;
  hipError_t e = hipEventRecord(c->fork, st);
  for (int i = 1; i < RESTORE_POOLS && e == hipSuccess; i++)
    if (used[i]) e = hipStreamWaitEvent(c->pool[i].stream, c->fork, 0);
  return e;
}

// st continues after what the pools' streams (used[i], i >= 1) hold.
hipError_t batch_join(DevCtx *c, const uint8_t *used, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int i = 1; i < RESTORE_POOLS && e == hipSuccess; i++)
    if (used[i]) {
      e = hipEventRecord(c->pool[i].join, c->pool[i].stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, c->pool[i].join, 0);
    }
  return e;
}

// The restore's shared buffers carved from the no-alloc array at `base`:
// sort ranks, segment counts, candidates and records (each with its sorted
// copy) at fixed sizes, the rest split into the join's partial segments.
RestoreBufs noalloc_bufs(const sketch *s, uint8_t *base) {
  RestoreBufs B = restore_bufs(s, s->ctx->pool[0]);   // every pool buffer replaced below
  const uint32_t jb = s->ctx->jblk;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    uint8_t *p = base + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  B.rank = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * NOALLOC_CAND));
  B.skeys = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * NOALLOC_CAND));
  B.segc[0] = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * jb));
  B.segc[1] = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * jb));
  B.cand = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * NOALLOC_CAND));
  B.cand_sorted = reinterpret_cast<uint32_t *>(take(sizeof(uint32_t) * NOALLOC_CAND));
  B.cand_cap = NOALLOC_CAND;
  B.spl = reinterpret_cast<uint4 *>(take(sizeof(uint4) * NOALLOC_SPL));
  B.spl_sorted = reinterpret_cast<uint4 *>(take(sizeof(uint4) * NOALLOC_SPL));
  B.spl_cap = NOALLOC_SPL;
  B.seg_cap = (NOALLOC_BYTES - off) / (2 * sizeof(uint2) * jb);
  B.part[0] = reinterpret_cast<uint2 *>(base + off);
  B.part[1] = B.part[0] + B.seg_cap * jb;
  return B;
}

// After the state copy has landed: grow any buffer that overflowed.
// *again = a buffer grew, so the restore must run again. Caller holds ctx->mu.
int restore_check(sketch *s, int estimate, bool *again) {
  const DevState &h = *s->h_state;
  DevCtx *c = s->ctx;
  RPool &p = c->pool[s->ran_pool];
  *again = false;
  if (h.saturated) return SKETCH_E_SATURATED;
  note_cost(s, h);
  // a stage overflowed if its count passed the capacity the run had; the
  // buffer grows only if it has not grown enough since
  size_t need_part = 0;
  for (uint32_t i = 2; i + 1 < s->p.r; i++) need_part = std::max<size_t>(need_part, h.seg_max[i]);
  if (need_part > s->ran_seg_cap) {
    if (need_part > p.seg_cap) {
      int rc = grow_partials(c, p, need_part);
      if (rc) return rc;
    }
    *again = true;
  }
  if (h.n_cand > s->ran_cand_cap) {
    if (h.n_cand > p.cand_cap) {
      int rc = grow_cand(c, p, h.n_cand);
      if (rc) return rc;
    }
    *again = true;
  }
  if (estimate && h.n_spl > s->ran_spl_cap) {
    if (h.n_spl > p.spl_cap) {
      int rc = grow_pool_spl(c, p, h.n_spl);
      if (rc) return rc;
    }
    if (h.n_spl > s->spl_sorted_cap) {
      int rc = grow_sorted(s, h.n_spl);
      if (rc) return rc;
    }
    *again = true;
  }
  return SKETCH_OK;
}

// Runs the restore pipeline until every buffer held its output (counts are
// exact on the device even past capacity, so one rerun per grown stage at
// most). Leaves the final state in s->h_state. Caller holds ctx->mu.
int run_restore(sketch *s, const Thresholds &t, int estimate, hipStream_t st) {
  for (int attempt = 0; attempt < 16; attempt++) {
    int rc = restore_launch(s, t, estimate, st);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(st));
    bool again;
    rc = restore_check(s, estimate, &again);
    if (rc || !again) return rc;
  }
  return fail(SKETCH_E_HIP, "restore: capacities did not settle");
}

// ------------------------------------------------------------------ update

UpdJob job_base(const sketch *s) {
  UpdJob J{};
  J.G = s->G;
  J.sk = s->d_sketch;
  J.words = s->words;
  J.nbins = s->nbins;
  J.hstride = s->bin_nblk;
  J.hist = s->hist;
  J.totals = s->totals;
  J.base = s->base;
  J.item_start = s->item_start;
  J.xslot = s->xslot;
  J.item_tile = s->item_tile;
  J.gcur = s->gcur;
  J.tst = s->tst;
  J.lez = s->lez;
  J.n_items = s->n_items;
  J.check = (uint32_t)s->update_check;
  return J;
}

bool wants_binned(const sketch *s, size_t n) {
  if (s->nbins > BIN_MAX) return false;
  return s->update_path == 2 || (s->update_path == 0 && n >= s->binned_min_pairs);
}

// A launch group: jobs that share the kernels (same r, path, check flag,
// scatter batch).
struct Group {
  uint32_t r;
  bool binned;
  uint32_t check;
  uint32_t ppt;
  uint32_t apply_grid;
  bool wide;                    // binned: more than 2048 tiles per sketch
  std::vector<UpdJob> jobs;
  size_t pairs = 0;             // binned: pairs of the jobs (the arena's share)
};

// The scatter batch (pairs per thread) of a binned launch of n jobs with
// the requested setting ppt.
uint32_t launch_ppt(const UpdJob *J, uint32_t n, uint32_t r, uint32_t ppt) {
  uint32_t max_tiles = 0;
  for (uint32_t j = 0; j < n; j++) max_tiles = std::max(max_tiles, J[j].nbins);
  return scatter_ppt(r, max_tiles, ppt);
}

// 32-bit words a binned job takes from the arena's code buffer: its code
// regions and spill area (job_code_words 64-bit words) and its tiles'
// spill-run lists (nbins * dmax uint2), 16-byte aligned.
size_t job_arena_words(const UpdJob &J, uint32_t r, uint32_t ppt) {
  const uint64_t w = code_words_bound(J.n, r, J.nbins, J.nblk, J.chunk);
  const uint64_t dmax = job_batches(J.nblk, J.chunk, ppt);
  return (size_t)(2 * job_code_words(w, J.nbins) + ((2 * J.nbins * dmax + 3) & ~3ull));
}

// Block and tile prefixes of one launch's jobs; for a binned launch, the
// code words and scratch tiles its jobs take from an arena.
void layout_launch(UpdJob *J, uint32_t n, bool binned, uint32_t r, uint32_t ppt, size_t *words,
                   size_t *tiles) {
  uint32_t blk = 0, tile = 0;
  *words = 0;
  *tiles = 0;
  const uint32_t pe = binned ? launch_ppt(J, n, r, ppt) : 0;
  for (uint32_t j = 0; j < n; j++) {
    J[j].blk0 = blk;
    J[j].tile0 = tile;
    blk += J[j].nblk;
    tile += J[j].nbins;
    if (binned) {
      const size_t w = code_words_bound(J[j].n, r, J[j].nbins, J[j].nblk, J[j].chunk);
      *words += job_arena_words(J[j], r, pe);
      *tiles += w / APPLY_ITEM + 1;
    }
  }
}

// Binned jobs' code buffers (regions, spill area, spill-run lists) and
// scratch tiles, packed one after another.
void place_arena(UpdJob *J, uint32_t n, uint32_t r, uint32_t ppt, uint32_t *codes,
                 uint32_t *scratch) {
  const uint32_t pe = launch_ppt(J, n, r, ppt);
  size_t wo = 0, to = 0;
  for (uint32_t j = 0; j < n; j++) {
    const uint64_t w = code_words_bound(J[j].n, r, J[j].nbins, J[j].nblk, J[j].chunk);
    J[j].codes = codes + wo;
    J[j].rcap = job_region_words(w, J[j].nbins);
    J[j].dmax = job_batches(J[j].nblk, J[j].chunk, pe);
    J[j].desc = reinterpret_cast<uint2 *>(codes + wo + 2 * job_code_words(w, J[j].nbins));
    J[j].scratch = scratch + to * (size_t)BIN_TILE_WORDS;
    wo += job_arena_words(J[j], r, pe);
    to += w / APPLY_ITEM + 1;
  }
}

// Launch a group's jobs now (caller holds c->mu), at most MAX_JOBS per
// launch; binned jobs take the device's shared arena.
int flush_group(DevCtx *c, Group &g, hipStream_t st) {
  for (size_t at = 0; at < g.jobs.size(); at += MAX_JOBS) {
    const uint32_t n = (uint32_t)std::min<size_t>(MAX_JOBS, g.jobs.size() - at);
    UpdJob *J = g.jobs.data() + at;
    size_t words, tiles;
    layout_launch(J, n, g.binned, g.r, g.ppt, &words, &tiles);
    if (g.binned) {
      int rc = ensure_arena(c, words, tiles);
      if (rc) return rc;
      place_arena(J, n, g.r, g.ppt, c->codes, c->scratch);
    }
    // only binned launches use the shared arena
    int rc = g.binned ? lane_enter(c->arena_lane, st) : SKETCH_OK;
    if (rc) return rc;
    rc = launch_jobs(c, J, n, g.binned, g.r, g.ppt, g.apply_grid, st);
    if (rc) return rc;
    rc = g.binned ? lane_leave(c->arena_lane, st) : SKETCH_OK;
    if (rc) return rc;
  }
  g.jobs.clear();
  return SKETCH_OK;
}

// Binned jobs share a launch only with sketches of the same tile class: the
// launch's largest sketch picks the scatter variant, and one of more than
// 2048 tiles would hold every job of the launch to its smaller batches.
size_t group_of(std::vector<Group> &groups, const sketch *s, const UpdJob &J, bool binned) {
  const bool wide = binned && s->nbins > 2048;
  for (size_t i = 0; i < groups.size(); i++) {
    const Group &g = groups[i];
    if (g.r == s->p.r && g.binned == binned && g.wide == wide &&
        (binned ? g.ppt == s->scatter_ppt : g.check == J.check))
      return i;
  }
  groups.push_back(Group{s->p.r, binned, J.check, s->scatter_ppt, s->apply_grid, wide, {}});
  return groups.size() - 1;
}

void add_job(std::vector<Group> &groups, const sketch *s, const UpdJob &J, bool binned) {
  Group &g = groups[group_of(groups, s, J, binned)];
  g.apply_grid = g.jobs.empty() ? s->apply_grid
                 : (g.apply_grid == 0 || s->apply_grid == 0) ? 0u
                                                             : std::max(g.apply_grid, s->apply_grid);
  g.jobs.push_back(J);
  if (binned) g.pairs += J.n;
}

// Pairs, blocks and pairs per block of a binned round of m pairs: about
// min_chunk pairs or more per block, at most the sketch's configured
// count. The count samples every BIN_SAMPLE-th batch of a block once the
// job has 256 samples' worth of batches over its blocks (fewer: a smaller
// stride; a block with fewer batches than the stride samples its first).
void bin_shape(const sketch *s, size_t m, size_t min_chunk, UpdJob &J) {
  J.n = m;
  const size_t want = (m + min_chunk - 1) / min_chunk;
  J.nblk = (uint32_t)std::max<size_t>(1, std::min<size_t>(s->bin_nblk, want));
  size_t chunk = (m + J.nblk - 1) / J.nblk;
  chunk += chunk & 1;
  J.chunk = chunk;
  J.nblk = (uint32_t)((m + chunk - 1) / chunk);
  const size_t batches = (chunk + 1024 * s->scatter_ppt - 1) / (1024 * s->scatter_ppt);
  // about 256 sampled batches over the job's blocks at least (32 per XCD
  // group, whose regions the estimates size), at most one in BIN_SAMPLE
  J.sample = s->bin_sample ? s->bin_sample
                           : (uint32_t)std::max<size_t>(
                                 1, std::min<size_t>(BIN_SAMPLE, batches * J.nblk / 256));
  J.rscale = s->bin_rscale;
}

// Checks the jobs of an update of several sketches on one device.
int check_update_jobs(const sketch_update_job_t *jobs, size_t n_jobs, const char *who) {
  if (!jobs) return fail(SKETCH_E_INVAL, "%s: NULL jobs", who);
  const int dev = jobs[0].sketch ? jobs[0].sketch->p.device : -1;
  for (size_t j = 0; j < n_jobs; j++) {
    const sketch *s = jobs[j].sketch;
    if (!s) return fail(SKETCH_E_INVAL, "%s: NULL handle (job %zu)", who, j);
    if (s->p.device != dev) return fail(SKETCH_E_INVAL, "%s: sketches on different devices", who);
    if (jobs[j].n_pairs && !jobs[j].d_pairs)
      return fail(SKETCH_E_INVAL, "%s: NULL pairs (job %zu)", who, j);
    if (((uintptr_t)jobs[j].d_pairs) & 7u)
      return fail(SKETCH_E_INVAL, "%s: pairs must be 8-byte aligned (job %zu)", who, j);
    for (size_t i = 0; i < j; i++)
      if (jobs[i].sketch == s)
        return fail(SKETCH_E_INVAL, "%s: a sketch appears twice (jobs %zu, %zu)", who, i, j);
  }
  return SKETCH_OK;
}

// Splits the update of several distinct sketches into launch groups and
// hands them, in order, to flush(Group&). A pass takes one round of every
// job with pairs left (a job's binned_round at most); a binned launch group
// holds at most ARENA_MAX_PAIRS pairs, and one that is full is flushed
// during the pass, the rest at its end, so a job's rounds run in order.
// Job j's per-sketch arrays come from base(j).
// Whether an update of n pairs at p takes binned rounds from its first pair
// on (no pair goes through the direct kernel first).
bool binned_from_start(const sketch *s, const uint32_t *p, size_t n) {
  return n && wants_binned(s, n) && !(((uintptr_t)p) & 15u);
}

// fresh (may be null): per job, 1 if the job's first binned round starts
// from a fresh sketch (binned_from_start must hold); consumed by that round.
template <class Base, class Flush>
int schedule_update(const sketch_update_job_t *jobs, size_t n_jobs, Base base, Flush flush,
                    char *fresh = nullptr) {
  std::vector<const uint32_t *> ptr(n_jobs);
  std::vector<size_t> left(n_jobs);
  std::vector<char> binned(n_jobs);
  std::vector<Group> groups;
  for (size_t j = 0; j < n_jobs; j++) {
    sketch *s = jobs[j].sketch;
    ptr[j] = jobs[j].d_pairs;
    left[j] = jobs[j].n_pairs;
    binned[j] = left[j] && wants_binned(s, left[j]);
    if (binned[j] && (((uintptr_t)ptr[j]) & 15u)) {
      // the count pass reads pairs 16 bytes at a time: the first pair goes
      // through the direct kernel so the rest starts 16-byte aligned
      UpdJob J = base(j);
      J.pairs = reinterpret_cast<const uint2 *>(ptr[j]);
      J.n = 1;
      J.nblk = 1;
      add_job(groups, s, J, false);
      ptr[j] += 2;
      left[j]--;
    }
  }
  // pairs per block at least: 4096 per binned job of the call, up to 32768.
  // A window alone spreads over many compute units (a 1M-pair window takes
  // 245 blocks, against 31 at 32k pairs per block); the jobs of a batch
  // share them, and more blocks per job would only add per-block work
  size_t n_binned = 0;
  for (size_t j = 0; j < n_jobs; j++) n_binned += binned[j] ? 1 : 0;
  const size_t min_chunk = std::min<size_t>(32768, 4096 * std::max<size_t>(1, n_binned));
  for (;;) {
    bool any = false;
    for (size_t j = 0; j < n_jobs; j++) {
      if (!left[j]) continue;
      sketch *s = jobs[j].sketch;
      UpdJob J = base(j);
      J.pairs = reinterpret_cast<const uint2 *>(ptr[j]);
      if (binned[j]) {
        Group &g = groups[group_of(groups, s, J, true)];
        if (g.pairs >= ARENA_MAX_PAIRS) {
          int rc = flush(g);
          if (rc) return rc;
          g.jobs.clear();
          g.pairs = 0;
        }
        const size_t m = std::min({left[j], s->binned_round, ARENA_MAX_PAIRS - g.pairs});
        bin_shape(s, m, min_chunk, J);
        if (fresh) {
          J.fresh = (uint32_t)fresh[j];
          fresh[j] = 0;
        }
        add_job(groups, s, J, true);
        ptr[j] += 2 * m;
        left[j] -= m;
      } else {
        J.n = left[j];
        J.nblk = (uint32_t)std::max<size_t>(
            1, std::min<size_t>((size_t)s->update_grid, (left[j] + 255) / 256));
        add_job(groups, s, J, false);
        left[j] = 0;
      }
      any = true;
    }
    for (Group &g : groups) {
      if (g.jobs.empty()) continue;
      int rc = flush(g);
      if (rc) return rc;
      g.jobs.clear();
      g.pairs = 0;
    }
    if (!any) break;
  }
  return SKETCH_OK;
}

// Checks the jobs of a batched restore: distinct sketches on one device,
// valid thresholds and outputs.
int check_restore_jobs(const sketch_restore_job_t *jobs, size_t n_jobs, const char *who) {
  if (!jobs) return fail(SKETCH_E_INVAL, "%s: NULL jobs", who);
  const int dev = jobs[0].sketch ? jobs[0].sketch->p.device : -1;
  for (size_t j = 0; j < n_jobs; j++) {
    const sketch_restore_job_t &J = jobs[j];
    if (!J.sketch) return fail(SKETCH_E_INVAL, "%s: NULL handle (job %zu)", who, j);
    if (J.sketch->p.device != dev)
      return fail(SKETCH_E_INVAL, "%s: sketches on different devices", who);
    if (!(J.theta > 0.0) || !isfinite(J.theta))
      return fail(SKETCH_E_INVAL, "%s: theta must be finite and > 0 (job %zu)", who, j);
    if (J.cap && !J.out) return fail(SKETCH_E_INVAL, "%s: NULL out with cap > 0 (job %zu)", who, j);
    for (size_t i = 0; i < j; i++)
      if (jobs[i].sketch == J.sketch)
        return fail(SKETCH_E_INVAL, "%s: a sketch appears twice (jobs %zu, %zu)", who, i, j);
  }
  return SKETCH_OK;
}

// The update of several distinct sketches on one device: every pair of every
// job is applied.
int update_jobs(const sketch_update_job_t *jobs, size_t n_jobs, hipStream_t st) {
  if (n_jobs == 0) return SKETCH_OK;
  int rc = check_update_jobs(jobs, n_jobs, "sketch_update");
  if (rc) return rc;
  DEVICE_GUARD(jobs[0].sketch->p.device);
  DevCtx *c = jobs[0].sketch->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  // a fresh sketch whose update is binned from its first pair skips its
  // zero fill; any other fresh sketch with pairs gets its zeros first
  std::vector<char> fresh(n_jobs, 0);
  for (size_t j = 0; j < n_jobs; j++) {
    sketch *s = jobs[j].sketch;
    if (jobs[j].n_pairs == 0) continue;
    rc = lane_enter(s->lane, st);
    if (rc) return rc;
    const bool binned = binned_from_start(s, jobs[j].d_pairs, jobs[j].n_pairs);
    if (s->fresh && binned) {
      fresh[j] = 1;
      s->fresh = false;
      s->lez_valid = s->lez != nullptr;     // every tile is written
    } else {
      rc = materialize(s, st);
      if (rc) return rc;
      if (!binned) s->lez_valid = false;    // the direct kernel sets bits
    }
  }
  rc = schedule_update(
      jobs, n_jobs, [&](size_t j) { return job_base(jobs[j].sketch); },
      [&](Group &g) { return flush_group(c, g, st); }, fresh.data());
  for (size_t j = 0; j < n_jobs && !rc; j++)
    if (jobs[j].n_pairs) rc = lane_leave(jobs[j].sketch->lane, st);
  return rc;
}


// ------------------------------------------------------------------ plans

}  // namespace

// A fixed batch captured once into a HIP graph (see sketch_plan_create).
// The graph references the sketches and their per-row restore arrays
// (fixed for a handle's life), the plan's own job tables, per-job update
// arrays, device states and sorted outputs, and the device's shared update
// arena and restore pool. The shared buffers can move (another call grows
// them): the plan notes the device context's generation when it captures
// and captures again when it has changed. Launches are ordered against
// other users of the shared buffers by the pool event, outside the graph.
struct PlanJob {
  sketch *s = nullptr;
  const uint32_t *pairs = nullptr;
  size_t n = 0;
  double theta = 0;
  Thresholds t{};
  uint32_t *hist = nullptr, *totals = nullptr, *base = nullptr, *item_start = nullptr,
           *xslot = nullptr, *n_items = nullptr, *item_tile = nullptr, *gcur = nullptr,
           *tst = nullptr;
  DevState *st = nullptr;
  DevState *h_state = nullptr, *d_h_state = nullptr;   // pinned
  uint4 *h_recs = nullptr, *d_h_recs = nullptr;         // pinned
  size_t h_recs_cap = 0, ran_h_recs_cap = 0;
  uint4 *sorted = nullptr;
  size_t sorted_cap = 0;
  size_t ran_spl_cap = 0;       // record capacity the captured restore has
  size_t ran_seg_cap = 0, ran_cand_cap = 0;   // pool capacities of the capture
  int pool = 0;                 // restore pool of the captured restore
  bool eager = false;           // this result comes from an eager rerun
  bool fresh = false;           // RESET plan: the first binned round writes every
                                // tile from zeros, so no zero fill
};

struct PlanLaunch {
  std::vector<UpdJob> h;
  UpdJob *d = nullptr;
  uint32_t *d_total = nullptr;
  bool binned = false;
  uint32_t r = 0, ppt = 0, apply_grid = 0;
};

struct sketch_plan {
  int dev = -1;
  int flags = 0;
  DevCtx *ctx = nullptr;
  std::vector<PlanJob> jobs;
  std::vector<PlanLaunch> launches;
  size_t arena_words = 0, arena_tiles = 0;   // largest launch's arena needs
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool dirty = true;            // a plan-owned buffer changed since the capture
  uint64_t gen = ~0ull;         // device context generation at the capture
  bool ran = false;             // the graph has run at least once
  hipStream_t run_stream = nullptr;
};

namespace {

void plan_free_graph(sketch_plan *P) {
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->exec = nullptr;
  P->graph = nullptr;
  P->dirty = true;
}

void plan_free(sketch_plan *P) {
  plan_free_graph(P);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  for (PlanJob &j : P->jobs) {
    dev_free(j.hist);
    dev_free(j.totals);
    dev_free(j.base);
    dev_free(j.item_start);
    dev_free(j.xslot);
    dev_free(j.n_items);
    dev_free(j.item_tile);
    dev_free(j.gcur);
    dev_free(j.tst);
    dev_free(j.st);
    dev_free(j.sorted);
    pinned_free(j.h_state, j.d_h_state);
    pinned_free(j.h_recs, j.d_h_recs);
  }
  for (PlanLaunch &L : P->launches) {
    dev_free(L.d);
    dev_free(L.d_total);
  }
  ctx_release(P->ctx);
  P->ctx = nullptr;
}

int plan_alloc_sorted(PlanJob &j, size_t cap) {
  dev_free(j.sorted);
  j.sorted_cap = 0;
  int rc = dev_alloc(&j.sorted, cap, "plan sorted records");
  if (!rc) j.sorted_cap = cap;
  return rc;
}

RestoreBufs plan_restore_bufs(const sketch_plan *P, const PlanJob &j) {
  const RPool &pool = P->ctx->pool[j.pool];
  RestoreBufs B = restore_bufs(j.s, pool);    // the sketch's rows, the job's pool
  // the zero counts are known valid at capture only when each run starts
  // the window and its update writes every tile
  B.lez = (P->flags & SKETCH_PLAN_RESET) && j.fresh ? j.s->lez : nullptr;
  B.st = j.st;
  B.spl_sorted = j.sorted;
  B.spl_cap = std::min(pool.spl_cap, j.sorted_cap);
  B.h_state = j.d_h_state;
  B.h_recs = j.d_h_recs;
  B.h_recs_cap = j.h_recs_cap;
  return B;
}

// Enqueue one whole run on st: resets, update launches, restores and the
// copies of the device states.
int plan_enqueue(sketch_plan *P, hipStream_t st) {
  if (P->flags & SKETCH_PLAN_RESET)
    for (PlanJob &j : P->jobs)
      if (!j.fresh) HIP_OK(launch_fill_u32(j.s->d_sketch, j.s->words, 0u, j.s->grid * 4, st));
  for (PlanLaunch &L : P->launches)
    HIP_OK(launch_update_jobs(L.h.data(), L.d, (uint32_t)L.h.size(), L.d_total, L.binned, L.r,
                              L.ppt, L.apply_grid, st));
  if (P->flags & SKETCH_PLAN_RESTORE) {
    std::vector<uint8_t> used(RESTORE_POOLS, 0);
    for (const PlanJob &j : P->jobs) used[j.pool] = 1;
    HIP_OK(batch_fork(P->ctx, used.data(), st));
    for (PlanJob &j : P->jobs) {
      hipStream_t js = pool_stream(P->ctx, j.pool, st);
      HIP_OK(launch_restore(j.s->G, j.s->d_sketch, plan_restore_bufs(P, j), j.t.zhot,
                            j.t.e_theta, 1, j.s->grid, js));
    }
    HIP_OK(batch_join(P->ctx, used.data(), st));
  }
  return SKETCH_OK;
}

// (Re)capture the graph of a run against the shared buffers as they are
// now. Caller holds ctx->mu; no run of the plan is in flight.
int plan_build_graph(sketch_plan *P) {
  DevCtx *c = P->ctx;
  plan_free_graph(P);
  int rc = ensure_arena(c, P->arena_words, P->arena_tiles);
  if (rc) return rc;
  if (P->flags & SKETCH_PLAN_RESTORE) {
    std::vector<const sketch *> ss;
    for (const PlanJob &j : P->jobs) ss.push_back(j.s);
    std::vector<int> pools;
    rc = assign_pools(c, ss, pools);
    if (rc) return rc;
    for (size_t i = 0; i < P->jobs.size(); i++) P->jobs[i].pool = pools[i];
  }
  for (PlanLaunch &L : P->launches) {
    if (!L.binned) continue;
    place_arena(L.h.data(), (uint32_t)L.h.size(), L.r, L.ppt, c->codes, c->scratch);
    HIP_OK(hipMemcpy(L.d, L.h.data(), sizeof(UpdJob) * L.h.size(), hipMemcpyHostToDevice));
  }
  HIP_OK(hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal));
  rc = plan_enqueue(P, P->cap);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(P->cap, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess)
    return fail(SKETCH_E_HIP, "plan: capture failed: %s", hipGetErrorString(e));
  P->graph = g;
  HIP_OK(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
  for (PlanJob &j : P->jobs) {
    const RPool &pool = c->pool[j.pool];
    j.ran_seg_cap = pool.seg_cap;
    j.ran_cand_cap = pool.cand_cap;
    j.ran_spl_cap = std::min(pool.spl_cap, j.sorted_cap);
    j.ran_h_recs_cap = j.h_recs_cap;
  }
  P->gen = c->gen;
  P->dirty = false;
  return SKETCH_OK;
}

}  // namespace

// ===================================================================== ABI

extern "C" {

void sketch_params_default(sketch_params_t *p) {
  if (!p) return;
  p->g = 1024;
  p->k = 14;
  p->r = 5;
  p->alpha = 6;
  p->seed = 0x1803114490000001ull;
  p->device = 0;
}

int sketch_params_check(const sketch_params_t *p) {
  return params_ok(p) ? SKETCH_OK : fail(SKETCH_E_INVAL, "invalid sketch parameters");
}

size_t sketch_bytes(const sketch_params_t *p) {
  if (!params_ok(p)) return 0;
  return (size_t)p->r * ((size_t)1 << p->k) * (p->g / 8);
}

int sketch_create(const sketch_params_t *params, sketch_t **out) {
  if (!out) return fail(SKETCH_E_INVAL, "sketch_create: out is NULL");
  *out = nullptr;
  if (!params_ok(params))
    return fail(SKETCH_E_INVAL,
                "sketch_create: invalid parameters (need g power of two in [32,65536], "
                "5<=k<=24, 3<=r<=8, 1<=alpha<=k, (r-2)*alpha+k>=32, k-alpha<=20)");
  int ndev = 0;
  HIP_OK(hipGetDeviceCount(&ndev));
  if (params->device < 0 || params->device >= ndev)
    return fail(SKETCH_E_INVAL, "sketch_create: device %d of %d", params->device, ndev);
  DEVICE_GUARD(params->device);
  hipDeviceProp_t prop;
  HIP_OK(hipGetDeviceProperties(&prop, params->device));

  sketch *s = new sketch();
  s->p = *params;
  s->G = make_geom(*params);
  s->lat = make_lattice(s->G.a0, params->k);
  s->words = sketch_bytes(params) / 4;
  s->n_cu = prop.multiProcessorCount;
  s->grid = s->n_cu * 8;
  s->update_grid = s->n_cu * 8;
  s->nbins = (uint32_t)((s->words + BIN_TILE_WORDS - 1) / BIN_TILE_WORDS);
  s->bin_nblk = (uint32_t)std::min<int>((int)BIN_BLOCKS_MAX, s->n_cu);
  // one apply workgroup per item: the dispatcher balances uneven tiles
  // (measured 60 us faster than one per compute unit on the 100M window)
  s->apply_grid = 0;
  // measured crossover on MI355X (100M-pair Zipf window): the binned update
  // wins from ~1e5 pairs at k = 14 and ~2e5 at k = 18
  s->binned_min_pairs = std::max<size_t>(s->words / 256, 1 << 14);

  const size_t n_le = (size_t)params->r << params->k;
  const size_t nb = (size_t)1 << (params->k - params->alpha);
  int rc = ctx_acquire(params->device, s->n_cu, &s->ctx);
  if (!rc) rc = lane_init(s->lane);
  if (!rc && hipEventCreateWithFlags(&s->restore_ev, hipEventDisableTiming) != hipSuccess) {
    s->restore_ev = nullptr;
    rc = fail(SKETCH_E_HIP, "sketch_create: hipEventCreate failed");
  }
  if (!rc) rc = dev_alloc(&s->d_sketch, s->words, "sketch");
  if (!rc) rc = dev_alloc(&s->st, 1, "state");
  if (!rc) rc = dev_alloc(&s->hotmask, n_le / 32, "hot bitmap");
  if (!rc) rc = dev_alloc(&s->he, n_le, "hot lists");
  if (!rc) rc = dev_alloc(&s->bk_off, (size_t)params->r * (nb + 1), "bucket offsets");
  if (!rc) rc = dev_alloc(&s->bk_cur, (size_t)params->r * nb, "bucket cursors");
  if (!rc) rc = dev_alloc(&s->bk_val, n_le, "bucket values");
  if (!rc) rc = grow_sorted(s, (size_t)1 << 12);
  if (!rc && s->nbins <= BIN_MAX) {
    rc = dev_alloc(&s->hist, (size_t)s->nbins * s->bin_nblk, "tile counts");
    if (!rc) rc = dev_alloc(&s->totals, s->nbins, "tile totals");
    if (!rc) rc = dev_alloc(&s->base, s->nbins + 1, "tile runs");
    if (!rc) rc = dev_alloc(&s->item_start, s->nbins + 1, "tile items");
    if (!rc) rc = dev_alloc(&s->xslot, s->nbins + 1, "tile scratch slots");
    if (!rc) rc = dev_alloc(&s->item_tile, ITEM_TILE_SLOTS(s->nbins), "item tiles");
    if (!rc) rc = dev_alloc(&s->gcur, (size_t)BIN_GROUPS * s->nbins, "tile region cursors");
    if (!rc) rc = dev_alloc(&s->tst, tile_state_words(s->nbins), "tile regions");
    if (!rc && lez_kept(params->g)) rc = dev_alloc(&s->lez, n_le, "LE zero counts");
    if (!rc) rc = dev_alloc(&s->n_items, 1, "tile item count");
  }
  if (!rc) rc = pinned_alloc(&s->h_state, &s->d_h_state, 1, "state");
  if (!rc) rc = pinned_alloc(&s->h_recs, &s->d_h_recs, (size_t)1 << 12, "records");
  if (!rc) s->h_recs_cap = (size_t)1 << 12;
  if (!rc) {
    hipError_t e = launch_fill_u32(s->d_sketch, s->words, 0u, s->grid, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess)
      rc = fail(SKETCH_E_HIP, "sketch_create: zero fill: %s", hipGetErrorString(e));
  }
  if (rc) {
    free_sketch(s);
    delete s;
    return rc;
  }
  *out = s;
  return SKETCH_OK;
}

void sketch_destroy(sketch_t *s) {
  if (!s) return;
  DeviceGuard guard(s->p.device);
  (void)hipDeviceSynchronize();
  free_sketch(s);
  delete s;
}

int sketch_update(sketch_t *s, const uint32_t *d_pairs, size_t n_pairs, void *hip_stream) {
  if (!s) return fail(SKETCH_E_INVAL, "sketch_update: NULL handle");
  if (n_pairs == 0) return SKETCH_OK;
  const sketch_update_job_t job{s, d_pairs, n_pairs};
  return update_jobs(&job, 1, (hipStream_t)hip_stream);
}

int sketch_update_batch(const sketch_update_job_t *jobs, size_t n_jobs, void *hip_stream) {
  return update_jobs(jobs, n_jobs, (hipStream_t)hip_stream);
}

int sketch_reset(sketch_t *s, void *hip_stream) {
  if (!s) return fail(SKETCH_E_INVAL, "sketch_reset: NULL handle");
  (void)hip_stream;
  s->fresh = true;                  // the zeros are written when needed
  s->lez_valid = false;
  return SKETCH_OK;
}

int sketch_merge(sketch_t *dst, const sketch_t *src, void *hip_stream) {
  if (!dst || !src) return fail(SKETCH_E_INVAL, "sketch_merge: NULL handle");
  if (dst == src) return SKETCH_OK;
  const sketch_params_t &a = dst->p, &b = src->p;
  if (a.g != b.g || a.k != b.k || a.r != b.r || a.alpha != b.alpha || a.seed != b.seed)
    return fail(SKETCH_E_INVAL, "sketch_merge: sketches differ in parameters or seed");
  if (a.device != b.device)
    return fail(SKETCH_E_INVAL, "sketch_merge: sketches on different devices");
  if (src->fresh) return SKETCH_OK;   // OR with zeros
  DEVICE_GUARD(a.device);
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = lane_enter(dst->lane, st);
  if (!rc) rc = lane_enter(src->lane, st);
  if (!rc) rc = materialize(dst, st);
  if (rc) return rc;
  HIP_OK(launch_or_u32(dst->d_sketch, src->d_sketch, dst->words, dst->grid * 4, st));
  dst->lez_valid = false;
  rc = lane_leave(dst->lane, st);
  if (!rc) rc = lane_leave(src->lane, st);
  return rc;
}

int sketch_restore(sketch_t *s, double theta, sketch_sp_t *out, size_t cap, size_t *n_out,
                   sketch_info_t *info, void *hip_stream) {
  if (!s || !n_out) return fail(SKETCH_E_INVAL, "sketch_restore: NULL handle or n_out");
  if (!(theta > 0.0) || !isfinite(theta))
    return fail(SKETCH_E_INVAL, "sketch_restore: theta must be finite and > 0");
  if (cap && !out) return fail(SKETCH_E_INVAL, "sketch_restore: NULL out with cap > 0");
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> lk(s->ctx->mu);
  const Thresholds t = thresholds(s, theta);
  int rc = run_restore(s, t, 1, st);
  if (rc != SKETCH_OK && rc != SKETCH_E_SATURATED) return rc;
  const DevState h = *s->h_state;
  fill_info(s, h, t.zmin, t.zhot, info);
  if (rc == SKETCH_E_SATURATED) {
    *n_out = 0;
    return fail(SKETCH_E_SATURATED, "sketch_restore: a row has no zero bit (psi = 1)");
  }
  *n_out = (size_t)h.n_spl;
  if (h.n_spl > cap)
    return fail(SKETCH_E_CAPACITY, "sketch_restore: %llu records, cap %zu", h.n_spl, cap);
  return copy_records(s, out, (size_t)h.n_spl, s->ran_h_recs_cap, st);
}

int sketch_restore_noalloc(sketch_t *s, double theta, sketch_sp_t *out, size_t cap,
                           size_t *n_out, sketch_info_t *info, void *hip_stream) {
  if (!s || !n_out) return fail(SKETCH_E_INVAL, "sketch_restore_noalloc: NULL handle or n_out");
  if (!(theta > 0.0) || !isfinite(theta))
    return fail(SKETCH_E_INVAL, "sketch_restore_noalloc: theta must be finite and > 0");
  if (cap && !out) return fail(SKETCH_E_INVAL, "sketch_restore_noalloc: NULL out with cap > 0");
  if (s->pending)
    return fail(SKETCH_E_INVAL, "sketch_restore_noalloc: a batched restore of this sketch "
                "was begun and not ended");
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  DevCtx *c = s->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->noalloc) return fail(SKETCH_E_HIP, "sketch_restore_noalloc: no work array on device");
  const Thresholds t = thresholds(s, theta);
  RestoreBufs B = noalloc_bufs(s, c->noalloc);
  // a join whose partial addresses outgrow the array gives way to the
  // lattice search, which makes none (both give the same candidates)
  for (int attempt = 0; attempt < 2; attempt++) {
    int rc = restore_launch_on(s, B, c->noalloc_lane, t, 1, st);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(st));
    const DevState &h = *s->h_state;
    if (h.saturated) break;
    uint32_t seg = 0;
    for (uint32_t i = 2; i + 1 < s->p.r; i++) seg = std::max(seg, h.seg_max[i]);
    if (seg <= B.seg_cap) break;
    if (attempt == 0 && s->lat.ok && B.cand_path != 1) {
      B.cand_path = 2;
      continue;
    }
    return fail(SKETCH_E_CAPACITY, "sketch_restore_noalloc: a join block's %u partial "
                "addresses exceed the work array's %zu", seg, B.seg_cap);
  }
  const DevState h = *s->h_state;
  fill_info(s, h, t.zmin, t.zhot, info);
  if (h.saturated) {
    *n_out = 0;
    return fail(SKETCH_E_SATURATED, "sketch_restore_noalloc: a row has no zero bit (psi = 1)");
  }
  if (h.n_cand > B.cand_cap)
    return fail(SKETCH_E_CAPACITY, "sketch_restore_noalloc: %llu candidates exceed the work "
                "array's %zu", h.n_cand, B.cand_cap);
  if (h.n_spl > B.spl_cap)
    return fail(SKETCH_E_CAPACITY, "sketch_restore_noalloc: %llu records exceed the work "
                "array's %zu", h.n_spl, B.spl_cap);
  *n_out = (size_t)h.n_spl;
  if (h.n_spl > cap)
    return fail(SKETCH_E_CAPACITY, "sketch_restore_noalloc: %llu records, cap %zu", h.n_spl, cap);
  const size_t n = (size_t)h.n_spl;
  if (n <= B.h_recs_cap) {          // k_publish wrote them to the pinned buffer
    if (n) memcpy(out, s->h_recs, n * sizeof(uint4));
    return SKETCH_OK;
  }
  // more than the pinned buffer holds: through it, a buffer's worth at a time
  for (size_t i = 0; i < n; i += B.h_recs_cap) {
    const size_t m = std::min(B.h_recs_cap, n - i);
    HIP_OK(hipMemcpyAsync(s->h_recs, B.spl_sorted + i, m * sizeof(uint4),
                          hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    memcpy(out + i, s->h_recs, m * sizeof(uint4));
  }
  return SKETCH_OK;
}

int sketch_restore_batch_begin(sketch_restore_job_t *jobs, size_t n_jobs, void *hip_stream) {
  if (n_jobs == 0) return SKETCH_OK;
  int rc = check_restore_jobs(jobs, n_jobs, "sketch_restore_batch_begin");
  if (rc) return rc;
  for (size_t j = 0; j < n_jobs; j++)
    if (jobs[j].sketch->pending)
      return fail(SKETCH_E_INVAL, "sketch_restore_batch_begin: job %zu's sketch has a restore "
                  "that was begun and not ended", j);
  DEVICE_GUARD(jobs[0].sketch->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  DevCtx *c = jobs[0].sketch->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  // the jobs spread over the restore pools (pools 1.. on their own streams,
  // forked from st and joined back to it), costliest first in each; every
  // restore enqueued, each one's end marked by its sketch's event
  std::vector<const sketch *> ss(n_jobs);
  for (size_t j = 0; j < n_jobs; j++) ss[j] = jobs[j].sketch;
  std::vector<int> pools;
  rc = assign_pools(c, ss, pools);
  if (rc) return rc;
  std::vector<size_t> order(n_jobs);
  for (size_t j = 0; j < n_jobs; j++) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return restore_cost(ss[a]) > restore_cost(ss[b]);
  });
  uint8_t used[RESTORE_POOLS] = {};
  for (int q : pools) used[q] = 1;
  if (batch_fork(c, used, st) != hipSuccess)
    return fail(SKETCH_E_HIP, "sketch_restore_batch_begin: stream fork failed");
  for (size_t j : order) {
    sketch *s = jobs[j].sketch;
    const hipStream_t js = pool_stream(c, pools[j], st);
    s->pend_t = thresholds(s, jobs[j].theta);
    rc = restore_launch_pool(s, s->pend_t, 1, pools[j], js);
    if (!rc && hipEventRecord(s->restore_ev, js) != hipSuccess)
      rc = fail(SKETCH_E_HIP, "sketch_restore_batch_begin: hipEventRecord failed");
    if (rc) return rc;
    s->pending = true;
  }
  if (batch_join(c, used, st) != hipSuccess)
    return fail(SKETCH_E_HIP, "sketch_restore_batch_begin: stream join failed");
  return SKETCH_OK;
}

int sketch_restore_batch_end(sketch_restore_job_t *jobs, size_t n_jobs, void *hip_stream) {
  if (n_jobs == 0) return SKETCH_OK;
  int rc = check_restore_jobs(jobs, n_jobs, "sketch_restore_batch_end");
  if (rc) return rc;
  for (size_t j = 0; j < n_jobs; j++)
    if (!jobs[j].sketch->pending)
      return fail(SKETCH_E_INVAL, "sketch_restore_batch_end: job %zu's sketch has no begun "
                  "restore", j);
  DEVICE_GUARD(jobs[0].sketch->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  DevCtx *c = jobs[0].sketch->ctx;
  int first_err = SKETCH_OK;
  for (size_t j = 0; j < n_jobs; j++) {
    sketch_restore_job_t &J = jobs[j];
    sketch *s = J.sketch;
    // wait for this restore only (outside the lock: other work may be queued)
    rc = hipEventSynchronize(s->restore_ev) == hipSuccess
             ? SKETCH_OK : fail(SKETCH_E_HIP, "sketch_restore_batch_end: hipEventSynchronize");
    std::lock_guard<std::mutex> lk(c->mu);
    s->pending = false;
    bool again = false;
    if (rc == SKETCH_OK) rc = restore_check(s, 1, &again);
    if (rc == SKETCH_OK && again) rc = run_restore(s, s->pend_t, 1, st);   // this job alone
    const DevState h = *s->h_state;
    if (rc == SKETCH_OK || rc == SKETCH_E_SATURATED)
      fill_info(s, h, s->pend_t.zmin, s->pend_t.zhot, J.info);
    J.n_out = rc == SKETCH_OK ? (size_t)h.n_spl : 0;
    if (rc == SKETCH_OK && h.n_spl > J.cap) rc = SKETCH_E_CAPACITY;
    if (rc == SKETCH_OK)
      rc = copy_records(s, J.out, (size_t)h.n_spl, s->ran_h_recs_cap, st);
    J.status = rc;
    if (rc && !first_err) first_err = rc;
  }
  if (first_err)
    return fail(first_err, "sketch_restore_batch: a job failed (see each job's status)");
  return SKETCH_OK;
}

int sketch_restore_batch(sketch_restore_job_t *jobs, size_t n_jobs, void *hip_stream) {
  int rc = sketch_restore_batch_begin(jobs, n_jobs, hip_stream);
  if (rc) return rc;
  return sketch_restore_batch_end(jobs, n_jobs, hip_stream);
}

int sketch_candidates(sketch_t *s, double theta, uint32_t *out, size_t cap, size_t *n_out,
                      void *hip_stream) {
  if (!s || !n_out) return fail(SKETCH_E_INVAL, "sketch_candidates: NULL handle or n_out");
  if (!(theta > 0.0) || !isfinite(theta))
    return fail(SKETCH_E_INVAL, "sketch_candidates: theta must be finite and > 0");
  if (cap && !out) return fail(SKETCH_E_INVAL, "sketch_candidates: NULL out with cap > 0");
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> lk(s->ctx->mu);
  int rc = run_restore(s, thresholds(s, theta), 0, st);
  if (rc == SKETCH_E_SATURATED) {
    *n_out = 0;
    return fail(SKETCH_E_SATURATED, "sketch_candidates: a row has no zero bit (psi = 1)");
  }
  if (rc) return rc;
  const DevState h = *s->h_state;
  *n_out = (size_t)h.n_cand;
  if (h.n_cand > cap)
    return fail(SKETCH_E_CAPACITY, "sketch_candidates: %llu candidates, cap %zu", h.n_cand, cap);
  if (h.n_cand)
    HIP_OK(hipMemcpyAsync(out, s->ctx->pool[0].cand_sorted, h.n_cand * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return SKETCH_OK;
}

int sketch_set_option(sketch_t *s, int option, int64_t value) {
  if (!s) return fail(SKETCH_E_INVAL, "sketch_set_option: NULL handle");
  switch (option) {
    case SKETCH_OPT_UPDATE_PATH:
      if (value < 0 || value > 2) break;
      if (value == 2 && s->nbins > BIN_MAX)
        return fail(SKETCH_E_INVAL, "sketch_set_option: sketch too large for the binned update");
      s->update_path = (int)value;
      return SKETCH_OK;
    case SKETCH_OPT_BINNED_MIN_PAIRS:
      if (value < 0) break;
      s->binned_min_pairs = (size_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_UPDATE_GRID:
      if (value < 1 || value > (1 << 20)) break;
      s->update_grid = (int)value;
      return SKETCH_OK;
    case SKETCH_OPT_UPDATE_CHECK:
      if (value < 0 || value > 1) break;
      s->update_check = (int)value;
      return SKETCH_OK;
    case SKETCH_OPT_SCATTER_PPT:
      if (value != 2 && value != 4 && value != 6) break;
      s->scatter_ppt = (uint32_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_BINNED_BLOCKS: {
      if (value < 1 || value > (int64_t)BIN_BLOCKS_MAX) break;
      if (s->hist && (uint32_t)value > s->bin_nblk) {
        // per-tile counts are [tiles][blocks]: widen (after pending work)
        DEVICE_GUARD(s->p.device);
        HIP_OK(hipDeviceSynchronize());
        dev_free(s->hist);
        int rc = dev_alloc(&s->hist, (size_t)s->nbins * (size_t)value, "tile counts");
        if (rc) return rc;
      }
      s->bin_nblk = (uint32_t)value;
      return SKETCH_OK;
    }
    case SKETCH_OPT_APPLY_BLOCKS:
      if (value < 0 || value > (1 << 20)) break;
      s->apply_grid = (uint32_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_BINNED_ROUND:
      if (value < 1024 || (uint64_t)value > ARENA_MAX_PAIRS) break;
      s->binned_round = (size_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_BINNED_SAMPLE:
      if (value < 0 || value > 1024) break;
      s->bin_sample = (uint32_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_BINNED_REGIONS:
      if (value < 0 || value > 1024) break;
      s->bin_rscale = (uint32_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_JOIN_BLOCKS:
      if (value < 0 || value > (int64_t)s->ctx->jblk) break;
      s->join_blocks = (uint32_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_CANDIDATES:
      if (value < 0 || value > 2) break;
      if (value == 2 && !s->lat.ok)
        return fail(SKETCH_E_INVAL, "sketch_set_option: the lattice search needs k <= 20");
      s->cand_path = (uint32_t)value;
      return SKETCH_OK;
    case SKETCH_OPT_TIMING:
      if (value < 0 || value > 1) break;
      if (value && !s->tev[0]) {
        DEVICE_GUARD(s->p.device);
        for (hipEvent_t &e : s->tev)
          if (hipEventCreate(&e) != hipSuccess) {
            e = nullptr;
            return fail(SKETCH_E_HIP, "sketch_set_option: hipEventCreate failed");
          }
      }
      s->timing = value != 0;
      s->timed = false;
      return SKETCH_OK;
    case SKETCH_OPT_TRIM_POOLS: {
      if (value < 0 || value > (1 << 24)) break;
      DEVICE_GUARD(s->p.device);
      std::lock_guard<std::mutex> lk(s->ctx->mu);
      return trim_pools(s->ctx, (size_t)value);
    }
    default:
      return fail(SKETCH_E_INVAL, "sketch_set_option: unknown option %d", option);
  }
  return fail(SKETCH_E_INVAL, "sketch_set_option: bad value %lld for option %d",
              (long long)value, option);
}

int sketch_timings(sketch_t *s, sketch_timings_t *out) {
  if (!s || !out) return fail(SKETCH_E_INVAL, "sketch_timings: NULL argument");
  if (!s->timed) return fail(SKETCH_E_INVAL, "sketch_timings: no timed restore has run");
  DEVICE_GUARD(s->p.device);
  HIP_OK(hipEventSynchronize(s->tev[5]));
  float ms[5];
  for (int i = 0; i < 5; i++) HIP_OK(hipEventElapsedTime(&ms[i], s->tev[i], s->tev[i + 1]));
  const DevState &h = *s->h_state;
  memset(out, 0, sizeof *out);
  out->hot_scan_ms = ms[0];
  out->rows_ms = ms[1];
  out->join_ms = ms[2];
  out->estimate_ms = ms[3];
  out->sort_publish_ms = ms[4];
  const uint64_t n_le = (uint64_t)s->p.r << s->p.k;
  out->hot_scan_bytes = s->timed_lez ? n_le * 4 : n_le * (s->p.g / 8);
  if (!h.saturated) {
    out->search = h.search;
    if (h.search == 2) {
      // every address of every hot row-0 LE: 2^(32-k) per LE
      out->lattice_points = (uint64_t)h.he_count[0] << (32 - s->p.k);
      out->join_outputs = h.n_cand;
    } else {
      // stage 1 probes every (CL_0, CL_1); stage i probes stage i-1's outputs
      uint64_t probes = (uint64_t)h.he_count[0] * h.he_count[1], outputs = 0;
      for (uint32_t i = 2; i + 1 < s->p.r; i++) {
        outputs += h.n_out[i];
        probes += h.n_out[i];
      }
      out->join_probes = probes;
      out->join_outputs = outputs + h.n_cand;
    }
    out->estimate_bytes = h.n_cand * (uint64_t)s->p.r * (s->p.g / 8);
  }
  return SKETCH_OK;
}

int sketch_download(const sketch_t *s, uint32_t *host_words, size_t n_words, void *hip_stream) {
  if (!s || !host_words) return fail(SKETCH_E_INVAL, "sketch_download: NULL argument");
  if (n_words != s->words)
    return fail(SKETCH_E_INVAL, "sketch_download: n_words %zu, sketch has %zu", n_words, s->words);
  if (s->fresh) {                   // all zero, not yet written
    memset(host_words, 0, n_words * 4);
    return SKETCH_OK;
  }
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = lane_enter(s->lane, st);
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(host_words, s->d_sketch, n_words * 4, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return SKETCH_OK;
}

int sketch_upload(sketch_t *s, const uint32_t *host_words, size_t n_words, void *hip_stream) {
  if (!s || !host_words) return fail(SKETCH_E_INVAL, "sketch_upload: NULL argument");
  if (n_words != s->words)
    return fail(SKETCH_E_INVAL, "sketch_upload: n_words %zu, sketch has %zu", n_words, s->words);
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  int rc = lane_enter(s->lane, st);
  if (rc) return rc;
  HIP_OK(hipMemcpyAsync(s->d_sketch, host_words, n_words * 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  s->fresh = false;
  s->lez_valid = false;
  return SKETCH_OK;
}


// ------------------------------------------------------------------ plans

int sketch_plan_create(const sketch_plan_job_t *jobs, size_t n_jobs, int flags,
                       sketch_plan_t **out) {
  if (!out) return fail(SKETCH_E_INVAL, "sketch_plan_create: out is NULL");
  *out = nullptr;
  if (n_jobs == 0 || !jobs) return fail(SKETCH_E_INVAL, "sketch_plan_create: no jobs");
  if (flags & ~(SKETCH_PLAN_RESET | SKETCH_PLAN_RESTORE))
    return fail(SKETCH_E_INVAL, "sketch_plan_create: unknown flags 0x%x", flags);
  std::vector<sketch_update_job_t> uj(n_jobs);
  for (size_t j = 0; j < n_jobs; j++) {
    uj[j] = sketch_update_job_t{jobs[j].sketch, jobs[j].d_pairs, jobs[j].n_pairs};
    if ((flags & SKETCH_PLAN_RESTORE) && (!(jobs[j].theta > 0.0) || !isfinite(jobs[j].theta)))
      return fail(SKETCH_E_INVAL, "sketch_plan_create: theta must be finite and > 0 (job %zu)",
                  j);
  }
  int rc = check_update_jobs(uj.data(), n_jobs, "sketch_plan_create");
  if (rc) return rc;
  const int dev = jobs[0].sketch->p.device;
  DEVICE_GUARD(dev);
  DevCtx *c = jobs[0].sketch->ctx;
  sketch_plan *P = new sketch_plan();
  P->dev = dev;
  P->flags = flags;
  {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    c->refs++;
  }
  P->ctx = c;
  P->jobs.resize(n_jobs);
  for (size_t j = 0; j < n_jobs && !rc; j++) {
    PlanJob &pj = P->jobs[j];
    sketch *s = jobs[j].sketch;
    pj.s = s;
    pj.pairs = jobs[j].d_pairs;
    pj.n = jobs[j].n_pairs;
    pj.theta = jobs[j].theta;
    pj.t = thresholds(s, pj.theta > 0 ? pj.theta : 1.0);
    if (s->nbins <= BIN_MAX) {
      rc = dev_alloc(&pj.hist, (size_t)s->nbins * s->bin_nblk, "plan tile counts");
      if (!rc) rc = dev_alloc(&pj.totals, s->nbins, "plan tile totals");
      if (!rc) rc = dev_alloc(&pj.base, s->nbins + 1, "plan tile runs");
      if (!rc) rc = dev_alloc(&pj.item_start, s->nbins + 1, "plan tile items");
      if (!rc) rc = dev_alloc(&pj.xslot, s->nbins + 1, "plan tile scratch slots");
      if (!rc) rc = dev_alloc(&pj.item_tile, ITEM_TILE_SLOTS(s->nbins), "plan item tiles");
      if (!rc) rc = dev_alloc(&pj.gcur, (size_t)BIN_GROUPS * s->nbins, "plan tile region cursors");
      if (!rc) rc = dev_alloc(&pj.tst, tile_state_words(s->nbins), "plan tile regions");
      if (!rc) rc = dev_alloc(&pj.n_items, 1, "plan tile item count");
    }
    if (!rc) rc = dev_alloc(&pj.st, 1, "plan state");
    if (!rc) rc = plan_alloc_sorted(pj, std::max<size_t>(s->spl_sorted_cap, (size_t)1 << 12));
    if (!rc) rc = pinned_alloc(&pj.h_state, &pj.d_h_state, 1, "plan state");
    if (!rc) rc = pinned_alloc(&pj.h_recs, &pj.d_h_recs, pj.sorted_cap, "plan records");
    if (!rc) pj.h_recs_cap = pj.sorted_cap;
  }
  if (!rc && hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess) {
    P->cap = nullptr;
    rc = fail(SKETCH_E_HIP, "plan: hipStreamCreate failed");
  }
  std::vector<char> fresh(n_jobs, 0);
  if (flags & SKETCH_PLAN_RESET)
    for (size_t j = 0; j < n_jobs; j++) {
      P->jobs[j].fresh = binned_from_start(uj[j].sketch, uj[j].d_pairs, uj[j].n_pairs);
      fresh[j] = P->jobs[j].fresh;
    }
  if (!rc) {
    std::lock_guard<std::mutex> lk(c->mu);
    // the update launches, with this plan's per-job arrays
    rc = schedule_update(
        uj.data(), n_jobs,
        [&](size_t j) {
          UpdJob J = job_base(uj[j].sketch);
          const PlanJob &pj = P->jobs[j];
          J.hist = pj.hist;
          J.totals = pj.totals;
          J.base = pj.base;
          J.item_start = pj.item_start;
          J.xslot = pj.xslot;
          J.n_items = pj.n_items;
          J.item_tile = pj.item_tile;
          J.gcur = pj.gcur;
          J.tst = pj.tst;
          return J;
        },
        [&](Group &g) {
          for (size_t at = 0; at < g.jobs.size(); at += MAX_JOBS) {
            const uint32_t n = (uint32_t)std::min<size_t>(MAX_JOBS, g.jobs.size() - at);
            PlanLaunch L;
            L.h.assign(g.jobs.begin() + at, g.jobs.begin() + at + n);
            size_t words, tiles;
            layout_launch(L.h.data(), n, g.binned, g.r, g.ppt, &words, &tiles);
            P->arena_words = std::max(P->arena_words, words);
            P->arena_tiles = std::max(P->arena_tiles, tiles);
            L.binned = g.binned;
            L.r = g.r;
            L.ppt = g.ppt;
            L.apply_grid = g.apply_grid;
            P->launches.push_back(std::move(L));
          }
          return SKETCH_OK;
        },
        fresh.data());
    for (size_t i = 0; i < P->launches.size() && !rc; i++) {
      PlanLaunch &L = P->launches[i];
      rc = dev_alloc(&L.d, L.h.size(), "plan job table");
      if (!rc) rc = dev_alloc(&L.d_total, 1, "plan item total");
      if (!rc) {
        hipError_t e = hipMemcpy(L.d, L.h.data(), sizeof(UpdJob) * L.h.size(),
                                 hipMemcpyHostToDevice);
        if (e != hipSuccess)
          rc = fail(SKETCH_E_HIP, "plan: job table upload: %s", hipGetErrorString(e));
      }
    }
    if (!rc) rc = pools_idle(c);          // nothing else uses the shared buffers now
    if (!rc) rc = arena_idle(c);
    if (!rc) rc = plan_build_graph(P);
  }
  if (rc) {
    plan_free(P);
    delete P;
    return rc;
  }
  *out = P;
  return SKETCH_OK;
}

int sketch_plan_run(sketch_plan_t *P, void *hip_stream) {
  if (!P) return fail(SKETCH_E_INVAL, "sketch_plan_run: NULL plan");
  DEVICE_GUARD(P->dev);
  DevCtx *c = P->ctx;
  hipStream_t st = (hipStream_t)hip_stream;
  std::lock_guard<std::mutex> lk(c->mu);
  if (P->dirty || P->gen != c->gen ||
      c->codes_cap < P->arena_words || c->scratch_tiles < P->arena_tiles) {
    if (P->ran) HIP_OK(hipStreamSynchronize(P->run_stream));   // the old graph is done
    int rc = pools_idle(c);
    if (!rc) rc = arena_idle(c);
    if (!rc) rc = plan_build_graph(P);
    if (rc) return rc;
  }
  // a plan that does not reset works on the sketches as they are: write the
  // zeros of fresh ones first; a resetting plan leaves none fresh
  for (PlanJob &j : P->jobs) {
    int rc = lane_enter(j.s->lane, st);
    if (rc) return rc;
    if (P->flags & SKETCH_PLAN_RESET) {
      j.s->fresh = false;
      j.s->lez_valid = j.fresh && j.s->lez;
    } else {
      int rc = materialize(j.s, st);
      if (rc) return rc;
      j.s->lez_valid = false;
    }
  }
  int rc = SKETCH_OK;
  for (RPool &p : c->pool)
    if (!rc && p.ready) rc = lane_enter(p.lane, st);
  if (!rc) rc = lane_enter(c->arena_lane, st);
  if (rc) return rc;
  HIP_OK(hipGraphLaunch(P->exec, st));
  for (RPool &p : c->pool)
    if (!rc && p.ready) rc = lane_leave(p.lane, st);
  if (!rc) rc = lane_leave(c->arena_lane, st);
  for (PlanJob &j : P->jobs)
    if (!rc) rc = lane_leave(j.s->lane, st);
  if (rc) return rc;
  P->ran = true;
  P->run_stream = st;
  return SKETCH_OK;
}

int sketch_plan_results(sketch_plan_t *P, sketch_restore_job_t *out, size_t n_out,
                        void *hip_stream) {
  if (!P) return fail(SKETCH_E_INVAL, "sketch_plan_results: NULL plan");
  if (!(P->flags & SKETCH_PLAN_RESTORE))
    return fail(SKETCH_E_INVAL, "sketch_plan_results: the plan has no restore");
  if (n_out != P->jobs.size() || !out)
    return fail(SKETCH_E_INVAL, "sketch_plan_results: need %zu result slots", P->jobs.size());
  for (size_t j = 0; j < n_out; j++) {
    if (out[j].sketch != P->jobs[j].s)
      return fail(SKETCH_E_INVAL, "sketch_plan_results: slot %zu is for another sketch", j);
    if (out[j].cap && !out[j].out)
      return fail(SKETCH_E_INVAL, "sketch_plan_results: NULL out with cap > 0 (slot %zu)", j);
  }
  if (!P->ran) return fail(SKETCH_E_INVAL, "sketch_plan_results: the plan has not run");
  DEVICE_GUARD(P->dev);
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_OK(hipStreamSynchronize(P->run_stream));
  HIP_OK(hipStreamSynchronize(st));
  DevCtx *c = P->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  int first_err = SKETCH_OK;
  for (size_t j = 0; j < n_out; j++) {
    PlanJob &pj = P->jobs[j];
    sketch *s = pj.s;
    sketch_restore_job_t &J = out[j];
    J.theta = pj.theta;
    const DevState *h = pj.h_state;
    const uint4 *src = pj.sorted;
    int rc = SKETCH_OK;
    pj.eager = false;
    note_cost(s, *h);
    if (h->saturated) {
      rc = SKETCH_E_SATURATED;
    } else {
      size_t need_part = 0;
      for (uint32_t i = 2; i + 1 < s->p.r; i++)
        need_part = std::max<size_t>(need_part, h->seg_max[i]);
      // a stage overflowed if its count passed the capacity the graph ran
      // with; the shared buffers grow as for an eager restore (which moves
      // them, so the next run captures again) and this job runs again alone
      if (need_part > pj.ran_seg_cap || h->n_cand > pj.ran_cand_cap ||
          h->n_spl > pj.ran_spl_cap) {
        if (h->n_spl > pj.sorted_cap) {
          rc = plan_alloc_sorted(pj, grown(h->n_spl, pj.sorted_cap));
          P->dirty = true;
        }
        // the job's pool grows for the next runs (a move recaptures the graph)
        RPool &pool = c->pool[pj.pool];
        if (!rc && need_part > pool.seg_cap) rc = grow_partials(c, pool, need_part);
        if (!rc && h->n_cand > pool.cand_cap) rc = grow_cand(c, pool, h->n_cand);
        if (!rc && h->n_spl > pool.spl_cap) rc = grow_pool_spl(c, pool, h->n_spl);
        if (!rc) rc = run_restore(s, pj.t, 1, st);
        h = s->h_state;
        src = s->spl_sorted;
        pj.eager = true;
      }
    }
    if (rc == SKETCH_OK || rc == SKETCH_E_SATURATED)
      fill_info(s, *h, pj.t.zmin, pj.t.zhot, J.info);
    const size_t n = rc == SKETCH_OK ? (size_t)h->n_spl : 0;
    J.n_out = n;
    if (rc == SKETCH_OK && n > J.cap) rc = SKETCH_E_CAPACITY;
    if (rc == SKETCH_OK && n) {
      if (pj.eager) {
        rc = copy_records(s, J.out, n, s->ran_h_recs_cap, st);   // the sketch's own copy
      } else if (n <= pj.ran_h_recs_cap) {
        memcpy(J.out, pj.h_recs, n * sizeof(uint4));
      } else {
        // more records than the pinned copy holds: from the device, and a
        // larger pinned copy for the next runs (the graph is captured again)
        hipError_t e = hipMemcpyAsync(J.out, src, n * sizeof(uint4), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = SKETCH_E_HIP;
        if (!rc && n > pj.h_recs_cap) {
          pinned_free(pj.h_recs, pj.d_h_recs);
          pj.h_recs_cap = 0;
          rc = pinned_alloc(&pj.h_recs, &pj.d_h_recs, n + n / 2, "plan records");
          if (!rc) pj.h_recs_cap = n + n / 2;
          P->dirty = true;
        }
      }
    }
    J.status = rc;
    if (rc && !first_err) first_err = rc;
  }
  HIP_OK(hipStreamSynchronize(st));
  if (first_err)
    return fail(first_err, "sketch_plan_results: a job failed (see each job's status)");
  return SKETCH_OK;
}

size_t sketch_plan_launches(const sketch_plan_t *P) { return P ? P->launches.size() : 0; }

void sketch_plan_destroy(sketch_plan_t *P) {
  if (!P) return;
  DeviceGuard guard(P->dev);
  (void)hipDeviceSynchronize();
  plan_free(P);
  delete P;
}

const char *sketch_last_error(void) { return g_err.c_str(); }

}  // extern "C"

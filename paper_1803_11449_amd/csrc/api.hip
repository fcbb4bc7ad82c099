// C ABI of libddhf (declared in include/ddhf.h): handle lifetime, argument
// checks, device memory, and the host side of the restore (capacity growth
// and the copies to the caller).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "ddhf.h"
#include "ddhf_internal.h"

using namespace ddhf;

struct sketch {
  sketch_params_t p;
  Geom G;
  uint32_t *d_sketch = nullptr;
  size_t words = 0;
  RestoreBufs B{};
  DevState *h_state = nullptr;  // pinned host copy of the device state
  int n_cu = 0;
  int grid = 0;          // blocks for grid-stride kernels
  int update_grid = 0;
  int update_variant = 1;
  int update_path = 0;   // 0 auto, 1 direct, 2 binned
  size_t binned_min_pairs = 0;
  size_t binned_round = (size_t)1 << 27;  // pairs per binned round (codes < 2^32)
  uint32_t nbins = 0;
  BinBufs BB{};
};

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

// Makes params.device current for the lifetime of the guard and puts the
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

template <typename T>
int dev_alloc(T **p, size_t count, const char *what) {
  *p = nullptr;
  hipError_t e = hipMalloc((void **)p, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? SKETCH_E_NOMEM : SKETCH_E_HIP,
                "hipMalloc(%s, %zu bytes): %s", what, count * sizeof(T),
                hipGetErrorString(e));
  }
  return SKETCH_OK;
}

template <typename T>
void dev_free(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

void free_all(sketch *s) {
  dev_free(s->d_sketch);
  RestoreBufs &B = s->B;
  dev_free(B.st);
  dev_free(B.hotmask);
  dev_free(B.he);
  dev_free(B.bk_off);
  dev_free(B.bk_cur);
  dev_free(B.bk_val);
  dev_free(B.part[0]);
  dev_free(B.part[1]);
  dev_free(B.segc[0]);
  dev_free(B.segc[1]);
  dev_free(B.cand);
  dev_free(B.cand_sorted);
  dev_free(B.rank);
  dev_free(B.spl);
  dev_free(B.spl_sorted);
  if (s->h_state) (void)hipHostFree(s->h_state);
  s->h_state = nullptr;
  BinBufs &BB = s->BB;
  dev_free(BB.hist);
  dev_free(BB.totals);
  dev_free(BB.base);
  dev_free(BB.item_start);
  dev_free(BB.xslot);
  dev_free(BB.n_items);
  dev_free(BB.codes);
  dev_free(BB.scratch);
  BB.codes_cap = 0;
}

// Codes buffer of the binned update for rounds of `pairs` pairs.
int ensure_codes(sketch *s, size_t pairs, hipStream_t st) {
  BinBufs &BB = s->BB;
  const size_t need = pairs * s->p.r;
  if (BB.codes_cap >= need) return SKETCH_OK;
  HIP_OK(hipStreamSynchronize(st));
  dev_free(BB.codes);
  dev_free(BB.scratch);
  BB.codes_cap = 0;
  int rc = dev_alloc(&BB.codes, need, "update codes");
  if (rc) return rc;
  // a tile cut into j items needs j-1 scratch tiles; j-1 < codes/APPLY_ITEM
  rc = dev_alloc(&BB.scratch, (need / APPLY_ITEM + 1) * (size_t)BIN_TILE_WORDS,
                 "update scratch tiles");
  if (rc) return rc;
  BB.codes_cap = need;
  return SKETCH_OK;
}

// Partial-address buffers: jblk segments of seg_cap entries each.
int grow_partials(sketch *s, size_t seg_need) {
  RestoreBufs &B = s->B;
  const size_t cap = std::max(seg_need + seg_need / 2, B.seg_cap * 2);
  dev_free(B.part[0]);
  dev_free(B.part[1]);
  B.seg_cap = 0;
  int rc = dev_alloc(&B.part[0], cap * B.jblk, "partials");
  if (rc) return rc;
  rc = dev_alloc(&B.part[1], cap * B.jblk, "partials");
  if (rc) return rc;
  B.seg_cap = cap;
  return SKETCH_OK;
}

int grow_cand(sketch *s, size_t need) {
  RestoreBufs &B = s->B;
  size_t cap = std::max(need + need / 2, B.cand_cap * 2);
  dev_free(B.cand);
  dev_free(B.cand_sorted);
  B.cand_cap = 0;
  int rc = dev_alloc(&B.cand, cap, "candidates");
  if (rc) return rc;
  rc = dev_alloc(&B.cand_sorted, cap, "candidates");
  if (rc) return rc;
  B.cand_cap = cap;
  return SKETCH_OK;
}

int grow_spl(sketch *s, size_t need) {
  RestoreBufs &B = s->B;
  size_t cap = std::max(need + need / 2, B.spl_cap * 2);
  dev_free(B.spl);
  dev_free(B.spl_sorted);
  B.spl_cap = 0;
  int rc = dev_alloc(&B.spl, cap, "records");
  if (rc) return rc;
  rc = dev_alloc(&B.spl_sorted, cap, "records");
  if (rc) return rc;
  B.spl_cap = cap;
  return SKETCH_OK;
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

// Runs the restore pipeline until every buffer held its output (counts are
// exact on the device even past capacity, so one rerun per grown stage at
// most). Leaves the final state in s->h_state.
int run_restore(sketch *s, double theta, int estimate, hipStream_t st, double *zmin_out,
                uint32_t *zhot_out) {
  const double e_theta = exp(-theta / (double)s->p.g);
  const double zmin = (double)s->p.g * e_theta;
  // hot <=> z0 < zmin <=> z0 <= ceil(zmin) - 1 for integer z0
  const double zc = ceil(zmin) - 1.0;
  const uint32_t zhot = zc < 0 ? 0u : (zc > (double)s->p.g ? s->p.g : (uint32_t)zc);
  *zmin_out = zmin;
  *zhot_out = zhot;
  for (int attempt = 0; attempt < 16; attempt++) {
    HIP_OK(launch_restore(s->G, s->d_sketch, s->B, zhot, e_theta, estimate, s->grid, st));
    HIP_OK(hipMemcpyAsync(s->h_state, s->B.st, sizeof(DevState), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const DevState &h = *s->h_state;
    if (h.saturated) return SKETCH_E_SATURATED;
    bool again = false;
    size_t need_part = 0;
    for (uint32_t i = 2; i + 1 < s->p.r; i++)
      need_part = std::max<size_t>(need_part, h.seg_max[i]);
    if (need_part > s->B.seg_cap) {
      int rc = grow_partials(s, need_part);
      if (rc) return rc;
      again = true;
    }
    if (h.n_cand > s->B.cand_cap) {
      int rc = grow_cand(s, h.n_cand);
      if (rc) return rc;
      again = true;
    }
    if (estimate && h.n_spl > s->B.spl_cap) {
      int rc = grow_spl(s, h.n_spl);
      if (rc) return rc;
      again = true;
    }
    if (!again) return SKETCH_OK;
  }
  return fail(SKETCH_E_HIP, "restore: capacities did not settle");
}

}  // namespace

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

  sketch *s = new sketch();
  s->p = *params;
  s->G = make_geom(*params);
  s->words = sketch_bytes(params) / 4;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, params->device) != hipSuccess) {
    delete s;
    return fail(SKETCH_E_HIP, "hipGetDeviceProperties failed");
  }
  s->n_cu = prop.multiProcessorCount;
  s->grid = s->n_cu * 8;
  s->update_grid = s->n_cu * 8;

  const size_t n_le = (size_t)params->r << params->k;
  const size_t nb = (size_t)1 << (params->k - params->alpha);
  RestoreBufs &B = s->B;
  int rc = SKETCH_OK;
  if (!rc) rc = dev_alloc(&s->d_sketch, s->words, "sketch");
  if (!rc) rc = dev_alloc(&B.st, 1, "state");
  if (!rc) rc = dev_alloc(&B.hotmask, n_le / 32, "hot bitmap");
  if (!rc) rc = dev_alloc(&B.he, n_le, "hot lists");
  if (!rc) rc = dev_alloc(&B.bk_off, (size_t)params->r * (nb + 1), "bucket offsets");
  if (!rc) rc = dev_alloc(&B.bk_cur, (size_t)params->r * nb, "bucket cursors");
  if (!rc) rc = dev_alloc(&B.bk_val, n_le, "bucket values");
  B.jblk = (uint32_t)(s->n_cu * 2);
  if (!rc) rc = dev_alloc(&B.rank, 16384, "sort ranks");
  if (!rc) rc = dev_alloc(&B.segc[0], B.jblk, "segment counts");
  if (!rc) rc = dev_alloc(&B.segc[1], B.jblk, "segment counts");
  if (!rc) rc = grow_partials(s, (size_t)1 << 12);
  if (!rc) rc = grow_cand(s, (size_t)1 << 16);
  if (!rc) rc = grow_spl(s, (size_t)1 << 16);
  s->nbins = (uint32_t)((s->words + BIN_TILE_WORDS - 1) / BIN_TILE_WORDS);
  s->BB.nblk = (uint32_t)std::min(1024, s->n_cu);
  s->BB.apply_grid = (uint32_t)s->n_cu;
  s->binned_min_pairs = std::max<size_t>(s->words / 8, 1 << 16);
  if (s->nbins <= BIN_MAX) {
    BinBufs &BB = s->BB;
    if (!rc) rc = dev_alloc(&BB.hist, (size_t)s->nbins * BB.nblk, "tile counts");
    if (!rc) rc = dev_alloc(&BB.totals, s->nbins, "tile totals");
    if (!rc) rc = dev_alloc(&BB.base, s->nbins + 1, "tile runs");
    if (!rc) rc = dev_alloc(&BB.item_start, s->nbins + 1, "tile items");
    if (!rc) rc = dev_alloc(&BB.xslot, s->nbins + 1, "tile scratch slots");
    if (!rc) rc = dev_alloc(&BB.n_items, 1, "tile item count");
  }
  if (!rc && hipHostMalloc((void **)&s->h_state, sizeof(DevState)) != hipSuccess) {
    s->h_state = nullptr;
    rc = fail(SKETCH_E_NOMEM, "hipHostMalloc(state) failed");
  }
  if (!rc) {
    hipError_t e = launch_fill_u32(s->d_sketch, s->words, 0u, s->grid, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) rc = fail(SKETCH_E_HIP, "sketch_create: zero fill: %s", hipGetErrorString(e));
  }
  if (rc) {
    free_all(s);
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
  free_all(s);
  delete s;
}

int sketch_update(sketch_t *s, const uint32_t *d_pairs, size_t n_pairs, void *hip_stream) {
  if (!s) return fail(SKETCH_E_INVAL, "sketch_update: NULL handle");
  if (n_pairs == 0) return SKETCH_OK;
  if (!d_pairs) return fail(SKETCH_E_INVAL, "sketch_update: NULL pairs");
  if (((uintptr_t)d_pairs) & 7u)
    return fail(SKETCH_E_INVAL, "sketch_update: pairs must be 8-byte aligned");
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  const bool can_bin = s->nbins <= BIN_MAX;
  const bool binned = can_bin && (s->update_path == 2 ||
                                  (s->update_path == 0 && n_pairs >= s->binned_min_pairs));
  if (binned) {
    int rc = ensure_codes(s, std::min(n_pairs, s->binned_round), st);
    if (rc) return rc;
    HIP_OK(launch_update_binned(s->G, s->d_sketch, s->words, d_pairs, n_pairs, s->BB, st));
    return SKETCH_OK;
  }
  HIP_OK(launch_update(s->G, s->d_sketch, d_pairs, n_pairs, s->update_grid,
                       s->update_variant, st));
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
      s->update_variant = (int)value;
      return SKETCH_OK;
    case SKETCH_OPT_BINNED_ROUND:
      if (value < 1024 || (uint64_t)value * s->p.r >= (1ull << 32)) break;
      s->binned_round = (size_t)value;
      return SKETCH_OK;
    default:
      return fail(SKETCH_E_INVAL, "sketch_set_option: unknown option %d", option);
  }
  return fail(SKETCH_E_INVAL, "sketch_set_option: bad value %lld for option %d",
              (long long)value, option);
}

int sketch_reset(sketch_t *s, void *hip_stream) {
  if (!s) return fail(SKETCH_E_INVAL, "sketch_reset: NULL handle");
  DEVICE_GUARD(s->p.device);
  HIP_OK(launch_fill_u32(s->d_sketch, s->words, 0u, s->grid * 4, (hipStream_t)hip_stream));
  return SKETCH_OK;
}

int sketch_restore(sketch_t *s, double theta, sketch_sp_t *out, size_t cap, size_t *n_out,
                   sketch_info_t *info, void *hip_stream) {
  if (!s || !n_out) return fail(SKETCH_E_INVAL, "sketch_restore: NULL handle or n_out");
  if (!(theta > 0.0) || !isfinite(theta))
    return fail(SKETCH_E_INVAL, "sketch_restore: theta must be finite and > 0");
  if (cap && !out) return fail(SKETCH_E_INVAL, "sketch_restore: NULL out with cap > 0");
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  double zmin;
  uint32_t zhot;
  int rc = run_restore(s, theta, 1, st, &zmin, &zhot);
  if (rc != SKETCH_OK && rc != SKETCH_E_SATURATED) return rc;
  const DevState h = *s->h_state;
  fill_info(s, h, zmin, zhot, info);
  if (rc == SKETCH_E_SATURATED) {
    *n_out = 0;
    return fail(SKETCH_E_SATURATED, "sketch_restore: a row has no zero bit (psi = 1)");
  }
  *n_out = (size_t)h.n_spl;
  if (h.n_spl > cap)
    return fail(SKETCH_E_CAPACITY, "sketch_restore: %llu records, cap %zu", h.n_spl, cap);
  static_assert(sizeof(sketch_sp_t) == sizeof(uint4), "record layout");
  if (h.n_spl)
    HIP_OK(hipMemcpyAsync(out, s->B.spl_sorted, h.n_spl * sizeof(uint4), hipMemcpyDeviceToHost,
                          st));
  HIP_OK(hipStreamSynchronize(st));
  return SKETCH_OK;
}

int sketch_candidates(sketch_t *s, double theta, uint32_t *out, size_t cap, size_t *n_out,
                      void *hip_stream) {
  if (!s || !n_out) return fail(SKETCH_E_INVAL, "sketch_candidates: NULL handle or n_out");
  if (!(theta > 0.0) || !isfinite(theta))
    return fail(SKETCH_E_INVAL, "sketch_candidates: theta must be finite and > 0");
  if (cap && !out) return fail(SKETCH_E_INVAL, "sketch_candidates: NULL out with cap > 0");
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
  double zmin;
  uint32_t zhot;
  int rc = run_restore(s, theta, 0, st, &zmin, &zhot);
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
    HIP_OK(hipMemcpyAsync(out, s->B.cand_sorted, h.n_cand * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  return SKETCH_OK;
}

int sketch_download(const sketch_t *s, uint32_t *host_words, size_t n_words, void *hip_stream) {
  if (!s || !host_words) return fail(SKETCH_E_INVAL, "sketch_download: NULL argument");
  if (n_words != s->words)
    return fail(SKETCH_E_INVAL, "sketch_download: n_words %zu, sketch has %zu", n_words, s->words);
  DEVICE_GUARD(s->p.device);
  hipStream_t st = (hipStream_t)hip_stream;
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
  HIP_OK(hipMemcpyAsync(s->d_sketch, host_words, n_words * 4, hipMemcpyHostToDevice, st));
  HIP_OK(hipStreamSynchronize(st));
  return SKETCH_OK;
}

const char *sketch_last_error(void) { return g_err.c_str(); }

}  // extern "C"

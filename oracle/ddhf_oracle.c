/*
 * DDHF super point detection: CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously correct
 * reference that the GPU library is checked against. Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * product path never does. It shares no code, header, table or helper with
 * the GPU library.
 *
 * Source: J. Xu, "Economical and efficient network super points detection
 * based on GPU" (arXiv 1803.11449).
 *   Sec. 3.1  linear estimator, eq. (1)
 *   Sec. 3.2  DHG hash group, eq. (2); update, Alg. 1
 *   Sec. 3.3  block inversion eq. (3); constraints on r, alpha, k; Lemma 1;
 *             flow-count estimate; Def. 1; Theorem 1; eq. (4); restore, Alg. 2
 *   Sec. 4.2  incremental restore, Algs. 3 and 4; candidate estimate
 *
 * Readings where the paper is silent or garbled (each listed in the design
 * notes of the repository):
 *   - H1 and DH0 are random hash functions the paper does not specify.
 *     Here both are multiply-add-shift hashes (Dietzfelbinger 1996) on the
 *     32-bit key with a 64-bit odd multiplier:
 *        DH0(x) = ((A0*x + B0) mod 2^64) >> (64 - k)
 *        H1(y)  = ((A1*y + B1) mod 2^64) >> (64 - log2 g)
 *     A0,B0,A1,B1 are the first four outputs of SplitMix64 (Steele, Lea and
 *     Flood 2014) started at the sketch seed; A0 and A1 have bit 0 forced to 1.
 *   - Zmin in Alg. 2 is read as g*exp(-theta/g); an LE is hot iff its zero
 *     count z0 < Zmin (strict, as printed).
 *   - Alg. 2's flag is set on a mismatch and then tested for false: read as
 *     "a mismatch rejects the tuple". Alg. 4 writes CL_0 xor CL_2 at stage i:
 *     read as CL_0 xor CL_i.
 *   - "Left" bits are the most significant ones: the top k-alpha bits of
 *     BL(i) must equal the low k-alpha bits of BL(i+1).
 *   - A rebuilt address is kept only if it is a 32-bit value and DH0 of it
 *     equals the CL_0 it was built from (the estimate step re-hashes the
 *     address to gather its LEs, so a tuple whose CL_0 is not DH0(a) does not
 *     describe a).
 *   - C = -g*ln(SZ/(g - g*psi^r)) is +inf when SZ = 0 and is reported.
 *   - A row with ZR(i) = 0 makes psi = 1: the sketch is saturated, error.
 *   - The report test is C >= theta (Alg. 2 skips C < theta).
 *   - The measured host is the source of a (src,dst) pair; dst is the
 *     opposite host whose hash picks the bit.
 *
 * Sketch layout (the one interface shared with the GPU library, by
 * necessity, since parity is bit-for-bit): uint32 words,
 *   word index = (i * 2^k + cell) * (g/32) + bit/32,  bit mask 1 << (bit%32)
 * for row i, LE (cell) and bit index within the LE.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_SATURATED (-5)

typedef struct {
  uint32_t g, k, r, alpha, log2g, words_per_le;
  uint64_t a0, b0, a1, b1;
} orc_t;

/* ---------------------------------------------------------------- params */

/* Constraints of Sec. 3.3: alpha <= k (no gap between neighbouring blocks)
 * and (r-2)*alpha + k >= 32 (the last block reaches bit 31). The others are
 * representational: g a power of two with at least one 32-bit word, k <= 24,
 * r <= 8. */
int orc_check_params(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha) {
  if (g < 32 || g > 65536 || (g & (g - 1)) != 0) return ORC_E_INVAL;
  if (k < 1 || k > 24) return ORC_E_INVAL;
  if (r < 3 || r > 8) return ORC_E_INVAL;
  if (alpha < 1 || alpha > k) return ORC_E_INVAL;
  if ((r - 2) * alpha + k < 32) return ORC_E_INVAL;
  return ORC_OK;
}

/* SplitMix64, as published by Steele, Lea and Flood (2014). */
static uint64_t splitmix64_next(uint64_t *state) {
  uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void orc_splitmix64(uint64_t seed, uint64_t *out, size_t n) {
  uint64_t s = seed;
  for (size_t i = 0; i < n; i++) out[i] = splitmix64_next(&s);
}

static int orc_init(orc_t *o, uint32_t g, uint32_t k, uint32_t r,
                    uint32_t alpha, uint64_t seed) {
  if (orc_check_params(g, k, r, alpha) != ORC_OK) return ORC_E_INVAL;
  o->g = g; o->k = k; o->r = r; o->alpha = alpha;
  o->log2g = 0;
  while ((1u << o->log2g) < g) o->log2g++;
  o->words_per_le = g / 32;
  uint64_t v[4];
  orc_splitmix64(seed, v, 4);
  o->a0 = v[0] | 1ull; o->b0 = v[1];
  o->a1 = v[2] | 1ull; o->b1 = v[3];
  return ORC_OK;
}

void orc_hash_coeffs(uint64_t seed, uint64_t *out4) {
  uint64_t v[4];
  orc_splitmix64(seed, v, 4);
  out4[0] = v[0] | 1ull; out4[1] = v[1];
  out4[2] = v[2] | 1ull; out4[3] = v[3];
}

/* ---------------------------------------------------------------- hashes */

/* DH0: the random, non-invertible hash of the measured host into [0,2^k). */
static uint32_t dh0(const orc_t *o, uint32_t a) {
  uint64_t x = o->a0 * (uint64_t)a + o->b0;
  return (uint32_t)(x >> (64 - o->k));
}

/* H1: the random hash of the opposite host to a bit index in [0,g). */
static uint32_t h1(const orc_t *o, uint32_t b) {
  uint64_t x = o->a1 * (uint64_t)b + o->b1;
  return (uint32_t)(x >> (64 - o->log2g));
}

/* Bit block BL(i): the k bits of a starting at bit (i-1)*alpha (Sec. 3.2). */
static uint32_t bit_block(const orc_t *o, uint32_t i, uint32_t a) {
  uint32_t shift = (i - 1) * o->alpha;
  uint32_t kmask = (uint32_t)((1ull << o->k) - 1);
  if (shift >= 32) return 0;
  return (a >> shift) & kmask;
}

/* DH_i, eq. (2): DH_0 for i = 0, else BL(i) xor DH_0(a). */
static uint32_t dh(const orc_t *o, uint32_t i, uint32_t a) {
  uint32_t c0 = dh0(o, a);
  if (i == 0) return c0;
  return bit_block(o, i, a) ^ c0;
}

int orc_dh(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha, uint64_t seed,
           uint32_t i, const uint32_t *a, uint32_t *out, size_t n) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, seed) || i >= r) return ORC_E_INVAL;
  for (size_t j = 0; j < n; j++) out[j] = dh(&o, i, a[j]);
  return ORC_OK;
}

int orc_h1(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha, uint64_t seed,
           const uint32_t *b, uint32_t *out, size_t n) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, seed)) return ORC_E_INVAL;
  for (size_t j = 0; j < n; j++) out[j] = h1(&o, b[j]);
  return ORC_OK;
}

/* ---------------------------------------------------------------- sketch */

static size_t le_index(const orc_t *o, uint32_t row, uint32_t cell) {
  return ((size_t)row << o->k) + cell;
}

static int le_bit(const orc_t *o, const uint32_t *sk, uint32_t row,
                  uint32_t cell, uint32_t bit) {
  size_t w = le_index(o, row, cell) * o->words_per_le + (bit >> 5);
  return (sk[w] >> (bit & 31)) & 1u;
}

static void le_set(const orc_t *o, uint32_t *sk, uint32_t row, uint32_t cell,
                   uint32_t bit) {
  size_t w = le_index(o, row, cell) * o->words_per_le + (bit >> 5);
  sk[w] |= 1u << (bit & 31);
}

static uint32_t le_ones(const orc_t *o, const uint32_t *sk, uint32_t row,
                        uint32_t cell) {
  const uint32_t *p = sk + le_index(o, row, cell) * o->words_per_le;
  uint32_t ones = 0;
  for (uint32_t w = 0; w < o->words_per_le; w++)
    ones += (uint32_t)__builtin_popcount(p[w]);
  return ones;
}

size_t orc_sketch_words(uint32_t g, uint32_t k, uint32_t r) {
  return (size_t)r * ((size_t)1 << k) * (g / 32);
}

/* Alg. 1 (Update DHLA), applied to each pair in turn: the bit H1(b) of the
 * LE DH_i(a) in every row i is set unless it is already 1. pairs holds
 * (a,b) interleaved: pairs[2j] = a (measured host), pairs[2j+1] = b. */
int orc_update(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha,
               uint64_t seed, uint32_t *sketch, const uint32_t *pairs,
               size_t n) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, seed)) return ORC_E_INVAL;
  for (size_t j = 0; j < n; j++) {
    uint32_t a = pairs[2 * j], b = pairs[2 * j + 1];
    uint32_t bit = h1(&o, b);
    for (uint32_t i = 0; i < o.r; i++) {
      uint32_t cell = dh(&o, i, a);
      if (le_bit(&o, sketch, i, cell, bit)) continue;
      le_set(&o, sketch, i, cell, bit);
    }
  }
  return ORC_OK;
}

/* Alg. 1 with the pairs shared out among nthreads threads (OpenMP), for the
 * CPU baseline's timing. Each bit is set with an atomic OR after Alg. 1's
 * test, so the sketch equals the sequential loop's (OR is order-free). */
int orc_update_omp(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha,
                   uint64_t seed, uint32_t *sketch, const uint32_t *pairs,
                   size_t n, int nthreads) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, seed)) return ORC_E_INVAL;
  int nt = nthreads > 0 ? nthreads : 1;
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t j = 0; j < (int64_t)n; j++) {
    uint32_t a = pairs[2 * j], b = pairs[2 * j + 1];
    uint32_t bit = h1(&o, b);
    for (uint32_t i = 0; i < o.r; i++) {
      size_t w = le_index(&o, i, dh(&o, i, a)) * o.words_per_le + (bit >> 5);
      uint32_t mask = 1u << (bit & 31);
      if (__atomic_load_n(&sketch[w], __ATOMIC_RELAXED) & mask) continue;
      __atomic_fetch_or(&sketch[w], mask, __ATOMIC_RELAXED);
    }
  }
  return ORC_OK;
}

/* z0 of every LE (g minus its weight |LA(i,j)|, Alg. 2) and ZR(i), the zero
 * count of row i (Sec. 3.3). z0 has r*2^k entries, zr has r. */
int orc_zero_counts(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha,
                    const uint32_t *sketch, uint32_t *z0, uint64_t *zr) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, 0)) return ORC_E_INVAL;
  for (uint32_t i = 0; i < r; i++) {
    uint64_t sum = 0;
    for (uint32_t j = 0; j < (1u << k); j++) {
      uint32_t z = g - le_ones(&o, sketch, i, j);
      if (z0) z0[le_index(&o, i, j)] = z;
      sum += z;
    }
    zr[i] = sum;
  }
  return ORC_OK;
}

/* Flow count and one-bit probability (Sec. 3.3):
 *   w(i)' = -g*2^k*ln(ZR(i)/(g*2^k)),  w' = mean of w(i)',
 *   psi   = 1 - exp(-w'/(g*2^k))          (Lemma 1)
 * and the thresholds
 *   Zmin  = g*exp(-theta/g)               (Alg. 2, hot test z0 < Zmin)
 *   D     = g - g*psi^r                   (eq. (4) denominator)
 * out = {psi, D, Zmin, w'}. */
int orc_scalars(uint32_t g, uint32_t k, uint32_t r, const uint64_t *zr,
                double theta, double *out) {
  double cells = (double)g * (double)((uint64_t)1 << k);
  double wsum = 0.0;
  for (uint32_t i = 0; i < r; i++) {
    if (zr[i] == 0) return ORC_E_SATURATED;
    double wi = -cells * log((double)zr[i] / cells);
    wsum += wi;
  }
  double w = wsum / (double)r;
  double psi = 1.0 - exp(-w / cells);
  out[0] = psi;
  out[1] = (double)g - (double)g * pow(psi, (double)r);
  out[2] = (double)g * exp(-theta / (double)g);
  out[3] = w;
  return ORC_OK;
}

/* HE(i): ascending list of LEs j of row i with z0 < Zmin (Alg. 2, first
 * loop). he must have room for r*2^k entries, row i at he + i*2^k. */
static void hot_lists(const orc_t *o, const uint32_t *sketch, double zmin,
                      uint32_t *he, uint32_t *he_n) {
  for (uint32_t i = 0; i < o->r; i++) {
    uint32_t n = 0;
    for (uint32_t j = 0; j < (1u << o->k); j++) {
      uint32_t z0 = o->g - le_ones(o, sketch, i, j);
      if ((double)z0 < zmin) he[((size_t)i << o->k) + n++] = j;
    }
    he_n[i] = n;
  }
}

int orc_hot_lists(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha,
                  const uint32_t *sketch, double theta, uint32_t *he,
                  uint32_t *he_n) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, 0)) return ORC_E_INVAL;
  hot_lists(&o, sketch, (double)g * exp(-theta / (double)g), he, he_n);
  return ORC_OK;
}

/* -------------------------------------------------------------- restore */

typedef struct { uint64_t sub; uint32_t c0; } partial_t;

typedef struct { partial_t *v; size_t n, cap; } plist_t;

static int plist_push(plist_t *l, uint64_t sub, uint32_t c0) {
  if (l->n == l->cap) {
    size_t nc = l->cap ? 2 * l->cap : 1024;
    partial_t *nv = (partial_t *)realloc(l->v, nc * sizeof(partial_t));
    if (!nv) return ORC_E_NOMEM;
    l->v = nv; l->cap = nc;
  }
  l->v[l->n].sub = sub; l->v[l->n].c0 = c0; l->n++;
  return ORC_OK;
}

typedef struct { uint32_t *v; size_t n, cap; } ulist_t;

static int ulist_push(ulist_t *l, uint32_t x) {
  if (l->n == l->cap) {
    size_t nc = l->cap ? 2 * l->cap : 1024;
    uint32_t *nv = (uint32_t *)realloc(l->v, nc * sizeof(uint32_t));
    if (!nv) return ORC_E_NOMEM;
    l->v = nv; l->cap = nc;
  }
  l->v[l->n++] = x;
  return ORC_OK;
}

static int cmp_u32(const void *x, const void *y) {
  uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
  return a < b ? -1 : (a > b ? 1 : 0);
}

static uint64_t shr64(uint64_t x, uint32_t s) { return s >= 64 ? 0 : x >> s; }

/* A rebuilt address is accepted when it fits in 32 bits and hashes back to
 * the LE of row 0 it was built from. */
static int accept_rebuilt(const orc_t *o, uint64_t a, uint32_t c0) {
  if (a >> 32) return 0;
  return dh0(o, (uint32_t)a) == c0;
}

/* Candidate join, Algs. 3 and 4 (Sec. 4.2), with plain nested loops.
 * Stage 1 walks HE(0) x HE(1) x HE(2): blk1 = CL0^CL1, blk2 = CL0^CL2; the
 * top k-alpha bits of blk1 must equal the low k-alpha bits of blk2; the
 * partial address is blk1 with the top alpha bits of blk2 appended above it.
 * Stage i (3..r-1) walks (partial, CL0) x HE(i): blk = CL0^CL_i; the top
 * k-alpha bits of the partial must equal the low k-alpha bits of blk; the top
 * alpha bits of blk are appended. At the last stage the address must be a
 * 32-bit value that re-hashes to CL0 (when rehash != 0).
 * cand receives the distinct accepted addresses, ascending. Returns the
 * candidate count (may exceed cap: then cand holds the first cap) or < 0. */
static int64_t join_incremental(const orc_t *o, const uint32_t *he,
                                const uint32_t *he_n, int rehash,
                                uint32_t *cand, size_t cap) {
  const uint32_t k = o->k, al = o->alpha, r = o->r;
  const uint64_t M = (1ull << (k - al)) - 1;
  const uint32_t *HE0 = he, *HE1 = he + ((size_t)1 << k),
                 *HE2 = he + ((size_t)2 << k);
  plist_t cur = {0}, nxt = {0};
  ulist_t out = {0};
  int64_t rc = 0;

  for (uint32_t x0 = 0; x0 < he_n[0]; x0++)
    for (uint32_t x1 = 0; x1 < he_n[1]; x1++)
      for (uint32_t x2 = 0; x2 < he_n[2]; x2++) {
        uint32_t c0 = HE0[x0];
        uint64_t blk1 = c0 ^ HE1[x1], blk2 = c0 ^ HE2[x2];
        if ((blk1 >> al) != (blk2 & M)) continue;
        uint64_t sub = blk1 | ((blk2 >> (k - al)) << k);
        if (plist_push(&cur, sub, c0)) { rc = ORC_E_NOMEM; goto done; }
      }

  for (uint32_t i = 3; i < r; i++) {
    const uint32_t *HEi = he + ((size_t)i << k);
    nxt.n = 0;
    for (size_t p = 0; p < cur.n; p++)
      for (uint32_t x = 0; x < he_n[i]; x++) {
        uint32_t c0 = cur.v[p].c0;
        uint64_t sub = cur.v[p].sub;
        uint64_t blk = c0 ^ HEi[x];
        if ((shr64(sub, (i - 1) * al) & M) != (blk & M)) continue;
        uint32_t pos = k + (i - 2) * al;
        uint64_t top = blk >> (k - al);
        uint64_t sub2 = sub;
        if (pos < 32) sub2 |= top << pos;
        else if (top) sub2 |= 1ull << 63; /* lands above bit 31: rejected */
        if (plist_push(&nxt, sub2, c0)) { rc = ORC_E_NOMEM; goto done; }
      }
    plist_t t = cur; cur = nxt; nxt = t;
  }

  for (size_t p = 0; p < cur.n; p++) {
    if (rehash) {
      if (!accept_rebuilt(o, cur.v[p].sub, cur.v[p].c0)) continue;
    } else if (cur.v[p].sub >> 32) {
      continue;
    }
    if (ulist_push(&out, (uint32_t)cur.v[p].sub)) { rc = ORC_E_NOMEM; goto done; }
  }
  if (out.n) qsort(out.v, out.n, sizeof(uint32_t), cmp_u32);
  /* without the re-hash test one address may come from several tuples */
  size_t u = 0;
  for (size_t p = 0; p < out.n; p++)
    if (u == 0 || out.v[u - 1] != out.v[p]) out.v[u++] = out.v[p];
  for (size_t p = 0; p < u && p < cap; p++) cand[p] = out.v[p];
  rc = (int64_t)u;
done:
  free(cur.v); free(nxt.v); free(out.v);
  return rc;
}

/* Every tuple of hot LEs, one per row (the search space of Alg. 2), judged
 * by what a tuple stands for: the 32-bit address a with DH_i(a) = CL_i in
 * every row. By eq. (3) such an a has BL(i)(a) = CL_0 ^ CL_i for i >= 1, and
 * since the blocks together cover bits 0..31 ((r-2)*alpha + k >= 32 and
 * alpha <= k, Sec. 3.3), that a, if it exists, is the OR of those blocks
 * placed at their offsets. The tuple names an address iff that OR satisfies
 * all r equations; no overlap rule is applied separately. Exponential in r:
 * tiny inputs only. */
static int64_t join_tuples(const orc_t *o, const uint32_t *he,
                           const uint32_t *he_n, uint32_t *cand, size_t cap) {
  const uint32_t k = o->k, al = o->alpha, r = o->r;
  uint64_t total = 1;
  for (uint32_t i = 0; i < r; i++) total *= he_n[i];
  ulist_t out = {0};
  for (uint64_t t = 0; t < total; t++) {
    uint32_t cl[8];
    uint64_t rem = t;
    for (uint32_t i = 0; i < r; i++) {
      cl[i] = he[((size_t)i << k) + (uint32_t)(rem % he_n[i])];
      rem /= he_n[i];
    }
    uint64_t a = 0;
    for (uint32_t i = 1; i < r; i++) {
      uint32_t s = (i - 1) * al;
      if (s < 32) a |= (uint64_t)(cl[0] ^ cl[i]) << s;
    }
    a &= 0xFFFFFFFFull;
    int names = 1;
    for (uint32_t i = 0; i < r && names; i++) names = dh(o, i, (uint32_t)a) == cl[i];
    if (!names) continue;
    if (ulist_push(&out, (uint32_t)a)) { free(out.v); return ORC_E_NOMEM; }
  }
  if (out.n) qsort(out.v, out.n, sizeof(uint32_t), cmp_u32);
  size_t u = 0;
  for (size_t p = 0; p < out.n; p++)
    if (u == 0 || out.v[u - 1] != out.v[p]) out.v[u++] = out.v[p];
  for (size_t p = 0; p < u && p < cap; p++) cand[p] = out.v[p];
  free(out.v);
  return (int64_t)u;
}

/* The candidate set by its definition: every 32-bit address whose r LEs
 * DH_i(a) are all hot. Scans all 2^32 addresses on nthreads threads. */
static int64_t join_bruteforce(const orc_t *o, const uint32_t *he,
                               const uint32_t *he_n, int nthreads,
                               uint32_t *cand, size_t cap) {
  const uint32_t r = o->r;
  size_t cells = (size_t)1 << o->k;
  uint8_t *hot = (uint8_t *)calloc(r * cells, 1);
  if (!hot) return ORC_E_NOMEM;
  for (uint32_t i = 0; i < r; i++)
    for (uint32_t x = 0; x < he_n[i]; x++) hot[i * cells + he[i * cells + x]] = 1;

  int nt = nthreads > 0 ? nthreads : 1;
  ulist_t *loc = (ulist_t *)calloc((size_t)nt, sizeof(ulist_t));
  int err = 0;
  const uint64_t chunks = 4096, per = (1ull << 32) / chunks;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 1)
  for (uint64_t c = 0; c < chunks; c++) {
    int tid = omp_get_thread_num();
    for (uint64_t a64 = c * per; a64 < (c + 1) * per; a64++) {
      uint32_t a = (uint32_t)a64;
      uint32_t c0 = dh0(o, a);
      if (!hot[c0]) continue;
      int all = 1;
      for (uint32_t i = 1; i < r && all; i++)
        all = hot[i * cells + (bit_block(o, i, a) ^ c0)];
      if (all && ulist_push(&loc[tid], a)) err = 1;
    }
  }
  int64_t n = 0;
  for (int t = 0; t < nt; t++) n += (int64_t)loc[t].n;
  uint32_t *all = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
  size_t q = 0;
  for (int t = 0; t < nt; t++) {
    if (all) memcpy(all + q, loc[t].v, loc[t].n * sizeof(uint32_t));
    q += loc[t].n;
    free(loc[t].v);
  }
  free(loc); free(hot);
  if (err || !all) { free(all); return ORC_E_NOMEM; }
  qsort(all, (size_t)n, sizeof(uint32_t), cmp_u32);
  for (int64_t p = 0; p < n && (size_t)p < cap; p++) cand[p] = all[p];
  free(all);
  return n;
}

/* Candidate set CAND for threshold theta.
 * mode 0: Algs. 3-4 (incremental join) with the re-hash test
 * mode 1: brute force over all 2^32 addresses
 * mode 2: every tuple of hot LEs judged by the address it names (tiny only)
 * mode 3: Algs. 3-4 without the re-hash test (distinct 32-bit results)
 * Returns the count (may exceed cap) or a negative error. */
int64_t orc_candidates(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha,
                       uint64_t seed, const uint32_t *sketch, double theta,
                       int mode, int nthreads, uint32_t *cand, size_t cap) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, seed)) return ORC_E_INVAL;
  uint32_t *he = (uint32_t *)malloc(((size_t)r << k) * sizeof(uint32_t));
  if (!he) return ORC_E_NOMEM;
  uint32_t he_n[8];
  hot_lists(&o, sketch, (double)g * exp(-theta / (double)g), he, he_n);
  int64_t n;
  switch (mode) {
    case 0: n = join_incremental(&o, he, he_n, 1, cand, cap); break;
    case 1: n = join_bruteforce(&o, he, he_n, nthreads, cand, cap); break;
    case 2: n = join_tuples(&o, he, he_n, cand, cap); break;
    case 3: n = join_incremental(&o, he, he_n, 0, cand, cap); break;
    default: n = ORC_E_INVAL;
  }
  free(he);
  return n;
}

/* ULE(a) = AND of a's r LEs (Sec. 3.2); SZ(a) = its zero count (Def. 1);
 * C(a) = -g*ln(SZ/(g - g*psi^r)) (eq. (4), from Theorem 1). */
int orc_estimate(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha,
                 uint64_t seed, const uint32_t *sketch, double psi,
                 const uint32_t *ips, size_t n, uint32_t *sz, double *c) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, seed)) return ORC_E_INVAL;
  double denom = (double)g - (double)g * pow(psi, (double)r);
  for (size_t j = 0; j < n; j++) {
    uint32_t ones = 0;
    for (uint32_t w = 0; w < o.words_per_le; w++) {
      uint32_t u = 0xFFFFFFFFu;
      for (uint32_t i = 0; i < r; i++)
        u &= sketch[le_index(&o, i, dh(&o, i, ips[j])) * o.words_per_le + w];
      ones += (uint32_t)__builtin_popcount(u);
    }
    uint32_t zs = g - ones;
    if (sz) sz[j] = zs;
    if (c) c[j] = -(double)g * log((double)zs / denom);
  }
  return ORC_OK;
}

/* Alg. 2 end to end: hot lists, candidate join (mode as in orc_candidates),
 * estimate by eq. (4), keep C >= theta. Outputs are ascending by address.
 * scal receives {psi, D, Zmin, w'}. Returns the SPL size (may exceed cap) or
 * a negative error. */
int64_t orc_restore(uint32_t g, uint32_t k, uint32_t r, uint32_t alpha,
                    uint64_t seed, const uint32_t *sketch, double theta,
                    int mode, int nthreads, uint32_t *ip_out, uint32_t *sz_out,
                    double *c_out, size_t cap, double *scal) {
  orc_t o;
  if (orc_init(&o, g, k, r, alpha, seed)) return ORC_E_INVAL;
  if (!(theta > 0.0)) return ORC_E_INVAL;
  uint64_t zr[8];
  orc_zero_counts(g, k, r, alpha, sketch, NULL, zr);
  double s[4];
  int rc = orc_scalars(g, k, r, zr, theta, s);
  if (scal) memcpy(scal, s, sizeof(s));
  if (rc) return rc;
  size_t ccap = 1 << 16;
  uint32_t *cand = NULL;
  int64_t nc;
  for (;;) {
    free(cand);
    cand = (uint32_t *)malloc(ccap * sizeof(uint32_t));
    if (!cand) return ORC_E_NOMEM;
    nc = orc_candidates(g, k, r, alpha, seed, sketch, theta, mode, nthreads, cand, ccap);
    if (nc < 0 || (size_t)nc <= ccap) break;
    ccap = (size_t)nc;
  }
  if (nc < 0) { free(cand); return nc; }
  uint32_t *sz = (uint32_t *)malloc((size_t)(nc ? nc : 1) * sizeof(uint32_t));
  double *c = (double *)malloc((size_t)(nc ? nc : 1) * sizeof(double));
  if (!sz || !c) { free(cand); free(sz); free(c); return ORC_E_NOMEM; }
  orc_estimate(g, k, r, alpha, seed, sketch, s[0], cand, (size_t)nc, sz, c);
  int64_t m = 0;
  for (int64_t j = 0; j < nc; j++) {
    if (c[j] < theta) continue;
    if ((size_t)m < cap) {
      if (ip_out) ip_out[m] = cand[j];
      if (sz_out) sz_out[m] = sz[j];
      if (c_out) c_out[m] = c[j];
    }
    m++;
  }
  free(cand); free(sz); free(c);
  return m;
}

/* -------------------------------------------------------- ground truth */

static int cmp_u64(const void *x, const void *y) {
  uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
  return a < b ? -1 : (a > b ? 1 : 0);
}

/* |CO(a)| for every measured host a (Sec. 3.1): the number of distinct
 * opposite hosts, by sorting the (a,b) keys and counting distinct ones per a.
 * Writes hosts ascending. Returns the number of distinct hosts (may exceed
 * cap) or a negative error. */
int64_t orc_exact_cardinality(const uint32_t *pairs, size_t n, uint32_t *host,
                              uint32_t *card, size_t cap) {
  uint64_t *key = (uint64_t *)malloc((n ? n : 1) * sizeof(uint64_t));
  if (!key) return ORC_E_NOMEM;
  for (size_t j = 0; j < n; j++)
    key[j] = ((uint64_t)pairs[2 * j] << 32) | pairs[2 * j + 1];
  qsort(key, n, sizeof(uint64_t), cmp_u64);
  int64_t hosts = 0;
  size_t j = 0;
  while (j < n) {
    uint32_t a = (uint32_t)(key[j] >> 32);
    uint32_t cnt = 0;
    uint64_t prev = 0;
    int first = 1;
    while (j < n && (uint32_t)(key[j] >> 32) == a) {
      if (first || key[j] != prev) cnt++;
      prev = key[j]; first = 0; j++;
    }
    if ((size_t)hosts < cap) { host[hosts] = a; card[hosts] = cnt; }
    hosts++;
  }
  free(key);
  return hosts;
}

/*
 * ddhf.h - C ABI of libddhf, the MI355X (gfx950) implementation of the
 * double direction hash functions (DDHF) super point detector of
 * J. Xu, "Economical and efficient network super points detection based on
 * GPU" (arXiv 1803.11449).
 *
 * The library owns one sketch per handle: r rows ("LA") of 2^k linear
 * estimators ("LE") of g bits each (the DHLA of Sec. 3.2), in device memory.
 * sketch_update streams (src,dst) IPv4 pairs into it (Alg. 1);
 * sketch_restore recovers the super points of the window from it (Alg. 2,
 * computed as in Sec. 4.2: hot-LE scan, candidate search by the incremental
 * join of Algs. 3-4 or by walking the addresses of each hot row-0 LE,
 * estimate by eq. (4)); sketch_reset starts a new window.
 *
 * Conventions for every entry point
 *  - Status codes are returned; nothing is thrown across the ABI. On failure
 *    sketch_last_error() gives a message (per calling thread).
 *  - hip_stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is issued on it in order.
 *  - A handle is not thread-safe: use one handle from one thread at a time.
 *    Several handles may share a device and a stream. Work a call enqueues
 *    on a sketch is ordered after the last work any earlier call enqueued
 *    on it, also from another stream (each handle keeps an event of its
 *    last work), and the device's shared scratch buffers are ordered the
 *    same way: the update's scratch and the restore's separately, so an
 *    update on one stream may run while a restore of another sketch runs
 *    on another.
 *  - The device is params->device; every call makes it current for its
 *    duration and restores the caller's current device before returning.
 *
 * Hash family (the paper leaves H1 and DH0 as unspecified random hashes):
 *   DH0(x) = ((A0*x + B0) mod 2^64) >> (64-k)           LE of row 0
 *   H1(y)  = ((A1*y + B1) mod 2^64) >> (64-log2 g)      bit inside the LE
 *   DH_i(x) = ((x >> (i-1)*alpha) mod 2^k) xor DH0(x)   eq. (2), i = 1..r-1
 * A0,B0,A1,B1 are the first four SplitMix64 outputs from params->seed
 * (A0, A1 with bit 0 set).
 *
 * Sketch layout in device memory (also the format of download/upload):
 * uint32 words; bit b of LE c in row i is bit (b % 32) of word
 *   (i * 2^k + c) * (g/32) + b/32.
 * One LE of the default g = 1024 is 128 bytes.
 */
#ifndef DDHF_H
#define DDHF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sketch sketch_t;

/* Sketch parameters (Sec. 3.2-3.3; the paper's experiments use g = 1024,
 * k = 14, r = 5, alpha = 6, Sec. 5).
 * Valid iff: g a power of two in [32, 65536]; 5 <= k <= 24; 3 <= r <= 8;
 * 1 <= alpha <= k; (r-2)*alpha + k >= 32 (Sec. 3.3: every address bit lies in
 * some block); k - alpha <= 20 (bucket tables of the join). */
typedef struct {
  uint32_t g;       /* bits per LE */
  uint32_t k;       /* log2 of the LEs per row */
  uint32_t r;       /* rows = hash functions */
  uint32_t alpha;   /* bit stride between neighbouring blocks */
  uint64_t seed;    /* seed of the hash coefficients */
  int32_t device;   /* HIP device ordinal */
} sketch_params_t;

/* One reported super point: its address, the zero count SZ of its ULE
 * (the AND of its r LEs, Def. 1) and its cardinality estimate
 * C = -g*ln(SZ/(g - g*psi^r)) (eq. (4)); est = +INFINITY when sz == 0. */
typedef struct {
  uint32_t ip;
  uint32_t sz;
  double est;
} sketch_sp_t;

/* Diagnostics of the last restore (all optional to read). */
typedef struct {
  uint64_t zr[8];           /* ZR(i): zero bits in row i (Sec. 3.3) */
  uint32_t he_count[8];     /* |HE(i)|: hot LEs in row i (Alg. 2) */
  uint64_t n_partials[8];   /* partial addresses after join stage i
                               (index 2 = Alg. 3, 3..r-2 = Alg. 4) */
  uint64_t n_candidates;    /* addresses whose r LEs are all hot */
  uint64_t n_reported;      /* super points (SZ <= szmax) */
  double psi;               /* one-bit probability (Lemma 1) */
  double d;                 /* g - g*psi^r (eq. (4)) */
  double zmin;              /* g*exp(-theta/g) (Alg. 2) */
  double trep;              /* d*exp(-theta/g): C >= theta <=> SZ <= trep */
  uint32_t zhot;            /* hot <=> z0 <= zhot (= ceil(zmin) - 1) */
  uint32_t szmax;           /* report <=> SZ <= szmax (= floor(trep)) */
} sketch_info_t;

enum {
  SKETCH_OK = 0,
  SKETCH_E_INVAL = -1,      /* bad argument or parameters */
  SKETCH_E_NOMEM = -2,      /* device or host allocation failed */
  SKETCH_E_HIP = -3,        /* a HIP runtime call failed */
  SKETCH_E_CAPACITY = -4,   /* output buffer too small; *n_out = needed */
  SKETCH_E_SATURATED = -5   /* a row has no zero bit left (psi = 1) */
};

/* Fill *p with the paper's defaults (g 1024, k 14, r 5, alpha 6), a fixed
 * seed and device 0. */
void sketch_params_default(sketch_params_t *p);

/* Check the parameters (see sketch_params_t); SKETCH_OK or SKETCH_E_INVAL. */
int sketch_params_check(const sketch_params_t *p);

/* Bytes of device memory the sketch itself takes: r * 2^k * g / 8.
 * 0 if the parameters are invalid. */
size_t sketch_bytes(const sketch_params_t *p);

/* Allocate a sketch on params->device with every bit 0 (Sec. 4: the DHLA
 * is zeroed at the start of a period), plus the restore work buffers.
 * *out receives the handle. Errors: INVAL (parameters, NULL), NOMEM, HIP. */
int sketch_create(const sketch_params_t *params, sketch_t **out);

/* Release the handle and all its device memory. Waits for the device. NULL
 * is ignored. */
void sketch_destroy(sketch_t *s);

/* Alg. 1 (Sec. 3.2, Sec. 4.1) for n_pairs pairs: for each (a,b), set bit
 * H1(b) of LE DH_i(a) in every row i. d_pairs is DEVICE memory holding
 * 2*n_pairs uint32 words, interleaved a0,b0,a1,b1,... (a = the measured
 * host, b = the opposite host), 8-byte aligned, owned by the caller and
 * kept alive until the stream has passed this call. Asynchronous on
 * hip_stream; accumulates into the window (OR is order-free, so any split
 * into calls gives the same sketch). n_pairs == 0 is a no-op.
 * Errors: INVAL (NULL handle, NULL or misaligned d_pairs with n_pairs > 0),
 * HIP (launch failure). */
int sketch_update(sketch_t *s, const uint32_t *d_pairs, size_t n_pairs,
                  void *hip_stream);

/* One sketch's share of a batched update. */
typedef struct {
  sketch_t *sketch;
  const uint32_t *d_pairs;   /* DEVICE memory, as for sketch_update */
  size_t n_pairs;
} sketch_update_job_t;

/* Alg. 1 for several sketches (links or windows of uneven size) in one set
 * of launches: each kernel of the update takes every job, so the batch
 * fills the GPU even when each job alone would not. The result is the same
 * as sketch_update on each job in turn. All sketches must be on one device
 * and distinct; pairs follow the rules of sketch_update. Asynchronous on
 * hip_stream. Errors: INVAL (NULL job list or handle, sketches on different
 * devices, a sketch twice, bad pairs pointer), NOMEM, HIP. */
int sketch_update_batch(const sketch_update_job_t *jobs, size_t n_jobs, void *hip_stream);

/* Alg. 2 (Sec. 3.3) computed as in Sec. 4.2: LEs with z0 < g*exp(-theta/g)
 * are hot; the candidates are every address whose r LEs are all hot (and
 * which re-hashes to its own LE in row 0), found by the join of Algs. 3-4
 * or by the lattice search, whichever the hot-list sizes make cheaper (the
 * same set either way; SKETCH_OPT_CANDIDATES forces one); each is reported iff
 * its eq. (4) estimate C >= theta (decided exactly as SZ <= floor(trep)).
 * out is HOST memory for cap records, filled ascending by address.
 * Synchronous: returns after the records are on the host. Does not change
 * the sketch, so it may be called again with another theta.
 * theta must be > 0. Errors: INVAL; CAPACITY (cap too small: *n_out = the
 * number needed, out untouched); SATURATED (some row has no zero bit);
 * NOMEM; HIP. *n_out (required) and *info (nullable) are written on
 * success, CAPACITY and SATURATED. */
int sketch_restore(sketch_t *s, double theta, sketch_sp_t *out, size_t cap,
                   size_t *n_out, sketch_info_t *info, void *hip_stream);

/* sketch_restore for callers that cannot allocate memory: code under HIP
 * graph capture, tight serving loops, hosts that forbid allocation while
 * running. It makes no device or host allocation and calls no allocating
 * library routine. Its work buffers (partial addresses, candidates, records
 * and their sorted copies, sort ranks) live in one fixed 64 MiB array per
 * GPU, set up when the first sketch on that GPU is created and held until
 * the process ends; the sketch's own restore arrays and pinned buffers
 * were allocated by sketch_create. Limits: at most 2^20 candidates and
 * 2^18 reported records; a join whose partial addresses outgrow the array
 * is redone by the lattice search (the same candidate set), or fails when
 * that search was ruled out (SKETCH_OPT_CANDIDATES = 1, or k > 20).
 * Beyond a limit it returns CAPACITY with a message naming it (*n_out is
 * then not set unless only cap was too small). Arguments, results and the
 * other errors are those of sketch_restore, and so is the output (the same
 * records, in the same order). Every call on a GPU shares that GPU's
 * array: the library orders calls through it like its other shared
 * buffers, but two threads calling it at once for handles on one GPU race
 * for the array (use one thread per GPU). */
int sketch_restore_noalloc(sketch_t *s, double theta, sketch_sp_t *out, size_t cap,
                           size_t *n_out, sketch_info_t *info, void *hip_stream);

/* One sketch's share of a batched restore. Inputs: sketch, theta, out
 * (HOST memory for cap records), cap, info (nullable). Outputs: n_out (the
 * number of records, also on CAPACITY) and status (the sketch_restore code
 * of this job). */
typedef struct {
  sketch_t *sketch;
  double theta;
  sketch_sp_t *out;
  size_t cap;
  sketch_info_t *info;
  size_t n_out;
  int status;
} sketch_restore_job_t;

/* sketch_restore for several distinct sketches on one device: every
 * restore is enqueued on hip_stream before one wait, so windows that close
 * together are reported together. Each job gets the result sketch_restore
 * would give it. Synchronous. Returns SKETCH_OK if every job succeeded,
 * else the first failing job's code (each job's status says which). Errors
 * before any work (NULL list or handle, bad theta or out, a sketch twice,
 * several devices): INVAL, with no job run. */
int sketch_restore_batch(sketch_restore_job_t *jobs, size_t n_jobs, void *hip_stream);

/* sketch_restore_batch in two halves, so that a caller can enqueue more
 * work (the next batch's update, on another stream) while these restores
 * run: the per-period cycle of Sec. 4 with one period's restore (Alg. 2,
 * Sec. 4.2) overlapping the next period's update (Alg. 1).
 * _begin checks the jobs and enqueues every restore on hip_stream, then
 * returns without waiting; it reads only the sketch and theta of each job.
 * _end waits for each job's restore (not for other work on the stream),
 * runs a job again on hip_stream if its output outgrew the shared buffers,
 * and fills out, info, n_out and status as sketch_restore_batch does.
 * Between the two calls the jobs' sketches may be used by no other call
 * except sketch_update / sketch_update_batch / sketch_reset, whose device
 * work the library orders after the pending restore (each sketch keeps an
 * event of its last work). _end must get the same sketches as _begin (in
 * any order, any subset at a time). Errors: as sketch_restore_batch; INVAL
 * also for a sketch with a restore begun and not ended (_begin) or none
 * begun (_end). */
int sketch_restore_batch_begin(sketch_restore_job_t *jobs, size_t n_jobs, void *hip_stream);
int sketch_restore_batch_end(sketch_restore_job_t *jobs, size_t n_jobs, void *hip_stream);

/* ---- plans: one window cycle of a fixed batch, replayed as a HIP graph ----
 *
 * The per-window cycle of Sec. 4 (reset the sketch, Alg. 1 over the
 * window's pairs, Alg. 2 at the window's end) for a fixed set of distinct
 * sketches whose pairs sit at fixed device addresses with fixed counts,
 * such as monitored links with one staging buffer each. The launches are
 * planned once (the same launches sketch_update_batch and
 * sketch_restore_batch would make) and captured into one HIP graph, so a
 * run is a single graph launch whatever the number of links and rounds.
 *
 * The plan owns its job tables, per-job update arrays and outputs, and
 * shares the device's update arena and restore buffers with every other
 * call (it captures again when another call has moved them). It reads the
 * sketches it was made with: destroy the plan before them, keep every
 * job's pairs valid while the plan is used, and order a run against other
 * work on the same sketches (same stream). Options set on a sketch after
 * sketch_plan_create do not apply to the plan. */
typedef struct sketch_plan sketch_plan_t;

typedef struct {
  sketch_t *sketch;
  const uint32_t *d_pairs;   /* DEVICE memory, as for sketch_update */
  size_t n_pairs;
  double theta;              /* restore threshold, > 0 with SKETCH_PLAN_RESTORE */
} sketch_plan_job_t;

enum {
  SKETCH_PLAN_RESET = 1,     /* a run starts with sketch_reset of every job */
  SKETCH_PLAN_RESTORE = 2    /* a run ends with the restore of every job */
};

/* Plans and captures. flags: SKETCH_PLAN_* bits. Synchronous (uploads the
 * job tables, allocates). Errors: INVAL (as sketch_update_batch, bad theta
 * or flags, no jobs), NOMEM, HIP. */
int sketch_plan_create(const sketch_plan_job_t *jobs, size_t n_jobs, int flags,
                       sketch_plan_t **out);

/* One run: one graph launch on hip_stream, asynchronous. */
int sketch_plan_run(sketch_plan_t *plan, void *hip_stream);

/* The last run's restore results, one slot per job in creation order
 * (out[j].sketch must be job j's sketch; out, cap and info as in
 * sketch_restore_batch; theta is written back). Waits for hip_stream. A
 * job whose output overflowed the plan's buffers is restored again on its
 * own and the buffers grow (the graph is rebuilt before the next run), so
 * every job gets exactly what sketch_restore would give. Returns SKETCH_OK
 * if every job succeeded, else the first failing job's code. */
int sketch_plan_results(sketch_plan_t *plan, sketch_restore_job_t *out, size_t n_out,
                        void *hip_stream);

/* Update launches in one run (each a set of kernels over many jobs). */
size_t sketch_plan_launches(const sketch_plan_t *plan);

/* Waits for the device, frees the plan. NULL is a no-op. */
void sketch_plan_destroy(sketch_plan_t *plan);

/* Start a new window: every bit of the sketch back to 0 (Sec. 4).
 * Enqueues nothing: the sketch is marked all zero, and the zeros are written
 * by the next call that needs them, on that call's stream. A binned update
 * from the window's first pair writes every tile from zeros instead of
 * reading it; a direct update, restore, merge into the sketch or plan run
 * without SKETCH_PLAN_RESET writes the zeros first; a download returns
 * zeros. hip_stream is unused. Errors: INVAL. */
int sketch_reset(sketch_t *s, void *hip_stream);

/* Merge the window of another monitor into this one: dst |= src, bit by bit
 * (the router-merge step of Sec. 4.2). The paper writes the merge as a
 * bit-wise AND; OR is what reproduces the sketch of the union of both pair
 * streams (a bit is set iff some pair of either stream sets it), so the
 * merged sketch equals the one a single monitor would have built. Both
 * sketches must have the same g, k, r, alpha and seed and be on one device.
 * Asynchronous on hip_stream; src is unchanged. Errors: INVAL, HIP. */
int sketch_merge(sketch_t *dst, const sketch_t *src, void *hip_stream);

/* ---- tuning ---- */

/* Options of sketch_set_option. The update has two kernels computing the
 * same sketch: "direct" (each pair sets its r bits with a check-then-
 * atomicOr in the sketch, Alg. 1 as written) and "binned" (the bit sets are
 * grouped by 160 KiB tile of the sketch and applied in LDS, one workgroup
 * per tile or part of a tile; sketches of up to 3276 tiles, 511.9 MiB). */
enum {
  SKETCH_OPT_UPDATE_PATH = 1,       /* 0 = choose by size (default),
                                       1 = direct, 2 = binned */
  SKETCH_OPT_BINNED_MIN_PAIRS = 2,  /* "choose by size": binned at and above
                                       this many pairs per call */
  SKETCH_OPT_UPDATE_GRID = 3,       /* blocks of the direct kernel */
  SKETCH_OPT_UPDATE_CHECK = 4,      /* direct kernel: 1 = test the bit before
                                       the atomicOr (default), 0 = always OR */
  SKETCH_OPT_BINNED_ROUND = 5,      /* binned: pairs per round, 1024 to 2^28
                                       (default 2^28); the round's
                                       codes (three per 8 bytes, in regions
                                       and a spill area of that size each)
                                       take about 5.4*r bytes per pair of
                                       device memory, allocated on first use */
  SKETCH_OPT_SCATTER_PPT = 6,       /* binned: pairs per thread in one LDS
                                       sorting batch: 2, 4 or 6 (default);
                                       capped by LDS at 4 for r in 6..7 and
                                       at 2 for r = 8. Sketches of more than
                                       2048 tiles (of 160 KiB) take 5 for
                                       r <= 5 up to 3072 tiles and 4 above
                                       (4 and 6 both ask for that), and 2
                                       for r >= 6 */
  SKETCH_OPT_BINNED_BLOCKS = 7,     /* binned: blocks of the count and
                                       scatter passes at most, 1..1024
                                       (default: one per compute unit); a
                                       window takes fewer when it has less
                                       than 4096 pairs per block per binned
                                       job of the call (32768 at most) */
  SKETCH_OPT_TRIM_POOLS = 8,        /* device-wide, acts at once: waits for
                                       pending work on the shared buffers,
                                       frees the update arena and reallocates
                                       the restore pool at `value` entries per
                                       buffer, 0..2^24 (0 = the initial sizes);
                                       both grow again on demand. Frees device
                                       memory for callers under a budget */
  SKETCH_OPT_APPLY_BLOCKS = 9,      /* binned: blocks of the apply pass;
                                       0 = one per apply item (default: the
                                       dispatcher balances uneven tiles), else
                                       that many blocks striding over the
                                       items */
  SKETCH_OPT_TIMING = 10,           /* 1 = every restore records timing
                                       events between its phases (read them
                                       with sketch_timings), 0 = off (default) */
  SKETCH_OPT_CANDIDATES = 11,       /* how the restore finds the addresses
                                       whose r LEs are all hot (the same set
                                       either way): 0 = the cheaper by the
                                       hot-list sizes (default), 1 = the join
                                       of Algs. 3-4, 2 = the lattice search
                                       (every address of each hot row-0 LE,
                                       enumerated from the structure of DH0,
                                       tested in rows 1..r-1; needs k <= 20) */
  SKETCH_OPT_BINNED_SAMPLE = 12,    /* binned: the count pass, which sizes
                                       each tile's code regions, reads every
                                       n-th batch of pairs, 1..1024 (1: all,
                                       regions sized exactly); 0 = 16 when
                                       the job has 4096 batches or more over
                                       its blocks, fewer below, keeping about
                                       256 sampled (default) */
  SKETCH_OPT_BINNED_REGIONS = 13,   /* binned: a region holds value/64 of its
                                       estimate plus 64 code words, 0..1024;
                                       0 = 9/8 of a sampled estimate, the
                                       exact count when every batch is read
                                       (default). Runs that do not fit go to
                                       a spill area (small values force that,
                                       for tests) */
  SKETCH_OPT_JOIN_BLOCKS = 14       /* blocks of each join stage (Algs. 3-4),
                                       1 to four per compute unit; 0
                                       (default) = four per compute unit, or
                                       one when the sketch's last restore
                                       had fewer stage-1 wave items (|HE(0)|
                                       times ceil(|HE(1)| / 64)) than compute
                                       units. Each block takes an equal share
                                       of the stage's items and writes its
                                       own segment of partial addresses */
};

/* Phases of the last restore that ran with SKETCH_OPT_TIMING on (device
 * time between events recorded on its stream), with the work each phase
 * did, for rooflines of the restore kernels (Alg. 2 and Algs. 3-4 as
 * computed in Sec. 4.2, eq. (4)). */
typedef struct {
  float hot_scan_ms;        /* state reset and hot scan: z0, ZR(i), hot bitmap */
  float rows_ms;            /* HE(i) compaction, bucket tables, scalars */
  float join_ms;            /* the candidate search: every join stage, or
                               the lattice search */
  float estimate_ms;        /* ULE gathers, SZ, C, report test */
  float sort_publish_ms;    /* sort by address, state and records to the host */
  uint64_t hot_scan_bytes;  /* bytes the hot scan read: the zero counts the
                               binned update kept (4 per LE) or the sketch */
  uint64_t join_probes;     /* bucket probes: |HE(0)|*|HE(1)| for stage 1,
                               then one per partial address of each stage */
  uint64_t join_outputs;    /* tuples the probes accepted, every stage (the
                               lattice search: the candidates) */
  uint64_t estimate_bytes;  /* candidates * r * g / 8 (the LEs gathered) */
  uint32_t search;          /* the search that ran: 1 join, 2 lattice (0: none,
                               the sketch was saturated) */
  uint32_t pad;
  uint64_t lattice_points;  /* lattice search: addresses of the hot row-0 LEs,
                               |HE(0)| * 2^(32-k); 0 for the join */
} sketch_timings_t;

/* The timings of the last timed restore of s (waits for its events).
 * Errors: INVAL (NULL argument, or no restore ran with timing on since
 * SKETCH_OPT_TIMING was set), HIP. */
int sketch_timings(sketch_t *s, sketch_timings_t *out);

/* Set a tuning option; results never depend on it. Errors: INVAL (NULL
 * handle, unknown option, value out of range, binned path on a sketch of
 * more than 4096 slices). */
int sketch_set_option(sketch_t *s, int option, int64_t value);

/* ---- test and checkpoint hooks ---- */

/* Copy the sketch to HOST memory host_words (n_words must equal
 * sketch_bytes()/4). Synchronous. Errors: INVAL, HIP. */
int sketch_download(const sketch_t *s, uint32_t *host_words, size_t n_words,
                    void *hip_stream);

/* Replace the sketch with HOST memory host_words (n_words must equal
 * sketch_bytes()/4). Synchronous. Errors: INVAL, HIP. */
int sketch_upload(sketch_t *s, const uint32_t *host_words, size_t n_words,
                  void *hip_stream);

/* The candidate set of sketch_restore before the estimate step: every
 * address whose r LEs are all hot for theta, ascending, into HOST memory
 * out. Synchronous. Errors as sketch_restore. */
int sketch_candidates(sketch_t *s, double theta, uint32_t *out, size_t cap,
                      size_t *n_out, void *hip_stream);

/* Message of the last failed call on this thread ("" if none). */
const char *sketch_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDHF_H */

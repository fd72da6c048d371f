/*
 * qrng.h -- C ABI of libqrng: QRNG post-processing on one AMD Instinct MI355X
 * (gfx950): min-entropy estimation with a statistical-distance correction and
 * Toeplitz-hashing randomness extraction over GF(2).
 *
 * Paper: Z. Zhao, "Performance Optimization on Practical Quantum Random
 * Number Generators: Modification on Min-entropy Evaluation and Acceleration
 * on Post Processing", arXiv 2011.04130.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Bit strings are packed LSB first into little-endian 64-bit words: bit b is
 * bit (b % 64) of word b / 64.  Raw ADC samples of N <= 8 bits are one byte
 * each; the byte buffer viewed as 64-bit words is the packed raw block (bit
 * 8t + i is bit i of sample t).  Bits past the stated length of an input are
 * ignored; output bits past m in the last word are written as 0.
 *
 * Device pointers ("_dev") refer to memory on the context's device and must be
 * 8-byte aligned.  The caller owns every buffer it passes; the library never
 * frees caller memory.  `stream` is a hipStream_t (NULL = the null stream).
 * Hash calls only enqueue work and return; results are ready when the stream
 * reaches that point.  Calls that return host values synchronise the stream.
 *
 * Errors: argument errors are detected before anything is enqueued and return
 * QRNG_EINVAL; HIP failures return QRNG_EDEVICE.  The library never aborts.
 * qrng_last_error() gives a thread-local message for the last failure.
 * A context may be used from one host thread at a time, and its workspace
 * (transform buffers, histogram scratch) is shared by its calls: work that
 * calls enqueue on different streams must not overlap in time.  Plans and
 * servers own their workspace.
 */
#ifndef QRNG_H
#define QRNG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QRNG_OK = 0,
  QRNG_EINVAL = -1,       /* bad argument (nothing was enqueued) */
  QRNG_ENOMEM = -2,       /* device or host allocation failed */
  QRNG_EDEVICE = -3,      /* a HIP call failed */
  QRNG_EUNSUPPORTED = -4, /* valid request this path cannot serve */
  QRNG_EBUSY = -5         /* resource limit (admission) reached */
} qrng_status;

/* Which extraction kernel to run.  All paths return identical bits. */
typedef enum {
  QRNG_PATH_AUTO = 0,   /* library picks (autotuned plan table if loaded) */
  QRNG_PATH_DIRECT = 1, /* bit-packed AND/parity mat-vec, O(mn); n+m-1 < 2^34 */
  QRNG_PATH_NTT = 2,    /* exact convolution mod 998244353, O(L log L) */
  QRNG_PATH_MFMA = 3    /* matrix-core product (fp4 operands, exact fp32 sums), shared-seed batches */
} qrng_path;

/* The set U over which the statistical distance is taken (Sec. II.C). */
typedef enum {
  QRNG_U_MODEL_ARGMAX = 0, /* U = {argmax P}, the paper's chain of bounds */
  QRNG_U_BOTH_ARGMAX = 1,  /* U = {argmax P, argmax P'}, every value tied for the
                              maximum of P included (never over-estimates) */
  QRNG_U_ALL = 2           /* U = all values: total-variation distance */
} qrng_u_mode;

/* Where the ideal (model) distribution's Gaussian parameters come from. */
typedef enum {
  QRNG_MODEL_FIT = 0,   /* mean and population s.d. of the same samples */
  QRNG_MODEL_GIVEN = 1, /* the caller's mu, sigma (sigma > 0) */
  /* Sec. II.B classical-noise subtraction: the samples' mean, and the
   * quantum part of their s.d., sigma_q^2 = sigma_fit^2 - sigma_c^2 with the
   * classical noise's s.d. sigma_c (measured with the source off) passed in
   * `sigma` (>= 0); sigma_c >= sigma_fit leaves a point-mass model. */
  QRNG_MODEL_QUANTUM = 2
} qrng_model;

typedef struct qrng_ctx qrng_ctx;

typedef struct {
  int32_t sample_bits; /* N, 1..8: ADC bits per sample */
  int32_t model;       /* qrng_model */
  double mu, sigma;    /* QRNG_MODEL_GIVEN: both; QRNG_MODEL_QUANTUM: sigma = sigma_c */
  int32_t u_mode;      /* qrng_u_mode */
  int32_t reserved;    /* must be 0 */
} qrng_me_opts;

typedef struct {
  double mu_hat, sigma_hat; /* model parameters used */
  double h_min;             /* -log2 max_x P(x), ideal model (Sec. II.A) */
  double h_actual;          /* -log2 max_x P'(x), observed histogram */
  double d_u;               /* (1/2) sum_{x in U} |P'(x) - P(x)| */
  double delta_h_m;         /* log2(d_U / 2^-(N+1) + 1) */
  double h_mod;             /* h_min - delta_h_m (Sec. II.C) */
  uint32_t argmax_model, argmax_empirical;
  uint64_t samples;
} qrng_me_result;

/* One block of a batched hash: raw bits x_pool[x_word_off*64 ...] (n bits)
 * hashed with the first n+m-1 bits of registered seed `seed_id` into
 * y_pool[y_word_off*64 ...] (m bits).  Blocks must not overlap in y. */
typedef struct {
  uint64_t x_word_off;
  uint64_t n;
  uint64_t m;
  uint64_t y_word_off;
  uint32_t seed_id;
  uint32_t flags; /* must be 0 */
} qrng_block;

/* Library version string (static storage). */
const char *qrng_version(void);

/* Thread-local text of the last error reported by this thread. */
const char *qrng_last_error(void);

/* Create a context on HIP device `device`: uploads the transform tables.
 * *ctx receives the handle; destroy it with qrng_destroy. */
qrng_status qrng_create(qrng_ctx **ctx, int device);

/* Wait for the context's outstanding work and release everything it owns
 * (workspace, cached seed spectra).  NULL is a no-op. */
void qrng_destroy(qrng_ctx *ctx);

/* Sec. II: histogram of S samples (uint8, values < 2^N) on the device, then
 * on the host: the Gaussian model P (fitted or given; codes 0 and 2^N-1 take
 * the clipped tails), H_min = -log2 max P, the observed P' = counts/S, the
 * statistical distance d_U over U, Delta H_m = log2(d_U / 2^-(N+1) + 1) and
 * H_modify = H_min - Delta H_m.  `counts_host` (nullable) receives the 2^N
 * counts.  Synchronises `stream`.  EINVAL if S == 0, N outside 1..8, a
 * sample is >= 2^N (detected after the histogram), or a given sigma <= 0. */
qrng_status qrng_minentropy(qrng_ctx *ctx, const uint8_t *samples_dev, uint64_t S,
                            const qrng_me_opts *opts, qrng_me_result *out_host,
                            uint64_t *counts_host, void *stream);

/* As qrng_minentropy on a random subset of the samples (Sec. II.C proposes
 * estimating on randomly chosen raw data): sample t counts when the high 32
 * bits of output t of SplitMix64 seeded with subset_seed -- mix(subset_seed +
 * (t+1) 0x9e3779b97f4a7c15), mix = the generator's published finaliser
 * (xor-shift 30, multiply 0xbf58476d1ce4e5b9, xor-shift 27, multiply
 * 0x94d049bb133111eb, xor-shift 31) -- are below keep_thr, so about
 * keep_thr / 2^32 of them count.  keep_thr == 0 counts every sample (the
 * plain estimate).  counts_host (nullable) receives the subset's counts;
 * out_host->samples is the number kept.  QRNG_EINVAL if none is kept. */
qrng_status qrng_minentropy_subset(qrng_ctx *ctx, const uint8_t *samples_dev, uint64_t S,
                                   const qrng_me_opts *opts, uint64_t subset_seed,
                                   uint32_t keep_thr, qrng_me_result *out_host,
                                   uint64_t *counts_host, void *stream);

/* Sec. III.B output length m = n H/N - 2 log2(1/eps), with H counted in whole
 * bits per sample (floor of h_mod, at least 0), the security term rounded up
 * (log2_inv_eps >= 0), and m clamped to [0, n].  Pure host function. */
qrng_status qrng_output_bits(uint64_t n, int sample_bits, double h_mod,
                             double log2_inv_eps, uint64_t *m_out);

/* Sec. III.B Toeplitz hash y = T x mod 2 of one block: x is n raw bits, the
 * seed is n+m-1 bits, T[i][j] = seed[n-1+i-j] (first row seed bits n-1 down to
 * 0, first column seed bits n-1 up to n+m-2), y is m bits.  y_dev holds
 * ceil(m/64) words and must not overlap x or the seed.  0 < n; m <= n; m == 0
 * is a no-op.  The NTT path needs n < 998244353.  Enqueued on `stream`. */
qrng_status qrng_toeplitz_hash(qrng_ctx *ctx, const uint64_t *x_dev, uint64_t n,
                               const uint64_t *seed_dev, uint64_t m, uint64_t *y_dev,
                               int path, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * hash as qrng_toeplitz_hash (same arguments, bits and errors) with every
 * intermediate buffer in a fixed scratch array of QRNG_NOALLOC_SCRATCH_BYTES
 * per device, which the library holds until the process ends.  The call
 * allocates nothing and creates nothing (no HIP events either, so
 * qrng_profile_* does not see it).  Limits: the transform path needs
 * 4 (nwin + 1) Nc bytes (one transform of Nc >= n+m-1 points: Nc <= 2^21,
 * so n+m-1 <= 2^21), the direct path about n/8 bytes; QRNG_EINVAL beyond
 * them, with nothing enqueued.  The matrix-core path uses no scratch.  Every
 * call on one device -- from any context -- shares that device's array, and
 * each call rewrites all of it that it reads: calls whose work overlaps in
 * time on one device (different streams, or different host threads) race
 * and must be ordered by the caller.  Enqueued on `stream`. */
#define QRNG_NOALLOC_SCRATCH_BYTES (16u << 20)
qrng_status qrng_toeplitz_hash_noalloc(qrng_ctx *ctx, const uint64_t *x_dev, uint64_t n,
                                       const uint64_t *seed_dev, uint64_t m, uint64_t *y_dev,
                                       int path, void *stream);

/* Register a seed of L bits for reuse (Sec. III.B: the seed a_1 .. a_{n+m-1}
 * is chosen once and applied to many raw blocks).  The memory must stay
 * unchanged and allocated until qrng_seed_unregister or qrng_destroy.  The
 * transform-domain copies of the seed's first 2^k bits, for every k from 10
 * up to min(23, ceil(log2 L)) -- one per transform length a block with this
 * seed can need -- are computed here, enqueued on `stream` after the caller's
 * earlier work there (the copy that filled the seed, say), and the call waits
 * for them; copies for blocks above 2^23 bits are computed on first use.
 * *seed_id receives the lowest free id (ids are below 4096: QRNG_EBUSY when
 * 4095 seeds are registered). */
qrng_status qrng_seed_register(qrng_ctx *ctx, const uint64_t *seed_dev, uint64_t L,
                               uint32_t *seed_id, void *stream);
qrng_status qrng_seed_unregister(qrng_ctx *ctx, uint32_t seed_id);

/* As qrng_toeplitz_hash with a registered seed (its first n+m-1 bits). */
qrng_status qrng_toeplitz_hash_seeded(qrng_ctx *ctx, const uint64_t *x_dev, uint64_t n,
                                      uint32_t seed_id, uint64_t m, uint64_t *y_dev,
                                      int path, void *stream);

/* The paper's own accelerated method (Sec. III.B, Definition 1 and Theorems
 * 1-2) in float64, for comparison with the exact paths: the seed's n+m-1 bits
 * and the raw block zero-padded to a power-of-two length N >= n+m-1 are
 * transformed together (one complex transform, the two real spectra
 * separated), multiplied, transformed back; the kept rows n-1 .. n+m-2 are
 * divided by N, rounded to the nearest integer and reduced mod 2.  Same
 * arguments and output as qrng_toeplitz_hash; n+m-1 <= 2^26; workspace of
 * 32 N bytes in the context.  max_err_dev (nullable, device double) receives
 * the largest distance of a kept value from its integer: the bits equal the
 * exact hash while it stays below 1/2 (it is about 1e-9 at N = 2^24).
 * Enqueued on `stream`. */
qrng_status qrng_toeplitz_hash_fft64(qrng_ctx *ctx, const uint64_t *x_dev, uint64_t n,
                                     const uint64_t *seed_dev, uint64_t m, uint64_t *y_dev,
                                     double *max_err_dev, void *stream);

/* Sec. III.D modified Toeplitz hash k = (A, I_m) x mod 2 with an (n-1)-bit
 * seed a: A is the m x (n-m) Toeplitz block A[i][j] = a[n-m-1+i-j] (seed bit
 * q is a_{q+1} of the paper; first row a[n-m-1] down to a[0], first column
 * a[n-m-1] up to a[n-2]) and the identity block adds raw bit n-m+i to key bit
 * i.  x is n raw bits, y is m bits (ceil(m/64) words, bits from m on written
 * as 0) and must not overlap x or the seed.  0 < n; m <= n; m == 0 is a
 * no-op; m == n gives y = x.  The product A x[0, n-m) runs on `path` like
 * qrng_toeplitz_hash on an (n-m)-bit block (m may exceed n-m here), then one
 * kernel adds the identity part.  Enqueued on `stream`. */
qrng_status qrng_modified_toeplitz_hash(qrng_ctx *ctx, const uint64_t *x_dev, uint64_t n,
                                        const uint64_t *seed_dev, uint64_t m, uint64_t *y_dev,
                                        int path, void *stream);
/* As qrng_modified_toeplitz_hash with a registered seed (its first n-1 bits;
 * the transform-domain copy is shared with ordinary hashes of the same
 * transform length). */
qrng_status qrng_modified_toeplitz_hash_seeded(qrng_ctx *ctx, const uint64_t *x_dev,
                                               uint64_t n, uint32_t seed_id, uint64_t m,
                                               uint64_t *y_dev, int path, void *stream);

/* One asynchronous pass of the whole path over a block of S 8-bit samples
 * (S a multiple of 8): the histogram and the min-entropy estimate of Sec. II,
 * the output length m of Sec. III.B (whole bits per sample, minus
 * ceil(2 log2_inv_eps), clamped to [0, m_cap]) and the Toeplitz hash of the
 * n = 8 S raw bits (the sample bytes themselves) with the first n+m-1 bits of
 * registered seed `seed_id` -- all on the device, without synchronising the
 * stream or copying anything to the host.  The transform is planned for
 * m_cap, so y_dev holds ceil(m_cap/64) words; bits from m to m_cap are 0.
 * m_dev / out_dev (nullable, device memory) receive m and the estimate
 * (qrng_me_result) when the stream reaches them.  The seed must have at
 * least n + m_cap - 1 bits.  Same estimate and bits as qrng_minentropy +
 * qrng_output_bits + qrng_toeplitz_hash_seeded.  The partial histograms
 * carry the call's tag and sample counts, checked before the estimate uses
 * them: should a check ever fail, the call fails closed -- m = 0 (no output
 * bits) and the estimate's fields NaN with samples = 0 -- rather than
 * extract with an unchecked length (qrng_minentropy returns QRNG_EDEVICE). */
qrng_status qrng_extract(qrng_ctx *ctx, const uint8_t *samples_dev, uint64_t S,
                         const qrng_me_opts *opts, double log2_inv_eps, uint32_t seed_id,
                         uint64_t m_cap, uint64_t *y_dev, uint64_t *m_dev,
                         qrng_me_result *out_dev, int path, void *stream);

/* Sec. III.E (Fig. 5): a long raw sequence cut into nblocks equal blocks.
 * Block b is the n bits starting at word b*x_stride_words of x_pool_dev; its
 * m-bit hash with the first n+m-1 bits of registered seed `seed_id` goes to
 * word b*y_stride_words of y_pool_dev.  Strides are at least ceil(n/64) and
 * ceil(m/64); the pools must not overlap.  Each block's bits equal
 * qrng_toeplitz_hash_seeded on that block alone.  Enqueued on `stream`. */
qrng_status qrng_toeplitz_hash_strided(qrng_ctx *ctx, const uint64_t *x_pool_dev, uint64_t n,
                                       uint64_t x_stride_words, uint32_t seed_id, uint64_t m,
                                       uint64_t *y_pool_dev, uint64_t y_stride_words,
                                       uint32_t nblocks, int path, void *stream);

/* Hash many blocks (Sec. III.E: a long raw sequence split into blocks, here
 * of any lengths) whose descriptors are in DEVICE memory: the library never
 * reads them on the host, so the descriptors may be written by earlier work on
 * `stream` and the whole call may be captured in a HIP graph.  Block b is
 * blocks_dev[b] (qrng_block: raw bits at word x_word_off of x_pool_dev, n
 * bits; m output bits at word y_word_off of y_pool_dev, bits past m in its last
 * word written as 0), hashed with the first n+m-1 bits of registered seed
 * seed_ids_or_null[b] (device memory, nblocks entries) or, when that pointer
 * is NULL, of blocks_dev[b].seed_id.  Each block's bits equal
 * qrng_toeplitz_hash_seeded on that block alone.
 * On the device each block is checked (flags 0, 0 < n < 2^31, m <= n, a
 * registered seed of at least n+m-1 bits, n+m-1 <= 2^23 and no longer than
 * the longest seed registered when the call was made), sorted by transform
 * length and hashed on the transform path; a block that fails a check is
 * skipped (its output untouched) and counted, see
 * qrng_toeplitz_hash_batched_rejected; m == 0 blocks are skipped.  The
 * caller guarantees that the offsets lie inside the pools and that outputs
 * do not overlap each other or the raw pool.  path: QRNG_PATH_AUTO or
 * QRNG_PATH_NTT (others: QRNG_EUNSUPPORTED; host-descriptor batches and
 * plans offer every path).  The context keeps per-class item lists for
 * nblocks blocks and a transform workspace of up to 4 GiB: the first call
 * with more blocks, or after a longer seed was registered, allocates them;
 * later calls allocate nothing.  Enqueued on `stream`. */
qrng_status qrng_toeplitz_hash_batched(qrng_ctx *ctx, const qrng_block *blocks_dev,
                                       uint32_t nblocks, const uint64_t *x_pool_dev,
                                       const uint32_t *seed_ids_or_null, uint64_t *y_pool_dev,
                                       int path, void *stream);

/* Number of descriptors the context's last qrng_toeplitz_hash_batched call
 * skipped as invalid (waits for `stream`, which must be the one that call
 * used). */
qrng_status qrng_toeplitz_hash_batched_rejected(qrng_ctx *ctx, uint32_t *count_host,
                                                void *stream);

/* As qrng_toeplitz_hash_batched with the descriptors in host memory
 * (`blocks_host`, each block's own seed_id), checked on the host before
 * anything is enqueued (EINVAL on the first bad one, overlapping outputs
 * included).  Blocks are grouped by shape and seed; `path` forces one path
 * for all (AUTO lets the library choose per group). */
qrng_status qrng_toeplitz_hash_batched_host(qrng_ctx *ctx, const qrng_block *blocks_host,
                                            uint32_t nblocks, const uint64_t *x_pool_dev,
                                            uint64_t *y_pool_dev, int path, void *stream);

/* ------------------------------------------------------------------ plans
 * An uneven batch fixed once and replayed (Sec. III.E: a raw sequence cut
 * into blocks, here of unequal lengths, each with the output length its own
 * Sec. II estimate allows).  Creating a plan validates the descriptors,
 * copies them to device memory, prepares the seed spectra, groups the blocks
 * by transform length (blocks of one length share each launch) and,
 * with QRNG_PLAN_GRAPH, records the launches as one HIP graph.  The pools and
 * m_dev / me_dev are bound to the plan: every execution reads x_pool_dev as
 * it is then and rewrites the outputs.
 *
 * QRNG_PLAN_ESTIMATE: block b's raw bits are its n/8 bytes of 8-bit samples
 *   (n a multiple of 64); its histogram and Sec. II estimate run on the
 *   device (opts, log2_inv_eps as in qrng_extract), m_dev[b] receives its
 *   output length m_b = min(blocks[b].m, n H/8 - ceil(2 log2_inv_eps)) and
 *   me_dev[b] (nullable) its estimate; blocks[b].m is the cap the output
 *   is sized for (bits from m_b up to it are written as 0).
 *   Without it each block's m is blocks[b].m and m_dev / me_dev are unused.
 * QRNG_PLAN_TUNE: time the candidate launch shapes of every transform-length
 *   class now (this runs the plan's kernels on `stream` and writes the
 *   outputs), keep the fastest, and remember it in the context's tuning
 *   table (qrng_tune_export / qrng_tune_import) for later plans.
 * QRNG_PLAN_GRAPH: qrng_plan_execute replays one HIP graph.
 *
 * Seeds used by a live plan cannot be unregistered (QRNG_EBUSY).  Each
 * block's result equals qrng_toeplitz_hash_seeded on that block alone (with
 * m = m_dev[b] under QRNG_PLAN_ESTIMATE).  One plan must not be executed on
 * two streams at once (its workspace is shared); qrng_destroy destroys the
 * context's remaining plans. */
enum {
  QRNG_PLAN_ESTIMATE = 1,
  QRNG_PLAN_GRAPH = 2,
  QRNG_PLAN_TUNE = 4
};

typedef struct qrng_plan qrng_plan;

typedef struct {
  uint32_t blocks;          /* descriptors */
  uint32_t classes;         /* transform-length classes launched together */
  uint32_t launches;        /* launch groups per execution (estimate included) */
  uint32_t graph;           /* 1 if executions replay a HIP graph */
  uint64_t workspace_bytes; /* device workspace the plan owns */
} qrng_plan_info;

qrng_status qrng_plan_create(qrng_ctx *ctx, const qrng_block *blocks_host, uint32_t nblocks,
                             const uint64_t *x_pool_dev, uint64_t *y_pool_dev,
                             uint64_t *m_dev, qrng_me_result *me_dev,
                             const qrng_me_opts *opts, double log2_inv_eps, int path,
                             uint32_t flags, void *stream, qrng_plan **plan);

/* Enqueue one execution of the plan on `stream`. */
qrng_status qrng_plan_execute(qrng_plan *plan, void *stream);

qrng_status qrng_plan_query(const qrng_plan *plan, qrng_plan_info *info);

/* Waits for the device, then frees the plan.  NULL is a no-op. */
void qrng_plan_destroy(qrng_plan *plan);

/* The context's tuning table as text, one line per entry
 * "ntt <log2 Nc> <ceil log2 class size> <shape>" (shape: log2 of the
 * per-launch workspace cap in bytes, 40 = none, -1 = one direct launch per
 * block) or "multi <ceil log2 block count> <form>" (1 = the persistent
 * three-launch form, 0 = per-class launches).  An entry that a tuning run
 * of this context measured is followed by a comment line
 * "# <entry key> measured <shape>:<ms> ..." with the time of every
 * candidate (qrng_tune_import skips '#' lines).  *len receives the length
 * without the terminating 0; buf (nullable) receives the text if cap > len. */
qrng_status qrng_tune_export(qrng_ctx *ctx, char *buf, uint64_t cap, uint64_t *len);

/* Merge a table written by qrng_tune_export (EINVAL on a malformed line,
 * nothing merged then). */
qrng_status qrng_tune_import(qrng_ctx *ctx, const char *text);

/* ---------------------------------------------------------------- serving
 * Continuous batching of extraction requests over a stream of raw windows.
 * The raw stream arrives in windows of W 8-bit samples (qrng_server_feed
 * copies each into one of the server's window slots).  Each window gets one
 * Sec. II estimate and is cut into blocks of n_s raw bits; each block hashes
 * (Sec. III.B, the server's seed) to m_s output bits, m_s = n_s H/8 -
 * ceil(2 log2(1/eps)) rounded down to a multiple of 64 (fewer rows of T are
 * still an extractor).  A request for R bits takes ceil(R/m_s) consecutive
 * unused blocks of ONE window (one estimate applies), and its output is their
 * hashes concatenated and cut to R bits, contiguous in the server's output
 * ring.  qrng_server_step admits queued requests first come first served
 * while the ring has room for their outputs (admission by memory) and
 * enqueues one hash launch per run of admitted blocks; a request whose head
 * does not fit in the rest of the current window moves the server to the
 * next window.  The bits a request receives depend only on the window and the
 * blocks it was given, never on the other requests batched with it.
 * A server belongs to one context and one host thread.  qrng_destroy
 * destroys the context's servers. */
typedef struct qrng_server qrng_server;

typedef struct {
  uint64_t window_samples; /* W: samples per window, a multiple of n_s / 8 */
  uint64_t block_bits;     /* n_s: multiple of 512, or 0 = chosen by timing candidates */
  uint64_t ring_bits;      /* output ring capacity, multiple of 64 */
  uint32_t window_slots;   /* windows held at once (>= 2) */
  uint32_t max_queue;      /* queued requests accepted (QRNG_EBUSY beyond) */
  uint32_t seed_id;        /* registered seed with >= 2 n_s - 1 bits */
  int32_t path;            /* hash path (QRNG_PATH_AUTO lets the library pick) */
  qrng_me_opts opts;       /* estimate options; sample_bits must be 8 */
  double log2_inv_eps;
} qrng_server_cfg;

typedef struct {
  uint64_t request_id;
  uint64_t bits;           /* R */
  uint64_t ring_word;      /* output starts at word ring_word of the ring */
  uint64_t window;         /* sequence number of the window (0, 1, ...) */
  uint64_t first_block;    /* its first block in that window */
  uint32_t blocks;         /* ceil(R / m_s) */
  int32_t status;          /* QRNG_OK, or QRNG_EUNSUPPORTED if R can never fit */
  uint64_t m_block;        /* m_s of that window */
} qrng_served;

typedef struct {
  uint64_t block_bits, blocks_per_window;
  uint64_t windows_fed, windows_used, blocks_hashed, bits_served;
  uint64_t queued, in_flight, ring_free_bits;
  uint64_t m_block;        /* m_s of the current window (0 before the first) */
} qrng_server_stats;

/* Create a server: allocates the window slots and the output ring, and
 * with block_bits == 0 times the candidate block lengths on one window's
 * worth of blocks (nominal H = 5 bits per sample) and keeps the one that
 * extracts the most bits per second. */
qrng_status qrng_server_create(qrng_ctx *ctx, const qrng_server_cfg *cfg, qrng_server **srv);

/* Copy W samples from samples_dev into a free window slot, enqueued on
 * `stream` after its earlier work, and enqueue the window's estimate.
 * QRNG_EBUSY if every slot holds a window still in use. */
qrng_status qrng_server_feed(qrng_server *srv, const uint8_t *samples_dev, void *stream);

/* Queue a request for `bits` > 0 output bits; *request_id receives its id.
 * QRNG_EBUSY if max_queue requests are already waiting. */
qrng_status qrng_server_submit(qrng_server *srv, uint64_t bits, uint64_t *request_id);

/* Queue up to `count` requests in order (bits_host[i] > 0 each, else
 * QRNG_EINVAL and none queued).  Requests 0 .. *accepted - 1 are queued
 * (acceptance stops at the first that would exceed max_queue) and
 * ids_host[i] receives the id of request i. */
qrng_status qrng_server_submit_many(qrng_server *srv, const uint64_t *bits_host, uint32_t count,
                                    uint64_t *ids_host, uint32_t *accepted);

/* Admit what fits and enqueue the hashes (never waits for the GPU except
 * for the estimate of a window it moves to).  *admitted (nullable) receives
 * the number of requests admitted. */
qrng_status qrng_server_step(qrng_server *srv, uint32_t *admitted);

/* Completed requests, oldest first, up to cap; *count receives how many were
 * written to out_host.  Their outputs are in the ring until released. */
qrng_status qrng_server_poll(qrng_server *srv, qrng_served *out_host, uint32_t cap,
                             uint32_t *count);

/* Give a completed request's ring space back. */
qrng_status qrng_server_release(qrng_server *srv, uint64_t request_id);

/* Release many: ids that hold no ring space or are not completed are
 * skipped. */
qrng_status qrng_server_release_many(qrng_server *srv, const uint64_t *ids_host, uint32_t count);

/* Copy a completed request's R output bits (ceil(R/64) words, bits past R
 * written as 0) to out_dev, enqueued on `stream`.  The ring space stays held
 * until qrng_server_release, which must come after the copy has run (the
 * server's later hashes may reuse the space at once). */
qrng_status qrng_server_read(qrng_server *srv, uint64_t request_id, uint64_t *out_dev,
                             void *stream);

/* Device pointer of the output ring (ring_bits / 64 words). */
qrng_status qrng_server_ring(qrng_server *srv, const uint64_t **ring_dev);

/* Device pointer of window slot data for window `window` while it is held
 * (for checking), and the slot's estimate (qrng_me_result, device memory). */
qrng_status qrng_server_window(qrng_server *srv, uint64_t window, const uint8_t **samples_dev,
                               const qrng_me_result **estimate_dev);

qrng_status qrng_server_query(qrng_server *srv, qrng_server_stats *stats);

/* Waits for the server's work, then frees it.  NULL is a no-op. */
void qrng_server_destroy(qrng_server *srv);

/* Measurement aid.  While enabled, every kernel the context launches is
 * bracketed by HIP events recorded on the stream it runs on (a few
 * microseconds of host overhead per launch; results are unchanged). */
qrng_status qrng_profile_enable(qrng_ctx *ctx, int on);

/* Name of kernel class `kernel_id` (0, 1, ...), NULL past the last class. */
const char *qrng_profile_kernel_name(int kernel_id);

/* Launch count and summed device time (ms) of one kernel class since the
 * last reset.  Waits for the recorded events. */
qrng_status qrng_profile_query(qrng_ctx *ctx, int kernel_id, uint64_t *launches,
                               double *total_ms);

/* Forget the recorded launches (waits for them first). */
qrng_status qrng_profile_reset(qrng_ctx *ctx);

/* Issue cost of single VALU instructions on this device, for the ALU
 * rooflines: cycles_out[i], i < min(n, QRNG_PROBE_OPS), receives the
 * shader-clock cycles one SIMD spends per wave64 instruction of op i (named
 * by qrng_profile_issue_op_name), measured with a kernel of independent
 * chains that keeps eight waves on every SIMD, timed with HIP events and
 * converted at clock_ghz (the device's peak shader clock, 2.4 on MI355X).
 * 4.0 is the nominal rate of a 16-lane SIMD.  Synchronous on `stream`;
 * allocates a small device buffer for the duration of the call. */
#define QRNG_PROBE_OPS 8
qrng_status qrng_profile_issue_rates(qrng_ctx *ctx, double clock_ghz, double *cycles_out,
                                     int n, void *stream);
const char *qrng_profile_issue_op_name(int op);

#ifdef __cplusplus
}
#endif

#endif /* QRNG_H */

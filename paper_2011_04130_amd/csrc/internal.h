// Internal interfaces between the C-ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qrng.h"

namespace qrng {

// ------------------------------------------------------- kernel timing hooks
// Every launch site brackets its kernel with prof_begin/prof_end.  They are
// no-ops unless the calling thread's context has timing enabled, in which
// case HIP events are recorded on the launch stream.
enum KernelId {
  KID_COLS_FWD = 0,   // four-step pass A (raw block or seed window columns)
  KID_ROWS_HASH,      // pass B: row transforms, seed product, inverse rows
  KID_ROWS_SEED,      // pass B for a seed window (forward only)
  KID_COLS_INV,       // pass C: inverse columns and bit packing
  KID_FUSED_HASH,     // whole transform in one kernel (Nc <= 2^15)
  KID_FUSED_SEED,
  KID_DIRECT,         // bit-packed direct product
  KID_DIRECT_PREP,    // output clear and raw-block reversal
  KID_HIST,           // sample histogram
  KID_MFMA,           // matrix-core product (fp4 operands)
  KID_MOD_TAIL,       // identity block of the modified Toeplitz hash
  KID_FFT64,          // the paper's float64 method (all its launches)
  KID_COUNT
};
const char* kernel_name(int kid);
void prof_begin(int kid, hipStream_t s);
void prof_end(int kid, hipStream_t s);

// Min-entropy finish on the device: model, H_min, d_U, Delta H_m, H_modify
// from the counts, and m = n H/N - 2 log2(1/eps) (whole bits per sample,
// clamped to [0, m_cap]).  `out` is a qrng_me_result (nullable), m_out a
// uint64 (nullable).
struct MeDevArgs {
  int N, model, u_mode;
  double mu, sigma;
  uint64_t n;
  double log2_inv_eps;
  uint64_t m_cap;
  void* out;
  uint64_t* m_out;
};

// ---------------------------------------------------------------- NTT path
// Per-sub-length twiddle tables (w, floor(w 2^32/p)) and the two-level
// Montgomery table of the 2^23-rd root used by the four-step twiddles.
struct TwTables {
  const uint2* fwd;    // entry (b, a) of a sub-length table at b * r + a
  const uint2* inv;
  const uint2* fwd_t;  // the same tables transposed: entry (b, a) at a * s + b
  const uint2* inv_t;
  const uint32_t* g_lo;  // 4096 entries: w^j 2^32 mod p
  const uint32_t* g_hi;  // 2048 entries: w^(4096 j) 2^32 mod p
};

// Host-built table contents (sizes in entries; fwd and inv hold
// 2 tw_total_entries(): the tables, then their transposed copies).
int tw_total_entries();
void build_tw_tables(uint2* fwd, uint2* inv, uint32_t* g_lo, uint32_t* g_hi);

// Shape of the exact convolution for an m x n hash.
struct NttPlan {
  int log_nc;       // transform length Nc = 2^log_nc
  int log1, log2;   // Nc = N1 * N2 (N1 = 1: one fused kernel)
  int nx, ny;       // raw-block chunks and output chunks
  int64_t bx, by;   // chunk lengths
  int nwin;         // seed windows = nx + ny - 1
};
bool ntt_make_plan(uint64_t n, uint64_t m, NttPlan* plan);
// The plan of one transform of length 2^log_nc (10 <= log_nc <= 23).
bool ntt_plan_for_length(int log_nc, NttPlan* plan);

// One block of an uneven batch whose blocks share a transform length
// (n+m-1 <= Nc <= 2^23 for each).  Raw bits at x_pool + x_bit, output at
// y_pool + y_bit (both multiples of 64), seed spectrum W (Nc words, from
// ntt_seed_spectra with one transform, Nc and the block's seed).
struct NttItem {
  uint64_t x_bit, y_bit;
  const uint32_t* W;
  uint32_t n, m;  // m: output bits planned (words up to m are written)
  uint32_t blk;   // index into the valid-length array m_arr
  uint32_t pad;
};
// workspace (uint32 entries) for seed windows and for one hash of `batch` blocks
uint64_t ntt_seed_elems(const NttPlan& p);
uint64_t ntt_work_elems(const NttPlan& p, int batch);

// Transform-domain seed: nwin arrays of Nc words (Montgomery form, 1/Nc folded).
// With one transform (nx = ny = 1) the spectrum is that of the seed's first
// Nc bits (seed_avail bits exist; the rest read as 0) and depends on the seed
// and Nc only; above 2^23 it depends on (n, m).  With two raw and two output
// chunks the three windows are stored as (W1, W0 - W1, W2 - W1).
hipError_t ntt_seed_spectra(const NttPlan& p, const uint32_t* seed_bits, uint64_t n,
                            uint64_t m, uint64_t seed_avail, uint32_t* W, uint32_t* work,
                            const TwTables& tw, hipStream_t s);
// Hash `batch` equal blocks: block z reads raw bits from x_bits + z*x_stride_bits
// and writes y_bits + z*y_stride_bits (both strides multiples of 64).
// m_dev (nullable): the valid output length computed on the device (<= m,
// which sizes the plan); output bits from it up to m are written as 0.
// `count` uneven blocks of one transform length: items is device memory;
// m_arr (nullable) holds valid output lengths (<= each item's m) by blk.
// Workspace: ntt_work_elems(p, count).
hipError_t ntt_hash_items(const NttPlan& p, const uint32_t* x_pool, const NttItem* items,
                          int count, uint32_t* y_pool, const uint64_t* m_arr, uint32_t* work,
                          const TwTables& tw, hipStream_t s);
// The min-entropy estimate of one block's 8-bit samples run inside the
// hash's first transform pass (extra workgroups; the estimate's m_out is the
// hash's m_dev).  scratch: hist_scratch_words() words, zero on first use and
// left zero by every call.
struct EstJob {
  const uint8_t* samples;
  uint64_t S;
  uint32_t* scratch;
  MeDevArgs me;
  uint32_t epoch;  // tag of this call (below 2^23; consecutive calls differ)
  uint32_t expect_xor;  // nonzero only in fault tests: the finish expects another tag
};
hipError_t ntt_hash(const NttPlan& p, const uint32_t* x_bits, uint64_t n, uint64_t m,
                    const uint32_t* W, uint32_t* y_bits, uint32_t* work, int batch,
                    uint64_t x_stride_bits, uint64_t y_stride_bits, const TwTables& tw,
                    hipStream_t s, const uint64_t* m_dev = nullptr,
                    const EstJob* est = nullptr);
// whether ntt_hash with this plan takes an EstJob (one block, split transform
// with columns of at least 2^7)
bool ntt_fuses_estimate(const NttPlan& p);

// ------------------------------------------- device-scheduled batches
// Registered seeds as the device sees them: entry `id` of a table of
// SEED_TABLE_CAP entries (ids 1 .. SEED_TABLE_CAP-1).  W[k] is the cached
// one-transform spectrum of length 2^k (BATCH_MIN_LOG <= k <= the seed's
// class), L == 0 marks a free id.
constexpr int SEED_TABLE_CAP = 4096;
constexpr int BATCH_MIN_LOG = 10, BATCH_MAX_LOG = 23;
constexpr int BATCH_CLASSES = BATCH_MAX_LOG - BATCH_MIN_LOG + 1;
constexpr int BATCH_REJECTED = BATCH_CLASSES;  // counts[] slot of skipped descriptors
constexpr int BATCH_COUNTS = 16;
struct DevSeed {
  uint64_t L;
  const uint32_t* W[BATCH_MAX_LOG + 1];
};
// Sorts nblocks descriptors (device memory) into per-class item lists
// (list k - BATCH_MIN_LOG holds cap items at items + (k - BATCH_MIN_LOG) cap)
// with their counts, after clearing the counts; descriptors that fail a check
// are counted in counts[BATCH_REJECTED] and skipped, as are blocks longer
// than 2^max_log (no class launch covers them).  seed_ids (nullable):
// block b's seed id, replacing blocks[b].seed_id.
hipError_t batch_classify(const qrng_block* blocks, uint32_t nblocks, const uint32_t* seed_ids,
                          const DevSeed* table, NttItem* items, uint32_t cap, int max_log,
                          uint32_t* counts, hipStream_t s);
// Items [item0, item0 + grid_items) of one transform-length class whose
// count is read on the device (items past it do nothing).  Workspace:
// ntt_work_elems(p, grid_items).
hipError_t ntt_hash_items_dev(const NttPlan& p, const uint32_t* x_pool, const NttItem* items,
                              const uint32_t* count, uint32_t item0, int grid_items,
                              uint32_t* y_pool, uint32_t* work, const TwTables& tw,
                              hipStream_t s);

// ------------------------------------- persistent multi-class passes (plans)
// An uneven batch whose blocks span several transform lengths, hashed by
// three persistent launches (one per four-step pass) instead of three per
// class.  Classes keep ntt_make_plan's split (rows of 2^10 .. 2^12 points),
// whose order the cached seed spectra follow.  A launch's workgroups pull
// work units from an atomic counter: pass A (512 threads): column tiles (32
// columns of one item); pass B (256 threads): the blocks' estimates (one unit
// each), then 2 or 4 rows of one item; pass C (512 threads): column tiles.  Classes are stored longest first, so the largest units are handed
// out first.  Each pass's unit-0 workgroup zeroes the counter of the pass
// before it (the counters start at 0), so the three launches can be replayed
// as a graph with no other node.
constexpr int MC_MAX = 16;
constexpr int MC_MIN_LOG = 16, MC_MAX_LOG = 21;  // transform lengths these launches cover
struct MeBatchArgs;
struct McInfo {
  uint32_t nclass;
  uint32_t units[3];  // units of passes A, B, C (B: nest estimate units first)
  uint32_t nest;
  uint32_t* counters;  // 3 unit counters (device, zero before the first launch)
};
// Bytes of the device argument block for the classes below.
uint64_t mc_args_bytes();
// Builds the host image of the argument block (copied to dev_args by the
// caller): class c has log_nc[c], items[c] items at items_dev[c] and
// workspace work[c] (items[c] << log_nc[c] words); m_arr: valid lengths by
// blk (nullable); est (nullable): the per-block estimates of pass B.
bool mc_build(void* host_image, McInfo* info, int nclass, const int* log_nc,
              const uint32_t* items, const NttItem* const* items_dev, uint32_t* const* work,
              const uint32_t* x_pool, uint32_t* y_pool, const uint64_t* m_arr,
              const MeBatchArgs* est, uint32_t nest, uint32_t* counters);
// One launch of pass `pass` (0, 1, 2) with `grid` workgroups.
hipError_t mc_launch(int pass, const void* dev_args, const McInfo& info, uint32_t grid,
                     const TwTables& tw, hipStream_t s);
// Workgroups of pass `pass` that fit the device at once.
uint32_t mc_grid(int pass, int num_cus);

// ------------------------------------------------------------- direct path
// `batch` blocks sharing one seed: block z reads x_bits + z*x_stride_bits and
// writes y_bits + z*y_stride_bits (strides multiples of 64).
uint64_t direct_work_words(uint64_t n, int batch);
hipError_t direct_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits,
                       uint64_t m, uint32_t* y_bits, uint32_t* work, int num_cus,
                       hipStream_t s, int batch, uint64_t x_stride_bits,
                       uint64_t y_stride_bits, const uint64_t* m_dev = nullptr);

// ------------------------------------------------- modified Toeplitz tail
// y (ceil(m/64) words) ^= raw bits off .. off+m-1 of x (n bits), or = them
// with `assign`; bits from m on are written as 0.
hipError_t xor_tail_bits(const uint64_t* x, uint64_t n, uint64_t off, uint64_t m, uint64_t* y,
                         bool assign, hipStream_t s);

// ------------------------------------------------- float64 FFT (comparison)
// The paper's circulant method in float64 at the power-of-two length
// fft64_length(n, m) >= n+m-1 (at most FFT64_MAX_LENGTH); workspace
// fft64_work_words uint32 words (two complex arrays); err (nullable, device)
// receives the largest distance of a kept value from its integer, as the
// bits of a double.
constexpr uint64_t FFT64_MAX_LENGTH = 1ull << 26;
uint64_t fft64_length(uint64_t n, uint64_t m);
uint64_t fft64_work_words(uint64_t n, uint64_t m);
hipError_t fft64_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits, uint64_t m,
                      uint64_t* y, unsigned long long* err, uint32_t* work, hipStream_t s);

// -------------------------------------------------------------- MFMA path
// `batch` blocks sharing one seed as one matrix-core product (strides as in
// ntt_hash).  No workspace.
hipError_t mfma_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits, uint64_t m,
                     uint32_t* y_bits, int batch, uint64_t x_stride_bits,
                     uint64_t y_stride_bits, hipStream_t s, const uint64_t* m_dev = nullptr);

// ------------------------------------------------------- histogram, estimate
constexpr int HIST_MAX_GROUPS = 256;
// uint32 words of the scratch (partial histograms and a ticket) one
// hist_estimate call or fused estimate uses; calls that share it must be
// ordered on one stream.
uint64_t hist_scratch_words();
// Two launches: histogram of S samples of N bits (N <= 8); counts_out
// (nullable, device) receives the 2^N counts, then the number of samples
// >= 2^N, then 1 if the partial counts passed the finish's consistency check
// (0: the estimate failed closed, m = 0); with `finish` the estimate and m
// are written on the device.  S < 2^40.  keep_thr > 0: only the samples the
// seeded generator keeps count (hist_dev.h, subset_keep).  epoch: tag of the
// call (below 2^23), written into and checked on every partial row.
hipError_t hist_estimate(const uint8_t* samples, uint64_t S, int N, uint32_t* scratch,
                         unsigned long long* counts_out, const MeDevArgs* finish,
                         hipStream_t s, uint64_t subset_seed = 0, uint32_t keep_thr = 0,
                         uint32_t epoch = 0, uint32_t expect_xor = 0);
// word of the fused estimate's ticket in the histogram scratch
uint64_t hist_ticket_word();

// Per-block estimates of an uneven batch of 8-bit sample blocks (one
// workgroup each): block b's histogram, estimate (out[b], nullable) and
// output length m_out[b] = min(m_cap, n H/8 - ceil(2 log2(1/eps))).
struct MeBlock {
  uint64_t byte_off;  // first sample (multiple of 8)
  uint32_t S;         // samples (multiple of 8)
  uint32_t pad;
  uint64_t n;         // raw bits the output length refers to (8 S)
  uint64_t m_cap;
};
struct MeBatchArgs {
  const uint8_t* pool;
  const MeBlock* blocks;  // device memory
  int model, u_mode;
  double mu, sigma;
  double log2_inv_eps;
  qrng_me_result* out;
  uint64_t* m_out;
};
hipError_t minentropy_blocks(const MeBatchArgs& a, int nblocks, hipStream_t s);

// ------------------------------------------------- issue-cost probe
constexpr int PROBE_OPS = 8;
const char* probe_op_name(int op);
// words of the probe's output buffer for a device of num_cus CUs
uint64_t probe_out_words(int num_cus);
// Cycles per wave64 instruction per SIMD of probe op `op` at clock_ghz
// (synchronous on s; out: probe_out_words words of device memory).
hipError_t probe_issue_cycles(int op, int num_cus, double clock_ghz, uint32_t* out,
                              hipStream_t s, double* cycles);

// ------------------------------------------------- context services
// (for the serving loop, which is built on the C ABI)
int ctx_num_cus(const qrng_ctx* c);
int ctx_device(const qrng_ctx* c);
// delta = +1 / -1 pins / unpins a registered seed (pinned seeds cannot be
// unregistered), 0 only looks it up; *L (nullable) receives its length.
// false if the id is unknown.
bool ctx_pin_seed(qrng_ctx* c, uint32_t seed_id, int delta, uint64_t* L);
// Servers are destroyed with their context.
void ctx_track_server(qrng_ctx* c, qrng_server* s, bool add);
// Records the last error text (returns st).
qrng_status set_error(qrng_status st, const char* fmt, ...);
// Validates estimator options (model, U mode, reserved field, parameters).
qrng_status check_me_opts(const qrng_me_opts& o);

}  // namespace qrng

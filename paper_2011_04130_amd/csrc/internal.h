// Internal interfaces between the C-ABI layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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
  KID_FUSED_HASH,     // whole transform in one kernel (Nc <= 2^14)
  KID_FUSED_SEED,
  KID_DIRECT,         // bit-packed direct product
  KID_DIRECT_PREP,    // output clear and raw-block reversal
  KID_HIST,           // sample histogram
  KID_MFMA,           // int8 matrix-core product
  KID_COUNT
};
const char* kernel_name(int kid);
void prof_begin(int kid, hipStream_t s);
void prof_end(int kid, hipStream_t s);

// ---------------------------------------------------------------- NTT path
// Per-sub-length twiddle tables (w, floor(w 2^32/p)) and the two-level
// Montgomery table of the 2^23-rd root used by the four-step twiddles.
struct TwTables {
  const uint2* fwd;
  const uint2* inv;
  const uint32_t* g_lo;  // 4096 entries: w^j 2^32 mod p
  const uint32_t* g_hi;  // 2048 entries: w^(4096 j) 2^32 mod p
};

// Host-built table contents (sizes in entries).
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
// workspace (uint32 entries) for seed windows and for one hash of `batch` blocks
uint64_t ntt_seed_elems(const NttPlan& p);
uint64_t ntt_work_elems(const NttPlan& p, int batch);

// Transform-domain seed: nwin arrays of Nc words (Montgomery form, 1/Nc folded).
hipError_t ntt_seed_spectra(const NttPlan& p, const uint32_t* seed_bits, uint64_t n,
                            uint64_t m, uint32_t* W, uint32_t* work,
                            const TwTables& tw, hipStream_t s);
// Hash `batch` equal blocks: block z reads raw bits from x_bits + z*x_stride_bits
// and writes y_bits + z*y_stride_bits (both strides multiples of 64).
// m_dev (nullable): the valid output length computed on the device (<= m,
// which sizes the plan); output bits from it up to m are written as 0.
hipError_t ntt_hash(const NttPlan& p, const uint32_t* x_bits, uint64_t n, uint64_t m,
                    const uint32_t* W, uint32_t* y_bits, uint32_t* work, int batch,
                    uint64_t x_stride_bits, uint64_t y_stride_bits, const TwTables& tw,
                    hipStream_t s, const uint64_t* m_dev = nullptr);

// ------------------------------------------------------------- direct path
// `batch` blocks sharing one seed: block z reads x_bits + z*x_stride_bits and
// writes y_bits + z*y_stride_bits (strides multiples of 64).
uint64_t direct_work_words(uint64_t n, int batch);
hipError_t direct_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits,
                       uint64_t m, uint32_t* y_bits, uint32_t* work, int num_cus,
                       hipStream_t s, int batch, uint64_t x_stride_bits,
                       uint64_t y_stride_bits, const uint64_t* m_dev = nullptr);

// -------------------------------------------------------------- MFMA path
// `batch` blocks sharing one seed as one int8 matrix product (strides as in
// ntt_hash).  No workspace.
hipError_t mfma_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits, uint64_t m,
                     uint32_t* y_bits, int batch, uint64_t x_stride_bits,
                     uint64_t y_stride_bits, hipStream_t s, const uint64_t* m_dev = nullptr);

// ------------------------------------------------------------- histogram
hipError_t histogram_u8(const uint8_t* samples, uint64_t S, int nbins,
                        unsigned long long* counts /* nbins + 1 */, int num_cus,
                        hipStream_t s);

// Min-entropy finish on the device (one workgroup): model, H_min, d_U,
// Delta H_m, H_modify from the counts, and m = n H/N - 2 log2(1/eps)
// (whole bits per sample, clamped to [0, m_cap]).  `out` is a qrng_me_result.
struct MeDevArgs {
  const unsigned long long* counts;
  int N, model, u_mode;
  double mu, sigma;
  uint64_t n;
  double log2_inv_eps;
  uint64_t m_cap;
  void* out;
  uint64_t* m_out;
};
hipError_t minentropy_device(const MeDevArgs& a, hipStream_t s);

}  // namespace qrng

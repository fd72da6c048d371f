// Toeplitz hashing of many equal blocks that share one seed on the int8
// matrix cores (paper Sec. III.B, the direct product k = T r; here for a
// whole batch at once, so it becomes a true matrix-matrix product).
//
// With B blocks as the columns of X (n x B, raw bits as int8 0/1) and
// A[i][j] = s[n-1+i-j] (the m x n Toeplitz matrix as int8), Y = A X holds
// in column b the integer row sums of block b; each is at most n, so int32
// accumulation is exact and the hash bit is Y & 1.
//
// Tiling (gfx950, v_mfma_i32_32x32x32_i8, wave64): a workgroup owns 128
// output rows x 128 blocks; wave w owns rows 32w..32w+31 and all 128 blocks
// (four 32x32 accumulators).  Per K-chunk of 128 raw bits the workgroup
// expands the 128 blocks' bits to bytes in LDS once (shared by the four
// waves); each wave builds its A fragments in registers straight from the
// seed bits (16 consecutive seed bits, reversed, expanded to 16 bytes), then
// issues 4 MFMAs per 32-bit K-step.  Fragment layout: lane l holds row or
// column l % 32 and 16 k-values of lane group l / 32 (the same k order on A
// and B, so the contraction over k is exact whatever the hardware's order).
#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int MT = 128;       // rows per workgroup
constexpr int NT = 128;       // blocks per workgroup
constexpr int KC = 128;       // raw bits per LDS fill
constexpr int BROW = KC + 16; // padded LDS row (bytes) of one block's expanded bits

// 4 bits -> 4 bytes holding 0/1 (bit t to the low bit of byte t)
__device__ __forceinline__ uint32_t expand4(uint32_t nib) {
  return (nib * 0x00204081u) & 0x01010101u;
}
// 16 bits -> 16 bytes
__device__ __forceinline__ v4i expand16(uint32_t w) {
  v4i r;
  r.x = (int)expand4(w & 15u);
  r.y = (int)expand4((w >> 4) & 15u);
  r.z = (int)expand4((w >> 8) & 15u);
  r.w = (int)expand4((w >> 12) & 15u);
  return r;
}

// 32 bits of a bit string starting at bit p (may be negative or run past
// nbits: those bits read as 0).
__device__ __forceinline__ uint32_t bits32_at(const uint32_t* __restrict__ s, int64_t p,
                                              int64_t nbits) {
  const int64_t w = p >> 5;  // floor division
  const uint32_t sh = (uint32_t)(p & 31);
  const int64_t nw = (nbits + 31) >> 5;
  const uint32_t lo = (w >= 0 && w < nw) ? s[w] : 0u;
  const uint32_t hi = (w + 1 >= 0 && w + 1 < nw) ? s[w + 1] : 0u;
  uint32_t v = sh ? ((lo >> sh) | (hi << (32u - sh))) : lo;
  // clear bits at or past nbits, and below 0
  const int64_t top = nbits - p;  // valid bits from p
  if (top < 32) v &= top <= 0 ? 0u : ((1u << (uint32_t)top) - 1u);
  if (p < 0) v &= (p <= -32) ? 0u : ~((1u << (uint32_t)(-p)) - 1u);
  return v;
}

struct MfmaArgs {
  const uint32_t* x;  // raw bits; block b at bit b * x_zs
  uint64_t x_zs;
  const uint32_t* seed;
  uint64_t n, m, L;
  uint32_t* y;  // output bits; block b at bit b * y_zs (multiple of 64)
  uint64_t y_zs;
  uint32_t nblocks;
  const uint64_t* m_dev;  // nullable: valid rows computed on the device
};

__global__ __launch_bounds__(256) void k_mfma(MfmaArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t bt[NT * BROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * MT + wave * 32;  // this wave's first row
  const uint32_t b0 = blockIdx.y * NT;
  const int64_t n = (int64_t)a.n;
  uint64_t mv = a.m;
  if (a.m_dev && *a.m_dev < mv) mv = *a.m_dev;

  v16i acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0;

  // fill roles: thread -> (block bl, half hf of the K-chunk)
  const int bl = tid >> 1, hf = tid & 1;
  const uint32_t bfill = b0 + bl;
  const int64_t arow = i0 + (lane & 31);  // A row of this lane
  const int kg = 16 * (lane >> 5);        // lane group's k offset in a K-step

  for (int64_t k0 = 0; k0 < n; k0 += KC) {
    // expand 64 raw bits of block bfill (k0 + 64 hf ...) to bytes in LDS
    {
      uint32_t w0 = 0, w1 = 0;
      if (bfill < a.nblocks) {
        const int64_t base = (int64_t)bfill * (int64_t)a.x_zs;
        const int64_t kk = k0 + 64 * hf;
        w0 = bits32_at(a.x, base + kk, base + n);
        w1 = bits32_at(a.x, base + kk + 32, base + n);
      }
      uint8_t* dst = bt + bl * BROW + 64 * hf;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint32_t w = q ? w1 : w0;
        v4i e0 = expand16(w & 0xFFFFu), e1 = expand16(w >> 16);
        *reinterpret_cast<v4i*>(dst + 32 * q) = e0;
        *reinterpret_cast<v4i*>(dst + 32 * q + 16) = e1;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / 32; ++ks) {
      // A fragment: row arow, k = k0 + 32 ks + kg + q (q < 16) needs seed bit
      // n-1+arow-k, i.e. the 16 bits ending at n-1+arow-(k0+32ks+kg), reversed
      const int64_t phi = n - 1 + arow - (k0 + 32 * ks + kg);
      const uint32_t w16 = bits32_at(a.seed, phi - 15, (int64_t)a.L) & 0xFFFFu;
      const v4i af = expand16(__builtin_bitreverse32(w16) >> 16);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const v4i bf =
            *reinterpret_cast<const v4i*>(bt + (32 * t + (lane & 31)) * BROW + 32 * ks + kg);
        acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af, bf, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // D layout: lane l holds column l % 32 (a block) and rows
  // 8 (r / 4) + 4 (l / 32) + r % 4 of its accumulator, r < 16
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    uint32_t w = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      w |= ((uint32_t)acc[t][r] & 1u) << row;
    }
    w |= __shfl_xor(w, 32);
    const uint32_t b = b0 + 32 * t + (lane & 31);
    if (lane < 32 && b < a.nblocks && i0 < (int64_t)a.m) {
      // rows past the valid length are 0
      const int64_t valid = (int64_t)mv - i0;
      if (valid < 32) w &= valid <= 0 ? 0u : ((1u << (uint32_t)valid) - 1u);
      a.y[((uint64_t)b * a.y_zs + (uint64_t)i0) >> 5] = w;
    }
  }
}

// zero the 32-bit word after the last written one where ceil(m/32) is odd,
// so each block's last 64-bit word has no stale high half
__global__ __launch_bounds__(256) void k_tail(uint32_t* __restrict__ y, uint64_t y_zs,
                                              uint64_t m, uint32_t nblocks) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b < nblocks) y[((uint64_t)b * y_zs >> 5) + (m + 31) / 32] = 0u;
}

}  // namespace

hipError_t mfma_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits, uint64_t m,
                     uint32_t* y_bits, int batch, uint64_t x_stride_bits,
                     uint64_t y_stride_bits, hipStream_t s, const uint64_t* m_dev) {
  MfmaArgs a{};
  a.x = x_bits;
  a.x_zs = x_stride_bits;
  a.seed = seed_bits;
  a.n = n;
  a.m = m;
  a.L = n + m - 1;
  a.y = y_bits;
  a.y_zs = y_stride_bits;
  a.nblocks = (uint32_t)batch;
  a.m_dev = m_dev;
  const dim3 grid((unsigned)((m + MT - 1) / MT), (unsigned)((batch + NT - 1) / NT));
  prof_begin(KID_MFMA, s);
  hipLaunchKernelGGL(k_mfma, grid, dim3(256), 0, s, a);
  if (((m + 31) / 32) & 1)
    hipLaunchKernelGGL(k_tail, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, y_bits,
                       y_stride_bits, m, (uint32_t)batch);
  prof_end(KID_MFMA, s);
  return hipGetLastError();
}

}  // namespace qrng

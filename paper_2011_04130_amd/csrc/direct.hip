// Direct Toeplitz hash over GF(2), O(m n) bit operations (paper Sec. III.B,
// the matrix product k = T r before any acceleration).
//
// Reindexing j' = n-1-j turns row i into a Hankel row:
//     y[i] = XOR_{j'} s[i + j'] AND xr[j'],   xr = x bit-reversed,
// so 32 consecutive rows i0..i0+31 read the same seed words and differ only
// in how xr is aligned against them.  For seed word u (bits 32u..32u+31 after
// i0) the bits of xr that meet it in row i0 + r form the 32-bit funnel shift
//     M(u, r) = (Xr[u] << r) | (Xr[u-1] >> (32 - r)),
// which is the same for every lane of a wave.  Each thread owns 32 rows and
// keeps 32 accumulators; per seed word it issues one vector load and 32
// three-input bit ops acc_r ^= S[u] & M(u, r) (one v_bitop3_b32 each on
// gfx950: 32 GF(2) multiply-adds per VALU op), while the masks come from
// 64-bit scalar shifts on the scalar unit.  The row parity is popcount & 1.
// Columns are split across workgroups; partial parities of a row are
// combined with 32-bit atomic XOR, which is order-independent, so the result
// is deterministic.
#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

// Xr[u], u < W = ceil(n/32): bit b is x[n-1-32u-b] (0 below bit 0).
// blockIdx.x = z * nb + (u / 256) for batch item z.
__global__ __launch_bounds__(256) void k_reverse(const uint32_t* __restrict__ x, uint64_t n,
                                                 uint64_t x_zs32, uint32_t* __restrict__ xr,
                                                 uint64_t W, uint32_t nb) {
  const uint64_t z = blockIdx.x / nb;
  const uint64_t u = (uint64_t)(blockIdx.x % nb) * 256 + threadIdx.x;
  if (u >= W) return;
  const uint32_t* __restrict__ xz = x + z * x_zs32;
  const int64_t lo = (int64_t)n - 32 * (int64_t)(u + 1);  // source of bit 31
  uint32_t w;
  if (lo >= 0) {
    const uint64_t q = (uint64_t)lo >> 5;
    const uint32_t sh = (uint32_t)lo & 31u;
    w = xz[q] >> sh;
    if (sh) w |= xz[q + 1] << (32u - sh);
  } else {
    w = xz[0] << (uint32_t)(-lo);
  }
  xr[z * W + u] = __builtin_bitreverse32(w);
}

// zero nw words of each batch item (item z at p + z * zs)
__global__ __launch_bounds__(256) void k_zero(uint32_t* __restrict__ p, uint64_t nw,
                                              uint64_t zs, uint32_t nb) {
  const uint64_t z = blockIdx.x / nb;
  const uint64_t i = (uint64_t)(blockIdx.x % nb) * 256 + threadIdx.x;
  if (i < nw) p[z * zs + i] = 0u;
}

constexpr int UNR = 8;

// One wave per workgroup.  Thread = row group i0 = 32 * (rb * 64 + lane) of
// batch item z (blockIdx.x = z * nrb + rb); blockIdx.y = column chunk
// [u0, u1) of the W+1 seed-word offsets.
__global__ __launch_bounds__(64) void k_direct(const uint32_t* __restrict__ S, uint64_t nsw,
                                               const uint32_t* __restrict__ Xr_all, uint64_t W,
                                               uint64_t m, uint64_t uchunk,
                                               uint32_t* __restrict__ y_all, uint64_t y_zs32,
                                               uint32_t nrb, const uint64_t* __restrict__ m_dev) {
  const uint64_t z = blockIdx.x / nrb;
  if (m_dev && *m_dev < m) m = *m_dev;  // valid rows computed on the device
  const uint64_t G = (m + 31) / 32;
  const uint64_t grp = (uint64_t)(blockIdx.x % nrb) * 64 + threadIdx.x;
  const uint32_t* __restrict__ Xr = Xr_all + z * W;
  uint32_t* __restrict__ y = y_all + z * y_zs32;
  const uint64_t u0 = (uint64_t)blockIdx.y * uchunk;
  const uint64_t uend = u0 + uchunk < W + 1 ? u0 + uchunk : W + 1;
  uint32_t acc[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) acc[r] = 0u;
  uint32_t xprev = u0 ? Xr[u0 - 1] : 0u;
  uint64_t u = u0;
  // UNR seed words at a time; loop bounds are uniform, the seed index is
  // clamped per lane
  for (; u + UNR <= uend; u += UNR) {
    uint32_t xv[UNR], sv[UNR];
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      xv[t] = (u + t < W) ? Xr[u + t] : 0u;
      const uint64_t si = grp + u + t;
      sv[t] = si < nsw ? S[si] : 0u;
    }
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const uint64_t pair = ((uint64_t)xv[t] << 32) | xprev;
#pragma unroll
      for (int r = 0; r < 32; ++r) acc[r] ^= sv[t] & (uint32_t)(pair >> (32 - r));
      xprev = xv[t];
    }
  }
  for (; u < uend; ++u) {
    const uint32_t xc = u < W ? Xr[u] : 0u;
    const uint64_t si = grp + u;
    const uint32_t sw = si < nsw ? S[si] : 0u;
    const uint64_t pair = ((uint64_t)xc << 32) | xprev;
#pragma unroll
    for (int r = 0; r < 32; ++r) acc[r] ^= sw & (uint32_t)(pair >> (32 - r));
    xprev = xc;
  }
  if (grp < G) {
    uint32_t o = 0;
#pragma unroll
    for (int r = 0; r < 32; ++r) o |= ((uint32_t)__popc(acc[r]) & 1u) << r;
    if (grp == G - 1 && (m & 31)) o &= (1u << (m & 31)) - 1u;
    if (o) atomicXor(&y[grp], o);
  }
}

}  // namespace

uint64_t direct_work_words(uint64_t n, int batch) { return (uint64_t)batch * ((n + 31) / 32); }

hipError_t direct_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits,
                       uint64_t m, uint32_t* y_bits, uint32_t* work, int num_cus,
                       hipStream_t s, int batch, uint64_t x_stride_bits,
                       uint64_t y_stride_bits, const uint64_t* m_dev) {
  const uint64_t W = (n + 31) / 32;
  const uint64_t L = n + m - 1;
  const uint64_t nsw = (L + 31) / 32;  // seed words holding bits < L
  const uint64_t ywords = 2 * ((m + 63) / 64);
  const uint32_t nbz = (uint32_t)((ywords + 255) / 256);
  prof_begin(KID_DIRECT_PREP, s);
  hipLaunchKernelGGL(k_zero, dim3(nbz * (uint32_t)batch), dim3(256), 0, s, y_bits, ywords,
                     y_stride_bits / 32, nbz);
  const uint32_t nbr = (uint32_t)((W + 255) / 256);
  hipLaunchKernelGGL(k_reverse, dim3(nbr * (uint32_t)batch), dim3(256), 0, s, x_bits, n,
                     x_stride_bits / 32, work, W, nbr);
  prof_end(KID_DIRECT_PREP, s);
  const uint64_t G = (m + 31) / 32;
  const uint32_t nrb = (uint32_t)((G + 63) / 64);
  // split the W+1 seed-word offsets so that the launch holds enough waves
  const uint64_t want_waves = (uint64_t)num_cus * 16;
  const uint64_t row_waves = (uint64_t)nrb * (uint64_t)batch;
  uint64_t nchunk = (want_waves + row_waves - 1) / row_waves;
  if (nchunk < 1) nchunk = 1;
  if (nchunk > 65535) nchunk = 65535;
  uint64_t uchunk = (W + 1 + nchunk - 1) / nchunk;
  if (uchunk < 64) uchunk = 64;
  nchunk = (W + 1 + uchunk - 1) / uchunk;
  prof_begin(KID_DIRECT, s);
  hipLaunchKernelGGL(k_direct, dim3(nrb * (uint32_t)batch, (uint32_t)nchunk), dim3(64), 0, s,
                     seed_bits, nsw, work, W, m, uchunk, y_bits, y_stride_bits / 32, nrb, m_dev);
  prof_end(KID_DIRECT, s);
  return hipGetLastError();
}

}  // namespace qrng

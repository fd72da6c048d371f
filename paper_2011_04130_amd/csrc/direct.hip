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

constexpr int UNR = 4;
// zero words after each reversed block, so that the product loop reads the
// words past W without bounds checks
constexpr uint64_t XPAD = 2 * UNR + 2;

// Xr[u], u < W = ceil(n/32): bit b is x[n-1-32u-b] (0 below bit 0); 0 for
// W <= u < W + XPAD.  Item z at xr + z (W + XPAD);
// blockIdx.x = z * nb + (u / 256) for batch item z.
__global__ __launch_bounds__(256) void k_reverse(const uint32_t* __restrict__ x, uint64_t n,
                                                 uint64_t x_zs32, uint32_t* __restrict__ xr,
                                                 uint64_t W, uint32_t nb) {
  const uint64_t z = blockIdx.x / nb;
  const uint64_t u = (uint64_t)(blockIdx.x % nb) * 256 + threadIdx.x;
  if (u >= W + XPAD) return;
  if (u >= W) {
    xr[z * (W + XPAD) + u] = 0u;
    return;
  }
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
  xr[z * (W + XPAD) + u] = __builtin_bitreverse32(w);
}

// zero nw words of each batch item (item z at p + z * zs)
__global__ __launch_bounds__(256) void k_zero(uint32_t* __restrict__ p, uint64_t nw,
                                              uint64_t zs, uint32_t nb) {
  const uint64_t z = blockIdx.x / nb;
  const uint64_t i = (uint64_t)(blockIdx.x % nb) * 256 + threadIdx.x;
  if (i < nw) p[z * zs + i] = 0u;
}

// Word 3 of a raw buffer resource on gfx9 (32-bit data format); the range
// check against num_records then returns 0 for bytes past the end.
constexpr int kRsrcWord3 = 0x00020000;

// acc ^ (a & b) as one three-input bit op (truth table 0x78 over the
// operands (acc, a, b)); b is wave-uniform and read from a scalar register.
__device__ __forceinline__ uint32_t xor_and(uint32_t acc, uint32_t a, uint32_t b) {
  uint32_t d;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x78" : "=v"(d) : "v"(acc), "v"(a), "s"(b));
  return d;
}

// One wave per workgroup.  Thread = KG row groups i0 = 32 * (rb * 64 KG +
// 64 k + lane), k < KG, of batch item z (blockIdx.x = z * nrb + rb); the KG
// groups share the wave-uniform masks.  blockIdx.y = column chunk [u0, u1)
// of the W+1 seed-word offsets.
template <int KG>
__global__ __launch_bounds__(64) void k_direct(const uint32_t* __restrict__ S, uint64_t nsw,
                                               const uint32_t* __restrict__ Xr_all, uint64_t W,
                                               uint64_t m, uint64_t uchunk,
                                               uint32_t* __restrict__ y_all, uint64_t y_zs32,
                                               uint32_t nrb, const uint64_t* __restrict__ m_dev) {
  const uint64_t z = blockIdx.x / nrb;
  if (m_dev && *m_dev < m) m = *m_dev;  // valid rows computed on the device
  const uint64_t G = (m + 31) / 32;
  const uint64_t grp = (uint64_t)(blockIdx.x % nrb) * 64 * KG + threadIdx.x;
  const uint32_t* __restrict__ Xr = Xr_all + z * (W + XPAD);
  uint32_t* __restrict__ y = y_all + z * y_zs32;
  const uint64_t u0 = (uint64_t)blockIdx.y * uchunk;
  const uint64_t uend = u0 + uchunk < W + 1 ? u0 + uchunk : W + 1;
  uint32_t acc[KG][32];
#pragma unroll
  for (int k = 0; k < KG; ++k)
#pragma unroll
    for (int r = 0; r < 32; ++r) acc[k][r] = 0u;
  uint32_t xprev = u0 ? Xr[u0 - 1] : 0u;
  uint64_t u = u0;
  // UNR seed words at a time, the next UNR words loaded while the current
  // ones are used; loop bounds are uniform.  Reversed-block words up to
  // W + 2 UNR exist (zero padding); seed words are read through a buffer
  // resource of nsw words, whose range check returns 0 past the end.
  const __amdgpu_buffer_rsrc_t srs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(S), 0, (int)(nsw * 4), kRsrcWord3);
  uint32_t xv[UNR], sv[UNR][KG];
  auto load = [&](uint64_t v, uint32_t* xo, uint32_t (*so)[KG]) {
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      xo[t] = Xr[v + t];
#pragma unroll
      for (int k = 0; k < KG; ++k)
        so[t][k] = __builtin_amdgcn_raw_buffer_load_b32(
            srs, (int)((uint32_t)(grp + 64 * k + v + t) * 4u), 0, 0);
    }
  };
  if (u + UNR <= uend) load(u, xv, sv);
  for (; u + UNR <= uend; u += UNR) {
    uint32_t xn[UNR], sn[UNR][KG];
    load(u + UNR, xn, sn);
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const uint64_t pair = ((uint64_t)xv[t] << 32) | xprev;
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        const uint32_t mk = (uint32_t)(pair >> (32 - r));
#pragma unroll
        for (int k = 0; k < KG; ++k) acc[k][r] = xor_and(acc[k][r], sv[t][k], mk);
        // keep each mask next to its uses (hoisting them all spills SGPRs)
        __builtin_amdgcn_sched_barrier(0);
      }
      xprev = xv[t];
    }
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      xv[t] = xn[t];
#pragma unroll
      for (int k = 0; k < KG; ++k) sv[t][k] = sn[t][k];
    }
  }
  for (; u < uend; ++u) {
    const uint32_t xc = Xr[u];
    const uint64_t pair = ((uint64_t)xc << 32) | xprev;
#pragma unroll
    for (int k = 0; k < KG; ++k) {
      const uint64_t si = grp + 64 * k + u;
      const uint32_t sw = si < nsw ? S[si] : 0u;
#pragma unroll
      for (int r = 0; r < 32; ++r) acc[k][r] = xor_and(acc[k][r], sw, (uint32_t)(pair >> (32 - r)));
    }
    xprev = xc;
  }
#pragma unroll
  for (int k = 0; k < KG; ++k) {
    const uint64_t g = grp + 64 * k;
    if (g < G) {
      uint32_t o = 0;
#pragma unroll
      for (int r = 0; r < 32; ++r) o |= ((uint32_t)__popc(acc[k][r]) & 1u) << r;
      if (g == G - 1 && (m & 31)) o &= (1u << (m & 31)) - 1u;
      if (o) atomicXor(&y[g], o);
    }
  }
}

}  // namespace

uint64_t direct_work_words(uint64_t n, int batch) {
  return (uint64_t)batch * ((n + 31) / 32 + XPAD);
}

hipError_t direct_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits,
                       uint64_t m, uint32_t* y_bits, uint32_t* work, int num_cus,
                       hipStream_t s, int batch, uint64_t x_stride_bits,
                       uint64_t y_stride_bits, const uint64_t* m_dev) {
  const uint64_t W = (n + 31) / 32;
  const uint64_t L = n + m - 1;
  const uint64_t nsw = (L + 31) / 32;  // seed words holding bits < L
  if (nsw >= (1ull << 29)) return hipErrorInvalidValue;  // 32-bit buffer offsets
  const uint64_t ywords = 2 * ((m + 63) / 64);
  const uint32_t nbz = (uint32_t)((ywords + 255) / 256);
  prof_begin(KID_DIRECT_PREP, s);
  hipLaunchKernelGGL(k_zero, dim3(nbz * (uint32_t)batch), dim3(256), 0, s, y_bits, ywords,
                     y_stride_bits / 32, nbz);
  const uint32_t nbr = (uint32_t)((W + XPAD + 255) / 256);
  hipLaunchKernelGGL(k_reverse, dim3(nbr * (uint32_t)batch), dim3(256), 0, s, x_bits, n,
                     x_stride_bits / 32, work, W, nbr);
  prof_end(KID_DIRECT_PREP, s);
  const uint64_t G = (m + 31) / 32;
  // split the W+1 seed-word offsets into chunks of at least kMinChunk so
  // that the launch holds enough waves; threads take KG row groups (sharing
  // the scalar masks) when the launch stays full with fewer of them
  constexpr uint64_t kMinChunk = 16;
  const uint64_t want_waves = (uint64_t)num_cus * 16;
  const uint64_t max_chunks = (W + 1 + kMinChunk - 1) / kMinChunk;
  int kg = 2;
  while (kg > 1 && ((G + 64 * kg - 1) / (64 * kg)) * (uint64_t)batch * max_chunks < want_waves)
    kg /= 2;
  const uint32_t nrb = (uint32_t)((G + 64 * kg - 1) / (64 * kg));
  const uint64_t row_waves = (uint64_t)nrb * (uint64_t)batch;
  uint64_t nchunk = (want_waves + row_waves - 1) / row_waves;
  if (nchunk < 1) nchunk = 1;
  if (nchunk > 65535) nchunk = 65535;
  uint64_t uchunk = (W + 1 + nchunk - 1) / nchunk;
  if (uchunk < kMinChunk) uchunk = kMinChunk;
  nchunk = (W + 1 + uchunk - 1) / uchunk;
  prof_begin(KID_DIRECT, s);
  const dim3 grid(nrb * (uint32_t)batch, (uint32_t)nchunk);
  const uint64_t ys = y_stride_bits / 32;
  if (kg == 2)
    hipLaunchKernelGGL(k_direct<2>, grid, dim3(64), 0, s, seed_bits, nsw, work, W, m, uchunk,
                       y_bits, ys, nrb, m_dev);
  else
    hipLaunchKernelGGL(k_direct<1>, grid, dim3(64), 0, s, seed_bits, nsw, work, W, m, uchunk,
                       y_bits, ys, nrb, m_dev);
  prof_end(KID_DIRECT, s);
  return hipGetLastError();
}

}  // namespace qrng

// Modified Toeplitz hash (paper Sec. III.D): k = (A, I_m) r with an (n-1)-bit
// seed.  A is the m x (n-m) Toeplitz block A[i][j] = a[n-m-1+i-j] (0-indexed
// seed bits), i.e. the Sec. III.B matrix of an (n-m)-column block with the
// same seed, so the product runs on the ordinary hash paths over the first
// n-m raw bits; the identity block then adds raw bit n-m+i to key bit i,
// which is this file's one kernel.
#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

// y[w] ^= raw bits off+64w .. off+64w+63 (assign: y[w] = those bits), for the
// ceil(m/64) words of y; bits from m on are 0.  x holds xw words.
__global__ __launch_bounds__(256) void k_xor_tail(const uint64_t* __restrict__ x, uint64_t xw,
                                                  uint64_t off, uint64_t m,
                                                  uint64_t* __restrict__ y, int assign) {
  const uint64_t w = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t nw = (m + 63) / 64;
  if (w >= nw) return;
  const uint64_t q = (off >> 6) + w;
  const uint32_t sh = (uint32_t)(off & 63);
  uint64_t v = q < xw ? x[q] >> sh : 0;
  if (sh && q + 1 < xw) v |= x[q + 1] << (64 - sh);
  if (w == nw - 1 && (m & 63)) v &= (1ull << (m & 63)) - 1;
  y[w] = assign ? v : (y[w] ^ v);
}

}  // namespace

hipError_t xor_tail_bits(const uint64_t* x, uint64_t n, uint64_t off, uint64_t m, uint64_t* y,
                         bool assign, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const uint64_t nw = (m + 63) / 64;
  prof_begin(KID_MOD_TAIL, s);
  hipLaunchKernelGGL(k_xor_tail, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, x,
                     (n + 63) / 64, off, m, y, assign ? 1 : 0);
  prof_end(KID_MOD_TAIL, s);
  return hipGetLastError();
}

}  // namespace qrng

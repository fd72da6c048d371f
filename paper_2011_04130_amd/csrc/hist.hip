// Histogram of N-bit ADC samples (one byte each) for the min-entropy estimate
// (paper Sec. II: P'(x) is the observed frequency of each sample value).
// Each wave counts into its own LDS sub-histogram (fewer same-address
// collisions), the workgroup merges them and adds to 64-bit global counters.
// Values >= nbins are counted in an extra bin so the host can reject them.
#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

constexpr int HB = 257;  // 256 values + out-of-range

__global__ __launch_bounds__(256) void k_hist(const uint8_t* __restrict__ s, uint64_t S,
                                              int nbins, unsigned long long* __restrict__ counts) {
  __shared__ uint32_t h[4][HB];
  const int wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 4 * HB; i += 256) (&h[0][0])[i] = 0u;
  __syncthreads();
  uint32_t* hw = h[wave];
  const uint32_t lim = (uint32_t)nbins;
  // bytes before the first 16-byte boundary and after the last are counted
  // one at a time by workgroup 0
  const uint64_t mis = (uint64_t)(reinterpret_cast<uintptr_t>(s) & 15u);
  const uint64_t head = mis ? (16 - mis < S ? 16 - mis : S) : 0;
  const uint64_t nvec = (S - head) / 16;
  const uint4* s4 = reinterpret_cast<const uint4*>(s + head);
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < nvec;
       i += (uint64_t)gridDim.x * 256) {
    const uint4 v = s4[i];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t x = (w[k] >> (8 * b)) & 255u;
        atomicAdd(&hw[x < lim ? x : 256u], 1u);
      }
  }
  if (blockIdx.x == 0) {
    for (uint64_t i = threadIdx.x; i < head; i += 256) {
      const uint32_t x = s[i];
      atomicAdd(&hw[x < lim ? x : 256u], 1u);
    }
    for (uint64_t i = head + nvec * 16 + threadIdx.x; i < S; i += 256) {
      const uint32_t x = s[i];
      atomicAdd(&hw[x < lim ? x : 256u], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < HB; b += 256) {
    const uint32_t t = h[0][b] + h[1][b] + h[2][b] + h[3][b];
    if (t) atomicAdd(&counts[b < nbins ? b : nbins], (unsigned long long)t);
  }
}

__global__ void k_clear64(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

hipError_t histogram_u8(const uint8_t* samples, uint64_t S, int nbins,
                        unsigned long long* counts, int num_cus, hipStream_t s) {
  hipLaunchKernelGGL(k_clear64, dim3(2), dim3(256), 0, s, counts, nbins + 1);
  const uint64_t nvec = S / 16 + 1;
  uint64_t blocks = (nvec + 255) / 256;
  const uint64_t cap = (uint64_t)num_cus * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  prof_begin(KID_HIST, s);
  hipLaunchKernelGGL(k_hist, dim3((unsigned)blocks), dim3(256), 0, s, samples, S, nbins, counts);
  prof_end(KID_HIST, s);
  return hipGetLastError();
}

}  // namespace qrng

// Histogram of N-bit ADC samples (one byte each) for the min-entropy estimate
// (paper Sec. II: P'(x) is the observed frequency of each sample value).
// Each wave counts into its own LDS sub-histogram (fewer same-address
// collisions), the workgroup merges them and adds to 64-bit global counters.
// Values >= nbins are counted in an extra bin so the host can reject them.
#include <math.h>

#include "common.h"
#include "internal.h"
#include "qrng.h"

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

// Block-wide reductions over the 256 threads of k_me_finish.
__device__ double block_sum(double v, double* sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
// index of the largest value, lowest index on ties
__device__ int block_argmax(double v, int idx, double* sh, int* shi) {
  sh[threadIdx.x] = v;
  shi[threadIdx.x] = idx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double a = sh[threadIdx.x], b = sh[threadIdx.x + o];
      const int ia = shi[threadIdx.x], ib = shi[threadIdx.x + o];
      if (b > a || (b == a && ib < ia)) {
        sh[threadIdx.x] = b;
        shi[threadIdx.x] = ib;
      }
    }
    __syncthreads();
  }
  const int r = shi[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
__device__ int block_min_index(int v, int* shi) {
  shi[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) shi[threadIdx.x] = min(shi[threadIdx.x], shi[threadIdx.x + o]);
    __syncthreads();
  }
  const int r = shi[0];
  __syncthreads();
  return r;
}

__device__ double phi_dev(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

// Sec. II on the device for one sample block, thread v (of 256) owning
// sample value v with count cv: the same estimate as the host finish of
// qrng_minentropy, then the output length of Sec. III.B.  sh: 257 doubles.
__device__ void me_estimate(double cv, int N, int model, int u_mode, double mu_given,
                            double sigma_given, uint64_t n, double log2_inv_eps, uint64_t m_cap,
                            qrng_me_result* out, uint64_t* m_out, double* sh, int* shi) {
  const int K = 1 << N;
  const int v = threadIdx.x;
  if (v >= K) cv = 0.0;
  const double S = block_sum(cv, sh);
  double mu, sigma;
  if (model == QRNG_MODEL_GIVEN) {
    mu = mu_given;
    sigma = sigma_given;
  } else {
    mu = block_sum((double)v * cv, sh) / S;
    sigma = sqrt(block_sum(((double)v - mu) * ((double)v - mu) * cv, sh) / S);
  }
  double P = 0.0;
  if (v < K) {
    if (sigma > 0.0) {
      const double lo = v == 0 ? 0.0 : phi_dev(((double)v - 0.5 - mu) / sigma);
      const double hi = v == K - 1 ? 1.0 : phi_dev(((double)v + 0.5 - mu) / sigma);
      P = hi - lo;
    } else {
      double at = floor(mu + 0.5);
      at = at < 0.0 ? 0.0 : (at > K - 1 ? K - 1 : at);
      P = (v == (int)at) ? 1.0 : 0.0;
    }
  }
  // model argmax: lowest value within 1e-9 (relative) of max P, as on the host
  const double pmax = block_max(v < K ? P : -1.0, sh);
  const int um = block_min_index(v < K && P >= pmax * (1.0 - 1e-9) ? v : 1 << 30, shi);
  const int ua = block_argmax(v < K ? cv : -1.0, v, sh, shi);
  bool inU;
  if (u_mode == QRNG_U_MODEL_ARGMAX)
    inU = v == um;
  else if (u_mode == QRNG_U_BOTH_ARGMAX)
    inU = v == um || v == ua;
  else
    inU = v < K;
  const double d = 0.5 * block_sum(inU ? fabs(cv / S - P) : 0.0, sh);
  if (v == ua) sh[256] = cv;
  __syncthreads();
  if (v == 0) {
    qrng_me_result r;
    r.mu_hat = mu;
    r.sigma_hat = sigma;
    r.h_min = -log2(pmax);
    const double ca = sh[256];
    r.h_actual = ca > 0 ? -log2(ca / S) : INFINITY;
    r.d_u = d;
    r.delta_h_m = log2(d * ldexp(1.0, N + 1) + 1.0);
    r.h_mod = r.h_min - r.delta_h_m;
    r.argmax_model = (uint32_t)um;
    r.argmax_empirical = (uint32_t)ua;
    r.samples = (uint64_t)S;
    if (out) *out = r;
    double h = floor(r.h_mod);
    if (!(h > 0)) h = 0;
    if (h > N) h = N;
    const uint64_t base = (uint64_t)((unsigned __int128)n * (uint64_t)h / (uint64_t)N);
    const double secd = ceil(2.0 * log2_inv_eps);
    const uint64_t sec = secd >= 1.8e19 ? ~0ull : (uint64_t)secd;
    uint64_t m = base > sec ? base - sec : 0;
    if (m > m_cap) m = m_cap;
    *m_out = m;
  }
}

__global__ __launch_bounds__(256) void k_me_finish(MeDevArgs a) {
  __shared__ double sh[257];
  __shared__ int shi[256];
  const int v = threadIdx.x;
  const double cv = v < (1 << a.N) ? (double)a.counts[v] : 0.0;
  me_estimate(cv, a.N, a.model, a.u_mode, a.mu, a.sigma, a.n, a.log2_inv_eps, a.m_cap,
              reinterpret_cast<qrng_me_result*>(a.out), a.m_out, sh, shi);
}

// One workgroup per block of an uneven batch: histogram of the block's
// 8-bit samples in LDS (one sub-histogram per wave), then its estimate and
// output length.  Sample bytes start 8-byte aligned; S is a multiple of 8.
__global__ __launch_bounds__(256) void k_block_estimate(MeBatchArgs a) {
  __shared__ uint32_t h[4][256];
  __shared__ double sh[257];
  __shared__ int shi[256];
  const MeBlock blk = a.blocks[blockIdx.x];
  const int v = threadIdx.x, wave = v >> 6;
  for (int i = v; i < 4 * 256; i += 256) (&h[0][0])[i] = 0u;
  __syncthreads();
  uint32_t* hw = h[wave];
  const uint2* s2 = reinterpret_cast<const uint2*>(a.pool + blk.byte_off);
  const uint32_t nv = blk.S >> 3;
  uint32_t i = v;
  for (; i + 3 * 256 < nv; i += 4 * 256) {
    uint2 w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = s2[i + k * 256];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        atomicAdd(&hw[(w[k].x >> (8 * b)) & 255u], 1u);
        atomicAdd(&hw[(w[k].y >> (8 * b)) & 255u], 1u);
      }
  }
  for (; i < nv; i += 256) {
    const uint2 w = s2[i];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      atomicAdd(&hw[(w.x >> (8 * b)) & 255u], 1u);
      atomicAdd(&hw[(w.y >> (8 * b)) & 255u], 1u);
    }
  }
  __syncthreads();
  const double cv = (double)(h[0][v] + h[1][v] + h[2][v] + h[3][v]);
  me_estimate(cv, 8, a.model, a.u_mode, a.mu, a.sigma, blk.n, a.log2_inv_eps, blk.m_cap,
              a.out ? a.out + blockIdx.x : nullptr, a.m_out + blockIdx.x, sh, shi);
}

}  // namespace

hipError_t minentropy_device(const MeDevArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_me_finish, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t minentropy_blocks(const MeBatchArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  prof_begin(KID_HIST, s);
  hipLaunchKernelGGL(k_block_estimate, dim3(nblocks), dim3(256), 0, s, a);
  prof_end(KID_HIST, s);
  return hipGetLastError();
}

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

// Histogram of N-bit ADC samples (one byte each) and the min-entropy estimate
// of paper Sec. II on the device (P'(x) is the observed frequency of each
// sample value; the model P, H_min, d_U, Delta H_m and H_modify follow), with
// the output length m of Sec. III.B.
//
// Two launches: every workgroup of the first counts its slice of the
// samples into LDS sub-histograms and stores their sum as its partial
// histogram; one workgroup of the second adds the partials up and computes
// the estimate (thread v owns value v).  (A single launch whose last
// workgroup finishes needs a device-scope fence in every workgroup, which
// costs an L2 write-back per workgroup on this multi-die part; the launch
// boundary is cheaper.)  Values >= 2^N are
// counted apart so the host can reject them.
#include <math.h>

#include "common.h"
#include "internal.h"
#include "qrng.h"

namespace qrng {

namespace {

constexpr int HB = 257;  // 256 values + out-of-range
constexpr int PS = 260;  // row stride of the partial counts (16-byte rows)

// ------------------------------------------------------- wave reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ double phi_dev(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

// Workgroup-wide reductions over 256 threads: within each wave by
// shuffles, then the four wave results through LDS (red: 4 doubles).
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}
__device__ __forceinline__ double block_max(double v, double* red) {
  v = wave_max(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}
__device__ __forceinline__ int block_min(int v, int* redi) {
  v = wave_min(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) redi[threadIdx.x >> 6] = v;
  __syncthreads();
  return min(min(redi[0], redi[1]), min(redi[2], redi[3]));
}
// two sums / two maxima / two minima in one round (red: 8 doubles)
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[4 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  a = (red[0] + red[1]) + (red[2] + red[3]);
  b = (red[4] + red[5]) + (red[6] + red[7]);
}
__device__ __forceinline__ void block_max2(double& a, double& b, double* red) {
  a = wave_max(a);
  b = wave_max(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[4 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  a = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  b = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
}
__device__ __forceinline__ void block_min2(int& a, int& b, int* redi) {
  a = wave_min(a);
  b = wave_min(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    redi[threadIdx.x >> 6] = a;
    redi[4 + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  a = min(min(redi[0], redi[1]), min(redi[2], redi[3]));
  b = min(min(redi[4], redi[5]), min(redi[6], redi[7]));
}
// Sec. II for one histogram, run by a workgroup of 256 threads: thread v
// owns sample value v with count cv.  Same formulas as the host finish of
// qrng_minentropy (reduction order differs).  Thread 0 writes `out`
// (nullable) and *m_out (nullable): m = min(m_cap, n H/N - ceil(2
// log2(1/eps))) with H the whole bits of H_modify in [0, N].
// lds: 256 + 12 doubles.
__device__ void me_estimate(double cv, int N, int model, int u_mode, double mu_given,
                            double sigma_given, uint64_t n, double log2_inv_eps, uint64_t m_cap,
                            qrng_me_result* out, uint64_t* m_out, double* lds) {
  const int K = 1 << N;
  const int v = threadIdx.x;
  double* red = lds + 256;
  int* redi = reinterpret_cast<int*>(lds + 264);
  if (v >= K) cv = 0.0;
  double S = cv, s1 = (double)v * cv;
  block_sum2(S, s1, red);
  double mu, sigma;
  if (model == QRNG_MODEL_GIVEN) {
    mu = mu_given;
    sigma = sigma_given;
  } else {
    mu = s1 / S;
    const double d = (double)v - mu;
    sigma = sqrt(block_sum(d * d * cv, red) / S);
  }
  // P(v) = Phi(v + 1/2) - Phi(v - 1/2), codes 0 and K-1 take the tails: each
  // boundary is evaluated once, by the thread below it
  double P = 0.0;
  if (sigma > 0.0) {
    const double up = v >= K - 1 ? 1.0 : phi_dev(((double)v + 0.5 - mu) / sigma);
    lds[v] = up;
    __syncthreads();
    const double lo = v == 0 ? 0.0 : lds[v - 1];
    if (v < K) P = up - lo;
  } else {
    double at = floor(mu + 0.5);
    at = at < 0.0 ? 0.0 : (at > K - 1 ? K - 1 : at);
    P = (v == (int)at) ? 1.0 : 0.0;
  }
  // model argmax: lowest value within 1e-9 (relative) of max P, as on the
  // host; observed argmax: the largest count, lowest value on ties
  double pmax = v < K ? P : -1.0, cmax = v < K ? cv : -1.0;
  block_max2(pmax, cmax, red);
  int um = v < K && P >= pmax * (1.0 - 1e-9) ? v : 1 << 30;
  int ua = v < K && cv == cmax ? v : 1 << 30;
  block_min2(um, ua, redi);
  bool inU;
  if (u_mode == QRNG_U_MODEL_ARGMAX)
    inU = v == um;
  else if (u_mode == QRNG_U_BOTH_ARGMAX)
    inU = v == um || v == ua;
  else
    inU = v < K;
  const double d = 0.5 * block_sum(inU ? fabs(cv / S - P) : 0.0, red);
  if (v == 0) {
    qrng_me_result r;
    r.mu_hat = mu;
    r.sigma_hat = sigma;
    r.h_min = -log2(pmax);
    r.h_actual = cmax > 0 ? -log2(cmax / S) : INFINITY;
    r.d_u = d;
    r.delta_h_m = log2(d * ldexp(1.0, N + 1) + 1.0);
    r.h_mod = r.h_min - r.delta_h_m;
    r.argmax_model = (uint32_t)um;
    r.argmax_empirical = (uint32_t)ua;
    r.samples = (uint64_t)S;
    if (out) *out = r;
    if (m_out) {
      double h = floor(r.h_mod);
      if (!(h > 0)) h = 0;
      if (h > N) h = N;
      // n h / N without a 128-bit product (h <= N <= 8)
      const uint64_t hh = (uint64_t)h;
      const uint64_t base = (n / N) * hh + (n % N) * hh / N;
      const double secd = ceil(2.0 * log2_inv_eps);
      const uint64_t sec = secd >= 1.8e19 ? ~0ull : (uint64_t)secd;
      uint64_t m = base > sec ? base - sec : 0;
      if (m > m_cap) m = m_cap;
      *m_out = m;
    }
  }
}

// Sub-histograms: copy c (of HC) at c * HB, used by lanes with lane % HC
// == c.  Same-value samples of one wave instruction then mostly hit
// different addresses (LDS atomics to one address serialise), and the copy
// stride HB = 257 = 1 (mod 32) puts one value's copies in different banks.
constexpr int HC = 32;
__device__ __forceinline__ void count_word(uint32_t* hw, uint32_t w, uint32_t lim) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t x = (w >> (8 * b)) & 255u;
    atomicAdd(&hw[x < lim ? x : 256u], 1u);
  }
}
// the merged count of value b over the HC copies
__device__ __forceinline__ uint32_t merged(const uint32_t* h, int b) {
  uint32_t t = 0;
#pragma unroll
  for (int c = 0; c < HC; ++c) t += h[c * HB + b];
  return t;
}

struct HistArgs {
  const uint8_t* s;
  uint64_t S;
  int N;
  uint32_t* part;               // G rows of PS words: HB partial counts, zero pad
  uint32_t G;                   // workgroups of the counting launch
  unsigned long long* counts;   // nullable: the 2^N + 1 summed counts
  bool finish;                  // run the estimate (MeDevArgs below)
  MeDevArgs me;
};

__global__ __launch_bounds__(256) void k_hist_part(HistArgs a) {
  __shared__ uint32_t h[HC * HB];
  const int tid = threadIdx.x;
  for (int i = tid; i < HC * HB; i += 256) h[i] = 0u;
  __syncthreads();
  uint32_t* hw = h + (tid % HC) * HB;
  const uint32_t lim = 1u << a.N;
  // bytes before the first 16-byte boundary and after the last are counted
  // one at a time by workgroup 0
  const uint64_t mis = (uint64_t)(reinterpret_cast<uintptr_t>(a.s) & 15u);
  const uint64_t head = mis ? (16 - mis < a.S ? 16 - mis : a.S) : 0;
  const uint64_t nvec = (a.S - head) / 16;
  const uint4* s4 = reinterpret_cast<const uint4*>(a.s + head);
  const uint64_t G = gridDim.x;
  // contiguous slice per workgroup, 4 vectors in flight per thread
  const uint64_t per = (nvec + G - 1) / G;
  const uint64_t v0 = (uint64_t)blockIdx.x * per;
  const uint64_t v1 = v0 + per < nvec ? v0 + per : nvec;
  uint64_t i = v0 + tid;
  for (; i + 3 * 256 < v1; i += 4 * 256) {
    uint4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = s4[i + k * 256];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      count_word(hw, v[k].x, lim);
      count_word(hw, v[k].y, lim);
      count_word(hw, v[k].z, lim);
      count_word(hw, v[k].w, lim);
    }
  }
  for (; i < v1; i += 256) {
    const uint4 v = s4[i];
    count_word(hw, v.x, lim);
    count_word(hw, v.y, lim);
    count_word(hw, v.z, lim);
    count_word(hw, v.w, lim);
  }
  if (blockIdx.x == 0) {
    for (uint64_t j = tid; j < head; j += 256) {
      const uint32_t x = a.s[j];
      atomicAdd(&hw[x < lim ? x : 256u], 1u);
    }
    for (uint64_t j = head + nvec * 16 + tid; j < a.S; j += 256) {
      const uint32_t x = a.s[j];
      atomicAdd(&hw[x < lim ? x : 256u], 1u);
    }
  }
  __syncthreads();
  uint32_t* mine = a.part + (uint64_t)blockIdx.x * PS;
  for (int b = tid; b < PS; b += 256) mine[b] = b < HB ? merged(h, b) : 0u;
}

__global__ __launch_bounds__(256) void k_hist_finish(HistArgs a) {
  __shared__ double lds[272];
  const int tid = threadIdx.x;
  const uint32_t lim = 1u << a.N;
  const uint64_t G = a.G;
  // The G partial rows were written by other dies, so every load misses the
  // local L2 and costs a full round trip: thread (q, c) adds bins 4c..4c+3
  // over quarter q of the rows with 16-byte loads, 16 in flight (one round
  // trip for the usual G <= 64); threads 0..63 add the out-of-range bin over
  // rows g = tid mod 64.  Thread b then owns bin b.
  __shared__ unsigned long long qs[4][256];
  __shared__ unsigned long long oobs[64];
  {
    const int c = tid & 63, q = tid >> 6;
    const uint64_t g0 = q * G / 4, g1 = (q + 1) * G / 4;
    const uint4* __restrict__ p4 = reinterpret_cast<const uint4*>(a.part) + c;
    unsigned long long s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    uint64_t g = g0;
    for (; g + 16 <= g1; g += 16) {
      uint4 x[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) x[k] = p4[(g + k) * (PS / 4)];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        s0 += x[k].x;
        s1 += x[k].y;
        s2 += x[k].z;
        s3 += x[k].w;
      }
    }
    for (; g < g1; ++g) {
      const uint4 x = p4[g * (PS / 4)];
      s0 += x.x;
      s1 += x.y;
      s2 += x.z;
      s3 += x.w;
    }
    qs[q][4 * c] = s0;
    qs[q][4 * c + 1] = s1;
    qs[q][4 * c + 2] = s2;
    qs[q][4 * c + 3] = s3;
    if (tid < 64) {
      unsigned long long o = 0;
      for (uint64_t r = tid; r < G; r += 64) o += a.part[r * PS + 256];
      oobs[tid] = o;
    }
  }
  __syncthreads();
  const uint64_t t = qs[0][tid] + qs[1][tid] + qs[2][tid] + qs[3][tid];
  uint64_t o = 0;
  if (tid == 0)
    for (int r = 0; r < 64; ++r) o += oobs[r];
  if (a.counts) {
    if (tid < (int)lim) a.counts[tid] = t;
    if (tid == 0) a.counts[lim] = o;
  }
  if (a.finish)
    me_estimate((double)t, a.N, a.me.model, a.me.u_mode, a.me.mu, a.me.sigma, a.me.n,
                a.me.log2_inv_eps, a.me.m_cap, reinterpret_cast<qrng_me_result*>(a.me.out),
                a.me.m_out, lds);
}

// One workgroup per block of an uneven batch: histogram of the block's
// 8-bit samples in LDS sub-histograms, then its estimate and output
// length.  Sample bytes start 8-byte aligned; S is a
// multiple of 8.
__global__ __launch_bounds__(256) void k_block_estimate(MeBatchArgs a) {
  __shared__ uint32_t h[HC * HB];
  const MeBlock blk = a.blocks[blockIdx.x];
  const int v = threadIdx.x;
  for (int i = v; i < HC * HB; i += 256) h[i] = 0u;
  __syncthreads();
  uint32_t* hw = h + (v % HC) * HB;
  const uint2* s2 = reinterpret_cast<const uint2*>(a.pool + blk.byte_off);
  const uint32_t nv = blk.S >> 3;
  uint32_t i = v;
  for (; i + 3 * 256 < nv; i += 4 * 256) {
    uint2 w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = s2[i + k * 256];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      count_word(hw, w[k].x, 256u);
      count_word(hw, w[k].y, 256u);
    }
  }
  for (; i < nv; i += 256) {
    const uint2 w = s2[i];
    count_word(hw, w.x, 256u);
    count_word(hw, w.y, 256u);
  }
  __syncthreads();
  __shared__ double lds[272];
  me_estimate((double)merged(h, v), 8, a.model, a.u_mode, a.mu,
              a.sigma, blk.n, a.log2_inv_eps, blk.m_cap, a.out ? a.out + blockIdx.x : nullptr,
              a.m_out + blockIdx.x, lds);
}

// workgroups for S samples: about 16 KiB each, at most 256 (the partials
// the last workgroup adds up)
unsigned hist_groups(uint64_t S) {
  uint64_t g = (S + (16u << 10) - 1) / (16u << 10);
  if (g < 1) g = 1;
  if (g > HIST_MAX_GROUPS) g = HIST_MAX_GROUPS;
  return (unsigned)g;
}

}  // namespace

uint64_t hist_scratch_words() { return (uint64_t)HIST_MAX_GROUPS * PS; }

hipError_t hist_estimate(const uint8_t* samples, uint64_t S, int N, uint32_t* scratch,
                         unsigned long long* counts_out, const MeDevArgs* finish,
                         hipStream_t s) {
  HistArgs a{};
  a.s = samples;
  a.S = S;
  a.N = N;
  a.part = scratch;
  a.G = hist_groups(S);
  a.counts = counts_out;
  a.finish = finish != nullptr;
  if (finish) a.me = *finish;
  prof_begin(KID_HIST, s);
  hipLaunchKernelGGL(k_hist_part, dim3(a.G), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_hist_finish, dim3(1), dim3(256), 0, s, a);
  prof_end(KID_HIST, s);
  return hipGetLastError();
}

hipError_t minentropy_blocks(const MeBatchArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  prof_begin(KID_HIST, s);
  hipLaunchKernelGGL(k_block_estimate, dim3(nblocks), dim3(256), 0, s, a);
  prof_end(KID_HIST, s);
  return hipGetLastError();
}

}  // namespace qrng

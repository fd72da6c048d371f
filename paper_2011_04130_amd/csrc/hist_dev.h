// Device-side pieces of the histogram and min-entropy estimate (paper
// Sec. II; output length of Sec. III.B), shared by the estimate kernels and
// by the first transform pass, whose extra workgroups can run the estimate
// alongside the column transforms.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "internal.h"
#include "qrng.h"

namespace qrng {
namespace hd {

constexpr int HB = 257;  // 256 values + out-of-range
constexpr int PS = 260;  // row stride of the partial counts (16-byte rows)
// two more words of a partial row: the call's tag, and the samples the
// workgroup examined mod 2^32 (the finish checks both before it trusts the
// rows)
constexpr int ROW_TAG = 257, ROW_SEEN = 258;
// the ticket of the fused estimate sits after the partial rows
constexpr uint64_t TICKET_WORD = (uint64_t)HIST_MAX_GROUPS * PS;

// ------------------------------------------------------- wave reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double phi_dev(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

// Pairwise combination of NW wave results (the same tree for every NW, so
// waves that hold only zeros leave the result bit-identical).
template <int NW>
__device__ inline double tree_sum(const double* r) {
  if constexpr (NW == 1)
    return r[0];
  else
    return tree_sum<NW / 2>(r) + tree_sum<NW / 2>(r + NW / 2);
}
template <int NW>
__device__ inline double tree_max(const double* r) {
  if constexpr (NW == 1)
    return r[0];
  else
    return fmax(tree_max<NW / 2>(r), tree_max<NW / 2>(r + NW / 2));
}
template <int NW>
__device__ inline int tree_min(const int* r) {
  if constexpr (NW == 1)
    return r[0];
  else
    return min(tree_min<NW / 2>(r), tree_min<NW / 2>(r + NW / 2));
}

// Workgroup-wide reductions over NW waves: within each wave by shuffles,
// then the wave results through LDS (red: NW doubles, or 2 NW for pairs).
template <int NW>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return tree_sum<NW>(red);
}
template <int NW>
__device__ inline void block_sum2(double& a, double& b, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[NW + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  a = tree_sum<NW>(red);
  b = tree_sum<NW>(red + NW);
}
template <int NW>
__device__ inline void block_max2(double& a, double& b, double* red) {
  a = wave_max(a);
  b = wave_max(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[NW + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  a = tree_max<NW>(red);
  b = tree_max<NW>(red + NW);
}
template <int NW>
__device__ inline void block_min2(int& a, int& b, int* redi) {
  a = wave_min(a);
  b = wave_min(b);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    redi[threadIdx.x >> 6] = a;
    redi[NW + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  a = tree_min<NW>(redi);
  b = tree_min<NW>(redi + NW);
}

// LDS doubles me_estimate<NT> uses
constexpr int me_lds_doubles(int NT) { return 256 + 3 * (NT / 64); }

// Sec. II for one histogram, run by a workgroup of NT >= 256 threads: thread
// v < 256 owns sample value v with count cv (threads from 2^N on hold 0).
// Same formulas as the host finish of qrng_minentropy (reduction order
// differs).  Thread 0 writes `out` (nullable) and *m_out (nullable): m =
// min(m_cap, n H/N - ceil(2 log2(1/eps))) with H the whole bits of H_modify
// in [0, N].  lds: me_lds_doubles(NT) doubles.
template <int NT>
__device__ void me_estimate(double cv, int N, int model, int u_mode, double mu_given,
                            double sigma_given, uint64_t n, double log2_inv_eps, uint64_t m_cap,
                            qrng_me_result* out, uint64_t* m_out, double* lds) {
  constexpr int NW = NT / 64;
  const int K = 1 << N;
  const int v = threadIdx.x;
  double* red = lds + 256;
  int* redi = reinterpret_cast<int*>(lds + 256 + 2 * NW);
  if (v >= K) cv = 0.0;
  double S = cv, s1 = (double)v * cv;
  block_sum2<NW>(S, s1, red);
  double mu, sigma;
  if (model == QRNG_MODEL_GIVEN) {
    mu = mu_given;
    sigma = sigma_given;
  } else {
    mu = s1 / S;
    const double d = (double)v - mu;
    // Sec. II.B: with the quantum model, the classical s.d. (sigma_given)
    // is taken out of the variance
    const double var = block_sum<NW>(d * d * cv, red) / S -
                       (model == QRNG_MODEL_QUANTUM ? sigma_given * sigma_given : 0.0);
    sigma = var > 0.0 ? sqrt(var) : 0.0;
  }
  // P(v) = Phi(v + 1/2) - Phi(v - 1/2), codes 0 and K-1 take the tails: each
  // boundary is evaluated once, by the thread below it
  double P = 0.0;
  if (sigma > 0.0) {
    const double up = v >= K - 1 ? 1.0 : phi_dev(((double)v + 0.5 - mu) / sigma);
    if (v < 256) lds[v] = up;
    __syncthreads();
    if (v < K) P = up - (v == 0 ? 0.0 : lds[v - 1]);
  } else {
    double at = floor(mu + 0.5);
    at = at < 0.0 ? 0.0 : (at > K - 1 ? K - 1 : at);
    P = (v == (int)at) ? 1.0 : 0.0;
  }
  // model argmax: lowest value within 1e-9 (relative) of max P, as on the
  // host (the two-argmax set takes all of them); observed argmax: the
  // largest count, lowest value on ties
  double pmax = v < K ? P : -1.0, cmax = v < K ? cv : -1.0;
  block_max2<NW>(pmax, cmax, red);
  const bool tied = v < K && P >= pmax * (1.0 - 1e-9);
  int um = tied ? v : 1 << 30;
  int ua = v < K && cv == cmax ? v : 1 << 30;
  block_min2<NW>(um, ua, redi);
  bool inU;
  if (u_mode == QRNG_U_MODEL_ARGMAX)
    inU = v == um;
  else if (u_mode == QRNG_U_BOTH_ARGMAX)
    inU = tied || v == ua;  // every value tied for max P, and argmax P'
  else
    inU = v < K;
  const double d = 0.5 * block_sum<NW>(inU ? fabs(cv / S - P) : 0.0, red);
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

// Sub-histograms: copy c (of HCW) at c * HB, used by lanes with lane % HCW
// == c.  Same-value samples of one wave instruction then mostly hit
// different addresses (LDS atomics to one address serialise), and the copy
// stride HB = 257 = 1 (mod 32) puts one value's copies in different banks.
constexpr int HC = 32;
__device__ inline void count_word(uint32_t* hw, uint32_t w, uint32_t lim) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t x = (w >> (8 * b)) & 255u;
    atomicAdd(&hw[x < lim ? x : 256u], 1u);
  }
}
// the merged count of value b over the HCW copies
template <int HCW>
__device__ inline uint32_t merged(const uint32_t* h, int b) {
  uint32_t t = 0;
#pragma unroll
  for (int c = 0; c < HCW; ++c) t += h[c * HB + b];
  return t;
}

// Block b of an uneven batch, run by a workgroup of NT threads: histogram of
// the block's 8-bit samples in LDS sub-histograms h (HC * HB words), then its
// estimate and output length (lds: me_lds_doubles(NT) doubles).  Sample
// bytes start 8-byte aligned; S is a multiple of 8.
template <int NT>
__device__ void block_estimate_body(const MeBatchArgs& a, uint32_t b, uint32_t* h, double* lds) {
  const MeBlock blk = a.blocks[b];
  const int v = threadIdx.x;
  for (int i = v; i < HC * HB; i += NT) h[i] = 0u;
  __syncthreads();
  uint32_t* hw = h + (v % HC) * HB;
  const uint2* s2 = reinterpret_cast<const uint2*>(a.pool + blk.byte_off);
  const uint32_t nv = blk.S >> 3;
  uint32_t i = v;
  for (; i + 3 * NT < nv; i += 4 * NT) {
    uint2 w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = s2[i + k * NT];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      count_word(hw, w[k].x, 256u);
      count_word(hw, w[k].y, 256u);
    }
  }
  for (; i < nv; i += NT) {
    const uint2 w = s2[i];
    count_word(hw, w.x, 256u);
    count_word(hw, w.y, 256u);
  }
  __syncthreads();
  me_estimate<NT>(v < 256 ? (double)merged<HC>(h, v) : 0.0, 8, a.model, a.u_mode, a.mu, a.sigma,
                  blk.n, a.log2_inv_eps, blk.m_cap, a.out ? a.out + b : nullptr, a.m_out + b,
                  lds);
}

// The estimate on a random subset of the samples (Sec. II.C suggests it as a
// cheaper route): sample t is kept when the high 32 bits of output t of the
// SplitMix64 generator seeded with `seed` (Steele, Lea and Flood's
// counter-based form: mix(seed + (t+1) 0x9e3779b97f4a7c15)) are below thr.
__device__ __forceinline__ bool subset_keep(uint64_t seed, uint64_t t, uint32_t thr) {
  uint64_t z = seed + (t + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (uint32_t)(z >> 32) < thr;
}

struct HistArgs {
  const uint8_t* s;
  uint64_t S;
  int N;
  uint64_t subset_seed;  // with keep_thr > 0, only the kept samples count
  uint32_t keep_thr;
  uint32_t* part;               // G rows of PS words: HB partial counts, zero pad
  uint32_t G;                   // workgroups that count
  unsigned long long* counts;   // nullable: the 2^N + 1 summed counts
  bool finish;                  // run the estimate (MeDevArgs below)
  MeDevArgs me;
  uint32_t epoch;               // tag of this call, written into every partial row
  uint32_t expect;              // tag the finish requires (epoch, except under fault tests)
};

// workgroups for S samples: about 16 KiB each, at most HIST_MAX_GROUPS (the
// partials the finish adds up)
__host__ __device__ inline unsigned hist_groups(uint64_t S) {
  uint64_t g = (S + (16u << 10) - 1) / (16u << 10);
  if (g < 1) g = 1;
  if (g > (uint64_t)HIST_MAX_GROUPS) g = HIST_MAX_GROUPS;
  return (unsigned)g;
}

// the 4 samples of word w, the first at sample index t, kept ones only
__device__ inline void count_word_subset(uint32_t* hw, uint32_t w, uint32_t lim, uint64_t t,
                                         uint64_t seed, uint32_t thr) {
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const uint32_t x = (w >> (8 * b)) & 255u;
    if (subset_keep(seed, t + b, thr)) atomicAdd(&hw[x < lim ? x : 256u], 1u);
  }
}

// Workgroup wg (of a.G) counts its contiguous slice of the samples into
// HCW LDS sub-histograms h (HCW * HB words) and stores their sum as partial
// row wg (with COHERENT as device-scope atomic stores, which write through
// to the level all dies share; with SUBSET only the kept samples).  Bytes
// before the first 16-byte boundary and after the last are counted one at a
// time by workgroup 0.
template <int NT, int HCW, bool COHERENT = false, bool SUBSET = false>
__device__ void hist_part_body(const HistArgs& a, uint32_t wg, uint32_t* h) {
  const int tid = threadIdx.x;
  for (int i = tid; i < HCW * HB; i += NT) h[i] = 0u;
  __syncthreads();
  uint32_t* hw = h + (tid % HCW) * HB;
  const uint32_t lim = 1u << a.N;
  const uint64_t mis = (uint64_t)(reinterpret_cast<uintptr_t>(a.s) & 15u);
  const uint64_t head = mis ? (16 - mis < a.S ? 16 - mis : a.S) : 0;
  const uint64_t nvec = (a.S - head) / 16;
  const uint4* s4 = reinterpret_cast<const uint4*>(a.s + head);
  const uint64_t G = a.G;
  // contiguous slice per workgroup, 4 vectors in flight per thread
  const uint64_t per = (nvec + G - 1) / G;
  const uint64_t v0 = (uint64_t)wg * per;
  const uint64_t v1 = v0 + per < nvec ? v0 + per : nvec;
  uint64_t i = v0 + tid;
  // vector i holds samples head + 16 i .. head + 16 i + 15
  auto count4 = [&](const uint4& v, uint64_t vi) {
    if constexpr (SUBSET) {
      const uint64_t t = head + 16 * vi;
      count_word_subset(hw, v.x, lim, t, a.subset_seed, a.keep_thr);
      count_word_subset(hw, v.y, lim, t + 4, a.subset_seed, a.keep_thr);
      count_word_subset(hw, v.z, lim, t + 8, a.subset_seed, a.keep_thr);
      count_word_subset(hw, v.w, lim, t + 12, a.subset_seed, a.keep_thr);
    } else {
      count_word(hw, v.x, lim);
      count_word(hw, v.y, lim);
      count_word(hw, v.z, lim);
      count_word(hw, v.w, lim);
    }
  };
  for (; i + 3 * NT < v1; i += 4 * NT) {
    uint4 v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = s4[i + k * NT];
#pragma unroll
    for (int k = 0; k < 4; ++k) count4(v[k], i + k * NT);
  }
  for (; i < v1; i += NT) count4(s4[i], i);
  auto count1 = [&](uint64_t j) {
    const uint32_t x = a.s[j];
    if (!SUBSET || subset_keep(a.subset_seed, j, a.keep_thr))
      atomicAdd(&hw[x < lim ? x : 256u], 1u);
  };
  if (wg == 0) {
    for (uint64_t j = tid; j < head; j += NT) count1(j);
    for (uint64_t j = head + nvec * 16 + tid; j < a.S; j += NT) count1(j);
  }
  __syncthreads();
  uint32_t* mine = a.part + (uint64_t)wg * PS;
  // samples this workgroup examined (its vectors, and the ragged ends for
  // workgroup 0): over all rows they add up to S
  const uint64_t seen = (v1 > v0 ? v1 - v0 : 0) * 16 + (wg == 0 ? a.S - nvec * 16 : 0);
  for (int b = tid; b < PS; b += NT) {
    const uint32_t v = b < HB ? merged<HCW>(h, b)
                              : (b == ROW_TAG ? a.epoch : (b == ROW_SEEN ? (uint32_t)seen : 0u));
    if constexpr (COHERENT)
      __hip_atomic_store(mine + b, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      mine[b] = v;
  }
}

struct FinishLds {
  unsigned long long qs[4][256];
  unsigned long long oobs[64];
  unsigned long long seen[64];
  uint32_t bad[64];
  uint32_t ok;
  double me[me_lds_doubles(512)];
};

// Sums the a.G partial rows and runs the estimate (NT >= 256 threads).  The
// rows were written by other dies, so every load misses the local L2 and
// costs a full round trip: thread (q, c) < 256 adds bins 4c..4c+3 over
// quarter q of the rows with 16-byte loads, 16 in flight (one round trip for
// the usual G <= 64); threads 0..63 add the out-of-range bin over rows
// g = tid mod 64.  Thread b < 256 then owns bin b.
template <int NT>
__device__ void hist_finish_body(const HistArgs& a, FinishLds& L) {
  const int tid = threadIdx.x;
  const uint32_t lim = 1u << a.N;
  const uint64_t G = a.G;
  if (tid < 256) {
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
    L.qs[q][4 * c] = s0;
    L.qs[q][4 * c + 1] = s1;
    L.qs[q][4 * c + 2] = s2;
    L.qs[q][4 * c + 3] = s3;
    if (tid < 64) {
      unsigned long long o = 0;
      for (uint64_t r = tid; r < G; r += 64) o += a.part[r * PS + 256];
      L.oobs[tid] = o;
    } else if (tid < 128) {
      // the rows' tags and examined-sample counts
      unsigned long long sn = 0;
      uint32_t bad = 0;
      for (uint64_t r = tid - 64; r < G; r += 64) {
        sn += a.part[r * PS + ROW_SEEN];
        bad |= a.part[r * PS + ROW_TAG] ^ a.expect;
      }
      L.seen[tid - 64] = sn;
      L.bad[tid - 64] = bad;
    }
  }
  __syncthreads();
  if (tid == 0) {
    unsigned long long sn = 0;
    uint32_t bad = 0;
    for (int r = 0; r < 64; ++r) {
      sn += L.seen[r];
      bad |= L.bad[r];
    }
    // every row carries this call's tag and together they examined every
    // sample: otherwise a row is stale or missing, and the estimate fails
    // closed (no output bits) instead of trusting it
    L.ok = bad == 0 && (uint32_t)sn == (uint32_t)a.S;  // rows hold the counts mod 2^32
  }
  __syncthreads();
  const bool ok = L.ok != 0;
  const uint64_t t = tid < 256 ? L.qs[0][tid] + L.qs[1][tid] + L.qs[2][tid] + L.qs[3][tid] : 0;
  if (a.counts) {
    if (tid < (int)lim) a.counts[tid] = t;
    if (tid == 0) {
      uint64_t o = 0;
      for (int r = 0; r < 64; ++r) o += L.oobs[r];
      a.counts[lim] = o;
      a.counts[lim + 1] = ok ? 1u : 0u;
    }
  }
  if (!a.finish) return;
  if (ok) {
    me_estimate<NT>((double)t, a.N, a.me.model, a.me.u_mode, a.me.mu, a.me.sigma, a.me.n,
                    a.me.log2_inv_eps, a.me.m_cap, reinterpret_cast<qrng_me_result*>(a.me.out),
                    a.me.m_out, L.me);
  } else if (tid == 0) {
    qrng_me_result r;
    const double nan = __builtin_nan("");
    r.mu_hat = r.sigma_hat = r.h_min = r.h_actual = r.d_u = r.delta_h_m = r.h_mod = nan;
    r.argmax_model = r.argmax_empirical = 0xffffffffu;
    r.samples = 0;
    if (a.me.out) *reinterpret_cast<qrng_me_result*>(a.me.out) = r;
    if (a.me.m_out) *a.me.m_out = 0;
  }
}

// One of a.G counting workgroups of a launch that also does other work: it
// stores its partial row, and the last of them to finish (a device-scope
// ticket) sums the rows and runs the estimate, then sets the ticket up for
// the next call.  The rows are published without a device-scope release
// fence, which would write back every dirty line of this die's L2 (the
// other work's output streams through it): they are stored write-through
// (device-scope atomic stores) and each thread waits until its stores have
// completed (s_waitcnt 0; a workgroup-scope release alone emits no wait for
// them) before the barrier that precedes the ticket.  The last workgroup
// invalidates its die's caches (device-scope acquire) before reading the
// rows.  lds: at least max(HCW * HB words,
// sizeof(FinishLds)) bytes, 16-byte aligned.
// The ticket word holds (tag, count): TICKET_COUNT_BITS low bits count the
// workgroups of the call with that tag.  The last workgroup of a call leaves
// the word at (next tag, 0), the tag the context's next call will carry, so
// in the normal sequence every workgroup takes its ticket with one atomic
// add.  A workgroup whose add finds another tag there (a replay with the
// same tag, another context's sequence, or a launch that never completed)
// joins through a compare-and-swap loop that starts the count afresh under
// its own tag, so a stuck ticket cannot silence later calls.
constexpr int TICKET_COUNT_BITS = 9;  // HIST_MAX_GROUPS = 256 fits
constexpr uint32_t TICKET_TAG_MASK = (1u << (32 - TICKET_COUNT_BITS)) - 1;
static_assert(2 * HIST_MAX_GROUPS <= (1 << TICKET_COUNT_BITS),
              "ticket count field: a stale count below G plus G adds never carries into the tag");

// Takes this workgroup's ticket; true for the last of the call's G.  Lock
// free: a failed compare-and-swap means another workgroup's succeeded, so
// the loop ends after at most G rounds.  The adds that land on a word with
// another tag are discarded when the loop replaces that word.
__device__ inline bool take_ticket(uint32_t* ticket, uint32_t epoch, uint32_t G) {
  constexpr uint32_t CM = (1u << TICKET_COUNT_BITS) - 1;
  const uint32_t tag = epoch << TICKET_COUNT_BITS;
  uint32_t old = atomicAdd(ticket, 1u);
  if ((old & ~CM) == tag) return (old & CM) + 1u == G;
  old = old + 1u;  // the word as this add left it (other adds may follow)
  for (uint32_t k = 0; k <= 2 * G; ++k) {
    const uint32_t cnt = (old & ~CM) == tag ? (old & CM) : 0u;
    const uint32_t seen = atomicCAS(ticket, old, tag | (cnt + 1u));
    if (seen == old) return cnt + 1u == G;
    old = seen;
  }
  return false;  // not reached: each failed round is another workgroup's success or add
}

template <int NT, int HCW>
__device__ void estimate_workgroup(const HistArgs& a, uint32_t wg, uint32_t* ticket,
                                   uint32_t* lds) {
  hist_part_body<NT, HCW, true>(a, wg, lds);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) lds[0] = take_ticket(ticket, a.epoch, a.G) ? 1u : 0u;
  __syncthreads();
  if (lds[0] == 0u) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  FinishLds& L = *reinterpret_cast<FinishLds*>(lds);
  hist_finish_body<NT>(a, L);
  // the next call's tag with a zero count: its workgroups then take their
  // tickets with one add each.  After a failed row check (a ticket that was
  // not this call's alone) the word keeps this call's tag, so late adds of
  // this call cannot leak into the next call's count: that call then starts
  // afresh through the compare-and-swap loop.
  if (threadIdx.x == 0) {
    const uint32_t next = L.ok ? a.epoch + 1u : a.epoch;
    atomicExch(ticket, (next & TICKET_TAG_MASK) << TICKET_COUNT_BITS);
  }
}

}  // namespace hd
}  // namespace qrng

// The paper's own accelerated method on the GPU (Sec. III.B: the circulant
// embedding of Definition 1, diagonalised by the DFT as in Theorems 1-2),
// in float64 as the paper computes it: k' = F^-1(F a . F r') with a the
// n+m-1 seed bits and r' the raw block zero-padded, both to a power-of-two
// length N >= n+m-1 (the kept rows never wrap, so padding leaves them
// unchanged); then round, mod 2, and keep rows n-1 .. n+m-2.  A comparison
// path beside the exact transform mod p: it is exact only while every kept
// value lies well within 1/2 of an integer, and it reports the largest
// distance it saw.
//
// Both real inputs share one complex transform (z = a + i r; the two spectra
// are separated from Z[k] and conj Z[N-k]), so a hash costs one forward and
// one inverse complex transform of length N plus two elementwise passes (and
// a packing pass, unless the first forward pass reads the bits itself).
// Transforms are Stockham autosort passes (no bit reversal): a radix 2/4/8
// pass first when log2 N is not a multiple of 4, a radix-16 pass, then
// radix-256 passes (two 16-point DFT steps through LDS per sweep of the
// array) while at least 8 levels remain, and a last radix-16 pass for the
// rest; 16-point DFTs in registers, twiddles from sincospi.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

struct cplx {
  double x, y;
};
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}

// cos and sin of 2 pi k / 16, k = 0..4 (the rest follow by symmetry)
constexpr double C16[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440,
                           0.38268343236508977173, 0.0};

// exp(sign 2 pi i e / 16), sign = -1 forward, +1 inverse
template <bool INV>
__device__ __forceinline__ cplx root16(int e) {
  e &= 15;
  // cos(2 pi e/16) and sin(2 pi e/16) from the first quadrant
  const int q = e >> 2, r = e & 3;
  double c, s;
  if (q == 0) {
    c = C16[r];
    s = C16[4 - r];
  } else if (q == 1) {
    c = -C16[4 - r];
    s = C16[r];
  } else if (q == 2) {
    c = -C16[r];
    s = -C16[4 - r];
  } else {
    c = C16[4 - r];
    s = -C16[r];
  }
  return {c, INV ? s : -s};
}

constexpr int ilg(int v) { return v <= 1 ? 0 : 1 + ilg(v >> 1); }
constexpr int brv(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

// In-register R-point DFT (R = 2, 4, 8, 16), natural order in and out:
// v[k] = sum_q v[q] exp(sign 2 pi i q k / R); radix-2 decimation in time on
// the bit-reversed input.
template <int R, bool INV>
__device__ __forceinline__ void dft_small(cplx (&v)[R]) {
  constexpr int LG = ilg(R);
  cplx t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[i] = v[brv(i, LG)];
#pragma unroll
  for (int half = 1; half < R; half *= 2) {
#pragma unroll
    for (int base = 0; base < R; base += 2 * half) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const cplx w = root16<INV>(j * (16 / (2 * half)));
        const cplx b = j == 0 ? t[base + j + half] : cmul(t[base + j + half], w);
        const cplx a = t[base + j];
        t[base + j] = cadd(a, b);
        t[base + j + half] = csub(a, b);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = t[i];
}


// Input q of the forward transform, (seed bit q, raw bit q), 0 past L and n.
struct PackedIn {
  const uint32_t* seed;
  uint64_t L;
  const uint32_t* x;
  uint64_t n;
  unsigned long long* err;  // cleared by the first thread (nullable)
};
__device__ __forceinline__ cplx packed_at(const PackedIn& p, uint64_t q) {
  const double a = q < p.L ? (double)((p.seed[q >> 5] >> (q & 31)) & 1u) : 0.0;
  const double r = q < p.n ? (double)((p.x[q >> 5] >> (q & 31)) & 1u) : 0.0;
  return {a, r};
}

// z[q] = (seed bit q, raw bit q) for q < N; clears *err.
__global__ __launch_bounds__(256) void k_fft_pack(PackedIn pk, cplx* __restrict__ z, uint64_t N) {
  const uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (q == 0 && pk.err) *pk.err = 0ull;
  if (q >= N) return;
  z[q] = packed_at(pk, q);
}

// One Stockham pass of radix R over N points: sub-transforms of length Ns
// are done; thread j combines R of them (inputs j + r N/R) into one of
// length Ns R at (j / Ns) Ns R + j mod Ns + r Ns.
template <int R, bool INV>
__global__ __launch_bounds__(256) void k_fft_pass(const cplx* __restrict__ in,
                                                  cplx* __restrict__ out, uint64_t N,
                                                  uint64_t Ns) {
  const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t stride = N / R;
  if (j >= stride) return;
  cplx v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = in[j + r * stride];
  const uint64_t k = j % Ns;
  if (Ns > 1) {
    // twiddle exp(sign 2 pi i r k / (Ns R)) = sincospi(sign 2 r k / (Ns R))
    const double base = (INV ? 2.0 : -2.0) * (double)k / (double)(Ns * R);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      double s, c;
      sincospi(base * r, &s, &c);
      v[r] = cmul(v[r], cplx{c, s});
    }
  }
  dft_small<R, INV>(v);
  const uint64_t o = (j / Ns) * Ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) out[o + r * Ns] = v[r];
}

// The first pass when it has radix 16 (Ns = 1: no twiddles, outputs j 16 +
// r): the 256 j of a workgroup own 4096 consecutive outputs, staged through
// LDS so that the stores are coalesced (N >= 4096).  BITS: the forward
// transform's first pass reads the seed and raw bits itself (no pack pass).
template <bool INV, bool BITS>
__global__ __launch_bounds__(256) void k_fft_first16(const cplx* __restrict__ in,
                                                     cplx* __restrict__ out, uint64_t N,
                                                     PackedIn pk) {
  __shared__ cplx st[256 * 17];  // [j][r], rows padded to 17
  const int t = threadIdx.x;
  const uint64_t stride = N >> 4;
  const uint64_t j = (uint64_t)blockIdx.x * 256 + t;
  cplx v[16];
  if constexpr (BITS) {
    if (j == 0 && pk.err) *pk.err = 0ull;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = packed_at(pk, j + r * stride);
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = in[j + r * stride];
  }
  dft_small<16, INV>(v);
#pragma unroll
  for (int r = 0; r < 16; ++r) st[t * 17 + r] = v[r];
  __syncthreads();
  cplx* __restrict__ o = out + (uint64_t)blockIdx.x * 4096;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = t + 256 * i;
    o[e] = st[(e >> 4) * 17 + (e & 15)];
  }
}

// The same pass with radix 256 = 16 x 16, both steps in LDS (Ns >= 16, N >=
// 4096): a workgroup takes 16 consecutive j (consecutive k, since 16 | Ns)
// and all 256 inputs of each.  With x[r] the twiddled inputs and r = r1 +
// 16 r2, r' = a + 16 b:  X[r'] = sum_r1 w16^(r1 b) w256^(r1 a) sum_r2
// x[r1 + 16 r2] w16^(r2 a), so thread (jj, q) first does the inner DFT for
// r1 = q, then the outer one for a = q.
template <bool INV>
__global__ __launch_bounds__(256) void k_fft_pass256(const cplx* __restrict__ in,
                                                     cplx* __restrict__ out, uint64_t N,
                                                     uint64_t Ns) {
  __shared__ cplx buf[256 * 17];  // [r][jj], rows padded to 17
  __shared__ cplx w256[256];      // exp(sign 2 pi i e / 256)
  const int t = threadIdx.x;
  const int jj = t & 15, q = t >> 4;
  const uint64_t stride = N >> 8;
  const uint64_t j0 = (uint64_t)blockIdx.x * 16;
  {
    double s, c;
    sincospi((double)t / 128.0, &s, &c);
    w256[t] = {c, INV ? s : -s};
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = q + 16 * i;
    buf[r * 17 + jj] = in[j0 + jj + (uint64_t)r * stride];
  }
  __syncthreads();
  const uint64_t j = j0 + jj;
  const uint64_t k = j % Ns;
  cplx v[16];
  // inner DFT over r2 for r1 = q, after the pass twiddle exp(sign 2 pi i r k / (Ns 256))
  const double base = (INV ? 2.0 : -2.0) * (double)k / (double)(Ns * 256);
#pragma unroll
  for (int r2 = 0; r2 < 16; ++r2) {
    const int r = q + 16 * r2;
    v[r2] = buf[r * 17 + jj];
    if (r) {
      double s, c;
      sincospi(base * r, &s, &c);
      v[r2] = cmul(v[r2], cplx{c, s});
    }
  }
  dft_small<16, INV>(v);
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 16; ++a)
    buf[(a * 16 + q) * 17 + jj] = a ? cmul(v[a], w256[(q * a) & 255]) : v[a];
  __syncthreads();
  // outer DFT over r1 for a = q
#pragma unroll
  for (int r1 = 0; r1 < 16; ++r1) v[r1] = buf[(q * 16 + r1) * 17 + jj];
  dft_small<16, INV>(v);
  const uint64_t o = (j / Ns) * Ns * 256 + k;
#pragma unroll
  for (int b = 0; b < 16; ++b) out[o + (uint64_t)(q + 16 * b) * Ns] = v[b];
}

// Separate the two real inputs' spectra from Z = F(a + i r) and multiply:
// A[k] = (Z[k] + conj Z[-k]) / 2, R[k] = (Z[k] - conj Z[-k]) / (2i).  Thread
// k <= N/2 writes P[k] and P[N-k] in place.
__global__ __launch_bounds__(256) void k_fft_product(cplx* __restrict__ Z, uint64_t N) {
  const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (k > N / 2) return;
  const uint64_t kk = (N - k) & (N - 1);
  const cplx zk = Z[k], zc = Z[kk];
  auto prod = [](cplx p, cplx q) {  // p = Z[k], q = Z[-k]
    const cplx a = {0.5 * (p.x + q.x), 0.5 * (p.y - q.y)};
    const cplx r = {0.5 * (p.y + q.y), -0.5 * (p.x - q.x)};
    return cmul(a, r);
  };
  const cplx pk = prod(zk, zc);
  const cplx pc = prod(zc, zk);
  Z[k] = pk;
  if (kk != k) Z[kk] = pc;
}

// Rows t = n-1+i, i < m: v = Re(k'[t]) / N, bit i = rint(v) & 1, packed with
// wave ballots (64 rows per word); bits from m on are 0.  *err = the largest
// |v - rint(v)| as the bits of a non-negative double: one atomic per
// workgroup at most, and none when the value already there is as large (a
// single address takes every atomic, so they are kept rare).
__global__ __launch_bounds__(256) void k_fft_bits(const cplx* __restrict__ K, uint64_t N,
                                                  uint64_t n, uint64_t m,
                                                  uint64_t* __restrict__ y,
                                                  unsigned long long* err) {
  __shared__ double wmax[4];
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t words = (m + 63) / 64;
  uint32_t bit = 0;
  double d = 0.0;
  if (i < m) {
    const double v = K[n - 1 + i].x / (double)N;
    const double rv = rint(v);
    bit = (uint32_t)((long long)rv & 1);
    d = fabs(v - rv);
  }
  const uint64_t bal = __ballot(bit);
  if ((threadIdx.x & 63) == 0 && (i >> 6) < words) y[i >> 6] = bal;
  if (!err) return;
  for (int o = 32; o > 0; o >>= 1) d = fmax(d, __shfl_xor(d, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double b = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    const unsigned long long bb = (unsigned long long)__double_as_longlong(b);
    if (b > 0.0 && bb > __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(err, bb);
  }
}

// Transform of length N from a (pk non-null: from the packed bits, a being
// only scratch) ping-ponging with b; *result is the buffer holding the output.
template <bool INV>
hipError_t transform(cplx* a, cplx* b, uint64_t N, const PackedIn* pk, hipStream_t s,
                     cplx** result) {
  int log = 0;
  while ((1ull << log) < N) ++log;
  // the first pass reads the bits itself when it is the staged radix-16 one
  const bool fuse = pk && log % 4 == 0 && N >= 4096;
  if (pk && !fuse)
    hipLaunchKernelGGL(k_fft_pack, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, *pk, a, N);
  cplx* in = a;
  cplx* out = b;
  uint64_t Ns = 1;
  auto pass = [&](int R) {
    const uint64_t threads = N / (uint64_t)R;
    const dim3 grid((unsigned)((threads + 255) / 256));
    switch (R) {
      case 2: hipLaunchKernelGGL((k_fft_pass<2, INV>), grid, dim3(256), 0, s, in, out, N, Ns); break;
      case 4: hipLaunchKernelGGL((k_fft_pass<4, INV>), grid, dim3(256), 0, s, in, out, N, Ns); break;
      case 8: hipLaunchKernelGGL((k_fft_pass<8, INV>), grid, dim3(256), 0, s, in, out, N, Ns); break;
      case 16:
        if (Ns == 1 && N >= 4096 && fuse)
          hipLaunchKernelGGL((k_fft_first16<INV, true>), dim3((unsigned)(N / 4096)), dim3(256), 0,
                             s, in, out, N, *pk);
        else if (Ns == 1 && N >= 4096)
          hipLaunchKernelGGL((k_fft_first16<INV, false>), dim3((unsigned)(N / 4096)), dim3(256),
                             0, s, in, out, N, PackedIn{});
        else
          hipLaunchKernelGGL((k_fft_pass<16, INV>), grid, dim3(256), 0, s, in, out, N, Ns);
        break;
      default:  // 256: 16 consecutive j per workgroup
        hipLaunchKernelGGL((k_fft_pass256<INV>), dim3((unsigned)(N / 4096)), dim3(256), 0, s, in,
                           out, N, Ns);
    }
    Ns *= (uint64_t)R;
    cplx* t = in;
    in = out;
    out = t;
  };
  // radix 2/4/8 first when log2 N is not a multiple of 4, then radix 16 (so
  // that Ns >= 16), then radix 256 while 8 or more levels remain
  if (log % 4) pass(1 << (log % 4));
  int rem = log - log % 4;
  if (rem >= 4) {
    pass(16);
    rem -= 4;
  }
  for (; rem >= 8; rem -= 8) pass(256);
  if (rem == 4) pass(16);
  *result = in;
  return hipGetLastError();
}

}  // namespace

uint64_t fft64_length(uint64_t n, uint64_t m) {
  const uint64_t L = n + m - 1;
  uint64_t N = 16;
  while (N < L) N <<= 1;
  return N;
}

uint64_t fft64_work_words(uint64_t n, uint64_t m) { return 8 * fft64_length(n, m); }

hipError_t fft64_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits, uint64_t m,
                      uint64_t* y, unsigned long long* err, uint32_t* work, hipStream_t s) {
  const uint64_t N = fft64_length(n, m);
  if (N > FFT64_MAX_LENGTH) return hipErrorInvalidValue;
  cplx* A = reinterpret_cast<cplx*>(work);
  cplx* B = A + N;
  const PackedIn pk{seed_bits, n + m - 1, x_bits, n, err};
  prof_begin(KID_FFT64, s);
  cplx* Z = nullptr;
  hipError_t e = transform<false>(A, B, N, &pk, s, &Z);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fft_product, dim3((unsigned)((N / 2 + 1 + 255) / 256)), dim3(256), 0, s,
                       Z, N);
    cplx* other = Z == A ? B : A;
    cplx* K = nullptr;
    e = transform<true>(Z, other, N, nullptr, s, &K);
    if (e == hipSuccess)
      hipLaunchKernelGGL(k_fft_bits, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, K, N, n,
                         m, y, err);
  }
  prof_end(KID_FFT64, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace qrng

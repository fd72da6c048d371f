// Shared device helpers of the HIP library: Z_p arithmetic for the exact
// number-theoretic transform, and bit-layout helpers.
//
// Bit layout everywhere: bit b of a bit string is bit (b % 32) of the
// little-endian 32-bit word b / 32 (the same memory as LSB-first 64-bit words).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qrng {

// p = 119 * 2^23 + 1, generator 3: the multiplicative group has a cyclic
// subgroup of every order 2^k, k <= 23, so cyclic convolutions of any
// power-of-two length up to 2^23 are exact over Z_p.  A Toeplitz hash sum is
// an integer in [0, n]; it is recovered exactly whenever n < p.
constexpr uint32_t P = 998244353u;
constexpr uint32_t P2 = 2u * P;
constexpr uint32_t GEN = 3u;
constexpr int LOG_MAX = 23;

constexpr uint32_t cpow(uint64_t b, uint64_t e) {
  uint64_t r = 1;
  b %= P;
  while (e) {
    if (e & 1) r = r * b % P;
    b = b * b % P;
    e >>= 1;
  }
  return (uint32_t)r;
}
// primitive 2^logn-th root of unity
constexpr uint32_t croot(int logn) {
  return cpow(cpow(GEN, (P - 1) >> LOG_MAX), 1ull << (LOG_MAX - logn));
}
constexpr uint32_t cinv(uint32_t a) { return cpow(a, P - 2); }
// Shoup companion floor(w 2^32 / p)
constexpr uint32_t shoup_q(uint32_t w) { return (uint32_t)(((uint64_t)w << 32) / P); }
// -p^-1 mod 2^32 (Newton iteration on the 2-adic inverse)
constexpr uint32_t neg_pinv() {
  uint32_t x = P;
  for (int i = 0; i < 5; ++i) x *= 2u - P * x;
  return 0u - x;
}
constexpr uint32_t NPINV = neg_pinv();
constexpr uint32_t MONT_R = (uint32_t)((1ull << 32) % P);            // 2^32 mod p
constexpr uint32_t MONT_R2 = (uint32_t)((uint64_t)MONT_R * MONT_R % P);

static_assert(((uint64_t)P * (0u - NPINV)) % (1ull << 32) == 1, "pinv");
static_assert(cpow(croot(23), 1u << 22) == P - 1, "root of order 2^23");
static_assert(4ull * P < (1ull << 32), "lazy range [0, 4p) fits 32 bits");

// [0, 4p) -> [0, 2p): x - 2p wraps above x when x < 2p, so min picks x.
__device__ __forceinline__ uint32_t red2(uint32_t x) { return min(x, x - P2); }
// [0, 2p) -> [0, p)
__device__ __forceinline__ uint32_t red1(uint32_t x) { return min(x, x - P); }

// Shoup product: a * w mod p in [0, 2p) for any a < 2^32, w < p, wq = shoup_q(w).
__device__ __forceinline__ uint32_t mul_shoup(uint32_t a, uint32_t w, uint32_t wq) {
  uint32_t q = __umulhi(a, wq);
  return a * w - q * P;
}

// Montgomery product a b 2^-32 mod p in [0, 2p), valid for a b < 2^32 p.
__device__ __forceinline__ uint32_t mul_mont(uint32_t a, uint32_t b) {
  uint32_t lo = a * b;
  uint32_t hi = __umulhi(a, b);
  uint32_t mq = lo * NPINV;
  uint32_t mh = __umulhi(mq, P);
  return hi + mh + (lo != 0u);
}

// Montgomery product with a factor t fixed ahead of time: with
// tp = t (-p^-1) mod 2^32, the reduction multiplier (a t)(-p^-1) mod 2^32 is
// a tp mod 2^32, so a t 2^-32 mod p takes three multiplications instead of
// four.  (a t + m p) / 2^32 is exact; its low-word carry is 1 exactly when
// m != 0 (p is odd).  Result in [0, 2p) for a t < 2^32 p.
__device__ __forceinline__ uint32_t mont_pre(uint32_t t) { return t * NPINV; }
__device__ __forceinline__ uint32_t mul_mont_pre(uint32_t a, uint32_t t, uint32_t tp) {
  const uint32_t m = a * tp;
  return __umulhi(a, t) + __umulhi(m, P) + (m != 0u);
}

constexpr int ilog2(uint32_t v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }
constexpr uint32_t bitrev(uint32_t v, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1u) << (bits - 1 - i);
  return r;
}

// Constant twiddles of the register transforms: powers of the 16th root.
struct Tw16 {
  uint32_t w[16], wq[16], iw[16], iwq[16];
};
constexpr Tw16 make_tw16() {
  Tw16 t{};
  uint32_t r = croot(4), ir = cinv(croot(4));
  uint32_t a = 1, b = 1;
  for (int i = 0; i < 16; ++i) {
    t.w[i] = a;
    t.wq[i] = shoup_q(a);
    t.iw[i] = b;
    t.iwq[i] = shoup_q(b);
    a = (uint32_t)((uint64_t)a * r % P);
    b = (uint32_t)((uint64_t)b * ir % P);
  }
  return t;
}

// a - b mod p in [0, 2p) for a, b in [0, 2p): a - b wraps to a large value
// exactly when a < b, and then a - b + 2p is the one in range
__device__ __forceinline__ uint32_t sub2(uint32_t a, uint32_t b) {
  const uint32_t d = a - b;
  return min(d, d + P2);
}

// In-register transform of R = 2, 4, 8 or 16 values.
// Forward (INV = false): decimation in frequency, natural order in,
//   bit-reversed order out: v[a'] = sum_a v[a] w_R^(a * bitrev(a')).
// Inverse (INV = true): decimation in time, bit-reversed order in, natural
//   order out, with w^-1 and no 1/R factor (the exact inverse times R).
// Inputs in [0, 2p); outputs in [0, 2p), except with LAZY (forward only):
// outputs 1 .. R-1 are left in [0, 4p), for a caller that multiplies each of
// them by a twiddle next (a Shoup product takes any 32-bit input).  Inside
// the inverse, a value whose next use is a twiddle product is left in
// [0, 4p) for the same reason.
template <int R, bool INV, bool LAZY = false>
__device__ __forceinline__ void dft_reg(uint32_t (&v)[R]) {
  constexpr Tw16 T = make_tw16();
  static_assert(!(INV && LAZY), "lazy outputs are a forward-transform option");
  if constexpr (!INV) {
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (i & h) continue;
        const int j = i & (h - 1);       // i mod h
        const int e = j * (8 / h);       // w_{2h}^j = w_16^(j 16/(2h))
        const bool lazy = LAZY && h == 1;  // last stage: outputs go to a twiddle
        uint32_t a = v[i], b = v[i + h];
        v[i] = (lazy && i != 0) ? a + b : red2(a + b);
        if (j != 0)
          v[i + h] = mul_shoup(a + P2 - b, T.w[e], T.wq[e]);
        else
          v[i + h] = lazy ? a + P2 - b : sub2(a, b);
      }
    }
  } else {
#pragma unroll
    for (int h = 1; h <= R / 2; h <<= 1) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (i & h) continue;
        const int j = i & (h - 1);
        const int e = j * (8 / h);
        uint32_t u = v[i];
        uint32_t t = (j == 0) ? v[i + h] : mul_shoup(v[i + h], T.iw[e], T.iwq[e]);
        // output x feeds the next stage's twiddle product when that stage
        // exists (2h <= R/2) and x is a multiplied operand there
        const int H = 2 * h;
        const bool mi = H <= R / 2 && (i & H) && (i & (H - 1));
        const bool mh = H <= R / 2 && ((i + h) & H) && ((i + h) & (H - 1));
        v[i] = mi ? u + t : red2(u + t);
        v[i + h] = mh ? u + P2 - t : sub2(u, t);
      }
    }
  }
}

// Word i of a uniform base pointer, i < 2^30: the byte offset is formed in
// 32 bits, so the access takes the scalar-base, 32-bit-offset address form
// instead of 64-bit address arithmetic per lane.
__device__ __forceinline__ uint32_t ld_w32(const uint32_t* __restrict__ base, uint32_t i) {
  return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + (i << 2));
}
__device__ __forceinline__ void st_w32(uint32_t* __restrict__ base, uint32_t i, uint32_t v) {
  *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) + (i << 2)) = v;
}

// bit b of a 32-bit-word bit string (caller guarantees the word exists)
__device__ __forceinline__ uint32_t get_bit(const uint32_t* __restrict__ w, uint64_t b) {
  return (w[b >> 5] >> (b & 31)) & 1u;
}

}  // namespace qrng

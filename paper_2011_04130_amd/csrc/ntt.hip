// Exact Toeplitz hashing through a number-theoretic transform (NTT) over
// Z_p, p = 998244353 (paper Sec. III.B: the circulant embedding and the
// convolution theorem, Theorems 1-2; here over Z_p instead of floating point,
// so no rounding step exists and the result is exact).
//
// With x zero-padded to the transform length Nc and the seed laid out as the
// window  w[q] = s[n-1+q] (q < h), w[q] = s[n-1+q-Nc] (q >= h)  (bits outside
// the seed are 0), the cyclic convolution (w * x)[t] equals row t of T x for
// every t < m, as long as Nc >= n+m-1: the needed seed offsets t-j lie in
// [-(n-1), m-1], an interval of length n+m-1 that the cyclic layout never
// folds onto itself.  Every row sum is an integer in [0, n] < p, so reducing
// the NTT result mod p and taking the low bit gives the hash bit (the paper's
// "round off and mod 2" step becomes an exact "& 1").
//
// Lengths above 2^23 (the largest power of two dividing p-1) are handled as a
// block Toeplitz product: x and y are cut into chunks of B = 2^22 bits, chunk
// pair (o, c) is a Toeplitz block whose seed window depends only on d = o - c,
// and y_o = sum_c T_{o-c} x_c is accumulated in the transform domain before a
// single inverse transform per output chunk.
//
// Transform structure (MI355X): Nc = N1 * N2 four-step.  Pass A transforms
// the N1-long columns (32 adjacent columns per workgroup: every LDS access of
// a half-wave is 32 consecutive words) and applies the w_Nc^(j2 k1) twiddle;
// pass B transforms each N2-long row, multiplies by the cached seed spectrum
// and runs the inverse row transform without leaving registers/LDS; pass C
// runs the inverse column transform and packs output bits with wave ballots.
// For Nc <= 2^14 a single fused kernel does everything from raw bits to hash
// bits.  Sub-transforms are radix-16 (radix-2/4/8 first round) register
// butterflies with LDS exchanges between rounds.  The forward transform uses
// decimation in frequency (natural order in, bit-reversed out) and the
// inverse decimation in time (bit-reversed in, natural out), so no permutation
// pass is ever needed: both operands of the pointwise product are in the same
// bit-reversed order.  Residues stay in [0, 2p) (lazy reduction); twiddles
// from tables use Shoup products, generated ones Montgomery products.
#include <utility>

#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

constexpr int MAX_LOG_SUB = 14;  // longest in-LDS sub-transform

// Offset of the (sub-length 2^lgR, radix 2^lgr) twiddle table.
constexpr int tw_off(int lgR, int lgr) {
  int off = 0;
  for (int l = 1; l < lgR; ++l) off += (1 << l) * (l < 4 ? l : 4);
  return off + (lgr - 1) * (1 << lgR);
}
constexpr int TW_TOTAL = tw_off(MAX_LOG_SUB + 1, 1);

// Round structure of a 2^LOG transform: a radix-2^(LOG%4) first round when
// LOG is not a multiple of 4, radix 16 after that.
template <int LOG>
struct RP {
  static constexpr int K = (LOG + 3) / 4;
  static constexpr int lgr(int k) { return (k == 0 && (LOG % 4) != 0) ? (LOG % 4) : 4; }
  static constexpr int lgR(int k) {
    int l = LOG;
    for (int i = 0; i < k; ++i) l -= lgr(i);
    return l;
  }
};

// Round k works on sub-arrays of length R = r * s; group g = (sub, b) owns the
// r elements sub*R + a*s + b.
template <int LOG, int k>
struct Geo {
  static constexpr int lgr = RP<LOG>::lgr(k), r = 1 << lgr;
  static constexpr int lgR = RP<LOG>::lgR(k), R = 1 << lgR;
  static constexpr int s = R / r;
  static constexpr int groups = (1 << LOG) / r;
  static constexpr int toff = tw_off(lgR, lgr);
  __device__ static __forceinline__ int pos(int g, int a) {
    return (g / s) * R + a * s + (g % s);
  }
};

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}
// E-1 down to B
template <int B, int E, class F>
__device__ __forceinline__ void static_for_down(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, E - 1>{});
    static_for_down<B, E - 1>(f);
  }
}

// Forward round on group g: load, radix-r DIF, twiddle w_R^(b bitrev(a')), store.
template <int LOG, int k, class LD, class ST>
__device__ __forceinline__ void fwd_group(int g, const uint2* __restrict__ twf, LD&& ld,
                                          ST&& st) {
  using G = Geo<LOG, k>;
  uint32_t v[G::r];
#pragma unroll
  for (int a = 0; a < G::r; ++a) v[a] = ld(G::pos(g, a));
  dft_reg<G::r, false>(v);
  if constexpr (G::s > 1) {
    const uint2* T = twf + G::toff + (g % G::s) * G::r;
#pragma unroll
    for (int a = 1; a < G::r; ++a) {
      uint2 t = T[a];
      v[a] = mul_shoup(v[a], t.x, t.y);
    }
  }
#pragma unroll
  for (int a = 0; a < G::r; ++a) st(G::pos(g, a), v[a]);
}

// Inverse round on group g: load, twiddle w_R^-(b bitrev(a')), radix-r DIT, store.
template <int LOG, int k, class LD, class ST>
__device__ __forceinline__ void inv_group(int g, const uint2* __restrict__ twi, LD&& ld,
                                          ST&& st) {
  using G = Geo<LOG, k>;
  uint32_t v[G::r];
#pragma unroll
  for (int a = 0; a < G::r; ++a) v[a] = ld(G::pos(g, a));
  if constexpr (G::s > 1) {
    const uint2* T = twi + G::toff + (g % G::s) * G::r;
#pragma unroll
    for (int a = 1; a < G::r; ++a) {
      uint2 t = T[a];
      v[a] = mul_shoup(v[a], t.x, t.y);
    }
  }
  dft_reg<G::r, true>(v);
#pragma unroll
  for (int a = 0; a < G::r; ++a) st(G::pos(g, a), v[a]);
}

// w_{2^23}^e in Montgomery form
__device__ __forceinline__ uint32_t gtw(const TwTables& tw, uint32_t e) {
  return mul_mont(tw.g_hi[e >> 12], tw.g_lo[e & 4095u]);
}

template <int LOG>
__device__ __forceinline__ int brev(int p) {
  return (int)(__builtin_bitreverse32((uint32_t)p) >> (32 - LOG));
}

// Transform position q of an item maps to bit off + (q < h ? q : q - Nc) of
// the source, or to 0 when that index falls outside [lo, hi).
struct BitMap {
  int64_t off, lo, hi, h;
};
constexpr int MAXMAP = 8;

__device__ __forceinline__ uint32_t map_bit(const uint32_t* __restrict__ bits, const BitMap& mp,
                                            int64_t q, int64_t Nc, uint64_t zo) {
  int64_t k = q < mp.h ? q : q - Nc;
  int64_t idx = mp.off + k;
  if (idx < mp.lo || idx >= mp.hi) return 0u;
  return get_bit(bits, (uint64_t)idx + zo);
}

// ----------------------------------------------------------------- pass A
struct ColFwdArgs {
  const uint32_t* bits;
  uint64_t zs;  // batch stride of the bit source
  BitMap map[MAXMAP];
  int nmap;
  int log2, log_nc;
  uint32_t* out;  // item y = blockIdx.y at out + y * Nc
};

constexpr int COLS = 32;   // columns per workgroup
constexpr int CSLOTS = 8;  // 256 threads = 32 columns x 8 slots

template <int LOG1>
__global__ __launch_bounds__(256) void k_cols_fwd(ColFwdArgs a, TwTables tw) {
  __shared__ uint32_t lds[(1 << LOG1) * COLS];
  const int c = threadIdx.x & (COLS - 1), slot = threadIdx.x >> 5;
  const int64_t Nc = (int64_t)1 << a.log_nc;
  const int j2 = blockIdx.x * COLS + c;
  const int mi = blockIdx.y % a.nmap;
  const uint64_t zo = (uint64_t)(blockIdx.y / a.nmap) * a.zs;
  const BitMap mp = a.map[mi];
  uint32_t* __restrict__ out = a.out + (uint64_t)blockIdx.y * Nc;
  const uint32_t gstep = (uint32_t)j2 << (LOG_MAX - a.log_nc);

  auto ld_bits = [&](int j1) -> uint32_t {
    return map_bit(a.bits, mp, ((int64_t)j1 << a.log2) + j2, Nc, zo);
  };
  auto ld_lds = [&](int j1) -> uint32_t { return lds[j1 * COLS + c]; };
  auto st_lds = [&](int j1, uint32_t v) { lds[j1 * COLS + c] = v; };
  auto st_out = [&](int p, uint32_t v) {
    uint32_t e = gstep * (uint32_t)brev<LOG1>(p);
    out[((int64_t)p << a.log2) + j2] = mul_mont(v, gtw(tw, e));
  };
  constexpr int K = RP<LOG1>::K;
  static_for<0, K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    using G = Geo<LOG1, k>;
    for (int g = slot; g < G::groups; g += CSLOTS) {
      if constexpr (K == 1)
        fwd_group<LOG1, k>(g, tw.fwd, ld_bits, st_out);
      else if constexpr (k == 0)
        fwd_group<LOG1, k>(g, tw.fwd, ld_bits, st_lds);
      else if constexpr (k == K - 1)
        fwd_group<LOG1, k>(g, tw.fwd, ld_lds, st_out);
      else
        fwd_group<LOG1, k>(g, tw.fwd, ld_lds, st_lds);
    }
    if constexpr (k < K - 1) __syncthreads();
  });
}

// ----------------------------------------------------------------- pass C
struct ColInvArgs {
  const uint32_t* in;  // item y = blockIdx.y at in + y * Nc
  int ny, log2, log_nc;
  uint32_t* y;    // output bits
  uint64_t y_zs;  // batch stride of the output (bits, multiple of 64)
  int64_t by;     // output chunk length
  uint64_t m;
};

template <int LOG1>
__global__ __launch_bounds__(256) void k_cols_inv(ColInvArgs a, TwTables tw) {
  __shared__ uint32_t lds[(1 << LOG1) * COLS];
  const int c = threadIdx.x & (COLS - 1), slot = threadIdx.x >> 5;
  const int lane = threadIdx.x & 63;
  const int64_t Nc = (int64_t)1 << a.log_nc;
  const int j2 = blockIdx.x * COLS + c;
  const int o = blockIdx.y % a.ny;
  const uint64_t ybase = (uint64_t)(blockIdx.y / a.ny) * a.y_zs + (uint64_t)o * a.by;
  const int64_t rem = (int64_t)a.m - (int64_t)o * a.by;
  const int64_t yvalid = rem < a.by ? rem : a.by;
  const int64_t ylimit = (yvalid + 63) & ~(int64_t)63;
  const uint32_t* __restrict__ in = a.in + (uint64_t)blockIdx.y * Nc;
  const uint32_t gstep = (uint32_t)j2 << (LOG_MAX - a.log_nc);
  constexpr uint32_t EMASK = (1u << LOG_MAX) - 1;

  auto ld_in = [&](int p) -> uint32_t {
    uint32_t e = (0u - gstep * (uint32_t)brev<LOG1>(p)) & EMASK;
    return mul_mont(in[((int64_t)p << a.log2) + j2], gtw(tw, e));
  };
  auto ld_lds = [&](int j1) -> uint32_t { return lds[j1 * COLS + c]; };
  auto st_lds = [&](int j1, uint32_t v) { lds[j1 * COLS + c] = v; };
  auto st_bits = [&](int j1, uint32_t v) {
    const int64_t t = ((int64_t)j1 << a.log2) + j2;
    const uint32_t bit = (t < yvalid) ? (red1(v) & 1u) : 0u;
    const uint64_t bal = __ballot(bit);
    const int64_t t0 = t - c;  // first column of this half-wave
    if ((lane & 31) == 0 && t0 < ylimit)
      a.y[(ybase + (uint64_t)t0) >> 5] = lane ? (uint32_t)(bal >> 32) : (uint32_t)bal;
  };
  constexpr int K = RP<LOG1>::K;
  static_for_down<0, K>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    using G = Geo<LOG1, k>;
    for (int g = slot; g < G::groups; g += CSLOTS) {
      if constexpr (K == 1)
        inv_group<LOG1, k>(g, tw.inv, ld_in, st_bits);
      else if constexpr (k == K - 1)
        inv_group<LOG1, k>(g, tw.inv, ld_in, st_lds);
      else if constexpr (k == 0)
        inv_group<LOG1, k>(g, tw.inv, ld_lds, st_bits);
      else
        inv_group<LOG1, k>(g, tw.inv, ld_lds, st_lds);
    }
    if constexpr (k > 0) __syncthreads();
  });
}

// ----------------------------------------------------------------- pass B
struct RowArgs {
  const uint32_t* in;  // residues (pass-A output); item at in + item * Nc + row * N2
  const uint32_t* bits;
  uint64_t zs;  // batch stride of the bit source (fused)
  BitMap map[MAXMAP];
  const uint32_t* W;  // seed spectra, window w at W + w * Nc
  int nx, ny, log_nc;
  uint32_t cw;    // seed mode: Nc^-1 2^64 mod p
  uint32_t* out;  // residues out (item * Nc + row * N2) or seed spectra
  uint32_t* y;    // output bits (fused)
  uint64_t y_zs;
  uint64_t m;
};

// One row of the four-step (or the whole transform when N1 = 1).
//  SEED:  forward transform of a seed window -> Montgomery-form spectrum row.
//  hash:  forward transforms of NX raw chunks, products with the seed
//         spectra summed per output chunk, inverse transform per output chunk.
// IN_BITS / OUT_BITS: the row is the whole transform and reads raw bits /
// writes hash bits directly.
template <int LOG2, int NX, bool IN_BITS, bool SEED, bool OUT_BITS>
__global__ __launch_bounds__((1 << LOG2) / 16) void k_rows(RowArgs a, TwTables tw) {
  constexpr int N2 = 1 << LOG2, T = N2 / 16, K = RP<LOG2>::K;
  static_assert(K >= 2, "rows are at least 2^5 long");
  static_assert(Geo<LOG2, K - 1>::r == 16 && Geo<LOG2, K - 1>::s == 1, "last round");
  __shared__ uint32_t lds[N2 + N2 / 16];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int row = blockIdx.x;
  const int zy = blockIdx.y;
  const int64_t Nc = (int64_t)1 << a.log_nc;

  auto ld_lds = [&](int i) -> uint32_t { return lds[i + (i >> 4)]; };
  auto st_lds = [&](int i, uint32_t v) { lds[i + (i >> 4)] = v; };

  uint32_t xs[NX][16];
  static_for<0, NX>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    const int item = SEED ? zy : zy * NX + c;
    if constexpr (IN_BITS) {
      const BitMap mp = a.map[SEED ? zy : c];
      const uint64_t zo = SEED ? 0 : (uint64_t)zy * a.zs;
      auto ld0 = [&](int q) -> uint32_t { return map_bit(a.bits, mp, q, Nc, zo); };
      for (int g = tid; g < Geo<LOG2, 0>::groups; g += T)
        fwd_group<LOG2, 0>(g, tw.fwd, ld0, st_lds);
    } else {
      const uint32_t* __restrict__ src = a.in + (uint64_t)item * Nc + (uint64_t)row * N2;
      auto ld0 = [&](int i) -> uint32_t { return src[i]; };
      for (int g = tid; g < Geo<LOG2, 0>::groups; g += T)
        fwd_group<LOG2, 0>(g, tw.fwd, ld0, st_lds);
    }
    __syncthreads();
    static_for<1, K - 1>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      for (int g = tid; g < Geo<LOG2, k>::groups; g += T)
        fwd_group<LOG2, k>(g, tw.fwd, ld_lds, st_lds);
      __syncthreads();
    });
#pragma unroll
    for (int e = 0; e < 16; ++e) xs[c][e] = ld_lds(tid * 16 + e);
    dft_reg<16, false>(xs[c]);
    __syncthreads();
  });

  if constexpr (SEED) {
    uint32_t* dst = a.out + (uint64_t)zy * Nc + (uint64_t)row * N2 + tid * 16;
#pragma unroll
    for (int e = 0; e < 16; e += 4) {
      uint4 w;
      w.x = red1(mul_mont(xs[0][e + 0], a.cw));
      w.y = red1(mul_mont(xs[0][e + 1], a.cw));
      w.z = red1(mul_mont(xs[0][e + 2], a.cw));
      w.w = red1(mul_mont(xs[0][e + 3], a.cw));
      *reinterpret_cast<uint4*>(dst + e) = w;
    }
    return;
  } else {
    for (int o = 0; o < a.ny; ++o) {
      uint32_t acc[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e] = 0;
      static_for<0, NX>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const uint32_t* wr =
            a.W + (uint64_t)(o - c + NX - 1) * Nc + (uint64_t)row * N2 + tid * 16;
#pragma unroll
        for (int e = 0; e < 16; e += 4) {
          uint4 w = *reinterpret_cast<const uint4*>(wr + e);
          acc[e + 0] = red2(acc[e + 0] + mul_mont(xs[c][e + 0], w.x));
          acc[e + 1] = red2(acc[e + 1] + mul_mont(xs[c][e + 1], w.y));
          acc[e + 2] = red2(acc[e + 2] + mul_mont(xs[c][e + 2], w.z));
          acc[e + 3] = red2(acc[e + 3] + mul_mont(xs[c][e + 3], w.w));
        }
      });
      dft_reg<16, true>(acc);
#pragma unroll
      for (int e = 0; e < 16; ++e) st_lds(tid * 16 + e, acc[e]);
      __syncthreads();
      static_for_down<1, K - 1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        for (int g = tid; g < Geo<LOG2, k>::groups; g += T)
          inv_group<LOG2, k>(g, tw.inv, ld_lds, st_lds);
        __syncthreads();
      });
      if constexpr (OUT_BITS) {
        // the row is the whole transform: position q is output bit q
        const uint64_t ybase = (uint64_t)zy * a.y_zs;
        const int64_t yvalid = (int64_t)a.m;
        const int64_t ylimit = (yvalid + 63) & ~(int64_t)63;
        uint64_t* y64 = reinterpret_cast<uint64_t*>(a.y);
        auto st_bits = [&](int q, uint32_t v) {
          const uint32_t bit = (q < yvalid) ? (red1(v) & 1u) : 0u;
          const uint64_t bal = __ballot(bit);
          const int64_t q0 = q - lane;
          if (lane == 0 && q0 < ylimit) y64[(ybase + (uint64_t)q0) >> 6] = bal;
        };
        for (int g = tid; g < Geo<LOG2, 0>::groups; g += T)
          inv_group<LOG2, 0>(g, tw.inv, ld_lds, st_bits);
      } else {
        uint32_t* dst = a.out + (uint64_t)(zy * a.ny + o) * Nc + (uint64_t)row * N2;
        auto st0 = [&](int i, uint32_t v) { dst[i] = v; };
        for (int g = tid; g < Geo<LOG2, 0>::groups; g += T)
          inv_group<LOG2, 0>(g, tw.inv, ld_lds, st0);
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ dispatch
template <int LOG1>
hipError_t launch_cols_fwd(const ColFwdArgs& a, dim3 grid, const TwTables& tw, hipStream_t s) {
  prof_begin(KID_COLS_FWD, s);
  hipLaunchKernelGGL(k_cols_fwd<LOG1>, grid, dim3(256), 0, s, a, tw);
  prof_end(KID_COLS_FWD, s);
  return hipGetLastError();
}
template <int LOG1>
hipError_t launch_cols_inv(const ColInvArgs& a, dim3 grid, const TwTables& tw, hipStream_t s) {
  prof_begin(KID_COLS_INV, s);
  hipLaunchKernelGGL(k_cols_inv<LOG1>, grid, dim3(256), 0, s, a, tw);
  prof_end(KID_COLS_INV, s);
  return hipGetLastError();
}

hipError_t cols_fwd(int log1, const ColFwdArgs& a, dim3 grid, const TwTables& tw,
                    hipStream_t s) {
  switch (log1) {
    case 1: return launch_cols_fwd<1>(a, grid, tw, s);
    case 2: return launch_cols_fwd<2>(a, grid, tw, s);
    case 3: return launch_cols_fwd<3>(a, grid, tw, s);
    case 4: return launch_cols_fwd<4>(a, grid, tw, s);
    case 5: return launch_cols_fwd<5>(a, grid, tw, s);
    case 6: return launch_cols_fwd<6>(a, grid, tw, s);
    case 7: return launch_cols_fwd<7>(a, grid, tw, s);
    case 8: return launch_cols_fwd<8>(a, grid, tw, s);
    case 9: return launch_cols_fwd<9>(a, grid, tw, s);
  }
  return hipErrorInvalidValue;
}
hipError_t cols_inv(int log1, const ColInvArgs& a, dim3 grid, const TwTables& tw,
                    hipStream_t s) {
  switch (log1) {
    case 1: return launch_cols_inv<1>(a, grid, tw, s);
    case 2: return launch_cols_inv<2>(a, grid, tw, s);
    case 3: return launch_cols_inv<3>(a, grid, tw, s);
    case 4: return launch_cols_inv<4>(a, grid, tw, s);
    case 5: return launch_cols_inv<5>(a, grid, tw, s);
    case 6: return launch_cols_inv<6>(a, grid, tw, s);
    case 7: return launch_cols_inv<7>(a, grid, tw, s);
    case 8: return launch_cols_inv<8>(a, grid, tw, s);
    case 9: return launch_cols_inv<9>(a, grid, tw, s);
  }
  return hipErrorInvalidValue;
}

template <int LOG2, int NX, bool IN_BITS, bool SEED, bool OUT_BITS>
hipError_t launch_rows(const RowArgs& a, dim3 grid, const TwTables& tw, hipStream_t s) {
  constexpr int kid = IN_BITS ? (SEED ? KID_FUSED_SEED : KID_FUSED_HASH)
                              : (SEED ? KID_ROWS_SEED : KID_ROWS_HASH);
  prof_begin(kid, s);
  hipLaunchKernelGGL((k_rows<LOG2, NX, IN_BITS, SEED, OUT_BITS>), grid, dim3((1 << LOG2) / 16),
                     0, s, a, tw);
  prof_end(kid, s);
  return hipGetLastError();
}

template <int NX, bool IN_BITS, bool SEED, bool OUT_BITS>
hipError_t rows_l(int log2, const RowArgs& a, dim3 grid, const TwTables& tw, hipStream_t s) {
  switch (log2) {
    case 10: return launch_rows<10, NX, IN_BITS, SEED, OUT_BITS>(a, grid, tw, s);
    case 11: return launch_rows<11, NX, IN_BITS, SEED, OUT_BITS>(a, grid, tw, s);
    case 12: return launch_rows<12, NX, IN_BITS, SEED, OUT_BITS>(a, grid, tw, s);
    case 13: return launch_rows<13, NX, IN_BITS, SEED, OUT_BITS>(a, grid, tw, s);
    case 14: return launch_rows<14, NX, IN_BITS, SEED, OUT_BITS>(a, grid, tw, s);
  }
  return hipErrorInvalidValue;
}

uint32_t host_pow(uint64_t b, uint64_t e) {
  uint64_t r = 1;
  b %= P;
  while (e) {
    if (e & 1) r = r * b % P;
    b = b * b % P;
    e >>= 1;
  }
  return (uint32_t)r;
}
uint32_t host_root(int logn) { return host_pow(host_pow(GEN, (P - 1) >> LOG_MAX), 1ull << (LOG_MAX - logn)); }
uint32_t host_mont(uint32_t v) { return (uint32_t)(((uint64_t)v << 32) % P); }
uint32_t host_bitrev(uint32_t v, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1u) << (bits - 1 - i);
  return r;
}
int ceil_log2(uint64_t v) {
  int k = 0;
  while ((1ull << k) < v) ++k;
  return k;
}

}  // namespace

// ------------------------------------------------------------ host side
int tw_total_entries() { return TW_TOTAL; }

void build_tw_tables(uint2* fwd, uint2* inv, uint32_t* g_lo, uint32_t* g_hi) {
  for (int lgR = 1; lgR <= MAX_LOG_SUB; ++lgR) {
    const uint32_t R = 1u << lgR;
    const uint32_t w = host_root(lgR), iw = host_pow(w, P - 2);
    for (int lgr = 1; lgr <= 4 && lgr <= lgR; ++lgr) {
      const uint32_t r = 1u << lgr, s = R / r;
      const int off = tw_off(lgR, lgr);
      for (uint32_t b = 0; b < s; ++b)
        for (uint32_t ap = 0; ap < r; ++ap) {
          const uint64_t e = (uint64_t)b * host_bitrev(ap, lgr) % R;
          const uint32_t f = host_pow(w, e), g = host_pow(iw, e);
          fwd[off + b * r + ap] = make_uint2(f, shoup_q(f));
          inv[off + b * r + ap] = make_uint2(g, shoup_q(g));
        }
    }
  }
  const uint32_t w23 = host_root(LOG_MAX);
  uint32_t t = 1;
  for (int j = 0; j < 4096; ++j) {
    g_lo[j] = host_mont(t);
    t = (uint32_t)((uint64_t)t * w23 % P);
  }
  const uint32_t w4096 = host_pow(w23, 4096);
  t = 1;
  for (int j = 0; j < 2048; ++j) {
    g_hi[j] = host_mont(t);
    t = (uint32_t)((uint64_t)t * w4096 % P);
  }
}

bool ntt_make_plan(uint64_t n, uint64_t m, NttPlan* p) {
  if (n == 0 || m == 0 || m > n || n >= P) return false;
  const uint64_t L = n + m - 1;
  if (L <= (1ull << LOG_MAX)) {
    p->log_nc = ceil_log2(L) < 10 ? 10 : ceil_log2(L);
    p->nx = p->ny = 1;
    p->bx = (int64_t)n;
    p->by = (int64_t)m;
  } else {
    const int64_t B = (int64_t)1 << (LOG_MAX - 1);
    p->log_nc = LOG_MAX;
    p->nx = (int)((n + B - 1) / B);
    p->ny = (int)((m + B - 1) / B);
    p->bx = p->by = B;
    if (p->nx > 4) return false;  // registers hold at most 4 raw chunks per row
  }
  const int k = p->log_nc;
  if (k <= MAX_LOG_SUB) {
    p->log1 = 0;
    p->log2 = k;
  } else {
    int l2 = k - 9;
    l2 = l2 < 10 ? 10 : (l2 > MAX_LOG_SUB ? MAX_LOG_SUB : l2);
    p->log2 = l2;
    p->log1 = k - l2;
  }
  p->nwin = p->nx + p->ny - 1;
  return true;
}

uint64_t ntt_seed_elems(const NttPlan& p) { return (uint64_t)p.nwin << p.log_nc; }

uint64_t ntt_work_elems(const NttPlan& p, int batch) {
  if (p.log1 == 0) return 0;
  return (uint64_t)batch * (uint64_t)(p.nx + p.ny) << p.log_nc;
}

hipError_t ntt_seed_spectra(const NttPlan& p, const uint32_t* seed_bits, uint64_t n,
                            uint64_t m, uint32_t* W, uint32_t* work, const TwTables& tw,
                            hipStream_t s) {
  const uint64_t L = n + m - 1;
  const int64_t Nc = (int64_t)1 << p.log_nc;
  if (p.nwin > MAXMAP) return hipErrorInvalidValue;
  BitMap maps[MAXMAP];
  for (int w = 0; w < p.nwin; ++w) {
    const int64_t d = w - (p.nx - 1);
    maps[w] = BitMap{(int64_t)n - 1 + d * p.by, 0, (int64_t)L, p.by};
  }
  const uint32_t cw = (uint32_t)((uint64_t)host_pow(Nc % P, P - 2) * host_mont(host_mont(1)) % P);
  RowArgs r{};
  r.bits = seed_bits;
  r.zs = 0;
  for (int w = 0; w < p.nwin; ++w) r.map[w] = maps[w];
  r.nx = 1;
  r.ny = 1;
  r.log_nc = p.log_nc;
  r.cw = cw;
  r.out = W;
  if (p.log1 == 0) {
    return rows_l<1, true, true, false>(p.log2, r, dim3(1, p.nwin), tw, s);
  }
  ColFwdArgs c{};
  c.bits = seed_bits;
  c.zs = 0;
  for (int w = 0; w < p.nwin; ++w) c.map[w] = maps[w];
  c.nmap = p.nwin;
  c.log2 = p.log2;
  c.log_nc = p.log_nc;
  c.out = work;
  hipError_t e = cols_fwd(p.log1, c, dim3((1u << p.log2) / COLS, p.nwin), tw, s);
  if (e != hipSuccess) return e;
  r.in = work;
  return rows_l<1, false, true, false>(p.log2, r, dim3(1u << p.log1, p.nwin), tw, s);
}

hipError_t ntt_hash(const NttPlan& p, const uint32_t* x_bits, uint64_t n, uint64_t m,
                    const uint32_t* W, uint32_t* y_bits, uint32_t* work, int batch,
                    uint64_t x_stride_bits, uint64_t y_stride_bits, const TwTables& tw,
                    hipStream_t s) {
  const int64_t Nc = (int64_t)1 << p.log_nc;
  RowArgs r{};
  r.W = W;
  r.nx = p.nx;
  r.ny = p.ny;
  r.log_nc = p.log_nc;
  r.y = y_bits;
  r.y_zs = y_stride_bits;
  r.m = m;
  if (p.log1 == 0) {
    r.bits = x_bits;
    r.zs = x_stride_bits;
    r.map[0] = BitMap{0, 0, (int64_t)n, Nc};
    return rows_l<1, true, false, true>(p.log2, r, dim3(1, batch), tw, s);
  }
  uint32_t* X = work;
  uint32_t* Z = work + ((uint64_t)batch * p.nx << p.log_nc);
  ColFwdArgs c{};
  c.bits = x_bits;
  c.zs = x_stride_bits;
  for (int k = 0; k < p.nx; ++k) {
    const int64_t lo = (int64_t)k * p.bx;
    const int64_t hi = lo + p.bx < (int64_t)n ? lo + p.bx : (int64_t)n;
    c.map[k] = BitMap{lo, lo, hi, Nc};
  }
  c.nmap = p.nx;
  c.log2 = p.log2;
  c.log_nc = p.log_nc;
  c.out = X;
  hipError_t e = cols_fwd(p.log1, c, dim3((1u << p.log2) / COLS, batch * p.nx), tw, s);
  if (e != hipSuccess) return e;
  r.in = X;
  r.out = Z;
  const dim3 rg(1u << p.log1, batch);
  switch (p.nx) {
    case 1: e = rows_l<1, false, false, false>(p.log2, r, rg, tw, s); break;
    case 2: e = rows_l<2, false, false, false>(p.log2, r, rg, tw, s); break;
    case 3: e = rows_l<3, false, false, false>(p.log2, r, rg, tw, s); break;
    case 4: e = rows_l<4, false, false, false>(p.log2, r, rg, tw, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  ColInvArgs ci{};
  ci.in = Z;
  ci.ny = p.ny;
  ci.log2 = p.log2;
  ci.log_nc = p.log_nc;
  ci.y = y_bits;
  ci.y_zs = y_stride_bits;
  ci.by = p.by;
  ci.m = m;
  return cols_inv(p.log1, ci, dim3((1u << p.log2) / COLS, batch * p.ny), tw, s);
}

}  // namespace qrng

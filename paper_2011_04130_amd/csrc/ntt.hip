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
// For Nc <= 2^15 a single fused kernel does everything from raw bits to hash
// bits.  Sub-transforms are radix-16 (radix-2/4/8 first round) register
// butterflies with LDS exchanges between rounds.  The forward transform uses
// decimation in frequency (natural order in, bit-reversed out) and the
// inverse decimation in time (bit-reversed in, natural out), so no permutation
// pass is ever needed: both operands of the pointwise product are in the same
// bit-reversed order.  Residues stay in [0, 2p) (lazy reduction); twiddles
// from tables use Shoup products, generated ones Montgomery products.
#include <utility>

#include <cstring>

#include "common.h"
#include "hist_dev.h"
#include "internal.h"

namespace qrng {

namespace {

constexpr int MAX_LOG_SUB = 15;    // longest in-LDS sub-transform (tables cover it)
constexpr int MAX_LOG_ROW = 14;    // longest four-step row (two rows share one CU's LDS)
constexpr int MAX_LOG_FUSED = 15;  // longest transform done whole by one workgroup

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
// r elements sub*R + a*s + b, a < r.
template <int LOG, int k>
struct Geo {
  static constexpr int lgr = RP<LOG>::lgr(k), r = 1 << lgr;
  static constexpr int lgR = RP<LOG>::lgR(k), R = 1 << lgR;
  static constexpr int s = R / r;
  static constexpr int groups = (1 << LOG) / r;
  static constexpr int toff = tw_off(lgR, lgr);
  // stride between consecutive a in the padded row layout (one pad word per
  // 16): linear because every round of a row has s == 1 or s % 16 == 0
  static constexpr int SP = s >= 16 ? s + s / 16 : 1;
  __device__ static __forceinline__ int pos0(int g) { return (g / s) * R + (g % s); }
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

// The r twiddles of one group as 16-byte loads (tables are 16-byte aligned:
// every table offset and group stride is an even number of entries).
template <int R>
__device__ __forceinline__ void load_tw(const uint2* __restrict__ T, uint2 (&t)[R]) {
  const uint4* T4 = reinterpret_cast<const uint4*>(T);
#pragma unroll
  for (int i = 0; i < R / 2; ++i) {
    const uint4 q = T4[i];
    t[2 * i] = make_uint2(q.x, q.y);
    t[2 * i + 1] = make_uint2(q.z, q.w);
  }
}

// One round on GPT groups g0 + u*gstep.  All loads are issued before any
// butterfly and all stores after, so the groups' arithmetic interleaves and
// hides load latency.  Forward: radix-r DIF then twiddle w_R^(b bitrev(a'));
// inverse: twiddle w_R^-(b bitrev(a')) then radix-r DIT.
// ld(g, a) / st(g, a, v) address element a of group g.
// TP: the tables in transposed order (entry (b, a) at a * s + b), so lanes
// that hold consecutive groups b read consecutive entries.
template <int R, int S, bool TP>
__device__ __forceinline__ void group_tw(const uint2* __restrict__ T, int b, uint2 (&t)[R]) {
  if constexpr (TP) {
#pragma unroll
    for (int a = 1; a < R; ++a) t[a] = T[a * S + b];
  } else {
    load_tw<R>(T + b * R, t);
  }
}

template <int LOG, int k, int GPT, bool INV, bool TP, class LD, class ST>
__device__ __forceinline__ void round_multi(int g0, int gstep, const uint2* __restrict__ tws,
                                            LD&& ld, ST&& st) {
  using G = Geo<LOG, k>;
  uint32_t v[GPT][G::r];
#pragma unroll
  for (int u = 0; u < GPT; ++u)
#pragma unroll
    for (int a = 0; a < G::r; ++a) v[u][a] = ld(g0 + u * gstep, a);
#pragma unroll
  for (int u = 0; u < GPT; ++u) {
    if constexpr (INV) {
      if constexpr (G::s > 1) {
        uint2 t[G::r];
        group_tw<G::r, G::s, TP>(tws + G::toff, (g0 + u * gstep) % G::s, t);
#pragma unroll
        for (int a = 1; a < G::r; ++a) v[u][a] = mul_shoup(v[u][a], t[a].x, t[a].y);
      }
      dft_reg<G::r, true>(v[u]);
    } else {
      // with twiddles to follow, outputs 1 .. r-1 may stay in [0, 4p)
      dft_reg<G::r, false, (G::s > 1)>(v[u]);
      if constexpr (G::s > 1) {
        uint2 t[G::r];
        group_tw<G::r, G::s, TP>(tws + G::toff, (g0 + u * gstep) % G::s, t);
#pragma unroll
        for (int a = 1; a < G::r; ++a) v[u][a] = mul_shoup(v[u][a], t[a].x, t[a].y);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < GPT; ++u)
#pragma unroll
    for (int a = 0; a < G::r; ++a) st(g0 + u * gstep, a, v[u][a]);
}

// Every group of round k, NT threads (this thread = t), at most GMAX groups
// in flight per thread.
template <int LOG, int k, int NT, int GMAX, bool INV, bool TP = false, class LD, class ST>
__device__ __forceinline__ void round_all(int t, const uint2* __restrict__ tws, LD&& ld, ST&& st) {
  constexpr int groups = Geo<LOG, k>::groups;
  if constexpr (groups >= NT) {
    constexpr int per = groups / NT;
    constexpr int gpt = per < GMAX ? per : GMAX;
#pragma unroll 1
    for (int it = 0; it < per / gpt; ++it)
      round_multi<LOG, k, gpt, INV, TP>(t + it * gpt * NT, NT, tws, ld, st);
  } else {
    if (t < groups) round_multi<LOG, k, 1, INV, TP>(t, NT, tws, ld, st);
  }
}

// w_{2^23}^e in Montgomery form
__device__ __forceinline__ uint32_t gtw(const TwTables& tw, uint32_t e) {
  return mul_mont(tw.g_hi[e >> 12], tw.g_lo[e & 4095u]);
}

template <int LOG>
__device__ __forceinline__ int brev(int p) {
  if constexpr (LOG == 0)
    return 0;
  else
    return (int)(__builtin_bitreverse32((uint32_t)p) >> (32 - LOG));
}

// Transform position q of an item maps to bit off + (q < h ? q : q - Nc) of
// the source, or to 0 when that index falls outside [lo, hi).  All indices
// fit 32 bits: the NTT path takes n < p < 2^30, so n+m-1 < 2^31.
struct BitMap {
  int32_t off, lo, hi, h;
};
constexpr int MAXMAP = 8;

// One transform (n+m-1 <= Nc): with the seed transformed as its first Nc
// bits S, the raw block is placed rotated by d = n-1, x'[j'] = x[(j'+d) mod
// Nc]; then (S * x')[t] = sum_j S[t+n-1-j] x[j] = row t of T x for t < m
// (t+n-1-j stays inside [0, n+m-1), no wrap).  The rotation costs nothing
// (it is a bit mapping), and the seed transform no longer depends on n, m.
__host__ __device__ __forceinline__ BitMap rotated_block(uint32_t n, int32_t Nc) {
  return BitMap{(int32_t)n - 1, 0, (int32_t)n, Nc - ((int32_t)n - 1)};
}

__device__ __forceinline__ uint32_t map_bit(const uint32_t* __restrict__ bits, const BitMap& mp,
                                            int32_t q, int32_t Nc) {
  const int32_t idx = mp.off + (q < mp.h ? q : q - Nc);
  if ((uint32_t)(idx - mp.lo) >= (uint32_t)(mp.hi - mp.lo)) return 0u;
  return (bits[(uint32_t)idx >> 5] >> (idx & 31)) & 1u;
}

// The 32 values of positions q0..q0+31 as one word (bit i = position q0+i).
// Fast path: no wrap point and no range edge inside, so the word is a
// funnel shift of two consecutive source words; otherwise bit by bit.
__device__ __forceinline__ uint32_t stage_word(const uint32_t* __restrict__ bits,
                                               const BitMap& mp, int32_t q0, int32_t Nc) {
  const int32_t q1 = q0 + 31;
  if (q1 < mp.h || q0 >= mp.h) {
    const int32_t i0 = mp.off + (q0 < mp.h ? q0 : q0 - Nc);
    if (i0 >= mp.lo && i0 + 31 < mp.hi) {
      const uint32_t w = (uint32_t)i0 >> 5, sh = (uint32_t)i0 & 31u;
      uint32_t v = bits[w] >> sh;
      if (sh) v |= bits[w + 1] << (32u - sh);
      return v;
    }
  }
  uint32_t v = 0;
  for (int i = 0; i < 32; ++i) v |= map_bit(bits, mp, q0 + i, Nc) << i;
  return v;
}

// Montgomery-form powers u^0..u^(R-1) of u = w^e (u^0 = 2^32 mod p).
template <int R>
__device__ __forceinline__ void mont_powers(const TwTables& tw, uint32_t e, uint32_t (&up)[R]) {
  up[0] = MONT_R;
  if constexpr (R > 1) {
    up[1] = gtw(tw, e);
#pragma unroll
    for (int t = 2; t < R; ++t) up[t] = mul_mont(up[t - 1], up[1]);
  }
}

// A radix-2 first round followed by a radix-16 round (columns of 2^9
// points): the thread that owns round-1 groups (0, b) and (1, b) holds both
// operands of every round-0 butterfly of them, so the two rounds run in
// registers with no LDS exchange or barrier between them.
template <int LOG1>
constexpr bool merge01() {
  return RP<LOG1>::lgr(0) == 1 && RP<LOG1>::K >= 3;
}

// Forward rounds 0 and 1 on input bits: bit q of this column is
// (wbits[q] >> c) & 1.  Round 0 on bits x0 (position q) and x1 (q + N/2):
// x0 + x1, and (x0 - x1) w_N^q = x0 w + x1 (p - w), no multiplication.
// st(g, e, v) stores element e of round-1 group g.  b: round-1 group index
// within its half, b < Geo<LOG1, 1>::s.
// The twiddles of these two rounds for group index b, loaded before the
// input bits are staged (they do not depend on them): w[a] = w_N^(a s1 + b)
// of round 0, t1 the round-1 group twiddles.
template <int LOG1>
struct Tw01 {
  uint32_t w[16];
  uint2 t1[16];
};
template <int LOG1>
__device__ __forceinline__ void load_tw01(int b, const uint2* __restrict__ tws, Tw01<LOG1>& t) {
  using G0 = Geo<LOG1, 0>;
  using G1 = Geo<LOG1, 1>;
#pragma unroll
  for (int a = 0; a < 16; ++a) t.w[a] = tws[G0::toff + 2 * (a * G1::s + b) + 1].x;
  group_tw<16, G1::s, false>(tws + G1::toff, b, t.t1);
}

template <int LOG1, class ST>
__device__ __forceinline__ void fwd_round01_bits(int b, const Tw01<LOG1>& tw01, bool upper_zero,
                                                 const uint32_t* __restrict__ wbits, int c,
                                                 ST&& st) {
  using G0 = Geo<LOG1, 0>;
  using G1 = Geo<LOG1, 1>;
  static_assert(G0::r == 2 && G1::r == 16 && G0::s == 16 * G1::s, "radix 2 then radix 16");
  uint32_t v[2][16];
  if (upper_zero) {
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int q = a * G1::s + b;
      const uint32_t x0 = (wbits[q] >> c) & 1u;
      v[0][a] = x0;
      v[1][a] = x0 ? tw01.w[a] : 0u;
    }
  } else {
#pragma unroll
    for (int a = 0; a < 16; ++a) {
      const int q = a * G1::s + b;
      const uint32_t w = tw01.w[a];  // w_N^q, N = 2^LOG1
      const uint32_t x0 = (wbits[q] >> c) & 1u, x1 = (wbits[q + G0::s] >> c) & 1u;
      v[0][a] = x0 + x1;
      v[1][a] = (x0 ? w : 0u) + (x1 ? P - w : 0u);
    }
  }
  const uint2 (&t)[16] = tw01.t1;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    dft_reg<16, false, true>(v[h]);
#pragma unroll
    for (int a = 1; a < 16; ++a) v[h][a] = mul_shoup(v[h][a], t[a].x, t[a].y);
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int a = 0; a < 16; ++a) st(h * G1::s + b, a, v[h][a]);
}

// Twiddles of the inverse rounds 1 and 0 for group index b (loaded ahead of
// the barrier before them): t1 the round-1 group twiddles, w[a] the Shoup
// pair of w_N^-(a s1 + b) for round 0.
template <int LOG1>
struct TwInv10 {
  uint2 t1[16];
  uint2 w[16];
};
template <int LOG1>
__device__ __forceinline__ void load_tw10(int b, const uint2* __restrict__ tws,
                                          TwInv10<LOG1>& t) {
  using G0 = Geo<LOG1, 0>;
  using G1 = Geo<LOG1, 1>;
  group_tw<16, G1::s, false>(tws + G1::toff, b, t.t1);
#pragma unroll
  for (int a = 0; a < 16; ++a) t.w[a] = tws[G0::toff + 2 * (a * G1::s + b) + 1];
}

// Inverse rounds 1 and 0 (the last two of a column): ld(g, e) reads element e
// of round-1 group g; out(q, e, v) receives position q + e N/2 (e = 0, 1).
// The upper outputs are formed only when need_hi.
template <int LOG1, class LD, class OUT>
__device__ __forceinline__ void inv_round10(int b, const TwInv10<LOG1>& tw10, bool need_hi,
                                            LD&& ld, OUT&& out) {
  using G0 = Geo<LOG1, 0>;
  using G1 = Geo<LOG1, 1>;
  static_assert(G0::r == 2 && G1::r == 16 && G0::s == 16 * G1::s, "radix 16 then radix 2");
  uint32_t v[2][16];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int a = 0; a < 16; ++a) v[h][a] = ld(h * G1::s + b, a);
  const uint2 (&t)[16] = tw10.t1;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int a = 1; a < 16; ++a) v[h][a] = mul_shoup(v[h][a], t[a].x, t[a].y);
    dft_reg<16, true>(v[h]);
  }
#pragma unroll
  for (int a = 0; a < 16; ++a) {
    const int q = a * G1::s + b;
    const uint2 w = tw10.w[a];  // w_N^-q
    const uint32_t u = v[0][a], tt = mul_shoup(v[1][a], w.x, w.y);
    out(q, 0, red2(u + tt));
    if (need_hi) out(q, 1, sub2(u, tt));
  }
}

// ----------------------------------------------------------------- pass A
struct ColFwdArgs {
  const uint32_t* bits;
  uint64_t zs;  // batch stride of the bit source (bits, multiple of 32)
  BitMap map[MAXMAP];
  int nmap;
  int log2, log_nc;
  uint32_t* out;  // item y = blockIdx.y at out + y * Nc
  const NttItem* items;  // non-null: item y is the raw block items[y] (nmap = 1)
  // non-null: item y exists only while item0 + y < *count (read on the device)
  const uint32_t* count;
  uint32_t item0;
  // hg > 0: workgroups x < hg of item 0 count samples for the min-entropy
  // estimate instead (those of other items exit), the last of them runs it
  uint32_t hg;
  // nonzero: every source bit at positions q >= Nc/2 is 0 (the chunks of the
  // split transform), so the first radix-2 round skips those inputs
  uint32_t upper_zero;
  uint32_t* ticket;
  hd::HistArgs est;
};

constexpr int COLS = 32;  // columns per workgroup (128-byte rows)
constexpr int CGMAX = 2;  // groups in flight per thread
// slots (threads per column) of a column workgroup, 32 columns each: enough
// for two radix-16 groups of the last round per thread, 2^LOG1 / 32 (16 slots,
// 512 threads, for 2^9-point columns; 2 for 2^6), at least 2.  With one slot
// per last-round group the short columns left half or more of their threads
// idle in that round and paid the per-thread twiddle set-up for 16 values.
// (Inverse 2^9-point columns once ran 32 slots, the extra waves hiding more
// of the input loads and barriers; with their last two rounds merged in
// registers, inv_round10, 16 slots keep two workgroups per CU.)
template <int LOG1, bool INV>
constexpr int cslots() {
  return LOG1 >= 9 ? 16 : ((1 << LOG1) / 32 > 2 ? (1 << LOG1) / 32 : 2);
}
// the estimate workgroups inside pass A need 256 threads (one per bin)
constexpr int EST_MIN_LOG1 = 8;

// sub-histogram copies of an estimate workgroup in the column LDS
template <int LOG1>
constexpr int est_copies() {
  return LOG1 >= 9 ? 32 : (LOG1 == 8 ? 16 : 8);
}

// Pass A on column block bx of item `item` (NS slots of 32 threads; lds:
// (1 << LOG1) * COLS words, wbits: 1 << LOG1 words).  MERGE: run the first
// two rounds as one register round where they allow it (merge01); the
// persistent kernels keep them apart (their register budget is shared by
// every column length).
template <int LOG1, int NS, bool MERGE = true>
__device__ __forceinline__ void cols_fwd_body(const ColFwdArgs& a, const TwTables& tw, int bx,
                                              int item, uint32_t* __restrict__ lds,
                                              uint32_t* __restrict__ wbits) {
  const int c = threadIdx.x & (COLS - 1), slot = threadIdx.x >> 5;
  const int32_t Nc = 1 << a.log_nc;
  const int j2 = bx * COLS + c;
  const uint32_t* __restrict__ bits;
  BitMap mp;
  if (a.items) {
    const NttItem& it = a.items[item];
    bits = a.bits + (it.x_bit >> 5);
    mp = rotated_block(it.n, Nc);
  } else {
    bits = a.bits + (uint64_t)(item / a.nmap) * (a.zs >> 5);
    mp = a.map[item % a.nmap];
  }
  uint32_t* __restrict__ out = a.out + (uint64_t)item * (uint32_t)Nc;
  const uint32_t gstep = (uint32_t)j2 << (LOG_MAX - a.log_nc);
  const int l2 = a.log2;

  // with one merged group per thread, its twiddles are loaded while the
  // input bits are staged
  constexpr bool MERGE1 = MERGE && merge01<LOG1>() && NS == Geo<LOG1, 1>::s;
  Tw01<LOG1> tw01;
  if constexpr (MERGE1) load_tw01<LOG1>(slot, tw.fwd, tw01);
  for (int j1 = threadIdx.x; j1 < (1 << LOG1); j1 += COLS * NS)
    wbits[j1] = stage_word(bits, mp, (j1 << l2) + bx * COLS, Nc);
  __syncthreads();
  auto ld_bits = [&](int g, int e) -> uint32_t {
    const int j1 = Geo<LOG1, 0>::pos0(g) + e * Geo<LOG1, 0>::s;
    return (wbits[j1] >> c) & 1u;
  };
  auto ld_lds_k = [&](auto kc) {
    return [&](int g, int e) -> uint32_t {
      using G = Geo<LOG1, decltype(kc)::value>;
      return lds[(G::pos0(g) + e * G::s) * COLS + c];
    };
  };
  auto st_lds_k = [&](auto kc) {
    return [&](int g, int e, uint32_t v) {
      using G = Geo<LOG1, decltype(kc)::value>;
      lds[(G::pos0(g) + e * G::s) * COLS + c] = v;
    };
  };
  constexpr int K = RP<LOG1>::K;
  // four-step twiddle w_Nc^(j2 k1) of last-round position p = g*r + e:
  // k1 = bitrev(p) = bitrev(e) 2^(LOG1-lgr) + bitrev(g), so the twiddle is
  // B_g U^bitrev(e) with U = w_Nc^(j2 2^(LOG1-lgr)) fixed per thread
  using GL = Geo<LOG1, K - 1>;
  static_assert(GL::s == 1, "last round works on contiguous groups");
  // (v U^f 2^-32) B_g 2^-32 with Montgomery-form U^f and B_g: both factors
  // are fixed before the values arrive, so both products take the
  // three-multiplication form (U^0 is the Montgomery one: skipped)
  uint32_t upow[GL::r], upre[GL::r];
  mont_powers<GL::r>(tw, (gstep << (LOG1 - GL::lgr)) & ((1u << LOG_MAX) - 1), upow);
#pragma unroll
  for (int f = 0; f < GL::r; ++f) upre[f] = mont_pre(upow[f]);
  uint32_t bg = 0, bgp = 0;
  auto st_out = [&](int g, int e, uint32_t v) {
    const int p = g * GL::r + e;
    if (e == 0) {
      bg = gtw(tw, gstep * (uint32_t)brev<LOG1 - GL::lgr>(g));
      bgp = mont_pre(bg);
    }
    const int f = brev<GL::lgr>(e);
    const uint32_t x = e ? mul_mont_pre(v, upow[f], upre[f]) : v;
    st_w32(out, ((uint32_t)p << l2) + j2, mul_mont_pre(x, bg, bgp));
  };
  auto round = [&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (K == 1)
      round_all<LOG1, k, NS, CGMAX, false>(slot, tw.fwd, ld_bits, st_out);
    else if constexpr (k == 0)
      round_all<LOG1, k, NS, CGMAX, false>(slot, tw.fwd, ld_bits, st_lds_k(kc));
    else if constexpr (k == K - 1)
      round_all<LOG1, k, NS, CGMAX, false>(slot, tw.fwd, ld_lds_k(kc), st_out);
    else
      round_all<LOG1, k, NS, CGMAX, false>(slot, tw.fwd, ld_lds_k(kc), st_lds_k(kc));
    if constexpr (k < K - 1) __syncthreads();
  };
  if constexpr (MERGE && merge01<LOG1>()) {
    if constexpr (MERGE1) {
      fwd_round01_bits<LOG1>(slot, tw01, a.upper_zero != 0, wbits, c,
                             st_lds_k(std::integral_constant<int, 1>{}));
    } else {
      for (int b = slot; b < Geo<LOG1, 1>::s; b += NS) {
        Tw01<LOG1> t01;
        load_tw01<LOG1>(b, tw.fwd, t01);
        fwd_round01_bits<LOG1>(b, t01, a.upper_zero != 0, wbits, c,
                               st_lds_k(std::integral_constant<int, 1>{}));
      }
    }
    __syncthreads();
    static_for<2, K>(round);
  } else {
    static_for<0, K>(round);
  }
}

template <int LOG1>
__global__ __launch_bounds__((COLS * cslots<LOG1, false>())) void k_cols_fwd(ColFwdArgs a,
                                                                            TwTables tw) {
  constexpr int NS = cslots<LOG1, false>();
  __shared__ __align__(16) uint32_t lds[(1 << LOG1) * COLS];
  __shared__ uint32_t wbits[1 << LOG1];  // row j1's 32 input bits of this column block
  if (blockIdx.x < a.hg) {
    if constexpr (LOG1 >= EST_MIN_LOG1) {
      static_assert(COLS * NS >= 256, "one estimate thread per bin");
      static_assert(est_copies<LOG1>() * hd::HB <= (1 << LOG1) * COLS &&
                        sizeof(hd::FinishLds) <= sizeof(lds),
                    "estimate workgroup fits the column LDS");
      if (blockIdx.y == 0)
        hd::estimate_workgroup<COLS * NS, est_copies<LOG1>()>(a.est, blockIdx.x, a.ticket,
                                                                  lds);
    }
    return;
  }
  if (a.count && a.item0 + blockIdx.y >= *a.count) return;
  cols_fwd_body<LOG1, NS>(a, tw, blockIdx.x - a.hg, blockIdx.y, lds, wbits);
}

// ----------------------------------------------------------------- pass C
struct ColInvArgs {
  const uint32_t* in;  // item y = blockIdx.y at in + y * Nc
  int ny, log2, log_nc;
  uint32_t* y;    // output bits
  uint64_t y_zs;  // batch stride of the output (bits, multiple of 64)
  int64_t by;     // output chunk length
  uint64_t m;     // output bits the plan covers (words up to m are written)
  const uint64_t* m_dev;  // nullable: the valid output length, read on the device (<= m)
  const NttItem* items;   // non-null: item y writes items[y] (ny = 1)
  const uint64_t* m_arr;  // with items, nullable: valid length of item y at m_arr[blk]
  const uint32_t* count;  // as in ColFwdArgs
  uint32_t item0;
};

// valid output bits: the plan's m, or the smaller length computed on the device
__device__ __forceinline__ uint64_t valid_bits(uint64_t m, const uint64_t* m_dev) {
  if (!m_dev) return m;
  const uint64_t d = *m_dev;
  return d < m ? d : m;
}

// Pass C on column block bx of item `item` (NS slots of 32 threads; lds:
// (1 << LOG1) * COLS words).  MERGE as in cols_fwd_body, for the last two
// rounds.
template <int LOG1, int NS, bool MERGE = true>
__device__ __forceinline__ void cols_inv_body(const ColInvArgs& a, const TwTables& tw, int bx,
                                              int item, uint32_t* __restrict__ lds) {
  const int c = threadIdx.x & (COLS - 1), slot = threadIdx.x >> 5;
  const int lane = threadIdx.x & 63;
  const int32_t Nc = 1 << a.log_nc;
  const int j2 = bx * COLS + c;
  const int o = item % a.ny;
  uint64_t ybase, m;
  const uint64_t* m_dev;
  if (a.items) {
    const NttItem& it = a.items[item];
    ybase = it.y_bit;
    m = it.m;
    m_dev = a.m_arr ? a.m_arr + it.blk : nullptr;
  } else {
    ybase = (uint64_t)(item / a.ny) * a.y_zs + (uint64_t)o * a.by;
    m = a.m;
    m_dev = a.m_dev;
  }
  const int64_t rem_cap = (int64_t)m - (int64_t)o * a.by;
  const int32_t ylimit = ((int32_t)(rem_cap < a.by ? rem_cap : a.by) + 63) & ~63;
  const int64_t rem = (int64_t)valid_bits(m, m_dev) - (int64_t)o * a.by;
  const int32_t yvalid = (int32_t)(rem < a.by ? (rem < 0 ? 0 : rem) : a.by);
  uint32_t* __restrict__ ywords = a.y + (ybase >> 5);
  const uint32_t* __restrict__ in = a.in + (uint64_t)item * (uint32_t)Nc;
  const uint32_t gstep = (uint32_t)j2 << (LOG_MAX - a.log_nc);
  constexpr uint32_t EMASK = (1u << LOG_MAX) - 1;
  const int l2 = a.log2;
  constexpr int K = RP<LOG1>::K;

  // inverse four-step twiddle, factored as in pass A
  using GL = Geo<LOG1, K - 1>;
  static_assert(GL::s == 1, "last round works on contiguous groups");
  uint32_t upow[GL::r], upre[GL::r];
  mont_powers<GL::r>(tw, (0u - (gstep << (LOG1 - GL::lgr))) & EMASK, upow);
#pragma unroll
  for (int f = 0; f < GL::r; ++f) upre[f] = mont_pre(upow[f]);
  uint32_t bg = 0, bgp = 0;
  auto ld_in = [&](int g, int e) -> uint32_t {
    const int p = g * GL::r + e;
    if (e == 0) {
      bg = gtw(tw, (0u - gstep * (uint32_t)brev<LOG1 - GL::lgr>(g)) & EMASK);
      bgp = mont_pre(bg);
    }
    const int f = brev<GL::lgr>(e);
    const uint32_t v = ld_w32(in, ((uint32_t)p << l2) + j2);
    const uint32_t x = e ? mul_mont_pre(v, upow[f], upre[f]) : v;
    return mul_mont_pre(x, bg, bgp);
  };
  auto ld_lds_k = [&](auto kc) {
    return [&](int g, int e) -> uint32_t {
      using G = Geo<LOG1, decltype(kc)::value>;
      return lds[(G::pos0(g) + e * G::s) * COLS + c];
    };
  };
  auto st_lds_k = [&](auto kc) {
    return [&](int g, int e, uint32_t v) {
      using G = Geo<LOG1, decltype(kc)::value>;
      lds[(G::pos0(g) + e * G::s) * COLS + c] = v;
    };
  };
  // natural-order position j1 -> output bit t = j1*N2 + j2; the 32 lanes of
  // a half-wave hold 32 consecutive bits of one output word
  auto st_bits = [&](int g, int e, uint32_t v) {
    const int j1 = Geo<LOG1, 0>::pos0(g) + e * Geo<LOG1, 0>::s;
    const int32_t t = (j1 << l2) + j2;
    const uint32_t bit = (t < yvalid) ? (red1(v) & 1u) : 0u;
    const uint64_t bal = __ballot(bit);
    const int32_t t0 = t - c;
    if ((lane & 31) == 0 && t0 < ylimit) ywords[t0 >> 5] = lane ? (uint32_t)(bal >> 32) : (uint32_t)bal;
  };
  auto round = [&](auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (K == 1)
      round_all<LOG1, k, NS, CGMAX, true>(slot, tw.inv, ld_in, st_bits);
    else if constexpr (k == K - 1)
      round_all<LOG1, k, NS, CGMAX, true>(slot, tw.inv, ld_in, st_lds_k(kc));
    else if constexpr (k == 0)
      round_all<LOG1, k, NS, CGMAX, true>(slot, tw.inv, ld_lds_k(kc), st_bits);
    else
      round_all<LOG1, k, NS, CGMAX, true>(slot, tw.inv, ld_lds_k(kc), st_lds_k(kc));
    if constexpr (k > 0) __syncthreads();
  };
  if constexpr (MERGE && merge01<LOG1>()) {
    // outputs at j1 >= N1/2 lie at bit t >= (N1/2) N2 of the chunk
    const bool need_hi = ((int64_t)Geo<LOG1, 0>::s << l2) < (int64_t)ylimit;
    if constexpr (NS == Geo<LOG1, 1>::s && K == 3) {
      // one merged group per thread: its twiddles are loaded between the
      // first round's work and its barrier, so they arrive during the wait
      round_all<LOG1, 2, NS, CGMAX, true>(slot, tw.inv, ld_in, st_lds_k(std::integral_constant<int, 2>{}));
      TwInv10<LOG1> t10;
      load_tw10<LOG1>(slot, tw.inv, t10);
      __syncthreads();
      inv_round10<LOG1>(slot, t10, need_hi, ld_lds_k(std::integral_constant<int, 1>{}), st_bits);
    } else {
      static_for_down<2, K>(round);
      for (int b = slot; b < Geo<LOG1, 1>::s; b += NS) {
        TwInv10<LOG1> t10;
        load_tw10<LOG1>(b, tw.inv, t10);
        inv_round10<LOG1>(b, t10, need_hi, ld_lds_k(std::integral_constant<int, 1>{}), st_bits);
      }
    }
  } else {
    static_for_down<0, K>(round);
  }
}

template <int LOG1>
__global__ __launch_bounds__((COLS * cslots<LOG1, true>())) void k_cols_inv(ColInvArgs a,
                                                                           TwTables tw) {
  constexpr int NS = cslots<LOG1, true>();
  __shared__ uint32_t lds[(1 << LOG1) * COLS];
  if (a.count && a.item0 + blockIdx.y >= *a.count) return;
  cols_inv_body<LOG1, NS>(a, tw, blockIdx.x, blockIdx.y, lds);
}

// ----------------------------------------------------------------- pass B
struct RowArgs {
  const uint32_t* in;  // residues (pass-A output); item at in + item * Nc + row * N2
  const uint32_t* bits;
  uint64_t zs;  // batch stride of the bit source (fused; bits, multiple of 32)
  BitMap map[MAXMAP];
  const uint32_t* W;  // seed spectra, window w at W + w * Nc
  int nx, ny, log_nc;
  uint32_t cw;    // seed mode: Nc^-1 2^64 mod p
  uint32_t* out;  // residues out (item * Nc + row * N2) or seed spectra
  uint32_t* y;    // output bits (fused)
  uint64_t y_zs;
  uint64_t m;
  const uint64_t* m_dev;  // nullable, as in ColInvArgs
  const NttItem* items;   // hash with nx = ny = 1: item zy is items[zy] (raw block,
  const uint64_t* m_arr;  // seed spectrum, output and valid length m_arr[blk])
  const uint32_t* count;  // as in ColFwdArgs
  uint32_t item0;
};

// Threads of a row kernel: every thread owns GPT groups of the last round.
template <int LOG2, int GPT>
constexpr int row_threads() {
  return (1 << LOG2) / (16 * GPT);
}

// One row of the four-step (or the whole transform when N1 = 1).
//  SEED:  forward transform of a seed window -> Montgomery-form spectrum row.
//  hash:  forward transforms of NX raw chunks, products with the seed
//         spectra summed per output chunk, inverse transform per output chunk.
// IN_BITS / OUT_BITS: the row is the whole transform and reads raw bits /
// writes hash bits directly.  The last forward round and the first inverse
// round act on the same 16 contiguous positions per group, so the seed
// product happens in registers between them.
// LDS words of one row buffer (one pad word per 16)
template <int LOG2>
constexpr int row_lds_words() {
  return (1 << LOG2) + (1 << LOG2) / 16;
}
// Two raw chunks of a hash are transformed side by side, one LDS buffer
// each, so every round of both rows shares one barrier (and, with two
// output chunks, so are the two inverse transforms).
template <int NX, bool IN_BITS, bool SEED, bool OUT_BITS>
constexpr bool rows_joint() {
  return NX == 2 && !SEED && !IN_BITS && !OUT_BITS;
}

// Row `row` of item zy, run by threads tid < row_threads<LOG2, GPT>() of
// the workgroup (every thread of the workgroup takes part in its barriers);
// lds: (JOINT ? 2 : 1) * row_lds_words<LOG2>() words; wbits (IN_BITS only):
// N2 / 32 words.
template <int LOG2, int NX, int GPT, bool IN_BITS, bool SEED, bool OUT_BITS>
__device__ __forceinline__ void rows_body(const RowArgs& a, const TwTables& tw, int tid, int row,
                                          int zy, uint32_t* __restrict__ ldsbase,
                                          uint32_t* __restrict__ wbits) {
  constexpr int N2 = 1 << LOG2, T = row_threads<LOG2, GPT>(), K = RP<LOG2>::K;
  static_assert(K >= 2, "rows are at least 2^5 long");
  static_assert(Geo<LOG2, K - 1>::r == 16 && Geo<LOG2, K - 1>::s == 1, "last round");
  constexpr bool JOINT = rows_joint<NX, IN_BITS, SEED, OUT_BITS>();
  uint32_t* const ldsb[2] = {ldsbase, ldsbase + row_lds_words<LOG2>()};
  uint32_t* const lds = ldsb[0];
  const int lane = tid & 63;
  const int32_t Nc = 1 << a.log_nc;
  const NttItem* desc = SEED ? nullptr : (a.items ? a.items + zy : nullptr);
  // transposed twiddle tables (lane-contiguous loads) pay off up to 2^13-point
  // rows; at 2^14 the per-group layout measured faster
  constexpr bool TPT = LOG2 < 14;
  const uint2* twf = TPT ? tw.fwd_t : tw.fwd;
  const uint2* twi = TPT ? tw.inv_t : tw.inv;

  auto ld_buf_k = [&](auto kc, const uint32_t* buf) {
    return [=](int g, int e) -> uint32_t {
      using G = Geo<LOG2, decltype(kc)::value>;
      const int p0 = G::pos0(g);
      return buf[p0 + (p0 >> 4) + e * G::SP];
    };
  };
  auto st_buf_k = [&](auto kc, uint32_t* buf) {
    return [=](int g, int e, uint32_t v) {
      using G = Geo<LOG2, decltype(kc)::value>;
      const int p0 = G::pos0(g);
      buf[p0 + (p0 >> 4) + e * G::SP] = v;
    };
  };
  auto ld_lds_k = [&](auto kc) { return ld_buf_k(kc, lds); };
  auto st_lds_k = [&](auto kc) { return st_buf_k(kc, lds); };
  using G0 = Geo<LOG2, 0>;
  constexpr std::integral_constant<int, 0> k0{};

  uint32_t xs[NX][GPT][16];
  if constexpr (JOINT) {
    static_for<0, NX>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const uint32_t* src = a.in + (uint64_t)(zy * NX + c) * (uint32_t)Nc + (uint64_t)row * N2;
      auto ld0 = [&](int g, int e) -> uint32_t { return src[G0::pos0(g) + e * G0::s]; };
      round_all<LOG2, 0, T, GPT, false, TPT>(tid, twf, ld0, st_buf_k(k0, ldsb[c]));
    });
    __syncthreads();
    static_for<1, K - 1>([&](auto kc) {
      static_for<0, NX>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        round_all<LOG2, decltype(kc)::value, T, GPT, false, TPT>(tid, twf, ld_buf_k(kc, ldsb[c]),
                                                                 st_buf_k(kc, ldsb[c]));
      });
      __syncthreads();
    });
    static_for<0, NX>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
#pragma unroll
      for (int u = 0; u < GPT; ++u) {
        const int g = tid + u * T;
#pragma unroll
        for (int e = 0; e < 16; ++e) xs[c][u][e] = ldsb[c][g * 17 + e];
      }
#pragma unroll
      for (int u = 0; u < GPT; ++u) dft_reg<16, false>(xs[c][u]);
    });
    __syncthreads();
  } else static_for<0, NX>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    const int item = SEED ? zy : zy * NX + c;
    if constexpr (IN_BITS) {
      // the whole transform's input bits, 32 positions per LDS word
      const BitMap mp = desc ? rotated_block(desc->n, Nc) : a.map[SEED ? zy : c];
      const uint32_t* __restrict__ bits =
          a.bits + (desc ? (desc->x_bit >> 5) : (SEED ? 0 : (uint64_t)zy * (a.zs >> 5)));
      for (int w = tid; w < N2 / 32; w += T) wbits[w] = stage_word(bits, mp, w * 32, Nc);
      __syncthreads();
      auto ld0 = [&](int g, int e) -> uint32_t {
        const int q = G0::pos0(g) + e * G0::s;
        return (wbits[q >> 5] >> (q & 31)) & 1u;
      };
      round_all<LOG2, 0, T, GPT, false, TPT>(tid, twf, ld0, st_lds_k(k0));
    } else {
      // no __restrict__: with one transform pass B works in place (in == out)
      const uint32_t* src = a.in + (uint64_t)item * (uint32_t)Nc + (uint64_t)row * N2;
      auto ld0 = [&](int g, int e) -> uint32_t { return src[G0::pos0(g) + e * G0::s]; };
      round_all<LOG2, 0, T, GPT, false, TPT>(tid, twf, ld0, st_lds_k(k0));
    }
    __syncthreads();
    static_for<1, K - 1>([&](auto kc) {
      round_all<LOG2, decltype(kc)::value, T, GPT, false, TPT>(tid, twf, ld_lds_k(kc), st_lds_k(kc));
      __syncthreads();
    });
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int g = tid + u * T;
#pragma unroll
      for (int e = 0; e < 16; ++e) xs[c][u][e] = lds[g * 17 + e];
    }
#pragma unroll
    for (int u = 0; u < GPT; ++u) dft_reg<16, false>(xs[c][u]);
    __syncthreads();
  });

  if constexpr (SEED) {
    // spectrum row layout: element e of last-round group g at
    // (e / 4) * N2/4 + 4 g + e % 4, so the hash's 16-byte loads of
    // consecutive groups (lanes) are consecutive
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      uint32_t* dst = a.out + (uint64_t)zy * (uint32_t)Nc + (uint64_t)row * N2 + (tid + u * T) * 4;
#pragma unroll
      for (int e = 0; e < 16; e += 4) {
        uint4 w;
        w.x = red1(mul_mont(xs[0][u][e + 0], a.cw));
        w.y = red1(mul_mont(xs[0][u][e + 1], a.cw));
        w.z = red1(mul_mont(xs[0][u][e + 2], a.cw));
        w.w = red1(mul_mont(xs[0][u][e + 3], a.cw));
        *reinterpret_cast<uint4*>(dst + (e / 4) * (N2 / 4)) = w;
      }
    }
    return;
  } else {
    // Two raw and two output chunks: the 2x2 block matrix is [[A, B], [C, A]]
    // (the diagonal blocks share a window), so with spectra stored as
    // (A, B-A, C-A) three products do: m1 = A (x0+x1), y0 = m1 + (B-A) x1,
    // y1 = m1 + (C-A) x0.  m1 takes x1's registers (x1 is not needed after
    // y0's products).
    const bool three = NX == 2 && a.ny == 2;
    if constexpr (JOINT) {
      if (three) {
        // y0 = A (x0 + x1) + (B - A) x1 into xs[0], y1 = A (x0 + x1) + (C - A) x0
        // into xs[1], then both inverse transforms side by side
        const uint32_t* wrow = a.W + (uint64_t)row * N2;
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
          const uint32_t* wa = wrow + (tid + u * T) * 4;
          const uint32_t* wb = wa + (uint32_t)Nc;
          const uint32_t* wc = wb + (uint32_t)Nc;
#pragma unroll
          for (int e = 0; e < 16; e += 4) {
            const uint4 va = *reinterpret_cast<const uint4*>(wa + (e / 4) * (N2 / 4));
            const uint4 vb = *reinterpret_cast<const uint4*>(wb + (e / 4) * (N2 / 4));
            const uint4 vc = *reinterpret_cast<const uint4*>(wc + (e / 4) * (N2 / 4));
            const uint32_t A4[4] = {va.x, va.y, va.z, va.w};
            const uint32_t B4[4] = {vb.x, vb.y, vb.z, vb.w};
            const uint32_t C4[4] = {vc.x, vc.y, vc.z, vc.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const uint32_t x0 = xs[0][u][e + i], x1 = xs[1][u][e + i];
              const uint32_t mm = mul_mont(red2(x0 + x1), A4[i]);
              xs[0][u][e + i] = red2(mm + mul_mont(x1, B4[i]));
              xs[1][u][e + i] = red2(mm + mul_mont(x0, C4[i]));
            }
          }
        }
        static_for<0, 2>([&](auto oc) {
          constexpr int o = decltype(oc)::value;
#pragma unroll
          for (int u = 0; u < GPT; ++u) {
            dft_reg<16, true>(xs[o][u]);
            const int g = tid + u * T;
#pragma unroll
            for (int e = 0; e < 16; ++e) ldsb[o][g * 17 + e] = xs[o][u][e];
          }
        });
        __syncthreads();
        static_for_down<1, K - 1>([&](auto kc) {
          static_for<0, 2>([&](auto oc) {
            constexpr int o = decltype(oc)::value;
            round_all<LOG2, decltype(kc)::value, T, GPT, true, TPT>(
                tid, twi, ld_buf_k(kc, ldsb[o]), st_buf_k(kc, ldsb[o]));
          });
          __syncthreads();
        });
        static_for<0, 2>([&](auto oc) {
          constexpr int o = decltype(oc)::value;
          uint32_t* __restrict__ dst =
              a.out + (uint64_t)(zy * 2 + o) * (uint32_t)Nc + (uint64_t)row * N2;
          auto st0 = [&](int g, int e, uint32_t v) { dst[G0::pos0(g) + e * G0::s] = v; };
          round_all<LOG2, 0, T, GPT, true, TPT>(tid, twi, ld_buf_k(k0, ldsb[o]), st0);
        });
        return;
      }
    }
    for (int o = 0; o < a.ny; ++o) {
      uint32_t acc[GPT][16];
#pragma unroll
      for (int u = 0; u < GPT; ++u)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[u][e] = 0;
      if constexpr (NX == 2) {
        if (three) {
          const uint32_t* wrow = a.W + (uint64_t)row * N2;
          if (o == 0) {
            // m1 = A (x0 + x1); acc = m1 + (B - A) x1
#pragma unroll
            for (int u = 0; u < GPT; ++u) {
              const uint32_t* wa = wrow + (tid + u * T) * 4;
              const uint32_t* wb = wa + (uint32_t)Nc;
#pragma unroll
              for (int e = 0; e < 16; e += 4) {
                const uint4 va = *reinterpret_cast<const uint4*>(wa + (e / 4) * (N2 / 4));
                const uint4 vb = *reinterpret_cast<const uint4*>(wb + (e / 4) * (N2 / 4));
                const uint32_t A4[4] = {va.x, va.y, va.z, va.w};
                const uint32_t B4[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const uint32_t x1 = xs[NX - 1][u][e + i];
                  const uint32_t mm = mul_mont(red2(xs[0][u][e + i] + x1), A4[i]);
                  acc[u][e + i] = red2(mm + mul_mont(x1, B4[i]));
                  xs[NX - 1][u][e + i] = mm;
                }
              }
            }
          } else {
            // acc = m1 + (C - A) x0
#pragma unroll
            for (int u = 0; u < GPT; ++u) {
              const uint32_t* wc = wrow + 2 * (uint64_t)(uint32_t)Nc + (tid + u * T) * 4;
#pragma unroll
              for (int e = 0; e < 16; e += 4) {
                const uint4 vc = *reinterpret_cast<const uint4*>(wc + (e / 4) * (N2 / 4));
                const uint32_t C4[4] = {vc.x, vc.y, vc.z, vc.w};
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  acc[u][e + i] = red2(xs[NX - 1][u][e + i] + mul_mont(xs[0][u][e + i], C4[i]));
              }
            }
          }
        }
      }
      if (!three) static_for<0, NX>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const uint32_t* wr = (desc ? desc->W : a.W + (uint64_t)(o - c + NX - 1) * (uint32_t)Nc) +
                             (uint64_t)row * N2;
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
          const uint32_t* wg = wr + (tid + u * T) * 4;
#pragma unroll
          for (int e = 0; e < 16; e += 4) {
            const uint4 w = *reinterpret_cast<const uint4*>(wg + (e / 4) * (N2 / 4));
            acc[u][e + 0] = red2(acc[u][e + 0] + mul_mont(xs[c][u][e + 0], w.x));
            acc[u][e + 1] = red2(acc[u][e + 1] + mul_mont(xs[c][u][e + 1], w.y));
            acc[u][e + 2] = red2(acc[u][e + 2] + mul_mont(xs[c][u][e + 2], w.z));
            acc[u][e + 3] = red2(acc[u][e + 3] + mul_mont(xs[c][u][e + 3], w.w));
          }
        }
      });
#pragma unroll
      for (int u = 0; u < GPT; ++u) {
        dft_reg<16, true>(acc[u]);
        const int g = tid + u * T;
#pragma unroll
        for (int e = 0; e < 16; ++e) lds[g * 17 + e] = acc[u][e];
      }
      __syncthreads();
      static_for_down<1, K - 1>([&](auto kc) {
        round_all<LOG2, decltype(kc)::value, T, GPT, true, TPT>(tid, twi, ld_lds_k(kc), st_lds_k(kc));
        __syncthreads();
      });
      if constexpr (OUT_BITS) {
        // the row is the whole transform: position q is output bit q
        const uint64_t m = desc ? desc->m : a.m;
        const uint64_t* m_dev = desc ? (a.m_arr ? a.m_arr + desc->blk : nullptr) : a.m_dev;
        const int32_t yvalid = (int32_t)valid_bits(m, m_dev);
        const int32_t ylimit = ((int32_t)m + 63) & ~63;
        uint64_t* __restrict__ y64 = reinterpret_cast<uint64_t*>(a.y) +
                                     (desc ? (desc->y_bit >> 6) : (uint64_t)zy * (a.y_zs >> 6));
        auto st_bits = [&](int g, int e, uint32_t v) {
          const int q = G0::pos0(g) + e * G0::s;
          const uint32_t bit = (q < yvalid) ? (red1(v) & 1u) : 0u;
          const uint64_t bal = __ballot(bit);
          const int q0 = q - lane;
          if (lane == 0 && q0 < ylimit) y64[q0 >> 6] = bal;
        };
        round_all<LOG2, 0, T, GPT, true, TPT>(tid, twi, ld_lds_k(k0), st_bits);
      } else {
        uint32_t* __restrict__ dst =
            a.out + (uint64_t)(zy * a.ny + o) * (uint32_t)Nc + (uint64_t)row * N2;
        auto st0 = [&](int g, int e, uint32_t v) { dst[G0::pos0(g) + e * G0::s] = v; };
        round_all<LOG2, 0, T, GPT, true, TPT>(tid, twi, ld_lds_k(k0), st0);
      }
      __syncthreads();
    }
  }
}

template <int LOG2, int NX, int GPT, bool IN_BITS, bool SEED, bool OUT_BITS>
__global__ __launch_bounds__((row_threads<LOG2, GPT>())) void k_rows(RowArgs a, TwTables tw) {
  constexpr bool JOINT = rows_joint<NX, IN_BITS, SEED, OUT_BITS>();
  __shared__ uint32_t ldsb[(JOINT ? 2 : 1) * row_lds_words<LOG2>()];
  __shared__ uint32_t wbits[IN_BITS ? (1 << LOG2) / 32 : 1];
  if (!SEED && a.count && a.item0 + blockIdx.y >= *a.count) return;
  rows_body<LOG2, NX, GPT, IN_BITS, SEED, OUT_BITS>(a, tw, threadIdx.x, blockIdx.x, blockIdx.y,
                                                   ldsb, wbits);
}

// Two raw and two output chunks: windows (W0, W1, W2) -> (W1, W0 - W1,
// W2 - W1), the order the three-product row pass reads (values in [0, p)).
__global__ __launch_bounds__(256) void k_combine3(uint32_t* __restrict__ W, uint32_t Nc) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= Nc) return;
  const uint32_t a = W[i], b = W[Nc + i], c = W[2 * (uint64_t)Nc + i];
  W[i] = b;
  W[Nc + i] = a >= b ? a - b : a + P - b;
  W[2 * (uint64_t)Nc + i] = c >= b ? c - b : c + P - b;
}

// ------------------------------------------ persistent multi-class passes
struct McClassDev {
  int log_nc, log1, log2, rpu;  // rpu: rows per pass-B unit
  uint32_t items;
  uint32_t u0[3];   // first unit of the class in passes A, B, C
  uint32_t per[3];  // units per item in passes A, B, C
  ColFwdArgs fa;
  RowArgs rb;
  ColInvArgs ic;
};
struct McDev {
  uint32_t nclass, nest;
  uint32_t units[3];
  uint32_t* counters;
  MeBatchArgs est;
  McClassDev cls[MC_MAX];
};

// Classes keep the split of ntt_make_plan (rows of 2^10 .. 2^12 points for
// these lengths, columns of 2^6 .. 2^9), which the cached seed spectra's
// order follows.
constexpr int MC_NS = 16;  // slots of 32 columns: 512 threads
constexpr int MC_T_COLS = COLS * MC_NS;
constexpr int MC_T_ROWS = 256;  // 2 rows of 2^12 points, or 4 shorter rows
constexpr int MC_MIN_LOG1 = MC_MIN_LOG - 10, MC_MAX_LOG1 = 9;  // column lengths

// Next unit of pass P for this workgroup (all threads get it); the taker of
// unit 0 clears the counter of the pass before (pass P-1 mod 3), which has
// completed: the launches run in stream order.
template <int P>
__device__ __forceinline__ uint32_t mc_next(const McDev* __restrict__ d, uint32_t* slot) {
  if (threadIdx.x == 0) {
    const uint32_t u = atomicAdd(&d->counters[P], 1u);
    if (u == 0) atomicExch(&d->counters[(P + 2) % 3], 0u);
    *slot = u;
  }
  __syncthreads();
  // the same value in every lane: keep it (and all that follows from it,
  // the class and its arguments) in scalar registers
  const uint32_t u = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();
  return u;
}

// the class of unit u of pass P (classes are in unit order)
template <int P>
__device__ __forceinline__ int mc_class(const McDev* __restrict__ d, uint32_t u) {
  int c = 0;
  while (c + 1 < (int)d->nclass && u >= d->cls[c + 1].u0[P]) ++c;
  return c;
}

// The tables as seen by one unit: the empty asm makes each pointer look
// rewritten, so the compiler cannot hoist a unit's table loads out of the
// unit loop (they would stay live, in registers, across all units).
__device__ __forceinline__ TwTables fresh_tables(const TwTables& tw) {
  TwTables t = tw;
  asm volatile("" : "+s"(t.fwd), "+s"(t.inv), "+s"(t.fwd_t), "+s"(t.inv_t), "+s"(t.g_lo),
               "+s"(t.g_hi));
  return t;
}

template <int L, int E, class F>
__device__ __forceinline__ void static_switch(int v, F&& f) {
  if constexpr (L <= E) {
    if (v == L)
      f(std::integral_constant<int, L>{});
    else
      static_switch<L + 1, E>(v, f);
  }
}

__global__ __launch_bounds__(MC_T_COLS, 4) void k_mc_cols_fwd(const McDev* __restrict__ d,
                                                          TwTables tw) {
  __shared__ __align__(16) uint32_t lds[(1 << MC_MAX_LOG1) * COLS];
  __shared__ uint32_t wbits[1 << MC_MAX_LOG1];
  __shared__ uint32_t slot;
  for (;;) {
    const uint32_t u = mc_next<0>(d, &slot);
    if (u >= d->units[0]) return;
    const McClassDev& C = d->cls[mc_class<0>(d, u)];
    const uint32_t local = u - C.u0[0];
    const int item = (int)(local / C.per[0]), tile = (int)(local % C.per[0]);
    const TwTables t = fresh_tables(tw);
    static_switch<MC_MIN_LOG1, MC_MAX_LOG1>(C.log1, [&](auto l) {
      cols_fwd_body<decltype(l)::value, MC_NS, false>(C.fa, t, tile, item, lds, wbits);
    });
  }
}

// The estimate unit as a call of its own: inlined, its double-precision
// code and the row transform would share one register allocation.
__device__ __noinline__ void mc_estimate_unit(const MeBatchArgs* a, uint32_t b, uint32_t* lds) {
  hd::block_estimate_body<MC_T_ROWS>(*a, b, lds,
                                     reinterpret_cast<double*>(lds + ((hd::HC * hd::HB + 1) & ~1)));
}

__global__ __launch_bounds__(MC_T_ROWS) void k_mc_rows(const McDev* __restrict__ d,
                                                      TwTables tw) {
  // MC_T_ROWS / row_threads rows of one item per unit, one per thread group
  constexpr int RW = (row_lds_words<12>() + 1) & ~1;  // 8-byte aligned
  static_assert(2 * row_threads<12, 2>() == MC_T_ROWS && 4 * row_threads<11, 2>() == MC_T_ROWS &&
                    4 * row_threads<10, 1>() == MC_T_ROWS && 4 * row_lds_words<11>() <= 2 * RW,
                "rows per workgroup");
  constexpr int EW = ((hd::HC * hd::HB + 1) & ~1) + 2 * hd::me_lds_doubles(MC_T_ROWS);
  __shared__ __align__(16) uint32_t lds[2 * RW > EW ? 2 * RW : EW];
  __shared__ uint32_t slot;
  for (;;) {
    const uint32_t u = mc_next<1>(d, &slot);
    if (u >= d->units[1]) return;
    if (u < d->nest) {
      mc_estimate_unit(&d->est, u, lds);  // block u's estimate: the m pass C reads
      continue;
    }
    const McClassDev& C = d->cls[mc_class<1>(d, u)];
    const uint32_t local = u - C.u0[1];
    const int item = (int)(local / C.per[1]);
    const int row0 = (int)(local % C.per[1]) * C.rpu;
    const TwTables t = fresh_tables(tw);
    if (C.log2 == 12) {
      constexpr int RT = row_threads<12, 2>();
      const int g = threadIdx.x / RT;
      rows_body<12, 1, 2, false, false, false>(C.rb, t, threadIdx.x - g * RT, row0 + g, item,
                                               lds + g * RW, nullptr);
    } else if (C.log2 == 11) {
      constexpr int RT = row_threads<11, 2>();
      const int g = threadIdx.x / RT;
      rows_body<11, 1, 2, false, false, false>(C.rb, t, threadIdx.x - g * RT, row0 + g, item,
                                               lds + g * row_lds_words<11>(), nullptr);
    } else {
      constexpr int RT = row_threads<10, 1>();
      const int g = threadIdx.x / RT;
      rows_body<10, 1, 1, false, false, false>(C.rb, t, threadIdx.x - g * RT, row0 + g, item,
                                               lds + g * row_lds_words<10>(), nullptr);
    }
  }
}

__global__ __launch_bounds__(MC_T_COLS, 4) void k_mc_cols_inv(const McDev* __restrict__ d,
                                                          TwTables tw) {
  __shared__ uint32_t lds[(1 << MC_MAX_LOG1) * COLS];
  __shared__ uint32_t slot;
  for (;;) {
    const uint32_t u = mc_next<2>(d, &slot);
    if (u >= d->units[2]) return;
    const McClassDev& C = d->cls[mc_class<2>(d, u)];
    const uint32_t local = u - C.u0[2];
    const int item = (int)(local / C.per[2]), tile = (int)(local % C.per[2]);
    const TwTables t = fresh_tables(tw);
    static_switch<MC_MIN_LOG1, MC_MAX_LOG1>(C.log1, [&](auto l) {
      cols_inv_body<decltype(l)::value, MC_NS, false>(C.ic, t, tile, item, lds);
    });
  }
}

// ------------------------------------------------------------ dispatch
template <int LOG1>
hipError_t launch_cols_fwd(const ColFwdArgs& a, dim3 grid, const TwTables& tw, hipStream_t s) {
  prof_begin(KID_COLS_FWD, s);
  hipLaunchKernelGGL(k_cols_fwd<LOG1>, grid, dim3(COLS * cslots<LOG1, false>()), 0, s, a, tw);
  prof_end(KID_COLS_FWD, s);
  return hipGetLastError();
}
template <int LOG1>
hipError_t launch_cols_inv(const ColInvArgs& a, dim3 grid, const TwTables& tw, hipStream_t s) {
  prof_begin(KID_COLS_INV, s);
  hipLaunchKernelGGL(k_cols_inv<LOG1>, grid, dim3(COLS * cslots<LOG1, true>()), 0, s, a, tw);
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

// groups of the last round per thread: 2 where a row has >= 128 groups
template <int LOG2>
constexpr int row_gpt() {
  return LOG2 >= 11 ? 2 : 1;
}

template <int LOG2, int NX, bool IN_BITS, bool SEED, bool OUT_BITS>
hipError_t launch_rows(const RowArgs& a, dim3 grid, const TwTables& tw, hipStream_t s) {
  constexpr int kid = IN_BITS ? (SEED ? KID_FUSED_SEED : KID_FUSED_HASH)
                              : (SEED ? KID_ROWS_SEED : KID_ROWS_HASH);
  constexpr int G = row_gpt<LOG2>();
  prof_begin(kid, s);
  hipLaunchKernelGGL((k_rows<LOG2, NX, G, IN_BITS, SEED, OUT_BITS>), grid,
                     dim3(row_threads<LOG2, G>()), 0, s, a, tw);
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
    case 15:
      // 2^15 points (139 KB of LDS) only as a whole transform in one workgroup
      if constexpr (IN_BITS && NX == 1) return launch_rows<15, NX, IN_BITS, SEED, OUT_BITS>(a, grid, tw, s);
      break;
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
          // transposed copy
          fwd[TW_TOTAL + off + ap * s + b] = make_uint2(f, shoup_q(f));
          inv[TW_TOTAL + off + ap * s + b] = make_uint2(g, shoup_q(g));
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
  // row sums are at most n < p; m may exceed n (the modified Toeplitz block)
  if (n == 0 || m == 0 || n >= P) return false;
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
  if (k <= MAX_LOG_FUSED) {
    p->log1 = 0;
    p->log2 = k;
  } else {
    // columns of 2^6 .. 2^9 points, rows of 2^10 .. 2^14; 2^9-point columns
    // where the rows allow, except at 2^17 and 2^18 points, where 2^11-point
    // rows (columns of 2^6 and 2^7) are 3-4 % faster on batches of blocks
    int l2 = (k == 17 || k == 18) ? 11 : k - 9;
    l2 = l2 < 10 ? 10 : (l2 > MAX_LOG_ROW ? MAX_LOG_ROW : l2);
    p->log2 = l2;
    p->log1 = k - l2;
  }
  p->nwin = p->nx + p->ny - 1;
  return true;
}

uint64_t ntt_seed_elems(const NttPlan& p) { return (uint64_t)p.nwin << p.log_nc; }

uint64_t ntt_work_elems(const NttPlan& p, int batch) {
  if (p.log1 == 0) return 0;
  // one transform: pass B overwrites pass A's residues row by row
  const uint64_t per = (p.nx == 1 && p.ny == 1) ? 1 : (uint64_t)(p.nx + p.ny);
  return (uint64_t)batch * per << p.log_nc;
}

hipError_t ntt_seed_spectra(const NttPlan& p, const uint32_t* seed_bits, uint64_t n,
                            uint64_t m, uint64_t seed_avail, uint32_t* W, uint32_t* work,
                            const TwTables& tw, hipStream_t s) {
  const uint64_t L = n + m - 1;
  const int64_t Nc = (int64_t)1 << p.log_nc;
  if (p.nwin > MAXMAP) return hipErrorInvalidValue;
  BitMap maps[MAXMAP];
  if (p.nx == 1 && p.ny == 1) {
    // one transform: the first Nc seed bits, whatever n and m (the raw block
    // carries the n-1 rotation, see ntt_hash)
    const uint64_t hi = seed_avail < (uint64_t)Nc ? seed_avail : (uint64_t)Nc;
    maps[0] = BitMap{0, 0, (int32_t)hi, (int32_t)Nc};
  } else {
    for (int w = 0; w < p.nwin; ++w) {
      const int64_t d = w - (p.nx - 1);
      maps[w] = BitMap{(int32_t)((int64_t)n - 1 + d * p.by), 0, (int32_t)L, (int32_t)p.by};
    }
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
  e = rows_l<1, false, true, false>(p.log2, r, dim3(1u << p.log1, p.nwin), tw, s);
  if (e != hipSuccess || !(p.nx == 2 && p.ny == 2)) return e;
  hipLaunchKernelGGL(k_combine3, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, s, W,
                     (uint32_t)Nc);
  return hipGetLastError();
}

hipError_t ntt_hash(const NttPlan& p, const uint32_t* x_bits, uint64_t n, uint64_t m,
                    const uint32_t* W, uint32_t* y_bits, uint32_t* work, int batch,
                    uint64_t x_stride_bits, uint64_t y_stride_bits, const TwTables& tw,
                    hipStream_t s, const uint64_t* m_dev, const EstJob* est) {
  const int64_t Nc = (int64_t)1 << p.log_nc;
  if (est && (batch != 1 || !ntt_fuses_estimate(p))) return hipErrorInvalidValue;
  RowArgs r{};
  r.W = W;
  r.nx = p.nx;
  r.ny = p.ny;
  r.log_nc = p.log_nc;
  r.y = y_bits;
  r.y_zs = y_stride_bits;
  r.m = m;
  r.m_dev = m_dev;
  if (p.log1 == 0) {
    r.bits = x_bits;
    r.zs = x_stride_bits;
    r.map[0] = rotated_block((uint32_t)n, (int32_t)Nc);
    return rows_l<1, true, false, true>(p.log2, r, dim3(1, batch), tw, s);
  }
  uint32_t* X = work;
  uint32_t* Z = (p.nx == 1 && p.ny == 1) ? X : work + ((uint64_t)batch * p.nx << p.log_nc);
  ColFwdArgs c{};
  c.bits = x_bits;
  c.zs = x_stride_bits;
  for (int k = 0; k < p.nx; ++k) {
    const int64_t lo = (int64_t)k * p.bx;
    const int64_t hi = lo + p.bx < (int64_t)n ? lo + p.bx : (int64_t)n;
    c.map[k] = BitMap{(int32_t)lo, (int32_t)lo, (int32_t)hi, (int32_t)Nc};
  }
  if (p.nx == 1 && p.ny == 1) c.map[0] = rotated_block((uint32_t)n, (int32_t)Nc);
  else c.upper_zero = 2 * p.bx <= Nc;  // chunk k covers positions q < bx only
  c.nmap = p.nx;
  c.log2 = p.log2;
  c.log_nc = p.log_nc;
  c.out = X;
  if (est) {
    c.est.s = est->samples;
    c.est.S = est->S;
    c.est.N = 8;
    c.est.part = est->scratch;
    c.est.G = hd::hist_groups(est->S);
    c.est.counts = nullptr;
    c.est.finish = true;
    c.est.me = est->me;
    c.est.epoch = est->epoch;
    c.est.expect = est->epoch ^ est->expect_xor;
    c.hg = c.est.G;
    c.ticket = est->scratch + hd::TICKET_WORD;
  }
  hipError_t e = cols_fwd(p.log1, c, dim3((1u << p.log2) / COLS + c.hg, batch * p.nx), tw, s);
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
  ci.m_dev = m_dev;
  return cols_inv(p.log1, ci, dim3((1u << p.log2) / COLS, batch * p.ny), tw, s);
}

bool ntt_fuses_estimate(const NttPlan& p) { return p.log1 >= EST_MIN_LOG1; }

bool ntt_plan_for_length(int log_nc, NttPlan* p) {
  if (log_nc < 10 || log_nc > LOG_MAX) return false;
  const uint64_t Nc = 1ull << log_nc;
  // n = m = Nc/2 gives L = Nc - 1, whose plan has exactly this length
  return ntt_make_plan(Nc / 2, Nc / 2, p) && p->log_nc == log_nc;
}

hipError_t ntt_hash_items(const NttPlan& p, const uint32_t* x_pool, const NttItem* items,
                          int count, uint32_t* y_pool, const uint64_t* m_arr, uint32_t* work,
                          const TwTables& tw, hipStream_t s) {
  if (p.nx != 1 || p.ny != 1) return hipErrorInvalidValue;
  if (count <= 0) return hipSuccess;
  RowArgs r{};
  r.nx = r.ny = 1;
  r.log_nc = p.log_nc;
  r.y = y_pool;
  r.bits = x_pool;
  r.items = items;
  r.m_arr = m_arr;
  if (p.log1 == 0) return rows_l<1, true, false, true>(p.log2, r, dim3(1, count), tw, s);
  ColFwdArgs c{};
  c.bits = x_pool;
  c.nmap = 1;
  c.log2 = p.log2;
  c.log_nc = p.log_nc;
  c.out = work;
  c.items = items;
  hipError_t e = cols_fwd(p.log1, c, dim3((1u << p.log2) / COLS, count), tw, s);
  if (e != hipSuccess) return e;
  r.in = work;
  r.out = work;
  e = rows_l<1, false, false, false>(p.log2, r, dim3(1u << p.log1, count), tw, s);
  if (e != hipSuccess) return e;
  ColInvArgs ci{};
  ci.in = work;
  ci.ny = 1;
  ci.log2 = p.log2;
  ci.log_nc = p.log_nc;
  ci.y = y_pool;
  ci.by = (int64_t)1 << p.log_nc;
  ci.items = items;
  ci.m_arr = m_arr;
  return cols_inv(p.log1, ci, dim3((1u << p.log2) / COLS, count), tw, s);
}

hipError_t ntt_hash_items_dev(const NttPlan& p, const uint32_t* x_pool, const NttItem* items,
                              const uint32_t* count, uint32_t item0, int grid_items,
                              uint32_t* y_pool, uint32_t* work, const TwTables& tw,
                              hipStream_t s) {
  if (p.nx != 1 || p.ny != 1) return hipErrorInvalidValue;
  if (grid_items <= 0) return hipSuccess;
  items += item0;
  RowArgs r{};
  r.nx = r.ny = 1;
  r.log_nc = p.log_nc;
  r.y = y_pool;
  r.bits = x_pool;
  r.items = items;
  r.count = count;
  r.item0 = item0;
  if (p.log1 == 0) return rows_l<1, true, false, true>(p.log2, r, dim3(1, grid_items), tw, s);
  ColFwdArgs c{};
  c.bits = x_pool;
  c.nmap = 1;
  c.log2 = p.log2;
  c.log_nc = p.log_nc;
  c.out = work;
  c.items = items;
  c.count = count;
  c.item0 = item0;
  hipError_t e = cols_fwd(p.log1, c, dim3((1u << p.log2) / COLS, grid_items), tw, s);
  if (e != hipSuccess) return e;
  r.in = work;
  r.out = work;
  e = rows_l<1, false, false, false>(p.log2, r, dim3(1u << p.log1, grid_items), tw, s);
  if (e != hipSuccess) return e;
  ColInvArgs ci{};
  ci.in = work;
  ci.ny = 1;
  ci.log2 = p.log2;
  ci.log_nc = p.log_nc;
  ci.y = y_pool;
  ci.by = (int64_t)1 << p.log_nc;
  ci.items = items;
  ci.count = count;
  ci.item0 = item0;
  return cols_inv(p.log1, ci, dim3((1u << p.log2) / COLS, grid_items), tw, s);
}

uint64_t mc_args_bytes() { return sizeof(McDev); }

bool mc_build(void* host_image, McInfo* info, int nclass, const int* log_nc,
              const uint32_t* items, const NttItem* const* items_dev, uint32_t* const* work,
              const uint32_t* x_pool, uint32_t* y_pool, const uint64_t* m_arr,
              const MeBatchArgs* est, uint32_t nest, uint32_t* counters) {
  if (nclass < 0 || nclass > MC_MAX) return false;
  McDev* d = static_cast<McDev*>(host_image);
  std::memset(d, 0, sizeof(McDev));
  d->nclass = (uint32_t)nclass;
  d->nest = est ? nest : 0;
  if (est) d->est = *est;
  d->counters = counters;
  uint64_t u[3] = {0, d->nest, 0};
  for (int c = 0; c < nclass; ++c) {
    const int k = log_nc[c];
    if (k < MC_MIN_LOG || k > MC_MAX_LOG || (c && k > log_nc[c - 1])) return false;
    McClassDev& C = d->cls[c];
    NttPlan np;
    if (!ntt_plan_for_length(k, &np) || np.log1 < MC_MIN_LOG1 || np.log1 > MC_MAX_LOG1 || np.log2 < 10 ||
        np.log2 > 12)
      return false;
    const int l2 = np.log2;  // the split the cached seed spectra are laid out for
    C.log_nc = k;
    C.log2 = l2;
    C.log1 = k - l2;
    C.rpu = l2 == 12 ? 2 : 4;
    C.items = items[c];
    C.per[0] = C.per[2] = (1u << l2) / COLS;
    C.per[1] = (1u << C.log1) / C.rpu;
    for (int p = 0; p < 3; ++p) {
      C.u0[p] = (uint32_t)u[p];
      u[p] += (uint64_t)C.items * C.per[p];
    }
    C.fa.bits = x_pool;
    C.fa.nmap = 1;
    C.fa.log2 = l2;
    C.fa.log_nc = k;
    C.fa.out = work[c];
    C.fa.items = items_dev[c];
    C.rb.nx = C.rb.ny = 1;
    C.rb.log_nc = k;
    C.rb.in = work[c];
    C.rb.out = work[c];
    C.rb.items = items_dev[c];
    C.rb.bits = x_pool;
    C.rb.y = y_pool;
    C.rb.m_arr = m_arr;
    C.ic.in = work[c];
    C.ic.ny = 1;
    C.ic.log2 = l2;
    C.ic.log_nc = k;
    C.ic.y = y_pool;
    C.ic.by = (int64_t)1 << k;
    C.ic.items = items_dev[c];
    C.ic.m_arr = m_arr;
  }
  for (int p = 0; p < 3; ++p) {
    if (u[p] >= (1ull << 32)) return false;
    d->units[p] = (uint32_t)u[p];
  }
  info->nclass = (uint32_t)nclass;
  for (int p = 0; p < 3; ++p) info->units[p] = d->units[p];
  info->nest = d->nest;
  info->counters = counters;
  return true;
}

uint32_t mc_grid(int pass, int num_cus) {
  int per = 0;
  const void* f = pass == 0 ? (const void*)k_mc_cols_fwd
                            : (pass == 1 ? (const void*)k_mc_rows : (const void*)k_mc_cols_inv);
  const int threads = pass == 1 ? MC_T_ROWS : MC_T_COLS;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, threads, 0) != hipSuccess || per < 1)
    per = 1;
  return (uint32_t)per * (uint32_t)num_cus;
}

hipError_t mc_launch(int pass, const void* dev_args, const McInfo& info, uint32_t grid,
                     const TwTables& tw, hipStream_t s) {
  const uint32_t units = info.units[pass];
  if (units == 0) return hipSuccess;
  const uint32_t g = grid < units ? grid : units;
  const McDev* d = static_cast<const McDev*>(dev_args);
  if (pass == 0) {
    prof_begin(KID_COLS_FWD, s);
    hipLaunchKernelGGL(k_mc_cols_fwd, dim3(g), dim3(MC_T_COLS), 0, s, d, tw);
    prof_end(KID_COLS_FWD, s);
  } else if (pass == 1) {
    prof_begin(KID_ROWS_HASH, s);
    hipLaunchKernelGGL(k_mc_rows, dim3(g), dim3(MC_T_ROWS), 0, s, d, tw);
    prof_end(KID_ROWS_HASH, s);
  } else {
    prof_begin(KID_COLS_INV, s);
    hipLaunchKernelGGL(k_mc_cols_inv, dim3(g), dim3(MC_T_COLS), 0, s, d, tw);
    prof_end(KID_COLS_INV, s);
  }
  return hipGetLastError();
}

}  // namespace qrng

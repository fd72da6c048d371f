// Toeplitz hashing of many equal blocks that share one seed on the int8
// matrix cores (paper Sec. III.B, the direct product k = T r; here for a
// whole batch at once, so it becomes a true matrix-matrix product).
//
// With B blocks as the columns of X (n x B, raw bits as int8 0/1) and
// A[i][j] = s[n-1+i-j] (the m x n Toeplitz matrix as int8), Y = A X holds
// in column b the integer row sums of block b; each is at most n, so int32
// accumulation is exact and the hash bit is Y & 1.
//
// Tiling (gfx950, v_mfma_i32_32x32x32_i8, wave64): a workgroup owns 128
// output rows x 256 blocks; each wave owns 64 blocks and all 128 rows
// (eight 32x32 accumulators).  B fragments (raw bits) are built in registers
// from the wave's own blocks; A fragments (the Toeplitz matrix) come from an
// LDS copy of the reversed seed window expanded to bytes, shared by the four
// waves.  Per 32-bit K-step a wave issues 8 MFMAs.  Fragment layout: lane l
// holds row or column l % 32 and 16 k-values of lane group l / 32 (the same
// k order on A and B, so the contraction over k is exact whatever the
// hardware's order).
#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int MT = 128;  // rows per workgroup
constexpr int KC = 512;  // raw bits per K-chunk

// 4 bits -> 4 bytes holding 0/1 (bit t to the low bit of byte t)
__device__ __forceinline__ uint32_t expand4(uint32_t nib) {
  return (nib * 0x00204081u) & 0x01010101u;
}
// 16 bits -> 16 bytes
__device__ __forceinline__ v4i expand16(uint32_t w) {
  v4i r;
  r.x = (int)expand4(w & 15u);
  r.y = (int)expand4((w >> 4) & 15u);
  r.z = (int)expand4((w >> 8) & 15u);
  r.w = (int)expand4((w >> 12) & 15u);
  return r;
}

// 32 bits of a bit string starting at bit p (may be negative or run past
// nbits: those bits read as 0).
__device__ __forceinline__ uint32_t bits32_at(const uint32_t* __restrict__ s, int64_t p,
                                              int64_t nbits) {
  const int64_t w = p >> 5;  // floor division
  const uint32_t sh = (uint32_t)(p & 31);
  const int64_t nw = (nbits + 31) >> 5;
  const uint32_t lo = (w >= 0 && w < nw) ? s[w] : 0u;
  const uint32_t hi = (w + 1 >= 0 && w + 1 < nw) ? s[w + 1] : 0u;
  uint32_t v = sh ? ((lo >> sh) | (hi << (32u - sh))) : lo;
  // clear bits at or past nbits, and below 0
  const int64_t top = nbits - p;  // valid bits from p
  if (top < 32) v &= top <= 0 ? 0u : ((1u << (uint32_t)top) - 1u);
  if (p < 0) v &= (p <= -32) ? 0u : ~((1u << (uint32_t)(-p)) - 1u);
  return v;
}

struct MfmaArgs {
  const uint32_t* x;  // raw bits; block b at bit b * x_zs (x_zs a multiple of 32)
  uint64_t x_zs;
  const uint32_t* seed;
  uint64_t n, m, L;
  uint32_t* y;  // output bits; block b at bit b * y_zs (multiple of 64)
  uint64_t y_zs;
  uint32_t nblocks;
  const uint64_t* m_dev;  // nullable: valid rows computed on the device
};

constexpr int WNB = 2;             // 32-block tiles per wave
constexpr int NTB = 4 * 32 * WNB;  // blocks per workgroup (4 waves)
constexpr int KW = KC / 32;        // raw words per block per K-chunk
constexpr int XROW = KW + 1;       // padded LDS row (words) of one block's chunk
constexpr int RSPAN = MT + KC;     // bytes of one shifted copy of the seed window
constexpr int RWORDS = RSPAN / 4 + 4;  // dwords of the window copy (+ read slack)

// Workgroup tile: MT = 128 rows x NTB = 256 blocks.  Wave w owns blocks
// 64w..64w+63 and all four 32-row tiles (8 accumulators).  A[i][k] =
// s[n-1+i-k]: for rows i0+ri and k = k0+kk the seed index is base - u with
// u = (MT-1) - ri + kk and base = n-1+i0-k0+MT-1, so one K-chunk needs the
// seed bits base-u, u < MT+KC, reversed ("rs[u]"), one byte each in LDS.
// An A fragment (16 consecutive u from any byte offset) is five dword reads
// and four byte-aligns.  Raw bits are staged per K-chunk with 16-byte loads.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mfma(MfmaArgs a) {
  // two buffers: chunk k is multiplied from one while chunk k+1 is staged
  // into the other, so each chunk needs one barrier
  __shared__ uint32_t rs[2][RWORDS];
  __shared__ uint32_t xs[2][NTB * XROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * MT;
  const int64_t n = (int64_t)a.n, L = (int64_t)a.L;
  const uint32_t bg = blockIdx.y * NTB;  // workgroup's first block
  uint64_t mv = a.m;
  if (a.m_dev && *a.m_dev < mv) mv = *a.m_dev;
  const int64_t nsw = (L + 31) >> 5;

  v16i acc[4][WNB];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < WNB; ++u)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[t][u][r] = 0;

  const int kg = 16 * (lane >> 5);  // lane group's k offset within a K-step
  const int rl = lane & 31;

  // Global reads of one K-chunk, issued one chunk ahead into registers:
  // NTB*KW raw words, 16 bytes per load (XPT per thread; four lanes read
  // one block's 64-byte run), and for threads j < RWORDS the two seed words
  // that hold window dword j's four bits.
  constexpr int XPT = NTB * KW / (4 * 256);
  static_assert(NTB * KW % (4 * 256) == 0 && KW % 4 == 0, "raw words per thread");
  static_assert(RWORDS <= 256, "one window dword per thread");
  const int64_t nw32 = 2 * (((int64_t)a.n + 63) >> 6);  // readable 32-bit words of a block
  // thread's raw rows: block bg + tid/4 + 64 e, words 4 (tid % 4) .. + 3
  const uint32_t b0 = bg + (uint32_t)(tid >> 2);
  const int q0 = 4 * (tid & 3);
  const uint64_t bstride = (uint64_t)64 * a.x_zs >> 5;  // words between e and e+1
  const uint32_t* xrow = a.x + ((uint64_t)b0 * a.x_zs >> 5) + q0;
  const bool full_group = bg + NTB <= a.nblocks;
  uint4 pre_x[XPT];
  uint32_t pre_s0 = 0, pre_s1 = 0;
  auto seed_word = [&](int64_t w) -> uint32_t {
    uint32_t v = (w >= 0 && w < nsw) ? a.seed[w] : 0u;
    const int64_t top = L - 32 * w;  // bits of word w below L
    if (top < 32) v &= top <= 0 ? 0u : ((1u << (uint32_t)top) - 1u);
    return v;
  };
  auto fetch = [&](int64_t k0) {
    const int64_t base = n - 1 + i0 - k0 + (MT - 1);
    if (tid < RWORDS) {
      // window dword tid: seed bits base-4 tid-3 .. base-4 tid
      const int64_t p = base - 4 * tid - 3;
      const int64_t w = p >> 5;  // floor
      pre_s0 = seed_word(w);
      pre_s1 = ((p & 31) > 28) ? seed_word(w + 1) : 0u;
    }
    const int64_t kw = k0 >> 5;
    if (full_group && k0 + KC <= n) {
      // whole chunk inside every block: plain 16-byte loads
#pragma unroll
      for (int e = 0; e < XPT; ++e)
        pre_x[e] = *reinterpret_cast<const uint4*>(xrow + e * bstride + kw);
      return;
    }
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
      const uint32_t b = b0 + 64 * e;
      const int64_t w0 = kw + q0;  // first word within the block
      uint32_t v[4] = {0u, 0u, 0u, 0u};
      if (b < a.nblocks) {
        const uint32_t* src = xrow + e * bstride + kw;
        if (w0 + 3 < nw32) {
          const uint4 t = *reinterpret_cast<const uint4*>(src);
          v[0] = t.x;
          v[1] = t.y;
          v[2] = t.z;
          v[3] = t.w;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (w0 + i < nw32) v[i] = src[i];
        }
        // bits at or past n read as 0
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t kb = 32 * (w0 + i);
          if (kb >= n)
            v[i] = 0u;
          else if (kb + 32 > n)
            v[i] &= (1u << (uint32_t)(n - kb)) - 1u;
        }
      }
      pre_x[e] = make_uint4(v[0], v[1], v[2], v[3]);
    }
  };
  // write the prefetched chunk (window start base) into buffer c
  auto stage = [&](int c, int64_t k0) {
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
      uint32_t* dst = xs[c] + ((tid >> 2) + 64 * e) * XROW + q0;
      dst[0] = pre_x[e].x;
      dst[1] = pre_x[e].y;
      dst[2] = pre_x[e].z;
      dst[3] = pre_x[e].w;
    }
    if (tid < RWORDS) {
      // bytes 4j .. 4j+3 = seed bits base-4j down to base-4j-3 (j = tid)
      const int64_t base = n - 1 + i0 - k0 + (MT - 1);
      const uint32_t ps = (uint32_t)((base - 4 * tid - 3) & 31);
      uint32_t w4 = pre_s0 >> ps;
      if (ps > 28) w4 |= pre_s1 << (32 - ps);
      const uint32_t rev = (__builtin_bitreverse32(w4 & 15u) >> 28) & 15u;
      rs[c][tid] = expand4(rev);
    }
  };
  fetch(0);
  stage(0, 0);
  __syncthreads();
  int c = 0;
  for (int64_t k0 = 0; k0 < n; k0 += KC, c ^= 1) {
    const bool more = k0 + KC < n;
    if (more) fetch(k0 + KC);
    const uint32_t* rsc = rs[c];
    const uint32_t* xsc = xs[c];
    // A fragment of row tile t at K-step ks: rows ri = 32t + rl, k offset
    // kk = 32 ks + kg, u0 = MT-1 - ri + kk.  The matrix is Toeplitz, so
    // (t, ks) and (t+1, ks+1) have the same u0: after the first K-step of a
    // chunk only tile 0's fragment is new, the others move down one tile.
    auto a_frag = [&](int t, int ks) {
      const int u0 = (MT - 1) - (32 * t + rl) + 32 * ks + kg;
      const int w = u0 >> 2;
      const uint32_t sh = (uint32_t)(u0 & 3);
      const uint32_t d0 = rsc[w], d1 = rsc[w + 1], d2 = rsc[w + 2], d3 = rsc[w + 3],
                     d4 = rsc[w + 4];
      v4i f;
      f.x = (int)__builtin_amdgcn_alignbyte(d1, d0, sh);
      f.y = (int)__builtin_amdgcn_alignbyte(d2, d1, sh);
      f.z = (int)__builtin_amdgcn_alignbyte(d3, d2, sh);
      f.w = (int)__builtin_amdgcn_alignbyte(d4, d3, sh);
      return f;
    };
    v4i af[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) af[t] = a_frag(t, 0);
#pragma unroll
    for (int ks = 0; ks < KW; ++ks) {
      if (ks > 0) {
        af[3] = af[2];
        af[2] = af[1];
        af[1] = af[0];
        af[0] = a_frag(0, ks);
      }
      v4i bf[WNB];
#pragma unroll
      for (int u = 0; u < WNB; ++u) {
        const int bl = wave * 32 * WNB + 32 * u + rl;
        bf[u] = expand16((xsc[bl * XROW + ks] >> kg) & 0xFFFFu);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < WNB; ++u)
          acc[t][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[t], bf[u], acc[t][u], 0, 0, 0);
    }
    if (more) stage(c ^ 1, k0 + KC);
    __syncthreads();
  }

  // D layout: lane l holds column l % 32 (a block) and rows
  // 8 (r / 4) + 4 (l / 32) + r % 4 of each accumulator, r < 16
  const uint32_t bw = bg + wave * 32 * WNB;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < WNB; ++u) {
      uint32_t w = 0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        w |= ((uint32_t)acc[t][u][r] & 1u) << row;
      }
      w |= __shfl_xor(w, 32);
      const uint32_t b = bw + 32 * u + rl;
      const int64_t it = i0 + 32 * t;
      if (lane < 32 && b < a.nblocks && it < (int64_t)a.m) {
        const int64_t valid = (int64_t)mv - it;  // rows past the valid length are 0
        if (valid < 32) w &= valid <= 0 ? 0u : ((1u << (uint32_t)valid) - 1u);
        a.y[((uint64_t)b * a.y_zs + (uint64_t)it) >> 5] = w;
      }
    }
}

// zero the 32-bit word after the last written one where ceil(m/32) is odd,
// so each block's last 64-bit word has no stale high half
__global__ __launch_bounds__(256) void k_tail(uint32_t* __restrict__ y, uint64_t y_zs,
                                              uint64_t m, uint32_t nblocks) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b < nblocks) y[((uint64_t)b * y_zs >> 5) + (m + 31) / 32] = 0u;
}

}  // namespace

hipError_t mfma_hash(const uint32_t* x_bits, uint64_t n, const uint32_t* seed_bits, uint64_t m,
                     uint32_t* y_bits, int batch, uint64_t x_stride_bits,
                     uint64_t y_stride_bits, hipStream_t s, const uint64_t* m_dev) {
  MfmaArgs a{};
  a.x = x_bits;
  a.x_zs = x_stride_bits;
  a.seed = seed_bits;
  a.n = n;
  a.m = m;
  a.L = n + m - 1;
  a.y = y_bits;
  a.y_zs = y_stride_bits;
  a.nblocks = (uint32_t)batch;
  a.m_dev = m_dev;
  const dim3 grid((unsigned)((m + MT - 1) / MT), (unsigned)((batch + NTB - 1) / NTB));
  prof_begin(KID_MFMA, s);
  hipLaunchKernelGGL(k_mfma, grid, dim3(256), 0, s, a);
  if (((m + 31) / 32) & 1)
    hipLaunchKernelGGL(k_tail, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, y_bits,
                       y_stride_bits, m, (uint32_t)batch);
  prof_end(KID_MFMA, s);
  return hipGetLastError();
}

}  // namespace qrng

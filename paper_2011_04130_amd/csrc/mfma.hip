// Toeplitz hashing of many equal blocks that share one seed on the matrix
// cores (paper Sec. III.B, the direct product k = T r; here for a whole batch
// at once, so it becomes a true matrix-matrix product).
//
// With B blocks as the columns of X (n x B, raw bits as 0/1) and A[i][j] =
// s[n-1+i-j] (the m x n Toeplitz matrix), Y = A X holds in column b the
// integer row sums of block b, and Y & 1 is block b's hash.
//
// Operands are fp4 (e2m1) on the gfx950 scaled matrix instructions
// (v_mfma_scale_f32_32x32x64_f8f6f4, unit scales) with fp32 accumulation: 0
// and 1 are exact fp4 codes (0b0000, 0b0010), each instruction adds 64
// products that are 0 or 1, and every partial sum is an integer of at most
// n < 2^24, so the fp32 accumulator holds the exact row sum whatever the
// order of the additions.  One such instruction contracts 64 k-values in the
// issue time of the int8 instruction's 32.
//
// Tiling: a workgroup owns 256 output rows x 128 blocks; each wave owns 32
// blocks and all eight 32-row tiles (eight 32x32 accumulators), so the
// wave's raw-bit fragment, which takes VALU work to expand to fp4, feeds
// eight instructions.  A fragments (the Toeplitz matrix) come from an LDS
// copy of the reversed seed window already expanded to fp4, shared by the
// four waves.  Fragment layout: lane l holds row or column l % 32 and 32
// k-values of lane group l / 32 (dword q, nibble i: k = 32 (l / 32) + 8 q +
// i), the same k order on A and B, so the contraction over k is exact
// whatever order the hardware adds in.
#include "common.h"
#include "internal.h"

namespace qrng {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

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

constexpr int MT = 256;            // rows per workgroup (8 tiles of 32)
constexpr int NTB = 128;           // blocks per workgroup (4 waves x 32)
constexpr int KC = 512;            // raw bits per K-chunk
constexpr int KW = KC / 32;        // raw words per block per K-chunk
constexpr int KS = KC / 64;        // instructions per tile per K-chunk
constexpr int XROW = KW + 1;       // padded LDS row (words) of one block's chunk
constexpr int RSPAN = MT + KC;     // nibbles of one shifted copy of the seed window
constexpr int RWORDS = RSPAN / 8 + 5;  // dwords of the window copy (+ read slack)
constexpr uint32_t SCALE_ONE = 0x7F;   // E8M0 exponent of 1.0

// 8 bits -> 8 nibbles: bit i to bit 4i + 1 (fp4 1.0 = 0b0010, 0 = 0b0000)
__device__ __forceinline__ uint32_t spread8(uint32_t b) {
  uint32_t x = (b & 0xFFu) << 1;
  x = (x | (x << 12)) & 0x001E001Eu;
  x = (x | (x << 6)) & 0x06060606u;
  x = (x | (x << 3)) & 0x22222222u;
  return x;
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mfma(MfmaArgs a) {
  typedef float v16f __attribute__((ext_vector_type(16)));
  typedef int v8i __attribute__((ext_vector_type(8)));
  __shared__ uint32_t rs[2][RWORDS];
  __shared__ uint32_t xs[2][NTB * XROW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * MT;
  const int64_t n = (int64_t)a.n, L = (int64_t)a.L;
  const uint32_t bg = blockIdx.y * NTB;
  uint64_t mv = a.m;
  if (a.m_dev && *a.m_dev < mv) mv = *a.m_dev;
  const int64_t nsw = (L + 31) >> 5;

  v16f acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.0f;

  const int g = lane >> 5;
  const int rl = lane & 31;

  // raw words of one K-chunk, one chunk ahead in registers: thread's rows are
  // blocks bg + tid/4 + 64 e, words 4 (tid % 4) .. + 3
  constexpr int XPT = NTB * KW / (4 * 256);
  static_assert(NTB * KW % (4 * 256) == 0 && KW % 4 == 0, "raw words per thread");
  static_assert(RWORDS <= 256, "one window dword per thread");
  const int64_t nw32 = 2 * (((int64_t)a.n + 63) >> 6);
  const uint32_t b0 = bg + (uint32_t)(tid >> 2);
  const int q0 = 4 * (tid & 3);
  const uint64_t bstride = (uint64_t)64 * a.x_zs >> 5;
  const uint32_t* xrow = a.x + ((uint64_t)b0 * a.x_zs >> 5) + q0;
  const bool full_group = bg + NTB <= a.nblocks;
  uint4 pre_x[XPT];
  uint32_t pre_s0 = 0, pre_s1 = 0;
  auto seed_word = [&](int64_t w) -> uint32_t {
    uint32_t v = (w >= 0 && w < nsw) ? a.seed[w] : 0u;
    const int64_t top = L - 32 * w;
    if (top < 32) v &= top <= 0 ? 0u : ((1u << (uint32_t)top) - 1u);
    return v;
  };
  auto fetch = [&](int64_t k0) {
    const int64_t base = n - 1 + i0 - k0 + (MT - 1);
    if (tid < RWORDS) {
      // window dword tid: seed bits base-8 tid-7 .. base-8 tid
      const int64_t p = base - 8 * tid - 7;
      const int64_t w = p >> 5;
      pre_s0 = seed_word(w);
      pre_s1 = ((p & 31) > 24) ? seed_word(w + 1) : 0u;
    }
    const int64_t kw = k0 >> 5;
    if (full_group && k0 + KC <= n) {
#pragma unroll
      for (int e = 0; e < XPT; ++e)
        pre_x[e] = *reinterpret_cast<const uint4*>(xrow + e * bstride + kw);
      return;
    }
#pragma unroll
    for (int e = 0; e < XPT; ++e) {
      const uint32_t b = b0 + 64 * e;
      const int64_t w0 = kw + q0;
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
      // nibbles 8j .. 8j+7 = seed bits base-8j down to base-8j-7 (j = tid)
      const int64_t base = n - 1 + i0 - k0 + (MT - 1);
      const uint32_t ps = (uint32_t)((base - 8 * tid - 7) & 31);
      uint32_t w8 = pre_s0 >> ps;
      if (ps > 24) w8 |= pre_s1 << (32 - ps);
      rs[c][tid] = spread8(__builtin_bitreverse32(w8 & 0xFFu) >> 24);
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
    // A fragment of row tile t at step ks: rows 32t + rl, k = 64 ks + 32 g +
    // j, u0 = MT-1 - (32t + rl) + 64 ks + 32 g = ub - 32 t + 64 ks.  Tiles
    // (t, ks) and (t+2, ks+1) share u0, so after a chunk's first step only
    // tiles 0, 1 are new.  The nibble shift ub % 8 is the same for every
    // (t, ks), and the dword index moves by constants (LDS immediate offsets).
    const int ub = (MT - 1) - rl + 32 * g;
    const uint32_t sh = (uint32_t)(ub & 7) * 4u;
    const uint32_t* rpb = rsc + (ub >> 3);
    auto a_frag = [&](int t, int ks) {
      const uint32_t* rp = rpb + (8 * ks - 4 * t);
      const uint32_t d0 = rp[0], d1 = rp[1], d2 = rp[2], d3 = rp[3], d4 = rp[4];
      v4i f;
      f.x = (int)__builtin_amdgcn_alignbit(d1, d0, sh);
      f.y = (int)__builtin_amdgcn_alignbit(d2, d1, sh);
      f.z = (int)__builtin_amdgcn_alignbit(d3, d2, sh);
      f.w = (int)__builtin_amdgcn_alignbit(d4, d3, sh);
      return f;
    };
    v4i af[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) af[t] = a_frag(t, 0);
    const int bl = wave * 32 + rl;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (ks > 0) {
#pragma unroll
        for (int t = 7; t >= 2; --t) af[t] = af[t - 2];
        af[1] = a_frag(1, ks);
        af[0] = a_frag(0, ks);
      }
      const uint32_t xw = xsc[bl * XROW + 2 * ks + g];
      // fp4 operands take the low four dwords of the eight-dword argument
      const v4i z4 = {0, 0, 0, 0};
      v4i b4;
      b4.x = (int)spread8(xw);
      b4.y = (int)spread8(xw >> 8);
      b4.z = (int)spread8(xw >> 16);
      b4.w = (int)spread8(xw >> 24);
      const v8i bf = __builtin_shufflevector(b4, z4, 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const v8i a8 = __builtin_shufflevector(af[t], z4, 0, 1, 2, 3, 4, 5, 6, 7);
        acc[t] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, bf, acc[t], 4, 4, 0,
                                                                 SCALE_ONE, 0, SCALE_ONE);
      }
    }
    if (more) stage(c ^ 1, k0 + KC);
    __syncthreads();
  }

  // D layout: lane l holds column l % 32 (a block) and rows
  // 8 (r / 4) + 4 (l / 32) + r % 4 of each accumulator, r < 16
  const uint32_t b = bg + wave * 32 + rl;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    uint32_t w = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      w |= ((uint32_t)acc[t][r] & 1u) << row;
    }
    w |= __shfl_xor(w, 32);
    const int64_t it = i0 + 32 * t;
    if (lane < 32 && b < a.nblocks && it < (int64_t)a.m) {
      const int64_t valid = (int64_t)mv - it;
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
  prof_begin(KID_MFMA, s);
  const dim3 grid((unsigned)((m + MT - 1) / MT), (unsigned)((batch + NTB - 1) / NTB));
  hipLaunchKernelGGL(k_mfma, grid, dim3(256), 0, s, a);
  if (((m + 31) / 32) & 1)
    hipLaunchKernelGGL(k_tail, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, y_bits,
                       y_stride_bits, m, (uint32_t)batch);
  prof_end(KID_MFMA, s);
  return hipGetLastError();
}

}  // namespace qrng

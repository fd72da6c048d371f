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
// blocks and all eight 32-row tiles (eight 32x32 accumulators).  Fragment
// layout: lane l holds row or column l % 32 and 32 k-values of lane group
// l / 32, dword q nibble i holding k = 32 (l / 32) + 4 i + q on both A and B
// (any order common to both gives the same sums).  So B's dword q is the
// raw word's bits q, q+4, ..., q+28 moved to the nibbles' 1.0 bit, one
// shift and one mask; and an A fragment depends only on where its window
// starts, so each K-chunk builds in LDS a table with one 16-byte row per
// window start (the four dwords of the fragment starting there, shared by
// the four waves) and every A fragment is one 16-byte LDS read.
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
constexpr int KC = 1024;           // raw bits per K-chunk
constexpr int KW = KC / 32;        // raw words per block per K-chunk
constexpr int KS = KC / 64;        // instructions per tile per K-chunk
constexpr int XROW = KW + 1;       // padded LDS row (words) of one block's chunk
constexpr int NV = MT + KC;        // window starts of one K-chunk (fragment table rows)
constexpr int VPT = NV / 256;      // table rows each thread builds
constexpr uint32_t FP4_ONES = 0x22222222u;  // fp4 1.0 (0b0010) in every nibble
constexpr uint32_t SCALE_ONE = 0x7F;   // E8M0 exponent of 1.0

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_mfma(MfmaArgs a) {
  typedef float v16f __attribute__((ext_vector_type(16)));
  typedef int v8i __attribute__((ext_vector_type(8)));
  __shared__ uint4 fv[2][NV];
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

  // raw words of one K-chunk, one chunk ahead in registers: TPB threads
  // share a block's KW words (16 bytes each); thread's rows are blocks
  // bg + tid/TPB + BPE e, words 4 (tid % TPB) .. + 3
  constexpr int TPB = KW / 4, BPE = 256 / TPB;
  constexpr int XPT = NTB / BPE;
  static_assert(KW % 4 == 0 && 256 % TPB == 0 && NTB % BPE == 0, "raw words per thread");
  static_assert(VPT * 256 == NV, "fragment table rows per thread");
  const int64_t nw32 = 2 * (((int64_t)a.n + 63) >> 6);
  const uint32_t b0 = bg + (uint32_t)(tid / TPB);
  const int q0 = 4 * (tid % TPB);
  const uint64_t bstride = (uint64_t)BPE * a.x_zs >> 5;
  const uint32_t* xrow = a.x + ((uint64_t)b0 * a.x_zs >> 5) + q0;
  const bool full_group = bg + NTB <= a.nblocks;
  uint4 pre_x[XPT];
  uint32_t pre_s[3] = {0u, 0u, 0u};
  auto seed_word = [&](int64_t w) -> uint32_t {
    uint32_t v = (w >= 0 && w < nsw) ? a.seed[w] : 0u;
    const int64_t top = L - 32 * w;
    if (top < 32) v &= top <= 0 ? 0u : ((1u << (uint32_t)top) - 1u);
    return v;
  };
  auto fetch = [&](int64_t k0) {
    const int64_t base = n - 1 + i0 - k0 + (MT - 1);
    {
      // table rows v = VPT tid + e read the 32 seed bits from base - v - 31:
      // together the bits from base - VPT tid - 31 - (VPT - 1), three words
      const int64_t wb = (base - VPT * tid - 31 - (VPT - 1)) >> 5;
      pre_s[0] = seed_word(wb);
      pre_s[1] = seed_word(wb + 1);
      pre_s[2] = seed_word(wb + 2);
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
      const uint32_t b = b0 + BPE * e;
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
      uint32_t* dst = xs[c] + (tid / TPB + BPE * e) * XROW + q0;
      dst[0] = pre_x[e].x;
      dst[1] = pre_x[e].y;
      dst[2] = pre_x[e].z;
      dst[3] = pre_x[e].w;
    }
    {
      // row v: dword q, nibble i = value u = v + 4i + q, i.e. seed bit
      // base - v - q - 4i = bit 31 - q - 4i of the 32 bits w from base - v -
      // 31; after the bit reversal R, that is bit 4i + q, moved to the
      // nibble's 1.0 bit (4i + 1) by one shift and one mask
      const int64_t p0 = n - 1 + i0 - k0 + (MT - 1) - VPT * tid - 31;
      const uint32_t o0 = (uint32_t)((p0 - (VPT - 1)) & 31);
#pragma unroll
      for (int e = 0; e < VPT; ++e) {
        const uint32_t o = o0 + (VPT - 1) - e;  // bit offset in the three words, < 32 + VPT
        const uint32_t w = o < 32 ? __builtin_amdgcn_alignbit(pre_s[1], pre_s[0], o)
                                  : __builtin_amdgcn_alignbit(pre_s[2], pre_s[1], o - 32);
        const uint32_t R = __builtin_bitreverse32(w);
        fv[c][VPT * tid + e] = make_uint4((R << 1) & FP4_ONES, R & FP4_ONES,
                                          (R >> 1) & FP4_ONES, (R >> 2) & FP4_ONES);
      }
    }
  };
  fetch(0);
  stage(0, 0);
  __syncthreads();
  int c = 0;
  for (int64_t k0 = 0; k0 < n; k0 += KC, c ^= 1) {
    const bool more = k0 + KC < n;
    if (more) fetch(k0 + KC);
    const uint4* fvc = fv[c];
    const uint32_t* xsc = xs[c];
    // A fragment of row tile t at step ks: rows 32t + rl, dword q nibble i =
    // k 64 ks + 32 g + 4i + q, i.e. value u0 + 4i + q with u0 = MT-1 - (32t +
    // rl) + 64 ks + 32 g = ub - 32 t + 64 ks: table row u0, one 16-byte
    // read at a per-lane address plus a constant.  Tiles (t, ks) and (t+2,
    // ks+1) share u0, so after a chunk's first step only tiles 0, 1 are new.
    const uint4* fvb = fvc + ((MT - 1) - rl + 32 * g);
    auto a_frag = [&](int t, int ks) {
      const uint4 d = fvb[64 * ks - 32 * t];
      v4i f;
      f.x = (int)d.x;
      f.y = (int)d.y;
      f.z = (int)d.z;
      f.w = (int)d.w;
      return f;
    };
    v4i af[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) af[t] = a_frag(t, 0);
    const int bl = wave * 32 + rl;
    // the chunk's steps in runs of eight (the register names of the fragment
    // rotation repeat every four steps, so a run ends where it began)
#pragma unroll 1
    for (int kh = 0; kh < KS; kh += 8)
#pragma unroll
    for (int kq = 0; kq < 8; ++kq) {
      const int ks = kh + kq;
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
      b4.x = (int)((xw << 1) & FP4_ONES);
      b4.y = (int)(xw & FP4_ONES);
      b4.z = (int)((xw >> 1) & FP4_ONES);
      b4.w = (int)((xw >> 2) & FP4_ONES);
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

// Issue-cost probe for single VALU instructions (a measurement aid for the
// ALU rooflines, not part of the hash path).  Every lane runs eight
// independent chains of one instruction (no dependency between consecutive
// instructions of a wave), enough waves fill every SIMD, and the only memory
// access is one store per lane at the end, so the kernel time over the
// instruction count gives the cycles a SIMD spends per wave64 instruction.
#include "internal.h"

namespace qrng {

namespace {

constexpr int PROBE_T = 256;         // threads per workgroup (4 waves)
constexpr int PROBE_UNROLL = 4;      // blocks of 8 instructions per loop turn
constexpr int PROBE_WAVES_SIMD = 8;  // resident waves per SIMD the grid provides

// eight independent chains: x_i = op(x_i, k) (one instruction each)
#define QRNG_CHAIN8(OP)                                                                          \
  asm volatile(OP " %0, %0, %8\n" OP " %1, %1, %8\n" OP " %2, %2, %8\n" OP " %3, %3, %8\n"      \
               OP " %4, %4, %8\n" OP " %5, %5, %8\n" OP " %6, %6, %8\n" OP " %7, %7, %8\n"      \
               : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7) \
               : "v"(k))

template <int OP>
__global__ __launch_bounds__(PROBE_T) void k_issue_probe(uint32_t* out, int iters, uint32_t seed) {
  uint32_t a0 = threadIdx.x + seed, a1 = a0 * 3u, a2 = a0 * 5u, a3 = a0 * 7u;
  uint32_t a4 = a0 * 11u, a5 = a0 * 13u, a6 = a0 * 17u, a7 = a0 * 19u;
  uint64_t b0 = a0, b1 = a1, b2 = a2, b3 = a3, b4 = a4, b5 = a5, b6 = a6, b7 = a7;
  const uint32_t k = seed | 1u;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < PROBE_UNROLL; ++r) {
      if constexpr (OP == 0) QRNG_CHAIN8("v_add_u32");
      if constexpr (OP == 1) QRNG_CHAIN8("v_sub_u32");
      if constexpr (OP == 2) QRNG_CHAIN8("v_min_u32");
      if constexpr (OP == 3) QRNG_CHAIN8("v_xor_b32");
      if constexpr (OP == 4) QRNG_CHAIN8("v_mul_lo_u32");
      if constexpr (OP == 5) QRNG_CHAIN8("v_mul_hi_u32");
      if constexpr (OP == 6)
        asm volatile(
            "v_mad_u64_u32 %0, vcc, %8, %9, %0\n v_mad_u64_u32 %1, vcc, %8, %9, %1\n"
            "v_mad_u64_u32 %2, vcc, %8, %9, %2\n v_mad_u64_u32 %3, vcc, %8, %9, %3\n"
            "v_mad_u64_u32 %4, vcc, %8, %9, %4\n v_mad_u64_u32 %5, vcc, %8, %9, %5\n"
            "v_mad_u64_u32 %6, vcc, %8, %9, %6\n v_mad_u64_u32 %7, vcc, %8, %9, %7\n"
            : "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3), "+v"(b4), "+v"(b5), "+v"(b6), "+v"(b7)
            : "v"(a0), "v"(k)
            : "vcc");
      if constexpr (OP == 7)
        asm volatile(
            "v_bitop3_b32 %0, %0, %8, %8 bitop3:0x78\n v_bitop3_b32 %1, %1, %8, %8 bitop3:0x78\n"
            "v_bitop3_b32 %2, %2, %8, %8 bitop3:0x78\n v_bitop3_b32 %3, %3, %8, %8 bitop3:0x78\n"
            "v_bitop3_b32 %4, %4, %8, %8 bitop3:0x78\n v_bitop3_b32 %5, %5, %8, %8 bitop3:0x78\n"
            "v_bitop3_b32 %6, %6, %8, %8 bitop3:0x78\n v_bitop3_b32 %7, %7, %8, %8 bitop3:0x78\n"
            : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
            : "v"(k));
    }
  }
  out[blockIdx.x * PROBE_T + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7 ^
                                            (uint32_t)(b0 ^ b1 ^ b2 ^ b3 ^ b4 ^ b5 ^ b6 ^ b7);
}
#undef QRNG_CHAIN8

const char* const kOpNames[PROBE_OPS] = {"v_add_u32",    "v_sub_u32",    "v_min_u32",
                                         "v_xor_b32",    "v_mul_lo_u32", "v_mul_hi_u32",
                                         "v_mad_u64_u32", "v_bitop3_b32"};

template <int OP>
hipError_t launch_probe(uint32_t* out, int grid, int iters, uint32_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_issue_probe<OP>, dim3(grid), dim3(PROBE_T), 0, s, out, iters, seed);
  return hipGetLastError();
}

hipError_t launch_op(int op, uint32_t* out, int grid, int iters, uint32_t seed, hipStream_t s) {
  switch (op) {
    case 0: return launch_probe<0>(out, grid, iters, seed, s);
    case 1: return launch_probe<1>(out, grid, iters, seed, s);
    case 2: return launch_probe<2>(out, grid, iters, seed, s);
    case 3: return launch_probe<3>(out, grid, iters, seed, s);
    case 4: return launch_probe<4>(out, grid, iters, seed, s);
    case 5: return launch_probe<5>(out, grid, iters, seed, s);
    case 6: return launch_probe<6>(out, grid, iters, seed, s);
    case 7: return launch_probe<7>(out, grid, iters, seed, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

const char* probe_op_name(int op) { return op >= 0 && op < PROBE_OPS ? kOpNames[op] : nullptr; }

uint64_t probe_out_words(int num_cus) {
  return (uint64_t)num_cus * 4 * PROBE_WAVES_SIMD * 64;
}

hipError_t probe_issue_cycles(int op, int num_cus, double clock_ghz, uint32_t* out,
                              hipStream_t s, double* cycles) {
  if (op < 0 || op >= PROBE_OPS || num_cus <= 0 || clock_ghz <= 0) return hipErrorInvalidValue;
  // PROBE_WAVES_SIMD waves on each of 4 SIMDs per CU; out holds one word per lane
  const int grid = num_cus * 4 * PROBE_WAVES_SIMD / (PROBE_T / 64);
  const int iters = 2000;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_op(op, out, grid, iters, 12345u, s);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch_op(op, out, grid, iters, 777u, s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return e;
  // wave instructions per SIMD: waves per SIMD x loop turns x 8 x unroll
  const double per_simd = (double)PROBE_WAVES_SIMD * iters * 8 * PROBE_UNROLL;
  *cycles = (double)ms * 1e-3 * clock_ghz * 1e9 / per_simd;
  return hipSuccess;
}

}  // namespace qrng

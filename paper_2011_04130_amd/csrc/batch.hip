// Device-side scheduling of a batch whose descriptors live in device memory
// (paper Sec. III.E: a raw sequence cut into blocks, here of uneven lengths,
// each block hashed as in Sec. III.B with the first n+m-1 bits of its seed).
// One thread per descriptor checks it and appends it to the item list of its
// transform length Nc = 2^ceil(log2(n+m-1)) (at least 2^10), pointing at the
// registered seed's cached spectrum of that length; the class launches that
// follow read the list lengths on the device, so the host never needs to see
// the descriptors and the whole batch can be captured in a HIP graph.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace qrng {

namespace {

__global__ __launch_bounds__(64) void k_batch_clear(uint32_t* __restrict__ counts) {
  if (threadIdx.x < BATCH_COUNTS) counts[threadIdx.x] = 0u;
}

__device__ __forceinline__ int ceil_log2_dev(uint64_t v) {
  return v <= 1 ? 0 : 64 - __builtin_clzll(v - 1);
}

__global__ __launch_bounds__(256) void k_batch_classify(const qrng_block* __restrict__ blocks,
                                                        uint32_t nblocks,
                                                        const uint32_t* __restrict__ seed_ids,
                                                        const DevSeed* __restrict__ table,
                                                        NttItem* __restrict__ items, uint32_t cap,
                                                        int max_log,
                                                        uint32_t* __restrict__ counts) {
  const uint32_t b = blockIdx.x * 256u + threadIdx.x;
  if (b >= nblocks) return;
  const qrng_block d = blocks[b];
  const uint32_t sid = seed_ids ? seed_ids[b] : d.seed_id;
  // the single-block call's checks: 0 < n, m <= n, a known seed long enough
  // for n+m-1 bits; this path also needs n < 2^31 and one transform of at
  // most 2^max_log points (the longest class the launches cover)
  bool ok = d.flags == 0 && d.n > 0 && d.m <= d.n && d.n < (1ull << 31) && sid > 0 &&
            sid < (uint32_t)SEED_TABLE_CAP;
  if (ok && d.m > 0) {
    const uint64_t L = d.n + d.m - 1;
    const uint64_t sl = table[sid].L;
    ok = sl > 0 && L <= sl && L <= (1ull << max_log);
    if (ok) {
      int k = ceil_log2_dev(L);
      if (k < BATCH_MIN_LOG) k = BATCH_MIN_LOG;
      const uint32_t* W = table[sid].W[k];
      ok = W != nullptr;
      if (ok) {
        const uint32_t i = atomicAdd(&counts[k - BATCH_MIN_LOG], 1u);
        NttItem it;
        it.x_bit = d.x_word_off * 64;
        it.y_bit = d.y_word_off * 64;
        it.W = W;
        it.n = (uint32_t)d.n;
        it.m = (uint32_t)d.m;
        it.blk = b;
        it.pad = 0;
        items[(uint64_t)(k - BATCH_MIN_LOG) * cap + i] = it;
      }
    }
  } else if (ok && table[sid].L == 0) {
    ok = false;  // m = 0 is a no-op, but only for a known seed
  }
  if (!ok) atomicAdd(&counts[BATCH_REJECTED], 1u);
}

}  // namespace

hipError_t batch_classify(const qrng_block* blocks, uint32_t nblocks, const uint32_t* seed_ids,
                          const DevSeed* table, NttItem* items, uint32_t cap, int max_log,
                          uint32_t* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_clear, dim3(1), dim3(64), 0, s, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nblocks == 0) return e;
  hipLaunchKernelGGL(k_batch_classify, dim3((nblocks + 255) / 256), dim3(256), 0, s, blocks,
                     nblocks, seed_ids, table, items, cap, max_log, counts);
  return hipGetLastError();
}

}  // namespace qrng

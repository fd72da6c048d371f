// Histogram of N-bit ADC samples (one byte each) and the min-entropy estimate
// of paper Sec. II on the device (P'(x) is the observed frequency of each
// sample value; the model P, H_min, d_U, Delta H_m and H_modify follow), with
// the output length m of Sec. III.B.
//
// Two launches: every workgroup of the first counts its slice of the
// samples into LDS sub-histograms and stores their sum as its partial
// histogram; one workgroup of the second adds the partials up and computes
// the estimate (thread v owns value v).  (A single launch whose last
// workgroup finishes, as estimate_workgroup does inside the transform's
// first pass, measured slower on its own than the launch boundary: with a
// device-scope fence per workgroup, an L2 write-back each on this multi-die
// part; with the rows stored write-through, the 1024-thread finish at the
// end of the counting.)  Values >= 2^N are counted apart so the host can
// reject them.
#include <math.h>

#include "common.h"
#include "hist_dev.h"
#include "internal.h"
#include "qrng.h"

namespace qrng {

using namespace hd;

namespace {

// threads of a counting workgroup
constexpr int PART_T = 1024;

__global__ __launch_bounds__(PART_T) void k_hist_part(HistArgs a) {
  __shared__ uint32_t h[HC * HB];
  hist_part_body<PART_T, HC>(a, blockIdx.x, h);
}

__global__ __launch_bounds__(PART_T) void k_hist_part_subset(HistArgs a) {
  __shared__ uint32_t h[HC * HB];
  hist_part_body<PART_T, HC, false, true>(a, blockIdx.x, h);
}

__global__ __launch_bounds__(256) void k_hist_finish(HistArgs a) {
  __shared__ FinishLds L;
  hist_finish_body<256>(a, L);
}

// One workgroup per block of an uneven batch (block_estimate_body).
__global__ __launch_bounds__(256) void k_block_estimate(MeBatchArgs a) {
  __shared__ uint32_t h[HC * HB];
  __shared__ double lds[me_lds_doubles(256)];
  block_estimate_body<256>(a, blockIdx.x, h, lds);
}

}  // namespace

uint64_t hist_scratch_words() { return TICKET_WORD + 64; }
uint64_t hist_ticket_word() { return TICKET_WORD; }

hipError_t hist_estimate(const uint8_t* samples, uint64_t S, int N, uint32_t* scratch,
                         unsigned long long* counts_out, const MeDevArgs* finish,
                         hipStream_t s, uint64_t subset_seed, uint32_t keep_thr,
                         uint32_t epoch, uint32_t expect_xor) {
  HistArgs a{};
  a.epoch = epoch;
  a.expect = epoch ^ expect_xor;
  a.s = samples;
  a.S = S;
  a.N = N;
  a.subset_seed = subset_seed;
  a.keep_thr = keep_thr;
  a.part = scratch;
  a.G = hist_groups(S);
  a.counts = counts_out;
  a.finish = finish != nullptr;
  if (finish) a.me = *finish;
  prof_begin(KID_HIST, s);
  if (keep_thr)
    hipLaunchKernelGGL(k_hist_part_subset, dim3(a.G), dim3(PART_T), 0, s, a);
  else
    hipLaunchKernelGGL(k_hist_part, dim3(a.G), dim3(PART_T), 0, s, a);
  hipLaunchKernelGGL(k_hist_finish, dim3(1), dim3(256), 0, s, a);
  prof_end(KID_HIST, s);
  return hipGetLastError();
}

hipError_t minentropy_blocks(const MeBatchArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  prof_begin(KID_HIST, s);
  hipLaunchKernelGGL(k_block_estimate, dim3(nblocks), dim3(256), 0, s, a);
  prof_end(KID_HIST, s);
  return hipGetLastError();
}

}  // namespace qrng

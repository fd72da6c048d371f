// C ABI of libqrng (declared in include/qrng.h): argument validation, device
// context, workspace and seed-spectrum cache, path selection, and the host
// part of the min-entropy estimate (paper Sec. II).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "qrng.h"
#include "internal.h"
#include "host_logic.h"

using namespace qrng;

namespace qrng {
const char* kernel_name(int kid) {
  static const char* names[KID_COUNT] = {"ntt_cols_fwd", "ntt_rows_hash", "ntt_rows_seed",
                                         "ntt_cols_inv", "ntt_fused_hash", "ntt_fused_seed",
                                         "direct",       "direct_prep",   "histogram",
                                         "mfma",         "modified_tail", "fft64"};
  return (kid >= 0 && kid < KID_COUNT) ? names[kid] : nullptr;
}
}  // namespace qrng

namespace {

thread_local std::string g_err;

qrng_status fail(qrng_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(QRNG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

struct Seed {
  const uint64_t* ptr;
  uint64_t L;
  uint32_t plans = 0;  // live plans and servers that use this seed
  // transform-domain seed windows for the NTT path: key (0, Nc) for one
  // transform of length Nc (shared by every block shape that fits it), key
  // (n, m) for the block-Toeplitz plans above 2^23 bits
  std::map<std::pair<uint64_t, uint64_t>, uint32_t*> spectra;
};

std::pair<uint64_t, uint64_t> spectra_key(const NttPlan& p, uint64_t n, uint64_t m) {
  if (p.nx == 1 && p.ny == 1) return {0, 1ull << p.log_nc};
  return {n, m};
}

bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

bool overlap(const void* a, uint64_t abytes, const void* b, uint64_t bbytes) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

uint64_t words64(uint64_t bits) { return (bits + 63) / 64; }

// Test-only fault injection, read from the environment on every call:
// QRNG_FAULT=launch makes the hash and estimate entry points fail with
// QRNG_EDEVICE before they enqueue anything; =ticket leaves a stale ticket
// (another call's tag, a partial count) before the fused estimate, as a
// launch that never completed would; =rows makes the estimate's finish
// expect another call's tag, so its consistency check fails.
enum Fault { FAULT_NONE = 0, FAULT_LAUNCH, FAULT_TICKET, FAULT_ROWS };
int fault_mode() {
  const char* e = std::getenv("QRNG_FAULT");
  if (!e) return FAULT_NONE;
  if (!std::strcmp(e, "launch")) return FAULT_LAUNCH;
  if (!std::strcmp(e, "ticket")) return FAULT_TICKET;
  if (!std::strcmp(e, "rows")) return FAULT_ROWS;
  return FAULT_NONE;
}

int ceil_log2_u64(uint64_t v) {
  int k = 0;
  while (k < 64 && (1ull << k) < v) ++k;
  return k;
}

// Scratch of qrng_toeplitz_hash_noalloc: one copy per device, alive until the
// process ends.  Host code never passes this name to a kernel (on the host it
// is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returned for the current device (qrng_ctx::noalloc).
constexpr uint64_t kNoAllocWords = QRNG_NOALLOC_SCRATCH_BYTES / 4;
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct ProfRec {
  int kid;
  hipEvent_t a, b;
};

struct qrng_ctx {
  int device = 0;
  // kernel timing (measurement aid)
  bool prof_on = false;
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> prof_pool;
  hipEvent_t prof_open = nullptr;
  int num_cus = 256;
  uint2* tw_fwd = nullptr;
  uint2* tw_inv = nullptr;
  uint32_t* g_lo = nullptr;
  uint32_t* g_hi = nullptr;
  TwTables tw{};
  uint32_t* work = nullptr;  // general workspace
  uint64_t work_words = 0;
  unsigned long long* counts_dev = nullptr;
  uint32_t* hist_scratch = nullptr;           // partial histograms + ticket (zeroed once)
  unsigned long long* counts_host = nullptr;  // pinned
  uint32_t* noalloc = nullptr;  // this device's copy of `scratch` (device address)
  uint32_t est_epoch = 0;       // tag of the latest histogram call (below 2^23)
  // device-descriptor batches: the device's view of the seed registry, the
  // per-class item lists with their counts, and the transform workspace
  DevSeed* seed_table = nullptr;  // SEED_TABLE_CAP entries
  NttItem* batch_items = nullptr;
  uint32_t* batch_counts = nullptr;
  uint32_t batch_cap = 0;
  uint32_t* batch_work = nullptr;
  uint64_t batch_work_bytes = 0;
  qrng_me_result* me_dev = nullptr;           // qrng_extract's default result slot
  uint64_t* m_dev = nullptr;                  // and output-length slot
  std::map<uint32_t, Seed> seeds;  // ids 1 .. SEED_TABLE_CAP - 1, lowest free id first
  std::set<qrng_plan*> plans;
  std::set<qrng_server*> servers;
  // autotuned launch shape per transform-length class: (log2 Nc, ceil log2
  // of the class size) -> sub-batch workspace cap as log2 bytes, or
  // kTuneDirect for one direct launch per block
  std::map<std::pair<int, int>, int> tune;
  // the times (ms) of every candidate the last tuning run measured, per key
  std::map<std::pair<int, int>, std::vector<std::pair<int, float>>> tune_ms;
};

namespace {

thread_local qrng_ctx* t_ctx = nullptr;

// Makes `c` the context whose timing hooks the kernel launches of this
// thread report to, for the duration of one C-ABI call.
struct CtxScope {
  qrng_ctx* prev;
  explicit CtxScope(qrng_ctx* c) : prev(t_ctx) { t_ctx = c; }
  ~CtxScope() { t_ctx = prev; }
};

hipEvent_t prof_event(qrng_ctx* c) {
  if (!c->prof_pool.empty()) {
    hipEvent_t e = c->prof_pool.back();
    c->prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_release(qrng_ctx* c) {
  for (auto& r : c->prof_recs) {
    c->prof_pool.push_back(r.a);
    c->prof_pool.push_back(r.b);
  }
  c->prof_recs.clear();
}

qrng_status ensure_work(qrng_ctx* c, uint64_t words) {
  if (words <= c->work_words) return QRNG_OK;
  if (c->work) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipFree(c->work));
    c->work = nullptr;
    c->work_words = 0;
  }
  uint64_t want = std::max<uint64_t>(words, 1u << 20);
  if (hipMalloc(&c->work, want * 4) != hipSuccess)
    return fail(QRNG_ENOMEM, "workspace of %llu bytes", (unsigned long long)(want * 4));
  c->work_words = want;
  return QRNG_OK;
}

qrng_status check_hash_args(qrng_ctx* ctx, const uint64_t* x, uint64_t n, const uint64_t* seed,
                            uint64_t m, const uint64_t* y, int path) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  if (!x || !seed || !y) return fail(QRNG_EINVAL, "null buffer");
  if (!aligned8(x) || !aligned8(seed) || !aligned8(y))
    return fail(QRNG_EINVAL, "buffers must be 8-byte aligned");
  if (n == 0) return fail(QRNG_EINVAL, "n must be positive");
  if (m > n) return fail(QRNG_EINVAL, "m (%llu) exceeds n (%llu)", (unsigned long long)m,
                         (unsigned long long)n);
  if (path < QRNG_PATH_AUTO || path > QRNG_PATH_MFMA) return fail(QRNG_EINVAL, "unknown path");
  if (m == 0) return QRNG_OK;
  const uint64_t L = n + m - 1;
  if (overlap(y, words64(m) * 8, x, words64(n) * 8))
    return fail(QRNG_EINVAL, "output overlaps the raw block");
  if (overlap(y, words64(m) * 8, seed, words64(L) * 8))
    return fail(QRNG_EINVAL, "output overlaps the seed");
  return QRNG_OK;
}

// Default path choice: the direct product costs m n / 32 bit-ops, the
// transform about 40 (n+m) log2(n+m) modular ops; the single-block crossover
// on MI355X sits near n = 2^15.  Many blocks sharing a seed make the fp4
// matrix-core product (cost m n per block) the fastest while m n stays within
// that of n = 2^16 at m = 5n/8 (measured on 2^30-bit batches at m = 5n/8,
// matrix cores against the transform: 905 vs 105 Gbit/s at n = 2^12, 319 vs
// 95 at 2^14, 170 vs 83 at 2^15, 114 vs 62 at 3 2^14, 86.6 vs 82.5 at 2^16,
// 43.7 vs 81 at 2^17).
int choose_path(uint64_t n, uint64_t m, uint64_t batch = 1) {
  if (batch >= 32 && n * m <= (5ull << 29)) return QRNG_PATH_MFMA;
  if (n < (1u << 15)) return QRNG_PATH_DIRECT;
  NttPlan p;
  if (!ntt_make_plan(n, m, &p)) return QRNG_PATH_DIRECT;
  return QRNG_PATH_NTT;
}

qrng_status run_direct(qrng_ctx* ctx, const uint64_t* x, uint64_t n, const uint64_t* seed,
                       uint64_t m, uint64_t* y, hipStream_t s, int batch, uint64_t xs,
                       uint64_t ys, const uint64_t* m_dev) {
  // the seed is read through a buffer resource with 32-bit byte offsets
  if (n + m - 1 >= (1ull << 34))
    return fail(QRNG_EINVAL, "direct path: n + m - 1 must be below 2^34");
  qrng_status st = ensure_work(ctx, direct_work_words(n, batch));
  if (st) return st;
  HIP_TRY(direct_hash(reinterpret_cast<const uint32_t*>(x), n,
                      reinterpret_cast<const uint32_t*>(seed), m, reinterpret_cast<uint32_t*>(y),
                      ctx->work, ctx->num_cus, s, batch, xs, ys, m_dev));
  return QRNG_OK;
}

// NTT hash; W == nullptr computes the seed windows into the workspace first.
qrng_status run_ntt(qrng_ctx* ctx, const uint64_t* x, uint64_t n, const uint64_t* seed,
                    const uint32_t* W, uint64_t m, uint64_t* y, hipStream_t s, int batch,
                    uint64_t xs, uint64_t ys, const uint64_t* m_dev,
                    const EstJob* est = nullptr) {
  NttPlan p;
  if (!ntt_make_plan(n, m, &p))
    return fail(QRNG_EUNSUPPORTED, "NTT path cannot hash n=%llu m=%llu", (unsigned long long)n,
                (unsigned long long)m);
  const uint64_t seed_words = W ? 0 : ntt_seed_elems(p);
  const uint64_t work = std::max<uint64_t>(ntt_work_elems(p, batch), ntt_work_elems(p, 1));
  qrng_status st = ensure_work(ctx, seed_words + work);
  if (st) return st;
  if (!W) {
    uint32_t* Wt = ctx->work + work;
    HIP_TRY(ntt_seed_spectra(p, reinterpret_cast<const uint32_t*>(seed), n, m, n + m - 1, Wt,
                             ctx->work, ctx->tw, s));
    W = Wt;
  }
  HIP_TRY(ntt_hash(p, reinterpret_cast<const uint32_t*>(x), n, m, W,
                   reinterpret_cast<uint32_t*>(y), ctx->work, batch, xs, ys, ctx->tw, s, m_dev,
                   est));
  return QRNG_OK;
}

// Cached seed windows of a registered seed for shape (n, m).
qrng_status seed_spectra(qrng_ctx* ctx, Seed& sd, uint64_t n, uint64_t m, hipStream_t s,
                         const uint32_t** out) {
  NttPlan p;
  if (!ntt_make_plan(n, m, &p))
    return fail(QRNG_EUNSUPPORTED, "NTT path cannot hash n=%llu m=%llu", (unsigned long long)n,
                (unsigned long long)m);
  const auto key = spectra_key(p, n, m);
  auto it = sd.spectra.find(key);
  if (it != sd.spectra.end()) {
    *out = it->second;
    return QRNG_OK;
  }
  uint32_t* W = nullptr;
  if (hipMalloc(&W, ntt_seed_elems(p) * 4) != hipSuccess)
    return fail(QRNG_ENOMEM, "seed spectra");
  qrng_status st = ensure_work(ctx, ntt_work_elems(p, 1) + 1);
  if (st) {
    (void)hipFree(W);
    return st;
  }
  hipError_t e = ntt_seed_spectra(p, reinterpret_cast<const uint32_t*>(sd.ptr), n, m, sd.L, W,
                                  ctx->work, ctx->tw, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(W);
    return fail(QRNG_EDEVICE, "seed spectra: %s", hipGetErrorString(e));
  }
  sd.spectra[key] = W;
  *out = W;
  return QRNG_OK;
}

// m_dev (nullable): valid output length computed on the device, <= m.
qrng_status hash_one(qrng_ctx* ctx, const uint64_t* x, uint64_t n, const uint64_t* seed,
                     Seed* sd, uint64_t m, uint64_t* y, int path, hipStream_t s, int batch,
                     uint64_t xs, uint64_t ys, const uint64_t* m_dev = nullptr,
                     const EstJob* est = nullptr) {
  if (fault_mode() == FAULT_LAUNCH)
    return fail(QRNG_EDEVICE, "injected launch failure (QRNG_FAULT=launch)");
  if (path == QRNG_PATH_AUTO) path = choose_path(n, m);
  if (path == QRNG_PATH_DIRECT) return run_direct(ctx, x, n, seed, m, y, s, batch, xs, ys, m_dev);
  if (path == QRNG_PATH_NTT) {
    const uint32_t* W = nullptr;
    if (sd) {
      qrng_status st = seed_spectra(ctx, *sd, n, m, s, &W);
      if (st) return st;
    }
    return run_ntt(ctx, x, n, seed, W, m, y, s, batch, xs, ys, m_dev, est);
  }
  if (path == QRNG_PATH_MFMA) {
    HIP_TRY(mfma_hash(reinterpret_cast<const uint32_t*>(x), n, reinterpret_cast<const uint32_t*>(seed),
                      m, reinterpret_cast<uint32_t*>(y), batch, xs, ys, s, m_dev));
    return QRNG_OK;
  }
  return fail(QRNG_EUNSUPPORTED, "path %d is not available for this call", path);
}

// Sec. III.D: the (n-m)-column Toeplitz product with the same seed, then the
// identity block's raw bits n-m .. n-1 added to the key.
qrng_status modified_hash(qrng_ctx* ctx, const uint64_t* x, uint64_t n, const uint64_t* seed,
                          Seed* sd, uint64_t m, uint64_t* y, int path, hipStream_t s) {
  const uint64_t w = n - m;
  if (w > 0) {
    qrng_status st = hash_one(ctx, x, w, seed, sd, m, y, path, s, 1, 0, 0);
    if (st) return st;
  }
  HIP_TRY(xor_tail_bits(x, n, w, m, y, w == 0, s));
  return QRNG_OK;
}

qrng_status check_modified_args(qrng_ctx* ctx, const uint64_t* x, uint64_t n,
                                const uint64_t* seed, uint64_t m, const uint64_t* y, int path) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  if (!x || !seed || !y) return fail(QRNG_EINVAL, "null buffer");
  if (!aligned8(x) || !aligned8(seed) || !aligned8(y))
    return fail(QRNG_EINVAL, "buffers must be 8-byte aligned");
  if (n == 0) return fail(QRNG_EINVAL, "n must be positive");
  if (m > n) return fail(QRNG_EINVAL, "m (%llu) exceeds n (%llu)", (unsigned long long)m,
                         (unsigned long long)n);
  if (path < QRNG_PATH_AUTO || path > QRNG_PATH_MFMA) return fail(QRNG_EINVAL, "unknown path");
  if (m == 0) return QRNG_OK;
  if (overlap(y, words64(m) * 8, x, words64(n) * 8))
    return fail(QRNG_EINVAL, "output overlaps the raw block");
  if (n > 1 && overlap(y, words64(m) * 8, seed, words64(n - 1) * 8))
    return fail(QRNG_EINVAL, "output overlaps the seed");
  return QRNG_OK;
}

}  // namespace

namespace qrng {
int ctx_num_cus(const qrng_ctx* c) { return c->num_cus; }
int ctx_device(const qrng_ctx* c) { return c->device; }
bool ctx_pin_seed(qrng_ctx* c, uint32_t seed_id, int delta, uint64_t* L) {
  auto it = c->seeds.find(seed_id);
  if (it == c->seeds.end()) return false;
  if (L) *L = it->second.L;
  if (delta > 0)
    ++it->second.plans;
  else if (delta < 0 && it->second.plans)
    --it->second.plans;
  return true;
}
void ctx_track_server(qrng_ctx* c, qrng_server* s, bool add) {
  if (add)
    c->servers.insert(s);
  else
    c->servers.erase(s);
}
qrng_status set_error(qrng_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

qrng_status check_me_opts(const qrng_me_opts& o) {
  if (o.model != QRNG_MODEL_FIT && o.model != QRNG_MODEL_GIVEN && o.model != QRNG_MODEL_QUANTUM)
    return fail(QRNG_EINVAL, "unknown model");
  if (o.u_mode < QRNG_U_MODEL_ARGMAX || o.u_mode > QRNG_U_ALL)
    return fail(QRNG_EINVAL, "unknown U mode");
  if (o.reserved != 0) return fail(QRNG_EINVAL, "reserved field must be 0");
  if (o.model == QRNG_MODEL_GIVEN && !(o.sigma > 0 && std::isfinite(o.sigma) && std::isfinite(o.mu)))
    return fail(QRNG_EINVAL, "given model needs finite mu and sigma > 0");
  if (o.model == QRNG_MODEL_QUANTUM && !(o.sigma >= 0 && std::isfinite(o.sigma)))
    return fail(QRNG_EINVAL, "the quantum model needs a finite classical s.d. sigma >= 0");
  return QRNG_OK;
}

void prof_begin(int kid, hipStream_t s) {
  qrng_ctx* c = t_ctx;
  if (!c || !c->prof_on) return;
  hipEvent_t e = prof_event(c);
  if (e && hipEventRecord(e, s) == hipSuccess) {
    c->prof_open = e;
  } else {
    if (e) c->prof_pool.push_back(e);
    c->prof_open = nullptr;
  }
  (void)kid;
}
void prof_end(int kid, hipStream_t s) {
  qrng_ctx* c = t_ctx;
  if (!c || !c->prof_on || !c->prof_open) return;
  hipEvent_t e = prof_event(c);
  if (e && hipEventRecord(e, s) == hipSuccess) {
    c->prof_recs.push_back(ProfRec{kid, c->prof_open, e});
  } else {
    c->prof_pool.push_back(c->prof_open);
    if (e) c->prof_pool.push_back(e);
  }
  c->prof_open = nullptr;
}
}  // namespace qrng

extern "C" {

qrng_status qrng_profile_enable(qrng_ctx* ctx, int on) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  ctx->prof_on = on != 0;
  return QRNG_OK;
}

const char* qrng_profile_kernel_name(int kernel_id) { return kernel_name(kernel_id); }

qrng_status qrng_profile_query(qrng_ctx* ctx, int kernel_id, uint64_t* launches,
                               double* total_ms) {
  if (!ctx || !launches || !total_ms) return fail(QRNG_EINVAL, "null argument");
  if (!kernel_name(kernel_id)) return fail(QRNG_EINVAL, "unknown kernel id %d", kernel_id);
  DeviceGuard g(ctx->device);
  uint64_t cnt = 0;
  double tot = 0.0;
  for (auto& r : ctx->prof_recs) {
    if (r.kid != kernel_id) continue;
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    ++cnt;
    tot += ms;
  }
  *launches = cnt;
  *total_ms = tot;
  return QRNG_OK;
}

qrng_status qrng_profile_reset(qrng_ctx* ctx) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  DeviceGuard g(ctx->device);
  for (auto& r : ctx->prof_recs) HIP_TRY(hipEventSynchronize(r.b));
  prof_release(ctx);
  return QRNG_OK;
}


qrng_status qrng_profile_issue_rates(qrng_ctx* ctx, double clock_ghz, double* cycles_out, int n,
                                     void* stream) {
  if (!ctx || !cycles_out || n < 0) return fail(QRNG_EINVAL, "null argument");
  if (!(clock_ghz > 0)) return fail(QRNG_EINVAL, "clock must be positive");
  static_assert(QRNG_PROBE_OPS == PROBE_OPS, "probe op count");
  DeviceGuard g(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* out = nullptr;
  if (hipMalloc(&out, probe_out_words(ctx->num_cus) * 4) != hipSuccess)
    return fail(QRNG_ENOMEM, "probe buffer");
  hipError_t e = hipSuccess;
  for (int op = 0; op < n && op < PROBE_OPS && e == hipSuccess; ++op)
    e = probe_issue_cycles(op, ctx->num_cus, clock_ghz, out, s, &cycles_out[op]);
  (void)hipStreamSynchronize(s);
  (void)hipFree(out);
  if (e != hipSuccess) return fail(QRNG_EDEVICE, "probe launch: %s", hipGetErrorString(e));
  return QRNG_OK;
}

const char* qrng_profile_issue_op_name(int op) { return probe_op_name(op); }

const char* qrng_version(void) { return "libqrng 0.1 (gfx950)"; }

const char* qrng_last_error(void) { return g_err.c_str(); }

qrng_status qrng_create(qrng_ctx** out, int device) {
  if (!out) return fail(QRNG_EINVAL, "null output handle");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(QRNG_EDEVICE, "no HIP device available");
  if (device < 0 || device >= ndev) return fail(QRNG_EINVAL, "device %d out of range", device);
  DeviceGuard g(device);
  qrng_ctx* c = new qrng_ctx();
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cus = prop.multiProcessorCount;
  const int T = tw_total_entries();
  std::vector<uint2> f(2 * T), iv(2 * T);
  std::vector<uint32_t> lo(4096), hi(2048);
  build_tw_tables(f.data(), iv.data(), lo.data(), hi.data());
  bool ok = hipMalloc(&c->tw_fwd, 2 * T * sizeof(uint2)) == hipSuccess &&
            hipMalloc(&c->tw_inv, 2 * T * sizeof(uint2)) == hipSuccess &&
            hipMalloc(&c->g_lo, 4096 * 4) == hipSuccess &&
            hipMalloc(&c->g_hi, 2048 * 4) == hipSuccess &&
            hipMalloc(&c->counts_dev, 258 * 8) == hipSuccess &&
            hipMalloc(&c->hist_scratch, hist_scratch_words() * 4) == hipSuccess &&
            hipMemset(c->hist_scratch, 0, hist_scratch_words() * 4) == hipSuccess &&
            hipMalloc(&c->me_dev, sizeof(qrng_me_result)) == hipSuccess &&
            hipMalloc(&c->seed_table, SEED_TABLE_CAP * sizeof(DevSeed)) == hipSuccess &&
            hipMemset(c->seed_table, 0, SEED_TABLE_CAP * sizeof(DevSeed)) == hipSuccess &&
            hipMalloc(&c->m_dev, 8) == hipSuccess &&
            hipHostMalloc(&c->counts_host, 258 * 8, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipMemcpy(c->tw_fwd, f.data(), 2 * T * sizeof(uint2), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(c->tw_inv, iv.data(), 2 * T * sizeof(uint2), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(c->g_lo, lo.data(), 4096 * 4, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(c->g_hi, hi.data(), 2048 * 4, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    qrng_destroy(c);
    return fail(QRNG_EDEVICE, "context setup on device %d failed", device);
  }
  c->tw = TwTables{c->tw_fwd, c->tw_inv, c->tw_fwd + T, c->tw_inv + T, c->g_lo, c->g_hi};
  // the allocation-free entry point's scratch: this device's address of the
  // file-scope array (each device holds its own copy)
  void* sp = nullptr;
  const hipError_t se = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
  if (se != hipSuccess || !sp) {
    qrng_destroy(c);
    return fail(QRNG_EDEVICE, "scratch symbol on device %d: %s", device, hipGetErrorString(se));
  }
  c->noalloc = static_cast<uint32_t*>(sp);
  *out = c;
  return QRNG_OK;
}

void qrng_destroy(qrng_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  while (!c->servers.empty()) qrng_server_destroy(*c->servers.begin());
  while (!c->plans.empty()) qrng_plan_destroy(*c->plans.begin());
  for (auto& kv : c->seeds)
    for (auto& sp : kv.second.spectra) (void)hipFree(sp.second);
  prof_release(c);
  for (hipEvent_t e : c->prof_pool) (void)hipEventDestroy(e);
  if (c->tw_fwd) (void)hipFree(c->tw_fwd);
  if (c->tw_inv) (void)hipFree(c->tw_inv);
  if (c->g_lo) (void)hipFree(c->g_lo);
  if (c->g_hi) (void)hipFree(c->g_hi);
  if (c->work) (void)hipFree(c->work);
  if (c->counts_dev) (void)hipFree(c->counts_dev);
  if (c->hist_scratch) (void)hipFree(c->hist_scratch);
  if (c->me_dev) (void)hipFree(c->me_dev);
  if (c->seed_table) (void)hipFree(c->seed_table);
  if (c->batch_items) (void)hipFree(c->batch_items);
  if (c->batch_counts) (void)hipFree(c->batch_counts);
  if (c->batch_work) (void)hipFree(c->batch_work);
  if (c->m_dev) (void)hipFree(c->m_dev);
  if (c->counts_host) (void)hipHostFree(c->counts_host);
  delete c;
}

qrng_status qrng_output_bits(uint64_t n, int sample_bits, double h_mod, double log2_inv_eps,
                             uint64_t* m_out) {
  if (!m_out) return fail(QRNG_EINVAL, "null output");
  if (sample_bits < 1 || sample_bits > 16) return fail(QRNG_EINVAL, "sample_bits out of range");
  if (std::isnan(h_mod) || std::isnan(log2_inv_eps) || log2_inv_eps < 0)
    return fail(QRNG_EINVAL, "bad entropy or security parameter");
  *m_out = host::output_bits_rule(n, sample_bits, h_mod, log2_inv_eps);
  return QRNG_OK;
}

qrng_status qrng_minentropy(qrng_ctx* ctx, const uint8_t* samples, uint64_t S,
                            const qrng_me_opts* opts, qrng_me_result* out,
                            uint64_t* counts_host, void* stream) {
  return qrng_minentropy_subset(ctx, samples, S, opts, 0, 0, out, counts_host, stream);
}

qrng_status qrng_minentropy_subset(qrng_ctx* ctx, const uint8_t* samples, uint64_t S,
                                   const qrng_me_opts* opts, uint64_t subset_seed,
                                   uint32_t keep_thr, qrng_me_result* out,
                                   uint64_t* counts_host, void* stream) {
  if (!ctx || !samples || !opts || !out) return fail(QRNG_EINVAL, "null argument");
  const int N = opts->sample_bits;
  if (N < 1 || N > 8) return fail(QRNG_EINVAL, "sample_bits must be 1..8 for byte samples");
  if (S == 0) return fail(QRNG_EINVAL, "no samples");
  if (S >= (1ull << 40)) return fail(QRNG_EINVAL, "at most 2^40 - 1 samples per call");
  if (qrng_status st_o = check_me_opts(*opts)) return st_o;
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int K = 1 << N;
  const int fm = fault_mode();
  if (fm == FAULT_LAUNCH) return fail(QRNG_EDEVICE, "injected launch failure (QRNG_FAULT=launch)");
  ctx->est_epoch = (ctx->est_epoch + 1) & ((1u << 23) - 1);
  HIP_TRY(hist_estimate(samples, S, N, ctx->hist_scratch, ctx->counts_dev, nullptr, s,
                        subset_seed, keep_thr, ctx->est_epoch, fm == FAULT_ROWS ? 1u : 0u));
  HIP_TRY(hipMemcpyAsync(ctx->counts_host, ctx->counts_dev, (K + 2) * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ctx->counts_host[K + 1] != 1 ||
      (!keep_thr && !host::counts_consistent(ctx->counts_host, K, ctx->counts_host[K], S)))
    return fail(QRNG_EDEVICE, "the partial histograms failed their consistency check");
  if (ctx->counts_host[K])
    return fail(QRNG_EINVAL, "%llu samples are >= 2^%d", ctx->counts_host[K], N);
  uint64_t kept = 0;
  for (int v = 0; v < K; ++v) kept += ctx->counts_host[v];
  if (kept == 0) return fail(QRNG_EINVAL, "the subset keeps no sample");
  if (counts_host)
    for (int v = 0; v < K; ++v) counts_host[v] = ctx->counts_host[v];
  host::minentropy_finish(ctx->counts_host, N, *opts, out);
  return QRNG_OK;
}

qrng_status qrng_toeplitz_hash(qrng_ctx* ctx, const uint64_t* x, uint64_t n,
                               const uint64_t* seed, uint64_t m, uint64_t* y, int path,
                               void* stream) {
  qrng_status st = check_hash_args(ctx, x, n, seed, m, y, path);
  if (st || m == 0) return st;
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  return hash_one(ctx, x, n, seed, nullptr, m, y, path, reinterpret_cast<hipStream_t>(stream),
                  1, 0, 0);
}

qrng_status qrng_toeplitz_hash_noalloc(qrng_ctx* ctx, const uint64_t* x, uint64_t n,
                                       const uint64_t* seed, uint64_t m, uint64_t* y, int path,
                                       void* stream) {
  qrng_status st = check_hash_args(ctx, x, n, seed, m, y, path);
  if (st || m == 0) return st;
  const int p = path == QRNG_PATH_AUTO ? choose_path(n, m) : path;
  DeviceGuard g(ctx->device);
  CtxScope off(nullptr);  // no timing events: this call creates nothing
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint32_t* const sc = ctx->noalloc;
  if (p == QRNG_PATH_DIRECT) {
    if (n + m - 1 >= (1ull << 34))
      return fail(QRNG_EINVAL, "direct path: n + m - 1 must be below 2^34");
    const uint64_t need = direct_work_words(n, 1);
    if (need > kNoAllocWords)
      return fail(QRNG_EINVAL, "no-alloc direct hash needs %llu scratch bytes, at most %llu",
                  (unsigned long long)(need * 4), (unsigned long long)QRNG_NOALLOC_SCRATCH_BYTES);
    // the reversal kernel rewrites every word the product reads (padding too)
    HIP_TRY(direct_hash(reinterpret_cast<const uint32_t*>(x), n,
                        reinterpret_cast<const uint32_t*>(seed), m, reinterpret_cast<uint32_t*>(y),
                        sc, ctx->num_cus, s, 1, 0, 0, nullptr));
    return QRNG_OK;
  }
  if (p == QRNG_PATH_NTT) {
    NttPlan pl;
    if (!ntt_make_plan(n, m, &pl))
      return fail(QRNG_EUNSUPPORTED, "NTT path cannot hash n=%llu m=%llu", (unsigned long long)n,
                  (unsigned long long)m);
    const uint64_t work = ntt_work_elems(pl, 1), need = work + ntt_seed_elems(pl);
    if (need > kNoAllocWords)
      return fail(QRNG_EINVAL, "no-alloc NTT hash needs %llu scratch bytes, at most %llu",
                  (unsigned long long)(need * 4), (unsigned long long)QRNG_NOALLOC_SCRATCH_BYTES);
    // the seed windows go after the transform workspace; both are written in
    // full before they are read, so nothing needs clearing
    uint32_t* W = sc + work;
    HIP_TRY(ntt_seed_spectra(pl, reinterpret_cast<const uint32_t*>(seed), n, m, n + m - 1, W, sc,
                             ctx->tw, s));
    HIP_TRY(ntt_hash(pl, reinterpret_cast<const uint32_t*>(x), n, m, W,
                     reinterpret_cast<uint32_t*>(y), sc, 1, 0, 0, ctx->tw, s));
    return QRNG_OK;
  }
  // the matrix-core product uses no scratch
  HIP_TRY(mfma_hash(reinterpret_cast<const uint32_t*>(x), n,
                    reinterpret_cast<const uint32_t*>(seed), m, reinterpret_cast<uint32_t*>(y), 1,
                    0, 0, s));
  return QRNG_OK;
}

qrng_status qrng_seed_register(qrng_ctx* ctx, const uint64_t* seed, uint64_t L,
                               uint32_t* seed_id, void* stream) {
  if (!ctx || !seed || !seed_id) return fail(QRNG_EINVAL, "null argument");
  if (!aligned8(seed)) return fail(QRNG_EINVAL, "seed must be 8-byte aligned");
  if (L == 0) return fail(QRNG_EINVAL, "empty seed");
  uint32_t id = 1;
  for (auto& kv : ctx->seeds) {
    if (kv.first != id) break;
    ++id;
  }
  if (id >= (uint32_t)SEED_TABLE_CAP)
    return fail(QRNG_EBUSY, "%d seeds are registered already", SEED_TABLE_CAP - 1);
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Seed sd{seed, L, 0, {}};
  // one-transform spectra of every length 2^k the seed can serve, computed
  // now on `stream` (after the caller's earlier work there, which may have
  // written the seed): device-descriptor batches look them up on the device
  DevSeed ds{};
  ds.L = L;
  const int top = std::min(BATCH_MAX_LOG, std::max(BATCH_MIN_LOG, ceil_log2_u64(L)));
  qrng_status st = QRNG_OK;
  for (int k = BATCH_MIN_LOG; k <= top && st == QRNG_OK; ++k) {
    NttPlan p;
    if (!ntt_plan_for_length(k, &p)) {
      st = fail(QRNG_EUNSUPPORTED, "no transform of length 2^%d", k);
      break;
    }
    uint32_t* W = nullptr;
    if (hipMalloc(&W, ntt_seed_elems(p) * 4) != hipSuccess) {
      st = fail(QRNG_ENOMEM, "seed spectrum of 2^%d points", k);
      break;
    }
    sd.spectra[{0, 1ull << k}] = W;
    st = ensure_work(ctx, ntt_work_elems(p, 1) + 1);
    if (st) break;
    const hipError_t e = ntt_seed_spectra(p, reinterpret_cast<const uint32_t*>(seed), 1, 1, L, W,
                                          ctx->work, ctx->tw, s);
    if (e != hipSuccess) st = fail(QRNG_EDEVICE, "seed spectrum: %s", hipGetErrorString(e));
    ds.W[k] = W;
  }
  if (st == QRNG_OK) {
    hipError_t e = hipMemcpyAsync(ctx->seed_table + id, &ds, sizeof ds, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(QRNG_EDEVICE, "seed registration: %s", hipGetErrorString(e));
  }
  if (st) {
    (void)hipStreamSynchronize(s);
    for (auto& sp : sd.spectra) (void)hipFree(sp.second);
    return st;
  }
  ctx->seeds[id] = sd;
  *seed_id = id;
  return QRNG_OK;
}

qrng_status qrng_seed_unregister(qrng_ctx* ctx, uint32_t seed_id) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  auto it = ctx->seeds.find(seed_id);
  if (it == ctx->seeds.end()) return fail(QRNG_EINVAL, "unknown seed id %u", seed_id);
  if (it->second.plans)
    return fail(QRNG_EBUSY, "seed %u is used by %u live plan(s)", seed_id, it->second.plans);
  DeviceGuard g(ctx->device);
  HIP_TRY(hipDeviceSynchronize());
  const DevSeed zero{};
  HIP_TRY(hipMemcpy(ctx->seed_table + seed_id, &zero, sizeof zero, hipMemcpyHostToDevice));
  for (auto& sp : it->second.spectra) (void)hipFree(sp.second);
  ctx->seeds.erase(it);
  return QRNG_OK;
}

qrng_status qrng_toeplitz_hash_fft64(qrng_ctx* ctx, const uint64_t* x, uint64_t n,
                                     const uint64_t* seed, uint64_t m, uint64_t* y,
                                     double* max_err_dev, void* stream) {
  qrng_status st = check_hash_args(ctx, x, n, seed, m, y, QRNG_PATH_AUTO);
  if (st || m == 0) return st;
  if (max_err_dev && !aligned8(max_err_dev))
    return fail(QRNG_EINVAL, "buffers must be 8-byte aligned");
  if (fft64_length(n, m) > FFT64_MAX_LENGTH)
    return fail(QRNG_EINVAL, "float64 method: n + m - 1 must be at most 2^26");
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  st = ensure_work(ctx, fft64_work_words(n, m));
  if (st) return st;
  HIP_TRY(fft64_hash(reinterpret_cast<const uint32_t*>(x), n,
                     reinterpret_cast<const uint32_t*>(seed), m, y,
                     reinterpret_cast<unsigned long long*>(max_err_dev), ctx->work,
                     reinterpret_cast<hipStream_t>(stream)));
  return QRNG_OK;
}

qrng_status qrng_modified_toeplitz_hash(qrng_ctx* ctx, const uint64_t* x, uint64_t n,
                                        const uint64_t* seed, uint64_t m, uint64_t* y, int path,
                                        void* stream) {
  qrng_status st = check_modified_args(ctx, x, n, seed, m, y, path);
  if (st || m == 0) return st;
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  return modified_hash(ctx, x, n, seed, nullptr, m, y, path,
                       reinterpret_cast<hipStream_t>(stream));
}

qrng_status qrng_modified_toeplitz_hash_seeded(qrng_ctx* ctx, const uint64_t* x, uint64_t n,
                                               uint32_t seed_id, uint64_t m, uint64_t* y,
                                               int path, void* stream) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  auto it = ctx->seeds.find(seed_id);
  if (it == ctx->seeds.end()) return fail(QRNG_EINVAL, "unknown seed id %u", seed_id);
  Seed& sd = it->second;
  qrng_status st = check_modified_args(ctx, x, n, sd.ptr, m, y, path);
  if (st || m == 0) return st;
  if (n - 1 > sd.L)
    return fail(QRNG_EINVAL, "seed has %llu bits, the modified hash needs %llu",
                (unsigned long long)sd.L, (unsigned long long)(n - 1));
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  return modified_hash(ctx, x, n, sd.ptr, &sd, m, y, path,
                       reinterpret_cast<hipStream_t>(stream));
}

qrng_status qrng_toeplitz_hash_seeded(qrng_ctx* ctx, const uint64_t* x, uint64_t n,
                                      uint32_t seed_id, uint64_t m, uint64_t* y, int path,
                                      void* stream) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  auto it = ctx->seeds.find(seed_id);
  if (it == ctx->seeds.end()) return fail(QRNG_EINVAL, "unknown seed id %u", seed_id);
  Seed& sd = it->second;
  qrng_status st = check_hash_args(ctx, x, n, sd.ptr, m, y, path);
  if (st || m == 0) return st;
  if (n + m - 1 > sd.L)
    return fail(QRNG_EINVAL, "seed has %llu bits, block needs %llu", (unsigned long long)sd.L,
                (unsigned long long)(n + m - 1));
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  return hash_one(ctx, x, n, sd.ptr, &sd, m, y, path, reinterpret_cast<hipStream_t>(stream), 1,
                  0, 0);
}

qrng_status qrng_extract(qrng_ctx* ctx, const uint8_t* samples, uint64_t S,
                         const qrng_me_opts* opts, double log2_inv_eps, uint32_t seed_id,
                         uint64_t m_cap, uint64_t* y, uint64_t* m_dev, qrng_me_result* out_dev,
                         int path, void* stream) {
  if (!ctx || !samples || !opts || !y) return fail(QRNG_EINVAL, "null argument");
  if (opts->sample_bits != 8) return fail(QRNG_EINVAL, "qrng_extract hashes 8-bit samples");
  if (qrng_status st_o = check_me_opts(*opts)) return st_o;
  if (std::isnan(log2_inv_eps) || log2_inv_eps < 0)
    return fail(QRNG_EINVAL, "bad security parameter");
  if (S == 0 || (S & 7)) return fail(QRNG_EINVAL, "S must be a positive multiple of 8");
  if (!aligned8(samples) || !aligned8(y) || (m_dev && !aligned8(m_dev)) ||
      (out_dev && !aligned8(out_dev)))
    return fail(QRNG_EINVAL, "buffers must be 8-byte aligned");
  auto it = ctx->seeds.find(seed_id);
  if (it == ctx->seeds.end()) return fail(QRNG_EINVAL, "unknown seed id %u", seed_id);
  Seed& sd = it->second;
  const uint64_t n = 8 * S;
  if (m_cap == 0 || m_cap > n) return fail(QRNG_EINVAL, "m_cap must be in [1, n]");
  if (n + m_cap - 1 > sd.L)
    return fail(QRNG_EINVAL, "seed has %llu bits, the plan needs %llu", (unsigned long long)sd.L,
                (unsigned long long)(n + m_cap - 1));
  if (path < QRNG_PATH_AUTO || path > QRNG_PATH_MFMA) return fail(QRNG_EINVAL, "unknown path");
  if (overlap(y, words64(m_cap) * 8, samples, S))
    return fail(QRNG_EINVAL, "output overlaps the samples");
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint64_t* md = m_dev ? m_dev : ctx->m_dev;
  MeDevArgs a{};
  a.N = 8;
  a.model = opts->model;
  a.u_mode = opts->u_mode;
  a.mu = opts->mu;
  a.sigma = opts->sigma;
  a.n = n;
  a.log2_inv_eps = log2_inv_eps;
  a.m_cap = m_cap;
  a.out = out_dev ? (void*)out_dev : (void*)ctx->me_dev;
  a.m_out = md;
  // on the split transform the estimate runs inside the hash's first pass
  const int hp = path == QRNG_PATH_AUTO ? choose_path(n, m_cap) : path;
  NttPlan pl;
  if (hp == QRNG_PATH_NTT && ntt_make_plan(n, m_cap, &pl) && ntt_fuses_estimate(pl)) {
    ctx->est_epoch = (ctx->est_epoch + 1) & ((1u << 23) - 1);
    const int fm = fault_mode();
    if (fm == FAULT_TICKET) {
      // a launch of another call that never completed: its tag, 7 counted
      const uint32_t stale = ((ctx->est_epoch ^ 0x55u) << 9) | 7u;
      HIP_TRY(hipMemcpyAsync(ctx->hist_scratch + hist_ticket_word(), &stale, 4,
                             hipMemcpyHostToDevice, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    const EstJob job{samples, S, ctx->hist_scratch, a, ctx->est_epoch,
                     fm == FAULT_ROWS ? 1u : 0u};
    return hash_one(ctx, reinterpret_cast<const uint64_t*>(samples), n, sd.ptr, &sd, m_cap, y,
                    hp, s, 1, 0, 0, md, &job);
  }
  if (fault_mode() == FAULT_LAUNCH)
    return fail(QRNG_EDEVICE, "injected launch failure (QRNG_FAULT=launch)");
  ctx->est_epoch = (ctx->est_epoch + 1) & ((1u << 23) - 1);
  HIP_TRY(hist_estimate(samples, S, 8, ctx->hist_scratch, nullptr, &a, s, 0, 0, ctx->est_epoch,
                        fault_mode() == FAULT_ROWS ? 1u : 0u));
  return hash_one(ctx, reinterpret_cast<const uint64_t*>(samples), n, sd.ptr, &sd, m_cap, y, path,
                  s, 1, 0, 0, md);
}

qrng_status qrng_toeplitz_hash_strided(qrng_ctx* ctx, const uint64_t* x_pool, uint64_t n,
                                       uint64_t x_stride_words, uint32_t seed_id, uint64_t m,
                                       uint64_t* y_pool, uint64_t y_stride_words,
                                       uint32_t nblocks, int path, void* stream) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  auto it = ctx->seeds.find(seed_id);
  if (it == ctx->seeds.end()) return fail(QRNG_EINVAL, "unknown seed id %u", seed_id);
  Seed& sd = it->second;
  qrng_status st = check_hash_args(ctx, x_pool, n, sd.ptr, m, y_pool, path);
  if (st || m == 0 || nblocks == 0) return st;
  if (x_stride_words < words64(n) || y_stride_words < words64(m))
    return fail(QRNG_EINVAL, "strides shorter than a block");
  if (n + m - 1 > sd.L) return fail(QRNG_EINVAL, "seed too short for the block shape");
  if (overlap(y_pool, (nblocks - 1) * y_stride_words * 8 + words64(m) * 8, x_pool,
              (nblocks - 1) * x_stride_words * 8 + words64(n) * 8))
    return fail(QRNG_EINVAL, "output pool overlaps the raw pool");
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int p = path == QRNG_PATH_AUTO ? choose_path(n, m, nblocks) : path;
  uint64_t cap = nblocks;
  if (p == QRNG_PATH_NTT) {
    NttPlan pl;
    if (ntt_make_plan(n, m, &pl)) {
      const uint64_t per = ntt_work_elems(pl, 1) * 4;
      if (per) cap = std::max<uint64_t>(1, (1ull << 30) / per);  // 1 GiB of workspace
    }
  }
  for (uint64_t b = 0; b < nblocks; b += cap) {
    const uint64_t cnt = std::min<uint64_t>(cap, nblocks - b);
    st = hash_one(ctx, x_pool + b * x_stride_words, n, sd.ptr, &sd, m, y_pool + b * y_stride_words,
                  p, s, (int)cnt, x_stride_words * 64, y_stride_words * 64);
    if (st) return st;
  }
  return QRNG_OK;
}

qrng_status qrng_toeplitz_hash_batched(qrng_ctx* ctx, const qrng_block* blocks_dev,
                                       uint32_t nblocks, const uint64_t* x_pool,
                                       const uint32_t* seed_ids_or_null, uint64_t* y_pool,
                                       int path, void* stream) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  if (nblocks == 0) return QRNG_OK;
  if (!blocks_dev || !x_pool || !y_pool) return fail(QRNG_EINVAL, "null argument");
  if (!aligned8(blocks_dev) || !aligned8(x_pool) || !aligned8(y_pool) ||
      (reinterpret_cast<uintptr_t>(seed_ids_or_null) & 3u))
    return fail(QRNG_EINVAL, "buffers must be aligned");
  if (path < QRNG_PATH_AUTO || path > QRNG_PATH_MFMA) return fail(QRNG_EINVAL, "unknown path");
  if (path != QRNG_PATH_AUTO && path != QRNG_PATH_NTT)
    return fail(QRNG_EUNSUPPORTED,
                "device descriptors run on the transform path (direct and matrix-core batches "
                "take host descriptors)");
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // classes a block can fall in: up to the longest registered seed's
  int top = BATCH_MIN_LOG;
  for (auto& kv : ctx->seeds)
    top = std::max(top, std::min(BATCH_MAX_LOG, ceil_log2_u64(kv.second.L)));
  // item lists (grown to the batch size; a larger batch allocates once)
  if (ctx->batch_cap < nblocks) {
    HIP_TRY(hipDeviceSynchronize());
    if (ctx->batch_items) (void)hipFree(ctx->batch_items);
    if (ctx->batch_counts) (void)hipFree(ctx->batch_counts);
    ctx->batch_items = nullptr;
    ctx->batch_counts = nullptr;
    ctx->batch_cap = 0;
    if (hipMalloc(&ctx->batch_items, (uint64_t)BATCH_CLASSES * nblocks * sizeof(NttItem)) !=
            hipSuccess ||
        hipMalloc(&ctx->batch_counts, BATCH_COUNTS * 4) != hipSuccess)
      return fail(QRNG_ENOMEM, "item lists for %u blocks", nblocks);
    ctx->batch_cap = nblocks;
  }
  // transform workspace: every class of four-step length runs in rounds of
  // as many items as it holds (at most 4 GiB, at least one item of the
  // longest class); rounds past a class's count do nothing
  const uint64_t want = std::min<uint64_t>(4ull << 30, (uint64_t)nblocks * (4ull << top));
  const uint64_t need = std::max<uint64_t>(want, 4ull << top);
  if (ctx->batch_work_bytes < need) {
    HIP_TRY(hipDeviceSynchronize());
    if (ctx->batch_work) (void)hipFree(ctx->batch_work);
    ctx->batch_work = nullptr;
    ctx->batch_work_bytes = 0;
    if (hipMalloc(&ctx->batch_work, need) != hipSuccess)
      return fail(QRNG_ENOMEM, "batch workspace of %llu bytes", (unsigned long long)need);
    ctx->batch_work_bytes = need;
  }
  const uint32_t cap = ctx->batch_cap;
  HIP_TRY(batch_classify(blocks_dev, nblocks, seed_ids_or_null, ctx->seed_table,
                         ctx->batch_items, cap, top, ctx->batch_counts, s));
  const uint32_t* xp = reinterpret_cast<const uint32_t*>(x_pool);
  uint32_t* yp = reinterpret_cast<uint32_t*>(y_pool);
  for (int k = BATCH_MIN_LOG; k <= top; ++k) {
    NttPlan p;
    if (!ntt_plan_for_length(k, &p)) return fail(QRNG_EUNSUPPORTED, "transform 2^%d", k);
    const NttItem* list = ctx->batch_items + (uint64_t)(k - BATCH_MIN_LOG) * cap;
    const uint32_t* cnt = ctx->batch_counts + (k - BATCH_MIN_LOG);
    const uint64_t per = ntt_work_elems(p, 1) * 4;
    const uint32_t round =
        per ? (uint32_t)std::min<uint64_t>(nblocks, ctx->batch_work_bytes / per) : nblocks;
    for (uint32_t i0 = 0; i0 < nblocks; i0 += round)
      HIP_TRY(ntt_hash_items_dev(p, xp, list, cnt, i0, (int)std::min(round, nblocks - i0), yp,
                                 ctx->batch_work, ctx->tw, s));
  }
  return QRNG_OK;
}

qrng_status qrng_toeplitz_hash_batched_rejected(qrng_ctx* ctx, uint32_t* count, void* stream) {
  if (!ctx || !count) return fail(QRNG_EINVAL, "null argument");
  *count = 0;
  if (!ctx->batch_counts) return QRNG_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(count, ctx->batch_counts + BATCH_REJECTED, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return QRNG_OK;
}

qrng_status qrng_toeplitz_hash_batched_host(qrng_ctx* ctx, const qrng_block* blocks,
                                            uint32_t nblocks, const uint64_t* x_pool,
                                            uint64_t* y_pool, int path, void* stream) {
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  if (nblocks == 0) return QRNG_OK;
  if (!blocks || !x_pool || !y_pool) return fail(QRNG_EINVAL, "null argument");
  if (!aligned8(x_pool) || !aligned8(y_pool)) return fail(QRNG_EINVAL, "pools must be aligned");
  if (path < QRNG_PATH_AUTO || path > QRNG_PATH_MFMA) return fail(QRNG_EINVAL, "unknown path");
  // validate every descriptor before enqueueing anything
  std::vector<std::pair<uint64_t, uint64_t>> yr;
  yr.reserve(nblocks);
  for (uint32_t i = 0; i < nblocks; ++i) {
    const qrng_block& b = blocks[i];
    if (b.flags) return fail(QRNG_EINVAL, "block %u: flags must be 0", i);
    if (b.n == 0 || b.m > b.n) return fail(QRNG_EINVAL, "block %u: need 0 < n and m <= n", i);
    auto it = ctx->seeds.find(b.seed_id);
    if (it == ctx->seeds.end()) return fail(QRNG_EINVAL, "block %u: unknown seed %u", i, b.seed_id);
    if (b.m && b.n + b.m - 1 > it->second.L)
      return fail(QRNG_EINVAL, "block %u: seed too short", i);
    if (b.m) yr.emplace_back(b.y_word_off, b.y_word_off + words64(b.m));
  }
  std::sort(yr.begin(), yr.end());
  for (size_t i = 1; i < yr.size(); ++i)
    if (yr[i].first < yr[i - 1].second) return fail(QRNG_EINVAL, "output ranges overlap");
  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // group equal shapes whose offsets advance by constant strides: one launch each
  std::map<std::tuple<uint64_t, uint64_t, uint32_t>, std::vector<uint32_t>> groups;
  for (uint32_t i = 0; i < nblocks; ++i)
    if (blocks[i].m) groups[{blocks[i].n, blocks[i].m, blocks[i].seed_id}].push_back(i);
  for (auto& kv : groups) {
    const uint64_t n = std::get<0>(kv.first), m = std::get<1>(kv.first);
    Seed& sd = ctx->seeds[std::get<2>(kv.first)];
    const std::vector<uint32_t>& ids = kv.second;
    int p = path == QRNG_PATH_AUTO ? choose_path(n, m, ids.size()) : path;
    size_t i = 0;
    while (i < ids.size()) {
      // longest run with constant x and y strides
      size_t j = i + 1;
      int64_t dx = 0, dy = 0;
      if (j < ids.size()) {
        dx = (int64_t)blocks[ids[j]].x_word_off - (int64_t)blocks[ids[i]].x_word_off;
        dy = (int64_t)blocks[ids[j]].y_word_off - (int64_t)blocks[ids[i]].y_word_off;
        if (dx < 0 || dy < 0) dx = dy = -1;
        while (dx >= 0 && j < ids.size() &&
               (int64_t)blocks[ids[j]].x_word_off - (int64_t)blocks[ids[j - 1]].x_word_off == dx &&
               (int64_t)blocks[ids[j]].y_word_off - (int64_t)blocks[ids[j - 1]].y_word_off == dy)
          ++j;
        if (dx < 0) j = i + 1;
      }
      // cap the batch so the transform workspace stays bounded (1 GiB)
      size_t cnt = j - i;
      if (p == QRNG_PATH_NTT) {
        NttPlan pl;
        if (ntt_make_plan(n, m, &pl)) {
          const uint64_t per = ntt_work_elems(pl, 1) * 4;
          const size_t cap = per ? std::max<uint64_t>(1, (1ull << 30) / per) : cnt;
          cnt = std::min(cnt, cap);
        }
      }
      cnt = std::min<size_t>(cnt, 1u << 20);
      const qrng_block& b0 = blocks[ids[i]];
      qrng_status st = hash_one(ctx, x_pool + b0.x_word_off, n, sd.ptr, &sd, m,
                                y_pool + b0.y_word_off, p, s, (int)cnt,
                                cnt > 1 ? (uint64_t)dx * 64 : 0, cnt > 1 ? (uint64_t)dy * 64 : 0);
      if (st) return st;
      i += cnt;
    }
  }
  return QRNG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ plans
// A plan fixes an uneven batch of blocks (Sec. III.E with per-block block
// lengths and, optionally, per-block Sec. II estimates) once: descriptors
// live in device memory, seed spectra are prepared, the launches are laid
// out per transform-length class and may be replayed as one HIP graph.

struct qrng_plan {
  qrng_ctx* ctx = nullptr;
  std::vector<uint32_t> seed_ids;  // seeds pinned while the plan lives
  std::vector<std::function<hipError_t(hipStream_t)>> steps;
  void* desc = nullptr;      // device: NttItem[] then MeBlock[]
  uint32_t* work = nullptr;  // device workspace owned by the plan
  uint64_t work_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t nblocks = 0, classes = 0;
  // persistent multi-class passes: argument block, unit counters, workspace
  void* mc_args = nullptr;
  uint32_t* mc_counters = nullptr;
  uint32_t* mc_work = nullptr;
  bool multi = false;
};

namespace {

constexpr int kTuneDirect = -1;
constexpr int kTuneDefaultCap = 27;  // 128 MiB of transform residues per launch
constexpr int kTuneNoCap = 40;

struct ClassInfo {
  int log_nc;
  std::vector<uint32_t> ids;  // block indices
  uint64_t item_off;          // first NttItem of the class in the device array
  uint64_t max_n;
};

// Sub-batches of a class under a workspace cap of 2^cap_log2 bytes.
int class_chunk(const NttPlan& p, size_t count, int cap_log2) {
  const uint64_t per = ntt_work_elems(p, 1) * 4;
  if (per == 0 || cap_log2 >= kTuneNoCap) return (int)std::min<size_t>(count, 1u << 16);
  const uint64_t c = std::max<uint64_t>(1, (1ull << cap_log2) / per);
  return (int)std::min<uint64_t>({c, (uint64_t)count, 1u << 16});
}

struct PlanBuild {
  qrng_ctx* ctx;
  const qrng_block* blocks;
  const uint64_t* x_pool;
  uint64_t* y_pool;
  const uint64_t* m_arr;  // device valid lengths (estimate mode) or null
  const NttItem* items_dev;
  std::vector<ClassInfo> classes;
  std::vector<uint32_t> singles;  // blocks hashed one launch each
  std::vector<int> single_path;
};

// Launch steps of one class under a given shape choice; *work_need gets the
// workspace (bytes) they use.
void class_steps(const PlanBuild& b, const ClassInfo& c, int choice, uint32_t** work_slot,
                 std::vector<std::function<hipError_t(hipStream_t)>>* out,
                 uint64_t* work_need) {
  qrng_ctx* ctx = b.ctx;
  NttPlan p;
  ntt_plan_for_length(c.log_nc, &p);
  *work_need = 0;
  if (choice == kTuneDirect) {
    for (uint32_t id : c.ids) {
      const qrng_block blk = b.blocks[id];
      const uint64_t* seed = ctx->seeds[blk.seed_id].ptr;
      const uint64_t* md = b.m_arr ? b.m_arr + id : nullptr;
      const uint64_t* x = b.x_pool + blk.x_word_off;
      uint64_t* y = b.y_pool + blk.y_word_off;
      *work_need = std::max<uint64_t>(*work_need, direct_work_words(blk.n, 1) * 4);
      const int ncu = ctx->num_cus;
      out->push_back([=](hipStream_t s) {
        return direct_hash(reinterpret_cast<const uint32_t*>(x), blk.n,
                           reinterpret_cast<const uint32_t*>(seed), blk.m,
                           reinterpret_cast<uint32_t*>(y), *work_slot, ncu, s, 1, 0, 0, md);
      });
    }
    return;
  }
  const int chunk = class_chunk(p, c.ids.size(), choice);
  const TwTables tw = ctx->tw;
  for (size_t i = 0; i < c.ids.size(); i += chunk) {
    const int cnt = (int)std::min<size_t>(chunk, c.ids.size() - i);
    *work_need = std::max<uint64_t>(*work_need, ntt_work_elems(p, cnt) * 4);
    const NttItem* items = b.items_dev + c.item_off + i;
    const uint32_t* xp = reinterpret_cast<const uint32_t*>(b.x_pool);
    uint32_t* yp = reinterpret_cast<uint32_t*>(b.y_pool);
    const uint64_t* ma = b.m_arr;
    out->push_back([=](hipStream_t s) {
      return ntt_hash_items(p, xp, items, cnt, yp, ma, *work_slot, tw, s);
    });
  }
}

int tune_key_count(size_t count) {
  int k = 0;
  while ((size_t(1) << k) < count) ++k;
  return k;
}

// Run `steps` eagerly: warm-up once, then the median of three timed runs (ms).
qrng_status time_steps(const std::vector<std::function<hipError_t(hipStream_t)>>& steps,
                       hipStream_t s, float* ms) {
  hipEvent_t a = nullptr, e = nullptr;
  HIP_TRY(hipEventCreate(&a));
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(QRNG_EDEVICE, "event");
  }
  float t[3] = {0, 0, 0};
  hipError_t err = hipSuccess;
  for (int r = -1; r < 3 && err == hipSuccess; ++r) {
    err = hipEventRecord(a, s);
    for (auto& f : steps)
      if (err == hipSuccess) err = f(s);
    if (err == hipSuccess) err = hipEventRecord(e, s);
    if (err == hipSuccess) err = hipEventSynchronize(e);
    if (err == hipSuccess && r >= 0) err = hipEventElapsedTime(&t[r], a, e);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(e);
  if (err != hipSuccess) return fail(QRNG_EDEVICE, "tuning run: %s", hipGetErrorString(err));
  std::sort(t, t + 3);
  *ms = t[1];
  return QRNG_OK;
}

qrng_status plan_alloc_work(qrng_plan* pl, uint64_t bytes) {
  if (bytes <= pl->work_bytes) return QRNG_OK;
  if (pl->work) {
    HIP_TRY(hipDeviceSynchronize());
    (void)hipFree(pl->work);
    pl->work = nullptr;
    pl->work_bytes = 0;
  }
  if (hipMalloc(&pl->work, bytes) != hipSuccess)
    return fail(QRNG_ENOMEM, "plan workspace of %llu bytes", (unsigned long long)bytes);
  pl->work_bytes = bytes;
  return QRNG_OK;
}

void plan_free(qrng_plan* pl) {
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->desc) (void)hipFree(pl->desc);
  if (pl->work) (void)hipFree(pl->work);
  if (pl->mc_args) (void)hipFree(pl->mc_args);
  if (pl->mc_counters) (void)hipFree(pl->mc_counters);
  if (pl->mc_work) (void)hipFree(pl->mc_work);
  for (uint32_t id : pl->seed_ids) {
    auto it = pl->ctx->seeds.find(id);
    if (it != pl->ctx->seeds.end() && it->second.plans) --it->second.plans;
  }
  pl->ctx->plans.erase(pl);
  delete pl;
}

}  // namespace

extern "C" {

qrng_status qrng_plan_create(qrng_ctx* ctx, const qrng_block* blocks, uint32_t nblocks,
                             const uint64_t* x_pool, uint64_t* y_pool, uint64_t* m_dev,
                             qrng_me_result* me_dev, const qrng_me_opts* opts,
                             double log2_inv_eps, int path, uint32_t flags, void* stream,
                             qrng_plan** out) {
  if (!out) return fail(QRNG_EINVAL, "null plan handle");
  *out = nullptr;
  if (!ctx) return fail(QRNG_EINVAL, "null context");
  if (!blocks || !x_pool || !y_pool || nblocks == 0)
    return fail(QRNG_EINVAL, "a plan needs blocks and both pools");
  if (flags & ~(uint32_t)(QRNG_PLAN_ESTIMATE | QRNG_PLAN_GRAPH | QRNG_PLAN_TUNE))
    return fail(QRNG_EINVAL, "unknown plan flags 0x%x", flags);
  if (!aligned8(x_pool) || !aligned8(y_pool) || (m_dev && !aligned8(m_dev)) ||
      (me_dev && !aligned8(me_dev)))
    return fail(QRNG_EINVAL, "buffers must be 8-byte aligned");
  if (path < QRNG_PATH_AUTO || path > QRNG_PATH_MFMA) return fail(QRNG_EINVAL, "unknown path");
  const bool estimate = (flags & QRNG_PLAN_ESTIMATE) != 0;
  if (estimate) {
    if (!opts || !m_dev) return fail(QRNG_EINVAL, "estimate plans need opts and m_dev");
    if (opts->sample_bits != 8) return fail(QRNG_EINVAL, "estimate plans take 8-bit samples");
    if (qrng_status st_o = check_me_opts(*opts)) return st_o;
    if (std::isnan(log2_inv_eps) || log2_inv_eps < 0)
      return fail(QRNG_EINVAL, "bad security parameter");
  }
  // validate every descriptor
  std::vector<std::pair<uint64_t, uint64_t>> yr;
  yr.reserve(nblocks);
  std::set<uint32_t> used;
  for (uint32_t i = 0; i < nblocks; ++i) {
    const qrng_block& b = blocks[i];
    if (b.flags) return fail(QRNG_EINVAL, "block %u: flags must be 0", i);
    if (b.n == 0 || b.m > b.n) return fail(QRNG_EINVAL, "block %u: need 0 < n and m <= n", i);
    if (b.n >= (1ull << 32)) return fail(QRNG_EINVAL, "block %u: n must be < 2^32", i);
    auto it = ctx->seeds.find(b.seed_id);
    if (it == ctx->seeds.end()) return fail(QRNG_EINVAL, "block %u: unknown seed %u", i, b.seed_id);
    if (b.m && b.n + b.m - 1 > it->second.L)
      return fail(QRNG_EINVAL, "block %u: seed too short", i);
    if (estimate && (b.n & 63)) return fail(QRNG_EINVAL, "block %u: n must be a multiple of 64", i);
    if (b.m) yr.emplace_back(b.y_word_off, b.y_word_off + words64(b.m));
    used.insert(b.seed_id);
  }
  std::sort(yr.begin(), yr.end());
  for (size_t i = 1; i < yr.size(); ++i)
    if (yr[i].first < yr[i - 1].second) return fail(QRNG_EINVAL, "output ranges overlap");

  DeviceGuard g(ctx->device);
  CtxScope cs(ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  qrng_plan* pl = new qrng_plan();
  pl->ctx = ctx;
  pl->nblocks = nblocks;
  ctx->plans.insert(pl);
  for (uint32_t id : used) {
    ctx->seeds[id].plans++;
    pl->seed_ids.push_back(id);
  }
  auto bail = [&](qrng_status st) {
    plan_free(pl);
    return st;
  };

  // classes: one transform of length Nc per block where possible
  PlanBuild b{ctx, blocks, x_pool, y_pool, estimate ? m_dev : nullptr, nullptr, {}, {}, {}};
  std::map<int, size_t> cls_of;
  for (uint32_t i = 0; i < nblocks; ++i) {
    const qrng_block& bl = blocks[i];
    if (!bl.m) continue;
    int p = path == QRNG_PATH_AUTO ? choose_path(bl.n, bl.m) : path;
    NttPlan np;
    const bool one = ntt_make_plan(bl.n, bl.m, &np) && np.nx == 1 && np.ny == 1;
    if ((path == QRNG_PATH_AUTO || path == QRNG_PATH_NTT) && one &&
        (p == QRNG_PATH_NTT || path == QRNG_PATH_AUTO)) {
      auto f = cls_of.find(np.log_nc);
      if (f == cls_of.end()) {
        f = cls_of.emplace(np.log_nc, b.classes.size()).first;
        b.classes.push_back(ClassInfo{np.log_nc, {}, 0, 0});
      }
      ClassInfo& c = b.classes[f->second];
      c.ids.push_back(i);
      c.max_n = std::max<uint64_t>(c.max_n, bl.n);
    } else {
      b.singles.push_back(i);
      b.single_path.push_back(p);
    }
  }
  pl->classes = (uint32_t)b.classes.size();

  // seed spectra (computed now, cached in the context) and item records
  std::vector<NttItem> items;
  for (ClassInfo& c : b.classes) {
    c.item_off = items.size();
    for (uint32_t id : c.ids) {
      const qrng_block& bl = blocks[id];
      const uint32_t* W = nullptr;
      qrng_status st = seed_spectra(ctx, ctx->seeds[bl.seed_id], bl.n, bl.m, s, &W);
      if (st) return bail(st);
      items.push_back(NttItem{bl.x_word_off * 64, bl.y_word_off * 64, W, (uint32_t)bl.n,
                              (uint32_t)bl.m, id, 0});
    }
  }
  for (size_t k = 0; k < b.singles.size(); ++k)
    if (b.single_path[k] == QRNG_PATH_NTT) {
      const qrng_block& bl = blocks[b.singles[k]];
      const uint32_t* W = nullptr;
      qrng_status st = seed_spectra(ctx, ctx->seeds[bl.seed_id], bl.n, bl.m, s, &W);
      if (st) return bail(st);
    }
  std::vector<MeBlock> meb;
  if (estimate)
    for (uint32_t i = 0; i < nblocks; ++i)
      meb.push_back(MeBlock{blocks[i].x_word_off * 8, (uint32_t)(blocks[i].n / 8), 0, blocks[i].n,
                            blocks[i].m});
  const uint64_t ib = items.size() * sizeof(NttItem), mb = meb.size() * sizeof(MeBlock);
  if (ib + mb) {
    if (hipMalloc(&pl->desc, ib + mb) != hipSuccess) return bail(fail(QRNG_ENOMEM, "descriptors"));
    if (ib && hipMemcpy(pl->desc, items.data(), ib, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(QRNG_EDEVICE, "descriptor upload"));
    if (mb && hipMemcpy((char*)pl->desc + ib, meb.data(), mb, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(QRNG_EDEVICE, "descriptor upload"));
  }
  b.items_dev = reinterpret_cast<const NttItem*>(pl->desc);

  // step 1: the per-block estimates
  std::vector<std::function<hipError_t(hipStream_t)>> head;
  MeBatchArgs est_args{};
  if (estimate) {
    MeBatchArgs& a = est_args;
    a.pool = reinterpret_cast<const uint8_t*>(x_pool);
    a.blocks = reinterpret_cast<const MeBlock*>((char*)pl->desc + ib);
    a.model = opts->model;
    a.u_mode = opts->u_mode;
    a.mu = opts->mu;
    a.sigma = opts->sigma;
    a.log2_inv_eps = log2_inv_eps;
    a.out = me_dev;
    a.m_out = m_dev;
    const int nb = (int)nblocks;
    head.push_back([=](hipStream_t st) { return minentropy_blocks(a, nb, st); });
  }

  // step 2: each class, in the tuned (or default) launch shape
  uint32_t** slot = &pl->work;
  // default shape: batched transforms, except classes of short blocks, where
  // the direct product wins (the single-block crossover near n = 2^15)
  std::vector<int> choice(b.classes.size(), kTuneDefaultCap);
  for (size_t k = 0; k < b.classes.size(); ++k) {
    const ClassInfo& c = b.classes[k];
    if (path == QRNG_PATH_AUTO && c.max_n < (1u << 15)) choice[k] = kTuneDirect;
    auto t = ctx->tune.find({c.log_nc, tune_key_count(c.ids.size())});
    if (t != ctx->tune.end() && (path == QRNG_PATH_AUTO || t->second != kTuneDirect))
      choice[k] = t->second;
  }
  if (flags & QRNG_PLAN_TUNE) {
    // the estimates decide the valid lengths the hashes read: run them once
    for (auto& f : head) {
      hipError_t e = f(s);
      if (e != hipSuccess) return bail(fail(QRNG_EDEVICE, "estimate: %s", hipGetErrorString(e)));
    }
    for (size_t k = 0; k < b.classes.size(); ++k) {
      const ClassInfo& c = b.classes[k];
      std::vector<int> cand = {kTuneNoCap, 30, 28, 27, 26, 24};
      if (path == QRNG_PATH_AUTO && c.max_n <= (1u << 16)) cand.push_back(kTuneDirect);
      float best = INFINITY;
      int best_c = choice[k];
      int last_chunk = -1;
      auto& meas = ctx->tune_ms[{c.log_nc, tune_key_count(c.ids.size())}];
      meas.clear();
      for (int cc : cand) {
        NttPlan np;
        ntt_plan_for_length(c.log_nc, &np);
        if (cc != kTuneDirect) {
          const int ch = class_chunk(np, c.ids.size(), cc);
          if (ch == last_chunk) continue;  // same launch shape as the previous cap
          last_chunk = ch;
        }
        std::vector<std::function<hipError_t(hipStream_t)>> st;
        uint64_t need = 0;
        class_steps(b, c, cc, slot, &st, &need);
        if (need > (8ull << 30)) continue;  // keep tuning runs within 8 GiB
        qrng_status e = plan_alloc_work(pl, need);
        if (e) return bail(e);
        float ms = 0;
        e = time_steps(st, s, &ms);
        if (e) return bail(e);
        meas.emplace_back(cc, ms);
        if (ms < best) best = ms, best_c = cc;
      }
      choice[k] = best_c;
      ctx->tune[{c.log_nc, tune_key_count(c.ids.size())}] = best_c;
    }
  }
  // items of the persistent multi-class launches by transform length: the
  // classes of 2^16 .. 2^21 points, and shorter classes raised to 2^16 points
  // when every seed they use has that spectrum (any length >= n+m-1 gives
  // the same bits)
  std::map<int, std::vector<NttItem>, std::greater<int>> mc_items;
  std::vector<bool> in_mc(b.classes.size(), false);
  if (path == QRNG_PATH_AUTO || path == QRNG_PATH_NTT) {
    for (size_t k = 0; k < b.classes.size(); ++k) {
      const ClassInfo& c = b.classes[k];
      if (c.log_nc > MC_MAX_LOG) continue;
      if (c.log_nc >= MC_MIN_LOG) {
        auto& v = mc_items[c.log_nc];
        v.insert(v.end(), items.begin() + (long)c.item_off,
                 items.begin() + (long)(c.item_off + c.ids.size()));
        in_mc[k] = true;
        continue;
      }
      std::vector<NttItem> up;
      for (uint32_t id : c.ids) {
        const auto& sp = ctx->seeds[blocks[id].seed_id].spectra;
        auto f = sp.find({0, 1ull << MC_MIN_LOG});
        if (f == sp.end()) break;
        const qrng_block& bl = blocks[id];
        up.push_back(NttItem{bl.x_word_off * 64, bl.y_word_off * 64, f->second, (uint32_t)bl.n,
                             (uint32_t)bl.m, id, 0});
      }
      if (up.size() == c.ids.size()) {
        auto& v = mc_items[MC_MIN_LOG];
        v.insert(v.end(), up.begin(), up.end());
        in_mc[k] = true;
      }
    }
  }
  if (mc_items.size() > (size_t)MC_MAX) {
    mc_items.clear();
    in_mc.assign(b.classes.size(), false);
  }

  uint64_t work_need = 0, work_other = 0;  // all per-class steps / those outside mc
  pl->steps = head;
  std::vector<std::function<hipError_t(hipStream_t)>> other;  // classes outside mc
  for (size_t k = 0; k < b.classes.size(); ++k) {
    uint64_t need = 0;
    class_steps(b, b.classes[k], choice[k], slot, &pl->steps, &need);
    work_need = std::max(work_need, need);
    if (!in_mc[k]) {
      class_steps(b, b.classes[k], choice[k], slot, &other, &need);
      work_other = std::max(work_other, need);
    }
  }
  std::vector<std::function<hipError_t(hipStream_t)>> singles_steps;
  const size_t singles_at = pl->steps.size();
  // blocks that need the split transform (or a forced path): one launch each
  for (size_t k = 0; k < b.singles.size(); ++k) {
    const uint32_t id = b.singles[k];
    const qrng_block bl = blocks[id];
    Seed& sd = ctx->seeds[bl.seed_id];
    const uint64_t* md = b.m_arr ? b.m_arr + id : nullptr;
    const uint32_t* x = reinterpret_cast<const uint32_t*>(x_pool + bl.x_word_off);
    uint32_t* y = reinterpret_cast<uint32_t*>(y_pool + bl.y_word_off);
    const uint32_t* seed = reinterpret_cast<const uint32_t*>(sd.ptr);
    const int p = b.single_path[k];
    if (p == QRNG_PATH_NTT) {
      NttPlan np;
      if (!ntt_make_plan(bl.n, bl.m, &np))
        return bail(fail(QRNG_EUNSUPPORTED, "block %u: NTT path cannot hash this shape", id));
      const uint32_t* W = nullptr;
      qrng_status st = seed_spectra(ctx, sd, bl.n, bl.m, s, &W);
      if (st) return bail(st);
      work_need = std::max<uint64_t>(work_need, ntt_work_elems(np, 1) * 4);
      const TwTables tw = ctx->tw;
      pl->steps.push_back([=](hipStream_t st) {
        return ntt_hash(np, x, bl.n, bl.m, W, y, *slot, 1, 0, 0, tw, st, md);
      });
    } else if (p == QRNG_PATH_DIRECT) {
      work_need = std::max<uint64_t>(work_need, direct_work_words(bl.n, 1) * 4);
      const int ncu = ctx->num_cus;
      pl->steps.push_back([=](hipStream_t st) {
        return direct_hash(x, bl.n, seed, bl.m, y, *slot, ncu, st, 1, 0, 0, md);
      });
    } else {
      pl->steps.push_back([=](hipStream_t st) {
        return mfma_hash(x, bl.n, seed, bl.m, y, 1, 0, 0, st, md);
      });
    }
  }
  work_other = std::max(work_other, [&] {
    // the singles' share of work_need
    uint64_t w = 0;
    for (size_t k = 0; k < b.singles.size(); ++k) {
      const qrng_block bl = blocks[b.singles[k]];
      NttPlan np;
      if (b.single_path[k] == QRNG_PATH_NTT && ntt_make_plan(bl.n, bl.m, &np))
        w = std::max<uint64_t>(w, ntt_work_elems(np, 1) * 4);
      else if (b.single_path[k] == QRNG_PATH_DIRECT)
        w = std::max<uint64_t>(w, direct_work_words(bl.n, 1) * 4);
    }
    return w;
  }());
  singles_steps.assign(pl->steps.begin() + (long)singles_at, pl->steps.end());

  // the persistent multi-class form: three launches for every class in mc
  // (with the per-block estimates inside the second), then the other classes
  // and the singles; used when the tuning table or tuning picks it
  if (!mc_items.empty()) {
    uint64_t words = 0, nit = 0;
    for (auto& kv : mc_items) {
      words += (uint64_t)kv.second.size() << kv.first;
      nit += kv.second.size();
    }
    if (hipMalloc(&pl->mc_work, words * 4) != hipSuccess)
      return bail(fail(QRNG_ENOMEM, "multi-class workspace of %llu bytes",
                       (unsigned long long)(words * 4)));
    if (hipMalloc(&pl->mc_args, mc_args_bytes() + nit * sizeof(NttItem)) != hipSuccess ||
        hipMalloc(&pl->mc_counters, 16) != hipSuccess ||
        hipMemset(pl->mc_counters, 0, 16) != hipSuccess)
      return bail(fail(QRNG_ENOMEM, "multi-class arguments"));
    NttItem* mc_dev_items =
        reinterpret_cast<NttItem*>(static_cast<char*>(pl->mc_args) + mc_args_bytes());
    std::vector<int> lg;
    std::vector<uint32_t> cnt;
    std::vector<const NttItem*> idev;
    std::vector<uint32_t*> wk;
    std::vector<NttItem> all;
    uint64_t off = 0;
    for (auto& kv : mc_items) {
      lg.push_back(kv.first);
      cnt.push_back((uint32_t)kv.second.size());
      idev.push_back(mc_dev_items + all.size());
      wk.push_back(pl->mc_work + off);
      off += (uint64_t)kv.second.size() << kv.first;
      all.insert(all.end(), kv.second.begin(), kv.second.end());
    }
    std::vector<char> img(mc_args_bytes());
    McInfo info{};
    if (!mc_build(img.data(), &info, (int)lg.size(), lg.data(), cnt.data(), idev.data(),
                  wk.data(), reinterpret_cast<const uint32_t*>(x_pool),
                  reinterpret_cast<uint32_t*>(y_pool), b.m_arr, estimate ? &est_args : nullptr,
                  nblocks, pl->mc_counters))
      return bail(fail(QRNG_EUNSUPPORTED, "multi-class layout"));
    if (hipMemcpy(pl->mc_args, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(mc_dev_items, all.data(), all.size() * sizeof(NttItem),
                  hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(QRNG_EDEVICE, "multi-class arguments upload"));
    std::vector<std::function<hipError_t(hipStream_t)>> multi;
    const void* margs = pl->mc_args;
    const TwTables tw = ctx->tw;
    for (int pass = 0; pass < 3; ++pass) {
      const uint32_t grid = mc_grid(pass, ctx->num_cus);
      multi.push_back([=](hipStream_t st) { return mc_launch(pass, margs, info, grid, tw, st); });
    }
    // the estimates run in pass B, so the other classes and the singles,
    // which read m, come after the three launches
    multi.insert(multi.end(), other.begin(), other.end());
    multi.insert(multi.end(), singles_steps.begin(), singles_steps.end());
    // default: per-class launches (measured faster on the 4096-block
    // workload: the single persistent kernel of each pass carries the
    // registers and LDS of its longest class into every unit)
    const std::pair<int, int> key{0, tune_key_count(nblocks)};
    bool use_multi = false;
    auto t = ctx->tune.find(key);
    if (t != ctx->tune.end()) use_multi = t->second != 0;
    if (flags & QRNG_PLAN_TUNE) {
      qrng_status e = plan_alloc_work(pl, std::max<uint64_t>(work_need, 256));
      if (e) return bail(e);
      float t_each = 0, t_multi = 0;
      e = time_steps(pl->steps, s, &t_each);
      if (!e) e = time_steps(multi, s, &t_multi);
      if (e) return bail(e);
      use_multi = t_multi <= t_each;
      ctx->tune[key] = use_multi ? 1 : 0;
      ctx->tune_ms[key] = {{0, t_each}, {1, t_multi}};
    }
    if (use_multi) {
      pl->steps = multi;
      pl->multi = true;
      work_need = work_other;
    } else {
      HIP_TRY(hipStreamSynchronize(s));
      (void)hipFree(pl->mc_work);
      pl->mc_work = nullptr;
    }
  }

  // the workspace now fits the chosen shapes (tuning may have left it larger)
  if (pl->work_bytes > 2 * work_need + (64u << 20)) {
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipFree(pl->work);
    pl->work = nullptr;
    pl->work_bytes = 0;
  }
  qrng_status st = plan_alloc_work(pl, std::max<uint64_t>(work_need, 256));
  if (st) return bail(st);

  if (flags & QRNG_PLAN_GRAPH) {
    // capture on a private stream, with the timing hooks off (no event nodes)
    HIP_TRY(hipStreamSynchronize(s));
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return bail(fail(QRNG_EDEVICE, "capture stream"));
    CtxScope off(nullptr);
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    for (auto& f : pl->steps)
      if (e == hipSuccess) e = f(cap);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cap, &gr);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, gr, nullptr, nullptr, 0);
    pl->graph = gr;
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return bail(fail(QRNG_EDEVICE, "graph capture: %s", hipGetErrorString(e)));
  }
  *out = pl;
  return QRNG_OK;
}

qrng_status qrng_plan_execute(qrng_plan* pl, void* stream) {
  if (!pl) return fail(QRNG_EINVAL, "null plan");
  DeviceGuard g(pl->ctx->device);
  CtxScope cs(pl->ctx);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (pl->exec) {
    HIP_TRY(hipGraphLaunch(pl->exec, s));
    return QRNG_OK;
  }
  for (auto& f : pl->steps) {
    const hipError_t e = f(s);
    if (e != hipSuccess) return fail(QRNG_EDEVICE, "plan step: %s", hipGetErrorString(e));
  }
  return QRNG_OK;
}

qrng_status qrng_plan_query(const qrng_plan* pl, qrng_plan_info* info) {
  if (!pl || !info) return fail(QRNG_EINVAL, "null argument");
  info->blocks = pl->nblocks;
  info->classes = pl->classes;
  info->launches = (uint32_t)pl->steps.size();
  info->graph = pl->exec ? 1u : 0u;
  info->workspace_bytes = pl->work_bytes;
  return QRNG_OK;
}

void qrng_plan_destroy(qrng_plan* pl) {
  if (!pl) return;
  DeviceGuard g(pl->ctx->device);
  (void)hipDeviceSynchronize();
  plan_free(pl);
}

qrng_status qrng_tune_export(qrng_ctx* ctx, char* buf, uint64_t cap, uint64_t* len) {
  if (!ctx || !len) return fail(QRNG_EINVAL, "null argument");
  std::ostringstream os;
  for (auto& kv : ctx->tune) {
    if (kv.first.first == 0)  // persistent multi-class form (1) or per-class launches (0)
      os << "multi " << kv.first.second << " " << kv.second << "\n";
    else
      os << "ntt " << kv.first.first << " " << kv.first.second << " " << kv.second << "\n";
    // what the last tuning run measured for this key, as comment lines
    // ("# <line> measured <choice>:<ms> ..."), which qrng_tune_import skips
    auto m = ctx->tune_ms.find(kv.first);
    if (m != ctx->tune_ms.end() && !m->second.empty()) {
      os << "# " << (kv.first.first == 0 ? "multi" : "ntt");
      if (kv.first.first) os << " " << kv.first.first;
      os << " " << kv.first.second << " measured";
      for (auto& cm : m->second) {
        char t[48];
        std::snprintf(t, sizeof t, " %d:%.3f", cm.first, (double)cm.second);
        os << t;
      }
      os << "\n";
    }
  }
  const std::string t = os.str();
  *len = t.size();
  if (buf) {
    if (cap < t.size() + 1) return fail(QRNG_EINVAL, "buffer holds %llu bytes, need %llu",
                                        (unsigned long long)cap, (unsigned long long)(t.size() + 1));
    std::memcpy(buf, t.c_str(), t.size() + 1);
  }
  return QRNG_OK;
}

qrng_status qrng_tune_import(qrng_ctx* ctx, const char* text) {
  if (!ctx || !text) return fail(QRNG_EINVAL, "null argument");
  std::istringstream is(text);
  std::string line;
  std::map<std::pair<int, int>, int> add;
  int ln = 0;
  while (std::getline(is, line)) {
    ++ln;
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    std::string tag;
    int a = 0, c = 0, v = 0;
    if (ls >> tag && tag == "multi") {
      if (!(ls >> c >> v) || c < 0 || c > 32 || (v != 0 && v != 1))
        return fail(QRNG_EINVAL, "tuning table line %d is malformed", ln);
      add[{0, c}] = v;
      continue;
    }
    if (tag != "ntt" || !(ls >> a >> c >> v) || a < 10 || a > 23 || c < 0 || c > 32 ||
        !(v == kTuneDirect || (v >= 10 && v <= kTuneNoCap)))
      return fail(QRNG_EINVAL, "tuning table line %d is malformed", ln);
    add[{a, c}] = v;
  }
  for (auto& kv : add) ctx->tune[kv.first] = kv.second;
  return QRNG_OK;
}

}  // extern "C"

// Serving loop of libqrng (declared in include/qrng.h): continuous batching
// of extraction requests over a stream of raw sample windows.
//
// Each window gets one min-entropy estimate (paper Sec. II) that fixes the
// output length m_s of its n_s-bit blocks (Sec. III.B); requests take
// consecutive blocks of one window and receive the concatenated hashes
// (Sec. III.E: a long raw sequence cut into blocks).  Admission is first come
// first served while the output ring has room; every step enqueues one
// strided hash per run of admitted blocks on the server's own stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <map>
#include <unordered_set>
#include <vector>

#include "host_logic.h"
#include "internal.h"
#include "qrng.h"

using namespace qrng;

namespace {

struct Window {
  uint64_t seq = 0;
  uint32_t slot = 0;
  hipEvent_t est = nullptr;   // estimate copied to the host
  hipEvent_t last = nullptr;  // last hash that reads the window
  bool used = false;          // a hash was enqueued on it
  bool known = false;         // m_s read back
  uint64_t m_s = 0;
  uint64_t cursor = 0;        // next unused block
};

struct Request {
  uint64_t id, bits;
};

struct Admitted {
  qrng_served info;
  hipEvent_t done;  // shared by the requests of one launch run (owned by `events`)
};

}  // namespace

// Hash launches allowed in flight: one running and one queued behind it.
// While both are busy, admitted requests wait and join a later, larger run
// (continuous batching without a launch per host step).
constexpr size_t kMaxRunsInFlight = 2;

struct qrng_server {
  qrng_ctx* ctx = nullptr;
  qrng_server_cfg cfg{};
  hipStream_t stream = nullptr;              // hashes
  hipStream_t est_stream = nullptr;          // window copies and estimates (never
                                             // queued behind hashes)
  uint8_t* slots = nullptr;                  // window_slots x W bytes
  uint32_t* hist = nullptr;                  // estimate scratch (zeroed once)
  qrng_me_result* me = nullptr;              // per slot
  uint64_t* m_dev = nullptr;                 // per slot
  uint64_t* m_host = nullptr;                // pinned, per slot
  uint64_t* ring = nullptr;
  uint64_t ring_words = 0;
  host::OutputRing out;                      // allocation of the ring's words
  std::map<uint64_t, uint64_t> region_of;    // request id -> start word
  std::map<uint64_t, uint64_t> served_bits;  // request id -> R, while its space is held
  std::deque<Window> windows;                // fed, oldest first
  std::vector<bool> slot_busy;
  std::deque<Request> queue;
  std::deque<Admitted> inflight;
  std::unordered_set<uint64_t> inflight_ids;  // admitted, not yet returned by poll
  std::deque<hipEvent_t> events;             // events of launch runs still referenced
  std::deque<hipEvent_t> runs;               // end events of launches that may still run
  std::vector<hipEvent_t> event_pool;
  uint64_t next_id = 1, fed = 0, used = 0, blocks_hashed = 0, bits_served = 0;
  uint64_t nblk = 0;                         // blocks per window
};

namespace {

qrng_status err(qrng_status st, const char* msg) { return set_error(st, "%s", msg); }

#define SRV_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return set_error(QRNG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

hipEvent_t get_event(qrng_server* s) {
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Drop windows that are exhausted and no longer read by pending hashes.
void retire_windows(qrng_server* s) {
  while (!s->windows.empty()) {
    Window& w = s->windows.front();
    if (!w.known || w.cursor < s->nblk) break;  // blocks left to hand out
    if (w.last && hipEventQuery(w.last) == hipErrorNotReady) break;
    if (w.est) s->event_pool.push_back(w.est);
    s->slot_busy[w.slot] = false;
    s->windows.pop_front();
  }
}

// Make the front window's m_s known (waits for its estimate).
qrng_status window_known(qrng_server* s, Window& w) {
  if (w.known) return QRNG_OK;
  SRV_HIP(hipEventSynchronize(w.est));
  w.m_s = s->m_host[w.slot] / 64 * 64;
  w.known = true;
  if (w.m_s == 0) w.cursor = s->nblk;  // no entropy: nothing to hand out
  return QRNG_OK;
}

qrng_status launch_run(qrng_server* s, const Window& w, uint64_t b0, uint64_t nb,
                       uint64_t ring_start, hipEvent_t* done) {
  const uint64_t n = s->cfg.block_bits;
  const uint64_t* x = reinterpret_cast<const uint64_t*>(
      s->slots + (uint64_t)w.slot * s->cfg.window_samples) + b0 * (n / 64);
  uint64_t* y = s->ring + ring_start % s->ring_words;
  qrng_status st = qrng_toeplitz_hash_strided(s->ctx, x, n, n / 64, s->cfg.seed_id, w.m_s, y,
                                              w.m_s / 64, (uint32_t)nb, s->cfg.path, s->stream);
  if (st) return st;
  hipEvent_t e = get_event(s);
  if (!e) return err(QRNG_EDEVICE, "event creation failed");
  SRV_HIP(hipEventRecord(e, s->stream));
  s->events.push_back(e);
  s->runs.push_back(e);
  *done = e;
  s->blocks_hashed += nb;
  return QRNG_OK;
}

// Time the strided hash of one window's worth of n-bit blocks (nominal
// m = 5n/8) and return extracted bits per second.
qrng_status time_block_length(qrng_server* s, uint64_t n, double* rate) {
  const uint64_t W = s->cfg.window_samples * 8;
  const uint64_t nb = W / n;
  uint64_t m = n * 5 / 8;
  const double sec = std::ceil(2.0 * s->cfg.log2_inv_eps);
  m = (uint64_t)std::max(0.0, (double)m - sec) / 64 * 64;
  *rate = 0;
  if (m == 0 || nb == 0 || nb * (m / 64) > s->ring_words) return QRNG_OK;
  hipEvent_t a = nullptr, b = nullptr;
  SRV_HIP(hipEventCreate(&a));
  SRV_HIP(hipEventCreate(&b));
  float best = 1e30f;
  qrng_status st = QRNG_OK;
  for (int r = 0; r < 4 && !st; ++r) {
    if (hipEventRecord(a, s->stream) != hipSuccess) st = QRNG_EDEVICE;
    if (!st)
      st = qrng_toeplitz_hash_strided(s->ctx, reinterpret_cast<const uint64_t*>(s->slots), n,
                                      n / 64, s->cfg.seed_id, m, s->ring, m / 64, (uint32_t)nb,
                                      s->cfg.path, s->stream);
    if (!st && (hipEventRecord(b, s->stream) != hipSuccess ||
                hipEventSynchronize(b) != hipSuccess))
      st = QRNG_EDEVICE;
    float ms = 0;
    if (!st && r > 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess) best = std::min(best, ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st) return st == QRNG_EDEVICE ? err(st, "tuning run failed") : st;
  *rate = (double)(nb * m) / (best * 1e-3);
  return QRNG_OK;
}

void free_server(qrng_server* s) {
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->est_stream) (void)hipStreamSynchronize(s->est_stream);
  for (auto& w : s->windows)
    if (w.est) s->event_pool.push_back(w.est);
  for (hipEvent_t e : s->events) s->event_pool.push_back(e);
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  if (s->slots) (void)hipFree(s->slots);
  if (s->hist) (void)hipFree(s->hist);
  if (s->me) (void)hipFree(s->me);
  if (s->m_dev) (void)hipFree(s->m_dev);
  if (s->m_host) (void)hipHostFree(s->m_host);
  if (s->ring) (void)hipFree(s->ring);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->est_stream) (void)hipStreamDestroy(s->est_stream);
  ctx_pin_seed(s->ctx, s->cfg.seed_id, -1, nullptr);
  ctx_track_server(s->ctx, s, false);
  delete s;
}

// Copy `words` words, keeping only the low `last_bits` bits of the last.
__global__ void k_copy_cut(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                           uint64_t words, uint32_t last_bits) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= words) return;
  uint64_t v = src[i];
  if (i == words - 1 && last_bits < 64) v &= (1ull << last_bits) - 1;
  dst[i] = v;
}

struct Dev {
  int prev = -1;
  explicit Dev(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != d) (void)hipSetDevice(d);
  }
  ~Dev() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" {

qrng_status qrng_server_create(qrng_ctx* ctx, const qrng_server_cfg* cfg, qrng_server** out) {
  if (!out) return err(QRNG_EINVAL, "null server handle");
  *out = nullptr;
  if (!ctx || !cfg) return err(QRNG_EINVAL, "null argument");
  const qrng_server_cfg& c = *cfg;
  if (c.opts.sample_bits != 8) return err(QRNG_EINVAL, "serving takes 8-bit samples");
  if (qrng_status st_o = check_me_opts(c.opts)) return st_o;
  if (std::isnan(c.log2_inv_eps) || c.log2_inv_eps < 0)
    return err(QRNG_EINVAL, "bad security parameter");
  if (c.block_bits % 512) return err(QRNG_EINVAL, "block_bits must be a multiple of 512");
  if (c.window_samples == 0 || c.window_samples > (1ull << 31))
    return err(QRNG_EINVAL, "window_samples must be in [1, 2^31]");
  if (c.ring_bits == 0 || c.ring_bits % 64) return err(QRNG_EINVAL, "ring_bits must be a positive multiple of 64");
  if (c.window_slots < 2 || c.window_slots > 1024) return err(QRNG_EINVAL, "window_slots must be in [2, 1024]");
  if (c.max_queue == 0) return err(QRNG_EINVAL, "max_queue must be positive");
  if (c.path < QRNG_PATH_AUTO || c.path > QRNG_PATH_MFMA) return err(QRNG_EINVAL, "unknown path");
  uint64_t L = 0;
  if (!ctx_pin_seed(ctx, c.seed_id, 0, &L)) return err(QRNG_EINVAL, "unknown seed id");
  if (c.block_bits && ((c.window_samples * 8) % c.block_bits))
    return err(QRNG_EINVAL, "window must hold whole blocks");
  if (c.block_bits && 2 * c.block_bits - 1 > L)
    return err(QRNG_EINVAL, "seed shorter than 2 block_bits - 1");

  Dev g(ctx_device(ctx));
  qrng_server* s = new qrng_server();
  s->ctx = ctx;
  s->cfg = c;
  ctx_pin_seed(ctx, c.seed_id, +1, nullptr);
  ctx_track_server(ctx, s, true);
  const uint32_t K = c.window_slots;
  bool ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
            hipStreamCreateWithFlags(&s->est_stream, hipStreamNonBlocking) == hipSuccess &&
            hipMalloc(&s->slots, (uint64_t)K * c.window_samples) == hipSuccess &&
            hipMalloc(&s->hist, hist_scratch_words() * 4) == hipSuccess &&
            hipMemset(s->hist, 0, hist_scratch_words() * 4) == hipSuccess &&
            hipMalloc(&s->me, (uint64_t)K * sizeof(qrng_me_result)) == hipSuccess &&
            hipMalloc(&s->m_dev, (uint64_t)K * 8) == hipSuccess &&
            hipHostMalloc(&s->m_host, (uint64_t)K * 8, hipHostMallocDefault) == hipSuccess &&
            hipMalloc(&s->ring, c.ring_bits / 8) == hipSuccess;
  if (!ok) {
    free_server(s);
    return err(QRNG_ENOMEM, "server buffers");
  }
  s->ring_words = c.ring_bits / 64;
  s->out.words = s->ring_words;
  s->slot_busy.assign(K, false);
  if (c.block_bits == 0) {
    // serving block length: the candidate that extracts the most bits/s
    double best = 0;
    uint64_t pick = 0;
    for (uint64_t n = 1u << 12; n <= (1u << 18); n <<= 1) {
      if ((c.window_samples * 8) % n || 2 * n - 1 > L) continue;
      s->cfg.block_bits = n;
      double r = 0;
      qrng_status st = time_block_length(s, n, &r);
      if (st) {
        free_server(s);
        return st;
      }
      if (r > best) best = r, pick = n;
    }
    if (!pick) {
      free_server(s);
      return err(QRNG_EINVAL, "no candidate block length fits the window, seed and ring");
    }
    s->cfg.block_bits = pick;
  }
  s->nblk = c.window_samples * 8 / s->cfg.block_bits;
  {
    // load the kernels of both run sizes now (a first launch loads its code
    // object and would stall the first requests): one block, then 64
    const uint64_t n = s->cfg.block_bits;
    for (uint32_t nb : {1u, 64u}) {
      if (nb > s->nblk || nb * (n / 128) > s->ring_words) continue;
      qrng_status st = qrng_toeplitz_hash_strided(ctx, reinterpret_cast<const uint64_t*>(s->slots),
                                                  n, n / 64, c.seed_id, n / 2, s->ring, n / 128,
                                                  nb, s->cfg.path, s->stream);
      if (st) {
        free_server(s);
        return st;
      }
    }
    if (hipStreamSynchronize(s->stream) != hipSuccess) {
      free_server(s);
      return err(QRNG_EDEVICE, "server warm-up failed");
    }
  }
  *out = s;
  return QRNG_OK;
}

qrng_status qrng_server_feed(qrng_server* s, const uint8_t* samples, void* stream) {
  if (!s || !samples) return err(QRNG_EINVAL, "null argument");
  Dev g(ctx_device(s->ctx));
  retire_windows(s);
  uint32_t slot = 0;
  while (slot < s->slot_busy.size() && s->slot_busy[slot]) ++slot;
  if (slot == s->slot_busy.size()) return err(QRNG_EBUSY, "every window slot is in use");
  const uint64_t W = s->cfg.window_samples;
  hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
  uint8_t* dst = s->slots + (uint64_t)slot * W;
  SRV_HIP(hipMemcpyAsync(dst, samples, W, hipMemcpyDeviceToDevice, cs));
  hipEvent_t copied = get_event(s);
  if (!copied) return err(QRNG_EDEVICE, "event creation failed");
  SRV_HIP(hipEventRecord(copied, cs));
  SRV_HIP(hipStreamWaitEvent(s->est_stream, copied, 0));
  s->event_pool.push_back(copied);  // reusable once recorded again later; waits are enqueued
  // the window's estimate, with n = n_s: m_s for its blocks
  MeDevArgs a{};
  a.N = 8;
  a.model = s->cfg.opts.model;
  a.u_mode = s->cfg.opts.u_mode;
  a.mu = s->cfg.opts.mu;
  a.sigma = s->cfg.opts.sigma;
  a.n = s->cfg.block_bits;
  a.log2_inv_eps = s->cfg.log2_inv_eps;
  a.m_cap = s->cfg.block_bits;
  a.out = s->me + slot;
  a.m_out = s->m_dev + slot;
  SRV_HIP(hist_estimate(dst, W, 8, s->hist, nullptr, &a, s->est_stream, 0, 0,
                        (uint32_t)((s->fed + 1) & ((1u << 23) - 1))));
  SRV_HIP(hipMemcpyAsync(s->m_host + slot, s->m_dev + slot, 8, hipMemcpyDeviceToHost,
                         s->est_stream));
  Window w;
  w.seq = s->fed++;
  w.slot = slot;
  w.est = get_event(s);
  if (!w.est) return err(QRNG_EDEVICE, "event creation failed");
  // hashes of this window start only after the host has waited for this
  // event (window_known), which orders them after the copy
  SRV_HIP(hipEventRecord(w.est, s->est_stream));
  s->slot_busy[slot] = true;
  s->windows.push_back(w);
  return QRNG_OK;
}

qrng_status qrng_server_submit(qrng_server* s, uint64_t bits, uint64_t* id) {
  if (!s || !id) return err(QRNG_EINVAL, "null argument");
  if (bits == 0) return err(QRNG_EINVAL, "a request needs at least one bit");
  if (s->queue.size() >= s->cfg.max_queue) return err(QRNG_EBUSY, "request queue is full");
  *id = s->next_id++;
  s->queue.push_back(Request{*id, bits});
  return QRNG_OK;
}

qrng_status qrng_server_submit_many(qrng_server* s, const uint64_t* bits, uint32_t count,
                                    uint64_t* ids, uint32_t* accepted) {
  if (!s || (count && (!bits || !ids)) || !accepted) return err(QRNG_EINVAL, "null argument");
  for (uint32_t i = 0; i < count; ++i)
    if (bits[i] == 0) return err(QRNG_EINVAL, "a request needs at least one bit");
  uint32_t k = 0;
  while (k < count && s->queue.size() < s->cfg.max_queue) {
    ids[k] = s->next_id++;
    s->queue.push_back(Request{ids[k], bits[k]});
    ++k;
  }
  *accepted = k;
  return QRNG_OK;
}

qrng_status qrng_server_release_many(qrng_server* s, const uint64_t* ids, uint32_t count) {
  if (!s || (count && !ids)) return err(QRNG_EINVAL, "null argument");
  for (uint32_t i = 0; i < count; ++i) {
    auto it = s->region_of.find(ids[i]);
    if (it == s->region_of.end() || s->inflight_ids.count(ids[i])) continue;
    s->out.release(it->second);
    s->region_of.erase(it);
    s->served_bits.erase(ids[i]);
  }
  s->out.reclaim();
  return QRNG_OK;
}

qrng_status qrng_server_step(qrng_server* s, uint32_t* admitted) {
  if (!s) return err(QRNG_EINVAL, "null server");
  Dev g(ctx_device(s->ctx));
  uint32_t adm = 0;
  retire_windows(s);
  while (!s->runs.empty() && hipEventQuery(s->runs.front()) == hipSuccess) s->runs.pop_front();
  if (s->runs.size() >= kMaxRunsInFlight) {
    if (admitted) *admitted = 0;
    return QRNG_OK;
  }
  // the current window is the oldest one with blocks left
  size_t wi = 0;
  while (!s->queue.empty() && wi < s->windows.size()) {
    Window& w = s->windows[wi];
    qrng_status st = window_known(s, w);
    if (st) return st;
    if (w.cursor >= s->nblk) {
      ++wi;
      continue;
    }
    // admit a run of requests on this window while blocks and ring space last
    std::vector<qrng_served> run;
    uint64_t run_start = 0, run_blocks = 0, b0 = w.cursor;
    bool ring_full = false, next_window = false;
    while (!s->queue.empty()) {
      const Request r = s->queue.front();
      const uint64_t k = (r.bits + w.m_s - 1) / w.m_s;
      if (k > s->nblk || k * (w.m_s / 64) > s->ring_words) {
        // can never be served: report it as failed
        qrng_served f{};
        f.request_id = r.id;
        f.bits = r.bits;
        f.status = QRNG_EUNSUPPORTED;
        f.m_block = w.m_s;
        s->inflight.push_back(Admitted{f, nullptr});
        s->queue.pop_front();
        continue;
      }
      if (w.cursor + k > s->nblk) {
        next_window = true;
        break;
      }
      uint64_t start = 0;
      if (!s->out.alloc(k * (w.m_s / 64), &start)) {
        ring_full = true;
        break;
      }
      if (!run.empty() && start != run_start + run_blocks * (w.m_s / 64)) {
        // the ring wrapped: launch what is contiguous so far
        hipEvent_t done = nullptr;
        st = launch_run(s, w, b0, run_blocks, run_start, &done);
        if (st) return st;
        for (auto& q : run) s->inflight.push_back(Admitted{q, done});
        w.last = done;
        if (!w.used) ++s->used;
        w.used = true;
        run.clear();
        b0 = w.cursor;
        run_blocks = 0;
      }
      if (run.empty()) run_start = start;
      qrng_served q{};
      q.request_id = r.id;
      q.bits = r.bits;
      q.ring_word = start % s->ring_words;
      q.window = w.seq;
      q.first_block = w.cursor;
      q.blocks = (uint32_t)k;
      q.status = QRNG_OK;
      q.m_block = w.m_s;
      s->region_of[r.id] = start;
      s->served_bits[r.id] = r.bits;
      s->inflight_ids.insert(r.id);
      run.push_back(q);
      run_blocks += k;
      w.cursor += k;
      s->queue.pop_front();
      ++adm;
    }
    if (!run.empty()) {
      hipEvent_t done = nullptr;
      st = launch_run(s, w, b0, run_blocks, run_start, &done);
      if (st) return st;
      for (auto& q : run) s->inflight.push_back(Admitted{q, done});
      w.last = done;
      if (!w.used) ++s->used;
      w.used = true;
    }
    if (ring_full) break;
    if (next_window) {
      w.cursor = s->nblk;  // first come first served: the head moves on
      ++wi;
    }
  }
  if (admitted) *admitted = adm;
  return QRNG_OK;
}

qrng_status qrng_server_poll(qrng_server* s, qrng_served* out, uint32_t cap, uint32_t* count) {
  if (!s || !count || (cap && !out)) return err(QRNG_EINVAL, "null argument");
  Dev g(ctx_device(s->ctx));
  uint32_t k = 0;
  while (k < cap && !s->inflight.empty()) {
    Admitted& a = s->inflight.front();
    if (a.done) {
      const hipError_t q = hipEventQuery(a.done);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return set_error(QRNG_EDEVICE, "hash run failed: %s", hipGetErrorString(q));
    }
    out[k++] = a.info;
    if (a.info.status == QRNG_OK) s->bits_served += a.info.bits;
    s->inflight_ids.erase(a.info.request_id);
    s->inflight.pop_front();
  }
  // events go back to the pool once no request or window refers to them;
  // events and the requests' references are both in launch order, so only
  // the oldest referenced event needs looking up
  hipEvent_t first_ref = nullptr;
  for (auto& a : s->inflight)
    if (a.done) {
      first_ref = a.done;
      break;
    }
  while (!s->events.empty()) {
    const hipEvent_t e = s->events.front();
    bool ref = e == first_ref || (!s->runs.empty() && e == s->runs.front());
    for (auto& w : s->windows)
      if (w.last == e) ref = true;
    if (ref) break;
    s->events.pop_front();
    s->event_pool.push_back(e);
  }
  retire_windows(s);
  *count = k;
  return QRNG_OK;
}

qrng_status qrng_server_release(qrng_server* s, uint64_t id) {
  if (!s) return err(QRNG_EINVAL, "null server");
  auto it = s->region_of.find(id);
  if (it == s->region_of.end()) return err(QRNG_EINVAL, "no ring space held by this request");
  if (s->inflight_ids.count(id)) return err(QRNG_EBUSY, "request not completed yet");
  s->out.release(it->second);
  s->region_of.erase(it);
  s->served_bits.erase(id);
  s->out.reclaim();
  return QRNG_OK;
}

qrng_status qrng_server_read(qrng_server* s, uint64_t id, uint64_t* out, void* stream) {
  if (!s || !out) return err(QRNG_EINVAL, "null argument");
  if ((reinterpret_cast<uintptr_t>(out) & 7u) != 0) return err(QRNG_EINVAL, "output must be 8-byte aligned");
  auto it = s->region_of.find(id);
  if (it == s->region_of.end()) return err(QRNG_EINVAL, "no ring space held by this request");
  if (s->inflight_ids.count(id)) return err(QRNG_EBUSY, "request not completed yet");
  if (!s->out.find(it->second)) return err(QRNG_EINVAL, "request region missing");
  // the request's bits: R of the words it holds
  const auto sb = s->served_bits.find(id);
  if (sb == s->served_bits.end()) return err(QRNG_EINVAL, "unknown request");
  const uint64_t bits = sb->second;
  Dev g(ctx_device(s->ctx));
  const uint64_t words = (bits + 63) / 64;
  const uint32_t last = (uint32_t)(bits - (words - 1) * 64);
  hipStream_t cs = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_copy_cut, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, cs,
                     s->ring + it->second % s->ring_words, out, words, last);
  SRV_HIP(hipGetLastError());
  return QRNG_OK;
}

qrng_status qrng_server_ring(qrng_server* s, const uint64_t** ring) {
  if (!s || !ring) return err(QRNG_EINVAL, "null argument");
  *ring = s->ring;
  return QRNG_OK;
}

qrng_status qrng_server_window(qrng_server* s, uint64_t window, const uint8_t** samples,
                               const qrng_me_result** est) {
  if (!s) return err(QRNG_EINVAL, "null server");
  for (auto& w : s->windows)
    if (w.seq == window) {
      if (samples) *samples = s->slots + (uint64_t)w.slot * s->cfg.window_samples;
      if (est) *est = s->me + w.slot;
      return QRNG_OK;
    }
  return err(QRNG_EINVAL, "window is not held");
}

qrng_status qrng_server_query(qrng_server* s, qrng_server_stats* st) {
  if (!s || !st) return err(QRNG_EINVAL, "null argument");
  st->block_bits = s->cfg.block_bits;
  st->blocks_per_window = s->nblk;
  st->windows_fed = s->fed;
  st->windows_used = s->used;
  st->blocks_hashed = s->blocks_hashed;
  st->bits_served = s->bits_served;
  st->queued = s->queue.size();
  st->in_flight = s->inflight.size();
  st->ring_free_bits = s->out.free_words() * 64;
  st->m_block = 0;
  for (auto& w : s->windows)
    if (w.known && w.cursor < s->nblk) {
      st->m_block = w.m_s;
      break;
    }
  return QRNG_OK;
}

void qrng_server_destroy(qrng_server* s) {
  if (!s) return;
  Dev g(ctx_device(s->ctx));
  free_server(s);
}

}  // extern "C"

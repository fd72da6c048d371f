// Host-side logic of libqrng that touches no device: the host finish of the
// min-entropy estimate (paper Sec. II), the output-length rule (Sec. III.B)
// and the serving loop's output ring.  Kept free of HIP so that it also
// builds as plain C++ for the host-only tests (sanitizer builds).
#pragma once
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "qrng.h"

namespace qrng {
namespace host {

inline double phi(double z) { return 0.5 * std::erfc(-z / std::sqrt(2.0)); }

// The counts of an estimate over every sample: the K bins plus the
// out-of-range bin must add up to the S samples counted, else a partial
// histogram was lost or counted twice and the estimate must not be used.
inline bool counts_consistent(const unsigned long long* c, int K, unsigned long long oob,
                              uint64_t S) {
  if (oob > S) return false;
  unsigned long long t = oob;
  for (int v = 0; v < K; ++v) {
    if (c[v] > S - t) return false;  // also catches wrap-around
    t += c[v];
  }
  return t == S;
}

constexpr double kTieRel = 1e-9;  // relative closeness treated as a tie of model bins

// Sec. II on the host: model P, H_min, d_U, Delta H_m, H_modify.
inline void minentropy_finish(const unsigned long long* c, int N, const qrng_me_opts& o,
                       qrng_me_result* r) {
  const int K = 1 << N;
  double S = 0.0;
  for (int v = 0; v < K; ++v) S += (double)c[v];
  double mu, sigma;
  if (o.model == QRNG_MODEL_GIVEN) {
    mu = o.mu;
    sigma = o.sigma;
  } else {
    double s1 = 0.0;
    for (int v = 0; v < K; ++v) s1 += (double)v * (double)c[v];
    mu = s1 / S;
    double s2 = 0.0;
    for (int v = 0; v < K; ++v) s2 += ((double)v - mu) * ((double)v - mu) * (double)c[v];
    // Sec. II.B: the quantum part of the variance, sigma_q^2 = sigma^2 - sigma_c^2
    const double var = s2 / S - (o.model == QRNG_MODEL_QUANTUM ? o.sigma * o.sigma : 0.0);
    sigma = var > 0.0 ? std::sqrt(var) : 0.0;
  }
  std::vector<double> P(K);
  if (sigma > 0.0) {
    for (int v = 0; v < K; ++v) {
      const double lo = v == 0 ? 0.0 : phi(((double)v - 0.5 - mu) / sigma);
      const double hi = v == K - 1 ? 1.0 : phi(((double)v + 0.5 - mu) / sigma);
      P[v] = hi - lo;
    }
  } else {  // every sample equal: the model is a point mass
    const double at = std::min<double>(std::max<double>(std::floor(mu + 0.5), 0.0), K - 1);
    for (int v = 0; v < K; ++v) P[v] = (v == (int)at) ? 1.0 : 0.0;
  }
  // model argmax: lowest value whose P is within kTieRel of the maximum (a
  // model centred between two codes has two equal bins; rounding must not
  // decide between them); observed argmax: lowest value on exact ties
  double pmax = P[0];
  int ua = 0;
  for (int v = 1; v < K; ++v) {
    pmax = std::max(pmax, P[v]);
    if (c[v] > c[ua]) ua = v;
  }
  int um = 0;
  while (P[um] < pmax * (1.0 - kTieRel)) ++um;
  std::vector<int> U;
  if (o.u_mode == QRNG_U_MODEL_ARGMAX) {
    U.push_back(um);
  } else if (o.u_mode == QRNG_U_BOTH_ARGMAX) {
    // every value tied for the model's maximum, and the observed argmax
    for (int v = 0; v < K; ++v)
      if (P[v] >= pmax * (1.0 - kTieRel) || v == ua) U.push_back(v);
  } else {
    for (int v = 0; v < K; ++v) U.push_back(v);
  }
  double d = 0.0;
  for (int u : U) d += std::fabs((double)c[u] / S - P[u]);
  d *= 0.5;
  r->mu_hat = mu;
  r->sigma_hat = sigma;
  r->h_min = -std::log2(pmax);
  r->h_actual = c[ua] ? -std::log2((double)c[ua] / S) : INFINITY;
  r->d_u = d;
  r->delta_h_m = std::log2(d * std::ldexp(1.0, N + 1) + 1.0);
  r->h_mod = r->h_min - r->delta_h_m;
  r->argmax_model = (uint32_t)um;
  r->argmax_empirical = (uint32_t)ua;
  r->samples = (uint64_t)S;
}


// Sec. III.B output length m = n H/N - 2 log2(1/eps): H in whole bits per
// sample (floor of h_mod, clamped to [0, N]), the security term rounded up,
// m clamped at 0.  Arguments are checked by the caller (N in 1..16, h_mod
// and log2_inv_eps not NaN, log2_inv_eps >= 0).
inline uint64_t output_bits_rule(uint64_t n, int N, double h_mod, double log2_inv_eps) {
  double h = std::floor(h_mod);
  if (!(h > 0)) h = 0;
  if (h > N) h = N;
  const uint64_t base = (uint64_t)((unsigned __int128)n * (uint64_t)h / (uint64_t)N);
  const double secd = std::ceil(2.0 * log2_inv_eps);
  const uint64_t sec = secd >= 1.8e19 ? UINT64_MAX : (uint64_t)secd;
  return base > sec ? base - sec : 0;
}

// The serving loop's output ring of `words` 64-bit words: regions at
// increasing (monotone) positions head, modulo the ring; a region that would
// cross the end starts at the beginning instead (the skipped tail is a region
// released at once).  Space comes back in allocation order: tail advances
// over released regions only.
struct OutputRing {
  struct Region {
    uint64_t words;
    bool released;
  };
  uint64_t words = 0;
  uint64_t head = 0, tail = 0;       // allocated / reclaimed (monotone)
  std::map<uint64_t, Region> regions;  // by monotone start

  // *start receives the monotone start (start % words is the ring word)
  bool alloc(uint64_t n, uint64_t* start) {
    const uint64_t R = words;
    if (n == 0 || n > R) return false;
    uint64_t pad = 0;
    const uint64_t pos = head % R;
    if (pos + n > R) pad = R - pos;
    if (head + pad + n - tail > R) return false;
    if (pad) {
      regions[head] = Region{pad, true};
      head += pad;
    }
    regions[head] = Region{n, false};
    *start = head;
    head += n;
    return true;
  }
  // marks a region released (false if no region starts there)
  bool release(uint64_t start) {
    auto r = regions.find(start);
    if (r == regions.end()) return false;
    r->second.released = true;
    return true;
  }
  const Region* find(uint64_t start) const {
    auto r = regions.find(start);
    return r == regions.end() ? nullptr : &r->second;
  }
  void reclaim() {
    while (!regions.empty() && regions.begin()->second.released) {
      tail = regions.begin()->first + regions.begin()->second.words;
      regions.erase(regions.begin());
    }
    if (regions.empty()) tail = head;
  }
  uint64_t free_words() const { return words - (head - tail); }
};

}  // namespace host
}  // namespace qrng

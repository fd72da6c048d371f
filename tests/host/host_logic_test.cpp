// Host-only test driver for the device-free logic of libqrng (host_logic.h),
// built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_logic.py.  Commands on stdin, one per line:
//   finish N model mu sigma u_mode c_0 .. c_{2^N - 1}
//       -> "finish mu sigma h_min h_actual d_u delta_h_m h_mod argmax_model"
//   bits n N h_mod log2_inv_eps          -> "bits m"
//   ring words seed steps                -> "ring ok allocated released" after a
//       randomized run of allocations and releases checked against the
//       ring's invariants (it aborts on the first violation)
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <iostream>
#include <random>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "host_logic.h"

using qrng::host::OutputRing;

static void check(bool c, const char* what) {
  if (!c) {
    std::fprintf(stderr, "ring invariant violated: %s\n", what);
    std::abort();
  }
}

static void ring_run(uint64_t words, uint64_t seed, int steps) {
  OutputRing r;
  r.words = words;
  std::mt19937_64 g(seed);
  struct Live {
    uint64_t start, n;
  };
  std::deque<Live> live;  // allocation order
  uint64_t allocated = 0, released = 0;
  for (int t = 0; t < steps; ++t) {
    if (live.empty() || g() % 3 != 0) {
      const uint64_t n = 1 + g() % (words / 3 + 1);
      const uint64_t before = r.free_words();
      uint64_t st = 0;
      if (r.alloc(n, &st)) {
        ++allocated;
        // inside the ring without wrapping, disjoint from every live region
        check(st % words + n <= words, "region crosses the end of the ring");
        for (auto& l : live) {
          const uint64_t a0 = st % words, b0 = l.start % words;
          check(a0 + n <= b0 || b0 + l.n <= a0, "live regions overlap");
        }
        check(r.free_words() + n <= before, "free space did not shrink");
        live.push_back(Live{st, n});
      } else {
        // refused only when it cannot fit: too long, or (with the skipped
        // tail of the ring when it would cross the end) over the free space
        const uint64_t pos = r.head % words;
        const uint64_t pad = pos + n > words ? words - pos : 0;
        check(n > words || pad + n > r.free_words(), "allocation refused with room left");
      }
    } else {
      // release a random live region (out of order), reclaim in order
      const size_t k = g() % live.size();
      check(r.release(live[k].start), "release of a live region failed");
      live.erase(live.begin() + (long)k);
      ++released;
      r.reclaim();
      check(r.head - r.tail <= words, "more than the ring in use");
      if (live.empty()) check(r.head == r.tail, "nothing live but space held");
      else check(r.tail <= live.front().start, "tail passed a live region");
    }
  }
  std::printf("ring ok %llu %llu\n", (unsigned long long)allocated,
              (unsigned long long)released);
}

int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    std::istringstream is(line);
    std::string cmd;
    is >> cmd;
    if (cmd == "finish") {
      int N, model, u_mode;
      double mu, sigma;
      is >> N >> model >> mu >> sigma >> u_mode;
      std::vector<unsigned long long> c(1u << N);
      for (auto& v : c) is >> v;
      qrng_me_opts o{};
      o.sample_bits = N;
      o.model = model;
      o.mu = mu;
      o.sigma = sigma;
      o.u_mode = u_mode;
      qrng_me_result r{};
      qrng::host::minentropy_finish(c.data(), N, o, &r);
      std::printf("finish %.17g %.17g %.17g %.17g %.17g %.17g %.17g %u\n", r.mu_hat,
                  r.sigma_hat, r.h_min, r.h_actual, r.d_u, r.delta_h_m, r.h_mod,
                  r.argmax_model);
    } else if (cmd == "counts") {
      int K;
      unsigned long long oob, S;
      is >> K >> oob >> S;
      std::vector<unsigned long long> c(K);
      for (auto& v : c) is >> v;
      std::printf("counts %d\n", qrng::host::counts_consistent(c.data(), K, oob, S) ? 1 : 0);
    } else if (cmd == "bits") {
      unsigned long long n;
      int N;
      double h, e;
      is >> n >> N >> h >> e;
      std::printf("bits %llu\n",
                  (unsigned long long)qrng::host::output_bits_rule(n, N, h, e));
    } else if (cmd == "ring") {
      unsigned long long w, seed;
      int steps;
      is >> w >> seed >> steps;
      ring_run(w, seed, steps);
    }
  }
  return 0;
}

// Host loops of the plan builder (parallel_ranges over the persistent worker
// pool): every part runs once on its own contiguous range, loops nested in a
// part run in place, the first exception in part order reaches the caller
// after every part ended, and callers on several threads at once each get
// their own results.  Built with ThreadSanitizer by test_host_pool.py.
#include <atomic>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "host_pool.h"

using afmm::parallel_ranges;

static int fail(const char* what) {
  std::printf("FAIL %s\n", what);
  return 1;
}

int main() {
  for (int rep = 0; rep < 100; ++rep) {
    const int64_t n = 100003;
    std::vector<int64_t> sum(16, 0), lo(16, -1), hi(16, -1);
    std::atomic<int> inner_bad{0};
    parallel_ranges(n, 16, [&](int64_t b, int64_t e, int p) {
      int64_t s = 0;
      for (int64_t i = b; i < e; ++i) s += i;
      sum[p] = s;
      lo[p] = b;
      hi[p] = e;
      std::vector<int64_t> w(4, 0);
      parallel_ranges(10, 4, [&](int64_t b2, int64_t e2, int q) { w[q] = e2 - b2; });
      if (w[0] + w[1] + w[2] + w[3] != 10) ++inner_bad;
    });
    int64_t tot = 0;
    for (int p = 0; p < 16; ++p) {
      tot += sum[p];
      if (lo[p] != n * p / 16 || hi[p] != n * (p + 1) / 16) return fail("range bounds");
    }
    if (tot != n * (n - 1) / 2) return fail("sum");
    if (inner_bad) return fail("nested loop");
    std::atomic<int> ran{0};
    std::string caught;
    try {
      parallel_ranges(1000, 8, [&](int64_t, int64_t, int p) {
        ++ran;
        if (p == 5) throw std::runtime_error("five");
        if (p == 3) throw std::runtime_error("three");
      });
    } catch (const std::runtime_error& e) {
      caught = e.what();
    }
    if (caught != "three" || ran != 8) return fail("exception");
  }
  std::vector<std::thread> callers;
  std::atomic<int> bad{0};
  for (int c = 0; c < 4; ++c)
    callers.emplace_back([&bad, c] {
      for (int r = 0; r < 100; ++r) {
        std::vector<int64_t> v(16, -1);
        parallel_ranges(16 * (c + 1), 16, [&](int64_t b, int64_t e, int p) { v[p] = e - b; });
        for (int64_t x : v)
          if (x != c + 1) ++bad;
      }
    });
  for (auto& t : callers) t.join();
  if (bad) return fail("concurrent callers");
  std::printf("ok\n");
  return 0;
}

// Minimal static-chunked parallel loop over std::thread.
#pragma once
#include <algorithm>
#include <atomic>
#include <thread>
#include <vector>

namespace fc {

template <class F>
void parallel_for(int64_t n, F&& f) {
  int nt = host_threads();
  if (n <= 0) return;
  if (nt <= 1 || n < 2) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  // dynamic chunks keep uneven work (cut cells) balanced
  std::atomic<int64_t> next(0);
  int64_t chunk = std::max<int64_t>(1, n / (int64_t(nt) * 16));
  std::vector<std::thread> pool;
  pool.reserve(nt);
  for (int t = 0; t < nt; ++t) {
    pool.emplace_back([&]() {
      for (;;) {
        int64_t s = next.fetch_add(chunk);
        if (s >= n) break;
        int64_t e = std::min(n, s + chunk);
        for (int64_t i = s; i < e; ++i) f(i);
      }
    });
  }
  for (auto& th : pool) th.join();
}

}  // namespace fc

// Host check of the multiply-shift division the lattice kernels use for
// run-time divisors (Granlund and Montgomery, division by invariant integers
// using multiplication): fdiv(n, make_fastdiv(d)) must equal n / d for every
// 32-bit n.  Built with hipcc (the helper is host and device code) and run
// on the CPU; prints the number of checked pairs and mismatches.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "dev_common.h"

int main() {
  std::vector<uint32_t> ds;
  for (uint32_t d = 1; d <= 4096; ++d) ds.push_back(d);
  for (int k = 12; k < 32; ++k) {
    const uint32_t p = 1u << k;
    ds.push_back(p - 1);
    ds.push_back(p);
    ds.push_back(p + 1);
    ds.push_back(p + p / 3);
  }
  ds.push_back(0xffffffffu);
  uint64_t checked = 0, bad = 0;
  uint64_t state = 0x9e3779b97f4a7c15ull;   // xorshift64 for sample numerators
  auto next = [&]() {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (uint32_t)(state >> 16);
  };
  for (uint32_t d : ds) {
    const fc::FastDiv f = fc::make_fastdiv(d);
    std::vector<uint32_t> ns = {0u, 1u, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7fffffffu,
                                0x80000000u, 0xfffffffeu, 0xffffffffu};
    for (uint32_t q = 1; q < 64; ++q) {   // around multiples of d
      const uint64_t m = (uint64_t)q * d * 977u;
      if (m <= 0xffffffffull) {
        ns.push_back((uint32_t)m);
        ns.push_back((uint32_t)m - 1);
      }
    }
    for (int r = 0; r < 2000; ++r) ns.push_back(next());
    for (uint32_t n = 0; n < 4096; ++n) ns.push_back(n);
    for (uint32_t n : ns) {
      ++checked;
      if (fc::fdiv(n, f) != n / d) {
        if (bad < 10) std::printf("mismatch n=%u d=%u got %u\n", n, d, fc::fdiv(n, f));
        ++bad;
      }
    }
  }
  std::printf("checked %llu mismatches %llu\n", (unsigned long long)checked,
              (unsigned long long)bad);
  return bad == 0 ? 0 : 1;
}

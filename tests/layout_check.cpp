// Host check of the stored layout of the symmetric local inverses
// (sym_offset): for every block size m, the (m/2 + 1) x m stored entries
// (k, i) map one-to-one onto [0, (m/2 + 1) m); for m <= 64 the entries
// (2j, i) and (2j + 1, i) of complete row pairs are adjacent, in that order
// (one two-wide load per lane), and an odd last stored row is contiguous in
// i.  Prints the number of block sizes checked and of failures.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "schwarz_dev.h"

int main() {
  int checked = 0, bad = 0;
  for (int m = 1; m <= 256; ++m) {
    const int h = m / 2;
    const int64_t n = (int64_t)(h + 1) * m;
    if (fc::sym_block_stride_dev(m) != n) ++bad;
    std::vector<int> seen((size_t)n, 0);
    for (int k = 0; k <= h; ++k)
      for (int i = 0; i < m; ++i) {
        const int64_t o = fc::sym_offset(k, i, m);
        if (o < 0 || o >= n) {
          ++bad;
          continue;
        }
        ++seen[(size_t)o];
      }
    for (int64_t o = 0; o < n; ++o)
      if (seen[(size_t)o] != 1) ++bad;
    if (m <= 64) {
      const int npair = (h + 1) & ~1;
      for (int k = 0; k + 1 < npair; k += 2)
        for (int i = 0; i < m; ++i)
          if (fc::sym_offset(k + 1, i, m) != fc::sym_offset(k, i, m) + 1 ||
              fc::sym_offset(k, i, m) != (int64_t)k * m + 2 * i)
            ++bad;
      if (npair < h + 1)
        for (int i = 0; i < m; ++i)
          if (fc::sym_offset(h, i, m) != (int64_t)h * m + i) ++bad;
    } else {
      for (int k = 0; k <= h; ++k)
        for (int i = 0; i < m; ++i)
          if (fc::sym_offset(k, i, m) != (int64_t)k * m + i) ++bad;
    }
    ++checked;
  }
  std::printf("block sizes %d failures %d\n", checked, bad);
  return bad == 0 ? 0 : 1;
}

// Host check of the pruner's epoch order (row_perm.h): for every n given on
// the command line and a few seeds and epochs, prints one line
//   n seed epoch bijective mean_walk fixed_points first_index
// where bijective is 1 when the order hits every row of 0..n-1 exactly once.
#define __host__
#define __device__
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "row_perm.h"

int main(int argc, char **argv) {
  const unsigned long long seeds[] = {0ULL, 1ULL, 0xdeadbeefULL};
  for (int a = 1; a < argc; ++a) {
    const long long n = atoll(argv[a]);
    for (unsigned long long seed : seeds)
      for (int epoch = 0; epoch < 3; ++epoch) {
        const RowPerm p = make_row_perm(n, seed, epoch);
        std::vector<unsigned char> hit((size_t)n, 0);
        bool ok = true;
        long long fixed = 0;
        for (long long i = 0; i < n; ++i) {
          const long long r = row_perm(p, i);
          if (r < 0 || r >= n || hit[(size_t)r]) { ok = false; break; }
          hit[(size_t)r] = 1;
          fixed += r == i;
        }
        // mean number of Feistel evaluations per index (cycle walking)
        const unsigned long long dom = 1ULL << (2 * p.h);
        printf("%lld %llu %d %d %.4f %lld %lld %llu\n", n, seed, epoch, ok ? 1 : 0,
               (double)dom / (double)n, fixed, row_perm(p, 0), dom);
      }
  }
  return 0;
}

// Row order of one training epoch of the learned pruner: a keyed
// pseudo-random permutation of 0..n-1, evaluated per index so that no index
// buffer is built or shuffled.  A balanced four-round Feistel network on
// 2h-bit integers (2^(2h) >= n) is a bijection of [0, 2^(2h)); cycle walking
// (apply it again while the result is >= n) restricts it to a bijection of
// [0, n) (Black and Rogaway, "Ciphers with arbitrary finite domains", 2002).
// The walk from an index below n returns below n within the index's cycle, and
// with 2^(2h) < 4n it takes fewer than four steps on average.  The round
// function is the SplitMix64 output mix (Steele, Lea and Flood, 2014) of the
// half and a round key.  Host and device share these functions, so the order
// can be checked on the host.
#pragma once

struct RowPerm {
  unsigned long long key[4];
  long long n;
  int h;    // half width in bits of the Feistel domain
  int on;   // 0: identity
};

__host__ __device__ inline unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__host__ __device__ inline long long row_perm(const RowPerm &p, long long i) {
  const unsigned long long mask = (1ULL << p.h) - 1ULL;
  unsigned long long x = (unsigned long long)i;
  do {
    unsigned long long l = x >> p.h, r = x & mask;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned long long t = l ^ (mix64(r ^ p.key[k]) & mask);
      l = r;
      r = t;
    }
    x = (l << p.h) | r;
  } while (x >= (unsigned long long)p.n);
  return (long long)x;
}

// Order of epoch `epoch` of a run seeded with `seed`, over n >= 1 rows.
__host__ __device__ inline RowPerm make_row_perm(long long n, unsigned long long seed, int epoch) {
  RowPerm p{};
  int b = 2;
  while (b < 62 && (1LL << b) < n) ++b;
  p.h = (b + 1) / 2;
  p.n = n;
  for (int k = 0; k < 4; ++k)
    p.key[k] = mix64(seed ^ mix64(0x9e3779b97f4a7c15ULL * (unsigned long long)(4 * epoch + k + 1)));
  p.on = 1;
  return p;
}

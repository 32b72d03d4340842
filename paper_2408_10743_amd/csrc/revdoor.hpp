// revdoor.hpp -- revolving-door order of the t-subsets of {0, .., P-1} and
// its ranking by the combinatorial number system.
//
// The order is the recursive list in which the t-subsets of {0, .., p-1}
// that avoid p-1 come first, in their own order, and those containing p-1
// follow, their other t-1 elements running backwards through the order of
// {0, .., p-2}.  Consecutive subsets then differ by one element out and one
// in, and the subset c_1 < .. < c_t has rank
//     C(c_t + 1, t) - 1 - rank(c_1 .. c_{t-1}),   rank of the empty set 0,
// since the C(c_t, t) subsets below c_t precede it.
//
// Plain C++: the includer may define QD_HD (e.g. __host__ __device__).
#pragma once
#include <cstdint>

#ifndef QD_HD
#define QD_HD
#endif

namespace qd {

// Subset of revolving-door rank `rank` (0 <= rank < C(P, t)) among the
// t-subsets of {0, .., P-1}, written in decreasing order to c[0..t-1].
// binom[p * ld + r] = C(p, r) for 0 <= p <= P, 0 <= r <= t.
QD_HD inline void revdoor_unrank(unsigned long long rank, int t, int P, const unsigned long long *binom, int ld,
                                 int *c) {
  int hi = P;  // elements of the remaining subset are below hi
  for (int k = 0; k < t; ++k) {
    const int r = t - k;
    // largest e < hi with C(e, r) <= rank (C(r - 1, r) = 0)
    int a = r - 1, b = hi - 1;
    while (a < b) {
      const int mid = (a + b + 1) >> 1;
      if (binom[static_cast<unsigned long long>(mid) * ld + r] <= rank) a = mid;
      else b = mid - 1;
    }
    c[k] = a;
    rank = binom[static_cast<unsigned long long>(a + 1) * ld + r] - 1 - rank;
    hi = a;
  }
}

// Rank of the subset c[0..t-1] given in decreasing order.
QD_HD inline unsigned long long revdoor_rank(int t, const int *c, const unsigned long long *binom, int ld) {
  unsigned long long rank = 0;
  for (int k = t - 1; k >= 0; --k) {
    const int r = t - k;
    rank = binom[static_cast<unsigned long long>(c[k] + 1) * ld + r] - 1 - rank;
  }
  return rank;
}

}  // namespace qd

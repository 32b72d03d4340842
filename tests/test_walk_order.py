"""The revolving-door order of the plain walk kernel (csrc/revdoor.hpp),
compiled with the host compiler and checked against the recursive
definition of the order written out here: the t-subsets of {0..p-1}
without p-1 in their own order, then those with p-1, the rest running
backwards through the (t-1)-subsets of {0..p-2}.  Also: consecutive
subsets, and the last and the first, differ by one element out and one
in, and rank inverts unrank."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "..", "paper_2408_10743_amd", "csrc", "revdoor.hpp")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "revdoor.hpp"
int main(int argc, char **argv) {
  const int P = std::atoi(argv[1]), t = std::atoi(argv[2]), ld = t + 1;
  std::vector<unsigned long long> B((P + 1) * ld, 0);
  for (int p = 0; p <= P; ++p)
    for (int r = 0; r <= t; ++r)
      B[p * ld + r] = r == 0 ? 1 : p == 0 ? 0 : B[(p - 1) * ld + r] + B[(p - 1) * ld + r - 1];
  const unsigned long long N = B[P * ld + t];
  for (unsigned long long i = 0; i < N; ++i) {
    int c[64];
    qd::revdoor_unrank(i, t, P, B.data(), ld, c);
    for (int k = 0; k < t; ++k) std::printf("%d ", c[k]);
    std::printf("| %llu\n", qd::revdoor_rank(t, c, B.data(), ld));
  }
  return 0;
}
"""


def revolving_door(p, t):
    """The order by its recursive definition, as sorted tuples."""
    if t == 0:
        return [()]
    if p < t:
        return []
    without = revolving_door(p - 1, t)
    with_last = [s + (p - 1,) for s in reversed(revolving_door(p - 1, t - 1))]
    return without + with_last


@pytest.fixture(scope="module")
def driver():
    d = tempfile.mkdtemp(prefix="qd_revdoor_")
    src = os.path.join(d, "drv.cpp")
    exe = os.path.join(d, "drv")
    with open(src, "w") as f:
        f.write(DRIVER)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", os.path.dirname(HEADER), src, "-o", exe])
    return exe


def run(exe, P, t):
    out = subprocess.check_output([exe, str(P), str(t)], text=True)
    subsets, ranks = [], []
    for line in out.splitlines():
        a, b = line.split("|")
        subsets.append(tuple(sorted(int(x) for x in a.split())))
        ranks.append(int(b))
    return subsets, ranks


@pytest.mark.parametrize("P", [1, 2, 3, 5, 8, 11])
def test_unrank_follows_the_definition(driver, P):
    for t in range(1, P + 1):
        subsets, ranks = run(driver, P, t)
        assert subsets == revolving_door(P, t), (P, t)
        assert ranks == list(range(len(subsets)))


def test_one_out_one_in(driver):
    """Consecutive subsets differ by one element each way, and so do the
    last and the first (the order is cyclic)."""
    for P, t in [(12, 3), (12, 6), (16, 8), (20, 2), (9, 1), (7, 6)]:
        subsets, _ = run(driver, P, t)
        assert len(set(subsets)) == len(subsets)
        for a, b in zip(subsets, subsets[1:] + subsets[:1]):
            assert len(set(a) - set(b)) == 1 and len(set(b) - set(a)) == 1, (a, b)

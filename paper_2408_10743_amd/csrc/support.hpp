// support.hpp -- device data layouts of the support kernels (support.hip):
// table builds and the upload scatter.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qd {

// Saved table (bottoms: combinations ordered by their largest package,
// structure of arrays in blocks of kBlock) or tops table (combinations
// ordered by their smallest package, largest first; 2D words per entry, the
// D x words then the D z words).
struct SavedParams {
  const uint32_t *elems;
  const unsigned long long *prefix;    // (P+1) x R: e_r(c_0..c_{h-1})
  const unsigned long long *suffix;    // (P+1) x R: e_r(c_h..c_{P-1})
  const unsigned char *csize;
  uint32_t *table;
  unsigned long long nent, nent_padded;  // nent_padded: multiple of kBuildGroup
  unsigned long long first;            // first thread of this table in the launch
  int P, R, u;
  int tops;                            // 1: build the tops table
  // Table of the same kind of depth u - 1, complete before this table is built
  // (NULL: unrank every package).  Entry k of depth u is one element of its
  // first package in build order (the largest; for tops the smallest) XOR an
  // entry of depth u - 1, in the same order.
  const uint32_t *src;
  int level;                           // host: launch wave (a build after its source's)
};

// Threads per workgroup of the table builder; a workgroup never spans two
// tables of one launch.
constexpr int kBuildGroup = 256;

// One launch builds the pending tables of one word count D.
struct BuildParams {
  const SavedParams *req;              // sorted by first
  int nreq;
  unsigned int lds;                    // dynamic LDS bytes (0: read counts from memory)
  unsigned long long threads;
  unsigned long long base;             // first thread of this launch (a slice of `threads`)
};

// Threads per launch at most: a dispatch packet counts its grid in 32-bit
// work-items, so larger builds go out in slices of this many threads.
constexpr unsigned long long kMaxLaunchThreads = 1ull << 31;

// One block move of a step's upload: `bytes` (a multiple of 16) from the
// step's device staging buffer at byte offset `src`, or zeros when src is
// kZeroFill, to `dst`.  With src == kEsymTables it instead writes the
// prefix and suffix tables e_r(c_0..c_{h-1}) and e_r(c_h..c_{P-1}),
// (P+1) x R each, saturating at kEsymSat, of the P package sizes found in
// the staging buffer at byte offset `sizes`.  The records of one launch
// never overlap and read only the staging buffer.
struct CopyRec {
  void *dst;
  unsigned long long src;
  unsigned long long bytes;
  unsigned long long sizes;
  int P, R;
};
constexpr unsigned long long kZeroFill = ~0ull;
constexpr unsigned long long kEsymTables = ~0ull - 1;
constexpr unsigned long long kEsymSat = 1ull << 62;
constexpr int kMaxEsymPackages = 256;  // packages per e_r table record; R <= kWave

// Matrix-core form of one saved table (RoundDesc::mtable): chunks of
// kChunk entries, `mks` K-steps each; entries at or past nent read as zero.
struct ExpandParams {
  const uint32_t *table;               // saved table, blocks of kBlock entries
  uint4 *mtable;                       // ceil(nent / kChunk) * mks * 64 uint4
  unsigned long long nent;
  unsigned long long first;            // first thread of this table in the launch
  int D, mks, pack;
};

// One launch expands every table queued for a step.
struct ExpandBatch {
  const ExpandParams *req;             // sorted by first; each starts a workgroup
  int nreq;
  unsigned long long threads;
  unsigned long long base;             // first thread of this launch (a slice of `threads`)
};

// Threads of a table's expansion (one per entry and K-step), rounded up to
// whole workgroups.
__host__ __device__ inline unsigned long long expand_threads(unsigned long long nent, int mks) {
  const unsigned long long t = (nent + kChunk - 1) / kChunk * mks * kChunk;
  return (t + 255) / 256 * 256;
}

__host__ __device__ inline unsigned int build_lds_bytes(int P, int u) { return static_cast<unsigned int>((P + 1) * (u + 1) * 8); }

}  // namespace qd

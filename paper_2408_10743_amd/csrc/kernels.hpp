// kernels.hpp -- device data layouts shared by the HIP kernels and their
// host-side launch code.
#pragma once
#include <cstdint>

namespace qd {

// Words of one element, witness or slot: x words 0..3, z words 4..7 (32-bit
// words of qubits 32w..32w+31; unused words are zero).
constexpr int kElemWords = 8;
// Lanes per wavefront and wavefronts per workgroup.
constexpr int kWave = 64;
constexpr int kWavesPerGroup = 4;
// Saved-table entries per block (structure of arrays inside a block).
constexpr int kBlock = 8;
// Low 32 bits of the state key when no slot is pending.
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;

// One group of a round: top combinations whose smallest package is h,
// paired with the saved-table prefix of combinations below h.
struct DevGroup {
  unsigned long long items;  // top combinations in the group
  unsigned long long len;    // usable saved-table entries
  unsigned long long tile0;  // first tile of the group
  unsigned long long nb;     // blocks of 64 items
  unsigned long long ns;     // segments of the table prefix
  int h;
  int pad;
};

// Per-code device state: key = (U << 32) | pending slot; count = visited
// combinations; wit = codeword of weight U (kElemWords words).
struct DevState {
  unsigned long long key;
  unsigned long long count;
  uint32_t wit[kElemWords];
};

struct RoundParams {
  const uint32_t *elems;               // package i element e: (3i+e)*kElemWords
  const uint32_t *table;               // saved sums, blocks of kBlock entries
  const DevGroup *groups;
  const unsigned long long *suffix;    // (P+1) x R: e_r(c_h..c_{P-1})
  const unsigned char *csize;          // elements per package (1 or 3)
  DevState *state;
  uint32_t *slots;                     // one witness slot per tile of a launch
  unsigned long long tile_lo, tile_hi; // tiles of this launch
  int ngroups, P, R, t, u;
  unsigned int seg;                    // table entries per tile (multiple of kBlock)
  int L_before;                        // lower bound already certified
};

struct SavedParams {
  const uint32_t *elems;
  const unsigned long long *prefix;    // (P+1) x R: e_r(c_0..c_{h-1})
  const unsigned char *csize;
  uint32_t *table;
  unsigned long long nent, nent_padded;
  int P, R, u;
};

}  // namespace qd

// kernels.hpp -- device data layouts of the enumeration kernels (round.hip,
// walk.hip), shared with their host-side launch code.
#pragma once
#include <hip/hip_runtime.h>

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
// Visited-combination counters are spread over separate 128-byte lines so
// the waves of a launch do not all update one address.
constexpr int kCounterStride = 16;  // unsigned long longs per line
// Deepest round the plain walk kernel (walk.hip) supports: packages per
// combination, each in a VGPR slot of its lane.
constexpr int kWalkMaxT = 8;

// One group of a round: top combinations whose smallest package is h,
// paired with the saved-table prefix of combinations below h.  Groups are
// sorted by len, longest first; cum = items of the groups before it.
struct DevGroup {
  unsigned long long items;  // top combinations in the group
  unsigned long long len;    // usable saved-table entries
  unsigned long long cum;    // items of the longer groups
  unsigned long long top0;   // first entry of the group in the tops table
  long long h;
  // Entries of the tops table one package shallower over packages h+1..:
  // with RoundDesc::tops_down, item i of the group is element i / f of
  // package h XOR that table's entry i % f.
  unsigned long long f;
};

// A run of table segments [s_begin, s_begin + nseg) that the same `e`
// longest groups reach; each segment is split into `tps` tiles of 64 tops
// taken from those groups' items in order.
struct DevRun {
  unsigned long long tile0;   // first tile of the run
  unsigned long long s_begin;
  unsigned long long items;   // items of the e groups
  unsigned long long tps;     // tiles per segment
  long long e;
};

// Per-code device state: key = (U << 32) | pending slot; count = visited
// combinations; words = 32-bit words whose weight was evaluated, summed over
// the visited combinations; wit = codeword of weight U (kElemWords words).
struct DevState {
  unsigned long long key;
  unsigned long long count;
  unsigned long long words;
  uint32_t wit[kElemWords];
};

// Visited counters per code (separate 128-byte lines); word 0 of a line
// counts combinations, word 1 the words evaluated for them.
constexpr int kCountersPerCode = 256;

// Part u of a walk round: the package sets with u one-row packages, ranked
// as (one-row subset, two-row subset), each in revolving-door order.
struct WalkPart {
  unsigned long long tile0;            // first wave of the part within the round
  unsigned long long subsets;          // C(P1, u) C(P2, t - u)
  unsigned long long c2;               // C(P2, t - u): two-row subsets
  int u;
  int pad;
};

// One piece of one (code, t, Gamma_j) round inside a launch.  A launch
// covers several pieces (several codes); pieces start at multiples of
// kWavesPerGroup tiles so a workgroup never spans two of them.
struct RoundDesc {
  const uint32_t *elems;               // package i element e: (3i+e)*kElemWords
  const uint32_t *table;               // saved sums, blocks of kBlock entries
  const uint32_t *tops;                // top codewords, 2D words each: x, then z (NULL: unrank)
  int tops_down;                       // 1: tops holds tops of t - u - 1 packages (DevGroup::f)
  int pad_tops;
  const DevGroup *groups;              // sorted by len, longest first
  const DevRun *runs;
  const unsigned long long *suffix;    // (P+1) x R: e_r(c_h..c_{P-1})
  const unsigned char *csize;          // elements per package (1 or 3)
  DevState *state;
  unsigned long long *counters;        // kCountersPerCode x kCounterStride
  const uint32_t *logicals;            // Modified BZ: logical operators, kElemWords each
  int nlogicals;                       // 0: every codeword may update U
  // The matrix's qubits are stored permuted: position inv[q] holds qubit q
  // (NULL: not permuted).  Witnesses are written back in qubit order.
  const unsigned char *inv;
  int n;
  // Partial weights: the weight of words 0..w-1 plus credit[w-1] bounds a
  // codeword's weight from below.  A tile that starts with U <= cap[w-1]
  // (smallest such w) evaluates w words first and the rest only for blocks
  // where some bound is below U; cap -1 disables w.
  int cap[3];
  int credit[3];
  unsigned long long tile_begin;       // first launch tile of the piece
  unsigned long long ntiles;           // tiles of the piece
  unsigned long long tile_lo;          // round tile of the piece's first tile
  unsigned long long slot0;            // first witness slot of the piece
  int ngroups, nruns, P, R, t, u;
  unsigned int seg;                    // table entries per tile (multiple of kBlock)
  int L_before;                        // lower bound already certified
  int stage;                           // 1: copy the groups to LDS; 2: also suffix
                                       //    columns and elements (unranking path)
  int commit;                          // 1 for the first piece of its code in the launch
  // Matrix-core form of the saved table (NULL: the vector-ALU loops only).
  // Every codeword half-word is read as three groups of 32 signs per word,
  // x, z and x ^ z (bit 0 -> +1, bit 1 -> -1): two codewords differ in a
  // group's popcount(a ^ b) positions, so the sign dot product of a group
  // is 32 - 2 popcount(a ^ b), and over x, z and x ^ z each qubit where
  // the sum is not identity contributes exactly 2 to the popcounts.  With
  // G groups, dot = 32 G - 4 wt.  K-step s (128 signs, one MFMA) holds the
  // groups x_s, z_s, x_s ^ z_s and a fourth group: for s = 0 the bias group
  // (32 values 2.0: against the tops' bias codes it adds 32 G, so the
  // products sum to 4 wt with no accumulator input); with mpack, for
  // s = D - 2 the last word packed as x | z << 10 | (x ^ z) << 20 (at most
  // 10 qubits in it); else empty.  mtable: chunk c of 16 entries, K-step s:
  // 64 lanes x 16 bytes at (c * mks + s) * 64 + lane, lane = 16 g + r for
  // group g of entry 16 c + r, dword i holding the e2m1 codes of bits
  // 8i..8i+7 (nibble j: bit 8i + j).  mks: K-steps stored per chunk (1: the
  // first word only, for partial weights).
  const uint4 *mtable;
  int mks, mpack;
  // Census (round kernel, qd_round_census): codewords of weight below
  // `below` are counted in census[0] and their weights summed in census[1]
  // (NULL: not taken).  Partial-weight tiles then complete every block that
  // may hold such a codeword, so both figures are exact.
  unsigned long long *census;
  int below;
  int pad_census;
  // Plain walk kernel (walk.hip) only.
  const unsigned long long *binom;     // C(p, r) at p * (t + 1) + r, p <= P, r <= t
  unsigned long long *wsum;            // sum of the walked codewords' weights (NULL: not taken)
  const unsigned short *pmap;          // the two-row packages (p2 of them), then the one-row ones
  const WalkPart *parts;               // the round's parts, by first wave
  unsigned long long per_lane;         // package sets per lane
  int nparts, p2;
};

struct LaunchParams {
  const RoundDesc *desc;               // sorted by tile_begin
  int ndesc;
  unsigned int lds;                    // dynamic LDS bytes of the launch
  unsigned long long tiles;            // multiple of kWavesPerGroup
  uint32_t *slots;                     // one witness slot per launch tile
};

// LDS bytes a round kernel launch needs when it stages its tables.
inline unsigned int round_lds_bytes(int P, int t, int u, int ngroups, int stage) {
  if (stage == 0) return 0u;
  unsigned int b = static_cast<unsigned int>(ngroups * sizeof(DevGroup));
  if (stage == 2) b += static_cast<unsigned int>((P + 1) * (t - u) * 8 + P * 3 * kElemWords * 4);
  return b;
}

// LDS bytes a walk kernel launch needs to stage binomials and elements.
inline unsigned int walk_lds_bytes(int P, int t) {
  return static_cast<unsigned int>((P + 1) * (t + 1) * 8 + P * 3 * kElemWords * 4);
}

// Matrix-core layout of table entries and tops (RoundDesc::mtable).
constexpr int kChunk = 16;             // table entries per chunk (MFMA rows)
// Chunks allocated past an expanded table's last (never written): the
// shared-chunk stream of the round kernel reads whole groups of chunks.
constexpr int kMtablePadChunks = 4;
constexpr int kMaxPackedQubits = 10;   // last word packed into a spare group

// e2m1 codes of 8 sign bits: nibble j is -1.0 (0xA) for bit j set, +1.0
// (0x2) otherwise.  Spreads bit j to bit 4j, then to the nibble's sign.
__device__ __forceinline__ uint32_t sign_nibbles(uint32_t b) {
  uint32_t x = b & 0xFFu;
  x = (x | (x << 12)) & 0x000F000Fu;
  x = (x | (x << 6)) & 0x03030303u;
  x = (x | (x << 3)) & 0x11111111u;
  return (x << 3) | 0x22222222u;
}

// Bias group of K-step 0 (the fourth group; never the packed one, which
// needs D >= 3 and sits in K-step D - 2): table entries hold e2m1 2.0 in
// all 32 places, and a top's B operand holds, in dwords 0-1 and 2-3, the
// codes of two values v_lo, v_hi with v_lo + v_hi = G, so the group adds
// 8 x 2 x (2 v_lo + 2 v_hi) = 32 G.  G is 3 (first word alone) or
// 3 KS + (KS < D): 6, 7, 9, 10 or 12.
constexpr uint32_t kBiasEntry = 0x44444444u;
__host__ __device__ constexpr uint32_t bias_code(int G, bool hi) {
  // e2m1 codes: 0x3 = 1.5, 0x5 = 3.0, 0x6 = 4.0, 0x7 = 6.0
  return (G == 3 ? 0x3u : G == 6 ? 0x5u : G == 7 ? (hi ? 0x6u : 0x5u) : G == 9 ? (hi ? 0x7u : 0x5u)
          : G == 10 ? (hi ? 0x7u : 0x6u) : G == 12 ? 0x7u : 0x0u) * 0x11111111u;
}
// Twice the e2m1 value of code c (0..7, sign clear): 0, 1, 2, 3, 4, 6, 8, 12.
constexpr int e2m1_twice(uint32_t c) { return c < 2 ? int(c) : int((2u + (c & 1u)) << ((c >> 1) - 1u)); }
// The bias group's products: 8 places per dword x entry 2.0 x the top's value.
constexpr int bias_sum(int G) {
  return 8 * 2 * (2 * e2m1_twice(bias_code(G, false) & 0xFu) + 2 * e2m1_twice(bias_code(G, true) & 0xFu)) / 2;
}
static_assert(e2m1_twice(0x2) == 2 && e2m1_twice(0x3) == 3 && e2m1_twice(0x5) == 6 && e2m1_twice(0x7) == 12 &&
                  kBiasEntry == 0x44444444u && e2m1_twice(0x4) == 4,
              "e2m1 codes");
static_assert(bias_sum(3) == 32 * 3 && bias_sum(6) == 32 * 6 && bias_sum(7) == 32 * 7 && bias_sum(9) == 32 * 9 &&
                  bias_sum(10) == 32 * 10 && bias_sum(12) == 32 * 12,
              "the bias group adds 32 G for every G a kernel uses");

// Group g of K-step s of a codeword: x_s, z_s, x_s ^ z_s, or (g = 3) the
// packed last word (xl, zl) when `packed` (else an empty group).
__device__ __forceinline__ uint32_t group_word(int g, bool packed, uint32_t x, uint32_t z, uint32_t xl,
                                               uint32_t zl) {
  return g == 0 ? x : g == 1 ? z : g == 2 ? x ^ z : packed ? xl | (zl << 10) | ((xl ^ zl) << 20) : 0u;
}

// XOR of element e of package pkg into a codeword of D words per half.
template <int D>
__device__ __forceinline__ void xor_elem(const uint32_t *__restrict__ elems, int pkg, int e,
                                         uint32_t (&ax)[D], uint32_t (&az)[D]) {
  const uint32_t *p = elems + (size_t(3) * pkg + e) * kElemWords;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ax[d] ^= p[d];
    az[d] ^= p[4 + d];
  }
}

}  // namespace qd

// round.hip -- the enumeration kernel of libqdist (gfx950).
//
// Enumeration scheme for one round (t packages of one generator matrix):
// a combination is split into its u lowest packages ("bottom") and the
// t - u others ("top").  All bottom combinations are precomputed once per
// matrix and depth u into a saved table ordered by their largest package,
// so the bottoms that fit below a top whose smallest package is h are a
// prefix of the table.  Each lane of a wavefront holds one top codeword in
// VGPRs; the wavefront streams a segment of the table through SGPRs (all
// lanes read the same entry), so each codeword costs one XOR per x word,
// one fused XOR-OR (v_bitop3) per z word, one v_bcnt per word and one MIN.
//
// Partial weights.  The host stores each matrix with the qubits that carry
// none of its pivots first.  Every package of a combination has a nonzero
// symbol at its own pivot qubit, so the weight of the first w words plus
// the chosen packages pivoted beyond them (a per-round credit) bounds the
// weight from below.  Once U is small enough, a tile evaluates w words per
// codeword and the remaining words only for the blocks where some bound is
// below U: the other codewords cannot improve U.
#include <hip/hip_runtime.h>

#include "kernels.hpp"
#include "wave.hpp"

namespace qd {

__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

__device__ __forceinline__ uint32_t min3(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t r;
  asm("v_min3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

__device__ __forceinline__ unsigned long long uniform64(unsigned long long v) {
  uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(v));
  uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(v >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_min(uint32_t v) { return wave_min_u32(v); }

// Weight of (lane codeword) ^ (table entry k); k is wavefront-uniform.
template <int D>
__device__ __forceinline__ uint32_t weight_at(const uint32_t *__restrict__ table, unsigned long long k,
                                              const uint32_t (&ax)[D], const uint32_t (&az)[D]) {
  const uint32_t *b = table + (k / kBlock) * (2 * D * kBlock) + (k % kBlock);
  uint32_t acc = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    uint32_t o = (ax[d] ^ b[d * kBlock]) | (az[d] ^ b[(D + d) * kBlock]);
    acc = d == 0 ? __builtin_popcount(o) : bcnt_acc(o, acc);
  }
  return acc;
}

// Census of one codeword weight: counted (and summed) when below `below`.
struct Census {
  uint32_t below = 0, cnt = 0, sum = 0;
  __device__ __forceinline__ void add(uint32_t w) {
    const bool in = w < below;
    cnt += in ? 1u : 0u;
    sum += in ? w : 0u;
  }
};

// Minimum over one block of kBlock table entries (SoA: word-major).  With
// kCensus the block's weights also enter the census.
template <int D, bool kCensus>
__device__ __forceinline__ uint32_t block_min(const uint32_t (&ax)[D], const uint32_t (&az)[D],
                                              const uint32_t *__restrict__ blk, uint32_t best, Census &cs) {
  uint32_t v[2 * D][kBlock];
#pragma unroll
  for (int j = 0; j < 2 * D; ++j)
#pragma unroll
    for (int e = 0; e < kBlock; ++e) v[j][e] = blk[j * kBlock + e];
  uint32_t w[kBlock];
#pragma unroll
  for (int e = 0; e < kBlock; ++e) {
    uint32_t acc = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      uint32_t o = (ax[d] ^ v[d][e]) | (az[d] ^ v[D + d][e]);
      acc = d == 0 ? __builtin_popcount(o) : bcnt_acc(o, acc);
    }
    w[e] = acc;
  }
  if constexpr (kCensus) {
#pragma unroll
    for (int e = 0; e < kBlock; ++e) cs.add(w[e]);
  }
  // One three-input min per pair of codewords.
#pragma unroll
  for (int e = 0; e < kBlock; e += 2) best = min3(best, w[e], w[e + 1]);
  return best;
}

// NB consecutive blocks with partial weights: words 0..W-1 first; if some
// lane's bound (partial weight + credit) falls below U (thr = U - credit),
// the blocks' remaining words are added and their full weights enter
// `best`.  `rec` counts the blocks evaluated in full.  With kCensus the
// completed blocks' weights enter the census (a block that is not completed
// holds no codeword of weight below thr + credit).
template <int D, int W, int NB, bool kCensus>
__device__ __forceinline__ uint32_t blocks_min_partial(const uint32_t (&ax)[D], const uint32_t (&az)[D],
                                                       const uint32_t *__restrict__ blk, uint32_t best,
                                                       uint32_t thr, uint32_t &rec, Census &cs) {
  constexpr int N = NB * kBlock;
  uint32_t w[N];
  {
    uint32_t v[2 * W][N];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int j = 0; j < W; ++j)
#pragma unroll
        for (int e = 0; e < kBlock; ++e) {
          v[j][b * kBlock + e] = blk[b * 2 * D * kBlock + j * kBlock + e];
          v[W + j][b * kBlock + e] = blk[b * 2 * D * kBlock + (D + j) * kBlock + e];
        }
#pragma unroll
    for (int e = 0; e < N; ++e) {
      uint32_t acc = 0;
#pragma unroll
      for (int d = 0; d < W; ++d) {
        uint32_t o = (ax[d] ^ v[d][e]) | (az[d] ^ v[W + d][e]);
        acc = d == 0 ? __builtin_popcount(o) : bcnt_acc(o, acc);
      }
      w[e] = acc;
    }
  }
  uint32_t pm = min3(w[0], w[1], w[2]);
#pragma unroll
  for (int e = 3; e + 1 < N; e += 2) pm = min3(pm, w[e], w[e + 1]);
  pm = min(pm, w[N - 1]);
  if (__ballot(pm < thr)) {  // rare once U is small: the blocks are evaluated in full
    uint32_t v[2 * (D - W)][N];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int j = 0; j < D - W; ++j)
#pragma unroll
        for (int e = 0; e < kBlock; ++e) {
          v[j][b * kBlock + e] = blk[b * 2 * D * kBlock + (W + j) * kBlock + e];
          v[D - W + j][b * kBlock + e] = blk[b * 2 * D * kBlock + (D + W + j) * kBlock + e];
        }
#pragma unroll
    for (int e = 0; e < N; ++e) {
#pragma unroll
      for (int d = 0; d < D - W; ++d) {
        uint32_t o = (ax[W + d] ^ v[d][e]) | (az[W + d] ^ v[D - W + d][e]);
        w[e] = bcnt_acc(o, w[e]);
      }
    }
    if constexpr (kCensus) {
#pragma unroll
      for (int e = 0; e < N; ++e) cs.add(w[e]);
    }
#pragma unroll
    for (int e = 0; e < N; e += 2) best = min3(best, w[e], w[e + 1]);
    rec += NB;
  }
  return best;
}

// Kernel variants by the entry-major blocks they use (qd_round_kernel).
constexpr int kEmEveryWord = 1, kEmPartial = 2;

// Entry-major blocks (every word evaluated): a block is kWave * K consecutive
// table entries, lane l holding entries e0 + l + 64 i (i < K) in VGPRs, and
// the wave's tops broadcast one at a time from the lane holding them
// (ds_bpermute).  Every operand of the XOR, the XOR-OR and the popcount is
// then a VGPR, which lets the VALU pair the bitwise operations; the
// streaming loop (block_min) reads its entries through SGPRs, and an
// operation with an SGPR operand never pairs.
template <int D>
struct EmK {
  static constexpr int K = D == 1 ? 16 : D <= 3 ? 8 : 4;  // entries per lane (VGPRs: 2D K)
};

__device__ __forceinline__ uint32_t bcast(uint32_t v, int src_lane) {
  return static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(src_lane << 2, static_cast<int>(v)));
}

// One entry-major block: entries [e0, e0 + 64 K) against the tops of lanes
// 0..ntop-1; returns the lane's minimum over its entries and those tops.
template <int D, bool kCensus>
__device__ __forceinline__ uint32_t em_block(const uint32_t *__restrict__ table, unsigned long long e0, uint32_t lane,
                                             const uint32_t (&ax)[D], const uint32_t (&az)[D], int ntop,
                                             uint32_t best, Census &cs) {
  constexpr int K = EmK<D>::K;
  uint32_t ex[K][D], ez[K][D];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const unsigned long long k = e0 + static_cast<unsigned long long>(i) * kWave + lane;
    const uint32_t *b = table + (k / kBlock) * (2 * D * kBlock) + (k % kBlock);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      ex[i][d] = b[d * kBlock];
      ez[i][d] = b[(D + d) * kBlock];
    }
  }
  uint32_t tx[D], tz[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    tx[d] = bcast(ax[d], 0);
    tz[d] = bcast(az[d], 0);
  }
  for (int j = 0; j < ntop; ++j) {
    uint32_t nx[D], nz[D];  // the next top, fetched while this one is evaluated
    const int jn = j + 1 < ntop ? j + 1 : j;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      nx[d] = bcast(ax[d], jn);
      nz[d] = bcast(az[d], jn);
    }
    uint32_t w[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      uint32_t acc = 0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const uint32_t o = (ex[i][d] ^ tx[d]) | (ez[i][d] ^ tz[d]);
        acc = d == 0 ? __builtin_popcount(o) : bcnt_acc(o, acc);
      }
      w[i] = acc;
    }
    if constexpr (kCensus) {
#pragma unroll
      for (int i = 0; i < K; ++i) cs.add(w[i]);
    }
#pragma unroll
    for (int i = 0; i < K; i += 2) best = min3(best, w[i], w[i + 1]);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      tx[d] = nx[d];
      tz[d] = nz[d];
    }
  }
  return best;
}

// Entry-major blocks with partial weights on the first word: lane l holds
// word 0 (x and z) of entries e0 + l + 64 i, i < kEmPartialK.  For each top
// the K first-word weights are formed from VGPR operands; when some lane's
// bound falls below U (thr = U - credit) the 64 K codewords of that top are
// completed, their remaining words read from the table, and their full
// weights enter `best` and the census.  `done` counts the completed tops.
constexpr int kEmPartialK = 8;

template <int D, bool kCensus>
__device__ __forceinline__ uint32_t em_block_partial(const uint32_t *__restrict__ table, unsigned long long e0,
                                                     uint32_t lane, const uint32_t (&ax)[D], const uint32_t (&az)[D],
                                                     int ntop, uint32_t best, uint32_t thr, Census &cs,
                                                     uint32_t &done) {
  constexpr int K = kEmPartialK;
  uint32_t ex[K], ez[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const unsigned long long k = e0 + static_cast<unsigned long long>(i) * kWave + lane;
    const uint32_t *b = table + (k / kBlock) * (2 * D * kBlock) + (k % kBlock);
    ex[i] = b[0];
    ez[i] = b[D * kBlock];
  }
  uint32_t tx = bcast(ax[0], 0), tz = bcast(az[0], 0);
  for (int j = 0; j < ntop; ++j) {
    const int jn = j + 1 < ntop ? j + 1 : j;
    const uint32_t nx = bcast(ax[0], jn), nz = bcast(az[0], jn);  // the next top's first word
    uint32_t w[K];
#pragma unroll
    for (int i = 0; i < K; ++i) w[i] = __builtin_popcount((ex[i] ^ tx) | (ez[i] ^ tz));
    uint32_t pm = min3(w[0], w[1], w[2]);
#pragma unroll
    for (int i = 3; i + 1 < K; i += 2) pm = min3(pm, w[i], w[i + 1]);
    pm = min(pm, w[K - 1]);
    if (__ballot(pm < thr)) {  // rare once U is small: this top's codewords in full
      uint32_t rx[D], rz[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        rx[d] = bcast(ax[d], j);
        rz[d] = bcast(az[d], j);
      }
      // One entry at a time, re-read from the table: few registers for a
      // rare path.
#pragma unroll 1
      for (int i = 0; i < K; ++i) {
        const unsigned long long k = e0 + static_cast<unsigned long long>(i) * kWave + lane;
        const uint32_t *b = table + (k / kBlock) * (2 * D * kBlock) + (k % kBlock);
        uint32_t full = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) full = bcnt_acc((b[d * kBlock] ^ rx[d]) | (b[(D + d) * kBlock] ^ rz[d]), full);
        if constexpr (kCensus) cs.add(full);
        best = min(best, full);
      }
      ++done;
    }
    tx = nx;
    tz = nz;
  }
  return best;
}

// The full blocks of a tile with partial weights, kPartialBlocks blocks per
// wait for their scalar loads.
constexpr int kPartialBlocks = 2;
template <int D, int W, bool kCensus>
__device__ __forceinline__ uint32_t partial_blocks(const uint32_t (&ax)[D], const uint32_t (&az)[D],
                                                   const uint32_t *__restrict__ blk, uint32_t nfull,
                                                   uint32_t best, uint32_t thr, uint32_t &rec, Census &cs) {
  uint32_t i = 0;
  for (; i + kPartialBlocks <= nfull; i += kPartialBlocks, blk += kPartialBlocks * 2 * D * kBlock)
    best = blocks_min_partial<D, W, kPartialBlocks, kCensus>(ax, az, blk, best, thr, rec, cs);
  for (; i < nfull; ++i, blk += 2 * D * kBlock)
    best = blocks_min_partial<D, W, 1, kCensus>(ax, az, blk, best, thr, rec, cs);
  return best;
}

// -- matrix cores -------------------------------------------------------------
// A chunk of kChunk table entries against the wave's 64 tops is four 16x16
// output blocks; K-step s of each is one fp4 MFMA over 128 signs (layout in
// kernels.hpp).  Entries are the A rows (lane 16 g + r: row r, group g),
// tops the B columns (lane 16 g + r: top 16 nb + r of block nb), and lane
// 16 q + r receives rows 4q..4q+3 of column r.  The tops' signs are
// negated, so the sign groups sum to -dot = 4 wt - 32 G, and the bias group
// of K-step 0 adds 32 G: the accumulator (zero input) ends at 4 wt, an
// exact non-negative float whose bits order like the weights.
// Every word on the matrix cores: kMfmaEveryWord picks the K-step layout per
// piece; kMfmaEveryPacked / kMfmaEveryPlain serve launches whose pieces all
// have the packed (K-steps D - 1) / plain (K-steps D) layout, with the
// registers of that layout only.
constexpr int kMfmaEveryWord = 3, kMfmaPartial = 4, kMfmaEveryPacked = 5, kMfmaEveryPlain = 6;
constexpr bool mfma_every_mode(int m) { return m == kMfmaEveryWord || m == kMfmaEveryPacked || m == kMfmaEveryPlain; }
typedef int v8i_t __attribute__((ext_vector_type(8)));
typedef float v4f_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f_t mfma_fp4(v8i_t a, v8i_t b, v4f_t c) {
  // e2m1 operands (format 4) on both sides, unit scales (E8M0 127).
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 4, 4, 0, 127, 0, 127);
}

__device__ __forceinline__ v8i_t mfma_operand(uint4 a) {
  return (v8i_t){static_cast<int>(a.x), static_cast<int>(a.y), static_cast<int>(a.z), static_cast<int>(a.w), 0, 0, 0,
                 0};
}

// B operands of K-steps 0..KU-1 from the wave's tops (lane l holds top l)
// for G sign groups: the tops' signs negated, so a column's products sum
// to 4 wt - 32 G, and the bias group of K-step 0 adds 32 G back (every top,
// so a top at or past ntop, whose other groups are zero, reads 8 G).  Each
// byte of a group word becomes its dword of negated e2m1 signs through
// `neg_lut` (256 entries in LDS, filled by the workgroup).
template <int D, int KU, int G>
__device__ __forceinline__ void mfma_tops(const uint32_t (&ax)[D], const uint32_t (&az)[D], uint32_t lane, int ntop,
                                          bool pack, const uint32_t *neg_lut, v8i_t (&B)[KU][4]) {
  const int g = static_cast<int>(lane >> 4);
  // Group g of a word from its x and z halves without branches: x, z or
  // x ^ z (g = 3: empty unless packed).
  const uint32_t mx = g == 0 || g == 2 ? ~0u : 0u, mz = g == 1 || g == 2 ? ~0u : 0u;
  const uint32_t lo = g == 3 ? bias_code(G, false) : 0u, hi = g == 3 ? bias_code(G, true) : 0u;
#pragma unroll
  for (int s = 0; s < KU; ++s)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int src = nb * kChunk + static_cast<int>(lane & 15);
      const bool packed = pack && s == D - 2;
      uint32_t w = (bcast(ax[s], src) & mx) ^ (bcast(az[s], src) & mz);
      if (packed) {
        const uint32_t xl = bcast(ax[D - 1], src), zl = bcast(az[D - 1], src);
        w = g == 3 ? xl | (zl << 10) | ((xl ^ zl) << 20) : w;
      }
      const bool on = src < ntop && (g < 3 || packed);
      // Every index is below 256: read all four, then choose.
      const uint32_t l0 = neg_lut[w & 0xFFu], l1 = neg_lut[(w >> 8) & 0xFFu], l2 = neg_lut[(w >> 16) & 0xFFu],
                     l3 = neg_lut[w >> 24];
      const uint32_t b0 = s == 0 ? lo : 0u, b1 = s == 0 ? hi : 0u;  // the bias group, or an empty one
      B[s][nb] = (v8i_t){static_cast<int>(on ? l0 : b0), static_cast<int>(on ? l1 : b0),
                         static_cast<int>(on ? l2 : b1), static_cast<int>(on ? l3 : b1), 0, 0, 0, 0};
    }
}

// Fills the workgroup's negated-sign table (a barrier must follow).
__device__ __forceinline__ void fill_neg_lut(uint32_t *neg_lut) {
  static_assert(kWave * kWavesPerGroup == 256, "one entry per thread");
  neg_lut[threadIdx.x] = sign_nibbles(threadIdx.x) ^ 0x88888888u;  // sign bit of every nibble flipped
}

// One chunk, every word, from its A operands: the four output blocks
// (4 wt as float bits of the lane's column of block nb, four rows each).
template <int KS>
__device__ __forceinline__ void mfma_every_chunk(const v8i_t (&A)[KS], const v8i_t (&B)[KS][4], v4f_t (&acc)[4]) {
  const v4f_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma_fp4(A[0], B[0][nb], zero);
#pragma unroll
  for (int s = 1; s < KS; ++s)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma_fp4(A[s], B[s][nb], acc[nb]);
}

// bd[nb] keeps the least 4 wt (as float bits) of the lane's column of block nb.
__device__ __forceinline__ void min_blocks(const v4f_t (&acc)[4], uint32_t (&bd)[4]) {
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    bd[nb] = min(min(bd[nb], __float_as_uint(acc[nb][0])), __float_as_uint(acc[nb][1]));
    bd[nb] = min(min(bd[nb], __float_as_uint(acc[nb][2])), __float_as_uint(acc[nb][3]));
  }
}

// One chunk on K-step 0: the least 4 w0 over the chunk's 16 x 64 outputs.
__device__ __forceinline__ uint32_t mfma_first_chunk(v8i_t A, const v8i_t (&B)[1][4]) {
  const v4f_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
  v4f_t acc[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) acc[nb] = mfma_fp4(A, B[0][nb], zero);
  uint32_t pm = 0xFFFFFFFFu;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    pm = min(min(pm, __float_as_uint(acc[nb][0])), __float_as_uint(acc[nb][1]));
    pm = min(min(pm, __float_as_uint(acc[nb][2])), __float_as_uint(acc[nb][3]));
  }
  return pm;
}

// Chunks shared by the four waves of a workgroup (same table segment):
// they stream through LDS in groups of kCoopChunks, double-buffered, each
// thread moving 16 bytes (wave u: chunk u of the group, K-step 0), so a
// chunk is read from memory once for the workgroup's 256 tops instead of
// once per wave.  Group g + 1 is loaded while group g is evaluated; one
// barrier per group.  The last group may reach past the shared chunks,
// at most kCoopChunks - 1 chunks past the table's last: that read stays
// in the expanded table's padding and its values are never used.
constexpr int kCoopChunks = 4;  // kCoopChunks * kWave = threads of a workgroup
static_assert(kCoopChunks * kWave == kWave * kWavesPerGroup && kCoopChunks <= kMtablePadChunks, "coop groups");

struct CoopStream {
  static constexpr int kPer = kCoopChunks * kWave;  // uint4 per buffer
  const uint4 *src;
  size_t step;
  uint4 r;
  __device__ __forceinline__ void start(const uint4 *__restrict__ mtab, int mks, uint32_t c) {
    step = static_cast<size_t>(kCoopChunks) * mks * kWave;
    src = mtab + (static_cast<size_t>(c) + threadIdx.x / kWave) * mks * kWave + threadIdx.x % kWave;
    r = *src;
  }
  __device__ __forceinline__ void next() {
    src += step;
    r = *src;
  }
  __device__ __forceinline__ void store(uint4 *buf) const { buf[threadIdx.x] = r; }
};

// Every word of chunks [ca, cz) against the wave's tops; the least weight
// over the lane's share of every valid top.  (Shared chunks do not pay
// here: eight MFMAs per chunk hide a wave's own loads.)
constexpr int kMfmaUnroll = 2;  // chunks per group of loads (a wave alone)
template <int D, int KS>
__device__ uint32_t mfma_every(const uint4 *__restrict__ mtab, uint32_t ca, uint32_t cz, uint32_t lane,
                               const uint32_t (&ax)[D], const uint32_t (&az)[D], int ntop, bool pack,
                               const uint32_t *neg_lut) {
  constexpr int G = 3 * KS + (KS < D ? 1 : 0);  // sign groups (packed last word: one)
  v8i_t B[KS][4];
  mfma_tops<D, KS, G>(ax, az, lane, ntop, pack, neg_lut, B);
  uint32_t bd[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
  if constexpr (KS <= 2) {
    // Software pipeline over pairs of chunks: a chunk's MFMAs are issued
    // before the minimum over the previous chunk's outputs, and the operands
    // of the next pair are loaded meanwhile (up to two chunks past cz: in the
    // table's padding, never used).  Y starts as all-ones bits, which leave
    // the minimum unchanged.
    static_assert(kMtablePadChunks >= 2, "prefetch past the last chunk");
    const uint4 *mb = mtab + static_cast<size_t>(ca) * KS * kWave + lane;
    constexpr size_t kStep = static_cast<size_t>(KS) * kWave;
    uint4 a0[KS], a1[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      a0[s] = mb[s * kWave];
      a1[s] = mb[kStep + s * kWave];
    }
    const float ones = __uint_as_float(0xFFFFFFFFu);
    v4f_t X[4], Y[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) Y[nb] = (v4f_t){ones, ones, ones, ones};
    uint32_t c = ca;
    for (; c + 2 <= cz; c += 2) {
      v8i_t A[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) A[s] = mfma_operand(a0[s]);
      mfma_every_chunk<KS>(A, B, X);  // chunk c
      mb += 2 * kStep;
#pragma unroll
      for (int s = 0; s < KS; ++s) a0[s] = mb[s * kWave];
      min_blocks(Y, bd);  // chunk c - 1
#pragma unroll
      for (int s = 0; s < KS; ++s) A[s] = mfma_operand(a1[s]);
      mfma_every_chunk<KS>(A, B, Y);  // chunk c + 1
#pragma unroll
      for (int s = 0; s < KS; ++s) a1[s] = mb[kStep + s * kWave];
      min_blocks(X, bd);
    }
    min_blocks(Y, bd);
    if (c < cz) {  // an odd last chunk, its operands in a0
      v8i_t A[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) A[s] = mfma_operand(a0[s]);
      mfma_every_chunk<KS>(A, B, X);
      min_blocks(X, bd);
    }
  } else {
    // Three or four K-steps: the pipeline's second set of outputs would cost
    // a wave per SIMD (over 128 VGPRs); chunks in pairs, loads first.
    uint32_t c = ca;
    const uint4 *mb = mtab + static_cast<size_t>(c) * KS * kWave + lane;
    for (; c + 2 <= cz; c += 2, mb += 2 * KS * kWave) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        v8i_t A[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) A[s] = mfma_operand(mb[(u * KS + s) * kWave]);
        v4f_t acc[4];
        mfma_every_chunk<KS>(A, B, acc);
        min_blocks(acc, bd);
      }
    }
    if (c < cz) {
      v8i_t A[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) A[s] = mfma_operand(mb[s * kWave]);
      v4f_t acc[4];
      mfma_every_chunk<KS>(A, B, acc);
      min_blocks(acc, bd);
    }
  }
  uint32_t best = 0xFFFFFFFFu;
#pragma unroll
  for (int nb = 0; nb < 4; ++nb)
    if (nb * kChunk + static_cast<int>(lane & 15) < ntop && bd[nb] != 0xFFFFFFFFu)
      best = min(best, static_cast<uint32_t>(__uint_as_float(bd[nb])) >> 2);
  return best;
}

// Partial weights on the first word, chunks [ca, cz) ([ca, cs) shared with
// the workgroup, sbuf: 2 x kCoopChunks x 64 uint4): K-step 0 alone gives
// 4 w0 (bias 96: the three groups of word 0); a chunk where some lane sees
// w0 below thr is completed on the vector ALU (the lane's own top against
// the chunk's two blocks, every word) and counted in `done`.
template <int D, bool kCensus>
__device__ __forceinline__ uint32_t complete_chunks(const uint32_t *__restrict__ table, uint32_t c, int nu,
                                                    const uint32_t *pm, uint32_t T, const uint32_t (&ax)[D],
                                                    const uint32_t (&az)[D], uint32_t best, uint32_t &done,
                                                    Census &cs) {
#pragma unroll 1
  for (int u = 0; u < nu; ++u) {
    if (!__ballot(pm[u] < T)) continue;
    const uint32_t *blk = table + static_cast<size_t>(c + u) * (kChunk / kBlock) * (2 * D * kBlock);
    best = block_min<D, kCensus>(ax, az, blk, best, cs);
    best = block_min<D, kCensus>(ax, az, blk + 2 * D * kBlock, best, cs);
    ++done;
  }
  return best;
}

// Chunks [cz, ct) past the full ones hold the rest of the lanes' entries
// (rel = entries of the tile before chunk cz; a lane's top reaches `span`
// entries, inactive lanes none): their outputs are masked per top and row,
// and a flagged chunk is completed entry by entry within each lane's span.
// tail_skip: entries of the lane decided by the first word alone.
template <int D, bool kCensus>
__device__ uint32_t mfma_partial(const uint32_t *__restrict__ table, const uint4 *__restrict__ mtab, int mks,
                                 uint32_t ca, uint32_t cs_end, uint32_t cz, uint32_t ct, uint32_t rel,
                                 unsigned long long k0, uint32_t span, uint32_t send, bool coop, uint4 *sbuf,
                                 uint32_t lane, const uint32_t (&ax)[D], const uint32_t (&az)[D], int ntop, bool pack,
                                 const uint32_t *neg_lut, uint32_t thr, uint32_t best, uint32_t &done,
                                 uint32_t &tail_skip, Census &cs) {
  v8i_t B[1][4];
  mfma_tops<D, 1, 3>(ax, az, lane, ntop, pack, neg_lut, B);  // the three groups of word 0
  const uint32_t T = __float_as_uint(static_cast<float>(4 * thr));
  uint32_t c = ca;
  if (coop) {
    CoopStream st;
    constexpr int kPer = CoopStream::kPer;
    st.start(mtab, mks, c);
    st.store(sbuf);
    __syncthreads();
    for (int g = 0; c < cs_end; ++g, c += kCoopChunks) {
      const int nu = min(kCoopChunks, static_cast<int>(cs_end - c));
      const bool more = c + kCoopChunks < cs_end;
      if (more) st.next();
      const uint4 *cur = sbuf + (g & 1) * kPer;
      uint32_t pm[kCoopChunks];
      if (nu == kCoopChunks) {  // a full group: one straight block the compiler can interleave
#pragma unroll
        for (int u = 0; u < kCoopChunks; ++u) pm[u] = mfma_first_chunk(mfma_operand(cur[u * kWave + lane]), B);
      } else {
#pragma unroll
        for (int u = 0; u < kCoopChunks; ++u)
          pm[u] = u < nu ? mfma_first_chunk(mfma_operand(cur[u * kWave + lane]), B) : 0xFFFFFFFFu;
      }
      const uint32_t any = min(min(pm[0], pm[1]), min(pm[2], pm[3]));
      if (__ballot(any < T)) best = complete_chunks<D, kCensus>(table, c, nu, pm, T, ax, az, best, done, cs);
      if (more) st.store(sbuf + ((g + 1) & 1) * kPer);
      __syncthreads();
    }
    c = cs_end;  // the last group may be short
  }
  const size_t stride = static_cast<size_t>(mks) * kWave;
  const uint4 *mb = mtab + static_cast<size_t>(c) * stride + lane;
  for (; c < cz; c += kMfmaUnroll, mb += kMfmaUnroll * stride) {
    const int nu = min(kMfmaUnroll, static_cast<int>(cz - c));
    uint32_t pm[kMfmaUnroll];
#pragma unroll
    for (int u = 0; u < kMfmaUnroll; ++u) pm[u] = u < nu ? mfma_first_chunk(mfma_operand(mb[u * stride]), B) : 0xFFFFFFFFu;
    uint32_t any = pm[0];
#pragma unroll
    for (int u = 1; u < kMfmaUnroll; ++u) any = min(any, pm[u]);
    if (__ballot(any < T)) best = complete_chunks<D, kCensus>(table, c, nu, pm, T, ax, az, best, done, cs);
  }
  if (ct > cz) {
    // Entries of the top of column r of block nb: lane 16 q + r holds rows
    // 4q..4q+3 of that column.
    const int q4 = static_cast<int>(lane >> 4) * 4;
    int lim[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const int src = nb * kChunk + static_cast<int>(lane & 15);
      const int sp = static_cast<int>(bcast(span, src));
      lim[nb] = (src < ntop ? sp : 0) - static_cast<int>(rel) - q4;
    }
    const uint4 *mb = mtab + static_cast<size_t>(cz) * mks * kWave + lane;
    for (uint32_t c = cz; c < ct; ++c, mb += static_cast<size_t>(mks) * kWave) {
      const v8i_t A = mfma_operand(*mb);
      const v4f_t zero = {0.0f, 0.0f, 0.0f, 0.0f};
      uint32_t pm = 0xFFFFFFFFu;
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) {
        const v4f_t acc = mfma_fp4(A, B[0][nb], zero);
        const int l = lim[nb] - static_cast<int>(c - cz) * kChunk;
#pragma unroll
        for (int i = 0; i < 4; ++i) pm = min(pm, i < l ? __float_as_uint(acc[i]) : 0xFFFFFFFFu);
      }
      const uint32_t r0 = rel + (c - cz) * kChunk;  // the chunk's first entry in the tile
      if (__ballot(pm < T)) {
        // Completed: every word of each lane's entries of the chunk.
        for (uint32_t i = r0; i < min(r0 + kChunk, send); ++i) {
          const uint32_t w = weight_at<D>(table, k0 + i, ax, az);
          if (i < span) best = min(best, w);
        }
      } else {
        tail_skip += span > r0 ? min(span - r0, static_cast<uint32_t>(kChunk)) : 0u;
      }
    }
  }
  return best;
}

// A tile's witness slot: the codeword in the matrix's stored qubit order
// (the commit kernel maps it back to qubit order).
template <int D>
__device__ __forceinline__ void write_slot(uint32_t *out, const uint32_t (&cx)[D], const uint32_t (&cz)[D]) {
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    out[d] = d < D ? cx[d < D ? d : 0] : 0u;
    out[4 + d] = d < D ? cz[d < D ? d : 0] : 0u;
  }
}

// Top combination number `item` of the group whose smallest package is h:
// the element of h is the most significant digit, then the remaining
// t-u-1 packages above h in lexicographic order.  F(j, r) = e_r(c_j..),
// read from column r of a table with `ld` columns.
template <int D>
__device__ void unrank_top(const unsigned long long *F, int ld, const uint32_t *elems,
                           const unsigned char *__restrict__ csize, int P, int r, int h,
                           unsigned long long item, uint32_t (&ax)[D], uint32_t (&az)[D]) {
  unsigned long long rest = item;
  const unsigned long long f = F[size_t(h + 1) * ld + r];
  int c = 0;
  while (rest >= f && c < 2) { rest -= f; ++c; }
  xor_elem<D>(elems, h, c, ax, az);
  for (int j = h + 1; r > 0 && j < P; ++j) {
    const unsigned long long fj = F[size_t(j + 1) * ld + (r - 1)];
    const unsigned long long cnt = fj * csize[j];
    if (rest < cnt) {
      int cj = 0;
      while (rest >= fj && cj < 2) { rest -= fj; ++cj; }
      xor_elem<D>(elems, j, cj, ax, az);
      --r;
    } else {
      rest -= cnt;
    }
  }
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) { return wave_max_u32(v); }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return wave_sum_u32(v); }

// Modified BZ: a codeword of the span is outside its radical (the
// stabilizer) when its symplectic product with some logical operator is 1.
template <int D>
__device__ bool admitted(const uint32_t (&cx)[D], const uint32_t (&cz)[D], const uint32_t *L, int nL) {
  for (int i = 0; i < nL; ++i) {
    const uint32_t *l = L + static_cast<size_t>(i) * kElemWords;
    uint32_t v = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) v ^= (cx[d] & l[4 + d]) ^ (cz[d] & l[d]);
    if (__builtin_popcount(v) & 1) return true;
  }
  return false;
}

// Workgroups per chunk dealt to one XCD (see qd_round_kernel).
constexpr uint32_t kXcdChunk = 16;

// One tile = one table segment [k0, k0 + seg) x 64 tops.  The tops of a
// tile come from every group whose table prefix reaches the segment, so
// lanes stay full; a lane stops at its own group's prefix length.  A launch
// holds pieces of the current rounds of several codes (RoundDesc).  With
// kCensus every piece also takes the census of its codewords below p.below.
// kMode: kEmEveryWord for launches whose pieces evaluate every word (their
// full blocks go through entry-major blocks first), kEmPartial for the
// others (entry-major blocks on the first word where partial weights decide
// on it).  The two hold different register sets, so each launch takes the
// one its pieces need.
template <int D, bool kCensus, int kMode>
__global__ __launch_bounds__(256) void qd_round_kernel(LaunchParams lp) {
  extern __shared__ unsigned long long smem[];
  // Consecutive workgroups land on different XCDs (round robin).  Deal them
  // to the XCDs in chunks of kXcdChunk consecutive workgroups instead: a
  // chunk's tiles share table segments (one L2), and every XCD gets chunks
  // from the whole launch, so pieces whose tiles cost different amounts
  // (rounds of other sizes, other codes) stay balanced across XCDs.
  const uint32_t xcd = blockIdx.x % 8, r = blockIdx.x / 8;
  const uint32_t wg = ((r / kXcdChunk) * 8 + xcd) * kXcdChunk + r % kXcdChunk;
  const unsigned long long wtile = static_cast<unsigned long long>(wg) * kWavesPerGroup;
  if (wtile >= lp.tiles) return;  // whole workgroup: launch padding
  const RoundDesc *const descs = lp.desc;
  const RoundDesc &p = descs[wave_last_le(lp.ndesc, wtile, [descs](int i) { return descs[i].tile_begin; })];
  // Matrix cores: each wave's shared-chunk range (first chunk << 32 | end),
  // ~0 for a wave that takes no part; chunk buffers of the workgroup.
  constexpr bool kMfmaEvery = mfma_every_mode(kMode);
  constexpr bool kMfma = kMfmaEvery || kMode == kMfmaPartial;
  constexpr bool kCoop = kMode == kMfmaPartial;
  __shared__ unsigned long long coop_slot[kWavesPerGroup];
  __shared__ uint4 coop_buf[kCoop ? 2 * kCoopChunks * kWave : 1];
  __shared__ uint32_t neg_lut[kMfma ? kWave * kWavesPerGroup : 1];
  if (kCoop && (threadIdx.x & (kWave - 1)) == 0) coop_slot[threadIdx.x / kWave] = ~0ull;
  if constexpr (kMfma) fill_neg_lut(neg_lut);

  // Unranking reads suffix columns, the group table and the elements with
  // data-dependent addresses: stage them in LDS once per workgroup.
  const int C = p.t - p.u;  // suffix columns 0..t-u-1
  const unsigned long long *F = p.suffix;
  const DevGroup *GR = p.groups;
  const uint32_t *E = p.elems;
  int ld = p.R;
  if (p.stage) {
    DevGroup *sG = reinterpret_cast<DevGroup *>(smem);
    for (int i = threadIdx.x; i < p.ngroups; i += blockDim.x) sG[i] = p.groups[i];
    GR = sG;
    if (p.stage == 2) {
      unsigned long long *sF = reinterpret_cast<unsigned long long *>(sG + p.ngroups);
      uint32_t *sE = reinterpret_cast<uint32_t *>(sF + (p.P + 1) * C);
      for (int i = threadIdx.x; i < (p.P + 1) * C; i += blockDim.x) sF[i] = p.suffix[size_t(i / C) * p.R + i % C];
      for (int i = threadIdx.x; i < p.P * 3 * kElemWords; i += blockDim.x) sE[i] = p.elems[i];
      F = sF;
      E = sE;
      ld = C;
    }
    if constexpr (!kMfma) __syncthreads();
  }
  if constexpr (kMfma) __syncthreads();  // staged tables, neg_lut; every wave's coop_slot cleared
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const unsigned long long local = wtile + wave - p.tile_begin;  // tile within the piece
  if (local >= p.ntiles) return;                                  // piece padding
  const unsigned long long g = p.tile_lo + local;                 // tile within the round
  DevState *st = p.state;
  // The key is read with plain loads: a stale (larger) U only delays the
  // early exit or triggers a redundant witness search; the atomicMin below
  // is what decides.
  unsigned long long key = uniform64(*reinterpret_cast<volatile unsigned long long *>(&st->key));
  if (static_cast<int>(key >> 32) <= p.L_before) return;  // bound already met

  const DevRun *const runs = p.runs;
  const DevRun &run = runs[wave_last_le(p.nruns, g, [runs](int i) { return runs[i].tile0; })];
  const unsigned long long rl = g - run.tile0;
  unsigned long long b, s;
  if ((rl >> 32) == 0 && (run.tps >> 32) == 0) {
    const uint32_t l32 = static_cast<uint32_t>(rl), t32 = static_cast<uint32_t>(run.tps);
    b = l32 % t32;
    s = run.s_begin + l32 / t32;
  } else {
    b = rl % run.tps;
    s = run.s_begin + rl / run.tps;
  }
  const unsigned long long k0 = s * p.seg;
  const unsigned long long k1 = k0 + p.seg;
  const unsigned long long item = b * kWave + lane;
  const bool active = item < run.items;

  uint32_t ax[D], az[D];
#pragma unroll
  for (int d = 0; d < D; ++d) ax[d] = az[d] = 0;
  unsigned long long lend = k1;  // this lane's end of the segment
  // The lane's group: the tile's 64 items are consecutive, so the group
  // of the first one is found by the whole wave at once, and a lane steps
  // past the groups that start inside the tile at or below its item (few,
  // usually none).
  const unsigned long long item0 = b * kWave;
  const int ne = static_cast<int>(run.e);
  int a = wave_last_le(ne, item0, [GR](int i) { return GR[i].cum; });
  for (int j = a + 1; j < ne; ++j) {
    const unsigned long long cj = GR[j].cum;  // the same for every lane
    if (cj >= item0 + kWave) break;
    if (item >= cj) a = j;
  }
  if (active) {
    lend = min(k1, GR[a].len);
    if (p.tops && p.tops_down) {
      // Element c of the smallest package XOR a top one package shallower.
      const unsigned long long f = GR[a].f;
      unsigned long long rest = item - GR[a].cum;
      int c = 0;
      while (rest >= f && c < 2) {
        rest -= f;
        ++c;
      }
      const uint32_t *tp = p.tops + rest * (2 * D);
      const uint32_t *el = p.elems + (size_t(3) * GR[a].h + c) * kElemWords;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        ax[d] = tp[d] ^ el[d];
        az[d] = tp[D + d] ^ el[4 + d];
      }
    } else if (p.tops) {
      const uint32_t *tp = p.tops + (GR[a].top0 + item - GR[a].cum) * (2 * D);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        ax[d] = tp[d];
        az[d] = tp[D + d];
      }
    } else {
      unrank_top<D>(F, ld, E, p.csize, p.P, p.t - p.u - 1, static_cast<int>(GR[a].h), item - GR[a].cum, ax,
                    az);
    }
  }
  // Entries [k0, k0 + sfull) are valid for every lane; up to k0 + send for some.
  const uint32_t span = static_cast<uint32_t>(lend - k0);
  const uint32_t sfull = __builtin_amdgcn_readfirstlane(wave_min(span));
  const uint32_t send = __builtin_amdgcn_readfirstlane(wave_max(active ? span : 0u));
  uint32_t best = 0xFFFFFFFFu;
  const uint32_t nfull = sfull / kBlock;
  const uint32_t *blk = p.table + (k0 / kBlock) * (2 * D * kBlock);
  // Words evaluated per codeword in the full blocks: the smallest w whose
  // cap admits the U this tile started with (D: no partial weights).  A
  // census raises that threshold to its own bound, so that every block that
  // may hold a codeword below it is completed.
  Census cs;
  if constexpr (kCensus) cs.below = static_cast<uint32_t>(p.below);
  const int U0 = kCensus ? max(static_cast<int>(key >> 32), p.below) : static_cast<int>(key >> 32);
  int W = D;
#pragma unroll
  for (int w = D - 1; w >= 1; --w)
    if (U0 <= p.cap[w - 1]) W = w;
  uint32_t rec = 0;  // full blocks evaluated in full
  // Every word: entry-major blocks over the wave's active tops (lanes
  // 0..nact-1: items grow with the lane), then the streaming loop for the
  // rest of the full blocks.  best_em and cs_em hold codewords of every
  // active top, whatever the lane's own top.
  uint32_t best_em = 0xFFFFFFFFu;
  Census cs_em;
  if constexpr (kCensus) cs_em.below = static_cast<uint32_t>(p.below);
  const int ntop = static_cast<int>(__popcll(__ballot(active)));
  uint32_t em_partial = 0, em_done = 0;  // entry-major blocks with partial weights; tops completed in them
  // Matrix cores: chunks [ca, cz) of kChunk entries inside the full blocks;
  // the full blocks before and after them (at most one each) stay on the
  // vector ALU.
  uint32_t ca = 0, cz = 0, ct = 0, mf_done = 0, tail_skip = 0;
  bool tail_mfma = false;  // partial weights: the entries past the full chunks on the matrix cores too
  if (kMfma && p.mtable) {
    const uint32_t c_lo = static_cast<uint32_t>((k0 + kChunk - 1) / kChunk);
    const uint32_t c_hi = static_cast<uint32_t>((k0 + nfull * kBlock) / kChunk);
    if (kMode == kMfmaPartial && D >= 2 && W == 1 && k0 % kChunk == 0) {
      ca = __builtin_amdgcn_readfirstlane(c_lo);
      cz = __builtin_amdgcn_readfirstlane(c_hi);
      ct = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>((k0 + send + kChunk - 1) / kChunk));
      tail_mfma = true;
    } else if (c_hi > c_lo && (kMfmaEvery ? W == D : W == 1)) {
      ca = __builtin_amdgcn_readfirstlane(c_lo);
      cz = __builtin_amdgcn_readfirstlane(c_hi);
    }
  }
  // The workgroup's four waves share chunks [ca, cs) when all of them take
  // part from the same first chunk (the same table segment).
  uint32_t cs_end = ca;
  bool coop = false;
  if constexpr (kCoop) {
    if (lane == 0 && cz > ca) coop_slot[wave] = (static_cast<unsigned long long>(ca) << 32) | cz;
    __syncthreads();  // the waves that returned early left ~0
    coop = cz > ca;
    cs_end = cz;
#pragma unroll
    for (int w = 0; w < kWavesPerGroup; ++w) {
      const unsigned long long v = coop_slot[w];
      coop = coop && v != ~0ull && static_cast<uint32_t>(v >> 32) == ca;
      cs_end = min(cs_end, static_cast<uint32_t>(v));
    }
    coop = __builtin_amdgcn_readfirstlane(coop ? 1u : 0u) != 0u;
    cs_end = coop ? __builtin_amdgcn_readfirstlane(cs_end) : ca;
  }
  const uint32_t head = static_cast<uint32_t>((static_cast<unsigned long long>(ca) * kChunk - k0) / kBlock);
  const uint32_t mid = (cz - ca) * (kChunk / kBlock);  // full blocks on the matrix cores
  if (kMfma && (mid > 0 || tail_mfma)) {
    if constexpr (kMfmaEvery) {
      constexpr int kPackedKs = D >= 3 ? D - 1 : D;
      if constexpr (kMode == kMfmaEveryPacked)
        best_em = mfma_every<D, kPackedKs>(p.mtable, ca, cz, lane, ax, az, ntop, true, neg_lut);
      else if constexpr (kMode == kMfmaEveryPlain)
        best_em = mfma_every<D, D>(p.mtable, ca, cz, lane, ax, az, ntop, false, neg_lut);
      else if (D >= 3 && p.mpack)
        best_em = mfma_every<D, kPackedKs>(p.mtable, ca, cz, lane, ax, az, ntop, true, neg_lut);
      else
        best_em = mfma_every<D, D>(p.mtable, ca, cz, lane, ax, az, ntop, false, neg_lut);
      for (uint32_t i = 0; i < head; ++i, blk += 2 * D * kBlock) best = block_min<D, kCensus>(ax, az, blk, best, cs);
      blk += mid * (2 * D * kBlock);
      for (uint32_t i = head + mid; i < nfull; ++i, blk += 2 * D * kBlock)
        best = block_min<D, kCensus>(ax, az, blk, best, cs);
    } else if constexpr (D >= 2) {
      const int c = p.credit[0];
      const uint32_t thr = U0 > c ? static_cast<uint32_t>(U0 - c) : 0u;
      const uint32_t rel = static_cast<uint32_t>(static_cast<unsigned long long>(cz) * kChunk - k0);
      best = mfma_partial<D, kCensus>(p.table, p.mtable, p.mks, ca, cs_end, cz, ct, rel, k0, active ? span : 0u,
                                      send, coop, coop_buf, lane, ax, az, ntop, p.mpack != 0, neg_lut, thr, best,
                                      mf_done, tail_skip, cs);
      if (tail_mfma) {
        rec = nfull;  // the full blocks are counted by mf_done and tail_skip
      } else {
        best = partial_blocks<D, 1, kCensus>(ax, az, blk, head, best, thr, rec, cs);
        best = partial_blocks<D, 1, kCensus>(ax, az, blk + (head + mid) * (2 * D * kBlock), nfull - head - mid,
                                             best, thr, rec, cs);
        rec += mid;  // the matrix-core blocks are counted by mf_done
      }
    }
  } else if (W == D) {
    constexpr uint32_t kEm = kWave * EmK<D>::K;
    const uint32_t nem = kMode == kEmEveryWord && ntop > 1 ? sfull / kEm : 0u;
    for (uint32_t bk = 0; bk < nem; ++bk)
      best_em = em_block<D, kCensus>(p.table, k0 + static_cast<unsigned long long>(bk) * kEm, lane, ax, az, ntop,
                                     best_em, cs_em);
    blk += (nem * kEm / kBlock) * (2 * D * kBlock);
    for (uint32_t i = nem * kEm / kBlock; i < nfull; ++i, blk += 2 * D * kBlock)
      best = block_min<D, kCensus>(ax, az, blk, best, cs);
  } else {
    const int c = p.credit[W - 1];
    const uint32_t thr = U0 > c ? static_cast<uint32_t>(U0 - c) : 0u;
    if constexpr (D >= 2 && kMode == kEmPartial) {
      if (W == 1) {  // entry-major blocks on the first word, then the streaming loop
        constexpr uint32_t kEm = kWave * kEmPartialK;
        em_partial = ntop > 1 ? sfull / kEm : 0u;
        for (uint32_t bk = 0; bk < em_partial; ++bk)
          best_em = em_block_partial<D, kCensus>(p.table, k0 + static_cast<unsigned long long>(bk) * kEm, lane, ax,
                                                 az, ntop, best_em, thr, cs_em, em_done);
        const uint32_t skip = em_partial * kEm / kBlock;
        best = partial_blocks<D, 1, kCensus>(ax, az, blk + skip * (2 * D * kBlock), nfull - skip, best, thr, rec,
                                             cs);
        rec += skip;  // the blocks the entry-major part covered are counted by em_done
      }
    } else if constexpr (D >= 2) {
      if (W == 1) best = partial_blocks<D, 1, kCensus>(ax, az, blk, nfull, best, thr, rec, cs);
    }
    if constexpr (D >= 3) {
      if (W == 2) best = partial_blocks<D, 2, kCensus>(ax, az, blk, nfull, best, thr, rec, cs);
    }
    if constexpr (D >= 4) {
      if (W == 3) best = partial_blocks<D, 3, kCensus>(ax, az, blk, nfull, best, thr, rec, cs);
    }
  }
  for (uint32_t i = tail_mfma ? send : nfull * kBlock; i < send; ++i) {
    const uint32_t w = weight_at<D>(p.table, k0 + i, ax, az);
    if (i < span) {
      best = min(best, w);
      if constexpr (kCensus) cs.add(w);
    }
  }
  if (!active) best = 0xFFFFFFFFu;
  const uint32_t wmin = wave_min(min(best, best_em));
  const uint32_t visited = wave_sum(active ? span : 0u);
  const uint32_t tail_skipped = tail_mfma ? wave_sum(tail_skip) : 0u;
  const unsigned long long nact = static_cast<unsigned long long>(ntop);
  if constexpr (kCensus) {
    // Per lane at most 64 seg codewords of weight <= 128: the wave sums fit 32 bits.
    const uint32_t ccnt = wave_sum((active ? cs.cnt : 0u) + cs_em.cnt);
    const uint32_t csum = wave_sum((active ? cs.sum : 0u) + cs_em.sum);
    if (lane == 0 && p.census) {
      atomicAdd(p.census, static_cast<unsigned long long>(ccnt));
      atomicAdd(p.census + 1, static_cast<unsigned long long>(csum));
    }
  }
  if (lane == 0) {
    // Words: D per visited codeword, less D - W for those of the full
    // blocks that the partial weights decided.
    // Entry-major blocks with partial weights: 64 K codewords per top,
    // every top not completed skipped D - 1 words for each.
    const unsigned long long skipped =
        static_cast<unsigned long long>(nfull - rec) * kBlock * (D - W) * nact +
        (static_cast<unsigned long long>(em_partial) * nact - em_done) * (kWave * kEmPartialK) * (D - 1) +
        (kMode == kMfmaPartial ? static_cast<unsigned long long>(cz - ca - mf_done) * kChunk * nact * (D - 1) : 0ull) +
        static_cast<unsigned long long>(tail_skipped) * (D - 1);
    unsigned long long *c = p.counters + static_cast<size_t>(wg % kCountersPerCode) * kCounterStride;
    atomicAdd(c, static_cast<unsigned long long>(visited));
    atomicAdd(c + 1, static_cast<unsigned long long>(visited) * D - skipped);
  }

  key = uniform64(*reinterpret_cast<volatile unsigned long long *>(&st->key));
  if (p.nlogicals > 0) {
    // Modified BZ: the tile's minimum may be a stabilizer element, which
    // must not update U.  Rare path: look for the least admitted weight
    // below U in this tile, then publish it as below.
    const uint32_t thr = static_cast<uint32_t>(key >> 32);
    if (wmin >= thr) return;
    uint32_t be = 0xFFFFFFFFu, kf = 0xFFFFFFFFu;
    for (uint32_t i = 0; i < send; ++i) {
      const uint32_t w = weight_at<D>(p.table, k0 + i, ax, az);
      if (active && i < span && w < thr && w < be) {
        const unsigned long long kk = k0 + i;
        const uint32_t *e = p.table + (kk / kBlock) * (2 * D * kBlock) + (kk % kBlock);
        uint32_t cx[D], cz[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          cx[d] = ax[d] ^ e[d * kBlock];
          cz[d] = az[d] ^ e[(D + d) * kBlock];
        }
        if (admitted<D>(cx, cz, p.logicals, p.nlogicals)) {
          be = w;
          kf = i;
        }
      }
    }
    const uint32_t wadm = wave_min(be);
    if (wadm >= thr) return;
    const unsigned long long mask = __ballot(be == wadm);
    const int winner = __ffsll(static_cast<long long>(mask)) - 1;
    if (static_cast<int>(lane) == winner) {
      const uint32_t slot = static_cast<uint32_t>(p.slot0 + local);
      const unsigned long long kk = k0 + kf;
      const uint32_t *e = p.table + (kk / kBlock) * (2 * D * kBlock) + (kk % kBlock);
      uint32_t cx[D], cz[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        cx[d] = ax[d] ^ e[d * kBlock];
        cz[d] = az[d] ^ e[(D + d) * kBlock];
      }
      write_slot<D>(lp.slots + static_cast<size_t>(slot) * kElemWords, cx, cz);
      atomicMin(&st->key, (static_cast<unsigned long long>(wadm) << 32) | slot);
    }
    return;
  }
  if (wmin < static_cast<uint32_t>(key >> 32)) {
    // Rare: this tile improves U.  Find where, write the codeword to this
    // tile's own slot, then publish (U, slot) with one 64-bit atomicMin.
    uint32_t kf = 0xFFFFFFFFu;
    for (uint32_t i = 0; i < send; ++i) {
      const uint32_t w = weight_at<D>(p.table, k0 + i, ax, az);
      if (i < span && w == wmin && kf == 0xFFFFFFFFu) kf = i;
    }
    const unsigned long long mask = __ballot(active && kf != 0xFFFFFFFFu);
    const int winner = __ffsll(static_cast<long long>(mask)) - 1;
    if (static_cast<int>(lane) == winner) {
      const uint32_t slot = static_cast<uint32_t>(p.slot0 + local);  // launch-wide slot
      const unsigned long long kk = k0 + kf;
      const uint32_t *e = p.table + (kk / kBlock) * (2 * D * kBlock) + (kk % kBlock);
      uint32_t cx[D], cz[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        cx[d] = ax[d] ^ e[d * kBlock];
        cz[d] = az[d] ^ e[(D + d) * kBlock];
      }
      write_slot<D>(lp.slots + static_cast<size_t>(slot) * kElemWords, cx, cz);
      atomicMin(&st->key, (static_cast<unsigned long long>(wmin) << 32) | slot);
    }
  }
}

// -- launch (host) -------------------------------------------------------------

template <int D>
void launch_round_d(const LaunchParams &lp, bool census, bool every_word, int mfma, dim3 grid, dim3 block,
                    hipStream_t s) {
#define QD_LAUNCH(C, M) hipLaunchKernelGGL((qd_round_kernel<D, C, M>), grid, block, lp.lds, s, lp)
  if (mfma && !census && every_word) {
    if constexpr (D >= 3) {  // a packed last word needs three words per half
      if (mfma == 2)
        QD_LAUNCH(false, kMfmaEveryPacked);
      else if (mfma == 1)
        QD_LAUNCH(false, kMfmaEveryWord);
      else
        QD_LAUNCH(false, kMfmaEveryPlain);
    } else {
      QD_LAUNCH(false, kMfmaEveryPlain);
    }
  } else if (mfma && !census && D >= 2) {
    QD_LAUNCH(false, kMfmaPartial);
  } else if (census) {
    if (every_word)
      QD_LAUNCH(true, kEmEveryWord);
    else
      QD_LAUNCH(true, kEmPartial);
  } else if (every_word) {
    QD_LAUNCH(false, kEmEveryWord);
  } else {
    QD_LAUNCH(false, kEmPartial);
  }
#undef QD_LAUNCH
}

// mfma: 0 vector ALU; matrix cores with 1 layouts mixed, 2 every piece packed,
// 3 every piece plain.
hipError_t launch_round(int D, const LaunchParams &lp, bool census, bool every_word, int mfma, hipStream_t s) {
  unsigned long long wgs = lp.tiles / kWavesPerGroup;
  wgs = (wgs + 8 * kXcdChunk - 1) / (8 * kXcdChunk) * (8 * kXcdChunk);  // the XCD dealing is a bijection
  dim3 grid(static_cast<uint32_t>(wgs)), block(kWave * kWavesPerGroup);
  switch (D) {
    case 1: launch_round_d<1>(lp, census, every_word, mfma, grid, block, s); break;
    case 2: launch_round_d<2>(lp, census, every_word, mfma, grid, block, s); break;
    case 3: launch_round_d<3>(lp, census, every_word, mfma, grid, block, s); break;
    case 4: launch_round_d<4>(lp, census, every_word, mfma, grid, block, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qd

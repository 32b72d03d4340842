// walk.hip -- the plain per-round enumeration kernel of libqdist (gfx950).
//
// One launch walks every combination of one (t, Gamma_j) round: t distinct
// packages and one nonzero element of each (Sec. 2.3).  It is not the
// default path (the saved-sum kernel in round.hip is); it is the plain
// per-code path the engine is measured against, and a second enumeration
// of a different order for the tests.
//
// A round is split into parts by u, the number of one-row packages in a
// set: part u holds the sets of u one-row and t - u two-row packages, each
// with 3^(t-u) element choices, and its sets are ranked as (one-row subset,
// two-row subset), each in revolving-door order (combinatorial number
// system, revdoor.hpp).  Lane l of the part's wave g takes the sets of rank
// [(64 g + l) K, (64 g + l + 1) K), K sets per lane: it unranks the first
// and reaches the next by one two-row package out and one in (when the
// two-row subset wraps around, the lane forms the set's codeword afresh).
// Within a set the lane walks the element choices of its two-row packages
// in reflected ternary Gray order: slot j of the lane holds one of them and
// digit j its element (0: r, 1: s, 2: r^s), and each step moves one digit
// by one, which XORs one element into the codeword (0 <-> 1: r^s; 1 <-> 2:
// r).  The walk continues from the digits where the previous set left them
// (all 2 after an even set, all 0 after an odd one), so the lane's sets are
// one reflected Gray walk.  Every lane of a wave is in the same part and at
// the same step, so the digit that moves is wave-uniform: its row sits at a
// static VGPR index (digits 0 and 1, 8 of every 9 steps) or is read from
// LDS (the others).  A step is one XOR per word, an OR and a v_bcnt per
// word, and a min, and every codeword is walked once.
#include <hip/hip_runtime.h>

#define QD_HD __host__ __device__
#include "kernels.hpp"
#include "revdoor.hpp"
#include "wave.hpp"

namespace qd {
namespace {

// Modes of a lane's walk: the minimum weight; the minimum and the sum of
// the weights of every codeword walked; the first codeword of a given
// weight (the witness re-scan).
constexpr int kWalkMin = 0, kWalkSum = 1, kWalkFind = 2;

__device__ __forceinline__ uint32_t min3u(uint32_t a, uint32_t b, uint32_t c) { return min(a, min(b, c)); }

__device__ __forceinline__ unsigned long long uniform64w(unsigned long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// 64-bit sums (combination and codeword counts; once per wave).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += static_cast<unsigned long long>(__shfl_xor(v, off));
  return v;
}

// A lane's two-row packages, one per digit.  Digits 0 and 1 move on 8 of
// every 9 steps: their rows sit in VGPRs, oriented for the current set (x:
// the row of the digit's first move in the set's even blocks, y: the other;
// an even set starts with its digits rising, x = r^s, y = r).  The other
// digits move once per 9 steps and read their row from the staged
// elements: bits 8 (j - 2) .. 8 (j - 2) + 7 of `high` hold slot j's package
// (a matrix has at most 2 x 128 packages), so the wave-uniform j selects it
// by a shift.
template <int D>
struct Slots {
  uint32_t x0[2 * D], y0[2 * D], x1[2 * D], y1[2 * D];
  unsigned long long high;
  int pkg[kWalkMaxT];
};

constexpr int kHighBits = 8;

__device__ __forceinline__ unsigned long long high_field(int p, int k) {
  return static_cast<unsigned long long>(p) << (kHighBits * (k - 2));
}

__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
  uint32_t r;
  asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
  return r;
}

// What a lane does with each weight it computes.
template <int D, int MODE>
struct Visit {
  uint32_t best = 0xFFFFFFFFu;  // over the lane's sets
  uint32_t sb = 0xFFFFFFFFu;    // over the current set
  uint32_t ssum = 0;            // weights of the current set (kWalkSum)
  unsigned long long wsum = 0;
  bool live = false;            // the current set is the lane's
  // kWalkFind
  uint32_t target = 0;
  bool found = false;
  uint32_t fc[2 * D];

  __device__ __forceinline__ void each(uint32_t w, const uint32_t (&c)[2 * D]) {
    if constexpr (MODE == kWalkSum) ssum += w;
    if constexpr (MODE == kWalkFind) {
      if (live && !found && w == target) {
        found = true;
#pragma unroll
        for (int i = 0; i < 2 * D; ++i) fc[i] = c[i];
      }
    }
  }
  __device__ __forceinline__ void one(uint32_t w, const uint32_t (&c)[2 * D]) {
    each(w, c);
    if constexpr (MODE != kWalkFind) sb = min(sb, w);
  }
  __device__ __forceinline__ void eight(const uint32_t (&w)[8]) {
    if constexpr (MODE != kWalkFind) {
      sb = min3u(sb, w[0], w[1]);
      sb = min3u(sb, w[2], w[3]);
      sb = min3u(sb, w[4], w[5]);
      sb = min3u(sb, w[6], w[7]);
    }
  }
  __device__ __forceinline__ void end_set() {
    if (live) {
      best = min(best, sb);
      wsum += ssum;
    }
    sb = 0xFFFFFFFFu;
    ssum = 0;
  }
};

// XOR a row into the codeword and return its weight.
template <int D>
__device__ __forceinline__ uint32_t flip(uint32_t (&c)[2 * D], const uint32_t (&row)[2 * D]) {
  uint32_t acc = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    c[d] ^= row[d];
    c[D + d] ^= row[D + d];
    const uint32_t o = c[d] | c[D + d];
    acc = d == 0 ? __builtin_popcount(o) : bcnt_acc(o, acc);
  }
  return acc;
}

template <int D>
__device__ __forceinline__ uint32_t weight_of(const uint32_t (&c)[2 * D]) {
  uint32_t acc = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) acc += __builtin_popcount(c[d] | c[D + d]);
  return acc;
}

// Eight steps of the walk moving digits 0 and 1 only (the steps between
// two multiples of 9).  Rising digits move 0 -> 1 (r^s) then 1 -> 2 (r),
// falling ones 2 -> 1 (r) then 1 -> 0 (r^s), and a digit turns at every
// move of the next one: an even block of a set XORs x0 y0 x1 y0 x0 y1 x0
// y0, an odd block (ODD) the same with x and y traded.
template <int D, int MODE, bool ODD>
__device__ __forceinline__ void block8(uint32_t (&c)[2 * D], const Slots<D> &s, Visit<D, MODE> &v) {
  const uint32_t(&x0)[2 * D] = ODD ? s.y0 : s.x0;
  const uint32_t(&y0)[2 * D] = ODD ? s.x0 : s.y0;
  const uint32_t(&x1)[2 * D] = ODD ? s.y1 : s.x1;
  const uint32_t(&y1)[2 * D] = ODD ? s.x1 : s.y1;
  uint32_t w[8];
  w[0] = flip<D>(c, x0); v.each(w[0], c);
  w[1] = flip<D>(c, y0); v.each(w[1], c);
  w[2] = flip<D>(c, x1); v.each(w[2], c);
  w[3] = flip<D>(c, y0); v.each(w[3], c);
  w[4] = flip<D>(c, x0); v.each(w[4], c);
  w[5] = flip<D>(c, y1); v.each(w[5], c);
  w[6] = flip<D>(c, x0); v.each(w[6], c);
  w[7] = flip<D>(c, y0); v.each(w[7], c);
  v.eight(w);
}

// XOR element number `el` (3 p + e) of the staged elements.
template <int D>
__device__ __forceinline__ uint32_t flip_elem(uint32_t (&c)[2 * D], const uint32_t *E, uint32_t el) {
  const uint4 *q = reinterpret_cast<const uint4 *>(E + static_cast<size_t>(el) * kElemWords);
  const uint4 qx = q[0], qz = q[1];
  const uint32_t rx[4] = {qx.x, qx.y, qx.z, qx.w}, rz[4] = {qz.x, qz.y, qz.z, qz.w};
  uint32_t acc = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    c[d] ^= rx[d];
    c[D + d] ^= rz[d];
    const uint32_t o = c[d] | c[D + d];
    acc = d == 0 ? __builtin_popcount(o) : bcnt_acc(o, acc);
  }
  return acc;
}

// Element e of package p (0: r, 1: s, 2: r^s).
template <int D>
__device__ __forceinline__ void load_elem(const uint32_t *E, int p, int e, uint32_t (&out)[2 * D]) {
  const uint32_t *q = E + (static_cast<size_t>(3) * p + e) * kElemWords;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    out[d] = q[d];
    out[D + d] = q[4 + d];
  }
}

// The rows of two-row package p's digit moves, oriented for a set of
// parity `odd`.
template <int D>
__device__ __forceinline__ void load_rows(const uint32_t *E, int p, bool odd, uint32_t (&x)[2 * D],
                                          uint32_t (&y)[2 * D]) {
  const uint32_t *qa = E + (static_cast<size_t>(3) * p + 2) * kElemWords;  // r^s
  const uint32_t *qb = E + (static_cast<size_t>(3) * p) * kElemWords;      // r
#pragma unroll
  for (int d = 0; d < D; ++d) {
    x[d] = odd ? qb[d] : qa[d];
    x[D + d] = odd ? qb[4 + d] : qa[4 + d];
    y[d] = odd ? qa[d] : qb[d];
    y[D + d] = odd ? qa[4 + d] : qb[4 + d];
  }
}

template <int D>
__device__ __forceinline__ void swap_rows(uint32_t (&x)[2 * D], uint32_t (&y)[2 * D]) {
#pragma unroll
  for (int i = 0; i < 2 * D; ++i) {
    const uint32_t tmp = x[i];
    x[i] = y[i];
    y[i] = tmp;
  }
}

// Step 9 m of a set moves digit j >= 2, where 3^(j-2) is the power of 3 in
// m; the digit rises when floor(9 m / 3^(j+1)) + o is even.
template <int D, int MODE>
__device__ __forceinline__ void step_high(uint32_t (&c)[2 * D], const Slots<D> &s, const uint32_t *E, uint32_t m,
                                          uint32_t o, Visit<D, MODE> &v) {
  uint32_t q = m;
  int j = 2;
  while (q % 3 == 0) {
    q /= 3;
    ++j;
  }
  const bool rise = (((q / 3) + o) & 1u) == 0;
  const bool use_a = (q % 3 == 1) == rise;  // 0 <-> 1 move: r^s; 1 <-> 2: r
  const uint32_t base = 3u * (static_cast<uint32_t>(s.high >> (kHighBits * (j - 2))) & 0xFFu);
  v.one(flip_elem<D>(c, E, use_a ? base + 2 : base), c);
}

// The package set of rank `rank` in part w (u one-row and td = t - u
// two-row packages): the two-row subset in two[0..td-1], the one-row subset
// in one[0..u-1], as package numbers of the matrix (pm lists the two-row
// packages, then the one-row ones).
__device__ __forceinline__ void unrank_set(unsigned long long rank, const WalkPart &w, int td, int p2, int p1,
                                           const unsigned long long *BN, int ld, const unsigned short *pm,
                                           int (&two)[kWalkMaxT], int (&one)[kWalkMaxT]) {
  int a[kWalkMaxT], b[kWalkMaxT];
  revdoor_unrank(rank % w.c2, td, p2, BN, ld, a);
  revdoor_unrank(rank / w.c2, w.u, p1, BN, ld, b);
#pragma unroll
  for (int k = 0; k < kWalkMaxT; ++k) {
    two[k] = k < td ? pm[a[k]] : -1;
    one[k] = k < w.u ? pm[p2 + b[k]] : -1;
  }
}

// A set's codeword with every digit at value v, and its rows, from scratch.
template <int D>
__device__ __forceinline__ void form_set(const uint32_t *E, const int (&two)[kWalkMaxT],
                                         const int (&one)[kWalkMaxT], int td, int u, int v, bool odd,
                                         Slots<D> &s, uint32_t (&c)[2 * D]) {
#pragma unroll
  for (int i = 0; i < 2 * D; ++i) c[i] = 0;
  s.high = 0;
#pragma unroll
  for (int k = 0; k < kWalkMaxT; ++k) {
    s.pkg[k] = two[k];
    uint32_t e[2 * D];
    if (k < td) {
      if (k >= 2) s.high |= high_field(two[k], k);
      if (k == 0) load_rows<D>(E, two[k], odd, s.x0, s.y0);
      if (k == 1) load_rows<D>(E, two[k], odd, s.x1, s.y1);
      load_elem<D>(E, two[k], v, e);
#pragma unroll
      for (int i = 0; i < 2 * D; ++i) c[i] ^= e[i];
    }
    if (k < u) {
      load_elem<D>(E, one[k], 0, e);
#pragma unroll
      for (int i = 0; i < 2 * D; ++i) c[i] ^= e[i];
    }
  }
}

// One lane's walk over the sets [s0, s1) of part w (s0 <= s1; rw >= s1 - s0
// is the wave's longest range; nstep = 3^td steps per set).  Returns through
// v; `walked` counts the codewords of the lane's sets.
template <int D, int MODE>
__device__ void walk_range(const RoundDesc &p, const WalkPart &w, const uint32_t *E, const unsigned long long *BN,
                           unsigned long long s0, unsigned long long s1, uint32_t rw, int td, uint32_t nstep,
                           Visit<D, MODE> &v, unsigned long long &walked) {
  const int ld = p.t + 1, u = w.u, p2 = p.p2, p1 = p.P - p.p2;
  Slots<D> s;
  uint32_t c[2 * D];
  int two[kWalkMaxT], one[kWalkMaxT];
  unrank_set(s0 < s1 ? s0 : 0ull, w, td, p2, p1, BN, ld, p.pmap, two, one);
#pragma unroll
  for (int i = 0; i < 2 * D; ++i) s.x0[i] = s.y0[i] = s.x1[i] = s.y1[i] = 0;
  form_set<D>(E, two, one, td, u, 0, false, s, c);
  for (uint32_t o = 0; o < rw; ++o) {
    v.live = s0 + o < s1;
    if (o > 0) {
      // Stop early once U meets the bound certified before this round.
      const unsigned long long key = uniform64w(*reinterpret_cast<volatile unsigned long long *>(&p.state->key));
      if (static_cast<int>(key >> 32) <= p.L_before) break;
      swap_rows<D>(s.x0, s.y0);  // the set's digits run the other way
      swap_rows<D>(s.x1, s.y1);
      if (v.live) {
        // Next set: the digits stand where the previous set's walk left
        // them.  Within one one-row subset, consecutive two-row subsets
        // differ by one package out and one in.
        const int vend = ((o - 1) & 1u) == 0 && td > 0 ? 2 : 0;
        const bool odd = (o & 1u) != 0;
        int nt[kWalkMaxT], no[kWalkMaxT];
        unrank_set(s0 + o, w, td, p2, p1, BN, ld, p.pmap, nt, no);
        int out = -1, in = -1, changed = 0;
        bool same_one = true;
#pragma unroll
        for (int k = 0; k < kWalkMaxT; ++k) {
          bool in_new = false, in_old = false;
#pragma unroll
          for (int k2 = 0; k2 < kWalkMaxT; ++k2) {
            in_new = in_new || (k < td && k2 < td && s.pkg[k] == nt[k2]);
            in_old = in_old || (k < td && k2 < td && nt[k] == s.pkg[k2]);
          }
          if (k < td && !in_new) {
            out = s.pkg[k];
            ++changed;
          }
          if (k < td && !in_old) in = nt[k];
          same_one = same_one && (k >= u || one[k] == no[k]);
        }
        if (changed == 1 && same_one && out >= 0 && in >= 0) {
          uint32_t eo[2 * D], ei[2 * D];
          load_elem<D>(E, out, vend, eo);
          load_elem<D>(E, in, vend, ei);
#pragma unroll
          for (int i = 0; i < 2 * D; ++i) c[i] ^= eo[i] ^ ei[i];
#pragma unroll
          for (int k = 0; k < kWalkMaxT; ++k)
            if (k < td && s.pkg[k] == out) {
              s.pkg[k] = in;
              if (k >= 2) s.high = (s.high & ~(0xFFull << (kHighBits * (k - 2)))) | high_field(in, k);
              if (k == 0) load_rows<D>(E, in, odd, s.x0, s.y0);
              if (k == 1) load_rows<D>(E, in, odd, s.x1, s.y1);
            }
        } else {
          form_set<D>(E, nt, no, td, u, vend, odd, s, c);
#pragma unroll
          for (int k = 0; k < kWalkMaxT; ++k) one[k] = no[k];
        }
      }
    }
    v.one(weight_of<D>(c), c);
    if (nstep == 3) {  // td = 1: digit 0 only
      v.one(flip<D>(c, s.x0), c);
      v.one(flip<D>(c, s.y0), c);
    } else if (nstep >= 9) {
      // Blocks k = 0 .. nb - 1 (nb = 3^(td-2) is odd), step 9 (k + 1) after
      // every block but the last.
      const uint32_t nb = nstep / 9;
      uint32_t k = 0;
      for (; k + 1 < nb; k += 2) {
        block8<D, MODE, false>(c, s, v);
        step_high<D, MODE>(c, s, E, k + 1, o, v);
        block8<D, MODE, true>(c, s, v);
        step_high<D, MODE>(c, s, E, k + 2, o, v);
      }
      block8<D, MODE, false>(c, s, v);
    }
    if (v.live) walked += nstep;
    v.end_set();
  }
}

template <int D, int MODE>
__global__ __launch_bounds__(256) void qd_walk_kernel(LaunchParams lp) {
  extern __shared__ unsigned long long smem[];
  const unsigned long long wtile = static_cast<unsigned long long>(blockIdx.x) * kWavesPerGroup;
  if (wtile >= lp.tiles) return;  // whole workgroup: launch padding
  const RoundDesc *const descs = lp.desc;
  const RoundDesc &p = descs[wave_last_le(lp.ndesc, wtile, [descs](int i) { return descs[i].tile_begin; })];
  // The elements and binomials are read with per-lane addresses when a lane
  // unranks or changes sets: stage them in LDS once per workgroup.
  const uint32_t *E = p.elems;
  const unsigned long long *BN = p.binom;
  if (p.stage) {
    unsigned long long *sB = smem;
    const int nb = (p.P + 1) * (p.t + 1);
    uint32_t *sE = reinterpret_cast<uint32_t *>(sB + nb);
    for (int i = threadIdx.x; i < nb; i += blockDim.x) sB[i] = p.binom[i];
    for (int i = threadIdx.x; i < p.P * 3 * kElemWords; i += blockDim.x) sE[i] = p.elems[i];
    __syncthreads();
    E = sE;
    BN = sB;
  }
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const unsigned long long local = wtile + wave - p.tile_begin;  // wave within the piece
  if (local >= p.ntiles) return;                                  // piece padding
  const unsigned long long g = p.tile_lo + local;                 // wave within the round
  DevState *st = p.state;
  unsigned long long key = uniform64w(*reinterpret_cast<volatile unsigned long long *>(&st->key));
  if (static_cast<int>(key >> 32) <= p.L_before) return;  // bound already met

  // The wave's part (sets of u one-row packages) and the lane's sets in it.
  const WalkPart *const parts = p.parts;
  const WalkPart w = parts[wave_last_le(p.nparts, g, [parts](int i) { return parts[i].tile0; })];
  const int td = p.t - w.u;  // digits: two-row packages per set
  const unsigned long long K = p.per_lane;
  unsigned long long s0 = ((g - w.tile0) * kWave + lane) * K;
  s0 = min(s0, w.subsets);
  const unsigned long long s1 = min(s0 + K, w.subsets);
  const uint32_t rw = wave_max_u32(static_cast<uint32_t>(s1 - s0));
  uint32_t nstep = 1;
  for (int i = 0; i < td; ++i) nstep *= 3;

  unsigned long long walked = 0;
  Visit<D, MODE> v;
  walk_range<D, MODE>(p, w, E, BN, s0, s1, rw, td, nstep, v, walked);
  const uint32_t wmin = wave_min_u32(v.best);
  const unsigned long long wsets = wave_sum_u64(walked), wwalked = wsets;
  unsigned long long wsum = 0;
  if constexpr (MODE == kWalkSum) wsum = wave_sum_u64(v.wsum);
  if (lane == 0) {
    unsigned long long *cnt = p.counters + static_cast<size_t>(g % kCountersPerCode) * kCounterStride;
    atomicAdd(cnt, wsets);
    atomicAdd(cnt + 1, wwalked * D);
    if (MODE == kWalkSum && p.wsum) atomicAdd(p.wsum, wsum);
  }

  key = uniform64w(*reinterpret_cast<volatile unsigned long long *>(&st->key));
  if (wmin >= static_cast<uint32_t>(key >> 32)) return;
  // Rare: this wave improves U.  Walk the lanes' ranges again for the first
  // codeword of weight wmin, write it to this wave's slot, then publish
  // (U, slot) with one 64-bit atomicMin.
  Visit<D, kWalkFind> f;
  f.target = wmin;
  unsigned long long fw = 0;
  walk_range<D, kWalkFind>(p, w, E, BN, s0, s1, rw, td, nstep, f, fw);
  const unsigned long long mask = __ballot(f.found);
  if (mask == 0) return;  // the walk stopped early: U already meets the bound
  const int winner = __ffsll(static_cast<long long>(mask)) - 1;
  if (static_cast<int>(lane) == winner) {
    const uint32_t slot = static_cast<uint32_t>(p.slot0 + local);
    uint32_t *out = lp.slots + static_cast<size_t>(slot) * kElemWords;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      out[d] = d < D ? f.fc[d < D ? d : 0] : 0u;
      out[4 + d] = d < D ? f.fc[D + (d < D ? d : 0)] : 0u;
    }
    atomicMin(&st->key, (static_cast<unsigned long long>(wmin) << 32) | slot);
  }
}

}  // namespace

// -- launch (host) -------------------------------------------------------------

hipError_t launch_walk(int D, const LaunchParams &lp, bool sum, hipStream_t s) {
  const unsigned long long wgs = (lp.tiles + kWavesPerGroup - 1) / kWavesPerGroup;
  dim3 grid(static_cast<uint32_t>(wgs)), block(kWave * kWavesPerGroup);
  switch (D * 2 + (sum ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((qd_walk_kernel<1, kWalkMin>), grid, block, lp.lds, s, lp); break;
    case 3: hipLaunchKernelGGL((qd_walk_kernel<1, kWalkSum>), grid, block, lp.lds, s, lp); break;
    case 4: hipLaunchKernelGGL((qd_walk_kernel<2, kWalkMin>), grid, block, lp.lds, s, lp); break;
    case 5: hipLaunchKernelGGL((qd_walk_kernel<2, kWalkSum>), grid, block, lp.lds, s, lp); break;
    case 6: hipLaunchKernelGGL((qd_walk_kernel<3, kWalkMin>), grid, block, lp.lds, s, lp); break;
    case 7: hipLaunchKernelGGL((qd_walk_kernel<3, kWalkSum>), grid, block, lp.lds, s, lp); break;
    case 8: hipLaunchKernelGGL((qd_walk_kernel<4, kWalkMin>), grid, block, lp.lds, s, lp); break;
    case 9: hipLaunchKernelGGL((qd_walk_kernel<4, kWalkSum>), grid, block, lp.lds, s, lp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qd

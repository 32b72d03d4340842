// kernels.hip -- gfx950 kernels of libqdist.
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
#include <hip/hip_runtime.h>

#include "kernels.hpp"

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

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), off)));
  return v;
}

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

// Minimum over one block of kBlock table entries (SoA: word-major).
template <int D>
__device__ __forceinline__ uint32_t block_min(const uint32_t (&ax)[D], const uint32_t (&az)[D],
                                              const uint32_t *__restrict__ blk, uint32_t best) {
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
  // One three-input min per pair of codewords.
#pragma unroll
  for (int e = 0; e < kBlock; e += 2) best = min3(best, w[e], w[e + 1]);
  return best;
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

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), off)));
  return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), off));
  return v;
}

// One tile = one table segment [k0, k0 + seg) x 64 tops.  The tops of a
// tile come from every group whose table prefix reaches the segment, so
// lanes stay full; a lane stops at its own group's prefix length.  A launch
// holds pieces of the current rounds of several codes (RoundDesc).
template <int D>
__global__ __launch_bounds__(256) void qd_round_kernel(LaunchParams lp) {
  extern __shared__ unsigned long long smem[];
  // Consecutive workgroups land on different XCDs; give each XCD a
  // contiguous range of tiles so its L2 sees a contiguous table range.
  const uint32_t per = gridDim.x / 8;
  const uint32_t wg = (blockIdx.x % 8) * per + blockIdx.x / 8;
  const unsigned long long wtile = static_cast<unsigned long long>(wg) * kWavesPerGroup;
  if (wtile >= lp.tiles) return;  // whole workgroup: launch padding
  int lo = 0, hi = lp.ndesc;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (lp.desc[mid].tile_begin <= wtile) lo = mid;
    else hi = mid;
  }
  const RoundDesc &p = lp.desc[lo];

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
    __syncthreads();
  }
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

  lo = 0;
  hi = p.nruns;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (p.runs[mid].tile0 <= g) lo = mid;
    else hi = mid;
  }
  const DevRun &run = p.runs[lo];
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
  if (active) {
    int a = 0, z = static_cast<int>(run.e);
    while (z - a > 1) {
      const int mid = (a + z) >> 1;
      if (GR[mid].cum <= item) a = mid;
      else z = mid;
    }
    lend = min(k1, GR[a].len);
    if (p.tops) {
      const uint4 *tp = reinterpret_cast<const uint4 *>(p.tops + (GR[a].top0 + item - GR[a].cum) * kElemWords);
      const uint4 tx = tp[0], tz = tp[1];
      const uint32_t vx[4] = {tx.x, tx.y, tx.z, tx.w}, vz[4] = {tz.x, tz.y, tz.z, tz.w};
#pragma unroll
      for (int d = 0; d < D; ++d) {
        ax[d] = vx[d];
        az[d] = vz[d];
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
  for (uint32_t i = 0; i < nfull; ++i, blk += 2 * D * kBlock) best = block_min<D>(ax, az, blk, best);
  for (uint32_t i = nfull * kBlock; i < send; ++i) {
    const uint32_t w = weight_at<D>(p.table, k0 + i, ax, az);
    if (i < span) best = min(best, w);
  }
  if (!active) best = 0xFFFFFFFFu;
  const uint32_t wmin = wave_min(best);
  const uint32_t visited = wave_sum(active ? span : 0u);
  if (lane == 0)
    atomicAdd(p.counters + static_cast<size_t>(wg % kCountersPerCode) * kCounterStride,
              static_cast<unsigned long long>(visited));

  key = uniform64(*reinterpret_cast<volatile unsigned long long *>(&st->key));
  if (wmin < static_cast<uint32_t>(key >> 32)) {
    // Rare: this tile improves U.  Find where, write the codeword to this
    // tile's own slot, then publish (U, slot) with one 64-bit atomicMin.
    uint32_t kf = 0xFFFFFFFFu;
    for (uint32_t i = 0; i < send; ++i) {
      const uint32_t w = weight_at<D>(p.table, k0 + i, ax, az);
      if (i < span && w == wmin && kf == 0xFFFFFFFFu) kf = i;
    }
    const unsigned long long mask = __ballot(active && best == wmin);
    const int winner = __ffsll(static_cast<long long>(mask)) - 1;
    if (static_cast<int>(lane) == winner) {
      const uint32_t slot = static_cast<uint32_t>(p.slot0 + local);  // launch-wide slot
      uint32_t *out = lp.slots + static_cast<size_t>(slot) * kElemWords;
      const unsigned long long kk = k0 + kf;
      const uint32_t *e = p.table + (kk / kBlock) * (2 * D * kBlock) + (kk % kBlock);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        out[d] = d < D ? (ax[d] ^ e[d * kBlock]) : 0u;
        out[4 + d] = d < D ? (az[d] ^ e[(D + d) * kBlock]) : 0u;
      }
      atomicMin(&st->key, (static_cast<unsigned long long>(wmin) << 32) | slot);
    }
  }
}

// Saved table: entry k is the k-th bottom combination of u packages in the
// order (largest package, its element, then the rest recursively), so the
// combinations inside packages [0, h) are entries [0, e_u(c_0..c_{h-1})).
// The tops table is the same construction over the packages in reverse
// order: combinations whose smallest package is h are the entries
// [e_u(c_{h+1}..), e_u(c_h..)).  One launch builds several tables; the
// counts E(h, r), r <= u, of a workgroup's table are staged in LDS.
template <int D>
__global__ __launch_bounds__(kBuildGroup) void qd_build_kernel(BuildParams bp) {
  extern __shared__ unsigned long long ecnt[];
  const unsigned long long wfirst = static_cast<unsigned long long>(blockIdx.x) * kBuildGroup;
  if (wfirst >= bp.threads) return;
  int lo = 0, hi = bp.nreq;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (bp.req[mid].first <= wfirst) lo = mid;
    else hi = mid;
  }
  const SavedParams &p = bp.req[lo];
  const int C = p.u + 1;
  // E(h, r): combinations of r packages among the first h (in build order).
  const bool staged = bp.lds >= build_lds_bytes(p.P, p.u);
  if (staged) {
    for (int i = threadIdx.x; i < (p.P + 1) * C; i += blockDim.x) {
      const int h = i / C, r = i % C;
      ecnt[i] = p.tops ? p.suffix[size_t(p.P - h) * p.R + r] : p.prefix[size_t(h) * p.R + r];
    }
    __syncthreads();
  }
  auto E = [&](int h, int r) {
    if (staged) return ecnt[h * C + r];
    return p.tops ? p.suffix[size_t(p.P - h) * p.R + r] : p.prefix[size_t(h) * p.R + r];
  };
  const unsigned long long k = wfirst + threadIdx.x - p.first;
  if (k >= p.nent_padded) return;
  uint32_t x[D], z[D];
#pragma unroll
  for (int d = 0; d < D; ++d) x[d] = z[d] = 0;
  if (k < p.nent) {
    unsigned long long rest = k;
    int hi2 = p.P;
    for (int r = p.u; r > 0; --r) {
      // largest h < hi2 with E(h, r) <= rest (E is nondecreasing in h)
      int a = r - 1, b = hi2 - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (E(mid, r) <= rest) a = mid;
        else b = mid - 1;
      }
      const int h = a;
      rest -= E(h, r);
      const unsigned long long f = E(h, r - 1);
      int c = 0;
      while (rest >= f && c < 2) { rest -= f; ++c; }
      xor_elem<D>(p.elems, p.tops ? p.P - 1 - h : h, c, x, z);
      hi2 = h;
    }
  }
  if (p.tops) {
    uint32_t *e = p.table + k * kElemWords;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      e[d] = d < D ? x[d] : 0u;
      e[4 + d] = d < D ? z[d] : 0u;
    }
  } else {
    uint32_t *b = p.table + (k / kBlock) * (2 * D * kBlock) + (k % kBlock);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      b[d * kBlock] = x[d];
      b[(D + d) * kBlock] = z[d];
    }
  }
}

// After a launch, one workgroup per code (its first piece): moves the
// codeword of the winning slot into the code's state and folds the code's
// spread counters into its visited count.
__global__ __launch_bounds__(256) void qd_commit_kernel(LaunchParams lp) {
  __shared__ unsigned long long part[256];
  const RoundDesc &p = lp.desc[blockIdx.x];
  if (!p.commit) return;  // another piece of the same code commits it
  unsigned long long sum = 0;
  for (int i = threadIdx.x; i < kCountersPerCode; i += blockDim.x) {
    sum += p.counters[static_cast<size_t>(i) * kCounterStride];
    p.counters[static_cast<size_t>(i) * kCounterStride] = 0;
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  DevState *st = p.state;
  st->count += part[0];
  const unsigned long long key = st->key;
  const uint32_t slot = static_cast<uint32_t>(key & 0xFFFFFFFFull);
  if (slot == kNoSlot) return;
#pragma unroll
  for (int w = 0; w < kElemWords; ++w) st->wit[w] = lp.slots[static_cast<size_t>(slot) * kElemWords + w];
  st->key = (key & ~0xFFFFFFFFull) | kNoSlot;
}

__device__ inline unsigned long long esym_step(unsigned long long a, unsigned long long b, unsigned c) {
  // a + c*b, saturating at kEsymSat (c <= 3)
  const unsigned long long cb = b > kEsymSat / 3 ? kEsymSat : min(b * c, kEsymSat);
  return a + cb > kEsymSat ? kEsymSat : a + cb;
}

// Applies a step's block moves: workgroup i handles record i, copying from
// the staging buffer or zero-filling in 16-byte vector stores, or building
// e_r tables (thread r owns column r; one step per package).
__global__ __launch_bounds__(256) void qd_scatter_kernel(const CopyRec *rec, const unsigned char *base) {
  const CopyRec r = rec[blockIdx.x];
  if (r.src == kEsymTables) {
    __shared__ unsigned long long col[64];
    unsigned long long *prefix = static_cast<unsigned long long *>(r.dst);
    unsigned long long *suffix = prefix + static_cast<size_t>(r.P + 1) * r.R;
    const int c = threadIdx.x;
    const bool own = c < r.R;
    for (int pass = 0; pass < 2; ++pass) {
      unsigned long long v = c == 0 ? 1ull : 0ull;
      unsigned long long *out = pass == 0 ? prefix : suffix;
      const int h0 = pass == 0 ? 0 : r.P;
      if (own) out[static_cast<size_t>(h0) * r.R + c] = v;
      for (int i = 0; i < r.P; ++i) {
        if (c < 64) col[c] = v;
        __syncthreads();
        const int h = pass == 0 ? i : r.P - 1 - i;       // package added
        const int row = pass == 0 ? i + 1 : r.P - 1 - i;  // row written
        if (own && c > 0) v = esym_step(v, col[c - 1], base[r.sizes + h]);
        if (own) out[static_cast<size_t>(row) * r.R + c] = v;
        __syncthreads();
      }
    }
    return;
  }
  uint4 *dst = static_cast<uint4 *>(r.dst);
  const unsigned long long n = r.bytes / 16;
  if (r.src == kZeroFill) {
    for (unsigned long long i = threadIdx.x; i < n; i += blockDim.x) dst[i] = make_uint4(0u, 0u, 0u, 0u);
  } else {
    const uint4 *src = reinterpret_cast<const uint4 *>(base + r.src);
    for (unsigned long long i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  }
}

// Integer VALU rate probe: 8 independent XOR / OR / popcount chains per lane.
__global__ __launch_bounds__(256) void qd_valu_kernel(uint32_t seed, uint32_t iters, uint32_t *out) {
  uint32_t a[8], c = seed * 2654435761u + threadIdx.x;
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = c + i * 0x9E3779B9u;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "v"(c));
      asm volatile("v_or_b32 %0, %1, %0" : "+v"(a[i]) : "v"(c));
      asm volatile("v_bcnt_u32_b32 %0, %0, %0" : "+v"(a[i]));
      asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "v"(c));
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) s ^= a[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// -- launch helpers (host) ---------------------------------------------------

hipError_t launch_round(int D, const LaunchParams &lp, hipStream_t s) {
  unsigned long long wgs = lp.tiles / kWavesPerGroup;
  wgs = (wgs + 7) / 8 * 8;
  dim3 grid(static_cast<uint32_t>(wgs)), block(kWave * kWavesPerGroup);
  switch (D) {
    case 1: hipLaunchKernelGGL(qd_round_kernel<1>, grid, block, lp.lds, s, lp); break;
    case 2: hipLaunchKernelGGL(qd_round_kernel<2>, grid, block, lp.lds, s, lp); break;
    case 3: hipLaunchKernelGGL(qd_round_kernel<3>, grid, block, lp.lds, s, lp); break;
    case 4: hipLaunchKernelGGL(qd_round_kernel<4>, grid, block, lp.lds, s, lp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_build(int D, const BuildParams &bp, hipStream_t s) {
  dim3 grid(static_cast<uint32_t>(bp.threads / kBuildGroup)), block(kBuildGroup);
  switch (D) {
    case 1: hipLaunchKernelGGL(qd_build_kernel<1>, grid, block, bp.lds, s, bp); break;
    case 2: hipLaunchKernelGGL(qd_build_kernel<2>, grid, block, bp.lds, s, bp); break;
    case 3: hipLaunchKernelGGL(qd_build_kernel<3>, grid, block, bp.lds, s, bp); break;
    case 4: hipLaunchKernelGGL(qd_build_kernel<4>, grid, block, bp.lds, s, bp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_commit(const LaunchParams &lp, hipStream_t s) {
  hipLaunchKernelGGL(qd_commit_kernel, dim3(lp.ndesc), dim3(256), 0, s, lp);
  return hipGetLastError();
}

hipError_t launch_scatter(const CopyRec *rec, int n, const unsigned char *base, hipStream_t s) {
  hipLaunchKernelGGL(qd_scatter_kernel, dim3(static_cast<uint32_t>(n)), dim3(256), 0, s, rec, base);
  return hipGetLastError();
}

hipError_t launch_valu(uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(qd_valu_kernel, dim3(blocks), dim3(256), 0, s, 12345u, iters, out);
  return hipGetLastError();
}

}  // namespace qd

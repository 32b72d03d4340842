// support.hip -- gfx950 support kernels of libqdist: table builds, the
// per-launch commit, the upload scatter and the VALU rate probe.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"
#include "support.hpp"

namespace qd {

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
  const unsigned long long wfirst = bp.base + static_cast<unsigned long long>(blockIdx.x) * kBuildGroup;
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
  if (k < p.nent && p.src) {
    // The first package in build order and its element, then entry `rest`
    // of the table of depth u - 1 (built by an earlier launch).
    const int r = p.u;
    int a = r - 1, b = p.P - 1;
    while (a < b) {
      const int mid = (a + b + 1) >> 1;
      if (E(mid, r) <= k) a = mid;
      else b = mid - 1;
    }
    unsigned long long rest = k - E(a, r);
    const unsigned long long f = E(a, r - 1);
    int c = 0;
    while (rest >= f && c < 2) { rest -= f; ++c; }
    xor_elem<D>(p.elems, p.tops ? p.P - 1 - a : a, c, x, z);
    if (p.tops) {
      const uint32_t *q = p.src + rest * (2 * D);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        x[d] ^= q[d];
        z[d] ^= q[D + d];
      }
    } else {
      const uint32_t *q = p.src + (rest / kBlock) * (2 * D * kBlock) + (rest % kBlock);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        x[d] ^= q[d * kBlock];
        z[d] ^= q[(D + d) * kBlock];
      }
    }
  } else if (k < p.nent) {
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
    uint32_t *e = p.table + k * (2 * D);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      e[d] = x[d];
      e[D + d] = z[d];
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
// codeword of the winning slot into the code's state, in qubit order, and
// folds the code's spread counters into its visited and evaluated-word
// counts.
// Matrix-core forms of a step's saved tables (ExpandBatch): thread t of a
// table reads entry 16 c + r of chunk c once and writes its four groups of
// K-step s (t = (c mks + s) 16 + r; the fourth of K-step 0 is the bias
// group); each of its four 16-byte stores meets those of the 15
// neighbouring entries in one contiguous 256-byte run.
__global__ __launch_bounds__(256) void qd_expand_kernel(ExpandBatch eb) {
  const unsigned long long wfirst = eb.base + static_cast<unsigned long long>(blockIdx.x) * blockDim.x;
  if (wfirst >= eb.threads) return;
  int lo = 0, hi = eb.nreq;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (eb.req[mid].first <= wfirst) lo = mid;
    else hi = mid;
  }
  const ExpandParams &ep = eb.req[lo];
  const unsigned long long nchunk = (ep.nent + kChunk - 1) / kChunk;
  // A table's threads number 16 per (chunk, K-step): below 2^32 for any
  // table the engine builds (at most 2^29 bytes, 8 bytes per entry or more).
  const uint32_t t = static_cast<uint32_t>(wfirst - ep.first) + threadIdx.x;
  const uint32_t cs = t / kChunk, r = t % kChunk;
  if (cs >= nchunk * ep.mks) return;
  const uint32_t mks = static_cast<uint32_t>(ep.mks);
  const uint32_t c = cs / mks;
  const int s = static_cast<int>(cs - c * mks);
  const int D = ep.D;
  const bool packed = ep.pack && s == D - 2;
  const unsigned long long e = static_cast<unsigned long long>(c) * kChunk + r;
  uint32_t x = 0, z = 0, xl = 0, zl = 0;
  if (e < ep.nent) {
    const uint32_t *b = ep.table + (e / kBlock) * (2 * D * kBlock) + e % kBlock;
    x = b[s * kBlock];
    z = b[(D + s) * kBlock];
    if (packed) {
      xl = b[(D - 1) * kBlock];
      zl = b[(2 * D - 1) * kBlock];
    }
  }
  uint4 *out = ep.mtable + static_cast<size_t>(cs) * kWave + r;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const uint32_t w = group_word(g, packed, x, z, xl, zl);
    uint4 o = {0u, 0u, 0u, 0u};
    if (e < ep.nent && (g < 3 || packed)) {
      o.x = sign_nibbles(w);
      o.y = sign_nibbles(w >> 8);
      o.z = sign_nibbles(w >> 16);
      o.w = sign_nibbles(w >> 24);
    } else if (e < ep.nent && s == 0) {
      o = uint4{kBiasEntry, kBiasEntry, kBiasEntry, kBiasEntry};
    }
    out[g * kChunk] = o;
  }
}

__global__ __launch_bounds__(256) void qd_commit_kernel(LaunchParams lp) {
  __shared__ unsigned long long part[2][256];
  const RoundDesc &p = lp.desc[blockIdx.x];
  if (!p.commit) return;  // another piece of the same code commits it
  unsigned long long sum = 0, words = 0;
  for (int i = threadIdx.x; i < kCountersPerCode; i += blockDim.x) {
    unsigned long long *c = p.counters + static_cast<size_t>(i) * kCounterStride;
    sum += c[0];
    words += c[1];
    c[0] = c[1] = 0;
  }
  part[0][threadIdx.x] = sum;
  part[1][threadIdx.x] = words;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) {
      part[0][threadIdx.x] += part[0][threadIdx.x + w];
      part[1][threadIdx.x] += part[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  DevState *st = p.state;
  const unsigned long long key = st->key;
  const uint32_t slot = static_cast<uint32_t>(key & 0xFFFFFFFFull);
  if (threadIdx.x == 0) {
    st->count += part[0][0];
    st->words += part[1][0];
  }
  if (slot == kNoSlot) return;
  // The slot holds the codeword in the stored qubit order of the matrix of
  // the piece that wrote it (slots are launch tiles; pieces are sorted by
  // their first tile).  Thread q < 128 moves qubit q back: it sits at
  // position inv[q].
  int lo = 0, hi = lp.ndesc;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (lp.desc[mid].slot0 <= slot) lo = mid;
    else hi = mid;
  }
  const RoundDesc &w = lp.desc[lo];
  const uint32_t *src = lp.slots + static_cast<size_t>(slot) * kElemWords;
  const int q = static_cast<int>(threadIdx.x);
  if (!w.inv) {
    if (q < kElemWords) st->wit[q] = src[q];
  } else if (q < 128) {
    const int from = q < w.n ? w.inv[q] : -1;
    const bool bx = from >= 0 && ((src[from >> 5] >> (from & 31)) & 1u);
    const bool bz = from >= 0 && ((src[4 + (from >> 5)] >> (from & 31)) & 1u);
    const unsigned long long mx = __ballot(bx), mz = __ballot(bz);
    if ((q & 63) == 0) {  // lane 0 of waves 0 and 1: qubits 64 (q / 64) .. + 63
      const int wd = 2 * (q >> 6);
      st->wit[wd] = static_cast<uint32_t>(mx);
      st->wit[wd + 1] = static_cast<uint32_t>(mx >> 32);
      st->wit[4 + wd] = static_cast<uint32_t>(mz);
      st->wit[4 + wd + 1] = static_cast<uint32_t>(mz >> 32);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) st->key = (key & ~0xFFFFFFFFull) | kNoSlot;
}

// Lane l gets lane l-1's value, lane 0 gets 0 (DPP wave_shr:1).
__device__ inline unsigned long long from_left_lane(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(v)), 0x138, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(v >> 32)), 0x138, 0xF, 0xF, false);
  return (static_cast<unsigned long long>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
}

__device__ inline unsigned long long esym_step(unsigned long long a, unsigned long long b, unsigned c) {
  // a + c*b, saturating at kEsymSat (c <= 3)
  const unsigned long long cb = b > kEsymSat / 3 ? kEsymSat : min(b * c, kEsymSat);
  return a + cb > kEsymSat ? kEsymSat : a + cb;
}

// Applies a step's block moves: workgroup i handles record i, copying from
// the staging buffer or zero-filling in 16-byte vector stores, or building
// e_r tables: wave 0 builds the prefix table and wave 1 the suffix table;
// lane r owns column r and takes column r-1 from lane r-1 at each package,
// whose size it reads from a register of the wave (lane h mod 64 of word
// h / 64).
__global__ __launch_bounds__(256) void qd_scatter_kernel(const CopyRec *rec, const unsigned char *base) {
  const CopyRec r = rec[blockIdx.x];
  if (r.src == kEsymTables) {
    const int wave = threadIdx.x / kWave, c = threadIdx.x % kWave;
    if (wave >= 2) return;
    uint32_t sz[kMaxEsymPackages / kWave];
#pragma unroll
    for (int q = 0; q < kMaxEsymPackages / kWave; ++q)
      sz[q] = q * kWave + c < r.P ? base[r.sizes + q * kWave + c] : 0u;
    unsigned long long *out = static_cast<unsigned long long *>(r.dst);
    if (wave == 1) out += static_cast<size_t>(r.P + 1) * r.R;  // suffix table
    const bool own = c < r.R;
    unsigned long long v = c == 0 ? 1ull : 0ull;
    if (own) out[static_cast<size_t>(wave == 0 ? 0 : r.P) * r.R + c] = v;
    for (int i = 0; i < r.P; ++i) {
      const int h = wave == 0 ? i : r.P - 1 - i;       // package added
      const int row = wave == 0 ? i + 1 : r.P - 1 - i;  // row written
      const int q = h / kWave;
      const uint32_t word = q == 0 ? sz[0] : q == 1 ? sz[1] : q == 2 ? sz[2] : sz[3];
      const uint32_t size = __builtin_amdgcn_readlane(word, h % kWave);
      const unsigned long long left = from_left_lane(v);
      if (c > 0) v = esym_step(v, left, size);
      if (own) out[static_cast<size_t>(row) * r.R + c] = v;
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

// Issue-rate probe of one instruction mix (see QD_MIX_* in qdist.h): 8
// independent chains per lane, each step three operations; the operands
// that the round kernel reads from SGPRs are either SGPRs or VGPRs here.
template <int MIX>
__global__ __launch_bounds__(256) void qd_mix_kernel(uint32_t seed, uint32_t iters, uint32_t *out) {
  uint32_t a[8], b[8], acc[8];
  const uint32_t t = threadIdx.x * 2654435761u + seed;
  uint32_t s0 = seed * 3u + 1u, s1 = seed * 5u + 7u;  // wavefront-uniform (SGPRs)
  const uint32_t v0 = t ^ 0x1234u, v1 = t ^ 0x9876u;  // per lane (VGPRs)
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = t + i;
    b[i] = t * (i + 3);
    acc[i] = 0;
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (MIX == 0 || MIX == 4) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "s"(s0));
      else if (MIX == 1 || MIX == 3) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(a[i]) : "v"(v0));
      else asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(acc[i]) : "v"(a[i]));
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (MIX == 0) asm volatile("v_bitop3_b32 %0, %1, %2, %0 bitop3:0xde" : "+v"(b[i]) : "v"(a[i]), "s"(s1));
      else if (MIX == 1) asm volatile("v_bitop3_b32 %0, %1, %2, %0 bitop3:0xde" : "+v"(b[i]) : "v"(a[i]), "v"(v1));
      else if (MIX == 2) asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(b[i]) : "v"(acc[i]));
      else if (MIX == 3) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(b[i]) : "v"(a[i]));
      else asm volatile("v_xor_b32 %0, %1, %0" : "+v"(b[i]) : "s"(s1));
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (MIX <= 1) asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(acc[i]) : "v"(b[i]));
      else if (MIX == 2) asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(a[i]) : "v"(b[i]));
      else if (MIX == 3) asm volatile("v_xor_b32 %0, %1, %0" : "+v"(acc[i]) : "v"(b[i]));
      else asm volatile("v_xor_b32 %0, %1, %0" : "+v"(acc[i]) : "s"(s0));
    }
    s0 = __builtin_amdgcn_readfirstlane(s0 + it);
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) r ^= a[i] ^ b[i] ^ acc[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
}

// -- launch helpers (host) ---------------------------------------------------

hipError_t launch_build(int D, const BuildParams &bp_all, hipStream_t s) {
  for (unsigned long long base = 0; base < bp_all.threads; base += kMaxLaunchThreads) {
    BuildParams bp = bp_all;
    bp.base = base;
    const unsigned long long n = std::min(bp_all.threads - base, kMaxLaunchThreads);
    dim3 grid(static_cast<uint32_t>(n / kBuildGroup)), block(kBuildGroup);
    switch (D) {
      case 1: hipLaunchKernelGGL(qd_build_kernel<1>, grid, block, bp.lds, s, bp); break;
      case 2: hipLaunchKernelGGL(qd_build_kernel<2>, grid, block, bp.lds, s, bp); break;
      case 3: hipLaunchKernelGGL(qd_build_kernel<3>, grid, block, bp.lds, s, bp); break;
      case 4: hipLaunchKernelGGL(qd_build_kernel<4>, grid, block, bp.lds, s, bp); break;
      default: return hipErrorInvalidValue;
    }
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  }
  return hipSuccess;
}

hipError_t launch_commit(const LaunchParams &lp, hipStream_t s) {
  hipLaunchKernelGGL(qd_commit_kernel, dim3(lp.ndesc), dim3(256), 0, s, lp);
  return hipGetLastError();
}

hipError_t launch_expand(const ExpandBatch &eb_all, hipStream_t s) {
  for (unsigned long long base = 0; base < eb_all.threads; base += kMaxLaunchThreads) {
    ExpandBatch eb = eb_all;
    eb.base = base;
    const unsigned long long n = std::min(eb_all.threads - base, kMaxLaunchThreads);
    hipLaunchKernelGGL(qd_expand_kernel, dim3(static_cast<uint32_t>(n / 256)), dim3(256), 0, s, eb);
    if (hipGetLastError() != hipSuccess) return hipErrorLaunchFailure;
  }
  return hipSuccess;
}

hipError_t launch_scatter(const CopyRec *rec, int n, const unsigned char *base, hipStream_t s) {
  hipLaunchKernelGGL(qd_scatter_kernel, dim3(static_cast<uint32_t>(n)), dim3(256), 0, s, rec, base);
  return hipGetLastError();
}

hipError_t launch_valu(uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(qd_valu_kernel, dim3(blocks), dim3(256), 0, s, 12345u, iters, out);
  return hipGetLastError();
}

hipError_t launch_mix(int mix, uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s) {
  const dim3 g(blocks), b(256);
  switch (mix) {
    case 0: hipLaunchKernelGGL(qd_mix_kernel<0>, g, b, 0, s, 1u, iters, out); break;
    case 1: hipLaunchKernelGGL(qd_mix_kernel<1>, g, b, 0, s, 1u, iters, out); break;
    case 2: hipLaunchKernelGGL(qd_mix_kernel<2>, g, b, 0, s, 1u, iters, out); break;
    case 3: hipLaunchKernelGGL(qd_mix_kernel<3>, g, b, 0, s, 1u, iters, out); break;
    case 4: hipLaunchKernelGGL(qd_mix_kernel<4>, g, b, 0, s, 1u, iters, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace qd

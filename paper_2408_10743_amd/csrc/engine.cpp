// engine.cpp -- step executor: device memory, per-code rounds, batched
// launches of the enumeration kernel, commit and readback.
#include "engine.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace qd {

hipError_t launch_round(int D, const LaunchParams &lp, bool census, bool every_word, int mfma, hipStream_t s);
hipError_t launch_expand(const ExpandBatch &eb, hipStream_t s);
hipError_t launch_walk(int D, const LaunchParams &lp, bool sum, hipStream_t s);
hipError_t launch_build(int D, const BuildParams &bp, hipStream_t s);
hipError_t launch_commit(const LaunchParams &lp, hipStream_t s);
hipError_t launch_scatter(const CopyRec *rec, int n, const unsigned char *base, hipStream_t s);

namespace {

constexpr int kDefaultSavedDepth = 4;                     // packages per saved-table entry
constexpr unsigned long long kMaxTableBytes = 1ull << 29;
constexpr unsigned long long kMaxTopEntries = 1ull << 24;  // at most 512 MB of tops (D = 4)
constexpr unsigned long long kTilesPerLaunch = 1ull << 22;
constexpr unsigned long long kTargetTiles = 1ull << 18;    // ~32 tiles per wave slot
constexpr unsigned kMinSeg = 1024, kMaxSeg = 4096;
// Rounds below kShortRound combinations of a step with few codes start from
// kShortSeg entries per tile: such a step is bound by each tile's chain of
// dependent table loads, so shorter tiles finish sooner.
constexpr unsigned long long kShortRound = 1ull << 24;
constexpr unsigned kShortSeg = 64;
// Rounds of at least this many combinations get the matrix-core form of
// their saved table (smaller ones stay on the vector ALU).
constexpr unsigned long long kMfmaMinRound = 1ull << 20;
// Partial weights for codes whose planned work reaches this many combinations.
constexpr double kPartialMinWork = 1e8;
constexpr unsigned kStageMaxBytes = 32768;
// Rounds of a code are grouped into one step while the step's total stays
// below the executor's limit (kSpecCombos unless set_spec_combos changed it).
constexpr unsigned long long kSpecCombos = 1ull << 36;
// Combinations a step may add past the planner's distance estimate, so that
// a low estimate costs small codes no extra step: at most kSpecExtraRatio
// times the work the estimate needed, and at most kSpecExtra.
constexpr unsigned long long kSpecExtra = 1ull << 24;
constexpr unsigned long long kSpecExtraRatio = 16;
// Rounds up to this size skip the saved and tops tables: every lane unranks
// its whole combination (no table-build launch for small codes).
constexpr unsigned long long kTinyRound = 1ull << 19;
// With a cancel flag, a code's step carries at most this many tiles (a long
// round then spans several steps, and the flag is seen between them).
constexpr unsigned long long kCancelTilesPerStep = 1ull << 15;
// Plain walk: waves per round the automatic choice of package sets per
// lane aims at, and the most sets a lane takes.
constexpr unsigned long long kWalkWaves = 1ull << 15;
constexpr unsigned long long kWalkMaxPerLane = 64;
constexpr int kWalkMaxOption = 4096;
// Staged offsets per round descriptor: groups, runs, binomials, walk package
// map and walk parts.
constexpr size_t kStagedPerDesc = 5;
// Tables of at least this many entries are built from the next smaller
// one of their kind.
constexpr unsigned long long kExtendMinEntries = 1ull << 17;
constexpr size_t kBigClass = size_t(64) << 20;
constexpr size_t kSlabMax = size_t(16) << 20;   // largest class carved from slabs
constexpr size_t kSlabBytes = size_t(64) << 20;

static_assert(kEsymSat == kSat, "device e_r tables saturate like the host's");

size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t size_class(size_t b) {
  size_t c = 256;
  while (c < b && c < kBigClass) c <<= 1;
  if (b > c) c = (b + kBigClass - 1) / kBigClass * kBigClass;
  return c;
}

void to_words(const BRow &r, uint32_t *w) {
  w[0] = uint32_t(r.x[0]); w[1] = uint32_t(r.x[0] >> 32);
  w[2] = uint32_t(r.x[1]); w[3] = uint32_t(r.x[1] >> 32);
  w[4] = uint32_t(r.z[0]); w[5] = uint32_t(r.z[0] >> 32);
  w[6] = uint32_t(r.z[1]); w[7] = uint32_t(r.z[1] >> 32);
}

BRow from_words(const uint32_t *w) {
  BRow r;
  r.x[0] = uint64_t(w[0]) | (uint64_t(w[1]) << 32);
  r.x[1] = uint64_t(w[2]) | (uint64_t(w[3]) << 32);
  r.z[0] = uint64_t(w[4]) | (uint64_t(w[5]) << 32);
  r.z[1] = uint64_t(w[6]) | (uint64_t(w[7]) << 32);
  return r;
}

bool in_span(const std::vector<BRow> &basis, int n, const BRow &v) {
  std::vector<BRow> rows = basis;
  const int k = make_basis(rows, n);
  rows.push_back(v);
  return make_basis(rows, n) == k;
}

// Saved-table depth for round t: u = t-2, so every top keeps two packages
// (a group then fills many lanes), within the cap and the table-size limit.
int saved_depth(const GammaDev &g, int D, int t, int cap, unsigned long long max_bytes) {
  int u = std::min(std::max(t - 2, 0), cap);
  while (u > 0 && g.prefix[size_t(g.P) * g.R + u] * 8ull * D > max_bytes) --u;
  return u;
}

// Table entries per tile: long enough to amortize a tile's setup, short
// enough that the round gives its share (1/sharing) of about kTargetTiles
// tiles per step, where `sharing` codes run their rounds in the same steps.
// Partial-weight rounds on the matrix cores aim at 1 / 2^kPartialMfmaFewer of
// the tiles: their chunks, tails included, cost a few MFMAs each, so a
// tile's setup is the largest cost beside them (config 3 to exact d: 2.0
// against 1.9 ms for a quarter of the tiles, the same for an eighth).
constexpr int kPartialMfmaFewer = 2;
unsigned choose_seg(unsigned long long planned, int sharing, unsigned long_seg, int fewer = 0) {
  const unsigned long long target =
      std::max<unsigned long long>(kTargetTiles / std::max(sharing, 1), 1024) >> fewer;
  const unsigned long long want = planned / (kWave * target);
  // Large rounds start from long_seg entries, and every round of a step
  // with many codes (their number fills the device) from kMinSeg: the
  // per-tile setup then costs a few % at most.
  unsigned seg = sharing > 8 ? kMinSeg : planned < kShortRound ? kShortSeg : long_seg;
  while (seg < want && seg < kMaxSeg) seg <<= 1;
  return seg;
}

// Tiles of one round.  Group h pairs the tops whose smallest package is h
// (c_h * e_{t-u-1}(c_{h+1}..)) with the first e_u(c_0..c_{h-1}) table
// entries.  Segment s of the table is shared by every group reaching it,
// so its tiles take 64 tops at a time from those groups together.
// With `scalar` (packages are F4 scalar orbits) group h keeps only the tops
// whose element of package h is element 0 (r): h is the smallest package of
// the top, so this picks one codeword of each class {c, alpha c, alpha^2 c}.
unsigned long long plan_round(const GammaDev &g, int t, int u, unsigned seg, bool scalar,
                              std::vector<DevGroup> &groups, std::vector<DevRun> &runs) {
  groups.clear();
  runs.clear();
  const int R = g.R, r = t - u - 1;
  for (int h = 0; h < g.P; ++h) {
    const unsigned long long items = g.suffix[size_t(h + 1) * R + r] * (scalar ? 1 : g.sizes[h]);
    const unsigned long long len = g.prefix[size_t(h) * R + u];
    if (!items || !len) continue;
    DevGroup grp{};
    grp.items = items;
    grp.len = len;
    grp.top0 = g.suffix[size_t(h + 1) * R + (t - u)];
    grp.f = g.suffix[size_t(h + 1) * R + r];
    grp.h = h;
    groups.push_back(grp);
  }
  std::stable_sort(groups.begin(), groups.end(), [](const DevGroup &a, const DevGroup &b) { return a.len > b.len; });
  unsigned long long cum = 0, tiles = 0;
  std::vector<unsigned long long> ns(groups.size());
  for (size_t i = 0; i < groups.size(); ++i) {
    groups[i].cum = cum;
    cum += groups[i].items;
    ns[i] = (groups[i].len + seg - 1) / seg;
  }
  // Segments [ns[e], ns[e-1]) are reached by exactly the e longest groups.
  const size_t G = groups.size();
  for (size_t e = G; e >= 1; --e) {
    const unsigned long long sa = e == G ? 0 : ns[e], sb = ns[e - 1];
    if (sa >= sb) continue;
    DevRun run{};
    run.tile0 = tiles;
    run.s_begin = sa;
    run.e = static_cast<long long>(e);
    run.items = e == G ? cum : groups[e].cum;
    run.tps = (run.items + kWave - 1) / kWave;
    tiles += (sb - sa) * run.tps;
    runs.push_back(run);
  }
  return tiles;
}

// Partial-weight rounds on the matrix cores: the depth u <= deepest that
// costs least, counting the bytes its tables take to write, the saved
// table (8D bytes per entry) with its expanded K-step 0 (64 bytes per
// entry) and the tops table (8D bytes per entry; tops over t - u >= 2
// packages read the table one package shallower), at the builds' rate, and
// the tiles of the round at a tile's setup cost (shallow tables leave many
// short groups, each a tile per 64 tops).  Among the depths whose tops fit
// a table.  The deepest table's expanded form alone can cost more than a
// tenth of the round.
constexpr double kBuildBytesPerS = 4e12;  // table builds and expansions, measured 3.8-4.4 TB/s
constexpr double kTileSetupS = 0.65e-9;   // ~350 VALU instructions per tile on 1024 SIMDs at 2.1 GHz
int partial_mfma_depth(const GammaDev &g, int D, int t, int deepest, unsigned long long max_tops, unsigned seg,
                       bool scalar) {
  int best = deepest;
  double least = -1.0;
  std::vector<DevGroup> hg;
  std::vector<DevRun> hr;
  for (int u = 1; u <= deepest; ++u) {
    const unsigned long long tops = g.suffix[size_t(t - u >= 2 ? t - u - 1 : t - u)];  // the table built
    if (tops > max_tops) continue;
    const double bytes = double(g.prefix[size_t(g.P) * g.R + u]) * (8.0 * D + double(kWave * sizeof(uint4)) / kChunk) +
                         double(tops) * (8.0 * D);
    const double cost = bytes / kBuildBytesPerS + double(plan_round(g, t, u, seg, scalar, hg, hr)) * kTileSetupS;
    if (least < 0 || cost < least) {
      least = cost;
      best = u;
    }
  }
  return best;
}

}  // namespace

unsigned rule_seg(unsigned long long planned, int sharing) { return choose_seg(planned, sharing, kMinSeg); }
int rule_depth_cap() { return kDefaultSavedDepth; }

// -- DevPool -------------------------------------------------------------------

DevPool::~DevPool() {
  for (void *p : all_) (void)hipFree(p);
}

// Classes up to kSlabMax are carved from slabs of kSlabBytes (or 8
// blocks), so a batch of small codes costs few hipMalloc calls; larger
// classes are allocations of their own.
void *DevPool::get(size_t bytes, size_t *cls) {
  if (arena_) {
    const size_t c = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
    if (c > arena_cap_ - arena_off_) return nullptr;
    void *p = arena_ + arena_off_;
    arena_off_ += c;
    *cls = c;
    return p;
  }
  const size_t c = size_class(std::max<size_t>(bytes, 1));
  auto &v = free_[c];
  if (v.empty()) {
    const size_t slab = c <= kSlabMax ? std::max(kSlabBytes, 8 * c) : c;
    void *p = nullptr;
    const double tm = now_ms();
    ++mallocs_;
    const hipError_t me = hipMalloc(&p, slab);
    malloc_ms_ += now_ms() - tm;
    if (me != hipSuccess) {
      (void)hipGetLastError();  // the failed allocation must not fail a later launch check
      // Give cached blocks of the large classes back to the driver and try
      // once more (slab blocks stay: their slab may be partly in use).
      for (auto &kv : free_) {
        if (kv.first <= kSlabMax) continue;
        for (void *q : kv.second) {
          (void)hipFree(q);
          all_.erase(std::find(all_.begin(), all_.end(), q));
          held_ -= kv.first;
        }
        kv.second.clear();
      }
      if (hipMalloc(&p, slab) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    all_.push_back(p);
    held_ += slab;
    for (size_t off = slab; off >= c; off -= c) v.push_back(static_cast<char *>(p) + (off - c));
  }
  void *p = v.back();
  v.pop_back();
  *cls = c;
  return p;
}

void DevPool::put(void *p, size_t cls) {
  if (p && !arena_) free_[cls].push_back(p);
}

// -- Staging -------------------------------------------------------------------

Staging::~Staging() {
  if (p_ && pageable_) std::free(p_);
  else if (p_) (void)hipHostFree(p_);
}

size_t Staging::put(const void *src, size_t bytes) {
  const size_t off = align16(n_), end = align16(off + bytes);
  if (end > cap_) {
    size_t cap = std::max<size_t>(cap_ ? 2 * cap_ : size_t(1) << 20, end);
    unsigned char *q = nullptr;
    if (pageable_) {
      q = static_cast<unsigned char *>(std::malloc(cap));
      if (!q) return SIZE_MAX;
    } else if (hipHostMalloc(reinterpret_cast<void **>(&q), cap, hipHostMallocDefault) != hipSuccess) {
      return SIZE_MAX;
    }
    if (n_) std::memcpy(q, p_, n_);
    if (p_ && pageable_) std::free(p_);
    else if (p_) (void)hipHostFree(p_);
    p_ = q;
    cap_ = cap;
  }
  std::memset(p_ + n_, 0, off - n_);
  if (bytes) std::memcpy(p_ + off, src, bytes);
  std::memset(p_ + off + bytes, 0, end - off - bytes);
  n_ = end;
  return off;
}

// -- Executor ------------------------------------------------------------------

Executor::Executor(hipStream_t stream, void *arena, size_t bytes)
    : mfma_min_round_(kMfmaMinRound), spec_combos_(kSpecCombos), long_seg_(kMinSeg), stream_(stream),
      max_table_bytes_(bytes / 4) {
  if (!arena) return;  // the caller has checked the device (a gfx950 holding the arena)
  pool_.set_arena(arena, bytes);
  staging_.set_pageable();
  // The arena keeps the last call's contents: the zero table is cleared here.
  const size_t zb = size_t(2) * 4 * kBlock * sizeof(uint32_t);
  size_t cls = 0;
  zero_table_ = static_cast<uint32_t *>(pool_.get(zb, &cls));
  if (!zero_table_ || hipMemsetAsync(zero_table_, 0, zb, stream_) != hipSuccess) return;
  ok_ = grow_states(64) == QD_OK;
}

Executor::Executor(hipStream_t stream)
    : mfma_min_round_(kMfmaMinRound), spec_combos_(kSpecCombos), long_seg_(kMinSeg),
      max_table_bytes_(kMaxTableBytes) {
  int dev = 0, cnt = 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0 || hipGetDevice(&dev) != hipSuccess ||
      hipGetDeviceProperties(&prop, dev) != hipSuccess || !std::strstr(prop.gcnArchName, "gfx950"))
    return;
  if (stream) {
    stream_ = stream;
  } else {
    if (hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess) return;
    own_stream_ = true;
  }
  // Depth 0 needs no build: one block of kBlock zero entries of up to 4 words per half.
  const size_t zb = size_t(2) * 4 * kBlock * sizeof(uint32_t);
  if (hipMalloc(reinterpret_cast<void **>(&zero_table_), zb) != hipSuccess) return;
  if (hipMemset(zero_table_, 0, zb) != hipSuccess) return;
  mtable_budget_ = prop.totalGlobalMem / 4;
  ok_ = grow_states(64) == QD_OK;
}

Executor::~Executor() {
  if (!pool_.arena()) {
    if (zero_table_) (void)hipFree(zero_table_);
    if (states_) (void)hipFree(states_);
    if (hstates_) (void)hipHostFree(hstates_);
  }
  for (hipEvent_t e : events_) (void)hipEventDestroy(e);
  if (own_stream_) (void)hipStreamDestroy(stream_);
}

bool Executor::alloc(PoolBuf &b, size_t bytes) {
  if (b.p && b.cls >= bytes) {
    b.bytes = bytes;
    return true;
  }
  release(b);
  b.p = pool_.get(bytes, &b.cls);
  b.bytes = bytes;
  return b.p != nullptr;
}

void Executor::release(PoolBuf &b) {
  if (b.p) pool_.put(b.p, b.cls);
  b = PoolBuf{};
}

int Executor::grow_states(int need) {
  if (nstates_ >= need) return QD_OK;
  const int cap = std::max(need, 2 * nstates_);
  DevState *d = nullptr, *h = nullptr;
  if (pool_.arena()) {  // fixed at construction: one state array in the arena
    size_t cls = 0;
    if (states_ || !(d = static_cast<DevState *>(pool_.get(sizeof(DevState) * cap, &cls)))) return QD_ERR_NOMEM;
    host_states_.assign(size_t(cap), DevState{});
    for (int i = cap - 1; i >= 0; --i) free_slots_.push_back(i);
    states_ = d;
    hstates_ = host_states_.data();
    nstates_ = cap;
    return QD_OK;
  }
  if (hipMalloc(reinterpret_cast<void **>(&d), sizeof(DevState) * cap) != hipSuccess) return QD_ERR_NOMEM;
  if (hipHostMalloc(reinterpret_cast<void **>(&h), sizeof(DevState) * cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(d);
    return QD_ERR_NOMEM;
  }
  std::memset(h, 0, sizeof(DevState) * cap);
  if (states_) {
    if (hipStreamSynchronize(stream_) != hipSuccess ||
        hipMemcpy(d, states_, sizeof(DevState) * nstates_, hipMemcpyDeviceToDevice) != hipSuccess)
      return QD_ERR_DEVICE;
    std::memcpy(h, hstates_, sizeof(DevState) * nstates_);
    (void)hipFree(states_);
    (void)hipHostFree(hstates_);
  }
  for (int i = cap - 1; i >= nstates_; --i) free_slots_.push_back(i);
  states_ = d;
  hstates_ = h;
  nstates_ = cap;
  return QD_OK;
}

void Executor::prepare(Job &job) {
  job.t0 = now_ms();
  qd_options &o = job.opt;
  std::memset(&job.S, 0, sizeof(job.S));
  if (o.resume) {  // the caller's memory is read here only
    const qd_resume &r = *o.resume;
    job.has_resume = true;
    job.r_t = r.t;
    job.r_j = r.j;
    job.r_U = r.U;
    job.r_structure = r.structure;
    if (r.witness) job.r_wit.assign(r.witness, r.witness + 2 * size_t(std::max(job.n, 0)));
    o.resume = nullptr;
  }
  if (o.diag != QD_DIAG_AUTO && o.diag != QD_DIAG_F2 && o.diag != QD_DIAG_F4 && o.diag != QD_DIAG_ISO) {
    job.status = QD_ERR_INVALID;
    return;
  }
  if (o.seg_len < 0 || o.seg_len % kBlock || o.saved_depth < -1 || o.max_gamma < 0 || o.tops_mode < 0 ||
      o.tops_mode > 2 || (o.filter != QD_FILTER_NONE && o.filter != QD_FILTER_STABILIZER) ||
      (o.scalar_classes != 0 && o.scalar_classes != -1) || (o.partial_weight < -1 || o.partial_weight > 1) ||
      (o.mixed_packages < -1 || o.mixed_packages > 1) || o.walk < 0 || o.walk > kWalkMaxOption ||
      (o.walk > 0 && o.filter != QD_FILTER_NONE) || (o.matrix_cores != 0 && o.matrix_cores != -1)) {
    job.status = QD_ERR_INVALID;
    return;
  }
  if (o.walk > 0) {
    // The plain walk enumerates every codeword of the paper's constructions
    // in the matrices' own qubit order.
    o.scalar_classes = -1;
    o.mixed_packages = -1;
    o.partial_weight = -1;
  }
  int rc = load_rows(job.G.data(), job.m, job.n, job.field, job.basis);
  if (rc) { job.status = rc; return; }
  const int n = job.n;
  job.rank = make_basis(job.basis, n);
  if (job.rank == 0) { job.status = QD_ERR_ZERO_CODE; return; }
  // Modified BZ: with no logical pair the span is self-orthogonal (k = 0)
  // and every codeword counts.
  if (o.filter == QD_FILTER_STABILIZER) logical_pairs(job.basis, job.logicals);
  if (job.use.empty()) {
    std::vector<Gamma> f4 = build_f4(job.basis, n, kMaxGamma);
    Gamma f2 = build_f2(job.basis, n);
    for (const Gamma &g : f4)
      if (!check_gamma(g, n)) { job.status = QD_ERR_INTERNAL; return; }
    if (!check_gamma(f2, n)) { job.status = QD_ERR_INTERNAL; return; }
    std::vector<Gamma> iso;
    const bool f4_linear = job.field == QD_FIELD_F4 || alpha_closed(job.basis, n);
    const bool f4_scalar = o.scalar_classes == 0 && f4_linear;
    job.pc = choose_plan(f4, f2, iso, n, job.rank, o.diag == QD_DIAG_ISO ? QD_DIAG_AUTO : o.diag, o.max_gamma,
                         f4_scalar);
    // Mixed packages for additive codes with unused qubits (scalar classes
    // need every package to have two rows).
    if (o.mixed_packages >= 0 && !f4_linear && job.rank < n && o.diag != QD_DIAG_F2 && o.diag != QD_DIAG_ISO &&
        (o.mixed_packages == 1 || job.pc.predicted_f4 >= kMixMinWork)) {
      if (!try_mixed_f4(job.basis, n, job.rank, job.pc.d_est, o.max_gamma, f4, job.caps)) {
        job.status = QD_ERR_INTERNAL;
        return;
      }
      if (!job.caps.empty())
        job.pc = choose_plan(f4, f2, iso, n, job.rank, o.diag == QD_DIAG_ISO ? QD_DIAG_AUTO : o.diag, o.max_gamma,
                             f4_scalar);
    }
    // The isometry matrices are built only when asked for, or when they
    // might beat the other constructions' predicted work.
    if (o.diag == QD_DIAG_ISO ||
        (o.diag == QD_DIAG_AUTO && job.pc.predicted >= kIsoMinWork &&
         iso_work_floor(n, job.rank, job.pc.d_est) < kIsoMargin * job.pc.predicted)) {
      iso = build_iso(job.basis, n, kMaxGamma);
      for (const Gamma &g : iso)
        if (!check_gamma_iso(g, n)) { job.status = QD_ERR_INTERNAL; return; }
      job.pc = choose_plan(f4, f2, iso, n, job.rank, o.diag, o.max_gamma, f4_scalar);
    }
    if (job.pc.diag == QD_DIAG_F2) job.use.push_back(f2);
    else if (job.pc.diag == QD_DIAG_ISO) job.use.assign(iso.begin(), iso.begin() + job.pc.h_used);
    else job.use.assign(f4.begin(), f4.begin() + job.pc.h_used);
    job.halve = job.pc.diag == QD_DIAG_ISO;
    if (f4_scalar && job.pc.diag == QD_DIAG_F4) job.scalar = make_scalar_orbits(job.use);
  }
  prepare_gammas(job);
}

void Executor::prepare_gammas(Job &job) {
  const int n = job.n;
  const int h = int(job.use.size());
  job.D = (n + 31) / 32;
  job.S.n = n; job.S.rank = job.rank; job.S.D = job.D; job.S.diag = job.pc.diag; job.S.h = h;
  job.S.d_estimate = job.pc.d_est; job.S.predicted = job.pc.predicted;
  job.S.logical_pairs = int(job.logicals.size() / 2);
  job.S.scalar_classes = job.scalar ? 1 : 0;
  for (int j = 0; j < QD_MAX_GAMMA; ++j)
    job.S.two_row_cap[j] = job.pc.diag == QD_DIAG_F4 && j < int(job.caps.size()) ? job.caps[j] : -1;
  job.tdone.assign(h, 0);
  job.delta.resize(h);
  for (int j = 0; j < h; ++j) {
    job.S.P[j] = job.use[j].P();
    job.S.delta[j] = job.delta[j] = job.use[j].delta;
  }
  job.L = lower_bound(job.tdone, job.delta, job.halve);
  job.U = n + 1;
  job.gd.assign(h, GammaDev{});
  // Partial weights need a second word, and pay only for codes with enough
  // work to outweigh reordering the matrices; with them off the qubit order
  // stays.
  job.partial = job.D >= 2 && (job.opt.partial_weight == 1 ||
                               (job.opt.partial_weight == 0 && job.pc.predicted >= kPartialMinWork));
  // Matrix cores: the last word goes into a spare group when it is short.
  // One word per half costs the vector ALU 5 operations per codeword, less
  // than a K-step of 128 signs on the matrix cores.
  job.mfma = job.opt.matrix_cores == 0 && job.opt.walk == 0 && job.D >= 2;
  job.mpack = job.D >= 3 && n - 32 * (job.D - 1) <= kMaxPackedQubits ? 1 : 0;
  job.mks = job.D - job.mpack;
  for (int j = 0; j < h; ++j) {
    GammaDev &g = job.gd[j];
    const Gamma &gm = job.use[j];
    g.P = gm.P();
    g.R = std::min(g.P, kTMax) + 1;
    g.delta = gm.delta;
    if (job.partial) g.order = qubit_order(gm, n, job.halve);
    g.h_elems.assign(size_t(g.P) * 3 * kElemWords, 0);
    g.h_csize.assign(g.P, 0);
    for (int i = 0; i < g.P; ++i) {
      const Package &p = gm.pk[i];
      to_words(permute_row(p.r, g.order), &g.h_elems[size_t(3 * i) * kElemWords]);
      if (p.dim == 2) {
        BRow rs = p.r;
        radd(rs, p.s);
        to_words(permute_row(p.s, g.order), &g.h_elems[size_t(3 * i + 1) * kElemWords]);
        to_words(permute_row(rs, g.order), &g.h_elems[size_t(3 * i + 2) * kElemWords]);
      }
      g.h_csize[i] = p.dim == 2 ? 3 : 1;
      g.sizes.push_back(g.h_csize[i]);
    }
    esym_tables(g.sizes, g.R - 1, g.prefix, g.suffix);
  }
  // FNV-1a over the matrices: construction, and every package's dimension,
  // pivot and rows.
  unsigned long long hsh = 14695981039346656037ull;
  auto mix = [&hsh](unsigned long long v) {
    for (int b = 0; b < 8; ++b) {
      hsh ^= (v >> (8 * b)) & 0xFF;
      hsh *= 1099511628211ull;
    }
  };
  mix(static_cast<unsigned long long>(job.pc.diag));
  mix(job.halve ? 1 : 0);
  mix(job.scalar ? 1 : 0);
  for (const Gamma &gm : job.use) {
    mix(gm.pk.size());
    mix(static_cast<unsigned long long>(gm.delta));
    for (const Package &p : gm.pk) {
      mix(static_cast<unsigned long long>(p.dim));
      mix(static_cast<unsigned long long>(static_cast<long long>(p.pivot)));
      for (int w = 0; w < 2; ++w) {
        mix(p.r.x[w]);
        mix(p.r.z[w]);
        mix(p.s.x[w]);
        mix(p.s.z[w]);
      }
    }
  }
  job.S.structure = hsh;
  if (job.has_resume) apply_resume(job);
}

// Starts a job at the resume point of an earlier call on the same matrices:
// rounds before (t, j) count as run, U and its witness as found.
void Executor::apply_resume(Job &job) {
  const int n = job.n, h = int(job.use.size());
  bool ok = job.r_structure == job.S.structure && job.r_j >= 0 && job.r_j < h && job.r_t >= 1 &&
            job.r_t <= kTMax + 1 && job.r_U >= 1 && job.r_U <= n + 1;
  BRow w;
  if (ok && job.r_U <= n) {
    ok = job.r_wit.size() == 2 * size_t(n);
    for (int q = 0; ok && q < n; ++q) {
      if (job.r_wit[q] > 1 || job.r_wit[n + q] > 1) ok = false;
      if (job.r_wit[q]) w.x[q >> 6] |= 1ull << (q & 63);
      if (job.r_wit[n + q]) w.z[q >> 6] |= 1ull << (q & 63);
    }
    ok = ok && rweight(w) == job.r_U && in_span(job.basis, n, w);
  }
  if (!ok) {
    job.status = QD_ERR_INVALID;
    return;
  }
  job.t = job.r_t;
  job.j = job.r_j;
  for (int jj = 0; jj < h; ++jj) job.tdone[jj] = std::min(job.use[jj].P(), jj < job.r_j ? job.r_t : job.r_t - 1);
  job.L = lower_bound(job.tdone, job.delta, job.halve);
  job.U = job.r_U;
  if (job.r_U <= n) job.wit = w;
  if (job.L >= job.U) job.done = true;
}

size_t Executor::footprint(const Job &job) {
  size_t b = size_t(kCountersPerCode) * kCounterStride * 8 + 64 * 1024;
  for (const GammaDev &g : job.gd) {
    b += g.h_elems.size() * 4 + g.prefix.size() * 16 + g.P;
    for (int u = 0; u <= std::min(kDefaultSavedDepth, g.R - 1); ++u)
      b += size_t(std::min<uint64_t>(g.prefix[size_t(g.P) * g.R + u] * 8ull * job.D, kMaxTableBytes));
    for (int k = 1; k <= std::min(3, g.R - 1); ++k)
      b += size_t(std::min<uint64_t>(g.suffix[k], kMaxTopEntries) * 8ull * job.D);
  }
  return b;
}

// Waits for the last flush's copy so the staging buffer can be reused.
int Executor::settle() {
  if (!inflight_) return QD_OK;
  inflight_ = false;
  staging_.clear();
  return hipStreamSynchronize(inflight_stream_) == hipSuccess ? QD_OK : QD_ERR_DEVICE;
}

// Takes a state slot and one data block for the job and stages their
// contents; they reach the device with the next step's flush.
int Executor::admit(Job &job, hipStream_t s) {
  (void)s;
  if (job.status) return job.status;
  if (const int rc = settle()) return rc;
  if (free_slots_.empty() && grow_states(nstates_ + 64) != QD_OK) return QD_ERR_NOMEM;
  job.state_slot = free_slots_.back();
  free_slots_.pop_back();
  DevState &hs = hstates_[job.state_slot];
  std::memset(&hs, 0, sizeof(hs));
  hs.key = (static_cast<unsigned long long>(job.U) << 32) | kNoSlot;  // n + 1, or a resumed U
  dirty_slots_.push_back(job.state_slot);
  // Block layout: counters | per Gamma_j elements, sizes, qubit order and
  // logical operators (both in its stored order), each 16-byte aligned as
  // Staging::put places them | per Gamma_j prefix and suffix tables, which
  // the device computes from the sizes.
  const size_t cb = size_t(kCountersPerCode) * kCounterStride * 8;
  const size_t lbytes = job.logicals.size() * kElemWords * 4;
  size_t a_bytes = 0, total = cb;
  for (const GammaDev &g : job.gd) {
    if (g.R > kWave || g.P > kMaxEsymPackages) return QD_ERR_INTERNAL;
    const size_t ga = align16(g.h_elems.size() * 4) + align16(g.h_csize.size()) + align16(g.order.pos.size()) +
                      align16(lbytes);
    a_bytes += ga;
    total += ga + 2 * g.prefix.size() * 8;
  }
  if (!alloc(job.data, total)) return QD_ERR_NOMEM;
  unsigned char *dev = static_cast<unsigned char *>(job.data.p);
  recs_.push_back({dev, kZeroFill, cb, 0, 0, 0});
  const size_t o0 = align16(staging_.size());
  unsigned char *a0 = dev + cb, *b = dev + cb + a_bytes;
  std::vector<uint32_t> lw(job.logicals.size() * kElemWords);
  for (GammaDev &g : job.gd) {
    const size_t oe = staging_.put(g.h_elems.data(), g.h_elems.size() * 4);
    const size_t oc = staging_.put(g.h_csize.data(), g.h_csize.size());
    if (oe == SIZE_MAX || oc == SIZE_MAX) return QD_ERR_NOMEM;
    g.elems = reinterpret_cast<const uint32_t *>(a0 + (oe - o0));
    g.csize = a0 + (oc - o0);
    if (!g.order.pos.empty()) {
      const size_t op = staging_.put(g.order.pos.data(), g.order.pos.size());
      if (op == SIZE_MAX) return QD_ERR_NOMEM;
      g.inv = a0 + (op - o0);
    }
    if (lbytes) {
      for (size_t i = 0; i < job.logicals.size(); ++i)
        to_words(permute_row(job.logicals[i], g.order), &lw[i * kElemWords]);
      const size_t ol = staging_.put(lw.data(), lbytes);
      if (ol == SIZE_MAX) return QD_ERR_NOMEM;
      g.logicals = reinterpret_cast<const uint32_t *>(a0 + (ol - o0));
    }
    g.dprefix = reinterpret_cast<const unsigned long long *>(b);
    g.dsuffix = g.dprefix + g.prefix.size();
    recs_.push_back({b, kEsymTables, 0, oc, g.P, g.R});
    b += 2 * g.prefix.size() * 8;
  }
  if (staging_.size() - o0 != a_bytes || size_t(b - dev) != total) return QD_ERR_INTERNAL;
  if (a_bytes) recs_.push_back({a0, o0, a_bytes, 0, 0, 0});
  job.S.host_ms = now_ms() - job.t0;
  return QD_OK;
}

// Queues the build of a table (saved bottoms of u packages, or with
// tops = true the u-package tops) for the next flush; the buffer is
// allocated now.
int Executor::ensure_table(Job &job, GammaDev &g, int u, bool tops) {
  PoolBuf &buf = tops ? g.tops[u] : g.table[u];
  if (buf.p) return QD_OK;
  const unsigned long long nent = tops ? g.suffix[u] : g.prefix[size_t(g.P) * g.R + u];
  // A large table is built from the one of its kind of depth u - 1 (queued
  // first if it is not there yet): one element XOR one smaller entry
  // instead of unranking u packages.
  int *levels = tops ? g.tops_level : g.table_level;
  const uint32_t *src = nullptr;
  int level = 0;
  if (u >= 2 && nent >= kExtendMinEntries) {
    if (const int rc = ensure_table(job, g, u - 1, tops)) return rc;
    src = static_cast<const uint32_t *>((tops ? g.tops : g.table)[u - 1].p);
    level = levels[u - 1] + 1;  // 0 when it was built by an earlier step
  }
  const unsigned long long padded = (nent + kBuildGroup - 1) / kBuildGroup * kBuildGroup;
  if (!alloc(buf, size_t(padded) * 2 * job.D * 4)) return QD_ERR_NOMEM;  // 2D words per entry, either kind
  SavedParams sp{};
  sp.elems = g.elems;
  sp.prefix = g.dprefix;
  sp.suffix = g.dsuffix;
  sp.csize = g.csize;
  sp.table = static_cast<uint32_t *>(buf.p);
  sp.nent = nent;
  sp.nent_padded = padded;
  sp.first = 0;
  sp.P = g.P;
  sp.R = g.R;
  sp.u = u;
  sp.tops = tops ? 1 : 0;
  sp.src = src;
  sp.level = level;
  levels[u] = level;
  level_marks_.push_back(&levels[u]);
  builds_[job.D].push_back(sp);
  return QD_OK;
}

void Executor::release_mtable(GammaDev &g, int u) {
  if (g.mtable[u].p) mtable_held_ -= std::min(mtable_held_, g.mtable[u].cls);
  release(g.mtable[u]);
  g.mtable_ks[u] = 0;
}

// Device tables of a job (none in flight).
void Executor::release_tables(Job &job) {
  for (GammaDev &g : job.gd)
    for (int u = 0; u <= kTMax; ++u) {
      release(g.table[u]);
      release(g.tops[u]);
      release_mtable(g, u);
    }
}

// Queues the matrix-core form of saved table u (built or queued) with mks
// K-steps per chunk for the next flush, after the table builds.
// Without room (the executor's budget for these copies, or device memory)
// the table keeps no such form and its rounds stay on the vector ALU.
int Executor::ensure_mtable(Job &job, GammaDev &g, int u, int mks) {
  if (g.mtable[u].p && g.mtable_ks[u] >= mks) return QD_OK;
  const unsigned long long nent = g.prefix[size_t(g.P) * g.R + u];
  const unsigned long long chunks = (nent + kChunk - 1) / kChunk + kMtablePadChunks;
  const size_t bytes = size_t(chunks) * mks * kWave * sizeof(uint4);
  release_mtable(g, u);
  if (mtable_held_ + bytes > mtable_budget_ || !alloc(g.mtable[u], bytes)) {
    release_mtable(g, u);
    return QD_OK;
  }
  mtable_held_ += g.mtable[u].cls;
  g.mtable_ks[u] = mks;
  ExpandParams ep;
  ep.table = static_cast<const uint32_t *>(g.table[u].p);
  ep.mtable = static_cast<uint4 *>(g.mtable[u].p);
  ep.nent = nent;
  ep.D = job.D;
  ep.mks = mks;
  ep.pack = job.mpack;
  expands_.push_back(ep);
  return QD_OK;
}

// Sends everything staged since the last step to the device in one copy:
// state resets and job data (applied by one scatter launch), each piece's
// groups and runs, the round descriptors (read in place; *desc_off is
// their offset) and the queued table builds, which it launches, one
// launch per word count D.  *base is the device copy of the staged bytes.
int Executor::flush(hipStream_t s, const unsigned char **base, size_t *desc_off) {
  *base = nullptr;
  for (int slot : dirty_slots_) {
    const size_t off = staging_.put(&hstates_[slot], sizeof(DevState));
    if (off == SIZE_MAX) return QD_ERR_NOMEM;
    recs_.push_back({states_ + slot, off, sizeof(DevState), 0, 0, 0});
  }
  dirty_slots_.clear();
  // One build launch per (wave, word count D): a table built from a smaller
  // one goes in a later wave than its source.
  std::vector<SavedParams> bl;
  struct BuildRange {
    int D;
    size_t b0, b1;
  };
  std::vector<BuildRange> ranges;
  int waves = 0;
  for (int D = 1; D <= 4; ++D)
    for (const SavedParams &sp : builds_[D]) waves = std::max(waves, sp.level + 1);
  for (int lv = 0; lv < waves; ++lv)
    for (int D = 1; D <= 4; ++D) {
      const size_t b0 = bl.size();
      unsigned long long first = 0;
      for (SavedParams sp : builds_[D]) {
        if (sp.level != lv) continue;
        sp.first = first;
        first += sp.nent_padded;
        bl.push_back(sp);
      }
      if (bl.size() > b0) ranges.push_back({D, b0, bl.size()});
    }
  for (int D = 1; D <= 4; ++D) builds_[D].clear();
  for (int *m : level_marks_) *m = -1;
  level_marks_.clear();
  if (staging_.size() == 0 && descs_.empty() && bl.empty() && recs_.empty() && expands_.empty()) return QD_OK;
  unsigned long long ex_threads = 0;
  for (ExpandParams &ep : expands_) {
    ep.first = ex_threads;
    ex_threads += expand_threads(ep.nent, ep.mks);
  }
  const size_t need = staging_.size() + align16(descs_.size() * sizeof(RoundDesc)) +
                      align16(bl.size() * sizeof(SavedParams)) + align16(recs_.size() * sizeof(CopyRec)) +
                      align16(expands_.size() * sizeof(ExpandParams));
  if (!alloc(stage_dev_, need)) return QD_ERR_NOMEM;
  const unsigned char *dev = static_cast<const unsigned char *>(stage_dev_.p);
  for (size_t i = 0; i < descs_.size(); ++i) {
    const size_t *o = &desc_groups_[kStagedPerDesc * i];
    descs_[i].groups = reinterpret_cast<const DevGroup *>(dev + o[0]);
    descs_[i].runs = reinterpret_cast<const DevRun *>(dev + o[1]);
    descs_[i].binom = reinterpret_cast<const unsigned long long *>(dev + o[2]);
    descs_[i].pmap = reinterpret_cast<const unsigned short *>(dev + o[3]);
    descs_[i].parts = reinterpret_cast<const WalkPart *>(dev + o[4]);
  }
  const size_t doff = staging_.put(descs_.data(), descs_.size() * sizeof(RoundDesc));
  const size_t boff = staging_.put(bl.data(), bl.size() * sizeof(SavedParams));
  const size_t roff = staging_.put(recs_.data(), recs_.size() * sizeof(CopyRec));
  const size_t eoff = staging_.put(expands_.data(), expands_.size() * sizeof(ExpandParams));
  if (doff == SIZE_MAX || boff == SIZE_MAX || roff == SIZE_MAX || eoff == SIZE_MAX) return QD_ERR_NOMEM;
  if (staging_.size() != need) return QD_ERR_INTERNAL;
  if (hipMemcpyAsync(stage_dev_.p, staging_.data(), need, hipMemcpyHostToDevice, s) != hipSuccess)
    return QD_ERR_DEVICE;
  inflight_ = true;
  inflight_stream_ = s;
  if (!recs_.empty() &&
      launch_scatter(reinterpret_cast<const CopyRec *>(dev + roff), int(recs_.size()), dev, s) != hipSuccess)
    return QD_ERR_DEVICE;
  recs_.clear();
  for (const BuildRange &r : ranges) {
    BuildParams bp;
    bp.req = reinterpret_cast<const SavedParams *>(dev + boff) + r.b0;
    bp.nreq = int(r.b1 - r.b0);
    bp.threads = 0;
    unsigned lds = 0;
    for (size_t i = r.b0; i < r.b1; ++i) {
      bp.threads += bl[i].nent_padded;
      lds = std::max(lds, build_lds_bytes(bl[i].P, bl[i].u));
    }
    bp.lds = lds <= kStageMaxBytes ? lds : 0u;
    if (launch_build(r.D, bp, s) != hipSuccess) return QD_ERR_DEVICE;
  }
  if (!expands_.empty()) {
    ExpandBatch eb;
    eb.req = reinterpret_cast<const ExpandParams *>(dev + eoff);
    eb.nreq = int(expands_.size());
    eb.threads = ex_threads;
    eb.base = 0;
    if (launch_expand(eb, s) != hipSuccess) return QD_ERR_DEVICE;
  }
  expands_.clear();
  *base = dev;
  *desc_off = doff;
  return QD_OK;
}

// Schedules the next rounds of a job with nothing in flight: consecutive
// rounds are grouped into one step while their total work stays small
// (about a microsecond of device time), so short codes need few steps.  A
// round scheduled speculatively only adds codewords: the bounds are still
// applied in round order when the step retires.
int Executor::schedule(Job &job, int sharing) {
  const int h = int(job.use.size());
  unsigned long long cum = 0;
  // Speculation: rounds are added while the scheduled ones would not yet
  // certify the planner's distance estimate, then (the estimate may be
  // low) only while the extra rounds stay cheap, and never past a bound
  // that meets the current upper bound.
  std::vector<int> tsim = job.tdone;
  const int stop_at = std::min(job.U, std::max(job.pc.d_est, 1));
  bool beyond = lower_bound(tsim, job.delta, job.halve) >= stop_at;
  unsigned long long extra = 0, extra_cap = 0;
  auto cap_extra = [&](unsigned long long needed) {
    extra_cap = std::min<unsigned long long>(kSpecExtra, kSpecExtraRatio * std::max<unsigned long long>(needed, 1));
  };
  if (beyond) cap_extra(job.planned_total);
  for (;;) {
    if (!job.single_round) {
      bool found = false;
      for (;;) {
        if (job.j >= h) { job.j = 0; ++job.t; }
        bool any = false;
        for (int j = 0; j < h; ++j) any = any || job.t <= job.use[j].P();
        if (!any) break;
        if (job.t > job.use[job.j].P()) { ++job.j; continue; }
        found = true;
        break;
      }
      if (!found) {
        if (job.fl.empty()) job.done = true;  // every round ran: nothing left to certify
        return QD_OK;
      }
    }
    GammaDev &g = job.gd[job.j];
    const int t = job.t;
    const uint64_t full = g.prefix[size_t(g.P) * g.R + t];
    const uint64_t planned = job.scalar && full < kSat ? full / 3 : full;  // e_t(3,..,3) = 3^t C(P, t)
    if (t > kTMax || (job.opt.cancel && *job.opt.cancel) || planned >= kSat ||
        (job.opt.budget && job.planned_total + cum + planned > job.opt.budget)) {
      if (job.fl.empty()) job.incomplete = job.done = true;
      return QD_OK;
    }
    if (beyond && !job.fl.empty()) {
      if (extra + planned > extra_cap) return QD_OK;
      extra += planned;
    }
    if (job.opt.walk > 0) {
      // Plain walk: this round alone in the step, in one launch.
      if (t > kWalkMaxT) {
        if (job.fl.empty()) job.incomplete = job.done = true;
        return QD_OK;
      }
      Flight f;
      f.t = t;
      f.j = job.j;
      f.walk = true;
      f.use_tops = false;
      f.L_before = job.single_round ? -1 : lower_bound(tsim, job.delta, job.halve);
      const size_t ld = size_t(t) + 1;
      f.binom.assign(size_t(g.P + 1) * ld, 0);
      for (int p = 0; p <= g.P; ++p)
        for (int r = 0; r <= t; ++r)
          f.binom[p * ld + r] = r == 0 ? 1 : p == 0 ? 0 : f.binom[(p - 1) * ld + r] + f.binom[(p - 1) * ld + r - 1];
      // Package map: the two-row packages, then the one-row ones.
      for (int i = 0; i < g.P; ++i)
        if (g.sizes[i] == 3) f.pmap.push_back(static_cast<unsigned short>(i));
      f.p2 = int(f.pmap.size());
      for (int i = 0; i < g.P; ++i)
        if (g.sizes[i] != 3) f.pmap.push_back(static_cast<unsigned short>(i));
      const int p1 = g.P - f.p2;
      auto C = [&](int n, int r) { return r < 0 || r > n ? 0ull : f.binom[size_t(n) * ld + r]; };
      const unsigned long long sets = f.binom[size_t(g.P) * ld + t];
      f.per_lane = job.opt.walk >= 2
                       ? static_cast<unsigned long long>(job.opt.walk)
                       : std::min(kWalkMaxPerLane, std::max<unsigned long long>(1, sets / (kWave * kWalkWaves)));
      // Part u: sets of u one-row and t - u two-row packages.
      f.tiles = 0;
      for (int u = std::max(0, t - f.p2); u <= std::min(t, p1); ++u) {
        WalkPart w{};
        w.tile0 = f.tiles;
        w.c2 = C(f.p2, t - u);
        w.subsets = C(p1, u) * w.c2;
        w.u = u;
        if (!w.subsets) continue;
        f.parts.push_back(w);
        f.tiles += (w.subsets + kWave * f.per_lane - 1) / (kWave * f.per_lane);
      }
      f.planned = planned;
      job.fl.push_back(std::move(f));
      ++job.j;
      return QD_OK;
    }
    Flight f;
    f.t = t;
    f.j = job.j;
    // The bound certified once the rounds before this one have finished; they
    // are in this step or earlier, so the round's waves may stop as soon as U
    // reaches it.
    f.L_before = job.single_round ? -1 : lower_bound(tsim, job.delta, job.halve);
    // A measured shape for this bucket, unless the caller fixed one.
    unsigned tseg = 0;
    int tdepth = 0;
    const bool tuned = tuned_ && !job.opt.seg_len && !job.opt.saved_depth &&
                       tune_lookup(job.D, planned, sharing, job.partial || job.force_words > 0 ? 1 : 0, &tseg, &tdepth);
    const int cap = job.opt.saved_depth < 0 ? 0
                    : job.opt.saved_depth   ? job.opt.saved_depth
                    : tuned                 ? tdepth
                                            : kDefaultSavedDepth;
    f.u = saved_depth(g, job.D, t, cap, max_table_bytes_);
    f.seg = job.opt.seg_len ? unsigned(job.opt.seg_len) : tuned ? tseg : choose_seg(planned, sharing, long_seg_);
    const int tm = job.opt.tops_mode;
    const unsigned long long max_tops = std::min(kMaxTopEntries, max_table_bytes_ / (8ull * job.D));
    const bool expanded = planned >= mfma_min_round_ && job.mfma && !arena() && !job.force_words &&
                          job.census_below == 0;  // the saved table gets its matrix-core form
    if (expanded && job.partial && !tuned && !job.opt.seg_len)
      f.seg = choose_seg(planned, sharing, long_seg_, kPartialMfmaFewer);
    if (expanded && job.partial && !tuned && job.opt.saved_depth == 0 && tm == 0 && planned > kTinyRound)
      f.u = partial_mfma_depth(g, job.D, t, f.u, max_tops, f.seg, job.scalar);
    f.tops_down = t - f.u >= 2;
    const int tops_depth = f.tops_down ? t - f.u - 1 : t - f.u;
    f.use_tops = tm == 1 || (tm == 0 && g.suffix[tops_depth] <= max_tops);
    if (planned <= kTinyRound && job.opt.saved_depth == 0 && tm == 0) {
      f.u = 0;
      f.use_tops = false;
    }
    int rc = f.u > 0 ? ensure_table(job, g, f.u, false) : QD_OK;
    if (!rc && f.use_tops) rc = ensure_table(job, g, tops_depth, true);
    if (!rc && f.u > 0 && expanded) rc = ensure_mtable(job, g, f.u, job.partial ? 1 : job.mks);
    if (rc) return rc;
    f.tiles = plan_round(g, t, f.u, f.seg, job.scalar, f.hg, f.hr);
    f.planned = planned;
    const int fj = f.j;
    job.fl.push_back(std::move(f));
    cum += planned;
    ++job.j;
    tsim[fj] = t;
    const int Lsim = lower_bound(tsim, job.delta, job.halve);
    if (job.single_round || cum >= spec_combos_ || t == job.use[fj].P() || Lsim >= job.U) return QD_OK;
    if (!beyond && Lsim >= stop_at) {
      beyond = true;
      cap_extra(job.planned_total + cum);
    }
  }
}

void Executor::drop_flights(Job &job) { job.fl.clear(); }

// Retires one finished round (in order): bounds, witness, log, stop test.
void Executor::end_round(Job &job, Flight &f) {
  const DevState &hs = hstates_[job.state_slot];
  const int Ud = int(hs.key >> 32);
  if (Ud < job.U) {
    job.U = Ud;
    job.wit = from_words(hs.wit);
  }
  // Visited combinations are counted per code; a step's count is given to
  // its rounds in order, each at most its planned size.
  const unsigned long long this_round = std::min<unsigned long long>(hs.count - job.visited, f.planned);
  job.visited += this_round;
  job.S.enumerated = hs.count;
  job.S.words = hs.words;
  job.planned_total += f.planned;
  job.tdone[f.j] = f.t;
  job.L = lower_bound(job.tdone, job.delta, job.halve);
  qd_stats &S = job.S;
  S.kernel_ms += f.ms;
  if (S.nlog < QD_MAX_LOG) {
    qd_round_log &lg = S.log[S.nlog];
    lg.t = f.t; lg.j = f.j; lg.L = job.L; lg.U = job.U; lg.saved_depth = f.u;
    lg.launches = f.launches; lg.combinations = this_round; lg.planned = f.planned;
    lg.kernel_ms = f.ms;
  }
  ++S.nlog;
  if (job.single_round || job.L >= job.U || f.t == job.use[f.j].P()) job.done = true;
}

int Executor::step(std::vector<Job *> &jobs, hipStream_t s) {
  // QD_TRACE=1 prints one line per step to stderr (launches, pieces,
  // tiles, host and device time).
  static const bool trace = std::getenv("QD_TRACE") && std::getenv("QD_TRACE")[0] == '1';
  const double ts0 = trace ? now_ms() : 0.0;
  if (const int rc = settle()) return rc;
  int sharing = 0;
  for (Job *jp : jobs) sharing += !jp->done && !jp->status;
  // A code cancelled with rounds still in flight stops before the first of
  // them; U and its witness are the best the device has found so far.
  for (Job *jp : jobs) {
    Job &job = *jp;
    if (job.done || job.status || job.fl.empty() || !job.opt.cancel || !*job.opt.cancel) continue;
    const DevState &hs = hstates_[job.state_slot];
    if (int(hs.key >> 32) < job.U) {
      job.U = int(hs.key >> 32);
      job.wit = from_words(hs.wit);
    }
    job.t = job.fl[0].t;
    job.j = job.fl[0].j;
    drop_flights(job);
    job.done = true;
    job.incomplete = job.L < job.U;  // a U found mid-round may already meet L
  }
  for (Job *jp : jobs) {
    if (jp->done || !jp->fl.empty() || jp->status) continue;
    const int rc = schedule(*jp, sharing);
    if (rc) { jp->status = rc; jp->done = true; }
  }
  const double ts_sched = trace ? now_ms() : 0.0;
  struct Launch {
    int D;
    bool walk, sum;  // plain walk kernel; with the weight sum
    bool every_word; // no piece uses partial weights (entry-major kernel)
    bool mfma;       // every code of the launch may use the matrix cores
    bool packed, plain;  // some piece with the packed / plain K-step layout
    bool any_mtable;     // some piece with the matrix-core form
    size_t d0, d1;
    unsigned long long tiles;
    unsigned lds;
    bool timed;
  };
  struct Member {
    Job *job;
    size_t flight;
  };
  std::vector<Launch> launches;
  std::vector<Member> members;  // job and flight of each descriptor
  descs_.clear();
  desc_groups_.clear();
  unsigned long long max_tiles = 0;
  // One launch per word count D for the saved-sum kernel, then per D for
  // the codes on the plain walk.
  // A piece goes to the matrix-core launch of its word count unless it is a
  // large round whose table has no matrix-core form (no room for one): those
  // get a launch of the vector-ALU kernel of their own, so the others keep
  // the matrix cores.  A code may then have pieces in both launches; each
  // launch commits it after its own pieces.
  auto matrix_class = [&](const Job &job, const Flight &f) {
    if (f.walk || !job.mfma || job.force_words || job.census_below > 0 || arena()) return false;
    if (f.u == 0) return true;
    const int need_ks = job.partial ? 1 : job.mks;
    return job.gd[f.j].mtable_ks[f.u] >= need_ks || f.planned < mfma_min_round_;
  };
  std::vector<unsigned long long> tiles_left(jobs.size());  // tiles each code may still send this step
  for (size_t i = 0; i < jobs.size(); ++i) tiles_left[i] = jobs[i]->opt.cancel ? kCancelTilesPerStep : ~0ull;
  for (int kind = 0; kind < 16; ++kind) {
    const int D = kind % 4 + 1;
    const bool walk = (kind / 4) % 2 == 1;
    const bool mclass = kind >= 8;
    if (walk && mclass) continue;
    Launch L{D, walk, false, true, mclass && !arena(), false, false, false, descs_.size(), 0, 0, 0, false};
    for (size_t ji = 0; ji < jobs.size(); ++ji) {
      Job *jp = jobs[ji];
      Job &job = *jp;
      if (job.done || job.D != D || job.status || (job.opt.walk > 0) != walk) continue;
      bool first = true;  // the first piece of the code in this launch commits it
      unsigned long long &job_left = tiles_left[ji];
      for (size_t fi = 0; fi < job.fl.size(); ++fi) {
        Flight &f = job.fl[fi];
        if (matrix_class(job, f) != mclass) continue;
        const unsigned long long left = f.tiles - f.sent;
        const unsigned long long take =
            std::min({left, kTilesPerLaunch - std::min(kTilesPerLaunch, L.tiles), job_left});
        job_left -= take;
        if (take == 0) continue;
        GammaDev &g = job.gd[f.j];
        RoundDesc d{};
        d.elems = g.elems;
        d.table = f.u == 0 ? zero_table_ : static_cast<const uint32_t *>(g.table[f.u].p);
        d.tops = f.use_tops ? static_cast<const uint32_t *>(g.tops[f.t - f.u - (f.tops_down ? 1 : 0)].p) : nullptr;
        d.tops_down = f.use_tops && f.tops_down ? 1 : 0;
        // The matrix-core form, when it holds the K-steps the piece needs.
        const int need_ks = job.partial ? 1 : job.mks;
        d.mtable = f.u > 0 && g.mtable_ks[f.u] >= need_ks ? static_cast<const uint4 *>(g.mtable[f.u].p) : nullptr;
        d.mks = g.mtable_ks[f.u];
        d.mpack = job.mpack;
        // A large round without the matrix-core form (no room for it) needs
        // the vector-ALU kernel; small rounds run its streaming loop anywhere.
        if (f.u > 0 && !d.mtable && f.planned >= mfma_min_round_) L.mfma = false;
        if (d.mtable) L.any_mtable = true;
        if (d.mtable) (job.mpack ? L.packed : L.plain) = true;
        // groups and runs travel with this step's upload (set by flush)
        const size_t go = staging_.put(f.hg.data(), f.hg.size() * sizeof(DevGroup));
        const size_t ro = staging_.put(f.hr.data(), f.hr.size() * sizeof(DevRun));
        const size_t bo = staging_.put(f.binom.data(), f.binom.size() * sizeof(unsigned long long));
        const size_t mo = staging_.put(f.pmap.data(), f.pmap.size() * sizeof(unsigned short));
        const size_t po = staging_.put(f.parts.data(), f.parts.size() * sizeof(WalkPart));
        if (go == SIZE_MAX || ro == SIZE_MAX || bo == SIZE_MAX || mo == SIZE_MAX || po == SIZE_MAX)
          return QD_ERR_NOMEM;
        for (size_t off : {go, ro, bo, mo, po}) desc_groups_.push_back(off);
        d.suffix = g.dsuffix;
        d.csize = g.csize;
        d.state = states_ + job.state_slot;
        d.counters = static_cast<unsigned long long *>(job.data.p);
        d.logicals = g.logicals;
        d.nlogicals = int(job.logicals.size());
        d.inv = g.inv;
        d.n = job.n;
        for (int w = 1; w <= 3; ++w) {
          if (job.force_words) {  // qd_round_min: w words first in every tile
            d.credit[w - 1] = 0;
            d.cap[w - 1] = w == job.force_words && w < job.D ? job.n + 1 : -1;
            continue;
          }
          // Words 0..w-1 hold min(32 w, nonpivot) qubits without pivots.
          const int q = std::min(32 * w, g.order.nonpivot);
          const bool on = job.partial && w < job.D && partial_limit(q) >= 0;
          d.credit[w - 1] = on ? partial_credit(f.t, g.delta, g.order.kin[w - 1], job.halve) : 0;
          d.cap[w - 1] = on ? partial_limit(q) + d.credit[w - 1] : -1;
        }
        d.tile_begin = L.tiles;
        d.ntiles = take;
        d.tile_lo = f.sent;
        d.slot0 = L.tiles;
        d.ngroups = int(f.hg.size());
        d.nruns = int(f.hr.size());
        d.P = g.P;
        d.R = g.R;
        d.t = f.t;
        d.u = f.u;
        d.seg = f.seg;
        d.L_before = f.L_before;
        d.stage = f.use_tops ? 1 : 2;
        d.commit = first ? 1 : 0;
        if (first) ++job.S.launches;
        first = false;
        unsigned lds = round_lds_bytes(d.P, d.t, d.u, d.ngroups, d.stage);
        if (f.walk) {
          d.per_lane = f.per_lane;
          d.nparts = int(f.parts.size());
          d.p2 = f.p2;
          d.wsum = job.want_wsum ? d.counters + 2 : nullptr;  // word 2 of the first counter line
          L.sum = L.sum || job.want_wsum;
          d.stage = 1;
          lds = walk_lds_bytes(d.P, d.t);
        } else if (job.census_below > 0) {
          d.census = d.counters + 3;  // words 3 and 4 of the first counter line
          d.below = job.census_below;
          L.sum = true;
        }
        if (lds > kStageMaxBytes) { d.stage = 0; lds = 0; }
        L.lds = std::max(L.lds, lds);
        L.timed = L.timed || job.opt.timing;
        L.every_word = L.every_word && !job.partial && !job.force_words;
        L.mfma = L.mfma && job.mfma && !job.force_words && job.census_below == 0;
        L.tiles += (take + kWavesPerGroup - 1) / kWavesPerGroup * kWavesPerGroup;
        f.sent += take;
        ++f.launches;
        descs_.push_back(d);
        members.push_back({jp, fi});
      }
    }
    L.d1 = descs_.size();
    L.mfma = L.mfma && L.any_mtable;  // only small rounds: the vector-ALU kernel
    if (L.d1 > L.d0) {
      launches.push_back(L);
      max_tiles = std::max(max_tiles, L.tiles);
    }
  }
  const unsigned char *base = nullptr;
  size_t desc_off = 0;
  const double ts_desc = trace ? now_ms() : 0.0;
  // The witness slots first: a step that cannot get them fails before it
  // uploads or builds anything.
  if (!launches.empty() && !alloc(slots_, size_t(max_tiles) * kElemWords * 4)) return QD_ERR_NOMEM;
  if (const int rc = flush(s, &base, &desc_off)) return rc;
  const double ts_flush = trace ? now_ms() : 0.0;
  if (!launches.empty()) {
    bool any_timed = false;  // events are created only for timed launches
    for (const Launch &L : launches) any_timed = any_timed || L.timed;
    while (any_timed && events_.size() < 2 * launches.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return QD_ERR_DEVICE;
      events_.push_back(e);
    }
    for (size_t i = 0; i < launches.size(); ++i) {
      const Launch &L = launches[i];
      LaunchParams lp;
      lp.desc = reinterpret_cast<const RoundDesc *>(base + desc_off) + L.d0;
      lp.ndesc = int(L.d1 - L.d0);
      lp.lds = L.lds;
      lp.tiles = L.tiles;
      lp.slots = static_cast<uint32_t *>(slots_.p);
      if (L.mfma && !L.walk)
        for (size_t d = L.d0; d < L.d1; ++d)
          if (descs_[d].commit) ++members[d].job->S.matrix_core_launches;
      if (L.timed && hipEventRecord(events_[2 * i], s) != hipSuccess) return QD_ERR_DEVICE;
      if ((L.walk ? launch_walk(L.D, lp, L.sum, s) : launch_round(L.D, lp, L.sum, L.every_word, !L.mfma ? 0 : L.packed && L.plain ? 1 : L.packed ? 2 : 3, s)) != hipSuccess) return QD_ERR_DEVICE;
      if (L.timed && hipEventRecord(events_[2 * i + 1], s) != hipSuccess) return QD_ERR_DEVICE;
      if (launch_commit(lp, s) != hipSuccess) return QD_ERR_DEVICE;
    }
  }
  const double ts1 = trace ? now_ms() : 0.0;
  if (hipMemcpyAsync(hstates_, states_, sizeof(DevState) * nstates_, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return QD_ERR_DEVICE;
  inflight_ = false;
  staging_.clear();
  if (trace) {
    std::fprintf(stderr,
                 "qd step: jobs %d host %.3f ms (schedule %.3f pieces %.3f flush %.3f launch %.3f; hipMalloc %d in "
                 "%.3f ms so far) wait %.3f ms",
                 sharing, ts1 - ts0, ts_sched - ts0, ts_desc - ts_sched, ts_flush - ts_desc, ts1 - ts_flush,
                 pool_.mallocs(), pool_.malloc_ms(), now_ms() - ts1);
    for (const Launch &L : launches)
      std::fprintf(stderr, " | D%d pieces %zu tiles %llu", L.D, L.d1 - L.d0, L.tiles);
    std::fprintf(stderr, "\n");
  }
  for (size_t i = 0; i < launches.size(); ++i) {
    const Launch &L = launches[i];
    if (!L.timed) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, events_[2 * i], events_[2 * i + 1]) != hipSuccess) return QD_ERR_DEVICE;
    // A launch's time is shared by its pieces in proportion to their tiles.
    for (size_t d = L.d0; d < L.d1; ++d) {
      const float share = ms * float(descs_[d].ntiles) / float(L.tiles);
      members[d].job->fl[members[d].flight].ms += share;
      members[d].job->S.enumerated_kernel_ms += share;
    }
  }
  for (Job *jp : jobs) {
    Job &job = *jp;
    if (job.done || job.status) continue;
    size_t k = 0;
    while (k < job.fl.size() && job.fl[k].sent == job.fl[k].tiles && !job.done) {
      end_round(job, job.fl[k]);
      ++k;
    }
    job.fl.erase(job.fl.begin(), job.fl.begin() + long(k));
    if (job.done) {
      drop_flights(job);
      release_tables(job);  // other codes of the batch may use the memory
    }
  }
  return QD_OK;
}

void Executor::retire(Job &job) {
  const double t1 = now_ms();
  // Uploads staged for a job that never reached a step still target its
  // memory: apply them before that memory can be handed to another job.
  if (!recs_.empty() || !dirty_slots_.empty()) {
    const unsigned char *base = nullptr;
    size_t off = 0;
    descs_.clear();
    desc_groups_.clear();
    if (settle() || flush(stream_, &base, &off) || settle()) job.status = job.status ? job.status : QD_ERR_DEVICE;
  }
  if (!job.status) {
    qd_stats &S = job.S;
    S.L = job.L;
    S.U = job.U;
    S.next_t = job.t;
    S.next_j = job.j;
    if (S.next_j >= int(job.use.size())) {
      S.next_j = 0;
      ++S.next_t;
    }
    S.combinations = job.visited;
    // The witness must have weight U and lie in the row space.
    bool wit_ok = job.U <= job.n && rweight(job.wit) == job.U && in_span(job.basis, job.n, job.wit);
    if (!job.logicals.empty()) {  // Modified BZ: the witness is no stabilizer
      bool outside = false;
      for (const BRow &l : job.logicals) outside = outside || sym_product(job.wit, l);
      wit_ok = wit_ok && outside;
    }
    if (job.single_round) {
      // U is the round minimum (n + 1 if the round is empty), not a distance
    } else if (job.incomplete) {
      job.status = (job.U > job.n || wit_ok) ? QD_INCOMPLETE : QD_ERR_INTERNAL;
    } else {
      job.status = wit_ok ? QD_OK : QD_ERR_INTERNAL;
    }
    S.wall_ms = t1 - job.t0;
  }
  if (job.want_wsum && job.data.p && !job.status &&
      hipMemcpy(&job.wsum, static_cast<unsigned long long *>(job.data.p) + 2, sizeof(job.wsum),
                hipMemcpyDeviceToHost) != hipSuccess)
    job.status = QD_ERR_DEVICE;
  if (job.census_below > 0 && job.data.p && !job.status &&
      hipMemcpy(job.census, static_cast<unsigned long long *>(job.data.p) + 3, sizeof(job.census),
                hipMemcpyDeviceToHost) != hipSuccess)
    job.status = QD_ERR_DEVICE;
  for (GammaDev &g : job.gd) {
    g.elems = nullptr; g.csize = nullptr; g.dprefix = g.dsuffix = nullptr;
    g.inv = nullptr; g.logicals = nullptr;
  }
  release_tables(job);
  release(job.data);
  drop_flights(job);
  if (job.state_slot >= 0) free_slots_.push_back(job.state_slot);
  job.state_slot = -1;
  job.t_done = t1;
}

int run_jobs(Executor &ex, std::vector<Job *> &jobs, hipStream_t s) {
  static const bool trace = std::getenv("QD_TRACE") && std::getenv("QD_TRACE")[0] == '1';
  const double t0 = trace ? now_ms() : 0.0;
  for (Job *jp : jobs) {
    if (jp->status) { jp->done = true; continue; }
    const int rc = ex.admit(*jp, s);
    if (rc) { jp->status = rc; jp->done = true; }
  }
  const double t1 = trace ? now_ms() : 0.0;
  for (;;) {
    bool any = false;
    for (Job *jp : jobs) any = any || !jp->done;
    if (!any) break;
    const int rc = ex.step(jobs, s);
    if (rc) {
      for (Job *jp : jobs)
        if (!jp->done) { jp->status = rc; jp->done = true; }
      break;
    }
  }
  const double t2 = trace ? now_ms() : 0.0;
  for (Job *jp : jobs) ex.retire(*jp);
  if (trace)
    std::fprintf(stderr, "qd run: jobs %zu admit %.3f ms steps %.3f ms retire %.3f ms\n", jobs.size(), t1 - t0,
                 t2 - t1, now_ms() - t2);
  return QD_OK;
}

int default_executor(Executor **ex, std::unique_lock<std::mutex> *lock) {
  static std::mutex mu;
  static std::vector<std::unique_ptr<Executor>> per_dev;
  static std::vector<std::unique_ptr<std::mutex>> locks;
  int dev = 0, cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0 || hipGetDevice(&dev) != hipSuccess) return QD_ERR_DEVICE;
  std::mutex *m = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    if (int(per_dev.size()) <= dev) {
      per_dev.resize(dev + 1);
      locks.resize(dev + 1);
    }
    if (!per_dev[dev]) {
      tune_autoload();
      per_dev[dev] = std::make_unique<Executor>();
      locks[dev] = std::make_unique<std::mutex>();
    }
    if (!per_dev[dev]->ok()) return QD_ERR_DEVICE;
    *ex = per_dev[dev].get();
    m = locks[dev].get();
  }
  *lock = std::unique_lock<std::mutex>(*m);
  return QD_OK;
}

}  // namespace qd

// engine.hpp -- the step executor shared by the single-code, batched and
// serving entry points.  A step launches, for every active code, the next
// piece of its current (t, Gamma_j) round; all pieces of codes with the
// same word count D go into one kernel launch (the saved-sum kernel, or the
// plain walk kernel for codes that ask for it), each followed by one commit
// launch, and the step ends with one readback of every code's state.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/qdist.h"
#include "host.hpp"
#include "kernels.hpp"
#include "support.hpp"

namespace qd {

constexpr int kTMax = 48;  // deepest round supported

// Grow-only caching allocator of device memory (size classes; blocks go
// back to a free list and are reused by later codes).
class DevPool {
 public:
  ~DevPool();
  void *get(size_t bytes, size_t *cls);
  void put(void *p, size_t cls);
  size_t held() const { return held_; }
  int mallocs() const { return mallocs_; }
  double malloc_ms() const { return malloc_ms_; }
  // Arena mode: blocks are carved in order from [base, base + cap), which
  // the caller owns, and are never given back (put is a no-op); nothing is
  // allocated from the driver.  get returns nullptr once the arena is full.
  void set_arena(void *base, size_t cap) {
    arena_ = static_cast<unsigned char *>(base);
    arena_cap_ = cap;
    arena_off_ = 0;
  }
  bool arena() const { return arena_ != nullptr; }

 private:
  unsigned char *arena_ = nullptr;
  size_t arena_cap_ = 0, arena_off_ = 0;
  int mallocs_ = 0;
  double malloc_ms_ = 0.0;
  std::map<size_t, std::vector<void *>> free_;
  std::vector<void *> all_;
  size_t held_ = 0;
};

struct PoolBuf {
  void *p = nullptr;
  size_t cls = 0;
  size_t bytes = 0;
};

// Device copy of one generator matrix and its saved / tops tables.  The
// elements, sizes and e_r tables live in the job's data block.
struct GammaDev {
  int P = 0, R = 0;
  std::vector<int> sizes;
  std::vector<uint64_t> prefix, suffix;  // e_r tables (host copies)
  std::vector<uint32_t> h_elems;         // in the stored qubit order
  std::vector<unsigned char> h_csize;
  QubitOrder order;                      // stored qubit order (partial weights)
  int delta = 0;
  const uint32_t *elems = nullptr;
  const unsigned char *csize = nullptr;
  const unsigned char *inv = nullptr;    // device copy of order.pos (NULL: unchanged)
  const uint32_t *logicals = nullptr;    // Modified BZ operators in the stored order
  const unsigned long long *dprefix = nullptr, *dsuffix = nullptr;
  PoolBuf table[kTMax + 1], tops[kTMax + 1];
  // Matrix-core form of table[u] (RoundDesc::mtable) and its K-steps per chunk.
  PoolBuf mtable[kTMax + 1];
  int mtable_ks[kTMax + 1];
  // Launch wave of a table build queued for the next flush (-1: none).
  int table_level[kTMax + 1], tops_level[kTMax + 1];
  GammaDev() {
    for (int &l : table_level) l = -1;
    for (int &l : tops_level) l = -1;
    for (int &k : mtable_ks) k = 0;
  }
};

// Pinned host bytes gathered between device steps and sent in one copy.
class Staging {
 public:
  ~Staging();
  // Appends bytes at a 16-byte aligned offset, which it returns; SIZE_MAX
  // if pinned memory runs out.
  size_t put(const void *src, size_t bytes);
  size_t size() const { return n_; }
  const unsigned char *data() const { return p_; }
  void clear() { n_ = 0; }
  // Ordinary (pageable) host memory instead of pinned memory.
  void set_pageable() { pageable_ = true; }

 private:
  unsigned char *p_ = nullptr;
  size_t n_ = 0, cap_ = 0;
  bool pageable_ = false;
};

// One scheduled (t, Gamma_j) round of a code and its tile plan.
struct Flight {
  int t = 0, j = 0, u = 0;
  unsigned seg = 0;
  bool use_tops = true;
  // Tops over t - u >= 2 packages come from the tops table one package
  // shallower: element c of the top's smallest package XOR that table's
  // entry (RoundDesc::tops_down), so the deepest tops table is not built.
  bool tops_down = false;
  int L_before = 0;  // bound certified before the step that scheduled it
  std::vector<DevGroup> hg;
  std::vector<DevRun> hr;
  unsigned long long tiles = 0, sent = 0, planned = 0;
  int launches = 0;
  float ms = 0.f;
  // Plain walk (qd_options.walk): one launch per round, its sets split
  // into parts by their one-row packages, one wave per 64 lanes of
  // per_lane sets each.
  bool walk = false;
  unsigned long long per_lane = 1;
  int p2 = 0;                             // two-row packages of the matrix
  std::vector<unsigned long long> binom;  // C(p, r), p <= P, r <= t
  std::vector<unsigned short> pmap;       // two-row packages, then one-row ones
  std::vector<WalkPart> parts;
};

// One code: request, plan, device data and progress through its rounds.
struct Job {
  // request
  std::vector<uint8_t> G;
  int m = 0, n = 0, field = 2;
  qd_options opt{};
  bool single_round = false;  // run exactly round t of use[0] (no early exit)
  uint64_t tag = 0;
  double t_submit = 0.0;
  // plan
  int status = QD_OK;
  int D = 1, rank = 0;
  std::vector<BRow> basis;
  std::vector<Gamma> use;
  PlanChoice pc;
  bool halve = false;  // isometry matrices: bounds count Hamming weight
  bool scalar = false; // one codeword per F4 scalar class
  bool partial = false; // partial weights (matrices stored in their qubit order)
  std::vector<int> caps; // mixed packages: two-row caps of the F4 matrices (empty: none)
  int force_words = 0;   // > 0: every tile evaluates this many words first (no credit)
  // Matrix cores for the saved-table rounds; mks K-steps per chunk with every
  // word (the last word packed into a spare group when mpack).
  bool mfma = false;
  int mks = 0, mpack = 0;
  // Resume point (copied from qd_options.resume by prepare)
  bool has_resume = false;
  int r_t = 0, r_j = 0, r_U = 0;
  std::vector<uint8_t> r_wit;
  unsigned long long r_structure = 0;
  bool want_wsum = false;        // plain walk: sum the weights of the walked codewords
  unsigned long long wsum = 0;   // (read back by retire)
  int census_below = 0;          // > 0: census of the codewords of weight below it
  unsigned long long census[2] = {0, 0};  // their count and weight sum (read back by retire)
  std::vector<BRow> logicals;  // Modified BZ: the admission test's operators
  std::vector<GammaDev> gd;
  int state_slot = -1;
  PoolBuf data;  // visited counters, then every Gamma_j's elements and tables
  // progress
  std::vector<int> tdone, delta;
  int L = 0, U = 0;
  BRow wit;
  unsigned long long visited = 0, planned_total = 0;
  int t = 1, j = 0;          // next round to schedule
  bool done = false, incomplete = false;
  std::vector<Flight> fl;    // rounds in flight, in order
  qd_stats S{};
  double t0 = 0.0;
  double t_done = 0.0;
};

class Executor {
 public:
  explicit Executor(hipStream_t stream = nullptr);
  // Arena executor: all device memory is carved from [arena, arena + bytes)
  // (the caller's), uploads go through pageable host memory, no stream or
  // event is created (stream may be the null stream) and nothing is
  // allocated from the driver; a request that does not fit fails with
  // QD_ERR_NOMEM from its step.  The caller checks the device: a gfx950
  // that holds the arena.
  Executor(hipStream_t stream, void *arena, size_t bytes);
  ~Executor();
  bool arena() const { return pool_.arena(); }
  bool ok() const { return ok_; }
  hipStream_t stream() const { return stream_; }
  size_t device_bytes() const { return pool_.held(); }
  // Combinations of one code's consecutive rounds that one step may carry
  // (more: fewer steps; less: shorter steps, e.g. for serving).
  void set_spec_combos(unsigned long long c) { spec_combos_ = c; }
  // Table entries per tile that large rounds start from (steps of fewer
  // than 9 codes): shorter tiles end steps sooner, e.g. for serving.
  void set_long_seg(unsigned seg) { long_seg_ = seg; }
  // Whether rounds take the measured launch shapes (tune_lookup) where
  // installed; the serving engine keeps its latency-minded model rules.
  void set_tuned(bool on) { tuned_ = on; }
  // Rounds of at least this many combinations take the matrix cores (with
  // the expansion of their saved table); smaller ones the vector ALU.
  void set_mfma_min_round(unsigned long long c) { mfma_min_round_ = c; }

  // Host-side preparation of a job (input check, basis, diagonalizations,
  // plan).  Thread-safe; touches no device state.
  static void prepare(Job &job);
  // The part of prepare() after the generator matrices are chosen.
  static void prepare_gammas(Job &job);
  // Starts a prepared job at its resume point (qd_options.resume).
  static void apply_resume(Job &job);
  // Device upload of a prepared job (needs a free state slot).
  int admit(Job &job, hipStream_t s);
  // One step over the given jobs; finished jobs get done = true.
  int step(std::vector<Job *> &jobs, hipStream_t s);
  // Final checks, outputs and release of the job's device memory.
  void retire(Job &job);
  // Estimated device bytes of a prepared job (admission control).
  static size_t footprint(const Job &job);

 private:
  int schedule(Job &job, int sharing);
  void end_round(Job &job, Flight &f);
  void drop_flights(Job &job);
  int ensure_table(Job &job, GammaDev &g, int u, bool tops);
  int ensure_mtable(Job &job, GammaDev &g, int u, int mks);
  void release_mtable(GammaDev &g, int u);
  void release_tables(Job &job);
  int flush(hipStream_t s, const unsigned char **base, size_t *desc_off);
  int settle();
  bool alloc(PoolBuf &b, size_t bytes);
  void release(PoolBuf &b);
  int grow_states(int need);

  bool ok_ = false;
  bool tuned_ = true;
  unsigned long long mfma_min_round_;
  unsigned long long spec_combos_;
  unsigned long_seg_;
  bool own_stream_ = false;
  hipStream_t stream_ = nullptr;
  DevPool pool_;
  // per-code states (device) and their pinned host mirror (arena executor:
  // ordinary host memory, host_states_)
  DevState *states_ = nullptr;
  DevState *hstates_ = nullptr;
  std::vector<DevState> host_states_;
  // Saved and tops tables of at most this many bytes (arena executor: a
  // quarter of the arena)
  unsigned long long max_table_bytes_;
  int nstates_ = 0;
  std::vector<int> free_slots_;
  std::vector<int> dirty_slots_;  // states to upload at the next flush
  // Uploads: staged host bytes, block moves of persistent data, and the
  // device buffer the staged bytes go to (transient launch data is read
  // from there directly).  After a flush the staged bytes stay in use
  // until the stream is synchronized (inflight_).
  Staging staging_;
  std::vector<CopyRec> recs_;
  PoolBuf stage_dev_;
  bool inflight_ = false;
  hipStream_t inflight_stream_ = nullptr;
  // launch resources
  PoolBuf slots_;
  uint32_t *zero_table_ = nullptr;  // the saved table of depth 0: one zero entry
  std::vector<SavedParams> builds_[5];  // queued table builds per word count
  std::vector<int *> level_marks_;      // table_level entries to clear after the flush
  std::vector<ExpandParams> expands_;   // queued matrix-core forms (after the builds)
  size_t mtable_budget_ = 0, mtable_held_ = 0;  // bytes of matrix-core forms: limit, held
  std::vector<RoundDesc> descs_;
  std::vector<size_t> desc_groups_;  // staged offsets of each piece's groups, runs, binomials,
                                     // package map and walk parts (kStagedPerDesc each)
  std::vector<hipEvent_t> events_;
};

// The executor of the current device for the synchronous entry points.
int default_executor(Executor **ex, std::unique_lock<std::mutex> *lock);

// Measured launch shapes (tune.cpp): the tuned segment length and saved-table
// depth cap for a round of `planned` combinations of a code with D words per
// half, in a step shared by `sharing` codes, on the partial-weight path
// (partial_words > 0) or not; false when no tuning is installed for that
// bucket.  tune_autoload installs the tuning file once per process.
bool tune_lookup(int D, unsigned long long planned, int sharing, int partial_words, unsigned *seg, int *depth);
void tune_autoload();
// The fixed rules' shape for such a round (no tuning installed).
unsigned rule_seg(unsigned long long planned, int sharing);
int rule_depth_cap();

// Runs a set of prepared jobs to completion on one executor.
int run_jobs(Executor &ex, std::vector<Job *> &jobs, hipStream_t s);

// One round over a caller-given package layout (rows: 2P rows of 2n bytes,
// dims 1 or 2 per package): the body of qd_round_min, qd_round_census,
// qd_round_walk and qd_round_min_noalloc.  Runs on `arena_ex` (an arena
// executor; QD_ERR_TOO_LARGE when the round does not fit its arena) or, when
// it is NULL, on the current device's default executor.
int one_round(const uint8_t *rows, const int *dims, int P, int n, int t, int partial_words, int walk, int *wmin,
              uint8_t *witness, unsigned long long *count, unsigned long long *weight_sum, int below,
              unsigned long long *census, Executor *arena_ex);

}  // namespace qd

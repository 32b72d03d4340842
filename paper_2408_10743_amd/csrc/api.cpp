// api.cpp -- C ABI of libqdist: per-device context, the round driver of
// the Brouwer-Zimmermann enumeration, and the entry points of qdist.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/qdist.h"
#include "host.hpp"
#include "kernels.hpp"

namespace qd {
hipError_t launch_round(int D, const RoundParams &p, hipStream_t s);
hipError_t launch_saved(int D, const SavedParams &p, hipStream_t s);
hipError_t launch_commit(DevState *st, const uint32_t *slots, unsigned long long *counters, hipStream_t s);
hipError_t launch_valu(uint32_t blocks, uint32_t iters, uint32_t *out, hipStream_t s);
}  // namespace qd

using namespace qd;

namespace {

constexpr int kTMax = 48;                         // deepest round supported
constexpr int kDefaultSavedDepth = 4;             // packages per saved-table entry
constexpr unsigned long long kMaxTableBytes = 1ull << 29;
constexpr unsigned long long kMaxTopEntries = 1ull << 24;  // 512 MB of tops
constexpr unsigned long long kTilesPerLaunch = 1ull << 20;
constexpr unsigned long long kTargetTiles = 1ull << 18;  // ~32 tiles per wave slot
constexpr unsigned kMinSeg = 256, kMaxSeg = 16384;
constexpr unsigned kStageMaxBytes = 32768;

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct DevBuf {
  void *p = nullptr;
  size_t cap = 0;
  bool ensure(size_t bytes) {
    if (bytes <= cap) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) return false;
    cap = bytes;
    return true;
  }
  template <class T> T *as() const { return static_cast<T *>(p); }
};

// Device copy of one generator matrix and its saved tables.
struct GammaDev {
  int P = 0, R = 0;
  std::vector<int> sizes;
  std::vector<uint64_t> prefix, suffix;  // host copies of the e_r tables
  std::vector<uint32_t> h_elems;         // host staging kept alive across async copies
  std::vector<unsigned char> h_csize;
  DevBuf elems, csize, dprefix, dsuffix;
  DevBuf table[kTMax + 1], tops[kTMax + 1];
  bool built[kTMax + 1] = {}, tbuilt[kTMax + 1] = {};
};

struct Ctx {
  int device = -1;
  bool ok = false;
  hipStream_t own = nullptr;
  std::mutex mu;
  GammaDev g[kMaxGamma];
  DevBuf groups, runs, slots, state, counters;
  std::vector<DevGroup> h_groups;  // host staging of the last round's tables
  std::vector<DevRun> h_runs;
  DevState *hstate = nullptr;  // pinned
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<hipEvent_t> pool;  // start/stop pairs of the current round
};

// Start/stop events for launch i of a round (created on first use).
bool launch_events(Ctx &c, size_t i, hipEvent_t *a, hipEvent_t *b) {
  while (c.pool.size() < 2 * (i + 1)) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    c.pool.push_back(e);
  }
  *a = c.pool[2 * i];
  *b = c.pool[2 * i + 1];
  return true;
}

std::mutex g_ctx_mu;
std::vector<std::unique_ptr<Ctx>> g_ctx;

int get_ctx(Ctx **out) {
  int dev = 0;
  int cnt = 0;
  if (hipGetDeviceCount(&cnt) != hipSuccess || cnt <= 0) return QD_ERR_DEVICE;
  if (hipGetDevice(&dev) != hipSuccess) return QD_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(g_ctx_mu);
  if (int(g_ctx.size()) <= dev) g_ctx.resize(dev + 1);
  if (!g_ctx[dev]) {
    auto c = std::make_unique<Ctx>();
    c->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && std::strstr(prop.gcnArchName, "gfx950") &&
        hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) == hipSuccess &&
        hipHostMalloc(reinterpret_cast<void **>(&c->hstate), sizeof(DevState), hipHostMallocDefault) == hipSuccess &&
        hipEventCreate(&c->e0) == hipSuccess && hipEventCreate(&c->e1) == hipSuccess)
      c->ok = true;
    g_ctx[dev] = std::move(c);
  }
  if (!g_ctx[dev]->ok) return QD_ERR_DEVICE;
  *out = g_ctx[dev].get();
  return QD_OK;
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

void unpack(const BRow &r, int n, uint8_t *out) {
  for (int q = 0; q < n; ++q) {
    out[q] = uint8_t((r.x[q >> 6] >> (q & 63)) & 1);
    out[n + q] = uint8_t((r.z[q >> 6] >> (q & 63)) & 1);
  }
}

// Uploads one generator matrix: elements r, s, r^s per package, sizes and
// the e_r tables used to unrank combinations.
int upload_gamma(GammaDev &gd, const Gamma &g, hipStream_t s) {
  gd.P = g.P();
  gd.R = std::min(gd.P, kTMax) + 1;
  gd.sizes.clear();
  std::vector<uint32_t> &el = gd.h_elems;
  std::vector<unsigned char> &cs = gd.h_csize;
  el.assign(size_t(gd.P) * 3 * kElemWords, 0);
  cs.assign(gd.P, 0);
  for (int i = 0; i < gd.P; ++i) {
    const Package &p = g.pk[i];
    to_words(p.r, &el[size_t(3 * i) * kElemWords]);
    if (p.dim == 2) {
      BRow rs = p.r;
      radd(rs, p.s);
      to_words(p.s, &el[size_t(3 * i + 1) * kElemWords]);
      to_words(rs, &el[size_t(3 * i + 2) * kElemWords]);
    }
    cs[i] = p.dim == 2 ? 3 : 1;
    gd.sizes.push_back(cs[i]);
  }
  esym_tables(gd.sizes, gd.R - 1, gd.prefix, gd.suffix);
  const size_t tb = gd.prefix.size() * sizeof(uint64_t);
  if (!gd.elems.ensure(el.size() * 4) || !gd.csize.ensure(cs.size() + 1) || !gd.dprefix.ensure(tb) ||
      !gd.dsuffix.ensure(tb))
    return QD_ERR_NOMEM;
  if (hipMemcpyAsync(gd.elems.p, el.data(), el.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(gd.csize.p, cs.data(), cs.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(gd.dprefix.p, gd.prefix.data(), tb, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(gd.dsuffix.p, gd.suffix.data(), tb, hipMemcpyHostToDevice, s) != hipSuccess)
    return QD_ERR_DEVICE;
  for (int u = 0; u <= kTMax; ++u) gd.built[u] = gd.tbuilt[u] = false;
  return QD_OK;
}

// Builds (once per matrix) the saved table of u-package bottoms, or with
// tops = true the table of u-package tops.
int ensure_table(GammaDev &gd, int D, int u, bool tops, hipStream_t s) {
  if (tops ? gd.tbuilt[u] : gd.built[u]) return QD_OK;
  const unsigned long long nent = tops ? gd.suffix[u] : gd.prefix[size_t(gd.P) * gd.R + u];
  const unsigned long long padded = (nent + kBlock - 1) / kBlock * kBlock;
  DevBuf &buf = tops ? gd.tops[u] : gd.table[u];
  if (!buf.ensure(size_t(padded) * (tops ? kElemWords : 2 * D) * 4)) return QD_ERR_NOMEM;
  SavedParams sp;
  sp.elems = gd.elems.as<uint32_t>();
  sp.prefix = gd.dprefix.as<unsigned long long>();
  sp.suffix = gd.dsuffix.as<unsigned long long>();
  sp.csize = gd.csize.as<unsigned char>();
  sp.table = buf.as<uint32_t>();
  sp.nent = nent;
  sp.nent_padded = padded;
  sp.P = gd.P;
  sp.R = gd.R;
  sp.u = u;
  sp.tops = tops ? 1 : 0;
  if (launch_saved(D, sp, s) != hipSuccess) return QD_ERR_DEVICE;
  (tops ? gd.tbuilt[u] : gd.built[u]) = true;
  return QD_OK;
}

// Saved-table depth for round t: u = t-2, so every top keeps two packages
// (a group then fills many lanes), within the cap and the table-size limit.
int saved_depth(const GammaDev &gd, int D, int t, int cap) {
  int u = std::min(std::max(t - 2, 0), cap);
  while (u > 0 && gd.prefix[size_t(gd.P) * gd.R + u] * 8ull * D > kMaxTableBytes) --u;
  return u;
}

// Table entries per tile: long enough to amortize a tile's setup (group
// search, unranking of 64 tops), short enough for ~kTargetTiles tiles.
unsigned choose_seg(unsigned long long planned) {
  const unsigned long long want = planned / (kWave * kTargetTiles);
  unsigned seg = kMinSeg;
  while (seg < want && seg < kMaxSeg) seg <<= 1;
  return seg;
}

struct RoundPlan {
  std::vector<DevGroup> groups;  // longest table prefix first
  std::vector<DevRun> runs;
  unsigned long long tiles = 0;
  unsigned long long combos = 0;
};

// Tiles of one round.  Group h pairs the tops whose smallest package is h
// (c_h * e_{t-u-1}(c_{h+1}..)) with the first e_u(c_0..c_{h-1}) table
// entries.  Segment s of the table is shared by every group reaching it,
// so its tiles take 64 tops at a time from those groups together.
void plan_round(const GammaDev &gd, int t, int u, unsigned seg, RoundPlan &rp) {
  rp.groups.clear();
  rp.runs.clear();
  rp.tiles = rp.combos = 0;
  const int R = gd.R, r = t - u - 1;
  for (int h = 0; h < gd.P; ++h) {
    const unsigned long long items = gd.suffix[size_t(h + 1) * R + r] * gd.sizes[h];
    const unsigned long long len = gd.prefix[size_t(h) * R + u];
    if (!items || !len) continue;
    DevGroup grp{};
    grp.items = items;
    grp.len = len;
    grp.top0 = gd.suffix[size_t(h + 1) * R + (t - u)];
    grp.h = h;
    rp.combos += items * len;
    rp.groups.push_back(grp);
  }
  std::stable_sort(rp.groups.begin(), rp.groups.end(),
                   [](const DevGroup &a, const DevGroup &b) { return a.len > b.len; });
  unsigned long long cum = 0;
  std::vector<unsigned long long> ns(rp.groups.size());
  for (size_t i = 0; i < rp.groups.size(); ++i) {
    rp.groups[i].cum = cum;
    cum += rp.groups[i].items;
    ns[i] = (rp.groups[i].len + seg - 1) / seg;
  }
  // Segments [ns[e], ns[e-1]) are reached by exactly the e longest groups.
  const size_t G = rp.groups.size();
  for (size_t e = G; e >= 1; --e) {
    const unsigned long long sa = e == G ? 0 : ns[e], sb = ns[e - 1];
    if (sa >= sb) continue;
    DevRun run{};
    run.tile0 = rp.tiles;
    run.s_begin = sa;
    run.e = static_cast<long long>(e);
    run.items = e == G ? cum : rp.groups[e].cum;
    run.tps = (run.items + kWave - 1) / kWave;
    rp.tiles += (sb - sa) * run.tps;
    rp.runs.push_back(run);
  }
}

struct RunOut {
  int U = 0;
  BRow wit;
  unsigned long long visited = 0;
  int launches = 0;
  float ms = 0.f;
};

// One (t, Gamma) round: saved table, tile plan, launches, commit, readback.
int run_round(Ctx &c, GammaDev &gd, int D, int t, int u, unsigned seg, int L_before, bool timing,
              int tops_mode, hipStream_t s, RunOut &ro) {
  int rc = ensure_table(gd, D, u, false, s);
  if (rc) return rc;
  // Tops come from a table when it is small enough, else lanes unrank them.
  const bool use_tops = tops_mode == 1 || (tops_mode == 0 && gd.suffix[t - u] <= kMaxTopEntries);
  if (use_tops && (rc = ensure_table(gd, D, t - u, true, s))) return rc;
  RoundPlan rp;
  plan_round(gd, t, u, seg, rp);
  c.h_groups.swap(rp.groups);  // the async copies read the context's copies
  c.h_runs.swap(rp.runs);
  const std::vector<DevGroup> &groups = c.h_groups;
  const std::vector<DevRun> &runs = c.h_runs;
  ro.launches = 0;
  ro.ms = 0.f;
  if (rp.tiles) {
    const size_t gb = groups.size() * sizeof(DevGroup), rb = runs.size() * sizeof(DevRun);
    if (!c.groups.ensure(gb) || !c.runs.ensure(rb) ||
        !c.slots.ensure(size_t(std::min(rp.tiles, kTilesPerLaunch)) * kElemWords * 4))
      return QD_ERR_NOMEM;
    if (hipMemcpyAsync(c.groups.p, groups.data(), gb, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c.runs.p, runs.data(), rb, hipMemcpyHostToDevice, s) != hipSuccess)
      return QD_ERR_DEVICE;
    RoundParams p;
    p.elems = gd.elems.as<uint32_t>();
    p.table = gd.table[u].as<uint32_t>();
    p.tops = use_tops ? gd.tops[t - u].as<uint32_t>() : nullptr;
    p.groups = c.groups.as<DevGroup>();
    p.runs = c.runs.as<DevRun>();
    p.suffix = gd.dsuffix.as<unsigned long long>();
    p.csize = gd.csize.as<unsigned char>();
    p.state = c.state.as<DevState>();
    p.counters = c.counters.as<unsigned long long>();
    p.slots = c.slots.as<uint32_t>();
    p.ngroups = int(groups.size());
    p.nruns = int(runs.size());
    p.P = gd.P;
    p.R = gd.R;
    p.t = t;
    p.u = u;
    p.seg = seg;
    p.L_before = L_before;
    p.stage = use_tops ? 1 : 2;
    if (round_lds_bytes(gd.P, t, u, p.ngroups, p.stage) > kStageMaxBytes) p.stage = 0;
    for (unsigned long long lo = 0; lo < rp.tiles; lo += kTilesPerLaunch) {
      p.tile_lo = lo;
      p.tile_hi = std::min(rp.tiles, lo + kTilesPerLaunch);
      hipEvent_t ea = nullptr, eb = nullptr;
      if (timing && (!launch_events(c, size_t(ro.launches), &ea, &eb) || hipEventRecord(ea, s) != hipSuccess))
        return QD_ERR_DEVICE;
      if (launch_round(D, p, s) != hipSuccess) return QD_ERR_DEVICE;
      if (timing && hipEventRecord(eb, s) != hipSuccess) return QD_ERR_DEVICE;
      if (launch_commit(p.state, p.slots, p.counters, s) != hipSuccess) return QD_ERR_DEVICE;
      ++ro.launches;
    }
  }
  if (hipMemcpyAsync(c.hstate, c.state.p, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return QD_ERR_DEVICE;
  if (timing) {
    for (int i = 0; i < ro.launches; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c.pool[2 * i], c.pool[2 * i + 1]) != hipSuccess) return QD_ERR_DEVICE;
      ro.ms += ms;
    }
  }
  ro.U = int(c.hstate->key >> 32);
  ro.wit = from_words(c.hstate->wit);
  ro.visited = c.hstate->count;
  return QD_OK;
}

int reset_state(Ctx &c, int n, hipStream_t s) {
  if (!c.state.ensure(sizeof(DevState))) return QD_ERR_NOMEM;
  const size_t cb = size_t(kCounters) * kCounterStride * sizeof(unsigned long long);
  if (c.counters.cap < cb) {
    if (!c.counters.ensure(cb)) return QD_ERR_NOMEM;
    if (hipMemsetAsync(c.counters.p, 0, cb, s) != hipSuccess) return QD_ERR_DEVICE;
  }
  std::memset(c.hstate, 0, sizeof(DevState));
  c.hstate->key = (static_cast<unsigned long long>(n + 1) << 32) | kNoSlot;
  if (hipMemcpyAsync(c.state.p, c.hstate, sizeof(DevState), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return QD_ERR_DEVICE;
  return QD_OK;
}

bool in_span(const std::vector<BRow> &basis, int n, const BRow &v) {
  std::vector<BRow> rows = basis;
  const int k = make_basis(rows, n);
  rows.push_back(v);
  return make_basis(rows, n) == k;
}

int distance_impl(const uint8_t *G, int m, int n, int field, const qd_options *opt, int *d,
                  uint8_t *witness, qd_stats *st) {
  const double t0 = now_ms();
  qd_options o{};
  if (opt) o = *opt;
  qd_stats local{};
  qd_stats &S = st ? *st : local;
  std::memset(&S, 0, sizeof(S));
  if (d) *d = -1;
  if (!d) return QD_ERR_INVALID;
  if (o.diag != QD_DIAG_AUTO && o.diag != QD_DIAG_F2 && o.diag != QD_DIAG_F4) return QD_ERR_INVALID;
  if (o.seg_len < 0 || o.seg_len % kBlock || o.saved_depth < 0 || o.max_gamma < 0 || o.tops_mode < 0 ||
      o.tops_mode > 2)
    return QD_ERR_INVALID;
  std::vector<BRow> rows;
  int rc = load_rows(G, m, n, field, rows);
  if (rc) return rc;
  const int k = make_basis(rows, n);
  if (k == 0) return QD_ERR_ZERO_CODE;
  std::vector<Gamma> f4 = build_f4(rows, n, kMaxGamma);
  Gamma f2 = build_f2(rows, n);
  for (const Gamma &g : f4)
    if (!check_gamma(g, n)) return QD_ERR_INTERNAL;
  if (!check_gamma(f2, n)) return QD_ERR_INTERNAL;
  PlanChoice pc = choose_plan(f4, f2, n, k, o.diag, o.max_gamma);
  std::vector<Gamma> use;
  if (pc.diag == QD_DIAG_F2) use.push_back(f2);
  else use.assign(f4.begin(), f4.begin() + pc.h_used);
  const int h = int(use.size());
  const int D = (n + 31) / 32;
  S.n = n; S.rank = k; S.D = D; S.diag = pc.diag; S.h = h;
  S.d_estimate = pc.d_est; S.predicted = pc.predicted;
  for (int j = 0; j < h; ++j) { S.P[j] = use[j].P(); S.delta[j] = use[j].delta; }

  Ctx *cp = nullptr;
  rc = get_ctx(&cp);
  if (rc) return rc;
  Ctx &c = *cp;
  std::lock_guard<std::mutex> lk(c.mu);
  hipStream_t s = o.stream ? static_cast<hipStream_t>(o.stream) : c.own;
  for (int j = 0; j < h; ++j)
    if ((rc = upload_gamma(c.g[j], use[j], s))) return rc;
  if ((rc = reset_state(c, n, s))) return rc;
  S.host_ms = now_ms() - t0;

  const int cap = o.saved_depth ? o.saved_depth : kDefaultSavedDepth;
  std::vector<int> tdone(h, 0), delta(h);
  for (int j = 0; j < h; ++j) delta[j] = use[j].delta;
  int L = lower_bound(tdone, delta);
  int U = n + 1;
  BRow wit;
  unsigned long long visited = 0, planned_total = 0;
  bool finished = false, incomplete = false;
  for (int t = 1; !finished && !incomplete; ++t) {
    bool any = false;
    for (int j = 0; j < h && !finished && !incomplete; ++j) {
      if (t > use[j].P()) continue;
      any = true;
      if (t > kTMax) { incomplete = true; break; }
      if (o.cancel && *o.cancel) { incomplete = true; break; }
      GammaDev &gd = c.g[j];
      const uint64_t planned = gd.prefix[size_t(gd.P) * gd.R + t];
      if (planned >= kSat || (o.budget && planned_total + planned > o.budget)) { incomplete = true; break; }
      const int u = saved_depth(gd, D, t, cap);
      const unsigned seg = o.seg_len ? unsigned(o.seg_len) : choose_seg(planned);
      RunOut ro;
      if ((rc = run_round(c, gd, D, t, u, seg, L, o.timing != 0, o.tops_mode, s, ro))) return rc;
      planned_total += planned;
      if (ro.U < U) { U = ro.U; wit = ro.wit; }
      const unsigned long long this_round = ro.visited - visited;
      visited = ro.visited;
      tdone[j] = t;
      L = lower_bound(tdone, delta);
      S.kernel_ms += ro.ms;
      if (S.nlog < QD_MAX_LOG) {
        qd_round_log &lg = S.log[S.nlog];
        lg.t = t; lg.j = j; lg.L = L; lg.U = U; lg.saved_depth = u; lg.launches = ro.launches;
        lg.combinations = this_round; lg.planned = planned; lg.kernel_ms = ro.ms;
      }
      ++S.nlog;
      if (L >= U || t == use[j].P()) finished = true;
    }
    if (!any) finished = true;
  }
  S.L = L; S.U = U; S.combinations = visited;
  if (U > n) return QD_ERR_INTERNAL;
  // The witness must have weight U and lie in the row space.
  if (rweight(wit) != U || !in_span(rows, n, wit)) return QD_ERR_INTERNAL;
  *d = U;
  if (witness) unpack(wit, n, witness);
  S.wall_ms = now_ms() - t0;
  return incomplete ? QD_INCOMPLETE : QD_OK;
}

}  // namespace

extern "C" {

int qd_distance(const uint8_t *G, int m, int n, int field, int *d, uint8_t *witness) {
  return distance_impl(G, m, n, field, nullptr, d, witness, nullptr);
}

int qd_distance_ex(const uint8_t *G, int m, int n, int field, const qd_options *opt, int *d,
                   uint8_t *witness, qd_stats *st) {
  return distance_impl(G, m, n, field, opt, d, witness, st);
}

int qd_distance_batch_ex(int count, const uint8_t *const *G, const int *m, const int *n,
                         const int *field, const qd_options *opt, int *d, uint8_t *const *witness,
                         int *status, qd_stats *st) {
  if (count < 0 || (count > 0 && (!G || !m || !n || !field || !d || !status))) return QD_ERR_INVALID;
  int first = QD_OK;
  for (int i = 0; i < count; ++i) {
    status[i] = distance_impl(G[i], m[i], n[i], field[i], opt, &d[i], witness ? witness[i] : nullptr,
                              st ? &st[i] : nullptr);
    if (status[i] < 0 && first == QD_OK) first = status[i];
  }
  return first;
}

int qd_distance_batch(int count, const uint8_t *const *G, const int *m, const int *n, const int *field,
                      int *d, uint8_t *const *witness, int *status) {
  return qd_distance_batch_ex(count, G, m, n, field, nullptr, d, witness, status, nullptr);
}

int qd_plan(const uint8_t *G, int m, int n, int field, int diag, int max_gamma, qd_plan_info *out) {
  if (!out) return QD_ERR_INVALID;
  std::memset(out, 0, sizeof(*out));
  if (diag != QD_DIAG_AUTO && diag != QD_DIAG_F2 && diag != QD_DIAG_F4) return QD_ERR_INVALID;
  if (max_gamma < 0) return QD_ERR_INVALID;
  std::vector<BRow> rows;
  int rc = load_rows(G, m, n, field, rows);
  if (rc) return rc;
  const int k = make_basis(rows, n);
  if (k == 0) return QD_ERR_ZERO_CODE;
  const int hmax = max_gamma > 0 ? std::min(max_gamma, kMaxGamma) : kMaxGamma;
  std::vector<Gamma> f4 = build_f4(rows, n, hmax);
  Gamma f2 = build_f2(rows, n);
  for (const Gamma &g : f4)
    if (!check_gamma(g, n)) return QD_ERR_INTERNAL;
  if (!check_gamma(f2, n)) return QD_ERR_INTERNAL;
  PlanChoice pc = choose_plan(f4, f2, n, k, diag, max_gamma);
  out->n = n;
  out->rank = k;
  out->d_estimate = pc.d_est;
  out->predicted_f2 = pc.predicted_f2;
  out->predicted_f4 = pc.predicted_f4;
  const int show = diag == QD_DIAG_AUTO ? pc.diag : diag;
  out->diag = show;
  std::vector<Gamma> gs;
  if (show == QD_DIAG_F2) gs.push_back(f2);
  else gs = f4;
  out->h = int(gs.size());
  out->h_used = show == pc.diag ? pc.h_used : out->h;
  for (int j = 0; j < out->h; ++j) {
    out->P[j] = gs[j].P();
    out->delta[j] = gs[j].delta;
    for (int i = 0; i < gs[j].P(); ++i) {
      out->dims[j][i] = gs[j].pk[i].dim;
      out->pivot[j][i] = gs[j].pk[i].pivot;
    }
  }
  return QD_OK;
}

int qd_round_min(const uint8_t *rows, const int *dims, int P, int n, int t, int *wmin, uint8_t *witness,
                 unsigned long long *count) {
  if (!rows || !dims || !wmin || !count || P <= 0 || P > 2 * kMaxN || t < 1 || n <= 0) return QD_ERR_INVALID;
  if (n > kMaxN) return QD_ERR_TOO_LARGE;
  Gamma g;
  for (int i = 0; i < P; ++i) {
    if (dims[i] != 1 && dims[i] != 2) return QD_ERR_INVALID;
    Package pk;
    pk.dim = dims[i];
    pk.pivot = i % kMaxN;
    std::vector<BRow> two;
    int rc = load_rows(rows + size_t(2 * i) * 2 * n, 2, n, QD_FIELD_F2, two);
    if (rc) return rc;
    pk.r = two[0];
    if (pk.dim == 2) pk.s = two[1];
    g.pk.push_back(pk);
  }
  *wmin = n + 1;
  *count = 0;
  if (t > P) return QD_OK;
  if (t > kTMax) return QD_ERR_TOO_LARGE;
  Ctx *cp = nullptr;
  int rc = get_ctx(&cp);
  if (rc) return rc;
  Ctx &c = *cp;
  std::lock_guard<std::mutex> lk(c.mu);
  hipStream_t s = c.own;
  GammaDev &gd = c.g[0];
  if ((rc = upload_gamma(gd, g, s))) return rc;
  if (gd.prefix[size_t(gd.P) * gd.R + t] >= kSat) return QD_ERR_TOO_LARGE;
  if ((rc = reset_state(c, n, s))) return rc;
  const int D = (n + 31) / 32;
  RunOut ro;
  const unsigned long long planned = gd.prefix[size_t(gd.P) * gd.R + t];
  if ((rc = run_round(c, gd, D, t, saved_depth(gd, D, t, kDefaultSavedDepth), choose_seg(planned), -1, false, 0,
                      s, ro)))
    return rc;
  *wmin = ro.U;
  *count = ro.visited;
  if (witness && ro.U <= n) unpack(ro.wit, n, witness);
  return QD_OK;
}

const char *qd_strerror(int status) {
  switch (status) {
    case QD_OK: return "ok";
    case QD_INCOMPLETE: return "incomplete: budget or cancel reached before the bounds met";
    case QD_ERR_INVALID: return "invalid argument";
    case QD_ERR_ZERO_CODE: return "the rows span the zero code";
    case QD_ERR_TOO_LARGE: return "problem too large (n > 128 or round beyond the supported depth)";
    case QD_ERR_NOMEM: return "device memory allocation failed";
    case QD_ERR_DEVICE: return "no usable gfx950 device or a HIP call failed";
    case QD_ERR_INTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

int qd_device_check(char *name, int len) {
  Ctx *c = nullptr;
  int rc = get_ctx(&c);
  if (name && len > 0) {
    name[0] = 0;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
      std::strncpy(name, prop.gcnArchName, size_t(len - 1));
      name[len - 1] = 0;
    }
  }
  return rc;
}

int qd_valu_peak(double *lane_ops_per_s) {
  if (!lane_ops_per_s) return QD_ERR_INVALID;
  Ctx *cp = nullptr;
  int rc = get_ctx(&cp);
  if (rc) return rc;
  Ctx &c = *cp;
  std::lock_guard<std::mutex> lk(c.mu);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return QD_ERR_DEVICE;
  const uint32_t blocks = uint32_t(cus) * 8, iters = 20000;
  DevBuf out;
  if (!out.ensure(size_t(blocks) * 256 * 4)) return QD_ERR_NOMEM;
  if (launch_valu(blocks, 100, out.as<uint32_t>(), c.own) != hipSuccess) return QD_ERR_DEVICE;
  float ms = 0.f;
  if (hipEventRecord(c.e0, c.own) != hipSuccess || launch_valu(blocks, iters, out.as<uint32_t>(), c.own) != hipSuccess ||
      hipEventRecord(c.e1, c.own) != hipSuccess || hipEventSynchronize(c.e1) != hipSuccess ||
      hipEventElapsedTime(&ms, c.e0, c.e1) != hipSuccess)
    return QD_ERR_DEVICE;
  (void)hipFree(out.p);
  const double ops = double(blocks) * 256.0 * double(iters) * 32.0;  // 8 chains x 4 ops
  *lane_ops_per_s = ops / (double(ms) * 1e-3);
  return QD_OK;
}

}  // extern "C"

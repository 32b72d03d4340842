// host.cpp -- input handling, diagonalizations and planning (host only).
#include "host.hpp"

#include <algorithm>
#include <cmath>

#include "../../include/qdist.h"

namespace qd {

int rweight(const BRow &a) {
  return __builtin_popcountll(a.x[0] | a.z[0]) + __builtin_popcountll(a.x[1] | a.z[1]);
}

static inline void setbit(uint64_t *w, int q) { w[q >> 6] |= uint64_t(1) << (q & 63); }

int load_rows(const uint8_t *G, int m, int n, int field, std::vector<BRow> &rows) {
  if (n <= 0 || m < 0 || (m > 0 && !G)) return QD_ERR_INVALID;
  if (n > kMaxN) return QD_ERR_TOO_LARGE;
  rows.clear();
  if (field == QD_FIELD_F2) {
    rows.resize(m);
    for (int i = 0; i < m; ++i) {
      const uint8_t *g = G + size_t(i) * 2 * n;
      for (int q = 0; q < n; ++q) {
        if (g[q] > 1 || g[n + q] > 1) return QD_ERR_INVALID;
        if (g[q]) setbit(rows[i].x, q);
        if (g[n + q]) setbit(rows[i].z, q);
      }
    }
    return QD_OK;
  }
  if (field != QD_FIELD_F4) return QD_ERR_INVALID;
  // a + alpha b and alpha (a + alpha b) = b + alpha (a + b).
  rows.resize(size_t(2) * m);
  for (int i = 0; i < m; ++i) {
    const uint8_t *g = G + size_t(i) * n;
    BRow &u = rows[2 * i], &v = rows[2 * i + 1];
    for (int q = 0; q < n; ++q) {
      if (g[q] > 3) return QD_ERR_INVALID;
      bool a = g[q] & 1, b = (g[q] >> 1) & 1;
      if (a) setbit(u.x, q);
      if (b) { setbit(u.z, q); setbit(v.x, q); }
      if (a != b) setbit(v.z, q);
    }
  }
  return QD_OK;
}

// Bit c of the 2n-bit row: c < n is x_c, else z_{c-n}.
static inline int rbit(const BRow &r, int c, int n) {
  if (c < n) return int((r.x[c >> 6] >> (c & 63)) & 1);
  c -= n;
  return int((r.z[c >> 6] >> (c & 63)) & 1);
}

int make_basis(std::vector<BRow> &rows, int n) {
  int k = 0;
  const int m = int(rows.size());
  for (int c = 0; c < 2 * n && k < m; ++c) {
    int p = k;
    while (p < m && !rbit(rows[p], c, n)) ++p;
    if (p == m) continue;
    std::swap(rows[k], rows[p]);
    for (int i = k + 1; i < m; ++i)
      if (rbit(rows[i], c, n)) radd(rows[i], rows[k]);
    ++k;
  }
  rows.resize(k);
  return k;
}

namespace {

// Kind of column q over the candidate rows: 2 if two different nonzero
// symbols occur, 1 if exactly one, 0 if none.
int column_kind(const std::vector<BRow> &w, const std::vector<char> &cand, int q) {
  unsigned seen = 0;
  for (size_t v = 0; v < w.size(); ++v)
    if (cand[v]) seen |= 1u << qsym(w[v], q);
  seen &= 0xEu;
  int c = __builtin_popcount(seen);
  return c >= 2 ? 2 : c;
}

struct PkIdx {
  int dim, pivot, r, s;
};

// Package selection, Sec. 2.3: columns with two different nonzero symbols
// first, then one; the chosen rows clear the column in every row of
// `scope` (to 0 for a two-row package, to {0, beta} for a one-row one).
void greedy_pass(std::vector<BRow> &w, std::vector<char> &cand, const std::vector<char> &scope,
                 const std::vector<char> &cols, int n, bool outside, std::vector<PkIdx> &out) {
  std::vector<char> done(n, 0), used(w.size(), 0);
  for (;;) {
    int q1 = -1, q2 = -1;
    for (int q = 0; q < n && q2 < 0; ++q) {
      if (!cols[q] || done[q]) continue;
      int k = column_kind(w, cand, q);
      if (k == 2) q2 = q;
      else if (k == 1 && q1 < 0) q1 = q;
    }
    const int q = q2 >= 0 ? q2 : q1;
    if (q < 0) break;
    const int dim = q2 >= 0 ? 2 : 1;
    done[q] = 1;
    int r = -1, s = -1;
    for (size_t v = 0; v < w.size() && r < 0; ++v)
      if (cand[v] && qsym(w[v], q)) r = int(v);
    const int sr = qsym(w[r], q);
    if (dim == 2) {
      for (size_t v = 0; v < w.size() && s < 0; ++v)
        if (cand[v] && qsym(w[v], q) && qsym(w[v], q) != sr) s = int(v);
      const int ss = qsym(w[s], q);
      BRow rs = w[r];
      radd(rs, w[s]);
      for (size_t v = 0; v < w.size(); ++v) {
        if (int(v) == r || int(v) == s || !scope[v]) continue;
        const int sv = qsym(w[v], q);
        if (sv == sr) radd(w[v], w[r]);
        else if (sv == ss) radd(w[v], w[s]);
        else if (sv) radd(w[v], rs);
      }
      cand[r] = cand[s] = 0;
      used[r] = used[s] = 1;
    } else {
      const int beta = (sr % 3) + 1;  // any nonzero symbol other than sr
      for (size_t v = 0; v < w.size(); ++v) {
        if (int(v) == r || !scope[v]) continue;
        const int sv = qsym(w[v], q);
        if (cand[v] ? sv == sr : (used[v] && (sv == sr || sv == (sr ^ beta)))) radd(w[v], w[r]);
      }
      cand[r] = 0;
      used[r] = 1;
    }
    out.push_back({dim, outside ? -1 : q, r, s});
  }
}

Gamma to_gamma(const std::vector<BRow> &w, const std::vector<PkIdx> &idx) {
  Gamma g;
  for (const PkIdx &p : idx) {
    Package pk;
    pk.dim = p.dim;
    pk.pivot = p.pivot;
    pk.r = w[p.r];
    if (p.dim == 2) pk.s = w[p.s];
    g.delta += p.pivot < 0;
    g.pk.push_back(pk);
  }
  return g;
}

}  // namespace

std::vector<Gamma> build_f4(const std::vector<BRow> &basis, int n, int max_gamma) {
  std::vector<Gamma> out;
  std::vector<char> taken(n, 0);
  const size_t k = basis.size();
  for (int j = 0; j < max_gamma; ++j) {
    std::vector<char> cols(n), all(n, 1);
    bool any = false;
    for (int q = 0; q < n; ++q) { cols[q] = !taken[q]; any = any || cols[q]; }
    if (!any) break;
    std::vector<BRow> w = basis;
    std::vector<char> cand(k, 1), scope(k, 1);
    std::vector<PkIdx> idx;
    greedy_pass(w, cand, scope, cols, n, false, idx);
    // Rows left over are zero on the allowed qubits: they still have to be
    // enumerated, as packages that add nothing to the bound.
    std::vector<char> left = cand;
    greedy_pass(w, cand, left, all, n, true, idx);
    Gamma g = to_gamma(w, idx);
    if (g.inside() == 0) break;
    for (const Package &p : g.pk)
      if (p.pivot >= 0) taken[p.pivot] = 1;
    out.push_back(std::move(g));
  }
  return out;
}

Gamma build_f2(const std::vector<BRow> &basis, int n) {
  std::vector<BRow> w = basis;
  const int k = int(w.size());
  std::vector<char> rem(k, 1);
  std::vector<int> first(n, -1), second(n, -1), half(n, 0);
  // [I | M1 ; 0 | M2]: a pivot on x_q, else (x <-> z swap) on z_q.
  for (int q = 0; q < n; ++q) {
    for (int h = 0; h < 2 && first[q] < 0; ++h) {
      const int c = h * n + q;
      int r = -1;
      for (int v = 0; v < k && r < 0; ++v)
        if (rem[v] && rbit(w[v], c, n)) r = v;
      if (r < 0) continue;
      for (int v = 0; v < k; ++v)
        if (v != r && rbit(w[v], c, n)) radd(w[v], w[r]);
      rem[r] = 0;
      first[q] = r;
      half[q] = h;
    }
  }
  // Reduced echelon form of M2 on the z-columns of x-pivoted qubits; each
  // pivot clears the whole qubit column in every other row.
  for (int q = 0; q < n; ++q) {
    if (first[q] < 0 || half[q] != 0) continue;
    int r = -1;
    for (int v = 0; v < k && r < 0; ++v)
      if (rem[v] && rbit(w[v], n + q, n)) r = v;
    if (r < 0) continue;
    for (int v = 0; v < k; ++v)
      if (v != r && rbit(w[v], n + q, n)) radd(w[v], w[r]);
    rem[r] = 0;
    second[q] = r;
  }
  Gamma g;
  for (int q = 0; q < n; ++q) {
    if (first[q] < 0) continue;
    Package pk;
    pk.pivot = q;
    pk.r = w[first[q]];
    if (second[q] >= 0) {
      pk.dim = 2;
      pk.s = w[second[q]];
    }
    g.pk.push_back(pk);
  }
  return g;
}

bool check_gamma(const Gamma &g, int n) {
  (void)n;
  std::vector<char> seen(kMaxN, 0);
  for (size_t i = 0; i < g.pk.size(); ++i) {
    const Package &p = g.pk[i];
    if (p.pivot < 0) continue;
    if (seen[p.pivot]) return false;
    seen[p.pivot] = 1;
    const int q = p.pivot, sr = qsym(p.r, q);
    if (!sr) return false;
    if (p.dim == 2 && (!qsym(p.s, q) || qsym(p.s, q) == sr)) return false;
    unsigned other = 0;
    for (size_t j = 0; j < g.pk.size(); ++j) {
      if (j == i) continue;
      other |= 1u << qsym(g.pk[j].r, q);
      if (g.pk[j].dim == 2) other |= 1u << qsym(g.pk[j].s, q);
    }
    other &= 0xEu;
    if (p.dim == 2 && other) return false;
    if (p.dim == 1 && (__builtin_popcount(other) > 1 || (other >> sr) & 1)) return false;
  }
  return true;
}

static inline uint64_t sat_add(uint64_t a, uint64_t b) { return (a + b > kSat) ? kSat : a + b; }
static inline uint64_t sat_mul(uint64_t a, int c) { return a > kSat / 3 ? kSat : std::min<uint64_t>(a * c, kSat); }

void esym_tables(const std::vector<int> &sizes, int rmax, std::vector<uint64_t> &prefix,
                 std::vector<uint64_t> &suffix) {
  const int P = int(sizes.size()), R = rmax + 1;
  prefix.assign(size_t(P + 1) * R, 0);
  suffix.assign(size_t(P + 1) * R, 0);
  prefix[0] = 1;
  for (int h = 0; h < P; ++h)
    for (int r = 0; r < R; ++r)
      prefix[size_t(h + 1) * R + r] =
          sat_add(prefix[size_t(h) * R + r], r ? sat_mul(prefix[size_t(h) * R + r - 1], sizes[h]) : 0);
  suffix[size_t(P) * R] = 1;
  for (int h = P - 1; h >= 0; --h)
    for (int r = 0; r < R; ++r)
      suffix[size_t(h) * R + r] = sat_add(
          suffix[size_t(h + 1) * R + r], r ? sat_mul(suffix[size_t(h + 1) * R + r - 1], sizes[h]) : 0);
}

uint64_t esym(const std::vector<int> &sizes, int t) {
  std::vector<uint64_t> e(t + 1, 0);
  e[0] = 1;
  for (int c : sizes)
    for (int r = t; r > 0; --r) e[r] = sat_add(e[r], sat_mul(e[r - 1], c));
  return e[t];
}

static double esym_d(const std::vector<int> &sizes, int t) {
  std::vector<double> e(t + 1, 0.0);
  e[0] = 1.0;
  for (int c : sizes)
    for (int r = t; r > 0; --r) e[r] += e[r - 1] * c;
  return e[t];
}

int lower_bound(const std::vector<int> &tdone, const std::vector<int> &delta) {
  int L = 0;
  for (size_t j = 0; j < tdone.size(); ++j) L += std::max(0, tdone[j] + 1 - delta[j]);
  return L;
}

int estimate_distance(int n, int k, int upper) {
  // log2 of the expected number of nonzero codewords of weight <= w in a
  // random code of 2^k words inside the 4^n symplectic space.
  double lk = k >= 60 ? double(k) : std::log2(std::ldexp(1.0, k) - 1.0);
  double acc = 0.0;
  for (int w = 1; w <= n; ++w) {
    double lc = (std::lgamma(n + 1.0) - std::lgamma(w + 1.0) - std::lgamma(n - w + 1.0)) / std::log(2.0) +
                w * std::log2(3.0);
    acc += std::exp2(lc - 2.0 * n + lk);
    if (acc >= 1.0) return std::max(1, std::min(upper, w));
  }
  return std::max(1, std::min(upper, n));
}

static std::vector<int> sizes_of(const Gamma &g) {
  std::vector<int> s;
  for (const Package &p : g.pk) s.push_back(p.dim == 2 ? 3 : 1);
  return s;
}

double predict_work(const std::vector<Gamma> &gs, int h, int d_est) {
  std::vector<int> tdone(h, 0), delta(h);
  std::vector<std::vector<int>> sz(h);
  for (int j = 0; j < h; ++j) {
    delta[j] = gs[j].delta;
    sz[j] = sizes_of(gs[j]);
  }
  if (lower_bound(tdone, delta) >= d_est) return 0.0;
  double w = 0.0;
  for (int t = 1; t <= kMaxN * 2; ++t) {
    for (int j = 0; j < h; ++j) {
      if (t > gs[j].P()) continue;
      w += esym_d(sz[j], t);
      tdone[j] = t;
      if (lower_bound(tdone, delta) >= d_est || t == gs[j].P()) return w;
    }
  }
  return w;
}

PlanChoice choose_plan(const std::vector<Gamma> &f4, const Gamma &f2, int n, int rank, int diag_req,
                       int max_gamma_req) {
  int upper = n;
  auto probe = [&](const Gamma &g) {
    for (const Package &p : g.pk) {
      upper = std::min(upper, rweight(p.r));
      if (p.dim == 2) {
        BRow rs = p.r;
        radd(rs, p.s);
        upper = std::min({upper, rweight(p.s), rweight(rs)});
      }
    }
  };
  for (const Gamma &g : f4) probe(g);
  probe(f2);
  PlanChoice pc;
  pc.d_est = estimate_distance(n, rank, upper);
  const int hmax = max_gamma_req > 0 ? std::min<int>(max_gamma_req, int(f4.size())) : int(f4.size());
  double best = -1.0;
  pc.predicted_f4 = -1.0;
  if (diag_req != QD_DIAG_F2) {
    for (int h = 1; h <= hmax; ++h) {
      double w = predict_work(f4, h, pc.d_est);
      if (pc.predicted_f4 < 0 || w < pc.predicted_f4) pc.predicted_f4 = w;
      if (best < 0 || w < best) {
        best = w;
        pc.diag = QD_DIAG_F4;
        pc.h_used = h;
      }
    }
  }
  pc.predicted_f2 = predict_work(std::vector<Gamma>{f2}, 1, pc.d_est);
  if (diag_req != QD_DIAG_F4 && (best < 0 || pc.predicted_f2 < best)) {
    best = pc.predicted_f2;
    pc.diag = QD_DIAG_F2;
    pc.h_used = 1;
  }
  pc.predicted = best;
  return pc;
}

}  // namespace qd

// host.cpp -- input handling, diagonalizations and planning (host only).
#include "host.hpp"

#include <algorithm>
#include <cmath>

#include "../../include/qdist.h"

namespace qd {

int rweight(const BRow &a) {
  return __builtin_popcountll(a.x[0] | a.z[0]) + __builtin_popcountll(a.x[1] | a.z[1]);
}


int load_rows(const uint8_t *G, int m, int n, int field, std::vector<BRow> &rows) {
  if (n <= 0 || m < 0 || (m > 0 && !G)) return QD_ERR_INVALID;
  if (n > kMaxN) return QD_ERR_TOO_LARGE;
  rows.clear();
  if (field == QD_FIELD_F2) {
    rows.resize(m);
    unsigned bad = 0;  // any byte above 1
    for (int i = 0; i < m; ++i) {
      const uint8_t *g = G + size_t(i) * 2 * n;
      for (int q = 0; q < n; ++q) {
        bad |= unsigned(g[q] | g[n + q]);
        rows[i].x[q >> 6] |= uint64_t(g[q] & 1) << (q & 63);
        rows[i].z[q >> 6] |= uint64_t(g[n + q] & 1) << (q & 63);
      }
    }
    return bad > 1 ? QD_ERR_INVALID : QD_OK;
  }
  if (field != QD_FIELD_F4) return QD_ERR_INVALID;
  // a + alpha b and alpha (a + alpha b) = b + alpha (a + b).
  rows.resize(size_t(2) * m);
  unsigned bad = 0;  // any byte above 3
  for (int i = 0; i < m; ++i) {
    const uint8_t *g = G + size_t(i) * n;
    BRow &u = rows[2 * i], &v = rows[2 * i + 1];
    for (int q = 0; q < n; ++q) {
      bad |= g[q];
      const uint64_t a = g[q] & 1, b = (g[q] >> 1) & 1, bit = uint64_t(1) << (q & 63);
      u.x[q >> 6] |= a ? bit : 0;
      u.z[q >> 6] |= b ? bit : 0;
      v.x[q >> 6] |= b ? bit : 0;
      v.z[q >> 6] |= (a ^ b) ? bit : 0;
    }
  }
  return bad > 3 ? QD_ERR_INVALID : QD_OK;
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

struct PkIdx {
  int dim, pivot, r, s;
};

// Package selection, Sec. 2.3: columns with two different nonzero symbols
// first, then one; the chosen rows clear the column in every row of
// `scope` (to 0 for a two-row package, to {0, beta} for a one-row one).
// With max2 >= 0, after max2 two-row packages every further package has
// one row, taken at the first column where some candidate row is nonzero.
void greedy_pass(std::vector<BRow> &w, std::vector<char> &cand, const std::vector<char> &scope,
                 const std::vector<char> &cols, int n, bool outside, std::vector<PkIdx> &out, int max2 = -1) {
  std::vector<char> used(w.size(), 0);
  int n2 = 0;
  uint64_t avail[2] = {0, 0};  // allowed qubits not pivoted yet
  for (int q = 0; q < n; ++q)
    if (cols[q]) avail[q >> 6] |= uint64_t(1) << (q & 63);
  for (;;) {
    // Per qubit, which nonzero symbols (x only, z only, both) the candidate
    // rows show; two different ones make a two-row column.
    uint64_t sx[2] = {0, 0}, sz[2] = {0, 0}, sy[2] = {0, 0};
    for (size_t v = 0; v < w.size(); ++v) {
      if (!cand[v]) continue;
      for (int i = 0; i < 2; ++i) {
        sx[i] |= w[v].x[i] & ~w[v].z[i];
        sz[i] |= w[v].z[i] & ~w[v].x[i];
        sy[i] |= w[v].x[i] & w[v].z[i];
      }
    }
    uint64_t k2[2], k1[2];
    for (int i = 0; i < 2; ++i) {
      const uint64_t two = (sx[i] & sz[i]) | (sx[i] & sy[i]) | (sz[i] & sy[i]);
      k2[i] = two & avail[i];
      k1[i] = (sx[i] | sz[i] | sy[i]) & ~two & avail[i];
    }
    auto first = [](const uint64_t *a) { return a[0] ? __builtin_ctzll(a[0]) : a[1] ? 64 + __builtin_ctzll(a[1]) : -1; };
    const bool allow2 = max2 < 0 || n2 < max2;
    if (!allow2)
      for (int i = 0; i < 2; ++i) k1[i] |= k2[i];
    const int q2 = allow2 ? first(k2) : -1, q = q2 >= 0 ? q2 : first(k1);
    if (q < 0) break;
    const int dim = q2 >= 0 ? 2 : 1;
    avail[q >> 6] &= ~(uint64_t(1) << (q & 63));
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
      ++n2;
    } else {
      // Every other row ends with 0 or beta at q: sr + sr = 0 and
      // (sr ^ beta) + sr = beta.  Candidates show only sr at a one-symbol
      // column; past the two-row cap they may show all three symbols.
      const int beta = sr == 1 ? 2 : 1;  // a nonzero symbol other than sr
      for (size_t v = 0; v < w.size(); ++v) {
        if (int(v) == r || !scope[v]) continue;
        const int sv = qsym(w[v], q);
        if ((cand[v] || used[v]) && (sv == sr || sv == (sr ^ beta))) radd(w[v], w[r]);
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

std::vector<Gamma> build_f4(const std::vector<BRow> &basis, int n, int max_gamma, const std::vector<int> &max2) {
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
    greedy_pass(w, cand, scope, cols, n, false, idx, j < int(max2.size()) ? max2[j] : -1);
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
  // Per package, the qubits where its rows show symbol 1 (x only), 2 (z
  // only) and 3 (both); prefix and suffix unions give every other
  // package's symbols at a pivot in O(1).
  struct Sym {
    uint64_t s[3][2];
  };
  const size_t P = g.pk.size();
  auto sym_of = [](const BRow &r, Sym &m) {
    for (int i = 0; i < 2; ++i) {
      m.s[0][i] |= r.x[i] & ~r.z[i];
      m.s[1][i] |= r.z[i] & ~r.x[i];
      m.s[2][i] |= r.x[i] & r.z[i];
    }
  };
  std::vector<Sym> pre(P + 1, Sym{}), suf(P + 1, Sym{});
  for (size_t j = 0; j < P; ++j) {
    Sym m{};
    sym_of(g.pk[j].r, m);
    if (g.pk[j].dim == 2) sym_of(g.pk[j].s, m);
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < 2; ++i) pre[j + 1].s[a][i] = pre[j].s[a][i] | m.s[a][i];
  }
  for (size_t j = P; j-- > 0;) {
    Sym m{};
    sym_of(g.pk[j].r, m);
    if (g.pk[j].dim == 2) sym_of(g.pk[j].s, m);
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < 2; ++i) suf[j].s[a][i] = suf[j + 1].s[a][i] | m.s[a][i];
  }
  std::vector<char> seen(kMaxN, 0);
  for (size_t i = 0; i < P; ++i) {
    const Package &p = g.pk[i];
    if (p.pivot < 0) continue;
    if (seen[p.pivot]) return false;
    seen[p.pivot] = 1;
    const int q = p.pivot, sr = qsym(p.r, q);
    if (!sr) return false;
    if (p.dim == 2 && (!qsym(p.s, q) || qsym(p.s, q) == sr)) return false;
    unsigned other = 0;  // nonzero symbols of the other packages' rows at q
    for (int a = 0; a < 3; ++a)
      if (((pre[i].s[a][q >> 6] | suf[i + 1].s[a][q >> 6]) >> (q & 63)) & 1) other |= 2u << a;
    if (p.dim == 2 && other) return false;
    if (p.dim == 1 && (__builtin_popcount(other) > 1 || (other >> sr) & 1)) return false;
  }
  return true;
}

int sym_product(const BRow &a, const BRow &b) {
  uint64_t v = 0;
  for (int i = 0; i < 2; ++i) v ^= (a.x[i] & b.z[i]) ^ (a.z[i] & b.x[i]);
  return __builtin_parityll(v);
}

int logical_pairs(const std::vector<BRow> &basis, std::vector<BRow> &out) {
  out.clear();
  std::vector<BRow> rem = basis;
  size_t head = 0;
  while (head < rem.size()) {
    const BRow a = rem[head++];
    size_t j = head;
    while (j < rem.size() && !sym_product(a, rem[j])) ++j;
    if (j == rem.size()) continue;  // a commutes with the whole span: radical
    const BRow b = rem[j];
    rem.erase(rem.begin() + long(j));
    // r + <r, b> a + <r, a> b commutes with both a and b.
    for (size_t i = head; i < rem.size(); ++i) {
      const int pa = sym_product(rem[i], a), pb = sym_product(rem[i], b);
      if (pb) radd(rem[i], a);
      if (pa) radd(rem[i], b);
    }
    out.push_back(a);
    out.push_back(b);
  }
  return int(out.size() / 2);
}

int iso_bit(const BRow &r, int c, int n) {
  if (c < 2 * n) return rbit(r, c, n);
  return rbit(r, c - 2 * n, n) ^ rbit(r, c - n, n);
}

std::vector<Gamma> build_iso(const std::vector<BRow> &basis, int n, int max_gamma) {
  const int k = int(basis.size()), KW = (k + 63) / 64, C = 3 * n;
  std::vector<char> used(C, 0);
  std::vector<Gamma> out;
  // Image columns of a row, as (column, ...) callbacks: x bits at q, z bits
  // at n + q, x^z bits at 2n + q.
  auto for_image_bits = [n](const BRow &r, auto &&f) {
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < 2; ++i) {
        uint64_t v = b == 0 ? r.x[i] : b == 1 ? r.z[i] : (r.x[i] ^ r.z[i]);
        while (v) {
          const int q = 64 * i + __builtin_ctzll(v);
          v &= v - 1;
          if (q < n) f(b * n + q);
        }
      }
  };
  while (int(out.size()) < max_gamma) {
    std::vector<BRow> w = basis;
    std::vector<int> piv(k, -1);
    // col[c * KW + i]: the rows whose image has a 1 in column c.
    std::vector<uint64_t> col(size_t(C) * KW, 0), pivoted(KW, 0), S(KW);
    for (int v = 0; v < k; ++v)
      for_image_bits(w[v], [&](int c) { col[size_t(c) * KW + (v >> 6)] |= uint64_t(1) << (v & 63); });
    int pivots = 0;
    for (int c = 0; c < C && pivots < k; ++c) {
      if (used[c]) continue;
      int p = -1;
      for (int i = 0; i < KW && p < 0; ++i) {
        const uint64_t f = col[size_t(c) * KW + i] & ~pivoted[i];
        if (f) p = 64 * i + __builtin_ctzll(f);
      }
      if (p < 0) continue;
      piv[p] = c;
      pivoted[p >> 6] |= uint64_t(1) << (p & 63);
      ++pivots;
      // Clear column c in every other row; their images change by row p's.
      bool any = false;
      for (int i = 0; i < KW; ++i) {
        S[i] = col[size_t(c) * KW + i] & ~(i == (p >> 6) ? uint64_t(1) << (p & 63) : 0);
        any = any || S[i];
      }
      if (!any) continue;
      for (int i = 0; i < KW; ++i)
        for (uint64_t v = S[i]; v; v &= v - 1) radd(w[64 * i + __builtin_ctzll(v)], w[p]);
      for_image_bits(w[p], [&](int c2) {
        for (int i = 0; i < KW; ++i) col[size_t(c2) * KW + i] ^= S[i];
      });
    }
    if (pivots == 0) break;
    Gamma g;
    for (int v = 0; v < k; ++v) {
      Package pk;
      pk.pivot = piv[v];
      pk.r = w[v];
      g.pk.push_back(pk);
      if (piv[v] >= 0) used[piv[v]] = 1;
      else ++g.delta;
    }
    out.push_back(g);
  }
  return out;
}

bool check_gamma_iso(const Gamma &g, int n) {
  std::vector<char> seen(3 * kMaxN, 0);
  int delta = 0;
  for (size_t i = 0; i < g.pk.size(); ++i) {
    const Package &p = g.pk[i];
    if (p.dim != 1) return false;
    if (p.pivot < 0) { ++delta; continue; }
    if (p.pivot >= 3 * n || seen[p.pivot] || !iso_bit(p.r, p.pivot, n)) return false;
    seen[p.pivot] = 1;
    for (size_t j = 0; j < g.pk.size(); ++j)
      if (j != i && iso_bit(g.pk[j].r, p.pivot, n)) return false;
  }
  return delta == g.delta;
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

int lower_bound(const std::vector<int> &tdone, const std::vector<int> &delta, bool halve) {
  int L = 0;
  for (size_t j = 0; j < tdone.size(); ++j) L += std::max(0, tdone[j] + 1 - delta[j]);
  return halve ? (L + 1) / 2 : L;
}

int estimate_distance(int n, int k, int upper) {
  // log2 of the expected number of nonzero codewords of weight <= w in a
  // random code of 2^k words inside the 4^n symplectic space; lc(w) =
  // log2(C(n, w) 3^w), updated from w - 1.
  const double lk = k >= 60 ? double(k) : std::log2(std::ldexp(1.0, k) - 1.0);
  const double l3 = std::log2(3.0);
  double acc = 0.0, lc = 0.0;
  for (int w = 1; w <= n; ++w) {
    lc += std::log2(double(n - w + 1) / double(w)) + l3;
    acc += std::exp2(lc - 2.0 * n + lk);
    if (acc >= 1.0) return std::max(1, std::min(upper, w));
  }
  return std::max(1, std::min(upper, n));
}

// e_t(sizes) as doubles for t = 0..P, one table per matrix.
static std::vector<double> esym_all(const Gamma &g) {
  std::vector<double> e(g.P() + 1, 0.0);
  e[0] = 1.0;
  for (const Package &p : g.pk) {
    const double c = p.dim == 2 ? 3.0 : 1.0;
    for (int r = g.P(); r > 0; --r) e[r] += e[r - 1] * c;
  }
  return e;
}

static double predict_with(const std::vector<Gamma> &gs, const std::vector<std::vector<double>> &E, int h,
                           int d_est, bool halve) {
  // The bound of lower_bound(), kept as it grows: finishing round t of
  // matrix j adds max(0, t + 1 - delta_j) - max(0, t - delta_j), i.e. 1
  // when t >= delta_j.
  int Lraw = 0;
  for (int j = 0; j < h; ++j) Lraw += std::max(0, 1 - gs[j].delta);
  auto bound = [&] { return halve ? (Lraw + 1) / 2 : Lraw; };
  if (bound() >= d_est) return 0.0;
  double w = 0.0;
  for (int t = 1; t <= kMaxN * 2; ++t) {
    for (int j = 0; j < h; ++j) {
      if (t > gs[j].P()) continue;
      w += E[j][t];
      if (t >= gs[j].delta) ++Lraw;
      if (bound() >= d_est || t == gs[j].P()) return w;
    }
  }
  return w;
}

double predict_work(const std::vector<Gamma> &gs, int h, int d_est, bool halve) {
  std::vector<std::vector<double>> E;
  for (int j = 0; j < h; ++j) E.push_back(esym_all(gs[j]));
  return predict_with(gs, E, h, d_est, halve);
}

double iso_work_floor(int n, int rank, int d_est) {
  // Information sets are disjoint subsets of the 3n image columns with at
  // most `rank` columns each, so after round t the Hamming bound is at most
  // full * (t + 1) + max(0, t + 1 - (rank - rest)); it must reach
  // 2 d_est - 1 (the bound is halved, rounding up).
  if (rank <= 0) return 0.0;
  const int full = 3 * n / rank, rest = 3 * n % rank, need = 2 * d_est - 1;
  for (int t = 0; t <= rank; ++t) {
    const int L = full * (t + 1) + std::max(0, t + 1 - (rank - rest));
    if (L >= need) {
      if (t == 0) return 0.0;
      double c = 1.0;  // C(rank, t): the least work of a round t on one matrix
      for (int i = 1; i <= t; ++i) c = c * double(rank - t + i) / double(i);
      return c;
    }
  }
  return 0.0;
}

bool alpha_closed(const std::vector<BRow> &basis, int n) {
  // In row echelon form every row's first nonzero column (x columns, then
  // z) is zero in the rows below it, so reducing by the rows in order
  // clears each pivot for good: v is in the span exactly when it ends zero.
  std::vector<int> piv(basis.size(), -1);
  for (size_t k = 0; k < basis.size(); ++k)
    for (int c = 0; c < 2 * n && piv[k] < 0; ++c)
      if (rbit(basis[k], c, n)) piv[k] = c;
  for (const BRow &b : basis) {
    BRow v = alpha_row(b);
    for (size_t k = 0; k < basis.size(); ++k)
      if (piv[k] >= 0 && rbit(v, piv[k], n)) radd(v, basis[k]);
    if (!rzero(v)) return false;  // a generic binary code fails at the first row
  }
  return true;
}

bool make_scalar_orbits(std::vector<Gamma> &gs) {
  for (const Gamma &g : gs)
    for (const Package &p : g.pk)
      if (p.dim != 2) return false;
  for (Gamma &g : gs)
    for (Package &p : g.pk) p.s = alpha_row(p.r);
  return true;
}

PlanChoice choose_plan(const std::vector<Gamma> &f4, const Gamma &f2, const std::vector<Gamma> &iso, int n,
                       int rank, int diag_req, int max_gamma_req, bool f4_scalar) {
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
  for (const Gamma &g : iso) probe(g);
  PlanChoice pc;
  pc.d_est = estimate_distance(n, rank, upper);
  double best = -1.0;
  // Matrices 1..h of one construction, for the h with the least work.
  auto consider = [&](const std::vector<Gamma> &gs, int diag, bool halve, double *pred) {
    const int hmax = max_gamma_req > 0 ? std::min<int>(max_gamma_req, int(gs.size())) : int(gs.size());
    std::vector<std::vector<double>> E;
    for (int j = 0; j < hmax; ++j) {
      E.push_back(esym_all(gs[j]));
      if (diag == QD_DIAG_F4 && f4_scalar)
        for (double &e : E.back()) e /= 3.0;
    }
    *pred = -1.0;
    for (int h = 1; h <= hmax; ++h) {
      const double w = predict_with(gs, E, h, pc.d_est, halve);
      if (*pred < 0 || w < *pred) *pred = w;
      if (diag_req != QD_DIAG_AUTO && diag_req != diag) continue;
      if (best < 0 || w < best) {
        best = w;
        pc.diag = diag;
        pc.h_used = h;
      }
    }
  };
  consider(f4, QD_DIAG_F4, false, &pc.predicted_f4);
  consider(std::vector<Gamma>{f2}, QD_DIAG_F2, false, &pc.predicted_f2);
  if (!iso.empty()) {
    // The isometry brings more matrices (tables, uploads, rounds), so the
    // automatic choice takes it only for a clear saving of real work.
    const PlanChoice other = pc;
    const double other_best = best;
    consider(iso, QD_DIAG_ISO, true, &pc.predicted_iso);
    if (diag_req == QD_DIAG_AUTO && pc.diag == QD_DIAG_ISO &&
        !(other_best >= kIsoMinWork && best < kIsoMargin * other_best)) {
      const double p_iso = pc.predicted_iso;
      pc = other;
      pc.predicted_iso = p_iso;
      best = other_best;
    }
  }
  pc.predicted = best;
  return pc;
}

// -- mixed packages --------------------------------------------------------------

std::vector<std::vector<int>> mixed_caps(int n, int rank, int d_est, int count) {
  std::vector<std::pair<double, std::vector<int>>> found;
  const int m = rank, slack = 2 * (n - m);
  if (m < 2 || slack <= 0 || d_est <= 2) return {};
  auto esym_d = [](int a, int b, int tmax) {
    std::vector<double> e(tmax + 1, 0.0);
    e[0] = 1.0;
    for (int i = 0; i < a + b; ++i) {
      const double c = i < a ? 3.0 : 1.0;
      for (int t = tmax; t > 0; --t) e[t] += e[t - 1] * c;
    }
    return e;
  };
  const int tmax = std::min(m, d_est);
  std::vector<std::vector<double>> E(m + 1);
  for (int b = m % 2; b <= std::min(m, slack); b += 2) E[b] = esym_d((m - b) / 2, b, tmax);
  for (int b1 = m % 2; b1 <= std::min(m, slack); b1 += 2)
    for (int b2 = m % 2; b2 <= std::min(m, slack); b2 += 2) {
      const int a1 = (m - b1) / 2, a2 = (m - b2) / 2;
      if (a1 + b1 + a2 + b2 > n || (b1 == m % 2 && b2 == m % 2)) continue;
      double w = 0.0;
      int L = 2;
      for (int t = 1; t <= tmax && L < d_est; ++t) {
        w += E[b1][t];
        if (++L >= d_est) break;
        w += E[b2][t];
        ++L;
      }
      found.push_back({w, {a1, a2}});
    }
  std::sort(found.begin(), found.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
  std::vector<std::vector<int>> out;
  for (size_t i = 0; i < found.size() && int(out.size()) < count; ++i) out.push_back(found[i].second);
  return out;
}

double best_predicted(const std::vector<Gamma> &gs, int d_est, int max_gamma, bool scalar) {
  const int hmax = max_gamma > 0 ? std::min<int>(max_gamma, int(gs.size())) : int(gs.size());
  std::vector<std::vector<double>> E;
  double best = -1.0;
  for (int j = 0; j < hmax; ++j) {
    E.push_back(esym_all(gs[j]));
    if (scalar)
      for (double &e : E.back()) e /= 3.0;
  }
  for (int h = 1; h <= hmax; ++h) {
    const double w = predict_with(gs, E, h, d_est, false);
    if (best < 0 || w < best) best = w;
  }
  return best;
}

bool try_mixed_f4(const std::vector<BRow> &basis, int n, int rank, int d_est, int max_gamma,
                  std::vector<Gamma> &f4, std::vector<int> &caps) {
  caps.clear();
  double best = best_predicted(f4, d_est, max_gamma, false);
  for (const std::vector<int> &c : mixed_caps(n, rank, d_est, 2)) {
    std::vector<Gamma> gs = build_f4(basis, n, 2, c);
    for (const Gamma &g : gs)
      if (!check_gamma(g, n)) return false;
    const double w = best_predicted(gs, d_est, max_gamma, false);
    if (w >= 0 && w < 0.95 * best) {
      best = w;
      f4 = std::move(gs);
      caps = c;
    }
  }
  return true;
}

// -- partial weights -----------------------------------------------------------

QubitOrder qubit_order(const Gamma &g, int n, bool iso) {
  QubitOrder o;
  std::vector<char> piv(n, 0);
  for (const Package &p : g.pk)
    if (p.pivot >= 0) piv[iso ? p.pivot % n : p.pivot] = 1;
  std::vector<unsigned char> pos(n);
  int k = 0;
  for (int q = 0; q < n; ++q)
    if (!piv[q]) pos[q] = static_cast<unsigned char>(k++);
  o.nonpivot = k;
  for (int q = 0; q < n; ++q)
    if (piv[q]) pos[q] = static_cast<unsigned char>(k++);
  bool identity = true;
  for (int q = 0; q < n; ++q) identity = identity && pos[q] == q;
  for (const Package &p : g.pk) {
    if (p.pivot < 0) continue;
    const int at = pos[iso ? p.pivot % n : p.pivot];
    for (int w = 0; w < 4; ++w) o.kin[w] += at < 32 * (w + 1);
  }
  if (identity) return o;
  o.pos = std::move(pos);
  for (int q = 0; q < n; ++q) {
    if (!o.runs.empty()) {
      QubitOrder::Run &b = o.runs.back();
      if (q == b.src + b.len && o.pos[q] == b.dst + b.len) {
        ++b.len;
        continue;
      }
    }
    o.runs.push_back({q, 1, int(o.pos[q])});
  }
  return o;
}

BRow permute_row(const BRow &r, const QubitOrder &o) {
  if (o.pos.empty()) return r;
  using u128 = unsigned __int128;
  const u128 x = (u128(r.x[1]) << 64) | r.x[0], z = (u128(r.z[1]) << 64) | r.z[0];
  u128 ox = 0, oz = 0;
  for (const QubitOrder::Run &run : o.runs) {
    const u128 m = run.len >= 128 ? ~u128(0) : (u128(1) << run.len) - 1;
    ox |= ((x >> run.src) & m) << run.dst;
    oz |= ((z >> run.src) & m) << run.dst;
  }
  BRow out;
  out.x[0] = uint64_t(ox); out.x[1] = uint64_t(ox >> 64);
  out.z[0] = uint64_t(oz); out.z[1] = uint64_t(oz >> 64);
  return out;
}

int partial_credit(int t, int delta, int kin, bool iso) {
  const int outside = std::max(0, t - delta - kin);
  return iso ? (outside + 1) / 2 : outside;
}

int partial_limit(int q) {
  if (q < 8) return -1;
  return int(std::floor(0.75 * q - 4.0 * std::sqrt(0.1875 * q)));
}

}  // namespace qd

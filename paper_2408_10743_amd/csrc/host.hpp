// host.hpp -- host side of libqdist: input checks, basis, the package-
// systematic generator matrices of the paper's two diagonalizations, the
// lower-bound schedule and the work planner.  No GPU code here.
#pragma once
#include <cstdint>
#include <vector>

namespace qd {

constexpr int kMaxN = 128;   // qubits; two 64-bit words per half
constexpr int kMaxGamma = 8;

// One binary row (x | z) over at most 128 qubits.
struct BRow {
  uint64_t x[2] = {0, 0};
  uint64_t z[2] = {0, 0};
};

inline int qsym(const BRow &r, int q) {  // F4 symbol x + 2z at qubit q
  return int((r.x[q >> 6] >> (q & 63)) & 1) | (int((r.z[q >> 6] >> (q & 63)) & 1) << 1);
}
inline void radd(BRow &a, const BRow &b) {
  a.x[0] ^= b.x[0]; a.x[1] ^= b.x[1]; a.z[0] ^= b.z[0]; a.z[1] ^= b.z[1];
}
// alpha * (x | z) = (z | x ^ z): the F4 scalar alpha on a row (Sec. 2.3
// convention a + alpha b <-> (a | b)).
inline BRow alpha_row(const BRow &r) {
  BRow o;
  for (int i = 0; i < 2; ++i) {
    o.x[i] = r.z[i];
    o.z[i] = r.x[i] ^ r.z[i];
  }
  return o;
}
inline bool rzero(const BRow &a) { return !(a.x[0] | a.x[1] | a.z[0] | a.z[1]); }
int rweight(const BRow &a);  // symplectic weight

// A package: {r} or {r, s, r^s} pivoted on `pivot` (-1: outside the set).
struct Package {
  int dim = 1;
  int pivot = -1;
  BRow r, s;
};

struct Gamma {
  std::vector<Package> pk;
  int delta = 0;  // packages with pivot == -1
  int P() const { return int(pk.size()); }
  int inside() const { return P() - delta; }
};

// Parses a caller matrix into binary rows; F4 rows expand to g, alpha*g.
// Returns QD status (0 ok).
int load_rows(const uint8_t *G, int m, int n, int field, std::vector<BRow> &rows);

// Reduces rows to a basis of their span (row echelon form); returns rank.
int make_basis(std::vector<BRow> &rows, int n);

// Diagonalization over F4 (Sec. 2.3), generalized to several matrices on
// disjoint qubit sets; at most max_gamma matrices, each with >= 1 package
// pivoted inside its own set.  max2[j] >= 0 caps matrix j's two-row
// packages pivoted inside its set: after that many its packages have one
// row each (mixed packages; missing or -1: no cap).
std::vector<Gamma> build_f4(const std::vector<BRow> &basis, int n, int max_gamma,
                            const std::vector<int> &max2 = {});

// Diagonalization over F2 (Sec. 2.2) with whole-qubit clearing: one matrix.
Gamma build_f2(const std::vector<BRow> &basis, int n);

// Checks the package invariants behind the lower bound; true when they hold.
bool check_gamma(const Gamma &g, int n);

// Saved_isometry (Sec. 2.4).  The image (x, z, x^z) of the code is a binary
// code of length 3n with Hamming weight = 2 x symplectic weight.  Matrix j
// is the reduced row echelon form of the basis on the image columns (q,
// n+q, 2n+q for x, z, x^z of qubit q) outside the information sets of the
// earlier matrices, scanned in that order; every package is one row,
// pivoted on its image column or -1 (delta).  At most max_gamma matrices,
// each with >= 1 pivot.  Its bounds count Hamming weight (lower_bound with
// halve = true).
std::vector<Gamma> build_iso(const std::vector<BRow> &basis, int n, int max_gamma);

// Reduced form of an isometry matrix: each pivot row has a 1 on its image
// column, every other row a 0; pivot columns distinct.
bool check_gamma_iso(const Gamma &g, int n);

// Bit of image column c (0 <= c < 3n) of a row.
int iso_bit(const BRow &r, int c, int n);

// Symplectic product <a, b>_s = a_x . b_z + a_z . b_x (mod 2).
int sym_product(const BRow &a, const BRow &b);

// Logical operator pairs of the span of `basis`: rows a_1, b_1, ..., a_k,
// b_k with <a_i, b_i>_s = 1 and every other product 0, spanning a
// complement of the span's radical (the stabilizer, for a normalizer).  A
// codeword of the span lies in the radical exactly when its product with
// every one of them is 0.  Returns k.
int logical_pairs(const std::vector<BRow> &basis, std::vector<BRow> &out);

// F4 scalar classes.  For an F4-linear code every package of the F4
// matrices has two rows; with s replaced by alpha r each package is the
// orbit {r, alpha r, alpha^2 r} (still a basis with the same invariants), so
// fixing the element of one designated package of a combination picks one
// codeword of each class {c, alpha c, alpha^2 c}.  Returns false, leaving
// the matrices unchanged, if some package has one row.
bool make_scalar_orbits(std::vector<Gamma> &gs);

// True when the span of `basis` is closed under alpha (an F4-linear code,
// whatever the input field): alpha times every basis row lies in the span.
// `basis` is in the row echelon form make_basis leaves.
bool alpha_closed(const std::vector<BRow> &basis, int n);

// Partial weights.  A matrix is stored with the qubits that carry none of
// its package pivots first, so the first words of a codeword hold its least
// constrained qubits.  pos[q] is the stored position of qubit q (empty when
// the order is unchanged); kin[w] counts the packages pivoted at stored
// positions below 32 (w + 1).  Isometry pivots are image columns; their
// qubit is the column modulo n.
struct QubitOrder {
  struct Run {
    int src, len, dst;  // qubits src..src+len-1 go to positions dst..dst+len-1
  };
  std::vector<unsigned char> pos;
  std::vector<Run> runs;  // the same map as maximal runs of consecutive qubits
  int nonpivot = 0;
  int kin[4] = {0, 0, 0, 0};
};
QubitOrder qubit_order(const Gamma &g, int n, bool iso);
BRow permute_row(const BRow &r, const QubitOrder &o);

// Lower bound on the weight of a t-package combination of a matrix outside
// its first stored words, of which kin packages are pivoted inside them:
// every chosen package pivoted outside has a nonzero symbol at its own pivot
// qubit (at most delta chosen packages have no pivot).  Pivot qubits are
// distinct, except for the isometry matrices, whose pivot columns are
// linearly independent and so at most two per qubit.
int partial_credit(int t, int delta, int kin, bool iso);

// The largest threshold below which the weight of q uniformly random
// qubits (each nonzero with probability 3/4) falls with probability about
// 3e-5 or less (mean minus four standard deviations); -1 when q < 8.  It
// only steers the kernel's choice of words, never the result.
int partial_limit(int q);

// Mixed packages (not in the paper).  When an additive code has fewer
// independent rows than qubits, two F4 matrices leave qubits unused;
// trading two-row packages for one-row ones spends them and lowers
// e_t(sizes).  Models two disjoint matrices with b_1, b_2 one-row packages
// (a_j = (rank - b_j) / 2 two-row ones, a_1 + b_1 + a_2 + b_2 <= n), both
// certifying a bound each round, and returns the caps {a_1, a_2} of the
// layouts with the least modelled work to reach d_est (at most `count`,
// best first, the all-two-row layout excluded).
std::vector<std::vector<int>> mixed_caps(int n, int rank, int d_est, int count);

// The least predicted work of matrices 1..h of a construction, over h.
double best_predicted(const std::vector<Gamma> &gs, int d_est, int max_gamma, bool scalar);

// Replaces the F4 matrices by capped ones (build_f4 with mixed_caps, two
// matrices) when that lowers their predicted work by at least 5%; `caps`
// receives the caps used (empty: unchanged).  Returns false if a capped
// matrix fails check_gamma (an internal error).  The automatic plan tries
// it from kMixMinWork predicted combinations: below that the extra
// constructions (0.1-0.4 ms on the host at n = 72-96) cost more than the
// saving.
constexpr double kMixMinWork = 1e10;
bool try_mixed_f4(const std::vector<BRow> &basis, int n, int rank, int d_est, int max_gamma,
                  std::vector<Gamma> &f4, std::vector<int> &caps);

// Elementary symmetric polynomials e_r of package sizes (1 or 3) as
// saturating 64-bit integers.  prefix[h][r] = e_r(c_0..c_{h-1}),
// suffix[h][r] = e_r(c_h..c_{P-1}); rmax columns + 1.
constexpr uint64_t kSat = uint64_t(1) << 62;
void esym_tables(const std::vector<int> &sizes, int rmax, std::vector<uint64_t> &prefix,
                 std::vector<uint64_t> &suffix);
uint64_t esym(const std::vector<int> &sizes, int t);

// Lower bound after matrix j has finished round t_j (t_j = 0: nothing yet):
// sum_j max(0, t_j + 1 - delta_j).  With halve (isometry matrices, whose
// bound counts Hamming weight, twice the symplectic weight) it is rounded
// up to half of that.
int lower_bound(const std::vector<int> &tdone, const std::vector<int> &delta, bool halve = false);

struct PlanChoice {
  int diag = 4;
  int h_used = 1;
  int d_est = 0;
  double predicted = 0;
  double predicted_f2 = 0, predicted_f4 = 0, predicted_iso = -1;
};

// Distance estimate for a code of rank k on n qubits with a known upper
// bound: the smaller of the upper bound and the weight where a random code
// of this size expects its first nonzero codeword.
int estimate_distance(int n, int k, int upper);

// Predicted combinations to certify distance d_est with the given matrices.
double predict_work(const std::vector<Gamma> &gs, int h, int d_est, bool halve = false);

// The automatic choice takes the isometry matrices only when the other
// constructions need at least kIsoMinWork combinations and the isometry
// less than kIsoMargin of that.
constexpr double kIsoMinWork = 1e8;
constexpr double kIsoMargin = 0.8;

// A lower bound on predict_work for any isometry matrices of a rank-`rank`
// code on n qubits (0 when none can be given): callers may skip building
// them when it exceeds a cheaper construction's prediction.
double iso_work_floor(int n, int rank, int d_est);

// Picks the construction (F2, F4 or isometry, or the one diag_req names)
// and the number of matrices with the least predicted work.
// f4_scalar: the F4 matrices will enumerate scalar classes (a third of
// their combinations).
PlanChoice choose_plan(const std::vector<Gamma> &f4, const Gamma &f2, const std::vector<Gamma> &iso, int n,
                       int rank, int diag_req, int max_gamma_req, bool f4_scalar = false);

}  // namespace qd

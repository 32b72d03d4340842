/*
 * qdo.c -- CPU oracle for the symplectic minimum distance (test
 * infrastructure only; see qdo.h).  Plain C, no blocking or fusion beyond
 * what the definitions need.  Bit-packed 64-bit words are used only inside
 * the enumeration loops; the diagonalizations work on one byte per bit so
 * each step can be compared with the matrices printed in the paper.
 */
#include "qdo.h"
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Small helpers on rows of 2n bytes.                                       */

static void row_add(uint8_t *dst, const uint8_t *src, int len) {
  for (int i = 0; i < len; ++i) dst[i] ^= src[i];
}

/* F4 symbol of qubit q: x + 2z encodes x + alpha*z (Sec. 2.3).  Adding rows
 * adds symbols, which is XOR of the two-bit codes. */
static int sym(const uint8_t *row, int n, int q) {
  return (row[q] & 1) | ((row[n + q] & 1) << 1);
}

/* Symplectic weight, Sec. 2: #{i : a_i != 0 or b_i != 0}. */
int qdo_symplectic_weight(const uint8_t *v, int n) {
  int w = 0;
  for (int i = 0; i < n; ++i)
    if (v[i] || v[n + i]) ++w;
  return w;
}

/* alpha*(a + alpha b) = b + alpha(a + b)  (alpha^2 = 1 + alpha). */
int qdo_expand(const uint8_t *G, int m, int n, int field, uint8_t *out) {
  if (m < 0 || n <= 0 || !G || !out) return QDO_ERR_INVALID;
  if (field == 2) {
    for (int i = 0; i < m * 2 * n; ++i) {
      if (G[i] > 1) return QDO_ERR_INVALID;
      out[i] = G[i];
    }
    return m;
  }
  if (field != 4) return QDO_ERR_INVALID;
  for (int i = 0; i < m; ++i) {
    uint8_t *g = out + (size_t)(2 * i) * 2 * n;
    uint8_t *ag = g + 2 * n;
    for (int q = 0; q < n; ++q) {
      int s = G[(size_t)i * n + q];
      if (s > 3) return QDO_ERR_INVALID;
      int a = s & 1, b = (s >> 1) & 1;
      g[q] = (uint8_t)a;
      g[n + q] = (uint8_t)b;
      ag[q] = (uint8_t)b;
      ag[n + q] = (uint8_t)(a ^ b);
    }
  }
  return 2 * m;
}

/* Gaussian elimination over F2; keeps the nonzero reduced rows.  Returns
 * the rank and, if basis != NULL, writes rank rows there. */
static int reduce_basis(const uint8_t *B, int m, int n, uint8_t *basis) {
  int len = 2 * n;
  uint8_t *M = (uint8_t *)malloc((size_t)(m > 0 ? m : 1) * len);
  if (!M) return QDO_ERR_NOMEM;
  memcpy(M, B, (size_t)m * len);
  int rank = 0;
  for (int c = 0; c < len && rank < m; ++c) {
    int p = -1;
    for (int r = rank; r < m; ++r)
      if (M[(size_t)r * len + c]) { p = r; break; }
    if (p < 0) continue;
    if (p != rank)
      for (int i = 0; i < len; ++i) {
        uint8_t t = M[(size_t)p * len + i];
        M[(size_t)p * len + i] = M[(size_t)rank * len + i];
        M[(size_t)rank * len + i] = t;
      }
    for (int r = 0; r < m; ++r)
      if (r != rank && M[(size_t)r * len + c])
        row_add(M + (size_t)r * len, M + (size_t)rank * len, len);
    ++rank;
  }
  if (basis) memcpy(basis, M, (size_t)rank * len);
  free(M);
  return rank;
}

int qdo_rank(const uint8_t *B, int m, int n) {
  if (m < 0 || n <= 0 || (!B && m)) return QDO_ERR_INVALID;
  return reduce_basis(B, m, n, NULL);
}

int qdo_in_rowspace(const uint8_t *B, int m, int n, const uint8_t *v) {
  int len = 2 * n;
  uint8_t *M = (uint8_t *)malloc((size_t)(m + 1) * len);
  if (!M) return QDO_ERR_NOMEM;
  memcpy(M, B, (size_t)m * len);
  memcpy(M + (size_t)m * len, v, len);
  int r0 = reduce_basis(M, m, n, NULL);
  int r1 = reduce_basis(M, m + 1, n, NULL);
  free(M);
  return r0 == r1 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Packed form for the enumeration loops: W words of x, then W words of z. */

static int words_of(int n) { return (n + 63) / 64; }

static void pack_row(const uint8_t *v, int n, uint64_t *out) {
  int W = words_of(n);
  memset(out, 0, sizeof(uint64_t) * 2 * W);
  for (int q = 0; q < n; ++q) {
    if (v[q]) out[q / 64] |= 1ull << (q % 64);
    if (v[n + q]) out[W + q / 64] |= 1ull << (q % 64);
  }
}

static void unpack_row(const uint64_t *c, int n, uint8_t *v) {
  int W = words_of(n);
  for (int q = 0; q < n; ++q) {
    v[q] = (uint8_t)((c[q / 64] >> (q % 64)) & 1);
    v[n + q] = (uint8_t)((c[W + q / 64] >> (q % 64)) & 1);
  }
}

/* Symplectic product <a, b>_s = a_x . b_z + a_z . b_x (mod 2). */
static int sym_product(const uint64_t *a, const uint64_t *b, int W) {
  int p = 0;
  for (int i = 0; i < W; ++i) p ^= __builtin_parityll((a[i] & b[W + i]) ^ (a[W + i] & b[i]));
  return p;
}

/* Modified BZ (Sec. 2.1): a codeword c of the span N of the rows updates U
 * only when it lies in C^{perp_s} \ C.  With N = C^{perp_s} the stabilizer
 * is C = N^{perp_s}, so c is admitted when its symplectic product with some
 * row of N is 1.  chk holds the m rows (2W words each); m = 0 admits every
 * codeword. */
static int admitted(const uint64_t *c, const uint64_t *chk, int m, int W) {
  if (m == 0) return 1;
  for (int r = 0; r < m; ++r)
    if (sym_product(c, chk + (size_t)r * 2 * W, W)) return 1;
  return 0;
}

/* The filter applies unless the span is self-orthogonal (the k = 0 case of
 * Sec. 2.1, where every codeword updates U): returns m or 0. */
static int filter_rows(const uint64_t *R, int m, int W) {
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j)
      if (sym_product(R + (size_t)i * 2 * W, R + (size_t)j * 2 * W, W)) return m;
  return 0;
}

static int packed_swt(const uint64_t *c, int W) {
  int w = 0;
  for (int i = 0; i < W; ++i) w += __builtin_popcountll(c[i] | c[W + i]);
  return w;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive minimum (the definition of the distance, Sec. 2).             */

static int brute_impl(const uint8_t *B, int m, int n, int nthreads, int filter, int *d,
                      uint8_t *witness) {
  if (!B || !d || m <= 0 || n <= 0) return m == 0 ? QDO_ERR_ZERO_CODE : QDO_ERR_INVALID;
  if (m > 40) return QDO_ERR_TOO_LARGE;
  int W = words_of(n);
  uint64_t *R = (uint64_t *)calloc((size_t)m * 2 * W, sizeof(uint64_t));
  if (!R) return QDO_ERR_NOMEM;
  for (int i = 0; i < m; ++i) pack_row(B + (size_t)i * 2 * n, n, R + (size_t)i * 2 * W);
  const int nchk = filter ? filter_rows(R, m, W) : 0;
  unsigned long long total = 1ull << m;
  int nchunks = m > 16 ? 256 : 1;
  unsigned long long chunk = total / (unsigned long long)nchunks;
  int best = n + 1;
  unsigned long long best_idx = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic)
  for (int ch = 0; ch < nchunks; ++ch) {
    unsigned long long lo = (unsigned long long)ch * chunk;
    unsigned long long hi = lo + chunk;
    if (lo == 0) lo = 1;
    /* codeword of Gray(lo) = XOR of the rows whose bit is set in lo^(lo>>1) */
    uint64_t c[8] = {0};
    unsigned long long g = lo ^ (lo >> 1);
    for (int r = 0; r < m; ++r)
      if ((g >> r) & 1)
        for (int i = 0; i < 2 * W; ++i) c[i] ^= R[(size_t)r * 2 * W + i];
    int lbest = n + 1;
    unsigned long long lidx = 0;
    for (unsigned long long i = lo; i < hi; ++i) {
      if (i != lo) {
        int r = __builtin_ctzll(i);
        for (int k = 0; k < 2 * W; ++k) c[k] ^= R[(size_t)r * 2 * W + k];
      }
      int w = packed_swt(c, W);
      if (w > 0 && w < lbest && admitted(c, R, nchk, W)) { lbest = w; lidx = i; }
    }
#pragma omp critical
    {
      if (lbest < best || (lbest == best && lidx < best_idx)) {
        best = lbest;
        best_idx = lidx;
      }
    }
  }
  int rc = QDO_OK;
  if (best > n) {
    rc = QDO_ERR_ZERO_CODE;
    *d = -1;
  } else {
    *d = best;
    if (witness) {
      uint64_t c[8] = {0};
      unsigned long long g = best_idx ^ (best_idx >> 1);
      for (int r = 0; r < m; ++r)
        if ((g >> r) & 1)
          for (int i = 0; i < 2 * W; ++i) c[i] ^= R[(size_t)r * 2 * W + i];
      unpack_row(c, n, witness);
    }
  }
  free(R);
  return rc;
}

int qdo_brute(const uint8_t *B, int m, int n, int nthreads, int *d,
              uint8_t *witness) {
  return brute_impl(B, m, n, nthreads, 0, d, witness);
}

int qdo_brute_stab(const uint8_t *B, int m, int n, int nthreads, int *d,
                   uint8_t *witness) {
  return brute_impl(B, m, n, nthreads, 1, d, witness);
}

/* Hamming weight of (a, b, a+b) for every nonzero combination (Sec. 2.4). */
int qdo_brute_iso_hamming(const uint8_t *B, int m, int n, int *dH) {
  if (!B || !dH || m <= 0 || n <= 0) return QDO_ERR_INVALID;
  if (m > 30) return QDO_ERR_TOO_LARGE;
  int len = 3 * n;
  uint8_t *iso = (uint8_t *)malloc((size_t)m * len);
  uint8_t *c = (uint8_t *)calloc(len, 1);
  if (!iso || !c) { free(iso); free(c); return QDO_ERR_NOMEM; }
  for (int i = 0; i < m; ++i)
    for (int q = 0; q < n; ++q) {
      uint8_t a = B[(size_t)i * 2 * n + q], b = B[(size_t)i * 2 * n + n + q];
      iso[(size_t)i * len + q] = a;
      iso[(size_t)i * len + n + q] = b;
      iso[(size_t)i * len + 2 * n + q] = a ^ b;
    }
  int best = len + 1;
  for (unsigned long long i = 1; i < (1ull << m); ++i) {
    row_add(c, iso + (size_t)__builtin_ctzll(i) * len, len);
    int w = 0;
    for (int k = 0; k < len; ++k) w += c[k];
    if (w > 0 && w < best) best = w;
  }
  free(iso);
  free(c);
  if (best > len) return QDO_ERR_ZERO_CODE;
  *dH = best;
  return QDO_OK;
}

/* ------------------------------------------------------------------------ */
/* Generator matrices made of packages.                                      */
/*                                                                          */
/* A package at pivot qubit q is either {r} or {r, s, r+s} (Sec. 2.3).      */
/* After the diagonalization every other row of the same matrix has the    */
/* symbol 0 at q (two-row package) or a symbol in {0, beta} with one beta   */
/* different from the symbol of r (one-row package), so a sum that uses one */
/* element from each of g packages pivoted on distinct qubits is nonzero on */
/* those g qubits.                                                          */

typedef struct {
  int dim;   /* 1 or 2 */
  int pivot; /* qubit, or -1 when the package is not pivoted in the set */
  int r, s;  /* row indices into the working matrix (s = -1 if dim 1) */
} pkg_t;

/* The column chosen next among `colok` columns not yet done: the first one
 * where the rows in `cand` show two different nonzero symbols, else the
 * first one where they show exactly one (Sec. 2.3: such columns are
 * prioritized).  With allow2 = 0 (mixed packages: the matrix has reached
 * its cap of two-row packages) it is the first column where some
 * candidate row is nonzero, for a one-row package.  Returns -1 if every
 * candidate row is zero there. */
static int pick_column(const uint8_t *R, int k, int n, const int *cand,
                       const int *colok, const int *done, int allow2, int *dim) {
  int first1 = -1;
  for (int q = 0; q < n; ++q) {
    if (!colok[q] || done[q]) continue;
    int mask = 0;
    for (int v = 0; v < k; ++v)
      if (cand[v]) mask |= 1 << sym(R + (size_t)v * 2 * n, n, q);
    mask &= 0xE; /* nonzero symbols 1, 2, 3 */
    int cnt = __builtin_popcount(mask);
    if (cnt >= 2 && allow2) { *dim = 2; return q; }
    if (cnt >= 1 && !allow2) { *dim = 1; return q; }
    if (cnt == 1 && first1 < 0) first1 = q;
  }
  *dim = 1;
  return first1;
}

/* Diagonalization over F4 restricted to rows in `cand` (pivots) and rows in
 * `clearset` (rows whose pivot columns get cleared), columns in `colok`.
 * Appends packages to pk and clears cand[] for the rows it uses.  max2 >= 0
 * caps the two-row packages of the pass (mixed packages); -1: no cap. */
static int diag_f4_pass(uint8_t *R, int k, int n, int *cand, const int *clearset,
                        const int *colok, int outside, int max2, pkg_t *pk, int np) {
  int len = 2 * n;
  int n2 = 0;
  int *done = (int *)calloc(n, sizeof(int));
  int *pivrow = (int *)calloc(k, sizeof(int)); /* used as a pivot row in this pass */
  for (;;) {
    int dim;
    int q = pick_column(R, k, n, cand, colok, done, max2 < 0 || n2 < max2, &dim);
    if (q < 0) break;
    done[q] = 1;
    int r = -1, s = -1;
    for (int v = 0; v < k; ++v)
      if (cand[v] && sym(R + (size_t)v * len, n, q)) { r = v; break; }
    int sr = sym(R + (size_t)r * len, n, q);
    if (dim == 2) {
      for (int v = 0; v < k; ++v) {
        int sv = cand[v] ? sym(R + (size_t)v * len, n, q) : 0;
        if (sv && sv != sr) { s = v; break; }
      }
      int ss = sym(R + (size_t)s * len, n, q);
      /* Clear the column in every other row: add r, s or r+s. */
      for (int v = 0; v < k; ++v) {
        if (v == r || v == s || !clearset[v]) continue;
        int sv = sym(R + (size_t)v * len, n, q);
        if (sv == 0) continue;
        if (sv == sr) {
          row_add(R + (size_t)v * len, R + (size_t)r * len, len);
        } else if (sv == ss) {
          row_add(R + (size_t)v * len, R + (size_t)s * len, len);
        } else {
          row_add(R + (size_t)v * len, R + (size_t)r * len, len);
          row_add(R + (size_t)v * len, R + (size_t)s * len, len);
        }
      }
      cand[r] = cand[s] = 0;
      pivrow[r] = pivrow[s] = 1;
      ++n2;
    } else {
      /* One-row package: every other row becomes 0 or one fixed beta != sr
       * at q (Sec. 2.3, "clear"): adding r takes sr to 0 and sr ^ beta to
       * beta.  Remaining rows show only sr at a one-symbol column; past a
       * two-row cap they may show all three symbols. */
      int beta = (sr == 1) ? 2 : 1;
      for (int v = 0; v < k; ++v) {
        if (v == r || !clearset[v] || !(cand[v] || pivrow[v])) continue;
        int sv = sym(R + (size_t)v * len, n, q);
        if (sv == sr || sv == (sr ^ beta))
          row_add(R + (size_t)v * len, R + (size_t)r * len, len);
      }
      cand[r] = 0;
      pivrow[r] = 1;
    }
    pk[np].dim = dim;
    pk[np].pivot = outside ? -1 : q;
    pk[np].r = r;
    pk[np].s = (dim == 2) ? s : -1;
    ++np;
  }
  free(done);
  free(pivrow);
  return np;
}

/* One generator matrix over the allowed qubits, at most max2 two-row
 * packages among those pivoted there (-1: no cap); leftover rows (zero on
 * all allowed qubits) are grouped by the same rule over all qubits and
 * counted as packages outside the set. */
static int build_f4(uint8_t *R, int k, int n, const int *allowed, int max2, pkg_t *pk) {
  int *cand = (int *)malloc(sizeof(int) * k);
  int *all = (int *)malloc(sizeof(int) * k);
  int *allcols = (int *)malloc(sizeof(int) * n);
  for (int v = 0; v < k; ++v) cand[v] = all[v] = 1;
  for (int q = 0; q < n; ++q) allcols[q] = 1;
  int np = diag_f4_pass(R, k, n, cand, all, allowed, 0, max2, pk, 0);
  int *left = (int *)malloc(sizeof(int) * k);
  for (int v = 0; v < k; ++v) left[v] = cand[v];
  np = diag_f4_pass(R, k, n, cand, left, allcols, 1, -1, pk, np);
  free(cand); free(all); free(allcols); free(left);
  return np;
}

/* Diagonalization over F2 (Sec. 2.2): column operations limited to qubit
 * permutations and per-qubit x<->z swaps give [I M1; 0 M2]; each pivot of
 * M2 (reduced echelon form) is merged with the identity row of the same
 * qubit into a two-row package.  The whole qubit column is cleared in every
 * other row, which the worked example of Sec. 2.2 needs. */
static int build_f2(uint8_t *R, int k, int n, pkg_t *pk) {
  int len = 2 * n;
  int *rem = (int *)malloc(sizeof(int) * k);
  int *prow = (int *)malloc(sizeof(int) * n);
  int *kind = (int *)malloc(sizeof(int) * n); /* 0 none, 1 x pivot, 2 z pivot */
  int *second = (int *)malloc(sizeof(int) * n);
  for (int v = 0; v < k; ++v) rem[v] = 1;
  for (int q = 0; q < n; ++q) {
    prow[q] = -1; kind[q] = 0; second[q] = -1;
    for (int half = 0; half < 2 && kind[q] == 0; ++half) {
      int col = half * n + q;
      int r = -1;
      for (int v = 0; v < k; ++v)
        if (rem[v] && R[(size_t)v * len + col]) { r = v; break; }
      if (r < 0) continue;
      for (int v = 0; v < k; ++v)
        if (v != r && R[(size_t)v * len + col])
          row_add(R + (size_t)v * len, R + (size_t)r * len, len);
      rem[r] = 0;
      prow[q] = r;
      kind[q] = half + 1;
    }
  }
  for (int q = 0; q < n; ++q) {
    if (kind[q] != 1) continue;
    int col = n + q;
    int r = -1;
    for (int v = 0; v < k; ++v)
      if (rem[v] && R[(size_t)v * len + col]) { r = v; break; }
    if (r < 0) continue;
    for (int v = 0; v < k; ++v)
      if (v != r && R[(size_t)v * len + col])
        row_add(R + (size_t)v * len, R + (size_t)r * len, len);
    rem[r] = 0;
    second[q] = r;
  }
  int np = 0, left = 0;
  for (int v = 0; v < k; ++v) left += rem[v];
  for (int q = 0; q < n; ++q) {
    if (!kind[q]) continue;
    pk[np].pivot = q;
    pk[np].r = prow[q];
    pk[np].s = second[q];
    pk[np].dim = second[q] >= 0 ? 2 : 1;
    ++np;
  }
  free(rem); free(prow); free(kind); free(second);
  return left ? -1 : np;
}

/* Self-check of the package invariants (the oracle refuses its own output
 * if they fail). */
static int check_packages(const uint8_t *R, int k, int n, const pkg_t *pk, int np) {
  int len = 2 * n;
  for (int i = 0; i < np; ++i) {
    if (pk[i].pivot < 0) continue;
    int q = pk[i].pivot;
    int sr = sym(R + (size_t)pk[i].r * len, n, q);
    if (!sr) return 0;
    if (pk[i].dim == 2) {
      int ss = sym(R + (size_t)pk[i].s * len, n, q);
      if (!ss || ss == sr) return 0;
    }
    int others = 0;
    for (int v = 0; v < k; ++v) {
      if (v == pk[i].r || v == pk[i].s) continue;
      int sv = sym(R + (size_t)v * len, n, q);
      if (sv) others |= 1 << sv;
    }
    if (pk[i].dim == 2 && others) return 0;
    if (pk[i].dim == 1 && (__builtin_popcount(others) > 1 || (others >> sr) & 1)) return 0;
  }
  return 1;
}

static int gamma_impl(const uint8_t *B, int m, int n, int diag, int max_gamma,
                      const int *max2, int cap, int *h_out, int *P, int *delta,
                      int *dims, int *pivot, uint8_t *rows) {
  if (!B || m <= 0 || n <= 0 || max_gamma <= 0 || cap < 2 * n || !h_out || !P ||
      !delta || !dims || !pivot)
    return m == 0 ? QDO_ERR_ZERO_CODE : QDO_ERR_INVALID;
  if (diag != QDO_DIAG_F2 && diag != QDO_DIAG_F4) return QDO_ERR_INVALID;
  int len = 2 * n;
  uint8_t *basis = (uint8_t *)malloc((size_t)m * len);
  uint8_t *R = (uint8_t *)malloc((size_t)m * len);
  pkg_t *pk = (pkg_t *)malloc(sizeof(pkg_t) * (2 * n + 1));
  int *used = (int *)calloc(n, sizeof(int));
  int *allowed = (int *)malloc(sizeof(int) * n);
  /* Rows that are already independent are used as given (the paper assumes
   * this, Sec. 2.2); otherwise a reduced basis of their span is taken. */
  int k = reduce_basis(B, m, n, basis);
  if (k == m) memcpy(basis, B, (size_t)m * len);
  int rc = k;
  int h = 0;
  if (k == 0) { rc = QDO_ERR_ZERO_CODE; goto done; }
  for (int j = 0; j < max_gamma; ++j) {
    memcpy(R, basis, (size_t)k * len);
    int np;
    if (diag == QDO_DIAG_F2) {
      if (j > 0) break; /* one matrix covers every pivotable qubit */
      np = build_f2(R, k, n, pk);
      if (np < 0) { rc = QDO_ERR_INVALID; goto done; }
    } else {
      int any = 0;
      for (int q = 0; q < n; ++q) { allowed[q] = !used[q]; any |= allowed[q]; }
      if (!any) break;
      np = build_f4(R, k, n, allowed, max2 ? max2[j] : -1, pk);
    }
    if (!check_packages(R, k, n, pk, np)) { rc = -5; goto done; }
    int inside = 0, dsum = 0;
    for (int i = 0; i < np; ++i) {
      inside += pk[i].pivot >= 0;
      dsum += pk[i].dim;
    }
    if (dsum != k) { rc = -6; goto done; }
    if (inside == 0) break; /* contributes nothing to the lower bound */
    P[h] = np;
    delta[h] = np - inside;
    for (int i = 0; i < np; ++i) {
      dims[h * cap + i] = pk[i].dim;
      pivot[h * cap + i] = pk[i].pivot;
      if (pk[i].pivot >= 0) used[pk[i].pivot] = 1;
      if (rows) {
        uint8_t *dst = rows + ((size_t)(h * cap + i) * 2) * len;
        memcpy(dst, R + (size_t)pk[i].r * len, len);
        if (pk[i].dim == 2)
          memcpy(dst + len, R + (size_t)pk[i].s * len, len);
        else
          memset(dst + len, 0, len);
      }
    }
    ++h;
  }
  *h_out = h;
done:
  free(basis); free(R); free(pk); free(used); free(allowed);
  return rc;
}

int qdo_gamma(const uint8_t *B, int m, int n, int diag, int max_gamma,
              int cap, int *h_out, int *P, int *delta, int *dims, int *pivot,
              uint8_t *rows) {
  return gamma_impl(B, m, n, diag, max_gamma, NULL, cap, h_out, P, delta, dims, pivot, rows);
}

int qdo_gamma_mixed(const uint8_t *B, int m, int n, int max_gamma, const int *max2,
                    int cap, int *h_out, int *P, int *delta, int *dims, int *pivot,
                    uint8_t *rows) {
  if (!max2) return QDO_ERR_INVALID;
  return gamma_impl(B, m, n, QDO_DIAG_F4, max_gamma, max2, cap, h_out, P, delta, dims, pivot, rows);
}

/* ------------------------------------------------------------------------ */
/* One round: t distinct packages, one nonzero element from each.           */

typedef struct {
  int P, t, W, n;
  const int *ne;        /* elements per package: 1 or 3 */
  const uint64_t *el;   /* package i element e at (i*3+e)*2W */
  const uint64_t *chk;  /* rows for the Modified-BZ admission test (nchk 0: none) */
  int nchk;
  int best;
  unsigned long long count;
  uint64_t bestc[8];
} round_ctx;

static void round_rec(round_ctx *c, int start, int depth, const uint64_t *cur) {
  int W2 = 2 * c->W;
  if (depth == c->t) {
    int w = packed_swt(cur, c->W);
    ++c->count;
    if (w < c->best && admitted(cur, c->chk, c->nchk, c->W)) {
      c->best = w;
      memcpy(c->bestc, cur, sizeof(uint64_t) * W2);
    }
    return;
  }
  uint64_t nxt[8];
  for (int i = start; i <= c->P - (c->t - depth); ++i)
    for (int e = 0; e < c->ne[i]; ++e) {
      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;
      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];
      round_rec(c, i + 1, depth + 1, nxt);
    }
}

/* Elements r, s, r+s of each package (Sec. 2.3: a three-row package). */
static uint64_t *package_elements(const uint8_t *rows, const int *dims, int P, int n,
                                  int *ne) {
  int W = words_of(n);
  uint64_t *el = (uint64_t *)calloc((size_t)P * 3 * 2 * W + 1, sizeof(uint64_t));
  if (!el) return NULL;
  for (int i = 0; i < P; ++i) {
    uint64_t *e0 = el + (size_t)(i * 3) * 2 * W;
    pack_row(rows + (size_t)(2 * i) * 2 * n, n, e0);
    ne[i] = 1;
    if (dims[i] == 2) {
      uint64_t *e1 = e0 + 2 * W, *e2 = e0 + 4 * W;
      pack_row(rows + (size_t)(2 * i + 1) * 2 * n, n, e1);
      for (int k = 0; k < 2 * W; ++k) e2[k] = e0[k] ^ e1[k];
      ne[i] = 3;
    }
  }
  return el;
}

static int round_impl(const uint8_t *rows, const int *dims, int P, int n, int t,
                      int nthreads, const uint64_t *chk, int nchk, int *wmin,
                      uint8_t *witness, unsigned long long *count) {
  if (!rows || !dims || P < 0 || n <= 0 || n > 256 || t < 1 || !wmin || !count)
    return QDO_ERR_INVALID;
  int W = words_of(n);
  int *ne = (int *)malloc(sizeof(int) * (P + 1));
  uint64_t *el = package_elements(rows, dims, P, n, ne);
  if (!ne || !el) { free(ne); free(el); return QDO_ERR_NOMEM; }
  int best = n + 1;
  int best_i = P;
  unsigned long long total = 0;
  uint64_t bestc[8] = {0};
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  /* The first (lowest) package of the subset is the unit of parallel work. */
#pragma omp parallel for schedule(dynamic)
  for (int i0 = 0; i0 < P; ++i0) {
    if (i0 > P - t) continue;
    round_ctx c;
    c.P = P; c.t = t; c.W = W; c.n = n; c.ne = ne; c.el = el;
    c.chk = chk; c.nchk = nchk;
    c.best = n + 1; c.count = 0;
    memset(c.bestc, 0, sizeof(c.bestc));
    uint64_t cur[8];
    for (int e = 0; e < ne[i0]; ++e) {
      const uint64_t *x = el + (size_t)(i0 * 3 + e) * 2 * W;
      for (int k = 0; k < 2 * W; ++k) cur[k] = x[k];
      round_rec(&c, i0 + 1, 1, cur);
    }
#pragma omp critical
    {
      total += c.count;
      if (c.best < best || (c.best == best && i0 < best_i)) {
        best = c.best;
        best_i = i0;
        memcpy(bestc, c.bestc, sizeof(bestc));
      }
    }
  }
  *wmin = best;
  *count = total;
  if (witness) unpack_row(bestc, n, witness);
  free(ne);
  free(el);
  return QDO_OK;
}

int qdo_round(const uint8_t *rows, const int *dims, int P, int n, int t,
              int nthreads, int *wmin, uint8_t *witness,
              unsigned long long *count) {
  return round_impl(rows, dims, P, n, t, nthreads, NULL, 0, wmin, witness, count);
}

/* Weight distribution of one round: hist[w] = number of combinations of t
 * distinct packages, one nonzero element of each (Sec. 2.3), whose sum has
 * symplectic weight w (Sec. 2).  Plain recursion over the same choices as
 * qdo_round, one tally per combination. */
typedef struct {
  int P, t, W;
  const int *ne;
  const uint64_t *el;
  unsigned long long *hist;  /* n+1 counters of this worker */
} hist_ctx;

static void hist_rec(hist_ctx *c, int start, int depth, const uint64_t *cur) {
  int W2 = 2 * c->W;
  if (depth == c->t) {
    ++c->hist[packed_swt(cur, c->W)];
    return;
  }
  uint64_t nxt[8];
  for (int i = start; i <= c->P - (c->t - depth); ++i)
    for (int e = 0; e < c->ne[i]; ++e) {
      const uint64_t *x = c->el + (size_t)(i * 3 + e) * W2;
      for (int k = 0; k < W2; ++k) nxt[k] = cur[k] ^ x[k];
      hist_rec(c, i + 1, depth + 1, nxt);
    }
}

int qdo_round_hist(const uint8_t *rows, const int *dims, int P, int n, int t,
                   int nthreads, unsigned long long *hist) {
  if (!rows || !dims || P < 0 || n <= 0 || n > 256 || t < 1 || !hist)
    return QDO_ERR_INVALID;
  int W = words_of(n);
  int *ne = (int *)malloc(sizeof(int) * (P + 1));
  uint64_t *el = package_elements(rows, dims, P, n, ne);
  if (!ne || !el) { free(ne); free(el); return QDO_ERR_NOMEM; }
  for (int w = 0; w <= n; ++w) hist[w] = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic)
  for (int i0 = 0; i0 < P; ++i0) {
    if (i0 > P - t) continue;
    unsigned long long *mine = (unsigned long long *)calloc((size_t)n + 1, sizeof(unsigned long long));
    hist_ctx c;
    c.P = P; c.t = t; c.W = W; c.ne = ne; c.el = el; c.hist = mine;
    uint64_t cur[8];
    for (int e = 0; e < ne[i0]; ++e) {
      const uint64_t *x = el + (size_t)(i0 * 3 + e) * 2 * W;
      for (int k = 0; k < 2 * W; ++k) cur[k] = x[k];
      hist_rec(&c, i0 + 1, 1, cur);
    }
#pragma omp critical
    {
      for (int w = 0; w <= n; ++w) hist[w] += mine[w];
    }
    free(mine);
  }
  free(ne);
  free(el);
  return QDO_OK;
}

/* ------------------------------------------------------------------------ */
/* Brouwer-Zimmermann (Sec. 2.1).                                           */
/* U: smallest weight seen (starts at the sentinel n+1).                   */
/* L: after Gamma_j has been enumerated through t_j packages, a codeword    */
/* not yet seen uses at least t_j+1 packages of every Gamma_j, at least     */
/* t_j+1-delta_j of them pivoted on distinct qubits of that matrix's own    */
/* set; the sets are disjoint, so L = sum_j max(0, t_j + 1 - delta_j).      */
/* With two matrices this is the bound of Sec. 2.3 (delta_2 = n_p - n_pp). */

static int bz_gamma_impl(int h, const int *P, const int *off, const int *delta,
                         const uint8_t *rows, const int *dims, int n, int nthreads,
                         const uint64_t *chk, int nchk, int *d, uint8_t *witness,
                         long long *log, int log_cap, int *nlog) {
  if (h <= 0 || !P || !off || !delta || !rows || !dims || n <= 0 || !d)
    return QDO_ERR_INVALID;
  int len = 2 * n;
  int U = n + 1;
  uint8_t *wit = (uint8_t *)calloc(len, 1);
  uint8_t *cand = (uint8_t *)calloc(len, 1);
  int *tdone = (int *)calloc(h, sizeof(int));
  int nl = 0;
  int finished = 0;
  for (int t = 1; !finished; ++t) {
    int any = 0;
    for (int j = 0; j < h && !finished; ++j) {
      if (t > P[j]) continue;
      any = 1;
      int w;
      unsigned long long cnt;
      int rc = round_impl(rows + (size_t)off[j] * 2 * len, dims + off[j], P[j], n, t,
                          nthreads, chk, nchk, &w, cand, &cnt);
      if (rc) { free(wit); free(cand); free(tdone); return rc; }
      if (w < U) {
        U = w;
        memcpy(wit, cand, len);
      }
      tdone[j] = t;
      int L = 0;
      for (int i = 0; i < h; ++i) {
        int c = tdone[i] + 1 - delta[i];
        L += c > 0 ? c : 0;
      }
      if (log && nl < log_cap) {
        long long *r = log + 5 * nl;
        r[0] = t; r[1] = j; r[2] = L; r[3] = U; r[4] = (long long)cnt;
      }
      ++nl;
      if (L >= U || t == P[j]) finished = 1; /* bound met, or every codeword seen */
    }
    if (!any) finished = 1;
  }
  if (nlog) *nlog = nl;
  *d = U;
  if (witness) memcpy(witness, wit, len);
  free(wit); free(cand); free(tdone);
  return U <= n ? QDO_OK : QDO_ERR_ZERO_CODE;
}

int qdo_bz_gamma(int h, const int *P, const int *off, const int *delta,
                 const uint8_t *rows, const int *dims, int n, int nthreads,
                 int *d, uint8_t *witness, long long *log, int log_cap,
                 int *nlog) {
  return bz_gamma_impl(h, P, off, delta, rows, dims, n, nthreads, NULL, 0, d, witness,
                       log, log_cap, nlog);
}

static int bz_impl(const uint8_t *B, int m, int n, int diag, int max_gamma, const int *max2,
                   int nthreads, int filter, int *d, uint8_t *witness, long long *log,
                   int log_cap, int *nlog) {
  if (!B || m <= 0 || n <= 0 || !d) return m == 0 ? QDO_ERR_ZERO_CODE : QDO_ERR_INVALID;
  int cap = 2 * n;
  int G = max_gamma > 0 ? max_gamma : 1;
  int *P = (int *)calloc(G, sizeof(int));
  int *off = (int *)calloc(G, sizeof(int));
  int *delta = (int *)calloc(G, sizeof(int));
  int *dims = (int *)calloc((size_t)G * cap, sizeof(int));
  int *piv = (int *)calloc((size_t)G * cap, sizeof(int));
  uint8_t *rows = (uint8_t *)calloc((size_t)G * cap * 2 * 2 * n, 1);
  int h = 0;
  int W = words_of(n);
  uint64_t *chk = (uint64_t *)calloc((size_t)m * 2 * W + 1, sizeof(uint64_t));
  int nchk = 0;
  if (chk && filter) {
    for (int i = 0; i < m; ++i) pack_row(B + (size_t)i * 2 * n, n, chk + (size_t)i * 2 * W);
    nchk = filter_rows(chk, m, W);
  }
  int rc = chk ? gamma_impl(B, m, n, diag, G, max2, cap, &h, P, delta, dims, piv, rows) : QDO_ERR_NOMEM;
  if (rc >= 0) {
    for (int j = 0; j < h; ++j) off[j] = j * cap;
    rc = bz_gamma_impl(h, P, off, delta, rows, dims, n, nthreads, chk, nchk, d, witness,
                       log, log_cap, nlog);
  } else {
    *d = -1;
  }
  free(P); free(off); free(delta); free(dims); free(piv); free(rows); free(chk);
  return rc;
}

int qdo_bz(const uint8_t *B, int m, int n, int diag, int max_gamma,
           int nthreads, int *d, uint8_t *witness, long long *log,
           int log_cap, int *nlog) {
  return bz_impl(B, m, n, diag, max_gamma, NULL, nthreads, 0, d, witness, log, log_cap, nlog);
}

int qdo_bz_mixed(const uint8_t *B, int m, int n, int max_gamma, const int *max2,
                 int nthreads, int *d, uint8_t *witness, long long *log,
                 int log_cap, int *nlog) {
  if (!max2) return QDO_ERR_INVALID;
  return bz_impl(B, m, n, QDO_DIAG_F4, max_gamma, max2, nthreads, 0, d, witness, log, log_cap, nlog);
}

int qdo_bz_stab(const uint8_t *B, int m, int n, int diag, int max_gamma,
                int nthreads, int *d, uint8_t *witness, long long *log,
                int log_cap, int *nlog) {
  return bz_impl(B, m, n, diag, max_gamma, NULL, nthreads, 1, d, witness, log, log_cap, nlog);
}

/* ------------------------------------------------------------------------ */
/* Saved_isometry (Sec. 2.4): Brouwer-Zimmermann for the Hamming weight of  */
/* the isometric image (a, b, a+b), a binary linear code of length 3n.      */

static void iso_image(const uint8_t *row, int n, uint8_t *out) {
  for (int q = 0; q < n; ++q) {
    out[q] = row[q];
    out[n + q] = row[n + q];
    out[2 * n + q] = row[q] ^ row[n + q];
  }
}

int qdo_gamma_iso(const uint8_t *B, int m, int n, int max_gamma, int *h_out,
                  int *k, int *pivcol, uint8_t *rows) {
  if (!B || m <= 0 || n <= 0 || max_gamma <= 0 || !h_out || !k || !pivcol)
    return QDO_ERR_INVALID;
  int len = 3 * n;
  uint8_t *basis = (uint8_t *)malloc((size_t)m * 2 * n);
  uint8_t *R = (uint8_t *)malloc((size_t)m * len);
  int *used = (int *)calloc(len, sizeof(int));   /* column in an earlier set */
  int *piv = (int *)malloc(sizeof(int) * m);     /* pivot column of each row */
  if (!basis || !R || !used || !piv) {
    free(basis); free(R); free(used); free(piv);
    return QDO_ERR_NOMEM;
  }
  int r = reduce_basis(B, m, n, basis);
  if (r == 0) { free(basis); free(R); free(used); free(piv); return QDO_ERR_ZERO_CODE; }
  int h = 0;
  while (h < max_gamma) {
    /* Gamma_{h+1}: the basis rows, reduced row echelon form on the columns
     * outside the earlier information sets, scanned left to right. */
    for (int i = 0; i < r; ++i) iso_image(basis + (size_t)i * 2 * n, n, R + (size_t)i * len);
    for (int i = 0; i < r; ++i) piv[i] = -1;
    int kk = 0;
    for (int c = 0; c < len && kk < r; ++c) {
      if (used[c]) continue;
      int p = -1;
      for (int i = 0; i < r; ++i)
        if (piv[i] < 0 && R[(size_t)i * len + c]) { p = i; break; }
      if (p < 0) continue;
      piv[p] = c;
      ++kk;
      for (int i = 0; i < r; ++i)
        if (i != p && R[(size_t)i * len + c]) row_add(R + (size_t)i * len, R + (size_t)p * len, len);
    }
    if (kk == 0) break;  /* no column left that carries information */
    for (int i = 0; i < r; ++i) {
      pivcol[h * r + i] = piv[i];
      if (piv[i] >= 0) used[piv[i]] = 1;
      if (rows) memcpy(rows + (size_t)(h * r + i) * len, R + (size_t)i * len, len);
    }
    k[h] = kk;
    ++h;
  }
  *h_out = h;
  free(basis); free(R); free(used); free(piv);
  return r;
}

typedef struct {
  int m, t, W;
  const uint64_t *el;  /* row i at i*W */
  int best;
  unsigned long long count;
  uint64_t bestc[8];
} hround_ctx;

static int packed_hw(const uint64_t *c, int W) {
  int w = 0;
  for (int i = 0; i < W; ++i) w += __builtin_popcountll(c[i]);
  return w;
}

static void hround_rec(hround_ctx *c, int start, int depth, const uint64_t *cur) {
  if (depth == c->t) {
    int w = packed_hw(cur, c->W);
    ++c->count;
    if (w < c->best) {
      c->best = w;
      memcpy(c->bestc, cur, sizeof(uint64_t) * c->W);
    }
    return;
  }
  uint64_t nxt[8];
  for (int i = start; i <= c->m - (c->t - depth); ++i) {
    const uint64_t *x = c->el + (size_t)i * c->W;
    for (int k = 0; k < c->W; ++k) nxt[k] = cur[k] ^ x[k];
    hround_rec(c, i + 1, depth + 1, nxt);
  }
}

/* Minimum Hamming weight over all sums of t distinct rows of one matrix
 * (m rows of len bytes). */
static int hamming_round(const uint8_t *rows, int m, int len, int t, int nthreads,
                         int *wmin, uint8_t *witness, unsigned long long *count) {
  int W = (len + 63) / 64;
  uint64_t *el = (uint64_t *)calloc((size_t)m * W + 1, sizeof(uint64_t));
  if (!el) return QDO_ERR_NOMEM;
  for (int i = 0; i < m; ++i)
    for (int b = 0; b < len; ++b)
      if (rows[(size_t)i * len + b]) el[(size_t)i * W + b / 64] |= 1ull << (b % 64);
  int best = len + 1, best_i = m;
  unsigned long long total = 0;
  uint64_t bestc[8] = {0};
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic)
  for (int i0 = 0; i0 < m; ++i0) {
    if (i0 > m - t) continue;
    hround_ctx c;
    c.m = m; c.t = t; c.W = W; c.el = el; c.best = len + 1; c.count = 0;
    memset(c.bestc, 0, sizeof(c.bestc));
    hround_rec(&c, i0 + 1, 1, el + (size_t)i0 * W);
#pragma omp critical
    {
      total += c.count;
      if (c.best < best || (c.best == best && i0 < best_i)) {
        best = c.best;
        best_i = i0;
        memcpy(bestc, c.bestc, sizeof(bestc));
      }
    }
  }
  *wmin = best;
  *count = total;
  if (witness)
    for (int b = 0; b < len; ++b) witness[b] = (uint8_t)((bestc[b / 64] >> (b % 64)) & 1);
  free(el);
  return QDO_OK;
}

int qdo_bz_iso(const uint8_t *B, int m, int n, int max_gamma, int nthreads,
               int *d, uint8_t *witness, long long *log, int log_cap, int *nlog) {
  if (!B || m <= 0 || n <= 0 || !d) return m == 0 ? QDO_ERR_ZERO_CODE : QDO_ERR_INVALID;
  if (3 * n > 512) return QDO_ERR_TOO_LARGE;
  int len = 3 * n;
  int G = max_gamma > 0 ? max_gamma : 1;
  int *k = (int *)calloc(G, sizeof(int));
  int *pivcol = (int *)calloc((size_t)G * m, sizeof(int));
  uint8_t *rows = (uint8_t *)calloc((size_t)G * m * len, 1);
  uint8_t *wit = (uint8_t *)calloc(len, 1);
  uint8_t *cand = (uint8_t *)calloc(len, 1);
  int *tdone = (int *)calloc(G, sizeof(int));
  if (!k || !pivcol || !rows || !wit || !cand || !tdone) {
    free(k); free(pivcol); free(rows); free(wit); free(cand); free(tdone);
    return QDO_ERR_NOMEM;
  }
  int h = 0;
  int r = qdo_gamma_iso(B, m, n, G, &h, k, pivcol, rows);
  if (r < 0) {
    *d = -1;
    free(k); free(pivcol); free(rows); free(wit); free(cand); free(tdone);
    return r;
  }
  /* Sec. 2.1 over the Hamming weight: U = least weight seen; a codeword not
   * seen after Gamma_j's round t_j sums at least t_j + 1 of its rows, at
   * least t_j + 1 - (r - k_j) of them pivot rows, each with its own 1 on
   * Gamma_j's information set; the sets are disjoint. */
  int U = len + 1, nl = 0, finished = 0;
  for (int t = 1; !finished; ++t) {
    if (t > r) break;
    for (int j = 0; j < h && !finished; ++j) {
      int w;
      unsigned long long cnt;
      int rc = hamming_round(rows + (size_t)j * r * len, r, len, t, nthreads, &w, cand, &cnt);
      if (rc) { free(k); free(pivcol); free(rows); free(wit); free(cand); free(tdone); return rc; }
      if (w < U) {
        U = w;
        memcpy(wit, cand, len);
      }
      tdone[j] = t;
      int L = 0;
      for (int i = 0; i < h; ++i) {
        int c = tdone[i] + 1 - (r - k[i]);
        L += c > 0 ? c : 0;
      }
      if (log && nl < log_cap) {
        long long *e = log + 5 * nl;
        e[0] = t; e[1] = j; e[2] = L; e[3] = U; e[4] = (long long)cnt;
      }
      ++nl;
      if (L >= U || t == r) finished = 1; /* bound met, or every codeword seen */
    }
  }
  if (nlog) *nlog = nl;
  /* d = d_H / 2 (Sec. 2.4); the witness is the (a|b) part of the image. */
  *d = U <= len ? U / 2 : -1;
  if (witness) memcpy(witness, wit, 2 * n);
  free(k); free(pivcol); free(rows); free(wit); free(cand); free(tdone);
  return U <= len ? QDO_OK : QDO_ERR_ZERO_CODE;
}

/*
 * qdo.h -- CPU oracle for the symplectic minimum distance of a binary
 * (additive) code.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the CPU-baseline leg of the benchmark call it; the library never does.
 *
 * Everything here is written to be checked by eye against the paper
 * (Hernando, Quintana-Orti, Grassl, "Fast Algorithms and Implementations for
 * Computing the Minimum Distance of Quantum Codes"):
 *   - symplectic weight and the distance of a set: Sec. 2, first two displays;
 *   - Brouwer-Zimmermann bounds U and L: Sec. 2.1;
 *   - Diagonalization_over_F2 with the appended rows: Sec. 2.2 (Alg. 1);
 *   - Diagonalization_over_F4, packages, principal columns and the lower
 *     bound contributed by a second generator matrix: Sec. 2.3 (Alg. 2);
 *   - the isometry (a,b) -> (a,b,a+b) and Saved_isometry, Brouwer-
 *     Zimmermann for the Hamming weight of the image: Sec. 2.4 (Alg. 3).
 *
 * Layout of a binary row: 2n bytes in {0,1}, x_1..x_n then z_1..z_n
 * (the paper's (a|b)).  F4 input: n bytes in {0,1,2,3}, code a+2b for the
 * symbol a + alpha*b (Sec. 2.3: a row (a,b) corresponds to a + alpha b).
 *
 * Parity status: every function below is pinned by the non-GPU tests
 * (paper examples, brute force, closed forms, invariances); none is
 * "parity unpinned".
 */
#ifndef QDO_H
#define QDO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define QDO_OK 0
#define QDO_ERR_INVALID (-1)
#define QDO_ERR_ZERO_CODE (-2)
#define QDO_ERR_TOO_LARGE (-3)
#define QDO_ERR_NOMEM (-4)

#define QDO_DIAG_F2 2
#define QDO_DIAG_F4 4

/* Symplectic weight #{i : x_i != 0 or z_i != 0} of one row (Sec. 2). */
int qdo_symplectic_weight(const uint8_t *v, int n);

/* Binary rows of the code.  field 2: copy of the m rows.  field 4: each F4
 * row g gives the two binary rows g and alpha*g, so the F2-span of the output
 * is the F4-span of the input.  out holds (field==4 ? 2m : m) rows. */
int qdo_expand(const uint8_t *G, int m, int n, int field, uint8_t *out);

/* Rank over F2 of m binary rows of length 2n. */
int qdo_rank(const uint8_t *B, int m, int n);

/* 1 if v (2n bytes) lies in the F2 row space of B, else 0. */
int qdo_in_rowspace(const uint8_t *B, int m, int n, const uint8_t *v);

/* Exhaustive minimum: every nonzero F2 combination of the m rows, visited in
 * binary reflected Gray order.  Rows may be dependent (zero sums are
 * skipped).  m <= 40.  witness: 2n bytes or NULL. */
int qdo_brute(const uint8_t *B, int m, int n, int nthreads, int *d,
              uint8_t *witness);

/* Exhaustive minimum Hamming weight of the isometric image (a,b,a+b) of the
 * row space (Sec. 2.4); equals twice the symplectic distance. */
int qdo_brute_iso_hamming(const uint8_t *B, int m, int n, int *dH);

/* Generator matrices Gamma_1..Gamma_h built by the diagonalization `diag`.
 *   h_out         number of matrices built (<= max_gamma)
 *   P[j]          packages of Gamma_j
 *   delta[j]      packages of Gamma_j whose pivot is outside its own qubit set
 *   dims[j*cap+i] 1 or 2: dimension of package i (2 means {r, s, r+s})
 *   pivot[j*cap+i] pivot qubit of package i, or -1 for the delta packages
 *   rows          optional: (j*cap+i)*2 + e -> row e of package i (2n bytes);
 *                 e = 1 unused for 1-dim packages
 * cap must be >= 2n.  Returns the rank on success, < 0 on error. */
int qdo_gamma(const uint8_t *B, int m, int n, int diag, int max_gamma,
              int cap, int *h_out, int *P, int *delta, int *dims, int *pivot,
              uint8_t *rows);

/* Mixed packages (not in the paper): the F4 construction where matrix j has
 * at most max2[j] two-row packages pivoted inside its set (max2 holds
 * max_gamma entries; -1: no cap).  Past the cap each package has one row,
 * pivoted at the first allowed column where a remaining row is nonzero,
 * and every other row is cleared to 0 or one symbol beta there.  Same
 * outputs as qdo_gamma. */
int qdo_gamma_mixed(const uint8_t *B, int m, int n, int max_gamma, const int *max2,
                    int cap, int *h_out, int *P, int *delta, int *dims, int *pivot,
                    uint8_t *rows);

/* One round of the enumeration: every choice of t distinct packages and one
 * nonzero element of each (Sec. 2.3, packages).  rows: P*2 rows of 2n bytes
 * (row 2i and, if dims[i] == 2, row 2i+1 span package i).  Writes the
 * minimum weight (n+1 if nothing was enumerated), one codeword reaching it,
 * and the number of combinations visited. */
int qdo_round(const uint8_t *rows, const int *dims, int P, int n, int t,
              int nthreads, int *wmin, uint8_t *witness,
              unsigned long long *count);

/* Weight distribution of the same round: hist[w] (n+1 entries) counts the
 * combinations whose sum has symplectic weight w.  Sum of hist = the
 * count of qdo_round; its least nonzero index below n+1 = its minimum. */
int qdo_round_hist(const uint8_t *rows, const int *dims, int P, int n, int t,
                   int nthreads, unsigned long long *hist);

/* Brouwer-Zimmermann over a given list of generator matrices (Sec. 2.1).
 * Gamma_j has P[j] packages starting at package offset off[j] of rows/dims,
 * delta[j] of which are not pivoted inside its own qubit set.
 * log: up to log_cap records of 5 long longs (t, j, L, U, combinations). */
int qdo_bz_gamma(int h, const int *P, const int *off, const int *delta,
                 const uint8_t *rows, const int *dims, int n, int nthreads,
                 int *d, uint8_t *witness, long long *log, int log_cap,
                 int *nlog);

/* Full pipeline: basis, generator matrices by `diag`, Brouwer-Zimmermann. */
int qdo_bz(const uint8_t *B, int m, int n, int diag, int max_gamma,
           int nthreads, int *d, uint8_t *witness, long long *log,
           int log_cap, int *nlog);

/* The same over the mixed-package F4 matrices of qdo_gamma_mixed. */
int qdo_bz_mixed(const uint8_t *B, int m, int n, int max_gamma, const int *max2,
                 int nthreads, int *d, uint8_t *witness, long long *log,
                 int log_cap, int *nlog);

/* Modified Brouwer-Zimmermann for a quantum stabilizer code (Sec. 2.1):
 * the rows of B generate the normalizer N = C^{perp_s}; the distance is the
 * least symplectic weight over N \ C, where the stabilizer C = N^{perp_s}
 * holds the codewords whose symplectic product with every row is 0.  When
 * N is self-orthogonal (k = 0) every nonzero codeword counts, as the paper
 * prescribes.  Same outputs as qdo_brute / qdo_bz; QDO_ERR_ZERO_CODE when no
 * codeword is admitted. */
int qdo_brute_stab(const uint8_t *B, int m, int n, int nthreads, int *d,
                   uint8_t *witness);
int qdo_bz_stab(const uint8_t *B, int m, int n, int diag, int max_gamma,
                int nthreads, int *d, uint8_t *witness, long long *log,
                int log_cap, int *nlog);

/* Saved_isometry (Sec. 2.4).  The image of each basis row (a|b) is
 * (a, b, a+b): a binary linear code of length 3n whose Hamming weights are
 * twice the symplectic weights.  Gamma_j is the reduced row echelon form of
 * the basis images on the columns outside the information sets of
 * Gamma_1..Gamma_{j-1}, scanned left to right (a-block, b-block,
 * (a+b)-block); its k[j] pivot columns form its information set.  Stops at
 * max_gamma matrices or when no column carries information.
 *   pivcol[j*r+i] pivot column of row i of Gamma_j, or -1
 *   rows          optional: (j*r+i) -> 3n bytes
 * where r is the rank (the return value; < 0 on error). */
int qdo_gamma_iso(const uint8_t *B, int m, int n, int max_gamma, int *h_out,
                  int *k, int *pivcol, uint8_t *rows);

/* Brouwer-Zimmermann for the Hamming weight (Sec. 2.1) over the matrices of
 * qdo_gamma_iso: round t sums t distinct rows of Gamma_j; after each round
 * L = sum_j max(0, t_j + 1 - (r - k_j)); stop when L >= U or a matrix has
 * run all r rows.  d = d_H / 2; witness: the 2n bytes (a|b) of the
 * codeword reaching d_H.  log records (t, j, L, U, combinations), with L
 * and U in Hamming units. */
int qdo_bz_iso(const uint8_t *B, int m, int n, int max_gamma, int nthreads,
               int *d, uint8_t *witness, long long *log, int log_cap, int *nlog);

#ifdef __cplusplus
}
#endif
#endif

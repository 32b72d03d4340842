/*
 * qdist.h -- C ABI of libqdist: exact symplectic minimum distance of binary
 * (additive) codes on an MI355X (gfx950) GPU, by Brouwer-Zimmermann
 * enumeration over package-systematic generator matrices.
 *
 * The operation is the one of Hernando, Quintana-Orti and Grassl, "Fast
 * Algorithms and Implementations for Computing the Minimum Distance of
 * Quantum Codes":
 *   d = min { wt_s(c) : c in C, c != 0 },  wt_s(a,b) = #{i : a_i or b_i != 0}
 * (Sec. 2, the first two displays), for the code C spanned by the rows of
 * a normalizer-type matrix (Sec. 2, the matrix A).  By default every
 * codeword updates U (the paper's modified algorithm does so for k = 0,
 * Sec. 2.1); QD_FILTER_STABILIZER applies its C^{perp_s} \ C test for k > 0.
 * The generator matrices are built by the diagonalizations of Sec. 2.2
 * (over F2) and Sec. 2.3 (over F4, with further matrices on the principal
 * columns), or as the information sets of the isometric image (Sec. 2.4);
 * the lower bound is the one of Sec. 2.1 and Sec. 2.3.
 *
 * Conventions for every entry point:
 *  - Buffers are host memory owned by the caller, read or written only
 *    during the call and never retained.
 *  - Matrix layout, row-major uint8:
 *      QD_FIELD_F2: m rows x 2n bytes in {0,1}; row = x_1..x_n | z_1..z_n
 *                   (the paper's (a|b)).
 *      QD_FIELD_F4: m rows x n bytes in {0,1,2,3}; code a + 2b is the
 *                   symbol a + alpha*b (Sec. 2.3).  The code is the F4-span
 *                   of the rows: each row g contributes g and alpha*g.
 *  - Rows need not be independent; the library works on a basis of their
 *    span.  A zero span is QD_ERR_ZERO_CODE.
 *  - 1 <= n <= QD_MAX_N.  Larger n is QD_ERR_TOO_LARGE.
 *  - On an error the return value is negative, *d is set to -1 (when d is
 *    not NULL) and the witness is left untouched.
 *  - The witness, when requested, is 2n bytes (x then z) of a codeword of
 *    weight d; any such codeword is a correct answer.
 *  - The current HIP device is used.  Calls from several threads are
 *    serialized per device.  There is no CPU fallback: without a usable
 *    gfx950 device the GPU entry points return QD_ERR_DEVICE.
 */
#ifndef QDIST_H
#define QDIST_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define QD_FIELD_F2 2
#define QD_FIELD_F4 4

#define QD_DIAG_AUTO 0
#define QD_DIAG_F2 2
#define QD_DIAG_F4 4
#define QD_DIAG_ISO 3 /* Saved_isometry (Sec. 2.4): binary information sets of the
                         image (x, z, x^z), bound on Hamming weight, d = d_H / 2 */

#define QD_FILTER_NONE 0       /* minimum over the whole span */
#define QD_FILTER_STABILIZER 1 /* Modified BZ (Sec. 2.1): the rows generate a normalizer
                                  N = C^{perp_s}; U takes only codewords of N outside the
                                  stabilizer C = N^{perp_s} (the radical of the span), so d is
                                  the quantum code's distance.  A self-orthogonal span (k = 0)
                                  counts every codeword, as the paper prescribes. */

#define QD_OK 0
#define QD_INCOMPLETE 1 /* budget, cancel or (plain walk) a round deeper than 8 packages:
                           *d = U, stats hold L <= d <= U */
#define QD_ERR_INVALID (-1)
#define QD_ERR_ZERO_CODE (-2)
#define QD_ERR_TOO_LARGE (-3)
#define QD_ERR_NOMEM (-4)
#define QD_ERR_DEVICE (-5)
#define QD_ERR_INTERNAL (-6)

#define QD_MAX_N 128
#define QD_MAX_GAMMA 8
#define QD_MAX_LOG 96

/* Resume point of a call that ended with QD_INCOMPLETE (its budget or
 * cancel flag stopped it before a round, or the plain walk reached a round
 * deeper than it supports): the rounds before (t, j) ran in full and found
 * U and a codeword of that weight.  A call on the same input with options
 * that give the same generator matrices (checked by `structure`) starts at
 * round (t, j) with these bounds and reaches the same distance. */
typedef struct qd_resume {
  int t, j;                   /* first round not run: qd_stats.next_t, next_j */
  int U;                      /* upper bound found: qd_stats.U (n + 1: none) */
  const uint8_t *witness;     /* 2n bytes of weight U as returned (NULL when U = n + 1) */
  unsigned long long structure; /* qd_stats.structure of that call */
} qd_resume;

/* Options of qd_distance_ex.  Zero-initialized means "library defaults". */
typedef struct qd_options {
  int diag;                   /* QD_DIAG_AUTO, QD_DIAG_F2, QD_DIAG_F4 or QD_DIAG_ISO */
  int max_gamma;              /* 0: planner decides; else at most this many matrices */
  unsigned long long budget;  /* stop before a round that would exceed this many
                                 combinations in total (0: no limit) -> QD_INCOMPLETE */
  const volatile int *cancel; /* host flag polled before each device step (NULL: none).
                                 With a flag a step carries at most 2^15 tiles of the
                                 code, so a long round spans several steps; a set flag
                                 stops the call before its first unfinished round
                                 (QD_INCOMPLETE, resumable) */
  void *stream;               /* hipStream_t for all work (NULL: the library's own) */
  int seg_len;                /* tuning override: table entries per tile, multiple of 8 (0: auto) */
  int saved_depth;            /* tuning override: max packages in the saved-sum table (0: auto;
                                 -1: none, each lane forms its whole combination -- the
                                 plain per-code path, for comparisons) */
  int timing;                 /* 1: time every enumeration launch with HIP events */
  int tops_mode;              /* tuning override: 0 auto, 1 tops from a table,
                                 2 tops unranked by each lane */
  int filter;                 /* QD_FILTER_NONE or QD_FILTER_STABILIZER */
  int scalar_classes;         /* F4-linear code (QD_FIELD_F4 input, or a binary span closed
                                 under alpha) with the F4 construction: 0 enumerate one
                                 codeword of each class {c, alpha c, alpha^2 c} (equal
                                 weights, a third of the work); -1 all */
  int partial_weight;         /* Partial weights: once U is small enough, decide a codeword
                                 from the weight of its first words plus the pivots its
                                 packages must hit beyond them, and evaluate the rest only
                                 where that bound is below U (same d and witness rules).
                                 0: for codes of two or more words per half whose planned
                                 work reaches 1e8 combinations; 1: for every code of two or
                                 more words per half; -1: never (every word of every
                                 codeword is evaluated) */
  int mixed_packages;         /* Additive codes with fewer independent rows than qubits, F4
                                 construction: 0 let the planner cap the two-row packages of
                                 the first two matrices (one-row packages spend the unused
                                 qubits) when that lowers the predicted work by 5% or more
                                 and the work reaches 1e10 combinations; 1 the same at any
                                 work; -1 never (two-row packages first, Sec. 2.3) */
  int walk;                   /* 0: the saved-sum engine.  k >= 1: the plain per-round walk,
                                 one launch per (t, Gamma_j) round and a readback of U after
                                 each: every lane unranks its first package set by its
                                 revolving-door rank (combinatorial number system), steps
                                 through k sets (k = 1: chosen from the round size) one
                                 package out and one in, and walks each set's element
                                 choices in reflected ternary Gray order, one element XOR
                                 per codeword.  Every codeword of the chosen matrices is
                                 enumerated (no scalar classes, mixed packages or partial
                                 weights).  Rounds of more than 8 packages end the call with
                                 QD_INCOMPLETE; QD_FILTER_STABILIZER is QD_ERR_INVALID.  At
                                 most 4096 */
  const qd_resume *resume;    /* continue an incomplete call (NULL: from the first round).
                                 Read during the call only.  A code whose matrices do not
                                 match resume->structure, or an invalid point or witness:
                                 QD_ERR_INVALID */
  int matrix_cores;           /* 0: rounds with a saved table run on the matrix cores
                                 (fp4 MFMA over +-1 sign vectors, exact: the weight of
                                 a XOR of two codewords is an affine function of the dot
                                 product of their signs over x, z and x ^ z), with an
                                 expanded copy of the table (64 bytes per entry and
                                 K-step, K-steps = words per half, one less when the last
                                 word has at most 10 qubits; 1 with partial weights);
                                 -1: vector ALU only.  Same d and witness rules either way */
} qd_options;

/* One (t, Gamma_j) round of the enumeration. */
typedef struct qd_round_log {
  int t, j;                   /* packages per combination, generator matrix */
  int L, U;                   /* bounds after the round */
  int saved_depth;            /* packages per saved-table entry used by the round */
  int launches;               /* enumeration kernel launches */
  unsigned long long combinations; /* combinations visited (exact count) */
  unsigned long long planned;      /* combinations in the full round, e_t(sizes) */
  float kernel_ms;            /* summed enumeration-kernel time (timing = 1) */
} qd_round_log;

/* Statistics of one qd_distance_ex call. */
typedef struct qd_stats {
  int n, rank, D;             /* D = 32-bit words per half on the device */
  int diag;                   /* construction used */
  int h;                      /* generator matrices enumerated */
  int P[QD_MAX_GAMMA];        /* packages per matrix */
  int delta[QD_MAX_GAMMA];    /* packages not pivoted inside the matrix's qubit set */
  int L, U;                   /* final bounds (L >= U unless QD_INCOMPLETE) */
  int d_estimate;             /* planner's distance estimate */
  double predicted;           /* planner's predicted combinations */
  unsigned long long combinations; /* combinations visited in total */
  unsigned long long enumerated; /* combinations the device enumerated: the visited ones
                                 plus those of rounds run ahead speculatively that the stop
                                 made unnecessary */
  unsigned long long words;   /* 32-bit words (of D per half) whose weight was evaluated,
                                 summed over the enumerated combinations: D x enumerated
                                 without partial weights, less with them */
  double host_ms;             /* input check, basis, diagonalization, planning */
  double kernel_ms;           /* summed enumeration-kernel time of the visited rounds
                                 (timing = 1) */
  double enumerated_kernel_ms; /* the same over every enumerated combination */
  double wall_ms;             /* whole call */
  int launches;               /* enumeration-kernel launches that carried its rounds
                                 (one launch may carry several consecutive rounds) */
  int logical_pairs;          /* QD_FILTER_STABILIZER: k, the logical operator pairs
                                 the admission test uses (0: no filter applied) */
  int scalar_classes;         /* 1: one codeword per F4 scalar class was enumerated */
  int two_row_cap[QD_MAX_GAMMA]; /* mixed packages: matrix j has at most this many two-row
                                 packages pivoted inside its set (-1: no cap) */
  int next_t, next_j;         /* first round not run (with QD_INCOMPLETE: the resume point) */
  unsigned long long structure; /* hash of the generator matrices enumerated (qd_resume) */
  int nlog;                   /* rounds run (entries in log, capped at QD_MAX_LOG) */
  qd_round_log log[QD_MAX_LOG];
  int matrix_core_launches;   /* of `launches`, those on the matrix cores (qd_options.matrix_cores) */
} qd_stats;

/* Structure chosen by the host planner (no GPU needed). */
typedef struct qd_plan_info {
  int n, rank;
  int diag;                   /* construction of the matrices below */
  int h;                      /* matrices built by that construction */
  int h_used;                 /* matrices the enumeration would use */
  int P[QD_MAX_GAMMA];
  int delta[QD_MAX_GAMMA];
  int dims[QD_MAX_GAMMA][2 * QD_MAX_N];   /* 1 or 2 per package */
  int pivot[QD_MAX_GAMMA][2 * QD_MAX_N];  /* qubit, or -1 for delta packages; for
                                             QD_DIAG_ISO the image column: q, n+q, 2n+q
                                             for x, z, x^z of qubit q */
  int d_estimate;
  double predicted_f2, predicted_f4;      /* predicted combinations per construction */
  double predicted_iso;
  int f4_two_row_cap[QD_MAX_GAMMA];       /* F4 matrices: the planner's cap on two-row packages
                                             (mixed packages, qd_options.mixed_packages = 0;
                                             -1: no cap) */
  int f4_scalar_classes;                  /* 1: the code is F4-linear, so the F4 prediction
                                             counts one codeword per scalar class */
} qd_plan_info;

/* Symplectic minimum distance of the code spanned by G (Sec. 2 definition,
 * computed with the Brouwer-Zimmermann bounds of Sec. 2.1).  witness: 2n
 * bytes or NULL.  Returns QD_OK or a negative error. */
int qd_distance(const uint8_t *G, int m, int n, int field, int *d, uint8_t *witness);

/* qd_distance with options and statistics (opt and st may be NULL). */
int qd_distance_ex(const uint8_t *G, int m, int n, int field, const qd_options *opt,
                   int *d, uint8_t *witness, qd_stats *st);

/* Distances of `count` independent codes.  Every code's rounds advance on
 * their own; each step of the batch launches the next rounds (or the next
 * piece of a large round) of every unfinished code together (one
 * enumeration launch per word count D), so small codes fill the device
 * jointly.  Arrays are indexed by code; witness
 * may be NULL or hold NULL entries; status[i] receives the per-code status
 * (as qd_distance).  Returns QD_OK when no code failed, else the first
 * negative status.  opt may be NULL; its budget and cancel apply to every
 * code.  Results equal those of qd_distance on each code alone. */
int qd_distance_batch(int count, const uint8_t *const *G, const int *m, const int *n,
                      const int *field, int *d, uint8_t *const *witness, int *status);
int qd_distance_batch_ex(int count, const uint8_t *const *G, const int *m, const int *n,
                         const int *field, const qd_options *opt, int *d,
                         uint8_t *const *witness, int *status, qd_stats *st);

/* Host-only: the generator matrices (Sec. 2.2 / Sec. 2.3 diagonalizations,
 * Sec. 2.4 information sets) and the planner's choice for one code.  diag = QD_DIAG_AUTO reports the
 * construction the planner picks.  No GPU is touched. */
int qd_plan(const uint8_t *G, int m, int n, int field, int diag, int max_gamma,
            qd_plan_info *out);

/* One enumeration round on the GPU over a caller-given package layout:
 * every choice of t distinct packages and one nonzero element of each
 * (Sec. 2.3, packages).  rows: 2P rows of 2n bytes; rows 2i and 2i+1 span
 * package i when dims[i] == 2, row 2i alone when dims[i] == 1.  Writes the
 * minimum symplectic weight (n + 1 when t > P), one codeword reaching it
 * (witness: 2n bytes or NULL) and the number of combinations visited.
 * partial_words = 0 evaluates every word of every codeword; 1 <= w < D
 * (D = 32-bit words per half) makes every tile evaluate words 0..w-1 first
 * and the rest only for blocks where some of those partial weights is
 * below the U the tile started with (no pivot credit: the packages carry
 * no pivots), which must give the same minimum and count. */
int qd_round_min(const uint8_t *rows, const int *dims, int P, int n, int t, int *wmin,
                 uint8_t *witness, unsigned long long *count,
                 int partial_words);

/* qd_round_min plus a census of the round's weight distribution (Sec. 2:
 * symplectic weight; Sec. 2.3: the round's combinations), taken by the same
 * enumeration kernel in the same tiles and blocks: below_count receives the
 * number of combinations whose codeword has weight < below, below_weight_sum
 * the sum of those weights (below > n + 1 counts every combination, so the
 * two are the round's size and total weight).  With partial_words = w the
 * tiles evaluate words 0..w-1 first and complete every block where some
 * partial weight is below max(U, below), so both figures stay exact.
 * below must be >= 1 (else QD_ERR_INVALID); other arguments and errors as
 * qd_round_min.  The output pointers must not be NULL. */
int qd_round_census(const uint8_t *rows, const int *dims, int P, int n, int t, int partial_words,
                    int below, int *wmin, uint8_t *witness, unsigned long long *count,
                    unsigned long long *below_count, unsigned long long *below_weight_sum);

/* -- Measured tuning of the launch shape -------------------------------------
 * The enumeration's launch shape per round is a segment length (saved-table
 * entries per tile) and a saved-table depth cap (packages per saved entry,
 * the "saving additions" of Sec. 2.1).  Without tuning the library picks
 * them by fixed rules; qd_tune_run measures them on the current device and
 * installs the fastest per bucket: word count D = 1..4, round size (nearest
 * of 2^20, 2^24, ..., 2^36 combinations) and codes sharing a step (1, 2-8,
 * more), for rounds that evaluate every word (rounds on partial weights
 * keep the fixed rules: a synthetic round has no pivot credit, so it does
 * not measure them faithfully).  For each bucket it times synthetic rounds
 * of random two-row packages under
 * every segment length in {64, 128, ..., 4096} and depth cap in {2, 3, 4}
 * (best of three runs after a warm-up; builds, launches and readbacks
 * included), and keeps the fixed rules' shape unless a candidate is faster
 * by more than 3%.  Installed shapes apply to every later call in the
 * process on every device, except the serving engine's (latency first) and
 * calls whose qd_options fix seg_len or saved_depth.  Results do not depend
 * on the shape.  The first GPU call of a process installs the file named by
 * $QD_TUNE_FILE, or tune_gfx950.json beside the library when that variable
 * is unset (an empty value: none).
 *
 * qd_tune_run: the sweep, stopped after max_seconds (> 0; QD_INCOMPLETE when
 * it stopped early, with the buckets measured so far installed).  json
 * (json_len bytes, may be NULL) receives the installed table as text;
 * QD_ERR_INVALID if it does not fit.  qd_tune_load installs such a text
 * (QD_ERR_INVALID if it does not parse; nothing changes then);
 * qd_tune_get writes the installed table; qd_tune_reset returns to the
 * fixed rules. */
int qd_tune_run(double max_seconds, char *json, size_t json_len);
int qd_tune_load(const char *json);
int qd_tune_get(char *json, size_t json_len);
int qd_tune_reset(void);

/* Device bytes of the fixed array qd_round_min_noalloc works in (per GPU). */
#define QD_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * qd_round_min with every device buffer it needs (elements, e_r tables,
 * saved and tops tables, tile plans, state, counters, witness slots) carved
 * from one fixed device array of QD_NOALLOC_SCRATCH_BYTES that each GPU
 * holds from the first call until the process ends.  It calls no hipMalloc,
 * hipFree, hipHostMalloc, stream or event creation; inputs are read from
 * host memory and uploaded from pageable memory.  Tables are kept to a
 * quarter of the array (shallower saved tables, unranked tops); a round
 * whose plan still does not fit returns QD_ERR_TOO_LARGE with no result
 * (its planning step fails before it uploads or launches).  stream: the HIP stream to run on (NULL: the null stream); the call
 * returns after the stream has finished its work.  Calls on one GPU share
 * its array and run one at a time within a process (they serialize on a
 * lock); every call re-initializes what it reads.  Outputs, partial_words
 * and errors as qd_round_min; QD_ERR_DEVICE without a gfx950 device. */
int qd_round_min_noalloc(const uint8_t *rows, const int *dims, int P, int n, int t, int *wmin,
                         uint8_t *witness, unsigned long long *count, int partial_words,
                         void *stream);

/* The same round with the plain walk kernel (qd_options.walk = per_lane:
 * package sets per lane, 1..4096, 1 choosing from the round size; others
 * QD_ERR_INVALID; t > 8 is QD_ERR_TOO_LARGE): minimum symplectic weight,
 * one codeword reaching it and the number of combinations, as
 * qd_round_min.  weight_sum (may be NULL) receives the sum of the
 * symplectic weights of the codewords of every combination of the round
 * (each walked once). */
int qd_round_walk(const uint8_t *rows, const int *dims, int P, int n, int t, int per_lane,
                  int *wmin, uint8_t *witness, unsigned long long *count,
                  unsigned long long *weight_sum);

/* -- Serving: continuous batching of distance requests ------------------------
 * A qd_engine owns a worker thread and a HIP stream.  Requests are checked
 * and planned on the submitting thread, then wait until the worker admits
 * them: first come first served, while fewer than max_active codes are on
 * the device and their estimated device footprint (generator matrices,
 * saved tables) fits mem_budget.  Every step of the worker launches the next
 * round piece of every admitted code together, so requests that arrive
 * while others run join the device work at the next step.  Results are
 * identical to qd_distance on the same input (the enumeration, bounds and
 * stopping rule do not depend on what else is in the step). */
typedef struct qd_engine qd_engine;

typedef struct qd_result {
  unsigned long long tag;     /* caller's tag from qd_engine_submit */
  int status;                 /* as qd_distance */
  int d;                      /* distance (-1 on error) */
  int L;                      /* certified lower bound (= d unless QD_INCOMPLETE) */
  int n;
  double latency_ms;          /* submit to completion */
  double queue_ms;            /* submit to admission */
  unsigned long long combinations;
} qd_result;

/* mem_budget: device bytes for admitted codes (0: 8 GiB); max_active: codes
 * on the device at once (0: 512); stream: hipStream_t or NULL (own stream).
 * Returns NULL without a usable gfx950 device. */
qd_engine *qd_engine_create(size_t mem_budget, int max_active, void *stream);

/* Copies G and queues it; opt may be NULL (its stream and timing fields are
 * ignored).  Returns QD_OK, or a negative status for a rejected request
 * (which is still reported by qd_engine_poll with that status). */
int qd_engine_submit(qd_engine *e, const uint8_t *G, int m, int n, int field, unsigned long long tag,
                     const qd_options *opt);

/* Moves up to max finished results to out (and their witnesses to
 * witness + i * 2 * QD_MAX_N when witness is not NULL), waiting up to
 * wait_ms for the first one.  Returns the number of results. */
int qd_engine_poll(qd_engine *e, qd_result *out, uint8_t *witness, int max, int wait_ms);

/* Requests submitted and not yet returned by qd_engine_poll. */
int qd_engine_outstanding(qd_engine *e);

/* Stops the worker: queued and running requests end as QD_INCOMPLETE and
 * are discarded.  The engine pointer is invalid afterwards. */
void qd_engine_destroy(qd_engine *e);

/* Human-readable status. */
const char *qd_strerror(int status);

/* Device probe: 0 when a gfx950 device is usable; name receives up to len-1
 * bytes of the device name. */
int qd_device_check(char *name, int len);

/* Sustained integer-VALU rate on the current device, measured by a chain of
 * independent 32-bit XOR/OR/popcount operations: lane-ops per second. */
int qd_valu_peak(double *lane_ops_per_s);

/* Integer-VALU issue rate of one fixed instruction mix, for reading the
 * round kernel's roofline: 8 independent chains per lane, 3 operations per
 * chain step, 16 workgroups of 256 lanes per CU.  Profiling counters of the
 * launch (SQ_ACTIVE_INST_VALU2 and the like) show which mixes dual-issue.
 *   QD_MIX_HOTLOOP_SGPR  XOR (SGPR operand), XOR-OR v_bitop3 (SGPR operand),
 *                        v_bcnt: the hot loop's per-word sequence
 *   QD_MIX_HOTLOOP_VGPR  the same with every operand in VGPRs
 *   QD_MIX_BCNT          v_bcnt only
 *   QD_MIX_XOR_VGPR      XOR only, VGPR operands
 *   QD_MIX_XOR_SGPR      XOR only, one SGPR operand
 * Writes lane-ops per second; QD_ERR_INVALID for an unknown mix. */
enum {
  QD_MIX_HOTLOOP_SGPR = 0,
  QD_MIX_HOTLOOP_VGPR = 1,
  QD_MIX_BCNT = 2,
  QD_MIX_XOR_VGPR = 3,
  QD_MIX_XOR_SGPR = 4
};
int qd_valu_mix(int mix, double *lane_ops_per_s);

#ifdef __cplusplus
}
#endif
#endif

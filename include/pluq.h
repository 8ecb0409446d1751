/*
 * pluq.h -- C ABI of the MI355X (gfx950) rank-profile-revealing PLUQ library.
 *
 * The library computes the PLUQ decomposition of Dumas, Pernet and Sultan,
 * "Simultaneous computation of the row and column rank profiles" (ISSAC 2013),
 * of an m x n matrix A of rank r over a prime field GF(p):
 *
 *     A = P [L; M] [U V] Q                      (Algorithm 1, Section 2)
 *
 * with L r x r unit lower triangular, U r x r upper triangular, and A
 * overwritten in place by the packed form [L\U V; M 0].  P and Q come from
 * the quad-recursive pivoting of Algorithm 1: the first r entries of P (of Q)
 * are the pivot rows (columns), so the row and column rank profiles of A and
 * of every leading k x t sub-matrix are read off P and Q (corollaries of
 * Section 4).
 *
 * Conventions common to every entry point
 * ---------------------------------------
 *  - Storage is row-major: element (i, j) is at A[i * lda + j], lda >= n.
 *  - Entries are canonical integers in [0, p), stored exactly in the chosen
 *    element type (int64, float64 or int32).  On return A again holds
 *    canonical values.
 *  - Permutation vectors are int64: P[i] is the original row of packed row i
 *    and Q[j] the original column of packed column j, so that
 *    A_in[P[i], Q[j]] == (L U)[i, j] for every i, j.
 *  - The result is unique: pivots in the order of Algorithm 1's four
 *    recursive calls with floor(m/2) x floor(n/2) splits, the non-pivot rows
 *    and columns after them in ascending order, and [L\U V; M 0] the LU
 *    factorisation without pivoting of A_in[P, Q].  No option changes it.
 *  - Moduli: p prime, 2 <= p < 2^26 is accepted (every product of two reduced
 *    residues is then exact in an IEEE double); the forms narrow it further
 *    (PLUQ_ERR_UNSUPPORTED): FP64 needs p < 2^25, INT8 p <= 65536, FP32
 *    p < 2^11.  Primality is not checked.
 *  - Device pointers are HIP device allocations of the calling process; host
 *    pointers are ordinary host memory.  The caller owns every buffer.
 *  - `stream` is a hipStream_t (NULL = the default stream).  All device work
 *    is issued on it.  Calls returning a host-visible result (r) synchronise
 *    the stream before returning.
 *  - Functions never throw; they return a pluq_status.  Arguments are
 *    validated before any device memory is touched.  PLUQ_ERR_DEVICE means a
 *    HIP call failed after work started: the contents of A, P and Q are then
 *    unspecified.
 *  - Calls are not re-entrant on the same buffers; distinct calls on distinct
 *    buffers and streams may run concurrently.
 */
#ifndef PLUQ_H
#define PLUQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PLUQ_OK = 0,
    PLUQ_ERR_ARG = 1,          /* bad dimension, leading dimension, null pointer */
    PLUQ_ERR_MODULUS = 2,      /* p outside [2, 2^26) */
    PLUQ_ERR_RANGE = 3,        /* an entry outside [0, p) (only with validation) */
    PLUQ_ERR_UNSUPPORTED = 4,  /* the requested form cannot be exact for this p */
    PLUQ_ERR_NOMEM = 5,        /* host allocation failed */
    PLUQ_ERR_DEVICE = 6,       /* a HIP call failed */
    PLUQ_ERR_WORKSPACE = 7     /* workspace smaller than pluq_workspace_size() */
} pluq_status;

/* Element storage type of the matrices passed in. */
typedef enum { PLUQ_I64 = 0, PLUQ_F64 = 1, PLUQ_I32 = 2 } pluq_dtype;

/* Arithmetic form of the matrix-multiply updates (the other steps are the
 * same in every form).  All forms give bit-identical results.
 *   FP64 -- float64 matrix cores, residues in symmetric form, products
 *           accumulated exactly and reduced once per chunk of the inner
 *           dimension (delayed reduction, Section 6): needs a chunk K >= 16
 *           with K * ((p-1)/2)^2 + 4p < 2^52, i.e. p < 2^25.
 *   INT8 -- each residue, moved into the window [-32896, 32639] (a or a - p),
 *           is written as two signed base-256 digits (one digit in
 *           [-128, 127] when p <= 256); the limb products run on the int8
 *           matrix cores with int32 accumulation and are recombined exactly
 *           in float64 (p <= 65536).  Updates smaller than about 2^26
 *           multiply-adds stay in the FP64 kernel.  Needs the larger
 *           workspace that pluq_workspace_size reports for this form.
 *   FP32 -- float32 matrix cores on symmetric residues, reduced (in float64)
 *           after at most K products with K * (p/2)^2 + p < 2^24, K >= 16,
 *           i.e. p < 2^11 (K = 1072 for p = 251).
 * The triangular-solve inverses and the base case use float64 arithmetic in
 * every form.  A form that cannot be exact for p gives PLUQ_ERR_UNSUPPORTED.
 */
typedef enum { PLUQ_FORM_FP64 = 0, PLUQ_FORM_INT8 = 1, PLUQ_FORM_FP32 = 2 } pluq_form;

typedef struct {
    int32_t form;             /* pluq_form */
    int32_t validate_entries; /* non-zero: scan A for entries outside [0,p) first */
    int32_t cutoff_override;  /* > 0: base-case tiles at most this many rows and columns (tuning only) */
    int32_t batch_panel;        /* batched form: panel width 8 or 16 (0: 8; tuning only) */
    int32_t batch_groups;       /* batched form: persistent work-groups per compute unit
                                   (0: 4 for panel 8, 2 for panel 16; tuning only) */
    int32_t no_speculation;     /* non-zero: no speculative first attempt (pluq_modp) and
                                   no room for it in pluq_workspace_size */
    int32_t branches;           /* concurrent recursion branches of pluq_modp: the calls
                                   PLUQ(F) and PLUQ(G) of a node, both at least
                                   pluq_tune.fork_min_dim (128) in each dimension,
                                   run side by side while a branch is free (0: 8; 1: none;
                                   at most 16); each branch needs its own workspace share
                                   (pluq_workspace_size counts them); the result does not
                                   depend on it */
    int32_t in_place;           /* non-zero: a workspace linear in m + n, independent of
                                   m n (Section 2's in-place remark): no copy of A (no
                                   speculative attempt), one branch, permutations through
                                   strips of 64 columns or rows, the INT8 form's digit
                                   planes for 512-deep pieces; same result, more launches */
} pluq_opts;

/* Human-readable name of a status code (static storage). */
const char *pluq_status_string(pluq_status s);

/* Library version string (static storage). */
const char *pluq_version(void);

/* Detail of the last failure on the calling thread (which HIP call or host
 * allocation failed, and its error string); "" if none.  Thread-local
 * storage, valid until the thread's next failing call. */
const char *pluq_last_error(void);

/*
 * Device workspace, in bytes, needed by pluq_modp for an m x n matrix of the
 * given element type, modulus and options (opts may be NULL for defaults).
 * Returns 0 for invalid arguments.
 */
size_t pluq_workspace_size(int64_t m, int64_t n, pluq_dtype dt, uint64_t p,
                           const pluq_opts *opts);

/*
 * PLUQ decomposition, Algorithm 1 (Section 2), of the m x n matrix at dA.
 *   dA       device, m x n row-major, leading dimension lda >= max(1, n);
 *            overwritten by [L\U V; M 0] (canonical residues).
 *   dP, dQ   device int64 arrays of length m and n (may be NULL when m or n
 *            is 0); receive P and Q as described above.
 *   r_out    host; receives the rank r.
 *   opts     NULL for defaults (FP64 form, no validation).
 *   dWork    device workspace of work_bytes >= pluq_workspace_size(...),
 *            256-byte aligned; its contents are scratch.
 * Unless opts->no_speculation is set, a matrix larger than one base-case
 * tile whose copy fits in 1 GiB is first decomposed speculatively: every
 * base-case tile is taken to be full rank in the identity order (a generic
 * rank profile) without waiting for its result; the workspace holds a copy
 * of A, and if any tile breaks the assumption A is restored from it and the
 * exact recursion runs from the start.  The result is the same either way;
 * only the time differs (faster on generic inputs, about one extra partial
 * attempt otherwise).
 *   stream   HIP stream all the work is ordered on (NULL: the null
 *            stream).  The call returns when the decomposition is complete.
 *            The two independent triangular solves of each recursion node
 *            share their launches (one grid carries both), so no other
 *            stream is used.
 * m == 0 or n == 0 gives r = 0 and identity permutations.
 * Errors: PLUQ_ERR_ARG, PLUQ_ERR_MODULUS, PLUQ_ERR_UNSUPPORTED,
 * PLUQ_ERR_WORKSPACE (all before A is touched), PLUQ_ERR_RANGE (validation
 * scan, A untouched), PLUQ_ERR_DEVICE.
 */
pluq_status pluq_modp(int64_t m, int64_t n, void *dA, int64_t lda, pluq_dtype dt,
                      uint64_t p, int64_t *dP, int64_t *dQ, int64_t *r_out,
                      const pluq_opts *opts, void *dWork, size_t work_bytes,
                      void *stream);

/*
 * Row and column rank profiles from P, Q and r (host arrays): the sorted
 * first r entries of P and of Q (last corollary of Section 4).
 * row_rp and col_rp receive r values each.
 */
pluq_status pluq_rank_profiles(int64_t m, int64_t n, int64_t r, const int64_t *P,
                               const int64_t *Q, int64_t *row_rp, int64_t *col_rp);

/*
 * Rank profiles of the leading k x t sub-matrix of A (first corollary of
 * Section 4): the sorted row and column indices of the non-zero entries of
 * the leading k x t block of P [I_r 0; 0 0] Q, i.e. the pivots (P[s], Q[s]),
 * s < r, with P[s] < k and Q[s] < t.  rows and cols (host, capacity >= r)
 * receive `*count` sorted indices each.
 */
pluq_status pluq_leading_rank_profiles(int64_t m, int64_t n, int64_t r,
                                       const int64_t *P, const int64_t *Q,
                                       int64_t k, int64_t t, int64_t *rows,
                                       int64_t *cols, int64_t *count);

/*
 * Batched PLUQ: `batch` independent matrices, each decomposed exactly as by
 * pluq_modp (same P, Q, r and packed factors), in one persistent kernel
 * launch on `stream` with every pivoting decision taken on the device.
 *   m, n, lda        host arrays of length batch; 0 <= m, n <= 512.
 *   dA, dP, dQ       host arrays of `batch` device pointers (A in place,
 *                    P of length m[b], Q of length n[b], int64).
 *   d_r              device int64 array of length batch; receives the ranks
 *                    (-1 for a matrix whose internal self-check failed).
 *   dWork/work_bytes device workspace >= pluq_batched_workspace_size(...),
 *                    256-byte aligned: a descriptor table and a backup copy
 *                    of every matrix.
 * Only the FP64 form's arithmetic is used (the updates are rank-16 and too
 * small for the matrix cores); opts may select the panel width and the
 * number of resident work-groups.
 *
 * pluq_modp_batched = pluq_batched_prepare + pluq_batched_run.
 *   prepare  validates the arguments and writes the descriptor table into
 *            dWork (synchronous host-to-device copy; no kernel).
 *   run      enqueues the single kernel on `stream` and returns: it makes
 *            no host-device transfer and no synchronisation, so it may be
 *            captured into a HIP graph and replayed; every replay works on
 *            the matrices the descriptors point to, in place.
 * Errors as for pluq_modp; PLUQ_ERR_UNSUPPORTED for a dimension above 512.
 */
size_t pluq_batched_workspace_size(int64_t batch, const int64_t *m, const int64_t *n,
                                   pluq_dtype dt, uint64_t p, const pluq_opts *opts);
pluq_status pluq_batched_prepare(int64_t batch, const int64_t *m, const int64_t *n,
                                 void *const *dA, const int64_t *lda, pluq_dtype dt,
                                 uint64_t p, int64_t *const *dP, int64_t *const *dQ,
                                 int64_t *d_r, const pluq_opts *opts, void *dWork,
                                 size_t work_bytes);
pluq_status pluq_batched_run(int64_t batch, pluq_dtype dt, uint64_t p, const pluq_opts *opts,
                             void *dWork, size_t work_bytes, void *stream);
pluq_status pluq_modp_batched(int64_t batch, const int64_t *m, const int64_t *n,
                              void *const *dA, const int64_t *lda, pluq_dtype dt,
                              uint64_t p, int64_t *const *dP, int64_t *const *dQ,
                              int64_t *d_r, const pluq_opts *opts, void *dWork,
                              size_t work_bytes, void *stream);

/* ---- tuning (performance only: no parameter changes any result) ----
 *
 * A process-wide table of tuned parameters, filled by the project's tuner
 * (paper_1301_4438_amd/tune.py writes a cache that the Python binding
 * loads).  An entry is keyed by (form, p class, element type, shape bucket):
 * form a pluq_form, or 3 for the batched form; p class 0 for p <= 256, 1 for
 * p <= 65536, 2 above; bucket floor(log2(min(m, n))) (0 for the batched
 * form); -1 in a key matches anything, and the most specific matching entry
 * wins.  A
 * zero field means the built-in default; explicit pluq_opts fields
 * (cutoff_override, batch_panel, batch_groups) take precedence.
 */
typedef struct {
    int32_t mm_tiles128;   /* an MM launch uses 128 x 128 tiles from this many such tiles on (0: 240) */
    int32_t mm_tiles64;    /* else 64 x 64 tiles from this many on, else 32 x 32 (0: 192) */
    int32_t cutoff;        /* base-case tile dimension, 16 .. 128 (0: 128) */
    int32_t fork_min_dim;  /* PLUQ(F) || PLUQ(G) when both are at least this (0: 128) */
    int64_t i8_min_work;   /* INT8 form: updates below this many multiply-adds stay in FP64 (0: 2^26) */
    int32_t batch_panel;   /* batched form: panel width 8 or 16 (0: 8) */
    int32_t batch_groups;  /* batched form: work-groups per compute unit (0: 4 for panel 8, 2 for 16) */
    int32_t strassen_min;  /* FP64 / FP32 forms: an MM update of the recursion whose three dimensions
                              are all at least this takes one level of Winograd's 7-product scheme
                              (>= 128; 0: 4096; a value above every dimension turns it off).  The
                              workspace holds it only when min(m, n) >= 2 * strassen_min at the time
                              of the size query; a smaller workspace keeps the classical update. */
} pluq_tune;

pluq_status pluq_tune_set(int32_t form, int32_t pclass, int32_t dtype, int32_t bucket, const pluq_tune *t);
void pluq_tune_clear(void);
/* The parameters a call with these arguments uses (defaults filled in);
 * returns 1 in *from_table when a table entry matched, else 0. */
pluq_status pluq_tune_get(int32_t form, uint64_t p, int32_t dtype, int64_t m, int64_t n, pluq_tune *out,
                          int32_t *from_table);

/* ---- outputs read off a decomposition by permutation (Sections 3, 4) ----
 *
 * All take the result of pluq_modp -- the packed X = [L\U V; M 0] (m x n,
 * row-major, ldx) and the device index vectors P, Q with the rank r -- and
 * a device workspace of pluq_post_workspace_size(m, n) bytes (256-byte
 * aligned); they are asynchronous on `stream` and leave X, P and Q
 * unchanged.  P and Q must be the vectors pluq_modp returned (entries out of
 * range are skipped, never used to address memory, but then the outputs are
 * unspecified).
 */
size_t pluq_post_workspace_size(int64_t m, int64_t n);

/*
 * The LEU decomposition of Section 3, A = Lbar E Ubar:
 *   Lbar = P [L 0; M I] P^T   (m x m, unit lower triangular by Section 3's
 *                              theorem) into dLbar (ldl >= m);
 *   Ubar = Q^T [U V; 0 I] Q   (n x n, upper triangular with non-zero
 *                              diagonal) into dUbar (ldu >= n);
 *   E = P [I_r 0; 0 0] Q      the rank profile matrix, as dErow (length m,
 *                              int64, may be NULL): the column of row i's
 *                              non-zero entry, or -1.
 * Element type dt for X, Lbar and Ubar.
 */
pluq_status pluq_leu(int64_t m, int64_t n, int64_t r, const void *dX, int64_t ldx,
                     pluq_dtype dt, const int64_t *dP, const int64_t *dQ, void *dLbar,
                     int64_t ldl, void *dUbar, int64_t ldu, int64_t *dErow, void *dWork,
                     size_t work_bytes, void *stream);

/*
 * Echelon factorizations taken from the LEU factors by permutation only:
 *   PLUQ_ECHELON_COLUMN: A = C R with C = the columns of Lbar at the pivot
 *     rows in ascending order (m x r, column echelon form: column k is zero
 *     above row prof[k], 1 there) into dF (ldf >= r), R = the rows of Ubar at
 *     the paired columns (r x n) into dG (ldg >= n), and prof = the row rank
 *     profile (r int64) -- the echelon factor of a CUP decomposition;
 *   PLUQ_ECHELON_ROW: A = L_E E with E = the rows of Ubar at the pivot
 *     columns in ascending order (r x n, row echelon form: row k is zero
 *     left of column prof[k], non-zero there) into dF (ldf >= n), L_E = the
 *     columns of Lbar at the paired rows (m x r) into dG (ldg >= r), and
 *     prof = the column rank profile -- the echelon factor of a PLE
 *     decomposition.
 * (The co-factors R and L_E are not triangular in general: the pivots of
 * Algorithm 1 come in the order of its recursion, not in the row or column
 * order a CUP or PLE elimination would take.)
 */
enum { PLUQ_ECHELON_COLUMN = 0, PLUQ_ECHELON_ROW = 1 };
pluq_status pluq_echelon(int32_t kind, int64_t m, int64_t n, int64_t r, const void *dX,
                         int64_t ldx, pluq_dtype dt, const int64_t *dP, const int64_t *dQ,
                         void *dF, int64_t ldf, void *dG, int64_t ldg, int64_t *dProf,
                         void *dWork, size_t work_bytes, void *stream);

/*
 * Ranks of leading sub-matrices, a batch of queries on the device (Section
 * 4: the rank of the leading k x t block is the number of rank profile
 * matrix entries in it): dranks[q] = rank(A[0:dk[q], 0:dt[q]]) for
 * q < nq (device int64 arrays).
 */
pluq_status pluq_leading_ranks(int64_t m, int64_t n, int64_t r, const int64_t *dP,
                               const int64_t *dQ, int64_t nq, const int64_t *dk,
                               const int64_t *dt, int64_t *dranks, void *dWork,
                               size_t work_bytes, void *stream);

/*
 * Row and column rank profiles of the leading k x t sub-matrix on the
 * device (the device form of pluq_leading_rank_profiles): drows, dcols
 * (device, capacity >= r) receive the sorted profiles and dcount[0],
 * dcount[1] (device int64) their lengths (equal: the block's rank).
 */
pluq_status pluq_leading_rank_profiles_device(int64_t m, int64_t n, int64_t r,
                                              const int64_t *dP, const int64_t *dQ,
                                              int64_t k, int64_t t, int64_t *drows,
                                              int64_t *dcols, int64_t *dcount, void *dWork,
                                              size_t work_bytes, void *stream);

/* ---- building blocks of Section 2 (device, for direct use and tests) ---- */

/*
 * MM(C, A, B) of Section 2: C <- C - A B mod p, with C m x n (ldc), A m x k
 * (lda), B k x n (ldb), all device, row-major, element type dt, canonical
 * residues.  `form` selects the matrix-core arithmetic (pluq_form); results
 * are identical for every form.  dWork/work_bytes: scratch for the INT8
 * form's limb planes (>= pluq_modmm_workspace_size, 256-byte aligned; may be
 * NULL when that is 0).  In the INT8 form this entry point always uses the
 * int8 matrix cores, whatever the size.  Asynchronous on `stream`.
 */
size_t pluq_modmm_workspace_size(int64_t m, int64_t n, int64_t k, int32_t form);
pluq_status pluq_modmm(int64_t m, int64_t n, int64_t k, void *dC, int64_t ldc,
                       const void *dA, int64_t lda, const void *dB, int64_t ldb,
                       pluq_dtype dt, uint64_t p, int32_t form, void *dWork,
                       size_t work_bytes, void *stream);

/*
 * MM(C, A, B) with one level of Winograd's form of Strassen's product: the
 * sub-cubic matrix product that Section 5's O(m n r^(omega-2)) bound counts
 * on.  A, B and C are cut into 2 x 2 blocks of floor(m/2) x floor(k/2),
 * floor(k/2) x floor(n/2) and floor(m/2) x floor(n/2); the 7 block products
 * run on the matrix cores of `form` (PLUQ_FORM_FP64 or PLUQ_FORM_FP32; the
 * INT8 form is PLUQ_ERR_UNSUPPORTED), the 8 operand sums and the output
 * combinations are reduced to canonical residues, and a last row, column or
 * inner index left over by odd sizes is updated classically.  Every
 * operation is exact mod p, so C ends bit-identical to pluq_modmm's.
 * Same arguments as pluq_modmm; dWork holds the block sums and two block
 * products: pluq_modmm_winograd_workspace_size(m, n, k, dt) bytes, 256-byte
 * aligned.  m, n and k must be at least 2 (else PLUQ_ERR_ARG).
 * Asynchronous on `stream`.  pluq_modp applies the same scheme to the large
 * updates of its recursion (pluq_tune.strassen_min).
 */
size_t pluq_modmm_winograd_workspace_size(int64_t m, int64_t n, int64_t k, pluq_dtype dt);
pluq_status pluq_modmm_winograd(int64_t m, int64_t n, int64_t k, void *dC, int64_t ldc,
                                const void *dA, int64_t lda, const void *dB, int64_t ldb,
                                pluq_dtype dt, uint64_t p, int32_t form, void *dWork,
                                size_t work_bytes, void *stream);

/*
 * pluq_modmm without a workspace argument and without allocating anything,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, semantics and results as pluq_modmm.  In the INT8 form the
 * digit planes go to a static 64 MiB device array of the library (one per
 * device, held until the process ends), so m + n may be at most 1048576 for
 * p <= 256 (one digit) and 524288 for larger p (two digits), else
 * PLUQ_ERR_WORKSPACE with the limit in pluq_last_error(); the other forms
 * use no scratch.  All calls on
 * one device share that array: calls that overlap on one device (on
 * different streams or threads) race and must be ordered by the caller.
 * Asynchronous on `stream`; the first call on a device looks the array's
 * address up once (hipGetSymbolAddress).
 */
pluq_status pluq_modmm_noalloc(int64_t m, int64_t n, int64_t k, void *dC, int64_t ldc,
                               const void *dA, int64_t lda, const void *dB, int64_t ldb,
                               pluq_dtype dt, uint64_t p, int32_t form, void *stream);

/*
 * TRSM of Section 2 (device, row-major, canonical residues, asynchronous):
 *   side = 0: B <- L^{-1} B, L r x r unit lower triangular (its diagonal and
 *             upper part are not read), B r x ncols;
 *   side = 1: B <- B U^{-1}, U r x r upper triangular with non-zero diagonal
 *             (its strict lower part is not read), B nrows x r.
 * `other` is ncols (side 0) or nrows (side 1).  The 64 x 64 diagonal blocks
 * of the triangle are inverted first (exactly, over the field) and the solve
 * then runs as matrix-multiply updates; dWork must hold
 * pluq_trsm_workspace_size(r, dt) bytes, 256-byte aligned.
 */
size_t pluq_trsm_workspace_size(int64_t r, pluq_dtype dt);
pluq_status pluq_trsm(int32_t side, int64_t r, int64_t other, const void *dT,
                      int64_t ldt, void *dB, int64_t ldb, pluq_dtype dt, uint64_t p,
                      int32_t form, void *dWork, size_t work_bytes, void *stream);

/*
 * Statistics of the last pluq_modp call on this thread (host): number of
 * recursion nodes, base cases, kernel launches and stream synchronisations.
 * Any pointer may be NULL.
 */
void pluq_last_stats(int64_t *nodes, int64_t *basecases, int64_t *launches,
                     int64_t *syncs);

/*
 * Per-kernel-class timing (host, per calling thread).  When enabled, every
 * kernel launch of pluq_modp is bracketed by HIP events on the caller's
 * stream and, per class, the launch count, the summed device time and the
 * algorithmic work are accumulated:
 *   flops -- 2 * M * N * K of each matrix-multiply update (twice the
 *            classical multiply-add count; for PLUQ_K_MODMM_I8 times the
 *            limb products per multiply-add, i.e. int8 operations), the
 *            matrix-core work of the solve leaves, 0 for the other classes;
 *   bytes -- compulsory HBM traffic of the launch (operands read once,
 *            outputs read and written once).
 * pluq_profile_enable(mask) resets the counters and records the classes
 * whose bit (1 << class) is set in mask (-1: all, 0: stop); untimed classes
 * cost nothing.  pluq_profile_read fills PLUQ_K_COUNT entries; launches of
 * the asynchronous entry points (pluq_modmm, pluq_trsm) that are still
 * pending are waited for first.
 */
enum {
    PLUQ_K_MODMM = 0,     /* MM updates (Schur complements, TRSM updates) */
    PLUQ_K_TRSM_LEAF = 1, /* triangular-solve leaves */
    PLUQ_K_PERM = 2,      /* row / column permutations */
    PLUQ_K_BASECASE = 3,  /* base-case tiles */
    PLUQ_K_SCAN = 4,      /* zero / range scans */
    PLUQ_K_LIMB = 5,      /* INT8 form: digit-plane split of MM operands */
    PLUQ_K_MODMM_I8 = 6,  /* INT8 form: limb GEMMs of the large MM updates */
    PLUQ_K_TRSM_DIAG = 7, /* triangular solves: inversion of the 64 x 64 diagonal blocks */
    PLUQ_K_BASECASE_RPM = 8, /* base case: rank-profile search of a non-generic tile */
    PLUQ_K_LINCOMB = 9,   /* Winograd's block sums and output combinations */
    PLUQ_K_COUNT = 10
};
typedef struct {
    int64_t launches;
    double ms;
    double flops;
    double bytes;
} pluq_kernel_stat;
void pluq_profile_enable(int32_t mask);
void pluq_profile_read(pluq_kernel_stat *out);

#ifdef __cplusplus
}
#endif

#endif /* PLUQ_H */

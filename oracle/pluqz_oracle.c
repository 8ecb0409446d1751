/*
 * Oracle for the rank-profile-revealing PLUQ decomposition over GF(p)
 * (Dumas, Pernet, Sultan, "Simultaneous computation of the row and column
 * rank profiles", ISSAC 2013).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, obviously-correct CPU
 * implementation used to check the GPU library.  Only the test-suite, the
 * smoke entry point and the benchmark's CPU-baseline leg may load it.  It
 * shares no code with the GPU path.
 *
 * All matrices are row-major int64 with entries in [0, p); every product is
 * reduced immediately with the C `%` operator on unsigned integers, so p must
 * be below 2^32 (p^2 + p then fits an unsigned 64-bit integer).
 *
 * The output convention ("PLUQ-Z") is the one computed by the paper's
 * Algorithm 1 (Section 2) with floor(m/2) x floor(n/2) splits and with the
 * leaves' index exchange read as a cyclic rotation:
 *   - the pivots are the r positions of the rank profile matrix (RPM),
 *     ordered by the quadrant recursion of Algorithm 1 (A1, F, G, R);
 *   - non-pivot rows and columns follow in ascending order (this is what the
 *     theorem of Section 3 requires for L-bar / U-bar to be triangular);
 *   - L\U, M and V are then the unique LU factorisation without pivoting of
 *     A[P, Q].
 * The three stages below compute exactly that:
 *   S1  oracle_rpm        -- the RPM, by Algorithm 2 (Section 7) with the
 *                            corrections listed at the function;
 *   S2  oracle_zorder     -- pivot order from the RPM, following the order of
 *                            the four recursive calls of Algorithm 1;
 *   S3  oracle_ordered_lu -- right-looking elimination without pivoting on
 *                            A[P, Q], asserting non-zero pivots and a zero
 *                            trailing block.
 * Further plain references of the building blocks of Section 2 (MM, TRSM)
 * are provided for kernel-level tests.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_NOMEM 5
#define ORC_ERR_SELFCHECK 8

typedef unsigned __int128 u128;

/* ---- field arithmetic (plain, one reduction per operation) ------------- */

static inline uint64_t fadd(uint64_t a, uint64_t b, uint64_t p) { return (a + b) % p; }
static inline uint64_t fsub(uint64_t a, uint64_t b, uint64_t p) { return (a + p - b) % p; }
static inline uint64_t fmul(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)(((u128)a * b) % p); }
/* c - a b mod p for a, b, c in [0, p), p < 2^32: c + p^2 - a b lies in
 * (0, p^2 + p) and is reduced by one `%` (the elimination's update). */
static inline uint64_t fmsub(uint64_t c, uint64_t a, uint64_t b, uint64_t p) { return (c + p * p - a * b) % p; }

/* Inverse by the extended Euclidean algorithm; a must be non-zero mod p. */
uint64_t oracle_inv(uint64_t a, uint64_t p)
{
    int64_t t = 0, newt = 1;
    int64_t r = (int64_t)p, newr = (int64_t)(a % p);
    while (newr != 0) {
        int64_t q = r / newr;
        int64_t tmp = t - q * newt; t = newt; newt = tmp;
        tmp = r - q * newr; r = newr; newr = tmp;
    }
    if (r != 1) return 0; /* not invertible */
    if (t < 0) t += (int64_t)p;
    return (uint64_t)t;
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

uint64_t oracle_mulmod(uint64_t a, uint64_t b, uint64_t p) { return fmul(a, b, p); }
uint64_t oracle_addmod(uint64_t a, uint64_t b, uint64_t p) { return fadd(a, b, p); }
uint64_t oracle_submod(uint64_t a, uint64_t b, uint64_t p) { return fsub(a, b, p); }

/* Rotate x[lo..hi] so that x[hi] moves to position lo and x[lo..hi-1] shift
 * up by one, keeping their order.  This is the reading of the paper's index
 * exchange T_{lo,hi} used throughout (leaves of Algorithm 1, Algorithm 2). */
static void rot_i64(int64_t *x, int64_t lo, int64_t hi)
{
    if (hi <= lo) return;
    int64_t v = x[hi];
    memmove(x + lo + 1, x + lo, (size_t)(hi - lo) * sizeof(int64_t));
    x[lo] = v;
}

/* Rotate whole rows lo..hi of an m x n matrix (row hi moves to row lo). */
static int rot_rows(int64_t *A, int64_t n, int64_t lo, int64_t hi)
{
    if (hi <= lo) return ORC_OK;
    int64_t *tmp = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!tmp) return ORC_ERR_NOMEM;
    memcpy(tmp, A + hi * n, (size_t)n * sizeof(int64_t));
    memmove(A + (lo + 1) * n, A + lo * n, (size_t)((hi - lo) * n) * sizeof(int64_t));
    memcpy(A + lo * n, tmp, (size_t)n * sizeof(int64_t));
    free(tmp);
    return ORC_OK;
}

/* Rotate whole columns lo..hi of an m x n matrix (column hi moves to lo). */
static void rot_cols(int64_t *A, int64_t m, int64_t n, int64_t lo, int64_t hi)
{
    if (hi <= lo) return;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) rot_i64(A + i * n, lo, hi);
}

/*
 * S1: rank profile matrix by Algorithm 2 (Section 7, iterative base case).
 *
 * Algorithm 2 grows a leading i x j sub-matrix along a Z-shaped path: it
 * first looks for a pivot in the new column j among the non-pivot rows
 * r..i-1, then in the new row i among the non-pivot columns r..j-1, then at
 * the corner (i, j); when none exists both dimensions grow by one.  The
 * printed listing is garbled in several places; this follows the reading:
 *   - the window updates are min(i+1, m), min(j+1, n) (printed as max);
 *   - the column window w is A[r..i-1, j] (its last index is misprinted);
 *   - the elimination loops over rows k = p+1..m-1 and the multiplier is
 *     A[k,q] / A[p,q] (printed with n and A[k,p]);
 *   - the pivot row and column are brought to position r by rotating WHOLE
 *     rows r..p and WHOLE columns r..q (the printed partial swaps, and
 *     plain transpositions, reorder non-pivot rows/columns and break the
 *     rank-profile property).
 * Only the rank profile matrix is kept from this stage: rpm_col[i] is the
 * column of the pivot of original row i, or -1.  Returns r, or -1 on
 * allocation failure or a modulus outside [2, 2^32).  A is m x n row-major (ld = n), overwritten.
 */
int64_t oracle_rpm(int64_t m, int64_t n, int64_t *A, uint64_t p, int64_t *rpm_col)
{
    if (p < 2 || p >= ((uint64_t)1 << 32)) return -1;
    int64_t *P = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *Q = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!P || !Q) { free(P); free(Q); return -1; }
    for (int64_t t = 0; t < m; ++t) { P[t] = t; rpm_col[t] = -1; }
    for (int64_t t = 0; t < n; ++t) Q[t] = t;

    int64_t r = 0, i = 0, j = 0;
    while (i < m || j < n) {
        int64_t pr = -1, qc = -1;
        /* w = A[r..i-1, j] */
        if (j < n) {
            for (int64_t t = r; t < i; ++t)
                if (A[t * n + j] != 0) { pr = t; break; }
        }
        if (pr >= 0) {
            qc = j;
            j = j + 1 < n ? j + 1 : n;
        } else {
            /* v = A[i, r..j-1] */
            if (i < m) {
                for (int64_t t = r; t < j; ++t)
                    if (A[i * n + t] != 0) { qc = t; break; }
            }
            if (qc >= 0) {
                pr = i;
                i = i + 1 < m ? i + 1 : m;
            } else if (i < m && j < n && A[i * n + j] != 0) {
                pr = i; qc = j;
                i = i + 1 < m ? i + 1 : m;
                j = j + 1 < n ? j + 1 : n;
            } else {
                i = i + 1 < m ? i + 1 : m;
                j = j + 1 < n ? j + 1 : n;
                continue;
            }
        }
        /* A[pr, qc] is a pivot: eliminate below it. */
        uint64_t inv = oracle_inv((uint64_t)A[pr * n + qc], p);
        const int64_t *prow = A + pr * n;
        #pragma omp parallel for schedule(static)
        for (int64_t k = pr + 1; k < m; ++k) {
            int64_t *rowk = A + k * n;
            uint64_t l = fmul((uint64_t)rowk[qc], inv, p);
            rowk[qc] = (int64_t)l;
            if (l == 0) continue;
            for (int64_t c = qc + 1; c < n; ++c)
                rowk[c] = (int64_t)fmsub((uint64_t)rowk[c], l, (uint64_t)prow[c], p);
        }
        if (rot_rows(A, n, r, pr) != ORC_OK) { free(P); free(Q); return -1; }
        rot_cols(A, m, n, r, qc);
        rot_i64(P, r, pr);
        rot_i64(Q, r, qc);
        r += 1;
    }
    for (int64_t t = 0; t < r; ++t) rpm_col[P[t]] = Q[t];
    free(P); free(Q);
    return r;
}

/*
 * S2: pivot order of Algorithm 1 (Section 2), from the RPM alone.
 *
 * A call of Algorithm 1 on the rows `rows` and columns `cols` (ascending
 * lists of original indices) finds exactly the RPM pairs inside rows x cols.
 * It splits at k = floor(|rows|/2), h = floor(|cols|/2) and returns the
 * pivots of its four recursive calls in the order
 *   PLUQ(A1)  on rows[:k]              x cols[:h]
 *   PLUQ(F)   on rows[:k] - rows(A1)   x cols[h:]
 *   PLUQ(G)   on rows[k:]              x cols[:h] - cols(A1)
 *   PLUQ(R)   on rows[k:] - rows(G)    x cols[h:] - cols(F)
 * which is the order fixed by the block permutations S and T.  A single row
 * or a single column holds at most one pivot (the leaves).
 */
typedef struct { int64_t *pr, *pc; int64_t cnt; } zout;

static int in_sorted(const int64_t *a, int64_t n, int64_t x)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < n && a[lo] == x;
}

/* rows minus the rows listed in (pr[0..cnt)), keeping ascending order */
static int64_t *minus_list(const int64_t *src, int64_t ns, const int64_t *rem, int64_t nrem, int64_t *nout)
{
    int64_t *sorted = (int64_t *)malloc((size_t)(nrem > 0 ? nrem : 1) * sizeof(int64_t));
    int64_t *out = (int64_t *)malloc((size_t)(ns > 0 ? ns : 1) * sizeof(int64_t));
    if (!sorted || !out) { free(sorted); free(out); return NULL; }
    memcpy(sorted, rem, (size_t)nrem * sizeof(int64_t));
    /* insertion sort: the lists are short relative to the cost of S1/S3 */
    for (int64_t a = 1; a < nrem; ++a) {
        int64_t v = sorted[a], b = a - 1;
        while (b >= 0 && sorted[b] > v) { sorted[b + 1] = sorted[b]; --b; }
        sorted[b + 1] = v;
    }
    int64_t c = 0;
    for (int64_t t = 0; t < ns; ++t)
        if (!in_sorted(sorted, nrem, src[t])) out[c++] = src[t];
    free(sorted);
    *nout = c;
    return out;
}

static int zrec(const int64_t *rows, int64_t nr, const int64_t *cols, int64_t nc,
                const int64_t *rpm_col, zout *o)
{
    if (nr == 0 || nc == 0) return ORC_OK;
    int64_t npiv = 0, lastr = -1;
    for (int64_t t = 0; t < nr; ++t) {
        int64_t c = rpm_col[rows[t]];
        if (c >= 0 && in_sorted(cols, nc, c)) { ++npiv; lastr = rows[t]; }
    }
    if (npiv == 0) return ORC_OK;
    if (nr == 1 || nc == 1) {
        /* a single row or column: at most one pivot */
        o->pr[o->cnt] = lastr; o->pc[o->cnt] = rpm_col[lastr]; o->cnt++;
        return ORC_OK;
    }
    int64_t k = nr / 2, h = nc / 2;
    int rc;
    int64_t s1 = o->cnt;
    if ((rc = zrec(rows, k, cols, h, rpm_col, o))) return rc;               /* A1 */
    int64_t e1 = o->cnt;
    int64_t n2r; int64_t *rows2 = minus_list(rows, k, o->pr + s1, e1 - s1, &n2r);
    if (!rows2) return ORC_ERR_NOMEM;
    if ((rc = zrec(rows2, n2r, cols + h, nc - h, rpm_col, o))) { free(rows2); return rc; }  /* F */
    free(rows2);
    int64_t e2 = o->cnt;
    int64_t n3c; int64_t *cols3 = minus_list(cols, h, o->pc + s1, e1 - s1, &n3c);
    if (!cols3) return ORC_ERR_NOMEM;
    if ((rc = zrec(rows + k, nr - k, cols3, n3c, rpm_col, o))) { free(cols3); return rc; }  /* G */
    free(cols3);
    int64_t e3 = o->cnt;
    int64_t n4r; int64_t *rows4 = minus_list(rows + k, nr - k, o->pr + e2, e3 - e2, &n4r);
    int64_t n4c; int64_t *cols4 = minus_list(cols + h, nc - h, o->pc + e1, e2 - e1, &n4c);
    if (!rows4 || !cols4) { free(rows4); free(cols4); return ORC_ERR_NOMEM; }
    rc = zrec(rows4, n4r, cols4, n4c, rpm_col, o);                         /* R */
    free(rows4); free(cols4);
    return rc;
}

/*
 * P, Q from the RPM: pivots in Algorithm 1's order, then the non-pivot rows
 * (columns) in ascending order.  P[i] is the original row of packed row i and
 * Q[j] the original column of packed column j.  Returns r, or -1.
 */
int64_t oracle_zorder(int64_t m, int64_t n, const int64_t *rpm_col, int64_t *P, int64_t *Q)
{
    int64_t *rows = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *cols = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t mn = m < n ? m : n;
    zout o;
    o.pr = (int64_t *)malloc((size_t)(mn > 0 ? mn : 1) * sizeof(int64_t));
    o.pc = (int64_t *)malloc((size_t)(mn > 0 ? mn : 1) * sizeof(int64_t));
    o.cnt = 0;
    char *rowp = (char *)calloc((size_t)(m > 0 ? m : 1), 1);
    char *colp = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t r = -1;
    if (!rows || !cols || !o.pr || !o.pc || !rowp || !colp) goto done;
    for (int64_t t = 0; t < m; ++t) rows[t] = t;
    for (int64_t t = 0; t < n; ++t) cols[t] = t;
    if (zrec(rows, m, cols, n, rpm_col, &o) != ORC_OK) goto done;
    r = o.cnt;
    for (int64_t t = 0; t < r; ++t) {
        P[t] = o.pr[t]; Q[t] = o.pc[t];
        rowp[o.pr[t]] = 1; colp[o.pc[t]] = 1;
    }
    {
        int64_t c = r;
        for (int64_t t = 0; t < m; ++t) if (!rowp[t]) P[c++] = t;
        c = r;
        for (int64_t t = 0; t < n; ++t) if (!colp[t]) Q[c++] = t;
    }
done:
    free(rows); free(cols); free(o.pr); free(o.pc); free(rowp); free(colp);
    return r;
}

/*
 * S3: X = A[P, Q] followed by r steps of right-looking elimination without
 * pivoting (the packed [L\U V; M 0] of the output contract of Algorithm 1).
 * Self-checks: every pivot X[s,s] is non-zero and X[r:, r:] == 0 at the end;
 * a failure returns ORC_ERR_SELFCHECK (it would mean S1 or S2 is wrong).
 * A is m x n (ld n), untouched; X is m x n (ld n), written.
 */
int oracle_ordered_lu(int64_t m, int64_t n, const int64_t *A, uint64_t p, int64_t r,
                      const int64_t *P, const int64_t *Q, int64_t *X)
{
    if (p < 2 || p >= ((uint64_t)1 << 32)) return ORC_ERR_ARG;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            X[i * n + j] = A[P[i] * n + Q[j]];
    for (int64_t s = 0; s < r; ++s) {
        uint64_t piv = (uint64_t)X[s * n + s];
        if (piv == 0) return ORC_ERR_SELFCHECK;
        uint64_t inv = oracle_inv(piv, p);
        const int64_t *urow = X + s * n;
        #pragma omp parallel for schedule(static)
        for (int64_t i = s + 1; i < m; ++i) {
            int64_t *row = X + i * n;
            uint64_t l = fmul((uint64_t)row[s], inv, p);
            row[s] = (int64_t)l;
            if (l == 0) continue;
            for (int64_t j = s + 1; j < n; ++j)
                row[j] = (int64_t)fmsub((uint64_t)row[j], l, (uint64_t)urow[j], p);
        }
    }
    for (int64_t i = r; i < m; ++i)
        for (int64_t j = r; j < n; ++j)
            if (X[i * n + j] != 0) return ORC_ERR_SELFCHECK;
    return ORC_OK;
}

/*
 * Full oracle: A (m x n, ld n, entries in [0,p)) -> P, Q, r and packed X.
 * A is not modified.
 */
int oracle_pluqz(int64_t m, int64_t n, const int64_t *A, uint64_t p,
                 int64_t *P, int64_t *Q, int64_t *X, int64_t *r_out)
{
    if (m < 0 || n < 0 || p < 2 || p >= ((uint64_t)1 << 32)) return ORC_ERR_ARG;
    *r_out = 0;
    for (int64_t t = 0; t < m; ++t) P[t] = t;
    for (int64_t t = 0; t < n; ++t) Q[t] = t;
    if (m == 0 || n == 0) return ORC_OK;
    int64_t *W = (int64_t *)malloc((size_t)m * (size_t)n * sizeof(int64_t));
    int64_t *rpm = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    if (!W || !rpm) { free(W); free(rpm); return ORC_ERR_NOMEM; }
    memcpy(W, A, (size_t)m * (size_t)n * sizeof(int64_t));
    int64_t r1 = oracle_rpm(m, n, W, p, rpm);
    free(W);
    if (r1 < 0) { free(rpm); return ORC_ERR_NOMEM; }
    int64_t r2 = oracle_zorder(m, n, rpm, P, Q);
    free(rpm);
    if (r2 < 0) return ORC_ERR_NOMEM;
    if (r2 != r1) return ORC_ERR_SELFCHECK;
    *r_out = r1;
    return oracle_ordered_lu(m, n, A, p, r1, P, Q, X);
}

/* ---- building blocks of Section 2, for kernel-level tests ------------- */

/* MM(C, A, B): C <- C - A.B mod p.  C m x n (ldc), A m x k (lda), B k x n (ldb). */
void oracle_mm(int64_t m, int64_t n, int64_t k, int64_t *C, int64_t ldc,
               const int64_t *A, int64_t lda, const int64_t *B, int64_t ldb, uint64_t p)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) {
            uint64_t acc = (uint64_t)C[i * ldc + j];
            for (int64_t t = 0; t < k; ++t)
                acc = fsub(acc, fmul((uint64_t)A[i * lda + t], (uint64_t)B[t * ldb + j], p), p);
            C[i * ldc + j] = (int64_t)acc;
        }
}

/* TRSM(L, B): B <- L^{-1} B, L r x r unit lower triangular (strict lower
 * part read from L, diagonal taken as 1), B r x n. */
void oracle_trsm_llu(int64_t r, int64_t n, const int64_t *L, int64_t ldl,
                     int64_t *B, int64_t ldb, uint64_t p)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < r; ++i) {
            uint64_t acc = (uint64_t)B[i * ldb + j];
            for (int64_t t = 0; t < i; ++t)
                acc = fsub(acc, fmul((uint64_t)L[i * ldl + t], (uint64_t)B[t * ldb + j], p), p);
            B[i * ldb + j] = (int64_t)acc;
        }
}

/* TRSM(B, U): B <- B U^{-1}, U r x r upper triangular with non-zero
 * diagonal, B m x r. */
void oracle_trsm_run(int64_t m, int64_t r, int64_t *B, int64_t ldb,
                     const int64_t *U, int64_t ldu, uint64_t p)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < r; ++j) {
            uint64_t acc = (uint64_t)B[i * ldb + j];
            for (int64_t t = 0; t < j; ++t)
                acc = fsub(acc, fmul((uint64_t)B[i * ldb + t], (uint64_t)U[t * ldu + j], p), p);
            B[i * ldb + j] = (int64_t)fmul(acc, oracle_inv((uint64_t)U[j * ldu + j], p), p);
        }
}

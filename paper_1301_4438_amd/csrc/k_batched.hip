// Batched form: many independent PLUQ decompositions (Algorithm 1's output,
// PLUQ-Z order) in one persistent launch, one 256-thread work-group per
// matrix at a time, every decision taken on the device.
//
// Per matrix (m, n <= BATCH_MAX_DIM), in place in its own storage:
//   0. copy A to a backup W in the workspace;
//   1. optimistic elimination without pivoting in the identity order,
//      blocked by KB columns: the panel A[s:m, s:s+KB] is factored in LDS,
//      the U rows right of it are solved with the panel's unit lower
//      triangle, and the trailing block gets one rank-KB update (one read
//      and write of each element per panel).  The identity order is PLUQ-Z
//      exactly when every pivot is non-zero, or when at the first zero pivot
//      (step r) the whole trailing block A[r:m, r:n] is zero: then the rank
//      profile matrix is the leading diagonal of size r;
//   2. otherwise (rare for random inputs): A is restored from W, its rank
//      profile matrix is found by row-order elimination (each row's pivot is
//      its leftmost non-zero entry outside earlier pivot columns: the
//      search of Algorithm 2, Section 7, blocked by KB rows), the pivot
//      order comes from the index-only quadrant recursion of Algorithm 1
//      (Section 2) over the rank profile matrix, the rows and columns of W
//      are gathered into A in that order and the elimination of step 1 runs
//      again with the rank known.
// The matrices are taken largest first (host sorts), work-group w handling
// entries w, w + G, w + 2G, ...  Each rank goes to the descriptor's R slot;
// a failed self-check (a zero pivot before the known rank, a non-zero
// trailing block after it, an overflow of the order's work lists) writes -1.
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

namespace {

constexpr int BT = 256;                    // threads per work-group
constexpr int BMAX = BATCH_MAX_DIM;        // largest m or n
constexpr int ZARENA = 2 * (2 * BMAX) + 256;
constexpr int ZSTACK = 48;
constexpr int INF = 0x7fffffff;

enum { F_ROFF, F_RLEN, F_COFF, F_CLEN, F_STAGE, F_K, F_H, F_OST, F_O1, F_O2, F_O3, F_ATOP, F_N };

template <int KB> struct LuMem {
    int32_t pan[BMAX * KB];    // panel rows s.., KB columns, canonical
    int32_t urow[KB * BMAX];   // solved U rows right of the panel, canonical
};
template <int KB> struct RpmMem {
    int32_t brow[KB * BMAX];   // current block of rows, canonical
    int32_t fsym[BMAX * KB];   // multipliers of the rows below (symmetric)
    int32_t bcol[KB];          // pivot column of the block's q-th pivot
    int32_t brw[KB];           // block row of the q-th pivot
    double binv[KB];           // inverse of the q-th pivot
    int32_t fb[KB];            // multipliers inside the block (symmetric)
};
struct ZMem {
    int32_t rmark[BMAX], cmark[BMAX];
    int32_t outr[BMAX], outc[BMAX];   // pivots in order, then non-pivots
    int32_t arena[ZARENA];
    int32_t fr[ZSTACK][F_N];
    int32_t ctl[8];                   // 0 top, 1 nout, 2 stamp, 3 arena top, 4 error
};
template <int KB> union BigMem {
    LuMem<KB> lu;
    RpmMem<KB> rpm;
    ZMem z;
};

__device__ __forceinline__ double sym(double v, const ModP &m) { return to_sym(v, m); }

// ----------------------------------------------------------------- LU ----

// Copy of an m x n block between two row-major arrays, eight loads in
// flight per thread before the stores.
template <typename T>
__device__ void copy_block(const T *src, int64_t lds, T *dst, int64_t ldd, int m, int n) {
    const int tid = threadIdx.x;
    const int total = m * n;
    for (int e0 = tid; e0 < total; e0 += 8 * BT) {
        T v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = e0 + j * BT;
            if (e < total) v[j] = src[(int64_t)(e / n) * lds + e % n];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = e0 + j * BT;
            if (e < total) dst[(int64_t)(e / n) * ldd + e % n] = v[j];
        }
    }
}

// Elimination without pivoting of the m x n matrix at A (in place), blocked
// by KB columns.  r_known < 0: optimistic, stop at the first zero pivot and
// succeed iff the trailing block is zero there; r_known >= 0: exactly that
// many pivots, all non-zero, and a zero trailing block.  Returns the rank,
// or -1 on failure.
template <typename T, int KB>
__device__ int blocked_lu(T *A, int64_t lda, int m, int n, int r_known, const ModP &mod, LuMem<KB> &L) {
    constexpr int RSTEP = BT / KB;   // panel rows per pass of the work-group
    const int tid = threadIdx.x;
    const int mn = min(m, n);
    const int rmax = r_known >= 0 ? r_known : mn;
    int s = 0;
    for (;;) {
        if (s >= rmax) {
            // all pivots taken; with a known rank below min(m, n) the rest
            // must be zero
            bool nz = false;
            if (s < mn) {
                const int R = m - s, W = n - s;
                for (int e = tid; e < R * W; e += BT) {
                    const int i = e / W, c = e % W;
                    nz |= to_f64(A[(int64_t)(s + i) * lda + s + c]) != 0.0;
                }
            }
            nz = __syncthreads_or(nz);
            return nz ? -1 : s;
        }
        const int kb = min(KB, mn - s);
        const int pr = m - s;
        const int pt = tid % KB, pi0 = tid / KB;
        // panel load: thread (pi0, pt) takes rows pi0, pi0 + RSTEP, ...
        for (int ib = pi0; ib < pr; ib += 8 * RSTEP) {
            double v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = ib + j * RSTEP;
                v[j] = (i < pr && pt < kb) ? to_f64(A[(int64_t)(s + i) * lda + s + pt]) : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int i = ib + j * RSTEP;
                if (i < pr) L.pan[i * KB + pt] = (int32_t)v[j];
            }
        }
        __syncthreads();
        const int tlim = min(kb, rmax - s);
        int kbe = kb;
        for (int t = 0; t < kb; ++t) {
            const double piv = (double)L.pan[t * KB + t];
            if (t >= tlim || piv == 0.0) {   // uniform
                kbe = t;
                break;
            }
            const double inv = inv_fermat(piv, mod);
            for (int i = t + 1 + tid; i < pr; i += BT) {
                const double ls = sym_reduce((double)L.pan[i * KB + t] * inv, mod);
                L.pan[i * KB + t] = (int32_t)(ls < 0.0 ? ls + mod.p : ls);
                for (int u = t + 1; u < kb; ++u) {
                    const double x = sym_reduce(fma(-ls, sym((double)L.pan[t * KB + u], mod), (double)L.pan[i * KB + u]), mod);
                    L.pan[i * KB + u] = (int32_t)(x < 0.0 ? x + mod.p : x);
                }
            }
            __syncthreads();
        }
        // a zero pivot at s + kbe (or the known rank reached inside the
        // panel): the panel's remaining block must be zero
        bool nz = false;
        if (kbe < kb)
            for (int e = tid; e < (pr - kbe) * (kb - kbe); e += BT) {
                const int i = kbe + e / (kb - kbe), u = kbe + e % (kb - kbe);
                nz |= L.pan[i * KB + u] != 0;
            }
        if (pt < kb)
            for (int i = pi0; i < pr; i += RSTEP) A[(int64_t)(s + i) * lda + s + pt] = from_f64<T>((double)L.pan[i * KB + pt]);
        // U rows s .. s+kbe-1 right of the panel: x <- L11^{-1} x per column
        const int c0 = s + kb, W = n - c0;
        for (int c = tid; c < W; c += BT) {
            double xs[KB];
#pragma unroll
            for (int t = 0; t < KB; ++t)
                if (t < kbe) xs[t] = to_f64(A[(int64_t)(s + t) * lda + c0 + c]);
#pragma unroll
            for (int t = 0; t < KB; ++t) {
                if (t < kbe) {
                    double acc = xs[t];
#pragma unroll
                    for (int u = 0; u < t; ++u) acc = fma(-sym((double)L.pan[t * KB + u], mod), xs[u], acc);
                    const double xsym = sym_reduce(acc, mod);
                    L.urow[t * BMAX + c] = (int32_t)(xsym < 0.0 ? xsym + mod.p : xsym);
                    xs[t] = xsym;
                }
            }
#pragma unroll
            for (int t = 0; t < KB; ++t)
                if (t < kbe) A[(int64_t)(s + t) * lda + c0 + c] = from_f64<T>((double)L.urow[t * BMAX + c]);
        }
        __syncthreads();
        // The panel's multipliers below the pivots as symmetric residues,
        // once, for the trailing update (they are already written back).
        for (int e = tid; e < (pr - kbe) * KB; e += BT) {
            const int i = kbe + e / KB;
            L.pan[i * KB + e % KB] = (int32_t)sym((double)L.pan[i * KB + e % KB], mod);
        }
        __syncthreads();
        // trailing update of rows s+kbe .., columns c0 ..: each thread owns a
        // column (its U entries in registers) and a set of rows, eight rows
        // loaded before any is written
        const int R = m - s - kbe;
        if (R > 0 && W > 0) {
            const int tpc = W >= BT ? 1 : BT / W;   // threads per column
            if (tid < (W >= BT ? BT : W * tpc)) {
                const int g = W >= BT ? 0 : tid / W;
                for (int c = (W >= BT ? tid : tid % W); c < W; c += BT) {
                    double u[KB];
#pragma unroll
                    for (int t = 0; t < KB; ++t) u[t] = (t < kbe) ? sym((double)L.urow[t * BMAX + c], mod) : 0.0;
                    for (int ib = g; ib < R; ib += 8 * tpc) {
                        double a[8];
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int i = ib + j * tpc;
                            a[j] = (i < R) ? to_f64(A[(int64_t)(s + kbe + i) * lda + c0 + c]) : 0.0;
                        }
#pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            const int i = ib + j * tpc;
                            if (i < R) {
                                double acc = a[j];
                                const int32_t *lrow = &L.pan[(kbe + i) * KB];
#pragma unroll
                                for (int t = 0; t < KB; ++t)
                                    if (t < kbe) acc = fma(-(double)lrow[t], u[t], acc);
                                double x = sym_reduce(acc, mod);
                                x = x < 0.0 ? x + mod.p : x;   // canonical
                                A[(int64_t)(s + kbe + i) * lda + c0 + c] = from_f64<T>(x);
                                if (kbe < kb) nz |= (x != 0.0);
                            }
                        }
                    }
                }
            }
        }
        nz = __syncthreads_or(nz);
        if (kbe < kb) {
            // stopped inside the panel
            const int r = s + kbe;
            if (r_known >= 0) return (r == r_known && !nz) ? r : -1;
            return nz ? -1 : r;
        }
        s += kb;
    }
}

// -------------------------------------------------------- rank profile ----

// Row-order search of the rank profile matrix, destroying A: rpm[i] = pivot
// column of row i or -1.  Blocks of KB rows: inside a block rows are reduced
// one after the other (pivot = leftmost non-zero entry in a column that is
// not yet a pivot column); the block's pivots are then applied to every row
// below in one pass.  Returns the rank.
template <typename T, int KB>
__device__ int rpm_search(T *A, int64_t lda, int m, int n, const ModP &mod, RpmMem<KB> &R, int32_t *rpm,
                          unsigned char *dead, int32_t *sred) {
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += BT) rpm[i] = -1;
    for (int c = tid; c < n; c += BT) dead[c] = 0;
    int r = 0;
    for (int i0 = 0; i0 < m; i0 += KB) {
        const int kb = min(KB, m - i0);
        __syncthreads();
        for (int e = tid; e < kb * n; e += BT) {
            const int t = e / n, c = e % n;
            R.brow[t * BMAX + c] = (int32_t)to_f64(A[(int64_t)(i0 + t) * lda + c]);
        }
        int q = 0;
        for (int t = 0; t < kb; ++t) {
            if (tid == 0) sred[0] = INF;
            __syncthreads();
            int best = INF;
            for (int c = tid; c < n; c += BT)
                if (!dead[c] && R.brow[t * BMAX + c] != 0) best = min(best, c);
            if (best != INF) atomicMin(&sred[0], best);
            __syncthreads();
            const int jc = sred[0];
            __syncthreads();
            if (jc == INF) continue;   // uniform: row i0+t depends on earlier rows
            const double inv = inv_fermat((double)R.brow[t * BMAX + jc], mod);
            if (tid == 0) {
                rpm[i0 + t] = jc;
                dead[jc] = 1;
                R.bcol[q] = jc;
                R.brw[q] = t;
                R.binv[q] = inv;
            }
            for (int u = t + 1 + tid; u < kb; u += BT)
                R.fb[u] = (int32_t)sym(mod_reduce((double)R.brow[u * BMAX + jc] * inv, mod), mod);
            __syncthreads();
            for (int e = tid; e < (kb - t - 1) * n; e += BT) {
                const int u = t + 1 + e / n, c = e % n;
                if (!dead[c]) {
                    const double x = fma(-(double)R.fb[u], sym((double)R.brow[t * BMAX + c], mod),
                                         (double)R.brow[u * BMAX + c]);
                    R.brow[u * BMAX + c] = (int32_t)mod_reduce(x, mod);
                }
            }
            ++q;
            ++r;
            __syncthreads();
        }
        const int below = m - i0 - kb;
        if (q == 0 || below <= 0) continue;
        // multipliers of each row below for the block's pivots, in order
        for (int ib = tid; ib < below; ib += BT) {
            const int64_t row = (int64_t)(i0 + kb + ib) * lda;
            double a[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k)
                if (k < q) a[k] = to_f64(A[row + R.bcol[k]]);
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                if (k < q) {
                    const double f = sym(mod_reduce(mod_reduce(a[k], mod) * R.binv[k], mod), mod);
                    R.fsym[ib * KB + k] = (int32_t)f;
#pragma unroll
                    for (int k2 = k + 1; k2 < KB; ++k2)
                        if (k2 < q)
                            a[k2] = mod_reduce(
                                fma(-f, sym((double)R.brow[R.brw[k] * BMAX + R.bcol[k2]], mod), a[k2]), mod);
                }
            }
        }
        __syncthreads();
        for (int e = tid; e < below * n; e += BT) {
            const int ib = e / n, c = e % n;
            if (dead[c]) continue;
            T *a = &A[(int64_t)(i0 + kb + ib) * lda + c];
            double acc = to_f64(*a);
#pragma unroll
            for (int k = 0; k < KB; ++k)
                if (k < q) acc = fma(-(double)R.fsym[ib * KB + k], sym((double)R.brow[R.brw[k] * BMAX + c], mod), acc);
            *a = from_f64<T>(mod_reduce(acc, mod));
        }
    }
    __syncthreads();
    return r;
}

// ------------------------------------------------------------ Z order ----

// Stream compaction over the whole work-group: dst <- [v in src[0:len) :
// keep(v)], order kept.  Returns the count (uniform).
template <class P>
__device__ int blk_filter(const int32_t *src, int len, int32_t *dst, P keep, int32_t *wcnt) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    int cnt = 0;
    for (int base = 0; base < len; base += BT) {
        const int idx = base + tid;
        const int32_t v = idx < len ? src[idx] : 0;
        const bool k = idx < len && keep(v);
        const uint64_t mask = __ballot(k);
        const int pos = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[wv] = __popcll(mask);
        __syncthreads();
        int off = cnt, tot = 0;
#pragma unroll
        for (int w = 0; w < BT / 64; ++w) {
            if (w < wv) off += wcnt[w];
            tot += wcnt[w];
        }
        if (k) dst[off + pos] = v;
        cnt += tot;
        __syncthreads();
    }
    return cnt;
}

// Pivot order of Algorithm 1 from the rank profile matrix (rpm[i] = pivot
// column of row i or -1): Z(rows, cols) = Z(A1) ++ Z(F) ++ Z(G) ++ Z(R) with
// the floor(|rows|/2) x floor(|cols|/2) split, F on the first rows minus
// those of Z(A1), G on the first columns minus those of Z(A1), R on the
// remaining rows minus those of Z(G) and columns minus those of Z(F).  A
// block with one row or one column holds at most one pivot.  Run by the
// whole work-group with an explicit stack.  On return z.outr / z.outc hold
// P and Q (pivots first, then non-pivot rows / columns ascending); returns
// the number of pivots, or -1 if the stack or the list arena overflowed.
__device__ int zorder(int m, int n, const int32_t *rpm, ZMem &z, int32_t *wcnt) {
    const int tid = threadIdx.x;
    for (int i = tid; i < m; i += BT) {
        z.arena[i] = i;
        z.rmark[i] = 0;
    }
    for (int j = tid; j < n; j += BT) {
        z.arena[m + j] = j;
        z.cmark[j] = 0;
    }
    if (tid == 0) {
        int *F = z.fr[0];
        F[F_ROFF] = 0; F[F_RLEN] = m; F[F_COFF] = m; F[F_CLEN] = n; F[F_STAGE] = 0;
        z.ctl[0] = 1; z.ctl[1] = 0; z.ctl[2] = 0; z.ctl[3] = m + n; z.ctl[4] = 0;
    }
    __syncthreads();
    for (;;) {
        const int top = z.ctl[0];
        if (top == 0 || z.ctl[4]) break;
        int *F = z.fr[top - 1];
        const int stage = F[F_STAGE];
        const int roff = F[F_ROFF], rlen = F[F_RLEN], coff = F[F_COFF], clen = F[F_CLEN];
        const int kk = F[F_K], hh = F[F_H];
        const int nout = z.ctl[1], stamp = z.ctl[2], atop = z.ctl[3];
        const int32_t *rows = z.arena + roff, *cols = z.arena + coff;
        __syncthreads();   // every thread has read the frame and the controls
        auto push = [&](int ro, int rl, int co, int cl) {
            if (top >= ZSTACK) {
                z.ctl[4] = 1;
                return;
            }
            int *C = z.fr[top];
            C[F_ROFF] = ro; C[F_RLEN] = rl; C[F_COFF] = co; C[F_CLEN] = cl; C[F_STAGE] = 0;
            z.ctl[0] = top + 1;
        };
        if (stage == 0) {
            bool leaf = (rlen == 0 || clen == 0);
            int cnt = 0;
            if (!leaf) {
                const int st = stamp + 1;
                for (int j = tid; j < clen; j += BT) z.cmark[cols[j]] = st;
                __syncthreads();
                bool has = false;
                for (int i = tid; i < rlen; i += BT) {
                    const int c = rpm[rows[i]];
                    if (c >= 0 && z.cmark[c] == st) {
                        has = true;
                        if (rlen == 1 || clen == 1) {   // the block's single pivot
                            z.outr[nout] = rows[i];
                            z.outc[nout] = c;
                        }
                    }
                }
                cnt = __syncthreads_count(has);
                if (tid == 0) z.ctl[2] = st;
                leaf = (cnt == 0 || rlen == 1 || clen == 1);
            }
            if (tid == 0) {
                if (leaf) {
                    if (cnt > 0) z.ctl[1] = nout + 1;
                    z.ctl[0] = top - 1;
                } else {
                    F[F_K] = rlen / 2;
                    F[F_H] = clen / 2;
                    F[F_OST] = nout;
                    F[F_STAGE] = 1;
                    F[F_ATOP] = atop;
                    push(roff, rlen / 2, coff, clen / 2);   // A1: prefix views
                }
            }
        } else if (stage == 1) {
            // F: rows[:k] without the rows of Z(A1), columns[h:]
            const int st = stamp + 1;
            const bool fits = atop + kk <= ZARENA;
            for (int q = F[F_OST] + tid; q < nout; q += BT) z.rmark[z.outr[q]] = st;
            __syncthreads();
            const int cnt =
                fits ? blk_filter(rows, kk, z.arena + atop, [&](int v) { return z.rmark[v] != st; }, wcnt) : 0;
            if (tid == 0) {
                z.ctl[2] = st;
                F[F_O1] = nout;
                F[F_STAGE] = 2;
                if (!fits) z.ctl[4] = 1;
                z.ctl[3] = atop + cnt;
                push(atop, cnt, coff + hh, clen - hh);
            }
        } else if (stage == 2) {
            // G: rows[k:], columns[:h] without the columns of Z(A1)
            const int base = F[F_ATOP];
            const int st = stamp + 1;
            const bool fits = base + hh <= ZARENA;
            for (int q = F[F_OST] + tid; q < F[F_O1]; q += BT) z.cmark[z.outc[q]] = st;
            __syncthreads();
            const int cnt =
                fits ? blk_filter(cols, hh, z.arena + base, [&](int v) { return z.cmark[v] != st; }, wcnt) : 0;
            if (tid == 0) {
                z.ctl[2] = st;
                F[F_O2] = nout;
                F[F_STAGE] = 3;
                if (!fits) z.ctl[4] = 1;
                z.ctl[3] = base + cnt;
                push(roff + kk, rlen - kk, base, cnt);
            }
        } else if (stage == 3) {
            // R: rows[k:] without the rows of Z(G), columns[h:] without the
            // columns of Z(F)
            const int base = F[F_ATOP];
            const int st1 = stamp + 1, st2 = stamp + 2;
            const bool fits = base + (rlen - kk) + (clen - hh) <= ZARENA;
            for (int q = F[F_O2] + tid; q < nout; q += BT) z.rmark[z.outr[q]] = st1;
            for (int q = F[F_O1] + tid; q < F[F_O2]; q += BT) z.cmark[z.outc[q]] = st2;
            __syncthreads();
            int cr = 0, cc = 0;
            if (fits) {
                cr = blk_filter(rows + kk, rlen - kk, z.arena + base, [&](int v) { return z.rmark[v] != st1; }, wcnt);
                cc = blk_filter(cols + hh, clen - hh, z.arena + base + cr,
                                [&](int v) { return z.cmark[v] != st2; }, wcnt);
            }
            if (tid == 0) {
                z.ctl[2] = st2;
                F[F_O3] = nout;
                F[F_STAGE] = 4;
                if (!fits) z.ctl[4] = 1;
                z.ctl[3] = base + cr + cc;
                push(base, cr, base + cr, cc);
            }
        } else {
            if (tid == 0) {
                z.ctl[3] = F[F_ATOP];
                z.ctl[0] = top - 1;
            }
        }
        __syncthreads();
    }
    const int r = z.ctl[1];
    const bool err = z.ctl[4] != 0;
    __syncthreads();
    if (err) return -1;
    // non-pivot rows and columns, ascending, after the pivots
    const int st = z.ctl[2] + 1;
    for (int q = tid; q < r; q += BT) {
        z.rmark[z.outr[q]] = st;
        z.cmark[z.outc[q]] = st;
    }
    __syncthreads();
    // the root lists at the arena's start are still 0..m-1 and 0..n-1
    blk_filter(z.arena, m, z.outr + r, [&](int v) { return z.rmark[v] != st; }, wcnt);
    blk_filter(z.arena + m, n, z.outc + r, [&](int v) { return z.cmark[v] != st; }, wcnt);
    return r;
}

// ------------------------------------------------------------- kernel ----

template <typename T, int KB>
__global__ __launch_bounds__(BT, KB == 8 ? 4 : 1) void batched_pluq_kernel(const BatchDesc *desc, int32_t batch, char *wbase,
                                                         ModP mod) {
    __shared__ BigMem<KB> big;
    __shared__ int32_t rpm[BMAX];
    __shared__ unsigned char dead[BMAX];
    __shared__ int32_t sred[8];
    const int tid = threadIdx.x;
    for (int b = blockIdx.x; b < batch; b += gridDim.x) {
        const BatchDesc d = desc[b];
        const int m = d.m, n = d.n;
        T *A = (T *)d.A;
        T *W = (T *)(wbase + d.woff);
        int r = 0;
        if (m > 0 && n > 0) {
            copy_block(A, d.lda, W, (int64_t)n, m, n);
            __syncthreads();
            r = blocked_lu<T, KB>(A, d.lda, m, n, -1, mod, big.lu);
            if (r >= 0) {
                for (int i = tid; i < m; i += BT) d.P[i] = i;
                for (int j = tid; j < n; j += BT) d.Q[j] = j;
            } else {
                copy_block((const T *)W, (int64_t)n, A, d.lda, m, n);
                __syncthreads();
                const int r1 = rpm_search<T, KB>(A, d.lda, m, n, mod, big.rpm, rpm, dead, sred);
                const int rz = zorder(m, n, rpm, big.z, sred);
                if (rz >= 0 && rz == r1) {
                    for (int i = tid; i < m; i += BT) d.P[i] = big.z.outr[i];
                    for (int j = tid; j < n; j += BT) d.Q[j] = big.z.outc[j];
                    for (int e = tid; e < m * n; e += BT) {
                        const int i = e / n, j = e % n;
                        A[(int64_t)i * d.lda + j] = W[(int64_t)big.z.outr[i] * n + big.z.outc[j]];
                    }
                    __syncthreads();
                    r = blocked_lu<T, KB>(A, d.lda, m, n, r1, mod, big.lu);
                } else {
                    r = -1;
                }
            }
        } else {
            for (int i = tid; i < m; i += BT) d.P[i] = i;
            for (int j = tid; j < n; j += BT) d.Q[j] = j;
        }
        if (tid == 0) *d.R = r;
        __syncthreads();
    }
}

template <typename T, int KB>
hipError_t launch_kb(const BatchDesc *desc, int32_t batch, char *wbase, double p, int grid, hipStream_t st) {
    ModP mod;
    mod.p = p;
    mod.pinv = 1.0 / p;
    mod.half = (double)((int64_t)p / 2);
    PLUQ_LAUNCH((batched_pluq_kernel<T, KB>), dim3(grid), dim3(BT), 0, st, desc, batch, wbase, mod);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_t(int kb, const BatchDesc *desc, int32_t batch, char *wbase, double p, int grid,
                    hipStream_t st) {
    switch (kb) {
    case 8: return launch_kb<T, 8>(desc, batch, wbase, p, grid, st);
    case 16: return launch_kb<T, 16>(desc, batch, wbase, p, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batched_pluq(int dtype, int kb, const BatchDesc *desc, int32_t batch, char *wbase, double p,
                               int grid, hipStream_t st) {
    if (batch <= 0) return hipSuccess;
    if (grid <= 0) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return launch_t<int64_t>(kb, desc, batch, wbase, p, grid, st);
    case DT_F64: return launch_t<double>(kb, desc, batch, wbase, p, grid, st);
    case DT_I32: return launch_t<int32_t>(kb, desc, batch, wbase, p, grid, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace pluq

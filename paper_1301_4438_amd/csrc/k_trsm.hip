// Triangular solves of Section 2, TRSM(L, B) and TRSM(B, U): the host driver
// splits a solve recursively at multiples of 64 into half-size solves and
// one MM update each (k_modmm.hip).  This file holds the two kernels the
// solves need besides MM:
//   * the inverses of all 64 x 64 diagonal blocks of the triangle, computed
//     in one launch before the recursion starts (stored as I - T_qq^{-1});
//   * the leaf solve of order r <= 256 in one launch: each work-group owns a
//     strip of 16 right-hand sides and runs the block forward substitution
//     X_q = T_qq^{-1} (B_q - sum_{j<q} T_qj X_j) over the 64-row blocks on
//     the float64 matrix cores, keeping its solved strip in LDS.
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

// Inverses of the 64 x 64 diagonal blocks of an r x r triangle, one
// work-group of 256 threads per block, written as W = I - T_qq^{-1}
// (canonical, row-major, 64 x 64 per block; rows and columns past the
// triangle's order behave as the identity).  An upper block is inverted
// through its transpose, (U^T)^{-1} = (U^{-1})^T, so both sides run the same
// lower-triangular scheme on X = L^{-1} split into 4 x 4 blocks of 16:
//   the four diagonal blocks D_k = L_kk^{-1} by forward substitution (one
//   wave each, a lane per column, the diagonal inverses computed first);
//   then the blocks below, by distance d = i - j = 1, 2, 3, one wave per
//   block of a distance on the float64 matrix cores:
//   T = sum_{k=j}^{i-1} L_ik X_kj,  X_ij = -D_i T.
// Products are of symmetric residues, reduced (symmetric reduction) after
// every 16 terms.
struct DiagSmem {
    double Ls[64][65];   // strict lower part (symmetric residues)
    double Xs[64][65];   // the inverse being built (symmetric)
    double dinv[64];
};

// Work-group body for diagonal block `blk`; the LDS comes from the caller so
// that one kernel can hold the lower and the upper case.
template <typename T, bool UPPER>
__device__ __forceinline__ void diag_inv_body(const T *Tm, int64_t ldt, int r, T *W, ModP mod, int blk,
                                              DiagSmem &sm) {
    auto &Ls = sm.Ls;
    auto &Xs = sm.Xs;
    auto &dinv = sm.dinv;
    const int tid = threadIdx.x;
    const int o = blk * 64;
    const int nb = min(64, r - o);
    const T *Tq = Tm + (int64_t)o * ldt + o;
    {
        // clamped addresses, so the 16 loads go out together
        T raw[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + 256 * q, a = e >> 6, b = e & 63;
            raw[q] = Tq[(int64_t)min(a, nb - 1) * ldt + min(b, nb - 1)];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + 256 * q, a = e >> 6, b = e & 63;
            const double v = (a < nb && b < nb) ? to_f64(raw[q]) : 0.0;
            // stored entry (a, b); the lower operand is L (UPPER: U^T)
            const int i = UPPER ? b : a, j = UPPER ? a : b;
            if (i > j) Ls[i][j] = to_sym(v, mod);
            else if (i < j) Ls[i][j] = 0.0;
            else dinv[i] = (!UPPER || a >= nb) ? 1.0 : v;
            Xs[a][b] = 0.0;
        }
    }
    __syncthreads();
    if (UPPER && tid < 64) dinv[tid] = inv_fermat(dinv[tid], mod);
    __syncthreads();
    const int lane = tid & 63, wv = tid >> 6;
    if (lane < 16) {
        const int base = 16 * wv, c = lane;
        const double di = 1.0;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            // two partial sums halve the dependent chain
            double s0 = (i == c) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
            for (int k = 0; k < i; k += 2) {
                s0 = fma(-Ls[base + i][base + k], x[k], s0);
                if (k + 1 < i) s1 = fma(-Ls[base + i][base + k + 1], x[k + 1], s1);
            }
            const double s = sym_reduce(s0 + s1, mod);
            x[i] = UPPER ? sym_reduce(s * dinv[base + i], mod) : s * di;
            Xs[base + i][base + c] = x[i];
        }
    }
    __syncthreads();
    // Off-diagonal 16 x 16 blocks by distance d = i - j: wave w computes the
    // block (w + d, w) when w < 4 - d, on the float64 matrix cores
    // (v_mfma_f64_16x16x4f64: A operand row lane % 16, inner index
    // lane / 16 + 4 kk; B operand inner index lane / 16 + 4 kk, column
    // lane % 16; accumulator element v at row lane / 16 + 4 v, column
    // lane % 16).  T = sum_k L_ik X_kj takes four products per k block (16
    // terms below 2^52, reduced per block); X_ij = -D_i T then takes T's
    // accumulator elements directly as its B operand (element kk holds rows
    // 4 kk + lane / 16, the rows step kk needs).
    {
        typedef double v4d __attribute__((ext_vector_type(4)));
        const int r16 = lane & 15, k4 = lane >> 4;
#pragma unroll
        for (int d = 1; d < 4; ++d) {
            if (wv < 4 - d) {
                const int j = wv, i = wv + d;
                v4d acc = {0.0, 0.0, 0.0, 0.0};
                for (int k = j; k < i; ++k) {
                    v4d part = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
                        part = __builtin_amdgcn_mfma_f64_16x16x4f64(Ls[16 * i + r16][16 * k + 4 * kk + k4],
                                                                     Xs[16 * k + 4 * kk + k4][16 * j + r16], part, 0,
                                                                     0, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[v] += sym_reduce(part[v], mod);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] = sym_reduce(acc[v], mod);
                v4d x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int kk = 0; kk < 4; ++kk)
                    x = __builtin_amdgcn_mfma_f64_16x16x4f64(Xs[16 * i + r16][16 * i + 4 * kk + k4], acc[kk], x, 0, 0,
                                                             0);
#pragma unroll
                for (int v = 0; v < 4; ++v) Xs[16 * i + k4 + 4 * v][16 * j + r16] = sym_reduce(-x[v], mod);
            }
            __syncthreads();
        }
    }
    T *Wq = W + (int64_t)blk * 64 * 64;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q, i = e >> 6, j = e & 63;
        const double x = UPPER ? Xs[j][i] : Xs[i][j];
        Wq[e] = from_f64<T>(mod_reduce((i == j ? 1.0 : 0.0) - x, mod));
    }
}

template <typename T, bool UPPER>
__global__ __launch_bounds__(256) void trsm_diag_inv_kernel(const T *Tm, int64_t ldt, int r, T *W, ModP mod) {
    __shared__ DiagSmem sm;
    diag_inv_body<T, UPPER>(Tm, ldt, r, W, mod, blockIdx.x, sm);
}

// The diagonal blocks of a lower and an upper triangle of the same order in
// one launch (the two solves of a recursion node): work-groups [0, nb) take
// the lower one, [nb, 2 nb) the upper one.
template <typename T>
__global__ __launch_bounds__(256) void trsm_diag_inv_pair_kernel(const T *Lm, int64_t ldl, const T *Um, int64_t ldu,
                                                                 int r, T *WL, T *WU, ModP mod, int nb) {
    __shared__ DiagSmem sm;
    if ((int)blockIdx.x < nb) diag_inv_body<T, false>(Lm, ldl, r, WL, mod, blockIdx.x, sm);
    else diag_inv_body<T, true>(Um, ldu, r, WU, mod, blockIdx.x - nb, sm);
}

// Leaf solve of order r <= TRSM_FUSE_MAX.  The lower case solves L X = B
// (L unit lower r x r, B r x nst, right-hand sides = columns); the upper case
// solves X U = B (B nst x r), i.e. U^T X^T = B^T, so both run as the lower
// system L' X' = B' with
//   lower: L'(i, k) = T(i, k),  B'(i, c) = B(i, c),  W'_q(i, k) = W_q(i, k);
//   upper: L'(i, k) = T(k, i),  B'(i, c) = B(c, i),  W'_q(i, k) = W_q(k, i)
// (W_q = I - T_qq^{-1} from the diagonal-inverse kernel).  Work-group g owns
// right-hand sides [16 g, 16 g + 16); wave w owns rows [16 w, 16 w + 16) of
// each 64-row block and one 16 x 16 matrix-core tile.  For block q:
//   acc = B'_q - sum_{j<q} L'_qj X_j,    X_q = acc - W'_q acc,
// written back to B and kept in LDS (symmetric residues) for later blocks.
// The 64 x 64 operand blocks (L'_qj, then W'_q) form one sequence of jobs:
// each is read from memory with whole-row loads (coalesced in both
// orientations), converted once to negated symmetric residues and stored in
// one of two LDS buffers; the loads of the job after next are issued before
// the current job's matrix-core operations, so memory latency hides behind
// two jobs.  One
// barrier per job: a buffer is rewritten two jobs after it was read, and
// every thread has passed the previous job's barrier by then.  Four
// accumulators take turns, so consecutive matrix-core operations are
// independent.  Exactness: the accumulators' sum is reduced once per kchunk
// products, at fixed points (between jobs when kchunk >= 64; after every 16
// products when RED16, p above about 2^23.5), never behind a run-time test
// between matrix-core operations.  Rows past r contribute zeros (W' is zero
// there), right-hand sides past nst are computed on zeros and not stored.
// A work-group solves a strip of 16 NT right-hand sides: each wave owns NT
// 16 x 16 matrix-core tiles of each 64-row block, which share every operand
// block loaded (NT = 2 when that still gives enough work-groups).
template <int NT>
struct LeafSmem {
    static constexpr int S = 16 * NT;   // right-hand sides of the strip
    double Xs[TRSM_FUSE_MAX][S + 1];    // solved strip (symmetric)
    double Acc[64][S + 1];              // B'_q - sum L' X (symmetric)
    double Ls[2][64][65];               // operand blocks (negated symmetric)
};
// work-groups for nst right-hand sides at NT tiles per wave
static inline int leaf_groups(int64_t nst, int nt) { return (int)cdiv64(nst, 16 * nt); }
// NT = 2 when strips of 32 still give at least this many work-groups
constexpr int LEAF_WIDE_MIN_GROUPS = 256;

// Work-group body for strip `blk`; the LDS comes from the caller.
template <typename T, bool UPPER, bool RED16, int NT>
__device__ __forceinline__ void trsm_leaf_body(const T *Tm, int64_t ldt, int r, T *B, int64_t ldb, int nst,
                                               const T *W, ModP mod, int kchunk, int blk, LeafSmem<NT> &sm) {
    typedef double v4d __attribute__((ext_vector_type(4)));
    constexpr int S = LeafSmem<NT>::S;
    auto &Xs = sm.Xs;
    auto &Acc = sm.Acc;
    auto &Ls = sm.Ls;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int c0 = blk * S;
    const int col = lane & 15;                 // right-hand side within a 16-wide tile
    const int kl = lane >> 4;                  // k offset of this lane's operand
    const int nb = (r + 63) / 64;
    bool cval[NT];
    int ccl[NT];                               // clamped right-hand sides (loads stay in range)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        cval[t] = c0 + 16 * t + col < nst;
        ccl[t] = cval[t] ? c0 + 16 * t + col : nst - 1;
    }

    // Job (q, j), j <= q: j < q is L'_qj, j == q is W'_q.  Thread tid moves
    // elements e = tid + 256 m, m < 16, of the 64 x 64 block: memory row
    // e / 64, memory column e % 64 (a whole 512-byte row per wave and load).
    // Job (q, j), j <= q: j < q is L'_qj, j == q is W'_q.  Thread tid moves
    // elements e = tid + 256 m, m < 16, of the 64 x 64 block: memory row
    // tid / 64 + 4 m, memory column tid % 64 (a whole 512-byte row per wave
    // and load); consecutive m are 4 memory rows apart.
    const int mr0 = tid >> 6, mc = tid & 63;
    auto load_job = [&](int q, int j, T *dst) {
        if (j == q) {
            const T *src = W + (int64_t)q * 4096 + tid;
#pragma unroll
            for (int m = 0; m < 16; ++m) dst[m] = src[256 * m];
        } else if (UPPER) {
            // T(64 j + mr, min(64 q + mc, r - 1)) = L'(64 q + mc, 64 j + mr)
            const int64_t step = 4 * ldt;
            const T *src = Tm + (int64_t)(64 * j + mr0) * ldt + min(64 * q + mc, r - 1);
#pragma unroll
            for (int m = 0; m < 16; ++m) dst[m] = src[m * step];
        } else {
            // L'(min(64 q + mr, r - 1), 64 j + mc): rows past r re-read row r - 1
            const int64_t step = 4 * ldt;
            const T *src = Tm + (int64_t)(64 * q + mr0) * ldt + 64 * j + mc;
            const T *last = Tm + (int64_t)(r - 1) * ldt + 64 * j + mc;
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                const T *ptr = (64 * q + mr0 + 4 * m < r) ? src + m * step : last;   // select the address
                dst[m] = *ptr;
            }
        }
    };
    auto store_job = [&](int q, int j, int buf, const T *pre) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int mr = mr0 + 4 * m;
            // operand entry (i, k) within the block; rows past r are zero
            const int i = UPPER ? mc : mr, k = UPPER ? mr : mc;
            const bool ok = (j == q) || (64 * q + i < r);
            Ls[buf][i][k] = ok ? -to_sym(to_f64(pre[m]), mod) : 0.0;
        }
    };
    auto reduce4 = [&](v4d *x) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            x[0][v] = mod_reduce((x[0][v] + x[1][v]) + (x[2][v] + x[3][v]), mod);
            x[1][v] = 0.0;
            x[2][v] = 0.0;
            x[3][v] = 0.0;
        }
    };
    // one 64-deep product: A operand from Ls[buf] (shared by the NT tiles),
    // B operands from rows [kb, kb + 64) of the LDS array bs
    auto mfma_job = [&](int buf, const double (*bs)[S + 1], int kb, v4d (*x)[4]) {
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const double av = Ls[buf][16 * wv + col][4 * ks + kl];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const double bv = bs[kb + 4 * ks + kl][16 * t + col];
                x[t][ks & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, x[t][ks & 3], 0, 0, 0);
                if (RED16 && (ks & 3) == 3) reduce4(x[t]);
            }
        }
    };

    T bq[NT][4];
    auto load_b = [&](int q) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 64 * q + 16 * wv + kl + 4 * v, ic = i < r ? i : r - 1;
                bq[t][v] = UPPER ? B[(int64_t)ccl[t] * ldb + ic] : B[(int64_t)ic * ldb + ccl[t]];
            }
    };
    // Jobs run as one flat sequence (q, j) = (0, 0), (1, 0), (1, 1), (2, 0),
    // ...; three register sets rotate (the loop is unrolled by three), so the
    // loads of job n + 2 are issued before job n is stored and have two whole
    // jobs' time to arrive (one job is shorter than a load from memory).
    T ra[16], rb[16], rc[16];
    v4d x[NT][4];
    int buf = 0, kacc = 0;
    auto do_job = [&](int q, int j, T (&cur)[16], T (&nxt)[16], int q2, int j2) {
        const int i0 = 64 * q;
        if (j == 0) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * wv + kl + 4 * v;
                    x[t][0][v] = (i < r && cval[t]) ? to_f64(bq[t][v]) : 0.0;
                    x[t][1][v] = 0.0;
                    x[t][2][v] = 0.0;
                    x[t][3][v] = 0.0;
                }
            if (q + 1 < nb) load_b(q + 1);
            kacc = 0;
        }
        if (q2 < nb) load_job(q2, j2, nxt);
        store_job(q, j, buf, cur);
        if (j == q) {
            // acc = B'_q - sum L' X, reduced: the W job's right operand
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                reduce4(x[t]);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double sv = to_sym(x[t][0][v], mod);
                    x[t][0][v] = sv;
                    Acc[16 * wv + kl + 4 * v][16 * t + col] = sv;
                }
            }
            kacc = 0;
        }
        __syncthreads();
        if (!RED16 && kacc + 64 > kchunk) {
#pragma unroll
            for (int t = 0; t < NT; ++t) reduce4(x[t]);
            kacc = 0;
        }
        if (j < q) mfma_job(buf, Xs, 64 * j, x);
        else mfma_job(buf, Acc, 0, x);
        kacc += 64;
        buf ^= 1;
        if (j == q) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                reduce4(x[t]);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + 16 * wv + kl + 4 * v;   // < 64 nb <= TRSM_FUSE_MAX
                    const double y = x[t][0][v];
                    const int c = 16 * t + col;
                    Xs[i][c] = (i < r) ? to_sym(y, mod) : 0.0;
                    if (i < r && cval[t]) {
                        if (UPPER) B[(int64_t)(c0 + c) * ldb + i] = from_f64<T>(y);
                        else B[(int64_t)i * ldb + c0 + c] = from_f64<T>(y);
                    }
                }
            }
        }
    };
    auto next = [](int &q, int &j) {
        if (j < q) ++j;
        else { ++q; j = 0; }
    };
    // jobs n, n + 1 and n + 2 (the one whose loads job n issues)
    int q = 0, j = 0, q1 = 0, j1 = 0;
    next(q1, j1);
    int q2 = q1, j2 = j1;
    next(q2, j2);
    load_b(0);
    load_job(0, 0, ra);
    if (q1 < nb) load_job(q1, j1, rb);
    auto shift = [&]() {
        q = q1; j = j1;
        q1 = q2; j1 = j2;
        next(q2, j2);
    };
    while (q < nb) {
        do_job(q, j, ra, rc, q2, j2);
        shift();
        if (q >= nb) break;
        do_job(q, j, rb, ra, q2, j2);
        shift();
        if (q >= nb) break;
        do_job(q, j, rc, rb, q2, j2);
        shift();
    }
}

template <typename T, bool UPPER, bool RED16, int NT>
__global__ __launch_bounds__(256) void trsm_leaf_kernel(const T *Tm, int64_t ldt, int r, T *B, int64_t ldb,
                                                        int nst, const T *W, ModP mod, int kchunk) {
    __shared__ LeafSmem<NT> sm;
    trsm_leaf_body<T, UPPER, RED16, NT>(Tm, ldt, r, B, ldb, nst, W, mod, kchunk, blockIdx.x, sm);
}

// The two leaf solves of a recursion node in one launch, L X = BD (lower,
// ncols right-hand sides) and X U = BE (upper, nrows right-hand sides), with
// triangles of the same order: work-groups [0, gD) take strips of BD, the
// rest strips of BE.
template <typename T, bool RED16, int NT>
__global__ __launch_bounds__(256) void trsm_leaf_pair_kernel(const T *Lm, int64_t ldl, const T *Um, int64_t ldu, int r,
                                                             T *BD, int64_t ldbd, int ncols, T *BE, int64_t ldbe,
                                                             int nrows, const T *WL, const T *WU, ModP mod, int kchunk,
                                                             int gD) {
    __shared__ LeafSmem<NT> sm;
    if ((int)blockIdx.x < gD)
        trsm_leaf_body<T, false, RED16, NT>(Lm, ldl, r, BD, ldbd, ncols, WL, mod, kchunk, blockIdx.x, sm);
    else
        trsm_leaf_body<T, true, RED16, NT>(Um, ldu, r, BE, ldbe, nrows, WU, mod, kchunk, blockIdx.x - gD, sm);
}

static ModP make_mod(double p) {
    ModP m;
    m.p = p;
    m.pinv = 1.0 / p;
    m.half = (double)((int64_t)p / 2);
    return m;
}

template <typename T>
static hipError_t diag_inv_t(int side, const void *Tm, int64_t ldt, int r, void *W, double p, hipStream_t st) {
    const dim3 grid((unsigned)cdiv64(r, 64));
    const ModP md = make_mod(p);
    if (side == 0)
        PLUQ_LAUNCH((trsm_diag_inv_kernel<T, false>), grid, dim3(256), 0, st, (const T *)Tm, ldt, r, (T *)W, md);
    else
        PLUQ_LAUNCH((trsm_diag_inv_kernel<T, true>), grid, dim3(256), 0, st, (const T *)Tm, ldt, r, (T *)W, md);
    return hipGetLastError();
}

hipError_t launch_trsm_diag_inv(int dtype, int side, const void *Tm, int64_t ldt, int64_t r, void *W, double p,
                                int kchunk, hipStream_t st) {
    if (r <= 0) return hipSuccess;
    if (kchunk < 1 || r > INT32_MAX) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return diag_inv_t<int64_t>(side, Tm, ldt, (int)r, W, p, st);
    case DT_F64: return diag_inv_t<double>(side, Tm, ldt, (int)r, W, p, st);
    case DT_I32: return diag_inv_t<int32_t>(side, Tm, ldt, (int)r, W, p, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t leaf_t(int side, const void *Tm, int64_t ldt, int r, void *B, int64_t ldb, int nst,
                         const void *W, double p, int kchunk, hipStream_t st) {
    const int nt = leaf_groups(nst, 2) >= LEAF_WIDE_MIN_GROUPS ? 2 : 1;
    const dim3 grid((unsigned)leaf_groups(nst, nt));
    const ModP md = make_mod(p);
#define PLUQ_LEAF(U, R16, NT)                                                                              \
    PLUQ_LAUNCH((trsm_leaf_kernel<T, U, R16, NT>), grid, dim3(256), 0, st, (const T *)Tm, ldt, r, (T *)B, ldb, nst, \
                (const T *)W, md, kchunk)
#define PLUQ_LEAF_NT(U, R16) \
    if (nt == 2) PLUQ_LEAF(U, R16, 2); else PLUQ_LEAF(U, R16, 1);
    const bool r16 = kchunk < 64;
    if (side == 0) {
        if (r16) { PLUQ_LEAF_NT(false, true) } else { PLUQ_LEAF_NT(false, false) }
    } else {
        if (r16) { PLUQ_LEAF_NT(true, true) } else { PLUQ_LEAF_NT(true, false) }
    }
#undef PLUQ_LEAF_NT
#undef PLUQ_LEAF
    return hipGetLastError();
}

template <typename T>
static hipError_t diag_inv_pair_t(const void *Lm, int64_t ldl, const void *Um, int64_t ldu, int r, void *WL, void *WU,
                                  double p, hipStream_t st) {
    const int nb = (int)cdiv64(r, 64);
    PLUQ_LAUNCH((trsm_diag_inv_pair_kernel<T>), dim3((unsigned)(2 * nb)), dim3(256), 0, st, (const T *)Lm, ldl,
                (const T *)Um, ldu, r, (T *)WL, (T *)WU, make_mod(p), nb);
    return hipGetLastError();
}

hipError_t launch_trsm_diag_inv_pair(int dtype, const void *Lm, int64_t ldl, const void *Um, int64_t ldu, int64_t r,
                                     void *WL, void *WU, double p, int kchunk, hipStream_t st) {
    if (r <= 0) return hipSuccess;
    if (kchunk < 1 || r > INT32_MAX / 2) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return diag_inv_pair_t<int64_t>(Lm, ldl, Um, ldu, (int)r, WL, WU, p, st);
    case DT_F64: return diag_inv_pair_t<double>(Lm, ldl, Um, ldu, (int)r, WL, WU, p, st);
    case DT_I32: return diag_inv_pair_t<int32_t>(Lm, ldl, Um, ldu, (int)r, WL, WU, p, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t leaf_pair_t(const void *Lm, int64_t ldl, const void *Um, int64_t ldu, int r, void *BD, int64_t ldbd,
                              int ncols, void *BE, int64_t ldbe, int nrows, const void *WL, const void *WU, double p,
                              int kchunk, hipStream_t st) {
    const int nt = leaf_groups(ncols, 2) + leaf_groups(nrows, 2) >= LEAF_WIDE_MIN_GROUPS ? 2 : 1;
    const int gD = leaf_groups(ncols, nt), gE = leaf_groups(nrows, nt);
    const ModP md = make_mod(p);
#define PLUQ_LEAF_PAIR(R16, NT)                                                                                     \
    PLUQ_LAUNCH((trsm_leaf_pair_kernel<T, R16, NT>), dim3((unsigned)(gD + gE)), dim3(256), 0, st, (const T *)Lm, ldl, \
                (const T *)Um, ldu, r, (T *)BD, ldbd, ncols, (T *)BE, ldbe, nrows, (const T *)WL, (const T *)WU, md, \
                kchunk, gD)
    if (kchunk < 64) {
        if (nt == 2) PLUQ_LEAF_PAIR(true, 2); else PLUQ_LEAF_PAIR(true, 1);
    } else {
        if (nt == 2) PLUQ_LEAF_PAIR(false, 2); else PLUQ_LEAF_PAIR(false, 1);
    }
#undef PLUQ_LEAF_PAIR
    return hipGetLastError();
}

hipError_t launch_trsm_leaf_pair(int dtype, const void *Lm, int64_t ldl, const void *Um, int64_t ldu, int64_t r,
                                 void *BD, int64_t ldbd, int64_t ncols, void *BE, int64_t ldbe, int64_t nrows,
                                 const void *WL, const void *WU, double p, int kchunk, hipStream_t st) {
    if (r <= 0 || ncols <= 0 || nrows <= 0) return hipErrorInvalidValue;
    if (r > TRSM_FUSE_MAX || kchunk < 16 || ncols > INT32_MAX / 2 || nrows > INT32_MAX / 2) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64:
        return leaf_pair_t<int64_t>(Lm, ldl, Um, ldu, (int)r, BD, ldbd, (int)ncols, BE, ldbe, (int)nrows, WL, WU, p,
                                    kchunk, st);
    case DT_F64:
        return leaf_pair_t<double>(Lm, ldl, Um, ldu, (int)r, BD, ldbd, (int)ncols, BE, ldbe, (int)nrows, WL, WU, p,
                                   kchunk, st);
    case DT_I32:
        return leaf_pair_t<int32_t>(Lm, ldl, Um, ldu, (int)r, BD, ldbd, (int)ncols, BE, ldbe, (int)nrows, WL, WU, p,
                                    kchunk, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_trsm_leaf(int dtype, int side, const void *Tm, int64_t ldt, int64_t r, void *B, int64_t ldb,
                            int64_t nst, const void *W, double p, int kchunk, hipStream_t st) {
    if (r <= 0 || nst <= 0) return hipSuccess;
    if (r > TRSM_FUSE_MAX || kchunk < 16 || nst > INT32_MAX) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return leaf_t<int64_t>(side, Tm, ldt, (int)r, B, ldb, (int)nst, W, p, kchunk, st);
    case DT_F64: return leaf_t<double>(side, Tm, ldt, (int)r, B, ldb, (int)nst, W, p, kchunk, st);
    case DT_I32: return leaf_t<int32_t>(side, Tm, ldt, (int)r, B, ldb, (int)nst, W, p, kchunk, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace pluq

// Base case of the recursion: the decomposition of a tile of at most
// TILE x TILE entries (TILE = 64 or 128), done by one work-group (256
// threads; 512 for the elimination of a 128 x 128 tile).
//
// The output must be exactly the one Algorithm 1 would produce on the tile
// (pivots in the order of its four recursive calls, non-pivot rows and
// columns ascending, then the LU of the permuted tile).  That order is a
// function of the tile's rank profile matrix alone, so the base case works in
// two kernels:
//   bc_rpm  -- the rank profile matrix: rows are taken in order and each
//              pivot is the first non-zero entry of the reduced row (the
//              row-major search of the row-rank-profile eliminations recalled
//              in Section 1; the reduced row's first non-zero column is where
//              the rank of the leading sub-matrices jumps);
//   bc_lu   -- elimination without pivoting of the tile gathered through the
//              row/column order, written back in packed form.
// bc_lu is also tried first on the tile as it is: when every pivot on the
// diagonal is non-zero (a generic rank profile, the case of Section 5's
// leading-constant analysis), or the remaining block is zero where the first
// zero pivot appears, the identity order is already the right one and the
// rank-profile pass is skipped.  The pivot order itself is computed on the
// host between the two kernels (index bookkeeping only).
//
// Layout: with NT threads, thread (ty, tx) = (tid / 16, tid % 16) holds the
// entries (ty + SY a, tx + 16 b), SY = NT / 16, in registers (RA x RB of
// them), so the shrinking trailing block stays evenly spread over the
// threads.  Register indices that depend on the step are resolved by
// wave-uniform switches, never by indexing.
// Pivot inverses come from an LDS table of inverses when p <= 65536, else
// from the extended Euclidean algorithm.
// Arithmetic uses delayed reduction (Section 6) inside the elimination: the
// update is one FMA of symmetric residues on an exact integer-valued double,
// an entry is reduced when it joins a pivot row or column, and every entry is
// reduced after `kchunk` steps so that no accumulator exceeds 2^52.
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

constexpr int BC_THREADS = 256;
// Threads of the elimination kernel for a tile: two waves per SIMD for the
// 128 x 128 tile (32 entries per thread), one for the 64 x 64 tile.
constexpr int bc_threads(int tile) { return tile > 64 ? 512 : 256; }
constexpr int BC_DIM = 128;            // largest tile
constexpr int BC_TAB_MAX = 65536;      // largest p with an LDS inverse table
constexpr size_t BC_TAB_BYTES = BC_TAB_MAX * sizeof(uint16_t);

// Inverse of every non-zero residue mod p (p <= 65536), as uint16.
__global__ __launch_bounds__(256) void build_inv_table_kernel(uint16_t *tab, ModP mod) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int p = (int)mod.p;
    if (a < p) tab[a] = (uint16_t)(a == 0 ? 0 : (int)mod_inv((double)a, mod));
}

// bc_lu step structure (one step = one pivot s):
//   P1  every thread finalises one entry of the pivot row or column: reads
//       its raw value from LDS, reduces it and publishes the symmetric
//       residue used by the update (the multipliers are the column scaled by
//       the pivot's inverse, which each thread looks up itself);
//   P2  every thread applies the rank-one update to its registers with
//       branch-free FMAs (inactive rows and columns were published as zero),
//       and the owners of row and column s+1 copy them to LDS for the next P1.
// Two barriers per step.  Once a row or column has been a pivot row or
// column its registers are never changed again (it is published as zero),
// so the result is read from the registers at the end: U entries reduced,
// L entries reduced and multiplied by their pivot's inverse (kept in LDS).
// A is written only on success, so a failed optimistic attempt leaves the
// input untouched.
struct BcShared {
    double row[BC_DIM];   // raw entries of the next pivot row
    double col[BC_DIM];   // raw entries of the next pivot column
    double Lb[BC_DIM];    // published multipliers (symmetric)
    double Ub[BC_DIM];    // published pivot row (symmetric)
    double inv[BC_DIM];   // inverse of each pivot
};

__device__ __forceinline__ double bc_inverse(double x, const ModP &mod, const uint16_t *tab) {
    if (x == 0.0) return 0.0;
    return tab ? (double)tab[(int)x] : mod_inv(x, mod);
}

template <typename T, int TILE, int NT>
__global__ __launch_bounds__(NT) void bc_lu_kernel(T *A, int64_t lda, int m, int n, const int32_t *rmap,
                                                   const int32_t *cmap, int r_known, ModP mod, int kchunk,
                                                   const uint16_t *gtab, int32_t *status, int32_t *specfail,
                                                   int32_t *errflag) {
    constexpr int SY = NT / 16;       // row stride of a thread's entries
    constexpr int RA = TILE / SY;     // rows per thread
    constexpr int RB = TILE / 16;     // columns per thread
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ BcShared sh;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const uint16_t *tab = nullptr;

    // copy the inverse table (16-byte words, in flight together)
    if (gtab) {
        const int words = ((int)mod.p + 7) / 8;
        const uint4 *src = (const uint4 *)gtab;
        uint4 *dst = (uint4 *)dyn;
        constexpr int PER = BC_TAB_MAX / 8 / NT;           // 16-byte words per thread
        constexpr int CH = 8;                               // loads in flight per thread
#pragma unroll
        for (int k0 = 0; k0 < PER; k0 += CH) {
            uint4 tmp[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int w = tid + (k0 + k) * NT;
                tmp[k] = (w < words) ? src[w] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int w = tid + (k0 + k) * NT;
                if (w < words) dst[w] = tmp[k];
            }
        }
        tab = (const uint16_t *)dyn;
    }

    double v[RA][RB];
#pragma unroll
    for (int a = 0; a < RA; ++a) {
        const int i = ty + SY * a;
        const int64_t gi = (i < m) ? (rmap ? rmap[i] : i) : 0;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int j = tx + 16 * b;
            double x = 0.0;
            if (i < m && j < n) x = to_f64(A[gi * lda + (cmap ? cmap[j] : j)]);
            v[a][b] = x;
        }
    }
    if (ty == 0) {
#pragma unroll
        for (int b = 0; b < RB; ++b) sh.row[tx + 16 * b] = v[0][b];
    }
    if (tx == 0) {
#pragma unroll
        for (int a = 0; a < RA; ++a) sh.col[ty + SY * a] = v[a][0];
    }
    __syncthreads();

    const int kmax = m < n ? m : n;
    const int steps = r_known >= 0 ? r_known : kmax;
    int r = steps;
    bool ok = true, stop = false;

    // One elimination step s whose row and column s+1 sit in register row
    // block QA and column block QB (compile-time constants, so the publish
    // needs no switch).  Returns false at a zero pivot (r and ok set).
    auto step = [&](int s, auto QA, auto QB) __attribute__((always_inline)) -> bool {
        constexpr int qa = decltype(QA)::value, qb = decltype(QB)::value;
        double piv = sym_reduce(sh.row[s], mod);
        if (piv == 0.0) {
            // zero pivot at (s, s): the identity order is right iff the rest is zero
            int any = 0;
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const int i = ty + SY * a, j = tx + 16 * b;
                    if (i >= s && j >= s && i < m && j < n) any |= (sym_reduce(v[a][b], mod) != 0.0);
                }
            any = __syncthreads_or(any);
            ok = (any == 0) && (r_known < 0);
            r = s;
            return false;
        }
        if (piv < 0.0) piv += mod.p;   // canonical, for the inverse
        const double inv = bc_inverse(piv, mod, tab);
        if (tid < TILE) {
            const int j = tid;
            const double u = sym_reduce(sh.row[j], mod);
            sh.Ub[j] = (j > s && j < n) ? u : 0.0;
            if (j == 0) sh.inv[s] = inv;
        } else if (tid < 2 * TILE) {
            const int i = tid - TILE;
            const bool act = (i > s) && (i < m);
            const double l = sym_reduce(sym_reduce(sh.col[i], mod) * inv, mod);
            sh.Lb[i] = act ? l : 0.0;
        }
        __syncthreads();
        double l[RA], u[RB];
#pragma unroll
        for (int a = 0; a < RA; ++a) l[a] = sh.Lb[ty + SY * a];
#pragma unroll
        for (int b = 0; b < RB; ++b) u[b] = sh.Ub[tx + 16 * b];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < RB; ++b) v[a][b] = fma(-l[a], u[b], v[a][b]);
        if (s + 1 < steps) {
            const int t = s + 1;
            if (ty == t % SY) {
#pragma unroll
                for (int b = 0; b < RB; ++b) sh.row[tx + 16 * b] = v[qa][b];
            }
            if (tx == (t & 15)) {
#pragma unroll
                for (int a = 0; a < RA; ++a) sh.col[ty + SY * a] = v[a][qb];
            }
        }
        __syncthreads();
        return true;
    };

    if (kchunk >= steps) {
        // No full-tile reduction needed: the steps run in blocks of 16 by the
        // index t = s + 1 of the row and column they publish, which sit in
        // register column block t / 16 and row block t / SY, unrolled.
#define PLUQ_BC_BLOCK(K)                                                                          \
    if constexpr ((K) < RB) {                                                                     \
        if (!stop) {                                                                              \
            const int tlo = (K) * 16 < 1 ? 1 : (K) * 16;                                          \
            const int thi = (K) * 16 + 16 <= steps ? (K) * 16 + 16 : steps + 1;                   \
            for (int t = tlo; t < thi; ++t) {                                                     \
                if (!step(t - 1, std::integral_constant<int, ((K) * 16) / SY>{},                  \
                          std::integral_constant<int, (K)>{})) {                                  \
                    stop = true;                                                                  \
                    break;                                                                        \
                }                                                                                 \
            }                                                                                     \
        }                                                                                         \
    }
        PLUQ_BC_BLOCK(0)
        PLUQ_BC_BLOCK(1)
        PLUQ_BC_BLOCK(2)
        PLUQ_BC_BLOCK(3)
        PLUQ_BC_BLOCK(4)
        PLUQ_BC_BLOCK(5)
        PLUQ_BC_BLOCK(6)
        PLUQ_BC_BLOCK(7)
#undef PLUQ_BC_BLOCK
        // the last step of a full tile (s = TILE - 1 publishes nothing)
        if (!stop && steps == 16 * RB) {
            if (!step(steps - 1, std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{})) stop = true;
        }
    } else {
    // Steps are taken in chunks of kchunk with a full-tile reduction between
    // chunks, so that the loop over the steps of a chunk carries the tile
    // registers through unchanged (a conditional reduction inside it makes
    // the compiler keep two copies of the tile).
    for (int s0 = 0; s0 < steps && !stop; s0 += kchunk) {
    const int s1 = (steps - s0 > kchunk) ? s0 + kchunk : steps;
    for (int s = s0; s < s1; ++s) {
        // ---- P1
        double piv = sym_reduce(sh.row[s], mod);
        if (piv == 0.0) {
            // zero pivot at (s, s): the identity order is right iff the rest is zero
            int any = 0;
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    const int i = ty + SY * a, j = tx + 16 * b;
                    if (i >= s && j >= s && i < m && j < n) any |= (sym_reduce(v[a][b], mod) != 0.0);
                }
            any = __syncthreads_or(any);
            ok = (any == 0) && (r_known < 0);
            r = s;
            stop = true;
            break;
        }
        if (piv < 0.0) piv += mod.p;   // canonical, for the inverse
        const double inv = bc_inverse(piv, mod, tab);
        if (tid < TILE) {
            const int j = tid;
            const double u = sym_reduce(sh.row[j], mod);
            sh.Ub[j] = (j > s && j < n) ? u : 0.0;
            if (j == 0) sh.inv[s] = inv;
        } else if (tid < 2 * TILE) {
            const int i = tid - TILE;
            const bool act = (i > s) && (i < m);
            const double l = sym_reduce(sym_reduce(sh.col[i], mod) * inv, mod);
            sh.Lb[i] = act ? l : 0.0;
        }
        __syncthreads();
        // ---- P2
        double l[RA], u[RB];
#pragma unroll
        for (int a = 0; a < RA; ++a) l[a] = sh.Lb[ty + SY * a];
#pragma unroll
        for (int b = 0; b < RB; ++b) u[b] = sh.Ub[tx + 16 * b];
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < RB; ++b) v[a][b] = fma(-l[a], u[b], v[a][b]);
        if (s + 1 < steps) {
            // owners of row / column s+1 copy them to LDS; the register
            // indices (s+1)/SY and (s+1)/16 are wave-uniform and resolved by
            // the switches
            const int t = s + 1;
#define PLUQ_BC_ROW(Q)                                                                        \
    if constexpr ((Q) < RA) {                                                                 \
        if (ty == t % SY) {                                                                   \
            _Pragma("unroll") for (int b = 0; b < RB; ++b) sh.row[tx + 16 * b] = v[(Q)][b];   \
        }                                                                                     \
    }
#define PLUQ_BC_COL(Q)                                                                        \
    if constexpr ((Q) < RB) {                                                                 \
        if (tx == (t & 15)) {                                                                 \
            _Pragma("unroll") for (int a = 0; a < RA; ++a) sh.col[ty + SY * a] = v[a][(Q)];   \
        }                                                                                     \
    }
            if constexpr (SY == 16) {
                // one switch: row and column s+1 sit at the same register index
                switch (t >> 4) {
                case 0: PLUQ_BC_ROW(0) PLUQ_BC_COL(0) break;
                case 1: PLUQ_BC_ROW(1) PLUQ_BC_COL(1) break;
                case 2: PLUQ_BC_ROW(2) PLUQ_BC_COL(2) break;
                case 3: PLUQ_BC_ROW(3) PLUQ_BC_COL(3) break;
                case 4: PLUQ_BC_ROW(4) PLUQ_BC_COL(4) break;
                case 5: PLUQ_BC_ROW(5) PLUQ_BC_COL(5) break;
                case 6: PLUQ_BC_ROW(6) PLUQ_BC_COL(6) break;
                case 7: PLUQ_BC_ROW(7) PLUQ_BC_COL(7) break;
                default: break;
                }
            } else {
                switch (t / SY) {
                case 0: PLUQ_BC_ROW(0) break;
                case 1: PLUQ_BC_ROW(1) break;
                case 2: PLUQ_BC_ROW(2) break;
                case 3: PLUQ_BC_ROW(3) break;
                case 4: PLUQ_BC_ROW(4) break;
                case 5: PLUQ_BC_ROW(5) break;
                case 6: PLUQ_BC_ROW(6) break;
                case 7: PLUQ_BC_ROW(7) break;
                default: break;
                }
                switch (t >> 4) {
                case 0: PLUQ_BC_COL(0) break;
                case 1: PLUQ_BC_COL(1) break;
                case 2: PLUQ_BC_COL(2) break;
                case 3: PLUQ_BC_COL(3) break;
                case 4: PLUQ_BC_COL(4) break;
                case 5: PLUQ_BC_COL(5) break;
                case 6: PLUQ_BC_COL(6) break;
                case 7: PLUQ_BC_COL(7) break;
                default: break;
                }
            }
#undef PLUQ_BC_ROW
#undef PLUQ_BC_COL
        }
        __syncthreads();
    }
    if (!stop && s1 < steps) {
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < RB; ++b) v[a][b] = sym_reduce(v[a][b], mod);
    }
    }
    }
    if (ok && r_known >= 0 && r < kmax) {
        // the rank is known: the block left after it must be zero
        int any = 0;
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const int i = ty + SY * a, j = tx + 16 * b;
                if (i >= r && j >= r && i < m && j < n) any |= (sym_reduce(v[a][b], mod) != 0.0);
            }
        ok = __syncthreads_or(any) == 0;
    }
    // speculative use (the caller assumed a full-rank tile in the identity
    // order): record a failed assumption in the sticky flag
    if (specfail && tid == 0 && (!ok || r != kmax)) *specfail = 1;
    // (errflag: the ordered elimination's self-check, read by the host later)
    if (errflag && tid == 0 && !ok) *errflag = 1;
    if (!ok) {
        if (tid == 0) { status[0] = r; status[1] = 0; }
        return;
    }
#pragma unroll
    for (int a = 0; a < RA; ++a) {
        const int i = ty + SY * a;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int j = tx + 16 * b;
            if (i < m && j < n) {
                double x = mod_reduce(v[a][b], mod);
                if (j < r && i > j) x = mod_mul(x, sh.inv[j], mod);   // L entry
                A[(int64_t)i * lda + j] = from_f64<T>(x);
            }
        }
    }
    if (tid == 0) { status[0] = r; status[1] = 1; }
}

// Rank profile matrix of the tile: status[0] = r, status[1 + i] = pivot
// column of row i or -1.  Rows are processed in order; the pivot of row i is
// the first non-zero entry of the reduced row among the columns that are not
// yet pivot columns.  (Taken for non-generic tiles only.)  Same register
// layout as the elimination kernel with 256 threads (R x R entries per
// thread); rows run in blocks of 16 so that the row owners' register row is
// a compile-time index; each thread keeps the pivot columns among its own
// columns as a bit mask; the pivot inverse comes from the LDS table when p
// <= 65536; the tile is reduced (symmetric reduction) after every block of 16
// rows, or after every pivot when RED1 (p close to 2^25).
template <typename T, bool RED1>
__global__ __launch_bounds__(BC_THREADS) void bc_rpm_kernel(const T *A, int64_t lda, int m, int n, ModP mod,
                                                            const uint16_t *gtab, int32_t *status) {
    constexpr int R = 8;
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ double Lb[BC_DIM];
    __shared__ double Ub[2][BC_DIM];
    __shared__ int mins[2][16];
    __shared__ double s_inv;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const uint16_t *tab = nullptr;
    if (gtab) {
        const int words = ((int)mod.p + 7) / 8;
        const uint4 *src = (const uint4 *)gtab;
        uint4 *dst = (uint4 *)dyn;
        constexpr int PER = BC_TAB_MAX / 8 / BC_THREADS;
        constexpr int CH = 8;
#pragma unroll
        for (int k0 = 0; k0 < PER; k0 += CH) {
            uint4 tmp[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int w = tid + (k0 + k) * BC_THREADS;
                tmp[k] = (w < words) ? src[w] : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const int w = tid + (k0 + k) * BC_THREADS;
                if (w < words) dst[w] = tmp[k];
            }
        }
        tab = (const uint16_t *)dyn;
    }
    double v[R][R];
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
        for (int b = 0; b < R; ++b) {
            const int i = ty + 16 * a, j = tx + 16 * b;
            v[a][b] = (i < m && j < n) ? to_f64(A[(int64_t)i * lda + j]) : 0.0;
        }
    if (tid < m) status[1 + tid] = -1;
    uint32_t dead = 0;   // bit b: column tx + 16 b is a pivot column
    __syncthreads();
    int r = 0;
    auto reduce_all = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b) v[a][b] = sym_reduce(v[a][b], mod);
    };
    auto row_step = [&](int i, auto AI) __attribute__((always_inline)) {
        constexpr int ai = decltype(AI)::value;
        const int buf = i & 1;
        if (ty == (i & 15)) {
            int first = 1 << 30;
#pragma unroll
            for (int b = 0; b < R; ++b) {
                const int j = tx + 16 * b;
                if (j < n && !((dead >> b) & 1u)) {
                    const double u = sym_reduce(v[ai][b], mod);
                    v[ai][b] = u;
                    Ub[buf][j] = u;
                    if (u != 0.0 && j < first) first = j;
                }
            }
            mins[buf][tx] = first;
        }
        __syncthreads();
        int jc = 1 << 30;
#pragma unroll
        for (int t = 0; t < 16; ++t) jc = min(jc, mins[buf][t]);
        if (jc >= n) return;   // dependent row (uniform)
        ++r;
        const int bj = jc >> 4;
        if (ty == (i & 15) && tx == (jc & 15)) {
            double pv = 0.0;
#pragma unroll
            for (int b = 0; b < R; ++b)
                if (b == bj) pv = v[ai][b];
            if (pv < 0.0) pv += mod.p;   // canonical, for the inverse
            s_inv = tab ? (double)tab[(int)pv] : mod_inv(pv, mod);
            status[1 + i] = jc;
        }
        if (tx == (jc & 15)) dead |= 1u << bj;
        __syncthreads();
        const double inv = s_inv;
        if (tx == (jc & 15)) {
#pragma unroll
            for (int a = 0; a < R; ++a) {
                const int k = ty + 16 * a;
                if (k > i && k < m) {
                    double c = 0.0;
#pragma unroll
                    for (int b = 0; b < R; ++b)
                        if (b == bj) c = v[a][b];
                    Lb[k] = sym_reduce(sym_reduce(c, mod) * inv, mod);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < R; ++a) {
            const int k = ty + 16 * a;
            if (k > i && k < m) {
                const double l = Lb[k];
#pragma unroll
                for (int b = 0; b < R; ++b) {
                    const int j = tx + 16 * b;
                    if (j < n && !((dead >> b) & 1u)) v[a][b] = fma(-l, Ub[buf][j], v[a][b]);
                }
            }
        }
        if (RED1) reduce_all();
        // Ub and mins are double-buffered: the next row's owners fill the
        // other half before its first barrier.  Lb and s_inv are rewritten
        // only after that barrier, which every thread reaches after this
        // update.
    };
#define PLUQ_RPM_BLOCK(K)                                                                         \
    {                                                                                             \
        const int ihi = (K) * 16 + 16 < m ? (K) * 16 + 16 : m;                                    \
        for (int i = (K) * 16; i < ihi; ++i) row_step(i, std::integral_constant<int, (K)>{});     \
        if (!RED1) reduce_all();                                                                  \
    }
    PLUQ_RPM_BLOCK(0)
    PLUQ_RPM_BLOCK(1)
    PLUQ_RPM_BLOCK(2)
    PLUQ_RPM_BLOCK(3)
    PLUQ_RPM_BLOCK(4)
    PLUQ_RPM_BLOCK(5)
    PLUQ_RPM_BLOCK(6)
    PLUQ_RPM_BLOCK(7)
#undef PLUQ_RPM_BLOCK
    __syncthreads();
    if (tid == 0) status[0] = r;
}

static ModP make_mod(double p) {
    ModP md;
    md.p = p;
    md.pinv = 1.0 / p;
    md.half = (double)((int64_t)p / 2);
    return md;
}

static bool g_tab_ok = false;

int bc_capacity() { return BC_DIM; }

// Dynamic LDS of the tile kernel: the 128 KB table of inverses when used.
hipError_t bc_init() {
    // The LDS inverse table needs a large dynamic LDS allocation; without it
    // the kernel computes inverses by the extended Euclidean algorithm.
    g_tab_ok = true;
#define PLUQ_SETLDS(K)                                                                                 \
    if (hipFuncSetAttribute((const void *)(K), hipFuncAttributeMaxDynamicSharedMemorySize,               \
                            (int)BC_TAB_BYTES) != hipSuccess)                                           \
        g_tab_ok = false;
    PLUQ_SETLDS((bc_lu_kernel<int64_t, 64, bc_threads(64)>))
    PLUQ_SETLDS((bc_lu_kernel<double, 64, bc_threads(64)>))
    PLUQ_SETLDS((bc_lu_kernel<int32_t, 64, bc_threads(64)>))
    PLUQ_SETLDS((bc_lu_kernel<int64_t, 128, bc_threads(128)>))
    PLUQ_SETLDS((bc_lu_kernel<double, 128, bc_threads(128)>))
    PLUQ_SETLDS((bc_lu_kernel<int32_t, 128, bc_threads(128)>))
    PLUQ_SETLDS((bc_rpm_kernel<int64_t, false>))
    PLUQ_SETLDS((bc_rpm_kernel<double, false>))
    PLUQ_SETLDS((bc_rpm_kernel<int32_t, false>))
    PLUQ_SETLDS((bc_rpm_kernel<int64_t, true>))
    PLUQ_SETLDS((bc_rpm_kernel<double, true>))
    PLUQ_SETLDS((bc_rpm_kernel<int32_t, true>))
#undef PLUQ_SETLDS
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        prop.sharedMemPerBlock < BC_TAB_BYTES + sizeof(BcShared) + 1024)
        g_tab_ok = false;
    (void)hipGetLastError();
    return hipSuccess;
}

int bc_tile_limit(double p) { (void)p; return BC_DIM; }

size_t bc_table_bytes(double p) { return (g_tab_ok && p <= BC_TAB_MAX) ? BC_TAB_BYTES : 0; }

hipError_t launch_build_inv_table(uint16_t *tab, double p, hipStream_t st) {
    if (p > BC_TAB_MAX) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)(((int64_t)p + 255) / 256);
    PLUQ_LAUNCH(build_inv_table_kernel, dim3(blocks), dim3(256), 0, st, tab, make_mod(p));
    return hipGetLastError();
}

template <int TILE>
static hipError_t bc_lu_t(int dtype, void *A, int64_t lda, int m, int n, const int32_t *rmap,
                          const int32_t *cmap, int r_known, double p, int kchunk, const uint16_t *tab,
                          int32_t *status, int32_t *specfail, int32_t *errflag, hipStream_t st) {
    const size_t lds = tab ? BC_TAB_BYTES : 0;
    const ModP md = make_mod(p);
    switch (dtype) {
    case DT_I64:
        PLUQ_LAUNCH((bc_lu_kernel<int64_t, TILE, bc_threads(TILE)>), dim3(1), dim3(bc_threads(TILE)), lds, st, (int64_t *)A, lda,
                    m, n, rmap, cmap, r_known, md, kchunk, tab, status, specfail, errflag);
        break;
    case DT_F64:
        PLUQ_LAUNCH((bc_lu_kernel<double, TILE, bc_threads(TILE)>), dim3(1), dim3(bc_threads(TILE)), lds, st, (double *)A, lda,
                    m, n, rmap, cmap, r_known, md, kchunk, tab, status, specfail, errflag);
        break;
    case DT_I32:
        PLUQ_LAUNCH((bc_lu_kernel<int32_t, TILE, bc_threads(TILE)>), dim3(1), dim3(bc_threads(TILE)), lds, st, (int32_t *)A, lda,
                    m, n, rmap, cmap, r_known, md, kchunk, tab, status, specfail, errflag);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bc_lu(int dtype, void *A, int64_t lda, int m, int n, const int32_t *rmap,
                        const int32_t *cmap, int r_known, double p, int kchunk, const uint16_t *tab,
                        int32_t *status, int32_t *specfail, int32_t *errflag, hipStream_t st) {
    if (m > BC_DIM || n > BC_DIM || m <= 0 || n <= 0 || kchunk < 1) return hipErrorInvalidValue;
    if (tab && p > BC_TAB_MAX) return hipErrorInvalidValue;
    // Steps between full-tile reductions for this kernel's bound: entries
    // start below p in magnitude, every step adds at most (p/2 + 1)^2 (the
    // multipliers and pivot-row entries are symmetric reductions), and the
    // sum must stay below 2^52.
    {
        const double h = std::floor(p / 2) + 1.0;
        const double c = std::floor((4503599627370496.0 - 2.0 * p) / (h * h));
        kchunk = c >= 1048576.0 ? 1048576 : (c < 1.0 ? 1 : (int)c);
    }
    if (m <= 64 && n <= 64)
        return bc_lu_t<64>(dtype, A, lda, m, n, rmap, cmap, r_known, p, kchunk, tab, status, specfail, errflag, st);
    return bc_lu_t<128>(dtype, A, lda, m, n, rmap, cmap, r_known, p, kchunk, tab, status, specfail, errflag, st);
}

hipError_t launch_bc_rpm(int dtype, const void *A, int64_t lda, int m, int n, double p, int kchunk,
                         const uint16_t *tab, int32_t *status, hipStream_t st) {
    if (m > BC_DIM || n > BC_DIM || m <= 0 || n <= 0 || kchunk < 1) return hipErrorInvalidValue;
    if (tab && p > BC_TAB_MAX) return hipErrorInvalidValue;
    // pivots between reductions for symmetric entries: every pivot adds at
    // most (p/2 + 1)^2 to an entry that starts below p in magnitude
    const double h = std::floor(p / 2) + 1.0;
    const bool red1 = (4503599627370496.0 - 2.0 * p) / (h * h) < 16.0;
    const size_t lds = tab ? BC_TAB_BYTES : 0;
    const ModP md = make_mod(p);
#define PLUQ_RPM(TT)                                                                                     \
    if (red1)                                                                                            \
        PLUQ_LAUNCH((bc_rpm_kernel<TT, true>), dim3(1), dim3(BC_THREADS), lds, st, (const TT *)A, lda, m, n, md, \
                    tab, status);                                                                        \
    else                                                                                                 \
        PLUQ_LAUNCH((bc_rpm_kernel<TT, false>), dim3(1), dim3(BC_THREADS), lds, st, (const TT *)A, lda, m, n, md, \
                    tab, status);
    switch (dtype) {
    case DT_I64: PLUQ_RPM(int64_t) break;
    case DT_F64: PLUQ_RPM(double) break;
    case DT_I32: PLUQ_RPM(int32_t) break;
    default: return hipErrorInvalidValue;
    }
#undef PLUQ_RPM
    return hipGetLastError();
}

}  // namespace pluq

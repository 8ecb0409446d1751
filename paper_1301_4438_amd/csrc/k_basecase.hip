// Base case of the recursion: the decomposition of a tile of at most
// 128 x 128 entries, done by one work-group.
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
// bc_lu runs one work-group of TILE / 16 waves per tile (TILE = 64 or 128),
// blocked by panels of 16 columns, each factored inside one wave; bc_rpm
// keeps the tile in registers, thread (ty, tx) = (tid / 16, tid % 16)
// holding entries (ty + 16 a, tx + 16 b).  The layouts are described at each
// kernel.
// Pivot inverses come from an LDS table of inverses when p <= 65536, else
// from the extended Euclidean algorithm.
// Arithmetic uses delayed reduction (Section 6): products of symmetric
// residues are accumulated exactly in float64 and reduced before any sum
// could pass 2^52.
#include <cmath>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

constexpr int BC_THREADS = 256;
constexpr int BC_DIM = 128;            // largest tile
constexpr int BC_TAB_MAX = 65536;      // largest p with an LDS inverse table
constexpr size_t BC_TAB_BYTES = BC_TAB_MAX * sizeof(uint16_t);

// Inverse of every non-zero residue mod p (p <= 65536), as uint16.
__global__ __launch_bounds__(256) void build_inv_table_kernel(uint16_t *tab, ModP mod) {
    const int a = blockIdx.x * 256 + threadIdx.x;
    const int p = (int)mod.p;
    if (a < p) tab[a] = (uint16_t)(a == 0 ? 0 : (int)mod_inv((double)a, mod));
}

// bc_lu: elimination without pivoting of a tile, blocked by panels of 16
// columns.  With TILE x TILE the tile size (64 or 128) there are NW =
// TILE / 16 waves; wave w owns column block w (columns 16w .. 16w+15) for the
// whole tile, held as NW matrix-core accumulator blocks of 16 x 16 (lane
// holds rows (lane / 16) + 4v, column lane % 16 of each block).
//
// Panel k (columns c0 = 16k .. c0+15) is factored by its owner, wave k, on
// its own: the column block goes through LDS into a row layout (lane l holds
// rows l and l + 64, all 16 columns) and the 16 steps run with the pivot row
// broadcast by lane reads, with no work-group barrier per pivot.  The steps
// are free of branches (a zero pivot, or the end of the steps asked for,
// turns the remaining steps into no-ops through their multipliers) and each
// updates the next pivot column first, so that the next pivot's reduction
// and table lookup overlap the update of the other columns.  The owner then
// publishes the negated multipliers below the panel (L21) and the panel's
// four block-column eliminators M_c (c = 0..3, 16 x 4 each): with D_c the
// unit lower 4 x 4 diagonal block of L11 at columns 4c..4c+3, M_c holds
// D_c^-1 - I in the chunk's rows and -L11[below, 4c..4c+3] D_c^-1 below them,
// so that A12 <- A12 + M_c A12[4c..4c+3], taken for c = 0..3, leaves
// U12 = L11^-1 A12.  After one barrier every later wave w forms its block of
// U12 that way (four matrix-core products) and applies the rank-16 update
// A22 <- A22 - L21 U12 to its column block with v_mfma_f64_16x16x4: a block
// row of the accumulator is already in the operand layout the instruction
// takes for B, so no data moves between the products.  The owner of the
// next panel does its own update first (at a raised wave priority) and goes
// on to factor while the others update theirs.  The published panels are
// double-buffered, so one barrier per panel suffices.  Values cross LDS as
// float: symmetric residues are at most p/2 + 1 <= 2^24 in magnitude for
// p < 2^25, exact in float.
//
// A zero pivot at step s (or the end of the r_known steps of an ordered
// elimination) ends the panel there: the owner publishes the steps done so
// far (zero multipliers in the remaining columns, an identity part of L11),
// the other waves apply that partial update, and the block left at (s, s)
// is tested for zero across the work-group: the identity order is right
// exactly when it is zero (r = s).
// Delayed reduction (Section 6): every quantity that enters a product is a
// symmetric residue, the panel accumulates at most 15 rank-one updates, the
// U12 chunks at most 12 products, and the trailing blocks are reduced before an update
// whenever kchunk products could be exceeded (every 8 products for p close
// to 2^25).
// The result goes through LDS (canonical residues as int32, over the
// inverse table, which is no longer needed) and is stored with whole rows
// per instruction.  A is written only on success, so a failed optimistic
// attempt leaves the input untouched.

typedef double bc_v4d __attribute__((ext_vector_type(4)));
typedef double bc_v8d __attribute__((ext_vector_type(8)));

// Value of x held by lane `src` (wave-uniform), for every lane.
__device__ __forceinline__ double bc_lane(double x, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), src);
    return __hiloint2double(hi, lo);
}

// Order of this wave's own LDS accesses (one wave's LDS instructions are
// executed in issue order; this keeps the compiler from reordering them).
__device__ __forceinline__ void bc_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Symmetric reduction x - round(x / p) p with the quotient rounded by adding
// and subtracting 1.5 * 2^52 (one fused multiply-add forms x / p + 1.5 * 2^52
// with a single rounding, which lands on an integer for |x / p| < 2^51):
// three full-rate operations, the same result bounds as sym_reduce
// (magnitude at most p/2 + 1, zero exactly when p divides x, |x| < 2^52).
__device__ __forceinline__ double bc_sym(double x, const ModP &m) {
    constexpr double MAGIC = 6755399441055744.0;
    const double q = fma(x, m.pinv, MAGIC) - MAGIC;
    return fma(-q, m.p, x);
}

constexpr int BC_XS = 17;                            // padded row stride (floats) of the panel buffers
constexpr int BC_OUT_BYTES = BC_DIM * (BC_DIM + 1) * 4;   // int32 result tile staged in LDS

template <int TILE> struct BcBlkShared {
    float xb[TILE * BC_XS];          // owner's column block, transposed (owner only)
    float pl[2][TILE * BC_XS];       // published panel: -L21 below it
    float pi[2][16 * BC_XS];         // published chunk eliminators M_0..M_3
    int flag[2][2];                  // steps done in the panel, zero pivot hit
};

template <typename T, int TILE, bool TAB>
__global__ __launch_bounds__(TILE * 4) void bc_lu_kernel(T *A, int64_t lda, int m, int n, const int32_t *rmap,
                                                         const int32_t *cmap, int r_known, ModP mod, int kchunk,
                                                         const uint16_t *gtab, int32_t *status, int32_t *specfail,
                                                         int32_t *errflag) {
    constexpr int NW = TILE / 16;   // waves = column blocks = block rows
    constexpr int NT = 64 * NW;
    constexpr int NH = TILE / 64;   // rows per lane in the row layout
    constexpr int XS = BC_XS;
    constexpr int OS = TILE + 1;    // row stride of the staged result
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ BcBlkShared<TILE> sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const uint16_t *tab = (const uint16_t *)dyn;

    // copy the inverse table (16-byte words, in flight together)
    if (TAB) {
        const int words = ((int)mod.p + 7) / 8;
        const uint4 *src = (const uint4 *)gtab;
        uint4 *dst = (uint4 *)dyn;
        constexpr int PER = BC_TAB_MAX / 8 / NT;
        constexpr int CH = 8;
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
    }

    // the column block of this wave, in accumulator layout: row indices
    // first (all in flight), then the entries (clamped addresses, all in
    // flight), then out-of-range entries masked to zero
    bc_v4d acc[NW];
    {
        const int j = 16 * wave + lr;
        const bool jin = j < n;
        const int jc = jin ? j : n - 1;
        const int64_t gj = cmap ? cmap[jc] : jc;
        int32_t ri[NW][4];
        if (rmap) {
#pragma unroll
            for (int b = 0; b < NW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) ri[b][v] = rmap[min(16 * b + lq + 4 * v, m - 1)];
        } else {
#pragma unroll
            for (int b = 0; b < NW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) ri[b][v] = min(16 * b + lq + 4 * v, m - 1);
        }
        T raw[NW][4];
#pragma unroll
        for (int b = 0; b < NW; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) raw[b][v] = A[(int64_t)ri[b][v] * lda + gj];
#pragma unroll
        for (int b = 0; b < NW; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[b][v] = (jin && 16 * b + lq + 4 * v < m) ? to_f64(raw[b][v]) : 0.0;
    }
    if (TAB) __syncthreads();   // the table is in LDS
    // After a wave has factored its panel, the same registers hold its column
    // block in row layout: rows lane + 64h, columns 16 wave + j.
#define RR(h, j) acc[((h) * 16 + (j)) >> 2][((h) * 16 + (j)) & 3]

    const int kmax = m < n ? m : n;
    const int steps = r_known >= 0 ? r_known : kmax;
    const double p = mod.p;
    // trailing blocks get at most 16 products per panel: reduce them before
    // each update unless NW - 1 updates fit in kchunk; every 8 products when
    // 16 do not
    const bool red_each = kchunk < 16 * NW;
    const bool red8 = kchunk < 16;

    int r = 0, klast = -1;
    bool zero_hit = false;
    for (int k = 0; k < NW; ++k) {
        const int c0 = 16 * k;
        if (c0 >= steps) break;   // steps == 0 only (otherwise the exit below)
        const int buf = k & 1;
        if (wave == k) {
            // ---- owner: column block -> row layout
#pragma unroll
            for (int b = 0; b < NW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    sh.xb[(16 * b + lq + 4 * v) * XS + lr] = (float)bc_sym(acc[b][v], mod);
            bc_wave_sync();
#pragma unroll
            for (int h = 0; h < NH; ++h)
#pragma unroll
                for (int j = 0; j < 16; ++j) RR(h, j) = (double)sh.xb[(lane + 64 * h) * XS + j];
            bc_wave_sync();
            // ---- factor the panel: steps s = c0 + C while s < steps and no
            // zero pivot has been met (later steps have zero multipliers);
            // cd counts the steps done, zh records a zero pivot
            int cd = 0;
            bool zh = false;
            double X[16];   // this lane's row of the chunk matrices M_c (below)
            auto factor = [&](auto HS) __attribute__((always_inline)) {
                constexpr int hs = decltype(HS)::value;
                // Pivot of step s (its row and column updated through step
                // s - 1): whether the step runs (good) and the inverse (0
                // when it does not, so that its multipliers vanish).
                bool good;
                double inv;
                auto pivot = [&](int s, double raw, bool alive) __attribute__((always_inline)) {
                    double pv = bc_sym(raw, mod);
                    pv = (pv < 0.0) ? pv + p : pv;
                    const bool run = alive && s < steps;
                    good = run && pv != 0.0;
                    zh = zh || (run && pv == 0.0);
                    if constexpr (TAB) inv = (double)tab[good ? (int)pv : 0];
                    else inv = mod_inv(good ? pv : 0.0, mod);
                };
                pivot(c0, bc_lane(RR(hs, 0), c0 & 63), true);
                // Step C: multipliers of column C, then the update of column
                // C + 1 and the next pivot (its reduction and inverse in
                // flight) before the update of the other columns.
                auto step = [&](auto CC) __attribute__((always_inline)) {
                    constexpr int C = decltype(CC)::value;
                    const int s = c0 + C;
                    cd = good ? C + 1 : cd;
                    // pivot row s, reduced in place, read from its lane
#pragma unroll
                    for (int j = C + 1; j < 16; ++j) RR(hs, j) = bc_sym(RR(hs, j), mod);
                    double u[16];
#pragma unroll
                    for (int j = C + 1; j < 16; ++j) u[j] = bc_lane(RR(hs, j), s & 63);
                    double lv[NH];
#pragma unroll
                    for (int h = hs; h < NH; ++h) {   // halves below hs hold rows above the panel
                        const bool act = good && lane + 64 * h > s;
                        // |x| <= p/2 + 1 + 15 (p/2 + 1)^2, so x * inv < 2^52 for
                        // p <= 65536 without reducing x first
                        const double x = TAB ? RR(h, C) : bc_sym(RR(h, C), mod);
                        const double l = bc_sym(x * inv, mod);
                        lv[h] = act ? l : 0.0;
                        RR(h, C) = act ? l : RR(h, C);
                    }
                    if constexpr (C + 1 < 16) {
#pragma unroll
                        for (int h = hs; h < NH; ++h) RR(h, C + 1) = fma(-lv[h], u[C + 1], RR(h, C + 1));
                        pivot(s + 1, bc_lane(RR(hs, C + 1), (s + 1) & 63), good);
#pragma unroll
                        for (int h = hs; h < NH; ++h)
#pragma unroll
                            for (int j = C + 2; j < 16; ++j) RR(h, j) = fma(-lv[h], u[j], RR(h, j));
                    }
                    __builtin_amdgcn_sched_barrier(0);
                };
#define PLUQ_S(C) step(std::integral_constant<int, C>{})
                PLUQ_S(0); PLUQ_S(1); PLUQ_S(2); PLUQ_S(3); PLUQ_S(4); PLUQ_S(5); PLUQ_S(6); PLUQ_S(7);
                PLUQ_S(8); PLUQ_S(9); PLUQ_S(10); PLUQ_S(11); PLUQ_S(12); PLUQ_S(13); PLUQ_S(14); PLUQ_S(15);
#undef PLUQ_S
                // ---- the panel's block-column eliminators, 4 columns at a
                // time: with D_c the unit lower 4 x 4 diagonal block of L11 at
                // columns 4c..4c+3 (entries of the steps done only), row t of
                // M_c is (D_c^-1 - I)[t - 4c] inside the chunk, -L[t][4c..]
                // D_c^-1 below it and 0 above, so that the update
                // A12 <- A12 + M_c A12[4c..4c+3] taken for c = 0..3 leaves
                // U12 = L11^-1 A12.  This lane forms the 16 entries of its
                // row t = lane + 64 hs - c0 (meaningful for the panel's rows).
                const int cdu = __builtin_amdgcn_readfirstlane(cd);
                const int t = lane + 64 * hs - c0;
                // with this row's multipliers masked to the columns q < t
                // (and to the steps done), -sum_{q >= g} L[t][4c+q] D_c^-1[q][g]
                // is D_c^-1[t-4c][g] for g < t - 4c inside the chunk, 0 on and
                // above its diagonal, the entry below it, and 0 above it
                const int qlim = min(t, cdu);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    // D_c's strict lower entries, from the rows' lanes
                    auto Lq = [&](int g, int q) __attribute__((always_inline)) {
                        const double x = bc_lane(RR(hs, 4 * c + q), (c0 + 4 * c + g) & 63);
                        return (4 * c + q < cdu) ? x : 0.0;
                    };
                    const double a10 = Lq(1, 0), a20 = Lq(2, 0), a21 = Lq(2, 1), a30 = Lq(3, 0), a31 = Lq(3, 1),
                                 a32 = Lq(3, 2);
                    // D_c^-1 by forward substitution (unit diagonal)
                    const double i10 = -a10;
                    const double i21 = -a21;
                    const double i20 = -bc_sym(fma(a21, i10, a20), mod);
                    const double i32 = -a32;
                    const double i31 = -bc_sym(fma(a32, i21, a31), mod);
                    const double i30 = -bc_sym(fma(a32, i20, fma(a31, i10, a30)), mod);
                    const double Di[4][4] = {{1.0, 0.0, 0.0, 0.0}, {i10, 1.0, 0.0, 0.0}, {i20, i21, 1.0, 0.0},
                                             {i30, i31, i32, 1.0}};
                    double lt[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) lt[q] = (4 * c + q < qlim) ? RR(hs, 4 * c + q) : 0.0;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        double d = 0.0;
#pragma unroll
                        for (int q = g; q < 4; ++q) d = fma(lt[q], Di[q][g], d);
                        X[4 * c + g] = -bc_sym(d, mod);
                    }
                }
            };
            if constexpr (NH == 1) {
                factor(std::integral_constant<int, 0>{});
            } else {
                if (c0 < 64) factor(std::integral_constant<int, 0>{});
                else factor(std::integral_constant<int, 1>{});
            }
            // ---- publish -L21 (the steps done; zero columns after them;
            // rows above the panel are written too but never read) and the
            // chunk matrices M_c
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int i = lane + 64 * h;
#pragma unroll
                for (int j = 0; j < 16; ++j)
                    sh.pl[buf][i * XS + j] = (i >= c0 + 16 && j < cd) ? -(float)RR(h, j) : 0.0f;
            }
            {
                const int t = lane + 64 * (c0 >> 6) - c0;
                if (t >= 0 && t < 16) {
#pragma unroll
                    for (int q = 0; q < 16; ++q) sh.pi[buf][t * XS + q] = (float)X[q];
                }
            }
            if (lane == 0) {
                sh.flag[buf][0] = cd;
                sh.flag[buf][1] = zh ? 1 : 0;
            }
        }
        __syncthreads();
        const int cd = sh.flag[buf][0];
        const bool zh = sh.flag[buf][1] != 0;
        if (wave > k) {
            // ---- U12 = L11^-1 A12 (four chunk products M_c A12[4c..4c+3],
            // each chunk reduced before it is used) and A22 <- A22 - L21 U12
            // for this column block
            const float *Mi = sh.pi[buf];
            const float *Lp = sh.pl[buf];
            auto update = [&](auto KK) __attribute__((always_inline)) {
                constexpr int K = decltype(KK)::value;
                float mi[4], la[NW][4];
#pragma unroll
                for (int c = 0; c < 4; ++c) mi[c] = Mi[lr * XS + 4 * c + lq];
#pragma unroll
                for (int b = K + 1; b < NW; ++b)
#pragma unroll
                    for (int c = 0; c < 4; ++c) la[b][c] = Lp[(16 * b + lr) * XS + 4 * c + lq];
                bc_v4d u = acc[K];
                u[0] = bc_sym(u[0], mod);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    u = __builtin_amdgcn_mfma_f64_16x16x4f64((double)mi[c], u[c], u, 0, 0, 0);
                    if (c < 3) u[c + 1] = bc_sym(u[c + 1], mod);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) u[v] = bc_sym(u[v], mod);
                acc[K] = u;
                if (red_each) {
#pragma unroll
                    for (int b = K + 1; b < NW; ++b)
#pragma unroll
                        for (int v = 0; v < 4; ++v) acc[b][v] = bc_sym(acc[b][v], mod);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) {
#pragma unroll
                    for (int b = K + 1; b < NW; ++b)
                        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)la[b][c], u[c], acc[b], 0, 0, 0);
                    if (c == 1 && red8) {
#pragma unroll
                        for (int b = K + 1; b < NW; ++b)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[b][v] = bc_sym(acc[b][v], mod);
                    }
                }
            };
            // the owner of the next panel goes first on its SIMD
            if (wave == k + 1) __builtin_amdgcn_s_setprio(2);
            switch (k) {
            case 0: update(std::integral_constant<int, 0>{}); break;
            case 1: if constexpr (NW > 1) update(std::integral_constant<int, 1>{}); break;
            case 2: if constexpr (NW > 2) update(std::integral_constant<int, 2>{}); break;
            case 3: if constexpr (NW > 3) update(std::integral_constant<int, 3>{}); break;
            case 4: if constexpr (NW > 4) update(std::integral_constant<int, 4>{}); break;
            case 5: if constexpr (NW > 5) update(std::integral_constant<int, 5>{}); break;
            case 6: if constexpr (NW > 6) update(std::integral_constant<int, 6>{}); break;
            default: break;
            }
            if (wave == k + 1) __builtin_amdgcn_s_setprio(0);
        }
        klast = k;
        if (zh || c0 + cd >= steps) {
            r = c0 + cd;
            zero_hit = zh;
            break;
        }
    }

    // The block left at (r, r) must be zero after a zero pivot (optimistic
    // attempt) or when fewer than min(m, n) steps were asked for.
    bool ok = !(zero_hit && r_known >= 0);
    const bool test = ok && (zero_hit || r < kmax);
    const bool rowlayout = wave <= klast;
    if (test) {
        int any = 0;
        if (rowlayout) {
#pragma unroll
            for (int h = 0; h < NH; ++h)
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const int i = lane + 64 * h, jg = 16 * wave + j;
                    if (i >= r && jg >= r && i < m && jg < n) any |= (bc_sym(RR(h, j), mod) != 0.0);
                }
        } else {
#pragma unroll
            for (int b = 0; b < NW; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * b + lq + 4 * v, jg = 16 * wave + lr;
                    if (i >= r && jg >= r && i < m && jg < n) any |= (bc_sym(acc[b][v], mod) != 0.0);
                }
        }
        ok = __syncthreads_or(any) == 0;
    } else {
        __syncthreads();   // every wave is past the table before it is overwritten
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
    // canonical residues into the LDS tile, then whole rows to A
    int32_t *out = (int32_t *)dyn;
    if (rowlayout) {
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int j = 0; j < 16; ++j) out[(lane + 64 * h) * OS + 16 * wave + j] = (int32_t)mod_reduce(RR(h, j), mod);
    } else {
#pragma unroll
        for (int b = 0; b < NW; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(16 * b + lq + 4 * v) * OS + 16 * wave + lr] = (int32_t)mod_reduce(acc[b][v], mod);
    }
#undef RR
    __syncthreads();
    constexpr int VE = 16 / (int)sizeof(T);   // elements per 16-byte store
    struct alignas(16) Vec { T x[VE]; };
    if (n == TILE && lda % VE == 0 && ((uintptr_t)A & 15) == 0) {
#pragma unroll
        for (int e = 0; e < TILE * TILE / VE / NT; ++e) {
            const int idx = (tid + NT * e) * VE;
            const int i = idx / TILE, j = idx % TILE;
            if (i < m) {
                Vec o;
#pragma unroll
                for (int q = 0; q < VE; ++q) o.x[q] = from_f64<T>((double)out[i * OS + j + q]);
                *(Vec *)&A[(int64_t)i * lda + j] = o;
            }
        }
    } else {
        for (int idx = tid; idx < m * n; idx += NT) {
            const int i = idx / n, j = idx - i * n;
            A[(int64_t)i * lda + j] = from_f64<T>((double)out[i * OS + j]);
        }
    }
    if (tid == 0) { status[0] = r; status[1] = 1; }
}

// Rank profile matrix of the tile: status[0] = r, status[1 + i] = pivot
// column of row i or -1.  Rows are processed in order; the pivot of row i is
// the first non-zero entry of the reduced row among the columns that are not
// yet pivot columns.  (Taken for non-generic tiles only.)  256 threads,
// thread (ty, tx) = (tid / 16, tid % 16) holding entries (ty + 16 a,
// tx + 16 b) in registers; rows run in blocks of 16 so that the row owners'
// register row is a compile-time index; each thread keeps the pivot columns
// among its own columns as a bit mask.  One barrier per row: the owners of
// row i reduce it and publish it (pivot and dead columns as 0) with their
// first non-zero column; after the barrier every thread finds the pivot
// column, reads the pivot and its inverse (LDS table when p <= 65536) itself,
// fetches column jc of its own rows from the lane of its 16-lane group that
// holds it (a within-wave shuffle of the register selected by the uniform
// index jc / 16), forms its multipliers, and applies the row with
// branch-free multiply-adds to its register rows of the current and later
// 16-row blocks (earlier blocks are finished; multipliers of rows <= i and
// published values of dead columns are 0).  Row i's values and first-column
// words are double-buffered by row parity, so the next row's owners can
// publish while the others still read.  The open rows are reduced
// (symmetric reduction) after every block of 16 rows, or after every pivot
// when RED1 (p close to 2^25).  A pivot row costs dependent latency more
// than arithmetic (the barrier, the first-column words, then the pivot and
// its inverse from LDS with the column shuffles issued in between, the
// multiplier chain), so the table is a compile-time choice (no branch
// between those steps) and the status store comes after the update.
template <typename T, bool RED1, bool TAB>
__global__ __launch_bounds__(BC_THREADS) void bc_rpm_kernel(const T *A, int64_t lda, int m, int n, ModP mod,
                                                            const uint16_t *gtab, int32_t *status) {
    constexpr int R = 8;
    extern __shared__ __align__(16) unsigned char dyn[];
    __shared__ double Ub[2][BC_DIM];
    __shared__ int mins[2][16];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const uint16_t *tab = nullptr;
    if (TAB) {
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
    bc_v8d v[R];   // v[a][b]: entry (ty + 16 a, tx + 16 b)
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
    // symmetric reduction of register blocks a0 .. R-1 (the rows still open)
    auto reduce_from = [&](auto A0) __attribute__((always_inline)) {
        constexpr int a0 = decltype(A0)::value;
#pragma unroll
        for (int a = a0; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b) v[a][b] = sym_reduce(v[a][b], mod);
    };
    // the first lane of this thread's 16-lane group (same ty) within the wave
    const int grp = tid & 48;
    auto row_step = [&](int i, auto AI) __attribute__((always_inline)) {
        constexpr int ai = decltype(AI)::value;
        const int buf = i & 1;
        if (ty == (i & 15)) {
            int first = 1 << 30;
#pragma unroll
            for (int b = 0; b < R; ++b) {
                const int j = tx + 16 * b;
                const bool live = j < n && !((dead >> b) & 1u);
                const double u = live ? sym_reduce(v[ai][b], mod) : 0.0;
                if (live) v[ai][b] = u;
                Ub[buf][j] = u;
                if (u != 0.0 && j < first) first = j;
            }
            mins[buf][tx] = first;
        }
        __syncthreads();
        int jc = 1 << 30;
#pragma unroll
        for (int t = 0; t < 16; ++t) jc = min(jc, mins[buf][t]);
        if (jc >= n) return;   // dependent row (uniform)
        ++r;
        const int bj = jc >> 4, sl = jc & 15;
        double pv = Ub[buf][jc];
        // column jc of rows ty + 16 a sits in lane grp + sl, register
        // v[a][bj]: fetched while the pivot and its inverse are read
        // (register blocks a < ai hold rows above row i, finished: skipped)
        const int bju = __builtin_amdgcn_readfirstlane(bj);
        double cs[R];
#pragma unroll
        for (int a = ai; a < R; ++a) cs[a] = __shfl(v[a][bju], grp + sl, 64);   // uniform index into the row's vector
        if (pv < 0.0) pv += mod.p;   // canonical, for the inverse
        double inv;
        if constexpr (TAB) inv = (double)tab[(int)pv];
        else inv = mod_inv(pv, mod);
        if (tx == sl) dead |= 1u << bj;
        double l[R];
#pragma unroll
        for (int a = ai; a < R; ++a) {
            const int k = ty + 16 * a;
            const double lv = sym_reduce(sym_reduce(cs[a], mod) * inv, mod);   // formed for every row: no branch
            l[a] = (k > i && k < m) ? lv : 0.0;
        }
        double u[R];
#pragma unroll
        for (int b = 0; b < R; ++b) u[b] = Ub[buf][tx + 16 * b];
#pragma unroll
        for (int a = ai; a < R; ++a)
#pragma unroll
            for (int b = 0; b < R; ++b) v[a][b] = fma(-l[a], u[b], v[a][b]);
        if (RED1) reduce_from(std::integral_constant<int, ai>{});
        if (tid == 0) status[1 + i] = jc;
        // Ub and mins of this row are read again only by threads that have
        // not yet passed the next row's barrier; the row after next rewrites
        // them after that barrier.
    };
#define PLUQ_RPM_BLOCK(K)                                                                         \
    {                                                                                             \
        const int ihi = (K) * 16 + 16 < m ? (K) * 16 + 16 : m;                                    \
        for (int i = (K) * 16; i < ihi; ++i) row_step(i, std::integral_constant<int, (K)>{});     \
        if (!RED1) reduce_from(std::integral_constant<int, (K) + 1 < R ? (K) + 1 : R>{});        \
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
    PLUQ_SETLDS((bc_lu_kernel<int64_t, 64, true>))
    PLUQ_SETLDS((bc_lu_kernel<double, 64, true>))
    PLUQ_SETLDS((bc_lu_kernel<int32_t, 64, true>))
    PLUQ_SETLDS((bc_lu_kernel<int64_t, 128, true>))
    PLUQ_SETLDS((bc_lu_kernel<double, 128, true>))
    PLUQ_SETLDS((bc_lu_kernel<int32_t, 128, true>))
    PLUQ_SETLDS((bc_rpm_kernel<int64_t, false, true>))
    PLUQ_SETLDS((bc_rpm_kernel<double, false, true>))
    PLUQ_SETLDS((bc_rpm_kernel<int32_t, false, true>))
#undef PLUQ_SETLDS
    hipError_t e = hipSuccess;
#define PLUQ_SETOUT(K)                                                                                 \
    if (e == hipSuccess)                                                                                \
        e = hipFuncSetAttribute((const void *)(K), hipFuncAttributeMaxDynamicSharedMemorySize, BC_OUT_BYTES);
    PLUQ_SETOUT((bc_lu_kernel<int64_t, 64, false>))
    PLUQ_SETOUT((bc_lu_kernel<double, 64, false>))
    PLUQ_SETOUT((bc_lu_kernel<int32_t, 64, false>))
    PLUQ_SETOUT((bc_lu_kernel<int64_t, 128, false>))
    PLUQ_SETOUT((bc_lu_kernel<double, 128, false>))
    PLUQ_SETOUT((bc_lu_kernel<int32_t, 128, false>))
#undef PLUQ_SETOUT
    if (e != hipSuccess) return e;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
        prop.sharedMemPerBlock < BC_TAB_BYTES + sizeof(BcBlkShared<BC_DIM>) + 1024)
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

template <int TILE, bool TAB>
static hipError_t bc_lu_t(int dtype, void *A, int64_t lda, int m, int n, const int32_t *rmap,
                          const int32_t *cmap, int r_known, double p, int kchunk, const uint16_t *tab,
                          int32_t *status, int32_t *specfail, int32_t *errflag, hipStream_t st) {
    // dynamic LDS: the table of inverses, later the staged result tile
    const size_t lds = TAB ? BC_TAB_BYTES : (size_t)BC_OUT_BYTES;
    const ModP md = make_mod(p);
    switch (dtype) {
    case DT_I64:
        PLUQ_LAUNCH((bc_lu_kernel<int64_t, TILE, TAB>), dim3(1), dim3(TILE * 4), lds, st, (int64_t *)A, lda, m, n,
                    rmap, cmap, r_known, md, kchunk, tab, status, specfail, errflag);
        break;
    case DT_F64:
        PLUQ_LAUNCH((bc_lu_kernel<double, TILE, TAB>), dim3(1), dim3(TILE * 4), lds, st, (double *)A, lda, m, n,
                    rmap, cmap, r_known, md, kchunk, tab, status, specfail, errflag);
        break;
    case DT_I32:
        PLUQ_LAUNCH((bc_lu_kernel<int32_t, TILE, TAB>), dim3(1), dim3(TILE * 4), lds, st, (int32_t *)A, lda, m, n,
                    rmap, cmap, r_known, md, kchunk, tab, status, specfail, errflag);
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
#define PLUQ_BC(TILE, TAB) bc_lu_t<TILE, TAB>(dtype, A, lda, m, n, rmap, cmap, r_known, p, kchunk, tab, status, specfail, errflag, st)
    if (m <= 64 && n <= 64) return tab ? PLUQ_BC(64, true) : PLUQ_BC(64, false);
    return tab ? PLUQ_BC(128, true) : PLUQ_BC(128, false);
#undef PLUQ_BC
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
    // red1 implies p > 65536: no table
#define PLUQ_RPM(TT)                                                                                     \
    if (red1)                                                                                            \
        PLUQ_LAUNCH((bc_rpm_kernel<TT, true, false>), dim3(1), dim3(BC_THREADS), 0, st, (const TT *)A, lda, m, n, \
                    md, nullptr, status);                                                                \
    else if (tab)                                                                                        \
        PLUQ_LAUNCH((bc_rpm_kernel<TT, false, true>), dim3(1), dim3(BC_THREADS), lds, st, (const TT *)A, lda, m, \
                    n, md, tab, status);                                                                 \
    else                                                                                                 \
        PLUQ_LAUNCH((bc_rpm_kernel<TT, false, false>), dim3(1), dim3(BC_THREADS), 0, st, (const TT *)A, lda, m, \
                    n, md, nullptr, status);
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

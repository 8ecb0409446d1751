// INT8-limb form of MM(C, A, B) (Section 2's Schur update), exact:
//     C <- C - sum_k A[i][k] B[k][j]   (mod p),   p <= 65536.
//
// Every operand a in [0, p) is moved into the window [-32896, 32639]
// (a itself when a <= 32639, else a - p) and written as two balanced signed
// base-256 digits, a = 256 d1 + d0 with d0, d1 in [-128, 127]; for p <= 256
// the window is [-128, 127] and one digit suffices.  The product then splits
// into limb products on the int8 matrix cores with int32 accumulation:
//     A.B = 2^16 S2 + 2^8 S1 + S0,
//     S0 = A0.B0,  S1 = A0.B1 + A1.B0,  S2 = A1.B1,
// where every term is at most 2^14 in magnitude, so for an inner dimension
// of at most KMAX_I8 = 16384 (one launch) |S1| <= 2^29 (int32 holds it) and
// the recombination 2^16 S2 + 2^8 S1 + S0 is below 2^45: it is formed
// exactly in float64,
// subtracted from C and reduced once per output (delayed reduction,
// Section 6).  Pivot inversion and everything outside MM stay in float64.
//
// Two kernels:
//   limb_split_kernel -- writes the digit planes of the operand blocks into
//     workspace, [rows][Kp] int8 with the inner dimension contiguous (B is
//     transposed on the way through LDS), zero-padded to a multiple of 64.
//   modmm_i8_kernel   -- 128 x 128 output tile per work-group: for two
//     digits 2 x 4 waves of 64 x 32 (2 x 1 blocks of v_mfma_i32_32x32x32_i8
//     per limb product; with the three limb sums a 64 x 64 wave tile would
//     leave one wave per SIMD), for one digit 2 x 2 waves of 64 x 64.
//     Updates with fewer than 1024 such tiles take 64 x 64 tiles of 2 x 2
//     waves of 32 x 32 instead, so that they still spread over the compute
//     units.  The planes are staged in LDS 64 bytes of K at a time (the four
//     16-byte chunks of a row permuted by an XOR of row bits, so that both
//     the fragment reads and the stores of a wave hit distinct banks); a
//     wave reads all fragments of a panel before its products.  With two
//     digits (and on the small tile) the panels are double-buffered: the
//     next panel's global loads are issued before the current panel's
//     matrix-core work and stored into the other buffer after it, so one
//     barrier per panel suffices.  Tiles are handed out XCD by XCD: the
//     work-groups that one XCD runs (hardware dispatch is round-robin over
//     the 8 XCDs) take a contiguous range of tiles in an order grouped by 8
//     tile rows, so that the A and B panels they share stay in that XCD's L2.
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int I8_GROUP = 8;   // tile rows per group of the tile order
// Tile shapes.  Large: 128 x 128, 8 waves of 64 x 32 (two digits) or 4 waves
// of 64 x 64 (one digit).  Small (SM): 64 x 64, 4 waves of 32 x 32, for
// updates whose 128 x 128 tiles would not fill the compute units.
__host__ __device__ constexpr int i8_tile(bool sm) { return sm ? 64 : 128; }
__host__ __device__ constexpr int i8_threads(int nl, bool sm) { return (nl == 2 && !sm) ? 512 : 256; }
__host__ __device__ constexpr int i8_blocks(int nl, bool sm) { return sm ? 2 : (nl == 2 ? 1 : 2); }
// below this many 128 x 128 tiles an update takes the 64 x 64 tiles
constexpr int64_t I8_SMALL_TILES = 1024;

// ------------------------------------------------------------------ split --

struct SplitArgs {
    SplitJob job[SPLIT_MAX_JOBS];
    int32_t count;
    int32_t thr;   // largest residue kept as is; larger ones become a - p
    ModP mod;
};

__device__ __forceinline__ int shifted(double a, int thr, double p) {
    return (int)((a > (double)thr) ? a - p : a);
}

__device__ __forceinline__ void digits(int v, int &d0, int &d1) {
    d0 = ((v + 128) & 255) - 128;
    d1 = (v - d0) >> 8;   // exact: v - d0 is a multiple of 256
}

// Row job: source rows x K, inner dimension contiguous (the A operand).
// Transposed job: source K x rows (the B operand, columns contiguous).  Both
// take a 64 x 64 tile per work-group through LDS so that both the reads and
// the plane writes are contiguous.
template <typename T, int NL>
__global__ __launch_bounds__(256) void limb_split_kernel(const SplitArgs args) {
    __shared__ int8_t tl[NL][64 * 68];
    int ji = 0;
#pragma unroll
    for (int q = 1; q < SPLIT_MAX_JOBS; ++q)
        if (q < args.count && (int)blockIdx.x >= args.job[q].blockStart) ji = q;
    const SplitJob &J = args.job[ji];
    const int b = blockIdx.x - J.blockStart;
    const T *X = (const T *)J.src;
    const double p = args.mod.p;
    const int thr = args.thr;
    const int tid = threadIdx.x;
    if (!J.trans) {
        // 64 rows x 64 inner positions per work-group: each load instruction
        // reads 64 consecutive entries of one row; the digits go to LDS
        // transposed (bytes of a row 68 apart, so the byte stores of a wave
        // hit distinct banks) and each thread writes 16 digits of one row
        const int tilesK = (int)(J.Kp / 64);
        const int r0 = (b / tilesK) * 64, kb = (b % tilesK) * 64;
#pragma unroll 4
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + 256 * e;
            const int rr = idx >> 6, kk = idx & 63;
            const int row = r0 + rr, k = kb + kk;
            const double a = (k < J.K && row < J.rows) ? to_f64(X[(int64_t)row * J.ld + k]) : 0.0;
            int d0, d1;
            digits(shifted(a, thr, p), d0, d1);
            tl[0][kk * 68 + rr] = (int8_t)d0;
            if (NL == 2) tl[NL - 1][kk * 68 + rr] = (int8_t)d1;
        }
        __syncthreads();
        const int rr = tid >> 2, c = (tid & 3) * 16;
        const int row = r0 + rr;
        if (row < J.rows) {
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                v4i w;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int8_t *s0 = &tl[l][(c + 4 * q) * 68 + rr];
                    w[q] = (int)((uint32_t)(uint8_t)s0[0] | ((uint32_t)(uint8_t)s0[68] << 8) |
                                 ((uint32_t)(uint8_t)s0[136] << 16) | ((uint32_t)(uint8_t)s0[204] << 24));
                }
                int8_t *d = (l == 0 ? J.dst0 : J.dst1) + (int64_t)row * J.ldd + kb + c;
                *(v4i *)d = w;
            }
        }
    } else {
        const int tilesK = (int)(J.Kp / 64);
        const int n0 = (b / tilesK) * 64, kb = (b % tilesK) * 64;
        // read 64 (k) x 64 (n) entries, n contiguous
#pragma unroll 4
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + 256 * e;
            const int kk = idx >> 6, nn = idx & 63;
            const int k = kb + kk, n = n0 + nn;
            const double a = (k < J.K && n < J.rows) ? to_f64(X[(int64_t)k * J.ld + n]) : 0.0;
            int d0, d1;
            digits(shifted(a, thr, p), d0, d1);
            tl[0][nn * 68 + kk] = (int8_t)d0;
            if (NL == 2) tl[NL - 1][nn * 68 + kk] = (int8_t)d1;
        }
        __syncthreads();
        const int nn = tid >> 2, c = (tid & 3) * 16;
        const int n = n0 + nn;
        if (n < J.rows) {
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                const int8_t *s = &tl[l][nn * 68 + c];
                v4i w;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    w[q] = (int)((uint32_t)(uint8_t)s[4 * q] | ((uint32_t)(uint8_t)s[4 * q + 1] << 8) |
                                 ((uint32_t)(uint8_t)s[4 * q + 2] << 16) | ((uint32_t)(uint8_t)s[4 * q + 3] << 24));
                int8_t *d = (l == 0 ? J.dst0 : J.dst1) + (int64_t)n * J.ldd + kb + c;
                *(v4i *)d = w;
            }
        }
    }
}

template <typename T, int NL>
static hipError_t split_t(SplitArgs &a, int total, hipStream_t st) {
    PLUQ_LAUNCH((limb_split_kernel<T, NL>), dim3(total), dim3(256), 0, st, a);
    return hipGetLastError();
}

template <int NL>
static hipError_t split_dt(int dtype, SplitArgs &a, int total, hipStream_t st) {
    switch (dtype) {
    case DT_I64: return split_t<int64_t, NL>(a, total, st);
    case DT_F64: return split_t<double, NL>(a, total, st);
    case DT_I32: return split_t<int32_t, NL>(a, total, st);
    }
    return hipErrorInvalidValue;
}

int i8_limbs(double p) { return p <= 256.0 ? 1 : (p <= 65536.0 ? 2 : 0); }

hipError_t launch_limb_split(int dtype, SplitJob *jobs, int njobs, double p, hipStream_t st) {
    const int nl = i8_limbs(p);
    if (nl == 0 || njobs <= 0 || njobs > SPLIT_MAX_JOBS) return hipErrorInvalidValue;
    SplitArgs a;
    a.count = njobs;
    a.thr = nl == 1 ? 127 : 32639;
    a.mod.p = p;
    a.mod.pinv = 1.0 / p;
    a.mod.half = (double)((int64_t)p / 2);
    int total = 0;
    for (int q = 0; q < njobs; ++q) {
        SplitJob &J = jobs[q];
        if (J.Kp % 64 || J.ldd % 16 || J.K > J.Kp) return hipErrorInvalidValue;
        J.blockStart = total;
        const int64_t blocks = cdiv64(J.rows, 64) * (J.Kp / 64);
        total += (int)blocks;
        a.job[q] = J;
    }
    if (total == 0) return hipSuccess;
    return nl == 1 ? split_dt<1>(dtype, a, total, st) : split_dt<2>(dtype, a, total, st);
}

// ------------------------------------------------------------------- GEMM --

struct I8Args {
    void *C;
    int64_t ldc;
    int32_t M, N, Kp, tilesN;
    const int8_t *a[2];
    const int8_t *b[2];
    int64_t lda, ldb;   // bytes between plane rows
    int32_t *nzflag;
    int32_t nzgen;
    ModP mod;
};

// Position of 16-byte chunk c of plane row `row` inside its 64-byte LDS row:
// c ^ (2 b2 + (b1 ^ b3)) with b_k bit k of the row.  The fragment reads (8 or
// 16 consecutive lanes on consecutive rows, one chunk) and the stores (2 or
// 4 consecutive rows, all four chunks) then fall on distinct banks, whether
// a 16-byte access is served 8 lanes at a time over 32 banks or 16 lanes at
// a time over 64.
__device__ __forceinline__ int i8_swz(int row, int c) {
    return (c ^ (((row >> 1) ^ (row >> 3)) & 1) ^ (row & 4) >> 1) * 16;
}

template <typename T, int NL, bool SM>
__global__ __launch_bounds__(i8_threads(NL, SM), i8_blocks(NL, SM)) void modmm_i8_kernel(const I8Args g) {
    constexpr int BM = i8_tile(SM), BN = i8_tile(SM), BK = 64, LDP = BK;
    constexpr int NS = NL == 2 ? 3 : 1;                // limb sums S0 (, S1, S2)
    constexpr int IB = SM ? 1 : 2;                     // 32-row blocks per wave
    constexpr int JB = (SM || NL == 2) ? 1 : 2;        // 32-column blocks per wave
    constexpr int NT = i8_threads(NL, SM), WN = BN / (32 * JB), RPTA = BM / (NT / 4), RPTB = BN / (NT / 4);
    // double-buffered panels for two digits and for the small tile; one
    // digit on the large tile keeps a single buffer (two barriers per
    // panel), which keeps two work-groups per compute unit
    constexpr bool DB = NL == 2 || SM;
    constexpr int NB = DB ? 2 : 1;
    __shared__ __attribute__((aligned(16))) int8_t As[NB][NL][BM * LDP];
    __shared__ __attribute__((aligned(16))) int8_t Bs[NB][NL][BN * LDP];

    // work-group -> tile: XCD x = blockIdx % 8 runs a contiguous range of
    // the tile order, which walks groups of I8_GROUP tile rows column by
    // column (a bijection onto [0, tiles) for any count)
    const int tiles = (int)gridDim.x, tilesN = g.tilesN, tilesM = tiles / tilesN;
    const int xcd = (int)blockIdx.x % 8, q = (int)blockIdx.x / 8;
    const int per = tiles / 8, rem = tiles % 8;
    const int t = xcd * per + min(xcd, rem) + q;
    const int gsz = I8_GROUP * tilesN, grp = t / gsz;
    const int gr0 = grp * I8_GROUP, grows = min(tilesM - gr0, I8_GROUP);
    const int tr = gr0 + (t - grp * gsz) % grows, tc = (t - grp * gsz) / grows;
    const int row0 = tr * BM, col0 = tc * BN;
    const int M = g.M, N = g.N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm0 = (wave / WN) * 32 * IB, wn0 = (wave % WN) * 32 * JB;

    v16i acc[NS][IB][JB];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int i = 0; i < IB; ++i)
#pragma unroll
            for (int j = 0; j < JB; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[s][i][j][v] = 0;

    // Global loads: 16 bytes per thread, plane and row, plane rows
    // tid/4 + r NT/4 (r < RPTA for A, RPTB for B), chunk tid%4.  Rows past M (N) are clamped
    // to the last valid row: their products only reach outputs that are
    // never stored.
    const int lr = tid >> 2, lc = (tid & 3) * 16;
    int64_t ar[RPTA], br[RPTB];
#pragma unroll
    for (int r = 0; r < RPTA; ++r) ar[r] = (int64_t)min(row0 + lr + r * (NT / 4), M - 1) * g.lda + lc;
#pragma unroll
    for (int r = 0; r < RPTB; ++r) br[r] = (int64_t)min(col0 + lr + r * (NT / 4), N - 1) * g.ldb + lc;
    v4i pa[NL][RPTA], pb[NL][RPTB];
    auto load = [&](int k0) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
#pragma unroll
            for (int r = 0; r < RPTA; ++r) pa[l][r] = *(const v4i *)(g.a[l] + ar[r] + k0);
#pragma unroll
            for (int r = 0; r < RPTB; ++r) pb[l][r] = *(const v4i *)(g.b[l] + br[r] + k0);
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
#pragma unroll
            for (int r = 0; r < RPTA; ++r) {
                const int row = lr + r * (NT / 4);
                *(v4i *)&As[buf][l][row * LDP + i8_swz(row, lc >> 4)] = pa[l][r];
            }
#pragma unroll
            for (int r = 0; r < RPTB; ++r) {
                const int row = lr + r * (NT / 4);
                *(v4i *)&Bs[buf][l][row * LDP + i8_swz(row, lc >> 4)] = pb[l][r];
            }
        }
    };

    const int steps = g.Kp / BK;
    if (DB && steps > 0) {
        load(0);
        stash(0);
    }
    if (!DB && steps > 0) load(0);
    if (DB) __syncthreads();
    for (int s = 0; s < steps; ++s) {
        const int buf = DB ? (s & 1) : 0;
        if (!DB) {
            __syncthreads();
            stash(0);
            __syncthreads();
        }
        // next panel in flight during this one's products; with two
        // buffers it is stored into the other one, which every wave
        // finished reading before the barrier that ended the previous step
        if (s + 1 < steps) load((s + 1) * BK);
        // All fragments of the panel are read before the first product
        // (v_mfma_i32_32x32x32_i8: lane holds row (A) / column (B) lane%32
        // and inner indices 16*(lane/32) .. +15 of a 32-deep step), so the
        // LDS latency is paid once per panel rather than between products.
        v4i fa[2][NL][IB], fb[2][NL][JB];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int kc = ks * 2 + (lane >> 5);   // 16-byte chunk of the 64-deep panel
#pragma unroll
            for (int l = 0; l < NL; ++l) {
#pragma unroll
                for (int i = 0; i < IB; ++i) {
                    const int row = wm0 + 32 * i + (lane & 31);
                    fa[ks][l][i] = *(const v4i *)&As[buf][l][row * LDP + i8_swz(row, kc)];
                }
#pragma unroll
                for (int j = 0; j < JB; ++j) {
                    const int row = wn0 + 32 * j + (lane & 31);
                    fb[ks][l][j] = *(const v4i *)&Bs[buf][l][row * LDP + i8_swz(row, kc)];
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < JB; ++j) {
                auto mfma = [&](int sidx, int i, int la, int lb) __attribute__((always_inline)) {
                    acc[sidx][i][j] =
                        __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[ks][la][i], fb[ks][lb][j], acc[sidx][i][j], 0, 0, 0);
                };
                if (NL == 2) {
                    // the two products into S1 of a block are IB + 1
                    // products apart
#pragma unroll
                    for (int i = 0; i < IB; ++i) {
                        mfma(0, i, 0, 0);
                        mfma(NS - 2, i, 0, NL - 1);
                    }
#pragma unroll
                    for (int i = 0; i < IB; ++i) {
                        mfma(NS - 1, i, NL - 1, NL - 1);
                        mfma(NS - 2, i, NL - 1, 0);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < IB; ++i) mfma(0, i, 0, 0);
                }
            }
        if (DB) {
            if (s + 1 < steps) stash(buf ^ 1);
            __syncthreads();
        }
    }

    // Epilogue: element v of a 32 x 32 block sits at row
    // 8*(v/4) + 4*(lane/32) + v%4 and column lane%32.  A block's 16 C
    // entries are loaded before any is used (clamped addresses), so those
    // loads are in flight together.
    const ModP mod = g.mod;
    T *C = (T *)g.C;
    bool nz = false;
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
        for (int i = 0; i < IB; ++i) {
            const int gc = col0 + wn0 + 32 * j + (lane & 31);
            double cv[16];
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int gr = row0 + wm0 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                cv[v] = to_f64(C[(int64_t)min(gr, M - 1) * g.ldc + min(gc, N - 1)]);
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int gr = row0 + wm0 + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                double t = (double)acc[0][i][j][v];
                if (NL == 2) t += 256.0 * (double)acc[NS - 2][i][j][v] + 65536.0 * (double)acc[NS - 1][i][j][v];
                if (gr < M && gc < N) {
                    const double x = mod_reduce(cv[v] - t, mod);
                    C[(int64_t)gr * g.ldc + gc] = from_f64<T>(x);
                    nz |= (x != 0.0);
                }
            }
        }
    if (nz && g.nzflag) *g.nzflag = g.nzgen;
}

template <typename T, int NL, bool SM>
static hipError_t i8_t(I8Args &a, int total, hipStream_t st) {
    PLUQ_LAUNCH((modmm_i8_kernel<T, NL, SM>), dim3(total), dim3(i8_threads(NL, SM)), 0, st, a);
    return hipGetLastError();
}

template <int NL, bool SM>
static hipError_t i8_dt(int dtype, I8Args &a, int total, hipStream_t st) {
    switch (dtype) {
    case DT_I64: return i8_t<int64_t, NL, SM>(a, total, st);
    case DT_F64: return i8_t<double, NL, SM>(a, total, st);
    case DT_I32: return i8_t<int32_t, NL, SM>(a, total, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_modmm_i8(int dtype, void *C, int64_t ldc, int M, int N, int Kp, const int8_t *const a[2],
                           const int8_t *const b[2], int64_t lda, int64_t ldb, double p, int32_t *nzflag,
                           int32_t nzgen, hipStream_t st) {
    const int nl = i8_limbs(p);
    if (nl == 0 || Kp % 64 || Kp > KMAX_I8 || lda % 16 || ldb % 16) return hipErrorInvalidValue;
    if (M <= 0 || N <= 0) return hipSuccess;
    I8Args g;
    g.C = C;
    g.ldc = ldc;
    g.M = M;
    g.N = N;
    g.Kp = Kp;
    const bool sm = cdiv64(M, 128) * cdiv64(N, 128) < I8_SMALL_TILES;
    const int tile = sm ? i8_tile(true) : i8_tile(false);
    g.tilesN = (int)cdiv64(N, tile);
    g.a[0] = a[0];
    g.a[1] = nl == 2 ? a[1] : a[0];
    g.b[0] = b[0];
    g.b[1] = nl == 2 ? b[1] : b[0];
    g.lda = lda;
    g.ldb = ldb;
    g.nzflag = nzflag;
    g.nzgen = nzgen;
    g.mod.p = p;
    g.mod.pinv = 1.0 / p;
    g.mod.half = (double)((int64_t)p / 2);
    const int total = (int)(cdiv64(M, tile) * g.tilesN);
    if (sm) return nl == 1 ? i8_dt<1, true>(dtype, g, total, st) : i8_dt<2, true>(dtype, g, total, st);
    return nl == 1 ? i8_dt<1, false>(dtype, g, total, st) : i8_dt<2, false>(dtype, g, total, st);
}

}  // namespace pluq

// MM(C, A, B) of Section 2 on the float64 matrix cores of gfx950:
//     C <- C - sum_s A_s B_s  (mod p)
// for up to four independent problems per launch (the Schur updates of one
// recursion level are issued together), each with up to two operand pairs
// accumulated into the same output (R <- H4 - K V2 - M3 O is one problem).
//
// Exactness: operands are mapped to symmetric residues |a| <= p/2, so each
// product is at most (p/2)^2 and a sum of `kchunk` of them plus a reduced
// residue stays below 2^52: every partial sum is an exactly representable
// integer whatever the summation order inside the matrix core.  The
// accumulator starts from C (loaded when the kernel starts, so no dependent
// read is left for the end), A is negated on load, the accumulator is reduced
// once per kchunk terms (delayed reduction, Section 6) and once before the
// store.  kchunk is at least 16 but may be below the panel depth BK (p near
// 2^25 in float64, p above about 2^10 in float32): the RED16 instances then
// reduce after every 16 products, at fixed points inside the panel.
//
// Tiling: the 128 x 128 tile runs 512 threads = 8 waves in a 2 x 4 grid,
// each wave owning a 64 x 32 sub-tile (two waves per SIMD; a 64 x 64 wave
// tile's accumulators would leave one), with double-buffered panels and one
// barrier per panel; the smaller tiles run 256 threads = 4 waves in a 2 x 2
// grid with one panel buffer.  Sub-tiles are made of 16 x 16 blocks computed
// with v_mfma_f64_16x16x4_f64.  Panels of depth BK are staged in LDS (A
// row-major, B row-major, both padded); global loads are lane-contiguous row
// segments; the next panel is fetched into registers while the current one is
// used.  64 x 64 and 32 x 32 tiles use BK = 64, so an update with K <= 64
// (the deep Schur updates) needs a single load phase.
//
// The same kernel in float32 (CT = float, v_mfma_f32_16x16x4_f32) is the
// FP32 form for small moduli: a float32 sum of integers is exact while it
// stays below 2^24, so with |a| <= p/2 at most kchunk32 = (2^24 - p) / (p/2)^2
// products (1072 for p = 251) are accumulated between reductions, which are
// done in float64.
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int MM_GROUP = 8;   // tile rows per group of the tile order

// Accumulator vector and output-row layout of the matrix-core instruction
// used for compute type CT.  Lane `lane` holds, in element v of its 16 x 16
// block, row row(lane, v) and column lane % 16.
template <typename CT> struct MfmaTraits;
template <> struct MfmaTraits<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
    static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct MfmaTraits<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
    static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

struct MMArgs {
    MMProblem prob[MM_MAX_PROBLEMS];
    int32_t count;
    int32_t kchunk;
    ModP mod;
};

// NTH threads: 2 x (NTH / 128) waves, each owning a (BM / 2) x (BN / (NTH /
// 128)) sub-tile.  DB: the A and B panels are double-buffered in LDS (one
// barrier per panel: the next panel is stored into the other buffer after
// the current one's products); otherwise one buffer and two barriers.
template <typename T, typename CT, int BM, int BN, int BK, bool RED16, int NTH, bool DB>
__global__ __launch_bounds__(NTH) void modmm_kernel(const MMArgs args) {
    typedef MfmaTraits<CT> MT;
    constexpr int WNW = NTH / 128;            // waves along N
    constexpr int WM = BM / 2, WN = BN / WNW;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int ELA = BM * BK / NTH;   // A elements loaded per thread and panel
    constexpr int ELB = BN * BK / NTH;   // B elements loaded per thread and panel
    // LDS row strides (elements) that keep the fragment reads free of bank
    // conflicts (32 banks of 4 bytes; a 64-lane read of 4-byte words is
    // served 32 lanes at a time, of 8-byte words 16 at a time): float64
    // needs an odd A stride, float32 an A stride of 2 and a B stride of 16
    // modulo 32 (lanes 0-15 and 16-31 read two consecutive inner indices).
    constexpr int PA = sizeof(CT) == 4 ? BK + 2 : BK + 1;
    constexpr int PB = sizeof(CT) == 4 ? BN + 16 : BN + 1;
    constexpr int NB = DB ? 2 : 1;
    static_assert(FN >= 1 && ELA >= 1 && ELB >= 1 && ELA <= 32 && ELB <= 32, "tile shape");
    __shared__ CT As[NB][BM * PA];
    __shared__ CT Bs[NB][BK * PB];

    // work-group -> tile: the work-groups one XCD runs (dispatch is
    // round-robin over the 8 XCDs) take a contiguous range of the launch's
    // tiles, and within a problem the tiles go in groups of MM_GROUP tile
    // rows, column by column, so the A and B panels that tiles running
    // together share stay in one XCD's L2 (a bijection for any tile count)
    const int tiles = (int)gridDim.x;
    const int xcd = (int)blockIdx.x % 8, qx = (int)blockIdx.x / 8;
    const int tile = xcd * (tiles / 8) + min(xcd, tiles % 8) + qx;
    int pi = 0;
#pragma unroll
    for (int q = 1; q < MM_MAX_PROBLEMS; ++q)
        if (q < args.count && tile >= args.prob[q].tileStart) pi = q;
    const MMProblem &P = args.prob[pi];
    const ModP mod = args.mod;
    const int M = P.M, N = P.N;
    const int t = tile - P.tileStart, tilesN = P.tilesN, tilesM = (M + BM - 1) / BM;
    const int gsz = MM_GROUP * tilesN, grp = t / gsz;
    const int gr0 = grp * MM_GROUP, grows = min(tilesM - gr0, MM_GROUP);
    const int row0 = (gr0 + (t - grp * gsz) % grows) * BM;
    const int col0 = ((t - grp * gsz) / grows) * BN;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm0 = (wave / WNW) * WM;
    const int wn0 = (wave % WNW) * WN;

    // accumulator <- C (canonical).
    T *C = (T *)P.C;
    typename MT::acc_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = row0 + wm0 + i * 16 + MT::row(lane, v);
                const int gc = col0 + wn0 + j * 16 + (lane & 15);
                acc[i][j][v] = (CT)to_f64(C[(int64_t)min(gr, M - 1) * P.ldc + min(gc, N - 1)]);
            }

    static_assert(BK % 16 == 0, "RED16 reduces at multiples of 16 products");
    const int K0 = P.K[0], K1 = P.K[1];
    const int steps0 = (K0 + BK - 1) / BK;
    const int steps = steps0 + (K1 + BK - 1) / BK;

    // Panel loads are branch-free: addresses are clamped into the operand (so
    // every load is valid) and out-of-range entries are masked to zero when
    // the raw values are converted, at the LDS store of the next iteration.
    // The loads of panel s+1 are thus all in flight during panel s's MFMAs.
    T ra[ELA], rb[ELB];
    uint32_t ma = 0, mb = 0;   // validity bit per loaded element
    auto load_step = [&](int s) {
        const int pair = (s < steps0) ? 0 : 1;
        const int k0 = (pair == 0 ? s : s - steps0) * BK;
        const int K = pair == 0 ? K0 : K1;
        const T *A = (const T *)P.A[pair];
        const T *B = (const T *)P.B[pair];
        const int64_t lda = P.lda[pair], ldb = P.ldb[pair];
        ma = 0;
        mb = 0;
#pragma unroll
        for (int e = 0; e < ELA; ++e) {
            const int idx = tid + NTH * e;
            const int gr = row0 + idx / BK, gk = k0 + idx % BK;
            ma |= (uint32_t)(gr < M && gk < K) << e;
            ra[e] = A[(int64_t)min(gr, M - 1) * lda + min(gk, K - 1)];
        }
#pragma unroll
        for (int e = 0; e < ELB; ++e) {
            const int idx = tid + NTH * e;
            const int gk = k0 + idx / BN, gc = col0 + idx % BN;
            mb |= (uint32_t)(gk < K && gc < N) << e;
            rb[e] = B[(int64_t)min(gk, K - 1) * ldb + min(gc, N - 1)];
        }
    };
    // the loaded panel, converted (A negated), into LDS buffer buf
    auto stash = [&](int buf) {
#pragma unroll
        for (int e = 0; e < ELA; ++e) {
            const int idx = tid + NTH * e;
            const CT v = (CT)-to_sym(to_f64(ra[e]), mod);
            As[buf][(idx / BK) * PA + idx % BK] = ((ma >> e) & 1u) ? v : (CT)0;
        }
#pragma unroll
        for (int e = 0; e < ELB; ++e) {
            const int idx = tid + NTH * e;
            const CT v = (CT)to_sym(to_f64(rb[e]), mod);
            Bs[buf][(idx / BN) * PB + idx % BN] = ((mb >> e) & 1u) ? v : (CT)0;
        }
    };

    auto reduce_acc = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[i][j][v] = (CT)mod_reduce((double)acc[i][j][v], mod);
    };

    int kacc = 0;
    auto compute = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            CT a[FM], b[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) a[i] = As[buf][(wm0 + i * 16 + (lane & 15)) * PA + kr];
#pragma unroll
            for (int j = 0; j < FN; ++j) b[j] = Bs[buf][kr * PB + wn0 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = MT::mfma(a[i], b[j], acc[i][j]);
            // 16 products since the last reduction: at most kchunk
            if (RED16 && (ks & 3) == 3) reduce_acc();
        }
    };
    if (DB) {
        if (steps > 0) {
            load_step(0);
            stash(0);
        }
        __syncthreads();
        for (int s = 0; s < steps; ++s) {
            const int buf = s & 1;
            // the next panel's loads are in flight during this one's
            // products; it goes into the other buffer, which every wave
            // finished reading before the barrier that ended the last step
            if (s + 1 < steps) load_step(s + 1);
            if (!RED16 && kacc + BK > args.kchunk) {
                reduce_acc();
                kacc = 0;
            }
            compute(buf);
            kacc += BK;
            if (s + 1 < steps) stash(buf ^ 1);
            __syncthreads();
        }
    } else {
        if (steps > 0) load_step(0);
        for (int s = 0; s < steps; ++s) {
            __syncthreads();
            stash(0);
            __syncthreads();
            if (s + 1 < steps) load_step(s + 1);
            if (!RED16 && kacc + BK > args.kchunk) {
                reduce_acc();
                kacc = 0;
            }
            compute(0);
            kacc += BK;
        }
    }

    bool nz = false;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gr = row0 + wm0 + i * 16 + MT::row(lane, v);
                const int gc = col0 + wn0 + j * 16 + (lane & 15);
                if (gr < M && gc < N) {
                    const double x = mod_reduce((double)acc[i][j][v], mod);
                    C[(int64_t)gr * P.ldc + gc] = from_f64<T>(x);
                    nz |= (x != 0.0);
                }
            }
    if (nz && P.nzflag) *P.nzflag = P.nzgen;
}

template <typename T, typename CT, int BM, int BN, int BK, int NTH, bool DB>
static hipError_t launch_t(MMArgs &args, int total, hipStream_t st) {
    if (args.kchunk < BK)
        PLUQ_LAUNCH((modmm_kernel<T, CT, BM, BN, BK, true, NTH, DB>), dim3(total), dim3(NTH), 0, st, args);
    else
        PLUQ_LAUNCH((modmm_kernel<T, CT, BM, BN, BK, false, NTH, DB>), dim3(total), dim3(NTH), 0, st, args);
    return hipGetLastError();
}

// The large tile runs 8 waves of 64 x 32 with double-buffered panels: a
// 64 x 64 wave tile's accumulators leave one wave per SIMD, with nothing to
// cover the barriers and load waits; the small tiles keep 4 waves.
template <typename T, typename CT>
static hipError_t launch_dt(MMArgs &args, int bm, int bn, int total, hipStream_t st) {
    if (bm == 128) return launch_t<T, CT, 128, 128, 32, 512, true>(args, total, st);
    if (bm == 64 && bn == 64) return launch_t<T, CT, 64, 64, 64, 256, false>(args, total, st);
    if (bm == 64) return launch_t<T, CT, 64, 32, 64, 256, false>(args, total, st);
    if (bn == 64) return launch_t<T, CT, 32, 64, 64, 256, false>(args, total, st);
    return launch_t<T, CT, 32, 32, 64, 256, false>(args, total, st);
}

template <typename CT>
static hipError_t launch_modmm(int dtype, MMProblem *probs, int nprob, double p, int kchunk, int t128, int t64,
                               hipStream_t st) {
    if (kchunk < 16 || kchunk % 16) return hipErrorInvalidValue;   // RED16 covers 16 products at a time
    MMArgs args;
    int n = 0;
    int64_t tiles128 = 0, tiles64 = 0;
    int inplace = 0;   // bit 0: some C is its B operand, bit 1: some C is its A operand
    for (int q = 0; q < nprob; ++q) {
        if (probs[q].M <= 0 || probs[q].N <= 0) continue;
        if ((probs[q].inplace == 1 && probs[q].M > 64) || (probs[q].inplace == 2 && probs[q].N > 64) ||
            probs[q].inplace < 0 || probs[q].inplace > 2)
            return hipErrorInvalidValue;
        args.prob[n++] = probs[q];
        tiles128 += cdiv64(probs[q].M, 128) * cdiv64(probs[q].N, 128);
        tiles64 += cdiv64(probs[q].M, 64) * cdiv64(probs[q].N, 64);
        if (probs[q].inplace) inplace |= 1 << (probs[q].inplace - 1);
    }
    if (n == 0) return hipSuccess;
    // Large updates use 128 x 128 tiles; smaller ones 64 x 64, and the small
    // updates of the deep recursion (fewer 64-tiles than compute units) 32 x
    // 32, so that more compute units share their matrix-core work (the tile
    // counts where the choice changes are tuned, 240 and 192 by default).  An
    // in-place update keeps 64 along the dimension it shares with C.
    int bm, bn;
    if (tiles128 >= t128) bm = bn = 128;
    else if (tiles64 >= t64 || inplace == 3) bm = bn = 64;
    else {
        bm = (inplace & 1) ? 64 : 32;
        bn = (inplace & 2) ? 64 : 32;
    }
    int total = 0;
    for (int q = 0; q < n; ++q) {
        MMProblem &pb = args.prob[q];
        pb.tileStart = total;
        pb.tilesN = (int)cdiv64(pb.N, bn);
        total += (int)(cdiv64(pb.M, bm) * pb.tilesN);
        if (pb.K[0] <= 0) pb.K[0] = 0;
        if (pb.K[1] <= 0) pb.K[1] = 0;
    }
    args.count = n;
    args.kchunk = kchunk;
    args.mod.p = p;
    args.mod.pinv = 1.0 / p;
    args.mod.half = (double)((int64_t)p / 2);
    switch (dtype) {
    case DT_I64: return launch_dt<int64_t, CT>(args, bm, bn, total, st);
    case DT_F64: return launch_dt<double, CT>(args, bm, bn, total, st);
    case DT_I32: return launch_dt<int32_t, CT>(args, bm, bn, total, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_modmm_f64(int dtype, MMProblem *probs, int nprob, double p, int kchunk, int t128, int t64,
                            hipStream_t st) {
    return launch_modmm<double>(dtype, probs, nprob, p, kchunk, t128, t64, st);
}

hipError_t launch_modmm_f32(int dtype, MMProblem *probs, int nprob, double p, int kchunk, int t128, int t64,
                            hipStream_t st) {
    return launch_modmm<float>(dtype, probs, nprob, p, kchunk, t128, t64, st);
}

}  // namespace pluq

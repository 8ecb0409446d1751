// Host-side launchers of the HIP kernels (implemented in k_*.hip).  Each
// launcher is asynchronous on the given stream and returns the
// hipGetLastError() of its launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pluq {

// One matrix-multiply update C <- C - sum_s A_s B_s (mod p), s < npairs.
// Pointers are element pointers (already offset to the block); all operands
// share the element type of the launch.
struct MMProblem {
    void *C;
    const void *A[2];
    const void *B[2];
    int64_t ldc;
    int64_t lda[2];
    int64_t ldb[2];
    int32_t K[2];
    int32_t M, N;
    int32_t *nzflag;   // if non-null: set to nzgen when an output element is non-zero
    int32_t nzgen;
    int32_t inplace;   // C is also an operand (an in-place product such as
                       // B <- B - W.B): 1 = C is the B operand (M <= 64),
                       // 2 = C is the A operand (N <= 64).  The tile then
                       // spans all of M (or N), so no work-group writes what
                       // another reads.  (The solves now use their own leaf
                       // kernel; the mode stays available.)
    int32_t tileStart; // filled by the launcher
    int32_t tilesN;    // filled by the launcher
};

constexpr int MM_MAX_PROBLEMS = 4;

// FP64 matrix-core form.  kchunk: number of inner-dimension terms that may
// be accumulated before a reduction (multiple of 16, >= 16).  t128 / t64:
// the launch takes 128 x 128 tiles from t128 such tiles on, else 64 x 64
// from t64 on, else 32 x 32 (tuning only).
hipError_t launch_modmm_f64(int dtype, MMProblem *probs, int nprob, double p, int kchunk, int t128, int t64,
                            hipStream_t st);
// FP32 matrix-core form (p < 2^11): kchunk products between reductions,
// kchunk * (p/2)^2 + p < 2^24.
hipError_t launch_modmm_f32(int dtype, MMProblem *probs, int nprob, double p, int kchunk, int t128, int t64,
                            hipStream_t st);

// INT8-limb form (p <= 65536).  Number of signed 8-bit digits per operand
// (1 for p <= 256, 2 for p <= 65536, 0 when the form cannot be exact).
int i8_limbs(double p);
// One block of digit planes to produce: the source block is rows x K
// (trans = 0, inner dimension contiguous: an A operand) or K x rows
// (trans = 1, a B operand); the planes dst0 / dst1 are [rows][ldd] int8 and
// receive columns [0, Kp) (Kp a multiple of 64; entries k >= K are zero).
struct SplitJob {
    const void *src;
    int64_t ld;
    int32_t rows, K, Kp, trans;
    int8_t *dst0, *dst1;
    int64_t ldd;
    int32_t blockStart;   // filled by the launcher
};
constexpr int SPLIT_MAX_JOBS = 4;
// inner dimension of one INT8 launch: the middle limb sum, at most
// 2 KMAX_I8 2^14 in magnitude, must fit int32
constexpr int KMAX_I8 = 16384;
hipError_t launch_limb_split(int dtype, SplitJob *jobs, int njobs, double p, hipStream_t st);
// C (M x N, ldc) <- C - sum over the Kp inner positions of the digit planes
// a (M rows of lda bytes) and b (N rows of ldb bytes), mod p; nzflag as in
// MMProblem.  Kp <= KMAX_I8, a multiple of 64.
hipError_t launch_modmm_i8(int dtype, void *C, int64_t ldc, int M, int N, int Kp, const int8_t *const a[2],
                           const int8_t *const b[2], int64_t lda, int64_t ldb, double p, int32_t *nzflag,
                           int32_t nzgen, hipStream_t st);

// Batched form: one descriptor per matrix (m, n <= BATCH_MAX_DIM).  W is the
// backup copy of the matrix (m x n dense, at wbase + woff); R receives the
// rank (-1 when a self-check fails).
constexpr int BATCH_MAX_DIM = 512;
struct BatchDesc {
    void *A;
    int64_t lda;
    int64_t *P, *Q, *R;
    int64_t woff;
    int32_t m, n;
};
// kb: panel width (8 or 16); grid: persistent work-groups.
hipError_t launch_batched_pluq(int dtype, int kb, const BatchDesc *desc, int32_t batch, char *wbase,
                               double p, int grid, hipStream_t st);

// Inverses of the 64 x 64 diagonal blocks of an r x r triangle (side 0:
// unit lower, side 1: upper non-unit), written as I - T_qq^{-1} (canonical,
// row-major, leading dimension 64) at W + q * 64 * 64.
constexpr int TRSM_NB = 64;
hipError_t launch_trsm_diag_inv(int dtype, int side, const void *T, int64_t ldt, int64_t r, void *W,
                                double p, int kchunk, hipStream_t st);

// Leaf solve of order r <= TRSM_FUSE_MAX in one launch, with the diagonal
// blocks' W = I - T_qq^{-1} from launch_trsm_diag_inv (W points at block 0
// of this triangle).  side 0: B (r x nst, ldb) <- L^{-1} B, L unit lower;
// side 1: B (nst x r, ldb) <- B U^{-1}, U upper.  kchunk: products summed
// between reductions (at least 16).
constexpr int TRSM_FUSE_MAX = 256;
hipError_t launch_trsm_leaf(int dtype, int side, const void *T, int64_t ldt, int64_t r, void *B, int64_t ldb,
                            int64_t nst, const void *W, double p, int kchunk, hipStream_t st);

// The two solves of a recursion node together, on triangles of the same
// order r: the diagonal blocks of L (unit lower, into WL) and U (upper, into
// WU) in one launch, and the leaves BD (r x ncols) <- L^{-1} BD and
// BE (nrows x r) <- BE U^{-1} in one launch (ncols, nrows > 0).
hipError_t launch_trsm_diag_inv_pair(int dtype, const void *L, int64_t ldl, const void *U, int64_t ldu, int64_t r,
                                     void *WL, void *WU, double p, int kchunk, hipStream_t st);
hipError_t launch_trsm_leaf_pair(int dtype, const void *L, int64_t ldl, const void *U, int64_t ldu, int64_t r,
                                 void *BD, int64_t ldbd, int64_t ncols, void *BE, int64_t ldbe, int64_t nrows,
                                 const void *WL, const void *WU, double p, int kchunk, hipStream_t st);

// dst[i][j] = src[rmap ? rmap[i] : i][cmap ? cmap[j] : j], rows x cols.
hipError_t launch_gather2d(int dtype, const void *src, int64_t lds, void *dst, int64_t ldd,
                           int64_t rows, int64_t cols, const int32_t *rmap,
                           const int32_t *cmap, hipStream_t st);

// Up to GATHER_MAX_JOBS gathers in one launch (dst[i][j] =
// src[rmap ? rmap[i] : i][cmap ? cmap[j] : j], rows x cols each); the jobs'
// destinations must not overlap each other's sources or destinations.
constexpr int GATHER_MAX_JOBS = 8;
struct GatherJob {
    const void *src;
    int64_t lds;
    void *dst;
    int64_t ldd;
    int64_t rows, cols;
    const int32_t *rmap, *cmap;
    int32_t blockStart, colBlocks, rowBlocks;   // filled by the launcher
};
struct GatherJobs {
    GatherJob job[GATHER_MAX_JOBS];
    int32_t count;
};
hipError_t launch_gather_jobs(int dtype, GatherJob *jobs, int njobs, hipStream_t st);

// *flag = gen if any element of the rows x cols block is non-zero.
hipError_t launch_zscan(int dtype, const void *A, int64_t lda, int64_t rows, int64_t cols,
                        int32_t *flag, int32_t gen, hipStream_t st);

// *flag = gen if any element is outside [0, p) (or not an integer, for f64).
hipError_t launch_rangescan(int dtype, const void *A, int64_t lda, int64_t rows,
                            int64_t cols, double p, int32_t *flag, int32_t gen,
                            hipStream_t st);

// Base case, elimination without pivoting of the m x n tile (m, n <= 128),
// gathered through rmap/cmap when given.  r_known < 0: optimistic mode (stop
// on the first zero pivot; success iff the trailing block is zero there);
// otherwise exactly r_known pivots are taken.  status[0] = r, status[1] = 1
// on success (tile written back in packed order), 0 on failure (tile left
// untouched).  specfail (optional): set to 1 unless the tile came out full
// rank in the identity order; errflag (optional): set to 1 on failure (both
// sticky, never cleared by the kernel).
hipError_t launch_bc_lu(int dtype, void *A, int64_t lda, int m, int n, const int32_t *rmap,
                        const int32_t *cmap, int r_known, double p, int kchunk, const uint16_t *inv_table,
                        int32_t *status, int32_t *specfail, int32_t *errflag, hipStream_t st);
// Table of inverses mod p (p <= 65536) used by bc_lu from LDS: bytes of the
// device buffer (0 when the device cannot hold it in LDS or p is larger),
// and the kernel that fills it.
size_t bc_table_bytes(double p);
// Largest tile dimension bc_lu accepts for this modulus when the table is used.
int bc_tile_limit(double p);
constexpr size_t BC_TABLE_RESERVE = 65536 * sizeof(uint16_t);
hipError_t launch_build_inv_table(uint16_t *tab, double p, hipStream_t st);
// Base case, rank profile matrix of the m x n tile: status[0] = r and
// status[1 + i] = pivot column of row i or -1.  The tile is not modified.
// inv_table: as for bc_lu (or null).
hipError_t launch_bc_rpm(int dtype, const void *A, int64_t lda, int m, int n, double p, int kchunk,
                         const uint16_t *inv_table, int32_t *status, hipStream_t st);
int bc_capacity();        // maximum rows (and columns) of a base-case tile
hipError_t bc_init();     // one-time set-up of the base-case kernels

// ---- Winograd's block sums and combinations (k_lincomb.hip) ----
// out (rows x cols, ldo) <- (c[0] X[0] + c[1] X[1] + c[2] X[2]) mod p,
// canonical; c[t] in {-1, 0, 1}, a null X[t] or zero c[t] is left out (all
// three left out: out <- 0).  out may be one of the X[t].  nzflag as in
// MMProblem.
struct LinComb {
    void *out;
    int64_t ldo;
    const void *X[3];
    int64_t ld[3];
    int32_t c[3];
    int64_t rows, cols;
    int32_t *nzflag;
    int32_t nzgen;
};
hipError_t launch_lincomb(int dtype, const LinComb &a, double p, hipStream_t st);

// ---- outputs derived by permutation (k_post.hip) ----
hipError_t launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_inverse_map(const int64_t *P, int64_t n, int32_t *inv, hipStream_t st);
hipError_t launch_pair(const int64_t *P, const int64_t *Q, int64_t m, int64_t n, int64_t r, int32_t *rowpair,
                       int32_t *colpair, hipStream_t st);
hipError_t launch_compact(const int32_t *pair, int64_t lim, int64_t plim, int64_t cap, int32_t *out, int64_t *out64,
                          int64_t *count, hipStream_t st);
hipError_t launch_compose(const int32_t *inv, const int32_t *sel, const int32_t *pair, int64_t n, int32_t *out,
                          hipStream_t st);
hipError_t launch_post_gather(int dtype, bool upper, const void *X, int64_t ldx, int64_t r, void *out, int64_t ldo,
                              int64_t rows, int64_t cols, const int32_t *rowmap, const int32_t *colmap,
                              hipStream_t st);
hipError_t launch_widen(const int32_t *in, int64_t n, int64_t *out, hipStream_t st);
hipError_t launch_leading_ranks(const int32_t *rowpair, int64_t m, const int64_t *ks, const int64_t *ts, int64_t nq,
                                int64_t *rank, hipStream_t st);

}  // namespace pluq

#include <hip/hip_ext.h>

namespace pluq {

// Events attached to the next kernel dispatch when kernels are being timed
// (null otherwise).  The events are recorded by the dispatch itself, so they
// bracket the kernel's execution and nothing else.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents g_launch_events;

}  // namespace pluq

#define PLUQ_LAUNCH(kernel, grid, block, shm, st, ...)                                              \
    hipExtLaunchKernelGGL(kernel, grid, block, shm, st, ::pluq::g_launch_events.start,            \
                          ::pluq::g_launch_events.stop, 0, __VA_ARGS__)

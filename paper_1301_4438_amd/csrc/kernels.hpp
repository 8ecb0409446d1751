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
    int32_t tileStart; // filled by the launcher
    int32_t tilesN;    // filled by the launcher
};

constexpr int MM_MAX_PROBLEMS = 4;

// FP64 matrix-core form.  kchunk: number of inner-dimension terms that may
// be accumulated before a reduction (multiple of 16, >= 16).
hipError_t launch_modmm_f64(int dtype, MMProblem *probs, int nprob, double p, int kchunk,
                            hipStream_t st);

// Left lower unit TRSM leaf: B (nb x ncols, ldb) <- L^{-1} B, nb <= 64.
hipError_t launch_trsm_llu_leaf(int dtype, const void *L, int64_t ldl, int nb, void *B,
                                int64_t ldb, int64_t ncols, double p, int kchunk,
                                hipStream_t st);
// Right upper non-unit TRSM leaf: B (nrows x nb, ldb) <- B U^{-1}, nb <= 64.
hipError_t launch_trsm_run_leaf(int dtype, void *B, int64_t ldb, int64_t nrows,
                                const void *U, int64_t ldu, int nb, double p, int kchunk,
                                hipStream_t st);

// dst[i][j] = src[rmap ? rmap[i] : i][cmap ? cmap[j] : j], rows x cols.
hipError_t launch_gather2d(int dtype, const void *src, int64_t lds, void *dst, int64_t ldd,
                           int64_t rows, int64_t cols, const int32_t *rmap,
                           const int32_t *cmap, hipStream_t st);

// *flag = gen if any element of the rows x cols block is non-zero.
hipError_t launch_zscan(int dtype, const void *A, int64_t lda, int64_t rows, int64_t cols,
                        int32_t *flag, int32_t gen, hipStream_t st);

// *flag = gen if any element is outside [0, p) (or not an integer, for f64).
hipError_t launch_rangescan(int dtype, const void *A, int64_t lda, int64_t rows,
                            int64_t cols, double p, int32_t *flag, int32_t gen,
                            hipStream_t st);

// Write the int64 vector v (length n) to dst.
hipError_t launch_store_i64(int64_t *dst, const int32_t *src, int64_t n, hipStream_t st);

// Base case, elimination without pivoting of the m x n tile (m*n <= cap),
// gathered through rmap/cmap when given.  r_known < 0: optimistic mode (stop
// on the first zero pivot; success iff the trailing block is zero there);
// otherwise exactly r_known pivots are taken.  status[0] = r, status[1] = 1
// on success (tile written back in packed order), 0 on failure (tile left
// untouched).
hipError_t launch_bc_lu(int dtype, void *A, int64_t lda, int m, int n, const int32_t *rmap,
                        const int32_t *cmap, int r_known, double p, int32_t *status,
                        hipStream_t st);
// Base case, rank profile matrix of the m x n tile: status[0] = r and
// status[1 + i] = pivot column of row i or -1.  The tile is not modified.
hipError_t launch_bc_rpm(int dtype, const void *A, int64_t lda, int m, int n, double p,
                         int32_t *status, hipStream_t st);
int bc_capacity();        // maximum m*n of a base-case tile
hipError_t bc_init();     // raise the dynamic LDS limit of the base-case kernels

}  // namespace pluq

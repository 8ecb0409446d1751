// Data-movement kernels of the recursion: the row and column permutations
// PermR / PermC of Section 2 (realised as gathers through a scratch strip),
// the all-zero test of a block (a zero block returns rank 0 with identity
// permutations without recursing), and the optional input range check.
// All are HBM-bound: one coalesced pass over the block.
#include <algorithm>
#include <climits>

#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

constexpr int PTHREADS = 256;

// dst[i][j] = src[rmap[i]][cmap[j]] (maps optional).  blockIdx.y walks rows
// in a grid-stride loop, blockIdx.x/threadIdx.x cover 256 columns.
template <typename T>
__global__ __launch_bounds__(PTHREADS) void gather2d_kernel(const T *src, int64_t lds, T *dst,
                                                            int64_t ldd, int64_t rows, int64_t cols,
                                                            const int32_t *rmap,
                                                            const int32_t *cmap) {
    const int64_t j = (int64_t)blockIdx.x * PTHREADS + threadIdx.x;
    if (j >= cols) return;
    const int64_t sj = cmap ? (int64_t)cmap[j] : j;
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) {
        const int64_t si = rmap ? (int64_t)rmap[i] : i;
        dst[i * ldd + j] = src[si * lds + sj];
    }
}

template <typename T>
__global__ __launch_bounds__(PTHREADS) void zscan_kernel(const T *A, int64_t lda, int64_t rows,
                                                         int64_t cols, int32_t *flag, int32_t gen) {
    const int64_t j = (int64_t)blockIdx.x * PTHREADS + threadIdx.x;
    if (j >= cols) return;
    bool nz = false;
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) nz |= (A[i * lda + j] != (T)0);
    if (nz) *flag = gen;
}

template <typename T>
__global__ __launch_bounds__(PTHREADS) void rangescan_kernel(const T *A, int64_t lda, int64_t rows,
                                                             int64_t cols, double p, int32_t *flag,
                                                             int32_t gen) {
    const int64_t j = (int64_t)blockIdx.x * PTHREADS + threadIdx.x;
    if (j >= cols) return;
    bool bad = false;
    for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) {
        const double v = to_f64(A[i * lda + j]);
        bad |= !(v >= 0.0 && v < p && v == floor(v));
    }
    if (bad) *flag = gen;
}

// Several gathers of disjoint blocks in one launch: job q owns work-groups
// [blockStart_q, blockStart_q + colBlocks_q * rowBlocks_q); work-group b of
// a job covers 256 columns (b % colBlocks) and the rows b / colBlocks,
// + rowBlocks, ...  dst[i][j] = src[rmap ? rmap[i] : i][cmap ? cmap[j] : j].
template <typename T>
__global__ __launch_bounds__(PTHREADS) void gather_jobs_kernel(const GatherJobs args) {
    int q = 0;
#pragma unroll
    for (int t = 1; t < GATHER_MAX_JOBS; ++t)
        if (t < args.count && (int)blockIdx.x >= args.job[t].blockStart) q = t;
    const GatherJob &J = args.job[q];
    const int b = (int)blockIdx.x - J.blockStart;
    const int64_t j = (int64_t)(b % J.colBlocks) * PTHREADS + threadIdx.x;
    if (j >= J.cols) return;
    const T *src = (const T *)J.src;
    T *dst = (T *)J.dst;
    const int64_t sj = J.cmap ? (int64_t)J.cmap[j] : j;
    for (int64_t i = b / J.colBlocks; i < J.rows; i += J.rowBlocks) {
        const int64_t si = J.rmap ? (int64_t)J.rmap[i] : i;
        dst[i * J.ldd + j] = src[si * J.lds + sj];
    }
}

hipError_t launch_gather_jobs(int dtype, GatherJob *jobs, int njobs, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    if (njobs > GATHER_MAX_JOBS) return hipErrorInvalidValue;
    GatherJobs a;
    a.count = 0;
    int64_t total = 0;
    for (int q = 0; q < njobs; ++q) {
        GatherJob J = jobs[q];
        if (J.rows <= 0 || J.cols <= 0) continue;
        J.colBlocks = (int32_t)cdiv64(J.cols, PTHREADS);
        // enough row-blocks to fill the GPU, capped by the row count
        int64_t rb = (4096 + J.colBlocks - 1) / J.colBlocks;
        J.rowBlocks = (int32_t)std::min<int64_t>(std::max<int64_t>(rb, 1), J.rows);
        J.blockStart = (int32_t)total;
        total += (int64_t)J.colBlocks * J.rowBlocks;
        a.job[a.count++] = J;
    }
    if (a.count == 0) return hipSuccess;
    if (total > INT32_MAX) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: PLUQ_LAUNCH(gather_jobs_kernel<int64_t>, dim3((unsigned)total), dim3(PTHREADS), 0, st, a); break;
    case DT_F64: PLUQ_LAUNCH(gather_jobs_kernel<double>, dim3((unsigned)total), dim3(PTHREADS), 0, st, a); break;
    case DT_I32: PLUQ_LAUNCH(gather_jobs_kernel<int32_t>, dim3((unsigned)total), dim3(PTHREADS), 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static dim3 grid2d(int64_t rows, int64_t cols) {
    const int64_t gx = cdiv64(cols, PTHREADS);
    // enough row-blocks to fill the GPU, capped by the row count
    int64_t gy = (4096 + gx - 1) / gx;
    if (gy > rows) gy = rows;
    if (gy > 65535) gy = 65535;
    if (gy < 1) gy = 1;
    return dim3((unsigned)gx, (unsigned)gy);
}

hipError_t launch_gather2d(int dtype, const void *src, int64_t lds, void *dst, int64_t ldd,
                           int64_t rows, int64_t cols, const int32_t *rmap, const int32_t *cmap,
                           hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 g = grid2d(rows, cols);
    switch (dtype) {
    case DT_I64:
        PLUQ_LAUNCH(gather2d_kernel<int64_t>, g, dim3(PTHREADS), 0, st, (const int64_t *)src, lds,
                           (int64_t *)dst, ldd, rows, cols, rmap, cmap);
        break;
    case DT_F64:
        PLUQ_LAUNCH(gather2d_kernel<double>, g, dim3(PTHREADS), 0, st, (const double *)src, lds,
                           (double *)dst, ldd, rows, cols, rmap, cmap);
        break;
    case DT_I32:
        PLUQ_LAUNCH(gather2d_kernel<int32_t>, g, dim3(PTHREADS), 0, st, (const int32_t *)src, lds,
                           (int32_t *)dst, ldd, rows, cols, rmap, cmap);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_zscan(int dtype, const void *A, int64_t lda, int64_t rows, int64_t cols,
                        int32_t *flag, int32_t gen, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 g = grid2d(rows, cols);
    switch (dtype) {
    case DT_I64:
        PLUQ_LAUNCH(zscan_kernel<int64_t>, g, dim3(PTHREADS), 0, st, (const int64_t *)A, lda, rows, cols, flag, gen);
        break;
    case DT_F64:
        PLUQ_LAUNCH(zscan_kernel<double>, g, dim3(PTHREADS), 0, st, (const double *)A, lda, rows, cols, flag, gen);
        break;
    case DT_I32:
        PLUQ_LAUNCH(zscan_kernel<int32_t>, g, dim3(PTHREADS), 0, st, (const int32_t *)A, lda, rows, cols, flag, gen);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rangescan(int dtype, const void *A, int64_t lda, int64_t rows, int64_t cols,
                            double p, int32_t *flag, int32_t gen, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 g = grid2d(rows, cols);
    switch (dtype) {
    case DT_I64:
        PLUQ_LAUNCH(rangescan_kernel<int64_t>, g, dim3(PTHREADS), 0, st, (const int64_t *)A, lda, rows, cols, p, flag, gen);
        break;
    case DT_F64:
        PLUQ_LAUNCH(rangescan_kernel<double>, g, dim3(PTHREADS), 0, st, (const double *)A, lda, rows, cols, p, flag, gen);
        break;
    case DT_I32:
        PLUQ_LAUNCH(rangescan_kernel<int32_t>, g, dim3(PTHREADS), 0, st, (const int32_t *)A, lda, rows, cols, p, flag, gen);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pluq

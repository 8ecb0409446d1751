// Leaves of the two triangular solves of Section 2, TRSM(L, B) and TRSM(B, U),
// for a triangle of order nb <= 64.  Larger solves are split recursively by
// the host driver into two half-size solves and one MM update, so almost all
// of their work runs on the matrix cores (k_modmm.hip).
//
// Arithmetic follows the delayed-reduction cost model of Section 6 (theorem
// on TRSM reductions): each unknown is one exact sum of products reduced once;
// the non-unit solve additionally multiplies by the inverse of the diagonal
// entry (a second reduction).  Residues are kept in symmetric form so that a
// sum of up to `kchunk` products stays below 2^52.
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

constexpr int TNB = 64;

// B (nb x ncols) <- L^{-1} B, L unit lower.  One thread per column of B; the
// strict lower triangle of L is broadcast from LDS.
template <typename T, bool CHUNK>
__global__ __launch_bounds__(256) void trsm_llu_leaf_kernel(const T *L, int64_t ldl, int nb,
                                                            T *B, int64_t ldb, int64_t ncols,
                                                            ModP mod, int kchunk) {
    __shared__ double Ls[TNB][TNB + 1];
    for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
        const int i = idx / nb, j = idx % nb;
        Ls[i][j] = (j < i) ? to_sym(to_f64(L[(int64_t)i * ldl + j]), mod) : 0.0;
    }
    __syncthreads();
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    double x[TNB];
#pragma unroll
    for (int i = 0; i < TNB; ++i)
        x[i] = (i < nb) ? to_sym(to_f64(B[(int64_t)i * ldb + col]), mod) : 0.0;
#pragma unroll
    for (int i = 1; i < TNB; ++i) {
        if (i < nb) {
            double acc = x[i];
#pragma unroll
            for (int j = 0; j < i; ++j) {
                acc = fma(-Ls[i][j], x[j], acc);
                if (CHUNK && ((j + 1) % kchunk) == 0) acc = mod_reduce(acc, mod);
            }
            x[i] = to_sym(mod_reduce(acc, mod), mod);
        }
    }
#pragma unroll
    for (int i = 0; i < TNB; ++i)
        if (i < nb) {
            const double v = x[i] < 0.0 ? x[i] + mod.p : x[i];
            B[(int64_t)i * ldb + col] = from_f64<T>(v);
        }
}

// B (nrows x nb) <- B U^{-1}, U upper with non-zero diagonal.  One thread per
// row of B; a 128-row tile of B is staged in LDS so global accesses stay
// coalesced.
constexpr int RUN_ROWS = 128;

template <typename T, bool CHUNK>
__global__ __launch_bounds__(RUN_ROWS) void trsm_run_leaf_kernel(T *B, int64_t ldb, int64_t nrows,
                                                                 const T *U, int64_t ldu, int nb,
                                                                 ModP mod, int kchunk) {
    __shared__ uint32_t Us[TNB][TNB + 1];
    __shared__ double Uinv[TNB];
    __shared__ uint32_t Bs[RUN_ROWS][TNB + 1];
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * RUN_ROWS;
    for (int idx = tid; idx < nb * nb; idx += RUN_ROWS) {
        const int i = idx / nb, j = idx % nb;
        Us[i][j] = (i <= j) ? (uint32_t)to_f64(U[(int64_t)i * ldu + j]) : 0u;
    }
    if (tid < nb) Uinv[tid] = mod_inv(to_f64(U[(int64_t)tid * ldu + tid]), mod);
    for (int idx = tid; idx < RUN_ROWS * nb; idx += RUN_ROWS) {
        const int r = idx / nb, j = idx % nb;
        const int64_t gr = row0 + r;
        Bs[r][j] = (gr < nrows) ? (uint32_t)to_f64(B[gr * ldb + j]) : 0u;
    }
    __syncthreads();
    if (row0 + tid < nrows) {
        double x[TNB];
#pragma unroll
        for (int j = 0; j < TNB; ++j) {
            if (j < nb) {
                double acc = to_sym((double)Bs[tid][j], mod);
#pragma unroll
                for (int i = 0; i < j; ++i) {
                    acc = fma(-x[i], to_sym((double)Us[i][j], mod), acc);
                    if (CHUNK && ((i + 1) % kchunk) == 0) acc = mod_reduce(acc, mod);
                }
                const double s = mod_reduce(acc, mod);
                x[j] = to_sym(mod_mul(s, Uinv[j], mod), mod);
                Bs[tid][j] = (uint32_t)(x[j] < 0.0 ? x[j] + mod.p : x[j]);
            } else {
                x[j] = 0.0;
            }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < RUN_ROWS * nb; idx += RUN_ROWS) {
        const int r = idx / nb, j = idx % nb;
        const int64_t gr = row0 + r;
        if (gr < nrows) B[gr * ldb + j] = from_f64<T>((double)Bs[r][j]);
    }
}

static ModP make_mod(double p) {
    ModP m;
    m.p = p;
    m.pinv = 1.0 / p;
    m.half = (double)((int64_t)p / 2);
    return m;
}

template <typename T>
static hipError_t llu_t(const void *L, int64_t ldl, int nb, void *B, int64_t ldb, int64_t ncols,
                        double p, int kchunk, hipStream_t st) {
    const dim3 grid((unsigned)cdiv64(ncols, 256));
    if (kchunk < TNB)
        hipLaunchKernelGGL((trsm_llu_leaf_kernel<T, true>), grid, dim3(256), 0, st, (const T *)L, ldl, nb,
                           (T *)B, ldb, ncols, make_mod(p), kchunk);
    else
        hipLaunchKernelGGL((trsm_llu_leaf_kernel<T, false>), grid, dim3(256), 0, st, (const T *)L, ldl, nb,
                           (T *)B, ldb, ncols, make_mod(p), kchunk);
    return hipGetLastError();
}

template <typename T>
static hipError_t run_t(void *B, int64_t ldb, int64_t nrows, const void *U, int64_t ldu, int nb,
                        double p, int kchunk, hipStream_t st) {
    const dim3 grid((unsigned)cdiv64(nrows, RUN_ROWS));
    if (kchunk < TNB)
        hipLaunchKernelGGL((trsm_run_leaf_kernel<T, true>), grid, dim3(RUN_ROWS), 0, st, (T *)B, ldb, nrows,
                           (const T *)U, ldu, nb, make_mod(p), kchunk);
    else
        hipLaunchKernelGGL((trsm_run_leaf_kernel<T, false>), grid, dim3(RUN_ROWS), 0, st, (T *)B, ldb, nrows,
                           (const T *)U, ldu, nb, make_mod(p), kchunk);
    return hipGetLastError();
}

hipError_t launch_trsm_llu_leaf(int dtype, const void *L, int64_t ldl, int nb, void *B, int64_t ldb,
                                int64_t ncols, double p, int kchunk, hipStream_t st) {
    if (nb <= 0 || ncols <= 0) return hipSuccess;
    if (nb > TNB) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return llu_t<int64_t>(L, ldl, nb, B, ldb, ncols, p, kchunk, st);
    case DT_F64: return llu_t<double>(L, ldl, nb, B, ldb, ncols, p, kchunk, st);
    case DT_I32: return llu_t<int32_t>(L, ldl, nb, B, ldb, ncols, p, kchunk, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_trsm_run_leaf(int dtype, void *B, int64_t ldb, int64_t nrows, const void *U,
                                int64_t ldu, int nb, double p, int kchunk, hipStream_t st) {
    if (nb <= 0 || nrows <= 0) return hipSuccess;
    if (nb > TNB) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return run_t<int64_t>(B, ldb, nrows, U, ldu, nb, p, kchunk, st);
    case DT_F64: return run_t<double>(B, ldb, nrows, U, ldu, nb, p, kchunk, st);
    case DT_I32: return run_t<int32_t>(B, ldb, nrows, U, ldu, nb, p, kchunk, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace pluq

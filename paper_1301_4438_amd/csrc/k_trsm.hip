// Leaves of the two triangular solves of Section 2, TRSM(L, B) and TRSM(B, U),
// for a triangle of order nb <= 64.  Larger solves are split recursively by
// the host driver into two half-size solves and one MM update, so almost all
// of their work runs on the matrix cores (k_modmm.hip).
//
// Each thread owns one right-hand side (a column of B for the left solve, a
// row of B for the right solve) in registers and eliminates right-looking:
// once unknown j is final it is subtracted from all later unknowns with
// independent fused multiply-adds.  With delayed reduction (Section 6, the
// theorem on TRSM reductions) an unknown is reduced once when it becomes
// final (and, for the non-unit solve, multiplied by the inverse of the
// diagonal entry: a second reduction); the running sums are exact
// integer-valued doubles of symmetric residues, reduced after `kchunk` terms
// if p is large enough to need it.
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

constexpr int TNB = 64;

// B (nb x ncols) <- L^{-1} B, L unit lower.  One thread per column of B; the
// strict lower triangle of L is broadcast from LDS.
template <typename T, bool CHUNK>
__global__ __launch_bounds__(64, 1) void trsm_llu_leaf_kernel(const T *L, int64_t ldl, int nb, T *B,
                                                              int64_t ldb, int64_t ncols, ModP mod,
                                                              int kchunk) {
    // LT[j][i] = L[i][j] (strict lower part, symmetric residues): the column
    // needed at step j is contiguous and is read as one batch of vector loads
    __shared__ __align__(16) double LT[TNB][TNB];
    // thread t loads column t of L: TNB independent loads in flight
    {
        const int t = threadIdx.x;
        double tmp[TNB];
#pragma unroll
        for (int i = 0; i < TNB; ++i) tmp[i] = (t < i && i < nb) ? to_f64(L[(int64_t)i * ldl + t]) : 0.0;
#pragma unroll
        for (int i = 0; i < TNB; ++i) LT[t][i] = to_sym(tmp[i], mod);
    }
    __syncthreads();
    const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= ncols) return;
    double x[TNB];
#pragma unroll
    for (int i = 0; i < TNB; ++i) x[i] = (i < nb) ? to_f64(B[(int64_t)i * ldb + col]) : 0.0;
#pragma unroll
    for (int j = 0; j < TNB; ++j) {
        if (j < nb) {
            double lc[TNB];
#pragma unroll
            for (int i = j + 1; i < TNB; ++i) lc[i] = LT[j][i];
            const double xj = to_sym(mod_reduce(x[j], mod), mod);
            x[j] = xj;
#pragma unroll
            for (int i = j + 1; i < TNB; ++i) x[i] = fma(-lc[i], xj, x[i]);
            if (CHUNK && ((j + 1) % kchunk) == 0) {
#pragma unroll
                for (int i = j + 1; i < TNB; ++i) x[i] = mod_reduce(x[i], mod);
            }
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
// row of B; a 64-row tile of B is staged in LDS so global accesses stay
// coalesced.
constexpr int RUN_ROWS = 64;

template <typename T, bool CHUNK>
__global__ __launch_bounds__(RUN_ROWS, 1) void trsm_run_leaf_kernel(T *B, int64_t ldb, int64_t nrows,
                                                                    const T *U, int64_t ldu, int nb,
                                                                    ModP mod, int kchunk) {
    __shared__ __align__(16) double Us[TNB][TNB];
    __shared__ double Uinv[TNB];
    __shared__ uint32_t Bs[RUN_ROWS][TNB + 1];
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * RUN_ROWS;
    // thread t loads column t of U and column t of the B tile: all loads of a
    // thread are independent and in flight together (coalesced across threads)
    {
        double tu[TNB];
        uint32_t tb[RUN_ROWS];
#pragma unroll
        for (int i = 0; i < TNB; ++i) tu[i] = (i < tid && tid < nb) ? to_f64(U[(int64_t)i * ldu + tid]) : 0.0;
#pragma unroll
        for (int r = 0; r < RUN_ROWS; ++r) {
            const int64_t gr = row0 + r;
            tb[r] = (gr < nrows && tid < nb) ? (uint32_t)to_f64(B[gr * ldb + tid]) : 0u;
        }
        const double d = (tid < nb) ? to_f64(U[(int64_t)tid * ldu + tid]) : 1.0;
#pragma unroll
        for (int i = 0; i < TNB; ++i) Us[i][tid] = to_sym(tu[i], mod);
#pragma unroll
        for (int r = 0; r < RUN_ROWS; ++r) Bs[r][tid] = tb[r];
        Uinv[tid] = mod_inv(d, mod);
    }
    __syncthreads();
    if (row0 + tid < nrows) {
        double x[TNB];
#pragma unroll
        for (int j = 0; j < TNB; ++j) x[j] = (j < nb) ? (double)Bs[tid][j] : 0.0;
#pragma unroll
        for (int j = 0; j < TNB; ++j) {
            if (j < nb) {
                double uc[TNB];
#pragma unroll
                for (int k = j + 1; k < TNB; ++k) uc[k] = Us[j][k];
                const double xj = to_sym(mod_mul(mod_reduce(x[j], mod), Uinv[j], mod), mod);
                x[j] = xj;
#pragma unroll
                for (int k = j + 1; k < TNB; ++k) x[k] = fma(-xj, uc[k], x[k]);
                if (CHUNK && ((j + 1) % kchunk) == 0) {
#pragma unroll
                    for (int k = j + 1; k < TNB; ++k) x[k] = mod_reduce(x[k], mod);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < TNB; ++j)
            if (j < nb) Bs[tid][j] = (uint32_t)(x[j] < 0.0 ? x[j] + mod.p : x[j]);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RUN_ROWS; ++r) {
        const int64_t gr = row0 + r;
        if (gr < nrows && tid < nb) B[gr * ldb + tid] = from_f64<T>((double)Bs[r][tid]);
    }
}

// Inverses of all diagonal blocks of a triangle at once (one work-group per
// 64 x 64 block), stored as I - T_qq^{-1} in canonical form, row-major with
// leading dimension 64, block q at W + q * 64 * 64.  A solve then applies
// them with the matrix cores: B_q <- B_q - (I - L_qq^{-1}) B_q = L_qq^{-1} B_q.
//
// Lower unit: thread t computes column t of L^{-1} (forward elimination of
// e_t, right-looking as in the leaf above).
template <typename T, bool CHUNK>
__global__ __launch_bounds__(64, 1) void trsm_diag_inv_llu_kernel(const T *L, int64_t ldl, int r, T *W,
                                                                  ModP mod, int kchunk) {
    __shared__ __align__(16) double LT[TNB][TNB];
    const int o = blockIdx.x * TNB;
    const int nb = min(TNB, r - o);
    const int t = threadIdx.x;
    const T *Lq = L + (int64_t)o * ldl + o;
    {
        double tmp[TNB];
#pragma unroll
        for (int i = 0; i < TNB; ++i) tmp[i] = (t < i && i < nb) ? to_f64(Lq[(int64_t)i * ldl + t]) : 0.0;
#pragma unroll
        for (int i = 0; i < TNB; ++i) LT[t][i] = to_sym(tmp[i], mod);
    }
    __syncthreads();
    double x[TNB];
#pragma unroll
    for (int i = 0; i < TNB; ++i) x[i] = (i == t) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < TNB; ++j) {
        if (j < nb) {
            double lc[TNB];
#pragma unroll
            for (int i = j + 1; i < TNB; ++i) lc[i] = LT[j][i];
            const double xj = to_sym(mod_reduce(x[j], mod), mod);
            x[j] = xj;
#pragma unroll
            for (int i = j + 1; i < TNB; ++i) x[i] = fma(-lc[i], xj, x[i]);
            if (CHUNK && ((j + 1) % kchunk) == 0) {
#pragma unroll
                for (int i = j + 1; i < TNB; ++i) x[i] = mod_reduce(x[i], mod);
            }
        }
    }
    T *Wq = W + (int64_t)blockIdx.x * TNB * TNB;
    if (t < nb) {
#pragma unroll
        for (int i = 0; i < TNB; ++i)
            if (i < nb) Wq[i * TNB + t] = from_f64<T>(i == t ? 0.0 : mod_reduce(-x[i], mod));
    }
}

// Upper non-unit: thread t computes row t of U^{-1} (right-looking solve of
// x U = e_t, with the diagonal inverses).
template <typename T, bool CHUNK>
__global__ __launch_bounds__(64, 1) void trsm_diag_inv_run_kernel(const T *U, int64_t ldu, int r, T *W,
                                                                  ModP mod, int kchunk) {
    __shared__ __align__(16) double Us[TNB][TNB];
    __shared__ double Uinv[TNB];
    const int o = blockIdx.x * TNB;
    const int nb = min(TNB, r - o);
    const int t = threadIdx.x;
    const T *Uq = U + (int64_t)o * ldu + o;
    {
        double tu[TNB];
#pragma unroll
        for (int i = 0; i < TNB; ++i) tu[i] = (i < t && t < nb) ? to_f64(Uq[(int64_t)i * ldu + t]) : 0.0;
        const double d = (t < nb) ? to_f64(Uq[(int64_t)t * ldu + t]) : 1.0;
#pragma unroll
        for (int i = 0; i < TNB; ++i) Us[i][t] = to_sym(tu[i], mod);
        Uinv[t] = mod_inv(d, mod);
    }
    __syncthreads();
    double x[TNB];
#pragma unroll
    for (int j = 0; j < TNB; ++j) x[j] = (j == t) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < TNB; ++j) {
        if (j < nb) {
            double uc[TNB];
#pragma unroll
            for (int k = j + 1; k < TNB; ++k) uc[k] = Us[j][k];
            const double xj = to_sym(mod_mul(mod_reduce(x[j], mod), Uinv[j], mod), mod);
            x[j] = xj;
#pragma unroll
            for (int k = j + 1; k < TNB; ++k) x[k] = fma(-xj, uc[k], x[k]);
            if (CHUNK && ((j + 1) % kchunk) == 0) {
#pragma unroll
                for (int k = j + 1; k < TNB; ++k) x[k] = mod_reduce(x[k], mod);
            }
        }
    }
    T *Wq = W + (int64_t)blockIdx.x * TNB * TNB;
    if (t < nb) {
#pragma unroll
        for (int j = 0; j < TNB; ++j)
            if (j < nb) Wq[t * TNB + j] = from_f64<T>(mod_reduce((j == t ? 1.0 : 0.0) - x[j], mod));
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
static hipError_t diag_inv_t(int side, const void *Tm, int64_t ldt, int r, void *W, double p, int kchunk,
                             hipStream_t st) {
    const dim3 grid((unsigned)cdiv64(r, TNB));
    const ModP md = make_mod(p);
    if (side == 0) {
        if (kchunk < TNB)
            PLUQ_LAUNCH((trsm_diag_inv_llu_kernel<T, true>), grid, dim3(64), 0, st, (const T *)Tm, ldt, r, (T *)W, md, kchunk);
        else
            PLUQ_LAUNCH((trsm_diag_inv_llu_kernel<T, false>), grid, dim3(64), 0, st, (const T *)Tm, ldt, r, (T *)W, md, kchunk);
    } else {
        if (kchunk < TNB)
            PLUQ_LAUNCH((trsm_diag_inv_run_kernel<T, true>), grid, dim3(64), 0, st, (const T *)Tm, ldt, r, (T *)W, md, kchunk);
        else
            PLUQ_LAUNCH((trsm_diag_inv_run_kernel<T, false>), grid, dim3(64), 0, st, (const T *)Tm, ldt, r, (T *)W, md, kchunk);
    }
    return hipGetLastError();
}

hipError_t launch_trsm_diag_inv(int dtype, int side, const void *Tm, int64_t ldt, int64_t r, void *W, double p,
                                int kchunk, hipStream_t st) {
    if (r <= 0) return hipSuccess;
    if (kchunk < 1 || r > INT32_MAX) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return diag_inv_t<int64_t>(side, Tm, ldt, (int)r, W, p, kchunk, st);
    case DT_F64: return diag_inv_t<double>(side, Tm, ldt, (int)r, W, p, kchunk, st);
    case DT_I32: return diag_inv_t<int32_t>(side, Tm, ldt, (int)r, W, p, kchunk, st);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t llu_t(const void *L, int64_t ldl, int nb, void *B, int64_t ldb, int64_t ncols,
                        double p, int kchunk, hipStream_t st) {
    const dim3 grid((unsigned)cdiv64(ncols, 64));
    if (kchunk < TNB)
        PLUQ_LAUNCH((trsm_llu_leaf_kernel<T, true>), grid, dim3(64), 0, st, (const T *)L, ldl, nb,
                           (T *)B, ldb, ncols, make_mod(p), kchunk);
    else
        PLUQ_LAUNCH((trsm_llu_leaf_kernel<T, false>), grid, dim3(64), 0, st, (const T *)L, ldl, nb,
                           (T *)B, ldb, ncols, make_mod(p), kchunk);
    return hipGetLastError();
}

template <typename T>
static hipError_t run_t(void *B, int64_t ldb, int64_t nrows, const void *U, int64_t ldu, int nb,
                        double p, int kchunk, hipStream_t st) {
    const dim3 grid((unsigned)cdiv64(nrows, RUN_ROWS));
    if (kchunk < TNB)
        PLUQ_LAUNCH((trsm_run_leaf_kernel<T, true>), grid, dim3(RUN_ROWS), 0, st, (T *)B, ldb, nrows,
                           (const T *)U, ldu, nb, make_mod(p), kchunk);
    else
        PLUQ_LAUNCH((trsm_run_leaf_kernel<T, false>), grid, dim3(RUN_ROWS), 0, st, (T *)B, ldb, nrows,
                           (const T *)U, ldu, nb, make_mod(p), kchunk);
    return hipGetLastError();
}

hipError_t launch_trsm_llu_leaf(int dtype, const void *L, int64_t ldl, int nb, void *B, int64_t ldb,
                                int64_t ncols, double p, int kchunk, hipStream_t st) {
    if (nb <= 0 || ncols <= 0) return hipSuccess;
    if (nb > TNB || kchunk < 1) return hipErrorInvalidValue;
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
    if (nb > TNB || kchunk < 1) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return run_t<int64_t>(B, ldb, nrows, U, ldu, nb, p, kchunk, st);
    case DT_F64: return run_t<double>(B, ldb, nrows, U, ldu, nb, p, kchunk, st);
    case DT_I32: return run_t<int32_t>(B, ldb, nrows, U, ldu, nb, p, kchunk, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace pluq

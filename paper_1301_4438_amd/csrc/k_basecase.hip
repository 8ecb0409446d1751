// Base case of the recursion: the decomposition of a tile small enough to sit
// in the LDS of one compute unit (m * n <= bc_capacity()).
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
//              the rank of the leading sub-matrices jumps).  The pivot of row
//              i is found with a wavefront ballot and find-first-set.
//   bc_lu   -- elimination without pivoting of the tile gathered through the
//              row/column order, written back in packed form.
// bc_lu is also tried first on the tile as it is: when every pivot on the
// diagonal is non-zero (a generic rank profile, the case of Section 5's
// leading-constant analysis), or the remaining block is zero where the first
// zero pivot appears, the identity order is already the right one and the
// rank-profile pass is skipped.  The pivot order itself is computed on the
// host between the two kernels (index bookkeeping only).
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

constexpr int BC_THREADS = 256;
constexpr int BC_CAP = 16384;                  // elements (u32) of a tile
constexpr int BC_LDS = BC_CAP * 4 + 16384 + 64; // tile + per-column flags + slack

template <typename T>
__global__ __launch_bounds__(BC_THREADS) void bc_lu_kernel(T *A, int64_t lda, int m, int n,
                                                           const int32_t *rmap,
                                                           const int32_t *cmap, int r_known,
                                                           ModP mod, int32_t *status) {
    extern __shared__ uint32_t S[];
    __shared__ double s_inv;
    __shared__ int s_zero;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < m * n; idx += BC_THREADS) {
        const int i = idx / n, j = idx % n;
        const int64_t gi = rmap ? rmap[i] : i;
        const int64_t gj = cmap ? cmap[j] : j;
        S[idx] = (uint32_t)to_f64(A[gi * lda + gj]);
    }
    __syncthreads();
    const int kmax = m < n ? m : n;
    const int steps = r_known >= 0 ? r_known : kmax;
    int r = steps;
    bool ok = true;
    for (int s = 0; s < steps; ++s) {
        if (tid == 0) {
            const double v = (double)S[s * n + s];
            s_zero = (v == 0.0);
            if (v != 0.0) s_inv = mod_inv(v, mod);
        }
        __syncthreads();
        if (s_zero) {
            // zero pivot: the identity order is right iff the rest is zero
            int any = 0;
            const int w = n - s;
            for (int idx = tid; idx < (m - s) * w; idx += BC_THREADS)
                any |= (S[(s + idx / w) * n + s + idx % w] != 0u);
            any = __syncthreads_or(any);
            ok = (any == 0);
            r = s;
            break;
        }
        const double inv = s_inv;
        for (int i = s + 1 + tid; i < m; i += BC_THREADS)
            S[i * n + s] = (uint32_t)mod_mul((double)S[i * n + s], inv, mod);
        __syncthreads();
        const int w = n - s - 1;
        const int cnt = (m - s - 1) * w;
        for (int idx = tid; idx < cnt; idx += BC_THREADS) {
            const int i = s + 1 + idx / w, j = s + 1 + idx % w;
            const uint32_t l = S[i * n + s];
            const uint32_t u = S[s * n + j];
            if (l != 0u && u != 0u)
                S[i * n + j] = (uint32_t)mod_reduce((double)S[i * n + j] - (double)l * (double)u, mod);
        }
        __syncthreads();
    }
    if (!ok) {
        if (tid == 0) { status[0] = r; status[1] = 0; }
        return;
    }
    for (int idx = tid; idx < m * n; idx += BC_THREADS) {
        const int i = idx / n, j = idx % n;
        A[(int64_t)i * lda + j] = from_f64<T>((double)S[idx]);
    }
    if (tid == 0) { status[0] = r; status[1] = 1; }
}

template <typename T>
__global__ __launch_bounds__(BC_THREADS) void bc_rpm_kernel(const T *A, int64_t lda, int m, int n,
                                                            ModP mod, int32_t *status) {
    extern __shared__ uint32_t S[];
    uint8_t *dead = (uint8_t *)(S + m * n);
    __shared__ int s_col[2];
    __shared__ double s_inv[2];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    for (int idx = tid; idx < m * n; idx += BC_THREADS)
        S[idx] = (uint32_t)to_f64(A[(int64_t)(idx / n) * lda + idx % n]);
    for (int j = tid; j < n; j += BC_THREADS) dead[j] = 0;
    __syncthreads();
    int r = 0;
    for (int i = 0; i < m; ++i) {
        const int buf = i & 1;
        if (tid < 64) {
            int found = -1;
            for (int c0 = 0; c0 < n; c0 += 64) {
                const int c = c0 + lane;
                const bool nz = (c < n) && S[i * n + c] != 0u && !dead[c];
                const unsigned long long mask = __ballot(nz);
                if (mask) { found = c0 + __ffsll((long long)mask) - 1; break; }
            }
            if (lane == 0) {
                s_col[buf] = found;
                status[1 + i] = found;
                if (found >= 0) {
                    s_inv[buf] = mod_inv((double)S[i * n + found], mod);
                    dead[found] = 1;
                }
            }
        }
        __syncthreads();
        const int jc = s_col[buf];
        if (jc < 0) continue;
        ++r;
        const double inv = s_inv[buf];
        const int cnt = (m - i - 1) * n;
        for (int idx = tid; idx < cnt; idx += BC_THREADS) {
            const int k = i + 1 + idx / n, c = idx % n;
            if (dead[c]) continue;
            const uint32_t u = S[i * n + c];
            if (u == 0u) continue;
            const uint32_t l = S[k * n + jc];
            if (l == 0u) continue;
            const double lm = mod_mul((double)l, inv, mod);
            S[k * n + c] = (uint32_t)mod_reduce((double)S[k * n + c] - lm * (double)u, mod);
        }
        __syncthreads();
    }
    if (tid == 0) status[0] = r;
}

static ModP make_mod(double p) {
    ModP md;
    md.p = p;
    md.pinv = 1.0 / p;
    md.half = (double)((int64_t)p / 2);
    return md;
}

int bc_capacity() { return BC_CAP; }

hipError_t bc_init() {
    hipError_t e;
#define PLUQ_SETLDS(K)                                                                              \
    e = hipFuncSetAttribute((const void *)(K), hipFuncAttributeMaxDynamicSharedMemorySize, BC_LDS); \
    if (e != hipSuccess) return e;
    PLUQ_SETLDS(bc_lu_kernel<int64_t>)
    PLUQ_SETLDS(bc_lu_kernel<double>)
    PLUQ_SETLDS(bc_lu_kernel<int32_t>)
    PLUQ_SETLDS(bc_rpm_kernel<int64_t>)
    PLUQ_SETLDS(bc_rpm_kernel<double>)
    PLUQ_SETLDS(bc_rpm_kernel<int32_t>)
#undef PLUQ_SETLDS
    return hipSuccess;
}

hipError_t launch_bc_lu(int dtype, void *A, int64_t lda, int m, int n, const int32_t *rmap,
                        const int32_t *cmap, int r_known, double p, int32_t *status,
                        hipStream_t st) {
    if ((int64_t)m * n > BC_CAP || m <= 0 || n <= 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)m * n * 4;
    switch (dtype) {
    case DT_I64:
        hipLaunchKernelGGL(bc_lu_kernel<int64_t>, dim3(1), dim3(BC_THREADS), lds, st, (int64_t *)A, lda, m, n,
                           rmap, cmap, r_known, make_mod(p), status);
        break;
    case DT_F64:
        hipLaunchKernelGGL(bc_lu_kernel<double>, dim3(1), dim3(BC_THREADS), lds, st, (double *)A, lda, m, n,
                           rmap, cmap, r_known, make_mod(p), status);
        break;
    case DT_I32:
        hipLaunchKernelGGL(bc_lu_kernel<int32_t>, dim3(1), dim3(BC_THREADS), lds, st, (int32_t *)A, lda, m, n,
                           rmap, cmap, r_known, make_mod(p), status);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_bc_rpm(int dtype, const void *A, int64_t lda, int m, int n, double p,
                         int32_t *status, hipStream_t st) {
    if ((int64_t)m * n > BC_CAP || m <= 0 || n <= 0) return hipErrorInvalidValue;
    const size_t lds = (size_t)m * n * 4 + (size_t)n + 16;
    switch (dtype) {
    case DT_I64:
        hipLaunchKernelGGL(bc_rpm_kernel<int64_t>, dim3(1), dim3(BC_THREADS), lds, st, (const int64_t *)A, lda,
                           m, n, make_mod(p), status);
        break;
    case DT_F64:
        hipLaunchKernelGGL(bc_rpm_kernel<double>, dim3(1), dim3(BC_THREADS), lds, st, (const double *)A, lda,
                           m, n, make_mod(p), status);
        break;
    case DT_I32:
        hipLaunchKernelGGL(bc_rpm_kernel<int32_t>, dim3(1), dim3(BC_THREADS), lds, st, (const int32_t *)A, lda,
                           m, n, make_mod(p), status);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pluq

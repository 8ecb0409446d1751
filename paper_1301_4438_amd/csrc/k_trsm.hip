// Triangular solves of Section 2, TRSM(L, B) and TRSM(B, U): the host driver
// splits a solve recursively at multiples of 64 into half-size solves and
// one MM update each; a leaf of order <= 64 is the in-place MM update
//     B <- B - (I - L_qq^{-1}) B    or    B <- B - B (I - U_qq^{-1}),
// so every multiply-add of a solve runs in the MM kernel (k_modmm.hip).  This
// file holds the one kernel the solves need besides MM: the inverses of all
// 64 x 64 diagonal blocks of the triangle, computed in one launch before the
// recursion starts.
#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

// Inverses of the 64 x 64 diagonal blocks of an r x r triangle, one
// work-group of 256 threads per block, written as W = I - T_qq^{-1}
// (canonical, row-major, 64 x 64 per block; rows and columns past the
// triangle's order behave as the identity).  An upper block is inverted
// through its transpose, (U^T)^{-1} = (U^{-1})^T, so both sides run the same
// lower-triangular scheme on X = L^{-1} split into 4 x 4 blocks of 16:
//   the four diagonal blocks D_k = L_kk^{-1} by forward substitution (one
//   wave each, a lane per column, the diagonal inverses computed first);
//   then the blocks below, by distance d = i - j = 1, 2, 3, all entries of a
//   distance at once:  T = sum_{k=j}^{i-1} L_ik X_kj,  X_ij = -D_i T.
// Products are of symmetric residues, reduced after every 16 terms.
template <typename T, bool UPPER>
__global__ __launch_bounds__(256) void trsm_diag_inv_kernel(const T *Tm, int64_t ldt, int r, T *W, ModP mod) {
    __shared__ double Ls[64][65];   // strict lower part (symmetric residues)
    __shared__ double Xs[64][65];   // the inverse being built (symmetric)
    __shared__ double Ts[3][16][17];
    __shared__ double dinv[64];
    const int tid = threadIdx.x;
    const int o = blockIdx.x * 64;
    const int nb = min(64, r - o);
    const T *Tq = Tm + (int64_t)o * ldt + o;
    {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + 256 * q, a = e >> 6, b = e & 63;
            v[q] = (a < nb && b < nb) ? to_f64(Tq[(int64_t)a * ldt + b]) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int e = tid + 256 * q, a = e >> 6, b = e & 63;
            // stored entry (a, b); the lower operand is L (UPPER: U^T)
            const int i = UPPER ? b : a, j = UPPER ? a : b;
            if (i > j) Ls[i][j] = to_sym(v[q], mod);
            else if (i < j) Ls[i][j] = 0.0;
            else dinv[i] = (!UPPER || a >= nb) ? 1.0 : v[q];
            Xs[a][b] = 0.0;
        }
    }
    __syncthreads();
    if (UPPER && tid < 64) dinv[tid] = inv_fermat(dinv[tid], mod);
    __syncthreads();
    const int lane = tid & 63, wv = tid >> 6;
    if (lane < 16) {
        const int base = 16 * wv, c = lane;
        double x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < i; ++k) s = fma(-Ls[base + i][base + k], x[k], s);
            x[i] = to_sym(mod_reduce(mod_reduce(s, mod) * dinv[base + i], mod), mod);
            Xs[base + i][base + c] = x[i];
        }
    }
    __syncthreads();
    const int a = tid >> 4, c = tid & 15;
#pragma unroll
    for (int d = 1; d < 4; ++d) {
        for (int b = 0; b < 4 - d; ++b) {
            const int j = b, i = b + d;
            double acc = 0.0;
            for (int k = j; k < i; ++k) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) s = fma(Ls[16 * i + a][16 * k + q], Xs[16 * k + q][16 * j + c], s);
                acc += mod_reduce(s, mod);
            }
            Ts[b][a][c] = to_sym(mod_reduce(acc, mod), mod);
        }
        __syncthreads();
        for (int b = 0; b < 4 - d; ++b) {
            const int j = b, i = b + d;
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) s = fma(Xs[16 * i + a][16 * i + q], Ts[b][q][c], s);
            Xs[16 * i + a][16 * j + c] = to_sym(mod_reduce(-s, mod), mod);
        }
        __syncthreads();
    }
    T *Wq = W + (int64_t)blockIdx.x * 64 * 64;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q, i = e >> 6, j = e & 63;
        const double x = UPPER ? Xs[j][i] : Xs[i][j];
        Wq[e] = from_f64<T>(mod_reduce((i == j ? 1.0 : 0.0) - x, mod));
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
static hipError_t diag_inv_t(int side, const void *Tm, int64_t ldt, int r, void *W, double p, hipStream_t st) {
    const dim3 grid((unsigned)cdiv64(r, 64));
    const ModP md = make_mod(p);
    if (side == 0)
        PLUQ_LAUNCH((trsm_diag_inv_kernel<T, false>), grid, dim3(256), 0, st, (const T *)Tm, ldt, r, (T *)W, md);
    else
        PLUQ_LAUNCH((trsm_diag_inv_kernel<T, true>), grid, dim3(256), 0, st, (const T *)Tm, ldt, r, (T *)W, md);
    return hipGetLastError();
}

hipError_t launch_trsm_diag_inv(int dtype, int side, const void *Tm, int64_t ldt, int64_t r, void *W, double p,
                                int kchunk, hipStream_t st) {
    if (r <= 0) return hipSuccess;
    if (kchunk < 1 || r > INT32_MAX) return hipErrorInvalidValue;
    switch (dtype) {
    case DT_I64: return diag_inv_t<int64_t>(side, Tm, ldt, (int)r, W, p, st);
    case DT_F64: return diag_inv_t<double>(side, Tm, ldt, (int)r, W, p, st);
    case DT_I32: return diag_inv_t<int32_t>(side, Tm, ldt, (int)r, W, p, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace pluq

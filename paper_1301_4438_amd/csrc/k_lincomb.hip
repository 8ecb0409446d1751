// Elementwise linear combinations of equally shaped blocks mod p: the block
// sums and differences of Winograd's form of Strassen's product and the
// combinations of its block products into C (the sub-cubic product behind
// Section 5's O(m n r^(omega-2)) count).  One coalesced HBM pass; every
// operand is a canonical residue, so a combination of three is below 3p in
// magnitude, exact in float64, and one reduction gives the canonical result.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

constexpr int LC_THREADS = 256;
constexpr int LC_PER = 4;   // columns per thread: LC_THREADS * LC_PER per work-group row

// out[i][j] = (sum_t c_t X_t[i][j]) mod p over the non-null operands;
// blockIdx.y walks rows in a grid-stride loop.  out may be one of the
// operands (each entry is read before it is written, by the same thread).
template <typename T>
__global__ __launch_bounds__(LC_THREADS) void lincomb_kernel(LinComb a, ModP mod) {
    T *out = (T *)a.out;
    const T *X[3] = {(const T *)a.X[0], (const T *)a.X[1], (const T *)a.X[2]};
    bool nz = false;
    for (int64_t i = blockIdx.y; i < a.rows; i += gridDim.y) {
#pragma unroll
        for (int e = 0; e < LC_PER; ++e) {
            const int64_t j = (int64_t)blockIdx.x * (LC_THREADS * LC_PER) + e * LC_THREADS + threadIdx.x;
            if (j < a.cols) {
                double s = 0.0;
#pragma unroll
                for (int t = 0; t < 3; ++t)
                    if (X[t] && a.c[t]) s += (double)a.c[t] * to_f64(X[t][i * a.ld[t] + j]);
                const double v = mod_reduce(s, mod);
                out[i * a.ldo + j] = from_f64<T>(v);
                nz |= (v != 0.0);
            }
        }
    }
    if (nz && a.nzflag) *a.nzflag = a.nzgen;
}

hipError_t launch_lincomb(int dtype, const LinComb &a, double p, hipStream_t st) {
    if (a.rows <= 0 || a.cols <= 0) return hipSuccess;
    for (int t = 0; t < 3; ++t)
        if (a.c[t] < -1 || a.c[t] > 1) return hipErrorInvalidValue;
    ModP mod;
    mod.p = p;
    mod.pinv = 1.0 / p;
    mod.half = (double)((int64_t)p / 2);
    const int64_t per = (int64_t)LC_THREADS * LC_PER;
    // about 8 rows per work-group, at most 65535 row groups
    const dim3 grid((unsigned)((a.cols + per - 1) / per), (unsigned)std::min<int64_t>((a.rows + 7) / 8, 65535));
    switch (dtype) {
    case DT_I64: PLUQ_LAUNCH(lincomb_kernel<int64_t>, grid, dim3(LC_THREADS), 0, st, a, mod); break;
    case DT_F64: PLUQ_LAUNCH(lincomb_kernel<double>, grid, dim3(LC_THREADS), 0, st, a, mod); break;
    case DT_I32: PLUQ_LAUNCH(lincomb_kernel<int32_t>, grid, dim3(LC_THREADS), 0, st, a, mod); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pluq

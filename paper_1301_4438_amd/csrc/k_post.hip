// Outputs read off a finished decomposition by permutation only (Sections 3
// and 4): the LEU decomposition, the column / row echelon factorizations,
// and the rank profiles and ranks of leading sub-matrices.
//
// With X the packed [L\U V; M 0] and the index vectors P, Q of pluq_modp:
//   Lbar = P [L 0; M I] P^T : Lbar[P[i], P[j]] = X[i][j] (i > j, j < r),
//                             1 on the diagonal, 0 elsewhere;
//   Ubar = Q^T [U V; 0 I] Q : Ubar[Q[i], Q[j]] = X[i][j] (j >= i, i < r),
//                             1 on the diagonal past r, 0 elsewhere;
//   E = P [I_r 0; 0 0] Q    : E[P[s], Q[s]] = 1 for s < r (the rank profile
//                             matrix).
// Every output entry is gathered: out[a][b] = Lbar or Ubar at
// (rowmap[a], colmap[b]) in the packed coordinates, i.e. one read of X and
// one coalesced write per entry (HBM bound).  The index maps (inverse
// permutations, the row <-> column pairing of the rank profile matrix and
// the sorted rank profiles) are built by small kernels; every index read
// from P or Q is range-checked, so malformed vectors cannot make a kernel
// access memory outside its buffers.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace pluq {

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t *x, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}

// inv[P[i]] = i for i < n (entries outside [0, n) are skipped).
__global__ __launch_bounds__(256) void inverse_map_kernel(const int64_t *P, int64_t n, int32_t *inv) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t v = P[i];
    if (v >= 0 && v < n) inv[v] = (int32_t)i;
}

// The rank profile matrix's pairing: rowpair[P[s]] = Q[s] and
// colpair[Q[s]] = P[s] for s < r (both filled with -1 beforehand).
__global__ __launch_bounds__(256) void pair_kernel(const int64_t *P, const int64_t *Q, int64_t m, int64_t n, int64_t r,
                                                   int32_t *rowpair, int32_t *colpair) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= r) return;
    const int64_t i = P[s], j = Q[s];
    if (i >= 0 && i < m && j >= 0 && j < n) {
        rowpair[i] = (int32_t)j;
        colpair[j] = (int32_t)i;
    }
}

// Ordered compaction by one work-group: the indices i < lim with
// 0 <= pair[i] < plim, ascending, into out (int32 and, when out64 is given,
// int64; at most cap of them are written); count[0] receives their number.
__global__ __launch_bounds__(1024) void compact_kernel(const int32_t *pair, int64_t lim, int64_t plim, int64_t cap,
                                                       int32_t *out, int64_t *out64, int64_t *count) {
    __shared__ int32_t part[1024];
    __shared__ int32_t base;
    const int tid = threadIdx.x;
    if (tid == 0) base = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < lim; c0 += 1024) {
        const int64_t i = c0 + tid;
        const int flag = (i < lim && pair[i] >= 0 && pair[i] < plim) ? 1 : 0;
        part[tid] = flag;
        __syncthreads();
        // inclusive scan (Hillis-Steele)
        for (int d = 1; d < 1024; d <<= 1) {
            const int v = tid >= d ? part[tid - d] : 0;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        if (flag && base + part[tid] - 1 < cap) {
            const int32_t pos = base + part[tid] - 1;
            if (out) out[pos] = (int32_t)i;
            if (out64) out64[pos] = i;
        }
        __syncthreads();
        if (tid == 1023) base += part[1023];
        __syncthreads();
    }
    if (tid == 0 && count) count[0] = base;
}

// map2[k] = inv[sel[k]] (a map through an inverse permutation), k < n.
__global__ __launch_bounds__(256) void compose_kernel(const int32_t *inv, const int32_t *sel, const int32_t *pair,
                                                     int64_t n, int32_t *out) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    // sel[k] is a pivot row (or column); pair, when given, takes it to its
    // partner first
    const int32_t s = pair ? pair[sel[k]] : sel[k];
    out[k] = s >= 0 ? inv[s] : 0;   // (s < 0 only for vectors that are not a decomposition's)
}

// out[a][b] = Lbar (UPPER = false) or Ubar (UPPER = true) of the packed X at
// packed coordinates (i, j) = (rowmap[a], colmap[b]).
template <typename T, bool UPPER>
__global__ __launch_bounds__(256) void post_gather_kernel(const T *X, int64_t ldx, int64_t r, T *out, int64_t ldo,
                                                          int64_t rows, int64_t cols, const int32_t *rowmap,
                                                          const int32_t *colmap) {
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= cols) return;
    const int64_t j = colmap[b];
    for (int64_t a = blockIdx.y; a < rows; a += gridDim.y) {
        const int64_t i = rowmap[a];
        T v;
        if (!UPPER) v = (j < r) ? ((i > j) ? X[i * ldx + j] : (T)(i == j ? 1 : 0)) : (T)(i == j ? 1 : 0);
        else v = (i < r) ? ((j >= i) ? X[i * ldx + j] : (T)0) : (T)(i == j ? 1 : 0);
        out[a * ldo + b] = v;
    }
}

// out64[i] = in[i] (int32 -> int64), i < n.
__global__ __launch_bounds__(256) void widen_kernel(const int32_t *in, int64_t n, int64_t *out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = in[i];
}

// rank[q] = #{i < k_q : 0 <= rowpair[i] < t_q}: the rank of the leading
// k_q x t_q sub-matrix (one work-group per query).
__global__ __launch_bounds__(256) void leading_ranks_kernel(const int32_t *rowpair, int64_t m, const int64_t *ks,
                                                            const int64_t *ts, int64_t nq, int64_t *rank) {
    __shared__ int32_t red[256];
    const int64_t q = blockIdx.x;
    if (q >= nq) return;
    const int64_t k = min(max(ks[q], (int64_t)0), m), t = ts[q];
    int32_t c = 0;
    for (int64_t i = threadIdx.x; i < k; i += 256) {
        const int32_t j = rowpair[i];
        c += (j >= 0 && j < t) ? 1 : 0;
    }
    red[threadIdx.x] = c;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) rank[q] = red[0];
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_fill_i32(int32_t *x, int64_t n, int32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    PLUQ_LAUNCH(fill_i32_kernel, dim3(nblk(n)), dim3(256), 0, st, x, n, v);
    return hipGetLastError();
}

hipError_t launch_inverse_map(const int64_t *P, int64_t n, int32_t *inv, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    PLUQ_LAUNCH(inverse_map_kernel, dim3(nblk(n)), dim3(256), 0, st, P, n, inv);
    return hipGetLastError();
}

hipError_t launch_pair(const int64_t *P, const int64_t *Q, int64_t m, int64_t n, int64_t r, int32_t *rowpair,
                       int32_t *colpair, hipStream_t st) {
    if (r <= 0) return hipSuccess;
    PLUQ_LAUNCH(pair_kernel, dim3(nblk(r)), dim3(256), 0, st, P, Q, m, n, r, rowpair, colpair);
    return hipGetLastError();
}

hipError_t launch_compact(const int32_t *pair, int64_t lim, int64_t plim, int64_t cap, int32_t *out, int64_t *out64,
                          int64_t *count, hipStream_t st) {
    PLUQ_LAUNCH(compact_kernel, dim3(1), dim3(1024), 0, st, pair, lim, plim, cap, out, out64, count);
    return hipGetLastError();
}

hipError_t launch_compose(const int32_t *inv, const int32_t *sel, const int32_t *pair, int64_t n, int32_t *out,
                          hipStream_t st) {
    if (n <= 0) return hipSuccess;
    PLUQ_LAUNCH(compose_kernel, dim3(nblk(n)), dim3(256), 0, st, inv, sel, pair, n, out);
    return hipGetLastError();
}

hipError_t launch_post_gather(int dtype, bool upper, const void *X, int64_t ldx, int64_t r, void *out, int64_t ldo,
                              int64_t rows, int64_t cols, const int32_t *rowmap, const int32_t *colmap,
                              hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const dim3 grid(nblk(cols), (unsigned)std::min<int64_t>(rows, 32768));
#define PLUQ_PG(TT)                                                                                        \
    if (upper)                                                                                             \
        PLUQ_LAUNCH((post_gather_kernel<TT, true>), grid, dim3(256), 0, st, (const TT *)X, ldx, r, (TT *)out, \
                    ldo, rows, cols, rowmap, colmap);                                                      \
    else                                                                                                   \
        PLUQ_LAUNCH((post_gather_kernel<TT, false>), grid, dim3(256), 0, st, (const TT *)X, ldx, r, (TT *)out, \
                    ldo, rows, cols, rowmap, colmap);
    switch (dtype) {
    case DT_I64: PLUQ_PG(int64_t) break;
    case DT_F64: PLUQ_PG(double) break;
    case DT_I32: PLUQ_PG(int32_t) break;
    default: return hipErrorInvalidValue;
    }
#undef PLUQ_PG
    return hipGetLastError();
}

hipError_t launch_widen(const int32_t *in, int64_t n, int64_t *out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    PLUQ_LAUNCH(widen_kernel, dim3(nblk(n)), dim3(256), 0, st, in, n, out);
    return hipGetLastError();
}

hipError_t launch_leading_ranks(const int32_t *rowpair, int64_t m, const int64_t *ks, const int64_t *ts, int64_t nq,
                                int64_t *rank, hipStream_t st) {
    if (nq <= 0) return hipSuccess;
    PLUQ_LAUNCH(leading_ranks_kernel, dim3((unsigned)nq), dim3(256), 0, st, rowpair, m, ks, ts, nq, rank);
    return hipGetLastError();
}

}  // namespace pluq

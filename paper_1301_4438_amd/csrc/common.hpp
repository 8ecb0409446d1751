// Device-side helpers shared by the HIP kernels: element loads/stores for the
// three storage types and exact arithmetic modulo a prime p < 2^26.
//
// Field elements are handled as integer-valued doubles.  With p < 2^26 every
// product of two residues is below 2^52 and therefore exact, and sums of such
// products stay exact while their magnitude is below 2^53 (delayed
// reduction: one reduction for a whole sum of products, Section 6).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pluq {

enum DType : int { DT_I64 = 0, DT_F64 = 1, DT_I32 = 2 };

template <typename T> __device__ __forceinline__ double to_f64(T v) { return (double)v; }
template <typename T> __device__ __forceinline__ T from_f64(double v) { return (T)v; }

struct ModP {
    double p;     // the prime
    double pinv;  // 1/p rounded
    double half;  // floor(p/2): residues above it map to negative symmetric form
};

// Exact reduction of an integer-valued double x, |x| < 2^52, into [0, p).
// q = floor(x/p) computed with one rounded product is off by at most one
// (relative error <= 2^-52 on a quotient below 2^51); fma gives x - q p
// exactly since the true value is a small integer; two fix-ups follow.
__device__ __forceinline__ double mod_reduce(double x, const ModP &m) {
    double q = floor(x * m.pinv);
    double r = fma(-q, m.p, x);
    r = (r < 0.0) ? r + m.p : r;
    r = (r >= m.p) ? r - m.p : r;
    return r;
}

// Canonical [0, p) -> symmetric (-p/2, p/2].
__device__ __forceinline__ double to_sym(double v, const ModP &m) {
    return (v > m.half) ? v - m.p : v;
}

// a * b mod p for canonical or symmetric residues.
__device__ __forceinline__ double mod_mul(double a, double b, const ModP &m) {
    return mod_reduce(a * b, m);
}

// Inverse of a non-zero residue a (canonical, < p < 2^26) by the extended
// Euclidean algorithm on 32-bit integers.  Returns 0 for a == 0.
__device__ __forceinline__ double mod_inv(double a_, const ModP &m) {
    int32_t p = (int32_t)m.p;
    int32_t t = 0, nt = 1;
    int32_t r = p, nr = (int32_t)a_;
    while (nr != 0) {
        int32_t q = r / nr;
        int32_t tmp = t - q * nt; t = nt; nt = tmp;
        tmp = r - q * nr; r = nr; nr = tmp;
    }
    if (r != 1) return 0.0;
    if (t < 0) t += p;
    return (double)t;
}

// Symmetric reduction x - rint(x / p) p: for |x| < 2^52 the rounded quotient
// is within one of the exact one and the fma is exact, so the result is
// congruent to x with magnitude at most p/2 + 1, and zero exactly when p
// divides x.  Three dependent operations instead of the canonical
// reduction's five plus fix-ups: the form used on latency-bound chains.
__device__ __forceinline__ double sym_reduce(double x, const ModP &m) {
    return fma(-rint(x * m.pinv), m.p, x);
}

// Inverse of a non-zero canonical residue by Fermat's little theorem,
// a^(p-2) mod p, square-and-multiply on exact float64 products of symmetric
// residues: a fixed, wave-uniform sequence of about 2 log2(p) modular
// products, shorter in latency than the Euclidean algorithm's chain of
// integer divisions.  Returns the canonical inverse.
__device__ __forceinline__ double inv_fermat(double a, const ModP &mod) {
    uint32_t e = (uint32_t)mod.p - 2u;
    double r = 1.0, b = a;
    while (e) {
        if (e & 1u) r = sym_reduce(r * b, mod);
        b = sym_reduce(b * b, mod);
        e >>= 1;
    }
    return r < 0.0 ? r + mod.p : r;
}

__host__ __device__ inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace pluq

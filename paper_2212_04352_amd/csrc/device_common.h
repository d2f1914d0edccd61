// device_common.h -- complex helpers and the per-element right-hand side of
// the fTWA equation of motion shared by the evolution kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ftwa {

template <typename T> struct Cplx;
template <> struct Cplx<float> { using type = float2; };
template <> struct Cplx<double> { using type = double2; };
template <typename T> using cplx_t = typename Cplx<T>::type;

template <typename T> __device__ __forceinline__ T fma_rn(T a, T b, T c);
template <> __device__ __forceinline__ float fma_rn<float>(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}
template <> __device__ __forceinline__ double fma_rn<double>(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) {
    C r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename C> __device__ __forceinline__ C conj(C a) {
    C r;
    r.x = a.x;
    r.y = -a.y;
    return r;
}

// Packed index of element (a, b) of a spin block (upper triangle, rows
// contiguous) and whether the stored element is its transpose (a > b).
__device__ __forceinline__ int64_t packed_at(int N, int a, int b, bool& transposed) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    transposed = a > b;
    return (int64_t)lo * N - (int64_t)lo * (lo - 1) / 2 + (hi - lo);
}

// Neighbour sums of element (i, j) of one spin block X (packed,
// trajectory-innermost with leading dimension ld; trajectory m):
//   col = sum_{k in nb(j)} X_ik,  row = sum_{k in nb(i)} X_kj,
// each as (v0 + v1) + v2 over the neighbours in ascending order, a missing
// neighbour (degree < 3) an exact zero.  nbj, nbi: the sites' neighbour
// rows (x, y, z ascending, w = degree; wave-uniform).  All six loads are
// issued before any sum; a missing neighbour's load reads element (i, j)
// itself.
template <typename T>
__device__ __forceinline__ void neighbour_sums(const cplx_t<T>* X, int64_t ld, int N, int4 nbj,
                                               int4 nbi, int i, int j, int64_t m,
                                               cplx_t<T>& col, cplx_t<T>& row) {
    using C = cplx_t<T>;
    const int kc[3] = {nbj.x, nbj.y, nbj.z};
    const int kr[3] = {nbi.x, nbi.y, nbi.z};
    C c[3], r[3];
    bool tc[3], tr[3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        const int k1 = n < nbj.w ? kc[n] : j;
        const int k2 = n < nbi.w ? kr[n] : i;
        c[n] = X[packed_at(N, i, k1, tc[n]) * ld + m];
        r[n] = X[packed_at(N, k2, j, tr[n]) * ld + m];
    }
#pragma unroll
    for (int n = 0; n < 3; ++n) {
        if (tc[n]) c[n].y = -c[n].y;
        if (tr[n]) r[n].y = -r[n].y;
        if (n >= nbj.w) c[n].x = c[n].y = 0;
        if (n >= nbi.w) r[n].x = r[n].y = 0;
    }
    col = cadd(cadd(c[0], c[1]), c[2]);
    row = cadd(cadd(r[0], r[1]), r[2]);
}

// f = i [ t (col - row) + a rho ] evaluated as: g = t*(col - row) per
// component, g = fma(a, rho, g) per component, f = (-g.im, g.re), where
// a = U (d_i - d_j) with d the other spin's diagonal (Eq. (6); the 1/2 of
// (rho_kk + 1/2) cancels between the two interaction terms).
template <typename T>
__device__ __forceinline__ cplx_t<T> rhs_element(cplx_t<T> col, cplx_t<T> row, cplx_t<T> rho,
                                                 T t, T a) {
    T gr = t * (col.x - row.x);
    T gi = t * (col.y - row.y);
    gr = fma_rn<T>(a, rho.x, gr);
    gi = fma_rn<T>(a, rho.y, gi);
    cplx_t<T> f;
    f.x = -gi;
    f.y = gr;
    return f;
}

// Runge-Kutta coefficient sets in the working precision (formed in FP64 and
// rounded once).
template <typename T> struct RKCoef {
    T half, full, sixth, two;
};

}  // namespace ftwa

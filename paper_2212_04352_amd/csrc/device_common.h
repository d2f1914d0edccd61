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

// f = i [ t (col - row) + a rho ] evaluated as: g = t*(col - row) per
// component, g = fma(a, rho, g) per component, f = (-g.im, g.re), where
// a = U (d_i - d_j) with d the other spin's diagonal (Eq. (5); the 1/2 of
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

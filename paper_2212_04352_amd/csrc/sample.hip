// sample.hip -- Gaussian initial phase-space points (Eq. (7) of
// arXiv:2212.04352, amplitude from the covariance of Appendix A.3; for a
// thermal initial state also the diagonal fluctuation of that covariance).
//
// One thread per (spin, packed element, trajectory); the trajectory index is
// the fastest grid dimension so that every wave stores 64 consecutive
// trajectories of one element (the packed layout keeps them contiguous).
#include "device_common.h"
#include "ftwa_internal.h"
#include "philox.h"

namespace ftwa {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void sample_kernel(int N, int64_t P, int64_t n_traj,
                                                     int64_t traj_offset, uint32_t instance,
                                                     uint64_t seed, const double* __restrict__ n0,
                                                     const double* __restrict__ shift,
                                                     const uint32_t* __restrict__ elem,
                                                     cplx_t<T>* __restrict__ rho, int thermal) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_traj) return;
    const int64_t row = blockIdx.y;  // s * P + p
    const int s = row >= P ? 1 : 0;
    const int64_t p = row - (int64_t)s * P;
    const uint32_t ij = elem[p];
    const int i = (int)(ij & 0xffffu), j = (int)(ij >> 16);
    const double ni = n0[s * N + i], nj = n0[s * N + j];
    double re = 0.0, im = 0.0;
    if (i == j) {
        re = ni - 0.5;
        if (shift) re += shift[s * N + i];
        const double var = ni * (1.0 - ni);  // thermal state: Var rho_ii (Appendix A.3)
        if (thermal && var != 0.0) {
            const PhiloxBlock b = philox4x32_10(
                {(uint32_t)i, (instance << 1) | (uint32_t)s, (uint32_t)(traj_offset + m), 2u}, seed);
            const double scale = 1.0 / 9007199254740992.0;  // 2^-53
            const double u1 = (double)(b.bits53_first() + 1u) * scale;
            const double u2 = (double)b.bits53_second() * scale;
            const double g = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.14159265358979323846 * u2);
            re += sqrt(var) * g;
        }
    } else {
        const double var = 0.5 * ((ni + nj) - (2.0 * ni) * nj);
        if (var != 0.0) {
            const uint32_t pair = (uint32_t)(i * N - (i * (i + 1)) / 2 + (j - i - 1));
            const PhiloxBlock b = philox4x32_10(
                {pair, (instance << 1) | (uint32_t)s, (uint32_t)(traj_offset + m), 0u}, seed);
            const double scale = 1.0 / 9007199254740992.0;  // 2^-53
            const double u1 = (double)(b.bits53_first() + 1u) * scale;
            const double u2 = (double)b.bits53_second() * scale;
            const double radius = sqrt(-log(u1));
            const double theta = 2.0 * 3.14159265358979323846 * u2;
            const double amp = sqrt(var);
            re = amp * (radius * cos(theta));
            im = amp * (radius * sin(theta));
        }
    }
    cplx_t<T> v;
    v.x = (T)re;
    v.y = (T)im;
    rho[row * n_traj + m] = v;
}

}  // namespace

ftwa_status launch_sample(const ftwa_instance& in, const DeviceTables& tab, uint64_t seed,
                          ftwa_dtype dtype, bool thermal, hipStream_t stream) {
    const int N = in.lat->N;
    const int64_t P = packed_count(N);
    if (in.n_traj == 0) return FTWA_OK;
    const dim3 block(256);
    const dim3 grid((unsigned)((in.n_traj + 255) / 256), (unsigned)(2 * P));
    if (dtype == FTWA_F64)
        hipLaunchKernelGGL(sample_kernel<double>, grid, block, 0, stream, N, P, in.n_traj,
                           in.traj_offset, in.instance, seed, in.n0, in.n_shift, tab.elem,
                           static_cast<double2*>(in.rho), thermal ? 1 : 0);
    else
        hipLaunchKernelGGL(sample_kernel<float>, grid, block, 0, stream, N, P, in.n_traj,
                           in.traj_offset, in.instance, seed, in.n0, in.n_shift, tab.elem,
                           static_cast<float2*>(in.rho), thermal ? 1 : 0);
    FTWA_LAUNCH_CHECK("sample_kernel");
    return FTWA_OK;
}

}  // namespace ftwa

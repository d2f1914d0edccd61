// api.hip -- the extern "C" entry points of libftwa that queue device work:
// sampling, observables, unpacking (time evolution: evolve.hip).  Arguments are checked
// here, on the host, before anything is launched.
#include <algorithm>
#include <string>

#include "device_common.h"
#include "ftwa_internal.h"

namespace ftwa {

namespace {

template <typename T>
__global__ __launch_bounds__(256) void observables_kernel(int D, double invM, int64_t n_rec,
                                                          const double* __restrict__ S1,
                                                          const double* __restrict__ S2,
                                                          double* __restrict__ C,
                                                          double* __restrict__ g2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t DD = (int64_t)D * D;
    if (e >= n_rec * DD) return;
    const int64_t r = e / DD;
    const int a = (int)((e - r * DD) / D), b = (int)(e - r * DD - (int64_t)a * D);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int64_t n2 = (int64_t)D * (D + 1) / 2;
    const double mab = S2[r * n2 + (int64_t)lo * D - (int64_t)lo * (lo - 1) / 2 + (hi - lo)] * invM;
    const double ma = S1[r * D + a] * invM, mb = S1[r * D + b] * invM;
    if (C) C[e] = mab - ma * mb;
    if (g2) g2[e] = (mab + 0.5 * (ma + mb) + 0.25) / ((ma + 0.5) * (mb + 0.5));
}

__global__ __launch_bounds__(256) void occupation_kernel(int64_t count, double invM,
                                                         const double* __restrict__ S1,
                                                         double* __restrict__ n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) n[e] = S1[e] * invM + 0.5;
}

template <typename C>
__global__ __launch_bounds__(256) void unpack_kernel(int N, int64_t n_traj, const C* __restrict__ rho,
                                                     C* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = (int64_t)2 * N * N;
    if (e >= per * n_traj) return;
    const int64_t m = e / per;
    const int64_t rem = e - m * per;
    const int s = (int)(rem / ((int64_t)N * N));
    const int i = (int)((rem / N) % N), j = (int)(rem % N);
    const int64_t P = (int64_t)N * (N + 1) / 2;
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int64_t p = (int64_t)lo * N - (int64_t)lo * (lo - 1) / 2 + (hi - lo);
    C v = rho[((int64_t)s * P + p) * n_traj + m];
    if (i > j) v.y = -v.y;
    out[e] = v;
}

}  // namespace

ftwa_status check_instances(const ftwa_instance* inst, int n_inst, bool need_moments,
                            const char* who) {
    if (!inst || n_inst < 1) return fail(FTWA_EINVAL, std::string(who) + ": no instances");
    for (int k = 0; k < n_inst; ++k) {
        const ftwa_instance& in = inst[k];
        const std::string tag = std::string(who) + ": instance " + std::to_string(k);
        if (!in.lat) return fail(FTWA_EINVAL, tag + " has no lattice");
        if (in.n_traj < 0) return fail(FTWA_EINVAL, tag + " has n_traj < 0");
        if (in.traj_offset < 0 || in.traj_offset + in.n_traj > (int64_t)1 << 32)
            return fail(FTWA_EINVAL, tag + ": trajectory indices must fit 32 bits");
        if (in.n_traj > 0 && (!in.rho || !in.n0)) return fail(FTWA_EINVAL, tag + ": NULL rho or n0");
        if (need_moments && (!in.S1 || !in.S2)) return fail(FTWA_EINVAL, tag + ": NULL S1 or S2");
        if (in.instance >= (1u << 31)) return fail(FTWA_EINVAL, tag + ": instance id too large");
        if (in.v_site && !in.v_env) return fail(FTWA_EINVAL, tag + ": v_site without v_env");
        if (in.u_mat && in.inv)
            return fail(FTWA_EINVAL, tag + ": invariant monitors hold the on-site energy, not u_mat");
        if (in.hop_w && in.inv)
            return fail(FTWA_EINVAL, tag + ": invariant monitors hold the real-hopping energy");
    }
    return FTWA_OK;
}

KernelTimer::~KernelTimer() {
    for (hipEvent_t e : events_) (void)hipEventDestroy(e);
}

ftwa_status KernelTimer::begin(hipStream_t s) {
    if (!enabled_) return FTWA_OK;
    hipEvent_t e;
    FTWA_HIP_TRY(hipEventCreate(&e));
    events_.push_back(e);
    FTWA_HIP_TRY(hipEventRecord(e, s));
    return FTWA_OK;
}

ftwa_status KernelTimer::end(hipStream_t s, int64_t launches, double work) {
    if (!enabled_) return FTWA_OK;
    hipEvent_t e;
    FTWA_HIP_TRY(hipEventCreate(&e));
    events_.push_back(e);
    FTWA_HIP_TRY(hipEventRecord(e, s));
    launches_ += launches;
    work_ += work;
    return FTWA_OK;
}

ftwa_status KernelTimer::finish(double* ms, int64_t* launches, double* work) {
    if (!enabled_) return FTWA_OK;
    double total = 0.0;
    if (!events_.empty()) FTWA_HIP_TRY(hipEventSynchronize(events_.back()));
    for (size_t k = 0; k + 1 < events_.size(); k += 2) {
        float dt = 0.f;
        FTWA_HIP_TRY(hipEventElapsedTime(&dt, events_[k], events_[k + 1]));
        total += dt;
    }
    if (ms) *ms = total;
    if (launches) *launches = launches_;
    if (work) *work = work_;
    return FTWA_OK;
}


namespace {
ftwa_status sample_all(const ftwa_instance* inst, int n_inst, uint64_t seed, ftwa_dtype dtype,
                       bool thermal, void* stream, const char* who) {
    ftwa_status st = check_instances(inst, n_inst, false, who);
    if (st != FTWA_OK) return st;
    if (dtype != FTWA_F64 && dtype != FTWA_F32) return fail(FTWA_EINVAL, "unknown dtype");
    for (int k = 0; k < n_inst; ++k) {
        DeviceTables tab;
        if ((st = device_tables(inst[k].lat, &tab)) != FTWA_OK) return st;
        if ((st = launch_sample(inst[k], tab, seed, dtype, thermal, (hipStream_t)stream)) !=
            FTWA_OK)
            return st;
    }
    return FTWA_OK;
}
}  // namespace
}  // namespace ftwa

using namespace ftwa;

extern "C" {

ftwa_status ftwa_sample(const ftwa_instance* inst, int n_inst, uint64_t seed, ftwa_dtype dtype,
                        void* stream) {
    return sample_all(inst, n_inst, seed, dtype, false, stream, "ftwa_sample");
}

ftwa_status ftwa_sample_thermal(const ftwa_instance* inst, int n_inst, uint64_t seed,
                                ftwa_dtype dtype, void* stream) {
    return sample_all(inst, n_inst, seed, dtype, true, stream, "ftwa_sample_thermal");
}

ftwa_status ftwa_observables(int n_sites, int64_t M, int n_rec, const double* S1, const double* S2,
                             double* n_out, double* C_out, double* g2_out, void* stream_) {
    if (n_sites < 1 || n_sites > kMaxSites) return fail(FTWA_EINVAL, "n_sites out of range");
    if (M < 1) return fail(FTWA_EINVAL, "M < 1");
    if (n_rec < 0) return fail(FTWA_EINVAL, "n_rec < 0");
    if (!S1 || !S2 || !n_out) return fail(FTWA_EINVAL, "NULL S1, S2 or n_out");
    hipStream_t stream = (hipStream_t)stream_;
    const int D = 2 * n_sites;
    const double invM = 1.0 / (double)M;
    const int64_t cnt = (int64_t)n_rec * D;
    if (cnt == 0) return FTWA_OK;
    hipLaunchKernelGGL(occupation_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream,
                       cnt, invM, S1, n_out);
    if (C_out || g2_out) {
        const int64_t tot = cnt * D;
        hipLaunchKernelGGL(observables_kernel<double>, dim3((unsigned)((tot + 255) / 256)), dim3(256),
                           0, stream, D, invM, (int64_t)n_rec, S1, S2, C_out, g2_out);
    }
    FTWA_LAUNCH_CHECK("observables");
    return FTWA_OK;
}

ftwa_status ftwa_unpack(int n_sites, int64_t n_traj, ftwa_dtype dtype, const void* rho, void* out,
                        void* stream_) {
    if (n_sites < 1 || n_sites > kMaxSites || n_traj < 0) return fail(FTWA_EINVAL, "bad sizes");
    if (n_traj == 0) return FTWA_OK;
    if (!rho || !out) return fail(FTWA_EINVAL, "NULL pointer");
    const int64_t tot = (int64_t)2 * n_sites * n_sites * n_traj;
    const dim3 grid((unsigned)((tot + 255) / 256));
    hipStream_t stream = (hipStream_t)stream_;
    if (dtype == FTWA_F64)
        hipLaunchKernelGGL(unpack_kernel<double2>, grid, dim3(256), 0, stream, n_sites, n_traj,
                           static_cast<const double2*>(rho), static_cast<double2*>(out));
    else if (dtype == FTWA_F32)
        hipLaunchKernelGGL(unpack_kernel<float2>, grid, dim3(256), 0, stream, n_sites, n_traj,
                           static_cast<const float2*>(rho), static_cast<float2*>(out));
    else
        return fail(FTWA_EINVAL, "unknown dtype");
    FTWA_LAUNCH_CHECK("unpack_kernel");
    return FTWA_OK;
}

}  // extern "C"

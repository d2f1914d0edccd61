// api.hip -- the extern "C" entry points of libftwa that queue device work:
// sampling, time evolution, observables, unpacking.  Arguments are checked
// here, on the host, before anything is launched.
#include <algorithm>
#include <string>

#include "device_common.h"
#include "ftwa_internal.h"

namespace ftwa {

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t cplx_bytes(ftwa_dtype d) { return d == FTWA_F64 ? 16 : 8; }

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
    }
    return FTWA_OK;
}

// How one instance is integrated, and where its scratch sits in the workspace.
struct InstancePlan {
    ftwa_path path = FTWA_PATH_STREAM;
    ResidentPlan res;
    int64_t chunk = 0;       // trajectories per pass
    size_t off_acc = 0, off_ya = 0, off_yb = 0, off_x = 0, off_mom = 0, off_mb = 0, off_inv = 0;
    size_t total = 0;
};

struct EvolvePlan {
    int64_t n_rec = 0;
    std::vector<InstancePlan> inst;
    size_t total = 0;        // max over instances (passes run one after another)
};

constexpr size_t kRecordBudget = (size_t)4 << 30;  // bytes of FP64 records per pass

ftwa_status plan_evolve(const ftwa_instance* inst, int n_inst, int64_t n_steps, int record_every,
                        ftwa_dtype dtype, const ftwa_tuning* tune, EvolvePlan* plan) {
    if (dtype != FTWA_F64 && dtype != FTWA_F32) return fail(FTWA_EINVAL, "unknown dtype");
    if (n_steps < 0) return fail(FTWA_EINVAL, "n_steps < 0");
    if (record_every < 1) return fail(FTWA_EINVAL, "record_every < 1");
    EvolvePlan p;
    p.n_rec = n_records(n_steps, record_every);
    if (p.n_rec > 65535) return fail(FTWA_EINVAL, "more than 65535 records");
    const ftwa_path want = tune ? tune->path : FTWA_PATH_AUTO;
    if (want != FTWA_PATH_AUTO && want != FTWA_PATH_STREAM && want != FTWA_PATH_RESIDENT)
        return fail(FTWA_EINVAL, "unknown path");
    for (int k = 0; k < n_inst; ++k) {
        const int N = inst[k].lat->N;
        const int64_t P = packed_count(N);
        const int D = 2 * N;
        InstancePlan ip;
        DeviceTables tab;
        ftwa_status st = device_tables(inst[k].lat, &tab);
        if (st != FTWA_OK) return st;
        const int force = tune ? tune->resident_config : -1;
        if (force >= resident_config_count())
            return fail(FTWA_EINVAL, "resident_config out of range");
        const bool can_res = resident_plan(N, dtype, tab, &ip.res, force);
        if (force >= 0 && !can_res)
            return fail(FTWA_ENOTSUP, "the forced resident configuration does not fit");
        if (want == FTWA_PATH_RESIDENT && !can_res)
            return fail(FTWA_ENOTSUP, "no resident configuration fits this lattice and dtype");
        ip.path = (want == FTWA_PATH_STREAM || !can_res) ? FTWA_PATH_STREAM : FTWA_PATH_RESIDENT;
        const int64_t traj = std::max<int64_t>(inst[k].n_traj, 1);
        int64_t chunk;
        if (ip.path == FTWA_PATH_STREAM) {
            chunk = tune && tune->traj_chunk > 0 ? tune->traj_chunk : 4096;
        } else {
            chunk = tune && tune->traj_chunk > 0 ? tune->traj_chunk : traj;
            chunk = std::min(chunk, resident_max_traj(ip.res));
        }
        const int64_t rec_cap = std::max<int64_t>(
            64, (int64_t)(kRecordBudget / ((size_t)p.n_rec * D * sizeof(double))));
        chunk = std::max<int64_t>(1, std::min({chunk, traj, rec_cap}));
        ip.chunk = chunk;
        size_t off = 0;
        if (ip.path == FTWA_PATH_STREAM) {
            const size_t state = (size_t)2 * P * chunk * cplx_bytes(dtype);
            ip.off_acc = off; off = align_up(off + state);
            ip.off_ya = off; off = align_up(off + state);
            ip.off_yb = off; off = align_up(off + state);
        } else {
            ip.off_mb = off; off = align_up(off + resident_mailbox_bytes(ip.res, N, dtype, chunk));
        }
        ip.off_x = off; off = align_up(off + (size_t)p.n_rec * D * chunk * sizeof(double));
        ip.off_mom = off; off = align_up(off + moments_workspace_bytes(D, chunk, p.n_rec));
        if (inst[k].inv) {  // per-trajectory hop/frob sums of every record
            ip.off_inv = off;
            off = align_up(off + (size_t)p.n_rec * 4 * chunk * sizeof(double));
        }
        ip.total = off;
        p.total = std::max(p.total, off);
        p.inst.push_back(ip);
    }
    *plan = p;
    return FTWA_OK;
}

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

}  // namespace ftwa

using namespace ftwa;

extern "C" {

ftwa_status ftwa_sample(const ftwa_instance* inst, int n_inst, uint64_t seed, ftwa_dtype dtype,
                        void* stream) {
    ftwa_status st = check_instances(inst, n_inst, false, "ftwa_sample");
    if (st != FTWA_OK) return st;
    if (dtype != FTWA_F64 && dtype != FTWA_F32) return fail(FTWA_EINVAL, "unknown dtype");
    for (int k = 0; k < n_inst; ++k) {
        DeviceTables tab;
        if ((st = device_tables(inst[k].lat, &tab)) != FTWA_OK) return st;
        if ((st = launch_sample(inst[k], tab, seed, dtype, (hipStream_t)stream)) != FTWA_OK) return st;
    }
    return FTWA_OK;
}

ftwa_status ftwa_evolve_workspace_size(const ftwa_instance* inst, int n_inst, int64_t n_steps,
                                       int record_every, ftwa_dtype dtype,
                                       const ftwa_tuning* tune, size_t* bytes) {
    if (!bytes) return fail(FTWA_EINVAL, "bytes is NULL");
    ftwa_status st = check_instances(inst, n_inst, false, "ftwa_evolve_workspace_size");
    if (st != FTWA_OK) return st;
    EvolvePlan plan;
    if ((st = plan_evolve(inst, n_inst, n_steps, record_every, dtype, tune, &plan)) != FTWA_OK)
        return st;
    *bytes = plan.total;
    return FTWA_OK;
}

ftwa_status ftwa_evolve(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                        int record_every, ftwa_dtype dtype, const ftwa_tuning* tune,
                        void* workspace, size_t workspace_bytes, void* stream_) {
    ftwa_status st = check_instances(inst, n_inst, true, "ftwa_evolve");
    if (st != FTWA_OK) return st;
    EvolvePlan plan;
    if ((st = plan_evolve(inst, n_inst, n_steps, record_every, dtype, tune, &plan)) != FTWA_OK)
        return st;
    if (workspace_bytes < plan.total || (!workspace && plan.total > 0))
        return fail(FTWA_EINVAL, "workspace smaller than ftwa_evolve_workspace_size");
    hipStream_t stream = (hipStream_t)stream_;
    char* ws = static_cast<char*>(workspace);
    KernelTimer timer(tune && tune->kernel_ms);
    std::vector<int*> error_words;
    for (int k = 0; k < n_inst; ++k) {
        const ftwa_instance& in = inst[k];
        const InstancePlan& ip = plan.inst[k];
        DeviceTables tab;
        if ((st = device_tables(in.lat, &tab)) != FTWA_OK) return st;
        const int N = in.lat->N;
        const int D = 2 * N;
        const int64_t P = packed_count(N);
        if ((st = zero_fill(in.S1, plan.n_rec * D, stream)) != FTWA_OK) return st;
        if ((st = zero_fill(in.S2, plan.n_rec * s2_count(D), stream)) != FTWA_OK) return st;
        if (in.inv && (st = zero_fill(in.inv, plan.n_rec * 4, stream)) != FTWA_OK) return st;
        double* X = reinterpret_cast<double*>(ws + ip.off_x);
        double* parts = in.inv ? reinterpret_cast<double*>(ws + ip.off_inv) : nullptr;
        auto finish_pass = [&](int64_t Mc) -> ftwa_status {
            ftwa_status s2 = moments_accumulate(D, Mc, plan.n_rec, X, in.S1, in.S2,
                                                ws + ip.off_mom, stream);
            if (s2 != FTWA_OK || !in.inv) return s2;
            return invariants_accumulate(N, Mc, plan.n_rec, in.lat->t, in.U, X, parts, in.inv,
                                         stream);
        };
        if (ip.path == FTWA_PATH_RESIDENT) {
            int* err = resident_error_word(ip.res, N, ip.chunk, ws + ip.off_mb);
            if (err) {
                if ((st = zero_words(reinterpret_cast<unsigned*>(err), 1, stream)) != FTWA_OK) return st;
                error_words.push_back(err);
            }
            for (int64_t m0 = 0; m0 < in.n_traj; m0 += ip.chunk) {
                ResidentPass pass;
                pass.N = N;
                pass.Mc = std::min(ip.chunk, in.n_traj - m0);
                pass.rho = static_cast<char*>(in.rho) + (size_t)m0 * cplx_bytes(dtype);
                pass.ldr = in.n_traj;
                pass.t = in.lat->t;
                pass.U = in.U;
                pass.dt = dt;
                pass.n_steps = n_steps;
                pass.record_every = record_every;
                pass.X = X;
                pass.inv_parts = parts;
                pass.mailbox = ws + ip.off_mb;
                if ((st = padded_descriptors(in.lat, ip.res.even_slots, ip.res.odd_slots,
                                             &pass.desc)) != FTWA_OK)
                    return st;
                if ((st = timer.begin(stream)) != FTWA_OK) return st;
                if ((st = resident_run(ip.res, pass, stream)) != FTWA_OK) return st;
                if ((st = timer.end(stream, 1, (double)pass.Mc * n_steps)) != FTWA_OK) return st;
                if ((st = finish_pass(pass.Mc)) != FTWA_OK) return st;
            }
            continue;
        }
        for (int64_t m0 = 0; m0 < in.n_traj; m0 += ip.chunk) {
            const int64_t Mc = std::min(ip.chunk, in.n_traj - m0);
            StreamChunk c;
            c.N = N;
            c.P = P;
            c.Mc = Mc;
            c.y = static_cast<char*>(in.rho) + (size_t)m0 * cplx_bytes(dtype);
            c.ldy = in.n_traj;
            c.acc = ws + ip.off_acc;
            c.ya = ws + ip.off_ya;
            c.yb = ws + ip.off_yb;
            c.t = in.lat->t;
            c.U = in.U;
            c.dt = dt;
            if ((st = record_diag(c, tab, dtype, X, stream)) != FTWA_OK) return st;
            if (parts && (st = record_inv(c, tab, dtype, parts, stream)) != FTWA_OK) return st;
            int64_t open_steps = 0;
            for (int64_t step = 1; step <= n_steps; ++step) {
                if (open_steps == 0 && (st = timer.begin(stream)) != FTWA_OK) return st;
                if ((st = stream_step(c, tab, dtype, stream)) != FTWA_OK) return st;
                ++open_steps;
                if (step % record_every == 0 || step == n_steps) {
                    if ((st = timer.end(stream, 4 * open_steps, (double)open_steps * Mc)) != FTWA_OK)
                        return st;
                    open_steps = 0;
                }
                if (step % record_every == 0) {
                    const int64_t r = step / record_every;
                    if ((st = record_diag(c, tab, dtype, X + r * D * Mc, stream)) != FTWA_OK)
                        return st;
                    if (parts && (st = record_inv(c, tab, dtype, parts + r * 4 * Mc, stream)) != FTWA_OK)
                        return st;
                }
            }
            if ((st = finish_pass(Mc)) != FTWA_OK) return st;
        }
    }
    if (tune && tune->kernel_ms)
        if ((st = timer.finish(tune->kernel_ms, tune->kernel_launches, tune->kernel_work)) != FTWA_OK)
            return st;
    for (const int* err : error_words) {
        bool timed_out = false;
        if ((st = resident_check_error(err, stream, &timed_out)) != FTWA_OK) return st;
        if (timed_out)
            return fail(FTWA_ETIMEOUT, "a spin-split workgroup pair timed out waiting for its partner");
    }
    // trajectories that became NaN or Inf are counted in inv[r][3]
    for (int k = 0; k < n_inst; ++k) {
        if (!inst[k].inv) continue;
        std::vector<double> h((size_t)plan.n_rec * 4);
        FTWA_HIP_TRY(hipMemcpyAsync(h.data(), inst[k].inv, h.size() * sizeof(double),
                                    hipMemcpyDeviceToHost, stream));
        FTWA_HIP_TRY(hipStreamSynchronize(stream));
        for (int64_t r = 0; r < plan.n_rec; ++r)
            if (h[(size_t)r * 4 + 3] > 0)
                return fail(FTWA_ENONFINITE, "instance " + std::to_string(k) +
                                                 ": a trajectory became non-finite by record " +
                                                 std::to_string(r));
    }
    return FTWA_OK;
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

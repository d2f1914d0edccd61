// evolve.hip -- ftwa_evolve and its batched forms: the plan of a run (which
// kernel path and configuration integrates each instance, how trajectories
// are split into passes, where every buffer sits in the workspace), the
// queueing of its launches, the HIP-graph form of the same launches, and the
// autotuner that picks resident configurations by timing them.
//
// Batching.  Instances whose resident configuration is the same form a group;
// each pass launches one persistent kernel per group over a device table of
// (instance, trajectory window) entries, so mixed lattice sizes and U values
// of a group run in one launch.  Instances that no resident configuration
// fits run on the stream path.  The per-element arithmetic does not depend on
// the grouping, the configuration or the pass split, so a batched run gives
// bitwise the same trajectories as one run per instance.
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ftwa_internal.h"

namespace ftwa {

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
size_t cplx_bytes(ftwa_dtype d) { return d == FTWA_F64 ? 16 : 8; }

constexpr size_t kRecordBudget = (size_t)4 << 30;  // FP64 record bytes per pass
constexpr int64_t kStreamChunk = 4096;

// Status block of a run at the start of its workspace (32-bit words): a
// marker, the timeout flag the multi-workgroup resident kernels set, the
// number of (instance, record) pairs whose invariant monitor counted a
// non-finite trajectory, and the first such pair as instance << 16 | record.
// Written only by kernels queued with the run, read by ftwa_evolve_check.
constexpr size_t kStatusBytes = 256;
constexpr uint32_t kStatusMagic = 0x46545741u;

__global__ void status_init_kernel(uint32_t* st) {
    if (threadIdx.x == 0) {
        st[0] = kStatusMagic;
        st[1] = 0u;
        st[2] = 0u;
        st[3] = 0xffffffffu;
    }
}

__global__ __launch_bounds__(64) void status_nonfinite_kernel(const double* __restrict__ inv,
                                                              int64_t n_rec, uint32_t inst,
                                                              uint32_t* st) {
    for (int64_t r = threadIdx.x; r < n_rec; r += blockDim.x)
        if (inv[r * 4 + 3] > 0.0) {
            atomicAdd(st + 2, 1u);
            atomicMin(st + 3, (inst << 16) | (uint32_t)r);
        }
}

// Launch-table entries travel to the device as kernel arguments (no host
// buffer has to outlive the call, and the write can be captured in a graph).
constexpr int kTableChunk = 16;
struct TableChunk {
    int n;
    ResidentInst e[kTableChunk];
};
static_assert(sizeof(ResidentInst) % 4 == 0, "table entries are copied as 32-bit words");
static_assert(sizeof(TableChunk) <= 3072, "kernel argument size");

__global__ __launch_bounds__(256) void write_table_kernel(ResidentInst* dst, TableChunk c) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(c.e);
    uint32_t* out = reinterpret_cast<uint32_t*>(dst);
    const int words = c.n * (int)(sizeof(ResidentInst) / 4);
    for (int w = threadIdx.x; w < words; w += blockDim.x) out[w] = src[w];
}

struct InstPlan {
    ftwa_path path = FTWA_PATH_STREAM;
    ResidentPlan res;
    int group = -1;
    int64_t chunk = 0;             // stream: trajectories per chunk; resident: per pass window
    size_t off_x = 0, off_inv = 0; // resident: this instance's record regions
    size_t off_hop = 0;            // resident with complex hopping: its ratio table
    size_t off_umat = 0;           // resident with a general interaction: u in dtype
};

struct LaunchDesc {                // one resident launch: a group in a pass
    int group = 0;
    int64_t first_entry = 0;       // into the uploaded table
    int n_entries = 0;
    int64_t n_items = 0;
    int64_t grid = 0;
    double work = 0;               // trajectory-steps
    bool unit_hop = true;          // every instance has t = 1
    bool potential = false;        // an instance carries an external potential
    bool hopping = false;          // every instance carries complex hopping
    bool interaction = false;      // every instance carries a general interaction
};

struct GroupPlan {
    int config = -1;
    size_t lds = 0;
    int Nmax = 0;
    std::vector<int> members;
    int64_t max_items = 0;
    size_t off_mb = 0;
};

struct Plan {
    int n_inst = 0;
    int64_t n_rec = 0, n_steps = 0;
    int record_every = 1;
    double dt = 0;
    ftwa_dtype dtype = FTWA_F64;
    int n_pass = 0;
    std::vector<InstPlan> inst;
    std::vector<GroupPlan> groups;
    std::vector<LaunchDesc> launches;  // pass-major
    // stream area
    size_t s_acc = 0, s_ya = 0, s_yb = 0, s_x = 0, s_mom = 0, s_inv = 0, s_D = 0, s_total = 0;
    size_t off_status = 0;  // the status block (kStatusBytes at the start of the workspace)
    // resident area
    size_t r_table = 0, r_mom = 0, r_total = 0;
    int64_t n_table = 0;
    size_t total = 0;
    // internal runs only (one instance): its state is stored at every record
    void* dump = nullptr;
    int64_t dump_stride = 0;
    // the launch table's entries, filled on the host by build_table and
    // written to r_table by kernels queued at the start of every run
    std::vector<ResidentInst> table;
    unsigned spin_limit = 0;   // 0: the kernels' default
    bool drop_partners = false;
};

void window(const Plan& p, const ftwa_instance& in, int k, int j, int64_t* m0, int64_t* Mc) {
    const int64_t c = p.inst[k].chunk;
    *m0 = std::min<int64_t>((int64_t)j * c, in.n_traj);
    *Mc = std::min<int64_t>(c, in.n_traj - *m0);
}

ftwa_status plan_evolve(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                        int record_every, ftwa_dtype dtype, const ftwa_tuning* tune, Plan* out) {
    if (dtype != FTWA_F64 && dtype != FTWA_F32) return fail(FTWA_EINVAL, "unknown dtype");
    if (n_steps < 0) return fail(FTWA_EINVAL, "n_steps < 0");
    if (record_every < 1) return fail(FTWA_EINVAL, "record_every < 1");
    Plan p;
    p.n_inst = n_inst;
    p.n_steps = n_steps;
    p.record_every = record_every;
    p.dt = dt;
    p.dtype = dtype;
    p.n_rec = n_records(n_steps, record_every);
    if (p.n_rec > 65535) return fail(FTWA_EINVAL, "more than 65535 records");
    const ftwa_path want = tune ? tune->path : FTWA_PATH_AUTO;
    if (want != FTWA_PATH_AUTO && want != FTWA_PATH_STREAM && want != FTWA_PATH_RESIDENT)
        return fail(FTWA_EINVAL, "unknown path");
    const int force = tune ? tune->resident_config : -1;
    if (force >= resident_config_count()) return fail(FTWA_EINVAL, "resident_config out of range");
    const int64_t user_chunk = tune && tune->traj_chunk > 0 ? tune->traj_chunk : 0;
    p.spin_limit = tune ? tune->spin_limit : 0;
    p.drop_partners = tune && tune->drop_partners;

    // ---- path and configuration of every instance
    // 8 config + 4 (general interaction) + 2 (complex hopping) + (external potential)
    std::map<int, int> group_of_config;
    for (int k = 0; k < n_inst; ++k) {
        InstPlan ip;
        const DeviceTables& tab = host_tables(inst[k].lat);
        const int N = inst[k].lat->N;
        int cfg = force;
        bool tuned_stream = false;
        if (cfg < 0 && want == FTWA_PATH_AUTO) {
            int c = -1;
            if (tuned_config(N, class_shape(tab), dtype, &c)) {
                if (c < 0) tuned_stream = true;
                cfg = c;
            }
        }
        // an external potential: the stream kernels, or a resident configuration
        // with the potential variant
        const bool pot = inst[k].v_site != nullptr;
        // a general interaction: the stream kernels, or a resident configuration
        // with the general-interaction variant (alone)
        const bool gint = inst[k].u_mat != nullptr;
        // complex hopping: the stream kernels, or a resident configuration with
        // the complex-hopping variant (alone)
        const bool hop = inst[k].hop_w != nullptr;
        const int n_var = (pot ? 1 : 0) + (hop ? 1 : 0) + (gint ? 1 : 0);
        if (n_var > 1 && (want == FTWA_PATH_RESIDENT || force >= 0))
            return fail(FTWA_ENOTSUP, "a potential, complex hopping and a general interaction "
                                      "together run on the stream path only");
        bool can_res = !tuned_stream && n_var <= 1 &&
                       resident_plan(N, dtype, tab, &ip.res, cfg, inst[k].inv == nullptr);
        if (gint && can_res) {
            // the configuration chosen for the on-site U, if it has the variant
            const int c0 = ip.res.config;
            can_res = resident_has_interaction(c0) &&
                      resident_plan(N, dtype, tab, &ip.res, c0, inst[k].inv == nullptr, false,
                                    false, true);
        }
        if (hop && can_res) {
            // the configuration chosen for real hopping, if it has the variant
            const int c0 = ip.res.config;
            can_res = resident_has_hop(c0) &&
                      resident_plan(N, dtype, tab, &ip.res, c0, inst[k].inv == nullptr, false,
                                    true);
        }
        if (pot && can_res) {
            // the configuration chosen without the potential, if it has the
            // potential variant (else the stream path)
            const int c0 = ip.res.config;
            can_res = resident_has_potential(c0) &&
                      resident_plan(N, dtype, tab, &ip.res, c0, inst[k].inv == nullptr, true);
        }
        if (force >= 0 && !can_res)
            return fail(FTWA_ENOTSUP, hop    ? "the forced resident configuration has no "
                                               "complex-hopping variant or does not fit"
                                      : gint ? "the forced resident configuration has no "
                                               "general-interaction variant or does not fit"
                                             : "the forced resident configuration does not fit");
        if (want == FTWA_PATH_RESIDENT && !can_res)
            return fail(FTWA_ENOTSUP, "no resident configuration fits this lattice and dtype");
        ip.path = (want == FTWA_PATH_STREAM || !can_res) ? FTWA_PATH_STREAM : FTWA_PATH_RESIDENT;
        if (ip.path == FTWA_PATH_RESIDENT) {
            // instances with a potential form groups of their own: their
            // launches run the potential variant, whose LDS layout holds the
            // profile and is sized for it
            const int key = 8 * ip.res.config + (gint ? 4 : 0) + (hop ? 2 : 0) + (pot ? 1 : 0);
            auto it = group_of_config.find(key);
            if (it == group_of_config.end()) {
                it = group_of_config.emplace(key, (int)p.groups.size()).first;
                GroupPlan g;
                g.config = ip.res.config;
                p.groups.push_back(g);
            }
            ip.group = it->second;
            GroupPlan& g = p.groups[ip.group];
            g.members.push_back(k);
            g.lds = std::max(g.lds, ip.res.lds);
            g.Nmax = std::max(g.Nmax, N);
        }
        p.inst.push_back(ip);
    }

    // ---- stream instances: chunks of trajectories, one after another
    size_t s_state = 0, s_x = 0, s_mom = 0, s_inv = 0, s_D = 0;
    for (int k = 0; k < n_inst; ++k) {
        InstPlan& ip = p.inst[k];
        if (ip.path != FTWA_PATH_STREAM) continue;
        const int N = inst[k].lat->N;
        const int D = 2 * N;
        const int64_t traj = std::max<int64_t>(inst[k].n_traj, 1);
        const int64_t rec_cap = std::max<int64_t>(
            64, (int64_t)(kRecordBudget / ((size_t)p.n_rec * D * sizeof(double))));
        int64_t chunk = user_chunk > 0 ? user_chunk : kStreamChunk;
        chunk = std::max<int64_t>(1, std::min({chunk, traj, rec_cap}));
        ip.chunk = chunk;
        s_state = std::max(s_state, (size_t)2 * packed_count(N) * chunk * cplx_bytes(dtype));
        s_x = std::max(s_x, (size_t)p.n_rec * D * chunk * sizeof(double));
        s_mom = std::max(s_mom, moments_workspace_bytes(D, chunk, p.n_rec));
        if (inst[k].inv) s_inv = std::max(s_inv, (size_t)p.n_rec * 4 * chunk * sizeof(double));
        if (inst[k].u_mat) s_D = std::max(s_D, (size_t)2 * N * chunk * sizeof(double));
    }
    size_t off = kStatusBytes;  // the run's status block comes first
    p.s_acc = off; off = align_up(off + s_state);
    p.s_ya = off;  off = align_up(off + s_state);
    p.s_yb = off;  off = align_up(off + s_state);
    p.s_x = off;   off = align_up(off + s_x);
    p.s_mom = off; off = align_up(off + s_mom);
    p.s_inv = off; off = align_up(off + s_inv);
    p.s_D = off;   off = align_up(off + s_D);
    p.s_total = off;

    // ---- resident instances: passes over trajectory windows.  Their area
    // follows the stream area (no overlap: the launch tables are uploaded
    // before the stream-path instances run, and must survive them)
    size_t rec_bytes = 0;
    for (int k = 0; k < n_inst; ++k) {
        if (p.inst[k].path != FTWA_PATH_RESIDENT) continue;
        const int D = 2 * inst[k].lat->N;
        rec_bytes += (size_t)p.n_rec * (D + (inst[k].inv ? 4 : 0)) * inst[k].n_traj * sizeof(double);
    }
    int64_t n_pass_goal = std::max<int64_t>(1, (int64_t)((rec_bytes + kRecordBudget - 1) / kRecordBudget));
    p.n_pass = 0;
    for (int k = 0; k < n_inst; ++k) {
        InstPlan& ip = p.inst[k];
        if (ip.path != FTWA_PATH_RESIDENT) continue;
        const int64_t M = inst[k].n_traj;
        int64_t c;
        if (user_chunk > 0) {
            c = user_chunk;
        } else {
            // whole rounds of the trajectories the group runs at once
            const int64_t align = std::max<int64_t>(
                1, resident_concurrency(ip.res.config, p.groups[ip.group].lds));
            c = (M + n_pass_goal - 1) / n_pass_goal;
            c = (c + align - 1) / align * align;
        }
        c = std::max<int64_t>(1, std::min(c, std::max<int64_t>(M, 1)));
        ip.chunk = c;
        p.n_pass = std::max<int>(p.n_pass, (int)((M + c - 1) / c));
    }
    off = p.s_total;
    for (int k = 0; k < n_inst; ++k) {
        InstPlan& ip = p.inst[k];
        if (ip.path != FTWA_PATH_RESIDENT) continue;
        const int D = 2 * inst[k].lat->N;
        ip.off_x = off; off = align_up(off + (size_t)p.n_rec * D * ip.chunk * sizeof(double));
        if (inst[k].hop_w) {
            ip.off_hop = off;
            off = align_up(off + (size_t)(2 * p.n_steps + 1) * inst[k].lat->N * 3 *
                                     cplx_bytes(p.dtype));
        }
        if (inst[k].u_mat) {
            ip.off_umat = off;
            off = align_up(off + (size_t)umat_rows(inst[k].lat->N) * inst[k].lat->N *
                                   cplx_bytes(p.dtype) / 2);
        }
        if (inst[k].inv) {
            ip.off_inv = off;
            off = align_up(off + (size_t)p.n_rec * 4 * ip.chunk * sizeof(double));
        }
    }
    size_t r_mom = 0;
    for (int k = 0; k < n_inst; ++k)
        if (p.inst[k].path == FTWA_PATH_RESIDENT)
            r_mom = std::max(r_mom, moments_workspace_bytes(2 * inst[k].lat->N, p.inst[k].chunk,
                                                            p.n_rec));
    p.r_mom = off; off = align_up(off + r_mom);
    // launches and their table entries
    int64_t entry = 0;
    for (int j = 0; j < p.n_pass; ++j)
        for (int gi = 0; gi < (int)p.groups.size(); ++gi) {
            GroupPlan& g = p.groups[gi];
            LaunchDesc L;
            L.group = gi;
            L.first_entry = entry;
            for (int k : g.members) {
                int64_t m0, Mc;
                window(p, inst[k], k, j, &m0, &Mc);
                if (Mc <= 0) continue;
                const int64_t per = resident_item_traj(g.config);
                L.n_items += (Mc + per - 1) / per;
                L.work += (double)Mc * n_steps;
                if (inst[k].lat->t != 1.0) L.unit_hop = false;
                if (inst[k].v_site) L.potential = true;
                if (inst[k].hop_w) L.hopping = true;
                if (inst[k].u_mat) L.interaction = true;
                ++L.n_entries;
            }
            entry += L.n_entries;
            g.max_items = std::max(g.max_items, L.n_items);
            L.grid = resident_grid(g.config, g.lds, std::max<int64_t>(L.n_items, 1));
            p.launches.push_back(L);
        }
    p.n_table = entry;
    for (GroupPlan& g : p.groups) {
        g.off_mb = off;
        off = align_up(off + resident_mailbox_bytes(g.config, g.Nmax, std::max<int64_t>(g.max_items, 1)));
    }
    p.r_table = off; off = align_up(off + (size_t)std::max<int64_t>(entry, 1) * sizeof(ResidentInst));
    p.r_total = off;
    p.total = p.r_total;
    *out = std::move(p);
    return FTWA_OK;
}

// Host work before the launches, nothing queued: the launch-table entries
// (their descriptor tables looked up; ftwa_lattice_upload created them) and
// the kernels' LDS limits.  Not under graph capture.
ftwa_status build_table(Plan& p, const ftwa_instance* inst, char* ws) {
    ftwa_status st;
    p.table.clear();
    p.table.reserve((size_t)p.n_table);
    for (int j = 0; j < p.n_pass; ++j)
        for (const GroupPlan& g : p.groups) {
            int64_t item0 = 0;
            const int64_t per = resident_item_traj(g.config);
            for (int k : g.members) {
                int64_t m0, Mc;
                window(p, inst[k], k, j, &m0, &Mc);
                if (Mc <= 0) continue;
                const InstPlan& ip = p.inst[k];
                ResidentInst e;
                e.N = inst[k].lat->N;
                e.P = (int)packed_count(e.N);
                e.Mc = Mc;
                e.rho = static_cast<char*>(inst[k].rho) + (size_t)m0 * cplx_bytes(p.dtype);
                e.ldr = inst[k].n_traj;
                e.part_words = 0;
                e.hmax = 0;
                if (resident_parts(g.config) > 1) {
                    if ((st = split_tables(inst[k].lat, resident_parts(g.config),
                                           ip.res.even_slots, ip.res.odd_slots, ip.res.bnd_entry,
                                           (int)cplx_bytes(p.dtype), &e.desc, &e.part_words,
                                           &e.hmax)) != FTWA_OK)
                        return st;
                } else if ((st = padded_descriptors(inst[k].lat, ip.res.even_slots,
                                                    ip.res.odd_slots, (int)cplx_bytes(p.dtype),
                                                    resident_spins(g.config) == 1, &e.desc)) !=
                           FTWA_OK) {
                    return st;
                }
                DeviceTables tab;
                if ((st = device_tables(inst[k].lat, &tab)) != FTWA_OK) return st;
                e.ord = tab.ord;
                e.nb = tab.nb;
                e.dpos = tab.dpos;
                e.t = inst[k].lat->t;
                e.U = inst[k].U;
                e.X = reinterpret_cast<double*>(ws + ip.off_x);
                e.inv_parts = inst[k].inv ? reinterpret_cast<double*>(ws + ip.off_inv) : nullptr;
                e.item0 = item0;
                item0 += (Mc + per - 1) / per;
                e.dump = p.dump ? static_cast<char*>(p.dump) + (size_t)m0 * cplx_bytes(p.dtype)
                                : nullptr;
                e.dump_stride = p.dump_stride;
                e.v_site = inst[k].v_site;
                e.v_env = inst[k].v_env;
                e.hop = inst[k].hop_w ? ws + ip.off_hop : nullptr;
                e.umat = inst[k].u_mat ? ws + ip.off_umat : nullptr;
                e.u_lds = inst[k].u_mat && ip.res.u_lds ? 1 : 0;
                p.table.push_back(e);
            }
        }
    // the stream path's tables must be on this device as well
    for (int k = 0; k < p.n_inst; ++k) {
        DeviceTables tab;
        if ((st = device_tables(inst[k].lat, &tab)) != FTWA_OK) return st;
    }
    for (const GroupPlan& g : p.groups)
        if ((st = resident_prepare(g.config, g.lds)) != FTWA_OK) return st;
    return FTWA_OK;
}

// Queues every launch of the run on `stream` (and nothing else: no host
// synchronisation), so that it can be captured into a graph.
ftwa_status execute(const Plan& p, const ftwa_instance* inst, char* ws, hipStream_t stream,
                    KernelTimer& timer, bool cooperative) {
    ftwa_status st;
    uint32_t* status = reinterpret_cast<uint32_t*>(ws + p.off_status);
    hipLaunchKernelGGL(status_init_kernel, dim3(1), dim3(64), 0, stream, status);
    FTWA_LAUNCH_CHECK("status_init_kernel");
    for (size_t e0 = 0; e0 < p.table.size(); e0 += kTableChunk) {
        TableChunk c;
        c.n = (int)std::min<size_t>(kTableChunk, p.table.size() - e0);
        std::memcpy(c.e, p.table.data() + e0, (size_t)c.n * sizeof(ResidentInst));
        hipLaunchKernelGGL(write_table_kernel, dim3(1), dim3(256), 0, stream,
                           reinterpret_cast<ResidentInst*>(ws + p.r_table) + e0, c);
        FTWA_LAUNCH_CHECK("write_table_kernel");
    }
    for (int k = 0; k < p.n_inst; ++k) {
        const ftwa_instance& in = inst[k];
        const int D = 2 * in.lat->N;
        if ((st = zero_fill(in.S1, p.n_rec * D, stream)) != FTWA_OK) return st;
        if ((st = zero_fill(in.S2, p.n_rec * s2_count(D), stream)) != FTWA_OK) return st;
        if (in.inv && (st = zero_fill(in.inv, p.n_rec * 4, stream)) != FTWA_OK) return st;
    }
    // ---- stream instances
    for (int k = 0; k < p.n_inst; ++k) {
        const InstPlan& ip = p.inst[k];
        if (ip.path != FTWA_PATH_STREAM) continue;
        const ftwa_instance& in = inst[k];
        DeviceTables tab;
        if ((st = device_tables(in.lat, &tab)) != FTWA_OK) return st;
        const int N = in.lat->N;
        const int D = 2 * N;
        double* X = reinterpret_cast<double*>(ws + p.s_x);
        double* parts = in.inv ? reinterpret_cast<double*>(ws + p.s_inv) : nullptr;
        for (int64_t m0 = 0; m0 < in.n_traj; m0 += ip.chunk) {
            const int64_t Mc = std::min(ip.chunk, in.n_traj - m0);
            StreamChunk c;
            c.N = N;
            c.P = packed_count(N);
            c.Mc = Mc;
            c.y = static_cast<char*>(in.rho) + (size_t)m0 * cplx_bytes(p.dtype);
            c.ldy = in.n_traj;
            c.acc = ws + p.s_acc;
            c.ya = ws + p.s_ya;
            c.yb = ws + p.s_yb;
            c.t = in.lat->t;
            c.U = in.U;
            c.dt = p.dt;
            c.v_site = in.v_site;
            c.v_env = in.v_env;
            c.u_mat = in.u_mat;
            c.D = in.u_mat ? ws + p.s_D : nullptr;
            c.hop_w = in.hop_w;
            if ((st = record_diag(c, tab, p.dtype, X, stream)) != FTWA_OK) return st;
            if (parts && (st = record_inv(c, tab, p.dtype, parts, stream)) != FTWA_OK) return st;
            int64_t open_steps = 0;
            for (int64_t step = 1; step <= p.n_steps; ++step) {
                if (open_steps == 0 && (st = timer.begin(stream)) != FTWA_OK) return st;
                c.step = step - 1;
                if ((st = stream_step(c, tab, p.dtype, stream)) != FTWA_OK) return st;
                ++open_steps;
                if (open_steps == 64 || step == p.n_steps) {
                    if ((st = timer.end(stream, 4 * open_steps, (double)Mc * open_steps)) != FTWA_OK)
                        return st;
                    open_steps = 0;
                }
                if (step % p.record_every == 0) {
                    const int64_t r = step / p.record_every;
                    if ((st = record_diag(c, tab, p.dtype, X + r * D * Mc, stream)) != FTWA_OK)
                        return st;
                    if (parts &&
                        (st = record_inv(c, tab, p.dtype, parts + r * 4 * Mc, stream)) != FTWA_OK)
                        return st;
                }
            }
            if ((st = moments_accumulate(D, Mc, p.n_rec, X, in.S1, in.S2, ws + p.s_mom, stream)) !=
                FTWA_OK)
                return st;
            if (parts && (st = invariants_accumulate(N, Mc, p.n_rec, in.lat->t, in.U, X, parts,
                                                     in.inv, stream)) != FTWA_OK)
                return st;
        }
    }
    // ---- resident groups, pass by pass
    // the ratio tables of the instances with complex hopping first
    for (int k = 0; k < p.n_inst; ++k) {
        const InstPlan& ip = p.inst[k];
        if (ip.path != FTWA_PATH_RESIDENT || !inst[k].hop_w) continue;
        DeviceTables tab;
        if ((st = device_tables(inst[k].lat, &tab)) != FTWA_OK) return st;
        // spin split: place order (the partner's diagonal); shared blocks:
        // site order
        const int32_t* const order = resident_spins(ip.res.config) == 1 ? tab.dpos : nullptr;
        if ((st = hop_table(inst[k].hop_w, tab.nb, order, inst[k].lat->N, p.n_steps, p.dtype,
                            ws + ip.off_hop, stream)) != FTWA_OK)
            return st;
    }
    for (int k = 0; k < p.n_inst; ++k) {
        const InstPlan& ip = p.inst[k];
        if (ip.path != FTWA_PATH_RESIDENT || !inst[k].u_mat) continue;
        if ((st = umat_table(inst[k].u_mat, inst[k].lat->N, p.dtype, ws + ip.off_umat, stream)) !=
            FTWA_OK)
            return st;
    }
    const ResidentInst* table = reinterpret_cast<const ResidentInst*>(ws + p.r_table);
    for (int j = 0; j < p.n_pass; ++j) {
        for (size_t gi = 0; gi < p.groups.size(); ++gi) {
            const LaunchDesc& Ld = p.launches[(size_t)j * p.groups.size() + gi];
            if (Ld.n_items == 0) continue;
            const GroupPlan& g = p.groups[gi];
            ResidentLaunch L;
            L.config = g.config;
            L.lds = g.lds;
            L.table = table + Ld.first_entry;
            L.n_entries = Ld.n_entries;
            L.n_items = Ld.n_items;
            L.grid = Ld.grid;
            L.Nmax = g.Nmax;
            L.dt = p.dt;
            L.n_steps = p.n_steps;
            L.record_every = p.record_every;
            L.mailbox = ws + g.off_mb;
            L.error = reinterpret_cast<int*>(status + 1);
            L.spin_limit = p.spin_limit;
            L.drop_partners = p.drop_partners;
            L.cooperative = cooperative;
            L.unit_hop = Ld.unit_hop;
            L.dumps = p.dump != nullptr;
            L.potential = Ld.potential;
            L.hopping = Ld.hopping;
            L.interaction = Ld.interaction;
            if ((st = timer.begin(stream)) != FTWA_OK) return st;
            if ((st = resident_launch(L, stream)) != FTWA_OK) return st;
            if ((st = timer.end(stream, 1, Ld.work)) != FTWA_OK) return st;
        }
        for (int k = 0; k < p.n_inst; ++k) {
            const InstPlan& ip = p.inst[k];
            if (ip.path != FTWA_PATH_RESIDENT) continue;
            const ftwa_instance& in = inst[k];
            int64_t m0, Mc;
            window(p, in, k, j, &m0, &Mc);
            if (Mc <= 0) continue;
            const int N = in.lat->N;
            double* X = reinterpret_cast<double*>(ws + ip.off_x);
            if ((st = moments_accumulate(2 * N, Mc, p.n_rec, X, in.S1, in.S2, ws + p.r_mom,
                                         stream)) != FTWA_OK)
                return st;
            if (in.inv &&
                (st = invariants_accumulate(N, Mc, p.n_rec, in.lat->t, in.U, X,
                                            reinterpret_cast<double*>(ws + ip.off_inv), in.inv,
                                            stream)) != FTWA_OK)
                return st;
        }
    }
    // ---- non-finite trajectories counted by the invariant monitors
    for (int k = 0; k < p.n_inst; ++k) {
        if (!inst[k].inv) continue;
        hipLaunchKernelGGL(status_nonfinite_kernel, dim3(1), dim3(64), 0, stream, inst[k].inv,
                           p.n_rec, (uint32_t)std::min(k, 0xffff), status);
        FTWA_LAUNCH_CHECK("status_nonfinite_kernel");
    }
    return FTWA_OK;
}

// Waits for `stream` and reports what the status block of the last run in
// the workspace recorded: a bounded wait that gave up (FTWA_ETIMEOUT), then
// non-finite trajectories (FTWA_ENONFINITE).
ftwa_status check_status(const char* ws, hipStream_t stream) {
    uint32_t h[4] = {0, 0, 0, 0};
    FTWA_HIP_TRY(hipMemcpyAsync(h, ws, sizeof(h), hipMemcpyDeviceToHost, stream));
    FTWA_HIP_TRY(hipStreamSynchronize(stream));
    if (h[0] != kStatusMagic) return fail(FTWA_EINVAL, "no ftwa_evolve run recorded in this workspace");
    if (h[1] != 0)
        return fail(FTWA_ETIMEOUT,
                    "a workgroup of a resident run timed out waiting for the others of its "
                    "trajectory (were they resident together?)");
    if (h[2] != 0)
        return fail(FTWA_ENONFINITE, "instance " + std::to_string(h[3] >> 16) +
                                         ": a trajectory became non-finite by record " +
                                         std::to_string(h[3] & 0xffffu));
    return FTWA_OK;
}

// ---------------------------------------------------------------- static workspace
// The workspace of ftwa_evolve_static: a fixed array in device memory that
// the code object brings with it (each device the library runs on holds its
// own copy until the process ends).  Its name is only a host-side stand-in:
// host code uses the device address hipGetSymbolAddress returns, kept per
// device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;  // device ordinal -> address of its copy

// The address of the current device's copy, looked up once per device.
ftwa_status static_scratch(char** out) {
    int dev = 0;
    FTWA_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        FTWA_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(FTWA_EHIP, "hipGetSymbolAddress returned no address");
        it = g_scratch_ptr.emplace(dev, static_cast<char*>(ptr)).first;
    }
    *out = it->second;
    return FTWA_OK;
}

// ---------------------------------------------------------------- tuning table
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t, int>, int> g_tuned;

int current_device() {
    int d = 0;
    (void)hipGetDevice(&d);
    return d;
}

}  // namespace

// ---------------------------------------------------------------- stored-state runs
// Resident integration of one instance (rho updated in place) that also
// stores the state at every record: record r >= 1 (after r * record_every
// steps) goes to dump + (r - 1) * dump_stride elements, in the layout of rho
// (leading dimension in.n_traj).  For the adjoint's checkpoints and segment
// states.  With ws == NULL only *bytes is set; fails with FTWA_ENOTSUP when
// no resident configuration fits.
ftwa_status evolve_stored(const ftwa_instance& in, double dt, int64_t n_steps, int record_every,
                          ftwa_dtype dtype, void* dump, int64_t dump_stride, char* ws,
                          size_t* bytes, hipStream_t stream) {
    ftwa_tuning tune;
    std::memset(&tune, 0, sizeof(tune));
    tune.path = FTWA_PATH_RESIDENT;
    tune.resident_config = -1;
    // These runs store the whole state at every record, so the shared-block
    // tiles with several trajectories per workgroup come first (their stores
    // of neighbouring trajectories share cache lines; the single-unit tiles
    // that ordinary runs prefer took the 54-site checkpoint run from 0.24 to
    // 0.38 s); otherwise the usual first fit (spin split, split kernel).
    static const int kStoredPreference[] = {0, 13, 1, 23, 24, 14, 2, 15, 3,
                                            4, 16, 5, 17, 6, 18, 7};
    const DeviceTables& tab = host_tables(in.lat);
    for (int c : kStoredPreference) {
        ResidentPlan rp;
        if (resident_plan(in.lat->N, dtype, tab, &rp, c, in.inv == nullptr)) {
            tune.resident_config = c;
            break;
        }
    }
    Plan plan;
    ftwa_status st = plan_evolve(&in, 1, dt, n_steps, record_every, dtype, &tune, &plan);
    if (st != FTWA_OK) return st;
    if (!ws) {
        *bytes = plan.total;
        return FTWA_OK;
    }
    if (*bytes < plan.total) return fail(FTWA_EINVAL, "stored-state run: workspace too small");
    plan.dump = dump;
    plan.dump_stride = dump_stride;
    if ((st = build_table(plan, &in, ws)) != FTWA_OK) return st;
    KernelTimer off(false);
    if ((st = execute(plan, &in, ws, stream, off, true)) != FTWA_OK) return st;
    return check_status(ws, stream);
}

bool tuned_config(int N, int64_t shape, ftwa_dtype dtype, int* config) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(current_device(), N, shape, (int)dtype));
    if (it == g_tuned.end()) return false;
    *config = it->second;
    return true;
}

void set_tuned_config(int N, int64_t shape, ftwa_dtype dtype, int config) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[std::make_tuple(current_device(), N, shape, (int)dtype)] = config;
}

}  // namespace ftwa

using namespace ftwa;

struct ftwa_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Plan plan;
    std::vector<ftwa_instance> inst;
    char* ws = nullptr;
};

extern "C" {

ftwa_status ftwa_lattice_upload(ftwa_lattice lat) {
    if (!lat) return fail(FTWA_EINVAL, "ftwa_lattice_upload: NULL lattice");
    ftwa_status st = upload_tables(lat);
    if (st != FTWA_OK) return st;
    const DeviceTables& tab = host_tables(lat);
    if (!tab.bipartite) return FTWA_OK;  // the stream path needs no descriptors
    int dev = 0;
    FTWA_HIP_TRY(hipGetDevice(&dev));
    const int N = lat->N;
    // every table a plan may look up: each configuration that holds the
    // lattice, in either precision, with and without the potential's layout
    for (int c = 0; c < resident_config_count(); ++c)
        for (ftwa_dtype dtype : {FTWA_F64, FTWA_F32})
            for (bool pot : {false, true}) {
                ResidentPlan rp;
                if (!resident_plan(N, dtype, tab, &rp, c, true, pot)) continue;
                const int eb = (int)cplx_bytes(dtype);
                const void* d = nullptr;
                std::string key;
                if (resident_parts(c) > 1) {
                    int pw = 0, hm = 0;
                    st = split_tables(lat, resident_parts(c), rp.even_slots, rp.odd_slots,
                                      rp.bnd_entry, eb, &d, &pw, &hm, true);
                    key = split_key(dev, resident_parts(c), rp.even_slots, rp.odd_slots,
                                    rp.bnd_entry, eb);
                } else {
                    st = padded_descriptors(lat, rp.even_slots, rp.odd_slots, eb,
                                            resident_spins(c) == 1, &d, true);
                    key = padded_key(dev, rp.even_slots, rp.odd_slots, eb, resident_spins(c) == 1);
                }
                if (st == FTWA_EHIP || st == FTWA_ENOMEM) return st;
                if (st != FTWA_OK) {
                    // this configuration cannot hold the lattice after all: a
                    // plan that picks it reports the same error
                    std::lock_guard<std::mutex> lock(lat->mu);
                    lat->table_err[key] = std::make_pair(st, std::string(ftwa_last_error()));
                }
                if ((st = resident_prepare(c, rp.lds)) != FTWA_OK) return st;
            }
    return FTWA_OK;
}

ftwa_status ftwa_evolve_workspace_size(const ftwa_instance* inst, int n_inst, int64_t n_steps,
                                       int record_every, ftwa_dtype dtype,
                                       const ftwa_tuning* tune, size_t* bytes) {
    ftwa_status st = check_instances(inst, n_inst, false, "ftwa_evolve_workspace_size");
    if (st != FTWA_OK) return st;
    if (!bytes) return fail(FTWA_EINVAL, "bytes is NULL");
    Plan plan;
    if ((st = plan_evolve(inst, n_inst, 0.0, n_steps, record_every, dtype, tune, &plan)) != FTWA_OK)
        return st;
    *bytes = plan.total;
    return FTWA_OK;
}

ftwa_status ftwa_evolve(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                        int record_every, ftwa_dtype dtype, const ftwa_tuning* tune,
                        void* workspace, size_t workspace_bytes, void* stream_) {
    ftwa_status st = check_instances(inst, n_inst, true, "ftwa_evolve");
    if (st != FTWA_OK) return st;
    Plan plan;
    if ((st = plan_evolve(inst, n_inst, dt, n_steps, record_every, dtype, tune, &plan)) != FTWA_OK)
        return st;
    if (workspace_bytes < plan.total || (!workspace && plan.total > 0))
        return fail(FTWA_EINVAL, "workspace smaller than ftwa_evolve_workspace_size");
    hipStream_t stream = (hipStream_t)stream_;
    char* ws = static_cast<char*>(workspace);
    if ((st = build_table(plan, inst, ws)) != FTWA_OK) return st;
    KernelTimer timer(tune && tune->kernel_ms);
    if ((st = execute(plan, inst, ws, stream, timer, true)) != FTWA_OK) return st;
    if (tune && tune->kernel_ms)
        if ((st = timer.finish(tune->kernel_ms, tune->kernel_launches, tune->kernel_work)) != FTWA_OK)
            return st;
    return FTWA_OK;
}

ftwa_status ftwa_evolve_check(const void* workspace, void* stream) {
    if (!workspace) {
        // the last ftwa_evolve_static run on the current device
        char* ptr = nullptr;
        ftwa_status st = static_scratch(&ptr);
        if (st != FTWA_OK) return st;
        return check_status(ptr, (hipStream_t)stream);
    }
    return check_status(static_cast<const char*>(workspace), (hipStream_t)stream);
}

ftwa_status ftwa_evolve_static(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                               int record_every, ftwa_dtype dtype, const ftwa_tuning* tune,
                               void* stream_) {
    ftwa_status st = check_instances(inst, n_inst, true, "ftwa_evolve_static");
    if (st != FTWA_OK) return st;
    if (tune && tune->kernel_ms)
        return fail(FTWA_EINVAL, "ftwa_evolve_static: kernel timing is not available");
    Plan plan;
    if ((st = plan_evolve(inst, n_inst, dt, n_steps, record_every, dtype, tune, &plan)) != FTWA_OK)
        return st;
    if (plan.total > kStaticScratchBytes)
        return fail(FTWA_EINVAL, "ftwa_evolve_static: this run needs " + std::to_string(plan.total) +
                                     " bytes of workspace, more than the static " +
                                     std::to_string(kStaticScratchBytes) +
                                     " (use ftwa_evolve with a workspace, or fewer trajectories "
                                     "per call)");
    char* ws = nullptr;
    if ((st = static_scratch(&ws)) != FTWA_OK) return st;
    if ((st = build_table(plan, inst, ws)) != FTWA_OK) return st;
    KernelTimer off(false);
    return execute(plan, inst, ws, (hipStream_t)stream_, off, true);
}

ftwa_status ftwa_evolve_graph(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                              int record_every, ftwa_dtype dtype, const ftwa_tuning* tune,
                              void* workspace, size_t workspace_bytes, void* stream_,
                              ftwa_graph* out) {
    ftwa_status st = check_instances(inst, n_inst, true, "ftwa_evolve_graph");
    if (st != FTWA_OK) return st;
    if (!out) return fail(FTWA_EINVAL, "out is NULL");
    if (tune && tune->kernel_ms) return fail(FTWA_EINVAL, "kernel timing is not available in a graph");
    auto* g = new (std::nothrow) ftwa_graph_s;
    if (!g) return fail(FTWA_ENOMEM, "graph handle");
    if ((st = plan_evolve(inst, n_inst, dt, n_steps, record_every, dtype, tune, &g->plan)) != FTWA_OK) {
        delete g;
        return st;
    }
    if (workspace_bytes < g->plan.total || (!workspace && g->plan.total > 0)) {
        delete g;
        return fail(FTWA_EINVAL, "workspace smaller than ftwa_evolve_workspace_size");
    }
    g->inst.assign(inst, inst + n_inst);
    g->ws = static_cast<char*>(workspace);
    (void)stream_;
    if ((st = build_table(g->plan, inst, g->ws)) != FTWA_OK) {
        delete g;
        return st;
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
        delete g;
        return fail(FTWA_EHIP, "hipStreamCreateWithFlags");
    }
    KernelTimer off(false);
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = execute(g->plan, g->inst.data(), g->ws, cs, off, false);
        hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
        if (st == FTWA_OK && e2 != hipSuccess) st = hip_fail(e2, "hipStreamEndCapture");
    } else {
        st = hip_fail(e, "hipStreamBeginCapture");
    }
    (void)hipStreamDestroy(cs);
    if (st == FTWA_OK) {
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
    }
    if (st != FTWA_OK) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return st;
    }
    *out = g;
    return FTWA_OK;
}

ftwa_status ftwa_graph_launch(ftwa_graph g, void* stream) {
    if (!g || !g->exec) return fail(FTWA_EINVAL, "invalid graph");
    FTWA_HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return FTWA_OK;
}

ftwa_status ftwa_graph_check(ftwa_graph g, void* stream) {
    if (!g) return fail(FTWA_EINVAL, "invalid graph");
    return check_status(g->ws, (hipStream_t)stream);
}

void ftwa_graph_free(ftwa_graph g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"

// ---------------------------------------------------------------- autotuner
namespace ftwa {
namespace {

constexpr int kProbeReps = 3;

struct Probe {
    std::vector<int> cands;  // resident configurations that fit, then -1 (stream path)
    int64_t Mp = 0;          // trajectories timed
    size_t off_rho = 0, off_s1 = 0, off_s2 = 0, off_ws = 0, total = 0;
};

ftwa_tuning probe_tuning(int cand) {
    ftwa_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.path = cand < 0 ? FTWA_PATH_STREAM : FTWA_PATH_RESIDENT;
    t.traj_chunk = 0;
    t.resident_config = cand;
    return t;
}

ftwa_instance probe_instance(const ftwa_instance& in, int64_t Mp, char* ws, const Probe& pr) {
    ftwa_instance q = in;
    q.n_traj = Mp;
    q.traj_offset = 0;
    q.rho = ws ? ws + pr.off_rho : nullptr;
    q.S1 = ws ? reinterpret_cast<double*>(ws + pr.off_s1) : nullptr;
    q.S2 = ws ? reinterpret_cast<double*>(ws + pr.off_s2) : nullptr;
    q.inv = nullptr;
    q.v_site = nullptr;  // the probes time the kernels without the potential term
    q.v_env = nullptr;
    q.u_mat = nullptr;   // and with the on-site interaction
    q.hop_w = nullptr;   // and real hopping
    return q;
}

ftwa_status plan_probe(const ftwa_instance& in, ftwa_dtype dtype, int probe_steps, Probe* out) {
    Probe pr;
    ftwa_status st;
    const DeviceTables& tab = host_tables(in.lat);
    const int N = in.lat->N;
    int64_t want = 0;
    for (int c = 0; c < resident_config_count(); ++c) {
        ResidentPlan rp;
        if (!resident_plan(N, dtype, tab, &rp, c)) continue;
        pr.cands.push_back(c);
        want = std::max(want, 2 * resident_concurrency(c, rp.lds));
    }
    pr.cands.push_back(-1);
    if (want == 0) want = kStreamChunk;
    pr.Mp = std::max<int64_t>(1, std::min(in.n_traj, want));
    const int D = 2 * N;
    size_t off = 0;
    pr.off_rho = off; off = align_up(off + (size_t)2 * packed_count(N) * pr.Mp * cplx_bytes(dtype));
    pr.off_s1 = off;  off = align_up(off + (size_t)2 * D * sizeof(double));
    pr.off_s2 = off;  off = align_up(off + (size_t)2 * s2_count(D) * sizeof(double));
    pr.off_ws = off;
    size_t ews = 0;
    const ftwa_instance q = probe_instance(in, pr.Mp, nullptr, pr);
    for (int c : pr.cands) {
        const ftwa_tuning t = probe_tuning(c);
        Plan p;
        if ((st = plan_evolve(&q, 1, 0.01, probe_steps, probe_steps, dtype, &t, &p)) != FTWA_OK)
            return st;
        ews = std::max(ews, p.total);
    }
    pr.total = align_up(off + ews);
    *out = pr;
    return FTWA_OK;
}

}  // namespace
}  // namespace ftwa

extern "C" {

ftwa_status ftwa_autotune_workspace_size(const ftwa_instance* inst, int n_inst, ftwa_dtype dtype,
                                         int probe_steps, size_t* bytes) {
    ftwa_status st = check_instances(inst, n_inst, false, "ftwa_autotune_workspace_size");
    if (st != FTWA_OK) return st;
    if (!bytes || probe_steps < 1) return fail(FTWA_EINVAL, "bytes is NULL or probe_steps < 1");
    if (dtype != FTWA_F64 && dtype != FTWA_F32) return fail(FTWA_EINVAL, "unknown dtype");
    size_t total = 0;
    for (int k = 0; k < n_inst; ++k) {
        Probe pr;
        if ((st = plan_probe(inst[k], dtype, probe_steps, &pr)) != FTWA_OK) return st;
        total = std::max(total, pr.total);
    }
    *bytes = total;
    return FTWA_OK;
}

ftwa_status ftwa_autotune(const ftwa_instance* inst, int n_inst, ftwa_dtype dtype, int probe_steps,
                          void* workspace, size_t workspace_bytes, void* stream_, int* configs) {
    ftwa_status st = check_instances(inst, n_inst, false, "ftwa_autotune");
    if (st != FTWA_OK) return st;
    if (probe_steps < 1) return fail(FTWA_EINVAL, "probe_steps < 1");
    if (dtype != FTWA_F64 && dtype != FTWA_F32) return fail(FTWA_EINVAL, "unknown dtype");
    hipStream_t stream = (hipStream_t)stream_;
    char* ws = static_cast<char*>(workspace);
    std::map<std::pair<int, int64_t>, int> decided;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    FTWA_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(FTWA_EHIP, "hipEventCreate");
    }
    auto done = [&](ftwa_status s) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return s;
    };
    for (int k = 0; k < n_inst; ++k) {
        const ftwa_instance& in = inst[k];
        if (in.n_traj < 1 || !in.rho || !in.n0) return done(fail(FTWA_EINVAL, "instance without trajectories"));
        DeviceTables tab;
        if ((st = device_tables(in.lat, &tab)) != FTWA_OK) return done(st);
        const int N = in.lat->N;
        const auto key = std::make_pair(N, class_shape(tab));
        auto it = decided.find(key);
        if (it != decided.end()) {
            if (configs) configs[k] = it->second;
            continue;
        }
        Probe pr;
        if ((st = plan_probe(in, dtype, probe_steps, &pr)) != FTWA_OK) return done(st);
        if (!ws || workspace_bytes < pr.total)
            return done(fail(FTWA_EINVAL, "workspace smaller than ftwa_autotune_workspace_size"));
        const ftwa_instance q = probe_instance(in, pr.Mp, ws, pr);
        const size_t cb = cplx_bytes(dtype);
        const size_t P2 = (size_t)2 * packed_count(N);
        int best = -1;
        double best_ms = -1.0;
        for (int c : pr.cands) {
            const ftwa_tuning t = probe_tuning(c);
            Plan p;
            if ((st = plan_evolve(&q, 1, 0.01, probe_steps, probe_steps, dtype, &t, &p)) != FTWA_OK)
                return done(st);
            char* ews = ws + pr.off_ws;
            if ((st = build_table(p, &q, ews)) != FTWA_OK) return done(st);
            // one warm-up run, then the fastest of kProbeReps timed runs
            float ms = -1.0f;
            for (int rep = 0; rep <= kProbeReps; ++rep) {
                FTWA_HIP_TRY(hipMemcpy2DAsync(ws + pr.off_rho, pr.Mp * cb, in.rho, in.n_traj * cb,
                                              pr.Mp * cb, P2, hipMemcpyDeviceToDevice, stream));
                KernelTimer off(false);
                FTWA_HIP_TRY(hipEventRecord(e0, stream));
                if ((st = execute(p, &q, ews, stream, off, true)) != FTWA_OK) return done(st);
                FTWA_HIP_TRY(hipEventRecord(e1, stream));
                FTWA_HIP_TRY(hipEventSynchronize(e1));
                float t = 0.0f;
                FTWA_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
                if (rep > 0 && (ms < 0 || t < ms)) ms = t;
            }
            if ((st = check_status(ews, stream)) != FTWA_OK) return done(st);
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
        set_tuned_config(N, class_shape(tab), dtype, best);
        decided[key] = best;
        if (configs) configs[k] = best;
    }
    return done(FTWA_OK);
}

}  // extern "C"

// ftwa_internal.h -- shared declarations of the libftwa host code and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ftwa.h"

namespace ftwa {

constexpr int kMaxDeg = 3;
constexpr int kMaxSites = 255;
constexpr int kMaxParts = 4;  // workgroups per spin block of the split resident kernel

// What a split configuration (one spin block over G workgroups, "parts") must
// hold for a lattice: the maxima over its parts.  Even class: "interior"
// elements (read no other part's element) and "boundary" elements (the
// diagonal and the elements other parts read); odd class: the exported ones
// and the rest.
struct SplitShape {
    int n_even = 0, n_odd = 0;  // owned elements of each class
    int int_gen = 0;            // interior elements that read a transpose
    int n_bnd = 0, bnd_gen = 0; // boundary elements, those of them that read a transpose
    int odd_gen = 0;            // odd elements that read a transpose
    int odd_x = 0;              // odd entries up to the last exported one
    int max_slots = 0;          // owned plus halo elements
    int max_halo = 0;           // halo elements
};

// Index tables of a lattice on one device (uploaded once, owned by the handle).
struct DeviceTables {
    int32_t* nb = nullptr;     // [N][4]: three neighbours (ascending, -1 padded), degree
    int32_t* off = nullptr;    // [N]: packed row start i*N - i*(i-1)/2
    uint32_t* elem = nullptr;  // [P]: packed element p -> i | j << 16
    int64_t n_even = 0;        // size of the even class (i, j on the same sublattice)
    int64_t n_gen_even = 0;    // leading even-class elements that read a transpose
    int64_t n_gen_odd = 0;     // leading odd-class elements that read a transpose
    bool bipartite = false;
    uint32_t* ord = nullptr;   // [P]: LDS slot (class order) -> a | b << 16, the
                               // element stored there is rho_ab ({a, b} = {i, j})
    int32_t* dpos = nullptr;   // [N]: site -> its position in the sublattice-major
                               // diagonal (the sites of one sublattice, ascending,
                               // then the other's)
    SplitShape split[kMaxParts + 1];  // by part count G = 2..kMaxParts (bipartite only)
    uint4* rdesc = nullptr;    // [2P][2]: descriptors of the on-chip reverse sweep with a
                               // packed X (N <= kReverseMaxSites; see reverse_descriptors)
    uint4* rdescf = nullptr;   // [2P][2]: the same with a full X (N <= kReverseFullMaxSites)
};

// Stencil descriptor of one element for the resident kernel.  Of every pair
// {i, j} the LDS holds one orientation rho_ab (a ranks before b in a
// bandwidth-reducing site order, so that few elements read a transposed
// neighbour).  Wide form (32 bytes, ResDesc), all offsets in bytes within the
// LDS block of one spin; the descriptor of the stored element rho_ij has
//   a.x, a.y, a.z: the column neighbours rho_ik, k in nb(j), ascending;
//   b.x, b.y, b.z: the row neighbours rho_kj, k in nb(i), ascending;
//     each = offset of the stored element | bit 31 set when the stored
//     element is rho_ki (read its conjugate); a missing neighbour reads the
//     zero slot P;
//   a.w: offset of the element itself (padding entries own the scratch slot
//     P+1);
//   b.w: offset of the diagonal value of site i | that of site j << 16 in the
//     other spin's block (diagonal first, element (i,i) at slot i).
// Compact form (16 bytes, uint4) of the spin-split kernels: 16-bit slot
// numbers instead of byte offsets,
//   x = c0 | c1 << 16, y = c2 | r0 << 16, z = r1 | r2 << 16 (bit 15 of a
//     neighbour's field: read its conjugate),
//   w = own slot | pos(i) << 16 | pos(j) << 24, pos = the site's place in the
//     partner's diagonal, a real array in sublattice-major order
//     (consecutive same-sublattice sites at consecutive words).
struct ResDesc {
    uint4 a, b;
};

}  // namespace ftwa

struct ftwa_lattice_s {
    int N = 0;
    int n_bonds = 0;
    double t = 1.0;
    std::vector<int32_t> nbr;   // [N][3], ascending, padded with -1
    std::vector<uint8_t> deg;   // [N]
    std::vector<uint8_t> sub;   // [N]
    std::mutex mu;
    std::map<int, ftwa::DeviceTables> dev;  // by HIP device ordinal
    // resident-path descriptors padded per class to whole slots, by
    // (device, even slots, odd slots, element bytes and diagonal layout)
    std::map<std::tuple<int, int64_t, int64_t, int>, void*> padded;
    std::vector<uint32_t> class_order;      // a | b << 16 of the stored elements in LDS-slot order
    std::vector<int32_t> diag_pos;          // site -> sublattice-major diagonal position
    std::vector<int32_t> rank;              // site -> bandwidth-reducing rank
    // split-kernel tables by (device, parts, even slots, odd slots, boundary
    // entry, element bytes): device blob, words per part, import capacity
    std::map<std::tuple<int, int, int64_t, int64_t, int64_t, int>, std::tuple<void*, int, int>> split;
    // host part of the tables (class sizes, split shapes; no device pointers),
    // computed when the lattice is built
    ftwa::DeviceTables host;
    // kernel tables ftwa_lattice_upload could not build, by split_key /
    // padded_key: the error it met
    std::map<std::string, std::pair<ftwa_status, std::string>> table_err;
};

namespace ftwa {

// Packed Hermitian storage of one spin block.
inline int64_t packed_count(int N) { return (int64_t)N * (N + 1) / 2; }
inline int64_t packed_row(int N, int i) { return (int64_t)i * N - (int64_t)i * (i - 1) / 2; }
inline int64_t n_records(int64_t n_steps, int record_every) { return n_steps / record_every + 1; }
inline int64_t s2_count(int D) { return (int64_t)D * (D + 1) / 2; }
// What the resident configurations that fit a lattice depend on besides N:
// the class sizes of its stored elements (tuning results are kept by it).
inline int64_t class_shape(const DeviceTables& t) {
    return t.n_even | (t.n_gen_even << 20) | (t.n_gen_odd << 40);
}

// Error reporting (thread-local message, see ftwa_last_error).
ftwa_status fail(ftwa_status st, const std::string& msg);
ftwa_status hip_fail(hipError_t e, const char* what);

#define FTWA_HIP_TRY(expr)                                                  \
    do {                                                                    \
        hipError_t _e = (expr);                                             \
        if (_e != hipSuccess) return ::ftwa::hip_fail(_e, #expr);           \
    } while (0)

#define FTWA_LAUNCH_CHECK(what)                                             \
    do {                                                                    \
        hipError_t _e = hipGetLastError();                                  \
        if (_e != hipSuccess) return ::ftwa::hip_fail(_e, what);            \
    } while (0)

// Host validation of an instance array (api.hip).
ftwa_status check_instances(const ftwa_instance* inst, int n_inst, bool need_moments,
                            const char* who);

// Host part of the tables, computed by ftwa_build_lattice(_bonds): class
// order, diagonal positions, class sizes and split shapes.
void compute_host_tables(ftwa_lattice lat);
const DeviceTables& host_tables(ftwa_lattice lat);
// The lattice's device tables on the current device (FTWA_EINVAL unless
// ftwa_lattice_upload ran there).
ftwa_status device_tables(ftwa_lattice lat, DeviceTables* out);
// Allocates and uploads the basic tables on the current device (idempotent).
ftwa_status upload_tables(ftwa_lattice lat);
std::string split_key(int dev, int G, int64_t even_slots, int64_t odd_slots, int64_t bnd_entry,
                      int elem_bytes);
std::string padded_key(int dev, int64_t even_slots, int64_t odd_slots, int elem_bytes,
                       bool compact);
// Descriptor table in LDS-slot order with the even class padded to
// even_slots entries and the odd class to odd_slots entries; padding entries
// own the scratch slot P+1 and read only the zero slot P.  compact selects
// the 16-byte form of the spin-split kernels (else the wide form with
// offsets for elem_bytes-byte elements).  Uploaded once per shape, element
// size and form by ftwa_lattice_upload (create = true); the compute calls
// only look it up.
ftwa_status padded_descriptors(ftwa_lattice lat, int64_t even_slots, int64_t odd_slots,
                               int elem_bytes, bool compact, const void** out,
                               bool create = false);

// Tables of the split resident kernel for G parts (uploaded once per shape by
// ftwa_lattice_upload).
// One block of *part_words 32-bit words per part:
//   [0..7]   n_even, n_own, n_import_even, n_import_odd, n_diag, 0, 0, 0
//   [8..)    descriptors (compact form, 16 bytes per entry, even_slots +
//            odd_slots entries; own field bit 15: the element is exported).
//            Even entries: the interior elements (those that read a
//            transpose first) up to bnd_entry, the boundary elements from
//            bnd_entry (the diagonal, then those that read a transpose), then
//            interior elements that did not fit before bnd_entry; odd entries:
//            those that read a transpose (exported first), the other exported
//            ones, the rest.
//   then     LDS slot -> a | b << 16 of the owned element (even_slots + odd_slots words)
//   then     imports: producer part << 16 | producer slot, *hmax words
//            (halo slot n_own + h takes import h; even halo first)
//   then     the site of even entry t < n_diag (its diagonal element)
// then, after the G blocks, [N]: site -> part << 16 | slot of its diagonal element.
ftwa_status split_tables(ftwa_lattice lat, int G, int64_t even_slots, int64_t odd_slots,
                         int64_t bnd_entry, int elem_bytes, const void** out, int* part_words,
                         int* hmax, bool create = false);

// ---------------------------------------------------------------- launches
// Sampling of rho(0) for one instance (sample.hip).
ftwa_status launch_sample(const ftwa_instance& in, const DeviceTables& tab, uint64_t seed,
                          ftwa_dtype dtype, bool thermal, hipStream_t stream);

// Copies of the diagonal variables into the record buffer X[a][m] (FP64).
struct RecordView {
    double* X;        // [D][Mc] for one record
    int64_t ldx;      // = Mc
};

// Stream path (evolve_stream.hip).
struct StreamChunk {
    int N;
    int64_t P;
    int64_t Mc;          // trajectories in this chunk
    void* y;             // instance rho, already offset by the chunk's first trajectory
    int64_t ldy;         // stride of y between packed elements (= instance n_traj)
    void* acc;           // workspace state copies, stride Mc
    void* ya;
    void* yb;
    double t, U, dt;
    // external on-site potential V_i(tau) = A(tau) v_i (NULL: none): v_site
    // [N], v_env the instance's envelope samples at half steps; `step` is the
    // index of the step being taken (its stages read v_env[2 step + 0/1/1/2])
    const double* v_site = nullptr;
    const double* v_env = nullptr;
    int64_t step = 0;
    // general interaction (NULL: on-site U): u_mat [N][N]; D the workspace
    // [2][N][Mc] (working precision) of D_i = sum_k u_ki (d_k + 1/2) per stage
    const double* u_mat = nullptr;
    void* D = nullptr;
    // complex hopping (NULL: real t): [2 n_steps + 1][N][3] complex ratios
    // j_ik / t of the instance at half steps, read like v_env
    const double* hop_w = nullptr;
};
ftwa_status stream_step(const StreamChunk& c, const DeviceTables& tab, ftwa_dtype dtype,
                        hipStream_t stream);
ftwa_status record_diag(const StreamChunk& c, const DeviceTables& tab, ftwa_dtype dtype,
                        double* X, hipStream_t stream);
// Per-trajectory invariant sums of one record (hop and frob per spin, FP64),
// written to parts[2 spins][2][Mc].
ftwa_status record_inv(const StreamChunk& c, const DeviceTables& tab, ftwa_dtype dtype,
                       double* parts, hipStream_t stream);
// inv[r] = max/sum over the chunk's trajectories of the drifts of record r
// from record 0 (trace, Weyl energy, Frobenius norm) and the non-finite count,
// combined with the values already in inv (max, max, max, +).
ftwa_status invariants_accumulate(int N, int64_t Mc, int64_t n_rec, double t, double U,
                                  const double* X, const double* parts, double* inv,
                                  hipStream_t stream);

// Moments of the records of one chunk: S1[r] += sum_m X[r][a][m],
// S2[r][ab] += sum_m X[r][a][m] X[r][b][m] (fixed summation order).
size_t moments_workspace_bytes(int D, int64_t Mc, int64_t n_rec);
ftwa_status moments_accumulate(int D, int64_t Mc, int64_t n_rec, const double* X,
                               double* S1, double* S2, void* scratch, hipStream_t stream);

ftwa_status zero_fill(double* p, int64_t n, hipStream_t stream);

// Descriptors of the on-chip reverse sweep: a pair (q0, q1) per element
// e = s P + p(i, j) of both spin blocks, in that order.  X is the LDS copy of
// a state: packed (entry e; full = false) or the full matrices of both spins
// (entry (s N + a) N + b for element (a, b) of spin s; full = true); W is
// always full.  q0: x = c0 | c1 << 16, y = c2 | r0 << 16, z = r1 | r2 << 16,
// with c_n the X entry of rho_ik (k the n-th neighbour of j, ascending) and r_n
// that of rho_kj (k the n-th neighbour of i); packed: bit 15 of a field marks a
// stored transpose (read its conjugate); a missing neighbour reads the zero
// entry after the last; w = yi | yj << 16, the entries (1 - s) N + i and
// (1 - s) N + j of the other spin's diagonal in a [2N] row.  q1: x = X entry
// of the element | of its transpose << 16 (packed: e twice), y = W entry of
// the element | of its transpose << 16, z = s N + i | (i == j) << 16, w = e.
constexpr int kReverseMaxSites = 180;      // packed X entries < 2^15, W entries < 2^16
constexpr int kReverseFullMaxSites = 64;   // full X: beyond this it no longer fits LDS
std::vector<uint4> reverse_descriptors(const ftwa_lattice_s& lat, bool full);

// One checkpoint segment of the on-chip reverse sweep (adjoint_resident.hip).
struct ReverseSegment {
    int N;
    int record_every;
    int64_t Mc, L, Lmax, base, n_steps;
    bool first, last;
    const uint4* desc;       // the packed-X and full-X descriptor tables
    const uint4* desc_full;
    const void* ckpt;   // y_base, trajectory-innermost [2P][Mc]
    void* seg;          // [Mc][Lmax][2P]
    void* lamT;         // [Mc][2P]
    void* lam_out;      // [2P][Mc] (diagonal entries, written by the last segment)
    double* partial;    // [2][Mc]
    const double* dL;   // [n_rec][2N]
    double scale, t, U, dt;
};
// The configuration of the on-chip reverse sweep for N sites (-1: none fits).
int reverse_resident_config(int N, ftwa_dtype dtype);
ftwa_status reverse_resident(int config, const ReverseSegment& s, hipStream_t stream);
ftwa_status zero_words(unsigned* p, int64_t n, hipStream_t stream);

// Resident path (evolve_resident.hip).
struct ResidentPlan {
    int config = -1;
    int spins_per_unit = 2;  // 1: one spin block per workgroup, pairs exchange diagonals
    int threads = 0;
    int units = 1;
    int64_t even_slots = 0;  // descriptor padding of the even / odd class
    int64_t odd_slots = 0;
    int64_t bnd_entry = 0;   // split configurations: first boundary entry of the even class
    size_t lds = 0;
    bool u_lds = false;      // shared blocks with a general interaction: lds includes a copy
                             // of u (umat_table's layout), which the kernel reads there
};
// One entry of a resident launch's table: a window of trajectories of one
// instance (device memory, read by the kernel).
struct ResidentInst {
    int N;
    int P;
    int64_t Mc;          // trajectories in the window (the record width)
    void* rho;           // instance state offset to the window's first trajectory
    int64_t ldr;         // instance n_traj
    const void* desc;    // padded_descriptors(lat, plan.even_slots, plan.odd_slots, bytes, S == 1)
    const uint32_t* ord; // DeviceTables::ord
    const int32_t* nb;   // DeviceTables::nb
    const int32_t* dpos; // DeviceTables::dpos
    double t, U;
    double* X;           // [n_rec][2N][Mc]
    double* inv_parts;   // NULL or [n_rec][2 spins][hop, frob][Mc]
    int64_t item0;       // first item of this entry (items of earlier entries before it)
    void* dump;          // NULL, or the state at record r >= 1 is stored at
                         // dump + (r - 1) * dump_stride elements (same layout and window
                         // offset as rho)
    int64_t dump_stride;
    int part_words;      // split configurations: desc is split_tables(...), one block per
    int hmax;            // part of part_words words; hmax: import capacity
    const double* v_site;  // NULL or [N]: external on-site potential profile (ftwa_instance)
    const double* v_env;   // its envelope at half steps from the start of the run
    const void* hop;       // NULL or the complex-hopping ratio table (hop_table)
    const void* umat;      // NULL or the general interaction in the working precision (umat_table)
    int u_lds;             // nonzero: the shared-block kernel copies umat into LDS per item
};
struct ResidentLaunch {
    int config;
    size_t lds;                 // dynamic LDS: max over the entries
    const ResidentInst* table;  // device
    int n_entries;
    int64_t n_items;
    int64_t grid;               // resident_grid(config, lds, n_items), fixed at plan time
    int Nmax;
    double dt;
    int64_t n_steps;
    int record_every;
    void* mailbox;              // resident_mailbox_bytes(config, Nmax, n_items) of scratch
    int* error;                 // the run's timeout word (set to 1 by a wait that gave up)
    unsigned spin_limit;        // polls before a bounded wait gives up (0: the default)
    bool drop_partners;         // fault injection: run only one workgroup of each pair
    bool cooperative;           // false under graph capture
    bool unit_hop;              // every instance of the launch has t = 1
    bool dumps;                 // an entry stores its state at records (ResidentInst::dump)
    bool potential;             // an entry carries an external potential (the POT variant)
    bool hopping;               // every entry carries complex hopping (the HOP variant)
    bool interaction;           // every entry carries a general interaction (the GINT variant)
};
// Picks the first kernel configuration that fits (or only `force_config` if >= 0).
// allow_split: the split configurations may be chosen (they keep no
// invariant sums); need_potential, need_hop, need_interaction: only
// configurations with an external-potential, complex-hopping or
// general-interaction variant (the FP32 spin split and the FP64 split kernel).
bool resident_plan(int N, ftwa_dtype dtype, const DeviceTables& tab, ResidentPlan* plan,
                   int force_config = -1, bool allow_split = true, bool need_potential = false,
                   bool need_hop = false, bool need_interaction = false);
int resident_config_count();
int resident_spins(int config);
int resident_parts(int config);  // workgroups per spin block (> 1: split tables)
bool resident_has_potential(int config);  // has the external-potential variant
bool resident_has_hop(int config);        // has the complex-hopping variant
bool resident_has_interaction(int config);  // has the general-interaction variant
// Rows of the general-interaction variant's u table: N rounded up to 32.
__host__ __device__ inline int umat_rows(int N) { return (N + 31) & ~31; }
// u_mat ([N][N] FP64, u_ki at k N + i) rounded once to dtype, blocked by four
// along k (((k / 4) N + i) 4 + k % 4), rows N..umat_rows(N)-1 zero (queued on
// stream; umat_rows(N) N elements).
ftwa_status umat_table(const double* u_mat, int N, ftwa_dtype dtype, void* out,
                       hipStream_t stream);
// The ratio table of the complex-hopping variant from ftwa_instance::hop_w
// ([2 n_steps + 1][N][3] complex FP64): [2 n_steps + 1][N][3] complex in dtype,
// row r's site i at place dpos[i] (at i when dpos is NULL), missing neighbours
// zero (queued on stream).
ftwa_status hop_table(const double* hop_w, const int32_t* nb, const int32_t* dpos, int N,
                      int64_t n_steps, ftwa_dtype dtype, void* out, hipStream_t stream);
int64_t resident_item_traj(int config);      // trajectories per item of the schedule
int64_t resident_max_pairs();
int64_t resident_concurrency(int config, size_t lds);  // trajectories in flight at once
int64_t resident_grid(int config, size_t lds, int64_t n_items);
size_t resident_mailbox_bytes(int config, int Nmax, int64_t n_items);
ftwa_status resident_prepare(int config, size_t lds);  // host only, not under graph capture
ftwa_status resident_launch(const ResidentLaunch& L, hipStream_t stream);

// Configurations chosen by ftwa_autotune, per (device, N, even-class size, dtype).
bool tuned_config(int N, int64_t shape, ftwa_dtype dtype, int* config);
// Resident run of one instance that stores its state at every record
// (evolve.hip; ws == NULL: workspace size query into *bytes).
ftwa_status evolve_stored(const ftwa_instance& in, double dt, int64_t n_steps, int record_every,
                          ftwa_dtype dtype, void* dump, int64_t dump_stride, char* ws,
                          size_t* bytes, hipStream_t stream);
void set_tuned_config(int N, int64_t shape, ftwa_dtype dtype, int config);

// Brackets launches of the dominant kernel with HIP events on one stream and
// sums their durations (optional, see ftwa_tuning::kernel_ms).
class KernelTimer {
public:
    explicit KernelTimer(bool enabled) : enabled_(enabled) {}
    ~KernelTimer();
    bool enabled() const { return enabled_; }
    ftwa_status begin(hipStream_t s);
    ftwa_status end(hipStream_t s, int64_t launches, double work);
    ftwa_status finish(double* ms, int64_t* launches, double* work);

private:
    bool enabled_;
    std::vector<hipEvent_t> events_;
    int64_t launches_ = 0;
    double work_ = 0.0;
};

}  // namespace ftwa

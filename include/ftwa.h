/*
 * ftwa.h -- C ABI of libftwa, the MI355X (gfx950) implementation of the
 * fermionic Truncated Wigner Approximation (fTWA) hot path for the
 * Fermi-Hubbard model on honeycomb (graphene) lattices.
 *
 * Paper: F. Rousse, O. Eriksson, M. Ogren, "Correlated quantum dynamics of
 * graphene", arXiv:2212.04352.  The library computes, on the GPU:
 *   1. Gaussian initial phase-space points rho(0) around a Fock state
 *      (Sec. III, Eq. (7));
 *   2. trajectories of the fTWA equation of motion (Sec. III, Eq. (6)) with
 *      nearest-neighbour hopping t and on-site U (Sec. II, Eq. (1)),
 *      integrated with the classical fourth-order Runge-Kutta method;
 *   3. FP64 ensemble moments of the diagonal variables, giving the site
 *      occupations (Eq. (5)), connected density-density correlations and g2
 *      (Eq. (10)).
 *
 * General rules for every entry point:
 *   - Return value: FTWA_OK (0) or a negative ftwa_status.  Nothing throws
 *     across the ABI.  ftwa_last_error() gives a message for the calling
 *     thread's last failure.
 *   - Arguments are validated on the host before any device work is queued;
 *     on an argument error nothing is launched and outputs are untouched.
 *   - "device" pointers are HIP device allocations owned by the caller; the
 *     library never frees them.  "host" pointers are ordinary memory.
 *   - Device work is queued asynchronously on `stream` (a hipStream_t; NULL
 *     means the default stream) of the current HIP device; the calls that
 *     queue it return without waiting for the device.  The caller
 *     synchronises before reading outputs.  The calls that wait are named
 *     as such: ftwa_lattice_upload, ftwa_evolve_check, ftwa_graph_check,
 *     ftwa_autotune, ftwa_adjoint (it sizes its passes from stored states),
 *     and ftwa_evolve only when its optional kernel timing is asked for.
 *   - The library allocates device memory only in ftwa_lattice_upload: a
 *     lattice's index and descriptor tables, once per lattice and device,
 *     freed by ftwa_free_lattice.  No other call allocates device memory;
 *     scratch memory comes from the caller through `workspace`.
 *
 * Data layout of the phase-space state ("packed layout"):
 *   For N sites, one spin block is Hermitian, so only its upper triangle
 *   i <= j is stored: P = N(N+1)/2 complex elements, element (i, j) at
 *   p(i, j) = i*N - i*(i-1)/2 + (j - i).  The trajectory index is innermost:
 *     rho[((s * P + p(i, j)) * n_traj + m)]   (s = 0 up, 1 down)
 *   each entry a complex number stored as (re, im) -- two doubles for
 *   FTWA_F64, two floats for FTWA_F32.  Diagonal entries are real (im = 0).
 *   rho_ji = conj(rho_ij) is implied.
 */
#ifndef FTWA_H
#define FTWA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FTWA_OK = 0,
    FTWA_EINVAL = -1,      /* invalid argument (detected on the host)          */
    FTWA_ENOMEM = -2,      /* host or device allocation failed                 */
    FTWA_EHIP = -3,        /* a HIP runtime call or kernel launch failed       */
    FTWA_ENOTSUP = -4,     /* valid request this build does not support        */
    FTWA_ENONFINITE = -5,  /* a trajectory became non-finite (NaN or Inf)      */
    FTWA_ETIMEOUT = -6     /* a cooperative kernel gave up waiting (bounded)   */
} ftwa_status;

typedef enum {
    FTWA_TORUS = 0,          /* a x b honeycomb unit cells, periodic; N = 2ab  */
    FTWA_ARMCHAIR_RECT = 1,  /* a x b brick-wall rectangle, degree-<2 sites
                                trimmed (10 x 20 gives the 198-site flake)     */
    FTWA_HEX_ZIGZAG = 2      /* zigzag hexagonal flake of a rings, N = 6 a^2  */
} ftwa_lattice_kind;

typedef enum { FTWA_F64 = 0, FTWA_F32 = 1 } ftwa_dtype;

typedef enum {
    FTWA_START_NEEL = 0,     /* up electrons on sublattice A, down on B        */
    FTWA_START_RANDOM = 1    /* seeded random half filling, one electron/site */
} ftwa_start;

typedef struct ftwa_lattice_s* ftwa_lattice;

/* ---------------------------------------------------------------- lattice */

/*
 * ftwa_build_lattice -- nearest-neighbour honeycomb graph with uniform
 * hopping t_hop on every bond (Sec. II: j_ij = J for neighbours, u_ij = U
 * delta_ij).  Geometries (the paper's own exist only in its figures):
 *   FTWA_TORUS (a, b >= 2): site 2*(x*b + y) + s; A(x,y) is bonded to
 *     B(x,y), B(x-1,y), B(x,y-1), indices modulo a and b.
 *   FTWA_ARMCHAIR_RECT (a rows, b columns, both >= 2): sites (r, c);
 *     bonds (r,c)-(r,c+1) and, when r + c is even, (r,c)-(r+1,c); sites of
 *     degree < 2 are removed repeatedly; survivors numbered row by row.
 *   FTWA_HEX_ZIGZAG (a >= 1 rings, b ignored): hexagons within hex distance
 *     a-1 of a centre hexagon on the same brick wall, sites numbered by
 *     (row, column).
 * Sublattice of site (r, c) is (r + c) mod 2 (torus: s).  Neighbour lists
 * are ascending.  N must be <= 255 (the kernels index sites in 8 bits).
 * out: receives a handle owned by the caller, released with
 * ftwa_free_lattice.  Errors: FTWA_EINVAL for bad sizes or N > 255.
 */
ftwa_status ftwa_build_lattice(ftwa_lattice_kind kind, int a, int b, double t_hop,
                               ftwa_lattice* out);

/*
 * ftwa_build_lattice_bonds -- any graph of degree <= 3 from an explicit bond
 * list (host arrays): bonds[2*k], bonds[2*k+1] are the sites of bond k,
 * sublattice[i] in {0, 1} (only used by FTWA_START_NEEL).  Duplicate bonds,
 * self bonds, degree > 3 or N > 255 give FTWA_EINVAL.
 */
ftwa_status ftwa_build_lattice_bonds(int n_sites, int n_bonds, const int32_t* bonds,
                                     const uint8_t* sublattice, double t_hop,
                                     ftwa_lattice* out);

/*
 * ftwa_lattice_info -- read-only views of the host tables: nbr[N][3]
 * (ascending, padded with -1), deg[N], sublattice[N].  The pointers stay
 * valid until ftwa_free_lattice.  Any output pointer may be NULL.
 */
ftwa_status ftwa_lattice_info(ftwa_lattice lat, int* n_sites, int* n_bonds,
                              const int32_t** nbr, const uint8_t** deg,
                              const uint8_t** sublattice);

/*
 * ftwa_lattice_upload -- allocates and uploads to the current HIP device
 * every device table the kernels read for this lattice: the neighbour and
 * packed-index tables, and the stencil descriptors of every resident kernel
 * configuration that holds the lattice in either precision (a few MB at
 * N = 198).  Synchronous; idempotent (a second call on the same device does
 * nothing).  Must run on a device before any call there that queues work for
 * the lattice (ftwa_sample, ftwa_evolve, ftwa_evolve_graph, ftwa_autotune,
 * ftwa_adjoint), which otherwise fail with FTWA_EINVAL before launching
 * anything.  Errors: FTWA_EINVAL (NULL lattice), FTWA_EHIP / FTWA_ENOMEM
 * when an allocation or copy fails.
 */
ftwa_status ftwa_lattice_upload(ftwa_lattice lat);

/* ftwa_free_lattice -- releases host and device tables; NULL is a no-op. */
void ftwa_free_lattice(ftwa_lattice lat);

/*
 * ftwa_fock_start -- initial occupations of a Fock state with one electron on
 * every site (Sec. IV.A), written to host n0_host[2][N] (0.0 or 1.0).
 * FTWA_START_RANDOM: Fisher-Yates permutation of the sites, swap partner of
 * position i drawn as floor(a (i+1) / 2^53) from the 53-bit integer a of
 * Philox4x32-10 counter (i, instance, 0, 1), key = seed; the first N/2 sites
 * of the permutation get an up electron.  Requires even N.
 */
ftwa_status ftwa_fock_start(ftwa_lattice lat, ftwa_start kind, uint64_t seed,
                            uint32_t instance, double* n0_host);

/* ---------------------------------------------------------------- problem */

/*
 * One problem instance.  All pointers are device pointers owned by the
 * caller; N = number of sites of `lat`, D = 2N,
 * n_rec = n_steps / record_every + 1 records (steps 0, record_every, ...).
 *   n0   [2][N] FP64     initial occupations n_{i s}(0) (may be fractional)
 *   rho  packed layout (see top of file), n_traj trajectories, in/out
 *   S1   [n_rec][D] FP64              sum_m x_m[a],       x_m[s*N+i] = rho_ii,s
 *   S2   [n_rec][D(D+1)/2] FP64       sum_m x_m[a] x_m[b], a <= b, packed as
 *                                     a*D - a*(a-1)/2 + (b-a)
 *   inv  [n_rec][4] FP64 or NULL      per record, maximum over trajectories of
 *        |tr rho_s(t) - tr rho_s(0)| (max over s), |H_W(t) - H_W(0)| (Weyl
 *        Hamiltonian, Appendix A.3), | |rho|_F^2(t) - |rho|_F^2(0) | (max over
 *        s), and the count of non-finite trajectories.
 *   n_shift [2][N] FP64 or NULL  shift of the initial diagonal: ftwa_sample
 *        writes rho_ii,s(0) = n0[s][i] - 1/2 + n_shift[s][i] while the
 *        off-diagonal noise amplitude uses n0 alone (the noise is held fixed
 *        under the shift); ftwa_adjoint returns the gradient with respect to it.
 *   v_site [N] FP64 or NULL, v_env [2 n_steps + 1] FP64  an external on-site
 *        potential V_i(tau) = A(tau) v_site[i] acting on both spins (Sec. III:
 *        the time dependence of an external potential enters Eq. (6) as
 *        explicit terms): ftwa_evolve adds i (V_i(tau) - V_j(tau)) rho_ij to
 *        the right-hand side, with A sampled by the caller at half steps from
 *        the start of the call, v_env[k] = A(k dt/2): step n uses v_env[2n] in
 *        its first Runge-Kutta stage, v_env[2n+1] in the second and third,
 *        v_env[2n+2] in the fourth.  Arithmetic: a = U (d_i - d_j), then
 *        a = a + A (v_i - v_j), A and v rounded once to the working precision.
 *        Integrated by the potential variants of the resident kernels (the
 *        shared-block tiles holding both spin blocks of a trajectory in one
 *        workgroup, FP32 and FP64; FP32 one workgroup per spin block; FP64
 *        split over several) where the automatic choice is one of them, else
 *        by the stream kernels (a forced resident path or configuration
 *        without the potential variant gives FTWA_ENOTSUP); ftwa_adjoint
 *        refuses it.
 *        v_env must hold 2 n_steps + 1 values (not checked: device memory).
 *   u_mat [N][N] FP64 or NULL  a general density-density interaction u_ij
 *        between opposite spins (Eq. (1); symmetric) in place of the on-site
 *        U (ignored then): Eq. (6)'s own form multiplies rho_ij,s by
 *        D_i - D_j, D_i = sum_k u_ki (rho_kk,sbar + 1/2), accumulated as
 *        D = fma(u_ki, d_k + 1/2, D) over ascending k in the working precision
 *        (u rounded once).  Integrated by the general-interaction variants
 *        of the resident kernels (shared-block tiles in FP32 and FP64, the
 *        FP32 spin split, the FP64 split kernel) where the automatic choice
 *        is one of them and the instance has neither v_site nor hop_w (u,
 *        rounded once, is staged by a kernel into the workspace; each stage
 *        forms D in LDS before the elements), else by the stream kernels (a
 *        per-stage kernel forms D for every site and trajectory); a forced
 *        resident path or configuration without the variant, or with v_site
 *        or hop_w, gives FTWA_ENOTSUP.  Invariant monitors (inv: their energy
 *        is the on-site form; FTWA_EINVAL) and ftwa_adjoint (FTWA_ENOTSUP)
 *        refuse it.
 *   hop_w [2 n_steps + 1][N][3] complex FP64 (interleaved re, im) or NULL
 *        complex, time-dependent hopping j_ik(tau) = t hop_w[h][i][n] for the
 *        neighbour k = nbr[i][n] of ftwa_lattice_info (Peierls phases; Sec. III:
 *        time dependence enters Eq. (6) as explicit terms), sampled at the
 *        half steps of v_env: step n reads table 2n in its first stage, 2n+1
 *        in the second and third, 2n+2 in the fourth.  The Hamiltonian is
 *        Hermitian, so the caller gives both directions of a bond as
 *        conjugates (not checked) and ftwa_evolve uses
 *        col = sum_{k in nb(j)} w_jk rho_ik, row = sum_{k in nb(i)} conj(w_ik)
 *        rho_kj in f_ij = i [t (col - row) + a rho_ij], each product as
 *        (fma(wr, xr, -(wi xi)), fma(wr, xi, wi xr)) with w rounded once to
 *        the working precision, slots summed in ascending order; slots
 *        n >= deg(i) are ignored (any finite or non-finite value).
 *        Integrated by the complex-hopping variants of the resident kernels
 *        (shared-block tiles in FP32 and FP64, the FP32 spin split, the FP64
 *        split kernel) where the automatic choice is one of them and the
 *        instance has no v_site (the ratios, rounded once and with unused
 *        slots zeroed, are staged by a kernel into the workspace; each stage
 *        keeps the ratios of up to 152 sites in LDS in the FP32 spin split,
 *        of all sites in the others), else by the stream kernels; a forced
 *        resident path or configuration without the variant, or with v_site,
 *        gives FTWA_ENOTSUP.  Invariant monitors
 *        (FTWA_EINVAL) and ftwa_adjoint (FTWA_ENOTSUP) refuse it.  Combines
 *        with v_site and u_mat on the stream kernels.  hop_w must hold
 *        (2 n_steps + 1) N 3 complex values (not checked: device memory).
 * Trajectory m of the instance has global index traj_offset + m; it keys the
 * random numbers, so any trajectory range reproduces the same trajectories.
 * `instance` enters the random-number counter (distinct streams per instance
 * of a batch).
 */
typedef struct {
    ftwa_lattice lat;
    double U;
    int64_t n_traj;
    int64_t traj_offset;
    uint32_t instance;
    const double* n0;
    void* rho;
    double* S1;
    double* S2;
    double* inv;
    const double* n_shift;
    const double* v_site;
    const double* v_env;
    const double* u_mat;
    const double* hop_w;
} ftwa_instance;

/*
 * ftwa_sample -- writes rho(0) of every trajectory of every instance
 * (Eq. (7)): rho_ii = n_i - 1/2 (+ n_shift, if given); for i < j,
 *   rho_ij = xi_ij sqrt((n_i + n_j - 2 n_i n_j) / 2),
 * xi complex normal (E|xi|^2 = 1, E xi^2 = 0) by Box-Muller from two 53-bit
 * uniforms of Philox4x32-10 with counter
 *   (i*N - i(i+1)/2 + j-i-1, instance<<1 | s, traj_offset + m, 0), key = seed:
 *   u1 = (a+1) 2^-53, u2 = b 2^-53, xi = sqrt(-ln u1) exp(2 pi i u2).
 * The noise is drawn in FP64; FTWA_F32 stores the FP64 values rounded.
 */
ftwa_status ftwa_sample(const ftwa_instance* inst, int n_inst, uint64_t seed,
                        ftwa_dtype dtype, void* stream);

/*
 * ftwa_sample_thermal -- as ftwa_sample, for an initial state that is
 * thermal in the site basis (non-integer occupations, Sec. III): the
 * Gaussian initial density then has the full covariance of Appendix A.3,
 * whose diagonal part is Var rho_ii = n_i (1 - n_i), independent of every
 * other element.  rho_ii = n_i - 1/2 (+ n_shift) + sqrt(n_i (1 - n_i)) g_i,
 * g_i a real standard normal from Philox4x32-10 with counter
 *   (i, instance<<1 | s, traj_offset + m, 2), key = seed:
 *   g = sqrt(-2 ln u1) cos(2 pi u2)  (u1, u2 as above);
 * the off-diagonal elements are those of ftwa_sample (same counters), so for
 * integer occupations both calls give identical points.  Same arguments,
 * errors and layout as ftwa_sample.
 */
ftwa_status ftwa_sample_thermal(const ftwa_instance* inst, int n_inst, uint64_t seed,
                                ftwa_dtype dtype, void* stream);

/* Tuning of ftwa_evolve; pass NULL for the automatic choice. */
typedef enum {
    FTWA_PATH_AUTO = 0,
    FTWA_PATH_STREAM = 1,    /* state in HBM, one launch per Runge-Kutta stage */
    FTWA_PATH_RESIDENT = 2   /* state held on chip for the whole horizon: one
                                workgroup per trajectory or spin block, or (FP64
                                blocks too large for one CU) a spin block over
                                2-4 workgroups of one XCD that exchange their
                                boundary rows every stage; not with inv in that
                                last case                                      */
} ftwa_path;

typedef struct {
    ftwa_path path;
    int traj_chunk;          /* trajectories per pass (0 = automatic)         */
    int resident_config;     /* index into the resident kernel table, or -1
                                for the automatic choice (FTWA_ENOTSUP if the
                                forced one does not fit the lattice)          */
    /* Optional timing of the dominant kernel (the Runge-Kutta kernel of the
       chosen path): when kernel_ms is not NULL, every launch of that kernel is
       bracketed by HIP events on `stream`, ftwa_evolve waits for the stream
       before returning, and writes the summed duration in milliseconds to
       *kernel_ms, the number of launches to *kernel_launches (if not NULL)
       and the trajectory-steps those launches advanced to *kernel_work (if
       not NULL; a stage launch counts 1/4 step per trajectory). */
    double* kernel_ms;
    int64_t* kernel_launches;
    double* kernel_work;
    /* Polls before a bounded wait of a multi-workgroup resident kernel gives
       up and the run reports FTWA_ETIMEOUT (0 = the default, about 2 s of
       polling). */
    unsigned spin_limit;
    /* Fault injection for tests of the timeout path; 0 in every production
       call.  Nonzero: every launch of a spin-split configuration (one
       workgroup per spin block) runs only the up-spin workgroups of eight
       pairs, whose partners are absent, so each of them gives up its first
       wait after spin_limit polls and exits; rho is left as it was and
       ftwa_evolve_check reports FTWA_ETIMEOUT. */
    int drop_partners;
} ftwa_tuning;

/*
 * ftwa_evolve_workspace_size -- bytes of device scratch ftwa_evolve needs for
 * these arguments (written to *bytes).
 */
ftwa_status ftwa_evolve_workspace_size(const ftwa_instance* inst, int n_inst,
                                       int64_t n_steps, int record_every,
                                       ftwa_dtype dtype, const ftwa_tuning* tune,
                                       size_t* bytes);

/*
 * ftwa_evolve -- integrates every trajectory of every instance for n_steps
 * steps of size dt with classical RK4 applied to Eq. (6):
 *   d rho_ij,s/dt = i [ t (sum_{k in nb(j)} rho_ik,s - sum_{k in nb(i)} rho_kj,s)
 *                       + U (rho_ii,sbar - rho_jj,sbar) rho_ij,s ],
 * overwriting rho with rho(n_steps dt), and fills S1/S2 (zeroed first) and
 * inv (if not NULL) at every record.  Arithmetic (FP32 or FP64 per dtype)
 * follows a fixed order -- neighbour sums in ascending order,
 * g = t (col - row), one fma per component for the U term, f = i g,
 * stage inputs fma(c, k, y), acc = k1, fma(2, k2, acc), fma(2, k3, acc),
 * acc + k4, y = fma(dt/6, acc, y) -- so results do not depend on the kernel
 * path, the tiling or the batch composition.  S1/S2 are always FP64.
 * workspace: device scratch of at least ftwa_evolve_workspace_size bytes;
 * it starts with the run's status block, which kernels of the run fill
 * (a timeout of a bounded wait, non-finite trajectories counted by the
 * invariant monitors) and ftwa_evolve_check reads.  The call queues the run
 * and returns without waiting (unless tune->kernel_ms asks for timing).
 * Errors, all detected on the host before anything is queued: FTWA_EINVAL
 * (sizes, NULL pointers, workspace too small, lattice not uploaded to this
 * device), FTWA_ENOTSUP when the resident path is forced and no
 * configuration holds the lattice, FTWA_EHIP on launch failure.  What
 * happens on the device is reported by ftwa_evolve_check.
 */
ftwa_status ftwa_evolve(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                        int record_every, ftwa_dtype dtype, const ftwa_tuning* tune,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * ftwa_evolve_check -- waits for `stream` and reads the status block of the
 * last run (ftwa_evolve or a graph launch) that used `workspace`:
 * FTWA_ETIMEOUT when the workgroups of a resident run that share a
 * trajectory were not resident together (a bounded wait gave up; rho and
 * the moments are then incomplete), else FTWA_ENONFINITE when an instance
 * with invariant monitors (inv) had a non-finite trajectory (inv[r][3]
 * counts them; the message names the first instance and record), else
 * FTWA_OK.  FTWA_EINVAL when the workspace holds no run's status.
 * workspace NULL: the status of the last ftwa_evolve_static run on the
 * current device.
 */
ftwa_status ftwa_evolve_check(const void* workspace, void* stream);

/*
 * ftwa_evolve_static -- ftwa_evolve for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same run, bitwise the same results, with the
 * workspace in a fixed 64 MiB array of device memory that the library holds
 * on every device it runs on (its address looked up once per device).  The
 * call allocates nothing; the caller still passes the instances' buffers,
 * and the lattices must have been uploaded (ftwa_lattice_upload).  Limit:
 * runs whose ftwa_evolve_workspace_size exceeds 64 MiB (67108864 bytes) are
 * refused with FTWA_EINVAL before anything is queued (a few thousand
 * trajectories with a few hundred records at N = 54; use ftwa_evolve, or
 * fewer trajectories per call).  Kernel timing (tune->kernel_ms) is refused.
 * All calls on one device share that array, and it keeps the last call's
 * contents (every run clears what must start at zero): calls that overlap on
 * one device -- on different streams, or from several threads -- race, so
 * the caller serialises them (one stream).  ftwa_evolve_check(NULL, stream)
 * reports the device status of the last such run.  Errors as ftwa_evolve.
 */
ftwa_status ftwa_evolve_static(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                               int record_every, ftwa_dtype dtype, const ftwa_tuning* tune,
                               void* stream);

/*
 * Batched launch as a HIP graph.  ftwa_evolve_graph plans the same run as
 * ftwa_evolve (same arguments; kernel timing is not available) and captures
 * every launch of the run, the writes of its launch table into `workspace`
 * included, into a graph on a stream of its own; nothing is computed yet and
 * `stream` is not used.  Instances whose
 * kernel configuration is the same are integrated by one persistent kernel
 * per pass over a table of (instance, trajectory window) entries, so a batch
 * of mixed lattice sizes and U values needs a handful of kernel nodes; the
 * results are bitwise those of one ftwa_evolve per instance.
 * ftwa_graph_launch queues the whole run on `stream` (one graph launch): it
 * re-zeroes S1/S2/inv and integrates the current rho for n_steps steps.  The
 * instance buffers and the workspace must stay allocated, and no other work
 * may use the workspace, while the graph exists.  ftwa_graph_check waits for
 * `stream` and reports what ftwa_evolve_check reports for the last launch
 * (FTWA_ETIMEOUT, FTWA_ENONFINITE).  Configurations whose trajectories span
 * several workgroups (a spin block each, or parts of one) rely on the GPU
 * running no other work that would keep those workgroups from being resident
 * together; their waits are bounded (FTWA_ETIMEOUT).
 */
typedef struct ftwa_graph_s* ftwa_graph;
ftwa_status ftwa_evolve_graph(const ftwa_instance* inst, int n_inst, double dt, int64_t n_steps,
                              int record_every, ftwa_dtype dtype, const ftwa_tuning* tune,
                              void* workspace, size_t workspace_bytes, void* stream,
                              ftwa_graph* out);
ftwa_status ftwa_graph_launch(ftwa_graph graph, void* stream);
ftwa_status ftwa_graph_check(ftwa_graph graph, void* stream);
void ftwa_graph_free(ftwa_graph graph);

/*
 * ftwa_autotune -- times every resident kernel configuration that fits each
 * distinct lattice of the instances (and the stream path) on a copy of the
 * instance's first trajectories (rho is not modified), `probe_steps` steps
 * each, and records the fastest per (device, lattice size, class sizes of
 * the lattice's stored elements, dtype); later plans with the automatic
 * choice use it.  configs (host, NULL or [n_inst])
 * receives the choice per instance (-1 = stream path).  Synchronises
 * `stream`; must not be called under graph capture.  workspace: at least
 * ftwa_autotune_workspace_size bytes.
 */
ftwa_status ftwa_autotune_workspace_size(const ftwa_instance* inst, int n_inst, ftwa_dtype dtype,
                                         int probe_steps, size_t* bytes);
ftwa_status ftwa_autotune(const ftwa_instance* inst, int n_inst, ftwa_dtype dtype, int probe_steps,
                          void* workspace, size_t workspace_bytes, void* stream, int* configs);

/*
 * ftwa_observables -- ensemble observables from the moments of M
 * trajectories (device pointers), plug-in estimators with divisor M:
 *   n_out [n_rec][D]      n_a = S1_a/M + 1/2                          (Eq. (5))
 *   C_out [n_rec][D][D]   C_ab = S2_ab/M - (S1_a/M)(S1_b/M)
 *   g2_out[n_rec][D][D]   (S2_ab/M + (S1_a+S1_b)/(2M) + 1/4)
 *                         / ((S1_a/M + 1/2)(S1_b/M + 1/2))            (Eq. (10))
 * with a = s*N + i.  The a = b entries of C and g2 are Weyl-symbol
 * variances, not same-site observables.  C_out and g2_out may be NULL.
 */
ftwa_status ftwa_observables(int n_sites, int64_t M, int n_rec, const double* S1,
                             const double* S2, double* n_out, double* C_out,
                             double* g2_out, void* stream);

/*
 * ftwa_unpack -- expands packed rho (n_traj trajectories) into full matrices
 * out[m][s][i][j] (complex, same precision as dtype), filling i > j with
 * conjugates.  Device pointers.
 */
ftwa_status ftwa_unpack(int n_sites, int64_t n_traj, ftwa_dtype dtype, const void* rho,
                        void* out, void* stream);

/*
 * ftwa_adjoint_workspace_size -- bytes of device scratch ftwa_adjoint needs.
 */
ftwa_status ftwa_adjoint_workspace_size(const ftwa_instance* inst, int64_t n_steps,
                                        int record_every, int ckpt_every, ftwa_dtype dtype,
                                        int64_t traj_chunk, size_t* bytes);

/*
 * ftwa_adjoint -- gradient of a loss of the ensemble occupations
 * nbar_a(r) = (1/n_total) sum_m rho_aa(t_r) + 1/2 (Eq. (5); a = s*N + i,
 * t_r = r * record_every * dt) with respect to U, t and the initial diagonal
 * shift, with the sampled noise held fixed, by the discrete adjoint of the
 * classical Runge-Kutta map of Eq. (6) (reverse sweep over the stages,
 * states recomputed from checkpoints every ckpt_every steps).
 *   inst          one instance; inst->rho holds rho(0) as written by
 *                 ftwa_sample (device, not modified); S1, S2, inv unused.
 *   n_total       the trajectory count in the mean (>= inst->n_traj; the
 *                 instance may be a slice of a larger ensemble).
 *   dL_dnbar      device FP64 [n_rec][2N], n_rec = n_steps/record_every + 1.
 *   grad          device FP64 [2 + 2N], overwritten: grad[0] = dL/dU,
 *                 grad[1] = dL/dt, grad[2 + s*N + i] = dL/dn_shift[s][i]
 *                 (= dL/d rho_ii,s(0)).  Accumulated in FP64 in a fixed
 *                 order (deterministic); the adjoint state is in dtype.
 *   traj_chunk    trajectories per pass (0 = all); smaller chunks need less
 *                 workspace and give the same result up to the order of the
 *                 final FP64 sums.
 * When a resident configuration fits the lattice and dtype, the checkpoints
 * come from one resident run that stores its state (the workspace also holds
 * its plan; the run synchronises `stream` once on the host), and, for up to
 * 71 sites in FP32 and 54 in FP64, the reverse sweep runs on chip: one
 * launch per segment, one workgroup per trajectory, which recomputes the
 * segment's states from its checkpoint and then runs the transposed stages
 * with the cotangent in registers.  Otherwise the segments and the reverse
 * sweep are per-stage stream launches.  The trajectories are the same either
 * way; the gradient agrees to rounding (the on-chip sweep forms some products
 * and row sums in the working precision).
 * Errors: FTWA_EINVAL (sizes, NULL pointers, workspace too small),
 * FTWA_EHIP on launch failure, FTWA_ETIMEOUT (a spin-split resident run's
 * bounded wait gave up).
 */
ftwa_status ftwa_adjoint(const ftwa_instance* inst, double dt, int64_t n_steps,
                         int record_every, int ckpt_every, ftwa_dtype dtype, int64_t n_total,
                         const double* dL_dnbar, double* grad, int64_t traj_chunk,
                         void* workspace, size_t workspace_bytes, void* stream);

/* ftwa_last_error -- message for the calling thread's last non-OK status. */
const char* ftwa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FTWA_H */

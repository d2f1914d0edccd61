// adjoint.hip -- gradient of losses of the ensemble occupations with respect
// to U, t and the initial diagonal, by the discrete adjoint of the classical
// Runge-Kutta map of the fTWA equation of motion (Eq. (6) of
// arXiv:2212.04352), with the sampled noise held fixed.
//
// Inner product: the state of one spin block is a Hermitian matrix and
// cotangents are taken with respect to the Frobenius inner product
// <A, B> = Re tr(A^H B); a cotangent is then itself Hermitian and is stored
// in the packed layout like the state.
//
// The right-hand side is f_s(Y) = i[Y_s, J] + i U [D_sbar, Y_s] with
// (Y J)_ij = t sum_{k in nb(j)} Y_ik, D = diag(Re Y_sbar).  For fixed D it is
// linear and skew with respect to <.,.>, so its transpose is minus itself:
//   (df^T a)_s = -f_s^lin(a_s; D from Y)
//                + on the diagonal (k,k): -2U sum_j Im(conj(a_sbar,kj) Y_sbar,kj)
// (the second line is the dependence of f_sbar on D_s).  Parameter
// derivatives:
//   <a, df/dU> = -sum_ij (d_i - d_j) Im(conj(a_ij) Y_ij)
//   <a, df/dt> = -<L(a), Y> = -sum_ij Im(conj(g_ij) Y_ij),  g = col(a) - row(a)
// (L = hopping part at t = 1, itself skew), each off-diagonal pair counted
// twice in the packed sums.
//
// Reverse sweep of one step y -> y+ with cotangent lam of y+:
//   a4 = h/6 lam;            mu4 = df(Y4)^T a4
//   a3 = h/3 lam + h mu4;    mu3 = df(Y3)^T a3
//   a2 = h/3 lam + h/2 mu3;  mu2 = df(Y2)^T a2
//   a1 = h/6 lam + h/2 mu2;  mu1 = df(y)^T a1
//   cotangent of y = lam + mu1 + mu2 + mu3 + mu4,
// and theta_bar += sum_s <a_s, df/dtheta(Y_s)>.  The stage inputs
// Y2 = y + h/2 k1, Y3 = y + h/2 k2, Y4 = y + h k3 are recomputed from y with
// the forward arithmetic; the states y of a segment are recomputed from its
// checkpoint.  All kernels use the trajectory-innermost layout of the stream
// path (a wave = 64 trajectories x a run of consecutive packed elements).
#include <algorithm>
#include <string>
#include <vector>

#include "device_common.h"
#include "ftwa_internal.h"

namespace ftwa {

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kElemsPerWave = 16;

struct WaveGrid {
    int64_t n_elem_chunks = 0;  // ceil(2P / kElemsPerWave)
    int64_t n_work = 0;         // waves
    int64_t blocks_per_xcd = 0;
};

WaveGrid make_grid(int64_t P, int64_t Mc) {
    WaveGrid g;
    g.n_elem_chunks = (2 * P + kElemsPerWave - 1) / kElemsPerWave;
    g.n_work = ((Mc + 63) / 64) * g.n_elem_chunks;
    const int64_t n_blocks = (g.n_work + kWavesPerBlock - 1) / kWavesPerBlock;
    g.blocks_per_xcd = (n_blocks + 7) / 8;
    return g;
}

dim3 grid_dim(const WaveGrid& g) { return dim3((unsigned)(g.blocks_per_xcd * 8)); }

__device__ __forceinline__ int64_t prow(int N, int i) {
    return (int64_t)i * N - (int64_t)i * (i - 1) / 2;
}

// (element chunk, trajectory) of this lane; consecutive virtual blocks run on
// one XCD (blocks are dealt round-robin to the 8 XCDs).
struct Lane {
    int64_t chunk, m;
    bool active, valid;
};
__device__ __forceinline__ Lane lane_work(const WaveGrid g, int64_t Mc) {
    const int64_t xcd = blockIdx.x % 8;
    const int64_t vblock = xcd * g.blocks_per_xcd + blockIdx.x / 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int64_t w = vblock * kWavesPerBlock + wave;
    Lane l;
    l.valid = w < g.n_work;
    const int64_t tb = l.valid ? w / g.n_elem_chunks : 0;
    l.chunk = l.valid ? w - tb * g.n_elem_chunks : 0;
    const int64_t m_raw = tb * 64 + threadIdx.x % 64;
    l.active = l.valid && m_raw < Mc;
    l.m = m_raw < Mc ? m_raw : Mc - 1;  // inactive lanes read in bounds, never write
    return l;
}

template <typename T>
__device__ __forceinline__ cplx_t<T> load_el(const cplx_t<T>* X, int64_t Mc, int N, int a, int b,
                                             int64_t m) {
    if (a <= b) return X[(prow(N, a) + (b - a)) * Mc + m];
    return conj(X[(prow(N, b) + (a - b)) * Mc + m]);
}

template <typename T> struct StageInArgs {
    int N;
    int64_t P, Mc;
    const int32_t* nb;
    const uint32_t* elem;
    T t, U, c;
    const cplx_t<T>* yin;  // stage input Y_s
    const cplx_t<T>* y;    // step start
    cplx_t<T>* yout;       // Y_{s+1} = fma(c, f(Y_s), y)
    WaveGrid g;
};

// Packed elements of a wave: (spin, i, j) of the first one from the element
// table, then advanced along the rows (the next row, then the other spin).
struct ElemWalk {
    int s, i, j;
    __device__ __forceinline__ void next(int N) {
        if (++j == N) {
            if (++i == N) {
                s = 1;
                i = 0;
            }
            j = i;
        }
    }
};
__device__ __forceinline__ ElemWalk walk_from(const uint32_t* elem, int64_t P, int64_t q0) {
    ElemWalk w;
    w.s = q0 >= P ? 1 : 0;
    const uint32_t ij = elem[q0 - w.s * P];
    w.i = (int)(ij & 0xffffu);
    w.j = (int)(ij >> 16);
    return w;
}

// nb4: the neighbour rows (also in A.nb) as a read-only argument, so that the
// wave-uniform row reads are scalar loads; all loads of an element are
// issued together.
template <typename T>
__global__ __launch_bounds__(256) void stage_input_kernel(StageInArgs<T> A,
                                                          const int4* __restrict__ nb4) {
    const Lane l = lane_work(A.g, A.Mc);
    if (!l.valid) return;
    const int64_t q0 = l.chunk * kElemsPerWave;
    const int64_t q1 = q0 + kElemsPerWave < 2 * A.P ? q0 + kElemsPerWave : 2 * A.P;
    ElemWalk w = walk_from(A.elem, A.P, q0);
    for (int64_t q = q0; q < q1; ++q, w.next(A.N)) {
        const int s = w.s, i = w.i, j = w.j;
        const int64_t p = q - s * A.P;
        const cplx_t<T>* Ys = A.yin + (int64_t)s * A.P * A.Mc;
        const cplx_t<T>* Yo = A.yin + (int64_t)(1 - s) * A.P * A.Mc;
        cplx_t<T> col, row;
        neighbour_sums<T>(Ys, A.Mc, A.N, nb4[j], nb4[i], i, j, l.m, col, row);
        const cplx_t<T> own = Ys[p * A.Mc + l.m];
        const T di = Yo[prow(A.N, i) * A.Mc + l.m].x, dj = Yo[prow(A.N, j) * A.Mc + l.m].x;
        const int64_t e = ((int64_t)s * A.P + p) * A.Mc + l.m;
        const cplx_t<T> yv = A.y[e];
        const T a = A.U * (di - dj);
        const cplx_t<T> k = rhs_element<T>(col, row, own, A.t, a);
        if (l.active) {
            cplx_t<T> nx;
            nx.x = fma_rn<T>(A.c, k.x, yv.x);
            nx.y = fma_rn<T>(A.c, k.y, yv.y);
            A.yout[e] = nx;
        }
    }
}

// The diagonal coupling term of the transposed right-hand side, one thread
// per (spin s, site i, trajectory): R[s][i][m] = sum_{k != i} Im(conj(a_ik) Y_ik)
// over the other spin's row i (ascending k), for the diagonal elements of
// the following vjp_kernel launch.
template <typename T>
__global__ __launch_bounds__(256) void diag_coupling_kernel(int N, int64_t P, int64_t Mc,
                                                            const cplx_t<T>* __restrict__ a,
                                                            const cplx_t<T>* __restrict__ Y,
                                                            T* __restrict__ R) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Mc) return;
    const int si = blockIdx.y;
    const int s = si >= N ? 1 : 0, i = si - s * N;
    const cplx_t<T>* Ao = a + (int64_t)(1 - s) * P * Mc;
    const cplx_t<T>* Yo = Y + (int64_t)(1 - s) * P * Mc;
    // eight sites at a time: their sixteen loads are issued before the sums
    // (the sum itself runs in ascending k)
    constexpr int B = 8;
    T acc = 0;
    for (int k0 = 0; k0 < N; k0 += B) {
        cplx_t<T> av[B], yv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int k = k0 + u < N ? k0 + u : i;  // past the row: a harmless in-bounds read
            bool tr;
            const int64_t e = packed_at(N, i, k, tr) * Mc + m;
            av[u] = Ao[e];
            yv[u] = Yo[e];
            if (tr) {
                av[u].y = -av[u].y;
                yv[u].y = -yv[u].y;
            }
        }
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int k = k0 + u;
            if (k < N && k != i)
                acc = acc + (av[u].x * yv[u].y - av[u].y * yv[u].x);  // Im(conj(a) y)
        }
    }
    R[(int64_t)si * Mc + m] = acc;
}

template <typename T> struct VjpArgs {
    int N;
    int64_t P, Mc;
    const int32_t* nb;
    const uint32_t* elem;
    T t, U;
    const cplx_t<T>* Y;    // stage input Y_s (both spins)
    const cplx_t<T>* a;    // cotangent a_s of k_s
    const cplx_t<T>* lam;  // cotangent of y+ (for the next a)
    cplx_t<T>* Lam;        // accumulating cotangent of y: Lam += mu_s
    cplx_t<T>* a_next;     // a_{s-1} = alpha lam + beta mu_s (NULL for s = 1)
    const T* R;            // [2][N][Mc]: diag_coupling_kernel of (a, Y)
    T alpha, beta;
    double* partial;       // [n_elem_chunks][2][Mc]: dU, dt partial sums
    WaveGrid g;
};

template <typename T>
__global__ __launch_bounds__(256) void vjp_kernel(VjpArgs<T> A, const int4* __restrict__ nb4) {
    const Lane l = lane_work(A.g, A.Mc);
    if (!l.valid) return;
    const int N = A.N;
    const int64_t Mc = A.Mc, m = l.m;
    const int64_t q0 = l.chunk * kElemsPerWave;
    const int64_t q1 = q0 + kElemsPerWave < 2 * A.P ? q0 + kElemsPerWave : 2 * A.P;
    double eU = 0.0, et = 0.0;
    ElemWalk wk = walk_from(A.elem, A.P, q0);
    for (int64_t q = q0; q < q1; ++q, wk.next(N)) {
        const int s = wk.s, i = wk.i, j = wk.j;
        const int64_t p = q - s * A.P;
        const cplx_t<T>* Ys = A.Y + (int64_t)s * A.P * Mc;
        const cplx_t<T>* Yo = A.Y + (int64_t)(1 - s) * A.P * Mc;
        const cplx_t<T>* As = A.a + (int64_t)s * A.P * Mc;
        cplx_t<T> col, row;
        neighbour_sums<T>(As, Mc, N, nb4[j], nb4[i], i, j, m, col, row);
        const cplx_t<T> own_a = As[p * Mc + m];
        const cplx_t<T> own_y = Ys[p * Mc + m];
        const T dd = Yo[prow(N, i) * Mc + m].x - Yo[prow(N, j) * Mc + m].x;
        // operands of the updates, loaded with the stencil
        const int64_t e = ((int64_t)s * A.P + p) * Mc + m;
        const T Rd = i == j ? A.R[((int64_t)s * N + i) * Mc + m] : (T)0;
        const cplx_t<T> Lv = A.Lam[e];
        cplx_t<T> lv;
        lv.x = lv.y = 0;
        if (A.a_next) lv = A.lam[e];
        const cplx_t<T> fl = rhs_element<T>(col, row, own_a, A.t, A.U * dd);
        cplx_t<T> mu;
        mu.x = -fl.x;
        mu.y = -fl.y;
        if (i == j) {
            // dependence of the other block's equation on this diagonal
            mu.x = fma_rn<T>((T)(-2) * A.U, Rd, mu.x);
        }
        // parameter partials in FP64
        const double w = i == j ? 1.0 : 2.0;
        const double im_ay = (double)own_a.x * own_y.y - (double)own_a.y * own_y.x;
        const double gx = (double)col.x - row.x, gy = (double)col.y - row.y;
        const double im_gy = gx * own_y.y - gy * own_y.x;
        eU -= w * (double)dd * im_ay;
        et -= w * im_gy;
        if (l.active) {
            cplx_t<T> L = Lv;
            L.x = L.x + mu.x;
            L.y = L.y + mu.y;
            A.Lam[e] = L;
            if (A.a_next) {
                cplx_t<T> an;
                an.x = fma_rn<T>(A.beta, mu.x, A.alpha * lv.x);
                an.y = fma_rn<T>(A.beta, mu.y, A.alpha * lv.y);
                A.a_next[e] = an;
            }
        }
    }
    if (l.active) {
        double* pu = A.partial + (l.chunk * 2) * Mc + m;
        pu[0] += eU;
        pu[Mc] += et;
    }
}

// Lam = lam, a4 = c lam (c = h/6), elementwise over both spins.
template <typename T>
__global__ __launch_bounds__(256) void step_init_kernel(int64_t n, const cplx_t<T>* __restrict__ lam,
                                                        cplx_t<T>* __restrict__ Lam,
                                                        cplx_t<T>* __restrict__ a4, T c) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const cplx_t<T> v = lam[e];
    Lam[e] = v;
    cplx_t<T> a;
    a.x = c * v.x;
    a.y = c * v.y;
    a4[e] = a;
}

// lam_ii,s += scale * w[s*N + i] for one record (the loss's direct
// dependence on the diagonal of y at that record).
template <typename T>
__global__ __launch_bounds__(256) void seed_kernel(int N, int64_t P, int64_t Mc,
                                                   cplx_t<T>* __restrict__ lam,
                                                   const double* __restrict__ w, double scale) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Mc) return;
    const int a = blockIdx.y;
    const int s = a >= N ? 1 : 0, i = a - s * N;
    cplx_t<T>* v = lam + ((int64_t)s * P + prow(N, i)) * Mc + m;
    v->x = v->x + (T)(scale * w[a]);
}

template <typename T>
__global__ __launch_bounds__(256) void copy_state_kernel(int64_t Mc, const cplx_t<T>* __restrict__ src,
                                                         int64_t ld_src, cplx_t<T>* __restrict__ dst,
                                                         int64_t ld_dst) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Mc) return;
    const int64_t e = blockIdx.y;
    dst[e * ld_dst + m] = src[e * ld_src + m];
}

// grad[0] += sum_{chunk, m} partial[chunk][0][m], grad[1] likewise with
// [1]; grad[2 + a] += sum_m Re lam_aa[m].  One block per output, fixed
// order (strided per thread, then a tree): deterministic.
template <typename T>
__global__ __launch_bounds__(256) void final_reduce_kernel(int N, int64_t P, int64_t Mc,
                                                           int64_t n_chunks,
                                                           const double* __restrict__ partial,
                                                           const cplx_t<T>* __restrict__ lam,
                                                           double* __restrict__ grad) {
    __shared__ double red[256];
    const int o = blockIdx.x;
    double acc = 0.0;
    if (o < 2) {
        const int64_t n = n_chunks * Mc;
        for (int64_t x = threadIdx.x; x < n; x += 256) {
            const int64_t c = x / Mc, m = x - c * Mc;
            acc += partial[(c * 2 + o) * Mc + m];
        }
    } else {
        const int a = o - 2;
        const int s = a >= N ? 1 : 0, i = a - s * N;
        const cplx_t<T>* row = lam + ((int64_t)s * P + prow(N, i)) * Mc;
        for (int64_t m = threadIdx.x; m < Mc; m += 256) acc += (double)row[m].x;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w /= 2) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) grad[o] += red[0];
}

struct AdjointLayout {
    int64_t Mc = 0, n_ckpt = 0, L = 0;
    size_t state = 0;
    size_t off_ckpt = 0, off_seg = 0, off_w3 = 0, off_lam = 0, off_part = 0, off_R = 0, total = 0;
    // forward checkpoints and segment states by resident runs that store their
    // state (when a resident configuration fits): their workspace and moments
    bool resident = false;
    size_t off_ev = 0, ev_bytes = 0, off_s1 = 0, off_s2 = 0;
    // the reverse sweep on chip (reverse_resident; -1: per-stage stream launches)
    int rev_config = -1;
};

// The instance of a stored-state run over Mc trajectories starting at `rho`
// (leading dimension Mc), moments into the layout's scratch.
ftwa_instance stored_run_instance(const ftwa_instance& in, int64_t Mc, void* rho, char* ws,
                                  const AdjointLayout& a) {
    ftwa_instance q = in;
    q.n_traj = Mc;
    q.traj_offset = 0;
    q.rho = rho;
    q.S1 = ws ? reinterpret_cast<double*>(ws + a.off_s1) : nullptr;
    q.S2 = ws ? reinterpret_cast<double*>(ws + a.off_s2) : nullptr;
    q.inv = nullptr;
    return q;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

ftwa_status plan_adjoint(const ftwa_instance* inst, int64_t n_steps, int record_every,
                         int ckpt_every, ftwa_dtype dtype, int64_t traj_chunk, AdjointLayout* out) {
    if (!inst || !inst->lat) return fail(FTWA_EINVAL, "ftwa_adjoint: no instance or lattice");
    if (dtype != FTWA_F64 && dtype != FTWA_F32) return fail(FTWA_EINVAL, "unknown dtype");
    if (n_steps < 0) return fail(FTWA_EINVAL, "n_steps < 0");
    if (record_every < 1) return fail(FTWA_EINVAL, "record_every < 1");
    if (ckpt_every < 1) return fail(FTWA_EINVAL, "ckpt_every < 1");
    if (inst->n_traj < 1) return fail(FTWA_EINVAL, "ftwa_adjoint: n_traj < 1");
    if (traj_chunk < 0) return fail(FTWA_EINVAL, "traj_chunk < 0");
    if (inst->v_site)
        return fail(FTWA_ENOTSUP, "ftwa_adjoint: no gradients through an external potential");
    if (inst->u_mat)
        return fail(FTWA_ENOTSUP, "ftwa_adjoint: no gradients with a general interaction");
    if (inst->hop_w)
        return fail(FTWA_ENOTSUP, "ftwa_adjoint: no gradients with complex hopping");
    AdjointLayout a;
    const int N = inst->lat->N;
    const int64_t P = packed_count(N);
    a.Mc = traj_chunk > 0 ? std::min<int64_t>(traj_chunk, inst->n_traj) : inst->n_traj;
    a.L = std::min<int64_t>(ckpt_every, std::max<int64_t>(n_steps, 1));
    a.n_ckpt = n_steps > 0 ? (n_steps + ckpt_every - 1) / ckpt_every : 0;
    a.state = (size_t)2 * P * a.Mc * (dtype == FTWA_F64 ? 16 : 8);
    const WaveGrid g = make_grid(P, a.Mc);
    size_t off = 0;
    a.off_ckpt = off; off = align_up(off + a.n_ckpt * a.state);
    a.off_seg = off;  off = align_up(off + a.L * a.state);
    a.off_w3 = off;   off = align_up(off + 3 * a.state);   // Y2, Y3, Y4 / acc, ya, yb
    a.off_lam = off;  off = align_up(off + 4 * a.state);   // lam, Lam, a (ping-pong)
    a.off_part = off; off = align_up(off + (size_t)g.n_elem_chunks * 2 * a.Mc * sizeof(double));
    a.off_R = off;    off = align_up(off + (size_t)2 * N * a.Mc * (dtype == FTWA_F64 ? 8 : 4));
    // stored-state runs: the forward (records every ckpt_every steps) and
    // the longest segment (records every step)
    const int64_t f_steps = (a.n_ckpt - 1) * ckpt_every, s_steps = a.L - 1;
    const ftwa_instance q = stored_run_instance(*inst, a.Mc, nullptr, nullptr, a);
    size_t bf = 0, bs = 0;
    if (evolve_stored(q, 0.01, std::max<int64_t>(f_steps, 1), ckpt_every, dtype, nullptr, 0,
                      nullptr, &bf, nullptr) == FTWA_OK &&
        evolve_stored(q, 0.01, std::max<int64_t>(s_steps, 1), 1, dtype, nullptr, 0, nullptr, &bs,
                      nullptr) == FTWA_OK) {
        a.resident = true;
        a.ev_bytes = std::max(bf, bs);
        const int64_t n_rec = std::max<int64_t>({a.n_ckpt, a.L, 2});
        const int D = 2 * N;
        a.off_ev = off; off = align_up(off + a.ev_bytes);
        a.off_s1 = off; off = align_up(off + (size_t)n_rec * D * sizeof(double));
        a.off_s2 = off; off = align_up(off + (size_t)n_rec * s2_count(D) * sizeof(double));
    }
    if (a.resident && a.n_ckpt > 0) a.rev_config = reverse_resident_config(N, dtype);
    a.total = off;
    *out = a;
    return FTWA_OK;
}

template <typename T>
ftwa_status adjoint_impl(const ftwa_instance& in, const DeviceTables& tab, const AdjointLayout& lay,
                         double dt, int64_t n_steps, int record_every, int ckpt_every,
                         int64_t n_total, const double* dL, double* grad, char* ws,
                         hipStream_t stream) {
    using C = cplx_t<T>;
    const int N = in.lat->N;
    const int64_t P = packed_count(N);
    const int D = 2 * N;
    const ftwa_dtype dtype = sizeof(T) == 8 ? FTWA_F64 : FTWA_F32;
    const T h2 = (T)(0.5 * dt), h1 = (T)dt, h6 = (T)(dt / 6.0), h3 = (T)(dt / 3.0);
    const double scale = 1.0 / (double)n_total;
    const dim3 blk(256);
    for (int64_t m0 = 0; m0 < in.n_traj; m0 += lay.Mc) {
        const int64_t Mc = std::min<int64_t>(lay.Mc, in.n_traj - m0);
        const size_t state = (size_t)2 * P * Mc;  // complex entries of one state
        auto st_at = [&](size_t off, int64_t k) {
            return reinterpret_cast<C*>(ws + off) + (size_t)k * state;
        };
        C* Y2 = st_at(lay.off_w3, 0);
        C* Y3 = st_at(lay.off_w3, 1);
        C* Y4 = st_at(lay.off_w3, 2);
        C* lam = st_at(lay.off_lam, 0);
        C* Lam = st_at(lay.off_lam, 1);
        C* aA = st_at(lay.off_lam, 2);
        C* aB = st_at(lay.off_lam, 3);
        double* partial = reinterpret_cast<double*>(ws + lay.off_part);
        const WaveGrid g = make_grid(P, Mc);
        const dim3 cgrid((unsigned)((Mc + 255) / 256), (unsigned)(2 * P));
        const C* rho0 = static_cast<const C*>(in.rho) + m0;

        StreamChunk sc;
        sc.N = N;
        sc.P = P;
        sc.Mc = Mc;
        sc.ldy = Mc;
        sc.acc = Y2;
        sc.ya = Y3;
        sc.yb = Y4;
        sc.t = in.lat->t;
        sc.U = in.U;
        sc.dt = dt;

        // ---- forward: checkpoints every ckpt_every steps
        ftwa_status st;
        if (lay.resident) {
            // one resident run from a working copy of rho(0), storing the
            // state at every checkpoint
            hipLaunchKernelGGL(copy_state_kernel<T>, cgrid, blk, 0, stream, Mc, rho0, in.n_traj,
                               st_at(lay.off_ckpt, 0), Mc);
            FTWA_LAUNCH_CHECK("copy_state_kernel");
            if (lay.n_ckpt > 1) {
                C* work = st_at(lay.off_seg, 0);
                hipLaunchKernelGGL(copy_state_kernel<T>, cgrid, blk, 0, stream, Mc,
                                   (const C*)st_at(lay.off_ckpt, 0), Mc, work, Mc);
                FTWA_LAUNCH_CHECK("copy_state_kernel");
                const ftwa_instance q = stored_run_instance(in, Mc, work, ws, lay);
                size_t b = lay.ev_bytes;
                if ((st = evolve_stored(q, dt, (lay.n_ckpt - 1) * ckpt_every, ckpt_every, dtype,
                                        st_at(lay.off_ckpt, 1), (int64_t)state, ws + lay.off_ev,
                                        &b, stream)) != FTWA_OK)
                    return st;
            }
        }
        for (int64_t k = 0; !lay.resident && k < lay.n_ckpt; ++k) {
            C* ck = st_at(lay.off_ckpt, k);
            if (k == 0) {
                hipLaunchKernelGGL(copy_state_kernel<T>, cgrid, blk, 0, stream, Mc, rho0,
                                   in.n_traj, ck, Mc);
            } else {
                hipLaunchKernelGGL(copy_state_kernel<T>, cgrid, blk, 0, stream, Mc,
                                   (const C*)st_at(lay.off_ckpt, k - 1), Mc, ck, Mc);
                sc.y = ck;
                for (int64_t n = 0; n < ckpt_every; ++n)
                    if ((st = stream_step(sc, tab, dtype, stream)) != FTWA_OK) return st;
            }
            FTWA_LAUNCH_CHECK("copy_state_kernel");
        }

        // ---- reverse sweep
        if (lay.rev_config >= 0) {
            // on chip, one launch per segment (last first)
            if ((st = zero_fill(partial, 2 * Mc, stream)) != FTWA_OK) return st;
            ReverseSegment rs;
            rs.N = N;
            rs.record_every = record_every;
            rs.Mc = Mc;
            rs.Lmax = lay.L;
            rs.n_steps = n_steps;
            rs.desc = tab.rdesc;
            rs.desc_full = tab.rdescf;
            rs.seg = st_at(lay.off_seg, 0);
            rs.lamT = lam;
            rs.lam_out = Lam;
            rs.partial = partial;
            rs.dL = dL;
            rs.scale = scale;
            rs.t = in.lat->t;
            rs.U = in.U;
            rs.dt = dt;
            for (int64_t k = lay.n_ckpt - 1; k >= 0; --k) {
                rs.base = k * ckpt_every;
                rs.L = std::min<int64_t>(ckpt_every, n_steps - rs.base);
                rs.first = k == lay.n_ckpt - 1;
                rs.last = k == 0;
                rs.ckpt = st_at(lay.off_ckpt, k);
                if ((st = reverse_resident(lay.rev_config, rs, stream)) != FTWA_OK) return st;
                FTWA_LAUNCH_CHECK("reverse_segment");
            }
            hipLaunchKernelGGL(final_reduce_kernel<T>, dim3((unsigned)(2 + D)), blk, 0, stream, N,
                               P, Mc, (int64_t)1, partial, (const C*)Lam, grad);
            FTWA_LAUNCH_CHECK("final_reduce_kernel");
            continue;
        }
        if ((st = zero_fill(reinterpret_cast<double*>(lam),
                            (int64_t)(state * sizeof(C) / sizeof(double)), stream)) != FTWA_OK)
            return st;
        if ((st = zero_fill(partial, g.n_elem_chunks * 2 * Mc, stream)) != FTWA_OK) return st;
        const dim3 sgrid((unsigned)((Mc + 255) / 256), (unsigned)D);
        auto seed = [&](int64_t step) -> ftwa_status {
            if (step % record_every != 0) return FTWA_OK;
            hipLaunchKernelGGL(seed_kernel<T>, sgrid, blk, 0, stream, N, P, Mc, lam,
                               dL + (step / record_every) * D, scale);
            FTWA_LAUNCH_CHECK("seed_kernel");
            return FTWA_OK;
        };
        if ((st = seed(n_steps)) != FTWA_OK) return st;

        StageInArgs<T> S;
        S.N = N; S.P = P; S.Mc = Mc; S.nb = tab.nb; S.elem = tab.elem;
        S.t = (T)in.lat->t; S.U = (T)in.U; S.g = g;
        VjpArgs<T> V;
        V.N = N; V.P = P; V.Mc = Mc; V.nb = tab.nb; V.elem = tab.elem;
        V.t = (T)in.lat->t; V.U = (T)in.U; V.partial = partial; V.g = g;
        T* const Rbuf = reinterpret_cast<T*>(ws + lay.off_R);
        const int4* const nb4 = reinterpret_cast<const int4*>(tab.nb);
        V.R = Rbuf;
        const int64_t n_el = (int64_t)state;
        const dim3 egrid((unsigned)((n_el + 255) / 256));

        for (int64_t k = lay.n_ckpt - 1; k >= 0; --k) {
            const int64_t base = k * ckpt_every;
            const int64_t L = std::min<int64_t>(ckpt_every, n_steps - base);
            // states y_base .. y_{base+L-1} of the segment
            hipLaunchKernelGGL(copy_state_kernel<T>, cgrid, blk, 0, stream, Mc,
                               (const C*)st_at(lay.off_ckpt, k), Mc, st_at(lay.off_seg, 0), Mc);
            FTWA_LAUNCH_CHECK("copy_state_kernel");
            if (lay.resident && L > 1) {
                // one resident run from a working copy (Y2 is free here)
                hipLaunchKernelGGL(copy_state_kernel<T>, cgrid, blk, 0, stream, Mc,
                                   (const C*)st_at(lay.off_ckpt, k), Mc, Y2, Mc);
                FTWA_LAUNCH_CHECK("copy_state_kernel");
                const ftwa_instance q = stored_run_instance(in, Mc, Y2, ws, lay);
                size_t b = lay.ev_bytes;
                if ((st = evolve_stored(q, dt, L - 1, 1, dtype, st_at(lay.off_seg, 1),
                                        (int64_t)state, ws + lay.off_ev, &b, stream)) != FTWA_OK)
                    return st;
            }
            for (int64_t n = 1; !lay.resident && n < L; ++n) {
                hipLaunchKernelGGL(copy_state_kernel<T>, cgrid, blk, 0, stream, Mc,
                                   (const C*)st_at(lay.off_seg, n - 1), Mc, st_at(lay.off_seg, n),
                                   Mc);
                sc.y = st_at(lay.off_seg, n);
                if ((st = stream_step(sc, tab, dtype, stream)) != FTWA_OK) return st;
            }
            for (int64_t n = L - 1; n >= 0; --n) {
                const C* y = st_at(lay.off_seg, n);
                // stage inputs with the forward arithmetic
                S.y = y;
                S.yin = y;  S.yout = Y2; S.c = h2;
                hipLaunchKernelGGL(stage_input_kernel<T>, grid_dim(g), blk, 0, stream, S, nb4);
                S.yin = Y2; S.yout = Y3; S.c = h2;
                hipLaunchKernelGGL(stage_input_kernel<T>, grid_dim(g), blk, 0, stream, S, nb4);
                S.yin = Y3; S.yout = Y4; S.c = h1;
                hipLaunchKernelGGL(stage_input_kernel<T>, grid_dim(g), blk, 0, stream, S, nb4);
                FTWA_LAUNCH_CHECK("stage_input_kernel");
                hipLaunchKernelGGL(step_init_kernel<T>, egrid, blk, 0, stream, n_el, lam, Lam, aA,
                                   h6);
                FTWA_LAUNCH_CHECK("step_init_kernel");
                V.lam = lam;
                V.Lam = Lam;
                auto vjp = [&]() {
                    hipLaunchKernelGGL(diag_coupling_kernel<T>, sgrid, blk, 0, stream, N, P, Mc,
                                       (const C*)V.a, V.Y, Rbuf);
                    hipLaunchKernelGGL(vjp_kernel<T>, grid_dim(g), blk, 0, stream, V, nb4);
                };
                V.Y = Y4; V.a = aA; V.a_next = aB; V.alpha = h3; V.beta = h1;
                vjp();
                V.Y = Y3; V.a = aB; V.a_next = aA; V.alpha = h3; V.beta = h2;
                vjp();
                V.Y = Y2; V.a = aA; V.a_next = aB; V.alpha = h6; V.beta = h2;
                vjp();
                V.Y = y;  V.a = aB; V.a_next = nullptr;
                vjp();
                FTWA_LAUNCH_CHECK("vjp_kernel");
                std::swap(lam, Lam);
                if ((st = seed(base + n)) != FTWA_OK) return st;
            }
        }
        hipLaunchKernelGGL(final_reduce_kernel<T>, dim3((unsigned)(2 + D)), blk, 0, stream, N, P,
                           Mc, g.n_elem_chunks, partial, lam, grad);
        FTWA_LAUNCH_CHECK("final_reduce_kernel");
    }
    return FTWA_OK;
}

}  // namespace

}  // namespace ftwa

using namespace ftwa;

extern "C" ftwa_status ftwa_adjoint_workspace_size(const ftwa_instance* inst, int64_t n_steps,
                                                   int record_every, int ckpt_every,
                                                   ftwa_dtype dtype, int64_t traj_chunk,
                                                   size_t* bytes) {
    if (!bytes) return fail(FTWA_EINVAL, "bytes is NULL");
    AdjointLayout lay;
    ftwa_status st = plan_adjoint(inst, n_steps, record_every, ckpt_every, dtype, traj_chunk, &lay);
    if (st != FTWA_OK) return st;
    *bytes = lay.total;
    return FTWA_OK;
}

extern "C" ftwa_status ftwa_adjoint(const ftwa_instance* inst, double dt, int64_t n_steps,
                                    int record_every, int ckpt_every, ftwa_dtype dtype,
                                    int64_t n_total, const double* dL_dnbar, double* grad,
                                    int64_t traj_chunk, void* workspace, size_t workspace_bytes,
                                    void* stream_) {
    AdjointLayout lay;
    ftwa_status st = plan_adjoint(inst, n_steps, record_every, ckpt_every, dtype, traj_chunk, &lay);
    if (st != FTWA_OK) return st;
    const ftwa_instance& in = *inst;
    if (!in.rho) return fail(FTWA_EINVAL, "ftwa_adjoint: rho is NULL");
    if (!dL_dnbar || !grad) return fail(FTWA_EINVAL, "ftwa_adjoint: NULL dL_dnbar or grad");
    if (n_total < in.n_traj) return fail(FTWA_EINVAL, "ftwa_adjoint: n_total < n_traj");
    if (!workspace || workspace_bytes < lay.total)
        return fail(FTWA_EINVAL, "ftwa_adjoint: workspace too small (" +
                                     std::to_string(workspace_bytes) + " < " +
                                     std::to_string(lay.total) + " bytes)");
    DeviceTables tab;
    if ((st = device_tables(in.lat, &tab)) != FTWA_OK) return st;
    hipStream_t stream = (hipStream_t)stream_;
    if ((st = zero_fill(grad, 2 + 2 * (int64_t)in.lat->N, stream)) != FTWA_OK) return st;
    char* ws = static_cast<char*>(workspace);
    if (dtype == FTWA_F64)
        return adjoint_impl<double>(in, tab, lay, dt, n_steps, record_every, ckpt_every, n_total,
                                    dL_dnbar, grad, ws, stream);
    return adjoint_impl<float>(in, tab, lay, dt, n_steps, record_every, ckpt_every, n_total,
                               dL_dnbar, grad, ws, stream);
}

// evolve_stream.hip -- "stream" path of the fTWA time integration: the state
// lives in HBM in the packed, trajectory-innermost layout and every stage of
// the classical Runge-Kutta step is one kernel launch over all elements of a
// chunk of trajectories.
//
// Equation of motion: Eq. (6) of arXiv:2212.04352 with j_ij = t on bonds and
// u_ij = U delta_ij:
//   f_ij = i [ t (sum_{k in nb(j)} rho_ik - sum_{k in nb(i)} rho_kj) + U (d_i - d_j) rho_ij ],
// d = diagonal of the other spin block.  A wave owns 64 consecutive
// trajectories and walks a run of packed elements; (i, j) and all neighbour
// indices are therefore wave-uniform (scalar registers) and every load is one
// coalesced 512 B (FP32) or 1 KiB (FP64) row segment.  Elements i > j are read
// as conjugates of the stored upper triangle.  With complex (Peierls)
// hopping j_ik = t w_ik the two sums become sum_{k in nb(j)} w_jk rho_ik and
// sum_{k in nb(i)} conj(w_ik) rho_kj (j_ki = conj(j_ik): the Hamiltonian is
// Hermitian), so both read only the rows of i and j of the ratio table.
#include "device_common.h"
#include "ftwa_internal.h"

namespace ftwa {

namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kElemsPerWave = 16;

template <typename T> struct StageArgs {
    int N;
    int64_t P;
    int64_t Mc;
    cplx_t<T>* y;
    int64_t ldy;
    const cplx_t<T>* yin;  // stage input
    int64_t ldin;
    cplx_t<T>* yout;       // next stage input (stages 1-3)
    cplx_t<T>* acc;        // Runge-Kutta accumulator, stride Mc
    const int32_t* nb;     // [N][4]
    const uint32_t* elem;  // [P]: packed element -> i | j << 16
    T t, U, c;             // c: this stage's coefficient (h/2, h/2, h, h/6)
    const double* vsite;   // NULL, or [N]: profile of the external on-site potential
    const double* env_at;  // its envelope at this stage's time
    const T* D;            // NULL (on-site U), or [2][N][Mc]: D_i of a general interaction
    const double2* hop;    // complex hopping: [N][3] ratios w_ik = j_ik / t at this stage's time
    int64_t n_elem_chunks; // ceil(2P / kElemsPerWave)
    int64_t n_work;        // n_traj_blocks * n_elem_chunks waves
    int64_t blocks_per_xcd;
};

__device__ __forceinline__ int64_t prow(int N, int i) {
    return (int64_t)i * N - (int64_t)i * (i - 1) / 2;
}

// The ratio w rounded once to T, conjugated if `cj`.
template <typename T>
__device__ __forceinline__ cplx_t<T> ratio(double2 w, bool cj) {
    cplx_t<T> r;
    r.x = (T)w.x;
    r.y = cj ? -(T)w.y : (T)w.y;
    return r;
}

// x <- w x: re = fma(wr, xr, -(wi xi)), im = fma(wr, xi, wi xr).
template <typename T>
__device__ __forceinline__ void cmul_ratio(cplx_t<T> w, cplx_t<T>& x) {
    const T re = fma_rn<T>(w.x, x.x, -(w.y * x.y));
    const T im = fma_rn<T>(w.x, x.y, w.y * x.x);
    x.x = re;
    x.y = im;
}

// Neighbour sums with complex hopping: col = sum_n w[j][n] rho_{i, nb(j)_n},
// row = sum_n conj(w[i][n]) rho_{nb(i)_n, j}, slots (ascending k) summed in
// order as in neighbour_sums.  wi: conj(w[i][.]) already in T (constant
// along a packed row); the ratios of j are read here (wave-uniform).
template <typename T>
__device__ __forceinline__ void hop_sums(const cplx_t<T>* X, int64_t ld, int N, int4 nbj,
                                         int4 nbi, int i, int j, int64_t m,
                                         const double2* __restrict__ w, const cplx_t<T>* wi,
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
        cmul_ratio<T>(ratio<T>(w[j * 3 + n], false), c[n]);
        cmul_ratio<T>(wi[n], r[n]);
        if (n >= nbj.w) c[n].x = c[n].y = 0;
        if (n >= nbi.w) r[n].x = r[n].y = 0;
    }
    col = cadd(cadd(c[0], c[1]), c[2]);
    row = cadd(cadd(r[0], r[1]), r[2]);
}

// nb4: the neighbour rows (also in A.nb) as a separate read-only argument,
// so that the wave-uniform row reads are scalar loads.  HOP: complex hopping.
template <typename T, int STAGE, bool HOP>
__global__ __launch_bounds__(256) void rk4_stage_stream(StageArgs<T> A,
                                                        const int4* __restrict__ nb4) {
    // XCD-aware numbering: blocks are dealt round-robin to the 8 XCDs, so
    // consecutive virtual blocks (neighbouring elements of the same
    // trajectories) are made to run on the same XCD and share its L2.
    const int64_t xcd = blockIdx.x % 8;
    const int64_t slot = blockIdx.x / 8;
    const int64_t vblock = xcd * A.blocks_per_xcd + slot;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int lane = threadIdx.x % 64;
    const int64_t w = vblock * kWavesPerBlock + wave;
    if (w >= A.n_work) return;
    const int64_t tb = w / A.n_elem_chunks;
    const int64_t chunk = w - tb * A.n_elem_chunks;
    const int64_t m_raw = tb * 64 + lane;
    const bool active = m_raw < A.Mc;
    const int64_t m = active ? m_raw : A.Mc - 1;  // inactive lanes load in bounds, never store
    const int N = A.N;
    const int64_t P = A.P;
    const int64_t q0 = chunk * kElemsPerWave;
    const int64_t q1 = q0 + kElemsPerWave < 2 * P ? q0 + kElemsPerWave : 2 * P;
    // (spin, i, j) of the first element, then advanced along the packed rows
    int s = q0 >= P ? 1 : 0;
    int i, j;
    {
        const uint32_t ij = A.elem[q0 - s * P];
        i = (int)(ij & 0xffffu);
        j = (int)(ij >> 16);
    }
    // complex hopping: conj(w[i][.]) in T, renewed when the row changes
    cplx_t<T> wi[3];
    if (HOP) {
#pragma unroll
        for (int n = 0; n < 3; ++n) wi[n] = ratio<T>(A.hop[i * 3 + n], true);
    }
    for (int64_t q = q0; q < q1; ++q) {
        const int64_t p = q - s * P;
        const cplx_t<T>* Ys = A.yin + (int64_t)s * P * A.ldin;
        const cplx_t<T>* Yo = A.yin + (int64_t)(1 - s) * P * A.ldin;
        // col = sum_{k in nb(j)} rho_ik, row = sum_{k in nb(i)} rho_kj,
        // ascending k (loads issued together)
        cplx_t<T> col, row;
        if (HOP)
            hop_sums<T>(Ys, A.ldin, N, nb4[j], nb4[i], i, j, m, A.hop, wi, col, row);
        else
            neighbour_sums<T>(Ys, A.ldin, N, nb4[j], nb4[i], i, j, m, col, row);
        const int64_t ep = p;
        const int64_t e_ws = ((int64_t)s * P + ep) * A.Mc + m;  // workspace index
        const int64_t e_y = ((int64_t)s * P + ep) * A.ldy + m;   // state index
        const cplx_t<T> own = Ys[ep * A.ldin + m];
        const T d_i = Yo[prow(N, i) * A.ldin + m].x;
        const T d_j = Yo[prow(N, j) * A.ldin + m].x;
        // operands of the update, loaded with the stencil (in bounds for
        // inactive lanes too)
        cplx_t<T> ac, yv;
        if (STAGE > 1) ac = A.acc[e_ws];
        if (STAGE > 1) yv = A.y[e_y];
        T a = A.D ? A.D[((int64_t)s * N + i) * A.Mc + m] - A.D[((int64_t)s * N + j) * A.Mc + m]
                  : A.U * (d_i - d_j);
        // external potential: a + A(tau) (v_i - v_j), each factor rounded once
        // to T (i, j and the envelope are wave-uniform: scalar loads)
        if (A.vsite) a = a + (T)*A.env_at * ((T)A.vsite[i] - (T)A.vsite[j]);
        const cplx_t<T> k = rhs_element<T>(col, row, own, A.t, a);
        if (STAGE == 1) {
            // Y_1 = y, so `own` is y itself
            if (active) {
                A.acc[e_ws] = k;
                cplx_t<T> nx;
                nx.x = fma_rn<T>(A.c, k.x, own.x);
                nx.y = fma_rn<T>(A.c, k.y, own.y);
                A.yout[e_ws] = nx;
            }
        } else if (STAGE == 2 || STAGE == 3) {
            if (active) {
                ac.x = fma_rn<T>((T)2, k.x, ac.x);
                ac.y = fma_rn<T>((T)2, k.y, ac.y);
                A.acc[e_ws] = ac;
                cplx_t<T> nx;
                nx.x = fma_rn<T>(A.c, k.x, yv.x);
                nx.y = fma_rn<T>(A.c, k.y, yv.y);
                A.yout[e_ws] = nx;
            }
        } else {
            if (active) {
                ac.x = ac.x + k.x;
                ac.y = ac.y + k.y;
                yv.x = fma_rn<T>(A.c, ac.x, yv.x);
                yv.y = fma_rn<T>(A.c, ac.y, yv.y);
                A.y[e_y] = yv;
            }
        }
        // next packed element: along the row, then the next row, then the
        // other spin
        if (++j == N) {
            if (++i == N) {
                s = 1;
                i = 0;
            }
            j = i;
            if (HOP && q + 1 < q1) {
#pragma unroll
                for (int n = 0; n < 3; ++n) wi[n] = ratio<T>(A.hop[i * 3 + n], true);
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void record_diag_kernel(int N, int64_t P, int64_t Mc,
                                                          const cplx_t<T>* __restrict__ y,
                                                          int64_t ldy, double* __restrict__ X) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Mc) return;
    const int a = blockIdx.y;  // s * N + i
    const int s = a >= N ? 1 : 0;
    const int i = a - s * N;
    const int64_t p = (int64_t)i * N - (int64_t)i * (i - 1) / 2;
    X[(int64_t)a * Mc + m] = (double)y[((int64_t)s * P + p) * ldy + m].x;
}

// D[s][i][m] = sum_k u_ki (d_k + 1/2) for spin block s from the other block's
// diagonal d of the stage input (the general interaction of Eq. (6)):
// fma over ascending k from 0, u rounded once to T.  One thread per
// trajectory; blocks over (trajectory block, site, spin), so u_ki is
// wave-uniform (scalar loads) and the diagonal loads are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void interaction_kernel(int N, int64_t P, int64_t Mc,
                                                          const cplx_t<T>* __restrict__ yin,
                                                          int64_t ldin,
                                                          const double* __restrict__ u,
                                                          T* __restrict__ D) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    const int s = blockIdx.z;
    const int64_t mm = m < Mc ? m : Mc - 1;  // in-bounds loads for the tail, no store
    const cplx_t<T>* Yo = yin + (int64_t)(1 - s) * P * ldin;
    T acc = 0;
    for (int k = 0; k < N; ++k) {
        const T dk = Yo[((int64_t)k * N - (int64_t)k * (k - 1) / 2) * ldin + mm].x;
        acc = fma_rn<T>((T)u[(int64_t)k * N + i], dk + (T)0.5, acc);
    }
    if (m < Mc) D[((int64_t)s * N + i) * Mc + m] = acc;
}

template <typename T>
ftwa_status step_impl(const StreamChunk& c, const DeviceTables& tab, hipStream_t stream) {
    StageArgs<T> A;
    A.N = c.N;
    A.P = c.P;
    A.Mc = c.Mc;
    A.y = static_cast<cplx_t<T>*>(c.y);
    A.ldy = c.ldy;
    A.acc = static_cast<cplx_t<T>*>(c.acc);
    A.nb = tab.nb;
    A.elem = tab.elem;
    A.t = (T)c.t;
    A.U = (T)c.U;
    A.n_elem_chunks = (2 * c.P + kElemsPerWave - 1) / kElemsPerWave;
    const int64_t n_tb = (c.Mc + 63) / 64;
    A.n_work = n_tb * A.n_elem_chunks;
    const int64_t n_blocks = (A.n_work + kWavesPerBlock - 1) / kWavesPerBlock;
    A.blocks_per_xcd = (n_blocks + 7) / 8;
    const dim3 grid((unsigned)(A.blocks_per_xcd * 8)), block(64 * kWavesPerBlock);
    cplx_t<T>* ya = static_cast<cplx_t<T>*>(c.ya);
    cplx_t<T>* yb = static_cast<cplx_t<T>*>(c.yb);
    const T c_half = (T)(0.5 * c.dt), c_full = (T)c.dt, c_sixth = (T)(c.dt / 6.0);
    const int4* nb4 = reinterpret_cast<const int4*>(tab.nb);
    // stage times t_n, t_n + h/2 (twice), t_n + h: envelope samples 2n, 2n+1, 2n+2
    A.vsite = c.v_site;
    const double* env = c.v_site ? c.v_env + 2 * c.step : nullptr;
    // general interaction: D of each stage input before the stage
    A.D = c.u_mat ? static_cast<T*>(c.D) : nullptr;
    const dim3 igrid((unsigned)((c.Mc + 255) / 256), (unsigned)c.N, 2u), iblock(256);
    auto interaction = [&](const cplx_t<T>* yin, int64_t ldin) {
        if (c.u_mat)
            hipLaunchKernelGGL((interaction_kernel<T>), igrid, iblock, 0, stream, c.N, c.P, c.Mc,
                               yin, ldin, c.u_mat, static_cast<T*>(c.D));
    };

    // complex hopping: the ratio table of the same half step as the envelope
    const size_t hop_half = (size_t)c.N * 3;
    const double2* hop = c.hop_w ? reinterpret_cast<const double2*>(c.hop_w) + 2 * c.step * hop_half
                                 : nullptr;
    auto stage = [&](auto kernel_plain, auto kernel_hop, int half) {
        A.env_at = env ? env + half : nullptr;
        A.hop = hop ? hop + half * hop_half : nullptr;
        interaction(A.yin, A.ldin);
        if (hop)
            hipLaunchKernelGGL(kernel_hop, grid, block, 0, stream, A, nb4);
        else
            hipLaunchKernelGGL(kernel_plain, grid, block, 0, stream, A, nb4);
    };

    A.yin = A.y; A.ldin = c.ldy; A.yout = ya; A.c = c_half;
    stage(rk4_stage_stream<T, 1, false>, rk4_stage_stream<T, 1, true>, 0);
    A.yin = ya; A.ldin = c.Mc; A.yout = yb; A.c = c_half;
    stage(rk4_stage_stream<T, 2, false>, rk4_stage_stream<T, 2, true>, 1);
    A.yin = yb; A.ldin = c.Mc; A.yout = ya; A.c = c_full;
    stage(rk4_stage_stream<T, 3, false>, rk4_stage_stream<T, 3, true>, 1);
    A.yin = ya; A.ldin = c.Mc; A.yout = nullptr; A.c = c_sixth;
    stage(rk4_stage_stream<T, 4, false>, rk4_stage_stream<T, 4, true>, 2);
    FTWA_LAUNCH_CHECK("rk4_stage_stream");
    return FTWA_OK;
}

}  // namespace

ftwa_status stream_step(const StreamChunk& c, const DeviceTables& tab, ftwa_dtype dtype,
                        hipStream_t stream) {
    return dtype == FTWA_F64 ? step_impl<double>(c, tab, stream) : step_impl<float>(c, tab, stream);
}

namespace {

// One thread per trajectory walks every packed element of both spins (the
// element index is uniform, so loads are coalesced over trajectories) and
// accumulates in FP64: hop_s = sum_i sum_{k in nb(i)} Re rho_ik (each bond
// twice) and frob_s = sum_ij |rho_ij|^2.
template <typename T>
__global__ __launch_bounds__(256) void record_inv_kernel(int N, int64_t P, int64_t Mc,
                                                         const cplx_t<T>* __restrict__ y,
                                                         int64_t ldy,
                                                         const uint32_t* __restrict__ elem,
                                                         const int32_t* __restrict__ nb,
                                                         double* __restrict__ parts) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= Mc) return;
    for (int s = 0; s < 2; ++s) {
        double hop = 0.0, frob = 0.0;
        for (int64_t p = 0; p < P; ++p) {
            const uint32_t ij = elem[p];
            const int i = (int)(ij & 0xffffu), j = (int)(ij >> 16);
            const cplx_t<T> v = y[((int64_t)s * P + p) * ldy + m];
            const double re = (double)v.x, im = (double)v.y;
            if (i == j) {
                frob += re * re;
            } else {
                frob += 2.0 * (re * re + im * im);
                const int d = nb[i * 4 + 3];
                bool bond = false;
                for (int n = 0; n < d; ++n) bond = bond || nb[i * 4 + n] == j;
                if (bond) hop += 2.0 * re;
            }
        }
        parts[(s * 2) * Mc + m] = hop;
        parts[(s * 2 + 1) * Mc + m] = frob;
    }
}

}  // namespace

ftwa_status record_inv(const StreamChunk& c, const DeviceTables& tab, ftwa_dtype dtype,
                       double* parts, hipStream_t stream) {
    const dim3 grid((unsigned)((c.Mc + 255) / 256)), block(256);
    if (dtype == FTWA_F64)
        hipLaunchKernelGGL(record_inv_kernel<double>, grid, block, 0, stream, c.N, c.P, c.Mc,
                           static_cast<const double2*>(c.y), c.ldy, tab.elem, tab.nb, parts);
    else
        hipLaunchKernelGGL(record_inv_kernel<float>, grid, block, 0, stream, c.N, c.P, c.Mc,
                           static_cast<const float2*>(c.y), c.ldy, tab.elem, tab.nb, parts);
    FTWA_LAUNCH_CHECK("record_inv_kernel");
    return FTWA_OK;
}

ftwa_status record_diag(const StreamChunk& c, const DeviceTables& tab, ftwa_dtype dtype,
                        double* X, hipStream_t stream) {
    (void)tab;
    const dim3 grid((unsigned)((c.Mc + 255) / 256), (unsigned)(2 * c.N)), block(256);
    if (dtype == FTWA_F64)
        hipLaunchKernelGGL(record_diag_kernel<double>, grid, block, 0, stream, c.N, c.P, c.Mc,
                           static_cast<const double2*>(c.y), c.ldy, X);
    else
        hipLaunchKernelGGL(record_diag_kernel<float>, grid, block, 0, stream, c.N, c.P, c.Mc,
                           static_cast<const float2*>(c.y), c.ldy, X);
    FTWA_LAUNCH_CHECK("record_diag_kernel");
    return FTWA_OK;
}

}  // namespace ftwa

// moments.hip -- FP64 ensemble moments of the diagonal phase-space variables
// (the stochastic averages of Eq. (5) and Eq. (10) of arXiv:2212.04352):
//   S1[r][a]  += sum_m X[r][a][m]
//   S2[r][ab] += sum_m X[r][a][m] X[r][b][m]      (a <= b, packed)
// X holds one chunk of trajectories, m innermost.  S2 is a symmetric rank-Mc
// update: 32 x 32 output tiles, 2 x 2 outputs per thread, the trajectory
// axis staged through LDS 64 at a time.  Each output is one FP64 fma chain
// in ascending m within a split; splits are added in split order, so the
// result is deterministic.
#include "ftwa_internal.h"

namespace ftwa {

namespace {

constexpr int kTile = 32;
constexpr int kMBlock = 64;

__device__ __forceinline__ int64_t s2_index(int a, int b, int D) {
    return (int64_t)a * D - (int64_t)a * (a - 1) / 2 + (b - a);
}

// tile pair index -> (ta, tb) with ta <= tb
__device__ __forceinline__ void tile_pair(int idx, int nt, int* ta, int* tb) {
    int a = 0;
    int rem = idx;
    while (rem >= nt - a) {
        rem -= nt - a;
        ++a;
    }
    *ta = a;
    *tb = a + rem;
}

__global__ __launch_bounds__(256) void s2_partial_kernel(int D, int64_t Mc, int n_split,
                                                         int64_t m_per_split,
                                                         const double* __restrict__ X,
                                                         double* __restrict__ out,
                                                         int64_t out_rec_stride,
                                                         int64_t out_split_stride,
                                                         int accumulate) {
    __shared__ double xa[kTile][kMBlock + 1];
    __shared__ double xb[kTile][kMBlock + 1];
    const int nt = (D + kTile - 1) / kTile;
    int ta, tb;
    tile_pair(blockIdx.x, nt, &ta, &tb);
    const int split = blockIdx.y;
    const int r = blockIdx.z;
    const int64_t m_lo = (int64_t)split * m_per_split;
    const int64_t m_hi = m_lo + m_per_split < Mc ? m_lo + m_per_split : Mc;
    const double* Xr = X + (int64_t)r * D * Mc;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int64_t m0 = m_lo; m0 < m_hi; m0 += kMBlock) {
        // stage 32 rows x 64 trajectories of each tile (zero beyond the ends)
        for (int e = threadIdx.x; e < kTile * kMBlock; e += 256) {
            const int row = e / kMBlock, col = e % kMBlock;
            const int64_t m = m0 + col;
            const int a = ta * kTile + row, b = tb * kTile + row;
            xa[row][col] = (a < D && m < m_hi) ? Xr[(int64_t)a * Mc + m] : 0.0;
            xb[row][col] = (b < D && m < m_hi) ? Xr[(int64_t)b * Mc + m] : 0.0;
        }
        __syncthreads();
        for (int mm = 0; mm < kMBlock; ++mm) {
            const double a0 = xa[ty][mm], a1 = xa[ty + 16][mm];
            const double b0 = xb[tx][mm], b1 = xb[tx + 16][mm];
            acc[0][0] = __builtin_fma(a0, b0, acc[0][0]);
            acc[0][1] = __builtin_fma(a0, b1, acc[0][1]);
            acc[1][0] = __builtin_fma(a1, b0, acc[1][0]);
            acc[1][1] = __builtin_fma(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            const int a = ta * kTile + ty + 16 * u, b = tb * kTile + tx + 16 * v;
            if (a >= D || b >= D || a > b) continue;
            double* dst = out + (int64_t)r * out_rec_stride + (int64_t)split * out_split_stride +
                          s2_index(a, b, D);
            *dst = accumulate ? *dst + acc[u][v] : acc[u][v];
        }
}

// S1 partial sums: one wave per (a, split, record), lanes stride m, then a
// fixed butterfly over the wave.
__global__ __launch_bounds__(64) void s1_partial_kernel(int D, int64_t Mc, int64_t m_per_split,
                                                        const double* __restrict__ X,
                                                        double* __restrict__ out,
                                                        int64_t out_rec_stride,
                                                        int64_t out_split_stride,
                                                        int accumulate) {
    const int a = blockIdx.x, split = blockIdx.y, r = blockIdx.z;
    const int64_t m_lo = (int64_t)split * m_per_split;
    const int64_t m_hi = m_lo + m_per_split < Mc ? m_lo + m_per_split : Mc;
    const double* row = X + ((int64_t)r * D + a) * Mc;
    double s = 0.0;
    for (int64_t m = m_lo + threadIdx.x; m < m_hi; m += 64) s += row[m];
    for (int off = 32; off > 0; off /= 2) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) {
        double* dst = out + (int64_t)r * out_rec_stride + (int64_t)split * out_split_stride + a;
        *dst = accumulate ? *dst + s : s;
    }
}

// S[r][k] += sum over splits (in order) of part[r][split][k]
__global__ __launch_bounds__(256) void add_splits_kernel(int64_t count, int n_split,
                                                         int64_t n_rec,
                                                         const double* __restrict__ part,
                                                         double* __restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count * n_rec) return;
    const int64_t r = e / count, k = e - r * count;
    double s = part[(r * n_split) * count + k];
    for (int sp = 1; sp < n_split; ++sp) s += part[(r * n_split + sp) * count + k];
    S[e] += s;
}

__global__ __launch_bounds__(256) void fill_zero_kernel(double* p, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0.0;
}

__global__ __launch_bounds__(256) void fill_zero_words_kernel(unsigned* p, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) p[e] = 0u;
}

int choose_splits(int D, int64_t Mc, int64_t n_rec) {
    const int nt = (D + kTile - 1) / kTile;
    const int64_t pairs = (int64_t)nt * (nt + 1) / 2;
    int64_t want = (4096 + pairs * n_rec - 1) / (pairs * n_rec);
    const int64_t max_split = (Mc + kMBlock - 1) / kMBlock;
    if (want > max_split) want = max_split;
    if (want < 1) want = 1;
    if (want > 64) want = 64;
    return (int)want;
}

}  // namespace

size_t moments_workspace_bytes(int D, int64_t Mc, int64_t n_rec) {
    const int n_split = choose_splits(D, Mc, n_rec);
    if (n_split == 1) return 0;
    return (size_t)n_rec * n_split * (size_t)(s2_count(D) + D) * sizeof(double);
}

ftwa_status moments_accumulate(int D, int64_t Mc, int64_t n_rec, const double* X, double* S1,
                               double* S2, void* scratch, hipStream_t stream) {
    if (Mc == 0 || n_rec == 0) return FTWA_OK;
    const int n_split = choose_splits(D, Mc, n_rec);
    const int64_t m_per = ((Mc + n_split - 1) / n_split + kMBlock - 1) / kMBlock * kMBlock;
    const int split_used = (int)((Mc + m_per - 1) / m_per);
    const int nt = (D + kTile - 1) / kTile;
    const int pairs = nt * (nt + 1) / 2;
    const int64_t n2 = s2_count(D);
    if (split_used == 1) {
        hipLaunchKernelGGL(s2_partial_kernel, dim3(pairs, 1, (unsigned)n_rec), dim3(256), 0, stream,
                           D, Mc, 1, m_per, X, S2, n2, 0, 1);
        hipLaunchKernelGGL(s1_partial_kernel, dim3(D, 1, (unsigned)n_rec), dim3(64), 0, stream, D,
                           Mc, m_per, X, S1, (int64_t)D, 0, 1);
        FTWA_LAUNCH_CHECK("moments (single split)");
        return FTWA_OK;
    }
    double* p2 = static_cast<double*>(scratch);
    double* p1 = p2 + (size_t)n_rec * split_used * n2;
    hipLaunchKernelGGL(s2_partial_kernel, dim3(pairs, split_used, (unsigned)n_rec), dim3(256), 0,
                       stream, D, Mc, split_used, m_per, X, p2, n2 * split_used, n2, 0);
    hipLaunchKernelGGL(s1_partial_kernel, dim3(D, split_used, (unsigned)n_rec), dim3(64), 0, stream,
                       D, Mc, m_per, X, p1, (int64_t)D * split_used, (int64_t)D, 0);
    hipLaunchKernelGGL(add_splits_kernel, dim3((unsigned)((n2 * n_rec + 255) / 256)), dim3(256), 0,
                       stream, n2, split_used, n_rec, p2, S2);
    hipLaunchKernelGGL(add_splits_kernel, dim3((unsigned)((D * n_rec + 255) / 256)), dim3(256), 0,
                       stream, (int64_t)D, split_used, n_rec, p1, S1);
    FTWA_LAUNCH_CHECK("moments");
    return FTWA_OK;
}

ftwa_status zero_fill(double* p, int64_t n, hipStream_t stream) {
    if (n <= 0) return FTWA_OK;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
    FTWA_LAUNCH_CHECK("fill_zero_kernel");
    return FTWA_OK;
}

namespace {

// One block per record r.  For every trajectory m of the chunk: trace of each
// spin, the Weyl Hamiltonian of Appendix A.3 (Eq. (A10) with j_ij = t on bonds,
// u_ij = U delta_ij),
//   H_W = -t (hop_up + hop_dn) + U sum_i (rho_ii,up + 1/2)(rho_ii,dn + 1/2),
// and the squared Frobenius norms, each compared with record 0.  Maxima over
// trajectories (exact, so order-independent) and the count of trajectories
// with a non-finite value are combined into inv[r].
__global__ __launch_bounds__(256) void invariants_kernel(int N, int64_t Mc, double t, double U,
                                                         const double* __restrict__ X,
                                                         const double* __restrict__ parts,
                                                         double* __restrict__ inv) {
    __shared__ double red[4][256];
    const int r = blockIdx.x;
    const int D = 2 * N;
    double m_tr = 0.0, m_hw = 0.0, m_fr = 0.0, bad = 0.0;
    for (int64_t m = threadIdx.x; m < Mc; m += 256) {
        double tr[2][2], hw[2], fr[2][2];
        bool finite = true;
        for (int q = 0; q < 2; ++q) {  // q = 0: record 0, q = 1: record r
            const int64_t rr = q == 0 ? 0 : r;
            const double* Xr = X + rr * D * Mc;
            double inter = 0.0;
            for (int s = 0; s < 2; ++s) {
                double acc = 0.0;
                for (int i = 0; i < N; ++i) acc += Xr[(int64_t)(s * N + i) * Mc + m];
                tr[q][s] = acc;
            }
            for (int i = 0; i < N; ++i)
                inter += (Xr[(int64_t)i * Mc + m] + 0.5) * (Xr[(int64_t)(N + i) * Mc + m] + 0.5);
            const double* pr = parts + rr * 4 * Mc;
            const double hop = pr[0 * Mc + m] + pr[2 * Mc + m];
            hw[q] = -t * hop + U * inter;
            fr[q][0] = pr[1 * Mc + m];
            fr[q][1] = pr[3 * Mc + m];
            finite = finite && isfinite(tr[q][0]) && isfinite(tr[q][1]) && isfinite(hw[q]) &&
                     isfinite(fr[q][0]) && isfinite(fr[q][1]);
        }
        if (!finite) {
            bad += 1.0;
            continue;
        }
        m_tr = fmax(m_tr, fmax(fabs(tr[1][0] - tr[0][0]), fabs(tr[1][1] - tr[0][1])));
        m_hw = fmax(m_hw, fabs(hw[1] - hw[0]));
        m_fr = fmax(m_fr, fmax(fabs(fr[1][0] - fr[0][0]), fabs(fr[1][1] - fr[0][1])));
    }
    red[0][threadIdx.x] = m_tr;
    red[1][threadIdx.x] = m_hw;
    red[2][threadIdx.x] = m_fr;
    red[3][threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w /= 2) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 3; ++k)
                red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + w]);
            red[3][threadIdx.x] += red[3][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = inv + (int64_t)r * 4;
        o[0] = fmax(o[0], red[0][0]);
        o[1] = fmax(o[1], red[1][0]);
        o[2] = fmax(o[2], red[2][0]);
        o[3] += red[3][0];
    }
}

}  // namespace

ftwa_status invariants_accumulate(int N, int64_t Mc, int64_t n_rec, double t, double U,
                                  const double* X, const double* parts, double* inv,
                                  hipStream_t stream) {
    if (Mc == 0 || n_rec == 0) return FTWA_OK;
    hipLaunchKernelGGL(invariants_kernel, dim3((unsigned)n_rec), dim3(256), 0, stream, N, Mc, t, U,
                       X, parts, inv);
    FTWA_LAUNCH_CHECK("invariants_kernel");
    return FTWA_OK;
}

ftwa_status zero_words(unsigned* p, int64_t n, hipStream_t stream) {
    if (n <= 0) return FTWA_OK;
    hipLaunchKernelGGL(fill_zero_words_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       p, n);
    FTWA_LAUNCH_CHECK("fill_zero_words_kernel");
    return FTWA_OK;
}

}  // namespace ftwa

// adjoint_resident.hip -- the reverse sweep of ftwa_adjoint on chip: one
// workgroup per trajectory holds both spin blocks of its state, the three
// recomputed stage inputs and the cotangents in registers and the current
// stencil input in LDS, for one checkpoint segment per launch.
//
// The arithmetic is that of the stream reverse sweep in adjoint.hip (the
// discrete adjoint of the classical Runge-Kutta map of Eq. (6) of
// arXiv:2212.04352, cotangents with respect to <A, B> = Re tr(A^H B)):
//   forward over the segment from its checkpoint, storing every state in a
//   per-trajectory scratch (the forward kernels' arithmetic: the states equal
//   theirs bit for bit);
//   then for each step, last first: the stage inputs Y2, Y3, Y4 from y, and
//     a4 = h/6 lam;             mu4 = df(Y4)^T a4
//     a3 = h/3 lam + h mu4;     mu3 = df(Y3)^T a3
//     a2 = h/3 lam + h/2 mu3;   mu2 = df(Y2)^T a2
//     a1 = h/6 lam + h/2 mu2;   mu1 = df(y)^T a1
//     lam <- lam + mu1 + mu2 + mu3 + mu4, seeded at the records,
//   with (df(Y)^T a)_s = -f_s^lin(a_s; D from Y) plus, on the diagonal (i,i),
//   -2U R_sbar,i, R_s,i = sum_{k != i} W_s,ik, W = Im(conj(a) Y) (a row sum
//   of the other spin block).
// Parameter sums (FP64 accumulators):
//   <a, df/dt> = -sum w Im(conj(g) Y), g = col(a) - row(a), w = 2 off the
//     diagonal (each stored element stands for two), 1 on it;
//   <a, df/dU> = -sum w (d_i - d_j) Im(conj(a_ij) Y_ij), d the other block's
//     diagonal; W is antisymmetric, so this equals -2 sum_{s,i} Y_s,ii
//     R_sbar,i and is taken from the row sums at the diagonal elements.
// The products Im(conj(g) Y), W and the row sums are formed in the working
// precision (the stream sweep forms the first in FP64 and sums the elements
// individually), so the gradients agree with it to rounding.  Every sum has a
// fixed order: repeated runs give identical bits.
//
// LDS (one trajectory): two copies of the stencil input X, W as a full
// matrix per spin ([2][N][N], the transposed entry holding -W, zero on the
// diagonal, so a row sum reads a contiguous row), the diagonals of the four
// stage inputs Yd[4][2N], the partial row sums Rp[2N][CH] and the per-wave
// parameter sums.  X is either packed (XF = false: the 2P stored elements,
// transposed reads conjugate) or, where it fits, the full matrix of both
// spins (XF: every element writes itself and its conjugate transpose, and
// the stencil reads without signs); after both, a zero entry for the missing
// neighbours of degree-1 and degree-2 sites.
#include <algorithm>

#include "device_common.h"
#include "ftwa_internal.h"

namespace ftwa {

namespace {

template <typename T> struct RevArgs {
    int N;
    int E;                  // 2P: stored elements of both spins
    int XN;                 // entries of one X copy (the zero entry last)
    int CH;                 // partial sums per row of the diagonal coupling
    int record_every;
    int64_t Mc;             // trajectories of the chunk (one workgroup each)
    int64_t L;              // steps of this segment
    int64_t Lmax;           // segment scratch per trajectory, in states
    int64_t base;           // global index of the segment's first step
    int64_t n_steps;
    bool first;             // the segment that ends at n_steps (lam starts at zero)
    bool last;              // the segment that starts at step 0
    const uint4* desc;      // [E][2] descriptors (see reverse_descriptors)
    const cplx_t<T>* ckpt;  // y_base, trajectory-innermost [E][Mc]
    cplx_t<T>* seg;         // [Mc][Lmax][E] states of the segment
    cplx_t<T>* lamT;        // [Mc][E] cotangent carried between segments
    cplx_t<T>* lam_out;     // [E][Mc] (diagonal entries written by the last segment)
    double* partial;        // [2][Mc] dL/dU, dL/dt sums per trajectory (accumulated)
    const double* dL;       // [n_rec][2N]
    double scale;           // 1 / n_total
    T t, U, h2, h1, h6, h3;
};

__device__ __forceinline__ uint32_t lo16(uint32_t w) { return w & 0xffffu; }
__device__ __forceinline__ uint32_t hi16(uint32_t w) { return w >> 16; }

// Neighbour field n of q0 (c0, c1, c2, r0, r1, r2).
__device__ __forceinline__ uint32_t fld(const uint4& q, int n) {
    const uint32_t w = n < 2 ? q.x : (n < 4 ? q.y : q.z);
    return (n & 1) ? hi16(w) : lo16(w);
}
template <typename T> __device__ __forceinline__ T sgn16(uint32_t f) {
    return (f & 0x8000u) ? (T)-1 : (T)1;
}

// col = sum_{k in nb(j)} X_ik and row = sum_{k in nb(i)} X_kj, each as
// (v0 + v1) + v2 -- the roundings of the forward kernels (a conjugate read
// changes only the sign of an imaginary part, which both forms apply exactly).
template <typename T, bool XF>
__device__ __forceinline__ void stencil(const cplx_t<T>* X, const uint4& q, cplx_t<T>& col,
                                        cplx_t<T>& row) {
    using C = cplx_t<T>;
    C v[6];
    uint32_t f[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        f[n] = fld(q, n);
        v[n] = X[XF ? f[n] : (f[n] & 0x7fffu)];
    }
    col.x = (v[0].x + v[1].x) + v[2].x;
    row.x = (v[3].x + v[4].x) + v[5].x;
    if constexpr (XF) {
        col.y = (v[0].y + v[1].y) + v[2].y;
        row.y = (v[3].y + v[4].y) + v[5].y;
    } else {
        col.y = fma_rn<T>(sgn16<T>(f[2]), v[2].y,
                          fma_rn<T>(sgn16<T>(f[1]), v[1].y, sgn16<T>(f[0]) * v[0].y));
        row.y = fma_rn<T>(sgn16<T>(f[5]), v[5].y,
                          fma_rn<T>(sgn16<T>(f[4]), v[4].y, sgn16<T>(f[3]) * v[3].y));
    }
}

template <typename T> __device__ __forceinline__ cplx_t<T> cfma(T c, cplx_t<T> k, cplx_t<T> y) {
    cplx_t<T> r;
    r.x = fma_rn<T>(c, k.x, y.x);
    r.y = fma_rn<T>(c, k.y, y.y);
    return r;
}

// Deterministic sum over the 64 lanes of a wave (fixed butterfly).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T, int NT, int U, bool XF>
__global__ __launch_bounds__(NT) void reverse_segment(RevArgs<T> A) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = A.N, E = A.E, CH = A.CH, XN = A.XN;
    const int tid = threadIdx.x;
    const int64_t m = blockIdx.x;
    C* const X0 = reinterpret_cast<C*>(smem);
    C* const X1 = X0 + XN;
    T* const Wf = reinterpret_cast<T*>(X1 + XN);  // [2][N][N]
    T* const Yd = Wf + 2 * N * N;                  // [4][2N]
    T* const Rp = Yd + 8 * N;                      // [2N][CH]
    double* const red = reinterpret_cast<double*>(
        smem + (((size_t)2 * XN * sizeof(C) + (size_t)(2 * N * N + 8 * N + 2 * N * CH) * sizeof(T) +
                 15) / 16 * 16));  // [NT / 64][2]

    C y[U], Y2[U], Y3[U], Y4[U], lam[U], Lam[U];
    // Descriptor pair of slot u: q0 = the six neighbour fields and
    // yi | yj << 16 (the entries of d_i, d_j in a Yd row: the other spin's
    // diagonal); q1 = own X entry | its transpose's << 16, own W entry | its
    // transpose's << 16, yown | diagonal flag << 16 (the element's own entry
    // in a Yd row), packed index e.
    //
    // fn(u, q0, q1) for every slot that holds an element.  With few slots
    // (DREG) the descriptors stay in registers (an empty asm statement that
    // claims to change them at every use keeps their decoded fields from being
    // hoisted out of the step loops, where they would stay live); with
    // more, the next slot's pair is read while this one is worked on and the
    // slots are scheduled one after the other (their loads hoisted together
    // would multiply the live registers).
    constexpr bool DREG = U <= 3;
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    uint4 d0[DREG ? U : 1], d1[DREG ? U : 1];
    if constexpr (DREG) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = tid + NT * u;
            d0[u] = p < E ? A.desc[2 * p] : z4;
            d1[u] = p < E ? A.desc[2 * p + 1] : z4;
        }
    }
    auto each = [&](auto fn) {
        if constexpr (DREG) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                __asm__ volatile("" : "+v"(d0[u].x), "+v"(d0[u].y), "+v"(d0[u].z), "+v"(d0[u].w));
                __asm__ volatile("" : "+v"(d1[u].x), "+v"(d1[u].y), "+v"(d1[u].z), "+v"(d1[u].w));
                if (tid + NT * u < E) fn(u, d0[u], d1[u]);
            }
        } else {
            uint4 na = tid < E ? A.desc[2 * tid] : z4, nb = tid < E ? A.desc[2 * tid + 1] : z4;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint4 a = na, b = nb;
                if (u + 1 < U) {
                    const int p1 = tid + NT * (u + 1);
                    na = p1 < E ? A.desc[2 * p1] : z4;
                    nb = p1 < E ? A.desc[2 * p1 + 1] : z4;
                }
                if (tid + NT * u < E) fn(u, a, b);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    auto is_diag = [](const uint4& b) { return (b.z >> 16) != 0u; };
    auto yown = [](const uint4& b) { return (int)lo16(b.z); };

    // ---- the carried cotangent
    C* const lamT = A.lamT + (size_t)m * E;
    each([&](int u, const uint4& a, const uint4& b) {
        if (A.first) {
            lam[u].x = 0;
            lam[u].y = 0;
            if (is_diag(b) && A.n_steps % A.record_every == 0)
                lam[u].x = lam[u].x +
                           (T)(A.scale * A.dL[(A.n_steps / A.record_every) * 2 * N + yown(b)]);
        } else {
            lam[u] = lamT[tid + NT * u];
        }
    });

    // writes value v of element u to X (and its conjugate to the transposed
    // entry of a full X) and, on the diagonal, its real part to Ydout
    auto put = [&](C* X, T* Ydout, const uint4& b, C v) {
        X[lo16(b.x)] = v;
        if constexpr (XF) {
            if (!is_diag(b)) X[hi16(b.x)] = conj(v);
        }
        if (is_diag(b)) Ydout[yown(b)] = v.x;
    };
    // W = Im(conj(av) Yv) of element u and -W at the transposed entry
    auto put_w = [&](const uint4& b, C av, C Yv) {
        const T w = av.x * Yv.y - av.y * Yv.x;
        Wf[lo16(b.y)] = w;
        if (!is_diag(b)) Wf[hi16(b.y)] = -w;
    };

    // ---- forward over the segment from its checkpoint
    C* const seg = A.seg + (size_t)m * A.Lmax * E;
    each([&](int u, const uint4& a, const uint4& b) {
        y[u] = A.ckpt[(int64_t)b.w * A.Mc + m];
        put(X0, Yd, b, y[u]);
    });
    if (tid == 0) {
        C z;
        z.x = 0;
        z.y = 0;
        X0[XN - 1] = z;
        X1[XN - 1] = z;
    }
    __syncthreads();

    // One stage of the forward map: k = f(Xin) with the diagonal of the
    // input at Ydin, own value own[u]; upd(u, q1, k).
    auto stage = [&](const C* Xin, const T* Ydin, const C* own, auto upd) {
        each([&](int u, const uint4& a, const uint4& b) {
            C col, row;
            stencil<T, XF>(Xin, a, col, row);
            const T av = A.U * (Ydin[lo16(a.w)] - Ydin[hi16(a.w)]);
            upd(u, b, rhs_element<T>(col, row, own[u], A.t, av));
        });
    };

    for (int64_t n = 1; n < A.L; ++n) {
        // store y_{n-1}
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (tid + NT * u < E) seg[(size_t)(n - 1) * E + tid + NT * u] = y[u];
        // acc in Lam, stage values in Y2
        stage(X0, Yd, y, [&](int u, const uint4& b, C k) {
            Lam[u] = k;
            Y2[u] = cfma<T>(A.h2, k, y[u]);
            put(X1, Yd + 2 * N, b, Y2[u]);
        });
        __syncthreads();
        stage(X1, Yd + 2 * N, Y2, [&](int u, const uint4& b, C k) {
            Lam[u] = cfma<T>((T)2, k, Lam[u]);
            Y2[u] = cfma<T>(A.h2, k, y[u]);
            put(X0, Yd + 4 * N, b, Y2[u]);
        });
        __syncthreads();
        stage(X0, Yd + 4 * N, Y2, [&](int u, const uint4& b, C k) {
            Lam[u] = cfma<T>((T)2, k, Lam[u]);
            Y2[u] = cfma<T>(A.h1, k, y[u]);
            put(X1, Yd + 6 * N, b, Y2[u]);
        });
        __syncthreads();
        stage(X1, Yd + 6 * N, Y2, [&](int u, const uint4& b, C k) {
            Lam[u] = cadd(Lam[u], k);
            y[u] = cfma<T>(A.h6, Lam[u], y[u]);
            put(X0, Yd, b, y[u]);
        });
        __syncthreads();
    }

    // ---- reverse
    double eU = 0.0, et = 0.0;
    // One transposed stage: a in Xa, stage input values Ys with diagonal at
    // Yds; mu accumulates into Lam and a_next = fma(beta, mu, alpha lam) goes
    // to Xn (with its W against Yn) unless this is the first stage.
    auto vjp = [&](const C* Xa, const T* Yds, const C* Ys, bool more, C* Xn, const C* Yn, T alpha,
                   T beta) {
        // partial row sums of W: row r = (s', i), sites [c KC, (c+1) KC) in
        // ascending order (the diagonal entry is zero), eight reads issued
        // before their sums
        const int KC = (N + CH - 1) / CH;
        for (int it = tid; it < 2 * N * CH; it += NT) {
            const int r = it / CH, c = it - r * CH;
            const T* Wr = Wf + r * N;
            const int k1 = min(N, c * KC + KC);
            T acc = 0;
            for (int k0 = c * KC; k0 < k1; k0 += 8) {
                T v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) v[q] = k0 + q < k1 ? Wr[k0 + q] : (T)0;
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (k0 + q < k1) acc = acc + v[q];
            }
            Rp[it] = acc;
        }
        __syncthreads();
        each([&](int u, const uint4& a, const uint4& b) {
            C col, row;
            stencil<T, XF>(Xa, a, col, row);
            const C own_a = Xa[lo16(b.x)];
            const C own_y = Ys[u];
            const T dd = Yds[lo16(a.w)] - Yds[hi16(a.w)];
            const T gx = col.x - row.x, gy = col.y - row.y;
            const T av = A.U * dd;
            // mu = -f^lin(a) = (gi, -gr) with f = (-gi, gr) as in rhs_element
            C mu;
            mu.x = fma_rn<T>(av, own_a.y, A.t * gy);
            mu.y = -fma_rn<T>(av, own_a.x, A.t * gx);
            const T im_gy = fma_rn<T>(-gy, own_y.x, gx * own_y.y);
            double w = 2.0;
            if (is_diag(b)) {
                // the row of the other spin block: the coupling term and its
                // share of dL/dU
                const T* rp = Rp + (size_t)lo16(a.w) * CH;
                T Rd = 0;
                for (int c = 0; c < CH; ++c) Rd = Rd + rp[c];
                mu.x = fma_rn<T>((T)(-2) * A.U, Rd, mu.x);
                eU = fma(-2.0 * (double)own_y.x, (double)Rd, eU);
                w = 1.0;
            }
            et = fma(-w, (double)im_gy, et);
            Lam[u] = cadd(Lam[u], mu);
            if (more) {
                C an;
                an.x = fma_rn<T>(beta, mu.x, alpha * lam[u].x);
                an.y = fma_rn<T>(beta, mu.y, alpha * lam[u].y);
                Xn[lo16(b.x)] = an;
                if constexpr (XF) {
                    if (!is_diag(b)) Xn[hi16(b.x)] = conj(an);
                }
                put_w(b, an, Yn[u]);
            }
        });
        __syncthreads();
    };

    for (int64_t n = A.L - 1; n >= 0; --n) {
        if (n < A.L - 1) {
            each([&](int u, const uint4& a, const uint4& b) {
                y[u] = seg[(size_t)n * E + tid + NT * u];
                put(X0, Yd, b, y[u]);
            });
            __syncthreads();
        }
        // stage inputs with the forward arithmetic
        stage(X0, Yd, y, [&](int u, const uint4& b, C k) {
            Y2[u] = cfma<T>(A.h2, k, y[u]);
            put(X1, Yd + 2 * N, b, Y2[u]);
        });
        __syncthreads();
        stage(X1, Yd + 2 * N, Y2, [&](int u, const uint4& b, C k) {
            Y3[u] = cfma<T>(A.h2, k, y[u]);
            put(X0, Yd + 4 * N, b, Y3[u]);
        });
        __syncthreads();
        stage(X0, Yd + 4 * N, Y3, [&](int u, const uint4& b, C k) {
            Y4[u] = cfma<T>(A.h1, k, y[u]);
            if (is_diag(b)) Yd[6 * N + yown(b)] = Y4[u].x;
            // a4 = h/6 lam (X1 was last read by the stage before the barrier)
            C a4;
            a4.x = A.h6 * lam[u].x;
            a4.y = A.h6 * lam[u].y;
            X1[lo16(b.x)] = a4;
            if constexpr (XF) {
                if (!is_diag(b)) X1[hi16(b.x)] = conj(a4);
            }
            put_w(b, a4, Y4[u]);
            Lam[u] = lam[u];
        });
        __syncthreads();
        vjp(X1, Yd + 6 * N, Y4, true, X0, Y3, A.h3, A.h1);
        vjp(X0, Yd + 4 * N, Y3, true, X1, Y2, A.h3, A.h2);
        vjp(X1, Yd + 2 * N, Y2, true, X0, y, A.h6, A.h2);
        vjp(X0, Yd, y, false, nullptr, nullptr, 0, 0);
        // lam <- Lam, seeded at the records
        const int64_t g = A.base + n;
        const bool rec = g % A.record_every == 0;
        each([&](int u, const uint4& a, const uint4& b) {
            lam[u] = Lam[u];
            if (rec && is_diag(b))
                lam[u].x = lam[u].x + (T)(A.scale * A.dL[(g / A.record_every) * 2 * N + yown(b)]);
        });
    }

    // ---- outputs
    each([&](int u, const uint4& a, const uint4& b) {
        if (A.last) {
            if (is_diag(b)) A.lam_out[(int64_t)b.w * A.Mc + m] = lam[u];
        } else {
            lamT[tid + NT * u] = lam[u];
        }
    });
    eU = wave_sum(eU);
    et = wave_sum(et);
    const int wave = tid / 64;
    if (tid % 64 == 0) {
        red[2 * wave] = eU;
        red[2 * wave + 1] = et;
    }
    __syncthreads();
    if (tid == 0) {
        double su = 0.0, st = 0.0;
        for (int w = 0; w < NT / 64; ++w) {
            su += red[2 * w];
            st += red[2 * w + 1];
        }
        A.partial[m] += su;
        A.partial[A.Mc + m] += st;
    }
}

struct RevConfig {
    bool f64;
    int NT, U;
    bool full;
    const void* fn;
};

template <typename T, int NT, int U, bool XF> constexpr RevConfig rev_cfg() {
    return RevConfig{sizeof(T) == 8, NT, U, XF, (const void*)&reverse_segment<T, NT, U, XF>};
}

// In order of preference: the first whose slots hold both spin blocks and
// whose LDS fits (the full X first).
const RevConfig kRevConfigs[] = {
    rev_cfg<float, 256, 1, true>(),   rev_cfg<float, 256, 4, true>(),
    rev_cfg<float, 1024, 3, true>(),  rev_cfg<float, 1024, 4, true>(),
    rev_cfg<float, 1024, 5, false>(), rev_cfg<double, 256, 1, true>(),
    rev_cfg<double, 256, 4, true>(),  rev_cfg<double, 768, 4, false>(),
};

constexpr size_t kRevMaxLds = 160 * 1024;

int rev_chunks(int N, int NT) {
    int ch = 1;
    while (ch < 8 && 2 * N * ch * 2 <= NT) ch *= 2;
    return ch;
}

int rev_xn(int N, bool full) {
    return full ? 2 * N * N + 1 : (int)(2 * packed_count(N)) + 1;
}

size_t rev_lds(int N, int NT, int CH, bool f64, bool full) {
    const size_t cb = f64 ? 16 : 8, tb = f64 ? 8 : 4;
    const size_t a = (size_t)2 * rev_xn(N, full) * cb +
                     (size_t)(2 * N * N + 8 * N + 2 * N * CH) * tb;
    return (a + 15) / 16 * 16 + (size_t)(NT / 64) * 2 * sizeof(double);
}

}  // namespace

int reverse_resident_config(int N, ftwa_dtype dtype) {
    const int E = (int)(2 * packed_count(N));
    const int n = (int)(sizeof(kRevConfigs) / sizeof(kRevConfigs[0]));
    for (int k = 0; k < n; ++k) {
        const RevConfig& c = kRevConfigs[k];
        if (c.f64 != (dtype == FTWA_F64)) continue;
        if (c.NT * c.U < E) continue;
        if (c.full ? N > kReverseFullMaxSites : N > kReverseMaxSites) continue;
        if (rev_lds(N, c.NT, rev_chunks(N, c.NT), c.f64, c.full) > kRevMaxLds) continue;
        return k;
    }
    return -1;
}

bool reverse_resident_full(int config) { return kRevConfigs[config].full; }

template <typename T>
ftwa_status reverse_resident_segment(int config, const ReverseSegment& s, hipStream_t stream) {
    const RevConfig& c = kRevConfigs[config];
    RevArgs<T> A;
    A.N = s.N;
    A.E = (int)(2 * packed_count(s.N));
    A.XN = rev_xn(s.N, c.full);
    A.CH = rev_chunks(s.N, c.NT);
    A.record_every = s.record_every;
    A.Mc = s.Mc;
    A.L = s.L;
    A.Lmax = s.Lmax;
    A.base = s.base;
    A.n_steps = s.n_steps;
    A.first = s.first;
    A.last = s.last;
    A.desc = c.full ? s.desc_full : s.desc;
    if (!A.desc) return fail(FTWA_EINVAL, "reverse_resident: no descriptor table");
    A.ckpt = static_cast<const cplx_t<T>*>(s.ckpt);
    A.seg = static_cast<cplx_t<T>*>(s.seg);
    A.lamT = static_cast<cplx_t<T>*>(s.lamT);
    A.lam_out = static_cast<cplx_t<T>*>(s.lam_out);
    A.partial = s.partial;
    A.dL = s.dL;
    A.scale = s.scale;
    A.t = (T)s.t;
    A.U = (T)s.U;
    A.h2 = (T)(0.5 * s.dt);
    A.h1 = (T)s.dt;
    A.h6 = (T)(s.dt / 6.0);
    A.h3 = (T)(s.dt / 3.0);
    const size_t lds = rev_lds(s.N, c.NT, A.CH, c.f64, c.full);
    FTWA_HIP_TRY(hipFuncSetAttribute(c.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kRevMaxLds));
    void* args[] = {&A};
    FTWA_HIP_TRY(hipLaunchKernel(c.fn, dim3((unsigned)s.Mc), dim3((unsigned)c.NT), args, lds,
                                 stream));
    return FTWA_OK;
}

ftwa_status reverse_resident(int config, const ReverseSegment& s, hipStream_t stream) {
    if (config < 0 || config >= (int)(sizeof(kRevConfigs) / sizeof(kRevConfigs[0])))
        return fail(FTWA_EINVAL, "reverse_resident: no such configuration");
    if (kRevConfigs[config].f64) return reverse_resident_segment<double>(config, s, stream);
    return reverse_resident_segment<float>(config, s, stream);
}

}  // namespace ftwa

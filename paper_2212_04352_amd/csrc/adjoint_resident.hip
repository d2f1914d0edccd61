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
//   with (df(Y)^T a)_s = -f_s^lin(a_s; D from Y) plus, on the diagonal (k,k),
//   -2U sum_{j != k} Im(conj(a_sbar,kj) Y_sbar,kj), and the parameter sums
//   <a, df/dU> = -sum (d_i - d_j) Im(conj(a_ij) Y_ij),
//   <a, df/dt> = -sum Im(conj(col(a) - row(a))_ij Y_ij), off-diagonal
//   elements counted twice.
// Only the diagonal coupling sum is taken in another order than the stream
// sweep (CH partial sums over consecutive sites, then the partials in
// order), so the gradients agree to rounding.  Every order is fixed:
// repeated runs give identical bits.
//
// LDS (one trajectory): two copies of the stencil input X[E + 1] (E = 2P
// elements of both spins, then a zero slot for missing neighbours), the
// products W[E] = Im(conj(a) Y) of the diagonal coupling, the diagonals of
// the four stage inputs Yd[4][2N], the partial row sums Rp[2N][CH] and the
// per-wave parameter sums.
#include <algorithm>

#include "device_common.h"
#include "ftwa_internal.h"

namespace ftwa {

namespace {

template <typename T> struct RevArgs {
    int N;
    int E;                  // 2P
    int CH;                 // partial sums per row of the diagonal coupling
    int record_every;
    int64_t Mc;             // trajectories of the chunk (one workgroup each)
    int64_t L;              // steps of this segment
    int64_t Lmax;           // segment scratch per trajectory, in states
    int64_t base;           // global index of the segment's first step
    int64_t n_steps;
    bool first;             // the segment that ends at n_steps (lam starts at zero)
    bool last;              // the segment that starts at step 0
    const uint4* desc;      // [E] stencil descriptors
    const cplx_t<T>* ckpt;  // y_base, trajectory-innermost [E][Mc]
    cplx_t<T>* seg;         // [Mc][Lmax][E] states of the segment
    cplx_t<T>* lamT;        // [Mc][E] cotangent carried between segments
    cplx_t<T>* lam_out;     // [E][Mc] (diagonal entries written by the last segment)
    double* partial;        // [2][Mc] dL/dU, dL/dt sums per trajectory (accumulated)
    const double* dL;       // [n_rec][2N]
    double scale;           // 1 / n_total
    T t, U, h2, h1, h6, h3;
};

// Stencil descriptor of element e = s P + p(i, j) (see reverse_descriptors):
//   x = c0 | c1 << 16, y = c2 | r0 << 16, z = r1 | r2 << 16: entries of X
//   (15 bits; bit 15: read the conjugate; a missing neighbour reads the zero
//   slot E), columns c_n = (i, k) for k in nb(j) ascending, rows r_n = (k, j)
//   for k in nb(i) ascending;
//   w = i | j << 8 | s << 16.
__device__ __forceinline__ uint32_t fld(const uint4& d, int n) {
    const uint32_t w = n < 2 ? d.x : (n < 4 ? d.y : d.z);
    return (n & 1) ? (w >> 16) : (w & 0xffffu);
}
template <typename T> __device__ __forceinline__ T sgn16(uint32_t f) {
    return (f & 0x8000u) ? (T)-1 : (T)1;
}

// col = sum_{k in nb(j)} X_ik and row = sum_{k in nb(i)} X_kj, each as
// (v0 + v1) + v2 with the imaginary parts as fma(sign, v.y, .) -- the same
// roundings as the forward kernels.
template <typename T>
__device__ __forceinline__ void stencil(const cplx_t<T>* X, const uint4& d, cplx_t<T>& col,
                                        cplx_t<T>& row) {
    using C = cplx_t<T>;
    C v[6];
    uint32_t f[6];
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        f[n] = fld(d, n);
        v[n] = X[f[n] & 0x7fffu];
    }
    col.x = (v[0].x + v[1].x) + v[2].x;
    col.y = fma_rn<T>(sgn16<T>(f[2]), v[2].y,
                      fma_rn<T>(sgn16<T>(f[1]), v[1].y, sgn16<T>(f[0]) * v[0].y));
    row.x = (v[3].x + v[4].x) + v[5].x;
    row.y = fma_rn<T>(sgn16<T>(f[5]), v[5].y,
                      fma_rn<T>(sgn16<T>(f[4]), v[4].y, sgn16<T>(f[3]) * v[3].y));
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

template <typename T, int NT, int U>
__global__ __launch_bounds__(NT) void reverse_segment(RevArgs<T> A) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = A.N, E = A.E, CH = A.CH;
    const int tid = threadIdx.x;
    const int64_t m = blockIdx.x;
    C* const X0 = reinterpret_cast<C*>(smem);
    C* const X1 = X0 + (E + 1);
    T* const W = reinterpret_cast<T*>(X1 + (E + 1));
    T* const Yd = W + E;                 // [4][2N]
    T* const Rp = Yd + 8 * N;            // [2N][CH]
    double* const red = reinterpret_cast<double*>(
        smem + (((size_t)(2 * (E + 1)) * sizeof(C) + (size_t)(E + 8 * N + 2 * N * CH) * sizeof(T) +
                 15) / 16 * 16));  // [NT / 64][2]

    C y[U], Y2[U], Y3[U], Y4[U], lam[U], Lam[U];
    auto site_i = [](const uint4& q) { return (int)(q.w & 0xffu); };
    auto site_j = [](const uint4& q) { return (int)((q.w >> 8) & 0xffu); };
    auto spin = [](const uint4& q) { return (int)((q.w >> 16) & 1u); };
    // fn(u, descriptor) for every slot that holds an element.  With few
    // slots (DREG) the descriptors stay in registers and the compiler may
    // interleave the slots; with more, the next slot's descriptor is read
    // while this one is worked on and the slots are scheduled one after the
    // other (their loads hoisted together would multiply the live registers).
    constexpr bool DREG = U <= 3;
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    uint4 dreg[DREG ? U : 1];
    if constexpr (DREG) {
#pragma unroll
        for (int u = 0; u < U; ++u) dreg[u] = tid + NT * u < E ? A.desc[tid + NT * u] : z4;
    }
    auto each = [&](auto fn) {
        if constexpr (DREG) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // an opaque copy: the decoded fields are not hoisted out of
                // the step loops (they would stay live in registers)
                uint4 q = dreg[u];
                __asm__ volatile("" : "+v"(q.x), "+v"(q.y), "+v"(q.z), "+v"(q.w));
                if (tid + NT * u < E) fn(u, q);
            }
        } else {
            uint4 dn = tid < E ? A.desc[tid] : z4;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint4 dc = dn;
                if (u + 1 < U) {
                    const int e1 = tid + NT * (u + 1);
                    dn = e1 < E ? A.desc[e1] : z4;
                }
                if (tid + NT * u < E) fn(u, dc);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };
    auto is_diag = [&](const uint4& q) { return site_i(q) == site_j(q); };

    // ---- the carried cotangent
    C* const lamT = A.lamT + (size_t)m * E;
    each([&](int u, const uint4& q) {
        if (A.first) {
            lam[u].x = 0;
            lam[u].y = 0;
            if (is_diag(q) && A.n_steps % A.record_every == 0)
                lam[u].x = lam[u].x + (T)(A.scale * A.dL[(A.n_steps / A.record_every) * 2 * N +
                                                         spin(q) * N + site_i(q)]);
        } else {
            lam[u] = lamT[tid + NT * u];
        }
    });

    // writes value v of element u to X and, on the diagonal, to Ydout
    auto put = [&](C* X, T* Ydout, int u, const uint4& q, C v) {
        X[tid + NT * u] = v;
        if (is_diag(q)) Ydout[spin(q) * N + site_i(q)] = v.x;
    };

    // ---- forward over the segment from its checkpoint
    C* const seg = A.seg + (size_t)m * A.Lmax * E;
    each([&](int u, const uint4& q) {
        y[u] = A.ckpt[(int64_t)(tid + NT * u) * A.Mc + m];
        put(X0, Yd, u, q, y[u]);
    });
    if (tid == 0) {
        C z;
        z.x = 0;
        z.y = 0;
        X0[E] = z;
        X1[E] = z;
    }
    __syncthreads();

    // One stage of the forward map: k = f(Xin) with the diagonal of the
    // input at Ydin, own value own[u]; upd(u, descriptor, k).
    auto stage = [&](const C* Xin, const T* Ydin, const C* own, auto upd) {
        each([&](int u, const uint4& q) {
            C col, row;
            stencil<T>(Xin, q, col, row);
            const int so = (1 - spin(q)) * N;
            const T a = A.U * (Ydin[so + site_i(q)] - Ydin[so + site_j(q)]);
            upd(u, q, rhs_element<T>(col, row, own[u], A.t, a));
        });
    };

    for (int64_t n = 1; n < A.L; ++n) {
        // store y_{n-1}
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (tid + NT * u < E) seg[(size_t)(n - 1) * E + tid + NT * u] = y[u];
        // acc in Lam, stage values in Y2
        stage(X0, Yd, y, [&](int u, const uint4& q, C k) {
            Lam[u] = k;
            Y2[u] = cfma<T>(A.h2, k, y[u]);
            put(X1, Yd + 2 * N, u, q, Y2[u]);
        });
        __syncthreads();
        stage(X1, Yd + 2 * N, Y2, [&](int u, const uint4& q, C k) {
            Lam[u] = cfma<T>((T)2, k, Lam[u]);
            Y2[u] = cfma<T>(A.h2, k, y[u]);
            put(X0, Yd + 4 * N, u, q, Y2[u]);
        });
        __syncthreads();
        stage(X0, Yd + 4 * N, Y2, [&](int u, const uint4& q, C k) {
            Lam[u] = cfma<T>((T)2, k, Lam[u]);
            Y2[u] = cfma<T>(A.h1, k, y[u]);
            put(X1, Yd + 6 * N, u, q, Y2[u]);
        });
        __syncthreads();
        stage(X1, Yd + 6 * N, Y2, [&](int u, const uint4& q, C k) {
            Lam[u] = cadd(Lam[u], k);
            y[u] = cfma<T>(A.h6, Lam[u], y[u]);
            put(X0, Yd, u, q, y[u]);
        });
        __syncthreads();
    }

    // ---- reverse
    double eU = 0.0, et = 0.0;
    // the product of the diagonal coupling for cotangent av and stage value Yv
    auto put_w = [&](int u, C av, C Yv) { W[tid + NT * u] = av.x * Yv.y - av.y * Yv.x; };
    // One transposed stage: a in Xa, stage input values Ys with diagonal at
    // Yds; mu accumulates into Lam and a_next = fma(beta, mu, alpha lam) goes
    // to Xn (with its W against Yn) unless this is the first stage.
    auto vjp = [&](const C* Xa, const T* Yds, const C* Ys, bool more, C* Xn, const C* Yn, T alpha,
                   T beta) {
        // partial row sums of W: row (s', i), sites [c KC, (c+1) KC) in
        // ascending order, eight reads issued before their sums
        const int KC = (N + CH - 1) / CH;
        for (int it = tid; it < 2 * N * CH; it += NT) {
            const int r = it / CH, c = it - r * CH;
            const int sp = r >= N ? 1 : 0, i = r - sp * N;
            const T* Ws = W + (size_t)sp * (E / 2);
            const int k1 = min(N, c * KC + KC);
            const int ri = i * N - i * (i - 1) / 2 - i;  // entry of (i, k) is ri + k for k >= i
            T acc = 0;
            for (int k0 = c * KC; k0 < k1; k0 += 8) {
                T v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int k = k0 + q;
                    // (k, i) is at k N - k (k - 1) / 2 + (i - k) for k < i
                    const int at = k >= i ? ri + k : k * N - k * (k - 1) / 2 + (i - k);
                    v[q] = k < k1 && k != i ? Ws[at] : (T)0;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int k = k0 + q;
                    if (k < k1 && k != i) acc = k > i ? acc + v[q] : acc - v[q];
                }
            }
            Rp[it] = acc;
        }
        __syncthreads();
        each([&](int u, const uint4& q) {
            const int e = tid + NT * u;
            const int i = site_i(q), j = site_j(q), so = (1 - spin(q)) * N;
            C col, row;
            stencil<T>(Xa, q, col, row);
            const C own_a = Xa[e];
            const C own_y = Ys[u];
            const T dd = Yds[so + i] - Yds[so + j];
            const C fl = rhs_element<T>(col, row, own_a, A.t, A.U * dd);
            C mu;
            mu.x = -fl.x;
            mu.y = -fl.y;
            double w = 2.0;
            if (i == j) {
                const T* rp = Rp + (size_t)(so + i) * CH;
                T Rd = 0;
                for (int c = 0; c < CH; ++c) Rd = Rd + rp[c];
                mu.x = fma_rn<T>((T)(-2) * A.U, Rd, mu.x);
                w = 1.0;
            }
            const double im_ay = (double)own_a.x * own_y.y - (double)own_a.y * own_y.x;
            const double gx = (double)col.x - row.x, gy = (double)col.y - row.y;
            const double im_gy = gx * own_y.y - gy * own_y.x;
            eU -= w * (double)dd * im_ay;
            et -= w * im_gy;
            Lam[u] = cadd(Lam[u], mu);
            if (more) {
                C an;
                an.x = fma_rn<T>(beta, mu.x, alpha * lam[u].x);
                an.y = fma_rn<T>(beta, mu.y, alpha * lam[u].y);
                Xn[e] = an;
                put_w(u, an, Yn[u]);
            }
        });
        __syncthreads();
    };

    for (int64_t n = A.L - 1; n >= 0; --n) {
        if (n < A.L - 1) {
            each([&](int u, const uint4& q) {
                y[u] = seg[(size_t)n * E + tid + NT * u];
                put(X0, Yd, u, q, y[u]);
            });
            __syncthreads();
        }
        // stage inputs with the forward arithmetic
        stage(X0, Yd, y, [&](int u, const uint4& q, C k) {
            Y2[u] = cfma<T>(A.h2, k, y[u]);
            put(X1, Yd + 2 * N, u, q, Y2[u]);
        });
        __syncthreads();
        stage(X1, Yd + 2 * N, Y2, [&](int u, const uint4& q, C k) {
            Y3[u] = cfma<T>(A.h2, k, y[u]);
            put(X0, Yd + 4 * N, u, q, Y3[u]);
        });
        __syncthreads();
        stage(X0, Yd + 4 * N, Y3, [&](int u, const uint4& q, C k) {
            Y4[u] = cfma<T>(A.h1, k, y[u]);
            if (is_diag(q)) Yd[6 * N + spin(q) * N + site_i(q)] = Y4[u].x;
            // a4 = h/6 lam (X1 was last read by the stage before the barrier)
            C a4;
            a4.x = A.h6 * lam[u].x;
            a4.y = A.h6 * lam[u].y;
            X1[tid + NT * u] = a4;
            put_w(u, a4, Y4[u]);
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
        each([&](int u, const uint4& q) {
            lam[u] = Lam[u];
            if (rec && is_diag(q))
                lam[u].x = lam[u].x + (T)(A.scale * A.dL[(g / A.record_every) * 2 * N +
                                                         spin(q) * N + site_i(q)]);
        });
    }

    // ---- outputs
    each([&](int u, const uint4& q) {
        const int e = tid + NT * u;
        if (A.last) {
            if (is_diag(q)) A.lam_out[(int64_t)e * A.Mc + m] = lam[u];
        } else {
            lamT[e] = lam[u];
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
    const void* fn;
};

template <typename T, int NT, int U> constexpr RevConfig rev_cfg() {
    return RevConfig{sizeof(T) == 8, NT, U, (const void*)&reverse_segment<T, NT, U>};
}

// In order of preference: the first whose slots hold both spin blocks and
// whose LDS fits.
const RevConfig kRevConfigs[] = {
    rev_cfg<float, 256, 1>(),  rev_cfg<float, 256, 4>(),   rev_cfg<float, 1024, 3>(),
    rev_cfg<float, 1024, 5>(), rev_cfg<double, 256, 1>(),  rev_cfg<double, 256, 4>(),
    rev_cfg<double, 768, 4>(),  rev_cfg<float, 512, 6>(),  rev_cfg<float, 768, 4>(),
};

constexpr size_t kRevMaxLds = 160 * 1024;

int rev_chunks(int N, int NT) {
    int ch = 1;
    while (ch < 8 && 2 * N * ch * 2 <= NT) ch *= 2;
    return ch;
}

size_t rev_lds(int N, int E, int NT, int CH, bool f64) {
    const size_t cb = f64 ? 16 : 8, tb = f64 ? 8 : 4;
    const size_t a = (size_t)2 * (E + 1) * cb + (size_t)(E + 8 * N + 2 * N * CH) * tb;
    return (a + 15) / 16 * 16 + (size_t)(NT / 64) * 2 * sizeof(double);
}

}  // namespace

int reverse_resident_config(int N, ftwa_dtype dtype) {
    const int E = (int)(2 * packed_count(N));
    if (E + 1 > 0x7fff) return -1;
    const int n = (int)(sizeof(kRevConfigs) / sizeof(kRevConfigs[0]));
    for (int k = 0; k < n; ++k) {
        const RevConfig& c = kRevConfigs[k];
        if (c.f64 != (dtype == FTWA_F64)) continue;
        if (c.NT * c.U < E) continue;
        if (rev_lds(N, E, c.NT, rev_chunks(N, c.NT), c.f64) > kRevMaxLds) continue;
        return k;
    }
    return -1;
}

template <typename T>
ftwa_status reverse_resident_segment(int config, const ReverseSegment& s, hipStream_t stream) {
    const RevConfig& c = kRevConfigs[config];
    RevArgs<T> A;
    A.N = s.N;
    A.E = (int)(2 * packed_count(s.N));
    A.CH = rev_chunks(s.N, c.NT);
    A.record_every = s.record_every;
    A.Mc = s.Mc;
    A.L = s.L;
    A.Lmax = s.Lmax;
    A.base = s.base;
    A.n_steps = s.n_steps;
    A.first = s.first;
    A.last = s.last;
    A.desc = s.desc;
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
    const size_t lds = rev_lds(s.N, A.E, c.NT, A.CH, c.f64);
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

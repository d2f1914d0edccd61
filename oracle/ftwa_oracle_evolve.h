/*
 * ftwa_oracle_evolve.h -- body of the oracle's equation of motion and
 * Runge-Kutta loop, included twice by ftwa_oracle.c (ORC_REAL = double, then
 * float).  Test infrastructure only; see ftwa_oracle.c.
 *
 * A trajectory is rho[spin][i][j] (full N x N complex, interleaved re/im).
 */
#define ORC_CAT2(a, b) a##b
#define ORC_CAT(a, b) ORC_CAT2(a, b)
#define ORC_NAME(base) ORC_CAT(base, ORC_SUFFIX)

/* x <- w x for a complex hop ratio w = (w_re, w_im): re = fma(w_re, x_re,
 * -(w_im x_im)), im = fma(w_re, x_im, w_im x_re). */
static void ORC_NAME(cmul_w)(ORC_REAL w_re, ORC_REAL w_im, ORC_REAL* x_re, ORC_REAL* x_im)
{
    const ORC_REAL re = ORC_FMA(w_re, *x_re, -(w_im * *x_im));
    const ORC_REAL im = ORC_FMA(w_re, *x_im, w_im * *x_re);
    *x_re = re;
    *x_im = im;
}

/*
 * Right-hand side of the fTWA equation of motion, Sec. III, Eq. (6), with
 * j_ij = t on bonds and u_ij = U delta_ij (Sec. II):
 *
 *   d rho_ij,s / dt = i [ t ( sum_{k in nb(j)} rho_ik,s - sum_{k in nb(i)} rho_kj,s )
 *                         + U ( rho_ii,sbar - rho_jj,sbar ) rho_ij,s ]
 *
 * (the 1/2 of (rho_kk + 1/2) cancels between the two u terms).  An external
 * on-site potential V_i (both spins) enters Eq. (6) like the U term, as the
 * explicit term + (V_i - V_j) rho_ij inside the bracket (Sec. III notes that
 * time dependence of such a potential appears as explicit terms of Eq. (6));
 * here V_i = A v_i with `vsite` = v (NULL: no potential) and A the envelope
 * at the stage time.  A general density-density interaction u_ij (`umat`,
 * [N][N] symmetric, NULL: on-site U) gives Eq. (6)'s own form: the factor of
 * rho_ij is D_i - D_j with D_i = sum_k u_ki (rho_kk,sbar + 1/2) (which is
 * U (d_i - d_j) for u = U delta up to rounding).  Evaluation order: each
 * neighbour sum starts from the first (smallest) neighbour and adds the
 * others in ascending order; g = t*(col - row); a = U*(d_i - d_j), or with
 * umat a = D_i - D_j where D_i = fma(u_ki, d_k + 1/2, D_i) over ascending k
 * from 0; then (potential) a = a + A*(v_i - v_j); a is applied with one fma
 * per component; f = i*g.
 *
 * Complex (Peierls) hopping, `hop` non-NULL ([N][3] complex ratios
 * w_ik = j_ik / t, slot n of site i for its neighbour k = nbr[i][n]): the two
 * hopping sums of Eq. (6) are taken literally, col = sum_{k in nb(j)} j_jk
 * rho_ik / t and row = sum_{k in nb(i)} j_ki rho_kj / t, j_ki read from k's
 * own row (the entry of k for its neighbour i), each product by cmul_w before
 * it enters the ascending sum.
 */
void ORC_NAME(oracle_rhs_hop)(int N, const int32_t* nbr, const uint8_t* deg,
                              ORC_REAL t, ORC_REAL U, const ORC_REAL* umat,
                              const ORC_REAL* vsite, ORC_REAL A, const ORC_REAL* hop,
                              const ORC_REAL* rho, ORC_REAL* f)
{
    const size_t NN2 = (size_t)N * N * 2;
    ORC_REAL* Dall = NULL;  /* [2][N]: D of each spin block (from the other's diagonal) */
    if (umat) {
        Dall = (ORC_REAL*)malloc(sizeof(ORC_REAL) * 2 * (size_t)N);
        if (!Dall) return;
        for (int s = 0; s < 2; ++s) {
            const ORC_REAL* Rbar = rho + (1 - s) * NN2;
            for (int i = 0; i < N; ++i) {
                ORC_REAL D = 0;
                for (int k = 0; k < N; ++k)
                    D = ORC_FMA(umat[k * N + i], Rbar[2 * (k * N + k)] + (ORC_REAL)0.5, D);
                Dall[s * N + i] = D;
            }
        }
    }
    for (int s = 0; s < 2; ++s) {
        const ORC_REAL* R = rho + s * NN2;
        const ORC_REAL* Rbar = rho + (1 - s) * NN2;
        ORC_REAL* F = f + s * NN2;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                ORC_REAL col_re = 0, col_im = 0, row_re = 0, row_im = 0;
                for (int n = 0; n < deg[j]; ++n) {
                    int k = nbr[j * ORC_MAXDEG + n];
                    ORC_REAL x_re = R[2 * (i * N + k)], x_im = R[2 * (i * N + k) + 1];
                    if (hop) {
                        /* j_jk / t = hop[j][n] (k = nbr[j][n]) times rho_ik */
                        const ORC_REAL* w = hop + 2 * (j * ORC_MAXDEG + n);
                        ORC_NAME(cmul_w)(w[0], w[1], &x_re, &x_im);
                    }
                    if (n == 0) {
                        col_re = x_re;
                        col_im = x_im;
                    } else {
                        col_re = col_re + x_re;
                        col_im = col_im + x_im;
                    }
                }
                for (int n = 0; n < deg[i]; ++n) {
                    int k = nbr[i * ORC_MAXDEG + n];
                    ORC_REAL x_re = R[2 * (k * N + j)], x_im = R[2 * (k * N + j) + 1];
                    if (hop) {
                        /* j_ki / t: the entry of k's row for its neighbour i */
                        int nk = 0;
                        while (nbr[k * ORC_MAXDEG + nk] != i) ++nk;
                        const ORC_REAL* w = hop + 2 * (k * ORC_MAXDEG + nk);
                        ORC_NAME(cmul_w)(w[0], w[1], &x_re, &x_im);
                    }
                    if (n == 0) {
                        row_re = x_re;
                        row_im = x_im;
                    } else {
                        row_re = row_re + x_re;
                        row_im = row_im + x_im;
                    }
                }
                ORC_REAL g_re = t * (col_re - row_re);
                ORC_REAL g_im = t * (col_im - row_im);
                ORC_REAL a = umat ? Dall[s * N + i] - Dall[s * N + j]
                                  : U * (Rbar[2 * (i * N + i)] - Rbar[2 * (j * N + j)]);
                if (vsite) a = a + A * (vsite[i] - vsite[j]);
                g_re = ORC_FMA(a, R[2 * (i * N + j)], g_re);
                g_im = ORC_FMA(a, R[2 * (i * N + j) + 1], g_im);
                F[2 * (i * N + j)] = -g_im; /* f = i * g */
                F[2 * (i * N + j) + 1] = g_re;
            }
    }
    free(Dall);
}

void ORC_NAME(oracle_rhs_gen)(int N, const int32_t* nbr, const uint8_t* deg,
                              ORC_REAL t, ORC_REAL U, const ORC_REAL* umat,
                              const ORC_REAL* vsite, ORC_REAL A,
                              const ORC_REAL* rho, ORC_REAL* f)
{
    ORC_NAME(oracle_rhs_hop)(N, nbr, deg, t, U, umat, vsite, A, NULL, rho, f);
}

void ORC_NAME(oracle_rhs_pot)(int N, const int32_t* nbr, const uint8_t* deg,
                              ORC_REAL t, ORC_REAL U, const ORC_REAL* vsite, ORC_REAL A,
                              const ORC_REAL* rho, ORC_REAL* f)
{
    ORC_NAME(oracle_rhs_gen)(N, nbr, deg, t, U, NULL, vsite, A, rho, f);
}

void ORC_NAME(oracle_rhs)(int N, const int32_t* nbr, const uint8_t* deg,
                          ORC_REAL t, ORC_REAL U, const ORC_REAL* rho, ORC_REAL* f)
{
    ORC_NAME(oracle_rhs_pot)(N, nbr, deg, t, U, NULL, (ORC_REAL)0, rho, f);
}

/*
 * Per-trajectory quantities conserved by the exact flow (used as checks):
 *   inv[0], inv[1]: trace of rho_up, rho_down;
 *   inv[2]: Weyl Hamiltonian, Appendix A.3, Eq. (A10):
 *           H_W = - sum_{ij s} j_ij rho_ij,s + U sum_i (rho_ii,up + 1/2)(rho_ii,dn + 1/2);
 *   inv[3], inv[4]: squared Frobenius norm of rho_up, rho_down.
 * Accumulated in FP64 in plain row-major order.
 */
static void ORC_NAME(invariants)(int N, const int32_t* nbr, const uint8_t* deg,
                                 double t, double U, const ORC_REAL* rho, double* inv)
{
    const size_t NN2 = (size_t)N * N * 2;
    double hop = 0.0, inter = 0.0;
    for (int s = 0; s < 2; ++s) {
        const ORC_REAL* R = rho + s * NN2;
        double tr = 0.0, fro = 0.0;
        for (int i = 0; i < N; ++i) {
            tr += (double)R[2 * (i * N + i)];
            for (int j = 0; j < N; ++j) {
                double re = (double)R[2 * (i * N + j)], im = (double)R[2 * (i * N + j) + 1];
                fro += re * re + im * im;
            }
            for (int n = 0; n < deg[i]; ++n) {
                int k = nbr[i * ORC_MAXDEG + n];
                hop += (double)R[2 * (i * N + k)];
            }
        }
        inv[s] = tr;
        inv[3 + s] = fro;
    }
    for (int i = 0; i < N; ++i)
        inter += ((double)rho[2 * (i * N + i)] + 0.5) * ((double)rho[NN2 + 2 * (i * N + i)] + 0.5);
    inv[2] = -t * hop + U * inter;
}

/*
 * Classical fourth-order Runge-Kutta for every trajectory (the paper does not
 * name its integrator).  With h = dt:
 *   k1 = f(y);  Y2 = y + (h/2) k1;  k2 = f(Y2);  Y3 = y + (h/2) k2;
 *   k3 = f(Y3); Y4 = y + h k3;      k4 = f(Y4);
 *   y <- y + (h/6) (k1 + 2 k2 + 2 k3 + k4).
 * Evaluation order: Y = fma(c, k, y); acc = k1; acc = fma(2, k2, acc);
 * acc = fma(2, k3, acc); acc = acc + k4; y = fma(h/6, acc, y).
 * The coefficients h/2, h, h/6 are formed in FP64 and rounded once to the
 * working precision.
 *
 * rho: [M][2][N][N] complex FP64 in/out (rounded to the working precision on
 * entry).  Records are taken at steps 0, record_every, 2 record_every, ...:
 *   X[r][m][s*N + i] = rho_ii,s (FP64), inv[r][m][0..4] (see invariants).
 * vsite (NULL or [N]) and env ([2 n_steps + 1]): the on-site potential
 * V_i(tau) = A(tau) v_i; step n (from t_n = n h) takes A = env[2n] in stage 1,
 * env[2n+1] (t_n + h/2) in stages 2 and 3, env[2n+2] (t_n + h) in stage 4;
 * v and A rounded once to the working precision.  umat (NULL or [N][N]): the
 * general interaction u_ij (U unused; rounded once); inv is then not
 * computed (its H_W holds the on-site form).  hopw (NULL or
 * [2 n_steps + 1][N][3] complex): hop ratios w_ik(tau) = j_ik(tau) / t at the
 * same half steps as env (no inv either); rounded once.
 */
int ORC_NAME(oracle_evolve_hop)(int N, const int32_t* nbr, const uint8_t* deg,
                                double t, double U, const double* umat, const double* vsite,
                                const double* env, const double* hopw, double dt,
                                int64_t n_steps, int record_every, int64_t M, double* rho_io,
                                double* X, double* inv)
{
    if (N <= 0 || M < 0 || n_steps < 0 || record_every <= 0) return -1;
    const size_t E = (size_t)2 * N * N * 2; /* reals per trajectory */
    const int64_t n_rec = n_steps / record_every + 1;
    const int D = 2 * N;
    const ORC_REAL tw = (ORC_REAL)t, Uw = (ORC_REAL)U;
    const ORC_REAL c_half = (ORC_REAL)(0.5 * dt), c_full = (ORC_REAL)dt;
    const ORC_REAL c_sixth = (ORC_REAL)(dt / 6.0), two = (ORC_REAL)2;
    ORC_REAL* vw = NULL;
    if (vsite) {
        if (!env) return -1;
        vw = (ORC_REAL*)malloc(sizeof(ORC_REAL) * (size_t)N);
        if (!vw) return -2;
        for (int i = 0; i < N; ++i) vw[i] = (ORC_REAL)vsite[i];
    }
    ORC_REAL* uw = NULL;
    if (umat) {
        if (inv) { free(vw); return -1; }
        uw = (ORC_REAL*)malloc(sizeof(ORC_REAL) * (size_t)N * N);
        if (!uw) { free(vw); return -2; }
        for (size_t q = 0; q < (size_t)N * N; ++q) uw[q] = (ORC_REAL)umat[q];
    }
    ORC_REAL* hw = NULL;  /* hop ratios of every half step, rounded once */
    const size_t HS = (size_t)N * ORC_MAXDEG * 2;
    if (hopw) {
        if (inv) { free(vw); free(uw); return -1; }
        hw = (ORC_REAL*)malloc(sizeof(ORC_REAL) * HS * (size_t)(2 * n_steps + 1));
        if (!hw) { free(vw); free(uw); return -2; }
        for (size_t q = 0; q < HS * (size_t)(2 * n_steps + 1); ++q) hw[q] = (ORC_REAL)hopw[q];
    }
    int failed = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        ORC_REAL* y = (ORC_REAL*)malloc(sizeof(ORC_REAL) * E);
        ORC_REAL* Y = (ORC_REAL*)malloc(sizeof(ORC_REAL) * E);
        ORC_REAL* k = (ORC_REAL*)malloc(sizeof(ORC_REAL) * E);
        ORC_REAL* acc = (ORC_REAL*)malloc(sizeof(ORC_REAL) * E);
        if (!y || !Y || !k || !acc) {
            failed = 1;
        } else {
            double* src = rho_io + (size_t)m * E;
            for (size_t e = 0; e < E; ++e) y[e] = (ORC_REAL)src[e];
            int64_t r = 0;
            for (int64_t step = 0; step <= n_steps; ++step) {
                if (step % record_every == 0) {
                    if (X)
                        for (int s = 0; s < 2; ++s)
                            for (int i = 0; i < N; ++i)
                                X[((size_t)r * M + m) * D + s * N + i] =
                                    (double)y[s * N * N * 2 + 2 * (i * N + i)];
                    if (inv)
                        ORC_NAME(invariants)(N, nbr, deg, t, U, y,
                                             inv + ((size_t)r * M + m) * 5);
                    ++r;
                }
                if (step == n_steps) break;
                /* stage 1 */
                ORC_NAME(oracle_rhs_hop)(N, nbr, deg, tw, Uw, uw, vw,
                                         vw ? (ORC_REAL)env[2 * step + 0] : (ORC_REAL)0,
                                         hw ? hw + (size_t)(2 * step + 0) * HS : NULL, y, k);
                for (size_t e = 0; e < E; ++e) {
                    acc[e] = k[e];
                    Y[e] = ORC_FMA(c_half, k[e], y[e]);
                }
                /* stage 2 */
                ORC_NAME(oracle_rhs_hop)(N, nbr, deg, tw, Uw, uw, vw,
                                         vw ? (ORC_REAL)env[2 * step + 1] : (ORC_REAL)0,
                                         hw ? hw + (size_t)(2 * step + 1) * HS : NULL, Y, k);
                for (size_t e = 0; e < E; ++e) {
                    acc[e] = ORC_FMA(two, k[e], acc[e]);
                    Y[e] = ORC_FMA(c_half, k[e], y[e]);
                }
                /* stage 3 */
                ORC_NAME(oracle_rhs_hop)(N, nbr, deg, tw, Uw, uw, vw,
                                         vw ? (ORC_REAL)env[2 * step + 1] : (ORC_REAL)0,
                                         hw ? hw + (size_t)(2 * step + 1) * HS : NULL, Y, k);
                for (size_t e = 0; e < E; ++e) {
                    acc[e] = ORC_FMA(two, k[e], acc[e]);
                    Y[e] = ORC_FMA(c_full, k[e], y[e]);
                }
                /* stage 4 */
                ORC_NAME(oracle_rhs_hop)(N, nbr, deg, tw, Uw, uw, vw,
                                         vw ? (ORC_REAL)env[2 * step + 2] : (ORC_REAL)0,
                                         hw ? hw + (size_t)(2 * step + 2) * HS : NULL, Y, k);
                for (size_t e = 0; e < E; ++e) {
                    acc[e] = acc[e] + k[e];
                    y[e] = ORC_FMA(c_sixth, acc[e], y[e]);
                }
            }
            (void)n_rec;
            for (size_t e = 0; e < E; ++e) src[e] = (double)y[e];
        }
        free(y); free(Y); free(k); free(acc);
    }
    free(vw);
    free(uw);
    free(hw);
    return failed ? -2 : 0;
}

int ORC_NAME(oracle_evolve_gen)(int N, const int32_t* nbr, const uint8_t* deg,
                                double t, double U, const double* umat, const double* vsite,
                                const double* env, double dt, int64_t n_steps,
                                int record_every, int64_t M, double* rho_io, double* X,
                                double* inv)
{
    return ORC_NAME(oracle_evolve_hop)(N, nbr, deg, t, U, umat, vsite, env, NULL, dt, n_steps,
                                       record_every, M, rho_io, X, inv);
}

int ORC_NAME(oracle_evolve_pot)(int N, const int32_t* nbr, const uint8_t* deg,
                                double t, double U, const double* vsite, const double* env,
                                double dt, int64_t n_steps, int record_every, int64_t M,
                                double* rho_io, double* X, double* inv)
{
    return ORC_NAME(oracle_evolve_gen)(N, nbr, deg, t, U, NULL, vsite, env, dt, n_steps,
                                       record_every, M, rho_io, X, inv);
}

int ORC_NAME(oracle_evolve)(int N, const int32_t* nbr, const uint8_t* deg,
                            double t, double U, double dt, int64_t n_steps,
                            int record_every, int64_t M, double* rho_io,
                            double* X, double* inv)
{
    return ORC_NAME(oracle_evolve_pot)(N, nbr, deg, t, U, NULL, NULL, dt, n_steps,
                                       record_every, M, rho_io, X, inv);
}

#undef ORC_NAME
#undef ORC_CAT
#undef ORC_CAT2

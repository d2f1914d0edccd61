/*
 * ftwa_oracle.c -- CPU oracle for the fTWA hot path (test infrastructure only).
 *
 * This file is NOT part of the product.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant generator with the HIP library.
 *
 * What it computes (Rousse, Eriksson, Ogren, "Correlated quantum dynamics of
 * graphene", arXiv:2212.04352), plainly and slowly, in FP64 unless asked for
 * FP32:
 *
 *   - honeycomb lattices with nearest-neighbour hopping j_ij = t and on-site
 *     interaction u_ij = U delta_ij (Sec. II, Eq. (1));
 *   - Gaussian initial phase-space points around a Fock state (Sec. III,
 *     Eq. (7); covariance derived in Appendix A.3);
 *   - trajectories of the fTWA equation of motion (Sec. III, Eq. (6)),
 *     integrated with the classical fourth-order Runge-Kutta method
 *     (the paper does not name its integrator);
 *   - stochastic averages of the diagonal phase-space variables, giving site
 *     occupations and density-density moments (Eq. (5), Eq. (10)).
 *
 * Conventions that the paper leaves open are fixed here and listed, with
 * their reasons, in the design notes of the repository:
 *   random numbers: Philox4x32-10 (Salmon et al., SC'11), keyed by the seed,
 *   with counter (pair index, instance<<1|spin, trajectory, tag);
 *   complex normal xi with E|xi|^2 = 1, E xi^2 = 0, by Box-Muller;
 *   neighbour sums taken in ascending neighbour order, explicit fma where
 *   stated, no other fused operations (build with -ffp-contract=off).
 *
 * Storage in this file: one trajectory is two full N x N complex matrices
 * rho[spin][i][j] (spin 0 = up, 1 = down), stored as interleaved doubles
 * (re, im), i.e. element (s, i, j) at offset 2*((s*N + i)*N + j).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXDEG 3

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of a multiply-xor bijection on a     */
/* 128-bit counter, the 64-bit key incremented by the Weyl constants between */
/* rounds.                                                                   */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                          uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t prod0 = (uint64_t)mult0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)mult1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Two 53-bit integers from one Philox block: a = x0:x1[31:11], b = x2:x3[31:11]. */
static void philox_53bit_pair(const uint32_t x[4], uint64_t* a, uint64_t* b)
{
    *a = ((uint64_t)x[0] << 21) | (uint64_t)(x[1] >> 11);
    *b = ((uint64_t)x[2] << 21) | (uint64_t)(x[3] >> 11);
}

static void seed_to_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
}

/* ------------------------------------------------------------------------ */
/* Lattices (Sec. II: nearest-neighbour hopping on a honeycomb, graphene).   */
/* The paper's own geometries exist only in its figures; the three families  */
/* below are this project's definitions.                                     */
/*   kind 0: periodic torus of a x b unit cells, site 2*(x*b + y) + s,        */
/*           A(x,y) bonded to B(x,y), B(x-1,y), B(x,y-1) (indices mod a, b).  */
/*   kind 1: brick-wall rectangle of a rows x b columns, horizontal bonds     */
/*           (r,c)-(r,c+1), vertical bonds (r,c)-(r+1,c) when r+c is even;    */
/*           sites of degree < 2 removed until none is left; row-major order. */
/*   kind 2: zigzag hexagonal flake of a rings: the hexagons at hex distance  */
/*           <= a-1 from a centre hexagon, drawn on the same brick wall,      */
/*           sites ordered by (row, column).                                  */
/* Output: neighbour lists sorted ascending, padded with -1.                  */
/* ------------------------------------------------------------------------ */
static int add_bond(int N, int32_t* nbr, uint8_t* deg, int u, int v)
{
    if (u == v || u < 0 || v < 0 || u >= N || v >= N) return -1;
    for (int k = 0; k < deg[u]; ++k)
        if (nbr[u * ORC_MAXDEG + k] == v) return 0; /* already present */
    if (deg[u] >= ORC_MAXDEG || deg[v] >= ORC_MAXDEG) return -1;
    nbr[u * ORC_MAXDEG + deg[u]++] = v;
    nbr[v * ORC_MAXDEG + deg[v]++] = u;
    return 1;
}

static void sort_neighbours(int N, int32_t* nbr, const uint8_t* deg)
{
    for (int s = 0; s < N; ++s) {
        int32_t* l = nbr + s * ORC_MAXDEG;
        for (int a = 0; a < deg[s]; ++a)
            for (int b = a + 1; b < deg[s]; ++b)
                if (l[b] < l[a]) { int32_t tmp = l[a]; l[a] = l[b]; l[b] = tmp; }
        for (int a = deg[s]; a < ORC_MAXDEG; ++a) l[a] = -1;
    }
}

static int pos_mod(int x, int m) { int r = x % m; return r < 0 ? r + m : r; }

/* Brick-wall bond rule shared by kinds 1 and 2. */
static int brick_bonded(int r0, int c0, int r1, int c1)
{
    if (r0 == r1 && (c1 - c0 == 1 || c0 - c1 == 1)) return 1;
    if (c0 == c1 && (r1 - r0 == 1 || r0 - r1 == 1)) {
        int rl = r0 < r1 ? r0 : r1;
        return pos_mod(rl + c0, 2) == 0;
    }
    return 0;
}

/* Builds the neighbour table of a set of brick-wall sites (rows rr, cols cc,
   already in the final numbering). */
static int brick_bonds(int N, const int* rr, const int* cc, int32_t* nbr,
                       uint8_t* deg, uint8_t* sub, int* n_bonds)
{
    memset(deg, 0, (size_t)N);
    int nb = 0;
    for (int u = 0; u < N; ++u)
        for (int v = u + 1; v < N; ++v)
            if (brick_bonded(rr[u], cc[u], rr[v], cc[v])) {
                if (add_bond(N, nbr, deg, u, v) != 1) return -1;
                ++nb;
            }
    for (int u = 0; u < N; ++u) sub[u] = (uint8_t)pos_mod(rr[u] + cc[u], 2);
    sort_neighbours(N, nbr, deg);
    *n_bonds = nb;
    return 0;
}

int oracle_build_lattice(int kind, int a, int b, int max_sites, int* n_sites,
                         int32_t* nbr, uint8_t* deg, uint8_t* sub, int* n_bonds)
{
    if (kind == 0) {
        if (a < 2 || b < 2) return -1;
        int N = 2 * a * b;
        if (N > max_sites) return -2;
        memset(deg, 0, (size_t)N);
        int nb = 0;
        for (int x = 0; x < a; ++x)
            for (int y = 0; y < b; ++y) {
                int A = 2 * (x * b + y);
                int B0 = 2 * (x * b + y) + 1;
                int B1 = 2 * (pos_mod(x - 1, a) * b + y) + 1;
                int B2 = 2 * (x * b + pos_mod(y - 1, b)) + 1;
                int targets[3] = {B0, B1, B2};
                for (int k = 0; k < 3; ++k) {
                    int r = add_bond(N, nbr, deg, A, targets[k]);
                    if (r < 0) return -1;
                    nb += r;
                }
            }
        for (int s = 0; s < N; ++s) sub[s] = (uint8_t)(s % 2);
        sort_neighbours(N, nbr, deg);
        *n_sites = N;
        *n_bonds = nb;
        return 0;
    }
    if (kind == 1) {
        if (a < 2 || b < 2) return -1;
        int R = a, C = b;
        int* alive = (int*)calloc((size_t)R * C, sizeof(int));
        for (int k = 0; k < R * C; ++k) alive[k] = 1;
        int changed = 1;
        while (changed) {
            changed = 0;
            for (int r = 0; r < R; ++r)
                for (int c = 0; c < C; ++c) {
                    if (!alive[r * C + c]) continue;
                    int d = 0;
                    if (c > 0 && alive[r * C + c - 1]) ++d;
                    if (c + 1 < C && alive[r * C + c + 1]) ++d;
                    if (r > 0 && alive[(r - 1) * C + c] && brick_bonded(r - 1, c, r, c)) ++d;
                    if (r + 1 < R && alive[(r + 1) * C + c] && brick_bonded(r, c, r + 1, c)) ++d;
                    if (d < 2) { alive[r * C + c] = 0; changed = 1; }
                }
        }
        int N = 0;
        for (int k = 0; k < R * C; ++k) N += alive[k];
        if (N > max_sites || N == 0) { free(alive); return -2; }
        int* rr = (int*)malloc(sizeof(int) * (size_t)N);
        int* cc = (int*)malloc(sizeof(int) * (size_t)N);
        int s = 0;
        for (int r = 0; r < R; ++r)
            for (int c = 0; c < C; ++c)
                if (alive[r * C + c]) { rr[s] = r; cc[s] = c; ++s; }
        int rc = brick_bonds(N, rr, cc, nbr, deg, sub, n_bonds);
        free(alive); free(rr); free(cc);
        *n_sites = N;
        return rc;
    }
    if (kind == 2) {
        if (a < 1) return -1;
        int n = a;
        /* bounding box of the flake in brick-wall coordinates */
        int rmin = -(n - 1), rmax = n, cmin = -3 * (n - 1), cmax = 3 * (n - 1) + 2;
        int R = rmax - rmin + 1, C = cmax - cmin + 1;
        int* mark = (int*)calloc((size_t)R * C, sizeof(int));
        for (int ha = -(n - 1); ha <= n - 1; ++ha)
            for (int hb = -(n - 1); hb <= n - 1; ++hb) {
                int dist = (abs(ha) + abs(hb) + abs(ha + hb)) / 2;
                if (dist > n - 1) continue;
                int r0 = hb, c0 = 2 * ha + hb; /* lower-left site of the hexagon */
                for (int dr = 0; dr < 2; ++dr)
                    for (int dc = 0; dc < 3; ++dc)
                        mark[(r0 + dr - rmin) * C + (c0 + dc - cmin)] = 1;
            }
        int N = 0;
        for (int k = 0; k < R * C; ++k) N += mark[k];
        if (N > max_sites) { free(mark); return -2; }
        int* rr = (int*)malloc(sizeof(int) * (size_t)N);
        int* cc = (int*)malloc(sizeof(int) * (size_t)N);
        int s = 0;
        for (int r = 0; r < R; ++r)
            for (int c = 0; c < C; ++c)
                if (mark[r * C + c]) { rr[s] = r + rmin; cc[s] = c + cmin; ++s; }
        int rc = brick_bonds(N, rr, cc, nbr, deg, sub, n_bonds);
        free(mark); free(rr); free(cc);
        *n_sites = N;
        return rc;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Initial occupations n_{i sigma}(0) of a Fock state (Sec. IV.A: every site  */
/* holds one electron of either spin).                                       */
/*   kind 0 (Neel): up on sublattice A, down on sublattice B.                */
/*   kind 1 (random): Fisher-Yates permutation of the sites drawn with        */
/*   Philox counter (i, instance, 0, 1); the first N/2 sites of the           */
/*   permutation hold an up electron, the others a down electron.            */
/* Output n0[spin*N + i].                                                    */
/* ------------------------------------------------------------------------ */
int oracle_fock_start(int N, const uint8_t* sub, int kind, uint64_t seed,
                      uint32_t instance, double* n0)
{
    if (kind == 0) {
        for (int i = 0; i < N; ++i) {
            n0[i] = sub[i] == 0 ? 1.0 : 0.0;
            n0[N + i] = sub[i] == 0 ? 0.0 : 1.0;
        }
        return 0;
    }
    if (kind == 1) {
        if (N % 2 != 0) return -1;
        int* perm = (int*)malloc(sizeof(int) * (size_t)N);
        for (int i = 0; i < N; ++i) perm[i] = i;
        uint32_t key[2];
        seed_to_key(seed, key);
        for (int i = N - 1; i >= 1; --i) {
            uint32_t ctr[4] = {(uint32_t)i, instance, 0u, 1u}, x[4];
            oracle_philox4x32_10(ctr, key, x);
            uint64_t a53, b53;
            philox_53bit_pair(x, &a53, &b53);
            unsigned __int128 prod = (unsigned __int128)a53 * (unsigned __int128)(i + 1);
            int j = (int)(prod >> 53);
            int tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
        }
        for (int k = 0; k < N; ++k) {
            int site = perm[k];
            int up = k < N / 2;
            n0[site] = up ? 1.0 : 0.0;
            n0[N + site] = up ? 0.0 : 1.0;
        }
        free(perm);
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Initial phase-space point of one trajectory (Eq. (7)):                    */
/*   rho_ii = n_i - 1/2,                                                     */
/*   rho_ij = xi_ij * sqrt((n_i + n_j - 2 n_i n_j)/2) for i < j,             */
/*   rho_ji = conj(rho_ij),                                                  */
/* xi complex normal with E|xi|^2 = 1 (the normalisation fixed by the        */
/* covariance in Appendix A.3).  Box-Muller on two 53-bit uniforms:          */
/*   u1 = (a+1) 2^-53 in (0,1], u2 = b 2^-53 in [0,1),                        */
/*   xi = sqrt(-ln u1) (cos 2 pi u2 + i sin 2 pi u2).                        */
/* Counter of pair (i<j): (i N - i(i+1)/2 + j-i-1, instance<<1|spin, m, 0).  */
/* rho_out: [M][2][N][N] complex, trajectory m has global index              */
/* traj_offset + m.                                                          */
/* ------------------------------------------------------------------------ */
void oracle_complex_normal(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                           double* re, double* im)
{
    uint32_t key[2], x[4];
    seed_to_key(seed, key);
    uint32_t ctr[4] = {c0, c1, c2, 0u};
    oracle_philox4x32_10(ctr, key, x);
    uint64_t a53, b53;
    philox_53bit_pair(x, &a53, &b53);
    const double two_m53 = 1.0 / 9007199254740992.0; /* 2^-53 */
    double u1 = (double)(a53 + 1u) * two_m53;
    double u2 = (double)b53 * two_m53;
    double r = sqrt(-log(u1));
    double theta = 2.0 * M_PI * u2;
    *re = r * cos(theta);
    *im = r * sin(theta);
}

/* ------------------------------------------------------------------------ */
/* Real standard normal for the diagonal of a thermal initial state: the     */
/* covariance of Appendix A.3 at alpha = beta = mu = nu = i is                */
/* (1 - n_i) n_i, and the diagonal is uncorrelated with every other element  */
/* (the off-diagonal occupations vanish in the site basis), so              */
/*   rho_ii = n_i - 1/2 + sqrt(n_i (1 - n_i)) g_i,                           */
/* g_i by Box-Muller from the two uniforms of counter                        */
/* (i, instance<<1|spin, m, 2):  g = sqrt(-2 ln u1) cos(2 pi u2).             */
/* ------------------------------------------------------------------------ */
double oracle_real_normal(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3)
{
    uint32_t key[2], x[4];
    seed_to_key(seed, key);
    uint32_t ctr[4] = {c0, c1, c2, c3};
    oracle_philox4x32_10(ctr, key, x);
    uint64_t a53, b53;
    philox_53bit_pair(x, &a53, &b53);
    const double two_m53 = 1.0 / 9007199254740992.0; /* 2^-53 */
    double u1 = (double)(a53 + 1u) * two_m53;
    double u2 = (double)b53 * two_m53;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

void oracle_sample(int N, const double* n0, uint64_t seed, uint32_t instance,
                   int64_t traj_offset, int64_t M, int thermal, double* rho_out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < M; ++m) {
        double* rho = rho_out + (size_t)m * 2 * N * N * 2;
        uint32_t gm = (uint32_t)(traj_offset + m);
        for (int s = 0; s < 2; ++s) {
            const double* n = n0 + s * N;
            double* R = rho + (size_t)s * N * N * 2;
            for (int i = 0; i < N; ++i) {
                double d = n[i] - 0.5;
                double var = n[i] * (1.0 - n[i]);
                if (thermal && var != 0.0)
                    d += sqrt(var) * oracle_real_normal(seed, (uint32_t)i,
                                                        (instance << 1) | (uint32_t)s, gm, 2u);
                R[2 * (i * N + i)] = d;
                R[2 * (i * N + i) + 1] = 0.0;
            }
            for (int i = 0; i < N; ++i)
                for (int j = i + 1; j < N; ++j) {
                    double var = 0.5 * ((n[i] + n[j]) - (2.0 * n[i]) * n[j]);
                    double re = 0.0, im = 0.0;
                    if (var != 0.0) {
                        uint32_t pair = (uint32_t)(i * N - (i * (i + 1)) / 2 + (j - i - 1));
                        double xr, xi;
                        oracle_complex_normal(seed, pair, (instance << 1) | (uint32_t)s,
                                              gm, &xr, &xi);
                        double amp = sqrt(var);
                        re = amp * xr;
                        im = amp * xi;
                    }
                    R[2 * (i * N + j)] = re;
                    R[2 * (i * N + j) + 1] = im;
                    R[2 * (j * N + i)] = re;
                    R[2 * (j * N + i) + 1] = -im;
                }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Equation of motion and Runge-Kutta integration, FP64 and FP32 variants.   */
/* ------------------------------------------------------------------------ */
#define ORC_REAL double
#define ORC_FMA fma
#define ORC_SUFFIX _f64
#include "ftwa_oracle_evolve.h"
#undef ORC_REAL
#undef ORC_FMA
#undef ORC_SUFFIX

#define ORC_REAL float
#define ORC_FMA fmaf
#define ORC_SUFFIX _f32
#include "ftwa_oracle_evolve.h"
#undef ORC_REAL
#undef ORC_FMA
#undef ORC_SUFFIX

/* ------------------------------------------------------------------------ */
/* Ensemble moments of the diagonal variables x_m = (rho_ii up, rho_ii down) */
/* (Eq. (5) and Eq. (10) need their first and second moments):               */
/*   S1[a] = sum_m x_m[a],  S2[a,b] = sum_m x_m[a] x_m[b]  (a <= b),         */
/* sums taken pairwise over m.  X: [n_rec][M][D], D = 2N.                    */
/* S2 is the packed upper triangle, index a*D - a(a-1)/2 + (b-a).            */
/* ------------------------------------------------------------------------ */
static double pairwise_sum(const double* v, int64_t n)
{
    if (n == 0) return 0.0;
    if (n == 1) return v[0];
    int64_t h = n / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, n - h);
}

void oracle_moments(int D, int64_t M, int n_rec, const double* X, double* S1,
                    double* S2)
{
    int64_t npair = (int64_t)D * (D + 1) / 2;
    #pragma omp parallel for schedule(dynamic)
    for (int r = 0; r < n_rec; ++r) {
        double* tmp = (double*)malloc(sizeof(double) * (size_t)(M > 0 ? M : 1));
        const double* Xr = X + (size_t)r * M * D;
        for (int a = 0; a < D; ++a) {
            for (int64_t m = 0; m < M; ++m) tmp[m] = Xr[m * D + a];
            S1[(size_t)r * D + a] = pairwise_sum(tmp, M);
            for (int b = a; b < D; ++b) {
                for (int64_t m = 0; m < M; ++m) tmp[m] = Xr[m * D + a] * Xr[m * D + b];
                int64_t idx = (int64_t)a * D - (int64_t)a * (a - 1) / 2 + (b - a);
                S2[(size_t)r * npair + idx] = pairwise_sum(tmp, M);
            }
        }
        free(tmp);
    }
}

/* ------------------------------------------------------------------------ */
/* Observables from the moments (plug-in estimators, divisor M):             */
/*   n_a   = S1_a/M + 1/2                              (Eq. (5), first line) */
/*   C_ab  = S2_ab/M - (S1_a/M)(S1_b/M)   connected density-density          */
/*   g2_ab = (S2_ab/M + (S1_a+S1_b)/(2M) + 1/4) / ((S1_a/M+1/2)(S1_b/M+1/2)) */
/*                                                              (Eq. (10))    */
/* a = spin*N + site.  C and g2 are full D x D matrices; their diagonal is   */
/* the Weyl-symbol variance, not a same-site observable.                     */
/* ------------------------------------------------------------------------ */
void oracle_observables(int N, int64_t M, int n_rec, const double* S1,
                        const double* S2, double* n_out, double* C_out,
                        double* g2_out)
{
    int D = 2 * N;
    int64_t npair = (int64_t)D * (D + 1) / 2;
    double invM = 1.0 / (double)M;
    for (int r = 0; r < n_rec; ++r) {
        const double* s1 = S1 + (size_t)r * D;
        const double* s2 = S2 + (size_t)r * npair;
        for (int a = 0; a < D; ++a) n_out[(size_t)r * D + a] = s1[a] * invM + 0.5;
        for (int a = 0; a < D; ++a)
            for (int b = 0; b < D; ++b) {
                int lo = a < b ? a : b, hi = a < b ? b : a;
                int64_t idx = (int64_t)lo * D - (int64_t)lo * (lo - 1) / 2 + (hi - lo);
                double mab = s2[idx] * invM;
                double ma = s1[a] * invM, mb = s1[b] * invM;
                if (C_out) C_out[((size_t)r * D + a) * D + b] = mab - ma * mb;
                if (g2_out)
                    g2_out[((size_t)r * D + a) * D + b] =
                        (mab + 0.5 * (ma + mb) + 0.25) / ((ma + 0.5) * (mb + 0.5));
            }
    }
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Forward-mode derivative (tangent) of the FP64 trajectories, for the
 * gradient of losses built on the site occupations.  Parameters: the
 * interaction U, the hopping t, and a shift of the initial diagonal
 * rho_ii,s(0) (the off-diagonal noise is held fixed).  The right-hand side
 * of Eq. (6),
 *   f_ij = i [ t (C_ij - R_ij) + U (d_i - d_j) rho_ij ],
 *   C_ij = sum_{k in nb(j)} rho_ik,  R_ij = sum_{k in nb(i)} rho_kj,
 *   d = diagonal of the other spin block,
 * is differentiated term by term along (rho', U', t'):
 *   f'_ij = i [ t' (C_ij - R_ij) + t (C'_ij - R'_ij)
 *               + U' (d_i - d_j) rho_ij + U (d'_i - d'_j) rho_ij
 *               + U (d_i - d_j) rho'_ij ],
 * and carried through the classical Runge-Kutta stages by the chain rule:
 *   k_s' = f'(Y_s, Y_s'),  Y_{s+1}' = y' + c_s k_s',
 *   y'  <- y' + (h/6) (k1' + 2 k2' + 2 k3' + k4').
 * Plain FP64 arithmetic in natural order (no fixed fma pattern: this is a
 * derivative check, not a bitwise reference).
 */
static void tangent_rhs(int N, const int32_t* nbr, const uint8_t* deg, double t, double U,
                        double dt_hop, double dU, const double* y, const double* yd,
                        double* f, double* fd)
{
    const size_t NN2 = (size_t)N * N * 2;
    for (int s = 0; s < 2; ++s) {
        const double* R = y + s * NN2;
        const double* Rd = yd + s * NN2;
        const double* B = y + (1 - s) * NN2;
        const double* Bd = yd + (1 - s) * NN2;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                double h_re = 0, h_im = 0, hd_re = 0, hd_im = 0;
                for (int n = 0; n < deg[j]; ++n) {
                    int k = nbr[j * ORC_MAXDEG + n];
                    h_re += R[2 * (i * N + k)];
                    h_im += R[2 * (i * N + k) + 1];
                    hd_re += Rd[2 * (i * N + k)];
                    hd_im += Rd[2 * (i * N + k) + 1];
                }
                for (int n = 0; n < deg[i]; ++n) {
                    int k = nbr[i * ORC_MAXDEG + n];
                    h_re -= R[2 * (k * N + j)];
                    h_im -= R[2 * (k * N + j) + 1];
                    hd_re -= Rd[2 * (k * N + j)];
                    hd_im -= Rd[2 * (k * N + j) + 1];
                }
                const double dd = B[2 * (i * N + i)] - B[2 * (j * N + j)];
                const double ddd = Bd[2 * (i * N + i)] - Bd[2 * (j * N + j)];
                const double r_re = R[2 * (i * N + j)], r_im = R[2 * (i * N + j) + 1];
                const double rd_re = Rd[2 * (i * N + j)], rd_im = Rd[2 * (i * N + j) + 1];
                /* g = t h + U dd rho,  f = i g */
                const double g_re = t * h_re + U * dd * r_re;
                const double g_im = t * h_im + U * dd * r_im;
                const double gd_re = dt_hop * h_re + t * hd_re + dU * dd * r_re +
                                     U * ddd * r_re + U * dd * rd_re;
                const double gd_im = dt_hop * h_im + t * hd_im + dU * dd * r_im +
                                     U * ddd * r_im + U * dd * rd_im;
                f[s * NN2 + 2 * (i * N + j)] = -g_im;
                f[s * NN2 + 2 * (i * N + j) + 1] = g_re;
                fd[s * NN2 + 2 * (i * N + j)] = -gd_im;
                fd[s * NN2 + 2 * (i * N + j) + 1] = gd_re;
            }
    }
}

/*
 * rho0: [M][2][N][N] complex FP64 (not modified); the direction is
 * (dU, dt_hop, dshift[2][N]) with rho_ii,s(0)' = dshift[s][i].
 * X, Xd: [n_rec][M][2N] diagonal records of rho and of its derivative.
 */
int oracle_evolve_tangent(int N, const int32_t* nbr, const uint8_t* deg, double t, double U,
                          double dt, int64_t n_steps, int record_every, int64_t M,
                          const double* rho0, double dU, double dt_hop, const double* dshift,
                          double* X, double* Xd)
{
    if (N <= 0 || M < 0 || n_steps < 0 || record_every <= 0) return -1;
    const size_t E = (size_t)2 * N * N * 2;
    const int D = 2 * N;
    const double ch = 0.5 * dt, cf = dt, c6 = dt / 6.0;
    const double cs[3] = {ch, ch, cf};
    int failed = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < M; ++m) {
        double* buf = (double*)malloc(sizeof(double) * E * 8);
        if (!buf) {
            failed = 1;
            continue;
        }
        double *y = buf, *yd = buf + E, *Y = buf + 2 * E, *Yd = buf + 3 * E;
        double *k = buf + 4 * E, *kd = buf + 5 * E, *acc = buf + 6 * E, *accd = buf + 7 * E;
        memcpy(y, rho0 + (size_t)m * E, sizeof(double) * E);
        memset(yd, 0, sizeof(double) * E);
        for (int s = 0; s < 2; ++s)
            for (int i = 0; i < N; ++i) yd[s * N * N * 2 + 2 * (i * N + i)] = dshift[s * N + i];
        int64_t r = 0;
        for (int64_t step = 0; step <= n_steps; ++step) {
            if (step % record_every == 0) {
                for (int s = 0; s < 2; ++s)
                    for (int i = 0; i < N; ++i) {
                        const size_t o = (size_t)s * N * N * 2 + 2 * (i * N + i);
                        X[((size_t)r * M + m) * D + s * N + i] = y[o];
                        Xd[((size_t)r * M + m) * D + s * N + i] = yd[o];
                    }
                ++r;
            }
            if (step == n_steps) break;
            memcpy(Y, y, sizeof(double) * E);
            memcpy(Yd, yd, sizeof(double) * E);
            for (int stage = 0; stage < 4; ++stage) {
                tangent_rhs(N, nbr, deg, t, U, dt_hop, dU, Y, Yd, k, kd);
                const double w = (stage == 0 || stage == 3) ? 1.0 : 2.0;
                for (size_t e = 0; e < E; ++e) {
                    acc[e] = stage == 0 ? k[e] : acc[e] + w * k[e];
                    accd[e] = stage == 0 ? kd[e] : accd[e] + w * kd[e];
                }
                if (stage < 3)
                    for (size_t e = 0; e < E; ++e) {
                        Y[e] = y[e] + cs[stage] * k[e];
                        Yd[e] = yd[e] + cs[stage] * kd[e];
                    }
            }
            for (size_t e = 0; e < E; ++e) {
                y[e] += c6 * acc[e];
                yd[e] += c6 * accd[e];
            }
        }
        free(buf);
    }
    return failed ? -2 : 0;
}

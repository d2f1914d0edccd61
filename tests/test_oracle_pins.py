"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Paper: Rousse, Eriksson, Ogren, "Correlated quantum dynamics of graphene",
arXiv:2212.04352.  Every test names the passage or identity it pins.  None of
them re-types the oracle's own formula: each compares with a closed form, a
printed value, an independent library routine, a conservation law, an exact
propagator or a statistical law, chosen so that a dropped term, a wrong sign, a
wrong index or a transposed operand in the oracle fails at least one of them.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as sst
from scipy.integrate import solve_ivp

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Philox4x32-10 (random numbers; the paper names no generator)
# ---------------------------------------------------------------------------
def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers(orc):
    for ctr, key, want in _kat_rows():
        assert list(orc.philox4x32_10(ctr, key)) == want


def test_philox_matches_rocrand(orc, tmp_path):
    """rocRAND's Philox4x32-10 is an independent implementation (host build)."""
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "rocrand_philox_check"
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-o", str(exe),
                    os.path.join(HERE, "rocrand_philox_check.cpp")], check=True,
                   capture_output=True)
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    text = "\n".join(" ".join(f"{int(v):08x}" for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    got = [[int(x, 16) for x in line.split()] for line in out.stdout.strip().splitlines()]
    for row, ref in zip(cases, got):
        assert list(orc.philox4x32_10(row[:4], row[4:])) == ref


# ---------------------------------------------------------------------------
# Lattices (Sec. II: nearest-neighbour honeycomb)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind,a,b,N,nb,deg2,deg3", [
    ("torus", 2, 3, 12, 18, 0, 12),
    ("torus", 3, 9, 54, 81, 0, 54),
    ("armchair", 10, 20, 198, 278, 38, 160),
    ("hex", 1, 0, 6, 6, 6, 0),
    ("hex", 2, 0, 24, 30, 12, 12),
    ("hex", 3, 0, 54, 72, 18, 36),
    ("hex", 4, 0, 96, 132, 24, 72),
    ("hex", 5, 0, 150, 210, 30, 120),
])
def test_lattice_counts(orc, kind, a, b, N, nb, deg2, deg3):
    lat = orc.Lattice(kind, a, b)
    assert lat.N == N and lat.n_bonds == nb
    assert int((lat.deg == 2).sum()) == deg2 and int((lat.deg == 3).sum()) == deg3
    # symmetric, ascending, bipartite and balanced (graphene has two sublattices)
    for i in range(lat.N):
        lst = list(lat.nbr[i, : lat.deg[i]])
        assert lst == sorted(lst)
        assert all(x == -1 for x in lat.nbr[i, lat.deg[i]:])
        for k in lst:
            assert i in lat.nbr[k, : lat.deg[k]]
            assert lat.sub[i] != lat.sub[k]
    assert int(lat.sub.sum()) * 2 == lat.N


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_hex_flake_closed_forms(orc, n):
    """Coronene-family flakes: 6n^2 atoms and 9n^2 - 3n bonds; Euler's formula
    for a planar benzenoid with h = 3n^2 - 3n + 1 hexagons gives E = V + h - 1."""
    lat = orc.Lattice("hex", n, 0)
    h = 3 * n * n - 3 * n + 1
    assert lat.N == 6 * n * n
    assert lat.n_bonds == 9 * n * n - 3 * n == lat.N + h - 1


@pytest.mark.parametrize("L1,L2", [(2, 3), (3, 9), (4, 4), (2, 2)])
def test_torus_spectrum_closed_form(orc, L1, L2):
    """Honeycomb Bloch bands: eigenvalues +-|1 + e^{i k1} + e^{i k2}|, k = 2 pi (p/L1, q/L2)."""
    lat = orc.Lattice("torus", L1, L2)
    ev = np.sort(np.linalg.eigvalsh(lat.hopping_matrix()))
    p, q = np.meshgrid(np.arange(L1), np.arange(L2), indexing="ij")
    e = np.abs(1 + np.exp(2j * np.pi * p / L1) + np.exp(2j * np.pi * q / L2)).ravel()
    assert np.allclose(ev, np.sort(np.concatenate([e, -e])), atol=1e-12)


def test_armchair_flake_geometry(orc):
    """10 x 20 brick wall with its two degree-1 corners trimmed: 81 hexagons by
    Euler's formula, spectrum symmetric (bipartite)."""
    lat = orc.Lattice("armchair", 10, 20)
    assert lat.n_bonds - lat.N + 1 == 81
    ev = np.sort(np.linalg.eigvalsh(lat.hopping_matrix()))
    assert np.allclose(ev, -ev[::-1], atol=1e-12)


# ---------------------------------------------------------------------------
# Fock starts (Sec. IV.A: each site singly occupied)
# ---------------------------------------------------------------------------
def test_fock_neel(orc):
    lat = orc.Lattice("torus", 2, 3)
    n0 = orc.fock_start(lat, "neel")
    assert np.array_equal(n0[0], 1.0 - lat.sub) and np.array_equal(n0[1], lat.sub * 1.0)


def test_fock_random(orc):
    lat = orc.Lattice("torus", 3, 9)
    ups = np.zeros(lat.N)
    K = 2000
    for inst in range(K):
        n0 = orc.fock_start(lat, "random", seed=0x2212043520000002, instance=inst)
        assert np.array_equal(n0[0] + n0[1], np.ones(lat.N))
        assert n0[0].sum() == lat.N // 2
        ups += n0[0]
    # a uniform permutation puts an up electron on every site with probability 1/2
    se = np.sqrt(0.25 / K)
    assert np.all(np.abs(ups / K - 0.5) < 5 * se)
    a = orc.fock_start(lat, "random", seed=5, instance=3)
    b = orc.fock_start(lat, "random", seed=5, instance=3)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Initial Gaussian sampling, Eq. (7) and the covariance of Appendix A.3
# ---------------------------------------------------------------------------
def test_sample_structure(orc):
    lat = orc.Lattice("torus", 2, 3)
    n0 = orc.fock_start(lat, "neel")
    rho = orc.sample(lat, n0, seed=11, M=8)
    for m in range(8):
        for s in range(2):
            R = rho[m, s]
            assert np.array_equal(R, R.conj().T)
            assert np.array_equal(np.diag(R).real, n0[s] - 0.5)
            same = n0[s][:, None] == n0[s][None, :]
            off = ~np.eye(lat.N, dtype=bool)
            assert np.all(R[same & off] == 0)
            assert np.all(np.abs(R[~same]) > 0)
    # subsets are exact: trajectory m of a run is trajectory m - off of a run
    # started at off (global trajectory index keys the generator)
    sub = orc.sample(lat, n0, seed=11, M=3, traj_offset=5)
    assert np.array_equal(sub, rho[5:8])


def test_sample_moments_match_appendix_covariance(orc):
    """cov(rho*_ab, rho_ab) = (n_a + n_b - 2 n_a n_b)/2 (Appendix A.3); mean 0,
    E rho_ab^2 = 0, |xi|^2 ~ Exp(1), arg xi uniform.  Checked also for
    fractional (thermal) occupations, where the amplitude is not 1/sqrt(2)."""
    N = 4
    lat = orc.Lattice.from_bonds(N, [(0, 1), (1, 2), (2, 3), (3, 0)], [0, 1, 0, 1])
    n0 = np.array([[1.0, 0.0, 0.3, 0.75], [0.0, 1.0, 0.6, 0.1]])
    M = 40000
    rho = orc.sample(lat, n0, seed=123, M=M)
    for s in range(2):
        for a in range(N):
            for b in range(a + 1, N):
                v = rho[:, s, a, b]
                var = 0.5 * (n0[s, a] + n0[s, b] - 2 * n0[s, a] * n0[s, b])
                if var == 0:
                    assert np.all(v == 0)
                    continue
                se = np.sqrt(var / M)
                assert abs(v.mean()) < 5 * se * np.sqrt(2)
                e2 = np.mean(np.abs(v) ** 2)
                assert abs(e2 - var) < 5 * var * np.sqrt(1.0 / M) * 1.5
                assert abs(np.mean(v * v)) < 5 * var * np.sqrt(2.0 / M)
                xi2 = np.abs(v) ** 2 / var
                assert sst.kstest(xi2, "expon").pvalue > 1e-4
                assert sst.kstest((np.angle(v) + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-4


def test_thermal_sample_diagonal_matches_appendix_covariance(orc):
    """Thermal (non-integer) initial state: the Appendix A.3 covariance at
    alpha = beta = mu = nu = i is n_i (1 - n_i), so rho_ii fluctuates about
    n_i - 1/2 with that variance, as a Gaussian, uncorrelated with the other
    diagonal entries and with the off-diagonal elements; the off-diagonal
    elements are those of the plain sampler (same counters)."""
    N = 4
    lat = orc.Lattice.from_bonds(N, [(0, 1), (1, 2), (2, 3), (3, 0)], [0, 1, 0, 1])
    n0 = np.array([[1.0, 0.0, 0.3, 0.75], [0.5, 1.0, 0.6, 0.1]])
    M = 40000
    rho = orc.sample(lat, n0, seed=321, M=M, thermal=True)
    plain = orc.sample(lat, n0, seed=321, M=M)
    off = ~np.eye(N, dtype=bool)
    assert np.array_equal(rho[:, :, off], plain[:, :, off])
    for s in range(2):
        d = rho[:, s, np.arange(N), np.arange(N)]
        assert np.all(d.imag == 0)
        for i in range(N):
            var = n0[s, i] * (1 - n0[s, i])
            x = d[:, i].real - (n0[s, i] - 0.5)
            if var == 0:   # integer occupation: the plain, deterministic diagonal
                assert np.all(x == 0)
                continue
            assert abs(x.mean()) < 5 * np.sqrt(var / M)
            assert abs(np.mean(x * x) - var) < 5 * var * np.sqrt(2.0 / M)
            assert sst.kstest(x / np.sqrt(var), "norm").pvalue > 1e-4
            # independent of the other diagonal entries and of the off-diagonal
            for k in range(N):
                if k != i and n0[s, k] * (1 - n0[s, k]) > 0:
                    y = d[:, k].real - (n0[s, k] - 0.5)
                    assert abs(np.mean(x * y)) < 5 * np.sqrt(var * n0[s, k] * (1 - n0[s, k]) / M)
            v = rho[:, s, 0, 2]
            assert abs(np.mean(x * v)) < 5 * np.sqrt(var * np.mean(np.abs(v) ** 2) / M) + 1e-12
    # one draw by hand: the counter (i, instance << 1 | s, m, 2) of the definition
    g = orc.real_normal(321, 2, (0 << 1) | 1, 7, 2)
    assert rho[7, 1, 2, 2].real == (n0[1, 2] - 0.5) + np.sqrt(n0[1, 2] * (1 - n0[1, 2])) * g


def test_real_normal_is_box_muller_of_the_philox_draw(orc):
    """g = sqrt(-2 ln u1) cos(2 pi u2) with u1 = (a+1) 2^-53, u2 = b 2^-53 and
    (a, b) the two 53-bit halves of the Philox4x32-10 block, checked against
    the block computed by the known-answer-tested Philox."""
    seed, ctr = 0x1234_5678_9abc_def0, (5, 3, 11, 2)
    x = orc.philox4x32_10(ctr, ((seed & 0xffffffff), seed >> 32))
    a = (int(x[0]) << 21) | (int(x[1]) >> 11)
    b = (int(x[2]) << 21) | (int(x[3]) >> 11)
    u1 = (a + 1) * 2.0 ** -53
    u2 = b * 2.0 ** -53
    want = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    assert abs(orc.real_normal(seed, *ctr) - want) <= 4e-16 * max(1.0, abs(want))


# ---------------------------------------------------------------------------
# Equation of motion, Eq. (6)
# ---------------------------------------------------------------------------
def _ring(N, t=1.0):
    return [(i, (i + 1) % N) for i in range(N)], [i % 2 for i in range(N)]


def test_rhs_worked_example(orc):
    """Appendix C.1: with site 1 (up) full, site 2 empty, rho_13 = rho_42 = 0,
    d rho_12,up/dt (0) = i j_12 - i u xi_12/sqrt(2)   (j = hopping, u = U).
    Sites 1..4 of the paper are 0..3 of a 4-ring with a Neel start."""
    bonds, sub = _ring(4)
    for t, U in [(1.0, 1.0), (0.7, 3.3), (1.3, -0.4)]:
        lat = orc.Lattice.from_bonds(4, bonds, sub, t=t)
        n0 = orc.fock_start(lat, "neel")
        rho = orc.sample(lat, n0, seed=99, M=1)[0]
        xi12 = rho[0, 0, 1] * np.sqrt(2)
        f = orc.rhs(lat, U, rho)
        assert abs(f[0, 0, 1] - (1j * t - 1j * U * xi12 / np.sqrt(2))) < 1e-14


def test_rhs_hermitian_and_real_diagonal(orc):
    lat = orc.Lattice("torus", 2, 3)
    n0 = orc.fock_start(lat, "random", seed=3)
    rho = orc.sample(lat, n0, seed=4, M=1)[0]
    f = orc.rhs(lat, 3.3, rho)
    for s in range(2):
        assert np.array_equal(f[s], f[s].conj().T)  # bitwise: f_ji = conj(f_ij)
        assert np.all(np.diag(f[s]).imag == 0)


def test_rhs_is_a_commutator_with_a_hermitian_generator(orc):
    """Eq. (6) equals i[rho, J] + i U [diag(rho_sbar), rho] in matrix form: the
    trace of f vanishes and f is anti-Hermitian-conjugate-symmetric; checked with
    random non-Hermitian input, where the stencil and the matrix product differ
    if an index is transposed."""
    lat = orc.Lattice("hex", 2, 0, t=0.8)
    rng = np.random.default_rng(1)
    N = lat.N
    rho = rng.normal(size=(2, N, N)) + 1j * rng.normal(size=(2, N, N))
    U = 2.1
    f = orc.rhs(lat, U, rho)
    J = lat.hopping_matrix()
    for s in range(2):
        D = np.diag(rho[1 - s].diagonal().real)
        want = 1j * (rho[s] @ J - J @ rho[s]) + 1j * U * (D @ rho[s] - rho[s] @ D)
        assert np.allclose(f[s], want, atol=1e-12)


# ---------------------------------------------------------------------------
# Runge-Kutta integration
# ---------------------------------------------------------------------------
def _rk4_free_propagator(J, rho0, dt, n):
    """U = 0: in J's eigenbasis each element is multiplied per step by the RK4
    stability polynomial P(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 at
    z = -i (lam_a - lam_b) dt (exact for the discrete map)."""
    lam, V = np.linalg.eigh(J)
    z = -1j * (lam[:, None] - lam[None, :]) * dt
    P = 1 + z + z**2 / 2 + z**3 / 6 + z**4 / 24
    out = np.empty_like(rho0)
    for s in range(2):
        t = V.T @ rho0[s] @ V
        out[s] = V @ (t * P**n) @ V.T
    return out


def test_free_fermions_exact_rk4_propagator(orc):
    lat = orc.Lattice("torus", 2, 3, t=1.0)
    n0 = orc.fock_start(lat, "neel")
    rho0 = orc.sample(lat, n0, seed=8, M=3)
    n = 300
    y, X, _ = orc.evolve(lat, 0.0, rho0, 0.01, n, record_every=100)
    J = lat.hopping_matrix()
    for m in range(3):
        want = _rk4_free_propagator(J, rho0[m], 0.01, n)
        assert np.max(np.abs(y[m] - want)) < 1e-12
        want_mid = _rk4_free_propagator(J, rho0[m], 0.01, 100)
        assert np.max(np.abs(X[1, m] - np.concatenate([want_mid[0].diagonal().real,
                                                        want_mid[1].diagonal().real]))) < 1e-12


def test_free_fermions_exponential_and_fourth_order(orc):
    """U = 0: rho(t) = e^{-iJt} rho(0) e^{iJt}; the RK4 error is within the
    truncation bound T (Delta lambda)^5 dt^4 / 120 and falls 16x when dt halves."""
    lat = orc.Lattice("torus", 2, 3)
    n0 = orc.fock_start(lat, "neel")
    rho0 = orc.sample(lat, n0, seed=9, M=1)
    T = 2.0
    J = lat.hopping_matrix()
    E = sla.expm(-1j * J * T)
    want = np.stack([E @ rho0[0, s] @ E.conj().T for s in range(2)])
    errs = []
    for dt in (0.04, 0.02):
        y, _, _ = orc.evolve(lat, 0.0, rho0, dt, int(round(T / dt)), record_every=1000)
        errs.append(np.max(np.abs(y[0] - want)))
    spread = np.ptp(np.linalg.eigvalsh(J))
    assert errs[1] < T * spread**5 * 0.02**4 / 120 * np.sqrt(lat.N)
    assert 12 < errs[0] / errs[1] < 20


def test_invariants(orc):
    """Trace is conserved to round-off (linear invariant of the commutator
    flow); rho stays Hermitian bitwise; the Weyl Hamiltonian H_W of Appendix A.3,
    Eq. (A10) and the Frobenius norm drift at O(dt^4) or faster (the norm of
    the RK4 stability polynomial on the imaginary axis deviates from 1 at
    sixth order per step, so that drift falls ~32x).  A sign error or a wrong
    spin index in the U term breaks energy conservation."""
    lat = orc.Lattice("torus", 2, 3)
    n0 = orc.fock_start(lat, "random", seed=2)
    rho0 = orc.sample(lat, n0, seed=5, M=2)
    drifts = []
    for dt in (0.04, 0.02):
        n = int(round(2.0 / dt))
        y, X, inv = orc.evolve(lat, 3.3, rho0, dt, n, record_every=n, want_inv=True)
        for m in range(2):
            for s in range(2):
                assert np.array_equal(y[m, s], y[m, s].conj().T)
        assert np.max(np.abs(inv[1, :, 0:2] - inv[0, :, 0:2])) < 1e-12 * lat.N
        drifts.append(np.max(np.abs(inv[1, :, 2:5] - inv[0, :, 2:5]), axis=0))
    ratio = drifts[0] / drifts[1]
    assert np.all(drifts[1] > 1e-11), drifts  # well above round-off
    assert np.all(ratio > 12) and np.all(ratio < 40), ratio


def test_energy_not_conserved_with_wrong_u_sign(orc):
    """Guard for the previous test: flipping the sign of U in the dynamics while
    measuring H_W with +U gives an O(1) energy drift, so the check has teeth."""
    lat = orc.Lattice("torus", 2, 3)
    n0 = orc.fock_start(lat, "random", seed=2)
    rho0 = orc.sample(lat, n0, seed=5, M=1)
    y, _, _ = orc.evolve(lat, -3.3, rho0, 0.02, 100, record_every=100)
    _, _, inv = orc.evolve(lat, 3.3, rho0, 0.02, 100, record_every=100, want_inv=True)
    J = lat.hopping_matrix()

    def hw(r):
        hop = sum(np.sum(J * r[s]).real for s in range(2))
        return -hop + 3.3 * np.sum((r[0].diagonal().real + 0.5) * (r[1].diagonal().real + 0.5))

    wrong = abs(hw(y[0]) - hw(rho0[0]))
    right = abs(inv[1, 0, 2] - hw(rho0[0]))
    assert wrong > 1e-3 and right < 1e-4 and wrong > 100 * right


def test_noise_free_trajectory_is_hartree_fock(orc):
    """Sec. III.A / Appendix A.2: with xi = 0 the fTWA trajectory is the
    Hartree-Fock solution of Eq. (A6), n_ij = rho_ij + delta_ij / 2.  The HF
    equations are integrated independently with an adaptive 8th-order method."""
    lat = orc.Lattice("hex", 2, 0)
    N = lat.N
    n0 = orc.fock_start(lat, "random", seed=7)
    rho0 = np.zeros((1, 2, N, N), dtype=complex)
    for s in range(2):
        rho0[0, s] = np.diag(n0[s] - 0.5)
    J = lat.hopping_matrix()
    U, T = 3.3, 2.0

    def hf(_t, v):
        n = v.reshape(2, N, N)
        out = np.empty_like(n)
        for s in range(2):
            # Eq. (A6): dn_ij/dt = i sum_l ( j_jl n_il - j_li n_lj + (u_il - u_lj) n_ll,sbar n_ij )
            nl = n[1 - s].diagonal()
            out[s] = 1j * (n[s] @ J.T - J.T @ n[s]) + 1j * U * (nl[:, None] - nl[None, :]) * n[s]
        return out.ravel()

    n_init = rho0[0] + 0.5 * np.eye(N)[None]
    sol = solve_ivp(hf, (0, T), n_init.ravel().astype(complex), method="DOP853",
                    rtol=1e-12, atol=1e-13)
    n_T = sol.y[:, -1].reshape(2, N, N)
    y, _, _ = orc.evolve(lat, U, rho0, 0.005, int(T / 0.005), record_every=1000)
    assert np.max(np.abs(y[0] + 0.5 * np.eye(N)[None] - n_T)) < 1e-8


# ---------------------------------------------------------------------------
# Ensemble statistics: moments, observables, Eq. (5) and Eq. (10)
# ---------------------------------------------------------------------------
def test_moments_against_matrix_products(orc):
    rng = np.random.default_rng(3)
    X = rng.normal(size=(3, 257, 10))
    S1, S2 = orc.moments(X)
    iu = np.triu_indices(10)
    for r in range(3):
        assert np.allclose(S1[r], X[r].sum(0), rtol=1e-13)
        assert np.allclose(S2[r], (X[r].T @ X[r])[iu], rtol=1e-12)


def test_observables_both_forms_of_g2(orc):
    """Eq. (10) written as a ratio of raw moments equals its second line, the
    mean of (rho_ii+1/2)(rho_jj+1/2) over the product of the means; n follows
    Eq. (5); C is the covariance of the diagonal variables."""
    rng = np.random.default_rng(4)
    N, M = 3, 500
    X = rng.uniform(-0.5, 0.5, size=(2, M, 2 * N))
    S1, S2 = orc.moments(X)
    n, C, g2 = orc.observables(N, M, S1, S2)
    for r in range(2):
        x = X[r]
        assert np.allclose(n[r], x.mean(0) + 0.5, atol=1e-14)
        assert np.allclose(C[r], np.cov(x.T, bias=True), atol=1e-13)
        p = x + 0.5
        want = (p.T @ p / M) / np.outer(p.mean(0), p.mean(0))
        assert np.allclose(g2[r], want, rtol=1e-12)


def test_free_fermion_ensemble_moments_are_exact(orc):
    """U = 0 is quadratic: the Gaussian phase-space ensemble reproduces the exact
    one-body density G(t) = e^{-iJt} n(0) e^{iJt} and, by Wick's theorem, the
    same-spin connected correlation -|G_ij|^2; opposite spins are uncorrelated.
    Statistical check within 5 standard errors."""
    lat = orc.Lattice("torus", 2, 3)
    N = lat.N
    n0 = orc.fock_start(lat, "neel")
    M, T, dt = 6000, 0.8, 0.01
    rho0 = orc.sample(lat, n0, seed=31, M=M)
    _, X, _ = orc.evolve(lat, 0.0, rho0, dt, int(round(T / dt)), record_every=int(round(T / dt)))
    x = X[1]
    J = lat.hopping_matrix()
    E = sla.expm(-1j * J * T)
    for s in range(2):
        G = E @ np.diag(n0[s]) @ E.conj().T
        nn = x[:, s * N:(s + 1) * N].mean(0) + 0.5
        se_n = x[:, s * N:(s + 1) * N].std(0) / np.sqrt(M)
        assert np.all(np.abs(nn - G.diagonal().real) < 5 * se_n + 1e-12)
    cov = np.cov(x.T, bias=True)
    dev = x - x.mean(0)
    for s in range(2):
        G = E @ np.diag(n0[s]) @ E.conj().T
        for i in range(N):
            for j in range(N):
                if i == j:
                    continue
                a, b = s * N + i, s * N + j
                se = np.std(dev[:, a] * dev[:, b]) / np.sqrt(M)
                assert abs(cov[a, b] + abs(G[i, j]) ** 2) < 5 * se + 1e-3
                c = (1 - s) * N + j
                se = np.std(dev[:, a] * dev[:, c]) / np.sqrt(M)
                assert abs(cov[a, c]) < 5 * se + 1e-3


def _antithetic(rho0):
    """Pairs (xi, -xi): the odd orders in the noise cancel exactly in means."""
    neg = rho0.copy()
    N = rho0.shape[-1]
    off = ~np.eye(N, dtype=bool)
    neg[:, :, off] *= -1
    return np.concatenate([rho0, neg])


def test_short_time_occupation_second_order(orc):
    """Appendix C.1-C.2, Eqs. (C3)-(C4) (with the sign of the epsilon^2 hopping
    term as printed there): E rho_11(eps) = 1/2 - sum_k j_1k^2 eps^2 for a full
    site with empty neighbours and E rho_22 = -1/2 + sum_k j_2k^2 eps^2 for an
    empty site with full neighbours, independent of U."""
    t = 0.9
    lat = orc.Lattice("torus", 2, 3, t=t)
    n0 = orc.fock_start(lat, "neel")
    rho0 = _antithetic(orc.sample(lat, n0, seed=77, M=400))
    for U in (0.0, 3.3):
        vals = []
        for eps in (0.02, 0.01):
            n = 4
            _, X, _ = orc.evolve(lat, U, rho0, eps / n, n, record_every=n)
            d = X[1].mean(0)[: lat.N] - X[0].mean(0)[: lat.N]
            vals.append(d / eps**2)
        rich = (4 * vals[1] - vals[0]) / 3  # removes the O(eps) remainder
        want = np.where(n0[0] == 1, -3 * t * t, 3 * t * t)
        assert np.allclose(rich, want, rtol=2e-2, atol=2e-2), (U, rich)


def test_short_time_g2_two_thirds(orc):
    """Appendix C.2, Eq. (C8): for an empty site 2 whose neighbours are all full,
    g2_{1 up, 2 up}(0+) = (sum_i j_2i^2 - j_12^2) / sum_i j_2i^2 = 2/3 with three
    neighbours (Sec. V, 198-site discussion)."""
    lat = orc.Lattice("torus", 2, 3)
    N = lat.N
    n0 = orc.fock_start(lat, "neel")  # up electrons on sublattice A
    rho0 = _antithetic(orc.sample(lat, n0, seed=5, M=3000))
    eps, n = 0.01, 2
    _, X, _ = orc.evolve(lat, 1.0, rho0, eps / n, n, record_every=n)
    S1, S2 = orc.moments(X)
    _, _, g2 = orc.observables(N, X.shape[1], S1, S2)
    vals = []
    for i in range(N):
        if n0[0, i] != 1:
            continue
        for j in lat.nbr[i, : lat.deg[i]]:
            vals.append(g2[1, i, j])
    assert abs(np.mean(vals) - 2.0 / 3.0) < 0.02, np.mean(vals)


def test_long_time_limits(orc):
    """Sec. IV.D and Appendix C.3, Eq. (C11) with Table I: at long times the
    occupations approach 1/2 (Sec. IV.B) and same-spin g2 between different
    sites approaches 2 C(n-2, n/2-2) / C(n-1, n/2-1) = (n-2)/(n-1) at half
    filling (10/11 for the 12-site torus).  Run at U = J as in the paper."""
    from math import comb
    lat = orc.Lattice("torus", 2, 3)
    N = lat.N
    n0 = orc.fock_start(lat, "neel")
    M = 800
    rho0 = orc.sample(lat, n0, seed=1, M=M)
    _, X, _ = orc.evolve(lat, 1.0, rho0, 0.02, 2500, record_every=250)
    S1, S2 = orc.moments(X)
    n, _, g2 = orc.observables(N, M, S1, S2)
    limit = 2 * comb(N - 2, N // 2 - 2) / comb(N - 1, N // 2 - 1)
    assert abs(limit - (N - 2) / (N - 1)) < 1e-15
    off = ~np.eye(N, dtype=bool)
    late = [g2[r][:N, :N][off].mean() for r in range(7, 11)]
    assert abs(np.mean(late) - limit) < 0.01
    assert np.all(np.abs(n[7:] - 0.5) < 0.06)

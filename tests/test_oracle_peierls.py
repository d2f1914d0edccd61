"""Pins of the oracle's complex (Peierls) hopping j_ik(tau) = t w_ik(tau) in
Eq. (6) (Sec. III: explicit time-dependent terms of the Hamiltonian enter the
equation of motion directly).  Pinned against the closed form of the
non-interacting flow, gauge covariance (static and time-dependent, the latter
against the on-site potential) and a reduction to real hopping; none of them
retypes the oracle's sums."""
import numpy as np
import scipy.linalg


def _random_rho(rng, N, M):
    a = rng.normal(size=(M, 2, N, N)) + 1j * rng.normal(size=(M, 2, N, N))
    return 0.5 * (a + np.conj(np.swapaxes(a, 2, 3)))


def _hop_table(lat, phase, n_half):
    """[n_half, N, 3] ratios w[h, i, n] = phase(h, i, k) for k = nbr[i, n]."""
    w = np.zeros((n_half, lat.N, 3), dtype=np.complex128)
    for i in range(lat.N):
        for n in range(lat.deg[i]):
            k = int(lat.nbr[i, n])
            for h in range(n_half):
                w[h, i, n] = phase(h, i, k)
    return w


def _random_flux_phase(rng, N):
    """Hermitian bond phases exp(i theta_ik), theta_ki = -theta_ik, random, so
    that every hexagon carries a flux (no gauge removes them)."""
    th = rng.uniform(-np.pi, np.pi, (N, N))
    th = np.triu(th, 1)
    th = th - th.T
    return th


def test_free_flow_closed_form(orc):
    """U = 0, static complex hopping J (Hermitian, random fluxes): the flow of
    Eq. (6) is rho' = i (rho J^T - J^T rho), solved by
    rho(T) = exp(-i J^T T) rho(0) exp(i J^T T) (scipy's expm).  Fourth-order
    convergence; the transposed hopping (J in place of J^T) misses by O(1)."""
    lat = orc.Lattice("hex", 2, 0, t=0.9)
    N = lat.N
    rng = np.random.default_rng(11)
    th = _random_flux_phase(rng, N)
    J = np.zeros((N, N), dtype=np.complex128)
    for i in range(N):
        for k in lat.nbr[i, :lat.deg[i]]:
            J[i, k] = lat.t * np.exp(1j * th[i, k])
    assert np.allclose(J, J.conj().T)
    rho0 = _random_rho(rng, N, 2)
    T = 1.0
    Ut = scipy.linalg.expm(-1j * J.T * T)
    exact = Ut @ rho0 @ Ut.conj().T
    Uw = scipy.linalg.expm(-1j * J * T)
    wrong = Uw @ rho0 @ Uw.conj().T
    errs = []
    for n in (50, 100):
        w = _hop_table(lat, lambda h, i, k: np.exp(1j * th[i, k]), 2 * n + 1)
        y, _, _ = orc.evolve(lat, 0.0, rho0, T / n, n, n, hop=w)
        errs.append(np.max(np.abs(y - exact)))
    assert errs[1] < 1e-6 and 12 < errs[0] / errs[1] < 20, errs
    assert np.max(np.abs(wrong - exact)) > 1e-1


def test_static_gauge_covariance(orc):
    """A pure gauge j'_ab = t conj(l_a) l_b (|l| = 1) on the interacting flow:
    the solution from rho'(0) = L rho(0) L^* is L rho(T) L^*, rho(T) the
    real-hopping solution (U != 0; equal up to rounding)."""
    lat = orc.Lattice("hex", 2, 0, t=1.0)
    N = lat.N
    rng = np.random.default_rng(12)
    chi = rng.uniform(-np.pi, np.pi, N)
    lam = np.exp(1j * chi)
    rho0 = _random_rho(rng, N, 2) * 0.3
    n = 40
    T = 0.6
    y, X, _ = orc.evolve(lat, 2.5, rho0, T / n, n, 10)
    L = np.diag(lam)
    rho0g = L @ rho0 @ L.conj().T
    w = _hop_table(lat, lambda h, i, k: np.conj(lam[i]) * lam[k], 2 * n + 1)
    yg, Xg, _ = orc.evolve(lat, 2.5, rho0g, T / n, n, 10, hop=w)
    assert np.max(np.abs(yg - L @ y @ L.conj().T)) < 1e-12
    assert np.max(np.abs(Xg - X)) < 1e-12
    # the opposite gauge (conj l_b l_a) is not a symmetry of this start
    wx = _hop_table(lat, lambda h, i, k: lam[i] * np.conj(lam[k]), 2 * n + 1)
    yx, _, _ = orc.evolve(lat, 2.5, rho0g, T / n, n, 10, hop=wx)
    assert np.max(np.abs(yx - L @ y @ L.conj().T)) > 1e-3


def test_time_dependent_gauge_equals_potential(orc):
    """A time-dependent gauge l_a(tau) = exp(i v_a B(tau)) makes the hopping
    j_ab = t exp(i (v_b - v_a) B(tau)) and adds the on-site potential
    V_a = v_a B'(tau): evolving rho'(0) = L(0) rho(0) L(0)^* under both gives
    L(T) rho(T) L(T)^*, rho the plain solution, up to the RK4 error (fourth
    order; the hop table and the envelope are both read at the half steps)."""
    lat = orc.Lattice("hex", 2, 0, t=1.0)
    N = lat.N
    rng = np.random.default_rng(13)
    v = rng.uniform(-1, 1, N)
    om, amp = 3.0, 0.8
    B = lambda tau: amp * np.sin(om * tau)
    A = lambda tau: amp * om * np.cos(om * tau)
    rho0 = _random_rho(rng, N, 2) * 0.3
    T = 1.0
    errs = []
    for n in (50, 100):
        dt = T / n
        y, _, _ = orc.evolve(lat, 2.0, rho0, dt, n, n)
        taus = 0.5 * dt * np.arange(2 * n + 1)
        w = _hop_table(lat, lambda h, i, k: np.exp(1j * (v[k] - v[i]) * B(taus[h])), 2 * n + 1)
        L0 = np.diag(np.exp(1j * v * B(0.0)))
        LT = np.diag(np.exp(1j * v * B(T)))
        yg, _, _ = orc.evolve(lat, 2.0, L0 @ rho0 @ L0.conj().T, dt, n, n, vsite=v,
                              env=A(taus), hop=w)
        errs.append(np.max(np.abs(yg - LT @ y @ LT.conj().T)))
    assert errs[1] < 1e-6 and 12 < errs[0] / errs[1] < 20, errs
    # without the potential the gauge is not compensated
    n = 100
    dt = T / n
    taus = 0.5 * dt * np.arange(2 * n + 1)
    w = _hop_table(lat, lambda h, i, k: np.exp(1j * (v[k] - v[i]) * B(taus[h])), 2 * n + 1)
    L0 = np.diag(np.exp(1j * v * B(0.0)))
    LT = np.diag(np.exp(1j * v * B(T)))
    y, _, _ = orc.evolve(lat, 2.0, rho0, dt, n, n)
    yn, _, _ = orc.evolve(lat, 2.0, L0 @ rho0 @ L0.conj().T, dt, n, n, hop=w)
    assert np.max(np.abs(yn - LT @ y @ LT.conj().T)) > 1e-2


def test_unit_ratios_reduce_to_real_hopping(orc):
    """w = 1 on every bond is the real-hopping equation: bitwise the plain
    oracle in both working precisions (1 * x and the zero imaginary part are
    exact in the complex product)."""
    lat = orc.Lattice("hex", 2, 0, t=1.0)
    rng = np.random.default_rng(14)
    rho0 = _random_rho(rng, lat.N, 2) * 0.3
    n = 12
    w = _hop_table(lat, lambda h, i, k: 1.0 + 0.0j, 2 * n + 1)
    for prec in ("f64", "f32"):
        y, X, _ = orc.evolve(lat, 1.7, rho0, 0.01, n, 4, precision=prec)
        yh, Xh, _ = orc.evolve(lat, 1.7, rho0, 0.01, n, 4, precision=prec, hop=w)
        assert np.array_equal(y, yh) and np.array_equal(X, Xh)

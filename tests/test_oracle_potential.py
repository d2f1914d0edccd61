"""Pins of the oracle's external on-site potential (the time-dependent term of
Eq. (6) that Sec. III describes for an external potential): the extra term
i (V_i(tau) - V_j(tau)) rho_ij with V_i(tau) = A(tau) v_i on both spins, the
envelope sampled at the Runge-Kutta stage times (t_n; t_n + h/2 twice;
t_n + h).  Pinned against closed forms and an independent integrator, not
against the oracle itself."""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _random_rho(rng, N, M):
    """M random Hermitian pairs of N x N blocks (not physical states: the
    equation is linear in rho at U = 0, which is all these pins use)."""
    a = rng.normal(size=(M, 2, N, N)) + 1j * rng.normal(size=(M, 2, N, N))
    return 0.5 * (a + np.conj(np.swapaxes(a, 2, 3)))


def _env(A, T, n_steps):
    h = T / n_steps
    return np.array([A(k * h / 2) for k in range(2 * n_steps + 1)])


def test_zero_hopping_phase_converges_at_fourth_order(orc):
    """t = 0, U = 0: every element evolves alone, rho_ij(T) = rho_ij(0)
    exp(i (v_i - v_j) int_0^T A); the RK4 error falls 16-fold per halving of
    h only when the stage times are t_n, t_n + h/2, t_n + h (a wrong sample
    or a sign error breaks it)."""
    lat = orc.Lattice("torus", 2, 3, t=0.0)
    N = lat.N
    rng = np.random.default_rng(1)
    rho0 = _random_rho(rng, N, 2)
    v = rng.uniform(-1, 1, N)
    A0, w, T = 2.0, 3.0, 2.0
    A = lambda tau: A0 * np.sin(w * tau)
    phase = A0 * (1 - np.cos(w * T)) / w
    exact = rho0 * np.exp(1j * (v[:, None] - v[None, :]) * phase)
    def errors(shift_mid):
        out = []
        for n in (40, 80, 160):
            env = _env(A, T, n)
            if shift_mid:  # the mid-step samples taken at t_n instead: a misplaced stage time
                env[1::2] = env[0:-1:2]
            y, _, _ = orc.evolve(lat, 0.0, rho0, T / n, n, n, vsite=v, env=env)
            out.append(np.max(np.abs(y - exact)))
        return out
    errs = errors(False)
    assert errs[0] < 1e-4
    for e0, e1 in zip(errs, errs[1:]):  # at least fourth order (this problem shows ~32)
        assert 13.0 < e0 / e1 < 40.0, errs
    bad = errors(True)
    assert bad[1] / bad[2] < 5.0 and bad[2] > 100 * errs[2], bad


def test_constant_potential_is_the_exact_conjugation(orc):
    """U = 0 with hopping and a constant envelope: rho(T) = e^{ihT} rho(0)
    e^{-ihT} with h = -J + diag(A v) (the sign of the potential relative to the
    hopping is fixed by this), within the RK4 truncation error."""
    from scipy.linalg import expm
    lat = orc.Lattice("hex", 2, 0)
    N = lat.N
    J = np.zeros((N, N))
    for i in range(N):
        for k in lat.nbr[i, :lat.deg[i]]:
            J[i, k] = lat.t
    rng = np.random.default_rng(2)
    rho0 = _random_rho(rng, N, 2)
    v = rng.uniform(-1, 1, N)
    A0, T, n = 0.7, 1.0, 400
    h1 = -J + np.diag(A0 * v)
    Uop = expm(1j * h1 * T)
    exact = Uop @ rho0 @ np.conj(Uop.T)
    y, _, _ = orc.evolve(lat, 0.0, rho0, T / n, n, n, vsite=v, env=np.full(2 * n + 1, A0))
    assert np.max(np.abs(y - exact)) < 1e-9
    # the opposite sign is far off
    Uneg = expm(1j * (-J - np.diag(A0 * v)) * T)
    assert np.max(np.abs(y - Uneg @ rho0 @ np.conj(Uneg.T))) > 1e-2


def test_pulse_with_hopping_matches_an_independent_integrator(orc):
    """U = 0, hopping and a Gaussian pulse: the oracle converges at fourth
    order to scipy's DOP853 solution of d rho/dt = i [h(t), rho]."""
    from scipy.integrate import solve_ivp
    lat = orc.Lattice("torus", 2, 3)
    N = lat.N
    J = np.zeros((N, N))
    for i in range(N):
        for k in lat.nbr[i, :lat.deg[i]]:
            J[i, k] = lat.t
    rng = np.random.default_rng(3)
    rho0 = _random_rho(rng, N, 1)
    v = np.array([(-1.0) ** s for s in lat.sub])  # staggered (sublattice) profile
    A = lambda tau: 1.5 * np.exp(-((tau - 1.0) / 0.3) ** 2) * np.cos(4.0 * tau)
    T = 2.0

    def f(tau, x):
        r = x.reshape(N, N)
        hh = -J + np.diag(A(tau) * v)
        return (1j * (hh @ r - r @ hh)).reshape(-1)
    ref = np.stack([solve_ivp(f, (0, T), rho0[0, s].reshape(-1).astype(complex), method="DOP853",
                              rtol=1e-12, atol=1e-13).y[:, -1].reshape(N, N) for s in range(2)])
    errs = []
    for n in (100, 200):
        y, _, _ = orc.evolve(lat, 0.0, rho0, T / n, n, n, vsite=v, env=_env(A, T, n))
        errs.append(np.max(np.abs(y[0] - ref)))
    assert errs[1] < 1e-6
    assert 12.0 < errs[0] / errs[1] < 20.0, errs


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_uniform_potential_changes_nothing(orc, precision):
    """V_i - V_j = 0 exactly for a uniform profile: bitwise the plain run (also
    at U != 0, where the U term shares the same factor a)."""
    lat = orc.Lattice("hex", 2, 0)
    n0 = orc.fock_start(lat, "random", 4)
    rho0 = orc.sample(lat, n0, 4, 3)
    n = 30
    y0, X0, _ = orc.evolve(lat, 3.3, rho0, 0.01, n, 10, precision=precision)
    y1, X1, _ = orc.evolve(lat, 3.3, rho0, 0.01, n, 10, precision=precision,
                           vsite=np.full(lat.N, 0.37), env=np.linspace(0, 2, 2 * n + 1))
    assert np.array_equal(y0, y1) and np.array_equal(X0, X1)

"""Pins of the oracle's general density-density interaction u_ij between
opposite spins (Eq. (1)); Eq. (6)'s own form then multiplies rho_ij by
sum_k (u_ki - u_kj)(rho_kk,sbar + 1/2).  Pinned against a closed form, a
conservation law and two reductions, not against the oracle itself."""
import numpy as np
import pytest


def _random_rho(rng, N, M):
    a = rng.normal(size=(M, 2, N, N)) + 1j * rng.normal(size=(M, 2, N, N))
    return 0.5 * (a + np.conj(np.swapaxes(a, 2, 3)))


def test_no_hopping_phase_uses_u_ki(orc):
    """t = 0: the diagonals are static and rho_ij,s(T) = rho_ij,s(0)
    exp(i (D_i - D_j) T), D_s = u^T (d_sbar + 1/2) computed here with numpy; a
    non-symmetric u makes the index order u_ki (not u_ik) visible.  Fourth-
    order convergence of the RK4 result."""
    lat = orc.Lattice("hex", 2, 0, t=0.0)
    N = lat.N
    rng = np.random.default_rng(5)
    rho0 = _random_rho(rng, N, 2)
    u = rng.uniform(0, 0.4, (N, N))  # not symmetric on purpose
    T = 1.0
    exact = np.empty_like(rho0)
    for m in range(2):
        for s in range(2):
            d = np.real(np.diagonal(rho0[m, 1 - s]))
            D = u.T @ (d + 0.5)
            exact[m, s] = rho0[m, s] * np.exp(1j * (D[:, None] - D[None, :]) * T)
    errs = []
    for n in (50, 100):
        y, _, _ = orc.evolve(lat, 0.0, rho0, T / n, n, n, umat=u)
        errs.append(np.max(np.abs(y - exact)))
    assert errs[1] < 1e-6 and 12 < errs[0] / errs[1] < 40, errs
    y_wrong = exact.copy()
    for m in range(2):
        for s in range(2):
            d = np.real(np.diagonal(rho0[m, 1 - s]))
            D = u @ (d + 0.5)
            y_wrong[m, s] = rho0[m, s] * np.exp(1j * (D[:, None] - D[None, :]) * T)
    assert np.max(np.abs(y_wrong - exact)) > 1e-2  # the transposed reading differs


def _weyl_energy(lat, u, rho):
    """H_W = -t sum_{ik in bonds, s} Re rho_ik,s + sum_ij u_ij (rho_ii,up + 1/2)(rho_jj,dn + 1/2)."""
    hop = 0.0
    for i in range(lat.N):
        for k in lat.nbr[i, :lat.deg[i]]:
            hop += np.real(rho[0, i, k] + rho[1, i, k])
    a = np.real(np.diagonal(rho[0])) + 0.5
    b = np.real(np.diagonal(rho[1])) + 0.5
    return -lat.t * hop + a @ u @ b


def test_weyl_energy_with_a_general_interaction_is_conserved(orc):
    """A symmetric long-range u with hopping conserves H_W (Appendix A.3's
    form with u_ij in place of U delta_ij) under the exact flow: the RK4 drift
    shrinks 16-fold per halving of dt (a dropped 1/2 or a wrong sign leaves an
    O(1) drift)."""
    lat = orc.Lattice("torus", 2, 3)
    N = lat.N
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, (N, N))
    u = 0.5 * (x + x.T) + np.diag(rng.uniform(2, 4, N))
    n0 = orc.fock_start(lat, "random", 3)
    rho0 = orc.sample(lat, n0, 3, 3)
    T = 2.0
    drifts = []
    for n in (100, 200):
        y, _, _ = orc.evolve(lat, 0.0, rho0, T / n, n, n, umat=u)
        drifts.append(max(abs(_weyl_energy(lat, u, y[m]) - _weyl_energy(lat, u, rho0[m]))
                          for m in range(3)))
    assert drifts[1] < 1e-6 and drifts[0] / drifts[1] > 12, drifts


def test_uniform_shift_of_u_changes_nothing(orc):
    """u_ij + c couples to the conserved particle number of the other spin: the
    same trajectories up to rounding."""
    lat = orc.Lattice("hex", 2, 0)
    N = lat.N
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, (N, N))
    u = 0.5 * (x + x.T)
    n0 = orc.fock_start(lat, "random", 5)
    rho0 = orc.sample(lat, n0, 5, 2)
    y0, _, _ = orc.evolve(lat, 0.0, rho0, 0.01, 50, 50, umat=u)
    y1, _, _ = orc.evolve(lat, 0.0, rho0, 0.01, 50, 50, umat=u + 0.8)
    assert np.max(np.abs(y0 - y1)) < 1e-10


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_on_site_u_reduces_to_the_hubbard_term(orc, precision):
    """u = U delta gives U (d_i - d_j) up to rounding (the 1/2 cancels)."""
    lat = orc.Lattice("torus", 2, 3)
    n0 = orc.fock_start(lat, "neel", 1)
    rho0 = orc.sample(lat, n0, 1, 3)
    y0, X0, _ = orc.evolve(lat, 3.3, rho0, 0.01, 40, 10, precision=precision)
    y1, X1, _ = orc.evolve(lat, 0.0, rho0, 0.01, 40, 10, precision=precision,
                           umat=3.3 * np.eye(lat.N))
    tol = 1e-12 if precision == "f64" else 1e-4
    assert np.max(np.abs(y0 - y1)) < tol

"""The paper's small-system comparison (Sec. IV.A-IV.C) on the GPU path: the
10-site cluster of two hexagons at half filling, U = J = 1, from the Fock
state of largest ground-state overlap (Appendix B.2; the Neel state, checked
on the CPU in test_oracle_ed.py), 10^5 trajectories to t = 5 as in the paper.

Three curves, as in the paper's figures of n_11 and n_55 and of g2:
  * fTWA: the library's sampling, Eq. (6) with RK4 and FP64 moments;
  * Hartree-Fock: the same kernels run on the one noise-free trajectory
    (xi = 0 in Eq. (7), Sec. III.A);
  * exact diagonalisation: oracle/exact.py (Eq. (8), Appendix B.1).
Checks (Sec. IV.B-IV.C): Hartree-Fock leaves ED (occupation error above
0.02) at t ~ 1 and fTWA about three times later; fTWA follows ED's
neighbour g2 until t ~ 2, starting near the short-time value 1/2 of
Eq. (C7).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 0x2212043520000006
U, DT, STEPS, REC = 1.0, 0.01, 500, 10
M = 100_000


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


@pytest.fixture(scope="module")
def curves(ft):
    import torch
    from oracle import exact

    lat = ft.Lattice("armchair", 2, 5)
    N = lat.N
    assert N == 10 and lat.n_bonds == 11
    n0 = lat.fock_start("neel")

    prob = ft.Problem.allocate(lat, U, M, n0, "f64")
    ft.sample(prob, SEED)
    ft.evolve(prob, DT, STEPS, REC)
    n_tw, _, g2_tw = ft.observables(prob)

    # Hartree-Fock: one trajectory holding the noise-free start
    hf = ft.Problem.allocate(lat, U, 1, n0, "f64")
    hf.rho.zero_()
    for s in range(2):
        for i in range(N):
            hf.rho[s, i * N - i * (i - 1) // 2, 0] = float(n0[s][i]) - 0.5
    ft.evolve(hf, DT, STEPS, REC)
    n_hf, _, _ = ft.observables(hf)
    torch.cuda.synchronize()

    J = np.zeros((N, N))
    for i in range(N):
        for k in lat.nbr[i][: lat.deg[i]]:
            J[i, k] = 1.0
    ed = exact.HubbardED(J, exact.hubbard_onsite(J, U), 5, 5)
    times = np.arange(STEPS // REC + 1) * DT * REC
    n_ed, nn_ed = ed.densities(ed.evolve(ed.fock_vector(np.asarray(n0)), times))
    with np.errstate(divide="ignore", invalid="ignore"):
        g2_ed = nn_ed / (n_ed[:, :, None] * n_ed[:, None, :])
    return dict(lat=lat, n0=np.asarray(n0), times=times, n_tw=n_tw.cpu().numpy(),
                g2_tw=g2_tw.cpu().numpy(), n_hf=n_hf.cpu().numpy(), n_ed=n_ed, g2_ed=g2_ed)


def _leaves(times, err, eps):
    idx = np.flatnonzero(err > eps)
    return times[idx[0]] if len(idx) else np.inf


def test_occupations_fTWA_follows_ed_three_times_longer_than_hf(curves):
    c = curves
    t = c["times"]
    e_tw = np.abs(c["n_tw"] - c["n_ed"]).max(axis=1)
    e_hf = np.abs(c["n_hf"] - c["n_ed"]).max(axis=1)
    t_tw, t_hf = _leaves(t, e_tw, 0.02), _leaves(t, e_hf, 0.02)
    print(f"\noccupation error > 0.02 first at: Hartree-Fock t = {t_hf:.2f}, fTWA t = {t_tw:.2f}")
    for tt in (0.5, 1.0, 2.0, 3.0, 4.0, 5.0):
        k = int(round(tt / (DT * REC)))
        print(f"  t = {tt:3.1f}: max|dn| fTWA {e_tw[k]:.4f}  HF {e_hf[k]:.4f}")
    assert 0.7 <= t_hf <= 1.3, t_hf
    assert t_tw >= 2.2, t_tw
    assert t_tw >= 2.0 * t_hf
    # both start exactly at the Fock occupations
    assert np.array_equal(c["n_tw"][0], c["n0"].reshape(-1))
    assert np.array_equal(c["n_hf"][0], c["n0"].reshape(-1))


def test_neighbour_g2_follows_ed_until_t2(curves):
    """Same-spin g2 between a full site i and its empty neighbour j of two
    neighbours: near Eq. (C7)'s 1/2 at short times and on ED's curve to
    t = 2 (Sec. IV.C: fTWA and ED agree until about t = 2)."""
    c = curves
    lat, n0, t = c["lat"], c["n0"], c["times"]
    pairs = [(i, int(j)) for i in range(lat.N) for j in lat.nbr[i][: lat.deg[i]]
             if n0[0, i] == 1 and n0[0, j] == 0 and lat.deg[j] == 2]
    assert len(pairs) >= 4
    k1 = int(round(0.1 / (DT * REC)))
    k2 = int(round(2.0 / (DT * REC)))
    for i, j in pairs:
        g_tw, g_ed = c["g2_tw"][:, i, j], c["g2_ed"][:, i, j]
        print(f"pair ({i},{j}): g2 fTWA/ED at t=0.1: {g_tw[k1]:.3f}/{g_ed[k1]:.3f}, "
              f"t=2: {g_tw[k2]:.3f}/{g_ed[k2]:.3f}")
        assert abs(g_tw[k1] - 0.5) < 0.05
        assert np.max(np.abs(g_tw[2:k2 + 1] - g_ed[2:k2 + 1])) < 0.03


def test_distant_g2_follows_ed_until_t2(curves):
    """g2 of the two initially full same-spin sites farthest apart (graph
    distance) leaves 1
    only once a correlation front has crossed (Sec. IV.C) and fTWA follows
    ED until t = 2."""
    c = curves
    lat, t = c["lat"], c["times"]
    N = lat.N
    dist = np.full((N, N), 99)
    for a in range(N):
        dist[a, a] = 0
        frontier = [a]
        while frontier:
            nxt = []
            for u in frontier:
                for v in lat.nbr[u][: lat.deg[u]]:
                    if dist[a, v] == 99:
                        dist[a, v] = dist[a, u] + 1
                        nxt.append(int(v))
            frontier = nxt
    full = c["n0"][0] == 1  # up electrons at t = 0: denominators near 1
    dist = np.where(np.outer(full, full), dist, -1)
    i, j = np.unravel_index(np.argmax(dist), dist.shape)
    k2 = int(round(2.0 / (DT * REC)))
    g_tw, g_ed = c["g2_tw"][:, i, j], c["g2_ed"][:, i, j]
    print(f"distant pair ({i},{j}) distance {dist[i, j]}: g2 fTWA/ED at t=2 {g_tw[k2]:.3f}/{g_ed[k2]:.3f}")
    assert abs(g_tw[1] - 1.0) < 0.01 and abs(g_ed[1] - 1.0) < 1e-3
    assert np.max(np.abs(g_tw[1:k2 + 1] - g_ed[1:k2 + 1])) < 0.05

"""GPU invariant monitors (trace, Weyl energy, Frobenius norm; non-finite
trajectories) against the oracle's per-trajectory invariants.

The device computes the per-trajectory sums in FP64 in another order than the
oracle, so the reported maxima agree to the rounding of sums of 2P terms
(P = N(N+1)/2): tolerance 4 sqrt(2P) eps64 times the largest invariant value.
The cases use a coarse step (dt = 0.05) so that the RK4 truncation error makes
the energy and norm drift visible far above that tolerance in FP64 too; in
FP32 the rounding drift dominates.
"""
import numpy as np
import pytest

from tests._util import pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


def _expected(inv_ref):
    """Maxima over trajectories of the drifts from record 0 (oracle layout
    [n_rec][M][tr_up, tr_dn, H_W, frob_up, frob_dn])."""
    d = np.abs(inv_ref - inv_ref[:1])
    return np.stack([np.max(d[:, :, 0:2], axis=(1, 2)), np.max(d[:, :, 2], axis=1),
                     np.max(d[:, :, 3:5], axis=(1, 2))], axis=1)


def _run(ft, orc, kind, a, b, U, M, steps, dt, re, dtype, path, seed=5):
    import torch
    olat = orc.Lattice(kind, a, b)
    n0 = orc.fock_start(olat, "random", seed)
    rho0 = orc.sample(olat, n0, seed, M)
    lat = ft.Lattice(kind, a, b)
    prob = ft.Problem.allocate(lat, U, M, n0, dtype, track_invariants=True)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    ft.evolve(prob, dt, steps, re, path=path)
    torch.cuda.synchronize()
    _, _, inv_ref = orc.evolve(olat, U, rho0, dt, steps, re, precision=dtype, want_inv=True)
    P = lat.N * (lat.N + 1) // 2
    tol = 4 * np.sqrt(2 * P) * np.finfo(np.float64).eps * max(1.0, np.max(np.abs(inv_ref[0])))
    return prob.inv.cpu().numpy(), _expected(inv_ref), tol


@pytest.mark.parametrize("path", ["stream", "resident"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind,a,b,U,M,steps", [
    ("torus", 2, 3, 3.3, 130, 200),   # 12 sites, ragged trajectory count
    ("hex", 2, 0, 1.7, 33, 60),       # degree-2 edge sites
])
def test_invariants_match_oracle(ft, orc, path, dtype, kind, a, b, U, M, steps):
    got, exp, tol = _run(ft, orc, kind, a, b, U, M, steps, 0.05, 10, dtype, path)
    assert got.shape == (exp.shape[0], 4)
    assert np.all(got[:, 3] == 0)
    assert np.all(got[0, :3] == 0)
    assert np.allclose(got[:, :3], exp, rtol=0, atol=tol), np.max(np.abs(got[:, :3] - exp))
    # the coarse step makes the drift visible: the check is not vacuous
    assert np.max(exp[:, 1]) > 1e3 * tol


def test_invariants_flake198_spin_split(ft, orc):
    got, exp, tol = _run(ft, orc, "armchair", 10, 20, 3.3, 6, 16, 0.01, 4, "f32", "resident")
    assert np.all(got[:, 3] == 0)
    assert np.allclose(got[:, :3], exp, rtol=0, atol=tol), np.max(np.abs(got[:, :3] - exp))
    assert np.max(exp) > 1e3 * tol


def test_invariants_fp64_flake198_take_the_stream_path(ft, orc):
    """The split resident kernel (FP64 at 198 sites) keeps no per-trajectory
    invariant sums: with monitors the automatic path is the stream path, and
    forcing the resident path is refused."""
    got, exp, tol = _run(ft, orc, "armchair", 10, 20, 3.3, 4, 8, 0.01, 4, "f64", "auto")
    assert np.all(got[:, 3] == 0)
    assert np.allclose(got[:, :3], exp, rtol=0, atol=tol), np.max(np.abs(got[:, :3] - exp))
    lat = ft.Lattice("armchair", 10, 20)
    prob = ft.Problem.allocate(lat, 3.3, 2, lat.fock_start("neel"), "f64", track_invariants=True)
    ft.sample(prob, 1)
    with pytest.raises(ft.FtwaError):
        ft.evolve(prob, 0.01, 1, 1, path="resident")


@pytest.mark.parametrize("path", ["stream", "resident"])
def test_non_finite_trajectory_is_reported(ft, path):
    """A NaN planted in one trajectory's rho(0) stays in that trajectory: the
    run reports FTWA_ENONFINITE and inv counts exactly one trajectory per record;
    the drifts of the other trajectories are still finite."""
    import torch
    lat = ft.Lattice("torus", 2, 3)
    prob = ft.Problem.allocate(lat, 3.3, 40, lat.fock_start("neel"), "f32",
                               track_invariants=True)
    ft.sample(prob, 9)
    prob.rho[0, 0, 3] = complex(float("nan"), 0.0)
    with pytest.raises(ft.FtwaError) as e:
        ft.evolve(prob, 0.01, 20, 5, path=path)
    assert e.value.status == -5
    torch.cuda.synchronize()
    inv = prob.inv.cpu().numpy()
    assert np.all(inv[:, 3] == 1)
    assert np.all(np.isfinite(inv[:, :3]))

"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Tolerances: integer work (lattices, Fock starts, Philox words) is bit-exact;
the FP64 and FP32 time evolutions follow the same operation order as the
oracle and are required to match it exactly (bitwise on rho); sampled rho(0)
differs only through the device's log/cos/sin (a few ulp); FP64 moments and
observables match to 1e-12 relative (summation order differs).
"""
import numpy as np
import pytest

from tests._util import pack, unpack, unpack_s2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


def _problem(ft, kind, a, b, U, M, start="neel", seed=1, dtype="f64", traj_offset=0, t=1.0):
    lat = ft.Lattice(kind, a, b, t)
    n0 = lat.fock_start(start, seed)
    return lat, n0, ft.Problem.allocate(lat, U, M, n0, dtype, traj_offset=traj_offset)


def _to_host(x):
    import torch
    torch.cuda.synchronize()
    return x.detach().cpu().numpy()


@pytest.mark.parametrize("kind,a,b,M,start,off", [("torus", 2, 3, 300, "neel", 0),
                                                 ("torus", 3, 9, 65, "random", 7),
                                                 ("armchair", 10, 20, 17, "neel", 1000)])
def test_sample_matches_oracle(ft, orc, kind, a, b, M, start, off):
    seed = 0x2212043520000001
    lat, n0, prob = _problem(ft, kind, a, b, 3.3, M, start, seed, traj_offset=off)
    ft.sample(prob, seed)
    got = unpack(_to_host(prob.rho), lat.N)
    ref = orc.sample(orc.Lattice(kind, a, b), n0, seed, M, traj_offset=off)
    # exact zero pattern and exact diagonal; off-diagonal within a few ulp
    assert np.array_equal(got == 0, ref == 0)
    assert np.array_equal(np.diagonal(got, axis1=2, axis2=3), np.diagonal(ref, axis1=2, axis2=3))
    assert np.max(np.abs(got - ref)) <= 8 * np.finfo(np.float64).eps * np.max(np.abs(ref))
    # FP32 storage is the FP64 value rounded once
    _, _, p32 = _problem(ft, kind, a, b, 3.3, M, start, seed, dtype="f32", traj_offset=off)
    ft.sample(p32, seed)
    got32 = unpack(_to_host(p32.rho), lat.N)
    assert np.max(np.abs(got32 - ref.astype(np.complex64))) <= 2 * np.finfo(np.float32).eps * 8


@pytest.mark.parametrize("kind,a,b,M,off", [("torus", 3, 9, 65, 7), ("armchair", 10, 20, 9, 300)])
def test_thermal_sample_matches_oracle(ft, orc, kind, a, b, M, off):
    """ftwa_sample_thermal (fractional occupations, diagonal fluctuations of
    the Appendix A.3 covariance) against the oracle: the off-diagonal part
    equals the plain sampler's, the diagonal within a few ulp (device
    log/cos), zeros where n is 0 or 1; then the trajectories evolve like the
    oracle's from the oracle's samples."""
    import torch
    seed = 0x2212043520000077
    lat = ft.Lattice(kind, a, b)
    N = lat.N
    rng = np.random.default_rng(5)
    n0 = np.clip(rng.uniform(-0.2, 1.2, size=(2, N)), 0.0, 1.0)  # some exactly 0 or 1
    prob = ft.Problem.allocate(lat, 3.3, M, n0, "f64", traj_offset=off)
    ft.sample(prob, seed, thermal=True)
    got = unpack(_to_host(prob.rho), lat.N)
    ref = orc.sample(orc.Lattice(kind, a, b), n0, seed, M, traj_offset=off, thermal=True)
    assert np.array_equal(got == 0, ref == 0)
    assert np.max(np.abs(got - ref)) <= 8 * np.finfo(np.float64).eps * np.max(np.abs(ref))
    plain = ft.Problem.allocate(lat, 3.3, M, n0, "f64", traj_offset=off)
    ft.sample(plain, seed)
    p = unpack(_to_host(plain.rho), lat.N)
    off_diag = ~np.eye(N, dtype=bool)
    assert np.array_equal(got[:, :, off_diag], p[:, :, off_diag])
    integer = (n0 == 0) | (n0 == 1)
    d_got = np.diagonal(got, axis1=2, axis2=3).real
    assert np.array_equal(d_got[:, integer], np.broadcast_to(n0 - 0.5, d_got.shape)[:, integer])
    # evolution from the oracle's thermal samples (resident FP32 path), bitwise
    p32 = ft.Problem.allocate(lat, 3.3, M, n0, "f32")
    p32.rho.copy_(torch.from_numpy(pack(ref.astype(np.complex64))))
    ft.evolve(p32, 0.01, 10, 5)
    y_ref, _, _ = orc.evolve(orc.Lattice(kind, a, b), 3.3, ref, 0.01, 10, 5, precision="f32")
    assert np.array_equal(unpack(_to_host(p32.rho), lat.N), y_ref.astype(np.complex64))


def _evolve_parity(ft, orc, kind, a, b, U, M, n_steps, dt, re, dtype, start="random", seed=3,
                   chunk=0, path="stream"):
    import torch
    olat = orc.Lattice(kind, a, b)
    n0 = orc.fock_start(olat, start, seed)
    rho0 = orc.sample(olat, n0, seed, M)
    lat = ft.Lattice(kind, a, b)
    prob = ft.Problem.allocate(lat, U, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    ft.evolve(prob, dt, n_steps, re, path=path, traj_chunk=chunk)
    y_ref, X_ref, _ = orc.evolve(olat, U, rho0, dt, n_steps, re, precision=dtype)
    got = unpack(_to_host(prob.rho), lat.N)
    S1, S2 = _to_host(prob.S1), _to_host(prob.S2)
    return got, y_ref.astype(cdt), S1, S2, X_ref


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind,a,b,U,M,steps,chunk", [
    ("torus", 2, 3, 3.3, 130, 200, 0),       # 12 sites, ragged trajectory count
    ("torus", 2, 3, 0.0, 64, 50, 0),         # free fermions
    ("torus", 3, 9, 3.3, 70, 60, 32),        # 54 sites, several chunks with a ragged tail
    ("hex", 2, 0, 1.7, 33, 40, 0),           # degree-2 edge sites
    ("armchair", 10, 20, 3.3, 20, 12, 0),    # 198-site flake
])
def test_evolve_stream_matches_oracle_bitwise(ft, orc, dtype, kind, a, b, U, M, steps, chunk):
    got, ref, S1, S2, X = _evolve_parity(ft, orc, kind, a, b, U, M, steps, 0.01, 10, dtype,
                                         chunk=chunk)
    assert np.array_equal(got, ref), np.max(np.abs(got - ref))
    S1r, S2r = orc.moments(X)
    assert np.allclose(S1, S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(S2, S2r, rtol=1e-12, atol=1e-12)


def test_observables_match_oracle(ft, orc):
    import torch
    got, ref, S1, S2, X = _evolve_parity(ft, orc, "torus", 2, 3, 3.3, 200, 100, 0.01, 10, "f64")
    S1r, S2r = orc.moments(X)
    N = 12
    n_r, C_r, g2_r = orc.observables(N, 200, S1r, S2r)
    D = 2 * N
    n = torch.empty((S1.shape[0], D), dtype=torch.float64, device="cuda")
    C = torch.empty((S1.shape[0], D, D), dtype=torch.float64, device="cuda")
    g2 = torch.empty_like(C)
    ft.ftwa_observables(N, 200, S1.shape[0], torch.from_numpy(S1).cuda(),
                        torch.from_numpy(S2).cuda(), n, C, g2)
    assert np.allclose(_to_host(n), n_r, rtol=0, atol=1e-13)
    assert np.allclose(_to_host(C), C_r, rtol=0, atol=1e-12)
    # g2 is 0/0 on sites a Fock start leaves empty: NaN on both sides
    assert np.allclose(_to_host(g2), g2_r, rtol=1e-11, atol=1e-12, equal_nan=True)
    assert np.allclose(unpack_s2(S2, D), unpack_s2(S2r, D), rtol=1e-12, atol=1e-13)


def test_full_pipeline_small_torus(ft, orc):
    """GPU sample -> evolve -> observables against the oracle's own pipeline on
    the 12-site torus workload (Neel start, U/t = 3.3, dt = 0.01 to T = 10,
    256 of its trajectories).  rho(0) differs by a few ulp (device
    log/cos/sin), which the dynamics amplifies by at most ~1e4 at this size."""
    import torch
    from workloads import SMALL_TORUS as W
    M = 256
    lat, n0, prob = _problem(ft, W.kind, W.a, W.b, W.U, M, W.start, W.seed)
    ft.sample(prob, W.seed)
    ft.evolve(prob, W.dt, W.n_steps, W.record_every)
    n, C, g2 = ft.observables(prob)
    olat = orc.Lattice(W.kind, W.a, W.b)
    rho0 = orc.sample(olat, n0, W.seed, M)
    _, X, _ = orc.evolve(olat, W.U, rho0, W.dt, W.n_steps, W.record_every)
    S1r, S2r = orc.moments(X)
    n_r, C_r, g2_r = orc.observables(lat.N, M, S1r, S2r)
    assert np.max(np.abs(_to_host(n) - n_r)) < 1e-9
    assert np.max(np.abs(_to_host(C) - C_r)) < 1e-9
    assert np.array_equal(np.isnan(_to_host(g2)), np.isnan(g2_r))
    assert np.nanmax(np.abs(_to_host(g2) - g2_r)) < 1e-8
    del torch


def test_errors_are_reported(ft):
    import torch
    lat, n0, prob = _problem(ft, "torus", 2, 3, 1.0, 4)
    ft.sample(prob, 1)
    d = prob.desc()
    d["S1"] = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtwaError):
        ft.ftwa_evolve([d], 0.01, 10, 0, "f64", None)  # record_every < 1
    with pytest.raises(ft.FtwaError):
        ft.ftwa_evolve([d], 0.01, 10, 1, "f64", None)  # workspace missing


# ----------------------------------------------------------------- resident path
@pytest.mark.parametrize("dtype,kind,a,b,U,M,steps,config,t", [
    ("f64", "torus", 2, 3, 3.3, 130, 200, -1, 1.0),    # one 64-thread unit per workgroup
    ("f32", "torus", 2, 3, 3.3, 130, 200, -1, 1.0),
    ("f64", "torus", 2, 3, 3.3, 130, 200, 0, 1.0),     # 16 trajectories per workgroup, ragged
    ("f32", "torus", 2, 3, 3.3, 130, 200, 4, 1.0),
    ("f64", "torus", 2, 3, 3.3, 130, 40, 25, 1.0),     # 8, 4 and 2 units per workgroup
    ("f32", "torus", 2, 3, 3.3, 130, 40, 26, 1.0),
    ("f64", "torus", 2, 3, 3.3, 130, 40, 27, 1.0),
    ("f32", "torus", 2, 3, 3.3, 130, 40, 28, 1.0),
    ("f64", "torus", 2, 3, 3.3, 130, 40, 29, 1.0),
    ("f32", "torus", 2, 3, 3.3, 130, 40, 30, 1.0),
    ("f64", "hex", 2, 0, 1.7, 33, 40, 1, 1.0),         # 128 x 8 tiles, ragged
    ("f32", "hex", 2, 0, 1.7, 33, 40, 5, 1.0),
    ("f64", "torus", 3, 9, 3.3, 70, 60, 35, 1.0),      # 384 x 1 (FP64), 256 x 4 (FP32)
    ("f32", "torus", 3, 9, 3.3, 70, 60, 17, 1.0),
    ("f64", "hex", 2, 0, 1.7, 33, 40, -1, 1.0),        # degree-2 edge sites
    ("f32", "hex", 2, 0, 1.7, 33, 40, -1, 1.0),
    ("f64", "torus", 3, 9, 3.3, 70, 60, -1, 1.0),      # 54 sites
    ("f32", "torus", 3, 9, 3.3, 70, 60, -1, 1.0),
    ("f64", "hex", 4, 0, 2.0, 10, 20, -1, 1.0),        # 96 sites, one trajectory per workgroup
    ("f32", "hex", 4, 0, 2.0, 10, 20, -1, 1.0),
    ("f32", "hex", 5, 0, 3.3, 9, 20, -1, 1.0),         # 150 sites: spin-split workgroup pairs
    ("f32", "armchair", 10, 20, 3.3, 12, 12, -1, 1.0),  # 198-site flake, spin split
    ("f32", "armchair", 10, 20, 3.3, 12, 12, 10, 1.0),  # alternative tile: 1024 threads per spin
    ("f32", "armchair", 10, 20, 3.3, 12, 12, 11, 1.0),  # alternative tile: 512 threads per spin
    ("f32", "hex", 4, 0, 2.0, 10, 20, 9, 1.0),          # spin split with padding-heavy slots
    ("f32", "armchair", 10, 20, 3.3, 12, 12, 12, 1.0),  # spin split, every slot general
    ("f32", "torus", 3, 9, 3.3, 70, 60, 6, 1.0),        # shared-block tiles, every slot general
    ("f64", "hex", 4, 0, 2.0, 10, 20, 3, 1.0),
    ("f64", "torus", 3, 9, 3.3, 70, 60, 23, 1.0),       # FP64 384 x 2 tiles (one general slot,
    ("f64", "torus", 3, 9, 3.3, 70, 60, 24, 1.0),       # every slot general), ragged items
    ("f64", "torus", 2, 3, 3.3, 130, 200, -1, 0.6),     # hopping t != 1 (general kernels)
    ("f32", "hex", 2, 0, 1.7, 33, 40, -1, 1.3),
    ("f32", "armchair", 10, 20, 3.3, 12, 12, -1, 0.8),
])
def test_evolve_resident_matches_oracle_bitwise(ft, orc, dtype, kind, a, b, U, M, steps, config,
                                                 t):
    import torch
    olat = orc.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 3)
    rho0 = orc.sample(olat, n0, 3, M)
    lat = ft.Lattice(kind, a, b, t)
    prob = ft.Problem.allocate(lat, U, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    ft.evolve(prob, 0.01, steps, 10, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, U, rho0, 0.01, steps, 10, precision=dtype)
    got = unpack(_to_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_to_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_to_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


def test_resident_and_stream_paths_agree(ft):
    """Both paths follow the same per-element arithmetic: identical states."""
    import torch
    lat = ft.Lattice("torus", 3, 9)
    n0 = lat.fock_start("random", 11)
    out = {}
    for path in ("stream", "resident"):
        prob = ft.Problem.allocate(lat, 3.3, 300, n0, "f32")
        ft.sample(prob, 11)
        ft.evolve(prob, 0.01, 100, 10, path=path)
        out[path] = (_to_host(prob.rho), _to_host(prob.S1), _to_host(prob.S2))
    assert np.array_equal(out["stream"][0], out["resident"][0])
    assert np.allclose(out["stream"][1], out["resident"][1], rtol=1e-13, atol=1e-13)
    assert np.allclose(out["stream"][2], out["resident"][2], rtol=1e-13, atol=1e-13)
    del torch


def test_resident_rejects_unfit_configuration(ft):
    big = ft.Lattice("torus", 9, 14)  # 252 sites: no FP64 block or part of it fits the LDS
    prob = ft.Problem.allocate(big, 3.3, 2, big.fock_start("neel"), "f64")
    ft.sample(prob, 1)
    with pytest.raises(ft.FtwaError):
        ft.evolve(prob, 0.01, 2, 1, path="resident")
    lat = ft.Lattice("armchair", 10, 20)
    prob = ft.Problem.allocate(lat, 3.3, 4, lat.fock_start("neel"), "f64")
    ft.sample(prob, 1)
    with pytest.raises(ft.FtwaError):
        ft.evolve(prob, 0.01, 2, 1, path="resident", config=0)  # one CU per trajectory


def test_flake198_full_batch_sampled_trajectories(ft, orc):
    """The benchmark's launch configuration (198-site flake, 32768 trajectories,
    FP32, resident spin-split kernel, records every 10 steps) on a shortened
    horizon: four trajectories spread over the batch start from the oracle's
    rho(0) and must end bitwise equal to the oracle; the moments of the whole
    batch must match the oracle's moments of the GPU records' own statistics
    (trace conservation: sum over sites of n is N/2 per spin for every record)."""
    import torch
    from workloads import FLAKE_198 as W
    M, steps = W.n_traj, 40
    lat = ft.Lattice(W.kind, W.a, W.b)
    n0 = lat.fock_start(W.start, W.seed)
    prob = ft.Problem.allocate(lat, W.U, M, n0, "f32")
    ft.sample(prob, W.seed)
    olat = orc.Lattice(W.kind, W.a, W.b)
    picks = [0, 4097, 20000, M - 1]
    refs = []
    for m in picks:
        r0 = orc.sample(olat, n0, W.seed, 1, traj_offset=m)
        prob.rho[:, :, m].copy_(torch.from_numpy(pack(r0.astype(np.complex64))[:, :, 0]))
        refs.append(r0)
    ft.evolve(prob, W.dt, steps, W.record_every, path="resident")
    torch.cuda.synchronize()
    for m, r0 in zip(picks, refs):
        y_ref, _, _ = orc.evolve(olat, W.U, r0, W.dt, steps, W.record_every, precision="f32")
        got = unpack(prob.rho[:, :, m:m + 1].cpu().numpy(), lat.N)
        assert np.array_equal(got, y_ref.astype(np.complex64)), m
    n, _, _ = ft.observables(prob)
    n = _to_host(n)
    N = lat.N
    # particle number per spin is conserved exactly by the flow (trace), and
    # the FP32 trajectories keep it to round-off
    assert np.allclose(n[:, :N].sum(1), N / 2, atol=1e-3)
    assert np.allclose(n[:, N:].sum(1), N / 2, atol=1e-3)

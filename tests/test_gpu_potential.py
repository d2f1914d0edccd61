"""An external on-site potential V_i(t) = A(t) v_i (the explicit time-dependent
term of Eq. (6) for an external potential, Sec. III) through the C ABI: the
stream kernels against the oracle bitwise (same operation order: a = U(d_i -
d_j), then a + A(v_i - v_j), A and v rounded once), batches mixing instances
with and without a potential, trajectory chunks, graph replays, the resident
variants (spin split, shared blocks, split kernel), and the paths that refuse
it."""
import numpy as np
import pytest

from tests._util import pack, unpack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


def _host(x):
    import torch
    torch.cuda.synchronize()
    return x.detach().cpu().numpy()


def _pulse(n_steps, dt, A0=1.3, t0=0.1, w=0.05, nu=6.0):
    tau = np.arange(2 * n_steps + 1) * dt / 2
    return A0 * np.exp(-((tau - t0) / w) ** 2) * np.cos(nu * tau)


def _setup(ft, orc, kind, a, b, M, dtype, seed, U=3.3, profile="staggered"):
    import torch
    olat = orc.Lattice(kind, a, b)
    lat = ft.Lattice(kind, a, b)
    n0 = orc.fock_start(olat, "random", seed)
    rho0 = orc.sample(olat, n0, seed, M)
    prob = ft.Problem.allocate(lat, U, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    if profile == "staggered":
        v = np.array([(-1.0) ** s for s in olat.sub])
    else:
        v = np.random.default_rng(seed).uniform(-1, 1, lat.N)
    return olat, lat, rho0, prob, v, cdt


def _attach(prob, v, env):
    import torch
    prob.v_site = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    prob.v_env = torch.from_numpy(np.ascontiguousarray(env, dtype=np.float64)).cuda()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind,a,b,M,steps,profile", [
    ("torus", 2, 3, 70, 60, "staggered"),
    ("hex", 2, 0, 33, 40, "random"),        # degree-2 edge sites
    ("armchair", 10, 20, 5, 12, "random"),  # 198 sites
])
@pytest.mark.parametrize("path", ["stream", "auto"])
def test_potential_matches_oracle_bitwise(ft, orc, dtype, kind, a, b, M, steps, profile, path):
    dt, re = 0.01, 4
    olat, lat, rho0, prob, v, cdt = _setup(ft, orc, kind, a, b, M, dtype, 7, profile=profile)
    env = _pulse(steps, dt)
    _attach(prob, v, env)
    ft.evolve(prob, dt, steps, re, path=path)  # auto: resident variants where they fit
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision=dtype,
                                 vsite=v, env=env)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)
    # and the potential did something
    y0, _, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision=dtype)
    assert np.max(np.abs(y_ref - y0)) > 1e-4


@pytest.mark.parametrize("kind,a,b,M,steps", [("hex", 5, 0, 9, 10), ("armchair", 10, 20, 7, 10)])
def test_potential_on_the_spin_split_resident_kernel(ft, orc, kind, a, b, M, steps):
    """FP32 at 150 and 198 sites: the spin-split resident kernel's potential
    variant (the profile in LDS beside the partner's diagonal, the envelope a
    wave-uniform value per stage) bitwise equal to the oracle."""
    dt, re = 0.01, 5
    olat, lat, rho0, prob, v, cdt = _setup(ft, orc, kind, a, b, M, "f32", 17, profile="random")
    env = _pulse(steps, dt, t0=0.04)
    _attach(prob, v, env)
    ft.evolve(prob, dt, steps, re, path="resident")
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision="f32",
                                 vsite=v, env=env)
    assert np.array_equal(unpack(_host(prob.rho), lat.N), y_ref.astype(cdt))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)


def test_potential_on_the_spin_split_resident_kernel_with_general_t(ft, orc):
    """FP32 at 198 sites with t = 0.8: the general-t potential variant (t = 1
    launches take the variant without the hopping multiply) bitwise equal to
    the oracle."""
    import torch
    dt, steps, re = 0.01, 10, 5
    olat = orc.Lattice("armchair", 10, 20, t=0.8)
    lat = ft.Lattice("armchair", 10, 20, t=0.8)
    n0 = orc.fock_start(olat, "random", 61)
    rho0 = orc.sample(olat, n0, 61, 6)
    prob = ft.Problem.allocate(lat, 3.3, 6, n0, "f32")
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(np.complex64))))
    v = np.random.default_rng(61).uniform(-1, 1, lat.N)
    env = _pulse(steps, dt, t0=0.04)
    _attach(prob, v, env)
    ft.evolve(prob, dt, steps, re, path="resident")
    y_ref, _, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision="f32", vsite=v, env=env)
    assert np.array_equal(unpack(_host(prob.rho), lat.N), y_ref.astype(np.complex64))


def test_resident_launch_mixing_entries_with_and_without_a_potential(ft, orc):
    """Two 198-site FP32 instances of one resident configuration, only the first
    with a potential (each in a launch of its own kind): each equals its own
    oracle run."""
    dt, steps, re = 0.01, 8, 4
    o1, l1, r1, p1, v1, _ = _setup(ft, orc, "armchair", 10, 20, 5, "f32", 21, profile="random")
    o2, l2, r2, p2, _, _ = _setup(ft, orc, "armchair", 10, 20, 6, "f32", 22, U=2.0)
    p2.instance = 1
    env = _pulse(steps, dt, t0=0.03)
    _attach(p1, v1, env)
    ft.evolve([p1, p2], dt, steps, re, path="resident")
    y1, _, _ = orc.evolve(o1, 3.3, r1, dt, steps, re, precision="f32", vsite=v1, env=env)
    y2, _, _ = orc.evolve(o2, 2.0, r2, dt, steps, re, precision="f32")
    assert np.array_equal(unpack(_host(p1.rho), l1.N), y1.astype(np.complex64))
    assert np.array_equal(unpack(_host(p2.rho), l2.N), y2.astype(np.complex64))


@pytest.mark.parametrize("dtype,kind,a,b,config,t", [
    ("f32", "torus", 2, 3, -1, 1.0), ("f64", "torus", 2, 3, -1, 1.0),
    ("f32", "torus", 3, 9, -1, 1.0), ("f64", "torus", 3, 9, -1, 1.0),
    ("f32", "torus", 3, 9, 6, 1.0),    # every slot general
    ("f64", "torus", 3, 9, 2, 1.0),
    ("f32", "torus", 3, 9, -1, 0.8),   # t != 1: the general-hopping variant
    ("f32", "hex", 4, 0, -1, 1.0), ("f64", "hex", 4, 0, -1, 1.0),
])
def test_potential_on_the_shared_block_tiles(ft, orc, dtype, kind, a, b, config, t):
    """The shared-block tiles' potential variant (the profile in LDS after the
    blocks, one value per site at the element stride, indexed by the
    descriptors' diagonal offsets) bitwise equal to the oracle, states and
    moments."""
    import torch
    dt, steps, re = 0.01, 12, 4
    olat = orc.Lattice(kind, a, b, t)
    lat = ft.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 23)
    rho0 = orc.sample(olat, n0, 23, 13)
    prob = ft.Problem.allocate(lat, 3.3, 13, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    v = np.random.default_rng(23).uniform(-1, 1, lat.N)
    env = _pulse(steps, dt, t0=0.04)
    _attach(prob, v, env)
    ft.evolve(prob, dt, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision=dtype,
                                 vsite=v, env=env)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind,a,b,config", [("hex", 5, 0, 19), ("hex", 5, 0, 20), ("hex", 5, 0, 21), ("hex", 5, 0, 22),
                                             ("armchair", 10, 20, 20), ("armchair", 10, 20, 21)])
def test_potential_on_the_split_kernel(ft, orc, kind, a, b, config):
    """FP64 at 150 and 198 sites: the split kernel's potential variant (the
    profile in LDS after the two diagonal copies, in their layout) bitwise
    equal to the oracle in every split configuration that fits."""
    dt, steps, re = 0.01, 10, 5
    olat, lat, rho0, prob, v, _ = _setup(ft, orc, kind, a, b, 7, "f64", 31, profile="random")
    env = _pulse(steps, dt, t0=0.04)
    _attach(prob, v, env)
    ft.evolve(prob, dt, steps, re, config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, vsite=v, env=env)
    assert np.array_equal(unpack(_host(prob.rho), lat.N), y_ref)
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


def test_split_kernel_batch_with_and_without_a_potential(ft, orc):
    """FP64, automatic path: a 198-site instance with a potential, a larger-M
    198-site instance without one and a 150-site instance with one, in one
    call (split kernel groups by configuration and potential)."""
    dt, steps, re = 0.01, 8, 4
    o1, l1, r1, p1, v1, _ = _setup(ft, orc, "armchair", 10, 20, 5, "f64", 41, profile="random")
    o2, l2, r2, p2, _, _ = _setup(ft, orc, "armchair", 10, 20, 9, "f64", 42, U=2.0)
    o3, l3, r3, p3, v3, _ = _setup(ft, orc, "hex", 5, 0, 6, "f64", 43, U=1.5)
    p2.instance, p3.instance = 1, 2
    env = _pulse(steps, dt, t0=0.03)
    _attach(p1, v1, env)
    _attach(p3, v3, env)
    ft.evolve([p1, p2, p3], dt, steps, re, path="resident")
    y1, _, _ = orc.evolve(o1, 3.3, r1, dt, steps, re, vsite=v1, env=env)
    y2, _, _ = orc.evolve(o2, 2.0, r2, dt, steps, re)
    y3, _, _ = orc.evolve(o3, 1.5, r3, dt, steps, re, vsite=v3, env=env)
    assert np.array_equal(unpack(_host(p1.rho), l1.N), y1)
    assert np.array_equal(unpack(_host(p2.rho), l2.N), y2)
    assert np.array_equal(unpack(_host(p3.rho), l3.N), y3)


def test_larger_instance_without_a_potential_beside_a_smaller_one_with_it(ft, orc):
    """FP32, both forced onto the 198-site configuration: a 198-site instance
    without a potential and a 150-site one with it.  The potential variant's
    LDS layout is larger by the profile, so the two run as launches of their
    own kinds, each sized for its entries; each equals its own oracle run."""
    dt, steps, re = 0.01, 8, 4
    o1, l1, r1, p1, _, _ = _setup(ft, orc, "armchair", 10, 20, 6, "f32", 51, U=2.0)
    o2, l2, r2, p2, v2, _ = _setup(ft, orc, "hex", 5, 0, 5, "f32", 52, profile="random")
    p2.instance = 1
    env = _pulse(steps, dt, t0=0.03)
    _attach(p2, v2, env)
    ft.evolve([p1, p2], dt, steps, re, config=9)
    y1, _, _ = orc.evolve(o1, 2.0, r1, dt, steps, re, precision="f32")
    y2, _, _ = orc.evolve(o2, 3.3, r2, dt, steps, re, precision="f32", vsite=v2, env=env)
    assert np.array_equal(unpack(_host(p1.rho), l1.N), y1.astype(np.complex64))
    assert np.array_equal(unpack(_host(p2.rho), l2.N), y2.astype(np.complex64))


def test_batch_chunks_and_mixed_instances(ft, orc):
    """One call with two instances, one with a potential and one without, in
    trajectory chunks of 16: each equals its own oracle run."""
    import torch
    dt, steps, re = 0.01, 20, 5
    o1, l1, r1, p1, v1, _ = _setup(ft, orc, "torus", 3, 9, 37, "f64", 11, U=2.0)
    o2, l2, r2, p2, _, _ = _setup(ft, orc, "hex", 2, 0, 21, "f64", 12, U=1.0)
    p2.instance = 1
    env = _pulse(steps, dt, A0=0.8, t0=0.05)
    _attach(p1, v1, env)
    ft.evolve([p1, p2], dt, steps, re, traj_chunk=16, path="stream")
    y1, _, _ = orc.evolve(o1, 2.0, r1, dt, steps, re, vsite=v1, env=env)
    y2, _, _ = orc.evolve(o2, 1.0, r2, dt, steps, re)
    assert np.array_equal(unpack(_host(p1.rho), l1.N), y1)
    assert np.array_equal(unpack(_host(p2.rho), l2.N), y2)
    torch.cuda.synchronize()


def test_graph_replays_with_a_potential(ft, orc):
    """A captured run with a potential (12 sites: the shared-block tile's
    variant) replayed twice equals two direct runs; the first replay also
    equals the oracle."""
    import torch
    dt, steps, re = 0.01, 10, 5
    olat, lat, rho0, prob, v, _ = _setup(ft, orc, "torus", 2, 3, 40, "f32", 13)
    env = _pulse(steps, dt)
    _attach(prob, v, env)
    ref = ft.Problem.allocate(lat, 3.3, 40, prob.n0.cpu().numpy(), "f32")
    ref.rho.copy_(prob.rho)
    ref.v_site, ref.v_env = prob.v_site, prob.v_env
    g = ft.EvolveGraph([prob], dt, steps, re)
    y_ref, _, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision="f32", vsite=v, env=env)
    for r in range(2):
        g.launch()
        g.check()
        ft.evolve(ref, dt, steps, re)
        torch.cuda.synchronize()
        assert torch.equal(prob.rho, ref.rho)
        if r == 0:
            assert np.array_equal(unpack(_host(prob.rho), lat.N), y_ref.astype(np.complex64))
    g.close()


def test_paths_that_refuse_a_potential(ft, orc):
    import torch
    olat, lat, rho0, prob, v, _ = _setup(ft, orc, "torus", 2, 3, 8, "f32", 14)
    _attach(prob, v, _pulse(4, 0.01))
    w = torch.zeros((2, 2 * lat.N), dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtwaError):
        ft.adjoint(prob, 0.01, 4, 4, 4, w)
    prob.v_env = None  # a profile needs its envelope
    with pytest.raises(ft.FtwaError):
        ft.evolve(prob, 0.01, 4, 2)

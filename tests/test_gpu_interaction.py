"""A general density-density interaction u_ij between opposite spins (Eq. (1),
Eq. (6)'s own form) through the C ABI: the stream kernels (a per-stage kernel
forming D_i = sum_k u_ki (d_k + 1/2), fma over ascending k), the FP32
spin-split resident kernels and the FP64 split kernel (D formed at the start
of every stage from the partner's diagonal) against the oracle bitwise,
together with an external potential, in a batch with an on-site instance, and
the paths that refuse it."""
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


def _long_range(olat, U, seed, decay=1.5):
    """u_ij = U on site, a screened tail exp(-|i - j| / decay) / 2 between
    sites (index distance as a stand-in for distance), symmetric."""
    N = olat.N
    idx = np.arange(N)
    u = 0.5 * np.exp(-np.abs(idx[:, None] - idx[None, :]) / decay)
    np.fill_diagonal(u, U)
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.05, 0.05, (N, N))
    return u + 0.5 * (x + x.T)


def _setup(ft, orc, kind, a, b, M, dtype, seed):
    import torch
    olat = orc.Lattice(kind, a, b)
    lat = ft.Lattice(kind, a, b)
    n0 = orc.fock_start(olat, "random", seed)
    rho0 = orc.sample(olat, n0, seed, M)
    prob = ft.Problem.allocate(lat, 0.0, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    u = _long_range(olat, 3.3, seed)
    prob.u_mat = torch.from_numpy(u).cuda()
    return olat, lat, rho0, prob, u, cdt


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind,a,b,M,steps", [("torus", 2, 3, 70, 50), ("hex", 2, 0, 33, 30),
                                              ("armchair", 10, 20, 5, 8)])
@pytest.mark.parametrize("path", ["stream", "auto"])
def test_interaction_matches_oracle_bitwise(ft, orc, dtype, kind, a, b, M, steps, path):
    dt, re = 0.01, 5
    olat, lat, rho0, prob, u, cdt = _setup(ft, orc, kind, a, b, M, dtype, 3)
    ft.evolve(prob, dt, steps, re, path=path)  # auto: resident variants where they fit
    y_ref, X_ref, _ = orc.evolve(olat, 0.0, rho0, dt, steps, re, precision=dtype, umat=u)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


def test_interaction_with_a_potential_and_an_on_site_neighbour(ft, orc):
    """One call: a general-u instance that also carries a time-dependent
    potential, and an on-site instance, in trajectory chunks of 16."""
    import torch
    dt, steps, re = 0.01, 20, 5
    o1, l1, r1, p1, u1, _ = _setup(ft, orc, "torus", 3, 9, 37, "f64", 8)
    tau = np.arange(2 * steps + 1) * dt / 2
    env = 0.9 * np.sin(7.0 * tau)
    v = np.array([(-1.0) ** s for s in o1.sub])
    p1.v_site = torch.from_numpy(v).cuda()
    p1.v_env = torch.from_numpy(env).cuda()
    o2 = orc.Lattice("hex", 2, 0)
    l2 = ft.Lattice("hex", 2, 0)
    n2 = orc.fock_start(o2, "random", 9)
    r2 = orc.sample(o2, n2, 9, 21)
    p2 = ft.Problem.allocate(l2, 1.7, 21, n2, "f64", instance=1)
    p2.rho.copy_(torch.from_numpy(pack(r2)))
    ft.evolve([p1, p2], dt, steps, re, traj_chunk=16)
    y1, _, _ = orc.evolve(o1, 0.0, r1, dt, steps, re, umat=u1, vsite=v, env=env)
    y2, _, _ = orc.evolve(o2, 1.7, r2, dt, steps, re)
    assert np.array_equal(unpack(_host(p1.rho), l1.N), y1)
    assert np.array_equal(unpack(_host(p2.rho), l2.N), y2)


@pytest.mark.parametrize("kind,a,b,config,t", [
    ("hex", 5, 0, -1, 1.0),          # 150 sites: the automatic choice (768 x (8,8))
    ("armchair", 10, 20, -1, 1.0),   # 198 sites: the automatic choice (768 x (13,13))
    ("armchair", 10, 20, 10, 1.0),   # 1024 x (10,10)
    ("armchair", 10, 20, 11, 1.0),   # 512 x (20,20)
    ("armchair", 10, 20, 12, 1.0),   # every slot general
    ("armchair", 10, 20, -1, 0.7),   # t != 1: the general-hopping variant
    ("hex", 4, 0, 9, 1.0),           # 96 sites on the 198-site tile
])
def test_resident_interaction_matches_oracle_bitwise(ft, orc, kind, a, b, config, t):
    """The spin-split resident kernel's general-interaction variant: per
    stage, each of the first N threads forms D_i over ascending k from the
    partner's diagonal in LDS and u (rounded once to FP32) from global memory;
    the elements take D_i - D_j as their U factor."""
    import torch
    dt, steps, re = 0.01, 8, 4
    olat = orc.Lattice(kind, a, b, t)
    lat = ft.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 14)
    M = 9
    rho0 = orc.sample(olat, n0, 14, M)
    prob = ft.Problem.allocate(lat, 0.0, M, n0, "f32")
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(np.complex64))))
    u = _long_range(olat, 3.3, 14)
    prob.u_mat = torch.from_numpy(u).cuda()
    ft.evolve(prob, dt, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 0.0, rho0, dt, steps, re, precision="f32", umat=u)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(np.complex64)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind,a,b,config,t", [
    ("hex", 5, 0, -1, 1.0),          # 150 sites: the automatic choice (two parts of 768)
    ("hex", 5, 0, 19, 0.7),          # two parts of 512, t != 1
    ("armchair", 10, 20, -1, 1.0),   # 198 sites: the automatic choice (three parts of 512)
    ("armchair", 10, 20, 21, 1.0),   # four parts of 512
])
def test_split_interaction_matches_oracle_bitwise(ft, orc, kind, a, b, config, t):
    """The FP64 split kernel's general-interaction variant: every part forms
    D_i over ascending k from the partner's whole diagonal (site-ordered copy
    in LDS) and u (FP64, blocked by four along k) per stage; the elements of
    every part take D_i - D_j as their U factor."""
    import torch
    dt, steps, re = 0.01, 8, 4
    olat = orc.Lattice(kind, a, b, t)
    lat = ft.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 15)
    M = 7
    rho0 = orc.sample(olat, n0, 15, M)
    prob = ft.Problem.allocate(lat, 0.0, M, n0, "f64")
    prob.rho.copy_(torch.from_numpy(pack(rho0)))
    u = _long_range(olat, 3.3, 15)
    prob.u_mat = torch.from_numpy(u).cuda()
    ft.evolve(prob, dt, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 0.0, rho0, dt, steps, re, umat=u)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dtype,kind,a,b,config,t", [
    ("f32", "torus", 2, 3, -1, 1.0), ("f64", "torus", 2, 3, -1, 1.0),
    ("f32", "torus", 3, 9, -1, 1.0), ("f64", "torus", 3, 9, -1, 1.0),
    ("f32", "torus", 3, 9, 6, 1.0),    # every slot general
    ("f64", "torus", 3, 9, 2, 1.0),
    ("f32", "torus", 3, 9, -1, 0.7),   # t != 1: the general-hopping variant
    ("f32", "hex", 4, 0, -1, 1.0), ("f64", "hex", 4, 0, -1, 1.0),
])
def test_shared_block_interaction_matches_oracle_bitwise(ft, orc, dtype, kind, a, b, config, t):
    """The shared-block tiles' general-interaction variant (both spins of a
    trajectory in one unit): per stage, threads t < 2N of each unit form D of
    both spins from the partner block's diagonal and u (blocked by four along
    k), the elements take D_i - D_j as their U factor."""
    import torch
    dt, steps, re = 0.01, 8, 4
    olat = orc.Lattice(kind, a, b, t)
    lat = ft.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 16)
    M = 11
    rho0 = orc.sample(olat, n0, 16, M)
    prob = ft.Problem.allocate(lat, 0.0, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    u = _long_range(olat, 3.3, 16)
    prob.u_mat = torch.from_numpy(u).cuda()
    ft.evolve(prob, dt, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 0.0, rho0, dt, steps, re, precision=dtype, umat=u)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_resident_interaction_next_to_on_site_instances(ft, orc, dtype):
    """One automatic call: a 198-site general-u instance (its own launch
    group, the variant's larger LDS layout) next to a 198-site on-site
    instance of the same configuration, several passes of windows (FP32:
    the spin-split tile; FP64: the split kernel)."""
    import torch
    dt, steps, re = 0.01, 6, 3
    o1, l1, r1, p1, u1, cdt = _setup(ft, orc, "armchair", 10, 20, 7, dtype, 21)
    n2 = orc.fock_start(o1, "random", 22)
    r2 = orc.sample(o1, n2, 22, 5)
    p2 = ft.Problem.allocate(l1, 3.3, 5, n2, dtype, instance=1)
    p2.rho.copy_(torch.from_numpy(pack(r2.astype(cdt))))
    ft.evolve([p1, p2], dt, steps, re, traj_chunk=3)
    y1, _, _ = orc.evolve(o1, 0.0, r1, dt, steps, re, precision=dtype, umat=u1)
    y2, _, _ = orc.evolve(o1, 3.3, r2, dt, steps, re, precision=dtype)
    assert np.array_equal(unpack(_host(p1.rho), l1.N), y1.astype(cdt))
    assert np.array_equal(unpack(_host(p2.rho), l1.N), y2.astype(cdt))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_resident_interaction_graph_replays(ft, orc, dtype):
    """The resident variant captured in a graph (staging u in the working
    precision is a kernel of the graph) and replayed twice equals two direct
    runs; the first replay also equals the oracle."""
    import torch
    dt, steps, re = 0.01, 6, 3
    olat, lat, rho0, prob, u, cdt = _setup(ft, orc, "armchair", 10, 20, 6, dtype, 8)
    ref = ft.Problem.allocate(lat, 0.0, 6, prob.n0.cpu().numpy(), dtype)
    ref.rho.copy_(prob.rho)
    ref.u_mat = prob.u_mat
    g = ft.EvolveGraph([prob], dt, steps, re, path="resident")
    y_ref, _, _ = orc.evolve(olat, 0.0, rho0, dt, steps, re, precision=dtype, umat=u)
    for r in range(2):
        g.launch()
        g.check()
        ft.evolve(ref, dt, steps, re, path="resident")
        torch.cuda.synchronize()
        assert torch.equal(prob.rho, ref.rho)
        if r == 0:
            assert np.array_equal(unpack(_host(prob.rho), lat.N), y_ref.astype(cdt))
    g.close()


def test_paths_that_refuse_a_general_interaction(ft, orc):
    import torch
    olat, lat, rho0, prob, u, _ = _setup(ft, orc, "armchair", 10, 20, 4, "f32", 5)
    # together with a potential: stream only
    prob.v_site = torch.zeros(lat.N, dtype=torch.float64, device="cuda")
    prob.v_env = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtwaError) as e:
        ft.evolve(prob, 0.01, 2, 1, path="resident")
    assert e.value.status == -4
    prob.v_site = prob.v_env = None
    w = torch.zeros((2, 2 * lat.N), dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtwaError):
        ft.adjoint(prob, 0.01, 2, 2, 2, w)
    prob.track_invariants = True
    with pytest.raises(ft.FtwaError):
        ft.evolve(prob, 0.01, 2, 1)

"""Complex, time-dependent (Peierls) hopping j_ik(tau) = t w_ik(tau) through
the C ABI: the stream kernels, the FP32 spin-split resident kernels (every
spin-split configuration, t = 1 and t != 1) and the FP64 split kernel (two,
three and four parts) against the oracle bitwise, the
ratio table built for each side from its own neighbour table; together with
an external potential and a general interaction in a batch with a
real-hopping instance; graph replays; and the paths that refuse it."""
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


def _phase_fn(N, seed, dt):
    """w_ik(tau_h) = exp(i (theta_ik + (x_k - x_i) B(tau_h))) for i < k (random
    static fluxes plus a uniform-field-like drive, B(tau) = 0.7 sin(5 tau)),
    conjugated for i > k so that both directions are exact conjugates."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi, np.pi, (N, N))
    x = rng.uniform(-1, 1, N)

    def w(h, i, k):
        a, b = (i, k) if i < k else (k, i)
        z = np.exp(1j * (th[a, b] + (x[b] - x[a]) * 0.7 * np.sin(5.0 * h * dt / 2)))
        return z if i < k else np.conj(z)
    return w


def _table(nbr, deg, fn, n_half, fill=0.0):
    N = len(deg)
    out = np.full((n_half, N, 3), fill, dtype=np.complex128)
    for i in range(N):
        for n in range(int(deg[i])):
            k = int(nbr[i, n])
            for h in range(n_half):
                out[h, i, n] = fn(h, i, k)
    return out


def _setup(ft, orc, kind, a, b, M, U, dtype, seed, steps, dt):
    import torch
    olat = orc.Lattice(kind, a, b)
    lat = ft.Lattice(kind, a, b)
    n0 = orc.fock_start(olat, "random", seed)
    rho0 = orc.sample(olat, n0, seed, M)
    prob = ft.Problem.allocate(lat, U, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    fn = _phase_fn(olat.N, seed, dt)
    w_orc = _table(olat.nbr, olat.deg, fn, 2 * steps + 1)
    # unused slots hold NaN on the device side: they must not be read into sums
    w_dev = _table(lat.nbr, lat.deg, fn, 2 * steps + 1, fill=np.nan)
    prob.hop_w = torch.from_numpy(w_dev).cuda()
    return olat, lat, rho0, prob, w_orc, cdt


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("kind,a,b,M,steps", [("torus", 2, 3, 70, 40), ("hex", 2, 0, 33, 30),
                                              ("armchair", 10, 20, 5, 6)])
@pytest.mark.parametrize("path", ["stream", "auto"])
def test_peierls_matches_oracle_bitwise(ft, orc, dtype, kind, a, b, M, steps, path):
    dt, re = 0.01, 5
    olat, lat, rho0, prob, w, cdt = _setup(ft, orc, kind, a, b, M, 3.3, dtype, 4, steps, dt)
    ft.evolve(prob, dt, steps, re, path=path)  # auto: resident variants where they fit
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision=dtype, hop=w)
    got = unpack(_host(prob.rho), lat.N)
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


def test_peierls_with_potential_interaction_and_a_plain_neighbour(ft, orc):
    """One call: an instance with complex hopping, a time-dependent potential
    and a general interaction, and a real-hopping on-site instance, in
    trajectory chunks of 16 (the ratio table follows the step index across
    chunks)."""
    import torch
    dt, steps, re = 0.01, 20, 5
    o1, l1, r1, p1, w1, _ = _setup(ft, orc, "torus", 3, 9, 37, 0.0, "f64", 8, steps, dt)
    tau = np.arange(2 * steps + 1) * dt / 2
    env = 0.9 * np.sin(7.0 * tau)
    v = np.array([(-1.0) ** s for s in o1.sub])
    p1.v_site = torch.from_numpy(v).cuda()
    p1.v_env = torch.from_numpy(env).cuda()
    idx = np.arange(o1.N)
    u = 0.5 * np.exp(-np.abs(idx[:, None] - idx[None, :]) / 1.5)
    np.fill_diagonal(u, 3.0)
    p1.u_mat = torch.from_numpy(u).cuda()
    o2 = orc.Lattice("hex", 2, 0)
    l2 = ft.Lattice("hex", 2, 0)
    n2 = orc.fock_start(o2, "random", 9)
    r2 = orc.sample(o2, n2, 9, 21)
    p2 = ft.Problem.allocate(l2, 1.7, 21, n2, "f64", instance=1)
    p2.rho.copy_(torch.from_numpy(pack(r2)))
    ft.evolve([p1, p2], dt, steps, re, traj_chunk=16)
    y1, _, _ = orc.evolve(o1, 0.0, r1, dt, steps, re, umat=u, vsite=v, env=env, hop=w1)
    y2, _, _ = orc.evolve(o2, 1.7, r2, dt, steps, re)
    assert np.array_equal(unpack(_host(p1.rho), l1.N), y1)
    assert np.array_equal(unpack(_host(p2.rho), l2.N), y2)


def test_graph_replays_with_complex_hopping(ft, orc):
    """A captured run with complex hopping replayed twice equals two direct
    runs (the tables are read at the step index of each replay's own run)."""
    import torch
    dt, steps, re = 0.01, 10, 5
    olat, lat, rho0, prob, w, _ = _setup(ft, orc, "torus", 2, 3, 40, 2.0, "f32", 6, steps, dt)
    ref = ft.Problem.allocate(lat, 2.0, 40, prob.n0.cpu().numpy(), "f32")
    ref.rho.copy_(prob.rho)
    ref.hop_w = prob.hop_w
    g = ft.EvolveGraph([prob], dt, steps, re)
    for _ in range(2):
        g.launch()
        g.check()
        ft.evolve(ref, dt, steps, re)
        torch.cuda.synchronize()
        assert torch.equal(prob.rho, ref.rho)
    g.close()


@pytest.mark.parametrize("kind,a,b,config,t", [
    ("hex", 5, 0, -1, 1.0),          # 150 sites: the automatic choice (768 x (8,8))
    ("armchair", 10, 20, -1, 1.0),   # 198 sites: the automatic choice (768 x (13,13))
    ("armchair", 10, 20, 10, 1.0),   # 1024 x (10,10)
    ("armchair", 10, 20, 11, 1.0),   # 512 x (20,20)
    ("armchair", 10, 20, 12, 1.0),   # every slot general
    ("armchair", 10, 20, -1, 0.8),   # t != 1: the general-hopping variant
    ("hex", 4, 0, 9, 1.3),           # 96 sites on the 198-site tile (padding-heavy slots)
])
def test_resident_peierls_matches_oracle_bitwise(ft, orc, kind, a, b, config, t):
    """The spin-split resident kernel's complex-hopping variant: the ratio
    table (prepared on the device in the place order of the partner's
    diagonal, missing neighbours zero while the caller's unused slots hold
    NaN) read from global memory per stage; both directions of a transposed
    orientation come out exact conjugates, so the state equals the oracle's."""
    import torch
    dt, steps, re = 0.01, 8, 4
    olat = orc.Lattice(kind, a, b, t)
    lat = ft.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 12)
    M = 9
    rho0 = orc.sample(olat, n0, 12, M)
    prob = ft.Problem.allocate(lat, 3.3, M, n0, "f32")
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(np.complex64))))
    fn = _phase_fn(olat.N, 12, dt)
    w = _table(olat.nbr, olat.deg, fn, 2 * steps + 1)
    prob.hop_w = torch.from_numpy(_table(lat.nbr, lat.deg, fn, 2 * steps + 1, fill=np.nan)).cuda()
    ft.evolve(prob, dt, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision="f32", hop=w)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(np.complex64)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind,a,b,config,t", [
    ("hex", 5, 0, -1, 1.0),          # 150 sites: the automatic choice (two parts of 768)
    ("hex", 5, 0, 19, 0.8),          # two parts of 512, t != 1
    ("armchair", 10, 20, -1, 1.0),   # 198 sites: the automatic choice (three parts of 512)
    ("armchair", 10, 20, 21, 1.0),   # four parts of 512
])
def test_split_peierls_matches_oracle_bitwise(ft, orc, kind, a, b, config, t):
    """The FP64 split kernel's complex-hopping variant: each stage's whole
    ratio table in LDS, read by the elements of every part through the
    descriptors' diagonal offsets; unused slots hold NaN on the caller's side."""
    import torch
    dt, steps, re = 0.01, 8, 4
    olat = orc.Lattice(kind, a, b, t)
    lat = ft.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 13)
    M = 7
    rho0 = orc.sample(olat, n0, 13, M)
    prob = ft.Problem.allocate(lat, 3.3, M, n0, "f64")
    prob.rho.copy_(torch.from_numpy(pack(rho0)))
    fn = _phase_fn(olat.N, 13, dt)
    w = _table(olat.nbr, olat.deg, fn, 2 * steps + 1)
    prob.hop_w = torch.from_numpy(_table(lat.nbr, lat.deg, fn, 2 * steps + 1, fill=np.nan)).cuda()
    ft.evolve(prob, dt, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, hop=w)
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
    ("f32", "torus", 3, 9, -1, 0.8),   # t != 1: the general-hopping variant
    ("f32", "hex", 4, 0, -1, 1.0), ("f64", "hex", 4, 0, -1, 1.0),
])
def test_shared_block_peierls_matches_oracle_bitwise(ft, orc, dtype, kind, a, b, config, t):
    """The shared-block tiles' complex-hopping variant: each stage's whole
    ratio table in LDS in site order, indexed by the descriptors' diagonal
    offsets; unused slots hold NaN on the caller's side."""
    import torch
    dt, steps, re = 0.01, 8, 4
    olat = orc.Lattice(kind, a, b, t)
    lat = ft.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, "random", 17)
    M = 11
    rho0 = orc.sample(olat, n0, 17, M)
    prob = ft.Problem.allocate(lat, 3.3, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    fn = _phase_fn(olat.N, 17, dt)
    w = _table(olat.nbr, olat.deg, fn, 2 * steps + 1)
    prob.hop_w = torch.from_numpy(_table(lat.nbr, lat.deg, fn, 2 * steps + 1, fill=np.nan)).cuda()
    ft.evolve(prob, dt, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision=dtype, hop=w)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_resident_peierls_graph_replays(ft, orc, dtype):
    """The resident variant (FP32: the spin-split tile; FP64: the split
    kernel) captured in a graph (the table preparation is a kernel of the
    graph) and replayed twice equals two direct runs; the first replay also
    equals the oracle."""
    import torch
    dt, steps, re = 0.01, 6, 3
    olat, lat, rho0, prob, w, cdt = _setup(ft, orc, "armchair", 10, 20, 6, 3.3, dtype, 7, steps,
                                           dt)
    ref = ft.Problem.allocate(lat, 3.3, 6, prob.n0.cpu().numpy(), dtype)
    ref.rho.copy_(prob.rho)
    ref.hop_w = prob.hop_w
    g = ft.EvolveGraph([prob], dt, steps, re, path="resident")
    y_ref, _, _ = orc.evolve(olat, 3.3, rho0, dt, steps, re, precision=dtype, hop=w)
    for r in range(2):
        g.launch()
        g.check()
        ft.evolve(ref, dt, steps, re, path="resident")
        torch.cuda.synchronize()
        assert torch.equal(prob.rho, ref.rho)
        if r == 0:
            assert np.array_equal(unpack(_host(prob.rho), lat.N), y_ref.astype(cdt))
    g.close()


def test_paths_that_refuse_complex_hopping(ft, orc):
    import torch
    olat, lat, rho0, prob, w, _ = _setup(ft, orc, "armchair", 10, 20, 4, 3.3, "f32", 5, 2, 0.01)
    # complex hopping together with a potential: stream only
    prob.v_site = torch.zeros(lat.N, dtype=torch.float64, device="cuda")
    prob.v_env = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtwaError) as e:
        ft.evolve(prob, 0.01, 2, 1, path="resident")
    assert e.value.status == -4
    prob.v_site = prob.v_env = None
    g = torch.zeros((2, 2 * lat.N), dtype=torch.float64, device="cuda")
    with pytest.raises(ft.FtwaError):
        ft.adjoint(prob, 0.01, 2, 2, 2, g)
    prob.track_invariants = True
    with pytest.raises(ft.FtwaError):
        ft.evolve(prob, 0.01, 2, 1)

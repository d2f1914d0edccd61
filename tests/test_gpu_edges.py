"""Edge cases of the evolution kernels against the oracle (through the C ABI):
no steps, degenerate parameters (U = 0, t = 0), graphs other than the honeycomb
generators (an open chain with degree-1 ends, an isolated site, an odd ring
that is not bipartite and so only has the stream path), and the largest
lattice the library accepts.  The evolved states must equal the oracle's
bitwise (same operation order); the moments to 1e-12.
"""
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


def _lattices(ft, orc, spec, t=1.0):
    kind = spec[0]
    if kind == "custom":
        _, n, bonds, sub = spec
        return (ft.Lattice("custom", 0, 0, t, bonds=bonds, sublattice=sub, n_sites=n),
                orc.Lattice.from_bonds(n, bonds, sub, t=t))
    _, a, b = spec
    return ft.Lattice(kind, a, b, t), orc.Lattice(kind, a, b, t)


def _run(ft, orc, spec, dtype, path, U=3.3, t=1.0, M=37, steps=25, re=5, seed=4, n0=None,
         config=-1):
    import torch
    lat, olat = _lattices(ft, orc, spec, t)
    if n0 is None:
        n0 = orc.fock_start(olat, "random", seed)
    rho0 = orc.sample(olat, n0, seed, M)
    prob = ft.Problem.allocate(lat, U, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    ft.evolve(prob, 0.01, steps, re, path=path, config=config)
    y_ref, X_ref, _ = orc.evolve(olat, U, rho0, 0.01, steps, re, precision=dtype)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)
    return got, rho0.astype(cdt)


CHAIN7 = ("custom", 7, [(k, k + 1) for k in range(6)], [k % 2 for k in range(7)])
# a comb with one isolated site: degrees 0..3
COMB = ("custom", 9, [(0, 1), (1, 2), (2, 3), (1, 4), (3, 5), (5, 6), (5, 7)],
        [0, 1, 0, 1, 0, 0, 1, 1, 0])
RING5 = ("custom", 5, [(k, (k + 1) % 5) for k in range(5)], [0, 1, 0, 1, 0])


@pytest.mark.parametrize("path", ["stream", "resident"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_zero_steps_leave_the_state(ft, orc, dtype, path):
    got, rho0 = _run(ft, orc, ("torus", 2, 3), dtype, path, steps=0, re=1)
    assert np.array_equal(got, rho0)


@pytest.mark.parametrize("path", ["stream", "resident"])
@pytest.mark.parametrize("U,t", [(0.0, 1.0), (3.3, 0.0), (-2.0, 0.7)])
def test_degenerate_parameters(ft, orc, U, t, path):
    got, rho0 = _run(ft, orc, ("hex", 2, 0), "f32", path, U=U, t=t)
    if t == 0.0:  # no hopping: the diagonal of each block is conserved exactly
        assert np.array_equal(np.diagonal(got, axis1=2, axis2=3),
                              np.diagonal(rho0, axis1=2, axis2=3))


@pytest.mark.parametrize("path", ["stream", "resident"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec", [CHAIN7, COMB], ids=["chain7", "comb"])
def test_other_bipartite_graphs(ft, orc, spec, dtype, path):
    sub = np.array(spec[3], dtype=float)
    _run(ft, orc, spec, dtype, path, M=70, n0=np.array([1.0 - sub, sub]))  # Neel-like start


@pytest.mark.parametrize("config", [19, 20, 21, 22], ids=["split2", "split3", "split4", "split2w"])
@pytest.mark.parametrize("spec", [CHAIN7, COMB, ("torus", 2, 3), ("hex", 1, 0)],
                         ids=["chain7", "comb", "torus12", "hex6"])
def test_split_kernel_on_small_and_irregular_graphs(ft, orc, spec, config):
    """The FP64 split configurations forced on graphs far smaller than they are
    made for: strips of one or two rows, parts that own no diagonal or no
    element at all, degree-0 and degree-1 sites."""
    n0 = None
    if spec[0] == "custom":
        sub = np.array(spec[3], dtype=float)
        n0 = np.array([1.0 - sub, sub])
    _run(ft, orc, spec, "f64", "resident", M=11, steps=9, re=3, n0=n0, config=config)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_odd_ring_runs_on_the_stream_path_only(ft, orc, dtype):
    _run(ft, orc, RING5, dtype, "auto", M=20, n0=np.array([[1, 0, 1, 0, 0.0], [0, 1, 0, 1, 1.0]]))
    lat, _ = _lattices(ft, orc, RING5)
    prob = ft.Problem.allocate(lat, 1.0, 4, np.array([[1, 0, 1, 0, 0.0], [0, 1, 0, 1, 1.0]]),
                               dtype)
    ft.sample(prob, 1)
    with pytest.raises(ft.FtwaError):
        ft.evolve(prob, 0.01, 2, 1, path="resident")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_largest_lattice(ft, orc, dtype):
    """A 9 x 14 torus, 252 sites (the library takes up to 255): the stream path
    in both precisions (no resident tile holds a block this large)."""
    _run(ft, orc, ("torus", 9, 14), dtype, "auto", M=3, steps=3, re=1)


@pytest.mark.parametrize("variant", ["potential", "interaction", "hopping"])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("spec", [CHAIN7, COMB], ids=["chain7", "comb"])
def test_variants_on_irregular_graphs(ft, orc, spec, dtype, variant):
    """The shared-block tiles' Hamiltonian variants on graphs with degree-1
    sites (unused ratio slots, NaN on the device side) and far fewer sites
    than the interaction table's padded rows, bitwise equal to the oracle."""
    import torch
    dt, steps, re = 0.01, 16, 4
    lat, olat = _lattices(ft, orc, spec)
    N = olat.N
    rng = np.random.default_rng(12)
    sub = np.array(spec[3], dtype=float)
    n0 = np.array([1.0 - sub, sub])  # Neel-like start (odd site counts)
    M = 19
    rho0 = orc.sample(olat, n0, 12, M)
    U = 0.0 if variant == "interaction" else 2.7
    prob = ft.Problem.allocate(lat, U, M, n0, dtype)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    if variant == "potential":
        v = rng.uniform(-1, 1, N)
        env = 1.2 * np.cos(3.0 * np.arange(2 * steps + 1) * dt / 2)
        prob.v_site = torch.from_numpy(v).cuda()
        prob.v_env = torch.from_numpy(env).cuda()
        kw = dict(vsite=v, env=env)
    elif variant == "interaction":
        idx = np.arange(N)
        u = 0.6 * np.exp(-np.abs(idx[:, None] - idx[None, :]))
        np.fill_diagonal(u, 2.9)
        prob.u_mat = torch.from_numpy(u).cuda()
        kw = dict(umat=u)
    else:
        th = rng.uniform(-np.pi, np.pi, (N, N))

        def table(nbr, deg, fill):
            w = np.full((2 * steps + 1, N, 3), fill, dtype=np.complex128)
            for i in range(N):
                for n in range(int(deg[i])):
                    k = int(nbr[i][n])
                    a, b = (i, k) if i < k else (k, i)
                    for h in range(2 * steps + 1):
                        z = np.exp(1j * (th[a, b] + 0.3 * h * dt))
                        w[h, i, n] = z if i < k else np.conj(z)
            return w

        prob.hop_w = torch.from_numpy(table(lat.nbr, lat.deg, np.nan)).cuda()
        kw = dict(hop=table(olat.nbr, olat.deg, 0.0))
    ft.evolve(prob, dt, steps, re, path="resident")
    y_ref, X_ref, _ = orc.evolve(olat, U, rho0, dt, steps, re, precision=dtype, **kw)
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref.astype(cdt)), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)

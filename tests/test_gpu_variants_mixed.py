"""One resident call mixing every Hamiltonian variant at 198 sites
(a general interaction, complex hopping, an external potential) with an
on-site 150-site instance: each instance forms a launch group of its own, with
its own LDS layout (FP32: the spin-split kernels; FP64: the split kernel), and
every result equals the oracle bitwise."""
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


def _problem(ft, orc, kind, a, b, U, M, dtype, seed, instance):
    import torch
    olat = orc.Lattice(kind, a, b)
    lat = ft.Lattice(kind, a, b)
    n0 = orc.fock_start(olat, "random", seed)
    rho0 = orc.sample(olat, n0, seed, M)
    prob = ft.Problem.allocate(lat, U, M, n0, dtype, instance=instance)
    cdt = np.complex128 if dtype == "f64" else np.complex64
    prob.rho.copy_(torch.from_numpy(pack(rho0.astype(cdt))))
    return olat, lat, rho0, prob, cdt


def _ratios(olat, n_half, dt, fill):
    """Unit-modulus ratios with static random fluxes and a drive; both
    directions of a bond exact conjugates; unused slots hold `fill`."""
    N = olat.N
    rng = np.random.default_rng(5)
    th = rng.uniform(-np.pi, np.pi, (N, N))
    x = rng.uniform(-1, 1, N)
    out = np.full((n_half, N, 3), fill, dtype=np.complex128)
    for i in range(N):
        for n in range(int(olat.deg[i])):
            k = int(olat.nbr[i, n])
            a, b = (i, k) if i < k else (k, i)
            for h in range(n_half):
                z = np.exp(1j * (th[a, b] + (x[b] - x[a]) * 0.6 * np.sin(4.0 * h * dt / 2)))
                out[h, i, n] = z if i < k else np.conj(z)
    return out


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_every_variant_in_one_resident_call(ft, orc, dtype):
    import torch
    dt, steps, re = 0.01, 6, 3
    # a general interaction
    oa, la, ra, pa, cdt = _problem(ft, orc, "armchair", 10, 20, 0.0, 5, dtype, 61, 0)
    idx = np.arange(oa.N)
    u = 0.5 * np.exp(-np.abs(idx[:, None] - idx[None, :]) / 2.0)
    np.fill_diagonal(u, 3.3)
    pa.u_mat = torch.from_numpy(u).cuda()
    # complex hopping
    ob, lb, rb, pb, _ = _problem(ft, orc, "armchair", 10, 20, 3.3, 4, dtype, 62, 1)
    w = _ratios(ob, 2 * steps + 1, dt, 0.0)
    pb.hop_w = torch.from_numpy(_ratios(ob, 2 * steps + 1, dt, np.nan)).cuda()
    # an external potential
    oc, lc, rc, pc, _ = _problem(ft, orc, "armchair", 10, 20, 2.0, 3, dtype, 63, 2)
    v = np.array([(-1.0) ** s for s in oc.sub])
    tau = np.arange(2 * steps + 1) * dt / 2
    env = 1.1 * np.cos(5.0 * tau)
    pc.v_site = torch.from_numpy(v).cuda()
    pc.v_env = torch.from_numpy(env).cuda()
    # on-site, another size
    od, ld, rd, pd, _ = _problem(ft, orc, "hex", 5, 0, 1.5, 6, dtype, 64, 3)

    ft.evolve([pa, pb, pc, pd], dt, steps, re, path="resident")
    refs = [
        orc.evolve(oa, 0.0, ra, dt, steps, re, precision=dtype, umat=u)[0],
        orc.evolve(ob, 3.3, rb, dt, steps, re, precision=dtype, hop=w)[0],
        orc.evolve(oc, 2.0, rc, dt, steps, re, precision=dtype, vsite=v, env=env)[0],
        orc.evolve(od, 1.5, rd, dt, steps, re, precision=dtype)[0],
    ]
    for p, lat, y in zip((pa, pb, pc, pd), (la, lb, lc, ld), refs):
        got = unpack(_host(p.rho), lat.N)
        assert np.array_equal(got, y.astype(cdt)), np.max(np.abs(got - y))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_every_variant_on_the_shared_block_tiles_in_one_call(ft, orc, dtype):
    """The same at 54 sites (the 3x9 torus: shared-block tiles, both spin
    blocks of a trajectory in one workgroup) with an on-site 12-site instance:
    four launch groups of the shared-block kernel, each equal to the oracle
    bitwise."""
    import torch
    dt, steps, re = 0.01, 8, 4
    oa, la, ra, pa, cdt = _problem(ft, orc, "torus", 3, 9, 0.0, 7, dtype, 71, 0)
    idx = np.arange(oa.N)
    u = 0.4 * np.exp(-np.abs(idx[:, None] - idx[None, :]) / 3.0)
    np.fill_diagonal(u, 2.5)
    pa.u_mat = torch.from_numpy(u).cuda()
    ob, lb, rb, pb, _ = _problem(ft, orc, "torus", 3, 9, 3.3, 9, dtype, 72, 1)
    w = _ratios(ob, 2 * steps + 1, dt, 0.0)
    pb.hop_w = torch.from_numpy(_ratios(ob, 2 * steps + 1, dt, np.nan)).cuda()
    oc, lc, rc, pc, _ = _problem(ft, orc, "torus", 3, 9, 2.0, 5, dtype, 73, 2)
    v = np.array([(-1.0) ** s for s in oc.sub])
    tau = np.arange(2 * steps + 1) * dt / 2
    env = 0.9 * np.sin(7.0 * tau)
    pc.v_site = torch.from_numpy(v).cuda()
    pc.v_env = torch.from_numpy(env).cuda()
    od, ld, rd, pd, _ = _problem(ft, orc, "torus", 2, 3, 1.5, 21, dtype, 74, 3)

    ft.evolve([pa, pb, pc, pd], dt, steps, re, path="resident")
    refs = [
        orc.evolve(oa, 0.0, ra, dt, steps, re, precision=dtype, umat=u)[0],
        orc.evolve(ob, 3.3, rb, dt, steps, re, precision=dtype, hop=w)[0],
        orc.evolve(oc, 2.0, rc, dt, steps, re, precision=dtype, vsite=v, env=env)[0],
        orc.evolve(od, 1.5, rd, dt, steps, re, precision=dtype)[0],
    ]
    for p, lat, y in zip((pa, pb, pc, pd), (la, lb, lc, ld), refs):
        got = unpack(_host(p.rho), lat.N)
        assert np.array_equal(got, y.astype(cdt)), np.max(np.abs(got - y))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_shared_block_variants_in_graph_replays(ft, orc, dtype):
    """The three shared-block variants at 54 sites captured in one graph (the
    staging kernels of u and of the ratio tables inside it) and replayed
    twice: every replay equals a direct run, the first also the oracle."""
    import torch
    dt, steps, re = 0.01, 6, 3
    oa, la, ra, pa, cdt = _problem(ft, orc, "torus", 3, 9, 0.0, 6, dtype, 81, 0)
    idx = np.arange(oa.N)
    u = 0.4 * np.exp(-np.abs(idx[:, None] - idx[None, :]) / 3.0)
    np.fill_diagonal(u, 2.5)
    pa.u_mat = torch.from_numpy(u).cuda()
    ob, lb, rb, pb, _ = _problem(ft, orc, "torus", 3, 9, 3.3, 5, dtype, 82, 1)
    w = _ratios(ob, 2 * steps + 1, dt, 0.0)
    pb.hop_w = torch.from_numpy(_ratios(ob, 2 * steps + 1, dt, np.nan)).cuda()
    oc, lc, rc, pc, _ = _problem(ft, orc, "torus", 3, 9, 2.0, 7, dtype, 83, 2)
    v = np.array([(-1.0) ** s for s in oc.sub])
    env = 0.9 * np.sin(7.0 * np.arange(2 * steps + 1) * dt / 2)
    pc.v_site = torch.from_numpy(v).cuda()
    pc.v_env = torch.from_numpy(env).cuda()
    probs = [pa, pb, pc]
    refs = []
    for p in probs:
        q = ft.Problem.allocate(p.lat, p.U, p.n_traj, p.n0.cpu().numpy(), dtype,
                                instance=p.instance)
        q.rho.copy_(p.rho)
        q.u_mat, q.hop_w, q.v_site, q.v_env = p.u_mat, p.hop_w, p.v_site, p.v_env
        refs.append(q)
    ys = [
        orc.evolve(oa, 0.0, ra, dt, steps, re, precision=dtype, umat=u)[0],
        orc.evolve(ob, 3.3, rb, dt, steps, re, precision=dtype, hop=w)[0],
        orc.evolve(oc, 2.0, rc, dt, steps, re, precision=dtype, vsite=v, env=env)[0],
    ]
    g = ft.EvolveGraph(probs, dt, steps, re, path="resident")
    for r in range(2):
        g.launch()
        g.check()
        ft.evolve(refs, dt, steps, re, path="resident")
        torch.cuda.synchronize()
        for p, q, lat, y in zip(probs, refs, (la, lb, lc), ys):
            assert torch.equal(p.rho, q.rho)
            if r == 0:
                assert np.array_equal(unpack(_host(p.rho), lat.N), y.astype(cdt))
    g.close()

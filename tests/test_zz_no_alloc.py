"""ftwa_evolve_static, the entry point that allocates nothing (its workspace
is the library's static device array), against ftwa_evolve with a caller
workspace: bitwise the same states and moments, on two calls in a row, the
second with a smaller input; runs beyond the static array's size are refused
before anything is queued."""
import pytest

pytestmark = pytest.mark.gpu

FTWA_EINVAL = -1


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


def _pair(ft, lat, U, M, n0, dtype, seed):
    a = ft.Problem.allocate(lat, U, M, n0, dtype)
    b = ft.Problem.allocate(lat, U, M, n0, dtype)
    ft.sample(a, seed)
    ft.sample(b, seed)
    return a, b


def _same(x, y):
    import torch
    return torch.equal(x.view(-1), y.view(-1))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_static_workspace_matches_caller_workspace(ft, dtype):
    import torch
    # first call: 54-site torus (resident path), 1024 trajectories, 200 steps
    lat54 = ft.Lattice("torus", 3, 9)
    n0 = lat54.fock_start("random", 0x2212043520000002)
    a, b = _pair(ft, lat54, 3.3, 1024, n0, dtype, 11)
    ft.evolve(a, 0.01, 200, 10)
    b.ensure_moments(21)
    ft.ftwa_evolve_static([b.desc()], 0.01, 200, 10, dtype)
    ft.ftwa_evolve_check(None)
    torch.cuda.synchronize()
    assert _same(a.rho, b.rho) and _same(a.S1, b.S1) and _same(a.S2, b.S2)

    # second call, smaller: a ragged 300-trajectory 12-site instance on the
    # stream path next to a 100-trajectory 54-site instance, 100 steps
    lat12 = ft.Lattice("torus", 2, 3)
    n12 = lat12.fock_start("neel")
    c, d = _pair(ft, lat12, 1.7, 300, n12, dtype, 12)
    e, f = _pair(ft, lat54, 2.5, 100, n0, dtype, 13)
    ft.evolve(c, 0.01, 100, 10, path="stream")
    ft.evolve(e, 0.01, 100, 10)
    for p in (d, f):
        p.ensure_moments(11)
    ft.ftwa_evolve_static([d.desc()], 0.01, 100, 10, dtype, path="stream")
    ft.ftwa_evolve_check(None)
    ft.ftwa_evolve_static([f.desc()], 0.01, 100, 10, dtype)
    ft.ftwa_evolve_check(None)
    torch.cuda.synchronize()
    for x, y in ((c, d), (e, f)):
        assert _same(x.rho, y.rho) and _same(x.S1, y.S1) and _same(x.S2, y.S2)


def test_static_workspace_refuses_oversized_runs(ft):
    import torch
    lat = ft.Lattice("torus", 3, 9)
    p = ft.Problem.allocate(lat, 3.3, 65536, lat.fock_start("neel"), "f32")
    p.ensure_moments(201)
    p.S1.zero_()
    before = p.S1.clone()
    with pytest.raises(ft.FtwaError) as e:
        ft.ftwa_evolve_static([p.desc()], 0.01, 2000, 10, "f32")
    assert e.value.status == FTWA_EINVAL and "static" in str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(p.S1, before)

"""Parity of the split resident kernel (one spin block spread over two or
three workgroups that exchange their boundary elements every stage) with the
oracle, through the C ABI.  The split configurations take FP64 blocks too
large for one CU; they are forced here on lattices of several sizes, so that
strips, halos and the exchange of diagonals are exercised at more than one
shape.  The evolved states must equal the oracle's bitwise (same operation
order) and the moments agree to 1e-12.
"""
import numpy as np
import pytest

from tests._util import pack, unpack

pytestmark = pytest.mark.gpu

SPLIT2, SPLIT3, SPLIT4 = 19, 20, 21  # configurations (FP64): 2, 3 and 4 workgroups per spin block
SPLIT2W = 22  # two workgroups of 768 threads


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


def _run(ft, orc, kind, a, b, config, M, steps, re, U=3.3, t=1.0, seed=11, start="random"):
    import torch
    lat = ft.Lattice(kind, a, b, t)
    olat = orc.Lattice(kind, a, b, t)
    n0 = orc.fock_start(olat, start, seed)
    rho0 = orc.sample(olat, n0, seed, M)
    prob = ft.Problem.allocate(lat, U, M, n0, "f64")
    prob.rho.copy_(torch.from_numpy(pack(rho0)))
    print(f"split parity: {kind} {a}x{b} N={lat.N} config={config} M={M} steps={steps}",
          flush=True)
    ft.evolve(prob, 0.01, steps, re, path="resident", config=config)
    y_ref, X_ref, _ = orc.evolve(olat, U, rho0, 0.01, steps, re, precision="f64")
    got = unpack(_host(prob.rho), lat.N)
    assert np.array_equal(got, y_ref), np.max(np.abs(got - y_ref))
    S1r, S2r = orc.moments(X_ref)
    assert np.allclose(_host(prob.S1), S1r, rtol=1e-12, atol=1e-12)
    assert np.allclose(_host(prob.S2), S2r, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind,a,b,config", [("hex", 4, 0, SPLIT2), ("hex", 4, 0, SPLIT3),
                                             ("hex", 4, 0, SPLIT4), ("torus", 3, 9, SPLIT2),
                                             ("hex", 5, 0, SPLIT2), ("hex", 5, 0, SPLIT3),
                                             ("hex", 5, 0, SPLIT4), ("hex", 4, 0, SPLIT2W),
                                             ("hex", 5, 0, SPLIT2W), ("torus", 3, 9, SPLIT2W),
                                             ("armchair", 10, 20, SPLIT3),
                                             ("armchair", 10, 20, SPLIT4)])
def test_split_matches_oracle(ft, orc, kind, a, b, config):
    _run(ft, orc, kind, a, b, config, M=37, steps=12, re=4)


def test_two_part_split_is_the_automatic_fp64_choice_at_150_sites(ft, orc):
    """More trajectories than groups in flight (items are taken in turns),
    U = -2 and t = 0.7 (the general hopping variant), no forced configuration."""
    _run(ft, orc, "hex", 5, 0, -1, M=70, steps=6, re=3, U=-2.0, t=0.7, start="neel")


def test_three_part_split_takes_items_in_turns(ft, orc):
    _run(ft, orc, "armchair", 10, 20, SPLIT3, M=45, steps=5, re=5, U=2.5, start="neel")


def test_fp64_at_198_sites_takes_the_split_path_by_default(ft, orc):
    """No forced configuration: the resident path exists for the 198-site FP64
    block (three workgroups per spin block) and matches the oracle."""
    _run(ft, orc, "armchair", 10, 20, -1, M=9, steps=4, re=2, start="neel")

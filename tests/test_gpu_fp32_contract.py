"""The stated accuracy of the FP32 form: FP32 trajectories (FP64 moments)
against the FP64 run on identical samples, both through the library.

Contract (workloads.fp32_contract): the ensemble occupations n (Eq. (5)) and
connected correlations C stay within 1e-4 of FP64 up to t32(U) (the full
horizon at U/t = 1; t = 8 at U/t = 3.3, where the dynamics is chaotic), and
past t32 FP32 and FP64 are statistically equivalent estimates
(|d| <= 3 sqrt(2) SE for all but 1 % of the observables).  Run at the 54-site
torus workload (random half filling, 16384 trajectories, T = 20, U/t = 1 and
3.3) and on the first 2048 trajectories of the 198-site flake workload
(Neel start, U/t = 3.3, dt = 0.005 to T = 20).
"""
import numpy as np
import pytest

from workloads import FLAKE_198, FP32_HORIZON, MID_TORUS, fp32_contract

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


def _pair(ft, W, U, M, every=1):
    """FP64 and FP32 runs from the same samples: (n, C, S1, S2) per dtype on
    the host, records thinned to every `every`-th."""
    import torch
    lat = ft.Lattice(W.kind, W.a, W.b, W.t_hop)
    n0 = lat.fock_start(W.start, W.seed)
    out = {}
    for dtype in ("f64", "f32"):
        p = ft.Problem.allocate(lat, U, M, n0, dtype)
        ft.sample(p, W.seed)
        ft.evolve(p, W.dt, W.n_steps, W.record_every)
        n, C, _ = ft.observables(p)
        torch.cuda.synchronize()
        sl = slice(None, None, every)
        out[dtype] = (n[sl].cpu().numpy(), C[sl].cpu().numpy(), p.S1[sl].cpu().numpy(),
                      p.S2[sl].cpu().numpy())
        del p, n, C
    times = (np.arange(W.n_steps // W.record_every + 1) * W.record_every * W.dt)[::every]
    return out, times


def _report(tag, c):
    keys = ("max_abs_dn_to_t32", "max_abs_dC_to_t32", "frac_dn_over_3sqrt2_se",
            "frac_dC_over_3sqrt2_se", "max_z_dn", "max_z_dC")
    print(f"\n{tag}: t32 = {c['t32']}, " + ", ".join(f"{k} = {c[k]:.3g}" for k in keys if k in c))


@pytest.mark.parametrize("U", [1.0, 3.3])
def test_fp32_contract_torus54(ft, U):
    W = MID_TORUS
    runs, times = _pair(ft, W, U, W.n_traj)
    n64, C64, S1, S2 = runs["f64"]
    n32, C32, _, _ = runs["f32"]
    c = fp32_contract(n32, C32, n64, C64, S1, S2, W.n_traj, times, FP32_HORIZON[U])
    _report(f"torus54 U={U}", c)
    assert c["holds"], c


def test_fp32_contract_flake198(ft):
    W = FLAKE_198
    M = 2048
    runs, times = _pair(ft, W, W.U, M, every=2)
    n64, C64, S1, S2 = runs["f64"]
    n32, C32, _, _ = runs["f32"]
    c = fp32_contract(n32, C32, n64, C64, S1, S2, M, times, FP32_HORIZON[W.U])
    _report("flake198 U=3.3", c)
    assert c["holds"], c

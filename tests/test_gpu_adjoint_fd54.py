"""Central finite differences of the gradient workload's loss (54-site torus,
Neel start, 4096 trajectories, U/t = 2.5 against the U/t = 3.3 target, FP64)
against the FP64 adjoint at T = 5 (500 steps, checkpoints every 50): along U,
t and one random direction of the per-site offsets, h = 1e-6, to 1e-5
relative (the accuracy the discrete adjoint of Eq. (6)'s Runge-Kutta map must
reach where the dynamics has not yet amplified rounding).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_adjoint_54_site_central_differences():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    import paper_2212_04352_amd as ft
    from workloads import ADJOINT_54 as W
    ft.load()
    lat = ft.Lattice(W.kind, W.a, W.b, W.t_hop)
    steps, h = 500, 1e-6
    _, g = bench._occupation_grad(W, lat, steps, "f64", W.U)
    spec, target = bench._fd_setup(W, lat, steps)
    v = np.random.default_rng(W.seed).standard_normal(lat.N)
    vt = torch.from_numpy(v).cuda()

    def L(dU=0.0, dt=0.0, dd=0.0):
        with torch.no_grad():
            return bench._fd_loss(spec, target, lat, W.U + dU, W.t_hop + dt, dd * vt)
    fd = [(L(dU=h) - L(dU=-h)) / (2 * h), (L(dt=h) - L(dt=-h)) / (2 * h),
          (L(dd=h) - L(dd=-h)) / (2 * h)]
    ad = [g[0], g[1], float(np.dot(g[2:], v))]
    print(f"\nadjoint {ad}\ncentral differences {fd}")
    for a, f in zip(ad, fd):
        assert abs(a - f) <= 1e-5 * abs(a), (ad, fd)

"""Pins of the oracle's gradient of occupation losses (forward-mode tangent of
the FP64 Runge-Kutta trajectories), against quantities fixed independently of
the tangent code: central finite differences of the oracle's forward
evolution, linearity of the free (U = 0) flow, and the forward records."""
import numpy as np
import pytest


def _case(orc, kind, a, b, start, seed, M):
    lat = orc.Lattice(kind, a, b)
    n0 = orc.fock_start(lat, start, seed)
    rho0 = orc.sample(lat, n0, seed, M)
    return lat, rho0


def _loss(orc, lat, U, rho0, dt, ns, re, target, shift=None, t=None):
    lat_t = lat if t is None else orc.Lattice(lat.kind, lat.a, lat.b, t=t)
    r = rho0.copy()
    if shift is not None:
        for s in range(2):
            r[:, s, np.arange(lat.N), np.arange(lat.N)] += shift[s]
    _, X, _ = orc.evolve(lat_t, U, r, dt, ns, re)
    return float(np.sum((X.mean(axis=1) + 0.5 - target) ** 2))


@pytest.mark.parametrize("kind,a,b,start", [("torus", 2, 3, "neel"), ("hex", 2, 0, "random")])
def test_tangent_gradient_matches_central_differences(orc, kind, a, b, start):
    lat, rho0 = _case(orc, kind, a, b, start, 11, 12)
    dt, ns, re = 0.02, 80, 10
    X, _ = orc.evolve_tangent(lat, 3.3, rho0, dt, ns, re)
    target = X.mean(axis=1) + 0.5
    L, gU, gt, gs = orc.occupation_loss_grad(lat, 2.5, rho0, dt, ns, re, target)
    assert L > 1e-4
    eps = 1e-5
    fd_U = (_loss(orc, lat, 2.5 + eps, rho0, dt, ns, re, target)
            - _loss(orc, lat, 2.5 - eps, rho0, dt, ns, re, target)) / (2 * eps)
    fd_t = (_loss(orc, lat, 2.5, rho0, dt, ns, re, target, t=1 + eps)
            - _loss(orc, lat, 2.5, rho0, dt, ns, re, target, t=1 - eps)) / (2 * eps)
    v = np.random.default_rng(3).standard_normal((2, lat.N))
    fd_v = (_loss(orc, lat, 2.5, rho0, dt, ns, re, target, shift=eps * v)
            - _loss(orc, lat, 2.5, rho0, dt, ns, re, target, shift=-eps * v)) / (2 * eps)
    scale = max(abs(gU), abs(gt), np.max(np.abs(gs)))
    assert abs(gU - fd_U) <= 1e-7 * scale
    assert abs(gt - fd_t) <= 1e-7 * scale
    assert abs(np.sum(gs * v) - fd_v) <= 1e-7 * scale * np.sum(np.abs(v))


def test_tangent_of_free_flow_is_the_flow_of_the_direction(orc):
    """At U = 0 the map rho(0) -> rho(t) is linear, so the derivative along a
    shift of rho_ii,s(0) is the forward evolution of the unit matrix E_ii in
    block s, whatever rho(0) is."""
    lat, rho0 = _case(orc, "torus", 2, 3, "neel", 5, 3)
    N = lat.N
    dt, ns, re = 0.01, 50, 10
    for s, i in [(0, 0), (1, 7)]:
        e = np.zeros((2, N))
        e[s, i] = 1.0
        _, Xd = orc.evolve_tangent(lat, 0.0, rho0, dt, ns, re, dshift=e)
        E = np.zeros((1, 2, N, N), dtype=np.complex128)
        E[0, s, i, i] = 1.0
        _, Xe, _ = orc.evolve(lat, 0.0, E, dt, ns, re)
        for m in range(rho0.shape[0]):
            assert np.allclose(Xd[:, m], Xe[:, 0], rtol=0, atol=1e-13)


def test_tangent_records_follow_the_forward_evolution(orc):
    lat, rho0 = _case(orc, "hex", 2, 0, "random", 2, 5)
    X, Xd = orc.evolve_tangent(lat, 1.7, rho0, 0.01, 60, 10, dU=1.0)
    _, Xf, _ = orc.evolve(lat, 1.7, rho0, 0.01, 60, 10)
    assert np.allclose(X, Xf, rtol=0, atol=1e-12)
    assert np.all(Xd[0] == 0) and np.max(np.abs(Xd[-1])) > 1e-4


def test_gradient_vanishes_at_the_target(orc):
    lat, rho0 = _case(orc, "torus", 2, 3, "neel", 1, 4)
    X, _ = orc.evolve_tangent(lat, 3.3, rho0, 0.02, 40, 10)
    L, gU, gt, gs = orc.occupation_loss_grad(lat, 3.3, rho0, 0.02, 40, 10, X.mean(axis=1) + 0.5)
    assert L == 0.0 and gU == 0.0 and gt == 0.0 and np.all(gs == 0)

"""Batched runs (several instances per ftwa_evolve call), their HIP-graph form
and the autotuner.  The per-element arithmetic does not depend on how
instances are grouped into launches, on the kernel configuration or on the
pass split, so every batched trajectory must equal the one-instance run
bitwise; moments agree to FP64 summation order (1e-13)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


MIXED = [("torus", 2, 3, 3.3, 40), ("hex", 2, 0, 0.7, 33), ("torus", 3, 9, 2.1, 19),
         ("hex", 4, 0, 3.9, 9), ("hex", 5, 0, 1.2, 5), ("armchair", 10, 20, 3.3, 4)]


def _problems(ft, spec, dtype, seed=17):
    probs = []
    for k, (kind, a, b, U, M) in enumerate(spec):
        lat = ft.Lattice(kind, a, b)
        p = ft.Problem.allocate(lat, U, M, lat.fock_start("random", seed, k), dtype, instance=k)
        ft.sample(p, seed)
        probs.append(p)
    return probs


def _snapshot(probs):
    import torch
    torch.cuda.synchronize()
    return [(p.rho.cpu().numpy().copy(), p.S1.cpu().numpy().copy(), p.S2.cpu().numpy().copy())
            for p in probs]


def _clone(ft, probs):
    out = []
    for p in probs:
        q = ft.Problem.allocate(p.lat, p.U, p.n_traj, p.n0.cpu().numpy(), p.dtype,
                                instance=p.instance)
        q.rho.copy_(p.rho)
        out.append(q)
    return out


def _assert_same(a, b):
    for (ra, s1a, s2a), (rb, s1b, s2b) in zip(a, b):
        assert np.array_equal(ra, rb)
        assert np.allclose(s1a, s1b, rtol=1e-13, atol=1e-13)
        assert np.allclose(s2a, s2b, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_evolve_matches_per_instance_runs(ft, dtype):
    """Mixed sizes and U in one call: FP32 uses three resident groups (two
    spin-split); FP64 mixes one-CU resident groups with the two- and
    three-part split kernels (150 and 198 sites)."""
    probs = _problems(ft, MIXED, dtype)
    single = _clone(ft, probs)
    for q in single:
        ft.evolve(q, 0.01, 12, 4)
    ft.evolve(probs, 0.01, 12, 4)
    _assert_same(_snapshot(probs), _snapshot(single))


def test_batched_passes_split_trajectories(ft):
    """A forced small window (traj_chunk) splits every instance into several
    passes of one launch per group; results are unchanged."""
    probs = _problems(ft, MIXED[:4], "f32", seed=3)
    ref = _clone(ft, probs)
    ft.evolve(ref, 0.01, 10, 5)
    ft.evolve(probs, 0.01, 10, 5, traj_chunk=7)
    _assert_same(_snapshot(probs), _snapshot(ref))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_graph_replays_match_direct_runs(ft, dtype):
    """The captured graph, replayed three times with eager work and
    synchronisation in between, follows three direct ftwa_evolve calls (FP64:
    with the split kernel's groups, whose exchange areas are cleared by a
    fill kernel inside the graph)."""
    import torch
    probs = _problems(ft, MIXED, dtype, seed=29)
    ref = _clone(ft, probs)
    g = ft.EvolveGraph(probs, 0.01, 8, 4)
    for rep in range(3):
        g.launch()
        g.check()
        ft.evolve(ref, 0.01, 8, 4)
        torch.cuda.synchronize()
        _assert_same(_snapshot(probs), _snapshot(ref))
        # eager work on the same stream between replays
        probs[0].S1.mul_(1.0)
    g.close()


def test_graph_batch_workload_shape(ft):
    """The mixed-batch workload's draws (64 instances, sizes from
    {24, 54, 96, 150, 198}, U on [0, 4], random Fock starts) at 24
    trajectories each and 6 steps: one graph launch equals 64 direct runs."""
    import torch
    from workloads import batch_instances
    spec = [(d["kind"], d["a"], d["b"], d["U"], 24) for d in batch_instances(n_traj=24)]
    probs = _problems(ft, spec, "f32", seed=0x2212043520000004)
    ref = _clone(ft, probs)
    g = ft.EvolveGraph(probs, 0.01, 6, 3)
    g.launch()
    g.check()
    for q in ref:
        ft.evolve(q, 0.01, 6, 3)
    torch.cuda.synchronize()
    _assert_same(_snapshot(probs), _snapshot(ref))
    g.close()


def test_autotune_choices_fit_and_keep_results(ft):
    import torch
    probs = _problems(ft, [("hex", 2, 0, 1.0, 64), ("hex", 4, 0, 2.0, 32),
                           ("armchair", 10, 20, 3.3, 16)], "f32", seed=5)
    torch.cuda.synchronize()
    before = [p.rho.cpu().numpy().copy() for p in probs]
    ref = _clone(ft, probs)
    cfgs = ft.autotune(probs, probe_steps=4)
    assert len(cfgs) == 3
    # states untouched by the probes
    torch.cuda.synchronize()
    for r0, p in zip(before, probs):
        assert np.array_equal(r0, p.rho.cpu().numpy())
    for c, p in zip(cfgs, probs):
        if c >= 0:  # the choice is a configuration that fits this lattice
            ft.evolve(p, 0.01, 1, 1, path="resident", config=c)
    probs = _problems(ft, [("hex", 2, 0, 1.0, 64), ("hex", 4, 0, 2.0, 32),
                           ("armchair", 10, 20, 3.3, 16)], "f32", seed=5)
    ft.evolve(probs, 0.01, 10, 5)               # automatic plan: the tuned choices
    for q in ref:
        ft.evolve(q, 0.01, 10, 5, path="stream")
    _assert_same(_snapshot(probs), _snapshot(ref))

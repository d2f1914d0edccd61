"""The execution contract of the C ABI (include/ftwa.h) on the GPU.

  * ftwa_evolve queues a run and returns before the device has finished it
    (the stream still holds work), and ftwa_evolve_check then waits and
    reports the run's status;
  * the timeout path of the spin-split resident kernel: with the partners
    forced absent from the host (fault-injection flag and a short spin
    limit) every waiting workgroup gives up, exits, leaves rho untouched, and
    ftwa_evolve_check reports FTWA_ETIMEOUT; the next run is clean;
  * a lattice whose tables were not uploaded to the device is refused before
    anything is queued.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FTWA_EINVAL, FTWA_ETIMEOUT = -1, -6


@pytest.fixture(scope="module")
def ft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_04352_amd as ft
    ft.load()
    return ft


def test_evolve_returns_before_the_run_ends(ft):
    """198-site flake, FP32, 16384 trajectories x 400 steps (about a second
    of device time): the call returns while the stream is still busy."""
    import torch
    lat = ft.Lattice("armchair", 10, 20)
    n0 = lat.fock_start("neel")
    prob = ft.Problem.allocate(lat, 3.3, 16384, n0, "f32")
    ft.sample(prob, 0x2212043520000003)
    ws = ft.evolve(prob, 0.005, 400, 10)  # warm-up and workspace, checked
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    ws = ft.evolve(prob, 0.005, 400, 10, workspace=ws, check=False)
    t_call = time.perf_counter() - t0
    busy = not stream.query()
    t1 = time.perf_counter()
    ft.ftwa_evolve_check(ws)  # waits, then reads the status block
    t_run = time.perf_counter() - t0
    print(f"\nftwa_evolve returned after {1e3 * t_call:.2f} ms; run done after {1e3 * t_run:.1f} ms "
          f"(check waited {1e3 * (time.perf_counter() - t1):.1f} ms)")
    assert busy, "the stream had finished when ftwa_evolve returned"
    assert stream.query()
    assert t_call < 0.25 * t_run


def test_timeout_path_reports_etimeout(ft):
    """Partners absent (only the up-spin workgroups of eight pairs run) and
    100 polls per wait: each workgroup gives up its first wait and exits."""
    import torch
    lat = ft.Lattice("armchair", 10, 20)
    n0 = lat.fock_start("neel")
    prob = ft.Problem.allocate(lat, 3.3, 64, n0, "f32")
    ft.sample(prob, 0x2212043520000003)
    torch.cuda.synchronize()
    before = prob.rho.clone()
    with pytest.raises(ft.FtwaError) as e:
        ft.evolve(prob, 0.005, 20, 10, path="resident", spin_limit=100, drop_partners=True)
    assert e.value.status == FTWA_ETIMEOUT, str(e.value)
    torch.cuda.synchronize()
    assert torch.equal(prob.rho, before)
    # the same problem runs normally afterwards and the status is clean again
    ft.evolve(prob, 0.005, 20, 10, path="resident")
    torch.cuda.synchronize()
    assert not torch.equal(prob.rho, before)
    assert np.isfinite(prob.rho.cpu().numpy()).all()


def test_not_uploaded_lattice_is_refused(ft):
    import torch
    lat = ft.Lattice("torus", 2, 3)
    prob = ft.Problem.allocate(lat, 3.3, 8, lat.fock_start("neel"), "f64")
    other = ft.Lattice("torus", 2, 3)  # same graph, never uploaded
    d = prob.desc()
    d["lat"] = other.handle
    prob.ensure_moments(2)
    d["S1"], d["S2"] = prob.S1, prob.S2
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    with pytest.raises(ft.FtwaError) as e:
        ft.ftwa_evolve([d], 0.01, 10, 10, "f64", ws)
    assert e.value.status == FTWA_EINVAL and "ftwa_lattice_upload" in str(e.value)
    with pytest.raises(ft.FtwaError) as e:
        ft.ftwa_sample([d], 1, "f64")
    assert e.value.status == FTWA_EINVAL

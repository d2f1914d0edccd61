"""MI355X (gfx950) fTWA hot path: Gaussian sampling of the one-body phase-space
matrix around a Fock state, RK4 trajectories of the fTWA equation of motion on
honeycomb lattices, and FP64 ensemble moments -> occupations, connected
density-density correlations and g2.

Paper: Rousse, Eriksson, Ogren, "Correlated quantum dynamics of graphene",
arXiv:2212.04352 (Sec. III, Eqs. (6)-(7) and (10)).

All computation runs in the HIP library libftwa.so (include/ftwa.h); this
package marshals torch tensors (device memory, streams) into it.  Importing
works without a GPU; calls that queue device work need one.
"""
from __future__ import annotations

from dataclasses import dataclass

from ._binding import (DTYPE, FtwaError, exiting, ftwa_adjoint,  # noqa: F401
                       ftwa_adjoint_workspace_size, ftwa_autotune, ftwa_autotune_workspace_size,
                       ftwa_build_lattice, ftwa_build_lattice_bonds, ftwa_evolve,
                       ftwa_evolve_check, ftwa_evolve_graph, ftwa_evolve_static,
                       ftwa_evolve_workspace_size,
                       ftwa_fock_start, ftwa_free_lattice, ftwa_graph_check, ftwa_graph_free,
                       ftwa_graph_launch, ftwa_lattice_info, ftwa_lattice_upload,
                       ftwa_last_error, ftwa_observables, ftwa_sample, ftwa_sample_thermal,
                       ftwa_unpack, load, new_timing)


def packed_count(N: int) -> int:
    return N * (N + 1) // 2


def n_records(n_steps: int, record_every: int) -> int:
    return n_steps // record_every + 1


class Lattice:
    """Owns an ftwa_lattice handle."""

    def __init__(self, kind: str, a: int, b: int = 0, t: float = 1.0, *, bonds=None,
                 sublattice=None, n_sites: int = 0):
        if kind == "custom":
            self.handle = ftwa_build_lattice_bonds(n_sites, bonds, sublattice, t)
        else:
            self.handle = ftwa_build_lattice(kind, a, b, t)
        self.kind, self.a, self.b, self.t = kind, a, b, float(t)
        self.N, self.n_bonds, self.nbr, self.deg, self.sub = ftwa_lattice_info(self.handle)

    def fock_start(self, kind: str = "neel", seed: int = 0, instance: int = 0):
        return ftwa_fock_start(self.handle, kind, seed, instance)

    def upload(self) -> None:
        """ftwa_lattice_upload on the current device (once; later calls return at once)."""
        ftwa_lattice_upload(self.handle)

    def close(self) -> None:
        """Releases the handle and its device tables now."""
        h = getattr(self, "handle", None)
        self.handle = None
        if h and ftwa_free_lattice is not None:
            ftwa_free_lattice(h)

    def __del__(self):
        # at interpreter exit the handle is left to the process's end
        if exiting is None or exiting():
            return
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Problem:
    """Device buffers of one instance (torch tensors on the current GPU)."""
    lat: Lattice
    U: float
    n_traj: int
    dtype: str
    n0: object
    rho: object
    S1: object = None
    S2: object = None
    traj_offset: int = 0
    instance: int = 0
    track_invariants: bool = False
    inv: object = None
    n_shift: object = None   # optional [2, N] FP64 device tensor (see ftwa_instance)
    v_site: object = None    # optional [N] FP64 device tensor: external potential profile
    v_env: object = None     # with v_site: [2 n_steps + 1] FP64 envelope at half steps
    u_mat: object = None     # optional [N, N] FP64 device tensor: general interaction u_ij
    hop_w: object = None     # optional [2 n_steps + 1, N, 3] complex128 device tensor:
                             # complex hopping ratios j_ik / t at half steps (Peierls)

    @classmethod
    def allocate(cls, lat: Lattice, U: float, n_traj: int, n0, dtype: str = "f64",
                 traj_offset: int = 0, instance: int = 0, device=None,
                 track_invariants: bool = False):
        import torch
        cdt = torch.complex128 if dtype == "f64" else torch.complex64
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(dev):
            lat.upload()
        n0_t = torch.as_tensor(n0, dtype=torch.float64).reshape(2, lat.N).to(dev).contiguous()
        rho = torch.empty((2, packed_count(lat.N), n_traj), dtype=cdt, device=dev)
        return cls(lat, float(U), int(n_traj), dtype, n0_t, rho, traj_offset=traj_offset,
                   instance=instance, track_invariants=track_invariants)

    def desc(self):
        return {"lat": self.lat.handle, "U": self.U, "n_traj": self.n_traj,
                "traj_offset": self.traj_offset, "instance": self.instance, "n0": self.n0,
                "rho": self.rho, "S1": self.S1, "S2": self.S2, "inv": self.inv,
                "n_shift": self.n_shift, "v_site": self.v_site, "v_env": self.v_env,
                "u_mat": self.u_mat, "hop_w": self.hop_w}

    def ensure_moments(self, n_rec: int):
        import torch
        D = 2 * self.lat.N
        if self.S1 is None or self.S1.shape[0] != n_rec:
            self.S1 = torch.empty((n_rec, D), dtype=torch.float64, device=self.rho.device)
            self.S2 = torch.empty((n_rec, D * (D + 1) // 2), dtype=torch.float64,
                                  device=self.rho.device)
        if self.track_invariants and (self.inv is None or self.inv.shape[0] != n_rec):
            # per record: max trace drift, max Weyl-energy drift, max Frobenius
            # drift (all vs record 0), number of non-finite trajectories
            self.inv = torch.empty((n_rec, 4), dtype=torch.float64, device=self.rho.device)


def sample(problems, seed: int, stream=None, thermal: bool = False) -> None:
    """ftwa_sample, or ftwa_sample_thermal (diagonal fluctuations of a
    thermal initial state) when `thermal`."""
    problems = problems if isinstance(problems, (list, tuple)) else [problems]
    dt = problems[0].dtype
    fn = ftwa_sample_thermal if thermal else ftwa_sample
    fn([p.desc() for p in problems], seed, dt, stream)


def evolve(problems, dt: float, n_steps: int, record_every: int = 10, path: str = "auto",
           traj_chunk: int = 0, workspace=None, stream=None, timing=None, config: int = -1,
           check: bool = True, spin_limit: int = 0, drop_partners: bool = False):
    """Runs ftwa_evolve; allocates the workspace as a torch tensor unless given.
    check: then waits for the stream and raises what ftwa_evolve_check
    reports (a timed-out wait, non-finite trajectories); with check=False the
    call returns as soon as the run is queued (call ftwa_evolve_check on the
    returned workspace later)."""
    import torch
    problems = problems if isinstance(problems, (list, tuple)) else [problems]
    dtype = problems[0].dtype
    n_rec = n_records(n_steps, record_every)
    for p in problems:
        p.ensure_moments(n_rec)
    descs = [p.desc() for p in problems]
    nbytes = ftwa_evolve_workspace_size(descs, n_steps, record_every, dtype, path, traj_chunk,
                                        config)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=problems[0].rho.device)
    ftwa_evolve(descs, dt, n_steps, record_every, dtype, workspace, path, traj_chunk, stream,
                timing, config, spin_limit, drop_partners)
    if check:
        ftwa_evolve_check(workspace, stream)
    return workspace


class EvolveGraph:
    """A whole ftwa_evolve run of one or more instances captured as one HIP
    graph (ftwa_evolve_graph).  launch() integrates the current states for
    n_steps steps and refills the moments; check() waits and reports spin-split
    timeouts and non-finite trajectories.  Keeps the problems and the
    workspace alive while it exists."""

    def __init__(self, problems, dt: float, n_steps: int, record_every: int = 10,
                 path: str = "auto", traj_chunk: int = 0, config: int = -1, stream=None):
        import torch
        problems = list(problems) if isinstance(problems, (list, tuple)) else [problems]
        self.problems = problems
        self.dtype = problems[0].dtype
        n_rec = n_records(n_steps, record_every)
        for p in problems:
            p.ensure_moments(n_rec)
        descs = [p.desc() for p in problems]
        nbytes = ftwa_evolve_workspace_size(descs, n_steps, record_every, self.dtype, path,
                                            traj_chunk, config)
        self.workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8,
                                     device=problems[0].rho.device)
        self.handle = ftwa_evolve_graph(descs, dt, n_steps, record_every, self.dtype,
                                        self.workspace, path, traj_chunk, config, stream)

    def launch(self, stream=None) -> None:
        ftwa_graph_launch(self.handle, stream)

    def check(self, stream=None) -> None:
        ftwa_graph_check(self.handle, stream)

    def close(self) -> None:
        h = getattr(self, "handle", None)
        self.handle = None
        if h and ftwa_graph_free is not None:
            ftwa_graph_free(h)

    def __del__(self):
        if exiting is None or exiting():
            return
        try:
            self.close()
        except Exception:
            pass


def autotune(problems, probe_steps: int = 10, stream=None):
    """Times the kernel configurations that fit each distinct lattice of the
    problems on copies of their first trajectories (states are not modified)
    and records the fastest for later automatic plans; returns the chosen
    configuration per problem (-1 = stream path)."""
    import torch
    problems = problems if isinstance(problems, (list, tuple)) else [problems]
    dtype = problems[0].dtype
    descs = [p.desc() for p in problems]
    nbytes = ftwa_autotune_workspace_size(descs, dtype, probe_steps)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=problems[0].rho.device)
    return ftwa_autotune(descs, dtype, probe_steps, ws, stream)


def observables(problem: Problem, n_total: int = None, stream=None):
    """(n [n_rec, 2N], C [n_rec, 2N, 2N], g2 [n_rec, 2N, 2N]) on the device."""
    import torch
    N = problem.lat.N
    D = 2 * N
    n_rec = problem.S1.shape[0]
    M = problem.n_traj if n_total is None else n_total
    dev = problem.S1.device
    n = torch.empty((n_rec, D), dtype=torch.float64, device=dev)
    C = torch.empty((n_rec, D, D), dtype=torch.float64, device=dev)
    g2 = torch.empty((n_rec, D, D), dtype=torch.float64, device=dev)
    ftwa_observables(N, M, n_rec, problem.S1, problem.S2, n, C, g2, stream)
    return n, C, g2


def adjoint(problem: Problem, dt: float, n_steps: int, record_every: int, ckpt_every: int,
            dL_dnbar, n_total: int = None, traj_chunk: int = 0, workspace=None, stream=None):
    """Gradient [2 + 2N] (dL/dU, dL/dt, dL/dn_shift[2][N]) of a loss of the
    ensemble occupations, given dL/dnbar [n_rec, 2N] (FP64, device), by the
    discrete adjoint of the Runge-Kutta map (ftwa_adjoint).  problem.rho must
    hold rho(0) as sampled; it is not modified.  Returns (grad, workspace)."""
    import torch
    M = problem.n_traj if n_total is None else n_total
    d = problem.desc()
    nbytes = ftwa_adjoint_workspace_size(d, n_steps, record_every, ckpt_every, problem.dtype,
                                         traj_chunk)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=problem.rho.device)
    grad = torch.empty(2 + 2 * problem.lat.N, dtype=torch.float64, device=problem.rho.device)
    dL = dL_dnbar.to(device=problem.rho.device, dtype=torch.float64).contiguous()
    ftwa_adjoint(d, dt, n_steps, record_every, ckpt_every, problem.dtype, M, dL, grad, workspace,
                 traj_chunk, stream)
    return grad, workspace


def unpack(problem: Problem, stream=None):
    """Full matrices [n_traj, 2, N, N] complex of the packed state."""
    import torch
    N = problem.lat.N
    out = torch.empty((problem.n_traj, 2, N, N), dtype=problem.rho.dtype, device=problem.rho.device)
    ftwa_unpack(N, problem.n_traj, problem.dtype, problem.rho, out, stream)
    return out

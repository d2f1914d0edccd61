"""torch.autograd interface to the adjoint of libftwa.

`occupations(U, t, shift, spec)` returns the ensemble site occupations
nbar[r, s*N + i] (Eq. (5) of arXiv:2212.04352) at the records
t_r = r * record_every * dt as a differentiable function of the interaction
U, the hopping t and the shift of the initial diagonal rho_ii,s(0) (shape
[2, N]; a per-site shift delta_i is delta.expand(2, N)).  The sampled
off-diagonal noise is held fixed.  The forward pass runs ftwa_sample,
ftwa_evolve and ftwa_observables; the backward pass re-samples rho(0) and
runs ftwa_adjoint (discrete adjoint of the Runge-Kutta map, checkpointed).
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import Lattice, Problem, adjoint, evolve, ftwa_observables, n_records, sample


@dataclass
class OccupationSpec:
    """Fixed (non-differentiated) description of the ensemble."""
    kind: str
    a: int
    b: int
    n0: object                 # [2, N] initial Fock occupations (host array)
    seed: int
    n_traj: int
    dt: float
    n_steps: int
    record_every: int = 10
    dtype: str = "f32"
    ckpt_every: int = 50
    path: str = "auto"         # forward kernel path
    traj_chunk: int = 0        # adjoint trajectories per pass (0 = all)
    instance: int = 0
    _lattices: dict = field(default_factory=dict, repr=False)

    def lattice(self, t: float) -> Lattice:
        lat = self._lattices.get(t)
        if lat is None:
            lat = Lattice(self.kind, self.a, self.b, t)
            self._lattices[t] = lat
        return lat

    def problem(self, U: float, t: float, shift, device) -> Problem:
        import torch
        lat = self.lattice(t)
        prob = Problem.allocate(lat, U, self.n_traj, self.n0, self.dtype, instance=self.instance,
                                device=device)
        prob.n_shift = shift.detach().to(device=device, dtype=torch.float64).reshape(
            2, lat.N).contiguous()
        sample(prob, self.seed)
        return prob


class OccupationDynamics:
    """Namespace holding the autograd.Function (built lazily so that importing
    this module does not import torch)."""
    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is not None:
            return cls._fn
        import torch

        class _Occupations(torch.autograd.Function):
            @staticmethod
            def forward(ctx, U, t, shift, spec):
                dev = shift.device
                prob = spec.problem(float(U), float(t), shift, dev)
                evolve(prob, spec.dt, spec.n_steps, spec.record_every, path=spec.path)
                N = prob.lat.N
                n_rec = n_records(spec.n_steps, spec.record_every)
                nbar = torch.empty((n_rec, 2 * N), dtype=torch.float64, device=dev)
                ftwa_observables(N, spec.n_traj, n_rec, prob.S1, prob.S2, nbar)
                ctx.spec = spec
                ctx.values = (float(U), float(t))
                ctx.like = tuple((x.device, x.dtype) if torch.is_tensor(x) else None
                                 for x in (U, t))
                ctx.save_for_backward(shift.detach().clone())
                return nbar

            @staticmethod
            def backward(ctx, g):
                spec = ctx.spec
                (shift,) = ctx.saved_tensors
                U, t = ctx.values
                prob = spec.problem(U, t, shift, shift.device)  # rho(0) again
                grad, _ = adjoint(prob, spec.dt, spec.n_steps, spec.record_every,
                                  spec.ckpt_every, g.contiguous(), traj_chunk=spec.traj_chunk)
                N = prob.lat.N

                def like(g, k):  # gradient on the device and dtype of its input
                    return None if ctx.like[k] is None else g.to(*ctx.like[k])
                gs = grad[2:].reshape(2, N).to(dtype=shift.dtype)
                return like(grad[0], 0), like(grad[1], 1), gs, None

        cls._fn = _Occupations
        return cls._fn


def occupations(U, t, shift, spec: OccupationSpec):
    """nbar [n_rec, 2N] (FP64, on shift's device), differentiable in U, t and
    shift (0-d tensors and a [2, N] tensor)."""
    return OccupationDynamics.function().apply(U, t, shift, spec)

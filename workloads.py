"""Seeded synthetic workloads of the fTWA hot path (inputs only).

This module defines the problem instances that tests and the benchmark run:
lattice family and size, hopping t, interaction U, Fock start, trajectory
count, time step and horizon, record cadence and seed.  It holds none of the
method's arithmetic and imports neither the library nor the oracle; both
sides receive these parameters.

The paper (arXiv:2212.04352) runs a 10-site two-hexagon cluster with 10^5
trajectories up to t = 5 and a 198-site honeycomb flake from a Neel-like
start (Sec. IV-V), with J = U; it names no integrator, step or trajectory
count for the large system.  The workloads below keep its geometry family and
sizes (up to 198 sites) and fix the unstated parameters.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    kind: str            # "torus" | "armchair" | "hex"
    a: int
    b: int
    U: float
    n_traj: int
    dt: float
    n_steps: int
    start: str           # "neel" | "random"
    seed: int
    record_every: int = 10
    t_hop: float = 1.0
    dtypes: tuple = ("f64",)
    extra_U: tuple = field(default_factory=tuple)

    @property
    def horizon(self) -> float:
        return self.dt * self.n_steps


# 12-site 2x3 torus, Neel, U/t = 3.3, 1024 trajectories, dt = 0.01 to T = 10, FP64
SMALL_TORUS = Workload("torus12_neel_fp64", "torus", 2, 3, 3.3, 1024, 0.01, 1000, "neel",
                       0x2212043520000001)
# 54-site 3x9 torus, random half filling, U/t in {1, 3.3}, 16384 trajectories, T = 20,
# FP64 and FP32 on identical samples
MID_TORUS = Workload("torus54_random_fp32_vs_fp64", "torus", 3, 9, 3.3, 16384, 0.01, 2000,
                     "random", 0x2212043520000002, dtypes=("f64", "f32"), extra_U=(1.0,))
# 198-site open flake (10 x 20 brick wall, trimmed), Neel, U/t = 3.3, 32768 trajectories,
# dt = 0.005 to T = 20, FP32 and FP64
FLAKE_198 = Workload("flake198_neel", "armchair", 10, 20, 3.3, 32768, 0.005, 4000, "neel",
                     0x2212043520000003, dtypes=("f32", "f64"))
# adjoint workload: 54-site torus, Neel, 4096 trajectories, 2000 steps
ADJOINT_54 = Workload("torus54_adjoint", "torus", 3, 9, 2.5, 4096, 0.01, 2000, "neel",
                      0x2212043520000005, dtypes=("f32",))

BATCH_SEED = 0x2212043520000004
BATCH_SIZES = (24, 54, 96, 150, 198)


def batch_instances(n_inst: int = 64, seed: int = BATCH_SEED, n_traj: int = 2048):
    """Mixed batch: site counts drawn uniformly from {24, 54, 96, 150, 198}
    (hex flakes of 2..5 rings and the 198-site flake), U/t uniform on [0, 4],
    random half-filled Fock starts (instance k uses instance id k)."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice(BATCH_SIZES, size=n_inst)
    Us = rng.uniform(0.0, 4.0, size=n_inst)
    out = []
    for k, (n, U) in enumerate(zip(sizes, Us)):
        if n == 198:
            geo = ("armchair", 10, 20)
        else:
            rings = {24: 2, 54: 3, 96: 4, 150: 5}[int(n)]
            geo = ("hex", rings, 0)
        out.append({"kind": geo[0], "a": geo[1], "b": geo[2], "U": float(U), "n_traj": n_traj,
                    "instance": k, "start": "random"})
    return out


# ---------------------------------------------------------------------------
# FP32 form: the stated accuracy against FP64 on identical samples.
#
# Up to the horizon t32(U) the FP32 ensemble observables stay within 1e-4
# (absolute) of the FP64 ones: max over sites of |n32 - n64| and over pairs
# a != b of |C32 - C64|.  At U/t = 3.3 the trajectories are chaotic (a
# rounding difference grows by ~1e7 by t = 20 in either precision), so past
# t32 the two runs are compared as statistically equivalent estimates of the
# same means: |dn_a| <= 3 sqrt(2) SE_a, with SE_a^2 = Var(x_a) / M from the
# FP64 moments; and |dC_ab| <= 3 sqrt(2) SE_ab with the Gaussian (Isserlis)
# SE_ab^2 = (Var_a Var_b + C_ab^2) / M.  Both must hold for all but 1 % of the
# (record, observable) pairs past t32.
FP32_HORIZON = {1.0: 20.0, 3.3: 8.0}
FP32_ABS_TOL = 1e-4
FP32_SE_FACTOR = 3.0
FP32_SE_EXCEED = 0.01


def fp32_contract(n32, C32, n64, C64, S1_64, S2_64, M, times, t32):
    """Acceptance statistics of the FP32 form (see above).  Arrays: n [R, D],
    C [R, D, D], S1 [R, D], S2 packed upper [R, D(D+1)/2] (FP64 run), times
    [R].  Returns a dict of the figures and `holds`."""
    n32, C32, n64, C64 = (np.asarray(x, dtype=np.float64) for x in (n32, C32, n64, C64))
    S1, S2 = np.asarray(S1_64, np.float64), np.asarray(S2_64, np.float64)
    times = np.asarray(times, np.float64)
    R, D = n64.shape
    diag = np.array([a * D - a * (a - 1) // 2 for a in range(D)])
    mean = S1 / M
    var = np.maximum(S2[:, diag] / M - mean * mean, 0.0)
    off = ~np.eye(D, dtype=bool)
    dn = np.abs(n32 - n64)
    dC = np.abs(C32 - C64)
    early = times <= t32 + 1e-9
    late = ~early
    out = {"t32": t32, "trajectories": int(M),
           "max_abs_dn_to_t32": float(dn[early].max()),
           "max_abs_dC_to_t32": float(dC[early][:, off].max())}
    ok = out["max_abs_dn_to_t32"] <= FP32_ABS_TOL and out["max_abs_dC_to_t32"] <= FP32_ABS_TOL
    if late.any():
        se_n = np.sqrt(var / M)
        zn = dn[late] / (np.sqrt(2.0) * np.maximum(se_n[late], 1e-300))
        se_C = np.sqrt((var[:, :, None] * var[:, None, :] + C64 * C64) / M)
        zC = (dC[late] / (np.sqrt(2.0) * np.maximum(se_C[late], 1e-300)))[:, off]
        out.update({"max_abs_dn_after_t32": float(dn[late].max()),
                    "frac_dn_over_3sqrt2_se": float(np.mean(zn > FP32_SE_FACTOR)),
                    "frac_dC_over_3sqrt2_se": float(np.mean(zC > FP32_SE_FACTOR)),
                    "max_z_dn": float(zn.max()), "max_z_dC": float(zC.max())})
        ok = ok and out["frac_dn_over_3sqrt2_se"] <= FP32_SE_EXCEED \
            and out["frac_dC_over_3sqrt2_se"] <= FP32_SE_EXCEED
    out["holds"] = bool(ok)
    return out

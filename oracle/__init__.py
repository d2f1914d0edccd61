"""CPU oracle for the fTWA hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

The arithmetic lives in ``ftwa_oracle.c`` (plain loops, FP64 unless FP32 is
asked for); this module compiles it with gcc when needed and wraps it with
ctypes, returning numpy arrays.  Full-matrix storage is used throughout:
one trajectory is ``rho[spin, i, j]`` complex, spin 0 = up, 1 = down.

Paper: Rousse, Eriksson, Ogren, "Correlated quantum dynamics of graphene"
(arXiv:2212.04352).  Each wrapper names the passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "ftwa_oracle.c"), os.path.join(_HERE, "ftwa_oracle_evolve.h")]
_LIB_PATH = os.path.join(_HERE, "libftwa_oracle.so")

MAXDEG = 3
KIND = {"torus": 0, "armchair": 1, "hex": 2}
START = {"neel": 0, "random": 1}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, FMA instructions, no contraction)."""
    stale = not os.path.exists(_LIB_PATH) or any(
        os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SRC)
    if force or stale:
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-mfma", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC[0], "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    i32, i64, u32, u64, dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                               ctypes.c_uint64, ctypes.c_double)
    lib.oracle_philox4x32_10.argtypes = [P(u32), P(u32), P(u32)]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_build_lattice.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         P(ctypes.c_int), P(i32), P(ctypes.c_uint8),
                                         P(ctypes.c_uint8), P(ctypes.c_int)]
    lib.oracle_fock_start.argtypes = [ctypes.c_int, P(ctypes.c_uint8), ctypes.c_int, u64, u32,
                                      P(dbl)]
    lib.oracle_complex_normal.argtypes = [u64, u32, u32, u32, P(dbl), P(dbl)]
    lib.oracle_complex_normal.restype = None
    lib.oracle_sample.argtypes = [ctypes.c_int, P(dbl), u64, u32, i64, i64, ctypes.c_int, P(dbl)]
    lib.oracle_real_normal.argtypes = [u64, u32, u32, u32, u32]
    lib.oracle_real_normal.restype = dbl
    lib.oracle_sample.restype = None
    for suffix, real in (("f64", dbl), ("f32", ctypes.c_float)):
        rhs = getattr(lib, f"oracle_rhs_{suffix}")
        rhs.argtypes = [ctypes.c_int, P(i32), P(ctypes.c_uint8), real, real, P(real), P(real)]
        rhs.restype = None
        ev = getattr(lib, f"oracle_evolve_{suffix}")
        ev.argtypes = [ctypes.c_int, P(i32), P(ctypes.c_uint8), dbl, dbl, dbl, i64, ctypes.c_int,
                       i64, P(dbl), P(dbl), P(dbl)]
        ev.restype = ctypes.c_int
        evp = getattr(lib, f"oracle_evolve_pot_{suffix}")
        evp.argtypes = [ctypes.c_int, P(i32), P(ctypes.c_uint8), dbl, dbl, P(dbl), P(dbl), dbl,
                        i64, ctypes.c_int, i64, P(dbl), P(dbl), P(dbl)]
        evp.restype = ctypes.c_int
        evg = getattr(lib, f"oracle_evolve_gen_{suffix}")
        evg.argtypes = [ctypes.c_int, P(i32), P(ctypes.c_uint8), dbl, dbl, P(dbl), P(dbl),
                        P(dbl), dbl, i64, ctypes.c_int, i64, P(dbl), P(dbl), P(dbl)]
        evg.restype = ctypes.c_int
        evh = getattr(lib, f"oracle_evolve_hop_{suffix}")
        evh.argtypes = [ctypes.c_int, P(i32), P(ctypes.c_uint8), dbl, dbl, P(dbl), P(dbl),
                        P(dbl), P(dbl), dbl, i64, ctypes.c_int, i64, P(dbl), P(dbl), P(dbl)]
        evh.restype = ctypes.c_int
    lib.oracle_moments.argtypes = [ctypes.c_int, i64, ctypes.c_int, P(dbl), P(dbl), P(dbl)]
    lib.oracle_moments.restype = None
    lib.oracle_observables.argtypes = [ctypes.c_int, i64, ctypes.c_int, P(dbl), P(dbl), P(dbl),
                                       P(dbl), P(dbl)]
    lib.oracle_observables.restype = None
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_num_threads.restype = None
    lib.oracle_evolve_tangent.argtypes = [ctypes.c_int, P(i32), P(ctypes.c_uint8), dbl, dbl, dbl,
                                          i64, ctypes.c_int, i64, P(dbl), dbl, dbl, P(dbl),
                                          P(dbl), P(dbl)]
    lib.oracle_evolve_tangent.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


# --------------------------------------------------------------------------
# Random numbers (convention of this project; the paper names no generator)
# --------------------------------------------------------------------------
def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    lib = _load()
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                             _ptr(out, ctypes.c_uint32))
    return out


def complex_normal(seed: int, c0: int, c1: int, c2: int) -> complex:
    """One Box-Muller complex normal xi (E|xi|^2 = 1) from counter (c0, c1, c2, 0)."""
    lib = _load()
    re, im = ctypes.c_double(), ctypes.c_double()
    lib.oracle_complex_normal(ctypes.c_uint64(seed), c0, c1, c2, ctypes.byref(re),
                              ctypes.byref(im))
    return complex(re.value, im.value)


# --------------------------------------------------------------------------
# Lattice (Sec. II) and Fock start (Sec. IV.A)
# --------------------------------------------------------------------------
class Lattice:
    def __init__(self, kind: str, a: int, b: int, t: float = 1.0, max_sites: int = 4096):
        lib = _load()
        nbr = np.full(max_sites * MAXDEG, -1, dtype=np.int32)
        deg = np.zeros(max_sites, dtype=np.uint8)
        sub = np.zeros(max_sites, dtype=np.uint8)
        n = ctypes.c_int()
        nb = ctypes.c_int()
        rc = lib.oracle_build_lattice(KIND[kind], int(a), int(b), max_sites, ctypes.byref(n),
                                      _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8),
                                      _ptr(sub, ctypes.c_uint8), ctypes.byref(nb))
        if rc != 0:
            raise ValueError(f"oracle lattice build failed ({rc}) for {kind} {a}x{b}")
        self.kind, self.a, self.b, self.t = kind, a, b, float(t)
        self.N = n.value
        self.n_bonds = nb.value
        self.nbr = nbr[: self.N * MAXDEG].reshape(self.N, MAXDEG).copy()
        self.deg = deg[: self.N].copy()
        self.sub = sub[: self.N].copy()

    @classmethod
    def from_bonds(cls, N: int, bonds, sub, t: float = 1.0) -> "Lattice":
        """A graph given by its bond list (degree <= 3), e.g. small rings."""
        lat = cls.__new__(cls)
        lat.kind, lat.a, lat.b, lat.t = "custom", N, 0, float(t)
        lat.N = int(N)
        nb = [[] for _ in range(N)]
        for u, v in bonds:
            if u == v or v in nb[u]:
                raise ValueError("bad bond")
            nb[u].append(v)
            nb[v].append(u)
        if max(len(x) for x in nb) > MAXDEG:
            raise ValueError("degree above 3")
        lat.nbr = np.full((N, MAXDEG), -1, dtype=np.int32)
        lat.deg = np.zeros(N, dtype=np.uint8)
        for i in range(N):
            lst = sorted(nb[i])
            lat.nbr[i, : len(lst)] = lst
            lat.deg[i] = len(lst)
        lat.sub = np.asarray(sub, dtype=np.uint8).copy()
        lat.n_bonds = len(bonds)
        return lat

    def hopping_matrix(self) -> np.ndarray:
        """Dense J with J_ij = t on bonds (the j_ij of Eq. (1))."""
        J = np.zeros((self.N, self.N))
        for i in range(self.N):
            for n in range(self.deg[i]):
                J[i, self.nbr[i, n]] = self.t
        return J

    def bonds(self):
        return [(i, int(k)) for i in range(self.N) for k in self.nbr[i, : self.deg[i]] if i < k]


def fock_start(lat: Lattice, kind: str = "neel", seed: int = 0, instance: int = 0) -> np.ndarray:
    """Initial occupations n0[spin, site] of a singly occupied Fock state."""
    lib = _load()
    n0 = np.zeros(2 * lat.N, dtype=np.float64)
    sub = np.ascontiguousarray(lat.sub)
    rc = lib.oracle_fock_start(lat.N, _ptr(sub, ctypes.c_uint8), START[kind],
                               ctypes.c_uint64(seed), instance, _ptr(n0, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle_fock_start failed")
    return n0.reshape(2, lat.N)


# --------------------------------------------------------------------------
# Sampling (Eq. (7)), equation of motion (Eq. (6)), RK4, moments, observables
# --------------------------------------------------------------------------
def sample(lat: Lattice, n0: np.ndarray, seed: int, M: int, traj_offset: int = 0,
           instance: int = 0, thermal: bool = False) -> np.ndarray:
    """Gaussian initial points rho(0), shape [M, 2, N, N] complex128 (Eq. (7));
    thermal: also the diagonal fluctuation Var rho_ii = n(1 - n) of the
    Appendix A.3 covariance."""
    lib = _load()
    n0c = np.ascontiguousarray(n0, dtype=np.float64).reshape(-1)
    out = np.zeros((M, 2, lat.N, lat.N), dtype=np.complex128)
    lib.oracle_sample(lat.N, _ptr(n0c, ctypes.c_double), ctypes.c_uint64(seed), instance,
                      traj_offset, M, 1 if thermal else 0,
                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def real_normal(seed: int, c0: int, c1: int, c2: int, c3: int) -> float:
    """One real standard normal of the thermal diagonal (Box-Muller on the
    Philox draw of counter (c0, c1, c2, c3))."""
    return float(_load().oracle_real_normal(ctypes.c_uint64(seed), c0, c1, c2, c3))


def rhs(lat: Lattice, U: float, rho: np.ndarray, precision: str = "f64") -> np.ndarray:
    """d rho/dt of one trajectory (Eq. (6)); rho shape [2, N, N] complex."""
    lib = _load()
    nbr = np.ascontiguousarray(lat.nbr.reshape(-1))
    deg = np.ascontiguousarray(lat.deg)
    if precision == "f64":
        r = np.ascontiguousarray(rho, dtype=np.complex128)
        f = np.zeros_like(r)
        lib.oracle_rhs_f64(lat.N, _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8),
                           lat.t, U, r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return f
    r = np.ascontiguousarray(rho, dtype=np.complex64)
    f = np.zeros_like(r)
    lib.oracle_rhs_f32(lat.N, _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8),
                       np.float32(lat.t), np.float32(U),
                       r.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                       f.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return f


def n_records(n_steps: int, record_every: int) -> int:
    return n_steps // record_every + 1


def evolve(lat: Lattice, U: float, rho: np.ndarray, dt: float, n_steps: int,
           record_every: int = 10, precision: str = "f64", want_inv: bool = False,
           vsite=None, env=None, umat=None, hop=None):
    """RK4 integration of every trajectory.  Returns (rho_final, X, inv).

    rho: [M, 2, N, N] complex128 (not modified).  X: [n_rec, M, 2N] diagonal
    records; inv: [n_rec, M, 5] (trace up, trace down, H_W, |rho_up|_F^2,
    |rho_dn|_F^2) or None.  vsite ([N]) and env ([2 n_steps + 1]): an
    external on-site potential V_i(tau) = env(tau) vsite[i] on both spins,
    env sampled at t_n and t_n + dt/2 of every step (see oracle_evolve_pot).
    umat ([N, N], symmetric): a general density-density interaction u_ij between
    opposite spins in place of the on-site U (see oracle_evolve_gen; no inv).
    hop ([2 n_steps + 1, N, 3] complex): complex hopping j_ik(tau) = t hop[h, i, n]
    for k = lat.nbr[i, n] at the half steps of env (Peierls phases; Hermitian:
    the entry of k for i is the conjugate; slots beyond deg are ignored; no inv).
    """
    lib = _load()
    if vsite is not None:
        vs = np.ascontiguousarray(vsite, dtype=np.float64).reshape(-1)
        ev = np.ascontiguousarray(env, dtype=np.float64).reshape(-1)
        if vs.size != lat.N or ev.size != 2 * n_steps + 1:
            raise ValueError("vsite needs N values and env 2 n_steps + 1")
    M = rho.shape[0]
    y = np.ascontiguousarray(rho, dtype=np.complex128).copy()
    n_rec = n_records(n_steps, record_every)
    X = np.zeros((n_rec, M, 2 * lat.N), dtype=np.float64)
    inv = np.zeros((n_rec, M, 5), dtype=np.float64) if want_inv else None
    nbr = np.ascontiguousarray(lat.nbr.reshape(-1))
    deg = np.ascontiguousarray(lat.deg)
    dptr = ctypes.POINTER(ctypes.c_double)
    if hop is not None:
        hw = np.ascontiguousarray(hop, dtype=np.complex128)
        if hw.shape != (2 * n_steps + 1, lat.N, 3) or want_inv:
            raise ValueError("hop must be [2 n_steps + 1, N, 3] (and records no invariants)")
        um = None if umat is None else np.ascontiguousarray(umat, dtype=np.float64)
        if um is not None and um.shape != (lat.N, lat.N):
            raise ValueError("umat must be N x N")
        fn = lib.oracle_evolve_hop_f64 if precision == "f64" else lib.oracle_evolve_hop_f32
        rc = fn(lat.N, _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8), lat.t, float(U),
                um.ctypes.data_as(dptr) if um is not None else None,
                vs.ctypes.data_as(dptr) if vsite is not None else None,
                ev.ctypes.data_as(dptr) if vsite is not None else None,
                hw.ctypes.data_as(dptr), float(dt), int(n_steps), int(record_every), M,
                y.ctypes.data_as(dptr), X.ctypes.data_as(dptr), None)
    elif umat is not None:
        um = np.ascontiguousarray(umat, dtype=np.float64)
        if um.shape != (lat.N, lat.N) or want_inv:
            raise ValueError("umat must be N x N (and records no invariants)")
        fn = lib.oracle_evolve_gen_f64 if precision == "f64" else lib.oracle_evolve_gen_f32
        rc = fn(lat.N, _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8), lat.t, float(U),
                um.ctypes.data_as(dptr), vs.ctypes.data_as(dptr) if vsite is not None else None,
                ev.ctypes.data_as(dptr) if vsite is not None else None, float(dt), int(n_steps),
                int(record_every), M, y.ctypes.data_as(dptr), X.ctypes.data_as(dptr), None)
    elif vsite is None:
        fn = lib.oracle_evolve_f64 if precision == "f64" else lib.oracle_evolve_f32
        rc = fn(lat.N, _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8), lat.t, float(U),
                float(dt), int(n_steps), int(record_every), M, y.ctypes.data_as(dptr),
                X.ctypes.data_as(dptr), inv.ctypes.data_as(dptr) if inv is not None else None)
    else:
        fn = lib.oracle_evolve_pot_f64 if precision == "f64" else lib.oracle_evolve_pot_f32
        rc = fn(lat.N, _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8), lat.t, float(U),
                vs.ctypes.data_as(dptr), ev.ctypes.data_as(dptr), float(dt), int(n_steps),
                int(record_every), M, y.ctypes.data_as(dptr), X.ctypes.data_as(dptr),
                inv.ctypes.data_as(dptr) if inv is not None else None)
    if rc != 0:
        raise RuntimeError(f"oracle evolve failed ({rc})")
    return y, X, inv


def evolve_tangent(lat: Lattice, U: float, rho0: np.ndarray, dt: float, n_steps: int,
                   record_every: int, dU: float = 0.0, dt_hop: float = 0.0, dshift=None):
    """FP64 trajectories and their derivative along (dU, dt_hop, dshift[2][N]),
    dshift shifting rho_ii,s(0) with the off-diagonal noise held fixed.
    Returns (X, Xd), both [n_rec, M, 2N] diagonal records."""
    lib = _load()
    M = rho0.shape[0]
    r0 = np.ascontiguousarray(rho0, dtype=np.complex128)
    n_rec = n_records(n_steps, record_every)
    X = np.zeros((n_rec, M, 2 * lat.N))
    Xd = np.zeros_like(X)
    ds = np.zeros(2 * lat.N) if dshift is None else np.ascontiguousarray(dshift, dtype=np.float64)
    ds = ds.reshape(-1)
    nbr = np.ascontiguousarray(lat.nbr.reshape(-1))
    deg = np.ascontiguousarray(lat.deg)
    dptr = ctypes.POINTER(ctypes.c_double)
    rc = lib.oracle_evolve_tangent(lat.N, _ptr(nbr, ctypes.c_int32), _ptr(deg, ctypes.c_uint8),
                                   lat.t, float(U), float(dt), int(n_steps), int(record_every), M,
                                   r0.ctypes.data_as(dptr), float(dU), float(dt_hop),
                                   ds.ctypes.data_as(dptr), X.ctypes.data_as(dptr),
                                   Xd.ctypes.data_as(dptr))
    if rc != 0:
        raise RuntimeError(f"oracle tangent failed ({rc})")
    return X, Xd


def occupation_loss_grad(lat: Lattice, U: float, rho0: np.ndarray, dt: float, n_steps: int,
                         record_every: int, target: np.ndarray):
    """Loss L = sum_{r,a} (nbar_a(r) - target_a(r))^2 over the ensemble-mean
    occupations nbar = mean_m X + 1/2 (Eq. (5)), and its gradient with respect
    to U, t and the initial diagonal shifts [2][N], each component from one
    tangent run (noise held fixed).  Returns (L, dU, dt, dshift[2][N])."""
    N = lat.N
    X, _ = evolve_tangent(lat, U, rho0, dt, n_steps, record_every)
    nbar = X.mean(axis=1) + 0.5
    resid = nbar - target
    L = float(np.sum(resid * resid))
    w = 2.0 * resid

    def directional(**kw):
        _, Xd = evolve_tangent(lat, U, rho0, dt, n_steps, record_every, **kw)
        return float(np.sum(w * Xd.mean(axis=1)))

    gU = directional(dU=1.0)
    gt = directional(dt_hop=1.0)
    gs = np.zeros(2 * N)
    for a in range(2 * N):
        e = np.zeros(2 * N)
        e[a] = 1.0
        gs[a] = directional(dshift=e)
    return L, gU, gt, gs.reshape(2, N)


def moments(X: np.ndarray):
    """S1 [n_rec, D] and packed-upper S2 [n_rec, D(D+1)/2] of X [n_rec, M, D]."""
    lib = _load()
    n_rec, M, D = X.shape
    Xc = np.ascontiguousarray(X, dtype=np.float64)
    S1 = np.zeros((n_rec, D))
    S2 = np.zeros((n_rec, D * (D + 1) // 2))
    dptr = ctypes.POINTER(ctypes.c_double)
    lib.oracle_moments(D, M, n_rec, Xc.ctypes.data_as(dptr), S1.ctypes.data_as(dptr),
                       S2.ctypes.data_as(dptr))
    return S1, S2


def observables(N: int, M: int, S1: np.ndarray, S2: np.ndarray):
    """(n [n_rec, 2N], C [n_rec, 2N, 2N], g2 [n_rec, 2N, 2N]) -- Eq. (5), Eq. (10)."""
    lib = _load()
    n_rec, D = S1.shape
    n = np.zeros((n_rec, D))
    C = np.zeros((n_rec, D, D))
    g2 = np.zeros((n_rec, D, D))
    dptr = ctypes.POINTER(ctypes.c_double)
    s1 = np.ascontiguousarray(S1)
    s2 = np.ascontiguousarray(S2)
    lib.oracle_observables(N, M, n_rec, s1.ctypes.data_as(dptr), s2.ctypes.data_as(dptr),
                           n.ctypes.data_as(dptr), C.ctypes.data_as(dptr),
                           g2.ctypes.data_as(dptr))
    return n, C, g2


def packed_index(a: int, b: int, D: int) -> int:
    lo, hi = (a, b) if a <= b else (b, a)
    return lo * D - lo * (lo - 1) // 2 + (hi - lo)

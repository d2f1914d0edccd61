"""Exact many-body dynamics of the Fermi-Hubbard model -- TEST INFRASTRUCTURE.

This module is part of the oracle: only ``tests/`` (and the oracle's own
users listed in ``oracle/__init__.py``) may import it.  It pins the fTWA
oracle against the quantum dynamics it approximates, on clusters small
enough to hold the whole many-body state.

What it computes (Sec. III.A, Eq. (8); Appendix B.1):
  * the basis of Slater determinants with fixed particle numbers per spin,
    C(N, p_up) x C(N, p_dn) states, each a bit mask of occupied sites per
    spin with creation operators in ascending site order, all up operators
    before all down ones;
  * the Hamiltonian of Eq. (1), H = -sum_{ij s} j_ij c+_is c_js
    + sum_ij u_ij n_i,up n_j,dn, as a sparse matrix in that basis;
  * |Psi(t)> = exp(-i H t) |Psi_0> (the paper writes exp(+iHt); H is real
    and every start here is a real Fock state, so real observables are even
    in t and the sign does not matter), by a full eigendecomposition for small
    bases and by scipy's expm_multiply otherwise;
  * the occupations <n_a(t)> and density-density moments <n_a n_b(t)>,
    a = s*N + i, which is what the fTWA moments of Eq. (5) estimate;
  * the ground state and the Fock basis vector of largest overlap with it
    (Appendix B.2), the paper's initial condition for its 10-site study.

Parity: pinned in tests/test_oracle_ed.py against a Hubbard dimer written by
hand, against a Jordan-Wigner construction of the full Fock space, and at
U = 0 against the free-fermion (Wick) closed form.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

EIGH_MAX_DIM = 1200


def sector_states(N: int, p: int) -> np.ndarray:
    """Bit masks of the C(N, p) determinants with p of N sites occupied, ascending."""
    states = [sum(1 << i for i in occ) for occ in combinations(range(N), p)]
    return np.array(sorted(states), dtype=np.int64)


def _popcount_below(s: int, i: int) -> int:
    return bin(s & ((1 << i) - 1)).count("1")


def one_body_operator(N: int, states: np.ndarray, h: np.ndarray) -> sp.csr_matrix:
    """sum_ij h_ij c+_i c_j on one spin species, in the basis `states`.

    c_j removes site j after passing the occupied sites below it, c+_i
    inserts site i after passing the occupied sites below it in the
    intermediate state; each pass contributes a factor -1."""
    index = {int(s): k for k, s in enumerate(states)}
    rows, cols, vals = [], [], []
    for k, s in enumerate(states):
        s = int(s)
        for j in range(N):
            if not (s >> j) & 1:
                continue
            s1 = s & ~(1 << j)
            sign1 = -1.0 if _popcount_below(s, j) % 2 else 1.0
            for i in range(N):
                hij = h[i, j]
                if hij == 0.0 or (s1 >> i) & 1:
                    continue
                s2 = s1 | (1 << i)
                sign2 = -1.0 if _popcount_below(s1, i) % 2 else 1.0
                rows.append(index[s2])
                cols.append(k)
                vals.append(hij * sign1 * sign2)
    d = len(states)
    return sp.csr_matrix((vals, (rows, cols)), shape=(d, d))


def occupation_table(N: int, states: np.ndarray) -> np.ndarray:
    """occ[k, i] = 1.0 if site i is occupied in determinant k."""
    return ((states[:, None] >> np.arange(N)[None, :]) & 1).astype(np.float64)


class HubbardED:
    """Eq. (1) with hopping matrix J (j_ij, real symmetric) and interaction
    matrix u (u_ij between i up and j down) in the sector of p_up up and
    p_dn down electrons.  Basis index = k_up * dim_dn + k_dn."""

    def __init__(self, J: np.ndarray, u: np.ndarray, p_up: int, p_dn: int):
        J = np.asarray(J, dtype=np.float64)
        u = np.asarray(u, dtype=np.float64)
        self.N = N = J.shape[0]
        self.up = sector_states(N, p_up)
        self.dn = sector_states(N, p_dn)
        self.occ_up = occupation_table(N, self.up)
        self.occ_dn = occupation_table(N, self.dn)
        du, dd = len(self.up), len(self.dn)
        self.dim = du * dd
        T_up = one_body_operator(N, self.up, -J)
        T_dn = one_body_operator(N, self.dn, -J)
        # the hopping of one spin commutes with the other spin's operators as
        # a pair, so the two sectors combine as a Kronecker sum
        H = sp.kron(T_up, sp.identity(dd)) + sp.kron(sp.identity(du), T_dn)
        # sum_ij u_ij n_i,up n_j,dn is diagonal: occ_up u occ_dn^T per pair
        inter = self.occ_up @ u @ self.occ_dn.T
        self.H = (H + sp.diags(inter.reshape(-1))).tocsr()

    def fock_vector(self, n0: np.ndarray) -> np.ndarray:
        """Basis vector of the Fock state n0[spin, site] (0/1 entries)."""
        n0 = np.asarray(n0)
        s_up = sum(1 << i for i in range(self.N) if n0[0, i] > 0.5)
        s_dn = sum(1 << i for i in range(self.N) if n0[1, i] > 0.5)
        k_up = int(np.searchsorted(self.up, s_up))
        k_dn = int(np.searchsorted(self.dn, s_dn))
        if self.up[k_up] != s_up or self.dn[k_dn] != s_dn:
            raise ValueError("Fock state outside this particle-number sector")
        psi = np.zeros(self.dim, dtype=np.complex128)
        psi[k_up * len(self.dn) + k_dn] = 1.0
        return psi

    def evolve(self, psi0: np.ndarray, times) -> np.ndarray:
        """States exp(-i H t) psi0 at every t of `times` (ascending, from 0)."""
        times = np.asarray(times, dtype=np.float64)
        if self.dim <= EIGH_MAX_DIM:
            w, V = np.linalg.eigh(self.H.toarray())
            c = V.T @ psi0
            phase = np.exp(-1j * np.outer(times, w))
            return (phase * c[None, :]) @ V.T
        step = (times[-1] - times[0]) / max(len(times) - 1, 1)
        if not np.allclose(times, times[0] + step * np.arange(len(times)), atol=1e-12):
            raise ValueError("expm_multiply needs equally spaced times")
        psi = psi0
        if times[0] != 0.0:
            psi = spla.expm_multiply(-1j * times[0] * self.H, psi0)
        return spla.expm_multiply(-1j * self.H, psi, start=0.0, stop=float(times[-1] - times[0]),
                                  num=len(times), endpoint=True)

    def densities(self, psi_t: np.ndarray):
        """(n [T, 2N], nn [T, 2N, 2N]) with n_a = <n_a>, nn_ab = <n_a n_b>,
        a = s*N + i.  The diagonal nn_aa equals n_a (n^2 = n)."""
        du, dd = len(self.up), len(self.dn)
        T = psi_t.shape[0]
        N = self.N
        n = np.zeros((T, 2 * N))
        nn = np.zeros((T, 2 * N, 2 * N))
        for k in range(T):
            P = (np.abs(psi_t[k]) ** 2).reshape(du, dd)
            pu = P.sum(axis=1)
            pd = P.sum(axis=0)
            n[k, :N] = pu @ self.occ_up
            n[k, N:] = pd @ self.occ_dn
            nn[k, :N, :N] = self.occ_up.T @ (pu[:, None] * self.occ_up)
            nn[k, N:, N:] = self.occ_dn.T @ (pd[:, None] * self.occ_dn)
            cross = self.occ_up.T @ P @ self.occ_dn
            nn[k, :N, N:] = cross
            nn[k, N:, :N] = cross.T
        return n, nn

    def ground_state(self):
        """(E0, psi0) of the lowest eigenpair."""
        if self.dim <= EIGH_MAX_DIM:
            w, V = np.linalg.eigh(self.H.toarray())
            return float(w[0]), V[:, 0]
        w, V = spla.eigsh(self.H, k=1, which="SA", tol=1e-12)
        return float(w[0]), V[:, 0]

    def largest_overlap_fock(self, psi: np.ndarray):
        """Occupations n0[2, N] of the basis vectors of largest |amplitude| in
        psi (all of them when several tie within 1e-9), largest first."""
        a = np.abs(psi)
        top = np.flatnonzero(a >= a.max() - 1e-9)
        out = []
        for k in top:
            ku, kd = divmod(int(k), len(self.dn))
            out.append(np.stack([self.occ_up[ku], self.occ_dn[kd]]))
        return out


def hubbard_onsite(J: np.ndarray, U: float) -> np.ndarray:
    """u_ij = U delta_ij (Sec. II)."""
    return U * np.eye(J.shape[0])

"""Explicit Fock-space objects for tiny systems (TEST INFRASTRUCTURE ONLY).

Spin orbitals are numbered alpha 0..M-1 then beta M..2M-1; a basis state is a
bit string n with bit j the occupation of spin orbital j.  Creation
operators follow Jordan-Wigner: a+_j |n> = (-1)^{sum_{i<j} n_i} |n + e_j> when
n_j = 0.  Nothing here uses Wick's theorem or determinants: states are built
by applying creation operators to the vacuum and the Hamiltonian of Eq. 2 is
assembled operator by operator.  Used only to pin ``oracle.msd`` and
``oracle.propagate``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class FockSpace:
    def __init__(self, M: int):
        if M > 7:
            raise ValueError("Fock space limited to M <= 7 spatial orbitals")
        self.M = M
        self.nmodes = 2 * M
        self.dim = 1 << self.nmodes
        self._cdag = [self._creation(j) for j in range(self.nmodes)]
        self._ann = [c.T.tocsr() for c in self._cdag]

    def _creation(self, j):
        states = np.arange(self.dim)
        empty = ((states >> j) & 1) == 0
        src = states[empty]
        dst = src | (1 << j)
        below = src & ((1 << j) - 1)
        parity = np.array([bin(int(b)).count("1") & 1 for b in below])
        data = np.where(parity == 1, -1.0, 1.0)
        return sp.csr_matrix((data, (dst, src)), shape=(self.dim, self.dim))

    def mode(self, p: int, spin: int) -> int:
        return p + spin * self.M

    def cdag(self, p, spin):
        return self._cdag[self.mode(p, spin)]

    def ann(self, p, spin):
        return self._ann[self.mode(p, spin)]

    def vacuum(self):
        v = np.zeros(self.dim, dtype=np.complex128)
        v[0] = 1.0
        return v

    # -- states ------------------------------------------------------------
    def determinant(self, occ_a, occ_b):
        """a+_{s1 a} .. a+_{sN a} a+_{t1 b} .. a+_{tN b} |0> (ascending lists)."""
        v = self.vacuum()
        ops = [self.cdag(int(p), 0) for p in sorted(occ_a)] + \
              [self.cdag(int(p), 1) for p in sorted(occ_b)]
        for op in reversed(ops):
            v = op @ v
        return v

    def slater(self, phi_a, phi_b):
        """prod_j (sum_p Phi^a_pj a+_pa) prod_j (sum_p Phi^b_pj a+_pb) |0>."""
        ops = []
        for spin, phi in ((0, phi_a), (1, phi_b)):
            for j in range(phi.shape[1]):
                op = sum(phi[p, j] * self.cdag(p, spin) for p in range(self.M))
                ops.append(op)
        v = self.vacuum()
        for op in reversed(ops):
            v = op @ v
        return v

    def trial(self, ci, occ_a, occ_b):
        """|Psi_T> = sum_I c_I |D_I>."""
        v = np.zeros(self.dim, dtype=np.complex128)
        for c, a, b in zip(ci, occ_a, occ_b):
            v += c * self.determinant(a, b)
        return v

    # -- operators ---------------------------------------------------------
    def one_body(self, mat, spins=(0, 1)):
        """sum_s sum_pq mat_pq a+_ps a_qs."""
        M = self.M
        op = sp.csr_matrix((self.dim, self.dim), dtype=np.complex128)
        for s in spins:
            for p in range(M):
                for q in range(M):
                    if mat[p, q] != 0:
                        op = op + mat[p, q] * (self.cdag(p, s) @ self.ann(q, s))
        return op

    def hamiltonian(self, h1, eri, e0):
        """Eq. 2 operator: E0 + sum h_pq a+_ps a_qs
        + 1/2 sum (pq|rs) a+_ps a+_rs' a_ss' a_qs  (all spins)."""
        M = self.M
        H = e0 * sp.identity(self.dim, dtype=np.complex128, format="csr")
        H = H + self.one_body(h1)
        for s1 in (0, 1):
            for s2 in (0, 1):
                for p in range(M):
                    for r in range(M):
                        cc = self.cdag(p, s1) @ self.cdag(r, s2)
                        if cc.nnz == 0:
                            continue
                        inner = sp.csr_matrix((self.dim, self.dim), dtype=np.complex128)
                        for q in range(M):
                            for s in range(M):
                                val = eri[p, q, r, s]
                                if val != 0:
                                    inner = inner + val * (self.ann(s, s2) @ self.ann(q, s1))
                        H = H + 0.5 * (cc @ inner)
        return H.tocsr()

    def sector(self, n_a, n_b):
        """Indices of basis states with n_a alpha and n_b beta electrons."""
        states = np.arange(self.dim)
        amask = (1 << self.M) - 1
        na = np.array([bin(int(s & amask)).count("1") for s in states])
        nb = np.array([bin(int(s >> self.M)).count("1") for s in states])
        return states[(na == n_a) & (nb == n_b)]

    def ground_state(self, H, n_a, n_b):
        """Lowest eigenpair of H inside the (n_a, n_b) sector (dense eigh)."""
        idx = self.sector(n_a, n_b)
        hs = H[idx][:, idx].toarray()
        evals, evecs = np.linalg.eigh(hs)
        vec = np.zeros(self.dim, dtype=np.complex128)
        vec[idx] = evecs[:, 0]
        return evals[0], vec

    def expansion(self, vec, n_a, n_b, tol=0.0):
        """Write a sector vector as (ci, occ_a, occ_b) with c_I = <D_I|vec>."""
        idx = self.sector(n_a, n_b)
        ci, oa, ob = [], [], []
        for s in idx:
            a = [p for p in range(self.M) if (s >> p) & 1]
            b = [p for p in range(self.M) if (s >> (p + self.M)) & 1]
            c = np.vdot(self.determinant(a, b), vec)
            if abs(c) > tol:
                ci.append(c)
                oa.append(a)
                ob.append(b)
        return (np.array(ci, dtype=np.complex128), np.array(oa, dtype=np.int32).reshape(len(ci), n_a),
                np.array(ob, dtype=np.int32).reshape(len(ci), n_b))


def eri_from_chol(chol):
    """(pq|rs) = sum_g L^g_pq L^g_rs."""
    return np.einsum("gpq,grs->pqrs", chol, chol)

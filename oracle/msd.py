"""Brute-force MSD trial quantities per walker (TEST INFRASTRUCTURE ONLY).

Conventions (the readings of the paper used everywhere in this repository):

* Trial (Sec. II.B, Eq. 15): |Psi_T> = sum_I c_I |D_I>, and <Psi_T| carries
  the conjugates c_I^*.  D_I = a+_{s1 a}..a+_{sN a} a+_{t1 b}..a+_{tN b}|0>
  with each spin's occupied orbitals in ascending order, alpha before beta.
* Walker (Sec. II.A): one Slater determinant per spin, Phi^s (M x N_s).  Its
  overlap with D_I is det(Phi^a[S_I^a, :]) det(Phi^b[S_I^b, :]) (Eq. 13 with
  Psi_T = the columns of the identity at S_I).
* Green's function (Eq. 14, whose brackets are garbled in the text):
  G_pq = <Psi_T| a+_p a_q |Phi> / <Psi_T|Phi>, one M x M matrix per spin.
  For one determinant with A = Phi[S, :], G_pq = [Phi A^{-1}]_{q, j(p)} for
  p = S_j and 0 for p outside S.
* Force bias (Eq. 7, read with the factor i of the Hubbard-Stratonovich
  transform of -dt/2 L^2): xbar_g = -i sqrt(dt) sum_s sum_pq L^g_pq G^s_pq.
* Hamiltonian (Eqs. 2-3): H = E0 + sum_pq h_pq E_pq
  + 1/2 sum_pqrs (pq|rs) sum_{s s'} a+_{ps} a+_{rs'} a_{ss'} a_{qs},
  (pq|rs) = sum_g L^g_pq L^g_rs.  h is the bare one-body matrix.
* Local energy (Sec. II.A, mixed estimator): E_L = <Psi_T|H|Phi>/<Psi_T|Phi>.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------------------
# small linear-algebra helpers
# ----------------------------------------------------------------------------

def adjugate(a: np.ndarray) -> np.ndarray:
    """adj(A) for a stack of square matrices, valid for singular A.

    adj(A) = det(A) A^{-1} where A is invertible; here written through the SVD
    A = U diag(s) V^H as det(U) det(V^H) V diag(prod_{j != i} s_j) U^H, which is
    a polynomial in A and stays exact for rank-deficient A.
    """
    a = np.asarray(a, dtype=np.complex128)
    n = a.shape[-1]
    if n == 0:
        return np.zeros_like(a)
    u, s, vh = np.linalg.svd(a)
    # prod over j != i of s_j, without dividing by s_i
    prod_others = np.empty_like(s)
    for i in range(n):
        prod_others[..., i] = np.prod(np.delete(s, i, axis=-1), axis=-1)
    phase = np.linalg.det(u) * np.linalg.det(vh)
    v = np.conj(np.swapaxes(vh, -1, -2))
    uh = np.conj(np.swapaxes(u, -1, -2))
    return phase[..., None, None] * (v * prod_others[..., None, :]) @ uh


# ----------------------------------------------------------------------------
# overlaps (Eqs. 13, 15)
# ----------------------------------------------------------------------------

def spin_overlaps(phi: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """det(Phi[S_I, :]) for every determinant I of one spin: shape (n_det,)."""
    occ = np.asarray(occ)
    if occ.shape[1] == 0:
        return np.ones(occ.shape[0], dtype=np.complex128)
    return np.linalg.det(phi[occ])


def det_overlaps(occ_a, occ_b, phi_a, phi_b) -> np.ndarray:
    """<D_I|Phi> for every determinant: product of the two spin dets."""
    return spin_overlaps(phi_a, occ_a) * spin_overlaps(phi_b, occ_b)


def trial_overlap(ci, occ_a, occ_b, phi_a, phi_b) -> complex:
    """<Psi_T|Phi> = sum_I c_I^* <D_I|Phi>."""
    return complex(np.sum(np.conj(ci) * det_overlaps(occ_a, occ_b, phi_a, phi_b)))


# ----------------------------------------------------------------------------
# Green's function (Eq. 14) and force bias (Eq. 7)
# ----------------------------------------------------------------------------

def weighted_det_green(phi: np.ndarray, occ_row: np.ndarray) -> np.ndarray:
    """det(A) * G for one determinant of one spin (A = Phi[S, :]).

    Row S_j of det(A) G is column j of Phi adj(A); all other rows are zero.
    Written with the adjugate so it is exact when A is singular (then
    <D|Phi> = 0 while <D|a+_p a_q|Phi> need not vanish).
    """
    M = phi.shape[0]
    out = np.zeros((M, M), dtype=np.complex128)
    if len(occ_row) == 0:
        return out
    a = phi[occ_row]
    out[occ_row, :] = (phi @ adjugate(a)).T
    return out


def green(ci, occ_a, occ_b, phi_a, phi_b):
    """Mixed Green's functions (G^a, G^b) of the MSD trial for one walker."""
    oa = spin_overlaps(phi_a, occ_a)
    ob = spin_overlaps(phi_b, occ_b)
    cc = np.conj(ci)
    o_t = np.sum(cc * oa * ob)
    M = phi_a.shape[0]
    ga = np.zeros((M, M), dtype=np.complex128)
    gb = np.zeros((M, M), dtype=np.complex128)
    for i in range(len(ci)):
        if cc[i] == 0:
            continue
        ga += cc[i] * ob[i] * weighted_det_green(phi_a, occ_a[i])
        gb += cc[i] * oa[i] * weighted_det_green(phi_b, occ_b[i])
    return ga / o_t, gb / o_t


def force_bias(chol, ga, gb, dt) -> np.ndarray:
    """xbar_g = -i sqrt(dt) sum_s sum_pq L^g_pq G^s_pq (Eq. 7)."""
    vbar = np.einsum("gpq,pq->g", chol, ga + gb)
    return -1j * np.sqrt(dt) * vbar


# ----------------------------------------------------------------------------
# local energy (mixed estimator)
# ----------------------------------------------------------------------------

def energy_sd_plain(h1, chol, e0, ga, gb) -> complex:
    """Single-determinant energy from its two Green's functions (Wick).

    E = E0 + sum_s sum_pq h_pq G^s_pq
        + 1/2 sum_pqrs (pq|rs) [ sum_{s s'} G^s_pq G^s'_rs - sum_s G^s_ps G^s_rq ]
    with (pq|rs) = sum_g L^g_pq L^g_rs.  Plain O(N_chol M^3) evaluation.
    """
    e = e0 + np.sum(h1 * (ga + gb))
    j = np.einsum("gpq,pq->g", chol, ga + gb)
    k = 0.0
    for g in (ga, gb):
        lg = np.einsum("gpq,rq->gpr", chol, g)   # (L G^T)
        k = k + np.einsum("gpr,grp->g", lg, lg)  # tr((L G^T)^2)
    return complex(e + 0.5 * np.sum(j * j - k))


def energy_sd_eri(h1, eri, e0, ga, gb) -> complex:
    """Same as energy_sd_plain but from an explicit 4-index (pq|rs) tensor."""
    e = e0 + np.sum(h1 * (ga + gb))
    gt = ga + gb
    coul = np.einsum("pqrs,pq,rs->", eri, gt, gt)
    exch = sum(np.einsum("pqrs,ps,rq->", eri, g, g) for g in (ga, gb))
    return complex(e + 0.5 * (coul - exch))


class _SpinCache:
    """Per-spin pieces of the single-determinant energy, keyed by orbital set.

    For a determinant with A = Phi[S, :] and Theta = Phi A^{-1}:
      one-body  tr(h[S, :] Theta)
      J_g       tr(L^g[S, :] Theta)
      K_g       tr((L^g[S, :] Theta)^2)
    These equal sum_pq h_pq G_pq, sum_pq L_pq G_pq and tr((L G^T)^2) for that
    determinant's G (cyclic trace with G = E_S Theta^T).
    """

    def __init__(self, h1, chol, phi, cond_max):
        self.h1, self.chol, self.phi = h1, chol, phi
        self.cond_max = cond_max
        self.cache = {}

    def get(self, occ_row):
        key = tuple(int(x) for x in occ_row)
        if key not in self.cache:
            occ = np.asarray(key, dtype=np.int64)
            n = len(occ)
            if n == 0:
                ng = self.chol.shape[0]
                self.cache[key] = (0.0, np.zeros(ng, complex), np.zeros(ng, complex))
            else:
                a = self.phi[occ]
                if np.linalg.cond(a) > self.cond_max:
                    raise np.linalg.LinAlgError(
                        f"orbital set {key}: singular block, brute-force energy undefined")
                theta = np.linalg.solve(a.T, self.phi.T).T   # Phi A^{-1}
                one = np.trace(self.h1[occ, :] @ theta)
                lsub = self.chol[:, occ, :]                  # (ng, n, M)
                q = lsub @ theta                             # (ng, n, n)
                jg = np.trace(q, axis1=1, axis2=2)
                kg = np.einsum("gij,gji->g", q, q)
                self.cache[key] = (one, jg, kg)
        return self.cache[key]


def local_energy(h1, chol, e0, ci, occ_a, occ_b, phi_a, phi_b, cond_max=1e10):
    """E_L = sum_I c_I^* <D_I|Phi> E_SD(G_I) / <Psi_T|Phi>.

    Each determinant's <D_I|H|Phi> is <D_I|Phi> times its single-determinant
    Wick energy, which needs the per-spin blocks Phi[S, :] to be invertible;
    a block worse conditioned than ``cond_max`` raises (use the Fock-space
    oracle for such cases).
    """
    oa = spin_overlaps(phi_a, occ_a)
    ob = spin_overlaps(phi_b, occ_b)
    cc = np.conj(ci)
    o_t = np.sum(cc * oa * ob)
    ca = _SpinCache(h1, chol, phi_a, cond_max)
    cb = _SpinCache(h1, chol, phi_b, cond_max)
    num = 0.0 + 0.0j
    for i in range(len(ci)):
        if cc[i] == 0:
            continue
        one_a, ja, ka = ca.get(occ_a[i])
        one_b, jb, kb = cb.get(occ_b[i])
        jt = ja + jb
        e_sd = e0 + one_a + one_b + 0.5 * np.sum(jt * jt - ka - kb)
        num += cc[i] * oa[i] * ob[i] * e_sd
    return complex(num / o_t)


# ----------------------------------------------------------------------------
# all walkers at once
# ----------------------------------------------------------------------------

def measure(h1, chol, e0, ci, occ_a, occ_b, phi_a, phi_b, dt,
            walkers=None, energy=True):
    """log <Psi_T|Phi_w>, xbar_w and E_L(w) for the selected walkers.

    Returns a dict of arrays indexed like ``walkers`` (default: all).
    """
    nw = phi_a.shape[0]
    sel = range(nw) if walkers is None else list(walkers)
    log_o, fb, el = [], [], []
    for w in sel:
        o_t = trial_overlap(ci, occ_a, occ_b, phi_a[w], phi_b[w])
        log_o.append(np.log(o_t))
        ga, gb = green(ci, occ_a, occ_b, phi_a[w], phi_b[w])
        fb.append(force_bias(chol, ga, gb, dt))
        if energy:
            el.append(local_energy(h1, chol, e0, ci, occ_a, occ_b, phi_a[w], phi_b[w]))
    out = dict(log_ovlp=np.array(log_o), force_bias=np.array(fb))
    if energy:
        out["e_loc"] = np.array(el)
    return out

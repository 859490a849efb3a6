"""Generalised-Wick CPU path of the MSD trial quantities (TEST INFRASTRUCTURE ONLY).

A second oracle path, for sizes where the brute-force one in ``oracle.msd``
cannot finish (10^4 - 10^6 determinants, 30-45 electrons per spin).  It
evaluates every determinant one at a time relative to the reference (paper
Sec. III and App. A; Eqs. 13-15): no grouping of determinants into spin
strings, no sharing of work between determinants, no precontracted
Cholesky-vector sums.  It is pinned against ``oracle.msd`` and explicit Fock
space in ``tests/test_oracle_wick.py``; it shares no code with the HIP
library.  Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
cpu_baseline leg may import it.

Notation, per walker and spin (row 0 of the occupation lists is the
reference R, N orbitals in ascending order):

* A = Phi[R, :], T = Phi A^{-1} (so T[R, :] = 1), G0 the reference
  determinant's Green's function: G0[R_j, q] = T[q, j], other rows zero.
* Determinant I of the spin has holes h_1 < .. < h_k in R and particles
  p_1 < .. < p_k outside R.  Its overlap ratio is
  <D_I|Phi> / <D_R|Phi> = sgn det X with X_mn = T[p_n, slot(h_m)] (k x k) and
  sgn the parity of the permutation that sorts R with slot(h_m) holding p_m.
* c~_I = conj(c_I) sgn_a sgn_b;  Obar = sum_I c~_I det X_a det X_b;
  <Psi_T|Phi> = Obar det A_a det A_b.

Green's function.  Along Phi -> (1 + eps E_pq) Phi, d log det A / d eps =
G0[p, q] and (Jacobi) d det X / d eps = -sum_mn adj(X)_nm (G0 - I)[p, p_n]
G0[h_m, q], so

  G = G0 - (G0 - I) C G0 / Obar,  C[p_n, h_m] += c~_I det X_other adj(X)_nm.

Local energy.  With Q^g = L^g[R, :] T, v0 = tr Q^g, ex0 = tr (Q^g Q^g),
Lambda^g = T[V, :] Q^g - (L^g T)[V, :], Xi^g = Lambda^g Q^g (V: the particle
orbitals) and Y^g_mn = Lambda^g[p_n, slot(h_m)], Z^g_mn = Xi^g[p_n, slot(h_m)],
expanding det((T + eps L^g T)[S_I, :]) to second order in eps gives (per
spin, d = det X)

  a(g) = d v0 - tr(adj(X) Y)                                 (= sgn r_I J_I)
  s(g) = d (v0^2 - ex0) + 2 tr(adj(X)(Z - v0 Y)) + 2 e2(X, Y)
                                                  (= sgn r_I (J_I^2 - K_I))

where J_I = tr(L^g[S,:] Theta_I), K_I = tr((L^g[S,:] Theta_I)^2) are the
single-determinant Coulomb and exchange pieces and e2(X, Y) is the t^2
coefficient of det(X + t Y).  Then

  E_L = E0 + sum_s tr(h G^s)
        + (1/Obar) sum_I c~_I sum_g [a_a a_b + 1/2 s_a d_b + 1/2 s_b d_a].

The sum over Cholesky vectors runs in ``wick_gamma.c`` (plain C loops, one
determinant at a time, OpenMP over determinants) because the same sums in
NumPy take minutes per walker at 2 x 10^5 determinants.
"""
from __future__ import annotations

import ctypes as C
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wick_gamma.c")
_LIB = os.path.join(_HERE, "libwick_gamma.so")
_lib = None


# ----------------------------------------------------------------------------
# the C part: build and load
# ----------------------------------------------------------------------------

def build_c(verbose: bool = False) -> str:
    """Compile ``wick_gamma.c`` into ``libwick_gamma.so`` beside it (gcc)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"oracle C part failed to compile\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, _LIB)
    if verbose:
        print(f"built {_LIB}")
    return _LIB


class _SpinIn(C.Structure):
    _fields_ = [("kmax", C.c_int32), ("pmax", C.c_int32), ("n_rows", C.c_int32),
                ("n_cols", C.c_int32), ("k", C.c_void_p), ("slot", C.c_void_p),
                ("prow", C.c_void_p), ("detx", C.c_void_p), ("adj", C.c_void_p),
                ("kmin", C.c_void_p), ("lam", C.c_void_p), ("xi", C.c_void_p),
                ("v0", C.c_void_p), ("ex0", C.c_void_p)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_c()
        lib = C.CDLL(_LIB)
        lib.wick_gamma_sums.argtypes = [C.c_int64, C.c_int32, C.POINTER(_SpinIn),
                                        C.POINTER(_SpinIn), C.c_void_p]
        lib.wick_gamma_sums.restype = None
        _lib = lib
    return _lib


# ----------------------------------------------------------------------------
# excitations relative to the reference (Sec. II.B, Eq. 15)
# ----------------------------------------------------------------------------

class Excitations:
    """Holes, particles and signs of every determinant of one spin relative to
    row 0 (the reference).

    k[I]             excitation order
    hole[I, m]       m-th hole orbital (ascending), padded with -1
    slot[I, m]       its position in the reference list
    part[I, n]       n-th particle orbital (ascending), padded with -1
    sign[I]          parity (+1 / -1) of the permutation that sorts the
                     reference list with slot[I, m] holding part[I, m]
    """

    def __init__(self, occ: np.ndarray, M: int):
        occ = np.asarray(occ, dtype=np.int64)
        n_det, N = occ.shape
        self.ref = np.sort(occ[0])
        self.N = N
        in_det = np.zeros((n_det, M), dtype=bool)
        if N:
            np.put_along_axis(in_det, occ, True, axis=1)
        in_ref = np.zeros(M, dtype=bool)
        in_ref[self.ref] = True
        holes = in_ref[None, :] & ~in_det
        parts = in_det & ~in_ref[None, :]
        self.k = holes.sum(axis=1).astype(np.int32)
        kmax = int(self.k.max()) if n_det else 0
        self.kmax = kmax
        orb = np.arange(M)
        # the k smallest marked orbitals of every row, ascending
        self.hole = np.sort(np.where(holes, orb, M), axis=1)[:, :kmax]
        self.part = np.sort(np.where(parts, orb, M), axis=1)[:, :kmax]
        pad = np.arange(kmax)[None, :] >= self.k[:, None]
        self.hole[pad] = -1
        self.part[pad] = -1
        slot_of = np.full(M, -1, dtype=np.int64)
        slot_of[self.ref] = np.arange(N)
        self.slot = np.where(pad, -1, slot_of[np.maximum(self.hole, 0)])
        self.sign = self._signs()

    def _signs(self, chunk: int = 4096) -> np.ndarray:
        n_det, N = self.hole.shape[0], self.N
        out = np.ones(n_det, dtype=np.int64)
        for i0 in range(0, n_det, chunk):
            i1 = min(n_det, i0 + chunk)
            lst = np.broadcast_to(self.ref, (i1 - i0, N)).copy()
            for m in range(self.kmax):
                rows = np.nonzero(self.k[i0:i1] > m)[0]
                lst[rows, self.slot[i0 + rows, m]] = self.part[i0 + rows, m]
            # parity = number of inversions mod 2
            inv = np.zeros(i1 - i0, dtype=np.int64)
            for j in range(N):
                inv += np.sum(lst[:, :j] > lst[:, j:j + 1], axis=1)
            out[i0:i1] = np.where(inv % 2 == 0, 1, -1)
        return out


# ----------------------------------------------------------------------------
# small-matrix pieces: determinant, adjugate, complementary two-minors
# ----------------------------------------------------------------------------

def _det(x: np.ndarray) -> np.ndarray:
    """det of a stack of k x k matrices (1 for k = 0)."""
    if x.shape[-1] == 0:
        return np.ones(x.shape[:-2], dtype=np.complex128)
    return np.linalg.det(x)


def _minor(x: np.ndarray, rows, cols) -> np.ndarray:
    """det of x without the given rows and columns, for a stack."""
    keep_r = [i for i in range(x.shape[-2]) if i not in rows]
    keep_c = [j for j in range(x.shape[-1]) if j not in cols]
    return _det(x[..., keep_r, :][..., :, keep_c])


def adjugate_cofactor(x: np.ndarray) -> np.ndarray:
    """adj(X)[n, m] = (-1)^(n+m) det(X without row m, column n), for a stack
    of k x k matrices; exact for singular X.  adj of a 1 x 1 matrix is [1]."""
    k = x.shape[-1]
    out = np.zeros(x.shape, dtype=np.complex128)
    for m in range(k):
        for n in range(k):
            out[..., n, m] = (-1) ** (n + m) * _minor(x, (m,), (n,))
    return out


def complementary_two_minors(x: np.ndarray) -> np.ndarray:
    """K[A, B] = (-1)^(m+m'+n+n') det(X without rows m, m' and columns n, n')
    for row pairs A = (m < m') and column pairs B = (n < n'), lexicographic;
    shape (..., P, P), P = k (k - 1) / 2.  The minor of a 2 x 2 matrix with
    both rows and columns removed is 1."""
    k = x.shape[-1]
    pairs = list(itertools.combinations(range(k), 2))
    out = np.zeros(x.shape[:-2] + (len(pairs), len(pairs)), dtype=np.complex128)
    for A, (m, m2) in enumerate(pairs):
        for B, (n, n2) in enumerate(pairs):
            out[..., A, B] = (-1) ** (m + m2 + n + n2) * _minor(x, (m, m2), (n, n2))
    return out


def e2_laplace(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Second-order coefficient of det(X + t Y) for one k x k pair (NumPy
    twin of the expansion the C part uses; for the pins)."""
    k = x.shape[-1]
    kk = complementary_two_minors(x)
    out = 0.0 + 0.0j
    for A, (m, m2) in enumerate(itertools.combinations(range(k), 2)):
        for B, (n, n2) in enumerate(itertools.combinations(range(k), 2)):
            out += kk[A, B] * (y[m, n] * y[m2, n2] - y[m, n2] * y[m2, n])
    return out


# ----------------------------------------------------------------------------
# per walker
# ----------------------------------------------------------------------------

class _Spin:
    """Reference pieces and per-determinant excitation matrices of one spin
    for one walker."""

    def __init__(self, phi: np.ndarray, ex: Excitations):
        self.ex = ex
        M = phi.shape[0]
        self.M = M
        if ex.N == 0:
            self.logdet = 0.0 + 0.0j
            self.T = np.zeros((M, 0), dtype=np.complex128)
        else:
            a = phi[ex.ref]
            sgn, logabs = np.linalg.slogdet(a)
            if sgn == 0:
                raise np.linalg.LinAlgError("singular reference block")
            self.logdet = complex(logabs) + 1j * np.angle(sgn)
            self.T = np.linalg.solve(a.T, phi.T).T          # Phi A^{-1}
        self.G0 = np.zeros((M, M), dtype=np.complex128)
        self.G0[ex.ref, :] = self.T.T

    def excitation_matrices(self, idx: np.ndarray, k: int) -> np.ndarray:
        """X[I, m, n] = T[p_n, slot(h_m)] for the determinants idx, all of order k."""
        ex = self.ex
        if k == 0:
            return np.zeros((len(idx), 0, 0), dtype=np.complex128)
        p = ex.part[idx, :k]
        sl = ex.slot[idx, :k]
        return self.T[p[:, None, :], sl[:, :, None]]


def _by_order(k: np.ndarray):
    for kk in np.unique(k):
        yield int(kk), np.nonzero(k == kk)[0]


def _det_and_adj(sp: _Spin, n_det: int):
    """det X and adj(X) (padded to kmax) of every determinant of one spin."""
    kmax = sp.ex.kmax
    d = np.ones(n_det, dtype=np.complex128)
    adj = np.zeros((n_det, kmax, kmax), dtype=np.complex128)
    for k, idx in _by_order(sp.ex.k):
        if k == 0:
            continue
        x = sp.excitation_matrices(idx, k)
        d[idx] = _det(x)
        adj[idx, :k, :k] = adjugate_cofactor(x)
    return d, adj


def walker_wick(h1, chol, e0, ci, ex_a: Excitations, ex_b: Excitations, phi_a, phi_b, dt,
                energy=True, chunk=8192, per_det=False):
    """log <Psi_T|Phi>, G^a, G^b, xbar and (optionally) E_L of one walker.

    per_det: also return ``two_body_det``, the per-determinant sums
    sum_g [a_a a_b + 1/2 s_a d_b + 1/2 s_b d_a] before the c~_I weighting
    (= det X_a det X_b times the determinant's own two-body energy), and
    ``det_x`` = (det X_a, det X_b) per determinant."""
    M = phi_a.shape[0]
    n_det = len(ci)
    sa, sb = _Spin(phi_a, ex_a), _Spin(phi_b, ex_b)
    da, adj_a = _det_and_adj(sa, n_det)
    db, adj_b = _det_and_adj(sb, n_det)
    ct = np.conj(ci) * ex_a.sign * ex_b.sign                 # c~_I
    obar = np.sum(ct * da * db)
    log_o = np.log(obar) + sa.logdet + sb.logdet

    # Green's functions from the cofactor matrices
    greens = []
    for sp, adj, d_other in ((sa, adj_a, db), (sb, adj_b, da)):
        c = np.zeros((M, M), dtype=np.complex128)
        w = ct * d_other
        for m in range(sp.ex.kmax):
            for n in range(sp.ex.kmax):
                sel = (sp.ex.k > m) & (sp.ex.k > n)
                np.add.at(c, (sp.ex.part[sel, n], sp.ex.hole[sel, m]), w[sel] * adj[sel, n, m])
        g = sp.G0 - (sp.G0 - np.eye(M)) @ c @ sp.G0 / obar
        greens.append(g)
    ga, gb = greens
    xbar = -1j * np.sqrt(dt) * np.einsum("gpq,pq->g", chol, ga + gb)
    out = dict(log_ovlp=log_o, green=(ga, gb), force_bias=xbar)
    if not energy:
        return out

    # Cholesky pieces per spin
    n_g = chol.shape[0]
    spins = []
    for sp in (sa, sb):
        ex = sp.ex
        if ex.N:
            q = chol[:, ex.ref, :] @ sp.T                     # Q^g = L^g[R, :] T
        else:
            q = np.zeros((n_g, 0, 0), dtype=np.complex128)
        v0 = np.trace(q, axis1=1, axis2=2)
        ex0 = np.einsum("gij,gji->g", q, q)
        vrows = np.unique(ex.part[ex.part >= 0])
        lam = sp.T[vrows, :][None] @ q - chol[:, vrows, :] @ sp.T   # Lambda^g
        xi = lam @ q                                                   # Xi^g
        row_of = np.full(M, -1, dtype=np.int64)
        row_of[vrows] = np.arange(len(vrows))
        prow = np.where(ex.part >= 0, row_of[np.maximum(ex.part, 0)], -1)
        spins.append(dict(
            v0=np.ascontiguousarray(v0), ex0=np.ascontiguousarray(ex0),
            lam=np.ascontiguousarray(np.transpose(lam, (1, 2, 0))),   # [row][col][g]
            xi=np.ascontiguousarray(np.transpose(xi, (1, 2, 0))),
            prow=prow.astype(np.int32), n_rows=len(vrows)))

    lib = _load()
    num = 0.0 + 0.0j
    parts = []
    for i0 in range(0, n_det, chunk):
        i1 = min(n_det, i0 + chunk)
        args = []
        keep = []
        for sp, info, d, adj in ((sa, spins[0], da, adj_a), (sb, spins[1], db, adj_b)):
            ex = sp.ex
            kmax = max(ex.kmax, 1)
            pmax = max(kmax * (kmax - 1) // 2, 1)
            kmin = np.zeros((i1 - i0, pmax, pmax), dtype=np.complex128)
            kk = ex.k[i0:i1]
            for k, idx in _by_order(kk):
                if k >= 2:
                    p = k * (k - 1) // 2
                    kmin[idx, :p, :p] = complementary_two_minors(
                        sp.excitation_matrices(i0 + idx, k))
            arrs = dict(
                k=np.ascontiguousarray(kk, dtype=np.int32),
                slot=np.ascontiguousarray(_pad(ex.slot[i0:i1], kmax), dtype=np.int32),
                prow=np.ascontiguousarray(_pad(info["prow"][i0:i1], kmax), dtype=np.int32),
                detx=np.ascontiguousarray(d[i0:i1]),
                adj=np.ascontiguousarray(_pad_sq(adj[i0:i1], kmax)),
                kmin=kmin)
            keep.append(arrs)
            s = _SpinIn(kmax, pmax, info["n_rows"], ex.N,
                        *[a.ctypes.data for a in (arrs["k"], arrs["slot"], arrs["prow"],
                                                  arrs["detx"], arrs["adj"], arrs["kmin"])],
                        info["lam"].ctypes.data, info["xi"].ctypes.data,
                        info["v0"].ctypes.data, info["ex0"].ctypes.data)
            args.append(s)
        res = np.zeros(i1 - i0, dtype=np.complex128)
        lib.wick_gamma_sums(i1 - i0, n_g, C.byref(args[0]), C.byref(args[1]), res.ctypes.data)
        num += np.sum(ct[i0:i1] * res)
        if per_det:
            parts.append(res)
    one_body = np.sum(h1 * (ga + gb))
    out["e_loc"] = complex(e0 + one_body + num / obar)
    if per_det:
        out["two_body_det"] = np.concatenate(parts) if parts else np.zeros(0, complex)
        out["det_x"] = (da, db)
    return out


def _pad(a: np.ndarray, k: int) -> np.ndarray:
    """Columns of a 2-D index array padded (with 0) or cut to k."""
    out = np.zeros((a.shape[0], k), dtype=np.int64)
    w = min(k, a.shape[1])
    out[:, :w] = np.maximum(a[:, :w], 0)
    return out


def _pad_sq(a: np.ndarray, k: int) -> np.ndarray:
    out = np.zeros((a.shape[0], k, k), dtype=np.complex128)
    w = min(k, a.shape[1])
    out[:, :w, :w] = a[:, :w, :w]
    return out


def measure(h1, chol, e0, ci, occ_a, occ_b, phi_a, phi_b, dt, walkers=None, energy=True):
    """log <Psi_T|Phi_w>, xbar_w, E_L(w) and G_w of the selected walkers (same
    keys as ``oracle.msd.measure``, plus ``green``: a list of (G^a, G^b))."""
    M = phi_a.shape[1]
    ex_a, ex_b = Excitations(occ_a, M), Excitations(occ_b, M)
    sel = range(phi_a.shape[0]) if walkers is None else list(walkers)
    res = [walker_wick(h1, chol, e0, np.asarray(ci, dtype=np.complex128), ex_a, ex_b,
                       phi_a[w], phi_b[w], dt, energy=energy) for w in sel]
    out = dict(log_ovlp=np.array([r["log_ovlp"] for r in res]),
               force_bias=np.array([r["force_bias"] for r in res]),
               green=[r["green"] for r in res])
    if energy:
        out["e_loc"] = np.array([r["e_loc"] for r in res])
    return out

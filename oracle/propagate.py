"""One phaseless AFQMC step per walker, written plainly (TEST INFRASTRUCTURE ONLY).

Readings of the paper used here:

* Eq. 4: h' = h - 1/2 sum_r (pr|rq) = h - 1/2 sum_g L^g L^g.
* Eq. 5 with the first-order (symmetric) split B(x) = e^{-dt h'/2}
  e^{VHS(x)} e^{-dt h'/2}, VHS(x) = i sqrt(dt) sum_g x_g L^g, applied to the
  walker's orbitals (Thouless); exp(VHS) is the Taylor polynomial
  sum_{n=0}^{n_taylor} VHS^n / n!.
* Eqs. 7-12: the walker is propagated with the shifted fields x - xbar;
  S = <Psi_T|Phi'>/<Psi_T|Phi>, I = S exp(x.xbar - xbar.xbar/2) with plain
  (bilinear, unconjugated) dot products, w <- w |I| max(0, cos arg S),
  optionally times exp(dt e_shift).  A walker whose weight is already 0 is
  left unchanged (frozen).
* Periodic re-orthonormalisation: Phi = Q R with diag(R) real positive,
  Phi <- Q, log <Psi_T|Phi> -= sum_s log det R^s.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import msd


def h_prime(h1, chol):
    """h'_pq = h_pq - 1/2 sum_g sum_r L^g_pr L^g_rq (Eq. 4)."""
    return h1 - 0.5 * np.einsum("gpr,grq->pq", chol, chol)


def one_body_half_step(h1, chol, dt):
    """B1 = expm(-dt h' / 2), the one-body factor on each side of e^{VHS}."""
    return scipy.linalg.expm(-0.5 * dt * h_prime(h1, chol))


def vhs(chol, shifted_fields, dt):
    """VHS = i sqrt(dt) sum_g y_g L^g for y = x - xbar (complex)."""
    return 1j * np.sqrt(dt) * np.einsum("g,gpq->pq", shifted_fields, chol)


def taylor_apply(v, phi, n_taylor):
    """sum_{n=0}^{n_taylor} V^n phi / n!, term by term."""
    out = phi.astype(np.complex128).copy()
    term = phi.astype(np.complex128).copy()
    for n in range(1, n_taylor + 1):
        term = v @ term / n
        out = out + term
    return out


def propagate_orbitals(phi, b1, v, n_taylor):
    """Phi' = B1 exp_T(V) B1 Phi."""
    return b1 @ taylor_apply(v, b1 @ phi, n_taylor)


def importance_weight(w, log_o_old, log_o_new, x, xbar, dt=0.0, e_shift=0.0):
    """Phaseless weight update (Eqs. 8-12) for one walker."""
    s = np.exp(log_o_new - log_o_old)
    imp = s * np.exp(np.dot(x, xbar) - 0.5 * np.dot(xbar, xbar))
    cos_theta = np.cos(np.angle(s))
    return w * abs(imp) * max(0.0, cos_theta) * np.exp(dt * e_shift)


def qr_positive(phi):
    """Phi = Q R with R upper triangular and diag(R) real positive."""
    q, r = np.linalg.qr(phi)
    d = np.diag(r)
    ph = d / np.abs(d)
    q = q * ph[None, :]
    r = np.conj(ph)[:, None] * r
    return q, r


def step(h1, chol, ci, occ_a, occ_b, phi_a, phi_b, weights, log_ovlp,
         x, dt, n_taylor=6, e_shift=0.0, do_qr=False, b1=None):
    """One propagation step for all walkers.

    Inputs are arrays over walkers; returns new (phi_a, phi_b, weights,
    log_ovlp, xbar).  ``log_ovlp`` must be log <Psi_T|Phi_w> of the inputs.
    """
    if b1 is None:
        b1 = one_body_half_step(h1, chol, dt)
    nw = phi_a.shape[0]
    pa, pb = phi_a.copy(), phi_b.copy()
    wts, lo = weights.copy(), log_ovlp.copy()
    xbars = np.zeros((nw, chol.shape[0]), dtype=np.complex128)
    for w in range(nw):
        ga, gb = msd.green(ci, occ_a, occ_b, phi_a[w], phi_b[w])
        xbar = msd.force_bias(chol, ga, gb, dt)
        xbars[w] = xbar
        if weights[w] == 0.0:
            continue
        v = vhs(chol, x[w] - xbar, dt)
        na = propagate_orbitals(phi_a[w], b1, v, n_taylor)
        nb = propagate_orbitals(phi_b[w], b1, v, n_taylor)
        lo_new = np.log(msd.trial_overlap(ci, occ_a, occ_b, na, nb))
        wts[w] = importance_weight(weights[w], log_ovlp[w], lo_new, x[w], xbar,
                                   dt, e_shift)
        if do_qr:
            qa, ra = qr_positive(na)
            qb, rb = qr_positive(nb)
            na, nb = qa, qb
            lo_new = lo_new - np.sum(np.log(np.diag(ra).real)) \
                - np.sum(np.log(np.diag(rb).real))
        pa[w], pb[w], lo[w] = na, nb, lo_new
    return pa, pb, wts, lo, xbars

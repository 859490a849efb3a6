"""Block driver around the propagation step (TEST INFRASTRUCTURE ONLY).

Plain CPU code that the tests compare the library's block driver against;
nothing on the product path imports it.

Readings of the paper used here:

* Sec. III.B and Listing 1: a block is 25 propagation steps with
  re-orthonormalisation and population control every 5 steps each and one
  local-energy estimate.  The paper does not say which population-control
  algorithm runs, nor where in the block the estimate is taken; this module
  takes the comb method (below) and measures once, after the block's last
  step (and after that step's population control).
* The comb: with cumulative weights C_i = w_0 + ... + w_i and total
  W = C_{n-1}, tooth k (k = 0 .. n-1) sits at t_k = (k + z) W / n for one
  uniform offset z in [0, 1) drawn by the caller; walker k of the new
  population is a copy of the walker i with C_{i-1} <= t_k < C_i, and every
  new weight is W / n.  A walker of weight 0 owns an empty interval and is
  never copied.  Each walker is copied floor or ceil of n w_i / W times, and
  on average over z exactly n w_i / W times.  If W is 0 nothing changes.
* The block's energy is the weighted mixed estimate
  E = sum_w w E_L(w) / sum_w w over walkers of positive weight; numerator
  and denominator are returned.

Parity pinned by tests/test_oracle_pins.py: identity on equal weights, the
floor/ceil copy counts, unbiasedness over a grid of offsets, zero-weight
walkers never copied, a brute-force tooth search on small inputs; the block
reduces to plain steps plus one measurement when population control is off.
"""
from __future__ import annotations

import numpy as np

from . import msd, propagate


def comb(weights, z):
    """Comb resampling: (parent index per new walker, new common weight)."""
    w = np.asarray(weights, dtype=np.float64)
    n = w.shape[0]
    c = np.cumsum(w)
    total = c[-1]
    if not total > 0.0:
        return np.arange(n), None
    teeth = (np.arange(n) + z) * total / n
    # smallest i with C_i > t_k
    parent = np.searchsorted(c, teeth, side="right")
    # a tooth rounded up onto W belongs to the last walker of positive weight
    last = int(np.nonzero(w > 0.0)[0][-1])
    parent = np.minimum(parent, last)
    return parent, total / n


def block(h1, chol, e0, ci, occ_a, occ_b, phi_a, phi_b, weights, log_ovlp, fields, dt, zs,
          n_taylor=6, e_shift=0.0, stabilize_freq=5, pop_freq=5, steps_before=0):
    """One block: len(fields) steps, comb after every pop_freq-th step (offsets
    zs in order), then one measurement.

    ``steps_before`` counts the steps taken before the block (the
    re-orthonormalisation schedule runs over the whole simulation).  Returns
    (phi_a, phi_b, weights, log_ovlp, e_loc, sum_w w E_L, sum_w w).
    """
    pa, pb = phi_a.copy(), phi_b.copy()
    wts, lo = weights.copy(), log_ovlp.copy()
    b1 = propagate.one_body_half_step(h1, chol, dt)
    j = 0
    for s in range(len(fields)):
        k = steps_before + s + 1
        do_qr = stabilize_freq > 0 and k % stabilize_freq == 0
        pa, pb, wts, lo, _ = propagate.step(h1, chol, ci, occ_a, occ_b, pa, pb, wts, lo,
                                            fields[s], dt, n_taylor=n_taylor,
                                            e_shift=e_shift, do_qr=do_qr, b1=b1)
        if pop_freq > 0 and (s + 1) % pop_freq == 0:
            parent, wn = comb(wts, zs[j])
            j += 1
            if wn is not None:
                pa, pb, lo = pa[parent], pb[parent], lo[parent]
                wts = np.full_like(wts, wn)
    out = msd.measure(h1, chol, e0, ci, occ_a, occ_b, pa, pb, dt, energy=True)
    e_loc = out["e_loc"]
    live = wts > 0.0  # a walker of weight 0 adds nothing (its E_L is not used)
    return (pa, pb, wts, lo, e_loc, np.sum(wts[live] * e_loc[live]), np.sum(wts[live]))

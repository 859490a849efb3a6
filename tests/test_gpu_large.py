"""GPU parity at the larger synthetic shapes, on sampled outputs.

The full batch runs on the GPU in its normal launch configuration; the oracle
recomputes a sample of walkers.  Brute-force local energies over 10^4 or more
determinants are beyond the oracle, so energies are compared with the same
batch and a truncated trial (the first determinants of the expansion).
"""
import numpy as np
import pytest

from oracle import msd
from paper_2406_08314_amd import MsdSystem
from synth import make_config

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _system(wl):
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
    return s


def test_cu_oxo_full_batch_overlap_green_force_bias():
    wl = make_config("cu_oxo")
    s = _system(wl)
    out = s.measure(wl.dt, energy=False)
    for w in (0, 17, 101, 255):
        ref = np.log(msd.trial_overlap(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w]))
        assert abs(np.exp(out["log_ovlp"][w] - ref) - 1) < TOL
    for w in (200,):
        ga, gb = msd.green(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w])
        fb = msd.force_bias(wl.chol, ga, gb, wl.dt)
        assert np.max(np.abs(out["force_bias"][w] - fb)) <= TOL * np.max(np.abs(fb))
        g_a, g_b = s.get_green(w)
        assert np.max(np.abs(g_a - ga)) <= TOL * max(1.0, np.max(np.abs(ga)))
        assert np.max(np.abs(g_b - gb)) <= TOL * max(1.0, np.max(np.abs(gb)))


def test_cu_oxo_full_batch_energy_truncated_trial():
    wl = make_config("cu_oxo", n_det=60)
    s = _system(wl)
    out = s.measure(wl.dt)
    for w in (250,):
        ref = msd.local_energy(wl.h1, wl.chol, wl.e0, wl.ci, wl.occ_a, wl.occ_b,
                               wl.phi_a[w], wl.phi_b[w])
        assert abs(out["e_loc"][w] - ref) <= TOL * max(1.0, abs(ref))

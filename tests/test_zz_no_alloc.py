"""The allocation-free population control (msd_population_control_noalloc)
against the handle-scratch entry point (msd_population_control_dev): two calls
in a row on one GPU, the second with a smaller system, each compared bit for
bit (parents, walkers, weights, log overlaps) with a twin handle; and the
size limit of the static scratch."""
import numpy as np
import pytest

from paper_2406_08314_amd import MsdError, MsdSystem
from synth import make_config, make_workload

pytestmark = pytest.mark.gpu


def _twin(wl, weights):
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a, wl.phi_b, weights)
    return s


def _weights(n, seed):
    rng = np.random.default_rng(seed)
    w = rng.lognormal(0.0, 0.8, n)
    w[rng.choice(n, size=max(1, n // 7), replace=False)] = 0.0  # never copied
    return w


def _compare(wl, z, seed):
    import torch

    w = _weights(wl.n_walkers, seed)
    a, b = _twin(wl, w), _twin(wl, w)
    pa = torch.full((wl.n_walkers,), -1, dtype=torch.int32, device="cuda:0")
    pb = torch.full((wl.n_walkers,), -2, dtype=torch.int32, device="cuda:0")
    a.population_control_dev(z, pa)
    b.population_control_noalloc(z, pb)
    torch.cuda.synchronize()
    assert torch.equal(pa, pb)
    assert int(pb.min()) >= 0
    assert np.all(w[pb.cpu().numpy()] > 0.0)
    ra, rb = a.get_walkers(), b.get_walkers()
    for x, y in zip(ra, rb):
        np.testing.assert_array_equal(x, y)
    # a second comb with the parents left to the scratch (parent = NULL)
    a.population_control_dev(0.5 * z)
    b.population_control_noalloc(0.5 * z)
    for x, y in zip(a.get_walkers(), b.get_walkers()):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_noalloc_comb_matches_handle_scratch_two_calls():
    big = make_config("medium", n_walkers=96, n_det=50)
    _compare(big, 0.37, 11)
    small = make_workload("small", M=20, n_alpha=4, n_beta=3, n_chol=10, n_det=12, k_max=2,
                          window=(3, 6), c_law="flat", n_walkers=9, seed=5)
    _compare(small, 0.81, 12)


def test_noalloc_comb_rejects_oversize():
    """512 walkers of 300 orbitals and 90 electrons need 221 MB of scratch,
    beyond the 128 MiB array: a clear error, and nothing changes."""
    wl = make_workload("big", M=300, n_alpha=45, n_beta=45, n_chol=1, n_det=2, k_max=1,
                       window=(1, 1), c_law="flat", n_walkers=512, seed=3)
    s = _twin(wl, np.ones(wl.n_walkers))
    with pytest.raises(MsdError) as e:
        s.population_control_noalloc(0.5)
    assert e.value.name == "MSD_ERR_UNSUPPORTED"
    assert "bytes of scratch" in str(e.value)
    pa, pb, w, lo = s.get_walkers()
    np.testing.assert_array_equal(pa, wl.phi_a)
    s.close()

"""GPU parity at the larger synthetic shapes, at full size, on sampled walkers.

The whole batch runs on the GPU in its normal launch configuration; the oracle
recomputes a sample of walkers.  Overlaps, Green's functions and force biases
are compared with the brute-force oracle (``oracle.msd``) where it finishes in
seconds (Cu-oxo shape); local energies, and everything at the Fe2S2 shape,
with the oracle's per-determinant generalised-Wick path (``oracle.wick``),
which is pinned to the brute-force oracle and to Fock space on small systems.
"""
import numpy as np
import pytest

from oracle import msd, wick
from paper_2406_08314_amd import MsdSystem
from synth import make_config, make_workload

pytestmark = pytest.mark.gpu

TOL = 1e-10
MIXED_E_TOL = 1e-4  # Ha: the mixed form's per-walker local-energy bound (0.1 mHa)


def _system(wl, precision="fp64"):
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det,
                  precision=precision)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
    return s


def _rel(gpu, ref, floor=1.0):
    gpu, ref = np.asarray(gpu), np.asarray(ref)
    return float(np.max(np.abs(gpu - ref))) / max(floor, float(np.max(np.abs(ref))))


@pytest.fixture(scope="module")
def cu_oxo():
    wl = make_config("cu_oxo")
    ex = (wick.Excitations(wl.occ_a, wl.M), wick.Excitations(wl.occ_b, wl.M))
    return wl, ex


@pytest.fixture(scope="module")
def fe2s2():
    wl = make_config("fe2s2")
    ex = (wick.Excitations(wl.occ_a, wl.M), wick.Excitations(wl.occ_b, wl.M))
    return wl, ex


def _wick_walker(wl, ex, w):
    return wick.walker_wick(wl.h1, wl.chol, wl.e0, np.asarray(wl.ci, dtype=np.complex128),
                            ex[0], ex[1], wl.phi_a[w], wl.phi_b[w], wl.dt)


def _check_walker(s, out, ref, w):
    assert abs(np.exp(out["log_ovlp"][w] - ref["log_ovlp"]) - 1) < TOL
    assert _rel(out["force_bias"][w], ref["force_bias"], floor=0.0) <= TOL
    assert abs(out["e_loc"][w] - ref["e_loc"]) <= TOL * max(1.0, abs(ref["e_loc"]))
    g_a, g_b = s.get_green(w)
    assert _rel(g_a, ref["green"][0]) <= TOL
    assert _rel(g_b, ref["green"][1]) <= TOL


def test_cu_oxo_full_batch_overlap_green_force_bias_brute_force(cu_oxo):
    """All 10,000 determinants, 256 walkers: overlaps of four walkers and the
    Green's function and force bias of one against brute-force determinants."""
    wl, _ = cu_oxo
    s = _system(wl)
    out = s.measure(wl.dt, energy=False)
    for w in (0, 17, 101, 255):
        ref = np.log(msd.trial_overlap(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w]))
        assert abs(np.exp(out["log_ovlp"][w] - ref) - 1) < TOL
    for w in (200,):
        ga, gb = msd.green(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w])
        fb = msd.force_bias(wl.chol, ga, gb, wl.dt)
        assert _rel(out["force_bias"][w], fb, floor=0.0) <= TOL
        g_a, g_b = s.get_green(w)
        assert _rel(g_a, ga) <= TOL
        assert _rel(g_b, gb) <= TOL


def test_cu_oxo_full_batch_energy(cu_oxo):
    """Full Cu-oxo shape with energies (M=200, N=30+30, 1,200 Cholesky vectors,
    10,000 determinants of orders up to 4, 256 walkers): log-overlap, G,
    force bias and E_L of two walkers against the oracle's Wick path."""
    wl, ex = cu_oxo
    s = _system(wl)
    out = s.measure(wl.dt)
    assert np.all(np.isfinite(out["e_loc"]))
    for w in (1, 250):
        _check_walker(s, out, _wick_walker(wl, ex, w), w)


def test_cu_oxo_full_batch_mixed_every_walker(cu_oxo):
    """The mixed form at the full Cu-oxo shape: every walker's local energy
    within 0.1 mHa of the FP64 form, overlaps identical (they stay FP64)."""
    wl, _ = cu_oxo
    ref = _system(wl).measure(wl.dt)
    out = _system(wl, "mixed").measure(wl.dt)
    np.testing.assert_array_equal(out["log_ovlp"], ref["log_ovlp"])
    de = np.abs(out["e_loc"] - ref["e_loc"])
    print(f"mixed-form max |dE_L| over {wl.n_walkers} Cu-oxo walkers: {de.max() * 1e3:.4f} mHa")
    assert de.max() <= MIXED_E_TOL


def test_fe2s2_full_batch_energy(fe2s2):
    """Full Fe2S2 shape with energies (M=300, N=45+45, 2,000 Cholesky vectors,
    200,000 determinants of orders up to 6, 512 walkers): log-overlap, G, force
    bias and E_L of one walker against the oracle's Wick path, plus one more
    walker's overlap against brute-force determinants."""
    wl, ex = fe2s2
    s = _system(wl)
    out = s.measure(wl.dt)
    assert np.all(np.isfinite(out["e_loc"]))
    _check_walker(s, out, _wick_walker(wl, ex, 1), 1)
    ref = np.log(msd.trial_overlap(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[3], wl.phi_b[3]))
    assert abs(np.exp(out["log_ovlp"][3] - ref) - 1) < TOL


@pytest.mark.parametrize("form", ["fp64", "fp64_general", "mixed"])
def test_fe2s2_shape_energy_high_orders(form):
    """Fe2S2 shapes (window 15 x 5, excitation orders up to 6) with a short
    trial: all quantities of sampled walkers against the brute-force oracle;
    the mixed form's local energies within 0.1 mHa.  fp64_general: the FP64
    form through the general contraction kernel's six-column-tile instance
    with T in registers (not the FP64 form's default here).  At this shape the
    mixed form keeps FP64 energies (its FP32 path would need that instance for
    the walkers far from the reference)."""
    precision = "mixed" if form == "mixed" else "fp64"
    wl = make_workload("fe2s2_small", M=300, n_alpha=45, n_beta=45, n_chol=2000, n_det=24,
                       k_max=6, window=(15, 5), c_law="power1", n_walkers=64,
                       seed=240608317, complex_ci=True)
    s = _system(wl, precision)
    if form == "fp64_general":
        s.set_tuning(lambda_variant=6)
    out = s.measure(wl.dt)
    if form == "fp64_general":
        assert s.get_tuning()["lambda_variant"] == 6
    walkers = [5, 40]
    ref = msd.measure(wl.h1, wl.chol, wl.e0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a, wl.phi_b,
                      wl.dt, walkers=walkers)
    for i, w in enumerate(walkers):
        assert abs(np.exp(out["log_ovlp"][w] - ref["log_ovlp"][i]) - 1) < TOL
        fb = ref["force_bias"][i]
        e = ref["e_loc"][i]
        if precision == "fp64":
            assert _rel(out["force_bias"][w], fb, floor=0.0) <= TOL
            assert abs(out["e_loc"][w] - e) <= TOL * max(1.0, abs(e))
            ga, gb = msd.green(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w])
            g_a, g_b = s.get_green(w)
            assert _rel(g_a, ga) <= TOL
            assert _rel(g_b, gb) <= TOL
        else:
            assert _rel(out["force_bias"][w], fb, floor=0.0) <= 1e-5
            err = abs(out["e_loc"][w] - e)
            print(f"mixed-form |dE_L| at the Fe2S2 shape, walker {w}: {err * 1e3:.4f} mHa "
                  f"(|E_L| = {abs(e):.1f} Ha)")
            assert err <= MIXED_E_TOL


@pytest.fixture(scope="module")
def million():
    """10^6 determinants on the Cu-oxo shape, 64 walkers, and the oracle's
    Wick-path result for walker 7."""
    wl = make_config("cu_oxo", n_det=1_000_000, n_walkers=64)
    ex = (wick.Excitations(wl.occ_a, wl.M), wick.Excitations(wl.occ_b, wl.M))
    return wl, _wick_walker(wl, ex, 7)


@pytest.mark.parametrize("energy_algo", [0, 4])
def test_cu_oxo_shape_million_determinants(million, energy_algo):
    """10^6 determinants (orders up to 4) on the Cu-oxo shape (M=200, N=30+30,
    1,200 Cholesky vectors), 64 walkers: one walker's log-overlap, Green's
    function, force bias and local energy against the oracle's Wick path, in
    the automatic energy form and in the W-form."""
    wl, ref = million
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det,
                  energy_algo=energy_algo)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
    out = s.measure(wl.dt)
    assert np.all(np.isfinite(out["e_loc"]))
    _check_walker(s, out, ref, 7)
    s.close()

"""GPU parity of the general fused Cholesky-contraction kernel (energy
intermediates on the matrix cores for any electron count up to 48 per spin,
up to 320 orbitals, windows of up to 32 x 32): every column-tile count, both
virtual-row-tile counts, both occupied-window paddings, ragged orbital slabs,
ragged vector chunks and several walker tiles, against the brute-force oracle
(1e-10 relative) and, in the mixed form, against FP64 (0.1 mHa)."""
import numpy as np
import pytest

from oracle import msd
from paper_2406_08314_amd import MsdSystem
from synth import make_workload

pytestmark = pytest.mark.gpu

TOL = 1e-10
MIXED_E_TOL = 1e-4

# (N_alpha, N_beta, M, n_chol, window (occ, vir), k_max, n_det, walkers)
SHAPES = {
    "n12_m40": (12, 12, 40, 24, (6, 10), 4, 40, 5),
    "n20_m100": (20, 18, 100, 30, (16, 24), 4, 60, 4),
    "n30_m150_unequal": (30, 28, 150, 20, (16, 32), 4, 40, 3),
    "n40_m96": (40, 40, 96, 16, (20, 12), 3, 30, 3),
    "n8_m70": (8, 8, 70, 40, (8, 20), 4, 50, 6),
    "n32_occ32": (32, 32, 72, 12, (32, 12), 3, 30, 3),
    # T beyond the LDS (FP64): the register-resident form of T
    "n20_m240": (20, 20, 240, 16, (12, 16), 3, 30, 3),
    "n16_m300": (16, 14, 300, 12, (10, 14), 3, 30, 3),
}


def _system(wl, precision="fp64", **tuning):
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det,
                  precision=precision)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
    if tuning:
        s.set_tuning(**tuning)
    return s


def _workload(name, seed=977):
    na, nb, M, ng, window, kmax, nd, nw = SHAPES[name]
    return make_workload(name, M=M, n_alpha=na, n_beta=nb, n_chol=ng, n_det=nd, k_max=kmax,
                         window=window, c_law="flat", n_walkers=nw, seed=seed, complex_ci=True)


def _check(wl, out, walkers):
    ref = msd.measure(wl.h1, wl.chol, wl.e0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a, wl.phi_b,
                      wl.dt, walkers=walkers)
    for i, w in enumerate(walkers):
        assert abs(np.exp(out["log_ovlp"][w] - ref["log_ovlp"][i]) - 1) < TOL
        fb = ref["force_bias"][i]
        assert np.max(np.abs(out["force_bias"][w] - fb)) <= TOL * np.max(np.abs(fb))
        e = ref["e_loc"][i]
        assert abs(out["e_loc"][w] - e) <= TOL * max(1.0, abs(e)), (w, out["e_loc"][w], e)


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_general_kernel_matches_oracle(name):
    wl = _workload(name)
    s = _system(wl)
    out = s.measure(wl.dt)
    assert s.get_tuning()["lambda_variant"] == 6
    _check(wl, out, [0, wl.n_walkers - 1])


@pytest.mark.parametrize("tuning", [
    dict(lambda_chunk=7),            # ragged chunks: 30 vectors in 7, 7, 7, 7, 2
    dict(lambda_chunk=1),
    dict(walker_tile=3),             # two walker tiles, the second partial
    dict(lambda_chunk=11, walker_tile=1),
])
def test_general_kernel_chunks_and_tiles(tuning):
    wl = _workload("n20_m100")
    s = _system(wl, lambda_variant=6, **tuning)
    out = s.measure(wl.dt)
    got = s.get_tuning()
    assert got["lambda_variant"] == 6
    for k, v in tuning.items():
        assert got[k] == v
    _check(wl, out, [1, 3])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_whole_string_items_match_row_pairs(precision):
    """Order-3 strings as whole-string items (one lane gathers the 3 x 3 block
    once per vector) against one row pair per lane: the same sums in another
    grouping (1e-10 relative in FP64; 1e-7 relative in the single-precision
    form, whose products round differently)."""
    wl = _workload("n30_m150_unequal")
    out = {}
    for whole in (1, 2):
        s = _system(wl, precision, second_whole=whole)
        out[whole] = s.measure(wl.dt)
        assert s.get_tuning()["second_whole"] == whole
    e1, e2 = out[1]["e_loc"], out[2]["e_loc"]
    tol = (TOL if precision == "fp64" else 1e-7) * max(1.0, np.max(np.abs(e1)))
    assert np.max(np.abs(e1 - e2)) <= tol
    if precision == "fp64":
        _check(wl, out[2], [0, wl.n_walkers - 1])


@pytest.mark.parametrize("name", ["n12_m40", "n30_m150_unequal", "n40_m96", "n20_m240"])
def test_general_kernel_mixed_against_fp64(name):
    wl = _workload(name)
    ref = _system(wl).measure(wl.dt)
    s = _system(wl, "mixed")
    out = s.measure(wl.dt)
    assert s.get_tuning()["lambda_variant"] == 6
    np.testing.assert_array_equal(out["log_ovlp"], ref["log_ovlp"])
    de = np.abs(out["e_loc"] - ref["e_loc"])
    assert de.max() <= MIXED_E_TOL, de.max()


def _flagged(wl, tmax=2.0):
    """Walkers whose max |T| over both spins exceeds tmax, T = Phi Phi[R, :]^-1
    with R the reference determinant's orbitals: the ones the mixed form sends
    to its FP64 pass."""
    out = []
    for w in range(wl.n_walkers):
        t = 0.0
        for phi, occ in ((wl.phi_a[w], wl.occ_a[0]), (wl.phi_b[w], wl.occ_b[0])):
            t = max(t, np.abs(phi @ np.linalg.inv(phi[occ])).max())
        out.append(t > tmax)
    return np.array(out)


@pytest.mark.parametrize("name", ["n20_m240", "n12_m40"])
def test_general_kernel_mixed_many_flagged_walkers(name):
    """Most walkers far from the reference: the mixed form's FP64 pass over the
    walker list takes several vector chunks per item (many listed walkers);
    their energies equal the FP64 form's up to summation order, the others stay
    within 0.1 mHa."""
    na, nb, M, _, window, kmax, nd, _ = SHAPES[name]
    wl = make_workload(name, M=M, n_alpha=na, n_beta=nb, n_chol=96, n_det=nd, k_max=kmax,
                       window=window, c_law="flat", n_walkers=48, seed=1201, complex_ci=True,
                       noise=1.0)
    flag = _flagged(wl)
    assert flag.sum() >= 22, flag.sum()  # at least two chunks per item
    ref = _system(wl).measure(wl.dt)
    s = _system(wl, "mixed")
    out = s.measure(wl.dt)
    assert s.get_tuning()["lambda_variant"] == 6
    e, e64 = out["e_loc"], ref["e_loc"]
    assert np.max(np.abs(e - e64)[flag]) <= TOL * max(1.0, np.max(np.abs(e64)))
    assert np.max(np.abs(e - e64)) <= MIXED_E_TOL

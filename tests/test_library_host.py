"""Host-side checks of the HIP library (no GPU needed): it loads, exports every
entry point of include/msd_afqmc.h, and its trial builder's excitation signs
satisfy the determinant identity det(Phi[S_I]) / det(Phi[R]) = sgn_I det X_I."""
import os
import re

import numpy as np
import pytest

from paper_2406_08314_amd import _lib, trial_analyze, MsdError
from synth import make_config, make_workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "msd_afqmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msd_[a-z_]+)\s*\(", text)))


def test_library_exports_header():
    lib = _lib.load()
    names = header_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, f"binding lacks {n}"


def test_status_strings():
    lib = _lib.load()
    for code in _lib.STATUS:
        assert lib.msd_status_string(code)


def _excitation_matrix(phi, ref, occ_row):
    """X_mn = T[p_n, slot(h_m)] with T = Phi Phi[ref]^{-1} (numpy)."""
    T = phi @ np.linalg.inv(phi[ref])
    S = set(occ_row.tolist())
    holes = sorted(set(ref) - S)
    parts = sorted(S - set(ref))
    slot = {r: j for j, r in enumerate(ref)}
    return np.array([[T[p, slot[h]] for p in parts] for h in holes]).reshape(len(holes), len(parts))


@pytest.mark.parametrize("cfg", ["tiny", "medium"])
def test_trial_signs_determinant_identity(cfg):
    wl = make_config(cfg, n_walkers=1)
    ka, kb, sg = trial_analyze(wl.M, wl.occ_a, wl.occ_b)
    ra, rb = list(wl.occ_a[0]), list(wl.occ_b[0])
    pa, pb = wl.phi_a[0], wl.phi_b[0]
    da0, db0 = np.linalg.det(pa[ra]), np.linalg.det(pb[rb])
    for I in range(0, wl.n_det, max(1, wl.n_det // 200)):
        xa = _excitation_matrix(pa, ra, wl.occ_a[I])
        xb = _excitation_matrix(pb, rb, wl.occ_b[I])
        assert xa.shape[0] == ka[I] and xb.shape[0] == kb[I]
        lhs = np.linalg.det(pa[wl.occ_a[I]]) * np.linalg.det(pb[wl.occ_b[I]]) / (da0 * db0)
        rhs = sg[I] * (np.linalg.det(xa) if ka[I] else 1.0) * (np.linalg.det(xb) if kb[I] else 1.0)
        assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(lhs)), I


def test_trial_signs_unsorted_reference_and_low_particles():
    # reference not the lowest orbitals: particles may lie below holes
    rng = np.random.default_rng(3)
    M = 9
    ref = [1, 4, 6, 8]
    occ = np.array([ref, [0, 4, 6, 8], [1, 2, 3, 8], [0, 2, 5, 7], [1, 4, 6, 7]], np.int32)
    occb = np.array([[0]] * 5, np.int32)
    ka, kb, sg = trial_analyze(M, occ, occb)
    phi = rng.standard_normal((M, 4)) + 1j * rng.standard_normal((M, 4))
    d0 = np.linalg.det(phi[ref])
    for I in range(5):
        x = _excitation_matrix(phi, ref, occ[I])
        lhs = np.linalg.det(phi[occ[I]]) / d0
        rhs = sg[I] * (np.linalg.det(x) if ka[I] else 1.0)
        assert abs(lhs - rhs) < 1e-10


@pytest.mark.parametrize("bad,frag", [
    (np.array([[0, 1, 2], [0, 1, 12]]), "outside"),
    (np.array([[0, 1, 2], [0, 1, 1]]), "repeated"),
    (np.array([[0, 1, -1], [0, 1, 2]]), "outside"),
])
def test_trial_validation_errors(bad, frag):
    occb = np.array([[0, 1, 2]] * len(bad), np.int32)
    with pytest.raises(MsdError) as ei:
        trial_analyze(12, bad.astype(np.int32), occb)
    assert ei.value.name == "MSD_ERR_TRIAL" and frag in str(ei.value)


def test_trial_excitation_order_limit():
    M = 24
    ref = list(range(9))
    exc = list(range(9, 18))
    occ = np.array([ref, exc], np.int32)
    occb = np.array([[0], [0]], np.int32)
    with pytest.raises(MsdError) as ei:
        trial_analyze(M, occ, occb)
    assert "exceeds" in str(ei.value)

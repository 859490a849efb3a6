"""Pins of the generalised-Wick CPU oracle path (``oracle.wick``).

It is tied to things other than itself: the brute-force determinant oracle
(``oracle.msd``, itself pinned to Fock space), explicit Jordan-Wigner Fock
space, the exact eigenvalue of an FCI trial, and the definitions of the
small-matrix pieces it uses (the t^2 coefficient of det(X + tY), X adj X =
det X, the overlap ratio det T[S, :]).  Excitation orders reach 6 per spin,
spins are unequal, and the walker-equal-to-reference case makes every
excitation matrix singular.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import fock, msd, wick
from synth import make_workload

RTOL = 1e-11


def rand_sym(rng, n, M, scale=1.0):
    a = rng.standard_normal((n, M, M))
    return scale * (a + a.transpose(0, 2, 1)) / 2


def cplx(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ----------------------------------------------------------------------------
# small-matrix pieces against their definitions
# ----------------------------------------------------------------------------

def e2_by_columns(x, y):
    """sum over column pairs n < n' of det(X with columns n, n' taken from Y)."""
    k = x.shape[0]
    tot = 0.0 + 0.0j
    for n, n2 in itertools.combinations(range(k), 2):
        z = x.copy()
        z[:, [n, n2]] = y[:, [n, n2]]
        tot += np.linalg.det(z)
    return tot


def e2_by_polynomial(x, y):
    """t^2 coefficient of det(X + tY): sample on a circle, discrete Fourier
    transform (exact for a polynomial of degree k < number of samples)."""
    k = x.shape[0]
    n = k + 1
    r = 0.5
    ts = r * np.exp(2j * np.pi * np.arange(n) / n)
    vals = np.array([np.linalg.det(x + t * y) for t in ts])
    # c_l r^l = (1/n) sum_j vals_j exp(-2 pi i j l / n)
    return np.sum(vals * np.exp(-2j * np.pi * 2 * np.arange(n) / n)) / n / r ** 2


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("rank_drop", [0, 1, 2])
def test_e2_matches_definitions(k, rank_drop):
    rng = np.random.default_rng(100 + 10 * k + rank_drop)
    x = cplx(rng, k, k)
    if rank_drop:
        x = cplx(rng, k, k - rank_drop) @ cplx(rng, k - rank_drop, k)
    y = cplx(rng, k, k)
    got = wick.e2_laplace(x, y)
    ref1 = e2_by_columns(x, y)
    ref2 = e2_by_polynomial(x, y)
    scale = max(1.0, abs(ref1))
    assert abs(got - ref1) < 1e-11 * scale
    assert abs(got - ref2) < 1e-9 * scale
    if k == 2:
        assert abs(got - np.linalg.det(y)) < 1e-12 * scale


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_adjugate_cofactor(k):
    rng = np.random.default_rng(k)
    for r in (k, k - 1, max(k - 2, 0)):
        x = cplx(rng, k, r) @ cplx(rng, r, k) if r else np.zeros((k, k), complex)
        adj = wick.adjugate_cofactor(x[None])[0]
        scale = 1e-12 * max(1.0, np.abs(x).max() ** k)
        np.testing.assert_allclose(x @ adj, np.linalg.det(x) * np.eye(k), atol=scale)
        np.testing.assert_allclose(adj, msd.adjugate(x), atol=scale)
        if k >= 2 and r <= k - 2:
            assert np.max(np.abs(adj)) < scale


def test_excitation_sign_is_overlap_ratio():
    """sgn det X = det(Phi[S, :]) / det(Phi[R, :]) for every determinant,
    orders 0..6, with occupation rows given in scrambled order."""
    rng = np.random.default_rng(21)
    M, N = 14, 7
    ref = np.sort(rng.choice(M, N, replace=False))
    virt = np.setdiff1d(np.arange(M), ref)
    rows = [ref.copy()]
    for k in range(1, 7):
        for _ in range(4):
            h = rng.choice(ref, k, replace=False)
            p = rng.choice(virt, k, replace=False)
            row = np.concatenate([np.setdiff1d(ref, h), p])
            rows.append(rng.permutation(row))
    occ = np.array(rows, np.int32)
    phi = cplx(rng, M, N)
    ex = wick.Excitations(occ, M)
    sp = wick._Spin(phi, ex)
    for i in range(len(rows)):
        k = ex.k[i]
        x = sp.excitation_matrices(np.array([i]), k)[0]
        ratio = np.linalg.det(phi[np.sort(occ[i])]) / np.linalg.det(phi[ex.ref])
        assert abs(ex.sign[i] * (np.linalg.det(x) if k else 1.0) - ratio) < 1e-10 * max(1, abs(ratio))


# ----------------------------------------------------------------------------
# whole-walker quantities against the brute-force oracle
# ----------------------------------------------------------------------------

def _compare(wl, e0, walkers, tol=RTOL):
    ref = msd.measure(wl.h1, wl.chol, e0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a, wl.phi_b, wl.dt,
                      walkers=walkers)
    got = wick.measure(wl.h1, wl.chol, e0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a, wl.phi_b,
                       wl.dt, walkers=walkers)
    for i, w in enumerate(walkers):
        assert abs(np.exp(got["log_ovlp"][i] - ref["log_ovlp"][i]) - 1) < tol
        fb = ref["force_bias"][i]
        assert np.max(np.abs(got["force_bias"][i] - fb)) <= tol * np.max(np.abs(fb))
        assert abs(got["e_loc"][i] - ref["e_loc"][i]) <= tol * max(1.0, abs(ref["e_loc"][i]))
        ga, gb = msd.green(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w])
        np.testing.assert_allclose(got["green"][i][0], ga, atol=tol * max(1, np.abs(ga).max()))
        np.testing.assert_allclose(got["green"][i][1], gb, atol=tol * max(1, np.abs(gb).max()))


@pytest.mark.parametrize("na,nb,seed", [(6, 5, 1), (6, 6, 2), (4, 7, 3)])
def test_wick_matches_brute_force_high_orders(na, nb, seed):
    """Orders up to 6 per spin (up to 8 in total), unequal spins, complex CI
    coefficients, walkers far from the reference."""
    window = (min(na, nb), 14 - max(na, nb))
    wl = make_workload("w", M=14, n_alpha=na, n_beta=nb, n_chol=6, n_det=70, k_max=8,
                       window=window, c_law="flat", n_walkers=3, seed=seed, complex_ci=True,
                       noise=0.4, dt=0.01)
    assert max(wick.Excitations(wl.occ_a, wl.M).kmax, wick.Excitations(wl.occ_b, wl.M).kmax) >= 4
    _compare(wl, 0.7, [0, 2])


def test_wick_matches_brute_force_synthetic_recipe():
    """The synthetic recipe's walkers (0.1-perturbed reference) and power-law
    coefficients, a window inside a larger orbital space."""
    wl = make_workload("w", M=30, n_alpha=8, n_beta=8, n_chol=20, n_det=200, k_max=4,
                       window=(6, 10), c_law="power1", n_walkers=2, seed=9)
    _compare(wl, 0.0, [0, 1])


def test_wick_no_beta_electrons():
    wl = make_workload("w", M=10, n_alpha=4, n_beta=0, n_chol=5, n_det=12, k_max=3,
                       window=(4, 6), c_law="flat", n_walkers=1, seed=4, complex_ci=True,
                       noise=0.3)
    _compare(wl, 0.2, [0])


def test_per_determinant_two_body_is_single_det_energy():
    """For every determinant the C sums equal det X_a det X_b times that
    determinant's own two-body Wick energy 1/2 sum_g[(J_a + J_b)^2 - K_a - K_b]
    (J, K by brute force from Theta_I = Phi Phi[S, :]^{-1})."""
    wl = make_workload("w", M=13, n_alpha=6, n_beta=5, n_chol=5, n_det=45, k_max=7,
                       window=(6, 7), c_law="flat", n_walkers=1, seed=8, complex_ci=True,
                       noise=0.35)
    ex_a, ex_b = wick.Excitations(wl.occ_a, wl.M), wick.Excitations(wl.occ_b, wl.M)
    res = wick.walker_wick(wl.h1, wl.chol, 0.0, wl.ci, ex_a, ex_b, wl.phi_a[0], wl.phi_b[0],
                           wl.dt, per_det=True, chunk=16)
    ca = msd._SpinCache(wl.h1, wl.chol, wl.phi_a[0], 1e12)
    cb = msd._SpinCache(wl.h1, wl.chol, wl.phi_b[0], 1e12)
    da, db = res["det_x"]
    for i in range(wl.n_det):
        _, ja, ka = ca.get(wl.occ_a[i])
        _, jb, kb = cb.get(wl.occ_b[i])
        e2 = 0.5 * np.sum((ja + jb) ** 2 - ka - kb)
        ref = da[i] * db[i] * e2
        assert abs(res["two_body_det"][i] - ref) < 1e-10 * max(1.0, abs(ref)), i


# ----------------------------------------------------------------------------
# Fock space
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def fs5():
    return fock.FockSpace(5)


def _fock_measure(fs, h1, chol, e0, ci, oa, ob, pa, pb, dt):
    psi = fs.trial(ci, oa, ob)
    phi = fs.slater(pa, pb)
    o = np.vdot(psi, phi)
    H = fs.hamiltonian(h1, fock.eri_from_chol(chol), e0)
    M = h1.shape[0]
    g = []
    for spin in (0, 1):
        gm = np.zeros((M, M), complex)
        for p in range(M):
            for q in range(M):
                gm[p, q] = np.vdot(psi, fs.cdag(p, spin) @ fs.ann(q, spin) @ phi) / o
        g.append(gm)
    xb = np.array([-1j * math.sqrt(dt) * np.vdot(psi, fs.one_body(l) @ phi) / o for l in chol])
    return o, g, xb, np.vdot(psi, H @ phi) / o


def test_wick_fock_unequal_spins(fs5):
    rng = np.random.default_rng(31)
    M, na, nb = 5, 2, 3
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 4, M, 0.5)
    occs = set()
    oa, ob = [], []
    while len(oa) < 10:
        a = tuple(sorted(rng.choice(M, na, replace=False)))
        b = tuple(sorted(rng.choice(M, nb, replace=False)))
        if (a, b) not in occs:
            occs.add((a, b))
            oa.append(a)
            ob.append(b)
    oa, ob = np.array(oa, np.int32), np.array(ob, np.int32)
    ci = cplx(rng, 10)
    pa, pb = cplx(rng, M, na), cplx(rng, M, nb)
    o, g, xb, el = _fock_measure(fs5, h1, chol, 0.37, ci, oa, ob, pa, pb, 0.005)
    got = wick.measure(h1, chol, 0.37, ci, oa, ob, pa[None], pb[None], 0.005)
    assert abs(np.exp(got["log_ovlp"][0]) - o) < 1e-12 * abs(o)
    np.testing.assert_allclose(got["green"][0][0], g[0], atol=1e-11)
    np.testing.assert_allclose(got["green"][0][1], g[1], atol=1e-11)
    np.testing.assert_allclose(got["force_bias"][0], xb, atol=1e-12)
    assert abs(got["e_loc"][0] - el) < 1e-10 * max(1, abs(el))


def test_wick_walker_equal_to_reference_fock(fs5):
    """Phi = the reference orbitals: every excitation matrix is zero (singular),
    yet singles feed G and singles and doubles feed E_L."""
    rng = np.random.default_rng(33)
    M, na, nb = 5, 2, 2
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 3, M, 0.6)
    oa = np.array([[0, 1], [0, 2], [1, 3], [2, 3], [0, 1], [3, 4], [2, 4]], np.int32)
    ob = np.array([[0, 1], [0, 1], [0, 4], [1, 2], [2, 3], [2, 4], [3, 4]], np.int32)
    ci = cplx(rng, 7)
    pa = np.eye(M)[:, :na].astype(complex)
    pb = np.eye(M)[:, :nb].astype(complex)
    o, g, xb, el = _fock_measure(fs5, h1, chol, -0.2, ci, oa, ob, pa, pb, 0.01)
    got = wick.measure(h1, chol, -0.2, ci, oa, ob, pa[None], pb[None], 0.01)
    assert abs(np.exp(got["log_ovlp"][0]) - o) < 1e-12 * abs(o)
    np.testing.assert_allclose(got["green"][0][0], g[0], atol=1e-12)
    np.testing.assert_allclose(got["green"][0][1], g[1], atol=1e-12)
    np.testing.assert_allclose(got["force_bias"][0], xb, atol=1e-12)
    assert abs(got["e_loc"][0] - el) < 1e-11 * max(1, abs(el))


@pytest.mark.parametrize("na,nb", [(2, 2), (3, 2)])
def test_wick_fci_trial_zero_variance(fs5, na, nb):
    rng = np.random.default_rng(41 + na)
    M = 5
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 5, M, 0.4)
    H = fs5.hamiltonian(h1, fock.eri_from_chol(chol), 0.5)
    e_fci, vec = fs5.ground_state(H, na, nb)
    ci, oa, ob = fs5.expansion(vec, na, nb)
    # the expansion's first row is the Wick reference
    for _ in range(3):
        pa, pb = cplx(rng, M, na), cplx(rng, M, nb)
        got = wick.measure(h1, chol, 0.5, ci, oa, ob, pa[None], pb[None], 0.01)
        assert abs(got["e_loc"][0] - e_fci) < 1e-10


def test_single_determinant_trial():
    """N_d = 1: the textbook single-determinant energy of G = [Phi A^-1]^T."""
    rng = np.random.default_rng(51)
    M, na, nb = 9, 4, 3
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 6, M, 0.5)
    oa = np.array([[0, 2, 5, 7]], np.int32)
    ob = np.array([[1, 3, 4]], np.int32)
    pa, pb = cplx(rng, M, na), cplx(rng, M, nb)
    got = wick.measure(h1, chol, 0.1, np.array([0.6 - 0.8j]), oa, ob, pa[None], pb[None], 0.01)
    ga = np.zeros((M, M), complex)
    gb = np.zeros((M, M), complex)
    ga[oa[0], :] = (pa @ np.linalg.inv(pa[oa[0]])).T
    gb[ob[0], :] = (pb @ np.linalg.inv(pb[ob[0]])).T
    np.testing.assert_allclose(got["green"][0][0], ga, atol=1e-12)
    ref = msd.energy_sd_plain(h1, chol, 0.1, ga, gb)
    assert abs(got["e_loc"][0] - ref) < 1e-11 * max(1, abs(ref))


def test_duplicate_and_zero_coefficient_determinants():
    """A determinant split into two equal halves and a zero-coefficient copy of
    another leave every output unchanged."""
    wl = make_workload("w", M=12, n_alpha=5, n_beta=4, n_chol=5, n_det=30, k_max=5,
                       window=(5, 7), c_law="flat", n_walkers=1, seed=12, complex_ci=True,
                       noise=0.3)
    base = wick.measure(wl.h1, wl.chol, 0.0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a, wl.phi_b, wl.dt)
    ci = np.concatenate([wl.ci, [wl.ci[7] / 2, 0.0]])
    ci[7] = wl.ci[7] / 2
    oa = np.concatenate([wl.occ_a, wl.occ_a[7:8], wl.occ_a[3:4]])
    ob = np.concatenate([wl.occ_b, wl.occ_b[7:8], wl.occ_b[9:10]])
    got = wick.measure(wl.h1, wl.chol, 0.0, ci, oa, ob, wl.phi_a, wl.phi_b, wl.dt)
    assert abs(got["e_loc"][0] - base["e_loc"][0]) < 1e-12 * abs(base["e_loc"][0])
    np.testing.assert_allclose(got["force_bias"][0], base["force_bias"][0], atol=1e-13)
    np.testing.assert_allclose(got["green"][0][0], base["green"][0][0], atol=1e-13)

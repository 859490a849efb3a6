"""Pins of the CPU oracle against things other than itself.

Each check ties the oracle to an independent fact: explicit Fock-space
second quantisation (Jordan-Wigner, no Wick, no determinants), closed forms
(Hubbard dimer), invariances, brute force on tiny inputs, and the exact
eigenvalue of an FCI trial (zero variance).  A dropped term, wrong sign,
transposed G or missing conjugate in the oracle fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import driver, fock, msd, propagate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------
# tiny random systems
# ----------------------------------------------------------------------------

def rand_sym(rng, n, M, scale=1.0):
    a = rng.standard_normal((n, M, M))
    return scale * (a + a.transpose(0, 2, 1)) / 2


def rand_walker(rng, M, N):
    return rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))


def rand_trial(rng, M, na, nb, nd, complex_ci=True):
    occs = set()
    oa, ob = [], []
    while len(oa) < nd:
        a = tuple(sorted(rng.choice(M, na, replace=False)))
        b = tuple(sorted(rng.choice(M, nb, replace=False)))
        if (a, b) in occs:
            continue
        occs.add((a, b))
        oa.append(a)
        ob.append(b)
    ci = rng.standard_normal(nd) + (1j * rng.standard_normal(nd) if complex_ci else 0)
    return ci.astype(np.complex128), np.array(oa, np.int32), np.array(ob, np.int32)


@pytest.fixture(scope="module")
def fs5():
    return fock.FockSpace(5)


@pytest.fixture(scope="module")
def sys5(fs5):
    rng = np.random.default_rng(11)
    M, na, nb = 5, 2, 3
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 4, M, 0.5)
    e0 = 0.37
    ci, oa, ob = rand_trial(rng, M, na, nb, 9)
    phi_a, phi_b = rand_walker(rng, M, na), rand_walker(rng, M, nb)
    H = fs5.hamiltonian(h1, fock.eri_from_chol(chol), e0)
    return dict(M=M, na=na, nb=nb, h1=h1, chol=chol, e0=e0, ci=ci, oa=oa, ob=ob,
                phi_a=phi_a, phi_b=phi_b, H=H)


# ----------------------------------------------------------------------------
# linear-algebra helpers
# ----------------------------------------------------------------------------

def cofactor_adjugate(a):
    n = a.shape[0]
    adj = np.zeros_like(a)
    for i in range(n):
        for j in range(n):
            minor = np.delete(np.delete(a, i, 0), j, 1)
            adj[j, i] = (-1) ** (i + j) * (np.linalg.det(minor) if n > 1 else 1.0)
    return adj


def leibniz_det(a):
    n = a.shape[0]
    tot = 0.0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        tot += (-1) ** inv * np.prod([a[perm[j], j] for j in range(n)])
    return tot


@pytest.mark.parametrize("rank", [4, 3, 1, 0])
def test_adjugate_matches_cofactors(rank):
    rng = np.random.default_rng(rank)
    a = rng.standard_normal((4, rank)) + 1j * rng.standard_normal((4, rank))
    b = rng.standard_normal((rank, 4)) + 1j * rng.standard_normal((rank, 4))
    m = a @ b if rank else np.zeros((4, 4), complex)
    np.testing.assert_allclose(msd.adjugate(m), cofactor_adjugate(m), atol=1e-12)


def test_spin_overlaps_leibniz():
    rng = np.random.default_rng(3)
    phi = rand_walker(rng, 6, 4)
    occ = np.array([[0, 1, 2, 3], [0, 2, 4, 5], [1, 3, 4, 5]])
    got = msd.spin_overlaps(phi, occ)
    ref = [leibniz_det(phi[o]) for o in occ]
    np.testing.assert_allclose(got, ref, rtol=1e-12)


# ----------------------------------------------------------------------------
# overlaps, Green's functions, force bias vs Fock space
# ----------------------------------------------------------------------------

def test_trial_overlap_fock(fs5, sys5):
    s = sys5
    psi = fs5.trial(s["ci"], s["oa"], s["ob"])
    phi = fs5.slater(s["phi_a"], s["phi_b"])
    ref = np.vdot(psi, phi)
    got = msd.trial_overlap(s["ci"], s["oa"], s["ob"], s["phi_a"], s["phi_b"])
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_green_fock(fs5, sys5):
    s = sys5
    psi = fs5.trial(s["ci"], s["oa"], s["ob"])
    phi = fs5.slater(s["phi_a"], s["phi_b"])
    o = np.vdot(psi, phi)
    ga, gb = msd.green(s["ci"], s["oa"], s["ob"], s["phi_a"], s["phi_b"])
    for spin, g in ((0, ga), (1, gb)):
        ref = np.zeros((s["M"], s["M"]), complex)
        for p in range(s["M"]):
            for q in range(s["M"]):
                op = fs5.cdag(p, spin) @ fs5.ann(q, spin)
                ref[p, q] = np.vdot(psi, op @ phi) / o
        np.testing.assert_allclose(g, ref, atol=1e-11)


def test_green_singular_blocks_fock(fs5):
    """Walker equal to the reference orbitals: every excited det has zero
    overlap, yet contributes to G (adjugate path)."""
    rng = np.random.default_rng(5)
    M, na, nb = 5, 2, 2
    phi_a = np.eye(M)[:, :na].astype(complex)
    phi_b = np.eye(M)[:, :nb].astype(complex)
    oa = np.array([[0, 1], [0, 2], [1, 3], [0, 1], [2, 4]], np.int32)
    ob = np.array([[0, 1], [0, 1], [0, 1], [1, 4], [0, 3]], np.int32)
    ci = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    psi = fs5.trial(ci, oa, ob)
    phi = fs5.slater(phi_a, phi_b)
    o = np.vdot(psi, phi)
    ga, gb = msd.green(ci, oa, ob, phi_a, phi_b)
    for spin, g in ((0, ga), (1, gb)):
        for p in range(M):
            for q in range(M):
                ref = np.vdot(psi, fs5.cdag(p, spin) @ fs5.ann(q, spin) @ phi) / o
                assert abs(g[p, q] - ref) < 1e-12


def test_green_invariants():
    rng = np.random.default_rng(7)
    M, na, nb = 9, 3, 4
    ci, oa, ob = rand_trial(rng, M, na, nb, 12)
    phi_a, phi_b = rand_walker(rng, M, na), rand_walker(rng, M, nb)
    ga, gb = msd.green(ci, oa, ob, phi_a, phi_b)
    # particle number
    assert abs(np.trace(ga) - na) < 1e-11 and abs(np.trace(gb) - nb) < 1e-11
    # gauge invariance Phi -> Phi U
    ua = rand_walker(rng, na, na)
    ub = rand_walker(rng, nb, nb)
    ga2, gb2 = msd.green(ci, oa, ob, phi_a @ ua, phi_b @ ub)
    np.testing.assert_allclose(ga2, ga, atol=1e-10)
    np.testing.assert_allclose(gb2, gb, atol=1e-10)
    # duplicated determinant with split coefficient, plus a zero-c det
    ci3 = np.concatenate([ci, [ci[4] / 2, 0.0]])
    ci3[4] = ci[4] / 2
    oa3 = np.concatenate([oa, oa[4:5], oa[0:1]])
    ob3 = np.concatenate([ob, ob[4:5], ob[1:2]])
    ga3, gb3 = msd.green(ci3, oa3, ob3, phi_a, phi_b)
    np.testing.assert_allclose(ga3, ga, atol=1e-11)
    np.testing.assert_allclose(gb3, gb, atol=1e-11)


def test_green_single_det_textbook():
    """N_d = 1: G^T = Phi (Psi^H Phi)^{-1} Psi^H for an arbitrary (non-unit)
    trial matrix Psi, by rotating the orbital basis; idempotent."""
    rng = np.random.default_rng(9)
    M, N = 7, 3
    phi = rand_walker(rng, M, N)
    occ = np.array([[1, 4, 5]], np.int32)
    ga, _ = msd.green(np.ones(1, complex), occ, np.zeros((1, 0), np.int32),
                      phi, np.zeros((M, 0), complex))
    psi = np.eye(M)[:, occ[0]]
    textbook = (phi @ np.linalg.inv(psi.conj().T @ phi) @ psi.conj().T).T
    np.testing.assert_allclose(ga, textbook, atol=1e-12)
    np.testing.assert_allclose(ga @ ga, ga, atol=1e-11)


def test_force_bias_identity_cholesky():
    rng = np.random.default_rng(13)
    M, na, nb = 6, 2, 3
    ci, oa, ob = rand_trial(rng, M, na, nb, 7)
    phi_a, phi_b = rand_walker(rng, M, na), rand_walker(rng, M, nb)
    chol = np.stack([np.eye(M)] * 3)
    ga, gb = msd.green(ci, oa, ob, phi_a, phi_b)
    dt = 0.01
    xb = msd.force_bias(chol, ga, gb, dt)
    np.testing.assert_allclose(xb, -1j * math.sqrt(dt) * (na + nb), atol=1e-11)


def test_force_bias_fock(fs5, sys5):
    s = sys5
    psi = fs5.trial(s["ci"], s["oa"], s["ob"])
    phi = fs5.slater(s["phi_a"], s["phi_b"])
    o = np.vdot(psi, phi)
    ga, gb = msd.green(s["ci"], s["oa"], s["ob"], s["phi_a"], s["phi_b"])
    dt = 0.005
    xb = msd.force_bias(s["chol"], ga, gb, dt)
    for g in range(s["chol"].shape[0]):
        lop = fs5.one_body(s["chol"][g])
        ref = -1j * math.sqrt(dt) * np.vdot(psi, lop @ phi) / o
        assert abs(xb[g] - ref) < 1e-11


# ----------------------------------------------------------------------------
# local energy
# ----------------------------------------------------------------------------

def test_local_energy_fock(fs5, sys5):
    s = sys5
    psi = fs5.trial(s["ci"], s["oa"], s["ob"])
    phi = fs5.slater(s["phi_a"], s["phi_b"])
    ref = np.vdot(psi, s["H"] @ phi) / np.vdot(psi, phi)
    got = msd.local_energy(s["h1"], s["chol"], s["e0"], s["ci"], s["oa"], s["ob"],
                           s["phi_a"], s["phi_b"])
    assert abs(got - ref) < 1e-10 * max(1.0, abs(ref))


@pytest.mark.parametrize("na,nb", [(2, 2), (2, 3)])
def test_fci_trial_zero_variance(fs5, na, nb):
    rng = np.random.default_rng(17 + na + nb)
    M = 5
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 5, M, 0.4)
    e0 = -1.25
    H = fs5.hamiltonian(h1, fock.eri_from_chol(chol), e0)
    e_fci, vec = fs5.ground_state(H, na, nb)
    ci, oa, ob = fs5.expansion(vec, na, nb)
    for _ in range(3):
        pa, pb = rand_walker(rng, M, na), rand_walker(rng, M, nb)
        el = msd.local_energy(h1, chol, e0, ci, oa, ob, pa, pb)
        assert abs(el - e_fci) < 1e-10


def test_hubbard_dimer_closed_form():
    with open(os.path.join(GOLDEN, "hubbard_dimer.json")) as f:
        gold = json.load(f)
    fs2 = fock.FockSpace(2)
    for case in gold["cases"]:
        t, U = case["t"], case["U"]
        h1 = np.array([[0.0, -t], [-t, 0.0]])
        chol = np.zeros((2, 2, 2))
        chol[0, 0, 0] = math.sqrt(U)
        chol[1, 1, 1] = math.sqrt(U)
        H = fs2.hamiltonian(h1, fock.eri_from_chol(chol), 0.0)
        e_fci, vec = fs2.ground_state(H, 1, 1)
        assert abs(e_fci - case["E0"]) < 1e-12
        ci, oa, ob = fs2.expansion(vec, 1, 1)
        rng = np.random.default_rng(1)
        el = msd.local_energy(h1, chol, 0.0, ci, oa, ob,
                              rand_walker(rng, 2, 1), rand_walker(rng, 2, 1))
        assert abs(el - case["E0"]) < 1e-12


def test_energy_cholesky_vs_eri_and_single_det():
    rng = np.random.default_rng(19)
    M, na, nb = 6, 3, 2
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 7, M, 0.5)
    eri = fock.eri_from_chol(chol)
    phi_a, phi_b = rand_walker(rng, M, na), rand_walker(rng, M, nb)
    oa = np.array([[0, 2, 5]], np.int32)
    ob = np.array([[1, 4]], np.int32)
    ga, gb = msd.green(np.ones(1, complex), oa, ob, phi_a, phi_b)
    e_plain = msd.energy_sd_plain(h1, chol, 0.3, ga, gb)
    e_eri = msd.energy_sd_eri(h1, eri, 0.3, ga, gb)
    assert abs(e_plain - e_eri) < 1e-11
    e_loc = msd.local_energy(h1, chol, 0.3, np.ones(1, complex), oa, ob, phi_a, phi_b)
    assert abs(e_loc - e_plain) < 1e-11


def test_energy_without_two_body():
    rng = np.random.default_rng(23)
    M, na, nb = 7, 2, 3
    h1 = rand_sym(rng, 1, M)[0]
    chol = np.zeros((3, M, M))
    ci, oa, ob = rand_trial(rng, M, na, nb, 10)
    phi_a, phi_b = rand_walker(rng, M, na), rand_walker(rng, M, nb)
    ga, gb = msd.green(ci, oa, ob, phi_a, phi_b)
    el = msd.local_energy(h1, chol, 0.5, ci, oa, ob, phi_a, phi_b)
    assert abs(el - (0.5 + np.sum(h1 * (ga + gb)))) < 1e-11


# ----------------------------------------------------------------------------
# propagation
# ----------------------------------------------------------------------------

def test_hprime_splits_hamiltonian():
    """H of Eq. 2 equals sum h' E + 1/2 sum_g Lhat_g^2 + E0 (Eq. 3-4)."""
    fs = fock.FockSpace(3)
    rng = np.random.default_rng(29)
    M = 3
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 3, M, 0.6)
    H = fs.hamiltonian(h1, fock.eri_from_chol(chol), 0.2)
    alt = 0.2 * np.eye(fs.dim) + fs.one_body(propagate.h_prime(h1, chol)).toarray()
    for g in range(3):
        lop = fs.one_body(chol[g]).toarray()
        alt = alt + 0.5 * lop @ lop
    np.testing.assert_allclose(H.toarray(), alt, atol=1e-12)


def test_hs_transform_sign():
    """int dx p(x) exp(i sqrt(dt) x Lhat) = exp(-dt/2 Lhat^2): checked with
    Gauss-Hermite quadrature in Fock space (pins the factor i in VHS)."""
    fs = fock.FockSpace(2)
    rng = np.random.default_rng(31)
    lmat = rand_sym(rng, 1, 2)[0]
    lop = fs.one_body(lmat).toarray()
    dt = 0.3
    xs, ws = np.polynomial.hermite_e.hermegauss(40)
    ws = ws / math.sqrt(2 * math.pi)
    lhs = sum(w * scipy.linalg.expm(1j * math.sqrt(dt) * x * lop) for x, w in zip(xs, ws))
    rhs = scipy.linalg.expm(-0.5 * dt * lop @ lop)
    np.testing.assert_allclose(lhs, rhs, atol=1e-10)


def test_thouless_orbital_update():
    """exp(sum_pq V_pq E_pq)|Phi> is the determinant of expm(V) Phi."""
    fs = fock.FockSpace(3)
    rng = np.random.default_rng(37)
    v = (rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))) * 0.4
    phi_a, phi_b = rand_walker(rng, 3, 2), rand_walker(rng, 3, 1)
    lhs = scipy.linalg.expm(fs.one_body(v).toarray()) @ fs.slater(phi_a, phi_b)
    ev = scipy.linalg.expm(v)
    rhs = fs.slater(ev @ phi_a, ev @ phi_b)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)


def test_taylor_truncation_bound():
    rng = np.random.default_rng(41)
    M, N = 10, 4
    chol = rand_sym(rng, 6, M, 1.0 / math.sqrt(M))
    y = rng.standard_normal(6) + 0.3j * rng.standard_normal(6)
    v = propagate.vhs(chol, y, 0.005)
    phi = rand_walker(rng, M, N)
    nv = np.linalg.norm(v, 2)
    exact = scipy.linalg.expm(v) @ phi
    for n in (2, 4, 6):
        approx = propagate.taylor_apply(v, phi, n)
        bound = nv ** (n + 1) / math.factorial(n + 1) * math.exp(nv) * np.linalg.norm(phi, 2)
        assert np.linalg.norm(approx - exact, 2) <= bound * (1 + 1e-8) + 1e-14


def test_zero_shifted_field_gives_one_body_only():
    rng = np.random.default_rng(43)
    M = 8
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 5, M, 0.3)
    dt = 0.01
    b1 = propagate.one_body_half_step(h1, chol, dt)
    v = propagate.vhs(chol, np.zeros(5), dt)
    phi = rand_walker(rng, M, 3)
    out = propagate.propagate_orbitals(phi, b1, v, 6)
    hp = h1.copy()
    for g in range(5):
        hp -= 0.5 * chol[g] @ chol[g]
    np.testing.assert_allclose(out, scipy.linalg.expm(-dt * hp) @ phi, atol=1e-12)


def test_weight_update_hand_values():
    # S = 2 exp(i pi/3), x = (1, 0), xbar = (0.5, 0): |I| = 2 e^{0.5 - 0.125},
    # cos(theta) = 1/2  ->  w' = w e^{0.375}.
    w = propagate.importance_weight(1.5, 0.0, math.log(2) + 1j * math.pi / 3,
                                    np.array([1.0, 0.0]), np.array([0.5, 0.0]))
    assert abs(w - 1.5 * math.exp(0.375)) < 1e-14
    # phase beyond pi/2 kills the walker
    assert propagate.importance_weight(1.0, 0.0, 2.0j, np.zeros(1), np.zeros(1)) == 0.0
    # complex xbar enters bilinearly: x = 0, xbar = i -> exp(+1/2)
    w = propagate.importance_weight(1.0, 0.0, 0.0, np.zeros(1), np.array([1j]))
    assert abs(w - math.exp(0.5)) < 1e-14


def test_force_bias_cancels_linear_field_response(fs5, sys5):
    """With xbar = -i sqrt(dt) <L>, I(x) has no O(sqrt(dt)) term in x: the
    antisymmetric part of I(x) in x is O(dt), not O(sqrt(dt))."""
    s = sys5
    dt = 1e-6
    ga, gb = msd.green(s["ci"], s["oa"], s["ob"], s["phi_a"], s["phi_b"])
    xbar = msd.force_bias(s["chol"], ga, gb, dt)
    b1 = np.eye(s["M"])
    lo = np.log(msd.trial_overlap(s["ci"], s["oa"], s["ob"], s["phi_a"], s["phi_b"]))

    def imp(x, xb):
        v = propagate.vhs(s["chol"], x - xb, dt)
        na = propagate.propagate_orbitals(s["phi_a"], b1, v, 6)
        nb = propagate.propagate_orbitals(s["phi_b"], b1, v, 6)
        ln = np.log(msd.trial_overlap(s["ci"], s["oa"], s["ob"], na, nb))
        return np.exp(ln - lo) * np.exp(np.dot(x, xb) - 0.5 * np.dot(xb, xb))

    e = np.zeros(s["chol"].shape[0])
    e[0] = 1.0
    with_fb = abs(imp(e, xbar) - imp(-e, xbar))
    without = abs(imp(e, 0 * xbar) - imp(-e, 0 * xbar))
    assert without > 10 * math.sqrt(dt) * 0.01
    assert with_fb < 50 * dt


def test_qr_positive():
    rng = np.random.default_rng(47)
    phi = rand_walker(rng, 12, 5)
    q, r = propagate.qr_positive(phi)
    np.testing.assert_allclose(q.conj().T @ q, np.eye(5), atol=1e-13)
    np.testing.assert_allclose(q @ r, phi, atol=1e-12)
    assert np.allclose(np.tril(r, -1), 0)
    d = np.diag(r)
    assert np.all(np.abs(d.imag) < 1e-14) and np.all(d.real > 0)


def test_step_overlap_bookkeeping():
    """After a step with QR, log_ovlp equals log <Psi_T|Phi_new> directly."""
    rng = np.random.default_rng(53)
    M, na, nb = 8, 2, 3
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, 6, M, 0.3)
    ci, oa, ob = rand_trial(rng, M, na, nb, 6)
    pa = np.stack([rand_walker(rng, M, na) for _ in range(3)])
    pb = np.stack([rand_walker(rng, M, nb) for _ in range(3)])
    lo = np.array([np.log(msd.trial_overlap(ci, oa, ob, pa[w], pb[w])) for w in range(3)])
    wts = np.array([1.0, 0.0, 2.0])
    x = rng.standard_normal((3, 6))
    na_, nb_, w2, lo2, _ = propagate.step(h1, chol, ci, oa, ob, pa, pb, wts, lo, x,
                                           0.01, do_qr=True)
    for w in range(3):
        direct = np.log(msd.trial_overlap(ci, oa, ob, na_[w], nb_[w]))
        assert abs(np.exp(direct - lo2[w]) - 1) < 1e-11
    # frozen walker unchanged
    np.testing.assert_array_equal(na_[1], pa[1])
    assert w2[1] == 0.0


# ----------------------------------------------------------------------------
# block driver: comb population control (Sec. III.B, Listing 1; the comb is
# the reading taken where the paper names no algorithm)
# ----------------------------------------------------------------------------

def _comb_brute(w, z):
    """Tooth k at (k + z) W / n goes to the first walker whose running sum
    passes it, found by walking the list (no library search)."""
    n, total = len(w), sum(w)
    out = []
    for k in range(n):
        t = (k + z) * total / n
        run, pick = 0.0, None
        for i, wi in enumerate(w):
            if run <= t < run + wi:
                pick = i
                break
            run += wi
        out.append(pick)
    return out


def test_comb_equal_weights_is_identity():
    for n in (1, 2, 7, 64):
        for z in (0.0, 0.25, 0.999):
            parent, wn = driver.comb(np.full(n, 1.5), z)
            np.testing.assert_array_equal(parent, np.arange(n))
            assert wn == 1.5


def test_comb_copy_counts_and_total_weight():
    rng = np.random.default_rng(71)
    for n in (3, 10, 57):
        w = rng.exponential(size=n)
        w[rng.random(n) < 0.2] = 0.0
        w[0] = 0.7  # at least one live walker
        for z in rng.random(5):
            parent, wn = driver.comb(w, z)
            cnt = np.bincount(parent, minlength=n)
            exp = n * w / w.sum()
            assert cnt.sum() == n
            assert np.all(cnt >= np.floor(exp) - 1e-9) and np.all(cnt <= np.ceil(exp) + 1e-9)
            assert np.all(cnt[w == 0.0] == 0)
            assert np.all(np.diff(parent) >= 0)
            assert abs(wn * n - w.sum()) < 1e-12 * w.sum()


def test_comb_unbiased_over_offsets():
    """Averaged over a midpoint grid of J offsets, walker i is copied
    n w_i / W times to within 1/J (exactly, for uniform z)."""
    w = np.array([0.3, 0.0, 2.2, 0.9, 0.05, 1.1, 0.0, 0.45])
    n, J = len(w), 2048
    mean = np.zeros(n)
    for j in range(J):
        parent, _ = driver.comb(w, (j + 0.5) / J)
        mean += np.bincount(parent, minlength=n)
    mean /= J
    np.testing.assert_allclose(mean, n * w / w.sum(), atol=1.0 / J)


def test_comb_brute_force_small():
    rng = np.random.default_rng(72)
    for _ in range(200):
        n = int(rng.integers(1, 9))
        # dyadic weights: every running sum is exact, so ties are real ties
        w = rng.integers(0, 5, size=n) / 4.0
        if w.sum() == 0:
            w[-1] = 0.25
        z = rng.integers(0, 8) / 8.0
        parent, _ = driver.comb(w, z)
        assert list(parent) == _comb_brute(list(w), z)


def test_comb_zero_weight_not_copied_at_ties():
    # teeth at 0 and W/2 land exactly on the empty interval of walker 0
    parent, wn = driver.comb(np.array([0.0, 1.0]), 0.0)
    assert list(parent) == [1, 1] and wn == 0.5
    parent, _ = driver.comb(np.array([1.0, 0.0, 1.0, 0.0]), 0.0)
    assert list(parent) == [0, 0, 2, 2]


def test_comb_all_frozen_changes_nothing():
    parent, wn = driver.comb(np.zeros(4), 0.3)
    assert wn is None and list(parent) == [0, 1, 2, 3]


def test_block_without_population_control_is_steps_plus_measure():
    rng = np.random.default_rng(73)
    M, na, nb, ng, nw = 6, 2, 2, 4, 3
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, ng, M, 0.3)
    ci, oa, ob = rand_trial(rng, M, na, nb, 5)
    pa = np.stack([rand_walker(rng, M, na) for _ in range(nw)])
    pb = np.stack([rand_walker(rng, M, nb) for _ in range(nw)])
    lo = np.array([np.log(msd.trial_overlap(ci, oa, ob, pa[w], pb[w])) for w in range(nw)])
    wts = np.array([1.0, 0.5, 2.0])
    x = rng.standard_normal((3, nw, ng))
    out = driver.block(h1, chol, 0.4, ci, oa, ob, pa, pb, wts, lo, x, 0.01, [],
                       stabilize_freq=2, pop_freq=0, steps_before=1)
    ra, rb, rw, rl = pa, pb, wts, lo
    for s in range(3):
        ra, rb, rw, rl, _ = propagate.step(h1, chol, ci, oa, ob, ra, rb, rw, rl, x[s], 0.01,
                                           do_qr=(s + 2) % 2 == 0)
    np.testing.assert_array_equal(out[0], ra)
    np.testing.assert_array_equal(out[2], rw)
    el = msd.measure(h1, chol, 0.4, ci, oa, ob, ra, rb, 0.01)["e_loc"]
    np.testing.assert_array_equal(out[4], el)
    assert abs(out[5] - np.sum(rw * el)) == 0 and out[6] == np.sum(rw)


def test_block_population_control_copies_whole_walkers():
    """After a combed block every walker is a copy of one propagated walker
    (orbitals, overlap together) and the weights are equal."""
    rng = np.random.default_rng(74)
    M, na, nb, ng, nw = 6, 2, 2, 4, 5
    h1 = rand_sym(rng, 1, M)[0]
    chol = rand_sym(rng, ng, M, 0.3)
    ci, oa, ob = rand_trial(rng, M, na, nb, 5)
    pa = np.stack([rand_walker(rng, M, na) for _ in range(nw)])
    pb = np.stack([rand_walker(rng, M, nb) for _ in range(nw)])
    lo = np.array([np.log(msd.trial_overlap(ci, oa, ob, pa[w], pb[w])) for w in range(nw)])
    wts = np.array([1.0, 0.2, 3.0, 0.0, 0.8])
    x = rng.standard_normal((2, nw, ng))
    out = driver.block(h1, chol, 0.0, ci, oa, ob, pa, pb, wts, lo, x, 0.01, [0.37],
                       stabilize_freq=0, pop_freq=2)
    ra, rb, rw, rl = pa, pb, wts, lo
    for s in range(2):
        ra, rb, rw, rl, _ = propagate.step(h1, chol, ci, oa, ob, ra, rb, rw, rl, x[s], 0.01)
    parent, wn = driver.comb(rw, 0.37)
    assert 3 not in parent  # the frozen walker is dropped
    np.testing.assert_array_equal(out[0], ra[parent])
    np.testing.assert_array_equal(out[1], rb[parent])
    np.testing.assert_array_equal(out[3], rl[parent])
    np.testing.assert_allclose(out[2], np.full(nw, rw.sum() / nw), rtol=0, atol=0)
    for w in range(nw):
        assert abs(np.exp(np.log(msd.trial_overlap(ci, oa, ob, out[0][w], out[1][w]))
                          - out[3][w]) - 1) < 1e-11

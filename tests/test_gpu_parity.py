"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

FP64 bar: 1e-10 relative (log-overlaps compared through exp(difference), force
biases relative to their largest element, energies relative to max(1, |E|)).
"""
import math

import numpy as np
import pytest

from oracle import fock, msd, propagate
from paper_2406_08314_amd import MsdError, MsdSystem
from synth import fields_for_step, make_config, make_workload

pytestmark = pytest.mark.gpu

TOL = 1e-10


def system_for(wl, **kw):
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det, **kw)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
    return s


def assert_logo(gpu, ref, tol=TOL):
    z = np.exp(np.asarray(gpu) - np.asarray(ref))
    assert np.max(np.abs(z - 1)) <= tol, np.max(np.abs(z - 1))


def assert_rel(gpu, ref, tol=TOL, floor=1.0):
    gpu, ref = np.asarray(gpu), np.asarray(ref)
    scale = max(floor, float(np.max(np.abs(ref))))
    err = float(np.max(np.abs(gpu - ref)))
    assert err <= tol * scale, (err, scale)


def oracle_walker(wl, w, dt, energy=True):
    r = msd.measure(wl.h1, wl.chol, wl.e0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a, wl.phi_b, dt,
                    walkers=[w], energy=energy)
    return {k: v[0] for k, v in r.items()}


def compare_walkers(wl, out, walkers, dt, energy=True, sys_=None):
    for w in walkers:
        ref = oracle_walker(wl, w, dt, energy)
        assert_logo(out["log_ovlp"][w], ref["log_ovlp"])
        assert_rel(out["force_bias"][w], ref["force_bias"], floor=0.0)
        if energy:
            assert_rel(out["e_loc"][w], ref["e_loc"])
        if sys_ is not None:
            ga, gb = sys_.get_green(w)
            ra, rb = msd.green(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w])
            assert_rel(ga, ra)
            assert_rel(gb, rb)


# ----------------------------------------------------------------------------
# measurement
# ----------------------------------------------------------------------------

def test_tiny_measure_all_walkers():
    wl = make_config("tiny")
    s = system_for(wl)
    out = s.measure(wl.dt)
    compare_walkers(wl, out, range(wl.n_walkers), wl.dt, sys_=s)
    # set_walkers stored the same log-overlaps
    _, _, w, lo = s.get_walkers()
    assert_logo(lo, out["log_ovlp"], 1e-13)
    np.testing.assert_array_equal(w, wl.weights)


def test_tiny_measure_is_reproducible():
    wl = make_config("tiny")
    s = system_for(wl)
    a = s.measure(wl.dt)
    b = s.measure(wl.dt)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("algo", [0, 3])
def test_medium_full_batch_sampled_walkers(algo):
    wl = make_config("medium")
    s = system_for(wl, energy_algo=algo)
    out = s.measure(wl.dt)
    lo_ref = np.array([np.log(msd.trial_overlap(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[w], wl.phi_b[w]))
                       for w in range(wl.n_walkers)])
    assert_logo(out["log_ovlp"], lo_ref)
    compare_walkers(wl, out, [0, 77, 127], wl.dt, sys_=s)


def test_medium_flat_coefficients():
    wl = make_config("medium", c_law="flat", n_walkers=16, n_det=400)
    s = system_for(wl)
    out = s.measure(wl.dt)
    compare_walkers(wl, out, [3, 15], wl.dt)


@pytest.mark.parametrize("na,nb,kmax,window,nd", [(6, 5, 10, (6, 8), 60), (4, 2, 6, (4, 6), 60),
                                                 (3, 0, 3, (3, 5), 40)])
def test_high_order_unequal_spins_complex_ci(na, nb, kmax, window, nd):
    wl = make_workload("edge", M=16, n_alpha=na, n_beta=nb, n_chol=20, n_det=nd, k_max=kmax,
                       window=window, c_law="flat", n_walkers=5, seed=77 + na, complex_ci=True,
                       noise=0.5)
    s = system_for(wl)
    out = s.measure(0.01)
    compare_walkers(wl, out, range(5), 0.01, sys_=s)


def _pair_entries(wl):
    """(entries, distinct pairs) of the opposite-spin pair table: a determinant
    with alpha order ka and beta order kb contributes ka^2 kb^2 entries, one per
    (alpha (particle, hole), beta (particle, hole)) combination."""
    ra, rb = set(wl.occ_a[0].tolist()), set(wl.occ_b[0].tolist())
    pairs, ent = set(), 0
    for a, b in zip(wl.occ_a, wl.occ_b):
        sa, sb = set(a.tolist()), set(b.tolist())
        xs = [(p, h) for p in sorted(sa - ra) for h in sorted(ra - sa)]
        ys = [(p, h) for p in sorted(sb - rb) for h in sorted(rb - sb)]
        ent += len(xs) * len(ys)
        pairs |= {(x, y) for x in xs for y in ys}
    return ent, len(pairs)


def test_pair_coefficients_walkers_on_lanes():
    """Pairs with many entries each (31 on average, 576 pairs) take the
    pair-coefficient form with the walkers on the lanes; 70 walkers leave the
    second block of 64 partly filled.  Walkers of both blocks against the
    brute-force oracle."""
    wl = make_workload("pairs", M=24, n_alpha=6, n_beta=6, n_chol=32, n_det=3000, k_max=4,
                       window=(4, 6), c_law="power1", n_walkers=70, seed=4242,
                       complex_ci=True, noise=0.3)
    ent, n_pair = _pair_entries(wl)
    assert ent >= 16 * n_pair  # the library's threshold for this form
    s = system_for(wl)
    out = s.measure(wl.dt)
    compare_walkers(wl, out, [0, 63, 64, 69], wl.dt)


def test_single_determinant():
    wl = make_config("tiny", n_det=1)
    s = system_for(wl)
    out = s.measure(wl.dt)
    compare_walkers(wl, out, range(wl.n_walkers), wl.dt, sys_=s)


def test_duplicate_rows_and_zero_coefficients():
    wl = make_config("tiny", complex_ci=True)
    base = system_for(wl).measure(wl.dt)
    ci = np.concatenate([wl.ci, [0.0, wl.ci[5] / 2]])
    ci[5] = wl.ci[5] / 2
    oa = np.concatenate([wl.occ_a, wl.occ_a[7:8], wl.occ_a[5:6]])
    ob = np.concatenate([wl.occ_b, wl.occ_b[2:3], wl.occ_b[5:6]])
    s = MsdSystem(wl.M, 3, 3, wl.n_chol, wl.n_walkers, len(ci))
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(ci, oa, ob)
    s.set_walkers(wl.phi_a, wl.phi_b)
    out = s.measure(wl.dt)
    assert_logo(out["log_ovlp"], base["log_ovlp"], 1e-12)
    assert_rel(out["force_bias"], base["force_bias"], 1e-12, floor=0.0)
    assert_rel(out["e_loc"], base["e_loc"], 1e-12)


def test_walker_equal_to_reference_fock():
    """Every excitation block X is exactly zero (or singular); the adjugate and
    minor forms must still give the exact G and E_L (Fock-space oracle)."""
    rng = np.random.default_rng(101)
    M, na, nb = 5, 2, 2
    h1 = rng.standard_normal((M, M))
    h1 = (h1 + h1.T) / 2
    chol = rng.standard_normal((4, M, M)) * 0.4
    chol = (chol + chol.transpose(0, 2, 1)) / 2
    oa = np.array([[0, 1], [0, 2], [1, 3], [2, 4], [0, 1], [3, 4]], np.int32)
    ob = np.array([[0, 1], [0, 1], [0, 4], [2, 3], [1, 2], [0, 3]], np.int32)
    ci = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    u = np.linalg.qr(rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))[0]
    pa = np.stack([np.eye(M)[:, :na] @ u, np.eye(M)[:, :na]]).astype(complex)
    pb = np.stack([np.eye(M)[:, :nb], np.eye(M)[:, :nb] @ u]).astype(complex)
    s = MsdSystem(M, na, nb, 4, 2, 6)
    s.set_hamiltonian(h1, chol, 0.1)
    s.set_trial(ci, oa, ob)
    s.set_walkers(pa, pb)
    out = s.measure(0.01)
    fs = fock.FockSpace(M)
    H = fs.hamiltonian(h1, fock.eri_from_chol(chol), 0.1)
    psi = fs.trial(ci, oa, ob)
    for w in range(2):
        phi = fs.slater(pa[w], pb[w])
        o = np.vdot(psi, phi)
        assert_logo(out["log_ovlp"][w], np.log(o), 1e-12)
        e_ref = np.vdot(psi, H @ phi) / o
        assert_rel(out["e_loc"][w], e_ref, 1e-11)
        ga, gb = s.get_green(w)
        for spin, g in ((0, ga), (1, gb)):
            for p in range(M):
                for q in range(M):
                    ref = np.vdot(psi, fs.cdag(p, spin) @ fs.ann(q, spin) @ phi) / o
                    assert abs(g[p, q] - ref) < 1e-11


def test_fci_trial_zero_variance_on_gpu():
    rng = np.random.default_rng(5)
    M, na, nb = 5, 2, 2
    h1 = rng.standard_normal((M, M))
    h1 = (h1 + h1.T) / 2
    chol = rng.standard_normal((5, M, M)) * 0.4
    chol = (chol + chol.transpose(0, 2, 1)) / 2
    fs = fock.FockSpace(M)
    H = fs.hamiltonian(h1, fock.eri_from_chol(chol), -0.7)
    e_fci, vec = fs.ground_state(H, na, nb)
    ci, oa, ob = fs.expansion(vec, na, nb)
    # put the largest coefficient first (the Wick reference)
    order = np.argsort(-np.abs(ci), kind="stable")
    ci, oa, ob = ci[order], oa[order], ob[order]
    nw = 6
    pa = rng.standard_normal((nw, M, na)) + 1j * rng.standard_normal((nw, M, na))
    pb = rng.standard_normal((nw, M, nb)) + 1j * rng.standard_normal((nw, M, nb))
    s = MsdSystem(M, na, nb, 5, nw, len(ci))
    s.set_hamiltonian(h1, chol, -0.7)
    s.set_trial(ci, oa, ob)
    s.set_walkers(pa, pb)
    out = s.measure(0.01)
    assert np.max(np.abs(out["e_loc"] - e_fci)) < 1e-10


# ----------------------------------------------------------------------------
# propagation
# ----------------------------------------------------------------------------

def run_oracle_steps(wl, walkers, n_steps, dt, stabilize, e_shift=0.0):
    idx = list(walkers)
    pa, pb = wl.phi_a[idx].copy(), wl.phi_b[idx].copy()
    wts = wl.weights[idx].copy()
    lo = np.array([np.log(msd.trial_overlap(wl.ci, wl.occ_a, wl.occ_b, pa[i], pb[i]))
                   for i in range(len(idx))])
    b1 = propagate.one_body_half_step(wl.h1, wl.chol, dt)
    for step in range(n_steps):
        x = fields_for_step(wl, step)[idx]
        do_qr = stabilize > 0 and (step + 1) % stabilize == 0
        pa, pb, wts, lo, _ = propagate.step(wl.h1, wl.chol, wl.ci, wl.occ_a, wl.occ_b, pa, pb,
                                             wts, lo, x, dt, e_shift=e_shift, do_qr=do_qr, b1=b1)
    return pa, pb, wts, lo


@pytest.mark.parametrize("stabilize", [2, 0])
def test_tiny_propagation_matches_oracle(stabilize):
    wl = make_config("tiny")
    s = system_for(wl, stabilize_freq=stabilize)
    n_steps = 6
    fields = np.stack([fields_for_step(wl, k) for k in range(n_steps)])
    s.propagate(fields, wl.dt, e_shift=0.3)
    pa, pb, w, lo = s.get_walkers()
    ra, rb, rw, rlo = run_oracle_steps(wl, range(wl.n_walkers), n_steps, wl.dt, stabilize, 0.3)
    assert_rel(pa, ra, 1e-10)
    assert_rel(pb, rb, 1e-10)
    assert_rel(w, rw, 1e-10)
    assert_logo(lo, rlo, 1e-10)


def test_medium_ten_steps_sampled_walkers():
    wl = make_config("medium")
    s = system_for(wl, stabilize_freq=5)
    n_steps = 10
    fields = np.stack([fields_for_step(wl, k) for k in range(n_steps)])
    s.propagate(fields, wl.dt)
    pa, pb, w, lo = s.get_walkers()
    sample = [0, 64, 127]
    ra, rb, rw, rlo = run_oracle_steps(wl, sample, n_steps, wl.dt, 5)
    assert_rel(pa[sample], ra, 1e-10)
    assert_rel(pb[sample], rb, 1e-10)
    assert_rel(w[sample], rw, 1e-10)
    assert_logo(lo[sample], rlo, 1e-10)
    # orthonormal after the last QR (walkers removed by the phaseless
    # constraint are frozen where they were)
    for i in sample:
        if w[i] == 0.0:
            continue
        np.testing.assert_allclose(pa[i].conj().T @ pa[i], np.eye(wl.n_alpha), atol=1e-12)


def test_frozen_walker_stays_put():
    wl = make_config("tiny")
    wts = wl.weights.copy()
    wts[2] = 0.0
    s = MsdSystem(wl.M, 3, 3, wl.n_chol, wl.n_walkers, wl.n_det, stabilize_freq=1)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a, wl.phi_b, wts)
    _, _, _, lo0 = s.get_walkers()
    s.propagate(fields_for_step(wl, 0), wl.dt)
    pa, pb, w, lo = s.get_walkers()
    np.testing.assert_array_equal(pa[2], wl.phi_a[2])
    assert w[2] == 0.0 and lo[2] == lo0[2]


# ----------------------------------------------------------------------------
# boundary behaviour
# ----------------------------------------------------------------------------

def test_device_entry_points_match_host():
    torch = pytest.importorskip("torch")
    wl = make_config("tiny")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream().cuda_stream
    s = MsdSystem(wl.M, 3, 3, wl.n_chol, wl.n_walkers, wl.n_det, stream=stream)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers_dev(torch.from_numpy(wl.phi_a).to(dev), torch.from_numpy(wl.phi_b).to(dev),
                      torch.from_numpy(wl.weights).to(dev))
    lo = torch.empty(wl.n_walkers, dtype=torch.complex128, device=dev)
    fb = torch.empty(wl.n_walkers, wl.n_chol, dtype=torch.complex128, device=dev)
    el = torch.empty(wl.n_walkers, dtype=torch.complex128, device=dev)
    s.measure_dev(wl.dt, lo, fb, el)
    torch.cuda.synchronize()
    host = system_for(wl).measure(wl.dt)
    np.testing.assert_array_equal(lo.cpu().numpy(), host["log_ovlp"])
    np.testing.assert_array_equal(fb.cpu().numpy(), host["force_bias"])
    np.testing.assert_array_equal(el.cpu().numpy(), host["e_loc"])
    x = torch.from_numpy(np.stack([fields_for_step(wl, k) for k in range(3)])).to(dev)
    s.propagate_dev(x, wl.dt, 0.0, 3)
    torch.cuda.synchronize()
    h = system_for(wl)
    h.propagate(x.cpu().numpy(), wl.dt)
    a = s.get_walkers()
    b = h.get_walkers()
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def _excitation_lists(wl, rng):
    """Occupation rows -> (ref, k, offsets, holes, parts) with each spin's
    holes and particles in a random pairing order."""
    ref = [wl.occ_a[0], wl.occ_b[0]]
    ks, hs, ps = [[], []], [], []
    offsets = [0]
    for I in range(wl.n_det):
        h_all, p_all = [], []
        for sp, occ in enumerate((wl.occ_a, wl.occ_b)):
            r, row = set(ref[sp].tolist()), set(occ[I].tolist())
            h = rng.permutation(sorted(r - row)).tolist()
            p = rng.permutation(sorted(row - r)).tolist()
            ks[sp].append(len(h))
            h_all += h
            p_all += p
        hs += h_all
        ps += p_all
        offsets.append(offsets[-1] + len(h_all))
    return (ref[0], ref[1], np.array(ks[0]), np.array(ks[1]), np.array(offsets),
            np.array(hs, dtype=np.int32), np.array(ps, dtype=np.int32))


def test_trial_from_excitation_lists_matches_occupations():
    wl = make_config("medium", n_walkers=8, n_det=300)
    ra, rb, ka, kb, off, hs, ps = _excitation_lists(wl, np.random.default_rng(5))
    a = system_for(wl).measure(wl.dt)
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial_exc(ra, rb, wl.ci, ka, kb, off, hs, ps)
    s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
    b = s.measure(wl.dt)
    for key in a:
        np.testing.assert_array_equal(a[key], b[key])
    w, lo = s.get_weights()
    np.testing.assert_array_equal(w, wl.weights)
    np.testing.assert_array_equal(lo, b["log_ovlp"])
    bad = ps.copy()
    bad[0] = ra[0]  # a particle inside the reference
    with pytest.raises(MsdError) as e:
        s.set_trial_exc(ra, rb, wl.ci, ka, kb, off, hs, bad)
    assert e.value.name == "MSD_ERR_TRIAL"
    with pytest.raises(MsdError) as e:
        s.set_trial_exc(ra, rb, wl.ci, ka, kb, off + 1, hs, ps)
    assert e.value.name == "MSD_ERR_TRIAL"


def test_error_paths():
    wl = make_config("tiny")
    s = MsdSystem(wl.M, 3, 3, wl.n_chol, wl.n_walkers, wl.n_det)
    with pytest.raises(MsdError) as e:
        s.measure(0.01)
    assert e.value.name == "MSD_ERR_STATE"
    s.set_hamiltonian(wl.h1, wl.chol, 0.0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    bad = wl.phi_a.copy()
    bad[4, :3, :] = 0.0  # walker 4: zero reference block
    with pytest.raises(MsdError) as e:
        s.set_walkers(bad, wl.phi_b)
    assert e.value.name == "MSD_ERR_SINGULAR" and "walker 4" in str(e.value)
    with pytest.raises(MsdError) as e:
        s.set_trial(wl.ci, np.where(wl.occ_a == 0, 99, wl.occ_a), wl.occ_b)
    assert e.value.name == "MSD_ERR_TRIAL"
    h = wl.h1.copy()
    h[0, 1] += 1.0
    with pytest.raises(MsdError) as e:
        s.set_hamiltonian(h, wl.chol, 0.0)
    assert e.value.name == "MSD_ERR_ARG"
    for v in (2, 3, 4, 7):  # retired or unknown energy-intermediate kernels
        with pytest.raises(MsdError) as e:
            s.set_tuning(lambda_variant=v)
        assert e.value.name == "MSD_ERR_ARG"


@pytest.mark.parametrize("algo", [1, 2, 3])
def test_energy_algorithms_agree_with_oracle(algo):
    """Both forms of the same-spin second-order terms (per-minor lists and
    row-pair items of each string), and the fused Cholesky contraction
    (algo 3), against the oracle, with excitation orders up to 6."""
    wl = make_workload("algo", M=20, n_alpha=5, n_beta=4, n_chol=24, n_det=80, k_max=6,
                       window=(4, 9), c_law="flat", n_walkers=4, seed=91 + algo,
                       complex_ci=True, noise=0.4)
    s = system_for(wl, energy_algo=algo)
    out = s.measure(0.01)
    compare_walkers(wl, out, range(4), 0.01)


def test_graph_replay_matches_eager():
    """Steps and measurements replayed from HIP graphs equal the eager
    launches bit for bit, across several replays (with eager work between
    them), both step variants (with and without QR) and a change of dt."""
    wl = make_config("medium", n_walkers=16, n_det=300)

    def make(graphs):
        s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det,
                      stabilize_freq=2, graphs=graphs)
        s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
        s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
        s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
        return s

    eager, graph = make(False), make(True)
    for k in range(5):
        dt = wl.dt if k < 3 else 2 * wl.dt
        x = fields_for_step(wl, k)
        for s in (eager, graph):
            s.propagate(x, dt, 0.1)
        a, b = eager.get_walkers(), graph.get_walkers()
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u, v)
        ma, mb = eager.measure(dt, energy=k % 2 == 0), graph.measure(dt, energy=k % 2 == 0)
        for key in ma:
            np.testing.assert_array_equal(ma[key], mb[key])


# ----------------------------------------------------------------------------
# mixed-precision form
# ----------------------------------------------------------------------------

MIXED_E_TOL = 1e-4  # Ha: the mixed form's per-walker local-energy bound (0.1 mHa)


def test_mixed_medium_full_batch_against_fp64():
    """Mixed form on the Medium system: every walker's local energy within
    0.1 mHa of the FP64 path, force biases within FP32 rounding, and the FP64
    parts (overlaps, Green's functions) unchanged."""
    wl = make_config("medium")
    ref = system_for(wl).measure(wl.dt)
    s = system_for(wl, precision="mixed")
    out = s.measure(wl.dt)
    np.testing.assert_array_equal(out["log_ovlp"], ref["log_ovlp"])
    de = np.abs(out["e_loc"] - ref["e_loc"])
    assert de.max() <= MIXED_E_TOL, de.max()
    assert_rel(out["force_bias"], ref["force_bias"], tol=1e-5, floor=0.0)
    # and against the oracle on two walkers
    for w in (0, 77):
        o = oracle_walker(wl, w, wl.dt)
        assert abs(out["e_loc"][w] - o["e_loc"]) <= MIXED_E_TOL


@pytest.mark.parametrize("kmax,na,nb,noise", [(6, 5, 4, 0.1), (3, 3, 0, 0.1), (6, 5, 4, 0.4)])
def test_mixed_high_orders_against_oracle(kmax, na, nb, noise):
    """Orders up to 6 in the single-precision kernels, at the recipe's walker
    noise (0.1) and far from the reference (noise 0.4, |E_L| ~ 18 with a large
    imaginary part from a small trial overlap): every local energy within
    0.1 mHa of the oracle."""
    wl = make_workload("mixed", M=20, n_alpha=na, n_beta=nb, n_chol=24, n_det=60, k_max=kmax,
                       window=(min(na, 4), 9), c_law="flat", n_walkers=4, seed=131 + kmax,
                       complex_ci=True, noise=noise)
    s = system_for(wl, precision="mixed")
    out = s.measure(0.01)
    for w in range(4):
        o = oracle_walker(wl, w, 0.01)
        assert_logo(out["log_ovlp"][w], o["log_ovlp"])
        err = abs(out["e_loc"][w] - o["e_loc"])
        print(f"noise {noise}, walker {w}: mixed |dE_L| = {err * 1e3:.4f} mHa")
        assert err <= MIXED_E_TOL
        assert_rel(out["force_bias"][w], o["force_bias"], tol=1e-5, floor=0.0)


def test_mixed_orders_above_six_use_fp64_energy():
    """Alpha excitations up to order 8 in the mixed form (through the W-form,
    which takes any order): these walkers are far from the reference (noise
    0.5) and get FP64 energies, equal to the FP64 form to 1e-10 relative."""
    wl = make_workload("mixed8", M=20, n_alpha=8, n_beta=5, n_chol=20, n_det=60, k_max=12,
                       window=(8, 10), c_law="flat", n_walkers=3, seed=83, complex_ci=True,
                       noise=0.5)
    a = system_for(wl).measure(0.01)
    b = system_for(wl, precision="mixed").measure(0.01)
    assert_rel(b["e_loc"], a["e_loc"])
    o = oracle_walker(wl, 1, 0.01)
    assert_rel(a["e_loc"][1], o["e_loc"])


def test_mixed_propagation_two_steps_close_to_fp64():
    """Two steps with FP32 VHS and force bias stay close to the FP64 steps
    (trajectories of the two forms drift apart slowly; only short runs are
    compared)."""
    wl = make_config("medium", n_walkers=16, n_det=200)
    a, b = system_for(wl), system_for(wl, precision="mixed")
    for k in range(2):
        x = fields_for_step(wl, k)
        a.propagate(x, wl.dt)
        b.propagate(x, wl.dt)
    pa, pb = a.get_walkers(), b.get_walkers()
    for u, v in zip(pa[:2], pb[:2]):
        assert np.max(np.abs(u - v)) <= 1e-5 * np.max(np.abs(u))
    # the weight's exponent x.xbar - xbar.xbar/2 sums N_chol = 320 terms whose
    # FP32 force biases carry relative errors ~1e-6: ~1e-4 relative per step
    np.testing.assert_array_equal(pa[2] == 0, pb[2] == 0)
    live = pa[2] > 0
    assert np.max(np.abs(pa[2][live] - pb[2][live]) / pa[2][live]) <= 5e-4


# ----------------------------------------------------------------------------
# batches of uneven systems
# ----------------------------------------------------------------------------

def test_uneven_batch_graph_matches_separate_systems():
    """Four systems of different M, N, n_chol, n_det and walker counts stepped
    by one graph per batch step equal the same systems stepped one by one."""
    torch = pytest.importorskip("torch")
    from paper_2406_08314_amd import MsdBatch
    from synth import make_uneven

    wls = make_uneven(4, M_range=(12, 40), N_max=8, n_det_range=(20, 300),
                      walker_range=(4, 16))
    dev = torch.device("cuda:0")

    def make(wl):
        s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det,
                      stabilize_freq=2)
        s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
        s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
        s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
        return s

    solo = [make(wl) for wl in wls]
    batched = [make(wl) for wl in wls]
    batch = MsdBatch(batched)
    for k in range(4):
        xs = [torch.from_numpy(fields_for_step(wl, k)).to(dev) for wl in wls]
        batch.step(xs, 0.01, 0.05, measure=True)
        for s, wl, x in zip(solo, wls, xs):
            s.propagate(x.cpu().numpy(), 0.01, 0.05)
        torch.cuda.synchronize()
        for s, b in zip(solo, batched):
            m = s.measure(0.01)
            mb = b.get_measurement()
            for key in ("log_ovlp", "force_bias", "e_loc"):
                np.testing.assert_array_equal(m[key], mb[key])
            for u, v in zip(s.get_walkers(), b.get_walkers()):
                np.testing.assert_array_equal(u, v)
    batch.close()


# ----------------------------------------------------------------------------
# launch-shape tuning
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("tuning", [
    dict(lambda_variant=1, lambda_chunk=5, second_gsplit=3, second_stage=1, fb_splitk=1,
         second_gather=2, second_copy=1),
    dict(lambda_variant=1, lambda_chunk=7, second_gsplit=1, second_stage=3, fb_splitk=3,
         second_gather=1, second_copy=2),
    dict(lambda_variant=1, lambda_chunk=32, second_gsplit=8, second_stage=4, fb_splitk=16),
    dict(lambda_variant=1, lambda_chunk=11, second_gsplit=2, second_stage=2, fb_splitk=4),
    dict(lambda_variant=1, lambda_chunk=1, second_gsplit=1, second_stage=1, fb_splitk=1),
    dict(lambda_variant=5, lambda_chunk=13, second_gsplit=2, second_stage=2, fb_splitk=4),
    dict(lambda_variant=5, lambda_chunk=1, walker_tile=4),
    dict(lambda_variant=5),
    dict(second_waves=16, second_stage=5, second_gsplit=3, second_copy=2),
    dict(second_waves=16, second_stage=3, second_gsplit=1, second_copy=1, second_gather=2),
    dict(walker_tile=4),
    dict(second_whole=1),                       # order-3 strings as row-pair items
    dict(second_whole=2, second_stage=3, second_gsplit=2, second_waves=8),
])
def test_tuning_overrides_keep_parity(tuning):
    """Ragged Cholesky chunks and stages (320 vectors split 5/7/3 ways) in
    every launch-shape override still match the oracle."""
    wl = make_config("medium", n_walkers=6, n_det=300)
    s = system_for(wl)
    s.set_tuning(**tuning)
    out = s.measure(wl.dt)
    got = s.get_tuning()
    for k, v in tuning.items():
        assert got[k] == v, (k, got)
    compare_walkers(wl, out, [0, 5], wl.dt)


def test_autotune_picks_valid_shapes_and_keeps_results():
    wl = make_config("medium", n_walkers=16, n_det=300)
    ref = system_for(wl).measure(wl.dt)
    for precision in ("fp64", "mixed"):
        s = system_for(wl, precision=precision)
        t = s.autotune(wl.dt, reps=2)
        assert 1 <= t["fb_splitk"] <= 16 and t["lambda_variant"] in (1, 5, 6)
        assert t["lambda_chunk"] >= 1 and t["second_gsplit"] >= 1 and t["second_stage"] >= 1
        out = s.measure(wl.dt)
        np.testing.assert_array_equal(out["log_ovlp"], ref["log_ovlp"])
        tol = 1e-10 * max(1.0, np.max(np.abs(ref["e_loc"]))) if precision == "fp64" else MIXED_E_TOL
        assert np.max(np.abs(out["e_loc"] - ref["e_loc"])) <= tol


@pytest.mark.parametrize("nv,n_chol", [(8, 20), (16, 21), (40, 20)])
def test_fused_contraction_row_tiles(nv, n_chol):
    """The fused contraction kernel at 1, 2 and 3 tiles of 16 restricted rows
    (n_vir_act + 8 = 16, 24, 48), with a partly filled group of four walkers
    and an odd number of Cholesky vectors (the trace pass takes them in
    pairs): FP64 against the oracle on every walker, the mixed form within
    0.1 mHa."""
    wl = make_workload("fused", M=8 + nv + 2, n_alpha=8, n_beta=8, n_chol=n_chol, n_det=150,
                       k_max=4, window=(8, nv), c_law="flat", n_walkers=5, seed=500 + nv)
    s = system_for(wl)
    out = s.measure(wl.dt)
    assert s.get_tuning()["lambda_variant"] == 5
    compare_walkers(wl, out, range(wl.n_walkers), wl.dt)
    m = system_for(wl, precision="mixed")
    outm = m.measure(wl.dt)
    assert m.get_tuning()["lambda_variant"] == 5
    assert np.max(np.abs(outm["e_loc"] - out["e_loc"])) <= MIXED_E_TOL


@pytest.mark.parametrize("variant", [1, 5])
def test_mixed_lambda_variants_against_fp64(variant):
    """Each single-precision energy-intermediate kernel that applies at Medium
    keeps every walker's local energy within 0.1 mHa of the FP64 path (32
    walkers; the general kernel's mixed form is checked in its own tests)."""
    wl = make_config("medium", n_walkers=32)
    ref = system_for(wl).measure(wl.dt)
    s = system_for(wl, precision="mixed")
    s.set_tuning(lambda_variant=variant)
    out = s.measure(wl.dt)
    assert s.get_tuning()["lambda_variant"] == variant
    assert np.max(np.abs(out["e_loc"] - ref["e_loc"])) <= MIXED_E_TOL

"""GPU parity of the block driver (comb population control, block energy)
against the CPU oracle (oracle/driver.py), through the C ABI."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import driver, msd
from paper_2406_08314_amd import MsdError, MsdSystem
from synth import fields_for_step, make_config

pytestmark = pytest.mark.gpu

TOL = 1e-10


def system_for(wl, weights=None, phi=None, n_walkers=None, **kw):
    nw = wl.n_walkers if n_walkers is None else n_walkers
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, nw, wl.n_det, **kw)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    pa, pb = phi if phi is not None else (wl.phi_a, wl.phi_b)
    s.set_walkers(pa, pb, wl.weights if weights is None else weights)
    return s


def dyadic_weights(rng, n, p_zero=0.2):
    """Weights k / 8 (some 0): every running sum is exact in any order, so
    the comb's decisions are fixed exactly, ties included."""
    w = rng.integers(1, 17, size=n) / 8.0
    w[rng.random(n) < p_zero] = 0.0
    w[0] = 1.0
    return w


@pytest.mark.parametrize("n_walkers", [8, 2600])
def test_comb_matches_oracle(n_walkers):
    """Parents bit-exact (dyadic weights, offsets on and off the tooth grid),
    copies bit-exact, new weights W / n."""
    wl = make_config("tiny")
    rng = np.random.default_rng(81)
    pa = np.resize(wl.phi_a, (n_walkers,) + wl.phi_a.shape[1:])
    pb = np.resize(wl.phi_b, (n_walkers,) + wl.phi_b.shape[1:])
    w = dyadic_weights(rng, n_walkers)
    s = system_for(wl, weights=w, phi=(pa, pb), n_walkers=n_walkers)
    print(f"comb n_walkers={n_walkers}", flush=True)
    for z in (0.0, 0.5, 0.3125, 0.73):
        a0, b0, w0, lo0 = s.get_walkers()
        parent = s.population_control(z)
        ref, wn = driver.comb(w0, z)
        np.testing.assert_array_equal(parent, ref)
        a1, b1, w1, lo1 = s.get_walkers()
        np.testing.assert_array_equal(a1, a0[ref])
        np.testing.assert_array_equal(b1, b0[ref])
        np.testing.assert_array_equal(lo1, lo0[ref])
        np.testing.assert_array_equal(w1, np.full(n_walkers, wn))
        assert np.all(w0[parent] > 0)
        # give the next round unequal weights again
        w = dyadic_weights(rng, n_walkers)
        s.set_walkers(a1, b1, w)


def test_comb_all_frozen_changes_nothing():
    wl = make_config("tiny")
    s = system_for(wl, weights=np.zeros(wl.n_walkers))
    before = s.get_walkers()
    parent = s.population_control(0.4)
    np.testing.assert_array_equal(parent, np.arange(wl.n_walkers))
    for u, v in zip(s.get_walkers(), before):
        np.testing.assert_array_equal(u, v)


def test_comb_device_entry_point_matches_host():
    torch = pytest.importorskip("torch")
    wl = make_config("tiny")
    rng = np.random.default_rng(82)
    w = dyadic_weights(rng, wl.n_walkers)
    h = system_for(wl, weights=w)
    d = system_for(wl, weights=w, stream=torch.cuda.current_stream().cuda_stream)
    par = torch.empty(wl.n_walkers, dtype=torch.int32, device="cuda:0")
    d.population_control_dev(0.61, par)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(par.cpu().numpy(), h.population_control(0.61))
    for u, v in zip(d.get_walkers(), h.get_walkers()):
        np.testing.assert_array_equal(u, v)


@pytest.mark.parametrize("graphs", [False, True])
def test_block_matches_oracle(graphs):
    """Six steps (QR every 2), comb after steps 3 and 6, one measurement:
    walkers, weights, overlaps, E_L and the weighted energy sums."""
    torch = pytest.importorskip("torch")
    wl = make_config("tiny")
    w = wl.weights.copy()
    w[5] = 0.0  # a frozen walker is never copied
    s = system_for(wl, weights=w, stabilize_freq=2, graphs=graphs)
    n_steps, zs = 6, [0.27, 0.81]
    fields = np.stack([fields_for_step(wl, k) for k in range(n_steps)])
    print(f"block graphs={graphs}", flush=True)
    num, den = s.run_block(torch.from_numpy(fields).to("cuda:0"), n_steps, wl.dt, 0.2, 3, zs)
    pa, pb, wt, lo = s.get_walkers()
    el = s.get_measurement(force_bias=False)["e_loc"]
    lo0 = np.array([np.log(msd.trial_overlap(wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[i],
                                             wl.phi_b[i])) for i in range(wl.n_walkers)])
    ra, rb, rw, rlo, rel, rnum, rden = driver.block(
        wl.h1, wl.chol, wl.e0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a, wl.phi_b, w, lo0, fields,
        wl.dt, zs, e_shift=0.2, stabilize_freq=2, pop_freq=3)
    scale = max(1.0, float(np.max(np.abs(ra))))
    assert np.max(np.abs(pa - ra)) <= TOL * scale
    assert np.max(np.abs(pb - rb)) <= TOL * max(1.0, float(np.max(np.abs(rb))))
    np.testing.assert_allclose(wt, rw, rtol=TOL, atol=0)
    assert np.max(np.abs(np.exp(lo - rlo) - 1)) <= TOL
    assert np.max(np.abs(el - rel)) <= TOL * max(1.0, float(np.max(np.abs(rel))))
    assert abs(num - rnum) <= TOL * abs(rnum) and abs(den - rden) <= TOL * rden
    # the library's measurement of the final walkers is the oracle's
    e_block = (num / den).real
    assert abs(e_block - (rnum / rden).real) <= TOL * abs(e_block)


def test_block_without_population_control_is_propagate_plus_measure():
    torch = pytest.importorskip("torch")
    wl = make_config("tiny")
    n_steps = 4
    fields = np.stack([fields_for_step(wl, k) for k in range(n_steps)])
    a = system_for(wl, stabilize_freq=2)
    num, den = a.run_block(torch.from_numpy(fields).to("cuda:0"), n_steps, wl.dt, 0.0, 0)
    b = system_for(wl, stabilize_freq=2)
    b.propagate(fields, wl.dt)
    out = b.measure(wl.dt)
    for u, v in zip(a.get_walkers(), b.get_walkers()):
        np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(a.get_measurement(force_bias=False)["e_loc"], out["e_loc"])
    _, _, w, _ = b.get_walkers()
    live = w > 0
    assert abs(den - w[live].sum()) <= 1e-14 * den
    assert abs(num - np.sum(w[live] * out["e_loc"][live])) <= 1e-12 * abs(num)


def test_driver_argument_errors():
    torch = pytest.importorskip("torch")
    wl = make_config("tiny")
    s = system_for(wl)
    for z in (-0.1, 1.0, float("nan")):
        with pytest.raises(MsdError) as e:
            s.population_control(z)
        assert e.value.name == "MSD_ERR_ARG"
    x = torch.zeros((5, wl.n_walkers, wl.n_chol), dtype=torch.float64, device="cuda:0")
    with pytest.raises(MsdError):
        s.run_block(x, 5, wl.dt, 0.0, 5, [])       # offsets missing
    with pytest.raises(MsdError):
        s.run_block(x, 5, wl.dt, 0.0, 5, [1.5])    # offset outside [0, 1)
    with pytest.raises(MsdError):
        s.run_block(x, 0, wl.dt, 0.0, 5, [])       # no steps


def test_comb_single_walker_and_timing_stage():
    """One walker: the comb copies it onto itself with its own weight; with
    timing on, the population-control stage is recorded once per call."""
    wl = make_config("tiny")
    s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, 1, wl.n_det, timing=True)
    s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
    s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
    s.set_walkers(wl.phi_a[:1], wl.phi_b[:1], np.array([0.625]))
    before = s.get_walkers()
    for z in (0.0, 0.99):
        assert list(s.population_control(z)) == [0]
    after = s.get_walkers()
    for u, v in zip(after, before):
        np.testing.assert_array_equal(u, v)
    t = s.timings()
    assert t["pop_control"][1] == 2


def test_block_with_timing_matches_block_with_graphs():
    """The same block through timed eager launches and through replayed
    graphs gives identical walkers and energy sums."""
    torch = pytest.importorskip("torch")
    wl = make_config("tiny")
    n_steps, zs = 4, [0.42, 0.07]
    fields = torch.from_numpy(np.stack([fields_for_step(wl, k) for k in range(n_steps)])).to(
        "cuda:0")
    out = []
    for kw in (dict(timing=True), dict(graphs=True)):
        s = system_for(wl, stabilize_freq=2, **kw)
        e = s.run_block(fields, n_steps, wl.dt, 0.1, 2, zs)
        out.append((e, s.get_walkers()))
    assert out[0][0] == out[1][0]
    for u, v in zip(out[0][1], out[1][1]):
        np.testing.assert_array_equal(u, v)


def test_comb_general_weights_against_oracle():
    """Non-dyadic weights (running sums round differently in the library's
    parallel scan and the oracle's sequential sum): parents equal wherever
    every tooth is farther than 1e-9 W from an interval boundary, and the
    copy counts are floor or ceil of n w_i / W."""
    wl = make_config("tiny")
    n_walkers = 3000
    rng = np.random.default_rng(83)
    pa = np.resize(wl.phi_a, (n_walkers,) + wl.phi_a.shape[1:])
    pb = np.resize(wl.phi_b, (n_walkers,) + wl.phi_b.shape[1:])
    w = rng.lognormal(sigma=1.0, size=n_walkers)
    w[rng.random(n_walkers) < 0.1] = 0.0
    s = system_for(wl, weights=w, phi=(pa, pb), n_walkers=n_walkers)
    for z in (0.113, 0.5821):
        _, _, w0, _ = s.get_walkers()
        parent = s.population_control(z)
        ref, wn = driver.comb(w0, z)
        c = np.cumsum(w0)
        teeth = (np.arange(n_walkers) + z) * c[-1] / n_walkers
        gap = np.min(np.abs(teeth[:, None] - c[None, :]))
        assert gap > 1e-9 * c[-1]  # no tooth is near a boundary for this seed
        np.testing.assert_array_equal(parent, ref)
        cnt = np.bincount(parent, minlength=n_walkers)
        exp = n_walkers * w0 / c[-1]
        assert np.all(cnt >= np.floor(exp)) and np.all(cnt <= np.ceil(exp))
        _, _, w1, _ = s.get_walkers()
        np.testing.assert_allclose(w1, wn, rtol=1e-14)
        s.set_walkers(pa, pb, rng.lognormal(sigma=1.0, size=n_walkers))

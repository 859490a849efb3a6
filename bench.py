"""Benchmark of the MSD-AFQMC hot path on one MI355X.

One step = one pass of the whole hot path over the walker batch:
  propagate (force bias -> VHS -> one-body/Taylor/one-body -> new overlap ->
  phaseless weights -> QR) followed by a full measurement (overlap, Green's
  function, force bias, local energy).
Metric: MSD Wick evaluations per second = n_walkers * n_det / step time, for the
FP64 form (``value``) and the mixed form (``mixed``), with the mixed form's
largest per-walker local-energy difference from FP64.
Workload (default): the binuclear Cu-oxo-cluster-shaped synthetic system
(M=200, N=30+30, 1,200 Cholesky vectors, 10,000 determinants of excitation
order <= 4, 256 walkers).  ``--config medium`` times the Medium system (M=64,
N=8+8, 320 vectors, 1,000 determinants, 128 walkers) instead; the default run
also reports Medium as a secondary record.

Prints ONE JSON line.  `--gpus N` with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
TRAFFIC_PROFILES = {
    # (stage, workload) or (stage, lambda variant, workload): committed counter
    # summaries of the stage's kernel at that workload
    ("energy_gamma", "medium"): os.path.join(ROOT, "profiles", "energy_second_medium_hbm_traffic.md"),
    ("energy_gamma", "cu_oxo"): os.path.join(ROOT, "profiles", "energy_second_cu_oxo_hbm_traffic.md"),
    ("lambda", 5, "medium"): os.path.join(ROOT, "profiles", "ltl_mfma_medium_hbm_traffic.md"),
    ("lambda", 6, "cu_oxo"): os.path.join(ROOT, "profiles", "ltl_general_cu_oxo_hbm_traffic.md"),
}


def measured_traffic(stage):
    """(HBM bytes per launch, launch shape) of the second-order energy kernel
    from the committed rocprofv3 counter summary, or None if the kernel source
    changed since the counters were taken.  The shape is (Cholesky split,
    vectors per LDS stage, stage copy mode)."""
    import hashlib
    try:
        text = open(TRAFFIC_PROFILES[stage]).read()  # stage: name or (name, variant)
    except (KeyError, OSError):
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch:", "source:", "launch_shape:")))
    try:
        fields = vals["source"].split()
        src, prefix = fields[0], fields[-1]
        digest = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
        if not digest.startswith(prefix):
            return None
        shape = tuple(int(v) for v in vals.get("launch_shape", "").split())
        return float(vals["traffic_bytes_per_launch"]), shape
    except (KeyError, OSError, ValueError, IndexError):
        return None


def stage_work(wl, lib_sys, stage):
    """Algorithmic work of one launch group of a stage: (amount, unit, bound)."""
    M, na, nb, NG, NW = wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers
    Ntot = na + nb
    tt = lib_sys.tables
    # the energy stages run once per walker tile: a launch group covers
    # NW / n_tiles walkers on average (the propagation GEMMs take all walkers)
    wt = lib_sys.get_tuning().get("walker_tile") or NW
    NWe = NW / -(-NW // max(wt, 1))
    if stage == "lt_gemm":  # both spins are separate launch groups; average them
        f = sum(2.0 * NG * (N + nv) * M * 2 * NWe * N for N, nv in
                ((na, tt["nv"][0]), (nb, tt["nv"][1]))) / 2
        return f, "flop", "mfma"
    if stage == "fb_gemm":
        return 2.0 * NG * tt["P_all"] * M * 2 * NW, "flop", "mfma"
    if stage == "vhs_gemm":
        return 2.0 * 2 * NW * NG * M * M, "flop", "mfma"
    if stage == "taylor":  # n_taylor complex GEMMs per launch group
        return 6 * 8.0 * M * M * Ntot * NW, "flop", "mfma"
    if stage == "one_body":
        return 4.0 * M * M * Ntot * NW, "flop", "mfma"
    if stage == "lambda" and lib_sys.get_tuning()["lambda_variant"] == 5:
        # fused contraction kernel: matrix-core bound.  Per walker, vector and
        # spin: LT = L[R u V, :] T (4 P N M flop, complex T), Lambda = T[V, :] Q
        # and Xi = Lambda Q (8 flop per complex MAC, nv N N each)
        f = 0.0
        for N, nv in ((na, tt["nv"][0]), (nb, tt["nv"][1])):
            f += NWe * NG * (4.0 * (N + nv) * N * M + 2 * 8.0 * nv * N * N)
        return f, "flop", "mfma"
    if stage == "lambda" and lib_sys.get_tuning()["lambda_variant"] == 6:
        # general fused contraction kernel: per walker, vector and spin LT =
        # L[R u V, :] T (4 P N M flop, real L times complex T, P = N + nv), Lambda
        # = T[V, :] Q (8 nv N N) and D = C Q_W^T for <C, Lambda Q> (8 nv no N)
        f = 0.0
        for N, nv, no in ((na, tt["nv"][0], tt["no"][0]), (nb, tt["nv"][1], tt["no"][1])):
            f += NWe * NG * (4.0 * (N + nv) * N * M + 8.0 * nv * N * N + 8.0 * nv * no * N)
        return f, "flop", "mfma"
    if stage == "traces":
        # Q = L[R, :] T (4 N N M flop) and tr QQ (8 N N) per walker, vector, spin
        return sum(NWe * NG * (4.0 * N * N * M + 8.0 * N * N) for N in (na, nb)), "flop", "mfma"
    if stage == "lambda":
        # matrix-core kernel: bound by its HBM stream (LT tiles in, Lambda
        # windows, ZW partials, v0 and ex0 out)
        chunk = lib_sys.get_tuning()["lambda_chunk"] or 16
        n_chunks = (NG + chunk - 1) // chunk
        b = 0.0
        for N, nv, no in ((na, tt["nv"][0], tt["no"][0]), (nb, tt["nv"][1], tt["no"][1])):
            b += NWe * NG * 16.0 * ((N + nv) * N + nv * no) + NWe * n_chunks * nv * no * 16.0
        b += 2 * 2 * NWe * NG * 16.0
        return b, "byte", "hbm"
    if stage == "energy_gamma" and lib_sys.get_tuning()["energy_form"] == 1:
        # W-form: per walker and Cholesky vector, the real GEMMs of the
        # interleaved windows give W^{ab}, W^{aa}, W^{bb} (8 flop per complex MAC)
        xa, xb = tt["nv"][0] * tt["no"][0], tt["nv"][1] * tt["no"][1]
        return NWe * NG * 8.0 * (xa * xa + xa * xb + xb * xb), "flop", "mfma"
    if stage == "energy_gamma":
        # per walker and Cholesky vector: one complex MAC per opposite-spin
        # pair; per string of order k, k(k-1)/2 x k(k-1)/2 two-by-two minors of
        # Y, each 2 complex products, a difference and a complex MAC (22 flop)
        f = 8.0 * tt["n_pair"]
        for sp in (0, 1):
            for k, n in tt["strings"][sp].items():
                p = k * (k - 1) // 2
                f += 22.0 * p * p * n
        return NWe * NG * f, "flop", "alu"
    return None


def cpu_baseline(wl, n_walk=2, n_det=None):
    """The brute-force oracle on a bounded sample: the first ``n_walk``
    walkers and the first ``n_det`` determinants of the trial (all if None),
    one propagation step + one full measurement.  The one-body propagator
    B1 = expm(-dt h'/2) is per-Hamiltonian set-up on both sides and is built
    before the clock starts."""
    from oracle import msd, propagate
    from synth import fields_for_step

    nd = wl.n_det if n_det is None else min(n_det, wl.n_det)
    ci, oa, ob = wl.ci[:nd], wl.occ_a[:nd], wl.occ_b[:nd]
    idx = list(range(n_walk))
    b1 = propagate.one_body_half_step(wl.h1, wl.chol, wl.dt)
    t0 = time.perf_counter()
    lo = np.array([np.log(msd.trial_overlap(ci, oa, ob, wl.phi_a[w], wl.phi_b[w])) for w in idx])
    pa, pb, _, _, _ = propagate.step(wl.h1, wl.chol, ci, oa, ob, wl.phi_a[idx], wl.phi_b[idx],
                                     wl.weights[idx], lo, fields_for_step(wl, 0)[idx], wl.dt,
                                     do_qr=True, b1=b1)
    msd.measure(wl.h1, wl.chol, wl.e0, ci, oa, ob, pa, pb, wl.dt)
    dt = time.perf_counter() - t0
    return {"value": n_walk * nd / dt, "unit": "walker*det/s", "cores": _threads(),
            "cpu_count": os.cpu_count(), "cpu_model": _cpu_model(), "kind": "oracle",
            "sample": f"brute-force oracle (complex128 NumPy): first {n_walk} of {wl.n_walkers} "
                      f"walkers x first {nd} of {wl.n_det} determinants (truncated trial), one "
                      f"step (propagate with QR + measure), {dt:.1f} s"}


def cpu_wick(wl, n_walk=2):
    """The oracle's per-determinant generalised-Wick path (NumPy + plain C,
    OpenMP over determinants) on the first ``n_walk`` walkers, all
    determinants, one measurement each (overlap, G, force bias, E_L)."""
    from oracle import wick

    t0 = time.perf_counter()
    wick.measure(wl.h1, wl.chol, wl.e0, wl.ci, wl.occ_a, wl.occ_b, wl.phi_a[:n_walk],
                 wl.phi_b[:n_walk], wl.dt)
    dt = time.perf_counter() - t0
    return {"value": n_walk * wl.n_det / dt, "unit": "walker*det/s", "cores": _threads(),
            "kind": "oracle (generalised-Wick CPU path)",
            "sample": f"first {n_walk} walkers x all {wl.n_det} determinants, one measurement, "
                      f"{dt:.1f} s"}


def _threads():
    from threadpoolctl import threadpool_info
    return int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


WORKLOADS = {
    "cu_oxo": "cu_oxo: M=200, N=30+30, Nchol=1200, Ndet=10000 (orders <= 4, window 16x32), "
              "256 walkers, dt=0.005, QR every step",
    "medium": "medium: M=64, N=8+8, Nchol=320, Ndet=1000 (orders 0-4), 128 walkers, dt=0.005, "
              "QR every step",
    "fe2s2": "fe2s2: M=300, N=45+45, Nchol=2000, Ndet=200000 (orders <= 6, window 15x5), "
             "512 walkers, dt=0.005, QR every step",
    "tiny": "tiny: M=12, N=3+3, Nchol=48, Ndet=20, 8 walkers, dt=0.005, QR every step",
}


def run_config(name, args, torch, stages=True, block=True):
    """Time one workload in both forms; returns a dict of results."""
    from paper_2406_08314_amd import MsdSystem
    from synth import fields_for_step, make_config

    wl = make_config(name)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()

    def system(timing, precision="fp64"):
        s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det, device=0,
                      stream=stream.cuda_stream, stabilize_freq=1, timing=timing,
                      graphs=not timing, precision=precision)
        s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
        s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
        s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
        s.tables = _tables(wl)
        return s

    n_total = args.warmup + args.steps
    fields = torch.from_numpy(np.stack([fields_for_step(wl, k) for k in range(n_total)])).to(dev)
    lo = torch.empty(wl.n_walkers, dtype=torch.complex128, device=dev)
    fb = torch.empty(wl.n_walkers, wl.n_chol, dtype=torch.complex128, device=dev)
    el = torch.empty(wl.n_walkers, dtype=torch.complex128, device=dev)

    def step(s, k):
        s.propagate_dev(fields[k].reshape(-1), wl.dt, 0.0, 1)
        s.measure_dev(wl.dt, lo, fb, el)

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        for k in range(n):
            fn(k)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), time.perf_counter() - t0

    tunings, extra = {}, {}

    def run_form(precision):
        """Graph-replayed steps and measurements of one form; also returns the
        local energies of the initial walkers (same input for both forms)."""
        s = system(False, precision)
        e_init = s.measure(wl.dt)["e_loc"]
        tunings[precision] = s.autotune(wl.dt, reps=3) if args.autotune else s.get_tuning()
        for k in range(args.warmup):
            step(s, k)
        ms, wall = timed(lambda k: step(s, args.warmup + k), args.steps)
        ms_meas, _ = timed(lambda k: s.measure_dev(wl.dt, lo, fb, el), args.steps)
        ms_prop, _ = timed(lambda k: s.propagate_dev(fields[k % n_total].reshape(-1), wl.dt,
                                                     0.0, 1), args.steps)
        # walkers far from the reference at this point (max |T| above the mixed
        # form's threshold: those get FP64 energies in the mixed form)
        pa, pb, _, _ = s.get_walkers()
        far = int(np.sum(_tmax(pa, wl.n_alpha, pb, wl.n_beta) > 2.0))
        # the measurement on the initial walkers (near the reference)
        s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
        s.measure_dev(wl.dt, lo, fb, el)
        ms_init, _ = timed(lambda k: s.measure_dev(wl.dt, lo, fb, el), args.steps)
        extra[precision] = {"propagate_only_ms": round(ms_prop / args.steps, 4),
                            "measure_initial_ms": round(ms_init / args.steps, 4),
                            "walkers_far_from_reference_after_steps": far}
        if block:
            # the paper's block shape: 25 propagation steps, population control
            # every 5, one measurement (weighted block energy), on the
            # library's block driver
            blk_fields = torch.stack([fields[j % n_total] for j in range(25)]).contiguous()
            zs = np.random.default_rng(wl.seed + 25).random(5)
            ms_block, _ = timed(lambda _: s.run_block(blk_fields, 25, wl.dt, 0.0, 5, zs), 2)
            extra[precision].update({
                "block_ms": round(ms_block / 2, 4),
                "block_note": "msd_run_block: 25 steps (QR every step), comb population "
                              "control every 5 steps, 1 measurement with the weighted block "
                              "energy"})
        s.close()
        return ms / args.steps, ms_meas / args.steps, wall, e_init

    nwd = wl.n_walkers * wl.n_det
    ms_step, ms_meas, wall, e64 = run_form("fp64")
    mx_step, mx_meas, _, emx = run_form("mixed")
    res = {"wl": wl, "value": nwd / (ms_step * 1e-3), "ms_per_step": ms_step, "wall_s": wall,
           "measure_only": {"value": nwd / (ms_meas * 1e-3), "ms": round(ms_meas, 4),
                            "note": "msd_measure_dev alone (overlap, G, force bias, E_L)"},
           **extra["fp64"]}
    res["mixed"] = {"value": nwd / (mx_step * 1e-3), "ms_per_step": round(mx_step, 4),
                    "measure_only_value": nwd / (mx_meas * 1e-3),
                    "measure_only_ms": round(mx_meas, 4),
                    "speedup_vs_fp64": round(ms_step / mx_step, 3),
                    "measure_speedup_vs_fp64": round(ms_meas / mx_meas, 3),
                    "measure_initial_speedup_vs_fp64": round(
                        extra["fp64"]["measure_initial_ms"] / extra["mixed"]["measure_initial_ms"], 3),
                    "note": "walkers with max|T| > 2 (T = Phi A^-1 relative to the reference) get "
                            "FP64 energies in the mixed form; the synthetic trajectories leave the "
                            "reference after the first step, the initial walkers stay near it",
                    "max_abs_dE_L_mHa": float(np.max(np.abs(emx - e64))) * 1e3,
                    "error_sample": f"all {wl.n_walkers} walkers, one measurement of the "
                                    f"initial walkers",
                    **extra["mixed"]}
    res["tuning"] = tunings
    if not stages:
        return res

    # instrumented passes of the same steps: HIP events around every stage
    def stage_pass(precision):
        s = system(True, precision)
        s.set_tuning(**{k: v for k, v in tunings[precision].items() if k != "energy_form"})
        for k in range(args.warmup):
            step(s, k)
        torch.cuda.synchronize()
        s.reset_timings()
        timed(lambda k: step(s, args.warmup + k), args.steps)
        return s

    sm = stage_pass("mixed")
    res["mixed"]["stages_ms"] = {k: round(v[0] / max(v[1], 1), 4)
                                 for k, v in sm.timings().items() if v[1]}
    sm.close()
    s = stage_pass("fp64")
    stages = s.timings()
    res["dominant_stage"] = max((k for k in stages if stages[k][1] > 0),
                                key=lambda k: stages[k][0])
    res["stages_ms"] = {k: round(v[0] / max(v[1], 1), 4) for k, v in stages.items() if v[1]}
    rl = rooflines(wl, s, stages, tunings["fp64"])
    res["roofline"] = rl[0] if rl else None
    res["roofline_next"] = rl[1] if len(rl) > 1 else None
    s.close()
    return res


def run_uneven(args, torch, steps=3, warmup=1):
    """The uneven batch of 32 independent systems: one batch step (propagate +
    measure every system) replayed as one HIP graph with a branch per system,
    against the same systems stepped one after another (each with its own
    graph replay), FP64 and mixed forms."""
    from paper_2406_08314_amd import MsdBatch, MsdSystem
    from synth import fields_for_step, make_uneven

    wls = make_uneven()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    fields = [torch.from_numpy(fields_for_step(wl, 0)).to(dev) for wl in wls]
    nwd = sum(wl.n_walkers * wl.n_det for wl in wls)
    dt = wls[0].dt

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    out = {"systems": len(wls), "walker_det_per_step": nwd,
           "shapes": "M 38-199, N 4-30 per spin, 5M Cholesky vectors, 151-90,740 "
                     "determinants (orders <= 4), 71-496 walkers"}
    for precision in ("fp64", "mixed"):
        systems = []
        for wl in wls:
            s = MsdSystem(wl.M, wl.n_alpha, wl.n_beta, wl.n_chol, wl.n_walkers, wl.n_det,
                          device=0, stream=stream.cuda_stream, graphs=True, precision=precision)
            s.set_hamiltonian(wl.h1, wl.chol, wl.e0)
            s.set_trial(wl.ci, wl.occ_a, wl.occ_b)
            s.set_walkers(wl.phi_a, wl.phi_b, wl.weights)
            systems.append(s)
        b = MsdBatch(systems, stream=stream.cuda_stream)
        eloc = [torch.empty(wl.n_walkers, dtype=torch.complex128, device=dev) for wl in wls]

        def batch_step():
            b.step(fields, dt, 0.0, measure=True)

        def separate():
            for s, f, e in zip(systems, fields, eloc):
                s.propagate_dev(f.reshape(-1), dt, 0.0, 1)
                s.measure_dev(dt, e_loc=e)

        for _ in range(warmup):
            batch_step()
            separate()
        ms_b = timed(batch_step, steps)
        ms_s = timed(separate, steps)
        out[precision] = {"batch_graph_ms": round(ms_b, 3), "separate_ms": round(ms_s, 3),
                          "value": nwd / (ms_b * 1e-3), "unit": "walker*det/s",
                          "speedup_vs_separate": round(ms_s / ms_b, 3)}
        b.close()
        for s in systems:
            s.close()
    out["mixed_speedup_vs_fp64"] = round(out["fp64"]["batch_graph_ms"] /
                                         out["mixed"]["batch_graph_ms"], 3)
    return out


def rooflines(wl, s, stages, t, count=2):
    """Roofline records of the ``count`` most expensive stages that have a
    work model, most expensive first."""
    out = []
    for name in sorted(stages, key=lambda k: -stages[k][0]):
        if len(out) == count:
            break
        work = stage_work(wl, s, name)
        if work is None or stages[name][1] == 0:
            continue
        amount, unit, bound = work
        avg_s = stages[name][0] / stages[name][1] * 1e-3
        if unit == "flop":
            ach, peak, u = amount / avg_s / 1e12, FP64_PEAK_TFLOPS, "TFLOP/s"
        else:
            ach, peak, u = amount / avg_s / 1e9, HBM_PEAK_GBS, "GB/s"
        traffic = None
        if name == "energy_gamma":
            prof = measured_traffic((name, wl.name))
            if prof and prof[1] == (t["second_gsplit"], t["second_stage"], t["second_copy"]):
                traffic = prof[0]
        elif name == "lambda":
            prof = measured_traffic(("lambda", t["lambda_variant"], wl.name))
            if prof and (not prof[1] or prof[1] == (t["lambda_chunk"],)):
                traffic = prof[0]
        lam_kernel = {1: "k_lambda_rows", 5: "k_ltl_mfma",
                      6: "k_ltl_general"}.get(t["lambda_variant"], "k_lambda")
        kernel = {"energy_gamma": "k_energy_second", "lambda": lam_kernel, "traces": "k_qtr",
                  "lt_gemm": "k_gemm_f64 (LT)"}.get(name, name)
        out.append({"kernel": kernel, "stage": name, "bound": bound,
                    "achieved": round(ach, 3), "peak": peak, "unit": u,
                    "frac": round(ach / peak, 4), "traffic": traffic,
                    "avg_launch_ms": round(avg_s * 1e3, 4),
                    "work_per_launch": amount, "work_unit": unit})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cu_oxo", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary Medium record of the default run")
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner before timing (default: the library's "
                         "own launch-shape heuristics, the shapes the committed profiles cover)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise copy kernel over MIB MiB (for "
                         "scaling rocprofv3 FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only (no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # plain elementwise kernel: reads n, writes n
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_each_way": n * 8, "copies": 3}))
        return

    torch.cuda.set_device(torch.device("cuda:0"))
    r = run_config(args.config, args, torch)
    wl = r.pop("wl")
    line = {
        "metric": "MSD Wick evals/s (walker*det/s), FP64 form; mixed form in 'mixed'",
        "value": r.pop("value"),
        "unit": "walker*det/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": f"synthetic (seeded {wl.name} system; no molecular integrals)",
        "config": {"workload": WORKLOADS[args.config], "global_batch": wl.n_walkers,
                   "n_det": wl.n_det, "parallelism": "none"},
        "roofline": r.pop("roofline"),
        "roofline_next": r.pop("roofline_next"),
        **r,
        "stage_timing_note": "stages_ms (average per timed launch group; some groups run once "
                             "per spin or per walker tile) and roofline from a second pass of "
                             "the same steps with HIP events around every stage (no graphs)",
    }
    if args.config != "medium" and not args.no_secondary:
        m = run_config("medium", args, torch, stages=False, block=False)
        m.pop("wl")
        line["secondary"] = {"medium": {"workload": WORKLOADS["medium"], **m},
                             "uneven_batch": run_uneven(args, torch)}
    if not args.no_cpu_baseline:
        n_det = 120 if args.config in ("cu_oxo", "fe2s2") else None
        n_walk = 2 if args.config in ("cu_oxo", "fe2s2") else 24
        line["cpu_baseline"] = cpu_baseline(wl, n_walk=n_walk, n_det=n_det)
        if args.config in ("cu_oxo", "fe2s2"):
            line["cpu_wick"] = cpu_wick(wl, n_walk=2 if args.config == "cu_oxo" else 1)
    print(json.dumps(line), flush=True)


def _tmax(pa, na, pb, nb):
    """Largest |T_pj| per walker over both spins, T = Phi Phi[R, :]^-1 with the
    reference R = the first N orbitals."""
    out = np.zeros(pa.shape[0])
    for w in range(pa.shape[0]):
        for phi, n in ((pa[w], na), (pb[w], nb)):
            if n:
                t = np.linalg.solve(phi[:n].T, phi.T).T
                out[w] = max(out[w], np.abs(t).max())
    return out


def _tables(wl):
    """Window sizes, distinct strings per order and distinct opposite-spin
    (particle, hole) pairs of the trial, from its occupation lists."""
    out = {"nv": [], "no": [], "strings": []}
    rows = set()
    exc = []
    for occ in (wl.occ_a, wl.occ_b):
        ref = set(occ[0].tolist())
        holes, parts = set(), set()
        strings = set()
        per_det = []
        for row in occ:
            r = set(row.tolist())
            h, p = tuple(sorted(ref - r)), tuple(sorted(r - ref))
            holes |= set(h)
            parts |= set(p)
            strings.add((h, p))
            per_det.append((h, p))
        out["nv"].append(len(parts))
        out["no"].append(len(holes))
        counts = {}
        for h, _ in strings:
            if len(h) >= 2:
                counts[len(h)] = counts.get(len(h), 0) + 1
        out["strings"].append(counts)
        rows |= ref | parts
        exc.append(per_det)
    pairs = set()
    for (ha, pa), (hb, pb) in zip(*exc):
        if ha and hb:
            xa = [(q, h) for q in pa for h in ha]
            xb = [(q, h) for q in pb for h in hb]
            pairs.update((x, y) for x in xa for y in xb)
    out["n_pair"] = len(pairs)
    out["P_all"] = len(rows)
    return out


if __name__ == "__main__":
    main()

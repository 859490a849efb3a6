"""Python binding of the MSD-AFQMC HIP library: argument marshalling only.

Host inputs are NumPy arrays (complex128 / float64 / int32, C order); device
inputs are any objects with ``data_ptr()`` (e.g. torch tensors on the GPU),
passed to the ``*_dev`` entry points.  Every computation happens in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib


class MsdError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.name = _lib.STATUS.get(status, str(status))
        super().__init__(f"{self.name}: {message}")


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class MsdSystem:
    """One walker batch on one device (see include/msd_afqmc.h)."""

    def __init__(self, M: int, n_alpha: int, n_beta: int, n_chol: int, n_walkers: int,
                 n_det: int, device: int = 0, stream: Optional[int] = None,
                 n_taylor: int = 6, stabilize_freq: int = 5, timing: bool = False,
                 energy_algo: int = 0, graphs: bool = False, precision: str = "fp64",
                 mixed_tmax: float = 0.0):
        self.lib = _lib.load()
        self.dims = _lib.MsdDims(M, n_alpha, n_beta, n_chol, n_walkers, 0, n_det)
        opts = _lib.MsdOptions()
        self.lib.msd_default_options(C.byref(opts))
        opts.n_taylor = n_taylor
        opts.stabilize_freq = stabilize_freq
        opts.timing = 1 if timing else 0
        opts.energy_algo = int(energy_algo)
        opts.graphs = 1 if graphs else 0
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        opts.precision = 1 if precision == "mixed" else 0
        opts.mixed_tmax = float(mixed_tmax)
        self.M, self.na, self.nb, self.ng, self.nw, self.nd = (
            M, n_alpha, n_beta, n_chol, n_walkers, n_det)
        h = C.c_void_p()
        st = self.lib.msd_create(C.byref(self.dims), C.byref(opts), device,
                                 C.c_void_p(stream) if stream else None, C.byref(h))
        if st != 0:
            msg = self.lib.msd_last_error(None) or b""
            raise MsdError(st, msg.decode())
        self.h = h

    # -- plumbing -----------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            msg = self.lib.msd_last_error(self.h) or b""
            raise MsdError(st, msg.decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.msd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inputs ---------------------------------------------------------------
    def set_hamiltonian(self, h1, chol, e0: float = 0.0):
        h1 = _host(h1, np.float64)
        chol = _host(chol, np.float64)
        self._check(self.lib.msd_set_hamiltonian(self.h, _ptr(h1), _ptr(chol), float(e0)))

    def set_trial(self, ci, occ_a, occ_b):
        ci = _host(ci, np.complex128)
        oa = _host(occ_a, np.int32)
        ob = _host(occ_b, np.int32)
        self._check(self.lib.msd_set_trial_occ(self.h, _ptr(ci), _ptr(oa), _ptr(ob)))

    def set_trial_exc(self, ref_a, ref_b, ci, k_a, k_b, offsets, holes, parts):
        """Trial as excitation lists (see msd_set_trial_exc)."""
        ra = _host(ref_a, np.int32)
        rb = _host(ref_b, np.int32)
        ci = _host(ci, np.complex128)
        ka = _host(k_a, np.int32)
        kb = _host(k_b, np.int32)
        off = _host(offsets, np.int64)
        h = _host(holes, np.int32)
        p = _host(parts, np.int32)
        self._check(self.lib.msd_set_trial_exc(self.h, _ptr(ra), _ptr(rb), int(ci.shape[0]),
                                               _ptr(ci), _ptr(ka), _ptr(kb), _ptr(off), _ptr(h),
                                               _ptr(p)))

    def set_walkers(self, phi_a, phi_b, weights=None):
        pa = _host(phi_a, np.complex128)
        pb = _host(phi_b, np.complex128)
        w = None if weights is None else _host(weights, np.float64)
        self._check(self.lib.msd_set_walkers(self.h, _ptr(pa), _ptr(pb), _ptr(w)))

    def set_walkers_dev(self, phi_a, phi_b, weights=None):
        self._check(self.lib.msd_set_walkers_dev(self.h, _ptr(phi_a), _ptr(phi_b),
                                                 _ptr(weights)))

    # -- outputs --------------------------------------------------------------
    def get_walkers(self):
        pa = np.empty((self.nw, self.M, self.na), np.complex128)
        pb = np.empty((self.nw, self.M, self.nb), np.complex128)
        w = np.empty(self.nw, np.float64)
        lo = np.empty(self.nw, np.complex128)
        self._check(self.lib.msd_get_walkers(self.h, _ptr(pa), _ptr(pb), _ptr(w), _ptr(lo)))
        return pa, pb, w, lo

    def get_weights(self):
        w = np.empty(self.nw, np.float64)
        lo = np.empty(self.nw, np.complex128)
        self._check(self.lib.msd_get_weights(self.h, _ptr(w), _ptr(lo)))
        return w, lo

    def measure(self, dt: float, energy: bool = True, force_bias: bool = True):
        lo = np.empty(self.nw, np.complex128)
        fb = np.empty((self.nw, self.ng), np.complex128) if force_bias else None
        el = np.empty(self.nw, np.complex128) if energy else None
        self._check(self.lib.msd_measure(self.h, float(dt), _ptr(lo), _ptr(fb), _ptr(el)))
        out = dict(log_ovlp=lo)
        if force_bias:
            out["force_bias"] = fb
        if energy:
            out["e_loc"] = el
        return out

    def measure_dev(self, dt: float, log_ovlp=None, force_bias=None, e_loc=None):
        self._check(self.lib.msd_measure_dev(self.h, float(dt), _ptr(log_ovlp),
                                             _ptr(force_bias), _ptr(e_loc)))

    def propagate(self, fields, dt: float, e_shift: float = 0.0):
        f = _host(fields, np.float64)
        if f.ndim == 2:
            f = f[None]
        self._check(self.lib.msd_propagate(self.h, _ptr(f), float(dt), float(e_shift),
                                           int(f.shape[0])))

    def propagate_dev(self, fields, dt: float, e_shift: float = 0.0, n_steps: int = 1):
        self._check(self.lib.msd_propagate_dev(self.h, _ptr(fields), float(dt), float(e_shift),
                                               int(n_steps)))

    def population_control(self, z: float):
        """Comb population control; returns the parent of every new walker."""
        parent = np.empty(self.nw, np.int32)
        self._check(self.lib.msd_population_control(self.h, float(z), _ptr(parent)))
        return parent

    def population_control_dev(self, z: float, parent=None):
        self._check(self.lib.msd_population_control_dev(self.h, float(z), _ptr(parent)))

    def population_control_noalloc(self, z: float, parent=None):
        """As population_control_dev, with the library's static scratch (no
        allocation; see msd_population_control_noalloc)."""
        self._check(self.lib.msd_population_control_noalloc(self.h, float(z), _ptr(parent)))

    def run_block(self, fields_dev, n_steps: int, dt: float, e_shift: float = 0.0,
                  pop_freq: int = 5, z=()):
        """One block; returns (sum_w w E_L as complex, sum_w w)."""
        zz = _host(np.asarray(z, dtype=np.float64).reshape(-1), np.float64)
        e = np.zeros(3, np.float64)
        self._check(self.lib.msd_run_block(self.h, _ptr(fields_dev), float(dt), float(e_shift),
                                           int(n_steps), int(pop_freq),
                                           _ptr(zz) if zz.size else None, _ptr(e)))
        return complex(e[0], e[1]), float(e[2])

    def get_green(self, walker: int):
        ga = np.empty((self.M, self.M), np.complex128)
        gb = np.empty((self.M, self.M), np.complex128)
        self._check(self.lib.msd_get_green(self.h, int(walker), _ptr(ga), _ptr(gb)))
        return ga, gb

    def get_measurement(self, force_bias: bool = True):
        """Host copies of the most recent measurement."""
        lo = np.empty(self.nw, np.complex128)
        fb = np.empty((self.nw, self.ng), np.complex128) if force_bias else None
        el = np.empty(self.nw, np.complex128)
        self._check(self.lib.msd_get_measurement(self.h, _ptr(lo), _ptr(fb), _ptr(el)))
        out = dict(log_ovlp=lo, e_loc=el)
        if force_bias:
            out["force_bias"] = fb
        return out

    _TUNING = ("fb_splitk", "lambda_variant", "lambda_chunk", "second_gsplit", "second_stage",
               "second_gather", "second_copy", "second_waves", "walker_tile", "energy_form",
               "second_whole")

    def get_tuning(self):
        t = _lib.MsdTuning()
        self._check(self.lib.msd_get_tuning(self.h, C.byref(t)))
        return {k: getattr(t, k) for k in self._TUNING}

    def set_tuning(self, **kw):
        """Launch-shape overrides (0 = automatic); see msd_tuning."""
        t = _lib.MsdTuning()
        for k, v in kw.items():
            if k not in self._TUNING or k == "energy_form":
                raise ValueError(f"unknown or read-only tuning field {k}")
            setattr(t, k, int(v))
        self._check(self.lib.msd_set_tuning(self.h, C.byref(t)))

    def autotune(self, dt: float, reps: int = 3):
        t = _lib.MsdTuning()
        self._check(self.lib.msd_autotune(self.h, float(dt), int(reps), C.byref(t)))
        return {k: getattr(t, k) for k in self._TUNING}

    def timings(self):
        n = 64
        names = (C.c_char_p * n)()
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        k = C.c_int32()
        self._check(self.lib.msd_get_timings(self.h, n, names, ms, cnt, C.byref(k)))
        return {names[i].decode(): (ms[i], cnt[i]) for i in range(k.value)}

    def reset_timings(self):
        self._check(self.lib.msd_reset_timings(self.h))


class MsdBatch:
    """Several MsdSystem handles stepped together, one HIP graph per step
    (see msd_batch_step)."""

    def __init__(self, systems, stream: Optional[int] = None):
        self.lib = _lib.load()
        self.systems = list(systems)  # keeps the handles alive
        arr = (C.c_void_p * len(self.systems))(*[s.h.value for s in self.systems])
        h = C.c_void_p()
        st = self.lib.msd_batch_create(arr, len(self.systems),
                                       C.c_void_p(stream) if stream else None, C.byref(h))
        if st != 0:
            raise MsdError(st, (self.lib.msd_last_error(None) or b"").decode())
        self.h = h

    def step(self, fields, dt: float, e_shift: float = 0.0, measure: bool = True):
        """fields: one device array per system ([n_walkers][n_chol] float64)."""
        if len(fields) != len(self.systems):
            raise ValueError("one field array per system")
        arr = (C.c_void_p * len(fields))(*[f.data_ptr() for f in fields])
        st = self.lib.msd_batch_step(self.h, arr, float(dt), float(e_shift), 1 if measure else 0)
        if st != 0:
            raise MsdError(st, (self.lib.msd_last_error(None) or b"").decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.msd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trial_analyze(M: int, occ_a, occ_b):
    """Excitation orders and signs per determinant (host-only library call)."""
    lib = _lib.load()
    oa = _host(occ_a, np.int32)
    ob = _host(occ_b, np.int32)
    nd = oa.shape[0]
    ka = np.empty(nd, np.int32)
    kb = np.empty(nd, np.int32)
    sg = np.empty(nd, np.int32)
    st = lib.msd_trial_analyze(M, oa.shape[1], ob.shape[1], nd, _ptr(oa), _ptr(ob), _ptr(ka),
                               _ptr(kb), _ptr(sg))
    if st != 0:
        raise MsdError(st, (lib.msd_last_error(None) or b"").decode())
    return ka, kb, sg

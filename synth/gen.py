"""Seeded generators for transition-metal-cluster-shaped MSD-AFQMC inputs.

Every array is drawn from ``numpy.random.default_rng(seed)``.  The recipe:

* Cholesky vectors L^g = (A + A^T) / (2 sqrt(M)), A ~ N(0, 1), real symmetric.
* One-body h = diag(linspace(-2, 2, M)) + 0.1 (B + B^T) / (2 sqrt(M)); E0 = 0.
* Reference occupations R = {0, ..., N-1} per spin.
* Excitation window: the top ``n_occ_act`` occupied and the bottom
  ``n_vir_act`` virtual orbitals of each spin.
* Determinants: total order k uniform in 1..k_max, k_alpha uniform in 0..k
  (redrawn when a spin's order exceeds its window), holes and particles
  uniform without replacement, duplicates rejected.  Det 0 is the reference.
* CI magnitudes by rank r (dets sorted by (order, random)), random sign,
  normalised to sum |c|^2 = 1.
* Walkers: orthonormal columns spanning a 0.1-Gaussian-perturbed reference,
  complex.
* Auxiliary fields: x ~ N(0, 1) per walker and Cholesky vector, one draw per
  step (seed + 1000 + step).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

BASE_SEED = 240608314


@dataclass
class Workload:
    name: str
    M: int
    n_alpha: int
    n_beta: int
    n_chol: int
    n_det: int
    n_walkers: int
    h1: np.ndarray          # (M, M) float64, real symmetric
    chol: np.ndarray        # (n_chol, M, M) float64, each real symmetric
    e0: float
    ci: np.ndarray          # (n_det,) complex128
    occ_a: np.ndarray       # (n_det, n_alpha) int32, ascending per row
    occ_b: np.ndarray       # (n_det, n_beta) int32
    phi_a: np.ndarray       # (n_walkers, M, n_alpha) complex128
    phi_b: np.ndarray       # (n_walkers, M, n_beta) complex128
    weights: np.ndarray     # (n_walkers,) float64
    dt: float = 0.005
    seed: int = BASE_SEED
    meta: dict = field(default_factory=dict)


# Named configurations (shapes of the paper's workloads, scaled to stand-ins).
CONFIGS = {
    "tiny": dict(M=12, n_alpha=3, n_beta=3, n_chol=48, n_det=20, k_max=2,
                 window=(3, 9), c_law="gauss_exp0.25", n_walkers=8, index=0),
    "medium": dict(M=64, n_alpha=8, n_beta=8, n_chol=320, n_det=1000, k_max=4,
                   window=(8, 56), c_law="exp0.5", n_walkers=128, index=1),
    "cu_oxo": dict(M=200, n_alpha=30, n_beta=30, n_chol=1200, n_det=10000,
                   k_max=4, window=(16, 32), c_law="power1", n_walkers=256,
                   index=2),
    "fe2s2": dict(M=300, n_alpha=45, n_beta=45, n_chol=2000, n_det=200000,
                  k_max=6, window=(15, 5), c_law="power1", n_walkers=512,
                  index=3),
}


def _symmetric(rng, n_mat, M):
    a = rng.standard_normal((n_mat, M, M))
    return (a + np.transpose(a, (0, 2, 1))) / (2.0 * np.sqrt(M))


def _draw_string_masks(rng, n, N, M, k, n_occ_act, n_vir_act):
    """Occupancy masks (n, M) for strings with k[i] holes/particles each."""
    masks = np.zeros((n, M), dtype=bool)
    masks[:, :N] = True
    if n == 0:
        return masks
    occ_act = np.arange(N - n_occ_act, N)
    vir_act = np.arange(N, N + n_vir_act)
    kmax = int(k.max()) if k.size else 0
    if kmax == 0:
        return masks
    hole_order = np.argsort(rng.random((n, n_occ_act)), axis=1)[:, :kmax]
    part_order = np.argsort(rng.random((n, n_vir_act)), axis=1)[:, :kmax]
    rows = np.arange(n)
    for j in range(kmax):
        sel = k > j
        masks[rows[sel], occ_act[hole_order[sel, j]]] = False
        masks[rows[sel], vir_act[part_order[sel, j]]] = True
    return masks


def _ci_magnitudes(rng, law, n):
    r = np.arange(n, dtype=np.float64)
    if law == "gauss_exp0.25":
        return rng.standard_normal(n) * np.exp(-0.25 * r)
    if law == "exp0.5":
        return np.exp(-0.5 * r) * rng.choice([-1.0, 1.0], size=n)
    if law == "flat":
        return rng.choice([-1.0, 1.0], size=n)
    if law == "power1":
        return (1.0 + r) ** -1.0 * rng.choice([-1.0, 1.0], size=n)
    raise ValueError(f"unknown CI law {law!r}")


def _masks_to_occ(masks, N):
    M = masks.shape[1]
    idx = np.where(masks, np.arange(M)[None, :], M)
    return np.sort(idx, axis=1)[:, :N].astype(np.int32)


def _draw_dets(rng, M, na, nb, n_det, k_max, window):
    no_act, nv_act = window
    kmax_a = min(no_act, nv_act, na, M - na)
    kmax_b = min(no_act, nv_act, nb, M - nb)
    ref = np.zeros((1, M), dtype=bool)
    ma_all = [np.concatenate([np.ones((1, na), bool), np.zeros((1, M - na), bool)], 1)]
    mb_all = [np.concatenate([np.ones((1, nb), bool), np.zeros((1, M - nb), bool)], 1)]
    order_all = [np.zeros(1, dtype=np.int64)]
    del ref
    seen = set()
    key0 = np.concatenate([ma_all[0], mb_all[0]], 1)
    seen.add(np.packbits(key0, axis=1).tobytes())
    have = 1
    tries = 0
    while have < n_det:
        tries += 1
        if tries > 200:
            raise ValueError("could not draw enough distinct determinants")
        batch = max(64, 2 * (n_det - have))
        k = rng.integers(1, k_max + 1, size=batch)
        ka = (rng.random(batch) * (k + 1)).astype(np.int64)
        kb = k - ka
        ok = (ka <= kmax_a) & (kb <= kmax_b)
        k, ka, kb = k[ok], ka[ok], kb[ok]
        ma = _draw_string_masks(rng, ka.size, na, M, ka, no_act, nv_act)
        mb = _draw_string_masks(rng, kb.size, nb, M, kb, no_act, nv_act)
        keys = np.packbits(np.concatenate([ma, mb], 1), axis=1)
        for i in range(k.size):
            kb_ = keys[i].tobytes()
            if kb_ in seen:
                continue
            seen.add(kb_)
            ma_all.append(ma[i:i + 1])
            mb_all.append(mb[i:i + 1])
            order_all.append(k[i:i + 1])
            have += 1
            if have == n_det:
                break
    ma = np.concatenate(ma_all, 0)
    mb = np.concatenate(mb_all, 0)
    order = np.concatenate(order_all, 0)
    # rank: reference first, then by (order, random)
    tiebreak = rng.random(n_det)
    tiebreak[0] = -1.0
    perm = np.lexsort((tiebreak, order))
    return _masks_to_occ(ma[perm], na), _masks_to_occ(mb[perm], nb), order[perm]


def _walkers(rng, n_walkers, M, N, noise):
    base = np.zeros((M, N), dtype=np.complex128)
    base[np.arange(N), np.arange(N)] = 1.0
    out = np.empty((n_walkers, M, N), dtype=np.complex128)
    for w in range(n_walkers):
        a = base + noise * (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N)))
        q, _ = np.linalg.qr(a)
        out[w] = q
    return out


def make_workload(name: str, M: int, n_alpha: int, n_beta: int, n_chol: int,
                  n_det: int, k_max: int, window, c_law: str, n_walkers: int,
                  seed: int, complex_ci: bool = False, noise: float = 0.1,
                  dt: float = 0.005) -> Workload:
    """Draw one synthetic system: Hamiltonian, CI trial, walkers."""
    rng = np.random.default_rng(seed)
    chol = _symmetric(rng, n_chol, M)
    b = _symmetric(rng, 1, M)[0]
    h1 = np.diag(np.linspace(-2.0, 2.0, M)) + 0.1 * b
    occ_a, occ_b, order = _draw_dets(rng, M, n_alpha, n_beta, n_det, k_max, window)
    mag = _ci_magnitudes(rng, c_law, n_det)
    if complex_ci:
        ci = mag * np.exp(1j * rng.uniform(0, 2 * np.pi, n_det))
    else:
        ci = mag.astype(np.complex128)
    ci = ci / np.linalg.norm(ci)
    phi_a = _walkers(rng, n_walkers, M, n_alpha, noise)
    phi_b = _walkers(rng, n_walkers, M, n_beta, noise)
    return Workload(name=name, M=M, n_alpha=n_alpha, n_beta=n_beta,
                    n_chol=n_chol, n_det=n_det, n_walkers=n_walkers,
                    h1=h1, chol=chol, e0=0.0, ci=ci, occ_a=occ_a, occ_b=occ_b,
                    phi_a=phi_a, phi_b=phi_b,
                    weights=np.ones(n_walkers), dt=dt, seed=seed,
                    meta=dict(k_max=k_max, window=tuple(window), c_law=c_law,
                              order=order))


def make_config(name: str, n_det: Optional[int] = None,
                n_walkers: Optional[int] = None, c_law: Optional[str] = None,
                complex_ci: bool = False) -> Workload:
    """One of the named configurations (optionally truncated)."""
    p = dict(CONFIGS[name])
    idx = p.pop("index")
    if n_det is not None:
        p["n_det"] = n_det
    if n_walkers is not None:
        p["n_walkers"] = n_walkers
    if c_law is not None:
        p["c_law"] = c_law
    return make_workload(name=name, seed=BASE_SEED + idx, complex_ci=complex_ci, **p)


def fields_for_step(wl: Workload, step: int) -> np.ndarray:
    """Auxiliary fields x ~ N(0,1), shape (n_walkers, n_chol), for one step."""
    rng = np.random.default_rng(wl.seed + 1000 + step)
    return rng.standard_normal((wl.n_walkers, wl.n_chol))


def make_uneven(n_systems: int = 32, M_range=(32, 200), N_max: int = 30,
                n_det_range=(100, 100_000), walker_range=(64, 512),
                seed: int = BASE_SEED + 4) -> list:
    """A batch of independent systems of uneven size: M uniform in M_range,
    N_alpha = N_beta uniform in [4, min(N_max, M/2)], n_chol = 5 M, n_det
    log-uniform in n_det_range with total excitation order <= 4, window
    min(N, 16) x min(M - N, 32), |c| ~ (1 + rank)^-1, walkers uniform in
    walker_range.  System i is drawn with seed + 1 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_systems):
        M = int(rng.integers(M_range[0], M_range[1] + 1))
        N = int(rng.integers(min(4, M // 2), min(N_max, M // 2) + 1))
        lo, hi = np.log(n_det_range[0]), np.log(n_det_range[1])
        nd = int(round(np.exp(rng.uniform(lo, hi))))
        nw = int(rng.integers(walker_range[0], walker_range[1] + 1))
        window = (min(N, 16), min(M - N, 32))
        out.append(make_workload(name=f"uneven{i}", M=M, n_alpha=N, n_beta=N, n_chol=5 * M,
                                 n_det=nd, k_max=4, window=window, c_law="power1",
                                 n_walkers=nw, seed=seed + 1 + i))
    return out

"""CPU oracle for the MSD-AFQMC hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, complex128 NumPy/SciPy code that computes what the GPU path
computes, straight from the definitions in the paper (Sec. II: Eqs. 3-15).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code with the HIP library and never
imports it.

Modules
-------
msd        trial overlaps, mixed Green's function, force bias, local energy
           by brute force over determinants (Eqs. 6-7, 13-15).
wick       the same quantities one determinant at a time relative to the
           reference (generalised Wick, Sec. III / App. A), for the large
           shapes; its Cholesky-vector sums are plain C (wick_gamma.c).
propagate  one phaseless step: VHS, Taylor exp(VHS), one-body half steps,
           weight update, QR re-orthonormalisation (Eqs. 4-5, 8-12).
driver     the block around the step: comb population control, weighted
           block energy (Sec. III.B, Listing 1).
fock       explicit second-quantised (Jordan-Wigner) Fock-space objects for
           tiny systems; used only to pin the modules above.
"""
from . import msd, propagate, driver, fock, wick  # noqa: F401

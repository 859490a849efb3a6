"""MI355X (gfx950) MSD-AFQMC hot path: generalised-Wick trial overlaps, Green's
functions, force biases, local energies and the Cholesky propagation step, as
hand-written HIP kernels behind a C ABI (include/msd_afqmc.h)."""
from .api import MsdBatch, MsdError, MsdSystem, trial_analyze  # noqa: F401

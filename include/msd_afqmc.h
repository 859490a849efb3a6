/*
 * msd_afqmc.h -- C ABI of the MI355X (gfx950) MSD-AFQMC hot-path library.
 *
 * The library evaluates, for a batch of walkers (each one Slater determinant
 * per spin), the quantities of phaseless AFQMC with a multi-Slater-determinant
 * (CI-expansion) trial:
 *   - the trial overlap <Psi_T|Phi>               (Sec. II.A Eq. 13, Eq. 15)
 *   - the mixed Green's function                  (Eq. 14)
 *   - the force bias xbar                         (Eq. 7)
 *   - the mixed local energy                      (Sec. II.A, generalised Wick)
 * through the generalised Wick theorem relative to a reference determinant
 * (Sec. III), and one propagation step                   (Eqs. 3-5, 8-12)
 *   - VHS = i sqrt(dt) sum_g (x_g - xbar_g) L^g, Phi <- B1 exp_T(VHS) B1 Phi
 *     with B1 = expm(-dt h'/2), h' = h - 1/2 sum_g L^g L^g (Eq. 4),
 *   - new overlaps, phaseless weights, periodic re-orthonormalisation (QR).
 *
 * Conventions
 *   Complex numbers are passed as interleaved (re, im) pairs of doubles.
 *   All arrays are row-major (C order), densely packed.
 *   Trial: c_I multiplies the determinant whose alpha and beta orbital sets
 *   are the rows of occ_a / occ_b, each set in ascending order, alpha
 *   creation operators before beta.  <Psi_T| carries conj(c_I).  Row 0 is the
 *   reference determinant of the Wick expansion; every other row is an
 *   excitation of it.  Rows are treated as sets (any order on input).
 *   Hamiltonian: H = E0 + sum h_pq E_pq + 1/2 sum (pq|rs) a+_p a+_r a_s a_q
 *   with (pq|rs) = sum_g L^g_pq L^g_rs; h and every L^g real symmetric.
 *   Green's function G^s_pq = <Psi_T|a+_ps a_qs|Phi>/<Psi_T|Phi>.
 *   Force bias xbar_g = -i sqrt(dt) sum_s sum_pq L^g_pq G^s_pq.
 *   Weight update: S = <Psi_T|Phi'>/<Psi_T|Phi>,
 *     w <- w |S exp(x.xbar - xbar.xbar/2)| max(0, cos arg S) exp(dt e_shift)
 *   (bilinear dot products).  A walker of weight 0 is frozen (not moved).
 *
 * Ownership and errors
 *   Inputs are caller-owned and copied before the call returns; outputs go to
 *   caller buffers.  No pointer is retained.  Every call returns msd_status
 *   (0 = success); no C++ exception crosses the ABI.  msd_last_error() gives
 *   a message naming the offending index.  A handle is bound to one device
 *   and one HIP stream; calls on one handle must not overlap.  "_dev" entry
 *   points take device pointers and are stream-ordered on the handle's
 *   stream (they return once the work is enqueued, except where noted).
 */
#ifndef MSD_AFQMC_H
#define MSD_AFQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MSD_OK = 0,
  MSD_ERR_ARG = -1,         /* null pointer, non-finite value, bad option    */
  MSD_ERR_SHAPE = -2,       /* inconsistent dimensions                        */
  MSD_ERR_TRIAL = -3,       /* invalid occupation lists / excitations         */
  MSD_ERR_SINGULAR = -4,    /* walker with zero overlap with the reference    */
  MSD_ERR_DEVICE = -5,      /* HIP runtime error                              */
  MSD_ERR_OOM = -6,         /* device allocation failed / plan too large      */
  MSD_ERR_STATE = -7,       /* call order (e.g. measure before set_trial)     */
  MSD_ERR_UNSUPPORTED = -8  /* shape outside what the kernels implement       */
} msd_status;

typedef struct msd_system msd_system;

/* Problem sizes.  M spatial orbitals, n_alpha/n_beta electrons, n_chol
 * Cholesky vectors, n_walkers walkers, n_det determinants in the trial. */
typedef struct {
  int32_t M;
  int32_t n_alpha;
  int32_t n_beta;
  int32_t n_chol;
  int32_t n_walkers;
  int32_t reserved;
  int64_t n_det;
} msd_dims;

typedef struct {
  int32_t n_taylor;       /* Taylor order of exp(VHS) (terms 0..n_taylor), default 6 */
  int32_t stabilize_freq; /* QR every this many propagate steps (0 = never), default 5 */
  int32_t timing;         /* 1: record HIP events around every kernel stage   */
  int32_t energy_algo;    /* second-order energy terms: 0 = automatic (the W-form where
                             its matrix-core GEMMs cost less than the direct form, else
                             per spin the direct form with fewest gathers), 1 = direct,
                             per-minor lists, 2 = direct, per-string; 3 = as 0 without
                             the W-form, with the fused Cholesky contraction (GEMM tile
                             consumed in LDS) where its tile fits; 4 = W-form:
                             W^{st} = sum_g Lambda^{s,g} (x) Lambda^{t,g} per walker by
                             matrix-core GEMMs over the Cholesky index, contracted with
                             the pair and minor coefficient lists (memory bounded by the
                             excitation window, independent of n_det)                 */
  int32_t graphs;         /* 1: record each measure / propagate step once as a HIP graph
                             (on a private stream) and replay it on the handle's stream;
                             ignored while timing is on.  Default 0                  */
  int32_t precision;      /* 0 = FP64 throughout (default).  1 = mixed form: the dense
                             Cholesky contractions (force bias, LT = L T, VHS) run as
                             FP32 MFMA GEMMs, the energy intermediates Lambda and the
                             Cholesky-vector sums of the second-order energy terms in
                             FP32; the reference inverse, k x k determinants and
                             cofactors, Taylor propagator, QR, overlaps and weights
                             stay FP64.  Walkers far from the reference get FP64
                             energies (see mixed_tmax).  Trials with excitation orders
                             above 6 per spin are evaluated in FP64 unless the W-form
                             applies (see energy_algo); so are all energies at 33-48
                             electrons per spin where T does not fit the LDS in FP64
                             (there the FP64 pass for far walkers would cost more than
                             the FP64 energy path).                                   */
  double mixed_tmax;      /* mixed form with the general contraction kernel: a walker
                             whose largest |T_pj| (T = Phi A^{-1}, the ratios of its
                             single-excitation overlaps to the reference overlap, Sec.
                             III) exceeds this gets its local energy from the FP64
                             energy kernels (the FP32 rounding of the Wick intermediates
                             grows with |T|^2).  0 = default 2.0; negative = never.   */
} msd_options;

/* Limits of this implementation. */
#define MSD_MAX_ELECTRONS 64    /* per spin (reference inverse and QR in LDS)  */
#define MSD_MAX_EXCITATION 8    /* holes per spin per determinant             */

const char* msd_status_string(msd_status s);
const char* msd_last_error(const msd_system* sys);

/* Fill *o with the defaults (n_taylor 6, stabilize_freq 5, timing 0). */
msd_status msd_default_options(msd_options* o);

/* Create a handle on HIP device `device`; `hip_stream` is a hipStream_t (NULL:
 * the default stream).  Allocates the walker state for d->n_walkers walkers.
 * MSD_ERR_SHAPE for non-positive sizes or n_alpha/n_beta > M or above
 * MSD_MAX_ELECTRONS; MSD_ERR_DEVICE / MSD_ERR_OOM from the runtime. */
msd_status msd_create(const msd_dims* d, const msd_options* o, int32_t device,
                      void* hip_stream, msd_system** out);
void msd_destroy(msd_system* sys);

/* Hamiltonian (Sec. II.A: Eq. 2 one-body h and E0, Eq. 3 Cholesky vectors,
 * Eq. 4 h' for the propagator).  h1: M*M doubles.  chol: n_chol*M*M doubles, row
 * g*M*M + p*M + q = L^g_pq.  Both must be symmetric to 1e-12 (MSD_ERR_ARG
 * names the first offending index otherwise).  Precomputes h' and the
 * one-body half-step factor for the time step passed to msd_propagate. */
msd_status msd_set_hamiltonian(msd_system* sys, const double* h1, const double* chol,
                               double e0);

/* Trial (Eq. 15).  ci: n_det complex (2*n_det doubles).  occ_a: n_det*n_alpha
 * int32, occ_b: n_det*n_beta int32.  Row 0 is the Wick reference.
 * MSD_ERR_TRIAL for an orbital outside [0, M), a repeated orbital in a row,
 * or more than MSD_MAX_EXCITATION holes per spin.  Duplicate rows are allowed
 * (their coefficients add). */
msd_status msd_set_trial_occ(msd_system* sys, const double* ci, const int32_t* occ_a,
                             const int32_t* occ_b);

/* Trial as excitations of a reference (Sec. II.B, Eq. 15), same meaning as
 * msd_set_trial_occ.  ref_a: n_alpha int32, ref_b: n_beta int32 (the reference
 * determinant's orbitals).  Determinant I has k_a[I] alpha and k_b[I] beta
 * holes: holes[offsets[I] + m] / parts[offsets[I] + m] for m < k_a[I] are its
 * alpha hole/particle orbitals, the next k_b[I] entries its beta ones; pairing
 * of holes with particles is irrelevant (the determinant is the orbital set
 * reference - holes + particles, in ascending order, as in msd_set_trial_occ).
 * offsets: n_det + 1 int64, offsets[0] = 0, offsets[I+1] - offsets[I] =
 * k_a[I] + k_b[I].  ci: n_det complex.  n_det must equal the handle's n_det
 * (MSD_ERR_SHAPE).  MSD_ERR_TRIAL for a hole outside the reference, a
 * particle inside it, a repeat, or inconsistent offsets. */
msd_status msd_set_trial_exc(msd_system* sys, const int32_t* ref_a, const int32_t* ref_b,
                             int64_t n_det, const double* ci, const int32_t* k_a,
                             const int32_t* k_b, const int64_t* offsets, const int32_t* holes,
                             const int32_t* parts);

/* Walkers (host arrays): the walker state of the weighted-walker expansion
 * of the ground state (Eq. 6, Sec. II.A): for each walker w its Slater
 * determinant |Phi_w> (orbital coefficients per spin) and its weight.
 * phi_a: n_walkers*M*n_alpha complex, [w][p][j]; phi_b likewise with n_beta;
 * weights: n_walkers doubles (NULL: all 1).  Needs the trial (MSD_ERR_STATE
 * otherwise): computes log <Psi_T|Phi_w>.  MSD_ERR_SINGULAR if a walker has a
 * singular reference block. */
msd_status msd_set_walkers(msd_system* sys, const double* phi_a, const double* phi_b,
                           const double* weights);
/* Same with device pointers (same layouts); synchronises the stream. */
msd_status msd_set_walkers_dev(msd_system* sys, const double* phi_a, const double* phi_b,
                               const double* weights);
/* Copy the walker state out (any pointer may be NULL).  log_ovlp: n_walkers
 * complex, log <Psi_T|Phi_w> (imaginary part defined modulo 2 pi). */
msd_status msd_get_walkers(msd_system* sys, double* phi_a, double* phi_b, double* weights,
                           double* log_ovlp);

/* Weights and log <Psi_T|Phi_w> only (Eqs. 8-12 state); same as
 * msd_get_walkers with NULL orbitals. */
msd_status msd_get_weights(msd_system* sys, double* weights, double* log_ovlp);

/* Measurement (Eq. 13/15 overlap, Eq. 14 mixed Green's function, Eq. 7 force
 * bias, the mixed-estimator local energy of Sec. II.A evaluated by the
 * generalised Wick theorem of Sec. III) of every walker: log_ovlp (n_walkers complex), force_bias
 * (n_walkers*n_chol complex, [w][g], uses time step dt), e_loc (n_walkers
 * complex).  Any output may be NULL; the energy stages run only if e_loc is
 * non-NULL.  Host pointers; synchronises the stream. */
msd_status msd_measure(msd_system* sys, double dt, double* log_ovlp, double* force_bias,
                       double* e_loc);
/* Same with device output pointers; stream-ordered, does not synchronise.
 * No singularity check is made here: a walker with a singular reference block
 * or zero trial overlap gets log_ovlp = (-inf, 0) and non-finite G-derived
 * outputs. */
msd_status msd_measure_dev(msd_system* sys, double dt, double* log_ovlp, double* force_bias,
                           double* e_loc);

/* n_steps propagation steps (Eq. 5 with the first-order split, Eqs. 8-12
 * phaseless weights, periodic re-orthonormalisation as in Listing 1).  fields: n_steps*n_walkers*n_chol doubles,
 * standard-normal auxiliary fields, [step][w][g] (host).  Each step: force
 * bias, VHS, Taylor propagator with one-body half steps, new overlap,
 * phaseless weight update, and QR every stabilize_freq steps (counted over
 * the life of the handle).  Synchronises the stream. */
msd_status msd_propagate(msd_system* sys, const double* fields, double dt, double e_shift,
                         int32_t n_steps);
/* Same with fields in device memory; stream-ordered, does not synchronise. */
msd_status msd_propagate_dev(msd_system* sys, const double* fields, double dt,
                             double e_shift, int32_t n_steps);

/* Population control by the comb method (the simulation block of Sec. III.B
 * and Listing 1 runs it every 5 steps; the paper names no algorithm, the comb
 * is the reading taken).  With cumulative weights C_i = w_0 + ... + w_i and
 * total W, tooth k (k = 0 .. n_walkers-1) sits at t_k = (k + z) W / n_walkers;
 * walker k of the new population is a copy (orbitals and log overlap) of the
 * walker i with C_{i-1} <= t_k < C_i, and every new weight is W / n_walkers.
 * A walker of weight 0 is never copied.  z: the comb offset, a uniform random
 * number in [0, 1) drawn by the caller (MSD_ERR_ARG otherwise).  parent:
 * n_walkers int32 receiving i for every new walker k, host memory
 * (synchronises) or NULL.  If W = 0 nothing changes.  MSD_ERR_STATE without
 * walkers. */
msd_status msd_population_control(msd_system* sys, double z, int32_t* parent);
/* Same with parent a device pointer (or NULL); stream-ordered, does not
 * synchronise. */
msd_status msd_population_control_dev(msd_system* sys, double z, int32_t* parent);
/* Same as msd_population_control_dev, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): it calls no allocator.  Its scratch (running sums,
 * parents when parent is NULL, the parents' log overlaps and the gathered
 * walkers, n_walkers * (M * (n_alpha + n_beta) * 16 + 28) bytes, each part
 * rounded up to 256 bytes) lives in one static device array of 128 MiB per
 * GPU, held from the library's first msd_create on that GPU until the process
 * ends; MSD_ERR_UNSUPPORTED if the handle needs more.  The array is shared by
 * every handle on the GPU and keeps the last call's contents: calls that
 * overlap on one GPU (concurrent streams or threads) race.  Results are
 * identical to msd_population_control_dev. */
msd_status msd_population_control_noalloc(msd_system* sys, double z, int32_t* parent);

/* One simulation block (Sec. III.B, Listing 1): n_steps propagation steps as
 * msd_propagate_dev (QR on the handle's stabilize_freq schedule), population
 * control (msd_population_control) after every pop_freq-th step of the block
 * (0 = never) with offsets z[0], z[1], ... (n_steps / pop_freq host doubles in
 * [0, 1)), then one measurement with energies (as msd_measure; read it with
 * msd_get_measurement).  fields: device pointer, n_steps*n_walkers*n_chol
 * standard-normal fields, [step][w][g].  energy (host, 3 doubles) receives
 * Re and Im of sum_w w E_L(w) and sum_w w over walkers of positive weight:
 * the block's weighted mixed energy is their ratio.  Synchronises;
 * MSD_ERR_SINGULAR as msd_measure. */
msd_status msd_run_block(msd_system* sys, const double* fields, double dt, double e_shift,
                         int32_t n_steps, int32_t pop_freq, const double* z, double* energy);

/* Green's functions (Eq. 14) of one walker (M*M complex each, G_pq at [p][q]) from
 * the most recent measure or propagate evaluation. */
msd_status msd_get_green(msd_system* sys, int32_t walker, double* g_a, double* g_b);

/* Stage timings accumulated since the last reset (timing option on).
 * names: up to max_stages C strings owned by the library; ms: total
 * milliseconds; counts: launches.  *n_stages receives the number written. */
msd_status msd_get_timings(msd_system* sys, int32_t max_stages, const char** names,
                           double* ms, int64_t* counts, int32_t* n_stages);
msd_status msd_reset_timings(msd_system* sys);

/* Launch-shape tuning of one handle.  Every field 0 = the library's choice;
 * msd_get_tuning reports the values in use (after the first measurement with
 * energies, when the energy plan exists).  Changing them never changes
 * results beyond floating-point summation order. */
typedef struct {
  int32_t fb_splitk;      /* K slices of the force-bias GEMM (1..16)                      */
  int32_t lambda_variant; /* energy intermediates: 1 = two-wave rows kernel over the
                             L^g T tiles (N <= 32 per spin; the one-wave generic kernel
                             beyond its limits), 5 = matrix-core kernel forming
                             the Cholesky contraction L^g T, Lambda and the first-order
                             contraction itself, so L^g T never goes through HBM (both
                             spins N = 8 with the whole occupied window, at most 56
                             active virtuals, M <= 64), 6 = general matrix-core kernel
                             forming L^g T, Q, Lambda and the first-order contraction
                             for up to 48 electrons per spin, M <= 320 and windows of
                             at most 32 x 32 (the default where 5 does not apply,
                             except in the FP64 form at 33-48 electrons where T does
                             not fit the LDS: there 1 is faster for whole batches).  A
                             variant that does not fit the shape falls back to 1.
                             2-4 (earlier kernels no workload picked) are rejected    */
  int32_t lambda_chunk;   /* Cholesky vectors per intermediates workgroup (1..NG); the
                             fused kernel's workgroup holds four walkers x two spins   */
  int32_t second_gsplit;  /* Cholesky-range split of the second-order kernel (1..64)      */
  int32_t second_stage;   /* Cholesky vectors per LDS stage of the second-order kernel
                             (1..32, bounded by 150 KB of LDS)                             */
  int32_t second_gather;  /* second-order kernel reads its LDS stage with 1 = LDS
                             instructions, 2 = generic (flat) loads                       */
  int32_t second_copy;    /* second-order kernel fills its LDS stage 1 = through
                             registers, 2 = by direct global-to-LDS loads (where the
                             Lambda rows are 16-byte aligned; else through registers)   */
  int32_t second_waves;   /* waves per second-order workgroup: 8 or 16 (16 only where
                             no spin has excitations above order 4; else 8)             */
  int32_t walker_tile;    /* walkers per pass of the energy stages (1..n_walkers); small
                             tiles keep the LT and Lambda intermediates of a pass in the
                             last-level cache                                            */
  int32_t energy_form;    /* read-only (msd_get_tuning): 1 when the second-order terms
                             run in the W-form (see energy_algo), 0 for the direct form;
                             ignored by msd_set_tuning                                     */
  int32_t second_whole;   /* same-spin strings of order 3 in the second-order kernel:
                             1 = one row pair (two columns of the string's 3 x 3 block)
                             per lane, 2 = one whole string per lane (its block gathered
                             once per Cholesky vector); 0 = automatic (2 where a spin
                             has at least 512 strings of order 3, else 1)              */
  int32_t reserved;
} msd_tuning;
msd_status msd_get_tuning(msd_system* sys, msd_tuning* out);
/* Sets overrides (validated; MSD_ERR_ARG names the bad field).  Drops the
 * energy plan and recorded graphs; they are rebuilt on the next call. */
msd_status msd_set_tuning(msd_system* sys, const msd_tuning* t);
/* Autotuner: times candidate values of each field in turn (fb_splitk,
 * walker_tile, lambda_variant, lambda_chunk, second_gather, second_copy,
 * second_waves, second_gsplit, second_stage) over `reps`
 * measurements with energies of the current walkers (time step dt), keeps the
 * fastest and leaves it set (*out, if not NULL, receives it).  Overwrites the
 * last-measurement buffers; walkers are unchanged.  Needs walkers. */
msd_status msd_autotune(msd_system* sys, double dt, int32_t reps, msd_tuning* out);

/* Results of the most recent measurement (msd_measure[_dev] or a measuring
 * msd_batch_step) copied to host buffers; any pointer may be NULL.  Layouts as
 * in msd_measure.  Synchronises the handle's stream. */
msd_status msd_get_measurement(msd_system* sys, double* log_ovlp, double* force_bias,
                               double* e_loc);

/* Batches of independent systems (walker sets, trials and Hamiltonians of
 * uneven sizes) stepped together: each msd_batch_step enqueues, for every
 * system, one propagation step (as msd_propagate_dev with n_steps = 1) and,
 * if do_measure, one measurement (as msd_measure_dev with energies), all on
 * the batch's stream.  With timing off on every system the whole step is
 * recorded once as one HIP graph (per combination of QR steps, measurement
 * flag, dt and e_shift) in which each system's launches form an independent
 * branch (so small systems can run side by side), and replayed afterwards;
 * graphs are re-recorded after any system's trial or Hamiltonian changes.  The systems must be on one
 * device and stay alive until msd_batch_destroy; they may still be used on
 * their own between batch steps (the batch orders itself against each
 * system's stream with events).  A batch is not thread-safe.
 * fields[i]: device pointer, n_walkers_i * n_chol_i standard-normal fields of
 * system i, [w][g].  No singularity check is made (see msd_measure_dev); read
 * results with msd_get_walkers / msd_get_weights / msd_get_measurement. */
typedef struct msd_batch msd_batch;
msd_status msd_batch_create(msd_system* const* systems, int32_t n, void* hip_stream,
                            msd_batch** out);
void msd_batch_destroy(msd_batch* b);
msd_status msd_batch_step(msd_batch* b, const double* const* fields, double dt, double e_shift,
                          int32_t do_measure);

/* Host-only excitation analysis of a trial (no device needed), for checking
 * the trial builder (excitations relative to the reference, Sec. II.B).  Per determinant: k_a/k_b = holes per spin, sign = the
 * product of both spins' excitation signs (+1/-1; the sign of the permutation
 * that sorts the reference with each hole replaced by its particle, holes
 * and particles each ascending).  Returns MSD_ERR_TRIAL like set_trial_occ. */
msd_status msd_trial_analyze(int32_t M, int32_t n_alpha, int32_t n_beta, int64_t n_det,
                             const int32_t* occ_a, const int32_t* occ_b, int32_t* k_a,
                             int32_t* k_b, int32_t* sign);

#ifdef __cplusplus
}
#endif

#endif /* MSD_AFQMC_H */

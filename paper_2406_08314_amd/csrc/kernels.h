// Launch interfaces of the HIP kernels (device pointers only).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace msd {

// ---------------------------------------------------------------- GEMM
struct GemmArgs {
  int M = 0, N = 0, K = 0, batch = 1;
  const double* A = nullptr;
  const double* B = nullptr;
  double* C = nullptr;
  double* Acc = nullptr;        // optional: Acc += result (same layout as C)
  int64_t lda = 0, ldb = 0, ldc = 0;
  int64_t strideA = 0, strideB = 0, strideC = 0;
  int64_t a_imag_off = 0;       // complex mode: offset of the imaginary plane of A
  const int* mask = nullptr;    // optional per-batch skip mask (0 = skip)
  int splitk = 1;               // >1: K split over blockIdx.z (batch must be 1)
  double* ws = nullptr;         // split-K workspace: splitk * M * N doubles
  double alpha = 1.0, beta = 0.0;
  bool a_kmaj = true, b_kmaj = false, cplx = false;
  // >0: column-blocked output, C element (m, n) at
  // (n / c_block) * M * c_block + m * c_block + n % c_block (ldc unused;
  // no batch, split-K, beta or Acc)
  int c_block = 0;
};
void launch_gemm(const GemmArgs& g, hipStream_t st);

// FP32 MFMA GEMM (real operands, FP32 accumulation), same operand conventions
// as GemmArgs; the result goes to C32 (float) or C64 (double).
struct GemmArgs32 {
  int M = 0, N = 0, K = 0, batch = 1;
  const float* A = nullptr;
  const float* B = nullptr;
  float* C32 = nullptr;
  double* C64 = nullptr;
  int64_t lda = 0, ldb = 0, ldc = 0;
  int64_t strideA = 0, strideB = 0, strideC = 0;
  const int* mask = nullptr;
  int splitk = 1;               // >1: K split over blockIdx.z (batch must be 1)
  float* ws = nullptr;          // split-K workspace: splitk * M * N floats
  double alpha = 1.0;
  bool a_kmaj = true, b_kmaj = false;
  int c_block = 0;  // as GemmArgs::c_block
};
void launch_gemm32(const GemmArgs32& g, hipStream_t st);
// Element-wise precision conversions (n elements).
void launch_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t st);

// Window layout of Lambda as the fused contraction kernels write it when the
// second-order terms read it (swz mode): mode 1, eight hole slots, entry
// (a, i) at a * 8 + (i ^ ((a >> 1) & 7)); mode 2, sixteen hole slots, entry
// (a, i) at a * 16 + (i ^ (a & 15)).  Either spreads a wave's gathers of one
// hole slot over the LDS banks.  Maps an unswizzled index a * n_o + i.
__host__ __device__ inline int lam_swizzle(int x, int mode = 1) {
  return mode == 2 ? (x & ~15) | ((x & 15) ^ ((x >> 4) & 15))  // n_o 16: the slot's four bits
                   : (x & ~7) | ((x & 7) ^ ((x >> 4) & 7));   // n_o 8: (a >> 1) & 7
}

// ---------------------------------------------------------------- device tables
struct DevSpin {
  int N = 0, U = 0, nv = 0, no = 0, P = 0;  // P = N + nv (rows R then V_act)
  int col0 = 0;                              // column offset in the walker matrix
  int A = 0, M2 = 0;                         // adj / minor entries per walker
  int n_minor = 0;
  const int* ref = nullptr;      // [N]
  const int* vir = nullptr;      // [nv]
  const int* nref = nullptr;     // [M - N] orbitals outside the reference, ascending
  const int* vpos = nullptr;     // [nv] position of each window virtual in nref
  const int* oslot = nullptr;    // [no]
  const int* rows = nullptr;     // [P]
  const int* k = nullptr;        // [U]
  const int* hslot = nullptr;    // [U*KMAX]
  const int* hwin = nullptr;
  const int* part = nullptr;
  const int* pwin = nullptr;
  const int* adj_off = nullptr;  // [U+1]
  const int* m2_off = nullptr;   // [U+1]
  const int* bw_ptr = nullptr;   // [U+1]
  const int* bw_det = nullptr;
  int n_seg = 0;                 // det lists cut into segments of <= 16
  const int* seg_ptr = nullptr;  // [n_seg+1] into bw_det
  const int* str_seg = nullptr;  // [U+1] segments of each string
  const int* c_ptr = nullptr;    // [nv*no+1]
  const int* c_adj = nullptr;
  const int* c_str = nullptr;
  const int* mn_idx = nullptr;   // [n_minor*4]
  const int* mn_ptr = nullptr;   // [n_minor+1]
  const int* mn_str = nullptr;
  const int* mn_m2 = nullptr;
  const int* mn_sgn = nullptr;
  const int* det_s = nullptr;    // [n_det]
  int bucket[KMAX + 2] = {0};
};

struct DevPairs {
  int n_pair = 0;
  const int* x = nullptr;
  const int* y = nullptr;
  const int64_t* ptr = nullptr;
  const int* det = nullptr;
  const int* fa = nullptr;
  const int* fb = nullptr;
};

// Per-spin walker-batch work arrays.
struct SpinWork {
  cd* T = nullptr;        // [M][NW][N]      T = Phi A^{-1}
  cd* logdetA = nullptr;  // [NW]
  cd* d = nullptr;        // [NW][U]         det X per string
  cd* adj = nullptr;      // [NW][A]         adj X per string
  cd* m2 = nullptr;       // [NW][M2]        second-order minors per string
  cd* B = nullptr;        // [NW][U]         CI weight per string
  cd* C = nullptr;        // [NW][nv*no]     first-order CI matrix
  cd* G = nullptr;        // [NW][P][M]      Green's function rows R u V_act
  double* onebody = nullptr;  // [NW*2]  complex
};

// ---------------------------------------------------------------- Wick kernels
void launch_ref_inverse(const cd* phi, int M, int Ntot, int NW, const DevSpin& sa,
                        const DevSpin& sb, cd* Ta, cd* Tb, cd* ldA, cd* ldB, int* flag,
                        hipStream_t st);
void launch_strings(const DevSpin& sa, const DevSpin& sb, const cd* Ta, const cd* Tb, int NW,
                    bool minors, const SpinWork& wa, const SpinWork& wb, hipStream_t st);
void launch_ovlp_partial(int64_t n_det, int NW, const int* sa, const int* sb, const cd* c,
                         const cd* da, int Ua, const cd* db, int Ub, cd* partial,
                         int n_chunks, int chunk, hipStream_t st);
void launch_ovlp_final(int NW, const cd* partial, int n_chunks, const cd* ldA,
                       const cd* ldB, cd* obar, cd* log_ovlp, int* flag, hipStream_t st);
void launch_ci_weights(const DevSpin& sa, const DevSpin& sb, const cd* det_c, const SpinWork& wa,
                       const SpinWork& wb, cd* seg_a, cd* seg_b, int NW, hipStream_t st);
void launch_ci_matrix(const DevSpin& sa, const DevSpin& sb, int NW, const SpinWork& wa,
                      const SpinWork& wb, hipStream_t st);
// G rows and the one-body energies onebody[spin][w] ([2][NW]); ob_part is
// scratch of 2 * NW * green_tiles(M) entries
int green_tiles(int M);
void launch_green(const DevSpin& sa, const DevSpin& sb, int M, int NW, const SpinWork& wa,
                  const SpinWork& wb, cd* onebody, const cd* obar, const double* h1,
                  cd* ob_part, hipStream_t st);
void launch_green_sum(int M, int NW, int P_all, const int* rmap_a, const int* rmap_b,
                      int Pa, int Pb, const cd* Ga, const cd* Gb, double* Gp,
                      hipStream_t st);
void launch_xbar(int NW, int NG, const double* raw, double sqrt_dt, cd* xbar, hipStream_t st);

// General fused contraction kernel (ltl_general.hip): for each walker of the
// tile, spin and Cholesky vector, LT = L[V u R, :] T on the matrix cores, then
// Q, per-wave partials of v0 = tr Q, ex0 = tr QQ and <C, Lambda window> per
// vector (v0 / ex0 / lamc, [2][NW][NG][parts]), the Lambda window (written
// like the other kernels) and per-wave partials of <C, Lambda Q> per chunk
// into czw ([2][NW][n_chunks * parts]).
// The S arrays come from launch_gather_general.
// With a walker list (wls.list: walker indices, wls.count: their number, both
// on the device), only the listed walkers of the tile are processed, by a
// persistent grid of the workgroups resident on wls.n_cu compute units; the
// mask is then ignored.
struct WalkerList {
  const int* list = nullptr;
  const int* count = nullptr;
  int n_cu = 0;
};
bool ltl_general_fits(const DevSpin& sa, const DevSpin& sb, int M, bool fp32);
// false where the FP64 instance that applies is the six-column-tile one with T
// in registers (six waves on a CU, spilling): it serves the mixed form's FP64
// pass over a few walkers, while the LT-GEMM path is faster for whole batches
bool ltl_general_fast64(const DevSpin& sa, const DevSpin& sb, int M);
int ltl_general_parts(const DevSpin& sa, const DevSpin& sb);
size_t ltl_general_s_elems(const DevSpin& sa, const DevSpin& sb, int M, int NG);
void launch_gather_general(const double* L, int NG, int M, const DevSpin& D, const DevSpin& sa,
                           const DevSpin& sb, double* S64, float* S32, hipStream_t st);
// swz: store the Lambda windows in lam_swizzle layout swz (0: plain).
void launch_ltl_general(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                        int g_chunk, int M, const double* Sa, const double* Sb, const cd* Ta,
                        const cd* Tb, cd* Lam_a, cd* Lam_b, const cd* Ca, const cd* Cb, cd* v0,
                        cd* ex0, cd* lamc, cd* czw, const int* wmask, int swz, hipStream_t st,
                        const WalkerList& wls = WalkerList());
// mask[w] = 1 where max |T| of walker w (either spin) exceeds tmax, rest[w] =
// 1 - mask[w]; list[0 .. *count) = the walkers with mask[w] = 1, in order
void launch_walker_tmax(int NW, int M, int na, int nb, const cd* Ta, const cd* Tb, double tmax,
                        int* mask, int* rest, int* list, int* count, hipStream_t st);
void launch_ltl_general32(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                          int g_chunk, int M, const float* Sa, const float* Sb, const cf* Ta,
                          const cf* Tb, cf* Lam_a, cf* Lam_b, const cd* Ca, const cd* Cb, cd* v0,
                          cd* ex0, cd* lamc, cd* czw, const int* wmask, int swz, hipStream_t st,
                          const WalkerList& wls = WalkerList());

// energy (one walker tile of WT walkers starting at w0)
void launch_lambda(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                   int g_chunk, const cd* Ta, const cd* Tb, const cd* LTa, const cd* LTb,
                   cd* Lam_a, cd* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a, cd* ZWpart_b,
                   hipStream_t st);
void launch_lambda32(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                     int g_chunk, const cf* Ta, const cf* Tb, const cf* LTa, const cf* LTb,
                     cf* Lam_a, cf* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a, cd* ZWpart_b,
                     hipStream_t st);
bool lambda_rows_fits(const DevSpin& sa, const DevSpin& sb, int* nmax);
void launch_lambda_rows(const DevSpin& sa, const DevSpin& sb, int nmax, int NW, int w0, int WT,
                        int NG, int g_chunk, const cd* Ta, const cd* Tb, const cd* LTa,
                        const cd* LTb, cd* Lam_a, cd* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a,
                        cd* ZWpart_b, hipStream_t st);
// Same in single precision (mixed form): T, LT and Lambda as cf; v0, ex0 and
// the ZW partial sums accumulate in double.
void launch_lambda_rows32(const DevSpin& sa, const DevSpin& sb, int nmax, int NW, int w0, int WT,
                          int NG, int g_chunk, const cf* Ta, const cf* Tb, const cf* LTa,
                          const cf* LTb, cf* Lam_a, cf* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a,
                          cd* ZWpart_b, hipStream_t st);
// Fused Cholesky contraction + energy intermediates on the matrix cores for
// N = 8 per spin with the whole occupied set in the window, n_vir_act <= 64
// and M <= 64: no LT in HBM.  S_a/S_b are the
// restricted rows of L per spin, k-major and padded, [NG][64][P16] with rows
// V_act then R (launch_gather_ltl); Lambda windows [w][g][a * N + i].
bool ltl_mfma_fits(const DevSpin& sa, const DevSpin& sb, int M, bool fp32);
size_t ltl_stage_elems(const DevSpin& sa, const DevSpin& sb);  // 64 * P16 per vector
int ltl_rows16(const DevSpin& sa, const DevSpin& sb);
void launch_gather_ltl(const double* L, int NG, int M, const DevSpin& D, int P16, double* S64,
                       float* S32, hipStream_t st);
// v0 of both spins ([2][NW][NG], from launch_qtr) enters ZW = sum_g Xi - v Lam;
// ZW is contracted with the first-order CI matrices Ca/Cb ([w][X]) per chunk
// of vectors: czw[2][NW][n_chunks] = sum_x C[w][x] ZW_chunk[x] (n_chunks =
// ceil(NG / g_chunk)), which launch_energy_final sums.
// swz: store the Lambda windows in the lam_swizzle layout.
void launch_ltl_mfma(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                     int g_chunk, int M, const double* Sa, const double* Sb, const cd* Ta,
                     const cd* Tb, cd* Lam_a, cd* Lam_b, const cd* v0, const cd* Ca,
                     const cd* Cb, cd* czw, bool swz, hipStream_t st);
void launch_ltl_mfma32(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                       int g_chunk, int M, const float* Sa, const float* Sb, const cf* Ta,
                       const cf* Tb, cf* Lam_a, cf* Lam_b, const cd* v0, const cd* Ca,
                       const cd* Cb, cd* czw, bool swz, hipStream_t st);
// FP64 mean-field traces v0, ex0 ([2][NW][NG]) of Q^g = L^g[R, :] T for the
// walkers w0 .. w0 + WT - 1 (N = 8 per spin, M <= 64); SRa/SRb are the
// reference rows of L, k-major [NG][64][8] (launch_gather_ltl with no
// virtuals and 8 rows).
void launch_qtr(int NW, int w0, int WT, int NG, int M, const double* SRa, const double* SRb,
                const cd* Ta, const cd* Tb, cd* v0, cd* ex0, int n_cu, hipStream_t st);
void init_ltl_attributes();
// adjT_a / adjT_b (A x NW each, or null): scratch for walker-fastest copies of
// the adjugates; given, the sums run with the walkers on the lanes (for pairs
// with many entries each)
void launch_pair_coef(const DevPairs& pr, int NW, const cd* det_c, const cd* adj_a, int Aa,
                      const cd* adj_b, int Ab, cd* coef, hipStream_t st, cd* adjT_a = nullptr,
                      cd* adjT_b = nullptr);
void launch_minor_coef(const DevSpin& s, int NW, const cd* B, int U, const cd* m2, cd* coef,
                       hipStream_t st);
// second-order energy terms; each launch writes blocks into partial[w][slot0 + ...]
// plan roles: ER_PAIRS, 2..6 = row-pair items of strings of that order, or
// ER_WHOLE | 3 = whole strings of order 3, one per lane (order 4 would keep 36
// complex minors per lane: they spill)
enum EnergyRole { ER_NONE = 0, ER_PAIRS = 1, ER_WHOLE = 0x10 };
constexpr int ER_MAX_ORDER = 6;
constexpr int ER_WAVES = 8;  // waves per workgroup of the merged second-order kernel
constexpr int ER_PAIRS_PER_WAVE = 256;  // 64 lanes x 4 pairs
void launch_energy_second(const DevSpin& sa, const DevSpin& sb, const DevPairs& pr,
                          const int4* plan, int n_itemblocks, int waves_per_block, int NW, int w0,
                          int WT, int NG, int n_gsplit, int G, int max_order, bool flat_gather,
                          bool use_dma, int swz, const cd* Lam_a, const cd* Lam_b, const cd* coef,
                          const cd* m2a, const cd* m2b, const cd* Ba, const cd* Bb, cd* partial,
                          int n_slots, int slot0, hipStream_t st, const int* wmask = nullptr,
                          const WalkerList& wls = WalkerList());
// Same with single-precision Lambda (mixed form); the minors, CI weights and
// the final products stay in double.
void launch_energy_second32(const DevSpin& sa, const DevSpin& sb, const DevPairs& pr,
                            const int4* plan, int n_itemblocks, int waves_per_block, int NW,
                            int w0, int WT, int NG, int n_gsplit, int G, int max_order,
                            bool flat_gather, bool use_dma, int swz, const cf* Lam_a, const cf* Lam_b,
                            const cd* coef, const cd* m2a, const cd* m2b, const cd* Ba,
                            const cd* Bb, cd* partial, int n_slots, int slot0, hipStream_t st,
                            const int* wmask = nullptr);
// W-form of the second-order terms: G^{st} = per-walker real GEMMs of the
// interleaved Lambda windows over the Cholesky index ([wl][2X_s][2X_t]); the
// pair and minor coefficient lists contracted with W into one slot per walker.
void launch_wform_contract(const DevSpin& sa, const DevSpin& sb, const DevPairs& pr, int NW,
                           int w0, int WT, const double* Gaa, const double* Gab,
                           const double* Gbb, const cd* coefAB, const cd* coef_a,
                           const cd* coef_b, cd* partial, int n_slots, int slot, hipStream_t st,
                           const int* wmask = nullptr);
int energy_minor_blocks(const DevSpin& s);
void launch_energy_minors(const DevSpin& s, int NW, int w0, int WT, int NG, int n_gsplit,
                          const cd* Lam, const cd* coef, cd* partial, int n_slots, int slot0,
                          hipStream_t st);
// czw (when not null, [2][NW][n_lchunks]) replaces the ZW partials: the
// first-order term is then the sum of those contracted partials.  lamc (when
// not null, [2][NW][NG][n_lparts]) adds -(v0_a + v0_b) <C, Lambda> per vector.
// wmask (when not null): only walkers with wmask[w] != 0 are assembled (as in
// launch_energy_second).  The second-order partials of a walker are the slots
// [e_lo, e_hi) of its row of epart (row length n_slots).
void launch_energy_final(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                         int n_lchunks, int n_slots, int e_lo, int e_hi, const cd* obar,
                         const cd* v0,
                         const cd* ex0, const cd* ZWpart_a, const cd* ZWpart_b,
                         const cd* Ca, const cd* Cb, const cd* czw, const cd* epart,
                         const cd* onebody_a, const cd* onebody_b, double e0, cd* e_loc,
                         const cd* lamc, int n_lparts, hipStream_t st,
                         const int* wmask = nullptr);

// ---------------------------------------------------------------- propagation
void launch_vhs_prep(int NW, int NG, const double* x, const cd* xbar, double sqrt_dt,
                     const double* weights, double* Y, hipStream_t st);
void launch_weights(int NW, int NG, const double* x, const cd* xbar, const cd* logo_new,
                    cd* logo, double* weights, double dt, double e_shift, hipStream_t st);
// Cholesky-QR of every unmasked walker; logo and the per-spin log det A
// (when not null) shift by -log det R
void launch_qr(cd* phi, int M, int Ntot, int NW, int na, int nb, const int* mask, double* ldet,
               cd* logo, cd* logdetA_a, cd* logdetA_b, hipStream_t st);
void launch_frozen_mask(int NW, const double* weights, int* mask, hipStream_t st);
// v0 = tr Q, ex0 = tr QQ in FP64 from Q tiles [wl][g][N x N] of both spins.
void launch_traces64(const cd* Qa, const cd* Qb, int Na, int Nb, int NW, int w0, int WT, int NG,
                     cd* v0, cd* ex0, hipStream_t st);
void launch_fill_i32(int* p, int n, int v, hipStream_t st);
void launch_copy_walkers(int NW, int M, int Ntot, int na, int nb, const cd* pa, const cd* pb,
                         cd* phi, bool to_internal, cd* out_a, cd* out_b, hipStream_t st);
// Comb population control: new weights W / n in place, parent[k] per new
// walker, copies of the parents' orbitals (per_w complex per walker) and log
// overlaps into phi_out / logo_out.  cum: NW doubles of scratch.
void launch_comb(int NW, double z, double* weights, double* cum, int* parent, const cd* phi,
                 const cd* logo, int64_t per_w, cd* phi_out, cd* logo_out, hipStream_t st);
// out[0] = sum_w w E_L, out[1] = (sum_w w, 0) over walkers of positive weight.
void launch_block_energy(int NW, const double* weights, const cd* eloc, cd* out,
                         hipStream_t st);
void launch_gather_rows(const double* L, int NG, int M, const int* rows, int P, double* out,
                        hipStream_t st);

// A2 + A6 fused (Cholesky contraction + energy intermediates) when the tile fits
bool chol_contract_fits(const DevSpin& sa, const DevSpin& sb, int* WB);
void launch_chol_contract(const DevSpin& sa, const DevSpin& sb, const double* Llt_a,
                          const double* Llt_b, const cd* Ta, const cd* Tb, cd* Lam_a, cd* Lam_b,
                          cd* ZW_a, cd* ZW_b, int M, int NW, int w0, int WT, int NG, int g_chunk,
                          int WB, cd* v0, cd* ex0, hipStream_t st);
void init_gemm_attributes();

// raise the dynamic-LDS limit of the kernels that may need more than 64 KB
void init_wick_attributes();
void init_prop_attributes();

}  // namespace msd

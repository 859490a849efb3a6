// Host runtime behind the C ABI declared in include/msd_afqmc.h.
//
// Owns the device memory of one walker batch, the trial tables and the
// Hamiltonian, and enqueues the kernel pipeline on the handle's stream:
//   measure   = reference inverse -> string dets/adjugates -> Obar ->
//               CI weights -> CI matrix -> Green's rows -> force-bias GEMM
//               [-> Cholesky GEMM -> Lam/Xi -> two-body coefficients ->
//                   Cholesky-vector loop -> energy assembly]
//   propagate = force bias -> VHS GEMM -> one-body half step -> Taylor chain
//               (complex GEMMs) -> one-body half step -> new overlap ->
//               weights [-> QR].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <mutex>
#include <vector>

#include "common.h"
#include "kernels.h"
#include "msd_afqmc.h"
#include "trial.h"

using msd::cd;
using msd::cf;

namespace {

struct Error {
  msd_status code;
  std::string msg;
};

[[noreturn]] void fail(msd_status c, const std::string& m) { throw Error{c, m}; }

void hip_check(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) fail(MSD_ERR_OOM, std::string(what) + ": out of device memory");
  if (e != hipSuccess) fail(MSD_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

enum Stage {
  ST_REF, ST_STR, ST_OVLP, ST_CIW, ST_CIM, ST_GREEN, ST_FB_GEMM, ST_LT_GEMM, ST_LAMBDA,
  ST_COEF, ST_EGAMMA, ST_EFINAL, ST_VHS_GEMM, ST_B1, ST_TAYLOR, ST_WEIGHTS, ST_QR, ST_TRACES,
  ST_POP, ST_GUARD, ST_COUNT
};
const char* kStageNames[ST_COUNT] = {
    "ref_inverse", "strings",  "overlap",   "ci_weights", "ci_matrix",    "green",
    "fb_gemm",     "lt_gemm",  "lambda",    "coef",       "energy_gamma", "energy_final",
    "vhs_gemm",    "one_body", "taylor",    "weights",    "qr",           "traces",
    "pop_control", "fp64_guard"};

// Minimal device arena: every allocation is recorded and freed together.
struct Arena {
  std::vector<void*> ptrs;
  template <class T>
  T* get(size_t n) {
    if (n == 0) n = 1;
    void* p = nullptr;
    hip_check(hipMalloc(&p, n * sizeof(T)), "hipMalloc");
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t st) {
    T* p = get<T>(v.size());
    if (!v.empty())
      hip_check(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st),
                "upload");
    return p;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

}  // namespace

struct msd_system {
  int dev = 0;
  int n_cu = 256;  // compute units of the device (workgroup-slot heuristics)
  hipStream_t st = nullptr;
  msd_dims d{};
  msd_options o{};
  std::string err;
  int M = 0, na = 0, nb = 0, Ntot = 0, NG = 0, NW = 0;
  int64_t ND = 0;
  bool have_ham = false, have_trial = false, have_walkers = false;
  Arena base, ham_mem, trial_mem, energy_mem;

  // Hamiltonian
  double* L = nullptr;    // [NG][M][M]
  double* h1 = nullptr;   // [M][M]
  double* B1 = nullptr;   // [M][M]  expm(-dt h'/2)
  double B1_dt = NAN;
  double e0 = 0.0;
  std::vector<double> h1_host, sumll_host;

  // trial
  msd::TrialTables tt;
  msd::DevSpin ds[2];
  msd::DevPairs dp;
  cd* det_c = nullptr;
  int P_all = 0;
  int* rmap[2] = {nullptr, nullptr};
  int* rows_all_dev = nullptr;
  double* L_rows = nullptr;   // [NG][P_all][M]
  double* L_lt[2] = {nullptr, nullptr};  // [NG][P_s][M]
  bool derived_ok = false;

  // walkers
  cd* phi = nullptr;       // [NW][M][Ntot]
  double* weights = nullptr;
  cd* logo = nullptr;
  int64_t steps_done = 0;
  // block driver: comb scratch (running sums, parents, parents' log overlaps)
  // and the weighted energy sums of the last block
  double* pc_cum = nullptr;
  int* pc_parent = nullptr;
  cd* pc_logo = nullptr;
  cd* blk = nullptr;

  // work
  msd::SpinWork sw[2];
  cd* obar = nullptr;
  cd* opart = nullptr;
  int n_ochunks = 1, ochunk = 2048;
  int* flag = nullptr;
  double* Gp = nullptr;
  double* xraw = nullptr;
  cd* xbar = nullptr;
  cd* logo_tmp = nullptr;
  cd* eloc = nullptr;
  cd* onebody = nullptr;   // [2][NW]
  cd* ob_part = nullptr;   // [2][NW][orbital tiles] one-body partials of the Green kernel
  cd* segp[2] = {nullptr, nullptr};  // CI-weight segment partials
  double* fb_ws = nullptr;           // split-K workspace of the force-bias GEMM
  int fb_splitk = 1, fb_splitk_auto = 1, fb_ws_cap = 0;
  msd_tuning tune{};                 // launch-shape overrides (0 = automatic)
  int lambda_variant = 1;            // resolved: 0 generic, 1 rows, 5 fused N = 8, 6 general
                                     // LT-tile kernel, 5 fused contraction + Lambda (N = 8),
                                     // 6 general fused contraction
  bool lambda_exact = false;         // N == nmax per spin and identity occupied window

  // mixed form: single-precision copies of the GEMM operands
  bool mixed = false;
  float* L32 = nullptr;                     // [NG][M][M]
  float* Llt32[2] = {nullptr, nullptr};     // [NG][P_s][M]
  float* Lrows32 = nullptr;                 // [NG][P_all][M]
  float* T32[2] = {nullptr, nullptr};       // [M][NW][N_s] complex
  float* Gp32 = nullptr;                    // [2 NW][P_all M]
  float* Y32 = nullptr;                     // [2 NW][NG]
  float* fb_ws32 = nullptr;
  cf* LT32[2] = {nullptr, nullptr};
  double* LR64[2] = {nullptr, nullptr};     // [NG][N_s][M] reference rows of L (FP64)
  cd* Q64[2] = {nullptr, nullptr};          // [wl][g][N_s x N_s] FP64 Q for the traces
  cd* czw = nullptr;  // [2][NW][n_lchunks] C . ZW per chunk (fused kernel)
  int lam_swz = 0;  // Lambda windows in lam_swizzle layout lam_swz (fused kernels; 0 plain)
  cf* Lam32[2] = {nullptr, nullptr};
  bool energy_mixed = false;                // mixed energy path usable for this trial

  // fused contraction + Lambda kernel: restricted rows of L per spin, k-major,
  // [NG][64][lf_P16], rows V_act then R (FP64, and FP32 in the mixed form)
  int lf_P16 = 0;
  bool lf_fits64 = false, lf_fits32 = false;
  double* Slf[2] = {nullptr, nullptr};
  float* Slf32[2] = {nullptr, nullptr};
  double* Slr[2] = {nullptr, nullptr};  // reference rows only, [NG][64][8] (traces)

  // general fused contraction kernel (N <= 48 per spin, M <= 320, window of
  // at most 32 virtual and 32 occupied orbitals): rows of L per spin, k-major,
  // [NG][Mpad][P16], window virtual rows then reference rows
  bool gl_fits = false, gl_fits32 = false;  // FP64 / FP32 instances apply
  bool gl_fast64 = true;  // the FP64 instance is the default for whole batches
  double* Sgl[2] = {nullptr, nullptr};
  float* Sgl32[2] = {nullptr, nullptr};
  cd* lamc = nullptr;  // [2][NW][NG][gl_parts]: <C, Lambda window> per vector
  int gl_parts = 1;
  // mixed form with the general kernel: walkers whose largest |T| exceeds
  // tmax get FP64 energies in a second, masked pass (FP64 Lambda windows)
  double tmax = 2.0;
  bool guard = false;
  int* gmask = nullptr;  // [NW] 1: FP64 pass
  int* fmask = nullptr;  // [NW] 1: single-precision pass (the complement of gmask)
  int* glist = nullptr;  // [NW + 1] the walkers of the FP64 pass, then their count
  int second_G64 = 1;    // LDS stage depth of the FP64 second-order pass
  int gl_chunk_guard = 1, n_lchunks_guard = 0;  // finer vector chunks: few walkers
  // the FP64 pass's second-order partials: a finer split of the Cholesky range
  // (few walkers) into slots of their own, [slot_guard, slot_guard_end)
  int gsplit_guard = 1, slot_guard = 0, slot_guard_end = 0;
  // W-form of the second-order terms: per-walker GEMMs over the Cholesky index
  // of the Lambda windows, [wl][2X_s][2X_t] for (aa, ab, bb), then the
  // coefficient lists contracted with them (one energy slot per walker)
  bool wform = false;
  double* Gw[3] = {nullptr, nullptr, nullptr};
  int slot_wform = 0;

  // energy work (lazily sized)
  int WT = 0, gl_chunk = 16, n_lchunks = 0;
  // second-order energy plan: per-spin algorithm and partial slots
  int gsplit = 1, n_slots = 0;
  int n_slots_main = 0;  // slots [0, n_slots_main) belong to the main energy pass
  bool use_strings[2] = {false, false};
  int slot_min[2] = {0, 0};
  // merged second-order kernel: wave plan (role | spin << 8, first string of
  // the order, first item, item end), ER_WAVES entries per item block
  std::vector<int4> plan_host;
  int4* plan = nullptr;
  int n_itemblocks = 0, slot_second = 0, second_G = 1, second_maxk = 0, second_waves = 8;
  bool second_flat = false;  // gathers through a generic pointer (see k_energy_second)
  bool second_whole_used = false;  // order-3 strings as whole-string items
  bool second_dma = true;    // stages Lambda by direct global-to-LDS loads
  cd* LT[2] = {nullptr, nullptr};
  cd* Lam[2] = {nullptr, nullptr};
  cd* v0 = nullptr;
  cd* ex0 = nullptr;
  cd* ZWp[2] = {nullptr, nullptr};
  cd* coefAB = nullptr;
  cd* adjT[2] = {nullptr, nullptr};  // walker-fastest adjugate copies (pairs with many entries)
  cd* coef2[2] = {nullptr, nullptr};
  cd* epart = nullptr;

  // propagation work
  double* Y = nullptr;
  double* VHS = nullptr;
  cd* term[2] = {nullptr, nullptr};
  cd* acc = nullptr;
  int* mask = nullptr;
  double* qr_ldet = nullptr;  // [NW][2] log det R per spin
  double* fields = nullptr;  // staging for host fields [NW][NG]

  // graph replay: one executable graph per (kind, variant), captured on a
  // private stream and launched on st; keyed by the scalars baked into it
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    double dt = 0.0, e_shift = 0.0;
  };
  hipStream_t cap_st = nullptr;
  GraphSlot g_step[2][2];     // [QR in this step][T fresh at the start]
  GraphSlot g_measure[2][2];  // [energy requested][T fresh at the start]
  uint64_t version = 0;  // bumped whenever captured graphs become stale
  void drop_graphs() {
    ++version;
    for (auto* set : {&g_step, &g_measure})
      for (auto& pair : *set)
        for (GraphSlot& g : pair) {
          if (g.exec) (void)hipGraphExecDestroy(g.exec);
          g.exec = nullptr;
        }
  }
  // T = Phi A^-1, the excitation determinants, Obar and log det A hold for
  // the current walkers: set by every overlap pass, kept by the QR step
  // (Phi -> Phi R^-1 leaves T and the determinants unchanged and shifts log
  // det A by -log det R), cleared by anything else that rewrites Phi or the
  // trial (population control, new walkers, a new trial).  A propagation step
  // then skips its first overlap pass and a measurement its reference inverse.
  bool t_fresh = false;
  bool graphs_on() const { return o.graphs && !o.timing; }

  // timing
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  double stage_ms[ST_COUNT] = {0};
  int64_t stage_n[ST_COUNT] = {0};

  hipEvent_t ev() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hip_check(hipEventCreate(&e), "hipEventCreate");
    return e;
  }
  void harvest() {
    if (pending.empty()) return;
    hip_check(hipStreamSynchronize(st), "synchronize");
    for (auto& p : pending) {
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, p.second.first, p.second.second), "elapsed");
      stage_ms[p.first] += ms;
      stage_n[p.first] += 1;
      pool.push_back(p.second.first);
      pool.push_back(p.second.second);
    }
    pending.clear();
  }
  template <class F>
  void timed(Stage s, F&& f) {
    if (!o.timing) {
      f();
      return;
    }
    hipEvent_t a = ev(), b = ev();
    hip_check(hipEventRecord(a, st), "record");
    f();
    hip_check(hipEventRecord(b, st), "record");
    pending.push_back({(int)s, {a, b}});
    if (pending.size() > 4096) harvest();
  }
  void sync() { hip_check(hipStreamSynchronize(st), "synchronize"); }
  void check_launch(const char* what) { hip_check(hipGetLastError(), what); }
};

namespace {

thread_local std::string g_err;

#define API_BEGIN \
  try {
#define API_END(sysp)                                        \
  }                                                          \
  catch (const Error& e) {                                   \
    if (sysp) (sysp)->err = e.msg;                           \
    g_err = e.msg;                                           \
    return e.code;                                           \
  }                                                          \
  catch (const std::bad_alloc&) {                            \
    if (sysp) (sysp)->err = "host allocation failed";        \
    return MSD_ERR_OOM;                                      \
  }                                                          \
  catch (...) {                                              \
    if (sysp) (sysp)->err = "unexpected internal error";     \
    return MSD_ERR_DEVICE;                                   \
  }                                                          \
  return MSD_OK;

void set_device(msd_system* s) { hip_check(hipSetDevice(s->dev), "hipSetDevice"); }

// expm of a small real matrix by scaling and squaring of its Taylor series.
std::vector<double> expm_host(const std::vector<double>& a, int n) {
  double norm = 0.0;
  for (int j = 0; j < n; ++j) {
    double c = 0.0;
    for (int i = 0; i < n; ++i) c += std::fabs(a[(size_t)i * n + j]);
    norm = std::max(norm, c);
  }
  int s = 0;
  while (norm / std::ldexp(1.0, s) > 0.25) ++s;
  const double scale = std::ldexp(1.0, -s);
  std::vector<double> x(a.size()), res((size_t)n * n, 0.0), term((size_t)n * n, 0.0),
      tmp((size_t)n * n);
  for (size_t i = 0; i < a.size(); ++i) x[i] = a[i] * scale;
  for (int i = 0; i < n; ++i) res[(size_t)i * n + i] = term[(size_t)i * n + i] = 1.0;
  auto mul = [n](const std::vector<double>& p, const std::vector<double>& q,
                 std::vector<double>& out) {
    std::fill(out.begin(), out.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        const double v = p[(size_t)i * n + k];
        if (v == 0.0) continue;
        const double* qr = &q[(size_t)k * n];
        double* orow = &out[(size_t)i * n];
        for (int j = 0; j < n; ++j) orow[j] += v * qr[j];
      }
  };
  for (int k = 1; k <= 24; ++k) {
    mul(term, x, tmp);
    for (size_t i = 0; i < tmp.size(); ++i) term[i] = tmp[i] / k;
    for (size_t i = 0; i < tmp.size(); ++i) res[i] += term[i];
  }
  for (int i = 0; i < s; ++i) {
    mul(res, res, tmp);
    res.swap(tmp);
  }
  return res;
}

void free_energy(msd_system* s) {
  s->drop_graphs();
  s->energy_mem.release();
  s->WT = 0;
}

// Cholesky rows restricted to the orbitals the Wick kernels touch (needs both
// the Hamiltonian and the trial).
void build_derived(msd_system* s) {
  if (s->derived_ok) return;
  if (!s->have_ham || !s->have_trial) fail(MSD_ERR_STATE, "Hamiltonian and trial must both be set");
  set_device(s);
  for (int sp = 0; sp < 2; ++sp) {
    const msd::DevSpin& D = s->ds[sp];
    msd::launch_gather_rows(s->L, s->NG, s->M, D.rows, D.P, s->L_lt[sp], s->st);
  }
  msd::launch_gather_rows(s->L, s->NG, s->M, s->rows_all_dev, s->P_all, s->L_rows, s->st);
  for (int sp = 0; sp < 2; ++sp)
    if (s->lf_fits64 || s->lf_fits32) {
      msd::launch_gather_ltl(s->L, s->NG, s->M, s->ds[sp], s->lf_P16, s->Slf[sp], s->Slf32[sp],
                             s->st);
      msd::DevSpin R = s->ds[sp];  // reference rows only
      R.nv = 0;
      msd::launch_gather_ltl(s->L, s->NG, s->M, R, 8, s->Slr[sp], nullptr, s->st);
    }
  if (s->gl_fits || s->gl_fits32)
    for (int sp = 0; sp < 2; ++sp)
      msd::launch_gather_general(s->L, s->NG, s->M, s->ds[sp], s->ds[0], s->ds[1], s->Sgl[sp],
                                 s->Sgl32[sp], s->st);
  if (s->mixed) {
    for (int sp = 0; sp < 2; ++sp) {
      msd::launch_f64_to_f32(s->L_lt[sp], s->Llt32[sp], (int64_t)s->NG * s->ds[sp].P * s->M, s->st);
      // the first N rows of a spin's row list are its reference orbitals
      msd::launch_gather_rows(s->L, s->NG, s->M, s->ds[sp].rows, s->ds[sp].N, s->LR64[sp], s->st);
    }
    msd::launch_f64_to_f32(s->L_rows, s->Lrows32, (int64_t)s->NG * s->P_all * s->M, s->st);
  }
  s->check_launch("gather rows");
  s->derived_ok = true;
}

void alloc_energy(msd_system* s) {
  if (s->WT > 0) return;
  const msd::DevSpin& A = s->ds[0];
  const msd::DevSpin& B = s->ds[1];
  const int NG = s->NG, NW = s->NW;
  int slot = 0;
  // Per spin: same-spin second-order terms as row-pair items of each string
  // (merged kernel) or as a list of distinct minors.  Cost per Cholesky vector
  // in LDS gathers plus complex products: a row-pair item of order k gathers 2k
  // values and forms k(k-1)/2 products; a distinct minor gathers 4 and forms 2.
  std::vector<int4>& pl = s->plan_host;
  pl.clear();
  s->second_maxk = 0;
  s->second_whole_used = false;
  const int np = s->dp.n_pair;
  {
    // W-form or direct form: algorithmic work per (walker, Cholesky vector)
    // of each at a rate typical of its kernels (direct: vector ALU and LDS
    // gathers; W-form: matrix-core GEMMs)
    double direct = 8.0 * np;
    for (int sp = 0; sp < 2; ++sp) {
      const msd::SpinTable& S = s->tt.s[sp];
      double fs = 0.0;
      for (int i = 0; i < S.U; ++i) {
        const double pk = S.k[i] * (S.k[i] - 1) / 2;
        fs += 22.0 * pk * pk;
      }
      const double fm = 20.0 * S.n_minor;
      direct += s->mixed ? fs : std::min(fs, fm);  // the mixed direct form runs strings
    }
    const double Xa = (double)A.nv * A.no, Xb = (double)B.nv * B.no;
    const double wf = 8.0 * (Xa * Xa + Xa * Xb + Xb * Xb);
    const double r_direct = s->mixed ? 40.0 : 25.0, r_mfma = s->mixed ? 80.0 : 40.0;
    s->wform = s->o.energy_algo == 4 ||
               (s->o.energy_algo == 0 && wf / r_mfma < direct / r_direct);
  }
  if (!s->wform)
    for (int f = 0; f < np; f += msd::ER_PAIRS_PER_WAVE) pl.push_back(int4{msd::ER_PAIRS, 0, f, np});
  for (int sp = 0; sp < 2; ++sp) {
    const msd::SpinTable& S = s->tt.s[sp];
    long c_str = 0;
    bool big = false;
    for (int i = 0; i < S.U; ++i) {
      const long k = S.k[i];
      if (k >= 2) c_str += k * (k - 1) / 2 * (2 * k + 3 * k * (k - 1) / 2);
      if (k > msd::ER_MAX_ORDER) big = true;
    }
    const long c_min = 10L * S.n_minor;
    bool strings = c_str < c_min;
    if (s->o.energy_algo == 1) strings = false;
    if (s->o.energy_algo == 2) strings = true;
    if (s->mixed) strings = true;  // the mixed direct form has only the row-pair kernel
    if (big) strings = false;  // orders above ER_MAX_ORDER only in the minor-list form
    if (s->wform) strings = false;  // the W-form reads the minor coefficient lists
    s->use_strings[sp] = strings;
    if (!strings) continue;
    for (int i = 0; i < S.U; ++i) s->second_maxk = std::max(s->second_maxk, (int)S.k[i]);
    for (int k = 2; k <= msd::ER_MAX_ORDER; ++k) {
      const int n_str = S.bucket[k + 1] - S.bucket[k];
      // whole order-3 strings where there are many (a whole-string wave does
      // about three row-pair waves' work: with few of them the workgroups
      // holding one wait on it at every stage barrier)
      const bool whole3 =
          k == 3 && (s->tune.second_whole == 2 || (s->tune.second_whole == 0 && n_str >= 512));
      s->second_whole_used = s->second_whole_used || whole3;
      if (whole3) {
        // whole strings: one lane per string gathers its 3 x 3 block once
        for (int f = 0; f < n_str; f += 64)
          pl.push_back(int4{(msd::ER_WHOLE | k) | (sp << 8), S.bucket[k], f, n_str});
        continue;
      }
      const int n_items = n_str * (k * (k - 1) / 2);
      for (int f = 0; f < n_items; f += 64) pl.push_back(int4{k | (sp << 8), S.bucket[k], f, n_items});
    }
  }
  // waves per workgroup; each workgroup stages only the spins its waves read
  // (pairs read both), recorded in bits 16-17 of every entry of the workgroup
  // default 16 (one workgroup per CU, deeper LDS stages) where the order-4
  // kernel applies
  const int want_w = s->tune.second_waves ? s->tune.second_waves : 16;
  const int wpb = (want_w == 16 && s->second_maxk <= 4) ? 16 : msd::ER_WAVES;
  s->second_waves = wpb;
  while (pl.size() % wpb) pl.push_back(int4{msd::ER_NONE, 0, 0, 0});
  s->n_itemblocks = (int)(pl.size() / wpb);
  for (int ib = 0; ib < s->n_itemblocks; ++ib) {
    int need = 0;
    for (int q = 0; q < wpb; ++q) {
      const int4 e = pl[ib * wpb + q];
      const int role = e.x & 0xff;
      if (role == msd::ER_PAIRS) need |= 3;
      else if (role != msd::ER_NONE) need |= 1 << (e.x >> 8);
    }
    for (int q = 0; q < wpb; ++q) pl[ib * wpb + q].x |= need << 16;
  }
  // energy intermediates: which kernel
  int nmax = 0;
  const bool rows_fit = msd::lambda_rows_fits(A, B, &nmax);
  // (the FP32 energy path needs an FP64 pass over the walkers far from the
  // reference; where the only FP64 instance of the general kernel is the
  // spilling six-tile one, that pass and the FP32 path together cost more
  // than the FP64 energy path, so the mixed form keeps FP64 energies there)
  s->energy_mixed = s->mixed && s->gl_fast64 &&
                    (s->wform || (s->use_strings[0] && s->use_strings[1]));
  s->lambda_exact = rows_fit && A.N == nmax && B.N == nmax;
  for (int sp = 0; sp < 2 && s->lambda_exact; ++sp) {
    const msd::SpinTable& S = s->tt.s[sp];
    if (S.no() != S.N) s->lambda_exact = false;
    for (int i = 0; i < S.no() && s->lambda_exact; ++i)
      if (S.occ_slot[i] != i) s->lambda_exact = false;
  }
  {
    // default: the fused contraction + Lambda kernel for N = 8 where it
    // applies, else the general fused contraction kernel, else the two-wave
    // rows kernel over the LT tiles, else (windows beyond the rows kernel's
    // limits) the generic one-wave kernel, variant 0
    int wb_cc = 0;  // the option energy_algo = 3 takes its own fused contraction kernel
    const bool cc = s->o.energy_algo == 3 && msd::chol_contract_fits(A, B, &wb_cc);
    const bool fused_ok =
        s->lambda_exact && !cc && (s->energy_mixed ? s->lf_fits32 : s->lf_fits64);
    const bool gen_ok = (s->energy_mixed ? s->gl_fits32 : s->gl_fits) && !cc;
    // (the FP64 form skips the six-tile register-T instance unless asked for:
    // the LT-GEMM path is faster there)
    const bool gen_default = gen_ok && (s->energy_mixed || s->gl_fast64);
    const int want = s->tune.lambda_variant ? s->tune.lambda_variant
                     : fused_ok                 ? 5
                     : gen_default              ? 6
                                                : 1;
    s->lambda_variant = (want == 6 && gen_ok)     ? 6
                        : (want == 5 && fused_ok) ? 5
                        : rows_fit                ? 1
                                                  : 0;
  }
  const bool fused_kernel = s->lambda_variant >= 5;  // LT never stored
  // walker tile: energy scratch of a tile within 16 GB
  const size_t per_w =
      (fused_kernel ? 0
                    : (size_t)NG * ((size_t)A.P * A.N + (size_t)B.P * B.N) * sizeof(cd)) +
      (size_t)NG * ((size_t)A.nv * A.no + (size_t)B.nv * B.no) * sizeof(cd) +
      (s->mixed && !fused_kernel ? (size_t)NG * ((size_t)A.N * A.N + (size_t)B.N * B.N) * sizeof(cd)
                                 : 0);
  const size_t Xa = (size_t)A.nv * A.no, Xb = (size_t)B.nv * B.no;
  const size_t per_w_all =
      per_w + (s->wform ? 4 * (Xa * Xa + Xa * Xb + Xb * Xb) * sizeof(double) : 0);
  const size_t budget = (size_t)16 << 30;
  int wt = (int)std::max<size_t>(1, std::min<size_t>(NW, budget / std::max<size_t>(per_w_all, 1)));
  if (s->tune.walker_tile > 0) wt = std::min(wt, s->tune.walker_tile);
  s->WT = wt;
  // split the Cholesky range so the second-order workgroups fill whole rounds
  // of the chip's workgroup slots (one 16-wave or two 8-wave workgroups per
  // CU): the best fill of rounds over splits 1 .. 8; on ties the smallest
  // split that makes at least 32 rounds, else the smallest.  Item blocks of
  // different orders cost differently, so the last round runs partly idle;
  // with 32 rounds or more that idle time is a small part of the launch.
  const int units = std::max(1, s->n_itemblocks);
  {
    const int slots = s->n_cu * (wpb == 16 ? 1 : 2);
    double best = -1.0;
    bool best_deep = false;
    for (int gs = 1; gs <= std::min(8, std::max(1, NG / 8)); ++gs) {
      const long nwg = (long)wt * units * gs;
      const long rounds = (nwg + slots - 1) / slots;
      const double fill = (double)nwg / ((double)rounds * slots) - (nwg < slots ? 1.0 : 0.0);
      const bool deep = rounds >= 32;
      if (fill > best + 1e-9 || (fill > best - 1e-9 && deep && !best_deep)) {
        best = std::max(best, fill);
        best_deep = deep;
        s->gsplit = gs;
      }
    }
  }
  if (s->tune.second_gsplit > 0) s->gsplit = std::min(s->tune.second_gsplit, NG);
  s->slot_second = slot;
  slot += s->n_itemblocks * s->gsplit;
  for (int sp = 0; sp < 2 && !s->wform; ++sp) {
    if (s->use_strings[sp]) continue;
    s->slot_min[sp] = slot;
    slot += msd::energy_minor_blocks(s->ds[sp]) * s->gsplit;
  }
  if (s->wform) s->slot_wform = slot++;
  {
    const int X = A.nv * A.no + B.nv * B.no;
    const int elem = s->energy_mixed ? 8 : 16;  // bytes per staged Lambda entry
    // two 8-wave workgroups or one 16-wave workgroup per CU share its LDS
    const int budget_lds = s->second_waves == 16 ? (144 << 10) : (72 << 10);
    s->second_G = std::max(1, std::min(8, (int)(budget_lds / (2 * elem * std::max(X, 1)))));
    if (s->tune.second_stage > 0)
      s->second_G = std::max(1, std::min(s->tune.second_stage,
                                         (int)((150 << 10) / (2 * elem * std::max(X, 1)))));
    s->second_flat = s->tune.second_gather == 2;
    s->second_dma = s->tune.second_copy != 1;
  }
  s->gl_parts = 1;
  if (s->tune.lambda_chunk > 0) {
    s->gl_chunk = std::min(s->tune.lambda_chunk, NG);
  } else if (s->lambda_variant == 5) {
    // workgroups of four walkers and one spin: about two per CU (four in FP32)
    const int n_wgrp = 2 * ((wt + 3) / 4), target = s->energy_mixed ? 1024 : 512;
    const int n_chunks = std::max(1, std::min(NG, (target + n_wgrp / 2) / n_wgrp));
    s->gl_chunk = (NG + n_chunks - 1) / n_chunks;
  } else if (s->lambda_variant == 6) {
    // one workgroup per (spin, walker, chunk): about four per CU over the launch
    const int n_wgrp = 2 * wt, target = 4 * s->n_cu;
    const int n_chunks = std::max(1, std::min(NG, (target + n_wgrp / 2) / n_wgrp));
    s->gl_chunk = (NG + n_chunks - 1) / n_chunks;
  } else {
    s->gl_chunk = std::min(32, NG);
  }
  s->n_lchunks = (NG + s->gl_chunk - 1) / s->gl_chunk;
  if (s->lambda_variant == 6) {
    s->gl_parts = msd::ltl_general_parts(A, B);
    s->n_lchunks *= s->gl_parts;  // one partial of sum C . ZW per (chunk, wave)
  }
  // only the row-pair / pair second-order kernel reads the windows then (the
  // minor-list form indexes them unswizzled)
  s->lam_swz = 0;
  if (s->use_strings[0] && s->use_strings[1]) {
    if (s->lambda_variant == 5 && A.no == 8 && B.no == 8) s->lam_swz = 1;
    if (s->lambda_variant == 6)
      s->lam_swz = A.no % 16 == 0 && B.no % 16 == 0 ? 2 : A.no % 8 == 0 && B.no % 8 == 0 ? 1 : 0;
  }
  // the mixed form's FP64 pass for walkers far from the reference (general kernel)
  s->guard = s->energy_mixed && s->lambda_variant == 6 && s->gl_fits && s->tmax > 0.0;
  s->n_slots_main = slot;
  if (s->guard && s->wform) {
    s->slot_guard = s->slot_wform;
    s->slot_guard_end = s->slot_wform + 1;
  } else if (s->guard) {
    // the FP64 pass may have a handful of walkers: split their Cholesky range
    // finely enough that they still spread over the chip
    s->gsplit_guard = std::max(s->gsplit, std::min(16, std::max(1, NG / 16)));
    s->slot_guard = slot;
    slot += s->n_itemblocks * s->gsplit_guard;
    s->slot_guard_end = slot;
  }
  s->n_slots = slot;  // every slot is written by exactly one workgroup of its pass
  Arena& E = s->energy_mem;
  for (int sp = 0; sp < 2; ++sp) {
    const msd::DevSpin& D = s->ds[sp];
    int wbf = 0;
    if (s->energy_mixed) {
      if (!fused_kernel) s->LT32[sp] = E.get<cf>((size_t)NG * D.P * wt * D.N);
      s->Lam32[sp] = E.get<cf>((size_t)wt * NG * D.nv * D.no);
      if (!fused_kernel) s->Q64[sp] = E.get<cd>((size_t)NG * D.N * wt * D.N);
    } else {
      if (!(s->o.energy_algo == 3 && msd::chol_contract_fits(s->ds[0], s->ds[1], &wbf)) &&
          !fused_kernel)
        s->LT[sp] = E.get<cd>((size_t)NG * D.P * wt * D.N);
      s->Lam[sp] = E.get<cd>((size_t)wt * NG * D.nv * D.no);
    }
    if (!fused_kernel) s->ZWp[sp] = E.get<cd>((size_t)wt * s->n_lchunks * D.nv * D.no);
    s->coef2[sp] = E.get<cd>((size_t)NW * D.n_minor);
  }
  if (s->guard) {
    for (int sp = 0; sp < 2; ++sp)
      s->Lam[sp] = E.get<cd>((size_t)wt * NG * s->ds[sp].nv * s->ds[sp].no);
    // the FP64 pass may have few walkers: split their vectors more finely so
    // that a handful of walkers still spreads over the chip
    const int n_chunks = std::max(1, std::min(NG, 48));
    s->gl_chunk_guard = (NG + n_chunks - 1) / n_chunks;
    s->n_lchunks_guard = (NG + s->gl_chunk_guard - 1) / s->gl_chunk_guard * s->gl_parts;
    const int X = A.nv * A.no + B.nv * B.no;
    const int budget_lds = s->second_waves == 16 ? (144 << 10) : (72 << 10);
    s->second_G64 = std::max(1, std::min(8, (int)(budget_lds / (2 * 16 * std::max(X, 1)))));
  }
  if (s->wform) {
    s->Gw[0] = E.get<double>((size_t)wt * 4 * Xa * Xa);
    s->Gw[1] = E.get<double>((size_t)wt * 4 * Xa * Xb);
    s->Gw[2] = E.get<double>((size_t)wt * 4 * Xb * Xb);
  }
  // the general kernel writes v0 and ex0 as per-wave partials
  s->v0 = E.get<cd>((size_t)2 * NW * NG * s->gl_parts);
  if (fused_kernel)
    s->czw = E.get<cd>((size_t)2 * NW * std::max(s->n_lchunks, s->n_lchunks_guard));
  if (s->lambda_variant == 6) s->lamc = E.get<cd>((size_t)2 * NW * NG * s->gl_parts);
  s->ex0 = E.get<cd>((size_t)2 * NW * NG * s->gl_parts);
  s->coefAB = E.get<cd>((size_t)NW * s->dp.n_pair);
  // pair coefficients with the walkers on the lanes where the pairs have 16
  // or more entries each on average (large trials with high orders)
  const int64_t n_ent = s->tt.pr_ptr.empty() ? 0 : s->tt.pr_ptr.back();
  s->adjT[0] = s->adjT[1] = nullptr;
  if (np > 0 && n_ent >= (int64_t)16 * np)
    for (int sp = 0; sp < 2; ++sp)
      s->adjT[sp] = E.get<cd>((size_t)std::max(s->ds[sp].A, 1) * NW);
  s->epart = E.get<cd>((size_t)NW * std::max(s->n_slots, 1));
  s->plan = E.upload(s->plan_host, s->st);
}

void need_ready(msd_system* s) {
  if (!s->have_ham) fail(MSD_ERR_STATE, "msd_set_hamiltonian has not been called");
  if (!s->have_trial) fail(MSD_ERR_STATE, "msd_set_trial_occ has not been called");
  build_derived(s);
}

void clear_flags(msd_system* s) { msd::launch_fill_i32(s->flag, s->NW, 0, s->st); }

// Runs `body` once on the handle's stream, or, with graphs on, replays the
// graph of `slot` (capturing it first, on the private stream, if it is missing
// or was made for other dt / e_shift).  Everything `body` allocates must be
// allocated before (the caller prepares lazily-sized buffers).
template <class F>
void run_or_replay(msd_system* s, msd_system::GraphSlot& slot, double dt, double e_shift,
                   F&& body) {
  if (!s->graphs_on()) {
    body();
    return;
  }
  if (slot.exec && (slot.dt != dt || slot.e_shift != e_shift)) {
    hip_check(hipGraphExecDestroy(slot.exec), "hipGraphExecDestroy");
    slot.exec = nullptr;
  }
  if (!slot.exec) {
    if (!s->cap_st) hip_check(hipStreamCreateWithFlags(&s->cap_st, hipStreamNonBlocking), "stream");
    hipStream_t user = s->st;
    s->st = s->cap_st;
    hipGraph_t g = nullptr;
    hip_check(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      body();
    } catch (...) {
      (void)hipStreamEndCapture(s->st, &g);
      if (g) (void)hipGraphDestroy(g);
      s->st = user;
      throw;
    }
    s->st = user;
    hip_check(hipStreamEndCapture(s->cap_st, &g), "end capture");
    hipError_t e = hipGraphInstantiate(&slot.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "hipGraphInstantiate");
    slot.dt = dt;
    slot.e_shift = e_shift;
  }
  hip_check(hipGraphLaunch(slot.exec, s->st), "hipGraphLaunch");
}

void check_flags(msd_system* s, const char* what) {
  std::vector<int> f(s->NW);
  hip_check(hipMemcpyAsync(f.data(), s->flag, sizeof(int) * s->NW, hipMemcpyDeviceToHost, s->st),
            "flags");
  s->sync();
  for (int w = 0; w < s->NW; ++w)
    if (f[w])
      fail(MSD_ERR_SINGULAR, std::string(what) + ": walker " + std::to_string(w) +
                                 " has a singular reference block or zero trial overlap");
}

// A1 + A3: T, log det A, per-string dets/adjugates (minors if requested),
// Obar and log <Psi_T|Phi> into `logo_out`.
void run_overlap(msd_system* s, bool minors, cd* logo_out, bool skip_ref = false) {
  if (!skip_ref)
    s->timed(ST_REF, [&] {
      msd::launch_ref_inverse(s->phi, s->M, s->Ntot, s->NW, s->ds[0], s->ds[1], s->sw[0].T,
                              s->sw[1].T, s->sw[0].logdetA, s->sw[1].logdetA, s->flag, s->st);
    });
  s->timed(ST_STR, [&] {
    msd::launch_strings(s->ds[0], s->ds[1], s->sw[0].T, s->sw[1].T, s->NW, minors, s->sw[0],
                        s->sw[1], s->st);
  });
  s->timed(ST_OVLP, [&] {
    msd::launch_ovlp_partial(s->ND, s->NW, s->ds[0].det_s, s->ds[1].det_s, s->det_c,
                             s->sw[0].d, s->ds[0].U, s->sw[1].d, s->ds[1].U, s->opart,
                             s->n_ochunks, s->ochunk, s->st);
    msd::launch_ovlp_final(s->NW, s->opart, s->n_ochunks, s->na ? s->sw[0].logdetA : nullptr,
                           s->nb ? s->sw[1].logdetA : nullptr, s->obar, logo_out, s->flag,
                           s->st);
  });
  s->check_launch("overlap");
}

// A4 + A5: CI weights, CI matrices, Green's rows, force bias into s->xbar.
void run_green_fb(msd_system* s, double dt) {
  s->timed(ST_CIW, [&] {
    msd::launch_ci_weights(s->ds[0], s->ds[1], s->det_c, s->sw[0], s->sw[1], s->segp[0],
                           s->segp[1], s->NW, s->st);
  });
  s->timed(ST_CIM, [&] { msd::launch_ci_matrix(s->ds[0], s->ds[1], s->NW, s->sw[0], s->sw[1], s->st); });
  s->timed(ST_GREEN, [&] {
    msd::launch_green(s->ds[0], s->ds[1], s->M, s->NW, s->sw[0], s->sw[1], s->onebody, s->obar,
                      s->h1, s->ob_part, s->st);
  });
  s->timed(ST_GREEN, [&] {
    msd::launch_green_sum(s->M, s->NW, s->P_all, s->rmap[0], s->rmap[1], s->ds[0].P,
                          s->ds[1].P, s->sw[0].G, s->sw[1].G, s->Gp, s->st);
  });
  if (s->mixed) {
    s->timed(ST_FB_GEMM, [&] {
      msd::launch_f64_to_f32(s->Gp, s->Gp32, (int64_t)2 * s->NW * s->P_all * s->M, s->st);
      msd::GemmArgs32 g;
      g.M = s->NG;
      g.N = 2 * s->NW;
      g.K = s->P_all * s->M;
      g.A = s->Lrows32;
      g.lda = g.K;
      g.a_kmaj = true;
      g.B = s->Gp32;
      g.ldb = g.K;
      g.b_kmaj = true;
      g.C64 = s->xraw;
      g.ldc = 2 * s->NW;
      g.splitk = s->fb_splitk;
      g.ws = s->fb_ws32;
      msd::launch_gemm32(g, s->st);
      msd::launch_xbar(s->NW, s->NG, s->xraw, std::sqrt(dt), s->xbar, s->st);
    });
    s->check_launch("green/force bias");
    return;
  }
  s->timed(ST_FB_GEMM, [&] {
    msd::GemmArgs g;
    g.M = s->NG;
    g.N = 2 * s->NW;
    g.K = s->P_all * s->M;
    g.A = s->L_rows;
    g.lda = g.K;
    g.a_kmaj = true;
    g.B = s->Gp;
    g.ldb = g.K;
    g.b_kmaj = true;
    g.C = s->xraw;
    g.ldc = 2 * s->NW;
    g.splitk = s->fb_splitk;
    g.ws = s->fb_ws;
    msd::launch_gemm(g, s->st);
    msd::launch_xbar(s->NW, s->NG, s->xraw, std::sqrt(dt), s->xbar, s->st);
  });
  s->check_launch("green/force bias");
}

void run_wform(msd_system* s, int w0, int wt, bool fp32, const int* wmask);

// A6 + A7 in the mixed form: FP32 copies of T, FP32 MFMA LT GEMM, FP32 Lambda
// and second-order Cholesky sums; v0, ex0, ZW, cofactors and the assembly in
// FP64.
void run_energy_mixed(msd_system* s) {
  const msd::DevSpin& A = s->ds[0];
  const msd::DevSpin& B = s->ds[1];
  // with the FP64 pass, the single-precision kernels skip the walkers it takes
  const int* fm = s->guard ? s->fmask : nullptr;
  int nmax = 0;
  msd::lambda_rows_fits(A, B, &nmax);
  s->timed(ST_LT_GEMM, [&] {
    for (int sp = 0; sp < 2; ++sp)
      msd::launch_f64_to_f32(reinterpret_cast<const double*>(s->sw[sp].T), s->T32[sp],
                             (int64_t)2 * s->M * s->NW * s->ds[sp].N, s->st);
  });
  for (int w0 = 0; w0 < s->NW; w0 += s->WT) {
    const int wt = std::min(s->WT, s->NW - w0);
    for (int sp = 0; sp < 2; ++sp) {
      const msd::DevSpin& D = s->ds[sp];
      if (D.N == 0) continue;
      s->timed(ST_LT_GEMM, [&] {
        if (s->lambda_variant < 5) {  // the fused kernels form LT themselves
        msd::GemmArgs32 g;
        g.M = s->NG * D.P;
        g.N = 2 * wt * D.N;
        g.K = s->M;
        g.A = s->Llt32[sp];
        g.lda = s->M;
        g.a_kmaj = true;
        g.B = s->T32[sp] + (size_t)2 * w0 * D.N;
        g.ldb = 2 * (int64_t)s->NW * D.N;
        g.b_kmaj = false;
        g.C32 = reinterpret_cast<float*>(s->LT32[sp]);
        g.c_block = 2 * D.N;  // LT tile of (walker, vector) contiguous: [wl][g][p][n]
        msd::launch_gemm32(g, s->st);
        }
        if (s->lambda_variant >= 5) return;  // traces from launch_qtr / the general kernel
        // FP64 Q = L[R, :] T for the mean-field traces
        msd::GemmArgs q;
        q.M = s->NG * D.N;
        q.N = 2 * wt * D.N;
        q.K = s->M;
        q.A = s->LR64[sp];
        q.lda = s->M;
        q.a_kmaj = true;
        q.B = reinterpret_cast<const double*>(s->sw[sp].T + (size_t)w0 * D.N);
        q.ldb = 2 * (int64_t)s->NW * D.N;
        q.b_kmaj = false;
        q.C = reinterpret_cast<double*>(s->Q64[sp]);
        q.c_block = 2 * D.N;
        msd::launch_gemm(q, s->st);
      });
    }
    if (s->lambda_variant == 5) {  // FP64 traces first: the fused kernel reads v0
      s->timed(ST_TRACES, [&] {
        msd::launch_qtr(s->NW, w0, wt, s->NG, s->M, s->Slr[0], s->Slr[1], s->sw[0].T, s->sw[1].T,
                        s->v0, s->ex0, s->n_cu, s->st);
      });
    }
    s->timed(ST_LAMBDA, [&] {
      const cf* Ta = reinterpret_cast<const cf*>(s->T32[0]);
      const cf* Tb = reinterpret_cast<const cf*>(s->T32[1]);
      if (s->lambda_variant == 6) {
        msd::launch_ltl_general32(A, B, s->NW, w0, wt, s->NG, s->gl_chunk, s->M, s->Sgl32[0],
                                  s->Sgl32[1], Ta, Tb, s->Lam32[0], s->Lam32[1], s->sw[0].C,
                                  s->sw[1].C, s->v0, s->ex0, s->lamc, s->czw, fm, s->lam_swz,
                                  s->st);
      } else if (s->lambda_variant == 5) {
        msd::launch_ltl_mfma32(A, B, s->NW, w0, wt, s->NG, s->gl_chunk, s->M, s->Slf32[0],
                               s->Slf32[1], Ta, Tb, s->Lam32[0], s->Lam32[1], s->v0, s->sw[0].C,
                               s->sw[1].C, s->czw, s->lam_swz != 0, s->st);
      } else if (s->lambda_variant == 0)
        msd::launch_lambda32(A, B, s->NW, w0, wt, s->NG, s->gl_chunk, Ta, Tb, s->LT32[0],
                             s->LT32[1], s->Lam32[0], s->Lam32[1], s->v0, s->ex0, s->ZWp[0],
                             s->ZWp[1], s->st);
      else
        msd::launch_lambda_rows32(A, B, nmax, s->NW, w0, wt, s->NG, s->gl_chunk, Ta, Tb,
                                  s->LT32[0], s->LT32[1], s->Lam32[0], s->Lam32[1], s->v0, s->ex0,
                                  s->ZWp[0], s->ZWp[1], s->st);
    });
    if (s->lambda_variant < 5) {  // the fused kernels form the traces themselves
      s->timed(ST_TRACES, [&] {
        msd::launch_traces64(s->Q64[0], s->Q64[1], A.N, B.N, s->NW, w0, wt, s->NG, s->v0, s->ex0,
                             s->st);
      });
    }
    s->timed(ST_EGAMMA, [&] {
      if (s->wform) {
        run_wform(s, w0, wt, true, fm);
        return;
      }
      msd::launch_energy_second32(A, B, s->dp, s->plan, s->n_itemblocks, s->second_waves, s->NW,
                                  w0, wt, s->NG, s->gsplit, s->second_G, s->second_maxk,
                                  s->second_flat, s->second_dma, s->lam_swz,
                                  s->Lam32[0],
                                  s->Lam32[1], s->coefAB, s->sw[0].m2, s->sw[1].m2, s->sw[0].B,
                                  s->sw[1].B, s->epart, s->n_slots, s->slot_second, s->st, fm);
    });
    s->timed(ST_EFINAL, [&] {
      msd::launch_energy_final(A, B, s->NW, w0, wt, s->NG, s->n_lchunks, s->n_slots, 0,
                               s->n_slots_main, s->obar,
                               s->v0, s->ex0, s->ZWp[0], s->ZWp[1], s->sw[0].C, s->sw[1].C,
                               s->lambda_variant >= 5 ? s->czw : nullptr, s->epart, s->onebody,
                               s->onebody + s->NW, s->e0, s->eloc,
                               s->lambda_variant == 6 ? s->lamc : nullptr, s->gl_parts, s->st,
                               fm);
    });
  }
  s->check_launch("energy");
}

// W-form for the walker tile [w0, w0 + wt): the three per-walker GEMMs of the
// Lambda windows (FP64, or FP32 with double output in the mixed form) and
// the contraction with the coefficient lists.
void run_wform(msd_system* s, int w0, int wt, bool fp32, const int* wmask) {
  const msd::DevSpin& A = s->ds[0];
  const msd::DevSpin& B = s->ds[1];
  const int X[2] = {A.nv * A.no, B.nv * B.no};
  const int pairs[3][2] = {{0, 0}, {0, 1}, {1, 1}};
  for (int q = 0; q < 3; ++q) {
    const int sa = pairs[q][0], sb = pairs[q][1];
    if (X[sa] == 0 || X[sb] == 0) continue;
    if (fp32) {
      msd::GemmArgs32 g;
      g.M = 2 * X[sa];
      g.N = 2 * X[sb];
      g.K = s->NG;
      g.batch = wt;
      g.A = reinterpret_cast<const float*>(s->Lam32[sa]);
      g.lda = 2 * X[sa];
      g.a_kmaj = false;
      g.strideA = (int64_t)s->NG * 2 * X[sa];
      g.B = reinterpret_cast<const float*>(s->Lam32[sb]);
      g.ldb = 2 * X[sb];
      g.b_kmaj = false;
      g.strideB = (int64_t)s->NG * 2 * X[sb];
      g.C64 = s->Gw[q];
      g.ldc = 2 * X[sb];
      g.strideC = (int64_t)4 * X[sa] * X[sb];
      g.mask = wmask ? wmask + w0 : nullptr;
      msd::launch_gemm32(g, s->st);
    } else {
      msd::GemmArgs g;
      g.M = 2 * X[sa];
      g.N = 2 * X[sb];
      g.K = s->NG;
      g.batch = wt;
      g.A = reinterpret_cast<const double*>(s->Lam[sa]);
      g.lda = 2 * X[sa];
      g.a_kmaj = false;
      g.strideA = (int64_t)s->NG * 2 * X[sa];
      g.B = reinterpret_cast<const double*>(s->Lam[sb]);
      g.ldb = 2 * X[sb];
      g.b_kmaj = false;
      g.strideB = (int64_t)s->NG * 2 * X[sb];
      g.C = s->Gw[q];
      g.ldc = 2 * X[sb];
      g.strideC = (int64_t)4 * X[sa] * X[sb];
      g.mask = wmask ? wmask + w0 : nullptr;
      msd::launch_gemm(g, s->st);
    }
  }
  msd::launch_wform_contract(A, B, s->dp, s->NW, w0, wt, s->Gw[0], s->Gw[1], s->Gw[2], s->coefAB,
                             s->coef2[0], s->coef2[1], s->epart, s->n_slots, s->slot_wform, s->st,
                             wmask);
}

// Mixed form: FP64 local energies for the walkers whose largest |T| exceeds
// tmax (the FP32 rounding of Q, Lambda and their products grows with |T|^2),
// through the general contraction kernel and the FP64 second-order kernel,
// every kernel skipping the walkers the mask leaves out (the single-precision
// pass skips exactly these walkers, so each walker is evaluated once).
void run_energy_guard(msd_system* s) {
  const msd::DevSpin& A = s->ds[0];
  const msd::DevSpin& B = s->ds[1];
  // the walkers of this pass as a list (persistent grids over their work
  // items: no launch of idle workgroups for the walkers left out)
  msd::WalkerList wls;
  wls.list = s->glist;
  wls.count = s->glist + s->NW;
  wls.n_cu = s->n_cu;
  s->timed(ST_GUARD, [&] {
    for (int w0 = 0; w0 < s->NW; w0 += s->WT) {
      const int wt = std::min(s->WT, s->NW - w0);
      msd::launch_ltl_general(A, B, s->NW, w0, wt, s->NG, s->gl_chunk_guard, s->M, s->Sgl[0],
                              s->Sgl[1], s->sw[0].T, s->sw[1].T, s->Lam[0], s->Lam[1], s->sw[0].C,
                              s->sw[1].C, s->v0, s->ex0, s->lamc, s->czw, s->gmask, s->lam_swz,
                              s->st, wls);
      if (s->wform)
        run_wform(s, w0, wt, false, s->gmask);
      else
        msd::launch_energy_second(A, B, s->dp, s->plan, s->n_itemblocks, s->second_waves, s->NW,
                                  w0, wt, s->NG, s->gsplit_guard, s->second_G64, s->second_maxk,
                                  s->second_flat, s->second_dma, s->lam_swz, s->Lam[0], s->Lam[1],
                                  s->coefAB, s->sw[0].m2, s->sw[1].m2, s->sw[0].B, s->sw[1].B,
                                  s->epart, s->n_slots, s->slot_guard, s->st, s->gmask, wls);
      msd::launch_energy_final(A, B, s->NW, w0, wt, s->NG, s->n_lchunks_guard, s->n_slots,
                               s->slot_guard, s->slot_guard_end,
                               s->obar, s->v0, s->ex0, s->ZWp[0], s->ZWp[1], s->sw[0].C,
                               s->sw[1].C, s->czw, s->epart, s->onebody, s->onebody + s->NW,
                               s->e0, s->eloc, s->lamc, s->gl_parts, s->st, s->gmask);
    }
  });
  s->check_launch("energy (FP64 pass)");
}

// A6 + A7: local energies into s->eloc (needs run_overlap with minors and run_green_fb).
void run_energy(msd_system* s) {
  alloc_energy(s);
  const msd::DevSpin& A = s->ds[0];
  const msd::DevSpin& B = s->ds[1];
  s->timed(ST_COEF, [&] {
    msd::launch_pair_coef(s->dp, s->NW, s->det_c, s->sw[0].adj, A.A, s->sw[1].adj, B.A,
                          s->coefAB, s->st, s->adjT[0], s->adjT[1]);
    for (int sp = 0; sp < 2; ++sp)
      if (!s->use_strings[sp])
        msd::launch_minor_coef(s->ds[sp], s->NW, s->sw[sp].B, s->ds[sp].U, s->sw[sp].m2,
                               s->coef2[sp], s->st);
  });
  if (s->energy_mixed) {
    if (s->guard)  // which walkers go to the FP64 pass (gmask) and which stay (fmask)
      s->timed(ST_GUARD, [&] {
        msd::launch_walker_tmax(s->NW, s->M, A.N, B.N, s->sw[0].T, s->sw[1].T, s->tmax,
                                s->gmask, s->fmask, s->glist, s->glist + s->NW, s->st);
      });
    run_energy_mixed(s);
    if (s->guard) run_energy_guard(s);
    return;
  }
  int wb = 0;
  const bool fused = s->o.energy_algo == 3 && msd::chol_contract_fits(A, B, &wb);
  for (int w0 = 0; w0 < s->NW; w0 += s->WT) {
    const int wt = std::min(s->WT, s->NW - w0);
    if (fused) {
      s->timed(ST_LAMBDA, [&] {
        msd::launch_chol_contract(A, B, s->L_lt[0], s->L_lt[1], s->sw[0].T, s->sw[1].T, s->Lam[0],
                                  s->Lam[1], s->ZWp[0], s->ZWp[1], s->M, s->NW, w0, wt, s->NG,
                                  s->gl_chunk, wb, s->v0, s->ex0, s->st);
      });
    } else {
      for (int sp = 0; sp < 2 && s->lambda_variant < 5; ++sp) {
        const msd::DevSpin& D = s->ds[sp];
        if (D.N == 0) continue;
        s->timed(ST_LT_GEMM, [&] {
          msd::GemmArgs g;
          g.M = s->NG * D.P;
          g.N = 2 * wt * D.N;
          g.K = s->M;
          g.A = s->L_lt[sp];
          g.lda = s->M;
          g.a_kmaj = true;
          g.B = reinterpret_cast<const double*>(s->sw[sp].T + (size_t)w0 * D.N);
          g.ldb = 2 * (int64_t)s->NW * D.N;
          g.b_kmaj = false;
          g.C = reinterpret_cast<double*>(s->LT[sp]);
          g.c_block = 2 * D.N;  // LT tile of (walker, vector) contiguous: [wl][g][p][n]
          msd::launch_gemm(g, s->st);
        });
      }
      int nmax = 0;
      if (s->lambda_variant == 5) {  // FP64 traces first: the fused kernel reads v0
        s->timed(ST_TRACES, [&] {
          msd::launch_qtr(s->NW, w0, wt, s->NG, s->M, s->Slr[0], s->Slr[1], s->sw[0].T,
                          s->sw[1].T, s->v0, s->ex0, s->n_cu, s->st);
        });
      }
      s->timed(ST_LAMBDA, [&] {
        if (s->lambda_variant == 6) {
          msd::launch_ltl_general(A, B, s->NW, w0, wt, s->NG, s->gl_chunk, s->M, s->Sgl[0],
                                  s->Sgl[1], s->sw[0].T, s->sw[1].T, s->Lam[0], s->Lam[1],
                                  s->sw[0].C, s->sw[1].C, s->v0, s->ex0, s->lamc, s->czw,
                                  nullptr, s->lam_swz, s->st);
        } else if (s->lambda_variant == 5) {
          msd::launch_ltl_mfma(A, B, s->NW, w0, wt, s->NG, s->gl_chunk, s->M, s->Slf[0],
                               s->Slf[1], s->sw[0].T, s->sw[1].T, s->Lam[0], s->Lam[1], s->v0,
                               s->sw[0].C, s->sw[1].C, s->czw, s->lam_swz != 0, s->st);
        } else if (s->lambda_variant == 1 && msd::lambda_rows_fits(A, B, &nmax))
          msd::launch_lambda_rows(A, B, nmax, s->NW, w0, wt, s->NG, s->gl_chunk, s->sw[0].T,
                                  s->sw[1].T, s->LT[0], s->LT[1], s->Lam[0], s->Lam[1], s->v0,
                                  s->ex0, s->ZWp[0], s->ZWp[1], s->st);
        else
          msd::launch_lambda(A, B, s->NW, w0, wt, s->NG, s->gl_chunk, s->sw[0].T, s->sw[1].T,
                             s->LT[0], s->LT[1], s->Lam[0], s->Lam[1], s->v0, s->ex0, s->ZWp[0],
                             s->ZWp[1], s->st);
      });
    }
    s->timed(ST_EGAMMA, [&] {
      if (s->wform) {
        run_wform(s, w0, wt, false, nullptr);
        return;
      }
      msd::launch_energy_second(A, B, s->dp, s->plan, s->n_itemblocks, s->second_waves, s->NW, w0,
                                wt, s->NG, s->gsplit, s->second_G, s->second_maxk,
                                s->second_flat, s->second_dma, s->lam_swz, s->Lam[0],
                                s->Lam[1],
                                s->coefAB, s->sw[0].m2, s->sw[1].m2, s->sw[0].B, s->sw[1].B,
                                s->epart, s->n_slots, s->slot_second, s->st);
      for (int sp = 0; sp < 2; ++sp) {
        const msd::DevSpin& D = s->ds[sp];
        if (D.nv * D.no == 0 || s->use_strings[sp]) continue;
        msd::launch_energy_minors(D, s->NW, w0, wt, s->NG, s->gsplit, s->Lam[sp], s->coef2[sp],
                                  s->epart, s->n_slots, s->slot_min[sp], s->st);
      }
    });
    s->timed(ST_EFINAL, [&] {
      msd::launch_energy_final(A, B, s->NW, w0, wt, s->NG, s->n_lchunks, s->n_slots, 0,
                               s->n_slots_main, s->obar,
                               s->v0, s->ex0, s->ZWp[0], s->ZWp[1], s->sw[0].C, s->sw[1].C,
                               s->lambda_variant >= 5 ? s->czw : nullptr, s->epart, s->onebody,
                               s->onebody + s->NW, s->e0, s->eloc,
                               s->lambda_variant == 6 ? s->lamc : nullptr, s->gl_parts, s->st);
    });
  }
  s->check_launch("energy");
}

// The measurement kernels (A1-A7) into logo_tmp, xbar, eloc.
void measure_body(msd_system* s, double dt, bool want_e) {
  // with T fresh the flags of the pass that made it still describe the walkers
  if (!s->t_fresh) clear_flags(s);
  run_overlap(s, want_e, s->logo_tmp, s->t_fresh);
  s->t_fresh = true;
  run_green_fb(s, dt);
  if (want_e) run_energy(s);
}

void measure_impl(msd_system* s, double dt, bool want_e) {
  need_ready(s);
  if (!s->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
  if (!(dt >= 0.0) || !std::isfinite(dt)) fail(MSD_ERR_ARG, "dt must be finite and >= 0");
  if (want_e && s->tt.max_k() > msd::KMAX) fail(MSD_ERR_UNSUPPORTED, "excitation order too high");
  if (want_e) alloc_energy(s);
  run_or_replay(s, s->g_measure[want_e ? 1 : 0][s->t_fresh ? 1 : 0], dt, 0.0,
                [&] { measure_body(s, dt, want_e); });
  s->t_fresh = true;
}

void ensure_b1(msd_system* s, double dt) {
  if (s->B1_dt == dt) return;
  const int M = s->M;
  std::vector<double> a((size_t)M * M);
  for (size_t i = 0; i < a.size(); ++i) a[i] = -0.5 * dt * (s->h1_host[i] - 0.5 * s->sumll_host[i]);
  std::vector<double> b1 = expm_host(a, M);
  hip_check(hipMemcpyAsync(s->B1, b1.data(), b1.size() * sizeof(double), hipMemcpyHostToDevice,
                           s->st),
            "B1 upload");
  s->sync();
  s->B1_dt = dt;
}

void one_body_gemm(msd_system* s, const cd* in, cd* out, const int* mask) {
  msd::GemmArgs g;
  g.M = s->M;
  g.N = 2 * s->Ntot;
  g.K = s->M;
  g.batch = s->NW;
  g.A = s->B1;
  g.lda = s->M;
  g.strideA = 0;
  g.a_kmaj = true;
  g.B = reinterpret_cast<const double*>(in);
  g.ldb = 2 * s->Ntot;
  g.strideB = 2 * (int64_t)s->M * s->Ntot;
  g.b_kmaj = false;
  g.C = reinterpret_cast<double*>(out);
  g.ldc = 2 * s->Ntot;
  g.strideC = 2 * (int64_t)s->M * s->Ntot;
  g.mask = mask;
  msd::launch_gemm(g, s->st);
}

// One propagation step (force bias, VHS, B1 exp_T(VHS) B1, new overlap,
// phaseless weights, QR if `qr`).
void propagate_step(msd_system* s, const double* x, double dt, double e_shift, bool qr) {
  const int NW = s->NW, NG = s->NG, M = s->M, Ntot = s->Ntot;
  const size_t mm = (size_t)M * M;
  clear_flags(s);
  msd::launch_frozen_mask(NW, s->weights, s->mask, s->st);
  // the overlap pass at the current walkers (the force bias needs T, the
  // determinants and Obar), unless the last pass left them valid
  if (!s->t_fresh) run_overlap(s, false, s->logo_tmp);
  run_green_fb(s, dt);
  s->timed(ST_VHS_GEMM, [&] {
    msd::launch_vhs_prep(NW, NG, x, s->xbar, std::sqrt(dt), s->weights, s->Y, s->st);
    if (s->mixed) {
      msd::launch_f64_to_f32(s->Y, s->Y32, (int64_t)2 * NW * NG, s->st);
      msd::GemmArgs32 g;
      g.M = 2 * NW;
      g.N = (int)mm;
      g.K = NG;
      g.A = s->Y32;
      g.lda = NG;
      g.a_kmaj = true;
      g.B = s->L32;
      g.ldb = (int64_t)mm;
      g.b_kmaj = false;
      g.C64 = s->VHS;
      g.ldc = (int64_t)mm;
      msd::launch_gemm32(g, s->st);
      return;
    }
    msd::GemmArgs g;
    g.M = 2 * NW;
    g.N = (int)mm;
    g.K = NG;
    g.A = s->Y;
    g.lda = NG;
    g.a_kmaj = true;
    g.B = s->L;
    g.ldb = (int64_t)mm;
    g.b_kmaj = false;
    g.C = s->VHS;
    g.ldc = (int64_t)mm;
    msd::launch_gemm(g, s->st);
  });
  s->timed(ST_B1, [&] { one_body_gemm(s, s->phi, s->term[0], s->mask); });
  s->timed(ST_TAYLOR, [&] {
    hip_check(hipMemcpyAsync(s->acc, s->term[0], sizeof(cd) * NW * M * Ntot,
                             hipMemcpyDeviceToDevice, s->st),
              "copy");
    for (int n = 1; n <= s->o.n_taylor; ++n) {
      msd::GemmArgs g;
      g.M = M;
      g.N = 2 * Ntot;
      g.K = M;
      g.batch = NW;
      g.A = s->VHS;
      g.lda = M;
      g.strideA = 2 * (int64_t)mm;
      g.a_imag_off = (int64_t)mm;
      g.a_kmaj = true;
      g.B = reinterpret_cast<const double*>(s->term[(n - 1) & 1]);
      g.ldb = 2 * Ntot;
      g.strideB = 2 * (int64_t)M * Ntot;
      g.b_kmaj = false;
      g.C = reinterpret_cast<double*>(s->term[n & 1]);
      g.ldc = 2 * Ntot;
      g.strideC = 2 * (int64_t)M * Ntot;
      g.Acc = reinterpret_cast<double*>(s->acc);
      g.alpha = 1.0 / n;
      g.cplx = true;
      g.mask = s->mask;
      msd::launch_gemm(g, s->st);
    }
  });
  s->timed(ST_B1, [&] { one_body_gemm(s, s->acc, s->phi, s->mask); });
  run_overlap(s, false, s->logo_tmp);
  s->timed(ST_WEIGHTS, [&] {
    msd::launch_weights(NW, NG, x, s->xbar, s->logo_tmp, s->logo, s->weights, dt, e_shift,
                        s->st);
  });
  s->t_fresh = true;  // the second pass above; the QR step keeps it
  if (qr) {
    s->timed(ST_QR, [&] {
      msd::launch_qr(s->phi, M, Ntot, NW, s->na, s->nb, s->mask, s->qr_ldet, s->logo,
                     s->sw[0].logdetA, s->sw[1].logdetA, s->st);
    });
  }
}

void propagate_impl(msd_system* s, const double* fields_dev, double dt, double e_shift,
                    int n_steps) {
  need_ready(s);
  if (!s->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
  if (!(dt > 0.0) || !std::isfinite(dt)) fail(MSD_ERR_ARG, "dt must be finite and > 0");
  if (!std::isfinite(e_shift)) fail(MSD_ERR_ARG, "e_shift must be finite");
  if (n_steps < 0) fail(MSD_ERR_ARG, "n_steps must be >= 0");
  ensure_b1(s, dt);
  const int NW = s->NW, NG = s->NG;
  for (int step = 0; step < n_steps; ++step) {
    const double* x = fields_dev + (size_t)step * NW * NG;
    s->steps_done++;
    const bool qr = s->o.stabilize_freq > 0 && s->steps_done % s->o.stabilize_freq == 0;
    if (s->graphs_on() && x != s->fields) {
      // the graph reads its fields from the staging buffer
      hip_check(hipMemcpyAsync(s->fields, x, sizeof(double) * NW * NG, hipMemcpyDeviceToDevice,
                               s->st),
                "fields");
      x = s->fields;
    }
    run_or_replay(s, s->g_step[qr ? 1 : 0][s->t_fresh ? 1 : 0], dt, e_shift, [&] {
      propagate_step(s, x, dt, e_shift, qr);
    });
    s->t_fresh = true;
    s->check_launch("propagate");
  }
}

// Comb population control of the walker state (orbitals, log overlaps,
// weights); parent (device, NW int32) receives the parent of every new walker
// (the handle's scratch if null).  The copies go through the Taylor
// accumulator, which holds nothing between steps.
void comb_impl(msd_system* s, double z, int* parent) {
  need_ready(s);
  if (!s->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
  if (!(z >= 0.0 && z < 1.0)) fail(MSD_ERR_ARG, "comb offset z must lie in [0, 1)");
  int* par = parent ? parent : s->pc_parent;
  s->t_fresh = false;  // walkers are replaced by copies of their parents
  s->timed(ST_POP, [&] {
    msd::launch_comb(s->NW, z, s->weights, s->pc_cum, par, s->phi, s->logo,
                     (int64_t)s->M * s->Ntot, s->acc, s->pc_logo, s->st);
    hip_check(hipMemcpyAsync(s->phi, s->acc, sizeof(cd) * s->NW * s->M * s->Ntot,
                             hipMemcpyDeviceToDevice, s->st),
              "copy");
    hip_check(hipMemcpyAsync(s->logo, s->pc_logo, sizeof(cd) * s->NW, hipMemcpyDeviceToDevice,
                             s->st),
              "copy");
  });
  s->check_launch("population control");
}

// ---------------------------------------------------------------------------
// Population control without allocation: its scratch (running sums, parents,
// parents' log overlaps, the gathered walkers) lives in one file-scope device
// array of NOALLOC_BYTES per GPU instead of the handle's buffers.  The array's
// device address is taken once per device, at handle creation with the device
// current (msd_create), and only that address is passed to kernels or copies.
// Every call on a GPU shares the array (calls that overlap on one GPU race);
// each region is fully written by the call before it is read, so nothing needs
// clearing between calls.
constexpr size_t NOALLOC_BYTES = (size_t)128 << 20;
constexpr int NOALLOC_MAX_DEV = 64;
__device__ __align__(256) unsigned char msd_noalloc_scratch[NOALLOC_BYTES];
void* g_noalloc_ptr[NOALLOC_MAX_DEV] = {};
std::mutex g_noalloc_mu;

void noalloc_init(int dev) {
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return;  // the entry point reports it
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[dev]) return;
  void* p = nullptr;
  hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(msd_noalloc_scratch)), "hipGetSymbolAddress");
  g_noalloc_ptr[dev] = p;
}

size_t noalloc_align(size_t n) { return (n + 255) / 256 * 256; }

void comb_noalloc_impl(msd_system* s, double z, int* parent) {
  need_ready(s);
  if (!s->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
  if (!(z >= 0.0 && z < 1.0)) fail(MSD_ERR_ARG, "comb offset z must lie in [0, 1)");
  void* base = (s->dev >= 0 && s->dev < NOALLOC_MAX_DEV) ? g_noalloc_ptr[s->dev] : nullptr;
  if (!base) fail(MSD_ERR_STATE, "no static scratch address for this device");
  const size_t NW = (size_t)s->NW, per_w = (size_t)s->M * s->Ntot;
  const size_t b_phi = noalloc_align(sizeof(cd) * NW * per_w);
  const size_t b_logo = noalloc_align(sizeof(cd) * NW);
  const size_t b_cum = noalloc_align(sizeof(double) * NW);
  const size_t b_par = noalloc_align(sizeof(int) * NW);
  const size_t need = b_phi + b_logo + b_cum + b_par;
  if (need > NOALLOC_BYTES)
    fail(MSD_ERR_UNSUPPORTED, "population control needs " + std::to_string(need) +
                                  " bytes of scratch; the allocation-free entry point holds " +
                                  std::to_string(NOALLOC_BYTES) + " bytes per GPU");
  unsigned char* b = static_cast<unsigned char*>(base);
  cd* phi_out = reinterpret_cast<cd*>(b);
  cd* logo_out = reinterpret_cast<cd*>(b + b_phi);
  double* cum = reinterpret_cast<double*>(b + b_phi + b_logo);
  int* par = parent ? parent : reinterpret_cast<int*>(b + b_phi + b_logo + b_cum);
  s->t_fresh = false;  // walkers are replaced by copies of their parents
  msd::launch_comb(s->NW, z, s->weights, cum, par, s->phi, s->logo, (int64_t)per_w, phi_out,
                   logo_out, s->st);
  hip_check(hipMemcpyAsync(s->phi, phi_out, sizeof(cd) * NW * per_w, hipMemcpyDeviceToDevice,
                           s->st),
            "copy");
  hip_check(hipMemcpyAsync(s->logo, logo_out, sizeof(cd) * NW, hipMemcpyDeviceToDevice, s->st),
            "copy");
  s->check_launch("population control");
}

void set_walkers_impl(msd_system* s, const cd* pa_dev, const cd* pb_dev, const double* w_dev) {
  if (!s->have_trial || !s->have_ham)
    fail(MSD_ERR_STATE, "msd_set_hamiltonian and msd_set_trial_occ must precede msd_set_walkers");
  s->t_fresh = false;
  msd::launch_copy_walkers(s->NW, s->M, s->Ntot, s->na, s->nb, pa_dev, pb_dev, s->phi, true,
                           nullptr, nullptr, s->st);
  if (w_dev) {
    hip_check(hipMemcpyAsync(s->weights, w_dev, sizeof(double) * s->NW, hipMemcpyDeviceToDevice,
                             s->st),
              "weights");
  } else {
    std::vector<double> ones(s->NW, 1.0);
    hip_check(hipMemcpyAsync(s->weights, ones.data(), sizeof(double) * s->NW,
                             hipMemcpyHostToDevice, s->st),
              "weights");
    s->sync();
  }
  s->have_walkers = true;
  s->steps_done = 0;
  need_ready(s);
  clear_flags(s);
  run_overlap(s, false, s->logo);
  check_flags(s, "msd_set_walkers");
  s->t_fresh = true;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

const char* msd_status_string(msd_status s) {
  switch (s) {
    case MSD_OK: return "ok";
    case MSD_ERR_ARG: return "invalid argument";
    case MSD_ERR_SHAPE: return "inconsistent dimensions";
    case MSD_ERR_TRIAL: return "invalid trial wavefunction";
    case MSD_ERR_SINGULAR: return "singular reference overlap";
    case MSD_ERR_DEVICE: return "device error";
    case MSD_ERR_OOM: return "out of memory";
    case MSD_ERR_STATE: return "call order";
    case MSD_ERR_UNSUPPORTED: return "unsupported shape";
  }
  return "unknown status";
}

const char* msd_last_error(const msd_system* sys) {
  return sys ? sys->err.c_str() : g_err.c_str();
}

msd_status msd_default_options(msd_options* o) {
  if (!o) return MSD_ERR_ARG;
  std::memset(o, 0, sizeof(*o));
  o->n_taylor = 6;
  o->stabilize_freq = 5;
  o->timing = 0;
  return MSD_OK;
}

msd_status msd_create(const msd_dims* d, const msd_options* o, int32_t device, void* hip_stream,
                      msd_system** out) {
  msd_system* sys = nullptr;
  API_BEGIN
  if (!d || !out) fail(MSD_ERR_ARG, "null argument");
  *out = nullptr;
  if (d->M <= 0 || d->n_alpha < 0 || d->n_beta < 0 || d->n_alpha + d->n_beta <= 0 ||
      d->n_chol <= 0 || d->n_walkers <= 0 || d->n_det <= 0)
    fail(MSD_ERR_SHAPE, "all sizes must be positive");
  if (d->n_alpha > d->M || d->n_beta > d->M) fail(MSD_ERR_SHAPE, "more electrons than orbitals");
  if (d->n_alpha > msd::NMAX_LDS || d->n_beta > msd::NMAX_LDS)
    fail(MSD_ERR_UNSUPPORTED, "at most 64 electrons per spin");
  msd_options opt;
  msd_default_options(&opt);
  if (o) opt = *o;
  if (opt.n_taylor < 0 || opt.n_taylor > 32 || opt.stabilize_freq < 0 || opt.energy_algo < 0 ||
      opt.energy_algo > 4 || opt.graphs < 0 || opt.graphs > 1 || opt.precision < 0 ||
      opt.precision > 1 || !std::isfinite(opt.mixed_tmax))
    fail(MSD_ERR_ARG, "invalid options");
  sys = new msd_system();
  sys->dev = device;
  sys->st = static_cast<hipStream_t>(hip_stream);
  sys->d = *d;
  sys->o = opt;
  sys->M = d->M;
  sys->na = d->n_alpha;
  sys->nb = d->n_beta;
  sys->Ntot = d->n_alpha + d->n_beta;
  sys->NG = d->n_chol;
  sys->NW = d->n_walkers;
  sys->ND = d->n_det;
  try {
    set_device(sys);
    hip_check(hipDeviceGetAttribute(&sys->n_cu, hipDeviceAttributeMultiprocessorCount, sys->dev),
              "hipDeviceGetAttribute");
    if (sys->n_cu < 1) sys->n_cu = 1;
    msd::init_wick_attributes();
    msd::init_ltl_attributes();
    msd::init_prop_attributes();
    msd::init_gemm_attributes();
    noalloc_init(sys->dev);
    Arena& A = sys->base;
    const int M = sys->M, NW = sys->NW, NG = sys->NG, Ntot = sys->Ntot;
    sys->phi = A.get<cd>((size_t)NW * M * Ntot);
    sys->weights = A.get<double>(NW);
    sys->logo = A.get<cd>(NW);
    sys->logo_tmp = A.get<cd>(NW);
    sys->pc_cum = A.get<double>(NW);
    sys->pc_parent = A.get<int>(NW);
    sys->pc_logo = A.get<cd>(NW);
    sys->blk = A.get<cd>(2);
    sys->obar = A.get<cd>(NW);
    sys->flag = A.get<int>(NW);
    sys->mask = A.get<int>(NW);
    sys->gmask = A.get<int>(NW);
    sys->fmask = A.get<int>(NW);
    sys->glist = A.get<int>(NW + 1);
    sys->qr_ldet = A.get<double>(2 * (size_t)NW);
    sys->xraw = A.get<double>((size_t)NG * 2 * NW);
    sys->xbar = A.get<cd>((size_t)NW * NG);
    sys->eloc = A.get<cd>(NW);
    sys->onebody = A.get<cd>(2 * (size_t)NW);
    sys->ob_part = A.get<cd>(2 * (size_t)NW * msd::green_tiles(M));
    sys->Y = A.get<double>((size_t)2 * NW * NG);
    sys->VHS = A.get<double>((size_t)2 * NW * M * M);
    sys->term[0] = A.get<cd>((size_t)NW * M * Ntot);
    sys->term[1] = A.get<cd>((size_t)NW * M * Ntot);
    sys->acc = A.get<cd>((size_t)NW * M * Ntot);
    sys->fields = A.get<double>((size_t)NW * NG);
    sys->L = A.get<double>((size_t)NG * M * M);
    sys->h1 = A.get<double>((size_t)M * M);
    sys->B1 = A.get<double>((size_t)M * M);
    for (int sp = 0; sp < 2; ++sp) {
      const int N = sp ? sys->nb : sys->na;
      sys->sw[sp].T = A.get<cd>((size_t)M * NW * std::max(N, 1));
      sys->sw[sp].logdetA = A.get<cd>(NW);
    }
    sys->mixed = opt.precision == 1;
    sys->tmax = opt.mixed_tmax == 0.0 ? 2.0 : opt.mixed_tmax;
    if (sys->mixed) {
      sys->L32 = A.get<float>((size_t)NG * M * M);
      sys->Y32 = A.get<float>((size_t)2 * NW * NG);
      for (int sp = 0; sp < 2; ++sp) {
        const int N = sp ? sys->nb : sys->na;
        sys->T32[sp] = A.get<float>((size_t)2 * M * NW * std::max(N, 1));
      }
    }
    hip_check(hipMemsetAsync(sys->flag, 0, sizeof(int) * NW, sys->st), "memset");
    hip_check(hipMemsetAsync(sys->sw[0].logdetA, 0, sizeof(cd) * NW, sys->st), "memset");
    hip_check(hipMemsetAsync(sys->sw[1].logdetA, 0, sizeof(cd) * NW, sys->st), "memset");
    sys->sync();
  } catch (...) {
    sys->base.release();
    delete sys;
    sys = nullptr;
    throw;
  }
  *out = sys;
  API_END(static_cast<msd_system*>(nullptr))
}

void msd_destroy(msd_system* sys) {
  if (!sys) return;
  (void)hipSetDevice(sys->dev);
  (void)hipStreamSynchronize(sys->st);
  sys->drop_graphs();
  if (sys->cap_st) (void)hipStreamDestroy(sys->cap_st);
  for (auto& p : sys->pending) {
    (void)hipEventDestroy(p.second.first);
    (void)hipEventDestroy(p.second.second);
  }
  for (hipEvent_t e : sys->pool) (void)hipEventDestroy(e);
  sys->energy_mem.release();
  sys->trial_mem.release();
  sys->ham_mem.release();
  sys->base.release();
  delete sys;
}

msd_status msd_set_hamiltonian(msd_system* sys, const double* h1, const double* chol, double e0) {
  API_BEGIN
  if (!sys || !h1 || !chol) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  const int M = sys->M, NG = sys->NG;
  if (!std::isfinite(e0)) fail(MSD_ERR_ARG, "e0 must be finite");
  for (int p = 0; p < M; ++p)
    for (int q = 0; q < M; ++q) {
      const double a = h1[(size_t)p * M + q], b = h1[(size_t)q * M + p];
      if (!std::isfinite(a) || std::fabs(a - b) > 1e-12 * std::max(1.0, std::fabs(a)))
        fail(MSD_ERR_ARG, "h1 not finite/symmetric at (" + std::to_string(p) + "," +
                              std::to_string(q) + ")");
    }
  for (int g = 0; g < NG; ++g) {
    const double* Lg = chol + (size_t)g * M * M;
    for (int p = 0; p < M; ++p)
      for (int q = p; q < M; ++q) {
        const double a = Lg[(size_t)p * M + q], b = Lg[(size_t)q * M + p];
        if (!std::isfinite(a) || std::fabs(a - b) > 1e-12 * std::max(1.0, std::fabs(a)))
          fail(MSD_ERR_ARG, "Cholesky vector " + std::to_string(g) + " not finite/symmetric at (" +
                                std::to_string(p) + "," + std::to_string(q) + ")");
      }
  }
  hip_check(hipMemcpyAsync(sys->L, chol, sizeof(double) * NG * M * M, hipMemcpyHostToDevice,
                           sys->st),
            "upload L");
  hip_check(hipMemcpyAsync(sys->h1, h1, sizeof(double) * M * M, hipMemcpyHostToDevice, sys->st),
            "upload h1");
  sys->h1_host.assign(h1, h1 + (size_t)M * M);
  sys->e0 = e0;
  std::vector<double> tmp((size_t)M * M);
  // sum_g L^g L^g = S^T S with S the (NG*M) x M stack of the (symmetric) L^g,
  // as one split-K GEMM
  const int64_t K = (int64_t)NG * M;
  const int tiles = ((M + 63) / 64) * ((M + 63) / 64);
  const int sk = (int)std::max<int64_t>(1, std::min<int64_t>(std::max(1, 256 / tiles), K / 256));
  double* dtmp = nullptr;
  hip_check(hipMalloc(&dtmp, sizeof(double) * M * M * (size_t)(1 + sk)), "hipMalloc");
  {
    msd::GemmArgs g;
    g.M = M;
    g.N = M;
    g.K = (int)K;
    g.A = sys->L;
    g.lda = M;
    g.a_kmaj = false;
    g.B = sys->L;
    g.ldb = M;
    g.b_kmaj = false;
    g.C = dtmp;
    g.ldc = M;
    g.splitk = sk;
    g.ws = dtmp + (size_t)M * M;
    msd::launch_gemm(g, sys->st);
  }
  hipError_t e1 = hipMemcpyAsync(tmp.data(), dtmp, sizeof(double) * M * M, hipMemcpyDeviceToHost,
                                 sys->st);
  hipError_t e2 = hipStreamSynchronize(sys->st);
  (void)hipFree(dtmp);
  hip_check(e1, "sum LL");
  hip_check(e2, "sum LL");
  sys->sumll_host = tmp;
  if (sys->mixed) msd::launch_f64_to_f32(sys->L, sys->L32, (int64_t)NG * M * M, sys->st);
  sys->B1_dt = NAN;
  sys->have_ham = true;
  sys->derived_ok = false;
  sys->drop_graphs();
  if (sys->have_trial) build_derived(sys);
  API_END(sys)
}

namespace {

// Force-bias split-K from the override or the automatic choice; grows the
// workspace (in the trial arena) when a larger split is asked for.
void apply_fb_splitk(msd_system* s) {
  const int64_t K = (int64_t)s->P_all * s->M;
  int sk = s->tune.fb_splitk > 0 ? s->tune.fb_splitk : s->fb_splitk_auto;
  sk = (int)std::max<int64_t>(1, std::min<int64_t>(sk, std::max<int64_t>(1, K / 16)));
  if (sk > 1 && sk > s->fb_ws_cap) {
    s->fb_ws = s->trial_mem.get<double>((size_t)sk * s->NG * 2 * s->NW);
    s->fb_ws32 = s->mixed ? s->trial_mem.get<float>((size_t)sk * s->NG * 2 * s->NW) : nullptr;
    s->fb_ws_cap = sk;
  }
  s->fb_splitk = sk;
}

// Shared by both trial entry points: occupation rows -> device tables.
void set_trial_rows(msd_system* sys, const double* ci, const int32_t* occ_a,
                    const int32_t* occ_b) {
  for (int64_t i = 0; i < 2 * sys->ND; ++i)
    if (!std::isfinite(ci[i])) fail(MSD_ERR_ARG, "CI coefficient " + std::to_string(i / 2) + " not finite");
  msd::TrialTables tt;
  std::vector<int32_t> dummy;
  std::string e = msd::build_trial(sys->M, sys->na, sys->nb, sys->ND, ci,
                                   occ_a ? occ_a : dummy.data(), occ_b ? occ_b : dummy.data(), &tt);
  if (!e.empty()) fail(MSD_ERR_TRIAL, e);
  // capacity checks of the LDS kernels
  for (int sp = 0; sp < 2; ++sp) {
    const msd::SpinTable& S = tt.s[sp];
    const size_t X = (size_t)S.nv() * S.no();
    if (X > 64 * 16)
      fail(MSD_ERR_UNSUPPORTED, "excitation window too large (n_vir_act * n_occ_act > 1024)");
    const size_t green_lds = (X + (size_t)S.nv() * S.N + (size_t)S.nv() * 64) * sizeof(cd);
    if (green_lds > 140 * 1024) fail(MSD_ERR_UNSUPPORTED, "excitation window too large for LDS");
  }
  {
    const msd::SpinTable& A = tt.s[0];
    const msd::SpinTable& B = tt.s[1];
    const size_t words = (size_t)A.nv() * A.N + (size_t)B.nv() * B.N +
                         std::max((size_t)A.N * A.N, (size_t)B.N * B.N) +
                         std::max((size_t)A.nv() * A.N, (size_t)B.nv() * B.N) +
                         (size_t)A.nv() * A.no() + (size_t)B.nv() * B.no();
    if (words * sizeof(cd) > 140 * 1024)
      fail(MSD_ERR_UNSUPPORTED, "Cholesky contraction tile exceeds LDS");
  }
  free_energy(sys);
  sys->trial_mem.release();
  sys->tt = std::move(tt);
  Arena& T = sys->trial_mem;
  hipStream_t st = sys->st;
  const int M = sys->M, NW = sys->NW, NG = sys->NG;
  std::vector<int> rows_all;
  for (int sp = 0; sp < 2; ++sp) {
    const msd::SpinTable& S = sys->tt.s[sp];
    msd::DevSpin& D = sys->ds[sp];
    D = msd::DevSpin();
    D.N = S.N;
    D.U = S.U;
    D.nv = S.nv();
    D.no = S.no();
    D.P = S.N + S.nv();
    D.col0 = sp ? sys->na : 0;
    D.A = S.adj_off[S.U];
    D.M2 = S.m2_off[S.U];
    D.n_minor = S.n_minor;
    std::vector<int> rows(S.ref);
    rows.insert(rows.end(), S.vir_act.begin(), S.vir_act.end());
    rows_all.insert(rows_all.end(), rows.begin(), rows.end());
    D.ref = T.upload(S.ref, st);
    D.vir = T.upload(S.vir_act, st);
    {
      // orbitals outside the reference, and each window virtual's place among them
      std::vector<char> in_ref(M, 0);
      for (int r : S.ref) in_ref[r] = 1;
      std::vector<int> nref, pos(M, -1), vpos;
      for (int p = 0; p < M; ++p)
        if (!in_ref[p]) {
          pos[p] = (int)nref.size();
          nref.push_back(p);
        }
      for (int v : S.vir_act) vpos.push_back(pos[v]);
      D.nref = T.upload(nref, st);
      D.vpos = T.upload(vpos, st);
    }
    D.oslot = T.upload(S.occ_slot, st);
    D.rows = T.upload(rows, st);
    D.k = T.upload(S.k, st);
    D.hslot = T.upload(S.hslot, st);
    D.hwin = T.upload(S.hwin, st);
    D.part = T.upload(S.part, st);
    D.pwin = T.upload(S.pwin, st);
    D.adj_off = T.upload(S.adj_off, st);
    D.m2_off = T.upload(S.m2_off, st);
    D.bw_ptr = T.upload(S.bw_ptr, st);
    D.bw_det = T.upload(S.bw_det, st);
    D.n_seg = (int)S.seg_ptr.size() - 1;
    D.seg_ptr = T.upload(S.seg_ptr, st);
    D.str_seg = T.upload(S.str_seg, st);
    D.c_ptr = T.upload(S.c_ptr, st);
    D.c_adj = T.upload(S.c_adj, st);
    D.c_str = T.upload(S.c_str, st);
    D.mn_idx = T.upload(S.mn_idx, st);
    D.mn_ptr = T.upload(S.mn_ptr, st);
    D.mn_str = T.upload(S.mn_str, st);
    D.mn_m2 = T.upload(S.mn_m2, st);
    D.mn_sgn = T.upload(S.mn_sgn, st);
    D.det_s = T.upload(sys->tt.det_s[sp], st);
    for (int k = 0; k < msd::KMAX + 2; ++k) D.bucket[k] = S.bucket[k];
    msd::SpinWork& W = sys->sw[sp];
    W.d = T.get<cd>((size_t)NW * S.U);
    W.adj = T.get<cd>((size_t)NW * std::max(D.A, 1));
    W.m2 = T.get<cd>((size_t)NW * std::max(D.M2, 1));
    W.B = T.get<cd>((size_t)NW * S.U);
    sys->segp[sp] = T.get<cd>((size_t)NW * std::max(D.n_seg, 1));
    W.C = T.get<cd>((size_t)NW * std::max(D.nv * D.no, 1));
    W.G = T.get<cd>((size_t)NW * D.P * M);
    sys->L_lt[sp] = T.get<double>((size_t)NG * D.P * M);
  }
  std::sort(rows_all.begin(), rows_all.end());
  rows_all.erase(std::unique(rows_all.begin(), rows_all.end()), rows_all.end());
  sys->P_all = (int)rows_all.size();
  for (int sp = 0; sp < 2; ++sp) {
    const msd::SpinTable& S = sys->tt.s[sp];
    std::vector<int> rm(sys->P_all, -1);
    for (int r = 0; r < sys->P_all; ++r) {
      const int orb = rows_all[r];
      for (int j = 0; j < S.N; ++j)
        if (S.ref[j] == orb) rm[r] = j;
      for (int a = 0; a < S.nv(); ++a)
        if (S.vir_act[a] == orb) rm[r] = S.N + a;
    }
    sys->rmap[sp] = T.upload(rm, st);
  }
  sys->rows_all_dev = T.upload(rows_all, st);
  {
    // enough (M-tile, N-tile, K-slice) workgroups to fill the chip, slices >= 256 deep
    const int64_t K = (int64_t)sys->P_all * M;
    const int64_t tiles = (int64_t)((NG + 63) / 64) * ((2 * NW + 63) / 64);
    int sk = (int)std::max<int64_t>(1, std::min<int64_t>(512 / std::max<int64_t>(tiles, 1), K / 256));
    sys->fb_splitk_auto = std::min(sk, 16);
    sys->fb_ws_cap = 0;
    apply_fb_splitk(sys);
  }
  sys->L_rows = T.get<double>((size_t)NG * sys->P_all * M);
  sys->Gp = T.get<double>((size_t)2 * NW * sys->P_all * M);
  sys->lf_fits64 = msd::ltl_mfma_fits(sys->ds[0], sys->ds[1], M, false);
  sys->lf_fits32 = sys->mixed && msd::ltl_mfma_fits(sys->ds[0], sys->ds[1], M, true);
  sys->lf_P16 = msd::ltl_rows16(sys->ds[0], sys->ds[1]);
  for (int sp = 0; sp < 2; ++sp) {
    const size_t n = (size_t)NG * msd::ltl_stage_elems(sys->ds[0], sys->ds[1]);
    sys->Slf[sp] = sys->lf_fits64 ? T.get<double>(n) : nullptr;
    sys->Slf32[sp] = sys->lf_fits32 ? T.get<float>(n) : nullptr;
    sys->Slr[sp] = (sys->lf_fits64 || sys->lf_fits32) ? T.get<double>((size_t)NG * 64 * 8) : nullptr;
  }
  sys->gl_fits = msd::ltl_general_fits(sys->ds[0], sys->ds[1], M, false);
  sys->gl_fast64 = msd::ltl_general_fast64(sys->ds[0], sys->ds[1], M);
  sys->gl_fits32 = sys->mixed && msd::ltl_general_fits(sys->ds[0], sys->ds[1], M, true);
  for (int sp = 0; sp < 2; ++sp) {
    const size_t n = (sys->gl_fits || sys->gl_fits32)
                         ? msd::ltl_general_s_elems(sys->ds[0], sys->ds[1], M, NG) : 0;
    sys->Sgl[sp] = sys->gl_fits ? T.get<double>(n) : nullptr;
    sys->Sgl32[sp] = sys->gl_fits32 ? T.get<float>(n) : nullptr;
  }
  if (sys->mixed) {
    sys->Gp32 = T.get<float>((size_t)2 * NW * sys->P_all * M);
    sys->Lrows32 = T.get<float>((size_t)NG * sys->P_all * M);
    for (int sp = 0; sp < 2; ++sp) {
      sys->Llt32[sp] = T.get<float>((size_t)NG * sys->ds[sp].P * M);
      sys->LR64[sp] = T.get<double>((size_t)NG * sys->ds[sp].N * M);
    }
  }
  sys->dp.n_pair = sys->tt.n_pair;
  sys->dp.x = T.upload(sys->tt.pr_x, st);
  sys->dp.y = T.upload(sys->tt.pr_y, st);
  sys->dp.ptr = T.upload(sys->tt.pr_ptr, st);
  sys->dp.det = T.upload(sys->tt.pr_det, st);
  sys->dp.fa = T.upload(sys->tt.pr_fa, st);
  sys->dp.fb = T.upload(sys->tt.pr_fb, st);
  sys->det_c = reinterpret_cast<cd*>(T.upload(sys->tt.det_c, st));
  sys->n_ochunks = (int)((sys->ND + sys->ochunk - 1) / sys->ochunk);
  sys->opart = T.get<cd>((size_t)NW * sys->n_ochunks);
  sys->derived_ok = false;
  sys->drop_graphs();
  sys->sync();
  sys->have_trial = true;
  sys->t_fresh = false;
  sys->have_walkers = false;
  if (sys->have_ham) build_derived(sys);
}

// Occupation rows of an excitation list: the reference with the holes removed
// and the particles added, sorted ascending.  Validates that every hole is in
// the reference and every particle outside it, without repeats.
void rows_from_excitations(const int32_t* ref, int N, int M, int64_t n_det, const int32_t* k,
                           const int64_t* offsets, const int32_t* holes, const int32_t* parts,
                           const int32_t* k_other, bool beta,
                           std::vector<int32_t>& rows) {
  const char* nm = beta ? "beta" : "alpha";
  std::vector<char> in_ref(M, 0);
  for (int j = 0; j < N; ++j) {
    if (ref[j] < 0 || ref[j] >= M) fail(MSD_ERR_TRIAL, std::string(nm) + " reference orbital out of range");
    if (in_ref[ref[j]]) fail(MSD_ERR_TRIAL, std::string(nm) + " reference orbital repeated");
    in_ref[ref[j]] = 1;
  }
  rows.assign((size_t)n_det * N, 0);
  std::vector<char> occ(M);
  for (int64_t I = 0; I < n_det; ++I) {
    const std::string who = "determinant " + std::to_string(I) + " (" + nm + "): ";
    const int kk = k[I];
    if (kk < 0 || kk > std::min(N, msd::KMAX) || kk > M - N)
      fail(MSD_ERR_TRIAL, who + "excitation order out of range");
    if (offsets[I] < 0 || offsets[I + 1] < offsets[I] ||
        offsets[I + 1] - offsets[I] != (int64_t)k[I] + k_other[I])
      fail(MSD_ERR_TRIAL, who + "offsets do not match k_a + k_b");
    const int64_t o = offsets[I] + (beta ? k_other[I] : 0);
    std::copy(in_ref.begin(), in_ref.end(), occ.begin());
    for (int m = 0; m < kk; ++m) {
      const int h = holes[o + m], p = parts[o + m];
      if (h < 0 || h >= M || !in_ref[h] || !occ[h]) fail(MSD_ERR_TRIAL, who + "bad hole " + std::to_string(h));
      occ[h] = 0;
      if (p < 0 || p >= M || in_ref[p] || occ[p] == 2) fail(MSD_ERR_TRIAL, who + "bad particle " + std::to_string(p));
      occ[p] = 2;
    }
    int32_t* r = rows.data() + (size_t)I * N;
    int c = 0;
    for (int q = 0; q < M; ++q)
      if (occ[q]) r[c++] = q;
  }
}

}  // namespace

msd_status msd_set_trial_occ(msd_system* sys, const double* ci, const int32_t* occ_a,
                             const int32_t* occ_b) {
  API_BEGIN
  if (!sys || !ci || (!occ_a && sys->na) || (!occ_b && sys->nb)) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  set_trial_rows(sys, ci, occ_a, occ_b);
  API_END(sys)
}

msd_status msd_set_trial_exc(msd_system* sys, const int32_t* ref_a, const int32_t* ref_b,
                             int64_t n_det, const double* ci, const int32_t* k_a,
                             const int32_t* k_b, const int64_t* offsets, const int32_t* holes,
                             const int32_t* parts) {
  API_BEGIN
  if (!sys || !ci || !k_a || !k_b || !offsets || (!ref_a && sys->na) || (!ref_b && sys->nb))
    fail(MSD_ERR_ARG, "null argument");
  if (n_det != sys->ND) fail(MSD_ERR_SHAPE, "n_det differs from the handle's n_det");
  if (offsets[0] != 0) fail(MSD_ERR_TRIAL, "offsets[0] must be 0");
  if (offsets[n_det] > 0 && (!holes || !parts)) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  std::vector<int32_t> ra, rb;
  rows_from_excitations(ref_a, sys->na, sys->M, n_det, k_a, offsets, holes, parts, k_b, false, ra);
  rows_from_excitations(ref_b, sys->nb, sys->M, n_det, k_b, offsets, holes, parts, k_a, true, rb);
  set_trial_rows(sys, ci, ra.data(), rb.data());
  API_END(sys)
}

msd_status msd_get_weights(msd_system* sys, double* weights, double* log_ovlp) {
  return msd_get_walkers(sys, nullptr, nullptr, weights, log_ovlp);
}



static void copy_out(msd_system* s, void* host, const void* dev, size_t bytes) {
  if (!host) return;
  hip_check(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s->st), "download");
}

static void copy_dd(msd_system* s, void* dst, const void* src, size_t bytes) {
  if (!dst) return;
  hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s->st), "copy");
}

msd_status msd_set_walkers(msd_system* sys, const double* phi_a, const double* phi_b,
                           const double* weights) {
  API_BEGIN
  if (!sys || (!phi_a && sys->na) || (!phi_b && sys->nb)) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  const size_t na = (size_t)sys->NW * sys->M * sys->na, nb = (size_t)sys->NW * sys->M * sys->nb;
  for (size_t i = 0; i < 2 * na; ++i)
    if (!std::isfinite(phi_a[i])) fail(MSD_ERR_ARG, "phi_a not finite at " + std::to_string(i / 2));
  for (size_t i = 0; i < 2 * nb; ++i)
    if (!std::isfinite(phi_b[i])) fail(MSD_ERR_ARG, "phi_b not finite at " + std::to_string(i / 2));
  if (weights)
    for (int w = 0; w < sys->NW; ++w)
      if (!std::isfinite(weights[w]) || weights[w] < 0)
        fail(MSD_ERR_ARG, "weight " + std::to_string(w) + " not finite and non-negative");
  // stage through the propagation buffers (same capacity: NW*M*Ntot complex)
  cd* da = sys->term[0];
  cd* db = sys->term[1];
  if (na) hip_check(hipMemcpyAsync(da, phi_a, na * sizeof(cd), hipMemcpyHostToDevice, sys->st), "upload");
  if (nb) hip_check(hipMemcpyAsync(db, phi_b, nb * sizeof(cd), hipMemcpyHostToDevice, sys->st), "upload");
  double* dw = nullptr;
  if (weights) {
    dw = sys->fields;
    hip_check(hipMemcpyAsync(dw, weights, sizeof(double) * sys->NW, hipMemcpyHostToDevice, sys->st),
              "upload");
  }
  set_walkers_impl(sys, da, db, dw);
  API_END(sys)
}

msd_status msd_set_walkers_dev(msd_system* sys, const double* phi_a, const double* phi_b,
                               const double* weights) {
  API_BEGIN
  if (!sys || (!phi_a && sys->na) || (!phi_b && sys->nb)) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  const size_t na = (size_t)sys->NW * sys->M * sys->na, nb = (size_t)sys->NW * sys->M * sys->nb;
  // copy first: the caller's buffers may alias nothing of ours, but the
  // packing kernel reads them while writing the walker matrix
  cd* da = sys->term[0];
  cd* db = sys->term[1];
  copy_dd(sys, da, phi_a, na * sizeof(cd));
  copy_dd(sys, db, phi_b, nb * sizeof(cd));
  double* dw = nullptr;
  if (weights) {
    dw = sys->fields;
    copy_dd(sys, dw, weights, sizeof(double) * sys->NW);
  }
  set_walkers_impl(sys, da, db, dw);
  API_END(sys)
}

msd_status msd_get_walkers(msd_system* sys, double* phi_a, double* phi_b, double* weights,
                           double* log_ovlp) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  if (!sys->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
  set_device(sys);
  const size_t na = (size_t)sys->NW * sys->M * sys->na, nb = (size_t)sys->NW * sys->M * sys->nb;
  msd::launch_copy_walkers(sys->NW, sys->M, sys->Ntot, sys->na, sys->nb, nullptr, nullptr, sys->phi,
                           false, sys->term[0], sys->term[1], sys->st);
  copy_out(sys, phi_a, sys->term[0], na * sizeof(cd));
  copy_out(sys, phi_b, sys->term[1], nb * sizeof(cd));
  copy_out(sys, weights, sys->weights, sizeof(double) * sys->NW);
  copy_out(sys, log_ovlp, sys->logo, sizeof(cd) * sys->NW);
  sys->sync();
  API_END(sys)
}

msd_status msd_measure(msd_system* sys, double dt, double* log_ovlp, double* force_bias,
                       double* e_loc) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  measure_impl(sys, dt, e_loc != nullptr);
  check_flags(sys, "msd_measure");
  copy_out(sys, log_ovlp, sys->logo_tmp, sizeof(cd) * sys->NW);
  copy_out(sys, force_bias, sys->xbar, sizeof(cd) * sys->NW * sys->NG);
  copy_out(sys, e_loc, sys->eloc, sizeof(cd) * sys->NW);
  sys->sync();
  API_END(sys)
}

msd_status msd_measure_dev(msd_system* sys, double dt, double* log_ovlp, double* force_bias,
                           double* e_loc) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  measure_impl(sys, dt, e_loc != nullptr);
  copy_dd(sys, log_ovlp, sys->logo_tmp, sizeof(cd) * sys->NW);
  copy_dd(sys, force_bias, sys->xbar, sizeof(cd) * sys->NW * sys->NG);
  copy_dd(sys, e_loc, sys->eloc, sizeof(cd) * sys->NW);
  API_END(sys)
}

msd_status msd_propagate(msd_system* sys, const double* fields, double dt, double e_shift,
                         int32_t n_steps) {
  API_BEGIN
  if (!sys || (!fields && n_steps > 0)) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  const size_t per = (size_t)sys->NW * sys->NG;
  for (size_t i = 0; i < per * (size_t)std::max(n_steps, 0); ++i)
    if (!std::isfinite(fields[i])) fail(MSD_ERR_ARG, "field " + std::to_string(i) + " not finite");
  for (int step = 0; step < n_steps; ++step) {
    hip_check(hipMemcpyAsync(sys->fields, fields + step * per, per * sizeof(double),
                             hipMemcpyHostToDevice, sys->st),
              "upload fields");
    propagate_impl(sys, sys->fields, dt, e_shift, 1);
  }
  sys->sync();
  API_END(sys)
}

msd_status msd_propagate_dev(msd_system* sys, const double* fields, double dt, double e_shift,
                             int32_t n_steps) {
  API_BEGIN
  if (!sys || (!fields && n_steps > 0)) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  propagate_impl(sys, fields, dt, e_shift, n_steps);
  API_END(sys)
}

msd_status msd_population_control(msd_system* sys, double z, int32_t* parent) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  comb_impl(sys, z, nullptr);
  copy_out(sys, parent, sys->pc_parent, sizeof(int) * sys->NW);
  sys->sync();
  API_END(sys)
}

msd_status msd_population_control_dev(msd_system* sys, double z, int32_t* parent) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  comb_impl(sys, z, parent);
  API_END(sys)
}

msd_status msd_population_control_noalloc(msd_system* sys, double z, int32_t* parent) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  comb_noalloc_impl(sys, z, parent);
  API_END(sys)
}

msd_status msd_run_block(msd_system* sys, const double* fields, double dt, double e_shift,
                         int32_t n_steps, int32_t pop_freq, const double* z, double* energy) {
  API_BEGIN
  if (!sys || !fields || !energy) fail(MSD_ERR_ARG, "null argument");
  if (n_steps < 1) fail(MSD_ERR_ARG, "n_steps must be >= 1");
  if (pop_freq < 0) fail(MSD_ERR_ARG, "pop_freq must be >= 0");
  const int n_comb = pop_freq > 0 ? n_steps / pop_freq : 0;
  if (n_comb > 0 && !z) fail(MSD_ERR_ARG, "null comb offsets");
  for (int j = 0; j < n_comb; ++j)
    if (!(z[j] >= 0.0 && z[j] < 1.0))
      fail(MSD_ERR_ARG, "comb offset " + std::to_string(j) + " outside [0, 1)");
  set_device(sys);
  const size_t per = (size_t)sys->NW * sys->NG;
  for (int step = 0, j = 0; step < n_steps; ++step) {
    propagate_impl(sys, fields + step * per, dt, e_shift, 1);
    if (pop_freq > 0 && (step + 1) % pop_freq == 0) comb_impl(sys, z[j++], nullptr);
  }
  measure_impl(sys, dt, true);
  msd::launch_block_energy(sys->NW, sys->weights, sys->eloc, sys->blk, sys->st);
  cd h[2];
  copy_out(sys, h, sys->blk, sizeof(h));
  check_flags(sys, "msd_run_block");  // synchronises: one wait for both copies
  energy[0] = h[0].re;
  energy[1] = h[0].im;
  energy[2] = h[1].re;
  API_END(sys)
}

msd_status msd_get_green(msd_system* sys, int32_t walker, double* g_a, double* g_b) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  if (walker < 0 || walker >= sys->NW) fail(MSD_ERR_ARG, "walker index out of range");
  if (!sys->have_trial) fail(MSD_ERR_STATE, "no trial");
  set_device(sys);
  const int M = sys->M;
  double* outs[2] = {g_a, g_b};
  for (int sp = 0; sp < 2; ++sp) {
    if (!outs[sp]) continue;
    const msd::SpinTable& S = sys->tt.s[sp];
    const int P = S.N + S.nv();
    std::vector<cd> rows((size_t)P * M);
    hip_check(hipMemcpyAsync(rows.data(), sys->sw[sp].G + (size_t)walker * P * M,
                             rows.size() * sizeof(cd), hipMemcpyDeviceToHost, sys->st),
              "download");
    sys->sync();
    std::vector<int> orb(S.ref);
    orb.insert(orb.end(), S.vir_act.begin(), S.vir_act.end());
    cd* out = reinterpret_cast<cd*>(outs[sp]);
    std::fill(out, out + (size_t)M * M, cd{0.0, 0.0});
    for (int r = 0; r < P; ++r)
      for (int q = 0; q < M; ++q) out[(size_t)orb[r] * M + q] = rows[(size_t)r * M + q];
  }
  API_END(sys)
}

msd_status msd_get_timings(msd_system* sys, int32_t max_stages, const char** names, double* ms,
                           int64_t* counts, int32_t* n_stages) {
  API_BEGIN
  if (!sys || !n_stages) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  sys->harvest();
  int n = 0;
  for (int i = 0; i < ST_COUNT && n < max_stages; ++i, ++n) {
    if (names) names[n] = kStageNames[i];
    if (ms) ms[n] = sys->stage_ms[i];
    if (counts) counts[n] = sys->stage_n[i];
  }
  *n_stages = n;
  API_END(sys)
}

msd_status msd_reset_timings(msd_system* sys) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  sys->harvest();
  for (int i = 0; i < ST_COUNT; ++i) {
    sys->stage_ms[i] = 0.0;
    sys->stage_n[i] = 0;
  }
  API_END(sys)
}

msd_status msd_trial_analyze(int32_t M, int32_t n_alpha, int32_t n_beta, int64_t n_det,
                             const int32_t* occ_a, const int32_t* occ_b, int32_t* k_a, int32_t* k_b,
                             int32_t* sign) {
  msd_system* none = nullptr;
  API_BEGIN
  if (!k_a || !k_b || !sign || (!occ_a && n_alpha) || (!occ_b && n_beta))
    fail(MSD_ERR_ARG, "null argument");
  if (M <= 0 || n_alpha < 0 || n_beta < 0 || n_alpha > M || n_beta > M)
    fail(MSD_ERR_SHAPE, "invalid sizes");
  std::vector<int32_t> dummy(1);
  std::string e = msd::analyze_trial(M, n_alpha, n_beta, n_det, occ_a ? occ_a : dummy.data(),
                                     occ_b ? occ_b : dummy.data(), k_a, k_b, sign);
  if (!e.empty()) fail(MSD_ERR_TRIAL, e);
  API_END(none)
}

}  // extern "C"

// ============================================================================
// Batches of independent systems: one graph per step for all of them
// ============================================================================

struct msd_batch {
  int dev = 0;
  hipStream_t st = nullptr;
  hipStream_t cap_st = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<msd_system*> sys;
  // one capture branch per system: the graph holds the systems' launch
  // chains as independent branches (forked from and joined to cap_st), so
  // the runtime may run the systems concurrently
  std::vector<hipStream_t> br_st;
  std::vector<hipEvent_t> fork_ev, join_ev;
  struct Entry {
    std::vector<uint64_t> versions;
    hipGraphExec_t exec = nullptr;
  };
  std::map<std::string, Entry> graphs;  // key: QR flags, measure flag, dt, e_shift
  void drop() {
    for (auto& kv : graphs)
      if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    graphs.clear();
  }
};

msd_status msd_batch_create(msd_system* const* systems, int32_t n, void* hip_stream,
                            msd_batch** out) {
  msd_batch* b = nullptr;
  API_BEGIN
  if (!systems || !out || n <= 0) fail(MSD_ERR_ARG, "null argument or empty batch");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!systems[i]) fail(MSD_ERR_ARG, "system " + std::to_string(i) + " is null");
    if (systems[i]->dev != systems[0]->dev)
      fail(MSD_ERR_ARG, "system " + std::to_string(i) + " is on another device");
    for (int j = 0; j < i; ++j)
      if (systems[j] == systems[i]) fail(MSD_ERR_ARG, "system " + std::to_string(i) + " repeated");
  }
  b = new msd_batch();
  b->dev = systems[0]->dev;
  b->st = static_cast<hipStream_t>(hip_stream);
  b->sys.assign(systems, systems + n);
  try {
    hip_check(hipSetDevice(b->dev), "hipSetDevice");
    hip_check(hipStreamCreateWithFlags(&b->cap_st, hipStreamNonBlocking), "stream");
    hip_check(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming), "event");
    b->br_st.assign(n, nullptr);
    b->fork_ev.assign(n, nullptr);
    b->join_ev.assign(n, nullptr);
    for (int i = 0; i < n; ++i) {
      hip_check(hipStreamCreateWithFlags(&b->br_st[i], hipStreamNonBlocking), "stream");
      hip_check(hipEventCreateWithFlags(&b->fork_ev[i], hipEventDisableTiming), "event");
      hip_check(hipEventCreateWithFlags(&b->join_ev[i], hipEventDisableTiming), "event");
    }
  } catch (...) {
    if (b->cap_st) (void)hipStreamDestroy(b->cap_st);
    for (hipStream_t x : b->br_st)
      if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t x : b->fork_ev)
      if (x) (void)hipEventDestroy(x);
    for (hipEvent_t x : b->join_ev)
      if (x) (void)hipEventDestroy(x);
    if (b->ev) (void)hipEventDestroy(b->ev);
    delete b;
    b = nullptr;
    throw;
  }
  *out = b;
  API_END(static_cast<msd_system*>(nullptr))
}

void msd_batch_destroy(msd_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->dev);
  (void)hipStreamSynchronize(b->st);
  b->drop();
  if (b->cap_st) (void)hipStreamDestroy(b->cap_st);
  for (hipStream_t x : b->br_st)
    if (x) (void)hipStreamDestroy(x);
  for (hipEvent_t x : b->fork_ev)
    if (x) (void)hipEventDestroy(x);
  for (hipEvent_t x : b->join_ev)
    if (x) (void)hipEventDestroy(x);
  if (b->ev) (void)hipEventDestroy(b->ev);
  delete b;
}

msd_status msd_batch_step(msd_batch* b, const double* const* fields, double dt, double e_shift,
                          int32_t do_measure) {
  API_BEGIN
  if (!b || !fields) fail(MSD_ERR_ARG, "null argument");
  hip_check(hipSetDevice(b->dev), "hipSetDevice");
  if (!(dt > 0.0) || !std::isfinite(dt)) fail(MSD_ERR_ARG, "dt must be finite and > 0");
  if (!std::isfinite(e_shift)) fail(MSD_ERR_ARG, "e_shift must be finite");
  const int n = (int)b->sys.size();
  bool timing = false;
  for (int i = 0; i < n; ++i) {
    msd_system* s = b->sys[i];
    const std::string who = "system " + std::to_string(i) + ": ";
    if (!fields[i]) fail(MSD_ERR_ARG, who + "null fields");
    try {
      need_ready(s);
      if (!s->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
      if (do_measure && s->tt.max_k() > msd::KMAX) fail(MSD_ERR_UNSUPPORTED, "excitation order too high");
      ensure_b1(s, dt);
      if (do_measure) alloc_energy(s);
    } catch (const Error& e) {
      throw Error{e.code, who + e.msg};
    }
    timing = timing || s->o.timing;
  }
  // order against work already queued on the systems' own streams
  for (msd_system* s : b->sys) {
    hip_check(hipEventRecord(b->ev, s->st), "record");
    hip_check(hipStreamWaitEvent(b->st, b->ev, 0), "wait");
  }
  std::string key = do_measure ? "m" : "p";
  std::vector<char> qr(n);
  for (int i = 0; i < n; ++i) {
    msd_system* s = b->sys[i];
    s->steps_done++;
    qr[i] = s->o.stabilize_freq > 0 && s->steps_done % s->o.stabilize_freq == 0;
    key += qr[i] ? '1' : '0';
    key += s->t_fresh ? 'f' : 'n';
    hip_check(hipMemcpyAsync(s->fields, fields[i], sizeof(double) * s->NW * s->NG,
                             hipMemcpyDeviceToDevice, b->st),
              "fields");
  }
  char buf[64];
  std::snprintf(buf, sizeof buf, "|%.17g|%.17g", dt, e_shift);
  key += buf;
  // branches: capture each system's launches on its own stream, forked from
  // and joined to st (graph capture); otherwise one after another on st
  auto body = [&](hipStream_t st, bool branches) {
    for (int i = 0; i < n; ++i) {
      msd_system* s = b->sys[i];
      hipStream_t own = s->st;
      hipStream_t run = st;
      if (branches) {
        hip_check(hipEventRecord(b->fork_ev[i], st), "fork");
        hip_check(hipStreamWaitEvent(b->br_st[i], b->fork_ev[i], 0), "fork");
        run = b->br_st[i];
      }
      s->st = run;
      try {
        propagate_step(s, s->fields, dt, e_shift, qr[i]);
        if (do_measure) measure_body(s, dt, true);
      } catch (...) {
        s->st = own;
        throw;
      }
      s->st = own;
      if (branches) {
        hip_check(hipEventRecord(b->join_ev[i], run), "join");
        hip_check(hipStreamWaitEvent(st, b->join_ev[i], 0), "join");
      }
    }
  };
  if (timing) {
    body(b->st, false);  // timing events cannot live in a graph: run the launches directly
  } else {
    std::vector<uint64_t> versions(n);
    for (int i = 0; i < n; ++i) versions[i] = b->sys[i]->version;
    msd_batch::Entry& e = b->graphs[key];
    if (e.exec && e.versions != versions) {
      hip_check(hipGraphExecDestroy(e.exec), "hipGraphExecDestroy");
      e.exec = nullptr;
    }
    if (!e.exec) {
      hipGraph_t g = nullptr;
      hip_check(hipStreamBeginCapture(b->cap_st, hipStreamCaptureModeThreadLocal), "begin capture");
      try {
        body(b->cap_st, true);
      } catch (...) {
        (void)hipStreamEndCapture(b->cap_st, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      hip_check(hipStreamEndCapture(b->cap_st, &g), "end capture");
      hipError_t err = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      hip_check(err, "hipGraphInstantiate");
      e.versions = versions;
    }
    hip_check(hipGraphLaunch(e.exec, b->st), "hipGraphLaunch");
  }
  for (msd_system* s : b->sys) s->t_fresh = true;  // each step ends with an overlap pass
  // later work on each system's stream sees this step
  hip_check(hipEventRecord(b->ev, b->st), "record");
  for (msd_system* s : b->sys) hip_check(hipStreamWaitEvent(s->st, b->ev, 0), "wait");
  hip_check(hipGetLastError(), "batch step");
  API_END(static_cast<msd_system*>(nullptr))
}

msd_status msd_get_measurement(msd_system* sys, double* log_ovlp, double* force_bias,
                               double* e_loc) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  if (!sys->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
  set_device(sys);
  copy_out(sys, log_ovlp, sys->logo_tmp, sizeof(cd) * sys->NW);
  copy_out(sys, force_bias, sys->xbar, sizeof(cd) * sys->NW * sys->NG);
  copy_out(sys, e_loc, sys->eloc, sizeof(cd) * sys->NW);
  sys->sync();
  API_END(sys)
}

// ============================================================================
// Launch-shape tuning and the autotuner
// ============================================================================

namespace {

void set_tuning_impl(msd_system* s, const msd_tuning& t) {
  auto bad = [](const char* f) { fail(MSD_ERR_ARG, std::string("tuning field ") + f + " out of range"); };
  if (t.fb_splitk < 0 || t.fb_splitk > 16) bad("fb_splitk");
  if (t.lambda_variant < 0 || t.lambda_variant > 6 ||
      (t.lambda_variant >= 2 && t.lambda_variant <= 4))
    bad("lambda_variant");
  if (t.lambda_chunk < 0) bad("lambda_chunk");
  if (t.second_gsplit < 0 || t.second_gsplit > 64) bad("second_gsplit");
  if (t.second_stage < 0 || t.second_stage > 32) bad("second_stage");
  if (t.second_gather < 0 || t.second_gather > 2) bad("second_gather");
  if (t.second_copy < 0 || t.second_copy > 2) bad("second_copy");
  if (t.second_waves != 0 && t.second_waves != 8 && t.second_waves != 16) bad("second_waves");
  if (t.walker_tile < 0) bad("walker_tile");
  if (t.second_whole < 0 || t.second_whole > 2) bad("second_whole");
  s->tune = t;
  s->tune.energy_form = 0;  // read-only
  free_energy(s);
  s->drop_graphs();
  if (s->have_trial) apply_fb_splitk(s);
}

double time_measures(msd_system* s, double dt, int reps) {
  measure_impl(s, dt, true);  // builds the plan; warms caches
  hipEvent_t a = s->ev(), b = s->ev();
  hip_check(hipEventRecord(a, s->st), "record");
  for (int r = 0; r < reps; ++r) measure_impl(s, dt, true);
  hip_check(hipEventRecord(b, s->st), "record");
  hip_check(hipEventSynchronize(b), "synchronize");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, a, b), "elapsed");
  s->pool.push_back(a);
  s->pool.push_back(b);
  return ms;
}

}  // namespace

msd_status msd_get_tuning(msd_system* sys, msd_tuning* out) {
  API_BEGIN
  if (!sys || !out) fail(MSD_ERR_ARG, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->fb_splitk = sys->fb_splitk;
  if (sys->WT > 0) {
    out->lambda_variant = sys->lambda_variant;
    out->lambda_chunk = sys->gl_chunk;
    out->second_gsplit = sys->gsplit;
    out->second_stage = sys->second_G;
    out->second_gather = sys->second_flat ? 2 : 1;
    out->second_copy = sys->second_dma ? 2 : 1;
    out->second_waves = sys->second_waves;
    out->walker_tile = sys->WT;
    out->energy_form = sys->wform ? 1 : 0;
    out->second_whole = sys->second_whole_used ? 2 : 1;
  }
  API_END(sys)
}

msd_status msd_set_tuning(msd_system* sys, const msd_tuning* t) {
  API_BEGIN
  if (!sys || !t) fail(MSD_ERR_ARG, "null argument");
  set_device(sys);
  set_tuning_impl(sys, *t);
  API_END(sys)
}

msd_status msd_autotune(msd_system* sys, double dt, int32_t reps, msd_tuning* out) {
  API_BEGIN
  if (!sys) fail(MSD_ERR_ARG, "null argument");
  if (reps < 1 || reps > 100) fail(MSD_ERR_ARG, "reps must be in 1..100");
  set_device(sys);
  need_ready(sys);
  if (!sys->have_walkers) fail(MSD_ERR_STATE, "walkers have not been set");
  const int32_t graphs = sys->o.graphs, timing = sys->o.timing;
  sys->o.graphs = 0;
  sys->o.timing = 0;
  msd_tuning best = sys->tune;
  try {
    // a candidate replaces the incumbent (the current value, automatic if
    // unset) only when it is faster by more than 3%, so timing noise does not
    // move the choice
    auto sweep = [&](int32_t msd_tuning::*field, const std::vector<int>& cands) {
      set_tuning_impl(sys, best);
      double t_best = time_measures(sys, dt, reps);
      int v_best = best.*field;
      for (int v : cands) {
        if (v == best.*field) continue;
        msd_tuning t = best;
        t.*field = v;
        set_tuning_impl(sys, t);
        const double ms = time_measures(sys, dt, reps);
        if (ms < 0.97 * t_best) {
          t_best = ms;
          v_best = v;
        }
      }
      best.*field = v_best;
      set_tuning_impl(sys, best);
    };
    sweep(&msd_tuning::fb_splitk, {1, 2, 4, 8, 16});
    {
      std::vector<int> c;
      for (int wt : {16, 32, 64, 128, 256, 512})
        if (wt < sys->NW) c.push_back(wt);
      c.push_back(sys->NW);
      sweep(&msd_tuning::walker_tile, c);
    }
    int nmax = 0;
    if (msd::lambda_rows_fits(sys->ds[0], sys->ds[1], &nmax) && nmax <= 16)
      sweep(&msd_tuning::lambda_variant, {1, 5, 6});
    sweep(&msd_tuning::lambda_chunk, {4, 8, 16, 32});
    sweep(&msd_tuning::second_gather, {1, 2});
    sweep(&msd_tuning::second_copy, {1, 2});
    sweep(&msd_tuning::second_waves, {8, 16});
    sweep(&msd_tuning::second_gsplit, {1, 2, 4, 8});
    {
      const int X = sys->ds[0].nv * sys->ds[0].no + sys->ds[1].nv * sys->ds[1].no;
      const int elem = sys->mixed ? 8 : 16;
      std::vector<int> c;
      for (int g : {1, 2, 3, 4, 6, 8})
        if ((size_t)2 * g * elem * std::max(X, 1) <= ((size_t)150 << 10)) c.push_back(g);
      sweep(&msd_tuning::second_stage, c);
    }
  } catch (...) {
    sys->o.graphs = graphs;
    sys->o.timing = timing;
    throw;
  }
  sys->o.graphs = graphs;
  sys->o.timing = timing;
  measure_impl(sys, dt, true);  // leaves the chosen plan built
  sys->sync();
  if (out) {
    std::memset(out, 0, sizeof(*out));
    out->fb_splitk = sys->fb_splitk;
    out->lambda_variant = sys->lambda_variant;
    out->lambda_chunk = sys->gl_chunk;
    out->second_gsplit = sys->gsplit;
    out->second_stage = sys->second_G;
    out->second_gather = sys->second_flat ? 2 : 1;
    out->second_copy = sys->second_dma ? 2 : 1;
    out->second_waves = sys->second_waves;
    out->walker_tile = sys->WT;
    out->energy_form = sys->wform ? 1 : 0;
    out->second_whole = sys->second_whole_used ? 2 : 1;
  }
  API_END(sys)
}

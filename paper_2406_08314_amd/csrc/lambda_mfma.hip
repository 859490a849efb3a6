// A2 + A6 on the matrix cores for shapes with N = 8 electrons per spin and the
// whole occupied set in the excitation window (slot i = orbital i of the
// reference): the fused Cholesky contraction + energy intermediates kernel
// (k_ltl_mfma, below) and the FP64 mean-field trace pass (k_qtr).

#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace msd {

namespace {

typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

template <class R>
struct Mfma;
template <>
struct Mfma<double> {
  typedef dvec4 acc_t;
  typedef cd cx_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // register r of lane l holds D[l/16 + 4r][l % 16]
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef fvec4 acc_t;
  typedef cf cx_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // register r of lane l holds D[4 (l/16) + r][l % 16]
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <class R>
__device__ __forceinline__ R wsum(R v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void dma16(const void* g, void* lds) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
#endif
}

constexpr int LM_N = 8;         // electrons per spin of these kernels

}  // namespace

// ============================================================================
// A2 + A6 fused on the matrix cores: the Cholesky contraction LT^g = L^g T and
// the energy intermediates of Sec. III in one pass, without LT in HBM.
//
// Workgroup = 4 walkers of one spin (one wave each) and a chunk of Cholesky
// vectors; two or more workgroups share a CU and run out of step.  Per vector
// g the spin's restricted rows of L^g, stored k-major as S[g][k][p] (p over
// V_act then R, zero padded to P16 rows and 64 k), are staged in LDS by
// direct global-to-LDS loads, double-buffered one vector ahead.  Each wave forms transposed products, so that the result registers
// of one MFMA are the B operand of the next (no transposes through LDS):
//   LT^T   = [Tr Ti]^T S                     (16 x P16; [Tr Ti] in registers)
//   Lam^T  = Bq^T [Tr Ti]_V^T - LT_V^T        (16 x n_v, 16 virtuals per tile)
//   ZW^T  += (Bq - v Bi)^T Lam^T              (v = v0_alpha + v0_beta)
// Bq = [[Qr Qi]; [-Qi Qr]] is the real form of Q = LT[R, :] (row vectors
// times Q), Bi that of the identity; the 16 rows are the real and imaginary
// parts of the N = 8 columns.  The last line is ZW += Xi - v Lam with
// Xi = Lam Q; v comes from the trace pass (launch_qtr) before this kernel.
// ZW itself is not stored: each wave contracts its chunk's ZW with the
// walker's first-order CI matrix C and writes the scalar.
// ============================================================================

namespace {

constexpr int LF_WB = 4;               // walkers per workgroup
constexpr int LF_WAVES = LF_WB;        // one wave per walker (one spin per workgroup)
constexpr int LF_K = 64;               // contraction length (orbitals, zero padded)
constexpr int LF_Q = LM_N * 16;        // Q scratch per wave (reals)

// The waits are s_waitcnt instructions the compiler sees (so its own wait
// placement stays exact); the signal fences keep memory accesses from moving
// across them.  Encoding of s_waitcnt: vmcnt bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8.
constexpr int LF_WAIT_ALL = 0;       // vmcnt(0) expcnt(0) lgkmcnt(0)
constexpr int LF_WAIT_LGKM = 0xC07F; // lgkmcnt(0) only
// every outstanding memory operation of the wave done (including direct LDS
// loads), then the workgroup barrier
__device__ __forceinline__ void lf_bar_all() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(LF_WAIT_ALL);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// LDS writes of this wave visible to its own later reads
__device__ __forceinline__ void lf_wave_lds() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(LF_WAIT_LGKM);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

size_t lf_lds_bytes(int P16, size_t rsize) {
  return (2 * (size_t)LF_K * P16 + (size_t)LF_WAVES * LF_Q) * rsize;
}

// Row order of the 16 x 16 operands: hardware row i holds logical row sig(i)
// (0..7 real parts, 8..15 imaginary parts of columns 0..7).  In FP64 the
// identity: register r of lane group q holds rows q and q + 8 for r = 0, 2
// (column q) and r = 1, 3 (column q + 4).  In FP32, where register r of lane
// group q holds hardware row 4q + r, rows 4q .. 4q+3 are re/im of column 2q,
// then of column 2q + 1.
template <class R>
__device__ __forceinline__ int lf_sig(int i) {
  if constexpr (sizeof(R) == 8) return i;
  else return ((i & 1) << 3) | (i >> 1);
}
// complex column held by a lane in registers (re, im) = (r0, r1) and (r2, r3)
// of the pair h = 0, 1
template <class R>
__device__ __forceinline__ void lf_pair(int q, int h, int* rre, int* rim, int* n) {
  if constexpr (sizeof(R) == 8) {
    *rre = h;
    *rim = h + 2;
    *n = q + 4 * h;
  } else {
    *rre = 2 * h;
    *rim = 2 * h + 1;
    *n = 2 * q + h;
  }
}


}  // namespace

template <class R, int NT>
__global__ __launch_bounds__(64 * LF_WAVES, 2) void k_ltl_mfma(
    DevSpin sa, DevSpin sb, int NW, int w0, int WT, int NG, int g_chunk, int n_chunks, int M,
    int P16, const R* __restrict__ Sa, const R* __restrict__ Sb,
    const typename Mfma<R>::cx_t* __restrict__ Ta, const typename Mfma<R>::cx_t* __restrict__ Tb,
    typename Mfma<R>::cx_t* __restrict__ Lam_a, typename Mfma<R>::cx_t* __restrict__ Lam_b,
    const cd* __restrict__ v0, const cd* __restrict__ Ca, const cd* __restrict__ Cb,
    cd* __restrict__ czw, bool swz) {
  typedef Mfma<R> MF;
  typedef typename MF::cx_t C;
  typedef typename MF::acc_t acc_t;
  extern __shared__ __align__(16) unsigned char lf_raw[];
  R* lds = reinterpret_cast<R*>(lf_raw);
  const int SE = LF_K * P16;  // reals of one spin's stage
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int qb = 2 * SE + wv * LF_Q;           // this wave's Q as [i][re 0..7 | im 0..7]
  // workgroups of one chunk of vectors are consecutive on an XCD (shared L^g)
  const int nb = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, per = nb >> 3, rem = nb & 7;
  const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + (b >> 3);
  const int n_wgrp = (WT + LF_WB - 1) / LF_WB;
  const int chunk = logical / (2 * n_wgrp), s2 = (logical / n_wgrp) & 1;
  const int wl = (logical % n_wgrp) * LF_WB + wv;
  const bool active = wl < WT;
  const int w = w0 + (active ? wl : 0);
  const int nv = s2 ? sb.nv : sa.nv, X = nv * LM_N;
  const int* __restrict__ vir = s2 ? sb.vir : sa.vir;
  const C* __restrict__ T = s2 ? Tb : Ta;
  C* __restrict__ Lam = s2 ? Lam_b : Lam_a;
  const int col = lane & 15, q = lane >> 4;
  const int jc = lf_sig<R>(col);  // logical row of this lane's A-operand row

  // A of LT^T: [Tr Ti]^T, row jc, k = orbital 4s + q
  R bt[LF_K / 4];
#pragma unroll
  for (int s = 0; s < LF_K / 4; ++s) {
    const int k = 4 * s + q;
    R v = R(0);
    if (k < M) {
      const C t = T[((size_t)k * NW + w) * LM_N + (jc & 7)];
      v = jc < 8 ? t.re : t.im;
    }
    bt[s] = v;
  }
  // B of Lam^T: [Tr Ti]_V^T, k = 4s + q, column = virtual 16 rt + col
  R av[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int a = rt * 16 + col, k = 4 * s + q;
      R v = R(0);
      if (a < nv) {
        const C t = T[((size_t)vir[a] * NW + w) * LM_N + (k & 7)];
        v = k < 8 ? t.re : t.im;
      }
      av[rt][s] = v;
    }
  acc_t zw[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) zw[rt] = acc_t{0, 0, 0, 0};

  const int g0 = chunk * g_chunk, g1 = min(NG, g0 + g_chunk);
  auto fetch = [&](int g, int buf) {
    constexpr int per16 = 16 / sizeof(R);
    const int n16 = SE / per16;
    const R* src = (s2 ? Sb : Sa) + (size_t)g * SE;
    const int dst = buf * SE;
    for (int c = wv; c * 64 < n16; c += LF_WAVES) {
      const int e = c * 64 + lane;
      if (e < n16) dma16(src + (size_t)e * per16, &lds[dst + c * 64 * per16]);
    }
  };
  // v = v0_alpha + v0_beta of the walker and vector (read one vector ahead)
  const cd* va = v0 + (size_t)w * NG;
  const cd* vb = v0 + ((size_t)NW + w) * NG;
  cd vnext{0.0, 0.0};
  if (g0 < g1) {
    fetch(g0, 0);
    vnext = va[g0] + vb[g0];
  }
  // window store Lam[w][g][a * 8 + n]
  acc_t lam_prev[4];
  auto store_window = [&](int g) __attribute__((always_inline)) {
    if (!active) return;
    C* lo = Lam + ((size_t)wl * NG + g) * X;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int a = rt * 16 + col;
      if (a < nv) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          int rre, rim, n;
          lf_pair<R>(q, h, &rre, &rim, &n);
          lo[a * LM_N + (swz ? n ^ ((a >> 1) & 7) : n)] = C{lam_prev[rt][rre], lam_prev[rt][rim]};
        }
      }
    }
  };
  int it = 0;
  for (int g = g0; g < g1; ++g, ++it) {
    const int buf = it & 1;
    lf_bar_all();  // this vector's stage has landed; the other buffer is free
    if (g + 1 < g1) fetch(g + 1, buf ^ 1);
    if (g > g0) store_window(g - 1);
    const R vr = R(vnext.re), vi = R(vnext.im);
    if (g + 1 < g1) vnext = va[g + 1] + vb[g + 1];
    const int sb0 = buf * SE;
    acc_t acc[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) acc[ct] = acc_t{0, 0, 0, 0};
    // B operands of step s + 1 are read while the MFMAs of step s run
    R bcur[NT], bnxt[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) bcur[ct] = lds[sb0 + q * P16 + ct * 16 + col];
#pragma unroll
    for (int s = 0; s < LF_K / 4; ++s) {
      if (s + 1 < LF_K / 4) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
          bnxt[ct] = lds[sb0 + (4 * (s + 1) + q) * P16 + ct * 16 + col];
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = MF::run(bt[s], bcur[ct], acc[ct]);
      if (s + 1 < LF_K / 4) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) bcur[ct] = bnxt[ct];
      }
      // this step's MFMAs, then the next step's LDS reads (their wait comes
      // after the MFMAs queued on the matrix pipe)
      __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, (NT + 1) / 2, 0);
    }
    // Q = columns nv .. nv + 7 of LT^T
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ct * 16 + col - nv;
        if (i >= 0 && i < LM_N) lds[qb + i * 16 + lf_sig<R>(MF::row(lane, r))] = acc[ct][r];
      }
    lf_wave_lds();
    // A operands: Bq^T (row jc, k = 4s + q) and (Bq - v Bi)^T (row jc, k = the
    // logical row that register s of lane group q holds in Lam^T)
    R bqa[4], bqz[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      {
        const int k = 4 * s + q;
        const R qr = lds[qb + (k & 7) * 16 + (jc & 7)], qi = lds[qb + (k & 7) * 16 + 8 + (jc & 7)];
        bqa[s] = k < 8 ? (jc < 8 ? qr : qi) : (jc < 8 ? -qi : qr);
      }
      {
        const int k = lf_sig<R>(MF::row(lane, s));
        const R qr = lds[qb + (k & 7) * 16 + (jc & 7)], qi = lds[qb + (k & 7) * 16 + 8 + (jc & 7)];
        R z = k < 8 ? (jc < 8 ? qr : qi) : (jc < 8 ? -qi : qr);
        if ((k & 7) == (jc & 7)) z -= ((k < 8) == (jc < 8)) ? vr : (k < 8 ? vi : -vi);
        bqz[s] = z;
      }
    }
    // Lam^T tiles (C = -LT_V^T; columns at or beyond nv are zero)
    acc_t lam[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        lam[rt][r] = (rt < NT && rt * 16 + col < nv) ? -acc[rt < NT ? rt : 0][r] : R(0);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) lam[rt] = MF::run(bqa[s], av[rt][s], lam[rt]);
    // ZW^T += (Bq - v Bi)^T Lam^T: register s of Lam^T is the B operand of step s
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) zw[rt] = MF::run(bqz[s], lam[rt][s], zw[rt]);
    // the window of this vector is stored early in the next iteration, so its
    // stores drain while that iteration runs rather than at its first barrier
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) lam_prev[rt] = lam[rt];
  }
  if (g0 < g1) store_window(g1 - 1);
  if (!active) return;
  // this chunk's ZW contracted with the walker's first-order CI matrix C
  // (same window layout [a * 8 + n]) in FP64: one partial of sum C . ZW per
  // (spin, walker, chunk), [2][NW][n_chunks]
  const cd* __restrict__ Cw = (s2 ? Cb : Ca) + (size_t)w * X;
  double pr = 0.0, pi = 0.0;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    const int a = rt * 16 + col;
    if (a < nv) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        int rre, rim, n;
        lf_pair<R>(q, h, &rre, &rim, &n);
        const cd c = Cw[a * LM_N + n];
        const double zr = (double)zw[rt][rre], zi = (double)zw[rt][rim];
        pr += c.re * zr - c.im * zi;
        pi += c.re * zi + c.im * zr;
      }
    }
  }
  pr = wsum(pr);
  pi = wsum(pi);
  if (lane == 0) czw[((size_t)s2 * NW + w) * n_chunks + chunk] = cd{pr, pi};
}

// S[g][k][p] = L^g[row(p), k]: p < nv the active virtual orbitals, then the N
// reference orbitals, zero beyond P and for k >= M.
template <class R>
__global__ void k_gather_lf(const double* __restrict__ L, int NG, int M, const int* __restrict__ rows,
                            int N, int nv, int P16, R* __restrict__ S) {
  const int64_t n = (int64_t)NG * LF_K * P16;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(e % P16);
    const int k = (int)((e / P16) % LF_K);
    const int64_t g = e / ((int64_t)P16 * LF_K);
    double v = 0.0;
    if (k < M && p < nv + N) {
      const int row = p < nv ? rows[N + p] : rows[p - nv];
      v = L[((size_t)g * M + row) * M + k];
    }
    S[e] = R(v);
  }
}

int ltl_rows16(const DevSpin& sa, const DevSpin& sb) {
  return (max(sa.nv, sb.nv) + LM_N + 15) / 16 * 16;
}

bool ltl_mfma_fits(const DevSpin& sa, const DevSpin& sb, int M, bool fp32) {
  for (const DevSpin* s : {&sa, &sb})  // the occupied-window order is checked by the caller
    if (s->N != LM_N || s->no != LM_N) return false;
  if (M > LF_K) return false;
  const int P16 = ltl_rows16(sa, sb);
  if (P16 > 64) return false;  // P = 8 + n_vir_act <= M <= 64
  return lf_lds_bytes(P16, fp32 ? 4 : 8) <= 160 * 1024;
}

size_t ltl_stage_elems(const DevSpin& sa, const DevSpin& sb) {
  return (size_t)LF_K * ltl_rows16(sa, sb);
}

void launch_gather_ltl(const double* L, int NG, int M, const DevSpin& D, int P16, double* S64,
                       float* S32, hipStream_t st) {
  const int64_t n = (int64_t)NG * LF_K * P16;
  if (n == 0) return;
  const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
  if (S64)
    hipLaunchKernelGGL(k_gather_lf<double>, dim3(blocks), dim3(256), 0, st, L, NG, M, D.rows, D.N,
                       D.nv, P16, S64);
  if (S32)
    hipLaunchKernelGGL(k_gather_lf<float>, dim3(blocks), dim3(256), 0, st, L, NG, M, D.rows, D.N,
                       D.nv, P16, S32);
}

namespace {
template <class R>
void launch_ltl_t(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                  int g_chunk, int M, const R* Sa, const R* Sb, const typename Mfma<R>::cx_t* Ta,
                  const typename Mfma<R>::cx_t* Tb, typename Mfma<R>::cx_t* Lam_a,
                  typename Mfma<R>::cx_t* Lam_b, const cd* v0, const cd* Ca, const cd* Cb, cd* czw,
                  bool swz, hipStream_t st) {
  const int P16 = ltl_rows16(sa, sb), NT = P16 / 16;
  const int n_chunks = (NG + g_chunk - 1) / g_chunk;
  const int n_wgrp = (WT + LF_WB - 1) / LF_WB;
  const dim3 grid(n_wgrp * n_chunks * 2), block(64 * LF_WAVES);
  const size_t lds = lf_lds_bytes(P16, sizeof(R));
#define LTL_CASE(nt)                                                                          \
  case nt:                                                                                    \
    hipLaunchKernelGGL((k_ltl_mfma<R, nt>), grid, block, lds, st, sa, sb, NW, w0, WT, NG,     \
                       g_chunk, n_chunks, M, P16, Sa, Sb, Ta, Tb, Lam_a, Lam_b, v0, Ca, Cb, czw, swz); \
    break;
  switch (NT) {
    LTL_CASE(1)
    LTL_CASE(2)
    LTL_CASE(3)
    LTL_CASE(4)
    default:
      break;
  }
#undef LTL_CASE
}
}  // namespace

void launch_ltl_mfma(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                     int g_chunk, int M, const double* Sa, const double* Sb, const cd* Ta,
                     const cd* Tb, cd* Lam_a, cd* Lam_b, const cd* v0, const cd* Ca,
                     const cd* Cb, cd* czw, bool swz, hipStream_t st) {
  launch_ltl_t<double>(sa, sb, NW, w0, WT, NG, g_chunk, M, Sa, Sb, Ta, Tb, Lam_a, Lam_b, v0, Ca,
                       Cb, czw, swz, st);
}

void launch_ltl_mfma32(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                       int g_chunk, int M, const float* Sa, const float* Sb, const cf* Ta,
                       const cf* Tb, cf* Lam_a, cf* Lam_b, const cd* v0, const cd* Ca,
                       const cd* Cb, cd* czw, bool swz, hipStream_t st) {
  launch_ltl_t<float>(sa, sb, NW, w0, WT, NG, g_chunk, M, Sa, Sb, Ta, Tb, Lam_a, Lam_b, v0, Ca,
                      Cb, czw, swz, st);
}

// ============================================================================
// Mean-field traces in FP64 on the matrix cores (N = 8 per spin, M <= 64):
// v0 = tr Q and ex0 = tr QQ of Q^g = L^g[R, :] T, two vectors per tile,
//   D = [Tr Ti]^T [S_R^g | S_R^{g+1}]        (16 x 16 = (16 x 64)(64 x 16)),
// D[j][c] = Re / Im (j < 8 / j >= 8) of Q^{g + c / 8}[c % 8][j % 8], with
// S_R^g[k][i] = L^g[R_i, k] (k-major, zero for k >= M).  One wave per
// (walker, spin) and chunk of vectors; the tile goes through LDS for the
// products Q_in Q_ni.
// ============================================================================

constexpr int QT_WAVES = 8;
constexpr int QT_LD = 17;  // row stride of the LDS tile (doubles)

// one DPP move of a double (row-local lane permutation dpp_ctrl)
template <int CTRL>
__device__ __forceinline__ double qt_dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// sum over the 16 lanes of a row, in every lane of it: xor 1 and xor 2 by
// quad permutations, then the half-row mirror (quads 0 <-> 1) and the row
// mirror (halves 0 <-> 1)
__device__ __forceinline__ double qt_sum16(double v) {
  v += qt_dpp<0xB1>(v);
  v += qt_dpp<0x4E>(v);
  v += qt_dpp<0x141>(v);
  v += qt_dpp<0x140>(v);
  return v;
}

__global__ __launch_bounds__(64 * QT_WAVES) void k_qtr(int NW, int w0, int WT, int NG, int g_chunk,
                                                       int M, const double* __restrict__ SRa,
                                                       const double* __restrict__ SRb,
                                                       const cd* __restrict__ Ta,
                                                       const cd* __restrict__ Tb,
                                                       cd* __restrict__ v0, cd* __restrict__ ex0) {
  __shared__ double dt[QT_WAVES][16 * QT_LD];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s2 = blockIdx.z, chunk = blockIdx.y;
  const int wl = blockIdx.x * QT_WAVES + wv;
  if (wl >= WT) return;  // no barriers below
  const int w = w0 + wl;
  const double* __restrict__ SR = s2 ? SRb : SRa;
  const cd* __restrict__ T = s2 ? Tb : Ta;
  const int col = lane & 15, q = lane >> 4;
  double bt[LF_K / 4];
#pragma unroll
  for (int s = 0; s < LF_K / 4; ++s) {
    const int k = 4 * s + q;
    double v = 0.0;
    if (k < M) {
      const cd t = T[((size_t)k * NW + w) * LM_N + (col & 7)];
      v = col < 8 ? t.re : t.im;
    }
    bt[s] = v;
  }
  double* d_t = dt[wv];
  // products: row q of lanes takes vector g + q (q < 2); lane col: i = col / 2,
  // n = 4 (col % 2) .. + 3
  const int h = q & 1, i = col >> 1, nb = 4 * (col & 1);
  const int g0 = chunk * g_chunk, g1 = min(NG, g0 + g_chunk);
  // B operands of the next vector pair are loaded while this pair is formed
  auto load = [&](int g, double* b) __attribute__((always_inline)) {
    const int gg = min(g + (col >> 3), NG - 1);  // the second of a last odd vector is unused
#pragma unroll
    for (int s = 0; s < LF_K / 4; ++s) b[s] = SR[((size_t)gg * LF_K + 4 * s + q) * LM_N + (col & 7)];
  };
  double bcur[LF_K / 4], bnxt[LF_K / 4];
  if (g0 < g1) load(g0, bcur);
  for (int g = g0; g < g1; g += 2) {
    if (g + 2 < g1) load(g + 2, bnxt);
    // two independent accumulation chains (even and odd k steps)
    dvec4 d = dvec4{0, 0, 0, 0}, e = dvec4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < LF_K / 4; s += 2) {
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(bt[s], bcur[s], d, 0, 0, 0);
      e = __builtin_amdgcn_mfma_f64_16x16x4f64(bt[s + 1], bcur[s + 1], e, 0, 0, 0);
    }
    d += e;
#pragma unroll
    for (int r = 0; r < 4; ++r) d_t[(q + 4 * r) * QT_LD + col] = d[r];
    cd x{0.0, 0.0}, dv{0.0, 0.0};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int n = nb + m;
      const cd qin{d_t[n * QT_LD + 8 * h + i], d_t[(8 + n) * QT_LD + 8 * h + i]};
      const cd qni{d_t[i * QT_LD + 8 * h + n], d_t[(8 + i) * QT_LD + 8 * h + n]};
      x = x + qin * qni;
      if (n == i) dv = qin;
    }
    x.re = qt_sum16(x.re);
    x.im = qt_sum16(x.im);
    dv.re = qt_sum16(dv.re);
    dv.im = qt_sum16(dv.im);
    if (col == 0 && q < 2 && g + h < g1) {
      v0[((size_t)s2 * NW + w) * NG + g + h] = dv;
      ex0[((size_t)s2 * NW + w) * NG + g + h] = x;
    }
    if (g + 2 < g1) {
#pragma unroll
      for (int s = 0; s < LF_K / 4; ++s) bcur[s] = bnxt[s];
    }
  }
}

void launch_qtr(int NW, int w0, int WT, int NG, int M, const double* SRa, const double* SRb,
                const cd* Ta, const cd* Tb, cd* v0, cd* ex0, int n_cu, hipStream_t st) {
  // about two workgroups per CU in one round; chunks even, so vector pairs
  // never straddle them
  const int n_wx = (WT + QT_WAVES - 1) / QT_WAVES;
  const int n_chunks = std::max(1, std::min((NG + 1) / 2, (2 * n_cu + n_wx) / (2 * n_wx)));
  int g_chunk = (NG + n_chunks - 1) / n_chunks;
  g_chunk += g_chunk & 1;
  const dim3 grid((WT + QT_WAVES - 1) / QT_WAVES, (NG + g_chunk - 1) / g_chunk, 2);
  hipLaunchKernelGGL(k_qtr, grid, dim3(64 * QT_WAVES), 0, st, NW, w0, WT, NG, g_chunk, M, SRa,
                     SRb, Ta, Tb, v0, ex0);
}

void init_ltl_attributes() {
  const int lim = 160 * 1024;
  for (const void* f :
       {(const void*)k_ltl_mfma<double, 1>, (const void*)k_ltl_mfma<double, 2>,
        (const void*)k_ltl_mfma<double, 3>, (const void*)k_ltl_mfma<double, 4>,
        (const void*)k_ltl_mfma<float, 1>, (const void*)k_ltl_mfma<float, 2>,
        (const void*)k_ltl_mfma<float, 3>, (const void*)k_ltl_mfma<float, 4>})
    hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

}  // namespace msd

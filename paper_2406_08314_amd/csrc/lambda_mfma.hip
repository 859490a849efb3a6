// A6 on the matrix cores: energy intermediates of Sec. III for shapes with
// N = 8 electrons per spin and the whole occupied set in the excitation
// window (slot i = orbital i of the reference).
//
// Per (walker w, Cholesky vector g, spin), with LT^g = L^g[R u V, :] T (P x N,
// P = N + n_vir_act, from the LT GEMM, one contiguous tile per (w, g)):
//   Q = LT[R, :],  v0 = tr Q,  ex0 = tr QQ,
//   Lam = T[V, :] Q - LT[V, :]            (n_vir_act x N)
//   Xi  = Lam Q                            (window columns = all N)
//   ZW += Xi - (v0_alpha + v0_beta) Lam     (summed over the workgroup's vectors)
//   Lam -> HBM (window layout [w][g][a * N + i]).
// In the mixed form v0 and ex0 come from FP64 tiles of Q (Q64a/b, [w][g][8 x 8])
// instead of the FP32 LT tile.
// Both complex products are real GEMMs on v_mfma_{f64,f32}_16x16x4:
//   [Lr Li] = [Tr Ti] [[Qr Qi]; [-Qi Qr]]   (64 x 16 = (64 x 16)(16 x 16))
// with A = [Tr Ti] of the walker's virtual rows held in registers for all
// vectors, C initialised with -LT[V, :], and Xi = [Lr Li] times the same
// block matrix.  One wave per (walker, chunk of vectors, spin); the LT tiles
// arrive by direct global-to-LDS loads, double-buffered one vector ahead.
#include <hip/hip_runtime.h>

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

constexpr int LM_N = 8;         // electrons per spin of this kernel
constexpr int LM_ROWS = 64;     // virtual rows (zero padded)
constexpr int LM_PMAX = LM_N + LM_ROWS;
constexpr int LS_LD = 2 * LM_N + 2;  // row stride (reals) of the Lambda transpose buffer

}  // namespace

template <class R>
__global__ __launch_bounds__(64) void k_lambda_mfma(DevSpin sa, DevSpin sb, int NW, int w0,
                                                    int WT, int NG, int g_chunk,
                                                    const typename Mfma<R>::cx_t* __restrict__ Ta,
                                                    const typename Mfma<R>::cx_t* __restrict__ Tb,
                                                    const typename Mfma<R>::cx_t* __restrict__ LTa,
                                                    const typename Mfma<R>::cx_t* __restrict__ LTb,
                                                    typename Mfma<R>::cx_t* __restrict__ Lam_a,
                                                    typename Mfma<R>::cx_t* __restrict__ Lam_b,
                                                    cd* __restrict__ v0, cd* __restrict__ ex0,
                                                    cd* __restrict__ ZWa, cd* __restrict__ ZWb,
                                                    const cd* __restrict__ Q64a,
                                                    const cd* __restrict__ Q64b) {
  typedef typename Mfma<R>::cx_t C;
  typedef typename Mfma<R>::acc_t acc_t;
  // LT tiles (double buffer) and the Lambda transpose, all in LDS
  __shared__ __align__(16) C lt[2][LM_PMAX * LM_N];
  __shared__ R ls[LM_ROWS * LS_LD];
  const int wl = blockIdx.x, chunk = blockIdx.y, n_chunks = gridDim.y, s2 = blockIdx.z;
  const int w = w0 + wl, lane = threadIdx.x;
  const int nv = s2 ? sb.nv : sa.nv, P = LM_N + nv, X = nv * LM_N;
  const int* __restrict__ vir = s2 ? sb.vir : sa.vir;
  const C* __restrict__ T = s2 ? Tb : Ta;
  const C* __restrict__ LT = s2 ? LTb : LTa;
  const C* __restrict__ LTo = s2 ? LTa : LTb;
  const int Po = LM_N + (s2 ? sa.nv : sb.nv);
  C* __restrict__ Lam = s2 ? Lam_b : Lam_a;
  cd* __restrict__ ZW = s2 ? ZWb : ZWa;
  const int col = lane & 15, kq = lane >> 4;  // MFMA operand column / k quarter

  // A = [Tr Ti] of the virtual rows: A[row][k], k < 8 real part of T[vir[row]][k],
  // k >= 8 imaginary part of T[vir[row]][k - 8]; operand lane l: row l % 16, k 4s + l / 16
  R av[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int row = rt * 16 + col, k = 4 * s + kq;
      R v = R(0);
      if (row < nv) {
        const C t = T[((size_t)vir[row] * NW + w) * LM_N + (k & 7)];
        v = k < 8 ? t.re : t.im;
      }
      av[rt][s] = v;
    }
  acc_t zw[4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) zw[rt] = acc_t{0, 0, 0, 0};

  const int g0 = chunk * g_chunk, g1 = min(NG, g0 + g_chunk);
  const int tile = P * LM_N;  // complex entries of one LT tile
  auto fetch = [&](int g, int b) {
    const C* src = LT + ((size_t)wl * NG + g) * tile;
    constexpr int per = 16 / sizeof(C);
    const int n16 = tile / per;
    for (int c = 0; c * 64 < n16; ++c) {
      const int e = c * 64 + lane;
      if (e < n16) dma16(src + (size_t)e * per, &lt[b][c * 64 * per]);
    }
  };
  if (g0 < g1) fetch(g0, 0);
  int it = 0;
  for (int g = g0; g < g1; ++g, ++it) {
    const int b = it & 1;
    __syncthreads();  // tile b has landed; the other buffer's readers are done
    if (g + 1 < g1) fetch(g + 1, b ^ 1);
    const C* Q = lt[b];  // rows 0..7 = Q, rows 8.. = LT[V]
    // traces: v0 (this spin and the other), ex0 = sum_jc Q_jc Q_cj; from the
    // FP64 Q tiles when given (mixed form), else from this tile
    R vr, vi;
    if (Q64a) {
      const cd* q = (s2 ? Q64b : Q64a) + ((size_t)wl * NG + g) * LM_N * LM_N;
      const cd* qo = (s2 ? Q64a : Q64b) + ((size_t)wl * NG + g) * LM_N * LM_N;
      const cd qe = q[(lane >> 3) * LM_N + (lane & 7)];
      cd x = qe * q[(lane & 7) * LM_N + (lane >> 3)];
      cd vd = (lane >> 3) == (lane & 7) ? qe : cd{0.0, 0.0};
      cd vo = lane < LM_N ? qo[lane * LM_N + lane] : cd{0.0, 0.0};
      vd.re = wsum(vd.re);
      vd.im = wsum(vd.im);
      x.re = wsum(x.re);
      x.im = wsum(x.im);
      vo.re = wsum(vo.re);
      vo.im = wsum(vo.im);
      if (lane == 0) {
        v0[((size_t)s2 * NW + w) * NG + g] = vd;
        ex0[((size_t)s2 * NW + w) * NG + g] = x;
      }
      vr = R(vd.re + vo.re);
      vi = R(vd.im + vo.im);
    } else {
      C qe = Q[(lane >> 3) * LM_N + (lane & 7)];
      C qt = Q[(lane & 7) * LM_N + (lane >> 3)];
      C x = qe * qt;
      C vd = (lane >> 3) == (lane & 7) ? qe : C{};
      const C* o = LTo + ((size_t)wl * NG + g) * Po * LM_N;
      C vo = lane < LM_N ? o[lane * LM_N + lane] : C{};
      vd.re = wsum(vd.re);
      vd.im = wsum(vd.im);
      x.re = wsum(x.re);
      x.im = wsum(x.im);
      vo.re = wsum(vo.re);
      vo.im = wsum(vo.im);
      if (lane == 0) {
        v0[((size_t)s2 * NW + w) * NG + g] = to_cd(vd);
        ex0[((size_t)s2 * NW + w) * NG + g] = to_cd(x);
      }
      vr = vd.re + vo.re;
      vi = vd.im + vo.im;
    }
    // block matrix [[Qr Qi]; [-Qi Qr]]: operand lane l, k 4s + l / 16, column l % 16
    R bq[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 4 * s + kq;
      const C q = Q[(k & 7) * LM_N + (col & 7)];
      bq[s] = k < 8 ? (col < 8 ? q.re : q.im) : (col < 8 ? -q.im : q.re);
    }
    // Lam = A Bq - LT[V]
    acc_t lam[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = rt * 16 + Mfma<R>::row(lane, r);
        R v = R(0);
        if (a < nv) {
          const C t = Q[(LM_N + a) * LM_N + (col & 7)];
          v = -(col < 8 ? t.re : t.im);
        }
        lam[rt][r] = v;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) lam[rt] = Mfma<R>::run(av[rt][s], bq[s], lam[rt]);
    }
    // Lambda to LDS (row-major [a][re 0..7 | im 0..7]) for the store and as the
    // A operand of Xi
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) ls[(rt * 16 + Mfma<R>::row(lane, r)) * LS_LD + col] = lam[rt][r];
    __syncthreads();
    // window store: Lam[w][g][a * 8 + i]
    C* lo = Lam + ((size_t)wl * NG + g) * X;
    for (int e = lane; e < X; e += 64) {
      const int a = e >> 3, i = e & 7;
      lo[e] = C{ls[a * LS_LD + i], ls[a * LS_LD + 8 + i]};
    }
    // Xi = [Lr Li] Bq and ZW += Xi - vsum Lam (the partner real/imaginary
    // column of a lane is lane ^ 8)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      acc_t xi = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        xi = Mfma<R>::run(ls[(rt * 16 + col) * LS_LD + 4 * s + kq], bq[s], xi);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const R own = lam[rt][r];
        const R other = __shfl_xor(own, 8, 64);
        const R lr = col < 8 ? own : other, li = col < 8 ? other : own;
        const R sl = col < 8 ? vr * lr - vi * li : vr * li + vi * lr;
        zw[rt][r] += xi[r] - sl;
      }
    }
  }
  // ZW partial of this chunk: [wl][chunk][a * 8 + i]
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const R own = zw[rt][r];
      const R other = __shfl_xor(own, 8, 64);
      const int a = rt * 16 + Mfma<R>::row(lane, r);
      if (col < 8 && a < nv)
        ZW[((size_t)wl * n_chunks + chunk) * X + a * LM_N + col] = cd{(double)own, (double)other};
    }
}

bool lambda_mfma_fits(const DevSpin& sa, const DevSpin& sb) {
  for (const DevSpin* s : {&sa, &sb})
    if (s->N != LM_N || s->no != LM_N || s->nv > LM_ROWS) return false;
  return true;  // the occupied-window order is checked by the caller
}

void launch_lambda_mfma(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                        int g_chunk, const cd* Ta, const cd* Tb, const cd* LTa, const cd* LTb,
                        cd* Lam_a, cd* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a, cd* ZWpart_b,
                        hipStream_t st) {
  const dim3 grid(WT, (NG + g_chunk - 1) / g_chunk, 2);
  hipLaunchKernelGGL(k_lambda_mfma<double>, grid, dim3(64), 0, st, sa, sb, NW, w0, WT, NG,
                     g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0, ZWpart_a, ZWpart_b,
                     (const cd*)nullptr, (const cd*)nullptr);
}

void launch_lambda_mfma32(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                          int g_chunk, const cf* Ta, const cf* Tb, const cf* LTa, const cf* LTb,
                          cf* Lam_a, cf* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a, cd* ZWpart_b,
                          const cd* Q64a, const cd* Q64b, hipStream_t st) {
  const dim3 grid(WT, (NG + g_chunk - 1) / g_chunk, 2);
  hipLaunchKernelGGL(k_lambda_mfma<float>, grid, dim3(64), 0, st, sa, sb, NW, w0, WT, NG,
                     g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0, ZWpart_a, ZWpart_b, Q64a,
                     Q64b);
}

}  // namespace msd

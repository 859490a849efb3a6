// A2 + A6 on the matrix cores for general shapes: the Cholesky contraction
// and the energy intermediates of the generalised-Wick local energy (Sec. III;
// App. A), for up to 64 electrons per spin, M <= 320 orbitals and an
// excitation window of at most 32 virtual and 32 occupied orbitals.
//
// Per (walker w, spin, Cholesky vector g), with T = Phi A^{-1} (M x N) and
// S^g = L^g[V u R, :] (rows: the n_v window virtual orbitals, zero padded to
// nv16, then the N reference orbitals, zero padded to Np):
//   LT  = S^g T                        (P16 x M)(M x N)
//   Q   = LT[R rows]  (= L^g[R, :] T),  v0 = tr Q,  ex0 = tr(Q Q)
//   Lam = T[V, :] Q - LT[V rows]       (n_v x N)
//   D   = C Q_W^T                      (n_v x n_o)(n_o x N), with C the walker's
//         first-order CI matrix and Q_W = Q[:, window slots]
//   czw += <Lam, D>                    (= <C, (Lam Q)[:, window slots]>, summed over g)
//   lc_g = <C, Lam[:, window slots]>   (per g; the energy assembly multiplies
//                                       it by v0_alpha + v0_beta of the same g)
//   Lam[:, window slots] -> HBM        (window layout [w][g][a * n_o + i])
// (<X, Y> = sum_ij X_ij Y_ij, no conjugation.)
//
// Every complex product is a real GEMM on v_mfma_{f64,f32}_16x16x4.  A complex
// matrix Z with Np columns is held as 2 Np real columns in tiles of 16: tile t
// holds Re Z[:, 8t .. 8t+7] in its columns 0-7 and Im of the same columns in
// 8-15, so the two parts of one complex entry sit in lanes l and l ^ 8.  Wave
// t of a workgroup owns column tile t of LT, Lam and D; its B operand of LT
// (the walker's T for those columns, all M orbitals) stays in registers for
// the whole chunk of vectors.  S^g streams through LDS in slabs of 16
// orbitals by direct global-to-LDS loads, a ring of four buffers over the
// flattened (vector, slab) sequence with three slabs in flight, so the next
// vector's first slabs load during the current vector's epilogue.  The
// traces v0, ex0 and lc_g are written as per-wave partials ([..][g][wave]),
// summed by the energy assembly.  One workgroup per (spin, vector chunk,
// walker).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace msd {

namespace {

typedef double gdvec4 __attribute__((ext_vector_type(4)));
typedef float gfvec4 __attribute__((ext_vector_type(4)));

template <class R>
struct GMfma;
template <>
struct GMfma<double> {
  typedef gdvec4 acc_t;
  typedef cd cx_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // register r of lane l holds D[l/16 + 4r][l % 16]
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct GMfma<float> {
  typedef gfvec4 acc_t;
  typedef cf cx_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // register r of lane l holds D[4 (l/16) + r][l % 16]
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int GL_KS = 16;      // orbitals per LDS slab of S^g
constexpr int GL_NB = 4;       // slab buffers (three slabs in flight)
constexpr int GL_VTMAX = 2;    // virtual row tiles (n_v <= 32)
constexpr int GL_OMAX = 32;    // window occupied orbitals
constexpr int GL_KSL2 = 11;    // T in registers at two workgroups per CU: at most 11 slabs

__device__ __forceinline__ void gl_dma16(const void* g, void* lds) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
#endif
}
// all of this wave's memory operations (including direct-to-LDS loads) done,
// then the workgroup barrier
__device__ __forceinline__ void gl_bar_all() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// at most N of this wave's vector-memory operations outstanding (the older
// ones, including direct-to-LDS loads, done) and all its LDS operations done,
// then the workgroup barrier.  gfx9 s_waitcnt: vmcnt in bits 3:0 and 15:14,
// expcnt 6:4, lgkmcnt 11:8.
template <int N>
__device__ __forceinline__ void gl_bar_vm_lds() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  constexpr int imm = (N & 15) | ((N >> 4) << 14) | (7 << 4);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(imm);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// this wave's LDS writes done, then the workgroup barrier
__device__ __forceinline__ void gl_bar_lds() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ double gl_wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// one DPP move (row-local lane permutation CTRL) of a float or a double;
// lanes of rows outside ROWS read 0
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float gl_dpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double gl_dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double gl_readlane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// sum over the wave without LDS: within each row of 16 lanes by DPP (quad
// swaps xor 1 and xor 2, then the half-row and row mirrors), then row 1 +=
// row 0 and row 3 += row 2 (broadcast of lane 15 of each row), then row 3 +=
// row 1 (broadcast of lane 31); lane 63 holds the total, returned
// wave-uniform
__device__ __forceinline__ double gl_wsum_dpp(double v) {
  v += gl_dpp<0xB1>(v);
  v += gl_dpp<0x4E>(v);
  v += gl_dpp<0x141>(v);
  v += gl_dpp<0x140>(v);
  v += gl_dpp<0x142, 0xA>(v);
  v += gl_dpp<0x143, 0xC>(v);
  return gl_readlane(v, 63);
}
// the value of lane l ^ 8 (the other part of the same complex entry in the
// tile layout): a rotation of each 16-lane row by 8
template <class R>
__device__ __forceinline__ R gl_other_part(R v) {
  return gl_dpp<0x128>(v);
}

// The orbital (K) axis of LT = L^g T is split at the reference: T[R, :] is
// the identity, so LT = L^g[:, nR] T[nR, :] + L^g[:, R] (nR: the M - N
// orbitals outside the reference).  Only the nR rows of T enter the
// matrix-core products (in slabs of 16, zero padded: gl_mn of them); the
// reference columns of L^g come first as Np / 16 slabs whose entries start
// the real part of LT.
__host__ __device__ inline int gl_mn(int M, int N) { return (M - N + GL_KS - 1) / GL_KS * GL_KS; }

struct GlShape {
  int nv16, Np, P16, no16, Mn;  // Mn: rows of T kept (outside the reference, padded)
};

__host__ __device__ inline GlShape gl_shape(int no, int M, int N, int NCT, int VT) {
  GlShape s;
  s.nv16 = VT * 16;
  s.Np = 8 * NCT;
  s.P16 = s.nv16 + s.Np;
  s.no16 = no <= 16 ? 16 : 32;
  s.Mn = gl_mn(M, N);
  return s;
}

// direct-load pieces (16 bytes) per slab, rounded up to whole waves of every
// wave of the workgroup: each wave issues the same number of slab loads, so a
// fixed vmcnt tells when a slab has landed; the loads beyond the slab land in
// a pad after the buffer
__host__ __device__ constexpr int gl_slab_loads(int P16, int rsize, int NCT) {
  const int pieces = GL_KS * P16 * rsize / 16;
  return (pieces + 64 * NCT - 1) / (64 * NCT);
}
__host__ __device__ constexpr int gl_slab_stride(int P16, int rsize, int NCT) {
  return gl_slab_loads(P16, rsize, NCT) * NCT * 64 * 16 / rsize;  // reals
}

// LDS reals: the slab ring (GL_NB buffers of 16 x P16, padded), Q (Np x Np
// complex, rows padded to 2 Np + 1 reals so that a wave's reads down a column
// of Q hit distinct banks), [Re C | Im C] k-major (2 no16 x nv16) and
// [Re T_V | Im T_V] k-major (2 Np x nv16).  With TL (the walker's T held in
// LDS, [Mn][2 Np + 1], instead of in registers): three slab buffers and no
// separate T_V block (its rows are read from T).
__host__ __device__ constexpr int gl_nb(bool TL) { return TL ? 3 : GL_NB; }
__host__ __device__ inline int gl_lds_reals(const GlShape& s, int rsize, int NCT, bool TL) {
  const int common = gl_nb(TL) * gl_slab_stride(s.P16, rsize, NCT) + s.Np * (2 * s.Np + 1) +
                     2 * s.no16 * s.nv16;
  if (TL) return common + s.Mn * (2 * s.Np + 1);
  return common + 2 * s.Np * s.nv16;
}

}  // namespace

// LIST: the instance that walks a walker list (a separate instance, so that
// the grid form's register allocation is not touched by the list form's item
// arithmetic)
template <class R, int NCT, int KSL, int VT, bool TL, bool LIST>
__global__ __launch_bounds__(64 * NCT, (TL || KSL > GL_KSL2) ? 1 : 2) void k_ltl_general(
    DevSpin sa, DevSpin sb, int NW, int w0, int WT, int NG, int g_chunk, int n_chunks, int M,
    const R* __restrict__ Sa, const R* __restrict__ Sb,
    const typename GMfma<R>::cx_t* __restrict__ Ta, const typename GMfma<R>::cx_t* __restrict__ Tb,
    typename GMfma<R>::cx_t* __restrict__ Lam_a, typename GMfma<R>::cx_t* __restrict__ Lam_b,
    const cd* __restrict__ Ca, const cd* __restrict__ Cb, cd* __restrict__ v0,
    cd* __restrict__ ex0, cd* __restrict__ lamc, cd* __restrict__ czw,
    const int* __restrict__ wmask, const int* __restrict__ wlist, const int* __restrict__ wcount,
    int swz) {
  typedef GMfma<R> MF;
  typedef typename MF::cx_t C;
  typedef typename MF::acc_t acc_t;
  constexpr int Np = 8 * NCT;
  constexpr int RT = VT + NCT / 2;  // row tiles of LT (P16 / 16)
  constexpr int P16 = 16 * RT;
  constexpr int nv16 = 16 * VT;
  extern __shared__ __align__(16) unsigned char gl_raw[];
  R* lds = reinterpret_cast<R*>(gl_raw);

  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int col = lane & 15, q = lane >> 4;
  const int part = col >> 3;             // 0: real part, 1: imaginary part
  const int j = 8 * wv + (col & 7);      // complex column of this lane
  // Work items (walker, vector chunk, spin): one per workgroup (grid mode),
  // or, with a walker list, a persistent grid striding over the items of the
  // listed walkers (a few walkers then still spread over the chip without a
  // launch of idle workgroups)
  // With a list, an item takes grp consecutive vector chunks: as few as still
  // give about two items per resident workgroup (single chunks for a handful
  // of listed walkers, runs as long as the grid mode's for a full list); its
  // <C, Lam Q> partial goes to the first chunk's slot and the others of its
  // group are cleared, so the slots still sum to the walker's total.
  int grp = 1, n_grp = n_chunks;
  if constexpr (LIST) {
    const int nl = max(*wcount, 1);
    const int want = min(n_chunks, (int)((2 * gridDim.x + 2 * nl - 1) / (2 * nl)));
    for (int d = n_chunks; d >= 1; --d)
      if (n_chunks % d == 0 && n_chunks / d >= want) {
        grp = d;
        break;
      }
    n_grp = n_chunks / grp;
  }
  const int n_items = LIST ? *wcount * 2 * n_grp : 1;
  for (int it = LIST ? (int)blockIdx.x : 0; it < n_items; it += LIST ? (int)gridDim.x : 1) {
  int wl, chunk, s2;
  if constexpr (LIST) {
    // listed walker fastest, as the grid order below: the workgroups resident
    // together stream the same slabs of L (one chunk of one spin)
    const int nl = *wcount;
    wl = wlist[it % nl] - w0;
    chunk = ((it / nl) % n_grp) * grp;
    s2 = it / (nl * n_grp);
    if (wl < 0 || wl >= WT) continue;  // listed walker outside this walker tile
  } else {
    const int b = blockIdx.x;
    wl = b % WT;
    chunk = (b / WT) % n_chunks;
    s2 = b / (WT * n_chunks);
    if (wmask && !wmask[w0 + wl]) return;  // walker not selected for this pass
  }
  const int g0 = chunk * g_chunk, g1 = min(NG, g0 + (LIST ? grp : 1) * g_chunk);
  if (g1 <= g0) continue;  // no vectors in this chunk (uniform)
  const int w = w0 + wl;
  if constexpr (LIST) {  // the <C, Lam Q> slots of the group's other chunks stay zero
    if (lane == 0)
      for (int c = 1; c < grp; ++c)
        czw[(((size_t)s2 * NW + w) * n_chunks + chunk + c) * NCT + wv] = cd{0.0, 0.0};
  }
  const DevSpin& D = s2 ? sb : sa;
  const int N = D.N, nv = D.nv, no = D.no, X = nv * no;
  const GlShape sh = gl_shape(no, M, N, NCT, VT);
  // per vector: n_rs slabs of the reference columns (added), then n_nr slabs
  // of L^g[:, nR] (products with T); srows rows of S per vector
  const int no16 = sh.no16, n_nr = sh.Mn / GL_KS, n_rs = Np / GL_KS, n_sl = n_nr + n_rs;
  const int srows = sh.Mn + Np;
  const C* __restrict__ T = s2 ? Tb : Ta;
  const R* __restrict__ S = s2 ? Sb : Sa;
  C* __restrict__ Lam = s2 ? Lam_b : Lam_a;
  const cd* __restrict__ Cw = (s2 ? Cb : Ca) + (size_t)w * X;

  // LDS carve-up
  constexpr int NB = gl_nb(TL);
  constexpr int SLOADS = gl_slab_loads(P16, (int)sizeof(R), NCT);
  constexpr int SSTRIDE = gl_slab_stride(P16, (int)sizeof(R), NCT);
  constexpr int QLD = 2 * Np + 1;           // row stride of Q and T (reals)
  R* sS = lds;                              // [NB][SSTRIDE] (16 x P16 used)
  R* sQ = sS + NB * SSTRIDE;                // [Np][QLD]: (re, im) of column j at 2j
  R* sCA = sQ + Np * QLD;                   // [2 no16][nv16]
  R* sTV = sCA + 2 * no16 * nv16;           // !TL: [2 Np][nv16]
  R* sT = sCA + 2 * no16 * nv16;            // TL: [Mn][QLD], column c of tile t at 16 t + c

  // window index of this lane's column (slot j), -1 outside the window
  int wi = -1;
  for (int i = 0; i < no; ++i)
    if (D.oslot[i] == j) wi = i;

  // offsets (reals) of Q[.][slot(i)] for this lane's window rows i = 4 u + q
  // of the D product, -1 beyond n_o
  int qs[GL_OMAX / 4];
#pragma unroll
  for (int u = 0; u < GL_OMAX / 4; ++u) qs[u] = 4 * u + q < no ? 2 * D.oslot[4 * u + q] : -1;

  const int nthr = 64 * NCT;
  for (int e = threadIdx.x; e < 2 * no16 * nv16; e += nthr) {
    const int k = e / nv16, a = e % nv16, kc = k % no16;
    R v = R(0);
    if (a < nv && kc < no) {
      const cd c = Cw[a * no + kc];
      v = R(k < no16 ? c.re : c.im);
    }
    sCA[e] = v;
  }
  // B operand of LT: T[k][j] (real or imaginary part) for k = 4s + q, in
  // registers (!TL) or in LDS (TL)
  R bt[TL ? 1 : 4 * KSL];
  int vrow[VT];  // TL: orbital of this lane's rows of T_V (-1 beyond n_v)
  if constexpr (TL) {
    // T[nR[k]][w][j] as 2 Np real columns per kept orbital k, in the tile layout
    for (int e = threadIdx.x; e < sh.Mn * 2 * Np; e += nthr) {
      const int k = e / (2 * Np), c = e % (2 * Np);
      const int jj = 8 * (c >> 4) + (c & 7), pp = (c >> 3) & 1;
      R v = R(0);
      if (k < M - N && jj < N) {
        const C t = T[((size_t)D.nref[k] * NW + w) * N + jj];
        v = pp ? t.im : t.re;
      }
      sT[k * QLD + c] = v;
    }
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) {
      const int a = vt * 16 + col;
      vrow[vt] = a < nv ? D.vpos[a] : -1;  // position of the virtual among the kept rows
    }
  } else {
    // [Re T_V | Im T_V]
    for (int e = threadIdx.x; e < 2 * Np * nv16; e += nthr) {
      const int k = e / nv16, a = e % nv16, kc = k % Np;
      R v = R(0);
      if (a < nv && kc < N) {
        const C t = T[((size_t)D.vir[a] * NW + w) * N + kc];
        v = k < Np ? t.re : t.im;
      }
      sTV[e] = v;
    }
#pragma unroll
    for (int s = 0; s < 4 * KSL; ++s) {
      const int k = 4 * s + q;  // kept row
      R v = R(0);
      if (k < M - N && j < N) {
        const C t = T[((size_t)D.nref[k] * NW + w) * N + j];
        v = part ? t.im : t.re;
      }
      bt[s] = v;
    }
  }

  // slab ring over the flattened (vector, slab) sequence: slab t = (g0 + t /
  // n_sl, t % n_sl) sits in buffer t % NB.  The slabs of consecutive vectors
  // are contiguous in S, so the fetch pointer advances by one slab per fetch.
  // Every step issues the same loads (past the last slab they re-read it into
  // a buffer nobody reads), so the wait before slab t is always the same
  // count: the loads of slabs t+1 .. t+NB-2 may be outstanding.
  const int n_t = (g1 - g0) * n_sl;
  constexpr int SLAB = GL_KS * P16;  // reals per slab in S
  const R* fsrc = S + (size_t)g0 * srows * P16;
  const R* const flast = fsrc + (size_t)(n_t - 1) * SLAB;
  int ft = 0, fbuf = 0, cb = 0;
  auto fetch_next = [&]() {
    constexpr int per16 = 16 / sizeof(R);
    const R* src = ft < n_t ? fsrc : flast;  // uniform
    R* dst = sS + fbuf * SSTRIDE;
    constexpr int n16 = SLAB / per16;
#pragma unroll
    for (int u = 0; u < SLOADS; ++u) {
      const int c = u * NCT + wv, e = min(c * 64 + lane, n16 - 1);  // pad lanes re-read
      gl_dma16(src + (size_t)e * per16, dst + c * 64 * per16);
    }
    fsrc += SLAB;
    ++ft;
    fbuf = fbuf + 1 == NB ? 0 : fbuf + 1;
  };
  // before the reads of slab t: slab t has landed and every wave is done
  // with slab t - 1, whose buffer then takes slab t + NB - 1
  auto slab_sync = [&]() {
    gl_bar_vm_lds<(NB - 2) * SLOADS>();
    fetch_next();
  };
  // one slab of LT: 4 k-steps of RT tiles
  auto slab = [&](acc_t* acc, int sl, auto&& bval) {
    slab_sync();
    const R* sb0 = sS + cb * SSTRIDE;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      R a[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) a[rt] = sb0[(4 * s + q) * P16 + rt * 16 + col];
      const R bv = bval(sl, s);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) acc[rt] = MF::run(a[rt], bv, acc[rt]);
    }
    cb = cb + 1 == NB ? 0 : cb + 1;
  };

  // <Lam, D> summed over the chunk: the sign of the real part (- on the
  // imaginary-part lanes) is applied once at the end
  double dot_re = 0.0, dot_im = 0.0;
  // lc_g = <C, Lam_W> coefficients of this lane's Lam entries: C at its
  // window entry, signed and zeroed outside the window.  Constant over the
  // chunk: read once with T in LDS, per vector with T in registers (whose
  // register budget is two workgroups per CU).
  gl_bar_lds();  // the C block is in LDS
  R lcr[VT][4], lci[VT][4];
  auto lc_read = [&]() {
#pragma unroll
    for (int vt = 0; vt < VT; ++vt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = vt * 16 + MF::row(lane, r);
        const bool inw = wi >= 0 && a < nv;
        const int wic = max(wi, 0);
        const R cr = inw ? sCA[wic * nv16 + a] : R(0);
        const R ci = inw ? sCA[(no16 + wic) * nv16 + a] : R(0);
        lcr[vt][r] = part ? -ci : cr;
        lci[vt][r] = part ? cr : ci;
      }
  };
  if constexpr (TL) lc_read();
  for (int u = 0; u < NB - 1; ++u) fetch_next();
  for (int g = g0; g < g1; ++g) {
    // ---- LT = S^g T over slabs of 16 orbitals
    acc_t acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt] = acc_t{0, 0, 0, 0};
    // the reference columns first (the order of the orbital sum the products
    // then continue): slab u holds L^g[p, r_j] for j = 16u .. 16u + 15, the
    // start of the real part of LT[p][j] (the wave's columns j lie in slab
    // wv / 2)
    for (int u = 0; u < n_rs; ++u) {
      slab_sync();
      const R* sb0 = sS + cb * SSTRIDE;
      if (u == (j >> 4)) {  // wave-uniform
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const R v = sb0[(j & 15) * P16 + rt * 16 + MF::row(lane, r)];
            acc[rt][r] += part ? R(0) : v;
          }
      }
      cb = cb + 1 == NB ? 0 : cb + 1;
    }
    if constexpr (TL) {
      // B from the LDS copy of T: a loop over the slabs, two at a time, the
      // operands of the next slab read from LDS while the current slab's
      // products run (the accumulators stay in place throughout).  A slab's
      // first k-step is issued before the synchronisation for the next slab;
      // the refill and the next slab's reads are then interleaved with the
      // other three k-steps, so the matrix cores have work queued while the
      // wave issues them.  The synchronisation also waits for this wave's
      // earlier LDS reads, so the buffer refilled there (the slab read before
      // the current one) is free in every wave.
      const R* tcol = sT + q * QLD + 16 * wv + col;
      auto read = [&](R (&a)[4][RT], R (&bv)[4], int sl) {
        const R* sb0 = sS + cb * SSTRIDE;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
#pragma unroll
          for (int rt = 0; rt < RT; ++rt) a[s][rt] = sb0[(4 * s + q) * P16 + rt * 16 + col];
          bv[s] = tcol[(16 * sl + 4 * s) * QLD];
        }
        cb = cb + 1 == NB ? 0 : cb + 1;
      };
      auto kstep = [&](const R (&a)[4][RT], const R (&bv)[4], int s) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt] = MF::run(a[s][rt], bv[s], acc[rt]);
      };
      // the current slab's k-steps 1..3 (3 RT products) with the next slab's
      // refill and reads (4 RT + 4 values, mostly merged pairwise by the
      // compiler) placed between them
      auto rest_and_next = [&](const R (&a)[4][RT], const R (&bv)[4], R (&na)[4][RT],
                               R (&nb)[4], int nsl) {
        slab_sync();
        __builtin_amdgcn_sched_barrier(0);
        read(na, nb, nsl);
        kstep(a, bv, 1);
        kstep(a, bv, 2);
        kstep(a, bv, 3);
        // two reads after each of the first products: every read is issued
        // well before the next slab's first product (an LDS read after a
        // direct-to-LDS load is waited for in full before its first use)
#pragma unroll
        for (int i = 0; i < 3 * RT / 2; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one product
          __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // two LDS reads
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 3 * RT - 3 * RT / 2, 0);
        __builtin_amdgcn_sched_barrier(0);
      };
      auto rest = [&](const R (&a)[4][RT], const R (&bv)[4]) {
        kstep(a, bv, 1);
        kstep(a, bv, 2);
        kstep(a, bv, 3);
      };
      if constexpr (RT <= 4) {
        R a0[4][RT], b0[4], a1[4][RT], b1[4];
        slab_sync();
        read(a0, b0, 0);
        int sl = 0;
        for (; sl + 2 < n_nr; sl += 2) {  // two slabs, each followed by another
          kstep(a0, b0, 0);
          __builtin_amdgcn_sched_barrier(0);
          rest_and_next(a0, b0, a1, b1, sl + 1);
          kstep(a1, b1, 0);
          __builtin_amdgcn_sched_barrier(0);
          rest_and_next(a1, b1, a0, b0, sl + 2);
        }
        // the last one or two slabs
        kstep(a0, b0, 0);
        __builtin_amdgcn_sched_barrier(0);
        if (sl + 1 < n_nr) {
          rest_and_next(a0, b0, a1, b1, sl + 1);
          kstep(a1, b1, 0);
          rest(a1, b1);
        } else {
          rest(a0, b0);
        }
      } else {
        // five or more row tiles: one operand set (a second one would spill)
        for (int sl = 0; sl < n_nr; ++sl) {
          R a0[4][RT], b0[4];
          slab_sync();
          read(a0, b0, sl);
          kstep(a0, b0, 0);
          rest(a0, b0);
        }
      }
    } else {
      // B from registers (compile-time indices): unrolled over KSL slabs
#pragma unroll
      for (int sl = 0; sl < KSL; ++sl)
        if (sl < n_nr) slab(acc, sl, [&](int l, int s) { return bt[4 * l + s]; });
    }
    // ---- Lam = T_V Q - LT_V: K = 2 Np over [Re T_V | Im T_V].  In FP64 the
    // B operand Q[k][j] is this lane's own accumulator (register r of lane
    // group q holds row q + 4r of its tile: row k = 4 kk + q is register kk %
    // 4 of tile kk / 4), the other part of the complex entry one DPP row
    // rotation away, so the products need no LDS and run before the barrier
    // that publishes Q; in FP32 (row 4q + r) Q is read back from LDS.
    constexpr bool EARLY_LAM = sizeof(R) == 8;
    acc_t lam[VT];
    // The LDS operands of the Lam and D products are read one group ahead:
    // a group's reads are issued after the first product of the group before
    // (once direct-to-LDS loads are in flight, the first use of an LDS read
    // waits for every LDS read issued before it, so reads issued any earlier
    // would be waited for with the previous group).
    constexpr int KK = 2 * Np / 4;  // k-steps of the Lam products
    auto lam_phase = [&]() {
#pragma unroll
      for (int vt = 0; vt < VT; ++vt)
#pragma unroll
        for (int r = 0; r < 4; ++r) lam[vt][r] = -acc[vt][r];
      R lav[KK][VT], lbq[EARLY_LAM ? 1 : KK];
      // A: [Re T_V | Im T_V] row a = vt * 16 + col, column k = 4 kk + q
      // (rows beyond n_v read row 0 and are zeroed); FP32: B = Q[k][j].  The
      // loaded values are not touched before their products (any arithmetic
      // on them would wait for the whole group of reads).
      auto lread = [&](int kk) {
        const int k = 4 * kk + q;
        const bool hi = kk >= Np / 4;  // imaginary rows of the block form of Q
        const int kr = hi ? k - Np : k;
        const int tcol = 16 * (kr >> 3) + 8 * (hi ? 1 : 0) + (kr & 7);
#pragma unroll
        for (int vt = 0; vt < VT; ++vt) {
          if constexpr (TL) lav[kk][vt] = sT[max(vrow[vt], 0) * QLD + tcol];
          else lav[kk][vt] = sTV[k * nv16 + vt * 16 + col];
        }
        if constexpr (!EARLY_LAM) {
          const int comp = hi ? 1 - part : part;
          lbq[kk] = sQ[kr * QLD + 2 * j + comp];
        }
      };
      auto lmma = [&](int kk) {
        R bq;
        if constexpr (EARLY_LAM) {
          const bool hi = kk >= Np / 4;
          const int kq = hi ? kk - Np / 4 : kk;
          const R own = acc[VT + kq / 4][kq % 4];
          if (hi) {
            const R oth = gl_other_part(own);
            bq = part ? oth : -oth;
          } else {
            bq = own;
          }
        } else {
          const bool hi = kk >= Np / 4;
          bq = hi && !part ? -lbq[kk] : lbq[kk];
        }
#pragma unroll
        for (int vt = 0; vt < VT; ++vt) {
          const R av = TL && vrow[vt] < 0 ? R(0) : lav[kk][vt];
          lam[vt] = MF::run(av, bq, lam[vt]);
        }
      };
      // groups of two k-steps
      lread(0);
      lread(1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int p = 0; p < KK / 2; ++p) {
        lmma(2 * p);
        lmma(2 * p + 1);
        if (p + 1 < KK / 2) {
          lread(2 * p + 2);
          lread(2 * p + 3);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 2);
        __builtin_amdgcn_sched_group_barrier(0x100, 2 * (VT + (EARLY_LAM ? 0 : 1)), 2);
        __builtin_amdgcn_sched_group_barrier(0x008, 2 * VT - 1, 2);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    if constexpr (EARLY_LAM) lam_phase();
    // ---- Q (rows >= nv16 of LT) and its window columns, transposed, to LDS
#pragma unroll
    for (int rt = VT; rt < RT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = rt * 16 + MF::row(lane, r) - nv16;
        sQ[i * QLD + 2 * j + part] = acc[rt][r];
      }
    gl_bar_lds();
    // ---- this wave's parts of the mean-field traces: v0 = sum_i Q_ii and
    // ex0 = sum_ij Q_ij Q_ji over the entries Q_ij in its columns (branch-free:
    // a lane holds Re Q_ij (part 0) or Im Q_ij (part 1))
    double vdg = 0.0, xr = 0.0, xi = 0.0;
#pragma unroll
    for (int rt = VT; rt < RT; ++rt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = rt * 16 + MF::row(lane, r) - nv16;
        const double a = (double)acc[rt][r];
        const double br = (double)sQ[j * QLD + 2 * i], bi = (double)sQ[j * QLD + 2 * i + 1];
        vdg += i == j ? a : 0.0;
        xr = fma(a, part ? -bi : br, xr);
        xi = fma(a, part ? br : bi, xi);
      }
    double vr = part ? 0.0 : vdg, vi = part ? vdg : 0.0;
    if constexpr (!EARLY_LAM) lam_phase();
    // ---- D = C Q_W^T: K = 2 no16 over [Re C | Im C]; the B operand is
    // Q[j][slot(i)] (k = i: real rows, k = no16 + i: imaginary rows)
    acc_t dd[VT];
#pragma unroll
    for (int vt = 0; vt < VT; ++vt) dd[vt] = acc_t{0, 0, 0, 0};
    auto dphase = [&](auto nc) {
      constexpr int NO16 = decltype(nc)::value;
      constexpr int NU = NO16 / 4;
      R qv[NU][2], ca[NU][2][VT];
      auto dread = [&](int u) {
        // rows beyond n_o read slot 0 and are zeroed
        const int o = j * QLD + max(qs[u], 0);
        qv[u][0] = sQ[o];
        qv[u][1] = sQ[o + 1];
#pragma unroll
        for (int vt = 0; vt < VT; ++vt) {
          ca[u][0][vt] = sCA[(4 * u + q) * nv16 + vt * 16 + col];
          ca[u][1][vt] = sCA[(NO16 + 4 * u + q) * nv16 + vt * 16 + col];
        }
      };
      dread(0);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const R qre = qs[u] >= 0 ? qv[u][0] : R(0), qim = qs[u] >= 0 ? qv[u][1] : R(0);
        const R blo = part ? qim : qre, bhi = part ? qre : -qim;
#pragma unroll
        for (int vt = 0; vt < VT; ++vt) dd[vt] = MF::run(ca[u][0][vt], blo, dd[vt]);
#pragma unroll
        for (int vt = 0; vt < VT; ++vt) dd[vt] = MF::run(ca[u][1][vt], bhi, dd[vt]);
        if (u + 1 < NU) dread(u + 1);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 3);
        __builtin_amdgcn_sched_group_barrier(0x100, 2 + 2 * VT, 3);
        __builtin_amdgcn_sched_group_barrier(0x008, 2 * VT - 1, 3);
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    if (no16 == 16) dphase(std::integral_constant<int, 16>{});
    else dphase(std::integral_constant<int, 32>{});
    // ---- <Lam, D> (accumulated), lc_g = <C, Lam_W> (branch-free), window store
    double lr = 0.0, li = 0.0;
    if constexpr (!TL) lc_read();
#pragma unroll
    for (int vt = 0; vt < VT; ++vt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double lv = (double)lam[vt][r];
        const double dv = (double)dd[vt][r];
        const double dp = (double)gl_other_part(dd[vt][r]);  // other part of D
        dot_re = fma(lv, dv, dot_re);
        dot_im = fma(lv, dp, dot_im);
        lr = fma((double)lcr[vt][r], lv, lr);
        li = fma((double)lci[vt][r], lv, li);
        const int a = vt * 16 + MF::row(lane, r);
        if (wi >= 0 && a < nv) {
          const int e = a * no + wi;
          R* dst = reinterpret_cast<R*>(Lam + ((size_t)wl * NG + g) * X + (swz ? lam_swizzle(e, swz) : e));
          dst[part] = lam[vt][r];
        }
      }
    lr = gl_wsum_dpp(lr);
    li = gl_wsum_dpp(li);
    vr = gl_wsum_dpp(vr);
    vi = gl_wsum_dpp(vi);
    xr = gl_wsum_dpp(xr);
    xi = gl_wsum_dpp(xi);
    if (lane == 0) {
      const size_t o = (((size_t)s2 * NW + w) * NG + g) * NCT + wv;
      lamc[o] = cd{lr, li};
      v0[o] = cd{vr, vi};
      ex0[o] = cd{xr, xi};
    }
  }
  dot_re = gl_wsum(part ? -dot_re : dot_re);
  dot_im = gl_wsum(dot_im);
  if (lane == 0) czw[((size_t)s2 * NW + w) * n_chunks * NCT + chunk * NCT + wv] = cd{dot_re, dot_im};
  gl_bar_all();  // the re-reads past the last slab have landed; the next item rewrites the LDS
  }
}

// S[g][k][p] = L^g[row(p), orb(k)]: p < nv the window virtual orbitals, nv16
// <= p < nv16 + N the reference orbitals, zero elsewhere; k = j < Np the
// reference orbital r_j (zero for j >= N), then k = Np + i the orbitals
// outside the reference (nref[i], zero beyond M - N).  Np + Mn rows per vector.
template <class R>
__global__ void k_gather_general(const double* __restrict__ L, int NG, int M, int Mn, int srows,
                                 const int* __restrict__ ref, int N, const int* __restrict__ nref,
                                 const int* __restrict__ vir, int nv, int nv16, int P16,
                                 R* __restrict__ S) {
  const int64_t n = (int64_t)NG * srows * P16;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(e % P16);
    const int k = (int)((e / P16) % srows);
    const int64_t g = e / ((int64_t)P16 * srows);
    const int Np = srows - Mn;
    int orb = -1;
    if (k < Np) orb = k < N ? ref[k] : -1;
    else if (k - Np < M - N) orb = nref[k - Np];
    int row = -1;
    if (p < nv) row = vir[p];
    else if (p >= nv16 && p < nv16 + N) row = ref[p - nv16];
    double v = 0.0;
    if (orb >= 0 && row >= 0) v = L[((size_t)g * M + row) * M + orb];
    S[e] = R(v);
  }
}

int ltl_general_nct(const DevSpin& sa, const DevSpin& sb) {
  const int n = std::max(sa.N, sb.N);
  return 2 * ((n + 15) / 16);
}

int ltl_general_vt(const DevSpin& sa, const DevSpin& sb) {
  return std::max(sa.nv, sb.nv) <= 16 ? 1 : 2;
}

// slabs of 16 kept rows of T (outside the reference) for the larger spin,
// rounded up to an instantiated count (T in registers needs it at compile time)
int ltl_general_ksl(int M, int Nmin) {
  const int n = gl_mn(M, Nmin) / GL_KS;
  for (int k : {4, 8, GL_KSL2, 20})
    if (n <= k) return k;
  return 0;
}

// Where the walker's T lives.  In FP64 at four column tiles (16 < N <= 32)
// T in LDS fills it, so one workgroup runs per CU and its barriers and
// epilogue leave the matrix cores idle; with T in registers (each wave holds
// its column tile, at most GL_KSL2 slabs: 44 values a lane) the LDS holds only
// the slab ring, Q, C and T_V and two workgroups share a CU, each one's
// products running through the other's waits.  Otherwise T in LDS where it
// fits (any precision, one or more workgroups per CU), else T in registers at
// one workgroup per CU (FP64, four or six column tiles, at most 20 slabs; six
// tiles always take the 20-slab instance).
enum GlMode { GL_NONE, GL_TL, GL_REG };
static GlMode gl_mode(const DevSpin& sa, const DevSpin& sb, int M, size_t rsize) {
  const int nct = ltl_general_nct(sa, sb), ksl = ltl_general_ksl(M, std::min(sa.N, sb.N));
  const GlShape s = gl_shape(std::max(sa.no, sb.no), M, std::min(sa.N, sb.N), nct,
                             ltl_general_vt(sa, sb));
  const size_t reg = (size_t)gl_lds_reals(s, 8, nct, false) * 8;
  if (rsize == 8 && nct == 4 && ksl <= GL_KSL2 && 2 * reg <= 160 * 1024) return GL_REG;
  if ((size_t)gl_lds_reals(s, (int)rsize, nct, true) * rsize <= 160 * 1024) return GL_TL;
  if (rsize == 8 && ((nct == 4 && ksl == 20) || nct == 6) && reg <= 160 * 1024) return GL_REG;
  return GL_NONE;
}

bool ltl_general_fits(const DevSpin& sa, const DevSpin& sb, int M, bool fp32) {
  const int nct = ltl_general_nct(sa, sb), ksl = ltl_general_ksl(M, std::min(sa.N, sb.N));
  if (nct < 2 || nct > 6 || ksl == 0) return false;
  for (const DevSpin* d : {&sa, &sb}) {
    if (d->N == 0 || d->nv == 0 || d->nv > GL_VTMAX * 16 || d->no > GL_OMAX) return false;
  }
  return gl_mode(sa, sb, M, fp32 ? 4 : 8) != GL_NONE;
}

bool ltl_general_fast64(const DevSpin& sa, const DevSpin& sb, int M) {
  return !(ltl_general_nct(sa, sb) == 6 && gl_mode(sa, sb, M, 8) == GL_REG);
}

// elements of one spin's S array (sized for the spin with more kept rows)
size_t ltl_general_s_elems(const DevSpin& sa, const DevSpin& sb, int M, int NG) {
  const GlShape s = gl_shape(std::max(sa.no, sb.no), M, std::min(sa.N, sb.N),
                             ltl_general_nct(sa, sb), ltl_general_vt(sa, sb));
  return (size_t)NG * (s.Mn + s.Np) * s.P16;
}

void launch_gather_general(const double* L, int NG, int M, const DevSpin& D, const DevSpin& sa,
                           const DevSpin& sb, double* S64, float* S32, hipStream_t st) {
  const GlShape s = gl_shape(D.no, M, D.N, ltl_general_nct(sa, sb), ltl_general_vt(sa, sb));
  const int srows = s.Mn + s.Np;
  const int64_t n = (int64_t)NG * srows * s.P16;
  if (n == 0) return;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 65536);
  if (S64)
    hipLaunchKernelGGL(k_gather_general<double>, dim3(blocks), dim3(256), 0, st, L, NG, M, s.Mn,
                       srows, D.ref, D.N, D.nref, D.vir, D.nv, s.nv16, s.P16, S64);
  if (S32)
    hipLaunchKernelGGL(k_gather_general<float>, dim3(blocks), dim3(256), 0, st, L, NG, M, s.Mn,
                       srows, D.ref, D.N, D.nref, D.vir, D.nv, s.nv16, s.P16, S32);
}

namespace {
template <class R, int NCT, int KSL, int VT, bool TL>
void gl_launch(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG, int g_chunk,
               int n_chunks, int M, const R* Sa, const R* Sb, const typename GMfma<R>::cx_t* Ta,
               const typename GMfma<R>::cx_t* Tb, typename GMfma<R>::cx_t* Lam_a,
               typename GMfma<R>::cx_t* Lam_b, const cd* Ca, const cd* Cb, cd* v0, cd* ex0,
               cd* lamc, cd* czw, const int* wmask, const WalkerList& wls, int swz,
               hipStream_t st) {
  const GlShape s = gl_shape(std::max(sa.no, sb.no), M, std::min(sa.N, sb.N), NCT, VT);
  const size_t lds = (size_t)gl_lds_reals(s, sizeof(R), NCT, TL) * sizeof(R);
  const void* fg = (const void*)k_ltl_general<R, NCT, KSL, VT, TL, false>;
  const void* fl = (const void*)k_ltl_general<R, NCT, KSL, VT, TL, true>;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute(fg, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipFuncSetAttribute(fl, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  const dim3 block(64 * NCT);
  if (wls.list) {  // persistent grid: the workgroups resident at once
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fl, (int)block.x, lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const dim3 grid(std::max(1, wls.n_cu) * per_cu);
    hipLaunchKernelGGL((k_ltl_general<R, NCT, KSL, VT, TL, true>), grid, block, lds, st, sa, sb,
                       NW, w0, WT, NG, g_chunk, n_chunks, M, Sa, Sb, Ta, Tb, Lam_a, Lam_b, Ca, Cb,
                       v0, ex0, lamc, czw, wmask, wls.list, wls.count, swz);
    return;
  }
  hipLaunchKernelGGL((k_ltl_general<R, NCT, KSL, VT, TL, false>), dim3(WT * n_chunks * 2), block,
                     lds, st, sa, sb, NW, w0, WT, NG, g_chunk, n_chunks, M, Sa, Sb, Ta, Tb, Lam_a,
                     Lam_b, Ca, Cb, v0, ex0, lamc, czw, wmask, nullptr, nullptr, swz);
}

template <class R>
void gl_dispatch(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                 int g_chunk, int M, const R* Sa, const R* Sb, const typename GMfma<R>::cx_t* Ta,
                 const typename GMfma<R>::cx_t* Tb, typename GMfma<R>::cx_t* Lam_a,
                 typename GMfma<R>::cx_t* Lam_b, const cd* Ca, const cd* Cb, cd* v0, cd* ex0,
                 cd* lamc, cd* czw, const int* wmask, const WalkerList& wls, int swz,
                 hipStream_t st) {
  const int nct = ltl_general_nct(sa, sb), ksl = ltl_general_ksl(M, std::min(sa.N, sb.N)),
            vt = ltl_general_vt(sa, sb);
  const int n_chunks = (NG + g_chunk - 1) / g_chunk;
  const bool tl = gl_mode(sa, sb, M, sizeof(R)) == GL_TL;
  // T in LDS: the slab count is a run-time loop bound (one instance each, KSL 0)
#define GL_CASE(n, k, v, t)                                                                     \
  if (nct == n && (t || ksl == k) && vt == v && tl == t)                                        \
    return gl_launch<R, n, t ? 0 : k, v, t>(sa, sb, NW, w0, WT, NG, g_chunk, n_chunks, M, Sa, Sb, \
                                           Ta, Tb, Lam_a, Lam_b, Ca, Cb, v0, ex0, lamc, czw, wmask, \
                                           wls, swz, st);
  GL_CASE(2, 0, 1, true)
  GL_CASE(2, 0, 2, true)
  GL_CASE(4, 0, 1, true)
  GL_CASE(4, 0, 2, true)
  GL_CASE(6, 0, 1, true)
  GL_CASE(6, 0, 2, true)
  if constexpr (sizeof(R) == 8) {  // T in registers (FP64, four column tiles)
    GL_CASE(4, 4, 1, false)
    GL_CASE(4, 4, 2, false)
    GL_CASE(4, 8, 1, false)
    GL_CASE(4, 8, 2, false)
    GL_CASE(4, GL_KSL2, 1, false)
    GL_CASE(4, GL_KSL2, 2, false)
    GL_CASE(4, 20, 1, false)
    GL_CASE(4, 20, 2, false)
    if (nct == 6 && !tl) {  // six column tiles: the 20-slab instance for any slab count
      if (vt == 1)
        return gl_launch<R, 6, 20, 1, false>(sa, sb, NW, w0, WT, NG, g_chunk, n_chunks, M, Sa,
                                            Sb, Ta, Tb, Lam_a, Lam_b, Ca, Cb, v0, ex0, lamc, czw,
                                            wmask, wls, swz, st);
      return gl_launch<R, 6, 20, 2, false>(sa, sb, NW, w0, WT, NG, g_chunk, n_chunks, M, Sa, Sb,
                                          Ta, Tb, Lam_a, Lam_b, Ca, Cb, v0, ex0, lamc, czw, wmask,
                                          wls, swz, st);
    }
  }
#undef GL_CASE
}
}  // namespace

int ltl_general_parts(const DevSpin& sa, const DevSpin& sb) { return ltl_general_nct(sa, sb); }

void launch_ltl_general(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                        int g_chunk, int M, const double* Sa, const double* Sb, const cd* Ta,
                        const cd* Tb, cd* Lam_a, cd* Lam_b, const cd* Ca, const cd* Cb, cd* v0,
                        cd* ex0, cd* lamc, cd* czw, const int* wmask, int swz, hipStream_t st,
                        const WalkerList& wls) {
  gl_dispatch<double>(sa, sb, NW, w0, WT, NG, g_chunk, M, Sa, Sb, Ta, Tb, Lam_a, Lam_b, Ca, Cb,
                      v0, ex0, lamc, czw, wmask, wls, swz, st);
}

void launch_ltl_general32(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                          int g_chunk, int M, const float* Sa, const float* Sb, const cf* Ta,
                          const cf* Tb, cf* Lam_a, cf* Lam_b, const cd* Ca, const cd* Cb, cd* v0,
                          cd* ex0, cd* lamc, cd* czw, const int* wmask, int swz, hipStream_t st,
                          const WalkerList& wls) {
  gl_dispatch<float>(sa, sb, NW, w0, WT, NG, g_chunk, M, Sa, Sb, Ta, Tb, Lam_a, Lam_b, Ca, Cb, v0,
                     ex0, lamc, czw, wmask, wls, swz, st);
}

// Walkers for the FP64 energy pass of the mixed form: mask[w] = 1 where the
// largest |T_pj| of either spin exceeds tmax, rest[w] = 1 - mask[w].  One
// workgroup per walker.
__global__ __launch_bounds__(256) void k_walker_tmax(int NW, int M, int na, int nb,
                                                     const cd* __restrict__ Ta,
                                                     const cd* __restrict__ Tb, double tmax,
                                                     int* __restrict__ mask,
                                                     int* __restrict__ rest) {
  __shared__ double red[256];
  const int w = blockIdx.x, tid = threadIdx.x;
  double m = 0.0;
  for (int e = tid; e < M * na; e += 256) {
    const cd t = Ta[((size_t)(e / na) * NW + w) * na + e % na];
    m = fmax(m, t.re * t.re + t.im * t.im);
  }
  for (int e = tid; e < M * nb; e += 256) {
    const cd t = Tb[((size_t)(e / nb) * NW + w) * nb + e % nb];
    m = fmax(m, t.re * t.re + t.im * t.im);
  }
  red[tid] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] = fmax(red[tid], red[tid + off]);
    __syncthreads();
  }
  if (tid == 0) {
    const int f = red[0] > tmax * tmax ? 1 : 0;
    mask[w] = f;
    rest[w] = 1 - f;
  }
}

// The walkers with mask[w] != 0 in increasing order, list[0 .. *count); one
// workgroup (a ballot per wave, the wave counts summed in order).
__global__ __launch_bounds__(1024) void k_walker_list(int NW, const int* __restrict__ mask,
                                                      int* __restrict__ list,
                                                      int* __restrict__ count) {
  __shared__ int wsum[16];
  __shared__ int base;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  if (tid == 0) base = 0;
  __syncthreads();
  for (int b = 0; b < NW; b += blockDim.x) {
    const int w = b + tid;
    const bool f = w < NW && mask[w] != 0;
    const unsigned long long bal = __ballot(f);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(bal);
    __syncthreads();
    int off = base;
    for (int q = 0; q < wave; ++q) off += wsum[q];
    if (f) list[off + before] = w;
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int q = 0; q < nwaves; ++q) t += wsum[q];
      base += t;
    }
    __syncthreads();
  }
  if (tid == 0) *count = base;
}

void launch_walker_tmax(int NW, int M, int na, int nb, const cd* Ta, const cd* Tb, double tmax,
                        int* mask, int* rest, int* list, int* count, hipStream_t st) {
  hipLaunchKernelGGL(k_walker_tmax, dim3(NW), dim3(256), 0, st, NW, M, na, nb, Ta, Tb, tmax, mask,
                     rest);
  hipLaunchKernelGGL(k_walker_list, dim3(1), dim3(1024), 0, st, NW, mask, list, count);
}

}  // namespace msd

// Generalised-Wick evaluation of the MSD trial (Sec. III, App. A of the paper;
// Mahajan & Sharma's reference-based form).
//
// Per walker and spin, with R the reference orbitals and A = Phi[R, :]:
//   T = Phi A^{-1}                       (M x N)
//   X_I = T[P_I, slot(H_I)]^T            (k x k per string)
//   Obar = sum_I c~_I det X^a_I det X^b_I, c~_I = conj(c_I) sgn^a_I sgn^b_I
//   B^s_str = sum_{I contains str} c~_I det X^{other spin}_I
//   C^s[a, i] = sum_str B^s_str adj(X_str)[n, m]      (a = p_n, i = h_m)
//   G = G0 - (G0 - I)[:, V] C G0[O, :] / Obar        (Eq. 14 for the MSD trial)
// Energy (factorised; every term is exact):
//   Q^g = L^g[R, :] T, v0 = tr Q, ex0 = tr QQ, Lam^g = T[V,:] Q^g - (L^g T)[V,:],
//   Xi^g = Lam^g Q^g,  ZW = sum_g Xi^g - (v0^a + v0^b) Lam^g,
//   E_L = E0 + sum_s tr(h G^s) + sum_g (v0a v0b + (v0a^2-ex0a + v0b^2-ex0b)/2)
//         + [ sum_s <C^s, ZW^s> + sum_g ( sum_pairs W_ab coef_ab
//                                        + sum_s sum_minors det2(Lam^s) coef_s ) ] / Obar
// with the opposite-spin coefficients coef_ab[(a,i),(b,j)] =
// sum_I c~_I adj(X^a_I)[n,m] adj(X^b_I)[n',m'] and the same-spin ones
// coef_s[(a,b),(i,j)] = sum_str B_str (-1)^{m+m'+n+n'} det X_str[~{m,m'}, ~{n,n'}].
// All reductions use fixed orders (no atomics): results are run-to-run
// reproducible.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace msd {

// ============================================================================
// small complex determinants
// ============================================================================

template <int n>
__device__ __forceinline__ cd det_small(const cd* a);

template <>
__device__ __forceinline__ cd det_small<0>(const cd*) { return cd{1.0, 0.0}; }
template <>
__device__ __forceinline__ cd det_small<1>(const cd* a) { return a[0]; }
template <>
__device__ __forceinline__ cd det_small<2>(const cd* a) { return a[0] * a[3] - a[1] * a[2]; }
template <>
__device__ __forceinline__ cd det_small<3>(const cd* a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}
template <>
__device__ __forceinline__ cd det_small<4>(const cd* a) {
  // expansion along row 0 with the 2x2 minors of rows 2-3 shared
  cd m01 = a[8] * a[13] - a[9] * a[12];
  cd m02 = a[8] * a[14] - a[10] * a[12];
  cd m03 = a[8] * a[15] - a[11] * a[12];
  cd m12 = a[9] * a[14] - a[10] * a[13];
  cd m13 = a[9] * a[15] - a[11] * a[13];
  cd m23 = a[10] * a[15] - a[11] * a[14];
  cd c0 = a[5] * m23 - a[6] * m13 + a[7] * m12;
  cd c1 = a[4] * m23 - a[6] * m03 + a[7] * m02;
  cd c2 = a[4] * m13 - a[5] * m03 + a[7] * m01;
  cd c3 = a[4] * m12 - a[5] * m02 + a[6] * m01;
  return a[0] * c0 - a[1] * c1 + a[2] * c2 - a[3] * c3;
}

// Determinant of an n x n matrix (row-major, leading dimension n) by LU with
// partial pivoting on a private copy; exact zero for an exactly singular pivot.
__device__ cd det_lu(const cd* a, int n) {
  cd w[KMAX * KMAX];
  for (int i = 0; i < n * n; ++i) w[i] = a[i];
  cd det{1.0, 0.0};
  for (int j = 0; j < n; ++j) {
    int piv = j;
    double best = abs2(w[j * n + j]);
    for (int i = j + 1; i < n; ++i) {
      double v = abs2(w[i * n + j]);
      if (v > best) { best = v; piv = i; }
    }
    if (best == 0.0) return cd{0.0, 0.0};
    if (piv != j) {
      for (int c = 0; c < n; ++c) {
        cd t = w[j * n + c];
        w[j * n + c] = w[piv * n + c];
        w[piv * n + c] = t;
      }
      det = -det;
    }
    cd p = w[j * n + j];
    det = det * p;
    for (int i = j + 1; i < n; ++i) {
      cd f = cdiv(w[i * n + j], p);
      for (int c = j + 1; c < n; ++c) w[i * n + c] -= f * w[j * n + c];
    }
  }
  return det;
}

// ============================================================================
// A1: reference overlap, log det A and T = Phi A^{-1} (Gauss-Jordan, LDS)
// ============================================================================

__global__ __launch_bounds__(256) void k_ref_inverse(const cd* __restrict__ phi, int M, int Ntot,
                                                     int NW, DevSpin sa, DevSpin sb,
                                                     cd* __restrict__ Ta, cd* __restrict__ Tb,
                                                     cd* __restrict__ lda_, cd* __restrict__ ldb_,
                                                     int* __restrict__ flag) {
  extern __shared__ cd aug[];  // [N][2N]
  __shared__ cd fac[NMAX_LDS];
  __shared__ int piv_s;
  const bool beta = blockIdx.y == 1;
  const DevSpin& s = beta ? sb : sa;
  cd* __restrict__ T = beta ? Tb : Ta;
  cd* __restrict__ logdetA = beta ? ldb_ : lda_;
  if (s.N == 0) return;
  const int w = blockIdx.x, tid = threadIdx.x, bd = blockDim.x;
  const int N = s.N, N2 = 2 * N;
  const cd* P = phi + (size_t)w * M * Ntot + s.col0;
  for (int e = tid; e < N * N2; e += bd) {
    int i = e / N2, c = e % N2;
    aug[e] = c < N ? P[(size_t)s.ref[i] * Ntot + c] : cd{c - N == i ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  double lmag = 0.0, larg = 0.0;
  int nswap = 0;
  bool singular = false;
  for (int j = 0; j < N; ++j) {
    if (tid == 0) {
      int piv = j;
      double best = abs2(aug[j * N2 + j]);
      for (int i = j + 1; i < N; ++i) {
        double v = abs2(aug[i * N2 + j]);
        if (v > best) { best = v; piv = i; }
      }
      piv_s = (best > 0.0 && best < INFINITY) ? piv : -1;
    }
    __syncthreads();
    const int piv = piv_s;
    if (piv < 0) { singular = true; break; }
    if (piv != j) {
      for (int c = tid; c < N2; c += bd) {
        cd t = aug[j * N2 + c];
        aug[j * N2 + c] = aug[piv * N2 + c];
        aug[piv * N2 + c] = t;
      }
      ++nswap;
    }
    __syncthreads();
    const cd p = aug[j * N2 + j];
    if (tid == 0) {
      lmag += 0.5 * log(abs2(p));
      larg += atan2(p.im, p.re);
    }
    const cd inv = cdiv(cd{1.0, 0.0}, p);
    for (int i = tid; i < N; i += bd) fac[i] = aug[i * N2 + j];
    __syncthreads();
    for (int c = j + 1 + tid; c < N2; c += bd) aug[j * N2 + c] = aug[j * N2 + c] * inv;
    __syncthreads();
    for (int e = tid; e < N * (N2 - j - 1); e += bd) {
      int i = e / (N2 - j - 1), c = j + 1 + e % (N2 - j - 1);
      if (i != j) aug[i * N2 + c] -= fac[i] * aug[j * N2 + c];
    }
    __syncthreads();
  }
  if (singular) {
    for (int e = tid; e < M * N; e += bd) {
      int q = e / N, c = e % N;
      T[((size_t)q * NW + w) * N + c] = cd{0.0, 0.0};
    }
    if (tid == 0) {
      flag[w] = 1;
      logdetA[w] = cd{-INFINITY, 0.0};
    }
    return;
  }
  if (tid == 0) logdetA[w] = cd{lmag, larg + ((nswap & 1) ? M_PI : 0.0)};
  for (int e = tid; e < M * N; e += bd) {
    int q = e / N, c = e % N;
    cd acc{0.0, 0.0};
    const cd* row = P + (size_t)q * Ntot;
    for (int i = 0; i < N; ++i) cfma(acc, row[i], aug[i * N2 + N + c]);
    T[((size_t)q * NW + w) * N + c] = acc;
  }
}

void launch_ref_inverse(const cd* phi, int M, int Ntot, int NW, const DevSpin& sa,
                        const DevSpin& sb, cd* Ta, cd* Tb, cd* ldA, cd* ldB, int* flag,
                        hipStream_t st) {
  const int N = max(sa.N, sb.N);
  if (N == 0) return;
  size_t lds = (size_t)N * 2 * N * sizeof(cd);
  hipLaunchKernelGGL(k_ref_inverse, dim3(NW, 2), dim3(256), lds, st, phi, M, Ntot, NW, sa, sb,
                     Ta, Tb, ldA, ldB, flag);
}

// ============================================================================
// A3: per-string excitation determinants, adjugates, second-order minors
// ============================================================================

template <int K>
__device__ __forceinline__ void sub1(const cd* X, int rm, int cn, cd* out) {
  int o = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    if (r == rm) continue;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      if (c == cn) continue;
      out[o++] = X[r * K + c];
    }
  }
}

template <int K>
__device__ __forceinline__ void sub2(const cd* X, int r0, int r1, int c0, int c1, cd* out) {
  int o = 0;
#pragma unroll
  for (int r = 0; r < K; ++r) {
    if (r == r0 || r == r1) continue;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      if (c == c0 || c == c1) continue;
      out[o++] = X[r * K + c];
    }
  }
}

struct StrOut {
  const cd* T;
  cd* d;
  cd* adj;
  cd* m2;
};

// One (string of order K, walker) per thread; tid counts the threads of
// order K.
template <int K>
__device__ __forceinline__ void strings_body(const DevSpin& s, const StrOut& o, int NW,
                                             bool minors, int64_t tid) {
  const cd* __restrict__ T = o.T;
  cd* __restrict__ d = o.d;
  cd* __restrict__ adj = o.adj;
  cd* __restrict__ m2 = o.m2;
  const int s0 = s.bucket[K], ns = s.bucket[K + 1] - s.bucket[K];
  if (tid >= (int64_t)ns * NW) return;
  const int str = s0 + (int)(tid % ns);
  const int w = (int)(tid / ns);
  const int N = s.N;
  cd X[K > 0 ? K * K : 1];
#pragma unroll
  for (int m = 0; m < K; ++m)
#pragma unroll
    for (int n = 0; n < K; ++n)
      X[m * K + n] =
          T[((size_t)s.part[str * KMAX + n] * NW + w) * N + s.hslot[str * KMAX + m]];
  d[(size_t)w * s.U + str] = det_small<K>(X);
  if constexpr (K >= 1) {
    cd* ao = adj + (size_t)w * s.A + s.adj_off[str];
#pragma unroll
    for (int n = 0; n < K; ++n)
#pragma unroll
      for (int m = 0; m < K; ++m) {
        cd sub[(K - 1) * (K - 1) > 0 ? (K - 1) * (K - 1) : 1];
        sub1<K>(X, m, n, sub);
        cd v = det_small<K - 1>(sub);
        ao[n * K + m] = ((n + m) & 1) ? -v : v;
      }
  }
  if constexpr (K >= 2) {
    if (minors) {
      constexpr int P = K * (K - 1) / 2;
      cd* mo = m2 + (size_t)w * s.M2 + s.m2_off[str];
#pragma unroll
      for (int m = 0; m < K; ++m)
#pragma unroll
        for (int mp = m + 1; mp < K; ++mp)
#pragma unroll
          for (int n = 0; n < K; ++n)
#pragma unroll
            for (int np = n + 1; np < K; ++np) {
              cd sub[(K - 2) * (K - 2) > 0 ? (K - 2) * (K - 2) : 1];
              sub2<K>(X, m, mp, n, np, sub);
              mo[pair_index(m, mp, K) * P + pair_index(n, np, K)] = det_small<K - 2>(sub);
            }
    }
  }
}

// Orders 0-4 in one launch: the blocks of order k are [first[k], first[k+1])
// (block-uniform dispatch); blockIdx.y is the spin.
struct StrGrid {
  int first[6];
};

__global__ __launch_bounds__(256) void k_strings_t(DevSpin sa, DevSpin sb, StrOut oa, StrOut ob,
                                                   int NW, bool minors, StrGrid g) {
  const bool beta = blockIdx.y == 1;
  const DevSpin& s = beta ? sb : sa;
  const StrOut& o = beta ? ob : oa;
  const int b = blockIdx.x;
  int k = 0;
  while (k < 4 && b >= g.first[k + 1]) ++k;
  const int64_t tid = (int64_t)(b - g.first[k]) * blockDim.x + threadIdx.x;
  switch (k) {
    case 0: strings_body<0>(s, o, NW, minors, tid); break;
    case 1: strings_body<1>(s, o, NW, minors, tid); break;
    case 2: strings_body<2>(s, o, NW, minors, tid); break;
    case 3: strings_body<3>(s, o, NW, minors, tid); break;
    default: strings_body<4>(s, o, NW, minors, tid); break;
  }
}

// Orders above 4: one thread per output entry of a (walker, string) -- the
// determinant, one adjugate entry or one complementary two-minor -- each a
// D x D determinant (D = K, K - 1, K - 2) gathered from T and evaluated by LU
// with partial pivoting in registers (sizes fixed at compile time, so the
// matrices stay in registers).  Consecutive threads write consecutive entries.
template <int D>
__device__ __forceinline__ cd det_fixed(cd* w) {
  if constexpr (D <= 4) {
    return det_small<D>(w);
  } else {
    // row swaps and the zero-pivot exit as selects, so every index is a
    // compile-time constant
    cd det{1.0, 0.0};
    bool zero = false;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      int piv = j;
      double best = abs2(w[j * D + j]);
#pragma unroll
      for (int i = j + 1; i < D; ++i) {
        const double v = abs2(w[i * D + j]);
        piv = v > best ? i : piv;
        best = v > best ? v : best;
      }
      zero = zero || best == 0.0;
      if (piv != j) det = -det;
#pragma unroll
      for (int i = j + 1; i < D; ++i) {
        const bool sw = i == piv;
#pragma unroll
        for (int c = j; c < D; ++c) {
          const cd a = w[j * D + c], b = w[i * D + c];
          w[j * D + c] = sw ? b : a;
          w[i * D + c] = sw ? a : b;
        }
      }
      const cd p = zero ? cd{1.0, 0.0} : w[j * D + j];
      det = det * p;
#pragma unroll
      for (int i = j + 1; i < D; ++i) {
        const cd f = cdiv(w[i * D + j], p);
#pragma unroll
        for (int c = j + 1; c < D; ++c) w[i * D + c] -= f * w[j * D + c];
      }
    }
    return zero ? cd{0.0, 0.0} : det;
  }
}

// WHICH: 0 determinant, 1 adjugate entries, 2 complementary two-minors
template <int K, int WHICH>
__global__ __launch_bounds__(256) void k_str_entries(DevSpin sa, DevSpin sb, StrOut oa, StrOut ob,
                                                     int NW) {
  constexpr int P = K * (K - 1) / 2;
  constexpr int E = WHICH == 0 ? 1 : WHICH == 1 ? K * K : P * P;
  constexpr int D = WHICH == 0 ? K : WHICH == 1 ? K - 1 : K - 2;
  const bool beta = blockIdx.y == 1;
  const DevSpin& s = beta ? sb : sa;
  const StrOut& o = beta ? ob : oa;
  const int s0 = s.bucket[K], ns = s.bucket[K + 1] - s.bucket[K];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)ns * NW * E) return;
  const int e = (int)(tid % E);
  const int64_t r = tid / E;
  const int str = s0 + (int)(r % ns), w = (int)(r / ns);
  // excluded rows (holes m) and columns (particles n)
  int xr0 = -1, xr1 = -1, xc0 = -1, xc1 = -1;
  if constexpr (WHICH == 1) {
    xc0 = e / K;  // adj(X)[n][m] = (-1)^(n+m) det X without row m, column n
    xr0 = e % K;
  } else if constexpr (WHICH == 2) {
    const int A = e / P, B = e % P;
    int acc = 0;
    for (int m = 0; m < K; ++m)
      for (int mp = m + 1; mp < K; ++mp, ++acc) {
        if (acc == A) {
          xr0 = m;
          xr1 = mp;
        }
        if (acc == B) {
          xc0 = m;
          xc1 = mp;
        }
      }
  }
  // u-th kept row / column: skip the excluded ones (x0 < x1, -1 = none), with
  // compile-time u so the index arrays stay in registers
  auto kept = [](int u, int x0, int x1) {
    int m = (x0 >= 0 && u >= x0) ? u + 1 : u;
    if (x1 >= 0 && m >= x1) ++m;
    return m;
  };
  int rs[D > 0 ? D : 1], cs[D > 0 ? D : 1];
#pragma unroll
  for (int u = 0; u < D; ++u) {
    rs[u] = s.hslot[str * KMAX + kept(u, xr0, xr1)];
    cs[u] = s.part[str * KMAX + kept(u, xc0, xc1)];
  }
  cd a[D > 0 ? D * D : 1];
  const cd* __restrict__ T = o.T;
  const int N = s.N;
#pragma unroll
  for (int u = 0; u < D; ++u)
#pragma unroll
    for (int v = 0; v < D; ++v) a[u * D + v] = T[((size_t)cs[v] * NW + w) * N + rs[u]];
  const cd det = det_fixed<D>(a);
  if constexpr (WHICH == 0) {
    o.d[(size_t)w * s.U + str] = det;
  } else if constexpr (WHICH == 1) {
    o.adj[(size_t)w * s.A + s.adj_off[str] + e] = ((xr0 + xc0) & 1) ? -det : det;
  } else {
    o.m2[(size_t)w * s.M2 + s.m2_off[str] + e] = det;
  }
}

template <int K>
static void launch_str_entries(const DevSpin& sa, const DevSpin& sb, const StrOut& oa,
                               const StrOut& ob, int NW, bool minors, hipStream_t st) {
  const int ns = max(sa.bucket[K + 1] - sa.bucket[K], sb.bucket[K + 1] - sb.bucket[K]);
  if (ns <= 0) return;
  constexpr int P = K * (K - 1) / 2;
  const int64_t n0 = (int64_t)ns * NW, n1 = n0 * K * K, n2 = n0 * P * P;
  hipLaunchKernelGGL((k_str_entries<K, 0>), dim3((unsigned)((n0 + 255) / 256), 2), dim3(256), 0,
                     st, sa, sb, oa, ob, NW);
  hipLaunchKernelGGL((k_str_entries<K, 1>), dim3((unsigned)((n1 + 255) / 256), 2), dim3(256), 0,
                     st, sa, sb, oa, ob, NW);
  if (minors)
    hipLaunchKernelGGL((k_str_entries<K, 2>), dim3((unsigned)((n2 + 255) / 256), 2), dim3(256), 0,
                       st, sa, sb, oa, ob, NW);
}

void launch_strings(const DevSpin& sa, const DevSpin& sb, const cd* Ta, const cd* Tb, int NW,
                    bool minors, const SpinWork& wa, const SpinWork& wb, hipStream_t st) {
  const StrOut oa{Ta, wa.d, wa.adj, wa.m2}, ob{Tb, wb.d, wb.adj, wb.m2};
  StrGrid g{};
  int64_t nb = 0;
  for (int k = 0; k <= KMAX; ++k) {
    const int ns = max(sa.bucket[k + 1] - sa.bucket[k], sb.bucket[k + 1] - sb.bucket[k]);
    const int64_t n = (int64_t)max(ns, 0) * NW;
    if (k <= 4) {
      g.first[k] = (int)nb;
      nb += (n + 255) / 256;
      continue;
    }
  }
  launch_str_entries<5>(sa, sb, oa, ob, NW, minors, st);
  launch_str_entries<6>(sa, sb, oa, ob, NW, minors, st);
  launch_str_entries<7>(sa, sb, oa, ob, NW, minors, st);
  launch_str_entries<8>(sa, sb, oa, ob, NW, minors, st);
  g.first[5] = (int)nb;
  if (nb > 0)
    hipLaunchKernelGGL(k_strings_t, dim3((unsigned)nb, 2), dim3(256), 0, st, sa, sb, oa, ob, NW,
                       minors, g);
}

// ============================================================================
// block reduction helper (fixed order)
// ============================================================================

__device__ cd block_reduce(cd v, cd* red) {
  const int tid = threadIdx.x, bd = blockDim.x;
  red[tid] = v;
  __syncthreads();
  for (int off = bd / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  cd r = red[0];
  __syncthreads();
  return r;
}

// ============================================================================
// A3: trial overlap Obar = sum_I c~_I det X^a det X^b (compensated sums)
// ============================================================================

__global__ __launch_bounds__(256) void k_ovlp_partial(int64_t n_det, int NW, const int* __restrict__ sa,
                                                      const int* __restrict__ sb,
                                                      const cd* __restrict__ c,
                                                      const cd* __restrict__ da, int Ua,
                                                      const cd* __restrict__ db, int Ub,
                                                      cd* __restrict__ partial, int n_chunks,
                                                      int chunk) {
  __shared__ cd red[256];
  const int w = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
  const int64_t I0 = (int64_t)ch * chunk;
  const int64_t I1 = min(n_det, I0 + chunk);
  double sr = 0, si = 0, cr = 0, ci = 0;  // Kahan sums
  for (int64_t I = I0 + tid; I < I1; I += blockDim.x) {
    cd t = c[I] * da[(size_t)w * Ua + sa[I]] * db[(size_t)w * Ub + sb[I]];
    double y = t.re - cr, z = sr + y;
    cr = (z - sr) - y;
    sr = z;
    y = t.im - ci;
    z = si + y;
    ci = (z - si) - y;
    si = z;
  }
  cd r = block_reduce(cd{sr, si}, red);
  if (tid == 0) partial[(size_t)w * n_chunks + ch] = r;
}

__global__ void k_ovlp_final(int NW, const cd* __restrict__ partial, int n_chunks,
                             const cd* __restrict__ ldA, const cd* __restrict__ ldB,
                             cd* __restrict__ obar, cd* __restrict__ log_ovlp, int* __restrict__ flag) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= NW) return;
  cd o{0.0, 0.0};
  for (int c = 0; c < n_chunks; ++c) o += partial[(size_t)w * n_chunks + c];
  obar[w] = o;
  const double a2 = abs2(o);
  cd la = ldA ? ldA[w] : cd{0.0, 0.0};
  cd lb = ldB ? ldB[w] : cd{0.0, 0.0};
  if (!(a2 > 0.0) || !(a2 < INFINITY)) {
    flag[w] = 1;
    log_ovlp[w] = cd{-INFINITY, 0.0};
    return;
  }
  log_ovlp[w] = cd{0.5 * log(a2) + la.re + lb.re, atan2(o.im, o.re) + la.im + lb.im};
}

void launch_ovlp_partial(int64_t n_det, int NW, const int* sa, const int* sb, const cd* c,
                         const cd* da, int Ua, const cd* db, int Ub, cd* partial, int n_chunks,
                         int chunk, hipStream_t st) {
  hipLaunchKernelGGL(k_ovlp_partial, dim3(n_chunks, NW), dim3(256), 0, st, n_det, NW, sa, sb,
                     c, da, Ua, db, Ub, partial, n_chunks, chunk);
}

void launch_ovlp_final(int NW, const cd* partial, int n_chunks, const cd* ldA, const cd* ldB,
                       cd* obar, cd* log_ovlp, int* flag, hipStream_t st) {
  hipLaunchKernelGGL(k_ovlp_final, dim3((NW + 127) / 128), dim3(128), 0, st, NW, partial,
                     n_chunks, ldA, ldB, obar, log_ovlp, flag);
}

// ============================================================================
// A4: CI weights per string and the first-order CI matrix (gather form of the
// paper's reduce_CI: each output entry sums its own contribution list)
// ============================================================================

// Segment sums of c~_I det X^{other}_I over each string's determinant list
// (segments of <= 16), then per-string sums of its segments in order.
// blockIdx.y selects the spin; the other spin's dets are read.
__global__ void k_ci_segments(DevSpin sa, DevSpin sb, const cd* __restrict__ det_c,
                              const cd* __restrict__ da, const cd* __restrict__ db, int NW,
                              cd* __restrict__ pa, cd* __restrict__ pb) {
  const bool beta = blockIdx.y == 1;
  const DevSpin& s = beta ? sb : sa;
  const DevSpin& o = beta ? sa : sb;
  const cd* __restrict__ d_other = beta ? da : db;
  cd* __restrict__ seg_part = beta ? pb : pa;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)s.n_seg * NW) return;
  const int seg = (int)(tid % s.n_seg), w = (int)(tid / s.n_seg);
  cd acc{0.0, 0.0};
  const cd* __restrict__ dw = d_other + (size_t)w * o.U;
  const int e1 = s.seg_ptr[seg + 1];
  int e = s.seg_ptr[seg];
  // groups of four: the index loads, then the value gathers, are issued
  // together; the products are added in list order as before
  for (; e + 4 <= e1; e += 4) {
    int I[4], js[4];
    cd c[4], d[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) I[k] = s.bw_det[e + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) js[k] = o.det_s[I[k]];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = det_c[I[k]];
      d[k] = dw[js[k]];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) cfma(acc, c[k], d[k]);
  }
  for (; e < e1; ++e) {
    const int I = s.bw_det[e];
    cfma(acc, det_c[I], dw[o.det_s[I]]);
  }
  seg_part[(size_t)w * s.n_seg + seg] = acc;
}

__global__ void k_ci_weights(DevSpin sa, DevSpin sb, int NW, const cd* __restrict__ pa,
                             const cd* __restrict__ pb, cd* __restrict__ Ba,
                             cd* __restrict__ Bb) {
  const bool beta = blockIdx.y == 1;
  const DevSpin& s = beta ? sb : sa;
  const cd* __restrict__ seg_part = beta ? pb : pa;
  cd* __restrict__ B = beta ? Bb : Ba;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)s.U * NW) return;
  const int str = (int)(tid % s.U), w = (int)(tid / s.U);
  cd acc{0.0, 0.0};
  for (int q = s.str_seg[str]; q < s.str_seg[str + 1]; ++q) acc += seg_part[(size_t)w * s.n_seg + q];
  B[(size_t)w * s.U + str] = acc;
}

void launch_ci_weights(const DevSpin& sa, const DevSpin& sb, const cd* det_c, const SpinWork& wa,
                       const SpinWork& wb, cd* seg_a, cd* seg_b, int NW, hipStream_t st) {
  int64_t n = (int64_t)max(sa.n_seg, sb.n_seg) * NW;
  hipLaunchKernelGGL(k_ci_segments, dim3((unsigned)((n + 255) / 256), 2), dim3(256), 0, st, sa, sb,
                     det_c, wa.d, wb.d, NW, seg_a, seg_b);
  n = (int64_t)max(sa.U, sb.U) * NW;
  hipLaunchKernelGGL(k_ci_weights, dim3((unsigned)((n + 255) / 256), 2), dim3(256), 0, st, sa, sb,
                     NW, seg_a, seg_b, wa.B, wb.B);
}

__global__ void k_ci_matrix(DevSpin sa, DevSpin sb, int NW, const cd* __restrict__ adja,
                            const cd* __restrict__ adjb, const cd* __restrict__ Ba,
                            const cd* __restrict__ Bb, cd* __restrict__ Ca, cd* __restrict__ Cb) {
  const bool beta = blockIdx.y == 1;
  const DevSpin& s = beta ? sb : sa;
  const cd* __restrict__ adj = beta ? adjb : adja;
  const cd* __restrict__ B = beta ? Bb : Ba;
  cd* __restrict__ C = beta ? Cb : Ca;
  const int X = s.nv * s.no;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)X * NW) return;
  const int e = (int)(tid % X), w = (int)(tid / X);
  cd acc{0.0, 0.0};
  const cd* __restrict__ aw = adj + (size_t)w * s.A;
  const cd* __restrict__ bw = B + (size_t)w * s.U;
  const int q1 = s.c_ptr[e + 1];
  int q = s.c_ptr[e];
  // groups of four loads in flight; products added in list order as before
  for (; q + 4 <= q1; q += 4) {
    int ia[4], ib[4];
    cd a[4], b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      ia[k] = s.c_adj[q + k];
      ib[k] = s.c_str[q + k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      a[k] = aw[ia[k]];
      b[k] = bw[ib[k]];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) cfma(acc, a[k], b[k]);
  }
  for (; q < q1; ++q) cfma(acc, aw[s.c_adj[q]], bw[s.c_str[q]]);
  C[(size_t)w * X + e] = acc;
}

void launch_ci_matrix(const DevSpin& sa, const DevSpin& sb, int NW, const SpinWork& wa,
                      const SpinWork& wb, hipStream_t st) {
  const int64_t n = (int64_t)max(sa.nv * sa.no, sb.nv * sb.no) * NW;
  if (n == 0) return;
  hipLaunchKernelGGL(k_ci_matrix, dim3((unsigned)((n + 255) / 256), 2), dim3(256), 0, st, sa, sb,
                     NW, wa.adj, wb.adj, wa.B, wb.B, wa.C, wb.C);
}

// ============================================================================
// A5: Green's function rows R u V_act and one-body energy
// ============================================================================

// One workgroup per (walker, spin, tile of G_QT orbitals q): the tile's rows
// of T (T[q][w][:], contiguous per q) are staged in LDS once, then
//   D[a][q]    = sum_i C[a][i] T[q][slot(i)]                 (n_v x G_QT)
//   G[r][q]    = T[q][r] - sum_a T_V[a][r] D[a][q] / Obar    (reference rows r < N)
//   G[N+a][q]  = D[a][q] / Obar                               (window virtual rows)
// and the tile's part of the one-body energy sum_{r,q} h1[row r][q] G[r][q]
// goes to ob_part[spin][w][tile] (summed by k_green_ob).
constexpr int G_QT = 16;

struct GreenIO {
  const cd* T;
  const cd* C;
  cd* G;
  cd* ob_part;
};

__global__ __launch_bounds__(256) void k_green(DevSpin sa, DevSpin sb, GreenIO ia, GreenIO ib,
                                               int M, int NW, int n_qt,
                                               const cd* __restrict__ obar,
                                               const double* __restrict__ h1) {
  const bool beta = blockIdx.y == 1;
  const DevSpin& s = beta ? sb : sa;
  const GreenIO& io = beta ? ib : ia;
  const cd* __restrict__ T = io.T;
  const cd* __restrict__ C = io.C;
  cd* __restrict__ G = io.G;
  extern __shared__ cd sm[];
  __shared__ cd red[256];
  const int nv = s.nv, no = s.no, N = s.N, P = s.P;
  const int w = blockIdx.x, qt = blockIdx.z, tid = threadIdx.x, bd = blockDim.x;
  const int q0 = qt * G_QT, nq = min(G_QT, M - q0);
  cd* Cs = sm;                 // [nv][no]
  cd* TV = Cs + nv * no;       // [nv][N]
  cd* Tq = TV + nv * N;        // [G_QT][N]: rows q0 .. q0 + nq of T
  cd* D = Tq + G_QT * N;       // [nv][G_QT]
  const cd inv_o = cdiv(cd{1.0, 0.0}, obar[w]);
  for (int e = tid; e < nv * no; e += bd) Cs[e] = C[(size_t)w * nv * no + e];
  for (int e = tid; e < nv * N; e += bd) {
    const int a = e / N, j = e % N;
    TV[e] = T[((size_t)s.vir[a] * NW + w) * N + j];
  }
  for (int e = tid; e < nq * N; e += bd) {
    const int ql = e / N, j = e % N;
    Tq[e] = T[((size_t)(q0 + ql) * NW + w) * N + j];
  }
  __syncthreads();
  for (int e = tid; e < nv * G_QT; e += bd) {
    const int a = e / G_QT, ql = e % G_QT;
    cd acc{0.0, 0.0};
    if (ql < nq)
      for (int i = 0; i < no; ++i) cfma(acc, Cs[a * no + i], Tq[ql * N + s.oslot[i]]);
    D[e] = acc;
  }
  __syncthreads();
  cd ob{0.0, 0.0};
  for (int e = tid; e < P * G_QT; e += bd) {
    const int r = e / G_QT, ql = e % G_QT, q = q0 + ql;
    if (ql >= nq) continue;
    cd g;
    if (r < N) {
      cd acc{0.0, 0.0};
      for (int a = 0; a < nv; ++a) cfma(acc, TV[a * N + r], D[a * G_QT + ql]);
      g = Tq[ql * N + r] - inv_o * acc;
    } else {
      g = inv_o * D[(r - N) * G_QT + ql];
    }
    G[((size_t)w * P + r) * M + q] = g;
    ob += h1[(size_t)s.rows[r] * M + q] * g;
  }
  const cd tot = block_reduce(ob, red);
  if (tid == 0) io.ob_part[(size_t)w * n_qt + qt] = tot;
}

// onebody[w] = sum over the orbital tiles of ob_part[w][tile] (both spins)
__global__ void k_green_ob(int n, int n_qt, const cd* __restrict__ ob_part,
                           cd* __restrict__ onebody) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cd t{0.0, 0.0};
  for (int z = 0; z < n_qt; ++z) t += ob_part[(size_t)i * n_qt + z];
  onebody[i] = t;
}

int green_tiles(int M) { return (M + G_QT - 1) / G_QT; }

void launch_green(const DevSpin& sa, const DevSpin& sb, int M, int NW, const SpinWork& wa,
                  const SpinWork& wb, cd* onebody, const cd* obar, const double* h1,
                  cd* ob_part, hipStream_t st) {
  size_t lds = 0;
  for (const DevSpin* s : {&sa, &sb})
    lds = max(lds, ((size_t)s->nv * s->no + (size_t)s->nv * s->N + (size_t)G_QT * s->N +
                    (size_t)s->nv * G_QT) * sizeof(cd));
  const int n_qt = green_tiles(M);
  const GreenIO ia{wa.T, wa.C, wa.G, ob_part}, ib{wb.T, wb.C, wb.G, ob_part + (size_t)NW * n_qt};
  hipLaunchKernelGGL(k_green, dim3(NW, 2, n_qt), dim3(256), lds, st, sa, sb, ia, ib, M, NW, n_qt,
                     obar, h1);
  hipLaunchKernelGGL(k_green_ob, dim3((2 * NW + 255) / 256), dim3(256), 0, st, 2 * NW, n_qt,
                     ob_part, onebody);
}

__global__ void k_green_sum(int M, int NW, int P_all, const int* __restrict__ rmap_a,
                            const int* __restrict__ rmap_b, int Pa, int Pb,
                            const cd* __restrict__ Ga, const cd* __restrict__ Gb,
                            double* __restrict__ Gp) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)P_all * M;
  if (tid >= per * NW) return;
  const int w = (int)(tid / per);
  const int64_t e = tid % per;
  const int r = (int)(e / M), q = (int)(e % M);
  cd g{0.0, 0.0};
  if (rmap_a[r] >= 0) g += Ga[((size_t)w * Pa + rmap_a[r]) * M + q];
  if (rmap_b[r] >= 0) g += Gb[((size_t)w * Pb + rmap_b[r]) * M + q];
  Gp[((size_t)w * 2) * per + e] = g.re;
  Gp[((size_t)w * 2 + 1) * per + e] = g.im;
}

void launch_green_sum(int M, int NW, int P_all, const int* rmap_a, const int* rmap_b, int Pa,
                      int Pb, const cd* Ga, const cd* Gb, double* Gp, hipStream_t st) {
  const int64_t n = (int64_t)P_all * M * NW;
  hipLaunchKernelGGL(k_green_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M, NW,
                     P_all, rmap_a, rmap_b, Pa, Pb, Ga, Gb, Gp);
}

// xbar[w][g] = -i sqrt(dt) vbar, vbar = raw[g][2w] + i raw[g][2w+1]
__global__ void k_xbar(int NW, int NG, const double* __restrict__ raw, double sqrt_dt,
                       cd* __restrict__ xbar) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)NW * NG) return;
  const int w = (int)(tid / NG), g = (int)(tid % NG);
  const double vr = raw[(size_t)g * 2 * NW + 2 * w], vi = raw[(size_t)g * 2 * NW + 2 * w + 1];
  xbar[tid] = cd{sqrt_dt * vi, -sqrt_dt * vr};
}

void launch_xbar(int NW, int NG, const double* raw, double sqrt_dt, cd* xbar, hipStream_t st) {
  const int64_t n = (int64_t)NW * NG;
  hipLaunchKernelGGL(k_xbar, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, NW, NG, raw,
                     sqrt_dt, xbar);
}

// ============================================================================
// A6: energy intermediates per (walker, Cholesky chunk): v0, ex0, Lam (window),
// and the chunk's share of ZW = sum_g Xi^g - (v0a + v0b) Lam^g.
// LT^s layout: row g*P + p, column wl*N + c (complex), row length WT*N.
// One wave per workgroup: barriers are cheap and reductions use shuffles.
// ============================================================================

__device__ __forceinline__ cf wave_sum(cf v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  return v;
}

__device__ __forceinline__ cd wave_sum(cd v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  return v;
}

// Sum of one value over the workgroup (LAM_WAVES waves), in every thread;
// red: LAM_WAVES entries of LDS.  Two barriers: red is free again on return.
constexpr int LAM_WAVES = 4;
template <class CT>
__device__ __forceinline__ CT lam_block_sum(CT v, CT* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  CT t{};
#pragma unroll
  for (int q = 0; q < LAM_WAVES; ++q) t += red[q];
  __syncthreads();
  return t;
}

// Generic form (any N, windows beyond the rows kernel): one workgroup of
// LAM_WAVES waves per (walker, vector chunk).  The waves share the LDS copies
// of T[V, :], each vector's Q and the Lambda rows, so the LDS per workgroup
// (the N x N Q tile dominates) carries four waves instead of one.
template <class CT>
__global__ __launch_bounds__(64 * LAM_WAVES) void k_lambda(DevSpin sa, DevSpin sb, int NW, int w0, int WT,
                                               int NG, int g_chunk, const CT* __restrict__ Ta,
                                               const CT* __restrict__ Tb,
                                               const CT* __restrict__ LTa,
                                               const CT* __restrict__ LTb,
                                               CT* __restrict__ Lam_a, CT* __restrict__ Lam_b,
                                               cd* __restrict__ v0, cd* __restrict__ ex0,
                                               cd* __restrict__ ZWa, cd* __restrict__ ZWb) {
  // LDS: ZW accumulators (double) first, then T[V,:] of both spins, Q and the
  // Lambda rows in the working precision
  extern __shared__ __align__(16) unsigned char sm_raw[];
  __shared__ CT red[LAM_WAVES];
  constexpr int NT = 64 * LAM_WAVES;
  const int wl = blockIdx.x, chunk = blockIdx.y, n_chunks = gridDim.y;
  const int w = w0 + wl, tid = threadIdx.x;
  cd* ZWs[2];
  ZWs[0] = reinterpret_cast<cd*>(sm_raw);         // [nv_a*no_a] accumulators
  ZWs[1] = ZWs[0] + sa.nv * sa.no;                // [nv_b*no_b]
  CT* TVa = reinterpret_cast<CT*>(ZWs[1] + sb.nv * sb.no);  // [nv_a*N_a]
  CT* TVb = TVa + sa.nv * sa.N;                   // [nv_b*N_b]
  CT* Q = TVb + sb.nv * sb.N;                     // [max N^2]
  CT* Lf = Q + max(sa.N * sa.N, sb.N * sb.N);     // [max nv*N]
  for (int e = tid; e < sa.nv * sa.no; e += NT) ZWs[0][e] = cd{0.0, 0.0};
  for (int e = tid; e < sb.nv * sb.no; e += NT) ZWs[1][e] = cd{0.0, 0.0};
  for (int e = tid; e < sa.nv * sa.N; e += NT) {
    const int a = e / sa.N, j = e % sa.N;
    TVa[e] = Ta[((size_t)sa.vir[a] * NW + w) * sa.N + j];
  }
  for (int e = tid; e < sb.nv * sb.N; e += NT) {
    const int a = e / sb.N, j = e % sb.N;
    TVb[e] = Tb[((size_t)sb.vir[a] * NW + w) * sb.N + j];
  }
  __syncthreads();

  const int g0 = chunk * g_chunk, g1 = min(NG, g0 + g_chunk);
  for (int g = g0; g < g1; ++g) {
    // traces of both spins first: ZW needs v0a + v0b
    CT va{}, vb{};
    for (int j = tid; j < sa.N; j += NT) va += LTa[(((size_t)wl * NG + g) * sa.P + j) * sa.N + j];
    for (int j = tid; j < sb.N; j += NT) vb += LTb[(((size_t)wl * NG + g) * sb.P + j) * sb.N + j];
    va = lam_block_sum(va, red);
    vb = lam_block_sum(vb, red);
    const CT vsum = va + vb;
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const DevSpin& S = s2 ? sb : sa;
      const CT* TV = s2 ? TVb : TVa;
      const int N = S.N, nv = S.nv, no = S.no, X = nv * no;
      if (N == 0) {  // spin without electrons: zero traces
        if (tid == 0) {
          v0[((size_t)s2 * NW + w) * NG + g] = cd{0.0, 0.0};
          ex0[((size_t)s2 * NW + w) * NG + g] = cd{0.0, 0.0};
        }
        continue;
      }
      const CT* base = (s2 ? LTb : LTa) + ((size_t)wl * NG + g) * S.P * N;
      const size_t ld = (size_t)N;
      CT x{};
      for (int e = tid; e < N * N; e += NT) {
        const int j = e / N, c = e % N;
        Q[e] = base[(size_t)j * ld + c];
      }
      __syncthreads();
      for (int e = tid; e < N * N; e += NT) {
        const int j = e / N, c = e % N;
        cfma(x, Q[e], Q[c * N + j]);
      }
      x = lam_block_sum(x, red);
      if (tid == 0) {
        v0[((size_t)s2 * NW + w) * NG + g] = to_cd(s2 ? vb : va);
        ex0[((size_t)s2 * NW + w) * NG + g] = to_cd(x);
      }
      for (int e = tid; e < nv * N; e += NT) {
        const int a = e / N, c = e % N;
        CT acc = -base[(size_t)(N + a) * ld + c];
        for (int j = 0; j < N; ++j) cfma(acc, TV[a * N + j], Q[j * N + c]);
        Lf[e] = acc;
      }
      __syncthreads();
      CT* Lo = (s2 ? Lam_b : Lam_a) + ((size_t)wl * NG + g) * X;
      cd* Z = ZWs[s2];
      for (int e = tid; e < X; e += NT) {
        const int a = e / no, i = e % no, oc = S.oslot[i];
        CT xi{};
        for (int c = 0; c < N; ++c) cfma(xi, Lf[a * N + c], Q[c * N + oc]);
        const CT lam = Lf[a * N + oc];
        Lo[e] = lam;
        Z[e] += to_cd(xi - vsum * lam);
      }
      __syncthreads();
    }
  }
  for (int s2 = 0; s2 < 2; ++s2) {
    const int X = (s2 ? sb : sa).nv * (s2 ? sb : sa).no;
    cd* ZW = s2 ? ZWb : ZWa;
    for (int e = tid; e < X; e += NT) ZW[((size_t)wl * n_chunks + chunk) * X + e] = ZWs[s2][e];
  }
}

// Row-per-lane form of the same computation: one wave per (walker, spin) in a
// workgroup of two waves, lane = virtual-orbital row a (n_vir_act <= 64).  Each
// lane keeps T[v_a, :], its Lam row, its Xi row and its ZW row in registers;
// Q^g is broadcast from LDS.  NMAX bounds N, NOMAX bounds n_occ_act.
constexpr int NOMAX = 16;

template <int NMAX, class CT>
__global__ __launch_bounds__(128) void k_lambda_rows(DevSpin sa, DevSpin sb, int NW, int w0,
                                                     int WT, int NG, int g_chunk,
                                                     const CT* __restrict__ Ta,
                                                     const CT* __restrict__ Tb,
                                                     const CT* __restrict__ LTa,
                                                     const CT* __restrict__ LTb,
                                                     CT* __restrict__ Lam_a,
                                                     CT* __restrict__ Lam_b,
                                                     cd* __restrict__ v0, cd* __restrict__ ex0,
                                                     cd* __restrict__ ZWa, cd* __restrict__ ZWb) {
  __shared__ CT Qs[2][NMAX * NMAX];
  __shared__ CT v0s[2];
  const int wl = blockIdx.x, chunk = blockIdx.y, n_chunks = gridDim.y;
  const int w = w0 + wl, lane = threadIdx.x & 63, s2 = threadIdx.x >> 6;
  const int N = s2 ? sb.N : sa.N, nv = s2 ? sb.nv : sa.nv, no = s2 ? sb.no : sa.no;
  const int P = s2 ? sb.P : sa.P, X = nv * no;
  const int* __restrict__ vir = s2 ? sb.vir : sa.vir;
  const int* __restrict__ oslot = s2 ? sb.oslot : sa.oslot;
  const CT* __restrict__ T = s2 ? Tb : Ta;
  const CT* __restrict__ LT = s2 ? LTb : LTa;
  CT* __restrict__ Lam = s2 ? Lam_b : Lam_a;
  cd* __restrict__ ZW = s2 ? ZWb : ZWa;
  const bool row = lane < nv;
  CT tv[NMAX];
  cd zw[NOMAX];
  int osl[NOMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j)
    tv[j] = (row && j < N) ? T[((size_t)vir[lane] * NW + w) * N + j] : CT{};
#pragma unroll
  for (int i = 0; i < NOMAX; ++i) {
    osl[i] = i < no ? oslot[i] : 0;
    zw[i] = cd{0.0, 0.0};
  }
  const size_t ld = (size_t)N;  // LT tile of (walker, vector): P x N, contiguous
  const int g0 = chunk * g_chunk, g1 = min(NG, g0 + g_chunk);
  for (int g = g0; g < g1; ++g) {
    const CT* base = LT + ((size_t)wl * NG + g) * P * N;
    // Q^g of this spin into LDS; traces
    CT v{}, x{};
    for (int e = lane; e < N * N; e += 64) {
      const int j = e / N, c = e % N;
      const CT q = base[(size_t)j * ld + c];
      Qs[s2][e] = q;
      if (j == c) v += q;
    }
    // this lane's LT^g[V, :] row (independent of the LDS writes above)
    CT ltv[NMAX];
#pragma unroll
    for (int c = 0; c < NMAX; ++c)
      ltv[c] = (row && c < N) ? base[(size_t)(N + lane) * ld + c] : CT{};
    v = wave_sum(v);
    if (lane == 0) v0s[s2] = v;
    __syncthreads();
    const CT* Q = Qs[s2];
    for (int e = lane; e < N * N; e += 64) {
      const int j = e / N, c = e % N;
      cfma(x, Q[e], Q[c * N + j]);
    }
    x = wave_sum(x);
    if (lane == 0 && N > 0) {
      v0[((size_t)s2 * NW + w) * NG + g] = to_cd(v);
      ex0[((size_t)s2 * NW + w) * NG + g] = to_cd(x);
    } else if (lane == 0) {
      v0[((size_t)s2 * NW + w) * NG + g] = cd{0.0, 0.0};
      ex0[((size_t)s2 * NW + w) * NG + g] = cd{0.0, 0.0};
    }
    const CT vsum = v0s[0] + v0s[1];
    if (row) {
      CT lam[NMAX];
#pragma unroll
      for (int c = 0; c < NMAX; ++c) {
        CT a = -ltv[c];
#pragma unroll
        for (int j = 0; j < NMAX; ++j)
          if (j < N && c < N) cfma(a, tv[j], Q[j * N + c]);
        lam[c] = a;
      }
      CT* Lo = Lam + ((size_t)wl * NG + g) * X + (size_t)lane * no;
#pragma unroll
      for (int i = 0; i < NOMAX; ++i) {
        if (i < no) {
          const int oc = osl[i];
          CT xi{}, lw{};
#pragma unroll
          for (int c = 0; c < NMAX; ++c) {
            if (c < N) cfma(xi, lam[c], Q[c * N + oc]);
            if (c == oc) lw = lam[c];
          }
          Lo[i] = lw;
          zw[i] += to_cd(xi - vsum * lw);
        }
      }
    }
    __syncthreads();
  }
  if (row) {
#pragma unroll
    for (int i = 0; i < NOMAX; ++i)
      if (i < no) ZW[((size_t)wl * n_chunks + chunk) * X + (size_t)lane * no + i] = zw[i];
  }
}

bool lambda_rows_fits(const DevSpin& sa, const DevSpin& sb, int* nmax) {
  const int n = max(sa.N, sb.N);
  if (sa.nv > 64 || sb.nv > 64 || sa.no > NOMAX || sb.no > NOMAX || n > 32) return false;
  *nmax = n <= 8 ? 8 : (n <= 16 ? 16 : 32);
  return true;
}

template <class CT>
void launch_lambda_rows_t(const DevSpin& sa, const DevSpin& sb, int nmax, int NW, int w0, int WT,
                          int NG, int g_chunk, const CT* Ta, const CT* Tb, const CT* LTa,
                          const CT* LTb, CT* Lam_a, CT* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a,
                          cd* ZWpart_b, hipStream_t st) {
  const int n_chunks = (NG + g_chunk - 1) / g_chunk;
  dim3 grid(WT, n_chunks);
  switch (nmax) {
    case 8: hipLaunchKernelGGL((k_lambda_rows<8, CT>), grid, dim3(128), 0, st, sa, sb, NW, w0, WT, NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0, ZWpart_a, ZWpart_b); break;
    case 16: hipLaunchKernelGGL((k_lambda_rows<16, CT>), grid, dim3(128), 0, st, sa, sb, NW, w0, WT, NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0, ZWpart_a, ZWpart_b); break;
    default: hipLaunchKernelGGL((k_lambda_rows<32, CT>), grid, dim3(128), 0, st, sa, sb, NW, w0, WT, NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0, ZWpart_a, ZWpart_b); break;
  }
}

void launch_lambda_rows(const DevSpin& sa, const DevSpin& sb, int nmax, int NW, int w0, int WT,
                        int NG, int g_chunk, const cd* Ta, const cd* Tb, const cd* LTa,
                        const cd* LTb, cd* Lam_a, cd* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a,
                        cd* ZWpart_b, hipStream_t st) {
  launch_lambda_rows_t<cd>(sa, sb, nmax, NW, w0, WT, NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b,
                           v0, ex0, ZWpart_a, ZWpart_b, st);
}

void launch_lambda_rows32(const DevSpin& sa, const DevSpin& sb, int nmax, int NW, int w0, int WT,
                          int NG, int g_chunk, const cf* Ta, const cf* Tb, const cf* LTa,
                          const cf* LTb, cf* Lam_a, cf* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a,
                          cd* ZWpart_b, hipStream_t st) {
  launch_lambda_rows_t<cf>(sa, sb, nmax, NW, w0, WT, NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b,
                           v0, ex0, ZWpart_a, ZWpart_b, st);
}

template <class CT>
static void launch_lambda_t(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                            int g_chunk, const CT* Ta, const CT* Tb, const CT* LTa,
                            const CT* LTb, CT* Lam_a, CT* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a,
                            cd* ZWpart_b, hipStream_t st) {
  const int n_chunks = (NG + g_chunk - 1) / g_chunk;
  const size_t words = (size_t)sa.nv * sa.N + (size_t)sb.nv * sb.N +
                       (size_t)max(sa.N * sa.N, sb.N * sb.N) +
                       (size_t)max(sa.nv * sa.N, sb.nv * sb.N);
  const size_t bytes = ((size_t)sa.nv * sa.no + (size_t)sb.nv * sb.no) * sizeof(cd) +
                       words * sizeof(CT);
  hipLaunchKernelGGL((k_lambda<CT>), dim3(WT, n_chunks), dim3(64 * LAM_WAVES), bytes, st, sa, sb, NW, w0, WT,
                     NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0, ZWpart_a, ZWpart_b);
}

void launch_lambda(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                   int g_chunk, const cd* Ta, const cd* Tb, const cd* LTa, const cd* LTb,
                   cd* Lam_a, cd* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a, cd* ZWpart_b,
                   hipStream_t st) {
  launch_lambda_t<cd>(sa, sb, NW, w0, WT, NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0,
                      ZWpart_a, ZWpart_b, st);
}

void launch_lambda32(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                     int g_chunk, const cf* Ta, const cf* Tb, const cf* LTa, const cf* LTb,
                     cf* Lam_a, cf* Lam_b, cd* v0, cd* ex0, cd* ZWpart_a, cd* ZWpart_b,
                     hipStream_t st) {
  launch_lambda_t<cf>(sa, sb, NW, w0, WT, NG, g_chunk, Ta, Tb, LTa, LTb, Lam_a, Lam_b, v0, ex0,
                      ZWpart_a, ZWpart_b, st);
}

// ============================================================================
// A7: two-body CI coefficients per walker
// ============================================================================

// coef[w][t] = sum over the entries e of pair t of c_det(e) adj_a[w][fa(e)]
// adj_b[w][fb(e)].  One thread per (pair, block of PC_W walkers): the entry's
// indices and CI coefficient are loaded once for the block, and each walker
// sums its entries in the same order as a thread per (pair, walker) would.
constexpr int PC_W = 8;

__global__ void k_pair_coef(DevPairs pr, int NW, const cd* __restrict__ det_c,
                            const cd* __restrict__ adj_a, int Aa, const cd* __restrict__ adj_b,
                            int Ab, cd* __restrict__ coef) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n_wb = (NW + PC_W - 1) / PC_W;
  if (tid >= (int64_t)pr.n_pair * n_wb) return;
  const int t = (int)(tid % pr.n_pair), w0 = (int)(tid / pr.n_pair) * PC_W;
  cd acc[PC_W];
  const cd* aa[PC_W];
  const cd* ab[PC_W];
#pragma unroll
  for (int j = 0; j < PC_W; ++j) {
    const int w = min(w0 + j, NW - 1);  // past the last walker: repeats it, not stored
    acc[j] = cd{0.0, 0.0};
    aa[j] = adj_a + (size_t)w * Aa;
    ab[j] = adj_b + (size_t)w * Ab;
  }
  for (int64_t e = pr.ptr[t]; e < pr.ptr[t + 1]; ++e) {
    const cd c = det_c[pr.det[e]];
    const int fa = pr.fa[e], fb = pr.fb[e];
#pragma unroll
    for (int j = 0; j < PC_W; ++j) cfma(acc[j], c * aa[j][fa], ab[j][fb]);
  }
#pragma unroll
  for (int j = 0; j < PC_W; ++j)
    if (w0 + j < NW) coef[(size_t)(w0 + j) * pr.n_pair + t] = acc[j];
}

// Walker-fastest copy of one spin's adjugates, adjT[f][w] = adj[w][f], in
// 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void k_adj_transpose(const cd* __restrict__ adj, int A, int NW,
                                                       cd* __restrict__ adjT) {
  __shared__ cd tile[32][33];
  const int f0 = blockIdx.x * 32, w0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int w = w0 + r, f = f0 + tx;
    if (w < NW && f < A) tile[r][tx] = adj[(size_t)w * A + f];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int f = f0 + r, w = w0 + tx;
    if (f < A && w < NW) adjT[(size_t)f * NW + w] = tile[tx][r];
  }
}

// The same sums with the walkers on the lanes: one wave per (pair, 64
// walkers), so the pair's entries (indices and CI coefficient) are
// wave-uniform and each adjugate read of a wave is one contiguous run of 64
// walkers' values in the walker-fastest copies.  Each walker sums its entries
// in the same order as above.
__global__ __launch_bounds__(256) void k_pair_coef_wl(DevPairs pr, int NW,
                                                      const cd* __restrict__ det_c,
                                                      const cd* __restrict__ adjT_a,
                                                      const cd* __restrict__ adjT_b,
                                                      cd* __restrict__ coef) {
  const int t = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (t >= pr.n_pair) return;  // wave-uniform; no barriers
  const int w = blockIdx.y * 64 + (threadIdx.x & 63);
  const int wc = min(w, NW - 1);  // past the last walker: repeats it, not stored
  cd acc{0.0, 0.0};
  const int64_t e1 = pr.ptr[t + 1];
#pragma unroll 4
  for (int64_t e = pr.ptr[t]; e < e1; ++e) {
    const cd c = det_c[pr.det[e]];
    cfma(acc, c * adjT_a[(size_t)pr.fa[e] * NW + wc], adjT_b[(size_t)pr.fb[e] * NW + wc]);
  }
  if (w < NW) coef[(size_t)w * pr.n_pair + t] = acc;
}

void launch_pair_coef(const DevPairs& pr, int NW, const cd* det_c, const cd* adj_a, int Aa,
                      const cd* adj_b, int Ab, cd* coef, hipStream_t st, cd* adjT_a,
                      cd* adjT_b) {
  if ((int64_t)pr.n_pair * NW == 0) return;
  if (adjT_a && adjT_b) {
    const dim3 ga((Aa + 31) / 32, (NW + 31) / 32), gb((Ab + 31) / 32, (NW + 31) / 32);
    hipLaunchKernelGGL(k_adj_transpose, ga, dim3(256), 0, st, adj_a, Aa, NW, adjT_a);
    hipLaunchKernelGGL(k_adj_transpose, gb, dim3(256), 0, st, adj_b, Ab, NW, adjT_b);
    hipLaunchKernelGGL(k_pair_coef_wl, dim3((pr.n_pair + 3) / 4, (NW + 63) / 64), dim3(256), 0,
                       st, pr, NW, det_c, adjT_a, adjT_b, coef);
    return;
  }
  const int64_t n = (int64_t)pr.n_pair * ((NW + PC_W - 1) / PC_W);
  hipLaunchKernelGGL(k_pair_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, pr, NW,
                     det_c, adj_a, Aa, adj_b, Ab, coef);
}

__global__ void k_minor_coef(DevSpin s, int NW, const cd* __restrict__ B, int U,
                             const cd* __restrict__ m2, cd* __restrict__ coef) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)s.n_minor * NW) return;
  const int t = (int)(tid % s.n_minor), w = (int)(tid / s.n_minor);
  cd acc{0.0, 0.0};
  for (int e = s.mn_ptr[t]; e < s.mn_ptr[t + 1]; ++e) {
    cd v = B[(size_t)w * U + s.mn_str[e]] * m2[(size_t)w * s.M2 + s.mn_m2[e]];
    if (s.mn_sgn[e] < 0) acc -= v;
    else acc += v;
  }
  coef[(size_t)w * s.n_minor + t] = acc;
}

void launch_minor_coef(const DevSpin& s, int NW, const cd* B, int U, const cd* m2, cd* coef,
                       hipStream_t st) {
  const int64_t n = (int64_t)s.n_minor * NW;
  if (n == 0) return;
  hipLaunchKernelGGL(k_minor_coef, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, NW,
                     B, U, m2, coef);
}

// ============================================================================
// A7: the Cholesky-vector loop.  Second-order energy terms
//   sum_g [ sum_pairs coef Lam^a_g[x] Lam^b_g[y]
//         + sum_s sum_strings B_str e2(X_str, Y_str^g)     (same spin) ]
// Every kernel streams Lam_g through LDS for its share of the Cholesky
// vectors (double-buffered stages of G_STAGE vectors) and writes one partial
// per workgroup into its own slot of partial[w][slot]; the energy assembly
// sums the slots in order.
// ============================================================================

constexpr int G_STAGE = 2;

// Same-spin terms as a list of distinct minors (orders above 6, or on
// request): coef_t sum_g (Lam[a,i] Lam[b,j] - Lam[a,j] Lam[b,i]) per minor t,
// 8 minors per thread.
constexpr int MINOR_THREADS = 256;

__global__ __launch_bounds__(MINOR_THREADS) void k_energy_minors(
    DevSpin s, int NW, int w0, int NG, int n_gsplit, const cd* __restrict__ Lam,
    const cd* __restrict__ coef, cd* __restrict__ partial, int n_slots, int slot0) {
  extern __shared__ cd sm[];
  __shared__ cd red[MINOR_THREADS];
  const int wl = blockIdx.x, gs = blockIdx.y, mb = blockIdx.z;
  const int w = w0 + wl, tid = threadIdx.x;
  const int X = s.nv * s.no;
  const int gper = (NG + n_gsplit - 1) / n_gsplit;
  const int g0 = gs * gper, g1 = min(NG, g0 + gper);
  constexpr int MPT = 8;
  int id[MPT][4];
  cd acc[MPT];
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    const int t = mb * MINOR_THREADS * MPT + j * MINOR_THREADS + tid;
    const bool ok = t < s.n_minor;
    // padding minors read entry 0 and are dropped below
#pragma unroll
    for (int q = 0; q < 4; ++q) id[j][q] = ok ? s.mn_idx[4 * t + q] : 0;
    acc[j] = cd{0.0, 0.0};
  }
  // stage buffer b starts at sm[b * G_STAGE * X] (integer offsets keep LDS addressing)
  auto stage = [&](int gb, int b) {
    const int G = min(G_STAGE, g1 - gb);
    const cd* src = Lam + ((size_t)wl * NG + gb) * X;
    for (int e = tid; e < G * X; e += MINOR_THREADS) sm[b * G_STAGE * X + e] = src[e];
  };
  if (g0 < g1) stage(g0, 0);
  __syncthreads();
  int it = 0;
  for (int gb = g0; gb < g1; gb += G_STAGE, ++it) {
    if (gb + G_STAGE < g1) stage(gb + G_STAGE, (it + 1) & 1);
    const int G = min(G_STAGE, g1 - gb);
    for (int gl = 0; gl < G; ++gl) {
      const int o = ((it & 1) * G_STAGE + gl) * X;
#pragma unroll
      for (int j = 0; j < MPT; ++j) {
        cfma(acc[j], sm[o + id[j][0]], sm[o + id[j][1]]);
        acc[j] -= sm[o + id[j][2]] * sm[o + id[j][3]];
      }
    }
    __syncthreads();
  }
  cd tot{0.0, 0.0};
#pragma unroll
  for (int j = 0; j < MPT; ++j) {
    const int t = mb * MINOR_THREADS * MPT + j * MINOR_THREADS + tid;
    if (t < s.n_minor) cfma(tot, coef[(size_t)w * s.n_minor + t], acc[j]);
  }
  red[tid] = tot;
  __syncthreads();
  for (int off = MINOR_THREADS / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0)
    partial[(size_t)w * n_slots + slot0 + (size_t)mb * n_gsplit + gs] = red[0];
}

// Row-pair items: one (string of order K, row pair m < m') per lane.  It needs
// rows m and m' of Y_mn = Lam[p_n, h_m] (2K gathers per Cholesky vector) and
// the K(K-1)/2 signed complementary minors of that row pair:
//   e2 += sum_{n<n'} (-1)^{m+m'+n+n'} det X[~{m,m'},~{n,n'}] (Y_mn Y_m'n' - Y_mn' Y_m'n).
// idx[] holds window offsets (p_n * n_occ_act + slot(h_m)) within the spin's
// Lambda row.
template <int K, class CT>
__device__ __forceinline__ void rp_setup(const int* __restrict__ hwin, const int* __restrict__ pwin,
                                         int no, int str, int rp, const cd* m2s, int* idx,
                                         CT* mm) {
  constexpr int P = K * (K - 1) / 2;
  int m = 0, mp = 1;
  for (int a = 0, q = 0; a < K; ++a)
    for (int b = a + 1; b < K; ++b, ++q)
      if (q == rp) { m = a; mp = b; }
#pragma unroll
  for (int n = 0; n < K; ++n) {
    const int col = pwin[str * KMAX + n] * no;
    idx[n] = col + hwin[str * KMAX + m];
    idx[K + n] = col + hwin[str * KMAX + mp];
  }
  const cd* src = m2s + rp * P;
  int q = 0;
#pragma unroll
  for (int n = 0; n < K; ++n)
#pragma unroll
    for (int np = n + 1; np < K; ++np, ++q) {
      cd v = src[q];
      if ((m + mp + n + np) & 1) v = -v;
      mm[q] = from_cd<CT>(v);
    }
}

// Gathers rows m and m' of Y for one Cholesky vector: y[0..K) and y[K..2K).
// sm: the LDS stage (indexed with an integer offset, so with the LDS array
// itself the compiler emits LDS instructions).
template <int K, class CT>
__device__ __forceinline__ void rp_load(const CT* sm, int base, const int* idx, CT* y) {
#pragma unroll
  for (int n = 0; n < 2 * K; ++n) y[n] = sm[base + idx[n]];
}

template <int K, class CT>
__device__ __forceinline__ void rp_math(const CT* y, const CT* mm, CT& acc) {
  const CT* y0 = y;
  const CT* y1 = y + K;
  if constexpr (K >= 4 && sizeof(CT) == sizeof(cd)) {
    // sum over n < n' of mm (y0_n y1_n' - y0_n' y1_n) = sum_n y0_n z_n with
    // z = S y1, S antisymmetric (S_nn' = mm for n < n'): K^2 complex MACs
    // instead of 3 per two-by-two minor.  FP64 only: in FP32 the terms of a
    // minor are better cancelled before they are weighted.
#pragma unroll
    for (int n = 0; n < K; ++n) {
      CT z{};
#pragma unroll
      for (int np = 0; np < K; ++np) {
        if (np == n) continue;
        const int a = n < np ? n : np, b = n < np ? np : n;
        const int q = a * (2 * K - a - 1) / 2 + (b - a - 1);  // index of the pair (a, b)
        if (n < np) cfma(z, mm[q], y1[np]);
        else cfma(z, -mm[q], y1[np]);
      }
      cfma(acc, y0[n], z);
    }
  } else {
    int q = 0;
#pragma unroll
    for (int n = 0; n < K; ++n)
#pragma unroll
      for (int np = n + 1; np < K; ++np, ++q) {
        // d = y0_n y1_n' - y0_n' y1_n as one fused chain per component
        auto re = y0[n].re * y1[np].re;
        re = fma(-y0[n].im, y1[np].im, re);
        re = fma(-y0[np].re, y1[n].re, re);
        re = fma(y0[np].im, y1[n].im, re);
        auto im = y0[n].re * y1[np].im;
        im = fma(y0[n].im, y1[np].re, im);
        im = fma(-y0[np].re, y1[n].im, im);
        im = fma(-y0[np].im, y1[n].re, im);
        cfma(acc, mm[q], CT{re, im});
      }
  }
}

// Merged second-order kernel.  Workgroup = (walker, Cholesky range, item
// block); each wave takes one plan entry: 64 x ER_PPL opposite-spin pairs, or
// 64 row-pair items of one spin and order.  The Lambda rows of the range are
// staged through LDS in double-buffered stages of G vectors, laid out
// [alpha: G x Xa][beta: G x Xb] so each stage is two contiguous copies.
constexpr int ER_PPL = 4;  // opposite-spin pairs per lane

// Direct global-to-LDS load of 16 bytes per lane: lane i of the wave writes
// lds + 16 i (lds must be wave-uniform).  Device-only instruction; the host
// pass of this file sees an empty body.
__device__ __forceinline__ void lds_dma16(const void* g, void* lds) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_global_load_lds(g, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
#endif
}

// FLATG: gather through a generic (flat) pointer to the LDS stage instead of
// LDS instructions.  The two paths group a wave's random 16-byte reads
// differently; which is faster is measured (launch-shape tuning).
template <class CT, int MAXK, bool FLATG>
__global__ __launch_bounds__((MAXK <= 4 ? 1024 : 512)) void k_energy_second(
    DevSpin sa, DevSpin sb, DevPairs pr, const int4* __restrict__ plan, int n_ib,
    int waves_per_block, int NW, int w0, int NG, int n_gsplit, int G, const CT* __restrict__ Lam_a,
    const CT* __restrict__ Lam_b, const cd* __restrict__ coef, const cd* __restrict__ m2a,
    const cd* __restrict__ m2b, const cd* __restrict__ Ba, const cd* __restrict__ Bb,
    cd* __restrict__ partial, int n_slots, int slot0, bool lds_dma, int swz,
    const int* __restrict__ wmask, const int* __restrict__ wlist, const int* __restrict__ wcount,
    int WT) {
  constexpr int NIDX = 2 * MAXK > 2 * ER_PPL ? 2 * MAXK : 2 * ER_PPL;
  constexpr int NMM = MAXK * (MAXK - 1) / 2;
  extern __shared__ __align__(16) unsigned char sm_raw[];
  CT* sm = reinterpret_cast<CT*>(sm_raw);
  __shared__ cd red[16];
  // Work items (item block, Cholesky range, walker): one per workgroup (grid
  // mode), or, with a walker list, a persistent grid striding over the items
  // of the listed walkers
  // Persistent mode is XCD-aware as well: workgroup b runs on XCD b % 8 and
  // takes the items of that XCD's contiguous share of the item list, so the
  // item blocks of one walker stay on one XCD (and its L2).
  const int n_items = wlist ? *wcount * n_ib * n_gsplit : 1;
  const bool xcd8 = wlist && gridDim.x % 8 == 0;
  const int x_share = (n_items + 7) / 8, x_lo = xcd8 ? (int)(blockIdx.x % 8) * x_share : 0;
  const int it_end = !wlist ? 1 : xcd8 ? min(n_items, x_lo + x_share) : n_items;
  const int it_step = !wlist ? 1 : xcd8 ? (int)gridDim.x / 8 : (int)gridDim.x;
  for (int it = !wlist ? 0 : xcd8 ? x_lo + (int)blockIdx.x / 8 : (int)blockIdx.x; it < it_end;
       it += it_step) {
  int ib, gs, wl;
  if (wlist) {
    ib = it % n_ib;
    gs = (it / n_ib) % n_gsplit;
    wl = wlist[it / (n_ib * n_gsplit)] - w0;
    if (wl < 0 || wl >= WT) continue;  // listed walker outside this walker tile
  } else {
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so the
    // item blocks of one (walker, Cholesky range), which stage the same
    // Lambda slabs, are given consecutive ids on one XCD and share its L2.
    const int nblk = gridDim.x, b = blockIdx.x;
    const int per = nblk / 8, rem = nblk % 8, xcd = b % 8;
    const int logical = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + b / 8;
    ib = logical % n_ib;
    gs = (logical / n_ib) % n_gsplit;
    wl = logical / (n_ib * n_gsplit);
    if (wmask && !wmask[w0 + wl]) return;  // walker not selected for this pass
  }
  const int w = w0 + wl, tid = threadIdx.x, lane = tid & 63;
  // wave index as a scalar: the plan entry, role and spin are then
  // wave-uniform registers and the role branches below are scalar branches
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int Xa = sa.nv * sa.no, Xb = sb.nv * sb.no, X = Xa + Xb;
  const int gper = (NG + n_gsplit - 1) / n_gsplit;
  const int g0 = gs * gper, g1 = min(NG, g0 + gper);
  // plan entry of this wave: (role | spin << 8, first string of the order,
  // first item, item end)
  const int4 pl = plan[ib * waves_per_block + wave];
  const int role = pl.x & 0xff, sp = (pl.x >> 8) & 0xff, need = (pl.x >> 16) & 3;
  int idx[NIDX];
  CT mm[NMM];
  CT acc[ER_PPL];
#pragma unroll
  for (int j = 0; j < NIDX; ++j) idx[j] = 0;
#pragma unroll
  for (int j = 0; j < NMM; ++j) mm[j] = CT{};
#pragma unroll
  for (int j = 0; j < ER_PPL; ++j) acc[j] = CT{};
  const bool whole = (role & ER_WHOLE) != 0;  // one string per lane (all its row pairs)
  const int item = role == ER_PAIRS ? pl.z + lane * ER_PPL : pl.z + lane;
  const bool live = role != ER_NONE && item < pl.w;
  int str = whole ? pl.y + item : 0;
  if (live && !whole) {
    if (role == ER_PAIRS) {
#pragma unroll
      for (int j = 0; j < ER_PPL; ++j) {
        const int t = item + j;
        const bool ok = t < pl.w;
        idx[j] = ok ? pr.x[t] : 0;  // padding pairs read entry 0 and are dropped below
        idx[ER_PPL + j] = ok ? pr.y[t] : 0;
      }
    } else {
      const int K = role;  // row-pair roles equal the string order
      const int P = K * (K - 1) / 2;
      str = pl.y + item / P;
      const int rp = item % P;
      const int* hwin = sp ? sb.hwin : sa.hwin;
      const int* pwin = sp ? sb.pwin : sa.pwin;
      const int no = sp ? sb.no : sa.no;
      const cd* m2s = (sp ? m2b + (size_t)w * sb.M2 + sb.m2_off[str]
                          : m2a + (size_t)w * sa.M2 + sa.m2_off[str]);
      switch (K) {
        case 2: rp_setup<2, CT>(hwin, pwin, no, str, rp, m2s, idx, mm); break;
        case 3: rp_setup<3, CT>(hwin, pwin, no, str, rp, m2s, idx, mm); break;
        case 4: rp_setup<4, CT>(hwin, pwin, no, str, rp, m2s, idx, mm); break;
        case 5: if constexpr (MAXK >= 5) rp_setup<5 <= MAXK ? 5 : 2, CT>(hwin, pwin, no, str, rp, m2s, idx, mm); break;
        default: if constexpr (MAXK >= 6) rp_setup<6 <= MAXK ? 6 : 2, CT>(hwin, pwin, no, str, rp, m2s, idx, mm); break;
      }
    }
    // windows stored in lam_swizzle layout swz (the hole slot of particle
    // row a XOR-ed with a function of a): spreads a wave's gathers over the
    // LDS banks
    if (swz) {
#pragma unroll
      for (int j = 0; j < NIDX; ++j) idx[j] = lam_swizzle(idx[j], swz);
    }
  }
  // stage buffer b (0/1) starts at sm[b * G * X]: [alpha G x Xa][beta G x Xb].
  // With lds_dma the copies are direct global-to-LDS loads (16 bytes per lane,
  // each wave filling 1 KB runs), which need no registers and no wait before
  // the next stage's arithmetic; the host enables it when every run start is
  // 16-byte aligned.
  const int nwaves = blockDim.x >> 6;
  auto copy = [&](const CT* src, int dst, int n) {
    if (lds_dma) {
      constexpr int per = 16 / sizeof(CT);  // elements per 16-byte lane load
      const int n16 = n / per;
      for (int c = wave; c * 64 < n16; c += nwaves) {
        const int e = c * 64 + lane;
        if (e < n16)
          lds_dma16(src + (size_t)e * per, sm + dst + c * 64 * per);
      }
    } else {
      for (int e = tid; e < n; e += blockDim.x) sm[dst + e] = src[e];
    }
  };
  auto stage = [&](int gb, int b) {  // only the spins this workgroup reads
    const int Gs = min(G, g1 - gb);
    const int d0 = b * G * X;
    if (need & 1) copy(Lam_a + ((size_t)wl * NG + gb) * Xa, d0, Gs * Xa);
    if (need & 2) copy(Lam_b + ((size_t)wl * NG + gb) * Xb, d0 + G * Xa, Gs * Xb);
  };
  const CT* gs_ = sm;
  if constexpr (FLATG) {
    uintptr_t u = reinterpret_cast<uintptr_t>(gs_);
    asm volatile("" : "+s"(u));  // opaque: the compiler cannot tell it is LDS
    gs_ = reinterpret_cast<const CT*>(u);
  }
  // The vector loop, instantiated once per role (role is wave-uniform, so
  // each wave runs exactly one instance and every instance passes the same
  // barriers): body(oa, ob, Gs) consumes one LDS stage.
  auto run_stages = [&](auto&& body) {
    if (g0 < g1) stage(g0, 0);
    __syncthreads();
    int it = 0;
    for (int gb = g0; gb < g1; gb += G, ++it) {
      if (gb + G < g1) stage(gb + G, (it + 1) & 1);
      const int oa = (it & 1) * G * X, ob = oa + G * Xa;
      if (live) body(oa, ob, min(G, g1 - gb));
      __syncthreads();
    }
  };
  // row-pair items of order K: the next vector's gathers are issued before
  // the current vector's arithmetic where the second register set fits
  // (FP64 items of order >= 3 would spill; they load each vector when used)
  auto rows = [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    constexpr bool prefetch = 2 * K * sizeof(CT) <= 64;
    const int Xs = sp ? Xb : Xa;
    run_stages([&](int oa, int ob, int Gs) {
      const int os = sp ? ob : oa;
      CT ya[2 * K];
      if constexpr (!prefetch) {
#pragma unroll 2
        for (int gl = 0; gl < Gs; ++gl) {
          rp_load<K, CT>(gs_, os + gl * Xs, idx, ya);
          rp_math<K, CT>(ya, mm, acc[0]);
        }
      } else {
        // straight-line ping-pong (no conditional loads inside the loop, so
        // each vector waits only for its own gathers)
        CT yb[2 * K];
        rp_load<K, CT>(gs_, os, idx, ya);
        int gl = 0;
        for (; gl + 2 < Gs; gl += 2) {
          rp_load<K, CT>(gs_, os + (gl + 1) * Xs, idx, yb);
          rp_math<K, CT>(ya, mm, acc[0]);
          rp_load<K, CT>(gs_, os + (gl + 2) * Xs, idx, ya);
          rp_math<K, CT>(yb, mm, acc[0]);
        }
        if (gl + 1 < Gs) {
          rp_load<K, CT>(gs_, os + (gl + 1) * Xs, idx, yb);
          rp_math<K, CT>(ya, mm, acc[0]);
          rp_math<K, CT>(yb, mm, acc[0]);
        } else {
          rp_math<K, CT>(ya, mm, acc[0]);
        }
      }
    });
  };
  // whole strings of order K: the K x K window block Y (Y[m][n] = Lambda at
  // particle n, hole m) is gathered once per vector and every row pair (m, m')
  // of the string is contracted from registers: K^2 gathers per string and
  // vector instead of 2K per row pair
  auto whole_rows = [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    constexpr int P = K * (K - 1) / 2;
    // window entry of (particle n, hole m) = pofs[n] + hofs[m] (offsets kept
    // per particle and per hole: 2K registers instead of K^2)
    int pofs[K], hofs[K];
    CT wmm[P * P];
#pragma unroll
    for (int j = 0; j < K; ++j) pofs[j] = hofs[j] = 0;
#pragma unroll
    for (int j = 0; j < P * P; ++j) wmm[j] = CT{};
    if (live) {
      const int* hwin = sp ? sb.hwin : sa.hwin;
      const int* pwin = sp ? sb.pwin : sa.pwin;
      const int no = sp ? sb.no : sa.no;
      const cd* m2s = (sp ? m2b + (size_t)w * sb.M2 + sb.m2_off[str]
                          : m2a + (size_t)w * sa.M2 + sa.m2_off[str]);
#pragma unroll
      for (int n = 0; n < K; ++n) {
        pofs[n] = pwin[str * KMAX + n] * no;
        hofs[n] = hwin[str * KMAX + n];
      }
      int rp = 0;
#pragma unroll
      for (int m = 0; m < K; ++m)
#pragma unroll
        for (int mp = m + 1; mp < K; ++mp, ++rp) {
          int q = 0;
#pragma unroll
          for (int n = 0; n < K; ++n)
#pragma unroll
            for (int np = n + 1; np < K; ++np, ++q) {
              cd v = m2s[rp * P + q];
              if ((m + mp + n + np) & 1) v = -v;
              wmm[rp * P + q] = from_cd<CT>(v);
            }
        }
    }
    const int Xs = sp ? Xb : Xa;
    run_stages([&](int oa, int ob, int Gs) {
      const int os = sp ? ob : oa;
      for (int gl = 0; gl < Gs; ++gl) {
        CT y[K * K];
        const int base = os + gl * Xs;
#pragma unroll
        for (int m = 0; m < K; ++m)
#pragma unroll
          for (int n = 0; n < K; ++n) {
            const int e = pofs[n] + hofs[m];
            y[m * K + n] = gs_[base + (swz ? lam_swizzle(e, swz) : e)];
          }
        int rp = 0;
#pragma unroll
        for (int m = 0; m < K; ++m)
#pragma unroll
          for (int mp = m + 1; mp < K; ++mp, ++rp) {
            CT yy[2 * K];
#pragma unroll
            for (int n = 0; n < K; ++n) {
              yy[n] = y[m * K + n];
              yy[K + n] = y[mp * K + n];
            }
            rp_math<K, CT>(yy, wmm + rp * P, acc[0]);
          }
      }
    });
  };
  if (role == (ER_WHOLE | 3)) {
    whole_rows(std::integral_constant<int, 3>{});
  } else if (role == ER_PAIRS) {
    run_stages([&](int oa, int ob, int Gs) {
      // each pair's operands for the next vector are loaded into its own
      // registers once the current product is formed (a second register
      // set for all four pairs would spill in FP64)
      CT xa[ER_PPL], xb[ER_PPL];
#pragma unroll
      for (int j = 0; j < ER_PPL; ++j) {
        xa[j] = gs_[oa + idx[j]];
        xb[j] = gs_[ob + idx[ER_PPL + j]];
      }
      for (int gl = 1; gl < Gs; ++gl) {
        const int x = oa + gl * Xa, y = ob + gl * Xb;
#pragma unroll
        for (int j = 0; j < ER_PPL; ++j) {
          cfma(acc[j], xa[j], xb[j]);
          xa[j] = gs_[x + idx[j]];
          xb[j] = gs_[y + idx[ER_PPL + j]];
        }
      }
#pragma unroll
      for (int j = 0; j < ER_PPL; ++j) cfma(acc[j], xa[j], xb[j]);
    });
  } else if (role == 2) {
    rows(std::integral_constant<int, 2>{});
  } else if (role == 3) {
    rows(std::integral_constant<int, 3>{});
  } else if (role == 4) {
    rows(std::integral_constant<int, 4>{});
  } else if (MAXK >= 5 && role == 5) {
    rows(std::integral_constant<int, (5 <= MAXK ? 5 : 2)>{});
  } else if (MAXK >= 6 && role >= 6) {
    rows(std::integral_constant<int, (6 <= MAXK ? 6 : 2)>{});
  } else {
    run_stages([](int, int, int) {});
  }
  cd tot{0.0, 0.0};
  if (live) {
    if (role == ER_PAIRS) {
#pragma unroll
      for (int j = 0; j < ER_PPL; ++j)
        if (item + j < pl.w) cfma(tot, coef[(size_t)w * pr.n_pair + item + j], to_cd(acc[j]));
    } else {
      tot = (sp ? Bb[(size_t)w * sb.U + str] : Ba[(size_t)w * sa.U + str]) * to_cd(acc[0]);
    }
  }
  tot = wave_sum(tot);
  if (lane == 0) red[wave] = tot;
  __syncthreads();
  if (tid == 0) {
    cd t{0.0, 0.0};
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += red[q];
    partial[(size_t)w * n_slots + slot0 + (size_t)ib * n_gsplit + gs] = t;
  }
  __syncthreads();  // the next item rewrites the LDS stages and red
  }
}

template <class CT>
static void launch_energy_second_t(const DevSpin& sa, const DevSpin& sb, const DevPairs& pr,
                                   const int4* plan, int n_itemblocks, int waves_per_block, int NW,
                                   int w0, int WT, int NG, int n_gsplit, int G, int max_order,
                                   bool flat_gather, bool use_dma, int swz, const CT* Lam_a, const CT* Lam_b, const cd* coef,
                                   const cd* m2a, const cd* m2b, const cd* Ba, const cd* Bb,
                                   cd* partial, int n_slots, int slot0, hipStream_t st,
                                   const int* wmask, const WalkerList& wls) {
  if (n_itemblocks == 0) return;
  const size_t lds = 2 * (size_t)G * (sa.nv * sa.no + sb.nv * sb.no) * sizeof(CT);
  dim3 grid(WT * n_gsplit * n_itemblocks);
  const dim3 block(64 * waves_per_block);
  if (wls.list) {  // persistent grid: the workgroups resident at once (LDS bound)
    const int per_cu = std::max(1, (int)((160u << 10) / std::max<size_t>(lds, 1)));
    const int by_waves = std::max(1, 32 / waves_per_block);
    grid = dim3(std::max(1, wls.n_cu) * std::min(per_cu, by_waves));
  }
#define MSD_ES(MK, FL)                                                                       \
  hipLaunchKernelGGL((k_energy_second<CT, MK, FL>), grid, block, lds, st, sa, sb, pr, plan,   \
                     n_itemblocks, waves_per_block, NW, w0, NG, n_gsplit, G, Lam_a, Lam_b, coef, \
                     m2a, m2b, Ba, Bb, partial, n_slots, slot0, lds_dma, swz, wmask, wls.list, \
                     wls.count, WT)
  // direct LDS loads need 16-byte aligned runs: every Lambda row of both spins
  // (and each spin's stage region) starts on a 16-byte boundary
  const int per = 16 / (int)sizeof(CT);
  const bool lds_dma = use_dma && (sa.nv * sa.no) % per == 0 && (sb.nv * sb.no) % per == 0;
  if (max_order <= 4) {
    if (flat_gather) MSD_ES(4, true); else MSD_ES(4, false);
  } else {
    if (flat_gather) MSD_ES(ER_MAX_ORDER, true); else MSD_ES(ER_MAX_ORDER, false);
  }
#undef MSD_ES
}

void launch_energy_second(const DevSpin& sa, const DevSpin& sb, const DevPairs& pr,
                          const int4* plan, int n_itemblocks, int waves_per_block, int NW, int w0,
                          int WT, int NG, int n_gsplit, int G, int max_order, bool flat_gather,
                          bool use_dma, int swz, const cd* Lam_a, const cd* Lam_b, const cd* coef,
                          const cd* m2a, const cd* m2b, const cd* Ba, const cd* Bb, cd* partial,
                          int n_slots, int slot0, hipStream_t st, const int* wmask,
                          const WalkerList& wls) {
  launch_energy_second_t<cd>(sa, sb, pr, plan, n_itemblocks, waves_per_block, NW, w0, WT, NG,
                             n_gsplit, G, max_order, flat_gather, use_dma, swz, Lam_a, Lam_b, coef, m2a, m2b, Ba, Bb,
                             partial, n_slots, slot0, st, wmask, wls);
}

void launch_energy_second32(const DevSpin& sa, const DevSpin& sb, const DevPairs& pr,
                            const int4* plan, int n_itemblocks, int waves_per_block, int NW,
                            int w0, int WT, int NG, int n_gsplit, int G, int max_order,
                            bool flat_gather, bool use_dma, int swz, const cf* Lam_a, const cf* Lam_b,
                            const cd* coef, const cd* m2a, const cd* m2b, const cd* Ba,
                            const cd* Bb, cd* partial, int n_slots, int slot0, hipStream_t st,
                            const int* wmask) {
  launch_energy_second_t<cf>(sa, sb, pr, plan, n_itemblocks, waves_per_block, NW, w0, WT, NG,
                             n_gsplit, G, max_order, flat_gather, use_dma, swz, Lam_a, Lam_b, coef, m2a, m2b, Ba, Bb,
                             partial, n_slots, slot0, st, wmask, WalkerList());
}

int energy_minor_blocks(const DevSpin& s) {
  return (s.n_minor + MINOR_THREADS * 8 - 1) / (MINOR_THREADS * 8);
}

void launch_energy_minors(const DevSpin& s, int NW, int w0, int WT, int NG, int n_gsplit,
                          const cd* Lam, const cd* coef, cd* partial, int n_slots, int slot0,
                          hipStream_t st) {
  const int nb = energy_minor_blocks(s);
  if (nb == 0) return;
  const size_t lds = 2 * (size_t)G_STAGE * s.nv * s.no * sizeof(cd);
  hipLaunchKernelGGL(k_energy_minors, dim3(WT, n_gsplit, nb), dim3(MINOR_THREADS), lds, st, s, NW,
                     w0, NG, n_gsplit, Lam, coef, partial, n_slots, slot0);
}

// ============================================================================
// W-form of the second-order terms (memory bounded by the excitation window)
// ============================================================================
// With W^{st}[x][y] = sum_g Lam^{s,g}[x] Lam^{t,g}[y] (x, y window entries), the
// second-order part of the numerator is
//   sum_pairs coefAB[x,y] W^{ab}[x][y]
//   + sum_s sum_minors coef_s[m] (W^{ss}[(a,i)][(b,j)] - W^{ss}[(a,j)][(b,i)]).
// W comes from a real GEMM over the interleaved (re, im) windows:
// G[2x + c][2y + d] = sum_g Lam_c[x] Lam_d[y], so W = (G_rr - G_ii) + i (G_ri + G_ir).
// One workgroup per walker; the sum goes to the walker's energy slot.
constexpr int WF_THREADS = 256;

__device__ __forceinline__ cd wf_at(const double* __restrict__ G, int ld, int x, int y) {
  const double* r0 = G + (size_t)(2 * x) * ld + 2 * y;
  const double* r1 = r0 + ld;
  return cd{r0[0] - r1[1], r0[1] + r1[0]};
}

__global__ __launch_bounds__(WF_THREADS) void k_wform_contract(
    DevSpin sa, DevSpin sb, DevPairs pr, int NW, int w0, const double* __restrict__ Gaa,
    const double* __restrict__ Gab, const double* __restrict__ Gbb, const cd* __restrict__ coefAB,
    const cd* __restrict__ coef_a, const cd* __restrict__ coef_b, cd* __restrict__ partial,
    int n_slots, int slot, const int* __restrict__ wmask) {
  __shared__ cd red[WF_THREADS];
  const int wl = blockIdx.x, w = w0 + wl, tid = threadIdx.x;
  if (wmask && !wmask[w]) return;  // walker not selected for this pass
  const int Xa = sa.nv * sa.no, Xb = sb.nv * sb.no;
  const double* ga = Gaa + (size_t)wl * 4 * Xa * Xa;
  const double* gab = Gab + (size_t)wl * 4 * Xa * Xb;
  const double* gb = Gbb + (size_t)wl * 4 * Xb * Xb;
  cd acc{0.0, 0.0};
  for (int p = tid; p < pr.n_pair; p += WF_THREADS)
    cfma(acc, coefAB[(size_t)w * pr.n_pair + p], wf_at(gab, 2 * Xb, pr.x[p], pr.y[p]));
  for (int m = tid; m < sa.n_minor; m += WF_THREADS) {
    const int* id = sa.mn_idx + 4 * m;
    cfma(acc, coef_a[(size_t)w * sa.n_minor + m],
         wf_at(ga, 2 * Xa, id[0], id[1]) - wf_at(ga, 2 * Xa, id[2], id[3]));
  }
  for (int m = tid; m < sb.n_minor; m += WF_THREADS) {
    const int* id = sb.mn_idx + 4 * m;
    cfma(acc, coef_b[(size_t)w * sb.n_minor + m],
         wf_at(gb, 2 * Xb, id[0], id[1]) - wf_at(gb, 2 * Xb, id[2], id[3]));
  }
  red[tid] = acc;
  __syncthreads();
  for (int off = WF_THREADS / 2; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) partial[(size_t)w * n_slots + slot] = red[0];
}

void launch_wform_contract(const DevSpin& sa, const DevSpin& sb, const DevPairs& pr, int NW,
                           int w0, int WT, const double* Gaa, const double* Gab,
                           const double* Gbb, const cd* coefAB, const cd* coef_a,
                           const cd* coef_b, cd* partial, int n_slots, int slot, hipStream_t st,
                           const int* wmask) {
  hipLaunchKernelGGL(k_wform_contract, dim3(WT), dim3(WF_THREADS), 0, st, sa, sb, pr, NW, w0, Gaa,
                     Gab, Gbb, coefAB, coef_a, coef_b, partial, n_slots, slot, wmask);
}

// ============================================================================
// Energy assembly per walker
// ============================================================================

__global__ __launch_bounds__(256) void k_energy_final(DevSpin sa, DevSpin sb, int NW, int w0,
                                                      int NG, int n_lchunks, int n_slots,
                                                      int e_lo, int e_hi,
                                                      const cd* __restrict__ obar,
                                                      const cd* __restrict__ v0,
                                                      const cd* __restrict__ ex0,
                                                      const cd* __restrict__ ZWa,
                                                      const cd* __restrict__ ZWb,
                                                      const cd* __restrict__ Ca,
                                                      const cd* __restrict__ Cb,
                                                      const cd* __restrict__ czw_part,
                                                      const cd* __restrict__ epart,
                                                      const cd* __restrict__ oba,
                                                      const cd* __restrict__ obb, double e0,
                                                      cd* __restrict__ e_loc,
                                                      const cd* __restrict__ lamc, int n_lparts,
                                                      const int* __restrict__ wmask) {
  __shared__ cd red[256];
  const int wl = blockIdx.x, w = w0 + wl, tid = threadIdx.x, bd = blockDim.x;
  if (wmask && !wmask[w]) return;  // walker not selected for this pass
  cd vab{0.0, 0.0}, kk{0.0, 0.0};
  const cd* va = v0 + (size_t)w * NG;
  const cd* vb = v0 + ((size_t)NW + w) * NG;
  const cd* xa = ex0 + (size_t)w * NG;
  const cd* xb = ex0 + ((size_t)NW + w) * NG;
  cd czw{0.0, 0.0};
  for (int g = tid; g < NG; g += bd) {
    if (lamc) {
      // the general contraction kernel writes v0, ex0 and <C^s, Lambda^s> as
      // per-wave partials [spin][w][g][part]; -(v0_alpha + v0_beta) <C^s,
      // Lambda^s> of this vector, both spins
      const size_t oa = ((size_t)w * NG + g) * n_lparts, ob = (((size_t)NW + w) * NG + g) * n_lparts;
      cd a{0.0, 0.0}, b{0.0, 0.0}, x{0.0, 0.0}, y{0.0, 0.0}, lc{0.0, 0.0};
      for (int p = 0; p < n_lparts; ++p) {
        a += v0[oa + p];
        b += v0[ob + p];
        x += ex0[oa + p];
        y += ex0[ob + p];
        lc += lamc[oa + p] + lamc[ob + p];
      }
      vab += a * b;
      kk += a * a - x + b * b - y;
      czw -= (a + b) * lc;
    } else {
      vab += va[g] * vb[g];
      kk += va[g] * va[g] - xa[g] + vb[g] * vb[g] - xb[g];
    }
  }
  cd first = vab + 0.5 * kk;
  first = block_reduce(first, red);
  const DevSpin* sp[2] = {&sa, &sb};
  const cd* ZW[2] = {ZWa, ZWb};
  const cd* C[2] = {Ca, Cb};
  if (czw_part) {  // already contracted with C per (spin, walker, chunk)
    for (int c = tid; c < 2 * n_lchunks; c += bd)
      czw += czw_part[((size_t)(c / n_lchunks) * NW + w) * n_lchunks + c % n_lchunks];
  } else {
    for (int s2 = 0; s2 < 2; ++s2) {
      const int X = sp[s2]->nv * sp[s2]->no;
      for (int e = tid; e < X; e += bd) {
        cd z{0.0, 0.0};
        for (int c = 0; c < n_lchunks; ++c) z += ZW[s2][((size_t)wl * n_lchunks + c) * X + e];
        czw += C[s2][(size_t)w * X + e] * z;
      }
    }
  }
  for (int c = e_lo + tid; c < e_hi; c += bd) czw += epart[(size_t)w * n_slots + c];  // slots
  czw = block_reduce(czw, red);
  if (tid == 0) e_loc[w] = cd{e0, 0.0} + oba[w] + obb[w] + first + cdiv(czw, obar[w]);
}

void launch_energy_final(const DevSpin& sa, const DevSpin& sb, int NW, int w0, int WT, int NG,
                         int n_lchunks, int n_slots, int e_lo, int e_hi, const cd* obar,
                         const cd* v0,
                         const cd* ex0, const cd* ZWpart_a, const cd* ZWpart_b, const cd* Ca,
                         const cd* Cb, const cd* czw, const cd* epart, const cd* onebody_a,
                         const cd* onebody_b, double e0, cd* e_loc, const cd* lamc,
                         int n_lparts, hipStream_t st, const int* wmask) {
  hipLaunchKernelGGL(k_energy_final, dim3(WT), dim3(256), 0, st, sa, sb, NW, w0, NG, n_lchunks,
                     n_slots, e_lo, e_hi, obar, v0, ex0, ZWpart_a, ZWpart_b, Ca, Cb, czw, epart,
                     onebody_a, onebody_b, e0, e_loc, lamc, n_lparts, wmask);
}

// out[g][r][q] = L[g][rows[r]][q]: Cholesky rows restricted to an orbital subset
__global__ void k_gather_rows(const double* __restrict__ L, int NG, int M,
                              const int* __restrict__ rows, int P, double* __restrict__ out) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)NG * P * M) return;
  const int q = (int)(tid % M);
  const int64_t gr = tid / M;
  const int r = (int)(gr % P), g = (int)(gr / P);
  out[tid] = L[((size_t)g * M + rows[r]) * M + q];
}

void launch_gather_rows(const double* L, int NG, int M, const int* rows, int P, double* out,
                        hipStream_t st) {
  const int64_t n = (int64_t)NG * P * M;
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, L, NG,
                     M, rows, P, out);
}

void init_wick_attributes() {
  const int lim = 150 * 1024;
  hipFuncSetAttribute((const void*)k_ref_inverse, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  hipFuncSetAttribute((const void*)k_green, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  hipFuncSetAttribute((const void*)k_lambda<cd>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  hipFuncSetAttribute((const void*)k_lambda<cf>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  for (const void* f : {(const void*)k_energy_second<cd, 4, false>,
                        (const void*)k_energy_second<cd, 4, true>,
                        (const void*)k_energy_second<cf, 4, false>,
                        (const void*)k_energy_second<cf, 4, true>,
                        (const void*)k_energy_second<cd, ER_MAX_ORDER, false>,
                        (const void*)k_energy_second<cd, ER_MAX_ORDER, true>,
                        (const void*)k_energy_second<cf, ER_MAX_ORDER, false>,
                        (const void*)k_energy_second<cf, ER_MAX_ORDER, true>})
    hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
  hipFuncSetAttribute((const void*)k_energy_minors, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

}  // namespace msd

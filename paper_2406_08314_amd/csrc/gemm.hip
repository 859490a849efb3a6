// FP64 MFMA GEMM for the dense Cholesky contractions and propagation products.
//
//   C[m][n] = alpha * sum_k A(m,k) B(k,n) + beta * C[m][n]      (row-major C)
//
// A(m,k) = A_KMAJ ? A[m*lda + k] : A[k*lda + m]
// B(k,n) = B_KMAJ ? B[n*ldb + k] : B[k*ldb + n]
// Batched over blockIdx.z with element strides; an optional per-batch mask
// skips batches whose mask entry is 0.
//
// Complex mode (CPLX): A is a planar complex matrix (real plane at A, imaginary
// plane at A + a_imag_off, same lda) and B, C hold interleaved complex values
// (real column 2c, imaginary column 2c+1; N counts real columns).  The complex
// product is evaluated as one real GEMM over 2K:
//   C = [Ar Ai] [B ; B~],  B~[:, 2c] = -B[:, 2c+1],  B~[:, 2c+1] = B[:, 2c].
// An optional accumulator (same layout as C) receives acc += C_new.
//
// Tiling for gfx950: 64x64 output tile per 256-thread workgroup (4 wave64),
// each wave 32x32 = 2x2 v_mfma_f64_16x16x4 tiles; K staged through LDS in
// slabs of 16 with a 16-double row pad so the two half-waves of each
// ds_read_b64 hit disjoint banks.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace msd {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64, GB_N = 64, GB_K = 16, GPAD = 16;

template <bool A_KMAJ, bool B_KMAJ, bool CPLX>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g) {
  const int bz = blockIdx.z;
  if (g.mask && g.mask[bz] == 0) return;
  const double* A = g.A + (int64_t)bz * g.strideA;
  const double* B = g.B + (int64_t)bz * g.strideB;
  double* C = g.C + (int64_t)bz * g.strideC;
  double* Acc = g.Acc ? g.Acc + (int64_t)bz * g.strideC : nullptr;

  __shared__ double As[GB_K][GB_M + GPAD];
  __shared__ double Bs[GB_K][GB_N + GPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.y * GB_M;
  const int n0 = blockIdx.x * GB_N;
  const int wm = (wave >> 1) * 32;
  const int wn = (wave & 1) * 32;

  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  const int Keff = CPLX ? 2 * g.K : g.K;
  for (int k0 = 0; k0 < Keff; k0 += GB_K) {
    // ---- stage A slab (GB_M x GB_K) into As[k][m]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int mm, kk;
      if (A_KMAJ) {
        mm = tid >> 2;
        kk = (tid & 3) * 4 + r;
      } else {
        kk = tid >> 4;
        mm = (tid & 15) * 4 + r;
      }
      const int gm = m0 + mm, gk = k0 + kk;
      double v = 0.0;
      if (gm < g.M && gk < Keff) {
        if (CPLX) {
          const bool im = gk >= g.K;
          const int kr = im ? gk - g.K : gk;
          const double* Ap = A + (im ? g.a_imag_off : 0);
          v = A_KMAJ ? Ap[(int64_t)gm * g.lda + kr] : Ap[(int64_t)kr * g.lda + gm];
        } else {
          v = A_KMAJ ? A[(int64_t)gm * g.lda + gk] : A[(int64_t)gk * g.lda + gm];
        }
      }
      As[kk][mm] = v;
    }
    // ---- stage B slab (GB_K x GB_N) into Bs[k][n]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int nn, kk;
      if (B_KMAJ) {
        nn = tid >> 2;
        kk = (tid & 3) * 4 + r;
      } else {
        kk = tid >> 4;
        nn = (tid & 15) * 4 + r;
      }
      const int gn = n0 + nn, gk = k0 + kk;
      double v = 0.0;
      if (gn < g.N && gk < Keff) {
        if (CPLX) {
          const bool im = gk >= g.K;
          const int kr = im ? gk - g.K : gk;
          int cn = gn;
          double sgn = 1.0;
          if (im) {
            cn = gn ^ 1;                  // swap real/imag column
            sgn = (gn & 1) ? 1.0 : -1.0;  // -Im into the real column
          }
          v = sgn * (B_KMAJ ? B[(int64_t)cn * g.ldb + kr] : B[(int64_t)kr * g.ldb + cn]);
        } else {
          v = B_KMAJ ? B[(int64_t)gn * g.ldb + gk] : B[(int64_t)gk * g.ldb + gn];
        }
      }
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GB_K; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a0 = As[kr][wm + (lane & 15)];
      double a1 = As[kr][wm + 16 + (lane & 15)];
      double b0 = Bs[kr][wn + (lane & 15)];
      double b1 = Bs[kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }

  // ---- epilogue: register r of lane l holds D[l/16 + 4r][l % 16]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          const int64_t off = (int64_t)gm * g.ldc + gn;
          double v = g.alpha * acc[i][j][r];
          if (g.beta != 0.0) v += g.beta * C[off];
          C[off] = v;
          if (Acc) Acc[off] += v;
        }
      }
}

template <bool AK, bool BK, bool CX>
static void launch_t(const GemmArgs& g, hipStream_t st) {
  dim3 grid((g.N + GB_N - 1) / GB_N, (g.M + GB_M - 1) / GB_M, g.batch);
  hipLaunchKernelGGL((k_gemm_f64<AK, BK, CX>), grid, dim3(256), 0, st, g);
}

void launch_gemm(const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  if (g.cplx) {
    if (g.a_kmaj && !g.b_kmaj) launch_t<true, false, true>(g, st);
    else if (g.a_kmaj && g.b_kmaj) launch_t<true, true, true>(g, st);
    else if (!g.a_kmaj && !g.b_kmaj) launch_t<false, false, true>(g, st);
    else launch_t<false, true, true>(g, st);
  } else {
    if (g.a_kmaj && !g.b_kmaj) launch_t<true, false, false>(g, st);
    else if (g.a_kmaj && g.b_kmaj) launch_t<true, true, false>(g, st);
    else if (!g.a_kmaj && !g.b_kmaj) launch_t<false, false, false>(g, st);
    else launch_t<false, true, false>(g, st);
  }
}

}  // namespace msd

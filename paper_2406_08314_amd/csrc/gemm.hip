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
// each wave 32x32 = 2x2 v_mfma_f64_16x16x4 tiles; K staged through two LDS
// buffers in slabs of 16 (the next slab's global loads are in flight while
// the current slab feeds the MFMAs; one barrier per slab), with a 16-double
// row pad so the two half-waves of each ds_read_b64 hit disjoint banks.
// Interior tiles of 16-byte-aligned operands use 16-byte global loads.
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace msd {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int GB_M = 64, GB_N = 64, GB_K = 16, GPAD = 16;

// Element (m, k) of A and (k, n) of B with bounds checks (zero outside), and in
// complex mode the [Ar Ai] / [B ; B~] views described above.
template <bool A_KMAJ, bool CPLX>
__device__ __forceinline__ double a_at(const GemmArgs& g, const double* A, int gm, int gk,
                                       int kend) {
  if (gm >= g.M || gk >= kend) return 0.0;
  if (CPLX) {
    const bool im = gk >= g.K;
    const int kr = im ? gk - g.K : gk;
    const double* Ap = A + (im ? g.a_imag_off : 0);
    return A_KMAJ ? Ap[(int64_t)gm * g.lda + kr] : Ap[(int64_t)kr * g.lda + gm];
  }
  return A_KMAJ ? A[(int64_t)gm * g.lda + gk] : A[(int64_t)gk * g.lda + gm];
}

template <bool B_KMAJ, bool CPLX>
__device__ __forceinline__ double b_at(const GemmArgs& g, const double* B, int gk, int gn,
                                       int kend) {
  if (gn >= g.N || gk >= kend) return 0.0;
  if (CPLX) {
    const bool im = gk >= g.K;
    const int kr = im ? gk - g.K : gk;
    int cn = gn;
    double sgn = 1.0;
    if (im) {
      cn = gn ^ 1;                  // swap real/imag column
      sgn = (gn & 1) ? 1.0 : -1.0;  // -Im into the real column
    }
    return sgn * (B_KMAJ ? B[(int64_t)cn * g.ldb + kr] : B[(int64_t)kr * g.ldb + cn]);
  }
  return B_KMAJ ? B[(int64_t)gn * g.ldb + gk] : B[(int64_t)gk * g.ldb + gn];
}

template <bool A_KMAJ, bool B_KMAJ, bool CPLX>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g) {
  const int bz = blockIdx.z;
  if (g.mask && g.mask[bz] == 0) return;
  // split-K: slice z owns K range [kbeg, kend) and writes a private partial
  const bool split = g.splitk > 1;
  const int kchunk = split ? ((g.K + g.splitk * GB_K - 1) / (g.splitk * GB_K)) * GB_K : 0;
  const int kbeg = split ? bz * kchunk : 0;
  const int kend = split ? min(g.K, kbeg + kchunk) : (CPLX ? 2 * g.K : g.K);
  const double* A = g.A + (split ? 0 : (int64_t)bz * g.strideA);
  const double* B = g.B + (split ? 0 : (int64_t)bz * g.strideB);
  double* C = split ? g.ws + (int64_t)bz * g.M * g.N : g.C + (int64_t)bz * g.strideC;
  const int64_t ldc = split ? g.N : g.ldc;
  double* Acc = (!split && g.Acc) ? g.Acc + (int64_t)bz * g.strideC : nullptr;

  __shared__ double As[2][GB_K][GB_M + GPAD];
  __shared__ double Bs[2][GB_K][GB_N + GPAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.y * GB_M;
  const int n0 = blockIdx.x * GB_N;
  const int wm = (wave >> 1) * 32;
  const int wn = (wave & 1) * 32;

  // per-thread staging coordinates: 4 consecutive elements along the
  // contiguous dimension of each operand
  const int a_mm = A_KMAJ ? (tid >> 2) : (tid & 15) * 4;
  const int a_kk = A_KMAJ ? (tid & 3) * 4 : (tid >> 4);
  const int b_nn = B_KMAJ ? (tid >> 2) : (tid & 15) * 4;
  const int b_kk = B_KMAJ ? (tid & 3) * 4 : (tid >> 4);
  // 16-byte loads are legal when every row start is 16-byte aligned
  const bool a_vec = ((g.lda & 1) == 0) && ((((uintptr_t)A) & 15) == 0) &&
                     (!CPLX || ((g.a_imag_off & 1) == 0 && (g.K & 3) == 0));
  const bool b_vec = ((g.ldb & 1) == 0) && ((((uintptr_t)B) & 15) == 0) &&
                     (!CPLX || (g.K & 3) == 0);
  const bool m_full = m0 + GB_M <= g.M;
  const bool n_full = n0 + GB_N <= g.N;

  auto load = [&](int k0, double* ra, double* rb) __attribute__((always_inline)) {
    const bool k_full = k0 + GB_K <= kend;
    // A
    if (a_vec && m_full && k_full) {
      const int gm = m0 + a_mm, gk = k0 + a_kk;
      const double* p;
      if (A_KMAJ) {
        if (CPLX) {
          const bool im = gk >= g.K;
          p = A + (im ? g.a_imag_off : 0) + (int64_t)gm * g.lda + (im ? gk - g.K : gk);
        } else {
          p = A + (int64_t)gm * g.lda + gk;
        }
      } else {
        if (CPLX) {
          const bool im = gk >= g.K;
          p = A + (im ? g.a_imag_off : 0) + (int64_t)(im ? gk - g.K : gk) * g.lda + gm;
        } else {
          p = A + (int64_t)gk * g.lda + gm;
        }
      }
      const double2 v0 = *reinterpret_cast<const double2*>(p);
      const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
      ra[0] = v0.x; ra[1] = v0.y; ra[2] = v1.x; ra[3] = v1.y;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        ra[r] = A_KMAJ ? a_at<A_KMAJ, CPLX>(g, A, m0 + a_mm, k0 + a_kk + r, kend)
                       : a_at<A_KMAJ, CPLX>(g, A, m0 + a_mm + r, k0 + a_kk, kend);
    }
    // B
    if (b_vec && n_full && k_full) {
      const int gn = n0 + b_nn, gk = k0 + b_kk;
      if (B_KMAJ) {
        // 4 consecutive k of one column
        if (CPLX) {
          const bool im = gk >= g.K;
          const int kr = im ? gk - g.K : gk;
          const int cn = im ? (gn ^ 1) : gn;
          const double sgn = im ? ((gn & 1) ? 1.0 : -1.0) : 1.0;
          const double* p = B + (int64_t)cn * g.ldb + kr;
          const double2 v0 = *reinterpret_cast<const double2*>(p);
          const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
          rb[0] = sgn * v0.x; rb[1] = sgn * v0.y; rb[2] = sgn * v1.x; rb[3] = sgn * v1.y;
        } else {
          const double* p = B + (int64_t)gn * g.ldb + gk;
          const double2 v0 = *reinterpret_cast<const double2*>(p);
          const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
          rb[0] = v0.x; rb[1] = v0.y; rb[2] = v1.x; rb[3] = v1.y;
        }
      } else {
        // 4 consecutive n (two complex pairs in complex mode) of one row
        if (CPLX) {
          const bool im = gk >= g.K;
          const int kr = im ? gk - g.K : gk;
          const double* p = B + (int64_t)kr * g.ldb + gn;
          const double2 v0 = *reinterpret_cast<const double2*>(p);
          const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
          if (im) {
            rb[0] = -v0.y; rb[1] = v0.x; rb[2] = -v1.y; rb[3] = v1.x;
          } else {
            rb[0] = v0.x; rb[1] = v0.y; rb[2] = v1.x; rb[3] = v1.y;
          }
        } else {
          const double* p = B + (int64_t)gk * g.ldb + gn;
          const double2 v0 = *reinterpret_cast<const double2*>(p);
          const double2 v1 = *reinterpret_cast<const double2*>(p + 2);
          rb[0] = v0.x; rb[1] = v0.y; rb[2] = v1.x; rb[3] = v1.y;
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        rb[r] = B_KMAJ ? b_at<B_KMAJ, CPLX>(g, B, k0 + b_kk + r, n0 + b_nn, kend)
                       : b_at<B_KMAJ, CPLX>(g, B, k0 + b_kk, n0 + b_nn + r, kend);
    }
  };

  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

  // K tiles go global -> registers two tiles ahead of their MFMAs (two
  // register sets, loop unrolled by two), registers -> LDS double buffer
  int buf = 0;
  auto store = [&](const double* ra, const double* rb) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (A_KMAJ) As[buf][a_kk + r][a_mm] = ra[r];
      else As[buf][a_kk][a_mm + r] = ra[r];
      if (B_KMAJ) Bs[buf][b_kk + r][b_nn] = rb[r];
      else Bs[buf][b_kk][b_nn + r] = rb[r];
    }
  };
  auto compute = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int kk = 0; kk < GB_K; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a0 = As[buf][kr][wm + (lane & 15)];
      const double a1 = As[buf][kr][wm + 16 + (lane & 15)];
      const double b0 = Bs[buf][kr][wn + (lane & 15)];
      const double b1 = Bs[buf][kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    buf ^= 1;
  };
  double ra0[4], rb0[4], ra1[4], rb1[4];
  if (kbeg < kend) load(kbeg, ra0, rb0);
  if (kbeg + GB_K < kend) load(kbeg + GB_K, ra1, rb1);
  for (int k0 = kbeg; k0 < kend; k0 += 2 * GB_K) {
    store(ra0, rb0);
    __syncthreads();
    if (k0 + 2 * GB_K < kend) load(k0 + 2 * GB_K, ra0, rb0);  // in flight for two tiles
    compute();
    if (k0 + GB_K >= kend) break;
    store(ra1, rb1);
    __syncthreads();
    if (k0 + 3 * GB_K < kend) load(k0 + 3 * GB_K, ra1, rb1);
    compute();
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
          const int64_t off = g.c_block > 0
                                  ? ((int64_t)(gn / g.c_block) * g.M + gm) * g.c_block +
                                        gn % g.c_block
                                  : (int64_t)gm * ldc + gn;
          if (split) {
            C[off] = acc[i][j][r];
            continue;
          }
          double v = g.alpha * acc[i][j][r];
          if (g.beta != 0.0) v += g.beta * C[off];
          C[off] = v;
          if (Acc) Acc[off] += v;
        }
      }
}

// Sum of the split-K partials in slice order (deterministic), then alpha/beta.
__global__ void k_splitk_reduce(GemmArgs g) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)g.M * g.N) return;
  const int m = (int)(tid / g.N), n = (int)(tid % g.N);
  // slices summed in order; four loads in flight per group (one wait each)
  const int64_t mn = (int64_t)g.M * g.N;
  double s = 0.0;
  int z = 0;
  for (; z + 4 <= g.splitk; z += 4) {
    const double a0 = g.ws[(z + 0) * mn + tid], a1 = g.ws[(z + 1) * mn + tid];
    const double a2 = g.ws[(z + 2) * mn + tid], a3 = g.ws[(z + 3) * mn + tid];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; z < g.splitk; ++z) s += g.ws[z * mn + tid];
  const int64_t off = (int64_t)m * g.ldc + n;
  double v = g.alpha * s;
  if (g.beta != 0.0) v += g.beta * g.C[off];
  g.C[off] = v;
}

template <bool AK, bool BK, bool CX>
static void launch_t(const GemmArgs& g, hipStream_t st) {
  const int z = g.splitk > 1 ? g.splitk : g.batch;
  dim3 grid((g.N + GB_N - 1) / GB_N, (g.M + GB_M - 1) / GB_M, z);
  hipLaunchKernelGGL((k_gemm_f64<AK, BK, CX>), grid, dim3(256), 0, st, g);
  if (g.splitk > 1) {
    const int64_t n = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g);
  }
}

void launch_gemm(const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  if (g.c_block > 0 && (g.batch != 1 || g.splitk > 1 || g.beta != 0.0 || g.Acc)) return;
  if (g.splitk > 1 && (g.batch != 1 || g.cplx || !g.ws || g.Acc)) return;  // unsupported combination
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

// ============================================================================
// FP32 MFMA GEMM (mixed-precision form): the same 64x64 tile, 4 waves of 2x2
// v_mfma_f32_16x16x4f32, K slabs of 16 double-buffered in LDS.  Row pad of 16
// floats puts the four k-rows read by one ds_read_b32 wave in disjoint banks.
// ============================================================================

typedef float float4_t __attribute__((ext_vector_type(4)));
constexpr int GPAD32 = 16;

template <bool A_KMAJ, bool B_KMAJ, bool OUT64>
__global__ __launch_bounds__(256) void k_gemm_f32(GemmArgs32 g) {
  const int bz = blockIdx.z;
  if (g.mask && g.mask[bz] == 0) return;
  const bool split = g.splitk > 1;
  const int kchunk = split ? ((g.K + g.splitk * GB_K - 1) / (g.splitk * GB_K)) * GB_K : 0;
  const int kbeg = split ? bz * kchunk : 0;
  const int kend = split ? min(g.K, kbeg + kchunk) : g.K;
  const float* A = g.A + (split ? 0 : (int64_t)bz * g.strideA);
  const float* B = g.B + (split ? 0 : (int64_t)bz * g.strideB);

  __shared__ float As[2][GB_K][GB_M + GPAD32];
  __shared__ float Bs[2][GB_K][GB_N + GPAD32];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.y * GB_M;
  const int n0 = blockIdx.x * GB_N;
  const int wm = (wave >> 1) * 32;
  const int wn = (wave & 1) * 32;
  const int a_mm = A_KMAJ ? (tid >> 2) : (tid & 15) * 4;
  const int a_kk = A_KMAJ ? (tid & 3) * 4 : (tid >> 4);
  const int b_nn = B_KMAJ ? (tid >> 2) : (tid & 15) * 4;
  const int b_kk = B_KMAJ ? (tid & 3) * 4 : (tid >> 4);
  const bool a_vec = ((g.lda & 3) == 0) && ((((uintptr_t)A) & 15) == 0);
  const bool b_vec = ((g.ldb & 3) == 0) && ((((uintptr_t)B) & 15) == 0);
  const bool m_full = m0 + GB_M <= g.M;
  const bool n_full = n0 + GB_N <= g.N;

  auto load = [&](int k0, float* ra, float* rb) __attribute__((always_inline)) {
    const bool k_full = k0 + GB_K <= kend;
    if (a_vec && m_full && k_full) {
      const int gm = m0 + a_mm, gk = k0 + a_kk;
      const float* p = A_KMAJ ? A + (int64_t)gm * g.lda + gk : A + (int64_t)gk * g.lda + gm;
      const float4 v = *reinterpret_cast<const float4*>(p);
      ra[0] = v.x; ra[1] = v.y; ra[2] = v.z; ra[3] = v.w;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + a_mm + (A_KMAJ ? 0 : r), gk = k0 + a_kk + (A_KMAJ ? r : 0);
        ra[r] = (gm < g.M && gk < kend)
                    ? (A_KMAJ ? A[(int64_t)gm * g.lda + gk] : A[(int64_t)gk * g.lda + gm])
                    : 0.f;
      }
    }
    if (b_vec && n_full && k_full) {
      const int gn = n0 + b_nn, gk = k0 + b_kk;
      const float* p = B_KMAJ ? B + (int64_t)gn * g.ldb + gk : B + (int64_t)gk * g.ldb + gn;
      const float4 v = *reinterpret_cast<const float4*>(p);
      rb[0] = v.x; rb[1] = v.y; rb[2] = v.z; rb[3] = v.w;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gn = n0 + b_nn + (B_KMAJ ? 0 : r), gk = k0 + b_kk + (B_KMAJ ? r : 0);
        rb[r] = (gn < g.N && gk < kend)
                    ? (B_KMAJ ? B[(int64_t)gn * g.ldb + gk] : B[(int64_t)gk * g.ldb + gn])
                    : 0.f;
      }
    }
  };

  float4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};

  // as the FP64 kernel: two register sets, global loads two tiles ahead
  int buf = 0;
  auto store = [&](const float* ra, const float* rb) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (A_KMAJ) As[buf][a_kk + r][a_mm] = ra[r];
      else As[buf][a_kk][a_mm + r] = ra[r];
      if (B_KMAJ) Bs[buf][b_kk + r][b_nn] = rb[r];
      else Bs[buf][b_kk][b_nn + r] = rb[r];
    }
  };
  auto compute = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int kk = 0; kk < GB_K; kk += 4) {
      const int kr = kk + (lane >> 4);
      const float a0 = As[buf][kr][wm + (lane & 15)];
      const float a1 = As[buf][kr][wm + 16 + (lane & 15)];
      const float b0 = Bs[buf][kr][wn + (lane & 15)];
      const float b1 = Bs[buf][kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    buf ^= 1;
  };
  float ra0[4], rb0[4], ra1[4], rb1[4];
  if (kbeg < kend) load(kbeg, ra0, rb0);
  if (kbeg + GB_K < kend) load(kbeg + GB_K, ra1, rb1);
  for (int k0 = kbeg; k0 < kend; k0 += 2 * GB_K) {
    store(ra0, rb0);
    __syncthreads();
    if (k0 + 2 * GB_K < kend) load(k0 + 2 * GB_K, ra0, rb0);
    compute();
    if (k0 + GB_K >= kend) break;
    store(ra1, rb1);
    __syncthreads();
    if (k0 + 3 * GB_K < kend) load(k0 + 3 * GB_K, ra1, rb1);
    compute();
  }

  // epilogue: register r of lane l holds D[4 (l/16) + r][l % 16]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < g.M && gn < g.N) {
          if (split) {
            g.ws[(int64_t)bz * g.M * g.N + (int64_t)gm * g.N + gn] = acc[i][j][r];
            continue;
          }
          const int64_t off = g.c_block > 0
                                  ? ((int64_t)(gn / g.c_block) * g.M + gm) * g.c_block +
                                        gn % g.c_block
                                  : (int64_t)bz * g.strideC + (int64_t)gm * g.ldc + gn;
          const double v = g.alpha * (double)acc[i][j][r];
          if (OUT64) g.C64[off] = v;
          else g.C32[off] = (float)v;
        }
      }
}

__global__ void k_splitk_reduce32(GemmArgs32 g) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)g.M * g.N) return;
  const int m = (int)(tid / g.N), n = (int)(tid % g.N);
  const int64_t mn = (int64_t)g.M * g.N;
  double s = 0.0;
  int z = 0;
  for (; z + 4 <= g.splitk; z += 4) {
    const float a0 = g.ws[(z + 0) * mn + tid], a1 = g.ws[(z + 1) * mn + tid];
    const float a2 = g.ws[(z + 2) * mn + tid], a3 = g.ws[(z + 3) * mn + tid];
    s += (double)a0;
    s += (double)a1;
    s += (double)a2;
    s += (double)a3;
  }
  for (; z < g.splitk; ++z) s += (double)g.ws[z * mn + tid];
  const int64_t off = (int64_t)m * g.ldc + n;
  if (g.C64) g.C64[off] = g.alpha * s;
  else g.C32[off] = (float)(g.alpha * s);
}

template <bool AK, bool BK>
static void launch32_t(const GemmArgs32& g, hipStream_t st) {
  const int z = g.splitk > 1 ? g.splitk : g.batch;
  dim3 grid((g.N + GB_N - 1) / GB_N, (g.M + GB_M - 1) / GB_M, z);
  if (g.C64) hipLaunchKernelGGL((k_gemm_f32<AK, BK, true>), grid, dim3(256), 0, st, g);
  else hipLaunchKernelGGL((k_gemm_f32<AK, BK, false>), grid, dim3(256), 0, st, g);
  if (g.splitk > 1) {
    const int64_t n = (int64_t)g.M * g.N;
    hipLaunchKernelGGL(k_splitk_reduce32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g);
  }
}

void launch_gemm32(const GemmArgs32& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  if (!g.C32 == !g.C64) return;                              // exactly one output
  if (g.c_block > 0 && (g.batch != 1 || g.splitk > 1)) return;
  if (g.splitk > 1 && (g.batch != 1 || !g.ws)) return;      // unsupported combination
  if (g.a_kmaj && !g.b_kmaj) launch32_t<true, false>(g, st);
  else if (g.a_kmaj && g.b_kmaj) launch32_t<true, true>(g, st);
  else if (!g.a_kmaj && !g.b_kmaj) launch32_t<false, false>(g, st);
  else launch32_t<false, true>(g, st);
}

__global__ void k_f64_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

void launch_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
}

}  // namespace msd

namespace msd {

// ============================================================================
// A2 + A6 fused: Cholesky contraction and energy intermediates.
// Workgroup = (group of WB walkers, chunk of Cholesky vectors).  For every g
// in the chunk and each spin the tile LT^g = L^g[R u V, :] T (P x 2N*WB real,
// P <= 64, 2N*WB <= 64) is formed with v_mfma_f64_16x16x4 into LDS and
// consumed there: v0 = tr Q, ex0 = tr QQ (Q = LT^g[R, :]),
// Lam = T[V,:] Q - LT^g[V,:], Xi = Lam Q[:, O], Lam window -> HBM, and
// ZW += Xi - (v0a + v0b) Lam accumulated in registers.
// ============================================================================

constexpr int CC_THREADS = 512;
constexpr int CC_ZPT = 4;  // window entries per thread and spin: WB*nv*no <= 2048

struct CCSpin {
  const double* Llt;  // [NG][P][M]
  const cd* T;        // [M][NW][N]
  cd* Lam;            // [WT][NG][X]   (walker-tile local)
  cd* ZW;             // [WT][n_chunks][X]
};

__device__ __forceinline__ cd wave_sum_cc(cd v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
  }
  return v;
}

__global__ __launch_bounds__(CC_THREADS) void k_chol_contract(DevSpin sa, DevSpin sb, CCSpin ca,
                                                              CCSpin cb, int M, int NW, int w0,
                                                              int WT, int NG, int g_chunk, int WB,
                                                              cd* __restrict__ v0,
                                                              cd* __restrict__ ex0) {
  // LDS: region0 holds the GEMM staging slabs, then T[V,:] of the walker
  // group and the full Lam rows; Ct holds the LT^g tile.
  extern __shared__ double smem[];
  typedef double Slab[GB_K][GB_M + GPAD];
  Slab* As = reinterpret_cast<Slab*>(smem);                              // [2]
  Slab* Bs = reinterpret_cast<Slab*>(smem + 2 * GB_K * (GB_M + GPAD));  // [2]
  __shared__ double Ct[64][64 + 1];
  __shared__ cd v0s[2][16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wg = blockIdx.x, chunk = blockIdx.y, n_chunks = gridDim.y;
  const int wl0 = wg * WB;                   // first tile-local walker of the group
  const int WBv = min(WB, WT - wl0);         // walkers present
  const int g0 = chunk * g_chunk, g1 = min(NG, g0 + g_chunk);
  const int wm = ((wave & 3) >> 1) * 32, wn = (wave & 1) * 32;
  const int Xa = sa.nv * sa.no, Xb = sb.nv * sb.no;

  cd za[CC_ZPT], zb[CC_ZPT];
#pragma unroll
  for (int q = 0; q < CC_ZPT; ++q) za[q] = zb[q] = cd{0.0, 0.0};

  for (int g = g0; g < g1; ++g) {
#pragma unroll 1
    for (int s2 = 0; s2 < 2; ++s2) {
      const DevSpin& S = s2 ? sb : sa;
      const CCSpin& C = s2 ? cb : ca;
      const int N = S.N, P = S.P, nv = S.nv, no = S.no, X = nv * no;
      if (N == 0) {
        if (tid < WBv) {
          const int w = w0 + wl0 + tid;
          v0[((size_t)s2 * NW + w) * NG + g] = cd{0.0, 0.0};
          ex0[((size_t)s2 * NW + w) * NG + g] = cd{0.0, 0.0};
          v0s[s2][tid] = cd{0.0, 0.0};
        }
        __syncthreads();
        continue;
      }
      // ---------------- tile GEMM: Ct[r][c] = sum_k L^g[r][k] Tcols[k][c]
      const int ncol = 2 * N * WBv;
      const double* Ab = C.Llt + (size_t)g * P * M;
      const double* Bb = reinterpret_cast<const double*>(C.T) + 2 * (size_t)(w0 + wl0) * N;
      const int64_t ldb = 2 * (int64_t)NW * N;
      double4_t acc[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
      // 512 threads stage 64x16 of A and 16x64 of B: 2 + 2 elements each
      const int a_mm = tid >> 3, a_kk = (tid & 7) * 2;
      const int b_kk = tid >> 5, b_nn = (tid & 31) * 2;
      double ra[2], rb[2];
      auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const int gk = k0 + a_kk + r;
          ra[r] = (a_mm < P && gk < M) ? Ab[(size_t)a_mm * M + gk] : 0.0;
          const int bk = k0 + b_kk, bn = b_nn + r;
          rb[r] = (bk < M && bn < ncol) ? Bb[(size_t)bk * ldb + bn] : 0.0;
        }
      };
      int buf = 0;
      load(0);
      for (int k0 = 0; k0 < M; k0 += GB_K) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          As[buf][a_kk + r][a_mm] = ra[r];
          Bs[buf][b_kk][b_nn + r] = rb[r];
        }
        __syncthreads();
        if (k0 + GB_K < M) load(k0 + GB_K);
        if (wave < 4) {
#pragma unroll
          for (int kk = 0; kk < GB_K; kk += 4) {
            const int kr = kk + (lane >> 4);
            const double a0 = As[buf][kr][wm + (lane & 15)];
            const double a1 = As[buf][kr][wm + 16 + (lane & 15)];
            const double b0 = Bs[buf][kr][wn + (lane & 15)];
            const double b1 = Bs[buf][kr][wn + 16 + (lane & 15)];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
          }
        }
        buf ^= 1;
      }
      if (wave < 4) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              Ct[wm + i * 16 + (lane >> 4) + 4 * r][wn + j * 16 + (lane & 15)] = acc[i][j][r];
      }
      __syncthreads();  // Ct complete; staging slabs free
      // complex view: Q_j(r, c) = Ct[r][j*2N + 2c] + i Ct[r][j*2N + 2c + 1]
      auto ct = [&](int r, int jw, int c) {
        return cd{Ct[r][jw * 2 * N + 2 * c], Ct[r][jw * 2 * N + 2 * c + 1]};
      };
      const int LW = nv * N;
      cd* TVs = reinterpret_cast<cd*>(smem);  // [WBv][nv][N]
      cd* Lf = TVs + (size_t)WB * LW;         // [WBv][nv][N]
      for (int e = tid; e < WBv * LW; e += CC_THREADS) {
        const int jw = e / LW, rem = e % LW, a = rem / N, jj = rem % N;
        TVs[e] = C.T[((size_t)S.vir[a] * NW + w0 + wl0 + jw) * N + jj];
      }
      // ---------------- v0, ex0 per walker (one wave per walker)
      for (int jw = wave; jw < WBv; jw += CC_THREADS / 64) {
        cd v{0.0, 0.0}, x{0.0, 0.0};
        for (int e = lane; e < N * N; e += 64) {
          const int r = e / N, c = e % N;
          cfma(x, ct(r, jw, c), ct(c, jw, r));
          if (r == c) v += ct(r, jw, c);
        }
        v = wave_sum_cc(v);
        x = wave_sum_cc(x);
        if (lane == 0) {
          const int w = w0 + wl0 + jw;
          v0s[s2][jw] = v;
          v0[((size_t)s2 * NW + w) * NG + g] = v;
          ex0[((size_t)s2 * NW + w) * NG + g] = x;
        }
      }
      __syncthreads();
      // ---------------- Lam full rows: Lam = T[V,:] Q - LT[V,:]
      for (int e = tid; e < WBv * LW; e += CC_THREADS) {
        const int jw = e / LW, rem = e % LW, a = rem / N, c = rem % N;
        const cd* tv = TVs + (size_t)jw * LW + a * N;
        cd accl = -ct(N + a, jw, c);
        for (int jj = 0; jj < N; ++jj) cfma(accl, tv[jj], ct(jj, jw, c));
        Lf[e] = accl;
      }
      __syncthreads();
      // ---------------- Xi, Lam window, ZW
#pragma unroll
      for (int q = 0; q < CC_ZPT; ++q) {
        const int e = tid + CC_THREADS * q;
        if (e < WBv * X) {
          const int jw = e / X, rem = e % X, a = rem / no, i = rem % no;
          const int oc = S.oslot[i];
          const cd* Lrow = Lf + (size_t)jw * LW + a * N;
          cd xi{0.0, 0.0};
          for (int c = 0; c < N; ++c) cfma(xi, Lrow[c], ct(c, jw, oc));
          const cd lam = Lrow[oc];
          C.Lam[((size_t)(wl0 + jw) * NG + g) * X + rem] = lam;
          if (s2 == 0) {
            za[q] += xi - v0s[0][jw] * lam;
          } else {
            zb[q] += xi - (v0s[0][jw] + v0s[1][jw]) * lam;
          }
        }
      }
      if (s2 == 1) {
        // the alpha accumulators still miss -v0b * Lam^a of this g; the alpha
        // window values were written by this same thread in the alpha pass
#pragma unroll
        for (int q = 0; q < CC_ZPT; ++q) {
          const int e = tid + CC_THREADS * q;
          if (e < WBv * Xa) {
            const int jw = e / Xa;
            za[q] -= v0s[1][jw] * ca.Lam[((size_t)(wl0 + jw) * NG + g) * Xa + e % Xa];
          }
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < CC_ZPT; ++q) {
    int e = tid + CC_THREADS * q;
    if (e < WBv * Xa) {
      const int jw = e / Xa;
      ca.ZW[((size_t)(wl0 + jw) * n_chunks + chunk) * Xa + e % Xa] = za[q];
    }
    if (e < WBv * Xb) {
      const int jw = e / Xb;
      cb.ZW[((size_t)(wl0 + jw) * n_chunks + chunk) * Xb + e % Xb] = zb[q];
    }
  }
}

static size_t chol_contract_lds(const DevSpin& sa, const DevSpin& sb, int WB) {
  const size_t tv_lf = 2 * (size_t)WB * max(sa.nv * sa.N, sb.nv * sb.N) * sizeof(cd);
  return max(tv_lf, 4 * (size_t)GB_K * (GB_M + GPAD) * sizeof(double));
}

bool chol_contract_fits(const DevSpin& sa, const DevSpin& sb, int* WB) {
  int nmax = max(sa.N, sb.N);
  if (nmax == 0 || nmax > 32 || sa.P > 64 || sb.P > 64) return false;
  int wb = min(64 / (2 * nmax), 16);
  if (wb * sa.nv * sa.no > CC_THREADS * CC_ZPT || wb * sb.nv * sb.no > CC_THREADS * CC_ZPT)
    return false;
  if (chol_contract_lds(sa, sb, wb) > 110 * 1024) return false;
  *WB = wb;
  return true;
}

void launch_chol_contract(const DevSpin& sa, const DevSpin& sb, const double* Llt_a,
                          const double* Llt_b, const cd* Ta, const cd* Tb, cd* Lam_a, cd* Lam_b,
                          cd* ZW_a, cd* ZW_b, int M, int NW, int w0, int WT, int NG, int g_chunk,
                          int WB, cd* v0, cd* ex0, hipStream_t st) {
  const int n_chunks = (NG + g_chunk - 1) / g_chunk;
  const CCSpin ca{Llt_a, Ta, Lam_a, ZW_a}, cb{Llt_b, Tb, Lam_b, ZW_b};
  dim3 grid((WT + WB - 1) / WB, n_chunks);
  hipLaunchKernelGGL(k_chol_contract, grid, dim3(CC_THREADS), chol_contract_lds(sa, sb, WB), st, sa,
                     sb, ca, cb, M, NW, w0, WT, NG, g_chunk, WB, v0, ex0);
}

void init_gemm_attributes() {
  hipFuncSetAttribute((const void*)k_chol_contract, hipFuncAttributeMaxDynamicSharedMemorySize,
                      112 * 1024);
}

}  // namespace msd

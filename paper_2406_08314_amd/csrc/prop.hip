// Propagation-step kernels (Eqs. 4-5, 8-12 and the periodic QR).
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace msd {

// Y rows (w, 0) = -sqrt(dt) Im(x - xbar), (w, 1) = sqrt(dt) Re(x - xbar), so that
// Y . L gives the real and imaginary planes of VHS = i sqrt(dt) sum_g (x - xbar)_g L^g.
__global__ void k_vhs_prep(int NW, int NG, const double* __restrict__ x,
                           const cd* __restrict__ xbar, double sqrt_dt,
                           const double* __restrict__ weights, double* __restrict__ Y) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)NW * NG) return;
  const int w = (int)(tid / NG), g = (int)(tid % NG);
  const cd xb = xbar[tid];
  const double yr = x[tid] - xb.re, yi = -xb.im;
  const bool live = weights[w] != 0.0;
  Y[((size_t)2 * w) * NG + g] = live ? -sqrt_dt * yi : 0.0;
  Y[((size_t)2 * w + 1) * NG + g] = live ? sqrt_dt * yr : 0.0;
}

void launch_vhs_prep(int NW, int NG, const double* x, const cd* xbar, double sqrt_dt,
                     const double* weights, double* Y, hipStream_t st) {
  const int64_t n = (int64_t)NW * NG;
  hipLaunchKernelGGL(k_vhs_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, NW, NG, x,
                     xbar, sqrt_dt, weights, Y);
}

// Phaseless weight update (Eqs. 8-12) for walkers that were live at the start
// of the step; the stored log-overlap moves to the propagated walker.
__global__ __launch_bounds__(256) void k_weights(int NW, int NG, const double* __restrict__ x,
                                                 const cd* __restrict__ xbar,
                                                 const cd* __restrict__ logo_new,
                                                 cd* __restrict__ logo,
                                                 double* __restrict__ weights, double dt,
                                                 double e_shift) {
  __shared__ cd red_xx[256], red_bb[256];
  const int w = blockIdx.x, tid = threadIdx.x;
  cd xx{0.0, 0.0}, bb{0.0, 0.0};
  for (int g = tid; g < NG; g += blockDim.x) {
    const cd xb = xbar[(size_t)w * NG + g];
    xx += x[(size_t)w * NG + g] * xb;
    bb += xb * xb;
  }
  red_xx[tid] = xx;
  red_bb[tid] = bb;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (tid < off) {
      red_xx[tid] += red_xx[tid + off];
      red_bb[tid] += red_bb[tid + off];
    }
    __syncthreads();
  }
  if (tid != 0) return;
  const double w0 = weights[w];
  if (w0 == 0.0) return;
  const cd ln = logo_new[w], lo = logo[w];
  const double dre = ln.re - lo.re, dim = ln.im - lo.im;
  // S = exp(dre + i dim); I = S exp(xx - bb/2)
  const cd e = red_xx[0] - 0.5 * red_bb[0];
  const double mag = exp(dre + e.re);
  const double cos_theta = cos(dim);
  double wn = w0 * mag * fmax(0.0, cos_theta) * exp(dt * e_shift);
  if (!(wn < INFINITY) || !(ln.re > -INFINITY)) wn = 0.0;
  weights[w] = wn;
  logo[w] = ln;
}

void launch_weights(int NW, int NG, const double* x, const cd* xbar, const cd* logo_new,
                    cd* logo, double* weights, double dt, double e_shift, hipStream_t st) {
  hipLaunchKernelGGL(k_weights, dim3(NW), dim3(256), 0, st, NW, NG, x, xbar, logo_new, logo,
                     weights, dt, e_shift);
}

__global__ void k_frozen_mask(int NW, const double* __restrict__ weights, int* __restrict__ mask) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < NW) mask[w] = weights[w] != 0.0;
}

void launch_frozen_mask(int NW, const double* weights, int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_frozen_mask, dim3((NW + 255) / 256), dim3(256), 0, st, NW, weights, mask);
}

// Plain fill (used instead of a memset node where the work may be captured
// into a graph).
__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_i32(int* p, int n, int v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
}

// Re-orthonormalisation Phi = Q R, diag(R) > 0, by Cholesky QR applied twice
// (Gram matrix, its Cholesky factor, Phi <- Phi R^{-1}); the log-overlap loses
// sum_j log R_jj.  One workgroup per walker and spin; walkers with mask 0 are
// skipped.
__global__ __launch_bounds__(256) void k_qr(cd* __restrict__ phi, int M, int Ntot, int NW, int na,
                                            int nb, const int* __restrict__ mask,
                                            double* __restrict__ ldet_out) {
  const int N = blockIdx.y ? nb : na, col0 = blockIdx.y ? na : 0;
  if (N == 0) return;
  extern __shared__ cd sm[];
  cd* R = sm;            // [N][N]  Gram -> upper Cholesky factor
  cd* Ri = sm + N * N;   // [N][N]  R^{-1}
  __shared__ double ldet;
  __shared__ int bad;
  const int w = blockIdx.x, tid = threadIdx.x, bd = blockDim.x;
  if (mask && mask[w] == 0) return;
  cd* P = phi + (size_t)w * M * Ntot + col0;
  if (tid == 0) {
    ldet = 0.0;
    bad = 0;
  }
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();
    for (int e = tid; e < N * N; e += bd) {
      const int i = e / N, j = e % N;
      cd acc{0.0, 0.0};
      if (i <= j)
        for (int q = 0; q < M; ++q) cfma(acc, conj(P[(size_t)q * Ntot + i]), P[(size_t)q * Ntot + j]);
      R[e] = acc;
      Ri[e] = cd{0.0, 0.0};
    }
    __syncthreads();
    // right-looking Cholesky of the Hermitian Gram matrix, upper factor in place
    for (int j = 0; j < N; ++j) {
      if (tid == 0) {
        const double dj = R[j * N + j].re;
        if (!(dj > 0.0) || !(dj < INFINITY)) bad = 1;
        const double r = sqrt(fmax(dj, 1e-300));
        R[j * N + j] = cd{r, 0.0};
        ldet += log(r);
      }
      __syncthreads();
      const double rinv = 1.0 / R[j * N + j].re;
      for (int c = j + 1 + tid; c < N; c += bd) R[j * N + c] = R[j * N + c] * rinv;
      __syncthreads();
      for (int e = tid; e < (N - j - 1) * (N - j - 1); e += bd) {
        const int r = j + 1 + e / (N - j - 1), c = j + 1 + e % (N - j - 1);
        if (r <= c) R[r * N + c] -= conj(R[j * N + r]) * R[j * N + c];
      }
      __syncthreads();
    }
    // columns of R^{-1}
    for (int c = tid; c < N; c += bd) {
      Ri[c * N + c] = cd{1.0 / R[c * N + c].re, 0.0};
      for (int i = c - 1; i >= 0; --i) {
        cd acc{0.0, 0.0};
        for (int l = i + 1; l <= c; ++l) cfma(acc, R[i * N + l], Ri[l * N + c]);
        Ri[i * N + c] = -acc * (1.0 / R[i * N + i].re);
      }
    }
    __syncthreads();
    for (int q = tid; q < M; q += bd) {
      cd* row = P + (size_t)q * Ntot;
      for (int j = N - 1; j >= 0; --j) {
        cd acc{0.0, 0.0};
        for (int i = 0; i <= j; ++i) cfma(acc, row[i], Ri[i * N + j]);
        row[j] = acc;
      }
    }
    __threadfence();
  }
  __syncthreads();
  if (tid == 0) ldet_out[2 * w + blockIdx.y] = bad ? INFINITY : ldet;
}

// log <Psi_T|Phi> -= sum_s log det R^s after the re-orthonormalisation, and
// log det A^s -= log det R^s (A^s = the reference rows of Phi^s, which become
// A^s (R^s)^-1; T = Phi A^-1 itself is unchanged)
__global__ void k_qr_logo(int NW, const int* __restrict__ mask, const double* __restrict__ ldet,
                          cd* __restrict__ logo, cd* __restrict__ lda, cd* __restrict__ ldb) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= NW || (mask && mask[w] == 0)) return;
  const double l = ldet[2 * w] + ldet[2 * w + 1];
  const cd o = logo[w];
  logo[w] = l < INFINITY ? cd{o.re - l, o.im} : cd{-INFINITY, 0.0};
  if (lda && ldet[2 * w] < INFINITY) lda[w] = cd{lda[w].re - ldet[2 * w], lda[w].im};
  if (ldb && ldet[2 * w + 1] < INFINITY) ldb[w] = cd{ldb[w].re - ldet[2 * w + 1], ldb[w].im};
}

void launch_qr(cd* phi, int M, int Ntot, int NW, int na, int nb, const int* mask, double* ldet,
               cd* logo, cd* logdetA_a, cd* logdetA_b, hipStream_t st) {
  const int N = max(na, nb);
  // one wave for small N (barrier-bound Cholesky steps; at most N*N Gram
  // entries, one row of Phi per lane and pass)
  const int bs = N <= 8 ? 64 : 256;
  hipLaunchKernelGGL(k_qr, dim3(NW, 2), dim3(bs), 2 * (size_t)N * N * sizeof(cd), st, phi, M, Ntot,
                     NW, na, nb, mask, ldet);
  hipLaunchKernelGGL(k_qr_logo, dim3((NW + 255) / 256), dim3(256), 0, st, NW, mask, ldet, logo,
                     logdetA_a, logdetA_b);
}

// Pack the per-spin boundary layouts [w][M][n_s] into the internal [w][M][Ntot]
// walker matrix (to_internal) or back.
__global__ void k_copy_walkers(int NW, int M, int Ntot, int na, int nb, const cd* __restrict__ pa,
                               const cd* __restrict__ pb, cd* __restrict__ phi, int to_internal,
                               cd* __restrict__ oa, cd* __restrict__ ob) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (int64_t)NW * M * Ntot) return;
  const int c = (int)(tid % Ntot);
  const int64_t wq = tid / Ntot;  // w*M + q
  if (to_internal) {
    phi[tid] = c < na ? pa[wq * na + c] : pb[wq * nb + (c - na)];
  } else {
    if (c < na) {
      if (oa) oa[wq * na + c] = phi[tid];
    } else {
      if (ob) ob[wq * nb + (c - na)] = phi[tid];
    }
  }
}

void launch_copy_walkers(int NW, int M, int Ntot, int na, int nb, const cd* pa, const cd* pb,
                         cd* phi, bool to_internal, cd* out_a, cd* out_b, hipStream_t st) {
  const int64_t n = (int64_t)NW * M * Ntot;
  hipLaunchKernelGGL(k_copy_walkers, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, NW, M,
                     Ntot, na, nb, pa, pb, phi, to_internal ? 1 : 0, out_a, out_b);
}

// out[p][q] = sum_g sum_r L^g_pr L^g_rq  (the exchange-like one-body term of Eq. 4)
// Mean-field traces in double precision for the mixed form: v0 = tr Q and
// ex0 = tr QQ of Q^g = L^g[R, :] T, from FP64 tiles [wl][g][N x N] (one wave
// per walker, vector and spin; lanes over the tile's entries).  They overwrite
// the values the single-precision intermediates kernel derived from the FP32 Q.
__global__ __launch_bounds__(64) void k_traces64(const cd* __restrict__ Qa,
                                                 const cd* __restrict__ Qb, int Na, int Nb,
                                                 int NW, int w0, int NG, cd* __restrict__ v0,
                                                 cd* __restrict__ ex0) {
  const int s2 = blockIdx.y, lane = threadIdx.x;
  const int wl = blockIdx.x / NG, g = blockIdx.x % NG;
  const int N = s2 ? Nb : Na;
  const cd* Q = (s2 ? Qb : Qa) + ((size_t)wl * NG + g) * N * N;
  cd v{0.0, 0.0}, x{0.0, 0.0};
  for (int e = lane; e < N * N; e += 64) {
    const int j = e / N, c = e % N;
    const cd q = Q[e];
    if (j == c) v += q;
    cfma(x, q, Q[c * N + j]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.re += __shfl_xor(v.re, off, 64);
    v.im += __shfl_xor(v.im, off, 64);
    x.re += __shfl_xor(x.re, off, 64);
    x.im += __shfl_xor(x.im, off, 64);
  }
  if (lane == 0) {
    v0[((size_t)s2 * NW + w0 + wl) * NG + g] = v;
    ex0[((size_t)s2 * NW + w0 + wl) * NG + g] = x;
  }
}

void launch_traces64(const cd* Qa, const cd* Qb, int Na, int Nb, int NW, int w0, int WT, int NG,
                     cd* v0, cd* ex0, hipStream_t st) {
  hipLaunchKernelGGL(k_traces64, dim3((unsigned)WT * NG, 2), dim3(64), 0, st, Qa, Qb, Na, Nb, NW,
                     w0, NG, v0, ex0);
}

// ---------------------------------------------------------------- block driver
// Population control by the comb (the block of Sec. III.B runs it every five
// steps): with cumulative weights C_i and total W, tooth k sits at
// t_k = (k + z) W / n and walker k of the new population copies the walker i
// with C_{i-1} <= t_k < C_i (a walker of weight 0 owns an empty interval);
// every new weight is W / n.  One workgroup: each thread sums a contiguous
// run of walkers, the run sums are scanned in LDS, and each thread then
// writes the running sums of its run and binary-searches its teeth.  If W is
// 0 nothing changes (parent[k] = k).
constexpr int COMB_THREADS = 1024;

__global__ __launch_bounds__(COMB_THREADS) void k_comb(int NW, double z,
                                                       double* __restrict__ weights,
                                                       double* __restrict__ cum,
                                                       int* __restrict__ parent) {
  __shared__ double part[COMB_THREADS];
  __shared__ int last_pos;
  const int tid = threadIdx.x;
  const int per = (NW + COMB_THREADS - 1) / COMB_THREADS;
  const int b = min(NW, tid * per), e = min(NW, b + per);
  double s = 0.0;
  int last = -1;
  for (int i = b; i < e; ++i) {
    s += weights[i];
    if (weights[i] > 0.0) last = i;
  }
  part[tid] = s;
  if (tid == 0) last_pos = -1;
  __syncthreads();
  if (last >= 0) atomicMax(&last_pos, last);
  for (int off = 1; off < COMB_THREADS; off <<= 1) {  // inclusive scan of run sums
    const double v = tid >= off ? part[tid - off] : 0.0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  double run = tid ? part[tid - 1] : 0.0;
  for (int i = b; i < e; ++i) {
    run += weights[i];
    cum[i] = run;
  }
  __syncthreads();  // running sums and last_pos visible to the workgroup
  const double total = part[COMB_THREADS - 1];
  const bool live = total > 0.0 && last_pos >= 0;
  for (int k = tid; k < NW; k += COMB_THREADS) {
    int p = k;
    if (live) {
      const double t = ((double)k + z) * total / (double)NW;
      int lo = 0, hi = NW;  // first i in [lo, hi) with cum[i] > t, else NW
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] > t) hi = mid;
        else lo = mid + 1;
      }
      p = min(lo, (int)last_pos);  // a tooth rounded onto W: last live walker
    }
    parent[k] = p;
  }
  __syncthreads();  // every read of the old weights is done
  if (live)
    for (int k = tid; k < NW; k += COMB_THREADS) weights[k] = total / (double)NW;
}

// Copies of the parents: phi_out[k] = phi[parent[k]], logo_out[k] = logo[parent[k]].
__global__ void k_comb_gather(int NW, int64_t per_w, const int* __restrict__ parent,
                              const cd* __restrict__ phi, const cd* __restrict__ logo,
                              cd* __restrict__ phi_out, cd* __restrict__ logo_out) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < (int64_t)NW * per_w) {
    const int k = (int)(tid / per_w);
    phi_out[tid] = phi[(int64_t)parent[k] * per_w + tid % per_w];
  }
  if (tid < NW) logo_out[tid] = logo[parent[tid]];
}

void launch_comb(int NW, double z, double* weights, double* cum, int* parent, const cd* phi,
                 const cd* logo, int64_t per_w, cd* phi_out, cd* logo_out, hipStream_t st) {
  hipLaunchKernelGGL(k_comb, dim3(1), dim3(COMB_THREADS), 0, st, NW, z, weights, cum, parent);
  const int64_t n = std::max((int64_t)NW * per_w, (int64_t)NW);
  hipLaunchKernelGGL(k_comb_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, NW,
                     per_w, parent, phi, logo, phi_out, logo_out);
}

// Weighted mixed estimate of a block: out[0] = sum_w w E_L(w), out[1] =
// (sum_w w, 0).  Walkers of weight 0 add nothing (their E_L is not read).
constexpr int BE_THREADS = 256;

__global__ __launch_bounds__(BE_THREADS) void k_block_energy(int NW,
                                                             const double* __restrict__ weights,
                                                             const cd* __restrict__ eloc,
                                                             cd* __restrict__ out) {
  __shared__ cd red[BE_THREADS];
  __shared__ double wred[BE_THREADS];
  const int tid = threadIdx.x;
  cd e{0.0, 0.0};
  double ws = 0.0;
  for (int w = tid; w < NW; w += BE_THREADS) {
    const double x = weights[w];
    if (x > 0.0) {
      e += x * eloc[w];
      ws += x;
    }
  }
  red[tid] = e;
  wred[tid] = ws;
  __syncthreads();
  for (int off = BE_THREADS / 2; off > 0; off >>= 1) {
    if (tid < off) {
      red[tid] += red[tid + off];
      wred[tid] += wred[tid + off];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = red[0];
    out[1] = cd{wred[0], 0.0};
  }
}

void launch_block_energy(int NW, const double* weights, const cd* eloc, cd* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_block_energy, dim3(1), dim3(BE_THREADS), 0, st, NW, weights, eloc, out);
}

}  // namespace msd

namespace msd {
void init_prop_attributes() {
  hipFuncSetAttribute((const void*)k_qr, hipFuncAttributeMaxDynamicSharedMemorySize, 140 * 1024);
}
}  // namespace msd

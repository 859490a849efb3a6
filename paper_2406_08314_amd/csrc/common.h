// Shared definitions for the MSD-AFQMC HIP library (host and device).
#pragma once

#include <stdint.h>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define MSD_HD __host__ __device__ __forceinline__
#else
#define MSD_HD inline
#endif

namespace msd {

constexpr int KMAX = 8;         // holes per spin per determinant (storage stride)
constexpr int NMAX_LDS = 64;    // electrons per spin handled by the LDS kernels

// Interleaved complex number, same memory layout as (re, im) pairs: cd in
// double precision, cf in single precision (mixed-precision intermediates).
template <class R>
struct cx {
  R re, im;
};
using cd = cx<double>;
using cf = cx<float>;

MSD_HD cd mk(double r, double i) { return cd{r, i}; }
template <class R> MSD_HD cx<R> operator+(cx<R> a, cx<R> b) { return cx<R>{a.re + b.re, a.im + b.im}; }
template <class R> MSD_HD cx<R> operator-(cx<R> a, cx<R> b) { return cx<R>{a.re - b.re, a.im - b.im}; }
template <class R> MSD_HD cx<R> operator-(cx<R> a) { return cx<R>{-a.re, -a.im}; }
template <class R> MSD_HD cx<R> operator*(cx<R> a, cx<R> b) {
  return cx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
MSD_HD cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
MSD_HD cd operator*(cd a, double s) { return cd{s * a.re, s * a.im}; }
MSD_HD cf operator*(float s, cf a) { return cf{s * a.re, s * a.im}; }
template <class R> MSD_HD cx<R>& operator+=(cx<R>& a, cx<R> b) { a.re += b.re; a.im += b.im; return a; }
template <class R> MSD_HD cx<R>& operator-=(cx<R>& a, cx<R> b) { a.re -= b.re; a.im -= b.im; return a; }
MSD_HD cd conj(cd a) { return cd{a.re, -a.im}; }
MSD_HD double abs2(cd a) { return a.re * a.re + a.im * a.im; }
// a += b * c (complex fused multiply-add written out)
template <class R> MSD_HD void cfma(cx<R>& a, cx<R> b, cx<R> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
// precision conversions
MSD_HD cd to_cd(cd a) { return a; }
MSD_HD cd to_cd(cf a) { return cd{(double)a.re, (double)a.im}; }
template <class C> MSD_HD C from_cd(cd a);
template <> MSD_HD cd from_cd<cd>(cd a) { return a; }
template <> MSD_HD cf from_cd<cf>(cd a) { return cf{(float)a.re, (float)a.im}; }
MSD_HD cd cdiv(cd a, cd b) {
  // Smith's algorithm for complex division.
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return cd{(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  } else {
    double r = b.re / b.im, den = b.re * r + b.im;
    return cd{(a.re * r + a.im) / den, (a.im * r - a.re) / den};
  }
}

// Number of pairs m < m' among k items, and the lexicographic index of (m, m').
MSD_HD int npairs(int k) { return k * (k - 1) / 2; }
MSD_HD int pair_index(int m, int mp, int k) {
  // pairs ordered (0,1),(0,2),..,(0,k-1),(1,2),..
  return m * (2 * k - m - 1) / 2 + (mp - m - 1);
}

}  // namespace msd

/*
 * Cholesky-vector sums of the generalised-Wick local energy, one determinant
 * at a time -- part of the CPU oracle, TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load
 * this file's library (through oracle/wick.py).  It shares nothing with the
 * HIP library.
 *
 * What it computes (paper Sec. II.A mixed estimator, Sec. III / App. A
 * generalised Wick theorem relative to the reference determinant, Eq. 15):
 * for every determinant I and every Cholesky vector g, per spin s,
 *
 *   a_s(g) = d v0(g) - tr(adj(X) Y(g))
 *   s_s(g) = d (v0(g)^2 - ex0(g)) + 2 tr(adj(X) (Z(g) - v0(g) Y(g))) + 2 e2(X, Y(g))
 *
 * with X the k x k excitation matrix of the spin (d = det X), Y(g) and Z(g)
 * the same entries gathered from Lambda^g and Xi^g, and
 *
 *   e2(X, Y) = sum_{m<m', n<n'} (-1)^{m+m'+n+n'} det X[^{m,m'}, ^{n,n'}]
 *              * (Y_mn Y_m'n' - Y_mn' Y_m'n)
 *
 * (the second-order coefficient of det(X + t Y), by Laplace expansion along
 * the two replaced columns).  The caller passes the signed complementary
 * minors K[A][B] = (-1)^{m+m'+n+n'} det X[^{m,m'}, ^{n,n'}], A running over
 * row pairs (m, m') and B over column pairs (n, n'), each in lexicographic
 * order of the determinant's own order k.  The output per determinant is
 *
 *   out[I] = sum_g [ a_a(g) a_b(g) + 1/2 s_a(g) d_b + 1/2 s_b(g) d_a ],
 *
 * whose c~_I-weighted sum over I, divided by Obar, is the two-body part of
 * E_L.  Plain loops: determinants in parallel (OpenMP), Cholesky vectors in
 * order inside each determinant.
 */
#include <stdint.h>
#include <stdlib.h>

typedef struct {
  double re, im;
} cx;

static inline cx cmul(cx a, cx b) {
  cx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
  return r;
}
static inline cx cadd(cx a, cx b) {
  cx r = {a.re + b.re, a.im + b.im};
  return r;
}
static inline cx csub(cx a, cx b) {
  cx r = {a.re - b.re, a.im - b.im};
  return r;
}
static inline cx cscale(cx a, double s) {
  cx r = {a.re * s, a.im * s};
  return r;
}

/* One spin's inputs.  lam and xi are laid out [row][col][g] (Cholesky vector
 * innermost): row = index into the spin's particle-orbital list, col = slot
 * of a reference orbital. */
typedef struct {
  int32_t kmax;       /* padded excitation order of slot/prow/adj */
  int32_t pmax;       /* kmax (kmax - 1) / 2: padded size of K */
  int32_t n_rows;     /* particle orbitals of this spin (rows of lam, xi) */
  int32_t n_cols;     /* reference orbitals of this spin (columns of lam, xi) */
  const int32_t* k;    /* [n_det] excitation order */
  const int32_t* slot; /* [n_det][kmax] slot of hole m (holes ascending) */
  const int32_t* prow; /* [n_det][kmax] row of particle n (particles ascending) */
  const cx* detx;      /* [n_det] det X */
  const cx* adj;       /* [n_det][kmax][kmax] adj(X)[n][m] */
  const cx* kmin;      /* [n_det][pmax][pmax] K[A][B] */
  const cx* lam;       /* [n_rows][n_cols][n_g] */
  const cx* xi;        /* [n_rows][n_cols][n_g] */
  const cx* v0;        /* [n_g] tr Q^g */
  const cx* ex0;       /* [n_g] tr (Q^g Q^g) */
} spin_in;

/* a_s(g) and s_s(g) of determinant i for every g. */
static void spin_terms(const spin_in* S, int64_t i, int32_t n_g, cx* a, cx* s) {
  const int k = S->k[i];
  const cx d = S->detx[i];
  const int32_t* slot = S->slot + i * S->kmax;
  const int32_t* prow = S->prow + i * S->kmax;
  const cx* adj = S->adj + i * (int64_t)S->kmax * S->kmax;
  const cx* kmin = S->kmin + i * (int64_t)S->pmax * S->pmax;
  const int64_t rs = (int64_t)S->n_cols * n_g; /* stride of a row of lam / xi */
  for (int32_t g = 0; g < n_g; ++g) {
    const cx v0 = S->v0[g];
    /* the reference part of both terms */
    cx tr_y = {0.0, 0.0}, tr_z = {0.0, 0.0};
    for (int m = 0; m < k; ++m)
      for (int n = 0; n < k; ++n) {
        const int64_t off = prow[n] * rs + (int64_t)slot[m] * n_g + g;
        const cx c = adj[n * S->kmax + m];
        tr_y = cadd(tr_y, cmul(c, S->lam[off]));
        tr_z = cadd(tr_z, cmul(c, S->xi[off]));
      }
    /* e2 by Laplace expansion over row pairs A = (m, m') and column pairs
     * B = (n, n'), both lexicographic */
    cx e2 = {0.0, 0.0};
    int A = 0;
    for (int m = 0; m < k; ++m)
      for (int m2 = m + 1; m2 < k; ++m2, ++A) {
        int B = 0;
        for (int n = 0; n < k; ++n)
          for (int n2 = n + 1; n2 < k; ++n2, ++B) {
            const cx y_mn = S->lam[prow[n] * rs + (int64_t)slot[m] * n_g + g];
            const cx y_m2n2 = S->lam[prow[n2] * rs + (int64_t)slot[m2] * n_g + g];
            const cx y_mn2 = S->lam[prow[n2] * rs + (int64_t)slot[m] * n_g + g];
            const cx y_m2n = S->lam[prow[n] * rs + (int64_t)slot[m2] * n_g + g];
            const cx minor2 = csub(cmul(y_mn, y_m2n2), cmul(y_mn2, y_m2n));
            e2 = cadd(e2, cmul(kmin[A * S->pmax + B], minor2));
          }
      }
    a[g] = csub(cmul(d, v0), tr_y);
    const cx mf = csub(cmul(v0, v0), S->ex0[g]);
    s[g] = cadd(cadd(cmul(d, mf), cscale(csub(tr_z, cmul(v0, tr_y)), 2.0)), cscale(e2, 2.0));
  }
}

/* out[i] = sum_g [a_a a_b + 1/2 s_a d_b + 1/2 s_b d_a] for i in [0, n_det). */
void wick_gamma_sums(int64_t n_det, int32_t n_g, const spin_in* sa, const spin_in* sb,
                     double* out) {
  cx* res = (cx*)out;
#pragma omp parallel
  {
    cx* buf = (cx*)malloc(sizeof(cx) * 4 * (size_t)(n_g > 0 ? n_g : 1));
    cx *aa = buf, *as = buf + n_g, *ba = buf + 2 * n_g, *bs = buf + 3 * n_g;
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_det; ++i) {
      spin_terms(sa, i, n_g, aa, as);
      spin_terms(sb, i, n_g, ba, bs);
      const cx da = sa->detx[i], db = sb->detx[i];
      cx acc = {0.0, 0.0};
      for (int32_t g = 0; g < n_g; ++g) {
        acc = cadd(acc, cmul(aa[g], ba[g]));
        acc = cadd(acc, cscale(cmul(as[g], db), 0.5));
        acc = cadd(acc, cscale(cmul(bs[g], da), 0.5));
      }
      res[i] = acc;
    }
    free(buf);
  }
}

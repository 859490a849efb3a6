// Host-side trial builder: turns a CI expansion (coefficients + occupation
// lists, Eq. 15) into the excitation tables the Wick kernels consume.
//
// Every determinant I is an excitation of the reference R (row 0) per spin:
// holes H_I = R \ S_I and particles P_I = S_I \ R, both ascending.  With
// X_mn = T[p_n, slot(h_m)] (T = Phi A^{-1}, A = Phi[R, :]),
//   <D_I|Phi> / <D_R|Phi> = sgn_I det X  (per spin),
// where sgn_I is the sign of the permutation that sorts the reference slot
// list with h_m replaced by p_m.  Determinants are factored into per-spin
// "strings" (distinct occupied sets) so that per-string quantities (det X,
// adj X, second-order minors) are evaluated once per walker.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "common.h"

namespace msd {

struct SpinTable {
  int N = 0;                      // electrons of this spin
  std::vector<int> ref;           // reference orbitals, ascending (size N)
  std::vector<int> occ_act;       // orbitals that are holes in some string, ascending
  std::vector<int> vir_act;       // orbitals that are particles in some string, ascending
  std::vector<int> occ_slot;      // slot in ref of each occ_act orbital
  int U = 0;                      // distinct strings (index 0 is the reference string)
  std::vector<int> k;             // [U] excitation order
  std::vector<int> hslot;         // [U*KMAX] slot in ref of hole m
  std::vector<int> hwin;          // [U*KMAX] index of hole m in occ_act
  std::vector<int> part;          // [U*KMAX] particle orbital n
  std::vector<int> pwin;          // [U*KMAX] index of particle n in vir_act
  std::vector<int> sign;          // [U] excitation sign
  std::vector<int> adj_off;       // [U+1] prefix sums of k^2
  std::vector<int> m2_off;        // [U+1] prefix sums of C(k,2)^2
  std::vector<int> bucket;        // [KMAX+2] strings are sorted by k: [bucket[k], bucket[k+1])
  // string -> determinants containing it (CSR)
  std::vector<int> bw_ptr;        // [U+1]
  std::vector<int> bw_det;        // determinant ids
  std::vector<int> seg_ptr;       // each string's list cut into segments of <= 16 ids
  std::vector<int> str_seg;       // [U+1] segment range of each string
  // first-order CI matrix entry (a, i) (a in vir_act, i in occ_act) -> (adj index, string)
  std::vector<int> c_ptr;         // [nv*no + 1]
  std::vector<int> c_adj;         // flat index into the walker's adj array
  std::vector<int> c_str;         // string id
  // same-spin second-order minors (a < b in vir_act, i < j in occ_act)
  int n_minor = 0;
  std::vector<int> mn_idx;        // [n_minor*4] window entries (a,i), (b,j), (a,j), (b,i)
  std::vector<int> mn_ptr;        // [n_minor + 1]
  std::vector<int> mn_str;        // contributing string
  std::vector<int> mn_m2;         // flat index into the walker's minor array
  std::vector<int> mn_sgn;        // (-1)^(m+m'+n+n')
  int nv() const { return (int)vir_act.size(); }
  int no() const { return (int)occ_act.size(); }
};

struct TrialTables {
  int M = 0;
  int64_t n_det = 0;
  SpinTable s[2];
  std::vector<int> det_s[2];      // [n_det] string id per spin
  std::vector<double> det_c;      // [2*n_det] conj(c_I) * sgn_a * sgn_b (interleaved)
  // opposite-spin pairs x = (a,i) alpha window entry, y = (b,j) beta window entry
  int n_pair = 0;
  std::vector<int> pr_x, pr_y;    // [n_pair]
  std::vector<int64_t> pr_ptr;    // [n_pair + 1]
  std::vector<int> pr_det;        // contributing determinant
  std::vector<int> pr_fa, pr_fb;  // flat adj indices (alpha, beta)
  int max_k() const;
};

// Builds the tables.  Returns an empty string on success, otherwise a message
// naming the offending determinant (the caller maps it to MSD_ERR_TRIAL).
std::string build_trial(int M, int na, int nb, int64_t n_det, const double* ci,
                        const int32_t* occ_a, const int32_t* occ_b, TrialTables* out);

// Excitation order and sign of every determinant (no tables).
std::string analyze_trial(int M, int na, int nb, int64_t n_det, const int32_t* occ_a,
                          const int32_t* occ_b, int32_t* k_a, int32_t* k_b, int32_t* sign);

}  // namespace msd

// Host-side trial builder (pure C++; no device code).  See trial.h.
#include "trial.h"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <unordered_map>

namespace msd {

namespace {

struct StringKey {
  // holes then particles, each ascending; k = holes.size()
  std::vector<int> v;
  bool operator==(const StringKey& o) const { return v == o.v; }
};
struct StringKeyHash {
  size_t operator()(const StringKey& s) const {
    uint64_t h = 1469598103934665603ull;
    for (int x : s.v) {
      h ^= (uint64_t)(uint32_t)x + 0x9e3779b97f4a7c15ull;
      h *= 1099511628211ull;
    }
    return (size_t)h;
  }
};

// Sorts one occupation row into `sorted`; returns "" or an error message.
std::string read_row(const int32_t* row, int N, int M, int64_t det, const char* spin,
                     std::vector<int>& sorted) {
  sorted.assign(row, row + N);
  for (int j = 0; j < N; ++j) {
    if (sorted[j] < 0 || sorted[j] >= M)
      return "determinant " + std::to_string(det) + ": " + spin + " orbital " +
             std::to_string(sorted[j]) + " outside [0, M)";
  }
  std::sort(sorted.begin(), sorted.end());
  for (int j = 1; j < N; ++j)
    if (sorted[j] == sorted[j - 1])
      return "determinant " + std::to_string(det) + ": " + spin + " orbital " +
             std::to_string(sorted[j]) + " repeated";
  return "";
}

// Holes (ref \ occ) and particles (occ \ ref), both ascending, for sorted lists.
void excitation(const std::vector<int>& ref, const std::vector<int>& occ, std::vector<int>& holes,
                std::vector<int>& parts) {
  holes.clear();
  parts.clear();
  size_t i = 0, j = 0;
  while (i < ref.size() || j < occ.size()) {
    if (j == occ.size() || (i < ref.size() && ref[i] < occ[j])) {
      holes.push_back(ref[i++]);
    } else if (i == ref.size() || occ[j] < ref[i]) {
      parts.push_back(occ[j++]);
    } else {
      ++i;
      ++j;
    }
  }
}

// Sign of the permutation sorting ref with holes[m] replaced by parts[m]:
// each replaced entry p_m crosses exactly the kept reference orbitals lying
// strictly between h_m and p_m; replaced entries never cross each other
// because both lists are ascending.
int excitation_sign(const std::vector<int>& ref, const std::vector<int>& holes,
                    const std::vector<int>& parts) {
  long cross = 0;
  for (size_t m = 0; m < holes.size(); ++m) {
    int lo = std::min(holes[m], parts[m]), hi = std::max(holes[m], parts[m]);
    auto b = std::upper_bound(ref.begin(), ref.end(), lo);
    auto e = std::lower_bound(ref.begin(), ref.end(), hi);
    long between = e - b;
    for (int h : holes)
      if (h > lo && h < hi) --between;
    cross += between;
  }
  return (cross & 1) ? -1 : 1;
}

}  // namespace

int TrialTables::max_k() const {
  int k = 0;
  for (int s2 = 0; s2 < 2; ++s2)
    for (int x : s[s2].k) k = std::max(k, x);
  return k;
}

std::string analyze_trial(int M, int na, int nb, int64_t n_det, const int32_t* occ_a,
                          const int32_t* occ_b, int32_t* k_a, int32_t* k_b, int32_t* sign) {
  if (n_det < 1) return "n_det must be at least 1";
  std::vector<int> ref[2], row, holes, parts;
  const int32_t* occ[2] = {occ_a, occ_b};
  int nel[2] = {na, nb};
  const char* nm[2] = {"alpha", "beta"};
  for (int sp = 0; sp < 2; ++sp) {
    std::string e = read_row(occ[sp], nel[sp], M, 0, nm[sp], ref[sp]);
    if (!e.empty()) return e;
  }
  for (int64_t I = 0; I < n_det; ++I) {
    int sg = 1;
    for (int sp = 0; sp < 2; ++sp) {
      std::string e = read_row(occ[sp] + I * nel[sp], nel[sp], M, I, nm[sp], row);
      if (!e.empty()) return e;
      excitation(ref[sp], row, holes, parts);
      if ((int)holes.size() > KMAX)
        return "determinant " + std::to_string(I) + ": " + nm[sp] + " excitation order " +
               std::to_string(holes.size()) + " exceeds " + std::to_string(KMAX);
      sg *= excitation_sign(ref[sp], holes, parts);
      (sp == 0 ? k_a : k_b)[I] = (int32_t)holes.size();
    }
    sign[I] = sg;
  }
  return "";
}

std::string build_trial(int M, int na, int nb, int64_t n_det, const double* ci,
                        const int32_t* occ_a, const int32_t* occ_b, TrialTables* out) {
  if (n_det < 1) return "n_det must be at least 1";
  if (n_det > (int64_t)INT32_MAX) return "n_det exceeds 2^31-1";
  TrialTables& t = *out;
  t = TrialTables();
  t.M = M;
  t.n_det = n_det;
  const int32_t* occ[2] = {occ_a, occ_b};
  int nel[2] = {na, nb};
  const char* nm[2] = {"alpha", "beta"};
  std::vector<int> row, holes, parts;
  std::vector<int> det_sign(n_det, 1);

  for (int sp = 0; sp < 2; ++sp) {
    SpinTable& S = t.s[sp];
    S.N = nel[sp];
    std::string e = read_row(occ[sp], S.N, M, 0, nm[sp], S.ref);
    if (!e.empty()) return e;
    std::unordered_map<StringKey, int, StringKeyHash> ids;
    std::vector<StringKey> keys;
    std::vector<int> first_sign;
    t.det_s[sp].resize(n_det);
    StringKey key;
    for (int64_t I = 0; I < n_det; ++I) {
      e = read_row(occ[sp] + I * S.N, S.N, M, I, nm[sp], row);
      if (!e.empty()) return e;
      excitation(S.ref, row, holes, parts);
      if ((int)holes.size() > KMAX)
        return "determinant " + std::to_string(I) + ": " + nm[sp] + " excitation order " +
               std::to_string(holes.size()) + " exceeds " + std::to_string(KMAX);
      key.v.assign(holes.begin(), holes.end());
      key.v.insert(key.v.end(), parts.begin(), parts.end());
      auto it = ids.find(key);
      int id;
      if (it == ids.end()) {
        id = (int)keys.size();
        ids.emplace(key, id);
        keys.push_back(key);
        first_sign.push_back(excitation_sign(S.ref, holes, parts));
      } else {
        id = it->second;
      }
      t.det_s[sp][I] = id;
      det_sign[I] *= first_sign[id];
    }
    // order strings by excitation order (the reference string, k = 0, first)
    int U = (int)keys.size();
    std::vector<int> order(U);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return keys[a].v.size() < keys[b].v.size();
    });
    std::vector<int> newid(U);
    for (int i = 0; i < U; ++i) newid[order[i]] = i;
    for (int64_t I = 0; I < n_det; ++I) t.det_s[sp][I] = newid[t.det_s[sp][I]];
    S.U = U;
    S.k.resize(U);
    S.sign.resize(U);
    S.hslot.assign((size_t)U * KMAX, 0);
    S.hwin.assign((size_t)U * KMAX, 0);
    S.part.assign((size_t)U * KMAX, 0);
    S.pwin.assign((size_t)U * KMAX, 0);
    std::vector<char> is_hole(M, 0), is_part(M, 0);
    for (int i = 0; i < U; ++i) {
      const StringKey& kk = keys[order[i]];
      int k = (int)kk.v.size() / 2;
      S.k[i] = k;
      S.sign[i] = first_sign[order[i]];
      for (int m = 0; m < k; ++m) {
        is_hole[kk.v[m]] = 1;
        is_part[kk.v[k + m]] = 1;
      }
    }
    std::vector<int> hwin_of(M, -1), pwin_of(M, -1), slot_of(M, -1);
    for (int j = 0; j < S.N; ++j) slot_of[S.ref[j]] = j;
    for (int p = 0; p < M; ++p) {
      if (is_hole[p]) {
        hwin_of[p] = (int)S.occ_act.size();
        S.occ_act.push_back(p);
        S.occ_slot.push_back(slot_of[p]);
      }
      if (is_part[p]) {
        pwin_of[p] = (int)S.vir_act.size();
        S.vir_act.push_back(p);
      }
    }
    for (int i = 0; i < U; ++i) {
      const StringKey& kk = keys[order[i]];
      int k = S.k[i];
      for (int m = 0; m < k; ++m) {
        int h = kk.v[m], p = kk.v[k + m];
        S.hslot[(size_t)i * KMAX + m] = slot_of[h];
        S.hwin[(size_t)i * KMAX + m] = hwin_of[h];
        S.part[(size_t)i * KMAX + m] = p;
        S.pwin[(size_t)i * KMAX + m] = pwin_of[p];
      }
    }
    S.bucket.assign(KMAX + 2, U);
    for (int i = U - 1; i >= 0; --i) S.bucket[S.k[i]] = i;
    for (int k = KMAX; k >= 0; --k)
      if (S.bucket[k] > S.bucket[k + 1]) S.bucket[k] = S.bucket[k + 1];
    S.adj_off.assign(U + 1, 0);
    S.m2_off.assign(U + 1, 0);
    for (int i = 0; i < U; ++i) {
      int k = S.k[i], p = npairs(k);
      S.adj_off[i + 1] = S.adj_off[i] + k * k;
      S.m2_off[i + 1] = S.m2_off[i] + p * p;
    }
    if (S.adj_off[U] < 0 || S.m2_off[U] < 0) return "trial tables exceed 2^31 entries";
  }
  if (t.s[0].k[t.det_s[0][0]] != 0 || t.s[1].k[t.det_s[1][0]] != 0)
    return "internal: determinant 0 must be the reference";

  // folded coefficients conj(c_I) * sgn
  t.det_c.resize(2 * n_det);
  for (int64_t I = 0; I < n_det; ++I) {
    t.det_c[2 * I] = ci[2 * I] * det_sign[I];
    t.det_c[2 * I + 1] = -ci[2 * I + 1] * det_sign[I];
  }

  for (int sp = 0; sp < 2; ++sp) {
    SpinTable& S = t.s[sp];
    const int U = S.U, nv = S.nv(), no = S.no();
    // string -> determinants
    S.bw_ptr.assign(U + 1, 0);
    for (int64_t I = 0; I < n_det; ++I) S.bw_ptr[t.det_s[sp][I] + 1]++;
    for (int i = 0; i < U; ++i) S.bw_ptr[i + 1] += S.bw_ptr[i];
    S.bw_det.resize(n_det);
    {
      std::vector<int> fill(S.bw_ptr.begin(), S.bw_ptr.end() - 1);
      for (int64_t I = 0; I < n_det; ++I) S.bw_det[fill[t.det_s[sp][I]]++] = (int)I;
    }
    // segments of at most 16 determinants (balanced CI-weight sums)
    S.str_seg.assign(U + 1, 0);
    S.seg_ptr.assign(1, 0);
    for (int i = 0; i < U; ++i) {
      for (int b = S.bw_ptr[i]; b < S.bw_ptr[i + 1]; b += 16)
        S.seg_ptr.push_back(std::min(b + 16, S.bw_ptr[i + 1]));
      S.str_seg[i + 1] = (int)S.seg_ptr.size() - 1;
    }
    // first-order CI entries
    S.c_ptr.assign((size_t)nv * no + 1, 0);
    for (int i = 0; i < U; ++i) {
      int k = S.k[i];
      for (int n = 0; n < k; ++n)
        for (int m = 0; m < k; ++m)
          S.c_ptr[(size_t)S.pwin[(size_t)i * KMAX + n] * no + S.hwin[(size_t)i * KMAX + m] + 1]++;
    }
    for (size_t e = 0; e < (size_t)nv * no; ++e) S.c_ptr[e + 1] += S.c_ptr[e];
    S.c_adj.resize(S.c_ptr.back());
    S.c_str.resize(S.c_ptr.back());
    {
      std::vector<int> fill(S.c_ptr.begin(), S.c_ptr.end() - 1);
      for (int i = 0; i < U; ++i) {
        int k = S.k[i];
        for (int n = 0; n < k; ++n)
          for (int m = 0; m < k; ++m) {
            size_t e = (size_t)S.pwin[(size_t)i * KMAX + n] * no + S.hwin[(size_t)i * KMAX + m];
            int pos = fill[e]++;
            S.c_adj[pos] = S.adj_off[i] + n * k + m;
            S.c_str[pos] = i;
          }
      }
    }
    // same-spin minors
    std::unordered_map<int64_t, int> mid;
    std::vector<int> cnt;
    std::vector<int64_t> mkey;
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int> fill;
      if (pass == 1) {
        S.n_minor = (int)cnt.size();
        S.mn_ptr.assign(S.n_minor + 1, 0);
        for (int q = 0; q < S.n_minor; ++q) S.mn_ptr[q + 1] = S.mn_ptr[q] + cnt[q];
        S.mn_str.resize(S.mn_ptr.back());
        S.mn_m2.resize(S.mn_ptr.back());
        S.mn_sgn.resize(S.mn_ptr.back());
        fill.assign(S.mn_ptr.begin(), S.mn_ptr.end() - 1);
        S.mn_idx.resize((size_t)S.n_minor * 4);
        for (int q = 0; q < S.n_minor; ++q) {
          int64_t key = mkey[q];
          int j = (int)(key % no);
          key /= no;
          int i2 = (int)(key % no);
          key /= no;
          int b = (int)(key % nv);
          int a = (int)(key / nv);
          S.mn_idx[4 * q + 0] = a * no + i2;
          S.mn_idx[4 * q + 1] = b * no + j;
          S.mn_idx[4 * q + 2] = a * no + j;
          S.mn_idx[4 * q + 3] = b * no + i2;
        }
      }
      for (int s2 = 0; s2 < U; ++s2) {
        int k = S.k[s2];
        if (k < 2) continue;
        int P = npairs(k);
        const int* pw = &S.pwin[(size_t)s2 * KMAX];
        const int* hw = &S.hwin[(size_t)s2 * KMAX];
        for (int m = 0; m < k; ++m)
          for (int mp = m + 1; mp < k; ++mp)
            for (int n = 0; n < k; ++n)
              for (int np = n + 1; np < k; ++np) {
                int64_t key = (((int64_t)pw[n] * nv + pw[np]) * no + hw[m]) * no + hw[mp];
                if (pass == 0) {
                  auto it = mid.find(key);
                  if (it == mid.end()) {
                    mid.emplace(key, (int)cnt.size());
                    cnt.push_back(1);
                    mkey.push_back(key);
                  } else {
                    cnt[it->second]++;
                  }
                } else {
                  int q = mid[key];
                  int pos = fill[q]++;
                  S.mn_str[pos] = s2;
                  S.mn_m2[pos] = S.m2_off[s2] + pair_index(m, mp, k) * P + pair_index(n, np, k);
                  S.mn_sgn[pos] = ((m + mp + n + np) & 1) ? -1 : 1;
                }
              }
      }
    }
  }

  // opposite-spin pairs
  {
    const SpinTable& A = t.s[0];
    const SpinTable& B = t.s[1];
    const int64_t xa = (int64_t)A.nv() * A.no(), xb = (int64_t)B.nv() * B.no();
    std::unordered_map<int64_t, int> pid;
    std::vector<int64_t> cnt;
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int64_t> fill;
      if (pass == 1) {
        // pairs in (x, y) order: lanes of the second-order kernel then gather
        // neighbouring (often equal) alpha entries, fewer LDS bank conflicts
        const int np = (int)cnt.size();
        std::vector<int> order(np), rank(np);
        for (int q = 0; q < np; ++q) order[q] = q;
        std::sort(order.begin(), order.end(), [&](int a, int b) {
          return t.pr_x[a] != t.pr_x[b] ? t.pr_x[a] < t.pr_x[b] : t.pr_y[a] < t.pr_y[b];
        });
        std::vector<int> px(np), py(np);
        std::vector<int64_t> pc(np);
        for (int q = 0; q < np; ++q) {
          rank[order[q]] = q;
          px[q] = t.pr_x[order[q]];
          py[q] = t.pr_y[order[q]];
          pc[q] = cnt[order[q]];
        }
        t.pr_x.swap(px);
        t.pr_y.swap(py);
        cnt.swap(pc);
        for (auto& kv : pid) kv.second = rank[kv.second];
        t.n_pair = (int)cnt.size();
        t.pr_ptr.assign(t.n_pair + 1, 0);
        for (int q = 0; q < t.n_pair; ++q) t.pr_ptr[q + 1] = t.pr_ptr[q] + cnt[q];
        t.pr_det.resize(t.pr_ptr.back());
        t.pr_fa.resize(t.pr_ptr.back());
        t.pr_fb.resize(t.pr_ptr.back());
        fill.assign(t.pr_ptr.begin(), t.pr_ptr.end() - 1);
      }
      for (int64_t I = 0; I < n_det; ++I) {
        int sa = t.det_s[0][I], sb = t.det_s[1][I];
        int ka = A.k[sa], kb = B.k[sb];
        if (ka == 0 || kb == 0) continue;
        for (int n = 0; n < ka; ++n)
          for (int m = 0; m < ka; ++m) {
            int64_t x = (int64_t)A.pwin[(size_t)sa * KMAX + n] * A.no() + A.hwin[(size_t)sa * KMAX + m];
            for (int n2 = 0; n2 < kb; ++n2)
              for (int m2 = 0; m2 < kb; ++m2) {
                int64_t y = (int64_t)B.pwin[(size_t)sb * KMAX + n2] * B.no() +
                            B.hwin[(size_t)sb * KMAX + m2];
                int64_t key = x * xb + y;
                if (pass == 0) {
                  auto it = pid.find(key);
                  if (it == pid.end()) {
                    pid.emplace(key, (int)cnt.size());
                    cnt.push_back(1);
                    t.pr_x.push_back((int)x);
                    t.pr_y.push_back((int)y);
                  } else {
                    cnt[it->second]++;
                  }
                } else {
                  int q = pid[key];
                  int64_t pos = fill[q]++;
                  t.pr_det[pos] = (int)I;
                  t.pr_fa[pos] = A.adj_off[sa] + n * ka + m;
                  t.pr_fb[pos] = B.adj_off[sb] + n2 * kb + m2;
                }
              }
          }
      }
    }
    (void)xa;
  }
  return "";
}

}  // namespace msd

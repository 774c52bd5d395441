// Host-side analysis for slr_setup (see slr_host.h).
//
// Paper: Li, Xi & Saad, "Schur complement based domain decomposition
// preconditioners with low-rank corrections" (2015).
//   Sec. 2.1  vertex-based partitioning: interior vs. local interface nodes
//   eq. Global / Global2  DD ordering [u_1..u_p ; y]
//   Sec. 5.2  local solves with B_i and with C
#include "slr_host.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <iterator>
#include <numeric>
#include <set>
#include <thread>

#include "slr.h"

namespace slr {

bool is_symmetric(int64_t n, const int64_t *rp, const int32_t *ci, const double *v) {
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      int64_t j = ci[e];
      if (j < 0 || j >= n) return false;
      const int32_t *b = ci + rp[j], *en = ci + rp[j + 1];
      const int32_t *f = std::lower_bound(b, en, (int32_t)i);
      if (f == en || *f != i) return false;
      if (v[rp[j] + (f - b)] != v[e]) return false;
    }
  }
  return true;
}

namespace {

// Build a level-scheduled sweep from per-row dependency lists.
// deps(i) lists the rows whose solved values row i needs; `order` is the
// elimination order (row indices in the order a sequential solve visits).
template <class Deps, class Emit>
void schedule(int32_t nrows, const std::vector<int32_t> &order, Deps deps, Emit emit, Sweep &sw) {
  std::vector<int32_t> lev(nrows, 0);
  int32_t nlev = 0;
  for (int32_t i : order) {
    int32_t l = 0;
    deps(i, [&](int32_t j) { l = std::max(l, lev[j] + 1); });
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  if (nrows == 0) nlev = 0;
  sw.nrows = nrows;
  sw.nlev = nlev;
  sw.levptr.assign(nlev + 1, 0);
  for (int32_t i = 0; i < nrows; ++i) sw.levptr[lev[i] + 1]++;
  for (int32_t l = 0; l < nlev; ++l) sw.levptr[l + 1] += sw.levptr[l];
  // stable within a level: ascending elimination position
  std::vector<int32_t> pos(sw.levptr.begin(), sw.levptr.end() - (nlev ? 1 : 0));
  sw.rows.assign(nrows, 0);
  for (int32_t i : order) sw.rows[pos[lev[i]]++] = i;
  sw.rp.assign(nrows + 1, 0);
  sw.ci.clear();
  sw.w.clear();
  sw.w_e.clear();
  sw.sc.assign(nrows, 0.0);
  sw.sc_e.assign(nrows, 0);
  for (int32_t t = 0; t < nrows; ++t) {
    int32_t i = sw.rows[t];
    emit(i, sw.sc[t], sw.sc_e[t], [&](int32_t j, double w, int32_t src) {
      sw.ci.push_back(j);
      sw.w.push_back(w);
      sw.w_e.push_back(src);
    });
    sw.rp[t + 1] = (int32_t)sw.ci.size();
  }
}

inline double r32(double x) { return (double)(float)x; }

// Forward and backward sweeps of a lower factor.
//   L L^T :  fwd  x_i = b_i / l_ii - sum_j (l_ij / l_ii) x_j
//            bwd  x_i = b_i / l_ii - sum_t (l_ti / l_ii) x_t
//   L D L^T (unit L): fwd  x_i = b_i - sum_j l_ij x_j
//                     bwd  x_i = b_i / d_i - sum_t l_ti x_t
// With fp32 storage the factor values are rounded to FP32 first and the
// stored coefficients are rounded again after the division.
void build_sweeps(const LowerFactor &F, bool fp32, Sweep &fwd, Sweep &bwd) {
  const int32_t n = F.n;
  std::vector<double> v = F.v;
  if (fp32)
    for (double &x : v) x = r32(x);
  auto rd = [&](double x) { return fp32 ? r32(x) : x; };
  const bool ldl = F.kind == 2;
  auto diag = [&](int32_t i) { return v[F.rp[i + 1] - 1]; };
  // transpose (strictly lower part) for the backward sweep
  std::vector<int32_t> tp(n + 1, 0), tj, te;
  std::vector<double> tv;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = F.rp[i]; e < F.rp[i + 1] - 1; ++e) tp[F.ci[e] + 1]++;
  for (int32_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
  tj.resize(tp[n]);
  tv.resize(tp[n]);
  te.resize(tp[n]);
  {
    std::vector<int32_t> fill(tp.begin(), tp.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t e = F.rp[i]; e < F.rp[i + 1] - 1; ++e) {
        int32_t c = F.ci[e];
        tj[fill[c]] = i;
        te[fill[c]] = e;
        tv[fill[c]++] = v[e];
      }
  }
  std::vector<int32_t> up(n), down(n);
  std::iota(up.begin(), up.end(), 0);
  for (int32_t i = 0; i < n; ++i) down[i] = n - 1 - i;
  schedule(
      n, up,
      [&](int32_t i, auto f) {
        for (int32_t e = F.rp[i]; e < F.rp[i + 1] - 1; ++e) f(F.ci[e]);
      },
      [&](int32_t i, double &sc, int32_t &sce, auto put) {
        double d = diag(i);
        sc = ldl ? 1.0 : rd(1.0 / d);
        sce = F.rp[i + 1] - 1;
        for (int32_t e = F.rp[i]; e < F.rp[i + 1] - 1; ++e)
          put(F.ci[e], ldl ? v[e] : rd(v[e] / d), e);
      },
      fwd);
  fwd.divided = !ldl;
  fwd.unit_sc = ldl;
  schedule(
      n, down,
      [&](int32_t i, auto f) {
        for (int32_t e = tp[i]; e < tp[i + 1]; ++e) f(tj[e]);
      },
      [&](int32_t i, double &sc, int32_t &sce, auto put) {
        double d = diag(i);
        sc = rd(1.0 / d);
        sce = F.rp[i + 1] - 1;
        for (int32_t e = tp[i]; e < tp[i + 1]; ++e) put(tj[e], ldl ? tv[e] : rd(tv[e] / d), te[e]);
      },
      bwd);
  bwd.divided = !ldl;
  bwd.unit_sc = false;
}

// Zero-fill incomplete factorisation on the pattern of tril(M) (Sec. 5.2 /
// Sec. 6 local solvers restricted to no fill).  The row being built is
// scattered into a dense work array; row j's entries are walked against it.
//   IC(0):    l_ij = (m_ij - sum_{k<j} l_ik l_jk) / l_jj,  l_ii = sqrt(m_ii - sum l_ik^2)
//   ILDL(0):  l_ij = (m_ij - sum_{k<j} l_ik d_k l_jk) / d_j, d_i = m_ii - sum l_ik^2 d_k
// Returns -1 - i on a failed pivot of row i, else 0.
int incomplete_factor(LowerFactor &F) {
  const int32_t n = F.n;
  const bool ldl = F.kind == 2;
  std::vector<double> dense(n, 0.0), d(n, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    int32_t a = F.rp[i], b = F.rp[i + 1] - 1;
    if (b < a || F.ci[b] != i) return -1 - i;
    double acc_d = 0.0;
    for (int32_t e = a; e < b; ++e) {
      int32_t j = F.ci[e];
      double s = 0.0;
      for (int32_t t = F.rp[j]; t < F.rp[j + 1] - 1; ++t) {
        int32_t k = F.ci[t];
        s += ldl ? dense[k] * F.v[t] * d[k] : dense[k] * F.v[t];
      }
      double pj = ldl ? d[j] : F.v[F.rp[j + 1] - 1];
      double l = (F.v[e] - s) / pj;
      F.v[e] = l;
      dense[j] = l;
      acc_d += ldl ? l * l * d[j] : l * l;
    }
    double piv = F.v[b] - acc_d;
    for (int32_t e = a; e < b; ++e) dense[F.ci[e]] = 0.0;
    if (ldl) {
      if (!(std::fabs(piv) >= 1e-300)) return -1 - i;
      d[i] = piv;
      F.v[b] = piv;
    } else {
      if (!(piv > 0.0)) return -1 - i;
      F.v[b] = std::sqrt(piv);
    }
  }
  return 0;
}

// Exact Cholesky in envelope (profile) storage: row i of L spans columns
// [first_i, i]; fill stays inside the envelope.
int envelope_cholesky(int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                      const std::vector<double> &v, LowerFactor &F) {
  std::vector<int32_t> first(n);
  std::vector<int64_t> start(n + 1, 0);
  for (int32_t i = 0; i < n; ++i) {
    first[i] = (rp[i + 1] > rp[i]) ? std::min(ci[rp[i]], i) : i;
    start[i + 1] = start[i] + (i - first[i] + 1);
  }
  std::vector<double> L(start[n], 0.0);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) L[start[i] + ci[e] - first[i]] = v[e];
  for (int32_t i = 0; i < n; ++i) {
    double *Li = &L[start[i]];
    for (int32_t j = first[i]; j <= i; ++j) {
      const double *Lj = &L[start[j]];
      int32_t k0 = std::max(first[i], first[j]);
      double s = Li[j - first[i]];
      for (int32_t k = k0; k < j; ++k) s -= Li[k - first[i]] * Lj[k - first[j]];
      if (j < i) {
        Li[j - first[i]] = s / Lj[j - first[j]];
      } else {
        if (!(s > 0.0)) return -1 - i;
        Li[i - first[i]] = std::sqrt(s);
      }
    }
  }
  F.n = n;
  F.kind = 0;
  F.rp.assign(n + 1, 0);
  F.ci.clear();
  F.v.clear();
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t j = first[i]; j <= i; ++j) {
      F.ci.push_back(j);
      F.v.push_back(L[start[i] + j - first[i]]);
    }
    F.rp[i + 1] = (int32_t)F.ci.size();
  }
  return 0;
}

// Threshold factorisation (ICT, or ILDLT when ldl), left-looking by
// columns.  Column j starts from column j of tril(M) (w_i = m_ij, i >= j;
// nrm = sum |m_ij|); each earlier column k with a kept l_jk (ascending k)
// subtracts l_ik f from w_i for its kept rows i >= j, f = l_jk (IC) or
// l_jk d_k (LDL); then l_jj = sqrt(w_j) (or d_j = w_j) and, for i > j in
// ascending order, l_ij = w_i / l_jj (or / d_j) is kept when |w_i| >= tau
// nrm.  The result is returned as row CSR with the diagonal last.
int threshold_factor(bool ldl, int32_t n, const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                     const std::vector<double> &v, double tau, LowerFactor &F) {
  // columns of tril(M)
  std::vector<int32_t> cptr(n + 1, 0), crow(ci.size());
  std::vector<double> cval(ci.size());
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) cptr[ci[e] + 1]++;
  for (int32_t j = 0; j < n; ++j) cptr[j + 1] += cptr[j];
  {
    std::vector<int32_t> pos(cptr.begin(), cptr.end() - 1);
    for (int32_t i = 0; i < n; ++i)
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        crow[pos[ci[e]]] = i;
        cval[pos[ci[e]]++] = v[e];
      }
  }
  // kept entries by column (rows ascending) and by row (columns ascending)
  std::vector<std::vector<std::pair<int32_t, double>>> col(n), row(n);
  std::vector<double> dg(n, 0.0), w(n, 0.0);
  std::vector<char> on(n, 0);
  std::vector<int32_t> pat;
  for (int32_t j = 0; j < n; ++j) {
    pat.clear();
    double nrm = 0.0;
    for (int32_t e = cptr[j]; e < cptr[j + 1]; ++e) {
      const int32_t i = crow[e];
      w[i] = cval[e];
      on[i] = 1;
      pat.push_back(i);
      nrm += std::fabs(cval[e]);
    }
    for (const auto &rk : row[j]) {
      const int32_t k = rk.first;
      const double f = ldl ? rk.second * dg[k] : rk.second;
      for (const auto &ck : col[k]) {
        const int32_t i = ck.first;
        if (i < j) continue;
        if (!on[i]) {
          on[i] = 1;
          w[i] = 0.0;
          pat.push_back(i);
        }
        w[i] -= ck.second * f;
      }
    }
    if (!on[j]) return -1 - j;
    const double piv = w[j];
    if (ldl ? !(std::fabs(piv) >= 1e-300) : !(piv > 0.0)) return -1 - j;
    const double dj = ldl ? piv : std::sqrt(piv);
    dg[j] = dj;
    std::sort(pat.begin(), pat.end());
    for (int32_t i : pat) {
      if (i > j && std::fabs(w[i]) >= tau * nrm) {
        const double l = w[i] / dj;
        col[j].emplace_back(i, l);
        row[i].emplace_back(j, l);
      }
      on[i] = 0;
      w[i] = 0.0;
    }
  }
  F.n = n;
  F.kind = ldl ? 2 : 0;
  F.rp.assign(n + 1, 0);
  F.ci.clear();
  F.v.clear();
  for (int32_t i = 0; i < n; ++i) {
    for (const auto &rk : row[i]) {
      F.ci.push_back(rk.first);
      F.v.push_back(rk.second);
    }
    F.ci.push_back(i);
    F.v.push_back(dg[i]);
    F.rp[i + 1] = (int32_t)F.ci.size();
  }
  return 0;
}

// factor a block given as the lower triangle (diag last) in local indices
int factor_block(int kind, int32_t n, std::vector<int32_t> &rp, std::vector<int32_t> &ci,
                 std::vector<double> &v, LowerFactor &F, double droptol) {
  if (kind == SLR_FACT_CHOL) return envelope_cholesky(n, rp, ci, v, F);
  if (kind == SLR_FACT_ICT || kind == SLR_FACT_ILDLT) return threshold_factor(kind == SLR_FACT_ILDLT, n, rp, ci, v,
                                                                              droptol, F);
  F.n = n;
  F.kind = kind == SLR_FACT_ILDLT0 ? 2 : 0;
  F.rp = rp;
  F.ci = ci;
  F.v = v;
  return incomplete_factor(F);
}

// Minimum degree ordering (the ordering that AMD approximates, Sec. 6 uses it
// on every B_i before ICT / ILDLT) with exact degrees: eliminating a node
// joins its remaining neighbours into a clique, and each step takes the
// remaining node of smallest degree, the smallest index among equal
// degrees.  adj: sorted neighbour lists without the node itself.  Returns
// the elimination order (new -> old local index).
std::vector<int32_t> min_degree_order(std::vector<std::vector<int32_t>> adj) {
  const int32_t n = (int32_t)adj.size();
  std::set<std::pair<int32_t, int32_t>> ready;   // (degree, node)
  for (int32_t i = 0; i < n; ++i) ready.insert({(int32_t)adj[i].size(), i});
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<int32_t> merged;
  while (!ready.empty()) {
    const int32_t p = ready.begin()->second;
    ready.erase(ready.begin());
    order.push_back(p);
    const std::vector<int32_t> nb = std::move(adj[p]);
    adj[p].clear();
    for (int32_t u : nb) {
      ready.erase({(int32_t)adj[u].size(), u});
      merged.clear();
      std::set_union(adj[u].begin(), adj[u].end(), nb.begin(), nb.end(), std::back_inserter(merged));
      merged.erase(std::remove_if(merged.begin(), merged.end(), [&](int32_t x) { return x == u || x == p; }),
                   merged.end());
      adj[u].swap(merged);
      ready.insert({(int32_t)adj[u].size(), u});
    }
  }
  return order;
}

// The recursive interface solver's analysis (Sec. 5.2), from C in HID
// order (lev: connector level of each interface position).  C1 = the nodes
// of the lowest level; its connected pieces must each be a contiguous
// range (so that C1 is block diagonal in this order).
int inner_setup(HostSetup &H, const std::vector<int32_t> &lev, int kind, bool fp32, double droptol,
                std::string &err) {
  const int64_t m = H.m, s = H.s;
  H.have_plan = false;
  if (s == 0 || (int64_t)lev.size() != s) {
    err = "the recursive interface solver needs an interface";
    return SLR_ERR_ARG;
  }
  const int32_t lmin = *std::min_element(lev.begin(), lev.end());
  int64_t s1 = 0;
  while (s1 < s && lev[s1] == lmin) ++s1;
  if (s1 == s) {
    err = "the HID order has a single connector level: nothing to recurse on";
    return SLR_ERR_ARG;
  }
  H.s1 = s1;
  const int64_t s2 = s - s1;
  // connected pieces of C1 (union-find), each a contiguous range
  std::vector<int64_t> root(s1);
  std::iota(root.begin(), root.end(), 0);
  auto find = [&](int64_t x) {
    while (root[x] != x) x = root[x] = root[root[x]];
    return x;
  };
  for (int64_t t = 0; t < s1; ++t)
    for (int64_t e = H.a_rp[m + t]; e < H.a_rp[m + t + 1]; ++e) {
      const int64_t c = H.a_ci[e] - m;
      if (c >= 0 && c < s1) {
        const int64_t a = find(t), b = find(c);
        if (a != b) root[std::max(a, b)] = std::min(a, b);
      }
    }
  std::vector<int64_t> starts;
  std::vector<char> seen(s1, 0);
  for (int64_t t = 0; t < s1; ++t) {
    const int64_t r = find(t);
    if (t == 0 || find(t - 1) != r) {
      if (seen[r]) {
        err = "a connector of the leading HID level is not contiguous";
        return SLR_ERR_ARG;
      }
      seen[r] = 1;
      starts.push_back(t);
    }
  }
  starts.push_back(s1);
  const int32_t nb = (int32_t)starts.size() - 1;
  H.c1blocks.assign(nb, Block());
  std::vector<int> rcs(nb, 0);
  auto build_block = [&](int32_t q) {
    Block &b = H.c1blocks[q];
    b.m0 = (int32_t)starts[q];
    b.m = (int32_t)(starts[q + 1] - starts[q]);
    std::vector<int32_t> rp(b.m + 1, 0), ci;
    std::vector<double> v;
    for (int32_t r = 0; r < b.m; ++r) {
      const int64_t t = m + b.m0 + r;
      bool has_e = false;
      for (int64_t e = H.a_rp[t]; e < H.a_rp[t + 1]; ++e) {
        const int64_t c = H.a_ci[e] - m;
        if (c < 0) continue;
        if (c < s1) {
          if (c <= t - m) {
            ci.push_back((int32_t)(c - b.m0));
            v.push_back(H.a_v[e]);
          }
        } else {
          if (!has_e) {
            b.e_row.push_back(r);
            b.e_ptr.push_back((int32_t)b.e_q.size());
            has_e = true;
          }
          b.e_q.push_back((int32_t)(c - s1));
          b.e_val.push_back(H.a_v[e]);
        }
      }
      rp[r + 1] = (int32_t)ci.size();
    }
    b.e_ptr.push_back((int32_t)b.e_q.size());
    b.t_ptr.assign(1, 0);
    LowerFactor F;
    rcs[q] = factor_block(kind, b.m, rp, ci, v, F, droptol);
    if (rcs[q] != 0) return;
    b.nnz_L = (int64_t)F.v.size();
    build_sweeps(F, fp32, b.fwd, b.bwd);
  };
  {
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
      for (int32_t q = next++; q < nb; q = next++) build_block(q);
    };
    const int32_t nth = (int32_t)std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16u));
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < std::min(nth, nb); ++t) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
  }
  H.nnz_LC1 = 0;
  for (int32_t q = 0; q < nb; ++q) {
    if (rcs[q] != 0) {
      err = "factorisation of the inner block C1 failed at interface row " +
            std::to_string(H.c1blocks[q].m0 + (-1 - rcs[q]));
      return SLR_ERR_C_NOT_SPD;
    }
    H.nnz_LC1 += H.c1blocks[q].nnz_L;
  }
  // C2 = L2 L2^T and F^T (rows of C2, columns in C1)
  std::vector<int32_t> rp(s2 + 1, 0), ci;
  std::vector<double> v;
  H.ft_rp.assign(1, 0);
  H.ft_ci.clear();
  H.ft_v.clear();
  for (int64_t t = 0; t < s2; ++t) {
    for (int64_t e = H.a_rp[m + s1 + t]; e < H.a_rp[m + s1 + t + 1]; ++e) {
      const int64_t c = H.a_ci[e] - m;
      if (c < 0) continue;
      if (c < s1) {
        H.ft_ci.push_back((int32_t)c);
        H.ft_v.push_back(H.a_v[e]);
      } else if (c - s1 <= t) {
        ci.push_back((int32_t)(c - s1));
        v.push_back(H.a_v[e]);
      }
    }
    rp[t + 1] = (int32_t)ci.size();
    H.ft_rp.push_back((int64_t)H.ft_ci.size());
  }
  LowerFactor F2;
  const int rc = factor_block(kind, (int32_t)s2, rp, ci, v, F2, droptol);
  if (rc != 0) {
    err = "factorisation of the inner block C2 failed at interface row " + std::to_string(s1 + (-1 - rc));
    return SLR_ERR_C_NOT_SPD;
  }
  H.nnz_LC2 = (int64_t)F2.v.size();
  build_sweeps(F2, fp32, H.c2fwd, H.c2bwd);
  H.nnz_LC = H.nnz_LC1 + H.nnz_LC2;
  return SLR_OK;
}

}  // namespace

int host_setup(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
               const int32_t *part, int32_t p, const SetupParams &prm, HostSetup &H,
               std::string &err) {
  if (n <= 0 || p <= 0 || n > INT32_MAX) {
    err = "bad sizes";
    return SLR_ERR_ARG;
  }
  if (!is_symmetric(n, rowptr, col, val)) {
    err = "A is not symmetric (pattern and values must match)";
    return SLR_ERR_NOT_SYMMETRIC;
  }
  H.has_sep = false;
  for (int64_t i = 0; i < n; ++i) {
    if (part[i] < -1 || part[i] >= p) {
      err = "partition label out of range";
      return SLR_ERR_PARTITION;
    }
    if (part[i] == -1) H.has_sep = true;
  }
  H.n = n;
  H.p = p;
  // Sec. 2.1: local interface = coupled to a node of another subdomain
  // (vertex-based); nodes labelled -1 are separator nodes (edge-based), and
  // coupling to one does not make a node interface
  std::vector<char> iface(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (part[i] < 0) {
      iface[i] = 1;
      continue;
    }
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
      if (part[col[e]] >= 0 && part[col[e]] != part[i]) {
        iface[i] = 1;
        break;
      }
  }
  // eq. Global: interiors by subdomain, then interface by owner, separator
  // nodes last; ascending original index inside each group
  std::vector<std::vector<int64_t>> inner(p), ifc(p);
  std::vector<int64_t> sep;
  for (int64_t i = 0; i < n; ++i) {
    if (part[i] < 0)
      sep.push_back(i);
    else
      (iface[i] ? ifc : inner)[part[i]].push_back(i);
  }
  if (prm.b_order == SLR_BORDER_MINDEG) {
    // each interior in the minimum degree order of its B_i (the subdomains
    // are independent: one host thread per subdomain at a time)
    std::vector<int32_t> loc(n, -1);
    for (int32_t q = 0; q < p; ++q)
      for (size_t t = 0; t < inner[q].size(); ++t) loc[inner[q][t]] = (int32_t)t;
    auto order_block = [&](int32_t q) {
      const std::vector<int64_t> &g = inner[q];
      std::vector<std::vector<int32_t>> adj(g.size());
      for (size_t t = 0; t < g.size(); ++t) {
        for (int64_t e = rowptr[g[t]]; e < rowptr[g[t] + 1]; ++e) {
          const int64_t j = col[e];
          if (j != g[t] && !iface[j] && part[j] == q) adj[t].push_back(loc[j]);
        }
        std::sort(adj[t].begin(), adj[t].end());
      }
      const std::vector<int32_t> o = min_degree_order(std::move(adj));
      std::vector<int64_t> g2(g.size());
      for (size_t t = 0; t < g.size(); ++t) g2[t] = g[o[t]];
      return g2;
    };
    std::vector<std::vector<int64_t>> ordered(p);
    std::atomic<int32_t> next{0};
    auto worker = [&]() {
      for (int32_t q = next++; q < p; q = next++) ordered[q] = order_block(q);
    };
    const int32_t nth = (int32_t)std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16u));
    std::vector<std::thread> pool;
    for (int32_t t = 1; t < std::min(nth, p); ++t) pool.emplace_back(worker);
    worker();
    for (auto &th : pool) th.join();
    inner.swap(ordered);
  } else if (prm.b_order != SLR_BORDER_NATURAL) {
    err = "unknown b_order";
    return SLR_ERR_ARG;
  }
  H.perm.clear();
  H.blocks.assign(p, Block());
  for (int32_t q = 0; q < p; ++q) {
    H.blocks[q].m0 = (int32_t)H.perm.size();
    H.blocks[q].m = (int32_t)inner[q].size();
    H.perm.insert(H.perm.end(), inner[q].begin(), inner[q].end());
  }
  H.m = (int64_t)H.perm.size();
  std::vector<int64_t> y;
  for (int32_t q = 0; q < p; ++q) y.insert(y.end(), ifc[q].begin(), ifc[q].end());
  y.insert(y.end(), sep.begin(), sep.end());
  H.s = (int64_t)y.size();
  const int64_t s = H.s, m = H.m;
  // interface positions before any colouring
  std::vector<int64_t> ypos(n, -1);
  for (int64_t t = 0; t < s; ++t) ypos[y[t]] = t;
  H.c_colors = 0;
  std::vector<int32_t> hid_lev;   // connector level of every interface position (HID order)
  if (prm.c_levels == 2 && prm.c_order != SLR_CORDER_HID) {
    err = "the recursive interface solver needs the HID order of C";
    return SLR_ERR_ARG;
  }
  if (prm.c_order == SLR_CORDER_MULTICOLOR && s > 0) {
    // greedy colouring in interface order, then a stable sort by colour
    std::vector<int32_t> color(s, -1);
    std::vector<int32_t> mark;
    int32_t ncol = 0;
    for (int64_t t = 0; t < s; ++t) {
      int64_t i = y[t];
      mark.assign(ncol + 1, 0);
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        int64_t u = ypos[col[e]];
        if (u >= 0 && color[u] >= 0) mark[color[u]] = 1;
      }
      int32_t c = 0;
      while (mark[c]) ++c;
      color[t] = c;
      ncol = std::max(ncol, c + 1);
    }
    std::vector<int64_t> idx(s);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return color[a] < color[b]; });
    std::vector<int64_t> y2(s);
    for (int64_t t = 0; t < s; ++t) y2[t] = y[idx[t]];
    y.swap(y2);
    H.c_colors = ncol;
  } else if (prm.c_order == SLR_CORDER_HID && s > 0) {
    // HID connectors (Sec. 5.2): key = the subdomains met in the node's
    // closed neighbourhood; by key size (the connector's level), then key,
    // then original index
    std::vector<std::vector<int32_t>> key(s);
    for (int64_t t = 0; t < s; ++t) {
      const int64_t i = y[t];
      std::vector<int32_t> &k = key[t];
      k.push_back(part[i]);
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) k.push_back(part[col[e]]);
      std::sort(k.begin(), k.end());
      k.erase(std::unique(k.begin(), k.end()), k.end());
    }
    std::vector<int64_t> idx(s);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
      if (key[a].size() != key[b].size()) return key[a].size() < key[b].size();
      if (key[a] != key[b]) return key[a] < key[b];
      return y[a] < y[b];
    });
    std::vector<int64_t> y2(s);
    hid_lev.resize(s);
    for (int64_t t = 0; t < s; ++t) {
      y2[t] = y[idx[t]];
      hid_lev[t] = (int32_t)key[idx[t]].size();
    }
    y.swap(y2);
  } else if (prm.c_order != SLR_CORDER_SUBDOMAIN) {
    err = "unknown c_order";
    return SLR_ERR_ARG;
  }
  H.perm.insert(H.perm.end(), y.begin(), y.end());
  H.iperm.assign(n, -1);
  for (int64_t t = 0; t < n; ++t) H.iperm[H.perm[t]] = t;

  // A in the internal order
  H.a_rp.assign(n + 1, 0);
  H.a_ci.clear();
  H.a_v.clear();
  H.a_ci.reserve(rowptr[n]);
  H.a_v.reserve(rowptr[n]);
  H.a_src.clear();
  H.a_src.reserve(rowptr[n]);
  {
    std::vector<std::pair<int32_t, int64_t>> row;
    for (int64_t t = 0; t < n; ++t) {
      int64_t i = H.perm[t];
      row.clear();
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) row.emplace_back((int32_t)H.iperm[col[e]], e);
      std::sort(row.begin(), row.end());
      for (auto &pr : row) {
        H.a_ci.push_back(pr.first);
        H.a_v.push_back(val[pr.second]);
        H.a_src.push_back(pr.second);
      }
      H.a_rp[t + 1] = (int64_t)H.a_ci.size();
    }
  }
  const bool fp32 = prm.fact_prec == SLR_FP32;
  H.have_plan = prm.plan && (prm.b_fact == SLR_FACT_IC0 || prm.b_fact == SLR_FACT_ILDLT0) &&
                prm.c_fact == SLR_FACT_IC0;
  if (H.have_plan) {
    H.fb = RefactorPlan();
    H.fb.kind = prm.b_fact == SLR_FACT_ILDLT0 ? 2 : 0;
    H.fb.rp.assign(1, 0);
  }
  // Blocks: B_i factor, E rows and E^T rows (vertex-based partitioning:
  // interior nodes of subdomain i couple only to the interface of i).
  H.nnz_E = 0;
  for (int32_t q = 0; q < p; ++q) {
    Block &b = H.blocks[q];
    std::vector<int32_t> rp(b.m + 1, 0), ci;
    std::vector<double> v;
    std::vector<int64_t> src;
    for (int32_t r = 0; r < b.m; ++r) {
      int64_t t = b.m0 + r;
      bool has_e = false;
      for (int64_t e = H.a_rp[t]; e < H.a_rp[t + 1]; ++e) {
        int64_t c = H.a_ci[e];
        if (c < m) {
          if (c < b.m0 || c >= b.m0 + b.m) {
            err = "interior nodes of two subdomains are coupled";
            return SLR_ERR_PARTITION;
          }
          if (c <= t) {
            ci.push_back((int32_t)(c - b.m0));
            v.push_back(H.a_v[e]);
            src.push_back(H.a_src[e]);
          }
        } else {
          if (!has_e) {
            b.e_row.push_back(r);
            b.e_ptr.push_back((int32_t)b.e_q.size());
            has_e = true;
          }
          b.e_q.push_back((int32_t)(c - m));
          b.e_val.push_back(H.a_v[e]);
          b.e_src.push_back(H.a_src[e]);
        }
      }
      rp[r + 1] = (int32_t)ci.size();
    }
    b.e_ptr.push_back((int32_t)b.e_q.size());
    H.nnz_E += (int64_t)b.e_q.size();
    LowerFactor F;
    int rc = factor_block(prm.b_fact, b.m, rp, ci, v, F, prm.droptol);
    if (rc != 0) {
      err = "factorisation of B_" + std::to_string(q) + " failed at local row " +
            std::to_string(-1 - rc);
      return SLR_ERR_BREAKDOWN;
    }
    b.nnz_L = (int64_t)F.v.size();
    build_sweeps(F, fp32, b.fwd, b.bwd);
    if (H.have_plan) {
      // incomplete factors keep the input pattern: entry e of the block's
      // factor is entry f_base + e of the global one
      RefactorPlan &P = H.fb;
      b.f_base = (int64_t)P.ci.size();
      for (int32_t r = 0; r < b.m; ++r) {
        for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
          P.ci.push_back(b.m0 + ci[e]);
          P.src.push_back(src[e]);
        }
        P.rp.push_back((int64_t)P.ci.size());
      }
    }
  }
  if (H.have_plan) {
    // levels of the B factorisation: level l of every block together (the
    // dependencies of a row are the columns of its factor row, as for the
    // forward sweep)
    int32_t nl = 0;
    for (const Block &b : H.blocks) nl = std::max(nl, b.fwd.nlev);
    std::vector<std::vector<int32_t>> by(nl);
    for (const Block &b : H.blocks)
      for (int32_t l = 0; l < b.fwd.nlev; ++l)
        for (int32_t t = b.fwd.levptr[l]; t < b.fwd.levptr[l + 1]; ++t) by[l].push_back(b.m0 + b.fwd.rows[t]);
    H.fb.lev.assign(1, 0);
    for (auto &v : by) {
      H.fb.rows.insert(H.fb.rows.end(), v.begin(), v.end());
      H.fb.lev.push_back((int32_t)H.fb.rows.size());
    }
  }
  // E^T: with separator nodes one CSR over all interface rows (a separator
  // row couples to the interiors of several subdomains); otherwise rows
  // grouped by owner subdomain for the B kernel's epilogue
  if (H.has_sep) {
    H.et_rp.assign(1, 0);
    H.et_ci.clear();
    H.et_v.clear();
    for (int64_t t = 0; t < s; ++t) {
      for (int64_t e = H.a_rp[m + t]; e < H.a_rp[m + t + 1]; ++e)
        if (H.a_ci[e] < m) {
          H.et_ci.push_back(H.a_ci[e]);
          H.et_v.push_back(H.a_v[e]);
        }
      H.et_rp.push_back((int64_t)H.et_ci.size());
    }
  }
  for (int64_t t = 0; t < s && !H.has_sep; ++t) {
    int64_t i = H.perm[m + t];
    Block &b = H.blocks[part[i]];
    b.t_q.push_back((int32_t)t);
    b.t_ptr.push_back((int32_t)b.t_j.size());
    for (int64_t e = H.a_rp[m + t]; e < H.a_rp[m + t + 1]; ++e) {
      int64_t c = H.a_ci[e];
      if (c < m) {
        if (c < b.m0 || c >= b.m0 + b.m) {
          err = "interface node coupled to the interior of another subdomain";
          return SLR_ERR_PARTITION;
        }
        b.t_j.push_back((int32_t)(c - b.m0));
        b.t_val.push_back(H.a_v[e]);
        b.t_src.push_back(H.a_src[e]);
      }
    }
  }
  for (auto &b : H.blocks) b.t_ptr.push_back((int32_t)b.t_j.size());
  if (H.has_sep) H.have_plan = false;
  const int c_kind = prm.c_fact == SLR_FACT_CHOL || prm.c_fact == SLR_FACT_ICT ? prm.c_fact : SLR_FACT_IC0;
  if (prm.c_levels == 2) return inner_setup(H, hid_lev, c_kind, fp32, prm.droptol, err);
  // C and its factor (Sec. 3.1: C = L L^T), in the interface order
  {
    std::vector<int32_t> rp(s + 1, 0), ci;
    std::vector<double> v;
    std::vector<int64_t> src;
    for (int64_t t = 0; t < s; ++t) {
      for (int64_t e = H.a_rp[m + t]; e < H.a_rp[m + t + 1]; ++e) {
        int64_t c = H.a_ci[e];
        if (c >= m && c <= m + t) {
          ci.push_back((int32_t)(c - m));
          v.push_back(H.a_v[e]);
          src.push_back(H.a_src[e]);
        }
      }
      rp[t + 1] = (int32_t)ci.size();
    }
    LowerFactor F;
    int rc = factor_block(c_kind, (int32_t)s, rp, ci, v, F, prm.droptol);
    if (rc != 0) {
      err = "factorisation of C failed at interface row " + std::to_string(-1 - rc);
      return SLR_ERR_C_NOT_SPD;
    }
    H.nnz_LC = (int64_t)F.v.size();
    build_sweeps(F, fp32, H.cfwd, H.cbwd);
    if (H.have_plan) {
      RefactorPlan &P = H.fc;
      P = RefactorPlan();
      P.kind = 0;
      P.rp.assign(rp.begin(), rp.end());
      P.ci = ci;
      P.src = src;
      P.lev = H.cfwd.levptr;
      P.rows = H.cfwd.rows;
      if (P.lev.empty()) P.lev.push_back(0);
    }
  }
  return SLR_OK;
}

}  // namespace slr

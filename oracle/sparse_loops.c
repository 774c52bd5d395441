/*
 * Oracle sparse loops for the SLR preconditioner (Li, Xi & Saad 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU FP64 oracle that
 * the device library is checked against.  It shares no code with the
 * device library and must never be linked into it.
 *
 * Plain, slow, obviously-correct loops over CSR arrays:
 *   - incomplete Cholesky IC(0) and incomplete LDL^T(0) on a fixed pattern
 *     (the local solvers of Sec. 5.2 / Sec. 6, restricted to zero fill),
 *     and their threshold-dropping forms ICT / ILDLT;
 *   - forward / backward triangular sweeps (the B and C solves of Sec. 5.2).
 *
 * Storage convention for a lower factor: CSR with sorted column indices,
 * the diagonal stored as the LAST entry of each row.  For LDL^T the stored
 * diagonal entries hold D and the strictly lower entries hold the unit
 * lower factor.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Merge-intersection of rows i and j of the partially built factor over
 * columns k < kmax: sum of l_ik * w_k * l_jk (w = d_k for LDL^T, 1 for IC). */
static double row_dot(const int64_t *rp, const int32_t *ci, const double *v,
                      int64_t i, int64_t j, int32_t kmax, const double *d) {
  double s = 0.0;
  int64_t a = rp[i], ae = rp[i + 1];
  int64_t b = rp[j], be = rp[j + 1];
  while (a < ae && b < be) {
    int32_t ca = ci[a], cb = ci[b];
    if (ca >= kmax || cb >= kmax) break;
    if (ca == cb) {
      s += v[a] * v[b] * (d ? d[ca] : 1.0);
      ++a; ++b;
    } else if (ca < cb) {
      ++a;
    } else {
      ++b;
    }
  }
  return s;
}

/* IC(0): on entry v holds tril(A) on the pattern (diag last); on exit the
 * unique L with (L L^T)_ij = a_ij on the pattern.  Returns 0, or -(i+1) if
 * the pivot of row i is not positive. */
int orc_ic0(int64_t n, const int64_t *rp, const int32_t *ci, double *v) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t e = rp[i + 1] - 1;              /* diagonal slot */
    if (ci[e] != i) return -(int)(i + 1);
    for (int64_t t = rp[i]; t < e; ++t) {
      int32_t j = ci[t];
      double s = row_dot(rp, ci, v, i, j, j, 0);
      double ljj = v[rp[j + 1] - 1];
      v[t] = (v[t] - s) / ljj;
    }
    double s = row_dot(rp, ci, v, i, i, (int32_t)i, 0);
    double piv = v[e] - s;
    if (!(piv > 0.0)) return -(int)(i + 1);
    v[e] = sqrt(piv);
  }
  return 0;
}

/* ILDL^T(0): on exit strictly-lower entries hold unit L, diagonal slots
 * hold D.  Returns -(i+1) when |d_i| < 1e-300. */
int orc_ildlt0(int64_t n, const int64_t *rp, const int32_t *ci, double *v,
               double *dwork) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t e = rp[i + 1] - 1;
    if (ci[e] != i) return -(int)(i + 1);
    for (int64_t t = rp[i]; t < e; ++t) {
      int32_t j = ci[t];
      double s = row_dot(rp, ci, v, i, j, j, dwork);
      v[t] = (v[t] - s) / dwork[j];
    }
    double s = row_dot(rp, ci, v, i, i, (int32_t)i, dwork);
    double di = v[e] - s;
    if (!(fabs(di) >= 1e-300)) return -(int)(i + 1);
    v[e] = di;
    dwork[i] = di;
  }
  return 0;
}

/* Solve L x = b in place (x holds b on entry).  unit != 0: unit diagonal. */
void orc_lower_solve(int64_t n, const int64_t *rp, const int32_t *ci,
                     const double *v, double *x, int unit) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t e = rp[i + 1] - 1;
    double s = x[i];
    for (int64_t t = rp[i]; t < e; ++t) s -= v[t] * x[ci[t]];
    x[i] = unit ? s : s / v[e];
  }
}

/* Solve L^T x = b in place using the rows of L (column sweep). */
void orc_upper_solve(int64_t n, const int64_t *rp, const int32_t *ci,
                     const double *v, double *x, int unit) {
  for (int64_t i = n - 1; i >= 0; --i) {
    int64_t e = rp[i + 1] - 1;
    double xi = unit ? x[i] : x[i] / v[e];
    x[i] = xi;
    for (int64_t t = rp[i]; t < e; ++t) x[ci[t]] -= v[t] * xi;
  }
}

/* x <- D^{-1} x with D the diagonal slots of an LDL^T factor. */
void orc_diag_solve(int64_t n, const int64_t *rp, const double *v, double *x) {
  for (int64_t i = 0; i < n; ++i) x[i] /= v[rp[i + 1] - 1];
}

/* Threshold incomplete factorisations (ICT / ILDLT, the local solvers of
 * Sec. 6 with threshold dropping), left-looking by columns.
 * Input: tril(A) as row CSR (diag last) of order n.  Column j:
 *   w_i = a_ij (i >= j);  nrm = sum_i |a_ij| over that column;
 *   for every k < j with a kept l_jk (ascending k), f = l_jk (IC) or
 *   l_jk d_k (LDL), and for every kept l_ik with i >= j: w_i -= l_ik f;
 *   pivot w_j: IC l_jj = sqrt(w_j) (w_j > 0), LDL d_j = w_j (|w_j| >= 1e-300);
 *   for i > j with w_i present, keep l_ij = w_i / l_jj (or / d_j) when
 *   |w_i| >= tau nrm.
 * Output: row CSR of L (columns ascending, diagonal last, the diagonal slot
 * holding l_jj or d_j), at most cap entries.  Returns 0; -(j+1) on a failed
 * pivot of column j; -(n+1) when cap is too small (*nnz_out: entries
 * needed). */
typedef struct { int32_t col; int32_t next; double val; } orc_lent;   /* entry l_ik of row i: column k */

int orc_ict(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, double tau, int ldl,
            int64_t cap, int64_t *orp, int32_t *oci, double *ov, int64_t *nnz_out) {
  int64_t nnz = rp[n];
  /* CSC of tril(A): column j holds rows i >= j */
  int64_t *cp = calloc(n + 1, sizeof(int64_t));
  int32_t *cr = malloc(sizeof(int32_t) * (nnz + 1));
  double *cv = malloc(sizeof(double) * (nnz + 1));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) cp[ci[e] + 1]++;
  for (int64_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
  int64_t *fill = malloc(sizeof(int64_t) * (n + 1));
  for (int64_t j = 0; j <= n; ++j) fill[j] = cp[j];
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      int32_t j = ci[e];
      cr[fill[j]] = (int32_t)i;
      cv[fill[j]++] = v[e];
    }
  /* L by columns (rows ascending, no diagonal) and, per row, the columns
   * that hold an entry in it (linked in ascending column order) */
  int64_t lcap = nnz + n + 16, ln = 0;
  int64_t *lcp = calloc(n + 1, sizeof(int64_t));
  int32_t *lr = malloc(sizeof(int32_t) * lcap);
  double *lv = malloc(sizeof(double) * lcap);
  int32_t *rhead = malloc(sizeof(int32_t) * n), *rtail = malloc(sizeof(int32_t) * n);
  int64_t rcap = lcap, rn = 0;
  orc_lent *rl = malloc(sizeof(orc_lent) * rcap);
  double *diag = malloc(sizeof(double) * n);
  double *w = calloc(n, sizeof(double));
  char *mark = calloc(n, 1);
  int32_t *pat = malloc(sizeof(int32_t) * n);
  for (int64_t i = 0; i < n; ++i) rhead[i] = rtail[i] = -1;
  int rc = 0;
  for (int64_t j = 0; j < n && rc == 0; ++j) {
    int64_t np = 0;
    double nrm = 0.0;
    for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
      int32_t i = cr[e];
      w[i] = cv[e];
      mark[i] = 1;
      pat[np++] = i;
      nrm += fabs(cv[e]);
    }
    for (int32_t t = rhead[j]; t >= 0; t = rl[t].next) {
      int32_t k = rl[t].col;
      double f = ldl ? rl[t].val * diag[k] : rl[t].val;
      for (int64_t e = lcp[k]; e < lcp[k + 1]; ++e) {
        int32_t i = lr[e];
        if (i < j) continue;
        if (!mark[i]) {
          mark[i] = 1;
          w[i] = 0.0;
          pat[np++] = i;
        }
        w[i] -= lv[e] * f;
      }
    }
    if (!mark[j]) {
      rc = -(int)(j + 1);
      break;
    }
    double piv = w[j];
    double dj;
    if (ldl) {
      if (!(fabs(piv) >= 1e-300)) { rc = -(int)(j + 1); break; }
      dj = piv;
    } else {
      if (!(piv > 0.0)) { rc = -(int)(j + 1); break; }
      dj = sqrt(piv);
    }
    diag[j] = dj;
    /* rows below the diagonal in ascending order (insertion sort) */
    for (int64_t a = 1; a < np; ++a) {
      int32_t x = pat[a];
      int64_t b = a - 1;
      while (b >= 0 && pat[b] > x) { pat[b + 1] = pat[b]; --b; }
      pat[b + 1] = x;
    }
    lcp[j] = ln;
    for (int64_t a = 0; a < np; ++a) {
      int32_t i = pat[a];
      if (i > j && fabs(w[i]) >= tau * nrm) {
        if (ln >= lcap) {
          lcap *= 2;
          lr = realloc(lr, sizeof(int32_t) * lcap);
          lv = realloc(lv, sizeof(double) * lcap);
        }
        double l = w[i] / dj;
        lr[ln] = i;
        lv[ln++] = l;
        if (rn >= rcap) {
          rcap *= 2;
          rl = realloc(rl, sizeof(orc_lent) * rcap);
        }
        rl[rn].col = (int32_t)j;
        rl[rn].next = -1;
        rl[rn].val = l;
        if (rtail[i] >= 0) rl[rtail[i]].next = (int32_t)rn; else rhead[i] = (int32_t)rn;
        rtail[i] = (int32_t)rn++;
      }
      mark[i] = 0;
      w[i] = 0.0;
    }
    lcp[j + 1] = ln;
  }
  /* row CSR of L, diagonal last */
  int64_t need = ln + n;
  *nnz_out = need;
  if (rc == 0 && need > cap) rc = -(int)(n + 1);
  if (rc == 0) {
    int64_t o = 0;
    orp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
      for (int32_t t = rhead[i]; t >= 0; t = rl[t].next) {
        oci[o] = rl[t].col;
        ov[o++] = rl[t].val;
      }
      oci[o] = (int32_t)i;
      ov[o++] = diag[i];
      orp[i + 1] = o;
    }
  }
  free(cp); free(cr); free(cv); free(fill); free(lcp); free(lr); free(lv);
  free(rhead); free(rtail); free(rl); free(diag); free(w); free(mark); free(pat);
  return rc;
}

/*
 * Oracle sparse loops for the SLR preconditioner (Li, Xi & Saad 2015).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is part of the CPU FP64 oracle that
 * the device library is checked against.  It shares no code with the
 * device library and must never be linked into it.
 *
 * Plain, slow, obviously-correct loops over CSR arrays:
 *   - incomplete Cholesky IC(0) and incomplete LDL^T(0) on a fixed pattern
 *     (the local solvers of Sec. 5.2 / Sec. 6, restricted to zero fill);
 *   - forward / backward triangular sweeps (the B and C solves of Sec. 5.2).
 *
 * Storage convention for a lower factor: CSR with sorted column indices,
 * the diagonal stored as the LAST entry of each row.  For LDL^T the stored
 * diagonal entries hold D and the strictly lower entries hold the unit
 * lower factor.
 */
#include <math.h>
#include <stdint.h>

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

// Launchers of the Krylov / Lanczos / utility kernels (slr_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>

namespace slr {

// Per-column Krylov state kept on the device (CG / flexible CG).
struct KState {
  double rz[2];   // r . z, double-buffered by iteration parity
  double al[2];   // alpha, double-buffered likewise
  double pq[2];   // p . A p (flexible CG), double-buffered likewise
  double alpha, beta;
  double rr;      // ||r||^2 of the recurrence residual
  double bb;      // ||b||^2
  double relres;  // final true relative residual
  int32_t active; // 1 while iterating
  int32_t status; // 0 converged, -8 not converged / broken down
  int32_t iters;  // iterations (updates of x and r) done
  int32_t start_it; // global iteration index of the column's first iteration
};

struct KArgs {
  double *X, *R, *Z, *P;      // n x ncols, leading dimension ld (internal order)
  double *Q;                  // w = A z (same layout)
  double *S;                  // s = A p (same layout)
  int64_t ld;
  KState *st;
  double *part;               // nblk x 4 ncols partials
  double *part2;              // nblk x ncols partials
  unsigned int *counter;      // unused
  int32_t nblk;
  int32_t maxit;
  double rtol2;
};

// Krylov kernels of CG / flexible CG (one reduction phase per iteration):
// CG_INIT (x = 0, partial b.b), CG_START (state), then per iteration, after
// the preconditioner, CG_SPMV (w = A z and the partials) and CG_UPDATE.
// CG_SPMV takes a one-column kernel when nc == 1; CG_SPMV_TILES always
// takes the column-tile kernel, whose column arithmetic does not depend on
// the number of columns (batches).
enum { CG_INIT = 0, CG_START, CG_SPMV, CG_UPDATE, CG_SPMV_TILES };

// Round an FP64 value for storage: FP32 is round-to-nearest-even; BF16 is
// round-to-nearest-even of the FP32-rounded value.
template <typename TU>
__device__ __forceinline__ TU round_store(double x);
template <>
__device__ __forceinline__ double round_store<double>(double x) {
  return x;
}
template <>
__device__ __forceinline__ float round_store<float>(double x) {
  return (float)x;
}
template <>
__device__ __forceinline__ __hip_bfloat16 round_store<__hip_bfloat16>(double x) {
  const float f = (float)x;
  uint32_t u = __float_as_uint(f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  __hip_bfloat16 r;
  unsigned short h = (unsigned short)u;
  __builtin_memcpy(&r, &h, sizeof(h));
  return r;
}

// y = a y + b M x for CSR M with int64 row pointers (a == 0: y only written)
void launch_spmv_axpby(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                       int64_t ldx, double *y, int64_t ldy, int32_t nrhs, double a, double b, hipStream_t st);
void launch_axpby(int64_t n, int32_t nrhs, double a, const double *x, int64_t ldx, double b, double *y,
                  int64_t ldy, hipStream_t st);
void launch_permute(int64_t n, const int64_t *idx, const double *src, int64_t lds, double *dst, int64_t ldd,
                    int32_t nrhs, bool scatter, hipStream_t st);
void launch_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                 int64_t ldx, double *y, int64_t ldy, int32_t nrhs, hipStream_t st);
void launch_cg(int op, int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const KArgs &K,
               int32_t c0, int32_t nc, int32_t flexible, int32_t it, hipStream_t st);
void launch_fold(const double *part, int32_t nb, int32_t ncol, double *out, double scale, hipStream_t st);
void launch_relres(int64_t n, const double *B, int64_t ldb, const double *AX, int64_t ldax, const KArgs &K,
                   int32_t c0, int32_t nc, hipStream_t st);
void launch_multidot(int64_t s, int32_t J, const double *V, int64_t ldv, const double *w, double *part,
                     int32_t nblk, double *out, unsigned int *counter, hipStream_t st);
// w -= V h; sqpart (optional) receives per-block sums of the updated w^2
// (returns the number of blocks)
int32_t launch_gemv_sub(int64_t s, int32_t J, const double *V, int64_t ldv, const double *h, double *w,
                        double *sqpart, hipStream_t st);
void launch_gemv_add(int64_t n, int32_t J, const double *V, int64_t ldv, const double *y, double *x,
                     hipStream_t st);
// w -= alpha v + beta_prev v_prev (alpha folded from the rb partials, kept in
// sc[0]; beta_prev = sc[1]); per-block ||w||^2 partials to sqpart (returns
// the block count, equal to launch_gemv_sub_fold's)
int32_t launch_lanczos_axpy(int64_t s, double *w, const double *v, const double *vprev, double *sc,
                            const double *apart, int32_t rb, double *sqpart, hipStream_t st);
// Gram-Schmidt coefficients V^T w (as launch_multidot_partial) of Lanczos
// step j behind the partial reorthogonalisation decision (omega recurrence
// from alpha, beta, sc[0] = alpha_j and the rbp partials of ||w||^2 in
// bpart; state om (3 rows of ld), frc / tn per step); rflag[j] receives the
// decision and the launch does nothing else when it is 0
int32_t launch_multidot_pro(int64_t s, int32_t J, const double *V, int64_t ldv, const double *w, double *part,
                            int32_t nblk, int32_t j, const double *alpha, const double *beta, const double *sc,
                            const double *bpart, int32_t rbp, double *om, int32_t ld, int *frc, double *tn,
                            int *rflag, hipStream_t st);
// aval: device pointer to alpha_j (or nullptr: alpha_j is sc[0])
void launch_lanczos_next(int64_t s, int32_t j, const double *w, double *vnext, double *sc, double *alpha,
                         double *beta, const double *bpart, int32_t rb, const double *aval, hipStream_t st);
// gate (optional, device): the launch does nothing when *gate == 0
int32_t launch_multidot_partial(int64_t s, int32_t J, const double *V, int64_t ldv, const double *w, double *part,
                                int32_t nblk, hipStream_t st, const int *gate = nullptr);
// w -= V h with h folded in each block from the rb multidot partials
// (block 0 stores h to hout when given); sqpart as for launch_gemv_sub
int32_t launch_gemv_sub_fold(int64_t s, int32_t J, const double *V, int64_t ldv, const double *hpart, int32_t rb,
                             double *w, double *hout, double *sqpart, hipStream_t st, const int *gate = nullptr);
void launch_scale_inv_sqrt(int64_t s, const double *w, double *out, const double *nrm2, hipStream_t st);
void launch_div_scalar(int64_t n, const double *w, double *v, const double *scale, hipStream_t st);
void launch_gmres_givens(int32_t j, int32_t ldh, double *Hm, const double *h1, const double *h2,
                         const double *hn2, double *cs, double *sn, double *g, double tol, int *flags,
                         double *vscale, hipStream_t st);
void launch_gmres_solve(int32_t jj, int32_t ldh, const double *Hm, const double *g, double *y, hipStream_t st);
// scratch: 6 m K doubles
void launch_tridiag_eig(int32_t m, const double *alpha, const double *beta, double *scratch, double *eval,
                        double *Y, int32_t K, int *info, hipStream_t st);
template <typename TU>
void launch_ritz(int64_t s, int32_t m, int32_t k, const double *V, int64_t ldv, const double *Y, double *U64,
                 TU *U, hipStream_t st);
template <typename TU>
void launch_round_copy(int64_t n, const double *src, TU *dst, hipStream_t st);
// rank-k block with U^T w from a row-major copy of U (FP64 / FP32): groups
// of the padded layout (ldk receives the padded row length), the copy from
// the column-major FP64 U (lr_rm_groups * 64 * (16 / sizeof(TU)) entries),
// and the block itself (the update reads the column-major U)
template <typename TU>
int64_t lr_rm_groups(int64_t s, int32_t k, int32_t &ldk);
template <typename TU>
void launch_lr_to_rm(const double *U64, int64_t s, int32_t k, TU *Urm, hipStream_t st);
template <typename TU>
void launch_lowrank_rm(const TU *Urm, const TU *U, int64_t s, int32_t k, const double *dsc, double rho,
                       const double *w, int64_t ldw, double *wout, int64_t ldo, int32_t nrhs, double *part,
                       int32_t nblk, double *cbuf, hipStream_t st);

}  // namespace slr

namespace slr {
void launch_lanczos_record(int32_t j, double *sc, double *alpha, double *beta, hipStream_t st);
void launch_lanczos_alpha(int32_t j, const double *h, double *sc, hipStream_t st);
// rank-k block on matrix cores: BF16 U (k <= 64) in 16 x 16 tiles, one copy
// in the layout of U^T W's A operand (Upt) and one in that of the update's
// B operand (Uup), lr_tile_entries(s, k) entries each
int64_t lr_tile_entries(int64_t s, int32_t k);
void launch_lr_to_tiles(const double *U64, int64_t s, int32_t k, __hip_bfloat16 *Upt, __hip_bfloat16 *Uup,
                        hipStream_t st);
void launch_lowrank_mfma(const __hip_bfloat16 *Upt, const __hip_bfloat16 *Uup, int64_t s, int32_t k,
                         const double *dsc, double rho, const double *w, int64_t ldw, double *wout, int64_t ldo,
                         int32_t nrhs, double *part, int32_t nblk, double *cbuf, hipStream_t st);
void launch_gmres_g0(int32_t len, const double *nrm2, double *g, hipStream_t st);
}  // namespace slr

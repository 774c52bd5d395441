// Device-side layout of an SLR preconditioner and the kernel launchers.
// All device vectors are FP64, column-major, in the internal DD order
// (interiors by subdomain, then the interface in C's factor order).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>

namespace slr {

// Per-subdomain descriptor of the batched B_i solves (offsets into the
// concatenated arrays of all subdomains).
struct BlockDesc {
  int32_t m0, m;                   // interior range in the internal order
  int32_t f_lev, f_nlev, f_row, f_rp, f_ent;  // forward sweep
  int32_t b_lev, b_nlev, b_row, b_rp, b_ent;  // backward sweep
  int32_t e_row, e_n, e_ptr;       // E rows: e_row[e_row + i], e_ptr[e_ptr + i]
  int32_t t_row, t_n, t_ptr;       // E^T rows (interface rows owned here)
};

// Concatenated level-scheduled sweeps (see slr_host.h, struct Sweep).
// rp entries are absolute offsets into ci / w.
template <typename TS>
struct SweepArrays {
  const int32_t *lev = nullptr;    // level pointers (local to the block)
  const int32_t *rows = nullptr;   // level-sorted local rows
  const int32_t *rp = nullptr;     // per-block nrows+1 absolute entry offsets
  const int32_t *ci = nullptr;     // local column indices
  const TS *w = nullptr;           // pre-scaled off-diagonal weights
  const TS *sc = nullptr;          // per-row scale
};

template <typename TS>
struct BlockArrays {
  const BlockDesc *desc = nullptr;
  SweepArrays<TS> fwd, bwd;
  const int32_t *e_row = nullptr, *e_ptr = nullptr, *e_q = nullptr;
  const TS *e_val = nullptr;
  const int32_t *t_q = nullptr, *t_ptr = nullptr, *t_j = nullptr;
  const TS *t_val = nullptr;
  int32_t max_m = 0;
  int32_t max_lev = 0;
};

// What one launch of the batched B kernel computes for each subdomain i
// and right-hand side column c (columns [0, nrhs)):
//   rhs   = a_f * f_i + b_y * E_i y           (prologue)
//   z     = B_i^{-1} rhs                      (forward + backward sweep in LDS)
//   u_i   = z                                 (if u != nullptr)
//   gout_q = c_g * g_q + d_t * (E^T z)_q      (epilogue, q owned by i; if gout)
struct BArgs {
  const double *f = nullptr;  int64_t ldf = 0;  double a_f = 0.0;
  const double *y = nullptr;  int64_t ldy = 0;  double b_y = 0.0;
  const double *g = nullptr;  int64_t ldg = 0;  double c_g = 0.0;
  double *gout = nullptr;     int64_t ldgo = 0; double d_t = 0.0;
  double *u = nullptr;        int64_t ldu = 0;
  int32_t nrhs = 1;
  int32_t R = 1;              // right-hand sides per workgroup
};

template <typename TS, typename TC>
void launch_bsolve(const BlockArrays<TS> &B, int32_t p, const BArgs &a, int32_t threads,
                   size_t lds_bytes, hipStream_t st);

// In-place level-scheduled sweep of one (interface) block on a global
// vector: x (ld, nrhs columns).  Deep schedules run in one workgroup per
// column; shallow ones launch once per level over the whole device.
template <typename TS, typename TC>
void launch_sweep(const SweepArrays<TS> &S, const int32_t *lev_host, int32_t nlev, int32_t nrows,
                  double *x, int64_t ldx, int32_t nrhs, bool one_wg, hipStream_t st);

// Rank-k block of eq. skt on w (s x nrhs, ld ldw), output to wout (ldo):
//   c = U^T w ;  c_i <- c_i * dsc_i ;  wout = rho * w + U c
template <typename TU>
void launch_lowrank(const TU *U, int64_t s, int32_t k, const double *dsc, double rho,
                    const double *w, int64_t ldw, double *wout, int64_t ldo, int32_t nrhs,
                    double *part, int32_t nblk, double *cbuf, unsigned int *counter,
                    hipStream_t st);

}  // namespace slr

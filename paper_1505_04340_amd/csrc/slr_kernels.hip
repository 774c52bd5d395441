// HIP kernels of the SLR preconditioner hot path for gfx950 (CDNA4).
//
// Paper: Li, Xi & Saad, "Schur complement based domain decomposition
// preconditioners with low-rank corrections" (2015).
//   batched B_i solves + E / E^T products ........ Sec. 2.2 (two B solves per apply), Sec. 5.2
//   interface solves with L (C = L L^T) .......... eq. S, Sec. 5.2
//   rank-k block (U_k, Lambda_k, theta) ........... eq. skt
//   Lanczos on H, tridiagonal eigensolve .......... eq. H, Sec. 5.1
//   Krylov accelerators (CG / GMRES) .............. Sec. 6
//
// Reductions are deterministic: every block writes a partial, and the
// last block to arrive (atomic ticket) sums the partials in block order.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstdint>

#include "slr_dev.h"
#include "slr_kern.h"

namespace slr {

template <typename TC, typename TS>
__device__ __forceinline__ TC cvt(TS x) {
  return (TC)x;
}
template <>
__device__ __forceinline__ float cvt<float, __hip_bfloat16>(__hip_bfloat16 x) {
  return __bfloat162float(x);
}
template <>
__device__ __forceinline__ double cvt<double, __hip_bfloat16>(__hip_bfloat16 x) {
  return (double)__bfloat162float(x);
}

// ---------------------------------------------------------------------------
// Deterministic block reduction helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;  // valid in lane 0
}

// Sum over the block (blockDim multiple of 64, <= 1024); result in thread 0.
__device__ double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  return r;
}

// Returns true in every thread of the last block to finish (after its
// partials became visible); resets the ticket for the next launch.
__device__ bool last_block(unsigned int *counter) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int t = atomicAdd(counter, 1u);
    last = (t == gridDim.x * gridDim.y - 1);
    if (last) *counter = 0u;
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// ---------------------------------------------------------------------------
// K1/K2: batched subdomain solves with fused E / E^T products
// ---------------------------------------------------------------------------
template <typename TS, typename TC>
__device__ __forceinline__ void sweep_lds(const SweepArrays<TS> &S, int row0, int rp0,
                                          const int32_t *lev, int nlev, TC *xs, int R, int Rg) {
  for (int l = 0; l < nlev; ++l) {
    const int a = lev[l], b = lev[l + 1];
    const int ntask = (b - a) * Rg;
    for (int t = threadIdx.x; t < ntask; t += blockDim.x) {
      const int q = t / Rg;
      const int r = t - q * Rg;
      const int slot = a + q;
      const int row = S.rows[row0 + slot];
      const int e0 = S.rp[rp0 + slot], e1 = S.rp[rp0 + slot + 1];
      TC acc = cvt<TC>(S.sc[row0 + slot]) * xs[row * R + r];
      for (int e = e0; e < e1; ++e) acc -= cvt<TC>(S.w[e]) * xs[S.ci[e] * R + r];
      xs[row * R + r] = acc;
    }
    __syncthreads();
  }
}

template <typename TS, typename TC>
__global__ void __launch_bounds__(1024) k_bsolve(BlockArrays<TS> B, BArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  TC *xs = reinterpret_cast<TC *>(smem);
  const BlockDesc d = B.desc[blockIdx.x];
  const int R = a.R;
  const int c0 = blockIdx.y * R;
  const int Rg = min(R, a.nrhs - c0);
  const int m = d.m;
  int32_t *levf = reinterpret_cast<int32_t *>(smem + sizeof(TC) * (size_t)B.max_m * R);
  int32_t *levb = levf + B.max_lev + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i <= d.f_nlev; i += nt) levf[i] = B.fwd.lev[d.f_lev + i];
  for (int i = tid; i <= d.b_nlev; i += nt) levb[i] = B.bwd.lev[d.b_lev + i];
  // prologue: rhs = a_f f_i + b_y E_i y
  for (int t = tid; t < m * Rg; t += nt) {
    const int r = t / m, row = t - r * m;
    double v = 0.0;
    if (a.a_f != 0.0) v = a.a_f * a.f[(int64_t)(d.m0 + row) + (int64_t)(c0 + r) * a.ldf];
    xs[row * R + r] = (TC)v;
  }
  __syncthreads();
  if (a.b_y != 0.0 && d.e_n > 0) {
    for (int t = tid; t < d.e_n * Rg; t += nt) {
      const int i = t / Rg, r = t - i * Rg;
      const int row = B.e_row[d.e_row + i];
      const int e0 = B.e_ptr[d.e_ptr + i], e1 = B.e_ptr[d.e_ptr + i + 1];
      const double *yc = a.y + (int64_t)(c0 + r) * a.ldy;
      TC acc = 0;
      for (int e = e0; e < e1; ++e) acc += cvt<TC>(B.e_val[e]) * (TC)yc[B.e_q[e]];
      xs[row * R + r] += (TC)a.b_y * acc;
    }
    __syncthreads();
  }
  sweep_lds<TS, TC>(B.fwd, d.f_row, d.f_rp, levf, d.f_nlev, xs, R, Rg);
  sweep_lds<TS, TC>(B.bwd, d.b_row, d.b_rp, levb, d.b_nlev, xs, R, Rg);
  if (a.u) {
    for (int t = tid; t < m * Rg; t += nt) {
      const int r = t / m, row = t - r * m;
      a.u[(int64_t)(d.m0 + row) + (int64_t)(c0 + r) * a.ldu] = (double)xs[row * R + r];
    }
  }
  if (a.gout) {
    for (int t = tid; t < d.t_n * Rg; t += nt) {
      const int i = t / Rg, r = t - i * Rg;
      const int q = B.t_q[d.t_row + i];
      const int e0 = B.t_ptr[d.t_ptr + i], e1 = B.t_ptr[d.t_ptr + i + 1];
      TC acc = 0;
      for (int e = e0; e < e1; ++e) acc += cvt<TC>(B.t_val[e]) * xs[B.t_j[e] * R + r];
      double gv = a.c_g != 0.0 ? a.c_g * a.g[q + (int64_t)(c0 + r) * a.ldg] : 0.0;
      a.gout[q + (int64_t)(c0 + r) * a.ldgo] = gv + a.d_t * (double)acc;
    }
  }
}

template <typename TS, typename TC>
void launch_bsolve(const BlockArrays<TS> &B, int32_t p, const BArgs &a, int32_t threads,
                   size_t lds_bytes, hipStream_t st) {
  static size_t attr_bytes = 0;
  if (lds_bytes > 65536 && lds_bytes > attr_bytes) {
    (void)hipFuncSetAttribute((const void *)k_bsolve<TS, TC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    attr_bytes = lds_bytes;
  }
  dim3 grid(p, (a.nrhs + a.R - 1) / a.R);
  hipLaunchKernelGGL((k_bsolve<TS, TC>), grid, dim3(threads), lds_bytes, st, B, a);
}

// ---------------------------------------------------------------------------
// K3: interface sweeps (L^{-1}, L^{-T}) on a global vector
// ---------------------------------------------------------------------------
template <typename TS, typename TC>
__device__ __forceinline__ void sweep_row(const SweepArrays<TS> &S, int slot, double *xc) {
  const int row = S.rows[slot];
  const int e0 = S.rp[slot], e1 = S.rp[slot + 1];
  TC acc = cvt<TC>(S.sc[slot]) * (TC)xc[row];
  for (int e = e0; e < e1; ++e) acc -= cvt<TC>(S.w[e]) * (TC)xc[S.ci[e]];
  xc[row] = (double)acc;
}

template <typename TS, typename TC>
__global__ void __launch_bounds__(1024) k_sweep_wg(SweepArrays<TS> S, int nlev, double *x, int64_t ldx) {
  extern __shared__ int32_t lev[];
  for (int i = threadIdx.x; i <= nlev; i += blockDim.x) lev[i] = S.lev[i];
  __syncthreads();
  double *xc = x + (int64_t)blockIdx.x * ldx;
  for (int l = 0; l < nlev; ++l) {
    const int a = lev[l], b = lev[l + 1];
    for (int t = a + threadIdx.x; t < b; t += blockDim.x) sweep_row<TS, TC>(S, t, xc);
    __syncthreads();
  }
}

template <typename TS, typename TC>
__global__ void __launch_bounds__(256) k_sweep_lvl(SweepArrays<TS> S, int a, int b, double *x, int64_t ldx) {
  const int t = a + blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b) return;
  sweep_row<TS, TC>(S, t, x + (int64_t)blockIdx.y * ldx);
}

template <typename TS, typename TC>
void launch_sweep(const SweepArrays<TS> &S, const int32_t *lev_host, int32_t nlev, int32_t nrows,
                  double *x, int64_t ldx, int32_t nrhs, bool one_wg, hipStream_t st) {
  if (nlev == 0 || nrhs == 0) return;
  if (one_wg) {
    hipLaunchKernelGGL((k_sweep_wg<TS, TC>), dim3(nrhs), dim3(512), sizeof(int32_t) * (nlev + 1), st, S,
                       nlev, x, ldx);
    return;
  }
  for (int l = 0; l < nlev; ++l) {
    const int a = lev_host[l], b = lev_host[l + 1];
    if (b <= a) continue;
    dim3 grid((b - a + 255) / 256, nrhs);
    hipLaunchKernelGGL((k_sweep_lvl<TS, TC>), grid, dim3(256), 0, st, S, a, b, x, ldx);
  }
}

// ---------------------------------------------------------------------------
// K4: rank-k block of eq. skt.  U row-major (s x k).
//   part[b][r][kk] = sum_{i in chunk b} U[i,kk] w[i,r]; the last block
//   sums the partials in block order and scales by dsc (-> cbuf[r*k+kk]);
//   then wout = rho w + U cbuf.
// ---------------------------------------------------------------------------
constexpr int LR_THREADS = 256;
constexpr int LR_COLS = 8;   // right-hand sides per pass

template <typename TU>
__global__ void __launch_bounds__(LR_THREADS) k_lr_partial(const TU *U, int64_t s, int k, int kpad,
                                                          const double *w, int64_t ldw, int nrhs,
                                                          double *part, double *cbuf, const double *dsc,
                                                          unsigned int *counter) {
  __shared__ double red[LR_THREADS / 64][64][LR_COLS];
  const int nb = gridDim.x;
  const int64_t chunk = (s + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(s, i0 + chunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int rpw = 64 / kpad;           // rows per wave
  const int sub = lane / kpad, kk = lane - sub * kpad;
  const int nw = LR_THREADS / 64;
  for (int c0 = 0; c0 < nrhs; c0 += LR_COLS) {
    const int nc = min(LR_COLS, nrhs - c0);
    double acc[LR_COLS];
#pragma unroll
    for (int r = 0; r < LR_COLS; ++r) acc[r] = 0.0;
    for (int64_t i = i0 + wid * rpw + sub; i < i1; i += nw * rpw) {
      const double u = (kk < k) ? cvt<double>(U[i * k + kk]) : 0.0;
#pragma unroll
      for (int r = 0; r < LR_COLS; ++r)
        if (r < nc) acc[r] += u * w[i + (int64_t)(c0 + r) * ldw];
    }
    // fold the rpw sub-rows of the wave, then the waves (fixed order)
#pragma unroll
    for (int r = 0; r < LR_COLS; ++r) {
      double v = acc[r];
      for (int o = kpad; o < 64; o <<= 1) v += __shfl_down(v, o, 64);
      acc[r] = v;
    }
    __syncthreads();
    if (sub == 0)
      for (int r = 0; r < LR_COLS; ++r) red[wid][kk][r] = acc[r];
    __syncthreads();
    for (int t = threadIdx.x; t < k * nc; t += blockDim.x) {
      const int r = t / k, q = t - r * k;
      double v = 0.0;
      for (int ww = 0; ww < nw; ++ww) v += red[ww][q][r];
      part[((int64_t)blockIdx.x * nrhs + c0 + r) * k + q] = v;
    }
  }
  if (last_block(counter)) {
    for (int t = threadIdx.x; t < k * nrhs; t += blockDim.x) {
      double v = 0.0;
      for (int b = 0; b < nb; ++b) v += part[(int64_t)b * nrhs * k + t];
      cbuf[t] = v * dsc[t % k];
    }
  }
}

template <typename TU>
__global__ void __launch_bounds__(256) k_lr_update(const TU *U, int64_t s, int k, const double *w,
                                                  int64_t ldw, double *wout, int64_t ldo, int nrhs,
                                                  const double *cbuf, double rho) {
  extern __shared__ double cs[];
  for (int t = threadIdx.x; t < k * nrhs; t += blockDim.x) cs[t] = cbuf[t];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s) return;
  for (int c0 = 0; c0 < nrhs; c0 += LR_COLS) {
    const int nc = min(LR_COLS, nrhs - c0);
    double acc[LR_COLS];
#pragma unroll
    for (int r = 0; r < LR_COLS; ++r) acc[r] = 0.0;
    for (int q = 0; q < k; ++q) {
      const double u = cvt<double>(U[i * k + q]);
#pragma unroll
      for (int r = 0; r < LR_COLS; ++r)
        if (r < nc) acc[r] += u * cs[(c0 + r) * k + q];
    }
    for (int r = 0; r < nc; ++r)
      wout[i + (int64_t)(c0 + r) * ldo] = rho * w[i + (int64_t)(c0 + r) * ldw] + acc[r];
  }
}

template <typename TU>
void launch_lowrank(const TU *U, int64_t s, int32_t k, const double *dsc, double rho,
                    const double *w, int64_t ldw, double *wout, int64_t ldo, int32_t nrhs,
                    double *part, int32_t nblk, double *cbuf, unsigned int *counter,
                    hipStream_t st) {
  if (s == 0 || nrhs == 0) return;
  if (k == 0) {
    launch_axpby(s, nrhs, rho, w, ldw, 0.0, wout, ldo, st);
    return;
  }
  int kpad = 1;
  while (kpad < k && kpad < 64) kpad <<= 1;
  if (k > 64) kpad = 64;  // lanes loop is not used for k > 64 (rejected at setup)
  hipLaunchKernelGGL((k_lr_partial<TU>), dim3(nblk), dim3(LR_THREADS), 0, st, U, s, k, kpad, w, ldw,
                     nrhs, part, cbuf, dsc, counter);
  hipLaunchKernelGGL((k_lr_update<TU>), dim3((unsigned)((s + 255) / 256)), dim3(256),
                     sizeof(double) * k * nrhs, st, U, s, k, w, ldw, wout, ldo, nrhs, cbuf, rho);
}

// ---------------------------------------------------------------------------
// Vector utilities
// ---------------------------------------------------------------------------
__global__ void k_axpby(int64_t n, int nrhs, double a, const double *x, int64_t ldx, double b, double *y,
                        int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = blockIdx.y;
  double v = a * x[i + r * ldx];
  if (b != 0.0) v += b * y[i + r * ldy];
  y[i + r * ldy] = v;
}

void launch_axpby(int64_t n, int32_t nrhs, double a, const double *x, int64_t ldx, double b, double *y,
                  int64_t ldy, hipStream_t st) {
  if (n == 0 || nrhs == 0) return;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, st, n, nrhs, a, x,
                     ldx, b, y, ldy);
}

// dst[t] = src[idx[t]] (gather) or dst[idx[t]] = src[t] (scatter), per column
__global__ void k_permute(int64_t n, const int64_t *idx, const double *src, int64_t lds, double *dst,
                          int64_t ldd, int scatter) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int r = blockIdx.y;
  if (scatter)
    dst[idx[t] + r * ldd] = src[t + r * lds];
  else
    dst[t + r * ldd] = src[idx[t] + r * lds];
}

void launch_permute(int64_t n, const int64_t *idx, const double *src, int64_t lds, double *dst, int64_t ldd,
                    int32_t nrhs, bool scatter, hipStream_t st) {
  if (n == 0 || nrhs == 0) return;
  hipLaunchKernelGGL(k_permute, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, st, n, idx, src, lds,
                     dst, ldd, scatter ? 1 : 0);
}

// ---------------------------------------------------------------------------
// K5: CSR SpMV y = A x (FP64, A in the internal order)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_spmv(int64_t n, const int64_t *rp, const int32_t *ci,
                                              const double *v, const double *x, int64_t ldx, double *y,
                                              int64_t ldy) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *xc = x + (int64_t)blockIdx.y * ldx;
  double acc = 0.0;
  for (int64_t e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * xc[ci[e]];
  y[i + (int64_t)blockIdx.y * ldy] = acc;
}

void launch_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                 int64_t ldx, double *y, int64_t ldy, int32_t nrhs, hipStream_t st) {
  if (n == 0 || nrhs == 0) return;
  hipLaunchKernelGGL(k_spmv, dim3((unsigned)((n + 255) / 256), nrhs), dim3(256), 0, st, n, rp, ci, v, x, ldx,
                     y, ldy);
}

// ---------------------------------------------------------------------------
// K6: Krylov BLAS-1 with fused deterministic reductions.
// KState holds per-column scalars; see slr_kern.h for the field meaning.
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

// Shared tail: partial[b][col] written by each block; the last block sums.
__device__ double fold_partials(const double *part, int nb, int ncol, int col) {
  double v = 0.0;
  for (int b = 0; b < nb; ++b) v += part[(int64_t)b * ncol + col];
  return v;
}

// q = A p for active columns, and p.q ; then alpha = rz / pq.
__global__ void __launch_bounds__(RED_THREADS) k_cg_spmv(int64_t n, const int64_t *rp, const int32_t *ci,
                                                         const double *v, KArgs K, int c0, int nc) {
  __shared__ double sh[RED_THREADS / 64];
  const int nb = gridDim.x;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    const double *pc = K.P + (int64_t)c * K.ld;
    double *qc = K.Q + (int64_t)c * K.ld;
    double acc = 0.0;
    if (K.st[c].active) {
      for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        double sum = 0.0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) sum += v[e] * pc[ci[e]];
        qc[i] = sum;
        acc += sum * pc[i];
      }
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) K.part[(int64_t)blockIdx.x * nc + cc] = t;
  }
  if (last_block(K.counter)) {
    for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
      KState &s = K.st[c0 + cc];
      const double pq = fold_partials(K.part, nb, nc, cc);
      if (s.active) {
        if (!(pq > 0.0) || !isfinite(pq)) {
          // indefinite or broken down: stop this column
          s.active = 0;
          s.status = -8;
          s.alpha = 0.0;
        } else {
          s.alpha = s.rz / pq;
        }
      } else {
        s.alpha = 0.0;
      }
    }
  }
}

// x += alpha p ; r -= alpha q ; rr = r.r ; convergence and iteration count
__global__ void __launch_bounds__(RED_THREADS) k_cg_update(int64_t n, KArgs K, int c0, int nc) {
  __shared__ double sh[RED_THREADS / 64];
  const int nb = gridDim.x;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    const KState &s = K.st[c];
    double acc = 0.0;
    if (s.active) {
      const double al = s.alpha;
      double *xc = K.X + (int64_t)c * K.ld;
      double *rc = K.R + (int64_t)c * K.ld;
      const double *pc = K.P + (int64_t)c * K.ld;
      const double *qc = K.Q + (int64_t)c * K.ld;
      for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        xc[i] += al * pc[i];
        const double r = rc[i] - al * qc[i];
        rc[i] = r;
        acc += r * r;
      }
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) K.part[(int64_t)blockIdx.x * nc + cc] = t;
  }
  if (last_block(K.counter)) {
    for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
      KState &s = K.st[c0 + cc];
      if (!s.active) continue;
      const double rr = fold_partials(K.part, nb, nc, cc);
      s.rr = rr;
      s.iters += 1;
      if (rr <= K.rtol2 * s.bb) {
        s.active = 0;
        s.status = 0;
      } else if (s.iters >= K.maxit || !isfinite(rr)) {
        s.active = 0;
        s.status = -8;
      }
    }
  }
}

// rz_new = r.z, zq = z.q ; beta (CG: rz_new/rz, flexible CG: -alpha zq/rz)
__global__ void __launch_bounds__(RED_THREADS) k_cg_beta(int64_t n, KArgs K, int c0, int nc, int flexible,
                                                         int init) {
  __shared__ double sh[RED_THREADS / 64];
  const int nb = gridDim.x;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    const KState &s = K.st[c];
    double a1 = 0.0, a2 = 0.0;
    if (s.active) {
      const double *rc = K.R + (int64_t)c * K.ld;
      const double *zc = K.Z + (int64_t)c * K.ld;
      const double *qc = K.Q + (int64_t)c * K.ld;
      for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        a1 += rc[i] * zc[i];
        if (flexible && !init) a2 += zc[i] * qc[i];
      }
    }
    double t1 = block_sum(a1, sh);
    double t2 = block_sum(a2, sh);
    if (threadIdx.x == 0) {
      K.part[((int64_t)blockIdx.x * nc + cc) * 2] = t1;
      K.part[((int64_t)blockIdx.x * nc + cc) * 2 + 1] = t2;
    }
  }
  if (last_block(K.counter)) {
    for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
      KState &s = K.st[c0 + cc];
      double rz = 0.0, zq = 0.0;
      for (int b = 0; b < nb; ++b) {
        rz += K.part[((int64_t)b * nc + cc) * 2];
        zq += K.part[((int64_t)b * nc + cc) * 2 + 1];
      }
      if (!s.active) {
        s.beta = 0.0;
        continue;
      }
      if (init) {
        s.beta = 0.0;
      } else {
        s.beta = flexible ? (-s.alpha * zq) / s.rz : rz / s.rz;
      }
      s.rz = rz;
    }
  }
}

// p = z + beta p (active columns)
__global__ void k_cg_p(int64_t n, KArgs K, int c0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = c0 + blockIdx.y;
  const KState &s = K.st[c];
  if (i >= n || !s.active) return;
  double *pc = K.P + (int64_t)c * K.ld;
  pc[i] = K.Z[i + (int64_t)c * K.ld] + s.beta * pc[i];
}

// column-wise squared norms into st[c].bb and reset the state (init)
__global__ void __launch_bounds__(RED_THREADS) k_cg_init(int64_t n, KArgs K, int c0, int nc) {
  __shared__ double sh[RED_THREADS / 64];
  const int nb = gridDim.x;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    const double *rc = K.R + (int64_t)c * K.ld;
    double *xc = K.X + (int64_t)c * K.ld;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      acc += rc[i] * rc[i];
      xc[i] = 0.0;
    }
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) K.part[(int64_t)blockIdx.x * nc + cc] = t;
  }
  if (last_block(K.counter)) {
    for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
      KState &s = K.st[c0 + cc];
      const double bb = fold_partials(K.part, nb, nc, cc);
      s.bb = bb;
      s.rr = bb;
      s.iters = 0;
      s.alpha = s.beta = s.rz = 0.0;
      s.relres = 0.0;
      if (bb > 0.0 && isfinite(bb)) {
        s.active = 1;
        s.status = -8;
      } else {
        s.active = 0;
        s.status = isfinite(bb) ? 0 : -8;
      }
    }
  }
}

// relres = ||b - A x|| / ||b|| (Q holds A x on entry, R0 = b)
__global__ void __launch_bounds__(RED_THREADS) k_relres(int64_t n, const double *B, int64_t ldb, const double *AX,
                                                        int64_t ldax, KArgs K, int c0, int nc) {
  __shared__ double sh[RED_THREADS / 64];
  const int nb = gridDim.x;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    double acc = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      const double d = B[i + (int64_t)cc * ldb] - AX[i + (int64_t)cc * ldax];
      acc += d * d;
    }
    (void)c;
    double t = block_sum(acc, sh);
    if (threadIdx.x == 0) K.part[(int64_t)blockIdx.x * nc + cc] = t;
  }
  if (last_block(K.counter)) {
    for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
      KState &s = K.st[c0 + cc];
      const double rr = fold_partials(K.part, nb, nc, cc);
      s.relres = s.bb > 0.0 ? sqrt(rr / s.bb) : 0.0;
    }
  }
}

void launch_cg(int op, int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const KArgs &K,
               int32_t c0, int32_t nc, int32_t flexible, hipStream_t st) {
  if (nc == 0) return;
  const int nb = K.nblk;
  switch (op) {
    case CG_INIT:
      hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(RED_THREADS), 0, st, n, K, c0, nc);
      break;
    case CG_SPMV:
      hipLaunchKernelGGL(k_cg_spmv, dim3(nb), dim3(RED_THREADS), 0, st, n, rp, ci, v, K, c0, nc);
      break;
    case CG_UPDATE:
      hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(RED_THREADS), 0, st, n, K, c0, nc);
      break;
    case CG_BETA:
      hipLaunchKernelGGL(k_cg_beta, dim3(nb), dim3(RED_THREADS), 0, st, n, K, c0, nc, flexible, 0);
      break;
    case CG_BETA_INIT:
      hipLaunchKernelGGL(k_cg_beta, dim3(nb), dim3(RED_THREADS), 0, st, n, K, c0, nc, flexible, 1);
      break;
    case CG_P:
      hipLaunchKernelGGL(k_cg_p, dim3((unsigned)((n + 255) / 256), nc), dim3(256), 0, st, n, K, c0);
      break;
    default:
      break;
  }
}

void launch_relres(int64_t n, const double *B, int64_t ldb, const double *AX, int64_t ldax, const KArgs &K,
                   int32_t c0, int32_t nc, hipStream_t st) {
  if (nc == 0) return;
  hipLaunchKernelGGL(k_relres, dim3(K.nblk), dim3(RED_THREADS), 0, st, n, B, ldb, AX, ldax, K, c0, nc);
}

// ---------------------------------------------------------------------------
// Single-vector reductions / Gram-Schmidt (Lanczos K7 and FGMRES K10), FP64
// ---------------------------------------------------------------------------
// out[j] = sum_i V[i + j*ldv] * w[i]  for j < J   (V^T w)
// Each block takes a contiguous row chunk; wave j-lanes reduce; the last
// block folds the partials (part: nblk x J) in block order.
__global__ void __launch_bounds__(256) k_multidot(int64_t s, int J, const double *V, int64_t ldv,
                                                  const double *w, double *part, double *out, double scale_out,
                                                  unsigned int *counter) {
  const int nb = gridDim.x;
  const int64_t chunk = (s + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(s, i0 + chunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = wid; j < J; j += nw) {
    const double *vj = V + (int64_t)j * ldv;
    double acc = 0.0;
    for (int64_t i = i0 + lane; i < i1; i += 64) acc += vj[i] * w[i];
    acc = wave_sum(acc);
    if (lane == 0) part[(int64_t)blockIdx.x * J + j] = acc;
  }
  if (last_block(counter)) {
    for (int j = threadIdx.x; j < J; j += blockDim.x) {
      double v = 0.0;
      for (int b = 0; b < nb; ++b) v += part[(int64_t)b * J + j];
      out[j] = v * scale_out;
    }
  }
}

// w[i] -= sum_j V[i + j*ldv] h[j]   (h on the device, J <= 1024)
__global__ void __launch_bounds__(256) k_gemv_sub(int64_t s, int J, const double *V, int64_t ldv,
                                                  const double *h, double *w) {
  __shared__ double hs[1024];
  for (int j = threadIdx.x; j < J; j += blockDim.x) hs[j] = h[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s) return;
  double acc = 0.0;
  for (int j = 0; j < J; ++j) acc += V[i + (int64_t)j * ldv] * hs[j];
  w[i] -= acc;
}

void launch_multidot(int64_t s, int32_t J, const double *V, int64_t ldv, const double *w, double *part,
                     int32_t nblk, double *out, unsigned int *counter, hipStream_t st) {
  hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(256), 0, st, s, J, V, ldv, w, part, out, 1.0, counter);
}

void launch_gemv_sub(int64_t s, int32_t J, const double *V, int64_t ldv, const double *h, double *w,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_sub, dim3((unsigned)((s + 255) / 256)), dim3(256), 0, st, s, J, V, ldv, h, w);
}

// Lanczos three-term step: a = v.w computed by multidot into sc[0];
//   w -= a v + b_prev v_prev   (b_prev = sc[1])
__global__ void k_lanczos_axpy(int64_t s, double *w, const double *v, const double *vprev, const double *sc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s) return;
  double t = w[i] - sc[0] * v[i];
  if (vprev) t -= sc[1] * vprev[i];
  w[i] = t;
}

void launch_lanczos_axpy(int64_t s, double *w, const double *v, const double *vprev, const double *sc,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_lanczos_axpy, dim3((unsigned)((s + 255) / 256)), dim3(256), 0, st, s, w, v, vprev, sc);
}

// v_next = w / beta, beta = sqrt(sc[2]) (sc[2] holds w.w)
__global__ void k_scale_inv_sqrt(int64_t s, const double *w, double *out, const double *nrm2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s) return;
  const double b = sqrt(*nrm2);
  out[i] = b > 0.0 ? w[i] / b : 0.0;
}

void launch_scale_inv_sqrt(int64_t s, const double *w, double *out, const double *nrm2, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv_sqrt, dim3((unsigned)((s + 255) / 256)), dim3(256), 0, st, s, w, out, nrm2);
}

// x += V y  (V: n x J, y on the device)
__global__ void __launch_bounds__(256) k_gemv_add(int64_t n, int J, const double *V, int64_t ldv,
                                                  const double *y, double *x) {
  __shared__ double ys[1024];
  for (int j = threadIdx.x; j < J; j += blockDim.x) ys[j] = y[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < J; ++j) acc += V[i + (int64_t)j * ldv] * ys[j];
  x[i] += acc;
}

void launch_gemv_add(int64_t n, int32_t J, const double *V, int64_t ldv, const double *y, double *x,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, J, V, ldv, y, x);
}

// ---------------------------------------------------------------------------
// FGMRES small dense work (one thread): Givens update of column j of the
// Hessenberg matrix and the least-squares residual (Saad's flexible GMRES).
// g: restart+1, cs/sn: restart, Hm: (restart+1) x restart column-major.
// hcol: the j+1 projections of this step (two CGS passes summed), hn2: w.w
// flags[0] <- 1 when |g_{j+1}| <= tol.
// ---------------------------------------------------------------------------
__global__ void k_gmres_givens(int j, int ldh, double *Hm, const double *h1, const double *h2, const double *hn2,
                               double *cs, double *sn, double *g, double tol, int *flags, double *vscale) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double *hc = Hm + (int64_t)j * ldh;
  for (int i = 0; i <= j; ++i) hc[i] = h1[i] + h2[i];
  const double hn = sqrt(*hn2);
  hc[j + 1] = hn;
  *vscale = hn;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * hc[i] + sn[i] * hc[i + 1];
    hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
    hc[i] = t;
  }
  const double den = hypot(hc[j], hc[j + 1]);
  cs[j] = den > 0.0 ? hc[j] / den : 1.0;
  sn[j] = den > 0.0 ? hc[j + 1] / den : 0.0;
  hc[j] = den;
  hc[j + 1] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  flags[0] = (fabs(g[j + 1]) <= tol) ? 1 : 0;
  flags[1] = (hn == 0.0) ? 1 : 0;
}

// y = R^{-1} g for the leading jj x jj upper-triangular part of Hm
__global__ void k_gmres_solve(int jj, int ldh, const double *Hm, const double *g, double *y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = jj - 1; i >= 0; --i) {
    double t = g[i];
    for (int c = i + 1; c < jj; ++c) t -= Hm[i + (int64_t)c * ldh] * y[c];
    y[i] = t / Hm[i + (int64_t)i * ldh];
  }
}

void launch_gmres_givens(int32_t j, int32_t ldh, double *Hm, const double *h1, const double *h2,
                         const double *hn2, double *cs, double *sn, double *g, double tol, int *flags,
                         double *vscale, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_givens, dim3(1), dim3(64), 0, st, j, ldh, Hm, h1, h2, hn2, cs, sn, g, tol, flags,
                     vscale);
}

void launch_gmres_solve(int32_t jj, int32_t ldh, const double *Hm, const double *g, double *y, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_solve, dim3(1), dim3(64), 0, st, jj, ldh, Hm, g, y);
}

// v = w / *scale
__global__ void k_div_scalar(int64_t n, const double *w, double *v, const double *scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = *scale;
  v[i] = sc != 0.0 ? w[i] / sc : 0.0;
}

void launch_div_scalar(int64_t n, const double *w, double *v, const double *scale, hipStream_t st) {
  hipLaunchKernelGGL(k_div_scalar, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, w, v, scale);
}

// ---------------------------------------------------------------------------
// K8: eigen-decomposition of the Lanczos tridiagonal T_m (m <= 1024) in one
// workgroup: implicit QL iterations with Wilkinson shifts (the tql2
// procedure of Bowdler, Martin, Reinsch & Wilkinson) computed by thread 0,
// the plane rotations accumulated into Z by all threads (each thread owns
// whole rows of Z).  Outputs: eval (descending, all m), Y (m x K, column j
// = eigenvector of the j-th largest), info (0 ok, 1 no convergence).
// Z: m x m scratch (row-major).
// ---------------------------------------------------------------------------
constexpr int EIG_MAXM = 1024;

__global__ void __launch_bounds__(256) k_tridiag_eig(int m, const double *alpha, const double *beta, double *Z,
                                                     double *eval, double *Y, int K, int *info) {
  __shared__ double d[EIG_MAXM], e[EIG_MAXM], cs[EIG_MAXM], sn[EIG_MAXM];
  __shared__ int ctl[4];  // [0]=lo, [1]=hi (rotations i = hi..lo), [2]=done, [3]=fail
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < m; i += nt) {
    d[i] = alpha[i];
    e[i] = (i + 1 < m) ? beta[i] : 0.0;
  }
  for (int64_t t = tid; t < (int64_t)m * m; t += nt) Z[t] = ((t / m) == (t % m)) ? 1.0 : 0.0;
  if (tid == 0) ctl[3] = 0;
  __syncthreads();
  int failed = 0;
  for (int l = 0; l < m; ++l) {
    int iter = 0;
    while (true) {
      if (tid == 0) {
        int mm = l;
        for (; mm < m - 1; ++mm) {
          const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
          if (fabs(e[mm]) <= 2.220446049250313e-16 * dd) break;
        }
        ctl[2] = (mm == l) ? 1 : 0;
        ctl[0] = l;
        ctl[1] = l - 1;  // empty range by default
        if (mm != l) {
          if (++iter > 60) {
            ctl[3] = 1;
            ctl[2] = 1;
          } else {
            // Wilkinson shift from the leading 2x2 block
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? fabs(r) : -fabs(r)));
            double s = 1.0, c = 1.0, p = 0.0;
            int i = mm - 1;
            bool early = false;
            for (; i >= l; --i) {
              double f = s * e[i];
              double b = c * e[i];
              r = hypot(f, g);
              e[i + 1] = r;
              if (r == 0.0) {
                d[i + 1] -= p;
                e[mm] = 0.0;
                early = true;
                break;
              }
              s = f / r;
              c = g / r;
              g = d[i + 1] - p;
              r = (d[i] - g) * s + 2.0 * c * b;
              p = s * r;
              d[i + 1] = g + p;
              g = c * r - b;
              cs[i] = c;
              sn[i] = s;
            }
            // rotations recorded for indices (early ? i+1 : l) .. mm-1
            ctl[0] = early ? i + 1 : l;
            ctl[1] = mm - 1;
            if (!early) {
              d[l] -= p;
              e[l] = g;
              e[mm] = 0.0;
            }
          }
        }
      }
      __syncthreads();
      const int lo = ctl[0], hi = ctl[1];
      for (int row = tid; row < m; row += nt) {
        double *zr = Z + (int64_t)row * m;
        for (int i = hi; i >= lo; --i) {
          const double f = zr[i + 1];
          zr[i + 1] = sn[i] * zr[i] + cs[i] * f;
          zr[i] = cs[i] * zr[i] - sn[i] * f;
        }
      }
      // read the control words before the barrier: thread 0 rewrites them
      // only after it
      const int done = ctl[2];
      failed = ctl[3];
      __syncthreads();
      if (done) break;
    }
    if (failed) break;
  }
  __syncthreads();
  // rank by decreasing eigenvalue (ties by index) and gather
  for (int i = tid; i < m; i += nt) {
    int rank = 0;
    for (int j = 0; j < m; ++j) rank += (d[j] > d[i]) || (d[j] == d[i] && j < i);
    eval[rank] = d[i];
    if (rank < K)
      for (int r = 0; r < m; ++r) Y[r + (int64_t)rank * m] = Z[(int64_t)r * m + i];
  }
  if (tid == 0) *info = failed;
}

void launch_tridiag_eig(int32_t m, const double *alpha, const double *beta, double *Z, double *eval, double *Y,
                        int32_t K, int *info, hipStream_t st) {
  hipLaunchKernelGGL(k_tridiag_eig, dim3(1), dim3(256), 0, st, m, alpha, beta, Z, eval, Y, K, info);
}

// Ritz vectors: U64[i, q] = sum_j V[i, j] Y[j, q]  (V: s x m col-major,
// Y: m x K col-major, U64 row-major s x k, k <= K).  Also writes the
// storage copy U (row-major, rounded to TU).
template <typename TU>
__global__ void __launch_bounds__(256) k_ritz(int64_t s, int m, int k, const double *V, int64_t ldv,
                                              const double *Y, double *U64, TU *U) {
  extern __shared__ double ys[];  // m x 16 tile (m <= 1024: 128 KiB)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int q0 = 0; q0 < k; q0 += 16) {
    const int nq = min(16, k - q0);
    __syncthreads();
    for (int t = threadIdx.x; t < m * nq; t += blockDim.x) {
      const int q = t / m, j = t - q * m;
      ys[j * 16 + q] = Y[j + (int64_t)(q0 + q) * m];
    }
    __syncthreads();
    if (i < s) {
      double acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0;
      for (int j = 0; j < m; ++j) {
        const double vj = V[i + (int64_t)j * ldv];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] += vj * ys[j * 16 + q];
      }
      for (int q = 0; q < nq; ++q) {
        U64[i * k + q0 + q] = acc[q];
        U[i * k + q0 + q] = round_store<TU>(acc[q]);
      }
    }
  }
}

template <typename TU>
void launch_ritz(int64_t s, int32_t m, int32_t k, const double *V, int64_t ldv, const double *Y, double *U64,
                 TU *U, hipStream_t st) {
  if (s == 0 || k == 0) return;
  const size_t lds = sizeof(double) * m * 16;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void *)k_ritz<TU>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL((k_ritz<TU>), dim3((unsigned)((s + 255) / 256)), dim3(256), lds, st, s, m, k, V, ldv, Y,
                     U64, U);
}

// storage copy of a row-major FP64 U (import path)
template <typename TU>
__global__ void k_round_copy(int64_t n, const double *src, TU *dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = round_store<TU>(src[i]);
}

template <typename TU>
void launch_round_copy(int64_t n, const double *src, TU *dst, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL((k_round_copy<TU>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, src, dst);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------
template void launch_bsolve<double, double>(const BlockArrays<double> &, int32_t, const BArgs &, int32_t, size_t,
                                            hipStream_t);
template void launch_bsolve<float, float>(const BlockArrays<float> &, int32_t, const BArgs &, int32_t, size_t,
                                          hipStream_t);
template void launch_bsolve<float, double>(const BlockArrays<float> &, int32_t, const BArgs &, int32_t, size_t,
                                           hipStream_t);
template void launch_sweep<double, double>(const SweepArrays<double> &, const int32_t *, int32_t, int32_t, double *,
                                           int64_t, int32_t, bool, hipStream_t);
template void launch_sweep<float, float>(const SweepArrays<float> &, const int32_t *, int32_t, int32_t, double *,
                                         int64_t, int32_t, bool, hipStream_t);
template void launch_sweep<float, double>(const SweepArrays<float> &, const int32_t *, int32_t, int32_t, double *,
                                          int64_t, int32_t, bool, hipStream_t);
template void launch_lowrank<double>(const double *, int64_t, int32_t, const double *, double, const double *,
                                     int64_t, double *, int64_t, int32_t, double *, int32_t, double *,
                                     unsigned int *, hipStream_t);
template void launch_lowrank<float>(const float *, int64_t, int32_t, const double *, double, const double *,
                                    int64_t, double *, int64_t, int32_t, double *, int32_t, double *, unsigned int *,
                                    hipStream_t);
template void launch_lowrank<__hip_bfloat16>(const __hip_bfloat16 *, int64_t, int32_t, const double *, double,
                                             const double *, int64_t, double *, int64_t, int32_t, double *, int32_t,
                                             double *, unsigned int *, hipStream_t);
template void launch_ritz<double>(int64_t, int32_t, int32_t, const double *, int64_t, const double *, double *,
                                  double *, hipStream_t);
template void launch_ritz<float>(int64_t, int32_t, int32_t, const double *, int64_t, const double *, double *,
                                 float *, hipStream_t);
template void launch_ritz<__hip_bfloat16>(int64_t, int32_t, int32_t, const double *, int64_t, const double *,
                                          double *, __hip_bfloat16 *, hipStream_t);
template void launch_round_copy<double>(int64_t, const double *, double *, hipStream_t);
template void launch_round_copy<float>(int64_t, const double *, float *, hipStream_t);
template void launch_round_copy<__hip_bfloat16>(int64_t, const double *, __hip_bfloat16 *, hipStream_t);

}  // namespace slr

namespace slr {

// Lanczos bookkeeping of step j: alpha[j] = sc[0], beta[j] = sqrt(sc[2]),
// and sc[1] <- beta[j] for the next three-term step.
__global__ void k_lanczos_record(int j, double *sc, double *alpha, double *beta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    alpha[j] = sc[0];
    const double b = sqrt(sc[2]);
    beta[j] = b;
    sc[1] = b;
  }
}

void launch_lanczos_record(int32_t j, double *sc, double *alpha, double *beta, hipStream_t st) {
  hipLaunchKernelGGL(k_lanczos_record, dim3(1), dim3(64), 0, st, j, sc, alpha, beta);
}

// g = [sqrt(*nrm2), 0, ..., 0] (length len)
__global__ void k_gmres_g0(int len, const double *nrm2, double *g) {
  for (int i = threadIdx.x; i < len; i += blockDim.x) g[i] = (i == 0) ? sqrt(*nrm2) : 0.0;
}

void launch_gmres_g0(int32_t len, const double *nrm2, double *g, hipStream_t st) {
  hipLaunchKernelGGL(k_gmres_g0, dim3(1), dim3(256), 0, st, len, nrm2, g);
}

}  // namespace slr

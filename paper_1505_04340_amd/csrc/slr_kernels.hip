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
// Reductions are deterministic and use no cross-block atomics or fences:
// every block writes a partial; after the kernel boundary either a small
// fold kernel or each consumer block sums the partials in a fixed order
// (lane-strided over blocks, then a fixed shuffle tree).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
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

// sum over the wave, valid in every lane
__device__ __forceinline__ double wave_allsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// max over the wave, valid in every lane
__device__ __forceinline__ double wave_allmax(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
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

// Lane `lane`'s share of a fold: part[b*ld + col] summed over b = lane,
// lane + 64, ... < nb, added in that order.  The loads go out eight at a
// time, so a fold of up to 512 partials costs one memory round trip.
__device__ __forceinline__ double lane_fold(const double *part, int nb, int64_t ld, int col, int lane) {
  double v = 0.0;
  for (int b0 = 0; b0 < nb; b0 += 8 * 64) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + lane + u * 64;
      t[u] = b < nb ? part[(int64_t)b * ld + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + lane + u * 64 < nb) v += t[u];
  }
  return v;
}

// N block sums at once (the same arithmetic as N calls of block_sum, with
// one pair of barriers); sh holds N * nw values, results in thread 0's v.
template <int N>
__device__ void block_sums(double *v, double *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < N; ++j) sh[j * nw + wid] = v[j];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double r = 0.0;
      for (int i = 0; i < nw; ++i) r += sh[j * nw + i];
      v[j] = r;
    }
}

// Deterministic parallel fold of per-block partials laid out part[b*ncol+col]:
// each wave folds whole columns (lanes stride over b, then a shuffle tree);
// f(col, value) runs in lane 0 of the folding wave.
template <class F>
__device__ __forceinline__ void fold_waves(const double *part, int nb, int ncol, F f) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int col = wid; col < ncol; col += nw) {
    const double v = wave_sum(lane_fold(part, nb, ncol, col, lane));
    if (lane == 0) f(col, v);
  }
}

// out[col] = scale * sum_b part[b*ncol + col]; one wave per column.
__global__ void __launch_bounds__(256) k_fold(const double *part, int nb, int ncol, double *out, double scale) {
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (col >= ncol) return;
  const double v = wave_sum(lane_fold(part, nb, ncol, col, lane));
  if (lane == 0) out[col] = v * scale;
}

void launch_fold(const double *part, int32_t nb, int32_t ncol, double *out, double scale, hipStream_t st) {
  if (ncol <= 0) return;
  hipLaunchKernelGGL(k_fold, dim3((unsigned)((ncol + 3) / 4)), dim3(256), 0, st, part, nb, ncol, out, scale);
}

// ---------------------------------------------------------------------------
// K1/K2: batched subdomain solves with fused E / E^T products
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int pad8(int x) { return (x + 7) & ~7; }
__host__ __device__ constexpr int pad16(int x) { return (x + 15) & ~15; }

// x lives in LDS column-major: column r of the workgroup's right-hand sides
// at xs[r * XS + row], XS = the largest subdomain size (a persistent item
// with its own column count: its subdomain's size), in a region of
// max_m * R + 1 values.
//
// One level of an ELL-packed sweep (any row width K) for one column, solved
// by one wave.  Rows of width K <= 8: one lane per row, entries subtracted
// in order.  Longer rows: G lanes per row (G = 4, 16, 64 for K <= 32, 128,
// beyond), lane g summing the entries g, g + G, ..., the partial sums added
// by a butterfly inside the group, then x_row = sc x_row - sum.  A group is
// active or idle as a whole, so its butterfly never mixes in an idle lane.
template <typename TS, typename TC, int G>
__device__ __forceinline__ void ell_rows_group(const uint16_t *rows, const TS *sc, const uint16_t *ci, const TS *w,
                                               int L, int K, TC *xc, int lane) {
  const int g = lane % G;
  for (int j = lane / G; j < L; j += 64 / G) {
    TC part = 0;
    // four entries per lane in flight: index and weight loads, then the
    // gathers, then the sums in entry order (entries past the row end are
    // clamped to its last one and not added, so no lane takes another path)
    for (int e0 = g; e0 < K; e0 += 4 * G) {
      int c[4];
      TC wv[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * G, K - 1);
        c[u] = ci[e * L + j];
        wv[u] = cvt<TC>(w[e * L + j]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = xc[c[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * G < K) part += wv[u] * xv[u];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, G);
    if (g == 0) {
      const int row = rows[j];
      xc[row] = cvt<TC>(sc[j]) * xc[row] - part;
    }
  }
}

// A column segment of a near-chain run (marker -2 in the header, then the
// column count and entry count): for each column in order, its row's value
// is final; every later run row that uses it subtracts weight x value.
// Within a column each target row appears once, so the lanes' updates
// never collide, and the wave's program order carries them to the next
// column.
template <typename TS, typename TC>
__device__ __forceinline__ void csc_segment_wave(const uint8_t *seg, TC *xc, int lane) {
  const int32_t *hdr = reinterpret_cast<const int32_t *>(seg);
  const int nc = hdr[1], nnz = hdr[2];
  const uint16_t *crow = reinterpret_cast<const uint16_t *>(seg + kEllHeaderBytes);
  const uint16_t *cptr = reinterpret_cast<const uint16_t *>(seg + kEllHeaderBytes + pad8(2 * nc));
  const uint16_t *tgt = reinterpret_cast<const uint16_t *>(seg + kEllHeaderBytes + pad8(2 * nc) + pad8(2 * (nc + 1)));
  const TS *w = reinterpret_cast<const TS *>(seg + kEllHeaderBytes + pad8(2 * nc) + pad8(2 * (nc + 1)) +
                                             pad8(2 * nnz));
  // the next column's row and entry range are read one column ahead
  int r = crow[0], e0 = cptr[0], e1 = cptr[1];
  for (int c = 0; c < nc; ++c) {
    const int rn = crow[min(c + 1, nc - 1)], en = cptr[min(c + 2, nc)];
    const TC xj = xc[r];
    for (int e = e0 + lane; e < e1; e += 64) {
      const int i = tgt[e];
      xc[i] -= cvt<TC>(w[e]) * xj;
    }
    r = rn;
    e0 = e1;
    e1 = en;
  }
}

template <typename TS, typename TC>
__device__ __forceinline__ void ell_level_wave(const uint8_t *seg, int L, TC *xc, int lane) {
  const int K = *reinterpret_cast<const int32_t *>(seg);
  if (K < 0) {
    csc_segment_wave<TS, TC>(seg, xc, lane);
    return;
  }
  const uint8_t *base = seg + kEllHeaderBytes;
  const uint16_t *rows = reinterpret_cast<const uint16_t *>(base);
  const int o_sc = pad8(2 * L);
  const TS *sc = reinterpret_cast<const TS *>(base + o_sc);
  const int o_ci = o_sc + pad8((int)sizeof(TS) * L);
  const uint16_t *ci = reinterpret_cast<const uint16_t *>(base + o_ci);
  const TS *w = reinterpret_cast<const TS *>(base + o_ci + pad8(2 * K * L));
  // lanes per row: enough that each lane holds few entries, no more than
  // the level's rows leave room for
  const int gk = K <= 4 ? 1 : (K <= 16 ? 4 : (K <= 64 ? 16 : 64));
  const int gl = L >= 64 ? 1 : (L >= 16 ? 4 : (L >= 4 ? 16 : 64));
  const int G = min(gk, gl);
  if (G == 1) {
    for (int j = lane; j < L; j += 64) {
      const int row = rows[j];
      TC acc = cvt<TC>(sc[j]) * xc[row];
      for (int e = 0; e < K; ++e) acc -= cvt<TC>(w[e * L + j]) * xc[(int)ci[e * L + j]];
      xc[row] = acc;
    }
  } else if (G == 4) {
    ell_rows_group<TS, TC, 4>(rows, sc, ci, w, L, K, xc, lane);
  } else if (G == 16) {
    ell_rows_group<TS, TC, 16>(rows, sc, ci, w, L, K, xc, lane);
  } else {
    ell_rows_group<TS, TC, 64>(rows, sc, ci, w, L, K, xc, lane);
  }
}

// Levels [l0, l1) of an ELL-packed sweep staged at sbase, for one column, by
// one wave with no barrier between levels: a wave's LDS accesses take
// effect in program order, and a level reads only rows of earlier levels.
template <typename TS, typename TC>
__device__ __forceinline__ void solve_staged_ell(const uint8_t *sbase, const int32_t *lev, const int32_t *lvb, int l0,
                                                 int l1, TC *xc, int lane) {
  for (int l = l0; l < l1; ++l) ell_level_wave<TS, TC>(sbase + (lvb[l] - lvb[l0]), lev[l + 1] - lev[l], xc, lane);
}

// Copy nv 16-byte vectors from src into the LDS at dst with direct
// global-to-LDS loads: each wave moves 64 consecutive vectors per
// instruction (lane l's vector to the wave's base + 16 l), no registers
// involved, so every load of the copy is in flight at once; lanes past the
// end are inactive.  gt - lane and gn are multiples of 64.  The loads are
// complete when this returns.
__device__ __forceinline__ void stage_dma(const uint4 *src, int nv, uint4 *dst, int gt, int gn) {
  const int lane = threadIdx.x & 63;
  for (int i0 = gt - lane; i0 < nv; i0 += gn) {
    const int i = i0 + lane;
    if (i < nv)
      __builtin_amdgcn_global_load_lds(static_cast<const void *>(src + i),
                                       (__attribute__((address_space(3))) void *)(dst + i0), 16, 0, 0);
  }
  __builtin_amdgcn_s_waitcnt(0);
}

// Fixed-width row records (see BlockDesc): KR int32 indices [row, columns,
// pad] and KR scale/weights [sc, w, pad] per row, read as 16-byte vectors.
template <int KR>
struct RowIdx {
  int v[KR];
};

template <int KR>
__device__ __forceinline__ void load_ridx(const int32_t *ix, int j, RowIdx<KR> &r) {
  const int4 *p = reinterpret_cast<const int4 *>(ix + j * KR);
#pragma unroll
  for (int q = 0; q < KR / 4; ++q) {
    const int4 t = p[q];
    r.v[4 * q] = t.x;
    r.v[4 * q + 1] = t.y;
    r.v[4 * q + 2] = t.z;
    r.v[4 * q + 3] = t.w;
  }
}

template <typename TS, int KR>
__device__ __forceinline__ void load_rwts(const TS *wr, int j, TS (&w)[KR]) {
  constexpr int per = 16 / (int)sizeof(TS);
  const uint4 *p = reinterpret_cast<const uint4 *>(wr + j * KR);
#pragma unroll
  for (int q = 0; q < KR / per; ++q) {
    const uint4 t = p[q];
    __builtin_memcpy(&w[q * per], &t, 16);
  }
}

// Levels [s, e) of a staged chunk, one column xc, one wave; lane i of mL /
// mOff holds the row count and stage offset of the chunk's level i, and
// every level in the range has at most 64 * NP rows.  Lane rows
// j = lane + 64u (u < NP) clamp to the level's last row: such a lane
// recomputes that row from the same inputs and stores the same value, so
// every pass is straight-line code.  Per level: the x gathers of all NP
// passes together with their scale/weight records, then the next level's
// index records (they do not depend on x), then the NP stores.  A wave's
// LDS accesses take effect in program order and a level depends only on
// earlier levels, so no barrier is needed.  Per row: x_row = sc x_row minus
// the weighted columns in entry order.
template <typename TS, typename TC, int KE, int NP>
__device__ __forceinline__ void solve_chunk(const uint8_t *stage, int mL, int mOff, int s, int e, TC *xc,
                                            int lane) {
  constexpr int KR = rec_width(KE);
  s = __builtin_amdgcn_readfirstlane(s);
  e = __builtin_amdgcn_readfirstlane(e);
  RowIdx<KR> cur[NP];
  {
    const int L0 = __builtin_amdgcn_readlane(mL, s);
    const int32_t *ix = reinterpret_cast<const int32_t *>(stage + __builtin_amdgcn_readlane(mOff, s));
#pragma unroll
    for (int u = 0; u < NP; ++u) load_ridx<KR>(ix, min(lane + 64 * u, L0 - 1), cur[u]);
  }
  for (int i = s; i < e; ++i) {
    const int L = __builtin_amdgcn_readlane(mL, i);
    const TS *wr = reinterpret_cast<const TS *>(stage + __builtin_amdgcn_readlane(mOff, i) + 4 * KR * L);
    TC xd[NP], xv[NP][KE];
    TS wv[NP][KR];
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      xd[u] = xc[cur[u].v[0]];
#pragma unroll
      for (int k = 0; k < KE; ++k) xv[u][k] = xc[cur[u].v[1 + k]];
      load_rwts<TS, KR>(wr, min(lane + 64 * u, L - 1), wv[u]);
    }
    const int in = i + 1 < e ? i + 1 : i;
    const int Ln = __builtin_amdgcn_readlane(mL, in);
    const int32_t *ixn = reinterpret_cast<const int32_t *>(stage + __builtin_amdgcn_readlane(mOff, in));
    RowIdx<KR> nxt[NP];
#pragma unroll
    for (int u = 0; u < NP; ++u) load_ridx<KR>(ixn, min(lane + 64 * u, Ln - 1), nxt[u]);
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      TC acc = cvt<TC>(wv[u][0]) * xd[u];
#pragma unroll
      for (int k = 0; k < KE; ++k) acc -= cvt<TC>(wv[u][1 + k]) * xv[u][k];
      xc[cur[u].v[0]] = acc;
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) cur[u] = nxt[u];
  }
}

// Levels [l0, l1) of one fixed-width sweep staged at sbase (level l's
// segment at sbase + lvb[l] - lvb[l0], at most 64 levels), column xc, one
// wave.  Lane i holds the row count and stage offset of level l0 + i; the
// levels run in maximal stretches that need the same number of row passes
// per lane (levels are at most 64 * rec_passes(KE) rows wide).
template <typename TS, typename TC, int KE>
__device__ __forceinline__ void solve_staged(const uint8_t *sbase, const int32_t *lev, const int32_t *lvb, int l0,
                                             int l1, TC *xc, int lane) {
  constexpr int NPMAX = rec_passes(KE);
  const int nl = l1 - l0;
  const int li = min(l0 + lane, l1 - 1);
  const int mL = lev[li + 1] - lev[li];
  const int mOff = lvb[li] - lvb[l0];
  const int npl = (mL + 63) >> 6;
  int s = 0;
  while (s < nl) {
    const int np = __builtin_amdgcn_readlane(npl, s);
    const unsigned long long other = __ballot(lane > s && lane < nl && npl != np);
    const int e = other ? __ffsll(other) - 1 : nl;
    if (np <= 1)
      solve_chunk<TS, TC, KE, 1>(sbase, mL, mOff, s, e, xc, lane);
    else if (np == 2)
      solve_chunk<TS, TC, KE, 2>(sbase, mL, mOff, s, e, xc, lane);
    else if constexpr (NPMAX >= 3) {
      if (np == 3)
        solve_chunk<TS, TC, KE, 3>(sbase, mL, mOff, s, e, xc, lane);
      else if constexpr (NPMAX >= 4)
        solve_chunk<TS, TC, KE, 4>(sbase, mL, mOff, s, e, xc, lane);
    }
    s = e;
  }
}

// The first chunk of a fixed-width sweep (the chunk sweeps_pipelined
// starts with: levels [0, l1) fitting `half` bytes, at most 64 levels),
// read straight from the global level offsets glvb, copied by the threads
// gt = 0 .. gn-1 of a group of whole waves.
__device__ __forceinline__ void stage_first(const uint8_t *data, const int32_t *glvb, int nlev, int half,
                                            uint8_t *stage, int gt, int gn) {
  const int lane = threadIdx.x & 63;
  const int cand = 1 + lane;
  const int b0 = glvb[0];
  const int v = glvb[min(cand, nlev)];
  const bool ok = cand <= nlev && (lane == 0 || v - b0 <= half);
  const int l1 = (int)__popcll(__ballot(ok));
  const int b1 = __builtin_amdgcn_readlane(v, l1 - 1);
  stage_dma(reinterpret_cast<const uint4 *>(data + b0), (b1 - b0) >> 4, reinterpret_cast<uint4 *>(stage), gt, gn);
}

// Both sweeps of one subdomain (fixed-width records for KE > 0, the ELL form
// for KE == 0), one wave per right-hand side column (wave w < Rg solves
// column w; its backward sweep follows its own forward sweep, so the
// columns need no barrier between them).  The two
// packed streams are cut into chunks of consecutive levels of one sweep
// (at most 64 levels, fitting half the stage) and double-buffered: while the
// solver waves run chunk c from one half, the other waves copy chunk c + 1
// into the other half; a barrier separates the rounds.  When every wave
// solves (Rg == waves) the copy runs after the solve instead.  staged0: the
// first chunk is already in the first half (stage_first, before a barrier).
template <typename TS, typename TC, int KE>
__device__ __forceinline__ void sweeps_pipelined(const uint8_t *fdata, const int32_t *levf, const int32_t *lvbf,
                                                 int fn, const uint8_t *bdata, const int32_t *levb,
                                                 const int32_t *lvbb, int bn, TC *xs, int XS, int Rg,
                                                 uint8_t *stage, int stage_bytes, bool staged0) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int half = (stage_bytes >> 1) & ~15;
  const bool stagers = Rg < nw;
  // end of the chunk starting at level l0: the largest l1 <= l0 + 64 with
  // levels [l0, l1) fitting half the stage (at least one level); lane i
  // tests l1 = l0 + 1 + i (the test is monotone in l1)
  auto chunk_end = [&](int sw, int l0) {
    const int32_t *lvb = sw ? lvbb : lvbf;
    const int nlev = sw ? bn : fn;
    const int cand = l0 + 1 + lane;
    const bool ok = cand <= nlev && (lane == 0 || lvb[min(cand, nlev)] - lvb[l0] <= half);
    return l0 + (int)__popcll(__ballot(ok));
  };
  auto copy_chunk = [&](int sw, int l0, int l1, uint8_t *dst, int gt, int gn) {
    const int32_t *lvb = sw ? lvbb : lvbf;
    const uint8_t *data = sw ? bdata : fdata;
    stage_dma(reinterpret_cast<const uint4 *>(data + lvb[l0]), (lvb[l1] - lvb[l0]) >> 4,
              reinterpret_cast<uint4 *>(dst), gt, gn);
  };
  int sw = fn > 0 ? 0 : 1;
  if (sw == 1 && bn == 0) return;
  int l0 = 0, l1 = chunk_end(sw, 0), b = 0;
  if (!staged0) {
    copy_chunk(sw, l0, l1, stage, threadIdx.x, blockDim.x);
    __syncthreads();
  }
  while (true) {
    int ns = sw, nl0 = l1;
    if (nl0 >= (sw ? bn : fn)) {
      ns = sw + 1;
      nl0 = 0;
      if (ns == 1 && bn == 0) ns = 2;
    }
    const bool more = ns < 2;
    const int nl1 = more ? chunk_end(ns, nl0) : 0;
    uint8_t *cur = stage + b * half, *nxt = stage + (b ^ 1) * half;
    if (wv < Rg) {
      for (int r = wv; r < Rg; r += nw) {
        if constexpr (KE > 0)
          solve_staged<TS, TC, KE>(cur, sw ? levb : levf, sw ? lvbb : lvbf, l0, l1, xs + r * XS, lane);
        else
          solve_staged_ell<TS, TC>(cur, sw ? levb : levf, sw ? lvbb : lvbf, l0, l1, xs + r * XS, lane);
      }
    } else if (more) {
      copy_chunk(ns, nl0, nl1, nxt, threadIdx.x - Rg * 64, blockDim.x - Rg * 64);
    }
    __syncthreads();
    if (!more) break;
    if (!stagers) {
      copy_chunk(ns, nl0, nl1, nxt, threadIdx.x, blockDim.x);
      __syncthreads();
    }
    sw = ns;
    l0 = nl0;
    l1 = nl1;
    b ^= 1;
  }
}

// One work item: subdomain sub and right-hand sides [cg * R, +Rg):
// prologue (f, E y) into LDS, forward and backward
// sweeps in LDS (or only one of them, by a.sweeps), then u and the E^T
// epilogue.  KE > 0: every packed row has exactly KE entries (padding has
// w = 0); KE == 0: the ELL form of any width.  Either way the sweeps run
// one wave per column with double-buffered staging.
template <typename TS, typename TC, int KE, bool XP>
__device__ __forceinline__ void bsolve_item(const BlockArrays<TS> &B, const BArgs &a, int sub, int c0, int Rg,
                                            int XS) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BlockDesc d = B.desc[sub];
  const int R = a.R;
  const int m = d.m;
  // LDS: [stage][dummy slots][x: max_m*R + 1 TC][levptr f, b][lvb f, b]; the
  // item's Rg columns of XS rows each fit the x region (XS*Rg <= max_m*R)
  uint8_t *stage = smem;
  TC *xs = reinterpret_cast<TC *>(smem + a.stage_bytes + kStageDummyBytes);
  int32_t *levf =
      reinterpret_cast<int32_t *>(smem + a.stage_bytes + kStageDummyBytes + pad16((int)sizeof(TC) * (B.max_m * R + 1)));
  int32_t *levb = levf + B.max_lev + 1;
  int32_t *lvbf = levb + B.max_lev + 1;
  int32_t *lvbb = lvbf + B.max_lev + 1;
  const int tid = threadIdx.x, nt = blockDim.x;
  TC *xdummy = reinterpret_cast<TC *>(stage + a.stage_bytes) + (tid & 63);
  // LDS position of each local row (XP false: the row itself)
  const uint16_t *xp = XP ? B.xpos + d.m0 : nullptr;
  // level pointers into LDS, then rhs = a_f f_i (loads batched 4 per
  // thread), by the threads gt = 0 .. gn-1
  auto prologue = [&](int gt, int gn) {
    for (int i = gt; i <= d.f_nlev; i += gn) {
      levf[i] = B.lev[d.f_lev + i];
      lvbf[i] = B.lvb[d.f_lvb + i];
    }
    for (int i = gt; i <= d.b_nlev; i += gn) {
      levb[i] = B.lev[d.b_lev + i];
      lvbb[i] = B.lvb[d.b_lvb + i];
    }
    const int mt = m * Rg;
    if constexpr (!XP && sizeof(TC) == 8) {
      if (a.a_f == 1.0) {
        // the f columns go straight into x by direct global-to-LDS loads
        // (4-byte words: a column need not start on 16 bytes), all in
        // flight at once; gt - lane and gn are multiples of 64
        const int lane = gt & 63, nd = 2 * m;
        for (int r = 0; r < Rg; ++r) {
          const uint32_t *src = reinterpret_cast<const uint32_t *>(a.f + d.m0 + (int64_t)(c0 + r) * a.ldf);
          uint32_t *dst = reinterpret_cast<uint32_t *>(xs + r * XS);
          for (int i0 = gt - lane; i0 < nd; i0 += gn) {
            const int i = i0 + lane;
            if (i < nd)
              __builtin_amdgcn_global_load_lds(static_cast<const void *>(src + i),
                                               (__attribute__((address_space(3))) void *)(dst + i0), 4, 0, 0);
          }
        }
        __builtin_amdgcn_s_waitcnt(0);
        return;
      }
    }
    if constexpr (XP) {
      // rows at their LDS positions
      for (int t0 = gt; t0 < mt; t0 += 4 * gn) {
        double v[4];
        int ps[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = min(t0 + u * gn, mt - 1);
          const int r = t / m, row = t - r * m;
          ps[u] = r * XS + (int)xp[row];
        }
        if (a.a_f != 0.0) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int t = min(t0 + u * gn, mt - 1);
            const int r = t / m, row = t - r * m;
            v[u] = a.a_f * a.f[(int64_t)(d.m0 + row) + (int64_t)(c0 + r) * a.ldf];
          }
        } else {
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          *(t0 + u * gn < mt ? xs + ps[u] : xdummy) = (TC)v[u];   // past the end: the lane's dummy slot
      }
      return;
    }
    for (int t0 = gt; t0 < mt; t0 += 4 * gn) {
      double v[4];
      if (a.a_f != 0.0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int t = min(t0 + u * gn, mt - 1);
          const int r = t / m, row = t - r * m;
          v[u] = a.a_f * a.f[(int64_t)(d.m0 + row) + (int64_t)(c0 + r) * a.ldf];
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u * gn;
        const int tt = min(t, mt - 1);
        const int r = tt / m, row = tt - r * m;
        *(t < mt ? xs + r * XS + row : xdummy) = (TC)v[u];   // past the end: the lane's dummy slot
      }
    }
  };
  // XP: LDS positions of the first rows this thread stores at the end
  // (rows tid + i * nt, two per register), fetched now so that the u store
  // waits on no global load
  constexpr int kPosPre = 8;
  uint32_t pre[kPosPre / 2];
  if constexpr (XP) {
    if (a.u && m > 0) {
#pragma unroll
      for (int i = 0; i < kPosPre / 2; ++i) {
        const int r0 = min(tid + 2 * i * nt, m - 1), r1 = min(tid + (2 * i + 1) * nt, m - 1);
        pre[i] = (uint32_t)xp[r0] | ((uint32_t)xp[r1] << 16);
      }
    }
  }
  // the sweeps this launch runs (a.sweeps: bit 0 forward, bit 1 backward)
  const int fn = (a.sweeps & 1) ? d.f_nlev : 0, bn = (a.sweeps & 2) ? d.b_nlev : 0;
  {
    // the upper half of the waves stages the first sweep chunk meanwhile
    if (tid >= nt / 2) {
      const int sw0 = fn > 0 ? 0 : 1;
      if (sw0 == 0 || bn > 0)
        stage_first(B.data + (sw0 ? d.b_data : d.f_data), B.lvb + (sw0 ? d.b_lvb : d.f_lvb),
                    sw0 ? bn : fn, (a.stage_bytes >> 1) & ~15, stage, tid - nt / 2, nt - nt / 2);
    } else {
      prologue(tid, nt / 2);
    }
  }
  __syncthreads();
  if (a.b_y != 0.0 && d.e_n > 0) {
    const int en = d.e_n;
    for (int t = tid; t < en * Rg; t += nt) {
      const int i = t / Rg, r = t - i * Rg;
      const int row = B.e_row[d.e_row + i];
      const double *yc = a.y + (int64_t)(c0 + r) * a.ldy;
      TC acc = 0;
      for (int e = 0; e < d.e_K; ++e) {
        const int64_t x = d.e_ent + (int64_t)e * en + i;
        acc += cvt<TC>(B.e_val[x]) * (TC)yc[B.e_q[x]];
      }
      xs[r * XS + row] += (TC)a.b_y * acc;
    }
    __syncthreads();
  }
  sweeps_pipelined<TS, TC, KE>(B.data + d.f_data, levf, lvbf, fn, B.data + d.b_data, levb, lvbb, bn, xs, XS, Rg,
                               stage, a.stage_bytes, true);
  if constexpr (XP) {
    if (a.u) {
      // each row's LDS position taken once for its Rg columns
      double *uc = a.u + d.m0 + (int64_t)c0 * a.ldu;
#pragma unroll
      for (int i = 0; i < kPosPre; ++i) {
        const int row = tid + i * nt;
        const int ps = (int)((pre[i / 2] >> (16 * (i & 1))) & 0xFFFFu);
        if (row < m)
          for (int r = 0; r < Rg; ++r) uc[row + (int64_t)r * a.ldu] = (double)xs[r * XS + ps];
      }
      for (int row = tid + kPosPre * nt; row < m; row += nt) {
        const int ps = (int)xp[row];
        for (int r = 0; r < Rg; ++r) uc[row + (int64_t)r * a.ldu] = (double)xs[r * XS + ps];
      }
    }
  } else if (a.u) {
    for (int t = tid; t < m * Rg; t += nt) {
      const int r = t / m, row = t - r * m;
      a.u[(int64_t)(d.m0 + row) + (int64_t)(c0 + r) * a.ldu] = (double)xs[r * XS + row];
    }
  }
  if (a.gout) {
    const int tn = d.t_n;
    for (int t = tid; t < tn * Rg; t += nt) {
      const int i = t / Rg, r = t - i * Rg;
      const int q = B.t_q[d.t_row + i];
      TC acc = 0;
      for (int e = 0; e < d.t_K; ++e) {
        const int64_t x = d.t_ent + (int64_t)e * tn + i;
        acc += cvt<TC>(B.t_val[x]) * xs[r * XS + (int)B.t_j[x]];
      }
      const double gv = a.c_g != 0.0 ? a.c_g * a.g[q + (int64_t)(c0 + r) * a.ldg] : 0.0;
      a.gout[q + (int64_t)(c0 + r) * a.ldgo] = gv + a.d_t * (double)acc;
    }
  }
}

// One launch of the batched B solves: one workgroup per (subdomain, column
// group), or a persistent grid walking its scheduled items (the shared
// memory is reused after a barrier between items).
template <typename TS, typename TC, int KE, bool XP>
__global__ void __launch_bounds__(1024) k_bsolve(BlockArrays<TS> B, BArgs a) {
  if (a.sched) {
    for (int it = a.sched_ptr[blockIdx.x]; it < a.sched_ptr[blockIdx.x + 1]; ++it) {
      const uint32_t item = (uint32_t)a.sched[it];
      const int sub = (int)(item & 0xFFFFu);
      if (a.var_cols) {
        // columns [c0, c0 + Rg) of the subdomain, with its own row stride
        const int c0 = (int)((item >> 16) & 0xFFu), Rg = (int)(item >> 24);
        bsolve_item<TS, TC, KE, XP>(B, a, sub, c0, Rg, B.desc[sub].m);
      } else {
        const int c0 = (int)(item >> 16) * a.R;
        bsolve_item<TS, TC, KE, XP>(B, a, sub, c0, min(a.R, a.nrhs - c0), B.max_m);
      }
      __syncthreads();
    }
  } else {
    const int c0 = blockIdx.y * a.R;
    bsolve_item<TS, TC, KE, XP>(B, a, blockIdx.x, c0, min(a.R, a.nrhs - c0), B.max_m);
  }
}

template <typename TS, typename TC, int KE, bool XP>
void launch_bsolve_k(const BlockArrays<TS> &B, int32_t p, const BArgs &a, int32_t threads, size_t lds_bytes,
                     hipStream_t st) {
  static size_t attr_bytes = 0;
  if (lds_bytes > 65536 && lds_bytes > attr_bytes) {
    (void)hipFuncSetAttribute((const void *)k_bsolve<TS, TC, KE, XP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bytes);
    attr_bytes = lds_bytes;
  }
  // persistent: p is the number of workgroups of the schedule
  dim3 grid(p, a.sched ? 1 : (a.nrhs + a.R - 1) / a.R);
  hipLaunchKernelGGL((k_bsolve<TS, TC, KE, XP>), grid, dim3(threads), lds_bytes, st, B, a);
}
// the variant with LDS positions (B.xpos) exists for the fixed-width forms
// only: the host keeps the row order for the ELL form
template <typename TS, typename TC, int KE>
void launch_bsolve_x(const BlockArrays<TS> &B, int32_t p, const BArgs &a, int32_t threads, size_t lds_bytes,
                     hipStream_t st) {
  if (B.xpos)
    launch_bsolve_k<TS, TC, KE, true>(B, p, a, threads, lds_bytes, st);
  else
    launch_bsolve_k<TS, TC, KE, false>(B, p, a, threads, lds_bytes, st);
}

// B.pack_K > 0: every packed row has exactly pack_K entries
template <typename TS, typename TC>
void launch_bsolve(const BlockArrays<TS> &B, int32_t p, const BArgs &a, int32_t threads,
                   size_t lds_bytes, hipStream_t st) {
  switch (B.pack_K) {
    case 1: launch_bsolve_x<TS, TC, 1>(B, p, a, threads, lds_bytes, st); break;
    case 2: launch_bsolve_x<TS, TC, 2>(B, p, a, threads, lds_bytes, st); break;
    case 3: launch_bsolve_x<TS, TC, 3>(B, p, a, threads, lds_bytes, st); break;
    case 4: launch_bsolve_x<TS, TC, 4>(B, p, a, threads, lds_bytes, st); break;
    default: launch_bsolve_k<TS, TC, 0, false>(B, p, a, threads, lds_bytes, st); break;
  }
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

// One level of a sweep with long rows: G lanes per row, lane g summing the
// entries g, g + G, ... (loads of a lane issued four at a time), the G
// partial sums added by a butterfly, then x_row = sc x_row - sum.
template <typename TS, typename TC, int G>
__global__ void __launch_bounds__(256) k_sweep_lvl_g(SweepArrays<TS> S, int a, int b, double *x, int64_t ldx) {
  const int g = threadIdx.x % G;
  const int t = a + (blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (t >= b) return;   // whole groups leave together
  double *xc = x + (int64_t)blockIdx.y * ldx;
  const int e0 = S.rp[t], e1 = S.rp[t + 1];
  TC part = 0;
  for (int e = e0 + g; e < e1; e += 4 * G) {
    TC wv[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ee = e + u * G;
      const bool ok = ee < e1;
      const int ec = ok ? ee : e0;
      wv[u] = ok ? cvt<TC>(S.w[ec]) : (TC)0;
      xv[u] = (TC)xc[S.ci[ec]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) part += wv[u] * xv[u];
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, G);
  if (g == 0) {
    const int row = S.rows[t];
    xc[row] = (double)(cvt<TC>(S.sc[t]) * (TC)xc[row] - part);
  }
}

// Whole sweep of a schedule with at most two levels, out of place
// (y = T^{-1} x): level-0 rows have no entries (y = sc x); level-1 rows
// depend on level-0 rows only, whose values sc_j x_j are folded into the
// stored weights w2 = w * sc_j, so every row reads x alone.  dv (optional,
// one column): per-block sums of dv[row] y[row] over the block's rows go to
// dpart[blockIdx.x] (a dot product with y, folded by the consumer).
template <typename TS, typename TC>
__global__ void __launch_bounds__(256) k_sweep2(SweepArrays<TS> S, int nrows, const double *x, int64_t ldx, double *y,
                                                int64_t ldy, const double *dv, double *dpart) {
  __shared__ double sh[4];
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const double *xc = x + (int64_t)blockIdx.y * ldx;
  double *yc = y + (int64_t)blockIdx.y * ldy;
  double d = 0.0;
  if (t < nrows) {
    const int row = S.rows[t];
    const int e0 = S.rp[t], e1 = S.rp[t + 1];
    TC acc = cvt<TC>(S.sc[t]) * (TC)xc[row];
    // four entries at a time: indices and weights, then the gathers, then
    // the subtractions in entry order (clamped loads past the row end are
    // not used)
    for (int e = e0; e < e1; e += 4) {
      int c[4];
      TC wv[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ee = min(e + u, e1 - 1);
        c[u] = S.ci[ee];
        wv[u] = cvt<TC>(S.w2[ee]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = (TC)xc[c[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e + u < e1) acc -= wv[u] * xv[u];
    }
    yc[row] = (double)acc;
    if (dv) d = (double)acc * dv[row];
  }
  if (dv) {
    const double b = block_sum(d, sh);
    if (threadIdx.x == 0) dpart[blockIdx.x] = b;
  }
}

template <typename TS, typename TC>
void launch_sweep2(const SweepArrays<TS> &S, int32_t nrows, const double *x, int64_t ldx, double *y, int64_t ldy,
                   int32_t nrhs, hipStream_t st, const double *dv, double *dpart) {
  if (nrows == 0 || nrhs == 0) return;
  hipLaunchKernelGGL((k_sweep2<TS, TC>), dim3((nrows + 255) / 256, nrhs), dim3(256), 0, st, S, nrows, x, ldx, y,
                     ldy, nrhs == 1 ? dv : nullptr, dpart);
}

template <typename TS, typename TC>
void launch_sweep(const SweepArrays<TS> &S, const int32_t *lev_host, int32_t nlev, int32_t nrows,
                  double *x, int64_t ldx, int32_t nrhs, bool one_wg, hipStream_t st, int32_t G) {
  if (nlev == 0 || nrhs == 0) return;
  if (G > 1) {
    // long rows: one launch per level, G lanes per row
    for (int l = 0; l < nlev; ++l) {
      const int a = lev_host[l], b = lev_host[l + 1];
      if (b <= a) continue;
      dim3 grid((unsigned)(((int64_t)(b - a) * G + 255) / 256), nrhs);
      if (G == 4)
        hipLaunchKernelGGL((k_sweep_lvl_g<TS, TC, 4>), grid, dim3(256), 0, st, S, a, b, x, ldx);
      else if (G == 8)
        hipLaunchKernelGGL((k_sweep_lvl_g<TS, TC, 8>), grid, dim3(256), 0, st, S, a, b, x, ldx);
      else
        hipLaunchKernelGGL((k_sweep_lvl_g<TS, TC, 16>), grid, dim3(256), 0, st, S, a, b, x, ldx);
    }
    return;
  }
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
// K4: rank-k block of eq. skt.  U column-major (s x k, leading dim s).
//   part[b][r][q] = sum_{i in chunk b} U[i,q] w[i,r]   (thread per row,
//   Q_T columns of U per pass held in registers, block-reduced in LDS);
//   the last block sums the partials in block order and scales by dsc
//   (-> cbuf[r*k+q]); then wout = rho w + U cbuf (thread per row).
// ---------------------------------------------------------------------------
constexpr int LR_THREADS = 256;
constexpr int LR_Q = 32;     // columns of U per register pass

template <typename TU>
__global__ void __launch_bounds__(LR_THREADS) k_lr_partial(const TU *U, int64_t s, int k, const double *w,
                                                          int64_t ldw, int nrhs, double *part) {
  __shared__ double red[LR_THREADS / 64][LR_Q];
  const int nb = gridDim.x;
  const int64_t chunk = (s + nb - 1) / nb;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(s, i0 + chunk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int r = 0; r < nrhs; ++r) {
    const double *wc = w + (int64_t)r * ldw;
    for (int q0 = 0; q0 < k; q0 += LR_Q) {
      double acc[LR_Q];
#pragma unroll
      for (int q = 0; q < LR_Q; ++q) acc[q] = 0.0;
      for (int64_t i = i0 + threadIdx.x; i < i1; i += LR_THREADS) {
        const double wi = wc[i];
        // columns past k are clamped to column k-1 (valid loads, unpredicated
        // so they issue as one batch); their sums are never stored
#pragma unroll
        for (int q = 0; q < LR_Q; ++q) acc[q] += cvt<double>(U[i + (int64_t)min(q0 + q, k - 1) * s]) * wi;
      }
#pragma unroll
      for (int q = 0; q < LR_Q; ++q) acc[q] = wave_sum(acc[q]);
      if (lane == 0)
#pragma unroll
        for (int q = 0; q < LR_Q; ++q) red[wid][q] = acc[q];
      __syncthreads();
      if (threadIdx.x < LR_Q && q0 + threadIdx.x < k) {
        double v = 0.0;
        for (int ww = 0; ww < LR_THREADS / 64; ++ww) v += red[ww][threadIdx.x];
        part[((int64_t)blockIdx.x * nrhs + r) * k + q0 + threadIdx.x] = v;
      }
      __syncthreads();
    }
  }
}

// cbuf[t] = dsc[t % k] * sum_b part[b*(k*nrhs) + t]
__global__ void __launch_bounds__(256) k_lr_fold(const double *part, int nb, int kn, int k, const double *dsc,
                                                 double *cbuf) {
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= kn) return;
  const double v = wave_sum(lane_fold(part, nb, kn, t, lane));
  if (lane == 0) cbuf[t] = v * dsc[t % k];
}

// one right-hand side: U entries in flight per lane in the update (LRU_QB1)
// and groups in flight per lane in the partial sums (LRR_GU1)
constexpr int LRU_QB1 = 16;
constexpr int LRR_GU1 = 16;
// RT columns per pass: each group of QB entries of a U row is loaded once
// for RT columns; every column sums its entries in the same order whatever
// RT and QB.  One column: w is loaded before the U entries.
template <typename TU, int RT, int QB>
__global__ void __launch_bounds__(256) k_lr_update(const TU *U, int64_t s, int k, const double *w,
                                                  int64_t ldw, double *wout, int64_t ldo, int nrhs,
                                                  const double *cbuf, double rho) {
  extern __shared__ double cs[];
  for (int t = threadIdx.x; t < k * nrhs; t += blockDim.x) cs[t] = cbuf[t];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s) return;
  double w1 = 0.0;
  if constexpr (RT == 1) w1 = w[i];
  for (int r0 = 0; r0 < nrhs; r0 += RT) {
    const int nr = min(RT, nrhs - r0);
    double acc[RT];
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[r] = 0.0;
    int q = 0;
    for (; q + QB <= k; q += QB) {
      double u[QB];
#pragma unroll
      for (int e = 0; e < QB; ++e) u[e] = cvt<double>(U[i + (int64_t)(q + e) * s]);
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const int rr = min(r, nr - 1);
#pragma unroll
        for (int e = 0; e < QB; ++e) acc[r] += u[e] * cs[(r0 + rr) * k + q + e];
      }
    }
    for (; q < k; ++q) {
      const double uq = cvt<double>(U[i + (int64_t)q * s]);
#pragma unroll
      for (int r = 0; r < RT; ++r) acc[r] += uq * cs[(r0 + min(r, nr - 1)) * k + q];
    }
    if constexpr (RT == 1) {
      wout[i] = fma(rho, w1, acc[0]);   // the fused form of the general case
    } else {
#pragma unroll
      for (int r = 0; r < RT; ++r)
        if (r < nr) wout[i + (int64_t)(r0 + r) * ldo] = rho * w[i + (int64_t)(r0 + r) * ldw] + acc[r];
    }
  }
}

template <typename TU>
void launch_lr_update(const TU *U, int64_t s, int32_t k, const double *w, int64_t ldw, double *wout, int64_t ldo,
                      int32_t nrhs, const double *cbuf, double rho, hipStream_t st) {
  const dim3 grid((unsigned)((s + 255) / 256));
  const size_t lds = sizeof(double) * k * nrhs;
  if (nrhs == 1)
    hipLaunchKernelGGL((k_lr_update<TU, 1, LRU_QB1>), grid, dim3(256), lds, st, U, s, k, w, ldw, wout, ldo, nrhs,
                       cbuf, rho);
  else if (nrhs <= 8)
    hipLaunchKernelGGL((k_lr_update<TU, 8, 8>), grid, dim3(256), lds, st, U, s, k, w, ldw, wout, ldo, nrhs, cbuf,
                       rho);
  else
    hipLaunchKernelGGL((k_lr_update<TU, 16, 8>), grid, dim3(256), lds, st, U, s, k, w, ldw, wout, ldo, nrhs, cbuf,
                       rho);
}

// ---------------------------------------------------------------------------
// K4 with U_k row-major (FP64 / FP32 storage).  U holds s rows of ldk
// entries (ldk: a power of two >= max(k, VEC); columns >= k and rows >= s
// are zero; the array is padded to whole groups).  A group is what one
// wave reads with one 16-byte load per lane: G = 64 VEC entries, lane l
// holding entries VEC l .. VEC l + VEC - 1, i.e. columns (VEC l) % ldk + v
// of row g RG + (VEC l) / ldk, RG = G / ldk.  Lanes with equal
// l % (ldk / VEC) own the same columns, so a column's sum needs a shuffle
// over only 64 VEC / ldk lanes.  The update U c reads the column-major U
// (one row per thread, which measured faster than the row-major form).
// ---------------------------------------------------------------------------
// Register tiles (template arguments of k_lr_partial_rm): LRR_RT right-hand
// sides per pass over U, LRR_GU groups in flight per lane: 1 x LRR_GU1 for
// one column, 4 x 4 up to four columns, 8 x 2 up to eight, 16 x 1 above
// (each column's sum is the same whatever the tile).

template <typename TU>
struct LrVec;
template <>
struct LrVec<double> {
  static constexpr int V = 2;
  typedef double2 T;
};
template <>
struct LrVec<float> {
  static constexpr int V = 4;
  typedef float4 T;
};

template <typename TU>
__device__ __forceinline__ void lr_unpack(const typename LrVec<TU>::T &x, double *u);
template <>
__device__ __forceinline__ void lr_unpack<double>(const double2 &x, double *u) {
  u[0] = x.x;
  u[1] = x.y;
}
template <>
__device__ __forceinline__ void lr_unpack<float>(const float4 &x, double *u) {
  u[0] = x.x;
  u[1] = x.y;
  u[2] = x.z;
  u[3] = x.w;
}

// partial sums U^T w over the groups of block b -> part[(b nrhs + r) k + q]
template <typename TU, int LRR_RT, int LRR_GU>
__global__ void __launch_bounds__(256) k_lr_partial_rm(const TU *U, int ldk, int64_t ng, int64_t s, int k,
                                                       const double *w, int64_t ldw, int nrhs, double *part) {
  constexpr int VEC = LrVec<TU>::V;
  typedef typename LrVec<TU>::T VT;
  __shared__ double red[4][64 * LRR_RT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t per = (ng + gridDim.x - 1) / gridDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * per, g1 = min(ng, g0 + per);
  const int RG = 64 * VEC / ldk;
  const int rof = VEC * lane / ldk;          // row of this lane inside a group
  const int cw = ldk / VEC;                  // lanes per row
  const VT *Uv = reinterpret_cast<const VT *>(U);
  for (int r0 = 0; r0 < nrhs; r0 += LRR_RT) {
    const int nr = min(LRR_RT, nrhs - r0);
    double acc[LRR_RT][VEC];
#pragma unroll
    for (int r = 0; r < LRR_RT; ++r)
#pragma unroll
      for (int v = 0; v < VEC; ++v) acc[r][v] = 0.0;
    for (int64_t gb = g0 + wv; gb < g1; gb += 4 * LRR_GU) {
      VT x[LRR_GU];
      double wr[LRR_GU][LRR_RT];
#pragma unroll
      for (int j = 0; j < LRR_GU; ++j) {
        const int64_t g = min(gb + 4 * j, g1 - 1);   // clamped groups add nothing (their weight is 0)
        x[j] = Uv[g * 64 + lane];
        const int64_t row = min(g * RG + rof, s - 1);
#pragma unroll
        for (int r = 0; r < LRR_RT; ++r)
          wr[j][r] = (r < nr && gb + 4 * j < g1) ? w[row + (int64_t)(r0 + r) * ldw] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < LRR_GU; ++j) {
        double u[VEC];
        lr_unpack<TU>(x[j], u);
#pragma unroll
        for (int r = 0; r < LRR_RT; ++r)
#pragma unroll
          for (int v = 0; v < VEC; ++v) acc[r][v] += u[v] * wr[j][r];
      }
    }
    // lanes l, l + cw, l + 2 cw, ... own the same columns
#pragma unroll
    for (int r = 0; r < LRR_RT; ++r)
#pragma unroll
      for (int v = 0; v < VEC; ++v) {
        double a = acc[r][v];
        for (int o = cw; o < 64; o <<= 1) a += __shfl_xor(a, o, 64);
        acc[r][v] = a;
      }
    if (lane < cw) {
#pragma unroll
      for (int r = 0; r < LRR_RT; ++r)
#pragma unroll
        for (int v = 0; v < VEC; ++v) red[wv][r * 64 + VEC * lane + v] = acc[r][v];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nr * ldk; t += blockDim.x) {
      const int r = t / ldk, q = t - r * ldk;
      if (q < k) {
        const double v = (red[0][r * 64 + q] + red[1][r * 64 + q]) + (red[2][r * 64 + q] + red[3][r * 64 + q]);
        part[((int64_t)blockIdx.x * nrhs + r0 + r) * k + q] = v;
      }
    }
    __syncthreads();
  }
}

// row-major padded copy of a column-major FP64 U (s x k)
template <typename TU>
__global__ void k_lr_to_rm(const double *U64, int64_t s, int k, int ldk, int64_t total, TU *Urm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t row = t / ldk;
  const int q = (int)(t - row * ldk);
  Urm[t] = (row < s && q < k) ? round_store<TU>(U64[row + (int64_t)q * s]) : (TU)0;
}

template <typename TU>
int64_t lr_rm_groups(int64_t s, int32_t k, int32_t &ldk) {
  constexpr int VEC = LrVec<TU>::V;
  ldk = VEC;
  while (ldk < k) ldk <<= 1;
  const int64_t RG = 64 * VEC / ldk;
  return (s + RG - 1) / RG;
}

template <typename TU>
void launch_lr_to_rm(const double *U64, int64_t s, int32_t k, TU *Urm, hipStream_t st) {
  int32_t ldk;
  const int64_t total = lr_rm_groups<TU>(s, k, ldk) * 64 * LrVec<TU>::V;
  if (total == 0) return;
  hipLaunchKernelGGL((k_lr_to_rm<TU>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, U64, s, k, ldk, total,
                     Urm);
}

// U^T w from the row-major copy Urm, the update from the column-major U
template <typename TU>
void launch_lowrank_rm(const TU *Urm, const TU *U, int64_t s, int32_t k, const double *dsc, double rho,
                       const double *w, int64_t ldw, double *wout, int64_t ldo, int32_t nrhs, double *part,
                       int32_t nblk, double *cbuf, hipStream_t st) {
  if (s == 0 || nrhs == 0) return;
  if (k == 0) {
    launch_axpby(s, nrhs, rho, w, ldw, 0.0, wout, ldo, st);
    return;
  }
  int32_t ldk;
  const int64_t ng = lr_rm_groups<TU>(s, k, ldk);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_lr_partial_rm<TU, 1, LRR_GU1>), dim3(nblk), dim3(256), 0, st, Urm, ldk, ng, s, k, w, ldw,
                       nrhs, part);
  else if (nrhs <= 4)
    hipLaunchKernelGGL((k_lr_partial_rm<TU, 4, 4>), dim3(nblk), dim3(256), 0, st, Urm, ldk, ng, s, k, w, ldw, nrhs,
                       part);
  else if (nrhs <= 8)
    hipLaunchKernelGGL((k_lr_partial_rm<TU, 8, 2>), dim3(nblk), dim3(256), 0, st, Urm, ldk, ng, s, k, w, ldw, nrhs,
                       part);
  else
    hipLaunchKernelGGL((k_lr_partial_rm<TU, 16, 1>), dim3(nblk), dim3(256), 0, st, Urm, ldk, ng, s, k, w, ldw, nrhs,
                       part);
  hipLaunchKernelGGL(k_lr_fold, dim3((unsigned)((k * nrhs + 3) / 4)), dim3(256), 0, st, part, nblk, k * nrhs, k,
                     dsc, cbuf);
  launch_lr_update<TU>(U, s, k, w, ldw, wout, ldo, nrhs, cbuf, rho, st);
}

// ---------------------------------------------------------------------------
// K4 on matrix cores (BF16 U_k, several right-hand sides).
// v_mfma_f32_16x16x16bf16_1k, one wave: D(16x16) += A(16x16) B(16x16) with
//   A: lane l holds A[l%16][4(l/16) + 0..3], B: lane l holds B[4(l/16)+0..3][l%16],
//   D: lane l register i holds D[4(l/16) + i][l%16].
// FP64 activations enter as three BF16 terms x = hi + mid + lo (each the
// nearest BF16 of what is left), so every product with a BF16 U entry is
// exact in FP32 and the contraction carries ~24 significant bits; only the
// stored U is rounded.  Accumulation is FP32 within a row chunk, FP64
// across chunks (the fold).
// ---------------------------------------------------------------------------
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
  return (short)u;
}
__device__ __forceinline__ float bf16_val(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

// x = hi + mid + lo, each BF16 (round to nearest even at every stage)
__device__ __forceinline__ void split3(double x, short &hi, short &mid, short &lo) {
  hi = bf16_bits((float)x);
  const double r1 = x - (double)bf16_val(hi);
  mid = bf16_bits((float)r1);
  const double r2 = r1 - (double)bf16_val(mid);
  lo = bf16_bits((float)r2);
}

constexpr int LRM_THREADS = 256;
constexpr int LRM_CT = 4;     // column tiles per pass (accumulators: kt x LRM_CT)

// BF16 U_k in 16 x 16 tiles of 512 bytes, each in the register layout of one
// MFMA operand, so that a lane loads its 4 entries as one 8-byte vector and
// a wave reads a whole tile in one coalesced 512-byte load.  Tile (b, t)
// covers rows 16 b .. 16 b + 15 and columns 16 t .. 16 t + 15 (zero
// padding past s and k) and sits at (b * kt + t) * 256 entries:
//   partial layout (A operand of U^T W): lane l, entry j = U[16 b + 4 (l/16) + j][16 t + l%16]
//   update layout (B operand of c^T U^T): lane l, entry j = U[16 b + l%16][16 t + 4 (l/16) + j]
__global__ void k_lr_to_tiles(const double *U64, int64_t s, int k, int kt, int64_t ntiles, short *Upt, short *Uup) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one thread per (tile, lane)
  if (g >= ntiles * 64) return;
  const int64_t tile = g >> 6;
  const int l = (int)(g & 63);
  const int64_t b = tile / kt;
  const int t = (int)(tile - b * kt);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t rp = 16 * b + 4 * (l >> 4) + j, ru = 16 * b + (l & 15);
    const int qp = 16 * t + (l & 15), qu = 16 * t + 4 * (l >> 4) + j;
    const double vp = (rp < s && qp < k) ? U64[rp + (int64_t)qp * s] : 0.0;
    const double vu = (ru < s && qu < k) ? U64[ru + (int64_t)qu * s] : 0.0;
    __hip_bfloat16 hp = round_store<__hip_bfloat16>(vp), hu = round_store<__hip_bfloat16>(vu);
    short sp, su;
    __builtin_memcpy(&sp, &hp, 2);
    __builtin_memcpy(&su, &hu, 2);
    Upt[g * 4 + j] = sp;
    Uup[g * 4 + j] = su;
  }
}

// part[b][c][q] = sum over the rows of chunk b of U[i,q] W[i,c], for all
// q < k, c < nrhs.  A block's chunk is a run of 16-row blocks (the split
// depends on s and the block count only); its 4 waves take every 4th row
// block, each accumulating all (q-tile, c-tile) pairs of a pass of up to
// LRM_CT column tiles: per row block W is loaded and split into its three
// BF16 terms once, and every U tile once.  The waves' sums are added in
// wave order through LDS.  A column's sums never depend on other columns.
__global__ void __launch_bounds__(LRM_THREADS) k_lr_partial_tiles(const short *Upt, int64_t s, int k,
                                                                  const double *W, int64_t ldw, int nrhs,
                                                                  double *part) {
  __shared__ float red[LRM_THREADS / 64][64][4];   // one (q-tile, c-tile) pair of every wave at a time
  const int kt = (k + 15) >> 4, nt = (nrhs + 15) >> 4;
  const int64_t nrb = (s + 15) >> 4;
  const int64_t per = (nrb + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(nrb, b0 + per);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t *U8 = reinterpret_cast<const uint64_t *>(Upt);
  for (int ct0 = 0; ct0 < nt; ct0 += LRM_CT) {
    const int nct = min(LRM_CT, nt - ct0);
    f32x4_t acc[4][LRM_CT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < LRM_CT; ++u) acc[t][u] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int64_t b = b0 + wid; b < b1; b += LRM_THREADS / 64) {
      bf16x4_t a[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint64_t v = t < kt ? U8[(b * kt + t) * 64 + lane] : 0ull;
        __builtin_memcpy(&a[t], &v, 8);
      }
#pragma unroll
      for (int u = 0; u < LRM_CT; ++u) {
        if (u >= nct) break;
        const int c = (ct0 + u) * 16 + (lane & 15);
        const bool cok = c < nrhs;
        bf16x4_t bh, bm, bl;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t row = 16 * b + 4 * (lane >> 4) + j;
          const double wv = (cok && row < s) ? W[row + (int64_t)c * ldw] : 0.0;
          short h, m, l;
          split3(wv, h, m, l);
          bh[j] = h;
          bm[j] = m;
          bl[j] = l;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (t >= kt) break;
          acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t], bh, acc[t][u], 0, 0, 0);
          acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t], bm, acc[t][u], 0, 0, 0);
          acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[t], bl, acc[t][u], 0, 0, 0);
        }
      }
    }
    // D[q][c]: q = 16 t + 4 (l/16) + i, c = 16 u + l%16; waves added in order
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= kt) break;
#pragma unroll
      for (int u = 0; u < LRM_CT; ++u) {
        if (u >= nct) break;
#pragma unroll
        for (int i = 0; i < 4; ++i) red[wid][lane][i] = acc[t][u][i];
        __syncthreads();
        {
          const int l = threadIdx.x >> 2, i = threadIdx.x & 3;
          const int q = 16 * t + 4 * (l >> 4) + i, c = (ct0 + u) * 16 + (l & 15);
          if (q < k && c < nrhs) {
            const float v = ((red[0][l][i] + red[1][l][i]) + red[2][l][i]) + red[3][l][i];
            part[((int64_t)blockIdx.x * nrhs + c) * k + q] = (double)v;
          }
        }
        __syncthreads();
      }
    }
  }
}

// wout[i,c] = rho w[i,c] + sum_q U[i,q] cbuf[c*k + q], as the transposed
// product (c x i) = c^T U^T: A = the coefficients (c-tile x q-tile, split
// into three BF16 terms in LDS), B = U tiles in the update layout; lane l
// register j then holds row 16 b + l%16 of column 16 u + 4 (l/16) + j, so
// 16 lanes store 16 consecutive rows of one column.  One wave per 16-row
// block; every column tile; U tiles loaded once per row block.
__global__ void __launch_bounds__(LRM_THREADS) k_lr_update_tiles(const short *Uup, int64_t s, int k,
                                                                 const double *w, int64_t ldw, double *wout,
                                                                 int64_t ldo, int nrhs, const double *cbuf,
                                                                 double rho) {
  extern __shared__ short cs3[];   // 3 x (npad x kpad), [term][c][q]
  const int kt = (k + 15) >> 4, kpad = kt * 16, npad = ((nrhs + 15) >> 4) * 16;
  for (int e = threadIdx.x; e < kpad * npad; e += blockDim.x) {
    const int c = e / kpad, q = e - c * kpad;
    const double v = (q < k && c < nrhs) ? cbuf[c * k + q] : 0.0;
    short h, m, l;
    split3(v, h, m, l);
    cs3[e] = h;
    cs3[kpad * npad + e] = m;
    cs3[2 * kpad * npad + e] = l;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * (LRM_THREADS / 64) + wid;
  if (16 * b >= s) return;
  const uint64_t *U8 = reinterpret_cast<const uint64_t *>(Uup);
  bf16x4_t ub[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint64_t v = t < kt ? U8[(b * kt + t) * 64 + lane] : 0ull;
    __builtin_memcpy(&ub[t], &v, 8);
  }
  const int64_t row = 16 * b + (lane & 15);
  for (int u = 0; u < npad / 16; ++u) {
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t >= kt) break;
      bf16x4_t ah, am, al;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // A[m = c][kk = q]: lane l holds A[l%16][4 (l/16) + j]
        const int e = (16 * u + (lane & 15)) * kpad + 16 * t + 4 * (lane >> 4) + j;
        ah[j] = cs3[e];
        am[j] = cs3[kpad * npad + e];
        al[j] = cs3[2 * kpad * npad + e];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, ub[t], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, ub[t], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, ub[t], acc, 0, 0, 0);
    }
    if (row < s) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * u + 4 * (lane >> 4) + i;
        if (c < nrhs) wout[row + (int64_t)c * ldo] = rho * w[row + (int64_t)c * ldw] + (double)acc[i];
      }
    }
  }
}

int64_t lr_tile_entries(int64_t s, int32_t k) { return ((s + 15) / 16) * (int64_t)((k + 15) / 16) * 256; }

void launch_lr_to_tiles(const double *U64, int64_t s, int32_t k, __hip_bfloat16 *Upt, __hip_bfloat16 *Uup,
                        hipStream_t st) {
  const int kt = (k + 15) / 16;
  const int64_t ntiles = ((s + 15) / 16) * kt;
  if (ntiles == 0) return;
  hipLaunchKernelGGL(k_lr_to_tiles, dim3((unsigned)((ntiles * 64 + 255) / 256)), dim3(256), 0, st, U64, s, k, kt,
                     ntiles, reinterpret_cast<short *>(Upt), reinterpret_cast<short *>(Uup));
}

void launch_lowrank_mfma(const __hip_bfloat16 *Upt, const __hip_bfloat16 *Uup, int64_t s, int32_t k,
                         const double *dsc, double rho, const double *w, int64_t ldw, double *wout, int64_t ldo,
                         int32_t nrhs, double *part, int32_t nblk, double *cbuf, hipStream_t st) {
  if (s == 0 || nrhs == 0 || k == 0) return;
  hipLaunchKernelGGL(k_lr_partial_tiles, dim3(nblk), dim3(LRM_THREADS), 0, st, reinterpret_cast<const short *>(Upt),
                     s, k, w, ldw, nrhs, part);
  hipLaunchKernelGGL(k_lr_fold, dim3((unsigned)((k * nrhs + 3) / 4)), dim3(256), 0, st, part, nblk, k * nrhs, k,
                     dsc, cbuf);
  const int kpad = ((k + 15) / 16) * 16, npad = ((nrhs + 15) / 16) * 16;
  const size_t lds = sizeof(short) * 3 * (size_t)kpad * npad;
  const int64_t nrb = (s + 15) / 16;
  hipLaunchKernelGGL(k_lr_update_tiles, dim3((unsigned)((nrb + 3) / 4)), dim3(LRM_THREADS), lds, st,
                     reinterpret_cast<const short *>(Uup), s, k, w, ldw, wout, ldo, nrhs, cbuf, rho);
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
  (void)counter;
  hipLaunchKernelGGL((k_lr_partial<TU>), dim3(nblk), dim3(LR_THREADS), 0, st, U, s, k, w, ldw, nrhs, part);
  hipLaunchKernelGGL(k_lr_fold, dim3((unsigned)((k * nrhs + 3) / 4)), dim3(256), 0, st, part, nblk, k * nrhs, k,
                     dsc, cbuf);
  launch_lr_update<TU>(U, s, k, w, ldw, wout, ldo, nrhs, cbuf, rho, st);
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
// y = A x for up to SPMV_T columns per thread (blockIdx.y picks the column
// tile): each row's entries are read once per tile; every column sums its
// row in entry order.
constexpr int SPMV_T = 8;

// acc[t] += sum_e v[e] x[ci[e] + (c0 + t) ldx] for the entries e0 <= e < e1
// of one CSR row, in entry order, for the columns t < T with act[t].  The
// value, index and gather loads of U entries at a time go out together
// (loads past the row end are clamped to its last entry and not added).
template <int T, int U>
__device__ __forceinline__ void csr_row_acc(int64_t e0, int64_t e1, const int32_t *ci, const double *v,
                                            const double *x, int64_t ldx, int c0, const bool *act, double *acc) {
  for (int64_t e = e0; e < e1; e += U) {
    double a[U], xv[U][T];
    int64_t j[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t ee = min(e + u, e1 - 1);
      a[u] = v[ee];
      j[u] = ci[ee];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < T; ++t) xv[u][t] = act[t] ? x[j[u] + (int64_t)(c0 + t) * ldx] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e + u < e1)
#pragma unroll
        for (int t = 0; t < T; ++t)
          if (act[t]) acc[t] += a[u] * xv[u][t];
  }
}

template <int T>
__global__ void __launch_bounds__(256) k_spmv(int64_t n, const int64_t *rp, const int32_t *ci,
                                              const double *v, const double *x, int64_t ldx, double *y,
                                              int64_t ldy, int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = blockIdx.y * T, nct = min(T, nrhs - c0);
  double acc[T];
  bool act[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    acc[t] = 0.0;
    act[t] = t < nct;
  }
  csr_row_acc<T, T == 1 ? 8 : 2>(rp[i], rp[i + 1], ci, v, x, ldx, c0, act, acc);
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (t < nct) y[i + (int64_t)(c0 + t) * ldy] = acc[t];
}

void launch_spmv(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                 int64_t ldx, double *y, int64_t ldy, int32_t nrhs, hipStream_t st) {
  if (n == 0 || nrhs == 0) return;
  const unsigned gx = (unsigned)((n + 255) / 256);
  if (nrhs == 1)
    hipLaunchKernelGGL(k_spmv<1>, dim3(gx, 1), dim3(256), 0, st, n, rp, ci, v, x, ldx, y, ldy, nrhs);
  else
    hipLaunchKernelGGL(k_spmv<SPMV_T>, dim3(gx, (nrhs + SPMV_T - 1) / SPMV_T), dim3(256), 0, st, n, rp, ci, v, x,
                       ldx, y, ldy, nrhs);
}

// y = a y + b M x for CSR M (int64 row pointers), SPMV_T columns per thread;
// with a == 0 y is only written.  Every column sums its row in entry order.
template <int T>
__global__ void __launch_bounds__(256) k_spmv_axpby(int64_t n, const int64_t *rp, const int32_t *ci,
                                                    const double *v, const double *x, int64_t ldx, double *y,
                                                    int64_t ldy, int nrhs, double a, double b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c0 = blockIdx.y * T, nct = min(T, nrhs - c0);
  double acc[T];
  bool act[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    acc[t] = 0.0;
    act[t] = t < nct;
  }
  csr_row_acc<T, T == 1 ? 8 : 2>(rp[i], rp[i + 1], ci, v, x, ldx, c0, act, acc);
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (t < nct) {
      double *yp = y + i + (int64_t)(c0 + t) * ldy;
      *yp = (a != 0.0 ? a * *yp : 0.0) + b * acc[t];
    }
}

void launch_spmv_axpby(int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const double *x,
                       int64_t ldx, double *y, int64_t ldy, int32_t nrhs, double a, double b, hipStream_t st) {
  if (n == 0 || nrhs == 0) return;
  const unsigned gx = (unsigned)((n + 255) / 256);
  if (nrhs == 1)
    hipLaunchKernelGGL(k_spmv_axpby<1>, dim3(gx, 1), dim3(256), 0, st, n, rp, ci, v, x, ldx, y, ldy, nrhs, a, b);
  else
    hipLaunchKernelGGL(k_spmv_axpby<SPMV_T>, dim3(gx, (nrhs + SPMV_T - 1) / SPMV_T), dim3(256), 0, st, n, rp, ci,
                       v, x, ldx, y, ldy, nrhs, a, b);
}

// ---------------------------------------------------------------------------
// K6: Krylov BLAS-1 with deterministic reductions, CG / flexible CG.
// Every reduction writes per-block partials part[b*width + col]; the next
// kernel's blocks each fold them (identically) in LDS.  No kernel reads a
// state field that a block of the same kernel writes, except `active`,
// whose update (active && !stop) gives the same answer before and after;
// the scalars carried between iterations are double-buffered by iteration
// parity (read from one slot, written to the other).
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;
constexpr int MAX_FOLD = 512;   // folded values per launch (up to 4 per column, 128 columns)

__device__ __forceinline__ void fold_to_lds(const double *part, int nb, int width, double *fin) {
  fold_waves(part, nb, width, [&](int col, double v) { fin[col] = v; });
  __syncthreads();
}

// Row chunks of the reduction kernels, which run RED_THREADS threads per
// block (a constant here, so that no row index waits for the launch's block
// size to be read).
template <int BD = RED_THREADS, class F>
__device__ __forceinline__ void chunk_rows(int64_t n, F f) {
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += BD) f(i);
}

// The rows chunk_rows gives this thread, i0 + t + j * blockDim.x, in
// batches of RPT: ld(r, i) issues row i's loads into register slot r, op(r,
// i) consumes them, rows in ascending order (so per-thread sums come out as
// with chunk_rows).  mid() runs once in every thread, after the first
// batch's loads went out and before any op: a fold whose result op needs
// overlaps with them.
template <int RPT, class Ld, class Mid, class Op>
__device__ __forceinline__ void chunk_rows_pf(int64_t n, Ld ld, Mid mid, Op op) {
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  constexpr int64_t bd = RED_THREADS;
  int64_t b = i0 + threadIdx.x;
#pragma unroll
  for (int r = 0; r < RPT; ++r)
    if (b + r * bd < i1) ld(r, b + r * bd);
  mid();
  while (b < i1) {
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      if (b + r * bd < i1) op(r, b + r * bd);
    b += RPT * bd;
    if (b >= i1) break;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      if (b + r * bd < i1) ld(r, b + r * bd);
  }
}

constexpr int CG_RPT = 4;   // rows per thread whose loads go out together

// One column, y = A x, the rows of this thread's chunk one at a time (BD
// threads per block): a row's pointer loads and own(i) (the loads of the
// row's own vector entries) go out together, then its entry loads, U per
// round (past the row's end clamped to its last entry, not added), then
// the gathers; emit(i, y_i) consumes them.  Entries are summed in order.
template <int U, int BD, class Own, class Emit>
__device__ __forceinline__ void spmv_rows(int64_t n, const int64_t *rp, const int32_t *ci, const double *v,
                                          const double *x, Own own, Emit emit) {
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += BD) {
    const int64_t e0 = rp[i], e1 = rp[i + 1];
    own(i);
    double y = 0.0;
    for (int64_t e = e0; e < e1; e += U) {
      double a[U], xv[U];
      int32_t j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t ee = min(e + u, e1 - 1);
        a[u] = v[ee];
        j[u] = ci[ee];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) xv[u] = x[j[u]];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (e + u < e1) y += a[u] * xv[u];
    }
    emit(i, y);
  }
}

// start: x = 0, partial b.b -> part2 (r holds b)
__global__ void __launch_bounds__(RED_THREADS) k_cg_init(int64_t n, KArgs K, int c0, int nc) {
  __shared__ double sh[RED_THREADS / 64];
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    const double *rc = K.R + (int64_t)c * K.ld;
    double *xc = K.X + (int64_t)c * K.ld;
    double acc = 0.0;
    chunk_rows(n, [&](int64_t i) {
      acc += rc[i] * rc[i];
      xc[i] = 0.0;
    });
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) K.part2[(int64_t)blockIdx.x * nc + cc] = t;
  }
}

// true residual: partial ||b - A x||^2 (AX holds A x) -> part2; then fold
__global__ void __launch_bounds__(RED_THREADS) k_relres(int64_t n, const double *B, int64_t ldb, const double *AX,
                                                        int64_t ldax, KArgs K, int nc) {
  __shared__ double sh[RED_THREADS / 64];
  for (int cc = 0; cc < nc; ++cc) {
    double acc = 0.0;
    chunk_rows(n, [&](int64_t i) {
      const double d = B[i + (int64_t)cc * ldb] - AX[i + (int64_t)cc * ldax];
      acc += d * d;
    });
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) K.part2[(int64_t)blockIdx.x * nc + cc] = t;
  }
}

__global__ void __launch_bounds__(RED_THREADS) k_relres2(KArgs K, int c0, int nc) {
  __shared__ double fin[MAX_FOLD];
  fold_to_lds(K.part2, K.nblk, nc, fin);
  for (int cc = threadIdx.x; cc < nc; cc += blockDim.x) {
    KState &s = K.st[c0 + cc];
    s.relres = s.bb > 0.0 ? sqrt(fin[cc] / s.bb) : 0.0;
  }
}

// ---------------------------------------------------------------------------
// CG and flexible CG with one reduction phase per iteration.  With z =
// M^{-1} r and w = A z of the current r, and s = A p kept beside p:
//   gamma = r.z, delta = z.w, and for the flexible form eps = z.s_prev;
//   plain (Chronopoulos and Gear):  beta = gamma / gamma_prev,
//                                   p.Ap = delta - beta gamma / alpha_prev
//   flexible (beta makes p A-orthogonal to p_prev):
//                                   beta = -eps / (p.Ap)_prev,
//                                   p.Ap = delta + beta eps
//   (beta = 0 and p.Ap = delta at a column's first iteration);
//   alpha = gamma / p.Ap ; p = z + beta p ; s = w + beta s ;
//   x += alpha p ; r -= alpha s.
// In exact arithmetic these are the iterates of the two-reduction forms (the
// flexible p.Ap uses p_prev . A z = z . A p_prev, A symmetric).  r.r of the
// current r is summed in the same pass, so the convergence test of r_i comes
// just before update i.  One iteration: preconditioner (z), k_cg_spmv (w
// and the partials), k_cg_update.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cg_np(int flexible) { return flexible ? 4 : 3; }

// w = A z ; partials gamma, delta, rho = r.r (, eps) ->
// part[b*np*nc + np*cc + (0, 1, 2 (, 3))]
// One column (slr_solve with one right-hand side): 512 threads per block,
// one row per thread at 512 rows per block, for the loads in flight.  No
// load waits for the column's state: an inactive column's w and partials
// are never used.
constexpr int CG_SPMV1_THREADS = 512;

__global__ void __launch_bounds__(CG_SPMV1_THREADS) k_cg_spmv1(int64_t n, const int64_t *rp, const int32_t *ci,
                                                                const double *v, KArgs K, int c0, int flexible) {
  __shared__ double sh[4 * (CG_SPMV1_THREADS / 64)];
  const int np = cg_np(flexible);
  const double *Z = K.Z + (int64_t)c0 * K.ld, *R = K.R + (int64_t)c0 * K.ld, *S = K.S + (int64_t)c0 * K.ld;
  double *W = K.Q + (int64_t)c0 * K.ld;
  double g = 0.0, d = 0.0, rr = 0.0, ep = 0.0, zv = 0.0, rv = 0.0, sv = 0.0;
  spmv_rows<8, CG_SPMV1_THREADS>(
      n, rp, ci, v, Z,
      [&](int64_t i) {
        zv = Z[i];
        rv = R[i];
        if (flexible) sv = S[i];
      },
      [&](int64_t i, double w) {
        W[i] = w;
        g += rv * zv;
        d += zv * w;
        rr += rv * rv;
        if (flexible) ep += zv * sv;
      });
  double t[4] = {g, d, rr, ep};
  block_sums<4>(t, sh);
  if (threadIdx.x == 0)
    for (int j = 0; j < np; ++j) K.part[(int64_t)blockIdx.x * np + j] = t[j];
}

// Column tiles of TT (several right-hand sides, and every batch): each row's
// entries are read once per tile, and a column's arithmetic (entry order,
// row order, block sums) does not depend on the tile it falls in or on the
// number of columns.
template <int TT>
__global__ void __launch_bounds__(RED_THREADS) k_cg_spmv(int64_t n, const int64_t *rp, const int32_t *ci,
                                                         const double *v, KArgs K, int c0, int nc, int flexible) {
  __shared__ double sh[4 * (RED_THREADS / 64)];
  const int np = cg_np(flexible);
  for (int ct = 0; ct < nc; ct += TT) {
    const int nct = min(TT, nc - ct);
    bool act[TT];
    double g[TT], d[TT], rr[TT], ep[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      act[t] = t < nct && K.st[c0 + ct + t].active;
      g[t] = d[t] = rr[t] = ep[t] = 0.0;
    }
    chunk_rows(n, [&](int64_t i) {
      double sum[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t) sum[t] = 0.0;
      csr_row_acc<TT, TT == 1 ? 8 : 2>(rp[i], rp[i + 1], ci, v, K.Z, K.ld, c0 + ct, act, sum);
#pragma unroll
      for (int t = 0; t < TT; ++t)
        if (act[t]) {
          const int64_t o = i + (int64_t)(c0 + ct + t) * K.ld;
          const double zi = K.Z[o], ri = K.R[o];
          K.Q[o] = sum[t];
          g[t] += ri * zi;
          d[t] += zi * sum[t];
          rr[t] += ri * ri;
          if (flexible) ep[t] += zi * K.S[o];
        }
    });
    for (int t = 0; t < nct; ++t) {
      double u[4] = {g[t], d[t], rr[t], ep[t]};
      block_sums<4>(u, sh);
      if (threadIdx.x == 0)
        for (int j = 0; j < np; ++j) K.part[(int64_t)blockIdx.x * np * nc + np * (ct + t) + j] = u[j];
    }
  }
}

// The decision of iteration `it` for one column from its folded partials f
// (gamma, delta, rho, eps): stop (converged, iteration limit, or a
// non-finite residual), break down (no positive curvature), or update with
// alpha, beta; pap = p.Ap of the new p.
struct CgStep {
  bool stop, ok, brk, first;
  int done;
  double alpha, beta, pap;
};

__device__ __forceinline__ CgStep cg_step(const KState &s, const double *f, int it, int maxit, double rtol2,
                                            int flexible) {
  CgStep q;
  const double gam = f[0], del = f[1], rho = f[2];
  q.done = it - s.start_it;
  q.ok = rho <= rtol2 * s.bb;
  q.stop = q.ok || q.done >= maxit || !isfinite(rho);
  q.first = q.done == 0;
  if (q.first) {
    q.beta = 0.0;
    q.pap = del;
  } else if (flexible) {
    q.beta = -f[3] / s.pq[(it - 1) & 1];
    q.pap = del + q.beta * f[3];
  } else {
    q.beta = gam / s.rz[(it - 1) & 1];
    q.pap = del - q.beta * gam / s.al[(it - 1) & 1];
  }
  q.alpha = gam / q.pap;
  q.brk = !(q.pap > 0.0) || !isfinite(q.alpha);
  return q;
}

// fold ; stop or p = z + beta p, s = w + beta s, x += alpha p, r -= alpha s
// (the first column's vectors are loaded while the partials are folded)
__global__ void __launch_bounds__(RED_THREADS) k_cg_update(int64_t n, KArgs K, int c0, int nc, int flexible,
                                                            int it) {
  __shared__ double fin[MAX_FOLD];
  const int np = cg_np(flexible);
  for (int cc = 0; cc < nc; ++cc) {
    const int c = c0 + cc;
    const KState &s = K.st[c];
    const bool live = s.active;
    const int64_t o = (int64_t)c * K.ld;
    double *X = K.X + o, *R = K.R + o, *P = K.P + o, *S = K.S + o;
    const double *Z = K.Z + o, *W = K.Q + o;
    double xv[CG_RPT], rv[CG_RPT], pv[CG_RPT], sv[CG_RPT], zv[CG_RPT], wv[CG_RPT];
    CgStep q{};
    bool go = false;
    chunk_rows_pf<CG_RPT>(
        n,
        [&](int r, int64_t i) {
          if (cc == 0 || live) {
            xv[r] = X[i];
            rv[r] = R[i];
            pv[r] = P[i];
            sv[r] = S[i];
            zv[r] = Z[i];
            wv[r] = W[i];
          }
        },
        [&]() {
          if (cc == 0) fold_to_lds(K.part, K.nblk, np * nc, fin);
          q = cg_step(s, fin + np * cc, it, K.maxit, K.rtol2, flexible);
          go = live && !q.stop && !q.brk;
        },
        [&](int r, int64_t i) {
          if (go) {
            const double pn = q.first ? zv[r] : zv[r] + q.beta * pv[r];
            const double sn = q.first ? wv[r] : wv[r] + q.beta * sv[r];
            P[i] = pn;
            S[i] = sn;
            X[i] = xv[r] + q.alpha * pn;
            R[i] = rv[r] - q.alpha * sn;
          }
        });
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int cc = threadIdx.x; cc < nc; cc += RED_THREADS) {
      KState &s = K.st[c0 + cc];
      if (!s.active) continue;
      const CgStep q = cg_step(s, fin + np * cc, it, K.maxit, K.rtol2, flexible);
      s.rr = fin[np * cc + 2];
      if (q.stop || q.brk) {
        s.active = 0;
        s.status = (q.stop && q.ok) ? 0 : -8;
        s.iters = q.done;
      } else {
        s.rz[it & 1] = fin[np * cc];
        s.al[it & 1] = q.alpha;
        s.pq[it & 1] = q.pap;
        s.alpha = q.alpha;
        s.beta = q.beta;
        s.iters = q.done + 1;
      }
    }
  }
}

// start of columns [c0, c0+nc) after k_cg_init (x = 0, partial b.b): fold
// b.b and set the state; the first iteration index is it0
__global__ void __launch_bounds__(RED_THREADS) k_cg_start(KArgs K, int c0, int nc, int it0) {
  __shared__ double fin[MAX_FOLD];
  fold_to_lds(K.part2, K.nblk, nc, fin);
  for (int cc = threadIdx.x; cc < nc; cc += RED_THREADS) {
    KState &s = K.st[c0 + cc];
    const double bb = fin[cc];
    s.bb = bb;
    s.rr = bb;
    s.iters = 0;
    s.start_it = it0;
    s.alpha = s.beta = 0.0;
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

void launch_cg(int op, int64_t n, const int64_t *rp, const int32_t *ci, const double *v, const KArgs &K,
               int32_t c0, int32_t nc, int32_t flexible, int32_t it, hipStream_t st) {
  if (nc == 0) return;
  const int nb = K.nblk;
  switch (op) {
    case CG_INIT:
      hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(RED_THREADS), 0, st, n, K, c0, nc);
      break;
    case CG_START:
      hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(RED_THREADS), 0, st, K, c0, nc, it);
      break;
    case CG_SPMV:
      if (nc == 1) {
        hipLaunchKernelGGL(k_cg_spmv1, dim3(nb), dim3(CG_SPMV1_THREADS), 0, st, n, rp, ci, v, K, c0, flexible);
        break;
      }
      [[fallthrough]];
    case CG_SPMV_TILES:
      hipLaunchKernelGGL(k_cg_spmv<SPMV_T>, dim3(nb), dim3(RED_THREADS), 0, st, n, rp, ci, v, K, c0, nc, flexible);
      break;
    case CG_UPDATE:
      hipLaunchKernelGGL(k_cg_update, dim3(nb), dim3(RED_THREADS), 0, st, n, K, c0, nc, flexible, it);
      break;
    default:
      break;
  }
}

void launch_relres(int64_t n, const double *B, int64_t ldb, const double *AX, int64_t ldax, const KArgs &K,
                   int32_t c0, int32_t nc, hipStream_t st) {
  if (nc == 0) return;
  hipLaunchKernelGGL(k_relres, dim3(K.nblk), dim3(RED_THREADS), 0, st, n, B, ldb, AX, ldax, K, nc);
  hipLaunchKernelGGL(k_relres2, dim3(1), dim3(RED_THREADS), 0, st, K, c0, nc);
}

// ---------------------------------------------------------------------------
// Single-vector reductions / Gram-Schmidt (Lanczos K7 and FGMRES K10), FP64
// ---------------------------------------------------------------------------
// out[j] = sum_i V[i + j*ldv] * w[i]  for j < J   (V^T w)
// Grid (RB, J): block (rb, j) sums column j over row chunk rb into
// part[rb*J + j] (four independent accumulators per thread); k_fold then
// sums the RB partials of every column.
__global__ void __launch_bounds__(256) k_multidot(int64_t s, int J, const double *V, int64_t ldv,
                                                  const double *w, double *part, const int *gate) {
  if (gate && *gate == 0) return;   // skipped step (partial reorthogonalisation)
  __shared__ double sh[4];
  const int rb = blockIdx.x, nb = gridDim.x, j = blockIdx.y;
  const int64_t chunk = (s + nb - 1) / nb;
  const int64_t i0 = (int64_t)rb * chunk, i1 = min(s, i0 + chunk);
  const double *vj = V + (int64_t)j * ldv;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int64_t step = blockDim.x;
  int64_t i = i0 + threadIdx.x;
  for (; i + 3 * step < i1; i += 4 * step) {
    a0 += vj[i] * w[i];
    a1 += vj[i + step] * w[i + step];
    a2 += vj[i + 2 * step] * w[i + 2 * step];
    a3 += vj[i + 3 * step] * w[i + 3 * step];
  }
  for (; i < i1; i += step) a0 += vj[i] * w[i];
  const double t = block_sum((a0 + a1) + (a2 + a3), sh);
  if (threadIdx.x == 0) part[(int64_t)rb * J + j] = t;
}

// sum_j V[i + j*ldv] c[j] in column order, 32 loads in flight (the last
// group clamps its column index and multiplies padding by zero)
__device__ __forceinline__ double dot_rows32(const double *V, int64_t ldv, int64_t i, const double *c, int J) {
  double acc = 0.0;
  for (int j0 = 0; j0 < J; j0 += 32) {
    double v[32];
#pragma unroll
    for (int e = 0; e < 32; ++e) v[e] = V[i + (int64_t)min(j0 + e, J - 1) * ldv];
#pragma unroll
    for (int e = 0; e < 32; ++e)
      if (j0 + e < J) acc += v[e] * c[j0 + e];
  }
  return acc;
}

// w[i] -= sum_j V[i + j*ldv] h[j]   (J <= 1024).  h is either on the
// device (hpart == nullptr) or folded here from the rb multidot partials
// hpart[b*J + j] (one thread per coefficient, partials in block order; block
// 0 also stores the folded h to hout when given).  sqpart (optional):
// per-block sums of the updated w[i]^2, block b at sqpart[b].  gate
// (optional): the whole grid returns at once when *gate == 0.
__global__ void __launch_bounds__(256) k_gemv_sub(int64_t s, int J, const double *V, int64_t ldv,
                                                  const double *h, double *w, const double *hpart, int rb,
                                                  double *sqpart, double *hout, const int *gate) {
  if (gate && *gate == 0) return;
  __shared__ double hs[1024];
  __shared__ double sh[4];
  if (hpart) {
    for (int j = threadIdx.x; j < J; j += blockDim.x) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int b = 0;
      for (; b + 3 < rb; b += 4) {
        a0 += hpart[(int64_t)b * J + j];
        a1 += hpart[(int64_t)(b + 1) * J + j];
        a2 += hpart[(int64_t)(b + 2) * J + j];
        a3 += hpart[(int64_t)(b + 3) * J + j];
      }
      for (; b < rb; ++b) a0 += hpart[(int64_t)b * J + j];
      const double v = (a0 + a1) + (a2 + a3);
      hs[j] = v;
      if (hout && blockIdx.x == 0) hout[j] = v;
    }
  } else {
    for (int j = threadIdx.x; j < J; j += blockDim.x) hs[j] = h[j];
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double wn = 0.0;
  if (i < s) {
    wn = w[i] - dot_rows32(V, ldv, i, hs, J);
    w[i] = wn;
  }
  if (sqpart) {
    const double t = block_sum(wn * wn, sh);
    if (threadIdx.x == 0) sqpart[blockIdx.x] = t;
  }
}

int32_t launch_multidot_partial(int64_t s, int32_t J, const double *V, int64_t ldv, const double *w, double *part,
                                int32_t nblk, hipStream_t st, const int *gate) {
  const int64_t rb =
      std::max<int64_t>(1, std::min<int64_t>({(int64_t)nblk, (1024 + J - 1) / J, (s + 1023) / 1024}));
  hipLaunchKernelGGL(k_multidot, dim3((unsigned)rb, J), dim3(256), 0, st, s, J, V, ldv, w, part, gate);
  return (int32_t)rb;
}

void launch_multidot(int64_t s, int32_t J, const double *V, int64_t ldv, const double *w, double *part,
                     int32_t nblk, double *out, unsigned int *counter, hipStream_t st) {
  // row chunks: about 1024 blocks in total, at least 2048 rows per chunk
  int64_t rb = std::max<int64_t>(1, std::min<int64_t>({(int64_t)nblk, (1024 + J - 1) / J, (s + 1023) / 1024}));
  (void)counter;
  hipLaunchKernelGGL(k_multidot, dim3((unsigned)rb, J), dim3(256), 0, st, s, J, V, ldv, w, part,
                     (const int *)nullptr);
  launch_fold(part, (int32_t)rb, J, out, 1.0, st);
}

int32_t launch_gemv_sub(int64_t s, int32_t J, const double *V, int64_t ldv, const double *h, double *w,
                        double *sqpart, hipStream_t st) {
  const unsigned nb = (unsigned)((s + 255) / 256);
  hipLaunchKernelGGL(k_gemv_sub, dim3(nb), dim3(256), 0, st, s, J, V, ldv, h, w, (const double *)nullptr, 0,
                     sqpart, (double *)nullptr, (const int *)nullptr);
  return (int32_t)nb;
}

int32_t launch_gemv_sub_fold(int64_t s, int32_t J, const double *V, int64_t ldv, const double *hpart, int32_t rb,
                             double *w, double *hout, double *sqpart, hipStream_t st, const int *gate) {
  const unsigned nb = (unsigned)((s + 255) / 256);
  hipLaunchKernelGGL(k_gemv_sub, dim3(nb), dim3(256), 0, st, s, J, V, ldv, (const double *)nullptr, w, hpart, rb,
                     sqpart, hout, gate);
  return (int32_t)nb;
}

// Lanczos three-term step: alpha = v.w folded from the rb multidot
// partials (block 0 stores it in sc[0]);  w -= alpha v + b_prev v_prev
// with b_prev = sc[1]; per-block sums of the new w^2 go to sqpart (same
// grid as k_gemv_sub, so either kernel's partials can be folded alike).
__global__ void __launch_bounds__(256) k_lanczos_axpy(int64_t s, double *w, const double *v, const double *vprev,
                                                      double *sc, const double *apart, int rb, double *sqpart) {
  __shared__ double al;
  __shared__ double sh[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // the vectors do not depend on alpha: their loads overlap with the fold
  double wi = 0.0, vi = 0.0, pi = 0.0, bp = 0.0;
  if (i < s) {
    wi = w[i];
    vi = v[i];
    if (vprev) {
      pi = vprev[i];
      bp = sc[1];
    }
  }
  fold_waves(apart, rb, 1, [&](int, double x) { al = x; });
  __syncthreads();
  const double a = al;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[0] = a;
  double t = 0.0;
  if (i < s) {
    t = wi - a * vi;
    if (vprev) t -= bp * pi;
    w[i] = t;
  }
  const double q = block_sum(t * t, sh);
  if (threadIdx.x == 0) sqpart[blockIdx.x] = q;
}

int32_t launch_lanczos_axpy(int64_t s, double *w, const double *v, const double *vprev, double *sc,
                            const double *apart, int32_t rb, double *sqpart, hipStream_t st) {
  const unsigned nb = (unsigned)((s + 255) / 256);
  hipLaunchKernelGGL(k_lanczos_axpy, dim3(nb), dim3(256), 0, st, s, w, v, vprev, sc, apart, rb, sqpart);
  return (int32_t)nb;
}

// Partial reorthogonalisation control for Lanczos step j (Sec. 5.1, the
// omega recurrence of Parlett and Simon), run at the start of every block
// of the step's (gated) Gram-Schmidt coefficient kernel.  Every block takes
// the same decision from the same data; the writer block records it.
// Thread l < j estimates om_{j+1,l} ~ v_{j+1}.v_l from rows om_j (row j % 3)
// and om_{j-1} (row (j+2) % 3) of om (3 rows of ld):
//   beta_j om_{j+1,l} = beta_l om_{j,l+1} + (alpha_l - alpha_j) om_{j,l}
//                       + beta_{l-1} om_{j,l-1} - beta_{j-1} om_{j-1,l}
// (unit diagonal), plus the rounding term e = eps sqrt(s) ||T_j|| with the
// estimate's sign; om_{j+1,j} = e / beta_j.  beta_j is the norm before any
// reorthogonalisation (folded from the rb partials bpart), alpha_j = sc[0],
// alpha_l / beta_l (l < j) from the recorded coefficients, ||T_j|| the
// running max of |alpha_i| + beta_i + beta_{i-1} (tn[j] before the step,
// tn[j+1] after).  Reorthogonalise when forced (frc[j]) or when some
// |om_{j+1,l}| exceeds sqrt(eps); a step triggered by the estimate forces
// the next one (frc[j+1]).  The decision goes to rflag[j]; a cleaned row is
// reset to e / beta_j.
struct ProArgs {
  int j;
  double sqrt_s;
  const double *alpha, *beta, *sc, *bpart;
  int rb;
  double *om;
  int ld;
  int *frc;
  double *tn;
  int *rflag;
};

__device__ int pro_step(const ProArgs &P, bool writer) {
  __shared__ double bsh, red[16];
  __shared__ int dosh;
  const int j = P.j;
  const double *W0 = P.om + (int64_t)(j % 3) * P.ld;
  const double *Wm = P.om + (int64_t)((j + 2) % 3) * P.ld;
  double *Wp = P.om + (int64_t)((j + 1) % 3) * P.ld;
  // the recurrence inputs of entry l = threadIdx.x do not depend on beta_j:
  // their loads go out before the fold
  struct EstIn {
    double up, prev, bl, al, w0, bl1, wl1;
  };
  auto est_in = [&](int l) {
    EstIn q;
    q.up = l + 1 == j ? 1.0 : W0[l + 1];
    q.prev = l == j - 1 ? 1.0 : Wm[l];
    q.bl = P.beta[l];
    q.al = P.alpha[l];
    q.w0 = W0[l];
    q.bl1 = l > 0 ? P.beta[l - 1] : 0.0;
    q.wl1 = l > 0 ? W0[l - 1] : 0.0;
    return q;
  };
  const int l0 = threadIdx.x;
  EstIn q0{};
  if (l0 < j) q0 = est_in(l0);
  const double aj = P.sc[0], bm = j > 0 ? P.beta[j - 1] : 0.0, tnj = P.tn[j];
  fold_waves(P.bpart, P.rb, 1, [&](int, double x) { bsh = sqrt(x); });
  __syncthreads();
  const double eps = 0x1p-52;
  const double bj = bsh;
  const double tnorm = fmax(tnj, fabs(aj) + bj + bm);
  const double e = eps * P.sqrt_s * tnorm;
  const double psi = bj > 0.0 ? e / bj : 1.0;
  auto est_of = [&](int l, const EstIn &q) {
    if (l == j) return psi;
    double t = q.bl * q.up + (q.al - aj) * q.w0 - bm * q.prev;
    if (l > 0) t += q.bl1 * q.wl1;
    t += copysign(e, t);
    return bj > 0.0 ? t / bj : 1.0;
  };
  auto est = [&](int l) { return l == j ? psi : est_of(l, l == l0 ? q0 : est_in(l)); };
  double m = 0.0;
  for (int l = threadIdx.x; l <= j; l += blockDim.x) m = fmax(m, fabs(est(l)));
  m = wave_allmax(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) mx = fmax(mx, red[i]);
    const int force = P.frc[j];
    const int big = mx > 0x1p-26;
    dosh = force || big;
    if (writer) {
      P.frc[j + 1] = force ? 0 : big;
      P.tn[j + 1] = tnorm;
      P.rflag[j] = dosh;
    }
  }
  __syncthreads();
  const int d = dosh;
  if (writer)
    for (int l = threadIdx.x; l <= j; l += blockDim.x) Wp[l] = d ? psi : est(l);
  return d;
}

// k_multidot preceded by the partial reorthogonalisation decision; the
// whole grid returns when the step is not cleaned
__global__ void __launch_bounds__(256) k_multidot_pro(int64_t s, int J, const double *V, int64_t ldv,
                                                      const double *w, double *part, ProArgs P) {
  if (!pro_step(P, blockIdx.x == 0 && blockIdx.y == 0)) return;
  __shared__ double sh[4];
  const int rb = blockIdx.x, nb = gridDim.x, jj = blockIdx.y;
  const int64_t chunk = (s + nb - 1) / nb;
  const int64_t i0 = (int64_t)rb * chunk, i1 = min(s, i0 + chunk);
  const double *vj = V + (int64_t)jj * ldv;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int64_t step = blockDim.x;
  int64_t i = i0 + threadIdx.x;
  for (; i + 3 * step < i1; i += 4 * step) {
    a0 += vj[i] * w[i];
    a1 += vj[i + step] * w[i + step];
    a2 += vj[i + 2 * step] * w[i + 2 * step];
    a3 += vj[i + 3 * step] * w[i + 3 * step];
  }
  for (; i < i1; i += step) a0 += vj[i] * w[i];
  const double t = block_sum((a0 + a1) + (a2 + a3), sh);
  if (threadIdx.x == 0) part[(int64_t)rb * J + jj] = t;
}

int32_t launch_multidot_pro(int64_t s, int32_t J, const double *V, int64_t ldv, const double *w, double *part,
                            int32_t nblk, int32_t j, const double *alpha, const double *beta, const double *sc,
                            const double *bpart, int32_t rbp, double *om, int32_t ld, int *frc, double *tn,
                            int *rflag, hipStream_t st) {
  const int64_t rb =
      std::max<int64_t>(1, std::min<int64_t>({(int64_t)nblk, (1024 + J - 1) / J, (s + 1023) / 1024}));
  ProArgs P{j, std::sqrt((double)s), alpha, beta, sc, bpart, rbp, om, ld, frc, tn, rflag};
  hipLaunchKernelGGL(k_multidot_pro, dim3((unsigned)rb, J), dim3(256), 0, st, s, J, V, ldv, w, part, P);
  return (int32_t)rb;
}

// End of Lanczos step j: beta_j = ||w|| folded from the rb multidot
// partials; v_{j+1} = w / beta_j (if vnext); block 0 records alpha_j
// (sc[0]) and beta_j and leaves beta_j in sc[1] for the next step.  sc[1]
// is read by the previous kernel only, so the write cannot race.
__global__ void __launch_bounds__(256) k_lanczos_next(int64_t s, int j, const double *w, double *vnext, double *sc,
                                                      double *alpha, double *beta, const double *bpart, int rb,
                                                      const double *aval) {
  __shared__ double bt;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double wi = (i < s && vnext) ? w[i] : 0.0;   // loaded while the norm is folded
  fold_waves(bpart, rb, 1, [&](int, double x) { bt = sqrt(x); });
  __syncthreads();
  const double b = bt;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    alpha[j] = aval ? *aval : sc[0];
    beta[j] = b;
    sc[1] = b;
  }
  if (i >= s || !vnext) return;
  vnext[i] = b > 0.0 ? wi / b : 0.0;
}

void launch_lanczos_next(int64_t s, int32_t j, const double *w, double *vnext, double *sc, double *alpha,
                         double *beta, const double *bpart, int32_t rb, const double *aval, hipStream_t st) {
  hipLaunchKernelGGL(k_lanczos_next, dim3((unsigned)((s + 255) / 256)), dim3(256), 0, st, s, j, w, vnext, sc, alpha,
                     beta, bpart, rb, aval);
}

// k_lanczos_next with the next step's first interface sweep fused: thread
// t also computes slot t of the two-level backward sweep y = L^{-T} v_{j+1}
// (out of place into tout) from w / beta_j at the slot's row and its
// dependencies, which are the stored v_{j+1} values, with the operations of
// k_sweep2 in its order, so tout equals that sweep of v_{j+1} bit for bit.
// The sweep row's loads (and those of its first LN_U dependencies) go out
// before beta_j is folded.  nw2: entries of the sweep's weight arrays.
constexpr int LN_U = 8;

template <typename TS>
__global__ void __launch_bounds__(256) k_lanczos_next_sweep(int64_t s, int j, const double *w, double *vnext,
                                                            double *sc, double *alpha, double *beta,
                                                            const double *bpart, int rb, const double *aval,
                                                            SweepArrays<TS> S, int64_t nw2, double *tout) {
  __shared__ double bt;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t ic = i < s ? i : s - 1;   // threads past the end load slot s - 1 and store nothing
  // wave 0 issues the fold's first 512 loads before the sweep row's chain
  // of loads, and adds them (in lane_fold's order) after it
  const int lane = threadIdx.x & 63;
  double fp[8];
  if (threadIdx.x < 64)
#pragma unroll
    for (int u = 0; u < 8; ++u) fp[u] = bpart[min(lane + u * 64, rb - 1)];
  const double wi = w[ic];
  const int row = S.rows[ic];
  const int e0 = S.rp[ic], e1 = S.rp[ic + 1];
  const double scv = cvt<double>(S.sc[ic]);
  const double wr = w[row];
  double wv[LN_U], xv[LN_U];
  if (nw2 > 0) {
    // padding repeats a valid entry of the array and is not used
    const int last = e1 > e0 ? e1 - 1 : (e0 > 0 ? e0 - 1 : 0);
#pragma unroll
    for (int u = 0; u < LN_U; ++u) {
      const int ee = min(e0 + u, last);
      wv[u] = cvt<double>(S.w2[ee]);
      xv[u] = w[S.ci[ee]];
    }
  }
  if (threadIdx.x < 64) {
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (lane + u * 64 < rb) v += fp[u];
    for (int b = lane + 512; b < rb; b += 64) v += bpart[b];
    v = wave_sum(v);
    if (lane == 0) bt = sqrt(v);
  }
  __syncthreads();
  const double b = bt;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    alpha[j] = aval ? *aval : sc[0];
    beta[j] = b;
    sc[1] = b;
  }
  if (i >= s) return;
  vnext[i] = b > 0.0 ? wi / b : 0.0;
  auto vs = [&](double x) { return b > 0.0 ? x / b : 0.0; };
  double acc = scv * vs(wr);
#pragma unroll
  for (int u = 0; u < LN_U; ++u)
    if (e0 + u < e1) acc -= wv[u] * vs(xv[u]);
  for (int e = e0 + LN_U; e < e1; ++e) acc -= cvt<double>(S.w2[e]) * vs(w[S.ci[e]]);
  tout[row] = acc;
}

template <typename TS>
void launch_lanczos_next_sweep(int64_t s, int32_t j, const double *w, double *vnext, double *sc, double *alpha,
                               double *beta, const double *bpart, int32_t rb, const double *aval,
                               const SweepArrays<TS> &S, int64_t nw2, double *tout, hipStream_t st) {
  hipLaunchKernelGGL((k_lanczos_next_sweep<TS>), dim3((unsigned)((s + 255) / 256)), dim3(256), 0, st, s, j, w, vnext,
                     sc, alpha, beta, bpart, rb, aval, S, nw2, tout);
}
template void launch_lanczos_next_sweep<double>(int64_t, int32_t, const double *, double *, double *, double *,
                                                double *, const double *, int32_t, const double *,
                                                const SweepArrays<double> &, int64_t, double *, hipStream_t);
template void launch_lanczos_next_sweep<float>(int64_t, int32_t, const double *, double *, double *, double *,
                                               double *, const double *, int32_t, const double *,
                                               const SweepArrays<float> &, int64_t, double *, hipStream_t);

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
  x[i] += dot_rows32(V, ldv, i, ys, J);
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
// K8: eigenpairs of the Lanczos tridiagonal T_m (m <= 1024), one workgroup.
//  (1) all eigenvalues by bisection on Sturm counts (one thread each);
//  (2) eigenvectors of the K largest by inverse iteration (one thread each,
//      tridiagonal LU with partial pivoting of T - lambda I, tiny pivots
//      replaced by eps ||T||), factors in interleaved global scratch;
//  (3) two rounds of: orthonormalise the K vectors (classical Gram-Schmidt
//      twice, in order of decreasing eigenvalue), then one more inverse-
//      iteration step; a final orthonormalisation.  Near-multiple
//      eigenvalues give nearly parallel first iterates; the rounds rotate
//      them back into the invariant subspace.
// Outputs: eval (descending, all m), Y (m x K column-major), info (0).
// scratch: 6 m K doubles.
// ---------------------------------------------------------------------------
constexpr int EIG_THREADS = 256;

// Sturm counts (eigenvalues of T below x) at NPT points at once, from the
// LDL^T pivots of T - x I: d_i = (a_i - x) - b_{i-1}^2 / d_{i-1}, a pivot
// smaller than pivmin replaced by -pivmin.  The quotient uses the hardware
// reciprocal refined by one Newton step (relative error of a few ulp,
// which keeps each pivot backward stable); the NPT chains interleave.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  const double e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

template <int NPT>
__device__ __forceinline__ void sturm_n(const double *a, const double *b2, int m, const double (&x)[NPT],
                                        double pivmin, int (&c)[NPT]) {
  double d[NPT];
#pragma unroll
  for (int q = 0; q < NPT; ++q) {
    d[q] = a[0] - x[q];
    if (fabs(d[q]) < pivmin) d[q] = -pivmin;
    c[q] = d[q] < 0.0;
  }
  // a[i] and b2[i-1] are read one step ahead of their use
  double an = a[min(1, m - 1)], bn = b2[0];
  for (int i = 1; i < m; ++i) {
    const double ai = an, bi = bn;
    an = a[min(i + 1, m - 1)];
    bn = b2[i];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      d[q] = fma(-bi, recip(d[q]), ai - x[q]);
      if (fabs(d[q]) < pivmin) d[q] = -pivmin;
      c[q] += d[q] < 0.0;
    }
  }
}

// One inverse-iteration solve (T - lam I) x <- x for column t of the
// row-major m x K block X (entry i at X[i*K + t]): Gaussian elimination of
// the tridiagonal with partial pivoting, the right-hand side eliminated
// along the way; the current pivot row lives in registers and the finished
// rows of U (diagonal, first and second superdiagonal, pivots below `tiny`
// moved to +-tiny) go to F (3 per row, stride K).  Memory operands are read
// one step ahead of the recurrence; quotients use the refined reciprocal.
__device__ void inv_iter(const double *a, const double *b, int m, double lam, double tiny, double *X, double *F,
                         int K, int t) {
  double d = a[0] - lam;
  double u = m > 1 ? b[0] : 0.0;
  double xi = X[t];
  double xnext = X[min(1, m - 1) * K + t];
  auto guard = [&](double v) { return fabs(v) < tiny ? (v < 0.0 ? -tiny : tiny) : v; };
  for (int i = 0; i + 1 < m; ++i) {
    const double l = b[i];
    double dn = a[i + 1] - lam;
    double un = i + 2 < m ? b[i + 1] : 0.0;
    double xn = xnext;
    xnext = X[min(i + 2, m - 1) * K + t];
    double r0, r1, r2, xo;
    if (fabs(d) >= fabs(l)) {
      const double f = d != 0.0 ? l * recip(d) : 0.0;
      r0 = d;
      r1 = u;
      r2 = 0.0;
      dn -= f * u;
      xn -= f * xi;
      xo = xi;
    } else {
      const double f = d * recip(l);
      r0 = l;
      r1 = dn;
      r2 = un;
      dn = u - f * dn;
      un = -f * un;
      xo = xn;
      xn = xi - f * xn;
    }
    F[(3 * i) * K + t] = guard(r0);
    F[(3 * i + 1) * K + t] = r1;
    F[(3 * i + 2) * K + t] = r2;
    X[i * K + t] = xo;
    d = dn;
    u = un;
    xi = xn;
  }
  // back substitution, last rows first
  double x1 = xi * recip(guard(d));
  X[(m - 1) * K + t] = x1;
  double x2 = 0.0;
  if (m < 2) return;
  int i = m - 2;
  double xv = X[i * K + t], f0 = F[(3 * i) * K + t], f1 = F[(3 * i + 1) * K + t], f2 = F[(3 * i + 2) * K + t];
  for (; i >= 0; --i) {
    const double cx = xv, c0 = f0, c1 = f1, c2 = f2;
    const int ip = max(i - 1, 0);
    xv = X[ip * K + t];
    f0 = F[(3 * ip) * K + t];
    f1 = F[(3 * ip + 1) * K + t];
    f2 = F[(3 * ip + 2) * K + t];
    const double v = (cx - c1 * x1 - c2 * x2) * recip(c0);
    X[i * K + t] = v;
    x2 = x1;
    x1 = v;
  }
}

// scale column t of X (stride K) to unit norm
__device__ void unit_col(double *x, int m, int K, int t) {
  double nr = 0.0;
  for (int i = 0; i < m; ++i) nr += x[i * K + t] * x[i * K + t];
  const double sc = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
  for (int i = 0; i < m; ++i) x[i * K + t] *= sc;
}

// classical Gram-Schmidt twice over the K columns of X (stride K), in
// column order; the whole workgroup cooperates (one wave per dot product).
// h: K + 1 doubles of LDS.
__device__ void cgs2_cols(double *x, int m, int K, double *h) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = 0; j < K; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = wid; i < j; i += nw) {
        double v = 0.0;
        for (int r = lane; r < m; r += 64) v += x[r * K + i] * x[r * K + j];
        v = wave_sum(v);
        if (lane == 0) h[i] = v;
      }
      __syncthreads();
      for (int r = threadIdx.x; r < m; r += blockDim.x) {
        double v = x[r * K + j];
        for (int i = 0; i < j; ++i) v -= h[i] * x[r * K + i];
        x[r * K + j] = v;
      }
      __syncthreads();
    }
    // normalise column j
    double v = 0.0;
    if (wid == 0) {
      for (int r = lane; r < m; r += 64) v += x[r * K + j] * x[r * K + j];
      v = wave_sum(v);
      if (lane == 0) h[K] = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    }
    __syncthreads();
    const double sc = h[K];
    for (int r = threadIdx.x; r < m; r += blockDim.x) x[r * K + j] *= sc;
    __syncthreads();
  }
}

// ortho_cols' Cholesky (LDS, all threads) and its triangular solve with a
// row of W in registers for K <= 64 (loops unrolled to 32 or 64 entries,
// columns past K idle).

// All threads: G (row-major K x K Gram matrix) = R^T R, right-looking in
// LDS.  Step j takes the pivot (the updated G[j][j]), writes row j of R over
// row j of G (R[j][l] = h_l / sqrt(pivot), h_l the updated entry, as the
// left-looking form) and subtracts R[j][q] R[j][l] from every entry (q, l)
// with j < q <= l, so each entry receives its updates in ascending j.  dg (K
// doubles) keeps the Gram diagonal for the pivot test; a pivot at or below
// 1e-8 of it sets *flag.
__device__ __forceinline__ void chol_lds(double *G, int K, double *dg, int *flag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int l = tid; l < K; l += nt) dg[l] = G[l * K + l];
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    const double piv = G[j * K + j];
    if (!(piv > 1e-8 * dg[j]) || !(piv > 0.0)) {
      if (tid == 0) *flag = 1;
      return;   // every thread takes the same exit
    }
    const double rs = 1.0 / sqrt(piv);
    __syncthreads();
    for (int l = j + tid; l < K; l += nt) G[j * K + l] = G[j * K + l] * rs;
    __syncthreads();
    // trailing block: columns by lane in a group of 32, rows by group, four
    // rows' operands loaded before their updates are stored
    const int rstep = nt >> 5;
    for (int l = j + 1 + (tid & 31); l < K; l += 32) {
      const double rl = G[j * K + l];
      for (int q0 = j + 1 + (tid >> 5); q0 <= l; q0 += 4 * rstep) {
        double rq[4], g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = min(q0 + u * rstep, l);
          rq[u] = G[j * K + q];
          g[u] = G[q * K + l];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q0 + u * rstep <= l) G[(q0 + u * rstep) * K + l] = g[u] - rq[u] * rl;
      }
    }
    __syncthreads();
  }
}

// One row w of W (K entries): w <- w R^{-1} by forward substitution in
// column order, R (upper triangle of G) read by broadcast.
template <int KR>
__device__ __forceinline__ void solve_row_regs(double *w, const double *G, int K) {
  double x[KR];
#pragma unroll
  for (int q = 0; q < KR; ++q) x[q] = q < K ? w[q] : 0.0;
#pragma unroll
  for (int j = 0; j < KR; ++j)
    if (j < K) {
      double v = x[j];
#pragma unroll
      for (int q = 0; q < j; ++q) v -= x[q] * G[q * K + j];
      x[j] = v / G[j * K + j];
    }
#pragma unroll
  for (int q = 0; q < KR; ++q)
    if (q < K) w[q] = x[q];
}

// Gram matrix G = W^T W of a row-major m x K block in global memory (K <=
// 64), upper triangle by pairs and mirrored, as the direct loop of
// ortho_cols: the rows go through LDS (S: GR_ROWS x K doubles) in chunks,
// and every pair keeps its four partial sums over the same rows in the same
// order (rows 4g + u into sum u, the rows past the last whole group into
// sum 0), so G is bit for bit the direct loop's.
constexpr int GR_ROWS = 64;
constexpr int GR_PMAX = (64 * 65 / 2 + EIG_THREADS - 1) / EIG_THREADS;
__device__ __forceinline__ void gram_staged(const double *W, int m, int K, double *G, double *S) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int npair = K * (K + 1) / 2;
  int pi[GR_PMAX], pj[GR_PMAX];
  double acc[GR_PMAX][4];
#pragma unroll
  for (int q = 0; q < GR_PMAX; ++q) {
    int i = 0, rem = min(tid + q * nt, npair - 1);
    while (rem >= K - i) {
      rem -= K - i;
      ++i;
    }
    pi[q] = i;
    pj[q] = i + rem;
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[q][u] = 0.0;
  }
  for (int r0 = 0; r0 < m; r0 += GR_ROWS) {
    const int nr = min(GR_ROWS, m - r0);
    __syncthreads();
    for (int e = tid; e < nr * K; e += nt) S[e] = W[(int64_t)r0 * K + e];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GR_PMAX; ++q)
      if (tid + q * nt < npair) {
        const int i = pi[q], j = pj[q];
        int rr = 0;
        for (; rr + 3 < nr; rr += 4) {
          acc[q][0] += S[rr * K + i] * S[rr * K + j];
          acc[q][1] += S[(rr + 1) * K + i] * S[(rr + 1) * K + j];
          acc[q][2] += S[(rr + 2) * K + i] * S[(rr + 2) * K + j];
          acc[q][3] += S[(rr + 3) * K + i] * S[(rr + 3) * K + j];
        }
        for (; rr < nr; ++rr) acc[q][0] += S[rr * K + i] * S[rr * K + j];
      }
  }
#pragma unroll
  for (int q = 0; q < GR_PMAX; ++q)
    if (tid + q * nt < npair) {
      const double v = (acc[q][0] + acc[q][1]) + (acc[q][2] + acc[q][3]);
      G[pi[q] * K + pj[q]] = v;
      G[pj[q] * K + pi[q]] = v;
    }
}

// Orthonormalise the K columns of the row-major m x K block W in column
// order by Cholesky QR, twice: G = W^T W, G = R^T R (R upper triangular),
// W <- W R^{-1}.  In exact arithmetic this is the Gram-Schmidt result; the
// second pass restores orthogonality to working accuracy.  A column that
// is (nearly) in the span of the earlier ones (Cholesky pivot below 1e-8 of
// the column's squared norm) sends the block to Gram-Schmidt twice instead.
// G: K*K doubles of LDS, h: K + 1, flag: one int of LDS.
template <bool WIDE>
__device__ __forceinline__ void ortho_cols(double *W, int m, int K, double *G, double *h, int *flag,
                                           double *S = nullptr) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int pass = 0; pass < 2; ++pass) {
    if (tid == 0) *flag = 0;
    // Gram matrix, upper triangle by pairs (i <= j), mirrored (W in global
    // memory with K <= 64: rows staged through S)
    const int npair = K * (K + 1) / 2;
    if (WIDE && S && K <= 64) gram_staged(W, m, K, G, S);
    for (int p = tid; p < npair && !(WIDE && S && K <= 64); p += nt) {
      int i = 0, rem = p;
      while (rem >= K - i) {
        rem -= K - i;
        ++i;
      }
      const int j = i + rem;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int r = 0;
      for (; r + 3 < m; r += 4) {
        s0 += W[r * K + i] * W[r * K + j];
        s1 += W[(r + 1) * K + i] * W[(r + 1) * K + j];
        s2 += W[(r + 2) * K + i] * W[(r + 2) * K + j];
        s3 += W[(r + 3) * K + i] * W[(r + 3) * K + j];
      }
      for (; r < m; ++r) s0 += W[r * K + i] * W[r * K + j];
      const double v = (s0 + s1) + (s2 + s3);
      G[i * K + j] = v;
      G[j * K + i] = v;
    }
    __syncthreads();
    // Cholesky G = R^T R, R in the upper triangle (row-major)
    chol_lds(G, K, h, flag);
    __syncthreads();
    if (*flag) break;
    // W <- W R^{-1}, one row per thread, by forward substitution in column
    // order (the row in registers when K <= 32, or K <= 64 with WIDE)
    if (K <= 32) {
      for (int r = tid; r < m; r += nt) solve_row_regs<32>(W + (int64_t)r * K, G, K);
    } else if (WIDE && K <= 64) {
      for (int r = tid; r < m; r += nt) solve_row_regs<64>(W + (int64_t)r * K, G, K);
    } else {
      for (int r = tid; r < m; r += nt) {
        for (int j = 0; j < K; ++j) {
          double v = W[r * K + j];
          for (int q = 0; q < j; ++q) v -= W[r * K + q] * G[q * K + j];
          W[r * K + j] = v / G[j * K + j];
        }
      }
    }
    __syncthreads();
  }
  if (*flag) cgs2_cols(W, m, K, h);
}

// Eigenvalues and the K leading eigenvectors of the symmetric tridiagonal
// T (diagonal alpha, off-diagonal beta), in three kernels:
//   k_eig_bisect  one wave per eigenvalue (the t-th largest, descending
//                 output): multisection, each lane evaluates the Sturm count
//                 at one of 64 interior points, so the bracket shrinks
//                 65-fold per step, down to a width of 2 ulp;
//   k_eig_invit   one wave per wanted eigenvector: inverse iteration from a
//                 fixed pseudo-random start (or the current vector), the
//                 factorisation and the vector in LDS, unit norm after each
//                 solve;
//   k_eig_ortho   one workgroup: orthonormalisation of the m x K block in
//                 column order (ortho_cols), to X or, at the end, to Y.
// Sequence: bisect; invit x3; ortho; invit x1; ortho.
__device__ __forceinline__ void gershgorin(const double *a, const double *b, int m, double &glo, double &ghi) {
  const int lane = threadIdx.x & 63;
  double lo = 1e300, hi = -1e300;
  for (int i = lane; i < m; i += 64) {
    const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - r);
    hi = fmax(hi, a[i] + r);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
  }
  glo = lo;
  ghi = hi;
}

__global__ void __launch_bounds__(64) k_eig_bisect(int m, const double *alpha, const double *beta, double *eval) {
  extern __shared__ double eig_lds[];
  double *a = eig_lds, *b = a + m, *b2 = b + m;
  const int lane = threadIdx.x, t = blockIdx.x;
  for (int i = lane; i < m; i += 64) {
    a[i] = alpha[i];
    b[i] = (i + 1 < m) ? beta[i] : 0.0;
    b2[i] = b[i] * b[i];
  }
  __syncthreads();
  double glo, ghi;
  gershgorin(a, b, m, glo, ghi);
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  const double eps = 2.220446049250313e-16;
  const double pivmin = 1e-290 + eps * eps * tnorm * tnorm;
  const int want = m - t;   // the t-th largest is the (m - t)-th smallest
  double lo = glo - eps * tnorm - 1e-300, hi = ghi + eps * tnorm + 1e-300;
  for (int it = 0; it < 100; ++it) {
    const double w = hi - lo;
    if (!(w > 2.0 * eps * (fabs(lo) + fabs(hi)))) break;
    double x[1];
    int c[1];
    x[0] = lo + w * (double)(lane + 1) / 65.0;
    sturm_n<1>(a, b2, m, x, pivmin, c);
    // new bracket: the largest point with fewer than `want` eigenvalues
    // below it, and the smallest point with at least `want`
    double nlo = c[0] < want ? x[0] : lo;
    double nhi = c[0] >= want ? x[0] : hi;
    for (int o = 32; o > 0; o >>= 1) {
      nlo = fmax(nlo, __shfl_xor(nlo, o, 64));
      nhi = fmin(nhi, __shfl_xor(nhi, o, 64));
    }
    if (!(nlo > lo || nhi < hi) || !(nlo < nhi)) break;   // no representable progress
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) eval[t] = 0.5 * (lo + hi);
}

// X: row-major m x K (column q at X[i*K + q]); eval descending
__global__ void __launch_bounds__(64) k_eig_invit(int m, const double *alpha, const double *beta,
                                                 const double *eval, double *X, int K, int iters, int init) {
  extern __shared__ double eig_lds[];
  double *a = eig_lds, *b = a + m, *x = b + m, *F = x + m;
  const int lane = threadIdx.x, q = blockIdx.x;
  for (int i = lane; i < m; i += 64) {
    a[i] = alpha[i];
    b[i] = (i + 1 < m) ? beta[i] : 0.0;
    if (init) {
      uint32_t z = (uint32_t)(i * 2654435761u) ^ (uint32_t)((q + 1) * 40503u);
      z ^= z >> 15;
      z *= 2246822519u;
      z ^= z >> 13;
      x[i] = 0.5 + (double)(z & 0xFFFF) / 65536.0;
    } else {
      x[i] = X[(size_t)i * K + q];
    }
  }
  __syncthreads();
  double glo, ghi;
  gershgorin(a, b, m, glo, ghi);
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  const double tiny = 2.220446049250313e-16 * tnorm + 1e-300;
  const double lam = eval[q];
  for (int rep = 0; rep < iters; ++rep) {
    if (lane == 0) inv_iter(a, b, m, lam, tiny, x, F, 1, 0);
    __syncthreads();
    double nr = 0.0;
    for (int i = lane; i < m; i += 64) nr += x[i] * x[i];
    nr = wave_allsum(nr);
    const double sc = nr > 0.0 ? 1.0 / sqrt(nr) : 0.0;
    for (int i = lane; i < m; i += 64) x[i] *= sc;
    __syncthreads();
  }
  for (int i = lane; i < m; i += 64) X[(size_t)i * K + q] = x[i];
}

// orthonormalise X (row-major m x K); final: write Y (column-major m x K)
__global__ void __launch_bounds__(EIG_THREADS) k_eig_ortho(int m, int K, double *X, double *Y, int xs_lds, int final_,
                                                          int *info) {
  extern __shared__ double eig_lds[];
  double *h = eig_lds, *G = h + (K + 1), *xl = G + (size_t)K * K;
  __shared__ int flag;
  const int tid = threadIdx.x, nt = blockDim.x;
  if (xs_lds) {
    // eight loads per thread in flight
    const int mk = m * K;
    for (int i0 = tid; i0 < mk; i0 += 8 * nt) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = X[min(i0 + u * nt, mk - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u * nt < mk) xl[i0 + u * nt] = t[u];
    }
    __syncthreads();
  }
  // W in LDS: its own inlined copy, which addresses W as LDS
  double *W = xs_lds ? xl : X;
  if (xs_lds) {
    ortho_cols<false>(xl, m, K, G, h, &flag);
  } else {
    // W through an opaque generic pointer: with flat accesses the compiler
    // schedules the 64-wide row solve without spilling registers
    double *Xg = X;
    asm volatile("" : "+s"(Xg));
    ortho_cols<true>(Xg, m, K, G, h, &flag, K <= 64 ? xl : nullptr);
  }
  if (final_) {
    for (int i = tid; i < m * K; i += nt) {
      const int r = i / K, q = i - r * K;
      Y[r + (int64_t)q * m] = W[i];
    }
    if (tid == 0) *info = 0;
  } else if (xs_lds) {
    for (int i = tid; i < m * K; i += nt) X[i] = xl[i];
  }
}

void launch_tridiag_eig(int32_t m, const double *alpha, const double *beta, double *scratch, double *eval,
                        double *Y, int32_t K, int *info, hipStream_t st) {
  if (m <= 0) return;
  hipLaunchKernelGGL(k_eig_bisect, dim3(m), dim3(64), sizeof(double) * 3 * m, st, m, alpha, beta, eval);
  if (K <= 0) {
    hipLaunchKernelGGL(k_eig_ortho, dim3(1), dim3(EIG_THREADS), sizeof(double) * 2, st, m, 0, scratch, Y, 0, 1,
                       info);
    return;
  }
  const size_t inv_lds = sizeof(double) * 6 * (size_t)m;
  static size_t inv_attr = 0, ort_attr = 0;
  if (inv_lds > 65536 && inv_lds > inv_attr) {
    (void)hipFuncSetAttribute((const void *)k_eig_invit, hipFuncAttributeMaxDynamicSharedMemorySize, (int)inv_lds);
    inv_attr = inv_lds;
  }
  const size_t base = sizeof(double) * (K + 1 + (size_t)K * K);
  const size_t xb = sizeof(double) * (size_t)m * K;
  const int xs_lds = base + xb <= 128 * 1024 ? 1 : 0;
  // block in global memory: K <= 64 stages rows for the Gram matrix
  const size_t gb = K <= 64 ? sizeof(double) * GR_ROWS * (size_t)K : 0;
  const size_t ort_lds = base + (xs_lds ? xb : gb);
  if (ort_lds > 65536 && ort_lds > ort_attr) {
    (void)hipFuncSetAttribute((const void *)k_eig_ortho, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ort_lds);
    ort_attr = ort_lds;
  }
  double *X = scratch;
  hipLaunchKernelGGL(k_eig_invit, dim3(K), dim3(64), inv_lds, st, m, alpha, beta, eval, X, K, 3, 1);
  hipLaunchKernelGGL(k_eig_ortho, dim3(1), dim3(EIG_THREADS), ort_lds, st, m, K, X, Y, xs_lds, 0, info);
  hipLaunchKernelGGL(k_eig_invit, dim3(K), dim3(64), inv_lds, st, m, alpha, beta, eval, X, K, 1, 0);
  hipLaunchKernelGGL(k_eig_ortho, dim3(1), dim3(EIG_THREADS), ort_lds, st, m, K, X, Y, xs_lds, 1, info);
}

// Ritz vectors: U64[i, q] = sum_j V[i, j] Y[j, q]  (V: s x m col-major,
// Y: m x K col-major, U64 column-major s x k, k <= K).  Also writes the
// storage copy U (column-major, rounded to TU).
// U = V Y (s x k), RT rows per thread (rows i + r * blockDim.x of the
// block's run), QT columns of Y per pass staged in LDS: every Y entry read
// from LDS serves RT rows.  A row's V loads go out eight at a time, a group
// ahead of their use, and each output sums over j in ascending order
// whatever QT and RT.
template <typename TU, int QT, int RT>
__global__ void __launch_bounds__(256) k_ritz(int64_t s, int m, int k, const double *V, int64_t ldv,
                                              const double *Y, double *U64, TU *U) {
  extern __shared__ __align__(16) double ys[];  // m x QT tile
  int64_t ir[RT], ic[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    ir[r] = (int64_t)blockIdx.x * blockDim.x * RT + (int64_t)r * blockDim.x + threadIdx.x;
    ic[r] = ir[r] < s ? ir[r] : s - 1;   // rows past the end load row s - 1 and store nothing
  }
  for (int q0 = 0; q0 < k; q0 += QT) {
    const int nq = min(QT, k - q0);
    __syncthreads();
    for (int t = threadIdx.x; t < m * QT; t += blockDim.x) {
      const int q = t / m, j = t - q * m;
      ys[j * QT + q] = q < nq ? Y[j + (int64_t)(q0 + q) * m] : 0.0;
    }
    __syncthreads();
    double acc[RT][QT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int q = 0; q < QT; ++q) acc[r][q] = 0.0;
    double vn[RT][8];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int u = 0; u < 8; ++u) vn[r][u] = V[ic[r] + (int64_t)min(u, m - 1) * ldv];
    for (int j0 = 0; j0 < m; j0 += 8) {
      double vj[RT][8];
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          vj[r][u] = vn[r][u];
          vn[r][u] = V[ic[r] + (int64_t)min(j0 + 8 + u, m - 1) * ldv];
        }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < m) {
          const double2 *yr = reinterpret_cast<const double2 *>(ys + (j0 + u) * QT);
#pragma unroll
          for (int q = 0; q < QT / 2; ++q) {
            const double2 y = yr[q];
#pragma unroll
            for (int r = 0; r < RT; ++r) {
              acc[r][2 * q] += vj[r][u] * y.x;
              acc[r][2 * q + 1] += vj[r][u] * y.y;
            }
          }
        }
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
      if (ir[r] < s)
#pragma unroll
        for (int q = 0; q < QT; ++q)
          if (q < nq) {
            U64[ir[r] + (int64_t)(q0 + q) * s] = acc[r][q];
            U[ir[r] + (int64_t)(q0 + q) * s] = round_store<TU>(acc[r][q]);
          }
  }
}

template <typename TU, int QT, int RT>
void launch_ritz_t(int64_t s, int32_t m, int32_t k, const double *V, int64_t ldv, const double *Y, double *U64,
                   TU *U, hipStream_t st) {
  static size_t attr = 0;
  const size_t lds = sizeof(double) * (size_t)m * QT;
  if (lds > 65536 && lds > attr) {
    (void)hipFuncSetAttribute((const void *)k_ritz<TU, QT, RT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    attr = lds;
  }
  const unsigned nb = (unsigned)((s + 256 * RT - 1) / (256 * RT));
  hipLaunchKernelGGL((k_ritz<TU, QT, RT>), dim3(nb), dim3(256), lds, st, s, m, k, V, ldv, Y, U64, U);
}

template <typename TU>
void launch_ritz(int64_t s, int32_t m, int32_t k, const double *V, int64_t ldv, const double *Y, double *U64,
                 TU *U, hipStream_t st) {
  if (s == 0 || k == 0) return;
  // 32 columns per pass when the tile fits 160 KiB of LDS, else 16 (m <=
  // 1024); two rows per thread when there are rows enough to fill the chip
  const bool wide = (size_t)m * 32 * sizeof(double) <= 160 * 1024;
  const bool two = s >= (int64_t)1 << 19;
  if (wide && two)
    launch_ritz_t<TU, 32, 2>(s, m, k, V, ldv, Y, U64, U, st);
  else if (wide)
    launch_ritz_t<TU, 32, 1>(s, m, k, V, ldv, Y, U64, U, st);
  else if (two)
    launch_ritz_t<TU, 16, 2>(s, m, k, V, ldv, Y, U64, U, st);
  else
    launch_ritz_t<TU, 16, 1>(s, m, k, V, ldv, Y, U64, U, st);
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
// Numeric refactorisation (same pattern, new values), Sec. 5.2 local solvers
// restricted to no fill: IC(0) / ILDL^T(0) level by level, then the stored
// sweep coefficients rewritten in place.
// ---------------------------------------------------------------------------
__global__ void k_gather(int64_t n, const int64_t *src, const double *val, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = val[src[i]];
}

__global__ void k_mirror_check(int64_t n, const int64_t *tr, const double *val, int *flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && val[tr[i]] != val[i]) *flag = 1;
}

void launch_mirror_check(int64_t n, const int64_t *tr, const double *val, int *flag, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mirror_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, tr, val, flag);
}

void launch_gather(int64_t n, const int64_t *src, const double *val, double *out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, src, val, out);
}

// One thread per row of the level.  Row i, entries e (ascending columns j,
// diagonal last):
//   IC(0):    l_ij = (a_ij - sum_k l_ik l_jk) / l_jj,  l_ii = sqrt(a_ii - sum_j l_ij^2)
//   ILDL(0):  l_ij = (a_ij - sum_k (l_ik l_jk) d_k) / d_j,  d_i = a_ii - sum_j (l_ij l_ij) d_j
// with k over the columns that rows i and j share (k < j), summed in row
// j's column order: the same operations, in the same order, as the host
// factorisation (whose dense scatter adds exact zeros for the others).
__global__ void k_fact_level(const int64_t *rp, const int32_t *ci, double *V, const int32_t *rows, int32_t r0,
                             int32_t r1, int32_t ldl, int *err) {
#pragma clang fp contract(off)
  const int32_t r = r0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (r >= r1) return;
  const int32_t i = rows[r];
  const int64_t a = rp[i], b = rp[i + 1] - 1;
  if (b < a || ci[b] != i) {
    *err = 1;
    return;
  }
  double acc = 0.0;
  for (int64_t e = a; e < b; ++e) {
    const int32_t j = ci[e];
    const int64_t ja = rp[j], jb = rp[j + 1] - 1;
    double s = 0.0;
    int64_t q = a;
    for (int64_t t = ja; t < jb; ++t) {
      const int32_t k = ci[t];
      while (q < e && ci[q] < k) ++q;
      if (q < e && ci[q] == k) {
        const double prod = V[q] * V[t];
        s += ldl ? prod * V[rp[k + 1] - 1] : prod;
      }
    }
    const double pj = V[jb];
    const double l = (V[e] - s) / pj;
    V[e] = l;
    acc += ldl ? (l * l) * pj : l * l;
  }
  const double piv = V[b] - acc;
  if (ldl) {
    if (!(fabs(piv) >= 1e-300)) *err = 1;
    V[b] = piv;
  } else {
    if (!(piv > 0.0)) *err = 1;
    V[b] = sqrt(piv);
  }
}

void launch_fact_level(const int64_t *rp, const int32_t *ci, double *V, const int32_t *rows, int32_t r0, int32_t r1,
                       int32_t ldl, int *err, hipStream_t st) {
  if (r1 <= r0) return;
  hipLaunchKernelGGL(k_fact_level, dim3((unsigned)((r1 - r0 + 255) / 256)), dim3(256), 0, st, rp, ci, V, rows, r0,
                     r1, ldl, err);
}

template <typename TS>
__global__ void k_rf_pack(int64_t nmap, const RfMap *map, const double *V, const double *val, uint8_t *base) {
#pragma clang fp contract(off)
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nmap) return;
  const RfMap m = map[t];
  auto rd = [](double x) { return (double)(TS)x; };
  double v = 0.0;
  switch (m.op) {
    case RF_SRC: v = val[m.a]; break;
    case RF_ONE: v = 1.0; break;
    case RF_RAW: v = rd(V[m.a]); break;
    case RF_RECIP: v = rd(1.0 / rd(V[m.a])); break;
    case RF_DIV: v = rd(rd(V[m.a]) / rd(V[m.b])); break;
    case RF_W2: v = rd(rd(rd(V[m.a]) / rd(V[m.b])) * rd(1.0 / rd(V[m.c]))); break;
    default: break;
  }
  *reinterpret_cast<TS *>(base + m.off) = (TS)v;
}

template <typename TS>
void launch_rf_pack(int64_t nmap, const RfMap *map, const double *V, const double *val, void *base,
                    hipStream_t st) {
  if (nmap <= 0) return;
  hipLaunchKernelGGL((k_rf_pack<TS>), dim3((unsigned)((nmap + 255) / 256)), dim3(256), 0, st, nmap, map, V, val,
                     (uint8_t *)base);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------
template int64_t lr_rm_groups<double>(int64_t, int32_t, int32_t &);
template int64_t lr_rm_groups<float>(int64_t, int32_t, int32_t &);
template void launch_lr_to_rm<double>(const double *, int64_t, int32_t, double *, hipStream_t);
template void launch_lr_to_rm<float>(const double *, int64_t, int32_t, float *, hipStream_t);
template void launch_lowrank_rm<double>(const double *, const double *, int64_t, int32_t, const double *, double,
                                        const double *, int64_t, double *, int64_t, int32_t, double *, int32_t,
                                        double *, hipStream_t);
template void launch_lowrank_rm<float>(const float *, const float *, int64_t, int32_t, const double *, double,
                                       const double *, int64_t, double *, int64_t, int32_t, double *, int32_t,
                                       double *, hipStream_t);
template void launch_rf_pack<double>(int64_t, const RfMap *, const double *, const double *, void *, hipStream_t);
template void launch_rf_pack<float>(int64_t, const RfMap *, const double *, const double *, void *, hipStream_t);
template void launch_bsolve<double, double>(const BlockArrays<double> &, int32_t, const BArgs &, int32_t, size_t,
                                            hipStream_t);
template void launch_bsolve<float, float>(const BlockArrays<float> &, int32_t, const BArgs &, int32_t, size_t,
                                          hipStream_t);
template void launch_bsolve<float, double>(const BlockArrays<float> &, int32_t, const BArgs &, int32_t, size_t,
                                           hipStream_t);
template void launch_sweep2<double, double>(const SweepArrays<double> &, int32_t, const double *, int64_t, double *,
                                            int64_t, int32_t, hipStream_t, const double *, double *);
template void launch_sweep2<float, float>(const SweepArrays<float> &, int32_t, const double *, int64_t, double *,
                                          int64_t, int32_t, hipStream_t, const double *, double *);
template void launch_sweep2<float, double>(const SweepArrays<float> &, int32_t, const double *, int64_t, double *,
                                           int64_t, int32_t, hipStream_t, const double *, double *);
template void launch_sweep<double, double>(const SweepArrays<double> &, const int32_t *, int32_t, int32_t, double *,
                                           int64_t, int32_t, bool, hipStream_t, int32_t);
template void launch_sweep<float, float>(const SweepArrays<float> &, const int32_t *, int32_t, int32_t, double *,
                                         int64_t, int32_t, bool, hipStream_t, int32_t);
template void launch_sweep<float, double>(const SweepArrays<float> &, const int32_t *, int32_t, int32_t, double *,
                                          int64_t, int32_t, bool, hipStream_t, int32_t);
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

// alpha_j = the first Gram-Schmidt pass's coefficient on v_j
__global__ void k_lanczos_alpha(int j, const double *h, double *sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc[0] = h[j];
}

void launch_lanczos_alpha(int32_t j, const double *h, double *sc, hipStream_t st) {
  hipLaunchKernelGGL(k_lanczos_alpha, dim3(1), dim3(64), 0, st, j, h, sc);
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

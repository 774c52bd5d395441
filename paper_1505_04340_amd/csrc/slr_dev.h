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
//
// Each sweep of each subdomain is packed as a level-sliced byte stream
// (built on the host, 16-byte aligned segments); lvb[l] is the byte offset
// of level l's segment (lvb[nlev] = total bytes).  For level l with L rows:
//
// Fixed width K (every row of every sweep padded to the problem's widest
// row K <= 4; padding has w = 0 and points at the row itself; levels wider
// than 64 * rec_passes(K) rows split), row records of KR = rec_width(K)
// entries:
//     idx   int32[L][KR]       [row, c_0, .., c_{K-1}, pad]  local indices
//     wts   TS[L][KR]          [sc, w_0, .., w_{K-1}, pad]   scale, weights
// Any width, ELL form, K = the widest row of the level (levels are cut into
// pieces of at most kEllLevelBytes on the host):
//     K     int32 (in a 16-byte header)
//     rows  uint16[L]          local row index
//     sc    TS[L]              row scale
//     ci    uint16[K*L]        column of entry e of row j at [e*L + j]
//     w     TS[K*L]            pre-divided weight, same layout
// each ELL section padded to 8 bytes and the segment to 16.  A run of
// consecutive levels of at most a few rows (a near-chain) is packed as ELL
// pieces holding the run's rows with their entries to rows before the run,
// then column segments (header int32 -2, ncol, nnz):
//     crow  uint16[ncol]       the run row finished by column c
//     cptr  uint16[ncol + 1]   its entries [cptr[c], cptr[c+1])
//     tgt   uint16[nnz]        a later run row that uses it
//     w     TS[nnz]            that row's pre-divided weight
// solved column by column (x[tgt] -= w x[crow]).
struct BlockDesc {
  int32_t m0, m;                   // interior range in the internal order
  int32_t f_nlev, f_K, f_lev, f_lvb;   // forward sweep: levels, width, levptr / lvb offsets
  int32_t b_nlev, b_K, b_lev, b_lvb;   // backward sweep
  int64_t f_data, b_data;          // byte offsets of the packed streams
  // E rows (interior rows coupled to the interface), ELL with width e_K:
  //   e_row[e_row + i] local row; e_q / e_val[e_ent + e*e_n + i] (padding: q 0, value 0)
  int32_t e_row, e_n, e_K, e_ent;
  // E^T rows (interface rows owned here), ELL with width t_K:
  //   t_q[t_row + i] interface index; t_j / t_val[t_ent + e*t_n + i] (padding: j 0, value 0)
  int32_t t_row, t_n, t_K, t_ent;
};

// Interface sweeps (C): level-scheduled CSR on the device, see slr_host.h.
// rp entries are absolute offsets into ci / w.
template <typename TS>
struct SweepArrays {
  const int32_t *lev = nullptr;    // level pointers
  const int32_t *rows = nullptr;   // level-sorted rows
  const int32_t *rp = nullptr;     // nrows+1 absolute entry offsets
  const int32_t *ci = nullptr;     // column indices
  const TS *w = nullptr;           // pre-scaled off-diagonal weights
  const TS *sc = nullptr;          // per-row scale
  const TS *w2 = nullptr;          // two-level schedules: w * sc of the dependency row
};

template <typename TS>
struct BlockArrays {
  const BlockDesc *desc = nullptr;
  const int32_t *lev = nullptr;    // level pointers of all sweeps
  const int32_t *lvb = nullptr;    // level byte offsets of all sweeps
  const uint8_t *data = nullptr;   // packed sweep streams
  const uint16_t *e_row = nullptr;
  const int32_t *e_q = nullptr;
  const TS *e_val = nullptr;
  const int32_t *t_q = nullptr;
  const uint16_t *t_j = nullptr;
  const TS *t_val = nullptr;
  // LDS position of interior row m0 + r of a block (r local): every local
  // index above (packed streams, E rows, E^T columns) is such a position;
  // null: position = local row in every block
  const uint16_t *xpos = nullptr;
  int32_t max_m = 0;
  int32_t max_lev = 0;
  int32_t max_level_bytes = 0;     // largest single level segment
  int32_t max_K = 0;               // widest packed row over all sweeps
  int32_t pack_K = 0;              // > 0: every packed row has exactly this width
};

// What one launch of the batched B kernel computes for each subdomain i
// and right-hand side column c (columns [0, nrhs)):
//   rhs   = a_f * f_i + b_y * E_i y           (prologue)
//   z     = B_i^{-1} rhs                      (forward + backward sweep in LDS)
//   u_i   = z                                 (if u != nullptr)
//   gout_q = c_g * g_q + d_t * (E^T z)_q      (epilogue, q owned by i; if gout)
// LDS bytes after the B kernel's stage that absorb the prologue's stores
// past the end of x's rows: one 16-byte slot per lane of a wave, so that
// such stores from one instruction never hit the same bank.
constexpr int kStageDummyBytes = 1024;
// ELL level segments: header bytes and the largest piece of a level
constexpr int kEllHeaderBytes = 16;
constexpr int kEllLevelBytes = 8192;

// Entries of a fixed-width row record: the row plus K columns, rounded up to
// a multiple of 4 so that records are whole 16-byte vectors.
__host__ __device__ constexpr int rec_width(int K) { return (K + 1 + 3) & ~3; }

// Row passes per lane the fixed-width sweep kernel unrolls for rows of width
// K (bounded by registers); the host splits wider levels into consecutive
// sub-levels of at most 64 * rec_passes(K) rows (rows of one level are
// independent, so any split of a level is a valid schedule).
__host__ __device__ constexpr int rec_passes(int K) { return K <= 2 ? 4 : (K == 3 ? 3 : 2); }

struct BArgs {
  const double *f = nullptr;  int64_t ldf = 0;  double a_f = 0.0;
  const double *y = nullptr;  int64_t ldy = 0;  double b_y = 0.0;
  const double *g = nullptr;  int64_t ldg = 0;  double c_g = 0.0;
  double *gout = nullptr;     int64_t ldgo = 0; double d_t = 0.0;
  double *u = nullptr;        int64_t ldu = 0;
  int32_t nrhs = 1;
  int32_t R = 1;              // right-hand sides per workgroup
  int32_t stage_bytes = 0;    // LDS staging buffer for the packed sweeps
  int32_t sweeps = 3;         // bit 0: forward sweep, bit 1: backward sweep
  // persistent launch (sched != nullptr): workgroup w takes the work items
  // sched[sched_ptr[w] .. sched_ptr[w+1]), each (column group << 16) |
  // subdomain, in that order; otherwise blockIdx.x is the subdomain and
  // blockIdx.y the column group
  const int32_t *sched = nullptr;
  const int32_t *sched_ptr = nullptr;
  // persistent with per-subdomain column counts: items are subdomain |
  // (first column << 16) | (columns << 24), each subdomain's x stored with
  // its own row count as stride, as many columns as the x region holds
  int32_t var_cols = 0;
};

// Numeric refactorisation on the device: one stored coefficient (TS) at
// byte offset `off` of its array, computed from factor values V (rounded to
// TS first when TS is FP32) or from the input matrix values:
//   RF_SRC    val[a]                     (E, E^T entries)
//   RF_ONE    1
//   RF_RAW    V[a]                        (unit-L weights of L D L^T)
//   RF_RECIP  rd(1 / V[a])                (row scales)
//   RF_DIV    rd(V[a] / V[b])             (pre-divided weights)
//   RF_W2     rd(rd(V[a] / V[b]) * rd(1 / V[c]))   (two-level interface weights)
// rd() rounds to TS, exactly as the host packing does.
enum { RF_SRC = 0, RF_ONE, RF_RAW, RF_RECIP, RF_DIV, RF_W2 };
struct RfMap {
  int64_t off;
  int32_t a, b, c, op;
};

template <typename TS>
void launch_rf_pack(int64_t nmap, const RfMap *map, const double *V, const double *val, void *base,
                    hipStream_t st);
// *flag = 1 if some val[e] != val[tr[e]] (tr: the mirror entry of each entry)
void launch_mirror_check(int64_t n, const int64_t *tr, const double *val, int *flag, hipStream_t st);
// out[e] = val[src[e]]
void launch_gather(int64_t n, const int64_t *src, const double *val, double *out, hipStream_t st);
// IC(0) (ldl = 0) or ILDL^T(0) (ldl = 1) of the rows rows[r0 .. r1) of the
// lower CSR (rp, ci, diagonal last) whose values V hold the matrix entries
// on entry; earlier rows must be final.  *err is set to 1 on a failed pivot.
void launch_fact_level(const int64_t *rp, const int32_t *ci, double *V, const int32_t *rows, int32_t r0, int32_t r1,
                       int32_t ldl, int *err, hipStream_t st);

template <typename TS, typename TC>
void launch_bsolve(const BlockArrays<TS> &B, int32_t p, const BArgs &a, int32_t threads,
                   size_t lds_bytes, hipStream_t st);

// In-place level-scheduled sweep of one (interface) block on a global
// vector: x (ld, nrhs columns).  Deep schedules run in one workgroup per
// column; shallow ones launch once per level over the whole device.
// G > 1 (sweeps with long rows): one launch per level, G lanes per row.
template <typename TS, typename TC>
void launch_sweep(const SweepArrays<TS> &S, const int32_t *lev_host, int32_t nlev, int32_t nrows,
                  double *x, int64_t ldx, int32_t nrhs, bool one_wg, hipStream_t st, int32_t G = 1);

// Out-of-place sweep of a schedule with at most two levels, one launch.
// dv (optional, nrhs == 1): per-block partial sums of dv . y to dpart
// ((nrows + 255) / 256 blocks).
template <typename TS, typename TC>
void launch_sweep2(const SweepArrays<TS> &S, int32_t nrows, const double *x, int64_t ldx, double *y, int64_t ldy,
                   int32_t nrhs, hipStream_t st, const double *dv = nullptr, double *dpart = nullptr);

// End of Lanczos step j (k_lanczos_next: beta_j from the partials bpart,
// v_{j+1} = w / beta_j, the recorded coefficients) together with the next
// step's first sweep: tout = L^{-T} v_{j+1} by the two-level backward
// schedule S (nw2 weight entries), equal to launch_sweep2 of v_{j+1}.
template <typename TS>
void launch_lanczos_next_sweep(int64_t s, int32_t j, const double *w, double *vnext, double *sc, double *alpha,
                               double *beta, const double *bpart, int32_t rb, const double *aval,
                               const SweepArrays<TS> &S, int64_t nw2, double *tout, hipStream_t st);

// Rank-k block of eq. skt on w (s x nrhs, ld ldw), output to wout (ldo);
// U column-major s x k:
//   c = U^T w ;  c_i <- c_i * dsc_i ;  wout = rho * w + U c
template <typename TU>
void launch_lowrank(const TU *U, int64_t s, int32_t k, const double *dsc, double rho,
                    const double *w, int64_t ldw, double *wout, int64_t ldo, int32_t nrhs,
                    double *part, int32_t nblk, double *cbuf, unsigned int *counter,
                    hipStream_t st);

}  // namespace slr

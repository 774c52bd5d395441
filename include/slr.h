/*
 * slr.h -- C ABI of the MI355X (gfx950) Schur-complement low-rank (SLR)
 * preconditioner library.
 *
 * Method: R. Li, Y. Xi, Y. Saad, "Schur complement based domain
 * decomposition preconditioners with low-rank corrections" (2015).
 *
 * Problem: A x = b with A sparse symmetric (eq. linsys), split by a p-way
 * vertex-based partition into interiors and an interface (Sec. 2.1,
 * eq. Global / Global2):
 *
 *        [ B   E ] [u]   [f]        S = C - E^T B^{-1} E      (eq. Schur)
 *        [ E^T C ] [y] = [g],       C = L L^T,  H = L^{-1} E^T B^{-1} E L^{-T}
 *
 * The preconditioner is M = [I; E^T B^{-1} I] [B E; 0 S~] (eq. M) with
 *   S~^{-1} = (1-theta)^{-1} C^{-1} + L^{-T} U_k [(I-Lambda_k)^{-1} - (1-theta)^{-1} I] U_k^T L^{-1}
 * (eq. skt written with Z_k = L^{-T} U_k), where (U_k, Lambda_k) are the k
 * largest Ritz pairs of H from Lanczos (Sec. 5.1) and theta = lambda_{k+1}
 * (Sec. 4) or 0 (eq. Lambda-1).
 *
 * Conventions shared by every entry point:
 *  - All integers are 0-based.  Vectors are FP64.  Blocks of nrhs vectors
 *    are column-major with leading dimension n (original node order).
 *  - Pointers named *_dev are device pointers (hipMalloc'd, or
 *    torch.Tensor.data_ptr()); all other pointers are host pointers.
 *  - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the default
 *    stream).  Calls that return host results synchronise that stream.
 *  - Every call returns SLR_OK (0) or a negative SLR_ERR_* code and never
 *    throws; slr_last_error() gives a message for the calling thread.
 *  - A context is not thread-safe.  Several contexts may share a device.
 *  - The library copies what it needs from caller buffers during a call
 *    and never retains caller pointers past the call.
 */
#ifndef SLR_H
#define SLR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
  SLR_OK = 0,
  SLR_ERR_ARG = -1,            /* invalid argument / unsupported option      */
  SLR_ERR_NOT_SYMMETRIC = -2,  /* A's pattern or values are not symmetric    */
  SLR_ERR_PARTITION = -3,      /* labels out of range / unsupported layout   */
  SLR_ERR_BREAKDOWN = -4,      /* factorisation pivot of a B_i failed        */
  SLR_ERR_C_NOT_SPD = -5,      /* factorisation of C failed (C must be SPD)  */
  SLR_ERR_RITZ_SINGULAR = -6,  /* |1 - lambda_i| < 1e-12 or |1 - theta| < 1e-12 */
  SLR_ERR_LANCZOS_SHORT = -7,  /* Lanczos produced fewer than the needed Ritz pairs */
  SLR_ERR_NOCONV = -8,         /* a right-hand side did not converge (x written) */
  SLR_ERR_OOM = -9,            /* device allocation failed                   */
  SLR_ERR_HIP = -10,           /* a HIP runtime call failed                  */
  SLR_ERR_ADMIT = -11          /* batch admission refused (no slot / memory) */
};

/* ---- options -------------------------------------------------------------- */
/* Choice of the shift in eq. skt: theta = lambda_{k+1} (Sec. 4), theta = the
 * smallest Ritz value of T_m (the lambda_s end of the interval of Sec. 4 on
 * which the condition number does not change), theta = 0 (truncation,
 * eq. Lambda-1), or the eq. Lambda-2 form with parameter eps:
 * on the k captured directions 1 - lambda_i is replaced by (1 - lambda_i)/eps,
 * elsewhere theta = 0, i.e. rho = 1 and the diagonal scales become
 * eps/(1 - lambda_i) - 1. */
enum { SLR_THETA_LAMBDA_K1 = 0, SLR_THETA_ZERO = 1, SLR_THETA_EPS = 2, SLR_THETA_LAMBDA_S = 3 };
/* Local solvers (Sec. 5.2, Sec. 6): exact Cholesky, zero-fill IC(0) /
 * ILDL^T(0), or the threshold forms ICT / ILDLT (left-looking by columns; an
 * entry of column j is kept when its updated value is at least droptol times
 * the 1-norm of column j of the lower triangle). */
enum { SLR_FACT_CHOL = 0, SLR_FACT_IC0 = 1, SLR_FACT_ILDLT0 = 2, SLR_FACT_ICT = 3, SLR_FACT_ILDLT = 4 };
/* Ordering of the interface for C's factor: by owner subdomain (eq. Global2),
 * greedy multicolour, or HID connectors (Sec. 5.2 names the Hierarchical
 * Interface Decomposition, which makes C's leading block block diagonal:
 * a node's key is the set of subdomains met in its closed neighbourhood;
 * by key size, then key, then original index). */
enum { SLR_CORDER_SUBDOMAIN = 0, SLR_CORDER_MULTICOLOR = 1, SLR_CORDER_HID = 2 };
/* Order of each subdomain's interior (the rows of B_i): ascending original
 * index, or the minimum degree order of B_i's graph (Sec. 6 reorders every
 * B_i by approximate minimum degree before ICT / ILDLT; here exact degrees
 * on the elimination graph, the smallest index among equal degrees). */
enum { SLR_BORDER_NATURAL = 0, SLR_BORDER_MINDEG = 1 };
enum { SLR_FP64 = 0, SLR_FP32 = 1, SLR_BF16 = 2 };
enum { SLR_PCG = 0, SLR_FCG = 1, SLR_FGMRES = 2 };
/* Reorthogonalisation of the Lanczos build (Sec. 5.1): two classical
 * Gram-Schmidt passes against all previous vectors on every step, or the
 * partial scheme of Parlett and Simon (one pass, only on steps where the
 * omega recurrence estimates a loss of orthogonality beyond sqrt(eps), and
 * on the step after). */
enum { SLR_REORTH_FULL = 0, SLR_REORTH_PARTIAL = 1 };

typedef struct {
  int64_t n;              /* order of A                                      */
  int64_t nnz;            /* stored entries (full symmetric pattern)         */
  const int64_t *rowptr;  /* host, n+1                                       */
  const int32_t *col;     /* host, nnz, sorted ascending within each row     */
  const double *val;      /* host, nnz                                       */
} slr_csr;

typedef struct {
  int32_t k;              /* rank of the correction (Sec. 4); 0 = none        */
  int32_t lanczos_steps;  /* 0 => 5k (Sec. 6)                                 */
  int32_t theta_mode;     /* SLR_THETA_LAMBDA_K1 (Sec. 4) | SLR_THETA_ZERO |
                             SLR_THETA_EPS (eq. Lambda-2, parameter eps) |
                             SLR_THETA_LAMBDA_S (Sec. 4)                      */
  int32_t b_fact;         /* local solver of the B_i (Sec. 5.2):
                             CHOL | IC0 | ILDLT0 | ICT | ILDLT               */
  int32_t c_fact;         /* factor of C = L L^T: CHOL | IC0 | ICT            */
  int32_t c_order;        /* ordering of the interface for C's factor         */
  int32_t fact_prec;      /* SLR_FP64 | SLR_FP32: storage and arithmetic of the
                             B_i / C solves inside the apply                   */
  int32_t uk_prec;        /* SLR_FP64 | SLR_FP32 | SLR_BF16: storage of U_k  */
  uint64_t seed;          /* Lanczos start vector when lanczos_v0 == NULL     */
  const double *lanczos_v0; /* host, n (original order); its interface
                               entries start Lanczos.  May be NULL.           */
  /* Optional low-rank part supplied by the caller instead of Lanczos
     (Sec. 5.3: an SLR preconditioner can be updated without rebuilding).
     U_in: host, s x k_in column-major, rows in the library's interface
     order (see slr_export perm); lambda_in: host, k_in.                      */
  int32_t k_in;
  const double *U_in;
  const double *lambda_in;
  double theta_in;        /* ignored under SLR_THETA_EPS                     */
  /* eq. Lambda-2 parameter, > 0 under SLR_THETA_EPS (SLR_ERR_ARG otherwise);
     unused by the other modes.  eps = 1 gives the SLR_THETA_ZERO
     preconditioner. */
  double eps;
  /* Rank from a target condition number (eq. condk): with cond_K > 1 the
     Lanczos build keeps the Ritz values above 1 - 1/cond_K, at most k of
     them (the rank in use, possibly 0, is reported in slr_info.k); 0
     keeps k.  Values in (0, 1] are SLR_ERR_ARG.  Ignored for an imported
     low-rank part. */
  double cond_K;
  /* SLR_REORTH_FULL | SLR_REORTH_PARTIAL.  slr_grow_lowrank always uses
     full reorthogonalisation (the omega estimates do not cover U_k). */
  int32_t reorth;
  /* 1: keep what slr_refactor needs (the input pattern, the factorisation
     plans and the maps of every stored coefficient; about 24 bytes per
     stored coefficient of device memory).  Needs incomplete factors (B:
     IC0 | ILDLT0, C: IC0) and nnz < 2^31; SLR_ERR_ARG otherwise. */
  int32_t refactor;
  /* drop tolerance of the ICT / ILDLT factors (>= 0; 0 keeps every entry,
     i.e. the exact factorisation).  Default 1e-3. */
  double droptol;
  /* SLR_BORDER_NATURAL | SLR_BORDER_MINDEG: order of the rows of each B_i
     (default NATURAL); every factor, level schedule and refactorisation
     plan follows it.  Other values are SLR_ERR_ARG. */
  int32_t b_order;
  /* Interface solver.  1 (default): C = L L^T from c_fact.  2: the recursive
     SLR on C of Sec. 5.2 -- with C in HID order (c_order must be
     SLR_CORDER_HID) C = [C1 F; F^T C2], C1 the nodes of the lowest connector
     level (block diagonal: its connected pieces, which must each be a
     contiguous range of the order), and C's solve is itself an SLR
     preconditioner with B := C1, E := F, C := C2 (both factored with
     c_fact), rank k2 from lanczos_steps2 inner Lanczos steps (full
     reorthogonalisation, started from the start vector's entries on C2) and
     theta2 = lambda_{k2+1}.  That inner preconditioner is used in the
     factored form K K^T (K^T in place of L^{-1}, K in place of L^{-T}):
       K^T v = (L1^{-1} v1, Q2 L2^{-1}(v2 - F^T C1^{-1} v1)),
       K w   = (L1^{-T}(w1 - L1^{-1} F b2), b2 = L2^{-T} Q2 w2),
     Q2 = G2^{1/2}, G2 = rho2 I + U2 D2 U2^T of eq. skt one level down; G2 must
     be positive definite (every inner Ritz value kept and theta2 below 1,
     else SLR_ERR_C_NOT_SPD).  Not with refactor; a single connector level
     is SLR_ERR_ARG. */
  int32_t c_levels;
  int32_t k2;             /* inner rank (0 => k), at most 64                 */
  int32_t lanczos_steps2; /* inner Lanczos steps (0 => 5 k2)                 */
} slr_opts;

typedef struct {
  int32_t method;         /* SLR_PCG | SLR_FCG (flexible CG) | SLR_FGMRES   */
  int32_t restart;        /* FGMRES restart length (default 40, Sec. 6)      */
  int32_t maxit;          /* default 300 (Sec. 6)                            */
  int32_t check_every;    /* CG / FCG: most iterations between host polls of
                             convergence (default 8; shorter near the end,
                             from the residual's decay)                    */
  double rtol;            /* ||r_j|| <= rtol ||b|| (default 1e-8, Sec. 6)     */
} slr_solve_opts;

typedef struct {
  int32_t iters;          /* iterations: updates of x (CG, FCG), Arnoldi     */
                          /* steps (FGMRES)                                  */
  int32_t status;         /* SLR_OK or SLR_ERR_NOCONV                        */
  double relres;          /* final true ||b - A x|| / ||b||, FP64            */
} slr_solve_info;

typedef struct {
  int64_t n, m, s;        /* unknowns, interior, interface                   */
  int32_t p;              /* subdomains                                      */
  int32_t k;              /* rank in use                                     */
  int32_t lanczos_steps;  /* steps actually taken                            */
  int32_t b_levels_max;   /* deepest level schedule of a B_i sweep           */
  int32_t c_levels;       /* level count of C's forward sweep                */
  int32_t c_colors;       /* colours (multicolour ordering) or 0             */
  int64_t nnz_LB, nnz_LC, nnz_E, nnz_A; /* incl. diagonals for L_B, L_C      */
  int64_t m_min, m_max;   /* smallest / largest subdomain interior           */
  double theta;
  double setup_host_s;    /* host factorisation + analysis time              */
  double setup_lanczos_s; /* device Lanczos + eigensolve time                */
  int64_t device_bytes;   /* persistent device memory held by the context    */
  int32_t lanczos_reorth; /* Lanczos steps that were reorthogonalised        */
  /* launch shapes chosen by slr_autotune (0: the built-in plan): B kernel
     threads per workgroup and LDS share 1/div, for one column and for
     several (with the most columns per workgroup); chunks of the rank-k
     partial sums */
  int32_t tune_b_threads1, tune_b_lds_div1;
  int32_t tune_b_threadsM, tune_b_lds_divM, tune_b_rmaxM;
  int32_t lr_chunks;
  /* recursive interface solver (c_levels 2; zero otherwise): nodes of C1,
     inner rank, inner Lanczos steps taken, deepest C1 block sweep, level
     count of C2's forward sweep, theta2 */
  int64_t s1;
  int32_t k2, lanczos_steps2;
  int32_t c1_levels, c2_levels;
  double theta2;
  int64_t nnz_LC1, nnz_LC2, nnz_F;  /* entries of L1, L2 and of F         */
  /* 1 or 2: several-column B solves run as a persistent grid (slr_autotune's
     or slr_set_bsolve_plan's choice; 2: columns per item by subdomain size) */
  int32_t tune_b_persistentM;
  /* subdomains whose B sweeps keep x in LDS in the forward sweep's level
     order rather than the row order (chosen at setup where a model of the
     LDS bank conflicts of the sweeps' gathers favours it clearly) */
  int32_t b_lds_level_order;
} slr_info;

typedef struct slr_ctx slr_ctx;
typedef struct slr_batch slr_batch;

/* slr_default_opts / slr_default_solve_opts: fill with the paper's defaults
 * (theta = lambda_{k+1}, IC(0) factors, 5k Lanczos steps, rtol 1e-8,
 * maxit 300, GMRES restart 40; Sec. 4 and Sec. 6). */
void slr_default_opts(slr_opts *o);
void slr_default_solve_opts(slr_solve_opts *o);

/* slr_setup: build the preconditioner for A and partition `part` (host, n
 * labels in -1..p-1; Sec. 2.1).  A node labelled q >= 0 coupled to a node
 * labelled r >= 0, r != q, is an interface node of q (vertex-based
 * partitioning); nodes labelled -1 are separator nodes (edge-based
 * partitioning: a vertex separator, all interface), and coupling to one
 * does not make a node interface.  Both kinds may be mixed; interior nodes
 * of two subdomains must not be coupled.  The interface is ordered by owner
 * subdomain with the separator nodes last (eq. Global2).  With separator
 * nodes E^T is applied as a CSR product after the B kernel (a separator row
 * couples to several subdomains).  Classification, DD ordering (eq.
 * Global), the B_i and C factorisations and level schedules run on the
 * host; the factors are uploaded and the Lanczos build of (U_k, Lambda_k,
 * theta) on H (eq. H, Sec. 5.1) runs on the device.  Errors: ARG (also
 * refactor with separator labels), NOT_SYMMETRIC, PARTITION (labels out of
 * range, coupled interiors), BREAKDOWN, C_NOT_SPD, RITZ_SINGULAR,
 * LANCZOS_SHORT, OOM, HIP. */
int slr_setup(const slr_csr *A, const int32_t *part, int32_t p, const slr_opts *o,
              void *hip_stream, slr_ctx **out);

/* slr_set_bsolve_plan: set the B kernel's launch shape for one column
 * (several == 0) or several columns (several != 0) instead of slr_autotune:
 * threads per workgroup (256, 512 or 1024; 0 restores the built-in plan
 * and ignores the rest), the share 1/lds_div of the LDS limit a workgroup
 * may take (1..8), the most columns per workgroup (1..16), and persistent =
 * 1 for a resident grid (as many workgroups as fit the compute units at
 * once) walking a schedule of (subdomain, column group) items, longest
 * first by each subdomain's levels and entries, each item given to the
 * workgroup with the least work so far; the batching form with subdomains
 * of uneven size (a launch with no more items than workgroups stays a plain
 * grid).  persistent = 2: the same, with each subdomain taking as many
 * columns per item as its own rows let the workgroup's x region hold (at
 * most one fewer than its waves), so small subdomains take more columns.  Results are bitwise the same under every plan.  SLR_ERR_ARG for
 * values out of range, a largest subdomain that does not fit the share, or
 * live batches. */
int slr_set_bsolve_plan(slr_ctx *c, int32_t several, int32_t threads, int32_t lds_div, int32_t rmax,
                        int32_t persistent);

/* slr_analyze: the host part of slr_setup only (classification, DD
 * ordering, factorisations, level schedules) -- no device memory is
 * touched.  Fills `info` (sizes, nnz, level depths; k, theta and the
 * Lanczos fields are 0; device_bytes is the estimated persistent device
 * footprint of slr_setup) and, if perm != NULL, the internal -> original
 * permutation (n int64).  Same errors as slr_setup's host part. */
int slr_analyze(const slr_csr *A, const int32_t *part, int32_t p, const slr_opts *o, slr_info *info,
                int64_t *perm);

/* slr_update_lowrank: rebuild (U_k, Lambda_k, theta) on the device by a
 * fresh Lanczos run on H with the resident factors (Sec. 5.1); k <= 64,
 * lanczos_steps 0 => 5k, lanczos_v0 as in slr_opts (NULL => seed); the
 * context's theta_mode, eps and cond_K apply.  An SLR preconditioner can be
 * improved this way without refactoring (Sec. 5.3).  SLR_ERR_ARG while
 * batches (slr_batch_create) exist on the context.  Synchronises
 * hip_stream.  Errors as slr_setup's Lanczos. */
int slr_update_lowrank(slr_ctx *c, int32_t k, int32_t lanczos_steps, const double *lanczos_v0,
                       void *hip_stream);

/* slr_grow_lowrank: add up to k_add vectors to the resident (U_k, Lambda_k)
 * without discarding them (Sec. 5.3, by deflation).  A Lanczos run on H
 * whose start vector (interface entries of lanczos_v0, or the seeded one)
 * and Gram-Schmidt passes are also orthogonalised against the current U_k
 * explores H on the complement of the captured directions; its k_add
 * largest Ritz pairs are appended (fewer under cond_K > 1, eq. condk) and
 * theta is recomputed from its Ritz values under the context's theta_mode
 * (lambda_{k+1}: the largest one not taken).  k + k_add <= 64; steps 0 =>
 * 5 k_add, at most min(s - k, 1024 - k).  A start vector inside span(U_k)
 * (norm of its projection <= 1e-12 after normalising) is SLR_ERR_ARG.  On
 * any error the resident low-rank part is unchanged.  SLR_ERR_ARG while
 * batches exist on the context.  Synchronises hip_stream. */
int slr_grow_lowrank(slr_ctx *c, int32_t k_add, int32_t lanczos_steps, const double *lanczos_v0,
                     void *hip_stream);

/* slr_refactor: new values for A with the pattern given to slr_setup (val:
 * nnz values in that CSR's order, on the host, or on the device when
 * on_device != 0; the call does not keep the pointer), for a context set up with
 * opts.refactor = 1.  The zero-fill factors of the B_i and of C (Sec. 5.2,
 * IC(0) / ILDL^T(0)) are recomputed on the device, level by level with the
 * schedules of the forward sweeps, and every stored coefficient of the
 * apply (sweep scales and weights, E, E^T, A for the Krylov products) is
 * rewritten in place in the context's storage precision; the results equal
 * those of a fresh slr_setup with the new values.  The low-rank part
 * (U_k, Lambda_k, theta) is kept: call slr_update_lowrank to rebuild it for
 * the new H.  Errors: SLR_ERR_NOT_SYMMETRIC (every value must equal its
 * mirror's; checked where the values are),
 * SLR_ERR_BREAKDOWN (a B_i pivot), SLR_ERR_C_NOT_SPD (a C pivot) -- after
 * which every stored coefficient is unchanged -- and SLR_ERR_ARG (no
 * opts.refactor, or batches exist on the context).  Synchronises
 * hip_stream. */
int slr_refactor(slr_ctx *c, const double *val, int32_t on_device, void *hip_stream);

/* slr_time_kernel: average device time (ms, via HIP events on hip_stream)
 * of `reps` back-to-back launches of one hot-path stage on nrhs internal
 * scratch columns, in the launch configuration slr_apply_dd uses:
 * 0 = first batched B solve (B^{-1} f with the E^T epilogue),
 * 1 = interface forward sweep, 2 = rank-k block, 3 = interface backward
 * sweep, 4 = second batched B solve (E y prologue), 5 = whole apply,
 * 6 = SpMV with A.  Inputs are deterministic filler values. */
int slr_time_kernel(slr_ctx *c, int32_t which, int32_t nrhs, int32_t reps, void *hip_stream, double *ms);

/* slr_autotune: time the batched B solve (first half of the apply, with its
 * E^T epilogue) for nrhs columns under every candidate launch shape --
 * threads per workgroup (1024, 512, 256), share of the LDS per workgroup
 * (1, 1/2, 1/4: that many workgroups fit a CU) and most columns per
 * workgroup -- and keep the fastest for one column (nrhs == 1) or for
 * several (nrhs > 1); then the number of row chunks of the rank-k partial
 * sums (128 ... 2048).  reps launches per candidate (0: 3), HIP events on
 * hip_stream.  The B kernel's results do not depend on the launch shape;
 * the rank-k chunks set the grouping of its sums, the same for every later
 * apply of the context (alone or in a batch).  The choices are reported in
 * slr_info (tune_*, lr_chunks) and kept by slr_export_setup.  SLR_ERR_ARG
 * while batches exist.  Synchronises hip_stream. */
int slr_autotune(slr_ctx *c, int32_t nrhs, int32_t reps, void *hip_stream);

/* slr_apply: z = M^{-1} r for nrhs vectors (eq. M with eq. skt).  r_dev,
 * z_dev: device, n x nrhs column-major, original order; may not alias.
 * Two B solves, one S~ solve (Sec. 2.2).  Asynchronous on hip_stream. */
int slr_apply(slr_ctx *c, const double *r_dev, double *z_dev, int32_t nrhs, void *hip_stream);

/* slr_apply_dd: as slr_apply but vectors are in the library's internal DD
 * order (interiors by subdomain, then interface; slr_export perm). */
int slr_apply_dd(slr_ctx *c, const double *r_dev, double *z_dev, int32_t nrhs, void *hip_stream);

/* slr_apply_dd_noalloc: slr_apply_dd for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, layout and results
 * (the same kernels in the same order, so the output equals slr_apply_dd's
 * bit for bit); the call allocates nothing.  The apply's scratch (two
 * s x nrhs interface blocks, the rank-k partials and coefficients, in all
 * 2 * 8 s nrhs + 8 k nrhs (chunks + 1) bytes, each part rounded up to 256)
 * comes from one fixed device array of 64 MiB per GPU, which the library
 * holds from its first slr_setup on that GPU until the process ends.
 * nrhs whose scratch exceeds 64 MiB is SLR_ERR_ARG (the message gives the
 * bytes needed); the context's device must be the current one (SLR_ERR_ARG
 * otherwise).  Every call on a GPU, from any context or stream, shares that
 * GPU's array and leaves its contents behind: calls that overlap on one GPU
 * (concurrent streams, threads) race and give wrong results; serialise
 * them.  Asynchronous on hip_stream. */
int slr_apply_dd_noalloc(slr_ctx *c, const double *r_dev, double *z_dev, int32_t nrhs, void *hip_stream);

/* slr_solve: preconditioned Krylov solve A x = b (Sec. 6: CG for SPD,
 * GMRES(40) for indefinite; flexible CG for reduced-precision factors).
 * b_dev, x_dev: device n x nrhs (original order); x0 = 0.  Stops when
 * ||r_j|| <= rtol ||b|| per column, or at maxit.  info: host array of
 * nrhs entries.  Returns SLR_ERR_NOCONV if any column failed (x is still
 * written).  FGMRES takes nrhs = 1.  Synchronises hip_stream. */
int slr_solve(slr_ctx *c, const double *b_dev, double *x_dev, int32_t nrhs,
              const slr_solve_opts *so, slr_solve_info *info, void *hip_stream);

/* slr_solve_workspace_bytes: device bytes of the workspace slr_solve
 * allocates for nrhs columns with the options `so` (NULL: the defaults);
 * for FGMRES it depends on the restart length (the basis and the
 * preconditioned basis: 2 restart + 1 vectors of n).  The context keeps
 * this workspace after the solve (see slr_trim). */
size_t slr_solve_workspace_bytes(const slr_ctx *c, int32_t nrhs, const slr_solve_opts *so);

/* slr_trim: release the scratch buffers a context keeps between calls to
 * avoid allocating again (the Lanczos build's basis and work vectors, the
 * FGMRES and CG workspaces, the original-order staging of slr_apply /
 * slr_spmv, and the apply workspace beyond one column).  The next call
 * that needs them allocates them again.  slr_query's device_bytes counts
 * them while they are kept; without slr_trim they live until slr_destroy.
 * Synchronises the device when the memory came from an allocator set with
 * slr_set_allocator. */
int slr_trim(slr_ctx *c);

/* slr_query: sizes, level depths, theta, timings, memory. */
int slr_query(const slr_ctx *c, slr_info *info);

/* slr_export: copy setup results to host buffers (any may be NULL):
 * perm (n int64, internal -> original index), ritz (lanczos_steps values,
 * descending), lambda (k), U (s x k column-major FP64, interface order),
 * alpha/beta (Lanczos tridiagonal, lanczos_steps each; beta's last entry is
 * the final residual norm). */
int slr_export(const slr_ctx *c, int64_t *perm, double *ritz, double *lambda,
               double *U, double *alpha, double *beta);

/* slr_export_inner: the recursive interface solver's inner low-rank part
 * (c_levels 2, Sec. 5.2 with Sec. 5.1 one level down) to host buffers (any
 * may be NULL): ritz2 (slr_info.lanczos_steps2 values, descending), lambda2
 * (k2), U2 (s2 x k2 column-major FP64, s2 = s - s1, rows in the interface
 * order after the s1 nodes of C1); theta2 is in slr_info.  SLR_ERR_ARG for
 * a context without it. */
int slr_export_inner(const slr_ctx *c, double *ritz2, double *lambda2, double *U2);

/* slr_export_setup: serialise the whole resident preconditioner -- the
 * DD ordering, A in that order, the packed B_i sweeps with E and E^T
 * (Sec. 2.1, Sec. 5.2), C's sweeps, the low-rank part (U_k in FP64,
 * Lambda_k, theta; Sec. 4, Sec. 5.1), the Lanczos coefficients and the
 * options -- into buf (host, cap bytes).  *bytes receives the size; with
 * buf == NULL only the size is returned.  cap < *bytes is SLR_ERR_ARG.
 * Current values are taken (after slr_refactor, the refactored ones).  The
 * layout is this library build's own (magic, length, records, FNV-1a
 * checksum), native byte order.  A context with the recursive interface
 * solver (c_levels 2) or with separator labels is SLR_ERR_ARG. */
int slr_export_setup(const slr_ctx *c, void *buf, size_t cap, size_t *bytes);

/* slr_import: a new context on the current device from slr_export_setup's
 * bytes (host; not retained), without the host analysis or the Lanczos
 * build.  Its apply and solves equal those of the exported context bit for
 * bit.  The imported context cannot slr_refactor (no refactorisation plan
 * is serialised).  Errors: SLR_ERR_ARG (wrong magic, length, checksum or
 * inconsistent sizes), SLR_ERR_OOM, SLR_ERR_HIP.  The content beyond its
 * structure is trusted: pass only bytes that slr_export_setup wrote. */
int slr_import(const void *buf, size_t bytes, void *hip_stream, slr_ctx **out);

/* slr_set_allocator: route every device allocation of the library (all
 * contexts and batches created or grown afterwards) through alloc(bytes,
 * user), which returns device memory of the current device or NULL
 * (reported as SLR_ERR_OOM), and free_(ptr, user) -- e.g. PyTorch's caching
 * allocator, so that PyTorch owns the memory.  Memory keeps the allocator
 * that made it: a later change frees older blocks through their own
 * free_.  The library synchronises the device before it hands memory back
 * through free_.  alloc == NULL or free_ == NULL restores hipMalloc /
 * hipFree.  Process-wide; call it while no other thread is inside the
 * library.  (Pinned host staging still uses hipHostMalloc; the 64 MiB
 * array of slr_apply_dd_noalloc is static.) */
typedef void *(*slr_alloc_fn)(size_t bytes, void *user);
typedef void (*slr_free_fn)(void *ptr, void *user);
void slr_set_allocator(slr_alloc_fn alloc, slr_free_fn free_, void *user);

/* slr_spmv: y = A x in the original order (device n x nrhs), FP64. */
int slr_spmv(slr_ctx *c, const double *x_dev, double *y_dev, int32_t nrhs, void *hip_stream);

/* ---- continuous batching (serving) -----------------------------------
 * A batch owns `max_cols` right-hand-side slots of one context, each with
 * its own Krylov state kept on the device.  Requests are admitted while
 * slots are free; slr_batch_step advances every active slot by `iters`
 * iterations; finished requests are returned by slr_batch_poll and their
 * slots are reused.  A column's arithmetic does not depend on the other
 * columns, so a result is the same alone and in a mix.  PCG / FCG only. */
int slr_batch_create(slr_ctx *c, int32_t max_cols, int32_t method, double rtol,
                     int32_t maxit, slr_batch **out);
/* Admit one request of nrhs columns: b_dev / x_dev device n x nrhs
 * (original order); x_dev is written when the request completes.  Returns
 * SLR_ERR_ADMIT when fewer than nrhs slots are free. */
int slr_batch_admit(slr_batch *b, const double *b_dev, double *x_dev, int32_t nrhs,
                    int64_t tag, void *hip_stream);
int slr_batch_step(slr_batch *b, int32_t iters, void *hip_stream);
/* Retire finished requests: writes up to max_done tags (and per-request
 * worst iteration count / relres / status) and returns how many. */
int slr_batch_poll(slr_batch *b, int64_t *tags, slr_solve_info *info, int32_t max_done,
                   void *hip_stream);
int slr_batch_active(const slr_batch *b);       /* columns in flight */
size_t slr_batch_bytes(const slr_batch *b);     /* device bytes held */
void slr_batch_destroy(slr_batch *b);

/* ---- misc ------------------------------------------------------------- */
/* slr_destroy: frees the context and its device memory; NULL is a no-op.
 * Destroy the context's batches first (they refer to it) and let its
 * streams' work finish. */
void slr_destroy(slr_ctx *c);
const char *slr_strerror(int code);
const char *slr_last_error(void);
int slr_device_lds_bytes(void);   /* LDS per workgroup the library plans for */

#ifdef __cplusplus
}
#endif
#endif /* SLR_H */

// Host-side analysis of the SLR preconditioner: classification, DD
// ordering, block extraction, local factorisations and level schedules.
// Everything here runs once per slr_setup; the results are uploaded.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace slr {

// One triangular sweep of one diagonal block, level scheduled.
// Row t of the level-sorted list computes
//     x[rows[t]] = sc[t] * x[rows[t]] - sum_e w[e] * x[ci[e]],  e in [rp[t], rp[t+1])
// in place: x holds the right-hand side on entry.  All indices are local
// to the block.  The off-diagonal weights are pre-divided by the pivot.
struct Sweep {
  int32_t nrows = 0, nlev = 0;
  std::vector<int32_t> levptr;  // nlev + 1, into the level-sorted rows
  std::vector<int32_t> rows;    // nrows
  std::vector<int32_t> rp;      // nrows + 1
  std::vector<int32_t> ci;
  std::vector<double> w;
  std::vector<double> sc;
  // Where the coefficients come from (entry indices of the factor's CSR
  // values, for a numeric refactorisation on the device): sc[t] uses entry
  // sc_e[t] (the row's diagonal), w[e] uses entry w_e[e] and, when
  // `divided`, the row's diagonal as divisor.  sc is 1 when `unit_sc`.
  std::vector<int32_t> sc_e, w_e;
  bool divided = true, unit_sc = false;
};

// Lower factor in CSR (sorted columns, diagonal last in each row).
// kind 0: L L^T (Cholesky / IC(0));  kind 2: unit L with D in the diagonal slots.
struct LowerFactor {
  int32_t n = 0;
  int kind = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v;
};

struct Block {            // one subdomain
  int32_t m0 = 0, m = 0;  // interior range in the internal order
  Sweep fwd, bwd;
  // E rows: interior rows (local) coupled to the interface
  std::vector<int32_t> e_row, e_ptr, e_q;   // e_q: interface index (0..s)
  std::vector<double> e_val;
  // E^T rows: interface rows owned by this subdomain
  std::vector<int32_t> t_q, t_ptr, t_j;     // t_j: local interior index
  std::vector<double> t_val;
  std::vector<int64_t> e_src, t_src;        // entries of the input CSR behind e_val / t_val
  int64_t nnz_L = 0;
  int64_t f_base = 0;                       // first entry of this block's factor in the global B factor
};

// Lower factor of a block-diagonal matrix for a device refactorisation:
// rows in the internal order, diagonal last; src[e] is the entry of the
// input CSR that holds the matrix value at e; rows[lev[l] .. lev[l+1]) are
// independent once all earlier levels are done.
struct RefactorPlan {
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<int64_t> src;
  std::vector<int32_t> lev, rows;
  int kind = 0;   // 0: IC(0), 2: ILDL^T(0)
};

struct HostSetup {
  int64_t n = 0, m = 0, s = 0;
  int32_t p = 0;
  std::vector<int64_t> perm;    // internal -> original
  std::vector<int64_t> iperm;   // original -> internal
  std::vector<Block> blocks;
  Sweep cfwd, cbwd;             // interface factor sweeps (indices 0..s)
  int64_t nnz_LC = 0, nnz_E = 0;
  int32_t c_colors = 0;
  // A in the internal order (for the Krylov SpMV)
  std::vector<int64_t> a_rp;
  std::vector<int32_t> a_ci;
  std::vector<double> a_v;
  std::vector<int64_t> a_src;   // input CSR entry of each a_v
  // device refactorisation plans (filled when the factors are incomplete
  // and SetupParams::plan is set)
  bool have_plan = false;
  RefactorPlan fb, fc;
  // Recursive interface solver (SetupParams::c_levels == 2, Sec. 5.2): in
  // HID order C = [C1 F; F^T C2] with C1 the s1 nodes of the lowest
  // connector level.  c1blocks: the connected pieces of C1's graph (each a
  // contiguous range; m0 / m local to C1), their factors' sweeps, and as E
  // rows their couplings F to C2 (e_q: index in C2).  C2's factor sweeps
  // in c2fwd / c2bwd; F^T as CSR over the C2 rows with C1 columns.
  // edge-based partitions (labels -1): E^T over all interface rows as CSR
  // (columns: interior indices), used instead of the blocks' E^T rows
  bool has_sep = false;
  std::vector<int64_t> et_rp;
  std::vector<int32_t> et_ci;
  std::vector<double> et_v;
  int64_t s1 = 0;
  std::vector<Block> c1blocks;
  Sweep c2fwd, c2bwd;
  std::vector<int64_t> ft_rp;
  std::vector<int32_t> ft_ci;
  std::vector<double> ft_v;
  int64_t nnz_LC1 = 0, nnz_LC2 = 0;
};

struct SetupParams {
  int b_fact = 1, c_fact = 1, c_order = 0, fact_prec = 0;
  int b_order = 0;         // SLR_BORDER_NATURAL | SLR_BORDER_MINDEG
  double droptol = 1e-3;   // threshold factors (ICT / ILDLT)
  bool plan = false;   // build the refactorisation plans
  int c_levels = 1;    // 2: recursive interface solver (needs the HID order)
};

// A symmetric in pattern and value: every (i, j) has a matching (j, i).
bool is_symmetric(int64_t n, const int64_t *rp, const int32_t *ci, const double *v);

// Returns 0 or an SLR_ERR_* code; `err` receives a message.
int host_setup(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
               const int32_t *part, int32_t p, const SetupParams &prm, HostSetup &out,
               std::string &err);

}  // namespace slr

// C ABI of the SLR preconditioner library (declared in include/slr.h).
//
// Paper: Li, Xi & Saad, "Schur complement based domain decomposition
// preconditioners with low-rank corrections" (2015).
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <queue>
#include <string>
#include <vector>

#include "slr.h"
#include "slr_dev.h"
#include "slr_host.h"
#include "slr_kern.h"

using namespace slr;

namespace {

thread_local std::string g_err;

// Scratch of slr_apply_dd_noalloc: one fixed array per GPU, held until the
// process ends, so that the call allocates nothing.  Host code never passes
// `scratch` itself to a kernel (on the host it names a stand-in, not device
// memory): it uses the device address that hipGetSymbolAddress returns for
// the current GPU, kept per device in g_scratch_dev.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
char *g_scratch_dev[kMaxDevices] = {};

constexpr int64_t pad8h(int64_t x) { return (x + 7) & ~int64_t(7); }
constexpr int64_t pad16h(int64_t x) { return (x + 15) & ~int64_t(15); }

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(SLR_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// compute units of the current device
int device_cu_count(void) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 256;
  return prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
}

// Device address of `scratch` on `dev`, which must be the current device:
// looked up once per device (hipGetSymbolAddress) and kept.
int scratch_address(int dev, char **out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return fail(SLR_ERR_ARG, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SLR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = (char *)p;
  }
  *out = g_scratch_dev[dev];
  return SLR_OK;
}

// Device memory of the library: hipMalloc / hipFree, or the caller's
// allocator (slr_set_allocator).  Each block remembers the allocator that
// made it, so that a change of allocator never frees memory through the
// wrong one.  Freeing through a caller's allocator first synchronises the
// device (hipFree's own behaviour), so that the caller may hand the memory
// out again at once.
struct AllocHook {
  slr_alloc_fn alloc = nullptr;
  slr_free_fn free_ = nullptr;
  void *user = nullptr;
};
std::mutex g_alloc_mu;
AllocHook g_alloc;

struct DevBlock {
  void *p = nullptr;
  size_t bytes = 0;
  AllocHook by;          // alloc == nullptr: hipMalloc
};

bool dev_malloc(size_t bytes, DevBlock &b) {
  AllocHook h;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    h = g_alloc;
  }
  b = DevBlock{};
  void *p = nullptr;
  if (h.alloc) {
    p = h.alloc(bytes, h.user);
    if (!p) return false;
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    return false;
  }
  b.p = p;
  b.bytes = bytes;
  b.by = h;
  return true;
}

void dev_free_all(std::vector<DevBlock> &v) {
  bool hooked = false;
  for (const DevBlock &b : v) hooked = hooked || (b.p && b.by.alloc);
  if (hooked) (void)hipDeviceSynchronize();
  for (DevBlock &b : v) {
    if (!b.p) continue;
    if (b.by.alloc) {
      if (b.by.free_) b.by.free_(b.p, b.by.user);
    } else {
      (void)hipFree(b.p);
    }
    b.p = nullptr;
  }
  v.clear();
}

// Device allocations owned by one object, freed together.
struct DevPool {
  std::vector<DevBlock> blocks;
  int64_t bytes = 0;
  template <typename T>
  T *alloc(size_t n) {
    if (n == 0) n = 1;
    DevBlock b;
    if (!dev_malloc(n * sizeof(T), b)) return nullptr;
    blocks.push_back(b);
    bytes += (int64_t)(n * sizeof(T));
    return (T *)b.p;
  }
  template <typename T>
  T *upload(const std::vector<T> &v) {
    T *p = alloc<T>(v.size());
    if (p && !v.empty()) {
      if (hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    }
    return p;
  }
  void release() {
    dev_free_all(blocks);
    bytes = 0;
  }
};

// A device buffer kept by its owner between calls (Arena).
struct KeptBuf {
  std::vector<DevBlock> blk;   // at most one block
  char *base = nullptr;
  size_t cap = 0;
  void release() {
    dev_free_all(blk);
    base = nullptr;
    cap = 0;
  }
};

// Sub-allocations (256-byte aligned) from a device buffer that its owner
// keeps between calls.  A request that does not fit gets an allocation of
// its own, freed at release(); release() then regrows the kept buffer to
// the whole size seen, so that the next call with the same sizes allocates
// nothing.  Contents are not preserved between calls.
struct Arena {
  KeptBuf &kb;
  size_t used = 0, want = 0;
  DevPool extra;
  explicit Arena(KeptBuf &k) : kb(k) {}
  template <typename T>
  T *alloc(size_t n) {
    if (n == 0) n = 1;
    const size_t b = (n * sizeof(T) + 255) & ~(size_t)255;
    want += b;
    if (used + b <= kb.cap) {
      T *p = (T *)(kb.base + used);
      used += b;
      return p;
    }
    return extra.alloc<T>(n);
  }
  void release() {
    extra.release();
    if (want > kb.cap) {
      kb.release();
      DevBlock b;
      if (dev_malloc(want, b)) {
        kb.blk.push_back(b);
        kb.base = (char *)b.p;
        kb.cap = want;
      }
    }
    used = want = 0;
  }
};

template <typename TS>
std::vector<TS> conv(const std::vector<double> &v) {
  std::vector<TS> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = (TS)v[i];
  return o;
}

// Scratch of one apply pipeline (one per context, one per batch).
struct ApplyWS {
  int32_t cap = 0;
  int32_t k = 0;              // rank the rank-k scratch is sized for
  double *W = nullptr;        // s x cap interface temporary
  double *W2 = nullptr;       // second s x cap interface temporary
  double *lr_part = nullptr;  // nblk x cap x k
  int32_t nblk = 0;            // rank-k partial chunks lr_part was sized for
  double *cbuf = nullptr;     // k x cap
  double *Z = nullptr;        // m x cap interior solution (edge-based partitions only)
  unsigned int *counter = nullptr;
  DevPool pool;
};

}  // namespace

struct slr_ctx {
  int device = 0;
  int64_t n = 0, m = 0, s = 0;
  int32_t p = 0;
  slr_opts opts{};
  int fact_prec = SLR_FP64, uk_prec = SLR_FP64;
  DevPool pool;
  // internal order
  std::vector<int64_t> perm_h;
  int64_t *perm = nullptr;
  int64_t *a_rp = nullptr;
  int32_t *a_ci = nullptr;
  double *a_v = nullptr;
  int64_t nnz_a = 0;
  // edge-based partitions (separator nodes): E^T as CSR over all interface
  // rows, applied after the B kernel instead of in its epilogue
  bool sep = false;
  int64_t *et_rp = nullptr;
  int32_t *et_ci = nullptr;
  double *et_v = nullptr;
  // B blocks and interface sweeps (one of the two precisions is used)
  BlockArrays<double> Bd;
  BlockArrays<float> Bf;
  SweepArrays<double> Cfd, Cbd;
  SweepArrays<float> Cff, Cbf;
  std::vector<int32_t> cf_lev_h, cb_lev_h;
  int32_t cf_nlev = 0, cb_nlev = 0;
  int64_t cb_nnz = 0;           // weight entries of the backward interface schedule
  bool c_one_wg = true;
  // lanes per row of the interface sweeps (> 1: rows long enough that one
  // launch per level with a group of lanes per row wins; set from the mean
  // row length of each sweep)
  int32_t cf_group = 1, cb_group = 1;
  bool c_two_level = false;     // interface schedules of <= 2 levels: one launch per sweep
  int32_t b_threads = 1024;
  int32_t n_cu = 256;           // compute units of the device
  int32_t b_max_m = 0, b_max_lev = 0, b_max_level_bytes = 0;
  int64_t b_data_bytes = 0;
  size_t lds_limit = 65536;
  // low-rank part
  int32_t k = 0;
  double theta = 0.0, rho = 1.0;
  void *U = nullptr;            // FP64 / FP32: s x k column-major; BF16: tiles of U^T W (matrix cores)
  void *Urm = nullptr;          // FP64 / FP32: row-major padded copy (U^T w); BF16: tiles of the update
  double *U64 = nullptr;        // s x k column-major, FP64 (export)
  double *dsc = nullptr;        // k scales (1-lambda)^{-1} - rho
  std::vector<double> lam_h, ritz_h, alpha_h, beta_h;
  int32_t lr_nblk = 256;       // group chunks of the row-major rank-k partials (set with U_k)
  int32_t lrm_nblk = 512;      // row chunks of the matrix-core rank-k partials
  int32_t lr_nblk_tuned = 0;   // slr_autotune's choice of lr_nblk (0: by the size of U_k)
  // launch shapes of the B kernel chosen by slr_autotune (threads == 0: the
  // built-in plan): threads per workgroup, the share of the LDS limit a
  // workgroup may take (1/lds_div), and the most columns per workgroup
  struct BTune {
    int32_t threads = 0, lds_div = 1, rmax = 16;
    int32_t persistent = 0;     // 1: a resident grid walks a longest-first schedule; 2: the same with
                                // each subdomain's own column count
  } tune1, tuneM;              // one column; several columns
  // schedules of the persistent B launch, by (column groups, workgroups)
  struct BSched {
    int32_t mode = 0, nrhs = 0, R = 0, nwg = 0, waves = 0;
    int32_t *ptr = nullptr, *items = nullptr;
  };
  std::vector<BSched> bsched;
  DevPool schedpool;
  std::vector<double> b_cost_h;  // per subdomain: work estimate of one B solve item
  std::vector<int32_t> b_m_h;    // per subdomain: interior rows
  DevPool lrpool;               // U, U64, dsc
  // Recursive interface solver (opts.c_levels == 2, Sec. 5.2): C = [C1 F;
  // F^T C2] in HID order.  The connectors of C1 form a block-diagonal
  // matrix solved by the B kernel (with only one of its sweeps where only
  // L1^{-1} or L1^{-T} is wanted; their E rows are F), C2 = L2 L2^T has
  // interface sweeps of its own, F^T is kept as CSR, and the inner rank-k2
  // correction enters through its square root Q2 = sq I + U2 diag(qd) U2^T.
  struct Inner {
    bool on = false;
    int64_t s1 = 0, s2 = 0;
    int32_t nb = 0;                 // connectors (blocks of C1)
    BlockArrays<double> Bd;
    BlockArrays<float> Bf;
    int32_t max_m = 0, max_lev = 0, max_level_bytes = 0;
    int64_t data_bytes = 0;
    SweepArrays<double> C2fd, C2bd;
    SweepArrays<float> C2ff, C2bf;
    std::vector<int32_t> f_lev_h, b_lev_h;
    int32_t f_nlev = 0, b_nlev = 0, f_group = 1, b_group = 1;
    bool one_wg = true;
    int64_t *ft_rp = nullptr;
    int32_t *ft_ci = nullptr;
    double *ft_v = nullptr;
    int32_t k2 = 0, steps = 0, nblk = 256;
    double theta2 = 0.0, sq = 1.0;
    double *U2 = nullptr, *U2rm = nullptr, *qd = nullptr;
    std::vector<double> lam_h, ritz_h;
    int64_t nnz_L1 = 0, nnz_L2 = 0;
  } ml;
  int32_t live_batches = 0;     // slr_batch objects on this context
  // numeric refactorisation (slr_refactor): the input pattern, the factor
  // plans and the coefficient maps, kept when opts.refactor is set
  struct Refactor {
    bool on = false;
    DevPool pool;
    std::vector<int64_t> tr_h;       // entry of A's mirror (j, i) of each entry (i, j)
    int64_t *tr = nullptr;
    double *stage = nullptr;         // pinned host staging of the values
    int64_t nnz = 0;
    double *val = nullptr;
    int *err = nullptr;
    int64_t *a_src = nullptr;
    struct Plan {
      int64_t *rp = nullptr;
      int32_t *ci = nullptr, *rows = nullptr;
      int64_t *src = nullptr;
      double *v = nullptr;
      int64_t nnz = 0;
      std::vector<int32_t> lev;
      int kind = 0;
    } fb, fc;
    struct Map {
      RfMap *m = nullptr;
      int64_t n = 0;
    } bdata, ev, tv, cfsc, cfw, cfw2, cbsc, cbw, cbw2;
  } rf;
  // stats
  slr_info info{};
  ApplyWS ws;
  // original <-> internal order scratch of slr_apply / slr_spmv
  DevPool ppool;
  int32_t pcap = 0;
  double *pr = nullptr, *pz = nullptr;
  // solve workspace
  DevPool spool;
  int32_t scap = 0;
  double *sX = nullptr, *sR = nullptr, *sZ = nullptr, *sP = nullptr, *sQ = nullptr, *sS = nullptr, *sB = nullptr;
  KState *sst = nullptr;
  double *spart = nullptr, *spart2 = nullptr;
  unsigned int *scnt = nullptr;
  // convergence polls of CG / FCG: two pinned slots of scap states each, and
  // the events that mark their copies done
  KState *hst = nullptr;
  int32_t hcap = 0;
  hipEvent_t pev[2] = {nullptr, nullptr};
  // FGMRES: per-step (converged, breakdown) flags of a cycle, pinned
  int *hfl = nullptr;
  int32_t hfl_cap = 0;
  // scratch of the Lanczos build, kept between builds
  KeptBuf lz;
  // scratch of FGMRES, kept between solves
  KeptBuf gm;
};

struct slr_batch {
  slr_ctx *c = nullptr;
  bool counted = false;         // included in c->live_batches
  int32_t cap = 0, method = SLR_PCG, maxit = 300;
  double rtol = 1e-8;
  DevPool pool;
  ApplyWS ws;
  double *X = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr, *S = nullptr, *B = nullptr;
  KState *st = nullptr;
  double *part = nullptr, *part2 = nullptr;
  unsigned int *counter = nullptr;
  int32_t it = 0;               // global iteration counter of the batch
  std::vector<int64_t> owner;   // request index per column, -1 free
  struct Req {
    int64_t tag;
    int32_t c0, nrhs;
    double *x_dev;
    bool live;
  };
  std::vector<Req> reqs;
  int32_t hi = 0;               // columns [0, hi) may be active
  std::vector<KState> st_h;
};

namespace {

constexpr int RED_NBLK = 512;   // blocks of the deterministic reductions

// The FGMRES workspace, carved from an Arena (or counted by ArenaCount).
struct FgmresWS {
  double *V, *Zb, *Bd, *X, *T, *Hm, *h1, *h2, *cs, *sn, *g, *y, *sc, *part;
  unsigned int *cnt;
  int *flags;
};
struct ArenaCount {
  size_t want = 0;
  template <typename T>
  T *alloc(size_t n) {
    want += (std::max<size_t>(n, 1) * sizeof(T) + 255) & ~(size_t)255;
    return nullptr;
  }
};
template <class AR>
void fgmres_layout(AR &a, int64_t n, int32_t mr, FgmresWS &w) {
  w.V = a.template alloc<double>((size_t)n * (mr + 1));
  w.Zb = a.template alloc<double>((size_t)n * mr);
  w.Bd = a.template alloc<double>(n);
  w.X = a.template alloc<double>(n);
  w.T = a.template alloc<double>(n);
  w.Hm = a.template alloc<double>((size_t)(mr + 1) * mr);
  w.h1 = a.template alloc<double>(mr + 1);
  w.h2 = a.template alloc<double>(mr + 1);
  w.cs = a.template alloc<double>(mr);
  w.sn = a.template alloc<double>(mr);
  w.g = a.template alloc<double>(mr + 1);
  w.y = a.template alloc<double>(mr);
  w.sc = a.template alloc<double>(4);
  w.part = a.template alloc<double>((size_t)RED_NBLK * (mr + 1));
  w.cnt = a.template alloc<unsigned int>(4);
  w.flags = a.template alloc<int>(2 * (size_t)mr);
}
int32_t fgmres_restart(int32_t restart) { return std::max(1, std::min(restart, 200)); }


// rank and chunk count the rank-k scratch of an apply must cover (the
// outer correction and, with the recursive interface solver, the inner one)
int32_t ws_rank(const slr_ctx *c) { return std::max({c->k, c->ml.k2, 1}); }
int32_t ws_chunks(const slr_ctx *c) { return std::max({c->lr_nblk, c->lrm_nblk, c->ml.on ? c->ml.nblk : 0}); }

int ws_ensure(slr_ctx *c, ApplyWS &w, int32_t nrhs) {
  const int32_t nb = ws_chunks(c), kk = ws_rank(c);
  if (w.cap >= nrhs && w.W && w.k >= kk && w.nblk >= nb && (!c->sep || w.Z)) return SLR_OK;
  w.pool.release();
  int32_t cap = std::max<int32_t>(nrhs, 1);
  w.W = w.pool.alloc<double>((size_t)std::max<int64_t>(c->s, 1) * cap);
  w.W2 = w.pool.alloc<double>((size_t)std::max<int64_t>(c->s, 1) * cap);
  w.lr_part = w.pool.alloc<double>((size_t)nb * cap * kk);
  w.cbuf = w.pool.alloc<double>((size_t)cap * kk);
  w.Z = c->sep ? w.pool.alloc<double>((size_t)std::max<int64_t>(c->m, 1) * cap) : nullptr;
  w.counter = w.pool.alloc<unsigned int>(16);
  if (!w.W || !w.W2 || !w.lr_part || !w.cbuf || !w.counter || (c->sep && !w.Z))
    return fail(SLR_ERR_OOM, "apply workspace");
  HIPCHK(hipMemset(w.counter, 0, 16 * sizeof(unsigned int)));
  w.cap = cap;
  w.k = kk;
  w.nblk = nb;
  return SLR_OK;
}

// Schedule of the persistent B launch for nrhs columns on nwg workgroups
// of `waves` waves with R columns of the largest subdomain: the items,
// longest first by the per-subdomain estimate, each given to the
// workgroup with the least work so far (longest-processing-time order).
// mode 1: items (subdomain, group of R columns); mode 2: each subdomain
// takes as many columns per item as its rows let the x region hold (at
// most one fewer than the waves, so that one wave stages, and 255).
// Kept per (mode, nrhs, R, nwg, waves).
const slr_ctx::BSched *b_schedule(slr_ctx *c, int32_t mode, int32_t nrhs, int32_t R, int32_t nwg, int32_t waves) {
  for (const auto &b : c->bsched)
    if (b.mode == mode && b.nrhs == nrhs && b.R == R && b.nwg == nwg && b.waves == waves) return &b;
  const int32_t p = c->p;
  std::vector<int32_t> items;
  if (mode == 1) {
    const int32_t ncg = (nrhs + R - 1) / R;
    for (int32_t g = 0; g < ncg; ++g)
      for (int32_t q = 0; q < p; ++q) items.push_back((g << 16) | q);
  } else {
    const int64_t cap = (int64_t)c->b_max_m * R;
    for (int32_t q = 0; q < p; ++q) {
      const int64_t mq = std::max<int64_t>(c->b_m_h[q], 1);
      const int32_t rq = (int32_t)std::max<int64_t>(1, std::min<int64_t>({cap / mq, std::max(waves - 1, 1), 255}));
      for (int32_t c0 = 0; c0 < nrhs; c0 += rq) {
        const int32_t rg = std::min(rq, nrhs - c0);
        items.push_back((int32_t)((uint32_t)q | ((uint32_t)c0 << 16) | ((uint32_t)rg << 24)));
      }
    }
  }
  std::stable_sort(items.begin(), items.end(),
                   [&](int32_t x, int32_t y) { return c->b_cost_h[x & 0xFFFF] > c->b_cost_h[y & 0xFFFF]; });
  std::vector<std::vector<int32_t>> per(nwg);
  std::priority_queue<std::pair<double, int32_t>, std::vector<std::pair<double, int32_t>>, std::greater<>> heap;
  for (int32_t w = 0; w < nwg; ++w) heap.emplace(0.0, w);
  for (int32_t it : items) {
    auto [load, w] = heap.top();
    heap.pop();
    per[w].push_back(it);
    heap.emplace(load + c->b_cost_h[it & 0xFFFF], w);
  }
  std::vector<int32_t> ptr(1, 0), flat;
  for (const auto &v : per) {
    flat.insert(flat.end(), v.begin(), v.end());
    ptr.push_back((int32_t)flat.size());
  }
  slr_ctx::BSched b;
  b.mode = mode;
  b.nrhs = nrhs;
  b.R = R;
  b.nwg = nwg;
  b.waves = waves;
  b.ptr = c->schedpool.upload(ptr);
  b.items = c->schedpool.upload(flat);
  if (!b.ptr || !b.items) return nullptr;
  c->bsched.push_back(b);
  return &c->bsched.back();
}

// LDS plan of the B kernel: right-hand sides per workgroup R and the
// staging buffer for the packed sweeps.  Total LDS = stage + pad16(x) +
// 16 (max_lev + 1).  R is the largest value (<= nrhs, <= 16) that still
// leaves a staging buffer of at least max(largest level, min(24 KiB,
// largest sweep)).  Returns false when not even R = 1 fits.
bool b_lds_plan_sz(int32_t max_m, int32_t max_lev, int32_t max_level_bytes, int64_t data_bytes, int32_t nrhs,
                   size_t tc_bytes, int32_t &R, int32_t &stage, size_t limit) {
  const int64_t fixed = 16 * (int64_t)(max_lev + 1) + kStageDummyBytes;
  // the fixed-width path double-buffers the stage: each half holds a level
  const int64_t need = std::max<int64_t>(2 * (int64_t)max_level_bytes, std::min<int64_t>(24576, data_bytes));
  for (int32_t r = std::min<int32_t>(std::max(nrhs, 1), 16); r >= 1; --r) {
    const int64_t xb = pad16h((int64_t)tc_bytes * (std::max(max_m, 1) * r + 1));
    const int64_t rest = ((int64_t)limit - fixed - xb) & ~int64_t(15);
    if (rest >= need) {
      R = r;
      stage = (int32_t)std::min<int64_t>(rest, pad16h(data_bytes));
      return true;
    }
  }
  return false;
}

bool b_lds_plan(const slr_ctx *c, int32_t nrhs, size_t tc_bytes, int32_t &R, int32_t &stage, size_t limit = 0) {
  return b_lds_plan_sz(c->b_max_m, c->b_max_lev, c->b_max_level_bytes, c->b_data_bytes, nrhs, tc_bytes, R, stage,
                       limit == 0 ? c->lds_limit : limit);
}

// With more subdomains than compute units and one right-hand side, the B
// kernel runs two workgroups per CU: half the threads (one solver wave,
// the rest staging) and at most half the LDS each, so that the second
// round of subdomains runs beside the first instead of after it.
template <typename TS, typename TC>
int run_bsolve(slr_ctx *c, const BlockArrays<TS> &B, const BArgs &a0, hipStream_t st) {
  BArgs a = a0;
  int32_t R = 0, stage = 0;
  int32_t threads = c->b_threads;
  const slr_ctx::BTune &tu = a.nrhs == 1 ? c->tune1 : c->tuneM;
  const bool pair = a.nrhs == 1 && (int64_t)c->p > (int64_t)c->n_cu;
  if (tu.threads > 0 && b_lds_plan(c, std::min(a.nrhs, tu.rmax), sizeof(TC), R, stage, c->lds_limit / tu.lds_div)) {
    threads = tu.threads;
  } else if (pair && b_lds_plan(c, a.nrhs, sizeof(TC), R, stage, c->lds_limit / 2)) {
    threads = c->b_threads / 2;
  } else if (!b_lds_plan(c, a.nrhs, sizeof(TC), R, stage)) {
    return fail(SLR_ERR_ARG, "a subdomain does not fit the LDS of one workgroup");
  }
  a.R = R;
  a.stage_bytes = stage;
  const size_t lds = (size_t)stage + kStageDummyBytes + pad16h((int64_t)sizeof(TC) * (c->b_max_m * R + 1)) +
                    16 * (size_t)(c->b_max_lev + 1);
  int32_t grid = c->p;
  if (tu.threads > 0 && tu.persistent) {
    // resident workgroups: by waves (32 per CU) and by LDS
    const int32_t per_cu = std::max<int32_t>(1, std::min<int32_t>(2048 / threads, (int32_t)(c->lds_limit / lds)));
    const int32_t nwg = c->n_cu * per_cu;
    const int32_t ncg = (a.nrhs + R - 1) / R;
    const int32_t mode = tu.persistent == 2 && a.nrhs <= 255 ? 2 : 1;
    if ((int64_t)c->p * ncg > nwg && c->p <= 65535 && ncg <= 32767) {
      const slr_ctx::BSched *sc = b_schedule(c, mode, a.nrhs, R, nwg, threads / 64);
      if (!sc) return fail(SLR_ERR_OOM, "persistent schedule");
      a.sched = sc->items;
      a.sched_ptr = sc->ptr;
      a.var_cols = mode == 2 ? 1 : 0;
      grid = nwg;
    }
  }
  launch_bsolve<TS, TC>(B, grid, a, threads, lds, st);
  return SLR_OK;
}

// B kernel dispatch by (storage, compute) precision
int bsolve(slr_ctx *c, const BArgs &a, bool compute64, hipStream_t st) {
  if (c->fact_prec == SLR_FP64) return run_bsolve<double, double>(c, c->Bd, a, st);
  if (compute64) return run_bsolve<float, double>(c, c->Bf, a, st);
  return run_bsolve<float, float>(c, c->Bf, a, st);
}

void csweep(slr_ctx *c, bool fwd, double *x, int64_t ldx, int32_t nrhs, bool compute64, hipStream_t st) {
  const int32_t nlev = fwd ? c->cf_nlev : c->cb_nlev;
  const int32_t *lev = fwd ? c->cf_lev_h.data() : c->cb_lev_h.data();
  const int32_t G = fwd ? c->cf_group : c->cb_group;
  if (c->fact_prec == SLR_FP64) {
    launch_sweep<double, double>(fwd ? c->Cfd : c->Cbd, lev, nlev, (int32_t)c->s, x, ldx, nrhs, c->c_one_wg, st, G);
  } else if (compute64) {
    launch_sweep<float, double>(fwd ? c->Cff : c->Cbf, lev, nlev, (int32_t)c->s, x, ldx, nrhs, c->c_one_wg, st, G);
  } else {
    launch_sweep<float, float>(fwd ? c->Cff : c->Cbf, lev, nlev, (int32_t)c->s, x, ldx, nrhs, c->c_one_wg, st, G);
  }
}

// out-of-place two-level interface sweep (multicolour schedules)
void csweep2(slr_ctx *c, bool fwd, const double *x, int64_t ldx, double *y, int64_t ldy, int32_t nrhs,
             bool compute64, hipStream_t st, const double *dv = nullptr, double *dpart = nullptr) {
  const int32_t s = (int32_t)c->s;
  if (c->fact_prec == SLR_FP64)
    launch_sweep2<double, double>(fwd ? c->Cfd : c->Cbd, s, x, ldx, y, ldy, nrhs, st, dv, dpart);
  else if (compute64)
    launch_sweep2<float, double>(fwd ? c->Cff : c->Cbf, s, x, ldx, y, ldy, nrhs, st, dv, dpart);
  else
    launch_sweep2<float, float>(fwd ? c->Cff : c->Cbf, s, x, ldx, y, ldy, nrhs, st, dv, dpart);
}

// ---- recursive interface solver (Sec. 5.2) --------------------------------
// C1 solves: the B kernel over the connectors (sweeps: 1 = L1^{-1} only,
// 2 = L1^{-T} only, 3 = both); a quarter of the LDS per workgroup when the
// connectors fit it, so that several share a compute unit.
int c1solve(slr_ctx *c, BArgs a, int32_t sweeps, bool compute64, hipStream_t st) {
  const slr_ctx::Inner &I = c->ml;
  a.sweeps = sweeps;
  const size_t tcb = (c->fact_prec == SLR_FP64 || compute64) ? 8 : 4;
  int32_t R = 0, stage = 0;
  if (!b_lds_plan_sz(I.max_m, I.max_lev, I.max_level_bytes, I.data_bytes, a.nrhs, tcb, R, stage, c->lds_limit / 4) &&
      !b_lds_plan_sz(I.max_m, I.max_lev, I.max_level_bytes, I.data_bytes, a.nrhs, tcb, R, stage, c->lds_limit))
    return fail(SLR_ERR_ARG, "a connector does not fit the LDS of one workgroup");
  a.R = R;
  a.stage_bytes = stage;
  const size_t lds = (size_t)stage + kStageDummyBytes + pad16h((int64_t)tcb * ((int64_t)I.max_m * R + 1)) +
                     16 * (size_t)(I.max_lev + 1);
  const int32_t threads = 256;
  if (c->fact_prec == SLR_FP64)
    launch_bsolve<double, double>(I.Bd, I.nb, a, threads, lds, st);
  else if (compute64)
    launch_bsolve<float, double>(I.Bf, I.nb, a, threads, lds, st);
  else
    launch_bsolve<float, float>(I.Bf, I.nb, a, threads, lds, st);
  return SLR_OK;
}

// x <- L2^{-1} x (fwd) or L2^{-T} x over the inner interface, in place
void c2sweep(slr_ctx *c, bool fwd, double *x, int64_t ldx, int32_t nrhs, bool compute64, hipStream_t st) {
  const slr_ctx::Inner &I = c->ml;
  const int32_t nlev = fwd ? I.f_nlev : I.b_nlev;
  const int32_t *lev = fwd ? I.f_lev_h.data() : I.b_lev_h.data();
  const int32_t G = fwd ? I.f_group : I.b_group;
  const int32_t s2 = (int32_t)I.s2;
  if (c->fact_prec == SLR_FP64)
    launch_sweep<double, double>(fwd ? I.C2fd : I.C2bd, lev, nlev, s2, x, ldx, nrhs, I.one_wg, st, G);
  else if (compute64)
    launch_sweep<float, double>(fwd ? I.C2ff : I.C2bf, lev, nlev, s2, x, ldx, nrhs, I.one_wg, st, G);
  else
    launch_sweep<float, float>(fwd ? I.C2ff : I.C2bf, lev, nlev, s2, x, ldx, nrhs, I.one_wg, st, G);
}

// x <- Q2 x = sq x + U2 diag(qd) U2^T x over the inner interface, in place
void q2(slr_ctx *c, double *x, int64_t ldx, int32_t nrhs, ApplyWS &w, hipStream_t st) {
  const slr_ctx::Inner &I = c->ml;
  launch_lowrank_rm<double>(I.U2rm, I.U2, I.s2, I.k2, I.qd, I.sq, x, ldx, x, ldx, nrhs, w.lr_part, I.nblk, w.cbuf,
                            st);
}

// x <- K^T x (in place of L^{-1} x; x: s x nrhs):
//   a1 = L1^{-1} x1,  x2 <- Q2 L2^{-1} (x2 - F^T L1^{-T} a1)
// scr: s1 x nrhs scratch (leading dimension lds).
int c_lower(slr_ctx *c, double *x, int64_t ldx, int32_t nrhs, bool compute64, double *scr, int64_t lds, ApplyWS &w,
            hipStream_t st) {
  const slr_ctx::Inner &I = c->ml;
  BArgs a;
  a.f = x; a.ldf = ldx; a.a_f = 1.0;
  a.u = x; a.ldu = ldx;
  a.nrhs = nrhs;
  int rc = c1solve(c, a, 1, compute64, st);
  if (rc) return rc;
  a.u = scr; a.ldu = lds;
  if ((rc = c1solve(c, a, 2, compute64, st))) return rc;
  launch_spmv_axpby(I.s2, I.ft_rp, I.ft_ci, I.ft_v, scr, lds, x + I.s1, ldx, nrhs, 1.0, -1.0, st);
  c2sweep(c, true, x + I.s1, ldx, nrhs, compute64, st);
  q2(c, x + I.s1, ldx, nrhs, w, st);
  return SLR_OK;
}

// x <- K x (in place of L^{-T} x):
//   x2 <- L2^{-T} Q2 x2,  x1 <- L1^{-T} (x1 - L1^{-1} F x2)
int c_upper(slr_ctx *c, double *x, int64_t ldx, int32_t nrhs, bool compute64, double *scr, int64_t lds, ApplyWS &w,
            hipStream_t st) {
  const slr_ctx::Inner &I = c->ml;
  q2(c, x + I.s1, ldx, nrhs, w, st);
  c2sweep(c, false, x + I.s1, ldx, nrhs, compute64, st);
  BArgs a;
  a.y = x + I.s1; a.ldy = ldx; a.b_y = 1.0;
  a.u = scr; a.ldu = lds;
  a.nrhs = nrhs;
  int rc = c1solve(c, a, 1, compute64, st);
  if (rc) return rc;
  launch_axpby(I.s1, nrhs, -1.0, scr, lds, 1.0, x, ldx, st);
  BArgs b;
  b.f = x; b.ldf = ldx; b.a_f = 1.0;
  b.u = x; b.ldu = ldx;
  b.nrhs = nrhs;
  return c1solve(c, b, 2, compute64, st);
}

void lowrank(slr_ctx *c, ApplyWS &w, const double *win, int64_t ldw, double *wout, int64_t ldo, int32_t nrhs,
             hipStream_t st) {
  const int k = c->k;
  switch (c->uk_prec) {
    case SLR_FP64:
      launch_lowrank_rm<double>((const double *)c->Urm, (const double *)c->U, c->s, k, c->dsc, c->rho, win, ldw,
                                wout, ldo, nrhs, w.lr_part, c->lr_nblk, w.cbuf, st);
      break;
    case SLR_FP32:
      launch_lowrank_rm<float>((const float *)c->Urm, (const float *)c->U, c->s, k, c->dsc, c->rho, win, ldw,
                               wout, ldo, nrhs, w.lr_part, c->lr_nblk, w.cbuf, st);
      break;
    default:
      // BF16 U_k always takes the matrix-core kernels, so that a column's
      // arithmetic never depends on how many columns share the launch
      if (k > 0)
        launch_lowrank_mfma((const __hip_bfloat16 *)c->U, (const __hip_bfloat16 *)c->Urm, c->s, k, c->dsc, c->rho,
                            win, ldw, wout, ldo, nrhs, w.lr_part, c->lrm_nblk, w.cbuf, st);
      else
        launch_axpby(c->s, nrhs, c->rho, win, ldw, 0.0, wout, ldo, st);
  }
}

// First B solve of the apply: W = g - E^T B^{-1} f for nrhs columns of r
// (ld ldr), into w.W (ld s).  Vertex-based partitions: the B kernel's
// epilogue; with separator nodes the B kernel leaves z = B^{-1} f in w.Z and
// W = g - E^T z follows as a CSR product over all interface rows.
int bsolve_first(slr_ctx *c, ApplyWS &w, const double *r, int64_t ldr, int32_t nrhs, hipStream_t st) {
  const int64_t m = c->m, s = c->s;
  BArgs a;
  a.f = r; a.ldf = ldr; a.a_f = 1.0;
  a.nrhs = nrhs;
  if (!c->sep) {
    a.g = r + m; a.ldg = ldr; a.c_g = 1.0;
    a.gout = w.W; a.ldgo = s; a.d_t = -1.0;
    return bsolve(c, a, false, st);
  }
  a.u = w.Z; a.ldu = m;
  int rc = bsolve(c, a, false, st);
  if (rc) return rc;
  launch_axpby(s, nrhs, 1.0, r + m, ldr, 0.0, w.W, s, st);
  launch_spmv_axpby(s, c->et_rp, c->et_ci, c->et_v, w.Z, m, w.W, s, nrhs, 1.0, -1.0, st);
  return SLR_OK;
}

// z = M^{-1} r in the internal order, eq. M with S~^{-1} of eq. skt:
//   (1) z_B = B^{-1} f ; W = g - E^T z_B          (B kernel, epilogue)
//   (2) W <- L^{-1} W                              (interface forward sweep)
//   (3) y' = rho W + U_k D U_k^T W                 (rank-k block)
//   (4) y = L^{-T} y'                              (interface backward sweep)
//   (5) u = B^{-1}(f - E y)                        (B kernel, prologue)
// With the recursive interface solver K^T and K take the place of L^{-1}
// and L^{-T} in (2) and (4).
int apply_dd(slr_ctx *c, ApplyWS &w, const double *r, int64_t ldr, double *z, int64_t ldz, int32_t nrhs,
             hipStream_t st) {
  if (nrhs <= 0) return SLR_OK;
  int rc = ws_ensure(c, w, nrhs);
  if (rc) return rc;
  const int64_t m = c->m, s = c->s;
  if (s > 0) {
    if ((rc = bsolve_first(c, w, r, ldr, nrhs, st))) return rc;
    if (c->ml.on) {
      if ((rc = c_lower(c, w.W, s, nrhs, false, w.W2, s, w, st))) return rc;
      lowrank(c, w, w.W, s, z + m, ldz, nrhs, st);
      if ((rc = c_upper(c, z + m, ldz, nrhs, false, w.W2, s, w, st))) return rc;
    } else if (c->c_two_level) {
      csweep2(c, true, w.W, s, w.W2, s, nrhs, false, st);
      lowrank(c, w, w.W2, s, w.W, s, nrhs, st);
      csweep2(c, false, w.W, s, z + m, ldz, nrhs, false, st);
    } else {
      csweep(c, true, w.W, s, nrhs, false, st);
      lowrank(c, w, w.W, s, z + m, ldz, nrhs, st);
      csweep(c, false, z + m, ldz, nrhs, false, st);
    }
  }
  if (m > 0) {
    BArgs a;
    a.f = r; a.ldf = ldr; a.a_f = 1.0;
    a.y = z + m; a.ldy = ldz; a.b_y = (s > 0) ? -1.0 : 0.0;
    a.u = z; a.ldu = ldz;
    a.nrhs = nrhs;
    if ((rc = bsolve(c, a, false, st))) return rc;
  }
  return SLR_OK;
}

// out = E^T B^{-1} E t for one interface vector (FP64 arithmetic on the
// stored factors); with separator nodes through c->ws.Z and the E^T CSR.
int bsolve_et(slr_ctx *c, const double *t, double *out, hipStream_t st) {
  const int64_t s = c->s;
  BArgs a;
  a.y = t; a.ldy = s; a.b_y = 1.0;
  a.nrhs = 1;
  if (!c->sep) {
    a.gout = out; a.ldgo = s; a.d_t = 1.0;
    return bsolve(c, a, true, st);
  }
  a.u = c->ws.Z; a.ldu = c->m;
  int rc = bsolve(c, a, true, st);
  if (rc) return rc;
  launch_spmv_axpby(s, c->et_rp, c->et_ci, c->et_v, c->ws.Z, c->m, out, s, 1, 0.0, 1.0, st);
  return SLR_OK;
}

// w = H v = L^{-1} E^T B^{-1} E L^{-T} v (eq. H), FP64 arithmetic on the
// stored factors; t: s-vector scratch.
// w = H v.  With dv and a two-level interface schedule, the last sweep also
// leaves the per-block partial sums of dv . w in dpart and *ndp receives
// their count (0 otherwise).  t_ready (two-level schedules): t already
// holds L^{-T} v (computed with the previous Lanczos step's end).
int apply_H(slr_ctx *c, const double *v, double *w, double *t, double *t2, hipStream_t st,
            const double *dv = nullptr, double *dpart = nullptr, int32_t *ndp = nullptr, bool t_ready = false) {
  if (ndp) *ndp = 0;
  const int64_t s = c->s;
  if (c->ml.on) {
    // H = K^T E^T B^{-1} E K (t2: scratch of the interface solves)
    launch_axpby(s, 1, 1.0, v, s, 0.0, t, s, st);
    int rc = c_upper(c, t, s, 1, true, t2, s, c->ws, st);
    if (rc) return rc;
    if ((rc = bsolve_et(c, t, w, st))) return rc;
    return c_lower(c, w, s, 1, true, t2, s, c->ws, st);
  }
  if (c->c_two_level) {
    if (!t_ready) csweep2(c, false, v, s, t, s, 1, true, st);
  } else {
    launch_axpby(s, 1, 1.0, v, s, 0.0, t, s, st);
    csweep(c, false, t, s, 1, true, st);
  }
  int rc = bsolve_et(c, t, c->c_two_level ? t2 : w, st);
  if (rc) return rc;
  if (c->c_two_level) {
    csweep2(c, true, t2, s, w, s, 1, true, st, dv, dpart);
    if (dv && ndp) *ndp = (int32_t)((s + 255) / 256);
  } else {
    csweep(c, true, w, s, 1, true, st);
  }
  return SLR_OK;
}

template <typename TU>
int upload_lowrank_T(slr_ctx *c, hipStream_t st) {
  TU *U = c->lrpool.alloc<TU>((size_t)c->s * c->k);
  if (!U) return fail(SLR_ERR_OOM, "U storage");
  launch_round_copy<TU>((int64_t)c->s * c->k, c->U64, U, st);
  c->U = U;
  return SLR_OK;
}

template <typename TU>
int upload_lowrank_rm(slr_ctx *c, hipStream_t st) {
  int32_t ldk;
  const int64_t ng = lr_rm_groups<TU>(c->s, c->k, ldk);
  const int64_t n = ng * 64 * (16 / (int64_t)sizeof(TU));
  // chunks of U^T w: about 128 row groups each (a few rounds of loads per
  // wave), at least 256 and at most 2048 (the fold reads chunks x k)
  c->lr_nblk = c->lr_nblk_tuned > 0 ? c->lr_nblk_tuned
                                     : (int32_t)std::min<int64_t>(2048, std::max<int64_t>(256, ng / 128));
  TU *U = c->lrpool.alloc<TU>((size_t)n);
  if (!U) return fail(SLR_ERR_OOM, "U storage");
  launch_lr_to_rm<TU>(c->U64, c->s, c->k, U, st);
  c->Urm = U;
  return SLR_OK;
}

int finish_lowrank(slr_ctx *c, hipStream_t st) {
  // scales of eq. skt: (1 - lambda_i)^{-1} - (1 - theta)^{-1}; under the
  // eq. Lambda-2 form rho = 1 and eps (1 - lambda_i)^{-1} - 1
  const bool eps_mode = c->opts.theta_mode == SLR_THETA_EPS;
  if (eps_mode) c->theta = 0.0;
  if (std::fabs(1.0 - c->theta) < 1e-12) return fail(SLR_ERR_RITZ_SINGULAR, "|1 - theta| < 1e-12");
  c->rho = 1.0 / (1.0 - c->theta);
  std::vector<double> d(std::max(c->k, 1), 0.0);
  for (int i = 0; i < c->k; ++i) {
    if (std::fabs(1.0 - c->lam_h[i]) < 1e-12) return fail(SLR_ERR_RITZ_SINGULAR, "|1 - lambda_i| < 1e-12");
    d[i] = eps_mode ? c->opts.eps / (1.0 - c->lam_h[i]) - 1.0 : 1.0 / (1.0 - c->lam_h[i]) - c->rho;
  }
  c->dsc = c->lrpool.upload(d);
  if (!c->dsc) return fail(SLR_ERR_OOM, "dsc");
  if (c->k == 0) return SLR_OK;
  c->Urm = nullptr;
  if (c->uk_prec == SLR_FP64) {
    c->U = c->U64;
    return upload_lowrank_rm<double>(c, st);
  }
  if (c->uk_prec == SLR_FP32) {
    const int rc = upload_lowrank_T<float>(c, st);
    return rc ? rc : upload_lowrank_rm<float>(c, st);
  }
  // BF16: the two tile layouts of the matrix-core kernels (U: U^T W, Urm: update)
  const int64_t ne = lr_tile_entries(c->s, c->k);
  __hip_bfloat16 *Upt = c->lrpool.alloc<__hip_bfloat16>((size_t)ne);
  __hip_bfloat16 *Uup = c->lrpool.alloc<__hip_bfloat16>((size_t)ne);
  if (!Upt || !Uup) return fail(SLR_ERR_OOM, "U storage");
  launch_lr_to_tiles(c->U64, c->s, c->k, Upt, Uup, st);
  c->U = Upt;
  c->Urm = Uup;
  return SLR_OK;
}

// Lanczos on H with CGS2 full reorthogonalisation (Sec. 5.1), then the
// tridiagonal eigensolve and the Ritz vectors U_k = V_m Y_k.  With k0 > 0
// the first k0 columns of c->U64 (and of c->lam_h) are kept and the run is
// deflated (Sec. 5.3): the start vector and every Gram-Schmidt pass are
// orthogonalised against them too, and up to kw new Ritz pairs are appended.
// The new U64 lives in a fresh pool that replaces c->lrpool only on success,
// so a failed growth leaves the resident low-rank part as it was.
// End of Lanczos step j: beta_j, v_{j+1} = w / beta_j (when vnext) and the
// recorded coefficients; with a two-level interface schedule the next
// step's first sweep t = L^{-T} v_{j+1} is computed in the same launch.
void lanczos_step_end(slr_ctx *c, int32_t j, const double *w, double *vnext, double *sc, double *al, double *be,
                      const double *bpart, int32_t rb, const double *aval, double *t, hipStream_t st) {
  if (vnext && c->c_two_level) {
    if (c->fact_prec == SLR_FP64)
      launch_lanczos_next_sweep<double>(c->s, j, w, vnext, sc, al, be, bpart, rb, aval, c->Cbd, c->cb_nnz, t, st);
    else
      launch_lanczos_next_sweep<float>(c->s, j, w, vnext, sc, al, be, bpart, rb, aval, c->Cbf, c->cb_nnz, t, st);
  } else {
    launch_lanczos_next(c->s, j, w, vnext, sc, al, be, bpart, rb, aval, st);
  }
}

int lanczos_build(slr_ctx *c, int32_t kw, int32_t k0, const double *v0_host, hipStream_t st) {
  const int64_t s = c->s;
  int32_t steps = c->opts.lanczos_steps > 0 ? c->opts.lanczos_steps : 5 * kw;
  steps = (int32_t)std::min<int64_t>(steps, std::max<int64_t>(s - k0, 1));
  if (k0 + steps > 1024) return fail(SLR_ERR_ARG, "at most 1024 Lanczos steps plus kept vectors");
  const bool need_k1 = c->opts.theta_mode == SLR_THETA_LAMBDA_K1;
  const bool lam_s = c->opts.theta_mode == SLR_THETA_LAMBDA_S;
  const int32_t nb = k0 + steps;   // basis columns: kept vectors, then the Lanczos vectors
  const bool pro = c->opts.reorth == SLR_REORTH_PARTIAL && k0 == 0;
  Arena tmp(c->lz);
  double *V = tmp.alloc<double>((size_t)s * nb);
  double *Wl = tmp.alloc<double>(s);
  double *T = tmp.alloc<double>(s);
  double *T2 = tmp.alloc<double>(s);
  double *h = tmp.alloc<double>(2048);
  double *sc = tmp.alloc<double>(4);
  double *al = tmp.alloc<double>(steps);
  double *be = tmp.alloc<double>(steps);
  double *part = tmp.alloc<double>((size_t)RED_NBLK * (nb + 1));
  double *part2 = tmp.alloc<double>((size_t)(s + 255) / 256 + 1);
  unsigned int *cnt = tmp.alloc<unsigned int>(4);
  // partial reorthogonalisation state: three omega rows, and per step the
  // force flag, the running ||T|| and the decision
  const int32_t ld_om = steps + 2;
  double *om = tmp.alloc<double>((size_t)3 * ld_om);
  int *frc = tmp.alloc<int>(steps + 1);
  double *tn = tmp.alloc<double>(steps + 1);
  int *rflag = tmp.alloc<int>(steps);
  if (!V || !Wl || !T || !T2 || !h || !sc || !al || !be || !part || !part2 || !cnt || !om || !frc || !tn || !rflag) {
    tmp.release();
    return fail(SLR_ERR_OOM, "Lanczos basis");
  }
  int rc = SLR_OK;
  auto bail = [&](int code) {
    tmp.release();
    return code;
  };
  HIPCHK(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned int), st));
  HIPCHK(hipMemsetAsync(sc, 0, 4 * sizeof(double), st));
  HIPCHK(hipMemsetAsync(frc, 0, sizeof(int) * (steps + 1), st));
  HIPCHK(hipMemsetAsync(tn, 0, sizeof(double) * (steps + 1), st));
  HIPCHK(hipMemsetAsync(rflag, 0, sizeof(int) * steps, st));
  // start vector: interface entries of v0 (original order), normalised
  std::vector<double> v0(s);
  for (int64_t q = 0; q < s; ++q) v0[q] = v0_host[c->perm_h[c->m + q]];
  double nv = 0.0;
  for (double x : v0) nv += x * x;
  nv = std::sqrt(nv);
  if (!(nv > 0.0)) return bail(fail(SLR_ERR_ARG, "Lanczos start vector is zero on the interface"));
  for (double &x : v0) x /= nv;
  double *V0 = V + (int64_t)k0 * s;
  if (k0 > 0) {
    // kept vectors first; the start vector loses its components along them
    // (two passes) and is normalised again; its norm is checked afterwards
    HIPCHK(hipMemcpyAsync(V, c->U64, sizeof(double) * s * k0, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(Wl, v0.data(), sizeof(double) * s, hipMemcpyHostToDevice, st));
    int32_t rb = 0;
    for (int pass = 0; pass < 2; ++pass) {
      const int32_t rbh = launch_multidot_partial(s, k0, V, s, Wl, part, RED_NBLK, st);
      rb = launch_gemv_sub_fold(s, k0, V, s, part, rbh, Wl, nullptr, pass == 1 ? part2 : nullptr, st);
    }
    launch_lanczos_next(s, 0, Wl, V0, sc, sc + 2, sc + 3, part2, rb, nullptr, st);
  } else {
    HIPCHK(hipMemcpyAsync(V0, v0.data(), sizeof(double) * s, hipMemcpyHostToDevice, st));
  }
  // All steps are queued without host round-trips.  The stopping test
  // (beta_j <= 1e-14 ||T_j||_inf) is applied afterwards to the recorded
  // coefficients: steps after a breakdown only produce basis columns that
  // are never used.
  // Step j: w = H v_j; two classical Gram-Schmidt passes against
  // [kept vectors, v_0 .. v_j].  The first pass's coefficient on v_j is
  // v_j . H v_j = alpha_j (it also removes the beta_{j-1} v_{j-1} term), so
  // the three-term recurrence is subsumed by the full reorthogonalisation.
  for (int32_t j = 0; j < steps && pro; ++j) {
    // partial reorthogonalisation: three-term step, then one Gram-Schmidt
    // pass against v_0 .. v_j whose kernels first take the omega-recurrence
    // decision and return at once when the step is not cleaned; beta_j is
    // folded from whichever kernel wrote the ||w||^2 partials last
    double *vj = V0 + (int64_t)j * s;
    // alpha_j = v_j . H v_j: partial sums from the last interface sweep when
    // it can give them, else a separate reduction
    int32_t rba = 0;
    if ((rc = apply_H(c, vj, Wl, T, T2, st, vj, part, &rba, j > 0))) return bail(rc);
    if (rba == 0) rba = launch_multidot_partial(s, 1, vj, s, Wl, part, RED_NBLK, st);
    const int32_t rb = launch_lanczos_axpy(s, Wl, vj, j > 0 ? vj - s : nullptr, sc, part, rba, part2, st);
    const int32_t rbh = launch_multidot_pro(s, j + 1, V0, s, Wl, part, RED_NBLK, j, al, be, sc, part2, rb, om, ld_om,
                                            frc, tn, rflag, st);
    launch_gemv_sub_fold(s, j + 1, V0, s, part, rbh, Wl, nullptr, part2, st, rflag + j);
    lanczos_step_end(c, j, Wl, j + 1 < steps ? vj + s : nullptr, sc, al, be, part2, rb, nullptr, T, st);
  }
  for (int32_t j = 0; j < steps && !pro; ++j) {
    double *vj = V0 + (int64_t)j * s;
    if ((rc = apply_H(c, vj, Wl, T, T2, st, nullptr, nullptr, nullptr, j > 0))) return bail(rc);
    const int32_t J = k0 + j + 1;
    int32_t rb = 0;
    for (int pass = 0; pass < 2; ++pass) {
      // coefficients V^T w as row-chunk partials, folded inside the update
      // (the first pass's coefficients go to h: h[k0 + j] = alpha_j); the
      // second pass also leaves the partial sums of ||w||^2 in part2
      const int32_t rbh = launch_multidot_partial(s, J, V, s, Wl, part, RED_NBLK, st);
      rb = launch_gemv_sub_fold(s, J, V, s, part, rbh, Wl, pass == 0 ? h : nullptr, pass == 1 ? part2 : nullptr, st);
    }
    lanczos_step_end(c, j, Wl, j + 1 < steps ? vj + s : nullptr, sc, al, be, part2, rb, h + k0 + j, T, st);
  }
  std::vector<double> ah(steps), bh(steps);
  double start_norm = 1.0;
  HIPCHK(hipMemcpyAsync(ah.data(), al, sizeof(double) * steps, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(bh.data(), be, sizeof(double) * steps, hipMemcpyDeviceToHost, st));
  if (k0 > 0) HIPCHK(hipMemcpyAsync(&start_norm, sc + 3, sizeof(double), hipMemcpyDeviceToHost, st));
  std::vector<int> rf(steps, 0);
  if (pro) HIPCHK(hipMemcpyAsync(rf.data(), rflag, sizeof(int) * steps, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (!(start_norm > 1e-12)) return bail(fail(SLR_ERR_ARG, "start vector lies in the span of U_k"));
  std::vector<double> alpha_h, beta_h;
  double tnorm = 0.0, bprev = 0.0;
  int32_t mm = 0;
  for (int32_t j = 0; j < steps; ++j) {
    if (!std::isfinite(ah[j]) || !std::isfinite(bh[j]))
      return bail(fail(SLR_ERR_BREAKDOWN, "non-finite Lanczos coefficients"));
    alpha_h.push_back(ah[j]);
    beta_h.push_back(bh[j]);
    mm = j + 1;
    tnorm = std::max(tnorm, std::fabs(ah[j]) + bh[j] + bprev);
    bprev = bh[j];
    if (bh[j] <= 1e-14 * tnorm) break;
  }
  int32_t nre = pro ? 0 : mm;
  for (int32_t j = 0; pro && j < mm; ++j) nre += rf[j] != 0;
  const int32_t need = need_k1 || lam_s ? kw + 1 : kw;
  if (mm < need) return bail(fail(SLR_ERR_LANCZOS_SHORT, "Lanczos produced fewer Ritz pairs than needed"));
  double *Z = tmp.alloc<double>((size_t)6 * mm * std::max(kw, 1));   // eigensolver scratch
  double *ev = tmp.alloc<double>(mm);
  double *Y = tmp.alloc<double>((size_t)mm * std::max(kw, 1));
  int *info = tmp.alloc<int>(1);
  if (!Z || !ev || !Y || !info) return bail(fail(SLR_ERR_OOM, "eigensolve"));
  launch_tridiag_eig(mm, al, be, Z, ev, Y, kw, info, st);
  DevPool nl;
  double *U64 = nl.alloc<double>((size_t)s * std::max(k0 + kw, 1));
  if (!U64) return bail(fail(SLR_ERR_OOM, "U"));
  if (k0 > 0) HIPCHK(hipMemcpyAsync(U64, V, sizeof(double) * s * k0, hipMemcpyDeviceToDevice, st));
  launch_ritz<double>(s, mm, kw, V0, s, Y, U64 + (int64_t)k0 * s, U64 + (int64_t)k0 * s, st);
  int info_h = 0;
  std::vector<double> ritz(mm, 0.0);
  HIPCHK(hipMemcpyAsync(&info_h, info, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ritz.data(), ev, sizeof(double) * mm, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  tmp.release();
  if (info_h) {
    nl.release();
    return fail(SLR_ERR_BREAKDOWN, "tridiagonal eigensolve did not converge");
  }
  // eq. condk: keep the new Ritz values above 1 - 1/K (at most kw); the
  // first k' new columns are the Ritz vectors of the k' largest values
  int32_t kk = kw;
  if (c->opts.cond_K > 1.0) {
    const double cut = 1.0 - 1.0 / c->opts.cond_K;
    kk = 0;
    while (kk < kw && ritz[kk] > cut) ++kk;
  }
  std::vector<double> lam(c->lam_h.begin(), c->lam_h.begin() + k0);
  lam.insert(lam.end(), ritz.begin(), ritz.begin() + kk);
  // commit: the new basis replaces the old low-rank part
  c->lrpool.release();
  c->lrpool = nl;
  c->U64 = U64;
  c->U = nullptr;
  c->Urm = nullptr;
  c->dsc = nullptr;
  c->k = k0 + kk;
  c->lam_h = lam;
  c->ritz_h = ritz;
  c->alpha_h = alpha_h;
  c->beta_h = beta_h;
  c->theta = need_k1 ? ritz[kk] : lam_s ? ritz[mm - 1] : 0.0;
  c->info.lanczos_steps = mm;
  c->info.lanczos_reorth = nre;
  return finish_lowrank(c, st);
}

// The recursive interface solver's inner low-rank part (Sec. 5.2 with
// Sec. 5.1 one level down): Lanczos with full reorthogonalisation (two
// classical Gram-Schmidt passes every step) on
//   H2 = L2^{-1} F^T C1^{-1} F L2^{-T}
// from the start vector's entries on the inner interface, the k2 largest
// Ritz pairs, theta2 = lambda_{k2+1}, and the square root Q2 of
// G2 = rho2 I + U2 D2 U2^T (eq. skt): sq = rho2^{1/2}, qd_i =
// (1 - lambda_i)^{-1/2} - sq.  G2 must be positive definite.
int lanczos_inner(slr_ctx *c, const double *v0_host, hipStream_t st) {
  slr_ctx::Inner &I = c->ml;
  const int64_t s1 = I.s1, s2 = I.s2;
  const int32_t kw = I.k2;
  I.theta2 = 0.0;
  I.sq = 1.0;
  I.steps = 0;
  if (kw == 0) {
    I.qd = c->pool.upload(std::vector<double>(1, 0.0));
    return I.qd ? SLR_OK : fail(SLR_ERR_OOM, "inner scales");
  }
  int32_t steps = c->opts.lanczos_steps2 > 0 ? c->opts.lanczos_steps2 : 5 * kw;
  steps = (int32_t)std::min<int64_t>(steps, std::max<int64_t>(s2, 1));
  if (steps > 1024) return fail(SLR_ERR_ARG, "at most 1024 inner Lanczos steps");
  Arena tmp(c->lz);
  double *V = tmp.alloc<double>((size_t)s2 * steps);
  double *Wl = tmp.alloc<double>(s2);
  double *T = tmp.alloc<double>(s2);
  double *Tu = tmp.alloc<double>(s1);
  double *h = tmp.alloc<double>(2048);
  double *sc = tmp.alloc<double>(4);
  double *al = tmp.alloc<double>(steps);
  double *be = tmp.alloc<double>(steps);
  double *part = tmp.alloc<double>((size_t)RED_NBLK * (steps + 1));
  double *part2 = tmp.alloc<double>((size_t)(s2 + 255) / 256 + 1);
  if (!V || !Wl || !T || !Tu || !h || !sc || !al || !be || !part || !part2) {
    tmp.release();
    return fail(SLR_ERR_OOM, "inner Lanczos basis");
  }
  auto bail = [&](int code) {
    tmp.release();
    return code;
  };
  HIPCHK(hipMemsetAsync(sc, 0, 4 * sizeof(double), st));
  std::vector<double> v0(s2);
  for (int64_t q = 0; q < s2; ++q) v0[q] = v0_host[c->perm_h[c->m + s1 + q]];
  double nv = 0.0;
  for (double x : v0) nv += x * x;
  nv = std::sqrt(nv);
  if (!(nv > 0.0)) return bail(fail(SLR_ERR_ARG, "Lanczos start vector is zero on the inner interface"));
  for (double &x : v0) x /= nv;
  HIPCHK(hipMemcpyAsync(V, v0.data(), sizeof(double) * s2, hipMemcpyHostToDevice, st));
  int rc = SLR_OK;
  for (int32_t j = 0; j < steps; ++j) {
    double *vj = V + (int64_t)j * s2;
    // w = H2 v_j: T = L2^{-T} v_j, Tu = C1^{-1} F T, w = L2^{-1} F^T Tu
    launch_axpby(s2, 1, 1.0, vj, s2, 0.0, T, s2, st);
    c2sweep(c, false, T, s2, 1, true, st);
    BArgs a;
    a.y = T; a.ldy = s2; a.b_y = 1.0;
    a.u = Tu; a.ldu = s1;
    a.nrhs = 1;
    if ((rc = c1solve(c, a, 3, true, st))) return bail(rc);
    launch_spmv_axpby(s2, I.ft_rp, I.ft_ci, I.ft_v, Tu, s1, Wl, s2, 1, 0.0, 1.0, st);
    c2sweep(c, true, Wl, s2, 1, true, st);
    int32_t rb = 0;
    for (int pass = 0; pass < 2; ++pass) {
      const int32_t rbh = launch_multidot_partial(s2, j + 1, V, s2, Wl, part, RED_NBLK, st);
      rb = launch_gemv_sub_fold(s2, j + 1, V, s2, part, rbh, Wl, pass == 0 ? h : nullptr, pass == 1 ? part2 : nullptr,
                                st);
    }
    launch_lanczos_next(s2, j, Wl, j + 1 < steps ? vj + s2 : nullptr, sc, al, be, part2, rb, h + j, st);
  }
  std::vector<double> ah(steps), bh(steps);
  HIPCHK(hipMemcpyAsync(ah.data(), al, sizeof(double) * steps, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(bh.data(), be, sizeof(double) * steps, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double tnorm = 0.0, bprev = 0.0;
  int32_t mm = 0;
  for (int32_t j = 0; j < steps; ++j) {
    if (!std::isfinite(ah[j]) || !std::isfinite(bh[j]))
      return bail(fail(SLR_ERR_BREAKDOWN, "non-finite inner Lanczos coefficients"));
    mm = j + 1;
    tnorm = std::max(tnorm, std::fabs(ah[j]) + bh[j] + bprev);
    bprev = bh[j];
    if (bh[j] <= 1e-14 * tnorm) break;
  }
  if (mm < kw + 1) return bail(fail(SLR_ERR_LANCZOS_SHORT, "inner Lanczos produced fewer Ritz pairs than needed"));
  double *Z = tmp.alloc<double>((size_t)6 * mm * kw);
  double *ev = tmp.alloc<double>(mm);
  double *Y = tmp.alloc<double>((size_t)mm * kw);
  int *info = tmp.alloc<int>(1);
  if (!Z || !ev || !Y || !info) return bail(fail(SLR_ERR_OOM, "inner eigensolve"));
  launch_tridiag_eig(mm, al, be, Z, ev, Y, kw, info, st);
  I.U2 = c->pool.alloc<double>((size_t)s2 * kw);
  if (!I.U2) return bail(fail(SLR_ERR_OOM, "U2"));
  launch_ritz<double>(s2, mm, kw, V, s2, Y, I.U2, I.U2, st);
  int info_h = 0;
  std::vector<double> ritz(mm, 0.0);
  HIPCHK(hipMemcpyAsync(&info_h, info, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ritz.data(), ev, sizeof(double) * mm, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  tmp.release();
  if (info_h) return fail(SLR_ERR_BREAKDOWN, "inner tridiagonal eigensolve did not converge");
  I.ritz_h = ritz;
  I.lam_h.assign(ritz.begin(), ritz.begin() + kw);
  I.theta2 = ritz[kw];
  I.steps = mm;
  if (!(I.theta2 < 1.0)) return fail(SLR_ERR_C_NOT_SPD, "inner correction not positive definite (theta2 >= 1)");
  for (double l : I.lam_h)
    if (!(l < 1.0)) return fail(SLR_ERR_C_NOT_SPD, "inner correction not positive definite (a Ritz value >= 1)");
  I.sq = std::sqrt(1.0 / (1.0 - I.theta2));
  std::vector<double> q(kw);
  for (int32_t i = 0; i < kw; ++i) q[i] = std::sqrt(1.0 / (1.0 - I.lam_h[i])) - I.sq;
  I.qd = c->pool.upload(q);
  int32_t ldk;
  const int64_t ng = lr_rm_groups<double>(s2, kw, ldk);
  I.nblk = (int32_t)std::min<int64_t>(2048, std::max<int64_t>(256, ng / 128));
  I.U2rm = c->pool.alloc<double>((size_t)ng * 64 * 2);
  if (!I.qd || !I.U2rm) return fail(SLR_ERR_OOM, "U2");
  launch_lr_to_rm<double>(I.U2, s2, kw, I.U2rm, st);
  return SLR_OK;
}

// Fixed-width sweeps: levels wider than 64 * rec_passes(K) rows are cut into
// consecutive sub-levels of at most that many rows (the rows of a level are
// independent, so the schedule stays valid and the arithmetic unchanged).
// Bytes of one ELL level segment of L rows of width K (layout in pack_sweep).
int64_t ell_segment_bytes(int64_t L, int64_t K, int64_t ts) {
  return pad16h(kEllHeaderBytes + pad8h(2 * L) + pad8h(ts * L) + pad8h(2 * K * L) + ts * K * L);
}

// Rows of one level are independent, so any split of a level is a valid
// schedule.  Fixed-width records: levels wider than 64 * rec_passes(K) rows
// are split (one straight-line pass per lane).  ELL form: each level is cut
// into consecutive pieces of at most kEllLevelBytes (or one row), each
// padded only to its own widest row.
Sweep split_levels(const Sweep &sw, int32_t Kfix, int64_t ts) {
  Sweep out = sw;
  out.levptr.assign(1, 0);
  for (int32_t l = 0; l < sw.nlev; ++l) {
    const int32_t a = sw.levptr[l], b = sw.levptr[l + 1];
    if (Kfix > 0) {
      const int32_t cap = 64 * rec_passes(Kfix);
      for (int32_t t = a; t < b; t += cap) out.levptr.push_back(std::min(t + cap, b));
      continue;
    }
    int32_t t0 = a, K = 0;
    for (int32_t t = a; t < b; ++t) {
      const int32_t Kt = std::max(K, sw.rp[t + 1] - sw.rp[t]);
      if (t > t0 && ell_segment_bytes(t + 1 - t0, Kt, ts) > kEllLevelBytes) {
        out.levptr.push_back(t);
        t0 = t;
        K = sw.rp[t + 1] - sw.rp[t];
      } else {
        K = Kt;
      }
    }
    out.levptr.push_back(b);
  }
  out.nlev = (int32_t)out.levptr.size() - 1;
  if (sw.levptr.empty()) out.levptr.clear();
  return out;
}

// Pack one sweep of one subdomain as the level-sliced byte stream the B
// kernel stages into LDS (layouts documented with BlockDesc): row records
// when every row has the fixed width Kfix > 0, else the ELL form.
// Coefficient maps of a device refactorisation (built while packing).
struct RfSweepMaps {
  std::vector<RfMap> sc, w, w2;
};
struct RfMaps {
  std::vector<RfMap> bdata, ev, tv;   // B sweep streams, E and E^T values
  RfSweepMaps cf, cb;                 // interface sweeps
};

// Coefficient sources of the stored scale / weights of sweep row t (for the
// device refactorisation; ebase = first entry of the factor).
RfMap rf_scale(const Sweep &sw, int32_t t, int64_t off, int64_t ebase) {
  if (sw.unit_sc) return RfMap{off, 0, 0, 0, RF_ONE};
  return RfMap{off, (int32_t)(ebase + sw.sc_e[t]), 0, 0, RF_RECIP};
}
RfMap rf_weight(const Sweep &sw, int32_t t, int32_t e, int64_t off, int64_t ebase) {
  if (sw.divided) return RfMap{off, (int32_t)(ebase + sw.w_e[e]), (int32_t)(ebase + sw.sc_e[t]), 0, RF_DIV};
  return RfMap{off, (int32_t)(ebase + sw.w_e[e]), 0, 0, RF_RAW};
}

template <typename TS>
void pack_sweep(const Sweep &sw, int32_t Kfix, std::vector<uint8_t> &data, std::vector<int32_t> &lvb, int32_t &K,
                int32_t &max_level_bytes, int64_t &offset, std::vector<RfMap> *map = nullptr, int64_t ebase = 0) {
  K = 0;
  for (int32_t t = 0; t < sw.nrows; ++t) K = std::max(K, sw.rp[t + 1] - sw.rp[t]);
  if (Kfix > 0) K = Kfix;
  offset = (int64_t)data.size();
  int64_t pos = 0;
  lvb.push_back(0);
  const int32_t KR = rec_width(K);
  for (int32_t l = 0; l < sw.nlev; ++l) {
    const int32_t a = sw.levptr[l], L = sw.levptr[l + 1] - a;
    int64_t size;
    if (Kfix > 0) {
      // row records: int32 [row, c_0 .. c_{K-1}, pad] then TS [sc, w_0 .. w_{K-1}, pad]
      const int64_t o_w = 4 * (int64_t)KR * L;
      size = o_w + (int64_t)sizeof(TS) * KR * L;
      data.resize(offset + pos + size, 0);
      uint8_t *base = data.data() + offset + pos;
      int32_t *ix = reinterpret_cast<int32_t *>(base);
      TS *wr = reinterpret_cast<TS *>(base + o_w);
      const int64_t wbase = offset + pos + o_w;
      for (int32_t j = 0; j < L; ++j) {
        const int32_t t = a + j, row = sw.rows[t];
        const int32_t e0 = sw.rp[t], cnt = sw.rp[t + 1] - e0;
        ix[(int64_t)j * KR] = row;
        wr[(int64_t)j * KR] = (TS)sw.sc[t];
        if (map) map->push_back(rf_scale(sw, t, wbase + (int64_t)sizeof(TS) * j * KR, ebase));
        for (int32_t e = 0; e + 1 < KR; ++e) {
          ix[(int64_t)j * KR + 1 + e] = e < cnt ? sw.ci[e0 + e] : row;
          wr[(int64_t)j * KR + 1 + e] = e < cnt ? (TS)sw.w[e0 + e] : (TS)0;
          if (map && e < cnt)
            map->push_back(rf_weight(sw, t, e0 + e, wbase + (int64_t)sizeof(TS) * ((int64_t)j * KR + 1 + e), ebase));
        }
      }
    } else {
      // this level's own width
      int32_t Kl = 0;
      for (int32_t j = 0; j < L; ++j) Kl = std::max(Kl, sw.rp[a + j + 1] - sw.rp[a + j]);
      const int32_t K = Kl;
      const int64_t o_rows = kEllHeaderBytes;
      const int64_t o_sc = o_rows + pad8h(2 * L), o_ci = o_sc + pad8h((int64_t)sizeof(TS) * L);
      const int64_t o_w = o_ci + pad8h(2 * (int64_t)K * L);
      size = ell_segment_bytes(L, K, sizeof(TS));
      data.resize(offset + pos + size, 0);
      uint8_t *base = data.data() + offset + pos;
      *reinterpret_cast<int32_t *>(base) = K;
      uint16_t *rows = reinterpret_cast<uint16_t *>(base + o_rows);
      TS *sc = reinterpret_cast<TS *>(base + o_sc);
      uint16_t *ci = reinterpret_cast<uint16_t *>(base + o_ci);
      TS *w = reinterpret_cast<TS *>(base + o_w);
      const int64_t sbase = offset + pos + o_sc, wbase = offset + pos + o_w;
      for (int32_t j = 0; j < L; ++j) {
        const int32_t t = a + j, row = sw.rows[t];
        rows[j] = (uint16_t)row;
        sc[j] = (TS)sw.sc[t];
        if (map) map->push_back(rf_scale(sw, t, sbase + (int64_t)sizeof(TS) * j, ebase));
        const int32_t e0 = sw.rp[t], cnt = sw.rp[t + 1] - e0;
        for (int32_t e = 0; e < K; ++e) {
          ci[(int64_t)e * L + j] = (uint16_t)(e < cnt ? sw.ci[e0 + e] : row);
          w[(int64_t)e * L + j] = e < cnt ? (TS)sw.w[e0 + e] : (TS)0;
          if (map && e < cnt)
            map->push_back(rf_weight(sw, t, e0 + e, wbase + (int64_t)sizeof(TS) * ((int64_t)e * L + j), ebase));
        }
      }
    }
    max_level_bytes = std::max<int32_t>(max_level_bytes, (int32_t)size);
    pos += size;
    lvb.push_back((int32_t)pos);
  }
}

// ELL-form sweep (any width) packed with its near-chains solved by
// columns.  A run of at least kColRunMin consecutive levels of at most
// kColRunRows rows each -- typically the long rows at the end of a minimum
// degree or threshold factor, each waiting for the previous one -- is
// packed as (1) ELL pieces holding the run's rows with their scale and the
// entries to rows before the run (independent rows: those rows are final),
// then (2) column segments: for each run row in order, the run rows after
// it that use it, with their weights.  The kernel then finishes a run row
// by a read of its value and updates the rows that use it, instead of one
// reduction per level.  Other levels are cut into ELL pieces as
// split_levels does.  Appends the segments' byte offsets to lvb and their
// row counts (prefix sums, from 0) to lev; returns the segment count.
constexpr int32_t kColRunRows = 8, kColRunMin = 8;

int64_t csc_segment_bytes(int64_t ncol, int64_t nnz, int64_t ts) {
  return pad16h(kEllHeaderBytes + pad8h(2 * ncol) + pad8h(2 * (ncol + 1)) + pad8h(2 * nnz) + ts * nnz);
}

template <typename TS>
int32_t pack_sweep_runs(const Sweep &sw, std::vector<uint8_t> &data, std::vector<int32_t> &lvb,
                        std::vector<int32_t> &lev, int32_t &K, int32_t &max_level_bytes, int64_t &offset) {
  const int64_t ts = sizeof(TS);
  K = 0;
  for (int32_t t = 0; t < sw.nrows; ++t) K = std::max(K, sw.rp[t + 1] - sw.rp[t]);
  offset = (int64_t)data.size();
  int64_t pos = 0;
  int32_t rows_done = 0, nseg = 0;
  lvb.push_back(0);
  lev.push_back(0);
  auto close_seg = [&](int64_t size, int32_t rows) {
    max_level_bytes = std::max<int32_t>(max_level_bytes, (int32_t)size);
    pos += size;
    lvb.push_back((int32_t)pos);
    rows_done += rows;
    lev.push_back(rows_done);
    ++nseg;
  };
  // one ELL piece: rows at sweep positions tl[a .. b), entries kept by keep(column)
  auto emit_ell = [&](const std::vector<int32_t> &tl, size_t a, size_t b, const std::vector<char> *skip) {
    const int32_t L = (int32_t)(b - a);
    auto keep = [&](int32_t col) { return !skip || !(*skip)[col]; };
    int32_t Kl = 0;
    for (size_t j = a; j < b; ++j) {
      int32_t c = 0;
      for (int32_t e = sw.rp[tl[j]]; e < sw.rp[tl[j] + 1]; ++e) c += keep(sw.ci[e]);
      Kl = std::max(Kl, c);
    }
    const int64_t o_sc = kEllHeaderBytes + pad8h(2 * L), o_ci = o_sc + pad8h(ts * L);
    const int64_t o_w = o_ci + pad8h(2 * (int64_t)Kl * L);
    const int64_t size = ell_segment_bytes(L, Kl, ts);
    data.resize(offset + pos + size, 0);
    uint8_t *base = data.data() + offset + pos;
    *reinterpret_cast<int32_t *>(base) = Kl;
    uint16_t *rows = reinterpret_cast<uint16_t *>(base + kEllHeaderBytes);
    TS *sc = reinterpret_cast<TS *>(base + o_sc);
    uint16_t *ci = reinterpret_cast<uint16_t *>(base + o_ci);
    TS *w = reinterpret_cast<TS *>(base + o_w);
    for (int32_t j = 0; j < L; ++j) {
      const int32_t t = tl[a + j], row = sw.rows[t];
      rows[j] = (uint16_t)row;
      sc[j] = (TS)sw.sc[t];
      int32_t e2 = 0;
      for (int32_t e = sw.rp[t]; e < sw.rp[t + 1]; ++e) {
        if (!keep(sw.ci[e])) continue;
        ci[(int64_t)e2 * L + j] = (uint16_t)sw.ci[e];
        w[(int64_t)e2 * L + j] = (TS)sw.w[e];
        ++e2;
      }
      for (; e2 < Kl; ++e2) {
        ci[(int64_t)e2 * L + j] = (uint16_t)row;
        w[(int64_t)e2 * L + j] = (TS)0;
      }
    }
    close_seg(size, L);
  };
  // ELL pieces of at most kEllLevelBytes (or one row) over tl
  auto emit_ell_cut = [&](const std::vector<int32_t> &tl, const std::vector<char> *skip) {
    size_t a = 0;
    int32_t Kc = 0;
    for (size_t j = 0; j < tl.size(); ++j) {
      int32_t c = 0;
      for (int32_t e = sw.rp[tl[j]]; e < sw.rp[tl[j] + 1]; ++e) c += !skip || !(*skip)[sw.ci[e]];
      const int32_t K2 = std::max(Kc, c);
      if (j > a && ell_segment_bytes((int64_t)(j + 1 - a), K2, ts) > kEllLevelBytes) {
        emit_ell(tl, a, j, skip);
        a = j;
        Kc = c;
      } else {
        Kc = K2;
      }
    }
    if (a < tl.size()) emit_ell(tl, a, tl.size(), skip);
  };
  std::vector<char> in_run(std::max(sw.nrows, 1), 0);
  std::vector<int32_t> tl;
  int32_t l = 0;
  while (l < sw.nlev) {
    int32_t r = l;
    while (r < sw.nlev && sw.levptr[r + 1] - sw.levptr[r] <= kColRunRows) ++r;
    if (r - l >= kColRunMin) {
      // run of levels [l, r): pre pieces, then column segments
      const int32_t t0 = sw.levptr[l], t1 = sw.levptr[r];
      tl.clear();
      for (int32_t t = t0; t < t1; ++t) {
        tl.push_back(t);
        in_run[sw.rows[t]] = 1;
      }
      emit_ell_cut(tl, &in_run);
      // columns: run row k (position t0 + k) -> (later run row, weight)
      const int32_t R = t1 - t0;
      std::vector<int32_t> cpos(std::max(sw.nrows, 1), -1);
      for (int32_t k = 0; k < R; ++k) cpos[sw.rows[t0 + k]] = k;
      std::vector<std::vector<std::pair<uint16_t, double>>> col(R);
      for (int32_t k = 0; k < R; ++k) {
        const int32_t t = t0 + k;
        for (int32_t e = sw.rp[t]; e < sw.rp[t + 1]; ++e)
          if (in_run[sw.ci[e]]) col[cpos[sw.ci[e]]].emplace_back((uint16_t)sw.rows[t], sw.w[e]);
      }
      int32_t c0 = 0;
      while (c0 < R) {
        int32_t c1 = c0 + 1;
        int64_t nnz = (int64_t)col[c0].size();
        while (c1 < R && csc_segment_bytes(c1 + 1 - c0, nnz + (int64_t)col[c1].size(), ts) <= kEllLevelBytes) {
          nnz += (int64_t)col[c1].size();
          ++c1;
        }
        const int32_t nc = c1 - c0;
        const int64_t size = csc_segment_bytes(nc, nnz, ts);
        data.resize(offset + pos + size, 0);
        uint8_t *base = data.data() + offset + pos;
        int32_t *hdr = reinterpret_cast<int32_t *>(base);
        hdr[0] = -2;
        hdr[1] = nc;
        hdr[2] = (int32_t)nnz;
        uint16_t *crow = reinterpret_cast<uint16_t *>(base + kEllHeaderBytes);
        uint16_t *cptr = reinterpret_cast<uint16_t *>(base + kEllHeaderBytes + pad8h(2 * nc));
        uint16_t *tgt = reinterpret_cast<uint16_t *>(base + kEllHeaderBytes + pad8h(2 * nc) + pad8h(2 * (nc + 1)));
        TS *w = reinterpret_cast<TS *>(base + kEllHeaderBytes + pad8h(2 * nc) + pad8h(2 * (nc + 1)) + pad8h(2 * nnz));
        int32_t e = 0;
        for (int32_t c = c0; c < c1; ++c) {
          crow[c - c0] = (uint16_t)sw.rows[t0 + c];
          cptr[c - c0] = (uint16_t)e;
          for (const auto &pr : col[c]) {
            tgt[e] = pr.first;
            w[e] = (TS)pr.second;
            ++e;
          }
        }
        cptr[nc] = (uint16_t)e;
        close_seg(size, nc);
        c0 = c1;
      }
      for (int32_t t = t0; t < t1; ++t) in_run[sw.rows[t]] = 0;
      l = r;
      continue;
    }
    // ordinary levels [l, max(r, l + 1))
    const int32_t le = std::max(r, l + 1);
    for (int32_t ll = l; ll < le; ++ll) {
      tl.clear();
      for (int32_t t = sw.levptr[ll]; t < sw.levptr[ll + 1]; ++t) tl.push_back(t);
      emit_ell_cut(tl, nullptr);
    }
    l = le;
  }
  return nseg;
}

// Sizes of a packed block set that the B kernel's LDS plan needs.
struct BSizes {
  int32_t max_m = 0, max_lev = 0, max_level_bytes = 0;
  int32_t level_order = 0;   // blocks whose LDS layout is the level order
  int64_t data_bytes = 0;
};

// Modelled LDS bank cost of a block's two sweeps with x laid out by pos
// (elements of eb bytes): the rows of a level in groups of 64 (one wave
// access each), one gather per entry slot plus the store; an access costs
// the largest number of distinct 4-byte words that fall into one of 64
// banks (its serialisation).
int64_t lds_sweep_cost(const Block &b, const std::vector<int32_t> &pos, int eb) {
  constexpr int kBanks = 64;
  const int32_t wpe = eb / 4;   // 4-byte words per element
  int64_t cost = 0;
  std::vector<int32_t> stamp((size_t)std::max(b.m, 1) * wpe, -1);   // last access that touched a word
  int32_t cnt[kBanks], id = 0;
  for (const Sweep *sw : {&b.fwd, &b.bwd})
    for (int32_t l = 0; l < sw->nlev; ++l)
      for (int32_t t0 = sw->levptr[l]; t0 < sw->levptr[l + 1]; t0 += 64) {
        const int32_t t1 = std::min(t0 + 64, sw->levptr[l + 1]);
        int32_t K = 0;
        for (int32_t t = t0; t < t1; ++t) K = std::max(K, sw->rp[t + 1] - sw->rp[t]);
        for (int32_t e = -1; e < K; ++e, ++id) {
          std::fill(cnt, cnt + kBanks, 0);
          int32_t worst = 0;
          for (int32_t t = t0; t < t1; ++t) {
            const int32_t c = (e >= 0 && e < sw->rp[t + 1] - sw->rp[t]) ? sw->ci[sw->rp[t] + e] : sw->rows[t];
            for (int32_t h = 0; h < wpe; ++h) {
              const int32_t w = pos[c] * wpe + h;
              if (stamp[w] == id) continue;
              stamp[w] = id;
              worst = std::max(worst, ++cnt[w % kBanks]);
            }
          }
          cost += worst;
        }
      }
  return cost;
}

// The LDS position of each row of a block.  In the input order the rows of
// one level of a stencil-like factor lie a grid line apart, so a wave's
// gathers can all fall into a few banks (a line length of 65 puts every
// lane of a 2-D anti-diagonal into the same bank).  In the forward sweep's
// level order the rows of a level sit side by side and so do the earlier
// rows that neighbouring lanes gather; but then the load of f and the store
// of u scatter.  The level order is taken when the modelled sweep cost in
// the input order is more than 3.5 times that in level order, else the
// identity.  Only rows of fixed small width (zero-fill factors) are
// modelled; other blocks keep the identity.
std::vector<int32_t> lds_positions(const Block &b, bool fixed_width, int eb) {
  std::vector<int32_t> id(std::max(b.m, 0)), pos(std::max(b.m, 0), -1);
  for (int32_t r = 0; r < b.m; ++r) id[r] = r;
  if (!fixed_width || b.fwd.nrows != b.m || (int32_t)b.fwd.rows.size() != b.m) return id;
  for (int32_t t = 0; t < b.m; ++t) {
    const int32_t r = b.fwd.rows[t];
    if (r < 0 || r >= b.m || pos[r] >= 0) return id;
    pos[r] = t;
  }
  return 2 * lds_sweep_cost(b, id, eb) > 7 * lds_sweep_cost(b, pos, eb) ? pos : id;
}

// Rename a block's local rows by pos: sweep rows and columns, E rows and
// E^T columns (same schedules, entry order and coefficients).
void relabel_block(Block &b, const std::vector<int32_t> &pos) {
  for (Sweep *sw : {&b.fwd, &b.bwd}) {
    for (int32_t &r : sw->rows) r = pos[r];
    for (int32_t &c : sw->ci) c = pos[c];
  }
  for (int32_t &r : b.e_row) r = pos[r];
  for (int32_t &r : b.t_j) r = pos[r];
}

// The fixed row width of a block set's packed sweeps: the widest row of any
// sweep when it is at most 4 (rows are padded to it), else 0 (ELL form).
int32_t packed_width(const std::vector<Block> &blocks) {
  int32_t widest = 0;
  for (const Block &b : blocks)
    for (const Sweep *sw : {&b.fwd, &b.bwd})
      for (int32_t t = 0; t < sw->nrows; ++t) widest = std::max(widest, sw->rp[t + 1] - sw->rp[t]);
  return (widest >= 1 && widest <= 4) ? widest : 0;
}

// Pack and upload a set of diagonal blocks (factor sweeps, E and E^T rows)
// for the B kernel.  Every local index in the packed data is an LDS
// position (lds_positions); B.xpos maps a block's rows to them, or is null
// when every block keeps the identity.
template <typename TS>
bool pack_blocks(DevPool &P, const std::vector<Block> &blocks, BlockArrays<TS> &B, BSizes &sz, RfMaps *rm) {
  const int32_t nbk = (int32_t)blocks.size();
  std::vector<BlockDesc> desc(nbk);
  std::vector<int32_t> lev, lvb;
  std::vector<uint8_t> data;
  std::vector<uint16_t> e_row, t_j, xpos;
  bool any_moved = false;
  std::vector<int32_t> e_q, t_q;
  std::vector<double> e_val, t_val;
  int32_t max_m = 0, max_lev = 0, max_lb = 0, max_K = 0;
  bool ok = true;
  const int32_t Kfix = packed_width(blocks);
  for (int32_t q = 0; q < nbk; ++q) {
    const Block &b0 = blocks[q];
    BlockDesc &d = desc[q];
    const std::vector<int32_t> pos = lds_positions(b0, Kfix > 0, (int)sizeof(TS));
    Block b = b0;
    relabel_block(b, pos);
    if ((int64_t)xpos.size() < (int64_t)b.m0 + b.m) xpos.resize((size_t)b.m0 + b.m, 0);
    bool moved = false;
    for (int32_t r = 0; r < b.m; ++r) {
      xpos[(size_t)b.m0 + r] = (uint16_t)pos[r];
      moved |= pos[r] != r;
    }
    any_moved |= moved;
    sz.level_order += moved;
    d.m0 = b.m0;
    d.m = b.m;
    if (b.m > 65535) ok = false;   // uint16 local indices
    max_m = std::max(max_m, b.m);
    if (Kfix == 0 && !rm) {
      // ELL form with near-chains by columns
      d.f_lev = (int32_t)lev.size();
      d.f_lvb = (int32_t)lvb.size();
      d.f_nlev = pack_sweep_runs<TS>(b.fwd, data, lvb, lev, d.f_K, max_lb, d.f_data);
      d.b_lev = (int32_t)lev.size();
      d.b_lvb = (int32_t)lvb.size();
      d.b_nlev = pack_sweep_runs<TS>(b.bwd, data, lvb, lev, d.b_K, max_lb, d.b_data);
      max_lev = std::max({max_lev, d.f_nlev, d.b_nlev});
    } else {
      const Sweep fs = split_levels(b.fwd, Kfix, sizeof(TS)), bs = split_levels(b.bwd, Kfix, sizeof(TS));
      max_lev = std::max({max_lev, fs.nlev, bs.nlev});
      d.f_nlev = fs.nlev;
      d.f_lev = (int32_t)lev.size();
      lev.insert(lev.end(), fs.levptr.begin(), fs.levptr.end());
      if (fs.levptr.empty()) lev.push_back(0);
      d.f_lvb = (int32_t)lvb.size();
      pack_sweep<TS>(fs, Kfix, data, lvb, d.f_K, max_lb, d.f_data, rm ? &rm->bdata : nullptr, b.f_base);
      d.b_nlev = bs.nlev;
      d.b_lev = (int32_t)lev.size();
      lev.insert(lev.end(), bs.levptr.begin(), bs.levptr.end());
      if (bs.levptr.empty()) lev.push_back(0);
      d.b_lvb = (int32_t)lvb.size();
      pack_sweep<TS>(bs, Kfix, data, lvb, d.b_K, max_lb, d.b_data, rm ? &rm->bdata : nullptr, b.f_base);
    }
    max_K = std::max({max_K, d.f_K, d.b_K});
    // E rows as ELL (width = longest row)
    d.e_row = (int32_t)e_row.size();
    d.e_n = (int32_t)b.e_row.size();
    d.e_K = 0;
    for (int32_t i = 0; i < d.e_n; ++i) d.e_K = std::max(d.e_K, b.e_ptr[i + 1] - b.e_ptr[i]);
    d.e_ent = (int32_t)e_q.size();
    for (int32_t i = 0; i < d.e_n; ++i) e_row.push_back((uint16_t)b.e_row[i]);
    e_q.resize(e_q.size() + (size_t)d.e_K * d.e_n, 0);
    e_val.resize(e_val.size() + (size_t)d.e_K * d.e_n, 0.0);
    for (int32_t i = 0; i < d.e_n; ++i)
      for (int32_t e = 0; e < b.e_ptr[i + 1] - b.e_ptr[i]; ++e) {
        e_q[d.e_ent + (size_t)e * d.e_n + i] = b.e_q[b.e_ptr[i] + e];
        e_val[d.e_ent + (size_t)e * d.e_n + i] = b.e_val[b.e_ptr[i] + e];
        if (rm)
          rm->ev.push_back(RfMap{(int64_t)sizeof(TS) * (int64_t)(d.e_ent + (size_t)e * d.e_n + i),
                                 (int32_t)b.e_src[b.e_ptr[i] + e], 0, 0, RF_SRC});
      }
    // E^T rows as ELL
    d.t_row = (int32_t)t_q.size();
    d.t_n = (int32_t)b.t_q.size();
    d.t_K = 0;
    for (int32_t i = 0; i < d.t_n; ++i) d.t_K = std::max(d.t_K, b.t_ptr[i + 1] - b.t_ptr[i]);
    d.t_ent = (int32_t)t_j.size();
    t_q.insert(t_q.end(), b.t_q.begin(), b.t_q.end());
    t_j.resize(t_j.size() + (size_t)d.t_K * d.t_n, 0);
    t_val.resize(t_val.size() + (size_t)d.t_K * d.t_n, 0.0);
    for (int32_t i = 0; i < d.t_n; ++i)
      for (int32_t e = 0; e < b.t_ptr[i + 1] - b.t_ptr[i]; ++e) {
        t_j[d.t_ent + (size_t)e * d.t_n + i] = (uint16_t)b.t_j[b.t_ptr[i] + e];
        t_val[d.t_ent + (size_t)e * d.t_n + i] = b.t_val[b.t_ptr[i] + e];
        if (rm)
          rm->tv.push_back(RfMap{(int64_t)sizeof(TS) * (int64_t)(d.t_ent + (size_t)e * d.t_n + i),
                                 (int32_t)b.t_src[b.t_ptr[i] + e], 0, 0, RF_SRC});
      }
  }
  if (data.empty()) data.resize(16, 0);
  B.desc = P.upload(desc);
  B.lev = P.upload(lev);
  B.lvb = P.upload(lvb);
  B.data = P.upload(data);
  B.e_row = P.upload(e_row); B.e_q = P.upload(e_q);
  B.e_val = P.upload(conv<TS>(e_val));
  B.t_q = P.upload(t_q); B.t_j = P.upload(t_j);
  B.t_val = P.upload(conv<TS>(t_val));
  B.xpos = any_moved ? P.upload(xpos) : nullptr;
  B.max_m = max_m;
  B.max_lev = max_lev;
  B.max_level_bytes = max_lb;
  B.max_K = max_K;
  B.pack_K = Kfix;
  sz.max_m = max_m;
  sz.max_lev = max_lev;
  sz.max_level_bytes = max_lb;
  sz.data_bytes = (int64_t)data.size();
  return ok && B.desc && B.lev && B.lvb && B.data && B.e_row && B.e_q && B.e_val && B.t_q && B.t_j && B.t_val &&
         (B.xpos || !any_moved);
}

// Upload one interface sweep (level-sorted rows, CSR weights, scales and,
// for schedules of at most two levels, the pre-multiplied weights w2).
template <typename TS>
bool upload_sweep(DevPool &P, const Sweep &sw, SweepArrays<TS> &S, RfSweepMaps *sm) {
  if (sm) {
    std::vector<int32_t> tof(sw.nrows, 0);
    for (int32_t t = 0; t < sw.nrows; ++t) tof[sw.rows[t]] = t;
    for (int32_t t = 0; t < sw.nrows; ++t) {
      sm->sc.push_back(rf_scale(sw, t, (int64_t)sizeof(TS) * t, 0));
      for (int32_t e = sw.rp[t]; e < sw.rp[t + 1]; ++e) {
        sm->w.push_back(rf_weight(sw, t, e, (int64_t)sizeof(TS) * e, 0));
        if (sw.nlev <= 2)
          sm->w2.push_back(RfMap{(int64_t)sizeof(TS) * e, sw.w_e[e], sw.sc_e[t], sw.sc_e[tof[sw.ci[e]]], RF_W2});
      }
    }
  }
  std::vector<int32_t> lv = sw.levptr;
  if (lv.empty()) lv.push_back(0);
  S.lev = P.upload(lv);
  S.rows = P.upload(sw.rows);
  S.rp = P.upload(sw.rp.empty() ? std::vector<int32_t>{0} : sw.rp);
  S.ci = P.upload(sw.ci);
  S.w = P.upload(conv<TS>(sw.w));
  S.sc = P.upload(conv<TS>(sw.sc));
  bool okw2 = true;
  if (sw.nlev <= 2) {
    // weights times the (stored) scale of the dependency row, rounded to TS
    std::vector<double> scr(sw.nrows, 0.0);
    for (int32_t t = 0; t < sw.nrows; ++t) scr[sw.rows[t]] = (double)(TS)sw.sc[t];
    std::vector<double> w2(sw.w.size());
    for (size_t e = 0; e < sw.w.size(); ++e) w2[e] = (double)(TS)sw.w[e] * scr[sw.ci[e]];
    S.w2 = P.upload(conv<TS>(w2));
    okw2 = S.w2 != nullptr;
  }
  return S.lev && S.rows && S.rp && S.ci && S.w && S.sc && okw2;
}

template <typename TS>
void upload_blocks(slr_ctx *c, const HostSetup &H, BlockArrays<TS> &B, SweepArrays<TS> &Cf, SweepArrays<TS> &Cb,
                   bool &ok, RfMaps *rm) {
  BSizes sz;
  ok = pack_blocks<TS>(c->pool, H.blocks, B, sz, rm);
  // work estimate of one item of a subdomain for the persistent schedule:
  // its dependent levels, plus its entries (staging)
  c->b_cost_h.clear();
  c->b_m_h.clear();
  for (const Block &b : H.blocks) {
    c->b_cost_h.push_back((double)(b.fwd.nlev + b.bwd.nlev) + (double)(b.fwd.ci.size() + b.bwd.ci.size()) / 256.0);
    c->b_m_h.push_back(b.m);
  }
  c->b_max_m = sz.max_m;
  c->info.b_lds_level_order = sz.level_order;
  c->b_max_lev = sz.max_lev;
  c->b_max_level_bytes = sz.max_level_bytes;
  c->b_data_bytes = sz.data_bytes;
  if (H.s1 > 0) return;   // the recursive interface solver has no single factor of C
  ok = ok && upload_sweep<TS>(c->pool, H.cfwd, Cf, rm ? &rm->cf : nullptr) &&
       upload_sweep<TS>(c->pool, H.cbwd, Cb, rm ? &rm->cb : nullptr);
}

// Lanes per row of an interface sweep launched one level at a time: by the
// mean row length (entries per row < 8: one lane per row).
int32_t sweep_group(const Sweep &sw) {
  const double mean = sw.nrows > 0 ? (double)sw.ci.size() / sw.nrows : 0.0;
  return mean < 8.0 ? 1 : (mean < 24.0 ? 4 : (mean < 64.0 ? 8 : 16));
}

// Upload the recursive interface solver's C1 blocks, C2 sweeps and F^T.
template <typename TS>
bool upload_inner(slr_ctx *c, const HostSetup &H, BlockArrays<TS> &B, SweepArrays<TS> &Cf, SweepArrays<TS> &Cb) {
  slr_ctx::Inner &I = c->ml;
  BSizes sz;
  bool ok = pack_blocks<TS>(c->pool, H.c1blocks, B, sz, nullptr);
  I.max_m = sz.max_m;
  I.max_lev = sz.max_lev;
  I.max_level_bytes = sz.max_level_bytes;
  I.data_bytes = sz.data_bytes;
  ok = ok && upload_sweep<TS>(c->pool, H.c2fwd, Cf, nullptr) && upload_sweep<TS>(c->pool, H.c2bwd, Cb, nullptr);
  I.ft_rp = c->pool.upload(H.ft_rp);
  I.ft_ci = c->pool.upload(H.ft_ci.empty() ? std::vector<int32_t>{0} : H.ft_ci);
  I.ft_v = c->pool.upload(H.ft_v.empty() ? std::vector<double>{0.0} : H.ft_v);
  return ok && I.ft_rp && I.ft_ci && I.ft_v;
}

int perm_ws(slr_ctx *c, int32_t nrhs) {
  if (c->pcap >= nrhs && c->pr) return SLR_OK;
  c->ppool.release();
  c->pr = c->ppool.alloc<double>((size_t)c->n * nrhs);
  c->pz = c->ppool.alloc<double>((size_t)c->n * nrhs);
  if (!c->pr || !c->pz) return fail(SLR_ERR_OOM, "permutation scratch");
  c->pcap = nrhs;
  return SLR_OK;
}

hipStream_t S(void *p) { return (hipStream_t)p; }

// Default Lanczos start vector: U[-1, 1) from SplitMix64 (Steele, Lea &
// Flood 2014) keyed by the original node index.
const double *seeded_v0(int64_t n, uint64_t seed, std::vector<double> &v0) {
  v0.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    v0[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
  return v0.data();
}

// Keep what slr_refactor needs: the input pattern (symmetry check), the
// gather maps of A / E / E^T, the factor plans and the coefficient maps.
bool rf_upload(slr_ctx *c, const HostSetup &H, const RfMaps &rm, const slr_csr *A) {
  auto &R = c->rf;
  auto &P = R.pool;
  // mirror entries (the symmetry test of new values becomes one pass)
  R.tr_h.assign(A->nnz, 0);
  for (int64_t i = 0; i < A->n; ++i)
    for (int64_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
      const int64_t j = A->col[e];
      const int32_t *b = A->col + A->rowptr[j], *en = A->col + A->rowptr[j + 1];
      R.tr_h[e] = A->rowptr[j] + (std::lower_bound(b, en, (int32_t)i) - b);
    }
  R.tr = P.upload(R.tr_h.empty() ? std::vector<int64_t>{0} : R.tr_h);
  if (hipHostMalloc((void **)&R.stage, sizeof(double) * std::max<int64_t>(A->nnz, 1), hipHostMallocDefault) !=
      hipSuccess)
    R.stage = nullptr;
  R.nnz = A->nnz;
  R.val = P.alloc<double>((size_t)std::max<int64_t>(A->nnz, 1));
  R.err = P.alloc<int>(4);
  R.a_src = P.upload(H.a_src);
  auto plan = [&](const RefactorPlan &F, slr_ctx::Refactor::Plan &D) {
    D.rp = P.upload(F.rp);
    D.ci = P.upload(F.ci.empty() ? std::vector<int32_t>{0} : F.ci);
    D.src = P.upload(F.src.empty() ? std::vector<int64_t>{0} : F.src);
    D.rows = P.upload(F.rows.empty() ? std::vector<int32_t>{0} : F.rows);
    D.nnz = (int64_t)F.ci.size();
    D.v = P.alloc<double>((size_t)std::max<int64_t>(D.nnz, 1));
    D.lev = F.lev;
    D.kind = F.kind;
    return D.rp && D.ci && D.src && D.rows && D.v;
  };
  auto map = [&](const std::vector<RfMap> &v, slr_ctx::Refactor::Map &D) {
    D.n = (int64_t)v.size();
    if (v.empty()) return true;
    D.m = P.upload(v);
    return D.m != nullptr;
  };
  bool ok = R.val && R.err && R.a_src && R.tr && R.stage && plan(H.fb, R.fb) && plan(H.fc, R.fc);
  ok = ok && map(rm.bdata, R.bdata) && map(rm.ev, R.ev) && map(rm.tv, R.tv);
  ok = ok && map(rm.cf.sc, R.cfsc) && map(rm.cf.w, R.cfw) && map(rm.cf.w2, R.cfw2);
  ok = ok && map(rm.cb.sc, R.cbsc) && map(rm.cb.w, R.cbw) && map(rm.cb.w2, R.cbw2);
  R.on = ok;
  return ok;
}

template <typename TS>
void rf_pack_all(slr_ctx *c, const BlockArrays<TS> &B, const SweepArrays<TS> &Cf, const SweepArrays<TS> &Cb,
                 hipStream_t st) {
  auto &R = c->rf;
  auto run = [&](const slr_ctx::Refactor::Map &m, const double *V, const void *base) {
    launch_rf_pack<TS>(m.n, m.m, V, R.val, const_cast<void *>(base), st);
  };
  run(R.bdata, R.fb.v, B.data);
  run(R.ev, nullptr, B.e_val);
  run(R.tv, nullptr, B.t_val);
  run(R.cfsc, R.fc.v, Cf.sc);
  run(R.cfw, R.fc.v, Cf.w);
  run(R.cfw2, R.fc.v, Cf.w2);
  run(R.cbsc, R.fc.v, Cb.sc);
  run(R.cbw, R.fc.v, Cb.w);
  run(R.cbw2, R.fc.v, Cb.w2);
}

// After a change of the low-rank part: workspace sized for the new k, stats.
int lowrank_done(slr_ctx *c, double t1, hipStream_t st) {
  int rc = ws_ensure(c, c->ws, std::max(c->ws.cap, 1));
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  c->info.k = c->k;
  c->info.theta = c->theta;
  c->info.setup_lanczos_s = now_s() - t1;
  c->info.device_bytes = c->pool.bytes + c->lrpool.bytes + c->ws.pool.bytes;
  return SLR_OK;
}

// ---- serialised setups (slr_export_setup / slr_import) -------------------
// Layout: the 8-byte magic, a u64 payload length, the payload, and the
// FNV-1a 64 hash of the payload.  The payload is a sequence of records:
// scalars as their bytes, host arrays and device arrays as a u64 byte count
// followed by the bytes.  Device arrays are written in a fixed order (the
// list below), so import can allocate and fill them in that order and
// point the same fields at them.
constexpr char kSetupMagic[8] = {'S', 'L', 'R', 'S', 'E', 'T', 'v', '2'};

uint64_t fnv1a(const uint8_t *p, size_t n) {
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

struct Writer {
  std::vector<uint8_t> out;
  void raw(const void *p, size_t n) {
    const uint8_t *b = (const uint8_t *)p;
    out.insert(out.end(), b, b + n);
  }
  template <typename T>
  void pod(const T &x) {
    raw(&x, sizeof(T));
  }
  template <typename T>
  void vec(const std::vector<T> &v) {
    pod<uint64_t>(v.size() * sizeof(T));
    raw(v.data(), v.size() * sizeof(T));
  }
};

struct Reader {
  const uint8_t *p;
  size_t n, pos = 0;
  bool ok = true;
  bool take(void *dst, size_t k) {
    if (!ok || k > n - pos) return ok = false;
    if (k) std::memcpy(dst, p + pos, k);
    pos += k;
    return true;
  }
  template <typename T>
  bool pod(T &x) {
    return take(&x, sizeof(T));
  }
  template <typename T>
  bool vec(std::vector<T> &v, uint64_t max_bytes = UINT64_MAX) {
    uint64_t b = 0;
    if (!pod(b) || b % sizeof(T) != 0 || b > n - pos || b > max_bytes) return ok = false;
    v.resize(b / sizeof(T));
    return take(v.data(), b);
  }
  // a device-array record: byte count and where its bytes are
  bool span(const uint8_t *&q, uint64_t &b) {
    if (!pod(b) || b > n - pos) return ok = false;
    q = p + pos;
    pos += b;
    return true;
  }
};

// The device arrays of a context that make up its preconditioner (not the
// low-rank part, not scratch), in serialisation order.  Absent arrays (w2
// of a deep interface schedule) are null.
template <typename TS>
std::vector<const void **> setup_fields(slr_ctx *c, BlockArrays<TS> &B, SweepArrays<TS> &Cf, SweepArrays<TS> &Cb) {
  auto f = [](auto &ptr) { return reinterpret_cast<const void **>(const_cast<void *>((const void *)&ptr)); };
  std::vector<const void **> v = {f(c->perm), f(c->a_rp), f(c->a_ci), f(c->a_v),
                                  f(B.desc), f(B.lev), f(B.lvb), f(B.data), f(B.e_row), f(B.e_q), f(B.e_val),
                                  f(B.t_q), f(B.t_j), f(B.t_val), f(B.xpos)};
  for (SweepArrays<TS> *S : {&Cf, &Cb})
    for (const void **q : {f(S->lev), f(S->rows), f(S->rp), f(S->ci), f(S->w), f(S->sc), f(S->w2)}) v.push_back(q);
  return v;
}

size_t pool_block_bytes(const DevPool &P, const void *ptr) {
  for (const DevBlock &b : P.blocks)
    if (b.p == ptr) return b.bytes;
  return 0;
}

int export_setup(const slr_ctx *cc, std::vector<uint8_t> &blob) {
  slr_ctx *c = const_cast<slr_ctx *>(cc);
  Writer w;
  slr_opts o = c->opts;
  o.lanczos_v0 = nullptr;
  o.U_in = nullptr;
  o.lambda_in = nullptr;
  o.k_in = 0;
  o.refactor = 0;
  w.pod(o);
  w.pod(c->n); w.pod(c->m); w.pod(c->s); w.pod(c->p);
  w.pod(c->fact_prec); w.pod(c->uk_prec);
  w.vec(c->cf_lev_h); w.vec(c->cb_lev_h);
  w.pod(c->cf_nlev); w.pod(c->cb_nlev); w.pod(c->cb_nnz);
  w.pod(c->c_one_wg); w.pod(c->c_two_level); w.pod(c->nnz_a); w.pod(c->cf_group); w.pod(c->cb_group);
  w.pod(c->b_max_m); w.pod(c->b_max_lev); w.pod(c->b_max_level_bytes); w.pod(c->b_data_bytes);
  auto dump = [&](auto &B, auto &Cf, auto &Cb) -> int {
    w.pod(B.max_m); w.pod(B.max_lev); w.pod(B.max_level_bytes); w.pod(B.max_K); w.pod(B.pack_K);
    for (const void **q : setup_fields(c, B, Cf, Cb)) {
      const size_t b = *q ? pool_block_bytes(c->pool, *q) : 0;
      if (*q && b == 0) return fail(SLR_ERR_ARG, "an array of the context is not in its pool");
      w.pod<uint64_t>(b);
      const size_t at = w.out.size();
      w.out.resize(at + b);
      if (b) HIPCHK(hipMemcpy(w.out.data() + at, *q, b, hipMemcpyDeviceToHost));
    }
    return SLR_OK;
  };
  int rc = c->fact_prec == SLR_FP64 ? dump(c->Bd, c->Cfd, c->Cbd) : dump(c->Bf, c->Cff, c->Cbf);
  if (rc) return rc;
  // launch shapes and rank-k chunks (slr_autotune)
  w.pod(c->tune1); w.pod(c->tuneM); w.pod(c->lr_nblk_tuned); w.pod(c->lrm_nblk);
  w.vec(c->b_cost_h);
  w.vec(c->b_m_h);
  // low-rank part (FP64; the stored precision is rebuilt from it on import)
  w.pod(c->k); w.pod(c->theta);
  std::vector<double> U((size_t)c->s * c->k);
  if (!U.empty()) HIPCHK(hipMemcpy(U.data(), c->U64, sizeof(double) * U.size(), hipMemcpyDeviceToHost));
  w.vec(U); w.vec(c->lam_h); w.vec(c->ritz_h); w.vec(c->alpha_h); w.vec(c->beta_h);
  w.pod(c->info);
  blob.clear();
  blob.insert(blob.end(), kSetupMagic, kSetupMagic + 8);
  const uint64_t len = w.out.size();
  blob.insert(blob.end(), (const uint8_t *)&len, (const uint8_t *)&len + 8);
  blob.insert(blob.end(), w.out.begin(), w.out.end());
  const uint64_t h = fnv1a(w.out.data(), w.out.size());
  blob.insert(blob.end(), (const uint8_t *)&h, (const uint8_t *)&h + 8);
  return SLR_OK;
}

int import_setup(const uint8_t *buf, size_t bytes, hipStream_t st, slr_ctx **out) {
  if (bytes < 24 || std::memcmp(buf, kSetupMagic, 8) != 0) return fail(SLR_ERR_ARG, "not a serialised SLR setup");
  uint64_t len = 0, h = 0;
  std::memcpy(&len, buf + 8, 8);
  if (len != bytes - 24) return fail(SLR_ERR_ARG, "serialised setup: length mismatch");
  std::memcpy(&h, buf + 16 + len, 8);
  if (h != fnv1a(buf + 16, len)) return fail(SLR_ERR_ARG, "serialised setup: checksum mismatch");
  Reader r{buf + 16, (size_t)len};
  slr_ctx *c = new slr_ctx();
  auto bad = [&](const char *what) {
    slr_destroy(c);
    return fail(SLR_ERR_ARG, std::string("serialised setup: ") + what);
  };
  (void)hipGetDevice(&c->device);
  {
    char *sp = nullptr;
    (void)scratch_address(c->device, &sp);
  }
  r.pod(c->opts);
  r.pod(c->n); r.pod(c->m); r.pod(c->s); r.pod(c->p);
  r.pod(c->fact_prec); r.pod(c->uk_prec);
  r.vec(c->cf_lev_h); r.vec(c->cb_lev_h);
  r.pod(c->cf_nlev); r.pod(c->cb_nlev); r.pod(c->cb_nnz);
  r.pod(c->c_one_wg); r.pod(c->c_two_level); r.pod(c->nnz_a); r.pod(c->cf_group); r.pod(c->cb_group);
  r.pod(c->b_max_m); r.pod(c->b_max_lev); r.pod(c->b_max_level_bytes); r.pod(c->b_data_bytes);
  if (!r.ok) return bad("truncated header");
  if (c->n < 0 || c->m < 0 || c->s < 0 || c->m + c->s != c->n || c->p < 1 ||
      (c->fact_prec != SLR_FP64 && c->fact_prec != SLR_FP32) || c->uk_prec < SLR_FP64 || c->uk_prec > SLR_BF16 ||
      (int64_t)c->cf_lev_h.size() != c->cf_nlev + 1 || (int64_t)c->cb_lev_h.size() != c->cb_nlev + 1)
    return bad("inconsistent sizes");
  c->lds_limit = (size_t)slr_device_lds_bytes();
  c->n_cu = device_cu_count();
  auto load = [&](auto &B, auto &Cf, auto &Cb) -> bool {
    r.pod(B.max_m); r.pod(B.max_lev); r.pod(B.max_level_bytes); r.pod(B.max_K); r.pod(B.pack_K);
    for (const void **q : setup_fields(c, B, Cf, Cb)) {
      const uint8_t *src = nullptr;
      uint64_t b = 0;
      if (!r.span(src, b)) return false;
      if (b == 0) {
        *q = nullptr;
        continue;
      }
      uint8_t *d = c->pool.alloc<uint8_t>(b);
      if (!d || hipMemcpy(d, src, b, hipMemcpyHostToDevice) != hipSuccess) return false;
      *q = d;
    }
    return true;
  };
  const bool ok = c->fact_prec == SLR_FP64 ? load(c->Bd, c->Cfd, c->Cbd) : load(c->Bf, c->Cff, c->Cbf);
  if (!ok) return bad("device arrays (truncated, or device memory exhausted)");
  if (pool_block_bytes(c->pool, c->perm) != sizeof(int64_t) * (size_t)std::max<int64_t>(c->n, 1) ||
      pool_block_bytes(c->pool, c->a_v) != sizeof(double) * (size_t)std::max<int64_t>(c->nnz_a, 1))
    return bad("array sizes do not match the problem");
  c->perm_h.resize(c->n);
  if (c->n) HIPCHK(hipMemcpy(c->perm_h.data(), c->perm, sizeof(int64_t) * c->n, hipMemcpyDeviceToHost));
  std::vector<double> U;
  r.pod(c->tune1); r.pod(c->tuneM); r.pod(c->lr_nblk_tuned); r.pod(c->lrm_nblk);
  r.vec(c->b_cost_h);
  r.vec(c->b_m_h);
  if ((int64_t)c->b_cost_h.size() != c->p || (int64_t)c->b_m_h.size() != c->p ||
      c->tune1.lds_div < 1 || c->tuneM.lds_div < 1 || c->tune1.threads < 0 || c->tune1.threads > 1024 ||
      c->tuneM.threads < 0 || c->tuneM.threads > 1024 || c->lrm_nblk < 1 || c->lr_nblk_tuned < 0)
    return bad("launch shapes");
  r.pod(c->k); r.pod(c->theta);
  r.vec(U); r.vec(c->lam_h); r.vec(c->ritz_h); r.vec(c->alpha_h); r.vec(c->beta_h);
  slr_info info{};
  r.pod(info);
  if (!r.ok || r.pos != r.n) return bad("truncated low-rank part");
  if (c->k < 0 || c->k > 64 || U.size() != (size_t)c->s * c->k || (int32_t)c->lam_h.size() != c->k)
    return bad("low-rank part does not match the problem");
  c->info = info;
  c->U64 = c->lrpool.upload(U.empty() ? std::vector<double>{0.0} : U);
  if (!c->U64) {
    slr_destroy(c);
    return fail(SLR_ERR_OOM, "U");
  }
  int rc = finish_lowrank(c, st);
  if (!rc) rc = ws_ensure(c, c->ws, 1);
  if (rc) {
    slr_destroy(c);
    return rc;
  }
  if (hipStreamSynchronize(st) != hipSuccess) {
    slr_destroy(c);
    return fail(SLR_ERR_HIP, "hipStreamSynchronize");
  }
  c->info.k = c->k;
  c->info.theta = c->theta;
  *out = c;
  return SLR_OK;
}

}  // namespace

extern "C" {

void slr_default_opts(slr_opts *o) {
  std::memset(o, 0, sizeof(*o));
  o->k = 16;
  o->lanczos_steps = 0;
  o->theta_mode = SLR_THETA_LAMBDA_K1;
  o->b_fact = SLR_FACT_IC0;
  o->c_fact = SLR_FACT_IC0;
  o->c_order = SLR_CORDER_SUBDOMAIN;
  o->fact_prec = SLR_FP64;
  o->uk_prec = SLR_FP64;
  o->seed = 7;
  o->eps = 0.0;
  o->cond_K = 0.0;
  o->reorth = SLR_REORTH_PARTIAL;
  o->refactor = 0;
  o->droptol = 1e-3;
  o->b_order = SLR_BORDER_NATURAL;
  o->c_levels = 1;
  o->k2 = 0;
  o->lanczos_steps2 = 0;
}

void slr_default_solve_opts(slr_solve_opts *o) {
  std::memset(o, 0, sizeof(*o));
  o->method = SLR_PCG;
  o->restart = 40;
  o->maxit = 300;
  o->check_every = 8;
  o->rtol = 1e-8;
}

const char *slr_strerror(int code) {
  switch (code) {
    case SLR_OK: return "ok";
    case SLR_ERR_ARG: return "invalid argument";
    case SLR_ERR_NOT_SYMMETRIC: return "matrix is not symmetric";
    case SLR_ERR_PARTITION: return "invalid or unsupported partition";
    case SLR_ERR_BREAKDOWN: return "factorisation or iteration breakdown";
    case SLR_ERR_C_NOT_SPD: return "interface matrix C is not SPD";
    case SLR_ERR_RITZ_SINGULAR: return "Ritz value too close to 1";
    case SLR_ERR_LANCZOS_SHORT: return "too few Lanczos Ritz pairs";
    case SLR_ERR_NOCONV: return "did not converge";
    case SLR_ERR_OOM: return "out of device memory";
    case SLR_ERR_HIP: return "HIP runtime error";
    case SLR_ERR_ADMIT: return "admission refused";
    default: return "unknown error";
  }
}

const char *slr_last_error(void) { return g_err.c_str(); }

int slr_device_lds_bytes(void) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 65536;
  return (int)prop.sharedMemPerBlock;
}

int slr_setup(const slr_csr *A, const int32_t *part, int32_t p, const slr_opts *o, void *hip_stream,
              slr_ctx **out) {
  if (!A || !part || !o || !out || !A->rowptr || !A->col || !A->val) return fail(SLR_ERR_ARG, "null argument");
  *out = nullptr;
  if (o->k < 0 || o->k > 64) return fail(SLR_ERR_ARG, "k must be in [0, 64]");
  if (o->theta_mode < SLR_THETA_LAMBDA_K1 || o->theta_mode > SLR_THETA_LAMBDA_S) return fail(SLR_ERR_ARG, "theta_mode");
  if (o->theta_mode == SLR_THETA_EPS && !(o->eps > 0.0)) return fail(SLR_ERR_ARG, "theta_mode eps needs eps > 0");
  if (!(o->cond_K == 0.0 || o->cond_K > 1.0)) return fail(SLR_ERR_ARG, "cond_K must be 0 or > 1");
  if (o->reorth != SLR_REORTH_FULL && o->reorth != SLR_REORTH_PARTIAL) return fail(SLR_ERR_ARG, "reorth");
  if (o->fact_prec != SLR_FP64 && o->fact_prec != SLR_FP32) return fail(SLR_ERR_ARG, "fact_prec");
  if (o->uk_prec < SLR_FP64 || o->uk_prec > SLR_BF16) return fail(SLR_ERR_ARG, "uk_prec");
  if (o->b_fact < SLR_FACT_CHOL || o->b_fact > SLR_FACT_ILDLT) return fail(SLR_ERR_ARG, "b_fact");
  if (o->c_fact != SLR_FACT_CHOL && o->c_fact != SLR_FACT_IC0 && o->c_fact != SLR_FACT_ICT)
    return fail(SLR_ERR_ARG, "c_fact");
  if (!(o->droptol >= 0.0)) return fail(SLR_ERR_ARG, "droptol must be >= 0");
  if (o->c_levels != 1 && o->c_levels != 2) return fail(SLR_ERR_ARG, "c_levels must be 1 or 2");
  if (o->c_levels == 2) {
    if (o->c_order != SLR_CORDER_HID) return fail(SLR_ERR_ARG, "c_levels 2 needs the HID order of C");
    if (o->refactor) return fail(SLR_ERR_ARG, "refactor is not available with c_levels 2");
    if (o->k2 < 0 || o->k2 > 64) return fail(SLR_ERR_ARG, "k2 must be in [0, 64]");
    if (o->lanczos_steps2 < 0) return fail(SLR_ERR_ARG, "lanczos_steps2 must be >= 0");
  }
  if (A->rowptr[A->n] != A->nnz) return fail(SLR_ERR_ARG, "rowptr[n] != nnz");
  if (o->refactor)
    for (int64_t i = 0; i < A->n; ++i)
      if (part[i] == -1) return fail(SLR_ERR_ARG, "refactor is not available with separator labels");
  hipStream_t st = S(hip_stream);
  const double t0 = now_s();
  HostSetup H;
  SetupParams prm;
  prm.b_fact = o->b_fact;
  prm.c_fact = o->c_fact;
  prm.c_order = o->c_order;
  prm.fact_prec = o->fact_prec;
  prm.droptol = o->droptol;
  prm.b_order = o->b_order;
  prm.c_levels = o->c_levels;
  prm.plan = o->refactor != 0;
  if (o->refactor && !((o->b_fact == SLR_FACT_IC0 || o->b_fact == SLR_FACT_ILDLT0) && o->c_fact == SLR_FACT_IC0))
    return fail(SLR_ERR_ARG, "refactor needs zero-fill factors (IC0 / ILDLT0 for B, IC0 for C)");
  if (o->refactor && A->nnz > INT32_MAX) return fail(SLR_ERR_ARG, "refactor takes at most 2^31-1 entries");
  std::string err;
  int rc = host_setup(A->n, A->rowptr, A->col, A->val, part, p, prm, H, err);
  if (rc) return fail(rc, err);
  slr_ctx *c = new slr_ctx();
  (void)hipGetDevice(&c->device);
  {
    // set-up of slr_apply_dd_noalloc's scratch on this device (a failure
    // here only disables that entry point; it retries on its first call)
    char *sp = nullptr;
    (void)scratch_address(c->device, &sp);
  }
  c->opts = *o;
  c->n = H.n;
  c->m = H.m;
  c->s = H.s;
  c->p = H.p;
  c->fact_prec = o->fact_prec;
  c->uk_prec = o->uk_prec;
  c->lds_limit = (size_t)slr_device_lds_bytes();
  c->n_cu = device_cu_count();
  c->perm_h = H.perm;
  auto destroy_fail = [&](int code) {
    slr_destroy(c);
    return code;
  };
  c->perm = c->pool.upload(H.perm);
  c->a_rp = c->pool.upload(H.a_rp);
  c->a_ci = c->pool.upload(H.a_ci);
  c->a_v = c->pool.upload(H.a_v);
  c->nnz_a = (int64_t)H.a_ci.size();
  bool ok = c->perm && c->a_rp && c->a_ci && c->a_v;
  if (H.has_sep) {
    c->sep = true;
    c->et_rp = c->pool.upload(H.et_rp);
    c->et_ci = c->pool.upload(H.et_ci.empty() ? std::vector<int32_t>{0} : H.et_ci);
    c->et_v = c->pool.upload(H.et_v.empty() ? std::vector<double>{0.0} : H.et_v);
    ok = ok && c->et_rp && c->et_ci && c->et_v;
  }
  RfMaps rmaps;
  RfMaps *rm = H.have_plan ? &rmaps : nullptr;
  if (c->fact_prec == SLR_FP64)
    upload_blocks<double>(c, H, c->Bd, c->Cfd, c->Cbd, ok, rm);
  else {
    bool ok2 = true;
    upload_blocks<float>(c, H, c->Bf, c->Cff, c->Cbf, ok2, rm);
    ok = ok && ok2;
  }
  if (!ok) return destroy_fail(fail(SLR_ERR_OOM, "factor upload (or a subdomain above 65535 rows)"));
  if (rm && !rf_upload(c, H, *rm, A)) return destroy_fail(fail(SLR_ERR_OOM, "refactorisation plan"));
  if (H.s1 > 0) {
    slr_ctx::Inner &I = c->ml;
    I.on = true;
    I.s1 = H.s1;
    I.s2 = H.s - H.s1;
    I.nb = (int32_t)H.c1blocks.size();
    for (const Block &b : H.c1blocks)
      if (b.m > 65535) return destroy_fail(fail(SLR_ERR_ARG, "a connector above 65535 rows"));
    const bool ok2 = c->fact_prec == SLR_FP64 ? upload_inner<double>(c, H, I.Bd, I.C2fd, I.C2bd)
                                              : upload_inner<float>(c, H, I.Bf, I.C2ff, I.C2bf);
    if (!ok2) return destroy_fail(fail(SLR_ERR_OOM, "inner interface solver upload"));
    I.f_lev_h = H.c2fwd.levptr;
    I.b_lev_h = H.c2bwd.levptr;
    I.f_nlev = H.c2fwd.nlev;
    I.b_nlev = H.c2bwd.nlev;
    I.one_wg = std::max(I.f_nlev, I.b_nlev) > 8;
    if (std::max(I.f_nlev, I.b_nlev) > 2) {
      I.f_group = sweep_group(H.c2fwd);
      I.b_group = sweep_group(H.c2bwd);
    }
    if (I.one_wg && sizeof(int32_t) * (size_t)(std::max(I.f_nlev, I.b_nlev) + 1) > c->lds_limit)
      return destroy_fail(fail(SLR_ERR_ARG, "inner level schedule too deep for one workgroup"));
    I.nnz_L1 = H.nnz_LC1;
    I.nnz_L2 = H.nnz_LC2;
    I.k2 = o->k2 > 0 ? o->k2 : o->k;
    int32_t R1 = 0, st1 = 0;
    if (!b_lds_plan_sz(I.max_m, I.max_lev, I.max_level_bytes, I.data_bytes, 1, 8, R1, st1, c->lds_limit))
      return destroy_fail(fail(SLR_ERR_ARG, "largest connector does not fit one workgroup's LDS"));
  }
  c->cf_lev_h = H.cfwd.levptr;
  c->cb_lev_h = H.cbwd.levptr;
  c->cf_nlev = H.cfwd.nlev;
  c->cb_nlev = H.cbwd.nlev;
  c->cb_nnz = (int64_t)H.cbwd.ci.size();
  // shallow interface schedules (multicolour) run one launch per level
  c->c_one_wg = std::max(c->cf_nlev, c->cb_nlev) > 8;
  // mean entries per row >= 8: one launch per level, lanes per row by length
  if (!(std::max(c->cf_nlev, c->cb_nlev) <= 2)) {
    c->cf_group = sweep_group(H.cfwd);
    c->cb_group = sweep_group(H.cbwd);
  }
  c->c_two_level = !c->ml.on && std::max(c->cf_nlev, c->cb_nlev) <= 2;
  if (c->c_one_wg && sizeof(int32_t) * (size_t)(std::max(c->cf_nlev, c->cb_nlev) + 1) > c->lds_limit)
    return destroy_fail(fail(SLR_ERR_ARG, "interface level schedule too deep for one workgroup"));
  {
    int32_t R1 = 0, st1 = 0;
    if (!b_lds_plan(c, 1, c->fact_prec == SLR_FP64 ? 8 : 4, R1, st1) || !b_lds_plan(c, 1, 8, R1, st1))
      return destroy_fail(fail(SLR_ERR_ARG, "largest subdomain does not fit one workgroup's LDS"));
  }
  // stats
  slr_info &I = c->info;
  I.n = c->n; I.m = c->m; I.s = c->s; I.p = c->p;
  I.b_levels_max = c->b_max_lev;
  I.c_levels = H.cfwd.nlev;
  I.c_colors = H.c_colors;
  I.nnz_LB = 0;
  I.m_min = INT64_MAX; I.m_max = 0;
  for (const auto &b : H.blocks) {
    I.nnz_LB += b.nnz_L;
    I.m_min = std::min<int64_t>(I.m_min, b.m);
    I.m_max = std::max<int64_t>(I.m_max, b.m);
  }
  I.nnz_LC = H.nnz_LC;
  I.nnz_E = H.nnz_E;
  I.nnz_A = c->nnz_a;
  I.setup_host_s = now_s() - t0;
  I.tune_b_lds_div1 = I.tune_b_lds_divM = 1;
  // low-rank part(s)
  const double t1 = now_s();
  std::vector<double> v0s;
  const double *v0p = o->lanczos_v0 ? o->lanczos_v0 : seeded_v0(c->n, o->seed, v0s);
  if ((rc = ws_ensure(c, c->ws, 1))) return destroy_fail(rc);
  if (c->ml.on) {
    if ((rc = lanczos_inner(c, v0p, st))) return destroy_fail(rc);
    if ((rc = ws_ensure(c, c->ws, 1))) return destroy_fail(rc);
    I.s1 = c->ml.s1;
    I.k2 = c->ml.k2;
    I.lanczos_steps2 = c->ml.steps;
    I.c1_levels = c->ml.max_lev;
    I.c2_levels = c->ml.f_nlev;
    I.theta2 = c->ml.theta2;
    I.nnz_LC1 = H.nnz_LC1;
    I.nnz_LC2 = H.nnz_LC2;
    I.nnz_F = (int64_t)H.ft_ci.size();
  }
  if (o->U_in && o->k_in > 0) {
    if (o->k_in > 64 || !o->lambda_in) return destroy_fail(fail(SLR_ERR_ARG, "imported low-rank part"));
    c->k = o->k_in;
    std::vector<double> Ucm(o->U_in, o->U_in + (size_t)c->s * c->k);   // column-major s x k
    c->U64 = c->lrpool.upload(Ucm);
    if (!c->U64) return destroy_fail(fail(SLR_ERR_OOM, "U"));
    c->lam_h.assign(o->lambda_in, o->lambda_in + c->k);
    c->ritz_h = c->lam_h;
    c->theta = o->theta_in;
    if ((rc = finish_lowrank(c, st))) return destroy_fail(rc);
  } else if (o->k > 0 && c->s > 0) {
    c->k = o->k;
    if ((rc = lanczos_build(c, o->k, 0, v0p, st))) return destroy_fail(rc);
  } else {
    c->k = 0;
    c->theta = 0.0;
    if ((rc = finish_lowrank(c, st))) return destroy_fail(rc);
  }
  HIPCHK(hipStreamSynchronize(st));
  I.k = c->k;
  I.theta = c->theta;
  I.setup_lanczos_s = now_s() - t1;
  if ((rc = ws_ensure(c, c->ws, 1))) return destroy_fail(rc);
  I.device_bytes = c->pool.bytes + c->lrpool.bytes + c->ws.pool.bytes;
  *out = c;
  return SLR_OK;
}

int slr_update_lowrank(slr_ctx *c, int32_t k, int32_t lanczos_steps, const double *lanczos_v0,
                       void *hip_stream) {
  if (!c || k < 0 || k > 64 || lanczos_steps < 0) return fail(SLR_ERR_ARG, "bad update arguments");
  if (c->live_batches > 0) return fail(SLR_ERR_ARG, "the context still has batches");
  hipStream_t st = S(hip_stream);
  HIPCHK(hipStreamSynchronize(st));
  c->opts.k = k;
  c->opts.lanczos_steps = lanczos_steps;
  const double t1 = now_s();
  int rc;
  if (k > 0 && c->s > 0) {
    std::vector<double> v0;
    const double *v0p = lanczos_v0 ? lanczos_v0 : seeded_v0(c->n, c->opts.seed, v0);
    rc = lanczos_build(c, k, 0, v0p, st);
  } else {
    c->lrpool.release();
    c->U = nullptr;
  c->Urm = nullptr;
    c->U64 = nullptr;
    c->dsc = nullptr;
    c->k = 0;
    c->theta = 0.0;
    c->lam_h.clear();
    c->ritz_h.clear();
    rc = finish_lowrank(c, st);
  }
  return rc ? rc : lowrank_done(c, t1, st);
}

int slr_grow_lowrank(slr_ctx *c, int32_t k_add, int32_t lanczos_steps, const double *lanczos_v0,
                     void *hip_stream) {
  if (!c || k_add <= 0 || lanczos_steps < 0 || c->k + k_add > 64) return fail(SLR_ERR_ARG, "bad grow arguments");
  if (c->live_batches > 0) return fail(SLR_ERR_ARG, "the context still has batches");
  if (c->s == 0) return fail(SLR_ERR_ARG, "no interface");
  hipStream_t st = S(hip_stream);
  HIPCHK(hipStreamSynchronize(st));
  const int32_t steps_keep = c->opts.lanczos_steps;
  c->opts.lanczos_steps = lanczos_steps;
  const double t1 = now_s();
  std::vector<double> v0;
  const double *v0p = lanczos_v0 ? lanczos_v0 : seeded_v0(c->n, c->opts.seed, v0);
  const int rc = lanczos_build(c, k_add, c->k, v0p, st);
  c->opts.lanczos_steps = steps_keep;
  if (rc) return rc;
  c->opts.k = c->k;
  return lowrank_done(c, t1, st);
}

int slr_refactor(slr_ctx *c, const double *val, int32_t on_device, void *hip_stream) {
  if (!c || !val) return fail(SLR_ERR_ARG, "null argument");
  auto &R = c->rf;
  if (!R.on) return fail(SLR_ERR_ARG, "the context was set up without opts.refactor");
  if (c->live_batches > 0) return fail(SLR_ERR_ARG, "the context still has batches");
  hipStream_t st = S(hip_stream);
  HIPCHK(hipMemsetAsync(R.err, 0, 4 * sizeof(int), st));
  if (on_device) {
    HIPCHK(hipMemcpyAsync(R.val, val, sizeof(double) * R.nnz, hipMemcpyDeviceToDevice, st));
    launch_mirror_check(R.nnz, R.tr, R.val, R.err + 2, st);
  } else {
    for (int64_t e = 0; e < R.nnz; ++e)
      if (val[R.tr_h[e]] != val[e]) return fail(SLR_ERR_NOT_SYMMETRIC, "A is not symmetric (values must match)");
    // the previous call's copy out of the staging buffer has completed (it
    // synchronises before returning)
    std::memcpy(R.stage, val, sizeof(double) * R.nnz);
    HIPCHK(hipMemcpyAsync(R.val, R.stage, sizeof(double) * R.nnz, hipMemcpyHostToDevice, st));
  }
  // factors into their own value arrays (level by level)
  launch_gather(R.fb.nnz, R.fb.src, R.val, R.fb.v, st);
  launch_gather(R.fc.nnz, R.fc.src, R.val, R.fc.v, st);
  for (size_t l = 0; l + 1 < R.fb.lev.size(); ++l)
    launch_fact_level(R.fb.rp, R.fb.ci, R.fb.v, R.fb.rows, R.fb.lev[l], R.fb.lev[l + 1], R.fb.kind == 2, R.err, st);
  for (size_t l = 0; l + 1 < R.fc.lev.size(); ++l)
    launch_fact_level(R.fc.rp, R.fc.ci, R.fc.v, R.fc.rows, R.fc.lev[l], R.fc.lev[l + 1], 0, R.err + 1, st);
  int e[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(e, R.err, sizeof(e), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // a failed pivot leaves every stored coefficient as it was
  if (e[2]) return fail(SLR_ERR_NOT_SYMMETRIC, "A is not symmetric (values must match)");
  if (e[0]) return fail(SLR_ERR_BREAKDOWN, "refactorisation of a B_i failed (pivot)");
  if (e[1]) return fail(SLR_ERR_C_NOT_SPD, "refactorisation of C failed (pivot)");
  launch_gather(c->nnz_a, R.a_src, R.val, c->a_v, st);
  if (c->fact_prec == SLR_FP64)
    rf_pack_all<double>(c, c->Bd, c->Cfd, c->Cbd, st);
  else
    rf_pack_all<float>(c, c->Bf, c->Cff, c->Cbf, st);
  HIPCHK(hipStreamSynchronize(st));
  return SLR_OK;
}

int slr_time_kernel(slr_ctx *c, int32_t which, int32_t nrhs, int32_t reps, void *hip_stream, double *ms) {
  if (!c || !ms || nrhs <= 0 || reps <= 0 || which < 0 || which > 6) return fail(SLR_ERR_ARG, "bad timing args");
  hipStream_t st = S(hip_stream);
  int rc = perm_ws(c, nrhs);
  if (rc) return rc;
  if ((rc = ws_ensure(c, c->ws, nrhs))) return rc;
  const int64_t n = c->n, m = c->m, s = c->s;
  // deterministic filler: r = 1 everywhere, then one apply to get realistic z
  std::vector<double> ones((size_t)n * nrhs, 1.0);
  HIPCHK(hipMemcpyAsync(c->pr, ones.data(), sizeof(double) * ones.size(), hipMemcpyHostToDevice, st));
  if ((rc = apply_dd(c, c->ws, c->pr, n, c->pz, n, nrhs, st))) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto one = [&]() -> int {
    switch (which) {
      case 0: return bsolve_first(c, c->ws, c->pr, n, nrhs, st);
      case 1:
        if (c->ml.on)
          return c_lower(c, c->ws.W, s, nrhs, false, c->ws.W2, s, c->ws, st);
        if (c->c_two_level)
          csweep2(c, true, c->ws.W, s, c->ws.W2, s, nrhs, false, st);
        else
          csweep(c, true, c->ws.W, s, nrhs, false, st);
        return SLR_OK;
      case 2: lowrank(c, c->ws, c->ws.W2, s, c->ws.W, s, nrhs, st); return SLR_OK;
      case 3:
        if (c->ml.on)
          return c_upper(c, c->pz + m, n, nrhs, false, c->ws.W2, s, c->ws, st);
        if (c->c_two_level)
          csweep2(c, false, c->ws.W, s, c->pz + m, n, nrhs, false, st);
        else
          csweep(c, false, c->pz + m, n, nrhs, false, st);
        return SLR_OK;
      case 4: {
        BArgs a;
        a.f = c->pr; a.ldf = n; a.a_f = 1.0;
        a.y = c->pz + m; a.ldy = n; a.b_y = -1.0;
        a.u = c->pz; a.ldu = n;
        a.nrhs = nrhs;
        return bsolve(c, a, false, st);
      }
      case 5: return apply_dd(c, c->ws, c->pr, n, c->pz, n, nrhs, st);
      default: launch_spmv(n, c->a_rp, c->a_ci, c->a_v, c->pr, n, c->pz, n, nrhs, st); return SLR_OK;
    }
  };
  if ((rc = one())) return rc;
  HIPCHK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i)
    if ((rc = one())) return rc;
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float t = 0.0f;
  HIPCHK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  return SLR_OK;
}

int slr_autotune(slr_ctx *c, int32_t nrhs, int32_t reps, void *hip_stream) {
  if (!c || nrhs <= 0 || nrhs > 128) return fail(SLR_ERR_ARG, "bad autotune arguments");
  if (c->live_batches > 0) return fail(SLR_ERR_ARG, "the context still has batches");
  if (reps <= 0) reps = 3;
  const bool one = nrhs == 1;
  slr_ctx::BTune &tu = one ? c->tune1 : c->tuneM;
  const slr_ctx::BTune keep = tu;
  const size_t tcb = (c->fact_prec == SLR_FP64) ? 8 : 4;
  // candidates: threads per workgroup, LDS share, most columns per workgroup
  std::vector<slr_ctx::BTune> cand;
  for (int32_t th : {1024, 512, 256})
    for (int32_t div : {1, 2, 4}) {
      if (th * div > 2048 || th * div < 512) continue;   // at most 32 waves per CU, at least 8 resident
      int32_t R = 0, stage = 0;
      if (!b_lds_plan(c, one ? 1 : std::min(nrhs, 16), tcb, R, stage, c->lds_limit / div)) continue;
      for (int32_t r = R; r >= 1; r = (r > 1 ? std::max(1, r / 2) : 0)) {
        cand.push_back(slr_ctx::BTune{th, div, r, 0});
        // several columns: the same shape as a persistent grid walking a
        // longest-first schedule of (subdomain, column group) items
        if (!one) {
          cand.push_back(slr_ctx::BTune{th, div, r, 1});
          cand.push_back(slr_ctx::BTune{th, div, r, 2});
        }
        if (one || r == 1) break;
      }
    }
  double best = 1e30;
  slr_ctx::BTune pick = keep;
  // the built-in plan first, as the reference
  tu = slr_ctx::BTune{};
  double ms = 0.0;
  int rc = slr_time_kernel(c, 0, nrhs, reps, hip_stream, &ms);
  if (rc) {
    tu = keep;
    return rc;
  }
  best = ms;
  pick = tu;
  for (const auto &cd : cand) {
    tu = cd;
    rc = slr_time_kernel(c, 0, nrhs, reps, hip_stream, &ms);
    if (rc) {
      tu = keep;
      return rc;
    }
    if (ms < best * 0.98) {
      best = ms;
      pick = cd;
    }
  }
  tu = pick;
  // chunks of the rank-k partials (the sums' grouping: every later apply of
  // this context, alone or in a batch, uses the same value)
  if (c->k > 0) {
    int32_t *nb = c->uk_prec == SLR_BF16 ? &c->lrm_nblk : &c->lr_nblk;
    const int32_t nb0 = *nb;
    double bl = 1e30;
    int32_t bnb = nb0;
    for (int32_t v : {nb0, 128, 256, 512, 1024, 2048}) {
      *nb = v;
      if ((rc = ws_ensure(c, c->ws, nrhs))) return rc;
      if ((rc = slr_time_kernel(c, 2, nrhs, reps, hip_stream, &ms))) {
        *nb = nb0;
        return rc;
      }
      if (ms < bl * (v == nb0 ? 1.0 : 0.98)) {
        bl = ms;
        bnb = v;
      }
    }
    *nb = bnb;
    if (c->uk_prec != SLR_BF16) c->lr_nblk_tuned = bnb;
    if ((rc = ws_ensure(c, c->ws, nrhs))) return rc;
  }
  c->info.tune_b_threads1 = c->tune1.threads;
  c->info.tune_b_lds_div1 = c->tune1.lds_div;
  c->info.tune_b_threadsM = c->tuneM.threads;
  c->info.tune_b_lds_divM = c->tuneM.lds_div;
  c->info.tune_b_rmaxM = c->tuneM.threads ? c->tuneM.rmax : 0;
  c->info.tune_b_persistentM = c->tuneM.threads ? c->tuneM.persistent : 0;
  c->info.lr_chunks = c->uk_prec == SLR_BF16 ? c->lrm_nblk : c->lr_nblk;
  return SLR_OK;
}

int slr_set_bsolve_plan(slr_ctx *c, int32_t several, int32_t threads, int32_t lds_div, int32_t rmax,
                        int32_t persistent) {
  if (!c) return fail(SLR_ERR_ARG, "null");
  if (c->live_batches > 0) return fail(SLR_ERR_ARG, "the context still has batches");
  slr_ctx::BTune &tu = several ? c->tuneM : c->tune1;
  if (threads == 0) {
    tu = slr_ctx::BTune{};
  } else {
    if ((threads != 256 && threads != 512 && threads != 1024) || lds_div < 1 || lds_div > 8 || rmax < 1 ||
        rmax > 16 || persistent < 0 || persistent > 2)
      return fail(SLR_ERR_ARG, "bad B launch plan");
    int32_t R = 0, stage = 0;
    const size_t tcb = (c->fact_prec == SLR_FP64) ? 8 : 4;
    if (!b_lds_plan(c, several ? std::min(rmax, 16) : 1, tcb, R, stage, c->lds_limit / lds_div) ||
        !b_lds_plan(c, 1, 8, R, stage, c->lds_limit / lds_div))
      return fail(SLR_ERR_ARG, "the largest subdomain does not fit that share of the LDS");
    tu = slr_ctx::BTune{threads, lds_div, rmax, persistent};
  }
  c->info.tune_b_threads1 = c->tune1.threads;
  c->info.tune_b_lds_div1 = c->tune1.lds_div;
  c->info.tune_b_threadsM = c->tuneM.threads;
  c->info.tune_b_lds_divM = c->tuneM.lds_div;
  c->info.tune_b_rmaxM = c->tuneM.threads ? c->tuneM.rmax : 0;
  c->info.tune_b_persistentM = c->tuneM.threads ? c->tuneM.persistent : 0;
  return SLR_OK;
}

int slr_analyze(const slr_csr *A, const int32_t *part, int32_t p, const slr_opts *o, slr_info *info,
                int64_t *perm) {
  if (!A || !part || !o || !info || !A->rowptr || !A->col || !A->val) return fail(SLR_ERR_ARG, "null argument");
  if (A->rowptr[A->n] != A->nnz) return fail(SLR_ERR_ARG, "rowptr[n] != nnz");
  const double t0 = now_s();
  HostSetup H;
  SetupParams prm;
  prm.b_fact = o->b_fact;
  prm.c_fact = o->c_fact;
  prm.c_order = o->c_order;
  prm.fact_prec = o->fact_prec;
  prm.droptol = o->droptol;
  prm.b_order = o->b_order;
  prm.c_levels = o->c_levels;
  if (o->c_levels != 1 && o->c_levels != 2) return fail(SLR_ERR_ARG, "c_levels must be 1 or 2");
  std::string err;
  int rc = host_setup(A->n, A->rowptr, A->col, A->val, part, p, prm, H, err);
  if (rc) return fail(rc, err);
  std::memset(info, 0, sizeof(*info));
  info->n = H.n; info->m = H.m; info->s = H.s; info->p = H.p;
  info->c_levels = H.cfwd.nlev;
  info->c_colors = H.c_colors;
  info->nnz_LC = H.nnz_LC;
  info->nnz_E = H.nnz_E;
  info->nnz_A = (int64_t)H.a_ci.size();
  info->m_min = INT64_MAX;
  const int64_t fb = o->fact_prec == SLR_FP32 ? 4 : 8;
  int64_t bytes = (int64_t)H.a_ci.size() * 12 + (H.n + 1) * 8 + H.n * 8;
  {
    const int32_t Kfix = packed_width(H.blocks);
    for (const auto &b : H.blocks) {
      const std::vector<int32_t> pos = lds_positions(b, Kfix > 0, (int)fb);
      for (int32_t r = 0; r < b.m; ++r)
        if (pos[r] != r) {
          ++info->b_lds_level_order;
          break;
        }
    }
  }
  for (const auto &b : H.blocks) {
    info->nnz_LB += b.nnz_L;
    info->b_levels_max = std::max({info->b_levels_max, b.fwd.nlev, b.bwd.nlev});
    info->m_min = std::min<int64_t>(info->m_min, b.m);
    info->m_max = std::max<int64_t>(info->m_max, b.m);
    bytes += (int64_t)(b.fwd.ci.size() + b.bwd.ci.size()) * (4 + fb) + (int64_t)b.m * (2 * (8 + fb) + 10) +
             (int64_t)(b.e_q.size() + b.t_j.size()) * (4 + fb);
  }
  bytes += (int64_t)(H.cfwd.ci.size() + H.cbwd.ci.size()) * (4 + fb) + H.s * 2 * (8 + fb);
  if (H.s1 > 0) {
    // the recursive interface solver: C1 blocks, C2 sweeps, F^T and U2
    const int32_t k2 = o->k2 > 0 ? o->k2 : o->k;
    info->s1 = H.s1;
    info->k2 = k2;
    info->c2_levels = H.c2fwd.nlev;
    info->nnz_LC1 = H.nnz_LC1;
    info->nnz_LC2 = H.nnz_LC2;
    info->nnz_F = (int64_t)H.ft_ci.size();
    for (const auto &b : H.c1blocks) {
      info->c1_levels = std::max({info->c1_levels, b.fwd.nlev, b.bwd.nlev});
      bytes += (int64_t)(b.fwd.ci.size() + b.bwd.ci.size()) * (4 + fb) + (int64_t)b.m * (2 * (8 + fb) + 2) +
               (int64_t)b.e_q.size() * (4 + fb);
    }
    bytes += (int64_t)(H.c2fwd.ci.size() + H.c2bwd.ci.size()) * (4 + fb) + (H.s - H.s1) * 2 * (8 + fb) +
             (int64_t)H.ft_ci.size() * 12 + (H.s - H.s1) * (int64_t)k2 * 16;
  }
  const int64_t ub = o->uk_prec == SLR_FP64 ? 8 : (o->uk_prec == SLR_FP32 ? 4 : 2);
  bytes += H.s * (int64_t)o->k * (8 + (o->uk_prec == SLR_FP64 ? 0 : ub));
  info->device_bytes = bytes;
  info->setup_host_s = now_s() - t0;
  if (perm) std::copy(H.perm.begin(), H.perm.end(), perm);
  return SLR_OK;
}

void slr_destroy(slr_ctx *c) {
  if (!c) return;
  if (c->rf.stage) (void)hipHostFree(c->rf.stage);
  if (c->hst) (void)hipHostFree(c->hst);
  c->lz.release();
  c->gm.release();
  if (c->hfl) (void)hipHostFree(c->hfl);
  for (hipEvent_t e : c->pev)
    if (e) (void)hipEventDestroy(e);
  c->rf.pool.release();
  c->pool.release();
  c->ws.pool.release();
  c->lrpool.release();
  c->ppool.release();
  c->spool.release();
  c->schedpool.release();
  delete c;
}

int slr_query(const slr_ctx *c, slr_info *info) {
  if (!c || !info) return fail(SLR_ERR_ARG, "null");
  *info = c->info;
  info->lr_chunks = c->uk_prec == SLR_BF16 ? c->lrm_nblk : c->lr_nblk;
  info->device_bytes =
      c->pool.bytes + c->lrpool.bytes + c->ws.pool.bytes + c->spool.bytes + c->ppool.bytes + c->rf.pool.bytes +
      c->schedpool.bytes + (int64_t)(c->lz.cap + c->gm.cap);
  return SLR_OK;
}

int slr_export(const slr_ctx *c, int64_t *perm, double *ritz, double *lambda, double *U, double *alpha,
               double *beta) {
  if (!c) return fail(SLR_ERR_ARG, "null");
  if (perm) std::copy(c->perm_h.begin(), c->perm_h.end(), perm);
  if (ritz) std::copy(c->ritz_h.begin(), c->ritz_h.end(), ritz);
  if (lambda) std::copy(c->lam_h.begin(), c->lam_h.end(), lambda);
  if (alpha) std::copy(c->alpha_h.begin(), c->alpha_h.end(), alpha);
  if (beta) std::copy(c->beta_h.begin(), c->beta_h.end(), beta);
  if (U && c->k > 0)
    HIPCHK(hipMemcpy(U, c->U64, sizeof(double) * (size_t)c->s * c->k, hipMemcpyDeviceToHost));
  return SLR_OK;
}

int slr_export_inner(const slr_ctx *c, double *ritz2, double *lambda2, double *U2) {
  if (!c) return fail(SLR_ERR_ARG, "null");
  if (!c->ml.on) return fail(SLR_ERR_ARG, "the context has no recursive interface solver");
  const slr_ctx::Inner &I = c->ml;
  if (ritz2) std::copy(I.ritz_h.begin(), I.ritz_h.end(), ritz2);
  if (lambda2) std::copy(I.lam_h.begin(), I.lam_h.end(), lambda2);
  if (U2 && I.k2 > 0) HIPCHK(hipMemcpy(U2, I.U2, sizeof(double) * (size_t)I.s2 * I.k2, hipMemcpyDeviceToHost));
  return SLR_OK;
}

int slr_export_setup(const slr_ctx *c, void *buf, size_t cap, size_t *bytes) {
  if (!c || !bytes) return fail(SLR_ERR_ARG, "null");
  if (c->ml.on) return fail(SLR_ERR_ARG, "a context with the recursive interface solver cannot be serialised");
  if (c->sep) return fail(SLR_ERR_ARG, "a context of an edge-based partition cannot be serialised");
  std::vector<uint8_t> blob;
  const int rc = export_setup(c, blob);
  if (rc) return rc;
  *bytes = blob.size();
  if (!buf) return SLR_OK;
  if (cap < blob.size()) return fail(SLR_ERR_ARG, "buffer smaller than the serialised setup (see *bytes)");
  std::memcpy(buf, blob.data(), blob.size());
  return SLR_OK;
}

int slr_import(const void *buf, size_t bytes, void *hip_stream, slr_ctx **out) {
  if (!buf || !out) return fail(SLR_ERR_ARG, "null");
  *out = nullptr;
  return import_setup((const uint8_t *)buf, bytes, S(hip_stream), out);
}

void slr_set_allocator(slr_alloc_fn alloc, slr_free_fn free_, void *user) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  if (alloc && free_) {
    g_alloc.alloc = alloc;
    g_alloc.free_ = free_;
    g_alloc.user = user;
  } else {
    g_alloc = AllocHook{};
  }
}

int slr_trim(slr_ctx *c) {
  if (!c) return fail(SLR_ERR_ARG, "null");
  c->lz.release();
  c->gm.release();
  c->spool.release();
  c->scap = 0;
  c->sX = c->sR = c->sZ = c->sP = c->sQ = c->sS = c->sB = nullptr;
  c->sst = nullptr;
  c->spart = c->spart2 = nullptr;
  c->scnt = nullptr;
  c->ppool.release();
  c->pcap = 0;
  c->pr = c->pz = nullptr;
  if (c->ws.cap > 1) {
    c->ws.pool.release();
    c->ws.W = nullptr;
    c->ws.cap = 0;
    const int rc = ws_ensure(c, c->ws, 1);
    if (rc) return rc;
  }
  return SLR_OK;
}

int slr_apply_dd(slr_ctx *c, const double *r_dev, double *z_dev, int32_t nrhs, void *hip_stream) {
  if (!c || !r_dev || !z_dev || nrhs < 0) return fail(SLR_ERR_ARG, "bad apply arguments");
  return apply_dd(c, c->ws, r_dev, c->n, z_dev, c->n, nrhs, S(hip_stream));
}

int slr_apply_dd_noalloc(slr_ctx *c, const double *r_dev, double *z_dev, int32_t nrhs, void *hip_stream) {
  if (!c || !r_dev || !z_dev || nrhs < 0) return fail(SLR_ERR_ARG, "bad apply arguments");
  if (nrhs == 0) return SLR_OK;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != c->device) return fail(SLR_ERR_ARG, "the context's device must be current");
  char *base = nullptr;
  int rc = scratch_address(dev, &base);
  if (rc) return rc;
  // the apply's scratch, carved as apply_dd's workspace would allocate it
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const int32_t nb = ws_chunks(c);
  const int32_t kk = ws_rank(c);
  const size_t s1 = (size_t)std::max<int64_t>(c->s, 1);
  const size_t bW = al(sizeof(double) * s1 * nrhs);
  const size_t bP = al(sizeof(double) * (size_t)nb * nrhs * kk);
  const size_t bC = al(sizeof(double) * (size_t)kk * nrhs);
  const size_t bZ = c->sep ? al(sizeof(double) * (size_t)std::max<int64_t>(c->m, 1) * nrhs) : 0;
  const size_t need = 2 * bW + bP + bC + bZ + 256;
  if (need > kNoAllocScratchBytes)
    return fail(SLR_ERR_ARG, "slr_apply_dd_noalloc needs " + std::to_string(need) + " bytes of scratch for " +
                                 std::to_string(nrhs) + " columns; the fixed scratch holds " +
                                 std::to_string(kNoAllocScratchBytes));
  ApplyWS w;
  w.W = (double *)base;
  w.W2 = (double *)(base + bW);
  w.lr_part = (double *)(base + 2 * bW);
  w.cbuf = (double *)(base + 2 * bW + bP);
  w.Z = c->sep ? (double *)(base + 2 * bW + bP + bC) : nullptr;
  w.counter = (unsigned int *)(base + 2 * bW + bP + bC + bZ);   // unused by the apply's kernels
  w.cap = nrhs;
  w.k = kk;
  w.nblk = nb;
  return apply_dd(c, w, r_dev, c->n, z_dev, c->n, nrhs, S(hip_stream));
}

int slr_apply(slr_ctx *c, const double *r_dev, double *z_dev, int32_t nrhs, void *hip_stream) {
  if (!c || !r_dev || !z_dev || nrhs < 0) return fail(SLR_ERR_ARG, "bad apply arguments");
  if (nrhs == 0) return SLR_OK;
  hipStream_t st = S(hip_stream);
  int rc = perm_ws(c, nrhs);
  if (rc) return rc;
  launch_permute(c->n, c->perm, r_dev, c->n, c->pr, c->n, nrhs, false, st);
  rc = apply_dd(c, c->ws, c->pr, c->n, c->pz, c->n, nrhs, st);
  if (rc == SLR_OK) launch_permute(c->n, c->perm, c->pz, c->n, z_dev, c->n, nrhs, true, st);
  return rc;
}

int slr_spmv(slr_ctx *c, const double *x_dev, double *y_dev, int32_t nrhs, void *hip_stream) {
  if (!c || !x_dev || !y_dev || nrhs < 0) return fail(SLR_ERR_ARG, "bad spmv arguments");
  if (nrhs == 0) return SLR_OK;
  hipStream_t st = S(hip_stream);
  int rc = perm_ws(c, nrhs);
  if (rc) return rc;
  launch_permute(c->n, c->perm, x_dev, c->n, c->pr, c->n, nrhs, false, st);
  launch_spmv(c->n, c->a_rp, c->a_ci, c->a_v, c->pr, c->n, c->pz, c->n, nrhs, st);
  launch_permute(c->n, c->perm, c->pz, c->n, y_dev, c->n, nrhs, true, st);
  return SLR_OK;
}

size_t slr_solve_workspace_bytes(const slr_ctx *c, int32_t nrhs, const slr_solve_opts *so) {
  if (!c) return 0;
  slr_solve_opts d;
  slr_default_solve_opts(&d);
  if (!so) so = &d;
  size_t n = (size_t)c->n;
  if (so->method == SLR_FGMRES) {
    ArenaCount ac;
    FgmresWS fw;
    fgmres_layout(ac, c->n, fgmres_restart(so->restart), fw);
    return ac.want;
  }
  return sizeof(double) * n * nrhs * 7 + sizeof(KState) * nrhs + sizeof(double) * RED_NBLK * nrhs * 5 +
         sizeof(double) * (size_t)c->s * nrhs;
}

}  // extern "C"

namespace {

int solve_ws(slr_ctx *c, int32_t nrhs) {
  if (c->scap >= nrhs && c->sX) return SLR_OK;
  c->spool.release();
  const size_t n = (size_t)c->n;
  c->sX = c->spool.alloc<double>(n * nrhs);
  c->sR = c->spool.alloc<double>(n * nrhs);
  c->sZ = c->spool.alloc<double>(n * nrhs);
  c->sP = c->spool.alloc<double>(n * nrhs);
  c->sQ = c->spool.alloc<double>(n * nrhs);
  c->sS = c->spool.alloc<double>(n * nrhs);
  c->sB = c->spool.alloc<double>(n * nrhs);
  c->sst = c->spool.alloc<KState>(nrhs);
  c->spart = c->spool.alloc<double>((size_t)RED_NBLK * nrhs * 4);
  c->spart2 = c->spool.alloc<double>((size_t)RED_NBLK * nrhs);
  c->scnt = c->spool.alloc<unsigned int>(4);
  if (!c->sX || !c->sR || !c->sZ || !c->sP || !c->sQ || !c->sS || !c->sB || !c->sst || !c->spart || !c->spart2 ||
      !c->scnt)
    return fail(SLR_ERR_OOM, "solve workspace");
  HIPCHK(hipMemset(c->scnt, 0, 4 * sizeof(unsigned int)));
  c->scap = nrhs;
  return SLR_OK;
}

KArgs kargs(double *X, double *R, double *Z, double *P, double *Q, double *S, int64_t ld, KState *st, double *part,
            double *part2, int maxit, double rtol) {
  KArgs K;
  K.X = X; K.R = R; K.Z = Z; K.P = P; K.Q = Q; K.S = S;
  K.ld = ld;
  K.st = st;
  K.part = part;
  K.part2 = part2;
  K.counter = nullptr;
  K.nblk = RED_NBLK;
  K.maxit = maxit;
  K.rtol2 = rtol * rtol;
  return K;
}

// CG / flexible CG (one reduction phase per iteration) start on columns
// [c0, c0+nc) whose R holds b (internal order): x = 0 and the state; it0 is
// the global index of their first iteration, which applies the
// preconditioner to r = b like every other.
int cg_start(slr_ctx *c, const KArgs &K, int32_t c0, int32_t nc, int flexible, int32_t it0, hipStream_t st) {
  launch_cg(CG_INIT, c->n, nullptr, nullptr, nullptr, K, c0, nc, flexible, it0, st);
  launch_cg(CG_START, c->n, nullptr, nullptr, nullptr, K, c0, nc, flexible, it0, st);
  return SLR_OK;
}

// one iteration (global index it) of every column in [c0, c0+nc):
// z = M^{-1} r, then w = A z with the partials, then the update.  tiles:
// the column-tile SpMV for any nc (batches, whose results must not depend
// on how many columns are in flight).
int cg_iter(slr_ctx *c, ApplyWS &w, const KArgs &K, int32_t c0, int32_t nc, int flexible, int32_t it,
            hipStream_t st, bool tiles = false) {
  int rc = apply_dd(c, w, K.R + (int64_t)c0 * K.ld, K.ld, K.Z + (int64_t)c0 * K.ld, K.ld, nc, st);
  if (rc) return rc;
  launch_cg(tiles ? CG_SPMV_TILES : CG_SPMV, c->n, c->a_rp, c->a_ci, c->a_v, K, c0, nc, flexible, it, st);
  launch_cg(CG_UPDATE, c->n, nullptr, nullptr, nullptr, K, c0, nc, flexible, it, st);
  return SLR_OK;
}

int poll_events(slr_ctx *c) {
  for (hipEvent_t &e : c->pev)
    if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  return SLR_OK;
}

int solve_cg(slr_ctx *c, const double *b_dev, double *x_dev, int32_t nrhs, const slr_solve_opts &so,
             slr_solve_info *info, hipStream_t st) {
  int rc = solve_ws(c, nrhs);
  if (rc) return rc;
  const int64_t n = c->n;
  const int flexible = so.method == SLR_FCG;
  KArgs K = kargs(c->sX, c->sR, c->sZ, c->sP, c->sQ, c->sS, n, c->sst, c->spart, c->spart2, so.maxit, so.rtol);
  launch_permute(n, c->perm, b_dev, n, c->sB, n, nrhs, false, st);
  launch_axpby(n, nrhs, 1.0, c->sB, n, 0.0, c->sR, n, st);
  if ((rc = cg_start(c, K, 0, nrhs, flexible, 1, st))) return rc;
  if (c->hcap < nrhs) {
    if (c->hst) (void)hipHostFree(c->hst);
    c->hst = nullptr;
    c->hcap = 0;
    HIPCHK(hipHostMalloc((void **)&c->hst, sizeof(KState) * 2 * (size_t)nrhs, hipHostMallocDefault));
    c->hcap = nrhs;
  }
  if ((rc = poll_events(c))) return rc;
  // Iterations launched after a column has converged still run the whole
  // preconditioner (only the Krylov update is gated), and a poll that finds
  // the stream empty lets the device idle until the next launch.  So the
  // state is copied to pinned memory after each block of iterations, the
  // next block is queued before the host waits for the previous copy, and
  // block lengths follow what the residual's decay between polls predicts:
  // queued work stops short of the predicted end and shrinks towards it.
  // The iterates do not depend on the block lengths.
  const int every = std::max(1, so.check_every);
  const double unknown = 1e30;
  std::vector<double> rr_prev(nrhs, -1.0);
  int launched = 0, npoll = 0, poll_it[2] = {0, 0};
  auto queue_block = [&](int nb) -> int {
    for (int j = 0; j < nb; ++j) {
      const int r = cg_iter(c, c->ws, K, 0, nrhs, flexible, launched + j + 1, st);
      if (r) return r;
    }
    launched += nb;
    const int sl = npoll & 1;
    poll_it[sl] = launched;
    HIPCHK(hipMemcpyAsync(c->hst + (size_t)sl * c->hcap, c->sst, sizeof(KState) * nrhs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipEventRecord(c->pev[sl], st));
    ++npoll;
    return SLR_OK;
  };
  auto block_len = [&](double ahead) {
    return std::min(so.maxit - launched, (int)std::min<double>(every, std::floor(0.8 * ahead)));
  };
  if ((rc = queue_block(std::min(every, so.maxit)))) return rc;
  // need: iterations still wanted after the newest poll read, it_read
  double need = unknown;
  int it_read = 1;  // r_0 = b (x starts at zero) is tested by iteration 1
  for (int seen = 0;; ++seen) {
    // poll `seen` is the newest queued; queue one more block behind it
    int nb = block_len(need - (launched - it_read));
    if (nb > 0 && (rc = queue_block(nb))) return rc;
    const int sl = seen & 1;
    HIPCHK(hipEventSynchronize(c->pev[sl]));
    const KState *h = c->hst + (size_t)sl * c->hcap;
    const int it = poll_it[sl];  // the update of iteration it tested r_{it-1}
    bool any = false;
    double nd = 0.0;
    for (int j = 0; j < nrhs; ++j) {
      const KState &x = h[j];
      if (!x.active) continue;
      any = true;
      const double prev = rr_prev[j] < 0.0 ? x.bb : rr_prev[j];
      const double tol = K.rtol2 * x.bb;
      double est = unknown;
      if (x.rr > tol && x.rr < prev && tol > 0.0 && it > it_read)
        est = std::log(tol / x.rr) / (std::log(x.rr / prev) / (it - it_read));
      nd = std::max(nd, est);
      rr_prev[j] = x.rr;
    }
    if (!any) break;
    need = nd;
    it_read = it;
    if (npoll == seen + 1) {
      // nothing queued behind this poll
      if (launched >= so.maxit) break;
      nb = std::max(1, block_len(need));
      if ((rc = queue_block(nb))) return rc;
    }
  }
  std::vector<KState> h(nrhs);
  // true residual ||b - A x|| / ||b|| in FP64
  launch_spmv(n, c->a_rp, c->a_ci, c->a_v, c->sX, n, c->sQ, n, nrhs, st);
  launch_relres(n, c->sB, n, c->sQ, n, K, 0, nrhs, st);
  launch_permute(n, c->perm, c->sX, n, x_dev, n, nrhs, true, st);
  HIPCHK(hipMemcpyAsync(h.data(), c->sst, sizeof(KState) * nrhs, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int worst = SLR_OK;
  for (int j = 0; j < nrhs; ++j) {
    info[j].iters = h[j].iters;
    info[j].relres = h[j].relres;
    info[j].status = (h[j].active == 0 && h[j].status == 0) ? SLR_OK : SLR_ERR_NOCONV;
    if (info[j].status) worst = SLR_ERR_NOCONV;
  }
  if (worst) g_err = "a right-hand side did not converge";
  return worst;
}

// Right-preconditioned flexible GMRES(restart) (Sec. 6 uses GMRES(40)),
// CGS2 Arnoldi, Givens rotations, x0 = 0, one right-hand side.
int solve_fgmres(slr_ctx *c, const double *b_dev, double *x_dev, const slr_solve_opts &so, slr_solve_info *info,
                 hipStream_t st) {
  const int64_t n = c->n;
  const int32_t mr = fgmres_restart(so.restart);
  Arena tmp(c->gm);
  FgmresWS fw;
  fgmres_layout(tmp, n, mr, fw);
  double *V = fw.V, *Zb = fw.Zb, *Bd = fw.Bd, *X = fw.X, *T = fw.T, *Hm = fw.Hm, *h1 = fw.h1, *h2 = fw.h2;
  double *cs = fw.cs, *sn = fw.sn, *g = fw.g, *y = fw.y, *sc = fw.sc, *part = fw.part;
  unsigned int *cnt = fw.cnt;
  int *flags = fw.flags;
  if (!V || !Zb || !Bd || !X || !T || !Hm || !h1 || !h2 || !cs || !sn || !g || !y || !sc || !part || !cnt ||
      !flags) {
    tmp.release();
    return fail(SLR_ERR_OOM, "FGMRES workspace");
  }
  int rc = SLR_OK;
  auto bail = [&](int code) {
    tmp.release();
    return code;
  };
  if ((rc = poll_events(c))) return bail(rc);
  if (c->hfl_cap < mr) {
    if (c->hfl) (void)hipHostFree(c->hfl);
    c->hfl = nullptr;
    c->hfl_cap = 0;
    if (hipHostMalloc((void **)&c->hfl, sizeof(int) * 2 * (size_t)mr, hipHostMallocDefault) != hipSuccess)
      return bail(fail(SLR_ERR_HIP, "FGMRES flags"));
    c->hfl_cap = mr;
  }
  HIPCHK(hipMemsetAsync(cnt, 0, 4 * sizeof(unsigned int), st));
  HIPCHK(hipMemsetAsync(X, 0, sizeof(double) * n, st));
  launch_permute(n, c->perm, b_dev, n, Bd, n, 1, false, st);
  launch_multidot(n, 1, Bd, n, Bd, part, RED_NBLK, sc + 3, cnt, st);
  double bb = 0.0;
  HIPCHK(hipMemcpyAsync(&bb, sc + 3, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double bn = std::sqrt(bb);
  const double tol = so.rtol * bn;
  int its = 0;
  bool conv = bn == 0.0;
  while (!conv && its < so.maxit) {
    // r = b - A x ; v_0 = r / ||r|| ; g = ||r|| e_1
    launch_spmv(n, c->a_rp, c->a_ci, c->a_v, X, n, T, n, 1, st);
    launch_axpby(n, 1, 1.0, Bd, n, -1.0, T, n, st);
    launch_multidot(n, 1, T, n, T, part, RED_NBLK, sc, cnt, st);
    launch_scale_inv_sqrt(n, T, V, sc, st);
    launch_gmres_g0(mr + 1, sc, g, st);
    // Step j's flags go to pinned memory, and step j + 1 is queued before
    // the host waits for them, so the device does not idle at each test.
    // A step queued past the end of a cycle writes only basis, Hessenberg
    // and rotation entries beyond the jj that the solve and update use.
    auto queue_step = [&](int j) -> int {
      double *vj = V + (int64_t)j * n, *zj = Zb + (int64_t)j * n, *w = V + (int64_t)(j + 1) * n;
      const int r = apply_dd(c, c->ws, vj, n, zj, n, 1, st);
      if (r) return r;
      launch_spmv(n, c->a_rp, c->a_ci, c->a_v, zj, n, w, n, 1, st);
      launch_multidot(n, j + 1, V, n, w, part, RED_NBLK, h1, cnt, st);
      launch_gemv_sub(n, j + 1, V, n, h1, w, nullptr, st);
      launch_multidot(n, j + 1, V, n, w, part, RED_NBLK, h2, cnt, st);
      launch_gemv_sub(n, j + 1, V, n, h2, w, nullptr, st);
      launch_multidot(n, 1, w, n, w, part, RED_NBLK, sc + 1, cnt, st);
      launch_gmres_givens(j, mr + 1, Hm, h1, h2, sc + 1, cs, sn, g, tol, flags + 2 * j, sc + 2, st);
      launch_div_scalar(n, w, w, sc + 2, st);
      HIPCHK(hipMemcpyAsync(c->hfl + 2 * j, flags + 2 * j, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipEventRecord(c->pev[j & 1], st));
      return SLR_OK;
    };
    const int cyc = std::min(mr, so.maxit - its);  // steps this cycle may take
    int jj = 0, queued = 1;
    if ((rc = queue_step(0))) return bail(rc);
    for (int j = 0; j < cyc; ++j) {
      if (queued < cyc) {
        if ((rc = queue_step(queued))) return bail(rc);
        ++queued;
      }
      HIPCHK(hipEventSynchronize(c->pev[j & 1]));
      ++its;
      jj = j + 1;
      const int *fl = c->hfl + 2 * j;
      if (fl[0]) conv = true;
      if (fl[0] || fl[1]) break;
    }
    launch_gmres_solve(jj, mr + 1, Hm, g, y, st);
    launch_gemv_add(n, jj, Zb, n, y, X, st);
  }
  // true residual
  launch_spmv(n, c->a_rp, c->a_ci, c->a_v, X, n, T, n, 1, st);
  launch_axpby(n, 1, 1.0, Bd, n, -1.0, T, n, st);
  launch_multidot(n, 1, T, n, T, part, RED_NBLK, sc, cnt, st);
  launch_permute(n, c->perm, X, n, x_dev, n, 1, true, st);
  double rr = 0.0;
  HIPCHK(hipMemcpyAsync(&rr, sc, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  tmp.release();
  info[0].iters = its;
  info[0].relres = bn > 0.0 ? std::sqrt(rr) / bn : 0.0;
  info[0].status = conv ? SLR_OK : SLR_ERR_NOCONV;
  if (!conv) g_err = "FGMRES did not converge";
  return conv ? SLR_OK : SLR_ERR_NOCONV;
}

}  // namespace

extern "C" {

int slr_solve(slr_ctx *c, const double *b_dev, double *x_dev, int32_t nrhs, const slr_solve_opts *so_in,
              slr_solve_info *info, void *hip_stream) {
  if (!c || !b_dev || !x_dev || !info || nrhs <= 0) return fail(SLR_ERR_ARG, "bad solve arguments");
  slr_solve_opts so;
  if (so_in)
    so = *so_in;
  else
    slr_default_solve_opts(&so);
  if (so.maxit <= 0 || !(so.rtol > 0.0)) return fail(SLR_ERR_ARG, "maxit / rtol");
  hipStream_t st = S(hip_stream);
  if (so.method == SLR_FGMRES) {
    if (nrhs != 1) return fail(SLR_ERR_ARG, "FGMRES takes one right-hand side");
    return solve_fgmres(c, b_dev, x_dev, so, info, st);
  }
  if (so.method != SLR_PCG && so.method != SLR_FCG) return fail(SLR_ERR_ARG, "method");
  if (nrhs > 128) return fail(SLR_ERR_ARG, "at most 128 right-hand sides per solve");
  return solve_cg(c, b_dev, x_dev, nrhs, so, info, st);
}

// ---------------------------------------------------------------------------
// continuous batching
// ---------------------------------------------------------------------------
int slr_batch_create(slr_ctx *c, int32_t max_cols, int32_t method, double rtol, int32_t maxit, slr_batch **out) {
  if (!c || !out || max_cols <= 0 || max_cols > 128 || (method != SLR_PCG && method != SLR_FCG) || !(rtol > 0) ||
      maxit <= 0)
    return fail(SLR_ERR_ARG, "bad batch arguments (max_cols must be in 1..128)");
  slr_batch *b = new slr_batch();
  b->c = c;
  b->cap = max_cols;
  b->method = method;
  b->rtol = rtol;
  b->maxit = maxit;
  const size_t n = (size_t)c->n;
  b->X = b->pool.alloc<double>(n * max_cols);
  b->R = b->pool.alloc<double>(n * max_cols);
  b->Z = b->pool.alloc<double>(n * max_cols);
  b->P = b->pool.alloc<double>(n * max_cols);
  b->Q = b->pool.alloc<double>(n * max_cols);
  b->S = b->pool.alloc<double>(n * max_cols);
  b->B = b->pool.alloc<double>(n * max_cols);
  b->st = b->pool.alloc<KState>(max_cols);
  b->part = b->pool.alloc<double>((size_t)RED_NBLK * max_cols * 4);
  b->part2 = b->pool.alloc<double>((size_t)RED_NBLK * max_cols);
  b->counter = b->pool.alloc<unsigned int>(4);
  if (!b->X || !b->R || !b->Z || !b->P || !b->Q || !b->S || !b->B || !b->st || !b->part || !b->part2 ||
      !b->counter) {
    slr_batch_destroy(b);
    return fail(SLR_ERR_OOM, "batch state");
  }
  if (hipMemset(b->counter, 0, 4 * sizeof(unsigned int)) != hipSuccess ||
      hipMemset(b->st, 0, sizeof(KState) * max_cols) != hipSuccess) {
    slr_batch_destroy(b);
    return fail(SLR_ERR_HIP, "batch init");
  }
  int rc = ws_ensure(c, b->ws, max_cols);
  if (rc) {
    slr_batch_destroy(b);
    return rc;
  }
  b->owner.assign(max_cols, -1);
  b->st_h.resize(max_cols);
  ++c->live_batches;
  b->counted = true;
  *out = b;
  return SLR_OK;
}

void slr_batch_destroy(slr_batch *b) {
  if (!b) return;
  if (b->counted) --b->c->live_batches;
  b->pool.release();
  b->ws.pool.release();
  delete b;
}

int slr_batch_active(const slr_batch *b) {
  if (!b) return 0;
  int a = 0;
  for (int64_t o : b->owner) a += o >= 0;
  return a;
}

size_t slr_batch_bytes(const slr_batch *b) { return b ? (size_t)(b->pool.bytes + b->ws.pool.bytes) : 0; }

int slr_batch_admit(slr_batch *b, const double *b_dev, double *x_dev, int32_t nrhs, int64_t tag, void *hip_stream) {
  if (!b || !b_dev || !x_dev || nrhs <= 0) return fail(SLR_ERR_ARG, "bad admit arguments");
  // first fit of nrhs contiguous free columns
  int32_t c0 = -1;
  for (int32_t i = 0; i + nrhs <= b->cap; ++i) {
    bool ok = true;
    for (int32_t j = 0; j < nrhs && ok; ++j) ok = b->owner[i + j] < 0;
    if (ok) {
      c0 = i;
      break;
    }
  }
  if (c0 < 0) return fail(SLR_ERR_ADMIT, "no free slots");
  slr_ctx *c = b->c;
  hipStream_t st = S(hip_stream);
  const int64_t n = c->n;
  KArgs K = kargs(b->X, b->R, b->Z, b->P, b->Q, b->S, n, b->st, b->part, b->part2, b->maxit, b->rtol);
  launch_permute(n, c->perm, b_dev, n, b->B + (int64_t)c0 * n, n, nrhs, false, st);
  launch_axpby(n, nrhs, 1.0, b->B + (int64_t)c0 * n, n, 0.0, b->R + (int64_t)c0 * n, n, st);
  int rc = cg_start(c, K, c0, nrhs, b->method == SLR_FCG, b->it + 1, st);
  if (rc) return rc;
  const int64_t rid = (int64_t)b->reqs.size();
  b->reqs.push_back({tag, c0, nrhs, x_dev, true});
  for (int32_t j = 0; j < nrhs; ++j) b->owner[c0 + j] = rid;
  b->hi = std::max(b->hi, c0 + nrhs);
  return SLR_OK;
}

int slr_batch_step(slr_batch *b, int32_t iters, void *hip_stream) {
  if (!b || iters < 0) return fail(SLR_ERR_ARG, "bad step arguments");
  if (b->hi == 0) return SLR_OK;
  slr_ctx *c = b->c;
  hipStream_t st = S(hip_stream);
  KArgs K = kargs(b->X, b->R, b->Z, b->P, b->Q, b->S, c->n, b->st, b->part, b->part2, b->maxit, b->rtol);
  for (int32_t i = 0; i < iters; ++i) {
    int rc = cg_iter(c, b->ws, K, 0, b->hi, b->method == SLR_FCG, ++b->it, st, true);
    if (rc) return rc;
  }
  return SLR_OK;
}

int slr_batch_poll(slr_batch *b, int64_t *tags, slr_solve_info *info, int32_t max_done, void *hip_stream) {
  if (!b || (max_done > 0 && (!tags || !info))) return fail(SLR_ERR_ARG, "bad poll arguments");
  if (b->hi == 0) return 0;
  slr_ctx *c = b->c;
  hipStream_t st = S(hip_stream);
  const int64_t n = c->n;
  if (hipMemcpyAsync(b->st_h.data(), b->st, sizeof(KState) * b->hi, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(SLR_ERR_HIP, "poll copy");
  KArgs K = kargs(b->X, b->R, b->Z, b->P, b->Q, b->S, n, b->st, b->part, b->part2, b->maxit, b->rtol);
  int32_t done = 0;
  std::vector<int64_t> fin;
  for (int64_t rid = 0; rid < (int64_t)b->reqs.size() && done < max_done; ++rid) {
    auto &rq = b->reqs[rid];
    if (!rq.live) continue;
    bool all = true;
    for (int32_t j = 0; j < rq.nrhs && all; ++j) all = b->st_h[rq.c0 + j].active == 0;
    if (!all) continue;
    // true residual of the request's columns, then x to the caller
    launch_spmv(n, c->a_rp, c->a_ci, c->a_v, b->X + (int64_t)rq.c0 * n, n, b->Q + (int64_t)rq.c0 * n, n, rq.nrhs,
                st);
    launch_relres(n, b->B + (int64_t)rq.c0 * n, n, b->Q + (int64_t)rq.c0 * n, n, K, rq.c0, rq.nrhs, st);
    launch_permute(n, c->perm, b->X + (int64_t)rq.c0 * n, n, rq.x_dev, n, rq.nrhs, true, st);
    fin.push_back(rid);
    ++done;
  }
  if (fin.empty()) return 0;
  if (hipMemcpyAsync(b->st_h.data(), b->st, sizeof(KState) * b->hi, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(SLR_ERR_HIP, "poll copy");
  for (size_t t = 0; t < fin.size(); ++t) {
    auto &rq = b->reqs[fin[t]];
    slr_solve_info w{0, SLR_OK, 0.0};
    for (int32_t j = 0; j < rq.nrhs; ++j) {
      const KState &k = b->st_h[rq.c0 + j];
      w.iters = std::max(w.iters, k.iters);
      w.relres = std::max(w.relres, k.relres);
      if (k.status != 0) w.status = SLR_ERR_NOCONV;
      b->owner[rq.c0 + j] = -1;
    }
    rq.live = false;
    tags[t] = rq.tag;
    info[t] = w;
  }
  int32_t hi = 0;
  for (int32_t i = 0; i < b->cap; ++i)
    if (b->owner[i] >= 0) hi = i + 1;
  b->hi = hi;
  return (int)fin.size();
}

}  // extern "C"

// Host side of libtrd: context, workspace, per-core plans and the orchestration of
// one core update (Alg. 1 body) and of the sweep loop.  Every compute step runs in a
// kernel on the caller's stream; the host only plans sizes and launches.
#include <math.h>

#include <cmath>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/trd.h"
#include "trd_internal.h"

namespace trd {
int64_t g_lds_max = 65536;
int g_num_cu = 256;
}

using namespace trd;

namespace {

thread_local std::string g_free_err;

// ring of per-sweep fit reports in mapped pinned host memory: slots of
// {sigma, conv[0], conv[1], flags, eta[0..N)}
constexpr int kRepSlots = 32;
constexpr int kRepStride = 4 + kMaxN;

struct SketchWS {
  // index lists per mode (device), capacity per mode
  int32_t* idx[kMaxN] = {nullptr};
  int64_t idx_cap[kMaxN] = {0};
  Layout L;                 // layout storage at capacity
  int64_t cap_rows = 0, cap_cols = 0, cap_slices = 0, cap_counts = 0, cap_slots = 0;
  bool ready = false;
  // leverage sampling: C and its inverse (one mode at a time), per-mode leverage and
  // running sums, per-sample importance weights
  double* levC = nullptr;
  double* levCi = nullptr;
  int64_t cap_levC = 0;
  double* lev[kMaxN] = {nullptr};
  double* cdf[kMaxN] = {nullptr};
  int64_t cap_lev[kMaxN] = {0};
  double* colw = nullptr;
  int64_t cap_colw = 0;
  // inside trd_fit: lev[j] / cdf[j] hold core j's distribution as it stands (a core's
  // leverage changes only with the core, once per sweep)
  bool lev_cache = false;
  bool lev_valid[kMaxN] = {false};
};

}  // namespace

struct trd_ctx {
  int device = 0;
  std::string err;
  std::vector<void*> allocs;
  size_t ws_bytes = 0;

  bool has_problem = false;
  bool has_shape = false;
  int N = 0;
  int64_t dims[kMaxN] = {0};
  int32_t ranks[kMaxN] = {0};
  int64_t strides[kMaxN] = {0};
  int dtype = 0;
  const void* X = nullptr;
  const uint8_t* mask = nullptr;
  int64_t nobs = 0;
  double maxabs = 0.0;            // max |x| over the observed entries
  std::vector<Split> splits;      // full-path split per core
  std::vector<Layout> layouts;    // full-path layout per core
  std::vector<TLayout> tlayouts;  // bitmask-tile layout per core (BF16 form, built on demand)
  int prec = TRD_PREC_NATIVE;     // precision of the entry passes
  int direction = TRD_DIR_SCALED;  // step direction and Gram of later updates
  int gram = TRD_GRAM_GLOBAL;
  int sampling = TRD_SAMPLE_RSTS;  // how a sketch picks its rows
  double lev_lambda = 1e-9;        // ridge of the leverage scores (the step's lambda_rel)
  uint16_t* Tb = nullptr; uint16_t* THb = nullptr; uint16_t* Vb = nullptr;
  uint16_t* Tb_lo = nullptr; uint16_t* Vb_lo = nullptr;  // split (BF16X3) remainders
  // Vb (and Vb_lo) in operand-fragment order, and Vb transposed in fragment order
  uint16_t* Vf = nullptr; uint16_t* Vf_lo = nullptr; uint16_t* VTf = nullptr;
  // per-entry weights of the last gradient pass (tile layouts), read by its line search
  uint16_t* wts = nullptr;  // fp16
  int64_t cap_wts = 0;
  int64_t cap_Tb = 0, cap_Vb = 0, cap_Tlo = 0, cap_Vlo = 0, cap_Vf = 0, cap_Vflo = 0;

  // tables and work buffers (sized for the largest core and sketch)
  void* T = nullptr; void* TH = nullptr; void* V = nullptr; void* S = nullptr;
  void* U = nullptr; void* chainA = nullptr; void* chainB = nullptr;
  int64_t cap_T = 0, cap_V = 0, cap_U = 0, cap_chain = 0, cap_S = 0;
  double* K[kMaxN] = {nullptr};
  double* Kl[kMaxN] = {nullptr};  // factors of the sampled cores (local Gram)
  double* P0 = nullptr; double* P1 = nullptr; double* G = nullptr; double* Cinv = nullptr;
  // second stream (default priority) for the FGMC Gram and its inverse, which depend only
  // on the other cores and so run beside the gradient pass; fork / join events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double* d64 = nullptr; double* h64 = nullptr; void* h_real = nullptr;
  int64_t cap_d = 0;
  double* part_pass = nullptr; int64_t cap_part_pass = 0;
  double* part_misc = nullptr; int64_t cap_part_misc = 0;
  double* scal = nullptr;         // device scalars, see kS* below
  uint32_t* flags = nullptr;      // [0] step flags, [1] fit flags
  float* resid = nullptr; int64_t cap_resid = 0;
  // core whose current residuals (tile layout, value order) the residual pass left in
  // resid, or -1: that core's next gradient pass reads them instead of forming xhat
  int resid_core = -1;
  uint32_t* qhist = nullptr; uint32_t* qstate = nullptr;
  float* qcand = nullptr; uint32_t* qcand_cnt = nullptr; int64_t cap_qcand = 0, cap_qcnt = 0;
  double* Dbuf[2] = {nullptr, nullptr}; double* M = nullptr;
  double* eta_hist = nullptr;     // [N] per sweep
  double* host_rep = nullptr;     // mapped pinned host memory: a ring of per-sweep reports
  double* host_rep_dev = nullptr; // its device address
  SketchWS sk;

  // profiling of the fused gradient pass
  bool prof = false;
  std::vector<hipEvent_t> ev_free, ev_pairs;
  int64_t prof_slots = 0, prof_entries = 0;
  int64_t* prof_nobs_dev = nullptr;  // device sum of sketch observed counts while profiling
};

namespace {

enum {
  kSigma = 0, kNum = 1, kDen = 2, kEta = 3, kStats = 4 /* 3 */, kMaxAbs = 7, kSigmaMin = 8,
  kConv = 9 /* 2 */, kLoss = 11, kTmp = 12 /* 4 */, kScalCount = 16
};

int fail(trd_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_free_err = msg;
  return code;
}

}  // namespace

int trd::fail_free(int code, const std::string& msg) { return fail(nullptr, code, msg); }

namespace {

#define CK(expr)                                                                          \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail(ctx, TRD_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));  \
  } while (0)

#define TRY(expr)                   \
  do {                              \
    int _r = (expr);                \
    if (_r != TRD_OK) return _r;    \
  } while (0)

int dev_alloc(trd_ctx* ctx, void** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    hipGetLastError();
    return fail(ctx, TRD_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
  }
  ctx->allocs.push_back(*p);
  ctx->ws_bytes += bytes;
  return TRD_OK;
}

template <typename P>
int alloc_n(trd_ctx* ctx, P** p, int64_t n) {
  return dev_alloc(ctx, (void**)p, (size_t)std::max<int64_t>(n, 1) * sizeof(P));
}

void free_all(trd_ctx* ctx) {
  for (void* p : ctx->allocs) hipFree(p);
  ctx->allocs.clear();
  ctx->ws_bytes = 0;
  if (ctx->host_rep) hipHostFree(ctx->host_rep);
  ctx->host_rep = nullptr;
  ctx->host_rep_dev = nullptr;
}

size_t esz(int dtype) { return dtype == 0 ? 4 : 8; }

// ---------------------------------------------------------------- planning

// counts[j]: indices of mode j taking part (I_j on the full path, s_j in a sketch).
// Column tiles of an nr x nc update: as wide as the LDS allows, or, for a small update
// (fill_rho >= 0, the observed density), narrower (down to 64 columns) until the row
// groups times the tiles reach the work-group target, so the whole device takes part.
int64_t plan_tiles(int64_t nr, int64_t nc, int64_t wmax, double fill_rho) {
  int64_t nct = (nc + wmax - 1) / wmax;
  if (fill_rho >= 0) {
    const int64_t nrg = (nr + kRowsPerWG - 1) / kRowsPerWG;
    const int64_t want = std::min((wg_target() + nrg - 1) / nrg, (nc + 63) / 64);
    nct = std::max(nct, want);
  }
  return std::max<int64_t>(1, nct);
}

// fill_rho >= 0: a small (sketched) update of that observed density, whose passes are
// bound by the longest work-group rather than by HBM: the split is chosen on the larger of
// its byte time and its per-work-group entry time, with tiles narrowed by plan_tiles
int plan_split(trd_ctx* ctx, int k, const int64_t* counts, Split& sp, int64_t& nrows,
               int64_t& ncols, int& ct_w, int& n_ct, double fill_rho = -1.0) {
  const int N = ctx->N;
  double best = -1;
  int bestp = -1;
  int64_t best_nct = 1;
  for (int p = 0; p <= N - 2; ++p) {
    const int s = (k + p + 1) % N;
    const int RR = ctx->ranks[k] * ctx->ranks[s];
    const int RRP = pass_rrp(RR);
    if (RRP < 0) continue;
    int64_t nr = counts[k], nc = 1;
    for (int t = 1; t <= p; ++t) nr *= counts[(k + t) % N];
    for (int t = p + 1; t <= N - 1; ++t) nc *= counts[(k + t) % N];
    const int64_t wmax = pass_ct_w(ctx->dtype, 0, RRP);
    const int64_t nct = plan_tiles(nr, nc, wmax, fill_rho);
    const int64_t nrg = (nr + kRowsPerWG - 1) / kRowsPerWG;
    int ncg, cpg;
    column_groups(nrg, (int)std::min<int64_t>(nct, 1 << 30), ncg, cpg);
    // bytes: the two tables (written, then read), the gradient partials of the column
    // groups (written, then read), and the column-table reads of every row group (from
    // L2, weighted 1/4, when the column table fits a fraction of one XCD's L2)
    const double esb = (double)esz(ctx->dtype);
    const double vbytes = (double)nc * RRP * esb;
    const double vw = vbytes <= 2.0 * (1 << 20) ? 0.25 : 1.0;
    double cost = 2.0 * (double)(nr + nc) * RRP * esb + 2.0 * (double)ncg * nr * RRP * esb +
                  vw * (double)nrg * vbytes;
    if (fill_rho >= 0) {
      // seconds: bytes at ~4 TB/s against ~1 ns per observed entry of the busiest group
      const double per_wg = fill_rho * (double)nr * (double)nc / ((double)nrg * ncg) * RRP / 32.0;
      cost = std::max(cost / 4e12, per_wg * 1e-9);
    }
    if (bestp < 0 || cost < best) {
      best = cost;
      bestp = p;
      best_nct = nct;
    }
  }
  if (bestp < 0)
    return fail(ctx, TRD_EUNSUPPORTED, "no subchain split with r_k * r_s <= 128 for core " +
                                           std::to_string(k));
  sp.k = k;
  sp.p = bestp;
  sp.q = N - 1 - bestp;
  for (int t = 1; t <= sp.p; ++t) sp.B[t - 1] = (k + t) % N;
  for (int t = sp.p + 1; t <= N - 1; ++t) sp.C[t - sp.p - 1] = (k + t) % N;
  sp.r_k = ctx->ranks[k];
  sp.r_k1 = ctx->ranks[(k + 1) % N];
  sp.r_s = ctx->ranks[(k + sp.p + 1) % N];
  sp.RR = sp.r_k * sp.r_s;
  sp.RRP = pass_rrp(sp.RR);
  nrows = counts[k];
  for (int t = 0; t < sp.p; ++t) nrows *= counts[sp.B[t]];
  ncols = 1;
  for (int t = 0; t < sp.q; ++t) ncols *= counts[sp.C[t]];
  n_ct = (int)best_nct;
  ct_w = (int)((ncols + n_ct - 1) / n_ct);
  if (ct_w > 0) n_ct = (int)((ncols + ct_w - 1) / ct_w);  // no empty trailing tile
  return TRD_OK;
}

void layout_dims(Layout& L, int64_t nrows, int64_t ncols, int ct_w, int n_ct) {
  L.nrows = nrows;
  L.ncols = ncols;
  L.ct_w = ct_w;
  L.n_ct = n_ct;
  L.n_rg = (nrows + kRowsPerWG - 1) / kRowsPerWG;
  L.n_slices = L.n_rg * n_ct * 4;
  column_groups(L.n_rg, n_ct, L.n_cg, L.cpg);
}

ModeSet rows_set(trd_ctx* ctx, const Split& sp, const int64_t* counts, const int32_t* const* lists) {
  ModeSet ms;
  ms.n = 1 + sp.p;
  for (int t = 0; t < ms.n; ++t) {
    const int m = t == 0 ? sp.k : sp.B[t - 1];
    ms.mode[t] = m;
    ms.count[t] = counts[m];
    ms.stride[t] = ctx->strides[m];
    ms.list[t] = (lists && m != sp.k) ? lists[m] : nullptr;
  }
  return ms;
}

ModeSet cols_set(trd_ctx* ctx, const Split& sp, const int64_t* counts, const int32_t* const* lists) {
  ModeSet ms;
  ms.n = sp.q;
  for (int t = 0; t < ms.n; ++t) {
    const int m = sp.C[t];
    ms.mode[t] = m;
    ms.count[t] = counts[m];
    ms.stride[t] = ctx->strides[m];
    ms.list[t] = lists ? lists[m] : nullptr;
  }
  return ms;
}

// count -> slices -> scan (-> fill when vals/cols are in place)
// cols_given: L.coloff already holds the column offsets (a uniform row sample)
int build_layout_head(trd_ctx* ctx, const Split& sp, const int64_t* counts,
                      const int32_t* const* lists, Layout& L, hipStream_t st, bool cols_given = false) {
  CK(launch_offsets(rows_set(ctx, sp, counts, lists), L.nrows, L.rowoff, st));
  if (!cols_given) CK(launch_offsets(cols_set(ctx, sp, counts, lists), L.ncols, L.coloff, st));
  CK(launch_zero(L.nobs_dev, sizeof(int64_t), st));
  CK(launch_count(L, ctx->mask, st));
  CK(launch_slices(L, st));
  CK(launch_scan(L, st));
  return TRD_OK;
}

int alloc_layout_index(trd_ctx* ctx, Layout& L) {
  TRY(alloc_n(ctx, &L.rowoff, L.nrows));
  TRY(alloc_n(ctx, &L.coloff, L.ncols));
  TRY(alloc_n(ctx, &L.counts, (int64_t)L.n_ct * L.n_rg * kRowsPerWG));
  TRY(alloc_n(ctx, &L.slice_len, L.n_slices));
  TRY(alloc_n(ctx, &L.slice_off, L.n_slices + 1));
  TRY(alloc_n(ctx, &L.total_dev, 1));
  TRY(alloc_n(ctx, &L.nobs_dev, 1));
  return TRD_OK;
}

// table sizes a split needs
void table_needs(trd_ctx* ctx, const Split& sp, const int64_t* counts, int64_t nrows, int64_t ncols,
                 int64_t& needT, int64_t& needV, int64_t& needU, int64_t& needChain) {
  int64_t nB = 1;
  for (int t = 0; t < sp.p; ++t) nB *= counts[sp.B[t]];
  needT = nrows * sp.RRP;
  needV = ncols * sp.RRP;
  needU = sp.p >= 2 ? nB * sp.r_k1 * sp.r_s : 0;
  needChain = std::max<int64_t>(nB, ncols) * kMaxRank * kMaxRank;
  (void)ctx;
}

int ensure_tables(trd_ctx* ctx, int64_t needT, int64_t needV, int64_t needU, int64_t needChain) {
  const size_t e = esz(ctx->dtype);
  if (needT > ctx->cap_T) {
    TRY(dev_alloc(ctx, &ctx->T, needT * e));
    TRY(dev_alloc(ctx, &ctx->TH, needT * e));
    ctx->cap_T = needT;
  }
  if (needV > ctx->cap_V) {
    TRY(dev_alloc(ctx, &ctx->V, needV * e));
    ctx->cap_V = needV;
  }
  if (needU > ctx->cap_U) {
    TRY(dev_alloc(ctx, &ctx->U, needU * e));
    ctx->cap_U = needU;
  }
  if (needChain > ctx->cap_chain) {
    TRY(dev_alloc(ctx, &ctx->chainA, needChain * e));
    TRY(dev_alloc(ctx, &ctx->chainB, needChain * e));
    ctx->cap_chain = needChain;
  }
  return TRD_OK;
}

int ensure_S(trd_ctx* ctx, int64_t need) {
  if (need > ctx->cap_S) {
    TRY(dev_alloc(ctx, &ctx->S, need * esz(ctx->dtype)));
    ctx->cap_S = need;
  }
  return TRD_OK;
}

int ensure_part(trd_ctx* ctx, int64_t need_pass, int64_t need_misc) {
  if (need_pass > ctx->cap_part_pass) {
    TRY(alloc_n(ctx, &ctx->part_pass, need_pass));
    ctx->cap_part_pass = need_pass;
  }
  if (need_misc > ctx->cap_part_misc) {
    TRY(alloc_n(ctx, &ctx->part_misc, need_misc));
    ctx->cap_part_misc = need_misc;
  }
  return TRD_OK;
}

// chunks of the B-mode range for the gradient contraction (split K): about two
// work-groups per CU over the (i_k, a) pair tiles, at least two B items per chunk
int contract_chunks(int64_t Ik, int64_t nB, int r_k) {
  const int64_t ntile = (Ik * r_k + 255) / 256;
  // about four work-groups per CU: enough loads in flight to stream the partials
  const int64_t by_grid = std::max<int64_t>(1, (4 * (int64_t)g_num_cu) / std::max<int64_t>(ntile, 1));
  const int64_t by_work = std::max<int64_t>(1, (nB + 1) / 2);
  return (int)std::min(by_grid, by_work);
}

// ---------------------------------------------------------------- per-update state

struct Update {
  Split sp;
  Layout* L = nullptr;
  TLayout* TL = nullptr;                  // non-null: matrix-core (BF16) passes
  const int64_t* counts = nullptr;        // per-mode counts of this update
  const int32_t* const* lists = nullptr;  // per-mode device lists (nullptr = full)
  bool rows = false;                      // row sample: columns = sampled fibres
  const double* colw = nullptr;           // importance weight per column (leverage sample)
  int64_t cnt[kMaxN];
  const int32_t* lst[kMaxN];
};

int sketch_layout(trd_ctx* ctx, int k, int64_t nrows, int64_t ncols, int ct_w, int n_ct);
// observed density of the bound problem (what a sketch of it holds on average)
double sketch_density(const trd_ctx* ctx) {
  double total = 1.0;
  for (int j = 0; j < ctx->N; ++j) total *= (double)ctx->dims[j];
  return total > 0 ? (double)ctx->nobs / total : 0.0;
}
int prepare_rows(trd_ctx* ctx, int k, const trd_sketch* sk, Update& up, hipStream_t st,
                 const void* const* cores);

// sample the sketch of update (t, k) and build its layout into the sketch workspace
int prepare_sketch(trd_ctx* ctx, int k, const trd_sketch* sk, Update& up, hipStream_t st,
                   const void* const* cores) {
  if (ctx->sampling != TRD_SAMPLE_RSTS) return prepare_rows(ctx, k, sk, up, st, cores);
  const int N = ctx->N;
  SketchWS& W = ctx->sk;
  for (int j = 0; j < N; ++j) {
    int64_t s = j == k ? ctx->dims[j] : std::min<int64_t>(std::max(1, sk->sizes[j]), ctx->dims[j]);
    up.cnt[j] = s;
  }
  // index lists: caller's or sampled
  for (int j = 0; j < N; ++j) {
    if (W.idx_cap[j] < ctx->dims[j]) {
      TRY(alloc_n(ctx, &W.idx[j], ctx->dims[j]));
      W.idx_cap[j] = ctx->dims[j];
    }
  }
  if (sk->idx) {
    // copy the caller's lists into the workspace, clamped into range (never read out of bounds)
    for (int j = 0; j < N; ++j)
      if (j != k) CK(launch_copy_clamp(sk->idx[j], up.cnt[j], ctx->dims[j], W.idx[j], ctx->flags, st));
    for (int j = 0; j < N; ++j) up.lst[j] = j == k ? nullptr : W.idx[j];
  } else {
    int32_t sizes[kMaxN];
    for (int j = 0; j < N; ++j) sizes[j] = (int32_t)up.cnt[j];
    CK(launch_sample(sk->seed, sk->sweep, k, N, ctx->dims, sizes, W.idx, st));
    for (int j = 0; j < N; ++j) up.lst[j] = j == k ? nullptr : W.idx[j];
  }
  int64_t nrows, ncols;
  int ct_w, n_ct;
  TRY(plan_split(ctx, k, up.cnt, up.sp, nrows, ncols, ct_w, n_ct, sketch_density(ctx)));
  TRY(sketch_layout(ctx, k, nrows, ncols, ct_w, n_ct));
  Layout& L = W.L;
  up.counts = up.cnt;
  up.lists = up.lst;
  up.L = &L;
  TRY(build_layout_head(ctx, up.sp, up.cnt, up.lst, L, st));
  CK(launch_fill(L, ctx->mask, ctx->X, ctx->dtype, st));
  return TRD_OK;
}

// the sketch workspace's layout, sized for an nrows x ncols update (grown, never shrunk)
int sketch_layout(trd_ctx* ctx, int k, int64_t nrows, int64_t ncols, int ct_w, int n_ct) {
  SketchWS& W = ctx->sk;
  Layout& L = W.L;
  layout_dims(L, nrows, ncols, ct_w, n_ct);
  const int64_t need_counts = (int64_t)n_ct * L.n_rg * kRowsPerWG;
  // dense bound: every slice as long as its tile is wide, rounded up to whole groups
  const int64_t need_slots = need_counts * (((int64_t)ct_w + kGroup - 1) / kGroup * kGroup);
  if (nrows > W.cap_rows) { TRY(alloc_n(ctx, &L.rowoff, nrows)); W.cap_rows = nrows; }
  if (ncols > W.cap_cols) { TRY(alloc_n(ctx, &L.coloff, ncols)); W.cap_cols = ncols; }
  if (need_counts > W.cap_counts) { TRY(alloc_n(ctx, &L.counts, need_counts)); W.cap_counts = need_counts; }
  if (L.n_slices > W.cap_slices) {
    TRY(alloc_n(ctx, &L.slice_len, L.n_slices));
    TRY(alloc_n(ctx, &L.slice_off, L.n_slices + 1));
    W.cap_slices = L.n_slices;
  }
  if (need_slots > W.cap_slots) {
    TRY(dev_alloc(ctx, &L.vals, need_slots * esz(ctx->dtype)));
    TRY(alloc_n(ctx, &L.cols, need_slots));
    W.cap_slots = need_slots;
  }
  if (!L.total_dev) {
    TRY(alloc_n(ctx, &L.total_dev, 1));
    TRY(alloc_n(ctx, &L.nobs_dev, 1));
  }
  L.slots_cap = W.cap_slots;
  L.slots = need_slots;  // upper bound; the device holds the exact value
  L.k = k;
  return TRD_OK;
}

// leverage distributions of every mode but k from the cores as they stand, and J draws
// from their product with importance weights (TRALS-S's sampler)
int sample_leverage(trd_ctx* ctx, const void* const* cores, int k, uint64_t seed, int t, int64_t J,
                    double lambda_rel, int64_t* off, int64_t* row, double* weight, hipStream_t st) {
  const int N = ctx->N;
  SketchWS& W = ctx->sk;
  int64_t maxR2 = 1;
  for (int j = 0; j < N; ++j)
    if (j != k) maxR2 = std::max<int64_t>(maxR2, (int64_t)ctx->ranks[j] * ctx->ranks[(j + 1) % N] *
                                                     ctx->ranks[j] * ctx->ranks[(j + 1) % N]);
  if (maxR2 > W.cap_levC) {
    TRY(alloc_n(ctx, &W.levC, maxR2));
    TRY(alloc_n(ctx, &W.levCi, maxR2));
    W.cap_levC = maxR2;
  }
  for (int j = 0; j < N; ++j) {
    if (j == k) continue;
    if (ctx->dims[j] > W.cap_lev[j]) {
      TRY(alloc_n(ctx, &W.lev[j], ctx->dims[j]));
      TRY(alloc_n(ctx, &W.cdf[j], ctx->dims[j]));
      W.cap_lev[j] = ctx->dims[j];
    }
    if (W.lev_cache && W.lev_valid[j]) continue;
    const int R = ctx->ranks[j] * ctx->ranks[(j + 1) % N];
    CK(launch_leverage_mode(ctx->dtype, cores[j], ctx->dims[j], R, W.levC, W.levCi, lambda_rel, W.lev[j],
                            W.cdf[j], ctx->flags + 3, st));
    W.lev_valid[j] = W.lev_cache;
  }
  CK(launch_sample_leverage(seed, t, k, N, ctx->dims, W.lev, W.cdf, J, off, row, weight, st));
  return TRD_OK;
}

// row sampling (the ablations of Sec. 6.1 that replace RStS): as many rows of the subchain
// unfolding as the sketch of these sizes holds, drawn independently with replacement,
// uniformly or by leverage (then with importance weights); the update's matrix has the I_k
// rows of core k and one column per sample
int prepare_rows(trd_ctx* ctx, int k, const trd_sketch* sk, Update& up, hipStream_t st,
                 const void* const* cores) {
  const int N = ctx->N;
  const bool lev = ctx->sampling == TRD_SAMPLE_LEVERAGE;
  if (sk->idx) return fail(ctx, TRD_EINVAL, "caller index lists are RStS sets: not with row sampling");
  if (lev && !cores) return fail(ctx, TRD_EINVAL, "leverage sampling needs the cores");
  int64_t J = 1;
  for (int j = 0; j < N; ++j) {
    up.cnt[j] = ctx->dims[j];
    up.lst[j] = nullptr;
    if (j != k) J *= std::min<int64_t>(std::max(1, sk->sizes[j]), ctx->dims[j]);
  }
  if (J > (int64_t)1 << 31) return fail(ctx, TRD_EUNSUPPORTED, "uniform row sample above 2^31 rows");
  Split& sp = up.sp;
  sp.k = k;
  sp.p = 0;
  sp.q = N - 1;
  for (int t = 1; t <= N - 1; ++t) sp.C[t - 1] = (k + t) % N;
  sp.r_k = ctx->ranks[k];
  sp.r_k1 = ctx->ranks[(k + 1) % N];
  sp.r_s = sp.r_k1;
  sp.RR = sp.r_k * sp.r_s;
  sp.RRP = pass_rrp(sp.RR);
  if (sp.RRP < 0) return fail(ctx, TRD_EUNSUPPORTED, "r_k * r_{k+1} above the pass width");
  int n_ct = (int)plan_tiles(ctx->dims[k], J, pass_ct_w(ctx->dtype, 0, sp.RRP), sketch_density(ctx));
  const int ct_w = (int)((J + n_ct - 1) / n_ct);
  if (ct_w > 0) n_ct = (int)((J + ct_w - 1) / ct_w);  // no empty trailing tile
  TRY(sketch_layout(ctx, k, ctx->dims[k], J, ct_w, n_ct));
  Layout& L = ctx->sk.L;
  up.counts = up.cnt;
  up.lists = up.lst;
  up.rows = true;
  up.L = &L;
  if (lev) {
    SketchWS& W = ctx->sk;
    if (J > W.cap_colw) {
      TRY(alloc_n(ctx, &W.colw, J));
      W.cap_colw = J;
    }
    TRY(sample_leverage(ctx, cores, k, sk->seed, sk->sweep, J, ctx->lev_lambda, L.coloff, nullptr, W.colw, st));
    up.colw = W.colw;
  } else {
    CK(launch_sample_rows(sk->seed, sk->sweep, k, N, ctx->dims, J, L.coloff, nullptr, st));
  }
  TRY(build_layout_head(ctx, sp, up.cnt, nullptr, L, st, true));
  CK(launch_fill(L, ctx->mask, ctx->X, ctx->dtype, st));
  return TRD_OK;
}

// work-groups per compute unit the matrix-core passes aim for: each column group adds a
// partial of the gradient (row factors, written by the pass and read by the contraction,
// or on B-major rows the pass's own 64-float partials of d), so fewer, longer walks are
// preferred to the denser grid of the other passes
constexpr int kTileWGPerCU = 6;

// shape of the bitmask-tile layout of a core-k matrix (nrows x ncols, split sp): block and
// column-tile counts and the column groups of the matrix-core passes (no device work)
void plan_tile(const Split& sp, int64_t nrows, int64_t ncols, int64_t Ik, TLayout& T) {
  T.nrows = nrows;
  T.ncols = ncols;
  // B-major rows where the gradient pass can contract its own row factors: TR ranks 8
  // around the split and at least 64 B items per slice (a 64-row block spans <= 2 slices)
  T.Ik = Ik;
  T.nB = Ik > 0 ? nrows / Ik : 1;
  T.bmaj = sp.p >= 1 && sp.r_k == 8 && sp.r_k1 == 8 && sp.r_s == 8 && T.nB >= 64 &&
           T.nB * Ik == nrows;
  T.K = tile_k(sp.RRP);  // covers the padded width the row-factor partials are stored with
  T.n_chunks = (T.ncols + 31) / 32;
  const int64_t cwmax = tile_cw(T.K);
  T.n_ct = (int)((T.n_chunks * 32 + cwmax - 1) / cwmax);
  T.n_chpt = (int)((T.n_chunks + T.n_ct - 1) / T.n_ct);
  T.CW = T.n_chpt * 32;
  T.n_ct = (int)((T.n_chunks + T.n_chpt - 1) / T.n_chpt);
  T.n_rb = (T.nrows + 63) / 64;
  T.n_rg = (T.n_rb + 3) / 4;
  column_groups(T.n_rg, T.n_ct, T.n_cg, T.cpg, (int64_t)g_num_cu * kTileWGPerCU);
  if (T.cpg * T.n_chpt > 63) {  // a wave's walk keeps its block offsets in one register
    T.cpg = std::max(1, 63 / T.n_chpt);
    T.n_cg = (T.n_ct + T.cpg - 1) / T.cpg;
  }
  T.n_blocks = T.n_rb * T.n_chunks;
}

// bitmask-tile layout of core k (same split as the ELL layout), built once on first use
int ensure_tile_layout(trd_ctx* ctx, int k, hipStream_t st) {
  TLayout& T = ctx->tlayouts[k];
  if (T.ready) return TRD_OK;
  const Split& sp = ctx->splits[k];
  const Layout& L = ctx->layouts[k];
  plan_tile(sp, L.nrows, L.ncols, ctx->dims[k], T);
  if ((int64_t)tpass_lds(kModeGradFast, T.K, T.CW) > g_lds_max)
    return fail(ctx, TRD_EUNSUPPORTED, "matrix-core pass does not fit the device LDS");
  T.rowoff = L.rowoff;
  T.coloff = L.coloff;
  TRY(alloc_n(ctx, &T.bcnt, T.n_blocks));
  TRY(alloc_n(ctx, &T.boff, T.n_blocks + 1));
  TRY(alloc_n(ctx, &T.total_dev, 1));
  CK(launch_tile_build(T, ctx->mask, ctx->X, ctx->dtype, false, st));
  CK(hipMemcpyAsync(&T.nobs, T.total_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  // slack: the pass prefetches up to 16 rounds of 64 entries without bounds branches
  TRY(alloc_n(ctx, &T.vals, T.nobs + kTileSlack));
  TRY(alloc_n(ctx, &T.pos, T.nobs + kTileSlack));
  CK(launch_zero(T.vals, (size_t)(T.nobs + kTileSlack) * sizeof(float), st));
  CK(launch_zero(T.pos, (size_t)(T.nobs + kTileSlack) * sizeof(uint16_t), st));
  CK(launch_tile_build(T, ctx->mask, ctx->X, ctx->dtype, true, st));
  // weights: one per entry, the same slack (the line search reads them like values; the
  // gradient pass's lanes past a block's end write their own slots past nobs); zeroed once
  // (fp16, read as aligned 32-bit words: one element more for an odd count)
  if (T.nobs + kTileSlack + 1 > ctx->cap_wts) {
    TRY(alloc_n(ctx, &ctx->wts, T.nobs + kTileSlack + 1));
    CK(launch_zero(ctx->wts, (size_t)(T.nobs + kTileSlack + 1) * sizeof(uint16_t), st));
    ctx->cap_wts = T.nobs + kTileSlack + 1;
  }
  T.ready = true;
  return TRD_OK;
}

bool bf16_form(int prec) { return prec == TRD_PREC_BF16 || prec == TRD_PREC_BF16X3; }

int prepare_update(trd_ctx* ctx, int k, const trd_sketch* sk, Update& up, hipStream_t st,
                   const void* const* cores = nullptr) {
  if (sk) return prepare_sketch(ctx, k, sk, up, st, cores);  // sketches use the ELL passes
  if (bf16_form(ctx->prec)) {
    TRY(ensure_tile_layout(ctx, k, st));
    up.TL = &ctx->tlayouts[k];
  }
  up.sp = ctx->splits[k];
  up.L = &ctx->layouts[k];
  for (int j = 0; j < ctx->N; ++j) {
    up.cnt[j] = ctx->dims[j];
    up.lst[j] = nullptr;
  }
  up.counts = up.cnt;
  up.lists = nullptr;
  return TRD_OK;
}

// ---------------------------------------------------------------- tables

ItemRef core_ref(trd_ctx* ctx, const void* core, int m, const int32_t* const* lists) {
  ItemRef r;
  r.ptr = core;
  r.stride = (int64_t)ctx->ranks[m] * ctx->ranks[(m + 1) % ctx->N];
  r.list = lists ? lists[m] : nullptr;
  return r;
}

// U(m_B) = product of the B cores (p >= 2 only; p == 1 uses the core directly)
int build_U(trd_ctx* ctx, const Update& up, const void* const* cores, ItemRef& Uref, int64_t& nB,
            hipStream_t st) {
  const Split& sp = up.sp;
  const int N = ctx->N;
  nB = 1;
  for (int t = 0; t < sp.p; ++t) nB *= up.counts[sp.B[t]];
  if (sp.p == 0) {
    Uref = ItemRef();
    return TRD_OK;
  }
  if (sp.p == 1) {
    Uref = core_ref(ctx, cores[sp.B[0]], sp.B[0], up.lists);
    return TRD_OK;
  }
  ItemRef L = core_ref(ctx, cores[sp.B[0]], sp.B[0], up.lists);
  int64_t nL = up.counts[sp.B[0]];
  const int r0 = ctx->ranks[sp.B[0]];
  int rB = ctx->ranks[(sp.B[0] + 1) % N];
  void* bufs[2] = {ctx->chainA, ctx->chainB};
  for (int t = 1; t < sp.p; ++t) {
    const int m = sp.B[t];
    const int rC = ctx->ranks[(m + 1) % N];
    void* out = (t == sp.p - 1) ? ctx->U : bufs[t & 1];
    CK(launch_merge(ctx->dtype, L, nL, r0, rB, core_ref(ctx, cores[m], m, up.lists), up.counts[m],
                    rC, out, (int64_t)r0 * rC, 0, st));
    L.ptr = out;
    L.stride = (int64_t)r0 * rC;
    L.list = nullptr;
    nL *= up.counts[m];
    rB = rC;
  }
  Uref = L;
  return TRD_OK;
}

int ensure_bf16_tables(trd_ctx* ctx, int64_t nrows, int64_t ncols, int K, hipStream_t st);

// T-like table: left(i_k) @ U(m_B), padded to RRP.  left in core layout (I_k items).  For
// the matrix-core passes the table is written directly as bf16, padded to K (out == T
// goes to Tb, out == TH to THb).
int build_rowtable(trd_ctx* ctx, const Update& up, const void* left, const ItemRef& Uref,
                   int64_t nB, void* out, hipStream_t st) {
  const Split& sp = up.sp;
  ItemRef L;
  L.ptr = left;
  L.stride = (int64_t)sp.r_k * sp.r_k1;
  const int64_t Ik = up.counts[sp.k];
  int64_t stride = sp.RRP;
  const bool bf = up.TL != nullptr;
  void* lo = nullptr;  // remainder table of the split form (reconstruction table only)
  if (bf) {
    TRY(ensure_bf16_tables(ctx, up.TL->nrows, up.TL->ncols, up.TL->K, st));
    if (out != ctx->TH && ctx->prec == TRD_PREC_BF16X3) lo = ctx->Tb_lo;
    out = out == ctx->TH ? (void*)ctx->THb : (void*)ctx->Tb;
    stride = up.TL->K;
  }
  if (sp.p == 0) {
    CK(launch_pack(ctx->dtype, L, Ik, sp.r_k, sp.r_k1, out, stride, 0, st, bf, lo));
  } else {
    CK(launch_merge(ctx->dtype, L, Ik, sp.r_k, sp.r_k1, Uref, nB, sp.r_s, out, stride, 0, st, bf,
                    lo));
  }
  return TRD_OK;
}

// the bf16 column table of the matrix-core passes in operand-fragment order (and its
// transpose; the split remainder without)
int fragment_coltable(trd_ctx* ctx, const Update& up, hipStream_t st) {
  const TLayout& TL = *up.TL;
  const bool split = ctx->prec == TRD_PREC_BF16X3;
  const int64_t nf = tile_frag_elems(TL.ncols, TL.K);
  if (nf > ctx->cap_Vf || (split && nf > ctx->cap_Vflo)) return TRD_ESTATE;
  CK(launch_fragments(ctx->Vb, TL.ncols, TL.K, ctx->Vf, ctx->VTf, st));
  if (split) CK(launch_fragments(ctx->Vb_lo, TL.ncols, TL.K, ctx->Vf_lo, nullptr, st));
  return TRD_OK;
}

// V^T(m_C): product of the C cores, stored transposed (a + r_k*c) and padded to RRP
int build_coltable(trd_ctx* ctx, const Update& up, const void* const* cores, hipStream_t st) {
  const Split& sp = up.sp;
  const int N = ctx->N;
  if (up.rows) {  // one chain per sampled fibre (ELL passes only)
    CK(launch_chain_cols(ctx->dtype, cores, N, sp.k, ctx->ranks, ctx->dims, ctx->strides, up.L->coloff,
                         up.L->ncols, ctx->V, sp.RRP, st));
    return TRD_OK;
  }
  const int m0 = sp.C[0];
  ItemRef L = core_ref(ctx, cores[m0], m0, up.lists);
  int64_t nL = up.counts[m0];
  const int r0 = ctx->ranks[m0];  // == r_s
  int rB = ctx->ranks[(m0 + 1) % N];
  // matrix-core passes: the final table goes straight to bf16, padded to K
  const bool bf = up.TL != nullptr;
  void* Vout = ctx->V;
  void* Vlo = nullptr;
  int64_t Vstride = sp.RRP;
  if (bf) {
    TRY(ensure_bf16_tables(ctx, up.TL->nrows, up.TL->ncols, up.TL->K, st));
    Vout = ctx->Vb;
    if (ctx->prec == TRD_PREC_BF16X3) Vlo = ctx->Vb_lo;
    Vstride = up.TL->K;
  }
  if (sp.q == 1) {
    CK(launch_pack(ctx->dtype, L, nL, r0, rB, Vout, Vstride, 1, st, bf, Vlo));
    if (bf) TRY(fragment_coltable(ctx, up, st));
    return TRD_OK;
  }
  void* bufs[2] = {ctx->chainA, ctx->chainB};
  for (int t = 1; t < sp.q; ++t) {
    const int m = sp.C[t];
    const int rC = ctx->ranks[(m + 1) % N];
    const bool last = t == sp.q - 1;
    void* out = last ? Vout : bufs[t & 1];
    CK(launch_merge(ctx->dtype, L, nL, r0, rB, core_ref(ctx, cores[m], m, up.lists), up.counts[m],
                    rC, out, last ? Vstride : (int64_t)r0 * rC, last ? 1 : 0, st, last && bf,
                    last ? Vlo : nullptr));
    L.ptr = out;
    L.stride = (int64_t)r0 * rC;
    L.list = nullptr;
    nL *= up.counts[m];
    rB = rC;
  }
  if (bf) TRY(fragment_coltable(ctx, up, st));
  return TRD_OK;
}

PassArgs pass_args(trd_ctx* ctx, const Update& up) {
  PassArgs a;
  memset(&a, 0, sizeof(a));
  const Layout& L = *up.L;
  a.T = ctx->T;
  a.TH = ctx->TH;
  a.V = ctx->V;
  a.S = ctx->S;
  a.vals = L.vals;
  a.cols = L.cols;
  a.slice_off = L.slice_off;
  a.slice_len = L.slice_len;
  a.resid = ctx->resid;
  a.colw = up.colw;
  a.partials = ctx->part_pass;
  a.sigma = ctx->scal + kSigma;
  a.nrows = L.nrows;
  a.ncols = L.ncols;
  a.n_rg = L.n_rg;
  a.ct_w = L.ct_w;
  a.RR = up.sp.RR;
  a.RRP = up.sp.RRP;
  a.n_ct = L.n_ct;
  a.n_cg = L.n_cg;
  a.cpg = L.cpg;
  return a;
}

int64_t n_wg(const Layout& L) { return L.n_rg * L.n_cg; }
int64_t up_nwg(const Update& up) { return up.TL ? up.TL->n_rg * up.TL->n_cg : n_wg(*up.L); }
// number of gradient partials of a pass (one per column group)
int up_nct(const Update& up) { return up.TL ? up.TL->n_cg : up.L->n_cg; }
const int64_t* up_nobs_dev(const Update& up) { return up.TL ? up.TL->total_dev : up.L->nobs_dev; }

int ensure_bf16_tables(trd_ctx* ctx, int64_t nrows, int64_t ncols, int K, hipStream_t st) {
  const bool split = ctx->prec == TRD_PREC_BF16X3;
  if (nrows * K > ctx->cap_Tb) {
    TRY(alloc_n(ctx, &ctx->Tb, nrows * K));
    TRY(alloc_n(ctx, &ctx->THb, nrows * K));
    ctx->cap_Tb = nrows * K;
  }
  if (split && nrows * K > ctx->cap_Tlo) {
    TRY(alloc_n(ctx, &ctx->Tb_lo, nrows * K));
    ctx->cap_Tlo = nrows * K;
  }
  // column tables as the builders write them ([ncols][K]); the passes read the
  // fragment-order copies below
  if (ncols * K > ctx->cap_Vb) {
    TRY(alloc_n(ctx, &ctx->Vb, ncols * K));
    ctx->cap_Vb = ncols * K;
  }
  if (split && ncols * K > ctx->cap_Vlo) {
    TRY(alloc_n(ctx, &ctx->Vb_lo, ncols * K));
    ctx->cap_Vlo = ncols * K;
  }
  // fragment-order copies read by the matrix-core passes (written whole, padding
  // included, after every column table)
  const int64_t nf = tile_frag_elems(ncols, K);
  if (nf > ctx->cap_Vf) {
    TRY(alloc_n(ctx, &ctx->Vf, nf));
    TRY(alloc_n(ctx, &ctx->VTf, nf));
    ctx->cap_Vf = nf;
  }
  if (split && nf > ctx->cap_Vflo) {
    TRY(alloc_n(ctx, &ctx->Vf_lo, nf));
    ctx->cap_Vflo = nf;
  }
  return TRD_OK;
}

// matrix-core pass (its bf16 tables are written by the table builders)
// keep_w: a gradient pass stores each entry's weight for the line search that follows it
// Uc: U(m_B) of a gradient pass that contracts its row factors itself (B-major layout)
int launch_tile_pass(trd_ctx* ctx, const Update& up, int mode, hipStream_t st, bool keep_w,
                     const ItemRef* Uc, KTiming tm = {}) {
  const TLayout& TL = *up.TL;
  const Split& sp = up.sp;
  TPassArgs a;
  memset(&a, 0, sizeof(a));
  a.T = ctx->Tb;
  a.TH = ctx->THb;
  a.Vf = ctx->Vf;
  a.VTf = ctx->VTf;
  if (ctx->prec == TRD_PREC_BF16X3) {
    a.T_lo = ctx->Tb_lo;
    a.Vf_lo = ctx->Vf_lo;
  }
  a.S = (float*)ctx->S;
  a.boff = TL.boff;
  a.vals = TL.vals;
  a.pos = TL.pos;
  a.resid = ctx->resid;
  // the residual pass also counts the first quantile digit (launch_quantile_init first)
  a.qhist = mode == kModeResid ? ctx->qhist : nullptr;
  a.partials = ctx->part_pass;
  a.sigma = ctx->scal + kSigma;
  a.nrows = TL.nrows;
  a.ncols = TL.ncols;
  a.n_chunks = TL.n_chunks;
  a.n_rb = TL.n_rb;
  a.n_rg = TL.n_rg;
  a.CW = TL.CW;
  a.n_chpt = TL.n_chpt;
  a.cpg = TL.cpg;
  a.n_cg = TL.n_cg;
  a.RR = sp.RR;
  a.RRP = sp.RRP;
  // eight register rounds only for blocks that average more than 224 entries (of 2048
  // positions): below that, a block rarely needs a fifth round from memory
  a.rounds = TL.n_blocks > 0 && TL.nobs > 224 * TL.n_blocks ? 8 : 4;
  a.nobs = TL.nobs;
  a.nB = TL.nB;
  a.Ik = TL.Ik;
  a.bmaj = TL.bmaj ? 1 : 0;
  const bool grad = mode == kModeGrad || mode == kModeGradFast || mode == kModeGradE;
  if (grad && Uc) {
    a.dpart = reinterpret_cast<float*>(ctx->part_misc);
    a.U = static_cast<const float*>(Uc->ptr);
    a.Us = Uc->stride;
  }
  if (keep_w && grad) a.wout = ctx->wts;
  if (mode == kModeGradE) {  // the residual pass's e; no reconstruction, no split tables
    a.vals = ctx->resid;
    a.T_lo = nullptr;
    a.Vf_lo = nullptr;
  }
  if (mode == kModeLS) {  // weights of this update's gradient pass; q needs no split tables
    a.win = ctx->wts;
    a.T_lo = nullptr;
    a.Vf_lo = nullptr;
  }
  CK(launch_tpass(mode, TL.K, a, st, tm));
  return TRD_OK;
}

int run_pass(trd_ctx* ctx, const Update& up, int mode, hipStream_t st, bool keep_w = false,
             const ItemRef* Uc = nullptr) {
  // profiling: the tile passes hand their start and stop events to the launch, which sets
  // them at the kernel's own start and end (no marker packets on the stream); the
  // sliced-ELL passes (FP32 form, sketches) are bracketed by records: the sketched updates
  // are short and launch-bound, and launches with events made their sweeps slower
  const bool timed = ctx->prof && (mode == kModeGrad || mode == kModeGradFast);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (timed) {
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
  }
  if (up.TL) {
    KTiming tm;
    tm.start = e0;
    tm.stop = e1;
    TRY(launch_tile_pass(ctx, up, mode, st, keep_w, Uc, tm));
    // a pass with no work-groups launches nothing: a zero-length interval
    if (timed && (up.TL->n_rg * up.TL->n_cg <= 0 || up.TL->n_chunks <= 0)) {
      CK(hipEventRecord(e0, st));
      CK(hipEventRecord(e1, st));
    }
  } else {
    PassArgs a = pass_args(ctx, up);
    if (timed) CK(hipEventRecord(e0, st));
    CK(launch_pass(ctx->dtype, 0, mode, a, st));
    if (timed) CK(hipEventRecord(e1, st));
  }
  if (timed) {
    ctx->ev_pairs.push_back(e0);
    ctx->ev_pairs.push_back(e1);
    ctx->prof_slots += up.TL ? up.TL->nobs : up.L->slots;
    if (up.lists) {  // sketch: count known on the device only
      if (!ctx->prof_nobs_dev) {
        TRY(alloc_n(ctx, &ctx->prof_nobs_dev, 1));
        CK(launch_zero(ctx->prof_nobs_dev, sizeof(int64_t), st));
      }
      CK(launch_accum_i64(ctx->prof_nobs_dev, up.L->nobs_dev, st));
    } else {
      ctx->prof_entries += up.L->nobs;
    }
  }
  return TRD_OK;
}

// gradient of eq. (9)/(15) for the prepared update: tables, pass, contraction -> d64
// keep_w: a line search of the same update follows (the matrix-core pass keeps the weights)
// deferred (optional): on B-major layouts the caller adds the pass's d partials itself
// (launch_dpart_direction, after the Gram inverse); *deferred tells whether it must
int do_grad(trd_ctx* ctx, const Update& up, const void* const* cores, void* d_out, double scale,
            double* stats_dev, hipStream_t st, ItemRef* Uout, int64_t* nBout, bool keep_w = false,
            bool* deferred = nullptr) {
  const Split& sp = up.sp;
  const Layout& L = *up.L;
  int64_t needT, needV, needU, needC;
  table_needs(ctx, sp, up.counts, L.nrows, L.ncols, needT, needV, needU, needC);
  TRY(ensure_tables(ctx, needT, needV, needU, needC));
  const int64_t Ik = up.counts[sp.k];
  int64_t nB = 1;
  for (int t = 0; t < sp.p; ++t) nB *= up.counts[sp.B[t]];
  const int nchunk = contract_chunks(Ik, nB, sp.r_k);
  // B-major tile layout: the pass writes 2 x 64 floats of d partials per (column group,
  // 64-row block) into part_misc instead of its row factors
  const int64_t ndpart = up.TL && up.TL->bmaj ? (int64_t)up.TL->n_cg * up.TL->n_rb * 64 : 0;
  // (+ Ik: the slices' shares of <d, h> after the partials, when the caller adds them)
  TRY(ensure_part(ctx, up_nwg(up) * 3,
                  std::max<int64_t>(std::max<int64_t>((int64_t)nchunk * Ik * sp.r_k * sp.r_k1, 8),
                                    ndpart > 0 ? ndpart + Ik : 0)));
  const int64_t nd = Ik * sp.r_k * sp.r_k1;
  if (nd > ctx->cap_d) {
    TRY(alloc_n(ctx, &ctx->d64, nd));
    TRY(alloc_n(ctx, &ctx->h64, nd));
    TRY(dev_alloc(ctx, &ctx->h_real, nd * esz(ctx->dtype)));
    ctx->cap_d = nd;
  }
  // the residual pass of this sweep left e for this core: the gradient pass reads it, needs
  // no row table, and the column tables that pass built (same cores) are still in place
  const bool reuse_e = !stats_dev && up.TL && ctx->resid_core == sp.k;
  ItemRef Uref;
  TRY(build_U(ctx, up, cores, Uref, nB, st));
  if (!reuse_e) {
    TRY(build_rowtable(ctx, up, cores[sp.k], Uref, nB, ctx->T, st));
    TRY(build_coltable(ctx, up, cores, st));
  }
  // the pass contracts its own row factors (FP32 U items, 16-byte aligned, no list)
  const bool tile_contract = ndpart > 0 && Uref.ptr && !Uref.list && Uref.stride >= 64 &&
                             Uref.stride % 4 == 0 &&
                             reinterpret_cast<uintptr_t>(Uref.ptr) % 16 == 0;
  if (!tile_contract) TRY(ensure_S(ctx, (int64_t)up_nct(up) * L.nrows * sp.RRP));
  TRY(run_pass(ctx, up, stats_dev ? kModeGrad : (reuse_e ? kModeGradE : kModeGradFast), st, keep_w,
               tile_contract ? &Uref : nullptr));
  ctx->resid_core = -1;  // the core changes with this update
  if (stats_dev) CK(launch_reduce_partials(ctx->part_pass, up_nwg(up), 3, stats_dev, st));
  if (deferred) *deferred = tile_contract && !d_out && scale == 1.0;
  if (tile_contract) {
    if (!(deferred && *deferred))
      CK(launch_dpart_finish(reinterpret_cast<const float*>(ctx->part_misc), up.TL->n_cg,
                             up.TL->n_rb, up.TL->nB, Ik, ctx->d64, static_cast<float*>(d_out),
                             scale, st));
    if (Uout) *Uout = Uref;
    if (nBout) *nBout = nB;
    return TRD_OK;
  }
  // a few column-group partials are added by the contraction as it loads S; many are
  // first summed by a streaming kernel
  int ncg = up_nct(up);
  if (ncg > 4) {
    CK(launch_sum_partials(ctx->dtype, ctx->S, ncg, L.nrows * sp.RRP, st));
    ncg = 1;
  }
  CK(launch_contract(ctx->dtype, ctx->S, sp.RRP, ncg, L.nrows * sp.RRP, Ik, nB, sp.r_k, sp.r_s,
                     sp.r_k1, Uref, ctx->part_misc, nchunk, st));
  CK(launch_contract_finish(ctx->dtype, ctx->part_misc, nchunk, Ik, sp.r_k * sp.r_k1, ctx->d64,
                            d_out, scale, st));
  if (Uout) *Uout = Uref;
  if (nBout) *nBout = nB;
  return TRD_OK;
}

int ensure_dense(trd_ctx* ctx) {
  if (ctx->G) return TRD_OK;
  int64_t maxR2 = 1, maxr2 = 1;
  for (int j = 0; j < ctx->N; ++j) {
    const int64_t R = (int64_t)ctx->ranks[j] * ctx->ranks[(j + 1) % ctx->N];
    maxR2 = std::max(maxR2, R * R);
    maxr2 = std::max<int64_t>(maxr2, (int64_t)ctx->ranks[j] * ctx->ranks[j]);
  }
  // K_j is r_j^2 x r_{j+1}^2; ring partial products are r_{k+1}^2 x r_m^2
  for (int j = 0; j < ctx->N; ++j) TRY(alloc_n(ctx, &ctx->K[j], maxR2));
  for (int j = 0; j < ctx->N; ++j) TRY(alloc_n(ctx, &ctx->Kl[j], maxR2));
  TRY(alloc_n(ctx, &ctx->P0, maxr2 * maxr2));
  TRY(alloc_n(ctx, &ctx->P1, maxr2 * maxr2));
  TRY(alloc_n(ctx, &ctx->G, maxR2));
  TRY(alloc_n(ctx, &ctx->Cinv, maxR2));
  return TRD_OK;
}

int refresh_K(trd_ctx* ctx, const void* const* cores, int j, hipStream_t st) {
  CK(launch_kron_factor(ctx->dtype, cores[j], ctx->ranks[j], ctx->dims[j], ctx->ranks[(j + 1) % ctx->N],
                        ctx->K[j], st));
  return TRD_OK;
}

// G^{!=k} from the cached factors (eq. 13): ring product in cyclic order, realigned.
// Ks: other factors (those of sampled cores), nullptr: the cached ones of the full cores
int ring_gram(trd_ctx* ctx, int k, double* G_out, hipStream_t st, double* const* Ks = nullptr) {
  CK(launch_ring_gram(ctx->N, ctx->ranks, k, Ks ? Ks : ctx->K, ctx->P0, ctx->P1, G_out, g_lds_max, st));
  return TRD_OK;
}

int set_sigma(trd_ctx* ctx, double sigma, hipStream_t st) {
  CK(launch_set_scalar(ctx->scal + kSigma, sigma, st));
  return TRD_OK;
}

int ensure_side(trd_ctx* ctx) {
  if (ctx->side) return TRD_OK;
  CK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
  CK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
  CK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  return TRD_OK;
}

// one full core update (eqs. 9-12 / 15-18); K factors of the other cores must be current,
// except that of core `stale` (>= 0), refreshed here first: with the scaled direction on the
// second stream, just before the Gram that reads it (its core was updated by the step before)
int do_step(trd_ctx* ctx, void* const* cores, int k, double lambda_rel, const trd_sketch* sk,
            double* eta_user, uint32_t* flags_user, hipStream_t st, int stale = -1,
            const uint32_t* halt = nullptr) {
  Update up;
  ctx->lev_lambda = lambda_rel;
  // the step's flags start at zero: on the full path with the scaled direction nothing
  // writes them before the Gram inverse on the second stream, which sets the whole word;
  // otherwise cleared here, before the sketch (it may flag clamping)
  const bool inverse_clears = ctx->direction == TRD_DIR_SCALED && !sk;
  if (!inverse_clears) CK(launch_zero(ctx->flags, sizeof(uint32_t), st));
  TRY(prepare_update(ctx, k, sk, up, st, cores));
  const Split& sp = up.sp;
  const int64_t Ik = ctx->dims[k];
  const int R = sp.r_k * sp.r_k1;
  // the unscaled direction (h = d) needs no Gram; the local Gram (sampled cores) differs
  // from the global one only under a sketch
  const bool scaled = ctx->direction == TRD_DIR_SCALED;
  const bool local = scaled && ctx->gram == TRD_GRAM_LOCAL && sk;
  if (local && up.rows)
    return fail(ctx, TRD_EUNSUPPORTED, "the local Gram matrix needs RStS index sets, not a row sample");
  if (stale >= 0 && !scaled) TRY(refresh_K(ctx, (const void* const*)cores, stale, st));
  if (scaled) {
    // G (eq. 13) and (G + lambda I)^{-1} need only the factors of the other cores: on the
    // side stream, after everything queued so far, while the gradient runs here
    TRY(ensure_side(ctx));
    CK(hipEventRecord(ctx->ev_fork, st));
    CK(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    if (stale >= 0) TRY(refresh_K(ctx, (const void* const*)cores, stale, ctx->side));
    if (local) {  // factors of the sampled slices I_j of every other core (Sec. 6.1)
      for (int j = 0; j < ctx->N; ++j)
        if (j != k)
          CK(launch_kron_factor(ctx->dtype, cores[j], ctx->ranks[j], up.cnt[j],
                                ctx->ranks[(j + 1) % ctx->N], ctx->Kl[j], ctx->side, up.lst[j]));
    }
    TRY(ring_gram(ctx, k, ctx->G, ctx->side, local ? ctx->Kl : nullptr));
    CK(launch_inverse(ctx->G, ctx->Cinv, R, lambda_rel, ctx->flags, ctx->side, inverse_clears));
    CK(hipEventRecord(ctx->ev_join, ctx->side));
  }
  ItemRef Uref;
  int64_t nB;
  bool deferred = false;
  TRY(do_grad(ctx, up, (const void* const*)cores, nullptr, 1.0, nullptr, st, &Uref, &nB, true,
              &deferred));
  if (scaled) CK(hipStreamWaitEvent(st, ctx->ev_join, 0));
  // <d, h> partials: per 256 elements of h, or (B-major layouts, where one kernel adds the
  // pass's d partials and applies the inverse per slice) per slice, after the d partials
  int64_t nbl = (Ik * R + 255) / 256;
  double* pnum = ctx->part_misc;
  if (deferred) {
    const TLayout& TL = *up.TL;
    nbl = Ik;
    pnum = ctx->part_misc + TL.n_cg * TL.n_rb * 64;
    CK(launch_dpart_direction(reinterpret_cast<const float*>(ctx->part_misc), TL.n_cg, TL.n_rb,
                              TL.nB, Ik, scaled ? ctx->Cinv : nullptr, ctx->flags, ctx->d64,
                              ctx->h64, static_cast<float*>(ctx->h_real), pnum, st));
  } else {
    TRY(ensure_part(ctx, 0, nbl));
    CK(launch_apply_inverse(ctx->d64, scaled ? ctx->Cinv : nullptr, Ik, R, ctx->h64, ctx->h_real,
                            ctx->dtype, ctx->part_misc, ctx->flags, st));
  }
  TRY(build_rowtable(ctx, up, ctx->h_real, Uref, nB, ctx->TH, st));
  TRY(run_pass(ctx, up, kModeLS, st));
  CK(launch_finish_step(ctx->dtype, pnum, nbl, ctx->part_pass, up_nwg(up),
                        up_nobs_dev(up), ctx->flags, flags_user, ctx->scal + kEta, eta_user, cores[k],
                        ctx->h64, Ik * R, halt, st));
  return TRD_OK;
}

int check_ctx(trd_ctx* ctx, bool need_problem = true) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  if (need_problem && !ctx->has_problem) return fail(ctx, TRD_ESTATE, "call trd_set_problem first");
  if (!ctx->has_shape) return fail(ctx, TRD_ESTATE, "call trd_set_shape or trd_set_problem first");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(ctx, TRD_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  return TRD_OK;
}

int check_cores(trd_ctx* ctx, const void* const* cores) {
  if (!cores) return fail(ctx, TRD_EINVAL, "cores is NULL");
  for (int j = 0; j < ctx->N; ++j)
    if (!cores[j]) return fail(ctx, TRD_EINVAL, "cores[" + std::to_string(j) + "] is NULL");
  return TRD_OK;
}

int check_sigma(trd_ctx* ctx, double sigma) {
  if (!(sigma > 0.0)) return fail(ctx, TRD_EINVAL, "sigma must be > 0 (or +inf)");
  return TRD_OK;
}

int check_sketch(trd_ctx* ctx, const trd_sketch* sk, int k) {
  if (!sk) return TRD_OK;
  for (int j = 0; j < ctx->N; ++j) {
    if (j == k) continue;
    if (sk->sizes[j] < 1) return fail(ctx, TRD_EINVAL, "sketch sizes must be >= 1");
    if (sk->idx && !sk->idx[j]) return fail(ctx, TRD_EINVAL, "sketch idx[j] is NULL");
  }
  return TRD_OK;
}

}  // namespace

// ==================================================================== C ABI

extern "C" {

int trd_create(trd_ctx** out, int device) {
  if (!out) return fail(nullptr, TRD_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0)
    return fail(nullptr, TRD_EDEVICE, std::string("no HIP device: ") + hipGetErrorString(e));
  if (device < 0 || device >= n) return fail(nullptr, TRD_EINVAL, "device index out of range");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail(nullptr, TRD_EDEVICE, hipGetErrorString(e));
  g_lds_max = (int64_t)prop.sharedMemPerBlock;
  if (prop.multiProcessorCount > 0) g_num_cu = prop.multiProcessorCount;
  trd_ctx* c = new (std::nothrow) trd_ctx();
  if (!c) return fail(nullptr, TRD_ENOMEM, "host allocation failed");
  c->device = device;
  *out = c;
  return TRD_OK;
}

void trd_destroy(trd_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (hipEvent_t ev : ctx->ev_pairs) hipEventDestroy(ev);
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  if (ctx->side) hipStreamDestroy(ctx->side);
  free_all(ctx);
  delete ctx;
}

const char* trd_last_error(const trd_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_free_err.c_str();
}

int trd_set_shape(trd_ctx* ctx, int N, const int64_t* dims, const int32_t* ranks, int dtype) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  if (N < 2 || N > kMaxN) return fail(ctx, TRD_EUNSUPPORTED, "N must be in [2, 8]");
  if (!dims || !ranks) return fail(ctx, TRD_EINVAL, "NULL argument");
  if (dtype != TRD_F32 && dtype != TRD_F64) return fail(ctx, TRD_EINVAL, "dtype must be TRD_F32 or TRD_F64");
  double total = 1.0;
  for (int j = 0; j < N; ++j) {
    if (dims[j] < 1) return fail(ctx, TRD_EINVAL, "dims must be >= 1");
    if (ranks[j] < 1) return fail(ctx, TRD_EINVAL, "ranks must be >= 1");
    if (ranks[j] > kMaxRank) return fail(ctx, TRD_EUNSUPPORTED, "ranks must be <= 16");
    total *= (double)dims[j];
  }
  if (total >= 4.6e18) return fail(ctx, TRD_EUNSUPPORTED, "prod(dims) must be < 2^62");
  hipError_t he = hipSetDevice(ctx->device);
  if (he != hipSuccess) return fail(ctx, TRD_EDEVICE, hipGetErrorString(he));
  CK(hipDeviceSynchronize());
  free_all(ctx);
  const int device = ctx->device;
  for (hipEvent_t ev : ctx->ev_pairs) hipEventDestroy(ev);
  if (ctx->ev_fork) hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) hipEventDestroy(ctx->ev_join);
  if (ctx->side) hipStreamDestroy(ctx->side);
  *ctx = trd_ctx();
  ctx->device = device;
  ctx->N = N;
  ctx->dtype = dtype;
  int64_t s = 1;
  for (int j = 0; j < N; ++j) {
    ctx->dims[j] = dims[j];
    ctx->ranks[j] = ranks[j];
    ctx->strides[j] = s;
    s *= dims[j];
  }
  TRY(alloc_n(ctx, &ctx->scal, kScalCount));
  TRY(alloc_n(ctx, &ctx->flags, 4));
  TRY(ensure_dense(ctx));
  ctx->has_shape = true;
  return TRD_OK;
}

int trd_set_problem(trd_ctx* ctx, int N, const int64_t* dims, const int32_t* ranks, int dtype,
                    const void* X, const uint8_t* mask, void* stream) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  if (N < 2 || N > kMaxN) return fail(ctx, TRD_EUNSUPPORTED, "N must be in [2, 8]");
  if (!dims || !ranks || !X || !mask) return fail(ctx, TRD_EINVAL, "NULL argument");
  if (dtype != TRD_F32 && dtype != TRD_F64) return fail(ctx, TRD_EINVAL, "dtype must be TRD_F32 or TRD_F64");
  double total = 1.0;
  for (int j = 0; j < N; ++j) {
    if (dims[j] < 1) return fail(ctx, TRD_EINVAL, "dims must be >= 1");
    if (ranks[j] < 1) return fail(ctx, TRD_EINVAL, "ranks must be >= 1");
    if (ranks[j] > kMaxRank) return fail(ctx, TRD_EUNSUPPORTED, "ranks must be <= 16");
    total *= (double)dims[j];
  }
  if (total >= 4.6e18) return fail(ctx, TRD_EUNSUPPORTED, "prod(dims) must be < 2^62");
  hipStream_t st = (hipStream_t)stream;
  TRY(trd_set_shape(ctx, N, dims, ranks, dtype));  // drops any previous problem
  ctx->X = X;
  ctx->mask = mask;
  TRY(alloc_n(ctx, &ctx->qhist, 2048));
  TRY(alloc_n(ctx, &ctx->qstate, 4));
  TRY(alloc_n(ctx, &ctx->eta_hist, N));
  CK(hipHostMalloc((void**)&ctx->host_rep, kRepSlots * kRepStride * sizeof(double),
                  hipHostMallocMapped));
  CK(hipHostGetDevicePointer((void**)&ctx->host_rep_dev, ctx->host_rep, 0));
  CK(launch_zero(ctx->flags, 4 * sizeof(uint32_t), st));

  ctx->splits.resize(N);
  ctx->layouts.resize(N);
  ctx->tlayouts.assign(N, TLayout());
  int64_t needT = 0, needV = 0, needU = 0, needC = 0, needPass = 0, needMisc = 8, needD = 0;
  for (int k = 0; k < N; ++k) {
    int64_t nrows, ncols;
    int ct_w, n_ct;
    TRY(plan_split(ctx, k, ctx->dims, ctx->splits[k], nrows, ncols, ct_w, n_ct));
    Layout& L = ctx->layouts[k];
    L.k = k;
    layout_dims(L, nrows, ncols, ct_w, n_ct);
    TRY(alloc_layout_index(ctx, L));
    TRY(build_layout_head(ctx, ctx->splits[k], ctx->dims, nullptr, L, st));
    CK(hipMemcpyAsync(&L.slots, L.total_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (L.slots > 0) {
      TRY(dev_alloc(ctx, &L.vals, (size_t)L.slots * esz(dtype)));
      TRY(alloc_n(ctx, &L.cols, L.slots));
    }
    L.slots_cap = L.slots;
    CK(launch_fill(L, mask, X, dtype, st));
    int64_t a, b, c2, d;
    table_needs(ctx, ctx->splits[k], ctx->dims, nrows, ncols, a, b, c2, d);
    needT = std::max(needT, a);
    needV = std::max(needV, b);
    needU = std::max(needU, c2);
    needC = std::max(needC, d);
    needPass = std::max(needPass, n_wg(L) * 3);
    const Split& sp = ctx->splits[k];
    int64_t nB = 1;
    for (int t = 0; t < sp.p; ++t) nB *= ctx->dims[sp.B[t]];
    const int64_t R = (int64_t)sp.r_k * sp.r_k1;
    needMisc = std::max(needMisc, (int64_t)contract_chunks(dims[k], nB, sp.r_k) * dims[k] * R);
    needMisc = std::max(needMisc, (dims[k] * R + 255) / 256);
    needD = std::max(needD, dims[k] * R);
  }
  // sweep-end convergence buffers (Alg. 1)
  {
    const int64_t IN = dims[N - 1];
    const int64_t R = (int64_t)ranks[N - 1] * ranks[0];
    TRY(alloc_n(ctx, &ctx->Dbuf[0], IN * IN));
    TRY(alloc_n(ctx, &ctx->Dbuf[1], IN * IN));
    TRY(alloc_n(ctx, &ctx->M, IN * R));
    needMisc = std::max(needMisc, 2 * ((IN * IN + 255) / 256));
  }
  TRY(ensure_tables(ctx, needT, needV, needU, needC));
  TRY(ensure_part(ctx, needPass, needMisc));
  TRY(alloc_n(ctx, &ctx->d64, needD));
  TRY(alloc_n(ctx, &ctx->h64, needD));
  TRY(dev_alloc(ctx, &ctx->h_real, needD * esz(dtype)));
  ctx->cap_d = needD;
  // residual buffer for the kernel-width quantile (layout of core 0)
  ctx->cap_resid = std::max<int64_t>(ctx->layouts[0].slots, 1);
  TRY(alloc_n(ctx, &ctx->resid, ctx->cap_resid));
  CK(launch_max_abs_observed(ctx->layouts[0], dtype, ctx->scal + kMaxAbs, st));
  CK(hipMemcpyAsync(&ctx->nobs, ctx->layouts[0].nobs_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(&ctx->maxabs, ctx->scal + kMaxAbs, sizeof(double), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  for (int k = 0; k < N; ++k) ctx->layouts[k].nobs = ctx->nobs;
  ctx->has_problem = true;
  return TRD_OK;
}

int trd_problem_info(const trd_ctx* ctx, int64_t* n_obs, size_t* workspace_bytes, int32_t* split) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  if (!ctx->has_problem) return fail(const_cast<trd_ctx*>(ctx), TRD_ESTATE, "no problem bound");
  if (n_obs) *n_obs = ctx->nobs;
  if (workspace_bytes) *workspace_bytes = ctx->ws_bytes;
  if (split)
    for (int k = 0; k < ctx->N; ++k) split[k] = ctx->splits[k].p;
  return TRD_OK;
}

int trd_workspace_bytes(int device, int N, const int64_t* dims, const int32_t* ranks, int dtype,
                        int precision, int64_t n_obs, size_t* bound, size_t* typical) {
  if (N < 2 || N > kMaxN) return fail(nullptr, TRD_EUNSUPPORTED, "N must be in [2, 8]");
  if (!dims || !ranks || (!bound && !typical)) return fail(nullptr, TRD_EINVAL, "NULL argument");
  if (dtype != TRD_F32 && dtype != TRD_F64) return fail(nullptr, TRD_EINVAL, "dtype must be TRD_F32 or TRD_F64");
  if (precision != TRD_PREC_NATIVE && !bf16_form(precision)) return fail(nullptr, TRD_EINVAL, "unknown precision");
  if (bf16_form(precision) && dtype != TRD_F32)
    return fail(nullptr, TRD_EUNSUPPORTED, "the BF16 form needs an FP32 problem");
  double total = 1.0;
  for (int j = 0; j < N; ++j) {
    if (dims[j] < 1) return fail(nullptr, TRD_EINVAL, "dims must be >= 1");
    if (ranks[j] < 1 || ranks[j] > kMaxRank) return fail(nullptr, TRD_EUNSUPPORTED, "ranks must be in [1, 16]");
    total *= (double)dims[j];
  }
  if (total >= 4.6e18) return fail(nullptr, TRD_EUNSUPPORTED, "prod(dims) must be < 2^62");
  int64_t nent = 1;
  for (int j = 0; j < N; ++j) nent *= dims[j];
  if (n_obs < 0 || n_obs > nent) return fail(nullptr, TRD_EINVAL, "n_obs must be in [0, prod(dims)]");
  // the planning depends on the device (LDS per work-group, compute units) as in trd_create
  {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device < 0 || device >= n)
      return fail(nullptr, TRD_EDEVICE, std::string("no HIP device ") + std::to_string(device));
    int lds = 0, cus = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return fail(nullptr, TRD_EDEVICE, hipGetErrorString(e));
    g_lds_max = lds;
    if (cus > 0) g_num_cu = cus;
  }
  // a host-only context holding the shape, for the planning functions
  trd_ctx c;
  c.N = N;
  c.dtype = dtype;
  for (int j = 0; j < N; ++j) {
    c.dims[j] = dims[j];
    c.ranks[j] = ranks[j];
  }
  const int64_t e = (int64_t)esz(dtype);
  auto al = [](int64_t bytes) -> int64_t { return bytes > 0 ? bytes : 256; };  // dev_alloc
  int64_t fixed = 0, ell_bound = 0, ell_typ = 0;
  // trd_set_shape: scalars, flags, FGMC factors (full and sampled), ring partials, G, inverse
  int64_t maxR2 = 1, maxr2 = 1;
  for (int j = 0; j < N; ++j) {
    const int64_t R = (int64_t)ranks[j] * ranks[(j + 1) % N];
    maxR2 = std::max(maxR2, R * R);
    maxr2 = std::max<int64_t>(maxr2, (int64_t)ranks[j] * ranks[j]);
  }
  fixed += al(16 * 8) + al(4 * 4) + 2 * N * al(maxR2 * 8) + 2 * al(maxr2 * maxr2 * 8) + 2 * al(maxR2 * 8);
  // trd_set_problem
  fixed += al(2048 * 4) + al(4 * 4) + al(N * 8) + al(8);  // (+ trd_profile's counter)
  int64_t needT = 0, needV = 0, needU = 0, needC = 0, needPass = 0, needMisc = 8, needD = 0;
  int64_t growS = 0, growPass = 0, slots0 = 0, slots0_typ = 0;
  std::vector<Split> sps(N);
  std::vector<int64_t> nr(N), nc(N);
  for (int k = 0; k < N; ++k) {
    int ct_w, n_ct;
    const int r = plan_split(&c, k, dims, sps[k], nr[k], nc[k], ct_w, n_ct);
    if (r != TRD_OK) return fail(nullptr, r, c.err);
    Layout L;
    layout_dims(L, nr[k], nc[k], ct_w, n_ct);
    fixed += al(L.nrows * 8) + al(L.ncols * 8) + al((int64_t)L.n_ct * L.n_rg * kRowsPerWG * 4) +
             al(L.n_slices * 4) + al((L.n_slices + 1) * 8) + 2 * al(8);
    // sliced ELL: 64 x (longest row of the 64-row slice, rounded up to kGroup) per slice;
    // at worst every observed entry of a slice sits in one row
    const int64_t wpad = (ct_w + kGroup - 1) / kGroup * kGroup;
    const int64_t dense = L.n_slices * kWave * wpad;
    const int64_t worst = std::min(dense, (int64_t)kWave * n_obs + (int64_t)kWave * (kGroup - 1) *
                                                                    std::min(L.n_slices, n_obs));
    // a uniformly random mask: row counts ~ Binomial(ct_w, rho); their maximum over 64 rows
    // stays below mean + 3 standard deviations + 1 with high probability
    const double rho = (double)n_obs / (double)nent;
    const double mu = rho * ct_w, sd = std::sqrt(std::max(0.0, mu * (1.0 - rho)));
    const int64_t mx = std::min<int64_t>(ct_w, (int64_t)std::ceil(mu + 3.0 * sd + 1.0));
    const int64_t typ = n_obs == 0 ? 0 : std::min(dense, L.n_slices * kWave * ((mx + kGroup - 1) / kGroup * kGroup));
    ell_bound += worst > 0 ? al(worst * e) + al(worst * 2) : 0;
    ell_typ += typ > 0 ? al(typ * e) + al(typ * 2) : 0;
    if (k == 0) {
      slots0 = worst;
      slots0_typ = typ;
    }
    int64_t a, b, c2, d;
    table_needs(&c, sps[k], dims, nr[k], nc[k], a, b, c2, d);
    needT = std::max(needT, a);
    needV = std::max(needV, b);
    needU = std::max(needU, c2);
    needC = std::max(needC, d);
    needPass = std::max(needPass, n_wg(L) * 3);
    int64_t nB = 1;
    for (int t = 0; t < sps[k].p; ++t) nB *= dims[sps[k].B[t]];
    const int64_t R = (int64_t)sps[k].r_k * sps[k].r_k1;
    needMisc = std::max(needMisc, (int64_t)contract_chunks(dims[k], nB, sps[k].r_k) * dims[k] * R);
    needMisc = std::max(needMisc, (dims[k] * R + 255) / 256);
    needD = std::max(needD, dims[k] * R);
    // gradient partials (grown per core on first use: summed, an upper bound)
    growS += al((int64_t)L.n_cg * L.nrows * sps[k].RRP * e);
  }
  {
    const int64_t IN = dims[N - 1], R = (int64_t)ranks[N - 1] * ranks[0];
    fixed += 2 * al(IN * IN * 8) + al(IN * R * 8);
    needMisc = std::max(needMisc, 2 * ((IN * IN + 255) / 256));
  }
  fixed += 2 * al(needT * e) + al(needV * e) + (needU > 0 ? al(needU * e) : 0) + 2 * al(needC * e);
  fixed += al(needPass * 8) + al(needMisc * 8) + 2 * al(needD * 8) + al(needD * e);
  int64_t bnd = fixed + ell_bound + growS, typ = fixed + ell_typ + growS;
  bnd += al(std::max<int64_t>(slots0, 1) * 4);      // residual keys (layout of core 0)
  typ += al(std::max<int64_t>(slots0_typ, 1) * 4);
  auto quantile_bytes = [&](int64_t nkeys) {
    const int64_t ng = quantile_grid(nkeys);
    return al(ng * quantile_seg_cap(nkeys) * 4) + al(ng * 4);
  };
  if (!bf16_form(precision)) {
    bnd += quantile_bytes(slots0);
    typ += quantile_bytes(slots0_typ);
  } else {
    // matrix-core passes: block layouts per core, stored weights, bf16 tables (grown per
    // core: summed), their gradient partials and stats, the residuals of the quantile pass
    const bool split = precision == TRD_PREC_BF16X3;
    int64_t tiles = 0;
    for (int k = 0; k < N; ++k) {
      TLayout T;
      plan_tile(sps[k], nr[k], nc[k], dims[k], T);
      if (T.bmaj) tiles += al(T.n_cg * T.n_rb * 2 * 64 * 4);  // the epilogue's d partials
      tiles += al(T.n_blocks * 4) + al((T.n_blocks + 1) * 8) + al(8) + al((n_obs + kTileSlack) * 4) +
               al((n_obs + kTileSlack) * 2);
      const int64_t K = T.K, nf = tile_frag_elems(nc[k], K);
      tiles += 2 * al(nr[k] * K * 2) + al(nc[k] * K * 2) + 2 * al(nf * 2);
      if (split) tiles += al(nr[k] * K * 2) + al(nc[k] * K * 2) + al(nf * 2);
      tiles += al((int64_t)T.n_cg * nr[k] * sps[k].RRP * e) + al(T.n_rg * T.n_cg * 3 * 8);
    }
    tiles += al((n_obs + kTileSlack + 1) * 2) + al((n_obs + kTileSlack) * 4) + quantile_bytes(n_obs);
    bnd += tiles;
    typ += tiles;
  }
  if (bound) *bound = (size_t)bnd;
  if (typical) *typical = (size_t)std::min(bnd, typ);
  return TRD_OK;
}

int trd_reconstruct(trd_ctx* ctx, const void* const* cores, const int64_t* lin_idx, int64_t n,
                    void* out, void* stream) {
  TRY(check_ctx(ctx, false));
  TRY(check_cores(ctx, cores));
  if (!out && n > 0) return fail(ctx, TRD_EINVAL, "out is NULL");
  if (n < 0) return fail(ctx, TRD_EINVAL, "n < 0");
  hipStream_t st = (hipStream_t)stream;
  if (!lin_idx) {
    int64_t tot = 1;
    for (int j = 0; j < ctx->N; ++j) tot *= ctx->dims[j];
    if (n != tot) return fail(ctx, TRD_EINVAL, "n must equal prod(dims) when lin_idx is NULL");
    // the whole tensor: one product of core 0's two subchain tables (Def. 2 halves)
    Update up;
    int64_t nrows, ncols;
    int ct_w, n_ct;
    if (plan_split(ctx, 0, ctx->dims, up.sp, nrows, ncols, ct_w, n_ct) == TRD_OK) {
      for (int j = 0; j < ctx->N; ++j) {
        up.cnt[j] = ctx->dims[j];
        up.lst[j] = nullptr;
      }
      up.counts = up.cnt;
      up.lists = nullptr;
      int64_t needT, needV, needU, needC;
      table_needs(ctx, up.sp, up.cnt, nrows, ncols, needT, needV, needU, needC);
      TRY(ensure_tables(ctx, needT, needV, needU, needC));
      ItemRef Uref;
      int64_t nB;
      TRY(build_U(ctx, up, cores, Uref, nB, st));
      TRY(build_rowtable(ctx, up, cores[0], Uref, nB, ctx->T, st));
      TRY(build_coltable(ctx, up, cores, st));
      CK(launch_table_product(ctx->dtype, ctx->T, ctx->V, nrows, ncols, up.sp.RRP, out, st));
      return TRD_OK;
    }
    ctx->err.clear();  // no split with r_0 r_s <= 128: one chain per entry below
  }
  CK(launch_reconstruct(ctx->dtype, ctx->N, ctx->dims, ctx->ranks, cores, lin_idx, n, out, st));
  return TRD_OK;
}

int trd_weights(const void* resid, int64_t n, int dtype, double sigma, void* w_out, void* stream) {
  trd_ctx* ctx = nullptr;
  if (!(sigma > 0.0)) return fail(nullptr, TRD_EINVAL, "sigma must be > 0 (or +inf)");
  if (dtype != TRD_F32 && dtype != TRD_F64) return fail(nullptr, TRD_EINVAL, "bad dtype");
  if (n < 0) return fail(nullptr, TRD_EINVAL, "n < 0");
  if (n > 0 && (!resid || !w_out)) return fail(nullptr, TRD_EINVAL, "NULL buffer");
  CK(launch_weights(dtype, resid, n, sigma, w_out, (hipStream_t)stream));
  return TRD_OK;
}

int trd_grad(trd_ctx* ctx, const void* const* cores, int k, double sigma, const trd_sketch* sketch,
             void* d_out, double* stats_dev, void* stream) {
  TRY(check_ctx(ctx));
  TRY(check_cores(ctx, cores));
  if (k < 0 || k >= ctx->N) return fail(ctx, TRD_EINVAL, "k out of range");
  TRY(check_sigma(ctx, sigma));
  TRY(check_sketch(ctx, sketch, k));
  if (!d_out) return fail(ctx, TRD_EINVAL, "d_out is NULL");
  hipStream_t st = (hipStream_t)stream;
  TRY(set_sigma(ctx, sigma, st));
  Update up;
  ctx->lev_lambda = 1e-9;
  TRY(prepare_update(ctx, k, sketch, up, st, cores));
  TRY(do_grad(ctx, up, cores, d_out, 1.0, stats_dev, st, nullptr, nullptr));
  return TRD_OK;
}

int trd_fgmc_gram(trd_ctx* ctx, const void* const* cores, int k, double* G_out, void* stream) {
  TRY(check_ctx(ctx, false));
  TRY(check_cores(ctx, cores));
  if (k < 0 || k >= ctx->N) return fail(ctx, TRD_EINVAL, "k out of range");
  if (!G_out) return fail(ctx, TRD_EINVAL, "G_out is NULL");
  hipStream_t st = (hipStream_t)stream;
  for (int j = 0; j < ctx->N; ++j)
    if (j != k) TRY(refresh_K(ctx, cores, j, st));
  TRY(ring_gram(ctx, k, G_out, st));
  return TRD_OK;
}

int trd_step(trd_ctx* ctx, void* const* cores, int k, double sigma, double lambda_rel,
             const trd_sketch* sketch, double* eta_dev, uint32_t* flags_dev, void* stream) {
  TRY(check_ctx(ctx));
  TRY(check_cores(ctx, (const void* const*)cores));
  if (k < 0 || k >= ctx->N) return fail(ctx, TRD_EINVAL, "k out of range");
  TRY(check_sigma(ctx, sigma));
  if (!(lambda_rel >= 0.0)) return fail(ctx, TRD_EINVAL, "lambda_rel must be >= 0");
  TRY(check_sketch(ctx, sketch, k));
  hipStream_t st = (hipStream_t)stream;
  TRY(set_sigma(ctx, sigma, st));
  for (int j = 0; j < ctx->N; ++j)
    if (j != k) TRY(refresh_K(ctx, (const void* const*)cores, j, st));
  TRY(do_step(ctx, cores, k, lambda_rel, sketch, eta_dev, flags_dev, st));
  return TRD_OK;
}

int trd_fit(trd_ctx* ctx, void* const* cores, const trd_fit_opts* o, trd_fit_report* rep,
            void* stream) {
  TRY(check_ctx(ctx));
  TRY(check_cores(ctx, (const void* const*)cores));
  if (!o) return fail(ctx, TRD_EINVAL, "opts is NULL");
  if (o->max_sweeps < 1) return fail(ctx, TRD_EINVAL, "max_sweeps must be >= 1");
  if (!(o->lambda_rel >= 0.0)) return fail(ctx, TRD_EINVAL, "lambda_rel must be >= 0");
  if (o->precision != TRD_PREC_NATIVE && !bf16_form(o->precision))
    return fail(ctx, TRD_EINVAL, "unknown precision");
  if (bf16_form(o->precision) && ctx->dtype != TRD_F32)
    return fail(ctx, TRD_EUNSUPPORTED, "the BF16 form needs an FP32 problem");
  if (o->sigma_mode == TRD_SIGMA_FIXED) TRY(check_sigma(ctx, o->sigma));
  else if (o->sigma_mode == TRD_SIGMA_GIVEN) {
    if (!o->sigma_given) return fail(ctx, TRD_EINVAL, "sigma_given is NULL");
    for (int t = 0; t < o->max_sweeps; ++t) TRY(check_sigma(ctx, o->sigma_given[t]));
  } else if (o->sigma_mode == TRD_SIGMA_QUANTILE) {
    if (!(o->q >= 0.0 && o->q <= 1.0) || !(o->c > 0.0) || !(o->shrink >= 0.0) || !(o->sigma_min_rel >= 0.0))
      return fail(ctx, TRD_EINVAL, "bad quantile parameters");
  } else {
    return fail(ctx, TRD_EINVAL, "unknown sigma_mode");
  }
  trd_sketch skb;
  const trd_sketch* sk = nullptr;
  if (o->use_sketch) {
    memset(&skb, 0, sizeof(skb));
    skb.seed = o->seed;
    for (int j = 0; j < kMaxN; ++j) skb.sizes[j] = o->sketch_sizes[j];
    TRY(check_sketch(ctx, &skb, -1));
    sk = &skb;
  }
  hipStream_t st = (hipStream_t)stream;
  const int N = ctx->N;
  for (int j = 0; j < N; ++j) TRY(refresh_K(ctx, (const void* const*)cores, j, st));
  // the fit's flags and its halt word (set by the report of a sweep that hit NOTSPD)
  CK(launch_zero(ctx->flags + 1, 2 * sizeof(uint32_t), st));
  const uint32_t* halt = ctx->flags + 2;
  if (o->sigma_mode == TRD_SIGMA_QUANTILE) {
    CK(launch_set_scalar(ctx->scal + kSigma, INFINITY, st));
    // sigma_min = sigma_min_rel * max |x| over the observed entries
    CK(launch_set_scalar(ctx->scal + kSigmaMin, o->sigma_min_rel * ctx->maxabs, st));
  }
  if (rep) {
    rep->sweeps = 0;
    rep->last_e = INFINITY;
    rep->last_sigma = 0;
    rep->flags = 0;
  }
  // on every exit: the caller's precision comes back, and no stored residuals outlive the
  // fit (a later step or backward on core 0 must form its own)
  struct FitGuard {
    trd_ctx* c; int saved;
    ~FitGuard() { c->prec = saved; c->resid_core = -1; c->sk.lev_cache = false; }
  } guard{ctx, ctx->prec};
  ctx->prec = o->precision;
  // leverage distributions are kept between updates of this fit (every core starts stale)
  ctx->sk.lev_cache = true;
  for (int j = 0; j < kMaxN; ++j) ctx->sk.lev_valid[j] = false;
  int cur = 0;
  int stale = -1;  // core whose K factor the next step refreshes (all are current here)
  // Without a stop test (tol <= 0) the host queues the sweeps without waiting for their
  // reports: each sweep's report goes to its slot of a ring in pinned host memory, read
  // when the ring is full and at the end.  A sweep that hit NOTSPD ends the run; the
  // halt word its report sets makes the steps of the sweeps queued after it change no
  // core, so the cores are those of the sweeps the report covers.
  const bool batched = !(o->tol > 0.0);
  int next_read = 0;  // first sweep whose report is unread
  bool stop = false;
  int status = TRD_OK;
  for (int t = 0; t < o->max_sweeps && !stop; ++t) {
    if (sk) skb.sweep = t;
    // kernel width for this sweep
    if (o->sigma_mode == TRD_SIGMA_FIXED) {
      TRY(set_sigma(ctx, o->sigma, st));
    } else if (o->sigma_mode == TRD_SIGMA_GIVEN) {
      TRY(set_sigma(ctx, o->sigma_given[t], st));
    } else {
      Update up;
      ctx->lev_lambda = o->lambda_rel;
      TRY(prepare_update(ctx, 0, sk, up, st, (const void* const*)cores));
      const Layout& L = *up.L;
      // residual slots: ELL slots (padding holds +inf) or exactly the observed entries
      const int64_t nkeys = up.TL ? up.TL->nobs : L.slots_cap;
      const int64_t* nkeys_dev = up.TL ? up.TL->total_dev : L.total_dev;
      // (tile layouts: the same slack as the values, for the gradient pass that reads e)
      const int64_t need = up.TL ? nkeys + kTileSlack : nkeys;
      if (need > ctx->cap_resid) {
        TRY(alloc_n(ctx, &ctx->resid, need));
        ctx->cap_resid = need;
      }
      {  // per work-group candidate segments of the quantile's third digit
        const int64_t ng = quantile_grid(nkeys), ncand = ng * quantile_seg_cap(nkeys);
        if (ncand > ctx->cap_qcand) {
          TRY(alloc_n(ctx, &ctx->qcand, ncand));
          ctx->cap_qcand = ncand;
        }
        if (ng > ctx->cap_qcnt) {
          TRY(alloc_n(ctx, &ctx->qcand_cnt, ng));
          ctx->cap_qcnt = ng;
        }
      }
      ctx->resid_core = -1;
      int64_t needT, needV, needU, needC;
      table_needs(ctx, up.sp, up.counts, L.nrows, L.ncols, needT, needV, needU, needC);
      TRY(ensure_tables(ctx, needT, needV, needU, needC));
      TRY(ensure_part(ctx, up_nwg(up) * 3, 8));
      ItemRef Uref;
      int64_t nB;
      TRY(build_U(ctx, up, (const void* const*)cores, Uref, nB, st));
      TRY(build_rowtable(ctx, up, cores[0], Uref, nB, ctx->T, st));
      TRY(build_coltable(ctx, up, (const void* const*)cores, st));
      if (up.TL) CK(launch_quantile_init(up_nobs_dev(up), o->q, ctx->qstate, ctx->qhist, st));
      TRY(run_pass(ctx, up, kModeResid, st));
      if (up.TL) ctx->resid_core = 0;  // core 0's update reads these residuals
      CK(launch_quantile_sigma(ctx->resid, nkeys, nkeys_dev, o->q, o->c, ctx->scal + kSigmaMin,
                               o->shrink, ctx->scal + kSigma, ctx->qhist, ctx->qstate,
                               up_nobs_dev(up), ctx->qcand, ctx->qcand_cnt, up.TL != nullptr, st));
    }
    for (int k = 0; k < N; ++k) {
      // the factor of the core updated last is refreshed by this step, beside its gradient
      TRY(do_step(ctx, cores, k, o->lambda_rel, sk, ctx->eta_hist + k, ctx->flags + 1, st,
                  stale, halt));
      ctx->sk.lev_valid[k] = false;  // core k changed
      stale = k;
    }
    // convergence matrix with G^{!=N} of the full cores (it does not involve core N): the
    // last update left it in G unless that update formed no Gram (gradient direction) or the
    // Gram of the sampled cores (local ablation); then it is formed here from the factors
    {
      const int64_t IN = ctx->dims[N - 1];
      const int R = ctx->ranks[N - 1] * ctx->ranks[0];
      if (ctx->direction != TRD_DIR_SCALED || (ctx->gram == TRD_GRAM_LOCAL && sk))
        TRY(ring_gram(ctx, N - 1, ctx->G, st));
      CK(launch_convergence(ctx->dtype, cores[N - 1], ctx->G, IN, R, ctx->M, ctx->Dbuf[cur],
                            ctx->Dbuf[cur ^ 1], t > 0 ? 1 : 0, ctx->part_misc, st));
      CK(launch_reduce_partials(ctx->part_misc, (IN * IN + 255) / 256, 2, ctx->scal + kConv, st));
    }
    CK(launch_pack_report(ctx->scal + kSigma, ctx->scal + kConv, ctx->flags + 1, ctx->eta_hist, N,
                          ctx->host_rep_dev + (t % kRepSlots) * kRepStride, ctx->flags + 2, st));
    cur ^= 1;
    if (batched && t + 1 < o->max_sweeps && (t + 1) % kRepSlots != 0) continue;
    CK(hipStreamSynchronize(st));
    for (int u = next_read; u <= t && !stop; ++u) {
      const double* hr = ctx->host_rep + (u % kRepSlots) * kRepStride;
      const double sigma = hr[0];
      const uint32_t flags = (uint32_t)hr[3];
      const double e = u > 0 ? sqrt(hr[1]) / sqrt(hr[2]) : INFINITY;
      if (rep) {
        rep->sweeps = u + 1;
        rep->last_e = e;
        rep->last_sigma = sigma;
        rep->flags |= flags;
        if (rep->e_hist) rep->e_hist[u] = e;
        if (rep->sigma_hist) rep->sigma_hist[u] = sigma;
        if (rep->eta_hist)
          for (int k = 0; k < N; ++k) rep->eta_hist[(int64_t)u * N + k] = hr[4 + k];
      }
      if (flags & TRD_FLAG_NOTSPD) {
        status = fail(ctx, TRD_ENOTSPD, "G + lambda I not positive definite (eq. 10)");
        stop = true;
      } else if (u > 0 && e < o->tol) {
        stop = true;
      }
    }
    next_read = t + 1;
  }
  return status;
}

int trd_loss_fwd(trd_ctx* ctx, const void* const* cores, double sigma, double* loss_dev, void* stream) {
  TRY(check_ctx(ctx));
  TRY(check_cores(ctx, cores));
  TRY(check_sigma(ctx, sigma));
  if (!loss_dev) return fail(ctx, TRD_EINVAL, "loss_dev is NULL");
  hipStream_t st = (hipStream_t)stream;
  TRY(set_sigma(ctx, sigma, st));
  Update up;
  TRY(prepare_update(ctx, 0, nullptr, up, st));
  const Layout& L = *up.L;
  ItemRef Uref;
  int64_t nB;
  TRY(build_U(ctx, up, cores, Uref, nB, st));
  TRY(build_rowtable(ctx, up, cores[0], Uref, nB, ctx->T, st));
  TRY(build_coltable(ctx, up, cores, st));
  TRY(ensure_part(ctx, up_nwg(up) * 3, 8));
  TRY(run_pass(ctx, up, kModeLoss, st));
  CK(launch_reduce_partials(ctx->part_pass, up_nwg(up), 3, ctx->scal + kTmp, st));
  CK(hipMemcpyAsync(loss_dev, ctx->scal + kTmp, sizeof(double), hipMemcpyDeviceToDevice, st));
  return TRD_OK;
}

int trd_loss_bwd(trd_ctx* ctx, const void* const* cores, double sigma, double grad_scale,
                 void* const* grads_out, void* stream) {
  TRY(check_ctx(ctx));
  TRY(check_cores(ctx, cores));
  TRY(check_sigma(ctx, sigma));
  if (!grads_out) return fail(ctx, TRD_EINVAL, "grads_out is NULL");
  for (int j = 0; j < ctx->N; ++j)
    if (!grads_out[j]) return fail(ctx, TRD_EINVAL, "grads_out[j] is NULL");
  hipStream_t st = (hipStream_t)stream;
  TRY(set_sigma(ctx, sigma, st));
  for (int k = 0; k < ctx->N; ++k) {
    Update up;
    TRY(prepare_update(ctx, k, nullptr, up, st));
    TRY(do_grad(ctx, up, cores, grads_out[k], -grad_scale, nullptr, st, nullptr, nullptr));
  }
  return TRD_OK;
}

int trd_sample_sketch(uint64_t seed, int t, int k, int N, const int64_t* dims, const int32_t* sizes,
                      int32_t* const* idx_out, void* stream) {
  trd_ctx* ctx = nullptr;
  if (N < 2 || N > kMaxN) return fail(nullptr, TRD_EINVAL, "N must be in [2, 8]");
  if (!dims || !sizes || !idx_out) return fail(nullptr, TRD_EINVAL, "NULL argument");
  if (k < 0 || k >= N) return fail(nullptr, TRD_EINVAL, "k out of range");
  int32_t s[kMaxN];
  for (int j = 0; j < N; ++j) {
    if (dims[j] < 1 || dims[j] > 0x7FFFFFFF) return fail(nullptr, TRD_EINVAL, "bad dims");
    if (j != k && sizes[j] < 1) return fail(nullptr, TRD_EINVAL, "sizes must be >= 1");
    if (!idx_out[j]) return fail(nullptr, TRD_EINVAL, "idx_out[j] is NULL");
    s[j] = (int32_t)std::min<int64_t>(j == k ? dims[j] : sizes[j], dims[j]);
  }
  CK(launch_sample(seed, t, k, N, dims, s, idx_out, (hipStream_t)stream));
  return TRD_OK;
}

int trd_sample_leverage(trd_ctx* ctx, const void* const* cores, int k, uint64_t seed, int t, int64_t J,
                        double lambda_rel, int64_t* rows_out, double* weights_out, void* stream) {
  TRY(check_ctx(ctx, false));
  TRY(check_cores(ctx, cores));
  if (k < 0 || k >= ctx->N) return fail(ctx, TRD_EINVAL, "k out of range");
  if (J < 0) return fail(ctx, TRD_EINVAL, "J must be >= 0");
  if (J > 0 && (!rows_out || !weights_out)) return fail(ctx, TRD_EINVAL, "NULL output");
  if (!(lambda_rel >= 0.0)) return fail(ctx, TRD_EINVAL, "lambda_rel must be >= 0");
  if (J == 0) return TRD_OK;
  return sample_leverage(ctx, cores, k, seed, t, J, lambda_rel, nullptr, rows_out, weights_out,
                         (hipStream_t)stream);
}

int trd_sample_rows(uint64_t seed, int t, int k, int N, const int64_t* dims, int64_t J, int64_t* rows_out,
                    void* stream) {
  trd_ctx* ctx = nullptr;
  if (N < 2 || N > kMaxN) return fail(nullptr, TRD_EINVAL, "N must be in [2, 8]");
  if (!dims || (!rows_out && J > 0)) return fail(nullptr, TRD_EINVAL, "NULL argument");
  if (k < 0 || k >= N) return fail(nullptr, TRD_EINVAL, "k out of range");
  if (J < 0) return fail(nullptr, TRD_EINVAL, "J must be >= 0");
  double M = 1.0;
  for (int j = 0; j < N; ++j) {
    if (dims[j] < 1 || dims[j] > 0x7FFFFFFF) return fail(nullptr, TRD_EINVAL, "bad dims");
    if (j != k) M *= (double)dims[j];
  }
  if (M >= 4.6e18) return fail(nullptr, TRD_EUNSUPPORTED, "row count must be < 2^62");
  CK(launch_sample_rows(seed, t, k, N, dims, J, nullptr, rows_out, (hipStream_t)stream));
  return TRD_OK;
}

int trd_sample_mask(uint64_t seed, int N, const int64_t* dims, double rho, int block,
                    double outlier_frac, uint8_t* mask_out, uint8_t* outlier_out, double* u_out,
                    void* stream) {
  trd_ctx* ctx = nullptr;
  if (N < 2 || N > kMaxN) return fail(nullptr, TRD_EINVAL, "N must be in [2, 8]");
  if (!dims || !mask_out) return fail(nullptr, TRD_EINVAL, "NULL argument");
  double total = 1.0;
  for (int j = 0; j < N; ++j) {
    if (dims[j] < 1) return fail(nullptr, TRD_EINVAL, "dims must be >= 1");
    total *= (double)dims[j];
  }
  if (total >= 4.6e18) return fail(nullptr, TRD_EUNSUPPORTED, "prod(dims) must be < 2^62");
  if (std::isnan(rho) || std::isnan(outlier_frac)) return fail(nullptr, TRD_EINVAL, "rho / outlier_frac is NaN");
  if (block < 0) return fail(nullptr, TRD_EINVAL, "block must be >= 0");
  CK(launch_sample_mask(seed, N, dims, rho, block, outlier_frac, mask_out, outlier_out, u_out,
                        (hipStream_t)stream));
  return TRD_OK;
}

int trd_set_precision(trd_ctx* ctx, int precision) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  if (precision != TRD_PREC_NATIVE && !bf16_form(precision))
    return fail(ctx, TRD_EINVAL, "unknown precision");
  if (bf16_form(precision)) {
    if (!ctx->has_problem) return fail(ctx, TRD_ESTATE, "call trd_set_problem first");
    if (ctx->dtype != TRD_F32) return fail(ctx, TRD_EUNSUPPORTED, "the BF16 form needs an FP32 problem");
  }
  ctx->prec = precision;
  return TRD_OK;
}

int trd_set_variant(trd_ctx* ctx, int direction, int gram, int sampling) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  if (direction != TRD_DIR_SCALED && direction != TRD_DIR_GRADIENT)
    return fail(ctx, TRD_EINVAL, "unknown direction");
  if (gram != TRD_GRAM_GLOBAL && gram != TRD_GRAM_LOCAL) return fail(ctx, TRD_EINVAL, "unknown gram");
  if (sampling != TRD_SAMPLE_RSTS && sampling != TRD_SAMPLE_ROWS && sampling != TRD_SAMPLE_LEVERAGE)
    return fail(ctx, TRD_EINVAL, "unknown sampling");
  if (gram == TRD_GRAM_LOCAL && sampling != TRD_SAMPLE_RSTS && direction == TRD_DIR_SCALED)
    return fail(ctx, TRD_EUNSUPPORTED, "the local Gram matrix needs RStS index sets, not a row sample");
  ctx->direction = direction;
  ctx->gram = gram;
  ctx->sampling = sampling;
  return TRD_OK;
}

int trd_profile(trd_ctx* ctx, int enable) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  ctx->prof = enable != 0;
  return TRD_OK;
}

int trd_profile_read(trd_ctx* ctx, int64_t* launches, double* total_ms, int64_t* slots,
                     int64_t* entries) {
  if (!ctx) return fail(nullptr, TRD_EINVAL, "null context");
  hipSetDevice(ctx->device);
  double ms = 0.0;
  const int64_t n = (int64_t)ctx->ev_pairs.size() / 2;
  for (int64_t i = 0; i < n; ++i) {
    hipEvent_t a = ctx->ev_pairs[2 * i], b = ctx->ev_pairs[2 * i + 1];
    hipError_t e = hipEventSynchronize(b);
    if (e != hipSuccess) return fail(ctx, TRD_EDEVICE, hipGetErrorString(e));
    float f = 0.f;
    e = hipEventElapsedTime(&f, a, b);
    if (e != hipSuccess) return fail(ctx, TRD_EDEVICE, hipGetErrorString(e));
    ms += f;
    hipEventDestroy(a);
    hipEventDestroy(b);
  }
  ctx->ev_pairs.clear();
  int64_t dev_entries = 0;
  if (ctx->prof_nobs_dev) {
    hipError_t e = hipMemcpy(&dev_entries, ctx->prof_nobs_dev, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ctx, TRD_EDEVICE, hipGetErrorString(e));
    e = hipMemset(ctx->prof_nobs_dev, 0, sizeof(int64_t));
    if (e != hipSuccess) return fail(ctx, TRD_EDEVICE, hipGetErrorString(e));
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (slots) *slots = ctx->prof_slots;
  if (entries) *entries = ctx->prof_entries + dev_entries;
  ctx->prof_slots = 0;
  ctx->prof_entries = 0;
  return TRD_OK;
}

}  // extern "C"

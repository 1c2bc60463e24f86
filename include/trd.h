/*
 * trd.h -- C ABI of libtrd: the per-core update sweep of auto-weighted robust
 * tensor-ring decomposition (AWRTRD) and its sketched form (SAWRTRD), He & Atia,
 * "Scalable and Robust Tensor Ring Decomposition for Large-scale Data", UAI 2023.
 *
 * Every call is extern "C", takes plain pointers and sizes, never throws, and
 * returns TRD_OK (0) or a negative TRD_E* code; trd_last_error() gives the message.
 * Calls that take a `stream` (a hipStream_t passed as void*, NULL = default
 * stream) only enqueue work on it and return before it runs, unless stated.
 *
 * Conventions (0-based indices):
 *  - Tensor X with dims I_0..I_{N-1} is column-major: entry (i_0..i_{N-1}) sits at
 *    l = sum_j i_j * prod_{j'<j} I_{j'} (the index linearisation of Def. 2).
 *  - ranks[j] is r_j; core j is r_j x I_j x r_{(j+1) mod N} (Def. 1) and is stored
 *    as its mode-2 unfolding Z_{j(2)} row-major: element (a, i, b) at
 *    i*r_j*r_{j+1} + b*r_j + a, so each lateral slice Z_j(i) is a contiguous
 *    column-major r_j x r_{j+1} matrix.  d and h of eqs. (9)-(10) use the same layout.
 *  - `cores` arguments are host arrays of N device pointers, one per core, in the
 *    problem dtype.
 *  - Limits: 2 <= N <= 8, 1 <= r_j <= 16, r_k * r_s <= 128 for the pair the fused
 *    pass contracts (r_s the rank at the split of the subchain), every
 *    r_k*r_{k+1} <= 256, dims >= 1, prod(dims) < 2^62, observed entries < 2^31.
 *
 * Ownership: the library owns only the workspace inside a trd_ctx.  X, mask, cores
 * and all outputs are borrowed caller memory; they must stay valid until the
 * enqueued work that reads or writes them has finished.
 */
#ifndef TRD_H
#define TRD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TRD_OK            0
#define TRD_EINVAL       -1   /* bad argument */
#define TRD_ENOMEM       -2   /* device allocation failed */
#define TRD_EDEVICE      -3   /* HIP runtime error */
#define TRD_ENOTSPD      -4   /* G + lambda I not positive definite (eq. 10) */
#define TRD_ESTATE       -5   /* call needs trd_set_problem first */
#define TRD_EUNSUPPORTED -6   /* size outside the limits above */

/* element types */
#define TRD_F32 0
#define TRD_F64 1

/* precision of the entry-wise passes (problem dtype TRD_F32 only for BF16) */
#define TRD_PREC_NATIVE 0     /* subchain tables and passes in the problem dtype */
#define TRD_PREC_BF16   1     /* subchain tables in bf16, residual/weights/accumulators fp32 */
#define TRD_PREC_BF16X3 2     /* as BF16, with the reconstruction from split bf16 tables
                                 (hi + lo, three matrix-core products): ~16-bit residuals */

/* device flag bits written by trd_step / trd_fit */
#define TRD_FLAG_EMPTY     1u /* the update touched no observed entry: eta = 0 */
#define TRD_FLAG_ZERO_DEN  2u /* line-search denominator <= 0 or not finite: eta = 0 */
#define TRD_FLAG_NOTSPD    4u /* G + lambda I not positive definite: h = 0, eta = 0 */
#define TRD_FLAG_CLAMPED   8u /* a caller's sketch index list (trd_sketch.idx) held indices
                                 outside [0, I_j): they were clamped into range */

/* kernel-width schedule modes for trd_fit */
#define TRD_SIGMA_FIXED    0
#define TRD_SIGMA_GIVEN    1
#define TRD_SIGMA_QUANTILE 2

typedef struct trd_ctx trd_ctx;

/*
 * Randomized subtensor sketch (RStS, Sec. 4.3.2, eq. 14, Alg. 1): for update k
 * every mode j != k keeps sizes[j] lateral slices chosen uniformly without
 * replacement (sorted ascending), mode k keeps all I_k.  When `idx` is NULL the
 * library draws the sets itself from (seed, sweep, k, j) with the counter-based
 * SplitMix64 generator described at trd_sample_sketch; otherwise idx[j] (host array
 * of N device pointers) holds the caller's sorted index list for mode j, of length
 * sizes[j] (ignored for j == k).
 */
typedef struct trd_sketch {
  uint64_t seed;
  int32_t sweep;
  int32_t sizes[8];
  const int32_t* const* idx;
} trd_sketch;

typedef struct trd_fit_opts {
  int32_t max_sweeps;        /* C of Alg. 1 */
  double tol;                /* epsilon of Alg. 1 (no test after the first sweep) */
  double lambda_rel;         /* lambda of eq. (10) = lambda_rel * tr(G) / R^2 */
  int32_t sigma_mode;        /* TRD_SIGMA_* */
  double sigma;              /* FIXED: kernel width (+inf = masked least squares) */
  const double* sigma_given; /* GIVEN: host array, one width per sweep */
  double q, c, shrink;       /* QUANTILE: sigma_t = max(c*Q_q|e|, sigma_min, shrink*sigma_{t-1}) */
  double sigma_min_rel;      /* QUANTILE: sigma_min = sigma_min_rel * max |x| over observed */
  int32_t use_sketch;        /* 0: full path (AWRTRD); 1: RStS (SAWRTRD) */
  int32_t sketch_sizes[8];
  uint64_t seed;
  int32_t precision;         /* TRD_PREC_* */
} trd_fit_opts;

typedef struct trd_fit_report {
  int32_t sweeps;            /* sweeps run */
  double last_e;             /* relative change of D^t at the last sweep */
  double last_sigma;
  uint32_t flags;            /* OR of the step flags over the run */
  double* e_hist;            /* optional host array [max_sweeps] (NULL = skip) */
  double* sigma_hist;        /* optional host array [max_sweeps] */
  double* eta_hist;          /* optional host array [max_sweeps * N] */
} trd_fit_report;

/* Create a context on HIP device `device`.  Allocates nothing on the device yet. */
int trd_create(trd_ctx** out, int device);
/* Free the context and its workspace.  NULL is ignored. */
void trd_destroy(trd_ctx* ctx);
/* Message of the last failure on ctx (or of the last context-free call when ctx is NULL). */
const char* trd_last_error(const trd_ctx* ctx);

/*
 * Bind only the shape (N, dims, TR ranks, dtype) without data: enough for
 * trd_reconstruct and trd_fgmc_gram.  Drops any previously bound problem and its
 * workspace.  Synchronizes the device.
 */
int trd_set_shape(trd_ctx* ctx, int N, const int64_t* dims, const int32_t* ranks, int dtype);

/*
 * Bind a problem (Alg. 1 inputs X, mask P of eq. 2, TR ranks) and build the
 * observed-entry layouts, one per core: for core k the entries are grouped as a
 * matrix whose rows are (i_k, the first modes of the cyclic subchain) and whose
 * columns are the remaining modes (Thm. 1), cut into 256-row x column tiles and
 * stored as 64-row sliced ELL lists (value, column-in-tile).
 *  X: device, prod(dims) values of `dtype` (column-major).  mask: device uint8, same
 *  size, nonzero = observed.  Values where mask == 0 are never used.  Both are read
 *  only during this call and by later RStS updates (so keep them alive while
 *  sketches are used).  Synchronizes `stream`.  Returns TRD_EUNSUPPORTED outside the
 *  limits in the file header.
 */
int trd_set_problem(trd_ctx* ctx, int N, const int64_t* dims, const int32_t* ranks, int dtype,
                    const void* X, const uint8_t* mask, void* stream);

/*
 * Device workspace of a problem of this shape, before binding it (needs no context and
 * allocates nothing): the buffers trd_set_problem allocates (observed-entry layouts,
 * subchain tables, FGMC factors, Gram and partial sums) plus those a full-path trd_fit,
 * trd_step or trd_grad in `precision` adds (block layouts, bf16 tables, stored weights,
 * gradient partials, quantile buffers).  RStS sketch buffers are not included.  The tensor
 * has n_obs observed entries (0 <= n_obs <= prod(dims)) out of the mask of eq. (2).
 *  bound (optional): an upper bound for any mask with n_obs observed entries (at worst a
 *    64-row slice of a layout pads every row to its longest one);
 *  typical (optional): the same for a mask drawn uniformly at random (observed with
 *    probability n_obs / prod(dims) independently), <= bound.
 * `device` (HIP device index) fixes the planning (LDS per work-group, compute units), as
 * for trd_create.  TRD_EDEVICE without a device; message: trd_last_error(NULL).
 */
int trd_workspace_bytes(int device, int N, const int64_t* dims, const int32_t* ranks, int dtype,
                        int precision, int64_t n_obs, size_t* bound, size_t* typical);

/* Host-side query: observed count, bytes of device workspace held, and the
 * subchain split chosen for core k (rows = I_k times the first `split` modes). */
int trd_problem_info(const trd_ctx* ctx, int64_t* n_obs, size_t* workspace_bytes, int32_t* split);

/*
 * TR reconstruction (Def. 1) (needs trd_set_shape or trd_set_problem): out[t] = Tr(Z_0(i_0) ... Z_{N-1}(i_{N-1})) for the
 * entry at column-major linear index lin_idx[t] (device int64, n entries), or for
 * every entry in column-major order when lin_idx is NULL (then n must equal
 * prod(dims)).  out: device, problem dtype.
 */
int trd_reconstruct(trd_ctx* ctx, const void* const* cores, const int64_t* lin_idx, int64_t n,
                    void* out, void* stream);

/*
 * Correntropy weights of eq. (7): w = exp(-e^2 / (2 sigma^2)) (sign reading: the
 * printed g'(x)/x is negative for the stated kernel; w in (0, 1], w(0) = 1).
 * sigma = +inf gives w = 1.  resid, w_out: device, n values of dtype.
 * TRD_EINVAL for sigma <= 0 or NaN.  Needs no context.
 */
int trd_weights(const void* resid, int64_t n, int dtype, double sigma, void* w_out, void* stream);

/*
 * Gradient of eq. (9) (full path) or eq. (15) (sketch != NULL) for core k:
 * d = (W o P o (X_[k] - Z_{k(2)} A^T)) A with A the subchain unfolding, W from the
 * current residual.  d_out: device, I_k * r_k * r_{k+1} values of the problem dtype
 * (core layout).  stats_dev: optional device double[3] receiving
 * {sum sigma^2 (1 - w), sum w e^2, observed count} over the touched entries.
 */
int trd_grad(trd_ctx* ctx, const void* const* cores, int k, double sigma, const trd_sketch* sketch,
             void* d_out, double* stats_dev, void* stream);

/*
 * Gram matrix G^{!=k} = A^T A of the full subchain by FGMC (Prop. 2, eq. 13): the
 * ring product of K_j = sum_i Z_j(i) (x) Z_j(i) over j != k in cyclic order, then
 * realigned.  G_out: device double, R x R row-major with R = r_k r_{k+1} and row
 * index a + b*r_k (a < r_k, b < r_{k+1}).  Computed in FP64.
 */
int trd_fgmc_gram(trd_ctx* ctx, const void* const* cores, int k, double* G_out, void* stream);

/*
 * trd_fgmc_gram without a context and without any device allocation, for callers that
 * cannot allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same result as trd_fgmc_gram for the same cores (the same kernels, in
 * the same order), on the current HIP device and `stream`.  dims, ranks: host arrays of N;
 * cores: host array of N device pointers (cores[k] is not read); G_out as for
 * trd_fgmc_gram.  Its factors and ring partials live in a fixed 2 MiB device array held by
 * each device the call runs on until the process ends: shapes that need more (the N - 1
 * factors r_j^2 r_{j+1}^2 doubles, plus 2 r_{k+1}^2 max_j r_j^2 when a factor side exceeds
 * 64; ranks <= 12 always fit) return TRD_EUNSUPPORTED.  Calls on one device share that
 * array: calls that overlap on a device race, so serialise them.  Errors: trd_last_error(NULL).
 */
int trd_fgmc_gram_noalloc(int N, const int64_t* dims, const int32_t* ranks, int dtype,
                          const void* const* cores, int k, double* G_out, void* stream);

/*
 * One core update (Alg. 1 body, eqs. 9-12 or 15-18): gradient, FGMC Gram of the
 * full cores, h = d (G + lambda I)^{-1} with lambda = lambda_rel * tr(G)/R^2,
 * exact line search eta = <d, h> / ||sqrt(W) o P o (h A^T)||^2, and the update
 * Z_k <- Z_k + eta * fold(h) (sign reading: d is the negative gradient, eta the
 * minimiser along +h).  cores[k] is updated in place.  eta_dev (optional device
 * double) receives eta; flags_dev (optional device uint32) is OR-ed with TRD_FLAG_*.
 * TR-ALS as a special case: on a fully observed tensor (P = 1) with sigma = +inf and
 * lambda_rel = 0 the step lands on the least-squares core X_[k] A (A^T A)^{-1} of one ALS
 * update (eta = 1), so trd_fit with TRD_SIGMA_FIXED, sigma = +inf and lambda_rel = 0 runs
 * TR-ALS sweeps.
 */
int trd_step(trd_ctx* ctx, void* const* cores, int k, double sigma, double lambda_rel,
             const trd_sketch* sketch, double* eta_dev, uint32_t* flags_dev, void* stream);

/*
 * Algorithm 1: sweeps k = 0..N-1 (Gauss-Seidel) until max_sweeps or the relative
 * change e = ||D^t - D^{t-1}||_F / ||D^t||_F of D^t = Z_{N(2)} G^{!=N} Z_{N(2)}^T
 * falls below tol (no test after the first sweep).  cores updated in place.
 * With tol > 0 it synchronizes `stream` once per sweep (the stop test reads e); with
 * tol <= 0 (a fixed number of sweeps) it queues the sweeps and synchronizes once per 32
 * sweeps and at the end.  Returns TRD_ENOTSPD if a step hit a non-positive-definite
 * G + lambda I: the run stops after that sweep (sweeps already queued after it change
 * no core), and the report covers the sweeps up to it.
 */
int trd_fit(trd_ctx* ctx, void* const* cores, const trd_fit_opts* opts, trd_fit_report* report,
            void* stream);

/*
 * Differentiation form: L = sum over observed of sigma^2 (1 - exp(-e^2 / 2 sigma^2))
 * (sigma = +inf: sum e^2 / 2), the Welsch loss equal to sum g_sigma(0) - g_sigma(e)
 * for the correntropy objective of eq. (4).  loss_dev: device double.
 */
int trd_loss_fwd(trd_ctx* ctx, const void* const* cores, double sigma, double* loss_dev, void* stream);
/*
 * Its gradient for every core at one point: dL/dZ_k = -fold(d_k) with d_k of eq. (9)
 * and W = w(E) at the same cores (half-quadratic identity); subchain tables are
 * recomputed per core, never stored for all k.  grads_out[k] (device, problem dtype,
 * core layout) receives grad_scale * dL/dZ_k.
 */
int trd_loss_bwd(trd_ctx* ctx, const void* const* cores, double sigma, double grad_scale,
                 void* const* grads_out, void* stream);

/*
 * Draw the RStS index sets of update k in sweep t on the device: for each mode
 * j != k, s_j = min(sizes[j], I_j) distinct indices of [0, I_j), uniform, sorted;
 * mode k gets 0..I_k-1.  Generator: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
 * in counter form, u(key, c) = mix64(key + (c+1) * 0x9E3779B97F4A7C15);
 * key = u(u(u(seed ^ 0x5253545300000000, t), k), j); bounded draws by Lemire's
 * multiply-shift with rejection on the top 32 bits; subsets by Floyd's algorithm.
 * idx_out: host array of N device pointers, idx_out[j] with room for min(sizes[j], I_j)
 * int32 (I_k for j == k).  Needs no context.
 */
int trd_sample_sketch(uint64_t seed, int t, int k, int N, const int64_t* dims, const int32_t* sizes,
                      int32_t* const* idx_out, void* stream);

/*
 * Draw the uniform row sample of update k in sweep t on the device (the row-sampling
 * ablation of Sec. 6.1, used in place of RStS under TRD_SAMPLE_ROWS): J rows of the
 * subchain unfolding Z^{!=k}_{[2]} (Thm. 1), independently and uniformly, with replacement.
 * Sample n takes index bounded(u(key_j, n), 0, I_j) of every mode j != k, where
 * key_j = u(u(u(seed ^ 0x55524F5700000000, t), k), j) and u and bounded are the generator
 * and the bounded draw described at trd_sample_sketch (the draw's own counter starting
 * at 0).  rows_out (device, J int64): the row index, little-endian over the modes
 * k+1, ..., N, 1, ..., k-1, in sample order.  Needs no context.
 */
int trd_sample_rows(uint64_t seed, int t, int k, int N, const int64_t* dims, int64_t J, int64_t* rows_out,
                    void* stream);

/*
 * Draw the leverage-score row sample of update k in sweep t on the device (the ablation of
 * Sec. 6.1 that applies TRALS-S's sampler, used under TRD_SAMPLE_LEVERAGE).  For every mode
 * j != k the leverage of the rows of core j's mode-2 unfolding Z_j(2) (I_j x r_j r_{j+1}) is
 * l(i) = z_i^T (C + lambda I)^{-1} z_i with C = Z_j(2)^T Z_j(2) and the ridge of eq. (10),
 * lambda = lambda_rel tr(C) / (r_j r_{j+1}); sample n takes the uniform
 * u = (u(key_j, n) >> 11) 2^-53 with key_j = u(u(u(seed ^ 0x4C45564500000000, t), k), j) (u as
 * at trd_sample_sketch) and the first slice i whose running sum l(0) + ... + l(i) in FP64
 * exceeds u times the total (a core whose leverages are all zero: the slice floor(u I_j)).
 * Its row has probability p = prod_j l(i_j) / total_j (1 / I_j for such a core).
 * rows_out (device, J int64): row indices as at trd_sample_rows; weights_out (device, J FP64):
 * the importance weights 1 / (J p).  ctx needs a shape; cores: N device pointers.
 */
int trd_sample_leverage(trd_ctx* ctx, const void* const* cores, int k, uint64_t seed, int t, int64_t J,
                        double lambda_rel, int64_t* rows_out, double* weights_out, void* stream);

/*
 * Seeded synthetic observation pattern on the device, bit-exact for a given seed:
 * mask_out[l] = 1 for an observed entry (column-major l), drawn with probability rho per
 * entry (block == 0) or per tile (block > 0: block x block tiles of modes 0 and 1, one draw
 * per tile and per index of modes 3.., shared by every index of mode 2: the missing-block
 * pattern of a video with mode 2 as the colour channel); outlier_out[l] (optional) = 1 for
 * an observed entry chosen with probability outlier_frac; u_out[l] (optional) = a uniform
 * double in [0, 1) per entry (53 bits), for an outlier's value or sign.  These are the
 * observation model of eq. (2) with gross outliers (Sec. 3-4); the paper does not fix a law.
 * Generator: the SplitMix64 counter form of trd_sample_sketch with keys
 * u(seed ^ 0x4D41534B00000000, 0 / 1 / 2) for mask / selection / uniform; an event of
 * probability p happens when the draw u(key, c) < floor(p * 2^64) (p >= 1: always, p <= 0:
 * never), with c = l, or the tile index i0/block + nbh*(i1/block + nbw*f) for the mask
 * (nbh, nbw tiles along modes 0 and 1, f the linear index of modes 3..); u = (draw >> 11) * 2^-53.
 * Device buffers of prod(dims) elements.  Needs no context.
 */
int trd_sample_mask(uint64_t seed, int N, const int64_t* dims, double rho, int block,
                    double outlier_frac, uint8_t* mask_out, uint8_t* outlier_out, double* u_out,
                    void* stream);

/*
 * Precision of the entry-wise passes of later trd_grad / trd_step / trd_loss_* calls
 * (trd_fit uses its own opts.precision).  TRD_PREC_BF16 (FP32 problems only): the
 * subchain tables are rounded to bf16 and the reconstruction and gradient contractions
 * run on the matrix cores (BF16 operands, FP32 accumulation); residuals, weights and the
 * FGMC Gram / scaled step stay in FP32 / FP64.  TRD_PREC_BF16X3 also keeps the bf16
 * remainder of every reconstruction-table element and adds the two cross products, so the
 * residual is accurate to about 2^-16 relative instead of 2^-8 (the gradient contraction
 * stays a single bf16 product).  RStS sketches always use the native passes.
 * The first BF16 use of a core builds its bitmask-tile layout (synchronizes the stream).
 */
int trd_set_precision(trd_ctx* ctx, int precision);

/*
 * Variants of the update for the ablations of Sec. 6.1, for later trd_step / trd_fit
 * calls on ctx (default: TRD_DIR_SCALED, TRD_GRAM_GLOBAL, the method itself).
 *   direction TRD_DIR_GRADIENT: step along d of eq. (9) / (15) instead of the scaled
 *     direction h of eq. (10) / (16); eta stays the exact line search of eq. (12) / (18)
 *     with h = d, and no Gram matrix is formed.
 *   gram TRD_GRAM_LOCAL: under an RStS sketch, scale with the Gram matrix of the sampled
 *     cores (the factors of eq. 13 summed over the sampled slices I_j only, which is
 *     A_I^T A_I of the sketched subchain unfolding) instead of the global one; without a
 *     sketch the two coincide.  Ignored with TRD_DIR_GRADIENT.
 *   sampling TRD_SAMPLE_ROWS: a sketch (trd_step / trd_grad / trd_fit with sizes) takes
 *     J = prod_{j != k} min(sizes[j], I_j) rows of Z^{!=k}_{[2]} drawn uniformly with
 *     replacement (trd_sample_rows, same seed and sweep) instead of the RStS index sets:
 *     the gradient, line search and kernel-width residuals use the mode-k fibres of the
 *     tensor at those rows (a row drawn twice counts twice), the Gram matrix stays global.
 *     Caller index lists (trd_sketch.idx) are rejected; with TRD_GRAM_LOCAL and the scaled
 *     direction it is TRD_EUNSUPPORTED.
 *   sampling TRD_SAMPLE_LEVERAGE: as TRD_SAMPLE_ROWS, with the J rows drawn by TRALS-S's
 *     leverage-score sampler from the cores as they stand (trd_sample_leverage, same seed,
 *     sweep and ridge: the step's lambda_rel, 1e-9 in trd_grad); each sampled entry counts
 *     with its row's importance weight 1 / (J p) in the gradient, the line search and the
 *     reported loss; the kernel-width residuals stay unweighted.
 * Returns TRD_EINVAL for other values (the context keeps its previous variant).
 */
#define TRD_DIR_SCALED   0
#define TRD_DIR_GRADIENT 1
#define TRD_GRAM_GLOBAL  0
#define TRD_GRAM_LOCAL   1
#define TRD_SAMPLE_RSTS  0
#define TRD_SAMPLE_ROWS  1
#define TRD_SAMPLE_LEVERAGE 2
int trd_set_variant(trd_ctx* ctx, int direction, int gram, int sampling);

/*
 * Per-launch timing of the fused reconstruct+weight+gradient pass, for measurement:
 * enable != 0 times every launch of that kernel on its stream with a pair of HIP events
 * (the matrix-core passes hand them to the launch, which sets them at the kernel's own
 * start and end; the sliced-ELL passes record them just before and after the launch);
 * trd_profile_read returns the number of launches and their summed duration (ms) and
 * summed entry slots since the last read, then resets the counters (synchronizes).
 */
int trd_profile(trd_ctx* ctx, int enable);
int trd_profile_read(trd_ctx* ctx, int64_t* launches, double* total_ms, int64_t* slots,
                     int64_t* entries);

#ifdef __cplusplus
}
#endif

#endif /* TRD_H */

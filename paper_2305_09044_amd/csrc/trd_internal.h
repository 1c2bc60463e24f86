// Internal declarations shared by the host orchestration and the kernel files.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace trd {

constexpr int kMaxN = 8;
constexpr int kMaxRank = 16;
constexpr int kMaxRR = 128;        // r_k * r_s of the fused pass
constexpr int kRowsPerWG = 256;    // rows of one work-group tile (4 waves x 64 lanes)
constexpr int kWave = 64;
constexpr uint16_t kPad = 0xFFFF;  // padding marker in the sliced-ELL column array
constexpr int kPassThreads = 256;
// Entries of a slice are stored in groups of kGroup per lane: entry t of lane l sits at
// slice_base + (t / kGroup) * (64 * kGroup) + l * kGroup + t % kGroup, so that one lane
// reads its next kGroup values and columns with wide loads.  Slice lengths are
// multiples of kGroup.
constexpr int kGroup = 8;
__host__ __device__ inline int64_t slot_of(int64_t base, int t, int lane) {
  return base + (int64_t)(t / kGroup) * (kWave * kGroup) + lane * kGroup + (t % kGroup);
}
constexpr uint32_t TRD_FLAG_EMPTY_BIT = 1u;     // mirrors TRD_FLAG_EMPTY
constexpr uint32_t TRD_FLAG_ZERO_DEN_BIT = 2u;  // mirrors TRD_FLAG_ZERO_DEN
constexpr uint32_t TRD_FLAG_NOTSPD_BIT = 4u;    // mirrors TRD_FLAG_NOTSPD
constexpr uint32_t TRD_FLAG_CLAMPED_BIT = 8u;   // mirrors TRD_FLAG_CLAMPED

// Optional start / stop events of a timed kernel launch.  They are handed to the launch
// itself (hipExtLaunchKernel), which sets them at the kernel's start and end without
// separate marker packets on the stream.
struct KTiming {
  hipEvent_t start = nullptr, stop = nullptr;
};
// KERN: a kernel name (parenthesised when it has template arguments)
#define TRD_LAUNCH(KERN, G, B, LDS, ST, TM, ...)                                          \
  do {                                                                                    \
    if ((TM).start || (TM).stop)                                                          \
      hipExtLaunchKernelGGL(KERN, G, B, (uint32_t)(LDS), ST, (TM).start, (TM).stop, 0u,   \
                            __VA_ARGS__);                                                 \
    else                                                                                  \
      hipLaunchKernelGGL(KERN, G, B, LDS, ST, __VA_ARGS__);                               \
  } while (0)

// largest dynamic LDS a work-group may request, and the compute-unit count (both set from
// the device at context creation)
extern int64_t g_lds_max;
extern int g_num_cu;
// work-groups a pass launch aims for: enough resident groups per CU to balance the tail
inline int64_t wg_target() { return (int64_t)g_num_cu * 8; }
// column groups for a row-group count and tile count: as few as give wg_target() groups
inline void column_groups(int64_t n_rg, int n_ct, int& n_cg, int& cpg,
                          int64_t target = wg_target()) {
  int64_t want = (target + n_rg - 1) / (n_rg > 0 ? n_rg : 1);
  if (want < 1) want = 1;
  if (want > n_ct) want = n_ct;
  cpg = (int)((n_ct + want - 1) / want);
  if (cpg < 1) cpg = 1;
  n_cg = (n_ct + cpg - 1) / cpg;
}

// Division of 32-bit unsigned numerators by a fixed divisor d >= 1 through a multiply-high
// (Granlund and Montgomery, 1994): s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1,
// n / d = (mulhi(n, m) + n) >> s, exact for every 32-bit n.
struct FastDiv {
  uint32_t d = 1, m = 1;
  int s = 0;
  FastDiv() = default;
  explicit FastDiv(uint32_t div) : d(div) {
    s = 0;
    while ((1ull << s) < d) ++s;
    m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  }
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return (uint32_t)(((uint64_t)__umulhi(n, m) + n) >> s);
  }
};

// A table of small column-major matrices ("items"), item t at ptr + idx(t) * stride.
struct ItemRef {
  const void* ptr = nullptr;
  int64_t stride = 0;              // elements between items
  const int32_t* list = nullptr;   // optional device index list (item t -> list[t])
};

// Mode description for index decoding of rows / columns of a core-k matrix.
struct ModeSet {
  int n = 0;
  int mode[kMaxN];
  int64_t count[kMaxN];            // number of indices of this mode in the set
  int64_t stride[kMaxN];           // stride of the mode in the column-major tensor
  const int32_t* list[kMaxN];      // index list (nullptr = identity)
};

// The observed entries of one core update, grouped as a matrix (rows x cols) and
// stored as 64-row sliced ELL inside 256-row x ct_w-column tiles.
struct Layout {
  int k = -1;
  int64_t nrows = 0, ncols = 0;
  int ct_w = 0, n_ct = 0;          // column tile width and count
  int n_cg = 0, cpg = 0;           // column groups walked by one work-group, tiles per group
  int64_t n_rg = 0;                // 256-row groups
  int64_t n_slices = 0;            // n_ct * n_rg * 4
  int64_t slots = 0;               // host copy of the total slot count (full path)
  int64_t slots_cap = 0;           // capacity of vals/cols
  int64_t* rowoff = nullptr;       // [nrows] tensor offset of each row
  int64_t* coloff = nullptr;       // [ncols] tensor offset of each column
  int32_t* counts = nullptr;       // [n_ct][n_rg*256]
  int32_t* slice_len = nullptr;    // [n_slices]
  int64_t* slice_off = nullptr;    // [n_slices + 1]
  void* vals = nullptr;            // [slots] problem dtype
  uint16_t* cols = nullptr;        // [slots]
  int64_t* total_dev = nullptr;    // device copy of slots
  int64_t* nobs_dev = nullptr;     // device observed count in this layout
  int64_t nobs = 0;                // host copy (full path)
};

// Split of the cyclic subchain for core k: rows = (k, B modes), cols = C modes.
struct Split {
  int k = 0, p = 0, q = 0;
  int B[kMaxN], C[kMaxN];
  int r_k = 0, r_k1 = 0, r_s = 0;  // r_s = rank between the B and C groups
  int RR = 0, RRP = 0;             // r_k * r_s and its padded width
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `st` and return a hipError_t from the launch.

// layout building
hipError_t launch_offsets(const ModeSet& ms, int64_t n, int64_t* out, hipStream_t st);
hipError_t launch_count(const Layout& L, const uint8_t* mask, hipStream_t st);
hipError_t launch_slices(const Layout& L, hipStream_t st);
hipError_t launch_scan(const Layout& L, hipStream_t st);
hipError_t launch_fill(const Layout& L, const uint8_t* mask, const void* X, int dtype,
                       hipStream_t st);
hipError_t launch_sample(uint64_t seed, int t, int k, int N, const int64_t* dims,
                         const int32_t* sizes, int32_t* const* out, hipStream_t st);
// uniform row sample of core k (J rows of the subchain unfolding, with replacement):
// column-major tensor offsets of the sampled fibres (i_k = 0) and/or row indices (either
// may be nullptr)
hipError_t launch_sample_rows(uint64_t seed, int t, int k, int N, const int64_t* dims, int64_t J,
                              int64_t* off, int64_t* row, hipStream_t st);
// leverage distribution of one core (mode-2 unfolding, I slices of R = r r' values): C and
// its ridge inverse (R x R FP64 scratch), leverage and running sums (I FP64 each)
hipError_t launch_leverage_mode(int dtype, const void* Z, int64_t I, int R, double* C, double* Ci,
                                double lambda_rel, double* lev, double* cdf, uint32_t* flags,
                                hipStream_t st);
// J leverage-sampled rows of the subchain unfolding of core k (lev/cdf of every mode j != k):
// tensor offsets and/or row indices (either may be nullptr) and importance weights 1 / (J p)
hipError_t launch_sample_leverage(uint64_t seed, int t, int k, int N, const int64_t* dims,
                                  const double* const* lev, const double* const* cdf, int64_t J,
                                  int64_t* off, int64_t* row, double* weight, hipStream_t st);
// mask (Bernoulli rho per entry, or per block x block tile of modes 0-1 at each index of
// modes 3.., shared by mode 2), outlier selection (observed and Bernoulli frac) and per-entry
// uniforms; sel and u may be nullptr
hipError_t launch_sample_mask(uint64_t seed, int N, const int64_t* dims, double rho, int block,
                              double frac, uint8_t* mask, uint8_t* sel, double* u, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
hipError_t launch_copy_clamp(const int32_t* in, int64_t n, int64_t dim, int32_t* out,
                             uint32_t* bad, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);
hipError_t launch_accum_i64(int64_t* dst, const int64_t* src, hipStream_t st);

// tables (Def. 2 merges)
// bf16_out: the table is written as bf16 bits (FP32 problems only), for the matrix-core
// passes; out_lo (with bf16_out) also receives the bf16 of each element's remainder
hipError_t launch_merge(int dtype, ItemRef L, int64_t nL, int rA, int rB, ItemRef R, int64_t nR,
                        int rC, void* out, int64_t out_stride, int transpose_out, hipStream_t st,
                        bool bf16_out = false, void* out_lo = nullptr);
// column table of sampled fibres: for each column n (tensor offset off[n], i_k = 0) the
// product Z_{k+1}(i_{k+1}) ... Z_{k-1}(i_{k-1}) (r_{k+1} x r_k), stored transposed
// (element (a, c) at a * r_k + c) and zero-padded to out_stride
hipError_t launch_chain_cols(int dtype, const void* const* cores, int N, int k, const int32_t* ranks,
                             const int64_t* dims, const int64_t* strides, const int64_t* off,
                             int64_t J, void* out, int64_t out_stride, hipStream_t st);
// out (column-major nrows x ncols, the whole tensor) = T V^T of the two subchain tables of
// core 0 (rows of RRP values each)
hipError_t launch_table_product(int dtype, const void* T, const void* V, int64_t nrows, int64_t ncols,
                                int RRP, void* out, hipStream_t st);
hipError_t launch_pack(int dtype, ItemRef in, int64_t n, int rA, int rB, void* out,
                       int64_t out_stride, int transpose_out, hipStream_t st,
                       bool bf16_out = false, void* out_lo = nullptr);
// in-place fixed-order sum of n_ct partial arrays of n elements into the first
hipError_t launch_sum_partials(int dtype, void* S, int n_ct, int64_t n, hipStream_t st);
hipError_t launch_contract(int dtype, const void* S, int RRP, int n_ct, int64_t pstride,
                           int64_t Ik, int64_t nB, int r_k, int r_s, int r_k1, ItemRef U,
                           double* part, int nchunk, hipStream_t st);
hipError_t launch_contract_finish(int dtype, const double* part, int nchunk, int64_t Ik, int RRk,
                                  double* d64, void* d_out, double scale, hipStream_t st);

// fused entry pass
enum PassMode { kModeGrad = 0, kModeLS = 1, kModeResid = 2, kModeLoss = 3, kModeGradFast = 4,
                // matrix-core passes only: GradFast reading the residuals the residual pass
                // stored for the same cores and layout (through `vals`) instead of forming xhat
                kModeGradE = 5 };
struct PassArgs {
  const void* T;        // [nrows][RRP]
  const void* TH;       // [nrows][RRP] (line search)
  const void* V;        // [ncols][RRP]
  void* S;              // [n_cg][nrows][RRP] per-column-group gradient partials
  const void* vals;
  const uint16_t* cols;
  const int64_t* slice_off;
  const int32_t* slice_len;
  float* resid;         // kModeResid output, one per slot
  const double* colw;   // per-column weights (leverage-sampled rows) or nullptr
  double* partials;     // [n_wg][3]
  const double* sigma;  // device scalar
  int64_t nrows, ncols, n_rg;
  int ct_w, RR, RRP, n_ct;
  int n_cg, cpg;        // column groups (one work-group each per row group), tiles per group
};
hipError_t launch_pass(int dtype, int prec, int mode, const PassArgs& a, hipStream_t st);
bool pass_supported(int RR);
int pass_rc(int RR);
int pass_rrp(int RR);
int64_t pass_ct_w(int dtype, int prec, int RRP);

// dense FP64 pieces
// K = sum over slices i of Z(i) (x) Z(i); idx: the I slices to sum (nullptr: all I)
hipError_t launch_kron_factor(int dtype, const void* Z, int r0, int64_t I, int r1, double* K,
                              hipStream_t st, const int32_t* idx = nullptr);
hipError_t launch_gemm64(const double* A, const double* B, double* C, int m, int kk, int n,
                         hipStream_t st, int r_k = 0, int r_k1 = 0);
hipError_t launch_finish_step(int dtype, const double* pnum, int64_t n_num, const double* pden,
                              int64_t n_den, const int64_t* nobs, uint32_t* flags,
                              uint32_t* flags_user, double* eta, double* eta_user, void* Z,
                              const double* h, int64_t nz, const uint32_t* halt, hipStream_t st);
hipError_t launch_realign(const double* P, double* G, int r_k, int r_k1, hipStream_t st);
// ring product of eq. 13 in one work-group (factor sides <= 64), realigned into G
struct RingArgs {
  const double* K[kMaxN];
  int rows[kMaxN], cols[kMaxN];  // factor f is rows[f] x cols[f]; cols[f] == rows[f + 1]
  int nf;
  int r_k, r_k1;
  double* G;
};
hipError_t launch_ring(const RingArgs& a, hipStream_t st);
// G^{!=k} (eq. 13) from the factors K[j], j != k (r_j^2 x r_{j+1}^2 FP64, row-major); P0 and P1
// hold r_{k+1}^2 * max_m r_m^2 doubles each (read only when a factor side exceeds 64)
hipError_t launch_ring_gram(int N, const int32_t* ranks, int k, const double* const* K, double* P0,
                            double* P1, double* G, int64_t lds_max, hipStream_t st);
// message of the last failure of a context-free call (trd_last_error(NULL)); returns code
int fail_free(int code, const std::string& msg);
// (G + lambda_rel tr(G)/n I)^-1; not SPD: zero and the NOTSPD bit ORed into *flags, or
// with assign the whole word set to that bit or 0 (the step's first writer of its flags)
hipError_t launch_inverse(const double* G, double* Cinv, int n, double lambda_rel,
                          uint32_t* flags, hipStream_t st, bool assign = false);
// Cinv == nullptr: h = d
hipError_t launch_apply_inverse(const double* d64, const double* Cinv, int64_t Ik, int n,
                                double* h64, void* h_real, int dtype, double* part_num,
                                const uint32_t* flags, hipStream_t st);
hipError_t launch_eta(const double* num, const double* den, const int64_t* nobs, double* eta,
                      uint32_t* flags, uint32_t* flags_user, double* eta_user, hipStream_t st);
hipError_t launch_update(int dtype, void* Z, const double* h64, const double* eta, int64_t n,
                         hipStream_t st);
hipError_t launch_reduce_partials(const double* part, int64_t n, int width, double* out,
                                  hipStream_t st);
hipError_t launch_set_scalar(double* p, double v, hipStream_t st);
hipError_t launch_pack_report(const double* sigma, const double* conv, const uint32_t* flags,
                              const double* eta, int N, double* out, uint32_t* halt,
                              hipStream_t st);
hipError_t launch_convergence(int dtype, const void* ZN, const double* G, int64_t IN, int n,
                              double* M, double* D, const double* Dprev, int have_prev,
                              double* part, hipStream_t st);
hipError_t launch_weights(int dtype, const void* r, int64_t n, double sigma, void* w,
                          hipStream_t st);
hipError_t launch_reconstruct(int dtype, int N, const int64_t* dims, const int32_t* ranks,
                              const void* const* cores, const int64_t* lin, int64_t n, void* out,
                              hipStream_t st);
hipError_t launch_max_abs_observed(const Layout& L, int dtype, double* out, hipStream_t st);

// ---------------------------------------------------------------- matrix-core (BF16) form
// Block tiles of one core-k matrix: 64-row x 32-column blocks, block b = rb * n_chunks + ch,
// each holding its observed values and in-block positions 32 r + c in increasing order.
struct TLayout {
  int64_t nrows = 0, ncols = 0;
  int K = 0;                       // padded contraction width (multiple of 32)
  int CW = 0, n_chpt = 0;          // column tile width (multiple of 32), chunks per tile
  int n_ct = 0, n_cg = 0, cpg = 0; // column tiles, column groups, tiles per group
  int64_t n_chunks = 0;            // 32-column chunks
  int64_t n_rb = 0, n_rg = 0;      // 64-row blocks, 256-row groups
  int64_t n_blocks = 0;            // n_rb * n_chunks
  // B-major rows (bmaj): tile row b + nB i_k holds the layout row i_k + I_k b, so that a
  // 64-row block spans at most two slices i_k and the gradient pass contracts its own row
  // factors (TPassArgs::dpart); otherwise tile rows are the layout rows
  int64_t nB = 1, Ik = 0;
  bool bmaj = false;
  const int64_t* rowoff = nullptr; // shared with the ELL layout of the same split
  const int64_t* coloff = nullptr;
  int32_t* bcnt = nullptr;         // [n_blocks]
  int64_t* boff = nullptr;         // [n_blocks + 1]
  int64_t* total_dev = nullptr;
  float* vals = nullptr;           // [nobs + slack]
  uint16_t* pos = nullptr;         // [nobs + slack]
  int64_t nobs = 0;
  bool ready = false;
};

struct TPassArgs {
  const uint16_t* T;     // [nrows][K] bf16
  const uint16_t* TH;    // [nrows][K] bf16 (line search)
  // column table in operand-fragment order, one 32-column chunk after another (zero past
  // the last column, one chunk of padding at the end): Vf for the reconstruction
  // products, VTf (the transpose) for the gradient products, Vf_lo the split remainder
  const uint16_t* Vf;
  const uint16_t* VTf;
  const uint16_t* T_lo;  // split tables (remainders), or nullptr
  const uint16_t* Vf_lo;
  float* S;              // [n_cg][nrows][RRP] per-column-group partials (layout row order)
  // B-major rows (gradient modes, K = 64, r_k = r_s = r_{k+1} = 8): instead of S, each
  // wave writes dpart[cg][rb][s][a + 8 beta] = sum over its rows of slice i0 + s (i0 the
  // slice of the block's first row) of sum_c S(row)[a + 8c] U(b)[beta + 8c]
  float* dpart;
  const float* U;        // U(m_B) items (r_k1 x r_s, index beta + r_k1 c), Us apart
  int64_t Us;
  int64_t nB, Ik;        // B items per slice and slices (B-major rows)
  int bmaj;
  const int64_t* boff;
  const float* vals;
  const uint16_t* pos;
  uint16_t* wout;        // gradient modes: weight per observed entry (fp16), in value order,
                         // with one slot per lane past nobs (or nullptr)
  const uint16_t* win;   // line search: those weights
  int64_t nobs;
  float* resid;          // kModeResid: e per observed entry, in value order
  uint32_t* qhist;       // kModeResid: first-digit histogram of the |e| keys (or nullptr)
  double* partials;      // [n_wg][3]
  const double* sigma;
  int64_t nrows, ncols, n_chunks, n_rb, n_rg;
  int CW, n_chpt, cpg, n_cg, RR, RRP;
  int rounds;            // entry rounds wanted in registers (K = 64: 8 for dense blocks)
};

// entries of slack after the value / position arrays of a tile layout
constexpr int64_t kTileSlack = 64 * 16 + 64;
int tile_k(int RR);
int64_t tile_cw(int K);
size_t tpass_lds(int mode, int K, int CW);
// elements of a fragment-order column table: whole chunks of 32 columns plus one chunk
// that the passes read ahead
inline int64_t tile_frag_elems(int64_t ncols, int K) { return ((ncols + 31) / 32 + 1) * 32 * K; }
// V [ncols][K] bf16 -> Vf (and VTf unless nullptr) in fragment order, padding included
hipError_t launch_fragments(const uint16_t* V, int64_t ncols, int K, uint16_t* Vf, uint16_t* VTf,
                            hipStream_t st);
hipError_t launch_tile_build(const TLayout& L, const uint8_t* mask, const void* X, int dtype,
                             bool fill, hipStream_t st);
hipError_t launch_tpass(int mode, int K, const TPassArgs& a, hipStream_t st, KTiming tm = {});
// d(i_k)[o] = scale * (fixed-order sum of the B-major epilogue partials of slice i_k)
hipError_t launch_dpart_finish(const float* part, int n_cg, int64_t n_rb, int64_t nB, int64_t Ik,
                               double* d64, float* d_out, double scale, hipStream_t st);
// the same sums followed by the scaled direction of the slice (rank 8: 64 x 64 inverse),
// h in FP64 and FP32 and the slice's share of <d, h> in pdh[i_k]
hipError_t launch_dpart_direction(const float* part, int n_cg, int64_t n_rb, int64_t nB, int64_t Ik,
                                  const double* Cinv, const uint32_t* flags, double* d64,
                                  double* h64, float* h_real, double* pdh, hipStream_t st);

// sigma quantile by radix select over float bit patterns
// radix select of the kernel-width quantile over the |e| keys: three digits (11, 11, 10
// bits).  With first_digit_done the first digit's histogram is already in hist (written
// by the residual pass after launch_quantile_init); otherwise the selection initialises
// the state and counts every digit itself.
hipError_t launch_quantile_init(const int64_t* nobs, double q, uint32_t* state, uint32_t* hist,
                                hipStream_t st);
// cand (quantile_grid(n_slots_hint) * quantile_seg_cap(n_slots_hint) keys) and cand_cnt
// (quantile_grid(n_slots_hint) counts), or nullptr: the keys sharing the first digit,
// gathered by the second digit's pass for the third
int quantile_grid(int64_t n_slots_hint);
int64_t quantile_seg_cap(int64_t n_slots_hint);
hipError_t launch_quantile_sigma(const float* keys, int64_t n_slots_hint, const int64_t* nslots,
                                 double q, double c, const double* sigma_min, double shrink,
                                 double* sigma, uint32_t* hist, uint32_t* state,
                                 const int64_t* nobs, float* cand, uint32_t* cand_cnt,
                                 bool first_digit_done, hipStream_t st);

}  // namespace trd

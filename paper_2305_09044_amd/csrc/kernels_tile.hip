// Matrix-core (MFMA) form of the fused entry passes: the BF16 precision form.
//
// The observed entries of a core-k matrix (rows = (i_k, first subchain modes), cols =
// the rest) are grouped in blocks of 64 rows x 32 columns.  A block stores its observed
// values and their in-block positions in increasing (r, c) order (r < 64, c < 32), each
// as the index 36 r + c of the entry in the per-wave LDS tiles (row stride 36).
// One wave owns a 64-row block row and walks its blocks (32-column chunks):
//   1. Xhat^T (32 cols x 64 rows) = V^T-items (32 x K) . T-items^T (K x 64) on the
//      matrix cores (Thm. 1): bf16 operands, FP32 accumulation, spilled to LDS;
//   2. each observed entry of the block (lane-parallel, in value order) reads its xhat,
//      forms e = x - xhat, w = exp(-e^2/2s^2) (eq. 7) and y = w e in FP32, and scatters
//      y (rounded to bf16) into a cleared 64 x 32 tile in LDS;
//   3. S^T (K x 64 rows) += V^T-items^T (K x 32 cols) . Y^T (32 cols x 64 rows) on the
//      matrix cores: the row factor of the gradient of eq. 9;
//   4. at the end of the walk, the row factors go out as they are, or, on B-major block
//      rows (TR ranks 8, rows ordered with the B-mode index fastest so that a block holds
//      one or two slices i_k), contracted with U(m_B) into 64-float partials of d.
// Matrix-core work covers every position of a block; vector work is per observed entry.
// Split form (SPLIT): the T and V tables also come as bf16 remainders (t = t_hi + t_lo),
// and Xhat adds the products t_hi v_lo and t_lo v_hi, so the reconstruction (and the
// residual) carries about 16 significant bits instead of 8; the gradient contraction
// stays a single bf16 product.
// A work-group (4 waves = 4 block rows) walks a group of column tiles; each wave keeps its
// S accumulators in registers and works on its own LDS tiles (no work-group barrier in
// the walk).  The column table is read in operand-fragment order (k_fragments): every
// operand load of a wave is one contiguous kilobyte, for the reconstruction (V^T items)
// and for the gradient products (V items, the transposed order).
#include "trd_internal.h"

namespace trd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// row stride (elements) of the per-wave LDS tiles, and so of the stored positions
constexpr int kTS = 36;
typedef float floatx16 __attribute__((ext_vector_type(16)));

// IEEE half bits of x (round to nearest even)
__device__ __forceinline__ uint16_t f16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (_Float16)x);
}

// order LDS accesses among the lanes of one wave (the tiles below are per wave)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- layout builder

struct TileArgs {
  const int64_t* rowoff;
  const int64_t* coloff;
  int32_t* bcnt;
  const int64_t* boff;
  float* vals;
  uint16_t* pos;
  int64_t nrows, ncols, n_chunks, n_blocks;
  int64_t nB, Ik;  // B-major rows (bmaj): tile row b + nB i_k is layout row i_k + Ik b
  int bmaj;
};

// layout row (the row tables' and the row offsets' order) of a tile row
__device__ __forceinline__ int64_t layout_row(int64_t t, int bmaj, int64_t nB, int64_t Ik) {
  if (!bmaj) return t;
  const int64_t ik = t / nB;
  return ik + Ik * (t - ik * nB);
}

static TileArgs targs(const TLayout& L) {
  TileArgs a;
  a.rowoff = L.rowoff; a.coloff = L.coloff; a.bcnt = L.bcnt; a.boff = L.boff;
  a.vals = L.vals; a.pos = L.pos;
  a.nrows = L.nrows; a.ncols = L.ncols; a.n_chunks = L.n_chunks; a.n_blocks = L.n_blocks;
  a.nB = L.nB; a.Ik = L.Ik; a.bmaj = L.bmaj ? 1 : 0;
  return a;
}

// Block b = rb * n_chunks + ch, one wave per block.  Round t covers p = 64 t + lane
// (row 2 t + lane / 32, column lane % 32), so the ballot of a round lists its observed
// entries in increasing (r, c).  Count pass (FILL = false): per-block counts;
// fill pass: values and positions at boff[b] onwards.
template <typename real, bool FILL>
__global__ __launch_bounds__(256) void k_tblock(TileArgs a, const uint8_t* __restrict__ mask,
                                                const real* __restrict__ X) {
  const int64_t b = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  if (b >= a.n_blocks) return;  // b is uniform over the wave
  const int64_t rb = b / a.n_chunks, ch = b % a.n_chunks;
  const int64_t col = ch * 32 + (l & 31);
  const bool col_ok = col < a.ncols;
  const int64_t co = col_ok ? a.coloff[col] : 0;
  int64_t out = FILL ? a.boff[b] : 0;
  int cnt = 0;
  for (int t = 0; t < 32; ++t) {
    const int p = 64 * t + l;
    const int64_t row = rb * 64 + (p >> 5);
    bool obs = false;
    int64_t off = 0;
    if (col_ok && row < a.nrows) {
      off = a.rowoff[layout_row(row, a.bmaj, a.nB, a.Ik)] + co;
      obs = mask[off] != 0;
    }
    const uint64_t bal = __ballot(obs);
    if constexpr (FILL) {
      if (obs) {
        const int pre = __popcll(bal & ((1ull << l) - 1ull));
        a.vals[out + pre] = (float)X[off];
        a.pos[out + pre] = (uint16_t)((p >> 5) * kTS + (p & 31));
      }
      out += __popcll(bal);
    } else {
      cnt += __popcll(bal);
    }
  }
  if (!FILL && l == 0) a.bcnt[b] = cnt;
}

// exclusive scan of int32 counts into int64 offsets (one work-group, fixed order)
__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ out, int64_t* total) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < n ? (int64_t)in[i] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t add = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < n) out[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[n] = carry;
    *total = carry;
  }
}

hipError_t launch_tile_build(const TLayout& L, const uint8_t* mask, const void* X, int dtype,
                             bool fill, hipStream_t st) {
  const unsigned nb = (unsigned)((L.n_blocks + 3) / 4);
  if (!fill) {
    hipLaunchKernelGGL((k_tblock<float, false>), dim3(nb), dim3(256), 0, st, targs(L), mask,
                       (const float*)nullptr);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, L.bcnt, L.n_blocks, L.boff,
                       L.total_dev);
  } else if (dtype == 0) {
    hipLaunchKernelGGL((k_tblock<float, true>), dim3(nb), dim3(256), 0, st, targs(L), mask,
                       (const float*)X);
  } else {
    hipLaunchKernelGGL((k_tblock<double, true>), dim3(nb), dim3(256), 0, st, targs(L), mask,
                       (const double*)X);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- the MFMA pass

// Per-wave LDS tiles, both with row stride kTS, so that one stored position indexes
// either.  The f32 rows (144 bytes, an odd multiple of 16) put the 16-byte spill stores of
// eight consecutive rows in distinct banks; the bf16 rows (72 bytes) are read as 8-byte
// halves, 32 rows to 32 distinct bank pairs.
constexpr int kXS = kTS;                // f32 stride of the xhat (and q) tile
constexpr int kYS = kTS;                // bf16 stride of the y tile
constexpr int kXTile = 64 * kXS;        // floats
constexpr int kYTile = 64 * kYS;        // bf16
constexpr int kXBytes = 4 * kXTile * 4; // four waves
constexpr int kYBytes = 4 * kYTile * 2;
// residual pass: work-group histogram of the first quantile digit (key >> 21, 11 bits)
constexpr int kQHistBins = 2048;
constexpr int kQHistBytes = kQHistBins * 4;

// entry rounds of 64 held in registers per chunk: 12 for K = 32; for K = 64 (plain form) 4
// or 8, chosen per layout by its mean entries per block (TPassArgs::rounds); 4 otherwise.
// A block with more entries than the rounds hold takes the remaining rounds from memory.
template <int K, bool SPLIT, bool WIDE> struct TileRounds {
  static constexpr int v = K <= 32 ? 12 : (K <= 64 && !SPLIT && WIDE ? 8 : 4);
};

size_t tpass_lds(int mode, int K, int CW) {
  (void)CW;
  if (mode == kModeGrad || mode == kModeGradFast) return (size_t)kXBytes + kYBytes;
  // the y tiles, then (K = 64, the B-major contraction) the tiles of the row-factor
  // reduction at the end of the walk (its own: the waves of a work-group finish their walks
  // at different times)
  if (mode == kModeGradE) return (size_t)kYBytes + (K == 64 ? kXBytes : 0);
  if (mode == kModeLS) return (size_t)kXBytes;  // the q tile only
  if (mode == kModeResid) return (size_t)kXBytes + kQHistBytes;
  return (size_t)kXBytes;
}

template <int K, int MODE, bool SPLIT, bool WIDE>
__global__ __launch_bounds__(256, (K >= 96 ? 1 : 2)) void k_tpass(
    TPassArgs a) {
  constexpr int KS = K / 16;       // k-steps of the reconstruction MFMA
  constexpr int MT = K / 32;       // m-tiles of the gradient MFMA
  constexpr int kR = TileRounds<K, SPLIT, WIDE>::v;  // entry rounds of 64 in registers per chunk
  constexpr bool kGradE = MODE == kModeGradE;
  constexpr bool kGrad = MODE == kModeGrad || MODE == kModeGradFast || kGradE;
  constexpr bool kLS = MODE == kModeLS;
  // the line search reads the weights the gradient pass stored (same cores, sigma and
  // layout, so the same values) and needs only the products q, not xhat
  // so does the gradient pass that reads the residuals of the residual pass (kGradE)
  constexpr bool kRecon = !kLS && !kGradE;
  constexpr bool kStats = MODE == kModeGrad || MODE == kModeLoss;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the wave index is uniform over the wave: keep it (and everything derived from it:
  // block row, block offsets, loop bounds) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63, h = l >> 5, li = l & 31;
  // (the pass that reads stored residuals keeps this tile after its y tiles, for the
  // reduction at the end of the walk)
  float* Xs = reinterpret_cast<float*>(smem_raw + (kGradE ? kYBytes : 0)) + w * kXTile;
  float* Qs = Xs;  // LS: the q tile in place of the xhat tile
  uint16_t* Ys = reinterpret_cast<uint16_t*>(smem_raw + (kRecon ? kXBytes : 0)) + w * kYTile;  // grad
  uint32_t* qh = reinterpret_cast<uint32_t*>(smem_raw + kXBytes);                     // resid
  if constexpr (MODE == kModeResid) {
    if (a.qhist) {
      for (int i = threadIdx.x; i < kQHistBins; i += 256) qh[i] = 0u;
      __syncthreads();
    }
  }

  const int64_t wg = blockIdx.x;
  const int64_t cg = wg / a.n_rg, g = wg % a.n_rg;
  const int64_t rb = g * 4 + w;
  const bool rb_ok = rb < a.n_rb;
  const int64_t gc_beg = cg * (int64_t)a.cpg * a.n_chpt;
  const int64_t gc_end = min(a.n_chunks, gc_beg + (int64_t)a.cpg * a.n_chpt);

  // B operand of the reconstruction: this wave's 64 T items (and TH for the line search)
  bf16x8 tb[kRecon ? 2 : 1][kRecon ? KS : 1];
  bf16x8 tlo[SPLIT && kRecon ? 2 : 1][SPLIT && kRecon ? KS : 1];
  bf16x8 thb[kLS ? 2 : 1][kLS ? KS : 1];
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const int64_t row = rb * 64 + 32 * n + li;
    const int64_t trow = row < a.nrows ? layout_row(row, a.bmaj, a.nB, a.Ik) : 0;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8 z = {};
      if constexpr (kRecon) {
        tb[n][s] = z;
        if (row < a.nrows)
          tb[n][s] = *reinterpret_cast<const bf16x8*>(a.T + trow * K + s * 16 + h * 8);
      }
      if constexpr (SPLIT && kRecon) {
        tlo[n][s] = z;
        if (row < a.nrows)
          tlo[n][s] = *reinterpret_cast<const bf16x8*>(a.T_lo + trow * K + s * 16 + h * 8);
      }
      if constexpr (kLS) {
        thb[n][s] = z;
        if (row < a.nrows)
          thb[n][s] = *reinterpret_cast<const bf16x8*>(a.TH + trow * K + s * 16 + h * 8);
      }
    }
  }

  // Wait for the table operands here, on every path: left pending into the chunk loop,
  // they make its first products wait for every load in flight, prefetches included.
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)

  const double sig = *a.sigma;
  const bool ls_limit = isinf(sig);
  const float inv2s2 = ls_limit ? 0.f : (float)(0.5 / (sig * sig));
  const float sig2 = ls_limit ? 0.f : (float)(sig * sig);
  const float k2 = inv2s2 * 1.4426950408889634f;  // exp(-u) = 2^(-u log2 e)

  floatx16 sacc[kGrad ? MT : 1][kGrad ? 2 : 1];
  if constexpr (kGrad) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int n = 0; n < 2; ++n) sacc[mt][n] = floatx16{};
  }
  float f0 = 0.f, f1 = 0.f, f2 = 0.f;

  // one observed entry: x, tile index p (36 r + c); `valid` false for lanes past the
  // block's entries (their p belongs to a later block or the zero slack, their y goes to
  // a padding column and their sums are dropped).  No branches, so a group of rounds issues its LDS reads
  // together.  In the least-squares limit k2 = 0 and the weight is exactly 1.
  // wkeep: where a gradient pass leaves the weight for a later store (nullptr: store now)
  // g: the entry's value in the wave's xhat (or q) tile, read beforehand by gather() so
  // that the tile reads of a group of rounds are in flight together
  // bits 0..11 of p: the tile index (< 64 kTS for every slot read: positions of this or a
  // later block, or zero slack); the bits above are ignored
  auto gather = [&](uint32_t p) -> float {
    if constexpr (kGradE) return 0.f;  // no tile: the stored residual is the entry's value
    else return Xs[(int)(p & 4095u)];
  };
  auto entry = [&](float x, uint32_t p, bool valid, int64_t idx, float* wkeep, float g) {
    const int pi = (int)(p & 4095u);
    if constexpr (kLS) {  // the low 16 bits of x hold the entry's weight (fp16)
      const float wv = (float)__builtin_bit_cast(_Float16, (uint16_t)(__float_as_uint(x) & 0xffffu));
      const float q = g;
      f0 = fmaf(valid ? wv * q : 0.f, q, f0);
      return;
    }
    float e;
    if constexpr (kGradE) {
      e = x;  // the stored residual
    } else {
      e = x - g;
    }
    const float wgt = __builtin_amdgcn_exp2f(-(e * e * k2));
    if constexpr (kGrad) {
      Ys[valid ? pi : 32] = __builtin_bit_cast(uint16_t, (__bf16)(wgt * e));
      // the weight, for the line search of this update (lanes past the block's entries
      // write a slot of their own past the last entry)
      if (wkeep) *wkeep = wgt;
      else if (a.wout) a.wout[valid ? idx : a.nobs + l] = f16_bits(wgt);
    }
    if constexpr (MODE == kModeResid) {
      if (valid) {  // e itself (a later gradient pass may reuse it); the keys are |e|
        a.resid[idx] = e;
        if (a.qhist) atomicAdd(&qh[__float_as_uint(fabsf(e)) >> 21], 1u);
      }
    }
    if constexpr (kStats) {
      const float uu = e * e * inv2s2;
      // sigma^2 (1 - exp(-u)), by its series at small u (no cancellation)
      float q = fmaf(uu, 1.0f / 120.0f, -1.0f / 24.0f);
      q = fmaf(uu, q, 1.0f / 6.0f);
      q = fmaf(uu, q, -0.5f);
      q = fmaf(uu, q, 1.0f);
      float lo = uu < 0.0625f ? sig2 * uu * q : sig2 * (1.f - wgt);
      if (ls_limit) lo = 0.5f * e * e;
      f0 += valid ? lo : 0.f;
      f1 += valid ? wgt * e * e : 0.f;
      f2 += valid ? 1.f : 0.f;
    }
  };

  // Software pipeline over the chunks.  In step gc the LDS tiles hold Xhat (and Q) of
  // chunk gc and Y of chunk gc - 1; one straight-line block issues the products of
  // Xhat(gc + 1) and of S += V^T Y(gc - 1) on the matrix cores and, while they run, the
  // vector work of the entries of chunk gc; then Xhat(gc + 1) is spilled.  Three register
  // sets of entries rotate without copies (unroll by three): the set of chunk gc - 1
  // gives the positions to clear in the y tile and is then reloaded with chunk gc + 2.
  // The value / position arrays and the fragment tables carry slack (>= 64 kR + 64
  // entries, one chunk) and the indices are clamped to the walk, so these loads need no
  // bounds branch; what they read past a block's end is never used.
  // Positions are read as the aligned 32-bit word that holds them and shifted at their
  // use: a 16-bit load would be widened right after it arrives, which makes the chunk
  // wait for its own prefetch.
  struct Set {
    float x[kR];
    uint32_t pw[kR];
    uint32_t sh;  // 16 when the position is the word's upper half
  };
  const int64_t bb = rb * a.n_chunks;
  // Block offsets of this wave's walk (at most 64 values, gc_beg .. gc_end): lane i holds
  // boff[bb + gc_beg + i] in a vector register and a chunk reads its offset back with
  // readlane.  A scalar load here would sit in the LDS-wait of every chunk (both are
  // counted by lgkmcnt); the vector load is waited for once.
  const int64_t bwin = (rb_ok && gc_beg < gc_end) ? a.boff[bb + min(gc_beg + l, gc_end)] : 0;
  auto boff_at = [&](int64_t gc) -> int64_t {  // gc in [gc_beg, gc_end]
    const int i = (int)(gc - gc_beg);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bwin, i);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)bwin >> 32), i);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };
  const uint32_t* posw = reinterpret_cast<const uint32_t*>(a.pos);
  const uint32_t* winw = reinterpret_cast<const uint32_t*>(a.win);  // line search
  auto load_set = [&](Set& S, int64_t bo) {
    S.sh = (uint32_t)((bo + l) & 1) * 16u;  // parity of bo + 64 t + l
    const int64_t w0 = (bo + l) >> 1;         // word of bo + 64 t + l: w0 + 32 t
#pragma unroll
    for (int t = 0; t < kR; ++t) {
      if constexpr (kLS)  // the word holding the entry's fp16 weight
        S.x[t] = __uint_as_float(winw[w0 + 32 * t]);
      else
        S.x[t] = a.vals[bo + 64 * t + l];
      S.pw[t] = posw[w0 + 32 * t];
    }
  };
  // A operand of the reconstruction (V^T items of one chunk): loaded for the next chunk
  // as soon as the current chunk's products have been issued
  bf16x8 av[KS];
  bf16x8 avlo[SPLIT ? KS : 1];
  auto load_av = [&](int64_t gc) {
    if constexpr (!kRecon && !kLS) return;  // no reconstruction-side products
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      av[s] = *reinterpret_cast<const bf16x8*>(a.Vf + gc * 32 * K + s * 512 + l * 8);
      if constexpr (SPLIT)
        avlo[s] = *reinterpret_cast<const bf16x8*>(a.Vf_lo + gc * 32 * K + s * 512 + l * 8);
    }
  };

  auto clear_y = [&]() {
    uint4* yz = reinterpret_cast<uint4*>(Ys);  // kYTile * 2 bytes, a multiple of 16
    constexpr int nv = kYTile * 2 / 16;
#pragma unroll
    for (int i = 0; i < (nv + 63) / 64; ++i)
      if (l + 64 * i < nv) yz[l + 64 * i] = uint4{0u, 0u, 0u, 0u};
  };

  // A operand of the gradient product (V^T rows of one chunk), read from the transposed
  // table.  Plain form with K <= 64: two buffers, the step that consumes one loads the next
  // chunk's rows into the other at its start, a whole step before their use (the buffer
  // index is a compile-time constant after unrolling).  The split and wide forms, K > 64
  // and the pass that reads stored residuals (which would lose a wave per SIMD) have no
  // registers to spare: one buffer, loaded at the end of the step before its use.
  constexpr bool kDB = kGrad && !kGradE && !SPLIT && !WIDE && K <= 64;
  bf16x8 aw[kDB ? 2 : 1][kGrad ? 2 : 1][kGrad ? MT : 1];
  auto load_aw = [&](int64_t gc, int buf) {
    if constexpr (!kDB) buf = 0;
    if constexpr (kGrad) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          aw[buf][s2][mt] = *reinterpret_cast<const bf16x8*>(a.VTf + gc * 32 * K +
                                                             (s2 * MT + mt) * 512 + l * 8);
    }
  };

  floatx16 xacc[2];
  floatx16 qacc[kLS ? 2 : 1];
  // Xhat^T (and Q^T) of one chunk from the operands in av (and avlo)
  auto recon = [&]() {
    if constexpr (kRecon) { xacc[0] = floatx16{}; xacc[1] = floatx16{}; }
    if constexpr (kLS) { qacc[0] = floatx16{}; qacc[1] = floatx16{}; }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        if constexpr (SPLIT && kRecon) {  // remainder products first, then the leading one
          xacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(avlo[s], tb[n][s], xacc[n], 0, 0, 0);
          xacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], tlo[n][s], xacc[n], 0, 0, 0);
        }
        if constexpr (kRecon)
          xacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], tb[n][s], xacc[n], 0, 0, 0);
        if constexpr (kLS)
          qacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], thb[n][s], qacc[n], 0, 0, 0);
      }
    }
  };
  // spill Xhat (and Q) to LDS as [row][col]: accumulator v of n-tile n holds col
  // 8 (v/4) + 4 h + v%4 of row 32 n + li
  auto spill = [&]() {
#pragma unroll
    for (int n = 0; n < 2; ++n) {
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        if constexpr (kRecon) {
          const float4 xv = {xacc[n][4 * q4], xacc[n][4 * q4 + 1], xacc[n][4 * q4 + 2],
                             xacc[n][4 * q4 + 3]};
          *reinterpret_cast<float4*>(Xs + (32 * n + li) * kXS + 8 * q4 + 4 * h) = xv;
        }
        if constexpr (kLS) {
          const float4 qv = {qacc[n][4 * q4], qacc[n][4 * q4 + 1], qacc[n][4 * q4 + 2],
                             qacc[n][4 * q4 + 3]};
          *reinterpret_cast<float4*>(Qs + (32 * n + li) * kXS + 8 * q4 + 4 * h) = qv;
        }
      }
    }
  };
  // B operand of the gradient product: Y^T fragments of the chunk in the y tile
  bf16x8 yb[kGrad ? 2 : 1][kGrad ? 2 : 1];
  auto read_y = [&]() {
    if constexpr (kGrad) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int n = 0; n < 2; ++n) {  // rows are 8-byte aligned: two 8-byte reads
          const uint2* yp =
              reinterpret_cast<const uint2*>(Ys + (32 * n + li) * kYS + 16 * s2 + 8 * h);
          const uint2 y0 = yp[0], y1 = yp[1];
          yb[s2][n] = __builtin_bit_cast(bf16x8, uint4{y0.x, y0.y, y1.x, y1.y});
        }
    }
  };
  // S^T += V^T-items^T . Y^T over a chunk's 32 columns (two k-steps of 16)
  auto grad_products = [&](int buf) {
    if constexpr (!kDB) buf = 0;
    if constexpr (kGrad) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int n = 0; n < 2; ++n)
            sacc[mt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw[buf][s2][mt], yb[s2][n],
                                                                  sacc[mt][n], 0, 0, 0);
    }
  };

  // [bo_cur, bo_end): entries of chunk gc; bo_nend: start of chunk gc + 2
  int64_t bo_cur = 0, bo_end = 0, bo_nend = 0;
  int nent_prev = 0;  // entries of chunk gc - 1 (0 before the first chunk)
  // P: set of chunk gc - 1 on entry, of chunk gc + 2 on exit; C: set of chunk gc; ab: the
  // gradient operand buffer holding the V^T rows of chunk gc - 1
  auto step = [&](int64_t gc, const Set& C, Set& P, int ab) {
    if (!rb_ok) return;  // uniform over the wave
    const int64_t bo_nn = boff_at(min(gc + 3, gc_end));
    const int nent = (int)(bo_end - bo_cur);

    // 1. y fragments of chunk gc - 1, then clear its positions (LDS accesses of a wave
    //    complete in order, so the clears follow the reads)
    if constexpr (kGrad) {
      read_y();
      if (nent_prev <= 64 * kR) {
#pragma unroll
        for (int t0 = 0; t0 < kR; t0 += 4) {
          if (64 * t0 < nent_prev) {
#pragma unroll
            for (int t = t0; t < t0 + 4; ++t) {  // no branch: other lanes clear padding
              const uint32_t p = P.pw[t] >> P.sh;
              Ys[64 * t + l < nent_prev ? (p & 4095u) : 32u] = 0;
            }
          }
        }
      } else {
        clear_y();
      }
    }
    // the set of chunk gc - 1 is free: load the entries of chunk gc + 2 (offset
    // bo_nend <= nobs)
    load_set(P, bo_nend);
    // (two-buffer form: the V^T rows of chunk gc, for the next step, into the other buffer)
    if constexpr (kDB) load_aw(gc, ab ^ 1);

    // 2. matrix-core products of Xhat(gc + 1) and S(gc - 1), with the first four rounds
    //    of entries of chunk gc in the same straight-line block
    // (the gradient products first: their operands are then free before the
    // reconstruction accumulators are live)
    grad_products(ab);
    recon();
    // without gradient products the registers allow loading the next reconstruction
    // operands here, a whole chunk ahead of their use
    if constexpr (!kGrad) load_av(min(gc + 2, a.n_chunks));
    float g[4];  // the tile reads of the first four rounds, issued together
#pragma unroll
    for (int t = 0; t < 4 && t < kR; ++t) g[t] = gather(C.pw[t] >> C.sh);
    float wk[4];  // weights of the first four rounds, stored after the operand loads below
#pragma unroll
    for (int t = 0; t < 4 && t < kR; ++t) {
      const int i = 64 * t + l;
      entry(kLS ? __uint_as_float(__float_as_uint(C.x[t]) >> C.sh) : C.x[t], C.pw[t] >> C.sh,
            i < nent, bo_cur + i, &wk[t], g[t]);
    }
    // interleave: a wave waits at every product it issues while the matrix core is busy
    // with the previous one, so the vector work of the entries goes in between
    // (not in the split form, whose registers are too tight for the longer live ranges)
    constexpr int kMfma = SPLIT ? 0 : (kRecon || kLS ? KS * 2 : 0) + (kGrad ? 4 * MT : 0);
#pragma unroll
    for (int i = 0; i < kMfma; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix-core product
      __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // three vector ALU instructions
    }
#pragma unroll
    for (int t0 = 4; t0 < kR; t0 += 4) {
      if (64 * t0 < nent) {
        float g4[4];
#pragma unroll
        for (int t = t0; t < t0 + 4; ++t) g4[t - t0] = gather(C.pw[t] >> C.sh);
#pragma unroll
        for (int t = t0; t < t0 + 4; ++t) {
          const int i = 64 * t + l;
          entry(kLS ? __uint_as_float(__float_as_uint(C.x[t]) >> C.sh) : C.x[t], C.pw[t] >> C.sh,
                i < nent, bo_cur + i, nullptr, g4[t - t0]);
        }
      }
    }
    for (int i0 = 64 * kR; i0 < nent; i0 += 64) {  // dense blocks: remaining rounds
      const int i = i0 + l;
      const bool valid = i < nent;
      float x = 0.f;
      if constexpr (kLS) x = valid ? __uint_as_float((uint32_t)a.win[bo_cur + i]) : 0.f;
      else x = valid ? a.vals[bo_cur + i] : 0.f;
      const uint32_t p = valid ? (uint32_t)a.pos[bo_cur + i] : 0u;
      entry(x, p, valid, bo_cur + i, nullptr, gather(p));
    }
    wave_sync();

    // 3. Xhat(gc + 1) into the tiles (after this chunk's reads of them)
    spill();
    wave_sync();
    // 4. gradient passes: operands of the next step, loaded once the registers are free:
    //    V^T rows of chunk gc and V^T items of chunk gc + 2 (clamped: the fragment tables
    //    end with one padding chunk)
    if constexpr (kGrad) {
      if constexpr (!kDB) load_aw(gc, 0);
      load_av(min(gc + 2, a.n_chunks));
      // the weights last: memory operations retire in order, so stores issued before the
      // operand loads would hold up the next step's wait for those operands
      if (a.wout) {
#pragma unroll
        for (int t = 0; t < 4 && t < kR; ++t) {
          const int i = 64 * t + l;
          a.wout[i < nent ? bo_cur + i : a.nobs + l] = f16_bits(wk[t]);
        }
      }
    }

    nent_prev = nent;
    bo_cur = bo_end;
    bo_end = bo_nend;
    bo_nend = bo_nn;
  };

  Set A, B, C;
  if constexpr (kGrad) clear_y();
  const bool walk = rb_ok && gc_beg < gc_end;
  if (walk) {
    bo_cur = boff_at(gc_beg);
    bo_end = boff_at(gc_beg + 1);
    bo_nend = boff_at(min(gc_beg + 2, gc_end));
    load_av(gc_beg);
    load_set(A, bo_cur);
    load_set(B, bo_end);
#pragma unroll
    for (int s2 = 0; s2 < (kGrad ? 2 : 1); ++s2)
#pragma unroll
      for (int mt = 0; mt < (kGrad ? MT : 1); ++mt) aw[0][s2][mt] = bf16x8{};  // no chunk gc_beg - 1
    recon();
    load_av(gc_beg + 1);  // <= n_chunks
    spill();
    wave_sync();
  }
  // the first loads land before the walk: otherwise the counted waits at the top of the
  // chunk loop must also cover these (register assignment differs between the two paths)
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  // three entry sets and two gradient operand buffers rotate: unrolled by six
  for (int64_t gc = gc_beg; gc < gc_end; gc += 6) {
    step(gc, A, C, 0);
    if (gc + 1 < gc_end) step(gc + 1, B, A, 1);
    if (gc + 2 < gc_end) step(gc + 2, C, B, 0);
    if (gc + 3 < gc_end) step(gc + 3, A, C, 1);
    if (gc + 4 < gc_end) step(gc + 4, B, A, 0);
    if (gc + 5 < gc_end) step(gc + 5, C, B, 1);
  }
  if (walk) {  // S of the last chunk: its V^T rows are in buffer (gc_end - gc_beg) & 1
    read_y();
    if (!kDB || ((gc_end - gc_beg) & 1) == 0) grad_products(0);
    else grad_products(1);
  }

  // S^T accumulator: lane l holds row 32 n + li of the block and, in register v,
  // j = 32 mt + 8 (v/4) + 4h + v%4
  bool contracted = false;
  if constexpr (kGrad && K == 64) {
    if (a.dpart && rb_ok) {  // (uniform over the wave)
      // B-major rows, r_k = r_s = r_{k+1} = 8: item j = a + 8c of a row factor has a = 4h +
      // v%4 and c = 4 mt + v/4, so the lane's part of D(i_k)[a + 8 beta] = sum_c S[a + 8c]
      // U(b)[beta + 8c] is a = 4h .. 4h + 3 for every beta.  The block's rows belong to
      // slice i0 and, past a slice boundary, i0 + 1: one reduction per slice.
      contracted = true;
      const int64_t t0 = rb * 64;
      const int64_t i0 = t0 / a.nB;
      const int64_t tl = min(t0 + 63, a.nrows - 1);
      const int nsl = (int)(tl / a.nB - i0) + 1;
      float* rtile = Xs;  // this wave's tile: [h][li][kXS]; the walk no longer reads it
      for (int sl = 0; sl < nsl; ++sl) {
        float acc[4][8];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int be = 0; be < 8; ++be) acc[u][be] = 0.f;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const int64_t t = t0 + 32 * n + li;
          const int64_t ik = t / a.nB;
          const bool in = t < a.nrows && ik == i0 + sl;
          const float* up = a.U + (in ? t - ik * a.nB : 0) * a.Us;
#pragma unroll
          for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int c = 4 * mt + q;
              const float4 u0 = *reinterpret_cast<const float4*>(up + 8 * c);
              const float4 u1 = *reinterpret_cast<const float4*>(up + 8 * c + 4);
              const float uv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const float sv = in ? sacc[mt][n][4 * q + u] : 0.f;
#pragma unroll
                for (int be = 0; be < 8; ++be) acc[u][be] = fmaf(sv, uv[be], acc[u][be]);
              }
            }
        }
        // the 32 lanes of each half h hold the same 32 outputs: add them in lane order
        wave_sync();
#pragma unroll
        for (int be = 0; be < 8; ++be)
          *reinterpret_cast<float4*>(rtile + (h * 32 + li) * kXS + 4 * be) =
              float4{acc[0][be], acc[1][be], acc[2][be], acc[3][be]};
        wave_sync();
        const int hh = l >> 5, oo = l & 31;  // output a = 4 hh + oo % 4, beta = oo / 4
        float sum = 0.f;
        for (int i = 0; i < 32; ++i) sum += rtile[(hh * 32 + i) * kXS + oo];
        a.dpart[((cg * a.n_rb + rb) * 2 + sl) * 64 + (4 * hh + (oo & 3)) + 8 * (oo >> 2)] = sum;
      }
    }
  }
  if constexpr (kGrad) {
    // otherwise the row factors themselves: four consecutive j per group of four
    // registers, stored as one 16-byte vector (RRP is a multiple of 4, so j0 < RRP covers
    // j0 + 3), at the row's layout position
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int64_t row = rb * 64 + 32 * n + li;
      if (contracted || row >= a.nrows) continue;
      float* sp = a.S + (cg * a.nrows + layout_row(row, a.bmaj, a.nB, a.Ik)) * a.RRP;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int j0 = mt * 32 + 8 * q + 4 * h;
          if (j0 < a.RRP)
            *reinterpret_cast<float4*>(sp + j0) =
                float4{sacc[mt][n][4 * q], sacc[mt][n][4 * q + 1], sacc[mt][n][4 * q + 2],
                       sacc[mt][n][4 * q + 3]};
        }
    }
  }

  double s0 = (double)f0, s1 = (double)f1, s2 = (double)f2;
  __shared__ double red[3][4];
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o);
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  if (l == 0) {
    red[0][w] = s0;
    red[1][w] = s1;
    red[2][w] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const double* r = red[threadIdx.x];
    a.partials[wg * 3 + threadIdx.x] = (r[0] + r[1]) + (r[2] + r[3]);
  }
  if constexpr (MODE == kModeResid) {  // the work-group's digit counts into the global one
    if (a.qhist)
      for (int i = threadIdx.x; i < kQHistBins; i += 256)
        if (qh[i]) atomicAdd(&a.qhist[i], qh[i]);
  }
}

int tile_k(int RR) { return (RR + 31) / 32 * 32; }

// column-tile width of the gradient pass: the bf16 V^T tile fills what the per-wave
// tiles leave of half the CU's LDS (two work-groups per CU)
// Fragment order of the column table, per 32-column chunk g (columns past ncols are 0):
//   Vf  [g][s < K/16][lane][8]:        V[32 g + lane % 32][16 s + 8 (lane / 32) + i]
//   VTf [g][s2 < 2][mt < K/32][lane][8]: V[32 g + 16 s2 + 8 (lane / 32) + i][32 mt + lane % 32]
// i.e. the A operands of the reconstruction and gradient products exactly as the lanes
// hold them, so that a wave reads each operand as one contiguous kilobyte.
__global__ __launch_bounds__(256) void k_fragments(const uint16_t* __restrict__ V, int64_t ncols,
                                                   int K, uint16_t* __restrict__ Vf,
                                                   uint16_t* __restrict__ VTf) {
  __shared__ __align__(16) uint16_t tile[32 * (128 + 8)];  // [column][k], row stride K + 8
  const int ks = K + 8;
  const int64_t g = blockIdx.x;
  const int64_t c0 = g * 32;
  const int kv = K / 8;
  for (int e = threadIdx.x; e < 32 * kv; e += 256) {
    const int c = e / kv, j = e - c * kv;
    uint4 u = uint4{0u, 0u, 0u, 0u};
    if (c0 + c < ncols) u = *reinterpret_cast<const uint4*>(V + (c0 + c) * K + 8 * j);
    *reinterpret_cast<uint4*>(tile + c * ks + 8 * j) = u;
  }
  __syncthreads();
  const int64_t base = g * 32 * K;
  const int nvec = 4 * K;  // 16-byte vectors per chunk, in either order
  for (int e = threadIdx.x; e < nvec; e += 256) {
    const int l = e & 63, li = l & 31, h = l >> 5;
    {  // Vf: e = s * 64 + lane
      const int s = e >> 6;
      *reinterpret_cast<uint4*>(Vf + base + 8 * e) =
          *reinterpret_cast<const uint4*>(tile + li * ks + 16 * s + 8 * h);
    }
    if (VTf) {  // VTf: e = (s2 * MT + mt) * 64 + lane
      const int MT = K / 32;
      const int q = e >> 6, s2 = q / MT, mt = q - s2 * MT;
      uint32_t w[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 16 * s2 + 8 * h + 2 * i;
        w[i] = (uint32_t)tile[c * ks + 32 * mt + li] | ((uint32_t)tile[(c + 1) * ks + 32 * mt + li] << 16);
      }
      *reinterpret_cast<uint4*>(VTf + base + 8 * e) = uint4{w[0], w[1], w[2], w[3]};
    }
  }
}

hipError_t launch_fragments(const uint16_t* V, int64_t ncols, int K, uint16_t* Vf, uint16_t* VTf,
                            hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  if (K <= 0 || K > 128 || K % 32 != 0) return hipErrorInvalidValue;
  const int64_t nch = (ncols + 31) / 32 + 1;  // the padding chunk included
  hipLaunchKernelGGL(k_fragments, dim3((unsigned)nch), dim3(256), 0, st, V, ncols, K, Vf, VTf);
  return hipGetLastError();
}

int64_t tile_cw(int K) {
  int64_t budget = g_lds_max >= 2 * 81920 ? 81920 - 1024 : g_lds_max - 1024;
  int64_t cw = (budget - kXBytes - kYBytes) / (2 * K) - 8;
  cw = cw / 32 * 32;
  if (cw < 32) cw = 32;
  return cw;
}

template <int K, bool SPLIT, bool WIDE>
static hipError_t launch_k(int mode, const TPassArgs& a, hipStream_t st, KTiming tm) {
  const int64_t nwg = a.n_rg * a.n_cg;
  const size_t lds = tpass_lds(mode, K, a.CW);
  if ((int64_t)lds > g_lds_max) return hipErrorInvalidConfiguration;
  dim3 g((unsigned)nwg), b(256);
  switch (mode) {
    case kModeGrad: TRD_LAUNCH((k_tpass<K, kModeGrad, SPLIT, WIDE>), g, b, lds, st, tm, a); break;
    case kModeGradFast:
      TRD_LAUNCH((k_tpass<K, kModeGradFast, SPLIT, WIDE>), g, b, lds, st, tm, a);
      break;
    case kModeLS: TRD_LAUNCH((k_tpass<K, kModeLS, SPLIT, WIDE>), g, b, lds, st, tm, a); break;
    case kModeResid: TRD_LAUNCH((k_tpass<K, kModeResid, SPLIT, WIDE>), g, b, lds, st, tm, a); break;
    case kModeGradE: TRD_LAUNCH((k_tpass<K, kModeGradE, SPLIT, WIDE>), g, b, lds, st, tm, a); break;
    default: TRD_LAUNCH((k_tpass<K, kModeLoss, SPLIT, WIDE>), g, b, lds, st, tm, a); break;
  }
  return hipGetLastError();
}

template <int K>
static hipError_t launch_ks(int mode, const TPassArgs& a, hipStream_t st, KTiming tm) {
  if (a.T_lo && a.Vf_lo) return launch_k<K, true, false>(mode, a, st, tm);
  if (K == 64 && a.rounds > 4) return launch_k<K, false, true>(mode, a, st, tm);
  return launch_k<K, false, false>(mode, a, st, tm);
}

hipError_t launch_tpass(int mode, int K, const TPassArgs& a, hipStream_t st, KTiming tm) {
  if (a.n_rg * a.n_cg <= 0 || a.n_chunks <= 0) return hipSuccess;
  // the grid and chunk walk must cover exactly the layout the pass indexes
  if ((a.T_lo == nullptr) != (a.Vf_lo == nullptr)) return hipErrorInvalidValue;
  if (a.CW % 32 != 0 || a.n_chpt != a.CW / 32 || a.cpg < 1 || a.n_rb > 4 * a.n_rg ||
      (int64_t)a.cpg * a.n_chpt > 63 ||
      (int64_t)a.n_cg * a.cpg * a.n_chpt < a.n_chunks ||
      (int64_t)(a.n_cg - 1) * a.cpg * a.n_chpt >= a.n_chunks || a.n_chunks * 32 < a.ncols ||
      a.n_rb * 64 < a.nrows || a.RRP > K)
    return hipErrorInvalidValue;
  // the fragment tables hold n_chunks + 1 chunks (tile_frag_elems), the passes read one
  // chunk ahead; the gradient products need the transposed one
  if (a.Vf == nullptr ||
      ((mode == kModeGrad || mode == kModeGradFast || mode == kModeGradE) && a.VTf == nullptr))
    return hipErrorInvalidValue;
  // B-major rows: tile rows are the layout rows of nB items per slice, and the epilogue
  // contraction (rank 8, K = 64) needs at least 64 rows per slice (a block spans <= 2)
  if (a.bmaj && (a.nB < 1 || a.Ik < 1 || a.nB * a.Ik != a.nrows)) return hipErrorInvalidValue;
  if (a.dpart && (K != 64 || !a.bmaj || a.nB < 64 || a.U == nullptr || a.Us < 64 ||
                  a.RR != 64 || a.RRP != 64))
    return hipErrorInvalidValue;
  switch (K) {
    case 32: return launch_ks<32>(mode, a, st, tm);
    case 64: return launch_ks<64>(mode, a, st, tm);
    case 96: return launch_ks<96>(mode, a, st, tm);
    case 128: return launch_ks<128>(mode, a, st, tm);
    default: return hipErrorInvalidValue;
  }
}

// d(i_k)[o] = scale * sum of the epilogue partials of slice i_k, the partial index running
// over the column groups, then over the 64-row blocks rb that hold rows of the slice (slot
// i_k - first slice of rb).  One work-group per slice; thread (o, g) adds partials g, g + 16,
// ... in order (its loads issued eight at a time before the sums), then the 16 group sums
// are added in a fixed tree.
__global__ __launch_bounds__(1024) void k_dpart_finish(const float* __restrict__ part, int n_cg,
                                                       int64_t n_rb, int64_t nB, int64_t Ik,
                                                       double* __restrict__ d64,
                                                       float* __restrict__ d_out, double scale) {
  __shared__ double red[16][64];
  const int64_t ik = blockIdx.x;
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t rb_lo = ik * nB / 64, rb_hi = ((ik + 1) * nB - 1) / 64;
  const int64_t nrb = rb_hi - rb_lo + 1, np = (int64_t)n_cg * nrb;
  auto at = [&](int64_t i) -> float {
    const int64_t cg = i / nrb, rb = rb_lo + (i - cg * nrb);
    const int64_t slot = ik - rb * 64 / nB;
    return part[((cg * n_rb + rb) * 2 + slot) * 64 + o];
  };
  double s = 0.0;
  int64_t i = g;
  for (; i + 16 * 7 < np; i += 16 * 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = at(i + 16 * u);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (double)v[u];
  }
  for (; i < np; i += 16) s += (double)at(i);
  red[g][o] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (g < w) red[g][o] += red[g + w][o];
    __syncthreads();
  }
  if (g == 0) {
    const double v = red[0][o] * scale;
    if (d64) d64[ik * 64 + o] = v;
    if (d_out) d_out[ik * 64 + o] = (float)v;
  }
}

hipError_t launch_dpart_finish(const float* part, int n_cg, int64_t n_rb, int64_t nB, int64_t Ik,
                               double* d64, float* d_out, double scale, hipStream_t st) {
  if (Ik <= 0) return hipSuccess;
  if (nB < 64 || n_cg < 1 || (Ik * nB + 63) / 64 > n_rb) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dpart_finish, dim3((unsigned)Ik), dim3(1024), 0, st, part, n_cg, n_rb, nB,
                     Ik, d64, d_out, scale);
  return hipGetLastError();
}


// The same sums, then the scaled direction of eq. (10) for the slice: h(i_k)[c] =
// sum_l d(i_k)[l] Cinv[l n + c] in order (Cinv == nullptr: h = d; the not-SPD flag set: h = 0),
// written as FP64 and FP32, and the slice's share of <d, h> (the line search's numerator)
// into pdh[i_k].  One work-group per slice; the matrix is 64 x 64 (rank 8).
__global__ __launch_bounds__(1024) void k_dpart_direction(const float* __restrict__ part, int n_cg,
                                                          int64_t n_rb, int64_t nB,
                                                          const double* __restrict__ Cinv,
                                                          const uint32_t* flags,
                                                          double* __restrict__ d64,
                                                          double* __restrict__ h64,
                                                          float* __restrict__ h_real,
                                                          double* __restrict__ pdh) {
  __shared__ double red[16][64];
  const int64_t ik = blockIdx.x;
  const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t rb_lo = ik * nB / 64, rb_hi = ((ik + 1) * nB - 1) / 64;
  const int64_t nrb = rb_hi - rb_lo + 1, np = (int64_t)n_cg * nrb;
  auto at = [&](int64_t i) -> float {
    const int64_t cg = i / nrb, rb = rb_lo + (i - cg * nrb);
    const int64_t slot = ik - rb * 64 / nB;
    return part[((cg * n_rb + rb) * 2 + slot) * 64 + o];
  };
  double s = 0.0;
  int64_t i = g;
  for (; i + 16 * 7 < np; i += 16 * 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = at(i + 16 * u);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (double)v[u];
  }
  for (; i < np; i += 16) s += (double)at(i);
  red[g][o] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (g < w) red[g][o] += red[g + w][o];
    __syncthreads();
  }
  if (g == 0) {  // one wave: output c = o
    const double dv = red[0][o];
    d64[ik * 64 + o] = dv;
    const bool bad = (*flags & TRD_FLAG_NOTSPD_BIT) != 0;
    double hv = 0.0;
    if (!Cinv)
      hv = dv;
    else if (!bad)
      for (int l = 0; l < 64; ++l) hv = fma(red[0][l], Cinv[l * 64 + o], hv);
    h64[ik * 64 + o] = hv;
    if (h_real) h_real[ik * 64 + o] = (float)hv;
    double c = dv * hv;
    for (int w = 32; w > 0; w >>= 1) c += __shfl_xor(c, w);
    if (o == 0) pdh[ik] = c;
  }
}

hipError_t launch_dpart_direction(const float* part, int n_cg, int64_t n_rb, int64_t nB, int64_t Ik,
                                  const double* Cinv, const uint32_t* flags, double* d64,
                                  double* h64, float* h_real, double* pdh, hipStream_t st) {
  if (Ik <= 0) return hipSuccess;
  if (nB < 64 || n_cg < 1 || (Ik * nB + 63) / 64 > n_rb) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dpart_direction, dim3((unsigned)Ik), dim3(1024), 0, st, part, n_cg, n_rb,
                     nB, Cinv, flags, d64, h64, h_real, pdh);
  return hipGetLastError();
}

}  // namespace trd

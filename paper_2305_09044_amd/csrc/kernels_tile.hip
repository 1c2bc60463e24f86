// Matrix-core (MFMA) form of the fused entry passes: the BF16 precision form.
//
// The observed entries of a core-k matrix (rows = (i_k, first subchain modes), cols =
// the rest) are grouped in blocks of 64 rows x 32 columns.  A block stores its observed
// values and their in-block positions p = 32 r + c (r < 64, c < 32), in increasing p.
// One wave owns a 64-row block row and walks its blocks (32-column chunks):
//   1. Xhat^T (32 cols x 64 rows) = V^T-items (32 x K) . T-items^T (K x 64) on the
//      matrix cores (Thm. 1): bf16 operands, FP32 accumulation, spilled to LDS;
//   2. each observed entry of the block (lane-parallel, in value order) reads its xhat,
//      forms e = x - xhat, w = exp(-e^2/2s^2) (eq. 7) and y = w e in FP32, and scatters
//      y (rounded to bf16) into a cleared 64 x 32 tile in LDS;
//   3. S^T (K x 64 rows) += V^T-items^T (K x 32 cols) . Y^T (32 cols x 64 rows) on the
//      matrix cores: the row factor of the gradient of eq. 9.
// Matrix-core work covers every position of a block; vector work is per observed entry.
// Split form (SPLIT): the T and V tables also come as bf16 remainders (t = t_hi + t_lo),
// and Xhat adds the products t_hi v_lo and t_lo v_hi, so the reconstruction (and the
// residual) carries about 16 significant bits instead of 8; the gradient contraction
// stays a single bf16 product.
// A work-group (4 waves = 4 block rows) walks a group of column tiles and keeps its S
// accumulators in registers; the V^T items of the current tile are staged transposed in
// LDS as the A operand of step 3.
#include "trd_internal.h"

namespace trd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

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
};

static TileArgs targs(const TLayout& L) {
  TileArgs a;
  a.rowoff = L.rowoff; a.coloff = L.coloff; a.bcnt = L.bcnt; a.boff = L.boff;
  a.vals = L.vals; a.pos = L.pos;
  a.nrows = L.nrows; a.ncols = L.ncols; a.n_chunks = L.n_chunks; a.n_blocks = L.n_blocks;
  return a;
}

// Block b = rb * n_chunks + ch, one wave per block.  Round t covers positions
// p = 64 t + lane (row 2 t + lane / 32, column lane % 32), so the ballot of a round lists
// its observed entries in increasing p.  Count pass (FILL = false): per-block counts;
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
      off = a.rowoff[row] + co;
      obs = mask[off] != 0;
    }
    const uint64_t bal = __ballot(obs);
    if constexpr (FILL) {
      if (obs) {
        const int pre = __popcll(bal & ((1ull << l) - 1ull));
        a.vals[out + pre] = (float)X[off];
        a.pos[out + pre] = (uint16_t)p;
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

// Per-wave LDS tiles.  Row strides are odd multiples of 16 bytes, so the 16-byte accesses
// of eight consecutive rows by eight lanes fall in distinct banks.
constexpr int kXS = 36;                 // f32 stride of the xhat (and q) tile
constexpr int kYS = 40;                 // bf16 stride of the y tile
constexpr int kXTile = 64 * kXS;        // floats
constexpr int kYTile = 64 * kYS;        // bf16
constexpr int kXBytes = 4 * kXTile * 4; // four waves
constexpr int kYBytes = 4 * kYTile * 2;

template <int K, bool SPLIT> struct TileRounds {
  static constexpr int v = K <= 32 ? 12 : (K <= 64 && !SPLIT ? 8 : 4);
};

size_t tpass_lds(int mode, int K, int CW) {
  if (mode == kModeGrad || mode == kModeGradFast)
    return (size_t)kXBytes + kYBytes + (size_t)K * (CW + 8) * 2;
  if (mode == kModeLS) return 2 * (size_t)kXBytes;
  return (size_t)kXBytes;
}

template <int K, int MODE, bool SPLIT>
__global__ __launch_bounds__(256, (K >= 96 ? 1 : 2)) void k_tpass(TPassArgs a) {
  constexpr int KS = K / 16;       // k-steps of the reconstruction MFMA
  constexpr int MT = K / 32;       // m-tiles of the gradient MFMA
  constexpr int kR = TileRounds<K, SPLIT>::v;  // entry rounds of 64 in registers per chunk
  constexpr bool kGrad = MODE == kModeGrad || MODE == kModeGradFast;
  constexpr bool kLS = MODE == kModeLS;
  constexpr bool kStats = MODE == kModeGrad || MODE == kModeLoss;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int CWP = a.CW + 8;
  // the wave index is uniform over the wave: keep it (and everything derived from it:
  // block row, block offsets, loop bounds) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63, h = l >> 5, li = l & 31;
  float* Xs = reinterpret_cast<float*>(smem_raw) + w * kXTile;
  float* Qs = reinterpret_cast<float*>(smem_raw + kXBytes) + w * kXTile;             // LS
  uint16_t* Ys = reinterpret_cast<uint16_t*>(smem_raw + kXBytes) + w * kYTile;       // grad
  uint16_t* Vc = reinterpret_cast<uint16_t*>(smem_raw + kXBytes + kYBytes);          // grad

  const int64_t wg = blockIdx.x;
  const int64_t cg = wg / a.n_rg, g = wg % a.n_rg;
  const int64_t rb = g * 4 + w;
  const bool rb_ok = rb < a.n_rb;
  const int64_t gc_beg = cg * (int64_t)a.cpg * a.n_chpt;
  const int64_t gc_end = min(a.n_chunks, gc_beg + (int64_t)a.cpg * a.n_chpt);

  // B operand of the reconstruction: this wave's 64 T items (and TH for the line search)
  bf16x8 tb[2][KS];
  bf16x8 tlo[SPLIT ? 2 : 1][SPLIT ? KS : 1];
  bf16x8 thb[kLS ? 2 : 1][kLS ? KS : 1];
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const int64_t row = rb * 64 + 32 * n + li;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8 z = {};
      tb[n][s] = z;
      if (row < a.nrows)
        tb[n][s] = *reinterpret_cast<const bf16x8*>(a.T + row * K + s * 16 + h * 8);
      if constexpr (SPLIT) {
        tlo[n][s] = z;
        if (row < a.nrows)
          tlo[n][s] = *reinterpret_cast<const bf16x8*>(a.T_lo + row * K + s * 16 + h * 8);
      }
      if constexpr (kLS) {
        thb[n][s] = z;
        if (row < a.nrows)
          thb[n][s] = *reinterpret_cast<const bf16x8*>(a.TH + row * K + s * 16 + h * 8);
      }
    }
  }

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

  // one observed entry: x, in-block position p; `valid` false for lanes past the block's
  // entries (their p is masked into the tile, their y goes to the tile's padding column
  // and their sums are dropped).  No branches, so a group of rounds issues its LDS reads
  // together.  In the least-squares limit k2 = 0 and the weight is exactly 1.
  auto entry = [&](float x, uint32_t p, bool valid, int64_t idx) {
    p &= 2047u;
    const int r = (int)(p >> 5), c = (int)(p & 31u);
    const float xh = Xs[r * kXS + c];
    const float e = x - xh;
    const float wgt = __builtin_amdgcn_exp2f(-(e * e * k2));
    if constexpr (kGrad)
      Ys[r * kYS + (valid ? c : 32)] = __builtin_bit_cast(uint16_t, (__bf16)(wgt * e));
    if constexpr (kLS) {
      const float q = Qs[r * kXS + c];
      f0 = fmaf(valid ? wgt * q : 0.f, q, f0);
    }
    if constexpr (MODE == kModeResid) {
      if (valid) a.resid[idx] = fabsf(e);
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

  // Software pipeline over the chunks, unrolled by two so that the two register sets
  // swap roles without copies: at the top of a chunk the next chunk's entries and
  // V^T-item operands are loaded into the idle set, so they have a whole chunk to
  // arrive.  The value / position arrays and the bf16 column table carry slack
  // (>= 64 kR + 64 entries, >= 64 items) and the offset index is clamped to the walk, so
  // these loads need no bounds branch; what they read past a block's end is never used.
  struct Set {
    float x[kR];
    uint32_t p[kR];
  };
  const int64_t bb = rb * a.n_chunks;
  auto load_set = [&](Set& S, int64_t bo) {
#pragma unroll
    for (int t = 0; t < kR; ++t) {
      S.x[t] = a.vals[bo + 64 * t + l];
      S.p[t] = a.pos[bo + 64 * t + l];
    }
  };
  // A operand of the reconstruction (V^T items of one chunk): loaded for the next chunk
  // as soon as the current chunk's products have been issued
  bf16x8 av[KS];
  bf16x8 avlo[SPLIT ? KS : 1];
  auto load_av = [&](int64_t gc) {
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      av[s] = *reinterpret_cast<const bf16x8*>(a.V + (gc * 32 + li) * K + s * 16 + h * 8);
      if constexpr (SPLIT)
        avlo[s] = *reinterpret_cast<const bf16x8*>(a.V_lo + (gc * 32 + li) * K + s * 16 + h * 8);
    }
  };

  constexpr int KV = K / 8;  // 16-byte vectors per table item
  // [bo_cur, bo_end): entries of the current chunk; bo_nend: end of the next one
  int64_t bo_cur = 0, bo_end = 0, bo_nend = 0;
  auto step = [&](int64_t gc, const Set& C, Set& N) {
    const int cc = (int)((gc - gc_beg) % a.n_chpt);  // chunk inside the current tile
    if constexpr (kGrad) {
      if (cc == 0) {  // new column tile: every wave is past the old one, restage V^T items
        __syncthreads();
        const int64_t col0 = gc * 32;
        const int nct = (int)min((int64_t)a.CW, a.ncols - col0);
        const int nvec = a.CW * KV;
        for (int i0 = 0; i0 < nvec; i0 += 4 * 256) {
          uint4 buf[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + 256 * u + threadIdx.x;
            const int c = i % a.CW, jv = i / a.CW;
            buf[u] = uint4{0u, 0u, 0u, 0u};
            if (i < nvec && c < nct)
              buf[u] = *reinterpret_cast<const uint4*>(a.V + (col0 + c) * K + 8 * jv);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + 256 * u + threadIdx.x;
            if (i < nvec) {
              const int c = i % a.CW, jv = i / a.CW;
              const uint32_t wv[4] = {buf[u].x, buf[u].y, buf[u].z, buf[u].w};
#pragma unroll
              for (int e = 0; e < 8; ++e)
                Vc[(8 * jv + e) * CWP + c] = (uint16_t)(wv[e >> 1] >> ((e & 1) * 16));
            }
          }
        }
        __syncthreads();
      }
    }
    if (!rb_ok) return;  // uniform over the wave; it still joins every tile barrier

    // prefetch the next chunk's entries (offset bo_end <= nobs)
    load_set(N, bo_end);
    const int64_t bo_nn = a.boff[bb + min(gc + 3, gc_end)];

    // 1. Xhat^T (and Q^T) of this chunk
    floatx16 xacc[2] = {floatx16{}, floatx16{}};
    floatx16 qacc[kLS ? 2 : 1];
    if constexpr (kLS) { qacc[0] = floatx16{}; qacc[1] = floatx16{}; }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        if constexpr (SPLIT) {  // remainder products first, then the leading one
          xacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(avlo[s], tb[n][s], xacc[n], 0, 0, 0);
          xacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], tlo[n][s], xacc[n], 0, 0, 0);
        }
        xacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], tb[n][s], xacc[n], 0, 0, 0);
        if constexpr (kLS)
          qacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], thb[n][s], qacc[n], 0, 0, 0);
      }
    }
    // the next chunk's operands (chunk index gc + 1 <= n_chunks: within the table slack)
    load_av(gc + 1);

    // 2. spill Xhat (and Q) to LDS as [row][col]; clear the y tile
    // accumulator v of n-tile n: col 8 (v/4) + 4 h + v%4, row 32 n + li
#pragma unroll
    for (int n = 0; n < 2; ++n) {
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const float4 xv = {xacc[n][4 * q4], xacc[n][4 * q4 + 1], xacc[n][4 * q4 + 2],
                           xacc[n][4 * q4 + 3]};
        *reinterpret_cast<float4*>(Xs + (32 * n + li) * kXS + 8 * q4 + 4 * h) = xv;
        if constexpr (kLS) {
          const float4 qv = {qacc[n][4 * q4], qacc[n][4 * q4 + 1], qacc[n][4 * q4 + 2],
                             qacc[n][4 * q4 + 3]};
          *reinterpret_cast<float4*>(Qs + (32 * n + li) * kXS + 8 * q4 + 4 * h) = qv;
        }
      }
    }
    if constexpr (kGrad) {
      uint4* yz = reinterpret_cast<uint4*>(Ys);
#pragma unroll
      for (int i = 0; i < kYTile * 2 / 16 / 64; ++i) yz[l + 64 * i] = uint4{0u, 0u, 0u, 0u};
    }
    wave_sync();

    // 3. the observed entries of the block, four rounds of 64 at a time
    const int nent = (int)(bo_end - bo_cur);
#pragma unroll
    for (int t0 = 0; t0 < kR; t0 += 4) {
      if (64 * t0 < nent) {
#pragma unroll
        for (int t = t0; t < t0 + 4; ++t) {
          const int i = 64 * t + l;
          entry(C.x[t], C.p[t], i < nent, bo_cur + i);
        }
      }
    }
    for (int i0 = 64 * kR; i0 < nent; i0 += 64) {  // dense blocks: remaining rounds
      const int i = i0 + l;
      const bool valid = i < nent;
      const float x = valid ? a.vals[bo_cur + i] : 0.f;
      const uint32_t p = valid ? (uint32_t)a.pos[bo_cur + i] : 0u;
      entry(x, p, valid, bo_cur + i);
    }
    wave_sync();

    // 4. S^T += V^T-items^T . Y^T over the chunk's 32 columns (two k-steps of 16)
    if constexpr (kGrad) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        bf16x8 yb[2];
#pragma unroll
        for (int n = 0; n < 2; ++n)
          yb[n] = *reinterpret_cast<const bf16x8*>(Ys + (32 * n + li) * kYS + 16 * s2 + 8 * h);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const bf16x8 aw = *reinterpret_cast<const bf16x8*>(Vc + (32 * mt + li) * CWP + cc * 32 +
                                                             16 * s2 + 8 * h);
#pragma unroll
          for (int n = 0; n < 2; ++n)
            sacc[mt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, yb[n], sacc[mt][n], 0, 0, 0);
        }
      }
    }
    wave_sync();  // tile reads done before the next chunk overwrites them

    bo_cur = bo_end;
    bo_end = bo_nend;
    bo_nend = bo_nn;
  };

  Set A, B;
  if (rb_ok && gc_beg < gc_end) {
    bo_cur = a.boff[bb + gc_beg];
    bo_end = a.boff[bb + gc_beg + 1];
    bo_nend = a.boff[bb + min(gc_beg + 2, gc_end)];
    load_set(A, bo_cur);
    load_av(gc_beg);
  }
  for (int64_t gc = gc_beg; gc < gc_end; gc += 2) {
    step(gc, A, B);
    if (gc + 1 < gc_end) step(gc + 1, B, A);
  }

  if constexpr (kGrad) {
    // S^T accumulator: lane l holds row 32 n + li of the block, j = 32 mt + 8 (v/4) + 4h + v%4
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int64_t row = rb * 64 + 32 * n + li;
      if (row >= a.nrows) continue;
      float* sp = a.S + (cg * a.nrows + row) * a.RRP;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int j = mt * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
          if (j < a.RRP) sp[j] = sacc[mt][n][v];
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
}

int tile_k(int RR) { return (RR + 31) / 32 * 32; }

// column-tile width of the gradient pass: the bf16 V^T tile fills what the per-wave
// tiles leave of half the CU's LDS (two work-groups per CU)
int64_t tile_cw(int K) {
  int64_t budget = g_lds_max >= 2 * 81920 ? 81920 - 1024 : g_lds_max - 1024;
  int64_t cw = (budget - kXBytes - kYBytes) / (2 * K) - 8;
  cw = cw / 32 * 32;
  if (cw < 32) cw = 32;
  return cw;
}

template <int K, bool SPLIT>
static hipError_t launch_k(int mode, const TPassArgs& a, hipStream_t st) {
  const int64_t nwg = a.n_rg * a.n_cg;
  const size_t lds = tpass_lds(mode, K, a.CW);
  if ((int64_t)lds > g_lds_max) return hipErrorInvalidConfiguration;
  dim3 g((unsigned)nwg), b(256);
  switch (mode) {
    case kModeGrad: hipLaunchKernelGGL((k_tpass<K, kModeGrad, SPLIT>), g, b, lds, st, a); break;
    case kModeGradFast:
      hipLaunchKernelGGL((k_tpass<K, kModeGradFast, SPLIT>), g, b, lds, st, a);
      break;
    case kModeLS: hipLaunchKernelGGL((k_tpass<K, kModeLS, SPLIT>), g, b, lds, st, a); break;
    case kModeResid: hipLaunchKernelGGL((k_tpass<K, kModeResid, SPLIT>), g, b, lds, st, a); break;
    default: hipLaunchKernelGGL((k_tpass<K, kModeLoss, SPLIT>), g, b, lds, st, a); break;
  }
  return hipGetLastError();
}

template <int K>
static hipError_t launch_ks(int mode, const TPassArgs& a, hipStream_t st) {
  return (a.T_lo && a.V_lo) ? launch_k<K, true>(mode, a, st) : launch_k<K, false>(mode, a, st);
}

hipError_t launch_tpass(int mode, int K, const TPassArgs& a, hipStream_t st) {
  if (a.n_rg * a.n_cg <= 0 || a.n_chunks <= 0) return hipSuccess;
  // the grid and chunk walk must cover exactly the layout the pass indexes
  if ((a.T_lo == nullptr) != (a.V_lo == nullptr)) return hipErrorInvalidValue;
  if (a.CW % 32 != 0 || a.n_chpt != a.CW / 32 || a.cpg < 1 || a.n_rb > 4 * a.n_rg ||
      (int64_t)a.n_cg * a.cpg * a.n_chpt < a.n_chunks ||
      (int64_t)(a.n_cg - 1) * a.cpg * a.n_chpt >= a.n_chunks || a.n_chunks * 32 < a.ncols ||
      a.n_rb * 64 < a.nrows || a.RRP > K)
    return hipErrorInvalidValue;
  switch (K) {
    case 32: return launch_ks<32>(mode, a, st);
    case 64: return launch_ks<64>(mode, a, st);
    case 96: return launch_ks<96>(mode, a, st);
    case 128: return launch_ks<128>(mode, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace trd

// Matrix-core (MFMA) form of the fused entry passes: the BF16 precision form.
//
// The observed entries of a core-k matrix (rows = (i_k, first subchain modes), cols =
// the rest) are stored as bitmask tiles: one 32-bit mask per (64-row x 32-column block,
// lane) plus the observed values of the block, compacted in (lane, bit) order.  Lane l,
// bit b = 16 n + v of a block covers
//     row = 64 rb + 32 n + l % 32,
//     col = 32 ch + 8 (v / 4) + 4 (l / 32) + v % 4,
// which is exactly where the 32x32 MFMA output register v of n-tile n of lane l lands
// when the reconstruction is computed transposed:
//     Xhat^T (32 cols x 64 rows) = V^T-items (32 x K) . T-items^T (K x 64)    (Thm. 1)
// so each lane finds xhat of its own positions in its own accumulators.  With the same
// k ordering, the weighted residuals y = w e of a lane are already the B operand of
//     S^T (K x 64 rows) += V^T-items^T (K x 32 cols) . Y^T (32 cols x 64 rows)  (eq. 9)
// so no transpose through LDS is needed.  V^T items are bf16; products accumulate in
// FP32; e, w, y are FP32 (y is rounded to bf16 as an MFMA operand).
#include "trd_internal.h"

namespace trd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

static int grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even (finite)
  uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// position (row offset in block, column offset in block) of lane l, bit b
__host__ __device__ inline void tile_pos(int l, int b, int& r, int& c) {
  const int n = b >> 4, v = b & 15;
  r = 32 * n + (l & 31);
  c = 8 * (v >> 2) + 4 * (l >> 5) + (v & 3);
}

// ---------------------------------------------------------------- layout builder

struct TileArgs {
  const int64_t* rowoff;
  const int64_t* coloff;
  uint32_t* masks;
  int32_t* bcnt;
  int64_t* boff;
  int64_t* total;
  int64_t nrows, ncols, n_rbp, n_blocks;
  int CW, n_ch;
};

static TileArgs targs(const TLayout& L) {
  TileArgs a;
  a.rowoff = L.rowoff; a.coloff = L.coloff; a.masks = L.masks; a.bcnt = L.bcnt; a.boff = L.boff;
  a.total = L.total_dev; a.nrows = L.nrows; a.ncols = L.ncols; a.n_rbp = L.n_rg * 4;
  a.n_blocks = L.n_blocks; a.CW = L.CW; a.n_ch = L.n_ch;
  return a;
}

// block id = ((ct * n_rbp) + rb) * n_ch + ch; one wave per block
__device__ inline void block_coords(const TileArgs& a, int64_t b, int64_t& ct, int64_t& rb, int64_t& ch) {
  ch = b % a.n_ch;
  const int64_t t = b / a.n_ch;
  rb = t % a.n_rbp;
  ct = t / a.n_rbp;
}

__global__ __launch_bounds__(256) void k_tmask(TileArgs a, const uint8_t* __restrict__ mask) {
  const int64_t b = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  if (b >= a.n_blocks) return;
  int64_t ct, rb, ch;
  block_coords(a, b, ct, rb, ch);
  const int64_t col_lim = min(a.ncols, (ct + 1) * (int64_t)a.CW);
  uint32_t m = 0;
#pragma unroll 4
  for (int bit = 0; bit < 32; ++bit) {
    int r, c;
    tile_pos(l, bit, r, c);
    const int64_t row = rb * 64 + r, col = ct * (int64_t)a.CW + ch * 32 + c;
    if (row < a.nrows && col < col_lim && mask[a.rowoff[row] + a.coloff[col]]) m |= 1u << bit;
  }
  a.masks[b * 64 + l] = m;
  int cnt = __popc(m);
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (l == 0) a.bcnt[b] = cnt;
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

// order LDS accesses among the lanes of one wave (the staging area is per wave)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_excl_scan(int v, int l, int* total) {
  int incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (l >= o) incl += t;
  }
  *total = __shfl(incl, 63);
  return incl - v;
}

template <typename real>
__global__ __launch_bounds__(256) void k_tfill(TileArgs a, const real* __restrict__ X,
                                               float* __restrict__ vals) {
  const int64_t b = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  if (b >= a.n_blocks) return;
  int64_t ct, rb, ch;
  block_coords(a, b, ct, rb, ch);
  const uint32_t m = a.masks[b * 64 + l];
  int total;
  const int pre = wave_excl_scan(__popc(m), l, &total);
  int64_t p = a.boff[b] + pre;
  for (int bit = 0; bit < 32; ++bit) {
    if (!((m >> bit) & 1u)) continue;
    int r, c;
    tile_pos(l, bit, r, c);
    const int64_t row = rb * 64 + r, col = ct * (int64_t)a.CW + ch * 32 + c;
    vals[p++] = (float)X[a.rowoff[row] + a.coloff[col]];
  }
}

hipError_t launch_tile_build(const TLayout& L, const uint8_t* mask, const void* X, int dtype,
                             bool fill, hipStream_t st) {
  const unsigned nb = (unsigned)((L.n_blocks + 3) / 4);
  if (!fill) {
    hipLaunchKernelGGL(k_tmask, dim3(nb), dim3(256), 0, st, targs(L), mask);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, L.bcnt, L.n_blocks, L.boff,
                       L.total_dev);
  } else if (dtype == 0) {
    hipLaunchKernelGGL(k_tfill<float>, dim3(nb), dim3(256), 0, st, targs(L), (const float*)X, L.vals);
  } else {
    hipLaunchKernelGGL(k_tfill<double>, dim3(nb), dim3(256), 0, st, targs(L), (const double*)X, L.vals);
  }
  return hipGetLastError();
}

// f32 table [n][in_stride] -> bf16 table [n][K], zero padded
__global__ void k_table_bf16(const float* __restrict__ in, int64_t n, int in_stride, int K,
                             uint16_t* __restrict__ out) {
  const int64_t total = n * K;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / K;
    const int j = (int)(t % K);
    out[t] = j < in_stride ? f2bf(in[i * in_stride + j]) : (uint16_t)0;
  }
}

hipError_t launch_table_bf16(const float* in, int64_t n, int in_stride, int K, uint16_t* out,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_table_bf16, dim3(grid_for(n * K, 256)), dim3(256), 0, st, in, n, in_stride,
                     K, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- the MFMA pass

template <int K, int MODE>
__global__ __launch_bounds__(256, 2) void k_tpass(TPassArgs a) {
  constexpr int KS = K / 16;       // k-steps of the reconstruction MFMA
  constexpr int MT = K / 32;       // m-tiles of the gradient MFMA
  constexpr bool kGrad = MODE == kModeGrad || MODE == kModeGradFast;
  constexpr bool kStats = MODE == kModeGrad || MODE == kModeLoss;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int CWP = a.CW + 8;
  uint16_t* Vc = reinterpret_cast<uint16_t*>(smem_raw);                        // [K][CWP]
  float* stage = reinterpret_cast<float*>(smem_raw + (size_t)K * CWP * 2);     // [4][2048]

  const int64_t wg = blockIdx.x;
  const int64_t ct = wg / a.n_rg, g = wg % a.n_rg;
  const int64_t col0 = ct * (int64_t)a.CW;
  const int nct = (int)min((int64_t)a.CW, a.ncols - col0);

  // transposed column table of this tile: Vc[j][c] = V^T-item(col0 + c)[j]
  for (int i = threadIdx.x; i < a.CW * K; i += 256) {
    const int c = i / K, j = i % K;
    Vc[j * CWP + c] = c < nct ? a.V[(col0 + c) * K + j] : (uint16_t)0;
  }
  __syncthreads();

  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, h = l >> 5, li = l & 31;
  const int64_t rb = g * 4 + w;
  float* st = stage + w * 2048;

  // B operand of the reconstruction: this wave's 64 T items (and TH for the line search)
  bf16x8 tb[2][KS];
  bf16x8 thb[(MODE == kModeLS) ? 2 : 1][(MODE == kModeLS) ? KS : 1];
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const int64_t row = rb * 64 + 32 * n + li;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8 z = {};
      tb[n][s] = z;
      if (row < a.nrows)
        tb[n][s] = *reinterpret_cast<const bf16x8*>(a.T + row * K + s * 16 + h * 8);
      if constexpr (MODE == kModeLS) {
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

  floatx16 sacc[kGrad ? MT : 1][kGrad ? 2 : 1];
  if constexpr (kGrad) {
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int n = 0; n < 2; ++n) sacc[mt][n] = floatx16{};
  }
  float f0 = 0.f, f1 = 0.f, f2 = 0.f;

  // software pipeline over the tile's 32-column chunks: masks / block offsets two chunks
  // ahead, the next chunk's values and V^T-item operands one chunk ahead (registers)
  constexpr int kPV = 16;  // values per lane prefetched per chunk (1024 per wave)
  const float k2 = inv2s2 * 1.4426950408889634f;  // exp(-u) = 2^(-u log2 e)
  const int64_t bbase = (ct * a.n_rbp + rb) * a.n_ch;
  const int nch = a.n_ch;
  uint32_t m_cur = a.masks[bbase * 64 + l];
  uint32_t m_nxt = nch > 1 ? a.masks[(bbase + 1) * 64 + l] : 0u;
  int64_t bo_cur = a.boff[bbase], bo_nxt = a.boff[bbase + 1];
  int64_t bo_nxt2 = nch > 1 ? a.boff[bbase + 2] : bo_nxt;
  // The value array and the bf16 column table are allocated with slack (>= 1024 floats,
  // >= CW items) so these prefetches never need a bounds branch; slots past a chunk's
  // values are never selected, and column items past the tile are finite.
  float pv[kPV];
#pragma unroll
  for (int i = 0; i < kPV; ++i) pv[i] = a.vals[bo_cur + l + 64 * i];
  bf16x8 av[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    av[s] = *reinterpret_cast<const bf16x8*>(a.V + (col0 + li) * K + s * 16 + h * 8);

  for (int ch = 0; ch < nch; ++ch) {
    const int total = (int)(bo_nxt - bo_cur);
    // stage this chunk's values (registers, plus a direct copy of any overflow)
#pragma unroll
    for (int i = 0; i < kPV; ++i) st[l + 64 * i] = pv[i];
    for (int i = l + 64 * kPV; i < total; i += 64) st[i] = a.vals[bo_cur + i];
    // Xhat^T (and Q^T) for the 32 columns of this chunk
    floatx16 xacc[2] = {floatx16{}, floatx16{}};
    floatx16 qacc[(MODE == kModeLS) ? 2 : 1];
    if constexpr (MODE == kModeLS) { qacc[0] = floatx16{}; qacc[1] = floatx16{}; }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        xacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], tb[n][s], xacc[n], 0, 0, 0);
        if constexpr (MODE == kModeLS)
          qacc[n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[s], thb[n][s], qacc[n], 0, 0, 0);
      }
    }
    // prefetch the next chunk
    uint32_t m_nn = 0u;
    int64_t bo_nn = bo_nxt2;
    if (ch + 1 < nch) {
#pragma unroll
      for (int i = 0; i < kPV; ++i) pv[i] = a.vals[bo_nxt + l + 64 * i];
      const int c = (ch + 1) * 32 + li;
#pragma unroll
      for (int s = 0; s < KS; ++s)
        av[s] = *reinterpret_cast<const bf16x8*>(a.V + (col0 + c) * K + s * 16 + h * 8);
      if (ch + 2 < nch) {
        m_nn = a.masks[(bbase + ch + 2) * 64 + l];
        bo_nn = a.boff[bbase + ch + 3];
      }
    }
    const uint32_t m = m_cur;
    int wtot;
    const int pre = wave_excl_scan(__popc(m), l, &wtot);
    const int64_t boff = bo_cur;
    wave_sync();  // staged values of this wave visible to all its lanes

    bf16x8 yv[kGrad ? 2 : 1][kGrad ? 2 : 1];  // [n][s2]: y of registers v = 8 s2 .. 8 s2 + 7
#pragma unroll
    for (int n = 0; n < 2; ++n) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int bit = n * 16 + v;
        const bool obs = (m >> bit) & 1u;
        const float xh = xacc[n][v];
        float x = xh;
        // idx <= this wave's value count <= 2048: the read is always in the staging area,
        // so it is issued unconditionally and the result selected
        const int idx = pre + __popc(m & ((1u << bit) - 1u));
        const float ld = st[idx];
        if (obs) x = ld;
        const float e = x - xh;
        const float uu = e * e * inv2s2;
        const float wgt = ls_limit ? 1.f : __builtin_amdgcn_exp2f(-(e * e * k2));
        if constexpr (kGrad) yv[n][v >> 3][v & 7] = (__bf16)(wgt * e);
        if constexpr (MODE == kModeLS) {
          const float q = qacc[n][v];
          f0 = fmaf(obs ? wgt * q : 0.f, q, f0);
        }
        if constexpr (MODE == kModeResid) {
          if (obs) a.resid[boff + idx] = fabsf(e);
        }
        if constexpr (kStats) {
          if (obs) {
            float lo;
            if (ls_limit) lo = 0.5f * e * e;
            else if (uu < 0.0625f) {
              float p = fmaf(uu, 1.0f / 120.0f, -1.0f / 24.0f);
              p = fmaf(uu, p, 1.0f / 6.0f);
              p = fmaf(uu, p, -0.5f);
              p = fmaf(uu, p, 1.0f);
              lo = sig2 * uu * p;
            } else {
              lo = sig2 * (1.f - wgt);
            }
            f0 += lo;
            f1 = fmaf(wgt * e, e, f1);
            f2 += 1.f;
          }
        }
      }
    }

    if constexpr (kGrad) {
      // S^T += V^T-items^T . Y^T; k slots of step s2: columns 16 s2 + 4h + {0..3} and
      // 16 s2 + 8 + 4h + {0..3}, i.e. this lane's y registers v = 8 s2 .. 8 s2 + 7
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int j = mt * 32 + li;
          const int cbase = ch * 32 + 16 * s2 + 4 * h;
          const bf16x4 lo = *reinterpret_cast<const bf16x4*>(Vc + j * CWP + cbase);
          const bf16x4 hi = *reinterpret_cast<const bf16x4*>(Vc + j * CWP + cbase + 8);
          const bf16x8 aw = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
          for (int n = 0; n < 2; ++n)
            sacc[mt][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw, yv[n][s2], sacc[mt][n], 0, 0, 0);
        }
      }
    }
    wave_sync();  // all lanes done with the staging area before the next chunk refills it
    m_cur = m_nxt;
    m_nxt = m_nn;
    bo_cur = bo_nxt;
    bo_nxt = bo_nxt2;
    bo_nxt2 = bo_nn;
  }

  if constexpr (kGrad) {
    // S^T accumulator: lane l holds row 32 n + li of the block, j = 32 mt + 8 (v/4) + 4h + v%4
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int64_t row = rb * 64 + 32 * n + li;
      if (row >= a.nrows) continue;
      float* sp = a.S + (ct * a.nrows + row) * a.RRP;
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

int64_t tile_cw(int K) {
  // LDS: K x (CW + 8) bf16 column table + 4 x 2048 floats of staging; two groups per CU
  int64_t budget = g_lds_max >= 2 * 65536 ? 65536 : 61440;
  if (budget > g_lds_max - 1024) budget = g_lds_max - 1024;
  int64_t cw = (budget - 4 * 2048 * 4) / (2 * K) - 8;
  cw = cw / 32 * 32;
  if (cw < 32) cw = 32;
  return cw;
}

template <int K>
static hipError_t launch_k(int mode, const TPassArgs& a, hipStream_t st) {
  const int64_t nwg = a.n_rg * a.n_ct;
  const size_t lds = (size_t)K * (a.CW + 8) * 2 + 4 * 2048 * 4;
  dim3 g((unsigned)nwg), b(256);
  switch (mode) {
    case kModeGrad: hipLaunchKernelGGL((k_tpass<K, kModeGrad>), g, b, lds, st, a); break;
    case kModeGradFast: hipLaunchKernelGGL((k_tpass<K, kModeGradFast>), g, b, lds, st, a); break;
    case kModeLS: hipLaunchKernelGGL((k_tpass<K, kModeLS>), g, b, lds, st, a); break;
    case kModeResid: hipLaunchKernelGGL((k_tpass<K, kModeResid>), g, b, lds, st, a); break;
    default: hipLaunchKernelGGL((k_tpass<K, kModeLoss>), g, b, lds, st, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_tpass(int mode, int K, const TPassArgs& a, hipStream_t st) {
  if (a.n_rg * a.n_ct <= 0) return hipSuccess;
  switch (K) {
    case 32: return launch_k<32>(mode, a, st);
    case 64: return launch_k<64>(mode, a, st);
    case 96: return launch_k<96>(mode, a, st);
    case 128: return launch_k<128>(mode, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace trd

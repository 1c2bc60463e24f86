// Observed-entry layouts (sliced ELL per core-k matrix) and RStS index sampling.
#include "trd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace trd {

// ---------------------------------------------------------------- small utilities

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

static int grid_for(int64_t n, int threads, int cap = 4096) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

// out[i] = in[i] clamped into [0, dim); any clamped entry sets TRD_FLAG_CLAMPED in *bad
__global__ void k_copy_clamp(const int32_t* __restrict__ in, int64_t n, int64_t dim,
                             int32_t* __restrict__ out, uint32_t* bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = in[i];
    if (v < 0 || v >= dim) {
      atomicOr(bad, TRD_FLAG_CLAMPED_BIT);
      v = v < 0 ? 0 : dim - 1;
    }
    out[i] = (int32_t)v;
  }
}

hipError_t launch_copy_clamp(const int32_t* in, int64_t n, int64_t dim, int32_t* out,
                             uint32_t* bad, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_clamp, dim3(grid_for(n, 256)), dim3(256), 0, st, in, n, dim, out, bad);
  return hipGetLastError();
}

__global__ void k_accum_i64(int64_t* dst, const int64_t* src) { *dst += *src; }

hipError_t launch_accum_i64(int64_t* dst, const int64_t* src, hipStream_t st) {
  hipLaunchKernelGGL(k_accum_i64, dim3(1), dim3(1), 0, st, dst, src);
  return hipGetLastError();
}

// Zero a buffer with a kernel (no memset node, so it is safe inside captured graphs).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  // callers only zero 4-byte-multiple buffers
  int64_t n = (int64_t)(bytes / 4);
  hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256)), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------- offsets
// out[t] = sum_j idx_j(t) * stride_j, t decoded little-endian over the mode counts.

__global__ void k_offsets(ModeSet ms, int64_t n, int64_t* out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = t, off = 0;
    for (int j = 0; j < ms.n; ++j) {
      int64_t d = rem % ms.count[j];
      rem /= ms.count[j];
      int64_t idx = ms.list[j] ? (int64_t)ms.list[j][d] : d;
      off += idx * ms.stride[j];
    }
    out[t] = off;
  }
}

hipError_t launch_offsets(const ModeSet& ms, int64_t n, int64_t* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_offsets, dim3(grid_for(n, 256)), dim3(256), 0, st, ms, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- count / slices / scan / fill
// Work-group w <-> (column tile ct, row group g) with w = ct * n_rg + g; thread t of the
// group owns row g*256 + t; slice id = w*4 + t/64, lane = t%64.

struct LayoutArgs {
  const int64_t* rowoff;
  const int64_t* coloff;
  int32_t* counts;
  int32_t* slice_len;
  int64_t* slice_off;
  int64_t* total;
  int64_t* nobs;
  int64_t nrows, ncols, n_rg, n_slices;
  int ct_w, n_ct;
};

static LayoutArgs largs(const Layout& L) {
  LayoutArgs a;
  a.rowoff = L.rowoff; a.coloff = L.coloff; a.counts = L.counts; a.slice_len = L.slice_len;
  a.slice_off = L.slice_off; a.total = L.total_dev; a.nobs = L.nobs_dev;
  a.nrows = L.nrows; a.ncols = L.ncols; a.n_rg = L.n_rg; a.n_slices = L.n_slices;
  a.ct_w = L.ct_w; a.n_ct = L.n_ct;
  return a;
}

// One wave per (column tile, row): lanes stride over the tile's columns, so 64 mask
// reads are in flight per step; counts in fixed column order.
__global__ __launch_bounds__(256) void k_count(LayoutArgs a, const uint8_t* __restrict__ mask) {
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;  // global wave
  const int lane = threadIdx.x & 63;
  const int64_t nrows_pad = a.n_rg * kRowsPerWG;
  if (gw >= nrows_pad * a.n_ct) return;
  const int64_t ct = gw / nrows_pad, row = gw % nrows_pad;
  int cnt = 0;
  if (row < a.nrows) {
    const int64_t col0 = ct * a.ct_w;
    const int64_t nct = min((int64_t)a.ct_w, a.ncols - col0);
    const int64_t ro = a.rowoff[row];
    for (int64_t c = lane; c < nct; c += 64) cnt += mask[ro + a.coloff[col0 + c]] != 0;
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  }
  if (lane == 0) a.counts[ct * nrows_pad + row] = cnt;
}

hipError_t launch_count(const Layout& L, const uint8_t* mask, hipStream_t st) {
  const int64_t waves = L.n_rg * kRowsPerWG * L.n_ct;
  hipLaunchKernelGGL(k_count, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, largs(L), mask);
  return hipGetLastError();
}

__global__ void k_slices(LayoutArgs a) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.n_slices) return;
  const int64_t w = s / 4, wave = s % 4;
  const int64_t ct = w / a.n_rg, g = w % a.n_rg;
  const int32_t* c = a.counts + ct * (a.n_rg * kRowsPerWG) + g * kRowsPerWG + wave * kWave;
  int mx = 0;
  long long sum = 0;
  for (int l = 0; l < kWave; ++l) {
    mx = max(mx, c[l]);
    sum += c[l];
  }
  a.slice_len[s] = (mx + kGroup - 1) / kGroup * kGroup;
  if (sum) atomicAdd((unsigned long long*)a.nobs, (unsigned long long)sum);
}

hipError_t launch_slices(const Layout& L, hipStream_t st) {
  hipLaunchKernelGGL(k_slices, dim3(grid_for(L.n_slices, 256, 1 << 30)), dim3(256), 0, st,
                     largs(L));
  return hipGetLastError();
}

// Exclusive scan of slice sizes (len * 64) by one work-group, in fixed order.
__global__ __launch_bounds__(1024) void k_scan(LayoutArgs a) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < a.n_slices; base += 1024) {
    int64_t i = base + threadIdx.x;
    int64_t v = i < a.n_slices ? (int64_t)a.slice_len[i] * kWave : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      int64_t add = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < a.n_slices) a.slice_off[i] = carry + buf[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.slice_off[a.n_slices] = carry;
    *a.total = carry;
  }
}

hipError_t launch_scan(const Layout& L, hipStream_t st) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, largs(L));
  return hipGetLastError();
}

// One wave per (column tile, row): the row's observed entries are written in column
// order to the row's ELL lane (row % 64) of its slice, then padded to the slice length.
template <typename real>
__global__ __launch_bounds__(256) void k_fill(LayoutArgs a, const uint8_t* __restrict__ mask,
                                              const real* __restrict__ X, real* __restrict__ vals,
                                              uint16_t* __restrict__ cols) {
  const int64_t gw = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t nrows_pad = a.n_rg * kRowsPerWG;
  if (gw >= nrows_pad * a.n_ct) return;
  const int64_t ct = gw / nrows_pad, row = gw % nrows_pad;
  const int64_t g = row / kRowsPerWG, in_g = row % kRowsPerWG;
  const int64_t sid = (ct * a.n_rg + g) * 4 + in_g / kWave;
  const int ell_lane = (int)(in_g % kWave);
  const int64_t base = a.slice_off[sid];
  const int len = a.slice_len[sid];
  int t = 0;  // entries written so far (wave uniform)
  if (row < a.nrows) {
    const int64_t col0 = ct * a.ct_w;
    const int64_t nct = min((int64_t)a.ct_w, a.ncols - col0);
    const int64_t ro = a.rowoff[row];
    for (int64_t c0 = 0; c0 < nct; c0 += 64) {
      const int64_t c = c0 + lane;
      int64_t off = 0;
      bool obs = false;
      if (c < nct) {
        off = ro + a.coloff[col0 + c];
        obs = mask[off] != 0;
      }
      const unsigned long long bal = __ballot(obs);
      if (obs) {
        const int pos = t + __popcll(bal & ((1ull << lane) - 1ull));
        const int64_t slot = slot_of(base, pos, ell_lane);
        vals[slot] = X[off];
        cols[slot] = (uint16_t)c;
      }
      t += __popcll(bal);
    }
  }
  for (int p = t + lane; p < len; p += 64) {
    const int64_t slot = slot_of(base, p, ell_lane);
    vals[slot] = real(0);
    cols[slot] = kPad;
  }
}

hipError_t launch_fill(const Layout& L, const uint8_t* mask, const void* X, int dtype,
                       hipStream_t st) {
  const int64_t waves = L.n_rg * kRowsPerWG * L.n_ct;
  const unsigned nb = (unsigned)((waves + 3) / 4);
  if (dtype == 0)
    hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(256), 0, st, largs(L), mask, (const float*)X,
                       (float*)L.vals, L.cols);
  else
    hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(256), 0, st, largs(L), mask, (const double*)X,
                       (double*)L.vals, L.cols);
  return hipGetLastError();
}

// max |x| over the observed entries of a layout (non-negative doubles compare like
// their bit patterns, so an integer atomic max is exact and order independent)
template <typename real>
__global__ void k_max_abs(const real* vals, const uint16_t* cols, const int64_t* total,
                          double* out) {
  const int64_t n = *total;
  unsigned long long best = 0ull;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (cols[i] != kPad) {
      double v = fabs((double)vals[i]);
      unsigned long long b = (unsigned long long)__double_as_longlong(v);
      best = b > best ? b : best;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long other = __shfl_xor(best, o);
    best = other > best ? other : best;
  }
  if ((threadIdx.x & 63) == 0 && best) atomicMax((unsigned long long*)out, best);
}

hipError_t launch_max_abs_observed(const Layout& L, int dtype, double* out, hipStream_t st) {
  hipError_t e = launch_zero(out, sizeof(double), st);
  if (e != hipSuccess) return e;
  if (dtype == 0)
    hipLaunchKernelGGL(k_max_abs<float>, dim3(1024), dim3(256), 0, st, (const float*)L.vals,
                       L.cols, L.total_dev, out);
  else
    hipLaunchKernelGGL(k_max_abs<double>, dim3(1024), dim3(256), 0, st, (const double*)L.vals,
                       L.cols, L.total_dev, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- RStS sampling
// SplitMix64 in counter form, Lemire bounded draws, Floyd subsets (integer only).

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t counter_u64(uint64_t key, uint64_t c) {
  return mix64(key + (c + 1ull) * 0x9E3779B97F4A7C15ull);
}
// n in [1, 2^31): the rejection threshold (2^32 - n) mod n in 32-bit arithmetic
__device__ uint64_t bounded(uint64_t key, uint64_t* ctr, uint64_t n) {
  const uint32_t n32 = (uint32_t)n;
  const uint32_t threshold = (0u - n32) % n32;
  for (;;) {
    const uint32_t x = (uint32_t)(counter_u64(key, (*ctr)++) >> 32);
    const uint64_t m = (uint64_t)x * n32;
    if ((uint32_t)m >= threshold) return m >> 32;
  }
}

struct SampleArgs {
  uint64_t seed;
  int t, k, N;
  int64_t dims[kMaxN];
  int32_t sizes[kMaxN];
  int32_t* out[kMaxN];
};

// Floyd's subset for mode j of one update per block.  For I_j up to kSampleBits the chosen
// set is a bitmap in LDS (membership in O(1), set by thread 0 in Floyd's order), and the
// sorted list is written by the whole block from the bitmap: word counts, a block scan,
// then each thread's bits in order.  Larger modes keep the sorted list in global memory.
constexpr int kSampleWords = 8192;                 // 32 KiB of LDS
constexpr int64_t kSampleBits = 32 * (int64_t)kSampleWords;

__global__ __launch_bounds__(256) void k_sample(SampleArgs a) {
  __shared__ uint32_t bits[kSampleWords];
  __shared__ int32_t part[4];  // per-wave totals of the 256-thread block
  const int j = blockIdx.x;
  const int64_t n = a.dims[j];
  int32_t* o = a.out[j];
  if (j == a.k || (int64_t)a.sizes[j] >= n) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) o[i] = (int32_t)i;
    return;
  }
  const int64_t s = a.sizes[j];
  uint64_t key = counter_u64(a.seed ^ 0x5253545300000000ull, (uint64_t)a.t);
  key = counter_u64(key, (uint64_t)a.k);
  key = counter_u64(key, (uint64_t)j);
  if (n <= kSampleBits) {
    const int nw = (int)((n + 31) / 32);
    for (int w = threadIdx.x; w < nw; w += blockDim.x) bits[w] = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t ctr = 0;
      for (int64_t jj = n - s; jj < n; ++jj) {
        const int64_t tv = (int64_t)bounded(key, &ctr, (uint64_t)(jj + 1));
        const bool taken = (bits[tv >> 5] >> (tv & 31)) & 1u;
        const int64_t v = taken ? jj : tv;  // jj itself is never taken yet
        bits[v >> 5] |= 1u << (v & 31);
      }
    }
    __syncthreads();
    // each thread owns a contiguous run of words: count, exclusive scan, write in order
    const int per = (nw + (int)blockDim.x - 1) / (int)blockDim.x;
    const int w0 = min(nw, (int)threadIdx.x * per), w1 = min(nw, w0 + per);
    int cnt = 0;
    for (int w = w0; w < w1; ++w) cnt += __popc(bits[w]);
    // exclusive block scan: inclusive within each wave by shuffles, then the wave totals
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(inc, o);
      if (lane >= o) inc += v;
    }
    if (lane == 63) part[wv] = inc;
    __syncthreads();
    int pos = inc - cnt;
    for (int i = 0; i < wv; ++i) pos += part[i];
    for (int w = w0; w < w1; ++w) {
      uint32_t b = bits[w];
      while (b) {
        const int q = __ffs(b) - 1;
        o[pos++] = w * 32 + q;
        b &= b - 1u;
      }
    }
    return;
  }
  if (threadIdx.x != 0) return;
  uint64_t ctr = 0;
  int64_t m = 0;  // current size of the sorted set in o[0..m)
  for (int64_t jj = n - s; jj < n; ++jj) {
    int64_t tv = (int64_t)bounded(key, &ctr, (uint64_t)(jj + 1));
    // membership by binary search
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (o[mid] < tv) lo = mid + 1; else hi = mid;
    }
    int64_t v = (lo < m && o[lo] == tv) ? jj : tv;
    // jj exceeds every element so far, so it goes to the end
    int64_t pos = (v == jj) ? m : lo;
    for (int64_t q = m; q > pos; --q) o[q] = o[q - 1];
    o[pos] = (int32_t)v;
    ++m;
  }
}

// ---------------------------------------------------------------- uniform row sampling
// J rows of the subchain unfolding of core k, drawn independently and uniformly with
// replacement: sample n takes index bounded(u(key_j, n), 0, I_j) of every mode j != k, with
// key_j = u(u(u(seed ^ "UROW", t), k), j), and u(key, c) the counter form of SplitMix64.
// Out: the tensor offset of the sampled mode-k fibre (at i_k = 0) and/or the row index
// (little-endian over the cyclic modes k+1, ..., k-1).

struct RowSampleArgs {
  uint64_t seed;
  int t, k, N;
  int64_t dims[kMaxN];
  int64_t strides[kMaxN];
  int64_t J;
  int64_t* off;
  int64_t* row;
};

__global__ __launch_bounds__(256) void k_sample_rows(RowSampleArgs a) {
  const uint64_t base = counter_u64(counter_u64(a.seed ^ 0x55524F5700000000ull, (uint64_t)a.t), (uint64_t)a.k);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.J;
       n += (int64_t)gridDim.x * blockDim.x) {
    int64_t off = 0, row = 0, rs = 1;
    for (int s = 1; s < a.N; ++s) {
      const int j = (a.k + s) % a.N;
      uint64_t ctr = 0;
      const int64_t i = (int64_t)bounded(counter_u64(counter_u64(base, (uint64_t)j), (uint64_t)n), &ctr,
                                         (uint64_t)a.dims[j]);
      off += i * a.strides[j];
      row += i * rs;
      rs *= a.dims[j];
    }
    if (a.off) a.off[n] = off;
    if (a.row) a.row[n] = row;
  }
}

// ---------------------------------------------------------------- leverage-score row sampling
// TRALS-S's sampler for the ablation of Sec. 6.1.  Per mode j != k: C = Z_(2)^T Z_(2) of the
// core's mode-2 unfolding (slice i is the contiguous r_j r_{j+1} vector z_i), its ridge
// inverse (the scaled-direction inverse kernel), the leverage l(i) = z_i^T C^{-1} z_i and
// the running sums of l in slice order.  Sample n then draws, per mode, the uniform
// u = (u64 >> 11) 2^-53 of u(key_j, n), key_j = u(u(u(seed ^ "LEVE", t), k), j), and takes the
// first slice whose running sum exceeds u * total; its probability p multiplies over the
// modes and the sample's weight is 1 / (J p).  A zero core (its Gram is not positive
// definite, the inverse comes back zero, every leverage is 0) is sampled uniformly.

template <typename real>
__global__ __launch_bounds__(256) void k_core_gram(const real* __restrict__ Z, int64_t I, int R,
                                                   double* __restrict__ C) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R * R) return;
  const int p = t / R, q = t % R;
  double acc = 0.0;
  for (int64_t i = 0; i < I; ++i) acc = fma((double)Z[i * R + p], (double)Z[i * R + q], acc);
  C[t] = acc;
}

// one wave per slice: lane p forms (C^{-1} z)_p for p = lane, lane + 64, ...; the wave sums
// z_p (C^{-1} z)_p
template <typename real>
__global__ __launch_bounds__(256) void k_leverage(const real* __restrict__ Z, int64_t I, int R,
                                                  const double* __restrict__ Ci, double* __restrict__ lev) {
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= I) return;  // whole waves (no barrier below)
  const real* z = Z + i * R;
  double acc = 0.0;
  for (int p = lane; p < R; p += 64) {
    double y = 0.0;
    for (int q = 0; q < R; ++q) y = fma(Ci[p * R + q], (double)z[q], y);
    acc = fma((double)z[p], y, acc);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) lev[i] = acc;
}

// running sums of lev in slice order, one work-group: each thread sums a contiguous run
// sequentially, then adds the totals of the runs before it
__global__ __launch_bounds__(256) void k_lev_scan(const double* __restrict__ lev, int64_t I,
                                                  double* __restrict__ cdf) {
  __shared__ double tot[256];
  const int64_t per = (I + 255) / 256;
  const int64_t b = threadIdx.x * per, e = min(I, b + per);
  double run = 0.0;
  for (int64_t i = b; i < e; ++i) run += lev[i];
  tot[threadIdx.x] = run;
  __syncthreads();
  double off = 0.0;
  for (int t = 0; t < (int)threadIdx.x; ++t) off += tot[t];
  run = off;
  for (int64_t i = b; i < e; ++i) {
    run += lev[i];
    cdf[i] = run;
  }
}

struct LevArgs {
  uint64_t seed;
  int t, k, N;
  int64_t dims[kMaxN];
  int64_t strides[kMaxN];
  const double* lev[kMaxN];
  const double* cdf[kMaxN];
  int64_t J;
  int64_t* off;
  int64_t* row;
  double* weight;
};

__global__ __launch_bounds__(256) void k_sample_leverage(LevArgs a) {
  const uint64_t base = counter_u64(counter_u64(a.seed ^ 0x4C45564500000000ull, (uint64_t)a.t), (uint64_t)a.k);
  for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.J;
       n += (int64_t)gridDim.x * blockDim.x) {
    int64_t off = 0, row = 0, rs = 1;
    double p = 1.0;
    for (int s = 1; s < a.N; ++s) {
      const int j = (a.k + s) % a.N;
      const int64_t I = a.dims[j];
      const double* cdf = a.cdf[j];
      const double total = cdf[I - 1];
      const double u = (double)(counter_u64(counter_u64(base, (uint64_t)j), (uint64_t)n) >> 11) * 0x1p-53;
      int64_t i;
      if (total > 0.0) {
        const double target = u * total;
        int64_t lo = 0, hi = I;  // first slice whose running sum exceeds the target
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (cdf[mid] > target) hi = mid; else lo = mid + 1;
        }
        i = lo < I ? lo : I - 1;
        p *= a.lev[j][i] / total;
      } else {  // a zero core has no leverage: its index is drawn uniformly
        i = (int64_t)floor(u * (double)I);
        i = i < I ? i : I - 1;
        p *= 1.0 / (double)I;
      }
      off += i * a.strides[j];
      row += i * rs;
      rs *= I;
    }
    if (a.off) a.off[n] = off;
    if (a.row) a.row[n] = row;
    a.weight[n] = 1.0 / ((double)a.J * p);
  }
}

hipError_t launch_leverage_mode(int dtype, const void* Z, int64_t I, int R, double* C, double* Ci,
                                double lambda_rel, double* lev, double* cdf, uint32_t* flags,
                                hipStream_t st) {
  const unsigned gb = (unsigned)((R * R + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_core_gram<float>, dim3(gb), dim3(256), 0, st, (const float*)Z, I, R, C);
  else
    hipLaunchKernelGGL(k_core_gram<double>, dim3(gb), dim3(256), 0, st, (const double*)Z, I, R, C);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_inverse(C, Ci, R, lambda_rel, flags, st);
  if (e != hipSuccess) return e;
  const unsigned lb = (unsigned)((I + 3) / 4);
  if (dtype == 0)
    hipLaunchKernelGGL(k_leverage<float>, dim3(lb), dim3(256), 0, st, (const float*)Z, I, R, Ci, lev);
  else
    hipLaunchKernelGGL(k_leverage<double>, dim3(lb), dim3(256), 0, st, (const double*)Z, I, R, Ci, lev);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lev_scan, dim3(1), dim3(256), 0, st, lev, I, cdf);
  return hipGetLastError();
}

hipError_t launch_sample_leverage(uint64_t seed, int t, int k, int N, const int64_t* dims,
                                  const double* const* lev, const double* const* cdf, int64_t J,
                                  int64_t* off, int64_t* row, double* weight, hipStream_t st) {
  if (J <= 0) return hipSuccess;
  LevArgs a;
  a.seed = seed; a.t = t; a.k = k; a.N = N; a.J = J; a.off = off; a.row = row; a.weight = weight;
  int64_t stride = 1;
  for (int j = 0; j < kMaxN; ++j) {
    a.dims[j] = j < N ? dims[j] : 1;
    a.strides[j] = stride;
    if (j < N) stride *= dims[j];
    a.lev[j] = j < N ? lev[j] : nullptr;
    a.cdf[j] = j < N ? cdf[j] : nullptr;
  }
  const int64_t blocks = std::min<int64_t>((J + 255) / 256, 8192);
  hipLaunchKernelGGL(k_sample_leverage, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- masks and outliers
// Per-entry (or per-tile) Bernoulli draws from the same counter generator: an event of
// probability p happens when the draw is below floor(p 2^64) (integer compare; p >= 1:
// always).  Keys: u(seed ^ "MASK", 0) for the mask, 1 for the outlier selection, 2 for the
// per-entry uniform u = (draw >> 11) 2^-53 in [0, 1).

struct MaskArgs {
  uint64_t key_m, key_o, key_u;
  uint64_t thr_m, thr_o;
  int all_m, all_o, none_o;
  int N, block;
  int64_t dims[kMaxN];
  int64_t n;
  int64_t nbh, nbw;
  uint8_t* mask;
  uint8_t* sel;
  double* u;
};

__global__ __launch_bounds__(256) void k_sample_mask(MaskArgs a) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < a.n;
       l += (int64_t)gridDim.x * blockDim.x) {
    uint64_t draw_at = (uint64_t)l;
    if (a.block > 0) {  // tile of modes 0 and 1 at this index of modes 3.. (mode 2 shared)
      int64_t rem = l;
      const int64_t i0 = rem % a.dims[0];
      rem /= a.dims[0];
      const int64_t i1 = rem % a.dims[1];
      rem /= a.dims[1];
      if (a.N >= 3) rem /= a.dims[2];
      draw_at = (uint64_t)(i0 / a.block + a.nbh * (i1 / a.block + a.nbw * rem));
    }
    const bool obs = a.all_m || counter_u64(a.key_m, draw_at) < a.thr_m;
    a.mask[l] = obs ? 1 : 0;
    if (a.sel) {
      const bool pick = obs && !a.none_o && (a.all_o || counter_u64(a.key_o, (uint64_t)l) < a.thr_o);
      a.sel[l] = pick ? 1 : 0;
    }
    if (a.u) a.u[l] = (double)(counter_u64(a.key_u, (uint64_t)l) >> 11) * 0x1p-53;
  }
}

// floor(p 2^64) for 0 < p < 1 (exact: p 2^64 is a double with the same mantissa)
static uint64_t prob_threshold(double p) { return (uint64_t)ldexp(p, 64); }

hipError_t launch_sample_mask(uint64_t seed, int N, const int64_t* dims, double rho, int block,
                              double frac, uint8_t* mask, uint8_t* sel, double* u, hipStream_t st) {
  MaskArgs a;
  memset(&a, 0, sizeof(a));
  const uint64_t base = seed ^ 0x4D41534B00000000ull;  // "MASK"
  auto host_u = [](uint64_t key, uint64_t c) {
    uint64_t z = key + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  a.key_m = host_u(base, 0);
  a.key_o = host_u(base, 1);
  a.key_u = host_u(base, 2);
  a.all_m = rho >= 1.0;
  a.thr_m = (rho > 0.0 && rho < 1.0) ? prob_threshold(rho) : 0;
  a.all_o = frac >= 1.0;
  a.none_o = !(frac > 0.0);
  a.thr_o = (frac > 0.0 && frac < 1.0) ? prob_threshold(frac) : 0;
  a.N = N;
  a.block = block;
  a.n = 1;
  for (int j = 0; j < N; ++j) {
    a.dims[j] = dims[j];
    a.n *= dims[j];
  }
  if (block > 0) {
    a.nbh = (dims[0] + block - 1) / block;
    a.nbw = (dims[1] + block - 1) / block;
  }
  a.mask = mask;
  a.sel = sel;
  a.u = u;
  if (a.n <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>((a.n + 255) / 256, (int64_t)g_num_cu * 64);
  hipLaunchKernelGGL(k_sample_mask, dim3((unsigned)g), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sample_rows(uint64_t seed, int t, int k, int N, const int64_t* dims, int64_t J,
                              int64_t* off, int64_t* row, hipStream_t st) {
  if (J <= 0) return hipSuccess;
  RowSampleArgs a;
  a.seed = seed; a.t = t; a.k = k; a.N = N; a.J = J; a.off = off; a.row = row;
  int64_t stride = 1;
  for (int j = 0; j < kMaxN; ++j) {
    a.dims[j] = j < N ? dims[j] : 1;
    a.strides[j] = stride;
    if (j < N) stride *= dims[j];
  }
  const int64_t blocks = std::min<int64_t>((J + 255) / 256, 8192);
  hipLaunchKernelGGL(k_sample_rows, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sample(uint64_t seed, int t, int k, int N, const int64_t* dims,
                         const int32_t* sizes, int32_t* const* out, hipStream_t st) {
  SampleArgs a;
  a.seed = seed; a.t = t; a.k = k; a.N = N;
  for (int j = 0; j < kMaxN; ++j) {
    a.dims[j] = j < N ? dims[j] : 1;
    a.sizes[j] = j < N ? sizes[j] : 1;
    a.out[j] = j < N ? out[j] : nullptr;
  }
  hipLaunchKernelGGL(k_sample, dim3(N), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace trd

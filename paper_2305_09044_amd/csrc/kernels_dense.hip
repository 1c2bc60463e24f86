// Small dense FP64 pieces of the update: FGMC factors and ring product (eq. 13),
// the scaled direction (eq. 10) through an in-LDS Gauss-Jordan inverse of the SPD
// matrix G + lambda I, the exact line-search step (eq. 12), the core update (eq. 11),
// the convergence matrix of Alg. 1, the weights of eq. (7) and TR reconstruction (Def. 1).
#include "trd_internal.h"

#include <cmath>
#include <cstring>

namespace trd {

static int grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// ---------------------------------------------------------------- FGMC

// K[(al*r0 + al2), (be*r1 + be2)] = sum_i Z(i)[al, be] * Z(i)[al2, be2]
// one wave per output element; lanes stride over i, then a fixed-order wave reduction.
// idx (nullptr: slices 0..I-1) lists the I slices to sum: the factor of a sampled core
template <typename real>
__global__ __launch_bounds__(256) void k_kron(const real* __restrict__ Z, int r0, int64_t I, int r1,
                                              const int32_t* __restrict__ idx,
                                              double* __restrict__ K) {
  const int64_t n = (int64_t)r0 * r0 * r1 * r1;
  const int cols = r1 * r1;
  const int lane = threadIdx.x & 63;
  const int64_t t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= n) return;
  const int rr = (int)(t / cols), cc = (int)(t % cols);
  const int al = rr / r0, al2 = rr % r0, be = cc / r1, be2 = cc % r1;
  const int64_t sl = (int64_t)r0 * r1;
  double s = 0.0;
  for (int64_t i = lane; i < I; i += 64) {
    const real* zi = Z + (idx ? (int64_t)idx[i] : i) * sl;
    s = fma((double)zi[al + r0 * be], (double)zi[al2 + r0 * be2], s);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) K[t] = s;
}

hipError_t launch_kron_factor(int dtype, const void* Z, int r0, int64_t I, int r1, double* K,
                              hipStream_t st, const int32_t* idx) {
  const int64_t n = (int64_t)r0 * r0 * r1 * r1;
  const unsigned nb = (unsigned)((n + 3) / 4);
  if (dtype == 0)
    hipLaunchKernelGGL(k_kron<float>, dim3(nb), dim3(256), 0, st, (const float*)Z, r0, I, r1, idx, K);
  else
    hipLaunchKernelGGL(k_kron<double>, dim3(nb), dim3(256), 0, st, (const double*)Z, r0, I, r1, idx,
                       K);
  return hipGetLastError();
}

// C = A (m x kk) @ B (kk x n), row-major FP64.  With r_k > 0 the product is the last
// factor of the FGMC ring (m = r_k1^2, n = r_k^2) and is stored realigned as G:
// element (b r_k1 + b2, a r_k + a2) goes to G[(a + b r_k), (a2 + b2 r_k)].
__global__ void k_gemm64(const double* __restrict__ A, const double* __restrict__ B,
                         double* __restrict__ C, int m, int kk, int n, int r_k, int r_k1) {
  const int64_t total = (int64_t)m * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t / n), j = (int)(t % n);
    double s = 0.0;
    for (int l = 0; l < kk; ++l) s = fma(A[(int64_t)i * kk + l], B[(int64_t)l * n + j], s);
    if (r_k > 0) {
      const int b = i / r_k1, b2 = i % r_k1, a = j / r_k, a2 = j % r_k;
      const int R = r_k * r_k1;
      C[(int64_t)(a + b * r_k) * R + (a2 + b2 * r_k)] = s;
    } else {
      C[t] = s;
    }
  }
}

hipError_t launch_gemm64(const double* A, const double* B, double* C, int m, int kk, int n,
                         hipStream_t st, int r_k, int r_k1) {
  hipLaunchKernelGGL(k_gemm64, dim3(grid_for((int64_t)m * n, 256)), dim3(256), 0, st, A, B, C, m,
                     kk, n, r_k, r_k1);
  return hipGetLastError();
}

// G[(a + b r_k), (a2 + b2 r_k)] = P[(b r_k1 + b2), (a r_k + a2)]
__global__ void k_realign(const double* __restrict__ P, double* __restrict__ G, int r_k, int r_k1) {
  const int R = r_k * r_k1;
  const int64_t total = (int64_t)R * R;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t / R), j = (int)(t % R);
    const int a = i % r_k, b = i / r_k, a2 = j % r_k, b2 = j / r_k;
    G[t] = P[(int64_t)(b * r_k1 + b2) * (r_k * r_k) + (a * r_k + a2)];
  }
}

hipError_t launch_realign(const double* P, double* G, int r_k, int r_k1, hipStream_t st) {
  const int64_t R = (int64_t)r_k * r_k1;
  hipLaunchKernelGGL(k_realign, dim3(grid_for(R * R, 256)), dim3(256), 0, st, P, G, r_k, r_k1);
  return hipGetLastError();
}

// The whole ring product of eq. 13 for factor sides <= 64 in one work-group.  The running
// product is kept transposed (Xt[l][i]) and the next factor as Y[l][j], both zero padded to
// 64 x 64 in LDS; thread (ti, tj) of a 16 x 16 grid accumulates the 4 x 4 block of rows
// 4 ti.. and columns 4 tj.. from two 32-byte reads per k-step, then stores it transposed
// as the next Xt.  The last product is realigned into G as above.
__global__ __launch_bounds__(256) void k_ring(RingArgs a) {
  extern __shared__ __align__(16) double sm[];
  double* Xt = sm;
  double* Y = sm + 4096;
  double* Zt = sm + 8192;
  const int tid = threadIdx.x;
  const int rows = a.rows[0];
  int inner = a.cols[0];
  {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = tid + 256 * q, l = t >> 6, i = t & 63;
      v[q] = (i < rows && l < inner) ? a.K[0][i * inner + l] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) Xt[tid + 256 * q] = v[q];
  }
  const int ti = tid >> 4, tj = tid & 15;
  for (int f = 1; f < a.nf; ++f) {
    const int cols = a.cols[f];
    {
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int t = tid + 256 * q, l = t >> 6, j = t & 63;
        v[q] = (l < inner && j < cols) ? a.K[f][l * cols + j] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) Y[tid + 256 * q] = v[q];
    }
    __syncthreads();
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
    for (int l = 0; l < inner; ++l) {
      const double2 x0 = *reinterpret_cast<const double2*>(Xt + l * 64 + 4 * ti);
      const double2 x1 = *reinterpret_cast<const double2*>(Xt + l * 64 + 4 * ti + 2);
      const double2 y0 = *reinterpret_cast<const double2*>(Y + l * 64 + 4 * tj);
      const double2 y1 = *reinterpret_cast<const double2*>(Y + l * 64 + 4 * tj + 2);
      const double xv[4] = {x0.x, x0.y, x1.x, x1.y};
      const double yv[4] = {y0.x, y0.y, y1.x, y1.y};
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(xv[u], yv[v], acc[u][v]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) Zt[(4 * tj + v) * 64 + 4 * ti + u] = acc[u][v];
    __syncthreads();
    double* tmp = Xt;
    Xt = Zt;
    Zt = tmp;
    inner = cols;
  }
  __syncthreads();
  const int r_k = a.r_k, r_k1 = a.r_k1, R = r_k * r_k1;
  for (int t = tid; t < rows * inner; t += 256) {
    const int i = t / inner, j = t % inner;
    const int b = i / r_k1, b2 = i % r_k1, al = j / r_k, a2 = j % r_k;
    a.G[(int64_t)(al + b * r_k) * R + (a2 + b2 * r_k)] = Xt[j * 64 + i];
  }
}

hipError_t launch_ring(const RingArgs& a, hipStream_t st) {
  if (a.nf < 1 || a.nf > kMaxN) return hipErrorInvalidValue;
  for (int f = 0; f < a.nf; ++f) {
    if (a.rows[f] > 64 || a.cols[f] > 64) return hipErrorInvalidValue;
    if (f > 0 && a.rows[f] != a.cols[f - 1]) return hipErrorInvalidValue;
  }
  if (a.rows[0] != a.r_k1 * a.r_k1 || a.cols[a.nf - 1] != a.r_k * a.r_k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ring, dim3(1), dim3(256), 3 * 4096 * sizeof(double), st, a);
  return hipGetLastError();
}

// G^{!=k} from the factors K[j] of the other cores (eq. 13): the ring product
// K_{k+1} ... K_N K_1 ... K_{k-1} in cyclic order, realigned.  Factor sides <= 64: the
// whole ring in one work-group when its three 64 x 64 tiles fit lds_max bytes of LDS;
// otherwise one FP64 product per factor through P0 / P1.
hipError_t launch_ring_gram(int N, const int32_t* ranks, int k, const double* const* K, double* P0,
                            double* P1, double* G, int64_t lds_max, hipStream_t st) {
  const int s1 = (k + 1) % N;
  const double* cur = K[s1];
  const int rows = ranks[s1] * ranks[s1];
  int inner = ranks[(s1 + 1) % N] * ranks[(s1 + 1) % N];
  if (N == 2) return launch_realign(cur, G, ranks[k], ranks[s1], st);
  RingArgs ra;
  memset(&ra, 0, sizeof(ra));
  bool fits = true;
  ra.nf = N - 1;
  for (int t = 1; t <= N - 1; ++t) {
    const int m = (k + t) % N;
    ra.K[t - 1] = K[m];
    ra.rows[t - 1] = ranks[m] * ranks[m];
    ra.cols[t - 1] = ranks[(m + 1) % N] * ranks[(m + 1) % N];
    fits = fits && ra.rows[t - 1] <= 64 && ra.cols[t - 1] <= 64;
  }
  ra.r_k = ranks[k];
  ra.r_k1 = ranks[s1];
  ra.G = G;
  if (fits && (int64_t)3 * 4096 * sizeof(double) <= lds_max) return launch_ring(ra, st);
  double* bufs[2] = {P0, P1};
  int which = 0;
  for (int t = 2; t <= N - 1; ++t) {
    const int m = (k + t) % N;
    const int cols = ranks[(m + 1) % N] * ranks[(m + 1) % N];
    hipError_t e;
    if (t == N - 1) {  // last factor: G realigned
      e = launch_gemm64(cur, K[m], G, rows, inner, cols, st, ranks[k], ranks[s1]);
    } else {
      e = launch_gemm64(cur, K[m], bufs[which], rows, inner, cols, st);
      cur = bufs[which];
      which ^= 1;
    }
    if (e != hipSuccess) return e;
    inner = cols;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- scaled direction

// Cinv = (G + lambda I)^{-1}, lambda = lambda_rel * tr(G) / n, by in-place Gauss-Jordan
// elimination without pivoting (stable for SPD matrices, whose pivots are the positive
// Schur-complement diagonals).  A pivot <= 64 eps * max diag (or not finite) marks the
// matrix as not positive definite: flag set, Cinv = 0.
template <bool kLDS>
__global__ __launch_bounds__(1024) void k_inverse(const double* __restrict__ G,
                                                  double* __restrict__ Cinv, int n,
                                                  double lambda_rel, uint32_t* flags,
                                                  int assign) {
  extern __shared__ double lds[];
  __shared__ double f[256];
  __shared__ double s_lam, s_thr;
  __shared__ int s_bad;
  double* A = kLDS ? lds : Cinv;
  const int nn = n * n;
  for (int t = threadIdx.x; t < nn; t += blockDim.x) A[t] = G[t];
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0.0, mx = 0.0;
    for (int i = 0; i < n; ++i) {
      tr += A[i * n + i];
      mx = fmax(mx, A[i * n + i]);
    }
    const double lam = lambda_rel * tr / n;
    s_lam = lam;
    s_thr = 64.0 * 2.220446049250313e-16 * (mx + lam);
    s_bad = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) A[i * n + i] += s_lam;
  __syncthreads();
  const int my_t = threadIdx.x, my_i = my_t / n, my_j = my_t % n;
  for (int k = 0; k < n; ++k) {
    const double piv = A[k * n + k];
    if (!(piv > s_thr) || !isfinite(piv)) {
      if (threadIdx.x == 0) s_bad = 1;
      break;  // uniform: every thread read the same pivot
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) f[i] = A[i * n + k];
    __syncthreads();
    const double inv = 1.0 / piv;
    for (int j = threadIdx.x; j < n; j += blockDim.x) A[k * n + j] = (j == k ? 1.0 : A[k * n + j]) * inv;
    __syncthreads();
    if (nn <= (int)blockDim.x) {
      if (my_t < nn && my_i != k) A[my_t] = (my_j == k ? 0.0 : A[my_t]) - f[my_i] * A[k * n + my_j];
    } else {
      for (int t = threadIdx.x; t < nn; t += blockDim.x) {
        const int i = t / n, j = t % n;
        if (i != k) A[t] = (j == k ? 0.0 : A[t]) - f[i] * A[k * n + j];
      }
    }
    __syncthreads();
  }
  __syncthreads();
  const bool bad = s_bad != 0;
  for (int t = threadIdx.x; t < nn; t += blockDim.x) Cinv[t] = bad ? 0.0 : A[t];
  if (threadIdx.x == 0) {
    if (assign) *flags = bad ? TRD_FLAG_NOTSPD_BIT : 0u;
    else if (bad) atomicOr(flags, TRD_FLAG_NOTSPD_BIT);
  }
}

__global__ __launch_bounds__(256) void k_inverse64(const double* __restrict__ G, int n,
                                                   double lambda_rel, double* __restrict__ Cinv,
                                                   uint32_t* flags, int assign);

hipError_t launch_inverse(const double* G, double* Cinv, int n, double lambda_rel,
                          uint32_t* flags, hipStream_t st, bool assign) {
  const int as = assign ? 1 : 0;
  if (n > 32 && n <= 64) {  // register form; smaller systems keep one element per thread
    hipLaunchKernelGGL(k_inverse64, dim3(1), dim3(256), 0, st, G, n, lambda_rel, Cinv, flags, as);
    return hipGetLastError();
  }
  // small systems run in one or a few waves: fewer barrier participants per step
  int threads = ((n * n + 63) / 64) * 64;
  if (threads > 1024) threads = 1024;
  if ((int64_t)n * n * (int64_t)sizeof(double) + 4096 <= g_lds_max) {
    hipLaunchKernelGGL(k_inverse<true>, dim3(1), dim3(threads), (size_t)n * n * sizeof(double), st,
                       G, Cinv, n, lambda_rel, flags, as);
  } else {
    hipLaunchKernelGGL(k_inverse<false>, dim3(1), dim3(1024), 0, st, G, Cinv, n, lambda_rel,
                       flags, as);
  }
  return hipGetLastError();
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Cinv = (G + lambda I)^{-1} for n <= 64 in one work-group of 256 threads, with the same
// elimination and the same SPD test as k_inverse.  Lane j of wave w keeps column j of rows
// w, w + 4, ..., w + 60 in registers; the pivot column of those rows comes from lane k of
// the same wave, the scaled pivot row from LDS (one barrier per step).
__global__ __launch_bounds__(256) void k_inverse64(const double* __restrict__ G, int n,
                                                   double lambda_rel, double* __restrict__ Cinv,
                                                   uint32_t* flags, int assign) {
  __shared__ double prow[2][64];
  __shared__ double s_lam, s_thr;
  __shared__ int s_bad;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j = threadIdx.x & 63;
  double A[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = w + 4 * q;
    A[q] = (i < n && j < n) ? G[i * n + j] : 0.0;
  }
  if (threadIdx.x == 0) {
    double tr = 0.0, mx = 0.0;
    for (int i = 0; i < n; ++i) {
      tr += G[i * n + i];
      mx = fmax(mx, G[i * n + i]);
    }
    const double lam = lambda_rel * tr / n;
    s_lam = lam;
    s_thr = 64.0 * 2.220446049250313e-16 * (mx + lam);
    s_bad = 0;
  }
  __syncthreads();
  const double lam = s_lam, thr = s_thr;
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (w + 4 * q == j && j < n) A[q] += lam;
  bool bad = false;
#pragma unroll
  for (int kq = 0; kq < 16; ++kq) {
#pragma unroll
    for (int kw = 0; kw < 4; ++kw) {
      const int k = 4 * kq + kw;
      if (k < n && !bad) {  // uniform over the group
        const int buf = k & 1;
        if (w == kw) {
          const double piv = readlane_f64(A[kq], k);
          if (!(piv > thr) || !isfinite(piv)) {
            if (j == 0) s_bad = 1;
          } else {
            prow[buf][j] = (j == k ? 1.0 : A[kq]) * (1.0 / piv);
          }
        }
        __syncthreads();
        bad = s_bad != 0;
        if (!bad) {
          const double pr = prow[buf][j];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const double f = readlane_f64(A[q], k);
            A[q] = (w + 4 * q == k) ? pr : (j == k ? 0.0 : A[q]) - f * pr;
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int i = w + 4 * q;
    if (i < n && j < n) Cinv[i * n + j] = bad ? 0.0 : A[q];
  }
  if (threadIdx.x == 0) {
    if (assign) *flags = bad ? TRD_FLAG_NOTSPD_BIT : 0u;
    else if (bad) atomicOr(flags, TRD_FLAG_NOTSPD_BIT);
  }
}

// h = d Cinv (I_k x n), written in FP64 and in the problem dtype; per-block partial
// sums of <d, h> (fixed order).  A NOTSPD flag zeroes h.  Cinv == nullptr: h = d (the
// unscaled direction).
template <typename real>
__global__ __launch_bounds__(256) void k_apply_inverse(const double* __restrict__ d64,
                                                       const double* __restrict__ Cinv, int64_t Ik,
                                                       int n, double* __restrict__ h64,
                                                       real* __restrict__ h_real,
                                                       double* __restrict__ part,
                                                       const uint32_t* flags) {
  __shared__ double red[4];
  __shared__ double Cs[64 * 64];  // Cinv staged when n <= 64
  const int64_t total = Ik * n;
  const bool bad = (*flags & TRD_FLAG_NOTSPD_BIT) != 0;
  const bool staged = Cinv && n <= 64;
  if (staged) {  // 256 threads, at most 16 elements each, all loads in flight first
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = threadIdx.x + 256 * q;
      v[q] = t < n * n ? Cinv[t] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int t = threadIdx.x + 256 * q;
      if (t < n * n) Cs[t] = v[q];
    }
    __syncthreads();
  }
  const double* Cp = staged ? Cs : Cinv;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double contrib = 0.0;
  if (t < total) {
    const int64_t i = t / n;
    const int c = (int)(t % n);
    double s = 0.0;
    if (!Cinv)
      s = d64[t];
    else if (!bad)
      for (int l = 0; l < n; ++l) s = fma(d64[i * n + l], Cp[(int64_t)l * n + c], s);
    h64[t] = s;
    if (h_real) h_real[t] = (real)s;
    contrib = d64[t] * s;
  }
  for (int o = 32; o > 0; o >>= 1) contrib += __shfl_xor(contrib, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = contrib;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_apply_inverse(const double* d64, const double* Cinv, int64_t Ik, int n,
                                double* h64, void* h_real, int dtype, double* part_num,
                                const uint32_t* flags, hipStream_t st) {
  const int64_t total = Ik * n;
  const int nb = (int)((total + 255) / 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_apply_inverse<float>, dim3(nb), dim3(256), 0, st, d64, Cinv, Ik, n, h64,
                       (float*)h_real, part_num, flags);
  else
    hipLaunchKernelGGL(k_apply_inverse<double>, dim3(nb), dim3(256), 0, st, d64, Cinv, Ik, n, h64,
                       (double*)h_real, part_num, flags);
  return hipGetLastError();
}

// out[c] = sum over rows r < n of part[r*width + c], c < width; one work-group,
// fixed per-thread assignment and fixed tree order.
__global__ __launch_bounds__(1024) void k_reduce(const double* __restrict__ part, int64_t n,
                                                 int width, double* __restrict__ out) {
  __shared__ double buf[1024];
  for (int c = 0; c < width; ++c) {
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += 1024) s += part[r * width + c];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
      if (threadIdx.x < o) buf[threadIdx.x] += buf[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = buf[0];
    __syncthreads();
  }
}

hipError_t launch_reduce_partials(const double* part, int64_t n, int width, double* out,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, st, part, n, width, out);
  return hipGetLastError();
}

__global__ void k_set_scalar(double* p, double v) { *p = v; }

hipError_t launch_set_scalar(double* p, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

// eta of eq. (12) = num / den; 0 with a flag when nothing was observed or den <= 0.
__global__ void k_eta(const double* num, const double* den, const int64_t* nobs, double* eta,
                      uint32_t* flags, uint32_t* flags_user, double* eta_user) {
  const double a = *num, b = *den;
  uint32_t f = *flags;
  double e = 0.0;
  if (*nobs == 0) f |= TRD_FLAG_EMPTY_BIT;
  if (!(b > 0.0) || !isfinite(b) || !isfinite(a)) f |= TRD_FLAG_ZERO_DEN_BIT;
  else e = a / b;
  if (f & TRD_FLAG_NOTSPD_BIT) e = 0.0;
  *eta = e;
  *flags = f;
  if (eta_user) *eta_user = e;
  if (flags_user) *flags_user |= f;
}

hipError_t launch_eta(const double* num, const double* den, const int64_t* nobs, double* eta,
                      uint32_t* flags, uint32_t* flags_user, double* eta_user, hipStream_t st) {
  hipLaunchKernelGGL(k_eta, dim3(1), dim3(1), 0, st, num, den, nobs, eta, flags, flags_user,
                     eta_user);
  return hipGetLastError();
}

// One work-group: num = sum of <d,h> partials, den = sum of the line-search pass
// partials (column 0 of [n_den][3]), eta of eq. (12) with its flags, then the update
// Z_k <- Z_k + eta h (eq. 11, '+' reading).  Fixed-order reductions.  halt (optional):
// a nonzero word there leaves Z unchanged (eta 0): a fit that stopped at an earlier sweep
// whose later sweeps were already queued.
template <typename real>
__global__ __launch_bounds__(1024) void k_finish_step(const double* __restrict__ pnum, int64_t n_num,
                                                      const double* __restrict__ pden, int64_t n_den,
                                                      const int64_t* nobs, uint32_t* flags,
                                                      uint32_t* flags_user, double* eta_out,
                                                      double* eta_user, real* __restrict__ Z,
                                                      const double* __restrict__ h, int64_t nz,
                                                      const uint32_t* halt) {
  __shared__ double bn[1024], bd[1024];
  __shared__ double s_eta;
  double a = 0.0, b = 0.0;  // (loops unrolled: a thread's loads are in flight together)
#pragma unroll 4
  for (int64_t r = threadIdx.x; r < n_num; r += 1024) a += pnum[r];
#pragma unroll 4
  for (int64_t r = threadIdx.x; r < n_den; r += 1024) b += pden[r * 3];
  bn[threadIdx.x] = a;
  bd[threadIdx.x] = b;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      bn[threadIdx.x] += bn[threadIdx.x + o];
      bd[threadIdx.x] += bd[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double num = bn[0], den = bd[0];
    uint32_t f = *flags;
    double e = 0.0;
    if (*nobs == 0) f |= TRD_FLAG_EMPTY_BIT;
    if (!(den > 0.0) || !isfinite(den) || !isfinite(num)) f |= TRD_FLAG_ZERO_DEN_BIT;
    else e = num / den;
    if (f & TRD_FLAG_NOTSPD_BIT) e = 0.0;
    if (halt && *halt) e = 0.0;
    *eta_out = e;
    *flags = f;
    if (eta_user) *eta_user = e;
    if (flags_user) *flags_user |= f;
    s_eta = e;
  }
  __syncthreads();
  const double e = s_eta;
  if (e != 0.0) {
#pragma unroll 4
    for (int64_t t = threadIdx.x; t < nz; t += 1024) Z[t] = (real)fma(e, h[t], (double)Z[t]);
  }
}

hipError_t launch_finish_step(int dtype, const double* pnum, int64_t n_num, const double* pden,
                              int64_t n_den, const int64_t* nobs, uint32_t* flags,
                              uint32_t* flags_user, double* eta, double* eta_user, void* Z,
                              const double* h, int64_t nz, const uint32_t* halt,
                              hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_finish_step<float>, dim3(1), dim3(1024), 0, st, pnum, n_num, pden, n_den,
                       nobs, flags, flags_user, eta, eta_user, (float*)Z, h, nz, halt);
  else
    hipLaunchKernelGGL(k_finish_step<double>, dim3(1), dim3(1024), 0, st, pnum, n_num, pden, n_den,
                       nobs, flags, flags_user, eta, eta_user, (double*)Z, h, nz, halt);
  return hipGetLastError();
}

// Z_k <- Z_k + eta * h (eq. 11 with the '+' reading)
template <typename real>
__global__ void k_update(real* __restrict__ Z, const double* __restrict__ h, const double* eta,
                         int64_t n) {
  const double e = *eta;
  if (e == 0.0) return;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    Z[t] = (real)fma(e, h[t], (double)Z[t]);
}

hipError_t launch_update(int dtype, void* Z, const double* h64, const double* eta, int64_t n,
                         hipStream_t st) {
  if (dtype == 0)
    hipLaunchKernelGGL(k_update<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, (float*)Z, h64,
                       eta, n);
  else
    hipLaunchKernelGGL(k_update<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, (double*)Z,
                       h64, eta, n);
  return hipGetLastError();
}

// Gather the per-sweep host-visible values into mapped pinned host memory:
// out = {sigma, conv[0], conv[1], (double)flags, eta[0..N)}.  halt (optional) is set once
// flags carry NOTSPD, so that the steps of sweeps queued after this one change no core.
__global__ void k_pack_report(const double* sigma, const double* conv, const uint32_t* flags,
                              const double* eta, int N, double* out, uint32_t* halt) {
  const uint32_t f = *flags;
  out[0] = *sigma;
  out[1] = conv[0];
  out[2] = conv[1];
  out[3] = (double)f;
  for (int k = 0; k < N; ++k) out[4 + k] = eta[k];
  if (halt && (f & TRD_FLAG_NOTSPD_BIT)) *halt = 1u;
  __threadfence_system();
}

hipError_t launch_pack_report(const double* sigma, const double* conv, const uint32_t* flags,
                              const double* eta, int N, double* out, uint32_t* halt,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_pack_report, dim3(1), dim3(1), 0, st, sigma, conv, flags, eta, N, out,
                     halt);
  return hipGetLastError();
}

// ---------------------------------------------------------------- convergence (Alg. 1)

// M = Z G (I_N x n); G is staged in LDS when n <= 64 (the sums are the same either way)
template <typename real>
__global__ __launch_bounds__(256) void k_zg(const real* __restrict__ Z, const double* __restrict__ G,
                                            int64_t IN, int n, double* __restrict__ M) {
  __shared__ double Gs[64 * 64];
  const bool staged = n <= 64;  // uniform over the grid
  if (staged) {  // (unrolled: the loads of a thread are in flight together)
#pragma unroll 8
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) Gs[t] = G[t];
    __syncthreads();
  }
  const int64_t total = IN * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t / n;
    const int c = (int)(t % n);
    const real* zr = Z + i * n;
    // the sum in order l = 0 .. n-1; unrolled so that a group of row loads is in flight
    // together instead of one round trip per term
    double s = 0.0;
    if (staged) {
#pragma unroll 16
      for (int l = 0; l < n; ++l) s = fma((double)zr[l], Gs[l * n + c], s);
    } else {
#pragma unroll 16
      for (int l = 0; l < n; ++l) s = fma((double)zr[l], G[(int64_t)l * n + c], s);
    }
    M[t] = s;
  }
}

// D = M Z^T, with per-block partials of sum (D - Dprev)^2 and sum D^2
template <typename real>
__global__ __launch_bounds__(256) void k_mzt(const double* __restrict__ M, const real* __restrict__ Z,
                                             int64_t IN, int n, double* __restrict__ D,
                                             const double* __restrict__ Dprev, int have_prev,
                                             double* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t total = IN * IN;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double a = 0.0, b = 0.0;
  if (t < total) {
    const int64_t i = t / IN, j = t % IN;
    const double* mr = M + i * n;
    const real* zr = Z + j * n;
    double s = 0.0;  // in order l = 0 .. n-1 (unrolled: the loads of a group overlap)
#pragma unroll 16
    for (int l = 0; l < n; ++l) s = fma(mr[l], (double)zr[l], s);
    D[t] = s;
    const double dd = have_prev ? s - Dprev[t] : s;
    a = dd * dd;
    b = s * s;
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const double* r = red[threadIdx.x];
    part[blockIdx.x * 2 + threadIdx.x] = (r[0] + r[1]) + (r[2] + r[3]);
  }
}

hipError_t launch_convergence(int dtype, const void* ZN, const double* G, int64_t IN, int n,
                              double* M, double* D, const double* Dprev, int have_prev,
                              double* part, hipStream_t st) {
  // part must hold 2 * ceil(IN*IN/256) doubles; the caller reduces it (width 2)
  if (dtype == 0) {
    hipLaunchKernelGGL(k_zg<float>, dim3(grid_for(IN * n, 256)), dim3(256), 0, st,
                       (const float*)ZN, G, IN, n, M);
    hipLaunchKernelGGL(k_mzt<float>, dim3((unsigned)((IN * IN + 255) / 256)), dim3(256), 0, st, M,
                       (const float*)ZN, IN, n, D, Dprev, have_prev, part);
  } else {
    hipLaunchKernelGGL(k_zg<double>, dim3(grid_for(IN * n, 256)), dim3(256), 0, st,
                       (const double*)ZN, G, IN, n, M);
    hipLaunchKernelGGL(k_mzt<double>, dim3((unsigned)((IN * IN + 255) / 256)), dim3(256), 0, st,
                       M, (const double*)ZN, IN, n, D, Dprev, have_prev, part);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- weights (eq. 7)

template <typename real>
__global__ void k_weights(const real* __restrict__ r, int64_t n, real inv2s2, int lim,
                          real* __restrict__ w) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const real e = r[t];
    w[t] = lim ? real(1) : exp(-(e * e) * inv2s2);
  }
}

hipError_t launch_weights(int dtype, const void* r, int64_t n, double sigma, void* w,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int lim = std::isinf(sigma) ? 1 : 0;
  const double inv = lim ? 0.0 : 0.5 / (sigma * sigma);
  if (dtype == 0)
    hipLaunchKernelGGL(k_weights<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, (const float*)r,
                       n, (float)inv, lim, (float*)w);
  else
    hipLaunchKernelGGL(k_weights<double>, dim3(grid_for(n, 256)), dim3(256), 0, st,
                       (const double*)r, n, inv, lim, (double*)w);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reconstruction (Def. 1)

struct CoreSet {
  const void* core[kMaxN];
  int64_t dims[kMaxN];
  int ranks[kMaxN];
  int N;
};

// x = sum_a (e_a^T Z_0(i_0) Z_1(i_1) ... Z_{N-1}(i_{N-1}))[a], one row vector at a time
template <typename real, int MAXR>
__global__ void k_reconstruct(CoreSet cs, const int64_t* __restrict__ lin, int64_t n,
                              int64_t total, real* __restrict__ out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = lin ? lin[t] : t;
    if (rem < 0 || rem >= total) {  // out-of-range request: NaN, no read
      out[t] = real(NAN);
      continue;
    }
    int64_t idx[kMaxN];
    for (int j = 0; j < cs.N; ++j) {
      idx[j] = rem % cs.dims[j];
      rem /= cs.dims[j];
    }
    const int r0 = cs.ranks[0];
    real total = real(0);
    for (int a = 0; a < r0; ++a) {
      real v[MAXR], nv[MAXR];
#pragma unroll
      for (int b = 0; b < MAXR; ++b) v[b] = b == a ? real(1) : real(0);
      int rin = r0;
      for (int j = 0; j < cs.N; ++j) {
        const int rout = cs.ranks[(j + 1) % cs.N];
        const real* zs = static_cast<const real*>(cs.core[j]) + idx[j] * (int64_t)rin * rout;
#pragma unroll
        for (int c = 0; c < MAXR; ++c) {
          real s = real(0);
          if (c < rout) {
#pragma unroll
            for (int b = 0; b < MAXR; ++b)
              if (b < rin) s = fma(v[b], zs[b + rin * c], s);
          }
          nv[c] = s;
        }
#pragma unroll
        for (int c = 0; c < MAXR; ++c) v[c] = nv[c];
        rin = rout;
      }
#pragma unroll
      for (int b = 0; b < MAXR; ++b)
        if (b == a) total += v[b];
    }
    out[t] = total;
  }
}

template <typename real>
static hipError_t recon_real(const CoreSet& cs, int maxr, const int64_t* lin, int64_t n, void* out,
                             hipStream_t st) {
  dim3 g(grid_for(n, 256, 1 << 16)), b(256);
  int64_t total = 1;
  for (int j = 0; j < cs.N; ++j) total *= cs.dims[j];
  if (maxr <= 4)
    hipLaunchKernelGGL((k_reconstruct<real, 4>), g, b, 0, st, cs, lin, n, total, (real*)out);
  else if (maxr <= 8)
    hipLaunchKernelGGL((k_reconstruct<real, 8>), g, b, 0, st, cs, lin, n, total, (real*)out);
  else
    hipLaunchKernelGGL((k_reconstruct<real, 16>), g, b, 0, st, cs, lin, n, total, (real*)out);
  return hipGetLastError();
}

hipError_t launch_reconstruct(int dtype, int N, const int64_t* dims, const int32_t* ranks,
                              const void* const* cores, const int64_t* lin, int64_t n, void* out,
                              hipStream_t st) {
  if (n <= 0) return hipSuccess;
  CoreSet cs;
  cs.N = N;
  int maxr = 1;
  for (int j = 0; j < kMaxN; ++j) {
    cs.core[j] = j < N ? cores[j] : nullptr;
    cs.dims[j] = j < N ? dims[j] : 1;
    cs.ranks[j] = j < N ? ranks[j] : 1;
    if (j < N && ranks[j] > maxr) maxr = ranks[j];
  }
  return dtype == 0 ? recon_real<float>(cs, maxr, lin, n, out, st)
                    : recon_real<double>(cs, maxr, lin, n, out, st);
}

// ---------------------------------------------------------------- kernel-width quantile
// Radix select of the element of rank floor((n-1) q) among non-negative float keys
// (padding slots hold +inf and sort last), digits of 11, 11 and 10 bits.
// state: [0] prefix, [1] remaining rank (as uint32 pair), [3] valid.

// With cand, the matching keys are also copied to this work-group's segment of cand
// (seg_cap keys from blockIdx.x * seg_cap; count in cand_cnt[blockIdx.x]), so that the next
// digit scans only them (k_qhist_seg).
__global__ __launch_bounds__(256) void k_qhist(const float* __restrict__ keys,
                                               const int64_t* __restrict__ nslots, int shift,
                                               int bits, const uint32_t* __restrict__ state,
                                               uint32_t* __restrict__ hist,
                                               float* __restrict__ cand,
                                               uint32_t* __restrict__ cand_cnt, int64_t seg_cap) {
  __shared__ uint32_t lh[2048];
  __shared__ uint32_t ncand;
  const uint32_t nb = 1u << bits;
  for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) lh[i] = 0u;
  if (threadIdx.x == 0) ncand = 0u;
  __syncthreads();
  float* seg = cand ? cand + (int64_t)blockIdx.x * seg_cap : nullptr;
  const int64_t n = *nslots;
  const uint32_t prefix = state[0];
  const int hi_shift = shift + bits;
  // four keys per lane per round (one 16-byte load); the round loop is uniform per wave
  const int64_t n4 = (n + 3) / 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n4; base += stride) {
    const int64_t i4 = base + threadIdx.x;
    float4 k4 = {0.f, 0.f, 0.f, 0.f};
    const bool full = 4 * i4 + 3 < n;
    if (full) k4 = reinterpret_cast<const float4*>(keys)[i4];
    const float kv[4] = {k4.x, k4.y, k4.z, k4.w};
    uint32_t keyv[4];
    bool matchv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = 4 * i4 + u;
      const bool in = i < n;
      // the key of a residual is its magnitude: the sign bit is dropped
      const uint32_t key = in ? (__float_as_uint(full ? kv[u] : keys[i]) & 0x7fffffffu) : 0u;
      const bool match = in && (hi_shift >= 32 || (key >> hi_shift) == prefix);
      if (match) atomicAdd(&lh[(key >> shift) & (nb - 1u)], 1u);
      keyv[u] = key;
      matchv[u] = match;
    }
    if (seg) {  // uniform over the wave: one LDS counter update per wave and round
      uint64_t bal[4];
      uint32_t tot = 0u;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bal[u] = __ballot(matchv[u]);
        tot += (uint32_t)__popcll(bal[u]);
      }
      if (tot) {  // uniform (from the ballots); every lane is active, lane 0 included
        const int lane = threadIdx.x & 63;
        const uint64_t below = (1ull << lane) - 1ull;
        uint32_t off = 0u;
        if (lane == 0) off = atomicAdd(&ncand, tot);
        off = (uint32_t)__builtin_amdgcn_readfirstlane((int)off);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (matchv[u]) seg[off + __popcll(bal[u] & below)] = __uint_as_float(keyv[u]);
          off += (uint32_t)__popcll(bal[u]);
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
    if (lh[i]) atomicAdd(&hist[i], lh[i]);
  if (seg && threadIdx.x == 0) cand_cnt[blockIdx.x] = ncand;
}

// the same digit histogram over the candidates k_qhist left in the segments
__global__ __launch_bounds__(256) void k_qhist_seg(const float* __restrict__ cand,
                                                   const uint32_t* __restrict__ cand_cnt,
                                                   int64_t seg_cap, int shift, int bits,
                                                   const uint32_t* __restrict__ state,
                                                   uint32_t* __restrict__ hist) {
  __shared__ uint32_t lh[2048];
  const uint32_t nb = 1u << bits;
  for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) lh[i] = 0u;
  __syncthreads();
  const uint32_t n = cand_cnt[blockIdx.x];
  const float* seg = cand + (int64_t)blockIdx.x * seg_cap;
  const uint32_t prefix = state[0];
  const int hi_shift = shift + bits;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t key = __float_as_uint(seg[i]) & 0x7fffffffu;
    if (hi_shift >= 32 || (key >> hi_shift) == prefix) atomicAdd(&lh[(key >> shift) & (nb - 1u)], 1u);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
    if (lh[i]) atomicAdd(&hist[i], lh[i]);
}

__global__ void k_qinit(const int64_t* nobs, double q, uint32_t* state, uint32_t* hist) {
  const int64_t n = *nobs;
  uint64_t rank = 0;
  if (n > 0) rank = (uint64_t)floor((double)(n - 1) * q);
  state[0] = 0u;
  state[1] = (uint32_t)(rank & 0xFFFFFFFFu);
  state[2] = (uint32_t)(rank >> 32);
  state[3] = n > 0 ? 1u : 0u;
  for (int i = 0; i < 2048; ++i) hist[i] = 0u;
}

__global__ __launch_bounds__(1024) void k_qpick(int bits, uint32_t* state, uint32_t* hist) {
  __shared__ unsigned long long sc[2048];
  __shared__ int found;
  const uint32_t nb = 1u << bits;
  const uint64_t rank = (uint64_t)state[1] | ((uint64_t)state[2] << 32);
  for (int i = threadIdx.x; i < 2048; i += 1024) sc[i] = (uint32_t)i < nb ? hist[i] : 0ull;
  if (threadIdx.x == 0) found = -1;
  __syncthreads();
  // inclusive scan, two elements per thread
  for (int o = 1; o < 2048; o <<= 1) {
    const int i0 = threadIdx.x, i1 = threadIdx.x + 1024;
    const unsigned long long a0 = i0 >= o ? sc[i0 - o] : 0ull;
    const unsigned long long a1 = i1 >= o ? sc[i1 - o] : 0ull;
    __syncthreads();
    sc[i0] += a0;
    sc[i1] += a1;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < (int)nb; i += 1024) {
    const unsigned long long excl = i ? sc[i - 1] : 0ull;
    if (excl <= rank && rank < sc[i]) found = i;  // exactly one bin qualifies
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t b = found >= 0 ? (uint32_t)found : nb - 1u;  // none: nothing observed
    const uint64_t excl = (found > 0) ? sc[found - 1] : 0ull;
    const uint64_t r = found >= 0 ? rank - excl : rank;
    state[0] = (state[0] << bits) | b;
    state[1] = (uint32_t)(r & 0xFFFFFFFFu);
    state[2] = (uint32_t)(r >> 32);
  }
  for (int i = threadIdx.x; i < (int)nb; i += 1024) hist[i] = 0u;
}

__global__ void k_qsigma(const uint32_t* state, double c, const double* sigma_min, double shrink,
                         double* sigma) {
  const double smin = *sigma_min;
  double s;
  if (state[3] == 0u) {
    s = smin > 0.0 ? smin : 1.0;
  } else {
    const double qv = (double)__uint_as_float(state[0]);
    s = fmax(c * qv, smin);
  }
  const double prev = *sigma;
  if (isfinite(prev)) s = fmax(s, shrink * prev);
  *sigma = s;
}

int quantile_grid(int64_t n_slots_hint) { return grid_for(n_slots_hint, 256, 2048); }
// keys one work-group of the histogram grid can see: its float4 groups times four
int64_t quantile_seg_cap(int64_t n_slots_hint) {
  const int64_t g = quantile_grid(n_slots_hint);
  const int64_t n4 = (n_slots_hint + 3) / 4;
  return std::max<int64_t>((n4 + g * 256 - 1) / (g * 256), 1) * 1024;
}

hipError_t launch_quantile_init(const int64_t* nobs, double q, uint32_t* state, uint32_t* hist,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_qinit, dim3(1), dim3(1), 0, st, nobs, q, state, hist);
  return hipGetLastError();
}

hipError_t launch_quantile_sigma(const float* keys, int64_t n_slots_hint, const int64_t* nslots,
                                 double q, double c, const double* sigma_min, double shrink,
                                 double* sigma, uint32_t* hist, uint32_t* state,
                                 const int64_t* nobs, float* cand, uint32_t* cand_cnt,
                                 bool first_digit_done, hipStream_t st) {
  if (!first_digit_done) hipLaunchKernelGGL(k_qinit, dim3(1), dim3(1), 0, st, nobs, q, state, hist);
  const int shifts[3] = {21, 10, 0};
  const int bitsv[3] = {11, 11, 10};
  const int g = quantile_grid(n_slots_hint);
  const int64_t seg = quantile_seg_cap(n_slots_hint);
  for (int r = 0; r < 3; ++r) {
    // the second digit also collects the keys that share the first one (per work-group
    // segments), the third scans only those
    if (r == 2 && cand)
      hipLaunchKernelGGL(k_qhist_seg, dim3(g), dim3(256), 0, st, (const float*)cand,
                         (const uint32_t*)cand_cnt, seg, shifts[r], bitsv[r], state, hist);
    else if (r > 0 || !first_digit_done)
      hipLaunchKernelGGL(k_qhist, dim3(g), dim3(256), 0, st, keys, nslots, shifts[r], bitsv[r],
                         state, hist, r == 1 ? cand : (float*)nullptr, cand_cnt, seg);
    hipLaunchKernelGGL(k_qpick, dim3(1), dim3(1024), 0, st, bitsv[r], state, hist);
  }
  hipLaunchKernelGGL(k_qsigma, dim3(1), dim3(1), 0, st, state, c, sigma_min, shrink, sigma);
  return hipGetLastError();
}

}  // namespace trd

// Subchain tables by batched core merging (Def. 2) and the contraction that turns the
// per-row gradient accumulators back into d of eq. (9).
#include "trd_internal.h"

namespace trd {

static int grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// out item (l + nL*j) = L(l) @ R(j): L(l) rA x rB, R(j) rB x rC, all column-major.
// Output element e of an item: (a, c) at a + rA*c, or at c + rC*a when transposed;
// positions rA*rC .. out_stride-1 are zero padding.
template <typename real>
__global__ void k_merge(const real* __restrict__ L, int64_t Ls, const int32_t* __restrict__ Llist,
                        int64_t nL, int rA, int rB, const real* __restrict__ R, int64_t Rs,
                        const int32_t* __restrict__ Rlist, int64_t nR, int rC,
                        real* __restrict__ out, int64_t out_stride, int transpose_out) {
  const int64_t total = nL * nR * out_stride;
  const int64_t used = (int64_t)rA * rC;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t item = t / out_stride;
    const int64_t e = t - item * out_stride;
    real acc = real(0);
    if (e < used) {
      int a, c;
      if (transpose_out) { c = (int)(e % rC); a = (int)(e / rC); }
      else { a = (int)(e % rA); c = (int)(e / rA); }
      const int64_t l = item % nL, j = item / nL;
      const real* Lp = L + (Llist ? (int64_t)Llist[l] : l) * Ls;
      const real* Rp = R + (Rlist ? (int64_t)Rlist[j] : j) * Rs;
      for (int b = 0; b < rB; ++b) acc = fma(Lp[a + rA * b], Rp[b + rB * c], acc);
    }
    out[t] = acc;
  }
}

hipError_t launch_merge(int dtype, ItemRef L, int64_t nL, int rA, int rB, ItemRef R, int64_t nR,
                        int rC, void* out, int64_t out_stride, int transpose_out, hipStream_t st) {
  const int64_t total = nL * nR * out_stride;
  if (total <= 0) return hipSuccess;
  dim3 g(grid_for(total, 256)), b(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_merge<float>, g, b, 0, st, (const float*)L.ptr, L.stride, L.list, nL, rA,
                       rB, (const float*)R.ptr, R.stride, R.list, nR, rC, (float*)out, out_stride,
                       transpose_out);
  else
    hipLaunchKernelGGL(k_merge<double>, g, b, 0, st, (const double*)L.ptr, L.stride, L.list, nL,
                       rA, rB, (const double*)R.ptr, R.stride, R.list, nR, rC, (double*)out,
                       out_stride, transpose_out);
  return hipGetLastError();
}

// Copy items (optionally through an index list), optionally transposed, zero padded.
template <typename real>
__global__ void k_pack(const real* __restrict__ in, int64_t is, const int32_t* __restrict__ list,
                       int64_t n, int rA, int rB, real* __restrict__ out, int64_t out_stride,
                       int transpose_out) {
  const int64_t total = n * out_stride;
  const int64_t used = (int64_t)rA * rB;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t item = t / out_stride;
    const int64_t e = t - item * out_stride;
    real v = real(0);
    if (e < used) {
      int a, b;
      if (transpose_out) { b = (int)(e % rB); a = (int)(e / rB); }
      else { a = (int)(e % rA); b = (int)(e / rA); }
      const real* p = in + (list ? (int64_t)list[item] : item) * is;
      v = p[a + rA * b];
    }
    out[t] = v;
  }
}

hipError_t launch_pack(int dtype, ItemRef in, int64_t n, int rA, int rB, void* out,
                       int64_t out_stride, int transpose_out, hipStream_t st) {
  const int64_t total = n * out_stride;
  if (total <= 0) return hipSuccess;
  dim3 g(grid_for(total, 256)), b(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_pack<float>, g, b, 0, st, (const float*)in.ptr, in.stride, in.list, n, rA,
                       rB, (float*)out, out_stride, transpose_out);
  else
    hipLaunchKernelGGL(k_pack<double>, g, b, 0, st, (const double*)in.ptr, in.stride, in.list, n,
                       rA, rB, (double*)out, out_stride, transpose_out);
  return hipGetLastError();
}

// float -> bf16, round to nearest even (finite inputs)
__global__ void k_to_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint32_t u = __float_as_uint(in[t]);
    uint32_t r = 0x7FFFu + ((u >> 16) & 1u);
    out[t] = (uint16_t)((u + r) >> 16);
  }
}

hipError_t launch_to_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n, 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

// S[row][j] = sum over column tiles c of Spart[c][row][j], fixed order (in place into tile 0)
template <typename real>
__global__ void k_sum_tiles(real* __restrict__ S, int n_ct, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    real acc = S[t];
    for (int c = 1; c < n_ct; ++c) acc += S[(int64_t)c * n + t];
    S[t] = acc;
  }
}

hipError_t launch_sum_tiles(int dtype, void* S, int n_ct, int64_t n, hipStream_t st) {
  if (n_ct <= 1 || n <= 0) return hipSuccess;
  dim3 g(grid_for(n, 256, 4096)), b(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_sum_tiles<float>, g, b, 0, st, (float*)S, n_ct, n);
  else
    hipLaunchKernelGGL(k_sum_tiles<double>, g, b, 0, st, (double*)S, n_ct, n);
  return hipGetLastError();
}

// D(i_k)[a, b] = sum_{m_B} sum_c St(i_k + I_k m_B)[a + r_k c] * U(m_B)[b + r_k1 c]
// (St^T U^T of the two-factor split of the gradient); St(row) is the fixed-order sum of
// the n_ct column-tile partials written by the gradient pass.  U.ptr == nullptr: no B modes,
// U = identity (r_s = r_k1) and D(i_k) = St(i_k).
// grid: (I_k, nchunk); block 256 threads, thread e < r_k*r_k1 owns one output.
template <typename real>
__global__ __launch_bounds__(256) void k_contract(const real* __restrict__ S, int RRP, int n_ct,
                                                  int64_t nrows, int64_t Ik,
                                                  int64_t nB, int r_k, int r_s, int r_k1,
                                                  const real* __restrict__ U, int64_t Us,
                                                  const int32_t* __restrict__ Ulist,
                                                  double* __restrict__ part, int nchunk) {
  __shared__ real srow[kMaxRR];
  __shared__ real urow[256];
  const int64_t ik = blockIdx.x;
  const int chunk = blockIdx.y;
  const int RRk = r_k * r_k1;
  const int e = threadIdx.x;
  const int a = e % r_k, b = e / r_k;
  const int64_t per = (nB + nchunk - 1) / nchunk;
  const int64_t m0 = chunk * per, m1 = min(nB, m0 + per);
  double acc = 0.0;
  for (int64_t m = m0; m < m1; ++m) {
    const real* sp = S + (ik + Ik * m) * RRP;
    __syncthreads();
    if (threadIdx.x < r_k * r_s) {
      real acc_s = real(0);
      for (int c = 0; c < n_ct; ++c) acc_s += sp[(int64_t)c * nrows * RRP + threadIdx.x];
      srow[threadIdx.x] = acc_s;
    }
    if (U && threadIdx.x < r_k1 * r_s) {
      const real* up = U + (Ulist ? (int64_t)Ulist[m] : m) * Us;
      urow[threadIdx.x] = up[threadIdx.x];
    }
    __syncthreads();
    if (e < RRk) {
      if (U) {
        real s = real(0);
        for (int c = 0; c < r_s; ++c) s = fma(srow[a + r_k * c], urow[b + r_k1 * c], s);
        acc += (double)s;
      } else {
        acc += (double)srow[a + r_k * b];
      }
    }
  }
  if (e < RRk) part[((int64_t)chunk * Ik + ik) * RRk + e] = acc;
}

hipError_t launch_contract(int dtype, const void* S, int RRP, int n_ct, int64_t nrows, int64_t Ik,
                           int64_t nB, int r_k, int r_s, int r_k1, ItemRef U, double* part,
                           int nchunk, hipStream_t st) {
  dim3 g((unsigned)Ik, (unsigned)nchunk), b(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_contract<float>, g, b, 0, st, (const float*)S, RRP, n_ct, nrows, Ik, nB,
                       r_k, r_s, r_k1, (const float*)U.ptr, U.stride, U.list, part, nchunk);
  else
    hipLaunchKernelGGL(k_contract<double>, g, b, 0, st, (const double*)S, RRP, n_ct, nrows, Ik, nB,
                       r_k, r_s, r_k1, (const double*)U.ptr, U.stride, U.list, part, nchunk);
  return hipGetLastError();
}

template <typename real>
__global__ void k_contract_finish(const double* __restrict__ part, int nchunk, int64_t Ik, int RRk,
                                  double* __restrict__ d64, real* __restrict__ d_out,
                                  double scale) {
  const int64_t n = Ik * RRk;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * n + t];
    s *= scale;
    if (d64) d64[t] = s;
    if (d_out) d_out[t] = (real)s;
  }
}

hipError_t launch_contract_finish(int dtype, const double* part, int nchunk, int64_t Ik, int RRk,
                                  double* d64, void* d_out, double scale, hipStream_t st) {
  int64_t n = Ik * RRk;
  dim3 g(grid_for(n, 256)), b(256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_contract_finish<float>, g, b, 0, st, part, nchunk, Ik, RRk, d64,
                       (float*)d_out, scale);
  else
    hipLaunchKernelGGL(k_contract_finish<double>, g, b, 0, st, part, nchunk, Ik, RRk, d64,
                       (double*)d_out, scale);
  return hipGetLastError();
}

}  // namespace trd

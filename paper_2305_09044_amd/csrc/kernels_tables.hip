// Subchain tables by batched core merging (Def. 2) and the contraction that turns the
// per-row gradient accumulators back into d of eq. (9).
#include "trd_internal.h"

#include <type_traits>

namespace trd {

static int grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__device__ __forceinline__ uint16_t bf16_bits(float f) {  // round to nearest even (finite)
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// store one element of a table: the problem type, or bf16 bits for the matrix-core passes;
// with out_lo also the bf16 of the remainder v - hi (split tables: hi + lo carries about
// 16 significant bits)
template <typename real, bool BF>
__device__ __forceinline__ void put(void* out, void* out_lo, int64_t i, real v) {
  if constexpr (BF) {
    const uint16_t hi = bf16_bits((float)v);
    static_cast<uint16_t*>(out)[i] = hi;
    if (out_lo) {
      const float hv = __uint_as_float((uint32_t)hi << 16);
      static_cast<uint16_t*>(out_lo)[i] = bf16_bits((float)v - hv);
    }
  } else {
    static_cast<real*>(out)[i] = v;
  }
}

// out item (l + nL*j) = L(l) @ R(j): L(l) rA x rB, R(j) rB x rC, all column-major.
// Output element (a, c) of an item sits at a + rA*c, or at c + rC*a when transposed;
// positions rA*rC .. out_stride-1 are zero padding.  One thread per output element
// (consecutive threads: consecutive elements, so the L reads coalesce and the R reads
// broadcast).  Small element counts: 32-bit indices with multiply-high divisions.
struct MergeDivs {
  FastDiv os, nL, rA, rC;
};

template <typename real, bool BF>
__global__ void k_merge32(const real* __restrict__ L, int64_t Ls, const int32_t* __restrict__ Llist,
                          uint32_t nL, int rA, int rB, const real* __restrict__ R, int64_t Rs,
                          const int32_t* __restrict__ Rlist, uint32_t total, int rC,
                          void* __restrict__ out, void* __restrict__ out_lo, uint32_t out_stride,
                          int transpose_out, MergeDivs dv) {
  const int used = rA * rC;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const uint32_t item = dv.os.div(t);
    const int e = (int)(t - item * out_stride);
    real acc = real(0);
    if (e < used) {
      int a, c;
      if (transpose_out) { a = (int)dv.rC.div((uint32_t)e); c = e - a * rC; }
      else { c = (int)dv.rA.div((uint32_t)e); a = e - c * rA; }
      const uint32_t j = dv.nL.div(item), l = item - j * nL;
      const real* Lp = L + (Llist ? (int64_t)Llist[l] : (int64_t)l) * Ls;
      const real* Rp = R + (Rlist ? (int64_t)Rlist[j] : (int64_t)j) * Rs;
      // in order over b; unrolled so that the operand loads of a group are in flight together
#pragma unroll 8
      for (int b = 0; b < rB; ++b) acc = fma(Lp[a + rA * b], Rp[b + rB * c], acc);
    }
    put<real, BF>(out, out_lo, (int64_t)t, acc);
  }
}

// Natural layout with rA, out_stride and the L item stride multiples of 4 (FP32): one
// thread per 4 consecutive rows a of an output column, one 16-byte L read per b.
template <bool BF>
__global__ void k_merge4(const float* __restrict__ L, int64_t Ls, const int32_t* __restrict__ Llist,
                         uint32_t nL, int rA, int rB, const float* __restrict__ R, int64_t Rs,
                         const int32_t* __restrict__ Rlist, uint32_t total4, int rC,
                         void* __restrict__ out, void* __restrict__ out_lo, uint32_t os4,
                         MergeDivs dv) {
  const int used = rA * rC;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total4; t += gridDim.x * blockDim.x) {
    const uint32_t item = dv.os.div(t);
    const int e = 4 * (int)(t - item * os4);
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (e < used) {
      const int c = (int)dv.rA.div((uint32_t)e);
      const int a = e - c * rA;
      const uint32_t j = dv.nL.div(item), l = item - j * nL;
      const float* Lp = L + (Llist ? (int64_t)Llist[l] : (int64_t)l) * Ls;
      const float* Rp = R + (Rlist ? (int64_t)Rlist[j] : (int64_t)j) * Rs;
#pragma unroll 8
      for (int b = 0; b < rB; ++b) {  // (in order; unrolled: loads of a group overlap)
        const float4 lv = *reinterpret_cast<const float4*>(Lp + a + rA * b);
        const float rv = Rp[b + rB * c];
        acc[0] = fmaf(lv.x, rv, acc[0]);
        acc[1] = fmaf(lv.y, rv, acc[1]);
        acc[2] = fmaf(lv.z, rv, acc[2]);
        acc[3] = fmaf(lv.w, rv, acc[3]);
      }
    }
    if constexpr (BF) {  // four bf16 in one 8-byte store (and four remainders)
      uint16_t hi[4], lo[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        hi[u] = bf16_bits(acc[u]);
        lo[u] = bf16_bits(acc[u] - __uint_as_float((uint32_t)hi[u] << 16));
      }
      reinterpret_cast<uint2*>(out)[t] =
          uint2{(uint32_t)hi[0] | ((uint32_t)hi[1] << 16), (uint32_t)hi[2] | ((uint32_t)hi[3] << 16)};
      if (out_lo)
        reinterpret_cast<uint2*>(out_lo)[t] = uint2{(uint32_t)lo[0] | ((uint32_t)lo[1] << 16),
                                                    (uint32_t)lo[2] | ((uint32_t)lo[3] << 16)};
    } else {
      reinterpret_cast<float4*>(out)[t] = float4{acc[0], acc[1], acc[2], acc[3]};
    }
  }
}

template <typename real, bool BF>
__global__ void k_merge(const real* __restrict__ L, int64_t Ls, const int32_t* __restrict__ Llist,
                        int64_t nL, int rA, int rB, const real* __restrict__ R, int64_t Rs,
                        const int32_t* __restrict__ Rlist, int64_t nR, int rC,
                        void* __restrict__ out, void* __restrict__ out_lo, int64_t out_stride,
                        int transpose_out) {
  const int64_t total = nL * nR * out_stride;
  const int used = rA * rC;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t item = t / out_stride;
    const int e = (int)(t - item * out_stride);
    real acc = real(0);
    if (e < used) {
      int a, c;
      if (transpose_out) { c = e % rC; a = e / rC; }
      else { a = e % rA; c = e / rA; }
      const int64_t l = item % nL, j = item / nL;
      const real* Lp = L + (Llist ? (int64_t)Llist[l] : l) * Ls;
      const real* Rp = R + (Rlist ? (int64_t)Rlist[j] : j) * Rs;
#pragma unroll 8
      for (int b = 0; b < rB; ++b) acc = fma(Lp[a + rA * b], Rp[b + rB * c], acc);
    }
    put<real, BF>(out, out_lo, t, acc);
  }
}

// The common square case (rA = rB = rC = R = 8, FP32 inputs): thread (item, c) forms the
// R outputs a + R c (a < R) of its item, (L_l . R_j)[:, c], from L_l and column c of R_j;
// the sums run over b in order, as in the kernels above, so the results are the same.
// R consecutive threads write one item row, so every store instruction of a wave writes
// one contiguous run.  With STAGE the nL left items are first copied to LDS (row stride
// R*R + 4 floats, so that the eight items a wave reads fall in different banks), and a
// work-group then forms kMergeReps consecutive groups of 256 / R items, so that one copy
// serves them all.
constexpr int kMergeReps = 4;
template <bool BF, int R, bool STAGE>
__global__ __launch_bounds__(256) void k_merge_item(
    const float* __restrict__ L, int64_t Ls, const int32_t* __restrict__ Llist, uint32_t nL,
    const float* __restrict__ Rm, int64_t Rs, const int32_t* __restrict__ Rlist, uint32_t nItems,
    void* __restrict__ out, void* __restrict__ out_lo, int os, FastDiv nLdiv) {
  static_assert(R == 8, "one 16-byte bf16 group per thread");
  extern __shared__ __align__(16) float Lsh[];
  constexpr int LS = R * R + 4;
  if constexpr (STAGE) {
    for (uint32_t e = threadIdx.x; e < nL * (R * R / 4); e += 256) {
      const uint32_t li = e / (R * R / 4), q = e - li * (R * R / 4);
      const float4 v = *reinterpret_cast<const float4*>(
          L + (Llist ? (int64_t)Llist[li] : (int64_t)li) * Ls + 4 * q);
      *reinterpret_cast<float4*>(Lsh + li * LS + 4 * q) = v;
    }
    __syncthreads();
  }
  constexpr int reps = STAGE ? kMergeReps : 1;
#pragma unroll
  for (int rp = 0; rp < reps; ++rp) {
  const uint64_t t = ((uint64_t)blockIdx.x * reps + rp) * 256u + threadIdx.x;
  const uint32_t item = (uint32_t)(t / R), c = (uint32_t)(t % R);
  if (item >= nItems) return;
  const uint32_t j = nLdiv.div(item), l = item - j * nL;
  const float* Lp = STAGE ? Lsh + l * LS : L + (Llist ? (int64_t)Llist[l] : (int64_t)l) * Ls;
  const float* Rp = Rm + (Rlist ? (int64_t)Rlist[j] : (int64_t)j) * Rs + R * c;
  float r[R];
#pragma unroll
  for (int i = 0; i < R / 4; ++i) {
    const float4 v = reinterpret_cast<const float4*>(Rp)[i];
    r[4 * i] = v.x; r[4 * i + 1] = v.y; r[4 * i + 2] = v.z; r[4 * i + 3] = v.w;
  }
  float acc[R];
#pragma unroll
  for (int a = 0; a < R; ++a) acc[a] = 0.f;
#pragma unroll
  for (int b = 0; b < R; ++b) {
#pragma unroll
    for (int a4 = 0; a4 < R / 4; ++a4) {
      const float4 v = *reinterpret_cast<const float4*>(Lp + R * b + 4 * a4);
      acc[4 * a4] = fmaf(v.x, r[b], acc[4 * a4]);
      acc[4 * a4 + 1] = fmaf(v.y, r[b], acc[4 * a4 + 1]);
      acc[4 * a4 + 2] = fmaf(v.z, r[b], acc[4 * a4 + 2]);
      acc[4 * a4 + 3] = fmaf(v.w, r[b], acc[4 * a4 + 3]);
    }
  }
  // outputs 8c .. 8c + 7 of the item row; the R values past R * R up to os are zeros,
  // written by the threads c < (os - R * R) / 8
  if constexpr (BF) {
    uint32_t hw[4] = {0u, 0u, 0u, 0u}, lw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint16_t hi = bf16_bits(acc[u]);
      const uint16_t lo = bf16_bits(acc[u] - __uint_as_float((uint32_t)hi << 16));
      hw[u >> 1] |= (uint32_t)hi << ((u & 1) * 16);
      lw[u >> 1] |= (uint32_t)lo << ((u & 1) * 16);
    }
    uint16_t* o = static_cast<uint16_t*>(out) + (int64_t)item * os;
    *reinterpret_cast<uint4*>(o + 8 * c) = uint4{hw[0], hw[1], hw[2], hw[3]};
    if (out_lo) {
      uint16_t* ol = static_cast<uint16_t*>(out_lo) + (int64_t)item * os;
      *reinterpret_cast<uint4*>(ol + 8 * c) = uint4{lw[0], lw[1], lw[2], lw[3]};
    }
    for (int z = R * R + 8 * (int)c; z < os; z += 8 * R) {
      *reinterpret_cast<uint4*>(o + z) = uint4{0u, 0u, 0u, 0u};
      if (out_lo)
        *reinterpret_cast<uint4*>(static_cast<uint16_t*>(out_lo) + (int64_t)item * os + z) =
            uint4{0u, 0u, 0u, 0u};
    }
  } else {
    float* o = static_cast<float*>(out) + (int64_t)item * os;
    *reinterpret_cast<float4*>(o + 8 * c) = float4{acc[0], acc[1], acc[2], acc[3]};
    *reinterpret_cast<float4*>(o + 8 * c + 4) = float4{acc[4], acc[5], acc[6], acc[7]};
    for (int z = R * R + 8 * (int)c; z < os; z += 8 * R) {
      *reinterpret_cast<float4*>(o + z) = float4{0.f, 0.f, 0.f, 0.f};
      *reinterpret_cast<float4*>(o + z + 4) = float4{0.f, 0.f, 0.f, 0.f};
    }
  }
  }
}

template <typename real, bool BF>
static void merge_idx(dim3 g, dim3 b, hipStream_t st, bool small, const ItemRef& L, int64_t nL,
                      int rA, int rB, const ItemRef& R, int64_t nR, int rC, void* out,
                      void* out_lo, int64_t out_stride, int transpose_out) {
  if constexpr (sizeof(real) == 4) {
    const uintptr_t ua = reinterpret_cast<uintptr_t>(out), ula = reinterpret_cast<uintptr_t>(out_lo);
    // (large tables only: with few items the element-parallel kernel below is faster)
    if (!transpose_out && rA == 8 && rB == 8 && rC == 8 && nL * nR >= 32768 &&
        nL * nR < ((int64_t)1 << 28) &&
        out_stride >= 64 && out_stride % 8 == 0 && L.stride % 4 == 0 && R.stride % 4 == 0 &&
        reinterpret_cast<uintptr_t>(L.ptr) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(R.ptr) % 16 == 0 && ua % 16 == 0 && ula % 16 == 0) {
      const uint32_t items = (uint32_t)(nL * nR);
      const size_t lds = (size_t)nL * (64 + 4) * sizeof(float);
      const unsigned ng = (unsigned)(((uint64_t)items * 8 + 255) / 256);
      if ((int64_t)lds <= 32768) {
        hipLaunchKernelGGL((k_merge_item<BF, 8, true>), dim3((ng + kMergeReps - 1) / kMergeReps), b,
                           lds, st,
                           (const float*)L.ptr, L.stride, L.list, (uint32_t)nL,
                           (const float*)R.ptr, R.stride, R.list, items, out, out_lo,
                           (int)out_stride, FastDiv((uint32_t)nL));
      } else {
        hipLaunchKernelGGL((k_merge_item<BF, 8, false>), dim3(ng), b, 0, st,
                           (const float*)L.ptr, L.stride, L.list, (uint32_t)nL,
                           (const float*)R.ptr, R.stride, R.list, items, out, out_lo,
                           (int)out_stride, FastDiv((uint32_t)nL));
      }
      return;
    }
    if (small && !transpose_out && rA % 4 == 0 && out_stride % 4 == 0 && L.stride % 4 == 0 &&
        reinterpret_cast<uintptr_t>(L.ptr) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(out) % (BF ? 8 : 16) == 0 &&
        reinterpret_cast<uintptr_t>(out_lo) % 8 == 0) {
      MergeDivs dv;
      dv.os = FastDiv((uint32_t)(out_stride / 4));
      dv.nL = FastDiv((uint32_t)nL);
      dv.rA = FastDiv((uint32_t)rA);
      const uint32_t total4 = (uint32_t)(nL * nR * out_stride / 4);
      dim3 g4((unsigned)((total4 + 255) / 256 < (1u << 20) ? (total4 + 255) / 256 : (1u << 20)));
      hipLaunchKernelGGL((k_merge4<BF>), g4, b, 0, st, (const float*)L.ptr, L.stride, L.list,
                         (uint32_t)nL, rA, rB, (const float*)R.ptr, R.stride, R.list, total4, rC,
                         out, out_lo, (uint32_t)(out_stride / 4), dv);
      return;
    }
  }
  if (small) {
    MergeDivs dv;
    dv.os = FastDiv((uint32_t)out_stride);
    dv.nL = FastDiv((uint32_t)nL);
    dv.rA = FastDiv((uint32_t)rA);
    dv.rC = FastDiv((uint32_t)rC);
    hipLaunchKernelGGL((k_merge32<real, BF>), g, b, 0, st, (const real*)L.ptr, L.stride, L.list,
                       (uint32_t)nL, rA, rB, (const real*)R.ptr, R.stride, R.list,
                       (uint32_t)(nL * nR * out_stride), rC, out, out_lo, (uint32_t)out_stride,
                       transpose_out, dv);
  } else {
    hipLaunchKernelGGL((k_merge<real, BF>), g, b, 0, st, (const real*)L.ptr, L.stride, L.list, nL,
                       rA, rB, (const real*)R.ptr, R.stride, R.list, nR, rC, out, out_lo,
                       out_stride, transpose_out);
  }
}

hipError_t launch_merge(int dtype, ItemRef L, int64_t nL, int rA, int rB, ItemRef R, int64_t nR,
                        int rC, void* out, int64_t out_stride, int transpose_out, hipStream_t st,
                        bool bf16_out, void* out_lo) {
  const int64_t total = nL * nR * out_stride;
  if (total <= 0) return hipSuccess;
  const int grid = grid_for(total, 256);
  const bool small = total + (int64_t)grid * 256 < ((int64_t)1 << 32);
  dim3 g(grid), b(256);
  if (bf16_out) {
    if (dtype != 0) return hipErrorInvalidValue;
    merge_idx<float, true>(g, b, st, small, L, nL, rA, rB, R, nR, rC, out, out_lo, out_stride,
                           transpose_out);
  } else if (dtype == 0) {
    merge_idx<float, false>(g, b, st, small, L, nL, rA, rB, R, nR, rC, out, nullptr, out_stride,
                            transpose_out);
  } else {
    merge_idx<double, false>(g, b, st, small, L, nL, rA, rB, R, nR, rC, out, nullptr, out_stride,
                             transpose_out);
  }
  return hipGetLastError();
}

// Copy items (optionally through an index list), optionally transposed, zero padded.
template <typename real, bool BF>
__global__ void k_pack(const real* __restrict__ in, int64_t is, const int32_t* __restrict__ list,
                       int64_t n, int rA, int rB, void* __restrict__ out,
                       void* __restrict__ out_lo, int64_t out_stride, int transpose_out) {
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
    put<real, BF>(out, out_lo, t, v);
  }
}

// ---------------------------------------------------------------- whole-tensor product
// The full reconstruction as one product of the two subchain tables of core 0: with rows
// (i_0, B modes) and columns (C modes) in little-endian order, entry (row, col) of
// T V^T is x at linear index row + nrows * col, so the column-major tensor is the
// column-major nrows x ncols product.  64 x 64 output tiles, the shared dimension staged
// through LDS 32 at a time; each thread holds a 4 x 4 block (4 consecutive rows of 4
// columns) and stores its rows as one contiguous run.

template <typename real>
__global__ __launch_bounds__(256) void k_table_product(const real* __restrict__ T, const real* __restrict__ V,
                                                       int64_t nrows, int64_t ncols, int RRP, int64_t nbr,
                                                       real* __restrict__ out) {
  constexpr int TM = 64, KC = 32;
  __shared__ real Ts[KC][TM + 1];
  __shared__ real Vs[KC][TM + 1];
  const int64_t br = blockIdx.x % nbr, bc = blockIdx.x / nbr;
  const int64_t r0 = br * TM, c0 = bc * TM;
  const int tr = threadIdx.x & 15, tc = threadIdx.x >> 4;
  real acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = real(0);
  for (int k0 = 0; k0 < RRP; k0 += KC) {
    // 64 items x 32 values of each table, 8 per thread, consecutive threads along k
    for (int e = threadIdx.x; e < TM * KC; e += 256) {
      const int it = e / KC, kk = e % KC;
      const int k = k0 + kk;
      const int64_t r = r0 + it, c = c0 + it;
      Ts[kk][it] = (r < nrows && k < RRP) ? T[r * RRP + k] : real(0);
      Vs[kk][it] = (c < ncols && k < RRP) ? V[c * RRP + k] : real(0);
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < KC; ++kk) {
      real a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = Ts[kk][4 * tr + i];
        b[i] = Vs[kk][4 * tc + i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t c = c0 + 4 * tc + j;
    if (c >= ncols) continue;
    real* o = out + c * nrows;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = r0 + 4 * tr + i;
      if (r < nrows) o[r] = acc[i][j];
    }
  }
}

hipError_t launch_table_product(int dtype, const void* T, const void* V, int64_t nrows, int64_t ncols,
                                int RRP, void* out, hipStream_t st) {
  if (nrows <= 0 || ncols <= 0) return hipSuccess;
  const int64_t nbr = (nrows + 63) / 64, nbc = (ncols + 63) / 64;
  if (nbr * nbc >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
  const dim3 g((unsigned)(nbr * nbc)), b(256);
  if (dtype != 0)  // FP64
    hipLaunchKernelGGL(k_table_product<double>, g, b, 0, st, (const double*)T, (const double*)V, nrows, ncols,
                       RRP, nbr, (double*)out);
  else
    hipLaunchKernelGGL(k_table_product<float>, g, b, 0, st, (const float*)T, (const float*)V, nrows, ncols,
                       RRP, nbr, (float*)out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- sampled-fibre chains
// Column table of a uniform row sample: every sampled column n carries its own multi-index,
// so the product of the N - 1 slices is formed per column (no shared partial products).
// One thread per (column, row a of the product): the row vector is carried through the
// chain in registers (ranks <= 16) and written in the transposed table layout.

struct ChainArgs {
  const void* cores[kMaxN];
  int ranks[kMaxN];
  int64_t dims[kMaxN], strides[kMaxN];
  int N, k;
  const int64_t* off;
  int64_t J;
  void* out;
  int64_t out_stride;
};

template <typename real>
__global__ __launch_bounds__(256) void k_chain_cols(ChainArgs a) {
  const int N = a.N, k = a.k;
  const int m0 = (k + 1) % N;
  const int rs = a.ranks[m0], rk = a.ranks[k];
  const int64_t total = a.J * rs;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = t / rs;
    const int ar = (int)(t - n * rs);
    const int64_t off = a.off[n];
    real v[kMaxRank], w[kMaxRank];
    {  // row ar of the first slice Z_{k+1}(i_{k+1})
      const int r0 = rs, r1 = a.ranks[(m0 + 1) % N];
      const int64_t i = (off / a.strides[m0]) % a.dims[m0];
      const real* Z = (const real*)a.cores[m0] + i * (int64_t)r0 * r1;
#pragma unroll
      for (int c = 0; c < kMaxRank; ++c) v[c] = c < r1 ? Z[ar + r0 * c] : real(0);
    }
    for (int s = 2; s < N; ++s) {  // times Z_m(i_m), m = k+2, ..., k-1
      const int m = (k + s) % N;
      const int r0 = a.ranks[m], r1 = a.ranks[(m + 1) % N];
      const int64_t i = (off / a.strides[m]) % a.dims[m];
      const real* Z = (const real*)a.cores[m] + i * (int64_t)r0 * r1;
#pragma unroll
      for (int c = 0; c < kMaxRank; ++c) {
        real acc = real(0);
#pragma unroll
        for (int b = 0; b < kMaxRank; ++b)
          if (b < r0 && c < r1) acc = fma(v[b], Z[b + r0 * c], acc);
        w[c] = acc;
      }
#pragma unroll
      for (int c = 0; c < kMaxRank; ++c) v[c] = w[c];
    }
    real* o = (real*)a.out + n * a.out_stride;
#pragma unroll
    for (int c = 0; c < kMaxRank; ++c)
      if (c < rk) o[ar * rk + c] = v[c];
    if (ar == rs - 1)
      for (int64_t e = (int64_t)rs * rk; e < a.out_stride; ++e) o[e] = real(0);
  }
}

hipError_t launch_chain_cols(int dtype, const void* const* cores, int N, int k, const int32_t* ranks,
                             const int64_t* dims, const int64_t* strides, const int64_t* off,
                             int64_t J, void* out, int64_t out_stride, hipStream_t st) {
  if (J <= 0) return hipSuccess;
  ChainArgs a;
  for (int j = 0; j < kMaxN; ++j) {
    a.cores[j] = j < N ? cores[j] : nullptr;
    a.ranks[j] = j < N ? ranks[j] : 1;
    a.dims[j] = j < N ? dims[j] : 1;
    a.strides[j] = j < N ? strides[j] : 1;
  }
  a.N = N;
  a.k = k;
  a.off = off;
  a.J = J;
  a.out = out;
  a.out_stride = out_stride;
  const int64_t total = J * ranks[(k + 1) % N];
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65535);
  if (dtype != 0)  // FP64
    hipLaunchKernelGGL(k_chain_cols<double>, dim3(blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_chain_cols<float>, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_pack(int dtype, ItemRef in, int64_t n, int rA, int rB, void* out,
                       int64_t out_stride, int transpose_out, hipStream_t st, bool bf16_out,
                       void* out_lo) {
  const int64_t total = n * out_stride;
  if (total <= 0) return hipSuccess;
  dim3 g(grid_for(total, 256)), b(256);
  if (bf16_out) {
    if (dtype != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_pack<float, true>), g, b, 0, st, (const float*)in.ptr, in.stride, in.list,
                       n, rA, rB, out, out_lo, out_stride, transpose_out);
  } else if (dtype == 0) {
    hipLaunchKernelGGL((k_pack<float, false>), g, b, 0, st, (const float*)in.ptr, in.stride,
                       in.list, n, rA, rB, out, nullptr, out_stride, transpose_out);
  } else {
    hipLaunchKernelGGL((k_pack<double, false>), g, b, 0, st, (const double*)in.ptr, in.stride,
                       in.list, n, rA, rB, out, nullptr, out_stride, transpose_out);
  }
  return hipGetLastError();
}

// S[0][t] = sum over the column-group partials c of S[c][t], fixed order, in place; four
// elements per thread (n is a multiple of 4: rows of RRP, RRP a multiple of 4).
// Many partials of a short S (small, sketched updates): the partials are split over the
// kSumLanes threads of an element group, each summing c = lane, lane + kSumLanes, ... in
// order, then combined by a fixed tree in LDS; the threads of a group read different
// partials, so the loads of one element are in flight together.
constexpr int kSumLanes = 16;

template <typename real>
__global__ __launch_bounds__(256) void k_sum_partials(real* __restrict__ S, int n_ct, int64_t n) {
  using V4 = typename std::conditional<sizeof(real) == 4, float4, double4>::type;
  const int64_t n4 = n / 4;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n4;
       t += (int64_t)gridDim.x * blockDim.x) {
    V4 acc = reinterpret_cast<const V4*>(S)[t];
#pragma unroll 4
    for (int c = 1; c < n_ct; ++c) {
      const V4 v = reinterpret_cast<const V4*>(S + (int64_t)c * n)[t];
      acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
    reinterpret_cast<V4*>(S)[t] = acc;
  }
}

template <typename real>
__global__ __launch_bounds__(256) void k_sum_partials_split(real* __restrict__ S, int n_ct, int64_t n) {
  using V4 = typename std::conditional<sizeof(real) == 4, float4, double4>::type;
  __shared__ V4 red[256];
  const int64_t n4 = n / 4;
  const int lane = threadIdx.x % kSumLanes;
  const int64_t t = blockIdx.x * (int64_t)(256 / kSumLanes) + threadIdx.x / kSumLanes;
  V4 acc;
  acc.x = acc.y = acc.z = acc.w = real(0);
  if (t < n4)
    for (int c = lane; c < n_ct; c += kSumLanes) {
      const V4 v = reinterpret_cast<const V4*>(S + (int64_t)c * n)[t];
      acc.x += v.x; acc.y += v.y; acc.z += v.z; acc.w += v.w;
    }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kSumLanes / 2; o > 0; o >>= 1) {
    if (lane < o) {
      V4 a = red[threadIdx.x];
      const V4 b = red[threadIdx.x + o];
      a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
      red[threadIdx.x] = a;
    }
    __syncthreads();
  }
  if (lane == 0 && t < n4) reinterpret_cast<V4*>(S)[t] = red[threadIdx.x];
}

hipError_t launch_sum_partials(int dtype, void* S, int n_ct, int64_t n, hipStream_t st) {
  if (n_ct <= 1 || n <= 0) return hipSuccess;
  if (n % 4 != 0) return hipErrorInvalidValue;
  dim3 b(256);
  // too few float4 elements to fill the device one per thread: split the partials
  if (n / 4 < 64 * 1024 && n_ct >= 2 * kSumLanes) {
    dim3 g((unsigned)((n / 4 + (256 / kSumLanes) - 1) / (256 / kSumLanes)));
    if (dtype == 0)
      hipLaunchKernelGGL(k_sum_partials_split<float>, g, b, 0, st, (float*)S, n_ct, n);
    else
      hipLaunchKernelGGL(k_sum_partials_split<double>, g, b, 0, st, (double*)S, n_ct, n);
    return hipGetLastError();
  }
  dim3 g(grid_for(n / 4, 256, 8192));
  if (dtype == 0)
    hipLaunchKernelGGL(k_sum_partials<float>, g, b, 0, st, (float*)S, n_ct, n);
  else
    hipLaunchKernelGGL(k_sum_partials<double>, g, b, 0, st, (double*)S, n_ct, n);
  return hipGetLastError();
}

// D(i_k)[a, b] = sum_{m_B} sum_c St(i_k + I_k m_B)[a + r_k c] * U(m_B)[b + r_k1 c]
// (St^T U^T of the two-factor split of the gradient); St is the summed row factor of the
// gradient pass.  U.ptr == nullptr: no B modes, U = identity (r_s = r_k1), D(i_k) = St(i_k).
// A split-K product: grid (pair tiles, nchunk); thread = one (i_k, a) pair, holding the
// r_k1 outputs D(i_k)[a, :] in registers while it walks the m_B of its chunk, with the
// next m_B's S values (summed over the n_ct column-group partials, pstride apart) loaded
// one step ahead.  The U item of an m_B is shared through LDS (double buffered, one
// barrier per m_B).  Partials per chunk go to part[chunk][i_k][a + r_k b].
template <typename real, int MAXR>
__global__ __launch_bounds__(256) void k_contract(const real* __restrict__ S, int RRP, int n_ct,
                                                  int64_t pstride, int64_t Ik, int64_t nB,
                                                  int r_k, int r_s, int r_k1,
                                                  const real* __restrict__ U, int64_t Us,
                                                  const int32_t* __restrict__ Ulist,
                                                  double* __restrict__ part, int nchunk) {
  __shared__ real Ua[2][MAXR * MAXR];
  const int64_t pa = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool ok = pa < Ik * r_k;
  const int64_t ik = ok ? pa / r_k : 0;
  const int a = ok ? (int)(pa - ik * r_k) : 0;
  const int chunk = blockIdx.y;
  const int64_t per = (nB + nchunk - 1) / nchunk;
  const int64_t m0 = chunk * per, m1 = min(nB, m0 + per);
  const int US = r_k1 * r_s;
  double acc[MAXR];
#pragma unroll
  for (int b = 0; b < MAXR; ++b) acc[b] = 0.0;
  // S values of the first m_B (all r_s of them, summed over the partials), loaded ahead
  auto load_s = [&](int64_t m, real* sv) {
    const real* sp = S + (ik + Ik * m) * RRP + a;
    // all loads of the step are issued before any is used (n_ct <= 4 here)
    real part_v[4][MAXR];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < MAXR; ++c)
        part_v[q][c] = (ok && c < r_s && m < m1 && q < n_ct) ? sp[(int64_t)q * pstride + r_k * c]
                                                             : real(0);
#pragma unroll
    for (int c = 0; c < MAXR; ++c)
      sv[c] = (part_v[0][c] + part_v[1][c]) + (part_v[2][c] + part_v[3][c]);
  };
  // thread t < US carries element t of the U item, one m_B ahead
  auto load_u = [&](int64_t m) -> real {
    if (!U || m >= m1 || (int)threadIdx.x >= US) return real(0);
    return U[(Ulist ? (int64_t)Ulist[m] : m) * Us + threadIdx.x];
  };
  real cur[MAXR], nxt[MAXR];
  load_s(m0, cur);
  real uval = load_u(m0);
  for (int64_t m = m0; m < m1; ++m) {
    const int buf = (int)((m - m0) & 1);
    if (U && (int)threadIdx.x < US) Ua[buf][threadIdx.x] = uval;  // shared by the group
    uval = load_u(m + 1);
    load_s(m + 1, nxt);  // next m_B's values in flight while this one is used
    __syncthreads();
    if (U) {
#pragma unroll
      for (int c = 0; c < MAXR; ++c) {
        if (c < r_s) {
          const double sv = (double)cur[c];
#pragma unroll
          for (int b = 0; b < MAXR; ++b)
            if (b < r_k1) acc[b] = fma(sv, (double)Ua[buf][b + r_k1 * c], acc[b]);
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < MAXR; ++b)
        if (b < r_k1) acc[b] += (double)cur[b];
    }
#pragma unroll
    for (int c = 0; c < MAXR; ++c) cur[c] = nxt[c];
  }
  if (ok) {
    double* pp = part + ((int64_t)chunk * Ik + ik) * (r_k * r_k1) + a;
#pragma unroll
    for (int b = 0; b < MAXR; ++b)
      if (b < r_k1) pp[r_k * b] = acc[b];
  }
}

template <typename real, int MAXR>
static void contract_r(dim3 g, dim3 b, hipStream_t st, const void* S, int RRP, int n_ct,
                       int64_t pstride, int64_t Ik, int64_t nB, int r_k, int r_s, int r_k1,
                       const ItemRef& U, double* part, int nchunk) {
  hipLaunchKernelGGL((k_contract<real, MAXR>), g, b, 0, st, (const real*)S, RRP, n_ct, pstride,
                     Ik, nB, r_k, r_s, r_k1, (const real*)U.ptr, U.stride, U.list, part, nchunk);
}

template <typename real>
static void contract_real(dim3 g, dim3 b, hipStream_t st, const void* S, int RRP, int n_ct,
                          int64_t pstride, int64_t Ik, int64_t nB, int r_k, int r_s, int r_k1,
                          const ItemRef& U, double* part, int nchunk) {
  const int mr = r_s > r_k1 ? r_s : r_k1;  // unroll bound: the smallest of 4, 8, 16 that fits
  if (mr <= 4) contract_r<real, 4>(g, b, st, S, RRP, n_ct, pstride, Ik, nB, r_k, r_s, r_k1, U, part, nchunk);
  else if (mr <= 8) contract_r<real, 8>(g, b, st, S, RRP, n_ct, pstride, Ik, nB, r_k, r_s, r_k1, U, part, nchunk);
  else contract_r<real, 16>(g, b, st, S, RRP, n_ct, pstride, Ik, nB, r_k, r_s, r_k1, U, part, nchunk);
}

// The same contraction for r_k = r_s = r_{k+1} = 8 (FP32 partials, RRP = 64): a work-group
// takes 32 slices i_k and a range of m_B; per m_B it loads the 32 rows of every partial as
// whole contiguous kilobytes, adds the partials in the same order as k_contract, and keeps
// the sum (and the U item) in LDS for the (i_k, a) threads.  Each thread's sums run in the
// same order as in k_contract, so the results are the same.
__global__ __launch_bounds__(256) void k_contract8(const float* __restrict__ S, int n_ct,
                                                   int64_t pstride, int64_t Ik, int64_t nB,
                                                   const float* __restrict__ U, int64_t Us,
                                                   const int32_t* __restrict__ Ulist,
                                                   double* __restrict__ part, int nchunk) {
  constexpr int RS = 72;  // LDS row stride: lanes (i_k, a) read distinct banks
  __shared__ __align__(16) float Ss[2][32 * RS];
  __shared__ float Ush[2][64];
  const int t = threadIdx.x;
  const int64_t ik0 = (int64_t)blockIdx.x * 32;
  const int chunk = blockIdx.y;
  const int64_t per = (nB + nchunk - 1) / nchunk;
  const int64_t m0 = chunk * per, m1 = min(nB, m0 + per);
  const int ikl = t >> 3, a = t & 7;
  const bool ok = ik0 + ikl < Ik;
  // this thread's two 16-byte pieces of the 32 x 64 block: rows f / 16, columns 4 (f % 16)
  float4 pre[2][4];
  float upre = 0.f;
  auto load = [&](int64_t m) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int f = t + 256 * u, row = f >> 4, c4 = f & 15;
      const bool in = m < m1 && ik0 + row < Ik;
      const float* sp = S + (ik0 + row + Ik * m) * 64 + 4 * c4;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        pre[u][q] = (in && q < n_ct) ? *reinterpret_cast<const float4*>(sp + (int64_t)q * pstride)
                                     : float4{0.f, 0.f, 0.f, 0.f};
    }
    if (t < 64) upre = m < m1 ? U[(Ulist ? (int64_t)Ulist[m] : m) * Us + t] : 0.f;
  };
  double acc[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) acc[b] = 0.0;
  load(m0);
  for (int64_t m = m0; m < m1; ++m) {
    const int buf = (int)((m - m0) & 1);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int f = t + 256 * u, row = f >> 4, c4 = f & 15;
      const float4 p0 = pre[u][0], p1 = pre[u][1], p2 = pre[u][2], p3 = pre[u][3];
      *reinterpret_cast<float4*>(&Ss[buf][row * RS + 4 * c4]) =
          float4{(p0.x + p1.x) + (p2.x + p3.x), (p0.y + p1.y) + (p2.y + p3.y),
                 (p0.z + p1.z) + (p2.z + p3.z), (p0.w + p1.w) + (p2.w + p3.w)};
    }
    if (t < 64) Ush[buf][t] = upre;
    __syncthreads();
    load(m + 1);  // the next m_B's rows in flight while this one is used
    if (ok) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const double sv = (double)Ss[buf][ikl * RS + a + 8 * c];
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[b] = fma(sv, (double)Ush[buf][b + 8 * c], acc[b]);
      }
    }
  }
  if (ok) {
    double* pp = part + ((int64_t)chunk * Ik + ik0 + ikl) * 64 + a;
#pragma unroll
    for (int b = 0; b < 8; ++b) pp[8 * b] = acc[b];
  }
}

hipError_t launch_contract(int dtype, const void* S, int RRP, int n_ct, int64_t pstride,
                           int64_t Ik, int64_t nB, int r_k, int r_s, int r_k1, ItemRef U,
                           double* part, int nchunk, hipStream_t st) {
  if (dtype == 0 && r_k == 8 && r_s == 8 && r_k1 == 8 && RRP == 64 && U.ptr && n_ct >= 1 &&
      n_ct <= 4 && pstride % 4 == 0 && reinterpret_cast<uintptr_t>(S) % 16 == 0) {
    dim3 g((unsigned)((Ik + 31) / 32), (unsigned)nchunk), b(256);
    hipLaunchKernelGGL(k_contract8, g, b, 0, st, (const float*)S, n_ct, pstride, Ik, nB,
                       (const float*)U.ptr, U.stride, U.list, part, nchunk);
    return hipGetLastError();
  }
  if (r_k1 > kMaxRank || r_s > kMaxRank || r_k * r_s > RRP || (!U.ptr && r_s != r_k1) ||
      r_k1 * r_s > 256 || n_ct < 1 || n_ct > 4)
    return hipErrorInvalidValue;
  const int64_t ntile = (Ik * r_k + 255) / 256;
  dim3 g((unsigned)ntile, (unsigned)nchunk), b(256);
  if (dtype == 0)
    contract_real<float>(g, b, st, S, RRP, n_ct, pstride, Ik, nB, r_k, r_s, r_k1, U, part, nchunk);
  else
    contract_real<double>(g, b, st, S, RRP, n_ct, pstride, Ik, nB, r_k, r_s, r_k1, U, part, nchunk);
  return hipGetLastError();
}

// d = scale * (sum over chunks of the contraction partials), fixed order: work-group of
// 1024 threads per 64 outputs, thread (o, g) sums chunks g, g + 16, ..., then the 16
// slices are added in a fixed tree.
template <typename real>
__global__ __launch_bounds__(1024) void k_contract_finish(const double* __restrict__ part,
                                                          int nchunk, int64_t Ik, int RRk,
                                                          double* __restrict__ d64,
                                                          real* __restrict__ d_out, double scale) {
  __shared__ double red[16][64];
  const int64_t n = Ik * RRk;
  const int o = threadIdx.x & 63, gs = threadIdx.x >> 6;
  const int64_t t = (int64_t)blockIdx.x * 64 + o;
  double s = 0.0;
  if (t < n) {
    // loads eight chunks ahead of the (in-order) sums
    int c = gs;
    for (; c + 16 * 7 < nchunk; c += 16 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(c + 16 * u) * n + t];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < nchunk; c += 16) s += part[(int64_t)c * n + t];
  }
  red[gs][o] = s;
  __syncthreads();
  for (int w = 8; w > 0; w >>= 1) {
    if (gs < w) red[gs][o] += red[gs + w][o];
    __syncthreads();
  }
  if (gs == 0 && t < n) {
    const double v = red[0][o] * scale;
    if (d64) d64[t] = v;
    if (d_out) d_out[t] = (real)v;
  }
}

hipError_t launch_contract_finish(int dtype, const double* part, int nchunk, int64_t Ik, int RRk,
                                  double* d64, void* d_out, double scale, hipStream_t st) {
  const int64_t n = Ik * RRk;
  if (n <= 0) return hipSuccess;
  dim3 g((unsigned)((n + 63) / 64)), b(1024);
  if (dtype == 0)
    hipLaunchKernelGGL(k_contract_finish<float>, g, b, 0, st, part, nchunk, Ik, RRk, d64,
                       (float*)d_out, scale);
  else
    hipLaunchKernelGGL(k_contract_finish<double>, g, b, 0, st, part, nchunk, Ik, RRk, d64,
                       (double*)d_out, scale);
  return hipGetLastError();
}

}  // namespace trd

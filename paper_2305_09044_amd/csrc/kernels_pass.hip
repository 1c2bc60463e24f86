// The fused entry pass over the observed entries of one core update.
//
// For core k the observed entries form a matrix whose row is (i_k, first modes of
// the cyclic subchain) and whose column is the remaining modes.  With
//   T(row) = Z_k(i_k) U(m_B)  (r_k x r_s)   and   V(col) = product of the C cores
// (r_s x r_k), the reconstruction of Thm. 1 is xhat = Tr(T V) = <T, V^T> (both stored
// flat in the same a + r_k*c order, zero padded to RRP).  One lane owns one row of a
// 64-row slice and walks that row's entries inside the work-group's column tile,
// whose V^T items sit in LDS.  Modes:
//   kModeGrad : e = x - xhat, w = exp(-e^2/2s^2) (eq. 7), S_ct(row) = sum w e V^T(col) over
//               the tile ct (the row factor of d in eq. 9, one partial per column tile),
//               plus loss / weighted-LS / count sums.
//   kModeLS   : q = <TH(row), V^T(col)> with TH = H(i_k) U(m_B), sum w q^2 (eq. 12).
//   kModeResid: |e| per slot for the kernel-width quantile (padding -> +inf).
//   kModeLoss : sum of sigma^2 (1 - w) (eq. 4 as a loss).
#include "trd_internal.h"

namespace trd {

template <typename real> struct VecOf;
template <> struct VecOf<float> { using T = float4; static constexpr int W = 4; };
template <> struct VecOf<double> { using T = double2; static constexpr int W = 2; };

__device__ __forceinline__ float fast_exp_neg(float u) { return __expf(-u); }
__device__ __forceinline__ double fast_exp_neg(double u) { return exp(-u); }

// 1 - exp(-u) for u >= 0 without cancellation at small u
__device__ __forceinline__ float one_minus_exp_neg(float u, float w) {
  if (u < 0.0625f) {
    // u - u^2/2 + u^3/6 - u^4/24 + u^5/120; truncation below 1e-9 relative at u = 1/16
    float p = fmaf(u, 1.0f / 120.0f, -1.0f / 24.0f);
    p = fmaf(u, p, 1.0f / 6.0f);
    p = fmaf(u, p, -0.5f);
    p = fmaf(u, p, 1.0f);
    return u * p;
  }
  return 1.0f - w;
}
__device__ __forceinline__ double one_minus_exp_neg(double u, double w) { return -expm1(-u); }

// elements per staged item in LDS: RRP rounded up to an odd number of 16-byte units
__host__ __device__ constexpr int lds_item_stride(int RRP, int esize) {
  return ((RRP * esize / 16) % 2 == 1) ? RRP : RRP + 16 / esize;
}

template <typename real, int RC, int MODE>
__global__ __launch_bounds__(kPassThreads, 2) void k_pass(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  real* Vs = reinterpret_cast<real*>(smem_raw);
  using V = typename VecOf<real>::T;
  constexpr int VW = VecOf<real>::W;
  constexpr int RRP = (RC + 3) / 4 * 4;   // storage stride of one table item
  constexpr int NV = RRP / VW;
  // LDS stride of one staged item: an odd number of 16-byte units, so that lanes reading
  // items of different columns at the same offset fall in different banks
  constexpr int SP = lds_item_stride(RRP, (int)sizeof(real));
  constexpr int NVS = SP / VW;
  constexpr bool kHoldV = RRP <= 64;
  constexpr bool kGrad = MODE == kModeGrad || MODE == kModeGradFast;

  // work-group = (column group cg, 256-row group g); it walks the column tiles of its
  // group, restaging V^T items per tile, and keeps the row factor in registers throughout
  const int64_t wg = blockIdx.x;
  const int64_t cg = wg / a.n_rg, g = wg % a.n_rg;
  const int64_t ct_beg = cg * a.cpg;
  const int64_t ct_end = min((int64_t)a.n_ct, ct_beg + a.cpg);

  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = g * kRowsPerWG + threadIdx.x;
  const bool row_ok = row < a.nrows;

  const double sig = *a.sigma;
  const real inv2s2 = isinf(sig) ? real(0) : real(0.5 / (sig * sig));
  const real sig2 = isinf(sig) ? real(0) : real(sig * sig);
  const bool ls_limit = isinf(sig);

  real t[RRP];
  real u[(kGrad || MODE == kModeLS) ? RRP : 1];
#pragma unroll
  for (int j = 0; j < RRP; ++j) t[j] = real(0);
#pragma unroll
  for (int j = 0; j < (int)(sizeof(u) / sizeof(real)); ++j) u[j] = real(0);
  if (row_ok) {
    const V* tp = reinterpret_cast<const V*>(static_cast<const real*>(a.T) + row * RRP);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      V q = tp[v];
      const real* qs = reinterpret_cast<const real*>(&q);
#pragma unroll
      for (int w = 0; w < VW; ++w) t[v * VW + w] = qs[w];
    }
    if constexpr (MODE == kModeLS) {
      const V* hp = reinterpret_cast<const V*>(static_cast<const real*>(a.TH) + row * RRP);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        V q = hp[v];
        const real* qs = reinterpret_cast<const real*>(&q);
#pragma unroll
        for (int w = 0; w < VW; ++w) u[v * VW + w] = qs[w];
      }
    }
  }

  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  real f0 = real(0);  // per-lane line-search sum (converted to double once per lane)
  constexpr int kGroupStride = kWave * kGroup;
  for (int64_t ct = ct_beg; ct < ct_end; ++ct) {
  const int64_t col0 = ct * a.ct_w;
  const int nct = (int)min((int64_t)a.ct_w, a.ncols - col0);
  if (ct > ct_beg) __syncthreads();  // every wave is done with the previous tile
  // stage the column tile's V^T items in LDS
  {
    const V* src = reinterpret_cast<const V*>(static_cast<const real*>(a.V) + col0 * RRP);
    V* dst = reinterpret_cast<V*>(Vs);
    const int n = nct * NV;
    for (int i = threadIdx.x; i < n; i += kPassThreads) dst[(i / NV) * NVS + i % NV] = src[i];
  }
  __syncthreads();
  const int64_t sid = (ct * a.n_rg + g) * 4 + wave;
  const int64_t off = a.slice_off[sid];
  const int len = a.slice_len[sid];
  // this lane's entries: groups of kGroup values / columns, one wide load each
  const real* __restrict__ vbase = static_cast<const real*>(a.vals) + off + lane * kGroup;
  const uint16_t* __restrict__ cbase = a.cols + off + lane * kGroup;
  const int ngroups = len / kGroup;

  auto process = [&](const real x, const int c, const int64_t slot) {
    const V* vp = reinterpret_cast<const V*>(Vs + c * SP);
    real vr[kHoldV ? RRP : 1];
    real xh0 = real(0), xh1 = real(0);
    real q0 = real(0), q1 = real(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      V q = vp[v];
      const real* qs = reinterpret_cast<const real*>(&q);
#pragma unroll
      for (int w = 0; w < VW; ++w) {
        const int j = v * VW + w;
        if (j < RC) {
          if (j & 1) xh1 = fma(t[j], qs[w], xh1); else xh0 = fma(t[j], qs[w], xh0);
          if constexpr (MODE == kModeLS) {
            if (j & 1) q1 = fma(u[j], qs[w], q1); else q0 = fma(u[j], qs[w], q0);
          }
        }
        if constexpr (kHoldV) vr[j] = qs[w];
      }
    }
    const real e = x - (xh0 + xh1);
    const real uu = e * e * inv2s2;
    const real w = ls_limit ? real(1) : fast_exp_neg(uu);
    // importance weight of the entry's column (leverage-sampled rows only)
    real cw = real(1);
    if constexpr (kGrad || MODE == kModeLS) {
      if (a.colw) cw = (real)a.colw[col0 + c];
    }
    if constexpr (kGrad) {
      const real y = w * e * cw;
      if constexpr (kHoldV) {
#pragma unroll
        for (int j = 0; j < RC; ++j) u[j] = fma(y, vr[j], u[j]);
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          V q = vp[v];
          const real* qs = reinterpret_cast<const real*>(&q);
#pragma unroll
          for (int ww = 0; ww < VW; ++ww)
            if (v * VW + ww < RC) u[v * VW + ww] = fma(y, qs[ww], u[v * VW + ww]);
        }
      }
      if constexpr (MODE == kModeGrad) {
        const real l = ls_limit ? real(0.5) * e * e : sig2 * one_minus_exp_neg(uu, w);
        s0 += (double)(l * cw);
        s1 += (double)(w * e * e * cw);
        s2 += 1.0;
      }
    } else if constexpr (MODE == kModeLS) {
      const real q = q0 + q1;
      f0 = fma(w * q * cw, q, f0);
    } else if constexpr (MODE == kModeResid) {
      a.resid[slot] = (float)fabs(e);
    } else {
      const real l = ls_limit ? real(0.5) * e * e : sig2 * one_minus_exp_neg(uu, w);
      s0 += (double)l;
      s2 += 1.0;
    }
  };

  struct Grp {
    V x[kGroup / VW];
    uint4 c;
  };
  auto load_group = [&](int g) {
    Grp r;
    const V* xp = reinterpret_cast<const V*>(vbase + (int64_t)g * kGroupStride);
#pragma unroll
    for (int i = 0; i < kGroup / VW; ++i) r.x[i] = xp[i];
    r.c = *reinterpret_cast<const uint4*>(cbase + (int64_t)g * kGroupStride);
    return r;
  };

  Grp cur;
  if (ngroups > 0) cur = load_group(0);
  for (int g = 0; g < ngroups; ++g) {
    Grp nxt;
    if (g + 1 < ngroups) nxt = load_group(g + 1);  // prefetch one group ahead
    const real* xs = reinterpret_cast<const real*>(cur.x);
    const uint32_t cw[4] = {cur.c.x, cur.c.y, cur.c.z, cur.c.w};
#pragma unroll
    for (int i = 0; i < kGroup; ++i) {
      const int c = (int)((cw[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu);
      const int64_t slot = off + (int64_t)g * kGroupStride + lane * kGroup + i;
      if (c == kPad) {
        if constexpr (MODE == kModeResid) a.resid[slot] = __int_as_float(0x7f800000);
        continue;
      }
      process(xs[i], c, slot);
    }
    cur = nxt;
  }
  }  // column tiles

  if constexpr (MODE == kModeLS) s0 = (double)f0;
  if constexpr (kGrad) {
    // per-column-group partial of the row factor, plain stores (summed in fixed order later)
    if (row_ok) {
      V* sp = reinterpret_cast<V*>(static_cast<real*>(a.S) + (cg * a.nrows + row) * RRP);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        V q;
        real* qs = reinterpret_cast<real*>(&q);
#pragma unroll
        for (int w = 0; w < VW; ++w) qs[w] = u[v * VW + w];
        sp[v] = q;
      }
    }
  }

  // work-group sums of the statistics, fixed order
  __shared__ double red[3][4];
  for (int o = 32; o > 0; o >>= 1) {
    s0 += __shfl_xor(s0, o);
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
    red[2][wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const double* r = red[threadIdx.x];
    a.partials[wg * 3 + threadIdx.x] = (r[0] + r[1]) + (r[2] + r[3]);
  }
}

// compute lengths with their own kernels; other r_k * r_s use the next larger one (the
// table items are zero padded, so the extra terms add nothing)
static const int kRCs[] = {4, 8, 9, 12, 16, 20, 24, 25, 28, 32, 36, 40, 48, 49, 56, 64, 80, 81, 100,
                           112, 128};

int pass_rc(int RR) {
  for (int v : kRCs)
    if (v >= RR) return v;
  return -1;
}

int pass_rrp(int RR) {
  const int rc = pass_rc(RR);
  return rc < 0 ? -1 : (rc + 3) / 4 * 4;
}

bool pass_supported(int RR) { return pass_rc(RR) > 0; }

int64_t pass_ct_w(int dtype, int prec, int RRP) {
  (void)prec;
  const int64_t bytes = dtype == 0 ? 4 : 8;
  // LDS budget of the column tile: two work-groups per CU when the device allows it
  int64_t budget = g_lds_max >= 2 * 65536 ? 65536 : 61440;
  if (budget > g_lds_max - 1024) budget = g_lds_max - 1024;
  int64_t w = budget / (lds_item_stride(RRP, (int)bytes) * bytes);
  if (w < 1) w = 1;
  if (w > 65535) w = 65535;
  return w;
}

template <typename real, int RC>
static hipError_t launch_rc(int mode, const PassArgs& a, hipStream_t st) {
  constexpr int RRP = (RC + 3) / 4 * 4;
  const int64_t nwg = a.n_rg * a.n_cg;
  const size_t lds = (size_t)a.ct_w * lds_item_stride(RRP, (int)sizeof(real)) * sizeof(real);
  dim3 g((unsigned)nwg), b(kPassThreads);
  switch (mode) {
    case kModeGrad: hipLaunchKernelGGL((k_pass<real, RC, kModeGrad>), g, b, lds, st, a); break;
    case kModeGradFast: hipLaunchKernelGGL((k_pass<real, RC, kModeGradFast>), g, b, lds, st, a); break;
    case kModeLS: hipLaunchKernelGGL((k_pass<real, RC, kModeLS>), g, b, lds, st, a); break;
    case kModeResid: hipLaunchKernelGGL((k_pass<real, RC, kModeResid>), g, b, lds, st, a); break;
    default: hipLaunchKernelGGL((k_pass<real, RC, kModeLoss>), g, b, lds, st, a); break;
  }
  return hipGetLastError();
}

template <typename real>
static hipError_t launch_real(int mode, const PassArgs& a, hipStream_t st) {
  switch (pass_rc(a.RR)) {
#define TRD_CASE(R) case R: return launch_rc<real, R>(mode, a, st);
    TRD_CASE(4) TRD_CASE(8) TRD_CASE(9) TRD_CASE(12) TRD_CASE(16) TRD_CASE(20) TRD_CASE(24)
    TRD_CASE(25) TRD_CASE(28) TRD_CASE(32) TRD_CASE(36) TRD_CASE(40) TRD_CASE(48) TRD_CASE(49)
    TRD_CASE(56) TRD_CASE(64) TRD_CASE(80) TRD_CASE(81) TRD_CASE(100) TRD_CASE(112) TRD_CASE(128)
#undef TRD_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pass(int dtype, int prec, int mode, const PassArgs& a, hipStream_t st) {
  (void)prec;
  if (a.n_rg * a.n_cg <= 0) return hipSuccess;
  if (pass_rrp(a.RR) != a.RRP) return hipErrorInvalidValue;
  if (a.cpg < 1 || (int64_t)a.n_cg * a.cpg < a.n_ct || (int64_t)(a.n_cg - 1) * a.cpg >= a.n_ct)
    return hipErrorInvalidValue;
  return dtype == 0 ? launch_real<float>(mode, a, st) : launch_real<double>(mode, a, st);
}

}  // namespace trd

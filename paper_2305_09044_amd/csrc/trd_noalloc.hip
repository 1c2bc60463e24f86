// FGMC Gram matrix (eq. 13) without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that forbid it).
//
// trd_fgmc_gram keeps its Kronecker factors and ring partials in a context's workspace.
// This variant needs no context: its factors and partials live in one file-scope device
// array of fixed size, resolved to a device address once per device with
// hipGetSymbolAddress and passed to the same kernels as that workspace would be.  Every
// element of the array that a call reads it has written first in the same call (the
// factor kernel writes each factor whole, each ring product its whole output), so nothing
// needs clearing between calls.  Calls on one device share the array: calls that overlap
// on one device (two streams, two host threads) race and must be serialised by the caller.
#include <mutex>
#include <string>

#include "../../include/trd.h"
#include "trd_internal.h"

namespace {

// 2 MiB of FP64: the N - 1 factors r_j^2 x r_{j+1}^2 plus, when a factor side exceeds 64,
// two ring partials r_{k+1}^2 x max r_m^2: every shape with ranks <= 12 fits, and rank 16
// at N = 3
constexpr int64_t kScratchDoubles = (2 << 20) / 8;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {nullptr};  // device address of `scratch`, per device
int64_t g_lds[kMaxDevices] = {0};            // largest dynamic LDS per work-group

}  // namespace

using namespace trd;

extern "C" int trd_fgmc_gram_noalloc(int N, const int64_t* dims, const int32_t* ranks, int dtype,
                                     const void* const* cores, int k, double* G_out, void* stream) {
  if (N < 2 || N > kMaxN) return fail_free(TRD_EUNSUPPORTED, "N must be in [2, 8]");
  if (!dims || !ranks || !cores || !G_out) return fail_free(TRD_EINVAL, "NULL argument");
  if (dtype != TRD_F32 && dtype != TRD_F64) return fail_free(TRD_EINVAL, "dtype must be TRD_F32 or TRD_F64");
  if (k < 0 || k >= N) return fail_free(TRD_EINVAL, "k out of range");
  for (int j = 0; j < N; ++j) {
    if (dims[j] < 1) return fail_free(TRD_EINVAL, "dims must be >= 1");
    if (ranks[j] < 1 || ranks[j] > kMaxRank) return fail_free(TRD_EUNSUPPORTED, "ranks must be in [1, 16]");
    if (j != k && !cores[j]) return fail_free(TRD_EINVAL, "cores[" + std::to_string(j) + "] is NULL");
  }
  // scratch plan: factor j at off[j], then the two ring partials
  int64_t off[kMaxN] = {0};
  int64_t need = 0;
  bool fits = true;
  int64_t maxc = 1;
  for (int t = 1; t <= N - 1; ++t) {
    const int j = (k + t) % N;
    const int64_t r0 = (int64_t)ranks[j] * ranks[j], r1 = (int64_t)ranks[(j + 1) % N] * ranks[(j + 1) % N];
    off[j] = need;
    need += r0 * r1;
    fits = fits && r0 <= 64 && r1 <= 64;
    maxc = r1 > maxc ? r1 : maxc;
  }
  const int64_t rows = (int64_t)ranks[(k + 1) % N] * ranks[(k + 1) % N];
  const int64_t part = (N > 2 && !fits) ? rows * maxc : 0;
  const int64_t p0 = need, p1 = need + part;
  need += 2 * part;
  if (need > kScratchDoubles)
    return fail_free(TRD_EUNSUPPORTED, "trd_fgmc_gram_noalloc: this shape needs " + std::to_string(need * 8) +
                                           " bytes of scratch, more than its fixed " +
                                           std::to_string(kScratchDoubles * 8) + " (use trd_fgmc_gram)");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_free(TRD_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail_free(TRD_EUNSUPPORTED, "device index above 63");
  double* base = nullptr;
  int64_t lds = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {  // first call on this device (it is current): resolve the array
      double* p = nullptr;
      e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail_free(TRD_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      int v = 0;
      e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
      if (e != hipSuccess)
        return fail_free(TRD_EDEVICE, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e));
      g_lds[dev] = v;
      g_scratch[dev] = p;
    }
    base = g_scratch[dev];
    lds = g_lds[dev];
  }
  hipStream_t st = (hipStream_t)stream;
  double* K[kMaxN] = {nullptr};
  for (int t = 1; t <= N - 1; ++t) {
    const int j = (k + t) % N;
    K[j] = base + off[j];
    e = launch_kron_factor(dtype, cores[j], ranks[j], dims[j], ranks[(j + 1) % N], K[j], st);
    if (e != hipSuccess) return fail_free(TRD_EDEVICE, std::string("FGMC factor: ") + hipGetErrorString(e));
  }
  e = launch_ring_gram(N, ranks, k, K, base + p0, base + p1, G_out, lds, st);
  if (e != hipSuccess) return fail_free(TRD_EDEVICE, std::string("FGMC ring: ") + hipGetErrorString(e));
  return TRD_OK;
}

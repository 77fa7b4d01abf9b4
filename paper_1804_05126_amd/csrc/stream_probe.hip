// Streaming-bandwidth probe: dst[i] = sum_s src_s[i] over nsrc float64 arrays
// (nsrc reads and one write per element).  A plain
// unit-stride kernel with no stencil, no LDS and no barrier, used to measure
// what this device's HBM delivers to a streaming kernel (the ceiling the
// solver's passes are compared with) and to scale hardware byte counters by a
// kernel of known traffic.
//
// Each thread moves 16 bytes per array per load (two doubles) and keeps
// kUnroll such loads per array in flight; the grid strides over the arrays.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kiops.h"

namespace {

constexpr int kProbeThreads = 256;
constexpr int kUnroll = 4;
constexpr int kProbeMaxSrc = 8;

struct ProbeArgs {
  const double* src[kProbeMaxSrc];
};

typedef double kiops_d2 __attribute__((ext_vector_type(2)));

template <int NS>
__global__ void __launch_bounds__(kProbeThreads) stream_probe_kernel(ProbeArgs a, double* dst, int64_t n2) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  const int64_t chunk = stride * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; base < n2; base += chunk) {
    kiops_d2 acc[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) acc[u] = kiops_d2{0.0, 0.0};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const kiops_d2* p = reinterpret_cast<const kiops_d2*>(a.src[s]);
      kiops_d2 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = base + (int64_t)u * stride;
        v[u] = i < n2 ? p[i] : kiops_d2{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) acc[u] += v[u];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * stride;
      if (i < n2) reinterpret_cast<kiops_d2*>(dst)[i] = acc[u];
    }
  }
}

template <int NS>
hipError_t launch(const ProbeArgs& a, double* dst, int64_t n2, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(stream_probe_kernel<NS>, dim3(blocks), dim3(kProbeThreads), 0, st, a, dst, n2);
  return hipGetLastError();
}

}  // namespace

extern "C" kiops_status kiops_stream_probe(const double* const* src, int nsrc, double* dst, int64_t n,
                                           int blocks, void* hip_stream) {
  if (!src || !dst || nsrc < 1 || nsrc > kProbeMaxSrc || n < 2 || (n & 1) || blocks < 1 || blocks > (1 << 20))
    return KIOPS_ERR_INVALID_ARG;
  ProbeArgs a{};
  for (int s = 0; s < nsrc; ++s) {
    if (!src[s] || (reinterpret_cast<uintptr_t>(src[s]) & 15)) return KIOPS_ERR_INVALID_ARG;
    a.src[s] = src[s];
  }
  if (reinterpret_cast<uintptr_t>(dst) & 15) return KIOPS_ERR_INVALID_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int64_t n2 = n / 2;
  hipError_t e = hipSuccess;
  switch (nsrc) {
    case 1: e = launch<1>(a, dst, n2, blocks, st); break;
    case 2: e = launch<2>(a, dst, n2, blocks, st); break;
    case 3: e = launch<3>(a, dst, n2, blocks, st); break;
    case 4: e = launch<4>(a, dst, n2, blocks, st); break;
    case 5: e = launch<5>(a, dst, n2, blocks, st); break;
    case 6: e = launch<6>(a, dst, n2, blocks, st); break;
    case 7: e = launch<7>(a, dst, n2, blocks, st); break;
    default: e = launch<8>(a, dst, n2, blocks, st); break;
  }
  return e == hipSuccess ? KIOPS_OK : KIOPS_ERR_DEVICE;
}

// Measurement kernel (no paper counterpart): the sustained VALU issue rate of
// the device under the library's own compiler flags (packed float32 off), the
// ceiling of the render kernels' ALU roofline.  Every lane runs 16
// independent dependency chains, so consecutive instructions of a wave never
// wait on each other and the SIMDs stay issue-bound.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ddvr_internal.h"

namespace {

constexpr int kChains = ddvr::kProbeChains;

template <int MODE>
__global__ __launch_bounds__(256) void k_valu_probe(float* out, int iters, float a, float b) {
  float x[kChains];
  uint32_t y[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    x[j] = (float)threadIdx.x * 1e-3f + (float)j;
    y[j] = threadIdx.x * 2654435761u + (uint32_t)j;
  }
  const uint32_t k = __float_as_uint(b);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      if (MODE == 0) x[j] = fmaf(x[j], a, b);
      else y[j] += k;
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += MODE == 0 ? x[j] : (float)y[j];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

namespace ddvr {

int launch_valu_probe(int mode, int blocks, int iters, float* out, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode == 0)
    hipLaunchKernelGGL(k_valu_probe<0>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else
    hipLaunchKernelGGL(k_valu_probe<1>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  return (int)hipGetLastError();
}

}  // namespace ddvr

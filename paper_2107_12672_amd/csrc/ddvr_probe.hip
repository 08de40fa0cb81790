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

// Chain j of a lane runs per round: MODE 0 a float32 FMA, 1 a 32-bit integer
// add, 2 the two alternating over the chains (float and integer work that the
// SIMD may overlap), 3 FMAs alternating with the hardware exp2 (the
// transcendental unit), 4 a float32 multiply then a max (two two-operand
// instructions), 5 a shift then an xor (two integer ones), 6 an FMA then a max,
// 7 float multiplies and integer maxes on alternating chains (no dependence
// between consecutive instructions; an integer max, because a float max of a
// loop-carried value is preceded by a canonicalising max of its own).
template <int MODE>
__global__ __launch_bounds__(256) void k_valu_probe(float* out, int iters, float a, float b) {
  float x[kChains];
  uint32_t y[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    x[j] = (float)threadIdx.x * 1e-3f + (float)j * 1e-2f;
    y[j] = threadIdx.x * 2654435761u + (uint32_t)j;
  }
  const uint32_t k = __float_as_uint(b);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      const bool odd = (j & 1) != 0;
      if (MODE == 0 || ((MODE == 2 || MODE == 3) && !odd)) x[j] = fmaf(x[j], a, b);
      else if (MODE == 1 || MODE == 2) y[j] += k;
      else if (MODE == 3) x[j] = __builtin_amdgcn_exp2f(-x[j]);   // stays in (0, 1]
      else if (MODE == 4) x[j] = fmaxf(x[j] * a, b);
      else if (MODE == 5) y[j] ^= y[j] >> 3;
      else if (MODE == 6) x[j] = fmaxf(fmaf(x[j], a, b), b);
      else if (odd) y[j] = max(y[j], k + (uint32_t)i);
      else x[j] = x[j] * a;
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    const bool odd = (j & 1) != 0;
    s += (MODE == 1 || MODE == 5 || ((MODE == 2 || MODE == 7) && odd)) ? (float)y[j] : x[j];
  }
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

namespace ddvr {

int launch_valu_probe(int mode, int blocks, int iters, float* out, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode == 0)
    hipLaunchKernelGGL(k_valu_probe<0>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else if (mode == 1)
    hipLaunchKernelGGL(k_valu_probe<1>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else if (mode == 2)
    hipLaunchKernelGGL(k_valu_probe<2>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else if (mode == 3)
    hipLaunchKernelGGL(k_valu_probe<3>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else if (mode == 4)
    hipLaunchKernelGGL(k_valu_probe<4>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else if (mode == 5)
    hipLaunchKernelGGL(k_valu_probe<5>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else if (mode == 6)
    hipLaunchKernelGGL(k_valu_probe<6>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  else
    hipLaunchKernelGGL(k_valu_probe<7>, dim3(blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-3f);
  return (int)hipGetLastError();
}

}  // namespace ddvr

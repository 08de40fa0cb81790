// Sustained VALU issue rate of the GPU: 8 independent chains per lane of
// non-packed fp32 FMAs (mode 0) or of 32-bit integer xor-adds (mode 1), all
// lanes active, 8 workgroups of 4 waves per CU.  The reference point of the
// render kernel's ALU roofline.
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o valu_peak valu_peak.hip && ./valu_peak
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
template <int MODE>
__global__ __launch_bounds__(256) void k(float* out, int iters, float a, float b) {
  float x[8];
  int y[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) { x[j] = threadIdx.x * 0.001f + j; y[j] = threadIdx.x + j; }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (MODE == 0) x[j] = fmaf(x[j], a, b);
      else y[j] = (y[j] ^ (int)b) + 7;
    }
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j] + (float)y[j];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
int main() {
  const int blocks = 256 * 8, iters = 20000;
  float* out;
  if (hipMalloc(&out, sizeof(float) * blocks * 256) != hipSuccess) return 1;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  for (int mode = 0; mode < 2; ++mode) {
    for (int rep = 0; rep < 2; ++rep) {
      (void)hipEventRecord(e0);
      if (mode == 0) hipLaunchKernelGGL(k<0>, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f, 0.001f);
      else hipLaunchKernelGGL(k<1>, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999f, 1.0f);
      (void)hipEventRecord(e1);
      (void)hipEventSynchronize(e1);
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double lane_ops = (double)blocks * 256 * iters * 8;
      if (rep) printf("mode %d: %.3f ms, %.3f T lane-ops/s, %.3f wave64-instr per CU per ns\n", mode, ms,
                      lane_ops / (ms * 1e-3) / 1e12, lane_ops / 64 / 256 / (ms * 1e6));
    }
  }
  (void)hipFree(out);
  return 0;
}

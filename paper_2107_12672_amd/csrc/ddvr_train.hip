// HIP kernels (gfx950) of the reconstruction loop around the renderer
// (Weiss & Westermann, arXiv 2107.12672, Sec. 5.1-5.3): the TF smoothing
// prior of eq. (tf-loss) and its counterpart on the densities in 3D, the
// opacity entropy of Sec. 5.1 with its gradient, one Adam step fused with the
// storage cast of the grid and the clearing of its gradient, and the
// trilinear resampling of the multi-resolution schedule.
//
// All of them are elementwise or stencil work bound by HBM bandwidth: one
// element per lane, x fastest (contiguous per wave), 4 elements per lane in
// the Adam step; reductions go through wave shuffles and one float64 atomic
// per workgroup.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "ddvr_internal.h"
#include "ddvr.h"

namespace ddvr {

namespace {

constexpr int kNT = 256;

// float64 sum over the workgroup, added to *out by thread 0
__device__ __forceinline__ void block_add(double x, double* out) {
  __shared__ double part[kNT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kNT / 64; ++w) s += part[w];
    if (s != 0.0) atomicAdd(out, s);
  }
}

// lam/(4 (R-1)) sum_c sum_r (T[r+1][c] - T[r][c])^2 and its gradient
__global__ __launch_bounds__(kNT) void k_tf_prior(const float* tf, int R, float w, float* dtf,
                                                  double* loss) {
  const int i = blockIdx.x * kNT + threadIdx.x;   // entry r*4 + c
  double l = 0.0;
  if (i < 4 * R) {
    const int r = i >> 2;
    float g = 0.0f;
    if (r > 0) g += 2.0f * w * (tf[i] - tf[i - 4]);
    if (r + 1 < R) {
      const float d = tf[i + 4] - tf[i];
      g -= 2.0f * w * d;
      l = (double)w * (double)d * (double)d;
    }
    if (dtf) dtf[i] += g;
  }
  if (loss) block_add(l, loss);
}

// lam * mean over neighbour pairs (V_p - V_q)^2: gradient w 2 sum_q (V_p - V_q)
// per vertex (its own output, no atomics); each pair's square is counted by
// its lower vertex
// (grid-stride over a capped grid: one float64 atomic per workgroup)
__global__ __launch_bounds__(kNT) void k_volume_prior(const float* V, int nx, int ny, int nz,
                                                      float w, float* dV, double* loss) {
  const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  double l = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kNT) {
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / nxy);
    const float c = V[i];
    float g = 0.0f;
    if (x > 0) g += c - V[i - 1];
    if (y > 0) g += c - V[i - nx];
    if (z > 0) g += c - V[i - nxy];
    float sq = 0.0f;
    if (x + 1 < nx) { const float d = V[i + 1] - c; g -= d; sq = fmaf(d, d, sq); }
    if (y + 1 < ny) { const float d = V[i + nx] - c; g -= d; sq = fmaf(d, d, sq); }
    if (z + 1 < nz) { const float d = V[i + nxy] - c; g -= d; sq = fmaf(d, d, sq); }
    if (dV) dV[i] += 2.0f * w * g;
    l += (double)w * (double)sq;
  }
  if (loss) block_add(l, loss);
}

__global__ void k_zero_f64(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// opacity entropy, pass 1: S = sum x, U = sum x log2 x (x > 0)
__global__ __launch_bounds__(kNT) void k_entropy_sums(const float* img, int64_t n, int stride,
                                                      int offset, double* work) {
  double s = 0.0, u = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * kNT) {
    const double x = (double)img[j * stride + offset];
    s += x;
    if (x > 0.0) u += x * log2(x);
  }
  block_add(s, work);
  __syncthreads();
  block_add(u, work + 1);
}

// pass 2: OE = (log2 S - U/S)/log2 N, the normalised entropy -sum p log2 p /
// log2 N with p = x/S; dOE/dx_j = (U/S - log2 x_j)/(S log2 N) (x_j > 0; the
// derivative is unbounded at 0, where none is added)
__global__ __launch_bounds__(kNT) void k_entropy_grad(const float* img, int64_t n, int stride,
                                                      int offset, const double* work,
                                                      double* value, float* dimg, float scale) {
  const double S = work[0], U = work[1];
  const double l2n = log2((double)n);
  if (blockIdx.x == 0 && threadIdx.x == 0 && value) *value = (log2(S) - U / S) / l2n;
  if (!dimg) return;
  const double k = (double)scale / (S * l2n), US = U / S;
  for (int64_t j = (int64_t)blockIdx.x * kNT + threadIdx.x; j < n; j += (int64_t)gridDim.x * kNT) {
    const float x = img[j * stride + offset];
    if (x > 0.0f) dimg[j * stride + offset] += (float)(k * (US - log2((double)x)));
  }
}

// The same two passes over every view of a batch in one launch each (the
// loss of a step plan): work item b = view * chunks + chunk, the chunks of a
// view striding over its pixels.  sums[2v], sums[2v+1] += S_v, U_v.
__global__ __launch_bounds__(kNT) void k_entropy_sums_views(const ViewDesc* views, int chunks,
                                                            int channels, double* sums) {
  const int v = blockIdx.x / chunks, c = blockIdx.x % chunks;
  const ViewDesc& vd = views[v];
  const int64_t n = (int64_t)vd.W * vd.H;
  const int off = channels - 1;
  double s = 0.0, u = 0.0;
  for (int64_t j = (int64_t)c * kNT + threadIdx.x; j < n; j += (int64_t)chunks * kNT) {
    const double x = (double)vd.image[j * channels + off];
    s += x;
    if (x > 0.0) u += x * log2(x);
  }
  block_add(s, sums + 2 * v);
  __syncthreads();
  block_add(u, sums + 2 * v + 1);
}

// pass 2: the view's d_image is WRITTEN (every channel): -scale dOE_v/dalpha
// on the alpha channel (0 where alpha = 0), 0 on the colour channels;
// oe[v] = OE_v and loss += -scale OE_v (chunk 0, thread 0).
__global__ __launch_bounds__(kNT) void k_entropy_grad_views(const ViewDesc* views, int chunks,
                                                            int channels, const double* sums,
                                                            double* oe, double* loss,
                                                            float scale) {
  const int v = blockIdx.x / chunks, c = blockIdx.x % chunks;
  const ViewDesc& vd = views[v];
  const int64_t n = (int64_t)vd.W * vd.H;
  const double S = sums[2 * v], U = sums[2 * v + 1];
  const double l2n = log2((double)n);
  if (c == 0 && threadIdx.x == 0) {
    const double val = (log2(S) - U / S) / l2n;
    oe[v] = val;
    if (loss) atomicAdd(loss, -(double)scale * val);
  }
  float* dimg = const_cast<float*>(vd.d_image);
  const double k = -(double)scale / (S * l2n), US = U / S;
  const int off = channels - 1;
  for (int64_t j = (int64_t)c * kNT + threadIdx.x; j < n; j += (int64_t)chunks * kNT) {
    const float x = vd.image[j * channels + off];
    for (int ch = 0; ch < off; ++ch) dimg[j * channels + ch] = 0.0f;
    dimg[j * channels + off] = x > 0.0f ? (float)(k * (US - log2((double)x))) : 0.0f;
  }
}

__device__ __forceinline__ unsigned short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);   // NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                                  // RNE
  return (unsigned short)(u >> 16);
}

// Adam (Kingma and Ba 2014, Algorithm 1) with bias corrections c1 =
// 1/(1 - beta1^t), c2 = 1/(1 - beta2^t), the clamp [lo, hi], the storage
// copy of the parameters and the clearing of the gradient, 4 elements per
// lane
__global__ __launch_bounds__(kNT) void k_adam(float* x, float* g, float* m, float* v, int64_t n,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2, float lo, float hi, void* store,
                                              int store_dtype, int zero_grad) {
  const int64_t i0 = ((int64_t)blockIdx.x * kNT + threadIdx.x) * 4;
  if (i0 >= n) return;
  const int cnt = (int)(n - i0 < 4 ? n - i0 : 4);
  const uintptr_t al = reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(g) |
                       reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v);
  if (cnt == 4 && (al & 15) == 0 &&
      (!store || (reinterpret_cast<uintptr_t>(store) & (store_dtype == DDVR_F32 ? 15 : 7)) == 0)) {
    // 16-byte loads and stores of 4 elements
    const float4 g4 = *reinterpret_cast<const float4*>(g + i0);
    float4 m4 = *reinterpret_cast<const float4*>(m + i0);
    float4 v4 = *reinterpret_cast<const float4*>(v + i0);
    float4 x4 = *reinterpret_cast<const float4*>(x + i0);
    float* gp = &const_cast<float4&>(g4).x;
    float* mp = &m4.x;
    float* vp = &v4.x;
    float* xp = &x4.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      mp[k] = fmaf(b1, mp[k], (1.0f - b1) * gp[k]);
      vp[k] = fmaf(b2, vp[k], (1.0f - b2) * gp[k] * gp[k]);
      const float xi = xp[k] - lr * (mp[k] * c1) / (sqrtf(vp[k] * c2) + eps);
      xp[k] = fminf(fmaxf(xi, lo), hi);
    }
    *reinterpret_cast<float4*>(x + i0) = x4;
    *reinterpret_cast<float4*>(m + i0) = m4;
    *reinterpret_cast<float4*>(v + i0) = v4;
    if (zero_grad) *reinterpret_cast<float4*>(g + i0) = make_float4(0.f, 0.f, 0.f, 0.f);
    if (store) {
      if (store_dtype == DDVR_BF16) {
        const uint32_t a = (uint32_t)to_bf16(xp[0]) | ((uint32_t)to_bf16(xp[1]) << 16);
        const uint32_t b = (uint32_t)to_bf16(xp[2]) | ((uint32_t)to_bf16(xp[3]) << 16);
        *reinterpret_cast<uint2*>(static_cast<unsigned short*>(store) + i0) = make_uint2(a, b);
      } else if (store_dtype == DDVR_F16) {
        __half* h = static_cast<__half*>(store) + i0;
#pragma unroll
        for (int k = 0; k < 4; ++k) h[k] = __float2half_rn(xp[k]);
      } else {
        *reinterpret_cast<float4*>(static_cast<float*>(store) + i0) = x4;
      }
    }
    return;
  }
  for (int k = 0; k < cnt; ++k) {
    const int64_t i = i0 + k;
    const float gi = g[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    const float mh = mi * c1, vh = vi * c2;
    float xi = x[i] - lr * mh / (sqrtf(vh) + eps);
    xi = fminf(fmaxf(xi, lo), hi);
    x[i] = xi;
    m[i] = mi;
    v[i] = vi;
    if (zero_grad) g[i] = 0.0f;
    if (store) {
      if (store_dtype == DDVR_BF16) static_cast<unsigned short*>(store)[i] = to_bf16(xi);
      else if (store_dtype == DDVR_F16) static_cast<__half*>(store)[i] = __float2half_rn(xi);
      else static_cast<float*>(store)[i] = xi;
    }
  }
}

// dst vertex (i, j, k) at source grid units (i (sx-1)/(dx-1), ...), trilinear
__global__ __launch_bounds__(kNT) void k_resample(const float* src, int C, int sx, int sy,
                                                  int sz, float* dst, int dx, int dy, int dz) {
  const int64_t dxy = (int64_t)dx * dy, n = dxy * dz;
  const int64_t i = (int64_t)blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  const int x = (int)(i % dx), y = (int)((i / dx) % dy), z = (int)(i / dxy);
  const int pos[3] = {x, y, z}, sn[3] = {sx, sy, sz}, dn[3] = {dx, dy, dz};
  int k[3];
  float f[3];
  // the position i (s-1)/(d-1) split exactly into cell and fraction in
  // integers, so the fraction carries only its own rounding
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t num = (int64_t)pos[a] * (sn[a] - 1), den = dn[a] - 1;
    int64_t kk = num / den;
    int64_t rem = num - kk * den;
    if (kk > sn[a] - 2) { kk = sn[a] - 2; rem = den; }   // the last vertex: f = 1
    k[a] = (int)kk;
    f[a] = (float)rem / (float)den;
  }
  // C interleaved channels per vertex, each interpolated on its own
  const int64_t ox = C, oy = (int64_t)C * sx, oz = (int64_t)C * sx * sy;
  const float* b0 = src + k[2] * oz + k[1] * oy + k[0] * ox;
  for (int c = 0; c < C; ++c) {
    const float* b = b0 + c;
    const float c00 = fmaf(f[0], b[ox] - b[0], b[0]);
    const float c10 = fmaf(f[0], b[oy + ox] - b[oy], b[oy]);
    const float c01 = fmaf(f[0], b[oz + ox] - b[oz], b[oz]);
    const float c11 = fmaf(f[0], b[oz + oy + ox] - b[oz + oy], b[oz + oy]);
    const float e0 = fmaf(f[1], c10 - c00, c00);
    const float e1 = fmaf(f[1], c11 - c01, c01);
    dst[i * C + c] = fmaf(f[2], e1 - e0, e0);
  }
}

unsigned blocks_for(int64_t n, int64_t per_block) {
  return (unsigned)((n + per_block - 1) / per_block);
}

}  // namespace

int launch_tf_prior(const float* tf, int R, float lam, float* dtf, double* loss, void* stream) {
  const float w = lam / (4.0f * (float)(R - 1));
  hipLaunchKernelGGL(k_tf_prior, dim3(blocks_for(4 * (int64_t)R, kNT)), dim3(kNT), 0,
                     static_cast<hipStream_t>(stream), tf, R, w, dtf, loss);
  return (int)hipGetLastError();
}

int launch_volume_prior(const float* V, int nx, int ny, int nz, float lam, float* dV,
                        double* loss, void* stream) {
  const int64_t pairs = (int64_t)(nx - 1) * ny * nz + (int64_t)nx * (ny - 1) * nz +
                        (int64_t)nx * ny * (nz - 1);
  const float w = (float)((double)lam / (double)(pairs > 0 ? pairs : 1));
  const int64_t n = (int64_t)nx * ny * nz;
  const unsigned blocks = (unsigned)(blocks_for(n, kNT) < 8192 ? blocks_for(n, kNT) : 8192);
  hipLaunchKernelGGL(k_volume_prior, dim3(blocks), dim3(kNT), 0,
                     static_cast<hipStream_t>(stream), V, nx, ny, nz, w, dV, loss);
  return (int)hipGetLastError();
}

int launch_opacity_entropy(const float* img, int64_t n, int stride, int offset, double* work,
                           double* value, float* dimg, float scale, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, work, 2);
  const unsigned blocks = (unsigned)(blocks_for(n, kNT) < 4096 ? blocks_for(n, kNT) : 4096);
  hipLaunchKernelGGL(k_entropy_sums, dim3(blocks), dim3(kNT), 0, s, img, n, stride, offset, work);
  hipLaunchKernelGGL(k_entropy_grad, dim3(blocks), dim3(kNT), 0, s, img, n, stride, offset,
                     (const double*)work, value, dimg, scale);
  return (int)hipGetLastError();
}

int launch_entropy_views(const ViewDesc* views, int nview, int64_t max_pix, int channels,
                         double* sums, double* oe, double* loss, float scale, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t chunks = blocks_for(max_pix, kNT);
  if (chunks > 256) chunks = 256;
  hipLaunchKernelGGL(k_zero_f64, dim3((2 * nview + 63) / 64), dim3(64), 0, s, sums, 2 * nview);
  hipLaunchKernelGGL(k_entropy_sums_views, dim3((unsigned)(nview * chunks)), dim3(kNT), 0, s,
                     views, (int)chunks, channels, sums);
  hipLaunchKernelGGL(k_entropy_grad_views, dim3((unsigned)(nview * chunks)), dim3(kNT), 0, s,
                     views, (int)chunks, channels, (const double*)sums, oe, loss, scale);
  return (int)hipGetLastError();
}

int launch_adam(float* x, float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                float eps, float c1, float c2, float lo, float hi, void* store, int store_dtype,
                int zero_grad, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 4 * kNT)), dim3(kNT), 0,
                     static_cast<hipStream_t>(stream), x, g, m, v, n, lr, b1, b2, eps, c1, c2,
                     lo, hi, store, store_dtype, zero_grad);
  return (int)hipGetLastError();
}

int launch_resample(const float* src, int channels, int sx, int sy, int sz, float* dst, int dx,
                    int dy, int dz, void* stream) {
  const int64_t n = (int64_t)dx * dy * dz;
  hipLaunchKernelGGL(k_resample, dim3(blocks_for(n, kNT)), dim3(kNT), 0,
                     static_cast<hipStream_t>(stream), src, channels, sx, sy, sz, dst, dx, dy,
                     dz);
  return (int)hipGetLastError();
}

}  // namespace ddvr

// HIP kernels (gfx950): density-from-colour estimation, the second stage of
// the reconstruction pipeline of Weiss & Westermann (arXiv 2107.12672,
// Sec. 5.4).  Every voxel of a pre-shaded colour volume (r, g, b, tau) draws
// candidate densities uniformly at random, maps each through the transfer
// function, and keeps the candidate of least cost
//   C(d) = ||C_T - C(d)||^2 + alpha log(1 + |tau_T - tau(d)|)
//          + beta sum over the 6-neighbourhood (d - d_i)^2,
// the neighbours d_i taken from the previous estimate (none in the first
// sweep; neighbours outside the grid are absent).  Ties keep the lowest
// candidate index.
//
// Mapping to CDNA4: one voxel per lane, x fastest, so the colour, previous
// estimate and output accesses of a wave are contiguous; the TF table is in
// LDS; the candidate loop is pure VALU (ALU-bound): a 64-bit counter add and
// the SplitMix64 finaliser per candidate, the TF lerp, and one log.  The
// neighbour term is evaluated as n (d - m)^2 plus the candidate-independent
// sum of (d_i - m)^2 (m the neighbours' mean), which is added once to the
// reported cost.
//
// Candidates: output n of the SplitMix64 stream (Steele, Lea and Flood,
// OOPSLA 2014) of the seed, mix(seed + (n + 1) gamma) with gamma =
// 0x9e3779b97f4a7c15 and the variant-13 finaliser (shifts 30, 27, 31,
// multipliers 0xbf58476d1ce4e5b9, 0x94d049bb133111eb); candidate k of voxel v
// in sweep t is output (t nvox + v) ncand + k, mapped to [0, 1) as its top
// 24 bits times 2^-24 (exact in float32).
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "ddvr_internal.h"
#include "ddvr.h"

namespace ddvr {

namespace {

typedef float dfc_f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned dfc_u32x2 __attribute__((ext_vector_type(2)));

template <int DT>
__device__ __forceinline__ float4 load_rgbt(const void* p, int64_t i) {
  if constexpr (DT == DDVR_F32) {
    const dfc_f32x4 x = ((const __attribute__((address_space(1))) dfc_f32x4*)p)[i];
    return make_float4(x.x, x.y, x.z, x.w);
  } else {
    const dfc_u32x2 u = ((const __attribute__((address_space(1))) dfc_u32x2*)p)[i];
    if constexpr (DT == DDVR_BF16) {
      return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                         __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
    } else {
      return make_float4(__half2float(__ushort_as_half((unsigned short)(u.x & 0xffffu))),
                         __half2float(__ushort_as_half((unsigned short)(u.x >> 16))),
                         __half2float(__ushort_as_half((unsigned short)(u.y & 0xffffu))),
                         __half2float(__ushort_as_half((unsigned short)(u.y >> 16))));
    }
  }
}

__device__ __forceinline__ uint64_t splitmix_finalise(uint64_t z) {
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

template <int DT>
__global__ __launch_bounds__(256) void k_density_from_color(const DfcParams p) {
  extern __shared__ __align__(16) float dfc_lds[];
  float4* tfl = reinterpret_cast<float4*>(dfc_lds);
  // (the table is copied by floats: its pointer need only be 4-byte aligned)
  for (int k = threadIdx.x; k < 4 * p.R; k += 256) dfc_lds[k] = p.tf[k];
  __syncthreads();

  const int64_t nxy = (int64_t)p.nx * p.ny, nvox = nxy * p.nz;
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = v < nvox;
  bool changed = false;
  if (live) {
    const int x = (int)(v % p.nx);
    const int y = (int)((v / p.nx) % p.ny);
    const int z = (int)(v / nxy);
    const float4 t = load_rgbt<DT>(p.cv, v);
    // neighbours of the previous estimate: count, mean, spread about the mean
    float nb[6];
    int nn = 0;
    if (p.d_prev) {
      if (x > 0) nb[nn++] = p.d_prev[v - 1];
      if (x + 1 < p.nx) nb[nn++] = p.d_prev[v + 1];
      if (y > 0) nb[nn++] = p.d_prev[v - p.nx];
      if (y + 1 < p.ny) nb[nn++] = p.d_prev[v + p.nx];
      if (z > 0) nb[nn++] = p.d_prev[v - nxy];
      if (z + 1 < p.nz) nb[nn++] = p.d_prev[v + nxy];
    }
    float m = 0.0f, spread = 0.0f;
    if (nn > 0) {
      for (int q = 0; q < nn; ++q) m += nb[q];
      m /= (float)nn;
      for (int q = 0; q < nn; ++q) spread = fmaf(nb[q] - m, nb[q] - m, spread);
    }
    const float bn = p.beta * (float)nn;
    // alpha log(1 + x) = (alpha ln 2) log2(1 + x); 1 + x >= 1 is never
    // subnormal, so the hardware log2 needs no range scaling
    const float aln2 = p.alpha * 0.69314718055994531f;
    const float rm1 = (float)(p.R - 1);
    // counter of candidate 0, advanced by gamma per candidate
    constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;
    const uint64_t n0 = ((uint64_t)p.iter * (uint64_t)nvox + (uint64_t)v) * (uint64_t)p.ncand;
    uint64_t ctr = p.seed + (n0 + 1) * kGamma;
    float best = INFINITY, bd = 0.0f;
    for (int k = 0; k < p.ncand; ++k, ctr += kGamma) {
      const float d = (float)(uint32_t)(splitmix_finalise(ctr) >> 40) * 5.9604644775390625e-8f;
      const float u = d * rm1;
      const int j = min((int)u, p.R - 2);
      const float phi = u - (float)j;
      const float4 a = tfl[j], b = tfl[j + 1];
      const float er = t.x - fmaf(phi, b.x - a.x, a.x);
      const float eg = t.y - fmaf(phi, b.y - a.y, a.y);
      const float eb = t.z - fmaf(phi, b.z - a.z, a.z);
      const float et = fabsf(t.w - fmaf(phi, b.w - a.w, a.w));
      float c = fmaf(er, er, fmaf(eg, eg, eb * eb));
      c = fmaf(aln2, __builtin_amdgcn_logf(1.0f + et), c);
      c = fmaf(bn, (d - m) * (d - m), c);
      if (c < best) { best = c; bd = d; }
    }
    p.d_out[v] = bd;
    if (p.cost_out) p.cost_out[v] = fmaf(p.beta, spread, best);
    changed = p.d_prev != nullptr && bd != p.d_prev[v];
  }
  if (p.n_changed) {
    const uint64_t m = __ballot(changed);
    if ((threadIdx.x & 63) == 0 && m)
      atomicAdd(p.n_changed, (unsigned)__popcll((unsigned long long)m));
  }
}

__global__ void k_fill_f32(float* p, float v) { *p = v; }

// Largest extinction (channel 3) of a colour volume: wave maxima, then one
// atomic per wave on the float's bit pattern (ordered as a signed integer for
// values >= 0 and reversed, as an unsigned one, below 0).
template <int DT>
__global__ __launch_bounds__(256) void k_color_tau_max(const void* cv, int64_t nvox, float* out) {
  float mx = -INFINITY;
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < nvox;
       v += (int64_t)gridDim.x * 256)
    mx = fmaxf(mx, load_rgbt<DT>(cv, v).w);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0 && mx > -INFINITY) {
    if (mx >= 0.0f) atomicMax(reinterpret_cast<int*>(out), __float_as_int(mx));
    else atomicMin(reinterpret_cast<unsigned*>(out), __float_as_uint(mx));
  }
}

}  // namespace

int launch_density_from_color(const DfcParams& p, int dtype, void* stream) {
  const int64_t nvox = (int64_t)p.nx * p.ny * p.nz;
  if (nvox <= 0) return 0;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 g((unsigned)((nvox + 255) / 256)), b(256);
  const size_t lds = (size_t)p.R * sizeof(float4);
  switch (dtype) {
    case DDVR_F16: hipLaunchKernelGGL(k_density_from_color<DDVR_F16>, g, b, lds, s, p); break;
    case DDVR_BF16: hipLaunchKernelGGL(k_density_from_color<DDVR_BF16>, g, b, lds, s, p); break;
    default: hipLaunchKernelGGL(k_density_from_color<DDVR_F32>, g, b, lds, s, p); break;
  }
  return (int)hipGetLastError();
}

int launch_color_tau_max(const void* cv, int dtype, int64_t nvox, float* out, void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(1), 0, s, out, -INFINITY);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  const int64_t want = (nvox + 255) / 256;
  const unsigned blocks = (unsigned)(want < 8192 ? (want > 0 ? want : 1) : 8192);
  switch (dtype) {
    case DDVR_F16: hipLaunchKernelGGL(k_color_tau_max<DDVR_F16>, dim3(blocks), dim3(256), 0, s, cv, nvox, out); break;
    case DDVR_BF16: hipLaunchKernelGGL(k_color_tau_max<DDVR_BF16>, dim3(blocks), dim3(256), 0, s, cv, nvox, out); break;
    default: hipLaunchKernelGGL(k_color_tau_max<DDVR_F32>, dim3(blocks), dim3(256), 0, s, cv, nvox, out); break;
  }
  return (int)hipGetLastError();
}

}  // namespace ddvr

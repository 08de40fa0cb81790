// HIP kernels (gfx950) of the differentiable direct volume renderer.
//
// Forward: Alg. 1 of Weiss & Westermann (arXiv 2107.12672, Sec. 4.1).
// Adjoint: Alg. 2 (Sec. 4.3) with the inversion trick of Sec. 4.4.
//
// Mapping to CDNA4:
//   * one ray per lane; a wave owns an 8x8 pixel block, a workgroup owns a
//     tile of WAVES such blocks (16x16 pixels for 4 waves);
//   * the tile marches slab-synchronously: its rays' samples are grouped into
//     slabs between planes of the grid axis closest to the tile's centre ray
//     (shells of constant distance from the eye where that cannot be used);
//     for every slab the workgroup computes the bounding box of the grid
//     cells its samples touch,
//     stages that brick of the density grid into LDS (converted to float32)
//     and, in the adjoint, accumulates the density gradient of the slab in an
//     LDS brick of fixed-point integers (ds_add_u32; ds_add_u64 for
//     emission-absorption), with a power-of-two scale per tile from a bound
//     on every entry, flushed once per slab with one global float atomic per
//     touched voxel (the paper accumulates per ray "on exit of the current
//     cell", Sec. 4.4 implementation paragraph; the brick is the same idea at
//     workgroup granularity);
//   * the transfer function lives in LDS; its gradient is accumulated per ray
//     in registers while the ray stays on one TF segment and flushed to an
//     LDS table on segment change (Sec. 5.2 "adjoint-delayed"), then to global
//     memory once per workgroup;
//   * absorption-only marches sum the samples of a ray inside one cell in
//     closed form (cell runs), forward and closed-form adjoint alike;
//   * camera and step-size gradients stay in registers per ray and are reduced
//     over the workgroup before one atomic per value;
//   * rays too opaque for the inversion go to a segment-checkpoint kernel that
//     marches one ray per lane in wave-uniform segments, with the density
//     gradient in per-wave LDS bricks and the TF gradient in a per-workgroup
//     LDS table;
//   * blockIdx is remapped so that each XCD (own L2) gets a contiguous range
//     of tiles.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "ddvr_internal.h"
#include "ddvr.h"

namespace ddvr {

// ---------------------------------------------------------------------------
// storage types of the density grid
// ---------------------------------------------------------------------------
// The grid and the gradients live in global memory; loads and atomics go
// through the global address space (not flat), so they count only against
// the vector-memory counter and can stay in flight across LDS traffic.
#define DDVR_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const DDVR_GLOBAL T* gmem(const void* p) {
  return (const DDVR_GLOBAL T*)p;
}
// float atomic add to global memory (gradients), result unused
__device__ __forceinline__ void gadd(float* p, float v) {
  (void)__hip_atomic_fetch_add((DDVR_GLOBAL float*)p, v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

template <int DT> struct Vox;
template <> struct Vox<DDVR_F32> {
  static __device__ __forceinline__ float ld(const void* p, int64_t i) {
    return gmem<float>(p)[i];
  }
};
template <> struct Vox<DDVR_F16> {
  static __device__ __forceinline__ float ld(const void* p, int64_t i) {
    return __half2float(__ushort_as_half(gmem<unsigned short>(p)[i]));
  }
};
template <> struct Vox<DDVR_BF16> {
  static __device__ __forceinline__ float ld(const void* p, int64_t i) {
    const uint32_t u = gmem<unsigned short>(p)[i];
    return __uint_as_float(u << 16);
  }
};

// Storage type chosen per view at run time (batches that mix grids of
// different storage types in one launch); the branch is uniform per tile.
constexpr int DT_DYN = 3;

template <int DT>
__device__ __forceinline__ float vload(const ViewDesc& vd, int64_t i) {
  if constexpr (DT == DT_DYN) {
    if (vd.dtype == DDVR_F16) return Vox<DDVR_F16>::ld(vd.vol, i);
    if (vd.dtype == DDVR_BF16) return Vox<DDVR_BF16>::ld(vd.vol, i);
    return Vox<DDVR_F32>::ld(vd.vol, i);
  } else {
    return Vox<DT>::ld(vd.vol, i);
  }
}

// ---------------------------------------------------------------------------
// f_camera: ray of one pixel, clipped against the grid box.
// Positions are carried in grid units: q = (x - b_min)/h.
// ---------------------------------------------------------------------------
struct RayG {
  float qo[3];   // entry point in grid units
  float dq[3];   // per-sample increment dt*omega/h
  float om[3];   // unit direction
  float t0;      // entry distance
  float wlen;    // |fwd + u*right + v*up|
  float u, v;    // pixel-plane coordinates
  int N;         // samples (0: miss or not a pixel)
  int axis;      // slab plane that defines t0 (-1: t0 = 0)
};

// The ray's setup runs in float64 (a few dozen operations per ray, against
// hundreds of samples): pixel coordinates, direction, box clip, entry point
// and step in grid units are rounded to float32 once, so that a sample's
// position carries ~1 ulp of error plus the march's own fmaf rounding.  In
// float32 the entry point alone (eye ~300 voxels away, t0 from a division)
// and the direction accumulated over the march lost ~1e-4 voxels, which
// moves trilinear weights by as much.  The grid box is exact in float64:
// h = 2/(nmax-1), b_min = -(n-1)/(nmax-1).
__device__ __forceinline__ void setup_ray(const ViewDesc& vd, int px, int py, bool valid,
                                          RayG& r) {
  const double u = 2.0 * ((double)px + 0.5) / (double)vd.W - 1.0;
  const double v = 1.0 - 2.0 * ((double)py + 0.5) / (double)vd.H;
  r.u = (float)u;
  r.v = (float)v;
  double w[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    w[a] = (double)vd.fwd[a] + u * (double)vd.right[a] + v * (double)vd.up[a];
  const double wl = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  r.wlen = (float)wl;
  double om[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    om[a] = w[a] / wl;
    r.om[a] = (float)om[a];
  }
  const int n3[3] = {vd.nx, vd.ny, vd.nz};
  const int nmax = max(vd.nx, max(vd.ny, vd.nz));
  const double inv_h = 0.5 * (double)(nmax - 1);
  double bmin[3];
  double tn = -INFINITY, tf = INFINITY;
  int ax = -1;
  bool ok = valid;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bmin[a] = -(double)(n3[a] - 1) / (double)(nmax - 1);
    const double e = (double)vd.eye[a], o = om[a];
    if (o == 0.0) {
      if (e < bmin[a] || e > -bmin[a]) ok = false;
      continue;
    }
    const double ta = (bmin[a] - e) / o, tb = (-bmin[a] - e) / o;
    const double lo = fmin(ta, tb), hi = fmax(ta, tb);
    if (lo > tn) { tn = lo; ax = a; }
    tf = fmin(tf, hi);
  }
  double t0 = tn;
  if (!(tn > 0.0)) { t0 = 0.0; ax = -1; }
  r.t0 = (float)t0;
  r.axis = ax;
  r.N = 0;
  // a degenerate frame (zero or non-finite direction) yields no samples
  if (!(wl > 0.0) || !(wl < INFINITY)) ok = false;
  if (ok && tf > t0 && (tf - t0) < 1e30) {
    const double n = ceil((tf - t0) / (double)vd.step);
    r.N = (int)fmin(n, (double)kMaxSamples);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.qo[a] = (float)(((double)vd.eye[a] + t0 * om[a] - bmin[a]) * inv_h);
    r.dq[a] = (float)((double)vd.step * om[a] * inv_h);
  }
}

// Trilinear cell of sample i: k = clamp(floor(q), 0, n-2), f = q - k.
// Samples lie inside the grid box, so q leaves [0, n-1) only by rounding; the
// position is clamped to [0, qhi] (qhi the float just below n-1) first, which
// moves it by at most one ulp, after which truncation is the floor and the
// fraction is exact: three instructions per axis (med3, cvt, fract).
// fmaf(i, dq, qo) is monotone in i, so the cells of a run of samples lie
// inside the box spanned by the run's first and last cells.
struct Cell {
  int k[3];
  float f[3];
};

// (sample indices stay below 2^22, so they are exact as floats and the march
// loops count in float)
__device__ __forceinline__ void locate(const RayG& r, float fi, const ViewDesc& vd, Cell& c) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float q = __builtin_amdgcn_fmed3f(fmaf(fi, r.dq[a], r.qo[a]), 0.0f, vd.qhi[a]);
    c.k[a] = (int)q;
    c.f[a] = __builtin_amdgcn_fractf(q);
  }
}

// 8 corner values, index = cx + 2*cy + 4*cz
template <int DT>
__device__ __forceinline__ void fetch_global(const ViewDesc& vd, const Cell& c, float* v) {
  const int64_t sx = 1, sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
  const int64_t b = c.k[2] * sz + c.k[1] * sy + c.k[0];
  v[0] = vload<DT>(vd, b);
  v[1] = vload<DT>(vd, b + sx);
  v[2] = vload<DT>(vd, b + sy);
  v[3] = vload<DT>(vd, b + sy + sx);
  v[4] = vload<DT>(vd, b + sz);
  v[5] = vload<DT>(vd, b + sz + sx);
  v[6] = vload<DT>(vd, b + sz + sy);
  v[7] = vload<DT>(vd, b + sz + sy + sx);
}

struct Brick {   // LDS brick of the current slab
  int x0, y0, z0;
  int bx, bxy;
  int size;
  int bx4, bxy4;  // row and plane strides in bytes
  int off4;       // -4*(x0 + y0*bx + z0*bxy)
  float inv_bx, inv_bxy;
};

// Byte offset in the brick of a cell's corner 0, 4*(k0 + k1*bx + k2*bxy) +
// off4, with 24-bit multiply-adds (operands < 2^24; the 32-bit result wraps
// back into range).
__device__ __forceinline__ int brick_base(const Brick& br, const Cell& c) {
  return (int)(__umul24((unsigned)c.k[2], (unsigned)br.bxy4) +
               __umul24((unsigned)c.k[1], (unsigned)br.bx4) +
               (unsigned)(4 * c.k[0] + br.off4));
}

// The 8 corners of a cell in the brick (index cx + 2*cy + 4*cz), as two
// adjacent floats at each of four byte addresses.
__device__ __forceinline__ void fetch_lds(const float* st, const Brick& br, int base, float* v) {
  const char* p0 = reinterpret_cast<const char*>(st) + base;
  const char* p1 = p0 + br.bx4;
  const char* p2 = p0 + br.bxy4;
  const char* p3 = p2 + br.bx4;
  v[0] = reinterpret_cast<const float*>(p0)[0];
  v[1] = reinterpret_cast<const float*>(p0)[1];
  v[2] = reinterpret_cast<const float*>(p1)[0];
  v[3] = reinterpret_cast<const float*>(p1)[1];
  v[4] = reinterpret_cast<const float*>(p2)[0];
  v[5] = reinterpret_cast<const float*>(p2)[1];
  v[6] = reinterpret_cast<const float*>(p3)[0];
  v[7] = reinterpret_cast<const float*>(p3)[1];
}

// float -> int32 rounding to nearest (halves up) in one instruction
// (floor(x + 0.5)); fixed-point values here stay below 2^29 in magnitude.
__device__ __forceinline__ int round_i32(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// float -> int64 rounding to nearest even for |x| < 2^51: adding 1.5 * 2^52
// in float64 leaves the rounded integer in the low mantissa bits.
__device__ __forceinline__ long long round_i64(float x) {
  const double m = 6755399441055744.0;
  return (long long)(__double_as_longlong((double)x + m) - __double_as_longlong(m));
}

// Add 8 corner values to the LDS gradient brick: float atomics, or (FIX)
// integer atomics of values already in fixed-point units -- 32-bit, or (WIDE)
// 64-bit entries at twice the brick's byte offsets.
template <bool FIX, bool WIDE = false>
__device__ __forceinline__ void lds_add8(float* acc, const Brick& br, int base, const float* g) {
  constexpr int SH = WIDE ? 1 : 0;
  char* p0 = reinterpret_cast<char*>(acc) + (base << SH);
  char* p1 = p0 + (br.bx4 << SH);
  char* p2 = p0 + (br.bxy4 << SH);
  char* p3 = p2 + (br.bx4 << SH);
  char* const pc[4] = {p0, p1, p2, p3};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (FIX && WIDE) {
      atomicAdd(reinterpret_cast<unsigned long long*>(pc[k]),
                (unsigned long long)round_i64(g[2 * k]));
      atomicAdd(reinterpret_cast<unsigned long long*>(pc[k]) + 1,
                (unsigned long long)round_i64(g[2 * k + 1]));
    } else if (FIX) {
      atomicAdd(reinterpret_cast<int*>(pc[k]), round_i32(g[2 * k]));
      atomicAdd(reinterpret_cast<int*>(pc[k]) + 1, round_i32(g[2 * k + 1]));
    } else {
      atomicAdd(reinterpret_cast<float*>(pc[k]), g[2 * k]);
      atomicAdd(reinterpret_cast<float*>(pc[k]) + 1, g[2 * k + 1]);
    }
  }
}

// f_interpolate and its derivative w.r.t. the cell-local coordinates f.
__device__ __forceinline__ float trilerp(const float* v, const float* f) {
  const float c00 = fmaf(f[0], v[1] - v[0], v[0]);
  const float c10 = fmaf(f[0], v[3] - v[2], v[2]);
  const float c01 = fmaf(f[0], v[5] - v[4], v[4]);
  const float c11 = fmaf(f[0], v[7] - v[6], v[6]);
  const float c0 = fmaf(f[1], c10 - c00, c00);
  const float c1 = fmaf(f[1], c11 - c01, c01);
  return fmaf(f[2], c1 - c0, c0);
}

__device__ __forceinline__ void trilerp_grad(const float* v, const float* f, float* g) {
  const float c00 = fmaf(f[0], v[1] - v[0], v[0]);
  const float c10 = fmaf(f[0], v[3] - v[2], v[2]);
  const float c01 = fmaf(f[0], v[5] - v[4], v[4]);
  const float c11 = fmaf(f[0], v[7] - v[6], v[6]);
  const float c0 = fmaf(f[1], c10 - c00, c00);
  const float c1 = fmaf(f[1], c11 - c01, c01);
  g[2] = c1 - c0;
  g[1] = fmaf(f[2], (c11 - c01) - (c10 - c00), c10 - c00);
  const float x00 = v[1] - v[0], x10 = v[3] - v[2], x01 = v[5] - v[4], x11 = v[7] - v[6];
  const float x0 = fmaf(f[1], x10 - x00, x00), x1 = fmaf(f[1], x11 - x01, x01);
  g[0] = fmaf(f[2], x1 - x0, x0);
}

__device__ __forceinline__ void trilerp_weights(const float* f, float* w) {
  const float gx = 1.0f - f[0], gy = 1.0f - f[1], gz = 1.0f - f[2];
  const float a00 = gy * gz, a10 = f[1] * gz, a01 = gy * f[2], a11 = f[1] * f[2];
  w[0] = gx * a00; w[1] = f[0] * a00;
  w[2] = gx * a10; w[3] = f[0] * a10;
  w[4] = gx * a01; w[5] = f[0] * a01;
  w[6] = gx * a11; w[7] = f[0] * a11;
}

// f_TF: knots at k/(R-1), density clamped to [0,1].
struct TFv {
  float r, g, b, tau, phi;
  int j;
  bool inside;
};

__device__ __forceinline__ void tf_eval(const float4* tf, int R, float d, TFv& s) {
  s.inside = (d >= 0.0f) && (d <= 1.0f);
  const float dc = fminf(fmaxf(d, 0.0f), 1.0f);
  const float u = dc * (float)(R - 1);
  const int j = min((int)u, R - 2);
  s.j = j;
  s.phi = u - (float)j;
  const float4 a = tf[j], b = tf[j + 1];
  s.r = fmaf(s.phi, b.x - a.x, a.x);
  s.g = fmaf(s.phi, b.y - a.y, a.y);
  s.b = fmaf(s.phi, b.z - a.z, a.z);
  s.tau = fmaf(s.phi, b.w - a.w, a.w);
}

// Pixel-local loss of the fused pass and its upstream gradient: L2
// (loss_scale (x - y)^2, seed 2 loss_scale (x - y)) or, with DDVR_LOSS_L1, the
// L1 loss of eq. (tf-loss) (loss_scale |x - y|, seed loss_scale sign(x - y),
// 0 where x = y).  `acc` collects the unscaled loss.
__device__ __forceinline__ float loss_seed(bool l1, float scale, float dlt, float& acc) {
  if (l1) {
    acc += fabsf(dlt);
    return dlt > 0.0f ? scale : (dlt < 0.0f ? -scale : 0.0f);
  }
  acc = fmaf(dlt, dlt, acc);
  return 2.0f * scale * dlt;
}

// ---------------------------------------------------------------------------
// workgroup helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int b, int G) {
  const int q = G >> 3, r = G & 7, x = b & 7, k = b >> 3;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Maximum over the 64 lanes of a wave with DPP row shifts and row
// broadcasts (full-rate VALU, no LDS round trips): after the row_shr steps
// lane 15 of each row holds the row maximum, row_bcast15/31 carry it into
// lane 63, which is read back as a uniform value.  Lanes a DPP step does not
// write keep INT_MIN, the identity.
__device__ __forceinline__ int wave_max_i32(int x) {
  constexpr int ID = -2147483647 - 1;
  x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x111, 0xf, 0xf, false));   // row_shr:1
  x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x112, 0xf, 0xf, false));   // row_shr:2
  x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x114, 0xf, 0xe, false));   // row_shr:4
  x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x118, 0xf, 0xc, false));   // row_shr:8
  x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x142, 0xa, 0xf, false));   // row_bcast:15
  x = max(x, __builtin_amdgcn_update_dpp(ID, x, 0x143, 0xc, 0xf, false));   // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}

template <int NT>
__device__ __forceinline__ void wg_max_n(int* v, int n, int* scratch) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // (n is a compile-time constant at every call: unrolled, v stays in registers)
#pragma unroll
  for (int k = 0; k < n; ++k) v[k] = wave_max_i32(v[k]);
  if (NW == 1) return;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < n; ++k) scratch[wid * 8 + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < n; ++k) {
    int x = scratch[k];
#pragma unroll
    for (int w = 1; w < NW; ++w) x = max(x, scratch[w * 8 + k]);
    v[k] = x;
  }
}

// A value every lane of the wave holds alike (a workgroup reduction's
// result), moved to a scalar register so that it takes no vector register
// while it stays live across the march loops.
__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float wave_uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

template <int NT>
__device__ __forceinline__ float wg_min_f(float x, float* scratch) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fminf(x, __shfl_xor(x, off, 64));
  if (NW == 1) return x;
  __syncthreads();
  if (lane == 0) scratch[wid] = x;
  __syncthreads();
  float r = scratch[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = fminf(r, scratch[w]);
  return r;
}

// sum of n floats over the workgroup; result valid in thread 0
template <int NT>
__device__ __forceinline__ void wg_sum_n(float* v, int n, float* scratch) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < n; ++k) {
    float x = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[k] = x;
  }
  if (NW == 1) return;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < n; ++k) scratch[wid * 16 + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < n; ++k) {
      float x = scratch[k];
      for (int w = 1; w < NW; ++w) x += scratch[w * 16 + k];
      v[k] = x;
    }
}

// Samples of a ray inside the slab [lo, hi) of tile sample offsets: the
// tile's samples are grouped by their index offset from the earliest entry
// point of the tile, so a slab is a shell of roughly constant distance from
// the eye.
__device__ __forceinline__ void slab_range(int lo, int hi, int off, int N, int& a, int& b) {
  a = min(max(lo - off, 0), N);
  b = min(max(hi - off, 0), N);
}

// Sum over the workgroup, returned to every thread.
template <int NT>
__device__ __forceinline__ float wg_sum_all(float x, float* scratch) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  if (NW == 1) return x;
  __syncthreads();
  if (lane == 0) scratch[wid] = x;
  __syncthreads();
  float r = scratch[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r += scratch[w];
  return r;
}

// Bounding box of the cells of every sample in the slab [lo, hi).
// Returns false if no ray has a sample in it.
// Bounding box of the cells of every lane's samples [a, b).
template <int NT>
__device__ __forceinline__ bool range_brick(const ViewDesc& vd, const RayG& r, int a, int b,
                                            int* iscratch, Brick& br) {
  int v[6];
  if (a < b) {
    Cell c0, c1;
    locate(r, (float)a, vd, c0);
    locate(r, (float)(b - 1), vd, c1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[k] = -min(c0.k[k], c1.k[k]);
      v[3 + k] = max(c0.k[k], c1.k[k]) + 1;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = -0x3fffffff;
  }
  wg_max_n<NT>(v, 6, iscratch);
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_uniform(v[k]);
  if (v[3] < 0) return false;
  br.x0 = -v[0]; br.y0 = -v[1]; br.z0 = -v[2];
  const int bx = v[3] - br.x0 + 1, by = v[4] - br.y0 + 1, bz = v[5] - br.z0 + 1;
  br.bx = bx;
  br.bxy = bx * by;
  br.size = br.bxy * bz;
  br.bx4 = 4 * bx;
  br.bxy4 = 4 * br.bxy;
  br.off4 = -4 * (br.x0 + br.y0 * bx + br.z0 * br.bxy);
  br.inv_bx = wave_uniform(1.0f / (float)bx);
  br.inv_bxy = wave_uniform(1.0f / (float)br.bxy);
  return true;
}

template <int NT>
__device__ __forceinline__ bool slab_brick(const ViewDesc& vd, const RayG& r, int off, int N,
                                           int lo, int hi, int* iscratch, Brick& br) {
  int a, b;
  slab_range(lo, hi, off, N, a, b);
  return range_brick<NT>(vd, r, a, b, iscratch, br);
}

// Choose the next slab of the march: starting at `pos` and running forward
// (dir = +1: [pos, pos+K)) or backward (dir = -1: [pos-K, pos)), with K
// halved until the brick fits `cap` voxels and doubled again after a slab
// that used less than a quarter of it.  Returns 0 = empty slab, 1 = fits
// (stage in LDS), 2 = does not fit even at the minimum length (direct global
// access); [lo, hi) is the chosen slab.
template <int NT>
__device__ __forceinline__ int pick_slab(const ViewDesc& vd, const RayG& r, int off, int N,
                                         int pos, int dir, int end, int cap, int& K, int kmax,
                                         int& lo, int& hi, int* iscratch, Brick& br) {
  constexpr int kmin = 4;
  for (;;) {
    if (dir > 0) { lo = pos; hi = min(pos + K, end); }
    else { hi = pos; lo = max(pos - K, end); }
    if (!slab_brick<NT>(vd, r, off, N, lo, hi, iscratch, br)) {
      K = min(2 * K, kmax);
      return 0;
    }
    if (cap > 0 && br.size <= cap) {
      if (4 * br.size < cap) K = min(2 * K, kmax);
      return 1;
    }
    if (cap <= 0 || K <= kmin) return 2;
    K = max(K >> 1, kmin);
  }
}

// Axis slabs of a tile.  Slabs lie between planes q_ax = const of the grid
// axis ax closest to the tile's centre ray, in march order (t = sgn * q_ax
// grows along every ray): an axis-aligned slab has a tight bounding box at
// any view angle, where a shell of constant distance from the eye cut
// obliquely through the grid spans a box many times its volume (the
// 4-channel brick holds a quarter of the scalar brick's vertices).  Each
// ray's samples between two planes form one index range; consecutive slabs
// share their boundary plane, so the ranges partition the ray.
__device__ __forceinline__ void tile_axis(const ViewDesc& vd, int tx, int ty, int tw, int th,
                                          const RayG& r, float& t0, float& dta) {
  const float uc = 2.0f * ((float)(tx * tw) + 0.5f * tw) / (float)vd.W - 1.0f;
  const float vc = 1.0f - 2.0f * ((float)(ty * th) + 0.5f * th) / (float)vd.H;
  float wc[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) wc[k] = vd.fwd[k] + uc * vd.right[k] + vc * vd.up[k];
  const int ax = fabsf(wc[0]) >= fabsf(wc[1]) ? (fabsf(wc[0]) >= fabsf(wc[2]) ? 0 : 2)
                                               : (fabsf(wc[1]) >= fabsf(wc[2]) ? 1 : 2);
  // The axis picks by 0/1 weights, not by a run-time array index or a select
  // of the ray's fields (the compiler turns either into an indexed load and
  // keeps the ray in scratch memory).  Exact for the finite values of rays
  // with samples, the only ones the slab walk reads.
  const float e0 = ax == 0 ? 1.0f : 0.0f, e1 = ax == 1 ? 1.0f : 0.0f, e2 = ax == 2 ? 1.0f : 0.0f;
  const float w = e0 * wc[0] + e1 * wc[1] + e2 * wc[2];
  const float sgn = w >= 0.0f ? 1.0f : -1.0f;
  t0 = sgn * (e0 * r.qo[0] + e1 * r.qo[1] + e2 * r.qo[2]);
  dta = sgn * (e0 * r.dq[0] + e1 * r.dq[1] + e2 * r.dq[2]);
}

// first sample index at or past plane t (clamped to [0, n])
__device__ __forceinline__ int axis_index(float t, float t0, float dta, int n) {
  return (int)fminf(fmaxf(ceilf((t - t0) / dta), 0.0f), (float)n);
}

// The tile's plane range [tlo, thi] covering every ray's samples [0, n);
// returns false if some ray with samples does not advance along the axis.
template <int NT>
__device__ __forceinline__ bool axis_range(float t0, float dta, int n, int* iscratch, int& tlo,
                                           int& thi) {
  const bool bad = n > 0 && !(dta > 0.0f);
  int v[3] = {n > 0 ? -(int)floorf(t0) : -0x3fffffff,
              n > 0 ? (int)ceilf(fmaf((float)(n - 1), dta, t0)) + 1 : -0x3fffffff, bad ? 1 : 0};
  wg_max_n<NT>(v, 3, iscratch);
  tlo = -v[0];
  thi = v[1];
  return v[2] == 0;
}

// A tile's walk through its slabs, shared by the forward (front to back) and
// the adjoint (back to front).  Axis slabs (tile_axis) bound a ray's samples
// by planes of one grid axis: their bricks stay tight at any view angle, and
// a brick row along x holds a long run of touched voxels (one global atomic
// request per 64 bytes of it when the gradient brick is flushed).  Distance
// shells group samples by their index offset `off` from the tile's earliest
// entry point; they serve launches without bricks and tiles where some ray
// does not advance along the axis.  Widths are in planes (axis) or samples
// (shells) and adapt per slab as in pick_slab.
struct SlabWalk {
  bool axis;
  // this ray's coordinate of sample 0 and its advance per sample: the plane
  // coordinate of its axis (axis slabs) or its sample offset and 1 (shells);
  // its samples between slab bounds [l, h) are [axis_index(l), axis_index(h))
  float t0, dta;
  float lo, hi;         // the tile's range: planes (axis) or offsets [0, end) (shells)
  float w, wmin, wmax;  // current slab width and its limits
};

// Set up the walk over samples [0, N) of every ray of the tile (N = 0: none).
// `tmin` is the tile's earliest entry distance (shells: a ray's offset is its
// entry distance past it in steps).
template <int NT>
__device__ __forceinline__ void walk_init(const ViewDesc& vd, const RayG& r, int N, int tx,
                                          int ty, int tw, int th, int cap, int kmax,
                                          bool want_axis, float tmin, int* iscratch,
                                          SlabWalk& w) {
  const int off = (cap > 0 && r.N > 0) ? (int)rintf((r.t0 - tmin) / vd.step) : 0;
  float t0, dta;
  tile_axis(vd, tx, ty, tw, th, r, t0, dta);
  want_axis = want_axis && cap > 0;
  const bool has = N > 0;
  int v[4] = {has ? off + N : 0,
              (want_axis && has) ? -(int)floorf(t0) : -0x3fffffff,
              (want_axis && has) ? (int)ceilf(fmaf((float)(N - 1), dta, t0)) + 1 : -0x3fffffff,
              (want_axis && has && !(dta > 0.0f)) ? 1 : 0};
  wg_max_n<NT>(v, 4, iscratch);
#pragma unroll
  for (int k = 0; k < 4; ++k) v[k] = wave_uniform(v[k]);
  w.axis = want_axis && v[3] == 0 && v[1] > -0x3fffffff;
  w.t0 = w.axis ? t0 : (float)off;
  w.dta = w.axis ? dta : 1.0f;
  const float K = (float)min(vd.slab_k, kmax);
  if (w.axis) {
    // a slab of K samples spans at most K step/h planes of its axis
    const float pps = vd.step * vd.inv_h;
    w.lo = (float)(-v[1]);
    w.hi = (float)v[2];
    w.w = wave_uniform(K * pps);
    w.wmin = wave_uniform(fmaxf(4.0f * pps, 0.25f));
    w.wmax = wave_uniform(fmaxf((float)kmax * pps, w.w));
  } else {
    w.lo = 0.0f;
    w.hi = (float)v[0];
    w.w = K;
    w.wmin = 4.0f;
    w.wmax = (float)kmax;
  }
}

// This ray's samples [a, b) between the slab bounds [l, h) (N samples; for
// shells the bounds and offsets are integers, so this is their index range).
__device__ __forceinline__ void walk_range(const SlabWalk& w, float l, float h, int N, int& a,
                                           int& b) {
  a = axis_index(l, w.t0, w.dta, N);
  b = axis_index(h, w.t0, w.dta, N);
  if (N <= 0) a = b = 0;
}

// The next slab from `pos` (dir +1: [pos, pos + w), -1: [pos - w, pos)),
// narrowed until its brick fits `cap` voxels and widened again after a slab
// that used less than a quarter of it.  Returns 0 = empty, 1 = fits (stage in
// LDS), 2 = does not fit at the minimum width (direct global access); [l, h)
// is the slab and [a, b) this ray's samples in it.
template <int NT>
__device__ __forceinline__ int walk_next(const ViewDesc& vd, const RayG& r, int N, SlabWalk& w,
                                         float pos, int dir, int cap, float& l, float& h,
                                         int& a, int& b, int* iscratch, Brick& br) {
  for (;;) {
    if (dir > 0) { l = pos; h = wave_uniform(fminf(pos + w.w, w.hi)); }
    else { h = pos; l = wave_uniform(fmaxf(pos - w.w, w.lo)); }
    walk_range(w, l, h, N, a, b);
    if (!range_brick<NT>(vd, r, a, b, iscratch, br)) {
      w.w = wave_uniform(fminf(2.0f * w.w, w.wmax));
      return 0;
    }
    if (cap > 0 && br.size <= cap) {
      if (4 * br.size < cap) w.w = wave_uniform(fminf(2.0f * w.w, w.wmax));
      return 1;
    }
    if (cap <= 0 || w.w <= w.wmin) return 2;
    w.w = wave_uniform(fmaxf(w.axis ? 0.5f * w.w : floorf(0.5f * w.w), w.wmin));
  }
}

// Offset in the grid of brick element idx (x fastest, then y, then z)
// relative to the brick's corner voxel.  Row and plane indices come from
// float reciprocals (exact: idx + 0.5 stays at least 0.5/bxy from a multiple
// of bxy and bricks hold < 2^21 elements); the offset uses 24-bit
// multiply-adds when the brick's span in the grid fits 31 bits (`narrow`).
template <bool NARROW>
__device__ __forceinline__ int64_t brick_goff(const Brick& br, int idx, int64_t sy, int64_t sz) {
  const int z = (int)fmaf((float)idx, br.inv_bxy, 0.5f * br.inv_bxy);
  const int rem = idx - __mul24(z, br.bxy);
  const int y = (int)fmaf((float)rem, br.inv_bx, 0.5f * br.inv_bx);
  const int x = rem - __mul24(y, br.bx);
  if (NARROW)
    return (int64_t)(uint32_t)(x + __umul24((unsigned)y, (unsigned)sy) +
                               __umul24((unsigned)z, (unsigned)sz));
  return x + y * sy + z * sz;
}

__device__ __forceinline__ bool brick_narrow(const Brick& br, int64_t sz) {
  return sz < (1 << 24) && (int64_t)(br.size / br.bxy) * sz < (int64_t(1) << 31);
}

// Copy the brick's grid values into LDS as float32: U loads in flight per
// lane (lanes past the end re-read the last element, so the loads need no
// branch) before the LDS writes.
template <int NT, int DT, bool NARROW>
__device__ __forceinline__ void stage_loads(const ViewDesc& vd, const Brick& br, float* stage,
                                            int64_t org, int64_t sy, int64_t sz) {
  constexpr int U = 8;
  for (int i0 = threadIdx.x; i0 < br.size; i0 += U * NT) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = vload<DT>(vd, org + brick_goff<NARROW>(br, min(i0 + u * NT, br.size - 1), sy, sz));
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * NT < br.size) stage[i0 + u * NT] = v[u];
  }
}

// Stage the brick's grid values (as float32) and/or zero its gradient
// accumulator.  The caller synchronises before the brick is read.
template <int NT, int DT, bool WIDE = false>
__device__ __forceinline__ void stage_brick(const ViewDesc& vd, const Brick& br, float* stage,
                                            float* acc) {
  const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
  const int64_t org = br.z0 * sz + br.y0 * sy + br.x0;
  if (stage) {
    if (brick_narrow(br, sz)) stage_loads<NT, DT, true>(vd, br, stage, org, sy, sz);
    else stage_loads<NT, DT, false>(vd, br, stage, org, sy, sz);
  }
  if (acc) {
    if (WIDE)
      for (int idx = threadIdx.x; idx < br.size; idx += NT)
        reinterpret_cast<long long*>(acc)[idx] = 0;
    else
      for (int idx = threadIdx.x; idx < br.size; idx += NT) acc[idx] = 0.0f;
  }
}

// Add the brick's gradient accumulator to the density gradient in global
// memory, one atomic per touched voxel.  FIX: the accumulator holds
// fixed-point values (see AdjState::qs; 64-bit ones when WIDE), scaled back
// by inv_qs.
template <int NT, bool FIX, bool WIDE = false>
__device__ __forceinline__ void flush_brick(const ViewDesc& vd, const Brick& br, const float* acc,
                                            float inv_qs) {
  const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
  float* const org = vd.dV + (br.z0 * sz + br.y0 * sy + br.x0);
  const bool narrow = brick_narrow(br, sz);
  for (int idx = threadIdx.x; idx < br.size; idx += NT) {
    float g;
    if (FIX && WIDE)
      g = (float)((double)reinterpret_cast<const long long*>(acc)[idx] * (double)inv_qs);
    else if (FIX)
      g = (float)reinterpret_cast<const int*>(acc)[idx] * inv_qs;
    else
      g = acc[idx];
    if (g != 0.0f)
      gadd(org + (narrow ? brick_goff<true>(br, idx, sy, sz)
                         : brick_goff<false>(br, idx, sy, sz)), g);
  }
}

// ---------------------------------------------------------------------------
// per-sample forward (Alg. 1 body)
// ---------------------------------------------------------------------------
struct FwdState {
  float C[3];
  float T;      // emission-absorption: running transmittance
  float sigma;  // absorption-only: running optical depth / dt
};

template <int MODEL, int DT, bool LDS>
__device__ __forceinline__ void march_fwd(const ViewDesc& vd, const RayG& r, int a, int b,
                                          const float* stage, const Brick& br,
                                          const float4* tfl, FwdState& s) {
  const float fb = (float)b;
  for (float fi = (float)a; fi < fb; fi += 1.0f) {
    Cell c;
    locate(r, fi, vd, c);
    float v[8];
    if (LDS) fetch_lds(stage, br, brick_base(br, c), v);
    else fetch_global<DT>(vd, c, v);
    const float d = trilerp(v, c.f);
    if (MODEL == DDVR_ABSORPTION) {
      s.sigma += d;
    } else {
      TFv t;
      tf_eval(tfl, vd.R, d, t);
      const float e = __expf(-vd.step * t.tau);
      // explicitly rounded (no contraction), shared bit for bit with march_tan
      const float w = __fmul_rn(s.T, __fsub_rn(1.0f, e));
      s.C[0] = fmaf(w, t.r, s.C[0]);
      s.C[1] = fmaf(w, t.g, s.C[1]);
      s.C[2] = fmaf(w, t.b, s.C[2]);
      s.T *= e;
    }
  }
}

// ---------------------------------------------------------------------------
// Absorption-only runs.  The samples of a ray inside one grid cell, x_i =
// x_o + i dt omega for i in [i0, i1), see one trilinear polynomial: along
// them the density, and every corner's trilinear weight, is a cubic in i
// whose odd central moments about the run's midpoint mu = (i0 + i1 - 1)/2
// vanish.  So the run's sum of densities, the sum Alg. 1 accumulates for
// tau = d, is m (d(mu) + (s2/2) d''), with m = i1 - i0, s2 = (m^2 - 1)/12 the
// mean squared distance of the indices from mu and d'' the second derivative
// along the ray per sample; the same holds for the sum of each corner's
// weight that the adjoint scatters (its d_hat is the same for every sample of
// a ray).  The numbers are the per-sample sums of Alg. 1 / Alg. 2, computed
// once per cell instead of once per sample.
// ---------------------------------------------------------------------------
struct RunGeo {
  float inv_dq[3];       // 1/dq per axis (1e30 where dq = 0: no boundary)
  float upq[3];          // up - q_o: up = 1 if the ray moves up the axis (or not at
                         // all), else 0
  float dxy, dxz, dyz;   // products of the per-sample steps of two axes
};

__device__ __forceinline__ void run_geo(const ViewDesc& vd, const RayG& r, RunGeo& g) {
  (void)vd;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    g.inv_dq[a] = r.dq[a] != 0.0f ? 1.0f / r.dq[a] : 1e30f;
    g.upq[a] = (r.dq[a] >= 0.0f ? 1.0f : 0.0f) - r.qo[a];
  }
  g.dxy = r.dq[0] * r.dq[1];
  g.dxz = r.dq[0] * r.dq[2];
  g.dyz = r.dq[1] * r.dq[2];
}

// Cell of sample fi (k as float and as int): the clamp of locate, without the
// fraction.
__device__ __forceinline__ void locate_cell(const RayG& r, float fi, const ViewDesc& vd,
                                            Cell& c, float* kf) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float q = __builtin_amdgcn_fmed3f(fmaf(fi, r.dq[a], r.qo[a]), 0.0f, vd.qhi[a]);
    kf[a] = floorf(q);
    c.k[a] = (int)kf[a];
  }
}

// One past the last sample of [fi, fb) in the cell kf of sample fi, at least
// fi + 1: the first index at or past the next cell face along each axis,
// ceil((k + (up - q_o))/dq).  Float rounding can move a boundary by one sample
// (that sample is then evaluated with the neighbouring cell's polynomial a
// hair outside [0, 1], where the trilinear interpolant is continuous, or
// starts a run of its own); the box faces end the ray anyway.
__device__ __forceinline__ float run_end(const RayG& r, const RunGeo& g, const float* kf,
                                         float fi, float fb) {
  float e = fb;
#pragma unroll
  for (int a = 0; a < 3; ++a) e = fminf(e, ceilf((kf[a] + g.upq[a]) * g.inv_dq[a]));
  return fmaxf(e, fi + 1.0f);
}

// Cell-local coordinates of the run's midpoint (not clamped: within rounding
// of [0, 1]).  The fma rounds mu dq + (q_o - k) once at the scale of the
// result (<= 1) instead of at the scale of the position (up to n); q_o - k is
// exact when k <= q_o (Sterbenz) and otherwise rounds at the scale of k.
__device__ __forceinline__ void run_mid(const RayG& r, const float* kf, float mu, float* f) {
#pragma unroll
  for (int a = 0; a < 3; ++a) f[a] = fmaf(mu, r.dq[a], r.qo[a] - kf[a]);
}

// Sum of the densities of an absorption-only run: m (d(mu) + s2/2 d''), with
// d'' = 2 (dxy d_xy + dxz d_xz + dyz d_yz), d_ab the mixed derivatives of the
// trilinear interpolant at the midpoint.
__device__ __forceinline__ float run_density_sum(const float* v, const float* f, float m,
                                                 const RunGeo& g) {
  const float x0 = v[1] - v[0], x1 = v[3] - v[2], x2 = v[5] - v[4], x3 = v[7] - v[6];
  const float c00 = fmaf(f[0], x0, v[0]);
  const float c10 = fmaf(f[0], x1, v[2]);
  const float c01 = fmaf(f[0], x2, v[4]);
  const float c11 = fmaf(f[0], x3, v[6]);
  const float c0 = fmaf(f[1], c10 - c00, c00);
  const float c1 = fmaf(f[1], c11 - c01, c01);
  const float d = fmaf(f[2], c1 - c0, c0);
  const float dxy0 = x1 - x0, dxy1 = x3 - x2;
  const float d_xy = fmaf(f[2], dxy1 - dxy0, dxy0);
  const float dxz0 = x2 - x0, dxz1 = x3 - x1;
  const float d_xz = fmaf(f[1], dxz1 - dxz0, dxz0);
  const float d_yz = (c11 - c01) - (c10 - c00);
  const float curv = fmaf(g.dxy, d_xy, fmaf(g.dxz, d_xz, g.dyz * d_yz));
  const float s2 = (m * m - 1.0f) * (1.0f / 12.0f);
  return m * fmaf(s2, curv, d);
}

// Sums over an absorption-only run of the 8 corner weights, w (index cx + 2cy
// + 4cz) = m (w_c(mu) + s2 (sx sy dxy z_c + sx sz dxz y_c + sy sz dyz x_c)),
// with x_c, y_c, z_c the corner's linear factors at mu and s = +1 for the
// lower corner of an axis, -1 for the upper (the sign of the factor's slope;
// only products of two signs appear); times `scale`.
__device__ __forceinline__ void run_weight_sums(const float* f, float m, const RunGeo& g,
                                                float scale, float* w) {
  // Corner (cx, cy, cz) sums to
  //   X (Y Z + s_y s_z e_yz) + s_x (s_y e_xy Z + s_z e_xz Y),
  // factored over (cy, cz); the run length and the scale ride on X, e_xy and
  // e_xz.
  const float s2 = (m * m - 1.0f) * (1.0f / 12.0f);
  const float sc = m * scale;
  const float exy = (s2 * sc) * g.dxy, exz = (s2 * sc) * g.dxz, eyz = s2 * g.dyz;
  const float X[2] = {(1.0f - f[0]) * sc, f[0] * sc};
  const float Y[2] = {1.0f - f[1], f[1]}, Z[2] = {1.0f - f[2], f[2]};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cy = q & 1, cz = q >> 1;
    const float sy = cy ? -1.0f : 1.0f, sz = cz ? -1.0f : 1.0f;
    const float P = fmaf(Y[cy], Z[cz], (sy * sz) * eyz);
    const float Q = fmaf(sy * exy, Z[cz], (sz * exz) * Y[cy]);
    w[2 * q] = fmaf(X[0], P, Q);
    w[2 * q + 1] = fmaf(X[1], P, -Q);
  }
}

// Forward of samples [a, b) of an absorption-only ray, one cell run at a time
// (LDS: corners from the staged brick; else gathered from the grid).
template <int DT, bool LDS>
__device__ __forceinline__ void march_fwd_ao_runs(const ViewDesc& vd, const RayG& r,
                                                  const RunGeo& g, int a, int b,
                                                  const float* stage, const Brick& br,
                                                  FwdState& s) {
  const float fb = (float)b;
  for (float fi = (float)a; fi < fb;) {
    Cell c;
    float kf[3];
    locate_cell(r, fi, vd, c, kf);
    const float fe = run_end(r, g, kf, fi, fb);
    const float m = fe - fi;
    float f[3];
    run_mid(r, kf, fmaf(0.5f, m - 1.0f, fi), f);
    float v[8];
    if (LDS) fetch_lds(stage, br, brick_base(br, c), v);
    else fetch_global<DT>(vd, c, v);
    s.sigma += run_density_sum(v, f, m, g);
    fi = fe;
  }
}

// ---------------------------------------------------------------------------
// per-ray adjoint state and per-sample adjoint (Alg. 2 body)
// ---------------------------------------------------------------------------
struct AdjState {
  float Chat[3];   // adjoint of the accumulated colour (constant along the ray)
  float ahat;      // adjoint of the accumulated opacity alpha^(i+1)
  float Tn;        // T^(i+1) (inversion state)
  float an;        // alpha^(i+1) (alpha-form inversion state)
  float P;         // absorption-only closed form: T^(i+1)*ahat^(i+1), constant
  float dh;        // absorption-only closed form: d_hat = dt*P of every sample
  float dhq;       // dh * qs (fixed-point units)
  // Ray sums behind the camera and step gradients, kept in float64: they add
  // up to thousands of terms of both signs (weighted by i), and float32 would
  // lose ~1e-3 of the result to cancellation on long rays.
  double xo_hat[3]; // sum of position adjoints
  double si[3];     // sum of i * position adjoints
  double dstep;     // Beer-Lambert part of the step adjoint
  // TF gradient of the current segment (registers, flushed on change)
  int tj;
  float tg0[4], tg1[4];
  // density gradient of the current cell (registers, flushed on cell exit)
  int ckey;        // LDS byte offset of the cell's corner 0 (staged slabs); -1: none
  int64_t gkey;    // global index of the cell's corner 0 (direct slabs); -1: none
  float cg[8];
  // Scale of the 32-bit fixed-point LDS accumulation used by the absorption-only
  // closed form (a power of two, uniform over the tile).  LDS integer atomics
  // run at the rate of plain stores, float ones serialise per lane.
  float qs;
};

// Add the registered density gradient of the current cell to the LDS brick
// (LDS) or to global memory (direct slabs), then clear it.
template <bool LDS, bool FIX, bool WIDE = false>
__device__ __forceinline__ void cell_flush(const ViewDesc& vd, const Brick& br, float* acc,
                                           AdjState& s) {
  if (LDS) {
    if (s.ckey < 0) return;
    lds_add8<FIX, WIDE>(acc, br, s.ckey, s.cg);
  } else {
    if (s.gkey < 0) return;
    const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
    float* g = vd.dV + s.gkey;
    gadd(g, s.cg[0]);
    gadd(g + 1, s.cg[1]);
    gadd(g + sy, s.cg[2]);
    gadd(g + sy + 1, s.cg[3]);
    gadd(g + sz, s.cg[4]);
    gadd(g + sz + 1, s.cg[5]);
    gadd(g + sz + sy, s.cg[6]);
    gadd(g + sz + sy + 1, s.cg[7]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) s.cg[k] = 0.0f;
  if (LDS) s.ckey = -1;
  else s.gkey = -1;
}

__device__ __forceinline__ void tf_flush(AdjState& s, float* dtf) {
  if (s.tj >= 0) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      if (s.tg0[ch] != 0.0f) atomicAdd(dtf + 4 * s.tj + ch, s.tg0[ch]);
      if (s.tg1[ch] != 0.0f) atomicAdd(dtf + 4 * (s.tj + 1) + ch, s.tg1[ch]);
      s.tg0[ch] = 0.0f; s.tg1[ch] = 0.0f;
    }
  }
}

// Adjoint of one sample i given T^(i) source.  `mode` selects how T^(i) is
// recovered: 0 closed form (AO), 1 T-form inversion, 2 alpha-form inversion,
// 3 caller supplies Ti (checkpoint), 4 the same with the density gradient in
// a float32 LDS brick.
template <int MODEL, int DT, bool LDS, int MODE, bool XH>
__device__ __forceinline__ void adj_sample(const ViewDesc& vd, const RayG& r, float fi,
                                           const float* stage, float* acc, const Brick& br,
                                           const float4* tfl, float* dtf, int gmask,
                                           bool need_v, bool cell_acc, AdjState& s,
                                           float Ti_given) {
  // the closed form and the inversions accumulate the LDS brick in fixed
  // point, 64-bit for emission-absorption (its scale bound is looser); the
  // checkpoint fallback's wave bricks (MODE 4) in float32, with the grid
  // gathered from global memory
  constexpr bool FIX = LDS && MODE <= 2;
  constexpr bool WIDE = MODEL == DDVR_EMISSION_ABSORPTION && MODE <= 2;
  Cell c;
  locate(r, fi, vd, c);
  // XH: camera or step gradients are compiled in (their float64 ray sums cost
  // registers the density-only kernels do not pay for)
  const bool need_xhat = XH && (gmask & (GRAD_CAM | GRAD_STEP)) != 0;
  float v[8];
  float d = 0.0f;
  int base = 0;
  if (LDS) base = brick_base(br, c);
  if (need_v) {
    if (LDS && MODE != 4) fetch_lds(stage, br, base, v);
    else fetch_global<DT>(vd, c, v);
    d = trilerp(v, c.f);
  }
  float d_hat;
  if (MODEL == DDVR_ABSORPTION && MODE == 0) {
    // T^(i)*e_i*ahat^(i+1) = T^(i+1)*ahat^(i+1) is invariant under the
    // inversion T^(i) = T^(i+1)/e_i, ahat^(i) = e_i*ahat^(i+1) (no emission).
    d_hat = s.dh;
    if (XH) s.dstep += (double)(d * s.P);
  } else {
    float rgb[3] = {0.0f, 0.0f, 0.0f}, tau;
    TFv t;
    if (MODEL == DDVR_EMISSION_ABSORPTION) {
      tf_eval(tfl, vd.R, d, t);
      rgb[0] = t.r; rgb[1] = t.g; rgb[2] = t.b;
      tau = t.tau;
    } else {
      tau = d;
    }
    const float e = __expf(-vd.step * tau);
    const float alpha = 1.0f - e;
    float Ti;
    if (MODE == 1) {
      Ti = s.Tn * __builtin_amdgcn_rcpf(e);
    } else if (MODE == 2) {
      const float ap = (alpha - s.an) / (alpha - 1.0f);   // eq. (inv-blend-forward)
      s.an = ap;
      Ti = 1.0f - ap;
    } else {
      Ti = Ti_given;
    }
    s.Tn = Ti;
    const float rc = rgb[0] * s.Chat[0] + rgb[1] * s.Chat[1] + rgb[2] * s.Chat[2];
    const float as_hat = Ti * (s.ahat + rc);            // adjoint of alpha_i
    s.ahat = fmaf(e, s.ahat, -alpha * rc);              // ahat^(i)
    const float ase = as_hat * e;
    const float tau_hat = ase * vd.step;
    if (XH) s.dstep += (double)(ase * tau);
    if (MODEL == DDVR_EMISSION_ABSORPTION) {
      const float w = alpha * Ti;
      const float g4[4] = {w * s.Chat[0], w * s.Chat[1], w * s.Chat[2], tau_hat};
      if (gmask & GRAD_TF) {
        if (t.j != s.tj) {
          tf_flush(s, dtf);
          s.tj = t.j;
        }
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
          s.tg0[ch] = fmaf(1.0f - t.phi, g4[ch], s.tg0[ch]);
          s.tg1[ch] = fmaf(t.phi, g4[ch], s.tg1[ch]);
        }
      }
      const float4 ta = tfl[t.j], tb = tfl[t.j + 1];
      const float u_hat = (tb.x - ta.x) * g4[0] + (tb.y - ta.y) * g4[1] +
                          (tb.z - ta.z) * g4[2] + (tb.w - ta.w) * g4[3];
      d_hat = t.inside ? (float)(vd.R - 1) * u_hat : 0.0f;
    } else {
      d_hat = tau_hat;
    }
  }
  if ((gmask & GRAD_V) && cell_acc) {
    // accumulate while the ray stays in this cell (Sec. 4.4: per-ray registers
    // flushed on exit of the current cell); the fixed-point route accumulates
    // in fixed-point units.  Weights w_c * d_hat with d_hat folded into the x
    // factors.
    const float dv = FIX ? (MODE == 0 ? s.dhq : d_hat * s.qs) : d_hat;
    const float gx = 1.0f - c.f[0], gy = 1.0f - c.f[1], gz = 1.0f - c.f[2];
    const float d0 = gx * dv, d1 = c.f[0] * dv;
    const float a00 = gy * gz, a10 = c.f[1] * gz, a01 = gy * c.f[2], a11 = c.f[1] * c.f[2];
    if (LDS) {
      if (base != s.ckey) {
        cell_flush<LDS, FIX, WIDE>(vd, br, acc, s);
        s.ckey = base;
      }
    } else {
      const int64_t key =
          (int64_t)c.k[2] * vd.nx * vd.ny + (int64_t)c.k[1] * vd.nx + c.k[0];
      if (key != s.gkey) {
        cell_flush<LDS, FIX, WIDE>(vd, br, acc, s);
        s.gkey = key;
      }
    }
    s.cg[0] = fmaf(d0, a00, s.cg[0]);
    s.cg[1] = fmaf(d1, a00, s.cg[1]);
    s.cg[2] = fmaf(d0, a10, s.cg[2]);
    s.cg[3] = fmaf(d1, a10, s.cg[3]);
    s.cg[4] = fmaf(d0, a01, s.cg[4]);
    s.cg[5] = fmaf(d1, a01, s.cg[5]);
    s.cg[6] = fmaf(d0, a11, s.cg[6]);
    s.cg[7] = fmaf(d1, a11, s.cg[7]);
  } else if (gmask & GRAD_V) {
    float w[8];
    trilerp_weights(c.f, w);
    if (LDS) {
      const float q = FIX ? (MODE == 0 ? s.dhq : d_hat * s.qs) : d_hat;
      float g[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) g[k] = w[k] * q;
      lds_add8<FIX, WIDE>(acc, br, base, g);
    } else {
      const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
      float* g = vd.dV + (c.k[2] * sz + c.k[1] * sy + c.k[0]);
      gadd(g, w[0] * d_hat);
      gadd(g + 1, w[1] * d_hat);
      gadd(g + sy, w[2] * d_hat);
      gadd(g + sy + 1, w[3] * d_hat);
      gadd(g + sz, w[4] * d_hat);
      gadd(g + sz + 1, w[5] * d_hat);
      gadd(g + sz + sy, w[6] * d_hat);
      gadd(g + sz + sy + 1, w[7] * d_hat);
    }
  }
  if (need_xhat) {
    float gd[3];
    trilerp_grad(v, c.f, gd);
    const float sc = d_hat * vd.inv_h;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float xh = sc * gd[a];
      s.xo_hat[a] += (double)xh;
      s.si[a] += (double)fi * (double)xh;
    }
  }
}

template <int MODEL, int DT, bool LDS, int MODE, bool XH>
__device__ __forceinline__ void march_adj(const ViewDesc& vd, const RayG& r, int a, int b,
                                          const float* stage, float* acc, const Brick& br,
                                          const float4* tfl, float* dtf, int gmask, bool need_v,
                                          bool cell_acc, AdjState& s) {
  const float fa = (float)a;
  for (float fi = (float)(b - 1); fi >= fa; fi -= 1.0f)
    adj_sample<MODEL, DT, LDS, MODE, XH>(vd, r, fi, stage, acc, br, tfl, dtf, gmask, need_v,
                                     cell_acc, s, 0.0f);
  constexpr bool FIX = LDS && MODE <= 2;
  constexpr bool WIDE = MODEL == DDVR_EMISSION_ABSORPTION;
  if (cell_acc) cell_flush<LDS, FIX, WIDE>(vd, br, acc, s);   // the brick changes with the slab
}

// Absorption-only closed form (d_hat = dt T_N ahat for every sample) of
// samples [a, b) with the density gradient only: one cell run at a time, its 8
// corner weight sums times d_hat added to the LDS brick in fixed point (dhq =
// d_hat qs).  The order of the runs does not matter: they march front to back.
__device__ __forceinline__ void march_adj_ao_runs(const ViewDesc& vd, const RayG& r,
                                                  const RunGeo& g, int a, int b, float* acc,
                                                  const Brick& br, const AdjState& s) {
  const float fb = (float)b;
  for (float fi = (float)a; fi < fb;) {
    Cell c;
    float kf[3];
    locate_cell(r, fi, vd, c, kf);
    const float fe = run_end(r, g, kf, fi, fb);
    const float m = fe - fi;
    float f[3];
    run_mid(r, kf, fmaf(0.5f, m - 1.0f, fi), f);
    float w[8];
    run_weight_sums(f, m, g, s.dhq, w);
    lds_add8<true>(acc, br, brick_base(br, c), w);
    fi = fe;
  }
}

// Camera adjoint of one ray (last line of Alg. 2 on [x_o_hat; omega_hat]).
// out[0..11] = d frame, out[12] = d step.
__device__ __forceinline__ void camera_adjoint(const ViewDesc& vd, const RayG& r,
                                               const AdjState& s, bool hit, float* out) {
#pragma unroll
  for (int k = 0; k < 13; ++k) out[k] = 0.0f;
  if (!hit) return;
  out[12] = (float)(s.dstep + (double)r.om[0] * s.si[0] + (double)r.om[1] * s.si[1] +
                    (double)r.om[2] * s.si[2]);
  float oh[3], eh[3];
  float t0h = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    oh[a] = (float)((double)vd.step * s.si[a] + (double)r.t0 * s.xo_hat[a]);
    eh[a] = (float)s.xo_hat[a];
    t0h += r.om[a] * (float)s.xo_hat[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a == r.axis) {
      eh[a] -= t0h / r.om[a];
      oh[a] -= t0h * r.t0 / r.om[a];
    }
  const float od = r.om[0] * oh[0] + r.om[1] * oh[1] + r.om[2] * oh[2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float wh = (oh[a] - r.om[a] * od) / r.wlen;
    out[a] = eh[a];
    out[3 + a] = wh;
    out[6 + a] = r.u * wh;
    out[9 + a] = r.v * wh;
  }
}

// ---------------------------------------------------------------------------
// the render kernel: forward, adjoint, or fused forward + L2 + adjoint
// ---------------------------------------------------------------------------
template <int WAVES> struct TileShape;
template <> struct TileShape<1> { static constexpr int BX = 1, BY = 1; };
template <> struct TileShape<2> { static constexpr int BX = 2, BY = 1; };
template <> struct TileShape<4> { static constexpr int BX = 2, BY = 2; };

// Lane -> pixel inside a tile (local coordinates lx, ly): each wave an 8x8
// block of adjacent pixels, or (interleaved) an 8x8 lattice of every other
// pixel, so that the lanes of a wave are two pixels apart.  Both maps are
// bijections of the tile.
template <int WAVES>
__device__ __forceinline__ void tile_pixel(bool interleaved, int wid, int lane, int& lx, int& ly) {
  using TS = TileShape<WAVES>;
  if (interleaved && WAVES > 1) {
    lx = 2 * (lane & 7) + (wid % TS::BX);
    ly = TS::BY == 2 ? 2 * (lane >> 3) + wid / 2 : (lane >> 3);
  } else {
    lx = (wid % TS::BX) * 8 + (lane & 7);
    ly = (wid / TS::BX) * 8 + (lane >> 3);
  }
}

// One tile of the render: forward, adjoint, or fused forward + L2 + adjoint.
template <int MODEL, int DT, int WAVES, int PASS, bool XH>
__device__ __forceinline__ void render_tile(const LaunchParams& p, const int item, float* smem) {
  constexpr int NT = WAVES * 64;
  constexpr int TW = 8 * TileShape<WAVES>::BX, TH = 8 * TileShape<WAVES>::BY;
  constexpr bool EA = MODEL == DDVR_EMISSION_ABSORPTION;

  int view = 0, tile = item;
  if (p.work) {
    const int w = p.work[item];
    view = w >> 20;
    tile = w & 0xFFFFF;
  }
  const ViewDesc vd = p.views ? p.views[view] : p.one;
  const int cap = p.lds_cap;
  const bool adj_pass = PASS != PASS_FWD;
  const bool want_dv = adj_pass && (p.grad_mask & GRAD_V) && vd.dV != nullptr;
  int gmask = p.grad_mask;
  if (!vd.dV) gmask &= ~GRAD_V;
  if (!vd.dTF) gmask &= ~GRAD_TF;
  if (!vd.dcam || !XH) gmask &= ~GRAD_CAM;
  if (!vd.dstep || !XH) gmask &= ~GRAD_STEP;

  // LDS carve-up: one brick region, or two when the adjoint needs the grid
  // values and a gradient accumulator at the same time
  // (the emission-absorption gradient brick holds 64-bit entries: 2 words
  // per voxel; the host keeps cap even so that they are 8-byte aligned)
  constexpr int ACCW = EA ? 2 : 1;
  float* stage = smem;
  float* acc = smem + (p.lds_two ? cap : 0);
  float4* tfl = reinterpret_cast<float4*>(smem + (p.lds_two ? (1 + ACCW) * cap : cap));
  float* dtf = reinterpret_cast<float*>(tfl) + (EA ? 4 * vd.R : 0);
  int* iscratch = reinterpret_cast<int*>(dtf + (EA ? 4 * vd.R : 0));
  float* fscratch = reinterpret_cast<float*>(iscratch);

  if (EA) {
    for (int k = threadIdx.x; k < 4 * vd.R; k += NT) {
      reinterpret_cast<float*>(tfl)[k] = vd.tf[k];
      dtf[k] = 0.0f;
    }
  }

  const int tx = tile % vd.tiles_x, ty = tile / vd.tiles_x;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // lane -> pixel of each pass (lane_map: 0 compact, 1 interleaved, 2 compact
  // forward + interleaved adjoint, 3 the reverse).  The forward gathers from
  // the staged brick best with adjacent rays in a wave; the adjoint's LDS
  // atomics collide less with rays two pixels apart.
  const bool il_fwd = p.lane_map == 1 || p.lane_map == 3;
  const bool il_adj = p.lane_map == 1 || p.lane_map == 2;
  int lx, ly;
  tile_pixel<WAVES>(PASS == PASS_ADJ ? il_adj : il_fwd, wid, lane, lx, ly);
  int px = tx * TW + lx, py = ty * TH + ly;
  bool valid = px < vd.W && py < vd.H;
  int64_t pix = (int64_t)py * vd.W + px;
  RayG r;
  setup_ray(vd, px, py, valid, r);
  bool hit = r.N > 0;
  RunGeo rg;
  if (MODEL == DDVR_ABSORPTION) run_geo(vd, r, rg);

  // slab bookkeeping (shared by both passes): the tile's earliest entry
  // distance (shells), the longest slab tried
  const int kmax = cap > 0 ? max(p.slab_kmax, 4) : kMaxSamples + 1;
  const bool want_axis = p.slab_axis != 0;
  float tmin = 0.0f;
  if (cap > 0) tmin = wg_min_f<NT>(hit ? r.t0 : INFINITY, fscratch);
  __syncthreads();   // TF table visible

  const int C = EA ? 4 : 1;
  float gimg[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  float TN = 1.0f;

  if (PASS == PASS_FWD || PASS == PASS_FUSED) {
    FwdState fs;
    fs.C[0] = fs.C[1] = fs.C[2] = 0.0f;
    fs.T = 1.0f;
    fs.sigma = 0.0f;
    SlabWalk sw;
    walk_init<NT>(vd, r, r.N, tx, ty, TW, TH, cap, kmax, want_axis, tmin, iscratch, sw);
    for (float pos = sw.lo; pos < sw.hi;) {
      float lo, hi;
      int a, b;
      Brick br;
      const int st = walk_next<NT>(vd, r, r.N, sw, pos, +1, cap, lo, hi, a, b, iscratch, br);
      if (st == 1) {
        stage_brick<NT, DT>(vd, br, stage, nullptr);
        __syncthreads();
        if (MODEL == DDVR_ABSORPTION) march_fwd_ao_runs<DT, true>(vd, r, rg, a, b, stage, br, fs);
        else march_fwd<MODEL, DT, true>(vd, r, a, b, stage, br, tfl, fs);
      } else if (st == 2) {
        // (a launch without bricks -- PLAIN, the per-sample baseline -- keeps
        // the per-sample march)
        if (MODEL == DDVR_ABSORPTION && cap > 0)
          march_fwd_ao_runs<DT, false>(vd, r, rg, a, b, stage, br, fs);
        else
          march_fwd<MODEL, DT, false>(vd, r, a, b, stage, br, tfl, fs);
      }
      pos = hi;
    }
    float out[4];
    if (EA) {
      TN = fs.T;
      out[0] = fs.C[0]; out[1] = fs.C[1]; out[2] = fs.C[2]; out[3] = 1.0f - TN;
    } else {
      TN = __expf(-vd.step * fs.sigma);
      out[0] = 1.0f - TN;
    }
    if (valid) {
      if (EA) reinterpret_cast<float4*>(vd.image)[pix] = make_float4(out[0], out[1], out[2], out[3]);
      else vd.image[pix] = out[0];
      if (vd.trans) vd.trans[pix] = TN;
    }
    if (PASS == PASS_FUSED) {
      float loss = 0.0f;
      if (valid) {
        for (int ch = 0; ch < C; ++ch) {
          const float dlt = out[ch] - vd.target[pix * C + ch];
          gimg[ch] = loss_seed((p.flags & DDVR_LOSS_L1) != 0, p.loss_scale, dlt, loss);
        }
      }
      if (p.loss_out) {
        float l = loss * p.loss_scale;
        wg_sum_n<NT>(&l, 1, fscratch);
        if (threadIdx.x == 0 && l != 0.0f) atomicAdd(p.loss_out, (double)l);
      }
    }
  }
  if (PASS == PASS_FWD) return;

  // Fused pass with different lane maps: hand each ray's T_N and upstream
  // gradient over to the lane that runs its adjoint, through the (now idle)
  // staging region, and set that lane's ray up again.
  // The ray itself travels along: its float64 setup is not repeated (that
  // would keep float64 temporaries live next to the forward's results).  The
  // hand-over needs (C + 1 + RAYW) words per lane of the (idle) brick regions;
  // with less, the adjoint keeps the forward's lane map.
  constexpr int RAYW = (int)(sizeof(RayG) / sizeof(float));
  const int hand_words = (p.lds_two ? 1 + ACCW : 1) * cap;
  if (PASS == PASS_FUSED && il_adj != il_fwd && hand_words >= (C + 1 + RAYW) * NT) {
    __syncthreads();                       // the forward's last brick reads are done
    const int lp = ly * TW + lx;
    stage[lp] = TN;
    for (int ch = 0; ch < C; ++ch) stage[(ch + 1) * NT + lp] = gimg[ch];
    {
      const float* rw = reinterpret_cast<const float*>(&r);
#pragma unroll
      for (int k = 0; k < RAYW; ++k) stage[(C + 1 + k) * NT + lp] = rw[k];
    }
    __syncthreads();
    tile_pixel<WAVES>(il_adj, wid, lane, lx, ly);
    const int lq = ly * TW + lx;
    TN = stage[lq];
    for (int ch = 0; ch < C; ++ch) gimg[ch] = stage[(ch + 1) * NT + lq];
    {
      float* rw = reinterpret_cast<float*>(&r);
#pragma unroll
      for (int k = 0; k < RAYW; ++k) rw[k] = stage[(C + 1 + k) * NT + lq];
    }
    px = tx * TW + lx;
    py = ty * TH + ly;
    valid = px < vd.W && py < vd.H;
    pix = (int64_t)py * vd.W + px;
    if (MODEL == DDVR_ABSORPTION) run_geo(vd, r, rg);
    hit = r.N > 0;
    // the staging region is next written after the adjoint's first brick
    // reduction, whose barriers order it after these reads
  }

  if (PASS == PASS_ADJ && valid) {
    TN = vd.trans[pix];
    for (int ch = 0; ch < C; ++ch) gimg[ch] = vd.d_image[pix * C + ch];
  }

  // choose the adjoint route of this ray; a ray with a zero upstream gradient
  // contributes nothing and is skipped
  const int mode = p.flags & DDVR_ADJ_MODE_MASK;
  const bool seeded = gimg[0] != 0.0f || gimg[1] != 0.0f || gimg[2] != 0.0f || gimg[3] != 0.0f;
  bool fallback = false;
  if (hit && seeded) {
    if (p.fb_all) fallback = true;
    else if (((EA && mode == DDVR_ADJ_AUTO) || mode == DDVR_ADJ_INVERT_ALPHA) &&
             !(TN >= p.fb_tmin))
      fallback = true;
    if (!p.fb_count) fallback = false;
  }
  {
    const uint64_t m = __ballot(fallback);
    if (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(p.fb_count, __popcll(m));
      base = __shfl(base, leader, 64);
      if (fallback) {
        const int my = base + __popcll(m & ((1ull << lane) - 1ull));
        if (my < p.fb_cap) p.fb_list[my] = ((int64_t)view << 32) | pix;
      }
    }
  }
  const int Nadj = (fallback || !seeded) ? 0 : r.N;

  AdjState s;
  s.Chat[0] = EA ? gimg[0] : 0.0f;
  s.Chat[1] = EA ? gimg[1] : 0.0f;
  s.Chat[2] = EA ? gimg[2] : 0.0f;
  s.ahat = EA ? gimg[3] : gimg[0];
  s.Tn = TN;
  s.an = 1.0f - TN;
  s.P = TN * s.ahat;
  s.xo_hat[0] = s.xo_hat[1] = s.xo_hat[2] = 0.0;
  s.si[0] = s.si[1] = s.si[2] = 0.0;
  s.dstep = 0.0;
  s.tj = -1;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) { s.tg0[ch] = 0.0f; s.tg1[ch] = 0.0f; }
  s.ckey = -1;
  s.gkey = -1;
#pragma unroll
  for (int k = 0; k < 8; ++k) s.cg[k] = 0.0f;

  // Fixed-point scale of the LDS density-gradient brick.  A straight ray has
  // at most lmax samples in the 2x2x2 cells around a voxel (chord <=
  // 2*sqrt(3) voxels), and each adds w*d_hat with trilinear weight |w| <= 1.
  // B bounds every brick entry by a sum over the tile's rays of per-ray
  // bounds on their contributions to one voxel:
  //  * absorption-only: d_hat = dt*T_N*ahat exactly in the closed form, so a
  //    ray adds at most lmax*|d_hat|; B = NT * lmax * max|d_hat|.  The T- and
  //    alpha-form inversions compute the same d_hat = dt T^(i) e_i ahat^(i+1)
  //    = dt T^(i+1) ahat^(i+1) (no emission: ahat^(i) = e_i ahat^(i+1)) up
  //    to the float32 drift of the recovered T^(i), which the margin below
  //    covers (relative 2 N 2^-24 <= 1/2 for the T-form at the sample cap,
  //    2^-14 for the alpha-form, whose rays with T_N < 2^-10 fall back);
  //  * emission-absorption (T- or alpha-form inversion): d_hat = (R-1) *
  //    (slope_rgb . alpha_i T^(i) Chat + slope_tau * tau_hat).  Along a ray
  //    sum_i alpha_i T^(i) = 1 - T_N <= 1, so the colour part adds at most
  //    (R-1) S_rgb |Chat|_1 in total; with P_i = T^(i) ahat^(i) the blend
  //    adjoint gives P_(i+1) = T_N ahat_N - sum_(j>i) T^(j) alpha_j (rgb_j .
  //    Chat), so e_i times the alpha adjoint is at most A = T_N |ahat_N| +
  //    2 rgbmax |Chat|_1 and the opacity part adds at most lmax (R-1) S_tau
  //    dt A (S: largest TF segment slopes, rgbmax: largest |colour|).
  //    B = the sum of these per-ray bounds over the tile.
  // qs = 2^(28 - ceil(log2 B)) keeps every partial sum below 2^28 in the
  // 32-bit brick (margin 8 for float32 rounding of the recovered T^(i)).  The
  // emission-absorption bound is looser (a sum over the tile of per-ray
  // worst cases), so its brick holds 64-bit entries and qs = 2^(50 - ceil(
  // log2 B)): every value stays below 2^51, the range of the float64
  // rounding of round_i64, and sums below 2^50 (margin 2^13 to overflow).
  // A tile whose bound is not finite (NaN or Inf upstream gradients or TF)
  // takes the float32 route without LDS bricks, which propagates them.
  const bool closed_form = !EA && mode == DDVR_ADJ_AUTO;
  const bool ao_bound = !EA && (mode == DDVR_ADJ_AUTO || mode == DDVR_ADJ_INVERT_T ||
                                mode == DDVR_ADJ_INVERT_ALPHA);
  s.qs = 1.0f;
  float inv_qs = 1.0f;
  bool fix_ok = true;
  {
    const bool lane_dv = want_dv && Nadj > 0;
    const float lmax = floorf(3.4641017f / (vd.step * vd.inv_h)) + 2.0f;
    // per-lane maxima, reduced in one pass: tile end, then the bound's factors
    constexpr int NV = EA ? 4 : 2;
    int v[NV];
    v[0] = 0;
    if (!EA) {
      v[1] = __float_as_int((ao_bound && lane_dv) ? fabsf(vd.step * s.P) : 0.0f);
    } else {
      float srgb = 0.0f, stau = 0.0f, rgbmax = 0.0f;
      if (want_dv) {
        for (int k = threadIdx.x; k < vd.R - 1; k += NT) {
          const float4 a = tfl[k], b = tfl[k + 1];
          srgb = fmaxf(srgb, fmaxf(fabsf(b.x - a.x), fmaxf(fabsf(b.y - a.y), fabsf(b.z - a.z))));
          stau = fmaxf(stau, fabsf(b.w - a.w));
          rgbmax = fmaxf(rgbmax, fmaxf(fmaxf(fabsf(a.x), fabsf(a.y)), fabsf(a.z)));
          rgbmax = fmaxf(rgbmax, fmaxf(fmaxf(fabsf(b.x), fabsf(b.y)), fabsf(b.z)));
        }
      }
      v[1] = __float_as_int(srgb);
      v[2] = __float_as_int(stau);
      v[3] = __float_as_int(rgbmax);
    }
    wg_max_n<NT>(v, NV, iscratch);
    float B;
    if (!EA) {
      B = __int_as_float(v[1]) * (float)NT * lmax;
    } else {
      float b = 0.0f;
      if (lane_dv) {
        const float c1 = fabsf(s.Chat[0]) + fabsf(s.Chat[1]) + fabsf(s.Chat[2]);
        const float A = fabsf(TN * s.ahat) + 2.0f * __int_as_float(v[3]) * c1;
        b = (float)(vd.R - 1) *
            (__int_as_float(v[1]) * c1 + lmax * __int_as_float(v[2]) * vd.step * A);
      }
      B = wg_sum_all<NT>(b, fscratch) * 1.0001f;   // margin for the float32 sum
    }
    if (!(B < INFINITY)) {
      fix_ok = false;
    } else if (B > 0.0f) {
      int ex;
      (void)frexpf(B, &ex);          // B < 2^ex
      const int e = (EA ? 50 : 28) - ex;
      if (e > 120) {
        fix_ok = false;              // subnormal-scale gradients: float32 route
      } else {
        s.qs = ldexpf(1.0f, max(e, -120));
        inv_qs = ldexpf(1.0f, -max(e, -120));
      }
    }
  }
  const bool use_fix = closed_form && fix_ok;
  // the brick holds fixed point on every route that stages it (a tile
  // without a finite bound stages nothing: acap = 0 below)
  const bool lds_fix = (ao_bound || EA) && fix_ok;
  s.dh = vd.step * s.P;
  s.dhq = s.dh * s.qs;
  const bool need_v = EA || (gmask & (GRAD_CAM | GRAD_STEP)) || !use_fix;
  const int acap = fix_ok ? cap : 0;
  SlabWalk sw;
  walk_init<NT>(vd, r, Nadj, tx, ty, TW, TH, cap, kmax, want_axis, tmin, iscratch, sw);
  for (float pos = sw.hi; pos > sw.lo;) {
    float lo, hi;
    int a, b;
    Brick br;
    const int st = walk_next<NT>(vd, r, Nadj, sw, pos, -1, acap, lo, hi, a, b, iscratch, br);
    pos = lo;
    if (st == 0) continue;
    if (st == 1) {
      stage_brick<NT, DT, EA>(vd, br, need_v ? stage : nullptr, want_dv ? acc : nullptr);
      __syncthreads();
      if (use_fix && !EA && !XH && want_dv)
        march_adj_ao_runs(vd, r, rg, a, b, acc, br, s);
      else if (use_fix)
        march_adj<MODEL, DT, true, 0, XH>(vd, r, a, b, stage, acc, br, tfl, dtf, gmask, need_v,
                                      p.cell_acc, s);
      else if (mode == DDVR_ADJ_INVERT_ALPHA)
        march_adj<MODEL, DT, true, 2, XH>(vd, r, a, b, stage, acc, br, tfl, dtf, gmask, need_v,
                                      p.cell_acc, s);
      else
        march_adj<MODEL, DT, true, 1, XH>(vd, r, a, b, stage, acc, br, tfl, dtf, gmask, need_v,
                                      p.cell_acc, s);
      __syncthreads();
      if (want_dv) {
        if (lds_fix) flush_brick<NT, true, EA>(vd, br, acc, inv_qs);
        else flush_brick<NT, false>(vd, br, acc, 1.0f);
      }
    } else {
      if (use_fix)
        march_adj<MODEL, DT, false, 0, XH>(vd, r, a, b, stage, acc, br, tfl, dtf, gmask, need_v,
                                       p.cell_acc, s);
      else if (mode == DDVR_ADJ_INVERT_ALPHA)
        march_adj<MODEL, DT, false, 2, XH>(vd, r, a, b, stage, acc, br, tfl, dtf, gmask, need_v,
                                       p.cell_acc, s);
      else
        march_adj<MODEL, DT, false, 1, XH>(vd, r, a, b, stage, acc, br, tfl, dtf, gmask, need_v,
                                       p.cell_acc, s);
    }
  }
  if (EA && (gmask & GRAD_TF)) tf_flush(s, dtf);

  if (XH && (gmask & (GRAD_CAM | GRAD_STEP))) {
    float cg[13];
    camera_adjoint(vd, r, s, Nadj > 0, cg);
    wg_sum_n<NT>(cg, 13, fscratch);
    if (threadIdx.x == 0) {
      if (gmask & GRAD_CAM)
        for (int k = 0; k < 12; ++k)
          if (cg[k] != 0.0f) gadd(vd.dcam + k, cg[k]);
      if ((gmask & GRAD_STEP) && cg[12] != 0.0f) gadd(vd.dstep, cg[12]);
    }
  }
  if (EA && (gmask & GRAD_TF)) {
    __syncthreads();
    for (int k = threadIdx.x; k < 4 * vd.R; k += NT)
      if (dtf[k] != 0.0f) gadd(vd.dTF + k, dtf[k]);
  }
}

// The render kernel.  With a fixed storage type: one tile per workgroup,
// blockIdx remapped so that each XCD takes a contiguous range of tiles.  With
// the storage type chosen per view (DT_DYN, used by uneven and mixed batches):
// persistent workgroups pop tiles from a queue ordered longest-first.  The two
// forms are separate instantiations because the tile loop costs registers.
template <int MODEL, int DT, int WAVES, int PASS, bool XH>
__global__ __launch_bounds__(WAVES * 64) void k_render(const LaunchParams p) {
  extern __shared__ __align__(16) float smem[];
  if constexpr (DT == DT_DYN) {
    __shared__ int s_item;
    for (;;) {
      if (threadIdx.x == 0) s_item = atomicAdd(p.queue, 1);
      __syncthreads();
      const int item = s_item;
      __syncthreads();
      if (item >= p.n_items) break;
      render_tile<MODEL, DT, WAVES, PASS, XH>(p, item, smem);
      __syncthreads();   // the next tile reuses the LDS
    }
  } else {
    render_tile<MODEL, DT, WAVES, PASS, XH>(p, p.xcd_remap ? xcd_remap(blockIdx.x, gridDim.x)
                                                           : (int)blockIdx.x, smem);
  }
}

// ---------------------------------------------------------------------------
// forward-mode derivatives (Sec. 4.2, forward differentiation)
// ---------------------------------------------------------------------------
// Every quantity of the forward march carries its derivatives along P
// directions in (camera frame, step) space, as the dual numbers of Sec. 4.2
// do.  The sample count N is piecewise constant in the camera and the step and
// is not differentiated (the same reading as the adjoint).

// Tangents of the ray's grid-unit positions: q_i' = qo' + i*dq'.
template <int P>
struct RayTan {
  float qo[P][3];
  float dq[P][3];
};

template <int P>
__device__ __forceinline__ void setup_tangent(const ViewDesc& vd, const RayG& r,
                                              const float (*dir)[13], RayTan<P>& t) {
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const float* de = dir[k];
    const float* dfw = dir[k] + 3;
    const float* drt = dir[k] + 6;
    const float* dup = dir[k] + 9;
    const float dstep = dir[k][12];
    // w = fwd + u right + v up, omega = w/|w|: omega' = (w' - omega (omega . w'))/|w|
    float wd[3], od = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      wd[a] = dfw[a] + r.u * drt[a] + r.v * dup[a];
      od = fmaf(r.om[a], wd[a], od);
    }
    float omd[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) omd[a] = (wd[a] - r.om[a] * od) / r.wlen;
    // entry distance t0 = (b - e_a)/omega_a on the entry plane a
    float t0d = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (a == r.axis) t0d = -(de[a] + r.t0 * omd[a]) / r.om[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      t.qo[k][a] = (de[a] + t0d * r.om[a] + r.t0 * omd[a]) * vd.inv_h;
      t.dq[k][a] = (dstep * r.om[a] + vd.step * omd[a]) * vd.inv_h;
    }
  }
}

template <int P>
struct TanState {
  float C[3], T, sigma;           // primal (as FwdState)
  float Cd[P][3], Td[P], sigd[P]; // derivatives
};

template <int MODEL, int DT, bool LDS, int P>
__device__ __forceinline__ void march_tan(const ViewDesc& vd, const RayG& r, const RayTan<P>& t,
                                          const float (*dir)[13], int a, int b,
                                          const float* stage, const Brick& br,
                                          const float4* tfl, TanState<P>& s) {
  const float fb = (float)b;
  for (float fi = (float)a; fi < fb; fi += 1.0f) {
    Cell c;
    locate(r, fi, vd, c);
    float v[8];
    if (LDS) fetch_lds(stage, br, brick_base(br, c), v);
    else fetch_global<DT>(vd, c, v);
    float g[3];
    trilerp_grad(v, c.f, g);            // d density / d q (grid units)
    const float d = trilerp(v, c.f);
    float dd[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      float x = 0.0f;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) x = fmaf(g[ax], fmaf(fi, t.dq[k][ax], t.qo[k][ax]), x);
      dd[k] = x;
    }
    if (MODEL == DDVR_ABSORPTION) {
      s.sigma += d;
#pragma unroll
      for (int k = 0; k < P; ++k) s.sigd[k] += dd[k];
    } else {
      TFv tv;
      tf_eval(tfl, vd.R, d, tv);
      const float4 ta = tfl[tv.j], tb = tfl[tv.j + 1];
      const float sc = tv.inside ? (float)(vd.R - 1) : 0.0f;   // d u / d density
      const float sr = sc * (tb.x - ta.x), sg = sc * (tb.y - ta.y), sb = sc * (tb.z - ta.z),
                  st = sc * (tb.w - ta.w);
      const float e = __expf(-vd.step * tv.tau);
      const float alpha = __fsub_rn(1.0f, e);
#pragma unroll
      for (int k = 0; k < P; ++k) {
        // c = alpha rgb: c' = alpha' rgb + alpha rgb'; C' += T' c + T c'; T' = T' e + T e'
        const float taud = st * dd[k];
        const float ed = -e * fmaf(dir[k][12], tv.tau, vd.step * taud);
        const float ad = -ed;
        const float ta = s.Td[k] * alpha;
        const float cd0 = fmaf(ad, tv.r, alpha * sr * dd[k]);
        const float cd1 = fmaf(ad, tv.g, alpha * sg * dd[k]);
        const float cd2 = fmaf(ad, tv.b, alpha * sb * dd[k]);
        s.Cd[k][0] = fmaf(ta, tv.r, fmaf(s.T, cd0, s.Cd[k][0]));
        s.Cd[k][1] = fmaf(ta, tv.g, fmaf(s.T, cd1, s.Cd[k][1]));
        s.Cd[k][2] = fmaf(ta, tv.b, fmaf(s.T, cd2, s.Cd[k][2]));
        s.Td[k] = fmaf(s.Td[k], e, s.T * ed);
      }
      // primal exactly as march_fwd (bitwise the same image)
      const float w = __fmul_rn(s.T, alpha);
      s.C[0] = fmaf(w, tv.r, s.C[0]);
      s.C[1] = fmaf(w, tv.g, s.C[1]);
      s.C[2] = fmaf(w, tv.b, s.C[2]);
      s.T *= e;
    }
  }
}

// One 16x16 tile per workgroup (4 waves, compact lane map), slab-synchronous
// LDS staging as in the forward of k_render.
template <int MODEL, int DT, int P>
__global__ __launch_bounds__(256) void k_tangent(const TangentParams p) {
  constexpr int WAVES = 4, NT = 256, TW = 16, TH = 16;
  constexpr bool EA = MODEL == DDVR_EMISSION_ABSORPTION;
  extern __shared__ __align__(16) float smem[];
  const ViewDesc& vd = p.one;
  const int cap = p.lds_cap;
  float* stage = smem;
  float4* tfl = reinterpret_cast<float4*>(smem + cap);
  int* iscratch = reinterpret_cast<int*>(reinterpret_cast<float*>(tfl) + (EA ? 4 * vd.R : 0));
  float* fscratch = reinterpret_cast<float*>(iscratch);
  if (EA)
    for (int k = threadIdx.x; k < 4 * vd.R; k += NT) reinterpret_cast<float*>(tfl)[k] = vd.tf[k];

  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % vd.tiles_x, ty = tile / vd.tiles_x;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int lx, ly;
  tile_pixel<WAVES>(false, wid, lane, lx, ly);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool valid = px < vd.W && py < vd.H;
  const int64_t pix = (int64_t)py * vd.W + px;
  RayG r;
  setup_ray(vd, px, py, valid, r);
  const bool hit = r.N > 0;
  RayTan<P> t;
  setup_tangent<P>(vd, r, p.dir, t);

  int off = 0, tile_end;
  const int kmax = cap > 0 ? max(p.slab_kmax, 4) : kMaxSamples + 1;
  if (cap > 0) {
    const float tmin = wg_min_f<NT>(hit ? r.t0 : INFINITY, fscratch);
    off = hit ? (int)rintf((r.t0 - tmin) / vd.step) : 0;
  }
  {
    int e = hit ? off + r.N : 0;
    wg_max_n<NT>(&e, 1, iscratch);
    tile_end = e;
  }
  __syncthreads();   // TF table visible

  TanState<P> s;
  s.C[0] = s.C[1] = s.C[2] = 0.0f;
  s.T = 1.0f;
  s.sigma = 0.0f;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    s.Cd[k][0] = s.Cd[k][1] = s.Cd[k][2] = 0.0f;
    s.Td[k] = 0.0f;
    s.sigd[k] = 0.0f;
  }
  int K = min(vd.slab_k, kmax);
  for (int pos = 0; pos < tile_end;) {
    int lo, hi;
    Brick br;
    const int st = pick_slab<NT>(vd, r, off, r.N, pos, +1, tile_end, cap, K, kmax, lo, hi,
                                 iscratch, br);
    int a, b;
    slab_range(lo, hi, off, r.N, a, b);
    if (st == 1) {
      stage_brick<NT, DT>(vd, br, stage, nullptr);
      __syncthreads();
      march_tan<MODEL, DT, true, P>(vd, r, t, p.dir, a, b, stage, br, tfl, s);
    } else if (st == 2) {
      march_tan<MODEL, DT, false, P>(vd, r, t, p.dir, a, b, stage, br, tfl, s);
    }
    pos = hi;
  }

  constexpr int C = EA ? 4 : 1;
  float out[4], outd[P][4];
  if (EA) {
    out[0] = s.C[0]; out[1] = s.C[1]; out[2] = s.C[2]; out[3] = 1.0f - s.T;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      outd[k][0] = s.Cd[k][0]; outd[k][1] = s.Cd[k][1]; outd[k][2] = s.Cd[k][2];
      outd[k][3] = -s.Td[k];
    }
  } else {
    // alpha = 1 - exp(-dt sigma): alpha' = T_N (dt' sigma + dt sigma')
    const float TN = __expf(-vd.step * s.sigma);
    out[0] = 1.0f - TN;
#pragma unroll
    for (int k = 0; k < P; ++k) outd[k][0] = TN * fmaf(p.dir[k][12], s.sigma, vd.step * s.sigd[k]);
  }
  if (valid) {
    if (vd.image)
      for (int ch = 0; ch < C; ++ch) vd.image[pix * C + ch] = out[ch];
    if (p.image_dot) {
      const int64_t plane = (int64_t)vd.W * vd.H * C;
#pragma unroll
      for (int k = 0; k < P; ++k)
        for (int ch = 0; ch < C; ++ch) p.image_dot[k * plane + pix * C + ch] = outd[k][ch];
    }
  }
  if (p.d_dir) {
    // forward-delayed: contract with the upstream gradient in the same pass
    float dk[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      float x = 0.0f;
      if (valid)
        for (int ch = 0; ch < C; ++ch) x = fmaf(vd.d_image[pix * C + ch], outd[k][ch], x);
      dk[k] = x;
    }
    wg_sum_n<NT>(dk, P, fscratch);
    if (threadIdx.x == 0)
      for (int k = 0; k < P; ++k)
        if (dk[k] != 0.0f) gadd(p.d_dir + k, dk[k]);
  }
}

// ---------------------------------------------------------------------------
// segment-checkpoint fallback (one ray per thread, queued by the main kernel)
// ---------------------------------------------------------------------------
// One queued ray per lane; all lanes of the wave call it together (`live`:
// the lane holds a ray).  TAB: the ray's TF gradient goes to the workgroup's
// LDS table `tab` (its view's dTF is the launch's fb_dtf), which the kernel
// adds to global memory once per workgroup; without it every TF-segment
// change of every ray would be a global atomic on the same few hundred
// floats.
//
// Segments: the wave splits sample indices into segments of K =
// ceil(sqrt(N_max)) samples (N_max: the wave's longest ray), so that its
// lanes march the same segment at a time.  The forward keeps T at every
// segment start; the adjoint re-marches a segment forward for its T^(i) (the
// same float32 products in the same order as the first pass) and then runs it
// back to front, in windows of sample indices.  When the wave's rays write
// one gradient grid and the cells a window touches fit the wave's LDS region
// `wacc`, the window's density gradient is accumulated there (float32 LDS
// atomics at each cell exit) and added to global memory once per touched
// voxel; otherwise every cell exit adds its 8 corners to global memory.
template <int MODEL, int DT, int FUSED, bool TAB>
__device__ __forceinline__ void fallback_ray(const LaunchParams& p, int64_t code, bool live,
                                             float* ws, float* tab, float* wacc) {
  constexpr bool EA = MODEL == DDVR_EMISSION_ABSORPTION;
  const int lane = threadIdx.x & 63;
  const int view = live ? (int)(code >> 32) : 0;
  const int64_t pix = live ? (code & 0xFFFFFFFFll) : 0;
  const ViewDesc vd = p.views ? p.views[view] : p.one;
  int gmask = p.grad_mask;
  if (!vd.dV) gmask &= ~GRAD_V;
  if (!vd.dTF) gmask &= ~GRAD_TF;
  if (!vd.dcam) gmask &= ~GRAD_CAM;
  if (!vd.dstep) gmask &= ~GRAD_STEP;
  float* const dtf = TAB ? tab : vd.dTF;
  const int px = (int)(pix % vd.W), py = (int)(pix / vd.W);
  RayG r;
  setup_ray(vd, px, py, live, r);
  const int N = live ? max(r.N, 0) : 0;
  const int Nw = wave_max_i32(N);
  if (Nw <= 0) return;
  const int C = EA ? 4 : 1;
  float gimg[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (N > 0) {
    for (int ch = 0; ch < C; ++ch) {
      float unused = 0.0f;
      if (FUSED)
        gimg[ch] = loss_seed((p.flags & DDVR_LOSS_L1) != 0, p.loss_scale,
                             vd.image[pix * C + ch] - vd.target[pix * C + ch], unused);
      else gimg[ch] = vd.d_image[pix * C + ch];
    }
  }
  const float4* tfl = reinterpret_cast<const float4*>(vd.tf);
  int K = (int)ceilf(sqrtf((float)Nw));
  while (K * K < Nw) ++K;
  const int nseg = (Nw + K - 1) / K;
  float* ck = ws;             // T at the start of every segment
  float* tseg = ws + nseg;    // T^(i) inside the current segment
  // forward: keep T at segment starts
  {
    float T = 1.0f;
    for (int i = 0; i < N; ++i) {
      if (i % K == 0) ck[i / K] = T;
      Cell c;
      locate(r, (float)i, vd, c);
      float v[8];
      fetch_global<DT>(vd, c, v);
      const float d = trilerp(v, c.f);
      float tau = d;
      if (EA) { TFv t; tf_eval(tfl, vd.R, d, t); tau = t.tau; }
      T *= __expf(-vd.step * tau);
    }
  }
  AdjState s;
  s.Chat[0] = EA ? gimg[0] : 0.0f;
  s.Chat[1] = EA ? gimg[1] : 0.0f;
  s.Chat[2] = EA ? gimg[2] : 0.0f;
  s.ahat = EA ? gimg[3] : gimg[0];
  s.Tn = 0.0f; s.an = 0.0f; s.P = 0.0f;
  s.xo_hat[0] = s.xo_hat[1] = s.xo_hat[2] = 0.0;
  s.si[0] = s.si[1] = s.si[2] = 0.0;
  s.dstep = 0.0;
  s.tj = -1;
  for (int ch = 0; ch < 4; ++ch) { s.tg0[ch] = 0.0f; s.tg1[ch] = 0.0f; }
  s.ckey = -1;
  s.gkey = -1;
  s.qs = 1.0f;
  s.dh = 0.0f; s.dhq = 0.0f;
  for (int k = 0; k < 8; ++k) s.cg[k] = 0.0f;
  // the wave's bricks need one gradient grid: that of its first lane with
  // samples, written by every lane with samples
  const uint64_t has = __builtin_amdgcn_ballot_w64(N > 0);
  const int first = __builtin_ctzll(has);
  const uint64_t dvp = reinterpret_cast<uint64_t>(vd.dV);
  const uint64_t dv0 =
      ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(dvp >> 32), first) << 32) |
      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)dvp, first);
  const int nx0 = __builtin_amdgcn_readlane(vd.nx, first);
  const int ny0 = __builtin_amdgcn_readlane(vd.ny, first);
  float* const g0 = reinterpret_cast<float*>(dv0);
  const bool bricks =
      wacc != nullptr && g0 != nullptr &&
      __builtin_amdgcn_ballot_w64(N > 0 && (dvp != dv0 || vd.nx != nx0 || vd.ny != ny0)) == 0;
  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int i0 = sg * K, i1 = min(N, i0 + K);   // i1 <= i0: no samples here
    if (i0 < i1) {
      tseg[0] = ck[sg];
      for (int i = i0; i < i1; ++i) {
        Cell c;
        locate(r, (float)i, vd, c);
        float v[8];
        fetch_global<DT>(vd, c, v);
        const float d = trilerp(v, c.f);
        float tau = d;
        if (EA) { TFv t; tf_eval(tfl, vd.R, d, t); tau = t.tau; }
        tseg[i - i0 + 1] = tseg[i - i0] * __expf(-vd.step * tau);
      }
    }
    // the segment back to front in windows of m sample indices (the same
    // indices in every lane), m halved until the window's brick fits and
    // doubled again after a window that used under a quarter of it
    int m = K;
    for (int e = min(Nw, i0 + K); e > i0;) {
      int lo, a, b, st;
      Brick br{};
      for (;;) {
        lo = max(i0, e - m);
        a = lo;
        b = min(e, i1);
        if (!bricks) { st = 2; break; }
        if (!range_brick<64>(vd, r, a, b, nullptr, br)) { st = 0; break; }
        if (br.size <= kFallbackBrick) { st = 1; break; }
        if (m <= 4) { st = 2; break; }
        m >>= 1;
      }
      if (st == 1) {
        for (int x = lane; x < br.size; x += 64) wacc[x] = 0.0f;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int i = b - 1; i >= a; --i)
          adj_sample<MODEL, DT, true, 4, true>(vd, r, (float)i, nullptr, wacc, br, tfl, dtf,
                                               gmask, true, true, s, tseg[i - i0]);
        cell_flush<true, false>(vd, br, wacc, s);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int64_t sy = nx0, sz = (int64_t)nx0 * ny0;
        float* const org = g0 + (br.z0 * sz + br.y0 * sy + br.x0);
        const bool narrow = brick_narrow(br, sz);
        for (int x = lane; x < br.size; x += 64) {
          const float g = wacc[x];
          if (g != 0.0f)
            gadd(org + (narrow ? brick_goff<true>(br, x, sy, sz) : brick_goff<false>(br, x, sy, sz)),
                 g);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (4 * br.size < kFallbackBrick) m = min(2 * m, K);
      } else if (st == 2) {
        // density gradient kept per cell in registers, one global atomic per
        // corner when the ray leaves the cell (or the window)
        for (int i = b - 1; i >= a; --i)
          adj_sample<MODEL, DT, false, 3, true>(vd, r, (float)i, nullptr, nullptr, br, tfl, dtf,
                                                gmask, true, true, s, tseg[i - i0]);
        cell_flush<false, false>(vd, br, nullptr, s);
      }
      e = lo;
    }
  }
  if (N <= 0) return;
  if (EA && (gmask & GRAD_TF)) tf_flush(s, dtf);
  if (gmask & (GRAD_CAM | GRAD_STEP)) {
    float cg[13];
    camera_adjoint(vd, r, s, true, cg);
    if (gmask & GRAD_CAM)
      for (int k = 0; k < 12; ++k) gadd(vd.dcam + k, cg[k]);
    if (gmask & GRAD_STEP) gadd(vd.dstep, cg[12]);
  }
}

template <int MODEL, int DT, int FUSED>
__global__ __launch_bounds__(256) void k_fallback(const LaunchParams p) {
  extern __shared__ __align__(16) float fb_smem[];
  // LDS: the TF table (emission-absorption, set by the host when every view
  // that wants a TF gradient writes the same dTF of fb_tf_R entries), then
  // one density brick region of kFallbackBrick floats per wave
  const bool tab = MODEL == DDVR_EMISSION_ABSORPTION && p.fb_dtf != nullptr;
  const int nt = tab ? 4 * p.fb_tf_R : 0;
  float* const wacc = fb_smem + nt + (threadIdx.x >> 6) * kFallbackBrick;
  if (tab) {
    for (int i = threadIdx.x; i < nt; i += blockDim.x) fb_smem[i] = 0.0f;
    __syncthreads();
  }
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  float* ws = p.fb_scratch + (int64_t)slot * p.fb_slot_floats;   // (used by live lanes only)
  const int64_t count = min((int64_t)*p.fb_count, p.fb_cap);
  const int64_t stride = (int64_t)p.fb_slots;
  // the lanes of a wave take consecutive queue entries, round after round
  // (the wave's loop is uniform: lanes without a ray ride along)
  for (int64_t q0 = (int64_t)(slot - lane); q0 < count; q0 += stride) {
    const int64_t q = q0 + lane;
    const bool live = slot < p.fb_slots && q < count;
    const int64_t code = live ? p.fb_list[q] : 0;
    if (tab) fallback_ray<MODEL, DT, FUSED, true>(p, code, live, ws, fb_smem, wacc);
    else fallback_ray<MODEL, DT, FUSED, false>(p, code, live, ws, nullptr, wacc);
  }
  if (tab) {
    __syncthreads();
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {
      const float g = fb_smem[i];
      if (g != 0.0f) gadd(p.fb_dtf + i, g);
    }
  }
}

// ---------------------------------------------------------------------------
// pre-shaded colour volume: (r, g, b, tau) at every vertex, each channel
// interpolated trilinearly, then the same Beer-Lambert segment and
// front-to-back blend as the emission-absorption model (Sec. 3.1; the volume
// Sec. 5.4 reconstructs when it optimises colours directly).  No transfer
// function; the density gradient becomes a 4-channel gradient.
//
// One ray per lane, 16x16-pixel tiles, direct gathers of the 8 corners (one
// 16-byte or 8-byte load per corner), the 4x8 corner gradients of the ray's
// current cell kept in registers and added to global memory when the ray
// leaves the cell.  The adjoint recovers T^(i) by the T-form inversion
// T^(i) = T^(i+1)/e_i (Sec. 4.4); a ray whose T_N is below 2^-100, where that
// inversion loses float32 range, runs instead in forward order with the
// identity alpha_hat^(i+1) T^(i+1) = g_alpha T_N - (C_N - C^(i+1)) . C_hat
// (no division; C_N, T_N from the forward).
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
template <int DT> struct Vox4;
template <> struct Vox4<DDVR_F32> {
  static __device__ __forceinline__ float4 ld(const void* p, int64_t i) {
    const f32x4 x = gmem<f32x4>(p)[i];
    return make_float4(x.x, x.y, x.z, x.w);
  }
};
template <> struct Vox4<DDVR_F16> {
  static __device__ __forceinline__ float4 ld(const void* p, int64_t i) {
    const u32x2 u = gmem<u32x2>(p)[i];
    return make_float4(__half2float(__ushort_as_half((unsigned short)(u.x & 0xffffu))),
                       __half2float(__ushort_as_half((unsigned short)(u.x >> 16))),
                       __half2float(__ushort_as_half((unsigned short)(u.y & 0xffffu))),
                       __half2float(__ushort_as_half((unsigned short)(u.y >> 16))));
  }
};
template <> struct Vox4<DDVR_BF16> {
  static __device__ __forceinline__ float4 ld(const void* p, int64_t i) {
    const u32x2 u = gmem<u32x2>(p)[i];
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  }
};

// corner values v[ch][cx + 2cy + 4cz]; b = vertex index of corner 0
template <int DT>
__device__ __forceinline__ void fetch_color(const ViewDesc& vd, int64_t b, float (*v)[8]) {
  const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
  const int64_t off[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float4 x = Vox4<DT>::ld(vd.vol, b + off[k]);
    v[0][k] = x.x; v[1][k] = x.y; v[2][k] = x.z; v[3][k] = x.w;
  }
}

__device__ __forceinline__ int64_t cell_index(const ViewDesc& vd, const Cell& c) {
  return ((int64_t)c.k[2] * vd.ny + c.k[1]) * vd.nx + c.k[0];
}

// Start of the slab-synchronous route's inversion.  A ray whose T_N is at least 2^-100 is inverted
// from its last sample.  Any other ray is inverted from sample K-1, K one
// past the last sample entered with T^(i) >= 2^-100: the samples after it
// carry T^(i) < 2^-100, and with non-negative extinction their share of every
// gradient is below 2^-100 of the upstream gradient.  Sample K-1 is adjoined
// with P = T^(i+1) alpha_hat^(i+1) = g_alpha T_N - (C_N - C^(i+1)) . C_hat
// (no division by the possibly underflowed T^(K)); alpha_hat^(K-1) =
// P^(K-1) / T^(K-1) then starts the T-form inversion with T^(K-1) >= 2^-100.
// ---------------------------------------------------------------------------
struct ColorCut {
  int K;        // samples the adjoint covers
  float TK1;    // T^(K-1)
  float CK[3];  // C^(K)
  // factors of the fixed-point bound (see k_color_lds): max |w_i|,
  // sum |w_i| m_i, max T^(i+1), max m_i; w_i = alpha_i T^(i), m_i = max |rgb_i|
  float maxw, swm, tmax, mmax;
};

__device__ __forceinline__ void color_fwd_init(float* C, float& T, ColorCut& cut) {
  C[0] = C[1] = C[2] = 0.0f;
  T = 1.0f;
  cut.K = 0;
  cut.TK1 = 1.0f;
  cut.CK[0] = cut.CK[1] = cut.CK[2] = 0.0f;
  cut.maxw = cut.swm = cut.tmax = cut.mmax = 0.0f;
}

// One sample of the colour forward from its 8 corners' (r, g, b, tau).
template <bool TRACK>
__device__ __forceinline__ void color_fwd_sample(const ViewDesc& vd, float fi, const Cell& c,
                                                 const float (*v)[8], float* C, float& T,
                                                 ColorCut& cut) {
  float q[4];
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) q[ch] = trilerp(v[ch], c.f);
  const float e = __expf(-vd.step * q[3]);
  const float Ti = T;
  // explicitly rounded (no contraction): every route renders the same image
  const float w = __fmul_rn(T, __fsub_rn(1.0f, e));
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) C[ch] = fmaf(w, q[ch], C[ch]);
  T *= e;
  if (TRACK) {
    if (Ti >= kFallbackTmin) {
      cut.K = (int)fi + 1;
      cut.TK1 = Ti;
      cut.CK[0] = C[0]; cut.CK[1] = C[1]; cut.CK[2] = C[2];
    }
    const float m = fmaxf(fabsf(q[0]), fmaxf(fabsf(q[1]), fabsf(q[2])));
    const float aw = fabsf(w);
    cut.maxw = fmaxf(cut.maxw, aw);
    cut.swm = fmaf(aw, m, cut.swm);
    cut.tmax = fmaxf(cut.tmax, T);
    cut.mmax = fmaxf(cut.mmax, m);
  }
}

// samples [a, b) of a ray with direct gathers
template <int DT, bool TRACK>
__device__ __forceinline__ void color_fwd_direct(const ViewDesc& vd, const RayG& r, int a, int b,
                                                 float* C, float& T, ColorCut& cut) {
  for (float fi = (float)a; fi < (float)b; fi += 1.0f) {
    Cell c;
    locate(r, fi, vd, c);
    float v[4][8];
    fetch_color<DT>(vd, cell_index(vd, c), v);
    color_fwd_sample<TRACK>(vd, fi, c, v, C, T, cut);
  }
}

template <int DT, bool TRACK>
__device__ __forceinline__ void color_march_fwd(const ViewDesc& vd, const RayG& r, int n,
                                                float* C, float& T, ColorCut& cut) {
  color_fwd_init(C, T, cut);
  color_fwd_direct<DT, TRACK>(vd, r, 0, n, C, T, cut);
}

// per-ray colour adjoint state
struct ColorAdj {
  float Chat[3];
  float ahat;       // inversion: alpha_hat^(i+1)
  float Tn;         // inversion: T^(i+1)
  float Cr[3], Tr;  // forward order: C^(i), T^(i)
  float CN[3];      // forward order: C_N
  float gaTN;       // forward order: g_alpha * T_N
  int64_t gkey;     // vertex index of the current cell's corner 0, -1: none
  float cg[4][8];   // gradient of the current cell's corners, per channel
};

__device__ __forceinline__ void color_flush(const ViewDesc& vd, ColorAdj& s) {
  if (s.gkey < 0) return;
  const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
  const int64_t off[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
  float* g = vd.dV + 4 * s.gkey;
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      gadd(g + 4 * off[k] + ch, s.cg[ch][k]);
      s.cg[ch][k] = 0.0f;
    }
  s.gkey = -1;
}

template <int DT, int PASS, bool XH>
__global__ __launch_bounds__(256) void k_color(const LaunchParams p) {
  constexpr int NT = 256, TW = 16, TH = 16;
  __shared__ float fscratch[64];
  const ViewDesc& vd = p.one;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % vd.tiles_x, ty = tile / vd.tiles_x;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int lx, ly;
  tile_pixel<4>(false, wid, lane, lx, ly);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool valid = px < vd.W && py < vd.H;
  const int64_t pix = (int64_t)py * vd.W + px;
  RayG r;
  setup_ray(vd, px, py, valid, r);
  const int N = r.N;

  float CN[3] = {0.0f, 0.0f, 0.0f}, TN = 1.0f;
  float gimg[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (PASS != PASS_ADJ) {
    // forward (Alg. 1 with per-channel interpolation in place of the TF)
    ColorCut cut;
    color_march_fwd<DT, false>(vd, r, N, CN, TN, cut);
    if (valid) {
      reinterpret_cast<float4*>(vd.image)[pix] = make_float4(CN[0], CN[1], CN[2], 1.0f - TN);
      if (vd.trans) vd.trans[pix] = TN;
    }
    if (PASS == PASS_FWD) return;
    float loss = 0.0f;
    if (valid) {
      const float out[4] = {CN[0], CN[1], CN[2], 1.0f - TN};
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const float dlt = out[ch] - vd.target[pix * 4 + ch];
        gimg[ch] = loss_seed((p.flags & DDVR_LOSS_L1) != 0, p.loss_scale, dlt, loss);
      }
    }
    if (p.loss_out) {
      float l = loss * p.loss_scale;
      wg_sum_n<NT>(&l, 1, fscratch);
      if (threadIdx.x == 0 && l != 0.0f) atomicAdd(p.loss_out, (double)l);
    }
  } else if (valid) {
    const float4 im = reinterpret_cast<const float4*>(vd.image)[pix];
    CN[0] = im.x; CN[1] = im.y; CN[2] = im.z;
    TN = vd.trans[pix];
    const float4 g = reinterpret_cast<const float4*>(vd.d_image)[pix];
    gimg[0] = g.x; gimg[1] = g.y; gimg[2] = g.z; gimg[3] = g.w;
  }

  // adjoint (Alg. 2)
  int gmask = p.grad_mask;
  if (!vd.dV) gmask &= ~GRAD_V;
  if (!vd.dcam) gmask &= ~GRAD_CAM;
  if (!vd.dstep) gmask &= ~GRAD_STEP;
  const bool need_xhat = XH && (gmask & (GRAD_CAM | GRAD_STEP)) != 0;
  const int mode = p.flags & DDVR_ADJ_MODE_MASK;
  const bool fwd_order =
      mode == DDVR_ADJ_RESIDUAL || (mode == DDVR_ADJ_AUTO && !(TN >= kFallbackTmin));
  ColorAdj s;
  s.Chat[0] = gimg[0]; s.Chat[1] = gimg[1]; s.Chat[2] = gimg[2];
  s.ahat = gimg[3];
  s.Tn = TN;
  s.Cr[0] = s.Cr[1] = s.Cr[2] = 0.0f;
  s.Tr = 1.0f;
  s.CN[0] = CN[0]; s.CN[1] = CN[1]; s.CN[2] = CN[2];
  s.gaTN = gimg[3] * TN;
  s.gkey = -1;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
#pragma unroll
    for (int k = 0; k < 8; ++k) s.cg[ch][k] = 0.0f;
  AdjState x;   // camera / step ray sums
  x.xo_hat[0] = x.xo_hat[1] = x.xo_hat[2] = 0.0;
  x.si[0] = x.si[1] = x.si[2] = 0.0;
  x.dstep = 0.0;

  const float lastf = (float)(N - 1);
  for (float kf = 0.0f; kf < (float)N; kf += 1.0f) {
    const float fi = fwd_order ? kf : lastf - kf;
    Cell c;
    locate(r, fi, vd, c);
    const int64_t key = cell_index(vd, c);
    float v[4][8];
    fetch_color<DT>(vd, key, v);
    float q[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) q[ch] = trilerp(v[ch], c.f);
    const float e = __expf(-vd.step * q[3]);
    const float alpha = 1.0f - e;
    const float rc = q[0] * s.Chat[0] + q[1] * s.Chat[1] + q[2] * s.Chat[2];
    float Ti, ase;   // T^(i), and alpha_hat_i * e_i = T^(i+1) (alpha_hat^(i+1) + rgb . C_hat)
    if (fwd_order) {
      Ti = s.Tr;
      const float w = __fmul_rn(Ti, __fsub_rn(1.0f, e));
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) s.Cr[ch] = fmaf(w, q[ch], s.Cr[ch]);
      s.Tr = Ti * e;
      const float res = s.gaTN - ((s.CN[0] - s.Cr[0]) * s.Chat[0] +
                                  (s.CN[1] - s.Cr[1]) * s.Chat[1] +
                                  (s.CN[2] - s.Cr[2]) * s.Chat[2]);
      ase = fmaf(s.Tr, rc, res);
    } else {
      Ti = s.Tn * __builtin_amdgcn_rcpf(e);
      ase = s.Tn * (s.ahat + rc);
      s.ahat = fmaf(e, s.ahat, -alpha * rc);
      s.Tn = Ti;
    }
    const float wgt = alpha * Ti;
    const float g4[4] = {wgt * s.Chat[0], wgt * s.Chat[1], wgt * s.Chat[2], ase * vd.step};
    if (XH) x.dstep += (double)(ase * q[3]);
    if (gmask & GRAD_V) {
      if (key != s.gkey) {
        color_flush(vd, s);
        s.gkey = key;
      }
      float w8[8];
      trilerp_weights(c.f, w8);
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
#pragma unroll
        for (int k = 0; k < 8; ++k) s.cg[ch][k] = fmaf(w8[k], g4[ch], s.cg[ch][k]);
    }
    if (need_xhat) {
      float gp[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        float gd[3];
        trilerp_grad(v[ch], c.f, gd);
#pragma unroll
        for (int a = 0; a < 3; ++a) gp[a] = fmaf(g4[ch], gd[a], gp[a]);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float xh = gp[a] * vd.inv_h;
        x.xo_hat[a] += (double)xh;
        x.si[a] += (double)fi * (double)xh;
      }
    }
  }
  if (gmask & GRAD_V) color_flush(vd, s);
  if (XH && (gmask & (GRAD_CAM | GRAD_STEP))) {
    float cg[13];
    camera_adjoint(vd, r, x, N > 0, cg);
    wg_sum_n<NT>(cg, 13, fscratch);
    if (threadIdx.x == 0) {
      if (gmask & GRAD_CAM)
        for (int k = 0; k < 12; ++k)
          if (cg[k] != 0.0f) gadd(vd.dcam + k, cg[k]);
      if ((gmask & GRAD_STEP) && cg[12] != 0.0f) gadd(vd.dstep, cg[12]);
    }
  }
}

// ---------------------------------------------------------------------------
// colour volume, slab-synchronous route: the tile's adjoint marches slab by
// slab back to front (as the scalar kernel does) and accumulates the
// 4-channel gradient of each slab's brick of vertices in LDS, flushed with
// one global atomic per touched vertex and channel.  The grid values are
// gathered directly (the forward's 8 corner loads per sample, from L2).
// ---------------------------------------------------------------------------
// per-ray state of the slab-synchronous colour adjoint
struct ColorAdjL {
  float Chat[3];
  float ahat;       // alpha_hat^(i+1)
  float Tn;         // T^(i+1)
  float P;          // first sample of a cut ray: T^(K) alpha_hat^(K)
  float fK1;        // index of that sample (-1: the ray is not cut)
  float TK1;        // T^(K-1)
  int ckey;         // LDS byte offset of the current cell's corner 0 (-1: none)
  int64_t gkey;     // vertex index of the current cell's corner 0 (direct slabs)
  // gradient of the current cell's corners: the colour channels' gradients
  // of a sample are one scalar alpha_i T^(i) times the ray's C_hat, so the
  // cell keeps sum w_c alpha_i T^(i) (ca) and the extinction part (ct) and
  // multiplies by C_hat (cq: C_hat times the channel's fixed-point scale) on
  // exit
  float ca[8], ct[8];
  float cq[3];
};

// Add the registered cell gradient to the LDS brick ([vertex][4] floats) or
// to global memory, then clear it.
// FIX: the brick holds 32-bit fixed point, channel ch scaled by qs[ch] (LDS
// integer atomics run at the rate of plain stores, float ones serialise).
template <bool LDS, bool FIX>
__device__ __forceinline__ void color_cell_flush(const ViewDesc& vd, const Brick& br, float* acc,
                                                 ColorAdjL& s, const float* qs) {
  if (LDS) {
    if (s.ckey < 0) return;
    char* p0 = reinterpret_cast<char*>(acc) + s.ckey;
    const int sy = 4 * br.bx4, sz = 4 * br.bxy4;
    const int off[8] = {0, 16, sy, sy + 16, sz, sz + 16, sz + sy, sz + sy + 16};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        if (FIX)
          atomicAdd(reinterpret_cast<int*>(p0 + off[k]) + ch, round_i32(s.ca[k] * s.cq[ch]));
        else
          atomicAdd(reinterpret_cast<float*>(p0 + off[k]) + ch, s.ca[k] * s.cq[ch]);
      }
      if (FIX)
        atomicAdd(reinterpret_cast<int*>(p0 + off[k]) + 3, round_i32(s.ct[k] * qs[3]));
      else
        atomicAdd(reinterpret_cast<float*>(p0 + off[k]) + 3, s.ct[k]);
      s.ca[k] = 0.0f;
      s.ct[k] = 0.0f;
    }
    s.ckey = -1;
  } else {
    if (s.gkey < 0) return;
    const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
    const int64_t off[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
    float* g = vd.dV + 4 * s.gkey;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) gadd(g + 4 * off[k] + ch, s.ca[k] * s.Chat[ch]);
      gadd(g + 4 * off[k] + 3, s.ct[k]);
      s.ca[k] = 0.0f;
      s.ct[k] = 0.0f;
    }
    s.gkey = -1;
  }
}

template <int DT, bool LDS, bool FIX, bool XH>
__device__ __forceinline__ void color_adj_sample(const ViewDesc& vd, const RayG& r, float fi,
                                                 float* acc, const Brick& br, int gmask,
                                                 bool need_xhat, ColorAdjL& s, AdjState& x,
                                                 const float* qs) {
  Cell c;
  locate(r, fi, vd, c);
  const int64_t vidx = cell_index(vd, c);
  float v[4][8];
  fetch_color<DT>(vd, vidx, v);
  float q[4];
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) q[ch] = trilerp(v[ch], c.f);
  const float e = __expf(-vd.step * q[3]);
  const float alpha = 1.0f - e;
  const float rc = q[0] * s.Chat[0] + q[1] * s.Chat[1] + q[2] * s.Chat[2];
  float Ti, ase;   // T^(i), and e_i times the adjoint of alpha_i
  if (fi == s.fK1) {
    Ti = s.TK1;
    ase = fmaf(s.TK1 * e, rc, s.P);
    s.ahat = (s.P - alpha * Ti * rc) / Ti;
  } else {
    Ti = s.Tn * __builtin_amdgcn_rcpf(e);
    ase = s.Tn * (s.ahat + rc);
    s.ahat = fmaf(e, s.ahat, -alpha * rc);
  }
  s.Tn = Ti;
  const float wgt = alpha * Ti;
  const float g4[4] = {wgt * s.Chat[0], wgt * s.Chat[1], wgt * s.Chat[2], ase * vd.step};
  if (XH) x.dstep += (double)(ase * q[3]);
  if (gmask & GRAD_V) {
    if (LDS) {
      const int key = 4 * brick_base(br, c);
      if (key != s.ckey) {
        color_cell_flush<true, FIX>(vd, br, acc, s, qs);
        s.ckey = key;
      }
    } else if (vidx != s.gkey) {
      color_cell_flush<false, false>(vd, br, acc, s, qs);
      s.gkey = vidx;
    }
    // trilinear weights with the two sample factors folded into the x terms
    const float gy = 1.0f - c.f[1], gz = 1.0f - c.f[2];
    const float a00 = gy * gz, a10 = c.f[1] * gz, a01 = gy * c.f[2], a11 = c.f[1] * c.f[2];
    const float w0 = (1.0f - c.f[0]) * wgt, w1 = c.f[0] * wgt;
    const float t0 = (1.0f - c.f[0]) * g4[3], t1 = c.f[0] * g4[3];
    s.ca[0] = fmaf(w0, a00, s.ca[0]); s.ca[1] = fmaf(w1, a00, s.ca[1]);
    s.ca[2] = fmaf(w0, a10, s.ca[2]); s.ca[3] = fmaf(w1, a10, s.ca[3]);
    s.ca[4] = fmaf(w0, a01, s.ca[4]); s.ca[5] = fmaf(w1, a01, s.ca[5]);
    s.ca[6] = fmaf(w0, a11, s.ca[6]); s.ca[7] = fmaf(w1, a11, s.ca[7]);
    s.ct[0] = fmaf(t0, a00, s.ct[0]); s.ct[1] = fmaf(t1, a00, s.ct[1]);
    s.ct[2] = fmaf(t0, a10, s.ct[2]); s.ct[3] = fmaf(t1, a10, s.ct[3]);
    s.ct[4] = fmaf(t0, a01, s.ct[4]); s.ct[5] = fmaf(t1, a01, s.ct[5]);
    s.ct[6] = fmaf(t0, a11, s.ct[6]); s.ct[7] = fmaf(t1, a11, s.ct[7]);
  }
  if (need_xhat) {
    float gp[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      float gd[3];
      trilerp_grad(v[ch], c.f, gd);
#pragma unroll
      for (int a = 0; a < 3; ++a) gp[a] = fmaf(g4[ch], gd[a], gp[a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float xh = gp[a] * vd.inv_h;
      x.xo_hat[a] += (double)xh;
      x.si[a] += (double)fi * (double)xh;
    }
  }
}

// Zero the brick's 4-channel accumulator / add it to the gradient in global
// memory (one atomic per touched vertex and channel).  The flush gives each
// lane one (vertex, channel) entry of the [vertex][4] brick, so a wave's
// atomic instruction covers 16 consecutive vertices, 256 contiguous bytes of
// the gradient where the brick row allows: four full 64-byte requests instead
// of sixteen quarter-filled ones per channel (device-scope float atomics are
// carried out past the per-XCD L2, one request per touched 64-byte segment).
template <int NT>
__device__ __forceinline__ void color_brick_zero(const Brick& br, float* acc) {
  float4* a4 = reinterpret_cast<float4*>(acc);
  for (int idx = threadIdx.x; idx < br.size; idx += NT) a4[idx] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int NT, bool FIX>
__device__ __forceinline__ void color_brick_flush(const ViewDesc& vd, const Brick& br,
                                                  const float* acc, const float* inv_qs) {
  const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
  float* const org = vd.dV + 4 * (br.z0 * sz + br.y0 * sy + br.x0);
  const bool narrow = brick_narrow(br, sz);
  const int n = 4 * br.size;
  // NT is a multiple of 4, so a lane keeps its channel for the whole loop
  static_assert(NT % 4 == 0, "lanes keep their channel");
  const int ch = threadIdx.x & 3;
  const float iq = ch == 0 ? inv_qs[0] : ch == 1 ? inv_qs[1] : ch == 2 ? inv_qs[2] : inv_qs[3];
  for (int e = threadIdx.x; e < n; e += NT) {
    const float g = FIX ? (float)reinterpret_cast<const int*>(acc)[e] * iq : acc[e];
    if (g == 0.0f) continue;
    const int idx = e >> 2;
    gadd(org + 4 * (narrow ? brick_goff<true>(br, idx, sy, sz)
                           : brick_goff<false>(br, idx, sy, sz)) + ch, g);
  }
}

// Stage the brick's (r, g, b, tau) as float4 per vertex, 4 loads in flight
// per lane.
template <int NT, int DT>
__device__ __forceinline__ void stage_color(const ViewDesc& vd, const Brick& br, float* stage) {
  const int64_t sy = vd.nx, sz = (int64_t)vd.nx * vd.ny;
  const int64_t org = br.z0 * sz + br.y0 * sy + br.x0;
  const bool narrow = brick_narrow(br, sz);
  float4* s4 = reinterpret_cast<float4*>(stage);
  constexpr int U = 4;
  for (int i0 = threadIdx.x; i0 < br.size; i0 += U * NT) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = min(i0 + u * NT, br.size - 1);
      v[u] = Vox4<DT>::ld(vd.vol, org + (narrow ? brick_goff<true>(br, idx, sy, sz)
                                                : brick_goff<false>(br, idx, sy, sz)));
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * NT < br.size) s4[i0 + u * NT] = v[u];
  }
}

// samples [a, b) of a ray from the staged brick
template <bool TRACK>
__device__ __forceinline__ void color_fwd_lds(const ViewDesc& vd, const RayG& r, int a, int b,
                                              const float* stage, const Brick& br, float* C,
                                              float& T, ColorCut& cut) {
  const int sy = 4 * br.bx4, sz = 4 * br.bxy4;
  for (float fi = (float)a; fi < (float)b; fi += 1.0f) {
    Cell c;
    locate(r, fi, vd, c);
    const char* p0 = reinterpret_cast<const char*>(stage) + 4 * brick_base(br, c);
    const int off[8] = {0, 16, sy, sy + 16, sz, sz + 16, sz + sy, sz + sy + 16};
    float v[4][8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float4 x = *reinterpret_cast<const float4*>(p0 + off[k]);
      v[0][k] = x.x; v[1][k] = x.y; v[2][k] = x.z; v[3][k] = x.w;
    }
    color_fwd_sample<TRACK>(vd, fi, c, v, C, T, cut);
  }
}

// The tile's colour forward, front to back over axis slabs: every slab whose
// brick fits `vcap` vertices is staged in LDS, the others gathered directly.
template <int DT, bool TRACK>
__device__ __forceinline__ void color_fwd_slabs(const ViewDesc& vd, const RayG& r, int tx,
                                                int ty, int n, float* stage, int* iscratch,
                                                int vcap, float* C, float& T, ColorCut& cut) {
  constexpr int NT = 256;
  color_fwd_init(C, T, cut);
  float t0, dta;
  tile_axis(vd, tx, ty, 16, 16, r, t0, dta);
  int tlo, thi;
  if (!axis_range<NT>(t0, dta, n, iscratch, tlo, thi)) {
    color_fwd_direct<DT, TRACK>(vd, r, 0, n, C, T, cut);
    return;
  }
  float dz = 4.0f;
  for (float tl = (float)tlo; tl < (float)thi;) {
    int st, a = 0, b = 0;
    float th;
    Brick br;
    for (;;) {
      th = fminf(tl + dz, (float)thi);
      a = axis_index(tl, t0, dta, n);
      b = axis_index(th, t0, dta, n);
      if (n <= 0) a = b = 0;
      if (!range_brick<NT>(vd, r, a, b, iscratch, br)) { st = 0; dz = fminf(2.0f * dz, 64.0f); break; }
      if (vcap > 0 && br.size <= vcap) {
        if (4 * br.size < vcap) dz = fminf(2.0f * dz, 64.0f);
        st = 1;
        break;
      }
      if (vcap <= 0 || dz <= 0.25f) { st = 2; break; }
      dz *= 0.5f;
    }
    tl = th;
    if (st == 1) {
      // the previous slab's reads finished before range_brick's barriers
      stage_color<NT, DT>(vd, br, stage);
      __syncthreads();
      color_fwd_lds<TRACK>(vd, r, a, b, stage, br, C, T, cut);
    } else if (st == 2) {
      color_fwd_direct<DT, TRACK>(vd, r, a, b, C, T, cut);
    }
  }
}

// The back-to-front slab march of a tile's colour adjoint.
template <int DT, bool FIX, bool XH>
__device__ __forceinline__ void color_adjoint_slabs(const ViewDesc& vd, const RayG& r, int tx,
                                                    int ty, int Nadj, float* acc, int* iscratch,
                                                    int vcap, int gmask,
                                                    bool need_xhat, bool want_dv, ColorAdjL& s,
                                                    AdjState& x, const float* qs,
                                                    const float* inv_qs) {
  constexpr int NT = 256, TW = 16, TH = 16;
  // axis slabs (tile_axis), back to front
  float t0, dt_ax;
  tile_axis(vd, tx, ty, TW, TH, r, t0, dt_ax);
  int tlo, thi;
  if (!axis_range<NT>(t0, dt_ax, Nadj, iscratch, tlo, thi)) {
    // some ray does not advance along the axis: the tile runs its rays whole
    // on the direct path
    const Brick none{};
    for (float fi = (float)(Nadj - 1); fi >= 0.0f; fi -= 1.0f)
      color_adj_sample<DT, false, false, XH>(vd, r, fi, acc, none, gmask, need_xhat, s, x, qs);
    if (want_dv) color_cell_flush<false, false>(vd, none, acc, s, qs);
    tlo = thi = 0;
  }
  const int acap = want_dv ? vcap : 0;
  float dz = 4.0f;
  for (float th = (float)thi; th > (float)tlo;) {
    int st, a = 0, b = 0;
    float tl;
    Brick br;
    for (;;) {
      tl = fmaxf(th - dz, (float)tlo);
      a = axis_index(tl, t0, dt_ax, Nadj);
      b = axis_index(th, t0, dt_ax, Nadj);
      if (Nadj <= 0) a = b = 0;
      if (!range_brick<NT>(vd, r, a, b, iscratch, br)) { st = 0; dz = fminf(2.0f * dz, 64.0f); break; }
      if (acap > 0 && br.size <= acap) {
        if (4 * br.size < acap) dz = fminf(2.0f * dz, 64.0f);
        st = 1;
        break;
      }
      if (acap <= 0 || dz <= 0.25f) { st = 2; break; }
      dz *= 0.5f;
    }
    th = tl;
    if (st == 0) continue;
    const float fa = (float)a;
    if (st == 1) {
      color_brick_zero<NT>(br, acc);
      __syncthreads();
      for (float fi = (float)(b - 1); fi >= fa; fi -= 1.0f)
        color_adj_sample<DT, true, FIX, XH>(vd, r, fi, acc, br, gmask, need_xhat, s, x, qs);
      if (want_dv) color_cell_flush<true, FIX>(vd, br, acc, s, qs);
      __syncthreads();
      color_brick_flush<NT, FIX>(vd, br, acc, inv_qs);
    } else {
      for (float fi = (float)(b - 1); fi >= fa; fi -= 1.0f)
        color_adj_sample<DT, false, false, XH>(vd, r, fi, acc, br, gmask, need_xhat, s, x, qs);
      if (want_dv) color_cell_flush<false, false>(vd, br, acc, s, qs);
    }
  }
}

template <int DT, int PASS, bool XH>
__device__ __forceinline__ void color_lds_tile(const LaunchParams& p, float* smem) {
  constexpr int NT = 256, TW = 16, TH = 16;
  // one (view, tile) item per workgroup: a single view's tiles, or a batch's
  // work list of (view << 20 | tile)
  const int item = xcd_remap(blockIdx.x, gridDim.x);
  int view = 0, tile = item;
  if (p.work) {
    const int w = p.work[item];
    view = w >> 20;
    tile = w & 0xFFFFF;
  }
  const ViewDesc vd = p.views ? p.views[view] : p.one;
  const int vcap = p.lds_cap;          // vertices per brick (4 floats each)
  float* acc = smem;
  int* iscratch = reinterpret_cast<int*>(smem + 4 * vcap);
  float* fscratch = reinterpret_cast<float*>(iscratch);
  const int tx = tile % vd.tiles_x, ty = tile / vd.tiles_x;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int lx, ly;
  tile_pixel<4>(false, wid, lane, lx, ly);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool valid = px < vd.W && py < vd.H;
  const int64_t pix = (int64_t)py * vd.W + px;
  RayG r;
  setup_ray(vd, px, py, valid, r);
  const int N = r.N;
  const bool hit = N > 0;
  const int mode = p.flags & DDVR_ADJ_MODE_MASK;

  float CN[3] = {0.0f, 0.0f, 0.0f}, TN = 1.0f;
  float gimg[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  // The forward runs in every pass: the adjoint pass re-marches it for the
  // start of each ray's inversion and the bound of the fixed-point brick
  // (reproducing the image and T_N the forward pass wrote, bit for bit).
  ColorCut cut;
  color_fwd_slabs<DT, PASS != PASS_FWD>(vd, r, tx, ty, N, acc, iscratch, vcap, CN, TN, cut);
  if (PASS != PASS_ADJ) {
    if (valid) {
      reinterpret_cast<float4*>(vd.image)[pix] = make_float4(CN[0], CN[1], CN[2], 1.0f - TN);
      if (vd.trans) vd.trans[pix] = TN;
    }
    if (PASS == PASS_FWD) return;
    float loss = 0.0f;
    if (valid) {
      const float out[4] = {CN[0], CN[1], CN[2], 1.0f - TN};
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const float dlt = out[ch] - vd.target[pix * 4 + ch];
        gimg[ch] = loss_seed((p.flags & DDVR_LOSS_L1) != 0, p.loss_scale, dlt, loss);
      }
    }
    if (p.loss_out) {
      float l = loss * p.loss_scale;
      wg_sum_n<NT>(&l, 1, fscratch);
      if (threadIdx.x == 0 && l != 0.0f) atomicAdd(p.loss_out, (double)l);
    }
  } else if (valid) {
    const float4 g = reinterpret_cast<const float4*>(vd.d_image)[pix];
    gimg[0] = g.x; gimg[1] = g.y; gimg[2] = g.z; gimg[3] = g.w;
  }
  const bool seeded = gimg[0] != 0.0f || gimg[1] != 0.0f || gimg[2] != 0.0f || gimg[3] != 0.0f;
  // where the inversion starts (INVERT_T: always at the last sample)
  const bool cutting = hit && seeded && mode == DDVR_ADJ_AUTO && !(TN >= kFallbackTmin);
  if (!cutting) cut.K = N;

  int gmask = p.grad_mask;
  if (!vd.dV) gmask &= ~GRAD_V;
  if (!vd.dcam) gmask &= ~GRAD_CAM;
  if (!vd.dstep) gmask &= ~GRAD_STEP;
  const bool need_xhat = XH && (gmask & (GRAD_CAM | GRAD_STEP)) != 0;
  const bool want_dv = (gmask & GRAD_V) != 0;
  const int Nadj = seeded ? cut.K : 0;

  ColorAdjL s;
  s.Chat[0] = gimg[0]; s.Chat[1] = gimg[1]; s.Chat[2] = gimg[2];
  s.ahat = gimg[3];
  s.Tn = TN;
  s.fK1 = -1.0f;
  s.TK1 = cut.TK1;
  s.P = 0.0f;
  if (cutting && Nadj > 0) {
    s.fK1 = (float)(Nadj - 1);
    s.P = gimg[3] * TN - ((CN[0] - cut.CK[0]) * gimg[0] + (CN[1] - cut.CK[1]) * gimg[1] +
                          (CN[2] - cut.CK[2]) * gimg[2]);
  }
  s.ckey = -1;
  s.gkey = -1;
#pragma unroll
  for (int k = 0; k < 8; ++k) s.ca[k] = s.ct[k] = 0.0f;
  AdjState x;
  x.xo_hat[0] = x.xo_hat[1] = x.xo_hat[2] = 0.0;
  x.si[0] = x.si[1] = x.si[2] = 0.0;
  x.dstep = 0.0;

  // Fixed-point scales of the brick, one per channel.  A vertex takes at
  // most lmax samples of a straight ray (its 2x2x2 cells: chord <= 2 sqrt 3
  // voxels), each adding a trilinear weight <= 1 times the sample's gradient:
  //  * colour channel c: alpha_i T^(i) C_hat_c, at most maxw |C_hat_c|;
  //  * extinction: dt times e_i alpha_hat_i = P^(i+1) + T^(i+1) rgb_i . C_hat
  //    with P^(i+1) = T^(i+1) alpha_hat^(i+1) = g_alpha T_N - sum_(j>i) w_j
  //    rgb_j . C_hat, at most |g_alpha| T_N + |C_hat|_1 (sum |w_j| m_j +
  //    max T * max m).
  // B_c sums these per-ray bounds over the tile; qs_c = 2^(28 - ceil(log2
  // B_c)) keeps every partial sum below 2^28 (margin for the float32 drift of
  // the recovered T^(i)).  A tile with a non-finite or subnormal-scale bound
  // accumulates float32 instead.
  float qs[4] = {1.0f, 1.0f, 1.0f, 1.0f}, inv_qs[4] = {1.0f, 1.0f, 1.0f, 1.0f};
  bool fix_ok = true;
  {
    float b4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (want_dv && Nadj > 0) {
      const float lmax = floorf(3.4641017f / (vd.step * vd.inv_h)) + 2.0f;
      const float c1 = fabsf(gimg[0]) + fabsf(gimg[1]) + fabsf(gimg[2]);
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) b4[ch] = lmax * fabsf(gimg[ch]) * cut.maxw;
      b4[3] = lmax * vd.step *
              (fabsf(gimg[3]) * TN + c1 * (cut.swm + cut.tmax * cut.mmax));
    }
    wg_sum_n<NT>(b4, 4, fscratch);
    __syncthreads();
    if (threadIdx.x == 0)
      for (int ch = 0; ch < 4; ++ch) fscratch[ch] = b4[ch];
    __syncthreads();
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const float B = fscratch[ch] * 1.0001f;   // margin for the float32 sums
      if (!(B < INFINITY)) {
        fix_ok = false;
      } else if (B > 0.0f) {
        int ex;
        (void)frexpf(B, &ex);          // B < 2^ex
        const int e = 28 - ex;
        if (e > 120) fix_ok = false;
        else {
          qs[ch] = ldexpf(1.0f, max(e, -120));
          inv_qs[ch] = ldexpf(1.0f, -max(e, -120));
        }
      }
    }
  }
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) s.cq[ch] = s.Chat[ch] * (fix_ok ? qs[ch] : 1.0f);
  if (fix_ok)
    color_adjoint_slabs<DT, true, XH>(vd, r, tx, ty, Nadj, acc, iscratch, vcap,
                                      gmask, need_xhat, want_dv, s, x, qs, inv_qs);
  else
    color_adjoint_slabs<DT, false, XH>(vd, r, tx, ty, Nadj, acc, iscratch, vcap,
                                       gmask, need_xhat, want_dv, s, x, qs, inv_qs);
  if (XH && (gmask & (GRAD_CAM | GRAD_STEP))) {
    float cg[13];
    camera_adjoint(vd, r, x, Nadj > 0, cg);
    wg_sum_n<NT>(cg, 13, fscratch);
    if (threadIdx.x == 0) {
      if (gmask & GRAD_CAM)
        for (int k = 0; k < 12; ++k)
          if (cg[k] != 0.0f) gadd(vd.dcam + k, cg[k]);
      if ((gmask & GRAD_STEP) && cg[12] != 0.0f) gadd(vd.dstep, cg[12]);
    }
  }
}

// The slab-synchronous colour kernel (one 16x16 tile per workgroup).
template <int DT, int PASS, bool XH>
__global__ __launch_bounds__(256) void k_color_lds(const LaunchParams p) {
  extern __shared__ __align__(16) float smem[];
  color_lds_tile<DT, PASS, XH>(p, smem);
}

// Forward-mode derivatives of the colour volume (direct gathers, one 16x16
// tile per workgroup): every channel's interpolated value carries its
// derivative along the P directions, q_c' = grad(q_c) . q' (grid units), and
// the blend propagates them as for the emission-absorption model with the
// channels in place of the TF's output.  The primal is bit for bit the
// colour forward's.
template <int DT, int P>
__global__ __launch_bounds__(256) void k_tangent_color(const TangentParams p) {
  constexpr int NT = 256, TW = 16, TH = 16;
  __shared__ float fscratch[64];
  const ViewDesc& vd = p.one;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int tx = tile % vd.tiles_x, ty = tile / vd.tiles_x;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int lx, ly;
  tile_pixel<4>(false, wid, lane, lx, ly);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool valid = px < vd.W && py < vd.H;
  const int64_t pix = (int64_t)py * vd.W + px;
  RayG r;
  setup_ray(vd, px, py, valid, r);
  RayTan<P> t;
  setup_tangent<P>(vd, r, p.dir, t);
  float C[3] = {0.0f, 0.0f, 0.0f}, T = 1.0f;
  float Cd[P][3], Td[P];
#pragma unroll
  for (int k = 0; k < P; ++k) { Cd[k][0] = Cd[k][1] = Cd[k][2] = 0.0f; Td[k] = 0.0f; }
  for (float fi = 0.0f; fi < (float)r.N; fi += 1.0f) {
    Cell c;
    locate(r, fi, vd, c);
    float v[4][8];
    fetch_color<DT>(vd, cell_index(vd, c), v);
    float q[4], qd[P][4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      q[ch] = trilerp(v[ch], c.f);
      float g[3];
      trilerp_grad(v[ch], c.f, g);
#pragma unroll
      for (int k = 0; k < P; ++k) {
        float x = 0.0f;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) x = fmaf(g[ax], fmaf(fi, t.dq[k][ax], t.qo[k][ax]), x);
        qd[k][ch] = x;
      }
    }
    const float e = __expf(-vd.step * q[3]);
    const float alpha = __fsub_rn(1.0f, e);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      // c = alpha rgb: c' = alpha' rgb + alpha rgb'; C' += T' c + T c'; T' = T' e + T e'
      const float ed = -e * fmaf(p.dir[k][12], q[3], vd.step * qd[k][3]);
      const float ad = -ed;
      const float ta = Td[k] * alpha;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const float cd = fmaf(ad, q[ch], alpha * qd[k][ch]);
        Cd[k][ch] = fmaf(ta, q[ch], fmaf(T, cd, Cd[k][ch]));
      }
      Td[k] = fmaf(Td[k], e, T * ed);
    }
    // primal exactly as the colour forward (bitwise the same image)
    const float w = __fmul_rn(T, alpha);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) C[ch] = fmaf(w, q[ch], C[ch]);
    T *= e;
  }
  if (valid) {
    if (vd.image)
      reinterpret_cast<float4*>(vd.image)[pix] = make_float4(C[0], C[1], C[2], 1.0f - T);
    if (p.image_dot) {
      const int64_t plane = (int64_t)vd.W * vd.H * 4;
#pragma unroll
      for (int k = 0; k < P; ++k)
        reinterpret_cast<float4*>(p.image_dot + k * plane)[pix] =
            make_float4(Cd[k][0], Cd[k][1], Cd[k][2], -Td[k]);
    }
  }
  if (p.d_dir) {
    // forward-delayed: contract with the upstream gradient in the same pass
    float dk[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
      float x = 0.0f;
      if (valid) {
        const float4 g = reinterpret_cast<const float4*>(vd.d_image)[pix];
        x = fmaf(g.x, Cd[k][0], fmaf(g.y, Cd[k][1], fmaf(g.z, Cd[k][2], -g.w * Td[k])));
      }
      dk[k] = x;
    }
    wg_sum_n<NT>(dk, P, fscratch);
    if (threadIdx.x == 0)
      for (int k = 0; k < P; ++k)
        if (dk[k] != 0.0f) gadd(p.d_dir + k, dk[k]);
  }
}

// float32 master -> storage copy (round to nearest even), 4 values per lane
__global__ void k_cast(const float* __restrict__ src, void* __restrict__ dst, int dtype,
                       int64_t n) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (i0 >= n) return;
  if (i0 + 4 <= n && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
    const float4 v = *reinterpret_cast<const float4*>(src + i0);
    const float x[4] = {v.x, v.y, v.z, v.w};
    if (dtype == DDVR_F16) {
      __half* d = static_cast<__half*>(dst) + i0;
      for (int k = 0; k < 4; ++k) d[k] = __float2half_rn(x[k]);
    } else if (dtype == DDVR_BF16) {
      uint16_t* d = static_cast<uint16_t*>(dst) + i0;
      for (int k = 0; k < 4; ++k) {
        const uint32_t u = __float_as_uint(x[k]);
        const bool nan = (u & 0x7fffffffu) > 0x7f800000u;
        d[k] = nan ? (uint16_t)((u >> 16) | 0x40u)
                   : (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
      }
    } else {
      *reinterpret_cast<float4*>(static_cast<float*>(dst) + i0) = v;
    }
    return;
  }
  for (int64_t i = i0; i < n && i < i0 + 4; ++i) {
    const float x = src[i];
    if (dtype == DDVR_F16) {
      static_cast<__half*>(dst)[i] = __float2half_rn(x);
    } else if (dtype == DDVR_BF16) {
      const uint32_t u = __float_as_uint(x);
      const bool nan = (u & 0x7fffffffu) > 0x7f800000u;
      static_cast<uint16_t*>(dst)[i] = nan ? (uint16_t)((u >> 16) | 0x40u)
                                           : (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    } else {
      static_cast<float*>(dst)[i] = x;
    }
  }
}

int launch_cast(const float* src, void* dst, int dtype, int64_t n, void* stream) {
  if (n <= 0) return 0;
  const int64_t threads = (n + 3) / 4;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), src, dst, dtype, n);
  return (int)hipGetLastError();
}

__global__ void k_zero_i32(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
// Persistent launches size the grid to the workgroups that fit the device at
// once (occupancy x CUs), capped by the number of tiles.
template <typename K>
static int persistent_blocks(K kernel, int threads, size_t lds, int n_items) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
      per_cu <= 0 || cus <= 0)
    return n_items < 1024 ? n_items : 1024;
  const int64_t b = (int64_t)cus * per_cu;
  return (int)(b < n_items ? b : n_items);
}

template <int MODEL, int DT, int WAVES, int PASS, bool XH>
static hipError_t launch4(const LaunchParams& p, int n_blocks, size_t lds, hipStream_t s) {
  auto kernel = k_render<MODEL, DT, WAVES, PASS, XH>;
  if (DT == DT_DYN) n_blocks = persistent_blocks(kernel, WAVES * 64, lds, p.n_items);
  hipLaunchKernelGGL(kernel, dim3(n_blocks), dim3(WAVES * 64), lds, s, p);
  return hipGetLastError();
}

template <int MODEL, int DT, int WAVES>
static hipError_t launch3(const LaunchParams& p, int pass, int n_blocks, size_t lds,
                          hipStream_t s) {
  const bool xh = (p.grad_mask & (GRAD_CAM | GRAD_STEP)) != 0;
  switch (pass) {
    case PASS_FWD: return launch4<MODEL, DT, WAVES, PASS_FWD, false>(p, n_blocks, lds, s);
    case PASS_ADJ:
      return xh ? launch4<MODEL, DT, WAVES, PASS_ADJ, true>(p, n_blocks, lds, s)
                : launch4<MODEL, DT, WAVES, PASS_ADJ, false>(p, n_blocks, lds, s);
    default:
      return xh ? launch4<MODEL, DT, WAVES, PASS_FUSED, true>(p, n_blocks, lds, s)
                : launch4<MODEL, DT, WAVES, PASS_FUSED, false>(p, n_blocks, lds, s);
  }
}

template <int MODEL, int DT>
static hipError_t launch2(const LaunchParams& p, int pass, int waves, int n_blocks, size_t lds,
                          hipStream_t s) {
  switch (waves) {
    case 1: return launch3<MODEL, DT, 1>(p, pass, n_blocks, lds, s);
    case 2: return launch3<MODEL, DT, 2>(p, pass, n_blocks, lds, s);
    default: return launch3<MODEL, DT, 4>(p, pass, n_blocks, lds, s);
  }
}

template <int MODEL>
static hipError_t launch1(const LaunchParams& p, int pass, int dtype, int waves, int n_blocks,
                          size_t lds, hipStream_t s) {
  switch (dtype) {
    case DDVR_F16: return launch2<MODEL, DDVR_F16>(p, pass, waves, n_blocks, lds, s);
    case DDVR_BF16: return launch2<MODEL, DDVR_BF16>(p, pass, waves, n_blocks, lds, s);
    case DT_DYN: return launch2<MODEL, DT_DYN>(p, pass, waves, n_blocks, lds, s);
    default: return launch2<MODEL, DDVR_F32>(p, pass, waves, n_blocks, lds, s);
  }
}

int launch_render(const LaunchParams& p, int pass, int model, int dtype, int waves, int n_blocks,
                  size_t lds_bytes, void* stream) {
  if (n_blocks <= 0) return 0;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const hipError_t e = model == DDVR_EMISSION_ABSORPTION
      ? launch1<DDVR_EMISSION_ABSORPTION>(p, pass, dtype, waves, n_blocks, lds_bytes, s)
      : launch1<DDVR_ABSORPTION>(p, pass, dtype, waves, n_blocks, lds_bytes, s);
  return (int)e;
}

template <int MODEL, int DT>
static hipError_t launch_fb2(const LaunchParams& p, int fused, int blocks, hipStream_t s) {
  const size_t lds = ((p.fb_dtf ? (size_t)p.fb_tf_R * 4 : 0) + 4 * (size_t)kFallbackBrick) *
                     sizeof(float);
  if (fused) hipLaunchKernelGGL((k_fallback<MODEL, DT, 1>), dim3(blocks), dim3(256), lds, s, p);
  else hipLaunchKernelGGL((k_fallback<MODEL, DT, 0>), dim3(blocks), dim3(256), lds, s, p);
  return hipGetLastError();
}

template <int MODEL>
static hipError_t launch_fb1(const LaunchParams& p, int dtype, int fused, int blocks,
                             hipStream_t s) {
  switch (dtype) {
    case DDVR_F16: return launch_fb2<MODEL, DDVR_F16>(p, fused, blocks, s);
    case DDVR_BF16: return launch_fb2<MODEL, DDVR_BF16>(p, fused, blocks, s);
    case DT_DYN: return launch_fb2<MODEL, DT_DYN>(p, fused, blocks, s);
    default: return launch_fb2<MODEL, DDVR_F32>(p, fused, blocks, s);
  }
}

template <int MODEL, int DT>
static hipError_t launch_tan2(const TangentParams& p, int n_blocks, size_t lds, hipStream_t s) {
  switch (p.ndir) {
    case 1: hipLaunchKernelGGL((k_tangent<MODEL, DT, 1>), dim3(n_blocks), dim3(256), lds, s, p); break;
    case 2: hipLaunchKernelGGL((k_tangent<MODEL, DT, 2>), dim3(n_blocks), dim3(256), lds, s, p); break;
    case 3: hipLaunchKernelGGL((k_tangent<MODEL, DT, 3>), dim3(n_blocks), dim3(256), lds, s, p); break;
    default: hipLaunchKernelGGL((k_tangent<MODEL, DT, 4>), dim3(n_blocks), dim3(256), lds, s, p); break;
  }
  return hipGetLastError();
}

template <int MODEL>
static hipError_t launch_tan1(const TangentParams& p, int dtype, int n_blocks, size_t lds,
                              hipStream_t s) {
  switch (dtype) {
    case DDVR_F16: return launch_tan2<MODEL, DDVR_F16>(p, n_blocks, lds, s);
    case DDVR_BF16: return launch_tan2<MODEL, DDVR_BF16>(p, n_blocks, lds, s);
    default: return launch_tan2<MODEL, DDVR_F32>(p, n_blocks, lds, s);
  }
}

template <int DT>
static hipError_t launch_tan_color(const TangentParams& p, int n_blocks, hipStream_t s) {
  switch (p.ndir) {
    case 1: hipLaunchKernelGGL((k_tangent_color<DT, 1>), dim3(n_blocks), dim3(256), 0, s, p); break;
    case 2: hipLaunchKernelGGL((k_tangent_color<DT, 2>), dim3(n_blocks), dim3(256), 0, s, p); break;
    case 3: hipLaunchKernelGGL((k_tangent_color<DT, 3>), dim3(n_blocks), dim3(256), 0, s, p); break;
    default: hipLaunchKernelGGL((k_tangent_color<DT, 4>), dim3(n_blocks), dim3(256), 0, s, p); break;
  }
  return hipGetLastError();
}

int launch_tangent(const TangentParams& p, int model, int dtype, int n_blocks, size_t lds_bytes,
                   void* stream) {
  const hipStream_t s = static_cast<hipStream_t>(stream);
  if (model == DDVR_COLOR) {
    switch (dtype) {
      case DDVR_F16: return (int)launch_tan_color<DDVR_F16>(p, n_blocks, s);
      case DDVR_BF16: return (int)launch_tan_color<DDVR_BF16>(p, n_blocks, s);
      default: return (int)launch_tan_color<DDVR_F32>(p, n_blocks, s);
    }
  }
  return (int)(model == DDVR_EMISSION_ABSORPTION
                   ? launch_tan1<DDVR_EMISSION_ABSORPTION>(p, dtype, n_blocks, lds_bytes, s)
                   : launch_tan1<DDVR_ABSORPTION>(p, dtype, n_blocks, lds_bytes, s));
}

int launch_fallback(const LaunchParams& p, int model, int dtype, int fused, void* stream) {
  if (p.fb_slots <= 0) return 0;
  const int blocks = (p.fb_slots + 255) / 256;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const hipError_t e = model == DDVR_EMISSION_ABSORPTION
      ? launch_fb1<DDVR_EMISSION_ABSORPTION>(p, dtype, fused, blocks, s)
      : launch_fb1<DDVR_ABSORPTION>(p, dtype, fused, blocks, s);
  return (int)e;
}

template <int DT>
static hipError_t launch_color2(const LaunchParams& p, int pass, bool xh, int blocks,
                                hipStream_t s) {
  const dim3 g(blocks), b(256);
  if (pass == PASS_FWD) hipLaunchKernelGGL((k_color<DT, PASS_FWD, false>), g, b, 0, s, p);
  else if (pass == PASS_ADJ && xh) hipLaunchKernelGGL((k_color<DT, PASS_ADJ, true>), g, b, 0, s, p);
  else if (pass == PASS_ADJ) hipLaunchKernelGGL((k_color<DT, PASS_ADJ, false>), g, b, 0, s, p);
  else if (xh) hipLaunchKernelGGL((k_color<DT, PASS_FUSED, true>), g, b, 0, s, p);
  else hipLaunchKernelGGL((k_color<DT, PASS_FUSED, false>), g, b, 0, s, p);
  return hipGetLastError();
}

template <int DT>
static hipError_t launch_color_lds2(const LaunchParams& p, int pass, bool xh, int blocks,
                                    size_t lds, hipStream_t s) {
  const dim3 g(blocks), b(256);
  if (pass == PASS_FWD) hipLaunchKernelGGL((k_color_lds<DT, PASS_FWD, false>), g, b, lds, s, p);
  else if (pass == PASS_ADJ && xh) hipLaunchKernelGGL((k_color_lds<DT, PASS_ADJ, true>), g, b, lds, s, p);
  else if (pass == PASS_ADJ) hipLaunchKernelGGL((k_color_lds<DT, PASS_ADJ, false>), g, b, lds, s, p);
  else if (xh) hipLaunchKernelGGL((k_color_lds<DT, PASS_FUSED, true>), g, b, lds, s, p);
  else hipLaunchKernelGGL((k_color_lds<DT, PASS_FUSED, false>), g, b, lds, s, p);
  return hipGetLastError();
}

int launch_color(const LaunchParams& p, int pass, int dtype, int slab, size_t lds_bytes,
                 void* stream) {
  if (p.n_items <= 0) return 0;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const bool xh = (p.grad_mask & (GRAD_CAM | GRAD_STEP)) != 0;
  if (slab) {
    switch (dtype) {
      case DDVR_F16: return (int)launch_color_lds2<DDVR_F16>(p, pass, xh, p.n_items, lds_bytes, s);
      case DDVR_BF16: return (int)launch_color_lds2<DDVR_BF16>(p, pass, xh, p.n_items, lds_bytes, s);
      default: return (int)launch_color_lds2<DDVR_F32>(p, pass, xh, p.n_items, lds_bytes, s);
    }
  }
  switch (dtype) {
    case DDVR_F16: return (int)launch_color2<DDVR_F16>(p, pass, xh, p.n_items, s);
    case DDVR_BF16: return (int)launch_color2<DDVR_BF16>(p, pass, xh, p.n_items, s);
    default: return (int)launch_color2<DDVR_F32>(p, pass, xh, p.n_items, s);
  }
}

int launch_zero_i32(int32_t* ptr, int n, void* stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_zero_i32, dim3((n + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), ptr, n);
  return (int)hipGetLastError();
}

}  // namespace ddvr

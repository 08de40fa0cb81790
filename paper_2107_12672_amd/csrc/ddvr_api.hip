// Host side of the C ABI declared in include/ddvr.h: argument validation,
// camera helpers, launch planning (tile grid, slab length, LDS budget),
// workspace layout of the checkpoint fallback, batches and graph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ddvr.h"
#include "ddvr_internal.h"

using namespace ddvr;

// Scratch of the allocation-free adjoint (ddvr_render_adjoint_noalloc): the
// checkpoint fallback's ray queue and per-slot storage.  One copy per device,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per
// device (static_scratch).
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

thread_local char g_err[512] = "no error";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(DDVR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Surface an asynchronous error left by an earlier launch.
int check_pending() {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "pending HIP error");
  return DDVR_OK;
}

// Device address of the current device's `scratch`, looked up on the first
// call on that device (with it current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "querying the current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(DDVR_ERR_UNSUPPORTED, "device %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "address of the static scratch");
    if (!p) return fail(DDVR_ERR_HIP, "address of the static scratch is NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DDVR_OK;
}

bool finite3(const float* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

constexpr int kFallbackSlots = 1 << 19;   // concurrent checkpoint slots (8 workgroups per CU)

// Launch shape of the render kernels (process-wide; see ddvr_set_tuning).
struct Tuning {
  int waves = 4;        // waves per workgroup: 1 -> 8x8, 2 -> 16x8, 4 -> 16x16 pixel tiles
  int lds_cap = 7168;   // voxels per LDS brick (clamped to the device's LDS per workgroup)
  int slab_k = 64;      // initial samples per slab
  int slab_kmax = 256;  // longest slab tried
  int cell_acc = 1;     // per-cell register accumulation of the density gradient
  int lane_map = 2;     // lane -> pixel maps: compact forward, interleaved adjoint
  int schedule = 0;     // batches: 0 auto, 1 one workgroup per tile, 2 persistent queue
  int slab_axis = 1;    // slabs between planes of a grid axis (0: distance shells)
};
Tuning g_tuning;

// 4-byte words of LDS per brick voxel: the staged grid value, plus the
// gradient brick's entry when the adjoint needs both (a 64-bit entry for
// emission-absorption)
int brick_words(int two, int model) {
  return two ? (model == DDVR_EMISSION_ABSORPTION ? 3 : 2) : 1;
}

size_t lds_bytes(int cap, int two, int model, int R) {
  const size_t tf = model == DDVR_EMISSION_ABSORPTION ? (size_t)R * 8 : 0;
  return ((size_t)brick_words(two, model) * cap + tf) * sizeof(float) + 64 * sizeof(int);
}

// Largest dynamic LDS allocation of one workgroup on the current device.
int lds_limit(int* lim) {
  int dev = 0;
  *lim = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return hip_fail(e, "querying the LDS limit");
  return DDVR_OK;
}

int check_lds(size_t bytes) {
  int lim = 0, rc = lds_limit(&lim);
  if (rc) return rc;
  if (bytes > (size_t)lim)
    return fail(DDVR_ERR_UNSUPPORTED, "launch needs %zu bytes of LDS, the device allows %d (lower "
                "lds_cap or the TF size)", bytes, lim);
  return DDVR_OK;
}

// Brick capacity that fits the device next to the TF tables and scratch.
// The emission-absorption adjoint's bricks (a 64-bit gradient entry beside
// each staged value) take 2/3 of `cap` voxels, the LDS bytes of `cap` voxels
// with 32-bit entries, so that as many workgroups fit per CU.  Kept even: the
// 64-bit entries start after `cap` staged floats and must be 8-byte aligned.
int fit_cap(int cap, int two, int model, int R, int* out) {
  *out = cap;
  if (cap <= 0) return DDVR_OK;
  if (two && model == DDVR_EMISSION_ABSORPTION) cap = std::max(2 * cap / 3, 64);
  int lim = 0, rc = lds_limit(&lim);
  if (rc) return rc;
  const size_t fixed = lds_bytes(0, two, model, R);
  if ((size_t)lim <= fixed + 256 * sizeof(float))
    return fail(DDVR_ERR_UNSUPPORTED, "TF of %d entries leaves no LDS for bricks", R);
  const int most = (int)((lim - fixed) / (brick_words(two, model) * sizeof(float)));
  *out = std::min(cap, most) & ~1;
  return DDVR_OK;
}

int tile_w(int waves) { return waves == 1 ? 8 : 16; }
int tile_h(int waves) { return waves == 4 ? 16 : 8; }

int validate_volume(const ddvr_volume* v) {
  if (!v) return fail(DDVR_ERR_NULL, "volume descriptor is NULL");
  if (!v->data) return fail(DDVR_ERR_NULL, "volume data is NULL");
  if (v->dtype != DDVR_F32 && v->dtype != DDVR_F16 && v->dtype != DDVR_BF16)
    return fail(DDVR_ERR_DTYPE, "unknown volume dtype %d", v->dtype);
  if (v->nx < 2 || v->ny < 2 || v->nz < 2)
    return fail(DDVR_ERR_SHAPE, "grid %dx%dx%d: every size must be >= 2", v->nx, v->ny, v->nz);
  if ((int64_t)v->nx * v->ny * v->nz > (int64_t)1 << 34)
    return fail(DDVR_ERR_SHAPE, "grid too large");
  return DDVR_OK;
}

int validate_tf(const ddvr_tf* tf, int model) {
  if (model == DDVR_ABSORPTION || model == DDVR_COLOR) return DDVR_OK;
  if (!tf) return fail(DDVR_ERR_NULL, "transfer function descriptor is NULL");
  if (!tf->rgba_tau) return fail(DDVR_ERR_NULL, "transfer function table is NULL");
  if (tf->R < 2 || tf->R > 4096) return fail(DDVR_ERR_SHAPE, "TF size R=%d not in [2, 4096]", tf->R);
  return DDVR_OK;
}

int validate_model(int model) {
  if (model != DDVR_ABSORPTION && model != DDVR_EMISSION_ABSORPTION && model != DDVR_COLOR)
    return fail(DDVR_ERR_VALUE, "unknown model %d", model);
  return DDVR_OK;
}

// The adjoint modes a model takes (flags already validated).
int validate_mode(int model, int flags) {
  const int mode = flags & DDVR_ADJ_MODE_MASK;
  if (model == DDVR_COLOR && (mode == DDVR_ADJ_INVERT_ALPHA || mode == DDVR_ADJ_CHECKPOINT))
    return fail(DDVR_ERR_UNSUPPORTED, "the colour model takes AUTO, INVERT_T or RESIDUAL");
  if (model != DDVR_COLOR && mode == DDVR_ADJ_RESIDUAL)
    return fail(DDVR_ERR_UNSUPPORTED, "the RESIDUAL adjoint mode is for the colour model");
  return DDVR_OK;
}

// Colour volumes are read one vertex (4 values) per load.
int validate_color_volume(const ddvr_volume* v) {
  const uintptr_t align = v->dtype == DDVR_F32 ? 16 : 8;
  if (reinterpret_cast<uintptr_t>(v->data) % align)
    return fail(DDVR_ERR_VALUE, "colour volume data must be %d-byte aligned", (int)align);
  return DDVR_OK;
}

int validate_camera(const ddvr_camera* c) {
  if (!c) return fail(DDVR_ERR_NULL, "camera is NULL");
  if (c->width <= 0 || c->height <= 0) return fail(DDVR_ERR_SHAPE, "image %dx%d", c->width, c->height);
  if ((int64_t)c->width * c->height > ((int64_t)1 << 31) - 1)
    return fail(DDVR_ERR_SHAPE, "image too large");
  if (!finite3(c->eye) || !finite3(c->fwd) || !finite3(c->right) || !finite3(c->up))
    return fail(DDVR_ERR_VALUE, "camera frame is not finite");
  return DDVR_OK;
}

float half_diag(const ddvr_volume* v) {
  const int nmax = std::max(v->nx, std::max(v->ny, v->nz));
  const double h = 2.0 / (nmax - 1);
  const double ex = (v->nx - 1) * h, ey = (v->ny - 1) * h, ez = (v->nz - 1) * h;
  return (float)(0.5 * std::sqrt(ex * ex + ey * ey + ez * ez));
}

int64_t max_samples(const ddvr_volume* v, float step) {
  return (int64_t)std::ceil(2.0 * half_diag(v) / step) + 1;
}

int validate_step(const ddvr_volume* v, float step) {
  if (!std::isfinite(step) || !(step > 0.0f)) return fail(DDVR_ERR_VALUE, "step %g must be > 0", step);
  if (max_samples(v, step) > kMaxSamples)
    return fail(DDVR_ERR_VALUE, "step %g gives more than %d samples per ray", step, kMaxSamples);
  return DDVR_OK;
}

void fill_view(ViewDesc& d, const ddvr_volume* v, const ddvr_tf* tf, const ddvr_camera* c,
               float step, int model, int cap) {
  std::memset(&d, 0, sizeof(d));
  for (int a = 0; a < 3; ++a) {
    d.eye[a] = c->eye[a]; d.fwd[a] = c->fwd[a]; d.right[a] = c->right[a]; d.up[a] = c->up[a];
  }
  d.W = c->width;
  d.H = c->height;
  d.step = step;
  d.vol = v->data;
  d.dtype = v->dtype;
  d.nx = v->nx; d.ny = v->ny; d.nz = v->nz;
  const int nmax = std::max(v->nx, std::max(v->ny, v->nz));
  const double h = 2.0 / (nmax - 1);
  d.h = (float)h;
  d.inv_h = (float)(0.5 * (nmax - 1));
  const int n[3] = {v->nx, v->ny, v->nz};
  for (int a = 0; a < 3; ++a) {
    d.bmin[a] = (float)(-0.5 * (n[a] - 1) * h);
    d.bmax[a] = (float)(0.5 * (n[a] - 1) * h);
    d.qhi[a] = std::nextafter((float)(n[a] - 1), 0.0f);
  }
  if (model == DDVR_EMISSION_ABSORPTION) { d.tf = tf->rgba_tau; d.R = tf->R; }
  const int tw = tile_w(g_tuning.waves), th = tile_h(g_tuning.waves);
  d.tiles_x = (c->width + tw - 1) / tw;
  d.tiles_y = (c->height + th - 1) / th;
  d.slab_k = cap > 0 ? g_tuning.slab_k : kMaxSamples + 1;
}


// Whether the adjoint needs the grid values and the gradient brick at once.
int needs_two_bricks(int pass, int model, int flags, int gmask) {
  if (pass == PASS_FWD) return 0;
  const int mode = flags & DDVR_ADJ_MODE_MASK;
  const bool need_v = model == DDVR_EMISSION_ABSORPTION || (gmask & (GRAD_CAM | GRAD_STEP)) ||
                      mode != DDVR_ADJ_AUTO;
  return need_v && (gmask & GRAD_V) ? 1 : 0;
}

int grad_mask_of(const ddvr_grads* g) {
  if (!g) return 0;
  return (g->d_volume ? GRAD_V : 0) | (g->d_tf ? GRAD_TF : 0) | (g->d_camera ? GRAD_CAM : 0) |
         (g->d_step ? GRAD_STEP : 0);
}

// Workspace of the checkpoint fallback:
//   [0, 256)                 queue length (int32)
//   [256, 256 + 8*cap)       queue of (view << 32 | pixel)
//   then slots*slot_floats   per-slot checkpoint storage
struct FbLayout {
  int64_t cap = 0;
  int slots = 0, slot_floats = 0;
  size_t bytes = 0;
};

// budget > 0: at most `budget` bytes (fewer slots, down to one workgroup's
// 256; the queue always holds every ray); L.bytes > budget when even that
// does not fit.
FbLayout fallback_layout(int64_t rays, int64_t nmax_samples, size_t budget = 0) {
  FbLayout L;
  L.cap = rays;
  int K = (int)std::ceil(std::sqrt((double)nmax_samples));
  while ((int64_t)K * K < nmax_samples) ++K;
  // a ray of N <= nmax_samples samples uses ceil(N/K) + K + 1 <= 2K + 1 floats
  L.slot_floats = ((2 * K + 4 + 63) / 64) * 64;
  L.slots = (int)std::min<int64_t>(kFallbackSlots, std::max<int64_t>(rays, 1));
  L.bytes = 256 + (size_t)8 * rays;
  L.bytes = (L.bytes + 255) / 256 * 256;
  const size_t slot_bytes = (size_t)L.slot_floats * sizeof(float);
  if (budget > 0) {
    const size_t room = budget > L.bytes ? budget - L.bytes : 0;
    const int64_t fit = (int64_t)(room / slot_bytes);
    L.slots = (int)std::max<int64_t>(std::min<int64_t>(L.slots, fit), std::min(256, L.slots));
  }
  L.bytes += (size_t)L.slots * slot_bytes;
  return L;
}

bool needs_fallback(int model, int flags) {
  if (model == DDVR_COLOR) return false;
  const int mode = flags & DDVR_ADJ_MODE_MASK;
  return mode == DDVR_ADJ_CHECKPOINT || mode == DDVR_ADJ_INVERT_ALPHA ||
         (model == DDVR_EMISSION_ABSORPTION && mode == DDVR_ADJ_AUTO);
}

int validate_flags(int flags) {
  const int mode = flags & DDVR_ADJ_MODE_MASK;
  if (mode > DDVR_ADJ_RESIDUAL) return fail(DDVR_ERR_VALUE, "unknown adjoint mode %d", mode);
  if (flags & ~(DDVR_ADJ_MODE_MASK | DDVR_LAUNCH_PLAIN | DDVR_LOSS_L1))
    return fail(DDVR_ERR_VALUE, "unknown flag bits 0x%x", flags);
  return DDVR_OK;
}

void attach_fallback(LaunchParams& p, const FbLayout& L, void* ws, int flags) {
  char* b = static_cast<char*>(ws);
  p.fb_count = reinterpret_cast<int32_t*>(b);
  p.fb_list = reinterpret_cast<int64_t*>(b + 256);
  p.fb_cap = L.cap;
  p.fb_tmin = (flags & DDVR_ADJ_MODE_MASK) == DDVR_ADJ_INVERT_ALPHA ? kFallbackTminAlpha
                                                                     : kFallbackTmin;
  p.fb_all = (flags & DDVR_ADJ_MODE_MASK) == DDVR_ADJ_CHECKPOINT ? 1 : 0;
  const size_t off = ((256 + (size_t)8 * L.cap) + 255) / 256 * 256;
  p.fb_scratch = reinterpret_cast<float*>(b + off);
  p.fb_slots = L.slots;
  p.fb_slot_floats = L.slot_floats;
}

// The fallback's LDS table for the TF gradient: used when every view that
// wants a TF gradient writes the same dTF, of one size of at most
// kFallbackTabR entries (16 KB of LDS per workgroup).
constexpr int kFallbackTabR = 1024;
void fallback_tf_table(LaunchParams& p, const ViewDesc* views, size_t n, int model) {
  p.fb_dtf = nullptr;
  p.fb_tf_R = 0;
  if (model != DDVR_EMISSION_ABSORPTION || !(p.grad_mask & GRAD_TF)) return;
  float* dtf = nullptr;
  int R = 0;
  for (size_t i = 0; i < n; ++i) {
    if (!views[i].dTF) continue;
    if (!dtf) {
      dtf = views[i].dTF;
      R = views[i].R;
    } else if (views[i].dTF != dtf || views[i].R != R) {
      return;
    }
  }
  if (!dtf || R > kFallbackTabR) return;
  p.fb_dtf = dtf;
  p.fb_tf_R = R;
}

int read_fallback_count(const LaunchParams& p, hipStream_t s, int32_t* out) {
  if (!out) return DDVR_OK;
  if (!p.fb_count) { *out = 0; return DDVR_OK; }
  int32_t n = 0;
  hipError_t e = hipMemcpyAsync(&n, p.fb_count, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading the fallback count");
  *out = n;
  return DDVR_OK;
}

// One view: forward / adjoint / fused.
int run_single(int pass, const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
               float step, int model, float* image, float* trans, const float* d_image,
               const float* target, float loss_scale, const ddvr_grads* grads, int flags,
               void* ws, size_t ws_bytes, int32_t* n_fb, double* loss_out, void* stream,
               bool ws_budget = false) {
  int rc;
  if ((rc = validate_model(model)) || (rc = validate_volume(vol)) || (rc = validate_tf(tf, model)) ||
      (rc = validate_camera(cam)) || (rc = validate_step(vol, step)) || (rc = validate_flags(flags)) ||
      (rc = validate_mode(model, flags)))
    return rc;
  if (model == DDVR_COLOR && (rc = validate_color_volume(vol))) return rc;
  if (!image) return fail(DDVR_ERR_NULL, "image is NULL");
  if (pass == PASS_ADJ) {
    if (!trans) return fail(DDVR_ERR_NULL, "transmittance is NULL (the adjoint needs T_N)");
    if (!d_image) return fail(DDVR_ERR_NULL, "d_image is NULL");
  }
  if (pass == PASS_FUSED && !target) return fail(DDVR_ERR_NULL, "target is NULL");
  if (!std::isfinite(loss_scale)) return fail(DDVR_ERR_VALUE, "loss_scale is not finite");
  const bool fb = pass != PASS_FWD && needs_fallback(model, flags);
  FbLayout L;
  if (fb) {
    if (pass == PASS_FUSED && !trans && (flags & DDVR_ADJ_MODE_MASK) == DDVR_ADJ_AUTO &&
        model == DDVR_EMISSION_ABSORPTION) {
      // the fallback kernel recomputes the loss gradient from the written image
    }
    L = fallback_layout((int64_t)cam->width * cam->height, max_samples(vol, step),
                        ws_budget ? ws_bytes : 0);
    if (ws_budget && L.bytes > ws_bytes)
      return fail(DDVR_ERR_WORKSPACE, "a %dx%d view with up to %lld samples per ray needs %zu "
                  "bytes of scratch, the library's static scratch holds %zu", cam->width,
                  cam->height, (long long)max_samples(vol, step), L.bytes, ws_bytes);
    if (!ws || ws_bytes < L.bytes)
      return fail(DDVR_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", L.bytes,
                  ws ? ws_bytes : (size_t)0);
  }
  if ((rc = check_pending())) return rc;

  const int cap = (flags & DDVR_LAUNCH_PLAIN) ? 0 : g_tuning.lds_cap;
  LaunchParams p;
  std::memset(&p, 0, sizeof(p));
  fill_view(p.one, vol, tf, cam, step, model, cap);
  p.one.image = image;
  p.one.trans = trans;
  p.one.d_image = d_image;
  p.one.target = target;
  if (grads) {
    p.one.dV = grads->d_volume;
    p.one.dTF = model == DDVR_EMISSION_ABSORPTION ? grads->d_tf : nullptr;
    p.one.dcam = grads->d_camera;
    p.one.dstep = grads->d_step;
  }
  p.views = nullptr;
  p.work = nullptr;
  p.n_items = p.one.tiles_x * p.one.tiles_y;
  p.xcd_remap = 1;
  p.flags = flags;
  p.grad_mask = grad_mask_of(grads);
  if (model != DDVR_EMISSION_ABSORPTION) p.grad_mask &= ~GRAD_TF;
  p.lds_two = needs_two_bricks(pass, model, flags, p.grad_mask);
  if ((rc = fit_cap(cap, p.lds_two, model, p.one.R, &p.lds_cap))) return rc;
  p.slab_kmax = g_tuning.slab_kmax;
  p.cell_acc = g_tuning.cell_acc;
  p.lane_map = g_tuning.lane_map;
  p.slab_axis = g_tuning.slab_axis;
  p.loss_scale = loss_scale;
  p.loss_out = pass == PASS_FUSED ? loss_out : nullptr;
  if (fb) {
    attach_fallback(p, L, ws, flags);
    fallback_tf_table(p, &p.one, 1, model);
  }

  hipError_t e;
  if (model == DDVR_COLOR) {
    // own kernels, 16x16-pixel tiles, no workspace: the slab-synchronous
    // route (the tuning's brick bytes hold lds_cap/4 vertices of 4 channels)
    // or, with PLAIN or the RESIDUAL mode, the direct route
    p.one.tiles_x = (cam->width + 15) / 16;
    p.one.tiles_y = (cam->height + 15) / 16;
    p.n_items = p.one.tiles_x * p.one.tiles_y;
    const int slab = cap > 0 && (flags & DDVR_ADJ_MODE_MASK) != DDVR_ADJ_RESIDUAL;
    p.lds_cap = slab ? std::max(cap / 4, 16) : 0;
    const size_t lds = slab ? (size_t)p.lds_cap * 4 * sizeof(float) + 64 * sizeof(int) : 0;
    if (slab && (rc = check_lds(lds))) return rc;
    e = (hipError_t)launch_color(p, pass, vol->dtype, slab, lds, stream);
    if (e != hipSuccess) return hip_fail(e, "colour render launch");
    if (n_fb) *n_fb = 0;
    return DDVR_OK;
  }
  const size_t lds = lds_bytes(p.lds_cap, p.lds_two, model, p.one.R);
  if ((rc = check_lds(lds))) return rc;
  if (fb && (e = (hipError_t)launch_zero_i32(p.fb_count, 1, stream)) != hipSuccess)
    return hip_fail(e, "zeroing the fallback queue");
  e = (hipError_t)launch_render(p, pass, model, vol->dtype, g_tuning.waves, p.n_items, lds,
                                stream);
  if (e != hipSuccess) return hip_fail(e, "render launch");
  if (fb) {
    e = (hipError_t)launch_fallback(p, model, vol->dtype, pass == PASS_FUSED ? 1 : 0, stream);
    if (e != hipSuccess) return hip_fail(e, "fallback launch");
  }
  if (n_fb) {
    if (!fb) *n_fb = 0;
    else if ((rc = read_fallback_count(p, static_cast<hipStream_t>(stream), n_fb))) return rc;
  }
  return DDVR_OK;
}

// ---- tiny forward-mode number for the camera chain rule -------------------
struct D4 {
  double v, d[4];
};
D4 cst(double v) { D4 r{v, {0, 0, 0, 0}}; return r; }
D4 var(double v, int k) { D4 r = cst(v); r.d[k] = 1.0; return r; }
D4 add(D4 a, D4 b) { D4 r{a.v + b.v, {}}; for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
D4 sub(D4 a, D4 b) { D4 r{a.v - b.v, {}}; for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
D4 mul(D4 a, D4 b) {
  D4 r{a.v * b.v, {}};
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
D4 dvd(D4 a, D4 b) {
  D4 r{a.v / b.v, {}};
  for (int k = 0; k < 4; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
D4 fn(double v, double dv, D4 a) { D4 r{v, {}}; for (int k = 0; k < 4; ++k) r.d[k] = dv * a.d[k]; return r; }
D4 dsin(D4 a) { return fn(std::sin(a.v), std::cos(a.v), a); }
D4 dcos(D4 a) { return fn(std::cos(a.v), -std::sin(a.v), a); }
D4 dtan(D4 a) { const double t = std::tan(a.v); return fn(t, 1.0 + t * t, a); }
D4 dsqrt(D4 a) { const double s = std::sqrt(a.v); return fn(s, 0.5 / s, a); }

// frame[12] = eye, fwd, right*sx, up*sy as functions of (yaw, pitch, dist, fovy)
void sphere_frame(double yaw, double pitch, double dist, double fovy, int W, int H, D4* f) {
  const D4 y = var(yaw, 0), p = var(pitch, 1), r = var(dist, 2), fo = var(fovy, 3);
  const D4 e0 = mul(mul(r, dcos(p)), dcos(y));
  const D4 e1 = mul(r, dsin(p));
  const D4 e2 = mul(mul(r, dcos(p)), dsin(y));
  const D4 len = dsqrt(add(add(mul(e0, e0), mul(e1, e1)), mul(e2, e2)));
  const D4 F0 = dvd(sub(cst(0), e0), len), F1 = dvd(sub(cst(0), e1), len),
           F2 = dvd(sub(cst(0), e2), len);
  const D4 rl = dsqrt(add(mul(F2, F2), mul(F0, F0)));
  const D4 R0 = dvd(sub(cst(0), F2), rl), R1 = cst(0.0), R2 = dvd(F0, rl);
  const D4 U0 = sub(mul(R1, F2), mul(R2, F1));
  const D4 U1 = sub(mul(R2, F0), mul(R0, F2));
  const D4 U2 = sub(mul(R0, F1), mul(R1, F0));
  const D4 sy = dtan(mul(fo, cst(0.5)));
  const D4 sx = mul(sy, cst((double)W / H));
  f[0] = e0; f[1] = e1; f[2] = e2;
  f[3] = F0; f[4] = F1; f[5] = F2;
  f[6] = mul(R0, sx); f[7] = mul(R1, sx); f[8] = mul(R2, sx);
  f[9] = mul(U0, sy); f[10] = mul(U1, sy); f[11] = mul(U2, sy);
}

int validate_sphere(float yaw, float pitch, float dist, float fovy, int W, int H) {
  if (!std::isfinite(yaw) || !std::isfinite(pitch) || !std::isfinite(dist) || !std::isfinite(fovy))
    return fail(DDVR_ERR_VALUE, "camera pose is not finite");
  if (!(std::fabs(pitch) < 1.5707963267948966 - 1e-6))
    return fail(DDVR_ERR_VALUE, "|pitch| must be < pi/2");
  if (!(dist > 0.0f)) return fail(DDVR_ERR_VALUE, "camera distance must be > 0");
  if (!(fovy > 0.0f) || !(fovy < 3.14159265f)) return fail(DDVR_ERR_VALUE, "fovy must be in (0, pi)");
  if (W <= 0 || H <= 0) return fail(DDVR_ERR_SHAPE, "image %dx%d", W, H);
  return DDVR_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// Samples of every tile of a view (host replay of the kernels' float64 ray
// setup): the cost model of the longest-first tile queue and the exact sample
// count of a batch.
static std::vector<int64_t> tile_samples(const ViewDesc& d, int tw, int th) {
  std::vector<int64_t> cost((size_t)d.tiles_x * d.tiles_y, 0);
  const int n3[3] = {d.nx, d.ny, d.nz};
  const int nmax = std::max(d.nx, std::max(d.ny, d.nz));
  double bmin[3];
  for (int a = 0; a < 3; ++a) bmin[a] = -(double)(n3[a] - 1) / (double)(nmax - 1);
  for (int py = 0; py < d.H; ++py)
    for (int px = 0; px < d.W; ++px) {
      const double u = 2.0 * ((double)px + 0.5) / (double)d.W - 1.0;
      const double v = 1.0 - 2.0 * ((double)py + 0.5) / (double)d.H;
      double w[3], om[3];
      for (int a = 0; a < 3; ++a)
        w[a] = (double)d.fwd[a] + u * (double)d.right[a] + v * (double)d.up[a];
      const double wl = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
      if (!(wl > 0.0) || !(wl < INFINITY)) continue;
      for (int a = 0; a < 3; ++a) om[a] = w[a] / wl;
      double tn = -INFINITY, tf = INFINITY;
      bool ok = true;
      for (int a = 0; a < 3; ++a) {
        const double e = (double)d.eye[a];
        if (om[a] == 0.0) {
          if (e < bmin[a] || e > -bmin[a]) ok = false;
          continue;
        }
        const double ta = (bmin[a] - e) / om[a], tb = (-bmin[a] - e) / om[a];
        tn = std::max(tn, std::min(ta, tb));
        tf = std::min(tf, std::max(ta, tb));
      }
      const double t0 = tn > 0.0 ? tn : 0.0;
      if (ok && tf > t0 && (tf - t0) < 1e30)
        cost[(size_t)(py / th) * d.tiles_x + px / tw] +=
            (int64_t)std::min(std::ceil((tf - t0) / (double)d.step), (double)kMaxSamples);
    }
  return cost;
}

struct ddvr_batch {
  int model = 0, flags = 0;
  Tuning tuning;
  std::vector<ViewDesc> views;
  int launch_dtype = 0;    // storage type of every view, or kDtypeDynamic if they differ
  int max_R = 2;
  int persistent = 0;      // 1: persistent workgroups on a longest-first tile queue
  int n_items = 0;
  ViewDesc* d_views = nullptr;
  int32_t* d_work = nullptr;
  int32_t* d_queue = nullptr;
  int64_t total_rays = 0, max_n = 1;
  int64_t samples = 0;
  int grad_mask = 0;
  // graph cache: one recorded graph per pass, each keyed on the arguments
  // captured into it, so alternating passes replay instead of re-recording
  struct GraphSlot {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    float scale = 0.0f;
    double* loss = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
  };
  GraphSlot slots[3];
  hipStream_t cap_stream = nullptr;
  int64_t graph_builds = 0;   // graphs recorded and instantiated so far
};

extern "C" {

int ddvr_abi_version(void) { return DDVR_ABI_VERSION; }

const char* ddvr_last_error(void) { return g_err; }

int ddvr_camera_from_sphere(float yaw, float pitch, float dist, float fovy, int32_t width,
                            int32_t height, ddvr_camera* out) {
  if (!out) return fail(DDVR_ERR_NULL, "output camera is NULL");
  int rc = validate_sphere(yaw, pitch, dist, fovy, width, height);
  if (rc) return rc;
  D4 f[12];
  sphere_frame(yaw, pitch, dist, fovy, width, height, f);
  for (int a = 0; a < 3; ++a) {
    out->eye[a] = (float)f[a].v;
    out->fwd[a] = (float)f[3 + a].v;
    out->right[a] = (float)f[6 + a].v;
    out->up[a] = (float)f[9 + a].v;
  }
  out->width = width;
  out->height = height;
  return DDVR_OK;
}

int ddvr_camera_grad_to_sphere(float yaw, float pitch, float dist, float fovy, int32_t width,
                               int32_t height, const float* d_frame, float* d_sphere) {
  if (!d_frame || !d_sphere) return fail(DDVR_ERR_NULL, "gradient pointer is NULL");
  int rc = validate_sphere(yaw, pitch, dist, fovy, width, height);
  if (rc) return rc;
  D4 f[12];
  sphere_frame(yaw, pitch, dist, fovy, width, height, f);
  for (int k = 0; k < 4; ++k) {
    double acc = 0.0;
    for (int j = 0; j < 12; ++j) acc += f[j].d[k] * (double)d_frame[j];
    d_sphere[k] = (float)acc;
  }
  return DDVR_OK;
}

int ddvr_camera_sphere_tangents(float yaw, float pitch, float dist, float fovy, int32_t width,
                                int32_t height, float* d_frame) {
  if (!d_frame) return fail(DDVR_ERR_NULL, "output pointer is NULL");
  int rc = validate_sphere(yaw, pitch, dist, fovy, width, height);
  if (rc) return rc;
  D4 f[12];
  sphere_frame(yaw, pitch, dist, fovy, width, height, f);
  for (int k = 0; k < 4; ++k)
    for (int j = 0; j < 12; ++j) d_frame[k * 12 + j] = (float)f[j].d[k];
  return DDVR_OK;
}

int ddvr_render_tangent(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                        float step_world, int32_t model, const ddvr_direction* dirs, int32_t ndir,
                        float* image, float* image_dot, const float* d_image, float* d_dir,
                        int32_t flags, void* hip_stream) {
  int rc;
  if ((rc = validate_model(model)) || (rc = validate_volume(vol)) || (rc = validate_tf(tf, model)) ||
      (rc = validate_camera(cam)) || (rc = validate_step(vol, step_world)))
    return rc;
  if (model == DDVR_COLOR && (rc = validate_color_volume(vol))) return rc;
  if (flags & ~DDVR_LAUNCH_PLAIN) return fail(DDVR_ERR_VALUE, "tangent flags: only DDVR_LAUNCH_PLAIN");
  if (!dirs) return fail(DDVR_ERR_NULL, "dirs is NULL");
  if (ndir < 1 || ndir > DDVR_MAX_DIRECTIONS)
    return fail(DDVR_ERR_VALUE, "ndir must be 1..%d", DDVR_MAX_DIRECTIONS);
  for (int k = 0; k < ndir; ++k) {
    for (int j = 0; j < 12; ++j)
      if (!std::isfinite(dirs[k].d_frame[j])) return fail(DDVR_ERR_VALUE, "direction %d is not finite", k);
    if (!std::isfinite(dirs[k].d_step)) return fail(DDVR_ERR_VALUE, "direction %d is not finite", k);
  }
  if (!image && !image_dot && !d_dir)
    return fail(DDVR_ERR_NULL, "nothing to write: image, image_dot and d_dir are NULL");
  if (d_dir && !d_image) return fail(DDVR_ERR_NULL, "d_dir needs d_image");
  if ((rc = check_pending())) return rc;

  const int cap = (flags & DDVR_LAUNCH_PLAIN) ? 0 : g_tuning.lds_cap;
  TangentParams p;
  std::memset(&p, 0, sizeof(p));
  // tangent kernels run 16x16-pixel tiles of 4 waves whatever the tuning says
  fill_view(p.one, vol, tf, cam, step_world, model, cap);
  p.one.tiles_x = (cam->width + 15) / 16;
  p.one.tiles_y = (cam->height + 15) / 16;
  p.one.image = image;
  p.one.d_image = d_image;
  if ((rc = fit_cap(cap, 0, model, p.one.R, &p.lds_cap))) return rc;
  p.slab_kmax = g_tuning.slab_kmax;
  p.ndir = ndir;
  for (int k = 0; k < ndir; ++k) {
    for (int j = 0; j < 12; ++j) p.dir[k][j] = dirs[k].d_frame[j];
    p.dir[k][12] = dirs[k].d_step;
  }
  p.image_dot = image_dot;
  p.d_dir = d_dir;
  // (the colour volume's tangent kernel gathers directly: no brick)
  const size_t lds = model == DDVR_COLOR ? 0 : lds_bytes(p.lds_cap, 0, model, p.one.R);
  if ((rc = check_lds(lds))) return rc;
  const hipError_t e = (hipError_t)launch_tangent(p, model, vol->dtype,
                                                   p.one.tiles_x * p.one.tiles_y, lds, hip_stream);
  if (e != hipSuccess) return hip_fail(e, "tangent launch");
  return DDVR_OK;
}

int ddvr_set_tuning(const ddvr_tuning* t) {
  if (!t) return fail(DDVR_ERR_NULL, "tuning is NULL");
  if (t->waves != 1 && t->waves != 2 && t->waves != 4)
    return fail(DDVR_ERR_VALUE, "waves must be 1, 2 or 4");
  if (t->lds_cap < 64 || t->lds_cap > 16384)
    return fail(DDVR_ERR_VALUE, "lds_cap must be in [64, 16384] voxels");
  if (t->slab_k < 4 || t->slab_kmax < t->slab_k || t->slab_kmax > 4096)
    return fail(DDVR_ERR_VALUE, "need 4 <= slab_k <= slab_kmax <= 4096");
  if (t->cell_acc != 0 && t->cell_acc != 1) return fail(DDVR_ERR_VALUE, "cell_acc is 0 or 1");
  if (t->lane_map < 0 || t->lane_map > 3) return fail(DDVR_ERR_VALUE, "lane_map is 0..3");
  if (t->schedule < 0 || t->schedule > 2) return fail(DDVR_ERR_VALUE, "schedule is 0, 1 or 2");
  if (t->slab_axis != 0 && t->slab_axis != 1) return fail(DDVR_ERR_VALUE, "slab_axis is 0 or 1");
  g_tuning.schedule = t->schedule;
  g_tuning.slab_axis = t->slab_axis;
  g_tuning.waves = t->waves;
  g_tuning.lds_cap = t->lds_cap;
  g_tuning.slab_k = t->slab_k;
  g_tuning.slab_kmax = t->slab_kmax;
  g_tuning.cell_acc = t->cell_acc;
  g_tuning.lane_map = t->lane_map;
  return DDVR_OK;
}

int ddvr_get_tuning(ddvr_tuning* t) {
  if (!t) return fail(DDVR_ERR_NULL, "tuning is NULL");
  t->waves = g_tuning.waves;
  t->lds_cap = g_tuning.lds_cap;
  t->slab_k = g_tuning.slab_k;
  t->slab_kmax = g_tuning.slab_kmax;
  t->cell_acc = g_tuning.cell_acc;
  t->lane_map = g_tuning.lane_map;
  t->schedule = g_tuning.schedule;
  t->slab_axis = g_tuning.slab_axis;
  return DDVR_OK;
}

int ddvr_cast_volume(const float* src, void* dst, int32_t dtype, int64_t n, void* hip_stream) {
  if (!src || !dst) return fail(DDVR_ERR_NULL, "source or destination is NULL");
  if (dtype != DDVR_F32 && dtype != DDVR_F16 && dtype != DDVR_BF16)
    return fail(DDVR_ERR_DTYPE, "unknown dtype %d", dtype);
  if (n < 0) return fail(DDVR_ERR_SHAPE, "negative element count");
  int rc = check_pending();
  if (rc) return rc;
  const hipError_t e = (hipError_t)launch_cast(src, dst, dtype, n, hip_stream);
  if (e != hipSuccess) return hip_fail(e, "cast launch");
  return DDVR_OK;
}

int ddvr_render_forward(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                        float step_world, int32_t model, float* image, float* transmittance,
                        int32_t flags, void* hip_stream) {
  if (flags & DDVR_ADJ_MODE_MASK)
    return fail(DDVR_ERR_VALUE, "forward flags must be 0 or DDVR_LAUNCH_PLAIN");
  return run_single(PASS_FWD, vol, tf, cam, step_world, model, image, transmittance, nullptr,
                    nullptr, 0.0f, nullptr, flags, nullptr, 0, nullptr, nullptr, hip_stream);
}

int ddvr_density_from_color(const ddvr_volume* color, const ddvr_tf* tf, const float* d_prev,
                            float alpha, float beta, uint64_t seed, int32_t sweep,
                            int32_t ncand, float* d_out, float* cost_out, uint32_t* n_changed,
                            void* hip_stream) {
  int rc;
  if ((rc = validate_volume(color)) || (rc = validate_color_volume(color)) ||
      (rc = validate_tf(tf, DDVR_EMISSION_ABSORPTION)))
    return rc;
  if (!d_out) return fail(DDVR_ERR_NULL, "d_out is NULL");
  if (d_prev && d_prev == d_out) return fail(DDVR_ERR_VALUE, "d_prev must not alias d_out");
  if (!std::isfinite(alpha) || !std::isfinite(beta))
    return fail(DDVR_ERR_VALUE, "alpha and beta must be finite");
  if (sweep < 0) return fail(DDVR_ERR_VALUE, "sweep must be >= 0");
  if (ncand < 1 || ncand > 65536) return fail(DDVR_ERR_VALUE, "ncand must be 1..65536");
  if ((rc = check_pending())) return rc;
  DfcParams p;
  std::memset(&p, 0, sizeof(p));
  p.cv = color->data;
  p.nx = color->nx; p.ny = color->ny; p.nz = color->nz;
  p.tf = tf->rgba_tau;
  p.R = tf->R;
  p.d_prev = d_prev;
  p.d_out = d_out;
  p.cost_out = cost_out;
  p.n_changed = n_changed;
  p.alpha = alpha;
  p.beta = beta;
  p.seed = seed;
  p.iter = sweep;
  p.ncand = ncand;
  const hipError_t e = (hipError_t)launch_density_from_color(p, color->dtype, hip_stream);
  if (e != hipSuccess) return hip_fail(e, "density-from-colour launch");
  return DDVR_OK;
}

int ddvr_color_tau_max(const ddvr_volume* color, float* out, void* hip_stream) {
  int rc;
  if ((rc = validate_volume(color)) || (rc = validate_color_volume(color))) return rc;
  if (!out) return fail(DDVR_ERR_NULL, "out is NULL");
  if ((rc = check_pending())) return rc;
  const int64_t nvox = (int64_t)color->nx * color->ny * color->nz;
  const hipError_t e =
      (hipError_t)launch_color_tau_max(color->data, color->dtype, nvox, out, hip_stream);
  if (e != hipSuccess) return hip_fail(e, "tau-max launch");
  return DDVR_OK;
}

int ddvr_tf_prior(const float* tf, int32_t R, float lambda, float* d_tf, double* loss_out,
                  void* hip_stream) {
  if (!tf) return fail(DDVR_ERR_NULL, "tf is NULL");
  if (R < 2 || R > (1 << 24)) return fail(DDVR_ERR_SHAPE, "R=%d not in [2, 2^24]", R);
  if (!std::isfinite(lambda)) return fail(DDVR_ERR_VALUE, "lambda is not finite");
  int rc;
  if ((rc = check_pending())) return rc;
  const hipError_t e = (hipError_t)launch_tf_prior(tf, R, lambda, d_tf, loss_out, hip_stream);
  return e == hipSuccess ? DDVR_OK : hip_fail(e, "tf prior launch");
}

int ddvr_volume_prior(const float* volume, int32_t nx, int32_t ny, int32_t nz, float lambda,
                      float* d_volume, double* loss_out, void* hip_stream) {
  if (!volume) return fail(DDVR_ERR_NULL, "volume is NULL");
  if (nx < 1 || ny < 1 || nz < 1 || (nx < 2 && ny < 2 && nz < 2) ||
      (int64_t)nx * ny * nz > ((int64_t)1 << 34))
    return fail(DDVR_ERR_SHAPE, "grid %dx%dx%d", nx, ny, nz);
  if (!std::isfinite(lambda)) return fail(DDVR_ERR_VALUE, "lambda is not finite");
  int rc;
  if ((rc = check_pending())) return rc;
  const hipError_t e =
      (hipError_t)launch_volume_prior(volume, nx, ny, nz, lambda, d_volume, loss_out, hip_stream);
  return e == hipSuccess ? DDVR_OK : hip_fail(e, "volume prior launch");
}

int ddvr_opacity_entropy(const float* image, int64_t npix, int32_t channels, double* work,
                         double* value_out, float* d_image, float scale, void* hip_stream) {
  if (!image || !work) return fail(DDVR_ERR_NULL, "image or work is NULL");
  if (npix < 2) return fail(DDVR_ERR_SHAPE, "need at least 2 pixels");
  if (channels != 1 && channels != 4) return fail(DDVR_ERR_VALUE, "channels must be 1 or 4");
  if (!std::isfinite(scale)) return fail(DDVR_ERR_VALUE, "scale is not finite");
  int rc;
  if ((rc = check_pending())) return rc;
  const hipError_t e = (hipError_t)launch_opacity_entropy(
      image, npix, channels, channels == 4 ? 3 : 0, work, value_out, d_image, scale, hip_stream);
  return e == hipSuccess ? DDVR_OK : hip_fail(e, "opacity entropy launch");
}

int ddvr_adam_step(float* param, float* grad, float* m, float* v, int64_t n, int32_t t,
                   float lr, float beta1, float beta2, float eps, float lo, float hi, void* store,
                   int32_t store_dtype, int32_t zero_grad, void* hip_stream) {
  if (!param || !grad || !m || !v) return fail(DDVR_ERR_NULL, "param, grad, m or v is NULL");
  if (n < 0) return fail(DDVR_ERR_SHAPE, "n < 0");
  if (t < 1) return fail(DDVR_ERR_VALUE, "step t must be >= 1");
  if (!std::isfinite(lr) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) ||
      !(eps >= 0.0f) || std::isnan(lo) || std::isnan(hi) || lo > hi)
    return fail(DDVR_ERR_VALUE, "Adam hyper-parameters out of range");
  if (store && store_dtype != DDVR_F32 && store_dtype != DDVR_F16 && store_dtype != DDVR_BF16)
    return fail(DDVR_ERR_DTYPE, "unknown store dtype %d", store_dtype);
  int rc;
  if ((rc = check_pending())) return rc;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)t)));
  const hipError_t e = (hipError_t)launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, c1,
                                               c2, lo, hi, store, store_dtype, zero_grad,
                                               hip_stream);
  return e == hipSuccess ? DDVR_OK : hip_fail(e, "Adam launch");
}

int ddvr_resample_channels(const float* src, int32_t channels, int32_t sx, int32_t sy,
                           int32_t sz, float* dst, int32_t dx, int32_t dy, int32_t dz,
                           void* hip_stream) {
  if (!src || !dst) return fail(DDVR_ERR_NULL, "src or dst is NULL");
  if (channels < 1 || channels > 4) return fail(DDVR_ERR_VALUE, "channels=%d not in [1, 4]", channels);
  if (sx < 2 || sy < 2 || sz < 2 || dx < 2 || dy < 2 || dz < 2 ||
      (int64_t)dx * dy * dz * channels > ((int64_t)1 << 34) ||
      (int64_t)sx * sy * sz * channels > ((int64_t)1 << 34))
    return fail(DDVR_ERR_SHAPE, "resample %dx%dx%d -> %dx%dx%d", sx, sy, sz, dx, dy, dz);
  const char* a = reinterpret_cast<const char*>(src);
  const char* b = reinterpret_cast<const char*>(dst);
  if (a < b + (int64_t)dx * dy * dz * channels * 4 && b < a + (int64_t)sx * sy * sz * channels * 4)
    return fail(DDVR_ERR_VALUE, "src and dst overlap");
  int rc;
  if ((rc = check_pending())) return rc;
  const hipError_t e =
      (hipError_t)launch_resample(src, channels, sx, sy, sz, dst, dx, dy, dz, hip_stream);
  return e == hipSuccess ? DDVR_OK : hip_fail(e, "resample launch");
}

int ddvr_resample_volume(const float* src, int32_t sx, int32_t sy, int32_t sz, float* dst,
                         int32_t dx, int32_t dy, int32_t dz, void* hip_stream) {
  return ddvr_resample_channels(src, 1, sx, sy, sz, dst, dx, dy, dz, hip_stream);
}

int ddvr_adjoint_workspace_size(const ddvr_volume* vol, const ddvr_camera* cam, float step_world,
                                int32_t model, int32_t flags, size_t* bytes) {
  int rc;
  if (!bytes) return fail(DDVR_ERR_NULL, "bytes is NULL");
  if ((rc = validate_model(model)) || (rc = validate_volume(vol)) || (rc = validate_camera(cam)) ||
      (rc = validate_step(vol, step_world)) || (rc = validate_flags(flags)) ||
      (rc = validate_mode(model, flags)))
    return rc;
  *bytes = needs_fallback(model, flags)
               ? fallback_layout((int64_t)cam->width * cam->height, max_samples(vol, step_world)).bytes
               : 0;
  return DDVR_OK;
}

int ddvr_render_adjoint(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                        float step_world, int32_t model, const float* image,
                        const float* transmittance, const float* d_image,
                        const ddvr_grads* grads, int32_t flags, void* workspace,
                        size_t workspace_bytes, int32_t* n_fallback_rays, void* hip_stream) {
  if (!grads) return fail(DDVR_ERR_NULL, "grads is NULL");
  return run_single(PASS_ADJ, vol, tf, cam, step_world, model, const_cast<float*>(image),
                    const_cast<float*>(transmittance), d_image, nullptr, 0.0f, grads, flags,
                    workspace, workspace_bytes, n_fallback_rays, nullptr, hip_stream);
}

int ddvr_render_adjoint_noalloc(const ddvr_volume* vol, const ddvr_tf* tf,
                                const ddvr_camera* cam, float step_world, int32_t model,
                                const float* image, const float* transmittance,
                                const float* d_image, const ddvr_grads* grads, int32_t flags,
                                int32_t* n_fallback_rays, void* hip_stream) {
  if (!grads) return fail(DDVR_ERR_NULL, "grads is NULL");
  int rc;
  if ((rc = validate_model(model)) || (rc = validate_flags(flags))) return rc;
  void* ws = nullptr;
  if (model != DDVR_COLOR && needs_fallback(model, flags) && (rc = static_scratch(&ws)))
    return rc;
  return run_single(PASS_ADJ, vol, tf, cam, step_world, model, const_cast<float*>(image),
                    const_cast<float*>(transmittance), d_image, nullptr, 0.0f, grads, flags,
                    ws, ws ? kStaticScratchBytes : 0, n_fallback_rays, nullptr, hip_stream,
                    true);
}

int ddvr_render_fused_l2(const ddvr_volume* vol, const ddvr_tf* tf, const ddvr_camera* cam,
                         float step_world, int32_t model, const float* target, float loss_scale,
                         float* image, float* transmittance, const ddvr_grads* grads,
                         int32_t flags, void* workspace, size_t workspace_bytes,
                         int32_t* n_fallback_rays, double* loss_out, void* hip_stream) {
  return run_single(PASS_FUSED, vol, tf, cam, step_world, model, image, transmittance, nullptr,
                    target, loss_scale, grads, flags, workspace, workspace_bytes,
                    n_fallback_rays, loss_out, hip_stream);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
int ddvr_batch_create(const ddvr_volume* vols, int32_t nvol, const ddvr_tf* tfs, int32_t ntf,
                      const ddvr_view* views, int32_t nview, int32_t model, int32_t flags,
                      float* const* d_volumes, float* const* d_tfs, void* hip_stream,
                      ddvr_batch** out) {
  int rc;
  if (!out) return fail(DDVR_ERR_NULL, "out is NULL");
  *out = nullptr;
  if (!vols || !views) return fail(DDVR_ERR_NULL, "volumes or views is NULL");
  if (nvol <= 0 || nview <= 0 || nview >= 2048)
    return fail(DDVR_ERR_SHAPE, "need 1..2047 views and >= 1 volume");
  if ((rc = validate_model(model)) || (rc = validate_flags(flags)) ||
      (rc = validate_mode(model, flags)))
    return rc;
  if (model == DDVR_COLOR &&
      ((flags & DDVR_LAUNCH_PLAIN) || (flags & DDVR_ADJ_MODE_MASK) == DDVR_ADJ_RESIDUAL))
    return fail(DDVR_ERR_UNSUPPORTED, "colour batches take the slab route only (no PLAIN, no RESIDUAL)");
  if (model == DDVR_EMISSION_ABSORPTION && (!tfs || ntf <= 0))
    return fail(DDVR_ERR_NULL, "emission-absorption batch without transfer functions");
  for (int i = 0; i < nvol; ++i) {
    if ((rc = validate_volume(&vols[i]))) return rc;
    if (model == DDVR_COLOR && (rc = validate_color_volume(&vols[i]))) return rc;
    if (model == DDVR_COLOR && vols[i].dtype != vols[0].dtype)
      return fail(DDVR_ERR_UNSUPPORTED, "colour batches need one storage type");
  }
  if (model == DDVR_EMISSION_ABSORPTION)
    for (int i = 0; i < ntf; ++i)
      if ((rc = validate_tf(&tfs[i], model))) return rc;
  const int cap = (flags & DDVR_LAUNCH_PLAIN) ? 0 : g_tuning.lds_cap;
  ddvr_batch* b = new (std::nothrow) ddvr_batch;
  if (!b) return fail(DDVR_ERR_VALUE, "out of host memory");
  b->tuning = g_tuning;
  b->model = model;
  b->flags = flags;
  b->views.resize(nview);
  int gmask = 0;
  for (int i = 0; i < nview; ++i) {
    const ddvr_view& v = views[i];
    if (v.volume < 0 || v.volume >= nvol) { delete b; return fail(DDVR_ERR_SHAPE, "view %d: bad volume index", i); }
    if (model == DDVR_EMISSION_ABSORPTION && (v.tf < 0 || v.tf >= ntf)) {
      delete b; return fail(DDVR_ERR_SHAPE, "view %d: bad TF index", i);
    }
    if ((rc = validate_camera(&v.cam)) || (rc = validate_step(&vols[v.volume], v.step_world))) {
      delete b; return rc;
    }
    if (!v.image) { delete b; return fail(DDVR_ERR_NULL, "view %d: image is NULL", i); }
    const ddvr_tf* tf = model == DDVR_EMISSION_ABSORPTION ? &tfs[v.tf] : nullptr;
    ViewDesc& d = b->views[i];
    fill_view(d, &vols[v.volume], tf, &v.cam, v.step_world, model, cap);
    if (model == DDVR_COLOR) {   // the colour kernel's 16x16 tiles
      d.tiles_x = (v.cam.width + 15) / 16;
      d.tiles_y = (v.cam.height + 15) / 16;
    }
    d.image = v.image;
    d.trans = v.transmittance;
    d.d_image = v.d_image;
    d.target = v.target;
    d.dV = d_volumes ? d_volumes[v.volume] : nullptr;
    d.dTF = (model == DDVR_EMISSION_ABSORPTION && d_tfs) ? d_tfs[v.tf] : nullptr;
    d.dcam = v.d_camera;
    d.dstep = v.d_step;
    gmask |= (d.dV ? GRAD_V : 0) | (d.dTF ? GRAD_TF : 0) | (d.dcam ? GRAD_CAM : 0) |
             (d.dstep ? GRAD_STEP : 0);
    d.dtype = vols[v.volume].dtype;
    if (i == 0) b->launch_dtype = d.dtype;
    else if (d.dtype != b->launch_dtype) b->launch_dtype = kDtypeDynamic;
    b->max_R = std::max(b->max_R, (int)d.R);
    b->total_rays += (int64_t)v.cam.width * v.cam.height;
    b->max_n = std::max<int64_t>(b->max_n, max_samples(&vols[v.volume], v.step_world));
    if ((int64_t)d.tiles_x * d.tiles_y >= (1 << 20)) {
      delete b; return fail(DDVR_ERR_SHAPE, "view %d: too many tiles", i);
    }
  }
  b->grad_mask = gmask;
  // Work list of (view << 20 | tile).  Even batches (every view the same image
  // size over one grid) keep views in order and tiles in raster order, one
  // workgroup per tile with contiguous ranges per XCD.  Uneven batches (or
  // schedule = 2) become a persistent launch whose workgroups pop tiles from a
  // queue ordered by estimated cost, longest first.
  const int tw = model == DDVR_COLOR ? 16 : tile_w(b->tuning.waves);
  const int th = model == DDVR_COLOR ? 16 : tile_h(b->tuning.waves);
  std::vector<std::pair<int64_t, int32_t>> items;
  bool even = true;
  for (int i = 0; i < nview; ++i) {
    const ViewDesc& d = b->views[i];
    const std::vector<int64_t> cost = tile_samples(d, tw, th);
    for (size_t t = 0; t < cost.size(); ++t) {
      items.emplace_back(cost[t], (int32_t)((i << 20) | (int)t));
      b->samples += cost[t];
    }
    if (d.W != b->views[0].W || d.H != b->views[0].H || d.vol != b->views[0].vol) even = false;
  }
  // batches mixing storage types always take the persistent (per-view type) launch
  // (the colour kernel takes one item per workgroup, in list order)
  b->persistent = model != DDVR_COLOR &&
                  (b->tuning.schedule == 2 || (b->tuning.schedule == 0 && !even) ||
                   b->launch_dtype == kDtypeDynamic);
  if (b->persistent) b->launch_dtype = kDtypeDynamic;
  if (b->persistent)
    std::stable_sort(items.begin(), items.end(),
                     [](const std::pair<int64_t, int32_t>& x,
                        const std::pair<int64_t, int32_t>& y) { return x.first > y.first; });
  std::vector<int32_t> work(items.size());
  for (size_t k = 0; k < items.size(); ++k) work[k] = items[k].second;
  b->n_items = (int)work.size();
  hipError_t e = hipMalloc(&b->d_views, sizeof(ViewDesc) * nview);
  if (e == hipSuccess) e = hipMalloc(&b->d_work, sizeof(int32_t) * work.size());
  if (e == hipSuccess) e = hipMalloc(&b->d_queue, 256);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_views, b->views.data(), sizeof(ViewDesc) * nview, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_work, work.data(), sizeof(int32_t) * work.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    ddvr_batch_destroy(b);
    return hip_fail(e, "batch descriptor upload");
  }
  *out = b;
  return DDVR_OK;
}

void ddvr_batch_destroy(ddvr_batch* b) {
  if (!b) return;
  for (auto& g : b->slots) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->d_views) (void)hipFree(b->d_views);
  if (b->d_work) (void)hipFree(b->d_work);
  if (b->d_queue) (void)hipFree(b->d_queue);
  delete b;
}

int ddvr_batch_workspace_size(const ddvr_batch* b, size_t* bytes) {
  if (!b || !bytes) return fail(DDVR_ERR_NULL, "batch or bytes is NULL");
  *bytes = needs_fallback(b->model, b->flags) ? fallback_layout(b->total_rays, b->max_n).bytes : 0;
  return DDVR_OK;
}

static int batch_enqueue(ddvr_batch* b, int pass, float loss_scale, double* loss_out, void* ws,
                         size_t ws_bytes, hipStream_t s) {
  if (pass < PASS_FWD || pass > PASS_FUSED) return fail(DDVR_ERR_VALUE, "unknown pass %d", pass);
  if (!std::isfinite(loss_scale)) return fail(DDVR_ERR_VALUE, "loss_scale is not finite");
  for (size_t i = 0; i < b->views.size(); ++i) {
    const ViewDesc& d = b->views[i];
    if (pass == PASS_ADJ && (!d.d_image || !d.trans))
      return fail(DDVR_ERR_NULL, "view %zu: adjoint needs d_image and transmittance", i);
    if (pass == PASS_FUSED && !d.target) return fail(DDVR_ERR_NULL, "view %zu: target is NULL", i);
  }
  const bool fb = pass != PASS_FWD && needs_fallback(b->model, b->flags);
  FbLayout L;
  if (fb) {
    L = fallback_layout(b->total_rays, b->max_n);
    if (!ws || ws_bytes < L.bytes)
      return fail(DDVR_ERR_WORKSPACE, "workspace of %zu bytes needed", L.bytes);
  }
  LaunchParams p;
  std::memset(&p, 0, sizeof(p));
  p.views = b->d_views;
  p.flags = b->flags;
  p.grad_mask = b->grad_mask;
  if (b->model == DDVR_COLOR) {
    p.lds_cap = std::max(b->tuning.lds_cap / 4, 16);
    p.loss_scale = loss_scale;
    p.loss_out = pass == PASS_FUSED ? loss_out : nullptr;
    p.work = b->d_work;
    p.n_items = b->n_items;
    p.xcd_remap = 1;
    const size_t lds = (size_t)p.lds_cap * 4 * sizeof(float) + 64 * sizeof(int);
    int rc;
    if ((rc = check_lds(lds))) return rc;
    const hipError_t e = (hipError_t)launch_color(p, pass, b->launch_dtype, 1, lds, s);
    return e == hipSuccess ? DDVR_OK : hip_fail(e, "colour batch launch");
  }
  p.lds_two = needs_two_bricks(pass, b->model, b->flags, b->grad_mask);
  {
    const int rc = fit_cap((b->flags & DDVR_LAUNCH_PLAIN) ? 0 : b->tuning.lds_cap, p.lds_two,
                           b->model, b->max_R, &p.lds_cap);
    if (rc) return rc;
  }
  p.slab_kmax = b->tuning.slab_kmax;
  p.cell_acc = b->tuning.cell_acc;
  p.lane_map = b->tuning.lane_map;
  p.slab_axis = b->tuning.slab_axis;
  p.loss_scale = loss_scale;
  p.loss_out = pass == PASS_FUSED ? loss_out : nullptr;
  p.work = b->d_work;
  p.n_items = b->n_items;
  p.xcd_remap = b->persistent ? 0 : 1;
  p.queue = b->persistent ? b->d_queue : nullptr;
  if (fb) {
    attach_fallback(p, L, ws, b->flags);
    fallback_tf_table(p, b->views.data(), b->views.size(), b->model);
  }
  const size_t lds = lds_bytes(p.lds_cap, p.lds_two, b->model, b->max_R);
  {
    const int rc = check_lds(lds);
    if (rc) return rc;
  }
  hipError_t e;
  if (fb && (e = (hipError_t)launch_zero_i32(p.fb_count, 1, s)) != hipSuccess)
    return hip_fail(e, "zeroing the fallback queue");
  if (p.queue && (e = (hipError_t)launch_zero_i32(p.queue, 1, s)) != hipSuccess)
    return hip_fail(e, "zeroing the tile queue");
  e = (hipError_t)launch_render(p, pass, b->model, b->launch_dtype, b->tuning.waves, b->n_items,
                                lds, s);
  if (e != hipSuccess) return hip_fail(e, "batch render launch");
  if (fb) {
    e = (hipError_t)launch_fallback(p, b->model, b->launch_dtype, pass == PASS_FUSED ? 1 : 0, s);
    if (e != hipSuccess) return hip_fail(e, "batch fallback launch");
  }
  return DDVR_OK;
}

int ddvr_batch_run(ddvr_batch* b, int32_t pass, float loss_scale, double* loss_out,
                   void* workspace, size_t workspace_bytes, void* hip_stream) {
  if (!b) return fail(DDVR_ERR_NULL, "batch is NULL");
  int rc = check_pending();
  if (rc) return rc;
  return batch_enqueue(b, pass, loss_scale, loss_out, workspace, workspace_bytes,
                       static_cast<hipStream_t>(hip_stream));
}

int ddvr_batch_run_graph(ddvr_batch* b, int32_t pass, float loss_scale, double* loss_out,
                         void* workspace, size_t workspace_bytes, void* hip_stream) {
  if (!b) return fail(DDVR_ERR_NULL, "batch is NULL");
  if (pass < PASS_FWD || pass > PASS_FUSED) return fail(DDVR_ERR_VALUE, "unknown pass %d", pass);
  int rc = check_pending();
  if (rc) return rc;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  ddvr_batch::GraphSlot& g = b->slots[pass];
  const bool same = g.exec && g.scale == loss_scale && g.loss == loss_out && g.ws == workspace &&
                    g.ws_bytes == workspace_bytes;
  hipError_t e;
  if (!same) {
    // the old graph may still run on the caller's stream: let it finish first
    if (g.exec && (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "waiting for the previous replay");
    if (g.exec) { (void)hipGraphExecDestroy(g.exec); g.exec = nullptr; }
    if (g.graph) { (void)hipGraphDestroy(g.graph); g.graph = nullptr; }
    if (!b->cap_stream && (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "capture stream");
    if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
      return hip_fail(e, "begin capture");
    rc = batch_enqueue(b, pass, loss_scale, loss_out, workspace, workspace_bytes, b->cap_stream);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(b->cap_stream, &gr);
    if (rc) { if (gr) (void)hipGraphDestroy(gr); return rc; }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    g.graph = gr;
    if ((e = hipGraphInstantiate(&g.exec, gr, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(gr);
      g.graph = nullptr;
      g.exec = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    g.scale = loss_scale;
    g.loss = loss_out;
    g.ws = workspace;
    g.ws_bytes = workspace_bytes;
    ++b->graph_builds;
  }
  if ((e = hipGraphLaunch(g.exec, s)) != hipSuccess) return hip_fail(e, "graph launch");
  return DDVR_OK;
}

int ddvr_batch_graph_builds(const ddvr_batch* b, int64_t* builds) {
  if (!b || !builds) return fail(DDVR_ERR_NULL, "batch or builds is NULL");
  *builds = b->graph_builds;
  return DDVR_OK;
}

// ---------------------------------------------------------------------------
// plans: the whole step of a batch recorded into one HIP graph
// ---------------------------------------------------------------------------
struct ddvr_plan {
  ddvr_batch* b = nullptr;
  int loss = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  double* d_sums = nullptr;   // entropy: [nview][2] sums, then [nview] OE values
};

void ddvr_plan_destroy(ddvr_plan* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->d_sums) (void)hipFree(p->d_sums);
  delete p;
}

// The launches of one step, enqueued on s (recorded once by plan_create).
static int plan_enqueue(ddvr_plan* p, float loss_scale, double* loss_out, void* ws,
                        size_t ws_bytes, hipStream_t s) {
  ddvr_batch* b = p->b;
  int rc;
  if (p->loss == DDVR_PLAN_LOSS_FUSED)
    return batch_enqueue(b, PASS_FUSED, loss_scale, loss_out, ws, ws_bytes, s);
  if ((rc = batch_enqueue(b, PASS_FWD, 0.0f, nullptr, ws, ws_bytes, s))) return rc;
  if (p->loss == DDVR_PLAN_LOSS_NEG_ENTROPY) {
    int64_t max_pix = 1;
    for (const ViewDesc& d : b->views) max_pix = std::max<int64_t>(max_pix, (int64_t)d.W * d.H);
    const int nv = (int)b->views.size();
    const hipError_t e = (hipError_t)launch_entropy_views(
        b->d_views, nv, max_pix, b->model == DDVR_ABSORPTION ? 1 : 4, p->d_sums,
        p->d_sums + 2 * nv, loss_out, loss_scale, s);
    if (e != hipSuccess) return hip_fail(e, "entropy launch");
  }
  return batch_enqueue(b, PASS_ADJ, 0.0f, nullptr, ws, ws_bytes, s);
}

int ddvr_plan_create(ddvr_batch* b, int32_t loss, float loss_scale, double* loss_out,
                     void* workspace, size_t workspace_bytes, void* hip_stream, ddvr_plan** out) {
  if (!out) return fail(DDVR_ERR_NULL, "out is NULL");
  *out = nullptr;
  if (!b) return fail(DDVR_ERR_NULL, "batch is NULL");
  if (loss != DDVR_PLAN_LOSS_GIVEN && loss != DDVR_PLAN_LOSS_FUSED &&
      loss != DDVR_PLAN_LOSS_NEG_ENTROPY)
    return fail(DDVR_ERR_VALUE, "unknown plan loss %d", loss);
  if (!std::isfinite(loss_scale)) return fail(DDVR_ERR_VALUE, "loss_scale is not finite");
  for (size_t i = 0; i < b->views.size(); ++i) {
    const ViewDesc& d = b->views[i];
    if (loss == DDVR_PLAN_LOSS_FUSED && !d.target)
      return fail(DDVR_ERR_NULL, "view %zu: the fused loss needs a target", i);
    if (loss != DDVR_PLAN_LOSS_FUSED && (!d.d_image || !d.trans))
      return fail(DDVR_ERR_NULL, "view %zu: the adjoint needs d_image and transmittance", i);
    if (loss == DDVR_PLAN_LOSS_NEG_ENTROPY && (int64_t)d.W * d.H < 2)
      return fail(DDVR_ERR_SHAPE, "view %zu: the entropy needs at least 2 pixels", i);
  }
  if (loss == DDVR_PLAN_LOSS_NEG_ENTROPY && b->model == DDVR_COLOR)
    return fail(DDVR_ERR_UNSUPPORTED, "entropy plans take scalar grids");
  size_t need = 0;
  if (b->model != DDVR_COLOR && needs_fallback(b->model, b->flags))
    need = fallback_layout(b->total_rays, b->max_n).bytes;
  if (need && (!workspace || workspace_bytes < need))
    return fail(DDVR_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  int rc = check_pending();
  if (rc) return rc;
  ddvr_plan* p = new (std::nothrow) ddvr_plan;
  if (!p) return fail(DDVR_ERR_VALUE, "out of host memory");
  p->b = b;
  p->loss = loss;
  hipError_t e = hipSuccess;
  if (loss == DDVR_PLAN_LOSS_NEG_ENTROPY)
    e = hipMalloc(&p->d_sums, sizeof(double) * 3 * b->views.size());
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    ddvr_plan_destroy(p);
    return hip_fail(e, "plan buffers");
  }
  // recording runs nothing: the caller's stream is only where replays go
  (void)hip_stream;
  if ((e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess) {
    ddvr_plan_destroy(p);
    return hip_fail(e, "begin capture");
  }
  rc = plan_enqueue(p, loss_scale, loss_out, workspace, workspace_bytes, p->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(p->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    ddvr_plan_destroy(p);
    return rc;
  }
  if (e != hipSuccess) {
    ddvr_plan_destroy(p);
    return hip_fail(e, "end capture");
  }
  p->graph = g;
  if ((e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
    p->exec = nullptr;
    ddvr_plan_destroy(p);
    return hip_fail(e, "graph instantiate");
  }
  *out = p;
  return DDVR_OK;
}

int ddvr_plan_execute(ddvr_plan* p, void* hip_stream) {
  if (!p) return fail(DDVR_ERR_NULL, "plan is NULL");
  int rc = check_pending();
  if (rc) return rc;
  const hipError_t e = hipGraphLaunch(p->exec, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? DDVR_OK : hip_fail(e, "graph launch");
}

int ddvr_plan_loss_terms(const ddvr_plan* p, double* out, int32_t n, void* hip_stream) {
  if (!p || !out) return fail(DDVR_ERR_NULL, "plan or out is NULL");
  if (p->loss != DDVR_PLAN_LOSS_NEG_ENTROPY)
    return fail(DDVR_ERR_UNSUPPORTED, "only entropy plans keep per-view terms");
  const int nv = (int)p->b->views.size();
  if (n != nv) return fail(DDVR_ERR_SHAPE, "the plan has %d views, %d asked", nv, n);
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipMemcpyAsync(out, p->d_sums + 2 * nv, sizeof(double) * nv,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? DDVR_OK : hip_fail(e, "reading the entropy terms");
}

int ddvr_valu_probe(int32_t mode, int32_t blocks, int32_t iters, float* out, int64_t* lane_ops,
                    void* hip_stream) {
  if (!out || !lane_ops) return fail(DDVR_ERR_NULL, "out or lane_ops is NULL");
  if (mode < 0 || mode > 7) return fail(DDVR_ERR_VALUE, "probe mode %d not in 0..7", mode);
  if (blocks <= 0 || blocks > (1 << 20) || iters <= 0)
    return fail(DDVR_ERR_SHAPE, "probe of %d workgroups x %d rounds", blocks, iters);
  int rc;
  if ((rc = check_pending())) return rc;
  const hipError_t e = (hipError_t)launch_valu_probe(mode, blocks, iters, out, hip_stream);
  if (e != hipSuccess) return hip_fail(e, "probe launch");
  // modes 4 to 6 run two instructions per chain and round
  *lane_ops = (int64_t)blocks * 256 * iters * kProbeChains * (mode >= 4 && mode <= 6 ? 2 : 1);
  return DDVR_OK;
}

int ddvr_batch_sample_count(const ddvr_batch* b, int64_t* samples) {
  if (!b || !samples) return fail(DDVR_ERR_NULL, "batch or samples is NULL");
  *samples = b->samples;   // replayed on the host when the batch was built
  return DDVR_OK;
}

}  // extern "C"

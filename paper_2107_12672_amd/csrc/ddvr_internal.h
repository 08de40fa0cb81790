// Internal launch descriptors shared by the host API and the HIP kernels.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace ddvr {

// One view of one grid, as the kernels see it (prepared on the host).
struct ViewDesc {
  // camera frame (Sec. 4.1 f_camera): eye, forward, pre-scaled right / up
  float eye[3], fwd[3], right[3], up[3];
  int32_t W, H;
  float step;             // dt, world units
  // grid (Sec. 3.1): vertex values [nz][ny][nx]
  const void* vol;
  int32_t dtype;          // storage type of vol (ddvr_dtype)
  int32_t nx, ny, nz;
  float h, inv_h;
  float bmin[3], bmax[3];
  float qhi[3];           // largest float below n-1 per axis (grid-unit clamp of positions)
  // transfer function [R][4]
  const float* tf;
  int32_t R;
  // outputs / inputs of the passes
  float* image;           // [H][W][C]
  float* trans;           // [H][W] or null
  const float* d_image;   // adjoint seed, or null
  const float* target;    // fused L2 target, or null
  // gradients (null = not requested)
  float* dV;
  float* dTF;
  float* dcam;            // [12]
  float* dstep;           // [1]
  // tiling
  int32_t tiles_x, tiles_y;
  int32_t slab_k;         // initial samples per slab (adapted per slab in the kernel)
  int32_t pad_;
};

// Per-launch parameters (passed by value as the kernel argument).
struct LaunchParams {
  const ViewDesc* views;  // device array (batched) or null -> use `one`
  ViewDesc one;           // inline descriptor of a single-view launch
  const int32_t* work;    // device list of (view << 20 | tile) items, or null
  int32_t n_items;        // number of tiles in the launch
  int32_t flags;          // adjoint mode | launch flags
  int32_t grad_mask;      // bit 0 dV, 1 dTF, 2 camera, 3 step
  int32_t lds_cap;        // voxels per LDS brick (0 = never stage)
  int32_t lds_two;        // 1: separate brick regions for grid values and gradients
  int32_t slab_kmax;      // longest slab (samples per ray) the adaptive march tries
  int32_t cell_acc;       // 1: density gradient kept in registers per cell
  int32_t lane_map;       // 1: lanes of a wave on every other pixel
  int32_t slab_axis;      // 1: slabs between planes of a grid axis; 0: distance shells
  int32_t xcd_remap;      // 1: contiguous tile ranges per XCD (one tile per workgroup)
  int32_t* queue;         // persistent launch: tile counter (zeroed before the launch)
  float loss_scale;       // fused L2
  double* loss_out;       // fused L2 accumulator or null
  // checkpoint fallback queue (workspace)
  int32_t* fb_count;      // [1] number of queued rays
  int64_t* fb_list;       // [fb_cap] (view << 32 | pixel)
  int64_t fb_cap;
  float fb_tmin;          // T_N threshold below which rays fall back
  int32_t fb_all;         // 1: every hit ray takes the checkpoint path
  float* fb_scratch;      // per-slot scratch for checkpointing
  int32_t fb_slots;       // number of concurrent checkpoint slots
  int32_t fb_slot_floats; // floats per slot
  float* fb_dtf;          // TF gradient every fallback ray that wants one writes (null: none
                          // or several; then each ray adds to its view's dTF directly)
  int32_t fb_tf_R;        // entries of that TF
};

// Forward-mode (tangent) launch: derivatives of the image along up to
// kMaxDirections directions in (camera frame, step) space.
constexpr int kMaxDirections = 4;
struct TangentParams {
  ViewDesc one;           // the view (image / trans / d_image pointers inside)
  int32_t lds_cap;        // voxels per LDS brick (0 = never stage)
  int32_t slab_kmax;
  int32_t ndir;           // 1..kMaxDirections
  float dir[kMaxDirections][13];   // d frame (12: eye, fwd, right, up) and d step
  float* image_dot;       // [ndir][H][W][C] or null (forward-immediate)
  float* d_dir;           // [ndir] += <d_image, image_dot_k> or null (forward-delayed)
};

// Density-from-colour sweep (one voxel per lane).
struct DfcParams {
  const void* cv;         // colour volume [nz][ny][nx][4] (r, g, b, tau), storage dtype
  int32_t nx, ny, nz;
  const float* tf;        // [R][4]
  int32_t R;
  const float* d_prev;    // [nz][ny][nx] previous estimate or null (no neighbour term)
  float* d_out;           // [nz][ny][nx]
  float* cost_out;        // [nz][ny][nx] or null
  uint32_t* n_changed;    // += voxels whose estimate changed, or null
  float alpha, beta;
  uint64_t seed;
  int32_t iter, ncand;
};

enum GradBits { GRAD_V = 1, GRAD_TF = 2, GRAD_CAM = 4, GRAD_STEP = 8 };

enum Pass { PASS_FWD = 0, PASS_ADJ = 1, PASS_FUSED = 2 };

// Host-side launchers implemented in ddvr_kernels.hip.
int launch_render(const LaunchParams& p, int pass, int model, int dtype, int waves, int n_blocks,
                  size_t lds_bytes, void* stream);
int launch_fallback(const LaunchParams& p, int model, int dtype, int fused, void* stream);
int launch_zero_i32(int32_t* ptr, int n, void* stream);
int launch_tangent(const TangentParams& p, int model, int dtype, int n_blocks, size_t lds_bytes,
                   void* stream);
// pre-shaded colour volume (one tile of 16x16 pixels per workgroup, p.n_items tiles):
// slab = 1 the slab-synchronous route (p.lds_cap vertices per brick, lds_bytes of
// dynamic LDS), 0 the direct route (one ray per lane, global atomics)
int launch_color(const LaunchParams& p, int pass, int dtype, int slab, size_t lds_bytes,
                 void* stream);
int launch_cast(const float* src, void* dst, int dtype, int64_t n, void* stream);
// implemented in ddvr_train.hip
int launch_tf_prior(const float* tf, int R, float lam, float* dtf, double* loss, void* stream);
int launch_volume_prior(const float* V, int nx, int ny, int nz, float lam, float* dV,
                        double* loss, void* stream);
int launch_opacity_entropy(const float* img, int64_t n, int stride, int offset, double* work,
                           double* value, float* dimg, float scale, void* stream);
// opacity entropy of every view's alpha (views: device array of nview
// descriptors; image [H][W][channels], alpha the last channel): d_image written,
// oe[v] = OE_v, loss += -scale sum OE_v; sums: 2*nview doubles of scratch
int launch_entropy_views(const ViewDesc* views, int nview, int64_t max_pix, int channels,
                         double* sums, double* oe, double* loss, float scale, void* stream);
int launch_adam(float* x, float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                float eps, float c1, float c2, float lo, float hi, void* store, int store_dtype,
                int zero_grad, void* stream);
int launch_resample(const float* src, int channels, int sx, int sy, int sz, float* dst, int dx,
                    int dy, int dz, void* stream);
// implemented in ddvr_dfc.hip
int launch_density_from_color(const DfcParams& p, int dtype, void* stream);
int launch_color_tau_max(const void* cv, int dtype, int64_t nvox, float* out, void* stream);

// implemented in ddvr_probe.hip: blocks x 256 lanes, iters x kProbeChains
// independent VALU operations per lane (mode 0 float32 FMA, 1 int32 add)
constexpr int kProbeChains = 16;
int launch_valu_probe(int mode, int blocks, int iters, float* out, void* stream);

constexpr int kDtypeDynamic = 3;        // storage type chosen per view; persistent launch
constexpr int kMaxSamples = 1 << 22;    // per-ray sample cap (validated on the host)
constexpr float kFallbackTmin = 7.888609052210118e-31f;   // 2^-100 (T-form inversion)
constexpr float kFallbackTminAlpha = 9.765625e-4f;         // 2^-10 (alpha-form inversion)
constexpr int kFallbackBrick = 4096;   // floats of LDS per wave for the fallback's segment bricks

}  // namespace ddvr

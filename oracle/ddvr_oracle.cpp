// FP64 CPU oracle for differentiable direct volume rendering.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
// calls this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code, header, table or helper with
// the HIP library.
//
// What it computes (Weiss & Westermann, "DiffDVR", arXiv 2107.12672):
//   * Sec. 3.1 / eq. (integral2): emission-absorption along arc-length rays,
//     discretised into N segments with Beer-Lambert opacity
//     alpha_i = 1 - exp(-dt * tau(d_i)) and front-to-back blending.
//   * Sec. 4.1 / Alg. 1 (Direct Volume Rendering Algorithm): f_camera ->
//     x_i = x_o + i*dt*omega -> trilinear f_interpolate -> piecewise-linear
//     f_TF -> f_blend, for i = 0..N-1.
//   * Sec. 4.3 / Alg. 2 (Adjoint Code of the DVR Algorithm) with the blending
//     adjoint of eq. (adj-blend-forward) and the inversion of eq.
//     (inv-blend-forward), Sec. 4.4.
//
// The ground-truth gradient is reverse-mode AD of the discrete forward with a
// stored per-ray tape (the non-inverted adjoint, Sec. 4.4 first paragraph).
// Every other route (T-form inversion, the paper's alpha-form inversion,
// segment checkpointing, the forward-order residual form and forward-mode
// dual numbers, Sec. 4.2) is a cross-variant that must agree with it.
//
// Readings where the paper is silent or garbled:
//   - blending adjoint: the colour-sample adjoint is (1 - alpha^(i)) * Chat
//     (the printed "(C - alpha^(i))" is a typo; it follows from eq.
//     blend-forward); Alg. 2's right-hand side "color_N" is read as
//     color_{i+1}; the camera line is read with hats on [x_o; omega].
//   - dt enters both the positions and the Beer-Lambert exponent; both terms
//     are differentiated.
//   - emission of a segment is premultiplied: c_i = alpha_i * rgb_i.
//   - x_o is the box entry point (t0 = 0 when the eye is inside the box); its
//     dependence on the camera through t0 is differentiated.  N = ceil(L/dt)
//     is piecewise constant and not differentiated.
//   - TF knots at k/(R-1); density clamped to [0,1] before lookup, with the
//     clamp's derivative taken as 1 on the closed interval [0,1].
//   - trilinear cell k = clamp(floor(q), 0, n-2), weights f = q - k.
//   - grid spacing h = 2/(max(n)-1), grid centred at the origin.
//   - camera: pinhole, up = +y, pixel centres, frame (eye, fwd, right*s_x,
//     up*s_y) with s_y = tan(fovy/2), s_x = s_y * W/H.
//   - AO (absorption-only) model: tau(d) = d per world unit, no clamp, rgb=0.
//   - pre-shaded colour volume (Sec. 5.4: the colour volume stores rgb
//     emission and absorption per voxel instead of a density mapped by a TF):
//     grid [nz][ny][nx][4] of (r, g, b, tau), each channel interpolated
//     trilinearly, then the same Beer-Lambert segment and blend as the
//     emission-absorption model.  In the code it is the emission model
//     without a TF (T == nullptr).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <limits>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// --------------------------------------------------------------------------
// Forward-mode dual number with one tangent (Sec. 4.2, the "fvar" idea).
// --------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double v_ = 0.0, double d_ = 0.0) : v(v_), d(d_) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.v * b.d + a.d * b.v); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual sin(Dual a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline Dual cos(Dual a) { return Dual(std::cos(a.v), -std::sin(a.v) * a.d); }
inline Dual tan(Dual a) { double t = std::tan(a.v); return Dual(t, (1.0 + t * t) * a.d); }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::exp; using std::sqrt; using std::sin; using std::cos; using std::tan;

constexpr double kPi = 3.14159265358979323846;

// --------------------------------------------------------------------------
// G1: the vertex grid.
// --------------------------------------------------------------------------
struct Grid {
  int n[3];          // nx, ny, nz
  double h;          // isotropic spacing
  double bmin[3], bmax[3];
};

Grid make_grid(int nx, int ny, int nz) {
  Grid g;
  g.n[0] = nx; g.n[1] = ny; g.n[2] = nz;
  int nmax = std::max(nx, std::max(ny, nz));
  g.h = 2.0 / double(nmax - 1);
  for (int a = 0; a < 3; ++a) {
    g.bmin[a] = -0.5 * double(g.n[a] - 1) * g.h;
    g.bmax[a] = 0.5 * double(g.n[a] - 1) * g.h;
  }
  return g;
}

inline int64_t vidx(const Grid& g, int x, int y, int z) {
  return (int64_t(z) * g.n[1] + y) * g.n[0] + x;
}

// --------------------------------------------------------------------------
// G2: camera frame from a pose on the enclosing sphere (Sec. 5.1: camera on a
// sphere facing the centre, longitude/latitude parameterisation).
// frame = [eye(3), fwd(3), right*s_x(3), up*s_y(3)].
// --------------------------------------------------------------------------
template <class S>
void camera_from_sphere(S yaw, S pitch, S dist, S fovy, int W, int H, S* f) {
  S e0 = dist * cos(pitch) * cos(yaw);
  S e1 = dist * sin(pitch);
  S e2 = dist * cos(pitch) * sin(yaw);
  S len = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  S F0 = -e0 / len, F1 = -e1 / len, F2 = -e2 / len;
  // right = normalize(F x (0,1,0)) = normalize((-F2, 0, F0))
  S rl = sqrt(F2 * F2 + F0 * F0);
  S R0 = -F2 / rl, R1 = S(0.0), R2 = F0 / rl;
  // up = right x F
  S U0 = R1 * F2 - R2 * F1;
  S U1 = R2 * F0 - R0 * F2;
  S U2 = R0 * F1 - R1 * F0;
  S sy = tan(fovy * S(0.5));
  S sx = sy * S(double(W) / double(H));
  f[0] = e0; f[1] = e1; f[2] = e2;
  f[3] = F0; f[4] = F1; f[5] = F2;
  f[6] = R0 * sx; f[7] = R1 * sx; f[8] = R2 * sx;
  f[9] = U0 * sy; f[10] = U1 * sy; f[11] = U2 * sy;
}

// --------------------------------------------------------------------------
// G2-G3: per-pixel ray and box clip (f_camera in Alg. 1).
// --------------------------------------------------------------------------
template <class S>
struct Ray {
  bool hit = false;
  double u = 0, v = 0;       // pixel-plane coordinates in [-1,1]
  S w[3];                    // un-normalised direction F + u*R + v*U
  S wlen;                    // |w|
  S omega[3];                // unit direction
  S t0;                      // entry distance (0 if the eye is inside)
  int entry_axis = -1;       // axis whose slab plane defines t0 (-1: t0 = 0)
  S xo[3];                   // entry point e + t0*omega
  int N = 0;                 // number of samples ceil(L/dt)
  double ratio = 0.0;        // L/dt (for tie detection in parity tests)
};

template <class S>
Ray<S> make_ray(const S* cam, int px, int py, int W, int H, const Grid& g, S dt) {
  Ray<S> r;
  r.u = 2.0 * (double(px) + 0.5) / double(W) - 1.0;
  r.v = 1.0 - 2.0 * (double(py) + 0.5) / double(H);
  for (int a = 0; a < 3; ++a) r.w[a] = cam[3 + a] + S(r.u) * cam[6 + a] + S(r.v) * cam[9 + a];
  r.wlen = sqrt(r.w[0] * r.w[0] + r.w[1] * r.w[1] + r.w[2] * r.w[2]);
  for (int a = 0; a < 3; ++a) r.omega[a] = r.w[a] / r.wlen;
  // slab method
  double tnear = -std::numeric_limits<double>::infinity();
  double tfar = std::numeric_limits<double>::infinity();
  int near_axis = -1;
  S tnear_s = S(0.0);
  for (int a = 0; a < 3; ++a) {
    double e = val(cam[a]);
    double o = val(r.omega[a]);
    if (o == 0.0) {
      if (e < g.bmin[a] || e > g.bmax[a]) return r;   // parallel and outside
      continue;
    }
    double ta = (g.bmin[a] - e) / o, tb = (g.bmax[a] - e) / o;
    double b_near = ta < tb ? g.bmin[a] : g.bmax[a];
    double tn = std::min(ta, tb), tf = std::max(ta, tb);
    if (tn > tnear) {
      tnear = tn; near_axis = a;
      tnear_s = (S(b_near) - cam[a]) / r.omega[a];
    }
    if (tf < tfar) tfar = tf;
  }
  double t0 = tnear > 0.0 ? tnear : 0.0;
  if (!(tfar > t0)) return r;   // miss
  r.hit = true;
  if (tnear > 0.0) { r.t0 = tnear_s; r.entry_axis = near_axis; }
  else { r.t0 = S(0.0); r.entry_axis = -1; }
  double L = tfar - t0;
  r.ratio = L / val(dt);
  r.N = int(std::ceil(r.ratio));
  for (int a = 0; a < 3; ++a) r.xo[a] = cam[a] + r.t0 * r.omega[a];
  return r;
}

// --------------------------------------------------------------------------
// G5: trilinear interpolation (f_interpolate, Sec. 3.1 vertex grid).
// --------------------------------------------------------------------------
template <class S>
struct Cell {
  int k[3];
  S f[3];
};

template <class S>
Cell<S> locate(const Grid& g, const S* x) {
  Cell<S> c;
  for (int a = 0; a < 3; ++a) {
    S q = (x[a] - S(g.bmin[a])) / S(g.h);
    int k = int(std::floor(val(q)));
    k = std::min(std::max(k, 0), g.n[a] - 2);
    c.k[a] = k;
    c.f[a] = q - S(double(k));
  }
  return c;
}

template <class S, class VS>
S trilinear(const Grid& g, const VS* V, const Cell<S>& c) {
  S d = S(0.0);
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        S w = (cx ? c.f[0] : S(1.0) - c.f[0]) * (cy ? c.f[1] : S(1.0) - c.f[1]) *
              (cz ? c.f[2] : S(1.0) - c.f[2]);
        d = d + w * S(V[vidx(g, c.k[0] + cx, c.k[1] + cy, c.k[2] + cz)]);
      }
  return d;
}

// Channel ch of a grid of 4-vectors [nz][ny][nx][4] (the colour volume).
template <class S, class VS>
S trilinear_ch(const Grid& g, const VS* V4, const Cell<S>& c, int ch) {
  S d = S(0.0);
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        S w = (cx ? c.f[0] : S(1.0) - c.f[0]) * (cy ? c.f[1] : S(1.0) - c.f[1]) *
              (cz ? c.f[2] : S(1.0) - c.f[2]);
        d = d + w * S(V4[4 * vidx(g, c.k[0] + cx, c.k[1] + cy, c.k[2] + cz) + ch]);
      }
  return d;
}

// --------------------------------------------------------------------------
// G6: piecewise-linear TF (f_TF), R regularly spaced knots at k/(R-1).
// --------------------------------------------------------------------------
template <class S>
struct TFSample {
  S rgb[3];
  S tau;
  int j = 0;
  S phi;
  bool inside = true;   // 0 <= d <= 1 (clamp derivative is 1)
};

template <class S, class TS>
TFSample<S> tf_lookup(S d, const TS* T, int R) {
  TFSample<S> s;
  S dc = d;
  if (val(d) < 0.0) { dc = S(0.0); s.inside = false; }
  else if (val(d) > 1.0) { dc = S(1.0); s.inside = false; }
  S u = dc * S(double(R - 1));
  int j = std::min(int(std::floor(val(u))), R - 2);
  j = std::max(j, 0);
  s.j = j;
  s.phi = u - S(double(j));
  for (int ch = 0; ch < 3; ++ch)
    s.rgb[ch] = (S(1.0) - s.phi) * S(T[4 * j + ch]) + s.phi * S(T[4 * (j + 1) + ch]);
  s.tau = (S(1.0) - s.phi) * S(T[4 * j + 3]) + s.phi * S(T[4 * (j + 1) + 3]);
  return s;
}

// --------------------------------------------------------------------------
// One sample of Alg. 1: position, density, TF, Beer-Lambert factor.
// --------------------------------------------------------------------------
template <class S>
struct Sample {
  S x[3];
  Cell<S> cell;
  S d;
  TFSample<S> tf;
  S e;        // exp(-dt*tau)
  S alpha;    // 1 - e
  S c[3];     // premultiplied emission alpha*rgb
};

template <class S, class VS, class TS>
Sample<S> eval_sample(const Grid& g, const VS* V, const TS* T, int R, bool ea,
                      const Ray<S>& r, S dt, int i) {
  Sample<S> s;
  for (int a = 0; a < 3; ++a) s.x[a] = r.xo[a] + S(double(i)) * dt * r.omega[a];
  s.cell = locate(g, s.x);
  if (ea && !T) {
    // colour volume: (r, g, b, tau) interpolated per channel, no TF
    for (int ch = 0; ch < 3; ++ch) s.tf.rgb[ch] = trilinear_ch(g, V, s.cell, ch);
    s.tf.tau = trilinear_ch(g, V, s.cell, 3);
    s.d = s.tf.tau;
  } else if (ea) {
    s.d = trilinear(g, V, s.cell);
    s.tf = tf_lookup(s.d, T, R);
  } else {
    s.d = trilinear(g, V, s.cell);
    s.tf.rgb[0] = s.tf.rgb[1] = s.tf.rgb[2] = S(0.0);
    s.tf.tau = s.d;
  }
  s.e = exp(-(dt * s.tf.tau));
  s.alpha = S(1.0) - s.e;
  for (int ch = 0; ch < 3; ++ch) s.c[ch] = s.alpha * s.tf.rgb[ch];
  return s;
}

// --------------------------------------------------------------------------
// Full forward for one ray (G7-G9): returns (C_N, T_N).
// --------------------------------------------------------------------------
template <class S, class VS, class TS>
void march(const Grid& g, const VS* V, const TS* T, int R, bool ea, const Ray<S>& r,
           S dt, S* C, S& Tr) {
  C[0] = C[1] = C[2] = S(0.0);
  Tr = S(1.0);
  for (int i = 0; i < r.N; ++i) {
    Sample<S> s = eval_sample(g, V, T, R, ea, r, dt, i);
    for (int ch = 0; ch < 3; ++ch) C[ch] = C[ch] + Tr * s.c[ch];
    Tr = Tr * s.e;
  }
}

// --------------------------------------------------------------------------
// Adjoint machinery (Alg. 2).  Accumulators of one thread.
// --------------------------------------------------------------------------
struct GradAcc {
  std::vector<double> dV, dTF;
  double dcam[12];
  double dstep;
  bool want_dV = true;
  void init(size_t nv, size_t ntf, bool with_dV) {
    want_dV = with_dV;
    dV.assign(with_dV ? nv : 0, 0.0); dTF.assign(ntf, 0.0);
    std::fill(dcam, dcam + 12, 0.0); dstep = 0.0;
  }
};

enum Variant { TAPE = 0, INV_T = 1, INV_ALPHA = 2, CHECKPOINT = 3, RESIDUAL = 4 };

// Per-sample adjoint below the blend: given tau_hat and rgb_hat of sample i,
// propagate through f_TF, f_interpolate and the position x_i (Alg. 2, the
// three lines after the blending line).  Accumulates into acc, xo_hat,
// om_hat and the step adjoint.
void adjoint_below_blend(const Grid& g, const double* V, const double* T, int R, bool ea,
                         const Ray<double>& r, double dt, int i, const Sample<double>& s,
                         double tau_hat, const double* rgb_hat, GradAcc& acc,
                         double* xo_hat, double* om_hat) {
  if (ea && !T) {
    // colour volume: every channel's value adjoint goes to its own grid
    const double g4[4] = {rgb_hat[0], rgb_hat[1], rgb_hat[2], tau_hat};
    const Cell<double>& c = s.cell;
    double dd_df[3] = {0.0, 0.0, 0.0};
    for (int cz = 0; cz < 2; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          double wx = cx ? c.f[0] : 1.0 - c.f[0];
          double wy = cy ? c.f[1] : 1.0 - c.f[1];
          double wz = cz ? c.f[2] : 1.0 - c.f[2];
          int64_t id = vidx(g, c.k[0] + cx, c.k[1] + cy, c.k[2] + cz);
          for (int ch = 0; ch < 4; ++ch) {
            if (acc.want_dV) acc.dV[4 * id + ch] += wx * wy * wz * g4[ch];
            double v = g4[ch] * V[4 * id + ch];
            dd_df[0] += (cx ? 1.0 : -1.0) * wy * wz * v;
            dd_df[1] += wx * (cy ? 1.0 : -1.0) * wz * v;
            dd_df[2] += wx * wy * (cz ? 1.0 : -1.0) * v;
          }
        }
    double om_dot = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double xh = dd_df[a] / g.h;
      xo_hat[a] += xh;
      om_hat[a] += double(i) * dt * xh;
      om_dot += r.omega[a] * xh;
    }
    acc.dstep += double(i) * om_dot;
    return;
  }
  // f_TF adjoint
  double d_hat;
  if (ea) {
    const int j = s.tf.j;
    const double phi = s.tf.phi;
    double g4[4] = {rgb_hat[0], rgb_hat[1], rgb_hat[2], tau_hat};
    double u_hat = 0.0;
    for (int ch = 0; ch < 4; ++ch) {
      acc.dTF[4 * j + ch] += (1.0 - phi) * g4[ch];
      acc.dTF[4 * (j + 1) + ch] += phi * g4[ch];
      u_hat += (T[4 * (j + 1) + ch] - T[4 * j + ch]) * g4[ch];
    }
    d_hat = s.tf.inside ? double(R - 1) * u_hat : 0.0;
  } else {
    d_hat = tau_hat;
  }
  // f_interpolate adjoint: V_hat and x_hat
  const Cell<double>& c = s.cell;
  double dd_df[3] = {0.0, 0.0, 0.0};
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        double wx = cx ? c.f[0] : 1.0 - c.f[0];
        double wy = cy ? c.f[1] : 1.0 - c.f[1];
        double wz = cz ? c.f[2] : 1.0 - c.f[2];
        int64_t id = vidx(g, c.k[0] + cx, c.k[1] + cy, c.k[2] + cz);
        if (acc.want_dV) acc.dV[id] += wx * wy * wz * d_hat;
        double v = V[id];
        dd_df[0] += (cx ? 1.0 : -1.0) * wy * wz * v;
        dd_df[1] += wx * (cy ? 1.0 : -1.0) * wz * v;
        dd_df[2] += wx * wy * (cz ? 1.0 : -1.0) * v;
      }
  double x_hat[3];
  for (int a = 0; a < 3; ++a) x_hat[a] = d_hat * dd_df[a] / g.h;
  // position x_i = x_o + i*dt*omega
  double om_dot = 0.0;
  for (int a = 0; a < 3; ++a) {
    xo_hat[a] += x_hat[a];
    om_hat[a] += double(i) * dt * x_hat[a];
    om_dot += r.omega[a] * x_hat[a];
  }
  acc.dstep += double(i) * om_dot;
}

// Blending + Beer-Lambert adjoint of sample i (eq. adj-blend-forward, with the
// reading of the colour term stated above), written with T = 1 - alpha.
// Inputs: Ti = T^(i), ahat_next = alpha_hat^(i+1); Chat constant along the ray.
// Returns alpha_hat^(i) and fills tau_hat, rgb_hat; adds the Beer-Lambert step
// term into acc.dstep.
double adjoint_blend(const Sample<double>& s, double Ti, double ahat_next, const double* Chat,
                     double dt, bool ea, double& tau_hat, double* rgb_hat, GradAcc& acc) {
  double chat[3], alpha_s_hat = Ti * ahat_next;   // adjoint of the sample opacity
  for (int ch = 0; ch < 3; ++ch) {
    chat[ch] = Ti * Chat[ch];                      // adjoint of the sample colour c_i
    if (ea) alpha_s_hat += s.tf.rgb[ch] * chat[ch];  // c_i = alpha_i * rgb_i
    rgb_hat[ch] = s.alpha * chat[ch];
  }
  double ahat_prev = s.e * ahat_next;
  if (ea) for (int ch = 0; ch < 3; ++ch) ahat_prev -= s.c[ch] * Chat[ch];
  // alpha_i = 1 - exp(-dt*tau)
  tau_hat = alpha_s_hat * dt * s.e;
  acc.dstep += alpha_s_hat * s.tf.tau * s.e;
  return ahat_prev;
}

// Camera adjoint (last line of Alg. 2, read as acting on [x_o_hat; omega_hat]):
// x_o = e + t0*omega, t0 from the entry slab plane, omega = w/|w|,
// w = F + u*R + v*U.
void adjoint_camera(const Ray<double>& r, const double* cam, const double* xo_hat,
                    const double* om_hat_in, double* dcam) {
  double om_hat[3] = {om_hat_in[0], om_hat_in[1], om_hat_in[2]};
  double t0_hat = 0.0;
  for (int a = 0; a < 3; ++a) {
    dcam[a] += xo_hat[a];
    om_hat[a] += r.t0 * xo_hat[a];
    t0_hat += r.omega[a] * xo_hat[a];
  }
  if (r.entry_axis >= 0) {
    // t0 = (b - e_a)/omega_a
    const int a = r.entry_axis;
    dcam[a] += -t0_hat / r.omega[a];
    om_hat[a] += -t0_hat * r.t0 / r.omega[a];
  }
  double od = r.omega[0] * om_hat[0] + r.omega[1] * om_hat[1] + r.omega[2] * om_hat[2];
  for (int a = 0; a < 3; ++a) {
    double w_hat = (om_hat[a] - r.omega[a] * od) / r.wlen;
    dcam[3 + a] += w_hat;
    dcam[6 + a] += r.u * w_hat;
    dcam[9 + a] += r.v * w_hat;
  }
  (void)cam;
}

// Whole adjoint of one ray.  gimg: [4] (EA: r,g,b,alpha) or [1] (AO: alpha).
void adjoint_ray(const Grid& g, const double* V, const double* T, int R, bool ea,
                 const double* cam, const Ray<double>& r, double dt, const double* gimg,
                 int variant, int ckK, GradAcc& acc) {
  if (!r.hit || r.N <= 0) return;
  const int N = r.N;
  double Chat[3] = {0.0, 0.0, 0.0};
  double ghat_alpha;
  if (ea) { Chat[0] = gimg[0]; Chat[1] = gimg[1]; Chat[2] = gimg[2]; ghat_alpha = gimg[3]; }
  else ghat_alpha = gimg[0];
  double xo_hat[3] = {0, 0, 0}, om_hat[3] = {0, 0, 0};
  double tau_hat, rgb_hat[3];

  if (variant == RESIDUAL) {
    // Forward-order route: alpha_hat^(i+1) * T^(i+1) = g_a*T_N - (C_N - C^(i+1)).Chat
    double CN[3], TN;
    march(g, V, T, R, ea, r, dt, CN, TN);
    double C[3] = {0, 0, 0}, Tr = 1.0;
    for (int i = 0; i < N; ++i) {
      Sample<double> s = eval_sample(g, V, T, R, ea, r, dt, i);
      double Ti = Tr;
      for (int ch = 0; ch < 3; ++ch) C[ch] += Ti * s.c[ch];
      Tr = Ti * s.e;
      double resid = ghat_alpha * TN;
      for (int ch = 0; ch < 3; ++ch) resid -= (CN[ch] - C[ch]) * Chat[ch];
      double rgbdot = 0.0;
      if (ea) for (int ch = 0; ch < 3; ++ch) rgbdot += s.tf.rgb[ch] * Chat[ch];
      // alpha_s_hat * e_i = T^(i+1)*(alpha_hat^(i+1) + rgb.Chat)
      double ase = resid + Tr * rgbdot;
      tau_hat = ase * dt;
      acc.dstep += ase * s.tf.tau;
      for (int ch = 0; ch < 3; ++ch) rgb_hat[ch] = s.alpha * Ti * Chat[ch];
      adjoint_below_blend(g, V, T, R, ea, r, dt, i, s, tau_hat, rgb_hat, acc, xo_hat, om_hat);
    }
    adjoint_camera(r, cam, xo_hat, om_hat, acc.dcam);
    return;
  }

  if (variant == CHECKPOINT) {
    // Segment checkpointing: keep T at every K-th sample, re-march each segment.
    const int K = ckK > 0 ? ckK : std::max(1, int(std::ceil(std::sqrt(double(N)))));
    const int nseg = (N + K - 1) / K;
    std::vector<double> Tck(nseg);
    double Tr = 1.0;
    for (int i = 0; i < N; ++i) {
      if (i % K == 0) Tck[i / K] = Tr;
      Sample<double> s = eval_sample(g, V, T, R, ea, r, dt, i);
      Tr = Tr * s.e;
    }
    double ahat = ghat_alpha;
    std::vector<double> Tseg(K + 1);
    for (int sg = nseg - 1; sg >= 0; --sg) {
      const int i0 = sg * K, i1 = std::min(N, i0 + K);
      Tseg[0] = Tck[sg];
      for (int i = i0; i < i1; ++i) {
        Sample<double> s = eval_sample(g, V, T, R, ea, r, dt, i);
        Tseg[i - i0 + 1] = Tseg[i - i0] * s.e;
      }
      for (int i = i1 - 1; i >= i0; --i) {
        Sample<double> s = eval_sample(g, V, T, R, ea, r, dt, i);
        ahat = adjoint_blend(s, Tseg[i - i0], ahat, Chat, dt, ea, tau_hat, rgb_hat, acc);
        adjoint_below_blend(g, V, T, R, ea, r, dt, i, s, tau_hat, rgb_hat, acc, xo_hat, om_hat);
      }
    }
    adjoint_camera(r, cam, xo_hat, om_hat, acc.dcam);
    return;
  }

  // TAPE / inversion variants: one forward march (the tape stores T^(i)).
  std::vector<double> tape;
  double Tcur;
  {
    double Tr = 1.0;
    if (variant == TAPE) { tape.resize(N + 1); tape[0] = 1.0; }
    for (int i = 0; i < N; ++i) {
      Sample<double> s = eval_sample(g, V, T, R, ea, r, dt, i);
      Tr = Tr * s.e;
      if (variant == TAPE) tape[i + 1] = Tr;
    }
    Tcur = Tr;   // T^(N): the only state the inversion keeps
  }
  double ahat = ghat_alpha;
  double acur = 1.0 - Tcur;   // alpha^(N) for the alpha-form
  for (int i = N - 1; i >= 0; --i) {
    Sample<double> s = eval_sample(g, V, T, R, ea, r, dt, i);
    double Ti;
    if (variant == TAPE) {
      Ti = tape[i];
    } else if (variant == INV_T) {
      Ti = Tcur / s.e;          // invert T^(i+1) = T^(i) * e_i
      Tcur = Ti;
    } else {                    // INV_ALPHA: eq. (inv-blend-forward)
      double a_prev = (s.alpha - acur) / (s.alpha - 1.0);
      acur = a_prev;
      Ti = 1.0 - a_prev;
    }
    ahat = adjoint_blend(s, Ti, ahat, Chat, dt, ea, tau_hat, rgb_hat, acc);
    adjoint_below_blend(g, V, T, R, ea, r, dt, i, s, tau_hat, rgb_hat, acc, xo_hat, om_hat);
  }
  adjoint_camera(r, cam, xo_hat, om_hat, acc.dcam);
}

int nthreads_max() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
int thread_id() {
#ifdef _OPENMP
  return omp_get_thread_num();
#else
  return 0;
#endif
}

bool check_common(int nx, int ny, int nz, int R, bool ea, int W, int H, double step) {
  if (nx < 2 || ny < 2 || nz < 2) return false;
  if (ea && R < 2) return false;
  if (W <= 0 || H <= 0) return false;
  if (!(step > 0.0) || !std::isfinite(step)) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// Density from colour (Sec. 5.4, second stage of the reconstruction
// pipeline): for every voxel, candidate densities drawn uniformly at random,
// each mapped through the TF, and the candidate of least cost
//   C(d) = ||C_T - C(d)||^2 + alpha log(1 + |tau_T - tau(d)|)
//          + beta sum over the 6-neighbourhood (d - d_i)^2
// kept.  (C_T, tau_T) is the voxel's entry of the colour volume; the
// neighbours d_i are those of the previous estimate (none in the first
// iteration), grid neighbours outside the volume are absent.  Ties keep the
// lowest candidate index.
//
// Candidates come from a counter-based generator: SplitMix64 (Steele, Lea and
// Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
// whose n-th output for seed s is mix(s + (n + 1) * gamma), gamma =
// 0x9e3779b97f4a7c15, with the variant-13 finaliser mix(z): z ^= z >> 30,
// z *= 0xbf58476d1ce4e5b9, z ^= z >> 27, z *= 0x94d049bb133111eb,
// z ^= z >> 31.  Candidate k of voxel v in iteration t is output n =
// (t * nvox + v) * ncand + k, mapped to [0, 1) as (x >> 40) * 2^-24.
// ---------------------------------------------------------------------------
static inline uint64_t splitmix_output(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9e3779b97f4a7c15ull;
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

static inline double candidate_density(uint64_t seed, uint64_t n) {
  return (double)(splitmix_output(seed, n) >> 40) * (1.0 / 16777216.0);
}

extern "C" {

// Camera frame (12 doubles) from yaw/pitch/dist/fovy in RADIANS.
int oracle_camera_from_sphere(double yaw, double pitch, double dist, double fovy, int W, int H,
                              double* frame) {
  if (!frame || W <= 0 || H <= 0) return -1;
  camera_from_sphere<double>(yaw, pitch, dist, fovy, W, H, frame);
  return 0;
}

// d frame / d (yaw, pitch, dist, fovy): jac[p*12 + k], by dual numbers.
int oracle_camera_jacobian(double yaw, double pitch, double dist, double fovy, int W, int H,
                           double* jac) {
  if (!jac || W <= 0 || H <= 0) return -1;
  for (int p = 0; p < 4; ++p) {
    Dual a(yaw, p == 0), b(pitch, p == 1), c(dist, p == 2), d(fovy, p == 3);
    Dual f[12];
    camera_from_sphere<Dual>(a, b, c, d, W, H, f);
    for (int k = 0; k < 12; ++k) jac[p * 12 + k] = f[k].d;
  }
  return 0;
}

// Forward render of the pixels listed in pix (or all W*H pixels, row-major,
// when pix == NULL).  model: 0 = absorption-only (1 channel: alpha),
// 1 = emission-absorption (4 channels: premultiplied r,g,b and alpha).
// Outputs (each may be NULL): image[npix*C], trans[npix] = T_N,
// nsamp[npix] = N, ratio[npix] = L/dt (0 for rays that miss).
int oracle_render(const double* V, int nx, int ny, int nz, const double* tf, int R,
                  const double* cam, int W, int H, double step, int model,
                  const int32_t* pix, int64_t npix, double* image, double* trans,
                  int32_t* nsamp, double* ratio) {
  if (model < 0 || model > 2) return -3;
  const bool ea = model >= 1;                 // emission: TF model or colour volume
  if (model == 2) tf = nullptr;
  if (!V || !cam || (model == 1 && !tf)) return -1;
  if (!check_common(nx, ny, nz, R, model == 1, W, H, step)) return -2;
  const Grid g = make_grid(nx, ny, nz);
  const int64_t n = pix ? npix : int64_t(W) * H;
  const int C = ea ? 4 : 1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < n; ++q) {
    const int64_t p = pix ? int64_t(pix[q]) : q;
    const int px = int(p % W), py = int(p / W);
    Ray<double> r = make_ray<double>(cam, px, py, W, H, g, step);
    double Cc[3] = {0, 0, 0}, Tr = 1.0;
    if (r.hit) march(g, V, tf, R, ea, r, step, Cc, Tr);
    if (image) {
      if (ea) { image[q * 4 + 0] = Cc[0]; image[q * 4 + 1] = Cc[1]; image[q * 4 + 2] = Cc[2];
                image[q * 4 + 3] = 1.0 - Tr; }
      else image[q * C] = 1.0 - Tr;
    }
    if (trans) trans[q] = Tr;
    if (nsamp) nsamp[q] = r.hit ? r.N : 0;
    if (ratio) ratio[q] = r.hit ? r.ratio : 0.0;
  }
  return 0;
}

// Adjoint: gradients of sum(d_image * image) w.r.t. V, TF, camera frame and
// step, ACCUMULATED (+=) into the given arrays (each may be NULL).
// d_image is indexed like the image of oracle_render (npix entries).
// variant: 0 stored tape (ground truth), 1 T-form inversion, 2 the paper's
// alpha-form inversion, 3 segment checkpointing (segment length ck_K, 0 =
// ceil(sqrt N)), 4 forward-order residual form.
int oracle_adjoint(const double* V, int nx, int ny, int nz, const double* tf, int R,
                   const double* cam, int W, int H, double step, int model,
                   const int32_t* pix, int64_t npix, const double* d_image, int variant,
                   int ck_K, double* dV, double* dTF, double* dcam, double* dstep) {
  if (model < 0 || model > 2) return -3;
  const bool ea = model >= 1;
  if (model == 2) { tf = nullptr; dTF = nullptr; }
  if (!V || !cam || !d_image || (model == 1 && !tf)) return -1;
  if (!check_common(nx, ny, nz, R, model == 1, W, H, step)) return -2;
  if (variant < 0 || variant > 4) return -3;
  const Grid g = make_grid(nx, ny, nz);
  const int64_t n = pix ? npix : int64_t(W) * H;
  const int C = ea ? 4 : 1;
  const size_t nv = size_t(nx) * ny * nz * (model == 2 ? 4 : 1);
  const size_t ntf = model == 1 ? size_t(R) * 4 : 0;
  // one float64 gradient copy per thread; bound their total to ~2 GiB so that
  // sparse pixel sets on large grids stay cheap
  int nt = nthreads_max();
  const double copy_bytes = 8.0 * double((dV ? nv : 0) + ntf) + 1.0;
  nt = std::max(1, std::min(nt, int((2.0 * (1 << 30)) / copy_bytes)));
  nt = int(std::max<int64_t>(1, std::min<int64_t>(nt, (n + 63) / 64)));
  std::vector<GradAcc> accs(nt);
#pragma omp parallel num_threads(nt)
  {
    GradAcc& acc = accs[thread_id()];
    acc.init(nv, ntf, dV != nullptr);
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; ++q) {
      const int64_t p = pix ? int64_t(pix[q]) : q;
      const int px = int(p % W), py = int(p / W);
      Ray<double> r = make_ray<double>(cam, px, py, W, H, g, step);
      adjoint_ray(g, V, tf, R, ea, cam, r, step, d_image + q * C, variant, ck_K, acc);
    }
  }
  for (int t = 0; t < nt; ++t) {
    if (dV) for (size_t k = 0; k < nv; ++k) dV[k] += accs[t].dV[k];
    if (dTF) for (size_t k = 0; k < ntf; ++k) dTF[k] += accs[t].dTF[k];
    if (dcam) for (int k = 0; k < 12; ++k) dcam[k] += accs[t].dcam[k];
    if (dstep) *dstep += accs[t].dstep;
  }
  return 0;
}

// Forward-mode (one tangent direction) render: image and its directional
// derivative along (V_dir, tf_dir, cam_dir, step_dir).  Directions may be
// NULL (= zero).  Outputs as oracle_render, plus image_dot / trans_dot.
int oracle_render_dual(const double* V, const double* V_dir, int nx, int ny, int nz,
                       const double* tf, const double* tf_dir, int R, const double* cam,
                       const double* cam_dir, int W, int H, double step, double step_dir,
                       int model, const int32_t* pix, int64_t npix, double* image,
                       double* image_dot, double* trans, double* trans_dot) {
  if (model < 0 || model > 2) return -3;
  const bool ea = model >= 1;
  if (model == 2) { tf = nullptr; tf_dir = nullptr; }
  if (!V || !cam || (model == 1 && !tf)) return -1;
  if (!check_common(nx, ny, nz, R, model == 1, W, H, step)) return -2;
  const Grid g = make_grid(nx, ny, nz);
  const size_t nv = size_t(nx) * ny * nz * (model == 2 ? 4 : 1);
  std::vector<Dual> Vd(nv), Td(model == 1 ? size_t(R) * 4 : 0);
  for (size_t k = 0; k < nv; ++k) Vd[k] = Dual(V[k], V_dir ? V_dir[k] : 0.0);
  for (size_t k = 0; k < Td.size(); ++k) Td[k] = Dual(tf[k], tf_dir ? tf_dir[k] : 0.0);
  Dual camd[12];
  for (int k = 0; k < 12; ++k) camd[k] = Dual(cam[k], cam_dir ? cam_dir[k] : 0.0);
  const Dual dt(step, step_dir);
  const int64_t n = pix ? npix : int64_t(W) * H;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n; ++q) {
    const int64_t p = pix ? int64_t(pix[q]) : q;
    const int px = int(p % W), py = int(p / W);
    Ray<Dual> r = make_ray<Dual>(camd, px, py, W, H, g, dt);
    Dual Cc[3] = {Dual(0), Dual(0), Dual(0)}, Tr(1.0);
    if (r.hit)
      march(g, Vd.data(), model == 2 ? static_cast<const Dual*>(nullptr) : Td.data(), R, ea, r,
            dt, Cc, Tr);
    if (ea) {
      for (int ch = 0; ch < 3; ++ch) {
        if (image) image[q * 4 + ch] = Cc[ch].v;
        if (image_dot) image_dot[q * 4 + ch] = Cc[ch].d;
      }
      if (image) image[q * 4 + 3] = 1.0 - Tr.v;
      if (image_dot) image_dot[q * 4 + 3] = -Tr.d;
    } else {
      if (image) image[q] = 1.0 - Tr.v;
      if (image_dot) image_dot[q] = -Tr.d;
    }
    if (trans) trans[q] = Tr.v;
    if (trans_dot) trans_dot[q] = Tr.d;
  }
  return 0;
}

// Single-point helpers exposed for the pin tests.
int oracle_trilinear(const double* V, int nx, int ny, int nz, const double* x, double* d) {
  if (!V || !x || !d || nx < 2 || ny < 2 || nz < 2) return -1;
  const Grid g = make_grid(nx, ny, nz);
  Cell<double> c = locate(g, x);
  *d = trilinear(g, V, c);
  return 0;
}

int oracle_tf_lookup(const double* tf, int R, double d, double* out4) {
  if (!tf || !out4 || R < 2) return -1;
  TFSample<double> s = tf_lookup(d, tf, R);
  out4[0] = s.rgb[0]; out4[1] = s.rgb[1]; out4[2] = s.rgb[2]; out4[3] = s.tau;
  return 0;
}

// Ray setup of one pixel: out[0..2] = x_o, out[3..5] = omega, out[6] = t0,
// out[7] = L/dt; returns N (0 for a miss) or <0 on error.
int oracle_ray(const double* cam, int nx, int ny, int nz, int W, int H, int px, int py,
               double step, double* out) {
  if (!cam || !out || nx < 2 || ny < 2 || nz < 2 || W <= 0 || H <= 0 || !(step > 0)) return -1;
  const Grid g = make_grid(nx, ny, nz);
  Ray<double> r = make_ray<double>(cam, px, py, W, H, g, step);
  for (int a = 0; a < 3; ++a) { out[a] = r.hit ? r.xo[a] : 0.0; out[3 + a] = r.omega[a]; }
  out[6] = r.hit ? r.t0 : 0.0;
  out[7] = r.hit ? r.ratio : 0.0;
  return r.hit ? r.N : 0;
}

// Per-sample trace of one pixel's ray (for invariant tests): for i < N and
// i < cap, d[i] = density, tau[i] = absorption, Tb[i] = T^(i) (transmittance
// before sample i), x[3i..3i+2] = position.  Returns N (0 for a miss).
int oracle_trace_ray(const double* V, int nx, int ny, int nz, const double* tf, int R,
                     const double* cam, int W, int H, int px, int py, double step, int model,
                     int cap, double* d, double* tau, double* Tb, double* x) {
  const bool ea = model == 1;
  if (!V || !cam || (ea && !tf)) return -1;
  if (!check_common(nx, ny, nz, R, ea, W, H, step)) return -2;
  const Grid g = make_grid(nx, ny, nz);
  Ray<double> r = make_ray<double>(cam, px, py, W, H, g, step);
  if (!r.hit) return 0;
  double Tr = 1.0;
  for (int i = 0; i < r.N && i < cap; ++i) {
    Sample<double> s = eval_sample(g, V, tf, R, ea, r, step, i);
    if (d) d[i] = s.d;
    if (tau) tau[i] = s.tf.tau;
    if (Tb) Tb[i] = Tr;
    if (x) for (int a = 0; a < 3; ++a) x[3 * i + a] = s.x[a];
    Tr *= s.e;
  }
  return r.N;
}

// Distance of each ray to the non-differentiable points of Alg. 1 (for the
// parity harness): face[q] = min over samples and axes of the distance (in
// voxels) of the sample to an interior cell face (where the trilinear
// gradient jumps); knot[q] = min over samples of the distance of
// u = d*(R-1) to a TF knot 0..R-1 (slope change or clamp end), EA only.
// Rays that miss get 1e30 in both.  entry[q] (may be NULL) = t0/|omega_a| for
// the entry plane a (0 when the eye is inside): how much an error in the ray
// direction is amplified into the entry point.
int oracle_kinks(const double* V, int nx, int ny, int nz, const double* tf, int R,
                 const double* cam, int W, int H, double step, int model,
                 const int32_t* pix, int64_t npix, double* face, double* knot, double* entry) {
  if (model < 0 || model > 2) return -3;
  const bool ea = model >= 1;
  if (model == 2) tf = nullptr;               // no TF knots in a colour volume
  if (!V || !cam || !face || !knot || (model == 1 && !tf)) return -1;
  if (!check_common(nx, ny, nz, R, model == 1, W, H, step)) return -2;
  const Grid g = make_grid(nx, ny, nz);
  const int64_t n = pix ? npix : int64_t(W) * H;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n; ++q) {
    const int64_t p = pix ? int64_t(pix[q]) : q;
    Ray<double> r = make_ray<double>(cam, int(p % W), int(p / W), W, H, g, step);
    double fmin = 1e30, kmin = 1e30;
    for (int i = 0; r.hit && i < r.N; ++i) {
      Sample<double> s = eval_sample(g, V, tf, R, ea, r, step, i);
      for (int a = 0; a < 3; ++a) {
        const double qa = (s.x[a] - g.bmin[a]) / g.h;
        const double k = std::round(qa);
        if (k >= 1.0 && k <= double(g.n[a] - 2)) fmin = std::min(fmin, std::fabs(qa - k));
      }
      if (ea && tf) {
        const double u = s.d * double(R - 1);
        const double k = std::round(u);
        if (k >= 0.0 && k <= double(R - 1)) kmin = std::min(kmin, std::fabs(u - k));
      }
    }
    face[q] = fmin;
    knot[q] = kmin;
    if (entry)
      entry[q] = (r.hit && r.entry_axis >= 0) ? r.t0 / std::fabs(r.omega[r.entry_axis]) : 0.0;
  }
  return 0;
}

int oracle_splitmix64(uint64_t seed, uint64_t n, uint64_t* out) {
  if (!out) return -1;
  *out = splitmix_output(seed, n);
  return 0;
}

// CV [nz][ny][nx][4] (r, g, b, tau), tf [R][4], d_prev [nz][ny][nx] or null.
// vox: the nsel voxel indices to evaluate, or null for every voxel.  Outputs
// per evaluated voxel q: d_out (the chosen candidate), cost_out (its cost),
// idx_out (its index); all_costs / all_cands [q][ncand] (every candidate's
// cost / density) if not null.
int oracle_density_from_color(const double* CV, int nx, int ny, int nz, const double* tf, int R,
                              const double* d_prev, double alpha, double beta, uint64_t seed,
                              int iter, int ncand, const int64_t* vox, int64_t nsel,
                              double* d_out, double* cost_out, int32_t* idx_out,
                              double* all_costs, double* all_cands) {
  if (!CV || !tf || !d_out || nx < 1 || ny < 1 || nz < 1 || R < 2 || ncand < 1 || iter < 0)
    return -1;
  const int64_t nvox = (int64_t)nx * ny * nz;
  const int64_t nq = vox ? nsel : nvox;
  if (vox)
    for (int64_t q = 0; q < nsel; ++q)
      if (vox[q] < 0 || vox[q] >= nvox) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < nq; ++q) {
    const int64_t v = vox ? vox[q] : q;
    const int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
    const double* t = CV + 4 * v;
    double nb[6];
    int nn = 0;
    if (d_prev) {
      if (x > 0) nb[nn++] = d_prev[v - 1];
      if (x + 1 < nx) nb[nn++] = d_prev[v + 1];
      if (y > 0) nb[nn++] = d_prev[v - nx];
      if (y + 1 < ny) nb[nn++] = d_prev[v + nx];
      if (z > 0) nb[nn++] = d_prev[v - (int64_t)nx * ny];
      if (z + 1 < nz) nb[nn++] = d_prev[v + (int64_t)nx * ny];
    }
    double best = 0.0, bestd = 0.0;
    int bi = -1;
    for (int k = 0; k < ncand; ++k) {
      const uint64_t n = ((uint64_t)iter * (uint64_t)nvox + (uint64_t)v) * (uint64_t)ncand +
                         (uint64_t)k;
      const double d = candidate_density(seed, n);
      const TFSample<double> m = tf_lookup(d, tf, R);
      double c = 0.0;
      for (int ch = 0; ch < 3; ++ch) c += (t[ch] - m.rgb[ch]) * (t[ch] - m.rgb[ch]);
      c += alpha * std::log(1.0 + std::fabs(t[3] - m.tau));
      double s = 0.0;
      for (int q = 0; q < nn; ++q) s += (d - nb[q]) * (d - nb[q]);
      c += beta * s;
      if (all_costs) all_costs[q * ncand + k] = c;
      if (all_cands) all_cands[q * ncand + k] = d;
      if (bi < 0 || c < best) { best = c; bestd = d; bi = k; }
    }
    d_out[q] = bestd;
    if (cost_out) cost_out[q] = best;
    if (idx_out) idx_out[q] = bi;
  }
  return 0;
}

int oracle_num_threads(void) { return nthreads_max(); }

// Threads of later parallel regions (timing of the oracle on one core and on
// all of them); returns the new maximum.
int oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
  return nthreads_max();
}

}  // extern "C"

// Test infrastructure: a driver that calls every entry point of the FP64
// oracle on small seeded problems (absorption-only, emission-absorption and
// colour volumes, every adjoint variant, forward mode, the helpers, density
// from colour, and argument errors), for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_oracle_sanitizers.py).  Prints "ok"
// and exits 0 when every call returned as expected with finite results.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int oracle_camera_from_sphere(double, double, double, double, int, int, double*);
int oracle_camera_jacobian(double, double, double, double, int, int, double*);
int oracle_render(const double*, int, int, int, const double*, int, const double*, int, int,
                  double, int, const int32_t*, int64_t, double*, double*, int32_t*, double*);
int oracle_adjoint(const double*, int, int, int, const double*, int, const double*, int, int,
                   double, int, const int32_t*, int64_t, const double*, int, int, double*,
                   double*, double*, double*);
int oracle_render_dual(const double*, const double*, int, int, int, const double*,
                       const double*, int, const double*, const double*, int, int, double,
                       double, int, const int32_t*, int64_t, double*, double*, double*, double*);
int oracle_trilinear(const double*, int, int, int, const double*, double*);
int oracle_tf_lookup(const double*, int, double, double*);
int oracle_ray(const double*, int, int, int, int, int, int, int, double, double*);
int oracle_trace_ray(const double*, int, int, int, const double*, int, const double*, int, int,
                     int, int, double, int, int, double*, double*, double*, double*);
int oracle_kinks(const double*, int, int, int, const double*, int, const double*, int, int,
                 double, int, const int32_t*, int64_t, double*, double*, double*);
int oracle_splitmix64(uint64_t, uint64_t, uint64_t*);
int oracle_density_from_color(const double*, int, int, int, const double*, int, const double*,
                              double, double, uint64_t, int, int, const int64_t*, int64_t,
                              double*, double*, int32_t*, double*, double*);
int oracle_num_threads(void);
int oracle_set_threads(int);
}

static int failures = 0;
#define EXPECT(c)                                                        \
  do {                                                                   \
    if (!(c)) {                                                          \
      std::fprintf(stderr, "check failed (line %d): %s\n", __LINE__, #c); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

static bool finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

int main() {
  std::mt19937_64 rng(2107);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  oracle_set_threads(2);
  EXPECT(oracle_num_threads() == 2);
  const int shapes[3][3] = {{6, 7, 5}, {2, 2, 2}, {9, 4, 6}};
  for (const auto& sh : shapes) {
    const int nx = sh[0], ny = sh[1], nz = sh[2];
    const size_t nv = size_t(nx) * ny * nz;
    std::vector<double> V(nv), CV(4 * nv);
    for (auto& x : V) x = U(rng);
    for (auto& x : CV) x = U(rng);
    for (const int R : {2, 5}) {
      std::vector<double> tf(4 * R);
      for (auto& x : tf) x = 3.0 * U(rng);
      const int W = 9, H = 8;
      std::vector<double> cam(12);
      EXPECT(oracle_camera_from_sphere(0.6, 0.3, 2.5, 1.0, W, H, cam.data()) == 0);
      std::vector<double> jac(48);
      EXPECT(oracle_camera_jacobian(0.6, 0.3, 2.5, 1.0, W, H, jac.data()) == 0 && finite(jac));
      const double step = 0.4 * 2.0 / (std::max(nx, std::max(ny, nz)) - 1);
      std::vector<int32_t> pix = {0, 5, 17, 40, 71};
      for (int model = 0; model < 3; ++model) {
        const double* vol = model == 2 ? CV.data() : V.data();
        const double* t = model == 1 ? tf.data() : nullptr;
        const int C = model == 0 ? 1 : 4;
        for (int sub = 0; sub < 2; ++sub) {
          const int32_t* pp = sub ? pix.data() : nullptr;
          const int64_t np = sub ? int64_t(pix.size()) : int64_t(W) * H;
          std::vector<double> img(np * C), tr(np), ratio(np);
          std::vector<int32_t> ns(np);
          EXPECT(oracle_render(vol, nx, ny, nz, t, R, cam.data(), W, H, step, model, pp, np,
                               img.data(), tr.data(), ns.data(), ratio.data()) == 0);
          EXPECT(finite(img) && finite(tr));
          std::vector<double> g(np * C);
          for (auto& x : g) x = U(rng) - 0.5;
          for (int variant = 0; variant < 5; ++variant) {
            if (variant == 4 && model != 2) continue;
            std::vector<double> dV(nv * (model == 2 ? 4 : 1)), dTF(4 * R), dcam(12), dstep(1);
            EXPECT(oracle_adjoint(vol, nx, ny, nz, t, R, cam.data(), W, H, step, model, pp, np,
                                  g.data(), variant, variant == 3 ? 3 : 0, dV.data(),
                                  model == 1 ? dTF.data() : nullptr, dcam.data(),
                                  dstep.data()) == 0);
            EXPECT(finite(dV) && finite(dTF) && finite(dcam) && finite(dstep));
          }
          std::vector<double> Vd(nv * (model == 2 ? 4 : 1)), tfd(4 * R), camd(12);
          for (auto& x : Vd) x = U(rng);
          for (auto& x : tfd) x = U(rng);
          for (auto& x : camd) x = 1e-3 * U(rng);
          std::vector<double> im2(np * C), imd(np * C), tr2(np), trd(np);
          EXPECT(oracle_render_dual(vol, Vd.data(), nx, ny, nz, t, model == 1 ? tfd.data() : nullptr,
                                    R, cam.data(), camd.data(), W, H, step, 0.01, model, pp, np,
                                    im2.data(), imd.data(), tr2.data(), trd.data()) == 0);
          EXPECT(finite(imd) && finite(trd));
          std::vector<double> face(np), knot(np), entry(np);
          EXPECT(oracle_kinks(vol, nx, ny, nz, t, R, cam.data(), W, H, step, model, pp, np,
                              face.data(), knot.data(), entry.data()) == 0);
        }
      }
      // helpers
      double x[3] = {0.1, -0.2, 0.3}, d = 0.0, o4[4];
      EXPECT(oracle_trilinear(V.data(), nx, ny, nz, x, &d) == 0 && std::isfinite(d));
      EXPECT(oracle_tf_lookup(tf.data(), R, 0.37, o4) == 0);
      EXPECT(oracle_tf_lookup(tf.data(), R, -2.0, o4) == 0 && oracle_tf_lookup(tf.data(), R, 7.0, o4) == 0);
      double ray[8];
      EXPECT(oracle_ray(cam.data(), nx, ny, nz, W, H, 4, 4, step, ray) >= 0);
      std::vector<double> td(64), tt(64), tb(64), tx(192);
      EXPECT(oracle_trace_ray(V.data(), nx, ny, nz, tf.data(), R, cam.data(), W, H, 4, 4, step, 1,
                              64, td.data(), tt.data(), tb.data(), tx.data()) >= 0);
      // density from colour: every voxel, then a selection with all costs
      std::vector<double> prev(nv), dout(nv), cost(nv);
      for (auto& p : prev) p = U(rng);
      std::vector<int32_t> idx(nv);
      EXPECT(oracle_density_from_color(CV.data(), nx, ny, nz, tf.data(), R, nullptr, 0.5, 1.0, 7,
                                       0, 16, nullptr, 0, dout.data(), cost.data(), idx.data(),
                                       nullptr, nullptr) == 0);
      std::vector<int64_t> sel = {0, int64_t(nv) - 1};
      std::vector<double> ac(2 * 16), an(2 * 16), d2(2), c2(2);
      EXPECT(oracle_density_from_color(CV.data(), nx, ny, nz, tf.data(), R, prev.data(), 0.5, 1.0,
                                       7, 3, 16, sel.data(), 2, d2.data(), c2.data(), nullptr,
                                       ac.data(), an.data()) == 0);
      EXPECT(finite(dout) && finite(cost) && finite(ac));
    }
  }
  std::vector<uint64_t> sm(8);
  EXPECT(oracle_splitmix64(1, 8, sm.data()) == 0);
  // argument errors return codes, never touch memory
  std::vector<double> V8(8, 0.5), cam(12);
  oracle_camera_from_sphere(0.1, 0.1, 2.5, 1.0, 4, 4, cam.data());
  EXPECT(oracle_render(nullptr, 2, 2, 2, nullptr, 0, cam.data(), 4, 4, 0.1, 0, nullptr, 0,
                       nullptr, nullptr, nullptr, nullptr) != 0);
  EXPECT(oracle_render(V8.data(), 2, 2, 2, nullptr, 0, cam.data(), 4, 4, 0.1, 7, nullptr, 0,
                       nullptr, nullptr, nullptr, nullptr) != 0);
  EXPECT(oracle_render(V8.data(), 1, 2, 2, nullptr, 0, cam.data(), 4, 4, 0.1, 0, nullptr, 0,
                       nullptr, nullptr, nullptr, nullptr) != 0);
  EXPECT(oracle_adjoint(V8.data(), 2, 2, 2, nullptr, 0, cam.data(), 4, 4, 0.1, 0, nullptr, 0,
                        nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr) != 0);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}

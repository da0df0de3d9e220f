// Host sanitizer driver for the CPU oracle: built with AddressSanitizer and
// UndefinedBehaviorSanitizer together with oracle/gsff_oracle.cpp, it calls
// every oracle entry point on small seeded scenes and on the degenerate ones
// (no Gaussians, everything culled, non-finite and zero parameters, a 1x1
// image, no feature channels).  A sanitizer report aborts the run; the
// driver itself checks only return codes and a few invariants.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../oracle/gsff_oracle.h"

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
double uni() {  // xorshift64*, [0, 1)
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0);
}

struct Scene {
  int64_t P;
  int32_t C;
  std::vector<double> means, log_scales, quats, logit, rgb, feat;
  orc_scene s;
  void make(int64_t n, int32_t c, int W, int H, double f) {
    P = n;
    C = c;
    means.resize(3 * P);
    log_scales.resize(3 * P);
    quats.resize(4 * P);
    logit.resize(P);
    rgb.resize(3 * P);
    feat.resize(P * C);
    for (int64_t i = 0; i < P; ++i) {
      const double z = 1.0 + 4.0 * uni();
      means[i] = (uni() * W - W / 2.0) * z / f;
      means[P + i] = (uni() * H - H / 2.0) * z / f;
      means[2 * P + i] = z;
      for (int k = 0; k < 3; ++k) log_scales[k * P + i] = -3.0 + 1.6 + 0.5 * (uni() - 0.5);
      for (int k = 0; k < 4; ++k) quats[k * P + i] = uni() - 0.5;
      logit[i] = 2.0 * (uni() - 0.5);
      for (int k = 0; k < 3; ++k) rgb[k * P + i] = uni();
    }
    for (auto& v : feat) v = uni() - 0.5;
    s = orc_scene{P,
                  C,
                  0,
                  means.data(),
                  log_scales.data(),
                  quats.data(),
                  logit.data(),
                  rgb.data(),
                  C > 0 ? feat.data() : nullptr};
  }
};

orc_camera camera(int W, int H, double f) {
  orc_camera c{};
  c.width = W;
  c.height = H;
  c.fx = c.fy = f;
  c.cx = W / 2.0;
  c.cy = H / 2.0;
  const double V[12] = {1, 0, 0, 0.01, 0, 1, 0, -0.02, 0, 0, 1, 0.03};
  for (int k = 0; k < 12; ++k) c.viewmat[k] = V[k];
  return c;
}

int g_fail = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s\n", what);
    ++g_fail;
  }
}

void exercise(Scene& sc, const orc_camera& cam, const char* name) {
  orc_settings st{0.2, 1.3, 0.3, 1.0 / 255.0, 0.99, 1e-4, 1, 0};
  const int64_t P = sc.P, HW = (int64_t)cam.width * cam.height;
  const int C = sc.C;
  std::vector<double> proj(P * ORC_PROJ_FIELDS + 1);
  expect(orc_project(&sc.s, &cam, &st, proj.data()) == 0, name);
  std::vector<double> rgb(3 * HW), depth(HW), alpha(HW), feat(C * HW + 1), T(HW), margin(HW);
  std::vector<int32_t> n(HW);
  uint64_t hash = 0;
  expect(orc_render(&sc.s, &cam, &st, rgb.data(), depth.data(), alpha.data(),
                    C ? feat.data() : nullptr, T.data(), n.data(), margin.data(), &hash) == 0,
         name);
  for (int64_t p = 0; p < HW; ++p) expect(alpha[p] >= 0.0 && alpha[p] < 1.0, "alpha in [0, 1)");
  std::vector<uint8_t> sure(P + 1), possible(P + 1), flags(P + 1);
  expect(orc_visibility(&sc.s, &cam, &st, 0.5, 0.005, sure.data(), possible.data()) == 0, name);
  std::vector<int32_t> px, py;
  for (int k = 0; k < 17; ++k) {
    px.push_back((int32_t)(uni() * cam.width));
    py.push_back((int32_t)(uni() * cam.height));
  }
  std::vector<double> pix(px.size() * (5 + C));
  expect(orc_render_pixels(&sc.s, &cam, &st, (int64_t)px.size(), px.data(), py.data(),
                           pix.data()) == 0,
         name);
  expect(orc_ambiguous(&sc.s, &cam, &st, 1e-3, 0, nullptr, nullptr, flags.data()) == 0, name);
  expect(orc_ambiguous(&sc.s, &cam, &st, 1e-3, (int64_t)px.size(), px.data(), py.data(),
                       flags.data()) == 0,
         name);
  std::vector<double> g_rgb(3 * HW), g_depth(HW), g_alpha(HW), g_feat(C * HW + 1);
  for (auto& v : g_rgb) v = uni() - 0.5;
  for (auto& v : g_depth) v = uni() - 0.5;
  for (auto& v : g_alpha) v = uni() - 0.5;
  for (auto& v : g_feat) v = uni() - 0.5;
  std::vector<double> dm(3 * P + 1), dls(3 * P + 1), dq(4 * P + 1), dlo(P + 1), drgb(3 * P + 1),
      df(P * C + 1), dpose(6), d2d(10 * P + 1);
  expect(orc_backward(&sc.s, &cam, &st, g_rgb.data(), g_depth.data(), g_alpha.data(),
                      C ? g_feat.data() : nullptr, dm.data(), dls.data(), dq.data(), dlo.data(),
                      drgb.data(), C ? df.data() : nullptr, dpose.data(), d2d.data()) == 0,
         name);
  for (int tile : {16, 5, 1}) {
    const int64_t nt = (int64_t)((cam.width + tile - 1) / tile) * ((cam.height + tile - 1) / tile);
    std::vector<int64_t> counts(nt);
    const int64_t total = orc_tile_lists(&sc.s, &cam, &st, tile, counts.data(), nullptr);
    expect(total >= 0, name);
    std::vector<int32_t> ids(total + 1);
    expect(orc_tile_lists(&sc.s, &cam, &st, tile, counts.data(), ids.data()) == total, name);
    int64_t out[4];
    expect(orc_work_counts(&sc.s, &cam, &st, tile, out) == 0, name);
    expect(out[0] == total, "work_counts pairs = tile_lists total");
  }
  std::printf("%s: P=%lld C=%d %dx%d ok\n", name, (long long)P, C, cam.width, cam.height);
}

}  // namespace

int main() {
  {
    Scene sc;
    sc.make(40, 3, 37, 29, 30.0);
    exercise(sc, camera(37, 29, 30.0), "small ragged");
  }
  {
    Scene sc;
    sc.make(300, 0, 64, 48, 50.0);
    exercise(sc, camera(64, 48, 50.0), "no features");
  }
  {
    Scene sc;
    sc.make(0, 4, 16, 16, 20.0);
    exercise(sc, camera(16, 16, 20.0), "empty");
  }
  {
    Scene sc;
    sc.make(25, 2, 1, 1, 2.0);
    exercise(sc, camera(1, 1, 2.0), "1x1 image");
  }
  {
    Scene sc;
    sc.make(30, 2, 24, 20, 25.0);
    const int64_t P = sc.P;
    for (int64_t i = 0; i < P; ++i) sc.means[2 * P + i] = -1.0 - (double)i;  // behind the camera
    exercise(sc, camera(24, 20, 25.0), "all culled");
  }
  {
    Scene sc;
    sc.make(30, 2, 24, 20, 25.0);
    const int64_t P = sc.P;
    sc.means[0] = NAN;
    sc.quats[1] = sc.quats[P + 1] = sc.quats[2 * P + 1] = sc.quats[3 * P + 1] = 0.0;
    sc.log_scales[2] = -INFINITY;
    sc.log_scales[3] = 8.0;   // a splat over the whole image
    sc.logit[4] = 30.0;       // opacity 1: the alpha clamp
    sc.logit[5] = -30.0;      // below alpha_min
    sc.means[2 * P + 6] = 0.2;  // on the near plane
    exercise(sc, camera(24, 20, 25.0), "degenerate parameters");
  }
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("oracle sanitizer run: all entry points ok\n");
  return 0;
}

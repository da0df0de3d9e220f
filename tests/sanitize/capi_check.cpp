// Host sanitizer driver for the C ABI: linked against a build of the host
// side (capi.hip compiled with AddressSanitizer and UndefinedBehaviorSanitizer
// on the host pass), it runs every host-only path that needs no GPU:
// versions and defaults, workspace sizes and layouts over a grid of sizes
// (including the unrepresentable ones), and argument validation of every
// entry point.  Every call with an invalid argument returns before anything
// is launched; the pointers passed are stand-ins that are never dereferenced.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <initializer_list>

#include "../../include/gsff.h"

namespace {

int g_fail = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, gsff_last_error());
    ++g_fail;
  }
}

void* fake() { return reinterpret_cast<void*>(uintptr_t{0x7F0000000000}); }
const float* ffake() { return static_cast<const float*>(fake()); }
float* wfake() { return static_cast<float*>(fake()); }
uint8_t* bfake() { return static_cast<uint8_t*>(fake()); }

void sizes() {
  const int64_t Ps[] = {0, 1, 2, 1000, 200000, 1 << 20, (int64_t{1} << 30) - 1, int64_t{1} << 30, -1};
  const int32_t Cs[] = {0, 1, 16, 64, 4096, 4097, -1};
  const int64_t Ms[] = {0, 1000, 5000000, 0xFFFFFFFEll, 0xFFFFFFFFll, -1};
  const int32_t WH[][2] = {{1, 1}, {64, 48}, {640, 480}, {1200, 680}, {3840, 2160},
                           {1048560, 16}, {1048576, 16}, {0, 5}};
  int ok = 0, rejected = 0;
  for (int64_t P : Ps)
    for (int32_t C : Cs)
      for (int64_t M : Ms)
        for (const auto& wh : WH) {
          size_t n = 0;
          gsff_ws_layout lay;
          std::memset(&lay, 0, sizeof(lay));
          const gsff_status a = gsff_workspace_size(P, C, M, wh[0], wh[1], &n);
          const gsff_status b = gsff_workspace_layout(P, C, M, wh[0], wh[1], &lay);
          expect(a == b, "size and layout agree on validity");
          if (a == GSFF_OK) {
            ++ok;
            expect(lay.total_bytes == n, "layout total = workspace size");
            expect(lay.status == 0 && lay.records % 256 == 0 && lay.grad2d < n,
                   "regions inside the workspace, 256-byte aligned");
          } else {
            ++rejected;
          }
        }
  expect(ok > 0 && rejected > 0, "some sizes valid, some rejected");
  size_t n = 0;
  expect(gsff_workspace_size(10, 0, 100, 8, 8, nullptr) != GSFF_OK, "NULL size output");
  for (int64_t px : {int64_t{0}, int64_t{1}, int64_t{307200}, int64_t{-1}})
    gsff_decoder_workspace_size(px, &n);
  for (int32_t K : {0, 1, 64, 65})
    for (int64_t px : {int64_t{0}, int64_t{307200}, int64_t{-1}})
      gsff_decoder_query_workspace_size(K, px, &n);
  for (int64_t P : {int64_t{0}, int64_t{1}, int64_t{1000000}, int64_t{-1}})
    gsff_scale_reg_workspace_size(P, &n);
  for (int64_t P : {int64_t{0}, int64_t{4096}, int64_t{4097}})
    gsff_f64_workspace_size(P, 4, 64, 48, &n);
  std::printf("workspace sizes: %d valid, %d rejected\n", ok, rejected);
}

void validation() {
  const gsff_status E = GSFF_ERR_INVALID_ARGUMENT;
  gsff_settings s;
  expect(gsff_default_settings(&s) == GSFF_OK, "defaults");
  gsff_gaussians g{10, 0, GSFF_DTYPE_F32, ffake(), ffake(), ffake(), ffake(), ffake(), nullptr};
  gsff_camera c{32, 32, 30.f, 30.f, 16.f, 16.f, ffake()};
  void* ws = reinterpret_cast<void*>(uintptr_t{0x100000});
  const size_t nb = size_t{1} << 30;
  const int64_t mp = 1000;
  float* o = wfake();
  expect(gsff_forward(nullptr, &c, &s, ws, nb, mp, o, o, o, nullptr, 0, nullptr) == E, "NULL g");
  expect(gsff_forward(&g, &c, &s, nullptr, nb, mp, o, o, o, nullptr, 0, nullptr) == E, "NULL ws");
  expect(gsff_forward(&g, &c, &s, ws, nb, mp, nullptr, o, o, nullptr, 0, nullptr) == E,
         "NULL output");
  expect(gsff_forward(&g, &c, &s, static_cast<char*>(ws) + 4, nb, mp, o, o, o, nullptr, 0,
                      nullptr) == E,
         "misaligned ws");
  expect(gsff_forward(&g, &c, &s, ws, 64, mp, o, o, o, nullptr, 0, nullptr) == E, "small ws");
  gsff_settings s2 = s;
  s2.alpha_min = 0.f;
  expect(gsff_forward(&g, &c, &s2, ws, nb, mp, o, o, o, nullptr, 0, nullptr) == E, "settings");
  s2 = s;
  s2.t_min = NAN;
  expect(gsff_forward(&g, &c, &s2, ws, nb, mp, o, o, o, nullptr, 0, nullptr) == E, "NaN t_min");
  gsff_gaussians g2 = g;
  g2.C = 4;
  g2.feat = fake();
  expect(gsff_forward(&g2, &c, &s, ws, nb, mp, o, o, o, nullptr, 0, nullptr) == E,
         "no feature output");
  g2.feat_dtype = 7;
  expect(gsff_forward(&g2, &c, &s, ws, nb, mp, o, o, o, o, 0, nullptr) == GSFF_ERR_UNSUPPORTED,
         "feature dtype");
  gsff_camera c2 = c;
  c2.width = 0;
  expect(gsff_forward(&g, &c2, &s, ws, nb, mp, o, o, o, nullptr, 0, nullptr) == E, "image size");
  c2 = c;
  c2.fx = -1.f;
  expect(gsff_forward(&g, &c2, &s, ws, nb, mp, o, o, o, nullptr, 0, nullptr) == E, "intrinsics");
  gsff_grads gr{o, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  expect(gsff_backward(&g, &c, &s, ws, nb, mp, nullptr, ffake(), ffake(), nullptr, &gr, 0,
                       nullptr) == E,
         "backward: no upstream");
  expect(gsff_backward(&g, &c, &s, ws, nb, mp, ffake(), ffake(), ffake(), nullptr, nullptr, 0,
                       nullptr) == E,
         "backward: no grads");
  expect(gsff_l1_grad(nullptr, nullptr, 10, 1.f, nullptr, nullptr, nullptr) == E, "l1");
  expect(gsff_read_status(nullptr, nullptr, nullptr, nullptr) == E, "status");
  expect(gsff_backward_tracking(&g, &c, &s, ws, nb, mp, ffake(), ffake(), ffake(), ffake(),
                                nullptr, nullptr, 0.9f, nullptr, nullptr, 0, nullptr) == E,
         "tracking: no pose gradient");
  expect(gsff_tracking_masks(ffake(), ffake(), 0, 8, 0.1f, 0.5f, bfake(), bfake(), nullptr) == E,
         "masks: size");
  expect(gsff_tracking_masks(ffake(), ffake(), 8, 8, -0.1f, 0.5f, bfake(), bfake(), nullptr) == E,
         "masks: threshold");
  expect(gsff_pose_adam_step(nullptr, ffake(), wfake(), 1, 1e-3f, 1e-3f, 0.9f, 0.999f, 1e-8f,
                             nullptr, nullptr, nullptr, nullptr) == E,
         "pose step: NULL");
  gsff_pose_convergence cv{0, 1e-3f, 1e-3f};
  expect(gsff_pose_adam_step(wfake(), ffake(), wfake(), 1, 1e-3f, 1e-3f, 0.9f, 0.999f, 1e-8f,
                             &cv, nullptr, nullptr, nullptr) == E,
         "pose step: window");
  expect(gsff_visibility(&g, &c, &s, ws, nb, mp, 0.5f, nullptr, nullptr) == E, "visibility");
  expect(gsff_covisibility(static_cast<const uint8_t*>(fake()), static_cast<const uint8_t*>(fake()),
                           -1, static_cast<uint32_t*>(fake()), nullptr) == E,
         "covisibility");
  expect(gsff_keyframe_test(static_cast<const uint8_t*>(fake()), static_cast<const uint8_t*>(fake()),
                            5, NAN, static_cast<uint32_t*>(fake()), static_cast<uint32_t*>(fake()),
                            nullptr) == E,
         "keyframe");
  gsff_adam_group grp[9];
  std::memset(grp, 0, sizeof(grp));
  expect(gsff_adam_step(grp, 9, 1, 0.9f, 0.999f, 1e-8f, nullptr) == E, "adam: groups");
  expect(gsff_scale_reg(ffake(), 0, 0.1f, wfake(), nb, nullptr, nullptr, 0, nullptr) == E,
         "scale reg");
  expect(gsff_decoder_query(fake(), ffake(), ffake(), ffake(), ffake(), ffake(), 65, 10, nullptr,
                            nullptr, nullptr, nullptr, ws, nb, nullptr) == E,
         "query: K");
  expect(gsff_decoder_query_noalloc(fake(), ffake(), ffake(), ffake(), ffake(), ffake(), 0, 10,
                                    nullptr, nullptr, nullptr, nullptr, nullptr) == E,
         "noalloc query: K");
  expect(gsff_decoder_forward(nullptr, ffake(), ffake(), ffake(), ffake(), fake(),
                              GSFF_DTYPE_BF16, 10, ws, nb, nullptr) == E,
         "decoder forward");
  gsff_gaussians_f64 g64{5000, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  gsff_camera_f64 c64{8, 8, 10.0, 10.0, 4.0, 4.0, static_cast<const double*>(fake())};
  double* d = static_cast<double*>(fake());
  expect(gsff_forward_f64(&g64, &c64, &s, ws, nb, d, d, d, nullptr, nullptr, nullptr) == E,
         "f64: P");
  int32_t kind = -1;
  expect(gsff_is_checked_build(&kind) == GSFF_OK && (kind == 0 || kind == 1), "build kind");
  expect(gsff_is_checked_build(nullptr) == E, "build kind: NULL");
  uint32_t chk[4];
  expect(gsff_read_checks(nullptr, chk, nullptr) == E, "read_checks: NULL workspace");
  expect(gsff_read_checks(ws, nullptr, nullptr) == E, "read_checks: NULL output");
  std::printf("argument validation: done\n");
}

}  // namespace

int main() {
  int32_t a = -1, b = -1;
  expect(gsff_version(&a, &b) == GSFF_OK && a >= 0, "version");
  sizes();
  validation();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("C ABI host sanitizer run: ok\n");
  return 0;
}

// Drives the host-side argument checks and the frame-table layout of the
// C-ABI calls (paper_2411_17660_amd/csrc/host_check.cpp) over valid, invalid
// and extreme arguments.  Built with g++ under the address and
// undefined-behaviour sanitizers by tests/test_sanitizers.py; prints
// "ok <cases>" and exits 0 when every case returns the expected status.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "host_check.h"

using namespace gsr;

static int g_cases = 0, g_fail = 0;

static void expect(const char* what, gsr_status got, gsr_status want) {
  ++g_cases;
  if (got != want) {
    ++g_fail;
    std::printf("FAIL %s: status %d, expected %d\n", what, (int)got, (int)want);
  }
}

static void expect_true(const char* what, bool ok) {
  ++g_cases;
  if (!ok) {
    ++g_fail;
    std::printf("FAIL %s\n", what);
  }
}

struct Args {
  gsr_settings s;
  int64_t n = 10;
  std::vector<float> means, log_scales, quats, opac, sh, poses, rgb, depth, alpha;
  std::vector<gsr_camera> cams;
  Args(int F = 2) {
    std::memset(&s, 0, sizeof s);
    s.sh_degree = 3;
    s.tile_w = 16;
    s.tile_h = 16;
    means.assign(3 * n, 0.f);
    log_scales.assign(3 * n, 0.f);
    quats.assign(4 * n, 0.f);
    opac.assign(n, 0.f);
    sh.assign(48 * n, 0.f);
    poses.assign(12 * F, 0.f);
    for (int f = 0; f < F; ++f) cams.push_back(gsr_camera{640, 480, 500.f, 500.f, 320.f, 240.f, 0.2f});
    rgb.assign(3 * 640 * 480 * F, 0.f);
    depth.assign(640 * 480 * F, 0.f);
    alpha.assign(640 * 480 * F, 0.f);
  }
  gsr_status run(char* msg = nullptr, size_t cap = 0) const {
    static char local[256];
    if (!msg) { msg = local; cap = sizeof local; }
    return check_forward(&s, n, means.data(), log_scales.data(), quats.data(), opac.data(),
                         sh.data(), (int32_t)cams.size(), cams.data(), poses.data(), rgb.data(),
                         depth.data(), alpha.data(), msg, cap);
  }
};

int main() {
  const gsr_status OK = GSR_OK, BAD = GSR_ERR_INVALID_ARGUMENT, UNS = GSR_ERR_UNSUPPORTED;
  const float nan = std::numeric_limits<float>::quiet_NaN();
  const float inf = std::numeric_limits<float>::infinity();
  char msg[256];

  { Args a; expect("valid forward", a.run(), OK); }
  {
    Args a;
    expect("settings NULL",
           check_forward(nullptr, a.n, a.means.data(), a.log_scales.data(), a.quats.data(),
                         a.opac.data(), a.sh.data(), 2, a.cams.data(), a.poses.data(),
                         a.rgb.data(), a.depth.data(), a.alpha.data(), msg, sizeof msg),
           BAD);
  }
  { Args a; a.n = -1; expect("n < 0", a.run(), BAD); }
  { Args a; a.n = (int64_t)1 << 31; expect("n = 2^31", a.run(), BAD); }
  { Args a; a.n = std::numeric_limits<int64_t>::max(); expect("n = INT64_MAX", a.run(), BAD); }
  { Args a; a.n = ((int64_t)1 << 31) - 1; expect("n * 2 just under 2^32", a.run(), OK); }
  {
    Args a(3);
    a.n = ((int64_t)1 << 31) - 1;
    expect("n * 3 >= 2^32", a.run(), BAD);
  }
  { Args a; a.cams.clear(); expect("F = 0", a.run(), BAD); }
  { Args a; a.s.sh_degree = -1; expect("sh_degree -1", a.run(), BAD); }
  { Args a; a.s.sh_degree = 4; expect("sh_degree 4", a.run(), BAD); }
  { Args a; a.s.tile_w = 16; a.s.tile_h = 32; expect("tile 16x32", a.run(), UNS); }
  { Args a; a.s.tile_w = 0; a.s.tile_h = 0; expect("tile 0x0", a.run(), UNS); }
  for (int b : {32, 64, 128}) { Args a; a.s.lds_batch = b; expect("lds batch ok", a.run(), OK); }
  for (int b : {-1, 1, 48, 256}) { Args a; a.s.lds_batch = b; expect("lds batch bad", a.run(), UNS); }
  { Args a; a.s.key_capacity = -1; expect("key_capacity -1", a.run(), BAD); }
  { Args a; a.s.key_capacity = (int64_t)1 << 32; expect("key_capacity 2^32", a.run(), BAD); }
  { Args a; a.s.key_capacity = ((int64_t)1 << 32) - 1; expect("key_capacity max", a.run(), OK); }
  {
    Args a;
    expect("cams NULL",
           check_forward(&a.s, a.n, a.means.data(), a.log_scales.data(), a.quats.data(),
                         a.opac.data(), a.sh.data(), 2, nullptr, a.poses.data(), a.rgb.data(),
                         a.depth.data(), a.alpha.data(), msg, sizeof msg),
           BAD);
    expect("poses NULL",
           check_forward(&a.s, a.n, a.means.data(), a.log_scales.data(), a.quats.data(),
                         a.opac.data(), a.sh.data(), 2, a.cams.data(), nullptr, a.rgb.data(),
                         a.depth.data(), a.alpha.data(), msg, sizeof msg),
           BAD);
    expect("rgb NULL",
           check_forward(&a.s, a.n, a.means.data(), a.log_scales.data(), a.quats.data(),
                         a.opac.data(), a.sh.data(), 2, a.cams.data(), a.poses.data(), nullptr,
                         a.depth.data(), a.alpha.data(), msg, sizeof msg),
           BAD);
    expect("means NULL, n > 0",
           check_forward(&a.s, a.n, nullptr, a.log_scales.data(), a.quats.data(), a.opac.data(),
                         a.sh.data(), 2, a.cams.data(), a.poses.data(), a.rgb.data(),
                         a.depth.data(), a.alpha.data(), msg, sizeof msg),
           BAD);
    expect("parameters NULL, n = 0",
           check_forward(&a.s, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 2, a.cams.data(),
                         a.poses.data(), a.rgb.data(), a.depth.data(), a.alpha.data(), msg,
                         sizeof msg),
           OK);
    const float* odd = reinterpret_cast<const float*>(
        reinterpret_cast<const char*>(a.means.data()) + 2);
    expect("misaligned means",
           check_forward(&a.s, a.n, odd, a.log_scales.data(), a.quats.data(), a.opac.data(),
                         a.sh.data(), 2, a.cams.data(), a.poses.data(), a.rgb.data(),
                         a.depth.data(), a.alpha.data(), msg, sizeof msg),
           BAD);
  }
  struct CamCase { const char* what; gsr_camera c; gsr_status want; };
  const CamCase cam_cases[] = {
      {"width 0", {0, 480, 500.f, 500.f, 320.f, 240.f, 0.2f}, BAD},
      {"height -1", {640, -1, 500.f, 500.f, 320.f, 240.f, 0.2f}, BAD},
      {"width 65536", {65536, 480, 500.f, 500.f, 320.f, 240.f, 0.2f}, BAD},
      {"65535 x 1", {65535, 1, 500.f, 500.f, 320.f, 0.f, 0.2f}, OK},
      {"fx 0", {640, 480, 0.f, 500.f, 320.f, 240.f, 0.2f}, BAD},
      {"fy -1", {640, 480, 500.f, -1.f, 320.f, 240.f, 0.2f}, BAD},
      {"fx NaN", {640, 480, nan, 500.f, 320.f, 240.f, 0.2f}, BAD},
      {"fy inf", {640, 480, 500.f, inf, 320.f, 240.f, 0.2f}, BAD},
      {"cx NaN", {640, 480, 500.f, 500.f, nan, 240.f, 0.2f}, BAD},
      {"cy -inf", {640, 480, 500.f, 500.f, 320.f, -inf, 0.2f}, BAD},
      {"cx outside the image", {640, 480, 500.f, 500.f, -1e6f, 1e6f, 0.2f}, OK},
      {"near 0", {640, 480, 500.f, 500.f, 320.f, 240.f, 0.f}, BAD},
      {"near -1", {640, 480, 500.f, 500.f, 320.f, 240.f, -1.f}, BAD},
      {"near NaN", {640, 480, 500.f, 500.f, 320.f, 240.f, nan}, BAD},
      {"near inf", {640, 480, 500.f, 500.f, 320.f, 240.f, inf}, BAD},
  };
  for (const CamCase& cc : cam_cases) {
    Args a;
    a.cams[1] = cc.c;
    expect(cc.what, a.run(), cc.want);
  }
  // messages: NULL or zero-capacity buffers are never written; a short
  // buffer is truncated and terminated
  { Args a; a.n = -1; expect("no message buffer", a.run(nullptr, 0), BAD); }
  {
    Args a;
    a.n = -1;
    char small[4] = {'x', 'x', 'x', 'x'};
    expect("short message buffer", a.run(small, sizeof small), BAD);
    expect_true("message truncated", small[3] == '\0' && std::strlen(small) == 3);
  }
  {
    Args a;
    a.s.tile_w = 7;
    char m[256];
    a.run(m, sizeof m);
    expect_true("message names the tile shape", std::strstr(m, "7x16") != nullptr);
  }
  // bits_for
  expect_true("bits_for(0)", bits_for(0) == 1);
  expect_true("bits_for(2)", bits_for(2) == 1);
  expect_true("bits_for(3)", bits_for(3) == 2);
  expect_true("bits_for(65536)", bits_for(65536) == 16);
  expect_true("bits_for(65537)", bits_for(65537) == 17);
  expect_true("bits_for(2^32)", bits_for((uint64_t)1 << 32) == 32);
  expect_true("bits_for(UINT64_MAX)", bits_for(std::numeric_limits<uint64_t>::max()) == 32);
  // frame tables
  {
    std::vector<gsr_camera> cams = {{1200, 680, 600.f, 600.f, 600.f, 340.f, 0.2f},
                                    {33, 17, 30.f, 30.f, 16.f, 8.f, 0.2f},
                                    {1, 1, 1.f, 1.f, 0.f, 0.f, 0.2f}};
    std::vector<FrameDesc> fr;
    int64_t T = -1, P = -1, mx = -1;
    expect("frame table",
           build_frames(3, cams.data(), 16, 8, fr, &T, &P, &mx, msg, sizeof msg), OK);
    expect_true("frame table size", fr.size() == 3);
    expect_true("tiles", T == 75 * 85 + 3 * 3 + 1);
    expect_true("pixels", P == 1200 * 680 + 33 * 17 + 1);
    expect_true("largest frame", mx == 1200 * 680);
    expect_true("offsets", fr[1].tile_offset == 75 * 85 && fr[2].tile_offset == 75 * 85 + 9 &&
                               fr[2].pixel_offset == 1200 * 680 + 33 * 17);
    expect_true("grid", fr[1].grid_x == 3 && fr[1].grid_y == 3 && fr[2].grid_x == 1);
  }
  {
    // 64 frames of 65535 x 65535 at 8x8 tiles: 2^26 tiles each, 2^32 in all
    std::vector<gsr_camera> cams(64, gsr_camera{65535, 65535, 1.f, 1.f, 0.f, 0.f, 0.2f});
    std::vector<FrameDesc> fr;
    int64_t T = 0, P = 0, mx = 0;
    expect("2^31 tiles rejected",
           build_frames(64, cams.data(), 8, 8, fr, &T, &P, &mx, msg, sizeof msg), BAD);
    expect_true("totals untouched on rejection", T == 0 && P == 0 && mx == 0);
    std::vector<gsr_camera> few(31, gsr_camera{65535, 65535, 1.f, 1.f, 0.f, 0.f, 0.2f});
    expect("just under 2^31 tiles",
           build_frames(31, few.data(), 8, 8, fr, &T, &P, &mx, msg, sizeof msg), OK);
    expect_true("tiles just under 2^31", T == (int64_t)31 * 8192 * 8192);
  }
  // image-space cameras and alignment
  {
    std::vector<gsr_camera> cams = {{64, 48, 50.f, 50.f, 32.f, 24.f, 0.2f}};
    expect("image cameras ok", check_image_cameras(1, cams.data(), msg, sizeof msg), OK);
    expect("image cameras none", check_image_cameras(0, cams.data(), msg, sizeof msg), BAD);
    expect("image cameras NULL", check_image_cameras(1, nullptr, msg, sizeof msg), BAD);
    cams[0].fx = 0.f;
    expect("image camera fx 0", check_image_cameras(1, cams.data(), msg, sizeof msg), BAD);
    float buf[4];
    const void* ok[] = {buf, nullptr, buf + 1};
    expect("aligned", check_aligned4(ok, 3, msg, sizeof msg), OK);
    const void* odd[] = {buf, reinterpret_cast<const char*>(buf) + 1};
    expect("misaligned", check_aligned4(odd, 2, msg, sizeof msg), BAD);
  }
  if (g_fail) {
    std::printf("%d of %d cases failed\n", g_fail, g_cases);
    return 1;
  }
  std::printf("ok %d\n", g_cases);
  return 0;
}

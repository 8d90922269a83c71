// host_check.cpp -- host-side argument checks and the frame table of a batch
// (no HIP dependency; see host_check.h).
#include "host_check.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>

namespace gsr {
namespace {

gsr_status reject(gsr_status code, char* msg, size_t cap, const char* fmt, ...) {
  if (msg && cap) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, cap, fmt, ap);
    va_end(ap);
  }
  return code;
}

}  // namespace

int bits_for(uint64_t v) {
  int b = 1;
  while (b < 32 && (1ull << b) < v) ++b;
  return b;
}

bool tile_shape_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 32 && th == 8) ||
         (tw == 16 && th == 8) || (tw == 32 && th == 16);
}

bool lds_batch_supported(int batch) { return batch == 32 || batch == 64 || batch == 128; }

gsr_status check_aligned4(const void* const* ptrs, int count, char* msg, size_t cap) {
  for (int i = 0; i < count; ++i)
    if (((uintptr_t)ptrs[i]) & 3u)
      return reject(GSR_ERR_INVALID_ARGUMENT, msg, cap, "pointer not 4-aligned");
  return GSR_OK;
}

gsr_status check_forward(const gsr_settings* s, int64_t n, const float* means,
                         const float* log_scales, const float* quats, const float* opac,
                         const float* sh, int32_t F, const gsr_camera* cams, const float* poses,
                         const float* rgb, const float* depth, const float* alpha, char* msg,
                         size_t cap) {
  const gsr_status bad = GSR_ERR_INVALID_ARGUMENT;
  if (!s) return reject(bad, msg, cap, "settings is NULL");
  if (n < 0) return reject(bad, msg, cap, "n < 0");
  if (n >= (int64_t)1 << 31) return reject(bad, msg, cap, "n >= 2^31");
  if (F < 1) return reject(bad, msg, cap, "n_frames < 1");
  if ((int64_t)F * n >= (int64_t)1 << 32) return reject(bad, msg, cap, "n * n_frames >= 2^32");
  if (s->sh_degree < 0 || s->sh_degree > 3)
    return reject(bad, msg, cap, "sh_degree %d not in [0,3]", s->sh_degree);
  if (!tile_shape_supported(s->tile_w, s->tile_h))
    return reject(GSR_ERR_UNSUPPORTED, msg, cap, "tile shape %dx%d not supported", s->tile_w,
                  s->tile_h);
  if (s->lds_batch != 0 && !lds_batch_supported(s->lds_batch))
    return reject(GSR_ERR_UNSUPPORTED, msg, cap, "lds_batch %d not supported (0, 32, 64 or 128)",
                  s->lds_batch);
  if (s->key_capacity < 0 || s->key_capacity >= ((int64_t)1 << 32))
    return reject(bad, msg, cap, "key_capacity out of range");
  if (!cams || !poses) return reject(bad, msg, cap, "cams/poses is NULL");
  if (!rgb || !depth || !alpha) return reject(bad, msg, cap, "output is NULL");
  if (n > 0 && (!means || !log_scales || !quats || !opac || !sh))
    return reject(bad, msg, cap, "parameter pointer is NULL");
  const void* ptrs[] = {means, log_scales, quats, opac, sh, poses, rgb, depth, alpha};
  gsr_status rc = check_aligned4(ptrs, 9, msg, cap);
  if (rc) return rc;
  for (int f = 0; f < F; ++f) {
    const gsr_camera& c = cams[f];
    if (c.width < 1 || c.height < 1 || c.width > 65535 || c.height > 65535)
      return reject(bad, msg, cap, "frame %d: size %dx%d", f, c.width, c.height);
    if (!(c.fx > 0.0f) || !(c.fy > 0.0f) || !std::isfinite(c.fx) || !std::isfinite(c.fy))
      return reject(bad, msg, cap, "frame %d: focal length not finite and > 0", f);
    if (!std::isfinite(c.cx) || !std::isfinite(c.cy))
      return reject(bad, msg, cap, "frame %d: principal point not finite", f);
    if (!(c.near_z > 0.0f) || !std::isfinite(c.near_z))
      return reject(bad, msg, cap, "frame %d: near_z not finite and > 0", f);
  }
  return GSR_OK;
}

gsr_status build_frames(int32_t F, const gsr_camera* cams, int tw, int th,
                        std::vector<FrameDesc>& out, int64_t* n_tiles, int64_t* n_pixels,
                        int64_t* max_frame_pixels, char* msg, size_t cap) {
  out.assign((size_t)F, FrameDesc{});
  int64_t T = 0, Px = 0, max_hw = 0;
  for (int f = 0; f < F; ++f) {
    const gsr_camera& c = cams[f];
    FrameDesc& d = out[(size_t)f];
    d.width = c.width;
    d.height = c.height;
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    d.near_z = c.near_z;
    d.grid_x = (c.width + tw - 1) / tw;
    d.grid_y = (c.height + th - 1) / th;
    if (T >= ((int64_t)1 << 31)) break;
    d.tile_offset = (int32_t)T;
    d.pixel_offset = Px;
    T += (int64_t)d.grid_x * d.grid_y;
    Px += (int64_t)c.width * c.height;
    if ((int64_t)c.width * c.height > max_hw) max_hw = (int64_t)c.width * c.height;
  }
  if (T >= ((int64_t)1 << 31)) return reject(GSR_ERR_INVALID_ARGUMENT, msg, cap, "too many tiles");
  *n_tiles = T;
  *n_pixels = Px;
  *max_frame_pixels = max_hw;
  return GSR_OK;
}

gsr_status check_image_cameras(int32_t F, const gsr_camera* cams, char* msg, size_t cap) {
  if (F <= 0 || !cams) return reject(GSR_ERR_INVALID_ARGUMENT, msg, cap, "no frames");
  for (int f = 0; f < F; ++f) {
    const gsr_camera& c = cams[f];
    if (c.width <= 0 || c.height <= 0 || c.width > 65535 || c.height > 65535 ||
        !(c.fx > 0.0f) || !(c.fy > 0.0f))
      return reject(GSR_ERR_INVALID_ARGUMENT, msg, cap, "camera %d invalid", f);
  }
  return GSR_OK;
}

}  // namespace gsr

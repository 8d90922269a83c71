// host_check.h -- the host-side argument checks and frame-table layout of the
// C-ABI calls (include/gsr.h), in plain C++ with no HIP dependency, so that
// they can be built and exercised on the CPU under the address and
// undefined-behaviour sanitizers.  runtime.hip calls these before any device
// work; a rejected call leaves every buffer and the context unchanged.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "gsr.h"

namespace gsr {

// One frame of a batch (the batch descriptor of the batched backward over
// several keyframes, paper Sec. 3.3): the camera, its tile grid and the
// offsets of its first tile and first pixel in the batch.  Passed to the
// kernels by value; the same layout on host and device.
struct FrameDesc {
  int32_t width, height;
  float fx, fy, cx, cy, near_z;
  int32_t grid_x, grid_y;
  int32_t tile_offset;   // first global tile id of the frame
  int64_t pixel_offset;  // first packed pixel of the frame
};

// Bits needed for values < v (1..32).  The tile sort uses bits_for(T + 1) so
// that the all-ones sentinel of an overflowed record never aliases a tile id.
int bits_for(uint64_t v);

// Tile shapes with compositing kernels: 16x16, 8x8, 32x8, 16x8, 32x16.
bool tile_shape_supported(int tw, int th);
// Gaussians staged per LDS round by the 3D compositing kernels: 32, 64, 128.
bool lds_batch_supported(int batch);

// Checks of a forward call (3D Gaussians or surfels): sizes, settings,
// NULL and 4-byte alignment of every pointer, and each camera (size in
// 1..65535, finite focal lengths > 0, finite principal point, finite
// near_z > 0).  Returns GSR_OK or the error code with a message in msg
// (always NUL-terminated when cap > 0).
gsr_status check_forward(const gsr_settings* s, int64_t n, const float* means,
                         const float* log_scales, const float* quats, const float* opac,
                         const float* sh, int32_t F, const gsr_camera* cams, const float* poses,
                         const float* rgb, const float* depth, const float* alpha, char* msg,
                         size_t cap);

// The frame table of a batch for tile shape tw x th (validated cameras):
// fills `out` (F entries) and the totals of tiles, pixels and the largest
// frame's pixels.  GSR_ERR_INVALID_ARGUMENT when the tiles reach 2^31.
gsr_status build_frames(int32_t F, const gsr_camera* cams, int tw, int th,
                        std::vector<FrameDesc>& out, int64_t* n_tiles, int64_t* n_pixels,
                        int64_t* max_frame_pixels, char* msg, size_t cap);

// Checks of the cameras of an image-space call (normal consistency): size
// in 1..65535 and focal lengths > 0.
gsr_status check_image_cameras(int32_t F, const gsr_camera* cams, char* msg, size_t cap);

// GSR_OK when every non-NULL pointer of ptrs[0..count) is 4-byte aligned.
gsr_status check_aligned4(const void* const* ptrs, int count, char* msg, size_t cap);

}  // namespace gsr

// launch.h -- host-side launchers of the kernels, shared by the sources that
// define them and by runtime.hip, which sequences them.  Internal to
// libgsr.so; every launcher enqueues on `st` and returns without waiting.
#pragma once
#include "gsr.h"
#include "gsr_device.h"

namespace gsr {

// preprocess.hip: EWA projection, records, per-record reduction, chain rule
void launch_preprocess_fwd(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                           const float* poses, const float* means, const float* log_scales,
                           const float* quats, const float* opac, const float* sh, int deg,
                           int tile_w, int tile_h, Record* rec, uint2* trect,
                           uint32_t* depth_key, uint32_t* rec_id, uint32_t* ntiles);
int64_t preprocess_bwd_waves(int64_t n);
void launch_preprocess_bwd(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                           const float* poses, const float* means, const float* log_scales,
                           const float* quats, const float* opac, const float* sh, int deg,
                           const uint32_t* order, const uint32_t* first_wide,
                           const uint32_t* keyoff, const uint32_t* ntiles, const float* partial,
                           const uint32_t* stamp, const uint32_t* epoch, uint64_t key_capacity,
                           double* grad2d, float* g_means, float* g_log_scales, float* g_quats,
                           float* g_opac, float* g_sh, double* twist_partial, float* g_twist);
void launch_bump_epoch(hipStream_t st, uint32_t* epoch);
// cls[r] = 1 + floor(log2(ntiles[r])) (0 when culled), idx[r] = r: the input
// of the radix sort that orders the per-record reduction
// Statistics of the last forward: out[0] += records with no tile (culled),
// out[1] += Gaussians with a non-finite parameter (log_per = 3 log-scales
// per Gaussian, or 2 for surfels; nb3 = 3 (d+1)^2 SH values).
void launch_cull_stats(hipStream_t st, uint64_t m, const uint32_t* ntiles, int64_t n,
                       const float* means, const float* log_scales, int log_per,
                       const float* quats, const float* opac, const float* sh, int nb3,
                       unsigned long long* out);
void launch_size_class(hipStream_t st, uint64_t m, const uint32_t* ntiles, uint32_t* cls,
                       uint32_t* idx);
// *first_wide = the first position of the ascending sorted classes whose
// record has 128 or more slots (m if none); the 3D backward reduces those
// records a wave each
void launch_wide_boundary(hipStream_t st, uint64_t m, const uint32_t* sorted_cls,
                          uint32_t* first_wide);

// sort.hip: depth sort, offsets, tile keys and their sort, ranges.
// radix_hist_elems / radix_scan_elems: u32 workspace of a sort of up to
// n_max keys whose widest digit serves `bits` key bits (0: 8-bit digits).
void launch_fill_u32(hipStream_t st, uint32_t* p, uint64_t n, uint32_t v);
// dst[0..n) = host[0..n), the descriptors travelling as kernel arguments
void launch_set_frames(hipStream_t st, const FrameDesc* host, int n, FrameDesc* dst);
// dst[i] = src[i] for n16 16-byte elements (plain copy, bandwidth reference)
void launch_copy16(hipStream_t st, const void* src, void* dst, uint64_t n16);
size_t radix_hist_elems(uint64_t n_max, int bits);
size_t scan_block_elems(uint64_t n_max);
size_t radix_scan_elems(uint64_t n_max, int bits);
bool launch_radix_sort(hipStream_t st, uint32_t* keys_a, uint32_t* vals_a, uint32_t* keys_b,
                       uint32_t* vals_b, const uint64_t* n_dev, uint64_t n_max, int bits,
                       uint32_t* hist, uint32_t* scan_tmp);
// skey: the sorted depth keys (all ones: culled); trect_sorted[i] and
// cnt_sorted[i]: the tile rect and tile count of record perm[i].
void launch_offsets_scan(hipStream_t st, const uint32_t* skey, const uint32_t* perm,
                         const uint2* trect, uint64_t m, uint32_t* cnt_sorted,
                         uint2* trect_sorted, uint64_t* offsets, uint64_t* block_tmp,
                         uint64_t* total);
// Tile keys are 16-bit when the tile ids and the all-ones sentinel fit
// (bits <= 16), else 32-bit; `keys` buffers hold that type.
bool tile_keys_16bit(int bits);
// keys/vals of the min(K, capacity) key slots in depth order (record order,
// then row-major inside each record's tile rect) and keyoff[r] of every
// record with a tile (all-ones past the capacity, raising *overflow).
void launch_keygen(hipStream_t st, uint64_t m, uint64_t n, const uint32_t* perm,
                   const uint32_t* cnt_sorted, const uint64_t* offsets, uint32_t* keyoff,
                   const uint2* trect_sorted, const FrameDesc* frames, uint64_t capacity,
                   int bits, void* keys, uint32_t* vals, uint32_t* overflow);
// Stable sort of min(*k_dev, k_max) tile keys (k_dev NULL: k_max) by the
// tile-id bits [0, bits); returns true if the result is in (keys_b, vals_b).
bool launch_tile_sort(hipStream_t st, void* keys_a, uint32_t* vals_a, void* keys_b,
                      uint32_t* vals_b, const uint64_t* k_dev, uint64_t k_max, int bits,
                      uint32_t* hist, uint32_t* scan_tmp);
void launch_ranges(hipStream_t st, const void* keys, int bits, const uint64_t* k_dev,
                   uint64_t k_max, uint64_t capacity, uint2* ranges, uint64_t n_tiles);

// raster.hip: compositing forward and backward
// med_pos (NULL: alpha-blended depth) selects the median depth: the forward
// writes, per pixel, the list position of the entry after which T first
// falls below 1/2 (-1: none) and outputs that entry's z as the depth; the
// backward routes g_depth to that entry's z only.
// Tiles are dispatched in per-XCD groups of neighbouring tiles
// (`xcd_groups`, else one group), longest expected work first by
// `prev_nproc` (processed entries of a previous forward over the same
// tiles) when given, else in spatial order.  order [n_tiles] is scratch.
void launch_composite_fwd(hipStream_t st, int tw, int th, int batch, int n_tiles, int F,
                          const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                          const Record* rec, const float* bg, float* rgb, float* depth,
                          float* alpha, float* t_final, int32_t* n_last, uint32_t* nproc,
                          const uint32_t* prev_nproc, uint32_t* order, bool xcd_groups,
                          unsigned long long* pairs, int32_t* med_pos);
void launch_composite_bwd(hipStream_t st, int tw, int th, int batch, int n_tiles, int F,
                          const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                          const Record* rec, const uint2* trect, const uint32_t* keyoff,
                          const uint32_t* nproc, const float* bg, const float* g_rgb,
                          const float* g_depth, const float* g_alpha, const float* t_final,
                          const int32_t* n_last, float* partial, uint32_t* stamp,
                          const uint32_t* epoch, uint32_t* order, bool xcd_groups,
                          const int32_t* med_pos);

// loss.hip
int loss_blocks_x(int64_t max_hw);
// The static scratch of the allocation-free L1 loss: its device address on
// `device` (the current device; resolved once, then cached) and its size.
hipError_t loss_scratch_init(int device, void** out);
size_t loss_scratch_bytes();
void launch_loss_l1(hipStream_t st, int F, int blocks_x, const FrameDesc* frames,
                    const float* rgb, const float* depth, const float* t_rgb,
                    const float* t_depth, float depth_weight, double* part, float* scale,
                    float* loss, float* g_rgb, float* g_depth, float* g_alpha);

// ssim.hip: rendering loss with SSIM.  tile_sums holds 4 doubles per padded
// block tile of every plane [F][3][tiles_pad]; part 3 x 3 * total_px doubles
// (the SSIM map's derivatives A, B, C per colour value); frame_sums [F][4]
// doubles (gradient scales and loss term per frame).
int ssim_tiles_pad(int max_w, int max_h);
void launch_loss_render(hipStream_t st, int F, int tiles_pad, const FrameDesc* frames,
                        int64_t total_px, const float* rgb, const float* depth,
                        const float* t_rgb, const float* t_depth, float lambda1, float lambda2,
                        double* part, double* tile_sums, double* frame_sums, float* loss,
                        float* ssim, float* g_rgb, float* g_depth, float* g_alpha);

// densify.hip: ADC statistics of the last backward (grad2d [m][kNG], ntiles
// [m], record r = f n + g), MCMC position noise and relocation.  src [n]:
// the live source of each dead Gaussian, -1 (or out of range) otherwise;
// cnt [n] (uint32) and rule [n][4] (double) are scratch.
void launch_densify_stats(hipStream_t st, int64_t n, int F, const uint32_t* ntiles,
                          const double* grad2d, float* grad_accum, float* count);
void launch_mcmc_noise(hipStream_t st, int64_t n, float* means, const float* log_scales,
                       const float* quats, const float* opac, const float* eps, float scale);
void launch_mcmc_relocate(hipStream_t st, int64_t n, int ksh3, float* means, float* log_scales,
                          float* quats, float* opac, float* sh, const int32_t* src,
                          uint32_t* cnt, double* rule);

// The compositing tile schedule (raster.hip): `order` lists the tiles group
// by group, longest first by `nproc` (entries a previous pass processed per
// tile; spatial order if NULL); launch tile_schedule_grid() workgroups.
void launch_tile_order(hipStream_t st, int n_tiles, int groups, const uint32_t* nproc,
                       uint32_t* order);
unsigned tile_schedule_grid(int n_tiles, int groups);
int tile_schedule_groups(bool xcd_groups);

// Sum of the per-wave twist partials [F][n_waves][6] into g_twist [F][6].
void launch_twist_reduce(hipStream_t st, int F, const double* twist_partial, int64_t n_waves,
                         float* g_twist);

// surfel.hip: the 2D surfel variant's preprocess (records of
// surfel_record_bytes() bytes in `rec`), forward compositing (rgb, depth,
// alpha, normal [sum 3HW], distortion; dist_aux [P][4] keeps the per-pixel
// reference depth and the distortion sums A, D_1, D_2 the backward needs) and backward (per-key partials of
// surfel_grad_values() floats, then the chain rule and twist); keys, sorts
// and ranges are shared.
size_t surfel_record_bytes();
size_t surfel_square_offset();  // byte offset of the box bounds sqx, sqy
int surfel_grad_values();
int64_t surfel_preprocess_bwd_waves(int64_t n);
void launch_surfel_preprocess(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                              const float* poses, const float* means, const float* log_scales,
                              const float* quats, const float* opac, const float* sh, int deg,
                              int tile_w, int tile_h, void* rec, uint2* trect,
                              uint32_t* depth_key, uint32_t* rec_id, uint32_t* ntiles);
void launch_surfel_fwd(hipStream_t st, int tw, int th, int n_tiles, int F,
                       const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                       const void* rec, const float* bg, float* rgb, float* depth, float* alpha,
                       float* normal, float* dist, float* t_final, int32_t* n_last,
                       float* dist_aux, uint32_t* nproc, const uint32_t* prev_nproc,
                       uint32_t* order, bool xcd_groups, unsigned long long* pairs);
void launch_surfel_bwd(hipStream_t st, int tw, int th, int n_tiles, int F,
                       const FrameDesc* frames, const uint2* ranges, const uint32_t* vals,
                       const void* rec, const uint2* trect, const uint32_t* keyoff,
                       const float* bg, const float* g_rgb, const float* g_depth,
                       const float* g_alpha, const float* g_normal, const float* g_dist,
                       const float* t_final, const int32_t* n_last, const float* dist_aux,
                       float* partial, uint32_t* stamp, const uint32_t* epoch,
                       const uint32_t* nproc, uint32_t* order, bool xcd_groups);
// Per-record sums of the stamped key partials, records in `order` (sorted by
// tile count so that a wave's groups do similar work): sgrad [m][values].
void launch_surfel_slot_reduce(hipStream_t st, uint64_t m, const uint32_t* order,
                               const uint32_t* keyoff, const uint32_t* ntiles,
                               const float* partial, const uint32_t* stamp,
                               const uint32_t* epoch, uint64_t key_capacity, double* sgrad);
void launch_surfel_preprocess_bwd(hipStream_t st, int64_t n, int F, const FrameDesc* frames,
                                  const float* poses, const float* means,
                                  const float* log_scales, const float* quats,
                                  const float* opac, const float* sh, int deg,
                                  const uint32_t* ntiles, const uint32_t* keyoff,
                                  const double* sgrad, uint64_t key_capacity, float* g_means,
                                  float* g_log_scales, float* g_quats, float* g_opac,
                                  float* g_sh, double* twist_partial, float* g_twist);

// normals.hip: the normal-consistency term of the surfel objective on packed
// depth / alpha [sum HW] and normal [sum 3HW] images of F frames (host
// cameras); adds its gradients to g_depth, g_alpha, g_normal and writes
// loss[0]; part holds sum_f normal_consistency_blocks(W_f, H_f) doubles.
int64_t normal_consistency_blocks(int W, int H);
void launch_normal_consistency(hipStream_t st, int F, const gsr_camera* cams,
                               const float* depth, const float* alpha, const float* normal,
                               float weight, double* part, float* loss, float* g_depth,
                               float* g_alpha, float* g_normal);

// adam.hip
void launch_adam(hipStream_t st, uint64_t n3, uint64_t nsh, float* means, const float* g_means,
                 float* m_means, float* v_means, float* sh, const float* g_sh, float* m_sh,
                 float* v_sh, int n_frames, float* poses, const float* g_twist, float* m_tw,
                 float* v_tw, float lr_means, float lr_sh, float lr_pose, float beta1,
                 float beta2, float eps, int32_t* step);

}  // namespace gsr

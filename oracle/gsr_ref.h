/*
 * gsr_ref.h -- FP64 CPU oracle of the differentiable tile rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no source
 * with the HIP path (paper_2411_17660_amd/csrc): no headers, constants or
 * helpers are common to both.
 *
 * What it computes (DROID-Splat, Sec. 3.3 "Differentiable Rendering" and the
 * rendering equation eqn:rendering; the 3DGS lineage it cites supplies the
 * EWA projection and tile culling):
 *   Gaussians (mean, log-scale, quaternion wxyz, opacity logit, SH colour)
 *   + pinhole cameras + world->camera poses  ->  RGB, depth (alpha-blended,
 *   or the median depth) and accumulated alpha per frame, and the exact analytic gradients of
 *   L = <G_C, RGB> + <G_D, D> + <G_A, Alpha> with respect to every Gaussian
 *   parameter and a left-perturbation twist (rho, phi) of every pose
 *   (Sec. 3.3 last paragraph; supplementary S1.3 "Feedback").
 * Where the paper is silent the readings are stated at each step below.
 *
 * All internal arithmetic is IEEE double; inputs are FP32 values widened.
 */
#ifndef GSR_REF_H
#define GSR_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  REF_OK = 0,
  REF_ERR_INVALID_ARGUMENT = 1,
  REF_ERR_OUT_OF_MEMORY = 3,
  REF_ERR_STATE = 5
};

typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy, near_z;
} ref_camera;

typedef struct {
  int32_t sh_degree;      /* 0..3 */
  float background[3];
  int32_t tile_w, tile_h; /* any positive sizes; results do not depend on them */
  int32_t n_threads;      /* OpenMP threads; <= 0 means 1 */
  int32_t depth_mode;     /* REF_DEPTH_BLENDED or REF_DEPTH_MEDIAN */
} ref_settings;

/* Depth output.  BLENDED: D = sum_i z_i a_i T_i.  MEDIAN (the depth at
 * which the pixel's transmittance first falls below 1/2): D = z_k of the
 * first blended entry k with T_k (1 - a_k) < 1/2, or 0 where T never falls
 * below 1/2; its gradient reaches that entry's z only (the choice of k is
 * piecewise constant). */
#define REF_DEPTH_BLENDED 0
#define REF_DEPTH_MEDIAN 1

/* Per-pixel flag bits: pixels whose discrete decisions sit so close to a
 * threshold that FP32 rounding on another implementation may flip them. */
#define REF_FLAG_ALPHA_BAND 1u   /* some evaluated entry has |a - A_MIN| < b_a A_MIN,
                                    b_a = max(1e-4, 8 eps32 (A dx^2 + 2|B dx dy| + C dy^2)) */
#define REF_FLAG_T_BAND 2u       /* some blend candidate has |T' - T_MIN| < b_t T_MIN,
                                    b_t = max(1e-4, 4 eps32 (blended so far + 1))      */
#define REF_FLAG_CLAMP_BAND 4u   /* some blended entry has |s G - A_MAX| < 1e-4 A_MAX   */
#define REF_FLAG_MEDIAN_BAND 8u  /* median mode: some blended entry has |T' - 1/2| < b_t / 2 */

typedef struct ref_state ref_state;

/* Forward render.  Outputs are caller-owned host arrays, packed per frame:
 * rgb [sum_f 3*H_f*W_f] (CHW per frame), depth and alpha [sum_f H_f*W_f].
 * On success *state receives the saved state for ref_backward and the
 * debug accessors; free it with ref_free.  n == 0 is valid. */
int ref_forward(const ref_settings* s, int64_t n, const float* means,
                const float* log_scales, const float* quats,
                const float* opacity_logits, const float* sh, int32_t n_frames,
                const ref_camera* cams, const float* poses, double* rgb,
                double* depth, double* alpha, ref_state** state);

/* Same with FP64 inputs (finite-difference pins perturb below FP32 resolution). */
int ref_forward_f64(const ref_settings* s, int64_t n, const double* means,
                    const double* log_scales, const double* quats,
                    const double* opacity_logits, const double* sh, int32_t n_frames,
                    const ref_camera* cams, const double* poses, double* rgb,
                    double* depth, double* alpha, ref_state** state);

/* Backward of L = <g_rgb,RGB> + <g_depth,D> + <g_alpha,Alpha>.  Gradient
 * outputs are overwritten: g_means [n,3], g_log_scales [n,3], g_quats [n,4],
 * g_opacity_logits [n], g_sh [n,(d+1)^2,3], g_twist [F,6] = (rho, phi). */
int ref_backward(ref_state* st, const double* g_rgb, const double* g_depth,
                 const double* g_alpha, double* g_means, double* g_log_scales,
                 double* g_quats, double* g_opacity_logits, double* g_sh,
                 double* g_twist);

void ref_free(ref_state* st);

/* ---- debug accessors (integer artefacts and intermediates) ---- */
int64_t ref_num_keys(const ref_state* st);
int64_t ref_num_tiles(const ref_state* st);
int64_t ref_num_pixels(const ref_state* st);
int64_t ref_pairs_evaluated(const ref_state* st); /* (pixel, entry) alpha-box hits */

/* Per record r = f*n + g:
 * ints[r*14 + :] = keep, x_lo, x_hi, y_lo, y_hi, tx_lo, tx_hi, ty_lo, ty_hi, n_tiles,
 *                   bx_lo, bx_hi, by_lo, by_hi
 *   (x/y: the 3-sigma pixel square; bx/by: the square clipped to the
 *   bounding box of {alpha >= 1/255}; tx/ty: the tiles of bx/by)
 * depth_bits[r]  = bits of fp32(z) (0 when culled)
 * vals[r*20 + :] = u, v, z, A, B, C, s_xx, s_xy, s_yy, lambda_max, radius,
 *                  opacity, c_r, c_g, c_b, raw_r, raw_g, raw_b, det, tz */
void ref_records(const ref_state* st, int32_t* ints, uint32_t* depth_bits,
                 double* vals);
/* tile_start [T+1] (CSR over global tile ids), entries [K] = g of each key. */
void ref_tile_lists(const ref_state* st, int64_t* tile_start, int32_t* entries);
/* Per pixel (packed like depth): flags, n_last (list position after the last
 * blended entry of the pixel's tile list), T_final. */
void ref_pixel_info(const ref_state* st, uint8_t* flags, int32_t* n_last,
                    double* t_final);
/* Screen-space gradients of every record accumulated by the last
 * ref_backward, [F*n][10]: dL/du, dL/dv, dL/dA, dL/dB, dL/dC (conic
 * q = A dx^2 + 2 B dx dy + C dy^2), dL/dopacity (of alpha = opacity G),
 * dL/dcolour[3], dL/dz.  Returns REF_ERR_STATE before the first backward. */
int ref_screen_grads(const ref_state* st, double* out);
/* Hash of every discrete decision (squares, tile lists, per-pixel blended
 * sets and stop positions, clamp states). */
uint64_t ref_decision_hash(const ref_state* st);

/* ---- building blocks exposed for pins ---- */
void ref_quat_to_rotmat(const double* q_wxyz, double* R /*row-major 3x3*/);
void ref_sh_basis(int32_t degree, const double* dir, double* out /*(d+1)^2*/);
void ref_sh_basis_grad(int32_t degree, const double* dir,
                       double* out /*(d+1)^2 x 3*/);

#ifdef __cplusplus
}
#endif
#endif

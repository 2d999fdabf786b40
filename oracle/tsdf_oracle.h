/*
 * tsdf_oracle.h -- CPU oracle for projective TSDF integration.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the test-suite, the smoke check and the benchmark's CPU-baseline leg compare
 * the HIP library against.  The product library never includes, links or
 * calls anything in this directory, and this directory includes nothing from
 * the product.
 *
 * What it computes (nvblox paper, §IV-B "Frame Integration", Eq. (1)-(2) and
 * the TSDF update functor that follows them):
 *   for each depth frame (pose T_LC, pinhole intrinsics), every voxel centre
 *   p_L is moved into the camera frame with T_CL = T_LC^{-1}, projected with
 *   the pinhole model, the depth image is sampled at the nearest pixel, the
 *   projective distance d_p = d - z is truncated, weighted, and folded into the
 *   voxel by a weighted average whose weight sum is capped.
 *   Blocks of 8x8x8 voxels are kept in a hash map (§IV-A) and a block exists
 *   once any of its voxels has been updated.
 *
 * Every routine is compiled twice: in binary32 (the parity oracle: the same
 * operations, in the same order, as the GPU library is required to perform)
 * and in binary64 (the error oracle).  Selected by `precision` = 32 or 64.
 *
 * Readings of points the paper leaves open (pixel convention, which voxels are
 * skipped behind the surface, the dropoff weight, the range limit, operation
 * order) are listed in the repository's design notes and restated next to the
 * code that implements them.
 */
#ifndef TSDF_ORACLE_H
#define TSDF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORA_WEIGHT_CONSTANT = 0, ORA_WEIGHT_LINEAR_DROPOFF = 1 };

typedef struct ora_map ora_map;

/* A new empty map.  voxel_size in metres, truncation in voxels
 * (epsilon = truncation_vox * voxel_size), max_weight caps the stored weight,
 * max_range bounds valid measurements (0 < d <= max_range).
 * Returns NULL on bad arguments or out of memory. */
ora_map *ora_create(int precision, float voxel_size, float truncation_vox,
                    float max_weight, float max_range, int weighting);
void ora_destroy(ora_map *m);

/* binary16 voxel storage for a binary32 map (precision 32 only, before the
 * first frame): after every update the stored distance and weight are
 * rounded to the nearest binary16 value, ties to even; the update arithmetic
 * stays binary32.  Returns 0, or -1 if not allowed. */
int ora_set_storage16(ora_map *m);

/* The binary16 value nearest to x (ties to even, overflow to infinity), as a
 * binary32; NaN, infinities and zeros pass through. */
float ora_round_binary16(float x);

/* Integrates one depth frame (row-major float32, width x height, metres) seen
 * from T_world_cam (row-major 4x4 float32) with K = {fx, fy, cx, cy}.
 * Returns the number of voxel updates, or -1 on bad arguments / no memory. */
long long ora_integrate_depth(ora_map *m, const float *depth, int width, int height,
                              const float K[4], const float T_world_cam[16]);
/* ora_integrate_depth on `threads` (>= 1) OpenMP threads: the blocks of the
 * scan box are measured in parallel, inserted one by one in the same scan
 * order and fused in parallel, so the map is bitwise the single-threaded one.
 * For timing the CPU baseline on all host cores. */
long long ora_integrate_depth_threads(ora_map *m, const float *depth, int width, int height,
                                      const float K[4], const float T_world_cam[16], int threads);
/* Same frame, with the paper-literal allocation: the blocks visited by a
 * walk through the block grid (Amanatides & Woo) along every valid pixel's
 * centre ray, from the camera to min(d + epsilon, max range), are allocated
 * (even when none of their voxels is updated) and integrated; voxels of other
 * blocks are not updated.  The touched list is the visited set. */
long long ora_integrate_depth_dda(ora_map *m, const float *depth, int width, int height,
                                  const float K[4], const float T_world_cam[16]);

/* Same, with this frame's own max range (> 0) in place of the map's. */
long long ora_integrate_depth_range(ora_map *m, const float *depth, int width, int height,
                                    const float K[4], const float T_world_cam[16], float max_range);

/* Integrates one spherical range image (Eq. (3); row-major float32,
 * width columns of azimuth x height rows of polar angle, Euclidean range in
 * metres) seen from T_world_sensor (sensor frame: x forward, y left, z up).
 * model = {azimuth start, azimuth field of view, polar start (from +z),
 * polar field of view, largest interpolated spread, max range (0: the
 * map's)}, angles in radians.  Returns the number of voxel updates or -1. */
long long ora_integrate_range(ora_map *m, const float *range, int width, int height,
                              const float model[6], const float T_world_sensor[16]);

/* Dense brute force of ora_integrate_range over the voxel box
 * [gmin, gmin + gdim), as ora_dense_integrate. */
long long ora_dense_integrate_range(int precision, float voxel_size, float truncation_vox, float max_weight,
                                    float max_range, int weighting, const float *range, int width, int height,
                                    const float model[6], const float T_world_sensor[16], const int32_t gmin[3],
                                    const int32_t gdim[3], double *dist, double *weight);

/* binary32 atan2 the binary32 oracle uses for Eq. (3) (Abramowitz & Stegun
 * 4.4.49 with octant reduction). */
float ora_atan2_f32(float y, float x);

long long ora_num_blocks(const ora_map *m);
/* Block indices (x, y, z), 3 int32 per block, in insertion order. */
void ora_blocks(const ora_map *m, int32_t *xyz);
/* Voxel distance and weight, 512 per block in insertion order, voxel
 * (lx, ly, lz) at lx + 8 ly + 64 lz.  binary32 values widen exactly. */
void ora_voxels(const ora_map *m, double *dist, double *weight);
/* Insertion index of block (x, y, z), or -1. */
long long ora_find_block(const ora_map *m, int32_t x, int32_t y, int32_t z);
/* Blocks updated by the last integrated frame; returns their count and, if
 * xyz is non-NULL, writes them (3 int32 each). */
long long ora_touched(const ora_map *m, int32_t *xyz);
/* Inclusive block-index box that the last frame scanned (its candidates). */
void ora_last_scan(const ora_map *m, int32_t bmin[3], int32_t bmax[3]);

/* Camera-from-world transform the oracle uses for Eq. (1), as doubles
 * (binary32 values when precision == 32). */
void ora_camera_from_world(int precision, const float T_world_cam[16], double R[9], double t[3]);

/* Dense brute force over the voxel box [gmin, gmin + gdim): no blocks, no hash,
 * no candidate set.  dist/weight (gdim[0]*gdim[1]*gdim[2] each, x fastest)
 * carry the state in and out.  Returns the number of voxel updates. */
long long ora_dense_integrate(int precision, float voxel_size, float truncation_vox,
                              float max_weight, float max_range, int weighting,
                              const float *depth, int width, int height,
                              const float K[4], const float T_world_cam[16],
                              const int32_t gmin[3], const int32_t gdim[3],
                              double *dist, double *weight);


/* ---- learned sensor model (see sensor_model_impl.h for the definition) ---- */

/* Number of parameters of the 27 -> 32 -> 32 -> 2 perceptron. */
#define ORA_SM_NPARAM 2018

/* The bfloat16 value nearest to x (ties to even), as a binary32. */
float ora_round_bf16(float x);

/* The 27 binary32 input features of every pixel (H x W x 27, zeros for
 * invalid pixels). */
void ora_sm_features(const float *depth, int width, int height, const float K[4], float max_range, float *feat);

/* Per-pixel weight and truncation maps of a depth frame under the
 * bfloat16-emulating binary32 forward (0 for invalid pixels).  params holds
 * ORA_SM_NPARAM bfloat16-representable values.  Returns 0 or -1. */
int ora_sm_maps(const float *depth, int width, int height, const float K[4], float max_range, float voxel_size,
                const float *params, float *w_map, float *eps_map);

/* Integrates a pinhole frame with per-pixel weights and truncation distances
 * in place of the map's weighting and epsilon.  Returns updates or -1. */
long long ora_integrate_learned(ora_map *m, const float *depth, int width, int height, const float K[4],
                                const float T_world_cam[16], const float *w_map, const float *eps_map);

/* Training loss of the sensor model over a window of frames (n_frames depth
 * images, row-major, and poses) against target distances of n_vox voxels
 * (global voxel indices, 3 int32 each), in binary64; writes dL/dparams
 * (ORA_SM_NPARAM doubles) and the number of voxels the prediction reaches.
 * emulate_bf16 rounds inputs and hidden activations to bfloat16.  Returns the
 * loss, or -1 when out of memory. */
double ora_sm_loss_grad(const float *params, int n_frames, const float *depths, int width, int height,
                        const float K[4], const float *T_world_cam, float voxel_size, float max_range,
                        long long n_vox, const int32_t *vox, const double *target, int emulate_bf16,
                        double *grad, long long *n_used);

#ifdef __cplusplus
}
#endif
#endif

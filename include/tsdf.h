/*
 * tsdf.h -- C ABI of the MI355X (gfx950) projective-TSDF integration library.
 *
 * The library implements the surface-reconstruction hot path of the nvblox
 * paper (Millane et al., "nvblox: GPU-Accelerated Incremental Signed Distance
 * Field Mapping"): a block-sparse TSDF layer (§IV-A: a GPU hash table from
 * integer block index to 8x8x8-voxel blocks stored contiguously) into which
 * depth frames are fused by projective integration (§IV-B: find the blocks in
 * view, allocate the missing ones, project every voxel into the depth image,
 * Eq. (1)-(2), and apply the truncated weighted-average TSDF update).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Frames.  T_world_cam is the sensor pose T_LC of §III: a row-major 4x4
 *   float32 rigid transform taking camera coordinates to world (layer)
 *   coordinates.  Camera frame: x right, y down, z forward.  A depth image
 *   stores camera-frame z in metres.
 * Voxels.  Voxel (gx, gy, gz) has its centre at ((g + 0.5) * voxel_size).
 *   Block (bx, by, bz) holds voxels 8b .. 8b+7 on each axis; inside a block
 *   voxel (lx, ly, lz) is stored at index lx + 8 ly + 64 lz.
 *   Block indices must stay within [-(2^20 - 1), 2^20 - 1] on every axis.
 * Pixels.  Pixel (i, j) covers [i, i+1) x [j, j+1); the depth image is
 *   row-major, height rows of width float32 values.  A pixel is a valid
 *   measurement iff 0 < d <= max_range; anything else (0, negative, NaN, Inf,
 *   beyond range) is skipped and is not an error.
 * Memory.  Pointers named *_dev are device pointers on the map's GPU; all
 *   other pointers are host memory, read or written during the call only.
 *   The map owns all of its device memory.  Device buffers passed in stay
 *   owned by the caller and must stay alive until the stream has passed the
 *   call.
 * Streams.  hip_stream is a hipStream_t (NULL = the default stream).  Calls
 *   that only enqueue GPU work return before it has run.  A map is not
 *   thread-safe: calls on one map must be ordered on one stream.
 * Errors.  Every function returns TSDF_OK (0) or a negative status; no
 *   exception crosses the ABI.  Device-side overflow (block pool, hash table,
 *   touched list) sets a sticky error word on the device that map_status()
 *   and the synchronising queries report as TSDF_EFULL; once observed, the
 *   map rejects further integration with TSDF_ESTATE until reserve() grows it.
 */
#ifndef TSDF_H
#define TSDF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define TSDF_API __attribute__((visibility("default")))
#else
#define TSDF_API
#endif

#define TSDF_OK 0
#define TSDF_EINVAL (-1)   /* bad argument: NULL pointer, size <= 0, non-finite or non-rigid pose, ... */
#define TSDF_ENOMEM (-2)   /* device allocation failed */
#define TSDF_EFULL (-3)    /* block pool, hash table or touched list overflowed (sticky) */
#define TSDF_EDEVICE (-4)  /* a HIP runtime call failed */
#define TSDF_ESTATE (-5)   /* the map is in a sticky error state */
#define TSDF_ESCRATCH (-6) /* integrate_depth_noalloc: the call needs more than its fixed scratch */

#define TSDF_WEIGHT_CONSTANT 0        /* f_w(d_p) = 1 */
#define TSDF_WEIGHT_LINEAR_DROPOFF 1  /* 1 for d_p >= -voxel_size, then linear to 0 at -epsilon */
#define TSDF_WEIGHT_LEARNED 2         /* per-pixel weight and truncation from the learned sensor
                                         model (tsdf_set_sensor_model); pinhole views only */

/* Allocation.  TSDF_ALLOC_EXACT: a frame allocates exactly the blocks in
 * which it updates at least one voxel.  TSDF_ALLOC_RAY_WALK: the paper's
 * literal rule (§IV-B: blocks in view are found by ray tracing through the
 * block grid, Amanatides & Woo): the blocks entered by the ray from the camera
 * through each valid pixel's centre, from depth 0 to min(d + epsilon,
 * max_range), are allocated whether or not a voxel of theirs is updated, and
 * voxels are updated only inside them (ties step x, then y, then z; a block
 * boundary exactly at the end depth is crossed).  The touched list is then the
 * visited set.  Ray-walk maps accept integrate_depth only (TSDF_EINVAL for
 * range images, batches and graph steps). */
#define TSDF_ALLOC_EXACT 0
#define TSDF_ALLOC_RAY_WALK 1

#define TSDF_STORAGE_FP32 0   /* (distance, weight) as two binary32: 8 B per voxel, 4 KiB per block */
#define TSDF_STORAGE_FP16 1   /* two binary16, rounded to nearest-even after each binary32 update:
                                 4 B per voxel, 2 KiB per block */

typedef struct tsdf_map tsdf_map;

typedef struct {
    float voxel_size_m;        /* voxel edge, metres, > 0 */
    float truncation_vox;      /* truncation distance epsilon in voxels, > 0 (epsilon = truncation_vox * voxel_size_m) */
    float max_weight;          /* cap on the stored weight, > 0 */
    float max_range_m;         /* measurements d > max_range_m are invalid, > 0 */
    int weighting;             /* TSDF_WEIGHT_* */
    int storage;               /* TSDF_STORAGE_*; the update arithmetic is binary32 either way */
    long long block_capacity;  /* number of 8^3-voxel blocks the pool holds, >= 1 */
    long long hash_capacity;   /* hash slots; 0 = smallest power of two >= 2 * block_capacity */
    int allocation;            /* TSDF_ALLOC_*: which blocks a frame allocates */
    int reserved;              /* 0 */
} tsdf_params;

/* Fills *p with the defaults: max_weight 100, max_range 5 m, constant weight,
 * binary32 storage, 2^18 blocks (1 GiB of voxels), automatic hash size. */
TSDF_API void tsdf_default_params(tsdf_params *p, float voxel_size_m, float truncation_vox);

/* Creates an empty map on the current HIP device (§IV-A).  create_map uses
 * the defaults above.  *out receives the handle; on failure *out is NULL and
 * the status is TSDF_EINVAL (bad parameters), TSDF_ENOMEM or TSDF_EDEVICE.
 * Synchronises the device once (initial clears). */
TSDF_API int create_map(float voxel_size_m, float truncation_vox, tsdf_map **out);
TSDF_API int create_map_ex(const tsdf_params *p, tsdf_map **out);

/* Frees the map and all its device memory after the device is idle.  NULL is
 * accepted (TSDF_OK). */
TSDF_API int destroy_map(tsdf_map *m);

/* Grows the map to hold block_capacity blocks (§IV-A: the block hash and the
 * block storage behind it).  The block pool is reallocated and every block
 * keeps its pool slot, voxels and touched-list entry; the hash grows to the
 * smallest power of two at least twice the new block capacity (it never
 * shrinks) and every allocated block's key is re-inserted into it on the
 * device.  Graphs captured by the map's steps (tsdf_step_*) are dropped and
 * re-captured on their next run.  A capacity not above the current one
 * changes nothing and returns TSDF_OK.
 * Recovery: reserve also clears a sticky TSDF_EFULL.  The calls that
 * overflowed did not update the blocks they could not allocate (those blocks
 * miss those calls' measurements; every other block is exact), so a caller
 * that needs an exact map reserves ahead of time (map_stats: blocks against
 * block_capacity) rather than after an overflow.
 * Synchronises the device, and must not be called while any stream is being
 * captured into a graph (TSDF_ESTATE, the map unchanged).  block_capacity:
 * 1 .. 2^30.  Errors: TSDF_EINVAL, TSDF_ESTATE, TSDF_ENOMEM (the map
 * unchanged), TSDF_EDEVICE. */
TSDF_API int reserve(tsdf_map *m, long long block_capacity);

/* Fuses one depth frame into the map (§IV-B, Eq. (1)-(2) and the TSDF update
 * functor):
 *   for every voxel v with centre p: p_C = T_CL p (T_CL = T_world_cam^{-1});
 *   if z > 0 and (u, v) = (fx x/z + cx, fy y/z + cy) falls in the image, the
 *   nearest pixel's depth d is valid, d_p = d - z >= -epsilon and the weight
 *   w = f_w(d_p) > 0, then with x = min(d_p, epsilon):
 *     D <- (D W + x w) / (W + w),   W <- min(W + w, max_weight).
 *   A block is allocated (zero distance, zero weight) the first time any of
 *   its voxels is updated; the blocks updated by this frame form the touched
 *   list (query_touched).
 * depth_dev: device float32[height][width], width * height <= 2^28.  K: host {fx, fy, cx, cy} with
 * fx, fy > 0.  T_world_cam: host row-major 4x4; its bottom row must be
 * (0 0 0 1) within 1e-6 and its rotation orthonormal within 1e-4.
 * Only enqueues work on hip_stream (no host synchronisation).
 * Errors: TSDF_EINVAL, TSDF_ESTATE, TSDF_EDEVICE. */
TSDF_API int integrate_depth(tsdf_map *m, const float *depth_dev, int width, int height,
                    const float K[4], const float T_world_cam[16], void *hip_stream);

/* integrate_depth for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, semantics and result as integrate_depth (the map afterwards
 * is bit-identical), and the map is still created by create_map_ex; but the
 * scratch integrate_depth allocates in the map on first use (the frame's
 * depth footprint pyramid and the candidate-block list of a compacted launch)
 * comes from one fixed device array of the library instead, about 9.3 MiB
 * per GPU (a pyramid of one image up to 4096 pixels a side, then 2^20
 * candidate entries), held on each GPU the function is used on until the
 * process ends.  The call makes no device allocation and no free.  Its first
 * call on a GPU looks the array's address up (hipGetSymbolAddress) with the
 * map's device current.
 * Limits: a frame whose candidate list could exceed 2^20 blocks (its block
 * lattice, the world box of the frustum out to max range + epsilon, holds
 * more than 2^20 blocks and the launch is compacted) is rejected with
 * TSDF_ESCRATCH before any work is enqueued.  Maps with learned weighting or
 * ray-walk allocation need per-map buffers and are rejected with
 * TSDF_EINVAL.  Kernel timing (tsdf_profile) does not record these calls.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams, maps or threads, not ordered on one stream) race on it
 * and give wrong maps; order them.  Nothing in the array needs clearing
 * between calls (each call rewrites what it reads).
 * Errors: those of integrate_depth, and TSDF_ESCRATCH. */
TSDF_API int integrate_depth_noalloc(tsdf_map *m, const float *depth_dev, int width, int height,
                                     const float K[4], const float T_world_cam[16], void *hip_stream);

/* A rotating LiDAR's range image (§III: Omega is the beam angles; Eq. (3)).
 * Row-major float32[height][width] of Euclidean ranges in metres; sensor frame
 * x forward, y left, z up.  Column i covers azimuths (atan2(y, x)) from
 * azimuth_start + i / alpha to azimuth_start + (i + 1) / alpha with
 * alpha = width / azimuth_fov; row j covers polar angles (from +z) from
 * polar_start + j / beta with beta = height / polar_fov; each beam sits at the
 * centre of its pixel.  A voxel's range is interpolated bilinearly between
 * the 4 beams around its direction, only when all 4 are valid and differ by
 * at most interp_max_diff_m (no interpolation across depth edges); the voxel
 * depth d_v is the Euclidean range of the voxel centre.  azimuth_fov >= 2 pi
 * (binary32 2 pi) makes columns wrap around. */
typedef struct {
    int width, height;            /* >= 2 each */
    float azimuth_start_rad;      /* finite */
    float azimuth_fov_rad;        /* (0, 2 pi] */
    float polar_start_rad;        /* [0, pi) */
    float polar_fov_rad;          /* > 0, polar_start + polar_fov <= pi */
    float interp_max_diff_m;      /* >= 0 */
    float max_range_m;            /* valid ranges are <= this; 0 = the map's max range */
} tsdf_lidar_model;

/* Fuses one range image into the map: integrate_depth with the spherical
 * projection of Eq. (3) in place of the pinhole and the interpolated range in
 * place of the nearest depth.  T_world_sensor as T_world_cam.  Only enqueues
 * work; errors as integrate_depth. */
TSDF_API int integrate_range(tsdf_map *m, const float *range_dev, const tsdf_lidar_model *lidar,
                             const float T_world_sensor[16], void *hip_stream);

/* One view of a batch: a depth or range image, its sensor model and its pose,
 * with the meaning and constraints of integrate_depth / integrate_range. */
#define TSDF_MAX_VIEWS 16
#define TSDF_MODEL_PINHOLE 0
#define TSDF_MODEL_SPHERICAL 1
typedef struct {
    const float *depth_dev;    /* device float32[height][width]: z-depth (pinhole) or range (spherical) */
    int width, height;
    int model;                 /* TSDF_MODEL_PINHOLE or TSDF_MODEL_SPHERICAL */
    float max_range_m;         /* valid measurements are <= this; 0 = the map's max range */
    float K[4];                /* pinhole: fx, fy, cx, cy; spherical: azimuth start, azimuth fov,
                                  polar start, polar fov (radians) */
    float interp_max_diff_m;   /* spherical: as in tsdf_lidar_model; pinhole: must be 0 */
    float reserved;            /* must be 0 */
    float T_world_cam[16];     /* row-major rigid pose */
} tsdf_depth_view;

/* Fuses n_views (1 .. TSDF_MAX_VIEWS) depth views in one launch.  The map
 * afterwards is bit-identical to calling integrate_depth on views[0],
 * views[1], ... in that order (§IV-B applied per view, per voxel, in order);
 * the views may be consecutive frames of one camera or the cameras of a rig,
 * of different sizes.  Each voxel's state is read once and written once per
 * call.  The touched list (query_touched) holds the blocks updated by any of
 * the views.  Only enqueues work; errors as integrate_depth. */
TSDF_API int integrate_depth_views(tsdf_map *m, const tsdf_depth_view *views, int n_views, void *hip_stream);

/* A batched step replayed from a hipGraph.  A step holds graphs of
 * [a copy of the step's launch arguments from pinned host memory to device
 * memory] + [the kernels of integrate_depth_views reading them: footprint
 * pre-pass, cull kernel and integration kernel, as the launch shape selects]
 * for two staging slots used alternately; each variant is captured and
 * instantiated on its first use (tsdf_step_create captures the plain one).
 * tsdf_step_run validates the views, writes the arguments and launches one
 * graph on hip_stream: the same result as integrate_depth_views, with one
 * graph launch as the only per-step submission.  with_spherical must be nonzero for steps holding range images.
 * A step belongs to its map and must be destroyed before it; runs on one map
 * must be ordered on one stream.  tsdf_step_run may wait for the replay before
 * last to finish (it reuses that one's staging slot). */
typedef struct tsdf_step tsdf_step;
TSDF_API int tsdf_step_create(tsdf_map *m, int with_spherical, tsdf_step **out);
TSDF_API int tsdf_step_run(tsdf_step *step, const tsdf_depth_view *views, int n_views, void *hip_stream);
TSDF_API int tsdf_step_destroy(tsdf_step *step);

/* Writes the indices of all allocated blocks, sorted ascending by (x, y, z),
 * as int32 triples to out_xyz_dev (room for `capacity` blocks; min(count,
 * capacity) are written) and the total count to *out_count (host).
 * Synchronises hip_stream.  (§IV-A: the set of allocated blocks.)  The sort's
 * work buffers belong to the map and are allocated on the first call.  A map
 * in a sticky error state can still be read (TSDF_OK; map_status reports the
 * state): it holds every block it could allocate.  Errors: TSDF_EINVAL (NULL
 * map or count, capacity < 0, NULL buffer with capacity > 0), TSDF_ENOMEM
 * (the work buffers), TSDF_EDEVICE. */
TSDF_API int query_blocks(tsdf_map *m, int32_t *out_xyz_dev, long long capacity, long long *out_count,
                 void *hip_stream);

/* Gathers the voxels of n_blocks blocks (int32 triples at blocks_xyz_dev):
 * the sampled field Phi of §III, the fused distance D and weight W of each
 * voxel, read through the block hash (§IV-A: block index -> block of 8^3
 * voxels stored contiguously).  out_dist_dev and out_weight_dev receive 512
 * float32 each per block in voxel order lx + 8 ly + 64 lz (binary16 storage
 * widens exactly), zeros for blocks that are not allocated and for indices
 * outside the block-index range.  All three buffers are caller-owned device
 * memory of n_blocks triples / n_blocks * 512 floats.
 * Only enqueues work.  Errors: TSDF_EINVAL (NULL map, n_blocks < 0, NULL
 * buffers with n_blocks > 0), TSDF_EDEVICE. */
TSDF_API int query_tsdf(tsdf_map *m, const int32_t *blocks_xyz_dev, long long n_blocks,
               float *out_dist_dev, float *out_weight_dev, void *hip_stream);

/* Writes n_blocks blocks into the map, each found or inserted in the block
 * hash as integration inserts blocks (§IV-A: block index -> block of 8^3
 * voxels): blocks_xyz_dev holds int32 triples, dist_dev and weight_dev 512
 * floats per block in the order query_tsdf writes them (voxel lx + 8 ly +
 * 64 lz), all caller-owned device memory read on hip_stream.  With
 * query_blocks and query_tsdf it saves and restores a map: the restored map
 * holds the same blocks and voxel values (binary16 storage rounds values that
 * are not binary16 numbers to nearest), and later integration continues from
 * them; the touched list and the running counters other than the block count
 * are not part of it.  A block already in the map is overwritten; each block
 * should appear once (duplicates race, one of their values wins).  Blocks
 * outside the block-index range are skipped.  A full pool or hash sets the
 * sticky TSDF_EFULL, reported by map_status and the next integration call
 * (reserve ahead: map_stats gives blocks and block_capacity).  Only enqueues.
 * Errors: TSDF_EINVAL (NULL map, n_blocks < 0, NULL buffers with n_blocks >
 * 0), TSDF_ESTATE (sticky error), TSDF_EDEVICE. */
TSDF_API int insert_blocks(tsdf_map *m, const int32_t *blocks_xyz_dev, long long n_blocks, const float *dist_dev,
                           const float *weight_dev, void *hip_stream);

/* Blocks with at least one voxel updated by the most recent integrate_depth
 * or integrate_depth_views call (the "updated blocks" that downstream layers consume, §IV-C), in
 * unspecified order, as int32 triples; same capacity / count contract as
 * query_blocks (a map in a sticky error state included).  Synchronises hip_stream. */
TSDF_API int query_touched(tsdf_map *m, int32_t *out_xyz_dev, long long capacity, long long *out_count,
                  void *hip_stream);

/* Running counters of a map. */
typedef struct {
    long long blocks;          /* allocated blocks */
    long long voxel_updates;   /* one per voxel per view that updated it */
    long long voxel_writes;    /* one per voxel per call that updated it (stores to the pool) */
    long long touched_blocks;  /* one per block per call in which any of its voxels was updated */
    long long launches;        /* integration calls enqueued */
    long long candidate_blocks;  /* one per block per call that survived culling and was measured */
    long long block_capacity;  /* blocks the pool holds (grows with reserve) */
    long long hash_capacity;   /* slots of the block hash */
    long long error_bits;      /* sticky device-side error bits (TSDF_ERR_*), 0 if healthy */
} tsdf_stats;

/* Device-side error bits behind TSDF_EFULL (tsdf_stats.error_bits). */
#define TSDF_ERR_POOL_FULL 1          /* a new block found no free pool slot */
#define TSDF_ERR_HASH_FULL 2          /* a new block's probe found no free hash slot */
#define TSDF_ERR_TOUCHED_OVERFLOW 4   /* the touched list ran out of room */
#define TSDF_ERR_INSERT_RACE 8        /* a published key's slot value never appeared (bounded wait) */
#define TSDF_ERR_WALK_OUTSIDE 16      /* a ray walk left the frame's block lattice */

/* Fills *out.  Synchronises hip_stream. */
TSDF_API int map_stats(tsdf_map *m, tsdf_stats *out, void *hip_stream);

/* Sticky device-side status: TSDF_OK or TSDF_EFULL.  Synchronises the device. */
TSDF_API int map_status(tsdf_map *m);

/* Static description of a status code (never NULL). */
TSDF_API const char *tsdf_strerror(int status);

/* Launch shape of the integration kernels (tuning only: results do not
 * depend on it).  Zero fields mean automatic.
 *   max_groups  cap on workgroups of 512 threads per launch (rounded down to a
 *               multiple of 8), 1 .. 65536; automatic: 512, and for a compacted
 *               integrate_depth launch every workgroup its list kernel keeps
 *               resident on the device (768 on MI355X);
 *   partitions  1, or 8: blocks are owned by 8 image bands, one per XCD, so
 *               each XCD reads about 1/8 of every depth image (lattice-walk
 *               launches; more than 1 turns compaction off);
 *   chunk       lattice blocks a wave culls per pass, 1 .. 64 (lattice-walk
 *               launches); 0 with one band: every thread of a workgroup culls
 *               one lattice block per pass (a workgroup's blocks strided
 *               across the lattice) and the workgroup's waves share its
 *               surviving blocks through LDS;
 *   footprint   footprint culling: a pre-pass reduces every view to the
 *               largest valid measurement per 8/16/32/64-pixel tile, and a
 *               block is skipped when its nearest point lies beyond the
 *               largest measurement under its image footprint plus epsilon
 *               (no voxel of it can be updated).  TSDF_FOOTPRINT_AUTO uses it
 *               for launches whose block lattice has at least 16384 blocks;
 *               views larger than 4096 pixels a side are never culled this way.
 *   staging     LDS staging of block depth footprints (integrate_depth with a
 *               pinhole view and constant or linear-dropoff weighting): a
 *               wave copies the pixel rectangle under its block's projected
 *               corners (widened by one pixel) into LDS with row loads when
 *               it holds at most 1024 pixels, and its voxels read their
 *               pixels there instead of gathering them from the image (§IV-B:
 *               each voxel samples its projection's nearest pixel; the values
 *               read are the same).  TSDF_STAGE_AUTO reads the image
 *               directly (faster on every workload measured); staging runs
 *               only with TSDF_STAGE_ALWAYS.
 * NULL restores the automatic choice.  Errors: TSDF_EINVAL. */
#define TSDF_FOOTPRINT_AUTO 0
#define TSDF_FOOTPRINT_NEVER 1
#define TSDF_FOOTPRINT_ALWAYS 2
#define TSDF_COMPACT_AUTO 0
#define TSDF_COMPACT_NEVER 1
#define TSDF_COMPACT_ALWAYS 2
#define TSDF_STAGE_AUTO 0
#define TSDF_STAGE_NEVER 1
#define TSDF_STAGE_ALWAYS 2
typedef struct {
    int max_groups, partitions, chunk, footprint;
    int compaction;   /* TSDF_COMPACT_*: a cull pre-pass compacts the surviving blocks into a list
                         that the integration kernel deals out evenly to its waves (automatic once
                         lattice blocks x views reach 16384, or for integrate_depth and
                         integrate_range once the lattice reaches 131072 blocks; one band only, not with ray-walk
                         allocation) */
    int staging;      /* TSDF_STAGE_* */
} tsdf_launch_config;
TSDF_API int tsdf_set_launch_config(tsdf_map *m, const tsdf_launch_config *config);

/* Kernel timing.  While enabled, every integration call (integrate_depth,
 * integrate_range, integrate_depth_views, tsdf_step_run) records a pair of HIP
 * events on its stream around all the kernels it enqueues (footprint, network
 * and ray-walk pre-passes, cull and integration kernels).  tsdf_profile_read
 * synchronises those events and returns the summed time in milliseconds and
 * the number of timed calls since the last enable; it then clears them.  At
 * most 65536 calls are kept.  The events themselves cost the stream a few
 * microseconds per call, so for throughput measure a run of calls between two
 * events of the caller's own. */
TSDF_API int tsdf_profile(tsdf_map *m, int enable);
TSDF_API int tsdf_profile_read(tsdf_map *m, double *total_ms, long long *launches);

/* ---- Learned sensor model --------------------------------------------------
 *
 * §IV-B lets the measurement weight follow the sensor's error model.  The
 * learned model is a per-pixel perceptron 27 -> 32 -> 32 -> 2 on the pixel's
 * depth neighbourhood: inputs are the 5 x 5 patch of depth differences q - d
 * (clipped to +-0.5 m, 0 outside the image or for invalid q), the depth d and
 * the incidence angle between the pixel's ray and the normal of the
 * back-projected depth (pi/2 without all four neighbours); outputs o give the
 * weight w = (o0 + sqrt(o0^2 + 4)) / 2 and the truncation distance
 * eps = voxel_size (1 + 7 s), s = (1 + o1 / sqrt(1 + o1^2)) / 2.  With weighting
 * TSDF_WEIGHT_LEARNED a voxel with projective distance d_p is updated when
 * d_p >= -eps and w > 0, with x = min(d_p, eps) and weight w, in place of the
 * map's epsilon and weighting function.
 *
 * Parameters: TSDF_SM_NPARAM binary32 values that are bfloat16 numbers (low
 * 16 bits zero), in the order W1[32][27], b1[32], W2[32][32], b2[32],
 * W3[2][32], b3[2] (row-major, output index first).  Inference rounds inputs
 * and hidden activations to bfloat16 and accumulates each dot product in
 * binary32, one fused multiply-add per term in index order from the bias. */
#define TSDF_SM_NPARAM 2018
#define TSDF_SM_MAX_FRAMES 16

/* Copies the parameters (host memory) to the map; needed before any
 * integration of a TSDF_WEIGHT_LEARNED map, which otherwise fails with
 * TSDF_EINVAL.  Waits for the device.  Errors: TSDF_EINVAL (NULL, a value that
 * is not a finite bfloat16 number), TSDF_ENOMEM, TSDF_EDEVICE.  Learned maps
 * reject range images and graph steps (TSDF_EINVAL). */
TSDF_API int tsdf_set_sensor_model(tsdf_map *m, const float *params);

/* The per-pixel (weight, truncation) pairs of one depth image: maps_dev
 * receives 2 floats per pixel, row-major; (0, 0) for invalid pixels
 * (outside 0 < d <= max_range).  params_dev: TSDF_SM_NPARAM floats in device
 * memory.  Enqueued on hip_stream.  Errors: TSDF_EINVAL, TSDF_EDEVICE. */
TSDF_API int tsdf_sensor_maps(const float *depth_dev, int width, int height, const float K[4], float max_range,
                              float voxel_size, const float *params_dev, float *maps_dev, void *hip_stream);

/* Training.  For a window of n_frames depth images (device pointers, all
 * width x height, poses T_world_cam: n_frames x 16 floats in host memory) and
 * n_vox target voxels (vox_dev: 3 int32 global voxel indices each, target_dev:
 * one float target distance each, device memory), the loss is
 *   L = (1/N) sum_v (D(v) - D*(v))^2,  D(v) = sum_f w_f x_f / sum_f w_f,
 * over the N target voxels that some frame updates under the model, x_f and w_f
 * as in integration with the pixel frame f projects v into (the fused distance
 * before any weight cap).  tsdf_sm_loss_grad writes dL/dparams to grad_dev
 * (TSDF_SM_NPARAM floats, overwritten) and, when loss_host is not NULL, waits
 * for the stream and stores {L, N} there.  The band test d_p >= -eps carries no
 * gradient; rounding to bfloat16 is differentiated as the identity.  The
 * loss and the gradient evaluate the perceptron on the matrix cores
 * (bfloat16 operands, binary32 sums in the matrix core's order), one function
 * for both, so the gradient is that of the loss computed; it differs from
 * the inference of integration and tsdf_sensor_maps (sequential binary32
 * sums) only in the rounding of the sums.  A
 * trainer holds the per-pixel work buffers of windows of up to max_frames
 * (<= TSDF_SM_MAX_FRAMES) images of one size; calls on one trainer must be
 * ordered on one stream. */
typedef struct tsdf_sm_trainer tsdf_sm_trainer;
TSDF_API int tsdf_sm_trainer_create(int width, int height, int max_frames, tsdf_sm_trainer **out);
TSDF_API int tsdf_sm_trainer_destroy(tsdf_sm_trainer *t);
TSDF_API int tsdf_sm_loss_grad(tsdf_sm_trainer *t, const float *params_dev, int n_frames,
                               const float *const *depth_dev, const float K[4], const float *T_world_cam,
                               float voxel_size, float max_range, long long n_vox, const int *vox_dev,
                               const float *target_dev, float *grad_dev, double *loss_host, void *hip_stream);

/* One Adam step on n parameters (device memory): moments m1, m2 and the
 * binary32 master copy are updated in place, params_dev receives the master
 * rounded to bfloat16 (the inference parameters).  step >= 1 is the step count
 * used for the bias corrections. */
TSDF_API int tsdf_sm_adam(float *master_dev, float *m1_dev, float *m2_dev, const float *grad_dev, float *params_dev,
                          int n, float lr, float beta1, float beta2, float eps, int step, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* TSDF_H */

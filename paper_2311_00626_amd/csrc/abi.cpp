// Host side of the C ABI declared in include/tsdf.h: argument validation,
// the per-frame constants (pose inverse, truncation constants, block lattice),
// map memory management and kernel launches.  No exception leaves this file.
#include "tsdf.h"
#include "tsdf_internal.hpp"
#include "sensor_model.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using namespace tsdf;

static_assert(TSDF_MAX_VIEWS == kMaxViews, "view batch limit");
static_assert(sizeof(ViewsArgs) <= 4096, "kernel argument size");

struct tsdf_map {
    tsdf_params p;
    int device;
    DeviceMap dm;
    int sticky;                           // host copy of an observed device error (TSDF_EFULL) or 0
    float eps, delta, span_inv;           // per-map constants in binary32
    int max_groups;                       // cap on integration workgroups per launch
    int cus = 0;                          // compute units of the map's device (0: unknown)
    tsdf_launch_config launch;            // explicit launch shape (0 fields = automatic)
    long long frames;                     // integrate calls launched so far (parity of the touched counters)
    float *tiles = nullptr;               // footprint pyramids, kMaxViews slots (allocated on first use)
    float *sm_params = nullptr;           // learned sensor model parameters (kSmParams)
    float2 *sm_maps = nullptr;            // per-pixel (weight, truncation), kMaxViews slots
    unsigned char *walk_marks = nullptr;  // ray-walk allocation: one byte per lattice entry
    long long walk_cap = 0;
    uint2 *cand = nullptr;                // compacted launches: candidate list
    long long cand_cap = 0;
    long long sm_slot = 0;                // pixels per slot of sm_maps
    // query_blocks work buffers, allocated on its first call (block_cap keys)
    unsigned long long *q_sorted = nullptr;
    void *q_temp = nullptr;
    size_t q_temp_bytes = 0;
    unsigned long long *q_count = nullptr;
    std::vector<tsdf_step *> steps;       // live graph steps of this map (reserve drops their graphs)
    // kernel timing
    bool profiling;
    std::vector<hipEvent_t> ev_start, ev_stop;
    size_t ev_used;
};

namespace {

constexpr long long kDefaultBlocks = 1ll << 18;
constexpr size_t kMaxTimedLaunches = 65536;

bool finite_all(const float *v, int n)
{
    for (int k = 0; k < n; ++k)
        if (!std::isfinite(v[k]))
            return false;
    return true;
}

bool params_valid(const tsdf_params *p)
{
    if (!p)
        return false;
    if (!(p->voxel_size_m > 0 && std::isfinite(p->voxel_size_m)))
        return false;
    if (!(p->truncation_vox > 0 && std::isfinite(p->truncation_vox)))
        return false;
    if (!(p->max_weight > 0 && std::isfinite(p->max_weight)))
        return false;
    if (!(p->max_range_m > 0 && std::isfinite(p->max_range_m)))
        return false;
    if (p->weighting != TSDF_WEIGHT_CONSTANT && p->weighting != TSDF_WEIGHT_LINEAR_DROPOFF &&
        p->weighting != TSDF_WEIGHT_LEARNED)
        return false;
    if (p->storage != TSDF_STORAGE_FP32 && p->storage != TSDF_STORAGE_FP16)
        return false;
    if (p->block_capacity < 1 || p->block_capacity > (1ll << 30))
        return false;
    if (p->hash_capacity < 0 || p->hash_capacity > (1ll << 31))
        return false;
    if (p->hash_capacity != 0 && (p->hash_capacity & (p->hash_capacity - 1)) != 0)
        return false;
    if (p->hash_capacity != 0 && p->hash_capacity < p->block_capacity)
        return false;
    if ((p->allocation != TSDF_ALLOC_EXACT && p->allocation != TSDF_ALLOC_RAY_WALK) || p->reserved != 0)
        return false;
    if (p->allocation == TSDF_ALLOC_RAY_WALK && p->weighting == TSDF_WEIGHT_LEARNED)
        return false;
    return true;
}

// Rigid-pose check: bottom row (0 0 0 1) within 1e-6, R^T R = I within 1e-4.
bool pose_valid(const float *T)
{
    if (!finite_all(T, 16))
        return false;
    if (std::fabs(T[12]) > 1e-6f || std::fabs(T[13]) > 1e-6f || std::fabs(T[14]) > 1e-6f ||
        std::fabs(T[15] - 1.0f) > 1e-6f)
        return false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0;
            for (int k = 0; k < 3; ++k)
                s += (double)T[4 * k + a] * (double)T[4 * k + b];
            if (std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-4)
                return false;
        }
    return true;
}

int hip_status(hipError_t e)
{
    if (e == hipSuccess)
        return TSDF_OK;
    if (e == hipErrorOutOfMemory)
        return TSDF_ENOMEM;
    return TSDF_EDEVICE;
}

void free_query_buffers(tsdf_map *m)
{
    (void)hipFree(m->q_sorted);
    (void)hipFree(m->q_temp);
    (void)hipFree(m->q_count);
    m->q_sorted = nullptr;
    m->q_temp = nullptr;
    m->q_count = nullptr;
    m->q_temp_bytes = 0;
}

void free_device(tsdf_map *m)
{
    DeviceMap &d = m->dm;
    (void)hipFree(d.keys);
    (void)hipFree(d.vals);
    (void)hipFree(d.pool);
    (void)hipFree(d.slot_keys);
    (void)hipFree(d.touched);
    (void)hipFree(d.counters);
    (void)hipFree(d.totals);
    d = DeviceMap{};
    (void)hipFree(m->tiles);
    m->tiles = nullptr;
    (void)hipFree(m->sm_params);
    m->sm_params = nullptr;
    (void)hipFree(m->sm_maps);
    m->sm_maps = nullptr;
    m->sm_slot = 0;
    (void)hipFree(m->walk_marks);
    m->walk_marks = nullptr;
    m->walk_cap = 0;
    (void)hipFree(m->cand);
    m->cand = nullptr;
    m->cand_cap = 0;
    free_query_buffers(m);
}

void free_events(tsdf_map *m)
{
    for (hipEvent_t e : m->ev_start)
        (void)hipEventDestroy(e);
    for (hipEvent_t e : m->ev_stop)
        (void)hipEventDestroy(e);
    m->ev_start.clear();
    m->ev_stop.clear();
    m->ev_used = 0;
}

// Per-view constants (the a1 step): camera-from-world pose and intrinsics,
// plus the world box that holds every voxel the view can update.
int camera_view(const tsdf_map *m, const float *depth, int width, int height, const float K[4],
                const float T[16], float max_range, CameraView &cv, double lo[3], double hi[3])
{
    // Inverse of the rigid pose: R^T exactly; each component of -R^T t is
    // accumulated in binary64 as ((R0i t0 + R1i t1) + R2i t2) and rounded once.
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            cv.R[3 * i + j] = T[4 * j + i];
    for (int i = 0; i < 3; ++i) {
        const double acc = ((double)T[0 * 4 + i] * (double)T[3] + (double)T[1 * 4 + i] * (double)T[7]) +
                           (double)T[2 * 4 + i] * (double)T[11];
        cv.t[i] = (float)(-acc);
    }
    cv.fx = K[0];
    cv.fy = K[1];
    cv.cx = K[2];
    cv.cy = K[3];
    cv.width = width;
    cv.height = height;
    cv.width_f = (float)width;
    cv.height_f = (float)height;
    cv.depth = depth;
    cv.d_max = max_range;
    cv.model = kModelPinhole;

    // An updated voxel has 0 < z <= d + eps <= max_range + eps and projects
    // into the image: it lies in the pyramid of the camera centre and the
    // image corners at that depth.
    const double zfar = (double)max_range + (double)m->eps;
    cv.zfar = (float)zfar;
    for (int a = 0; a < 3; ++a)
        lo[a] = hi[a] = (double)T[4 * a + 3];
    for (int c = 0; c < 4; ++c) {
        const double u = (c & 1) ? (double)width : 0.0;
        const double v = (c & 2) ? (double)height : 0.0;
        const double pc[3] = {(u - K[2]) / K[0] * zfar, (v - K[3]) / K[1] * zfar, zfar};
        for (int a = 0; a < 3; ++a) {
            double w = (double)T[4 * a + 3];
            for (int b = 0; b < 3; ++b)
                w += (double)T[4 * a + b] * pc[b];
            lo[a] = std::min(lo[a], w);
            hi[a] = std::max(hi[a], w);
        }
    }
    double extent = 0;
    for (int a = 0; a < 3; ++a)
        extent = std::max(extent, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
    // Culling slack: half a voxel plus a generous bound on binary32 rounding
    // of coordinates of magnitude `extent`, scaled into each plane's units.
    const double e = 0.5 * (double)m->p.voxel_size_m + 1e-5 * (1.0 + extent + zfar);
    cv.margin_u = (float)(e * ((double)K[0] + std::fabs((double)K[2]) + (double)width));
    cv.margin_v = (float)(e * ((double)K[1] + std::fabs((double)K[3]) + (double)height));
    return TSDF_OK;
}

// Per-view constants of a spherical range image (Eq. (3)); the pose as for a
// camera.  Columns and rows per radian are binary32 divisions, as in the
// oracle.  Every updated voxel lies within R = max_range + eps of the sensor
// and inside the polar band, so inside the sensor-frame box
// [-R, R]^2 x [min(0, R cos phi_end), max(0, R cos phi_start)].
int spherical_view(const tsdf_map *m, const float *range, int width, int height, const float A[4], float interp,
                   const float T[16], float max_range, CameraView &cv, double lo[3], double hi[3])
{
    const float K[4] = {1.0f, 1.0f, 0.0f, 0.0f};
    camera_view(m, range, width, height, K, T, max_range, cv, lo, hi);
    cv.model = kModelSpherical;
    cv.az_start = A[0];
    cv.alpha = (float)width / A[1];
    cv.pol_start = A[2];
    cv.beta = (float)height / A[3];
    cv.interp_diff = interp;
    cv.full_circle = A[1] >= 6.28318548f ? 1 : 0;
    for (int a = 0; a < 3; ++a)
        cv.origin[a] = T[4 * a + 3];
    cv.cos_pol_start = (float)std::cos((double)A[2]);
    cv.cos_pol_end = (float)std::cos((double)A[2] + (double)A[3]);
    const double R = (double)max_range + (double)m->eps;
    cv.zfar = (float)R;
    const double zlo = std::min(0.0, R * std::cos((double)A[2] + (double)A[3]));
    const double zhi = std::max(0.0, R * std::cos((double)A[2]));
    for (int a = 0; a < 3; ++a)
        lo[a] = hi[a] = (double)T[4 * a + 3];
    for (int c = 0; c < 8; ++c) {
        const double pc[3] = {(c & 1) ? R : -R, (c & 2) ? R : -R, (c & 4) ? zhi : zlo};
        for (int a = 0; a < 3; ++a) {
            double w = (double)T[4 * a + 3];
            for (int b = 0; b < 3; ++b)
                w += (double)T[4 * a + b] * pc[b];
            lo[a] = std::min(lo[a], w);
            hi[a] = std::max(hi[a], w);
        }
    }
    return TSDF_OK;
}

bool lidar_valid(int width, int height, const float A[4], float interp, float max_range)
{
    if (width < 2 || height < 2 || (long long)width * (long long)height > (1ll << 28))
        return false;
    if (!finite_all(A, 4) || !std::isfinite(interp) || !std::isfinite(max_range))
        return false;
    const double pi = 3.14159265358979323846;
    if (!(A[1] > 0.0f && A[1] <= 6.28318548f && A[3] > 0.0f && A[2] >= 0.0f && A[2] < pi &&
          (double)A[2] + (double)A[3] <= pi + 1e-6))
        return false;
    return interp >= 0.0f && max_range >= 0.0f;
}

void map_consts(const tsdf_map *m, double max_extent, double max_zfar, MapConsts &mc)
{
    mc.vs = m->p.voxel_size_m;
    mc.eps = m->eps;
    mc.delta = m->delta;
    mc.span_inv = m->span_inv;
    mc.w_max = m->p.max_weight;
    mc.margin_z = (float)(0.5 * (double)m->p.voxel_size_m + 1e-5 * (1.0 + max_extent + max_zfar));
}

// The culling tests of a single pinhole view (lane_block_in_pinhole and
// lane_block_footprint_pinhole, with their margins) as linear functions of
// the lattice-relative block index, in binary64 (PinholeCull).  A frustum
// plane a x + b y + c z + d of the camera frame is largest over a block at
// the corner the positive components of its edge terms pick: its value at
// the block's lower corner plus the positive parts of those terms.
void pinhole_cull(const CameraView &cv, const MapConsts &mc, const Lattice &lat, PinholeCull &pc)
{
    const double e = 8.0 * (double)mc.vs;
    double cam[12];
    for (int a = 0; a < 3; ++a) {
        double c = (double)cv.t[a];
        for (int k = 0; k < 3; ++k) {
            cam[4 * a + k] = e * (double)cv.R[3 * a + k];
            c += e * (double)cv.R[3 * a + k] * (double)lat.lat_min[k];
        }
        cam[4 * a + 3] = c;
    }
    const double fx = cv.fx, fy = cv.fy, cx = cv.cx, cy = cv.cy;
    const double planes[6][5] = {{fx, 0.0, cx, 0.0, cv.margin_u},
                                 {-fx, 0.0, (double)cv.width_f - cx, 0.0, cv.margin_u},
                                 {0.0, fy, cy, 0.0, cv.margin_v},
                                 {0.0, -fy, (double)cv.height_f - cy, 0.0, cv.margin_v},
                                 {0.0, 0.0, 1.0, 0.0, mc.margin_z},
                                 {0.0, 0.0, -1.0, (double)cv.zfar, mc.margin_z}};
    for (int q = 0; q < 6; ++q) {
        const double *P = planes[q];
        double t = P[0] * cam[3] + P[1] * cam[7] + P[2] * cam[11] + P[3] + P[4];
        for (int k = 0; k < 3; ++k) {
            const double A = P[0] * cam[k] + P[1] * cam[4 + k] + P[2] * cam[8 + k];
            pc.plane[4 * q + k] = (float)A;
            t += std::max(0.0, A);
        }
        pc.plane[4 * q + 3] = (float)t;
    }
    for (int k = 0; k < 12; ++k)
        pc.cam[k] = (float)cam[k];
    pc.valid = 1;
}

// Block lattice of a world box, widened by one voxel.
int lattice_of(const tsdf_map *m, const double lo[3], const double hi[3], Lattice &lat)
{
    const double vs = (double)m->p.voxel_size_m;
    const double edge = 8.0 * vs;
    for (int a = 0; a < 3; ++a) {
        const double bl = std::floor((lo[a] - vs) / edge);
        const double bh = std::floor((hi[a] + vs) / edge);
        if (!(bl >= -kBlockCoordMax && bh <= kBlockCoordMax))
            return TSDF_EINVAL;
        lat.lat_min[a] = (int)bl;
        lat.lat_dim[a] = (int)(bh - bl) + 1;
    }
    lat.n_lat = (long long)lat.lat_dim[0] * lat.lat_dim[1] * lat.lat_dim[2];
    if (lat.n_lat >= (1ll << 31))
        return TSDF_EINVAL;
    set_lattice_divisors(lat);
    return TSDF_OK;
}

double box_extent(const double lo[3], const double hi[3])
{
    double e = 0;
    for (int a = 0; a < 3; ++a)
        e = std::max(e, std::max(std::fabs(lo[a]), std::fabs(hi[a])));
    return e;
}

// Argument checks shared by the integration entry points.
bool view_args_valid(const float *depth_dev, int width, int height, const float K[4], const float T[16])
{
    if (!depth_dev || !K || !T || width <= 0 || height <= 0)
        return false;
    // byte offsets into the depth image must stay below 2^31 (buffer addressing)
    if ((long long)width * (long long)height > (1ll << 28) || width > (1 << 24) || height > (1 << 24))
        return false;
    if (!finite_all(K, 4) || !(K[0] > 0) || !(K[1] > 0))
        return false;
    return pose_valid(T);
}

// Optional kernel timing around one launch.
bool timing_begin(tsdf_map *m, hipStream_t s)
{
    if (!m->profiling || m->ev_used >= kMaxTimedLaunches)
        return false;
    if (m->ev_used == m->ev_start.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess)
            return false;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return false;
        }
        m->ev_start.push_back(a);
        m->ev_stop.push_back(b);
    }
    return hipEventRecord(m->ev_start[m->ev_used], s) == hipSuccess;
}

void timing_end(tsdf_map *m, hipStream_t s, bool timed)
{
    if (timed && hipEventRecord(m->ev_stop[m->ev_used], s) == hipSuccess)
        ++m->ev_used;
}

// Makes the map's device current (a no-op when it already is).
hipError_t use_device(const tsdf_map *m)
{
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != m->device)
        e = hipSetDevice(m->device);
    return e;
}

// Launch shape (tuned on MI355X).  Small lattices (a few blocks per wave) are
// latency-bound: one block per wave pass keeps every touched block on its own
// wave.  Large lattices (fine voxels, long ranges) cull 8 blocks per wave pass.
// Image-band ownership per XCD (partitions = 8) cuts L2 fills but measured
// slower on both regimes, so it is only used when asked for.  Fields of the
// map's launch configuration override these choices.
int schedule(const tsdf_map *m, Lattice &lat)
{
    const tsdf_launch_config &lc = m->launch;
    long long max_groups = lc.max_groups > 0 ? lc.max_groups : m->max_groups;
    max_groups = std::max<long long>(kPartitions, max_groups / kPartitions * kPartitions);
    const long long full_waves = max_groups * kWavesPerGroup;
    const int parts = lc.partitions > 0 ? lc.partitions : 1;
    long long groups = (lat.n_lat + kWavesPerGroup - 1) / kWavesPerGroup;
    groups = (groups + kPartitions - 1) / kPartitions * kPartitions;
    groups = std::max<long long>(kPartitions, std::min<long long>(groups, max_groups));
    const long long chunk = lc.chunk > 0 ? lc.chunk : (lat.n_lat > 4 * full_waves ? 8 : 1);
    lat.chunk = (int)std::max(1ll, std::min<long long>(chunk, kMaxChunk));
    lat.partitions = parts;
    // automatic chunk, one band: the walk culls and compacts per workgroup
    lat.group_scan = (lc.chunk == 0 && parts == 1) ? 1 : 0;
    return (int)groups;
}

// Footprint culling policy for one launch: explicit, or automatic when the
// lattice is large enough for the culled measurement work to outweigh the
// pyramid pass.
constexpr long long kFootprintAutoLattice = 1ll << 14;

bool use_footprint(const tsdf_map *m, const Lattice &lat)
{
    if (m->launch.footprint == TSDF_FOOTPRINT_NEVER)
        return false;
    if (m->launch.footprint == TSDF_FOOTPRINT_ALWAYS)
        return true;
    return lat.n_lat >= kFootprintAutoLattice;
}

hipError_t ensure_tiles(tsdf_map *m)
{
    if (m->tiles)
        return hipSuccess;
    return hipMalloc((void **)&m->tiles, sizeof(float) * (size_t)kMaxViews * (size_t)kTileFloatsPerView);
}

// Points the view at pyramid slot `slot` (nothing for images beyond the
// pyramid's largest side).
void attach_tiles(float *tiles, CameraView &cv, int slot)
{
    cv.tiles = nullptr;
    if (!tiles || cv.width > kTileMaxSide || cv.height > kTileMaxSide)
        return;
    int off = 0;
    for (int l = 0; l < kTileLevels; ++l) {
        const int ts = 1 << (kTileBaseShift + l);
        cv.tile_cols[l] = (cv.width + ts - 1) / ts;
        cv.tile_rows[l] = (cv.height + ts - 1) / ts;
        cv.tile_off[l] = off;
        off += cv.tile_cols[l] * cv.tile_rows[l];
    }
    cv.tiles = tiles + (size_t)slot * (size_t)kTileFloatsPerView;
}

// Builds the pyramid of a single-view launch when the policy asks for it.
// Scratch buffers a call uses instead of the map's own (the no-allocation
// entry point): a footprint pyramid slot and a candidate list.
struct CallScratch {
    float *tiles;
    uint2 *cand;
    long long cand_cap;
};

hipError_t prepare_footprint(tsdf_map *m, FrameArgs &fa, hipStream_t s, const CallScratch *sc)
{
    if (!use_footprint(m, fa.lat))
        return hipSuccess;
    if (sc) {
        attach_tiles(sc->tiles, fa.cam, 0);
    } else {
        hipError_t e = ensure_tiles(m);
        if (e != hipSuccess)
            return e;
        attach_tiles(m->tiles, fa.cam, 0);
    }
    ViewsArgs va;
    std::memset(&va, 0, sizeof(va));
    va.cam[0] = fa.cam;
    va.n_views = 1;
    return launch_footprint_tiles(va, s);
}

hipError_t prepare_footprint(tsdf_map *m, ViewsArgs &va, hipStream_t s, bool launch)
{
    if (!use_footprint(m, va.lat))
        return hipSuccess;
    hipError_t e = ensure_tiles(m);
    if (e != hipSuccess)
        return e;
    for (int v = 0; v < va.n_views; ++v)
        attach_tiles(m->tiles, va.cam[v], v);
    return launch ? launch_footprint_tiles(va, s) : hipSuccess;
}

// Learned weighting: per-pixel (weight, truncation) maps of the views,
// slot v for view v, evaluated from the map's sensor-model parameters.
hipError_t ensure_sm_maps(tsdf_map *m, long long pixels)
{
    if (m->sm_maps && m->sm_slot >= pixels)
        return hipSuccess;
    long long slot = std::max<long long>(pixels, 640ll * 480ll);
    if (m->sm_maps) {
        hipError_t e = hipDeviceSynchronize();    // earlier launches may still read the old maps
        if (e != hipSuccess)
            return e;
    }
    (void)hipFree(m->sm_maps);
    m->sm_maps = nullptr;
    m->sm_slot = 0;
    hipError_t e = hipMalloc((void **)&m->sm_maps, sizeof(float2) * (size_t)slot * kMaxViews);
    if (e == hipSuccess)
        m->sm_slot = slot;
    return e;
}

SmView sm_view_of(const CameraView &cv)
{
    SmView v;
    v.depth = cv.depth;
    v.width = cv.width;
    v.height = cv.height;
    v.fx = cv.fx;
    v.fy = cv.fy;
    v.cx = cv.cx;
    v.cy = cv.cy;
    v.d_max = cv.d_max;
    return v;
}

hipError_t prepare_learned(tsdf_map *m, CameraView *cams, int n_views, hipStream_t s)
{
    if (m->p.weighting != TSDF_WEIGHT_LEARNED)
        return hipSuccess;
    long long px = 0;
    for (int v = 0; v < n_views; ++v)
        px = std::max<long long>(px, (long long)cams[v].width * cams[v].height);
    hipError_t e = ensure_sm_maps(m, px);
    for (int v = 0; v < n_views && e == hipSuccess; ++v) {
        float2 *out = m->sm_maps + (size_t)v * (size_t)m->sm_slot;
        e = launch_sm_maps(sm_view_of(cams[v]), m->p.voxel_size_m, m->sm_params, out, s);
        cams[v].sm_maps = out;
    }
    return e;
}

// Compacted launch policy: explicit, or automatic once the culling work
// (lattice blocks x views) is large; one band only, and not with ray-walk
// marks (the marks are the candidates).  For the single view of
// integrate_depth or integrate_range (one_view) the walk, which culls and
// compacts per workgroup, stays ahead up to larger lattices: on 640x480
// frames of a box room it is 4-12 % faster at lattices of 39 k-90 k blocks
// (2-1.5 cm voxels) and the list 3-5 % faster at 153 k (1.25 cm); on a
// 1024x64 LiDAR with 25 m of reach the walk is 6 % faster at 10 k-21 k
// blocks (20 cm), 2 % at 80 k-170 k (10 cm), and the list 16 % faster from
// 650 k (5 cm).
constexpr long long kCompactAutoWork = 1ll << 14;
constexpr long long kCompactAutoOneView = 1ll << 17;

bool use_compaction(const tsdf_map *m, const Lattice &lat, int n_views, bool one_view = false)
{
    if (m->p.allocation == TSDF_ALLOC_RAY_WALK || (m->launch.partitions > 1))
        return false;
    if (m->launch.compaction == TSDF_COMPACT_NEVER)
        return false;
    if (m->launch.compaction == TSDF_COMPACT_ALWAYS)
        return true;
    if (one_view)
        return lat.n_lat >= kCompactAutoOneView;
    return lat.n_lat * n_views >= kCompactAutoWork;
}

// LDS staging of block footprints for a single pinhole view, on request
// only: measured against direct gathers it lost on every workload tried
// (640x480 frames at 1, 2 and 4 cm: the copy adds a load -> LDS write -> LDS
// read step to a latency-bound chain and reads more pixels than the voxels
// sample), so the automatic choice is direct reads.
bool use_staging(const tsdf_map *m, const CameraView &)
{
    return m->p.weighting != TSDF_WEIGHT_LEARNED && m->launch.staging == TSDF_STAGE_ALWAYS;
}

// Points the lattice at a candidate list large enough for every block of it.
hipError_t prepare_compaction(tsdf_map *m, Lattice &lat, int n_views, const CallScratch *sc = nullptr,
                              bool one_view = false)
{
    lat.cand = nullptr;
    if (!use_compaction(m, lat, n_views, one_view))
        return hipSuccess;
    if (sc) {
        if (lat.n_lat > sc->cand_cap)
            return hipErrorOutOfMemory;   // the caller checked the size first
        lat.cand = sc->cand;
        return hipSuccess;
    }
    if (!m->cand || m->cand_cap < lat.n_lat) {
        if (m->cand) {
            hipError_t e = hipDeviceSynchronize();   // earlier launches may still read the old list
            if (e != hipSuccess)
                return e;
        }
        (void)hipFree(m->cand);
        m->cand = nullptr;
        m->cand_cap = 0;
        // twice the lattice: a growing lattice reallocates (a device
        // synchronisation and a free in the middle of the stream) rarely
        long long cap = std::max<long long>(2 * lat.n_lat, 1ll << 18);
        hipError_t e = hipMalloc((void **)&m->cand, sizeof(uint2) * (size_t)cap);
        if (e == hipErrorOutOfMemory) {   // no room for the headroom: the lattice itself
            (void)hipGetLastError();
            cap = lat.n_lat;
            e = hipMalloc((void **)&m->cand, sizeof(uint2) * (size_t)cap);
        }
        if (e != hipSuccess)
            return e;
        m->cand_cap = cap;
    }
    lat.cand = m->cand;
    return hipSuccess;
}

// Ray-walk allocation: widens the lattice by one block on every side (the
// walk stays inside the frustum, the margin absorbs binary32 rounding at its
// ends), marks the visited blocks and points the view at the marks.
hipError_t prepare_walk(tsdf_map *m, FrameArgs &fa, const float T[16], hipStream_t s)
{
    if (m->p.allocation != TSDF_ALLOC_RAY_WALK)
        return hipSuccess;
    Lattice &lat = fa.lat;
    for (int a = 0; a < 3; ++a) {
        lat.lat_min[a] -= 1;
        lat.lat_dim[a] += 2;
    }
    lat.n_lat = (long long)lat.lat_dim[0] * lat.lat_dim[1] * lat.lat_dim[2];
    if (lat.n_lat >= (1ll << 31))
        return hipErrorInvalidValue;
    set_lattice_divisors(lat);
    if (!m->walk_marks || m->walk_cap < lat.n_lat) {
        if (m->walk_marks) {
            hipError_t e = hipDeviceSynchronize();   // earlier launches may still read the old marks
            if (e != hipSuccess)
                return e;
        }
        (void)hipFree(m->walk_marks);
        m->walk_marks = nullptr;
        m->walk_cap = 0;
        long long cap = std::max<long long>(2 * lat.n_lat, 1ll << 20);   // as the candidate list
        hipError_t e = hipMalloc((void **)&m->walk_marks, (size_t)cap);
        if (e == hipErrorOutOfMemory) {
            (void)hipGetLastError();
            cap = lat.n_lat;
            e = hipMalloc((void **)&m->walk_marks, (size_t)cap);
        }
        if (e == hipSuccess)
            e = launch_fill_u8(m->walk_marks, cap, s);   // from here on the integration kernel keeps it zero
        if (e != hipSuccess)
            return e;
        m->walk_cap = cap;
    }
    DdaArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j)
            a.Rwc[3 * i + j] = T[4 * i + j];
        a.o[i] = T[4 * i + 3];
    }
    a.fx = fa.cam.fx;
    a.fy = fa.cam.fy;
    a.cx = fa.cam.cx;
    a.cy = fa.cam.cy;
    a.width = fa.cam.width;
    a.height = fa.cam.height;
    a.depth = fa.cam.depth;
    a.d_max = fa.cam.d_max;
    a.eps = m->eps;
    a.vs = m->p.voxel_size_m;
    a.lat = lat;
    a.marks = m->walk_marks;
    a.overflow = m->dm.counters + kErrorBits;
    fa.cam.dda_marks = m->walk_marks;
    lat.partitions = 1;
    return launch_dda_mark(a, s);
}

struct CounterSnapshot {
    uint32_t c[kNumCounterWords];
    unsigned long long t[kNumTotalWords];
};

int read_counters(tsdf_map *m, CounterSnapshot &cs, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(cs.c, m->dm.counters, sizeof(cs.c), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cs.t, m->dm.totals, sizeof(cs.t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_status(e);
    if (cs.c[kErrorBits] != 0)
        m->sticky = TSDF_EFULL;
    return TSDF_OK;
}

// Touched count of each sub-list for the most recent frame (zeros before the first).
void last_touched_counts(const tsdf_map *m, const CounterSnapshot &cs, long long n[kSubLists])
{
    for (int k = 0; k < kSubLists; ++k)
        n[k] = 0;
    if (m->frames == 0)
        return;
    const int parity = (int)((m->frames - 1) & 1);
    for (int k = 0; k < kSubLists; ++k)
        n[k] = std::min<long long>(cs.c[touched_counter(parity, k)], m->dm.block_cap);
}

}  // namespace

extern "C" {

void tsdf_default_params(tsdf_params *p, float voxel_size_m, float truncation_vox)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    p->voxel_size_m = voxel_size_m;
    p->truncation_vox = truncation_vox;
    p->max_weight = 100.0f;
    p->max_range_m = 5.0f;
    p->weighting = TSDF_WEIGHT_CONSTANT;
    p->block_capacity = kDefaultBlocks;
    p->hash_capacity = 0;
}

int create_map_ex(const tsdf_params *p, tsdf_map **out)
{
    if (!out)
        return TSDF_EINVAL;
    *out = nullptr;
    if (!params_valid(p))
        return TSDF_EINVAL;
    tsdf_map *m = new (std::nothrow) tsdf_map();
    if (!m)
        return TSDF_ENOMEM;
    m->p = *p;
    long long hc = p->hash_capacity;
    if (hc == 0) {
        hc = 64;
        while (hc < 2 * p->block_capacity)
            hc *= 2;
    }
    m->p.hash_capacity = hc;
    // binary32 per-map constants, the same operations the oracle performs
    m->eps = p->truncation_vox * p->voxel_size_m;
    m->delta = p->voxel_size_m;
    m->span_inv = m->eps > m->delta ? 1.0f / (m->eps - m->delta) : 0.0f;
    if (p->weighting == TSDF_WEIGHT_LEARNED)
        m->eps = 8.0f * p->voxel_size_m;    // bound of every per-pixel truncation (culling only)
    m->max_groups = 512;   // a multiple of kPartitions
    m->launch = tsdf_launch_config{0, 0, 0, 0, 0};
    m->frames = 0;
    m->profiling = false;
    m->ev_used = 0;
    m->sticky = 0;

    hipError_t e = hipGetDevice(&m->device);
    if (e == hipSuccess && hipDeviceGetAttribute(&m->cus, hipDeviceAttributeMultiprocessorCount, m->device) !=
                               hipSuccess) {
        (void)hipGetLastError();
        m->cus = 0;
    }
    DeviceMap &d = m->dm;
    const size_t bc = (size_t)p->block_capacity;
    if (e == hipSuccess) e = hipMalloc(&d.keys, sizeof(unsigned long long) * (size_t)hc);
    if (e == hipSuccess) e = hipMalloc(&d.vals, sizeof(uint32_t) * (size_t)hc);
    const size_t vb = voxel_bytes(p->storage);
    if (e == hipSuccess) e = hipMalloc(&d.pool, vb * kBlockVoxels * bc);
    if (e == hipSuccess) e = hipMalloc(&d.slot_keys, sizeof(unsigned long long) * bc);
    if (e == hipSuccess) e = hipMalloc(&d.touched, sizeof(uint32_t) * bc * kSubLists);
    if (e == hipSuccess) e = hipMalloc(&d.counters, sizeof(uint32_t) * kNumCounterWords);
    if (e == hipSuccess) e = hipMalloc(&d.totals, sizeof(unsigned long long) * kNumTotalWords);
    if (e == hipSuccess) e = hipMemset(d.keys, 0xFF, sizeof(unsigned long long) * (size_t)hc);
    if (e == hipSuccess) e = hipMemset(d.vals, 0xFF, sizeof(uint32_t) * (size_t)hc);
    if (e == hipSuccess) e = hipMemset(d.pool, 0, vb * kBlockVoxels * bc);
    if (e == hipSuccess) e = hipMemset(d.slot_keys, 0xFF, sizeof(unsigned long long) * bc);
    if (e == hipSuccess) e = hipMemset(d.counters, 0, sizeof(uint32_t) * kNumCounterWords);
    if (e == hipSuccess) e = hipMemset(d.totals, 0, sizeof(unsigned long long) * kNumTotalWords);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_device(m);
        delete m;
        return hip_status(e);
    }
    d.hash_mask = (uint32_t)(hc - 1);
    d.block_cap = (uint32_t)bc;
    d.storage = p->storage;
    *out = m;
    return TSDF_OK;
}

int create_map(float voxel_size_m, float truncation_vox, tsdf_map **out)
{
    tsdf_params p;
    tsdf_default_params(&p, voxel_size_m, truncation_vox);
    return create_map_ex(&p, out);
}

int destroy_map(tsdf_map *m)
{
    if (!m)
        return TSDF_OK;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    free_events(m);
    free_device(m);
    delete m;
    return TSDF_OK;
}

}  // extern "C"

namespace {

// integrate_depth with the map's own scratch buffers (sc == nullptr, which
// allocates them on first use) or with the fixed scratch `sc`.
int integrate_depth_call(tsdf_map *m, const float *depth_dev, int width, int height, const float K[4],
                         const float T_world_cam[16], void *hip_stream, const CallScratch *sc)
{
    if (!m || !view_args_valid(depth_dev, width, height, K, T_world_cam))
        return TSDF_EINVAL;
    if (m->p.weighting == TSDF_WEIGHT_LEARNED && !m->sm_params)
        return TSDF_EINVAL;
    if (sc && (m->p.weighting == TSDF_WEIGHT_LEARNED || m->p.allocation == TSDF_ALLOC_RAY_WALK))
        return TSDF_EINVAL;
    if (m->sticky)
        return TSDF_ESTATE;
    FrameArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    double lo[3], hi[3];
    int st = camera_view(m, depth_dev, width, height, K, T_world_cam, m->p.max_range_m, fa.cam, lo, hi);
    if (st == TSDF_OK)
        st = lattice_of(m, lo, hi, fa.lat);
    if (st != TSDF_OK)
        return st;
    map_consts(m, box_extent(lo, hi), (double)fa.cam.zfar, fa.mc);
    if (sc && use_compaction(m, fa.lat, 1, true) && fa.lat.n_lat > sc->cand_cap)
        return TSDF_ESCRATCH;
    fa.parity = (int)(m->frames & 1);
    fa.stage = use_staging(m, fa.cam) ? 1 : 0;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = use_device(m);
    // every kernel of the call, pre-passes included (not with the fixed
    // scratch: the first timed call creates events)
    const bool timed = e == hipSuccess && !sc && timing_begin(m, s);
    const bool walk = m->p.allocation == TSDF_ALLOC_RAY_WALK;
    if (e == hipSuccess && !walk)
        e = prepare_footprint(m, fa, s, sc);
    if (e == hipSuccess)
        e = prepare_learned(m, &fa.cam, 1, s);
    if (e == hipSuccess)
        e = prepare_walk(m, fa, T_world_cam, s);
    if (e == hipSuccess)
        e = prepare_compaction(m, fa.lat, 1, sc, true);
    if (e != hipSuccess)
        return hip_status(e);
    int groups = schedule(m, fa.lat);
    if (walk)
        fa.lat.partitions = 1;    // every lattice entry is read by exactly one thread
    else
        pinhole_cull(fa.cam, fa.mc, fa.lat, fa.pc);
    int fill_cus = 0;
    if (fa.lat.cand) {
        // the list kernel's grid: as given, else every workgroup the chip
        // keeps resident (interleaved on one MI355X, 768 against 512 groups
        // made 640x480 frames 1-2.6 % faster at 1 and 1.25 cm; 640, which
        // leaves some CUs a group short, 1.5-3 % slower)
        groups = (int)std::max<long long>(kPartitions, (m->launch.max_groups > 0 ? m->launch.max_groups : m->max_groups) /
                                                           kPartitions * kPartitions);
        if (m->launch.max_groups <= 0 && m->cus > 0)
            fill_cus = m->cus;
        e = launch_cull_frame(m->dm, fa, s);
        if (e != hipSuccess)
            return hip_status(e);
    }
    e = launch_integrate_depth(m->dm, fa, m->p.weighting, groups, s, fill_cus);
    if (e != hipSuccess) {
        if (walk)   // the marks were set but not consumed: clear them for the next frame
            (void)launch_fill_u8(m->walk_marks, fa.lat.n_lat, s);
        return hip_status(e);
    }
    timing_end(m, s, timed);
    ++m->frames;
    return TSDF_OK;
}

}  // namespace

extern "C" {

int integrate_depth(tsdf_map *m, const float *depth_dev, int width, int height, const float K[4],
                    const float T_world_cam[16], void *hip_stream)
{
    return integrate_depth_call(m, depth_dev, width, height, K, T_world_cam, hip_stream, nullptr);
}

int integrate_depth_noalloc(tsdf_map *m, const float *depth_dev, int width, int height, const float K[4],
                            const float T_world_cam[16], void *hip_stream)
{
    if (!m || !view_args_valid(depth_dev, width, height, K, T_world_cam))
        return TSDF_EINVAL;
    hipError_t e = use_device(m);
    void *ptr = nullptr;
    if (e == hipSuccess)
        e = noalloc_scratch(&ptr);
    if (e != hipSuccess)
        return hip_status(e);
    CallScratch sc;
    sc.tiles = reinterpret_cast<float *>(ptr);
    sc.cand = reinterpret_cast<uint2 *>(reinterpret_cast<unsigned char *>(ptr) + kNoAllocTileBytes);
    sc.cand_cap = kNoAllocMaxCandidates;
    return integrate_depth_call(m, depth_dev, width, height, K, T_world_cam, hip_stream, &sc);
}

int integrate_range(tsdf_map *m, const float *range_dev, const tsdf_lidar_model *lidar,
                    const float T_world_sensor[16], void *hip_stream)
{
    if (!m || !range_dev || !lidar || !T_world_sensor || !pose_valid(T_world_sensor))
        return TSDF_EINVAL;
    const float A[4] = {lidar->azimuth_start_rad, lidar->azimuth_fov_rad, lidar->polar_start_rad,
                        lidar->polar_fov_rad};
    if (!lidar_valid(lidar->width, lidar->height, A, lidar->interp_max_diff_m, lidar->max_range_m))
        return TSDF_EINVAL;
    if (m->p.weighting == TSDF_WEIGHT_LEARNED || m->p.allocation == TSDF_ALLOC_RAY_WALK)
        return TSDF_EINVAL;    // both are defined on pinhole depth images, one frame per launch
    if (m->sticky)
        return TSDF_ESTATE;
    const float range = lidar->max_range_m > 0.0f ? lidar->max_range_m : m->p.max_range_m;
    FrameArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    double lo[3], hi[3];
    spherical_view(m, range_dev, lidar->width, lidar->height, A, lidar->interp_max_diff_m, T_world_sensor, range,
                   fa.cam, lo, hi);
    int st = lattice_of(m, lo, hi, fa.lat);
    if (st != TSDF_OK)
        return st;
    map_consts(m, box_extent(lo, hi), (double)fa.cam.zfar, fa.mc);
    fa.parity = (int)(m->frames & 1);
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = use_device(m);
    const bool timed = e == hipSuccess && timing_begin(m, s);   // every kernel of the call, pre-passes included
    if (e == hipSuccess)
        e = prepare_footprint(m, fa, s, nullptr);
    if (e == hipSuccess)
        e = prepare_learned(m, &fa.cam, 1, s);
    if (e == hipSuccess)
        e = prepare_compaction(m, fa.lat, 1, nullptr, true);
    if (e != hipSuccess)
        return hip_status(e);
    int groups = schedule(m, fa.lat);
    if (fa.lat.cand) {
        groups = (int)std::max<long long>(kPartitions, (m->launch.max_groups > 0 ? m->launch.max_groups : m->max_groups) /
                                                           kPartitions * kPartitions);
        e = launch_cull_frame(m->dm, fa, s);
        if (e != hipSuccess)
            return hip_status(e);
    }
    e = launch_integrate_depth(m->dm, fa, m->p.weighting, groups, s);
    if (e != hipSuccess)
        return hip_status(e);
    timing_end(m, s, timed);
    ++m->frames;
    return TSDF_OK;
}

} // extern "C"

namespace {

// Validates a batch of views and fills the launch arguments (not the parity).
int build_views_args(tsdf_map *m, const tsdf_depth_view *views, int n_views, ViewsArgs &va, bool &spherical)
{
    if (!views || n_views < 1 || n_views > TSDF_MAX_VIEWS)
        return TSDF_EINVAL;
    for (int v = 0; v < n_views; ++v) {
        const tsdf_depth_view &w = views[v];
        if (w.reserved != 0.0f || !(w.max_range_m >= 0.0f && std::isfinite(w.max_range_m)))
            return TSDF_EINVAL;
        if (w.model == TSDF_MODEL_PINHOLE) {
            if (w.interp_max_diff_m != 0.0f || !view_args_valid(w.depth_dev, w.width, w.height, w.K, w.T_world_cam))
                return TSDF_EINVAL;
        } else if (w.model == TSDF_MODEL_SPHERICAL) {
            if (!w.depth_dev || !pose_valid(w.T_world_cam) ||
                !lidar_valid(w.width, w.height, w.K, w.interp_max_diff_m, w.max_range_m))
                return TSDF_EINVAL;
        } else {
            return TSDF_EINVAL;
        }
    }
    std::memset(&va, 0, sizeof(va));
    spherical = false;
    double lo[3], hi[3], max_zfar = 0;
    for (int v = 0; v < n_views; ++v) {
        double vlo[3], vhi[3];
        const float range = views[v].max_range_m > 0.0f ? views[v].max_range_m : m->p.max_range_m;
        const int st = views[v].model == TSDF_MODEL_SPHERICAL
                           ? spherical_view(m, views[v].depth_dev, views[v].width, views[v].height, views[v].K,
                                            views[v].interp_max_diff_m, views[v].T_world_cam, range, va.cam[v],
                                            vlo, vhi)
                           : camera_view(m, views[v].depth_dev, views[v].width, views[v].height, views[v].K,
                                         views[v].T_world_cam, range, va.cam[v], vlo, vhi);
        if (st != TSDF_OK)
            return st;
        spherical = spherical || views[v].model == TSDF_MODEL_SPHERICAL;
        max_zfar = std::max(max_zfar, (double)va.cam[v].zfar);
        for (int a = 0; a < 3; ++a) {
            lo[a] = v == 0 ? vlo[a] : std::min(lo[a], vlo[a]);
            hi[a] = v == 0 ? vhi[a] : std::max(hi[a], vhi[a]);
        }
    }
    const int st = lattice_of(m, lo, hi, va.lat);
    if (st != TSDF_OK)
        return st;
    va.n_views = n_views;
    map_consts(m, box_extent(lo, hi), max_zfar, va.mc);
    return TSDF_OK;
}

}  // namespace

// A replayable batched step: two instantiated hipGraphs, each [copy of the
// step's launch arguments from a pinned staging slot to device memory] +
// [the batched integration kernel reading them], used alternately so that a
// slot is rewritten only after its previous replay has finished.
// Graph variants of a step, captured on first use: bit 0 = footprint
// pre-pass, bit 1 = compacted launch (cull kernel + list kernel), bit 2 = the
// cull kernel tests a block's views one lane each (the views share a model).
constexpr int kStepFootprint = 1;
constexpr int kStepCompact = 2;
constexpr int kStepLaneViews = 4;
constexpr int kStepModes = 8;

struct tsdf_step {
    tsdf_map *m;
    bool spherical;
    int groups;
    ViewsArgs *pinned[2];
    ViewsArgs *dev[2];
    hipGraph_t graph[2][kStepModes];
    hipGraphExec_t exec[2][kStepModes];
    hipEvent_t done[2];
    bool pending[2];
    int next;
};

// Destroys the step's captured graphs; each is captured again on its next use.
static void step_drop_graphs(tsdf_step *st)
{
    for (int k = 0; k < 2; ++k)
        for (int mode = 0; mode < kStepModes; ++mode) {
            if (st->exec[k][mode])
                (void)hipGraphExecDestroy(st->exec[k][mode]);
            if (st->graph[k][mode])
                (void)hipGraphDestroy(st->graph[k][mode]);
            st->exec[k][mode] = nullptr;
            st->graph[k][mode] = nullptr;
        }
}

static void step_free(tsdf_step *st)
{
    step_drop_graphs(st);
    for (int k = 0; k < 2; ++k) {
        if (st->done[k])
            (void)hipEventDestroy(st->done[k]);
        if (st->pinned[k])
            (void)hipHostFree(st->pinned[k]);
        if (st->dev[k])
            (void)hipFree(st->dev[k]);
    }
    delete st;
}

// Captures the replay of staging slot k in one mode: the argument upload,
// then only the kernels of that mode, all reading the uploaded arguments.
static hipError_t step_capture(tsdf_step *st, int k, int mode)
{
    tsdf_map *m = st->m;
    if (st->graph[k][mode]) {   // left by an earlier capture whose instantiation failed
        (void)hipGraphDestroy(st->graph[k][mode]);
        st->graph[k][mode] = nullptr;
    }
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess)
        return e;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = hipMemcpyAsync(st->dev[k], st->pinned[k], sizeof(ViewsArgs), hipMemcpyHostToDevice, cs);
        if (e1 == hipSuccess && (mode & kStepFootprint))
            e1 = launch_footprint_tiles_dev(st->dev[k], cs);
        if (e1 == hipSuccess && (mode & kStepCompact))
            e1 = launch_cull_views_dev(m->dm, st->dev[k], kCullGroups, (mode & kStepLaneViews) != 0, cs);
        if (e1 == hipSuccess)
            e1 = launch_integrate_views_dev(m->dm, st->dev[k], st->spherical, m->p.weighting, st->groups,
                                            (mode & kStepCompact) != 0, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &st->graph[k][mode]);
        e = e1 != hipSuccess ? e1 : e2;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&st->exec[k][mode], st->graph[k][mode], nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    return e;
}

extern "C" {

int integrate_depth_views(tsdf_map *m, const tsdf_depth_view *views, int n_views, void *hip_stream)
{
    if (!m)
        return TSDF_EINVAL;
    ViewsArgs va;
    bool spherical = false;
    int st = build_views_args(m, views, n_views, va, spherical);
    if (st != TSDF_OK)
        return st;
    if (m->p.weighting == TSDF_WEIGHT_LEARNED && (spherical || !m->sm_params))
        return TSDF_EINVAL;
    if (m->p.allocation == TSDF_ALLOC_RAY_WALK)
        return TSDF_EINVAL;
    if (m->sticky)
        return TSDF_ESTATE;
    va.parity = (int)(m->frames & 1);
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = use_device(m);
    const bool timed = e == hipSuccess && timing_begin(m, s);   // every kernel of the call, pre-passes included
    if (e == hipSuccess)
        e = prepare_footprint(m, va, s, true);
    if (e == hipSuccess)
        e = prepare_learned(m, va.cam, va.n_views, s);
    if (e == hipSuccess)
        e = prepare_compaction(m, va.lat, va.n_views);
    if (e != hipSuccess)
        return hip_status(e);
    int groups = schedule(m, va.lat);
    if (va.lat.cand) {
        groups = (int)std::max<long long>(kPartitions, (m->launch.max_groups > 0 ? m->launch.max_groups : m->max_groups) /
                                                           kPartitions * kPartitions);
        e = launch_cull_views(m->dm, va, s);
        if (e != hipSuccess)
            return hip_status(e);
    }
    e = launch_integrate_views(m->dm, va, m->p.weighting, groups, s);
    if (e != hipSuccess)
        return hip_status(e);
    timing_end(m, s, timed);
    ++m->frames;
    return TSDF_OK;
}

int tsdf_step_create(tsdf_map *m, int with_spherical, tsdf_step **out)
{
    if (!m || !out)
        return TSDF_EINVAL;
    *out = nullptr;
    if (m->p.weighting == TSDF_WEIGHT_LEARNED || m->p.allocation == TSDF_ALLOC_RAY_WALK)
        return TSDF_EINVAL;
    tsdf_step *st = new (std::nothrow) tsdf_step();
    if (!st)
        return TSDF_ENOMEM;
    st->m = m;
    st->spherical = with_spherical != 0;
    const tsdf_launch_config &lc = m->launch;
    long long groups = lc.max_groups > 0 ? lc.max_groups : m->max_groups;
    st->groups = (int)std::max<long long>(kPartitions, groups / kPartitions * kPartitions);
    hipError_t e = use_device(m);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipHostMalloc((void **)&st->pinned[k], sizeof(ViewsArgs), hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipMalloc((void **)&st->dev[k], sizeof(ViewsArgs));
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&st->done[k], hipEventDisableTiming);
        if (e == hipSuccess)
            std::memset(st->pinned[k], 0, sizeof(ViewsArgs));
    }
    // the plain lattice-walk replay up front, so that capture errors surface here
    if (e == hipSuccess)
        e = step_capture(st, 0, 0);
    if (e != hipSuccess) {
        step_free(st);
        return hip_status(e);
    }
    try {
        m->steps.push_back(st);
    } catch (...) {
        step_free(st);
        return TSDF_ENOMEM;
    }
    *out = st;
    return TSDF_OK;
}

int tsdf_step_run(tsdf_step *st, const tsdf_depth_view *views, int n_views, void *hip_stream)
{
    if (!st)
        return TSDF_EINVAL;
    tsdf_map *m = st->m;
    ViewsArgs va;
    bool spherical = false;
    int rc = build_views_args(m, views, n_views, va, spherical);
    if (rc != TSDF_OK)
        return rc;
    if (spherical && !st->spherical)
        return TSDF_EINVAL;
    if (m->sticky)
        return TSDF_ESTATE;
    va.parity = (int)(m->frames & 1);
    Lattice lat = va.lat;
    (void)schedule(m, lat);      // chunk and partitions for this lattice; the grid is fixed
    va.lat.chunk = lat.chunk;
    va.lat.partitions = lat.partitions;
    hipError_t e = use_device(m);
    if (e == hipSuccess)
        e = prepare_footprint(m, va, nullptr, false);   // the graph builds the pyramids
    if (e == hipSuccess)
        e = prepare_compaction(m, va.lat, va.n_views);              // and culls into the list
    if (e != hipSuccess)
        return hip_status(e);
    int mode = va.lat.cand ? (kStepCompact | (views_share_model(va) ? kStepLaneViews : 0)) : 0;
    for (int v = 0; v < va.n_views; ++v)
        if (va.cam[v].tiles)
            mode |= kStepFootprint;
    const int k = st->next;
    if (st->pending[k] && (e = hipEventSynchronize(st->done[k])) != hipSuccess)
        return hip_status(e);
    if (!st->exec[k][mode] && (e = step_capture(st, k, mode)) != hipSuccess)
        return hip_status(e);
    *st->pinned[k] = va;
    hipStream_t s = (hipStream_t)hip_stream;
    const bool timed = timing_begin(m, s);
    e = hipGraphLaunch(st->exec[k][mode], s);
    if (e == hipSuccess)
        e = hipEventRecord(st->done[k], s);
    if (e != hipSuccess)
        return hip_status(e);
    timing_end(m, s, timed);
    st->pending[k] = true;
    st->next = k ^ 1;
    ++m->frames;
    return TSDF_OK;
}

int tsdf_step_destroy(tsdf_step *st)
{
    if (!st)
        return TSDF_OK;
    (void)use_device(st->m);
    for (int k = 0; k < 2; ++k)
        if (st->pending[k])
            (void)hipEventSynchronize(st->done[k]);
    std::vector<tsdf_step *> &v = st->m->steps;
    v.erase(std::remove(v.begin(), v.end(), st), v.end());
    step_free(st);
    return TSDF_OK;
}

int reserve(tsdf_map *m, long long block_capacity)
{
    if (!m || block_capacity < 1 || block_capacity > (1ll << 30))
        return TSDF_EINVAL;
    if (block_capacity <= (long long)m->dm.block_cap)
        return TSDF_OK;
    // no stream of this process may be capturing: the device is synchronised
    // and memory is allocated and freed below
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(nullptr, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)
        return TSDF_ESTATE;
    hipError_t e = use_device(m);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();    // every queued launch has read the old buffers
    if (e != hipSuccess)
        return hip_status(e);
    const DeviceMap old = m->dm;
    long long hc = (long long)old.hash_mask + 1;
    while (hc < 2 * block_capacity)
        hc *= 2;
    const size_t bc = (size_t)block_capacity;
    const size_t vb = voxel_bytes(old.storage) * kBlockVoxels;
    uint32_t used = 0;
    e = hipMemcpy(&used, old.counters + kNumBlocks, sizeof(used), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_status(e);
    used = std::min(used, old.block_cap);   // slots past the old capacity were never published
    DeviceMap d = old;
    d.keys = nullptr;
    d.vals = nullptr;
    d.pool = nullptr;
    d.slot_keys = nullptr;
    d.touched = nullptr;
    if (e == hipSuccess) e = hipMalloc(&d.keys, sizeof(unsigned long long) * (size_t)hc);
    if (e == hipSuccess) e = hipMalloc(&d.vals, sizeof(uint32_t) * (size_t)hc);
    if (e == hipSuccess) e = hipMalloc(&d.pool, vb * bc);
    if (e == hipSuccess) e = hipMalloc(&d.slot_keys, sizeof(unsigned long long) * bc);
    if (e == hipSuccess) e = hipMalloc(&d.touched, sizeof(uint32_t) * bc * kSubLists);
    if (e == hipSuccess) e = hipMemset(d.keys, 0xFF, sizeof(unsigned long long) * (size_t)hc);
    if (e == hipSuccess) e = hipMemset(d.vals, 0xFF, sizeof(uint32_t) * (size_t)hc);
    // blocks keep their pool slots; the new tail of the pool is zero (fresh blocks need no clearing)
    if (e == hipSuccess && used > 0) e = hipMemcpy(d.pool, old.pool, vb * used, hipMemcpyDeviceToDevice);
    if (e == hipSuccess) e = hipMemset((char *)d.pool + vb * used, 0, vb * (bc - used));
    if (e == hipSuccess && used > 0)
        e = hipMemcpy(d.slot_keys, old.slot_keys, sizeof(unsigned long long) * used, hipMemcpyDeviceToDevice);
    if (e == hipSuccess)
        e = hipMemset(d.slot_keys + used, 0xFF, sizeof(unsigned long long) * (bc - used));
    // the last launch's touched sub-lists, at the new stride
    for (int k = 0; k < kSubLists && e == hipSuccess; ++k)
        e = hipMemcpy(d.touched + (size_t)k * bc, old.touched + (size_t)k * old.block_cap,
                      sizeof(uint32_t) * old.block_cap, hipMemcpyDeviceToDevice);
    if (e == hipSuccess && used > 0)
        e = launch_rehash(d.slot_keys, used, d.keys, d.vals, (uint32_t)(hc - 1), nullptr);
    // recovery: the counter drops back to the slots in use and the error word clears
    const uint32_t zero = 0;
    if (e == hipSuccess) e = hipMemcpy(d.counters + kNumBlocks, &used, sizeof(used), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d.counters + kErrorBits, &zero, sizeof(zero), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipDeviceSynchronize();
        (void)hipFree(d.keys);
        (void)hipFree(d.vals);
        (void)hipFree(d.pool);
        (void)hipFree(d.slot_keys);
        (void)hipFree(d.touched);
        return hip_status(e);
    }
    // graphs of the map's steps hold the old buffers: capture them again on their next run
    for (tsdf_step *st : m->steps) {
        for (int k = 0; k < 2; ++k)
            if (st->pending[k]) {
                (void)hipEventSynchronize(st->done[k]);
                st->pending[k] = false;
            }
        step_drop_graphs(st);
    }
    (void)hipFree(old.keys);
    (void)hipFree(old.vals);
    (void)hipFree(old.pool);
    (void)hipFree(old.slot_keys);
    (void)hipFree(old.touched);
    free_query_buffers(m);
    d.hash_mask = (uint32_t)(hc - 1);
    d.block_cap = (uint32_t)bc;
    m->dm = d;
    m->p.block_capacity = block_capacity;
    m->p.hash_capacity = hc;
    m->sticky = 0;
    return TSDF_OK;
}

int query_blocks(tsdf_map *m, int32_t *out_xyz_dev, long long capacity, long long *out_count, void *hip_stream)
{
    if (!m || !out_count || capacity < 0 || (capacity > 0 && !out_xyz_dev))
        return TSDF_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(m->device) != hipSuccess)
        return TSDF_EDEVICE;
    CounterSnapshot cs;
    int st = read_counters(m, cs, s);
    if (st != TSDF_OK)
        return st;
    const long long n = std::min<long long>(cs.c[kNumBlocks], m->dm.block_cap);
    *out_count = 0;
    if (n == 0)
        return TSDF_OK;
    // work buffers sized for the whole pool, kept for later calls
    hipError_t e = hipSuccess;
    if (!m->q_sorted)
        e = hipMalloc((void **)&m->q_sorted, sizeof(unsigned long long) * (size_t)m->dm.block_cap);
    if (e == hipSuccess && !m->q_count)
        e = hipMalloc((void **)&m->q_count, sizeof(unsigned long long));
    size_t need = 0;
    if (e == hipSuccess)
        e = sort_keys(m->dm.slot_keys, m->q_sorted, n, nullptr, &need, s);
    if (e == hipSuccess && (!m->q_temp || need > m->q_temp_bytes)) {
        size_t full = 0;   // the work space of a full pool, so that later calls never grow it
        e = sort_keys(m->dm.slot_keys, m->q_sorted, m->dm.block_cap, nullptr, &full, s);
        if (e == hipSuccess) {
            (void)hipFree(m->q_temp);
            m->q_temp = nullptr;
            m->q_temp_bytes = 0;
            const size_t bytes = std::max<size_t>(std::max(need, full), 1);
            e = hipMalloc(&m->q_temp, bytes);
            if (e == hipSuccess)
                m->q_temp_bytes = bytes;
        }
    }
    if (e == hipSuccess) {
        size_t bytes = m->q_temp_bytes;
        e = sort_keys(m->dm.slot_keys, m->q_sorted, n, m->q_temp, &bytes, s);
    }
    // every slot below the count holds its key; the count of valid keys is
    // taken on the device all the same (an unwritten slot keeps kEmptyKey,
    // which sorts last)
    if (e == hipSuccess)
        e = launch_count_valid(m->q_sorted, n, m->q_count, s);
    if (e == hipSuccess && capacity > 0)
        e = launch_decode_keys(m->q_sorted, std::min(n, capacity), out_xyz_dev, s);
    unsigned long long valid = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&valid, m->q_count, sizeof(valid), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_status(e);
    *out_count = (long long)valid;
    return TSDF_OK;   // a map in a sticky error state is still readable
}

int query_tsdf(tsdf_map *m, const int32_t *blocks_xyz_dev, long long n_blocks, float *out_dist_dev,
               float *out_weight_dev, void *hip_stream)
{
    if (!m || n_blocks < 0 || (n_blocks > 0 && (!blocks_xyz_dev || !out_dist_dev || !out_weight_dev)))
        return TSDF_EINVAL;
    if (n_blocks == 0)
        return TSDF_OK;
    if (hipSetDevice(m->device) != hipSuccess)
        return TSDF_EDEVICE;
    return hip_status(launch_query_tsdf(m->dm, blocks_xyz_dev, n_blocks, out_dist_dev, out_weight_dev,
                                        (hipStream_t)hip_stream));
}

int insert_blocks(tsdf_map *m, const int32_t *blocks_xyz_dev, long long n_blocks, const float *dist_dev,
                  const float *weight_dev, void *hip_stream)
{
    if (!m || n_blocks < 0 || (n_blocks > 0 && (!blocks_xyz_dev || !dist_dev || !weight_dev)))
        return TSDF_EINVAL;
    if (m->sticky)
        return TSDF_ESTATE;
    if (n_blocks == 0)
        return TSDF_OK;
    if (use_device(m) != hipSuccess)
        return TSDF_EDEVICE;
    return hip_status(launch_insert_blocks(m->dm, blocks_xyz_dev, n_blocks, dist_dev, weight_dev,
                                           (hipStream_t)hip_stream));
}

int query_touched(tsdf_map *m, int32_t *out_xyz_dev, long long capacity, long long *out_count, void *hip_stream)
{
    if (!m || !out_count || capacity < 0 || (capacity > 0 && !out_xyz_dev))
        return TSDF_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipSetDevice(m->device) != hipSuccess)
        return TSDF_EDEVICE;
    CounterSnapshot cs;
    int st = read_counters(m, cs, s);
    if (st != TSDF_OK)
        return st;
    long long per[kSubLists];
    last_touched_counts(m, cs, per);
    long long n = 0;
    for (int k = 0; k < kSubLists; ++k)
        n += per[k];
    *out_count = n;
    long long written = 0;
    for (int k = 0; k < kSubLists && written < capacity; ++k) {
        const long long take = std::min(per[k], capacity - written);
        if (take <= 0)
            continue;
        hipError_t e = launch_gather_touched(m->dm, k, take, out_xyz_dev + 3 * written, s);
        if (e != hipSuccess)
            return hip_status(e);
        written += take;
    }
    if (written > 0) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return hip_status(e);
    }
    return TSDF_OK;
}

int map_stats(tsdf_map *m, tsdf_stats *out, void *hip_stream)
{
    if (!m || !out)
        return TSDF_EINVAL;
    if (hipSetDevice(m->device) != hipSuccess)
        return TSDF_EDEVICE;
    CounterSnapshot cs;
    int st = read_counters(m, cs, (hipStream_t)hip_stream);
    if (st != TSDF_OK)
        return st;
    unsigned long long upd = 0, wr = 0, cand = 0;
    for (int k = 0; k < kSubLists; ++k) {
        upd += cs.t[kTotalUpdates + k * kTotalsStride];
        wr += cs.t[kTotalWrites + k * kTotalsStride];
        cand += cs.t[kTotalCandidates + k * kTotalsStride];
    }
    long long per[kSubLists];
    last_touched_counts(m, cs, per);
    long long touched = (long long)cs.t[kTotalTouched];
    for (int k = 0; k < kSubLists; ++k)
        touched += per[k];
    out->blocks = std::min<long long>(cs.c[kNumBlocks], m->dm.block_cap);
    out->voxel_updates = (long long)upd;
    out->voxel_writes = (long long)wr;
    out->touched_blocks = touched;
    out->launches = m->frames;
    out->candidate_blocks = (long long)cand;
    out->block_capacity = (long long)m->dm.block_cap;
    out->hash_capacity = (long long)m->dm.hash_mask + 1;
    out->error_bits = (long long)cs.c[kErrorBits];
    return TSDF_OK;
}

int map_status(tsdf_map *m)
{
    if (!m)
        return TSDF_EINVAL;
    if (hipSetDevice(m->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        return TSDF_EDEVICE;
    CounterSnapshot cs;
    int st = read_counters(m, cs, nullptr);
    if (st != TSDF_OK)
        return st;
    return m->sticky;
}

const char *tsdf_strerror(int status)
{
    switch (status) {
    case TSDF_OK: return "ok";
    case TSDF_EINVAL: return "invalid argument";
    case TSDF_ENOMEM: return "out of device memory";
    case TSDF_EFULL: return "map capacity exceeded (block pool, hash table or touched list)";
    case TSDF_EDEVICE: return "HIP runtime error";
    case TSDF_ESTATE: return "map is in a sticky error state";
    case TSDF_ESCRATCH: return "call needs more than the fixed scratch of the no-allocation entry point";
    default: return "unknown status";
    }
}

int tsdf_set_launch_config(tsdf_map *m, const tsdf_launch_config *lc)
{
    if (!m)
        return TSDF_EINVAL;
    tsdf_launch_config c = {0, 0, 0, 0, 0, 0};
    if (lc)
        c = *lc;
    if (c.max_groups < 0 || c.max_groups > 65536 || c.chunk < 0 || c.chunk > kMaxChunk ||
        (c.footprint != TSDF_FOOTPRINT_AUTO && c.footprint != TSDF_FOOTPRINT_NEVER &&
         c.footprint != TSDF_FOOTPRINT_ALWAYS) ||
        (c.compaction != TSDF_COMPACT_AUTO && c.compaction != TSDF_COMPACT_NEVER &&
         c.compaction != TSDF_COMPACT_ALWAYS) ||
        (c.partitions != 0 && c.partitions != 1 && c.partitions != kPartitions) ||
        (c.staging != TSDF_STAGE_AUTO && c.staging != TSDF_STAGE_NEVER && c.staging != TSDF_STAGE_ALWAYS))
        return TSDF_EINVAL;
    m->launch = c;
    return TSDF_OK;
}

int tsdf_profile(tsdf_map *m, int enable)
{
    if (!m)
        return TSDF_EINVAL;
    m->profiling = enable != 0;
    m->ev_used = 0;
    return TSDF_OK;
}

int tsdf_profile_read(tsdf_map *m, double *total_ms, long long *launches)
{
    if (!m || !total_ms || !launches)
        return TSDF_EINVAL;
    double sum = 0;
    for (size_t k = 0; k < m->ev_used; ++k) {
        if (hipEventSynchronize(m->ev_stop[k]) != hipSuccess)
            return TSDF_EDEVICE;
        float ms = 0;
        if (hipEventElapsedTime(&ms, m->ev_start[k], m->ev_stop[k]) != hipSuccess)
            return TSDF_EDEVICE;
        sum += ms;
    }
    *total_ms = sum;
    *launches = (long long)m->ev_used;
    m->ev_used = 0;
    return TSDF_OK;
}

}  // extern "C"

// ---- learned sensor model ------------------------------------------------

struct tsdf_sm_trainer {
    int width, height, max_frames;
    int device;
    float2 *maps;      // max_frames x H x W (weight, truncation)
    float *gw, *ge;    // max_frames x H x W gradients with respect to weight and truncation
    double *acc;       // [0] sum of squared errors, [1] voxels reached
};

namespace {

bool bf16_params_valid(const float *p, int n)
{
    for (int k = 0; k < n; ++k) {
        uint32_t u;
        std::memcpy(&u, &p[k], 4);
        if (!std::isfinite(p[k]) || (u & 0xFFFFu) != 0)
            return false;
    }
    return true;
}

// Camera-from-world of a rigid pose, as for integration: R^T exactly, -R^T t
// accumulated in binary64 and rounded once.
void pose_inverse(const float T[16], float R[9], float t[3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            R[3 * i + j] = T[4 * j + i];
    for (int i = 0; i < 3; ++i) {
        const double acc = ((double)T[0 * 4 + i] * (double)T[3] + (double)T[1 * 4 + i] * (double)T[7]) +
                           (double)T[2 * 4 + i] * (double)T[11];
        t[i] = (float)(-acc);
    }
}

void trainer_free(tsdf_sm_trainer *t)
{
    (void)hipFree(t->maps);
    (void)hipFree(t->gw);
    (void)hipFree(t->ge);
    (void)hipFree(t->acc);
    delete t;
}

}  // namespace

extern "C" {

int tsdf_set_sensor_model(tsdf_map *m, const float *params)
{
    if (!m || !params || !bf16_params_valid(params, kSmParams))
        return TSDF_EINVAL;
    hipError_t e = use_device(m);
    if (e == hipSuccess && !m->sm_params)
        e = hipMalloc((void **)&m->sm_params, sizeof(float) * kSmParams);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();   // no launch may still read the previous parameters
    if (e == hipSuccess)
        e = hipMemcpy(m->sm_params, params, sizeof(float) * kSmParams, hipMemcpyHostToDevice);
    return hip_status(e);
}

int tsdf_sensor_maps(const float *depth_dev, int width, int height, const float K[4], float max_range,
                     float voxel_size, const float *params_dev, float *maps_dev, void *hip_stream)
{
    if (!depth_dev || !params_dev || !maps_dev || !K || width <= 0 || height <= 0 ||
        (long long)width * height > (1ll << 28) || !finite_all(K, 4) || !(K[0] > 0.0f && K[1] > 0.0f) ||
        !(max_range > 0.0f && std::isfinite(max_range)) || !(voxel_size > 0.0f && std::isfinite(voxel_size)))
        return TSDF_EINVAL;
    SmView v{depth_dev, width, height, K[0], K[1], K[2], K[3], max_range};
    return hip_status(launch_sm_maps(v, voxel_size, params_dev, (float2 *)maps_dev, (hipStream_t)hip_stream));
}

int tsdf_sm_trainer_create(int width, int height, int max_frames, tsdf_sm_trainer **out)
{
    if (!out)
        return TSDF_EINVAL;
    *out = nullptr;
    if (width <= 0 || height <= 0 || (long long)width * height > (1ll << 26) || max_frames < 1 ||
        max_frames > kSmMaxFrames)
        return TSDF_EINVAL;
    tsdf_sm_trainer *t = new (std::nothrow) tsdf_sm_trainer();
    if (!t)
        return TSDF_ENOMEM;
    t->width = width;
    t->height = height;
    t->max_frames = max_frames;
    const size_t px = (size_t)width * height * (size_t)max_frames;
    hipError_t e = hipGetDevice(&t->device);
    if (e == hipSuccess) e = hipMalloc((void **)&t->maps, sizeof(float2) * px);
    if (e == hipSuccess) e = hipMalloc((void **)&t->gw, sizeof(float) * px);
    if (e == hipSuccess) e = hipMalloc((void **)&t->ge, sizeof(float) * px);
    if (e == hipSuccess) e = hipMalloc((void **)&t->acc, sizeof(double) * 2);
    if (e != hipSuccess) {
        trainer_free(t);
        return hip_status(e);
    }
    *out = t;
    return TSDF_OK;
}

int tsdf_sm_trainer_destroy(tsdf_sm_trainer *t)
{
    if (!t)
        return TSDF_OK;
    (void)hipSetDevice(t->device);
    (void)hipDeviceSynchronize();
    trainer_free(t);
    return TSDF_OK;
}

int tsdf_sm_loss_grad(tsdf_sm_trainer *t, const float *params_dev, int n_frames, const float *const *depth_dev,
                      const float K[4], const float *T_world_cam, float voxel_size, float max_range, long long n_vox,
                      const int *vox_dev, const float *target_dev, float *grad_dev, double *loss_host,
                      void *hip_stream)
{
    if (!t || !params_dev || !depth_dev || !K || !T_world_cam || !grad_dev || n_frames < 1 ||
        n_frames > t->max_frames || n_vox < 0 || (n_vox > 0 && (!vox_dev || !target_dev)) || !finite_all(K, 4) ||
        !(K[0] > 0.0f && K[1] > 0.0f) || !(max_range > 0.0f && std::isfinite(max_range)) ||
        !(voxel_size > 0.0f && std::isfinite(voxel_size)))
        return TSDF_EINVAL;
    for (int f = 0; f < n_frames; ++f)
        if (!depth_dev[f] || !pose_valid(T_world_cam + 16 * f))
            return TSDF_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(t->device);
    const long long wh = (long long)t->width * t->height;
    SmLossArgs la;
    std::memset(&la, 0, sizeof(la));
    SmBackArgs ba;
    std::memset(&ba, 0, sizeof(ba));
    for (int f = 0; f < n_frames && e == hipSuccess; ++f) {
        SmView v{depth_dev[f], t->width, t->height, K[0], K[1], K[2], K[3], max_range};
        float2 *maps = t->maps + (size_t)f * (size_t)wh;
        e = launch_sm_maps_mfma(v, voxel_size, params_dev, maps, s);   // the function the backward recomputes
        SmFrame &fr = la.frames[f];
        pose_inverse(T_world_cam + 16 * f, fr.R, fr.t);
        fr.depth = depth_dev[f];
        fr.maps = maps;
        fr.gw = t->gw + (size_t)f * (size_t)wh;
        fr.ge = t->ge + (size_t)f * (size_t)wh;
        ba.views[f] = v;
    }
    if (e == hipSuccess) e = launch_sm_fill(t->gw, wh * n_frames, 0.0f, s);
    if (e == hipSuccess) e = launch_sm_fill(t->ge, wh * n_frames, 0.0f, s);
    if (e == hipSuccess) e = launch_sm_fill(grad_dev, kSmParams, 0.0f, s);
    la.n_frames = n_frames;
    la.width = t->width;
    la.height = t->height;
    la.fx = K[0];
    la.fy = K[1];
    la.cx = K[2];
    la.cy = K[3];
    la.d_max = max_range;
    la.vs = voxel_size;
    la.n_vox = n_vox;
    la.vox = vox_dev;
    la.target = target_dev;
    la.acc = t->acc;
    if (e == hipSuccess) e = launch_sm_loss(la, s);
    ba.n_frames = n_frames;
    ba.width = t->width;
    ba.height = t->height;
    ba.vs = voxel_size;
    ba.params = params_dev;
    ba.gw = t->gw;
    ba.ge = t->ge;
    ba.acc = t->acc;
    ba.grad = grad_dev;
    if (e == hipSuccess) e = launch_sm_backward(ba, s);
    if (e == hipSuccess && loss_host) {
        double acc[2];
        e = hipMemcpyAsync(acc, t->acc, sizeof(acc), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess) {
            loss_host[0] = acc[1] > 0.0 ? acc[0] / acc[1] : 0.0;
            loss_host[1] = acc[1];
        }
    }
    return hip_status(e);
}

int tsdf_sm_adam(float *master_dev, float *m1_dev, float *m2_dev, const float *grad_dev, float *params_dev, int n,
                 float lr, float beta1, float beta2, float eps, int step, void *hip_stream)
{
    if (!master_dev || !m1_dev || !m2_dev || !grad_dev || !params_dev || n <= 0 || step < 1 ||
        !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return TSDF_EINVAL;
    return hip_status(launch_sm_adam(master_dev, m1_dev, m2_dev, grad_dev, params_dev, n, lr, beta1, beta2, eps, step,
                                     (hipStream_t)hip_stream));
}

}  // extern "C"

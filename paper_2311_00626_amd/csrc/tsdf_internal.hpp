// Internal declarations shared by the HIP kernels and the host ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsdf {

constexpr unsigned long long kEmptyKey = ~0ull;     // hash slot never used
constexpr uint32_t kInvalidSlot = 0xFFFFFFFFu;      // hash value not yet published
constexpr uint32_t kNoSlot = 0xFFFFFFFEu;           // key inserted when the pool was full: no block
constexpr int kBlockVoxels = 512;                   // 8 x 8 x 8 voxels per block (§IV-A)
constexpr int kKeyBits = 21;                        // bits per packed block coordinate
constexpr int kKeyOffset = 1 << 20;                 // block coordinate bias
constexpr int kBlockCoordMax = (1 << 20) - 1;       // |block index| limit on every axis
constexpr int kWavesPerGroup = 8;                   // 512-thread workgroups of wave64
constexpr int kQueryWavesPerGroup = 4;              // 256-thread workgroups for the query kernels
constexpr int kSubLists = 8;                        // touched list split over 8 counters / cache lines
constexpr int kPartitions = 8;                      // XCDs: block ownership bands, one per XCD
constexpr int kXcds = 8;               // MI355X: 8 XCDs, workgroups dispatched round-robin
constexpr int kMaxChunk = 64;
// Cull kernel of a compacted launch: threads per workgroup, and the most
// workgroups a launch uses (the grid strides over larger lattices).  Three
// 512-thread groups fit a CU at the kernel's register use where one
// 1024-thread group did, which keeps more footprint lookups in flight.
constexpr int kCullThreads = 512;
constexpr int kCullGroups = 2048;                       // lattice blocks culled together by one wave
constexpr int kLineWords = 32;                      // 128-byte line in 32-bit words

// Weighting functions (the tsdf_params weighting codes).
constexpr int kWeightConstant = 0;
constexpr int kWeightDropoff = 1;
constexpr int kWeightLearned = 2;

// Learned sensor model: a per-pixel perceptron 27 -> 32 -> 32 -> 2 with
// parameters W1[32][27], b1[32], W2[32][32], b2[32], W3[2][32], b3[2].
constexpr int kSmIn = 27, kSmHidden = 32, kSmOut = 2;
constexpr int kSmW1 = 0, kSmB1 = kSmW1 + kSmHidden * kSmIn, kSmW2 = kSmB1 + kSmHidden,
              kSmB2 = kSmW2 + kSmHidden * kSmHidden, kSmW3 = kSmB2 + kSmHidden, kSmB3 = kSmW3 + kSmOut * kSmHidden,
              kSmParams = kSmB3 + kSmOut;

// Depth footprint pyramid: per view, the largest valid measurement of every
// tile of 8, 16, 32 and 64 pixels; images up to kTileMaxSide pixels a side.
constexpr int kTileLevels = 4;
constexpr int kTileBaseShift = 3;                    // level l tiles are 8 << l pixels wide
constexpr int kTileMaxSide = 4096;
constexpr long long kTileFloatsPerView = 348160;     // sum over levels of (4096 / (8 << l))^2
constexpr int kTileSuper = 64;                       // pixels a side of one pyramid workgroup

// Counter words, one hot counter per 128-byte line so that atomics on
// different counters never share a line.
enum Counter : int {
    kNumBlocks = 0,                                  // pool slots handed out (may exceed capacity after overflow)
    kErrorBits = 1 * kLineWords,                     // sticky ErrorBits
    kTouchedBase = 2 * kLineWords,                   // [parity][sub-list] touched counts
    kCandBase = (2 + 2 * kSubLists) * kLineWords,    // [parity] candidate-list lengths (compacted launches)
    kNumCounterWords = (4 + 2 * kSubLists) * kLineWords
};
__host__ __device__ constexpr int cand_counter(int parity)
{
    return kCandBase + parity * kLineWords;
}
__host__ __device__ constexpr int touched_counter(int parity, int sub)
{
    return kTouchedBase + (parity * kSubLists + sub) * kLineWords;
}
constexpr int kTotalsStride = 16;                   // 64-bit words per 128-byte line
enum Total : int {
    kTotalUpdates = 0,                               // kSubLists lines of voxel-update sub-totals
    kTotalWrites = kSubLists * kTotalsStride,        // kSubLists lines of voxel-write sub-totals
    kTotalTouched = 2 * kSubLists * kTotalsStride,   // touched blocks of completed earlier launches
    kTotalCandidates = (2 * kSubLists + 1) * kTotalsStride,   // kSubLists lines: candidate blocks measured
    kNumTotalWords = (3 * kSubLists + 1) * kTotalsStride
};

enum ErrorBits : uint32_t {
    kErrPoolFull = 1u,
    kErrHashFull = 2u,
    kErrTouchedOverflow = 4u,
    kErrInsertRace = 8u,
    kErrWalkOutside = 16u,     // a ray walk left the frame's lattice (a bound was too small)
};

// Device-side view of a map.  Passed to kernels by value.
struct DeviceMap {
    unsigned long long *keys;        // [hash_mask + 1] packed block keys, kEmptyKey = free
    uint32_t *vals;                  // [hash_mask + 1] pool slot of the key, kInvalidSlot until published
    void *pool;                      // [block_cap * 512] (distance, weight) per voxel: float2 or half2
    unsigned long long *slot_keys;   // [block_cap] key of each pool slot
    uint32_t *touched;               // [kSubLists][block_cap] pool slots touched by the last frame
    uint32_t *counters;              // [kNumCounterWords]
    unsigned long long *totals;      // [kNumTotalWords] running totals
    uint32_t hash_mask;
    uint32_t block_cap;
    int storage;                     // 0: binary32 pairs, 1: binary16 pairs
};

constexpr uint32_t voxel_bytes(int storage) { return storage == 1 ? 4u : 8u; }

constexpr int kModelPinhole = 0;                    // depth camera, Eq. (2)
constexpr int kModelSpherical = 1;                  // rotating LiDAR range image, Eq. (3)

// One depth view and its pose (host-computed, passed by value).
struct CameraView {
    float R[9];             // sensor-from-world rotation, row-major (T_CL of Eq. (1))
    float t[3];             // sensor-from-world translation
    float fx, fy, cx, cy;   // pinhole intrinsics (Eq. (2))
    float width_f, height_f;
    int width, height;
    const float *depth;     // device float32[height][width]: z-depth or range
    float d_max;            // max valid measurement of this view
    float zfar;             // pinhole: no voxel beyond this camera z is updated; spherical: range
    float margin_u, margin_v;   // conservative slack of the side culling planes
    int model;              // kModelPinhole or kModelSpherical
    // spherical model (Eq. (3)); sensor frame x forward, y left, z up
    float az_start, alpha;  // azimuth of column 0's left edge, columns per radian
    float pol_start, beta;  // polar angle (from +z) of row 0's top edge, rows per radian
    float interp_diff;      // largest spread of the 4 interpolated ranges
    int full_circle;        // columns wrap around
    float origin[3];        // sensor centre in the world (range culling)
    float cos_pol_start, cos_pol_end;   // polar band edges (cone culling)
    // learned sensor model: per-pixel (weight, truncation) pairs (pinhole views)
    const float2 *sm_maps;
    // ray-walk allocation: byte per lattice entry, set for the blocks the walk
    // visited (nullptr: exact-touch allocation with culling)
    unsigned char *dda_marks;     // ray-walk marks over the lattice; the integration kernel clears
                                  // each mark it reads, so the map is all zero between frames
    // depth footprint pyramid of this view (nullptr: no footprint culling)
    float *tiles;
    int tile_cols[kTileLevels];         // tiles per row at each level
    int tile_rows[kTileLevels];
    int tile_off[kTileLevels];          // float offset of each level from `tiles`
};

// Per-map constants in binary32.
struct MapConsts {
    float vs;               // voxel edge
    float eps;              // truncation distance epsilon
    float delta;            // start of the linear weight dropoff behind the surface
    float span_inv;         // 1 / (epsilon - delta)
    float w_max;            // weight cap
    float margin_z;         // conservative slack of the near/far culling planes
};

// Block lattice scanned by one launch.  Waves cull `chunk` consecutive
// lattice entries at a time, one per lane.
struct Lattice {
    int lat_min[3];         // inclusive lower corner (block indices)
    int lat_dim[3];
    long long n_lat;        // lat_dim[0] * lat_dim[1] * lat_dim[2], below 2^31
    // Division of a lattice index n < 2^31 by lat_dim[a] (a = 0, 1) as a
    // multiply and shift: n / d = (n * div_m[a]) >> div_s[a] with
    // s = 31 + ceil(log2 d) and m = ceil(2^s / d) < 2^32.  Exact: writing
    // m d = 2^s + e with 0 <= e < d, n m / 2^s = n / d + n e / (d 2^s), and
    // n e < 2^31 d <= 2^s, so the added term is below 1 / d and the floor
    // does not move (set_lattice_divisors).
    uint32_t div_m[2];
    int div_s[2];
    int chunk;              // 1 .. kMaxChunk
    int partitions;         // 1 or kPartitions ownership bands
    int group_scan;         // nonzero: the walk culls and compacts per workgroup (scan_lattice_group)
    // Compacted launches: a cull kernel writes the surviving blocks (lattice
    // index, view mask) here and the integration kernel deals them out to its
    // waves; nullptr: the integration kernel walks the lattice itself.
    uint2 *cand;
};

// Multiply-shift divisors of a lattice's x and y extents (Lattice::div_m).
inline void set_lattice_divisors(Lattice &lat)
{
    for (int a = 0; a < 2; ++a) {
        const unsigned long long d = (unsigned long long)lat.lat_dim[a];
        int c = 0;
        while ((1ull << c) < d)
            ++c;
        const int s = 31 + c;
        lat.div_s[a] = s;
        lat.div_m[a] = (uint32_t)(((1ull << s) + d - 1) / d);
    }
}

// Culling of a single pinhole view in lattice-relative block coordinates
// l = b - lat_min (set by the host once the launch's lattice is known).  The
// camera-frame corner of block l is cam[4a] l_x + cam[4a+1] l_y + cam[4a+2]
// l_z + cam[4a+3] on axis a (the first three columns are the camera-frame
// block edges), and each frustum plane's largest value over the block, plus
// its margin, is plane[4p] l_x + plane[4p+1] l_y + plane[4p+2] l_z +
// plane[4p+3]: the block is culled where that is negative.
struct PinholeCull {
    float cam[12];
    float plane[24];
    int valid;              // 0: the launch culls through CameraView alone
};

// Arguments of a single-frame launch.
struct FrameArgs {
    CameraView cam;
    MapConsts mc;
    Lattice lat;
    PinholeCull pc;
    int parity;             // launch counter & 1: selects this launch's touched counters
    int stage;              // nonzero: stage block depth footprints in LDS (pinhole, fixed weighting)
};

// Arguments of a multi-view launch: views are fused per voxel in array order.
constexpr int kMaxViews = 16;
struct ViewsArgs {
    CameraView cam[kMaxViews];
    int n_views;
    MapConsts mc;
    Lattice lat;
    int parity;
};

__host__ __device__ inline unsigned long long pack_key(int x, int y, int z)
{
    return ((unsigned long long)(uint32_t)(x + kKeyOffset) << (2 * kKeyBits)) |
           ((unsigned long long)(uint32_t)(y + kKeyOffset) << kKeyBits) |
           (unsigned long long)(uint32_t)(z + kKeyOffset);
}

__host__ __device__ inline void unpack_key(unsigned long long k, int &x, int &y, int &z)
{
    const unsigned long long m = (1ull << kKeyBits) - 1ull;
    x = (int)((k >> (2 * kKeyBits)) & m) - kKeyOffset;
    y = (int)((k >> kKeyBits) & m) - kKeyOffset;
    z = (int)(k & m) - kKeyOffset;
}

// splitmix64 finaliser: spreads packed keys over the table.
__host__ __device__ inline unsigned long long hash_key(unsigned long long k)
{
    k ^= k >> 30;
    k *= 0xBF58476D1CE4E5B9ull;
    k ^= k >> 27;
    k *= 0x94D049BB133111EBull;
    k ^= k >> 31;
    return k;
}

// Linear probing from the first slot of the key's 16-slot bucket: the first
// probe window is then exactly one 128-byte line of keys and one 64-byte line
// of values.  Every insert and lookup scans slots in the same order from here.
constexpr uint32_t kBucketSlots = 16;
__host__ __device__ inline uint32_t probe_start(unsigned long long key, uint32_t mask)
{
    return (uint32_t)hash_key(key) & mask & ~(kBucketSlots - 1u);
}
// What a probe-window lane that reads no slot holds: bit 63 set, so it is
// neither kEmptyKey nor any packed key (3 x 21 bits).
constexpr unsigned long long kNoKey = ~0ull - 1ull;

// Kernel launchers (integrate.hip, query.hip).
// groups: workgroups of the launch; with fill_cus > 0 a compacted launch
// (fa.lat.cand) instead takes as many as its list kernel keeps resident on
// fill_cus compute units (a multiple of kPartitions, at least kPartitions).
hipError_t launch_integrate_depth(const DeviceMap &dm, const FrameArgs &fa, int weighting, int groups,
                                  hipStream_t stream, int fill_cus = 0);
hipError_t launch_integrate_views(const DeviceMap &dm, const ViewsArgs &va, int weighting, int groups,
                                  hipStream_t stream);
// list: the compacted form (the cull kernel ran before it), else the lattice walk
hipError_t launch_integrate_views_dev(const DeviceMap &dm, const ViewsArgs *va_dev, bool spherical, int weighting,
                                      int groups, bool list, hipStream_t stream);
hipError_t launch_query_tsdf(const DeviceMap &dm, const int32_t *xyz, long long n, float *dist,
                             float *weight, hipStream_t stream);
hipError_t launch_decode_keys(const unsigned long long *keys, long long n, int32_t *xyz,
                              hipStream_t stream);
// Compacted launches (integrate.hip, integrate_views.hip): the cull kernels
// fill lat.cand; the list kernels integrate its entries.
hipError_t launch_cull_frame(const DeviceMap &dm, const FrameArgs &fa, hipStream_t stream);
// Finds or inserts n blocks (int32 triples) and writes their 512 (distance,
// weight) pairs each (insert.hip).
hipError_t launch_insert_blocks(const DeviceMap &dm, const int32_t *xyz, long long n, const float *dist,
                                const float *weight, hipStream_t stream);
hipError_t launch_cull_views(const DeviceMap &dm, const ViewsArgs &va, hipStream_t stream);
// lane_views: the views share one camera model (see views_share_model)
hipError_t launch_cull_views_dev(const DeviceMap &dm, const ViewsArgs *va_dev, int groups, bool lane_views,
                                 hipStream_t stream);
// true when every view of the batch has the first view's camera model
bool views_share_model(const ViewsArgs &va);

// Ray-walk allocation pre-pass (dda.hip).
struct DdaArgs {
    float Rwc[9];           // world-from-camera rotation, row-major
    float o[3];             // camera centre in the world
    float fx, fy, cx, cy;
    int width, height;
    const float *depth;
    float d_max, eps, vs;
    Lattice lat;            // the launch's lattice (marks are indexed by lattice entry)
    unsigned char *marks;
    uint32_t *overflow;     // set when a walk leaves the lattice (a bound was too small)
};
// Marks the blocks the frame's pixel rays enter (the mark map must be zero).
hipError_t launch_dda_mark(const DdaArgs &a, hipStream_t stream);
// Zeroes n bytes (the mark map when it is allocated, or after a failed frame).
hipError_t launch_fill_u8(unsigned char *p, long long n, hipStream_t stream);

// Builds the footprint pyramids of the views whose `tiles` is set.
hipError_t launch_footprint_tiles(const ViewsArgs &va, hipStream_t stream);
hipError_t launch_footprint_tiles_dev(const ViewsArgs *va_dev, hipStream_t stream);
hipError_t launch_gather_touched(const DeviceMap &dm, int sub, long long n, int32_t *xyz, hipStream_t stream);
// temp == nullptr: *temp_bytes receives the work space n keys need
hipError_t sort_keys(const unsigned long long *in, unsigned long long *out, long long n, void *temp,
                     size_t *temp_bytes, hipStream_t stream);
// *count = number of keys before the first kEmptyKey of n ascending keys
hipError_t launch_count_valid(const unsigned long long *keys, long long n, unsigned long long *count,
                              hipStream_t stream);
// Inserts the keys of pool slots [0, n) into an empty table of mask + 1 slots.
hipError_t launch_rehash(const unsigned long long *slot_keys, uint32_t n, unsigned long long *keys, uint32_t *vals,
                         uint32_t mask, hipStream_t stream);

// Fixed scratch of the no-allocation entry point (noalloc.hip): one view's
// footprint pyramid, then a candidate list of kNoAllocMaxCandidates entries.
constexpr size_t kNoAllocTileBytes = sizeof(float) * (size_t)kTileFloatsPerView;   // a multiple of 256
constexpr long long kNoAllocMaxCandidates = 1ll << 20;
constexpr size_t kNoAllocScratchBytes = kNoAllocTileBytes + 8u * (size_t)kNoAllocMaxCandidates;
static_assert(kNoAllocTileBytes % 256 == 0, "candidate list alignment");
// Device address of the scratch on the current device (looked up once per device).
hipError_t noalloc_scratch(void **out);

}  // namespace tsdf

// Device-side building blocks shared by the integration kernels: wave
// primitives, raw buffer access, the block hash (find / find-or-insert),
// frustum culling of blocks, the per-voxel measurement of a pinhole depth
// image and the touched-list compaction.
//
// Every floating-point statement in measure_pinhole and fuse is one IEEE
// binary32 operation in the order the CPU oracle uses (files including this
// header are compiled with -ffp-contract=off and correctly rounded division).
#pragma once

#include "tsdf_internal.hpp"

namespace tsdf {
namespace dev {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ int wave_bcast(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Raw buffer descriptors (word 3 of the gfx9-family resource: 32-bit data
// format).  A load whose offset is at or past num_records returns 0 and a
// store there is dropped, which predicates memory per lane without a branch.
constexpr int kBufferFlags = 0x00020000;
constexpr uint32_t kOutOfRange = 0x80000000u;
typedef unsigned int b64_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, kBufferFlags);
}

__device__ __forceinline__ float2 load_f2(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

__device__ __forceinline__ void store_f2(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64_t, v), r, off, 0, 0);
}

// Voxel storage: a (distance, weight) pair as two binary32 (STORAGE 0) or as
// two binary16 rounded to nearest-even (STORAGE 1, IEEE conversion); the
// update arithmetic is binary32 in both cases and binary16 widens exactly.
template <int STORAGE> struct VoxelIO;

template <> struct VoxelIO<0> {
    static constexpr uint32_t kBytes = 8;
    // the value a store followed by a load would give back
    __device__ static __forceinline__ float2 quantize(float2 v) { return v; }
    __device__ static __forceinline__ float2 load(__amdgpu_buffer_rsrc_t r, uint32_t off) { return load_f2(r, off); }
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 v)
    {
        store_f2(r, off, v);
    }
};

template <> struct VoxelIO<1> {
    static constexpr uint32_t kBytes = 4;
    __device__ static __forceinline__ float2 quantize(float2 v)
    {
        return make_float2((float)(_Float16)v.x, (float)(_Float16)v.y);
    }
    __device__ static __forceinline__ float2 load(__amdgpu_buffer_rsrc_t r, uint32_t off)
    {
        const uint32_t bits = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        const _Float16 d = __builtin_bit_cast(_Float16, (unsigned short)(bits & 0xFFFFu));
        const _Float16 w = __builtin_bit_cast(_Float16, (unsigned short)(bits >> 16));
        return make_float2((float)d, (float)w);
    }
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 v)
    {
        const unsigned short d = __builtin_bit_cast(unsigned short, (_Float16)v.x);
        const unsigned short w = __builtin_bit_cast(unsigned short, (_Float16)v.y);
        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)d | ((uint32_t)w << 16), r, off, 0, 0);
    }
};

// Buffer descriptor of one block of the pool.
template <int STORAGE>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const DeviceMap &dm, uint32_t slot)
{
    constexpr uint32_t bytes = kBlockVoxels * VoxelIO<STORAGE>::kBytes;
    return make_rsrc((const char *)dm.pool + (size_t)slot * bytes, bytes);
}

// Hash loads bypass the per-CU cache: other waves of the same launch insert keys.
__device__ __forceinline__ unsigned long long load_key(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_val(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One probe window: lane l < width reads slot (start + base + l) & mask, the
// other lanes hold kNoKey.  The first window of a key covers its 16-slot
// bucket (one key line, one value line), later windows 64 slots each.
struct ProbeWindow {
    unsigned long long k;
    uint32_t v;
};

__device__ __forceinline__ ProbeWindow load_window(const DeviceMap &dm, uint32_t start, uint32_t base, uint32_t width)
{
    ProbeWindow w{kNoKey, kInvalidSlot};
    if ((uint32_t)lane_id() < width) {
        const uint32_t pos = (start + base + (uint32_t)lane_id()) & dm.hash_mask;
        w.k = load_key(&dm.keys[pos]);
        w.v = load_val(&dm.vals[pos]);
    }
    return w;
}

// The first window of a key (its bucket).
__device__ __forceinline__ ProbeWindow load_first_window(const DeviceMap &dm, uint32_t start)
{
    return load_window(dm, start, 0, kBucketSlots);
}

// Pool slot behind a hit found at window position f_hit (waits, bounded, for
// a value that is published after its key), or kInvalidSlot when the key was
// inserted after the pool ran out (its inserter recorded the overflow).
__device__ __forceinline__ uint32_t slot_of_hit(const DeviceMap &dm, uint32_t start, uint32_t base, int f_hit,
                                               uint32_t v)
{
    uint32_t slot = (uint32_t)__shfl((int)v, f_hit);
    if (slot == kInvalidSlot) {
        const uint32_t at = (start + base + (uint32_t)f_hit) & dm.hash_mask;
        if (lane_id() == 0) {
            for (int spin = 0; slot == kInvalidSlot && spin < (1 << 20); ++spin)
                slot = load_val(&dm.vals[at]);
            if (slot == kInvalidSlot)
                atomicOr(&dm.counters[kErrorBits], kErrInsertRace);
        }
        slot = (uint32_t)wave_bcast((int)slot);
    }
    return slot == kNoSlot ? kInvalidSlot : slot;
}

// Read-only lookup of `key` (wave-uniform) starting from its preloaded first
// window: the pool slot, or kInvalidSlot if the key is absent.  Windows are
// scanned in probe order; the first slot holding the key or empty decides.
__device__ inline uint32_t find_block(const DeviceMap &dm, unsigned long long key, uint32_t start, ProbeWindow w)
{
    uint32_t width = kBucketSlots;
    for (uint32_t base = 0; base <= dm.hash_mask; base += width, width = 64) {
        if (base != 0)
            w = load_window(dm, start, base, 64);
        const unsigned long long m_hit = __ballot(w.k == key);
        const unsigned long long m_free = __ballot(w.k == kEmptyKey);
        const int f_hit = m_hit ? __builtin_ctzll(m_hit) : 64;
        const int f_free = m_free ? __builtin_ctzll(m_free) : 64;
        if (f_hit < f_free)
            return (uint32_t)wave_bcast((int)slot_of_hit(dm, start, base, f_hit, w.v));
        if (f_free < 64)
            return kInvalidSlot;
    }
    return kInvalidSlot;
}

// Wave-cooperative find-or-insert of `key` (wave-uniform).  Lanes look at the
// slots of one window at a time, in probe order; the first slot that holds
// the key or is empty decides.  w is the key's first window, loaded ahead of
// time.  An insert claims the empty slot for the key first and only then
// reserves a pool slot, so waves racing on one key take exactly one pool
// slot between them; the losers find the key and wait for its published
// value.  Returns the pool slot, or kInvalidSlot after recording an overflow.
__device__ inline uint32_t find_or_insert(const DeviceMap &dm, unsigned long long key, uint32_t start, ProbeWindow w)
{
    const int lane = lane_id();
    const uint32_t mask = dm.hash_mask;
    uint32_t base = 0, width = kBucketSlots;
    bool loaded = true;
    while (base <= mask) {
        if (!loaded)
            w = load_window(dm, start, base, width);
        loaded = false;
        const unsigned long long m_hit = __ballot(w.k == key);
        const unsigned long long m_free = __ballot(w.k == kEmptyKey);
        const int f_hit = m_hit ? __builtin_ctzll(m_hit) : 64;
        const int f_free = m_free ? __builtin_ctzll(m_free) : 64;
        if (f_hit < f_free)
            return (uint32_t)wave_bcast((int)slot_of_hit(dm, start, base, f_hit, w.v));
        if (f_free == 64) {
            base += width;
            width = 64;
            continue;
        }
        const uint32_t at = (start + base + (uint32_t)f_free) & mask;
        uint32_t got = kInvalidSlot;   // lane 0: the value it published for `at`
        if (lane == 0 && atomicCAS(&dm.keys[at], kEmptyKey, key) == kEmptyKey) {
            got = atomicAdd(&dm.counters[kNumBlocks], 1u);
            if (got < dm.block_cap) {
                dm.slot_keys[got] = key;
            } else {
                atomicOr(&dm.counters[kErrorBits], kErrPoolFull);
                got = kNoSlot;   // waiters on this key stop waiting and skip it
            }
            __hip_atomic_store(&dm.vals[at], got, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        got = (uint32_t)wave_bcast((int)got);
        if (got != kInvalidSlot)
            return got == kNoSlot ? kInvalidSlot : got;
        // the slot went to another key (or to this key from elsewhere): reload this window
    }
    if (lane == 0)
        atomicOr(&dm.counters[kErrorBits], kErrHashFull);
    return kInvalidSlot;
}

// Lane-level culling of one block against a pinhole view.  Each frustum plane
// is a linear function f of the camera-frame point; over the block (a box
// with corner p0 and edges E R[:,k] in camera coordinates) its maximum is
// f(p0) + sum_k max(0, f(E R[:,k])).  The block is dropped when that maximum is
// below -margin for some plane; the margin exceeds the binary32 error of any
// voxel's projection, so no block holding an updated voxel is ever dropped.
__device__ __forceinline__ bool lane_block_in_pinhole(const CameraView &cv, const MapConsts &mc, int bx, int by,
                                                      int bz)
{
    const float e = 8.0f * mc.vs;
    const float X = (float)(8 * bx) * mc.vs, Y = (float)(8 * by) * mc.vs, Z = (float)(8 * bz) * mc.vs;
    const float x0 = cv.R[0] * X + cv.R[1] * Y + cv.R[2] * Z + cv.t[0];
    const float y0 = cv.R[3] * X + cv.R[4] * Y + cv.R[5] * Z + cv.t[1];
    const float z0 = cv.R[6] * X + cv.R[7] * Y + cv.R[8] * Z + cv.t[2];
    float ex[3], ey[3], ez[3];   // camera-frame edge vectors of the block
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ex[k] = e * cv.R[k];
        ey[k] = e * cv.R[3 + k];
        ez[k] = e * cv.R[6 + k];
    }
    auto box_max = [&](float a, float b, float c, float d) {   // max of a x + b y + c z + d
        float m = a * x0 + b * y0 + c * z0 + d;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            m += fmaxf(0.0f, a * ex[k] + b * ey[k] + c * ez[k]);
        return m;
    };
    if (box_max(cv.fx, 0.0f, cv.cx, 0.0f) < -cv.margin_u)                        // u >= 0
        return false;
    if (box_max(-cv.fx, 0.0f, cv.width_f - cv.cx, 0.0f) < -cv.margin_u)          // u <= W
        return false;
    if (box_max(0.0f, cv.fy, cv.cy, 0.0f) < -cv.margin_v)                        // v >= 0
        return false;
    if (box_max(0.0f, -cv.fy, cv.height_f - cv.cy, 0.0f) < -cv.margin_v)         // v <= H
        return false;
    if (box_max(0.0f, 0.0f, 1.0f, 0.0f) < -mc.margin_z)                          // z > 0
        return false;
    if (box_max(0.0f, 0.0f, -1.0f, cv.zfar) < -mc.margin_z)                      // z <= zfar
        return false;
    return true;
}

// Lane-level culling of one block against a spherical view.  Dropped when
// the block's closest point is farther than the largest usable range, or when
// all 8 corners lie strictly inside the cone above the polar band (or below
// it): z - |p| cos(phi_start) and -z + |p| cos(phi_end) are concave, so their
// minimum over the box is at a corner.
__device__ __forceinline__ bool lane_block_in_spherical(const CameraView &cv, const MapConsts &mc, int bx, int by,
                                                        int bz)
{
    const float e = 8.0f * mc.vs;
    const float lo[3] = {(float)(8 * bx) * mc.vs, (float)(8 * by) * mc.vs, (float)(8 * bz) * mc.vs};
    float d2 = 0.0f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float below = lo[a] - cv.origin[a];
        const float above = cv.origin[a] - (lo[a] + e);
        const float g = fmaxf(0.0f, fmaxf(below, above));
        d2 += g * g;
    }
    const float reach = cv.zfar + mc.margin_z;
    if (d2 > reach * reach)
        return false;
    float min_up = 3.0e38f, min_down = 3.0e38f;
    for (int c = 0; c < 8; ++c) {
        const float X = lo[0] + ((c & 1) ? e : 0.0f), Y = lo[1] + ((c & 2) ? e : 0.0f),
                    Z = lo[2] + ((c & 4) ? e : 0.0f);
        const float x = cv.R[0] * X + cv.R[1] * Y + cv.R[2] * Z + cv.t[0];
        const float y = cv.R[3] * X + cv.R[4] * Y + cv.R[5] * Z + cv.t[1];
        const float z = cv.R[6] * X + cv.R[7] * Y + cv.R[8] * Z + cv.t[2];
        const float r = sqrtf(x * x + y * y + z * z);
        min_up = fminf(min_up, z - r * cv.cos_pol_start);
        min_down = fminf(min_down, -z + r * cv.cos_pol_end);
    }
    if (cv.cos_pol_start > 0.0f && min_up > mc.margin_z)
        return false;
    if (cv.cos_pol_end < 0.0f && min_down > mc.margin_z)
        return false;
    return true;
}


// atan on [0, 1]: the polynomial of Abramowitz & Stegun, Handbook of
// Mathematical Functions, formula 4.4.49 (|error| <= 2e-8), Horner's rule in
// binary32; atan2 by octant reduction, (0, 0) -> 0.  The CPU oracle evaluates
// the same operations, so column and row decisions agree bit for bit.
__device__ __forceinline__ float atan_unit(float t)
{
    const float t2 = t * t;
    float p = 0.0028662257f;
    p = p * t2 + -0.0161657367f;
    p = p * t2 + 0.0429096138f;
    p = p * t2 + -0.0752896400f;
    p = p * t2 + 0.1065626393f;
    p = p * t2 + -0.1420889944f;
    p = p * t2 + 0.1999355085f;
    p = p * t2 + -0.3333314528f;
    p = p * t2 + 1.0f;
    return p * t;
}

__device__ __forceinline__ float atan2_as(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const bool swap = ay > ax;
    // one division: selecting between two quotients would compute both
    const float t = (swap ? ax : ay) / (swap ? ay : ax);
    float a = atan_unit(t);
    if (swap)
        a = 1.57079637f - a;
    if (x < 0.0f)
        a = 3.14159274f - a;
    a = y < 0.0f ? -a : a;
    return (ax == 0.0f && ay == 0.0f) ? 0.0f : a;
}

// Largest valid measurement over the pixel rectangle [i0, i1] x [j0, j1]
// (inside the image) from the view's footprint pyramid, at the finest level
// where the rectangle spans at most 3 x 3 tiles; `ok` is false when even the
// coarsest level needs more.
__device__ __forceinline__ float footprint_max(const CameraView &cv, int i0, int i1, int j0, int j1, bool &ok)
{
    int l = 0;
    while (l < kTileLevels - 1 && (((i1 >> (kTileBaseShift + l)) - (i0 >> (kTileBaseShift + l))) > 2 ||
                                   ((j1 >> (kTileBaseShift + l)) - (j0 >> (kTileBaseShift + l))) > 2))
        ++l;
    const int sh = kTileBaseShift + l;
    const int a0 = i0 >> sh, a1 = i1 >> sh, b0 = j0 >> sh, b1 = j1 >> sh;
    ok = a1 - a0 <= 2 && b1 - b0 <= 2;
    const int off = l == 0 ? cv.tile_off[0] : l == 1 ? cv.tile_off[1] : l == 2 ? cv.tile_off[2] : cv.tile_off[3];
    const int cols = l == 0 ? cv.tile_cols[0] : l == 1 ? cv.tile_cols[1] : l == 2 ? cv.tile_cols[2] : cv.tile_cols[3];
    const float *T = cv.tiles + off;
    float m = 0.0f;
    if (ok) {
        // a fixed 3 x 3 window, repeated indices clamped into [a0, a1] x [b0, b1]
#pragma unroll
        for (int db = 0; db < 3; ++db) {
            const int b = min(b0 + db, b1);
#pragma unroll
            for (int da = 0; da < 3; ++da)
                m = fmaxf(m, T[b * cols + min(a0 + da, a1)]);
        }
    }
    return m;
}

// Footprint culling against a pinhole view.  The voxels of a block project
// inside the rectangle of its 8 projected corners (the projection of a box in
// front of the camera is the convex hull of its corners' projections) and
// have depth at least the corners' minimum z.  An updated voxel has z <= d + eps
// for the valid measurement d of its pixel, so the block is dropped when its
// minimum z exceeds the footprint's largest measurement + eps (+ the rounding
// slack margin_z).  Corners are projected with a fast reciprocal and the
// rectangle is widened by 2 pixels, far beyond the binary32 error of either
// projection.  Blocks reaching within 1 mm of the camera plane are kept.
__device__ __forceinline__ bool lane_block_footprint_pinhole(const CameraView &cv, const MapConsts &mc, int bx,
                                                             int by, int bz)
{
    const float e = 8.0f * mc.vs;
    const float X = (float)(8 * bx) * mc.vs, Y = (float)(8 * by) * mc.vs, Z = (float)(8 * bz) * mc.vs;
    float zmin = 3.0e38f, umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float px = X + ((c & 1) ? e : 0.0f), py = Y + ((c & 2) ? e : 0.0f), pz = Z + ((c & 4) ? e : 0.0f);
        const float x = cv.R[0] * px + cv.R[1] * py + cv.R[2] * pz + cv.t[0];
        const float y = cv.R[3] * px + cv.R[4] * py + cv.R[5] * pz + cv.t[1];
        const float z = cv.R[6] * px + cv.R[7] * py + cv.R[8] * pz + cv.t[2];
        const float r = __builtin_amdgcn_rcpf(fmaxf(z, 1e-3f));
        const float u = cv.fx * (x * r) + cv.cx;
        const float v = cv.fy * (y * r) + cv.cy;
        zmin = fminf(zmin, z);
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        vmin = fminf(vmin, v);
        vmax = fmaxf(vmax, v);
    }
    if (!(zmin > 1e-3f))
        return true;
    const float lo_u = fmaxf(umin - 2.0f, 0.0f), hi_u = fminf(umax + 2.0f, cv.width_f - 1.0f);
    const float lo_v = fmaxf(vmin - 2.0f, 0.0f), hi_v = fminf(vmax + 2.0f, cv.height_f - 1.0f);
    if (hi_u < lo_u || hi_v < lo_v)
        return false;
    bool ok;
    const float dm = footprint_max(cv, (int)lo_u, (int)hi_u, (int)lo_v, (int)hi_v, ok);
    return !ok || zmin <= dm + mc.eps + mc.margin_z;
}

// Footprint culling against a spherical view.  Every voxel centre lies in
// the block's bounding sphere (centre c, radius rho), so its range is at least
// |c| - rho and its azimuth and polar angle lie within the half-angle
// asin(rho / distance) of the sphere's (taken about the z axis for the
// azimuth); the columns and rows it interpolates from follow, with one of
// slack on each side.  The block is dropped when |c| - rho exceeds the
// largest valid range over those pixels + eps.  Blocks whose sphere nearly
// reaches the sensor are kept; so are those nearly reaching the z axis (all
// azimuths), and, for a partial-circle sensor, those straddling azimuth +-pi.
__device__ __forceinline__ bool lane_block_footprint_spherical(const CameraView &cv, const MapConsts &mc, int bx,
                                                               int by, int bz)
{
    const float e = 8.0f * mc.vs;
    const float X = ((float)(8 * bx) + 4.0f) * mc.vs, Y = ((float)(8 * by) + 4.0f) * mc.vs,
                Z = ((float)(8 * bz) + 4.0f) * mc.vs;
    const float x = cv.R[0] * X + cv.R[1] * Y + cv.R[2] * Z + cv.t[0];
    const float y = cv.R[3] * X + cv.R[4] * Y + cv.R[5] * Z + cv.t[1];
    const float z = cv.R[6] * X + cv.R[7] * Y + cv.R[8] * Z + cv.t[2];
    const float rad = 0.866026f * e * 1.001f + mc.margin_z;
    const float R2 = x * x + y * y + z * z;
    const float Rc = sqrtf(R2);
    if (!(Rc > 1.05f * rad + 1e-3f))
        return true;
    // rows
    const float phi_c = atan2_as(sqrtf(x * x + y * y), z);
    const float hp = atan2_as(rad, sqrtf(R2 - rad * rad));
    const float v_lo = (phi_c - hp - cv.pol_start) * cv.beta, v_hi = (phi_c + hp - cv.pol_start) * cv.beta;
    const float r_lo = fmaxf(floorf(v_lo - 0.5f) - 1.0f, 0.0f);
    const float r_hi = fminf(floorf(v_hi - 0.5f) + 2.0f, cv.height_f - 1.0f);
    if (r_hi < r_lo)
        return false;
    const int j0 = (int)r_lo, j1 = (int)r_hi;
    // columns
    const float rho2 = x * x + y * y;
    if (!(sqrtf(rho2) > 1.05f * rad + 1e-3f))
        return true;
    const float theta_c = atan2_as(y, x);
    const float ha = atan2_as(rad, sqrtf(rho2 - rad * rad));
    const float W = cv.width_f;
    float c_lo = floorf((theta_c - ha - cv.az_start) * cv.alpha - 0.5f) - 1.0f;
    float c_hi = floorf((theta_c + ha - cv.az_start) * cv.alpha - 0.5f) + 2.0f;
    float dm;
    bool ok = true;
    if (cv.full_circle) {
        if (c_hi - c_lo + 1.0f >= W)
            return true;
        // columns wrap modulo W: shift c_lo into [0, W); c_hi < c_lo + W - 1
        const float k = floorf(c_lo / W);
        c_lo = fminf(fmaxf(c_lo - k * W, 0.0f), W - 1.0f);
        c_hi = c_hi - k * W;
        if (c_hi >= W) {
            // [c_lo, W - 1] and [0, c_hi - W]
            bool ok2;
            dm = fmaxf(footprint_max(cv, (int)c_lo, cv.width - 1, j0, j1, ok),
                       footprint_max(cv, 0, (int)fminf(c_hi - W, W - 1.0f), j0, j1, ok2));
            ok = ok && ok2;
        } else {
            if (!(c_hi >= c_lo))
                return true;
            dm = footprint_max(cv, (int)c_lo, (int)c_hi, j0, j1, ok);
        }
    } else {
        if (theta_c - ha < -3.14159265f || theta_c + ha > 3.14159265f)
            return true;
        c_lo = fmaxf(c_lo, 0.0f);
        c_hi = fminf(c_hi, W - 1.0f);
        if (c_hi < c_lo)
            return false;
        dm = footprint_max(cv, (int)c_lo, (int)c_hi, j0, j1, ok);
    }
    return !ok || Rc - rad <= dm + mc.eps + mc.margin_z;
}

// Culling of block (bx, by, bz) against one view: false only when no voxel
// of the block can be updated.  PINHOLE: the view is known to be a pinhole
// camera (single-view pinhole launches compile no spherical test).
template <bool PINHOLE = false>
__device__ __forceinline__ bool lane_block_in_view(const CameraView &cv, const MapConsts &mc, int bx, int by, int bz)
{
    if (!PINHOLE && cv.model == kModelSpherical) {
        if (!lane_block_in_spherical(cv, mc, bx, by, bz))
            return false;
        return !cv.tiles || lane_block_footprint_spherical(cv, mc, bx, by, bz);
    }
    if (!lane_block_in_pinhole(cv, mc, bx, by, bz))
        return false;
    return !cv.tiles || lane_block_footprint_pinhole(cv, mc, bx, by, bz);
}

// Ownership band of a block (one per XCD): the image-column band of the
// block centre in the first view that sees the centre; the lattice index
// otherwise.  Every wave computes the same band for a block, so exactly one
// partition processes it, and a partition's waves touch about 1/kPartitions of
// each image.
__device__ __forceinline__ int block_band(const CameraView *cams, int n_views, const MapConsts &mc, int bx, int by,
                                          int bz, uint32_t lb)
{
    const float X = ((float)(8 * bx) + 4.0f) * mc.vs, Y = ((float)(8 * by) + 4.0f) * mc.vs,
                Z = ((float)(8 * bz) + 4.0f) * mc.vs;
    for (int v = 0; v < n_views; ++v) {
        const CameraView &cv = cams[v];
        const float x = cv.R[0] * X + cv.R[1] * Y + cv.R[2] * Z + cv.t[0];
        const float y = cv.R[3] * X + cv.R[4] * Y + cv.R[5] * Z + cv.t[1];
        const float z = cv.R[6] * X + cv.R[7] * Y + cv.R[8] * Z + cv.t[2];
        if (cv.model == kModelSpherical) {
            const float u = (atan2_as(y, x) - cv.az_start) * cv.alpha;
            if (u >= 0.0f && u < cv.width_f)
                return min((int)(u * (float)kPartitions / cv.width_f), kPartitions - 1);
            continue;
        }
        if (!(z > 0.0f))
            continue;
        const float u = cv.fx * (x / z) + cv.cx;
        const float w = cv.fy * (y / z) + cv.cy;
        if (u >= 0.0f && u < cv.width_f && w >= 0.0f && w < cv.height_f)
            return min((int)(u * (float)kPartitions / cv.width_f), kPartitions - 1);
    }
    return (int)(lb % (uint32_t)kPartitions);
}

// Position of workgroup g among the `groups` of a launch in the order that
// consecutive work items are dealt out (item k of a pass goes to the group at
// position k).  Workgroups are dispatched to the 8 XCDs round-robin (group g
// runs on XCD g mod 8), so the order lists XCD 0's groups first, then XCD
// 1's, and so on: consecutive items land on different CUs of one XCD.
__device__ __forceinline__ uint32_t spread_position(uint32_t g, uint32_t groups)
{
    if (groups % (uint32_t)kXcds != 0u)
        return g;
    return (g % (uint32_t)kXcds) * (groups / (uint32_t)kXcds) + g / (uint32_t)kXcds;
}

// Block indices of lattice entry lb (x fastest), with the lattice's
// multiply-shift divisors in place of two integer divisions.
__device__ __forceinline__ uint32_t lattice_div(uint32_t n, uint32_t m, int s)
{
    return (uint32_t)(((unsigned long long)n * (unsigned long long)m) >> s);
}
__device__ __forceinline__ void lattice_block(const Lattice &lat, uint32_t lb, int &bx, int &by, int &bz)
{
    const uint32_t rest = lattice_div(lb, lat.div_m[0], lat.div_s[0]);
    const uint32_t z = lattice_div(rest, lat.div_m[1], lat.div_s[1]);
    bx = lat.lat_min[0] + (int)(lb - rest * (uint32_t)lat.lat_dim[0]);
    by = lat.lat_min[1] + (int)(rest - z * (uint32_t)lat.lat_dim[1]);
    bz = lat.lat_min[2] + (int)z;
}

// Culling of block b against a single pinhole view with the host's
// precomputed planes (PinholeCull): the same tests as lane_block_in_pinhole
// and lane_block_footprint_pinhole, evaluated in lattice-relative
// coordinates with fused multiply-adds; the margins are those of the
// CameraView tests, far above the binary32 error of either evaluation.
__device__ __forceinline__ bool lane_block_pinhole_precomputed(const PinholeCull &pc, const CameraView &cv,
                                                               const MapConsts &mc, const Lattice &lat, int bx,
                                                               int by, int bz)
{
    const float lx = (float)(bx - lat.lat_min[0]), ly = (float)(by - lat.lat_min[1]), lz = (float)(bz - lat.lat_min[2]);
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (fmaf(pc.plane[4 * q], lx, fmaf(pc.plane[4 * q + 1], ly, fmaf(pc.plane[4 * q + 2], lz, pc.plane[4 * q + 3]))) <
            0.0f)
            return false;
    if (!cv.tiles)
        return true;
    float cx0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        cx0[a] = fmaf(pc.cam[4 * a], lx, fmaf(pc.cam[4 * a + 1], ly, fmaf(pc.cam[4 * a + 2], lz, pc.cam[4 * a + 3])));
    float zmin = 3.0e38f, umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float p[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a] = cx0[a];
            if (c & 1)
                p[a] += pc.cam[4 * a];
            if (c & 2)
                p[a] += pc.cam[4 * a + 1];
            if (c & 4)
                p[a] += pc.cam[4 * a + 2];
        }
        const float r = __builtin_amdgcn_rcpf(fmaxf(p[2], 1e-3f));
        const float u = fmaf(cv.fx, p[0] * r, cv.cx);
        const float v = fmaf(cv.fy, p[1] * r, cv.cy);
        zmin = fminf(zmin, p[2]);
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        vmin = fminf(vmin, v);
        vmax = fmaxf(vmax, v);
    }
    if (!(zmin > 1e-3f))
        return true;
    const float lo_u = fmaxf(umin - 2.0f, 0.0f), hi_u = fminf(umax + 2.0f, cv.width_f - 1.0f);
    const float lo_v = fmaxf(vmin - 2.0f, 0.0f), hi_v = fminf(vmax + 2.0f, cv.height_f - 1.0f);
    if (hi_u < lo_u || hi_v < lo_v)
        return false;
    bool ok;
    const float dm = footprint_max(cv, (int)lo_u, (int)hi_u, (int)lo_v, (int)hi_v, ok);
    return !ok || zmin <= dm + mc.eps + mc.margin_z;
}

// Lattice block lb of the launch: its block indices and the views whose
// culling it survives (bit v), or, with ray-walk marks, 1 when the walk
// marked it (the mark is cleared for the next frame: each entry is read by
// exactly one thread).
template <bool PINHOLE>
__device__ __forceinline__ uint32_t lattice_candidate(const Lattice &lat, const CameraView *cams, int n_views,
                                                      const MapConsts &mc, uint32_t lb, int &bx, int &by, int &bz,
                                                      const PinholeCull *pc)
{
    lattice_block(lat, lb, bx, by, bz);
    uint32_t vmask = 0;
    if (cams[0].dda_marks) {
        vmask = cams[0].dda_marks[lb] ? 1u : 0u;
        if (vmask)
            cams[0].dda_marks[lb] = 0;
    } else if (pc) {
        vmask = lane_block_pinhole_precomputed(*pc, cams[0], mc, lat, bx, by, bz) ? 1u : 0u;
    } else {
        for (int v = 0; v < n_views; ++v)
            if (lane_block_in_view<PINHOLE>(cams[v], mc, bx, by, bz))
                vmask |= 1u << v;
    }
    return vmask;
}

// Walk of a launch's lattice compacted per workgroup (one band): each pass
// gives every thread of the grid one lattice block, the blocks of a
// workgroup strided across the whole lattice (block lb goes to the workgroup
// at position lb mod groups, in the XCD-aware order of spread_position), so
// that every workgroup draws about the same number of surviving blocks from
// anywhere in the frame; a workgroup collects its survivors in LDS and its
// waves take them in turn, so no wave handles more than its share.
template <bool PINHOLE, class Body>
__device__ __forceinline__ void scan_lattice_group(const Lattice &lat, const CameraView *cams, int n_views,
                                                   const MapConsts &mc, Body &&body, const PinholeCull *pc)
{
    constexpr uint32_t kThreads = 64u * (uint32_t)kWavesPerGroup;
    __shared__ uint32_t s_lb[kThreads], s_vm[kThreads];
    __shared__ uint32_t s_count[kWavesPerGroup];
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const uint32_t groups = gridDim.x;
    const uint32_t pos = spread_position(blockIdx.x, groups);
    const uint32_t n_lat = (uint32_t)lat.n_lat;
    const unsigned long long per_pass = (unsigned long long)groups * kThreads;
    // the loop runs the same number of times in every thread of the workgroup
    for (unsigned long long base = 0; base < n_lat; base += per_pass) {
        const unsigned long long item = base + (unsigned long long)threadIdx.x * groups + pos;
        uint32_t vmask = 0;
        int bx = 0, by = 0, bz = 0;
        if (item < n_lat)
            vmask = lattice_candidate<PINHOLE>(lat, cams, n_views, mc, (uint32_t)item, bx, by, bz, pc);
        const unsigned long long keep = __ballot(vmask != 0);
        if (lane == 0)
            s_count[wave] = (uint32_t)__popcll(keep);
        __syncthreads();
        uint32_t at = 0, total = 0;
        for (int k = 0; k < kWavesPerGroup; ++k) {
            at += k < wave ? s_count[k] : 0u;
            total += s_count[k];
        }
        if (vmask != 0) {
            const uint32_t i = at + (uint32_t)__popcll(keep & ((1ull << lane) - 1ull));
            s_lb[i] = (uint32_t)item;
            s_vm[i] = vmask;
        }
        __syncthreads();
        for (uint32_t i = (uint32_t)wave; i < total; i += (uint32_t)kWavesPerGroup) {
            const uint32_t lb = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_lb[i]);
            const uint32_t svm = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_vm[i]);
            int sbx, sby, sbz;
            lattice_block(lat, lb, sbx, sby, sbz);
            body(sbx, sby, sbz, svm);
        }
        __syncthreads();   // s_lb, s_vm and s_count are rewritten by the next pass
    }
}

// Walks the launch's lattice for this wave.  With P = lat.partitions bands,
// the partition of the workgroup (blockIdx.x mod P, the XCD it runs on when
// P = 8) scans all chunks; each lane bands and culls one block of a chunk of
// lat.chunk consecutive lattice blocks, and the surviving blocks of this
// partition are handed to body(bx, by, bz, view_mask) one at a time
// (wave-uniform).  Waves never wait for each other.  With ray-walk marks, a
// lattice block is a candidate exactly when marked.  lat.group_scan selects
// the workgroup-compacted walk (scan_lattice_group).  pc: the host's plane
// table for a single pinhole view, or null for the CameraView tests.
template <bool PINHOLE = false, class Body>
__device__ __forceinline__ void scan_lattice(const Lattice &lat, const CameraView *cams, int n_views,
                                             const MapConsts &mc, Body &&body, const PinholeCull *pc = nullptr)
{
    if (lat.group_scan) {
        scan_lattice_group<PINHOLE>(lat, cams, n_views, mc, body, pc);
        return;
    }
    const int lane = lane_id();
    const uint32_t P = (uint32_t)lat.partitions;
    const int part = (int)(blockIdx.x % P);
    // consecutive chunks go to different workgroups: neighbouring lattice
    // blocks survive culling together, and spread this way their waves share
    // no SIMD.  The order is XCD-aware (spread_position): a run of consecutive
    // chunks stays on one XCD, whose L2 then serves their shared depth pixels
    const uint32_t groups_pp = gridDim.x / P;
    const uint32_t waves_pp = groups_pp * (uint32_t)kWavesPerGroup;
    const uint32_t wave_pp = (threadIdx.x >> 6) * groups_pp + spread_position(blockIdx.x / P, groups_pp);
    const uint32_t chunk = (uint32_t)lat.chunk;
    const uint32_t n_lat = (uint32_t)lat.n_lat;
    const uint32_t n_chunks = (n_lat + chunk - 1) / chunk;
    for (uint32_t c = wave_pp; c < n_chunks; c += waves_pp) {
        const uint32_t lb = c * chunk + (uint32_t)lane;
        uint32_t vmask = 0;
        int bx = 0, by = 0, bz = 0;
        if ((uint32_t)lane < chunk && lb < n_lat) {
            lattice_block(lat, lb, bx, by, bz);
            if (cams[0].dda_marks) {
                // ray-walk allocation: the walk decides; the mark is cleared
                // for the next frame (each entry is read by one lane only)
                vmask = cams[0].dda_marks[lb] ? 1u : 0u;
                if (vmask)
                    cams[0].dda_marks[lb] = 0;
            }
            else if (P == 1 || block_band(cams, n_views, mc, bx, by, bz, lb) == part) {
                if (pc)
                    vmask = lane_block_pinhole_precomputed(*pc, cams[0], mc, lat, bx, by, bz) ? 1u : 0u;
                else
                    for (int v = 0; v < n_views; ++v)
                        if (lane_block_in_view<PINHOLE>(cams[v], mc, bx, by, bz))
                            vmask |= 1u << v;
            }
        }
        unsigned long long todo = __ballot(vmask != 0);
        while (todo) {
            const int src = __builtin_ctzll(todo);
            todo &= todo - 1;
            const int sbx = __builtin_amdgcn_readlane(bx, src);
            const int sby = __builtin_amdgcn_readlane(by, src);
            const int sbz = __builtin_amdgcn_readlane(bz, src);
            const uint32_t svm = (uint32_t)__builtin_amdgcn_readlane((int)vmask, src);
            body(sbx, sby, sbz, svm);
        }
    }
}

// Eq. (1)-(2) and the TSDF measurement (§IV-B) of the lane's 8 voxels
// (column (px, py), z-slabs of block row bz) against one pinhole view.
// Returns the hit mask (bit s: voxel of slab s is updated) with the truncated
// distance xs[s] and weight ws[s].  The 8 depth gathers are issued together;
// a voxel outside the image reads through an out-of-range offset (value 0,
// an invalid depth).
template <int WEIGHTING>
__device__ __forceinline__ uint32_t measure_pinhole(const CameraView &cv, const MapConsts &mc, float px, float py,
                                                    int bz, float xs[8], float ws[8])
{
    const uint32_t width = (uint32_t)cv.width;
    const __amdgpu_buffer_rsrc_t depth = make_rsrc(cv.depth, 4u * width * (uint32_t)cv.height);
    // p_C = ((R0 px + R1 py) + R2 pz) + t; the first sum is shared by the column
    const float ax = cv.R[0] * px + cv.R[1] * py;
    const float ay = cv.R[3] * px + cv.R[4] * py;
    const float az = cv.R[6] * px + cv.R[7] * py;
    float zc[8];
    uint32_t pix_off[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const float pz = ((float)(8 * bz + s) + 0.5f) * mc.vs;
        const float xc = (ax + cv.R[2] * pz) + cv.t[0];
        const float yc = (ay + cv.R[5] * pz) + cv.t[1];
        zc[s] = (az + cv.R[8] * pz) + cv.t[2];
        const float r = 1.0f / zc[s];
        const float u = cv.fx * (xc * r) + cv.cx;
        const float v = cv.fy * (yc * r) + cv.cy;
        // nearest pixel: (i, j) covers [i, i+1) x [j, j+1)
        const bool ok = zc[s] > 0.0f && u >= 0.0f && u < cv.width_f && v >= 0.0f && v < cv.height_f;
        const uint32_t i = (uint32_t)(ok ? u : 0.0f);
        const uint32_t j = (uint32_t)(ok ? v : 0.0f);
        pix_off[s] = ok ? 4u * (j * width + i) : kOutOfRange;
    }
    float d[8];
#pragma unroll
    for (int s = 0; s < 8; ++s)
        d[s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(depth, pix_off[s], 0, 0));
    uint32_t hit = 0;
    if constexpr (WEIGHTING == kWeightLearned) {
        // learned sensor model: the pixel's own (weight, truncation) pair
        const __amdgpu_buffer_rsrc_t maps = make_rsrc(cv.sm_maps, 8u * width * (uint32_t)cv.height);
        float2 we[8];
#pragma unroll
        for (int s = 0; s < 8; ++s)
            we[s] = load_f2(maps, pix_off[s] == kOutOfRange ? kOutOfRange : 2u * pix_off[s]);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const float dp = d[s] - zc[s];
            const float e = we[s].y;
            const bool upd = d[s] > 0.0f && d[s] <= cv.d_max && dp >= -e && we[s].x > 0.0f;
            xs[s] = dp < e ? dp : e;
            ws[s] = we[s].x;
            hit |= (upd ? 1u : 0u) << s;
        }
        return hit;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        // valid measurement, truncation band (skip below -eps), weight > 0
        const float dp = d[s] - zc[s];
        float wm = 1.0f;
        if (WEIGHTING == 1 && dp < -mc.delta)
            wm = (mc.eps + dp) * mc.span_inv;
        const bool upd = d[s] > 0.0f && d[s] <= cv.d_max && dp >= -mc.eps && wm > 0.0f;
        xs[s] = dp < mc.eps ? dp : mc.eps;
        ws[s] = wm;
        hit |= (upd ? 1u : 0u) << s;
    }
    return hit;
}

// LDS staging of a block's depth footprint.  The voxel centres of a block in
// front of the camera project inside the rectangle of its 8 projected corners
// (the projection of a box is the hull of its corners' projections); widened
// by one pixel and clipped to the image, that rectangle is copied into the
// wave's LDS region with row-contiguous loads when it holds at most
// kStagePixels pixels, and each voxel then reads its nearest pixel there.  A
// voxel whose pixel lies outside the rectangle (only through rounding at its
// edge) reads the image directly, so every voxel sees exactly the value a
// direct read gives.
constexpr int kStagePixels = 1024;   // 4 KiB of LDS per wave

struct StageRect {
    int u0, v0, w, h;   // w * h == 0: not staged
};

// Footprint rectangle of block (bx, by, bz) (wave-uniform): lane c computes
// corner c & 7 and the extremes are reduced over each group of 8 lanes.
__device__ __forceinline__ StageRect stage_rect(const CameraView &cv, const MapConsts &mc, int bx, int by, int bz)
{
    const int c = lane_id() & 7;
    const float e = 8.0f * mc.vs;
    const float px = (float)(8 * bx) * mc.vs + ((c & 1) ? e : 0.0f);
    const float py = (float)(8 * by) * mc.vs + ((c & 2) ? e : 0.0f);
    const float pz = (float)(8 * bz) * mc.vs + ((c & 4) ? e : 0.0f);
    const float x = cv.R[0] * px + cv.R[1] * py + cv.R[2] * pz + cv.t[0];
    const float y = cv.R[3] * px + cv.R[4] * py + cv.R[5] * pz + cv.t[1];
    float z = cv.R[6] * px + cv.R[7] * py + cv.R[8] * pz + cv.t[2];
    float u = cv.fx * (x / z) + cv.cx;
    float v = cv.fy * (y / z) + cv.cy;
    float umax = u, vmax = v;
#pragma unroll
    for (int m = 1; m < 8; m <<= 1) {
        z = fminf(z, __shfl_xor(z, m));
        u = fminf(u, __shfl_xor(u, m));
        v = fminf(v, __shfl_xor(v, m));
        umax = fmaxf(umax, __shfl_xor(umax, m));
        vmax = fmaxf(vmax, __shfl_xor(vmax, m));
    }
    StageRect r{0, 0, 0, 0};
    auto uniform = [](float f) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, f)));
    };
    if (!(uniform(z) > 1e-3f))
        return r;
    const float lo_u = fmaxf(floorf(uniform(u)) - 1.0f, 0.0f);
    const float lo_v = fmaxf(floorf(uniform(v)) - 1.0f, 0.0f);
    const float hi_u = fminf(floorf(uniform(umax)) + 1.0f, cv.width_f - 1.0f);
    const float hi_v = fminf(floorf(uniform(vmax)) + 1.0f, cv.height_f - 1.0f);
    // NaN or an empty rectangle fails these tests
    if (!(hi_u >= lo_u && hi_v >= lo_v))
        return r;
    const float area = (hi_u - lo_u + 1.0f) * (hi_v - lo_v + 1.0f);
    if (!(area <= (float)kStagePixels))
        return r;
    r.u0 = (int)lo_u;
    r.v0 = (int)lo_v;
    r.w = (int)(hi_u - lo_u) + 1;
    r.h = (int)(hi_v - lo_v) + 1;
    return r;
}

// Copies the rectangle into `region` (row-major, r.w floats a row): a pass
// of the wave loads 64 / w rows at once when a row fits the wave (lane ->
// (row, column) by one division per block), one row-chunk at a time
// otherwise.  All of a pass's loads are issued before its LDS writes.
__device__ __forceinline__ void stage_copy(const CameraView &cv, const StageRect &r, float *region)
{
    const int lane = lane_id();
    const __amdgpu_buffer_rsrc_t depth = make_rsrc(cv.depth, 4u * (uint32_t)cv.width * (uint32_t)cv.height);
    if (r.w <= 64) {
        const int rows = 64 / r.w;                 // rows per pass
        const int q = lane / r.w, col = lane - q * r.w;
        const bool active = q < rows;
        for (int base = 0; base < r.h; base += 4 * rows) {
            float val[4];
            int at[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = base + t * rows + q;
                const bool ok = active && row < r.h;
                at[t] = ok ? row * r.w + col : -1;
                const uint32_t off = ok ? 4u * ((uint32_t)(r.v0 + row) * (uint32_t)cv.width + (uint32_t)(r.u0 + col))
                                        : kOutOfRange;
                val[t] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(depth, off, 0, 0));
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (at[t] >= 0)
                    region[at[t]] = val[t];
        }
    } else {
        for (int row = 0; row < r.h; ++row)
            for (int col = lane; col < r.w; col += 64)
                region[row * r.w + col] = __builtin_bit_cast(
                    float, __builtin_amdgcn_raw_buffer_load_b32(
                               depth, 4u * ((uint32_t)(r.v0 + row) * (uint32_t)cv.width + (uint32_t)(r.u0 + col)), 0,
                               0));
    }
    // the wave's own writes are read back by other lanes of the same wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// measure_pinhole (constant or linear-dropoff weighting) with the depth
// footprint staged in `region` when the block's rectangle is small enough.
template <int WEIGHTING>
__device__ __forceinline__ uint32_t measure_pinhole_staged(const CameraView &cv, const MapConsts &mc, int bx, int by,
                                                           float px, float py, int bz, float xs[8], float ws[8],
                                                           float *region)
{
    const StageRect r = stage_rect(cv, mc, bx, by, bz);
    if (r.w * r.h == 0)
        return measure_pinhole<WEIGHTING>(cv, mc, px, py, bz, xs, ws);
    // the previous block's reads of the region are complete before it is rewritten
    __builtin_amdgcn_wave_barrier();
    stage_copy(cv, r, region);
    const uint32_t width = (uint32_t)cv.width;
    const __amdgpu_buffer_rsrc_t depth = make_rsrc(cv.depth, 4u * width * (uint32_t)cv.height);
    const float ax = cv.R[0] * px + cv.R[1] * py;
    const float ay = cv.R[3] * px + cv.R[4] * py;
    const float az = cv.R[6] * px + cv.R[7] * py;
    float zc[8], d[8];
    uint32_t pix_off[8];
    uint32_t outside = 0;   // bit s: voxel s projects into the image but outside the rectangle
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const float pz = ((float)(8 * bz + s) + 0.5f) * mc.vs;
        const float xc = (ax + cv.R[2] * pz) + cv.t[0];
        const float yc = (ay + cv.R[5] * pz) + cv.t[1];
        zc[s] = (az + cv.R[8] * pz) + cv.t[2];
        const float rz = 1.0f / zc[s];
        const float u = cv.fx * (xc * rz) + cv.cx;
        const float v = cv.fy * (yc * rz) + cv.cy;
        const bool ok = zc[s] > 0.0f && u >= 0.0f && u < cv.width_f && v >= 0.0f && v < cv.height_f;
        const uint32_t i = (uint32_t)(ok ? u : 0.0f);
        const uint32_t j = (uint32_t)(ok ? v : 0.0f);
        const uint32_t li = i - (uint32_t)r.u0, lj = j - (uint32_t)r.v0;
        const bool in_rect = li < (uint32_t)r.w && lj < (uint32_t)r.h;
        pix_off[s] = ok && !in_rect ? 4u * (j * width + i) : kOutOfRange;
        outside |= (ok && !in_rect ? 1u : 0u) << s;
        d[s] = ok && in_rect ? region[lj * (uint32_t)r.w + li] : 0.0f;
    }
    if (__ballot(outside != 0) != 0ull) {
#pragma unroll
        for (int s = 0; s < 8; ++s)
            if ((outside >> s) & 1u)
                d[s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(depth, pix_off[s], 0, 0));
    }
    uint32_t hit = 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const float dp = d[s] - zc[s];
        float wm = 1.0f;
        if (WEIGHTING == 1 && dp < -mc.delta)
            wm = (mc.eps + dp) * mc.span_inv;
        const bool upd = d[s] > 0.0f && d[s] <= cv.d_max && dp >= -mc.eps && wm > 0.0f;
        xs[s] = dp < mc.eps ? dp : mc.eps;
        ws[s] = wm;
        hit |= (upd ? 1u : 0u) << s;
    }
    return hit;
}

// Eq. (3) and the TSDF measurement (§IV-B) of the lane's 8 voxels against a
// spherical range image: azimuth theta = atan2(y, x), polar angle phi =
// atan2(sqrt(x^2 + y^2), z) (the angle acos(z / r)), pixel coordinates
// u = (theta - theta_start) alpha, v = (phi - phi_start) beta; the range is
// interpolated bilinearly between the 4 beam centres around (u, v) only when
// all 4 are valid and their spread is at most interp_diff; the voxel depth is
// its Euclidean range.  Same operation order as the CPU oracle.
template <int WEIGHTING>
__device__ __forceinline__ uint32_t measure_spherical(const CameraView &cv, const MapConsts &mc, float px, float py,
                                                      int bz, float xs[8], float ws[8])
{
    const uint32_t width = (uint32_t)cv.width;
    const __amdgpu_buffer_rsrc_t range = make_rsrc(cv.depth, 4u * width * (uint32_t)cv.height);
    const float ax = cv.R[0] * px + cv.R[1] * py;
    const float ay = cv.R[3] * px + cv.R[4] * py;
    const float az = cv.R[6] * px + cv.R[7] * py;
    uint32_t hit = 0;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const float pz = ((float)(8 * bz + s) + 0.5f) * mc.vs;
        const float xc = (ax + cv.R[2] * pz) + cv.t[0];
        const float yc = (ay + cv.R[5] * pz) + cv.t[1];
        const float zc = (az + cv.R[8] * pz) + cv.t[2];
        const float rv = sqrtf((xc * xc + yc * yc) + zc * zc);
        const float theta = atan2_as(yc, xc);
        const float phi = atan2_as(sqrtf(xc * xc + yc * yc), zc);
        const float uc = (theta - cv.az_start) * cv.alpha - 0.5f;
        const float vc = (phi - cv.pol_start) * cv.beta - 0.5f;
        const float fi = floorf(uc), fj = floorf(vc);
        const float fu = uc - fi, fv = vc - fj;
        // rows never wrap; columns wrap for a full circle
        const bool row_ok = rv > 0.0f && fj >= 0.0f && fj + 1.0f <= cv.height_f - 1.0f;
        int i0 = row_ok ? (int)fi : 0;
        int i1;
        bool col_ok;
        if (cv.full_circle) {
            // i0 mod width; conditional adds cover every column an azimuth
            // start within two turns produces, the division the rest
            const int w = cv.width;
            if (i0 >= -2 * w && i0 < 3 * w) {
                i0 += i0 < 0 ? w : 0;
                i0 += i0 < 0 ? w : 0;
                i0 -= i0 >= w ? w : 0;
                i0 -= i0 >= w ? w : 0;
            } else {
                i0 = ((i0 % w) + w) % w;
            }
            i1 = i0 + 1 < w ? i0 + 1 : 0;
            col_ok = true;
        } else {
            col_ok = i0 >= 0 && i0 + 1 <= cv.width - 1;
            i1 = i0 + 1;
        }
        const bool ok = row_ok && col_ok;
        const uint32_t j0 = ok ? (uint32_t)fj : 0u;
        const uint32_t o00 = ok ? 4u * (j0 * width + (uint32_t)i0) : kOutOfRange;
        const uint32_t o10 = ok ? 4u * (j0 * width + (uint32_t)i1) : kOutOfRange;
        const uint32_t o01 = ok ? o00 + 4u * width : kOutOfRange;
        const uint32_t o11 = ok ? o10 + 4u * width : kOutOfRange;
        const float r00 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(range, o00, 0, 0));
        const float r10 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(range, o10, 0, 0));
        const float r01 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(range, o01, 0, 0));
        const float r11 = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(range, o11, 0, 0));
        const bool valid = r00 > 0.0f && r00 <= cv.d_max && r10 > 0.0f && r10 <= cv.d_max && r01 > 0.0f &&
                           r01 <= cv.d_max && r11 > 0.0f && r11 <= cv.d_max;
        float mn = r00 < r10 ? r00 : r10, mx = r00 < r10 ? r10 : r00;
        mn = r01 < mn ? r01 : mn;
        mx = r01 > mx ? r01 : mx;
        mn = r11 < mn ? r11 : mn;
        mx = r11 > mx ? r11 : mx;
        const float d = (1.0f - fv) * ((1.0f - fu) * r00 + fu * r10) + fv * ((1.0f - fu) * r01 + fu * r11);
        const float dp = d - rv;
        float wm = 1.0f;
        if (WEIGHTING == 1 && dp < -mc.delta)
            wm = (mc.eps + dp) * mc.span_inv;
        const bool upd = ok && valid && mx - mn <= cv.interp_diff && dp >= -mc.eps && wm > 0.0f;
        xs[s] = dp < mc.eps ? dp : mc.eps;
        ws[s] = wm;
        hit |= (upd ? 1u : 0u) << s;
    }
    return hit;
}

// SPHERICAL: 0 = every view is a pinhole camera (the spherical code is not
// compiled in), 1 = the view's model decides.
template <int WEIGHTING, int SPHERICAL>
__device__ __forceinline__ uint32_t measure_view(const CameraView &cv, const MapConsts &mc, float px, float py,
                                                 int bz, float xs[8], float ws[8])
{
    if (SPHERICAL && cv.model == kModelSpherical)
        return measure_spherical<WEIGHTING>(cv, mc, px, py, bz, xs, ws);
    return measure_pinhole<WEIGHTING>(cv, mc, px, py, bz, xs, ws);
}

// Weighted average with capped weight (§IV-B):
// D <- (D W + x w) / (W + w),  W <- min(W + w, w_max).
__device__ __forceinline__ float2 fuse(float2 dw, float x, float w, float w_max)
{
    const float n = dw.x * dw.y + x * w;
    const float sum = dw.y + w;
    return make_float2(n / sum, sum < w_max ? sum : w_max);
}

// Touched-list compaction helpers.  Each wave keeps its touched pool slots in
// one register (lane i holds entry i); a workgroup reserves room for all of its
// waves with one atomic on its sub-list counter.
__device__ __forceinline__ void write_touched(const DeviceMap &dm, int sub, uint32_t base, uint32_t pending, int n)
{
    const int lane = lane_id();
    if (lane < n) {
        const uint32_t at = base + (uint32_t)lane;
        if (at < dm.block_cap)
            dm.touched[(size_t)sub * dm.block_cap + at] = pending;
        else
            atomicOr(&dm.counters[kErrorBits], kErrTouchedOverflow);
    }
}

// Walk launches (small lattices, a few blocks per wave) reserve a touched
// block's entry as soon as its pool slot is known: the atomic's round trip
// then overlaps the block's voxel traffic instead of ending the launch, and
// lane 0 writes the entry (write_touched_entry) once the voxel stores are
// issued.  On large lattices the same-address atomics would queue up, so
// compacted launches collect entries per wave and reserve per workgroup.
__device__ __forceinline__ uint32_t reserve_touched(const DeviceMap &dm, int parity, int sub)
{
    uint32_t at = 0;
    if (lane_id() == 0)
        at = atomicAdd(&dm.counters[touched_counter(parity, sub)], 1u);
    return at;   // meaningful in lane 0
}

__device__ __forceinline__ void write_touched_entry(const DeviceMap &dm, int sub, uint32_t at, uint32_t slot)
{
    if (lane_id() == 0) {
        if (at < dm.block_cap)
            dm.touched[(size_t)sub * dm.block_cap + at] = slot;
        else
            atomicOr(&dm.counters[kErrorBits], kErrTouchedOverflow);
    }
}

// A wave whose private list is full reserves room on its own (rare).
__device__ __forceinline__ void flush_wave(const DeviceMap &dm, int parity, int sub, uint32_t pending, int n)
{
    uint32_t base = 0;
    if (lane_id() == 0)
        base = atomicAdd(&dm.counters[touched_counter(parity, sub)], (uint32_t)n);
    write_touched(dm, sub, (uint32_t)wave_bcast((int)base), pending, n);
}

// Records `slot` in the wave's private list.
__device__ __forceinline__ void push_touched(const DeviceMap &dm, int parity, int sub, uint32_t slot,
                                             uint32_t &pending, int &n_pending)
{
    if (lane_id() == n_pending)
        pending = slot;
    if (++n_pending == 64) {
        flush_wave(dm, parity, sub, pending, n_pending);
        n_pending = 0;
    }
}

// End of a launch: prefix sum over the workgroup's waves, one atomic on the
// sub-list counter, entries written; voxel-update, voxel-write and
// candidate-block counts summed likewise.
template <int WAVES>
__device__ __forceinline__ void finish_group(const DeviceMap &dm, int parity, int sub, uint32_t pending,
                                             int n_pending, uint32_t n_updates, uint32_t n_writes,
                                             uint32_t n_candidates)
{
    __shared__ uint32_t s_count[WAVES];
    __shared__ uint32_t s_updates[WAVES];
    __shared__ uint32_t s_writes[WAVES];
    __shared__ uint32_t s_cands[WAVES];
    __shared__ uint32_t s_base;
    const int wave = (int)(threadIdx.x >> 6);
    if (lane_id() == 0) {
        s_count[wave] = (uint32_t)n_pending;
        s_updates[wave] = n_updates;
        s_writes[wave] = n_writes;
        s_cands[wave] = n_candidates;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t total = 0, upd = 0, wr = 0, cand = 0;
        for (int k = 0; k < WAVES; ++k) {
            total += s_count[k];
            upd += s_updates[k];
            wr += s_writes[k];
            cand += s_cands[k];
        }
        s_base = total ? atomicAdd(&dm.counters[touched_counter(parity, sub)], total) : 0u;
        if (upd)
            atomicAdd(&dm.totals[kTotalUpdates + sub * kTotalsStride], (unsigned long long)upd);
        if (wr)
            atomicAdd(&dm.totals[kTotalWrites + sub * kTotalsStride], (unsigned long long)wr);
        if (cand)
            atomicAdd(&dm.totals[kTotalCandidates + sub * kTotalsStride], (unsigned long long)cand);
    }
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < wave; ++k)
        before += s_count[k];
    write_touched(dm, sub, s_base + before, pending, n_pending);
}

// Once per launch (workgroup 0, after its own work): the previous launch
// (stream-ordered, complete) counted into the other parity; fold its touched
// count into the running total and clear it for the next launch.  Nothing in
// this launch touches the other parity's counters, so where in the launch
// this runs does not matter; at the end its returning atomics delay no
// workgroup's first pass.
__device__ __forceinline__ void fold_previous_launch(const DeviceMap &dm, int parity)
{
    if (blockIdx.x == 0 && threadIdx.x < kSubLists) {
        const uint32_t prev = atomicExch(&dm.counters[touched_counter(parity ^ 1, (int)threadIdx.x)], 0u);
        if (prev != 0)
            atomicAdd(&dm.totals[kTotalTouched], (unsigned long long)prev);
    }
    // the candidate count of the other parity is next used by the following
    // launch's cull kernel, which runs after this launch
    if (blockIdx.x == 0 && threadIdx.x == kSubLists)
        atomicExch(&dm.counters[cand_counter(parity ^ 1)], 0u);
}

// Lanes a compacted launch's cull kernel gives each lattice block: one per
// view, rounded up to a power of two (a wave holds 64 / lanes blocks).
__host__ __device__ __forceinline__ int cull_lanes_per_block(int n_views)
{
    int lanes = 1;
    while (lanes < n_views)
        lanes <<= 1;
    return lanes;
}

// Cull kernel of a compacted launch.  LANE_VIEWS: lane (block, view) tests
// one lattice block against one view (grid-stride over blocks x
// lanes-per-block) and one ballot gives each block's view mask -- for batches
// whose views share one camera model; when pinhole and spherical views mix, a
// wave would run both tests with few lanes each, so then every lane tests its
// block against all views in turn.  The first lane of a block with a nonzero
// mask appends (lattice index, view mask) to lat.cand.  A workgroup reserves
// its room with one atomic on the launch's candidate counter per pass (an LDS
// prefix over its waves' counts), and the views' parameters are copied into
// LDS once per workgroup: read view after view from the argument block, each
// is a chain of cold scalar loads on every CU.
template <bool LANE_VIEWS, bool PINHOLE = false>
__device__ __forceinline__ void cull_to_list(const DeviceMap &dm, const Lattice &lat, const CameraView *cams,
                                             int n_views, const MapConsts &mc, int parity,
                                             const PinholeCull *pc = nullptr)
{
    constexpr int kWaves = kCullThreads / 64;
    __shared__ uint32_t s_count[kWaves];
    __shared__ uint32_t s_base;
    __shared__ CameraView s_cams[kMaxViews];
    {
        static_assert(sizeof(CameraView) % 4 == 0, "CameraView is copied in 32-bit words");
        const uint32_t words = (uint32_t)n_views * (uint32_t)(sizeof(CameraView) / 4);
        const uint32_t *src = reinterpret_cast<const uint32_t *>(cams);
        uint32_t *dst = reinterpret_cast<uint32_t *>(s_cams);
        for (uint32_t k = threadIdx.x; k < words; k += (uint32_t)kCullThreads)
            dst[k] = src[k];
    }
    __syncthreads();
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int lanes = LANE_VIEWS ? cull_lanes_per_block(n_views) : 1;
    const int shift = __builtin_ctz((unsigned)lanes);
    const int view = lane & (lanes - 1);
    const int group = lane & ~(lanes - 1);                         // first lane of the block's group
    const unsigned long long group_mask = lanes == 64 ? ~0ull : ((1ull << lanes) - 1ull);
    const unsigned long long n_lat = (unsigned long long)lat.n_lat;
    const unsigned long long n_work = n_lat << shift;
    const unsigned long long stride = (unsigned long long)gridDim.x * (unsigned long long)kCullThreads;
    // the loop runs the same number of times in every thread of the workgroup
    for (unsigned long long base = (unsigned long long)blockIdx.x * kCullThreads; base < n_work; base += stride) {
        const unsigned long long item = base + threadIdx.x;
        const uint32_t lb = (uint32_t)(item >> shift);
        uint32_t vmask = 0;
        if (item < n_work && view < n_views) {
            int bx, by, bz;
            lattice_block(lat, lb, bx, by, bz);
            if constexpr (LANE_VIEWS) {
                if constexpr (PINHOLE)   // a single pinhole view with its precomputed planes
                    vmask = lane_block_pinhole_precomputed(*pc, s_cams[view], mc, lat, bx, by, bz) ? 1u : 0u;
                else
                    vmask = lane_block_in_view(s_cams[view], mc, bx, by, bz) ? 1u : 0u;
            } else {
                for (int v = 0; v < n_views; ++v)
                    if (lane_block_in_view(s_cams[v], mc, bx, by, bz))
                        vmask |= 1u << v;
            }
        }
        if constexpr (LANE_VIEWS)
            vmask = (uint32_t)((__ballot(vmask != 0u) >> group) & group_mask);
        const bool lead = view == 0 && vmask != 0u;
        const unsigned long long keep = __ballot(lead);
        if (lane == 0)
            s_count[wave] = (uint32_t)__popcll(keep);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t total = 0;
            for (int k = 0; k < kWaves; ++k)
                total += s_count[k];
            s_base = total ? atomicAdd(&dm.counters[cand_counter(parity)], total) : 0u;
        }
        __syncthreads();
        uint32_t at = s_base;
        for (int k = 0; k < wave; ++k)
            at += s_count[k];
        if (lead)
            lat.cand[at + (uint32_t)__popcll(keep & ((1ull << lane) - 1ull))] = make_uint2(lb, vmask);
        __syncthreads();   // s_count and s_base are rewritten by the next pass
    }
}

// List walk of a compacted launch: the waves of the grid take the
// candidates round-robin (wave-uniform) and hand each to body(bx, by, bz,
// view_mask).  The count was written by the cull kernel earlier on the stream.
template <class Body>
__device__ __forceinline__ void scan_list(const DeviceMap &dm, const Lattice &lat, int parity, Body &&body)
{
    const uint32_t n = __hip_atomic_load(&dm.counters[cand_counter(parity)], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t count = (uint32_t)__builtin_amdgcn_readfirstlane((int)n);
    const uint32_t waves = gridDim.x * (uint32_t)kWavesPerGroup;
    // consecutive entries go to different workgroups of one XCD, as in scan_lattice
    for (uint32_t i = (threadIdx.x >> 6) * gridDim.x + spread_position(blockIdx.x, gridDim.x); i < count;
         i += waves) {
        const uint2 e = lat.cand[i];
        const uint32_t lb = (uint32_t)__builtin_amdgcn_readfirstlane((int)e.x);
        const uint32_t vmask = (uint32_t)__builtin_amdgcn_readfirstlane((int)e.y);
        int bx, by, bz;
        lattice_block(lat, lb, bx, by, bz);
        body(bx, by, bz, vmask);
    }
}

}  // namespace dev
}  // namespace tsdf

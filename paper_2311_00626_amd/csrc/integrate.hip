// Projective TSDF integration of one depth frame (nvblox §IV-B), fused into a
// single gfx950 kernel.
//
// One wave64 owns one block of the frame's block lattice at a time:
//   1. culling  -- the block's 8 corners are tested against the view frustum
//                  (side planes, camera plane, far plane); a block whose
//                  corners are all outside one plane cannot hold an updated
//                  voxel.  The lattice enumerates every block index once, so
//                  the candidate set has no duplicates to remove.
//   2. measure  -- lane (lx, ly) walks the 8 z-slabs of the block; each voxel
//                  is moved into the camera frame (Eq. (1)), projected with the
//                  pinhole model (Eq. (2)), the nearest pixel is sampled and
//                  the truncated projective distance and its weight are kept
//                  in registers.  A ballot tells whether any voxel changes.
//   3. allocate -- only then is the block looked up in the block hash and, if
//                  new, inserted (64-bit atomicCAS) with a fresh zeroed pool
//                  slot (§IV-A).
//   4. update   -- the weighted average runs on coalesced 512-byte slab loads
//                  and stores of (distance, weight) pairs.
//   5. compact  -- the block's pool slot is appended to the touched list with
//                  one atomic per wave; the last workgroup to finish publishes
//                  the frame's touched count and resets the frame counters, so
//                  the call needs no host synchronisation or memset.
//
// Bit-exactness: every floating-point statement in measure/update is one IEEE
// binary32 operation, in the order the CPU oracle uses, and the file is
// compiled with -ffp-contract=off (no fused multiply-add) and correctly
// rounded division.
#include "tsdf_internal.hpp"

namespace tsdf {
namespace {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ int wave_bcast(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ unsigned long long load_key(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-cooperative find-or-insert of `key` (wave-uniform) in the block hash.
// The 64 lanes probe 64 consecutive slots per step; the first slot in probe
// order that holds the key or is empty decides.  Returns the pool slot, or
// kInvalidSlot after recording an overflow in the error word.
__device__ uint32_t find_or_insert(const DeviceMap &dm, unsigned long long key)
{
    const int lane = lane_id();
    const uint32_t mask = dm.hash_mask;
    const uint32_t h = (uint32_t)hash_key(key) & mask;
    uint32_t fresh = kInvalidSlot;   // pool slot reserved for an insert (wave-uniform)
    uint32_t base = 0;
    while (base <= mask) {
        const uint32_t pos = (h + base + (uint32_t)lane) & mask;
        const unsigned long long k = load_key(&dm.keys[pos]);
        const unsigned long long m_hit = __ballot(k == key);
        const unsigned long long m_free = __ballot(k == kEmptyKey);
        const int f_hit = m_hit ? __builtin_ctzll(m_hit) : 64;
        const int f_free = m_free ? __builtin_ctzll(m_free) : 64;
        if (f_hit < f_free) {
            const uint32_t at = (h + base + (uint32_t)f_hit) & mask;
            uint32_t slot = 0;
            if (lane == 0) {
                // a key is published before its value; wait (bounded) for the value
                slot = __hip_atomic_load(&dm.vals[at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                for (int spin = 0; slot == kInvalidSlot && spin < (1 << 20); ++spin)
                    slot = __hip_atomic_load(&dm.vals[at], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (slot == kInvalidSlot)
                    atomicOr(&dm.counters[kErrorBits], kErrInsertRace);
            }
            return (uint32_t)wave_bcast((int)slot);
        }
        if (f_free == 64) {
            base += 64;
            continue;
        }
        const uint32_t at = (h + base + (uint32_t)f_free) & mask;
        int won = 0;
        if (lane == 0) {
            if (fresh == kInvalidSlot) {
                fresh = atomicAdd(&dm.counters[kNumBlocks], 1u);
                if (fresh >= dm.block_cap) {
                    atomicOr(&dm.counters[kErrorBits], kErrPoolFull);
                    fresh = kInvalidSlot;
                }
            }
            if (fresh != kInvalidSlot) {
                const unsigned long long prev = atomicCAS(&dm.keys[at], kEmptyKey, key);
                if (prev == kEmptyKey) {
                    dm.slot_keys[fresh] = key;
                    __hip_atomic_store(&dm.vals[at], fresh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    won = 1;
                } else if (prev == key) {
                    won = 2;   // the same key landed concurrently: read it on the next probe
                }
            }
        }
        fresh = (uint32_t)wave_bcast((int)fresh);
        won = wave_bcast(won);
        if (fresh == kInvalidSlot)
            return kInvalidSlot;
        if (won == 1)
            return fresh;
        // slot taken by another key (or by this key from elsewhere): probe this window again
    }
    if (lane_id() == 0)
        atomicOr(&dm.counters[kErrorBits], kErrHashFull);
    return kInvalidSlot;
}

// Block culling against the frustum planes.  Lane c (mod 8) evaluates corner
// c; a block is dropped when all 8 corners are outside one plane by more than
// the margin, which exceeds the binary32 error of any voxel's projection.
__device__ __forceinline__ bool block_in_view(const FrameArgs &fa, int bx, int by, int bz)
{
    const int c = lane_id() & 7;
    const float X = (float)(8 * bx + ((c & 1) ? 8 : 0)) * fa.vs;
    const float Y = (float)(8 * by + ((c & 2) ? 8 : 0)) * fa.vs;
    const float Z = (float)(8 * bz + ((c & 4) ? 8 : 0)) * fa.vs;
    const float xc = fa.R[0] * X + fa.R[1] * Y + fa.R[2] * Z + fa.t[0];
    const float yc = fa.R[3] * X + fa.R[4] * Y + fa.R[5] * Z + fa.t[1];
    const float zc = fa.R[6] * X + fa.R[7] * Y + fa.R[8] * Z + fa.t[2];
    const bool out_l = fa.fx * xc + fa.cx * zc < -fa.margin_u;
    const bool out_r = (fa.width_f - fa.cx) * zc - fa.fx * xc < -fa.margin_u;
    const bool out_t = fa.fy * yc + fa.cy * zc < -fa.margin_v;
    const bool out_b = (fa.height_f - fa.cy) * zc - fa.fy * yc < -fa.margin_v;
    const bool out_n = zc < -fa.margin_z;
    const bool out_f = zc > fa.zfar + fa.margin_z;
    const unsigned long long all = 0xFFull;
    return !(((__ballot(out_l) & all) == all) || ((__ballot(out_r) & all) == all) ||
             ((__ballot(out_t) & all) == all) || ((__ballot(out_b) & all) == all) ||
             ((__ballot(out_n) & all) == all) || ((__ballot(out_f) & all) == all));
}

// Eq. (1)-(2) and the TSDF measurement for one voxel.  (ax, ay, az) are the
// row partial sums R[r][0] px + R[r][1] py of the lane's column, shared by its
// 8 voxels; adding R[r][2] pz and t[r] afterwards is the oracle's order
// ((R0 px + R1 py) + R2 pz) + t.
template <int WEIGHTING>
__device__ __forceinline__ bool measure(const FrameArgs &fa, const float *__restrict__ depth,
                                        float ax, float ay, float az, float pz, float &x, float &w)
{
    const float xc = (ax + fa.R[2] * pz) + fa.t[0];
    const float yc = (ay + fa.R[5] * pz) + fa.t[1];
    const float zc = (az + fa.R[8] * pz) + fa.t[2];
    if (!(zc > 0.0f))
        return false;
    const float r = 1.0f / zc;
    const float u = fa.fx * (xc * r) + fa.cx;
    const float v = fa.fy * (yc * r) + fa.cy;
    if (!(u >= 0.0f && u < fa.width_f && v >= 0.0f && v < fa.height_f))
        return false;
    const int i = (int)u;
    const int j = (int)v;
    const float d = depth[(size_t)j * (size_t)fa.width + (size_t)i];
    if (!(d > 0.0f && d <= fa.d_max))
        return false;
    const float dp = d - zc;
    if (!(dp >= -fa.eps))
        return false;
    float wm = 1.0f;
    if (WEIGHTING == 1 && dp < -fa.delta)
        wm = (fa.eps + dp) * fa.span_inv;
    if (!(wm > 0.0f))
        return false;
    x = dp < fa.eps ? dp : fa.eps;
    w = wm;
    return true;
}

template <int WEIGHTING>
__global__ __launch_bounds__(256) void integrate_depth_kernel(DeviceMap dm, FrameArgs fa,
                                                              const float *__restrict__ depth)
{
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int lx = lane & 7;
    const int ly = lane >> 3;
    const uint32_t stride = gridDim.x * kWavesPerGroup;
    const uint32_t n_lat = (uint32_t)fa.n_lat;          // the host keeps it below 2^31
    const uint32_t dim_x = (uint32_t)fa.lat_dim[0], dim_y = (uint32_t)fa.lat_dim[1];

    for (uint32_t lb = blockIdx.x * kWavesPerGroup + (uint32_t)wave; lb < n_lat; lb += stride) {
        const uint32_t rest = lb / dim_x;
        const int bx = fa.lat_min[0] + (int)(lb - rest * dim_x);
        const int by = fa.lat_min[1] + (int)(rest % dim_y);
        const int bz = fa.lat_min[2] + (int)(rest / dim_y);
        if (!block_in_view(fa, bx, by, bz))
            continue;

        // voxel centres: ((float)g + 0.5) * voxel_size
        const float px = ((float)(8 * bx + lx) + 0.5f) * fa.vs;
        const float py = ((float)(8 * by + ly) + 0.5f) * fa.vs;
        const float ax = fa.R[0] * px + fa.R[1] * py;
        const float ay = fa.R[3] * px + fa.R[4] * py;
        const float az = fa.R[6] * px + fa.R[7] * py;
        float xs[8], ws[8];
        uint32_t hit = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const float pz = ((float)(8 * bz + s) + 0.5f) * fa.vs;
            xs[s] = 0.0f;
            ws[s] = 0.0f;
            if (measure<WEIGHTING>(fa, depth, ax, ay, az, pz, xs[s], ws[s]))
                hit |= 1u << s;
        }
        if (__ballot(hit != 0) == 0ull)
            continue;

        const uint32_t slot = find_or_insert(dm, pack_key(bx, by, bz));
        if (slot == kInvalidSlot)
            continue;

        float2 *vox = dm.pool + (size_t)slot * kBlockVoxels + lane;
        int n_upd = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const unsigned long long m = __ballot((hit >> s) & 1u);
            n_upd += __popcll(m);
            if ((hit >> s) & 1u) {
                float2 dw = vox[64 * s];
                const float n = dw.x * dw.y + xs[s] * ws[s];
                const float sum = dw.y + ws[s];
                dw.x = n / sum;
                dw.y = sum < fa.w_max ? sum : fa.w_max;
                vox[64 * s] = dw;
            }
        }
        if (lane == 0) {
            const uint32_t at = atomicAdd(&dm.counters[kTouched], 1u);
            if (at < dm.block_cap)
                dm.touched[at] = slot;
            else
                atomicOr(&dm.counters[kErrorBits], kErrTouchedOverflow);
            atomicAdd(&dm.totals[0], (unsigned long long)n_upd);
        }
    }

    // The last workgroup to finish publishes the frame's touched count and
    // clears the per-frame counters for the next launch.
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&dm.counters[kGroupsDone], 1u);
        if (done == gridDim.x - 1) {
            __threadfence();
            const uint32_t n = atomicAdd(&dm.counters[kTouched], 0u);
            atomicExch(&dm.counters[kTouchedLast], n < dm.block_cap ? n : dm.block_cap);
            atomicAdd(&dm.totals[1], (unsigned long long)n);
            atomicExch(&dm.counters[kTouched], 0u);
            atomicExch(&dm.counters[kGroupsDone], 0u);
        }
    }
}

}  // namespace

hipError_t launch_integrate_depth(const DeviceMap &dm, const FrameArgs &fa, int weighting,
                                  const float *depth, int groups, hipStream_t stream)
{
    const dim3 grid((unsigned)groups), block(64 * kWavesPerGroup);
    if (weighting == 1)
        hipLaunchKernelGGL(integrate_depth_kernel<1>, grid, block, 0, stream, dm, fa, depth);
    else
        hipLaunchKernelGGL(integrate_depth_kernel<0>, grid, block, 0, stream, dm, fa, depth);
    return hipGetLastError();
}

}  // namespace tsdf

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

// Raw buffer descriptors (word 3 of the gfx9-family resource: 32-bit data
// format).  A load whose offset is at or past num_records returns 0 and a
// store there is dropped, which predicates memory per lane without a branch.
constexpr int kBufferFlags = 0x00020000;
constexpr uint32_t kOutOfRange = 0x80000000u;
typedef unsigned int b64_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int wave_bcast(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Hash loads bypass the per-CU cache: other waves of the same launch insert keys.
__device__ __forceinline__ unsigned long long load_key(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t load_val(const uint32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-cooperative find-or-insert of `key` (wave-uniform) in the block hash.
// The 64 lanes look at 64 consecutive slots per step; the first slot in probe
// order that holds the key or is empty decides.  (k0, v0) is the first window,
// loaded by the caller ahead of time so that its latency overlaps the depth
// gathers.  Returns the pool slot, or kInvalidSlot after recording an overflow
// in the error word.
__device__ uint32_t find_or_insert(const DeviceMap &dm, unsigned long long key, uint32_t h,
                                   unsigned long long k0, uint32_t v0)
{
    const int lane = lane_id();
    const uint32_t mask = dm.hash_mask;
    uint32_t fresh = kInvalidSlot;   // pool slot reserved for an insert (wave-uniform)
    uint32_t base = 0;
    unsigned long long k = k0;
    uint32_t v = v0;
    bool loaded = true;
    while (base <= mask) {
        if (!loaded) {
            const uint32_t pos = (h + base + (uint32_t)lane) & mask;
            k = load_key(&dm.keys[pos]);
            v = load_val(&dm.vals[pos]);
        }
        loaded = false;
        const unsigned long long m_hit = __ballot(k == key);
        const unsigned long long m_free = __ballot(k == kEmptyKey);
        const int f_hit = m_hit ? __builtin_ctzll(m_hit) : 64;
        const int f_free = m_free ? __builtin_ctzll(m_free) : 64;
        if (f_hit < f_free) {
            uint32_t slot = (uint32_t)__shfl((int)v, f_hit);
            if (slot == kInvalidSlot) {
                // a key is published before its value: wait (bounded) for the value
                const uint32_t at = (h + base + (uint32_t)f_hit) & mask;
                if (lane == 0) {
                    for (int spin = 0; slot == kInvalidSlot && spin < (1 << 20); ++spin)
                        slot = load_val(&dm.vals[at]);
                    if (slot == kInvalidSlot)
                        atomicOr(&dm.counters[kErrorBits], kErrInsertRace);
                }
                slot = (uint32_t)wave_bcast((int)slot);
            }
            return slot;
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
                }
            }
        }
        fresh = (uint32_t)wave_bcast((int)fresh);
        won = wave_bcast(won);
        if (fresh == kInvalidSlot)
            return kInvalidSlot;
        if (won == 1)
            return fresh;
        // the slot went to another key (or to this key from elsewhere): reload this window
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

// Appends n pending touched slots of one wave (lane i holds the i-th) at
// `base` of sub-list `sub`.
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

// A wave whose private list is full reserves room on its own (rare).
__device__ __forceinline__ void flush_wave(const DeviceMap &dm, int parity, int sub, uint32_t pending, int n)
{
    uint32_t base = 0;
    if (lane_id() == 0)
        base = atomicAdd(&dm.counters[touched_counter(parity, sub)], (uint32_t)n);
    write_touched(dm, sub, (uint32_t)wave_bcast((int)base), pending, n);
}

template <int WEIGHTING>
__global__ __launch_bounds__(64 * kWavesPerGroup) void integrate_depth_kernel(DeviceMap dm, FrameArgs fa,
                                                              const float *__restrict__ depth)
{
    const int lane = lane_id();
    const int wave = (int)(threadIdx.x >> 6);
    const int lx = lane & 7;
    const int ly = lane >> 3;
    const uint32_t stride = gridDim.x * kWavesPerGroup;
    const uint32_t n_lat = (uint32_t)fa.n_lat;          // the host keeps it below 2^31
    const uint32_t dim_x = (uint32_t)fa.lat_dim[0], dim_y = (uint32_t)fa.lat_dim[1];
    const uint32_t width = (uint32_t)fa.width;

    const __amdgpu_buffer_rsrc_t depth_rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)depth, (short)0, (int)(4u * width * (uint32_t)fa.height), kBufferFlags);
    const int parity = fa.parity;
    const int sub = (int)(blockIdx.x % kSubLists);
    __shared__ uint32_t s_count[kWavesPerGroup];
    __shared__ uint32_t s_updates[kWavesPerGroup];
    __shared__ uint32_t s_base;

    // The previous frame (stream-ordered, complete) used the other parity:
    // fold its touched count into the running total and clear it for the next frame.
    if (blockIdx.x == 0 && threadIdx.x < kSubLists) {
        const uint32_t prev = atomicExch(&dm.counters[touched_counter(parity ^ 1, (int)threadIdx.x)], 0u);
        if (prev != 0)
            atomicAdd(&dm.totals[kTotalTouched], (unsigned long long)prev);
    }

    uint32_t pending = kInvalidSlot;   // wave-local touched list: lane i holds entry i
    int n_pending = 0;                 // wave-uniform
    uint32_t n_updates = 0;            // wave-uniform

    for (uint32_t lb = blockIdx.x * kWavesPerGroup + (uint32_t)wave; lb < n_lat; lb += stride) {
        const uint32_t rest = lb / dim_x;
        const int bx = fa.lat_min[0] + (int)(lb - rest * dim_x);
        const int by = fa.lat_min[1] + (int)(rest % dim_y);
        const int bz = fa.lat_min[2] + (int)(rest / dim_y);
        if (!block_in_view(fa, bx, by, bz))
            continue;

        // first hash probe window, consumed only if the block is touched
        const unsigned long long key = pack_key(bx, by, bz);
        const uint32_t h = (uint32_t)hash_key(key) & dm.hash_mask;
        const uint32_t pos0 = (h + (uint32_t)lane) & dm.hash_mask;
        const unsigned long long k0 = load_key(&dm.keys[pos0]);
        const uint32_t v0 = load_val(&dm.vals[pos0]);

        // Eq. (1)-(2) for the lane's 8 voxels.  Voxel centre p = ((float)g + 0.5) * vs;
        // p_C = ((R0 px + R1 py) + R2 pz) + t, the first sum shared by the column.
        const float px = ((float)(8 * bx + lx) + 0.5f) * fa.vs;
        const float py = ((float)(8 * by + ly) + 0.5f) * fa.vs;
        const float ax = fa.R[0] * px + fa.R[1] * py;
        const float ay = fa.R[3] * px + fa.R[4] * py;
        const float az = fa.R[6] * px + fa.R[7] * py;
        float zc[8];
        uint32_t pix_off[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const float pz = ((float)(8 * bz + s) + 0.5f) * fa.vs;
            const float xc = (ax + fa.R[2] * pz) + fa.t[0];
            const float yc = (ay + fa.R[5] * pz) + fa.t[1];
            zc[s] = (az + fa.R[8] * pz) + fa.t[2];
            const float r = 1.0f / zc[s];
            const float u = fa.fx * (xc * r) + fa.cx;
            const float v = fa.fy * (yc * r) + fa.cy;
            // nearest pixel: (i, j) covers [i, i+1) x [j, j+1); a voxel outside the
            // image gets an out-of-range offset, whose buffer load returns 0 (invalid)
            const bool ok = zc[s] > 0.0f && u >= 0.0f && u < fa.width_f && v >= 0.0f && v < fa.height_f;
            const uint32_t i = (uint32_t)(ok ? u : 0.0f);
            const uint32_t j = (uint32_t)(ok ? v : 0.0f);
            pix_off[s] = ok ? 4u * (j * width + i) : kOutOfRange;
        }
        // all 8 gathers in flight together
        float d[8];
#pragma unroll
        for (int s = 0; s < 8; ++s)
            d[s] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(depth_rsrc, pix_off[s], 0, 0));

        // TSDF measurement: valid depth, truncation band, weight
        float xs[8], ws[8];
        uint32_t hit = 0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const float dp = d[s] - zc[s];
            float wm = 1.0f;
            if (WEIGHTING == 1 && dp < -fa.delta)
                wm = (fa.eps + dp) * fa.span_inv;
            const bool upd = d[s] > 0.0f && d[s] <= fa.d_max && dp >= -fa.eps && wm > 0.0f;
            xs[s] = dp < fa.eps ? dp : fa.eps;
            ws[s] = wm;
            hit |= (upd ? 1u : 0u) << s;
        }
        if (__ballot(hit != 0) == 0ull)
            continue;

        const uint32_t slot = (uint32_t)wave_bcast((int)find_or_insert(dm, key, h, k0, v0));
        if (slot == kInvalidSlot)
            continue;

        // weighted average with capped weight on coalesced 512-byte slabs; lanes
        // whose voxel is not updated use an out-of-range offset (no load, no store)
        const __amdgpu_buffer_rsrc_t blk = __builtin_amdgcn_make_buffer_rsrc(
            (void *)(dm.pool + (size_t)slot * kBlockVoxels), (short)0, kBlockVoxels * 8, kBufferFlags);
        uint32_t off[8];
        float2 dw[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            off[s] = ((hit >> s) & 1u) ? 8u * (uint32_t)(64 * s + lane) : kOutOfRange;
            dw[s] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(blk, off[s], 0, 0));
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            // D <- (D W + x w) / (W + w),  W <- min(W + w, w_max)
            const float n = dw[s].x * dw[s].y + xs[s] * ws[s];
            const float sum = dw[s].y + ws[s];
            dw[s].x = n / sum;
            dw[s].y = sum < fa.w_max ? sum : fa.w_max;
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            n_updates += (uint32_t)__popcll(__ballot((hit >> s) & 1u));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64_t, dw[s]), blk, off[s], 0, 0);
        }
        // touched-block compaction: the wave keeps its list in one register
        if (lane == n_pending)
            pending = slot;
        if (++n_pending == 64) {
            flush_wave(dm, parity, sub, pending, n_pending);
            n_pending = 0;
        }
    }
    // Workgroup compaction of the touched list: prefix sum over the waves'
    // counts, one atomic per workgroup on its sub-list counter.
    if (lane == 0) {
        s_count[wave] = (uint32_t)n_pending;
        s_updates[wave] = n_updates;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t total = 0, upd = 0;
        for (int k = 0; k < kWavesPerGroup; ++k) {
            total += s_count[k];
            upd += s_updates[k];
        }
        s_base = total ? atomicAdd(&dm.counters[touched_counter(parity, sub)], total) : 0u;
        if (upd)
            atomicAdd(&dm.totals[kTotalUpdates + sub * kTotalsStride], (unsigned long long)upd);
    }
    __syncthreads();
    uint32_t before = 0;
    for (int k = 0; k < wave; ++k)
        before += s_count[k];
    write_touched(dm, sub, s_base + before, pending, n_pending);
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

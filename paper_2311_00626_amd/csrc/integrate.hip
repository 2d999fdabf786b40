// Projective TSDF integration of one depth frame (nvblox §IV-B), fused into a
// single gfx950 kernel.
//
// One wave64 owns one block of the frame's block lattice at a time:
//   1. culling  -- lanes test consecutive lattice blocks against the view
//                  frustum (side planes, camera plane, far plane) and keep the
//                  blocks of their workgroup's band (XCD-local image columns);
//                  the lattice enumerates every block index once, so the
//                  candidate set has no duplicates to remove.
//   2. measure  -- lane (lx, ly) projects the 8 voxels of its column
//                  (Eq. (1)-(2)), samples the nearest pixel and keeps the
//                  truncated projective distance and weight in registers; the
//                  first hash probe window is already in flight.
//   3. allocate -- only if a ballot finds an updated voxel is the block looked
//                  up in the block hash and, if new, inserted (64-bit
//                  atomicCAS) with a fresh zeroed pool slot (§IV-A); with
//                  ray-walk allocation every block the walk visited is.
//   4. update   -- the weighted average runs on 512-byte slab loads and stores
//                  of (distance, weight) pairs, predicated per lane.
//   5. compact  -- a touched block's pool slot is appended to the touched
//                  list: on small lattices with an atomic issued as soon as
//                  the slot is known, on large ones collected in a wave
//                  register and reserved with one atomic per workgroup;
//                  counters are double-buffered by launch parity, so a frame
//                  needs no host synchronisation, memset or end-of-kernel
//                  fence.
#include "device_common.hpp"

namespace tsdf {
namespace {

using namespace dev;

// LIST: the candidates come from the cull kernel's list (compacted launch)
// instead of this kernel's own walk of the lattice.  STAGE: a pinhole view's
// depth footprint is staged in LDS per block (measure_pinhole_staged).
template <int WEIGHTING, int STORAGE, int SPHERICAL, bool LIST, bool STAGE>
__device__ __forceinline__ void integrate_depth_body(const DeviceMap &dm, const FrameArgs &fa)
{
    static_assert(!STAGE || (SPHERICAL == 0 && WEIGHTING != kWeightLearned), "staging: pinhole, fixed weighting");
    __shared__ float s_stage[STAGE ? kWavesPerGroup * kStagePixels : 1];
    float *const region = s_stage + (STAGE ? (threadIdx.x >> 6) * kStagePixels : 0);
    const int lane = lane_id();
    const int lx = lane & 7;
    const int ly = lane >> 3;
    const int parity = fa.parity;
    const int sub = (int)(blockIdx.x % kSubLists);

    uint32_t pending = kInvalidSlot;   // wave-local touched list: lane i holds entry i
    int n_pending = 0;                 // wave-uniform
    uint32_t n_updates = 0;            // wave-uniform

    uint32_t n_cands = 0;              // wave-uniform: candidate blocks measured
    auto block = [&](int bx, int by, int bz, uint32_t) {
        ++n_cands;
        // first hash probe window, consumed only if the block is touched
        const unsigned long long key = pack_key(bx, by, bz);
        const uint32_t h = probe_start(key, dm.hash_mask);
        const ProbeWindow w0 = load_first_window(dm, h);

        // voxel centre p = ((float)g + 0.5) * vs
        const float px = ((float)(8 * bx + lx) + 0.5f) * fa.mc.vs;
        const float py = ((float)(8 * by + ly) + 0.5f) * fa.mc.vs;
        float xs[8], ws[8];
        uint32_t hit;
        if constexpr (STAGE)
            hit = measure_pinhole_staged<WEIGHTING>(fa.cam, fa.mc, bx, by, px, py, bz, xs, ws, region);
        else
            hit = measure_view<WEIGHTING, SPHERICAL>(fa.cam, fa.mc, px, py, bz, xs, ws);
        // ray-walk allocation keeps every visited block, updated or not
        if (!fa.cam.dda_marks && __ballot(hit != 0) == 0ull)
            return;

        const uint32_t slot = find_or_insert(dm, key, h, w0);
        if (slot == kInvalidSlot)
            return;

        // lanes whose voxel is not updated use an out-of-range offset: no load, no store
        using IO = VoxelIO<STORAGE>;
        const __amdgpu_buffer_rsrc_t blk = block_rsrc<STORAGE>(dm, slot);
        uint32_t off[8];
        float2 dw[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            off[s] = ((hit >> s) & 1u) ? IO::kBytes * (uint32_t)(64 * s + lane) : kOutOfRange;
            dw[s] = IO::load(blk, off[s]);
        }
        // the touched entry is reserved behind the voxel loads: its result is
        // taken into a scalar register as soon as it is awaited, and awaited
        // ahead of the loads it would put a full round trip before them
        uint32_t at = 0;
        if constexpr (!LIST)
            at = reserve_touched(dm, parity, sub);
#pragma unroll
        for (int s = 0; s < 8; ++s)
            dw[s] = fuse(dw[s], xs[s], ws[s], fa.mc.w_max);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            n_updates += (uint32_t)__popcll(__ballot((hit >> s) & 1u));
            IO::store(blk, off[s], dw[s]);
        }
        if constexpr (LIST)
            push_touched(dm, parity, sub, slot, pending, n_pending);
        else
            write_touched_entry(dm, sub, at, slot);
    };
    if constexpr (LIST)
        scan_list(dm, fa.lat, parity, block);
    else
        scan_lattice<SPHERICAL == 0>(fa.lat, &fa.cam, 1, fa.mc, block);   // (the plane table's kernel arguments cost the walk more than it saves)
    // one write per update: a single view updates a voxel at most once
    finish_group<kWavesPerGroup>(dm, parity, sub, pending, n_pending, n_updates, n_updates, n_cands);
    fold_previous_launch(dm, parity);
}

// With binary32 storage five waves per SIMD cap the walking kernel at 96
// VGPRs (a frame of 640x480 at 4 cm runs 2 % faster than uncapped at ~109).
// The binary16 form, with its conversions, runs slower under that cap, and
// already under a four-wave one (its code changes at 102 VGPRs), so it keeps
// the compiler's own choice (two waves: the minimum a 512-thread group needs).
template <int WEIGHTING, int STORAGE, int SPHERICAL, bool STAGE = false>
__global__ __launch_bounds__(64 * kWavesPerGroup, STORAGE == 0 ? 5 : 2) void integrate_depth_kernel(DeviceMap dm,
                                                                                                   FrameArgs fa)
{
    integrate_depth_body<WEIGHTING, STORAGE, SPHERICAL, false, STAGE>(dm, fa);
}

template <int WEIGHTING, int STORAGE, int SPHERICAL, bool STAGE = false>
__global__ __launch_bounds__(64 * kWavesPerGroup) void integrate_depth_list_kernel(DeviceMap dm, FrameArgs fa)
{
    integrate_depth_body<WEIGHTING, STORAGE, SPHERICAL, true, STAGE>(dm, fa);
}

// PINHOLE: a pinhole view with the host's precomputed planes (fa.pc); else
// any single view through its CameraView.
template <bool PINHOLE>
__global__ __launch_bounds__(kCullThreads) void cull_frame_kernel(DeviceMap dm, FrameArgs fa)
{
    cull_to_list<true, PINHOLE>(dm, fa.lat, &fa.cam, 1, fa.mc, fa.parity, &fa.pc);
}

}  // namespace

hipError_t launch_cull_frame(const DeviceMap &dm, const FrameArgs &fa, hipStream_t stream)
{
    const unsigned groups = (unsigned)std::max<long long>(
        1, std::min<long long>((fa.lat.n_lat + kCullThreads - 1) / kCullThreads, kCullGroups));  // one view: one lane per block
    if (fa.pc.valid)
        hipLaunchKernelGGL(cull_frame_kernel<true>, dim3(groups), dim3(kCullThreads), 0, stream, dm, fa);
    else
        hipLaunchKernelGGL(cull_frame_kernel<false>, dim3(groups), dim3(kCullThreads), 0, stream, dm, fa);
    return hipGetLastError();
}

// Workgroups of 64 * kWavesPerGroup threads that one compute unit keeps
// resident for kernel k (1 if the runtime cannot say).
static int resident_per_cu(const void *k)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * kWavesPerGroup, 0) != hipSuccess || n < 1) {
        (void)hipGetLastError();
        n = 1;
    }
    return n;
}

// The compacted launch: `groups` workgroups, or with fill_cus > 0 every
// workgroup that fill_cus compute units keep resident (a multiple of
// kPartitions for spread_position, at least kPartitions).
template <int WEIGHTING, int STORAGE, int SPHERICAL, bool STAGE>
static void launch_list(const DeviceMap &dm, const FrameArgs &fa, int groups, int fill_cus, hipStream_t stream)
{
    if (fill_cus > 0) {
        static const int per_cu =
            resident_per_cu(reinterpret_cast<const void *>(&integrate_depth_list_kernel<WEIGHTING, STORAGE, SPHERICAL, STAGE>));
        groups = std::max(kPartitions, per_cu * fill_cus / kPartitions * kPartitions);
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_depth_list_kernel<WEIGHTING, STORAGE, SPHERICAL, STAGE>),
                       dim3((unsigned)groups), dim3(64 * kWavesPerGroup), 0, stream, dm, fa);
}

template <int WEIGHTING, int STORAGE, int SPHERICAL, bool STAGE>
static void launch_walk(const DeviceMap &dm, const FrameArgs &fa, int groups, hipStream_t stream)
{
    hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_depth_kernel<WEIGHTING, STORAGE, SPHERICAL, STAGE>),
                       dim3((unsigned)groups), dim3(64 * kWavesPerGroup), 0, stream, dm, fa);
}

template <int WEIGHTING, int STORAGE, int SPHERICAL, bool STAGE>
static void launch_form(const DeviceMap &dm, const FrameArgs &fa, int groups, int fill_cus, hipStream_t stream)
{
    if (fa.lat.cand)
        launch_list<WEIGHTING, STORAGE, SPHERICAL, STAGE>(dm, fa, groups, fill_cus, stream);
    else
        launch_walk<WEIGHTING, STORAGE, SPHERICAL, STAGE>(dm, fa, groups, stream);
}

template <int WEIGHTING, int SPHERICAL>
static void launch_depth_storage(const DeviceMap &dm, const FrameArgs &fa, int groups, int fill_cus,
                                 hipStream_t stream)
{
    if constexpr (SPHERICAL == 0 && WEIGHTING != kWeightLearned) {
        if (fa.stage) {
            if (dm.storage == 1)
                launch_form<WEIGHTING, 1, 0, true>(dm, fa, groups, fill_cus, stream);
            else
                launch_form<WEIGHTING, 0, 0, true>(dm, fa, groups, fill_cus, stream);
            return;
        }
    }
    if (dm.storage == 1)
        launch_form<WEIGHTING, 1, SPHERICAL, false>(dm, fa, groups, fill_cus, stream);
    else
        launch_form<WEIGHTING, 0, SPHERICAL, false>(dm, fa, groups, fill_cus, stream);
}

hipError_t launch_integrate_depth(const DeviceMap &dm, const FrameArgs &fa, int weighting, int groups,
                                  hipStream_t stream, int fill_cus)
{
    const bool spherical = fa.cam.model == kModelSpherical;
    if (weighting == kWeightLearned) {
        if (spherical || !fa.cam.sm_maps)
            return hipErrorInvalidValue;
        launch_depth_storage<kWeightLearned, 0>(dm, fa, groups, fill_cus, stream);
    } else if (weighting == kWeightDropoff) {
        if (spherical)
            launch_depth_storage<kWeightDropoff, 1>(dm, fa, groups, fill_cus, stream);
        else
            launch_depth_storage<kWeightDropoff, 0>(dm, fa, groups, fill_cus, stream);
    } else {
        if (spherical)
            launch_depth_storage<kWeightConstant, 1>(dm, fa, groups, fill_cus, stream);
        else
            launch_depth_storage<kWeightConstant, 0>(dm, fa, groups, fill_cus, stream);
    }
    return hipGetLastError();
}

}  // namespace tsdf

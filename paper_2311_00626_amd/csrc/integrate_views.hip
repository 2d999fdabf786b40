// Projective TSDF integration of a batch of depth views in one launch
// (nvblox §IV-B applied to several frames or sensors at once).
//
// The result is bit-identical to integrating the views one after another in
// array order: every voxel is owned by one wave, which loads its (distance,
// weight) once, applies the views' updates in order in registers (each update
// is the same sequence of binary32 operations as a single-frame launch) and
// stores it once.  Block allocation follows the same rule as for one frame: a
// block exists once any view updates any of its voxels.
//
// With binary16 storage the register state is rounded to binary16 after each
// view, so the batch stays bit-identical to storing and reloading per view.
//
// Per block of the union lattice of all views:
//   1. culling against every view's frustum -> view mask (wave-uniform), only
//      for blocks of the workgroup's band (XCD-local image columns); in a
//      compacted launch the cull kernel has done this and the blocks come
//      from its list;
//   2. view 0 of the mask is measured while the first hash window is in flight;
//   3. the block is looked up; an existing block's 512 voxels are loaded while
//      the next view is being measured (software pipeline of depth 2);
//   4. each view's updates are fused in registers, in view order;
//   5. a block with any updated voxel is inserted if new, the updated voxels
//      are stored (buffer stores predicated per lane) and its pool slot joins
//      the touched list.
#include "device_common.hpp"

namespace tsdf {
namespace {

using namespace dev;

// LIST: candidates from the cull kernel's list instead of the lattice walk.
template <int WEIGHTING, int STORAGE, int SPHERICAL, bool LIST>
__device__ __forceinline__ void integrate_views_body(const DeviceMap &dm, const ViewsArgs &va)
{
    const int lane = lane_id();
    const int lx = lane & 7;
    const int ly = lane >> 3;
    const int parity = va.parity;
    const int sub = (int)(blockIdx.x % kSubLists);

    uint32_t pending = kInvalidSlot;
    int n_pending = 0;
    uint32_t n_updates = 0;   // voxel updates, one per voxel per view
    uint32_t n_writes = 0;    // voxels stored, one per voxel per launch

    uint32_t n_cands = 0;     // candidate blocks measured (one per block per launch)
    auto block = [&](int bx, int by, int bz, uint32_t vmask) {
        ++n_cands;
        const unsigned long long key = pack_key(bx, by, bz);
        const uint32_t h = probe_start(key, dm.hash_mask);
        const ProbeWindow w0 = load_first_window(dm, h);

        const float px = ((float)(8 * bx + lx) + 0.5f) * va.mc.vs;
        const float py = ((float)(8 * by + ly) + 0.5f) * va.mc.vs;

        // view pipeline: (xa, wa, ha) holds the measured, not yet fused view
        float xa[8], wa[8];
        int v = __builtin_ctz(vmask);
        uint32_t rest = vmask & (vmask - 1);
        uint32_t ha = measure_view<WEIGHTING, SPHERICAL>(va.cam[v], va.mc, px, py, bz, xa, wa);

        // state of an existing block, loaded while the next view is measured
        using IO = VoxelIO<STORAGE>;
        const uint32_t found = find_block(dm, key, h, w0);
        float2 dw[8];
        if (found != kInvalidSlot) {
            const __amdgpu_buffer_rsrc_t blk = block_rsrc<STORAGE>(dm, found);
#pragma unroll
            for (int s = 0; s < 8; ++s)
                dw[s] = IO::load(blk, IO::kBytes * (uint32_t)(64 * s + lane));
        } else {
#pragma unroll
            for (int s = 0; s < 8; ++s)
                dw[s] = make_float2(0.0f, 0.0f);
        }

        uint32_t any = 0;
        while (true) {
            float xb[8], wb[8];
            uint32_t hb = 0;
            const bool more = rest != 0;
            if (more) {
                v = __builtin_ctz(rest);
                rest &= rest - 1;
                hb = measure_view<WEIGHTING, SPHERICAL>(va.cam[v], va.mc, px, py, bz, xb, wb);
            }
            // fuse the pending view, in view order; the state is rounded to the
            // storage precision after every view, exactly as a store and reload would
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                n_updates += (uint32_t)__popcll(__ballot((ha >> s) & 1u));
                if ((ha >> s) & 1u)
                    dw[s] = IO::quantize(fuse(dw[s], xa[s], wa[s], va.mc.w_max));
            }
            any |= ha;
            if (!more)
                break;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                xa[s] = xb[s];
                wa[s] = wb[s];
            }
            ha = hb;
        }
        if (__ballot(any != 0) == 0ull)
            return;

        const uint32_t slot = found != kInvalidSlot ? found : find_or_insert(dm, key, h, w0);
        if (slot == kInvalidSlot)
            return;
        const __amdgpu_buffer_rsrc_t blk = block_rsrc<STORAGE>(dm, slot);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            n_writes += (uint32_t)__popcll(__ballot((any >> s) & 1u));
            IO::store(blk, ((any >> s) & 1u) ? IO::kBytes * (uint32_t)(64 * s + lane) : kOutOfRange, dw[s]);
        }
        // reserved behind the stores: its result is awaited where it is taken
        uint32_t at = 0;
        if constexpr (!LIST)
            at = reserve_touched(dm, parity, sub);
        if constexpr (LIST)
            push_touched(dm, parity, sub, slot, pending, n_pending);
        else
            write_touched_entry(dm, sub, at, slot);
    };
    if constexpr (LIST)
        scan_list(dm, va.lat, parity, block);
    else
        scan_lattice(va.lat, va.cam, va.n_views, va.mc, block);
    finish_group<kWavesPerGroup>(dm, parity, sub, pending, n_pending, n_updates, n_writes, n_cands);
    fold_previous_launch(dm, parity);
}

// Arguments passed by value (eager launches).  Four waves per SIMD (two
// workgroups per CU) cap the kernel at 128 VGPRs.
template <int WEIGHTING, int STORAGE, int SPHERICAL>
__global__ __launch_bounds__(64 * kWavesPerGroup, 4) void integrate_views_kernel(DeviceMap dm, ViewsArgs va)
{
    integrate_views_body<WEIGHTING, STORAGE, SPHERICAL, false>(dm, va);
}

template <int WEIGHTING, int STORAGE, int SPHERICAL>
__global__ __launch_bounds__(64 * kWavesPerGroup, 4) void integrate_views_list_kernel(DeviceMap dm, ViewsArgs va)
{
    integrate_views_body<WEIGHTING, STORAGE, SPHERICAL, true>(dm, va);
}

// Arguments read from device memory (graph replays: the host rewrites them
// between replays through a captured copy).  The host replays the graph of the
// scheduling form the arguments select; each kernel also checks it and exits
// at once on a mismatch.
template <int WEIGHTING, int STORAGE, int SPHERICAL>
__global__ __launch_bounds__(64 * kWavesPerGroup, 4) void integrate_views_kernel_dev(DeviceMap dm,
                                                                                  const ViewsArgs *__restrict__ va)
{
    if (va->lat.cand)
        return;
    integrate_views_body<WEIGHTING, STORAGE, SPHERICAL, false>(dm, *va);
}

template <int WEIGHTING, int STORAGE, int SPHERICAL>
__global__ __launch_bounds__(64 * kWavesPerGroup, 4) void integrate_views_list_kernel_dev(
    DeviceMap dm, const ViewsArgs *__restrict__ va)
{
    if (!va->lat.cand)
        return;
    integrate_views_body<WEIGHTING, STORAGE, SPHERICAL, true>(dm, *va);
}

template <bool LANE_VIEWS>
__global__ __launch_bounds__(kCullThreads) void cull_views_kernel(DeviceMap dm, ViewsArgs va)
{
    cull_to_list<LANE_VIEWS>(dm, va.lat, va.cam, va.n_views, va.mc, va.parity);
}

template <bool LANE_VIEWS>
__global__ __launch_bounds__(kCullThreads) void cull_views_kernel_dev(DeviceMap dm, const ViewsArgs *__restrict__ va)
{
    if (!va->lat.cand)
        return;
    cull_to_list<LANE_VIEWS>(dm, va->lat, va->cam, va->n_views, va->mc, va->parity);
}

}  // namespace

bool views_share_model(const ViewsArgs &va)
{
    for (int v = 1; v < va.n_views; ++v)
        if (va.cam[v].model != va.cam[0].model)
            return false;
    return true;
}

hipError_t launch_cull_views(const DeviceMap &dm, const ViewsArgs &va, hipStream_t stream)
{
    const bool lane_views = views_share_model(va);
    const long long work = va.lat.n_lat * (lane_views ? cull_lanes_per_block(va.n_views) : 1);
    const unsigned groups = (unsigned)std::max<long long>(1, std::min<long long>((work + kCullThreads - 1) / kCullThreads,
                                                                                 kCullGroups));
    if (lane_views)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(cull_views_kernel<true>), dim3(groups), dim3(kCullThreads), 0, stream, dm, va);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(cull_views_kernel<false>), dim3(groups), dim3(kCullThreads), 0, stream, dm,
                           va);
    return hipGetLastError();
}

hipError_t launch_cull_views_dev(const DeviceMap &dm, const ViewsArgs *va_dev, int groups, bool lane_views,
                                 hipStream_t stream)
{
    if (lane_views)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(cull_views_kernel_dev<true>), dim3((unsigned)groups), dim3(kCullThreads), 0,
                           stream, dm, va_dev);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(cull_views_kernel_dev<false>), dim3((unsigned)groups), dim3(kCullThreads),
                           0, stream, dm, va_dev);
    return hipGetLastError();
}

template <int WEIGHTING, int SPHERICAL>
static void launch_views_storage(const DeviceMap &dm, const ViewsArgs &va, dim3 grid, dim3 block, hipStream_t stream)
{
    if (va.lat.cand) {
        if (dm.storage == 1)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_list_kernel<WEIGHTING, 1, SPHERICAL>), grid, block, 0,
                               stream, dm, va);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_list_kernel<WEIGHTING, 0, SPHERICAL>), grid, block, 0,
                               stream, dm, va);
    } else if (dm.storage == 1) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_kernel<WEIGHTING, 1, SPHERICAL>), grid, block, 0, stream,
                           dm, va);
    } else {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_kernel<WEIGHTING, 0, SPHERICAL>), grid, block, 0, stream,
                           dm, va);
    }
}

hipError_t launch_integrate_views(const DeviceMap &dm, const ViewsArgs &va, int weighting, int groups,
                                  hipStream_t stream)
{
    const dim3 grid((unsigned)groups), block(64 * kWavesPerGroup);
    bool spherical = false;
    for (int v = 0; v < va.n_views; ++v)
        spherical = spherical || va.cam[v].model == kModelSpherical;
    if (weighting == kWeightLearned) {
        if (spherical)
            return hipErrorInvalidValue;
        launch_views_storage<kWeightLearned, 0>(dm, va, grid, block, stream);
    } else if (weighting == kWeightDropoff) {
        if (spherical)
            launch_views_storage<kWeightDropoff, 1>(dm, va, grid, block, stream);
        else
            launch_views_storage<kWeightDropoff, 0>(dm, va, grid, block, stream);
    } else {
        if (spherical)
            launch_views_storage<kWeightConstant, 1>(dm, va, grid, block, stream);
        else
            launch_views_storage<kWeightConstant, 0>(dm, va, grid, block, stream);
    }
    return hipGetLastError();
}

// Both the walking and the list kernel (each returns at once unless the
// replay's arguments select it).
template <int WEIGHTING, int SPHERICAL>
static void launch_views_dev_storage(const DeviceMap &dm, const ViewsArgs *va, bool list, dim3 grid, dim3 block,
                                     hipStream_t stream)
{
    if (list) {
        if (dm.storage == 1)
            hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_list_kernel_dev<WEIGHTING, 1, SPHERICAL>), grid, block,
                               0, stream, dm, va);
        else
            hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_list_kernel_dev<WEIGHTING, 0, SPHERICAL>), grid, block,
                               0, stream, dm, va);
    } else if (dm.storage == 1) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_kernel_dev<WEIGHTING, 1, SPHERICAL>), grid, block, 0,
                           stream, dm, va);
    } else {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(integrate_views_kernel_dev<WEIGHTING, 0, SPHERICAL>), grid, block, 0,
                           stream, dm, va);
    }
}

hipError_t launch_integrate_views_dev(const DeviceMap &dm, const ViewsArgs *va_dev, bool spherical, int weighting,
                                      int groups, bool list, hipStream_t stream)
{
    const dim3 grid((unsigned)groups), block(64 * kWavesPerGroup);
    if (weighting == kWeightLearned)
        return hipErrorInvalidValue;
    if (weighting == kWeightDropoff) {
        if (spherical)
            launch_views_dev_storage<kWeightDropoff, 1>(dm, va_dev, list, grid, block, stream);
        else
            launch_views_dev_storage<kWeightDropoff, 0>(dm, va_dev, list, grid, block, stream);
    } else {
        if (spherical)
            launch_views_dev_storage<kWeightConstant, 1>(dm, va_dev, list, grid, block, stream);
        else
            launch_views_dev_storage<kWeightConstant, 0>(dm, va_dev, list, grid, block, stream);
    }
    return hipGetLastError();
}

}  // namespace tsdf

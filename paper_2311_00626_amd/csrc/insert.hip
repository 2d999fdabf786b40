// Re-insertion of saved blocks (restoring a map from a dump of query_blocks +
// query_tsdf): each block is found or inserted in the block hash exactly as
// integration inserts blocks (§IV-A: block index -> block of 8^3 voxels),
// and its 512 (distance, weight) pairs are written to its pool slot.
#include "device_common.hpp"

namespace tsdf {
namespace {

using namespace dev;

constexpr int kInsertWaves = 4;

// One wave per block (grid-stride).  Blocks outside the block-index range
// are skipped; a full pool or hash records the sticky overflow (as in
// integration) and the block is skipped.
template <int STORAGE>
__global__ __launch_bounds__(64 * kInsertWaves) void insert_blocks_kernel(DeviceMap dm,
                                                                          const int32_t *__restrict__ xyz,
                                                                          long long n,
                                                                          const float *__restrict__ dist,
                                                                          const float *__restrict__ weight)
{
    using IO = VoxelIO<STORAGE>;
    const int lane = lane_id();
    const long long stride = (long long)gridDim.x * kInsertWaves;
    for (long long b = (long long)blockIdx.x * kInsertWaves + (threadIdx.x >> 6); b < n; b += stride) {
        const int x = wave_bcast(xyz[3 * b]), y = wave_bcast(xyz[3 * b + 1]), z = wave_bcast(xyz[3 * b + 2]);
        if (!(x >= -kBlockCoordMax && x <= kBlockCoordMax && y >= -kBlockCoordMax && y <= kBlockCoordMax &&
              z >= -kBlockCoordMax && z <= kBlockCoordMax))
            continue;
        const unsigned long long key = pack_key(x, y, z);
        const uint32_t h = probe_start(key, dm.hash_mask);
        const uint32_t slot = find_or_insert(dm, key, h, load_first_window(dm, h));
        if (slot == kInvalidSlot)
            continue;
        const __amdgpu_buffer_rsrc_t blk = block_rsrc<STORAGE>(dm, slot);
        const float *d = dist + b * kBlockVoxels;
        const float *w = weight + b * kBlockVoxels;
#pragma unroll
        for (int s = 0; s < kBlockVoxels / 64; ++s) {
            const int k = 64 * s + lane;   // voxel lx + 8 ly + 64 lz, the pool's order
            IO::store(blk, IO::kBytes * (uint32_t)k, make_float2(d[k], w[k]));
        }
    }
}

}  // namespace

hipError_t launch_insert_blocks(const DeviceMap &dm, const int32_t *xyz, long long n, const float *dist,
                                const float *weight, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    const unsigned groups = (unsigned)std::max<long long>(1, std::min<long long>((n + kInsertWaves - 1) / kInsertWaves,
                                                                                  4096));
    if (dm.storage == 1)
        hipLaunchKernelGGL(insert_blocks_kernel<1>, dim3(groups), dim3(64 * kInsertWaves), 0, stream, dm, xyz, n,
                           dist, weight);
    else
        hipLaunchKernelGGL(insert_blocks_kernel<0>, dim3(groups), dim3(64 * kInsertWaves), 0, stream, dm, xyz, n,
                           dist, weight);
    return hipGetLastError();
}

}  // namespace tsdf

// Read-side kernels of the block map (voxel gathers by block index, key
// decoding, touched-list export, the key sort behind query_blocks) and the
// rehash that moves the block hash to a larger table.
#include "tsdf_internal.hpp"

#include <rocprim/device/device_radix_sort.hpp>

namespace tsdf {
namespace {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Read-only wave-cooperative probe: pool slot of `key`, or kInvalidSlot.
// Same probe order as the integration kernels: the key's 16-slot bucket,
// then 64-slot windows.
__device__ uint32_t find_block(const DeviceMap &dm, unsigned long long key)
{
    const int lane = lane_id();
    const uint32_t mask = dm.hash_mask;
    const uint32_t start = probe_start(key, mask);
    uint32_t width = kBucketSlots;
    for (uint32_t base = 0; base <= mask; base += width, width = 64) {
        const uint32_t pos = (start + base + (uint32_t)lane) & mask;
        const unsigned long long k = (uint32_t)lane < width ? dm.keys[pos] : kNoKey;
        const unsigned long long m_hit = __ballot(k == key);
        const unsigned long long m_free = __ballot(k == kEmptyKey);
        const int f_hit = m_hit ? __builtin_ctzll(m_hit) : 64;
        const int f_free = m_free ? __builtin_ctzll(m_free) : 64;
        if (f_hit < f_free)
            return dm.vals[(start + base + (uint32_t)f_hit) & mask];
        if (f_free < 64)
            return kInvalidSlot;
    }
    return kInvalidSlot;
}

__global__ __launch_bounds__(256) void query_tsdf_kernel(DeviceMap dm, const int32_t *__restrict__ xyz,
                                                         long long n, float *__restrict__ dist,
                                                         float *__restrict__ weight)
{
    const int lane = lane_id();
    const long long stride = (long long)gridDim.x * kQueryWavesPerGroup;
    for (long long b = (long long)blockIdx.x * kQueryWavesPerGroup + (threadIdx.x >> 6); b < n; b += stride) {
        const int x = xyz[3 * b], y = xyz[3 * b + 1], z = xyz[3 * b + 2];
        const bool in_range = x >= -kBlockCoordMax && x <= kBlockCoordMax && y >= -kBlockCoordMax &&
                              y <= kBlockCoordMax && z >= -kBlockCoordMax && z <= kBlockCoordMax;
        uint32_t slot = kInvalidSlot;
        if (in_range)
            slot = find_block(dm, pack_key(x, y, z));
        if (slot >= dm.block_cap)
            slot = kInvalidSlot;
        float *d = dist + b * kBlockVoxels;
        float *w = weight + b * kBlockVoxels;
        for (int k = lane; k < kBlockVoxels; k += 64) {
            float2 v = make_float2(0.0f, 0.0f);
            if (slot != kInvalidSlot) {
                const size_t at = (size_t)slot * kBlockVoxels + k;
                if (dm.storage == 1) {
                    const _Float16 *p = (const _Float16 *)dm.pool + 2 * at;
                    v = make_float2((float)p[0], (float)p[1]);
                } else {
                    v = ((const float2 *)dm.pool)[at];
                }
            }
            d[k] = v.x;
            w[k] = v.y;
        }
    }
}

// Decodes sorted keys into block indices; empty keys (pool slots reserved
// but never published) sort last and are skipped.
__global__ void decode_keys_kernel(const unsigned long long *__restrict__ keys, long long n,
                                   int32_t *__restrict__ xyz)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const unsigned long long k = keys[i];
        if (k == kEmptyKey)
            continue;
        int x, y, z;
        unpack_key(k, x, y, z);
        xyz[3 * i] = x;
        xyz[3 * i + 1] = y;
        xyz[3 * i + 2] = z;
    }
}

// Number of published keys among n ascending keys: the position of the first
// empty key.  Exactly one thread writes it (the last published key, or the
// first entry when every key is empty).
__global__ void count_valid_kernel(const unsigned long long *__restrict__ keys, long long n,
                                   unsigned long long *__restrict__ count)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const bool here = keys[i] != kEmptyKey;
        const bool next = i + 1 < n && keys[i + 1] != kEmptyKey;
        if (here && !next)
            *count = (unsigned long long)(i + 1);
        else if (i == 0 && !here)
            *count = 0ull;
    }
}

// Re-inserts the key of every pool slot below n into an empty table (linear
// probing from the key's probe start, the order the wave-cooperative probes
// scan):
// the pool slot becomes the key's value.  Slots that hold no key are skipped.
// Keys of distinct pool slots are distinct, so every insert claims a new slot;
// the table has more slots than keys, so every probe ends.
__global__ void rehash_kernel(const unsigned long long *__restrict__ slot_keys, uint32_t n,
                              unsigned long long *__restrict__ keys, uint32_t *__restrict__ vals, uint32_t mask)
{
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n; s += gridDim.x * blockDim.x) {
        const unsigned long long key = slot_keys[s];
        if (key == kEmptyKey)
            continue;
        uint32_t pos = probe_start(key, mask);
        for (uint32_t probe = 0; probe <= mask; ++probe, pos = (pos + 1u) & mask) {
            if (atomicCAS(&keys[pos], kEmptyKey, key) == kEmptyKey) {
                vals[pos] = s;
                break;
            }
        }
    }
}

__global__ void gather_touched_kernel(DeviceMap dm, int sub, long long n, int32_t *__restrict__ xyz)
{
    const uint32_t *list = dm.touched + (size_t)sub * dm.block_cap;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        int x, y, z;
        unpack_key(dm.slot_keys[list[i]], x, y, z);
        xyz[3 * i] = x;
        xyz[3 * i + 1] = y;
        xyz[3 * i + 2] = z;
    }
}

int grid_for(long long n, int per_group)
{
    long long g = (n + per_group - 1) / per_group;
    if (g < 1)
        g = 1;
    if (g > 16384)
        g = 16384;
    return (int)g;
}

}  // namespace

hipError_t launch_query_tsdf(const DeviceMap &dm, const int32_t *xyz, long long n, float *dist,
                             float *weight, hipStream_t stream)
{
    hipLaunchKernelGGL(query_tsdf_kernel, dim3(grid_for(n, kQueryWavesPerGroup)), dim3(64 * kQueryWavesPerGroup), 0,
                       stream, dm, xyz, n, dist, weight);
    return hipGetLastError();
}

hipError_t launch_decode_keys(const unsigned long long *keys, long long n, int32_t *xyz, hipStream_t stream)
{
    hipLaunchKernelGGL(decode_keys_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, keys, n, xyz);
    return hipGetLastError();
}

hipError_t launch_gather_touched(const DeviceMap &dm, int sub, long long n, int32_t *xyz, hipStream_t stream)
{
    hipLaunchKernelGGL(gather_touched_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, dm, sub, n, xyz);
    return hipGetLastError();
}

hipError_t launch_count_valid(const unsigned long long *keys, long long n, unsigned long long *count,
                              hipStream_t stream)
{
    hipLaunchKernelGGL(count_valid_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, keys, n, count);
    return hipGetLastError();
}

hipError_t launch_rehash(const unsigned long long *slot_keys, uint32_t n, unsigned long long *keys, uint32_t *vals,
                         uint32_t mask, hipStream_t stream)
{
    hipLaunchKernelGGL(rehash_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, slot_keys, n, keys, vals, mask);
    return hipGetLastError();
}

// Ascending radix sort of packed keys; the packing puts x in the high bits, so
// the order is lexicographic in (x, y, z).  With temp == nullptr only sets
// *temp_bytes to the work space that n keys need.  Only enqueues work.
hipError_t sort_keys(const unsigned long long *in, unsigned long long *out, long long n, void *temp,
                     size_t *temp_bytes, hipStream_t stream)
{
    return rocprim::radix_sort_keys(temp, *temp_bytes, in, out, (size_t)n, 0, 64, stream);
}

}  // namespace tsdf

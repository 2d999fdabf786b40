// Depth footprint pyramids: a conservative filter on the candidate blocks of
// projective integration (§IV-B).  A voxel is updated only where its pixel
// holds a valid measurement d and its depth is at most d + epsilon, so a block
// whose nearest point lies farther than the largest valid measurement under
// its image footprint, plus epsilon, holds no updated voxel.  The pyramid
// stores that largest measurement for every tile of 8, 16, 32 and 64 pixels,
// so that a footprint of any size up to a few hundred pixels is covered by at
// most 3 x 3 tiles of one level.
//
// One workgroup of 256 threads reduces one 64 x 64 pixel super-tile: each
// thread takes a 4 x 4 patch (rows of 64 contiguous floats per 16 threads),
// and the four levels follow by 2 x 2 reductions in LDS.  Workgroups stride
// over the super-tiles of all views of the launch.
#include "device_common.hpp"

namespace tsdf {
namespace {

using namespace dev;

constexpr int kThreads = 256;

__device__ __forceinline__ float valid_or_zero(float d, float d_max)
{
    return (d > 0.0f && d <= d_max) ? d : 0.0f;   // NaN and +inf fail
}

__device__ void build_pyramids(const ViewsArgs &va)
{
    __shared__ float s4[16][17];
    __shared__ float s8[8][9];
    __shared__ float s16[4][4];
    __shared__ float s32[2][2];

    const int t = (int)threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    uint32_t first[kMaxViews + 1];
    first[0] = 0;
    for (int v = 0; v < va.n_views; ++v) {
        const CameraView &cv = va.cam[v];
        const uint32_t n = cv.tiles ? (uint32_t)((cv.width + kTileSuper - 1) / kTileSuper) *
                                          (uint32_t)((cv.height + kTileSuper - 1) / kTileSuper)
                                    : 0u;
        first[v + 1] = first[v] + n;
    }
    const uint32_t total = first[va.n_views];
    for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
        int v = 0;
        while (item >= first[v + 1])
            ++v;
        const CameraView &cv = va.cam[v];
        const uint32_t k = item - first[v];
        const uint32_t sup_cols = (uint32_t)((cv.width + kTileSuper - 1) / kTileSuper);
        const int sx = (int)(k % sup_cols), sy = (int)(k / sup_cols);
        const int x0 = kTileSuper * sx + 4 * tx, y0 = kTileSuper * sy + 4 * ty;

        // pixels beyond the image edge read through an out-of-range offset
        // (value 0, which the maximum ignores): no branch, all 16 loads in flight
        const __amdgpu_buffer_rsrc_t img = make_rsrc(cv.depth, 4u * (uint32_t)cv.width * (uint32_t)cv.height);
        float px[16];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int y = y0 + r, x = x0 + c;
                const uint32_t off =
                    (y < cv.height && x < cv.width) ? 4u * (uint32_t)(y * cv.width + x) : kOutOfRange;
                px[4 * r + c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, off, 0, 0));
            }
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            m = fmaxf(m, valid_or_zero(px[k], cv.d_max));
        s4[ty][tx] = m;
        __syncthreads();
        if (t < 64) {
            const int i = t & 7, j = t >> 3;
            const float m8 = fmaxf(fmaxf(s4[2 * j][2 * i], s4[2 * j][2 * i + 1]),
                                   fmaxf(s4[2 * j + 1][2 * i], s4[2 * j + 1][2 * i + 1]));
            s8[j][i] = m8;
            const int c = 8 * sx + i, r = 8 * sy + j;
            if (c < cv.tile_cols[0] && r < cv.tile_rows[0])
                cv.tiles[cv.tile_off[0] + r * cv.tile_cols[0] + c] = m8;
        }
        __syncthreads();
        if (t < 16) {
            const int i = t & 3, j = t >> 2;
            const float m16 = fmaxf(fmaxf(s8[2 * j][2 * i], s8[2 * j][2 * i + 1]),
                                    fmaxf(s8[2 * j + 1][2 * i], s8[2 * j + 1][2 * i + 1]));
            s16[j][i] = m16;
            const int c = 4 * sx + i, r = 4 * sy + j;
            if (c < cv.tile_cols[1] && r < cv.tile_rows[1])
                cv.tiles[cv.tile_off[1] + r * cv.tile_cols[1] + c] = m16;
        }
        __syncthreads();
        if (t < 4) {
            const int i = t & 1, j = t >> 1;
            const float m32 = fmaxf(fmaxf(s16[2 * j][2 * i], s16[2 * j][2 * i + 1]),
                                    fmaxf(s16[2 * j + 1][2 * i], s16[2 * j + 1][2 * i + 1]));
            s32[j][i] = m32;
            const int c = 2 * sx + i, r = 2 * sy + j;
            if (c < cv.tile_cols[2] && r < cv.tile_rows[2])
                cv.tiles[cv.tile_off[2] + r * cv.tile_cols[2] + c] = m32;
        }
        __syncthreads();
        if (t == 0) {
            const float m64 = fmaxf(fmaxf(s32[0][0], s32[0][1]), fmaxf(s32[1][0], s32[1][1]));
            cv.tiles[cv.tile_off[3] + sy * cv.tile_cols[3] + sx] = m64;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void footprint_tiles_kernel(ViewsArgs va)
{
    build_pyramids(va);
}

__global__ __launch_bounds__(kThreads) void footprint_tiles_kernel_dev(const ViewsArgs *__restrict__ va)
{
    build_pyramids(*va);
}

}  // namespace

hipError_t launch_footprint_tiles(const ViewsArgs &va, hipStream_t stream)
{
    long long total = 0;
    for (int v = 0; v < va.n_views; ++v)
        if (va.cam[v].tiles)
            total += (long long)((va.cam[v].width + kTileSuper - 1) / kTileSuper) *
                     ((va.cam[v].height + kTileSuper - 1) / kTileSuper);
    if (total == 0)
        return hipSuccess;
    const unsigned groups = (unsigned)std::min<long long>(total, 1024);
    hipLaunchKernelGGL(footprint_tiles_kernel, dim3(groups), dim3(kThreads), 0, stream, va);
    return hipGetLastError();
}

// Graph replays: the views are read from device memory, the grid is fixed.
hipError_t launch_footprint_tiles_dev(const ViewsArgs *va_dev, hipStream_t stream)
{
    hipLaunchKernelGGL(footprint_tiles_kernel_dev, dim3(512), dim3(kThreads), 0, stream, va_dev);
    return hipGetLastError();
}

}  // namespace tsdf

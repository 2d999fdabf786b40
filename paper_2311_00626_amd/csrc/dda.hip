// Paper-literal allocation (§IV-B: the blocks in view are found by ray
// tracing through the block grid, Amanatides & Woo).  One thread per pixel:
// for a valid measurement d, the ray from the camera centre through the pixel
// centre is walked through the grid of blocks (edge 8 vs) from depth 0 to
// min(d + epsilon, max range) (depth along the optical axis; the direction has
// unit camera z); every block entered is marked in a byte map over the
// frame's block lattice, which the integration kernel then takes as its
// candidate set (and allocates in full), clearing every mark it reads.  Ties step x, then y, then z; a
// boundary exactly at the end depth is crossed.  The binary32 operations and
// their order are fixed so that the visited set is reproducible exactly.
#include "device_common.hpp"

namespace tsdf {
namespace {

__global__ __launch_bounds__(256) void fill_u8_kernel(unsigned char *p, long long n)
{
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256)
        p[k] = 0;
}

__global__ __launch_bounds__(256) void dda_mark_kernel(DdaArgs a)
{
    const long long n = (long long)a.width * a.height;
    const float B = 8.0f * a.vs;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const float d = a.depth[p];
        if (!(d > 0.0f && d <= a.d_max))
            continue;
        const int j = (int)(p / a.width), i = (int)(p - (long long)j * a.width);
        const float u = (((float)i + 0.5f) - a.cx) / a.fx;
        const float v = (((float)j + 0.5f) - a.cy) / a.fy;
        float te = d + a.eps;
        if (!(te <= a.d_max))
            te = a.d_max;
        float dir[3], tmax[3], tdel[3];
        int c[3], step[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            dir[k] = (a.Rwc[3 * k] * u + a.Rwc[3 * k + 1] * v) + a.Rwc[3 * k + 2];
            c[k] = (int)floorf(a.o[k] / B);
            if (dir[k] > 0.0f) {
                step[k] = 1;
                tmax[k] = ((float)(c[k] + 1) * B - a.o[k]) / dir[k];
                tdel[k] = B / dir[k];
            } else if (dir[k] < 0.0f) {
                step[k] = -1;
                tmax[k] = ((float)c[k] * B - a.o[k]) / dir[k];
                tdel[k] = B / -dir[k];
            } else {
                step[k] = 0;
                tmax[k] = __builtin_inff();
                tdel[k] = __builtin_inff();
            }
        }
        // lattice offsets as unsigned 32-bit values: a block below the lattice
        // wraps to a large offset, so one compare per axis tests both ends; the
        // lattice holds fewer than 2^31 entries, so the entry index fits too
        const uint32_t dim_x = (uint32_t)a.lat.lat_dim[0], dim_y = (uint32_t)a.lat.lat_dim[1],
                       dim_z = (uint32_t)a.lat.lat_dim[2];
        for (int it = 0; it < (1 << 16); ++it) {
            const uint32_t x = (uint32_t)(c[0] - a.lat.lat_min[0]);
            const uint32_t y = (uint32_t)(c[1] - a.lat.lat_min[1]);
            const uint32_t z = (uint32_t)(c[2] - a.lat.lat_min[2]);
            if (x < dim_x && y < dim_y && z < dim_z)
                a.marks[x + dim_x * (y + dim_y * z)] = 1;
            else
                atomicOr(a.overflow, (uint32_t)kErrWalkOutside);
            const int ax = (tmax[0] <= tmax[1] && tmax[0] <= tmax[2]) ? 0 : (tmax[1] <= tmax[2] ? 1 : 2);
            if (!(tmax[ax] <= te))
                break;
            c[ax] += step[ax];
            tmax[ax] += tdel[ax];
        }
    }
}

}  // namespace

hipError_t launch_fill_u8(unsigned char *p, long long n, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    const unsigned groups = (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(fill_u8_kernel, dim3(groups), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_dda_mark(const DdaArgs &a, hipStream_t stream)
{
    const long long n = (long long)a.width * a.height;
    const unsigned groups = (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(dda_mark_kernel, dim3(groups), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace tsdf

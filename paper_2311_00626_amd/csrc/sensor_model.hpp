// Launch arguments of the learned-sensor-model kernels (sensor_model.hip).
#pragma once

#include "tsdf_internal.hpp"

namespace tsdf {

constexpr int kSmMaxFrames = 16;   // frames per training window

// One pinhole depth image (device memory) and its intrinsics.
struct SmView {
    const float *depth;
    int width, height;
    float fx, fy, cx, cy;
    float d_max;
};

// One frame of a training window.
struct SmFrame {
    float R[9], t[3];          // camera-from-world, as for integration
    const float *depth;        // H x W
    const float2 *maps;        // per-pixel (weight, truncation)
    float *gw, *ge;            // dL/dw, dL/deps per pixel (accumulated)
};

struct SmLossArgs {
    SmFrame frames[kSmMaxFrames];
    int n_frames;
    int width, height;
    float fx, fy, cx, cy, d_max, vs;
    long long n_vox;
    const int *vox;            // 3 global voxel indices per target voxel
    const float *target;       // target distance per voxel
    double *acc;               // [0] sum of squared errors, [1] voxels reached
};

struct SmBackArgs {
    SmView views[kSmMaxFrames];
    int n_frames;
    int width, height;
    float vs;
    const float *params;
    const float *gw, *ge;      // frame-major, n_frames x H x W
    const double *acc;
    float *grad;               // kSmParams, accumulated
};

hipError_t launch_sm_maps(const SmView &v, float vs, const float *params, float2 *out, hipStream_t stream);
// The same maps from the matrix-core forward pass that training differentiates.
hipError_t launch_sm_maps_mfma(const SmView &v, float vs, const float *params, float2 *out, hipStream_t stream);
hipError_t launch_sm_fill(float *p, long long n, float value, hipStream_t stream);
hipError_t launch_sm_loss(const SmLossArgs &a, hipStream_t stream);
hipError_t launch_sm_backward(const SmBackArgs &a, hipStream_t stream);
hipError_t launch_sm_adam(float *master, float *m1, float *m2, const float *grad, float *params, int n, float lr,
                          float beta1, float beta2, float eps, int step, hipStream_t stream);

}  // namespace tsdf

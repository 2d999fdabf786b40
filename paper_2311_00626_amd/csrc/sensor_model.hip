// Learned sensor model: per-pixel measurement weight and truncation distance
// from a 27 -> 32 -> 32 -> 2 perceptron on the pixel's depth neighbourhood,
// in place of a fixed weighting function (§IV-B lets the weight follow the
// sensor's error model).
//
// Inputs of pixel (i, j) with valid depth d: the 5 x 5 patch of differences
// q - d clipped to [-0.5, 0.5] m (0 outside the image or for invalid q), d,
// and the incidence angle between the pixel's ray and the normal of the
// back-projected depth (central differences; pi/2 without all 4 neighbours).
// Outputs o: weight w = (o0 + sqrt(o0^2 + 4)) / 2 and truncation
// eps = vs (1 + 7 s) with s = (1 + o1 / sqrt(1 + o1^2)) / 2.
//
// Inference for integration (sm_maps_kernel) rounds inputs and hidden
// activations to bfloat16 and accumulates every dot product in binary32, one
// fused multiply-add per term in index order from the bias; with parameters
// that are bfloat16 values this reproduces the CPU reference bit for bit.
//
// Training runs the same perceptron on the matrix cores
// (v_mfma_f32_16x16x32_bf16: bfloat16 inputs, weights and activations,
// binary32 accumulation in the matrix core's own order): the loss's maps
// (sm_maps_mfma_kernel) and the backward's recomputation of the forward pass
// are one function, so the gradient is exactly that of the loss evaluated.
// It differs from the inference function only in the rounding of the sums.
//
// Training computes the gradient of
//   L = (1/N) sum_v (D(v) - D*(v))^2,  D(v) = sum_f w_f x_f / sum_f w_f,
// over target voxels v of a window of frames (x_f = min(d_p, eps_f) of the
// pixel frame f projects v into): sm_fuse_loss_kernel evaluates D(v) and
// scatters dL/dw and dL/deps onto the pixels, sm_backward_kernel
// back-propagates them through the perceptron and reduces the parameter
// gradient over 64-pixel tiles staged in LDS, and sm_adam_kernel updates a
// binary32 master copy and its bfloat16 rounding.
#include "device_common.hpp"

#include "sensor_model.hpp"

namespace tsdf {
namespace {

using namespace dev;

// Round to the nearest bfloat16, ties to even (gfx950's v_cvt_pk_bf16_f32;
// infinities stay infinite, binary32 values beyond the bfloat16 range round
// to infinity, as in the bit-level definition).
__device__ __forceinline__ float round_bf16(float x)
{
    return (float)(__bf16)x;
}

__device__ __forceinline__ bool sm_valid(float d, float d_max) { return d > 0.0f && d <= d_max; }

// Depth of pixel (i, j) through a buffer descriptor over the image: outside
// the image the offset is out of range and the load returns 0, an invalid
// depth, so every gather is issued without a branch and all of a pixel's
// gathers are in flight together.
__device__ __forceinline__ uint32_t sm_off(const SmView &v, int i, int j)
{
    return (i >= 0 && i < v.width && j >= 0 && j < v.height) ? 4u * (uint32_t)(j * v.width + i) : kOutOfRange;
}

__device__ __forceinline__ float sm_load(__amdgpu_buffer_rsrc_t img, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(img, off, 0, 0));
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t sm_image(const SmView &v)
{
    return make_rsrc(v.depth, 4u * (uint32_t)v.width * (uint32_t)v.height);
}

// pi/2 unless all 4 neighbours (left, right, up, down) are valid (a pixel on
// the image border has a neighbour outside, which reads as invalid)
__device__ float sm_incidence_of(const SmView &v, int i, int j, float d, float dl, float dr, float du, float dd)
{
    const float half_pi = 1.57079637f;
    if (!(sm_valid(dl, v.d_max) && sm_valid(dr, v.d_max) && sm_valid(du, v.d_max) && sm_valid(dd, v.d_max)))
        return half_pi;
    const float rxl = (((float)(i - 1) + 0.5f) - v.cx) / v.fx, rxc = (((float)i + 0.5f) - v.cx) / v.fx;
    const float rxr = (((float)(i + 1) + 0.5f) - v.cx) / v.fx;
    const float ryu = (((float)(j - 1) + 0.5f) - v.cy) / v.fy, ryc = (((float)j + 0.5f) - v.cy) / v.fy;
    const float ryd = (((float)(j + 1) + 0.5f) - v.cy) / v.fy;
    const float ax = dr * rxr - dl * rxl, ay = dr * ryc - dl * ryc, az = dr - dl;
    const float bx = dd * rxc - du * rxc, by = dd * ryd - du * ryu, bz = dd - du;
    const float nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const float px = d * rxc, py = d * ryc, pz = d;
    const float dot = (nx * px + ny * py) + nz * pz;
    const float cx = ny * pz - nz * py, cy = nz * px - nx * pz, cz = nx * py - ny * px;
    const float cr = sqrtf((cx * cx + cy * cy) + cz * cz);
    return atan2_as(cr, fabsf(dot));
}

__device__ float sm_incidence(const SmView &v, __amdgpu_buffer_rsrc_t img, int i, int j, float d)
{
    const float dl = sm_load(img, sm_off(v, i - 1, j)), dr = sm_load(img, sm_off(v, i + 1, j));
    const float du = sm_load(img, sm_off(v, i, j - 1)), dd = sm_load(img, sm_off(v, i, j + 1));
    return sm_incidence_of(v, i, j, d, dl, dr, du, dd);
}

// The 27 inputs, already rounded to bfloat16.
__device__ __forceinline__ void sm_inputs(const SmView &v, int i, int j, float d, float x[kSmIn])
{
    const __amdgpu_buffer_rsrc_t img = sm_image(v);
    float dq[25];
#pragma unroll
    for (int dj = -2; dj <= 2; ++dj)
#pragma unroll
        for (int di = -2; di <= 2; ++di)
            dq[(dj + 2) * 5 + (di + 2)] = sm_load(img, sm_off(v, i + di, j + dj));
#pragma unroll
    for (int k = 0; k < 25; ++k) {
        float q = 0.0f;
        if (sm_valid(dq[k], v.d_max)) {
            q = dq[k] - d;
            q = q < -0.5f ? -0.5f : (q > 0.5f ? 0.5f : q);
        }
        x[k] = round_bf16(q);
    }
    x[25] = round_bf16(d);
    x[26] = round_bf16(sm_incidence(v, img, i, j, d));
}

// The parameter buffer seen through the constant address space: a kernel that
// never writes it reads it with scalar loads even where a barrier stands
// between the loads and the kernel's start.
typedef const __attribute__((address_space(4))) float *ConstParams;

__device__ __forceinline__ ConstParams as_constant(const float *p)
{
    return (ConstParams)p;
}

// Forward through the hidden layers with parameters P (binary32 multiply-adds
// in index order from the bias; hidden activations rounded to bfloat16), to
// the binary32 outputs o.  Layer 2 takes the first layer's units four at a
// time as they are computed: each second-layer sum still adds its terms in
// index order, so the result is that of evaluating the layers one after the
// other, with 4 instead of 32 first-layer activations held in registers.
template <typename Params>
__device__ __forceinline__ void sm_forward(Params P, const float x[kSmIn], float o[kSmOut])
{
    float h2[kSmHidden];
#pragma unroll
    for (int k = 0; k < kSmHidden; ++k)
        h2[k] = P[kSmB2 + k];
#pragma unroll 1
    for (int m0 = 0; m0 < kSmHidden; m0 += 4) {
        float h1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float a = P[kSmB1 + m0 + q];
#pragma unroll
            for (int i = 0; i < kSmIn; ++i)
                a = __builtin_fmaf(P[kSmW1 + kSmIn * (m0 + q) + i], x[i], a);
            h1[q] = round_bf16(a > 0.0f ? a : 0.0f);
        }
#pragma unroll
        for (int k = 0; k < kSmHidden; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                h2[k] = __builtin_fmaf(P[kSmW2 + kSmHidden * k + m0 + q], h1[q], h2[k]);
    }
#pragma unroll
    for (int k = 0; k < kSmHidden; ++k)
        h2[k] = round_bf16(h2[k] > 0.0f ? h2[k] : 0.0f);
#pragma unroll
    for (int c = 0; c < kSmOut; ++c) {
        float a = P[kSmB3 + c];
#pragma unroll
        for (int m = 0; m < kSmHidden; ++m)
            a = __builtin_fmaf(P[kSmW3 + kSmHidden * c + m], h2[m], a);
        o[c] = a;
    }
}

// ---- forward pass on the matrix cores ----------------------------------
//
// v_mfma_f32_16x16x32_bf16 computes D = A B + C for A 16 x 32 and B 32 x 16
// (bfloat16) and C, D 16 x 16 (binary32).  Lane l (g = l / 16, m = l mod 16)
// supplies A[m][8 g + j] and B[8 g + j][m] (j = 0..7) and holds D[4 g + i][m]
// (i = 0..3).  The layers are evaluated transposed, units along M and pixels
// along N: a 16-pixel sub-tile is one column block, H^T = W X^T + b.  A
// layer's output then sits where the next layer's B operand needs it: lane
// (g, m) holds units 4 g + i of each half of the previous layer for pixel m,
// so the next layer's K slots 8 g + j of lane group g are taken to be the
// units {4 g .. 4 g + 3, 16 + 4 g .. 16 + 4 g + 3}, and the weights are
// loaded in that order (a dot product's terms may come in any order).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Hidden unit behind K slot 8 g + j of layers 2 and 3.
__device__ __forceinline__ int sm_slot_unit(int g, int j)
{
    return j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4);
}

// The perceptron's parameters as this lane's operands (once per wave).  The
// weights are bfloat16 values (the parameter format), so the conversions
// are exact; biases enter the accumulators in binary32.
struct SmOperands {
    bf16x8 w1[2], w2[2], w3;   // A operands of layer 1 and 2 (two 16-unit halves) and layer 3
    f32x4 b1[2], b2[2], b3;    // accumulator start values
};

template <typename Params>
__device__ __forceinline__ SmOperands sm_operands(Params P)
{
    const int l = lane_id(), g = l >> 4, m = l & 15;
    SmOperands W;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int unit = 16 * h + m;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            W.w1[h][j] = (__bf16)(k < kSmIn ? P[kSmW1 + kSmIn * unit + (k < kSmIn ? k : 0)] : 0.0f);
            W.w2[h][j] = (__bf16)P[kSmW2 + kSmHidden * unit + sm_slot_unit(g, j)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            W.b1[h][i] = P[kSmB1 + 16 * h + 4 * g + i];
            W.b2[h][i] = P[kSmB2 + 16 * h + 4 * g + i];
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
        W.w3[j] = (__bf16)(m < kSmOut ? P[kSmW3 + kSmHidden * (m < kSmOut ? m : 0) + sm_slot_unit(g, j)] : 0.0f);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        W.b3[i] = g == 0 && i < kSmOut ? P[kSmB3 + (i < kSmOut ? i : 0)] : 0.0f;
    return W;
}

__device__ __forceinline__ f32x4 relu_bf16(f32x4 a)
{
    f32x4 h;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        h[i] = round_bf16(a[i] > 0.0f ? a[i] : 0.0f);
    return h;
}

__device__ __forceinline__ bf16x8 sm_pack(const f32x4 h[2])
{
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        b[i] = (__bf16)h[0][i];       // exact: already bfloat16 values
        b[4 + i] = (__bf16)h[1][i];
    }
    return b;
}

// Forward pass of one 16-pixel sub-tile: x holds inputs 8 g .. 8 g + 7 of
// pixel m (bfloat16, zero beyond the 27th).  h1[h][i], h2[h][i]: the bfloat16
// activations of unit 16 h + 4 g + i for pixel m; o[0], o[1] (lane group 0):
// the pixel's binary32 outputs.  Every call with the same operands gives the
// same results, so inference and the training backward evaluate one function.
__device__ __forceinline__ void sm_forward_tile(const SmOperands &W, bf16x8 x, f32x4 h1[2], f32x4 h2[2], f32x4 &o)
{
#pragma unroll
    for (int h = 0; h < 2; ++h)
        h1[h] = relu_bf16(__builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w1[h], x, W.b1[h], 0, 0, 0));
    const bf16x8 a1 = sm_pack(h1);
#pragma unroll
    for (int h = 0; h < 2; ++h)
        h2[h] = relu_bf16(__builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w2[h], a1, W.b2[h], 0, 0, 0));
    const bf16x8 a2 = sm_pack(h2);
    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.w3, a2, W.b3, 0, 0, 0);
}

__device__ __forceinline__ float2 sm_outputs(const float o[kSmOut], float vs)
{
    const float w = 0.5f * (o[0] + sqrtf(o[0] * o[0] + 4.0f));
    const float s = 0.5f + 0.5f * (o[1] / sqrtf(1.0f + o[1] * o[1]));
    return make_float2(w, vs * (1.0f + 7.0f * s));
}

constexpr int kMapThreads = 256;

// Inference: one pixel per thread.  The parameters are read straight from the
// (read-only) parameter buffer: every lane of a wave reads the same one, so
// they arrive through scalar loads and feed the multiply-adds as scalar
// operands, leaving the LDS port free.
__global__ __launch_bounds__(kMapThreads) void sm_maps_kernel(SmView v, float vs, const float *__restrict__ params,
                                                              float2 *__restrict__ out)
{
    const float *__restrict__ P = params;
    const int n = v.width * v.height;
    for (int p = (int)(blockIdx.x * kMapThreads + threadIdx.x); p < n; p += (int)(gridDim.x * kMapThreads)) {
        const int j = p / v.width, i = p - j * v.width;
        const float d = v.depth[p];
        if (!sm_valid(d, v.d_max)) {
            out[p] = make_float2(0.0f, 0.0f);
            continue;
        }
        float x[kSmIn], o[kSmOut];
        sm_inputs(v, i, j, d, x);
        sm_forward(P, x, o);
        out[p] = sm_outputs(o, vs);
    }
}

// Training maps on the matrix cores.  A wave takes 64 pixels, one per lane,
// gathers their inputs (sm_inputs, as the backward does), stages them in its
// LDS tile, and runs the forward pass as four 16-pixel sub-tiles of five
// MFMAs, building each sub-tile's operands from the tile exactly as the
// backward's recomputation does (so the two agree bit for bit); lane group 0
// writes the pixels' (weight, truncation).  Invalid pixels get (0, 0).
__global__ __launch_bounds__(kMapThreads) void sm_maps_mfma_kernel(SmView v, float vs,
                                                                   const float *__restrict__ params,
                                                                   float2 *__restrict__ out)
{
    constexpr int kWaves = kMapThreads / 64;
    __shared__ float X[kWaves][64][kSmIn + 1];   // column kSmIn: 1 for a valid pixel
    const SmOperands W = sm_operands(as_constant(params));
    const int lane = lane_id(), wave = (int)(threadIdx.x >> 6), g = lane >> 4, m = lane & 15;
    float(*Xw)[kSmIn + 1] = X[wave];
    const long long n = (long long)v.width * v.height;
    const long long n_tiles = (n + 63) / 64;
    const long long waves = (long long)gridDim.x * kWaves;
    for (long long tile = (long long)blockIdx.x * kWaves + wave; tile < n_tiles; tile += waves) {
        const long long p = tile * 64 + lane;
        float x[kSmIn];
        bool valid = false;
        if (p < n) {
            const float d = v.depth[p];
            if (sm_valid(d, v.d_max)) {
                const int j = (int)(p / v.width), i = (int)(p - (long long)j * v.width);
                sm_inputs(v, i, j, d, x);
                valid = true;
            }
        }
        if (!valid) {
#pragma unroll
            for (int k = 0; k < kSmIn; ++k)
                x[k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < kSmIn; ++k)
            Xw[lane][k] = x[k];
        Xw[lane][kSmIn] = valid ? 1.0f : 0.0f;
        // the wave's own LDS writes are read back by other lanes of the wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int t = 16 * st + m;
            bf16x8 xb;
#pragma unroll
            for (int jj = 0; jj < 8; ++jj)
                xb[jj] = (__bf16)(8 * g + jj < kSmIn ? Xw[t][8 * g + jj < kSmIn ? 8 * g + jj : 0] : 0.0f);
            f32x4 h1[2], h2[2], o;
            sm_forward_tile(W, xb, h1, h2, o);
            const long long q = tile * 64 + t;
            if (g == 0 && q < n) {
                const float ov[kSmOut] = {o[0], o[1]};
                out[q] = Xw[t][kSmIn] != 0.0f ? sm_outputs(ov, vs) : make_float2(0.0f, 0.0f);
            }
        }
        // the tile's reads are complete before the next pass rewrites it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---- training ------------------------------------------------------------

constexpr int kLossThreads = 256;

__global__ __launch_bounds__(kLossThreads) void sm_fuse_loss_kernel(SmLossArgs a)
{
    __shared__ double red[2][kLossThreads / 64];
    double loss = 0.0, used = 0.0;
    const long long stride = (long long)gridDim.x * kLossThreads;
    const uint32_t wh = (uint32_t)a.width * (uint32_t)a.height;
    for (long long v = (long long)blockIdx.x * kLossThreads + threadIdx.x; v < a.n_vox; v += stride) {
        const float px = ((float)a.vox[3 * v] + 0.5f) * a.vs;
        const float py = ((float)a.vox[3 * v + 1] + 0.5f) * a.vs;
        const float pz = ((float)a.vox[3 * v + 2] + 0.5f) * a.vs;
        // Every frame of the window at once: the pixel offsets first, then all
        // depth and map gathers together (an offset out of range for a frame the
        // voxel does not project into, or past the window, reads zeros, which
        // fail the validity tests), then the contributions in frame order.
        uint32_t off[kSmMaxFrames];
        float zc[kSmMaxFrames];
#pragma unroll
        for (int f = 0; f < kSmMaxFrames; ++f) {
            const SmFrame &fr = a.frames[f];
            const float xc = ((fr.R[0] * px + fr.R[1] * py) + fr.R[2] * pz) + fr.t[0];
            const float yc = ((fr.R[3] * px + fr.R[4] * py) + fr.R[5] * pz) + fr.t[1];
            zc[f] = ((fr.R[6] * px + fr.R[7] * py) + fr.R[8] * pz) + fr.t[2];
            const float r = 1.0f / zc[f];
            const float u = a.fx * (xc * r) + a.cx;
            const float w_ = a.fy * (yc * r) + a.cy;
            const bool in = f < a.n_frames && zc[f] > 0.0f && u >= 0.0f && u < (float)a.width && w_ >= 0.0f &&
                            w_ < (float)a.height;
            off[f] = in ? (uint32_t)(int)w_ * (uint32_t)a.width + (uint32_t)(int)u : kOutOfRange;
        }
        float d[kSmMaxFrames];
        float2 we[kSmMaxFrames];
#pragma unroll
        for (int f = 0; f < kSmMaxFrames; ++f) {
            const bool in = off[f] != kOutOfRange;
            d[f] = sm_load(make_rsrc(a.frames[f].depth, 4u * wh), in ? 4u * off[f] : kOutOfRange);
            we[f] = load_f2(make_rsrc(a.frames[f].maps, 8u * wh), in ? 8u * off[f] : kOutOfRange);
        }
        float sw = 0.0f, swx = 0.0f;
        float x[kSmMaxFrames];
        uint32_t used_frames = 0u, clipped = 0u;
#pragma unroll
        for (int f = 0; f < kSmMaxFrames; ++f) {
            const float dp = d[f] - zc[f];
            const bool ok = sm_valid(d[f], a.d_max) && dp >= -we[f].y && we[f].x > 0.0f;
            x[f] = dp < we[f].y ? dp : we[f].y;
            if (ok) {
                sw += we[f].x;
                swx += we[f].x * x[f];
                used_frames |= 1u << f;
                if (dp > we[f].y)
                    clipped |= 1u << f;
            }
        }
        if (!(sw > 0.0f))
            continue;
        const float D = swx / sw;
        const float diff = D - a.target[v];
        const float gD = 2.0f * diff;
        loss += (double)diff * (double)diff;
        used += 1.0;
#pragma unroll
        for (int f = 0; f < kSmMaxFrames; ++f) {
            if (used_frames & (1u << f)) {
                atomicAdd(&a.frames[f].gw[off[f]], gD * (x[f] - D) / sw);
                if (clipped & (1u << f))
                    atomicAdd(&a.frames[f].ge[off[f]], gD * we[f].x / sw);
            }
        }
    }
    // workgroup sums, one double atomic per workgroup and quantity
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        loss += __shfl_xor(loss, off);
        used += __shfl_xor(used, off);
    }
    const int wave = (int)threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = loss;
        red[1][wave] = used;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double l = 0.0, u = 0.0;
        for (int k = 0; k < kLossThreads / 64; ++k) {
            l += red[0][k];
            u += red[1][k];
        }
        if (u > 0.0) {
            atomicAdd(&a.acc[0], l);
            atomicAdd(&a.acc[1], u);
        }
    }
}

constexpr int kTile = 64;            // pixels per LDS tile; one wave per workgroup

typedef float v16f __attribute__((ext_vector_type(16)));

// Element (t, m) of a 64 x 32 tile in LDS, rows rotated by t: a lane writing
// its own row and 32 lanes reading one column of a row both touch 32 distinct
// banks without a padding column, which keeps a workgroup's tiles small
// enough for four workgroups (one per SIMD) on a compute unit.
__device__ __forceinline__ int tile_at(int t, int m)
{
    return t * kSmHidden + ((m + t) & (kSmHidden - 1));
}

// Per 64-pixel tile: recompute the forward pass on the matrix cores (the
// inference function, sm_forward_tile, on four 16-pixel sub-tiles whose
// inputs come from the X tile), then per pixel back-propagate dL/dw and
// dL/deps to the hidden layers.  Per tile (staged in LDS) the weight gradients
// are sums of outer products over the pixels -- dense contractions -- and run
// on the matrix cores: dW1 (32 x 27) += G1^T X and dW2 (32 x 32) += G2^T H1 as
// 32 steps of v_mfma_f32_32x32x2_f32 each (two pixels per step).  Lane l
// supplies A[l mod 32][l / 32] and B[l / 32][l mod 32]; accumulator register r
// of lane l holds row 8 (r / 4) + 4 (l / 32) + r mod 4, column l mod 32.  The
// small W3 and bias sums stay on the vector units.
__global__ __launch_bounds__(64) void sm_backward_kernel(SmBackArgs a)
{
    __shared__ float X[kTile][kSmIn + 1];   // column kSmIn is padding (zero)
    __shared__ float H1[kTile * kSmHidden], H2[kTile * kSmHidden];
    __shared__ float G1[kTile * kSmHidden], G2[kTile * kSmHidden];
    __shared__ float GO[kTile][kSmOut];
    const int lane = (int)threadIdx.x;
    const int col = lane & 31, half = lane >> 5;
    // the weights are read-only here and the same for every lane: scalar loads, as in inference
    const ConstParams P = as_constant(a.params);
    const SmOperands W = sm_operands(P);
    const int g = lane >> 4, m16 = lane & 15;
    const double n_used = a.acc[1];
    const float scale = n_used > 0.0 ? (float)(1.0 / n_used) : 0.0f;
    v16f acc_w1 = {}, acc_w2 = {};
    float acc_w3 = 0.0f;   // W3[half][col]
    float acc_b = 0.0f;    // b1[col] (half 0) or b2[col] (half 1)
    float acc_b3 = 0.0f;   // b3[lane], lanes 0 and 1
    // Tiles never straddle two frames, so a tile's frame (and the buffer
    // descriptor of its image) is the same for the whole wave.
    const long long per_frame = (long long)a.width * a.height;
    const long long tiles_per_frame = (per_frame + kTile - 1) / kTile;
    const long long n_tiles = tiles_per_frame * a.n_frames;
    for (long long tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int f = (int)(tile / tiles_per_frame);
        const long long k = (tile - (long long)f * tiles_per_frame) * kTile + lane;
        float x[kSmIn], h1[kSmHidden], h2[kSmHidden];
        float go0 = 0.0f, go1 = 0.0f, gw = 0.0f, ge = 0.0f;
        bool active = false;
        if (k < per_frame) {
            const long long p = (long long)f * per_frame + k;
            gw = a.gw[p];
            ge = a.ge[p];
            const SmView &v = a.views[f];
            const float d = v.depth[k];
            if ((gw != 0.0f || ge != 0.0f) && sm_valid(d, v.d_max)) {
                const int j = (int)k / v.width, i = (int)k - j * v.width;
                sm_inputs(v, i, j, d, x);
                active = true;
            }
        }
        if (!active) {
#pragma unroll
            for (int m = 0; m < kSmIn; ++m)
                x[m] = 0.0f;
        }
        // forward pass on the matrix cores, the same function inference evaluates:
        // four 16-pixel sub-tiles, inputs read back from the X tile
#pragma unroll
        for (int m = 0; m < kSmIn; ++m)
            X[lane][m] = x[m];
        X[lane][kSmIn] = 0.0f;
        __syncthreads();
#pragma unroll
        for (int st = 0; st < kTile / 16; ++st) {
            const int t = 16 * st + m16;
            bf16x8 xb;
#pragma unroll
            for (int jj = 0; jj < 8; ++jj)
                xb[jj] = (__bf16)(8 * g + jj < kSmIn ? X[t][8 * g + jj < kSmIn ? 8 * g + jj : 0] : 0.0f);
            f32x4 th1[2], th2[2], to;
            sm_forward_tile(W, xb, th1, th2, to);
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    H1[tile_at(t, 16 * h + 4 * g + i)] = th1[h][i];
                    H2[tile_at(t, 16 * h + 4 * g + i)] = th2[h][i];
                }
            if (g == 0) {
                GO[t][0] = to[0];
                GO[t][1] = to[1];
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int m = 0; m < kSmHidden; ++m) {
                h1[m] = H1[tile_at(lane, m)];
                h2[m] = H2[tile_at(lane, m)];
            }
            const float o0 = GO[lane][0], o1 = GO[lane][1];
            go0 = scale * gw * 0.5f * (1.0f + o0 / sqrtf(o0 * o0 + 4.0f));
            const float q = 1.0f + o1 * o1;
            go1 = scale * ge * a.vs * 7.0f * 0.5f / (q * sqrtf(q));
        } else {
#pragma unroll
            for (int m = 0; m < kSmHidden; ++m)
                h1[m] = h2[m] = 0.0f;
        }
        // back-propagation through the hidden layers (ReLU masks from the activations)
        float g2[kSmHidden], g1[kSmHidden];
#pragma unroll
        for (int m = 0; m < kSmHidden; ++m) {
            const float gh = __builtin_fmaf(P[kSmW3 + kSmHidden + m], go1, P[kSmW3 + m] * go0);
            g2[m] = h2[m] > 0.0f ? gh : 0.0f;
        }
        // W2^T g2 row by row of W2 (each sum still runs over k2 in order), one
        // fused multiply-add per term: the gradient is checked against the
        // binary64 oracle to a tolerance, not bit for bit
#pragma unroll
        for (int m = 0; m < kSmHidden; ++m)
            g1[m] = 0.0f;
#pragma unroll 4
        for (int k2 = 0; k2 < kSmHidden; ++k2) {
#pragma unroll
            for (int m = 0; m < kSmHidden; ++m)
                g1[m] = __builtin_fmaf(P[kSmW2 + kSmHidden * k2 + m], g2[k2], g1[m]);
        }
#pragma unroll
        for (int m = 0; m < kSmHidden; ++m)
            g1[m] = h1[m] > 0.0f ? g1[m] : 0.0f;
#pragma unroll
        for (int m = 0; m < kSmHidden; ++m) {
            H1[tile_at(lane, m)] = h1[m];
            H2[tile_at(lane, m)] = h2[m];
            G1[tile_at(lane, m)] = g1[m];
            G2[tile_at(lane, m)] = g2[m];
        }
        GO[lane][0] = go0;
        GO[lane][1] = go1;
        __syncthreads();
        // dW1 += G1^T X, dW2 += G2^T H1 on the matrix cores, two pixels per step
        const int xcol = col < kSmIn ? col : 0;   // X has 27 columns: the index stays in the row
#pragma unroll 4
        for (int st = 0; st < kTile / 2; ++st) {
            const int t = 2 * st + half;
            const float xr = X[t][xcol];   // read unconditionally: the loop body stays one block
            const float xv = col < kSmIn ? xr : 0.0f;
            const int tc = tile_at(t, col);
            acc_w1 = __builtin_amdgcn_mfma_f32_32x32x2f32(G1[tc], xv, acc_w1, 0, 0, 0);
            acc_w2 = __builtin_amdgcn_mfma_f32_32x32x2f32(G2[tc], H1[tc], acc_w2, 0, 0, 0);
        }
        // W3, b1 / b2 and b3 on the vector units
        {
            const float *Gb = half ? G2 : G1;
            float s3 = 0.0f, sb = 0.0f, sb3 = 0.0f;
            for (int t = 0; t < kTile; ++t) {
                s3 += GO[t][half] * H2[tile_at(t, col)];
                sb += Gb[tile_at(t, col)];
                sb3 += GO[t][lane & 1];
            }
            acc_w3 += s3;
            acc_b += sb;
            acc_b3 += sb3;
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r / 4) + 4 * half + (r % 4);
        if (col < kSmIn && acc_w1[r] != 0.0f)
            atomicAdd(&a.grad[kSmW1 + kSmIn * row + col], acc_w1[r]);
        if (acc_w2[r] != 0.0f)
            atomicAdd(&a.grad[kSmW2 + kSmHidden * row + col], acc_w2[r]);
    }
    if (acc_w3 != 0.0f)
        atomicAdd(&a.grad[kSmW3 + kSmHidden * half + col], acc_w3);
    if (acc_b != 0.0f)
        atomicAdd(&a.grad[(half ? kSmB2 : kSmB1) + col], acc_b);
    if (lane < kSmOut && acc_b3 != 0.0f)
        atomicAdd(&a.grad[kSmB3 + lane], acc_b3);
}

__global__ void sm_fill_kernel(float *p, long long n, float v)
{
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        p[k] = v;
}

__global__ void sm_zero_acc_kernel(double *acc)
{
    if (threadIdx.x < 2)
        acc[threadIdx.x] = 0.0;
}

__global__ void sm_adam_kernel(float *master, float *m1, float *m2, const float *grad, float *params, int n, float lr,
                               float beta1, float beta2, float eps, float corr1, float corr2)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n)
        return;
    const float g = grad[k];
    const float a = beta1 * m1[k] + (1.0f - beta1) * g;
    const float b = beta2 * m2[k] + (1.0f - beta2) * g * g;
    m1[k] = a;
    m2[k] = b;
    const float w = master[k] - lr * (a / corr1) / (sqrtf(b / corr2) + eps);
    master[k] = w;
    params[k] = round_bf16(w);
}

}  // namespace

hipError_t launch_sm_maps(const SmView &v, float vs, const float *params, float2 *out, hipStream_t stream)
{
    const long long n = (long long)v.width * v.height;
    const unsigned groups = (unsigned)std::max<long long>(1, std::min<long long>((n + kMapThreads - 1) / kMapThreads,
                                                                                  2048));
    hipLaunchKernelGGL(sm_maps_kernel, dim3(groups), dim3(kMapThreads), 0, stream, v, vs, params, out);
    return hipGetLastError();
}

hipError_t launch_sm_maps_mfma(const SmView &v, float vs, const float *params, float2 *out, hipStream_t stream)
{
    const long long tiles = ((long long)v.width * v.height + 63) / 64;   // 64 pixels per wave pass
    const long long waves_per_group = kMapThreads / 64;
    const unsigned groups = (unsigned)std::max<long long>(
        1, std::min<long long>((tiles + waves_per_group - 1) / waves_per_group, 2048));
    hipLaunchKernelGGL(sm_maps_mfma_kernel, dim3(groups), dim3(kMapThreads), 0, stream, v, vs, params, out);
    return hipGetLastError();
}

hipError_t launch_sm_fill(float *p, long long n, float value, hipStream_t stream)
{
    if (n <= 0)
        return hipSuccess;
    const unsigned groups = (unsigned)std::min<long long>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(sm_fill_kernel, dim3(groups), dim3(256), 0, stream, p, n, value);
    return hipGetLastError();
}

hipError_t launch_sm_loss(const SmLossArgs &a, hipStream_t stream)
{
    hipLaunchKernelGGL(sm_zero_acc_kernel, dim3(1), dim3(64), 0, stream, a.acc);
    if (a.n_vox > 0) {
        const unsigned groups =
            (unsigned)std::min<long long>((a.n_vox + kLossThreads - 1) / kLossThreads, 4096);
        hipLaunchKernelGGL(sm_fuse_loss_kernel, dim3(groups), dim3(kLossThreads), 0, stream, a);
    }
    return hipGetLastError();
}

hipError_t launch_sm_backward(const SmBackArgs &a, hipStream_t stream)
{
    const long long tiles = (((long long)a.width * a.height + kTile - 1) / kTile) * a.n_frames;
    // One round of resident workgroups (the LDS tiles bound how many share a
    // compute unit): a grid beyond that leaves a partial second round.
    int dev = 0, cus = 0, per_cu = 0;
    long long resident = 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sm_backward_kernel, 64, 0) == hipSuccess &&
        cus > 0 && per_cu > 0)
        resident = (long long)cus * per_cu;
    const unsigned groups =
        (unsigned)std::max<long long>(1, std::min<long long>(tiles, resident));
    hipLaunchKernelGGL(sm_backward_kernel, dim3(groups), dim3(64), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_sm_adam(float *master, float *m1, float *m2, const float *grad, float *params, int n, float lr,
                          float beta1, float beta2, float eps, int step, hipStream_t stream)
{
    const float corr1 = 1.0f - (float)std::pow((double)beta1, (double)step);
    const float corr2 = 1.0f - (float)std::pow((double)beta2, (double)step);
    hipLaunchKernelGGL(sm_adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, master, m1, m2, grad,
                       params, n, lr, beta1, beta2, eps, corr1, corr2);
    return hipGetLastError();
}

}  // namespace tsdf

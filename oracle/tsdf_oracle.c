/*
 * tsdf_oracle.c -- CPU oracle for projective TSDF integration (nvblox §IV).
 *
 * TEST INFRASTRUCTURE ONLY (see tsdf_oracle.h).  Plain C99, built with
 * -ffp-contract=off -fno-fast-math so every binary32 operation is one
 * correctly rounded IEEE-754 operation.  Single-threaded, except
 * ora_integrate_depth_threads (OpenMP), which times the CPU baseline on all
 * host cores and gives the single-threaded result bit for bit.
 *
 * The sparse map follows the paper's two-level layout (§IV-A): a hash table
 * from integer block index (x, y, z) to a block of 8 x 8 x 8 voxels stored
 * contiguously.  The hash here is a plain open-addressing table of int32
 * triples with linear probing; blocks live in growable arrays in insertion
 * order.
 */
#include "tsdf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    float voxel_size, truncation_vox, max_weight, max_range;
    int weighting;
} ora_params;

typedef struct {
    int32_t x, y, z;
    int64_t index;   /* -1 = empty slot */
} ora_slot;

struct ora_map {
    int precision;            /* 32 or 64 */
    int storage16;            /* 1: voxels stored as binary16 (precision 32 only) */
    ora_params p;
    ora_slot *table;          /* hash table, size table_size (power of two) */
    long long table_size;
    long long n_blocks, cap_blocks;
    int32_t *coords;          /* 3 per block */
    void *dist, *weight;      /* 512 REAL per block */
    long long *touched;       /* indices of blocks updated by the last frame */
    long long n_touched, cap_touched;
    int32_t scan_min[3], scan_max[3];
};

static uint64_t slot_hash(int32_t x, int32_t y, int32_t z)
{
    /* three large odd multipliers, xor-folded */
    uint64_t h = (uint64_t)(uint32_t)x * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)y * 0xC2B2AE3D27D4EB4Full;
    h ^= (uint64_t)(uint32_t)z * 0x165667B19E3779F9ull;
    return h ^ (h >> 29);
}

static long long table_probe(const ora_slot *table, long long size, int32_t x, int32_t y, int32_t z)
{
    long long s = (long long)(slot_hash(x, y, z) & (uint64_t)(size - 1));
    for (;;) {
        const ora_slot *e = &table[s];
        if (e->index < 0 || (e->x == x && e->y == y && e->z == z))
            return s;
        s = (s + 1) & (size - 1);
    }
}

static int table_grow(ora_map *m)
{
    long long ns = m->table_size ? 2 * m->table_size : 1024;
    ora_slot *t = (ora_slot *)malloc((size_t)ns * sizeof(ora_slot));
    if (!t)
        return -1;
    for (long long k = 0; k < ns; ++k)
        t[k].index = -1;
    for (long long b = 0; b < m->n_blocks; ++b) {
        int32_t *c = &m->coords[3 * b];
        long long s = table_probe(t, ns, c[0], c[1], c[2]);
        t[s].x = c[0];
        t[s].y = c[1];
        t[s].z = c[2];
        t[s].index = b;
    }
    free(m->table);
    m->table = t;
    m->table_size = ns;
    return 0;
}

static size_t real_size(const ora_map *m) { return m->precision == 32 ? sizeof(float) : sizeof(double); }

static int blocks_grow(ora_map *m)
{
    long long nc = m->cap_blocks ? 2 * m->cap_blocks : 256;
    size_t rs = real_size(m);
    int32_t *c = (int32_t *)realloc(m->coords, (size_t)nc * 3 * sizeof(int32_t));
    if (!c)
        return -1;
    m->coords = c;
    void *d = realloc(m->dist, (size_t)nc * 512 * rs);
    if (!d)
        return -1;
    m->dist = d;
    void *w = realloc(m->weight, (size_t)nc * 512 * rs);
    if (!w)
        return -1;
    m->weight = w;
    m->cap_blocks = nc;
    return 0;
}

/* Index of block (x, y, z), inserting it with all voxels at distance 0 and
 * weight 0 if it is not yet in the map.  -1 when out of memory. */
static long long map_find_or_insert(ora_map *m, int32_t x, int32_t y, int32_t z)
{
    if (2 * (m->n_blocks + 1) > m->table_size && table_grow(m) != 0)
        return -1;
    long long s = table_probe(m->table, m->table_size, x, y, z);
    if (m->table[s].index >= 0)
        return m->table[s].index;
    if (m->n_blocks == m->cap_blocks && blocks_grow(m) != 0)
        return -1;
    long long b = m->n_blocks++;
    m->coords[3 * b + 0] = x;
    m->coords[3 * b + 1] = y;
    m->coords[3 * b + 2] = z;
    size_t rs = real_size(m);
    memset((char *)m->dist + (size_t)b * 512 * rs, 0, 512 * rs);
    memset((char *)m->weight + (size_t)b * 512 * rs, 0, 512 * rs);
    m->table[s].x = x;
    m->table[s].y = y;
    m->table[s].z = z;
    m->table[s].index = b;
    return b;
}

/* IEEE 754 rounding of a binary32 value to binary16 (11 significant bits,
 * exponents down to -14, subnormal quantum 2^-24, largest finite 65504). */
float ora_round_binary16(float x)
{
    if (!isfinite(x) || x == 0.0f)
        return x;
    float ax = fabsf(x);
    int e;
    (void)frexpf(ax, &e);                /* ax = m 2^e, 0.5 <= m < 1 */
    int qexp = e - 11;                   /* quantum of an 11-bit significand */
    if (qexp < -24)
        qexp = -24;                      /* subnormal range */
    const float q = ldexpf(1.0f, qexp);
    float r = nearbyintf(ax / q) * q;    /* exact scaling; nearest, ties to even */
    if (r > 65504.0f)
        r = INFINITY;
    return copysignf(r, x);
}

static int touched_push(ora_map *m, long long b)
{
    if (m->n_touched == m->cap_touched) {
        long long nc = m->cap_touched ? 2 * m->cap_touched : 256;
        long long *t = (long long *)realloc(m->touched, (size_t)nc * sizeof(long long));
        if (!t)
            return -1;
        m->touched = t;
        m->cap_touched = nc;
    }
    m->touched[m->n_touched++] = b;
    return 0;
}

/* atan on [0, 1]: the polynomial of Abramowitz & Stegun, Handbook of
 * Mathematical Functions, formula 4.4.49 (|error| <= 2e-8), evaluated by
 * Horner's rule in binary32. */
static float atan_unit_f32(float t)
{
    const float t2 = t * t;
    float p = 0.0028662257f;
    p = p * t2 + -0.0161657367f;
    p = p * t2 + 0.0429096138f;
    p = p * t2 + -0.0752896400f;
    p = p * t2 + 0.1065626393f;
    p = p * t2 + -0.1420889944f;
    p = p * t2 + 0.1999355085f;
    p = p * t2 + -0.3333314528f;
    p = p * t2 + 1.0f;
    return p * t;
}

/* atan2 in binary32 from atan on [0, 1] by octant reduction; (0, 0) -> 0. */
float ora_atan2_f32(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    if (ax == 0.0f && ay == 0.0f)
        return 0.0f;
    const int swap = ay > ax;
    const float t = swap ? ax / ay : ay / ax;
    float a = atan_unit_f32(t);
    if (swap)
        a = 1.57079637f - a;
    if (x < 0.0f)
        a = 3.14159274f - a;
    return y < 0.0f ? -a : a;
}

static int key_cmp(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

#define REAL float
#define SFX _f32
#define SQRT sqrtf
#define FLOOR floorf
#define ATAN2 ora_atan2_f32
#include "oracle_impl.h"
#undef REAL
#undef SFX
#undef SQRT
#undef FLOOR
#undef ATAN2

#define REAL double
#define SFX _f64
#define SQRT sqrt
#define FLOOR floor
#define ATAN2 atan2
#include "oracle_impl.h"
#undef REAL
#undef SFX
#undef SQRT
#undef FLOOR
#undef ATAN2

static int params_ok(int precision, float vs, float tau, float wmax, float dmax, int weighting)
{
    return (precision == 32 || precision == 64) && vs > 0 && tau > 0 && wmax > 0 && dmax > 0 &&
           (weighting == ORA_WEIGHT_CONSTANT || weighting == ORA_WEIGHT_LINEAR_DROPOFF);
}

ora_map *ora_create(int precision, float voxel_size, float truncation_vox, float max_weight,
                    float max_range, int weighting)
{
    if (!params_ok(precision, voxel_size, truncation_vox, max_weight, max_range, weighting))
        return NULL;
    ora_map *m = (ora_map *)calloc(1, sizeof(ora_map));
    if (!m)
        return NULL;
    m->precision = precision;
    m->p.voxel_size = voxel_size;
    m->p.truncation_vox = truncation_vox;
    m->p.max_weight = max_weight;
    m->p.max_range = max_range;
    m->p.weighting = weighting;
    m->scan_max[0] = m->scan_max[1] = m->scan_max[2] = -1;
    return m;
}

int ora_set_storage16(ora_map *m)
{
    if (!m || m->precision != 32 || m->n_blocks != 0)
        return -1;
    m->storage16 = 1;
    return 0;
}

void ora_destroy(ora_map *m)
{
    if (!m)
        return;
    free(m->table);
    free(m->coords);
    free(m->dist);
    free(m->weight);
    free(m->touched);
    free(m);
}

static int frame_args_ok(const float *depth, int width, int height, const float K[4], const float T[16])
{
    if (!depth || !K || !T || width <= 0 || height <= 0)
        return 0;
    if (!(K[0] > 0 && K[1] > 0 && isfinite(K[2]) && isfinite(K[3]) && isfinite(K[0]) && isfinite(K[1])))
        return 0;
    for (int k = 0; k < 16; ++k)
        if (!isfinite(T[k]))
            return 0;
    return 1;
}

long long ora_integrate_depth(ora_map *m, const float *depth, int width, int height,
                              const float K[4], const float T[16])
{
    if (!m || !frame_args_ok(depth, width, height, K, T))
        return -1;
    return m->precision == 32 ? integrate_f32(m, depth, width, height, K, T)
                              : integrate_f64(m, depth, width, height, K, T);
}

long long ora_integrate_depth_threads(ora_map *m, const float *depth, int width, int height, const float K[4],
                                      const float T[16], int threads)
{
    if (!m || !frame_args_ok(depth, width, height, K, T) || threads < 1)
        return -1;
    return m->precision == 32 ? integrate_threads_f32(m, depth, width, height, K, T, threads)
                              : integrate_threads_f64(m, depth, width, height, K, T, threads);
}

long long ora_integrate_depth_dda(ora_map *m, const float *depth, int width, int height, const float K[4],
                                  const float T[16])
{
    if (!m || !frame_args_ok(depth, width, height, K, T))
        return -1;
    return m->precision == 32 ? integrate_dda_f32(m, depth, width, height, K, T)
                              : integrate_dda_f64(m, depth, width, height, K, T);
}

long long ora_integrate_depth_range(ora_map *m, const float *depth, int width, int height,
                                    const float K[4], const float T[16], float max_range)
{
    if (!m || !(max_range > 0) || !isfinite(max_range))
        return -1;
    const float saved = m->p.max_range;
    m->p.max_range = max_range;
    const long long n = ora_integrate_depth(m, depth, width, height, K, T);
    m->p.max_range = saved;
    return n;
}

long long ora_integrate_range(ora_map *m, const float *range, int width, int height,
                              const float model[6], const float T[16])
{
    if (!m || !range || !model || !T || width <= 1 || height <= 1)
        return -1;
    if (!(model[1] > 0 && model[3] > 0 && model[4] >= 0 && isfinite(model[0]) && isfinite(model[1]) &&
          isfinite(model[2]) && isfinite(model[3]) && isfinite(model[4]) && model[5] >= 0 && isfinite(model[5])))
        return -1;
    for (int k = 0; k < 16; ++k)
        if (!isfinite(T[k]))
            return -1;
    const float saved = m->p.max_range;
    if (model[5] > 0)
        m->p.max_range = model[5];
    const long long n = m->precision == 32 ? integrate_any_f32(m, range, width, height, NULL, model, T)
                                           : integrate_any_f64(m, range, width, height, NULL, model, T);
    m->p.max_range = saved;
    return n;
}

long long ora_dense_integrate_range(int precision, float voxel_size, float truncation_vox, float max_weight,
                                    float max_range, int weighting, const float *range, int width, int height,
                                    const float model[6], const float T[16], const int32_t gmin[3],
                                    const int32_t gdim[3], double *dist, double *weight)
{
    if (!params_ok(precision, voxel_size, truncation_vox, max_weight, max_range, weighting) || !range ||
        !model || !T || width <= 1 || height <= 1 || !gmin || !gdim || !dist || !weight)
        return -1;
    ora_params p = {voxel_size, truncation_vox, max_weight, model[5] > 0 ? model[5] : max_range, weighting};
    return precision == 32 ? dense_range_f32(&p, range, width, height, model, T, gmin, gdim, dist, weight)
                           : dense_range_f64(&p, range, width, height, model, T, gmin, gdim, dist, weight);
}

long long ora_num_blocks(const ora_map *m) { return m ? m->n_blocks : 0; }

void ora_blocks(const ora_map *m, int32_t *xyz)
{
    memcpy(xyz, m->coords, (size_t)m->n_blocks * 3 * sizeof(int32_t));
}

void ora_voxels(const ora_map *m, double *dist, double *weight)
{
    if (m->precision == 32)
        export_voxels_f32(m, dist, weight);
    else
        export_voxels_f64(m, dist, weight);
}

long long ora_find_block(const ora_map *m, int32_t x, int32_t y, int32_t z)
{
    if (!m || m->table_size == 0)
        return -1;
    long long s = table_probe(m->table, m->table_size, x, y, z);
    return m->table[s].index;
}

long long ora_touched(const ora_map *m, int32_t *xyz)
{
    if (xyz)
        for (long long k = 0; k < m->n_touched; ++k)
            memcpy(&xyz[3 * k], &m->coords[3 * m->touched[k]], 3 * sizeof(int32_t));
    return m->n_touched;
}

void ora_last_scan(const ora_map *m, int32_t bmin[3], int32_t bmax[3])
{
    memcpy(bmin, m->scan_min, sizeof(m->scan_min));
    memcpy(bmax, m->scan_max, sizeof(m->scan_max));
}

void ora_camera_from_world(int precision, const float T[16], double R[9], double t[3])
{
    if (precision == 32)
        camera_from_world_f32(T, R, t);
    else
        camera_from_world_f64(T, R, t);
}

long long ora_dense_integrate(int precision, float voxel_size, float truncation_vox,
                              float max_weight, float max_range, int weighting,
                              const float *depth, int width, int height,
                              const float K[4], const float T[16],
                              const int32_t gmin[3], const int32_t gdim[3],
                              double *dist, double *weight)
{
    if (!params_ok(precision, voxel_size, truncation_vox, max_weight, max_range, weighting) ||
        !frame_args_ok(depth, width, height, K, T) || !gmin || !gdim || !dist || !weight)
        return -1;
    ora_params p = {voxel_size, truncation_vox, max_weight, max_range, weighting};
    return precision == 32 ? dense_f32(&p, depth, width, height, K, T, gmin, gdim, dist, weight)
                           : dense_f64(&p, depth, width, height, K, T, gmin, gdim, dist, weight);
}

#include "sensor_model_impl.h"

/*
 * oracle_impl.h -- precision-generic body of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see tsdf_oracle.h).
 *
 * Included by tsdf_oracle.c once with REAL = float (suffix _f32) and once with
 * REAL = double (suffix _f64).  Every arithmetic statement below is a single
 * IEEE-754 operation in REAL, evaluated left to right as written; the file is
 * compiled without contraction or fast-math so the binary32 instance performs
 * exactly these roundings.
 */

#define FN_(a, b) a##b
#define FN2(a, b) FN_(a, b)
#define FN(name) FN2(name, SFX)

/* Per-frame constants in REAL.  Paper §IV-B: T_CL is the inverse of the sensor
 * pose T_LC (§III); epsilon is the truncation distance. */
typedef struct {
    REAL R[9];          /* camera-from-world rotation, row-major */
    REAL t[3];          /* camera-from-world translation */
    REAL fx, fy, cx, cy;
    REAL width_r, height_r;
    int width, height;
    REAL vs;            /* voxel edge */
    REAL eps;           /* truncation distance epsilon */
    REAL delta;         /* start of the linear weight dropoff behind the surface */
    REAL span_inv;      /* 1 / (epsilon - delta) */
    REAL w_max, d_max;
    int weighting;
    const float *depth;
    /* spherical range images (Eq. (3)) */
    REAL az_start, alpha;     /* azimuth of column 0's left edge; columns per radian */
    REAL pol_start, beta;     /* polar angle (from +z) of row 0's top edge; rows per radian */
    REAL interp_diff;         /* largest spread of the 4 interpolated ranges */
    int full_circle;          /* columns wrap around (azimuth field of view >= 2 pi) */
    /* learned sensor model: per-pixel weight and truncation distance (NULL otherwise) */
    const float *w_map, *eps_map;
} FN(frame);

/* Frame set-up.  The inverse of a rigid pose is (R^T, -R^T t).  R^T is exact;
 * each component of -R^T t is accumulated in binary64 from the binary32 pose,
 * in the order ((R0i t0 + R1i t1) + R2i t2), and rounded once to REAL. */
static void FN(frame_setup)(FN(frame) *f, const ora_params *p, const float *depth,
                            int width, int height, const float K[4], const float T[16])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            f->R[3 * i + j] = (REAL)T[4 * j + i];
    for (int i = 0; i < 3; ++i) {
        double acc = ((double)T[0 * 4 + i] * (double)T[3] + (double)T[1 * 4 + i] * (double)T[7])
                     + (double)T[2 * 4 + i] * (double)T[11];
        f->t[i] = (REAL)(-acc);
    }
    f->fx = (REAL)K[0];
    f->fy = (REAL)K[1];
    f->cx = (REAL)K[2];
    f->cy = (REAL)K[3];
    f->width = width;
    f->height = height;
    f->width_r = (REAL)width;
    f->height_r = (REAL)height;
    f->vs = (REAL)p->voxel_size;
    f->eps = (REAL)p->truncation_vox * f->vs;
    /* Linear dropoff (the paper only says the weight may follow a sensor
     * model): weight 1 down to one voxel behind the surface, then falling
     * linearly to 0 at -epsilon. */
    f->delta = f->vs;
    f->span_inv = f->eps > f->delta ? (REAL)1 / (f->eps - f->delta) : (REAL)0;
    f->w_max = (REAL)p->max_weight;
    f->d_max = (REAL)p->max_range;
    f->weighting = p->weighting;
    f->depth = depth;
    f->w_map = 0;
    f->eps_map = 0;
}

/* The TSDF functor after sampling (§IV-B): truncation band, weight, clamp.
 * d is a valid measurement and dp = d - d_v the projective distance. */
static int FN(measure_tail)(const FN(frame) *f, REAL dp, REAL *x, REAL *wm)
{
    /* voxels more than epsilon behind the surface are skipped, not clamped */
    if (!(dp >= -f->eps))
        return 0;
    REAL w = (REAL)1;
    if (f->weighting == ORA_WEIGHT_LINEAR_DROPOFF && dp < -f->delta)
        w = (f->eps + dp) * f->span_inv;
    if (!(w > 0))
        return 0;
    *x = dp < f->eps ? dp : f->eps;
    *wm = w;
    return 1;
}

/* One voxel against one frame (§IV-B, Eq. (1)-(2) and the TSDF functor).
 * g = global voxel index.  Returns 1 and the truncated distance *x and the
 * measurement weight *wm when the voxel is updated; 0 when it is not. */
static int FN(voxel_measure)(const FN(frame) *f, int32_t gx, int32_t gy, int32_t gz,
                             REAL *x, REAL *wm)
{
    const REAL half = (REAL)0.5;
    /* voxel centre p_L */
    REAL px = ((REAL)gx + half) * f->vs;
    REAL py = ((REAL)gy + half) * f->vs;
    REAL pz = ((REAL)gz + half) * f->vs;
    /* Eq. (1): p_C = T_CL p_L */
    REAL xc = ((f->R[0] * px + f->R[1] * py) + f->R[2] * pz) + f->t[0];
    REAL yc = ((f->R[3] * px + f->R[4] * py) + f->R[5] * pz) + f->t[1];
    REAL zc = ((f->R[6] * px + f->R[7] * py) + f->R[8] * pz) + f->t[2];
    if (!(zc > 0))
        return 0;
    /* Eq. (2), pinhole: u = fu x/z + cu, v = fv y/z + cv */
    REAL r = (REAL)1 / zc;
    REAL u = f->fx * (xc * r) + f->cx;
    REAL v = f->fy * (yc * r) + f->cy;
    /* nearest-neighbour sample: pixel (i, j) covers [i, i+1) x [j, j+1) */
    if (!(u >= 0 && u < f->width_r && v >= 0 && v < f->height_r))
        return 0;
    int32_t i = (int32_t)u;
    int32_t j = (int32_t)v;
    const size_t idx = (size_t)j * (size_t)f->width + (size_t)i;
    REAL d = (REAL)f->depth[idx];
    /* a measurement is valid iff 0 < d <= max range (NaN, Inf, <= 0 fail) */
    if (!(d > 0 && d <= f->d_max))
        return 0;
    /* projective distance; voxel depth d_v is the camera-frame z for a depth image */
    REAL dp = d - zc;
    if (f->w_map) {
        /* learned sensor model: the pixel's own truncation distance and weight
         * replace epsilon and the weighting function */
        REAL e = (REAL)f->eps_map[idx];
        if (!(dp >= -e))
            return 0;
        REAL w = (REAL)f->w_map[idx];
        if (!(w > 0))
            return 0;
        *x = dp < e ? dp : e;
        *wm = w;
        return 1;
    }
    return FN(measure_tail)(f, dp, x, wm);
}

/* One voxel against a spherical range image (Eq. (3)).  Sensor frame: x
 * forward, y left, z up; azimuth theta = atan2(y, x), polar angle phi measured
 * from +z (computed as atan2(sqrt(x^2 + y^2), z), the same angle as acos(z/r));
 * column coordinate u = (theta - theta_start) alpha, row v = (phi - phi_start)
 * beta, pixel (i, j) covering [i, i+1) x [j, j+1) with its beam at the centre.
 * The range is interpolated bilinearly between the four beam centres around
 * (u, v), and only when all four are valid and their spread is at most
 * interp_diff, so that no value is interpolated across a foreground/background
 * edge.  The voxel depth d_v is the Euclidean range of the voxel centre. */
static int FN(voxel_measure_range)(const FN(frame) *f, int32_t gx, int32_t gy, int32_t gz, REAL *x, REAL *wm)
{
    const REAL half = (REAL)0.5, one = (REAL)1;
    REAL px = ((REAL)gx + half) * f->vs;
    REAL py = ((REAL)gy + half) * f->vs;
    REAL pz = ((REAL)gz + half) * f->vs;
    REAL xc = ((f->R[0] * px + f->R[1] * py) + f->R[2] * pz) + f->t[0];
    REAL yc = ((f->R[3] * px + f->R[4] * py) + f->R[5] * pz) + f->t[1];
    REAL zc = ((f->R[6] * px + f->R[7] * py) + f->R[8] * pz) + f->t[2];
    REAL rv = SQRT((xc * xc + yc * yc) + zc * zc);
    if (!(rv > 0))
        return 0;
    REAL theta = ATAN2(yc, xc);
    REAL phi = ATAN2(SQRT(xc * xc + yc * yc), zc);
    REAL uc = (theta - f->az_start) * f->alpha - half;
    REAL vc = (phi - f->pol_start) * f->beta - half;
    REAL fi = FLOOR(uc), fj = FLOOR(vc);
    REAL fu = uc - fi, fv = vc - fj;
    int32_t j0 = (int32_t)fj;
    if (j0 < 0 || j0 + 1 > f->height - 1)
        return 0;
    int32_t i0 = (int32_t)fi, i1;
    if (f->full_circle) {
        i0 = ((i0 % f->width) + f->width) % f->width;
        i1 = (i0 + 1) % f->width;
    } else {
        if (i0 < 0 || i0 + 1 > f->width - 1)
            return 0;
        i1 = i0 + 1;
    }
    const float *row0 = f->depth + (size_t)j0 * (size_t)f->width;
    const float *row1 = row0 + f->width;
    REAL r00 = (REAL)row0[i0], r10 = (REAL)row0[i1], r01 = (REAL)row1[i0], r11 = (REAL)row1[i1];
    if (!(r00 > 0 && r00 <= f->d_max && r10 > 0 && r10 <= f->d_max && r01 > 0 && r01 <= f->d_max &&
          r11 > 0 && r11 <= f->d_max))
        return 0;
    REAL mn = r00 < r10 ? r00 : r10, mx = r00 < r10 ? r10 : r00;
    mn = r01 < mn ? r01 : mn;
    mx = r01 > mx ? r01 : mx;
    mn = r11 < mn ? r11 : mn;
    mx = r11 > mx ? r11 : mx;
    if (!(mx - mn <= f->interp_diff))
        return 0;
    REAL d = (one - fv) * ((one - fu) * r00 + fu * r10) + fv * ((one - fu) * r01 + fu * r11);
    REAL dp = d - rv;
    return FN(measure_tail)(f, dp, x, wm);
}

/* Frame set-up of a spherical range image: pose as for a camera, then the
 * angular model (columns and rows per radian computed in REAL). */
static void FN(range_setup)(FN(frame) *f, const ora_params *p, const float *range, int width, int height,
                            const float model[5], const float T[16])
{
    const float K[4] = {1, 1, 0, 0};
    FN(frame_setup)(f, p, range, width, height, K, T);
    f->az_start = (REAL)model[0];
    f->alpha = (REAL)width / (REAL)model[1];
    f->pol_start = (REAL)model[2];
    f->beta = (REAL)height / (REAL)model[3];
    f->interp_diff = (REAL)model[4];
    f->full_circle = (REAL)model[1] >= (REAL)6.28318548f;
}

/* Weighted average with capped weight sum (§IV-B): the running distance is
 * averaged with the uncapped weight sum; only the stored weight is capped. */
static void FN(voxel_fuse)(REAL *D, REAL *W, REAL x, REAL wm, REAL w_max)
{
    REAL n = *D * *W + x * wm;
    REAL s = *W + wm;
    *D = n / s;
    *W = s < w_max ? s : w_max;
}

/* Inclusive block box containing every voxel that can be updated by the
 * frame: such a voxel has 0 < z_c <= d + epsilon <= zfar and projects inside
 * the image, so it lies in the pyramid spanned by the camera centre and the
 * four image corners at depth zfar.  The box of that pyramid is widened by one
 * voxel on every side.  Returns 0 if the frame has no valid pixel. */
static int FN(scan_box)(const FN(frame) *f, const float K[4], const float T[16],
                        int32_t bmin[3], int32_t bmax[3])
{
    double zmax = -1.0;
    for (size_t k = 0; k < (size_t)f->width * (size_t)f->height; ++k) {
        float d = f->depth[k];
        if (d > 0 && d <= (float)f->d_max && (double)d > zmax)
            zmax = (double)d;
    }
    if (zmax <= 0)
        return 0;
    double zfar = zmax + (double)f->eps;
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a)
        lo[a] = hi[a] = (double)T[4 * a + 3];   /* camera centre */
    for (int c = 0; c < 4; ++c) {
        double u = (c & 1) ? (double)f->width : 0.0;
        double v = (c & 2) ? (double)f->height : 0.0;
        double pc[3] = {(u - K[2]) / K[0] * zfar, (v - K[3]) / K[1] * zfar, zfar};
        for (int a = 0; a < 3; ++a) {
            double w = (double)T[4 * a + 3];
            for (int b = 0; b < 3; ++b)
                w += (double)T[4 * a + b] * pc[b];
            if (w < lo[a]) lo[a] = w;
            if (w > hi[a]) hi[a] = w;
        }
    }
    double edge = 8.0 * (double)f->vs;
    for (int a = 0; a < 3; ++a) {
        bmin[a] = (int32_t)floor((lo[a] - (double)f->vs) / edge);
        bmax[a] = (int32_t)floor((hi[a] + (double)f->vs) / edge);
    }
    return 1;
}

/* Block box of a spherical range image: every updated voxel lies within
 * max valid range + epsilon of the sensor and inside the polar band, so inside
 * the sensor-frame box [-R, R]^2 x [min(0, R cos phi_end), max(0, R cos phi_start)],
 * whose world box, widened by one voxel, is returned.  0 if no pixel is valid. */
static int FN(scan_box_range)(const FN(frame) *f, const float model[5], const float T[16],
                              int32_t bmin[3], int32_t bmax[3])
{
    double rmax = -1.0;
    for (size_t k = 0; k < (size_t)f->width * (size_t)f->height; ++k) {
        float d = f->depth[k];
        if (d > 0 && d <= (float)f->d_max && (double)d > rmax)
            rmax = (double)d;
    }
    if (rmax <= 0)
        return 0;
    const double R = rmax + (double)f->eps;
    const double zlo = fmin(0.0, R * cos((double)model[2] + (double)model[3]));
    const double zhi = fmax(0.0, R * cos((double)model[2]));
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a)
        lo[a] = hi[a] = (double)T[4 * a + 3];
    for (int c = 0; c < 8; ++c) {
        const double pc[3] = {(c & 1) ? R : -R, (c & 2) ? R : -R, (c & 4) ? zhi : zlo};
        for (int a = 0; a < 3; ++a) {
            double w = (double)T[4 * a + 3];
            for (int b = 0; b < 3; ++b)
                w += (double)T[4 * a + b] * pc[b];
            if (w < lo[a]) lo[a] = w;
            if (w > hi[a]) hi[a] = w;
        }
    }
    double edge = 8.0 * (double)f->vs;
    for (int a = 0; a < 3; ++a) {
        bmin[a] = (int32_t)floor((lo[a] - (double)f->vs) / edge);
        bmax[a] = (int32_t)floor((hi[a] + (double)f->vs) / edge);
    }
    return 1;
}

static REAL *FN(dist_ptr)(ora_map *m) { return (REAL *)m->dist; }
static REAL *FN(weight_ptr)(ora_map *m) { return (REAL *)m->weight; }

/* One frame into the sparse map.  Every block of the scan box is evaluated
 * voxel by voxel; a block that has at least one updated voxel is looked up or
 * inserted in the block hash (§IV-A) and its updated voxels are fused.
 * model == NULL: pinhole depth image; otherwise a spherical range image. */
static long long FN(integrate_prepared)(ora_map *m, FN(frame) *fp, const float K[4], const float *model,
                                        const float T[16]);

static long long FN(integrate_any)(ora_map *m, const float *depth, int width, int height,
                                   const float K[4], const float *model, const float T[16])
{
    FN(frame) f;
    if (model)
        FN(range_setup)(&f, &m->p, depth, width, height, model, T);
    else
        FN(frame_setup)(&f, &m->p, depth, width, height, K, T);
    return FN(integrate_prepared)(m, &f, K, model, T);
}

/* A pinhole frame with the learned sensor model's per-pixel weight and
 * truncation maps.  The scan box reaches the largest truncation of any valid
 * pixel behind the farthest measurement. */
static long long FN(integrate_learned)(ora_map *m, const float *depth, int width, int height, const float K[4],
                                       const float T[16], const float *w_map, const float *eps_map)
{
    FN(frame) f;
    FN(frame_setup)(&f, &m->p, depth, width, height, K, T);
    f.w_map = w_map;
    f.eps_map = eps_map;
    REAL emax = 0;
    for (size_t k = 0; k < (size_t)width * (size_t)height; ++k) {
        const float d = depth[k];
        if (d > 0 && d <= (float)f.d_max && (REAL)eps_map[k] > emax)
            emax = (REAL)eps_map[k];
    }
    f.eps = emax;
    return FN(integrate_prepared)(m, &f, K, NULL, T);
}

/* Paper-literal allocation (§IV-B: the blocks in view are found by ray
 * tracing through the block grid, Amanatides & Woo): for every valid pixel,
 * the ray from the camera centre through the pixel centre is walked through
 * the grid of blocks (edge 8 vs) from depth 0 to min(d + epsilon, max range)
 * (depth along the optical axis; the ray direction has unit camera z).  A
 * block is visited when the walk enters it; at a tie the walk steps x, then
 * y, then z; a boundary exactly at the end depth is crossed.  Writes the
 * packed keys of the visited blocks (with repeats) to *keys and returns
 * their number, or -1 when out of memory. */
static long long FN(dda_keys)(const FN(frame) *f, const float T[16], uint64_t **keys)
{
    const REAL half = (REAL)0.5;
    const REAL B = (REAL)8 * f->vs;
    const REAL o[3] = {(REAL)T[3], (REAL)T[7], (REAL)T[11]};
    long long n = 0, cap = 1 << 16;
    uint64_t *out = (uint64_t *)malloc((size_t)cap * sizeof(uint64_t));
    if (!out)
        return -1;
    for (int j = 0; j < f->height; ++j)
        for (int i = 0; i < f->width; ++i) {
            const REAL d = (REAL)f->depth[(size_t)j * (size_t)f->width + (size_t)i];
            if (!(d > 0 && d <= f->d_max))
                continue;
            const REAL a = (((REAL)i + half) - f->cx) / f->fx;
            const REAL b = (((REAL)j + half) - f->cy) / f->fy;
            REAL dir[3], tmax[3], tdel[3];
            int32_t c[3], step[3];
            REAL te = d + f->eps;
            if (!(te <= f->d_max))
                te = f->d_max;
            for (int k = 0; k < 3; ++k) {
                dir[k] = ((REAL)T[4 * k] * a + (REAL)T[4 * k + 1] * b) + (REAL)T[4 * k + 2];
                c[k] = (int32_t)FLOOR(o[k] / B);
                if (dir[k] > 0) {
                    step[k] = 1;
                    tmax[k] = ((REAL)(c[k] + 1) * B - o[k]) / dir[k];
                    tdel[k] = B / dir[k];
                } else if (dir[k] < 0) {
                    step[k] = -1;
                    tmax[k] = ((REAL)c[k] * B - o[k]) / dir[k];
                    tdel[k] = B / -dir[k];
                } else {
                    step[k] = 0;
                    tmax[k] = (REAL)INFINITY;
                    tdel[k] = (REAL)INFINITY;
                }
            }
            for (int it = 0; it < (1 << 16); ++it) {
                if (n == cap) {
                    cap *= 2;
                    uint64_t *g = (uint64_t *)realloc(out, (size_t)cap * sizeof(uint64_t));
                    if (!g) {
                        free(out);
                        return -1;
                    }
                    out = g;
                }
                out[n++] = ((uint64_t)(uint32_t)(c[0] + (1 << 20)) << 42) |
                           ((uint64_t)(uint32_t)(c[1] + (1 << 20)) << 21) | (uint64_t)(uint32_t)(c[2] + (1 << 20));
                const int ax = (tmax[0] <= tmax[1] && tmax[0] <= tmax[2]) ? 0 : (tmax[1] <= tmax[2] ? 1 : 2);
                if (!(tmax[ax] <= te))
                    break;
                c[ax] += step[ax];
                tmax[ax] += tdel[ax];
            }
        }
    *keys = out;
    return n;
}

static long long FN(integrate_dda)(ora_map *m, const float *depth, int width, int height, const float K[4],
                                   const float T[16])
{
    FN(frame) f;
    FN(frame_setup)(&f, &m->p, depth, width, height, K, T);
    m->n_touched = 0;
    uint64_t *keys = 0;
    long long nk = FN(dda_keys)(&f, T, &keys);
    if (nk < 0)
        return -1;
    qsort(keys, (size_t)nk, sizeof(uint64_t), key_cmp);
    long long updates = 0;
    REAL xs[512], ws[512];
    unsigned char hit[512];
    for (long long q = 0; q < nk; ++q) {
        if (q > 0 && keys[q] == keys[q - 1])
            continue;
        const int32_t bx = (int32_t)((keys[q] >> 42) & 0x1FFFFF) - (1 << 20);
        const int32_t by = (int32_t)((keys[q] >> 21) & 0x1FFFFF) - (1 << 20);
        const int32_t bz = (int32_t)(keys[q] & 0x1FFFFF) - (1 << 20);
        for (int k = 0; k < 512; ++k)
            hit[k] = (unsigned char)FN(voxel_measure)(&f, 8 * bx + (k & 7), 8 * by + ((k >> 3) & 7),
                                                      8 * bz + (k >> 6), &xs[k], &ws[k]);
        long long b = map_find_or_insert(m, bx, by, bz);
        if (b < 0 || touched_push(m, b) != 0) {
            free(keys);
            return -1;
        }
        REAL *D = FN(dist_ptr)(m) + 512 * b;
        REAL *W = FN(weight_ptr)(m) + 512 * b;
        for (int k = 0; k < 512; ++k)
            if (hit[k]) {
                FN(voxel_fuse)(&D[k], &W[k], xs[k], ws[k], f.w_max);
                if (m->storage16) {
                    D[k] = (REAL)ora_round_binary16((float)D[k]);
                    W[k] = (REAL)ora_round_binary16((float)W[k]);
                }
                ++updates;
            }
    }
    free(keys);
    return updates;
}

static long long FN(integrate_prepared)(ora_map *m, FN(frame) *fp, const float K[4], const float *model,
                                        const float T[16])
{
    FN(frame) f = *fp;
    m->n_touched = 0;
    int32_t bmin[3], bmax[3];
    const int any_valid = model ? FN(scan_box_range)(&f, model, T, bmin, bmax) : FN(scan_box)(&f, K, T, bmin, bmax);
    if (!any_valid) {
        for (int a = 0; a < 3; ++a) { m->scan_min[a] = 0; m->scan_max[a] = -1; }
        return 0;
    }
    for (int a = 0; a < 3; ++a) { m->scan_min[a] = bmin[a]; m->scan_max[a] = bmax[a]; }
    long long updates = 0;
    REAL xs[512], ws[512];
    unsigned char hit[512];
    for (int32_t bz = bmin[2]; bz <= bmax[2]; ++bz)
        for (int32_t by = bmin[1]; by <= bmax[1]; ++by)
            for (int32_t bx = bmin[0]; bx <= bmax[0]; ++bx) {
                int any = 0;
                for (int lz = 0; lz < 8; ++lz)
                    for (int ly = 0; ly < 8; ++ly)
                        for (int lx = 0; lx < 8; ++lx) {
                            int k = lx + 8 * ly + 64 * lz;
                            hit[k] = (unsigned char)(model
                                ? FN(voxel_measure_range)(&f, 8 * bx + lx, 8 * by + ly, 8 * bz + lz, &xs[k], &ws[k])
                                : FN(voxel_measure)(&f, 8 * bx + lx, 8 * by + ly, 8 * bz + lz, &xs[k], &ws[k]));
                            any |= hit[k];
                        }
                if (!any)
                    continue;
                long long b = map_find_or_insert(m, bx, by, bz);
                if (b < 0)
                    return -1;
                if (touched_push(m, b) != 0)
                    return -1;
                REAL *D = FN(dist_ptr)(m) + 512 * b;
                REAL *W = FN(weight_ptr)(m) + 512 * b;
                for (int k = 0; k < 512; ++k)
                    if (hit[k]) {
                        FN(voxel_fuse)(&D[k], &W[k], xs[k], ws[k], f.w_max);
                        if (m->storage16) {
                            D[k] = (REAL)ora_round_binary16((float)D[k]);
                            W[k] = (REAL)ora_round_binary16((float)W[k]);
                        }
                        ++updates;
                    }
            }
    return updates;
}

static long long FN(integrate)(ora_map *m, const float *depth, int width, int height,
                               const float K[4], const float T[16])
{
    return FN(integrate_any)(m, depth, width, height, K, NULL, T);
}

/* The same frame as FN(integrate), spread over `threads` OpenMP threads for
 * timing the CPU baseline on all host cores.  The scan box is taken in the
 * same block order in chunks: the chunk's blocks are measured in parallel
 * (each voxel exactly as above, into per-block buffers), then looked up or
 * inserted one after the other in scan order, so the map receives the same
 * block indices in the same order, then fused in parallel (distinct blocks).
 * The result is bitwise the single-threaded one. */
static long long FN(integrate_threads)(ora_map *m, const float *depth, int width, int height, const float K[4],
                                       const float T[16], int threads)
{
    enum { CHUNK = 2048 };
    FN(frame) f;
    FN(frame_setup)(&f, &m->p, depth, width, height, K, T);
    m->n_touched = 0;
    int32_t bmin[3], bmax[3];
    if (!FN(scan_box)(&f, K, T, bmin, bmax)) {
        for (int a = 0; a < 3; ++a) { m->scan_min[a] = 0; m->scan_max[a] = -1; }
        return 0;
    }
    for (int a = 0; a < 3; ++a) { m->scan_min[a] = bmin[a]; m->scan_max[a] = bmax[a]; }
    const long long nx = (long long)bmax[0] - bmin[0] + 1, ny = (long long)bmax[1] - bmin[1] + 1;
    const long long nz = (long long)bmax[2] - bmin[2] + 1, n_lat = nx * ny * nz;
    REAL *xs = (REAL *)malloc((size_t)CHUNK * 512 * sizeof(REAL));
    REAL *ws = (REAL *)malloc((size_t)CHUNK * 512 * sizeof(REAL));
    unsigned char *hit = (unsigned char *)malloc((size_t)CHUNK * 512);
    unsigned char *any = (unsigned char *)malloc(CHUNK);
    long long *slot = (long long *)malloc((size_t)CHUNK * sizeof(long long));
    long long updates = 0;
    int failed = !xs || !ws || !hit || !any || !slot;
    for (long long c0 = 0; c0 < n_lat && !failed; c0 += CHUNK) {
        const int nc = (int)(n_lat - c0 < CHUNK ? n_lat - c0 : CHUNK);
#pragma omp parallel for num_threads(threads) schedule(dynamic, 16)
        for (int q = 0; q < nc; ++q) {
            const long long lb = c0 + q;   /* scan order: x fastest, then y, then z */
            const int32_t bx = bmin[0] + (int32_t)(lb % nx), by = bmin[1] + (int32_t)((lb / nx) % ny),
                          bz = bmin[2] + (int32_t)(lb / (nx * ny));
            int a = 0;
            for (int k = 0; k < 512; ++k) {
                hit[512 * q + k] = (unsigned char)FN(voxel_measure)(&f, 8 * bx + (k & 7), 8 * by + ((k >> 3) & 7),
                                                                     8 * bz + (k >> 6), &xs[512 * q + k],
                                                                     &ws[512 * q + k]);
                a |= hit[512 * q + k];
            }
            any[q] = (unsigned char)a;
        }
        for (int q = 0; q < nc && !failed; ++q) {
            slot[q] = -1;
            if (!any[q])
                continue;
            const long long lb = c0 + q;
            slot[q] = map_find_or_insert(m, bmin[0] + (int32_t)(lb % nx), bmin[1] + (int32_t)((lb / nx) % ny),
                                         bmin[2] + (int32_t)(lb / (nx * ny)));
            if (slot[q] < 0 || touched_push(m, slot[q]) != 0)
                failed = 1;
        }
        if (failed)
            break;
        long long n_upd = 0;
#pragma omp parallel for num_threads(threads) schedule(dynamic, 16) reduction(+ : n_upd)
        for (int q = 0; q < nc; ++q) {
            if (slot[q] < 0)
                continue;
            REAL *D = FN(dist_ptr)(m) + 512 * slot[q];
            REAL *W = FN(weight_ptr)(m) + 512 * slot[q];
            for (int k = 0; k < 512; ++k)
                if (hit[512 * q + k]) {
                    FN(voxel_fuse)(&D[k], &W[k], xs[512 * q + k], ws[512 * q + k], f.w_max);
                    if (m->storage16) {
                        D[k] = (REAL)ora_round_binary16((float)D[k]);
                        W[k] = (REAL)ora_round_binary16((float)W[k]);
                    }
                    ++n_upd;
                }
        }
        updates += n_upd;
    }
    free(xs);
    free(ws);
    free(hit);
    free(any);
    free(slot);
    return failed ? -1 : updates;
}

static void FN(export_voxels)(const ora_map *m, double *dist, double *weight)
{
    const REAL *D = (const REAL *)m->dist;
    const REAL *W = (const REAL *)m->weight;
    for (long long k = 0; k < 512 * m->n_blocks; ++k) {
        dist[k] = (double)D[k];
        weight[k] = (double)W[k];
    }
}

static long long FN(dense)(const ora_params *p, const float *depth, int width, int height,
                           const float K[4], const float T[16],
                           const int32_t gmin[3], const int32_t gdim[3],
                           double *dist, double *weight)
{
    FN(frame) f;
    FN(frame_setup)(&f, p, depth, width, height, K, T);
    long long updates = 0;
    size_t k = 0;
    for (int32_t z = 0; z < gdim[2]; ++z)
        for (int32_t y = 0; y < gdim[1]; ++y)
            for (int32_t x = 0; x < gdim[0]; ++x, ++k) {
                REAL xv, wv;
                if (!FN(voxel_measure)(&f, gmin[0] + x, gmin[1] + y, gmin[2] + z, &xv, &wv))
                    continue;
                REAL D = (REAL)dist[k], W = (REAL)weight[k];
                FN(voxel_fuse)(&D, &W, xv, wv, f.w_max);
                dist[k] = (double)D;
                weight[k] = (double)W;
                ++updates;
            }
    return updates;
}

static long long FN(dense_range)(const ora_params *p, const float *range, int width, int height,
                                 const float model[6], const float T[16],
                                 const int32_t gmin[3], const int32_t gdim[3], double *dist, double *weight)
{
    FN(frame) f;
    FN(range_setup)(&f, p, range, width, height, model, T);
    long long updates = 0;
    size_t k = 0;
    for (int32_t z = 0; z < gdim[2]; ++z)
        for (int32_t y = 0; y < gdim[1]; ++y)
            for (int32_t x = 0; x < gdim[0]; ++x, ++k) {
                REAL xv, wv;
                if (!FN(voxel_measure_range)(&f, gmin[0] + x, gmin[1] + y, gmin[2] + z, &xv, &wv))
                    continue;
                REAL D = (REAL)dist[k], W = (REAL)weight[k];
                FN(voxel_fuse)(&D, &W, xv, wv, f.w_max);
                dist[k] = (double)D;
                weight[k] = (double)W;
                ++updates;
            }
    return updates;
}

static void FN(camera_from_world)(const float T[16], double R[9], double t[3])
{
    ora_params p = {0};
    p.voxel_size = 1.0f;
    p.truncation_vox = 1.0f;
    FN(frame) f;
    float K[4] = {1, 1, 0, 0};
    FN(frame_setup)(&f, &p, 0, 1, 1, K, T);
    for (int k = 0; k < 9; ++k) R[k] = (double)f.R[k];
    for (int k = 0; k < 3; ++k) t[k] = (double)f.t[k];
}

#undef FN
#undef FN2
#undef FN_

/*
 * sensor_model_impl.h -- the learned sensor model of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see tsdf_oracle.h).  Included once, at the end of
 * tsdf_oracle.c.
 *
 * The paper lets the measurement weight follow the sensor's error model
 * (§IV-B, TSDF update).  Here that model is a per-pixel multilayer perceptron
 * 27 -> 32 -> 32 -> 2 evaluated on the pixel's neighbourhood:
 *   inputs   x[0..24]  depth differences q - d over the 5 x 5 patch centred
 *                      on the pixel (row-major, the centre is 0), clipped to
 *                      [-0.5, 0.5] m, 0 where q is outside the image or invalid;
 *            x[25]     the depth d;
 *            x[26]     the incidence angle between the viewing ray and the
 *                      normal of the back-projected depth (central
 *                      differences), pi/2 when a 4-neighbour is missing;
 *   hidden   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2);
 *   outputs  o = W3 h2 + b3;  weight w = (o0 + sqrt(o0^2 + 4)) / 2 > 0;
 *            truncation eps = vs (1 + 7 s), s = (1 + o1 / sqrt(1 + o1^2)) / 2,
 *            so eps lies in (vs, 8 vs).
 * Both output maps are algebraic (sqrt and division only) so that every
 * implementation computes them with correctly rounded operations; o = 0 gives
 * w = 1 and eps = 4.5 vs exactly.
 *
 * Inference precision: parameters are bfloat16 values; inputs and hidden
 * activations are rounded to bfloat16 (round to nearest, ties to even); every
 * sum is accumulated in binary32 in index order, starting from the bias, one
 * fused multiply-add (a single rounding) per term.  The outputs are binary32.
 *
 * Parameter layout (2018 floats): W1[32][27], b1[32], W2[32][32], b2[32],
 * W3[2][32], b3[2], row-major (output index first).
 */

enum {
    SM_IN = 27, SM_H = 32, SM_OUT = 2,
    SM_W1 = 0, SM_B1 = SM_W1 + SM_H * SM_IN, SM_W2 = SM_B1 + SM_H, SM_B2 = SM_W2 + SM_H * SM_H,
    SM_W3 = SM_B2 + SM_H, SM_B3 = SM_W3 + SM_OUT * SM_H, SM_NPARAM = SM_B3 + SM_OUT
};

float ora_round_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u)
        return x;                                  /* infinities and NaN */
    u += 0x7fffu + ((u >> 16) & 1u);                /* nearest, ties to even */
    u &= 0xffff0000u;
    memcpy(&x, &u, 4);
    return x;
}

static int sm_valid(float d, float d_max) { return d > 0.0f && d <= d_max; }

/* binary32 incidence angle at pixel (i, j) of depth d. */
static float sm_incidence_f32(const float *D, int W, int H, const float K[4], float d_max, int i, int j, float d)
{
    const float half_pi = 1.57079637f;
    if (i < 1 || i > W - 2 || j < 1 || j > H - 2)
        return half_pi;
    const float dl = D[(size_t)j * W + i - 1], dr = D[(size_t)j * W + i + 1];
    const float du = D[(size_t)(j - 1) * W + i], dd = D[(size_t)(j + 1) * W + i];
    if (!(sm_valid(dl, d_max) && sm_valid(dr, d_max) && sm_valid(du, d_max) && sm_valid(dd, d_max)))
        return half_pi;
    /* back-projection of pixel centres: P = depth ((c + 0.5 - cx) / fx, (r + 0.5 - cy) / fy, 1) */
    const float rxl = (((float)(i - 1) + 0.5f) - K[2]) / K[0], rxc = (((float)i + 0.5f) - K[2]) / K[0];
    const float rxr = (((float)(i + 1) + 0.5f) - K[2]) / K[0];
    const float ryu = (((float)(j - 1) + 0.5f) - K[3]) / K[1], ryc = (((float)j + 0.5f) - K[3]) / K[1];
    const float ryd = (((float)(j + 1) + 0.5f) - K[3]) / K[1];
    const float ax = dr * rxr - dl * rxl, ay = dr * ryc - dl * ryc, az = dr - dl;
    const float bx = dd * rxc - du * rxc, by = dd * ryd - du * ryu, bz = dd - du;
    const float nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const float px = d * rxc, py = d * ryc, pz = d;
    const float dot = (nx * px + ny * py) + nz * pz;
    const float cx = ny * pz - nz * py, cy = nz * px - nx * pz, cz = nx * py - ny * px;
    const float cr = sqrtf((cx * cx + cy * cy) + cz * cz);
    return ora_atan2_f32(cr, fabsf(dot));
}

void ora_sm_features(const float *D, int W, int H, const float K[4], float d_max, float *feat)
{
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            float *f = feat + (size_t)SM_IN * ((size_t)j * W + i);
            const float d = D[(size_t)j * W + i];
            if (!sm_valid(d, d_max)) {
                for (int k = 0; k < SM_IN; ++k)
                    f[k] = 0.0f;
                continue;
            }
            for (int dj = -2; dj <= 2; ++dj)
                for (int di = -2; di <= 2; ++di) {
                    const int ii = i + di, jj = j + dj;
                    float v = 0.0f;
                    if (ii >= 0 && ii < W && jj >= 0 && jj < H) {
                        const float q = D[(size_t)jj * W + ii];
                        if (sm_valid(q, d_max)) {
                            v = q - d;
                            v = v < -0.5f ? -0.5f : (v > 0.5f ? 0.5f : v);
                        }
                    }
                    f[(dj + 2) * 5 + (di + 2)] = v;
                }
            f[25] = d;
            f[26] = sm_incidence_f32(D, W, H, K, d_max, i, j, d);
        }
}

/* bfloat16-emulating binary32 forward of one pixel. */
static void sm_forward_f32(const float *P, const float *feat, float vs, float *w, float *e)
{
    float x[SM_IN], h1[SM_H], h2[SM_H], o[SM_OUT];
    for (int m = 0; m < SM_IN; ++m)
        x[m] = ora_round_bf16(feat[m]);
    for (int k = 0; k < SM_H; ++k) {
        float a = P[SM_B1 + k];
        for (int m = 0; m < SM_IN; ++m)
            a = fmaf(P[SM_W1 + SM_IN * k + m], x[m], a);
        h1[k] = ora_round_bf16(a > 0.0f ? a : 0.0f);
    }
    for (int k = 0; k < SM_H; ++k) {
        float a = P[SM_B2 + k];
        for (int m = 0; m < SM_H; ++m)
            a = fmaf(P[SM_W2 + SM_H * k + m], h1[m], a);
        h2[k] = ora_round_bf16(a > 0.0f ? a : 0.0f);
    }
    for (int c = 0; c < SM_OUT; ++c) {
        float a = P[SM_B3 + c];
        for (int m = 0; m < SM_H; ++m)
            a = fmaf(P[SM_W3 + SM_H * c + m], h2[m], a);
        o[c] = a;
    }
    *w = 0.5f * (o[0] + sqrtf(o[0] * o[0] + 4.0f));
    const float s = 0.5f + 0.5f * (o[1] / sqrtf(1.0f + o[1] * o[1]));
    *e = vs * (1.0f + 7.0f * s);
}

int ora_sm_maps(const float *D, int W, int H, const float K[4], float d_max, float vs, const float *params,
                float *w_map, float *eps_map)
{
    if (!D || !K || !params || !w_map || !eps_map || W <= 0 || H <= 0)
        return -1;
    float *feat = (float *)malloc((size_t)W * H * SM_IN * sizeof(float));
    if (!feat)
        return -1;
    ora_sm_features(D, W, H, K, d_max, feat);
    for (size_t k = 0; k < (size_t)W * H; ++k) {
        if (sm_valid(D[k], d_max)) {
            sm_forward_f32(params, feat + SM_IN * k, vs, &w_map[k], &eps_map[k]);
        } else {
            w_map[k] = 0.0f;
            eps_map[k] = 0.0f;
        }
    }
    free(feat);
    return 0;
}

long long ora_integrate_learned(ora_map *m, const float *depth, int width, int height, const float K[4],
                                const float T[16], const float *w_map, const float *eps_map)
{
    if (!m || !w_map || !eps_map || !frame_args_ok(depth, width, height, K, T))
        return -1;
    return m->precision == 32 ? integrate_learned_f32(m, depth, width, height, K, T, w_map, eps_map)
                              : integrate_learned_f64(m, depth, width, height, K, T, w_map, eps_map);
}

/* ------------------------------------------------------------------------
 * Training loss and its gradient, in binary64.
 *
 * For a window of frames and a list of target voxels v (global indices) with
 * target distances D*(v): every frame f whose pixel p_f(v) updates v under
 * the model's (w, eps) contributes x_f = min(d_p, eps_f) with weight w_f; the
 * prediction is the uncapped weighted average D(v) = sum w_f x_f / sum w_f
 * (the fused distance before any weight cap), and
 *   L = (1 / N) sum_v (D(v) - D*(v))^2  over the N voxels with sum w_f > 0.
 * dD/dw_f = (x_f - D) / sum w;  dD/dx_f = w_f / sum w;  dx_f/deps_f = 1 when
 * the clamp is active (d_p > eps_f), else 0; the band test d_p >= -eps_f is a
 * discrete decision and carries no gradient.  The perceptron is
 * differentiated through its ReLUs; with emulate_bf16 the forward rounds
 * inputs and hidden activations to bfloat16 as inference does, and the
 * backward treats those roundings as the identity.
 * ---------------------------------------------------------------------- */

static double sm_round_d(double v, int emulate) { return emulate ? (double)ora_round_bf16((float)v) : v; }

static double sm_incidence_f64(const float *D, int W, int H, const float K[4], float d_max, int i, int j, double d)
{
    const double half_pi = 1.5707963267948966;
    if (i < 1 || i > W - 2 || j < 1 || j > H - 2)
        return half_pi;
    const double dl = D[(size_t)j * W + i - 1], dr = D[(size_t)j * W + i + 1];
    const double du = D[(size_t)(j - 1) * W + i], dd = D[(size_t)(j + 1) * W + i];
    if (!(sm_valid((float)dl, d_max) && sm_valid((float)dr, d_max) && sm_valid((float)du, d_max) &&
          sm_valid((float)dd, d_max)))
        return half_pi;
    const double fx = K[0], fy = K[1], cxk = K[2], cyk = K[3];
    const double rxl = ((i - 1) + 0.5 - cxk) / fx, rxc = (i + 0.5 - cxk) / fx, rxr = ((i + 1) + 0.5 - cxk) / fx;
    const double ryu = ((j - 1) + 0.5 - cyk) / fy, ryc = (j + 0.5 - cyk) / fy, ryd = ((j + 1) + 0.5 - cyk) / fy;
    const double ax = dr * rxr - dl * rxl, ay = dr * ryc - dl * ryc, az = dr - dl;
    const double bx = dd * rxc - du * rxc, by = dd * ryd - du * ryu, bz = dd - du;
    const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const double px = d * rxc, py = d * ryc, pz = d;
    const double dot = nx * px + ny * py + nz * pz;
    const double cx = ny * pz - nz * py, cy = nz * px - nx * pz, cz = nx * py - ny * px;
    return atan2(sqrt(cx * cx + cy * cy + cz * cz), fabs(dot));
}

typedef struct {
    double x[SM_IN], a1[SM_H], h1[SM_H], a2[SM_H], h2[SM_H], o[SM_OUT], w, e;
} sm_pixel;

static void sm_forward_f64(const float *P, const float *D, int W, int H, const float K[4], float d_max, double vs,
                           int i, int j, int emulate, sm_pixel *px)
{
    const double d = D[(size_t)j * W + i];
    for (int dj = -2; dj <= 2; ++dj)
        for (int di = -2; di <= 2; ++di) {
            const int ii = i + di, jj = j + dj;
            double v = 0.0;
            if (ii >= 0 && ii < W && jj >= 0 && jj < H) {
                const float q = D[(size_t)jj * W + ii];
                if (sm_valid(q, d_max)) {
                    v = (double)q - d;
                    v = v < -0.5 ? -0.5 : (v > 0.5 ? 0.5 : v);
                }
            }
            px->x[(dj + 2) * 5 + (di + 2)] = sm_round_d(v, emulate);
        }
    px->x[25] = sm_round_d(d, emulate);
    px->x[26] = sm_round_d(sm_incidence_f64(D, W, H, K, d_max, i, j, d), emulate);
    for (int k = 0; k < SM_H; ++k) {
        double a = P[SM_B1 + k];
        for (int m = 0; m < SM_IN; ++m)
            a += (double)P[SM_W1 + SM_IN * k + m] * px->x[m];
        px->a1[k] = a;
        px->h1[k] = sm_round_d(a > 0 ? a : 0, emulate);
    }
    for (int k = 0; k < SM_H; ++k) {
        double a = P[SM_B2 + k];
        for (int m = 0; m < SM_H; ++m)
            a += (double)P[SM_W2 + SM_H * k + m] * px->h1[m];
        px->a2[k] = a;
        px->h2[k] = sm_round_d(a > 0 ? a : 0, emulate);
    }
    for (int c = 0; c < SM_OUT; ++c) {
        double a = P[SM_B3 + c];
        for (int m = 0; m < SM_H; ++m)
            a += (double)P[SM_W3 + SM_H * c + m] * px->h2[m];
        px->o[c] = a;
    }
    px->w = 0.5 * (px->o[0] + sqrt(px->o[0] * px->o[0] + 4.0));
    const double s = 0.5 + 0.5 * (px->o[1] / sqrt(1.0 + px->o[1] * px->o[1]));
    px->e = vs * (1.0 + 7.0 * s);
}

double ora_sm_loss_grad(const float *params, int n_frames, const float *depths, int W, int H, const float K[4],
                        const float *T, float voxel_size, float d_max, long long n_vox, const int32_t *vox,
                        const double *target, int emulate_bf16, double *grad, long long *n_used)
{
    const size_t npx = (size_t)W * H;
    sm_pixel *pxs = (sm_pixel *)calloc((size_t)n_frames * npx, sizeof(sm_pixel));
    unsigned char *ok = (unsigned char *)calloc((size_t)n_frames * npx, 1);
    double *gw = (double *)calloc((size_t)n_frames * npx, sizeof(double));
    double *ge = (double *)calloc((size_t)n_frames * npx, sizeof(double));
    double (*cam)[12] = (double (*)[12])malloc((size_t)n_frames * sizeof(double[12]));
    if (!pxs || !ok || !gw || !ge || !cam) {
        free(pxs); free(ok); free(gw); free(ge); free(cam);
        return -1.0;
    }
    const double vs = voxel_size;
    for (int f = 0; f < n_frames; ++f) {
        double R[9], t[3];
        camera_from_world_f64(T + 16 * f, R, t);
        for (int k = 0; k < 9; ++k) cam[f][k] = R[k];
        for (int k = 0; k < 3; ++k) cam[f][9 + k] = t[k];
        const float *D = depths + (size_t)f * npx;
        for (int j = 0; j < H; ++j)
            for (int i = 0; i < W; ++i) {
                const size_t k = (size_t)j * W + i;
                if (!sm_valid(D[k], d_max))
                    continue;
                ok[f * npx + k] = 1;
                sm_forward_f64(params, D, W, H, K, d_max, vs, i, j, emulate_bf16, &pxs[f * npx + k]);
            }
    }
    /* fusion, loss and the gradient with respect to each pixel's (w, eps) */
    double loss = 0.0;
    long long used = 0;
    for (long long v = 0; v < n_vox; ++v) {
        const double p[3] = {((double)vox[3 * v] + 0.5) * vs, ((double)vox[3 * v + 1] + 0.5) * vs,
                             ((double)vox[3 * v + 2] + 0.5) * vs};
        double sw = 0.0, swx = 0.0, Dp = 0.0, gD = 0.0;
        for (int stage = 0; stage < 2; ++stage) {
            for (int f = 0; f < n_frames; ++f) {
                const double *c = cam[f];
                const double xc = c[0] * p[0] + c[1] * p[1] + c[2] * p[2] + c[9];
                const double yc = c[3] * p[0] + c[4] * p[1] + c[5] * p[2] + c[10];
                const double zc = c[6] * p[0] + c[7] * p[1] + c[8] * p[2] + c[11];
                if (!(zc > 0))
                    continue;
                const double u = K[0] * (xc / zc) + K[2], vv = K[1] * (yc / zc) + K[3];
                if (!(u >= 0 && u < W && vv >= 0 && vv < H))
                    continue;
                const size_t k = (size_t)(int)vv * W + (size_t)(int)u;
                if (!ok[f * npx + k])
                    continue;
                const sm_pixel *q = &pxs[f * npx + k];
                const double dp = (double)depths[f * npx + k] - zc;
                if (!(dp >= -q->e) || !(q->w > 0))
                    continue;
                const double x = dp < q->e ? dp : q->e;
                if (stage == 0) {
                    sw += q->w;
                    swx += q->w * x;
                } else {
                    gw[f * npx + k] += gD * (x - Dp) / sw;
                    if (dp > q->e)
                        ge[f * npx + k] += gD * q->w / sw;
                }
            }
            if (stage == 0) {
                if (!(sw > 0))
                    break;
                Dp = swx / sw;
                gD = 2.0 * (Dp - target[v]);
                loss += (Dp - target[v]) * (Dp - target[v]);
                ++used;
            }
        }
    }
    for (int k = 0; k < SM_NPARAM; ++k)
        grad[k] = 0.0;
    const double scale = used > 0 ? 1.0 / (double)used : 0.0;
    for (size_t k = 0; k < (size_t)n_frames * npx; ++k) {
        if (!ok[k] || (gw[k] == 0.0 && ge[k] == 0.0))
            continue;
        const sm_pixel *q = &pxs[k];
        double go[SM_OUT];
        go[0] = scale * gw[k] * 0.5 * (1.0 + q->o[0] / sqrt(q->o[0] * q->o[0] + 4.0));
        const double r = 1.0 + q->o[1] * q->o[1];
        go[1] = scale * ge[k] * vs * 7.0 * 0.5 / (r * sqrt(r));
        double gh2[SM_H], gh1[SM_H];
        for (int m = 0; m < SM_H; ++m)
            gh2[m] = 0.0;
        for (int c = 0; c < SM_OUT; ++c) {
            grad[SM_B3 + c] += go[c];
            for (int m = 0; m < SM_H; ++m) {
                grad[SM_W3 + SM_H * c + m] += go[c] * q->h2[m];
                gh2[m] += (double)params[SM_W3 + SM_H * c + m] * go[c];
            }
        }
        for (int m = 0; m < SM_H; ++m)
            gh1[m] = 0.0;
        for (int kk = 0; kk < SM_H; ++kk) {
            const double ga = q->a2[kk] > 0 ? gh2[kk] : 0.0;
            grad[SM_B2 + kk] += ga;
            for (int m = 0; m < SM_H; ++m) {
                grad[SM_W2 + SM_H * kk + m] += ga * q->h1[m];
                gh1[m] += (double)params[SM_W2 + SM_H * kk + m] * ga;
            }
        }
        for (int kk = 0; kk < SM_H; ++kk) {
            const double ga = q->a1[kk] > 0 ? gh1[kk] : 0.0;
            grad[SM_B1 + kk] += ga;
            for (int m = 0; m < SM_IN; ++m)
                grad[SM_W1 + SM_IN * kk + m] += ga * q->x[m];
        }
    }
    if (n_used)
        *n_used = used;
    free(pxs); free(ok); free(gw); free(ge); free(cam);
    return used > 0 ? loss / (double)used : 0.0;
}

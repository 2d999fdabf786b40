/* Host-side driver for the sanitizer test: calls every entry point of the C
 * ABI with invalid arguments (and the creation path, which on a machine
 * without a GPU fails at its first device call), checks each status, and
 * exits 0 when all match.  Built and linked with AddressSanitizer and
 * UndefinedBehaviorSanitizer against a library whose host code carries the
 * same instrumentation, so any out-of-bounds access, use of freed memory or
 * undefined behaviour on these paths aborts the run. */
#include "tsdf.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

static int failures = 0;

#define EXPECT(call, want)                                                                     \
    do {                                                                                       \
        const int got_ = (call);                                                               \
        if (got_ != (want)) {                                                                  \
            fprintf(stderr, "%s:%d: %s returned %d, expected %d\n", __FILE__, __LINE__, #call, \
                    got_, (int)(want));                                                        \
            ++failures;                                                                        \
        }                                                                                      \
    } while (0)

int main(void)
{
    tsdf_map *m = (tsdf_map *)0x1;
    const float K[4] = {500.0f, 500.0f, 320.0f, 240.0f};
    const float Kbad[4] = {0.0f, 500.0f, 320.0f, 240.0f};
    const float I[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    float shear[16];
    memcpy(shear, I, sizeof(I));
    shear[1] = 0.5f;                       /* not a rotation */
    float nanpose[16];
    memcpy(nanpose, I, sizeof(I));
    nanpose[3] = NAN;
    long long n = -1;
    tsdf_stats st;
    tsdf_params p;

    /* creation: bad parameters never reach the device */
    EXPECT(create_map(0.0f, 4.0f, &m), TSDF_EINVAL);
    if (m != NULL) {
        fprintf(stderr, "create_map left a handle after EINVAL\n");
        ++failures;
    }
    EXPECT(create_map(0.05f, -1.0f, &m), TSDF_EINVAL);
    EXPECT(create_map(NAN, 4.0f, &m), TSDF_EINVAL);
    EXPECT(create_map(0.05f, 4.0f, NULL), TSDF_EINVAL);
    EXPECT(create_map_ex(NULL, &m), TSDF_EINVAL);
    tsdf_default_params(&p, 0.05f, 4.0f);
    tsdf_default_params(NULL, 0.05f, 4.0f);
    p.hash_capacity = 3;
    EXPECT(create_map_ex(&p, &m), TSDF_EINVAL);
    tsdf_default_params(&p, 0.05f, 4.0f);
    p.block_capacity = 1024;
    p.hash_capacity = 512;
    EXPECT(create_map_ex(&p, &m), TSDF_EINVAL);
    tsdf_default_params(&p, 0.05f, 4.0f);
    p.weighting = 9;
    EXPECT(create_map_ex(&p, &m), TSDF_EINVAL);
    tsdf_default_params(&p, 0.05f, 4.0f);
    p.allocation = TSDF_ALLOC_RAY_WALK;
    p.weighting = TSDF_WEIGHT_LEARNED;
    EXPECT(create_map_ex(&p, &m), TSDF_EINVAL);

    /* valid parameters: succeeds on a GPU machine, fails cleanly without one */
    tsdf_default_params(&p, 0.05f, 4.0f);
    p.block_capacity = 64;
    m = NULL;
    const int cs = create_map_ex(&p, &m);
    if (cs == TSDF_OK) {
        EXPECT(reserve(m, 0), TSDF_EINVAL);
        EXPECT(reserve(m, (1ll << 30) + 1), TSDF_EINVAL);
        EXPECT(reserve(m, 32), TSDF_OK);
        EXPECT(integrate_depth(m, NULL, 640, 480, K, I, NULL), TSDF_EINVAL);
        EXPECT(integrate_depth(m, (const float *)16, 0, 480, K, I, NULL), TSDF_EINVAL);
        EXPECT(integrate_depth(m, (const float *)16, 640, 480, Kbad, I, NULL), TSDF_EINVAL);
        EXPECT(integrate_depth(m, (const float *)16, 640, 480, K, shear, NULL), TSDF_EINVAL);
        EXPECT(integrate_depth(m, (const float *)16, 640, 480, K, nanpose, NULL), TSDF_EINVAL);
        EXPECT(integrate_depth(m, (const float *)16, 1 << 20, 1 << 20, K, I, NULL), TSDF_EINVAL);
        EXPECT(integrate_depth_noalloc(m, NULL, 640, 480, K, I, NULL), TSDF_EINVAL);
        EXPECT(integrate_depth_noalloc(m, (const float *)16, 640, 480, K, shear, NULL), TSDF_EINVAL);
        EXPECT(insert_blocks(m, NULL, 1, (const float *)16, (const float *)16, NULL), TSDF_EINVAL);
        EXPECT(insert_blocks(m, (const int32_t *)16, -1, (const float *)16, (const float *)16, NULL), TSDF_EINVAL);
        EXPECT(insert_blocks(m, NULL, 0, NULL, NULL, NULL), TSDF_OK);
        EXPECT(destroy_map(m), TSDF_OK);
    } else if (cs != TSDF_EDEVICE && cs != TSDF_ENOMEM) {
        fprintf(stderr, "create_map_ex returned %d\n", cs);
        ++failures;
    }

    /* every entry point on a NULL map */
    m = NULL;
    EXPECT(reserve(NULL, 1024), TSDF_EINVAL);
    EXPECT(integrate_depth(NULL, (const float *)16, 4, 4, K, I, NULL), TSDF_EINVAL);
    EXPECT(integrate_depth_noalloc(NULL, (const float *)16, 4, 4, K, I, NULL), TSDF_EINVAL);
    EXPECT(insert_blocks(NULL, (const int32_t *)16, 1, (const float *)16, (const float *)16, NULL), TSDF_EINVAL);
    tsdf_lidar_model lm = {1024, 64, 0.0f, 6.2831855f, 1.2915f, 0.5585f, 0.2f, 25.0f};
    EXPECT(integrate_range(NULL, (const float *)16, &lm, I, NULL), TSDF_EINVAL);
    EXPECT(integrate_range(NULL, (const float *)16, NULL, I, NULL), TSDF_EINVAL);
    tsdf_depth_view views[2];
    memset(views, 0, sizeof(views));
    EXPECT(integrate_depth_views(NULL, views, 1, NULL), TSDF_EINVAL);
    EXPECT(query_blocks(NULL, NULL, 0, &n, NULL), TSDF_EINVAL);
    EXPECT(query_touched(NULL, NULL, 0, &n, NULL), TSDF_EINVAL);
    EXPECT(query_tsdf(NULL, NULL, 0, NULL, NULL, NULL), TSDF_EINVAL);
    EXPECT(map_stats(NULL, &st, NULL), TSDF_EINVAL);
    EXPECT(map_status(NULL), TSDF_EINVAL);
    EXPECT(destroy_map(NULL), TSDF_OK);
    tsdf_step *step = (tsdf_step *)0x1;
    EXPECT(tsdf_step_create(NULL, 0, &step), TSDF_EINVAL);
    EXPECT(tsdf_step_create(NULL, 0, NULL), TSDF_EINVAL);
    EXPECT(tsdf_step_run(NULL, views, 1, NULL), TSDF_EINVAL);
    EXPECT(tsdf_step_destroy(NULL), TSDF_OK);
    tsdf_launch_config lc = {0, 0, 0, 0, 0, 0};
    EXPECT(tsdf_set_launch_config(NULL, &lc), TSDF_EINVAL);
    EXPECT(tsdf_profile(NULL, 1), TSDF_EINVAL);
    double ms = 0;
    EXPECT(tsdf_profile_read(NULL, &ms, &n), TSDF_EINVAL);
    for (int s = 1; s >= -99; --s)
        if (tsdf_strerror(s) == NULL || tsdf_strerror(s)[0] == '\0') {
            fprintf(stderr, "tsdf_strerror(%d) is empty\n", s);
            ++failures;
        }

    /* learned sensor model */
    float params[TSDF_SM_NPARAM];
    memset(params, 0, sizeof(params));
    EXPECT(tsdf_set_sensor_model(NULL, params), TSDF_EINVAL);
    EXPECT(tsdf_sensor_maps(NULL, 4, 4, K, 5.0f, 0.05f, NULL, NULL, NULL), TSDF_EINVAL);
    EXPECT(tsdf_sensor_maps((const float *)16, 4, 4, K, -5.0f, 0.05f, (const float *)16, (float *)16, NULL),
           TSDF_EINVAL);
    tsdf_sm_trainer *tr = (tsdf_sm_trainer *)0x1;
    EXPECT(tsdf_sm_trainer_create(0, 10, 1, &tr), TSDF_EINVAL);
    EXPECT(tsdf_sm_trainer_create(10, 10, TSDF_SM_MAX_FRAMES + 1, &tr), TSDF_EINVAL);
    EXPECT(tsdf_sm_trainer_create(10, 10, 1, NULL), TSDF_EINVAL);
    EXPECT(tsdf_sm_trainer_destroy(NULL), TSDF_OK);
    const float *frames[1] = {(const float *)16};
    EXPECT(tsdf_sm_loss_grad(NULL, params, 1, frames, K, I, 0.05f, 5.0f, 0, NULL, NULL, (float *)16, NULL, NULL),
           TSDF_EINVAL);
    EXPECT(tsdf_sm_adam(NULL, NULL, NULL, NULL, NULL, TSDF_SM_NPARAM, 1e-3f, 0.9f, 0.999f, 1e-8f, 1, NULL),
           TSDF_EINVAL);
    EXPECT(tsdf_sm_adam((float *)16, (float *)16, (float *)16, (const float *)16, (float *)16, TSDF_SM_NPARAM,
                        1e-3f, 0.9f, 0.999f, 1e-8f, 0, NULL),
           TSDF_EINVAL);

    if (failures == 0)
        printf("abi argument checks: all passed\n");
    return failures == 0 ? 0 : 1;
}

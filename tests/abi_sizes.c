/* Prints the size and field offsets of the ABI's structs as the C compiler
 * lays them out from include/tsdf.h, for comparison with the ctypes
 * mirrors of the Python binding. */
#include "tsdf.h"

#include <stddef.h>
#include <stdio.h>

#define FIELD(s, f) printf("%s.%s %zu\n", #s, #f, offsetof(s, f))

int main(void)
{
    printf("tsdf_params %zu\n", sizeof(tsdf_params));
    FIELD(tsdf_params, weighting);
    FIELD(tsdf_params, block_capacity);
    FIELD(tsdf_params, hash_capacity);
    FIELD(tsdf_params, allocation);
    printf("tsdf_stats %zu\n", sizeof(tsdf_stats));
    FIELD(tsdf_stats, candidate_blocks);
    FIELD(tsdf_stats, error_bits);
    printf("tsdf_launch_config %zu\n", sizeof(tsdf_launch_config));
    FIELD(tsdf_launch_config, compaction);
    FIELD(tsdf_launch_config, staging);
    printf("tsdf_depth_view %zu\n", sizeof(tsdf_depth_view));
    FIELD(tsdf_depth_view, K);
    FIELD(tsdf_depth_view, T_world_cam);
    printf("tsdf_lidar_model %zu\n", sizeof(tsdf_lidar_model));
    FIELD(tsdf_lidar_model, max_range_m);
    return 0;
}

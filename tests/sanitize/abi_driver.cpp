// Drives the host side of libtsdf (argument validation, buffer sizing, the
// marching-cubes case table, status strings) with valid and invalid
// arguments, for a build of the library's host code under AddressSanitizer
// and UndefinedBehaviorSanitizer (test infrastructure: compiled and run by
// tests/test_sanitizers.py on a machine without a GPU; no call here reaches
// the device).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "tsdf.h"
#include "tsdf_batch.h"
#include "tsdf_icp.h"
#include "tsdf_mesh.h"

static tsdf_volume_desc desc()
{
    tsdf_volume_desc d;
    memset(&d, 0, sizeof(d));
    d.dims[0] = 256, d.dims[1] = 256, d.dims[2] = 256;
    d.voxel_size = 0.004;
    d.origin[0] = -0.5, d.origin[1] = -0.5, d.origin[2] = 0.2;
    d.trunc_voxels = 4.0;
    d.capacity_blocks = 1u << 14;
    d.hash_slots = 1u << 15;
    d.storage = TSDF_F32;
    d.q_hat = 1e-4;
    d.max_width = 640, d.max_height = 480;
    d.dense_index = 1;
    return d;
}

int main()
{
    int bad = 0;
    uint64_t bytes = 0;
    tsdf_volume_desc d = desc();
    bad += tsdf_volume_bytes(&d, &bytes) != TSDF_OK || bytes == 0;
    d.storage = TSDF_F16;
    bad += tsdf_volume_bytes(&d, &bytes) != TSDF_OK;
    const int32_t bad_dims[][3] = {{250, 256, 256}, {16384, 8, 8}, {0, 8, 8}, {-8, 8, 8}, {8192, 8192, 8192}};
    for (auto &g : bad_dims) {
        tsdf_volume_desc e = desc();
        memcpy(e.dims, g, sizeof(e.dims));
        bad += tsdf_volume_bytes(&e, &bytes) == TSDF_OK && (g[0] <= 0 || g[0] % 8 || g[0] > 8192);
    }
    {
        tsdf_volume_desc e = desc();
        e.voxel_size = NAN;
        bad += tsdf_volume_bytes(&e, &bytes) != TSDF_EINVAL;
        e = desc();
        e.capacity_blocks = 0xffffffffu;
        e.hash_slots = 0x80000000u;
        bad += tsdf_volume_bytes(&e, &bytes) != TSDF_EINVAL;
        e = desc();
        e.max_width = 1 << 30;
        e.max_height = 1 << 30;
        (void)tsdf_volume_bytes(&e, &bytes);
    }
    bad += tsdf_volume_bytes(nullptr, &bytes) != TSDF_EINVAL;
    tsdf_volume *h = nullptr;
    bad += tsdf_create_volume(nullptr, nullptr, 0, nullptr, &h) != TSDF_EINVAL;
    bad += tsdf_integrate_frame(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != TSDF_EINVAL;
    bad += tsdf_raycast(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) != TSDF_EINVAL;
    bad += tsdf_query_stats(nullptr, nullptr) != TSDF_EINVAL;
    bad += tsdf_evict_workspace_bytes(nullptr) != 0 || tsdf_mesh_workspace_bytes(nullptr) != 0;
    for (int s = 0; s < 8; ++s) bad += tsdf_status_string((tsdf_status)s) == nullptr;   // the enum's range
    int32_t edges[15];
    int total = 0;
    for (int c = -2; c < 258; ++c) {
        const int n = tsdf_mesh_case(c, edges);
        bad += (c < 0 || c > 255) ? n != -1 : (n < 0 || n > 5);
        total += n > 0 ? n : 0;
    }
    bad += tsdf_icp_workspace_bytes(0, 480) != 0 || tsdf_icp_workspace_bytes(16384, 16384) == 0;
    tsdf_intrinsics K = {525.0, 525.0, 319.5, 239.5, 640, 480};
    const double eye[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    tsdf_icp_params prm = {0.02, 0.9, 0.005, 1, 0};
    bad += tsdf_icp_run(nullptr, &K, nullptr, nullptr, eye, eye, &prm, 1, nullptr, 0, nullptr, nullptr) != TSDF_EINVAL;
    bad += tsdf_icp_run_noalloc(nullptr, &K, nullptr, nullptr, eye, eye, &prm, 1, nullptr, nullptr) != TSDF_EINVAL;
    K.width = 0;
    bad += tsdf_icp_step(nullptr, &K, nullptr, nullptr, eye, nullptr, &prm, nullptr, 0, nullptr, nullptr) !=
           TSDF_EINVAL;
    bad += tsdf_batch_bytes(0) != 0 || tsdf_batch_bytes(65) != 0 || tsdf_batch_bytes(16) == 0;
    printf("host checks: %d failures, %d table triangles\n", bad, total);
    return bad == 0 && total > 0 ? 0 : 1;
}

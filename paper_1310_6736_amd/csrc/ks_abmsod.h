// Host launcher of the ABMSOD search kernel (ks_abmsod.hip).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/ks.h"
#include "ks_device.h"

namespace ks {

// Candidates: n_start start positions x R radii (r_min .. r_max); ids seed * R +
// r - r_min.
struct AbmArgs {
    long long n_start;
    int R, r_min, r_max, max_iter;
    int replicas;           // histogram replicas per wave (abmsod_replicas)
    double threshold;
};

int abmsod_replicas(int B);
size_t abmsod_lds_bytes(int B);
int abmsod_blocks_per_cu();
// One search over vols[0] (bins prepared); out: device array of n_start * R
// records; cnt->queue_head[1] must be 0.
hipError_t launch_abmsod(const VolDesc* vols, const AbmArgs& a, int B, int grid, ks_ellipsoid* out, Counters* cnt,
                         hipStream_t st);

}  // namespace ks

// Device-side data layout shared by the kernels and their host launchers.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace ks {

// Packed per-replica mean-shift accumulator (one uint64 per bin per replica),
// two's-complement fields of a sum of signed voxel terms (mod 2^64):
//   bits  0..9   net voxel count
//   bits 10..31  sum of dx'
//   bits 32..47  sum of dy'
//   bits 48..63  sum of dz'
// (d' = offset from the sweep's reference point + s).  A replica takes at most
// 511 voxels between flushes and 511 * max|d'| < 2^15, so every field decodes.
constexpr int kSmaxLimit = 32;
constexpr int kBinsLimit = 256;

// Largest count a decision table must cover: the final quadrant pass reads the
// centred cube of half-width s_max + 1.
constexpr int32_t kTableMax = (2 * (kSmaxLimit + 1) + 1) * (2 * (kSmaxLimit + 1) + 1) * (2 * (kSmaxLimit + 1) + 1);

// Decision tables, built once per context on the host (index = integer count):
//   cl[c]  = c * ln c   (cl[0] = 0)
//   sq[c]  = sqrt(c)
//   rsq[c] = 1 / sqrt(c) (rsq[0] unused)
struct Tables {
    const double* cl;
    const double* sq;
    const double* rsq;
};

// One volume of a search.
struct VolDesc {
    const void* raw;        // input voxels, dense, x fastest
    uint8_t* bins;          // bin volume, x fastest, row pitch xp (multiple of 16)
    uint8_t* bins_t;        // the same bins, y fastest: byte (x * Z + z) * yp + y
    int32_t X, Y, Z, xp;
    int64_t slice;          // xp * Y
    int32_t yp, pad2;       // y pitch of bins_t (multiple of 16)
    int64_t slice_t;        // yp * Z
    int32_t win;            // 1: window-level binning over [win_lo, win_hi]; voxels outside get bin B
    int32_t win_lo, win_hi, pad3;
    int32_t dtype, B, sp, s_min, s_max, method, max_iter;
    int32_t gx, gy, gz, ox, oy, oz;  // seed grid
    int32_t S;              // s_max - s_min + 1
    int32_t rank_by;        // output order: 0 saliency Y, 1 pdf change W
    int64_t traj_base;      // first slot of this volume in the trajectory records
    int64_t n_traj;
    double h_min, y_min;
    int32_t* minmax;        // [2] device scratch: vmin, vmax
    int64_t reg_off;        // first slot of this volume in the region output
    int32_t cap;            // region capacity of this volume
    int32_t pad1;
    const int32_t* seeds;   // explicit start positions (x, y, z) x gx, or null: the seed grid
};

// A run of tasks with the same window sizes: task task_begin + i is the i-th
// start position, x fastest, of the box [bx, bx + bw) x [by, by + bh) x [bz, ..)
// of the seed grid (or of the seed list, gx x 1 x 1) of volume `vol`: its
// quadrant trajectory, or its mean-shift trajectories of the scales scale ..
// scale_hi, run in that order by one wavefront (each starts from the previous
// one's window at the seed).
struct TaskSeg {
    int64_t task_begin;
    int64_t count;          // bw * bh * (box depth)
    int32_t vol;
    int32_t scale;          // mean-shift: the first scale of the group; quadrant: 0
    int32_t scale_hi;       // mean-shift: the last scale of the group; quadrant: 0
    int32_t bx, by, bz, bw, bh;
};

// Mean-shift task queues of one launch: one per XCD (workgroups are dispatched
// to the 8 XCDs round robin); queue k holds tasks begin[k] .. end[k] - 1.  A
// search split into several launches has one such block per launch; launch c
// counts the tasks taken from queue k in Counters::xq_head[c][k].
constexpr int kXcds = 8;
constexpr int kMaxMsChunks = 8;
struct XcdQueues {
    int64_t begin[kXcds];
    int64_t end[kXcds];
};

// Result of one trajectory (80 bytes).
struct TrajRec {
    int32_t x0, y0, z0, x, y, z;
    int32_t scale, iters, stop, keep;
    double objective;
    double y64;
    double key64;           // rank key: y64, or W at s* in decision precision
    float h32, w32, y32;
    int32_t seed;           // trajectory id within its volume
};

// Sort record of a kept trajectory: ordered by vol, ky (= ~bits(key64): rank key
// descending; keys are non-negative doubles), kpos (= s<<48 | z<<32 | y<<16 | x),
// then seed.
struct SortRec {
    uint64_t vol;
    uint64_t ky;
    uint64_t kpos;
    uint32_t seed;
    uint32_t idx;           // index of the TrajRec
};

struct Counters {
    unsigned long long evals, window_evals, voxel_visits, final_visits;
    unsigned long long queue_head[2];   // task queues (quadrant; ABMSOD candidates)
    unsigned long long xq_head[kMaxMsChunks][kXcds];  // mean-shift queues, per launch and XCD
    unsigned long long n_sort;          // kept trajectories
    unsigned long long swept;           // voxels actually swept by the searches
    unsigned long long lds_ops;         // lane-level LDS atomic operations of the searches
};

// Launch-time tuning of the mean-shift evaluation: replicas per wavefront,
// 1 << rl for windows of half-width > s_small and 1 << rl_small otherwise; a
// later evaluation of a trajectory updates its running window when the voxels
// that leave and enter it are fewer than incr_pct percent of the window (0:
// never); group: scales per task of the launch's task runs.
struct MsTune {
    int32_t rl, rl_small, s_small, incr_pct;
    int32_t group, pad;
};

// Seed id of task i of a run (its box's points in x-fastest order).
__device__ __forceinline__ long long seg_seed(const VolDesc& v, const TaskSeg& sg, long long i) {
    const long long row = i / sg.bw;
    const long long ix = i - row * sg.bw;
    const long long iz = row / sg.bh;
    const long long iy = row - iz * sg.bh;
    return (sg.bx + ix) + (long long)v.gx * ((sg.by + iy) + (long long)v.gy * (sg.bz + iz));
}

// Start position of seed `seed` of a volume: the listed position, or grid point
// (o + kx sp, o + ky sp, o + kz sp) with the seed index x fastest.
__device__ __forceinline__ void seed_pos(const VolDesc& v, long long seed, int* p) {
    if (v.seeds) {
        p[0] = v.seeds[3 * seed];
        p[1] = v.seeds[3 * seed + 1];
        p[2] = v.seeds[3 * seed + 2];
        return;
    }
    const long long gxy = (long long)v.gx * v.gy;
    const int gz = (int)(seed / gxy);
    const long long r = seed - (long long)gz * gxy;
    const int gy = (int)(r / v.gx);
    const int gx = (int)(r - (long long)gy * v.gx);
    p[0] = v.ox + gx * v.sp;
    p[1] = v.oy + gy * v.sp;
    p[2] = v.oz + gz * v.sp;
}

}  // namespace ks

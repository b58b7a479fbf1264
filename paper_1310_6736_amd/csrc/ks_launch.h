// Host launchers of the kernels in ks_kernels.hip.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "ks_device.h"

namespace ks {

// Same layout as the public ks_region.
struct ks_region_dev {
    int32_t x, y, z, scale;
    float saliency, entropy, pdf_change;
    int32_t seed;
};

// Byte offsets of the quadrant kernel's dynamic LDS.
struct LdsQuad {
    size_t hist_off, eps_off, hrow_off, arow_off, nrow_off, h32_off, res_off, bytes;
    int hist_words;
    int pad;
};

struct PrepArgs {
    VolDesc* vols;
    int nvol;
    Counters* cnt;
    int* vol_nfound;
    int* vol_base;
    long long max_voxels;   // largest X*Y*Z of the volumes
    long long max_words;    // largest (xp/4)*Y*Z
    int max_tx, max_ty;     // largest 64-voxel tile counts in x and y of a mean-shift volume
    int max_z;              // largest Z of a mean-shift volume (0: none)
};

struct SearchArgs {
    const VolDesc* vols;
    const TaskSeg* segs;
    int nseg;
    long long ntask;
    Tables tb;
    TrajRec* rec;
    Counters* cnt;
};

struct RankArgs {
    const VolDesc* vols;
    int nvol;
    const TrajRec* rec;
    SortRec* sr;                // 2 * n_pad records (merge ping-pong)
    Counters* cnt;
    unsigned long long n_pad;   // power of two >= total trajectories, >= 2
    long long max_traj;         // largest per-volume trajectory count
    int* bsum;                  // n_pad/1024 + 1 ints
    int* vol_base;
    int* vol_nfound;
    ks_region_dev* regions;
};

hipError_t launch_prep(const PrepArgs& a, hipStream_t st);
// xq: the launch's queues in device memory; chunk: the launch's index within the search.
hipError_t launch_search_ms(const SearchArgs& a, const XcdQueues* xq, int chunk, int grid, const MsTune& tune,
                            int hist_words, int maxB, hipStream_t st);
hipError_t launch_search_quad(const SearchArgs& a, int grid, int rq, const LdsQuad& lay, int maxB, hipStream_t st);
hipError_t launch_hook_ms(const VolDesc* vols, int kind, int n, const int* xyz, const int* sc, int rl, int hist_words,
                          int maxB, void* out, hipStream_t st);
// Dense Kadir-Brady map of vols[0]: K = S + 2 histogram rows of B bins per wave.
hipError_t launch_saliency_map(const VolDesc* vols, Tables tb, float* sal, uint8_t* scl, Counters* cnt, int K, int B,
                               int grid, hipStream_t st);
int max_blocks_map(int K, int B);
hipError_t launch_hook_quad(const VolDesc* vols, int kind, int lo, int hi, int n, const int* xyz, int rq,
                            const LdsQuad& lay, uint32_t* out, hipStream_t st);
hipError_t launch_rank(const RankArgs& a, hipStream_t st);
// Size of the static device array of the allocation-free entry point, and the
// address of `device`'s copy (looked up once per device, with it current).
constexpr size_t kScratchBytes = (size_t)96 << 20;
hipError_t scratch_address(int device, void** ptr);
// sq[c] = sqrt(c), rs[c] = 1/sqrt(c) (rs[0] = 0) for c < n, by the mean-shift search's device code.
hipError_t launch_count_roots(int n, double* sq, double* rs, hipStream_t st);
int max_blocks_ms(int hist_words, int maxB);
int max_blocks_quad(size_t lds_bytes, int maxB);

}  // namespace ks

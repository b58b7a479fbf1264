// Host-side context and planning structures of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/ks.h"
#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

// Grow-only device allocation: by at least 1.5x (4 KiB granules).
struct Buffer {
    void* ptr = nullptr;
    size_t cap = 0;
    ks_status ensure(size_t bytes, int* generation);
    void release();
};

inline size_t granule(size_t bytes) { return (bytes + 4095) & ~(size_t)4095; }

struct PinnedBuffer {
    void* ptr = nullptr;
    size_t cap = 0;
    ks_status ensure(size_t bytes);
    void release();
};

// One volume of a request as the runtime sees it.
struct VolIn {
    const void* raw;
    int32_t dtype;
    int32_t dims[3];
    int32_t bins, spacing;
    int32_t scales[2];
    int32_t method, max_iter;
    int32_t capacity;
    ks_options opt{};
    const int32_t* seeds = nullptr;  // host (x, y, z) start positions, or null: the seed grid
    int64_t n_seeds = 0;
};

// The per-call arena of a context: descriptors + task segments + seed lists,
// bin volumes, trajectory records, sort records, block sums, per-volume ints,
// results (in this order).
constexpr int kArenaBuffers = 7;
enum { kArVols = 0, kArBins, kArRec, kArSort, kArBsum, kArVolInt, kArOut };

// Bytes that plan() asks of each arena buffer for `in`.
void arena_needs(const std::vector<VolIn>& in, size_t need[kArenaBuffers]);

// Memory a plan places its arena and host copies in, instead of the context's
// grow-only buffers: one device range (each arena buffer at a 256-byte aligned
// offset) and two host ranges, all owned by the caller.
struct FixedArena {
    char* dev;
    size_t dev_bytes;
    char* stage;        // host staging of the upload
    size_t stage_bytes;
    char* out;          // host copy of the results
    size_t out_bytes;
};

struct Plan {
    char* dev[kArenaBuffers] = {};  // the arena buffers this plan uses
    char* stage = nullptr;          // host staging of the upload
    char* hout = nullptr;           // host copy of the results
    int nvol = 0;
    std::vector<VolDesc> vols;
    std::vector<TaskSeg> segs_q, segs_m;
    long long ntask_q = 0, ntask_m = 0;
    int64_t xq_begin[kXcds + 1] = {};  // the mean-shift tasks of XCD k's queue: xq_begin[k] .. xq_begin[k + 1] - 1
    int ms_chunks = 1;                 // launches the mean-shift search is split into
    long long total_traj = 0, total_regions = 0, max_traj = 0, max_voxels = 0, max_words = 0;
    int max_tx = 0, max_ty = 0, max_z = 0;  // mean-shift volumes: 64-voxel x, y tiles and Z
    unsigned long long n_pad = 2;
    int maxS_quad = 0, maxB_quad = 0, maxB_ms = 0;
    int rl = 4, rl_small = 3, rq = 0, ms_hist_words = 0;
    int ms_group = 1;       // mean-shift scales per task
    LdsQuad lay{};
    int* vol_nfound = nullptr;
    int* vol_base = nullptr;
    Counters* cnt = nullptr;        // the counter block, inside the result allocation
    size_t out_nf_off = 0, out_cnt_off = 0, out_bytes = 0;  // result layout (device and host copy)
    std::vector<size_t> seed_off;   // per volume: int offset of its seed list after the segments
    std::vector<const int32_t*> seed_src;  // per volume: the caller's host list, or null
    size_t seed_ints = 0;
};

struct GraphEntry {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
};

struct Context {
    static constexpr int kEvents = 8;   // phases 0..3, then mean-shift and quadrant search begin/end
    int device = 0;
    int num_cu = 256;
    bool profiling = false;
    int ms_rl_pref = 4;
    int ms_rl_small_pref = 2;
    int ms_s_small = 6;
    int ms_incr_pct = 100;  // running-window updates while cheaper than a fresh window
    bool overlap = true;    // quadrant and mean-shift searches of one call on two streams
    int ms_group = 0;       // mean-shift scales per task (one seed, consecutive scales); 0: by the task count
    ks_options opts{};      // selection and order for ks_detect_device / ks_seed_traces
    bool use_seeds = false; // explicit start positions for ks_detect_device / ks_seed_traces
    std::vector<int32_t> seeds;
    int quad_rq_pref = 0;
    int grid_pct = 100;     // persistent grid size, percent of the resident capacity
    int ms_chunks = 1;      // launches per mean-shift search (1..kMaxMsChunks)
    int generation = 0;
    Tables tables{};
    Buffer tables_buf, d_vols, d_abm, d_bins, d_rec, d_sr, d_bsum, d_volint, d_regions, d_hook,
        d_hook_out, d_raw;
    PinnedBuffer h_stage, h_out;
    hipStream_t aux = nullptr;
    hipStream_t batch_stream = nullptr;
    hipEvent_t ev[kEvents] = {};
    hipEvent_t fork_ev = nullptr, join_ev = nullptr, order_ev = nullptr;
    std::vector<GraphEntry> graphs;
    ks_run_stats last{};
    char* scratch = nullptr;   // this device's static array (allocation-free entry point), or null

    ks_status init(int32_t dev);
    void destroy();
    hipError_t ensure_aux();
    Buffer& arena(int i);
    // Device bytes the arena holds now, after a plan(in) (buffers only grow), and
    // for `in` alone (freshly allocated).
    size_t arena_held();
    size_t arena_after(const std::vector<VolIn>& in);
    static size_t arena_fresh(const std::vector<VolIn>& in);
    void arena_release();
    ks_status plan(const std::vector<VolIn>& in, Plan& p, const FixedArena* fixed = nullptr);
    ks_status upload(const Plan& p, hipStream_t st);
    ks_status enqueue_search(const Plan& p, hipStream_t st, bool with_rank, bool timed);
    ks_status download(const Plan& p, hipStream_t st);
    void collect_stats(const Plan& p, bool timed);
    ks_status begin_detect(const std::vector<VolIn>& in, hipStream_t st, Plan& p);
    void end_detect(const std::vector<VolIn>& in, const Plan& p, std::vector<std::vector<ks_region>>* out,
                    std::vector<int>* nfound);
    ks_status detect_volumes(const std::vector<VolIn>& in, hipStream_t st, std::vector<std::vector<ks_region>>* out,
                             std::vector<int>* nfound);
    ks_status detect_batch_graph(const std::vector<VolIn>& in, hipStream_t st,
                                 std::vector<std::vector<ks_region>>* out, std::vector<int>* nfound);
};

bool options_ok(const ks_options& o);  // thresholds not NaN, known rank key, window lo <= hi
bool options_fit(const ks_options& o, int32_t bins);  // a window level needs bins <= 255
ks_status check_request(const void* vol, int32_t dtype, const int32_t* dims, int32_t bins, int32_t spacing,
                        const int32_t* scales, int32_t method, int32_t max_iter);
// Start positions inside the volume, n >= 0, and at most 2^31 - 1 trajectories.
ks_status check_seeds(const int32_t* dims, const int32_t* scales, int32_t method, const int32_t* seeds, int64_t n);
int64_t num_trajectories(const int32_t* dims, int32_t spacing, const int32_t* scales, int32_t method);
int64_t num_trajectories(const VolIn& v);  // of the grid or of the seed list
size_t bins_bytes(const int32_t* dims);
int pick_ms_rl(int maxB, int pref);
int pick_quad_rq(int maxS, int maxB, int pref);
LdsQuad quad_layout(int maxS, int maxB, int rq);

}  // namespace ks

extern "C" ks_status ks_context_set_tuning(ks_context* ctx, int32_t ms_replicas_log2, int32_t quad_replicas_log2);
extern "C" ks_status ks_context_set_tuning_small(ks_context* ctx, int32_t ms_small_replicas_log2, int32_t s_small);

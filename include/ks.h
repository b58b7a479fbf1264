/*
 * ks.h -- C ABI of the MI355X (gfx950) library for seed-grid Kadir-Brady
 * salient-region search in 3D volumes.
 *
 * The method (Thota, Vaswani, Kale, Vydyanathan, "Fast 3D Salient Region
 * Detection in Medical Images using GPUs"): a sparse grid of seeds (Sec. 2.2,
 * Alg. 1, first step) moves toward local entropy maxima, either by the
 * quadrant method (Sec. 2.2, Alg. 1; 8 octants in 3D) or by saliency shift, a
 * mean-shift toward the uniform pmf (Sec. 2.3, Eq. 4-6); the converged centres
 * are scored by Kadir-Brady saliency, entropy times the change of the pdf with
 * scale (Sec. 1; Sec. 2.2 after Alg. 1; Sec. 2.3 after Eq. 6), and the best are
 * kept (Sec. 3.1 keeps the top 20).
 *
 * Conventions shared by every entry point:
 *  - Volumes are dense arrays of voxels with dims = {X, Y, Z}, x fastest:
 *    index = x + X*(y + Y*z).  dtype is one of ks_dtype.  Each dim is in
 *    [1, 65535] and ceil(X/16)*16*Y*Z < 2^31.
 *  - bins in [2, 256]: a voxel v falls in bin floor((v - vmin)*bins / (vmax - vmin + 1))
 *    over the volume's own [vmin, vmax] (the paper's beta(s), Eq. 4, left
 *    undefined there).
 *  - seed_spacing >= 1: seeds sit at o + k*seed_spacing on each axis with
 *    o = seed_spacing/2 (or (dim-1)/2 when that is outside the volume); seed ids
 *    run x fastest.  Quadrant: one trajectory per seed.  Mean-shift: one per
 *    (seed, scale) pair, trajectory id = seed_id*S + (s - s_min), S = s_max-s_min+1.
 *  - scales = {s_min, s_max}, 1 <= s_min <= s_max <= 32.  A scale s is a
 *    half-width: the mean-shift window is the cube P + [-s, s]^3; the quadrant
 *    octant window of scale k is {P + sigma*u : u in [0,k]^3}.
 *  - max_iter >= 0 bounds the accepted moves of each trajectory.
 *  - Histogram counts are exact integers.  Decisions (argmax over scale, moves,
 *    acceptance, entropy peaks, ranking) use IEEE double in a fixed order and give
 *    bit-identical results to the CPU reference; reported entropy, pdf change and
 *    saliency are float32.
 *  - Ownership: the caller owns every buffer it passes; the library owns
 *    contexts and servers, freed only by the matching *_destroy.
 *  - Errors: the return value is the status.  Outputs are written only on
 *    KS_OK.  *n_found is the total number of regions; only min(capacity, *n_found)
 *    are written (snprintf convention, not an error).  Argument checks happen
 *    before any GPU call and return KS_E_INVALID.
 *  - Threading: a context serves one host thread at a time.  The server API is
 *    thread-safe.
 *  - stream arguments are hipStream_t values passed as void* (NULL: the
 *    default stream).
 */
#ifndef KS_H
#define KS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KS_OK = 0,
    KS_E_INVALID = -1,    /* bad argument */
    KS_E_NOMEM = -2,      /* device or host allocation failed */
    KS_E_DEVICE = -3,     /* a HIP call failed; the context should be destroyed */
    KS_E_TOO_LARGE = -4,  /* request larger than the server's HBM budget */
    KS_E_NOT_READY = -5,  /* server result not available yet */
    KS_E_SHUTDOWN = -6    /* server is shutting down */
} ks_status;

typedef enum { KS_U8 = 0, KS_U16 = 1, KS_I16 = 2 } ks_dtype;
typedef enum { KS_QUADRANT = 0, KS_MEANSHIFT = 1 } ks_method;
typedef enum { KS_STOP_MAX_ITER = 0, KS_STOP_ZERO_MOVE = 1, KS_STOP_CLAMPED = 2, KS_STOP_REJECTED = 3 } ks_stop;

/* One detected region: centre, scale s* (half-width), float32 saliency Y = H*W,
 * entropy H and pdf change W at s*, and the id of the (lowest) trajectory that
 * converged there. */
typedef struct {
    int32_t x, y, z, scale;
    float saliency, entropy, pdf_change;
    int32_t seed;
} ks_region;

/* Final state of one trajectory. */
typedef struct {
    int32_t x0, y0, z0;    /* start */
    int32_t x, y, z;       /* converged position */
    int32_t scale;         /* s* (quadrant: 0 if the entropy has no peak over scale) */
    int32_t iters;         /* accepted moves */
    int32_t stop;          /* ks_stop */
    int32_t keep;          /* 1 if the trajectory yields a region */
    double objective;      /* E (quadrant) or sum_b sqrt(c_b)/sqrt(N) (mean-shift) at the end */
    double saliency64;     /* decision-precision saliency at s* */
    float saliency, entropy, pdf_change;
    int32_t pad;
} ks_seed_trace;

/* Work counters and device times of the last call on a context. */
typedef struct {
    int64_t trajectories;  /* trajectories searched */
    int64_t evals;         /* trajectory evaluations in the search */
    int64_t window_evals;  /* seed-scale windows evaluated, including the final saliency pass */
    int64_t voxel_visits;  /* in-volume voxels read by the search evaluations */
    int64_t final_visits;  /* in-volume voxels read by the final saliency pass */
    int64_t regions;       /* regions found (sum over volumes) */
    double ms_prep, ms_search, ms_rank, ms_total; /* device time per phase (only with profiling on) */
    int64_t swept_voxels;  /* voxels the searches actually swept: with running-window updates
                              of the mean-shift search, fewer than voxel_visits + final_visits */
    int64_t lds_ops;       /* lane-level LDS atomic additions of the searches (histogram
                              scatter, including the adds of padding bytes into spare slots) */
    double ms_search_quad, ms_search_ms; /* device time of each search launch (profiling on;
                              0 for a method the call does not run) */
} ks_run_stats;

/* Selection and order of the output regions.  A trajectory yields a region when
 * its decision-precision entropy H > h_min and saliency Y > y_min (the entropy
 * and saliency thresholds of Sec. 1 and Sec. 2.3, given no values there; default
 * 0 with strict >).  Regions are ranked by rank_by descending: KS_RANK_SALIENCY
 * (Y = H * W, default) or KS_RANK_PDF_CHANGE (W, the ranking of the PET
 * experiment, Sec. 3.1), ties by (scale, z, y, x) ascending.  All zero = the
 * defaults. */
enum { KS_RANK_SALIENCY = 0, KS_RANK_PDF_CHANGE = 1 };
typedef struct {
    double h_min, y_min;
    int32_t rank_by;
    /* Window level (Sec. 3.2: entropy over the intensity range of the structure
     * of interest).  window = 1: voxels with win_lo <= v <= win_hi are binned
     * over that range, ((v - win_lo) * bins) / (win_hi - win_lo + 1); voxels
     * outside take part in no histogram, and N is the count of those that do (a
     * window with none has H = 0, no move and W = 0).  Needs bins <= 255.
     * window = 0: the volume's own range (default). */
    int32_t window;
    int32_t win_lo, win_hi;
} ks_options;

typedef struct ks_context ks_context;
typedef struct ks_server ks_server;

/* Human-readable name of a status. */
const char* ks_status_str(ks_status s);

/* Create a context on a HIP device: builds the decision tables and the work
 * arena.  Destroy frees every device allocation of the context. */
ks_status ks_context_create(int32_t device, ks_context** out);
ks_status ks_context_destroy(ks_context* ctx);

/* Turn per-phase device timing (HIP events) on or off; off by default. */
ks_status ks_context_set_profiling(ks_context* ctx, int32_t on);

/* Tuning of the scatter kernels (defaults: 2^4 replicas per wave for mean-shift
 * windows of half-width > 6 and 2^2 up to 6, one octant histogram per quadrant
 * workgroup, measured on the PET-like and MR-like workloads;
 * ks_context_autotune picks them for a given workload).
 * ms_replicas_log2 in [2,6]: packed LDS histogram replicas per wavefront of the
 * mean-shift scatter, 2^value (also sets the small-window value);
 * quad_replicas_log2 in [0,3]: replicas per workgroup of the octant scatter.
 * Fewer replicas: more same-address LDS atomics, fewer slots to clear; more
 * replicas: more LDS per wavefront, lower occupancy.  Results do not depend on
 * the tuning.  Values that do not fit the LDS budget of a call are lowered. */
ks_status ks_context_set_tuning(ks_context* ctx, int32_t ms_replicas_log2, int32_t quad_replicas_log2);

/* Mean-shift windows of half-width <= s_small use 2^ms_small_replicas_log2
 * replicas (ms_small_replicas_log2 in [2,6], s_small >= 0). */
ks_status ks_context_set_tuning_small(ks_context* ctx, int32_t ms_small_replicas_log2, int32_t s_small);

/* Autotuning by window-size class: runs the search of one request (device
 * volume, ks_detect_device parameters) under a set of candidate tunings and
 * keeps, in the context, the fastest by device time of the search launch:
 * mean-shift, the replicas per wave of large windows (2^3..2^5), then the
 * replicas and the half-width bound of the small-window class (2^2..2^3 up to
 * s_small in {4, 6, 8}); quadrant, the replicas per workgroup (2^0..2^2, as the
 * LDS budget allows).  Each candidate is timed `reps` times (1..16) after one
 * warm-up and scored by its fastest run.  Results of later calls do not depend
 * on the tuning.  Leaves profiling as it was; out: NULL or the chosen
 * {ms_replicas_log2, ms_small_replicas_log2, s_small, quad_replicas_log2}. */
ks_status ks_context_autotune(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                              int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                              int32_t max_iter, int32_t reps, int32_t out[4], void* stream);

/* Options for the context's later ks_detect_device and ks_seed_traces calls
 * (ks_detect always uses the defaults; batch and server requests carry their
 * own); the window level also applies to the context's ks_saliency_map,
 * ks_bin_volume and ks_histograms calls.  NULL restores the defaults.
 * KS_E_INVALID for an unknown rank_by or window flag, win_lo > win_hi or a NaN
 * threshold (and, at the call, a window level with bins > 255). */
ks_status ks_context_set_options(ks_context* ctx, const ks_options* options);

/* Running-window updates of the mean-shift search (Sec. 2.3 evaluates Eq. 4-6 on
 * the window at every new position; consecutive windows of a trajectory
 * overlap).  A later evaluation of a trajectory takes the voxels that leave the
 * window out of its totals and adds those that enter, when the two regions
 * together hold fewer than incremental_pct percent of the window's voxels
 * (0..200; 0: every evaluation sweeps its whole window; default 100).  The final
 * pass reuses the counts of the window at P*.  Counts and offset sums are
 * integers, so results do not depend on the value. */
ks_status ks_context_set_ms_update(ks_context* ctx, int32_t incremental_pct);

/* Explicit start positions for the context's later ks_detect_device and
 * ks_seed_traces calls, in place of the seed grid (whose spacing is then only
 * validated): a warm start from earlier detections, as when tracking a region
 * from frame to frame with the converged regions of the previous frame (Sec. 4).
 * seeds: host array of 3 * n_seeds int32 (x, y, z), copied by the call; every
 * seed starts one quadrant trajectory, or one mean-shift trajectory per scale
 * (trajectory id = seed index * S + scale - scales[0]), and a region's `seed`
 * field is that id.  NULL restores the grid.  KS_E_INVALID for n_seeds < 0 or a
 * null list with n_seeds > 0; at the call, for a seed outside the volume or more
 * than 2^31 - 1 trajectories.  An empty list finds no region. */
ks_status ks_context_set_seeds(ks_context* ctx, const int32_t* seeds, int64_t n_seeds);

/* Mean-shift scales per task: a wavefront runs one seed's trajectories of
 * scales_per_task consecutive scales in ascending order, each starting from the
 * previous one's first window plus the shell between the two (1..8), or 0 (the
 * default): the largest group of up to 4 that still leaves 16 tasks per
 * resident wavefront.  Results do not depend on it. */
ks_status ks_context_set_ms_group(ks_context* ctx, int32_t scales_per_task);

/* Splits each mean-shift search into `launches` launches (1..8, default 1), each
 * taking an equal share of every queue's tasks, so that work of other streams
 * (other server slots, other callers) gets the device between them instead of
 * waiting for one long persistent launch to drain.  Results do not depend on
 * it. */
ks_status ks_context_set_ms_chunks(ks_context* ctx, int32_t launches);

/* Runs the quadrant and mean-shift searches of one call (a batch holding both
 * methods) concurrently on two streams, so that the blocks of each fill the
 * other's tail (on = 1, the default), or one after the other (0).  Results do
 * not depend on it. */
ks_status ks_context_set_overlap(ks_context* ctx, int32_t on);

/* Counters and times of the last detect/batch call on this context.  Times are
 * taken with profiling on: HIP events on the launch streams around the phases
 * and each search (in ks_detect_batch, event-record nodes of its captured
 * graph). */
ks_status ks_last_stats(ks_context* ctx, ks_run_stats* out);

/* Detection on a host volume (synchronous).  Uses a library-owned context on
 * device 0.  out: host array of capacity regions, ranked by saliency
 * descending, then scale, z, y, x ascending; duplicates of (x,y,z,scale) keep
 * the lowest trajectory id. */
ks_status ks_detect(const void* volume, ks_dtype dtype, const int32_t dims[3], int32_t bins, int32_t seed_spacing,
                    const int32_t scales[2], ks_method method, int32_t max_iter, ks_region* out, int32_t capacity,
                    int32_t* n_found);

/* Same, on a device-resident volume.  Work is queued on `stream`; the call
 * returns after the results are in `out` (host).  d_volume must stay valid
 * until then. */
ks_status ks_detect_device(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                           int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                           int32_t max_iter, ks_region* out, int32_t capacity, int32_t* n_found, void* stream);

/* ks_detect_device for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * detection, kernels and results, with the work memory (descriptors, bin
 * volumes, trajectory and sort records, results) in a static device array of
 * 96 MiB that the library holds on each GPU it runs on until the process ends.
 * The call allocates no device or pinned host memory (no hipMalloc,
 * hipHostMalloc or hipFree); it copies through pageable host memory.  The
 * caller passes the volume and the output as for ks_detect_device, and the
 * context (created beforehand) supplies the decision tables, options and seed
 * list.  KS_E_TOO_LARGE when the detection's work memory exceeds the array (it
 * holds, for example, the MR-like 256 x 256 x 160 mean-shift detection of
 * 430,080 trajectories with a capacity of a few thousand regions); otherwise
 * the errors of ks_detect_device.  Every call on one GPU uses that GPU's array,
 * whatever the context: calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller.  Returns when the results
 * are in `out`. */
ks_status ks_detect_device_noalloc(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                                   int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                                   int32_t max_iter, ks_region* out, int32_t capacity, int32_t* n_found,
                                   void* stream);

/* Per-trajectory final states of a search on a device volume (test and debug
 * hook).  out: host array of capacity traces in trajectory-id order; *n is the
 * number of trajectories. */
ks_status ks_seed_traces(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                         int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                         int32_t max_iter, ks_seed_trace* out, int32_t capacity, int32_t* n, void* stream);

/* Bin volume of a device volume (test hook): out is a host array of X*Y*Z bytes,
 * x fastest. */
ks_status ks_bin_volume(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                        int32_t bins, uint8_t* out, void* stream);

/* Window histograms on a device volume (test hook), through the same device
 * code as the search.  xyz: host, 3n positions; scale: host, n half-widths.
 *   KS_HIST_CUBE      counts of P + [-s,s]^3 clipped to the volume:      uint32 [n][B]
 *   KS_HIST_OCTANTS   counts of the 8 octant cubes of every scale k in
 *                     [range[0], range[1]] (Alg. 1 windows):             uint32 [n][8][K][B]
 *   KS_HIST_MEANSHIFT counts and per-bin sums of (v - P) over the cube
 *                     P + [-s,s]^3 (Eq. 4 with a flat kernel, Eq. 6):     int32  [n][4][B]
 *                     (rows: count, sum dx, sum dy, sum dz)
 *   KS_HIST_SHELLS    counts of the centred cubes of every half-width s in
 *                     [range[0], range[1]] (saliency pass):               uint32 [n][K][B]
 *   KS_HIST_MS_MOVE   as KS_HIST_MEANSHIFT at Q, reached by the running-window
 *                     update from the window at P; xyz holds 6n values, P then
 *                     Q per window (any two positions in the volume):     int32  [n][4][B]
 *   KS_HIST_MS_INNER  counts of P + [-s,s]^3, of P + [-(s-1),s-1]^3 through
 *                     the shell subtraction, and of the same inner cube swept
 *                     directly (mean-shift final pass):                  uint32 [n][3][B]
 * K = range[1] - range[0] + 1.  out is a host buffer of the stated size. */
enum {
    KS_HIST_CUBE = 0,
    KS_HIST_OCTANTS = 1,
    KS_HIST_MEANSHIFT = 2,
    KS_HIST_SHELLS = 3,
    KS_HIST_MS_MOVE = 4,
    KS_HIST_MS_INNER = 5
};
ks_status ks_histograms(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3], int32_t bins,
                        int32_t kind, const int32_t range[2], int32_t n, const int32_t* xyz, const int32_t* scale,
                        void* out, void* stream);

/* Test hook: the square roots of window counts that the mean-shift decisions
 * take on the device (Sec. 2.3: the bin weights of Eq. 5 and the coefficient
 * of Eq. 4 with the uniform target), computed by the search's own device code:
 * sq[c] = sqrt(c) and rsq[c] = 1/sqrt(c) (rsq[0] = 0) for every count c in
 * 0..n-1.  sq, rsq: host arrays of n doubles, owned by the caller.  KS_E_INVALID
 * for n < 1, n > 2^24 or a null pointer.  Returns when both are written. */
ks_status ks_count_roots(ks_context* ctx, int32_t n, double* sq, double* rsq, void* stream);


/* Dense Kadir-Brady saliency map (the every-voxel search that the seed grid
 * replaces, Sec. 1 and Sec. 2.1): at every voxel of the device volume, the
 * saliency step of the quadrant method with no search before it: centred cubes
 * of half-width scales[0]-1 .. scales[1]+1, entropy peaks over scale in
 * [scales[0], scales[1]], and the peak with the largest Y = H * W (first on
 * ties, decisions in double as in ks_detect).  d_scale (uint8) receives s* or 0
 * where there is no peak, d_saliency (float32) the saliency H * W at s* or 0;
 * both are device arrays of X*Y*Z elements, x fastest, owned by the caller.
 * Returns after the map is written.  Same validation as ks_detect with spacing
 * 1; KS_E_INVALID for a null output. */
ks_status ks_saliency_map(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3], int32_t bins,
                          const int32_t scales[2], float* d_saliency, uint8_t* d_scale, void* stream);

/* ------------------------------------------------------------------ ABMSOD */

/* One ABMSOD candidate (Sec. 2.3, Alg. 2): an ellipsoidal window of centre x and
 * bandwidth H, the voxels v with (v - x)^T H^-1 (v - x) <= 5 (the solid ellipsoid
 * whose uniform second moment is H). */
typedef struct {
    int32_t x0, y0, z0;    /* start position */
    int32_t radius;        /* start radius r: H = (r + 1/2)^2 / 5 I */
    double x[3];           /* centre of the best iteration */
    double h[6];           /* its bandwidth H: xx, yy, zz, xy, xz, yz */
    double rho;            /* best Bhattacharyya coefficient to the uniform pmf (0: none) */
    double entropy;        /* entropy (nats) of the Gaussian-weighted pmf behind it */
    int32_t iters;         /* iterations done */
    int32_t stop;          /* ks_abm_stop */
} ks_ellipsoid;

typedef enum {
    KS_ABM_MAX_ITER = 0,      /* max_iter iterations */
    KS_ABM_CONVERGED = 1,     /* centre moved < 0.01 voxel and H < 0.01 of its largest diagonal entry */
    KS_ABM_DETERIORATED = 2,  /* coefficient fell more than `threshold` below the best (Alg. 2) */
    KS_ABM_EMPTY = 3,         /* a window held no counted voxel */
    KS_ABM_DEGENERATE = 4     /* the new H was not positive definite */
} ks_abm_stop;

/* ABMSOD search with the uniform target pmf (Sec. 2.3: Eq. 4 with the Gaussian
 * profile exp(-d/2) of Alg. 2, the move of Eq. 5, the bandwidth of Eq. 7) from
 * every start position (the seed grid of seed_spacing, or the context's seed
 * list) and every start radius r in [radii[0], radii[1]]: candidate id =
 * seed * R + r - radii[0], R = radii[1] - radii[0] + 1.  One iteration moves the
 * centre to the Gaussian- and weight-weighted mean of its window (weights
 * sqrt(q_b / p_b) of the voxel's bin, q_b = 1/B), then, at the new centre with
 * the same H, measures the coefficient rho = sum_b sqrt(p_b q_b) and re-estimates
 * H as the weight-weighted second moment of the window about the new centre; a
 * new H whose half-extent sqrt(5 H_aa) exceeds radii[1] + 1/2 is scaled down to
 * it, and new centres are clamped to the volume.  The best coefficient so far
 * and its (centre, H) are kept (Alg. 2); see ks_abm_stop for the ends.  The
 * binning, including a window level, follows the context's options.  Sums of
 * the Gaussian profile are taken in 2^-40 fixed point (order-independent);
 * everything else is IEEE double.
 * out: host array of capacity candidates in id order; *n = number of candidates
 * (capacity 0: count only).  KS_E_INVALID as for ks_seed_traces, or for radii
 * outside 1..32, max_iter < 0, or a NaN threshold.  Returns when out is
 * written. */
ks_status ks_abmsod(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3], int32_t bins,
                    int32_t seed_spacing, const int32_t radii[2], int32_t max_iter, double threshold,
                    ks_ellipsoid* out, int32_t capacity, int32_t* n, void* stream);

/* One request of a batch or of the server. */
typedef struct {
    const void* volume;    /* device pointer (ks_detect_batch) or host pointer (ks_server_submit) */
    int32_t dtype;         /* ks_dtype */
    int32_t dims[3];
    int32_t bins;
    int32_t seed_spacing;
    int32_t scales[2];
    int32_t method;        /* ks_method */
    int32_t max_iter;
    ks_options options;
    /* Start positions in place of the seed grid (see ks_context_set_seeds): host
     * array of 3 * n_seeds int32 (x, y, z), read during the call (the server
     * copies it at submit); NULL: the grid of seed_spacing. */
    const int32_t* seeds;
    int64_t n_seeds;
    /* Server requests: the most regions a poll of this request will return, in
     * rank order (0: every region); the server keeps and copies only those.
     * ks_detect_batch takes the capacity of each ks_result instead. */
    int32_t max_regions;
    int32_t reserved;      /* 0 */
} ks_request;

typedef struct {
    ks_region* regions;    /* host array supplied by the caller */
    int32_t capacity;
    int32_t n_found;       /* written by the library */
    int32_t status;        /* ks_status of this request */
    int32_t pad;
} ks_result;

/* Batched detection of n device-resident volumes of any sizes and methods in
 * one captured launch sequence: per-volume range scan and binning, one
 * persistent search over every trajectory of every volume, one ranking pass.
 * Each volume's result equals ks_detect_device on it alone.  The work is queued
 * on `stream`; a NULL stream (which cannot be captured) means the context's own
 * stream, ordered after everything queued on the null stream before the call.
 * Returns when the results are in `results`. */
ks_status ks_detect_batch(ks_context* ctx, int32_t n, const ks_request* reqs, ks_result* results, void* stream);

/* Autotuning for a batch (the shapes the batch's captured launch sequence
 * uses): runs ks_detect_batch's launch sequence over the n requests under
 * candidate tunings and keeps, in the context, the fastest by device time of
 * the whole sequence (prep, searches, ranking), one parameter at a time:
 * mean-shift replicas per wave for large windows (2^3..2^5) and for small ones
 * (2^2..2^3), the small-window half-width bound (4, 6, 8), the scales per
 * mean-shift task (0 = by the task count, 1..4), then the quadrant replicas per
 * workgroup (2^0..2^2, as the LDS budget allows).  Each candidate is timed reps
 * times (1..16) after one warm-up and scored by its fastest run.  Results do
 * not depend on the tuning.  out: NULL or the chosen {ms_replicas_log2,
 * ms_small_replicas_log2, s_small, quad_replicas_log2, ms_scales_per_task}.
 * KS_E_INVALID for n < 1, a null request list or reps outside 1..16, and as
 * ks_detect_batch for the requests. */
ks_status ks_context_autotune_batch(ks_context* ctx, int32_t n, const ks_request* reqs, int32_t reps, int32_t out[5],
                                    void* stream);

/* ------------------------------------------------------------- measurement */

/* Roofline microbenchmarks behind the reported fractions (for callers measuring
 * the library, not part of a detection).  Runs one benchmark on `device`; *rate
 * is bytes/s (KS_ROOF_COPY: bytes read + written by a streaming copy of 1 GiB) or
 * lane-level LDS atomic additions per second (the others: every lane its own
 * address; SHARED4: four lanes per address, all equal).  KS_E_INVALID for an
 * unknown kind or a null rate. */
enum { KS_ROOF_COPY = 0, KS_ROOF_LDS_ADD64 = 1, KS_ROOF_LDS_ADD32 = 2, KS_ROOF_LDS_ADD64_SHARED4 = 3 };
ks_status ks_roofline(int32_t device, int32_t kind, double* rate);

/* ---------------------------------------------------------------- serving */

typedef struct {
    int64_t submitted, admitted, completed, refused, queued_now, in_flight;
    int64_t bytes_in_use, budget_bytes;  /* device bytes the slots hold for requests now; the budget */
    double p50_ms, p99_ms, mean_ms;      /* submit -> result ready, completed requests */
    double volumes_per_s;                /* completed / (last completion - first submit) */
    int64_t bytes_peak;                  /* largest bytes_in_use since the server started */
} ks_server_stats_t;

/* A server owns max_slots contexts on `device`, each with its own stream, and a
 * budget of device memory for requests (hbm_budget bytes): the device memory
 * its slots hold for them (volume copies, bin volumes, trajectory and sort
 * records, results) never exceeds it.  Pending requests are admitted oldest
 * first while the busy slots' memory plus the batch's own fits the budget,
 * grouped into batches of about ten milliseconds of estimated device work, one
 * batch per free slot; a slot's buffers grow to exactly what its batches need,
 * and idle slots give theirs back when a new batch would not fit beside them.
 * A batch that arrives while others run is launched at once on its own stream
 * and its work overlaps theirs on the device.  A large request (a full-size
 * mean-shift search of the MR-like kind) runs alone in its batch, one at a time,
 * while smaller requests pass it in the queue and run beside it.  Outside the budget, each slot holds the
 * fixed decision tables (7.2 MB) from creation to destruction. */
ks_status ks_server_create(int32_t device, size_t hbm_budget, int32_t max_slots, ks_server** out);
/* Copies the host volume; returns a ticket.  KS_E_TOO_LARGE if the request
 * alone would need more device memory than the budget. */
ks_status ks_server_submit(ks_server* s, const ks_request* req, uint64_t* ticket);
/* KS_E_NOT_READY until the request is done; then writes its regions once:
 * min(capacity, *n_found, the request's max_regions when set) of them in rank
 * order, *n_found being the total the request found. */
ks_status ks_server_poll(ks_server* s, uint64_t ticket, ks_region* out, int32_t capacity, int32_t* n_found);
/* A request of a tracked sequence (Sec. 4: tracking seeded from the converged
 * regions of the previous frame).  Frames of one track (any int64 id) are run in
 * submission order, each only after the one before it has completed; other
 * requests may pass a waiting frame.  A frame starts from the positions of the
 * first max_seeds regions, in rank order and with repeated positions taken once,
 * of the track's last completed frame; the track's first frame, and a frame
 * after one that found no region or failed, uses the request's own seeds or
 * grid.  max_seeds >= 1.  Results are polled like any other request. */
ks_status ks_server_submit_tracked(ks_server* s, const ks_request* req, int64_t track, int32_t max_seeds,
                                   uint64_t* ticket);
/* Blocks until every submitted request is done. */
ks_status ks_server_drain(ks_server* s);
ks_status ks_server_stats(ks_server* s, ks_server_stats_t* out);
/* Starts a new measurement window: clears the latency samples and the
 * submitted/admitted/completed/refused counts and the throughput clock; requests
 * already queued or in flight are still served and counted when they complete.
 * Lets a caller warm a server (device buffers grow to the workload's sizes on
 * first use) before measuring it. */
ks_status ks_server_reset_stats(ks_server* s);
ks_status ks_server_destroy(ks_server* s);

#ifdef __cplusplus
}
#endif
#endif /* KS_H */

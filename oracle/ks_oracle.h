/*
 * CPU oracle for seed-grid Kadir-Brady salient-region search in 3D.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded
 * restatement of the method (quadrant method: Sec. 2.2, Alg. 1; saliency shift:
 * Sec. 2.3, Eq. 4-6; Kadir-Brady saliency: Sec. 1 and Sec. 2.1) used to check
 * the GPU library.  Only the tests, the package's smoke check and the CPU
 * baseline leg of the benchmark may call it.  It shares no code with the GPU
 * library.
 *
 * Volumes: dims = {X, Y, Z}, x fastest, index = x + X*(y + Y*z).
 */
#ifndef KS_ORACLE_H
#define KS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { KSO_U8 = 0, KSO_U16 = 1, KSO_I16 = 2 };
enum { KSO_QUADRANT = 0, KSO_MEANSHIFT = 1 };
enum { KSO_STOP_MAX_ITER = 0, KSO_STOP_ZERO_MOVE = 1, KSO_STOP_CLAMPED = 2, KSO_STOP_REJECTED = 3 };
/* Rank key of the output: saliency Y = H * W (default), or the pdf change W. */
enum { KSO_RANK_SALIENCY = 0, KSO_RANK_PDF_CHANGE = 1 };

/* Outcome of one trajectory (a grid seed for the quadrant method, a
 * (grid seed, scale) pair for mean-shift). */
typedef struct {
    int64_t traj;          /* trajectory id */
    int32_t x0, y0, z0;    /* start position */
    int32_t x, y, z;       /* converged position P* */
    int32_t scale;         /* s* (quadrant: 0 when there is no entropy peak) */
    int32_t iters;         /* accepted moves */
    int32_t stop;          /* KSO_STOP_* */
    int32_t keep;          /* 1 if it yields a region */
    double objective;      /* final objective: E (quadrant) or rho (mean-shift) */
    double h64, w64, y64;  /* decision-precision entropy, pdf change, saliency at s* */
    double h_ref, y_ref;   /* accurate entropy and saliency at s* */
} kso_traj;

typedef struct {
    int32_t x, y, z, scale;
    double saliency, entropy, pdf_change, key;
    int64_t seed;
} kso_region;

typedef struct {
    int64_t evals;          /* trajectory evaluations (search windows) */
    int64_t window_evals;   /* seed-scale window evaluations incl. the final pass */
    int64_t voxel_visits;   /* in-volume voxels of the evaluated bricks/windows */
} kso_stats;

/* Step 1 of the search: intensity -> bin index (the paper's beta(s), Eq. 4). */
int kso_bin_volume(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, uint8_t* out);
/* Window-level binning (Sec. 3.2): voxels in [lo, hi] -> ((v - lo) * bins) /
 * (hi - lo + 1); voxels outside -> the value `bins`, which every histogram
 * ignores (it is not counted, and N is the count of the voxels that are). */
int kso_bin_volume_window(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, int32_t lo,
                          int32_t hi, uint8_t* out);

/* Entropies of one count vector: decision precision (H64) and accurate (Href). */
/* Alternative readings of points the paper leaves open, for tests that check
 * that the choice does not change the results (default 0, 0): sums over bins and
 * over the 8 octants in ascending order instead of the pairwise trees, and
 * H64 = ln N - S/N instead of (N ln N - S)/N.  Process-wide; not thread-safe. */
void kso_set_readings(int sequential_sums, int ln_n_form);

/* The two additions to Alg. 2 that the ABMSOD search makes (default 1, 1): the
 * stop when the centre and the bandwidth no longer move, and the cap on the
 * bandwidth at the largest start window.  For tests; process-wide. */
void kso_set_abm_readings(int convergence_stop, int bandwidth_cap);

double kso_entropy64(const uint32_t* counts, int32_t bins);
double kso_entropy_ref(const uint32_t* counts, int32_t bins);

/* Histograms of windows clipped to the volume, over a bin volume. */
int kso_hist_cube(const uint8_t* bv, const int32_t dims[3], int32_t bins, int32_t x, int32_t y, int32_t z,
                  int32_t s, uint32_t* counts);
int kso_hist_octant(const uint8_t* bv, const int32_t dims[3], int32_t bins, int32_t x, int32_t y, int32_t z,
                    int32_t j, int32_t k, uint32_t* counts);

/* One quadrant evaluation at P: eps[8*S] (j-major), kstar[8], E, delta[3]. */
int kso_eval_quadrant(const uint8_t* bv, const int32_t dims[3], int32_t bins, const int32_t p[3], int32_t s_min,
                      int32_t s_max, double* eps, int32_t* kstar, double* E, double* delta);
/* One mean-shift evaluation at (P, s): counts[B], msum[3B] (per bin sum of v-P),
 * delta[3], rho. */
int kso_eval_meanshift(const uint8_t* bv, const int32_t dims[3], int32_t bins, const int32_t p[3], int32_t s,
                       uint32_t* counts, int64_t* msum, double* delta, double* rho);

/* Number of trajectories of a search. */
int64_t kso_num_trajectories(const int32_t dims[3], int32_t spacing, const int32_t scales[2], int32_t method);

/* Run the trajectories listed in ids[0..n) (all when ids == NULL, n ignored).
 * window: NULL, or {lo, hi} for window-level binning. */
int kso_run(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
            int32_t spacing, const int32_t scales[2], int32_t method, int32_t max_iter, double h_min, double y_min,
            const int64_t* ids, int64_t n, kso_traj* out, kso_stats* stats);

/* As kso_run / kso_detect with the trajectories starting at n_seeds given
 * positions (x, y, z) instead of the seed grid (trajectory id = seed index, times
 * S plus the scale index for mean-shift): a tracking warm start from earlier
 * detections (Sec. 4). */
int kso_run_seeded(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                   const int32_t* seeds, int64_t n_seeds, const int32_t scales[2], int32_t method, int32_t max_iter,
                   double h_min, double y_min, kso_traj* out, kso_stats* stats);
int kso_detect_seeded(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                      const int32_t* seeds, int64_t n_seeds, const int32_t scales[2], int32_t method,
                      int32_t max_iter, double h_min, double y_min, int32_t rank_by, kso_region* out,
                      int32_t capacity, int32_t* n_found, kso_stats* stats);

/* ABMSOD (Sec. 2.3, Eq. 4, 5, 7, Alg. 2) with the uniform target pmf: a
 * candidate is a centre x (real) and a bandwidth H (symmetric positive definite
 * 3x3); its window is the voxels v with (v-x)^T H^-1 (v-x) <= 5, weighted by
 * the Gaussian profile g = exp(-d/2).  One iteration moves x to the g*w-weighted
 * mean of the window (Eq. 5, w = sqrt(q_b/p_b) of the voxel's bin), then, at the
 * new centre with the same H, measures the Bhattacharyya coefficient rho to the
 * uniform pmf and re-estimates H by Eq. 7 (w-weighted second moment about the
 * new centre).  The best rho so far and its (x, H) are kept; the search stops
 * when rho falls more than `threshold` below the best (Alg. 2), after max_iter
 * iterations, when x moves less than KSO_ABM_TOL voxel and H less than
 * KSO_ABM_TOL of its largest diagonal entry, when a window holds no counted
 * voxel, or when the new H is not positive definite.  A new H whose bounding
 * half-extent sqrt(5 H_aa) exceeds that of the largest start window (r + 1/2 for
 * the largest radius r) is scaled down to it.
 * Candidates: every start position (grid or seed list) x every radius r in
 * [radii[0], radii[1]] (id = seed * R + r - radii[0]), starting from
 * H = (r + 1/2)^2/5 I, the ball of radius r + 1/2 (whose boundary passes through
 * no lattice point, so that rounding cannot move a voxel in or out). */
enum { KSO_ABM_MAX_ITER = 0, KSO_ABM_CONVERGED = 1, KSO_ABM_DETERIORATED = 2, KSO_ABM_EMPTY = 3,
       KSO_ABM_DEGENERATE = 4 };
#define KSO_ABM_TOL 0.01
typedef struct {
    int64_t id;
    int32_t x0, y0, z0, radius;  /* start position and radius */
    double x[3];                 /* best centre */
    double h[6];                 /* its bandwidth: xx, yy, zz, xy, xz, yz */
    double rho;                  /* best Bhattacharyya coefficient (0: none) */
    double entropy;              /* entropy (nats) of the weighted pmf behind it */
    int32_t iters, stop;         /* iterations done, KSO_ABM_* */
} kso_ellipsoid;
/* seeds: NULL for the grid of `spacing`, else n_seeds positions (x, y, z);
 * ids: NULL for every candidate, else the n candidate ids to run.  Stats:
 * evals = window histograms (two per iteration), voxel_visits = window voxels
 * of all four passes of every iteration.  -1 for a seed outside the volume or
 * bad radii. */
int kso_abmsod(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
               int32_t spacing, const int32_t* seeds, int64_t n_seeds, const int32_t radii[2], int32_t max_iter,
               double threshold, const int64_t* ids, int64_t n, kso_ellipsoid* out, kso_stats* stats);

/* Dense Kadir-Brady map: at every voxel, s* of the saliency step of the quadrant
 * method (0: no entropy peak) and the saliency at s* (sal: accurate Y_ref;
 * sal64, if not NULL: decision-precision Y).  x fastest. */
int kso_saliency_map(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                     const int32_t scales[2], float* sal, uint8_t* scale, double* sal64);

/* Full detection: run every trajectory, keep those with H > h_min and Y > y_min,
 * dedup on (x, y, z, scale) and rank by rank_by (KSO_RANK_*) descending, ties by
 * scale, z, y, x ascending.  Writes min(capacity, n) regions; *n_found is the
 * total. */
int kso_detect(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
               int32_t spacing, const int32_t scales[2], int32_t method, int32_t max_iter, double h_min, double y_min,
               int32_t rank_by, kso_region* out, int32_t capacity, int32_t* n_found, kso_stats* stats);

/* Step 8 alone, on the records of kso_run (any subset order; shards of one run
 * concatenated give the same result as kso_detect on the whole run). */
int kso_rank(const kso_traj* t, int64_t n, int32_t rank_by, kso_region* out, int32_t capacity, int32_t* n_found);

#ifdef __cplusplus
}
#endif
#endif

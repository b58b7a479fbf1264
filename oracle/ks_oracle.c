/*
 * CPU oracle for seed-grid Kadir-Brady salient-region search in 3D.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow, single-threaded restatement of the
 * method, used to check the GPU library.  Every window histogram is built
 * directly with nested loops over the clipped window; no shells, prefix sums or
 * incremental updates.  Decision arithmetic is IEEE double in the fixed order
 * stated below, compiled without contraction (-ffp-contract=off).
 *
 * Readings of the paper that this file implements (the paper leaves them open):
 *  - bins: beta(v) = floor((v - vmin) * B / (vmax - vmin + 1)) over the volume's
 *    own range (Eq. 4 uses beta without defining it);
 *  - entropy uses the natural log (Eq. 1-2);
 *  - windows are clipped to the volume and N is the in-volume voxel count;
 *  - quadrant method in 3D uses the 8 octant cubes {P + sigma_j*u : u in [0,k]^3}
 *    (Sec. 2.2, Alg. 1), displacement d_j = k*_j * sigma_j (the 3D analogue of
 *    sqrt(2)*k_opt along the quadrant diagonal);
 *  - the mean-shift kernel is flat over the cube P + [-s,s]^3, so p_b = c_b/N and
 *    -K' is constant and cancels in Eq. 6;
 *  - moves are rounded half away from zero to whole voxels and accepted only if
 *    the objective strictly increases (best-so-far idea of Alg. 2), otherwise the
 *    search stops at the last accepted position;
 *  - saliency (Sec. 1, Sec. 2.1): entropy peaks over scale, pdf change
 *    W(s) = s^2/(2s-1) * sum_b |p_s(b) - p_{s-1}(b)|, Y = H * W;
 *  - window level (Sec. 3.2): voxels in [lo, hi] are binned over that range,
 *    the others take part in no histogram and N counts the voxels inside;
 *  - tracking (Sec. 4): a run may start from a list of positions instead of
 *    the grid (every scale per position for mean-shift);
 *  - ABMSOD (Sec. 2.3, Eq. 5, 7, Alg. 2): the ellipsoid (v-x)^T H^-1 (v-x) <= 5
 *    (uniform second moment H), Gaussian profile exp(-d/2), start H = (r+1/2)^2/5 I,
 *    Eq. 7 weighted by w alone about the new centre, best coefficient kept; see
 *    kso_abmsod in the header for the stops.
 *
 * Fixed summation order shared by definition (not by code) with the GPU path:
 * every sum over bins is a pairwise halving tree over Bp terms, where Bp is the
 * smallest power of two >= max(B, 64), absent bins contributing 0; the sum over
 * the 8 octants is the halving tree ((e0+e1)+(e2+e3))+((e4+e5)+(e6+e7)).
 */
#include "ks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

static int64_t vidx(const int32_t dims[3], int32_t x, int32_t y, int32_t z) {
    return (int64_t)x + (int64_t)dims[0] * ((int64_t)y + (int64_t)dims[1] * (int64_t)z);
}

static int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int32_t read_voxel(const void* vol, int32_t dtype, int64_t i) {
    if (dtype == KSO_U8) return ((const uint8_t*)vol)[i];
    if (dtype == KSO_U16) return ((const uint16_t*)vol)[i];
    return ((const int16_t*)vol)[i];
}

static int32_t padded_terms(int32_t bins) {
    int32_t n = 64;
    while (n < bins) n *= 2;
    return n;
}

/* Pairwise halving sum of v[lo .. lo+len), entries at index >= n count as 0. */
static double pairwise(const double* v, int32_t n, int32_t lo, int32_t len) {
    if (len == 1) return lo < n ? v[lo] : 0.0;
    return pairwise(v, n, lo, len / 2) + pairwise(v, n, lo + len / 2, len / 2);
}

/* Alternative readings, for tests that check that the choice does not change
 * the results: sums over bins (and over the 8 octants) in ascending order, and
 * H64 = ln N - S/N. */
static int g_sequential_sums = 0, g_ln_n_form = 0;

void kso_set_readings(int sequential_sums, int ln_n_form) {
    g_sequential_sums = sequential_sums != 0;
    g_ln_n_form = ln_n_form != 0;
}

/* The two additions to Alg. 2 (readings R32, R33), on by default. */
static int g_abm_convergence_stop = 1, g_abm_bandwidth_cap = 1;

void kso_set_abm_readings(int convergence_stop, int bandwidth_cap) {
    g_abm_convergence_stop = convergence_stop != 0;
    g_abm_bandwidth_cap = bandwidth_cap != 0;
}

static double sum_octants(const double* e) {
    if (g_sequential_sums) return ((((((e[0] + e[1]) + e[2]) + e[3]) + e[4]) + e[5]) + e[6]) + e[7];
    return ((e[0] + e[1]) + (e[2] + e[3])) + ((e[4] + e[5]) + (e[6] + e[7]));
}

static double sum_bins(const double* v, int32_t bins) {
    if (g_sequential_sums) {
        double s = 0.0;
        for (int32_t b = 0; b < bins; ++b) s += v[b];
        return s;
    }
    return pairwise(v, bins, 0, padded_terms(bins));
}


/* ---------------------------------------------------------------- binning */

/* Window-level binning (Sec. 3.2: entropy over the intensity range of the
 * structure of interest): voxels in [lo, hi] get ((v - lo) * bins) / (hi - lo + 1),
 * voxels outside get the value `bins`, which every histogram below ignores. */
int kso_bin_volume_window(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, int32_t lo,
                          int32_t hi, uint8_t* out) {
    int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
    int64_t width = (int64_t)hi - lo + 1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = read_voxel(vol, dtype, i);
        out[i] = (v < lo || v > hi) ? (uint8_t)bins : (uint8_t)(((v - lo) * bins) / width);
    }
    return 0;
}

static void bin_any(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                    uint8_t* out) {
    if (window) kso_bin_volume_window(vol, dtype, dims, bins, window[0], window[1], out);
    else kso_bin_volume(vol, dtype, dims, bins, out);
}

int kso_bin_volume(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, uint8_t* out) {
    int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
    int32_t vmin = read_voxel(vol, dtype, 0), vmax = vmin;
    for (int64_t i = 1; i < n; ++i) {
        int32_t v = read_voxel(vol, dtype, i);
        if (v < vmin) vmin = v;
        if (v > vmax) vmax = v;
    }
    int64_t width = (int64_t)vmax - vmin + 1;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = read_voxel(vol, dtype, i);
        out[i] = (uint8_t)(((v - vmin) * bins) / width);
    }
    return 0;
}

/* ---------------------------------------------------------------- entropy */

/* H64 = (N ln N - sum_b c_b ln c_b) / N, the decision-precision Shannon entropy
 * of p_b = c_b / N (Eq. 1 with the natural log); a window whose voxels all fall in
 * one bin gives exactly 0. */
static double entropy64_n(const uint32_t* c, int32_t bins, int64_t N) {
    if (N == 0) return 0.0;
    double* t = (double*)malloc(sizeof(double) * (size_t)bins);
    for (int32_t b = 0; b < bins; ++b) t[b] = c[b] > 0 ? (double)c[b] * log((double)c[b]) : 0.0;
    double S = sum_bins(t, bins);
    free(t);
    if (g_ln_n_form) return log((double)N) - S / (double)N;
    return ((double)N * log((double)N) - S) / (double)N;
}

/* Accurate entropy -sum p ln p; for p > 1/2, ln p = log1p(-(N-c)/N). */
static double entropy_ref_n(const uint32_t* c, int32_t bins, int64_t N) {
    if (N == 0) return 0.0;
    double h = 0.0;
    for (int32_t b = 0; b < bins; ++b) {
        if (c[b] == 0) continue;
        double p = (double)c[b] / (double)N;
        double lp = (2 * (int64_t)c[b] > N) ? log1p(-(double)(N - (int64_t)c[b]) / (double)N) : log(p);
        h -= p * lp;
    }
    return h;
}

static int64_t total(const uint32_t* c, int32_t bins) {
    int64_t n = 0;
    for (int32_t b = 0; b < bins; ++b) n += c[b];
    return n;
}

double kso_entropy64(const uint32_t* counts, int32_t bins) { return entropy64_n(counts, bins, total(counts, bins)); }
double kso_entropy_ref(const uint32_t* counts, int32_t bins) { return entropy_ref_n(counts, bins, total(counts, bins)); }

/* ---------------------------------------------------------------- windows */

/* Counts of bins in the box [x0,x1]x[y0,y1]x[z0,z1] clipped to the volume; voxels
 * outside a window level (value >= bins) are not counted.  Returns the count. */
static int64_t box_hist(const uint8_t* bv, const int32_t dims[3], int32_t bins, int32_t x0, int32_t x1, int32_t y0,
                        int32_t y1, int32_t z0, int32_t z1, uint32_t* c) {
    memset(c, 0, sizeof(uint32_t) * (size_t)bins);
    x0 = x0 < 0 ? 0 : x0; y0 = y0 < 0 ? 0 : y0; z0 = z0 < 0 ? 0 : z0;
    x1 = x1 >= dims[0] ? dims[0] - 1 : x1;
    y1 = y1 >= dims[1] ? dims[1] - 1 : y1;
    z1 = z1 >= dims[2] ? dims[2] - 1 : z1;
    int64_t n = 0;
    for (int32_t z = z0; z <= z1; ++z)
        for (int32_t y = y0; y <= y1; ++y)
            for (int32_t x = x0; x <= x1; ++x) {
                int32_t b = bv[vidx(dims, x, y, z)];
                if (b >= bins) continue;
                c[b] += 1;
                n += 1;
            }
    return n;
}

static int64_t box_volume(const int32_t dims[3], int32_t x0, int32_t x1, int32_t y0, int32_t y1, int32_t z0,
                          int32_t z1) {
    x0 = x0 < 0 ? 0 : x0; y0 = y0 < 0 ? 0 : y0; z0 = z0 < 0 ? 0 : z0;
    x1 = x1 >= dims[0] ? dims[0] - 1 : x1;
    y1 = y1 >= dims[1] ? dims[1] - 1 : y1;
    z1 = z1 >= dims[2] ? dims[2] - 1 : z1;
    if (x1 < x0 || y1 < y0 || z1 < z0) return 0;
    return (int64_t)(x1 - x0 + 1) * (y1 - y0 + 1) * (z1 - z0 + 1);
}

/* Octant j: bit 0 -> x, bit 1 -> y, bit 2 -> z; a set bit means the + direction. */
static int32_t octant_sign(int32_t j, int32_t axis) { return ((j >> axis) & 1) ? 1 : -1; }

static int64_t octant_hist(const uint8_t* bv, const int32_t dims[3], int32_t bins, const int32_t p[3], int32_t j,
                           int32_t k, uint32_t* c) {
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (octant_sign(j, a) > 0) { lo[a] = p[a]; hi[a] = p[a] + k; }
        else { lo[a] = p[a] - k; hi[a] = p[a]; }
    }
    return box_hist(bv, dims, bins, lo[0], hi[0], lo[1], hi[1], lo[2], hi[2], c);
}

static int64_t cube_hist(const uint8_t* bv, const int32_t dims[3], int32_t bins, const int32_t p[3], int32_t s,
                         uint32_t* c) {
    return box_hist(bv, dims, bins, p[0] - s, p[0] + s, p[1] - s, p[1] + s, p[2] - s, p[2] + s, c);
}

int kso_hist_cube(const uint8_t* bv, const int32_t dims[3], int32_t bins, int32_t x, int32_t y, int32_t z, int32_t s,
                  uint32_t* counts) {
    int32_t p[3] = {x, y, z};
    cube_hist(bv, dims, bins, p, s, counts);
    return 0;
}

int kso_hist_octant(const uint8_t* bv, const int32_t dims[3], int32_t bins, int32_t x, int32_t y, int32_t z,
                    int32_t j, int32_t k, uint32_t* counts) {
    int32_t p[3] = {x, y, z};
    octant_hist(bv, dims, bins, p, j, k, counts);
    return 0;
}

/* ------------------------------------------------------- quadrant method */

/* Alg. 1 body: per octant j and scale k the entropy eps_jk of W_jk(P); per octant
 * the first maximising scale k*_j; normalised entropies eps_j / E; and the
 * effective displacement delta = sum_j (eps_j / E) * k*_j * sigma_j, evaluated
 * as (sum_j eps_j * k*_j * sigma_j) / E. */
int kso_eval_quadrant(const uint8_t* bv, const int32_t dims[3], int32_t bins, const int32_t p[3], int32_t s_min,
                      int32_t s_max, double* eps, int32_t* kstar, double* E, double* delta) {
    int32_t S = s_max - s_min + 1;
    uint32_t* c = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)bins);
    double best[8];
    for (int32_t j = 0; j < 8; ++j) {
        kstar[j] = s_min;
        best[j] = 0.0;
        for (int32_t k = s_min; k <= s_max; ++k) {
            int64_t N = octant_hist(bv, dims, bins, p, j, k, c);
            double e = entropy64_n(c, bins, N);
            eps[j * S + (k - s_min)] = e;
            if (k == s_min || e > best[j]) { best[j] = e; kstar[j] = k; }
        }
    }
    free(c);
    *E = sum_octants(best);
    for (int a = 0; a < 3; ++a) {
        if (*E == 0.0) { delta[a] = 0.0; continue; }
        double t[8];
        for (int32_t j = 0; j < 8; ++j) t[j] = best[j] * (double)(kstar[j] * octant_sign(j, a));
        delta[a] = sum_octants(t) / *E;
    }
    return 0;
}

/* -------------------------------------------------------- saliency shift */

/* Eq. 4-6 with a flat kernel over C_s(P) and the uniform target q_b = 1/B:
 * w(v) = sqrt(q_b / p_b) = sqrt(N / (B c_b)) for v in bin b, so
 * x_new - P = sum_v w(v)(v-P) / sum_v w(v) = (sum_b M_b / sqrt(c_b)) / (sum_b sqrt(c_b)),
 * with M_b = sum over the window voxels in bin b of (v - P).  The Bhattacharyya
 * coefficient rho = sum_b sqrt(p_b q_b) is used without its constant factor
 * 1/sqrt(B): rho~ = (sum_b sqrt(c_b)) / sqrt(N). */
int kso_eval_meanshift(const uint8_t* bv, const int32_t dims[3], int32_t bins, const int32_t p[3], int32_t s,
                       uint32_t* counts, int64_t* msum, double* delta, double* rho) {
    memset(counts, 0, sizeof(uint32_t) * (size_t)bins);
    memset(msum, 0, sizeof(int64_t) * 3 * (size_t)bins);
    int64_t N = 0;
    for (int32_t z = p[2] - s; z <= p[2] + s; ++z)
        for (int32_t y = p[1] - s; y <= p[1] + s; ++y)
            for (int32_t x = p[0] - s; x <= p[0] + s; ++x) {
                if (x < 0 || y < 0 || z < 0 || x >= dims[0] || y >= dims[1] || z >= dims[2]) continue;
                int32_t b = bv[vidx(dims, x, y, z)];
                if (b >= bins) continue;
                counts[b] += 1;
                msum[3 * b + 0] += x - p[0];
                msum[3 * b + 1] += y - p[1];
                msum[3 * b + 2] += z - p[2];
                N += 1;
            }
    double* t = (double*)malloc(sizeof(double) * (size_t)bins);
    for (int32_t b = 0; b < bins; ++b) t[b] = counts[b] > 0 ? sqrt((double)counts[b]) : 0.0;
    double D = sum_bins(t, bins);
    for (int a = 0; a < 3; ++a) {
        for (int32_t b = 0; b < bins; ++b)
            t[b] = counts[b] > 0 ? (double)msum[3 * b + a] * (1.0 / sqrt((double)counts[b])) : 0.0;
        double num = sum_bins(t, bins);
        delta[a] = D > 0.0 ? num / D : 0.0;
    }
    free(t);
    *rho = N > 0 ? D / sqrt((double)N) : 0.0;
    return 0;
}

/* ------------------------------------------------------------- saliency */

/* pdf change between scales s-1 and s: s^2/(2s-1) * sum_b |c_s/N_s - c_{s-1}/N_{s-1}|,
 * the numerator taken exactly as sum_b |c_s N_{s-1} - c_{s-1} N_s|. */
static double pdf_change(const uint32_t* cs, int64_t Ns, const uint32_t* cp, int64_t Np, int32_t bins, int32_t s) {
    if (Ns == 0 || Np == 0) return 0.0;  /* only with a window level: no counted voxel */
    int64_t A = 0;
    for (int32_t b = 0; b < bins; ++b) {
        int64_t d = (int64_t)cs[b] * Np - (int64_t)cp[b] * Ns;
        A += d < 0 ? -d : d;
    }
    return ((double)(s * s) / (double)(2 * s - 1)) * ((double)A / ((double)Ns * (double)Np));
}

/* Saliency at the converged position (Sec. 2.2 after Alg. 1; Sec. 2.3 before the
 * ABMSOD paragraph): quadrant -> entropy peaks over s in [s_min, s_max] of the
 * centred cube C_s(P*), best peak by H*W; mean-shift -> the trajectory's own scale. */
static void saliency(const uint8_t* bv, const int32_t dims[3], int32_t bins, const int32_t p[3], int32_t method,
                     int32_t s_min, int32_t s_max, int32_t own_s, double h_min, double y_min, kso_traj* t,
                     kso_stats* st) {
    int32_t lo = method == KSO_QUADRANT ? s_min - 1 : own_s - 1;
    int32_t hi = method == KSO_QUADRANT ? s_max + 1 : own_s;
    int32_t n = hi - lo + 1;
    uint32_t* c = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)bins * (size_t)n);
    int64_t* N = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    double* H = (double*)malloc(sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        N[i] = cube_hist(bv, dims, bins, p, lo + i, c + (size_t)i * bins);
        H[i] = entropy64_n(c + (size_t)i * bins, bins, N[i]);
    }
    st->window_evals += n;
    st->voxel_visits += box_volume(dims, p[0] - hi, p[0] + hi, p[1] - hi, p[1] + hi, p[2] - hi, p[2] + hi);
    int32_t best = -1;
    double bestY = 0.0;
    if (method == KSO_QUADRANT) {
        for (int32_t s = s_min; s <= s_max; ++s) {
            int32_t i = s - lo;
            if (!(H[i] > H[i - 1] && H[i] > H[i + 1])) continue;
            double W = pdf_change(c + (size_t)i * bins, N[i], c + (size_t)(i - 1) * bins, N[i - 1], bins, s);
            double Y = H[i] * W;
            if (best < 0 || Y > bestY) { best = s; bestY = Y; }
        }
    } else {
        best = own_s;
    }
    t->scale = best < 0 ? 0 : best;
    t->keep = 0;
    t->h64 = t->w64 = t->y64 = t->h_ref = t->y_ref = 0.0;
    if (best >= 0) {
        int32_t i = best - lo;
        double W = pdf_change(c + (size_t)i * bins, N[i], c + (size_t)(i - 1) * bins, N[i - 1], bins, best);
        t->h64 = H[i];
        t->w64 = W;
        t->y64 = H[i] * W;
        t->h_ref = entropy_ref_n(c + (size_t)i * bins, bins, N[i]);
        t->y_ref = t->h_ref * W;
        t->keep = (t->h64 > h_min && t->y64 > y_min) ? 1 : 0;
    }
    free(c); free(N); free(H);
}

/* ------------------------------------------------------------ trajectories */

static void grid_dims(const int32_t dims[3], int32_t sp, int32_t g[3], int32_t o[3]) {
    for (int a = 0; a < 3; ++a) {
        o[a] = sp / 2;
        if (o[a] >= dims[a]) o[a] = (dims[a] - 1) / 2;
        g[a] = (dims[a] - 1 - o[a]) / sp + 1;
    }
}

int64_t kso_num_trajectories(const int32_t dims[3], int32_t spacing, const int32_t scales[2], int32_t method) {
    int32_t g[3], o[3];
    grid_dims(dims, spacing, g, o);
    int64_t n = (int64_t)g[0] * g[1] * g[2];
    return method == KSO_MEANSHIFT ? n * (scales[1] - scales[0] + 1) : n;
}

typedef struct {
    const uint8_t* bv;
    const int32_t* dims;
    int32_t bins, method, s_min, s_max;
    double* eps;
    uint32_t* counts;
    int64_t* msum;
} eval_ctx;

/* One evaluation: objective and proposed displacement at P. */
static void evaluate(eval_ctx* e, const int32_t p[3], int32_t s, double* obj, double delta[3], kso_stats* st) {
    st->evals += 1;
    if (e->method == KSO_QUADRANT) {
        int32_t kstar[8];
        kso_eval_quadrant(e->bv, e->dims, e->bins, p, e->s_min, e->s_max, e->eps, kstar, obj, delta);
        st->window_evals += 8 * (e->s_max - e->s_min + 1);
        int32_t r = e->s_max;
        st->voxel_visits += box_volume(e->dims, p[0] - r, p[0] + r, p[1] - r, p[1] + r, p[2] - r, p[2] + r);
    } else {
        kso_eval_meanshift(e->bv, e->dims, e->bins, p, s, e->counts, e->msum, delta, obj);
        st->window_evals += 1;
        st->voxel_visits += box_volume(e->dims, p[0] - s, p[0] + s, p[1] - s, p[1] + s, p[2] - s, p[2] + s);
    }
}

/* The search loop shared by both methods (Alg. 1 loop; Alg. 2 acceptance):
 * round the proposed move, stop if it is zero, if clamping leaves P unchanged,
 * if the objective does not strictly increase, or after max_iter accepted moves. */
static void run_trajectory(eval_ctx* e, int32_t max_iter, const int32_t p0[3], int32_t s, kso_traj* t, kso_stats* st) {
    int32_t p[3] = {p0[0], p0[1], p0[2]};
    double obj, delta[3];
    evaluate(e, p, s, &obj, delta, st);
    int32_t it = 0, stop;
    for (;;) {
        if (it == max_iter) { stop = KSO_STOP_MAX_ITER; break; }
        int32_t m[3];
        for (int a = 0; a < 3; ++a) m[a] = (int32_t)round(delta[a]);
        if (m[0] == 0 && m[1] == 0 && m[2] == 0) { stop = KSO_STOP_ZERO_MOVE; break; }
        int32_t q[3];
        for (int a = 0; a < 3; ++a) q[a] = clampi(p[a] + m[a], 0, e->dims[a] - 1);
        if (q[0] == p[0] && q[1] == p[1] && q[2] == p[2]) { stop = KSO_STOP_CLAMPED; break; }
        double obj2, delta2[3];
        evaluate(e, q, s, &obj2, delta2, st);
        if (!(obj2 > obj)) { stop = KSO_STOP_REJECTED; break; }
        for (int a = 0; a < 3; ++a) { p[a] = q[a]; delta[a] = delta2[a]; }
        obj = obj2;
        it += 1;
    }
    t->x0 = p0[0]; t->y0 = p0[1]; t->z0 = p0[2];
    t->x = p[0]; t->y = p[1]; t->z = p[2];
    t->iters = it;
    t->stop = stop;
    t->objective = obj;
}

/* Trajectories start at the seed grid, or (seeds != NULL) at the n_seeds listed
 * positions (x, y, z): a tracking warm start from earlier detections (Sec. 4). */
static int seeds_ok(const int32_t dims[3], const int32_t* seeds, int64_t n_seeds) {
    if (n_seeds < 0) return 0;
    for (int64_t i = 0; seeds && i < n_seeds; ++i)
        for (int a = 0; a < 3; ++a)
            if (seeds[3 * i + a] < 0 || seeds[3 * i + a] >= dims[a]) return 0;
    return 1;
}

static int run_impl(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                    int32_t spacing, const int32_t* seeds, int64_t n_seeds, const int32_t scales[2], int32_t method,
                    int32_t max_iter, double h_min, double y_min, const int64_t* ids, int64_t n, kso_traj* out,
                    kso_stats* stats) {
    if (!seeds_ok(dims, seeds, n_seeds)) return -1;
    int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
    uint8_t* bv = (uint8_t*)malloc((size_t)nv);
    bin_any(vol, dtype, dims, bins, window, bv);
    int32_t g[3], o[3];
    grid_dims(dims, spacing, g, o);
    int32_t S = scales[1] - scales[0] + 1;
    int64_t ntraj = seeds ? n_seeds * (method == KSO_MEANSHIFT ? S : 1)
                          : kso_num_trajectories(dims, spacing, scales, method);
    if (ids == NULL) n = ntraj;
    eval_ctx e;
    e.bv = bv; e.dims = dims; e.bins = bins; e.method = method; e.s_min = scales[0]; e.s_max = scales[1];
    e.eps = (double*)malloc(sizeof(double) * 8 * (size_t)S);
    e.counts = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)bins);
    e.msum = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)bins);
    kso_stats st = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = ids ? ids[i] : i;
        int64_t seed = method == KSO_MEANSHIFT ? id / S : id;
        int32_t s = method == KSO_MEANSHIFT ? scales[0] + (int32_t)(id % S) : 0;
        int32_t gx = (int32_t)(seed % g[0]);
        int32_t gy = (int32_t)((seed / g[0]) % g[1]);
        int32_t gz = (int32_t)(seed / ((int64_t)g[0] * g[1]));
        int32_t p0[3] = {o[0] + gx * spacing, o[1] + gy * spacing, o[2] + gz * spacing};
        if (seeds) {
            p0[0] = seeds[3 * seed]; p0[1] = seeds[3 * seed + 1]; p0[2] = seeds[3 * seed + 2];
        }
        kso_traj* t = out + i;
        t->traj = id;
        run_trajectory(&e, max_iter, p0, s, t, &st);
        int32_t pf[3] = {t->x, t->y, t->z};
        saliency(bv, dims, bins, pf, method, scales[0], scales[1], s, h_min, y_min, t, &st);
    }
    if (stats) *stats = st;
    free(e.eps); free(e.counts); free(e.msum); free(bv);
    return 0;
}

int kso_run(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
            int32_t spacing, const int32_t scales[2], int32_t method, int32_t max_iter, double h_min, double y_min,
            const int64_t* ids, int64_t n, kso_traj* out, kso_stats* stats) {
    return run_impl(vol, dtype, dims, bins, window, spacing, NULL, 0, scales, method, max_iter, h_min, y_min, ids, n,
                    out, stats);
}

int kso_run_seeded(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                   const int32_t* seeds, int64_t n_seeds, const int32_t scales[2], int32_t method, int32_t max_iter,
                   double h_min, double y_min, kso_traj* out, kso_stats* stats) {
    return run_impl(vol, dtype, dims, bins, window, 1, seeds, n_seeds, scales, method, max_iter, h_min, y_min, NULL,
                    0, out, stats);
}

/* ----------------------------------------------------- dense saliency map */

/* The every-voxel Kadir-Brady search (Sec. 1, Sec. 2.1): at every voxel the
 * saliency step of the quadrant method (centred cubes of half-width
 * s_min-1 .. s_max+1, entropy peaks, Y = H * W) with no search before it.
 * Writes s* (0 when there is no peak) and the accurate saliency Y_ref = H_ref * W
 * at s* (0 when there is no peak), x fastest. */
int kso_saliency_map(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                     const int32_t scales[2], float* sal, uint8_t* scale, double* sal64) {
    int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
    uint8_t* bv = (uint8_t*)malloc((size_t)nv);
    bin_any(vol, dtype, dims, bins, window, bv);
    kso_stats st = {0, 0, 0};
    for (int64_t i = 0; i < nv; ++i) {
        int32_t p[3] = {(int32_t)(i % dims[0]), (int32_t)((i / dims[0]) % dims[1]),
                        (int32_t)(i / ((int64_t)dims[0] * dims[1]))};
        kso_traj t;
        saliency(bv, dims, bins, p, KSO_QUADRANT, scales[0], scales[1], 0, 0.0, 0.0, &t, &st);
        scale[i] = (uint8_t)t.scale;
        sal[i] = (float)t.y_ref;
        if (sal64) sal64[i] = t.y64;
    }
    free(bv);
    return 0;
}

/* ------------------------------------------------------------- ranking */

/* Order: rank key (decision precision) descending, then scale, z, y, x, seed
 * ascending.  Equal (x,y,z,scale) records carry equal keys, so duplicates are
 * adjacent and the first one holds the smallest seed. */
static int region_cmp(const void* pa, const void* pb) {
    const kso_region* a = (const kso_region*)pa;
    const kso_region* b = (const kso_region*)pb;
    if (a->key != b->key) return a->key > b->key ? -1 : 1;
    if (a->scale != b->scale) return a->scale < b->scale ? -1 : 1;
    if (a->z != b->z) return a->z < b->z ? -1 : 1;
    if (a->y != b->y) return a->y < b->y ? -1 : 1;
    if (a->x != b->x) return a->x < b->x ? -1 : 1;
    if (a->seed != b->seed) return a->seed < b->seed ? -1 : 1;
    return 0;
}

/* Step 8: the kept trajectories' regions, deduplicated on (x, y, z, scale)
 * (smallest trajectory id kept) and ranked; the order does not depend on the
 * order of the input records. */
int kso_rank(const kso_traj* t, int64_t n, int32_t rank_by, kso_region* out, int32_t capacity, int32_t* n_found) {
    kso_region* r = (kso_region*)malloc(sizeof(kso_region) * (size_t)(n > 0 ? n : 1));
    if (!r) return -1;
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (!t[i].keep) continue;
        kso_region* g = r + m++;
        g->x = t[i].x; g->y = t[i].y; g->z = t[i].z; g->scale = t[i].scale;
        g->saliency = t[i].y_ref; g->entropy = t[i].h_ref; g->pdf_change = t[i].w64;
        g->key = rank_by == KSO_RANK_PDF_CHANGE ? t[i].w64 : t[i].y64;
        g->seed = t[i].traj;
    }
    qsort(r, (size_t)m, sizeof(kso_region), region_cmp);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (u > 0) {
            kso_region* p = r + u - 1;
            if (p->x == r[i].x && p->y == r[i].y && p->z == r[i].z && p->scale == r[i].scale) continue;
        }
        r[u++] = r[i];
    }
    for (int64_t i = 0; i < u && i < capacity; ++i) out[i] = r[i];
    *n_found = (int32_t)u;
    free(r);
    return 0;
}

static int detect_impl(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                       int32_t spacing, const int32_t* seeds, int64_t n_seeds, const int32_t scales[2],
                       int32_t method, int32_t max_iter, double h_min, double y_min, int32_t rank_by,
                       kso_region* out, int32_t capacity, int32_t* n_found, kso_stats* stats) {
    if (!seeds_ok(dims, seeds, n_seeds)) return -1;
    int64_t n = seeds ? n_seeds * (method == KSO_MEANSHIFT ? scales[1] - scales[0] + 1 : 1)
                      : kso_num_trajectories(dims, spacing, scales, method);
    kso_traj* t = (kso_traj*)malloc(sizeof(kso_traj) * (size_t)(n > 0 ? n : 1));
    run_impl(vol, dtype, dims, bins, window, spacing, seeds, n_seeds, scales, method, max_iter, h_min, y_min, NULL, 0,
             t, stats);
    const int rc = kso_rank(t, n, rank_by, out, capacity, n_found);
    free(t);
    return rc;
}

int kso_detect(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
               int32_t spacing, const int32_t scales[2], int32_t method, int32_t max_iter, double h_min, double y_min,
               int32_t rank_by, kso_region* out, int32_t capacity, int32_t* n_found, kso_stats* stats) {
    return detect_impl(vol, dtype, dims, bins, window, spacing, NULL, 0, scales, method, max_iter, h_min, y_min,
                       rank_by, out, capacity, n_found, stats);
}

int kso_detect_seeded(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
                      const int32_t* seeds, int64_t n_seeds, const int32_t scales[2], int32_t method,
                      int32_t max_iter, double h_min, double y_min, int32_t rank_by, kso_region* out,
                      int32_t capacity, int32_t* n_found, kso_stats* stats) {
    return detect_impl(vol, dtype, dims, bins, window, 1, seeds, n_seeds, scales, method, max_iter, h_min, y_min,
                       rank_by, out, capacity, n_found, stats);
}

/* ------------------------------------------------ ABMSOD (Sec. 2.3, Alg. 2) */

/* Symmetric 3x3 matrices are stored as {xx, yy, zz, xy, xz, yz}. */

/* Inverse by cofactors; 0 unless the matrix is positive definite (leading
 * minors and determinant > 0). */
static int sym3_inverse(const double h[6], double inv[6]) {
    double a = h[0], d = h[1], f = h[2], b = h[3], c = h[4], e = h[5];
    double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    double det = a * c00 + b * c01 + c * c02;
    if (!(a > 0.0) || !(a * d - b * b > 0.0) || !(det > 0.0)) return 0;
    inv[0] = c00 / det;
    inv[1] = (a * f - c * c) / det;
    inv[2] = (a * d - b * b) / det;
    inv[3] = c01 / det;
    inv[4] = c02 / det;
    inv[5] = (b * c - a * e) / det;
    return 1;
}

/* Squared Mahalanobis distance u^T H^-1 u. */
static double mahal(const double inv[6], const double u[3]) {
    return inv[0] * u[0] * u[0] + inv[1] * u[1] * u[1] + inv[2] * u[2] * u[2] +
           2.0 * (inv[3] * u[0] * u[1] + inv[4] * u[0] * u[2] + inv[5] * u[1] * u[2]);
}

/* The window of bandwidth H at x: the voxels v of the volume with
 * (v - x)^T H^-1 (v - x) <= 5, the solid ellipsoid whose uniform second moment
 * is H.  Its bounding box has half-extent sqrt(5 H_aa) along axis a. */
typedef struct {
    const uint8_t* bv;
    const int32_t* dims;
    int32_t bins;
    int64_t visits;
} abm_ctx;

enum { ABM_HIST = 0, ABM_MEAN = 1, ABM_COV = 2 };

/* One pass over the window at x with inverse bandwidth inv:
 *   ABM_HIST: G[b] += exp(-d/2) (the Gaussian profile of Alg. 2, unnormalised p_b)
 *   ABM_MEAN: acc[0] += g w, acc[1..3] += g w v      (Eq. 5; -K' of the Gaussian is g/2)
 *   ABM_COV:  acc[0] += w,   acc[1..6] += w (x - v)(x - v)^T   (Eq. 7)
 * with w = w_of_bin[bin(v)]; voxels of the sentinel bin (window level) are skipped. */
static void abm_pass(abm_ctx* c, int kind, const double x[3], const double h[6], const double inv[6],
                     const double* w_of_bin, double* G, double* acc) {
    int32_t lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        double e = sqrt(5.0 * h[a]);
        double l = ceil(x[a] - e), u = floor(x[a] + e);
        lo[a] = l < 0 ? 0 : (int32_t)l;
        hi[a] = u > c->dims[a] - 1 ? c->dims[a] - 1 : (int32_t)u;
    }
    for (int32_t z = lo[2]; z <= hi[2]; ++z)
        for (int32_t y = lo[1]; y <= hi[1]; ++y)
            for (int32_t vx = lo[0]; vx <= hi[0]; ++vx) {
                double u[3] = {vx - x[0], y - x[1], z - x[2]};
                double d = mahal(inv, u);
                if (!(d <= 5.0)) continue;
                c->visits += 1;
                int32_t b = c->bv[vidx(c->dims, vx, y, z)];
                if (b >= c->bins) continue;
                if (kind == ABM_HIST) {
                    G[b] += exp(-d / 2.0);
                } else if (kind == ABM_MEAN) {
                    double gw = exp(-d / 2.0) * w_of_bin[b];
                    acc[0] += gw;
                    acc[1] += gw * vx;
                    acc[2] += gw * y;
                    acc[3] += gw * z;
                } else {
                    double w = w_of_bin[b];
                    acc[0] += w;
                    acc[1] += w * u[0] * u[0];
                    acc[2] += w * u[1] * u[1];
                    acc[3] += w * u[2] * u[2];
                    acc[4] += w * u[0] * u[1];
                    acc[5] += w * u[0] * u[2];
                    acc[6] += w * u[1] * u[2];
                }
            }
}

/* Weights of Eq. 5 for the uniform target q_b = 1/B: w_b = sqrt(q_b / p_b),
 * p_b = G_b / sum G.  Returns sum G (0: empty window). */
static double abm_weights(const double* G, int32_t bins, double* w) {
    double tot = 0.0;
    for (int32_t b = 0; b < bins; ++b) tot += G[b];
    for (int32_t b = 0; b < bins; ++b) w[b] = G[b] > 0.0 ? sqrt((1.0 / bins) / (G[b] / tot)) : 0.0;
    return tot;
}

static void abm_trajectory(abm_ctx* c, const int32_t p0[3], int32_t r, int32_t r_cap, int32_t max_iter,
                           double threshold, kso_ellipsoid* t, kso_stats* st) {
    const int32_t B = c->bins;
    double* G = (double*)calloc((size_t)B, sizeof(double));
    double* w = (double*)calloc((size_t)B, sizeof(double));
    double x[3] = {p0[0], p0[1], p0[2]};
    /* the ball of radius r + 1/2: its boundary passes through no lattice point */
    const double h0 = (r + 0.5) * (r + 0.5) / 5.0;
    double h[6] = {h0, h0, h0, 0.0, 0.0, 0.0};
    double inv[6];
    double best = 0.0;
    t->x[0] = x[0]; t->x[1] = x[1]; t->x[2] = x[2];
    memcpy(t->h, h, sizeof(h));
    t->rho = 0.0;
    t->entropy = 0.0;
    int32_t it = 0, stop = KSO_ABM_MAX_ITER;
    while (it < max_iter) {
        sym3_inverse(h, inv);
        /* position step (Eq. 4, 5) at x */
        memset(G, 0, sizeof(double) * (size_t)B);
        abm_pass(c, ABM_HIST, x, h, inv, NULL, G, NULL);
        st->evals += 1;
        if (abm_weights(G, B, w) == 0.0) { stop = KSO_ABM_EMPTY; break; }
        double m[4] = {0, 0, 0, 0};
        abm_pass(c, ABM_MEAN, x, h, inv, w, NULL, m);
        double xn[3];
        for (int a = 0; a < 3; ++a) {
            xn[a] = m[a + 1] / m[0];
            if (xn[a] < 0.0) xn[a] = 0.0;
            if (xn[a] > c->dims[a] - 1) xn[a] = c->dims[a] - 1;
        }
        /* bandwidth step (Eq. 7) and coefficient at x_new with the same H */
        memset(G, 0, sizeof(double) * (size_t)B);
        abm_pass(c, ABM_HIST, xn, h, inv, NULL, G, NULL);
        st->evals += 1;
        double tot = abm_weights(G, B, w);
        if (tot == 0.0) { stop = KSO_ABM_EMPTY; break; }
        double rho = 0.0, ent = 0.0;
        for (int32_t b = 0; b < B; ++b) {
            if (G[b] <= 0.0) continue;
            double p = G[b] / tot;
            rho += sqrt(p * (1.0 / B));
            ent -= p * log(p);
        }
        double s[7] = {0, 0, 0, 0, 0, 0, 0};
        abm_pass(c, ABM_COV, xn, h, inv, w, NULL, s);
        double hn[6], tmp[6];
        for (int k = 0; k < 6; ++k) hn[k] = s[k + 1] / s[0];
        if (!sym3_inverse(hn, tmp)) { stop = KSO_ABM_DEGENERATE; break; }
        /* keep the window within the largest start window: half-extent r_cap + 1/2 */
        double hmax = hn[0] > hn[1] ? hn[0] : hn[1];
        if (hn[2] > hmax) hmax = hn[2];
        const double cap2 = (r_cap + 0.5) * (r_cap + 0.5);
        if (g_abm_bandwidth_cap && 5.0 * hmax > cap2) {
            double f = cap2 / (5.0 * hmax);
            for (int k = 0; k < 6; ++k) hn[k] *= f;
        }
        /* best-so-far tracking and the termination test of Alg. 2 */
        double delta = best - rho;
        if (rho > best) {
            best = rho;
            memcpy(t->x, xn, sizeof(xn));
            memcpy(t->h, hn, sizeof(hn));
            t->rho = rho;
            t->entropy = ent;
        }
        it += 1;
        double dx = 0.0, dh = 0.0, hd = h[0];
        for (int a = 0; a < 3; ++a) dx = fmax(dx, fabs(xn[a] - x[a]));
        for (int k = 0; k < 6; ++k) dh = fmax(dh, fabs(hn[k] - h[k]));
        hd = fmax(hd, fmax(h[1], h[2]));
        memcpy(x, xn, sizeof(xn));
        memcpy(h, hn, sizeof(hn));
        if (delta > threshold) { stop = KSO_ABM_DETERIORATED; break; }
        if (g_abm_convergence_stop && dx < KSO_ABM_TOL && dh < KSO_ABM_TOL * hd) {
            stop = KSO_ABM_CONVERGED;
            break;
        }
    }
    t->iters = it;
    t->stop = stop;
    free(G);
    free(w);
}

int kso_abmsod(const void* vol, int32_t dtype, const int32_t dims[3], int32_t bins, const int32_t* window,
               int32_t spacing, const int32_t* seeds, int64_t n_seeds, const int32_t radii[2], int32_t max_iter,
               double threshold, const int64_t* ids, int64_t n, kso_ellipsoid* out, kso_stats* stats) {
    if (!seeds_ok(dims, seeds, n_seeds)) return -1;
    if (radii[0] < 1 || radii[0] > radii[1]) return -1;
    int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
    uint8_t* bv = (uint8_t*)malloc((size_t)nv);
    bin_any(vol, dtype, dims, bins, window, bv);
    int32_t g[3], o[3];
    grid_dims(dims, spacing, g, o);
    int32_t R = radii[1] - radii[0] + 1;
    int64_t n_start = seeds ? n_seeds : (int64_t)g[0] * g[1] * g[2];
    if (ids == NULL) n = n_start * R;
    abm_ctx c = {bv, dims, bins, 0};
    kso_stats st = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        int64_t id = ids ? ids[i] : i;
        int64_t seed = id / R;
        int32_t r = radii[0] + (int32_t)(id % R);
        int32_t p0[3];
        if (seeds) {
            p0[0] = seeds[3 * seed]; p0[1] = seeds[3 * seed + 1]; p0[2] = seeds[3 * seed + 2];
        } else {
            p0[0] = o[0] + (int32_t)(seed % g[0]) * spacing;
            p0[1] = o[1] + (int32_t)((seed / g[0]) % g[1]) * spacing;
            p0[2] = o[2] + (int32_t)(seed / ((int64_t)g[0] * g[1])) * spacing;
        }
        kso_ellipsoid* t = out + i;
        t->id = id;
        t->x0 = p0[0]; t->y0 = p0[1]; t->z0 = p0[2];
        t->radius = r;
        abm_trajectory(&c, p0, r, radii[1], max_iter, threshold, t, &st);
    }
    st.window_evals = st.evals;
    st.voxel_visits = c.visits;
    if (stats) *stats = st;
    free(bv);
    return 0;
}

// ABMSOD search with the uniform target pmf (Sec. 2.3: Eq. 4 with the Gaussian
// profile of Alg. 2, the move of Eq. 5, the bandwidth estimate of Eq. 7, and the
// best-coefficient tracking and termination of Alg. 2).
//
// One wavefront per candidate (start position, start radius), persistent: a
// wave pops candidates, largest radius first, from a device counter.  An
// iteration makes three sweeps of the ellipsoid, a row interval per lane:
//   1. Gaussian-weighted histogram and per-bin first moments at x, from which
//      the weighted mean of Eq. 5 follows (the weights depend on the bin only)
//                                                   (LDS, 64-bit fixed point)
//   2. Gaussian-weighted histogram at x_new         (LDS)
//   3. weighted second moment at x_new (Eq. 7)     (registers, wave sum)
// Window membership is (v-x)^T H^-1 (v-x) <= 5, evaluated per voxel.  The
// histograms add exp(-d/2) rounded to 2^-40 (the moments exp(-d/2) (v - x) to
// 2^-32) with 64-bit integer LDS atomics into replicas per wave, so their totals
// do not depend on the order of the additions; the register sums are reduced
// by a fixed butterfly, which leaves the same bits in every lane, so every lane
// takes the same decisions.
#include <hip/hip_runtime.h>

#include <math.h>

#include "../../include/ks.h"
#include "ks_abmsod.h"
#include "ks_device.h"

namespace ks {
namespace {

constexpr double kFix = 1099511627776.0;         // 2^40
constexpr double kUnfix = 1.0 / 1099511627776.0;
constexpr double kFixM = 4294967296.0;           // 2^32
constexpr double kUnfixM = 1.0 / 4294967296.0;
constexpr double kTol = 0.01;
// Occupancy: the kernel is held to 128 VGPRs (4 waves per SIMD; what does not
// fit is spilled outside the voxel loops) and launched with 16 waves per CU.
#ifndef KS_ABM_BLOCKS
#define KS_ABM_BLOCKS 16
#endif
#ifndef KS_ABM_WAVES
#define KS_ABM_WAVES 4
#endif
constexpr int kBlocksPerCu = KS_ABM_BLOCKS;

enum { kHist = 0, kHistMean = 1, kCov = 2 };

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Inverse of a symmetric 3x3 matrix {xx, yy, zz, xy, xz, yz} by cofactors;
// false unless positive definite.
__device__ __forceinline__ bool sym3_inv(const double h[6], double inv[6]) {
    const double a = h[0], d = h[1], f = h[2], b = h[3], c = h[4], e = h[5];
    const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
    const double det = a * c00 + b * c01 + c * c02;
    if (!(a > 0.0) || !(a * d - b * b > 0.0) || !(det > 0.0)) return false;
    inv[0] = c00 / det;
    inv[1] = (a * f - c * c) / det;
    inv[2] = (a * d - b * b) / det;
    inv[3] = c01 / det;
    inv[4] = c02 / det;
    inv[5] = (b * c - a * e) / det;
    return true;
}

// The Gaussian weight g = exp(-d/2) along a row of a sweep.  d is a quadratic in
// the voxel's x with second difference 2 H^-1_xx, so from one voxel to the next
// g is multiplied by r = exp(-(d(x+1) - d(x))/2), and r by q = exp(-H^-1_xx).  The
// pair is taken exactly (two exps) at a row's first voxel inside the window and
// again after every kRowAnchor voxels, and advanced by the two products on every
// voxel in between (relative error below 1e-13 in a check over random
// bandwidths and rows, inside the sweep's 2^-40 fixed point).  All lanes take
// the first anchor at once, before their rows' loops, at the voxel the closed
// form names as the first inside; an anchor anywhere else (a row whose rounding
// of d disagrees, a long row) is taken where it falls.
constexpr int kRowAnchor = 32;
struct RowWeight {
    double g, r;
    int left;        // voxels until the next exact anchor (0: anchor at the next voxel inside)
    int at;          // the voxel of the precomputed anchor
    double ga, ra;   // g and r there
};

__device__ __forceinline__ double row_step_exponent(const double inv[6], double u0, double u1, double u2) {
    return -(inv[0] * (2.0 * u0 + 1.0) + 2.0 * (inv[3] * u1 + inv[4] * u2)) / 2.0;
}

// One voxel of a sweep: the membership test (v-x)^T H^-1 (v-x) <= 5 and the
// sweep's accumulation.
//   kHist:     hist[bin] += round(g 2^40), g = exp(-d/2)      (this lane's replica)
//   kHistMean: as kHist, and hist[(1..3) B + bin] += round(g (v - x)_a 2^32)
//   kCov:      acc[0] += w, acc[1..6] += w (v - x)(v - x)^T   (Eq. 7)
template <int KIND>
__device__ __forceinline__ void abm_voxel(const VolDesc& v, int vx, int vy, int vz, int b, const double x[3],
                                          const double inv[6], double q, RowWeight& rw, unsigned long long* hist,
                                          const double* wtab, double* acc, unsigned& visits) {
    const double u0 = vx - x[0], u1 = vy - x[1], u2 = vz - x[2];
    const double d = inv[0] * u0 * u0 + inv[1] * u1 * u1 + inv[2] * u2 * u2 +
                     2.0 * (inv[3] * u0 * u1 + inv[4] * u0 * u2 + inv[5] * u1 * u2);
    const bool in = d <= 5.0;
    if (KIND == kHist || KIND == kHistMean) {
        if (in && rw.left <= 0) {
            if (vx == rw.at) {
                rw.g = rw.ga;
                rw.r = rw.ra;
            } else {
                rw.g = exp(-d / 2.0);
                rw.r = exp(row_step_exponent(inv, u0, u1, u2));
            }
            rw.left = kRowAnchor;
        }
    }
    if (in) {
        ++visits;
        if (b < v.B) {
            if (KIND == kHist || KIND == kHistMean) {
                const double g = rw.g;
                atomicAdd(&hist[b], (unsigned long long)__double2ull_rn(g * kFix));
                if (KIND == kHistMean) {
                    const int B = v.B;
                    atomicAdd(&hist[B + b], (unsigned long long)__double2ll_rn(g * u0 * kFixM));
                    atomicAdd(&hist[2 * B + b], (unsigned long long)__double2ll_rn(g * u1 * kFixM));
                    atomicAdd(&hist[3 * B + b], (unsigned long long)__double2ll_rn(g * u2 * kFixM));
                }
            } else {
                const double wb = wtab[b];
                acc[0] += wb;
                acc[1] += wb * u0 * u0;
                acc[2] += wb * u1 * u1;
                acc[3] += wb * u2 * u2;
                acc[4] += wb * u0 * u1;
                acc[5] += wb * u0 * u2;
                acc[6] += wb * u1 * u2;
            }
        }
    }
    if (KIND == kHist || KIND == kHistMean) {
        // on to the next voxel of the row (also past the window's end: the
        // window's voxels of a row are contiguous, but a rounding of d must not
        // leave g a voxel behind)
        if (rw.left > 0) {
            rw.g *= rw.r;
            rw.r *= q;
            --rw.left;
        }
    }
}

__device__ __forceinline__ int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

// One sweep of the window of bandwidth h at x, a row (y, z) per lane.  The
// slice of the ellipsoid at z = x_z + c is the ellipse of the Schur complement
// Hc = H_xy,xy - H_xy,z H_z,xy / H_zz, centred at x_xy + c H_xy,z / H_zz, of
// squared radius 5 - c^2 / H_zz in the metric of Hc, and its row at y has a
// closed-form x interval; the lane walks that interval widened by one voxel at
// each end (the exact test decides membership), four voxels per dword load.
// Returns the lane's count of window voxels.
template <int KIND>
__device__ __forceinline__ unsigned abm_sweep(const VolDesc& v, const double x[3], const double h[6],
                                              const double inv[6], unsigned long long* hist, const double* wtab,
                                              double* acc, int lane) {
    unsigned visits = 0;
    const double h22 = h[2];
    const double ey = sqrt(5.0 * h[1]), ez = sqrt(5.0 * h22);
    const int ylo = clampi((int)ceil(x[1] - ey) - 1, 0, v.Y - 1), yhi = clampi((int)floor(x[1] + ey) + 1, 0, v.Y - 1);
    const int zlo = clampi((int)ceil(x[2] - ez) - 1, 0, v.Z - 1), zhi = clampi((int)floor(x[2] + ez) + 1, 0, v.Z - 1);
    const double k0 = h[4] / h22, k1 = h[5] / h22;
    const double c00 = h[0] - h[4] * k0, c11 = h[1] - h[5] * k1, c01 = h[3] - h[4] * k1;
    const double qy = c01 / c11, c00r = c00 - c01 * qy;
    const double q = KIND == kCov ? 0.0 : exp(-inv[0]);   // the row weight's ratio of ratios
    // The rows that can touch the ellipse, slice by slice: at z the row y meets it
    // when (y - x_y - c k1)^2 <= c11 (5 - c^2 / H_zz + 1), the bound of the exact
    // test below; the range is widened by a row at each end so that rounding
    // cannot drop a row the test would take.  Lane l of the wave takes slice
    // z0 + l; the slices' rows are laid end to end and dealt to the lanes, so
    // that no lane idles on a row outside the ellipse.
    for (int z0 = zlo; z0 <= zhi; z0 += 64) {
        int ya = 0, cnt = 0;
        if (z0 + lane <= zhi) {
            const double c = (z0 + lane) - x[2];
            const double rr1 = 5.0 - c * c / h22 + 1.0;
            if (rr1 >= 0.0) {
                const double yc = x[1] + c * k1, half = sqrt(c11 * rr1);
                ya = max((int)ceil(yc - half) - 1, ylo);
                const int yb = min((int)floor(yc + half) + 1, yhi);
                cnt = max(yb - ya + 1, 0);
            }
        }
        int pre = cnt;  // inclusive prefix over the lanes' slices
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(pre, o, 64);
            if (lane >= o) pre += t;
        }
        const int total = __shfl(pre, 63, 64);
        for (int row0 = 0; row0 < total; row0 += 64) {
            // the slice of this row: the number of slices whose prefix is <= row
            // (the lane shuffles run with every lane active; rows past the end
            // are dropped after them)
            const int row = row0 + lane;
            int l = 0;
#pragma unroll
            for (int b = 32; b >= 1; b >>= 1) {
                const int pl = __shfl(pre, l + b - 1, 64);
                l += pl <= row ? b : 0;
            }
            const int before = __shfl(pre, l > 0 ? l - 1 : 0, 64);
            const int yl = __shfl(ya, l, 64);
            if (row >= total) continue;
            const int vz = z0 + l, vy = yl + (row - (l > 0 ? before : 0));
        const double c = vz - x[2];
        const double rr = 5.0 - c * c / h22;
        const double t = vy - (x[1] + c * k1);
        const double rx = rr - t * t / c11;
        if (rx < -1.0) continue;    // at least a voxel from the ellipse
        const double mx = x[0] + c * k0 + qy * t, ex = sqrt(rx > 0.0 ? rx * c00r : 0.0);
        const int xa = clampi((int)ceil(mx - ex) - 1, 0, v.X - 1);
        const int xb = clampi((int)floor(mx + ex) + 1, 0, v.X - 1);
        const uint8_t* rowp = v.bins + (int64_t)vz * v.slice + (int64_t)vy * v.xp;
        RowWeight rw{0.0, 0.0, 0, -1, 0.0, 0.0};
        if (KIND != kCov) {
            // the first anchor of every lane's row at once: the first voxel at or
            // past the ellipse's x interval (d computed as the voxel test does)
            const int xf = clampi((int)ceil(mx - ex), xa, xb);
            const double u0 = xf - x[0], u1 = vy - x[1], u2 = vz - x[2];
            const double d = inv[0] * u0 * u0 + inv[1] * u1 * u1 + inv[2] * u2 * u2 +
                             2.0 * (inv[3] * u0 * u1 + inv[4] * u0 * u2 + inv[5] * u1 * u2);
            if (d <= 5.0) {
                rw.at = xf;
                rw.ga = exp(-d / 2.0);
                rw.ra = exp(row_step_exponent(inv, u0, u1, u2));
            }
        }
        for (int x4 = xa & ~3; x4 <= xb; x4 += 4) {
            const uint32_t word = *reinterpret_cast<const uint32_t*>(rowp + x4);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int vx = x4 + k;
                if (vx < xa || vx > xb) continue;
                abm_voxel<KIND>(v, vx, vy, vz, (word >> (8 * k)) & 0xFFu, x, inv, q, rw, hist, wtab, acc, visits);
            }
        }
        }
    }
    return visits;
}

// Folds the R replicas (stride 4 B words each: totals, then the three moment
// rows) into per-bin totals and clears them, writes the Eq. 5 weights
// sqrt(q_b / p_b) (q_b = 1/B) into wtab and returns the total (fixed point).
// rho and ent receive sum_b sqrt(p_b q_b) and -sum_b p_b ln p_b.  With moments,
// shift receives the Eq. 5 move sum_b w_b M_b / sum_b w_b G_b.
__device__ __forceinline__ unsigned long long abm_fold(unsigned long long* hist, double* wtab, int B, int R,
                                                       int lane, bool moments, double& rho, double& ent,
                                                       double shift[3]) {
    __syncthreads();
    unsigned long long part = 0;
    long long mom[4][3];   // per-lane moments of up to 4 bins (B <= 256)
    for (int b = lane, i = 0; b < B; b += 64, ++i) {
        unsigned long long s = 0;
        long long m0 = 0, m1 = 0, m2 = 0;
        for (int r = 0; r < R; ++r) {
            unsigned long long* h = hist + r * 4 * B;
            s += h[b];
            h[b] = 0;
            if (moments) {
                m0 += (long long)h[B + b];
                m1 += (long long)h[2 * B + b];
                m2 += (long long)h[3 * B + b];
                h[B + b] = 0;
                h[2 * B + b] = 0;
                h[3 * B + b] = 0;
            }
        }
        mom[i][0] = m0; mom[i][1] = m1; mom[i][2] = m2;
        part += s;
        wtab[b] = (double)s;    // raw total until the sum over bins is known
    }
    const unsigned long long tot = wave_sum_u64(part);
    const double totd = (double)tot * kUnfix;
    double r0 = 0.0, e0 = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0, dn = 0.0;
    for (int b = lane, i = 0; b < B; b += 64, ++i) {
        const double g = wtab[b] * kUnfix;
        double wb = 0.0;
        if (g > 0.0) {
            const double p = g / totd;
            wb = sqrt((1.0 / B) / p);
            r0 += sqrt(p * (1.0 / B));
            e0 -= p * log(p);
            if (moments) {
                dn += wb * g;
                n0 += wb * ((double)mom[i][0] * kUnfixM);
                n1 += wb * ((double)mom[i][1] * kUnfixM);
                n2 += wb * ((double)mom[i][2] * kUnfixM);
            }
        }
        wtab[b] = wb;
    }
    rho = wave_sum(r0);
    ent = wave_sum(e0);
    if (moments) {
        const double den = wave_sum(dn);
        shift[0] = wave_sum(n0) / den;
        shift[1] = wave_sum(n1) / den;
        shift[2] = wave_sum(n2) / den;
    }
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KS_ABM_WAVES))) void k_abmsod(const VolDesc* vols, AbmArgs a,
                                                                                              ks_ellipsoid* out, Counters* cnt) {
    extern __shared__ unsigned long long smem[];
    // the best-so-far centre, bandwidth, coefficient and entropy of the wave's
    // candidate (written and read by lane 0 only; kept out of registers)
    __shared__ double s_keep[11];
    const VolDesc& v = vols[0];
    const int lane = threadIdx.x;
    const int B = v.B;
    const int R = a.replicas;
    unsigned long long* hist_all = smem;
    double* wtab = reinterpret_cast<double*>(smem + 4 * R * B);
    for (int i = lane; i < 4 * R * B; i += 64) hist_all[i] = 0;
    __syncthreads();
    unsigned long long* hist = hist_all + (lane & (R - 1)) * 4 * B;    // this lane's replica
    const long long ntask = a.n_start * a.R;
    const double cap2 = (a.r_max + 0.5) * (a.r_max + 0.5);
    for (;;) {
        unsigned long long t0 = 0;
        if (lane == 0) t0 = atomicAdd(&cnt->queue_head[1], 1ull);
        const long long t = (long long)__shfl((long long)t0, 0, 64);
        if (t >= ntask) break;
        const int ridx = a.R - 1 - (int)(t / a.n_start);
        const long long seed = t % a.n_start;
        const long long id = seed * a.R + ridx;
        const int r = a.r_min + ridx;
        int p0[3];
        seed_pos(v, seed, p0);
        double x[3] = {(double)p0[0], (double)p0[1], (double)p0[2]};
        const double h0 = (r + 0.5) * (r + 0.5) / 5.0;
        double h[6] = {h0, h0, h0, 0.0, 0.0, 0.0};
        double inv[6];
        double best = 0.0;
        if (lane == 0) {
            for (int k = 0; k < 3; ++k) s_keep[k] = x[k];
            for (int k = 0; k < 6; ++k) s_keep[3 + k] = h[k];
            s_keep[9] = 0.0;
            s_keep[10] = 0.0;
        }
        int it = 0, stop = KS_ABM_MAX_ITER;
        unsigned visits = 0;
        int evals = 0;
        while (it < a.max_iter) {
            sym3_inv(h, inv);
            // Eq. 4 and 5 at x: one pass gives the histogram and the per-bin moments
            // (window voxels counted for the histogram and the mean, as two passes)
            visits += 2 * abm_sweep<kHistMean>(v, x, h, inv, hist, wtab, nullptr, lane);
            ++evals;
            double rho, ent, m[3];
            if (abm_fold(hist_all, wtab, B, R, lane, true, rho, ent, m) == 0) { stop = KS_ABM_EMPTY; break; }
            const double dims[3] = {(double)(v.X - 1), (double)(v.Y - 1), (double)(v.Z - 1)};
            double xn[3];
            for (int k = 0; k < 3; ++k) {
                xn[k] = x[k] + m[k];
                xn[k] = xn[k] < 0.0 ? 0.0 : (xn[k] > dims[k] ? dims[k] : xn[k]);
            }
            // coefficient and Eq. 7 at x_new with the same H
            visits += abm_sweep<kHist>(v, xn, h, inv, hist, wtab, nullptr, lane);
            ++evals;
            if (abm_fold(hist_all, wtab, B, R, lane, false, rho, ent, m) == 0) { stop = KS_ABM_EMPTY; break; }
            double s[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            visits += abm_sweep<kCov>(v, xn, h, inv, hist, wtab, s, lane);
            for (int k = 0; k < 7; ++k) s[k] = wave_sum(s[k]);
            __syncthreads();
            double hn[6], tmp[6];
            for (int k = 0; k < 6; ++k) hn[k] = s[k + 1] / s[0];
            if (!sym3_inv(hn, tmp)) { stop = KS_ABM_DEGENERATE; break; }
            double hmax = hn[0] > hn[1] ? hn[0] : hn[1];
            if (hn[2] > hmax) hmax = hn[2];
            if (5.0 * hmax > cap2) {
                const double f = cap2 / (5.0 * hmax);
                for (int k = 0; k < 6; ++k) hn[k] *= f;
            }
            // best-so-far tracking and the termination test of Alg. 2
            const double delta = best - rho;
            if (rho > best) {
                best = rho;
                if (lane == 0) {
                    for (int k = 0; k < 3; ++k) s_keep[k] = xn[k];
                    for (int k = 0; k < 6; ++k) s_keep[3 + k] = hn[k];
                    s_keep[9] = rho;
                    s_keep[10] = ent;
                }
            }
            ++it;
            double dx = 0.0, dh = 0.0, hd = h[0];
            for (int k = 0; k < 3; ++k) dx = fmax(dx, fabs(xn[k] - x[k]));
            for (int k = 0; k < 6; ++k) dh = fmax(dh, fabs(hn[k] - h[k]));
            hd = fmax(hd, fmax(h[1], h[2]));
            for (int k = 0; k < 3; ++k) x[k] = xn[k];
            for (int k = 0; k < 6; ++k) h[k] = hn[k];
            if (delta > a.threshold) { stop = KS_ABM_DETERIORATED; break; }
            if (dx < kTol && dh < kTol * hd) { stop = KS_ABM_CONVERGED; break; }
        }
        const unsigned long long nv = wave_sum_u64((unsigned long long)visits);
        if (lane == 0) {
            ks_ellipsoid e;
            e.x0 = p0[0]; e.y0 = p0[1]; e.z0 = p0[2];
            e.radius = r;
            for (int k = 0; k < 3; ++k) e.x[k] = s_keep[k];
            for (int k = 0; k < 6; ++k) e.h[k] = s_keep[3 + k];
            e.rho = s_keep[9];
            e.entropy = s_keep[10];
            e.iters = it;
            e.stop = stop;
            out[id] = e;
            atomicAdd(&cnt->evals, (unsigned long long)evals);
            atomicAdd(&cnt->voxel_visits, nv);
        }
    }
}

}  // namespace

int abmsod_replicas(int B) { return B <= 128 ? 4 : 2; }

size_t abmsod_lds_bytes(int B) { return (size_t)abmsod_replicas(B) * 4 * B * 8 + (size_t)B * 8; }

int abmsod_blocks_per_cu() { return kBlocksPerCu; }

hipError_t launch_abmsod(const VolDesc* vols, const AbmArgs& a, int B, int grid, ks_ellipsoid* out, Counters* cnt,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_abmsod, dim3(grid), dim3(64), abmsod_lds_bytes(B), st, vols, a, out, cnt);
    return hipGetLastError();
}

}  // namespace ks

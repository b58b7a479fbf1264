// gfx950 kernels of the seed-grid Kadir-Brady search.
//
// Work split (one volume or a batch of volumes alike):
//   k_prep_init / k_minmax / k_quantize  per-volume range scan and binning into a
//                                         uint8 bin volume with 16-byte row pitch
//   k_search_ms    persistent; one wavefront runs one mean-shift trajectory at a
//                  time (Sec. 2.3): per evaluation it scatters the window's voxels
//                  into wave-private packed LDS histograms (count + three offset
//                  sums in one 64-bit LDS add), merges them lane-per-bin and takes
//                  the move and the Bhattacharyya objective by butterfly sums
//   k_search_quad  persistent; one 256-thread workgroup runs one quadrant
//                  trajectory (Sec. 2.2, Alg. 1): per evaluation, 8 octant passes
//                  scatter the octant brick into shell-bucketed LDS histograms,
//                  prefix them over the shell radius and take all entropies
//   both kernels end each trajectory with the Kadir-Brady saliency pass at the
//   converged position and write one TrajRec
//   k_compact / bitonic / dedup / emit    rank on the device
//
// Decision arithmetic (argmax over scale, moves, acceptance, peaks, ranking) is
// IEEE double with contraction disabled (-ffp-contract=off) and every sum over
// bins taken as a pairwise halving tree over max(64, pow2 >= B) terms: the lane
// butterfly below produces exactly that tree.
#include <limits.h>

#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double bfly_sum(double v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = v + __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ float bfly_sumf(float v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = v + __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ long long bfly_sumll(long long v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v = v + __shfl_xor(v, m, 64);
    return v;
}

// Halving tree over a lane's m (1, 2 or 4) contiguous bins.
__device__ __forceinline__ double local_pw(const double* v, int m) {
    if (m == 1) return v[0];
    if (m == 2) return v[0] + v[1];
    return (v[0] + v[1]) + (v[2] + v[3]);
}

__device__ __forceinline__ int bins_per_lane(int B) { return B <= 64 ? 1 : (B <= 128 ? 2 : 4); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t clipped_len(int c, int r, int n) {
    int lo = c - r < 0 ? 0 : c - r;
    int hi = c + r > n - 1 ? n - 1 : c + r;
    return hi - lo + 1;
}

__device__ __forceinline__ int64_t cube_count(const VolDesc& v, int px, int py, int pz, int r) {
    return clipped_len(px, r, v.X) * clipped_len(py, r, v.Y) * clipped_len(pz, r, v.Z);
}

// Lane layout of a box scan: each active lane owns one dword column d of a row
// (oy, oz) inside a tile of ty x tz rows; tiles then sweep the box.
struct TileMap {
    int ty, tz;
    int oy, oz, d;
    bool on;
};

__device__ __forceinline__ TileMap tile_map(int nd, int ny, int nz, int nt, int tid) {
    TileMap m;
    m.ty = min(ny, nt / nd);
    m.tz = min(nz, nt / (m.ty * nd));
    int per_z = m.ty * nd;
    m.on = tid < m.tz * per_z;
    m.oz = tid / per_z;
    int rem = tid - m.oz * per_z;
    m.oy = rem / nd;
    m.d = rem - m.oy * nd;
    return m;
}

__device__ __forceinline__ uint32_t load_word(const VolDesc& v, int y, int z, int x0) {
    const uint8_t* p = v.bins + (size_t)z * (size_t)v.slice + (size_t)y * (size_t)v.xp + (size_t)x0;
    return *reinterpret_cast<const uint32_t*>(p);
}

// ------------------------------------------------------------------ prep

__global__ void k_prep_init(VolDesc* vols, int nvol, Counters* cnt, int* vol_nfound, int* vol_base) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nvol) {
        vols[t].minmax[0] = INT_MAX;
        vols[t].minmax[1] = INT_MIN;
        vol_nfound[t] = 0;
        vol_base[t] = 0;
    }
    if (t == 0) {
        cnt->evals = cnt->window_evals = cnt->voxel_visits = cnt->final_visits = 0;
        cnt->queue_head[0] = cnt->queue_head[1] = 0;
        cnt->n_sort = 0;
    }
}

__device__ __forceinline__ int read_raw(const void* raw, int dtype, int64_t i) {
    if (dtype == 0) return static_cast<const uint8_t*>(raw)[i];
    if (dtype == 1) return static_cast<const uint16_t*>(raw)[i];
    return static_cast<const int16_t*>(raw)[i];
}

__global__ __launch_bounds__(256) void k_minmax(const VolDesc* vols) {
    const VolDesc& v = vols[blockIdx.y];
    const int64_t n = (int64_t)v.X * v.Y * v.Z;
    int lo = INT_MAX, hi = INT_MIN;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int a = read_raw(v.raw, v.dtype, i);
        lo = min(lo, a);
        hi = max(hi, a);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        lo = min(lo, __shfl_xor(lo, m, 64));
        hi = max(hi, __shfl_xor(hi, m, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMin(&v.minmax[0], lo);
        atomicMax(&v.minmax[1], hi);
    }
}

// bin = floor((v - vmin) * B / (vmax - vmin + 1)); 4 voxels of a padded row per thread.
__global__ __launch_bounds__(256) void k_quantize(const VolDesc* vols) {
    const VolDesc& v = vols[blockIdx.y];
    const int qx = v.xp >> 2;
    const int64_t n = (int64_t)qx * v.Y * v.Z;
    const int vmin = v.minmax[0];
    const uint32_t width = (uint32_t)(v.minmax[1] - vmin + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t row = i / qx;
        int x0 = (int)(i - row * qx) * 4;
        int y = (int)(row % v.Y);
        int z = (int)(row / v.Y);
        uint32_t word = 0;
        int64_t base = (int64_t)v.X * ((int64_t)y + (int64_t)v.Y * z);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int x = x0 + k;
            if (x < v.X) {
                uint32_t d = (uint32_t)(read_raw(v.raw, v.dtype, base + x) - vmin);
                word |= ((d * (uint32_t)v.B) / width) << (8 * k);
            }
        }
        *reinterpret_cast<uint32_t*>(v.bins + row * v.xp + x0) = word;
    }
}

// ------------------------------------------------- mean-shift window scatter

// Scatter the cube P + [-s, s]^3 (clipped) of one wavefront into its packed
// per-replica LDS histogram hist[(bin << rl) + replica] and flush into per-lane
// bin totals c/f1/f2/f3 (bins lane*m .. lane*m+m-1).  Search mode: f1..f3 are the
// sums of (dx+s), (dy+s), (dz+s).  Final mode: f1 counts the voxels of the inner
// cube of half-width s-1, f2 = f3 = 0.
template <bool FINAL>
__device__ void ms_window(const VolDesc& v, int px, int py, int pz, int s, int rl, unsigned long long* hist, int lane,
                          int* c, int* f1, int* f2, int* f3) {
    const int B = v.B;
    const int m = bins_per_lane(B);
#pragma unroll
    for (int t = 0; t < 4; ++t) c[t] = f1[t] = f2[t] = f3[t] = 0;
    const int xa = max(px - s, 0), xb = min(px + s, v.X - 1);
    const int ya = max(py - s, 0), yb = min(py + s, v.Y - 1);
    const int za = max(pz - s, 0), zb = min(pz + s, v.Z - 1);
    const int ny = yb - ya + 1, nz = zb - za + 1;
    const int da = xa >> 2, nd = (xb >> 2) - da + 1;
    const TileMap tm = tile_map(nd, ny, nz, 64, lane);
    const int R = 1 << rl;
    const int rep = lane & (R - 1);
    const uint32_t shift = (uint32_t)rl + 3;
    const uint32_t trash = ((uint32_t)((B << rl) | rep)) << 3;
    const uint32_t repoff = (uint32_t)rep << 3;
    const int x0 = (da + tm.d) * 4;
    uint32_t lo[4], off[4], wid[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = x0 + k;
        const bool ok = x >= xa && x <= xb;
        const int dx = x - px;
        lo[k] = FINAL ? (1u | ((uint32_t)(dx < s && dx > -s) << 10)) : (1u | ((uint32_t)(dx + s) << 10));
        off[k] = ok ? repoff : trash;
        wid[k] = ok ? 8u : 0u;
    }
    // Each replica may take kMaxPerReplica voxels between flushes: a step adds at
    // most 4 voxels per lane and 64/R lanes share a replica.
    const int flush_every = (kMaxPerReplica << rl) >> 8;
    int since = 0;
    for (int iz0 = 0; iz0 < nz; iz0 += tm.tz) {
        for (int iy0 = 0; iy0 < ny; iy0 += tm.ty) {
            const int iy = iy0 + tm.oy, iz = iz0 + tm.oz;
            if (tm.on && iy < ny && iz < nz) {
                const int y = ya + iy, z = za + iz;
                const uint32_t w = load_word(v, y, z, x0);
                uint32_t hi;
                uint32_t le[4];
                if (FINAL) {
                    const bool inner = (y - py < s) && (py - y < s) && (z - pz < s) && (pz - z < s);
                    hi = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) le[k] = inner ? lo[k] : 1u;
                } else {
                    hi = (uint32_t)(y - py + s) | ((uint32_t)(z - pz + s) << 16);
#pragma unroll
                    for (int k = 0; k < 4; ++k) le[k] = lo[k];
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t b = __builtin_amdgcn_ubfe(w, 8 * k, wid[k]);
                    const uint32_t addr = (b << shift) + off[k];
                    atomicAdd(reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(hist) + addr),
                              ((unsigned long long)hi << 32) | le[k]);
                }
            }
            if (++since == flush_every) {
                since = 0;
                __syncthreads();
                for (int t = 0; t < m; ++t) {
                    const int b = lane * m + t;
                    if (b < B) {
                        unsigned long long* e = hist + ((size_t)b << rl);
                        for (int i = 0; i < R; ++i) {
                            const int r = (i + lane) & (R - 1);
                            const unsigned long long val = e[r];
                            e[r] = 0ull;
                            c[t] += (int)(val & 0x3FFull);
                            f1[t] += (int)((val >> 10) & 0xFFFFull);
                            f2[t] += (int)((val >> 32) & 0xFFFFull);
                            f3[t] += (int)(val >> 48);
                        }
                    }
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    for (int t = 0; t < m; ++t) {
        const int b = lane * m + t;
        if (b < B) {
            unsigned long long* e = hist + ((size_t)b << rl);
            for (int i = 0; i < R; ++i) {
                const int r = (i + lane) & (R - 1);
                const unsigned long long val = e[r];
                e[r] = 0ull;
                c[t] += (int)(val & 0x3FFull);
                f1[t] += (int)((val >> 10) & 0xFFFFull);
                f2[t] += (int)((val >> 32) & 0xFFFFull);
                f3[t] += (int)(val >> 48);
            }
        }
    }
    __syncthreads();
}

struct EvalOut {
    double obj, dx, dy, dz;
};

// Eq. 4-6 with a flat kernel and the uniform target: move = (sum_b M_b/sqrt(c_b)) /
// (sum_b sqrt(c_b)), objective rho~ = (sum_b sqrt(c_b)) / sqrt(N).
__device__ EvalOut ms_eval(const VolDesc& v, const Tables& tb, int px, int py, int pz, int s, int rl,
                           unsigned long long* hist, int lane) {
    int c[4], f1[4], f2[4], f3[4];
    ms_window<false>(v, px, py, pz, s, rl, hist, lane, c, f1, f2, f3);
    const int m = bins_per_lane(v.B);
    double sq[4], tx[4], ty[4], tz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool nz = t < m && c[t] > 0;
        const double rs = nz ? tb.rsq[c[t]] : 0.0;
        sq[t] = nz ? tb.sq[c[t]] : 0.0;
        tx[t] = nz ? (double)(f1[t] - c[t] * s) * rs : 0.0;
        ty[t] = nz ? (double)(f2[t] - c[t] * s) * rs : 0.0;
        tz[t] = nz ? (double)(f3[t] - c[t] * s) * rs : 0.0;
    }
    const double D = bfly_sum(local_pw(sq, m));
    const double nx = bfly_sum(local_pw(tx, m));
    const double ny = bfly_sum(local_pw(ty, m));
    const double nzs = bfly_sum(local_pw(tz, m));
    const int64_t N = cube_count(v, px, py, pz, s);
    EvalOut e;
    e.obj = D / tb.sq[N];
    e.dx = D > 0.0 ? nx / D : 0.0;
    e.dy = D > 0.0 ? ny / D : 0.0;
    e.dz = D > 0.0 ? nzs / D : 0.0;
    return e;
}

struct Saliency {
    int scale, keep;
    double y64;
    float h32, w32, y32;
};

__device__ __forceinline__ float entropy_term32(int c, int64_t N) {
    if (c <= 0) return 0.0f;
    const float p = (float)c / (float)N;
    const float lp = (2 * (int64_t)c > N) ? log1pf(-(float)(N - c) / (float)N) : logf(p);
    return -p * lp;
}

// Kadir-Brady saliency at the trajectory's own scale (mean-shift).
__device__ Saliency ms_saliency(const VolDesc& v, const Tables& tb, int px, int py, int pz, int s, int rl,
                                unsigned long long* hist, int lane) {
    int c[4], in[4], u2[4], u3[4];
    ms_window<true>(v, px, py, pz, s, rl, hist, lane, c, in, u2, u3);
    const int m = bins_per_lane(v.B);
    const int64_t Ns = cube_count(v, px, py, pz, s);
    const int64_t Np = cube_count(v, px, py, pz, s - 1);
    double cl[4];
    long long a = 0;
    float h = 0.0f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        cl[t] = t < m ? tb.cl[c[t]] : 0.0;
        if (t < m) {
            long long d = (long long)c[t] * Np - (long long)in[t] * Ns;
            a += d < 0 ? -d : d;
            h += entropy_term32(c[t], Ns);
        }
    }
    const double S = bfly_sum(local_pw(cl, m));
    const long long A = bfly_sumll(a);
    const float H32 = bfly_sumf(h);
    const double H64 = (tb.cl[Ns] - S) / (double)Ns;
    const double W64 = ((double)(s * s) / (double)(2 * s - 1)) * ((double)A / ((double)Ns * (double)Np));
    Saliency r;
    r.scale = s;
    r.y64 = H64 * W64;
    r.keep = (H64 > v.h_min && r.y64 > v.y_min) ? 1 : 0;
    r.h32 = H32;
    r.w32 = ((float)(s * s) / (float)(2 * s - 1)) * ((float)A / ((float)Ns * (float)Np));
    r.y32 = r.h32 * r.w32;
    return r;
}

// ----------------------------------------------------- task decoding, loop

__device__ __forceinline__ int find_seg(const TaskSeg* segs, int nseg, long long t) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].task_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void seed_pos(const VolDesc& v, long long seed, int* p) {
    const long long gxy = (long long)v.gx * v.gy;
    const int gz = (int)(seed / gxy);
    const long long r = seed - (long long)gz * gxy;
    const int gy = (int)(r / v.gx);
    const int gx = (int)(r - (long long)gy * v.gx);
    p[0] = v.ox + gx * v.sp;
    p[1] = v.oy + gy * v.sp;
    p[2] = v.oz + gz * v.sp;
}

__device__ __forceinline__ int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

struct LocalCounts {
    unsigned long long evals, window_evals, voxel_visits, final_visits;
};

// ------------------------------------------------------- mean-shift kernel

__global__ __launch_bounds__(64) void k_search_ms(const VolDesc* vols, const TaskSeg* segs, int nseg, long long ntask,
                                                  Tables tb, TrajRec* out, Counters* cnt, int rl, int hist_words) {
    extern __shared__ unsigned long long hist[];
    const int lane = threadIdx.x;
    for (int i = lane; i < hist_words; i += 64) hist[i] = 0ull;
    __syncthreads();
    LocalCounts lc = {0, 0, 0, 0};
    for (;;) {
        long long t = 0;
        if (lane == 0) t = (long long)atomicAdd(&cnt->queue_head[1], 1ull);
        t = __shfl(t, 0, 64);
        if (t >= ntask) break;
        const int si = uniform(find_seg(segs, nseg, t));
        const TaskSeg sg = segs[si];
        const VolDesc v = vols[sg.vol];
        const long long seed = sg.seed_begin + (t - sg.task_begin);
        const int s = sg.scale;
        int p0[3];
        seed_pos(v, seed, p0);
        int p[3] = {p0[0], p0[1], p0[2]};
        EvalOut cur = ms_eval(v, tb, p[0], p[1], p[2], s, rl, hist, lane);
        lc.evals += 1;
        lc.window_evals += 1;
        lc.voxel_visits += cube_count(v, p[0], p[1], p[2], s);
        int it = 0, stop;
        for (;;) {
            if (it == v.max_iter) { stop = 0; break; }
            const int mx = (int)round(cur.dx), my = (int)round(cur.dy), mz = (int)round(cur.dz);
            if (mx == 0 && my == 0 && mz == 0) { stop = 1; break; }
            const int qx = clampi(p[0] + mx, 0, v.X - 1);
            const int qy = clampi(p[1] + my, 0, v.Y - 1);
            const int qz = clampi(p[2] + mz, 0, v.Z - 1);
            if (qx == p[0] && qy == p[1] && qz == p[2]) { stop = 2; break; }
            const EvalOut nxt = ms_eval(v, tb, qx, qy, qz, s, rl, hist, lane);
            lc.evals += 1;
            lc.window_evals += 1;
            lc.voxel_visits += cube_count(v, qx, qy, qz, s);
            if (!(nxt.obj > cur.obj)) { stop = 3; break; }
            p[0] = qx; p[1] = qy; p[2] = qz;
            cur = nxt;
            it += 1;
        }
        const Saliency sal = ms_saliency(v, tb, p[0], p[1], p[2], s, rl, hist, lane);
        lc.final_visits += cube_count(v, p[0], p[1], p[2], s);
        lc.window_evals += 2;
        if (lane == 0) {
            const long long local = seed * v.S + (s - v.s_min);
            TrajRec r;
            r.x0 = p0[0]; r.y0 = p0[1]; r.z0 = p0[2];
            r.x = p[0]; r.y = p[1]; r.z = p[2];
            r.scale = sal.scale; r.iters = it; r.stop = stop; r.keep = sal.keep;
            r.objective = cur.obj; r.y64 = sal.y64;
            r.h32 = sal.h32; r.w32 = sal.w32; r.y32 = sal.y32;
            r.seed = (int32_t)local;
            out[v.traj_base + local] = r;
        }
    }
    if (lane == 0) {
        atomicAdd(&cnt->evals, lc.evals);
        atomicAdd(&cnt->window_evals, lc.window_evals);
        atomicAdd(&cnt->voxel_visits, lc.voxel_visits);
        atomicAdd(&cnt->final_visits, lc.final_visits);
    }
}

// ------------------------------------------------ quadrant: bucketed scatter

// Scatter the box [xa,xb]x[ya,yb]x[za,zb] into hist[((row*B + bin) << rq) + replica]
// (uint32), row = max(max(|x-cx|,|y-cy|,|z-cz|) - base, 0); bytes outside the box go
// to row trash_row.
template <int NT>
__device__ void bucket_scatter(const VolDesc& v, int xa, int xb, int ya, int yb, int za, int zb, int cx, int cy,
                               int cz, int base, int trash_row, int rq, uint32_t* hist, int tid) {
    const int ny = yb - ya + 1, nz = zb - za + 1;
    const int da = xa >> 2, nd = (xb >> 2) - da + 1;
    const TileMap tm = tile_map(nd, ny, nz, NT, tid);
    const uint32_t rowbytes = (uint32_t)v.B << (rq + 2);
    const uint32_t rep4 = (uint32_t)(tid & ((1 << rq) - 1)) << 2;
    const uint32_t bshift = (uint32_t)rq + 2;
    const int x0 = (da + tm.d) * 4;
    uint32_t rx[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int x = x0 + k;
        const bool ok = x >= xa && x <= xb;
        const int r = ok ? max(abs(x - cx) - base, 0) : trash_row;
        rx[k] = (uint32_t)r * rowbytes + rep4;
    }
    for (int iz0 = 0; iz0 < nz; iz0 += tm.tz) {
        for (int iy0 = 0; iy0 < ny; iy0 += tm.ty) {
            const int iy = iy0 + tm.oy, iz = iz0 + tm.oz;
            if (tm.on && iy < ny && iz < nz) {
                const int y = ya + iy, z = za + iz;
                const uint32_t w = load_word(v, y, z, x0);
                const int rr = max(max(abs(y - cy), abs(z - cz)) - base, 0);
                const uint32_t RR = (uint32_t)rr * rowbytes + rep4;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t b = (w >> (8 * k)) & 0xFFu;
                    const uint32_t addr = max(rx[k], RR) + (b << bshift);
                    atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(hist) + addr), 1u);
                }
            }
        }
    }
}

// Sum replicas, prefix over rows: cnt[r][b] = voxels of bin b in rows 0..r.
// Clears the histogram rows 0..nrows (the last one is the trash row).
template <int NT>
__device__ void bucket_merge(uint32_t* hist, uint32_t* cnt, int nrows, int B, int rq, int tid) {
    const int R = 1 << rq;
    for (int b = tid; b < B; b += NT) {
        uint32_t acc = 0;
        for (int r = 0; r <= nrows; ++r) {
            uint32_t sum = 0;
            for (int q = 0; q < R; ++q) {
                const int idx = ((r * B + b) << rq) + ((q + b) & (R - 1));
                sum += hist[idx];
                hist[idx] = 0u;
            }
            if (r < nrows) {
                acc += sum;
                cnt[r * B + b] = acc;
            }
        }
    }
}

// H64 = (cl[N] - sum_b cl[c_b]) / N of row r, summed by the lane butterfly.
__device__ __forceinline__ double row_entropy64(const uint32_t* row, int B, int64_t N, const Tables& tb, int lane) {
    const int m = bins_per_lane(B);
    double v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int b = lane * m + t;
        v[t] = (t < m && b < B) ? tb.cl[row[b]] : 0.0;
    }
    const double S = bfly_sum(local_pw(v, m));
    return (tb.cl[N] - S) / (double)N;
}

struct QuadLds {
    uint32_t* hist;
    uint32_t* cnt;
    double* eps;    // [8][S]
    double* hrow;   // [S+2]
    long long* arow; // [S+2]
    double* res;    // [4]
};

__device__ __forceinline__ QuadLds quad_lds(char* smem, const LdsQuad& L) {
    QuadLds q;
    q.hist = reinterpret_cast<uint32_t*>(smem + L.hist_off);
    q.cnt = reinterpret_cast<uint32_t*>(smem + L.cnt_off);
    q.eps = reinterpret_cast<double*>(smem + L.eps_off);
    q.hrow = reinterpret_cast<double*>(smem + L.hrow_off);
    q.arow = reinterpret_cast<long long*>(smem + L.arow_off);
    q.res = reinterpret_cast<double*>(smem + L.res_off);
    return q;
}

// Alg. 1 body in 3D: octant entropies for every scale, per octant the first
// maximising scale, E = sum of the 8 maxima, move = sum_j eps_j k*_j sigma_j / E.
template <int NT>
__device__ EvalOut quad_eval(const VolDesc& v, const Tables& tb, int px, int py, int pz, int rq, const QuadLds& L,
                             int tid) {
    const int S = v.S, B = v.B;
    const int wave = tid >> 6, lane = tid & 63;
    for (int j = 0; j < 8; ++j) {
        const int sx = (j & 1) ? 1 : -1, sy = (j & 2) ? 1 : -1, sz = (j & 4) ? 1 : -1;
        const int xa = sx > 0 ? px : max(px - v.s_max, 0), xb = sx > 0 ? min(px + v.s_max, v.X - 1) : px;
        const int ya = sy > 0 ? py : max(py - v.s_max, 0), yb = sy > 0 ? min(py + v.s_max, v.Y - 1) : py;
        const int za = sz > 0 ? pz : max(pz - v.s_max, 0), zb = sz > 0 ? min(pz + v.s_max, v.Z - 1) : pz;
        bucket_scatter<NT>(v, xa, xb, ya, yb, za, zb, px, py, pz, v.s_min, S, rq, L.hist, tid);
        __syncthreads();
        bucket_merge<NT>(L.hist, L.cnt, S, B, rq, tid);
        __syncthreads();
        const int rx = sx > 0 ? v.X - 1 - px : px, ry = sy > 0 ? v.Y - 1 - py : py, rz = sz > 0 ? v.Z - 1 - pz : pz;
        for (int r = wave; r < S; r += NT / 64) {
            const int k = v.s_min + r;
            const int64_t N = (int64_t)(min(k, rx) + 1) * (min(k, ry) + 1) * (min(k, rz) + 1);
            const double h = row_entropy64(L.cnt + r * B, B, N, tb, lane);
            if (lane == 0) L.eps[j * S + r] = h;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double best[8];
        int ks[8];
        for (int j = 0; j < 8; ++j) {
            best[j] = L.eps[j * S];
            ks[j] = v.s_min;
            for (int r = 1; r < S; ++r) {
                const double e = L.eps[j * S + r];
                if (e > best[j]) { best[j] = e; ks[j] = v.s_min + r; }
            }
        }
        const double E = ((best[0] + best[1]) + (best[2] + best[3])) + ((best[4] + best[5]) + (best[6] + best[7]));
        double d[3];
        for (int a = 0; a < 3; ++a) {
            double t[8];
            for (int j = 0; j < 8; ++j) t[j] = best[j] * (double)(ks[j] * (((j >> a) & 1) ? 1 : -1));
            const double num = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
            d[a] = E == 0.0 ? 0.0 : num / E;
        }
        L.res[0] = E; L.res[1] = d[0]; L.res[2] = d[1]; L.res[3] = d[2];
    }
    __syncthreads();
    EvalOut e;
    e.obj = L.res[0]; e.dx = L.res[1]; e.dy = L.res[2]; e.dz = L.res[3];
    __syncthreads();
    return e;
}

// Kadir-Brady saliency at P* for the quadrant method: centred cubes of every
// half-width s in [s_min-1, s_max+1], entropy peaks over s in [s_min, s_max], the
// peak with the largest H*W (first on ties).
template <int NT>
__device__ Saliency quad_saliency(const VolDesc& v, const Tables& tb, int px, int py, int pz, int rq,
                                  const QuadLds& L, int tid) {
    const int S = v.S, B = v.B;
    const int nrows = S + 2;
    const int base = v.s_min - 1;
    const int wave = tid >> 6, lane = tid & 63;
    const int R = v.s_max + 1;
    bucket_scatter<NT>(v, max(px - R, 0), min(px + R, v.X - 1), max(py - R, 0), min(py + R, v.Y - 1),
                       max(pz - R, 0), min(pz + R, v.Z - 1), px, py, pz, base, nrows, rq, L.hist, tid);
    __syncthreads();
    bucket_merge<NT>(L.hist, L.cnt, nrows, B, rq, tid);
    __syncthreads();
    const int m = bins_per_lane(B);
    for (int r = wave; r < nrows; r += NT / 64) {
        const int s = base + r;
        const int64_t N = cube_count(v, px, py, pz, s);
        const double h = row_entropy64(L.cnt + r * B, B, N, tb, lane);
        long long a = 0;
        if (r > 0) {
            const int64_t Np = cube_count(v, px, py, pz, s - 1);
            for (int t = 0; t < m; ++t) {
                const int b = lane * m + t;
                if (b < B) {
                    long long d = (long long)L.cnt[r * B + b] * Np - (long long)L.cnt[(r - 1) * B + b] * N;
                    a += d < 0 ? -d : d;
                }
            }
        }
        a = bfly_sumll(a);
        if (lane == 0) { L.hrow[r] = h; L.arow[r] = a; }
    }
    __syncthreads();
    if (tid == 0) {
        int best = -1;
        double bestY = 0.0;
        for (int s = v.s_min; s <= v.s_max; ++s) {
            const int r = s - base;
            if (!(L.hrow[r] > L.hrow[r - 1] && L.hrow[r] > L.hrow[r + 1])) continue;
            const int64_t N = cube_count(v, px, py, pz, s);
            const int64_t Np = cube_count(v, px, py, pz, s - 1);
            const double W = ((double)(s * s) / (double)(2 * s - 1)) * ((double)L.arow[r] / ((double)N * (double)Np));
            const double Y = L.hrow[r] * W;
            if (best < 0 || Y > bestY) { best = s; bestY = Y; }
        }
        L.res[0] = (double)best;
        L.res[1] = bestY;
    }
    __syncthreads();
    Saliency out;
    const int best = (int)L.res[0];
    out.scale = best < 0 ? 0 : best;
    out.y64 = best < 0 ? 0.0 : L.res[1];
    out.keep = 0;
    out.h32 = out.w32 = out.y32 = 0.0f;
    if (best >= 0) {
        const int r = best - base;
        const int64_t N = cube_count(v, px, py, pz, best);
        const int64_t Np = cube_count(v, px, py, pz, best - 1);
        float h = 0.0f;
        for (int t = 0; t < m; ++t) {
            const int b = lane * m + t;
            if (b < B) h += entropy_term32((int)L.cnt[r * B + b], N);
        }
        out.h32 = bfly_sumf(h);
        const long long A = L.arow[r];
        out.w32 = ((float)(best * best) / (float)(2 * best - 1)) * ((float)A / ((float)N * (float)Np));
        out.y32 = out.h32 * out.w32;
        out.keep = (L.hrow[r] > v.h_min && out.y64 > v.y_min) ? 1 : 0;
    }
    __syncthreads();
    return out;
}

// --------------------------------------------------------- quadrant kernel

__global__ __launch_bounds__(256) void k_search_quad(const VolDesc* vols, const TaskSeg* segs, int nseg,
                                                     long long ntask, Tables tb, TrajRec* out, Counters* cnt,
                                                     int rq, LdsQuad lay) {
    extern __shared__ __align__(16) char smem[];
    __shared__ long long s_task;
    const int tid = threadIdx.x;
    {
        uint32_t* h = reinterpret_cast<uint32_t*>(smem + lay.hist_off);
        for (int i = tid; i < lay.hist_words; i += 256) h[i] = 0u;
    }
    const QuadLds L = quad_lds(smem, lay);
    __syncthreads();
    LocalCounts lc = {0, 0, 0, 0};
    for (;;) {
        if (tid == 0) s_task = (long long)atomicAdd(&cnt->queue_head[0], 1ull);
        __syncthreads();
        const long long t = s_task;
        __syncthreads();
        if (t >= ntask) break;
        const int si = uniform(find_seg(segs, nseg, t));
        const TaskSeg sg = segs[si];
        const VolDesc v = vols[sg.vol];
        const long long seed = sg.seed_begin + (t - sg.task_begin);
        int p0[3];
        seed_pos(v, seed, p0);
        int p[3] = {p0[0], p0[1], p0[2]};
        EvalOut cur = quad_eval<256>(v, tb, p[0], p[1], p[2], rq, L, tid);
        lc.evals += 1;
        lc.window_evals += 8ull * v.S;
        lc.voxel_visits += cube_count(v, p[0], p[1], p[2], v.s_max);
        int it = 0, stop;
        for (;;) {
            if (it == v.max_iter) { stop = 0; break; }
            const int mx = (int)round(cur.dx), my = (int)round(cur.dy), mz = (int)round(cur.dz);
            if (mx == 0 && my == 0 && mz == 0) { stop = 1; break; }
            const int qx = clampi(p[0] + mx, 0, v.X - 1);
            const int qy = clampi(p[1] + my, 0, v.Y - 1);
            const int qz = clampi(p[2] + mz, 0, v.Z - 1);
            if (qx == p[0] && qy == p[1] && qz == p[2]) { stop = 2; break; }
            const EvalOut nxt = quad_eval<256>(v, tb, qx, qy, qz, rq, L, tid);
            lc.evals += 1;
            lc.window_evals += 8ull * v.S;
            lc.voxel_visits += cube_count(v, qx, qy, qz, v.s_max);
            if (!(nxt.obj > cur.obj)) { stop = 3; break; }
            p[0] = qx; p[1] = qy; p[2] = qz;
            cur = nxt;
            it += 1;
        }
        const Saliency sal = quad_saliency<256>(v, tb, p[0], p[1], p[2], rq, L, tid);
        lc.final_visits += cube_count(v, p[0], p[1], p[2], v.s_max + 1);
        lc.window_evals += (unsigned long long)v.S + 2ull;
        if (tid == 0) {
            TrajRec r;
            r.x0 = p0[0]; r.y0 = p0[1]; r.z0 = p0[2];
            r.x = p[0]; r.y = p[1]; r.z = p[2];
            r.scale = sal.scale; r.iters = it; r.stop = stop; r.keep = sal.keep;
            r.objective = cur.obj; r.y64 = sal.y64;
            r.h32 = sal.h32; r.w32 = sal.w32; r.y32 = sal.y32;
            r.seed = (int32_t)seed;
            out[v.traj_base + seed] = r;
        }
    }
    if (tid == 0) {
        atomicAdd(&cnt->evals, lc.evals);
        atomicAdd(&cnt->window_evals, lc.window_evals);
        atomicAdd(&cnt->voxel_visits, lc.voxel_visits);
        atomicAdd(&cnt->final_visits, lc.final_visits);
    }
}

// ------------------------------------------------------------ test hooks

__global__ __launch_bounds__(64) void k_hook_ms(const VolDesc* vols, int kind, int n, const int* xyz, const int* sc,
                                                int rl, int hist_words, void* outp) {
    extern __shared__ unsigned long long hist[];
    const int lane = threadIdx.x;
    for (int i = lane; i < hist_words; i += 64) hist[i] = 0ull;
    __syncthreads();
    const VolDesc v = vols[0];
    const int B = v.B, m = bins_per_lane(B);
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int px = xyz[3 * w], py = xyz[3 * w + 1], pz = xyz[3 * w + 2], s = sc[w];
        int c[4], f1[4], f2[4], f3[4];
        if (kind == 0) ms_window<true>(v, px, py, pz, s, rl, hist, lane, c, f1, f2, f3);
        else ms_window<false>(v, px, py, pz, s, rl, hist, lane, c, f1, f2, f3);
        for (int t = 0; t < m; ++t) {
            const int b = lane * m + t;
            if (b >= B) continue;
            if (kind == 0) {
                static_cast<uint32_t*>(outp)[(size_t)w * B + b] = (uint32_t)c[t];
            } else {
                int* o = static_cast<int*>(outp) + (size_t)w * 4 * B;
                o[b] = c[t];
                o[B + b] = f1[t] - c[t] * s;
                o[2 * B + b] = f2[t] - c[t] * s;
                o[3 * B + b] = f3[t] - c[t] * s;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_hook_quad(const VolDesc* vols, int kind, int lo, int hi, int n,
                                                   const int* xyz, int rq, LdsQuad lay, uint32_t* outp) {
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x;
    {
        uint32_t* h = reinterpret_cast<uint32_t*>(smem + lay.hist_off);
        for (int i = tid; i < lay.hist_words; i += 256) h[i] = 0u;
    }
    const QuadLds L = quad_lds(smem, lay);
    __syncthreads();
    const VolDesc v = vols[0];
    const int B = v.B, K = hi - lo + 1;
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int px = xyz[3 * w], py = xyz[3 * w + 1], pz = xyz[3 * w + 2];
        if (kind == 1) {
            for (int j = 0; j < 8; ++j) {
                const int sx = (j & 1) ? 1 : -1, sy = (j & 2) ? 1 : -1, sz = (j & 4) ? 1 : -1;
                const int xa = sx > 0 ? px : max(px - hi, 0), xb = sx > 0 ? min(px + hi, v.X - 1) : px;
                const int ya = sy > 0 ? py : max(py - hi, 0), yb = sy > 0 ? min(py + hi, v.Y - 1) : py;
                const int za = sz > 0 ? pz : max(pz - hi, 0), zb = sz > 0 ? min(pz + hi, v.Z - 1) : pz;
                bucket_scatter<256>(v, xa, xb, ya, yb, za, zb, px, py, pz, lo, K, rq, L.hist, tid);
                __syncthreads();
                bucket_merge<256>(L.hist, L.cnt, K, B, rq, tid);
                __syncthreads();
                for (int i = tid; i < K * B; i += 256) outp[((size_t)w * 8 + j) * K * B + i] = L.cnt[i];
                __syncthreads();
            }
        } else {
            bucket_scatter<256>(v, max(px - hi, 0), min(px + hi, v.X - 1), max(py - hi, 0), min(py + hi, v.Y - 1),
                                max(pz - hi, 0), min(pz + hi, v.Z - 1), px, py, pz, lo, K, rq, L.hist, tid);
            __syncthreads();
            bucket_merge<256>(L.hist, L.cnt, K, B, rq, tid);
            __syncthreads();
            for (int i = tid; i < K * B; i += 256) outp[(size_t)w * K * B + i] = L.cnt[i];
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ ranking

__device__ __forceinline__ bool rec_less(const SortRec& a, const SortRec& b) {
    if (a.vol != b.vol) return a.vol < b.vol;
    if (a.ky != b.ky) return a.ky < b.ky;
    if (a.kpos != b.kpos) return a.kpos < b.kpos;
    return a.seed < b.seed;
}

__global__ __launch_bounds__(256) void k_compact(const VolDesc* vols, const TrajRec* rec, SortRec* sr,
                                                 Counters* cnt) {
    const VolDesc& v = vols[blockIdx.y];
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < v.n_traj;
         i += (long long)gridDim.x * blockDim.x) {
        const TrajRec r = rec[v.traj_base + i];
        if (!r.keep) continue;
        const unsigned long long k = atomicAdd(&cnt->n_sort, 1ull);
        SortRec o;
        o.vol = blockIdx.y;
        o.ky = ~(uint64_t)__double_as_longlong(r.y64 + 0.0);
        o.kpos = ((uint64_t)r.scale << 48) | ((uint64_t)r.z << 32) | ((uint64_t)r.y << 16) | (uint64_t)r.x;
        o.seed = (uint32_t)r.seed;
        o.idx = (uint32_t)(v.traj_base + i);
        sr[k] = o;
    }
}

__global__ __launch_bounds__(256) void k_sort_fill(SortRec* sr, unsigned long long n_pad, const Counters* cnt) {
    const unsigned long long count = cnt->n_sort;
    for (unsigned long long i = count + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        SortRec o;
        o.vol = ~0ull; o.ky = ~0ull; o.kpos = ~0ull; o.seed = ~0u; o.idx = ~0u;
        sr[i] = o;
    }
}

__device__ __forceinline__ void cswap(SortRec* a, unsigned i, unsigned j) {
    const SortRec x = a[i], y = a[j];
    if (rec_less(y, x)) { a[i] = y; a[j] = x; }
}

// Stages with block size <= L (L = 2 * blockDim) in LDS: flip step then halving
// steps, every block ascending.  start_k: first stage to run (2 for a full local
// sort; a stage's halving steps only when start_k == 0).
__global__ __launch_bounds__(1024) void k_sort_local(SortRec* sr, unsigned L, unsigned k_first, unsigned j_first,
                                                     const Counters* cnt) {
    extern __shared__ SortRec lsr[];
    const unsigned long long count = cnt->n_sort;
    const unsigned long long start = (unsigned long long)blockIdx.x * L;
    if (start >= count) return;
    for (unsigned i = threadIdx.x; i < L; i += blockDim.x) lsr[i] = sr[start + i];
    __syncthreads();
    if (k_first == 0) {
        // halving steps j_first .. 1 of a stage whose flip already ran
        for (unsigned j = j_first; j >= 1; j >>= 1) {
            for (unsigned p = threadIdx.x; p < L / 2; p += blockDim.x) {
                const unsigned i = (p / j) * 2 * j + (p % j);
                cswap(lsr, i, i + j);
            }
            __syncthreads();
        }
    } else {
        for (unsigned k = 2; k <= L; k <<= 1) {
            for (unsigned p = threadIdx.x; p < L / 2; p += blockDim.x) {
                const unsigned i = (p / (k / 2)) * k + (p % (k / 2));
                cswap(lsr, i, i ^ (k - 1));
            }
            __syncthreads();
            for (unsigned j = k / 4; j >= 1; j >>= 1) {
                for (unsigned p = threadIdx.x; p < L / 2; p += blockDim.x) {
                    const unsigned i = (p / j) * 2 * j + (p % j);
                    cswap(lsr, i, i + j);
                }
                __syncthreads();
            }
        }
    }
    for (unsigned i = threadIdx.x; i < L; i += blockDim.x) sr[start + i] = lsr[i];
}

__global__ __launch_bounds__(256) void k_sort_global(SortRec* sr, unsigned long long n_pad, unsigned long long k,
                                                     unsigned long long j, int flip, const Counters* cnt) {
    const unsigned long long count = cnt->n_sort;
    for (unsigned long long p = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; p < n_pad / 2;
         p += (unsigned long long)gridDim.x * blockDim.x) {
        unsigned long long i, q;
        if (flip) {
            i = (p / (k / 2)) * k + (p % (k / 2));
            q = i ^ (k - 1);
        } else {
            i = (p / j) * 2 * j + (p % j);
            q = i + j;
        }
        if (i >= count) continue;
        const SortRec x = sr[i], y = sr[q];
        if (rec_less(y, x)) { sr[i] = y; sr[q] = x; }
    }
}

__device__ __forceinline__ bool first_of_region(const SortRec* sr, unsigned long long i) {
    if (i == 0) return true;
    const SortRec& a = sr[i];
    const SortRec& b = sr[i - 1];
    return a.vol != b.vol || a.kpos != b.kpos;
}

// Per 1024-element block: number of distinct regions; per volume: regions found.
__global__ __launch_bounds__(1024) void k_dedup_count(const SortRec* sr, const Counters* cnt, int* bsum,
                                                      int* vol_nfound) {
    __shared__ int wsum[16];
    const unsigned long long count = cnt->n_sort;
    const unsigned long long i = (unsigned long long)blockIdx.x * 1024 + threadIdx.x;
    int f = 0;
    if (i < count && first_of_region(sr, i)) {
        f = 1;
        atomicAdd(&vol_nfound[sr[i].vol], 1);
    }
    int s = f;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        bsum[blockIdx.x] = t;
    }
}

// Exclusive scan of the block sums (one block, sequential chunks).
__global__ __launch_bounds__(1024) void k_scan_bsum(int* bsum, int nblk) {
    __shared__ int buf[1024];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblk; base += 1024) {
        const int i = base + threadIdx.x;
        const int x = i < nblk ? bsum[i] : 0;
        buf[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nblk) bsum[i] = carry + buf[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
}

// Global region rank g of every first-of-region element; volume base ranks.
__global__ __launch_bounds__(1024) void k_dedup_rank(const SortRec* sr, const Counters* cnt, const int* bsum,
                                                     int* grank, int* vol_base) {
    __shared__ int buf[1024];
    const unsigned long long count = cnt->n_sort;
    const unsigned long long i = (unsigned long long)blockIdx.x * 1024 + threadIdx.x;
    const int f = (i < count && first_of_region(sr, i)) ? 1 : 0;
    buf[threadIdx.x] = f;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    if (f) {
        const int g = bsum[blockIdx.x] + buf[threadIdx.x] - 1;
        grank[i] = g;
        if (i == 0 || sr[i].vol != sr[i - 1].vol) vol_base[sr[i].vol] = g;
    }
}

__global__ __launch_bounds__(256) void k_emit(const SortRec* sr, const Counters* cnt, const int* grank,
                                              const int* vol_base, const VolDesc* vols, const TrajRec* rec,
                                              ks_region_dev* regions) {
    const unsigned long long count = cnt->n_sort;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (unsigned long long)gridDim.x * blockDim.x) {
        if (!first_of_region(sr, i)) continue;
        const int vol = (int)sr[i].vol;
        const int pos = grank[i] - vol_base[vol];
        const VolDesc& v = vols[vol];
        if (pos >= v.cap) continue;
        const TrajRec r = rec[sr[i].idx];
        ks_region_dev o;
        o.x = r.x; o.y = r.y; o.z = r.z; o.scale = r.scale;
        o.saliency = r.y32; o.entropy = r.h32; o.pdf_change = r.w32;
        o.seed = r.seed;
        regions[v.reg_off + pos] = o;
    }
}

// ------------------------------------------------------------ launchers

static int grid_for(long long n, int threads, int cap) {
    long long g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_init, dim3((a.nvol + 255) / 256), dim3(256), 0, st, a.vols, a.nvol, a.cnt,
                       a.vol_nfound, a.vol_base);
    const int gx = grid_for(a.max_voxels, 256, 2048);
    hipLaunchKernelGGL(k_minmax, dim3(gx, a.nvol), dim3(256), 0, st, a.vols);
    const int gq = grid_for(a.max_words, 256, 4096);
    hipLaunchKernelGGL(k_quantize, dim3(gq, a.nvol), dim3(256), 0, st, a.vols);
    return hipGetLastError();
}

hipError_t launch_search_ms(const SearchArgs& a, int grid, int rl, int hist_words, hipStream_t st) {
    if (a.ntask <= 0) return hipSuccess;
    const size_t lds = (size_t)hist_words * 8;
    hipLaunchKernelGGL(k_search_ms, dim3(grid), dim3(64), lds, st, a.vols, a.segs, a.nseg, a.ntask, a.tb, a.rec,
                       a.cnt, rl, hist_words);
    return hipGetLastError();
}

hipError_t launch_search_quad(const SearchArgs& a, int grid, int rq, const LdsQuad& lay, hipStream_t st) {
    if (a.ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_search_quad, dim3(grid), dim3(256), lay.bytes, st, a.vols, a.segs, a.nseg, a.ntask, a.tb,
                       a.rec, a.cnt, rq, lay);
    return hipGetLastError();
}

hipError_t launch_hook_ms(const VolDesc* vols, int kind, int n, const int* xyz, const int* sc, int rl, int hist_words,
                          void* out, hipStream_t st) {
    hipLaunchKernelGGL(k_hook_ms, dim3(grid_for(n, 1, 4096)), dim3(64), (size_t)hist_words * 8, st, vols, kind, n,
                       xyz, sc, rl, hist_words, out);
    return hipGetLastError();
}

hipError_t launch_hook_quad(const VolDesc* vols, int kind, int lo, int hi, int n, const int* xyz, int rq,
                            const LdsQuad& lay, uint32_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_hook_quad, dim3(grid_for(n, 1, 4096)), dim3(256), lay.bytes, st, vols, kind, lo, hi, n, xyz,
                       rq, lay, out);
    return hipGetLastError();
}

hipError_t launch_rank(const RankArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_compact, dim3(grid_for(a.max_traj, 256, 1024), a.nvol), dim3(256), 0, st, a.vols, a.rec,
                       a.sr, a.cnt);
    const unsigned long long n_pad = a.n_pad;
    hipLaunchKernelGGL(k_sort_fill, dim3(grid_for((long long)n_pad, 256, 4096)), dim3(256), 0, st, a.sr, n_pad,
                       a.cnt);
    const unsigned L = n_pad < 2048 ? (unsigned)n_pad : 2048u;
    const unsigned nblk_local = (unsigned)(n_pad / L);
    const size_t lds = (size_t)L * sizeof(SortRec);
    const unsigned threads = L / 2 < 1024 ? (L / 2 > 0 ? L / 2 : 1) : 1024;
    hipLaunchKernelGGL(k_sort_local, dim3(nblk_local), dim3(threads), lds, st, a.sr, L, 2u, 0u, a.cnt);
    for (unsigned long long k = 2ull * L; k <= n_pad; k <<= 1) {
        hipLaunchKernelGGL(k_sort_global, dim3(grid_for((long long)(n_pad / 2), 256, 8192)), dim3(256), 0, st, a.sr,
                           n_pad, k, 0ull, 1, a.cnt);
        for (unsigned long long j = k / 4; j >= L; j >>= 1) {
            hipLaunchKernelGGL(k_sort_global, dim3(grid_for((long long)(n_pad / 2), 256, 8192)), dim3(256), 0, st,
                               a.sr, n_pad, k, j, 0, a.cnt);
        }
        hipLaunchKernelGGL(k_sort_local, dim3(nblk_local), dim3(threads), lds, st, a.sr, L, 0u, L / 2, a.cnt);
    }
    const int nblk = (int)((n_pad + 1023) / 1024);
    hipLaunchKernelGGL(k_dedup_count, dim3(nblk), dim3(1024), 0, st, a.sr, a.cnt, a.bsum, a.vol_nfound);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, st, a.bsum, nblk);
    hipLaunchKernelGGL(k_dedup_rank, dim3(nblk), dim3(1024), 0, st, a.sr, a.cnt, a.bsum, a.grank, a.vol_base);
    hipLaunchKernelGGL(k_emit, dim3(grid_for((long long)n_pad, 256, 4096)), dim3(256), 0, st, a.sr, a.cnt, a.grank,
                       a.vol_base, a.vols, a.rec, a.regions);
    return hipGetLastError();
}

int max_blocks_ms(int hist_words) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_ms, 64, (size_t)hist_words * 8) != hipSuccess)
        return 1;
    return nb < 1 ? 1 : nb;
}

int max_blocks_quad(size_t lds_bytes) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_quad, 256, lds_bytes) != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

}  // namespace ks

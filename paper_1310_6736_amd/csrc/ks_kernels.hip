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
//                  trajectory (Sec. 2.2, Alg. 1): per evaluation it scatters the 8
//                  octant bricks into shell-bucketed LDS histograms (one region per
//                  octant), prefixes them over the shell radius and takes all 8*S
//                  entropies in one pass
//   both kernels end each trajectory with the Kadir-Brady saliency pass at the
//   converged position and write one TrajRec
//   k_compact / bitonic / merge / dedup   rank on the device
//
// Voxel bricks are read with buffer loads: the lane part of the address is fixed
// for a whole window and each step adds one scalar offset, with several steps'
// loads in flight before their bytes are scattered.
//
// Decision arithmetic (argmax over scale, moves, acceptance, peaks, ranking) is
// IEEE double with contraction disabled (-ffp-contract=off) and every sum over
// bins taken as a pairwise halving tree over max(64, pow2 >= B) terms: the lane
// butterfly below produces exactly that tree.
#include <limits.h>

#include <map>
#include <mutex>
#include <tuple>

#include "ks_device.h"
#include "ks_launch.h"

namespace ks {

// ------------------------------------------------------------------ helpers

// Sweep pipelines: rows per group of loads, groups of loads in flight (measured:
// the mean-shift sweeps, many of them a few rows long, run best with a short
// pipeline; the quadrant brick sweep with narrow groups).  The mean-shift line
// walk, with less loop control per step, runs best with groups of three.
#ifndef KS_MS_UNROLL
#define KS_MS_UNROLL 2
#endif
#ifndef KS_MS_LINE_UNROLL
#define KS_MS_LINE_UNROLL 3
#endif
#ifndef KS_MS_DEPTH
#define KS_MS_DEPTH 1
#endif
#ifndef KS_QUAD_UNROLL
#define KS_QUAD_UNROLL 1
#endif
#ifndef KS_QUAD_DEPTH
#define KS_QUAD_DEPTH 2
#endif
#ifndef KS_QUAD_WB
#define KS_QUAD_WB 8
#endif
#ifndef KS_QUAD_THREADS
#define KS_QUAD_THREADS 256
#endif
constexpr int kMsUnroll = KS_MS_UNROLL, kMsDepth = KS_MS_DEPTH, kMsLineUnroll = KS_MS_LINE_UNROLL;
constexpr int kQuadUnroll = KS_QUAD_UNROLL, kQuadDepth = KS_QUAD_DEPTH;
constexpr int kQuadWB = KS_QUAD_WB;  // bytes (voxels) per lane and step of the octant scatter
// Load offset past the end of every bin volume (volumes stay below 2^31 bytes):
// the buffer range check turns such a load into 0 without a memory access.
constexpr uint32_t kPastEnd = 0x80000000u;

// Moves a double across lanes with a DPP pattern (VALU only, no LDS traffic).
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_double(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Pairwise halving-tree sum over the 64 lanes (lane i holds term i): pairs of
// lanes, then groups of 4, 8 and 16 by DPP (xor 1, xor 2, half-row mirror, row
// mirror: each pairs a block with its neighbour block), then the four row sums
// as (r0 + r1) + (r2 + r3).  Every lane returns the same total.
__device__ __forceinline__ double bfly_sum(double v) {
    v = v + dpp_double<0xB1>(v);   // quad_perm [1,0,3,2]
    v = v + dpp_double<0x4E>(v);   // quad_perm [2,3,0,1]
    v = v + dpp_double<0x141>(v);  // row_half_mirror
    v = v + dpp_double<0x140>(v);  // row_mirror
    return (lane_double(v, 0) + lane_double(v, 16)) + (lane_double(v, 32) + lane_double(v, 48));
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

// Halving tree over a lane's M (1, 2 or 4) contiguous bins.
template <int M>
__device__ __forceinline__ double local_pw(const double* v) {
    if (M == 1) return v[0];
    if (M == 2) return v[0] + v[1];
    return (v[0] + v[1]) + (v[2] + v[3]);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Row stride (in counters) of the shell-bucketed histograms: room for bin B (the
// voxels outside a window level, never read) and odd, so that equal bins of
// neighbouring rows fall in different LDS banks.
__device__ __forceinline__ int row_stride(int B) { return (B + 1) | 1; }

__device__ __forceinline__ int64_t clipped_len(int c, int r, int n) {
    int lo = c - r < 0 ? 0 : c - r;
    int hi = c + r > n - 1 ? n - 1 : c + r;
    return hi - lo + 1;
}

__device__ __forceinline__ int64_t cube_count(const VolDesc& v, int px, int py, int pz, int r) {
    return clipped_len(px, r, v.X) * clipped_len(py, r, v.Y) * clipped_len(pz, r, v.Z);
}

// A copy of the bin volume as seen by a sweep: bytes along the fast axis are
// contiguous, rows along the row axis are `pitch` bytes apart and slices along
// the slice axis `slab` bytes apart.  Two copies exist: x fast (rows y, slices
// z; every volume) and y fast (rows z, slices x; mean-shift volumes), so that
// a box thin in x is swept along y instead of touching one cache line per voxel.
struct Layout {
    const uint8_t* base;
    uint32_t pitch, slab;
    int32_t bytes;
};

__device__ __forceinline__ Layout layout_x(const VolDesc& v) {
    return Layout{v.bins, (uint32_t)v.xp, (uint32_t)v.slice, (int32_t)(v.slice * v.Z)};
}

__device__ __forceinline__ Layout layout_t(const VolDesc& v) {
    return Layout{v.bins_t, (uint32_t)v.yp, (uint32_t)v.slice_t, (int32_t)(v.slice_t * v.X)};
}

// Buffer descriptor of a layout; base and size are made scalar explicitly so that
// every load of a sweep uses one descriptor held in SGPRs.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t layout_rsrc(const Layout& L) {
    const uint64_t a = reinterpret_cast<uint64_t>(L.base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    void* p = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
    const int bytes = __builtin_amdgcn_readfirstlane(L.bytes);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, bytes, 0x00020000);
}

// floor(a / d) for 0 <= a <= 1024 and 1 <= d <= 1024 from the hardware float
// reciprocal: (a + 1/2) / d is at least 1/(2d) away from an integer, far more
// than the rounding of the reciprocal (1 ulp) and of the product (checked for
// every such a and d with the reciprocal off by one ulp either way).  Box
// extents, dword counts and lane indices of the sweeps are all in that range.
__device__ __forceinline__ int small_div(int a, int d) {
    return (int)(((float)a + 0.5f) * __builtin_amdgcn_rcpf((float)d));
}

// A box of a layout swept by NT lanes: fast coordinates [fa, fb], nr rows
// ra, ra + rstep, ... and ns slices sa, sa + sstep, ...  Each active lane owns one
// column of WB bytes (a dword or a qword) of one row of a ty x tz tile of rows; the tile then steps through
// the box, first along the rows, then along the slices.  All fields except the
// lane ones are uniform.
struct Sweep {
    int ny, nz, nd, ty, tz;
    uint32_t pr, ps;    // bytes between consecutive rows, slices of the box
    // lane part
    int lim_y, lim_z;   // rows and slices of the box from the lane's tile position on (lim_y -1: lane unused)
    int oy, oz, x0;     // row and slice index in the tile, fast coordinate of byte 0
    uint32_t voff;      // byte offset of the lane's dword at the first step
};

// The lane part of a sweep whose uniform fields (ny, nz, nd, ty, tz, pr, ps) are
// set: the lane's tile position, limits and first offset.  da is the box's first
// dword (or qword) of the fast axis, ra and sa its first row and slice.
template <int WB = 4>
__device__ __forceinline__ void sweep_lane(const Layout& L, Sweep& w, int da, int ra, int sa, int tid) {
    const int per_z = w.ty * w.nd;
    w.oz = small_div(tid, per_z);
    const int rem = tid - w.oz * per_z;
    w.oy = small_div(rem, w.nd);
    const int d = rem - w.oy * w.nd;
    w.x0 = (da + d) * WB;
    const bool on = tid < w.tz * per_z;
    w.lim_y = on ? w.ny - w.oy : -1;
    w.lim_z = w.nz - w.oz;
    w.voff = (uint32_t)sa * L.slab + (uint32_t)ra * L.pitch + (uint32_t)w.oz * w.ps + (uint32_t)w.oy * w.pr +
             (uint32_t)w.x0;
}

template <int NT, int WB = 4>
__device__ __forceinline__ Sweep make_sweep(const Layout& L, int fa, int fb, int ra, int nr, int rstep, int sa,
                                            int ns, int sstep, int tid) {
    static_assert(WB == 4 || WB == 8, "a lane loads a dword or a qword");
    constexpr int kShift = WB == 8 ? 3 : 2;
    Sweep w;
    w.ny = nr;
    w.nz = ns;
    w.pr = L.pitch * (uint32_t)rstep;
    w.ps = L.slab * (uint32_t)sstep;
    const int da = fa >> kShift;
    w.nd = (fb >> kShift) - da + 1;
    const int rmax = uniform(small_div(NT, w.nd));  // rows one step can take
    w.ty = min(w.ny, rmax);
    w.tz = min(w.nz, uniform(small_div(rmax, w.ty)));
    if (NT > 64) {
        // a workgroup's tile: the ty x tz with ty * tz <= rmax that takes the
        // fewest steps ceil(ny / ty) * ceil(nz / tz) (ty = min(ny, rmax) alone
        // leaves most lanes idle in the last row tile of a box a little taller
        // than rmax)
        int best = small_div(w.ny + w.ty - 1, w.ty) * small_div(w.nz + w.tz - 1, w.tz);
        for (int tz = 2; tz <= min(w.nz, rmax); ++tz) {
            const int ty = min(w.ny, small_div(rmax, tz));
            const int st = small_div(w.ny + ty - 1, ty) * small_div(w.nz + tz - 1, tz);
            if (st < best) {
                best = st;
                w.ty = ty;
                w.tz = tz;
            }
        }
        w.ty = uniform(w.ty);
        w.tz = uniform(w.tz);
    }
    sweep_lane<WB>(L, w, da, ra, sa, tid);
    return w;
}

// Walks the sweep's steps in groups of U steps, keeping D groups of loads in
// flight: the loads of group g + D are issued right after group g is scattered.
// Calls f(word, iy0, iz0, acc) for every step in which the lane's row lies
// inside the box (word: WB voxels, a dword or a qword; iy0, iz0: the step's row
// and slice offset;
// acc = iy0 * ay + iz0 * az, a uniform 64-bit value the caller adds to its
// per-lane terms).  The load offset and acc advance by additions; a group of
// steps whose tiles lie wholly inside the box skips the per-lane row tests.  `used` counts
// the voxels each lane has scattered since the last flush, across calls:
// before a group that would take it past `limit`, flush() runs (uniformly) and
// the count restarts.  Loads for steps past the last one get an offset beyond
// the descriptor's end: they return 0 without a memory access.
template <int WB>
struct LaneWord;
template <>
struct LaneWord<4> {
    using T = uint32_t;
    static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t off) {
        return __builtin_amdgcn_raw_buffer_load_b32(rs, voff, off, 0);
    }
};
template <>
struct LaneWord<8> {
    using T = uint64_t;
    static __device__ __forceinline__ T load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t off) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, off, 0);
        return ((uint64_t)v[1] << 32) | v[0];
    }
};

template <int U, int D, int WB = 4, typename F, typename G>
__device__ __forceinline__ void run_sweep(const Layout& L, const Sweep& w, uint64_t ay, uint64_t az, int& used,
                                          int limit, F&& f, G&& flush) {
    using Word = typename LaneWord<WB>::T;
    const __amdgpu_buffer_rsrc_t rs = layout_rsrc(L);
    const uint32_t xp = (uint32_t)uniform((int)w.pr), slice = (uint32_t)uniform((int)w.ps);
    const int nz = uniform(w.nz), ny = uniform(w.ny), ty = uniform(w.ty), tz = uniform(w.tz);
    const uint32_t dy = (uint32_t)ty * xp, dz = (uint32_t)tz * slice;
    const uint64_t day = (uint64_t)(uint32_t)ty * ay, daz = (uint64_t)(uint32_t)tz * az;
    const int lim_y = w.lim_y, lim_z = w.lim_z;
    constexpr int kGroupVoxels = U * WB;
    // the step about to be loaded
    int iy0 = 0, iz0 = 0;
    uint32_t off = 0, zoff = 0;
    uint64_t acc = 0, zacc = 0;
    Word buf[D][U];
    int by[D][U], bz[D][U];
    uint64_t bacc[D][U];
    bool full[D][U];
    auto load = [&](int g, int u) {
        by[g][u] = iy0;
        bz[g][u] = iz0;
        bacc[g][u] = acc;
        full[g][u] = iy0 + ty <= ny && iz0 + tz <= nz;
        buf[g][u] = LaneWord<WB>::load(rs, w.voff, iz0 < nz ? off : kPastEnd);
        iy0 += ty;
        off += dy;
        acc += day;
        if (iy0 >= ny) {
            iy0 = 0;
            iz0 += tz;
            zoff += dz;
            zacc += daz;
            off = zoff;
            acc = zacc;
        }
    };
#pragma unroll
    for (int g = 0; g < D; ++g) {
#pragma unroll
        for (int u = 0; u < U; ++u) load(g, u);
    }
    bool live = true;
    while (live) {
#pragma unroll
        for (int g = 0; g < D; ++g) {
            // a group that starts past the last step ends the sweep
            live = live && bz[g][0] < nz;
            if (live) {
                if (used + kGroupVoxels > limit) {
                    used = 0;
                    flush();
                }
                bool gfull = true;
#pragma unroll
                for (int u = 0; u < U; ++u) gfull = gfull && full[g][u];
                if (gfull) {
                    // every step's tile inside the box: only the unused lanes sit out
                    if (lim_y >= 0) {
#pragma unroll
                        for (int u = 0; u < U; ++u) f(buf[g][u], by[g][u], bz[g][u], bacc[g][u]);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (by[g][u] < lim_y && bz[g][u] < lim_z) f(buf[g][u], by[g][u], bz[g][u], bacc[g][u]);
                    }
                }
                used += kGroupVoxels;
            }
            // with several groups in flight, refilled on every path (past the end
            // the loads touch no memory), so that the waits on the loads in flight
            // are the same on all of them
            if (D > 1 || live) {
#pragma unroll
                for (int u = 0; u < U; ++u) load(g, u);
            }
        }
    }
}

// run_sweep for a box whose tiles form one line: all its rows fit in one tile
// (ty == ny: the tile steps through the slices) or it has one slice (nz == 1: the
// tile steps through the rows).  One counter and one offset advance per step, with
// no wrap from rows to slices; same calls of f and flush as run_sweep.
template <int U, int D, int WB = 4, typename F, typename G>
__device__ __forceinline__ void run_sweep_line(const Layout& L, const Sweep& w, uint64_t ay, uint64_t az, int& used,
                                               int limit, F&& f, G&& flush) {
    using Word = typename LaneWord<WB>::T;
    const __amdgpu_buffer_rsrc_t rs = layout_rsrc(L);
    const int ny = uniform(w.ny), nz = uniform(w.nz), ty = uniform(w.ty), tz = uniform(w.tz);
    const bool rows = ty < ny;   // then nz == 1
    const int n = rows ? ny : nz, t = rows ? ty : tz;
    const uint32_t dd = rows ? (uint32_t)ty * (uint32_t)uniform((int)w.pr) : (uint32_t)tz * (uint32_t)uniform((int)w.ps);
    const uint64_t dacc = rows ? (uint64_t)(uint32_t)ty * ay : (uint64_t)(uint32_t)tz * az;
    // rows (or slices) of the line from the lane's tile position on; -1: lane unused
    const int lim = w.lim_y < 0 ? -1 : (rows ? w.lim_y : w.lim_z);
    constexpr int kGroupVoxels = U * WB;
    int i0 = 0;   // the step about to be loaded
    uint32_t off = 0;
    uint64_t acc = 0;
    Word buf[D][U];
    int bi[D][U];
    uint64_t bacc[D][U];
    auto load = [&](int g, int u) {
        bi[g][u] = i0;
        bacc[g][u] = acc;
        buf[g][u] = LaneWord<WB>::load(rs, w.voff, i0 < n ? off : kPastEnd);
        i0 += t;
        off += dd;
        acc += dacc;
    };
#pragma unroll
    for (int g = 0; g < D; ++g) {
#pragma unroll
        for (int u = 0; u < U; ++u) load(g, u);
    }
    bool live = true;
    while (live) {
#pragma unroll
        for (int g = 0; g < D; ++g) {
            live = live && bi[g][0] < n;
            if (live) {
                if (used + kGroupVoxels > limit) {
                    used = 0;
                    flush();
                }
                // the group's last tile inside the line: all of them are
                if (bi[g][U - 1] + t <= n) {
                    if (lim >= 0) {
#pragma unroll
                        for (int u = 0; u < U; ++u)
                            f(buf[g][u], rows ? bi[g][u] : 0, rows ? 0 : bi[g][u], bacc[g][u]);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (bi[g][u] < lim) f(buf[g][u], rows ? bi[g][u] : 0, rows ? 0 : bi[g][u], bacc[g][u]);
                    }
                }
                used += kGroupVoxels;
            }
            if (D > 1 || live) {
#pragma unroll
                for (int u = 0; u < U; ++u) load(g, u);
            }
        }
    }
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
        for (int c = 0; c < kMaxMsChunks; ++c)
            for (int k = 0; k < kXcds; ++k) cnt->xq_head[c][k] = 0;
        cnt->n_sort = 0;
        cnt->swept = 0;
        cnt->lds_ops = 0;
    }
}

__device__ __forceinline__ int read_raw(const void* raw, int dtype, int64_t i) {
    if (dtype == 0) return static_cast<const uint8_t*>(raw)[i];
    if (dtype == 1) return static_cast<const uint16_t*>(raw)[i];
    return static_cast<const int16_t*>(raw)[i];
}

// Range scan: per-thread, per-wave and per-block reduction, one atomic pair per
// block.  A 16-byte aligned volume is read in 16-byte words (the voxels of a
// whole number of words), the rest voxel by voxel.
__global__ __launch_bounds__(256) void k_minmax(const VolDesc* vols) {
    __shared__ int slo[4], shi[4];
    const VolDesc& v = vols[blockIdx.y];
    const int64_t n = (int64_t)v.X * v.Y * v.Z;
    const int per_word = v.dtype == 0 ? 16 : 8;
    const int64_t nw = (reinterpret_cast<uintptr_t>(v.raw) & 15) == 0 ? n / per_word : 0;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (int64_t)gridDim.x * blockDim.x;
    int lo = INT_MAX, hi = INT_MIN;
    const uint4* words = static_cast<const uint4*>(v.raw);
    for (int64_t w = gid; w < nw; w += stride) {
        const uint4 q = words[w];
        const uint32_t d[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (v.dtype == 0) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int a = (int)((d[k] >> (8 * b)) & 0xffu);
                    lo = min(lo, a);
                    hi = max(hi, a);
                }
            } else {
                const int a0 = v.dtype == 1 ? (int)(d[k] & 0xffffu) : (int)(int16_t)(d[k] & 0xffffu);
                const int a1 = v.dtype == 1 ? (int)(d[k] >> 16) : (int)(int16_t)(d[k] >> 16);
                lo = min(lo, min(a0, a1));
                hi = max(hi, max(a0, a1));
            }
        }
    }
    for (int64_t i = nw * per_word + gid; i < n; i += stride) {
        const int a = read_raw(v.raw, v.dtype, i);
        lo = min(lo, a);
        hi = max(hi, a);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        lo = min(lo, __shfl_xor(lo, m, 64));
        hi = max(hi, __shfl_xor(hi, m, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        slo[threadIdx.x >> 6] = lo;
        shi[threadIdx.x >> 6] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            lo = min(lo, slo[w]);
            hi = max(hi, shi[w]);
        }
        atomicMin(&v.minmax[0], lo);
        atomicMax(&v.minmax[1], hi);
    }
}

// bin = floor((v - vmin) * B / (vmax - vmin + 1)), or over a window level (Sec.
// 3.2) with B for the voxels outside it; 4 voxels of a padded row per thread.
__global__ __launch_bounds__(256) void k_quantize(const VolDesc* vols) {
    const VolDesc& v = vols[blockIdx.y];
    const int qx = v.xp >> 2;
    const int64_t n = (int64_t)qx * v.Y * v.Z;
    const int vmin = v.minmax[0];
    // window level: voxels outside [win_lo, win_hi] get bin B (never counted)
    const int lo = v.win ? v.win_lo : vmin;
    const uint32_t width = v.win ? (uint32_t)(v.win_hi - v.win_lo + 1) : (uint32_t)(v.minmax[1] - vmin + 1);
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
                const int r = read_raw(v.raw, v.dtype, base + x);
                const uint32_t d = (uint32_t)(r - lo);
                const uint32_t b = (v.win && (r < v.win_lo || r > v.win_hi)) ? (uint32_t)v.B : (d * (uint32_t)v.B) / width;
                word |= b << (8 * k);
            }
        }
        *reinterpret_cast<uint32_t*>(v.bins + row * v.xp + x0) = word;
    }
}

// The y-fastest copy of a mean-shift volume's bins: one 64 x 64 (x, y) tile of
// one z plane per workgroup, transposed through LDS.  Bytes past Y in a row of
// the copy are written as 0.
__global__ __launch_bounds__(256) void k_transpose(const VolDesc* vols, int tiles_x) {
    __shared__ uint32_t tile[64][17];
    const VolDesc& v = vols[blockIdx.z];
    if (v.method != 1 || (int)blockIdx.y >= v.Z) return;
    const int x0 = (int)(blockIdx.x % (unsigned)tiles_x) * 64, y0 = (int)(blockIdx.x / (unsigned)tiles_x) * 64;
    if (x0 >= v.X || y0 >= v.yp) return;
    const int z = blockIdx.y;
    for (int i = threadIdx.x; i < 64 * 16; i += 256) {
        const int r = i >> 4, c = i & 15;
        const int y = y0 + r, x = x0 + 4 * c;
        uint32_t w = 0;
        if (y < v.Y && x < v.xp) w = *reinterpret_cast<const uint32_t*>(v.bins + z * v.slice + (int64_t)y * v.xp + x);
        tile[r][c] = w;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 16; i += 256) {
        const int xr = i >> 4, c = i & 15;
        const int x = x0 + xr, y = y0 + 4 * c;
        if (x >= v.X || y >= v.yp) continue;
        uint32_t w = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) w |= ((tile[4 * c + k][xr >> 2] >> (8 * (xr & 3))) & 0xFFu) << (8 * k);
        *reinterpret_cast<uint32_t*>(v.bins_t + ((int64_t)x * v.Z + z) * v.yp + y) = w;
    }
}

// ------------------------------------------------- mean-shift window scatter
//
// A wavefront sweeps the voxels of one or more boxes into 2^rl replicas of a
// packed 64-bit LDS counter per bin, hist[(bin << rl) + replica], and flushes
// them into per-lane totals of its M bins.  A voxel at offset d from the
// reference point adds
//     sign * (1 + dx' * 2^10 + dy' * 2^32 + dz' * 2^48)   (mod 2^64),  d' = d + s,
// so a replica word holds the net count (bits 0-9) and the sums of dx' (10-31),
// dy' (32-47) and dz' (48-63) of its voxels.  Voxels leave a window with sign -1;
// the fields are then two's complement, and they decode exactly while each stays
// in its signed range: at most 511 voxels per replica between flushes and
// 511 * max|d'| < 2^15.  Sweeps that only add keep every field non-negative and
// take up to 1023 voxels per replica (1023 * 2s < 2^16).

template <int M>
struct BinAcc {
    int c[M], f1[M], f2[M], f3[M];
};

template <int M>
__device__ __forceinline__ void acc_clear(BinAcc<M>& a) {
#pragma unroll
    for (int t = 0; t < M; ++t) a.c[t] = a.f1[t] = a.f2[t] = a.f3[t] = 0;
}

// Adds the four fields of a replica word to the totals of bin t.  SIGNED: the
// fields are two's complement (a sweep with voxels leaving the window); else all
// are non-negative.  With the low word L = c + dx'*2^10 in 32-bit range, the high
// word of w - L is hi + (L < 0) and holds dy' + dz'*2^16.
template <int M, bool SIGNED>
__device__ __forceinline__ void unpack_add(unsigned long long w, int t, BinAcc<M>& a) {
    const uint32_t lo = (uint32_t)w, hi = (uint32_t)(w >> 32);
    if (SIGNED) {
        const int c = __builtin_amdgcn_sbfe((int)lo, 0, 10);
        const int fx = (int)(lo - (uint32_t)c) >> 10;
        const uint32_t h = hi + (lo >> 31);
        const int fy = __builtin_amdgcn_sbfe((int)h, 0, 16);
        const int fz = (int)(h - (uint32_t)fy) >> 16;
        a.c[t] += c; a.f1[t] += fx; a.f2[t] += fy; a.f3[t] += fz;
    } else {
        a.c[t] += (int)(lo & 0x3FFu);
        a.f1[t] += (int)(lo >> 10);
        a.f2[t] += (int)(hi & 0xFFFFu);
        a.f3[t] += (int)(hi >> 16);
    }
}

// Adds the replica words of the lane's bins to its totals and clears them.
template <int M, bool SIGNED>
__device__ __forceinline__ void ms_flush(unsigned long long* hist, int rl, int B, int lane, BinAcc<M>& a) {
    const int half = 1 << (rl - 1);  // replica pairs; rl >= 1
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const int b = lane * M + t;
        if (b < B) {
            unsigned long long* e = hist + ((size_t)b << rl);
            for (int i = 0; i < half; ++i) {
                const int r = ((i + lane) & (half - 1)) << 1;
                ulonglong2* p = reinterpret_cast<ulonglong2*>(e + r);
                const ulonglong2 q = *p;
                *p = make_ulonglong2(0ull, 0ull);
                unpack_add<M, SIGNED>(q.x, t, a);
                unpack_add<M, SIGNED>(q.y, t, a);
            }
        }
    }
}

// --------------------------------------------------- mean-shift box sets
//
// Between two evaluations of a trajectory the window moves from P to Q = P + D
// with |D_a| <= s and most of its voxels stay.  The totals at Q follow from those
// at P: shift the offset sums of all of P's voxels by -c_b * D, then sweep the
// voxels of W(P) \ W(Q) with sign -1 and those of W(Q) \ W(P) with sign +1, all
// relative to Q.  Counts and offset sums are integers, so the totals equal a
// fresh sweep of W(Q) exactly.  The final pass needs the counts of the inner
// cube P + [-(s-1), s-1]^3: the window's counts less its shell (the voxels at
// Chebyshev distance exactly s), or the inner cube swept directly, whichever is
// smaller.

// Coordinates xa, xa + xs, ..., up to xb along x (likewise y, z); steps other
// than 1 take the two opposite faces of a shell in one sweep.
struct Box {
    int xa, xb, ya, yb, za, zb;
    int xs, ys, zs;
};

// The one or two face coordinates c - s, c + s that lie in [0, n-1], as a strided
// range lo, hi, step (empty: lo > hi).
__device__ __forceinline__ void face_range(int c, int s, int n, int& lo, int& hi, int& step) {
    const bool a = c - s >= 0, b = c + s < n;
    lo = a ? c - s : c + s;
    hi = b ? c + s : c - s;
    step = 2 * s;
    if (!a && !b) { lo = 0; hi = -1; }
}

// [p-s, p+s] minus [q-s, q+s], clipped to [0, n-1] (one interval; empty: lo > hi).
__device__ __forceinline__ void range_minus(int p, int q, int s, int n, int& lo, int& hi) {
    if (q > p) {
        lo = p - s; hi = min(p + s, q - s - 1);
    } else if (q < p) {
        lo = max(p - s, q + s + 1); hi = p + s;
    } else {
        lo = 0; hi = -1;
    }
    lo = max(lo, 0);
    hi = min(hi, n - 1);
}

// Box i (0..2) of the clipped cube P + [-s,s]^3 minus the clipped cube
// Q + [-s,s]^3: outside Q's x range; inside it but outside Q's y range; inside
// both but outside Q's z range.
__device__ __forceinline__ Box minus_box(const VolDesc& v, int px, int py, int pz, int qx, int qy, int qz, int s,
                                         int i) {
    Box b;
    b.xs = b.ys = b.zs = 1;
    b.xa = max(max(px, qx) - s, 0); b.xb = min(min(px, qx) + s, v.X - 1);
    b.ya = max(py - s, 0); b.yb = min(py + s, v.Y - 1);
    b.za = max(pz - s, 0); b.zb = min(pz + s, v.Z - 1);
    if (i == 0) {
        range_minus(px, qx, s, v.X, b.xa, b.xb);
    } else if (i == 1) {
        range_minus(py, qy, s, v.Y, b.ya, b.yb);
    } else {
        b.ya = max(max(py, qy) - s, 0); b.yb = min(min(py, qy) + s, v.Y - 1);
        range_minus(pz, qz, s, v.Z, b.za, b.zb);
    }
    return b;
}

// Sets of disjoint boxes, described by scalars so that box i is computed where it
// is swept:
//   kFull   the clipped cube P + [-s,s]^3                        (sign +1, ref P)
//   kMove   W(P) \ W(Q) (boxes 0-2, sign -1), W(Q) \ W(P) (3-5, +1)  (ref Q)
//   kShell  the faces of the clipped cube P + [-s,s]^3 (s >= 1), its voxels at
//           Chebyshev distance exactly s: both x faces, both y faces (x inside),
//           both z faces (x, y inside)                            (+1, ref P)
//   kInner  the clipped cube P + [-(s-1), s-1]^3                 (+1, ref P)
constexpr int kFull = 0, kMove = 1, kShell = 2, kInner = 3;

struct BoxSet {
    int kind, px, py, pz, qx, qy, qz, s;
};

__device__ __forceinline__ int box_count(const BoxSet& bs) {
    return bs.kind == kMove ? 6 : bs.kind == kShell ? 3 : 1;
}

__device__ __forceinline__ Box box_at(const VolDesc& v, const BoxSet& bs, int i, int& sign) {
    const int s = bs.s, px = bs.px, py = bs.py, pz = bs.pz;
    sign = 1;
    Box b;
    if (bs.kind == kMove) {
        if (i < 3) {
            sign = -1;
            b = minus_box(v, px, py, pz, bs.qx, bs.qy, bs.qz, s, i);
        } else {
            b = minus_box(v, bs.qx, bs.qy, bs.qz, px, py, pz, s, i - 3);
        }
    } else if (bs.kind == kShell) {
        b.xs = b.ys = b.zs = 1;
        // across the faces of axis i: the full range along axes before i, the
        // inner range along axes after it
        b.xa = max(px - s + 1, 0); b.xb = min(px + s - 1, v.X - 1);
        b.ya = i < 1 ? max(py - s, 0) : max(py - s + 1, 0);
        b.yb = i < 1 ? min(py + s, v.Y - 1) : min(py + s - 1, v.Y - 1);
        b.za = max(pz - s, 0); b.zb = min(pz + s, v.Z - 1);
        if (i == 0) face_range(px, s, v.X, b.xa, b.xb, b.xs);
        else if (i == 1) face_range(py, s, v.Y, b.ya, b.yb, b.ys);
        else face_range(pz, s, v.Z, b.za, b.zb, b.zs);
    } else {
        const int r = bs.kind == kInner ? s - 1 : s;
        b.xs = b.ys = b.zs = 1;
        b.xa = max(px - r, 0); b.xb = min(px + r, v.X - 1);
        b.ya = max(py - r, 0); b.yb = min(py + r, v.Y - 1);
        b.za = max(pz - r, 0); b.zb = min(pz + r, v.Z - 1);
    }
    return b;
}

// Voxels that a running-window update from P to Q sweeps: |W(P)| + |W(Q)| minus
// twice their intersection (a box: per axis the overlap of the two clipped
// ranges), which equals the summed volumes of the six move boxes.
__device__ __forceinline__ int64_t move_volume(const VolDesc& v, int px, int py, int pz, int qx, int qy, int qz,
                                               int s) {
    auto overlap = [s](int p, int q, int n) {
        const int lo = max(max(p, q) - s, 0), hi = min(min(p, q) + s, n - 1);
        return (int64_t)max(hi - lo + 1, 0);
    };
    const int64_t both = overlap(px, qx, v.X) * overlap(py, qy, v.Y) * overlap(pz, qz, v.Z);
    return cube_count(v, px, py, pz, s) + cube_count(v, qx, qy, qz, s) - 2 * both;
}

// Sweeps the boxes of bs into the packed LDS histogram and adds them (with their
// signs) to acc: counts and sums of d + s, d relative to the set's reference
// point.  Each box is swept a dword column per lane; bytes outside it go to the
// trash slots at trash_base, past every bin layout.  The flush budget runs across
// the boxes.
// Voxels per replica between flushes for a running-window update at half-width
// s: the fields are signed and |d'| <= 3s, so 511 * 3s < 2^15 bounds them.
__device__ __forceinline__ int move_budget(int s) { return min(511, 32767 / (3 * s)); }

template <int M>
__device__ __forceinline__ unsigned long long ms_sweep(const VolDesc& v, BoxSet bs, int rl, int trash_base,
                                                       int move_per_rep, unsigned long long* hist, int lane,
                                                       BinAcc<M>& acc) {
    bs.kind = uniform(bs.kind); bs.px = uniform(bs.px); bs.py = uniform(bs.py); bs.pz = uniform(bs.pz);
    bs.qx = uniform(bs.qx); bs.qy = uniform(bs.qy); bs.qz = uniform(bs.qz); bs.s = uniform(bs.s);
    rl = uniform(rl);
    const int s = bs.s, B = v.B;
    const bool mv = bs.kind == kMove;
    const int rx = mv ? bs.qx : bs.px, ry = mv ? bs.qy : bs.py, rz = mv ? bs.qz : bs.pz;
    const int R = 1 << rl;
    const int rep = lane & (R - 1);
    const uint32_t shift = (uint32_t)rl + 3;
    const uint32_t trash = (uint32_t)(trash_base + rep) << 3;
    const uint32_t repoff = (uint32_t)rep << 3;
    // Voxels per replica between flushes: without leaving voxels every field is
    // non-negative and 1023 * 2s < 2^16; with them, move_budget(s).
    const int per_rep = mv ? uniform(move_per_rep) : 1023;
    const int limit = (per_rep << rl) >> 6;
    char* hb = reinterpret_cast<char*>(hist);
    auto flush = [&]() {
        __syncthreads();
        if (mv) ms_flush<M, true>(hist, rl, B, lane, acc);
        else ms_flush<M, false>(hist, rl, B, lane, acc);
        __syncthreads();
    };
    int used = 0;
    unsigned long long ops = 0;   // LDS atomic operations of all lanes (uniform)
    const int nb = box_count(bs);
    // Lane i < nb works out box i of the set and its tiling, all boxes at once in
    // vector registers; the loop reads box i's figures from lane i.  (Box by box
    // in scalar registers, the geometry of a small box cost more scalar
    // instructions than its sweep.)
    const int bi = lane < nb ? lane : 0;
    int bsg;
    const Box b = box_at(v, bs, bi, bsg);
    bool has = lane < nb && b.xa <= b.xb && b.ya <= b.yb && b.za <= b.zb;
    if (mv) {
        // a move box lies outside the other window along axis i % 3: none if the
        // move has no component along it
        const int a = bi >= 3 ? bi - 3 : bi;
        has = has && (a == 0 ? bs.qx - bs.px : a == 1 ? bs.qy - bs.py : bs.qz - bs.pz) != 0;
    }
    // sweep along y (the y-fast copy) when x is strided or the box is thinner in
    // x than in y; the fast axis is never strided.  Axes (fast, row, slice):
    // (x, y, z), or (y, z, x) on the y-fast copy.
    const bool btr = b.xs != 1 || (b.ys == 1 && b.xb - b.xa < b.yb - b.ya);
    const int bfa = btr ? b.ya : b.xa, bfb = btr ? b.yb : b.xb;
    const int bra = btr ? b.za : b.ya, brs = btr ? b.zs : b.ys;
    const int bsa = btr ? b.xa : b.za, bss = btr ? b.xs : b.zs;
    const int bnr = small_div((btr ? b.zb : b.yb) - bra, brs) + 1;
    const int bns = small_div((btr ? b.xb : b.zb) - bsa, bss) + 1;
    // the tile of make_sweep<64>: as many rows as 64 lanes hold, then slices
    const int bnd = (bfb >> 2) - (bfa >> 2) + 1;
    const int brmax = small_div(64, bnd);
    const int bty = min(bnr, brmax);
    const int btz = min(bns, small_div(brmax, bty));
    // signs and strides (a stride is 1 or 2s) in one word: fewer reads per box
    const int bflags = (btr ? 1 : 0) | (bsg < 0 ? 2 : 0) | (brs << 2) | (bss << 10);
    const Layout Lx = layout_x(v), Lt = layout_t(v);
    unsigned long long todo = __ballot(has);
#pragma unroll 1
    while (todo) {
        const int i = __builtin_ctzll(todo);
        todo &= todo - 1;
        auto pick = [i](int x) { return __builtin_amdgcn_readlane(x, i); };
        const int flags = pick(bflags);
        const bool tr = (flags & 1) != 0;
        const int sg = (flags & 2) ? -1 : 1;
        const int rst = (flags >> 2) & 0xFF, sst = flags >> 10;
        const int fa = pick(bfa), fb = pick(bfb), ra = pick(bra), sa = pick(bsa);
        const Layout L = tr ? Lt : Lx;
        Sweep w;
        w.ny = pick(bnr);
        w.nz = pick(bns);
        w.nd = pick(bnd);
        w.ty = pick(bty);
        w.tz = pick(btz);
        w.pr = L.pitch * (uint32_t)rst;
        w.ps = L.slab * (uint32_t)sst;
        sweep_lane<4>(L, w, fa >> 2, ra, sa, lane);
        // axes (fast, row, slice) -> packed fields: x at bit 10, y at 32, z at 48
        const int fr = tr ? ry : rx, rr = tr ? rz : ry, sr = tr ? rx : rz;
        const int shf = tr ? 32 : 10, shr = tr ? 48 : 32, shs = tr ? 10 : 48;
        // the box's sign applied to a packed value (two's complement: -x = ~x + 1)
        const unsigned long long neg = sg < 0 ? ~0ull : 0ull;
        auto signed_ = [neg](unsigned long long x) { return (x ^ neg) - neg; };
        // the lane's first voxel: a count of 1 and its offsets d + s from the
        // reference point along the fast, row and slice axes (negative offsets
        // wrap, as their sums do)
        auto field = [](int d, int sh) { return (unsigned long long)(long long)d << sh; };
        const unsigned long long cp0 =
            signed_(1ull + field(w.x0 - fr + s, shf) + field(ra + w.oy * rst - rr + s, shr) +
                    field(sa + w.oz * sst - sr + s, shs));
        const unsigned long long cdf = signed_(1ull << shf);
        unsigned long long cp[4];
        uint32_t off[4], wid[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int f = w.x0 + k;
            const bool ok = f >= fa && f <= fb;
            cp[k] = k == 0 ? cp0 : cp[k - 1] + cdf;
            off[k] = ok ? repoff : trash;
            wid[k] = ok ? 8u : 0u;
        }
        const unsigned long long smr = signed_(field(rst, shr));
        const unsigned long long sms = signed_(field(sst, shs));
        // every (row, dword) of the box is scattered once, four adds each
        ops += 4ull * (unsigned)(w.nd * w.ny * w.nz);
        auto scatter = [&](uint32_t word, int, int, uint64_t step) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t bin = __builtin_amdgcn_ubfe(word, 8 * k, wid[k]);
                atomicAdd(reinterpret_cast<unsigned long long*>(hb + (bin << shift) + off[k]), cp[k] + step);
            }
        };
        // a move box one voxel thick (the usual case) is a line of tiles
        if (w.ty >= w.ny || w.nz == 1)
            run_sweep_line<kMsLineUnroll, kMsDepth>(L, w, smr, sms, used, limit, scatter, flush);
        else
            run_sweep<kMsUnroll, kMsDepth>(L, w, smr, sms, used, limit, scatter, flush);
    }
    if (used > 0) flush();
    return ops;
}

struct EvalOut {
    double obj, dx, dy, dz;
};

// N of a window under a window level: the voxels counted in bins 0..B-1.
template <int M>
__device__ __forceinline__ int64_t window_total(const int* c) {
    long long n = 0;
#pragma unroll
    for (int t = 0; t < M; ++t) n += c[t];
    return (int64_t)bfly_sumll(n);
}

// Eq. 4-6 with a flat kernel and the uniform target: move = (sum_b M_b/sqrt(c_b)) /
// (sum_b sqrt(c_b)), objective rho~ = (sum_b sqrt(c_b)) / sqrt(N), from the
// window totals (f = sums of d + s).  sqrt and 1/sqrt of the integer counts are
// computed here rather than loaded: the device's double sqrt and division are
// correctly rounded, as the host's are, so the values equal the host-built
// tables bit for bit (the mean-shift traces compare the objective with ==).
// sqrt(c) and 1/sqrt(c) of a count c >= 0 (1/sqrt(0) taken as 0): IEEE double
// square root and division, both correctly rounded.
__device__ __forceinline__ void count_roots(int c, double& sq, double& rs) {
    const double sc = sqrt((double)c);
    sq = sc;
    rs = c > 0 ? 1.0 / sc : 0.0;
}

template <int M>
__device__ EvalOut ms_moments(const VolDesc& v, const Tables& tb, int px, int py, int pz, int s, const BinAcc<M>& a) {
    double sq[M], tx[M], ty[M], tz[M];
#pragma unroll
    for (int t = 0; t < M; ++t) {
        const bool nz = a.c[t] > 0;
        double sc, rs;
        count_roots(a.c[t], sc, rs);
        sq[t] = nz ? sc : 0.0;
        tx[t] = nz ? (double)(a.f1[t] - a.c[t] * s) * rs : 0.0;
        ty[t] = nz ? (double)(a.f2[t] - a.c[t] * s) * rs : 0.0;
        tz[t] = nz ? (double)(a.f3[t] - a.c[t] * s) * rs : 0.0;
    }
    const double D = bfly_sum(local_pw<M>(sq));
    const double nx = bfly_sum(local_pw<M>(tx));
    const double ny = bfly_sum(local_pw<M>(ty));
    const double nzs = bfly_sum(local_pw<M>(tz));
    const int64_t N = v.win ? window_total<M>(a.c) : cube_count(v, px, py, pz, s);
    EvalOut e;
    e.obj = N > 0 ? D / sqrt((double)N) : 0.0;
    e.dx = D > 0.0 ? nx / D : 0.0;
    e.dy = D > 0.0 ? ny / D : 0.0;
    e.dz = D > 0.0 ? nzs / D : 0.0;
    return e;
}

struct Saliency {
    int scale, keep;
    double y64, w64;
    float h32, w32, y32;
};

__device__ __forceinline__ float entropy_term32(int c, int64_t N) {
    if (c <= 0) return 0.0f;
    const float p = (float)c / (float)N;
    const float lp = (2 * (int64_t)c > N) ? log1pf(-(float)(N - c) / (float)N) : logf(p);
    return -p * lp;
}

// Kadir-Brady saliency at the trajectory's own scale (mean-shift) from the
// counts of the window (cs) and of its inner cube of half-width s-1 (cin).
template <int M>
__device__ Saliency ms_saliency(const VolDesc& v, const Tables& tb, int px, int py, int pz, int s, const int* cs,
                                const int* cin) {
    const int64_t Ns = v.win ? window_total<M>(cs) : cube_count(v, px, py, pz, s);
    const int64_t Np = v.win ? window_total<M>(cin) : cube_count(v, px, py, pz, s - 1);
    double cl[M];
    long long am = 0;
    float h = 0.0f;
#pragma unroll
    for (int t = 0; t < M; ++t) {
        cl[t] = tb.cl[cs[t]];
        long long d = (long long)cs[t] * Np - (long long)cin[t] * Ns;
        am += d < 0 ? -d : d;
        h += entropy_term32(cs[t], Ns);
    }
    const double S = bfly_sum(local_pw<M>(cl));
    const long long A = bfly_sumll(am);
    const float H32 = bfly_sumf(h);
    // with a window level a window may count no voxel: H = 0, W = 0
    const double H64 = Ns > 0 ? (tb.cl[Ns] - S) / (double)Ns : 0.0;
    const bool wok = Ns > 0 && Np > 0;
    const double W64 = wok ? ((double)(s * s) / (double)(2 * s - 1)) * ((double)A / ((double)Ns * (double)Np)) : 0.0;
    Saliency r;
    r.scale = s;
    r.y64 = H64 * W64;
    r.w64 = W64;
    r.keep = (H64 > v.h_min && r.y64 > v.y_min) ? 1 : 0;
    r.h32 = H32;
    r.w32 = wok ? ((float)(s * s) / (float)(2 * s - 1)) * ((float)A / ((float)Ns * (float)Np)) : 0.0f;
    r.y32 = r.h32 * r.w32;
    return r;
}

// ----------------------------------------------------- task decoding, loop

__device__ __forceinline__ int find_seg(const TaskSeg* __restrict__ segs, int nseg, long long t) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (segs[mid].task_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

struct LocalCounts {
    unsigned long long evals, window_evals, voxel_visits, final_visits, swept;
    unsigned int lds_ops;   // this lane's LDS atomic operations
};

// The search loop shared by both methods: round the proposed move, stop if it is
// zero, if clamping leaves P unchanged, if the objective does not strictly
// increase, or after max_iter accepted moves.  Every lane holds the same values;
// positions and the stop decision are made scalar with readfirstlane.
struct TrajOut {
    int p[3];
    int iters, stop;
    double obj;
};

template <typename Eval>
__device__ __forceinline__ TrajOut run_trajectory(const VolDesc& v, const int* p0, Eval&& eval, LocalCounts& lc,
                                                  int visit_r, int win_evals) {
    TrajOut o;
    o.p[0] = p0[0]; o.p[1] = p0[1]; o.p[2] = p0[2];
    EvalOut cur = eval(o.p[0], o.p[1], o.p[2]);
    lc.evals += 1;
    lc.window_evals += (unsigned long long)win_evals;
    lc.voxel_visits += cube_count(v, o.p[0], o.p[1], o.p[2], visit_r);
    int it = 0, stop;
    for (;;) {
        if (it == v.max_iter) { stop = 0; break; }
        const int mx = uniform((int)round(cur.dx));
        const int my = uniform((int)round(cur.dy));
        const int mz = uniform((int)round(cur.dz));
        if (mx == 0 && my == 0 && mz == 0) { stop = 1; break; }
        const int qx = clampi(o.p[0] + mx, 0, v.X - 1);
        const int qy = clampi(o.p[1] + my, 0, v.Y - 1);
        const int qz = clampi(o.p[2] + mz, 0, v.Z - 1);
        if (qx == o.p[0] && qy == o.p[1] && qz == o.p[2]) { stop = 2; break; }
        const EvalOut nxt = eval(qx, qy, qz);
        lc.evals += 1;
        lc.window_evals += (unsigned long long)win_evals;
        lc.voxel_visits += cube_count(v, qx, qy, qz, visit_r);
        if (!uniform(nxt.obj > cur.obj ? 1 : 0)) { stop = 3; break; }
        o.p[0] = qx; o.p[1] = qy; o.p[2] = qz;
        cur = nxt;
        it += 1;
    }
    o.iters = it;
    o.stop = stop;
    o.obj = cur.obj;
    return o;
}

__device__ __forceinline__ void write_rec(TrajRec* dst, const int* p0, const TrajOut& o, const Saliency& sal,
                                          int32_t id, int rank_by) {
    TrajRec r;
    r.x0 = p0[0]; r.y0 = p0[1]; r.z0 = p0[2];
    r.x = o.p[0]; r.y = o.p[1]; r.z = o.p[2];
    r.scale = sal.scale; r.iters = o.iters; r.stop = o.stop; r.keep = sal.keep;
    r.objective = o.obj; r.y64 = sal.y64;
    r.key64 = rank_by == 1 ? sal.w64 : sal.y64;
    r.h32 = sal.h32; r.w32 = sal.w32; r.y32 = sal.y32;
    r.seed = id;
    *dst = r;
}

// ------------------------------------------------------- mean-shift kernel

// Per trajectory: the window totals follow the trajectory (one sweep per
// evaluation: the whole window first, later the difference regions when they
// are the smaller sweep), and the final pass reuses the counts of the window at
// P*.  Every sweep of the kernel goes through the one ms_sweep call below, so
// the scatter code is instantiated once per tile walk (line and general).
// Up to 64 bins (one per lane) the kernel is held to 128 VGPRs: four waves per SIMD.
template <int M, bool GROUPED>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(M == 1 ? 4 : 1))) void k_search_ms(const VolDesc* __restrict__ vols,
                                                  const TaskSeg* __restrict__ segs, int nseg,
                                                  const XcdQueues* __restrict__ xq, int chunk, Tables tb,
                                                  TrajRec* out,
                                                  Counters* cnt, MsTune tune, int hist_words) {
    extern __shared__ unsigned long long hist[];
    const int lane = threadIdx.x;
    for (int i = lane; i < hist_words; i += 64) hist[i] = 0ull;
    __syncthreads();
    LocalCounts lc = {0, 0, 0, 0, 0, 0u};
    unsigned long long ms_ops = 0;   // LDS atomic operations of the wave's lanes
    const int trash_base = hist_words - 64;
    // A window level's sentinel bin B is scattered into but never read or
    // cleared; its words, at B << rl, hold counts until the replica layout
    // changes, where they would be read as bins below B: cleared then.
    int dirty = -1, dirty_len = 0;
    // The wave's XCD queue first (its tasks cover one part of each volume, so
    // the XCD's L2 holds their windows), then the other XCDs' queues in turn.
    const int xcd = (int)(blockIdx.x & (kXcds - 1));
    unsigned int drained = 0;   // lane 0: queues found empty
    for (;;) {
        long long t = -1;
        if (lane == 0) {
            for (int k = 0; k < kXcds && t < 0; ++k) {
                const int q = (xcd + k) & (kXcds - 1);
                if (drained & (1u << q)) continue;
                const long long i = (long long)atomicAdd(&cnt->xq_head[chunk][q], 1ull);
                const long long b = xq->begin[q];
                if (b + i < xq->end[q]) t = b + i;
                else drained |= 1u << q;
            }
        }
        t = __shfl(t, 0, 64);
        if (t < 0) break;
        const int si = uniform(find_seg(segs, nseg, t));
        const TaskSeg sg = segs[si];
        const VolDesc& v = vols[sg.vol];
        const long long seed = seg_seed(v, sg, t - sg.task_begin);
        int p0[3];
        seed_pos(v, seed, p0);
        // The group's scales in ascending order: the first window of scale s is
        // the first window of s - 1 (kept in `first`) plus the shell at distance s.
        BinAcc<M> first;
        acc_clear<M>(first);
        const int s_last = GROUPED ? uniform(sg.scale_hi) : uniform(sg.scale);
        for (int s = uniform(sg.scale); s <= s_last; ++s) {
        // replicas per wavefront by window size class
        const int rl = s <= tune.s_small ? tune.rl_small : tune.rl;
        const int move_per_rep = move_budget(s);
        const int sentinel = v.win ? (v.B << rl) : -1;
        if (dirty >= 0 && (dirty != sentinel || dirty_len != (1 << rl))) {
            for (int i = lane; i < dirty_len; i += 64) hist[dirty + i] = 0ull;
            __syncthreads();
        }
        dirty = sentinel;
        dirty_len = 1 << rl;
        // Search state (Sec. 2.3): accepted position P, window of the totals W,
        // candidate Q; phase 0 evaluates P0, 1 a candidate, 2 the final pass.
        int px = p0[0], py = p0[1], pz = p0[2];
        int wx = px, wy = py, wz = pz;
        int qx = px, qy = py, qz = pz;
        int phase = 0, it = 0, stop = 0;
        EvalOut cur = {0.0, 0.0, 0.0, 0.0};
        BinAcc<M> a;
        acc_clear<M>(a);
        int cprev[M], cs[M];
#pragma unroll
        for (int k = 0; k < M; ++k) cprev[k] = cs[k] = 0;
        bool use_shell = false;
        for (;;) {
            BoxSet bs = {kFull, px, py, pz, 0, 0, 0, s};
            if (phase == 1) {
                const int64_t nq = cube_count(v, qx, qy, qz, s);
                const BoxSet mv = {kMove, wx, wy, wz, qx, qy, qz, s};
                const int64_t nd = move_volume(v, wx, wy, wz, qx, qy, qz, s);
#pragma unroll
                for (int k = 0; k < M; ++k) cprev[k] = a.c[k];
                if (100 * nd < (int64_t)tune.incr_pct * nq) {
                    const int dx = qx - wx, dy = qy - wy, dz = qz - wz;
#pragma unroll
                    for (int k = 0; k < M; ++k) {
                        a.f1[k] -= a.c[k] * dx;
                        a.f2[k] -= a.c[k] * dy;
                        a.f3[k] -= a.c[k] * dz;
                    }
                    bs = mv;
                    lc.swept += (unsigned long long)nd;
                } else {
                    acc_clear<M>(a);
                    bs = BoxSet{kFull, qx, qy, qz, 0, 0, 0, s};
                    lc.swept += (unsigned long long)nq;
                }
                wx = qx; wy = qy; wz = qz;
            } else if (phase == 2) {
                const bool here = wx == px && wy == py && wz == pz;
#pragma unroll
                for (int k = 0; k < M; ++k) cs[k] = here ? a.c[k] : cprev[k];
                const int64_t Ns = cube_count(v, px, py, pz, s), Np = cube_count(v, px, py, pz, s - 1);
                use_shell = Ns - Np < Np;
                acc_clear<M>(a);
                bs = BoxSet{use_shell ? kShell : kInner, px, py, pz, 0, 0, 0, s};
                lc.swept += (unsigned long long)(use_shell ? Ns - Np : Np);
            } else if (GROUPED && s > sg.scale) {
                // shift the kept offset sums from d + (s-1) to d + s, then add the shell
                a = first;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    a.f1[k] += a.c[k];
                    a.f2[k] += a.c[k];
                    a.f3[k] += a.c[k];
                }
                bs = BoxSet{kShell, px, py, pz, 0, 0, 0, s};
                lc.swept += (unsigned long long)(cube_count(v, px, py, pz, s) - cube_count(v, px, py, pz, s - 1));
            } else {
                lc.swept += (unsigned long long)cube_count(v, px, py, pz, s);
            }
            ms_ops += ms_sweep<M>(v, bs, rl, trash_base, move_per_rep, hist, lane, a);
            if (phase == 2) break;
            if (GROUPED && phase == 0) first = a;
            // an evaluation at W (= P0 in phase 0, Q in phase 1)
            const EvalOut e = ms_moments<M>(v, tb, wx, wy, wz, s, a);
            lc.evals += 1;
            lc.window_evals += 1;
            lc.voxel_visits += cube_count(v, wx, wy, wz, s);
            if (phase == 1) {
                if (!uniform(e.obj > cur.obj ? 1 : 0)) {
                    stop = 3;
                    phase = 2;
                    continue;
                }
                px = qx; py = qy; pz = qz;
                it += 1;
            }
            cur = e;
            // the next move from P: stop on max_iter, a zero move or a clamped one
            phase = 2;
            if (it == v.max_iter) { stop = 0; continue; }
            const int mx = uniform((int)round(cur.dx));
            const int my = uniform((int)round(cur.dy));
            const int mz = uniform((int)round(cur.dz));
            if (mx == 0 && my == 0 && mz == 0) { stop = 1; continue; }
            qx = clampi(px + mx, 0, v.X - 1);
            qy = clampi(py + my, 0, v.Y - 1);
            qz = clampi(pz + mz, 0, v.Z - 1);
            if (qx == px && qy == py && qz == pz) { stop = 2; continue; }
            phase = 1;
        }
        int cin[M];
#pragma unroll
        for (int k = 0; k < M; ++k) cin[k] = use_shell ? cs[k] - a.c[k] : a.c[k];
        const Saliency sal = ms_saliency<M>(v, tb, px, py, pz, s, cs, cin);
        lc.final_visits += cube_count(v, px, py, pz, s);
        lc.window_evals += 2;
        if (lane == 0) {
            TrajOut o;
            o.p[0] = px; o.p[1] = py; o.p[2] = pz;
            o.iters = it; o.stop = stop; o.obj = cur.obj;
            const long long local = seed * v.S + (s - v.s_min);
            write_rec(out + v.traj_base + local, p0, o, sal, (int32_t)local, v.rank_by);
        }
        }
    }
    if (lane == 0) {
        atomicAdd(&cnt->evals, lc.evals);
        atomicAdd(&cnt->window_evals, lc.window_evals);
        atomicAdd(&cnt->voxel_visits, lc.voxel_visits);
        atomicAdd(&cnt->final_visits, lc.final_visits);
        atomicAdd(&cnt->swept, lc.swept);
    }
    if (lane == 0) atomicAdd(&cnt->lds_ops, ms_ops);
}

// ------------------------------------------------ quadrant: bucketed scatter

// Scatter the box into hist (uint32 counters) at byte offset
//   region + ((row*B + bin) << rq)*4 + replica*4,
// row = max(max(|x-cx|,|y-cy|,|z-cz|) - base, 0); bytes outside the box go to
// row trash_row.
template <int NT>
__device__ __forceinline__ unsigned int bucket_scatter(const VolDesc& v, int xa, int xb, int ya, int yb, int za, int zb,
                                                       int cx, int cy, int cz, int base, int trash_row, int rq,
                                                       uint32_t region, uint32_t* hist, int tid) {
    constexpr int WB = kQuadWB;  // voxels per lane and step
    const Layout L = layout_x(v);
    const Sweep w = make_sweep<NT, WB>(L, xa, xb, ya, yb - ya + 1, 1, za, zb - za + 1, 1, tid);
    const uint32_t rowbytes = (uint32_t)row_stride(v.B) << (rq + 2);
    const uint32_t rep4 = ((uint32_t)(tid & ((1 << rq) - 1)) << 2) + region;
    const uint32_t bshift = (uint32_t)rq + 2;
    uint32_t rx[WB];
#pragma unroll
    for (int k = 0; k < WB; ++k) {
        const int x = w.x0 + k;
        const bool ok = x >= xa && x <= xb;
        const int r = ok ? max(abs(x - cx) - base, 0) : trash_row;
        rx[k] = (uint32_t)r * rowbytes + rep4;
    }
    const int dy0 = ya + w.oy - cy, dz0 = za + w.oz - cz;
    int used = 0;
    unsigned int ops = 0;
    run_sweep<kQuadUnroll, kQuadDepth, WB>(
        L, w, 0, 0, used, INT_MAX,
        [&](typename LaneWord<WB>::T word, int iy0, int iz0, uint64_t) {
            const uint32_t lo = (uint32_t)word, hi = (uint32_t)((uint64_t)word >> 32);
            const int rr = max(max(abs(dy0 + iy0), abs(dz0 + iz0)) - base, 0);
            const uint32_t RR = (uint32_t)rr * rowbytes + rep4;
#pragma unroll
            for (int k = 0; k < WB; ++k) {
                const uint32_t b = __builtin_amdgcn_ubfe(k < 4 ? lo : hi, 8 * (k & 3), 8);
                const uint32_t addr = max(rx[k], RR) + (b << bshift);
                atomicAdd(reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(hist) + addr), 1u);
            }
            ops += WB;
        },
        []() {});
    return ops;
}

// One sweep over the brick P + [-R, R]^3 (clipped) for all 8 octants: a voxel
// at offset d goes to octant j (bit a set when d_a > 0), and to the mirrored
// octants along every axis with d_a = 0 (the planes through P belong to both
// sides); row = max(max|d_a| - base, 0), octant j's region at byte
// j * region_bytes.  Per voxel: one bit-field extract, one max, two adds and one
// LDS add; the x-plane voxel of a lane costs one more add per step, and the rare
// rows on the y or z plane take a separate path.
template <int NT>
__device__ __forceinline__ unsigned int octant_scatter(const VolDesc& v, int px, int py, int pz, int Rr, int base,
                                                       int trash_row, int rq, uint32_t region_bytes, uint32_t* hist,
                                                       int tid) {
    constexpr int WB = kQuadWB;  // voxels per lane and step
    const int xa = max(px - Rr, 0), xb = min(px + Rr, v.X - 1);
    const int ya = max(py - Rr, 0), yb = min(py + Rr, v.Y - 1);
    const int za = max(pz - Rr, 0), zb = min(pz + Rr, v.Z - 1);
    const Layout L = layout_x(v);
    const Sweep w = make_sweep<NT, WB>(L, xa, xb, ya, yb - ya + 1, 1, za, zb - za + 1, 1, tid);
    const uint32_t rowbytes = (uint32_t)row_stride(v.B) << (rq + 2);
    const uint32_t rep4 = (uint32_t)(tid & ((1 << rq) - 1)) << 2;
    const uint32_t bshift = (uint32_t)rq + 2;
    uint32_t rx[WB], ax[WB];
    int kx = -1;
#pragma unroll
    for (int k = 0; k < WB; ++k) {
        const int x = w.x0 + k;
        const bool ok = x >= xa && x <= xb;
        const int r = ok ? max(abs(x - px) - base, 0) : trash_row;
        rx[k] = __umul24((uint32_t)r, rowbytes) + rep4;
        ax[k] = x > px ? region_bytes : 0u;
        if (ok && x == px) kx = k;
    }
    // the lane's voxel on the plane x = px (if any): byte kx, mirrored to the + side
    const bool xdup = kx >= 0;
    const bool kxhi = kx >= 4;
    const uint32_t kxs = xdup ? 8u * (uint32_t)(kx & 3) : 0u;
    const uint32_t rxd = rep4;  // |x - px| = 0: row max(-base, 0) = 0
    const int dy0 = ya + w.oy - py, dz0 = za + w.oz - pz;
    const uint32_t ry2 = 2u * region_bytes, rz4 = 4u * region_bytes;
    char* hb = reinterpret_cast<char*>(hist);
    int used = 0;
    unsigned int ops = 0;
    run_sweep<kQuadUnroll, kQuadDepth, WB>(
        L, w, 0, 0, used, INT_MAX,
        [&](typename LaneWord<WB>::T word, int iy0, int iz0, uint64_t) {
            const uint32_t lo = (uint32_t)word, hi = (uint32_t)((uint64_t)word >> 32);
            const int dy = dy0 + iy0, dz = dz0 + iz0;
            const uint32_t RR = __umul24((uint32_t)max(max(abs(dy), abs(dz)) - base, 0), rowbytes) + rep4;
            const uint32_t ayz = (dy > 0 ? ry2 : 0u) + (dz > 0 ? rz4 : 0u);
#pragma unroll
            for (int k = 0; k < WB; ++k) {
                const uint32_t b = __builtin_amdgcn_ubfe(k < 4 ? lo : hi, 8 * (k & 3), 8);
                atomicAdd(reinterpret_cast<uint32_t*>(hb + (max(rx[k], RR) + (b << bshift) + ax[k] + ayz)), 1u);
            }
            if (xdup) {
                const uint32_t b = __builtin_amdgcn_ubfe(kxhi ? hi : lo, kxs, 8);
                atomicAdd(reinterpret_cast<uint32_t*>(hb + (max(rxd, RR) + (b << bshift) + region_bytes + ayz)), 1u);
            }
            if (dy == 0 || dz == 0) {
                // rows on the y or z plane: the mirrored copies
                const uint32_t ym = dy == 0 ? ry2 : 0u, zm = dz == 0 ? rz4 : 0u;
                auto mirror = [&](uint32_t b, uint32_t rk, uint32_t xk) {
                    const uint32_t ak = max(rk, RR) + (b << bshift) + xk + ayz;
                    if (ym) atomicAdd(reinterpret_cast<uint32_t*>(hb + ak + ym), 1u);
                    if (zm) atomicAdd(reinterpret_cast<uint32_t*>(hb + ak + zm), 1u);
                    if (ym && zm) atomicAdd(reinterpret_cast<uint32_t*>(hb + ak + ym + zm), 1u);
                };
#pragma unroll
                for (int k = 0; k < WB; ++k) mirror(__builtin_amdgcn_ubfe(k < 4 ? lo : hi, 8 * (k & 3), 8), rx[k], ax[k]);
                if (xdup) mirror(__builtin_amdgcn_ubfe(kxhi ? hi : lo, kxs, 8), rxd, region_bytes);
                ops += (xdup ? WB + 1u : (unsigned)WB) * ((ym ? 1u : 0u) + (zm ? 1u : 0u) + (ym && zm ? 1u : 0u));
            }
            ops += xdup ? WB + 1u : (unsigned)WB;
        },
        []() {});
    return ops;
}

// Sum the replicas of every (region, bin) and prefix over rows 0..nrows-1, in
// place: replica 0 of row r then holds the voxels of bin b in rows 0..r; other
// replicas and the trash row are cleared.  Rows go kMergeRows at a time: their
// loads are issued together, then the prefix and the stores.
constexpr int kMergeRows = 8;

template <int NT>
__device__ __forceinline__ void bucket_merge(uint32_t* hist, int nreg, int nrows, int B, int rq, int tid) {
    const int R = 1 << rq;
    const int rows_total = nrows + 1;
    const int Bs = row_stride(B);
    for (int p = tid; p < nreg * B; p += NT) {
        const int g = p / B, b = p - g * B;
        const int e0 = (g * rows_total * Bs + b) << rq, de = Bs << rq;
        uint32_t acc = 0;
        for (int r0 = 0; r0 <= nrows; r0 += kMergeRows) {
            uint32_t c[kMergeRows];
#pragma unroll
            for (int i = 0; i < kMergeRows; ++i) {
                const int e = e0 + (r0 + i) * de;
                c[i] = 0;
                if (r0 + i <= nrows) {
                    c[i] = hist[e];
                    for (int q = 1; q < R; ++q) c[i] += hist[e + q];
                }
            }
#pragma unroll
            for (int i = 0; i < kMergeRows; ++i) {
                const int r = r0 + i, e = e0 + r * de;
                if (r > nrows) break;
                for (int q = 1; q < R; ++q) hist[e + q] = 0u;
                acc += c[i];
                hist[e] = r < nrows ? acc : 0u;
            }
        }
    }
}

__device__ __forceinline__ uint32_t merged(const uint32_t* hist, int g, int rows_total, int r, int B, int b, int rq) {
    return hist[((g * rows_total + r) * row_stride(B) + b) << rq];
}

struct QuadLds {
    uint32_t* hist;
    double* eps;     // [8][S]
    double* hrow;    // [S+2]
    long long* arow; // [S+2]
    long long* nrow; // [S+2] counted voxels of each centred cube
    float* h32row;   // [S+2]
    double* res;     // [4]
};

__device__ __forceinline__ QuadLds quad_lds(char* smem, const LdsQuad& L) {
    QuadLds q;
    q.hist = reinterpret_cast<uint32_t*>(smem + L.hist_off);
    q.eps = reinterpret_cast<double*>(smem + L.eps_off);
    q.hrow = reinterpret_cast<double*>(smem + L.hrow_off);
    q.arow = reinterpret_cast<long long*>(smem + L.arow_off);
    q.nrow = reinterpret_cast<long long*>(smem + L.nrow_off);
    q.h32row = reinterpret_cast<float*>(smem + L.h32_off);
    q.res = reinterpret_cast<double*>(smem + L.res_off);
    return q;
}

// Entropy H64 = (cl[N] - sum_b cl[c_b]) / N of merged rows; wave w takes rows
// w, w + NW, ..., kRowBatch at a time so that their table loads are in flight
// together; N of a row from nrow(g, r), or (win) the row's counted voxels, and
// H = 0 for a row that counts none.  Lane i of the wave finishes row i of the
// batch (its cl[N] load, issued with the bins' loads when N is known up front,
// and the division), so the batch's tails run side by side.  The replica-0
// counters read here are cleared.
constexpr int kRowBatch = 8;

template <int NT, int M, typename NF>
__device__ __forceinline__ void rows_entropy(uint32_t* hist, int nreg, int nrows, int B, int rq, const Tables& tb,
                                             NF&& nrow, bool win, double* out, int tid) {
    const int wave = tid >> 6, lane = tid & 63;
    const int rows_total = nrows + 1;
    const int nq = nreg * nrows;
    for (int q0 = wave; q0 < nq; q0 += kRowBatch * (NT / 64)) {
        // the row this lane finishes (lanes 0 .. kRowBatch-1)
        const int qm = q0 + lane * (NT / 64);
        const bool mine = lane < kRowBatch && qm < nq;
        int64_t Nm = 0;
        double clN = 0.0;
        if (!win && mine) {
            const int g = qm / nrows, r = qm - g * nrows;
            Nm = nrow(g, r);
            clN = tb.cl[Nm];
        }
        double v[kRowBatch][M];
        int cn[kRowBatch];
#pragma unroll
        for (int i = 0; i < kRowBatch; ++i) {
            const int q = q0 + i * (NT / 64);
            const int g = q / nrows, r = q - g * nrows;
            cn[i] = 0;
#pragma unroll
            for (int t = 0; t < M; ++t) {
                const int b = lane * M + t;
                uint32_t c = 0;
                if (q < nq && b < B) {
                    const int e = ((g * rows_total + r) * row_stride(B) + b) << rq;
                    c = hist[e];
                    hist[e] = 0u;
                }
                v[i][t] = tb.cl[c];
                cn[i] += (int)c;
            }
        }
        double Sm = 0.0;
        long long wm = 0;
#pragma unroll
        for (int i = 0; i < kRowBatch; ++i) {
            const double S = bfly_sum(local_pw<M>(v[i]));
            Sm = lane == i ? S : Sm;
            if (win) {
                const long long wn = bfly_sumll((long long)cn[i]);
                wm = lane == i ? wn : wm;
            }
        }
        if (win && mine) {
            Nm = (int64_t)wm;
            clN = tb.cl[Nm];
        }
        if (mine) out[qm] = Nm > 0 ? (clN - Sm) / (double)Nm : 0.0;
    }
}

// Merge and entropy in one pass for the octant regions: wave w takes regions
// w, w + NW, ...; a lane keeps the running sum over rows of its bins' counts
// (replicas summed), so row r's counts (the cube of half-width s_min + r) never
// go back to LDS; RB rows at a time, their table loads in flight together, and
// lane i finishes row i of the batch as in rows_entropy.  Every counter of the
// regions, trash rows included, is cleared.
template <int NT, int M, typename NF>
__device__ __forceinline__ void merge_entropy(uint32_t* hist, int nreg, int nrows, int B, int rq, const Tables& tb,
                                              NF&& nrow, bool win, double* out, int tid) {
    constexpr int RB = 8;
    const int wave = tid >> 6, lane = tid & 63;
    const int rows_total = nrows + 1, Bs = row_stride(B), R = 1 << rq;
    for (int g = wave; g < nreg; g += NT / 64) {
        uint32_t acc[M];
#pragma unroll
        for (int t = 0; t < M; ++t) acc[t] = 0u;
        const int gb = g * rows_total * Bs;
        for (int r0 = 0; r0 < nrows; r0 += RB) {
            const int rm = r0 + lane;
            const bool mine = lane < RB && rm < nrows;
            int64_t Nm = 0;
            double clN = 0.0;
            if (!win && mine) {
                Nm = nrow(g, rm);
                clN = tb.cl[Nm];
            }
            uint32_t c[RB][M];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    const int b = lane * M + t;
                    c[i][t] = 0u;
                    if (r0 + i < nrows && b < B) {
                        const int e = (gb + (r0 + i) * Bs + b) << rq;
                        c[i][t] = hist[e];
                        for (int q = 1; q < R; ++q) c[i][t] += hist[e + q];
                    }
                }
            }
            double v[RB][M];
            int cn[RB];
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                cn[i] = 0;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    const int b = lane * M + t;
                    const bool ok = r0 + i < nrows && b < B;
                    if (ok) {
                        const int e = (gb + (r0 + i) * Bs + b) << rq;
                        for (int q = 0; q < R; ++q) hist[e + q] = 0u;
                    }
                    acc[t] += c[i][t];
                    v[i][t] = tb.cl[ok ? acc[t] : 0u];
                    cn[i] += ok ? (int)acc[t] : 0;
                }
            }
            double Sm = 0.0;
            long long wm = 0;
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const double S = bfly_sum(local_pw<M>(v[i]));
                Sm = lane == i ? S : Sm;
                if (win) {
                    const long long wn = bfly_sumll((long long)cn[i]);
                    wm = lane == i ? wn : wm;
                }
            }
            if (win && mine) {
                Nm = (int64_t)wm;
                clN = tb.cl[Nm];
            }
            if (mine) out[g * nrows + rm] = Nm > 0 ? (clN - Sm) / (double)Nm : 0.0;
        }
        // the trash row
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int b = lane * M + t;
            if (b < B) {
                const int e = (gb + nrows * Bs + b) << rq;
                for (int q = 0; q < R; ++q) hist[e + q] = 0u;
            }
        }
    }
}

// Alg. 1 body in 3D: octant entropies for every scale, per octant the first
// maximising scale, E = sum of the 8 maxima, move = sum_j eps_j k*_j sigma_j / E.
template <int NT, int M>
__device__ __forceinline__ EvalOut quad_eval(const VolDesc& v, const Tables& tb, int px, int py, int pz, int rq, const QuadLds& L,
                             int tid, unsigned int& ops) {
    px = uniform(px); py = uniform(py); pz = uniform(pz);
    const int S = v.S, B = v.B;
    const uint32_t region_bytes = (uint32_t)(S + 1) * (uint32_t)row_stride(B) << (rq + 2);
    ops += octant_scatter<NT>(v, px, py, pz, v.s_max, v.s_min, S, rq, region_bytes, L.hist, tid);
    __syncthreads();
    merge_entropy<NT, M>(
        L.hist, 8, S, B, rq, tb,
        [&](int j, int r) {
            const int k = v.s_min + r;
            const int rx = (j & 1) ? v.X - 1 - px : px, ry = (j & 2) ? v.Y - 1 - py : py;
            const int rz = (j & 4) ? v.Z - 1 - pz : pz;
            return (int64_t)(min(k, rx) + 1) * (min(k, ry) + 1) * (min(k, rz) + 1);
        },
        v.win != 0, L.eps, tid);
    __syncthreads();
    if (tid < 64) {
        // lane j < 8 scans octant j over k (first maximum); lane 0 combines
        double best = 0.0;
        int ks = v.s_min;
        if (tid < 8) {
            best = L.eps[tid * S];
            for (int r = 1; r < S; ++r) {
                const double e = L.eps[tid * S + r];
                if (e > best) { best = e; ks = v.s_min + r; }
            }
        }
        double b8[8];
        int k8[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            b8[j] = __shfl(best, j, 64);
            k8[j] = __shfl(ks, j, 64);
        }
        if (tid == 0) {
            const double E = ((b8[0] + b8[1]) + (b8[2] + b8[3])) + ((b8[4] + b8[5]) + (b8[6] + b8[7]));
            double d[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double t[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) t[j] = b8[j] * (double)(k8[j] * (((j >> a) & 1) ? 1 : -1));
                const double num = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
                d[a] = E == 0.0 ? 0.0 : num / E;
            }
            L.res[0] = E; L.res[1] = d[0]; L.res[2] = d[1]; L.res[3] = d[2];
        }
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
template <int NT, int M>
__device__ __forceinline__ Saliency quad_saliency(const VolDesc& v, const Tables& tb, int px, int py, int pz, int rq,
                                  const QuadLds& L, int tid, unsigned int& ops) {
    px = uniform(px); py = uniform(py); pz = uniform(pz);
    const int S = v.S, B = v.B;
    const int nrows = S + 2;
    const int base = v.s_min - 1;
    const int wave = tid >> 6, lane = tid & 63;
    const int R = v.s_max + 1;
    ops += bucket_scatter<NT>(v, max(px - R, 0), min(px + R, v.X - 1), max(py - R, 0), min(py + R, v.Y - 1),
                       max(pz - R, 0), min(pz + R, v.Z - 1), px, py, pz, base, nrows, rq, 0u, L.hist, tid);
    __syncthreads();
    bucket_merge<NT>(L.hist, 1, nrows, B, rq, tid);
    __syncthreads();
    // N of every centred cube: its in-volume voxels, or with a window level the
    // voxels it counts
    for (int r = wave; r < nrows; r += NT / 64) {
        long long n = 0;
        if (v.win) {
#pragma unroll
            for (int t = 0; t < M; ++t) {
                const int b = lane * M + t;
                if (b < B) n += merged(L.hist, 0, nrows + 1, r, B, b, rq);
            }
            n = bfly_sumll(n);
        } else {
            n = cube_count(v, px, py, pz, base + r);
        }
        if (lane == 0) L.nrow[r] = n;
    }
    __syncthreads();
    // pdf change numerators and float entropies need the counts: read them before
    // rows_entropy clears them
    for (int r = wave; r < nrows; r += NT / 64) {
        const int64_t N = L.nrow[r];
        const int64_t Np = r > 0 ? L.nrow[r - 1] : 1;
        long long a = 0;
        float h = 0.0f;
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int b = lane * M + t;
            if (b < B) {
                const uint32_t c = merged(L.hist, 0, nrows + 1, r, B, b, rq);
                h += entropy_term32((int)c, N);
                if (r > 0) {
                    long long d = (long long)c * Np - (long long)merged(L.hist, 0, nrows + 1, r - 1, B, b, rq) * N;
                    a += d < 0 ? -d : d;
                }
            }
        }
        a = bfly_sumll(a);
        h = bfly_sumf(h);
        if (lane == 0) {
            L.arow[r] = a;
            L.h32row[r] = h;
        }
    }
    __syncthreads();
    rows_entropy<NT, M>(
        L.hist, 1, nrows, B, rq, tb, [&](int, int r) { return (int64_t)L.nrow[r]; }, false, L.hrow, tid);
    __syncthreads();
    if (tid == 0) {
        int best = -1;
        double bestY = 0.0;
        for (int s = v.s_min; s <= v.s_max; ++s) {
            const int r = s - base;
            if (!(L.hrow[r] > L.hrow[r - 1] && L.hrow[r] > L.hrow[r + 1])) continue;
            const int64_t N = L.nrow[r];
            const int64_t Np = L.nrow[r - 1];
            // a peak has H > 0, so N > 0; with a window level the smaller cube may count none
            const double W = Np > 0 ? ((double)(s * s) / (double)(2 * s - 1)) *
                                          ((double)L.arow[r] / ((double)N * (double)Np))
                                    : 0.0;
            const double Y = L.hrow[r] * W;
            if (best < 0 || Y > bestY) { best = s; bestY = Y; }
        }
        L.res[0] = (double)best;
        L.res[1] = bestY;
    }
    __syncthreads();
    Saliency out;
    const int best = uniform((int)L.res[0]);
    out.scale = best < 0 ? 0 : best;
    out.y64 = best < 0 ? 0.0 : L.res[1];
    out.w64 = 0.0;
    out.keep = 0;
    out.h32 = out.w32 = out.y32 = 0.0f;
    if (best >= 0) {
        const int r = best - base;
        const int64_t N = L.nrow[r];
        const int64_t Np = L.nrow[r - 1];
        const long long A = L.arow[r];
        const bool wok = N > 0 && Np > 0;
        out.w64 = wok ? ((double)(best * best) / (double)(2 * best - 1)) * ((double)A / ((double)N * (double)Np)) : 0.0;
        out.h32 = L.h32row[r];
        out.w32 = wok ? ((float)(best * best) / (float)(2 * best - 1)) * ((float)A / ((float)N * (float)Np)) : 0.0f;
        out.y32 = out.h32 * out.w32;
        out.keep = (L.hrow[r] > v.h_min && out.y64 > v.y_min) ? 1 : 0;
    }
    __syncthreads();
    return out;
}

// --------------------------------------------------------- quadrant kernel

constexpr int kQuadThreads = KS_QUAD_THREADS;  // threads per trajectory (one workgroup)

template <int M>
__global__ __launch_bounds__(kQuadThreads) void k_search_quad(const VolDesc* __restrict__ vols,
                                                             const TaskSeg* __restrict__ segs, int nseg,
                                                             long long ntask, Tables tb, TrajRec* out,
                                                             Counters* cnt, int rq, LdsQuad lay) {
    extern __shared__ __align__(16) char smem[];
    __shared__ long long s_task;
    const int tid = threadIdx.x;
    {
        uint32_t* h = reinterpret_cast<uint32_t*>(smem + lay.hist_off);
        for (int i = tid; i < lay.hist_words; i += kQuadThreads) h[i] = 0u;
    }
    const QuadLds L = quad_lds(smem, lay);
    __syncthreads();
    LocalCounts lc = {0, 0, 0, 0, 0, 0u};
    for (;;) {
        if (tid == 0) s_task = (long long)atomicAdd(&cnt->queue_head[0], 1ull);
        __syncthreads();
        const long long t = s_task;
        __syncthreads();
        if (t >= ntask) break;
        const int si = uniform(find_seg(segs, nseg, t));
        const TaskSeg sg = segs[si];
        const VolDesc& v = vols[sg.vol];
        const long long seed = seg_seed(v, sg, t - sg.task_begin);
        int p0[3];
        seed_pos(v, seed, p0);
        const TrajOut o = run_trajectory(
            v, p0, [&](int x, int y, int z) { return quad_eval<kQuadThreads, M>(v, tb, x, y, z, rq, L, tid, lc.lds_ops); }, lc, v.s_max,
            8 * v.S);
        const Saliency sal = quad_saliency<kQuadThreads, M>(v, tb, o.p[0], o.p[1], o.p[2], rq, L, tid, lc.lds_ops);
        lc.final_visits += cube_count(v, o.p[0], o.p[1], o.p[2], v.s_max + 1);
        lc.window_evals += (unsigned long long)v.S + 2ull;
        lc.swept = lc.voxel_visits + lc.final_visits;
        if (tid == 0) write_rec(out + v.traj_base + seed, p0, o, sal, (int32_t)seed, v.rank_by);
    }
    if (tid == 0) {
        atomicAdd(&cnt->evals, lc.evals);
        atomicAdd(&cnt->window_evals, lc.window_evals);
        atomicAdd(&cnt->voxel_visits, lc.voxel_visits);
        atomicAdd(&cnt->final_visits, lc.final_visits);
        atomicAdd(&cnt->swept, lc.swept);
    }
    const unsigned long long ops = (unsigned long long)bfly_sumll((long long)lc.lds_ops);
    if ((tid & 63) == 0) atomicAdd(&cnt->lds_ops, ops);
}

// ------------------------------------------------------ dense saliency map
//
// The every-voxel Kadir-Brady search that the seed grid avoids (Sec. 1,
// Sec. 2.1): at every voxel the centred cubes of half-width s_min-1 .. s_max+1,
// their entropies, the entropy peaks over scale and Y = H * W at the best peak,
// with the decision arithmetic of the quadrant method's final pass.  One
// wavefront slides along an x row: it builds the cube histograms of the row's
// first voxel, and for each next voxel takes column x - s out of and column
// x + s + 1 into the histogram of every half-width s (a y-z square each, swept
// along y in the y-fastest copy).

// Adds delta (mod 2^32) to the u32 counter of every voxel's bin in the box, row
// at byte offset rowoff; bytes outside the box go to the lane's trash word.
__device__ __forceinline__ unsigned int map_box(const VolDesc& v, int xa, int xb, int ya, int yb, int za, int zb,
                                                uint32_t* hist, uint32_t rowoff, uint32_t trash, uint32_t delta,
                                                int lane) {
    xa = uniform(xa); xb = uniform(xb); ya = uniform(ya); yb = uniform(yb); za = uniform(za); zb = uniform(zb);
    if (xa > xb || ya > yb || za > zb) return 0u;
    const bool tr = xb - xa < yb - ya;
    const Layout L = tr ? layout_t(v) : layout_x(v);
    const Sweep w = tr ? make_sweep<64>(L, ya, yb, za, zb - za + 1, 1, xa, xb - xa + 1, 1, lane)
                       : make_sweep<64>(L, xa, xb, ya, yb - ya + 1, 1, za, zb - za + 1, 1, lane);
    const int fa = tr ? ya : xa, fb = tr ? yb : xb;
    uint32_t off[4], wid[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int f = w.x0 + k;
        const bool ok = f >= fa && f <= fb;
        off[k] = ok ? rowoff : trash;
        wid[k] = ok ? 8u : 0u;
    }
    char* hb = reinterpret_cast<char*>(hist);
    unsigned int ops = 0;
    int used = 0;
    run_sweep<kMsUnroll, kMsDepth>(
        L, w, 0, 0, used, INT_MAX,
        [&](uint32_t word, int, int, uint64_t) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t bin = __builtin_amdgcn_ubfe(word, 8 * k, wid[k]);
                atomicAdd(reinterpret_cast<uint32_t*>(hb + off[k] + (bin << 2)), delta);
            }
            ops += 4;
        },
        []() {});
    return ops;
}

template <int M>
__global__ __launch_bounds__(64) void k_saliency_map(const VolDesc* __restrict__ vols, Tables tb,
                                                     float* __restrict__ sal, uint8_t* __restrict__ scl,
                                                     Counters* cnt) {
    extern __shared__ uint32_t hmap[];
    const int lane = threadIdx.x;
    const VolDesc& v = vols[0];
    const int B = v.B, Bs = row_stride(B);
    const int lo = v.s_min - 1, K = v.S + 2;  // rows: half-widths lo .. s_max + 1
    const uint32_t trash = (uint32_t)(K * Bs + lane) << 2;
    unsigned int ops = 0;
    const long long rows = (long long)v.Y * v.Z;
    for (long long r = blockIdx.x; r < rows; r += gridDim.x) {
        const int y = (int)(r % v.Y), z = (int)(r / v.Y);
        for (int i = lane; i < K * Bs; i += 64) hmap[i] = 0u;
        __syncthreads();
        for (int i = 0; i < K; ++i) {
            const int s = lo + i;
            ops += map_box(v, 0, min(s, v.X - 1), max(y - s, 0), min(y + s, v.Y - 1), max(z - s, 0),
                           min(z + s, v.Z - 1), hmap, (uint32_t)(i * Bs) << 2, trash, 1u, lane);
        }
        __syncthreads();
        for (int x = 0; x < v.X; ++x) {
            // entropies of every row, streaming: the peak test of half-width
            // s - 1 runs once H(s) is known
            int best = -1;
            double bestY = 0.0;
            double hA = 0.0, hB = 0.0;
            long long aB = 0;
            int64_t nA = 1, nB = 1;
            for (int i = 0; i < K; ++i) {
                const int s = lo + i;
                uint32_t cc[M];
                long long nsum = 0;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    const int b = lane * M + t;
                    cc[t] = b < B ? hmap[i * Bs + b] : 0u;
                    nsum += cc[t];
                }
                // N: the cube's in-volume voxels, or with a window level the voxels it counts
                const int64_t N = v.win ? (int64_t)bfly_sumll(nsum) : cube_count(v, x, y, z, s);
                double cl[M];
                long long am = 0;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    const int b = lane * M + t;
                    cl[t] = tb.cl[cc[t]];
                    if (i > 0 && b < B) {
                        const long long d = (long long)cc[t] * nB - (long long)hmap[(i - 1) * Bs + b] * N;
                        am += d < 0 ? -d : d;
                    }
                }
                const double S = bfly_sum(local_pw<M>(cl));
                const double H = N > 0 ? (tb.cl[N] - S) / (double)N : 0.0;
                const long long A = i > 0 ? bfly_sumll(am) : 0ll;
                if (i >= 2) {
                    const int sp = s - 1;
                    if (hB > hA && hB > H) {
                        const double W = nA > 0 ? ((double)(sp * sp) / (double)(2 * sp - 1)) *
                                                      ((double)aB / ((double)nB * (double)nA))
                                                : 0.0;
                        const double Y = hB * W;
                        if (best < 0 || Y > bestY) { best = sp; bestY = Y; }
                    }
                }
                hA = hB; hB = H; aB = A; nA = nB; nB = N;
            }
            float y32 = 0.0f;
            if (best >= 0) {
                const int rb = best - lo;
                int64_t N = cube_count(v, x, y, z, best), Np = cube_count(v, x, y, z, best - 1);
                if (v.win) {
                    long long n0 = 0, n1 = 0;
#pragma unroll
                    for (int t = 0; t < M; ++t) {
                        const int b = lane * M + t;
                        if (b < B) {
                            n0 += hmap[rb * Bs + b];
                            n1 += hmap[(rb - 1) * Bs + b];
                        }
                    }
                    N = (int64_t)bfly_sumll(n0);
                    Np = (int64_t)bfly_sumll(n1);
                }
                long long am = 0;
                float h = 0.0f;
#pragma unroll
                for (int t = 0; t < M; ++t) {
                    const int b = lane * M + t;
                    if (b < B) {
                        const uint32_t c = hmap[rb * Bs + b];
                        h += entropy_term32((int)c, N);
                        const long long d = (long long)c * Np - (long long)hmap[(rb - 1) * Bs + b] * N;
                        am += d < 0 ? -d : d;
                    }
                }
                const float h32 = bfly_sumf(h);
                const long long A = bfly_sumll(am);
                const float w32 = Np > 0 ? ((float)(best * best) / (float)(2 * best - 1)) *
                                               ((float)A / ((float)N * (float)Np))
                                         : 0.0f;
                y32 = h32 * w32;
            }
            if (lane == 0) {
                const int64_t idx = (int64_t)x + (int64_t)v.X * ((int64_t)y + (int64_t)v.Y * z);
                sal[idx] = y32;
                scl[idx] = (uint8_t)(best < 0 ? 0 : best);
            }
            __syncthreads();
            if (x + 1 < v.X) {
                for (int i = 0; i < K; ++i) {
                    const int s = lo + i;
                    const int ya = max(y - s, 0), yb = min(y + s, v.Y - 1), za = max(z - s, 0), zb = min(z + s, v.Z - 1);
                    const uint32_t ro = (uint32_t)(i * Bs) << 2;
                    if (x - s >= 0) ops += map_box(v, x - s, x - s, ya, yb, za, zb, hmap, ro, trash, 0xFFFFFFFFu, lane);
                    if (x + 1 + s < v.X) ops += map_box(v, x + 1 + s, x + 1 + s, ya, yb, za, zb, hmap, ro, trash, 1u, lane);
                }
                __syncthreads();
            }
        }
    }
    const unsigned long long tot = (unsigned long long)bfly_sumll((long long)ops);
    if (lane == 0) atomicAdd(&cnt->lds_ops, tot);
}

// ------------------------------------------------------------ test hooks

// kind 0: counts of the cube; 1: counts and offset sums of the cube at P; 2: the
// same at Q, reached by the running-window update from P (xyz holds P then Q);
// 3: counts of the cube, of its inner cube through the shell, and of the inner
// cube swept directly.
template <int M>
__global__ __launch_bounds__(64) void k_hook_ms(const VolDesc* vols, int kind, int n, const int* xyz, const int* sc,
                                                int rl, int hist_words, void* outp) {
    extern __shared__ unsigned long long hist[];
    const int lane = threadIdx.x;
    for (int i = lane; i < hist_words; i += 64) hist[i] = 0ull;
    __syncthreads();
    const VolDesc& v = vols[0];
    const int B = v.B;
    const int trash_base = hist_words - 64;
    const int stride = kind == 2 ? 6 : 3;
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int px = xyz[stride * w], py = xyz[stride * w + 1], pz = xyz[stride * w + 2], s = sc[w];
        BinAcc<M> a, e;
        acc_clear<M>(a);
        acc_clear<M>(e);
        ms_sweep<M>(v, BoxSet{kFull, px, py, pz, 0, 0, 0, s}, rl, trash_base, move_budget(s), hist, lane, a);
        int sh[M], bx[M];
        if (kind == 2) {
            const int qx = xyz[6 * w + 3], qy = xyz[6 * w + 4], qz = xyz[6 * w + 5];
#pragma unroll
            for (int k = 0; k < M; ++k) {
                a.f1[k] -= a.c[k] * (qx - px);
                a.f2[k] -= a.c[k] * (qy - py);
                a.f3[k] -= a.c[k] * (qz - pz);
            }
            ms_sweep<M>(v, BoxSet{kMove, px, py, pz, qx, qy, qz, s}, rl, trash_base, move_budget(s), hist, lane, a);
        } else if (kind == 3) {
            ms_sweep<M>(v, BoxSet{kShell, px, py, pz, 0, 0, 0, s}, rl, trash_base, move_budget(s), hist, lane, e);
#pragma unroll
            for (int k = 0; k < M; ++k) sh[k] = a.c[k] - e.c[k];
            acc_clear<M>(e);
            ms_sweep<M>(v, BoxSet{kInner, px, py, pz, 0, 0, 0, s}, rl, trash_base, move_budget(s), hist, lane, e);
#pragma unroll
            for (int k = 0; k < M; ++k) bx[k] = e.c[k];
        }
#pragma unroll
        for (int t = 0; t < M; ++t) {
            const int b = lane * M + t;
            if (b >= B) continue;
            if (kind == 0) {
                static_cast<uint32_t*>(outp)[(size_t)w * B + b] = (uint32_t)a.c[t];
            } else if (kind == 3) {
                uint32_t* o = static_cast<uint32_t*>(outp) + (size_t)w * 3 * B;
                o[b] = (uint32_t)a.c[t];
                o[B + b] = (uint32_t)sh[t];
                o[2 * B + b] = (uint32_t)bx[t];
            } else {
                int* o = static_cast<int*>(outp) + (size_t)w * 4 * B;
                o[b] = a.c[t];
                o[B + b] = a.f1[t] - a.c[t] * s;
                o[2 * B + b] = a.f2[t] - a.c[t] * s;
                o[3 * B + b] = a.f3[t] - a.c[t] * s;
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
    const uint32_t region_bytes = (uint32_t)(K + 1) * (uint32_t)row_stride(B) << (rq + 2);
    for (int w = blockIdx.x; w < n; w += gridDim.x) {
        const int px = xyz[3 * w], py = xyz[3 * w + 1], pz = xyz[3 * w + 2];
        const int nreg = kind == 1 ? 8 : 1;
        if (kind == 1) {
            octant_scatter<256>(v, px, py, pz, hi, lo, K, rq, region_bytes, L.hist, tid);
        } else {
            bucket_scatter<256>(v, max(px - hi, 0), min(px + hi, v.X - 1), max(py - hi, 0), min(py + hi, v.Y - 1),
                                max(pz - hi, 0), min(pz + hi, v.Z - 1), px, py, pz, lo, K, rq, 0u, L.hist, tid);
        }
        __syncthreads();
        bucket_merge<256>(L.hist, nreg, K, B, rq, tid);
        __syncthreads();
        for (int i = tid; i < nreg * K * B; i += 256) {
            const int g = i / (K * B), rem = i - g * K * B, r = rem / B, b = rem - r * B;
            const int e = ((g * (K + 1) + r) * row_stride(B) + b) << rq;
            outp[(size_t)w * nreg * K * B + i] = L.hist[e];
        }
        __syncthreads();
        for (int i = tid; i < nreg * K * B; i += 256) {
            const int g = i / (K * B), rem = i - g * K * B, r = rem / B, b = rem - r * B;
            L.hist[((g * (K + 1) + r) * row_stride(B) + b) << rq] = 0u;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ ranking

__device__ __forceinline__ bool rec_less(const SortRec& a, const SortRec& b) {
    if (a.vol != b.vol) return a.vol < b.vol;
    if (a.ky != b.ky) return a.ky < b.ky;
    if (a.kpos != b.kpos) return a.kpos < b.kpos;
    return a.seed < b.seed;
}

// Kept trajectories into sort records; one counter atomic per block and pass of
// the loop (the records' order is irrelevant: the sort keys are distinct).
__global__ __launch_bounds__(256) void k_compact(const VolDesc* vols, const TrajRec* rec, SortRec* sr,
                                                 Counters* cnt) {
    __shared__ unsigned int wn[4];
    __shared__ unsigned long long bbase;
    const VolDesc& v = vols[blockIdx.y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (long long b = (long long)blockIdx.x * blockDim.x; b < v.n_traj; b += (long long)gridDim.x * blockDim.x) {
        const long long i = b + threadIdx.x;
        TrajRec r;
        bool keep = false;
        if (i < v.n_traj) {
            r = rec[v.traj_base + i];
            keep = r.keep != 0;
        }
        const unsigned long long m = __ballot(keep);
        if (lane == 0) wn[wave] = (unsigned int)__popcll(m);
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned int t = wn[0] + wn[1] + wn[2] + wn[3];
            bbase = t ? atomicAdd(&cnt->n_sort, (unsigned long long)t) : 0ull;
        }
        __syncthreads();
        unsigned long long k = bbase;
        for (int w = 0; w < wave; ++w) k += wn[w];
        k += (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
        if (keep) {
            SortRec o;
            o.vol = blockIdx.y;
            o.ky = ~(uint64_t)__double_as_longlong(r.key64 + 0.0);
            o.kpos = ((uint64_t)r.scale << 48) | ((uint64_t)r.z << 32) | ((uint64_t)r.y << 16) | (uint64_t)r.x;
            o.seed = (uint32_t)r.seed;
            o.idx = (uint32_t)(v.traj_base + i);
            sr[k] = o;
        }
        __syncthreads();
    }
}

// A record of the lane `lane ^ m` of the same wavefront (m < 64).
__device__ __forceinline__ SortRec shfl_xor_rec(const SortRec& r, unsigned m) {
    uint32_t w[8];
    static_assert(sizeof(SortRec) == sizeof(w), "SortRec is 8 dwords");
    __builtin_memcpy(w, &r, sizeof(w));
#pragma unroll
    for (int t = 0; t < 8; ++t) w[t] = (uint32_t)__shfl_xor((int)w[t], (int)m, 64);
    SortRec o;
    __builtin_memcpy(&o, w, sizeof(w));
    return o;
}

// Sorts each block of L records (L = blockDim, a power of two) with a bitonic
// network whose every stage leaves its blocks ascending: in the stage for
// blocks of k, each record is first compared with its mirror i ^ (k - 1), then
// with i ^ j for j = k/4 .. 1 (half-cleaners); the lower index keeps the
// smaller record.  One record per thread, in registers: partners within the
// wavefront (distance < 64) come by lane shuffles, the others through LDS.
// Blocks past the real records are skipped; the last real block is filled up
// with all-ones padding records, which sort to its end.
__global__ __launch_bounds__(512) void k_sort_local(SortRec* sr, unsigned L, const Counters* cnt) {
    extern __shared__ SortRec lsr[];
    const unsigned long long count = cnt->n_sort;
    const unsigned long long start = (unsigned long long)blockIdx.x * L;
    if (start >= count) return;
    const unsigned i = threadIdx.x;
    SortRec r;
    if (start + i < count) {
        r = sr[start + i];
    } else {
        r.vol = ~0ull; r.ky = ~0ull; r.kpos = ~0ull; r.seed = ~0u; r.idx = ~0u;
    }
    for (unsigned k = 2; k <= L; k <<= 1) {
        for (unsigned j = k / 2; j >= 1; j >>= 1) {
            const unsigned m = j == k / 2 ? k - 1 : j;
            SortRec o;
            if (m < 64) {
                o = shfl_xor_rec(r, m);
            } else {
                lsr[i] = r;
                __syncthreads();
                o = lsr[i ^ m];
                __syncthreads();
            }
            if ((i < (i ^ m)) == rec_less(o, r)) r = o;
        }
    }
    sr[start + i] = r;
}

// One merge level: src holds sorted runs of `width` records (keys distinct,
// 2 * width a multiple of kMergeTile); run pairs are merged into dst.  A block
// writes kMergeTile consecutive outputs of one pair (merge-path tiles): wave 0
// finds how many records of the first run precede the tile's first output,
// wave 1 the same for the tile's end, the block stages the two sub-runs between
// in LDS, and a record's place in the tile is its index in its sub-run plus the
// number of the other sub-run's records ordered before it.  Only the first
// `count` records are real.
constexpr int kMergeTile = 512;

// Records of A among the first d outputs of merge(A, B): the first i in
// [max(0, d - lb), min(d, la)] with i = min(d, la) or B[d-1-i] < A[i] (monotone
// in i).  A 64-ary search, one candidate per lane and one ballot per round; the
// whole wave gets the result.
__device__ long long merge_split(const SortRec* A, long long la, const SortRec* B, long long lb, long long d,
                                 int lane) {
    long long lo = d > lb ? d - lb : 0;
    long long hi = d < la ? d : la;
    while (hi > lo) {
        const long long stride = (hi - lo + 63) / 64;
        const long long c = lo + lane * stride;
        const bool t = c >= hi || rec_less(B[d - 1 - c], A[c]);
        const unsigned long long m = __ballot(t);
        if (m == 0ull) {
            lo += 63 * stride + 1;
        } else {
            const int k = __ffsll((long long)m) - 1;
            if (k == 0) break;
            const long long top = lo + k * stride;
            lo += (k - 1) * stride + 1;
            hi = top < hi ? top : hi;
        }
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_merge(const SortRec* src, SortRec* dst, unsigned long long width,
                                               const Counters* cnt) {
    __shared__ SortRec tile[kMergeTile];
    __shared__ long long split[2];
    const unsigned long long count = cnt->n_sort;
    const unsigned long long g0 = (unsigned long long)blockIdx.x * kMergeTile;
    if (g0 >= count) return;
    const unsigned long long a0 = g0 / (2 * width) * (2 * width), b0 = a0 + width;
    const long long la = (long long)(count - a0 < width ? count - a0 : width);
    const long long lb = count > b0 ? (long long)(count - b0 < width ? count - b0 : width) : 0;
    const long long d0 = (long long)(g0 - a0);
    const long long d1 = d0 + kMergeTile < la + lb ? d0 + kMergeTile : la + lb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave < 2) {
        const long long sp = merge_split(src + a0, la, src + b0, lb, wave ? d1 : d0, lane);
        if (lane == 0) split[wave] = sp;
    }
    __syncthreads();
    const long long i0 = split[0], i1 = split[1];
    const int na = (int)(i1 - i0), n = (int)(d1 - d0), nb = n - na;
    const SortRec* sa = src + a0 + i0;
    const SortRec* sb = src + b0 + (d0 - i0);
    for (int k = threadIdx.x; k < n; k += blockDim.x) tile[k] = k < na ? sa[k] : sb[k - na];
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const SortRec x = tile[k];
        const bool in_a = k < na;
        const SortRec* other = in_a ? tile + na : tile;
        int lo = 0, hi = in_a ? nb : na;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rec_less(other[mid], x)) lo = mid + 1;
            else hi = mid;
        }
        dst[g0 + (in_a ? k : k - na) + lo] = x;
    }
}

__device__ __forceinline__ bool first_of_region(const SortRec* sr, unsigned long long i) {
    if (i == 0) return true;
    const SortRec& a = sr[i];
    const SortRec& b = sr[i - 1];
    return a.vol != b.vol || a.kpos != b.kpos;
}

// Per 1024-element block: number of distinct regions; per volume: regions found.
// Each wavefront counts the regions of the first volume among its lanes; the
// block adds the counts of consecutive wavefronts with the same volume (the
// records are sorted by volume) in one atomic, and a lane of a later volume
// within a wavefront (a volume boundary) adds its own.
__global__ __launch_bounds__(1024) void k_dedup_count(const SortRec* sr, const Counters* cnt, int* bsum,
                                                      int* vol_nfound) {
    __shared__ int wsum[16], wvol[16], wcnt[16];
    const unsigned long long count = cnt->n_sort;
    const unsigned long long i = (unsigned long long)blockIdx.x * 1024 + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int f = (i < count && first_of_region(sr, i)) ? 1 : 0;
    const int vol = i < count ? (int)sr[i].vol : -1;
    const unsigned long long fmask = __ballot(f);
    int lv = -1, lc = 0;
    if (fmask) {
        const int lead = __ffsll((long long)fmask) - 1;
        lv = __shfl(vol, lead, 64);
        const bool same = f && vol == lv;
        lc = (int)__popcll(__ballot(same));
        if (f && !same) atomicAdd(&vol_nfound[vol], 1);
    }
    int s = f;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m, 64);
    if (lane == 0) {
        wsum[wave] = s;
        wvol[wave] = lv;
        wcnt[wave] = lc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0, rv = -1, rc = 0;
        for (int w = 0; w < 16; ++w) {
            t += wsum[w];
            if (wcnt[w] == 0) continue;
            if (wvol[w] != rv) {
                if (rc) atomicAdd(&vol_nfound[rv], rc);
                rv = wvol[w];
                rc = 0;
            }
            rc += wcnt[w];
        }
        if (rc) atomicAdd(&vol_nfound[rv], rc);
        bsum[blockIdx.x] = t;
    }
}

// Exclusive scan of n ints from in to out (one 1024-thread block, sequential
// chunks; in == out allowed).
__device__ void block_exclusive_scan(const int* in, int* out, int n, int* buf, int* carry) {
    if (threadIdx.x == 0) *carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int i = base + threadIdx.x;
        const int x = i < n ? in[i] : 0;
        buf[threadIdx.x] = x;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) out[i] = *carry + buf[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 1023) *carry += buf[1023];
        __syncthreads();
    }
}

// Exclusive scans of the block sums (in place) and of the per-volume region
// counts (the volumes' first global ranks: records are sorted by volume).
__global__ __launch_bounds__(1024) void k_scan_bsum(int* bsum, int nblk, const int* vol_nfound, int* vol_base,
                                                    int nvol) {
    __shared__ int buf[1024];
    __shared__ int carry;
    block_exclusive_scan(bsum, bsum, nblk, buf, &carry);
    block_exclusive_scan(vol_nfound, vol_base, nvol, buf, &carry);
}

// Global region rank g of every first-of-region record, and its region written
// at g - (its volume's first rank) when that is below the volume's capacity.
__global__ __launch_bounds__(1024) void k_dedup_rank(const SortRec* sr, const Counters* cnt, const int* bsum,
                                                     const int* vol_base, const VolDesc* vols, const TrajRec* rec,
                                                     ks_region_dev* regions) {
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
        const int vol = (int)sr[i].vol;
        const int pos = g - vol_base[vol];
        const VolDesc& v = vols[vol];
        if (pos < v.cap) {
            const TrajRec r = rec[sr[i].idx];
            ks_region_dev o;
            o.x = r.x; o.y = r.y; o.z = r.z; o.scale = r.scale;
            o.saliency = r.y32; o.entropy = r.h32; o.pdf_change = r.w32;
            o.seed = r.seed;
            regions[v.reg_off + pos] = o;
        }
    }
}

// ------------------------------------------------------------ launchers
// ------------------------------------------------------------ launchers

static int grid_for(long long n, int threads, int cap) {
    long long g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    return (int)(g > cap ? cap : g);
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_prep_init, dim3((a.nvol + 255) / 256), dim3(256), 0, st, a.vols, a.nvol, a.cnt,
                       a.vol_nfound, a.vol_base);
    const int gx = grid_for(a.max_voxels, 256 * 32, 512);
    hipLaunchKernelGGL(k_minmax, dim3(gx, a.nvol), dim3(256), 0, st, a.vols);
    const int gq = grid_for(a.max_words, 256, 4096);
    hipLaunchKernelGGL(k_quantize, dim3(gq, a.nvol), dim3(256), 0, st, a.vols);
    if (a.max_z > 0)
        hipLaunchKernelGGL(k_transpose, dim3(a.max_tx * a.max_ty, a.max_z, a.nvol), dim3(256), 0, st, a.vols,
                           a.max_tx);
    return hipGetLastError();
}

int bins_per_lane_host(int B) { return B <= 64 ? 1 : (B <= 128 ? 2 : 4); }

hipError_t launch_search_ms(const SearchArgs& a, const XcdQueues* xq, int chunk, int grid, const MsTune& tune,
                            int hist_words, int maxB, hipStream_t st) {
    if (a.ntask <= 0) return hipSuccess;
    const size_t lds = (size_t)hist_words * 8;
    const int M = bins_per_lane_host(maxB);
    // one scale per task: the kernel without the group bookkeeping (fewer registers)
#define KS_LAUNCH_MS(MM, GG)                                                                                   \
    hipLaunchKernelGGL((k_search_ms<MM, GG>), dim3(grid), dim3(64), lds, st, a.vols, a.segs, a.nseg, xq, chunk, \
                       a.tb, a.rec, a.cnt, tune, hist_words)
    const bool g = tune.group > 1;
    if (M == 1) { if (g) KS_LAUNCH_MS(1, true); else KS_LAUNCH_MS(1, false); }
    else if (M == 2) { if (g) KS_LAUNCH_MS(2, true); else KS_LAUNCH_MS(2, false); }
    else { if (g) KS_LAUNCH_MS(4, true); else KS_LAUNCH_MS(4, false); }
#undef KS_LAUNCH_MS
    return hipGetLastError();
}

hipError_t launch_search_quad(const SearchArgs& a, int grid, int rq, const LdsQuad& lay, int maxB, hipStream_t st) {
    if (a.ntask <= 0) return hipSuccess;
    const int M = bins_per_lane_host(maxB);
    if (M == 1)
        hipLaunchKernelGGL(k_search_quad<1>, dim3(grid), dim3(kQuadThreads), lay.bytes, st, a.vols, a.segs, a.nseg, a.ntask,
                           a.tb, a.rec, a.cnt, rq, lay);
    else if (M == 2)
        hipLaunchKernelGGL(k_search_quad<2>, dim3(grid), dim3(kQuadThreads), lay.bytes, st, a.vols, a.segs, a.nseg, a.ntask,
                           a.tb, a.rec, a.cnt, rq, lay);
    else
        hipLaunchKernelGGL(k_search_quad<4>, dim3(grid), dim3(kQuadThreads), lay.bytes, st, a.vols, a.segs, a.nseg, a.ntask,
                           a.tb, a.rec, a.cnt, rq, lay);
    return hipGetLastError();
}

hipError_t launch_hook_ms(const VolDesc* vols, int kind, int n, const int* xyz, const int* sc, int rl, int hist_words,
                          int maxB, void* out, hipStream_t st) {
    const int M = bins_per_lane_host(maxB);
    const size_t lds = (size_t)hist_words * 8;
    if (M == 1)
        hipLaunchKernelGGL(k_hook_ms<1>, dim3(grid_for(n, 1, 4096)), dim3(64), lds, st, vols, kind, n, xyz, sc, rl,
                           hist_words, out);
    else if (M == 2)
        hipLaunchKernelGGL(k_hook_ms<2>, dim3(grid_for(n, 1, 4096)), dim3(64), lds, st, vols, kind, n, xyz, sc, rl,
                           hist_words, out);
    else
        hipLaunchKernelGGL(k_hook_ms<4>, dim3(grid_for(n, 1, 4096)), dim3(64), lds, st, vols, kind, n, xyz, sc, rl,
                           hist_words, out);
    return hipGetLastError();
}

hipError_t launch_hook_quad(const VolDesc* vols, int kind, int lo, int hi, int n, const int* xyz, int rq,
                            const LdsQuad& lay, uint32_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_hook_quad, dim3(grid_for(n, 1, 4096)), dim3(256), lay.bytes, st, vols, kind, lo, hi, n, xyz,
                       rq, lay, out);
    return hipGetLastError();
}

// The mean-shift decisions' roots of every count 0..n-1 (test hook).
__global__ __launch_bounds__(256) void k_count_roots(int n, double* sq, double* rs) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        double a, b;
        count_roots(c, a, b);
        sq[c] = a;
        rs[c] = b;
    }
}

hipError_t launch_count_roots(int n, double* sq, double* rs, hipStream_t st) {
    hipLaunchKernelGGL(k_count_roots, dim3(grid_for(n, 256, 1024)), dim3(256), 0, st, n, sq, rs);
    return hipGetLastError();
}

// Device memory of the allocation-free detection entry point: one array per
// GPU, alive until the process ends.  Host code never uses the array's name as
// an address: scratch_address() looks up this GPU's copy once and hands out
// that pointer.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void** ptr) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    // the caller has made `device` current
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
    *ptr = p;
    return hipSuccess;
}

hipError_t launch_rank(const RankArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_compact, dim3(grid_for(a.max_traj, 256, 1024), a.nvol), dim3(256), 0, st, a.vols, a.rec,
                       a.sr, a.cnt);
    const unsigned long long n_pad = a.n_pad;
    // sorted runs of L records in LDS, then merge levels ping-ponging between the
    // two halves of the sort buffer
    const unsigned L = n_pad < 512 ? (unsigned)n_pad : 512u;
    const unsigned nblk_local = (unsigned)(n_pad / L);
    const size_t lds = (size_t)L * sizeof(SortRec);
    const unsigned threads = L;
    hipLaunchKernelGGL(k_sort_local, dim3(nblk_local), dim3(threads), lds, st, a.sr, L, a.cnt);
    SortRec* src = a.sr;
    SortRec* dst = a.sr + n_pad;
    for (unsigned long long width = L; width < n_pad; width <<= 1) {
        if ((2 * width) % kMergeTile != 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_merge, dim3((unsigned)((n_pad + kMergeTile - 1) / kMergeTile)), dim3(256), 0, st, src,
                           dst, width, a.cnt);
        SortRec* t = src;
        src = dst;
        dst = t;
    }
    const SortRec* sorted = src;
    const int nblk = (int)((n_pad + 1023) / 1024);
    hipLaunchKernelGGL(k_dedup_count, dim3(nblk), dim3(1024), 0, st, sorted, a.cnt, a.bsum, a.vol_nfound);
    hipLaunchKernelGGL(k_scan_bsum, dim3(1), dim3(1024), 0, st, a.bsum, nblk, a.vol_nfound, a.vol_base, a.nvol);
    hipLaunchKernelGGL(k_dedup_rank, dim3(nblk), dim3(1024), 0, st, sorted, a.cnt, a.bsum, a.vol_base, a.vols, a.rec,
                       a.regions);
    return hipGetLastError();
}

hipError_t launch_saliency_map(const VolDesc* vols, Tables tb, float* sal, uint8_t* scl, Counters* cnt, int K, int B,
                               int grid, hipStream_t st) {
    const size_t lds = ((size_t)K * (size_t)(B | 1) + 64) * 4;
    const int M = bins_per_lane_host(B);
    if (M == 1) hipLaunchKernelGGL(k_saliency_map<1>, dim3(grid), dim3(64), lds, st, vols, tb, sal, scl, cnt);
    else if (M == 2) hipLaunchKernelGGL(k_saliency_map<2>, dim3(grid), dim3(64), lds, st, vols, tb, sal, scl, cnt);
    else hipLaunchKernelGGL(k_saliency_map<4>, dim3(grid), dim3(64), lds, st, vols, tb, sal, scl, cnt);
    return hipGetLastError();
}

int max_blocks_map(int K, int B) {
    int nb = 0;
    const size_t lds = ((size_t)K * (size_t)(B | 1) + 64) * 4;
    const int M = bins_per_lane_host(B);
    hipError_t e = M == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_saliency_map<1>, 64, lds)
                 : M == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_saliency_map<2>, 64, lds)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_saliency_map<4>, 64, lds);
    if (e != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

// Resident blocks per CU from the occupancy calculator, cached per device and
// launch shape (the query costs host time on every detection otherwise).
static int cached_occupancy(int kind, int M, size_t lds, int (*query)(int M, size_t lds)) {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, size_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return query(M, lds);
    const auto key = std::make_tuple(dev, kind, M, lds);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int nb = query(M, lds);
    std::lock_guard<std::mutex> g(mu);
    cache[key] = nb;
    return nb;
}

static int query_ms(int M, size_t lds) {
    int nb = 0;
    hipError_t e = M == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_ms<1, false>, 64, lds)
                 : M == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_ms<2, false>, 64, lds)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_ms<4, false>, 64, lds);
    if (e != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

static int query_quad(int M, size_t lds) {
    int nb = 0;
    hipError_t e = M == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_quad<1>, kQuadThreads, lds)
                 : M == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_quad<2>, kQuadThreads, lds)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_search_quad<4>, kQuadThreads, lds);
    if (e != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

int max_blocks_ms(int hist_words, int maxB) {
    return cached_occupancy(0, bins_per_lane_host(maxB), (size_t)hist_words * 8, query_ms);
}

int max_blocks_quad(size_t lds_bytes, int maxB) {
    return cached_occupancy(1, bins_per_lane_host(maxB), lds_bytes, query_quad);
}

}  // namespace ks

// Host runtime of the C ABI: contexts, argument checks, work planning, the launch
// sequence (prep -> persistent searches -> device ranking), hooks and batching.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ks.h"
#include "ks_device.h"
#include "ks_launch.h"
#include "ks_runtime.h"
#include "ks_abmsod.h"

namespace ks {

// ------------------------------------------------------------ validation

static bool dims_ok(const int32_t* d) {
    if (!d) return false;
    for (int a = 0; a < 3; ++a)
        if (d[a] < 1 || d[a] > 65535) return false;
    // the bin volume, rows padded to 16 bytes, is addressed with 32-bit offsets
    return (int64_t)((d[0] + 15) & ~15) * d[1] * d[2] < (int64_t(1) << 31);
}

bool options_ok(const ks_options& o) {
    return o.h_min == o.h_min && o.y_min == o.y_min && (o.rank_by == KS_RANK_SALIENCY || o.rank_by == KS_RANK_PDF_CHANGE) &&
           (o.window == 0 || (o.window == 1 && o.win_lo <= o.win_hi));
}

bool options_fit(const ks_options& o, int32_t bins) { return o.window == 0 || bins <= 255; }

ks_status check_request(const void* vol, int32_t dtype, const int32_t* dims, int32_t bins, int32_t spacing,
                        const int32_t* scales, int32_t method, int32_t max_iter) {
    if (!vol || !dims || !scales) return KS_E_INVALID;
    if (dtype < KS_U8 || dtype > KS_I16) return KS_E_INVALID;
    if (!dims_ok(dims)) return KS_E_INVALID;
    if (bins < 2 || bins > kBinsLimit) return KS_E_INVALID;
    if (spacing < 1) return KS_E_INVALID;
    if (scales[0] < 1 || scales[0] > scales[1] || scales[1] > kSmaxLimit) return KS_E_INVALID;
    if (method != KS_QUADRANT && method != KS_MEANSHIFT) return KS_E_INVALID;
    if (max_iter < 0) return KS_E_INVALID;
    return KS_OK;
}

static int64_t grid_count(int32_t dim, int32_t sp, int32_t* o) {
    int32_t off = sp / 2;
    if (off >= dim) off = (dim - 1) / 2;
    *o = off;
    return (dim - 1 - off) / sp + 1;
}

int64_t num_trajectories(const int32_t* dims, int32_t spacing, const int32_t* scales, int32_t method) {
    int32_t o;
    int64_t n = grid_count(dims[0], spacing, &o) * grid_count(dims[1], spacing, &o) * grid_count(dims[2], spacing, &o);
    return method == KS_MEANSHIFT ? n * (scales[1] - scales[0] + 1) : n;
}

int64_t num_trajectories(const VolIn& v) {
    if (!v.seeds) return num_trajectories(v.dims, v.spacing, v.scales, v.method);
    return v.method == KS_MEANSHIFT ? v.n_seeds * (v.scales[1] - v.scales[0] + 1) : v.n_seeds;
}

ks_status check_seeds(const int32_t* dims, const int32_t* scales, int32_t method, const int32_t* seeds, int64_t n) {
    if (n < 0 || (n > 0 && !seeds)) return KS_E_INVALID;
    const int64_t per = method == KS_MEANSHIFT ? scales[1] - scales[0] + 1 : 1;
    if (n > (int64_t)INT32_MAX / per) return KS_E_INVALID;
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            if (seeds[3 * i + a] < 0 || seeds[3 * i + a] >= dims[a]) return KS_E_INVALID;
    return KS_OK;
}

// Bin volume x fastest (rows padded to 16 bytes), then the y-fastest copy.
static size_t bins_x_bytes(const int32_t* dims) {
    const size_t xp = ((size_t)dims[0] + 15) & ~(size_t)15;
    return (xp * dims[1] * dims[2] + 255) & ~(size_t)255;
}

size_t bins_bytes(const int32_t* dims) {
    const size_t yp = ((size_t)dims[1] + 15) & ~(size_t)15;
    return bins_x_bytes(dims) + ((yp * dims[2] * dims[0] + 255) & ~(size_t)255);
}

// ------------------------------------------------------------ context

static ks_status hip_fail(hipError_t e) { return e == hipErrorOutOfMemory ? KS_E_NOMEM : KS_E_DEVICE; }
#define KS_HIP(call)                                    \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) return hip_fail(_e);      \
    } while (0)

ks_status Buffer::ensure(size_t bytes, int* generation) {
    if (bytes <= cap) return KS_OK;
    // grow by at least 1.5x so that a slowly rising size reallocates rarely
    const size_t want = granule(std::max(bytes, cap + cap / 2));
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(&ptr, want);
    if (e != hipSuccess) {
        ptr = nullptr;
        return hip_fail(e);
    }
    cap = want;
    if (generation) ++*generation;
    return KS_OK;
}

void Buffer::release() {
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    cap = 0;
}

ks_status PinnedBuffer::ensure(size_t bytes) {
    if (bytes <= cap) return KS_OK;
    size_t want = (std::max(std::max(bytes, (size_t)4096), cap + cap / 2) + 4095) & ~(size_t)4095;
    if (ptr) hipHostFree(ptr);
    ptr = nullptr;
    cap = 0;
    if (hipHostMalloc(&ptr, want, hipHostMallocDefault) != hipSuccess) {
        ptr = nullptr;
        return KS_E_NOMEM;
    }
    cap = want;
    return KS_OK;
}

void PinnedBuffer::release() {
    if (ptr) hipHostFree(ptr);
    ptr = nullptr;
    cap = 0;
}

ks_status Context::init(int32_t dev) {
    device = dev;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || dev < 0 || dev >= n) return KS_E_DEVICE;
    KS_HIP(hipSetDevice(dev));
    hipDeviceProp_t prop;
    KS_HIP(hipGetDeviceProperties(&prop, dev));
    num_cu = prop.multiProcessorCount;
    // Decision tables: the same libm calls a plain CPU implementation makes.
    const size_t n_tab = (size_t)kTableMax + 1;
    std::vector<double> cl(n_tab), sq(n_tab), rsq(n_tab);
    for (size_t c = 0; c < n_tab; ++c) {
        const double d = (double)c;
        cl[c] = c > 0 ? d * std::log(d) : 0.0;
        sq[c] = std::sqrt(d);
        rsq[c] = c > 0 ? 1.0 / std::sqrt(d) : 0.0;
    }
    ks_status st = tables_buf.ensure(3 * n_tab * sizeof(double), nullptr);
    if (st != KS_OK) return st;
    double* base = static_cast<double*>(tables_buf.ptr);
    KS_HIP(hipMemcpy(base, cl.data(), n_tab * sizeof(double), hipMemcpyHostToDevice));
    KS_HIP(hipMemcpy(base + n_tab, sq.data(), n_tab * sizeof(double), hipMemcpyHostToDevice));
    KS_HIP(hipMemcpy(base + 2 * n_tab, rsq.data(), n_tab * sizeof(double), hipMemcpyHostToDevice));
    tables.cl = base;
    tables.sq = base + n_tab;
    tables.rsq = base + 2 * n_tab;
    for (int i = 0; i < kEvents; ++i) KS_HIP(hipEventCreate(&ev[i]));
    KS_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
    KS_HIP(hipEventCreateWithFlags(&join_ev, hipEventDisableTiming));
    KS_HIP(hipEventCreateWithFlags(&order_ev, hipEventDisableTiming));
    // the device's static array of the allocation-free entry point (null if the
    // lookup fails: that entry point then reports KS_E_DEVICE)
    void* sp = nullptr;
    scratch = scratch_address(dev, &sp) == hipSuccess ? static_cast<char*>(sp) : nullptr;
    return KS_OK;
}

void Context::destroy() {
    hipSetDevice(device);
    for (auto& g : graphs)
        if (g.exec) hipGraphExecDestroy(g.exec);
    graphs.clear();
    Buffer* bufs[] = {&tables_buf, &d_vols, &d_abm, &d_bins, &d_rec, &d_sr, &d_bsum,
                      &d_volint, &d_regions, &d_hook, &d_hook_out, &d_raw};
    for (Buffer* b : bufs) b->release();
    h_stage.release();
    h_out.release();
    if (aux) hipStreamDestroy(aux);
    if (batch_stream) hipStreamDestroy(batch_stream);
    for (int i = 0; i < kEvents; ++i)
        if (ev[i]) hipEventDestroy(ev[i]);
    if (fork_ev) hipEventDestroy(fork_ev);
    if (join_ev) hipEventDestroy(join_ev);
    if (order_ev) hipEventDestroy(order_ev);
}

// ------------------------------------------------------------ planning

static unsigned long long next_pow2(unsigned long long n) {
    unsigned long long p = 2;
    while (p < n) p <<= 1;
    return p;
}

// Replica counts: as many as fit a per-workgroup LDS budget (more replicas, fewer
// same-address LDS atomics; fewer, cheaper merges).
int pick_ms_rl(int maxB, int pref) {
    int rl = pref;
    while (rl > 2 && (((size_t)maxB + 1) * ((size_t)1 << rl) + 64) * 8 > 36 * 1024) --rl;
    return rl;
}

// Quadrant LDS: 8 octant regions of (S+1) rows (S shells and a trash row) x B bins
// x replicas; the saliency pass reuses it as one region of S+3 rows.
LdsQuad quad_layout(int maxS, int maxB, int rq) {
    LdsQuad L;
    size_t off = 0;
    L.hist_off = off;
    L.hist_words = (int)(8 * ((size_t)maxS + 1) * (((size_t)maxB + 1) | 1) * ((size_t)1 << rq));
    off += (size_t)L.hist_words * 4;
    off = (off + 15) & ~(size_t)15;
    L.eps_off = off;
    off += 8 * (size_t)maxS * 8;
    L.hrow_off = off;
    off += (size_t)(maxS + 2) * 8;
    L.arow_off = off;
    off += (size_t)(maxS + 2) * 8;
    L.nrow_off = off;
    off += (size_t)(maxS + 2) * 8;
    L.h32_off = off;
    off += (size_t)(maxS + 2) * 4;
    off = (off + 15) & ~(size_t)15;
    L.res_off = off;
    off += 4 * 8;
    L.bytes = (off + 15) & ~(size_t)15;
    L.pad = 0;
    return L;
}

int pick_quad_rq(int maxS, int maxB, int pref) {
    int rq = pref;
    while (rq > 0 && quad_layout(maxS, maxB, rq).bytes > 64 * 1024) --rq;
    return rq;
}

// Byte layout of the result allocation: regions, per-volume region counts, the
// counter block.
static void result_layout(size_t nvol, int64_t regs, size_t* nf_off, size_t* cnt_off, size_t* bytes) {
    *nf_off = sizeof(ks_region) * (size_t)std::max<int64_t>(regs, 0);
    *cnt_off = (*nf_off + sizeof(int) * nvol + 63) & ~(size_t)63;
    *bytes = *cnt_off + sizeof(Counters);
}

void arena_needs(const std::vector<VolIn>& in, size_t need[kArenaBuffers]) {
    int64_t traj = 0, regs = 0;
    size_t bins = 0, seed_ints = 0, segs = 1;
    for (const VolIn& v : in) {
        traj += num_trajectories(v);
        regs += v.capacity;
        bins += bins_bytes(v.dims);
        if (v.seeds) seed_ints += 3 * (size_t)v.n_seeds;
        // at most one task run per scale and XCD (mean-shift) or one (quadrant)
        segs += v.method == KS_MEANSHIFT ? (size_t)(v.scales[1] - v.scales[0] + 1) * kXcds : 1;
    }
    const unsigned long long n_pad = next_pow2((unsigned long long)std::max<int64_t>(traj, 2));
    size_t nf_off, cnt_off, out_bytes;
    result_layout(in.size(), regs, &nf_off, &cnt_off, &out_bytes);
    need[0] = std::max<size_t>(sizeof(VolDesc) * in.size() + sizeof(XcdQueues) * kMaxMsChunks + sizeof(TaskSeg) * segs +
                                   sizeof(int32_t) * seed_ints,
                               256);
    need[1] = std::max<size_t>(bins, 256);
    need[2] = sizeof(TrajRec) * (size_t)std::max<int64_t>(traj, 1);
    need[3] = 2 * sizeof(SortRec) * n_pad;
    need[4] = sizeof(int) * (n_pad / 1024 + 2);
    need[5] = sizeof(int) * 3 * in.size();
    need[6] = out_bytes;
}

Buffer& Context::arena(int i) {
    switch (i) {
        case 0: return d_vols;
        case 1: return d_bins;
        case 2: return d_rec;
        case 3: return d_sr;
        case 4: return d_bsum;
        case 5: return d_volint;
        default: return d_regions;
    }
}

size_t Context::arena_held() {
    size_t n = 0;
    for (int i = 0; i < kArenaBuffers; ++i) n += arena(i).cap;
    return n;
}

size_t Context::arena_after(const std::vector<VolIn>& in) {
    size_t need[kArenaBuffers];
    arena_needs(in, need);
    size_t n = 0;
    for (int i = 0; i < kArenaBuffers; ++i) {
        const Buffer& b = arena(i);
        n += need[i] <= b.cap ? b.cap : granule(std::max(need[i], b.cap + b.cap / 2));
    }
    return n;
}

size_t Context::arena_fresh(const std::vector<VolIn>& in) {
    size_t need[kArenaBuffers];
    arena_needs(in, need);
    size_t n = 0;
    for (int i = 0; i < kArenaBuffers; ++i) n += granule(need[i]);
    return n;
}

void Context::arena_release() {
    for (int i = 0; i < kArenaBuffers; ++i) arena(i).release();
    ++generation;  // captured graphs hold the old addresses
}

ks_status Context::plan(const std::vector<VolIn>& in, Plan& p, const FixedArena* fixed) {
    p = Plan();
    const int nvol = (int)in.size();
    p.nvol = nvol;
    p.vols.resize(nvol);
    size_t bins_total = 0;
    std::vector<size_t> bins_off(nvol);
    int64_t traj = 0, regs = 0;
    for (int i = 0; i < nvol; ++i) {
        const VolIn& r = in[i];
        VolDesc& v = p.vols[i];
        std::memset(&v, 0, sizeof(v));
        v.raw = r.raw;
        v.X = r.dims[0]; v.Y = r.dims[1]; v.Z = r.dims[2];
        v.xp = (v.X + 15) & ~15;
        v.slice = (int64_t)v.xp * v.Y;
        v.yp = (v.Y + 15) & ~15;
        v.slice_t = (int64_t)v.yp * v.Z;
        v.dtype = r.dtype; v.B = r.bins; v.sp = r.spacing;
        v.s_min = r.scales[0]; v.s_max = r.scales[1]; v.S = v.s_max - v.s_min + 1;
        v.method = r.method; v.max_iter = r.max_iter;
        v.gx = (int32_t)grid_count(v.X, v.sp, &v.ox);
        v.gy = (int32_t)grid_count(v.Y, v.sp, &v.oy);
        v.gz = (int32_t)grid_count(v.Z, v.sp, &v.oz);
        p.seed_off.push_back(p.seed_ints);
        if (r.seeds) {  // a list of n_seeds positions in place of the grid
            v.gx = (int32_t)r.n_seeds; v.gy = 1; v.gz = 1;
            v.ox = v.oy = v.oz = 0;
            p.seed_ints += 3 * (size_t)r.n_seeds;
        }
        v.traj_base = traj;
        v.n_traj = num_trajectories(r);
        v.h_min = r.opt.h_min; v.y_min = r.opt.y_min; v.rank_by = r.opt.rank_by;
        v.win = r.opt.window; v.win_lo = r.opt.win_lo; v.win_hi = r.opt.win_hi;
        v.reg_off = regs;
        v.cap = r.capacity;
        bins_off[i] = bins_total;
        bins_total += bins_bytes(r.dims);
        traj += v.n_traj;
        regs += r.capacity;
        p.max_traj = std::max<long long>(p.max_traj, v.n_traj);
        p.max_voxels = std::max<long long>(p.max_voxels, (long long)v.X * v.Y * v.Z);
        p.max_words = std::max<long long>(p.max_words, (long long)(v.xp / 4) * v.Y * v.Z);
        if (v.method == KS_MEANSHIFT) {
            p.max_tx = std::max(p.max_tx, (v.X + 63) / 64);
            p.max_ty = std::max(p.max_ty, (v.yp + 63) / 64);
            p.max_z = std::max(p.max_z, v.Z);
        }
        if (v.method == KS_QUADRANT) {
            p.maxS_quad = std::max(p.maxS_quad, v.S);
            p.maxB_quad = std::max(p.maxB_quad, v.B);
        } else {
            p.maxB_ms = std::max(p.maxB_ms, v.B);
        }
    }
    p.total_traj = traj;
    p.total_regions = regs;
    p.n_pad = next_pow2((unsigned long long)std::max<int64_t>(traj, 2));
    // Mean-shift scales per task: a task runs a seed's consecutive scales, each
    // starting from the previous one's first window; groups shorten the sweeps
    // but lengthen the tasks, so they are used only while the queue still holds
    // at least 16 tasks per resident wavefront.
    int G = ms_group;
    if (G <= 0 && p.maxB_ms > 0) {
        const int mb = std::max(p.maxB_ms, 2);
        const int rl = std::max(pick_ms_rl(mb, ms_rl_pref), pick_ms_rl(mb, ms_rl_small_pref));
        const long long resident = (long long)max_blocks_ms(((mb + 1) << rl) + 64, p.maxB_ms) * num_cu;
        auto tasks = [&](int g) {
            long long n = 0;
            for (const VolDesc& v : p.vols)
                if (v.method == KS_MEANSHIFT) n += (long long)v.gx * v.gy * v.gz * ((v.S + g - 1) / g);
            return n;
        };
        G = 1;
        while (G < 4 && tasks(G + 1) >= 16 * resident) ++G;
    }
    G = std::max(1, G);
    p.ms_group = G;
    // Task runs, longest windows first (largest-processing-time order).  The
    // mean-shift tasks go to one queue per XCD: each run's start positions are
    // cut into 2 x 2 x 2 boxes (halves of the grid along each axis; a seed list
    // into 8 ranges) and box k goes to XCD k's queue, so that the windows an XCD
    // works on at once lie in one part of the volume and share its L2; each
    // queue holds its runs longest windows first.
    struct Run { TaskSeg s; double cost; int method; int xcd; };
    std::vector<Run> runs;
    for (int i = 0; i < nvol; ++i) {
        const VolDesc& v = p.vols[i];
        const int64_t seeds = (int64_t)v.gx * v.gy * v.gz;
        if (seeds == 0) continue;
        Run r;
        r.s.task_begin = 0; r.s.count = seeds; r.s.vol = i; r.s.scale = 0; r.s.scale_hi = 0;
        r.s.bx = r.s.by = r.s.bz = 0; r.s.bw = v.gx; r.s.bh = v.gy;
        r.xcd = 0;
        if (v.method == KS_QUADRANT) {
            const double w = 2.0 * v.s_max + 2.0;
            r.cost = w * w * w;
            r.method = KS_QUADRANT;
            runs.push_back(r);
            continue;
        }
        r.method = KS_MEANSHIFT;
        // groups of G consecutive scales, the largest group first
        for (int hi = v.s_max; hi >= v.s_min; hi -= G) {
            const int lo = std::max(v.s_min, hi - G + 1);
            r.s.scale = lo;
            r.s.scale_hi = hi;
            r.cost = 0.0;
            for (int s = lo; s <= hi; ++s) {
                const double w = 2.0 * s + 1.0;
                r.cost += w * w * w;
            }
            const bool list = in[i].seeds != nullptr;
            for (int k = 0; k < kXcds; ++k) {
                Run b = r;
                b.xcd = k;
                int x0, x1, y0 = 0, y1 = v.gy, z0 = 0, z1 = v.gz;
                if (list) {  // a seed list: 8 ranges of the list
                    x0 = (int)((int64_t)v.gx * k / kXcds);
                    x1 = (int)((int64_t)v.gx * (k + 1) / kXcds);
                } else {
                    const int hx = (v.gx + 1) / 2, hy = (v.gy + 1) / 2, hz = (v.gz + 1) / 2;
                    x0 = (k & 1) ? hx : 0; x1 = (k & 1) ? v.gx : hx;
                    y0 = (k & 2) ? hy : 0; y1 = (k & 2) ? v.gy : hy;
                    z0 = (k & 4) ? hz : 0; z1 = (k & 4) ? v.gz : hz;
                }
                const int64_t n = (int64_t)(x1 - x0) * (y1 - y0) * (z1 - z0);
                if (n <= 0) continue;
                b.s.count = n;
                b.s.bx = x0; b.s.by = y0; b.s.bz = z0; b.s.bw = x1 - x0; b.s.bh = y1 - y0;
                runs.push_back(b);
            }
        }
    }
    std::stable_sort(runs.begin(), runs.end(), [](const Run& a, const Run& b) {
        if (a.xcd != b.xcd) return a.xcd < b.xcd;
        return a.cost > b.cost;
    });
    int next_q = 0;
    for (const Run& r : runs) {
        std::vector<TaskSeg>& segs = r.method == KS_QUADRANT ? p.segs_q : p.segs_m;
        long long& nt = r.method == KS_QUADRANT ? p.ntask_q : p.ntask_m;
        if (r.method == KS_MEANSHIFT)
            while (next_q <= r.xcd) p.xq_begin[next_q++] = nt;
        TaskSeg s = r.s;
        s.task_begin = nt;
        nt += s.count;
        segs.push_back(s);
    }
    while (next_q <= kXcds) p.xq_begin[next_q++] = p.ntask_m;
    p.ms_chunks = std::max(1, std::min(ms_chunks, kMaxMsChunks));
    // Device memory: descriptors, task segments and seed lists in one allocation
    // laid out as the host staging area, so that one copy uploads them; results
    // in one allocation laid out as the host copy, so that one copy downloads
    // them (regions, per-volume region counts, the counter block).
    ks_status st;
    const size_t vol_bytes = sizeof(VolDesc) * (size_t)nvol;
    // after the descriptors: the mean-shift queues of each launch, then the task segments
    const size_t seg_bytes = sizeof(XcdQueues) * kMaxMsChunks + sizeof(TaskSeg) * (p.segs_q.size() + p.segs_m.size() + 1);
    const size_t stage_bytes = vol_bytes + seg_bytes + sizeof(int32_t) * p.seed_ints;
    result_layout((size_t)nvol, regs, &p.out_nf_off, &p.out_cnt_off, &p.out_bytes);
    size_t need[kArenaBuffers];
    arena_needs(in, need);
    if (need[kArVols] < stage_bytes || need[kArBins] < bins_total || need[kArOut] != p.out_bytes)
        return KS_E_INVALID;  // arena_needs disagrees with the plan
    if (fixed) {
        // the caller's ranges: KS_E_TOO_LARGE if the plan does not fit them
        size_t off = 0;
        for (int i = 0; i < kArenaBuffers; ++i) {
            p.dev[i] = fixed->dev + off;
            off += (need[i] + 255) & ~(size_t)255;
        }
        if (off > fixed->dev_bytes || stage_bytes > fixed->stage_bytes || p.out_bytes > fixed->out_bytes)
            return KS_E_TOO_LARGE;
        p.stage = fixed->stage;
        p.hout = fixed->out;
    } else {
        for (int i = 0; i < kArenaBuffers; ++i) {
            if ((st = arena(i).ensure(need[i], &generation)) != KS_OK) return st;
            p.dev[i] = static_cast<char*>(arena(i).ptr);
        }
        // host staging (descriptors, segments, seed lists) and the result copy
        if ((st = h_stage.ensure(stage_bytes)) != KS_OK) return st;
        if ((st = h_out.ensure(p.out_bytes)) != KS_OK) return st;
        p.stage = static_cast<char*>(h_stage.ptr);
        p.hout = static_cast<char*>(h_out.ptr);
    }
    p.cnt = reinterpret_cast<Counters*>(p.dev[kArOut] + p.out_cnt_off);
    int* volint = reinterpret_cast<int*>(p.dev[kArVolInt]);
    for (int i = 0; i < nvol; ++i) {
        p.vols[i].bins = reinterpret_cast<uint8_t*>(p.dev[kArBins]) + bins_off[i];
        p.vols[i].bins_t = p.vols[i].bins + bins_x_bytes(in[i].dims);
        p.vols[i].minmax = volint + 2 * i;
        p.vols[i].seeds = in[i].seeds ? reinterpret_cast<const int32_t*>(p.dev[kArVols] + vol_bytes + seg_bytes) +
                                            p.seed_off[i]
                                      : nullptr;
    }
    p.seed_src.resize(nvol);
    for (int i = 0; i < nvol; ++i) p.seed_src[i] = in[i].seeds;
    p.vol_nfound = reinterpret_cast<int*>(p.dev[kArOut] + p.out_nf_off);
    p.vol_base = volint + 2 * nvol;
    p.rl = pick_ms_rl(std::max(p.maxB_ms, 2), ms_rl_pref);
    p.rl_small = pick_ms_rl(std::max(p.maxB_ms, 2), ms_rl_small_pref);
    p.rq = pick_quad_rq(std::max(p.maxS_quad, 1), std::max(p.maxB_quad, 2), quad_rq_pref);
    p.lay = quad_layout(std::max(p.maxS_quad, 1), std::max(p.maxB_quad, 2), p.rq);
    // bins of the larger layout plus one trash slot per replica
    p.ms_hist_words = ((std::max(p.maxB_ms, 2) + 1) << std::max(p.rl, p.rl_small)) + 64;
    return KS_OK;
}

// Writes the plan's tables into the pinned staging buffer and queues their upload.
ks_status Context::upload(const Plan& p, hipStream_t st) {
    char* h = p.stage;
    const size_t vol_bytes = sizeof(VolDesc) * (size_t)p.nvol;
    const size_t seg_bytes = sizeof(XcdQueues) * kMaxMsChunks + sizeof(TaskSeg) * (p.segs_q.size() + p.segs_m.size() + 1);
    std::memcpy(h, p.vols.data(), vol_bytes);
    // launch c takes part c of every XCD queue, in the queue's longest-first order
    XcdQueues* hq = reinterpret_cast<XcdQueues*>(h + vol_bytes);
    std::memset(hq, 0, sizeof(XcdQueues) * kMaxMsChunks);
    for (int c = 0; c < p.ms_chunks; ++c)
        for (int k = 0; k < kXcds; ++k) {
            const int64_t b = p.xq_begin[k], n = p.xq_begin[k + 1] - b;
            hq[c].begin[k] = b + n * c / p.ms_chunks;
            hq[c].end[k] = b + n * (c + 1) / p.ms_chunks;
        }
    TaskSeg* hs = reinterpret_cast<TaskSeg*>(h + vol_bytes + sizeof(XcdQueues) * kMaxMsChunks);
    size_t ns = 0;
    for (const TaskSeg& s : p.segs_q) hs[ns++] = s;
    for (const TaskSeg& s : p.segs_m) hs[ns++] = s;
    std::memset(hs + ns, 0, sizeof(TaskSeg));
    int32_t* hseed = reinterpret_cast<int32_t*>(h + vol_bytes + seg_bytes);
    for (int i = 0; i < p.nvol; ++i)
        if (p.seed_src[i])
            std::memcpy(hseed + p.seed_off[i], p.seed_src[i], sizeof(int32_t) * 3 * (size_t)p.vols[i].gx);
    KS_HIP(hipMemcpyAsync(p.dev[kArVols], h, vol_bytes + seg_bytes + sizeof(int32_t) * p.seed_ints,
                          hipMemcpyHostToDevice, st));
    return KS_OK;
}

// Records ev on st.  Inside a stream capture the record becomes an explicit
// event-record node after the stream's current capture dependencies (an event
// that hipEventRecord records during a capture cannot be timed after a replay
// on this runtime, while event-record nodes can).
static hipError_t mark(hipEvent_t ev, hipStream_t st) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &cs);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusActive) return hipEventRecord(ev, st);
    unsigned long long id = 0;
    hipGraph_t g = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    if ((e = hipStreamGetCaptureInfo_v2(st, &cs, &id, &g, &deps, &nd)) != hipSuccess) return e;
    hipGraphNode_t node;
    if ((e = hipGraphAddEventRecordNode(&node, g, deps, nd, ev)) != hipSuccess) return e;
    return hipStreamUpdateCaptureDependencies(st, &node, 1, hipStreamSetCaptureDependencies);
}

// The second stream of two-method calls, created on first use: streams share
// the device's few hardware queues round robin, so a context that never runs
// both methods at once takes none.
hipError_t Context::ensure_aux() {
    return aux ? hipSuccess : hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
}

ks_status Context::enqueue_search(const Plan& p, hipStream_t st, bool with_rank, bool timed) {
    VolDesc* dv = reinterpret_cast<VolDesc*>(p.dev[kArVols]);
    const XcdQueues* dxq = reinterpret_cast<const XcdQueues*>(p.dev[kArVols] + sizeof(VolDesc) * (size_t)p.nvol);
    TaskSeg* ds = reinterpret_cast<TaskSeg*>(p.dev[kArVols] + sizeof(VolDesc) * (size_t)p.nvol +
                                             sizeof(XcdQueues) * kMaxMsChunks);
    Counters* dc = p.cnt;
    TrajRec* rec = reinterpret_cast<TrajRec*>(p.dev[kArRec]);
    if (timed) KS_HIP(mark(ev[0], st));
    PrepArgs pa;
    pa.vols = dv; pa.nvol = p.nvol; pa.cnt = dc; pa.vol_nfound = p.vol_nfound; pa.vol_base = p.vol_base;
    pa.max_voxels = p.max_voxels; pa.max_words = p.max_words;
    pa.max_tx = p.max_tx; pa.max_ty = p.max_ty; pa.max_z = p.max_z;
    KS_HIP(launch_prep(pa, st));
    if (timed) KS_HIP(mark(ev[1], st));
    SearchArgs sq;
    sq.vols = dv; sq.segs = ds; sq.nseg = (int)p.segs_q.size(); sq.ntask = p.ntask_q; sq.tb = tables;
    sq.rec = rec; sq.cnt = dc;
    SearchArgs sm = sq;
    sm.segs = ds + p.segs_q.size(); sm.nseg = (int)p.segs_m.size(); sm.ntask = p.ntask_m;
    // with both methods and overlap on, the mean-shift search runs on the aux stream
    // beside the quadrant search, so that each fills the other's tail
    const bool fork = p.ntask_q > 0 && p.ntask_m > 0 && overlap;
    if (fork) KS_HIP(ensure_aux());
    hipStream_t sm_st = fork ? aux : st;
    if (fork) {
        KS_HIP(hipEventRecord(fork_ev, st));
        KS_HIP(hipStreamWaitEvent(aux, fork_ev, 0));
    }
    if (p.ntask_q > 0) {
        const int per_cu = max_blocks_quad(p.lay.bytes, p.maxB_quad);
        const long long g = std::min<long long>(p.ntask_q, std::max<long long>(1, (long long)per_cu * num_cu * grid_pct / 100));
        if (timed) KS_HIP(mark(ev[6], st));
        KS_HIP(launch_search_quad(sq, (int)g, p.rq, p.lay, p.maxB_quad, st));
        if (timed) KS_HIP(mark(ev[7], st));
    }
    if (p.ntask_m > 0) {
        const int per_cu = max_blocks_ms(p.ms_hist_words, p.maxB_ms);
        const long long g = std::min<long long>(p.ntask_m, std::max<long long>(1, (long long)per_cu * num_cu * grid_pct / 100));
        MsTune tune;
        tune.rl = p.rl;
        tune.rl_small = p.rl_small;
        tune.s_small = ms_s_small;
        tune.incr_pct = ms_incr_pct;
        tune.group = p.ms_group;
        tune.pad = 0;
        if (timed) KS_HIP(mark(ev[4], sm_st));
        for (int c = 0; c < p.ms_chunks; ++c)
            KS_HIP(launch_search_ms(sm, dxq + c, c, (int)g, tune, p.ms_hist_words, p.maxB_ms, sm_st));
        if (timed) KS_HIP(mark(ev[5], sm_st));
    }
    if (fork) {
        KS_HIP(hipEventRecord(join_ev, aux));
        KS_HIP(hipStreamWaitEvent(st, join_ev, 0));
    }
    if (timed) KS_HIP(mark(ev[2], st));
    if (with_rank) {
        RankArgs ra;
        ra.vols = dv; ra.nvol = p.nvol; ra.rec = rec; ra.sr = reinterpret_cast<SortRec*>(p.dev[kArSort]); ra.cnt = dc;
        ra.n_pad = p.n_pad; ra.max_traj = p.max_traj; ra.bsum = reinterpret_cast<int*>(p.dev[kArBsum]);
        ra.vol_base = p.vol_base; ra.vol_nfound = p.vol_nfound;
        ra.regions = reinterpret_cast<ks_region_dev*>(p.dev[kArOut]);
        KS_HIP(launch_rank(ra, st));
    }
    if (timed) KS_HIP(mark(ev[3], st));
    return KS_OK;
}

ks_status Context::download(const Plan& p, hipStream_t st) {
    KS_HIP(hipMemcpyAsync(p.hout, p.dev[kArOut], p.out_bytes, hipMemcpyDeviceToHost, st));
    return KS_OK;
}

void Context::collect_stats(const Plan& p, bool timed) {
    const char* h = p.hout;
    const int* nf = reinterpret_cast<const int*>(h + p.out_nf_off);
    Counters c;
    std::memcpy(&c, h + p.out_cnt_off, sizeof(Counters));
    std::memset(&last, 0, sizeof(last));
    last.trajectories = p.total_traj;
    last.evals = (int64_t)c.evals;
    last.window_evals = (int64_t)c.window_evals;
    last.voxel_visits = (int64_t)c.voxel_visits;
    last.final_visits = (int64_t)c.final_visits;
    last.swept_voxels = (int64_t)c.swept;
    last.lds_ops = (int64_t)c.lds_ops;
    for (int i = 0; i < p.nvol; ++i) last.regions += nf[i];
    if (timed) {
        float a = 0, b = 0, d = 0;
        hipEventElapsedTime(&a, ev[0], ev[1]);
        hipEventElapsedTime(&b, ev[1], ev[2]);
        hipEventElapsedTime(&d, ev[2], ev[3]);
        last.ms_prep = a; last.ms_search = b; last.ms_rank = d; last.ms_total = a + b + d;
        float m = 0, q = 0;
        if (p.ntask_m > 0) hipEventElapsedTime(&m, ev[4], ev[5]);
        if (p.ntask_q > 0) hipEventElapsedTime(&q, ev[6], ev[7]);
        last.ms_search_ms = m; last.ms_search_quad = q;
    }
}

ks_status Context::begin_detect(const std::vector<VolIn>& in, hipStream_t st, Plan& p) {
    KS_HIP(hipSetDevice(device));
    ks_status s = plan(in, p);
    if (s != KS_OK) return s;
    if ((s = upload(p, st)) != KS_OK) return s;
    if ((s = enqueue_search(p, st, true, profiling)) != KS_OK) return s;
    return download(p, st);
}

void Context::end_detect(const std::vector<VolIn>& in, const Plan& p, std::vector<std::vector<ks_region>>* out,
                         std::vector<int>* nfound) {
    collect_stats(p, profiling);
    const char* h = p.hout;
    const ks_region* regs = reinterpret_cast<const ks_region*>(h);
    const int* nf = reinterpret_cast<const int*>(h + p.out_nf_off);
    out->assign(in.size(), {});
    nfound->assign(in.size(), 0);
    for (size_t i = 0; i < in.size(); ++i) {
        (*nfound)[i] = nf[i];
        const int w = std::min(nf[i], in[i].capacity);
        (*out)[i].assign(regs + p.vols[i].reg_off, regs + p.vols[i].reg_off + w);
    }
}

ks_status Context::detect_volumes(const std::vector<VolIn>& in, hipStream_t st, std::vector<std::vector<ks_region>>* out,
                                  std::vector<int>* nfound) {
    Plan p;
    ks_status s = begin_detect(in, st, p);
    if (s != KS_OK) return s;
    KS_HIP(hipStreamSynchronize(st));
    end_detect(in, p, out, nfound);
    return KS_OK;
}


// Batched detection through a captured graph: the launch sequence of a batch
// with a given shape is captured once and replayed; only the small tables are
// re-uploaded before each replay.
ks_status Context::detect_batch_graph(const std::vector<VolIn>& in, hipStream_t st,
                                      std::vector<std::vector<ks_region>>* out, std::vector<int>* nfound) {
    KS_HIP(hipSetDevice(device));
    if (!st) {
        // The null stream cannot be captured: run on the context's own stream,
        // ordered after the work already queued on the null stream (which may be
        // writing the volumes).
        if (!batch_stream) KS_HIP(hipStreamCreateWithFlags(&batch_stream, hipStreamNonBlocking));
        KS_HIP(hipEventRecord(order_ev, nullptr));
        KS_HIP(hipStreamWaitEvent(batch_stream, order_ev, 0));
        st = batch_stream;
    }
    Plan p;
    ks_status s = plan(in, p);
    if (s != KS_OK) return s;
    // with profiling on, the graph also holds event-record nodes around the
    // phases and the searches
    const bool timed = profiling;
    std::vector<int64_t> key;
    key.push_back(generation);
    key.push_back(timed ? 1 : 0);
    key.push_back(ms_rl_pref);
    key.push_back(ms_rl_small_pref);
    key.push_back(ms_s_small);
    key.push_back(quad_rq_pref);
    key.push_back(overlap ? 1 : 0);
    key.push_back(p.ms_group);
    key.push_back(p.ms_chunks);
    for (const VolIn& v : in) {
        key.push_back((int64_t)(intptr_t)v.raw);
        key.push_back(v.dtype); key.push_back(v.dims[0]); key.push_back(v.dims[1]); key.push_back(v.dims[2]);
        key.push_back(v.bins); key.push_back(v.spacing); key.push_back(v.scales[0]); key.push_back(v.scales[1]);
        key.push_back(v.method); key.push_back(v.max_iter); key.push_back(v.capacity);
        int64_t hb, yb;
        std::memcpy(&hb, &v.opt.h_min, sizeof(hb));
        std::memcpy(&yb, &v.opt.y_min, sizeof(yb));
        key.push_back(hb); key.push_back(yb); key.push_back(v.opt.rank_by);
        key.push_back(v.seeds ? v.n_seeds : -1);
    }
    // the second stream of a two-method batch exists before the capture starts
    if (p.ntask_q > 0 && p.ntask_m > 0 && overlap) KS_HIP(ensure_aux());
    hipGraphExec_t exec = nullptr;
    for (const GraphEntry& g : graphs)
        if (g.key == key) exec = g.exec;
    if ((s = upload(p, st)) != KS_OK) return s;
    if (!exec) {
        hipGraph_t graph = nullptr;
        KS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        ks_status cs = enqueue_search(p, st, true, timed);
        if (cs == KS_OK) cs = download(p, st);
        hipError_t e = hipStreamEndCapture(st, &graph);
        if (cs != KS_OK) {
            if (graph) hipGraphDestroy(graph);
            return cs;
        }
        if (e != hipSuccess) return hip_fail(e);
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e);
        if (graphs.size() >= 8) {
            hipGraphExecDestroy(graphs.front().exec);
            graphs.erase(graphs.begin());
        }
        GraphEntry ge;
        ge.key = key;
        ge.exec = exec;
        graphs.push_back(ge);
    }
    KS_HIP(hipGraphLaunch(exec, st));
    KS_HIP(hipStreamSynchronize(st));
    collect_stats(p, timed);
    const char* h = p.hout;
    const ks_region* regs = reinterpret_cast<const ks_region*>(h);
    const int* nf = reinterpret_cast<const int*>(h + p.out_nf_off);
    out->assign(in.size(), {});
    nfound->assign(in.size(), 0);
    for (size_t i = 0; i < in.size(); ++i) {
        (*nfound)[i] = nf[i];
        const int w = std::min(nf[i], in[i].capacity);
        (*out)[i].assign(regs + p.vols[i].reg_off, regs + p.vols[i].reg_off + w);
    }
    return KS_OK;
}

}  // namespace ks

// ================================================================ C ABI

using namespace ks;

struct ks_context : public Context {};

extern "C" {

const char* ks_status_str(ks_status s) {
    switch (s) {
        case KS_OK: return "ok";
        case KS_E_INVALID: return "invalid argument";
        case KS_E_NOMEM: return "out of memory";
        case KS_E_DEVICE: return "device error";
        case KS_E_TOO_LARGE: return "request larger than the budget";
        case KS_E_NOT_READY: return "not ready";
        case KS_E_SHUTDOWN: return "shutting down";
    }
    return "unknown status";
}

ks_status ks_context_create(int32_t device, ks_context** out) {
    if (!out) return KS_E_INVALID;
    ks_context* c = new (std::nothrow) ks_context();
    if (!c) return KS_E_NOMEM;
    ks_status s = c->init(device);
    if (s != KS_OK) {
        c->destroy();
        delete c;
        return s;
    }
    *out = c;
    return KS_OK;
}

ks_status ks_context_destroy(ks_context* ctx) {
    if (!ctx) return KS_E_INVALID;
    ctx->destroy();
    delete ctx;
    return KS_OK;
}

ks_status ks_context_set_profiling(ks_context* ctx, int32_t on) {
    if (!ctx) return KS_E_INVALID;
    ctx->profiling = on != 0;
    return KS_OK;
}

ks_status ks_context_set_tuning(ks_context* ctx, int32_t ms_replicas_log2, int32_t quad_replicas_log2) {
    if (!ctx || ms_replicas_log2 < 2 || ms_replicas_log2 > 6 || quad_replicas_log2 < 0 || quad_replicas_log2 > 3)
        return KS_E_INVALID;
    ctx->ms_rl_pref = ms_replicas_log2;
    ctx->ms_rl_small_pref = ms_replicas_log2;
    ctx->quad_rq_pref = quad_replicas_log2;
    return KS_OK;
}

ks_status ks_context_set_tuning_small(ks_context* ctx, int32_t ms_small_replicas_log2, int32_t s_small) {
    if (!ctx || ms_small_replicas_log2 < 2 || ms_small_replicas_log2 > 6 || s_small < 0) return KS_E_INVALID;
    ctx->ms_rl_small_pref = ms_small_replicas_log2;
    ctx->ms_s_small = s_small;
    return KS_OK;
}

static ks_status apply_ctx_seeds(const ks_context* ctx, VolIn& v);

ks_status ks_context_autotune(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                              int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                              int32_t max_iter, int32_t reps, int32_t out[4], void* stream) {
    if (!ctx || reps < 1 || reps > 16) return KS_E_INVALID;
    ks_status s = check_request(d_volume, dtype, dims, bins, seed_spacing, scales, method, max_iter);
    if (s != KS_OK) return s;
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = seed_spacing; v.scales[0] = scales[0]; v.scales[1] = scales[1]; v.method = method;
    v.max_iter = max_iter; v.capacity = 1;
    v.opt = ctx->opts;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    if ((s = apply_ctx_seeds(ctx, v)) != KS_OK) return s;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const bool prof = ctx->profiling;
    ctx->profiling = true;
    // device time of the search launch under the context's current tuning: the
    // fastest of reps runs after a warm-up
    auto measure = [&](double* best) -> ks_status {
        std::vector<std::vector<ks_region>> res;
        std::vector<int> nf;
        *best = 1e30;
        for (int r = 0; r <= reps; ++r) {
            ks_status e = ctx->detect_volumes({v}, st, &res, &nf);
            if (e != KS_OK) return e;
            const double t = method == KS_MEANSHIFT ? ctx->last.ms_search_ms : ctx->last.ms_search_quad;
            if (r > 0 && t < *best) *best = t;
        }
        return KS_OK;
    };
    double t;
    if (method == KS_MEANSHIFT) {
        // large-window class first (the small class at its current setting), then the small class
        int best_rl = ctx->ms_rl_pref;
        double best_t = 1e30;
        for (int rl = 3; rl <= 5 && s == KS_OK; ++rl) {
            ctx->ms_rl_pref = rl;
            if ((s = measure(&t)) == KS_OK && t < best_t) { best_t = t; best_rl = rl; }
        }
        ctx->ms_rl_pref = best_rl;
        int best_rls = ctx->ms_rl_small_pref, best_ss = ctx->ms_s_small;
        for (int rls = 2; rls <= 3 && s == KS_OK; ++rls)
            for (int ss = 4; ss <= 8 && s == KS_OK; ss += 2) {
                ctx->ms_rl_small_pref = rls;
                ctx->ms_s_small = ss;
                if ((s = measure(&t)) == KS_OK && t < best_t) { best_t = t; best_rls = rls; best_ss = ss; }
            }
        ctx->ms_rl_small_pref = best_rls;
        ctx->ms_s_small = best_ss;
    } else {
        int best_rq = ctx->quad_rq_pref;
        double best_t = 1e30;
        for (int rq = 0; rq <= 2 && s == KS_OK; ++rq) {
            if (pick_quad_rq(scales[1] - scales[0] + 1, bins, rq) != rq) break;  // beyond the LDS budget
            ctx->quad_rq_pref = rq;
            if ((s = measure(&t)) == KS_OK && t < best_t) { best_t = t; best_rq = rq; }
        }
        ctx->quad_rq_pref = best_rq;
    }
    ctx->profiling = prof;
    if (s != KS_OK) return s;
    if (out) {
        out[0] = ctx->ms_rl_pref; out[1] = ctx->ms_rl_small_pref; out[2] = ctx->ms_s_small; out[3] = ctx->quad_rq_pref;
    }
    return KS_OK;
}

ks_status ks_context_set_options(ks_context* ctx, const ks_options* options) {
    if (!ctx) return KS_E_INVALID;
    if (!options) {
        ctx->opts = ks_options{};
        return KS_OK;
    }
    if (!options_ok(*options)) return KS_E_INVALID;
    ctx->opts = *options;
    return KS_OK;
}

ks_status ks_context_set_ms_update(ks_context* ctx, int32_t incremental_pct) {
    if (!ctx || incremental_pct < 0 || incremental_pct > 200) return KS_E_INVALID;
    ctx->ms_incr_pct = incremental_pct;
    return KS_OK;
}

ks_status ks_context_set_ms_group(ks_context* ctx, int32_t scales_per_task) {
    if (!ctx || scales_per_task < 0 || scales_per_task > 8) return KS_E_INVALID;
    ctx->ms_group = scales_per_task;
    return KS_OK;
}

ks_status ks_context_set_ms_chunks(ks_context* ctx, int32_t launches) {
    if (!ctx || launches < 1 || launches > kMaxMsChunks) return KS_E_INVALID;
    ctx->ms_chunks = launches;
    return KS_OK;
}

ks_status ks_context_set_overlap(ks_context* ctx, int32_t on) {
    if (!ctx || (on != 0 && on != 1)) return KS_E_INVALID;
    ctx->overlap = on != 0;
    return KS_OK;
}

ks_status ks_context_set_seeds(ks_context* ctx, const int32_t* seeds, int64_t n_seeds) {
    if (!ctx) return KS_E_INVALID;
    if (!seeds) {
        ctx->use_seeds = false;
        ctx->seeds.clear();
        return KS_OK;
    }
    if (n_seeds < 0 || n_seeds > (int64_t)INT32_MAX) return KS_E_INVALID;
    ctx->seeds.assign(seeds, seeds + 3 * n_seeds);
    ctx->use_seeds = true;
    return KS_OK;
}

// The context's seed list on a request, validated against its volume.
static ks_status apply_ctx_seeds(const ks_context* ctx, VolIn& v) {
    if (!ctx->use_seeds) return KS_OK;
    const int64_t n = (int64_t)ctx->seeds.size() / 3;
    // a non-null pointer even for an empty list
    static const int32_t kNone[3] = {0, 0, 0};
    v.seeds = n ? ctx->seeds.data() : kNone;
    v.n_seeds = n;
    return check_seeds(v.dims, v.scales, v.method, v.seeds, n);
}

ks_status ks_last_stats(ks_context* ctx, ks_run_stats* out) {
    if (!ctx || !out) return KS_E_INVALID;
    *out = ctx->last;
    return KS_OK;
}

static ks_status check_out(ks_region* out, int32_t capacity, int32_t* n_found) {
    if (!n_found || capacity < 0 || (capacity > 0 && !out)) return KS_E_INVALID;
    return KS_OK;
}

ks_status ks_detect_device(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                           int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                           int32_t max_iter, ks_region* out, int32_t capacity, int32_t* n_found, void* stream) {
    if (!ctx) return KS_E_INVALID;
    ks_status s = check_request(d_volume, dtype, dims, bins, seed_spacing, scales, method, max_iter);
    if (s != KS_OK) return s;
    if ((s = check_out(out, capacity, n_found)) != KS_OK) return s;
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = seed_spacing; v.scales[0] = scales[0]; v.scales[1] = scales[1]; v.method = method;
    v.max_iter = max_iter; v.capacity = capacity;
    v.opt = ctx->opts;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    if ((s = apply_ctx_seeds(ctx, v)) != KS_OK) return s;
    std::vector<std::vector<ks_region>> res;
    std::vector<int> nf;
    s = ctx->detect_volumes({v}, static_cast<hipStream_t>(stream), &res, &nf);
    if (s != KS_OK) return s;
    if (!res[0].empty()) std::memcpy(out, res[0].data(), sizeof(ks_region) * res[0].size());
    *n_found = nf[0];
    return KS_OK;
}

ks_status ks_detect_device_noalloc(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                                   int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                                   int32_t max_iter, ks_region* out, int32_t capacity, int32_t* n_found,
                                   void* stream) {
    if (!ctx) return KS_E_INVALID;
    ks_status s = check_request(d_volume, dtype, dims, bins, seed_spacing, scales, method, max_iter);
    if (s != KS_OK) return s;
    if ((s = check_out(out, capacity, n_found)) != KS_OK) return s;
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = seed_spacing; v.scales[0] = scales[0]; v.scales[1] = scales[1]; v.method = method;
    v.max_iter = max_iter; v.capacity = capacity;
    v.opt = ctx->opts;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    if ((s = apply_ctx_seeds(ctx, v)) != KS_OK) return s;
    if (!ctx->scratch) return KS_E_DEVICE;
    // the arena in the device's static array; the host copies in pageable memory
    size_t need[kArenaBuffers];
    arena_needs({v}, need);
    size_t dev_bytes = 0;
    for (int i = 0; i < kArenaBuffers; ++i) dev_bytes += (need[i] + 255) & ~(size_t)255;
    if (dev_bytes > kScratchBytes) return KS_E_TOO_LARGE;
    std::vector<char> stage(need[kArVols]), hout(need[kArOut]);
    const FixedArena fx = {ctx->scratch, kScratchBytes, stage.data(), stage.size(), hout.data(), hout.size()};
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return KS_E_DEVICE;
    Plan p;
    if ((s = ctx->plan({v}, p, &fx)) != KS_OK) return s;
    if ((s = ctx->upload(p, st)) != KS_OK) return s;
    if ((s = ctx->enqueue_search(p, st, true, ctx->profiling)) != KS_OK) return s;
    if ((s = ctx->download(p, st)) != KS_OK) return s;
    if (hipStreamSynchronize(st) != hipSuccess) return KS_E_DEVICE;
    ctx->collect_stats(p, ctx->profiling);
    const int nf = *reinterpret_cast<const int*>(p.hout + p.out_nf_off);
    const int w = std::min(nf, capacity);
    if (w > 0) std::memcpy(out, p.hout, sizeof(ks_region) * (size_t)w);
    *n_found = nf;
    return KS_OK;
}

static std::mutex g_default_mu;
static ks_context* g_default = nullptr;

ks_status ks_detect(const void* volume, ks_dtype dtype, const int32_t dims[3], int32_t bins, int32_t seed_spacing,
                    const int32_t scales[2], ks_method method, int32_t max_iter, ks_region* out, int32_t capacity,
                    int32_t* n_found) {
    ks_status s = check_request(volume, dtype, dims, bins, seed_spacing, scales, method, max_iter);
    if (s != KS_OK) return s;
    if ((s = check_out(out, capacity, n_found)) != KS_OK) return s;
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default) {
        s = ks_context_create(0, &g_default);
        if (s != KS_OK) return s;
    }
    hipSetDevice(g_default->device);
    const size_t esz = dtype == KS_U8 ? 1 : 2;
    const size_t bytes = esz * (size_t)dims[0] * dims[1] * dims[2];
    if ((s = g_default->d_raw.ensure(bytes, &g_default->generation)) != KS_OK) return s;
    if (hipMemcpy(g_default->d_raw.ptr, volume, bytes, hipMemcpyHostToDevice) != hipSuccess) return KS_E_DEVICE;
    return ks_detect_device(g_default, g_default->d_raw.ptr, dtype, dims, bins, seed_spacing, scales, method,
                            max_iter, out, capacity, n_found, nullptr);
}

ks_status ks_seed_traces(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3],
                         int32_t bins, int32_t seed_spacing, const int32_t scales[2], ks_method method,
                         int32_t max_iter, ks_seed_trace* out, int32_t capacity, int32_t* n, void* stream) {
    if (!ctx) return KS_E_INVALID;
    ks_status s = check_request(d_volume, dtype, dims, bins, seed_spacing, scales, method, max_iter);
    if (s != KS_OK) return s;
    if (!n || capacity < 0 || (capacity > 0 && !out)) return KS_E_INVALID;
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = seed_spacing; v.scales[0] = scales[0]; v.scales[1] = scales[1]; v.method = method;
    v.max_iter = max_iter; v.capacity = 0;
    v.opt = ctx->opts;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    if ((s = apply_ctx_seeds(ctx, v)) != KS_OK) return s;
    if (capacity == 0) {  // count only
        *n = (int32_t)num_trajectories(v);
        return KS_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return KS_E_DEVICE;
    Plan p;
    if ((s = ctx->plan({v}, p)) != KS_OK) return s;
    if ((s = ctx->upload(p, st)) != KS_OK) return s;
    if ((s = ctx->enqueue_search(p, st, false, false)) != KS_OK) return s;
    std::vector<TrajRec> rec((size_t)p.total_traj);
    if (!rec.empty() && hipMemcpyAsync(rec.data(), p.dev[kArRec], sizeof(TrajRec) * rec.size(),
                                       hipMemcpyDeviceToHost, st) != hipSuccess)
        return KS_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return KS_E_DEVICE;
    const int64_t w = std::min<int64_t>(capacity, p.total_traj);
    for (int64_t i = 0; i < w; ++i) {
        const TrajRec& r = rec[(size_t)i];
        ks_seed_trace& t = out[i];
        t.x0 = r.x0; t.y0 = r.y0; t.z0 = r.z0; t.x = r.x; t.y = r.y; t.z = r.z;
        t.scale = r.scale; t.iters = r.iters; t.stop = r.stop; t.keep = r.keep;
        t.objective = r.objective; t.saliency64 = r.y64;
        t.saliency = r.y32; t.entropy = r.h32; t.pdf_change = r.w32; t.pad = 0;
    }
    *n = (int32_t)p.total_traj;
    return KS_OK;
}

ks_status ks_bin_volume(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3], int32_t bins,
                        uint8_t* out, void* stream) {
    if (!ctx || !out) return KS_E_INVALID;
    const int32_t sc[2] = {1, 1};
    ks_status s = check_request(d_volume, dtype, dims, bins, 1, sc, KS_QUADRANT, 0);
    if (s != KS_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return KS_E_DEVICE;
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = 1 << 20; v.scales[0] = 1; v.scales[1] = 1; v.method = KS_QUADRANT; v.max_iter = 0; v.capacity = 0;
    v.opt.window = ctx->opts.window; v.opt.win_lo = ctx->opts.win_lo; v.opt.win_hi = ctx->opts.win_hi;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    Plan p;
    if ((s = ctx->plan({v}, p)) != KS_OK) return s;
    if ((s = ctx->upload(p, st)) != KS_OK) return s;
    PrepArgs pa;
    pa.vols = reinterpret_cast<VolDesc*>(p.dev[kArVols]); pa.nvol = 1; pa.cnt = p.cnt;
    pa.vol_nfound = p.vol_nfound; pa.vol_base = p.vol_base; pa.max_voxels = p.max_voxels; pa.max_words = p.max_words;
    pa.max_tx = p.max_tx; pa.max_ty = p.max_ty; pa.max_z = p.max_z;
    if (launch_prep(pa, st) != hipSuccess) return KS_E_DEVICE;
    const VolDesc& d = p.vols[0];
    if (hipMemcpy2DAsync(out, (size_t)d.X, d.bins, (size_t)d.xp, (size_t)d.X, (size_t)d.Y * d.Z,
                         hipMemcpyDeviceToHost, st) != hipSuccess)
        return KS_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return KS_E_DEVICE;
    return KS_OK;
}

ks_status ks_saliency_map(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3], int32_t bins,
                          const int32_t scales[2], float* d_saliency, uint8_t* d_scale, void* stream) {
    if (!ctx || !d_saliency || !d_scale) return KS_E_INVALID;
    ks_status s = check_request(d_volume, dtype, dims, bins, 1, scales, KS_QUADRANT, 0);
    if (s != KS_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return KS_E_DEVICE;
    // prep as for a mean-shift volume (the map's column sweeps read the y-fast copy)
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = 1 << 20; v.scales[0] = scales[0]; v.scales[1] = scales[1]; v.method = KS_MEANSHIFT;
    v.max_iter = 0; v.capacity = 0;
    v.opt.window = ctx->opts.window; v.opt.win_lo = ctx->opts.win_lo; v.opt.win_hi = ctx->opts.win_hi;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    Plan p;
    if ((s = ctx->plan({v}, p)) != KS_OK) return s;
    if ((s = ctx->upload(p, st)) != KS_OK) return s;
    PrepArgs pa;
    pa.vols = reinterpret_cast<VolDesc*>(p.dev[kArVols]); pa.nvol = 1; pa.cnt = p.cnt;
    pa.vol_nfound = p.vol_nfound; pa.vol_base = p.vol_base; pa.max_voxels = p.max_voxels; pa.max_words = p.max_words;
    pa.max_tx = p.max_tx; pa.max_ty = p.max_ty; pa.max_z = p.max_z;
    if (ctx->profiling) KS_HIP(hipEventRecord(ctx->ev[0], st));
    if (launch_prep(pa, st) != hipSuccess) return KS_E_DEVICE;
    const int K = scales[1] - scales[0] + 3;
    const long long rows = (long long)dims[1] * dims[2];
    const int grid = (int)std::min<long long>(rows, (long long)max_blocks_map(K, bins) * ctx->num_cu);
    if (ctx->profiling) KS_HIP(hipEventRecord(ctx->ev[1], st));
    if (launch_saliency_map(reinterpret_cast<VolDesc*>(p.dev[kArVols]), ctx->tables, d_saliency, d_scale,
                            p.cnt, K, bins, grid, st) != hipSuccess)
        return KS_E_DEVICE;
    if (ctx->profiling) KS_HIP(hipEventRecord(ctx->ev[2], st));
    Counters c;
    if (hipMemcpyAsync(&c, p.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st) != hipSuccess)
        return KS_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return KS_E_DEVICE;
    std::memset(&ctx->last, 0, sizeof(ctx->last));
    ctx->last.trajectories = (int64_t)dims[0] * dims[1] * dims[2];
    ctx->last.lds_ops = (int64_t)c.lds_ops;
    if (ctx->profiling) {
        float a = 0, b = 0;
        hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]);
        hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]);
        ctx->last.ms_prep = a; ctx->last.ms_search = b; ctx->last.ms_total = a + b;
    }
    return KS_OK;
}

ks_status ks_abmsod(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3], int32_t bins,
                    int32_t seed_spacing, const int32_t radii[2], int32_t max_iter, double threshold,
                    ks_ellipsoid* out, int32_t capacity, int32_t* n, void* stream) {
    if (!ctx || !n || capacity < 0 || (capacity > 0 && !out) || threshold != threshold) return KS_E_INVALID;
    ks_status s = check_request(d_volume, dtype, dims, bins, seed_spacing, radii, KS_MEANSHIFT, max_iter);
    if (s != KS_OK) return s;
    // prep as a quadrant volume (no y-fast copy); one start per seed
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = seed_spacing; v.scales[0] = radii[0]; v.scales[1] = radii[1]; v.method = KS_QUADRANT;
    v.max_iter = 0; v.capacity = 0;
    v.opt.window = ctx->opts.window; v.opt.win_lo = ctx->opts.win_lo; v.opt.win_hi = ctx->opts.win_hi;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    if ((s = apply_ctx_seeds(ctx, v)) != KS_OK) return s;
    const int R = radii[1] - radii[0] + 1;
    const int64_t n_start = num_trajectories(v);
    if (n_start * R > (int64_t)INT32_MAX) return KS_E_INVALID;
    const int64_t total = n_start * R;
    if (capacity == 0) {  // count only
        *n = (int32_t)total;
        return KS_OK;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return KS_E_DEVICE;
    Plan p;
    if ((s = ctx->plan({v}, p)) != KS_OK) return s;
    if ((s = ctx->d_abm.ensure(sizeof(ks_ellipsoid) * (size_t)std::max<int64_t>(total, 1), &ctx->generation)) != KS_OK)
        return s;
    if ((s = ctx->upload(p, st)) != KS_OK) return s;
    PrepArgs pa;
    pa.vols = reinterpret_cast<VolDesc*>(p.dev[kArVols]); pa.nvol = 1; pa.cnt = p.cnt;
    pa.vol_nfound = p.vol_nfound; pa.vol_base = p.vol_base; pa.max_voxels = p.max_voxels; pa.max_words = p.max_words;
    pa.max_tx = p.max_tx; pa.max_ty = p.max_ty; pa.max_z = p.max_z;
    if (ctx->profiling) KS_HIP(hipEventRecord(ctx->ev[0], st));
    if (launch_prep(pa, st) != hipSuccess) return KS_E_DEVICE;
    if (ctx->profiling) KS_HIP(hipEventRecord(ctx->ev[1], st));
    if (total > 0) {
        AbmArgs a;
        a.n_start = n_start; a.R = R; a.r_min = radii[0]; a.r_max = radii[1]; a.max_iter = max_iter;
        a.replicas = abmsod_replicas(bins);
        a.threshold = threshold;
        const int grid = (int)std::min<int64_t>(total, (int64_t)abmsod_blocks_per_cu() * ctx->num_cu);
        if (launch_abmsod(reinterpret_cast<VolDesc*>(p.dev[kArVols]), a, bins, grid,
                          static_cast<ks_ellipsoid*>(ctx->d_abm.ptr), p.cnt,
                          st) != hipSuccess)
            return KS_E_DEVICE;
    }
    if (ctx->profiling) KS_HIP(hipEventRecord(ctx->ev[2], st));
    const int64_t w = std::min<int64_t>(capacity, total);
    if (w > 0 && hipMemcpyAsync(out, ctx->d_abm.ptr, sizeof(ks_ellipsoid) * (size_t)w, hipMemcpyDeviceToHost, st) !=
                     hipSuccess)
        return KS_E_DEVICE;
    Counters c;
    if (hipMemcpyAsync(&c, p.cnt, sizeof(Counters), hipMemcpyDeviceToHost, st) != hipSuccess)
        return KS_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return KS_E_DEVICE;
    std::memset(&ctx->last, 0, sizeof(ctx->last));
    ctx->last.trajectories = total;
    ctx->last.evals = (int64_t)c.evals;
    ctx->last.window_evals = (int64_t)c.evals;
    ctx->last.voxel_visits = (int64_t)c.voxel_visits;
    if (ctx->profiling) {
        float a0 = 0, b0 = 0;
        hipEventElapsedTime(&a0, ctx->ev[0], ctx->ev[1]);
        hipEventElapsedTime(&b0, ctx->ev[1], ctx->ev[2]);
        ctx->last.ms_prep = a0; ctx->last.ms_search = b0; ctx->last.ms_total = a0 + b0;
    }
    *n = (int32_t)total;
    return KS_OK;
}

ks_status ks_histograms(ks_context* ctx, const void* d_volume, ks_dtype dtype, const int32_t dims[3], int32_t bins,
                        int32_t kind, const int32_t range[2], int32_t n, const int32_t* xyz, const int32_t* scale,
                        void* out, void* stream) {
    if (!ctx || !out || n < 0 || (n > 0 && !xyz)) return KS_E_INVALID;
    if (kind < KS_HIST_CUBE || kind > KS_HIST_MS_INNER) return KS_E_INVALID;
    const int32_t sc[2] = {1, 1};
    ks_status s = check_request(d_volume, dtype, dims, bins, 1, sc, KS_QUADRANT, 0);
    if (s != KS_OK) return s;
    const bool per_window = kind != KS_HIST_OCTANTS && kind != KS_HIST_SHELLS;
    const int stride = kind == KS_HIST_MS_MOVE ? 6 : 3;
    if (per_window && n > 0 && !scale) return KS_E_INVALID;
    if (!per_window && (!range || range[0] < 0 || range[0] > range[1] || range[1] > kSmaxLimit + 1))
        return KS_E_INVALID;
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < stride; ++a)
            if (xyz[stride * i + a] < 0 || xyz[stride * i + a] >= dims[a % 3]) return KS_E_INVALID;
        if (per_window && (scale[i] < 1 || scale[i] > kSmaxLimit)) return KS_E_INVALID;
    }
    if (n == 0) return KS_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return KS_E_DEVICE;
    VolIn v;
    v.raw = d_volume; v.dtype = dtype; std::memcpy(v.dims, dims, sizeof(v.dims)); v.bins = bins;
    v.spacing = 1 << 20; v.scales[0] = 1; v.scales[1] = 1;
    v.method = per_window ? KS_MEANSHIFT : KS_QUADRANT; v.max_iter = 0; v.capacity = 0;
    v.opt.window = ctx->opts.window; v.opt.win_lo = ctx->opts.win_lo; v.opt.win_hi = ctx->opts.win_hi;
    if (!options_fit(v.opt, bins)) return KS_E_INVALID;
    Plan p;
    if ((s = ctx->plan({v}, p)) != KS_OK) return s;
    if ((s = ctx->upload(p, st)) != KS_OK) return s;
    PrepArgs pa;
    pa.vols = reinterpret_cast<VolDesc*>(p.dev[kArVols]); pa.nvol = 1; pa.cnt = p.cnt;
    pa.vol_nfound = p.vol_nfound; pa.vol_base = p.vol_base; pa.max_voxels = p.max_voxels; pa.max_words = p.max_words;
    pa.max_tx = p.max_tx; pa.max_ty = p.max_ty; pa.max_z = p.max_z;
    if (launch_prep(pa, st) != hipSuccess) return KS_E_DEVICE;
    const size_t in_bytes = sizeof(int32_t) * (size_t)(stride + 1) * (size_t)n;
    if ((s = ctx->d_hook.ensure(in_bytes, &ctx->generation)) != KS_OK) return s;
    std::vector<int32_t> hin((size_t)(stride + 1) * n);
    std::memcpy(hin.data(), xyz, sizeof(int32_t) * (size_t)stride * (size_t)n);
    if (per_window) std::memcpy(hin.data() + (size_t)stride * n, scale, sizeof(int32_t) * (size_t)n);
    if (hipMemcpyAsync(ctx->d_hook.ptr, hin.data(), in_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
        return KS_E_DEVICE;
    const int32_t* dxyz = static_cast<const int32_t*>(ctx->d_hook.ptr);
    const int32_t* dsc = dxyz + (size_t)stride * n;
    const int K = per_window ? 1 : range[1] - range[0] + 1;
    size_t out_bytes;
    if (kind == KS_HIST_CUBE) out_bytes = sizeof(uint32_t) * (size_t)n * bins;
    else if (kind == KS_HIST_MEANSHIFT || kind == KS_HIST_MS_MOVE) out_bytes = sizeof(int32_t) * (size_t)n * 4 * bins;
    else if (kind == KS_HIST_MS_INNER) out_bytes = sizeof(uint32_t) * (size_t)n * 3 * bins;
    else if (kind == KS_HIST_OCTANTS) out_bytes = sizeof(uint32_t) * (size_t)n * 8 * K * bins;
    else out_bytes = sizeof(uint32_t) * (size_t)n * K * bins;
    if ((s = ctx->d_hook_out.ensure(out_bytes, &ctx->generation)) != KS_OK) return s;
    hipError_t e;
    if (per_window) {
        const int rl = pick_ms_rl(bins, ctx->ms_rl_pref);
        const int hook_kind = kind == KS_HIST_CUBE ? 0 : kind == KS_HIST_MEANSHIFT ? 1 : kind == KS_HIST_MS_MOVE ? 2 : 3;
        e = launch_hook_ms(reinterpret_cast<VolDesc*>(p.dev[kArVols]), hook_kind, n, dxyz, dsc, rl,
                           ((bins + 1) << rl) + 64, bins, ctx->d_hook_out.ptr, st);
    } else {
        const int rq = pick_quad_rq(K, bins, ctx->quad_rq_pref);
        const LdsQuad lay = quad_layout(K, bins, rq);
        e = launch_hook_quad(reinterpret_cast<VolDesc*>(p.dev[kArVols]), kind, range[0], range[1], n, dxyz, rq, lay,
                             static_cast<uint32_t*>(ctx->d_hook_out.ptr), st);
    }
    if (e != hipSuccess) return KS_E_DEVICE;
    if (hipMemcpyAsync(out, ctx->d_hook_out.ptr, out_bytes, hipMemcpyDeviceToHost, st) != hipSuccess)
        return KS_E_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return KS_E_DEVICE;
    return KS_OK;
}

ks_status ks_count_roots(ks_context* ctx, int32_t n, double* sq, double* rsq, void* stream) {
    if (!ctx || !sq || !rsq || n < 1 || n > (1 << 24)) return KS_E_INVALID;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return KS_E_DEVICE;
    const size_t bytes = (size_t)n * sizeof(double);
    ks_status s = ctx->d_hook_out.ensure(2 * bytes, &ctx->generation);
    if (s != KS_OK) return s;
    double* d = static_cast<double*>(ctx->d_hook_out.ptr);
    if (launch_count_roots(n, d, d + n, st) != hipSuccess) return KS_E_DEVICE;
    if (hipMemcpyAsync(sq, d, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(rsq, d + n, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return KS_E_DEVICE;
    return KS_OK;
}

// The batch requests as runtime volumes (capacity: of each result, or 1).
static ks_status batch_volumes(int32_t n, const ks_request* reqs, const ks_result* results, std::vector<VolIn>& in) {
    in.assign((size_t)n, VolIn{});
    for (int i = 0; i < n; ++i) {
        const ks_request& r = reqs[i];
        ks_status s = check_request(r.volume, r.dtype, r.dims, r.bins, r.seed_spacing, r.scales, r.method, r.max_iter);
        if (s != KS_OK) return s;
        if (results && (results[i].capacity < 0 || (results[i].capacity > 0 && !results[i].regions)))
            return KS_E_INVALID;
        if (!options_ok(r.options) || !options_fit(r.options, r.bins)) return KS_E_INVALID;
        VolIn& v = in[(size_t)i];
        v.raw = r.volume; v.dtype = r.dtype; std::memcpy(v.dims, r.dims, sizeof(v.dims)); v.bins = r.bins;
        v.spacing = r.seed_spacing; v.scales[0] = r.scales[0]; v.scales[1] = r.scales[1]; v.method = r.method;
        v.max_iter = r.max_iter; v.capacity = results ? results[i].capacity : 1;
        v.opt = r.options;
        if (r.seeds || r.n_seeds) {
            if ((s = check_seeds(r.dims, r.scales, r.method, r.seeds, r.n_seeds)) != KS_OK) return s;
            v.seeds = r.seeds;
            v.n_seeds = r.n_seeds;
        }
    }
    return KS_OK;
}

ks_status ks_context_autotune_batch(ks_context* ctx, int32_t n, const ks_request* reqs, int32_t reps, int32_t out[5],
                                    void* stream) {
    if (!ctx || n < 1 || !reqs || reps < 1 || reps > 16) return KS_E_INVALID;
    std::vector<VolIn> in;
    ks_status s = batch_volumes(n, reqs, nullptr, in);
    if (s != KS_OK) return s;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const bool prof = ctx->profiling;
    ctx->profiling = true;
    // device time of the batch's launch sequence (prep, searches, ranking) under
    // the context's current tuning: the fastest of reps runs after a warm-up
    auto measure = [&](double* best) -> ks_status {
        std::vector<std::vector<ks_region>> res;
        std::vector<int> nf;
        *best = 1e30;
        for (int r = 0; r <= reps; ++r) {
            ks_status e = ctx->detect_volumes(in, st, &res, &nf);
            if (e != KS_OK) return e;
            if (r > 0 && ctx->last.ms_total < *best) *best = ctx->last.ms_total;
        }
        return KS_OK;
    };
    bool has_ms = false, has_q = false;
    int maxS_q = 1, maxB_q = 2;
    for (const VolIn& v : in) {
        if (v.method == KS_MEANSHIFT) has_ms = true;
        else {
            has_q = true;
            maxS_q = std::max(maxS_q, v.scales[1] - v.scales[0] + 1);
            maxB_q = std::max(maxB_q, v.bins);
        }
    }
    // one parameter at a time, each kept at its best before the next
    double best = 1e30, t;
    auto tryv = [&](int* knob, int value) {
        if (s != KS_OK) return;
        const int old = *knob;
        *knob = value;
        if ((s = measure(&t)) != KS_OK) return;
        if (t < best) best = t;
        else *knob = old;
    };
    s = measure(&best);
    if (has_ms) {
        const int base_rl = ctx->ms_rl_pref, base_rls = ctx->ms_rl_small_pref, base_ss = ctx->ms_s_small;
        for (int rl = 3; rl <= 5; ++rl) if (rl != base_rl) tryv(&ctx->ms_rl_pref, rl);
        for (int rls = 2; rls <= 3; ++rls) if (rls != base_rls) tryv(&ctx->ms_rl_small_pref, rls);
        for (int ss = 4; ss <= 8; ss += 2) if (ss != base_ss) tryv(&ctx->ms_s_small, ss);
        const int base_g = ctx->ms_group;
        for (int g = 0; g <= 4; ++g) if (g != base_g) tryv(&ctx->ms_group, g);
    }
    if (has_q) {
        const int base_rq = ctx->quad_rq_pref;
        for (int rq = 0; rq <= 2; ++rq)
            if (rq != base_rq && pick_quad_rq(maxS_q, maxB_q, rq) == rq) tryv(&ctx->quad_rq_pref, rq);
    }
    ctx->profiling = prof;
    if (s != KS_OK) return s;
    if (out) {
        out[0] = ctx->ms_rl_pref; out[1] = ctx->ms_rl_small_pref; out[2] = ctx->ms_s_small; out[3] = ctx->quad_rq_pref;
        out[4] = ctx->ms_group;
    }
    return KS_OK;
}

ks_status ks_detect_batch(ks_context* ctx, int32_t n, const ks_request* reqs, ks_result* results, void* stream) {
    if (!ctx || n < 0 || (n > 0 && (!reqs || !results))) return KS_E_INVALID;
    std::vector<VolIn> in;
    ks_status bs = batch_volumes(n, reqs, results, in);
    if (bs != KS_OK) return bs;
    if (n == 0) return KS_OK;
    std::vector<std::vector<ks_region>> res;
    std::vector<int> nf;
    ks_status s = ctx->detect_batch_graph(in, static_cast<hipStream_t>(stream), &res, &nf);
    if (s != KS_OK) return s;
    for (int i = 0; i < n; ++i) {
        if (!res[(size_t)i].empty())
            std::memcpy(results[i].regions, res[(size_t)i].data(), sizeof(ks_region) * res[(size_t)i].size());
        results[i].n_found = nf[(size_t)i];
        results[i].status = KS_OK;
    }
    return KS_OK;
}

}  // extern "C"

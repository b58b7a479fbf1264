// Continuous-batching detection server.
//
// A scheduler thread owns the GPU work.  Each tick it admits, oldest first, the
// pending requests whose device memory fits beside the busy slots' within the
// HBM budget, up to about ten milliseconds of estimated device work, groups them
// into one batched launch sequence on a free slot (own context and stream), and
// retires slots whose completion event has fired.  Several slots are in flight at once, so the
// next batch's upload and launch overlap the current one and its blocks fill
// the device as the current launch's tail drains.  A
// request's result does not depend on what it was batched with: every trajectory
// is computed independently and ranked within its own volume.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ks.h"
#include "ks_runtime.h"

namespace {

using Clock = std::chrono::steady_clock;

double now_ms() {
    return std::chrono::duration<double, std::milli>(Clock::now().time_since_epoch()).count();
}

struct SrvReq {
    ks::VolIn in;
    void* host = nullptr;          // pinned copy of the submitted volume (from the server's pool)
    size_t host_bytes = 0, host_cap = 0;
    size_t footprint = 0;          // device bytes it needs alone, at most
    double work = 0;               // estimated voxel visits
    double t_submit = 0, t_done = 0;
    int status = KS_E_NOT_READY;
    std::vector<ks_region> regions;
    int n_found = 0;
    std::vector<int32_t> seeds;    // own start positions, or those handed over by the track
    bool own_seeds = false;
    int64_t track = -1;            // tracked sequence, or -1
    int32_t max_seeds = 0;
};

// A tracked sequence: whether a frame is admitted and not yet complete, and the
// start positions its next frame takes (empty: the frame's own seeds or grid).
struct Track {
    bool busy = false;
    std::vector<int32_t> seeds;
};

// Pinned host buffers for the submitted volumes, reused across requests: a
// volume is copied once, at submit, and uploaded from there by DMA.  At most
// kPoolCache bytes of free buffers are kept.
class PinnedPool {
  public:
    static constexpr size_t kPoolCache = (size_t)2 << 30;
    void* get(size_t bytes, size_t* cap) {
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = free_.lower_bound(bytes);
            if (it != free_.end() && it->first <= 2 * bytes + 4096) {
                void* p = it->second;
                *cap = it->first;
                cached_ -= it->first;
                free_.erase(it);
                return p;
            }
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, std::max<size_t>(bytes, 1), hipHostMallocDefault) != hipSuccess) return nullptr;
        *cap = std::max<size_t>(bytes, 1);
        return p;
    }
    void put(void* p, size_t cap) {
        if (!p) return;
        {
            std::lock_guard<std::mutex> lk(mu_);
            if (cached_ + cap <= kPoolCache) {
                free_.emplace(cap, p);
                cached_ += cap;
                return;
            }
        }
        hipHostFree(p);
    }
    ~PinnedPool() {
        for (auto& f : free_) hipHostFree(f.second);
    }

  private:
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    size_t cached_ = 0;
};

struct Slot {
    ks::Context ctx;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    ks::Buffer raw;                // device copies of the batch's volumes
    std::vector<uint64_t> tickets;
    std::vector<ks::VolIn> in;
    ks::Plan plan;
    bool busy = false;
    bool large = false;            // the batch is one large request
    // device bytes held for requests: the context's per-call arena and the volumes
    size_t held() { return ctx.arena_held() + raw.cap; }
    void release() {
        ctx.arena_release();
        raw.release();
    }
};

const int32_t kNoSeeds[3] = {0, 0, 0};  // an empty start list (not the grid)

}  // namespace

struct ks_server {
    int device = 0;
    size_t budget = 0;
    int max_slots = 1;
    std::mutex mu;
    std::condition_variable cv;
    std::condition_variable done_cv;
    std::thread worker;
    bool stop = false;
    ks_status fatal = KS_OK;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> pending;
    std::map<uint64_t, SrvReq> reqs;
    std::map<int64_t, Track> tracks;
    std::vector<Slot*> slots;
    PinnedPool pool;
    size_t in_use = 0, peak = 0;   // device bytes the slots hold for requests
    int64_t submitted = 0, admitted = 0, completed = 0, refused = 0, in_flight = 0;
    double first_submit = -1, last_done = 0;
    std::vector<double> latencies;
    bool ready = false;
    ks_status init_status = KS_OK;

    void run();
    bool tick();
    void account();
    ks_status submit(const ks_request* req, int64_t track, int32_t max_seeds, uint64_t* ticket);
};

// Device bytes a request holds while it runs alone on a slot: its volume copy
// and the per-call arena of its plan.
static size_t request_bytes(const ks::VolIn& v, size_t host_bytes) {
    return ks::Context::arena_fresh({v}) + ks::granule((host_bytes + 255) & ~(size_t)255);
}

static double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

// Estimated voxel visits of a request's search: seeds x the window voxels of one
// evaluation round x a typical evaluation count per trajectory.  Used only to
// bound a batch's work so that results come back in pieces of a few ms of device
// time instead of one long launch.
static double work_estimate(const ks::VolIn& v, int64_t n_seeds) {
    const double seeds = (double)n_seeds;
    double win = 0;
    if (v.method == KS_QUADRANT) {
        const double w = 2.0 * v.scales[1] + 1.0;
        win = 5.0 * w * w * w;
    } else {
        for (int s = v.scales[0]; s <= v.scales[1]; ++s) {
            const double w = 2.0 * s + 1.0;
            win += 6.0 * w * w * w;
        }
    }
    const double vox = (double)v.dims[0] * v.dims[1] * v.dims[2];
    return seeds * std::min(win, 64.0 * vox);
}

// Completes a tracked frame: the next frame of its track starts from the first
// max_seeds distinct positions of its regions in rank order (none: its own seeds
// or grid).
static void hand_over(Track& tr, const SrvReq& r) {
    tr.busy = false;
    tr.seeds.clear();
    if (r.status != KS_OK) return;
    for (const ks_region& g : r.regions) {
        if ((int32_t)(tr.seeds.size() / 3) >= r.max_seeds) break;
        bool seen = false;
        for (size_t k = 0; k < tr.seeds.size() && !seen; k += 3)
            seen = tr.seeds[k] == g.x && tr.seeds[k + 1] == g.y && tr.seeds[k + 2] == g.z;
        if (!seen) tr.seeds.insert(tr.seeds.end(), {g.x, g.y, g.z});
    }
}

// Work of one batch: about 10 ms of device time at the measured visit rates.
constexpr double kBatchWork = 2.0e10;
// A request above this estimated work (the MR-like volumes: a full-size mean-
// shift search) is large: large requests run one at a time, each alone in its
// batch, so that one is not slowed by another, while small requests pass them
// in the queue and run beside them.  (Splitting the large search into several
// launches, or giving it or the small batches beside it a part of the device,
// measured no better at any load: the small requests gained what the large
// ones lost.)
constexpr double kLargeWork = 3.0e10;

// One scheduler step; returns true if it did any work.
bool ks_server::tick() {
    bool worked = false;
    // Retire finished slots.
    for (Slot* sl : slots) {
        if (!sl->busy) continue;
        hipError_t q = hipEventQuery(sl->done);
        if (q == hipErrorNotReady) continue;
        std::vector<std::vector<ks_region>> res;
        std::vector<int> nf;
        if (q == hipSuccess) sl->ctx.end_detect(sl->in, sl->plan, &res, &nf);
        const double t = now_ms();
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < sl->tickets.size(); ++i) {
            auto it = reqs.find(sl->tickets[i]);
            if (it == reqs.end()) continue;
            SrvReq& r = it->second;
            if (q == hipSuccess) {
                r.regions = std::move(res[i]);
                r.n_found = nf[i];
                r.status = KS_OK;
            } else {
                r.status = KS_E_DEVICE;
                fatal = KS_E_DEVICE;
            }
            if (r.track >= 0) hand_over(tracks[r.track], r);
            r.t_done = t;
            pool.put(r.host, r.host_cap);
            r.host = nullptr;
            latencies.push_back(t - r.t_submit);
            completed += 1;
            in_flight -= 1;
            last_done = t;
        }
        sl->busy = false;
        sl->tickets.clear();
        worked = true;
        done_cv.notify_all();
    }
    // Admit pending requests into a free slot as one batch, oldest first, while
    // the busy slots' bytes plus the batch's own (its volumes and a freshly
    // sized arena) fit the budget.
    Slot* free_slot = nullptr;
    for (Slot* sl : slots)
        if (!sl->busy) { free_slot = sl; break; }
    if (!free_slot) return worked;
    size_t busy_bytes = 0;
    bool large_running = false;
    for (Slot* sl : slots)
        if (sl->busy) {
            busy_bytes += sl->held();
            large_running = large_running || sl->large;
        }
    std::vector<uint64_t> take;
    std::vector<ks::VolIn> batch;
    size_t raw_bytes = 0;
    bool large = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        double work = 0;
        for (auto it = pending.begin(); it != pending.end();) {
            SrvReq& r = reqs[*it];
            // a tracked frame waits for the frame before it; others pass it
            if (r.track >= 0 && tracks[r.track].busy) {
                ++it;
                continue;
            }
            // a large request waits while another runs, and goes alone; small
            // requests pass it meanwhile
            const bool big = r.work > kLargeWork;
            if (big && (large_running || !take.empty())) {
                ++it;
                continue;
            }
            if (!take.empty() && work + r.work > kBatchWork) break;
            // the start positions it will run from: its own list, or the track's
            const std::vector<int32_t>* list = r.own_seeds ? &r.seeds : nullptr;
            if (r.track >= 0 && !tracks[r.track].seeds.empty()) list = &tracks[r.track].seeds;
            ks::VolIn v = r.in;
            if (list) {
                v.seeds = list->empty() ? kNoSeeds : list->data();
                v.n_seeds = (int64_t)list->size() / 3;
            }
            batch.push_back(v);
            const size_t rb = raw_bytes + ((r.host_bytes + 255) & ~(size_t)255);
            if (busy_bytes + ks::Context::arena_fresh(batch) + ks::granule(rb) > budget) {
                batch.pop_back();
                break;   // oldest first: no overtaking
            }
            raw_bytes = rb;
            work += r.work;
            if (r.track >= 0) {
                Track& tr = tracks[r.track];
                tr.busy = true;
                if (!tr.seeds.empty()) r.seeds = tr.seeds;
            }
            if (list) {
                r.in.seeds = r.seeds.empty() ? kNoSeeds : r.seeds.data();
                r.in.n_seeds = (int64_t)r.seeds.size() / 3;
            }
            take.push_back(*it);
            it = pending.erase(it);
            if (big) {
                large = true;
                break;
            }
        }
        admitted += (int64_t)take.size();
        in_flight += (int64_t)take.size();
    }
    if (take.empty()) return worked;
    Slot* sl = free_slot;
    // Room for the batch: its slot's buffers grow (by at least 1.5x) to what it
    // needs; while the total would pass the budget, idle slots give their buffers
    // back (largest first), then this slot (it then allocates the batch's size
    // only).
    auto total_after = [&]() {
        size_t t = 0;
        for (Slot* o : slots)
            t += o != sl ? o->held()
                         : sl->ctx.arena_after(batch) + (raw_bytes <= sl->raw.cap ? sl->raw.cap : ks::granule(raw_bytes));
        return t;
    };
    std::vector<Slot*> idle;
    for (Slot* o : slots)
        if (!o->busy && o != sl && o->held() > 0) idle.push_back(o);
    std::sort(idle.begin(), idle.end(), [](Slot* a, Slot* b) { return a->held() > b->held(); });
    for (Slot* o : idle) {
        if (total_after() <= budget) break;
        o->release();
    }
    if (total_after() > budget) sl->release();
    sl->busy = true;
    sl->large = large;
    sl->tickets = take;
    sl->in.clear();
    size_t raw_total = 0;
    std::vector<size_t> offs;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t t : take) {
            offs.push_back(raw_total);
            raw_total += (reqs[t].host_bytes + 255) & ~(size_t)255;
        }
    }
    ks_status st = sl->raw.ensure(std::max<size_t>(raw_total, 256), nullptr);
    if (st == KS_OK) {
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < take.size() && st == KS_OK; ++i) {
            SrvReq& r = reqs[take[i]];
            char* dst = static_cast<char*>(sl->raw.ptr) + offs[i];
            // from the request's pinned copy straight to the device
            if (hipMemcpyAsync(dst, r.host, r.host_bytes, hipMemcpyHostToDevice, sl->stream) != hipSuccess)
                st = KS_E_DEVICE;
            ks::VolIn v = r.in;
            v.raw = dst;
            sl->in.push_back(v);
        }
    }
    if (st == KS_OK) st = sl->ctx.begin_detect(sl->in, sl->stream, sl->plan);
    if (st == KS_OK && hipEventRecord(sl->done, sl->stream) != hipSuccess) st = KS_E_DEVICE;
    account();
    if (st != KS_OK) {
        std::lock_guard<std::mutex> lk(mu);
        for (uint64_t t : take) {
            SrvReq& r = reqs[t];
            r.status = st;
            r.t_done = now_ms();
            completed += 1;
            in_flight -= 1;
            if (r.track >= 0) hand_over(tracks[r.track], r);
        }
        sl->busy = false;
        if (st == KS_E_DEVICE) fatal = st;
        // the pinned copies go back to the pool once the stream no longer reads them
        hipStreamSynchronize(sl->stream);
        for (uint64_t t : take) {
            SrvReq& r = reqs[t];
            pool.put(r.host, r.host_cap);
            r.host = nullptr;
        }
        done_cv.notify_all();
    }
    return true;
}

// Device bytes the slots hold for requests, and their high-water mark.
void ks_server::account() {
    size_t t = 0;
    for (Slot* o : slots) t += o->held();
    std::lock_guard<std::mutex> lk(mu);
    in_use = t;
    peak = std::max(peak, t);
}

void ks_server::run() {
    ks_status st = KS_OK;
    if (hipSetDevice(device) != hipSuccess) st = KS_E_DEVICE;
    for (int i = 0; i < max_slots && st == KS_OK; ++i) {
        Slot* sl = new Slot();
        // every launch takes the full persistent grid: a slot's blocks start as the
        // blocks of the launch before it retire, so the device never runs a
        // partial grid once the other slots have drained
        st = sl->ctx.init(device);
        if (st == KS_OK && hipEventCreateWithFlags(&sl->done, hipEventDisableTiming) != hipSuccess) st = KS_E_DEVICE;
        slots.push_back(sl);
    }
    // the slots' streams one after another: streams take the device's hardware
    // queues round robin, so consecutive ones land on different queues and one
    // slot's work does not wait behind another's
    for (Slot* sl : slots)
        if (st == KS_OK && hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess) st = KS_E_DEVICE;
    {
        std::lock_guard<std::mutex> lk(mu);
        init_status = st;
        ready = true;
    }
    cv.notify_all();
    if (st != KS_OK) return;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(mu);
            if (stop && pending.empty() && in_flight == 0) break;
        }
        const bool worked = tick();
        if (!worked) {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait_for(lk, std::chrono::microseconds(100));
        }
    }
}

extern "C" {

ks_status ks_server_create(int32_t device, size_t hbm_budget, int32_t max_slots, ks_server** out) {
    if (!out || hbm_budget == 0 || max_slots < 1 || max_slots > 16 || device < 0) return KS_E_INVALID;
    ks_server* s = new (std::nothrow) ks_server();
    if (!s) return KS_E_NOMEM;
    s->device = device;
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    s->worker = std::thread([s] { s->run(); });
    ks_status st;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv.wait(lk, [s] { return s->ready; });
        st = s->init_status;
    }
    if (st != KS_OK) {
        ks_server_destroy(s);
        return st;
    }
    *out = s;
    return KS_OK;
}

}  // extern "C"

ks_status ks_server::submit(const ks_request* req, int64_t track, int32_t max_seeds, uint64_t* ticket) {
    ks_server* s = this;
    ks_status st = ks::check_request(req->volume, req->dtype, req->dims, req->bins, req->seed_spacing, req->scales,
                                     req->method, req->max_iter);
    if (st != KS_OK) return st;
    if (!ks::options_ok(req->options) || !ks::options_fit(req->options, req->bins)) return KS_E_INVALID;
    if (req->max_regions < 0) return KS_E_INVALID;
    const bool own = req->seeds || req->n_seeds;
    if (own && (st = ks::check_seeds(req->dims, req->scales, req->method, req->seeds, req->n_seeds)) != KS_OK)
        return st;
    SrvReq r;
    r.in.raw = nullptr;
    r.in.dtype = req->dtype;
    std::memcpy(r.in.dims, req->dims, sizeof(r.in.dims));
    r.in.bins = req->bins;
    r.in.spacing = req->seed_spacing;
    r.in.scales[0] = req->scales[0];
    r.in.scales[1] = req->scales[1];
    r.in.method = req->method;
    r.in.max_iter = req->max_iter;
    r.in.opt = req->options;
    r.track = track;
    r.max_seeds = max_seeds;
    r.own_seeds = own;
    if (own) r.seeds.assign(req->seeds, req->seeds + 3 * req->n_seeds);
    // trajectories of the largest start set the request may run with
    const int64_t per = req->method == KS_MEANSHIFT ? req->scales[1] - req->scales[0] + 1 : 1;
    int64_t n_start = own ? req->n_seeds
                          : ks::num_trajectories(req->dims, req->seed_spacing, req->scales, KS_QUADRANT);
    if (track >= 0) n_start = std::max<int64_t>(n_start, max_seeds);
    // every region it can find, or the top max_regions of them
    int64_t cap = std::min<int64_t>(std::max<int64_t>(n_start * per, 1), 1 << 20);
    if (req->max_regions > 0) cap = std::min<int64_t>(cap, req->max_regions);
    r.in.capacity = (int32_t)cap;
    const size_t esz = req->dtype == KS_U8 ? 1 : 2;
    const size_t bytes = esz * (size_t)req->dims[0] * req->dims[1] * req->dims[2];
    {
        // the most it can need alone: n_start listed start positions
        ks::VolIn u = r.in;
        u.seeds = kNoSeeds;
        u.n_seeds = n_start;
        r.footprint = request_bytes(u, bytes);
    }
    r.work = work_estimate(r.in, n_start);
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop) return KS_E_SHUTDOWN;
    if (s->fatal != KS_OK) return s->fatal;
    if (r.footprint > s->budget) {
        s->refused += 1;
        return KS_E_TOO_LARGE;
    }
    lk.unlock();
    r.host = s->pool.get(bytes, &r.host_cap);
    if (!r.host) return KS_E_NOMEM;
    r.host_bytes = bytes;
    std::memcpy(r.host, req->volume, bytes);
    lk.lock();
    r.t_submit = now_ms();
    if (s->first_submit < 0) s->first_submit = r.t_submit;
    const uint64_t t = s->next_ticket++;
    s->reqs.emplace(t, std::move(r));
    s->pending.push_back(t);
    s->submitted += 1;
    *ticket = t;
    lk.unlock();
    s->cv.notify_all();
    return KS_OK;
}

extern "C" {

ks_status ks_server_submit(ks_server* s, const ks_request* req, uint64_t* ticket) {
    if (!s || !req || !ticket) return KS_E_INVALID;
    return s->submit(req, -1, 0, ticket);
}

ks_status ks_server_submit_tracked(ks_server* s, const ks_request* req, int64_t track, int32_t max_seeds,
                                   uint64_t* ticket) {
    if (!s || !req || !ticket || track < 0 || max_seeds < 1) return KS_E_INVALID;
    const int64_t per = req->method == KS_MEANSHIFT ? (int64_t)req->scales[1] - req->scales[0] + 1 : 1;
    if (per < 1 || max_seeds > (int64_t)INT32_MAX / per) return KS_E_INVALID;
    return s->submit(req, track, max_seeds, ticket);
}

ks_status ks_server_poll(ks_server* s, uint64_t ticket, ks_region* out, int32_t capacity, int32_t* n_found) {
    if (!s || !n_found || capacity < 0 || (capacity > 0 && !out)) return KS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return KS_E_INVALID;
    SrvReq& r = it->second;
    if (r.status == KS_E_NOT_READY) return KS_E_NOT_READY;
    const ks_status st = (ks_status)r.status;
    if (st == KS_OK) {
        const int w = std::min<int>(capacity, (int)r.regions.size());
        if (w > 0) std::memcpy(out, r.regions.data(), sizeof(ks_region) * (size_t)w);
        *n_found = r.n_found;
    }
    s->reqs.erase(it);
    return st;
}

ks_status ks_server_drain(ks_server* s) {
    if (!s) return KS_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    s->done_cv.wait(lk, [s] { return (s->pending.empty() && s->in_flight == 0) || s->fatal != KS_OK; });
    return s->fatal;
}

ks_status ks_server_stats(ks_server* s, ks_server_stats_t* out) {
    if (!s || !out) return KS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->admitted = s->admitted;
    out->completed = s->completed;
    out->refused = s->refused;
    out->queued_now = (int64_t)s->pending.size();
    out->in_flight = s->in_flight;
    out->bytes_in_use = (int64_t)s->in_use;
    out->budget_bytes = (int64_t)s->budget;
    out->bytes_peak = (int64_t)s->peak;
    out->p50_ms = percentile(s->latencies, 0.50);
    out->p99_ms = percentile(s->latencies, 0.99);
    double sum = 0;
    for (double x : s->latencies) sum += x;
    out->mean_ms = s->latencies.empty() ? 0.0 : sum / (double)s->latencies.size();
    const double span = s->last_done - s->first_submit;
    out->volumes_per_s = (s->completed > 0 && span > 0) ? (double)s->completed / (span / 1000.0) : 0.0;
    return KS_OK;
}

ks_status ks_server_reset_stats(ks_server* s) {
    if (!s) return KS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    s->latencies.clear();
    s->submitted = s->admitted = s->completed = s->refused = 0;
    // with work still queued or running the window starts now, else at the next submit
    s->first_submit = (s->in_flight > 0 || !s->pending.empty()) ? now_ms() : -1;
    s->last_done = 0;
    return KS_OK;
}

ks_status ks_server_destroy(ks_server* s) {
    if (!s) return KS_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (Slot* sl : s->slots) {
        if (sl->stream) hipStreamSynchronize(sl->stream);
        sl->ctx.destroy();
        sl->raw.release();
        if (sl->done) hipEventDestroy(sl->done);
        if (sl->stream) hipStreamDestroy(sl->stream);
        delete sl;
    }
    // volumes of requests that never ran
    for (auto& kv : s->reqs) s->pool.put(kv.second.host, kv.second.host_cap);
    delete s;
    return KS_OK;
}

}  // extern "C"

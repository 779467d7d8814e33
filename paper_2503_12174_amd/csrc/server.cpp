// server.cpp -- continuous-batching request loop.
//
// One scheduler thread per server owns a HIP stream (default priority) on the
// context's device.  Requests are admitted while the device-memory estimate of all
// admitted requests fits the budget and a descriptor slot is free.  Every launch
// wave packs whole-pixel segments of all active requests into shared path queues:
// raygen / finalize / adj_pixel run per segment, trace / shade / shadow (and their
// adjoint forms) run once over the shared queues and read each path's request
// descriptor from a device table by slot.  Compensation-step requests (forward +
// VJP) put their segments first so their replay fills a dense queue prefix.  A
// request completes when its last wave (and its gradient reduction) has passed on
// the device; its latency is measured from submit to that point on the host clock.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <thread>

#include "runtime.hpp"

using namespace dpcs;

namespace {

using clk = std::chrono::steady_clock;

// first-fit allocator of offsets inside one device arena
class Arena {
  public:
    void reset(size_t size) {
        size_ = size;
        free_.clear();
        if (size) free_.push_back({0, size});
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                it->first += bytes;
                it->second -= bytes;
                if (it->second == 0) free_.erase(it);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        auto it = free_.begin();
        while (it != free_.end() && it->first < off) ++it;
        it = free_.insert(it, {off, bytes});
        auto nx = std::next(it);   // coalesce with neighbours
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    size_t size_ = 0;
    std::list<std::pair<size_t, size_t>> free_;
};

struct Req {
    uint64_t id = 0;
    dpcs_scene scene = nullptr;
    dpcs_render_params params{};
    ReqDesc r{};
    const float* proj = nullptr;
    float* out = nullptr;
    const float* grad = nullptr;
    const float* target = nullptr;
    dpcs_grads grads{};
    bool adjoint = false;
    int64_t npix = 0, next_pixel = 0;
    size_t bytes = 0, off = 0;
    int slot = -1;
    clk::time_point t_submit, t_admit, t_launch;   // submit, admission, first wave launched
    bool launched = false;
    hipEvent_t ready = nullptr;   // recorded on the caller's input stream at submit
    hipEvent_t done = nullptr;
    int32_t status = DPCS_OK;
    bool scheduled_all = false;
};

struct Seg {
    Req* q;
    uint32_t a, b;   // pixels
};

// Binning buffers of the loop's compensation waves (map cotangents sorted by tile and
// summed in fixed point, as a single request's VJP does), carved for the largest binned
// map (1024 x 1024: 16-texel tiles, 4096 of them); a wave binds them to its request's
// map size.  Layout: records, sorted records, stage blocks, count, bins, chunk row bases.
size_t loop_bins_bytes(int64_t cap, int C, int RS) {
    const size_t rec = 4 * (size_t)RS * cap;
    const size_t stage = 8 * (size_t)((cap + ACC_CHUNK - 1) / ACC_CHUNK + MAP_MAX_BINS) * (MAP_MAX_T + 1) *
                         (MAP_MAX_T + 1) * C;
    const size_t rows = 4 * (size_t)((cap + BIN_CHUNK - 1) / BIN_CHUNK) * MAP_MAX_BINS;
    auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
    return 2 * up(rec) + up(stage) + up(4) + up(4 * (3 * (size_t)MAP_MAX_BINS + 2)) + up(rows);
}

// the buffers at base as bins of a W x H map (false: the map is too large to bin)
bool loop_bins_view(char* base, int64_t cap, int C, int RS, int W, int H, MapBins& mb) {
    mb = MapBins{};
    int T = 0, nbx = 0, nby = 0;
    if (!base || !map_tiling(W, H, T, nbx, nby)) return false;
    auto up = [](size_t n) { return (n + 255) & ~size_t(255); };
    const size_t rec = 4 * (size_t)RS * cap;
    const size_t stage = 8 * (size_t)((cap + ACC_CHUNK - 1) / ACC_CHUNK + MAP_MAX_BINS) * (MAP_MAX_T + 1) *
                         (MAP_MAX_T + 1) * C;
    char* b = base;
    mb.rec = (float*)b;
    b += up(rec);
    mb.sorted = (float*)b;
    b += up(rec);
    mb.stage = (long long*)b;
    b += up(stage);
    mb.count = (uint32_t*)b;
    b += up(4);
    mb.bins = (uint32_t*)b;
    b += up(4 * (3 * (size_t)MAP_MAX_BINS + 2));
    mb.rowbase = (uint32_t*)b;
    mb.cap = cap;
    mb.W = W;
    mb.H = H;
    mb.T = T;
    mb.nbx = nbx;
    mb.nby = nby;
    mb.nb = nbx * nby;
    return true;
}

size_t request_bytes(const ReqDesc& r, bool adjoint) {
    const size_t nEp = (size_t)r.Wp * r.Hp, nT = (size_t)r.tw * r.th;
    size_t b = 16 * nEp + 256 + 16 * nT + 256;          // E_p, packed maps
    if (adjoint) b += 16 * nEp + 256 + 20 * nT + 256 + 256;   // dE_p, map cotangents, scalars
    return b;
}

}  // namespace

struct dpcs_server_s {
    dpcs_context ctx = nullptr;
    hipStream_t st = nullptr;
    // a depth's shadow rays run on `side` (default priority, own spill region) beside the
    // next depth's closest hit on `st`, ordered by the two events (null side: one stream)
    hipStream_t side = nullptr;
    hipEvent_t ev_shade = nullptr, ev_shadow = nullptr;
    int* spill2 = nullptr;
    size_t budget = 0, shared_bytes = 0, admitted_bytes = 0;
    int max_slots = 0;
    int64_t cap = 0;
    ReqDesc* table = nullptr;
    char* arena_base = nullptr;
    Arena arena;
    void* qbuf = nullptr;
    Queues q{};
    AdjQueues aq{};
    uint32_t* rec = nullptr;     // path records of a wave's compensation segments
    int64_t rec_cap = 0;         // words
    char* tex_bins = nullptr;    // binning buffers (texture maps, E_p) of one-request
    char* ep_bins = nullptr;     // compensation waves, or null: every wave scatters directly
    int64_t tex_bins_cap = 0, ep_bins_cap = 0;
    int64_t st_binned = 0;       // waves whose compensation gradients were binned
    std::vector<int> free_slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req*> queued;
    std::vector<Req*> active, finishing;
    std::deque<std::tuple<uint64_t, int32_t, double>> completed;
    bool stop = false;
    int64_t st_submitted = 0, st_completed = 0, st_rejected = 0, st_waves = 0, st_samples = 0, st_peak = 0;
    int64_t st_replayed = 0, st_retraced = 0;   // waves whose compensation segments replayed / re-traced
    int64_t st_wait_us = 0, st_admit_us = 0, st_run_us = 0;   // summed latency parts of completed requests
    int64_t lat_cap = 0;         // most paths per wave
    std::thread worker;
    std::string err;
    void run();
    void admit_locked(Launch& l);
    void wave(Launch& l);
};

void dpcs_server_s::admit_locked(Launch& l) {
    while (!queued.empty() && !free_slots.empty()) {
        Req* q = queued.front();
        if (admitted_bytes + q->bytes + shared_bytes > budget) break;   // FIFO: wait for memory
        size_t off = 0;
        if (!arena.alloc(q->bytes, &off)) break;
        queued.pop_front();
        q->off = off;
        q->slot = free_slots.back();
        free_slots.pop_back();
        admitted_bytes += q->bytes;
        st_peak = std::max<int64_t>(st_peak, (int64_t)(admitted_bytes + shared_bytes));
        q->t_admit = clk::now();
        // the request's inputs were produced on the caller's stream: the loop's first
        // launch for it waits for everything queued there before submit
        (void)hipStreamWaitEvent(l.st, q->ready, 0);
        // carve the request's device state from its arena region
        char* base = arena_base + off;
        auto take = [&](size_t n) {
            char* p = base;
            base += (n + 255) & ~size_t(255);
            return (void*)p;
        };
        ReqDesc& r = q->r;
        const size_t nEp = (size_t)r.Wp * r.Hp, nT = (size_t)r.tw * r.th;
        float4* Ep = (float4*)take(16 * nEp);
        float4* tex = (float4*)take(16 * nT);
        launch_prf(l, r, Ep);
        launch_pack_tex(l, r, q->params.albedo, q->params.brdf == DPCS_BRDF_GGX ? q->params.roughness : nullptr, tex);
        r.Ep = Ep;
        r.tex4 = tex;
        if (q->adjoint) {
            r.dEp = (float*)take(16 * nEp);
            r.d_tex = (float*)take(20 * nT);
            r.d_acc = (float*)take(128);
            ZeroList zl(l);
            zl.add(r.dEp, 4 * (int64_t)nEp);
            zl.add(r.d_tex, 5 * (int64_t)nT);
            zl.add(r.d_acc, 32);
            zl.launch();
        }
        active.push_back(q);
    }
}

void dpcs_server_s::wave(Launch& l) {
    // Fill the wave's capacity with whole pixels, least remaining work first (shortest
    // remaining processing time: small requests finish within a wave or two instead of
    // sharing every wave with the large ones); then order the segments with the
    // compensation steps first so their replay has a dense queue prefix.
    std::vector<Req*> pick;
    for (Req* q : active)
        if (!q->scheduled_all) pick.push_back(q);
    if (pick.empty()) return;
    auto remaining = [](const Req* q) {
        return (q->npix - q->next_pixel) * (int64_t)q->r.spp * (q->adjoint ? 2 : 1);
    };
    std::stable_sort(pick.begin(), pick.end(), [&](const Req* a, const Req* b) { return remaining(a) < remaining(b); });
    // one scene per wave (the scene of the request with the least remaining work): every
    // ray of the wave is then on one tree, whose top levels the traversal stages in LDS,
    // and the wave's node and triangle reads share one tree in L2
    const dpcs_scene scene = pick.front()->scene;
    pick.erase(std::remove_if(pick.begin(), pick.end(), [&](const Req* q) { return q->scene != scene; }), pick.end());
    std::vector<std::pair<Req*, int64_t>> take;   // request, pixels this wave
    // waves are cut to lat_cap paths, alone or not, so that a newcomer waits for short
    // waves only (a full wave of 4M paths at depth 4 with its adjoint takes ~3.5 ms;
    // 2^21 paths measured better than 2^20 for the loop's throughput and p99 at 50
    // requests/s, and better than full waves for p50 and p99)
    int64_t room = std::min(cap, lat_cap);
    room = std::max<int64_t>(room, pick.front()->r.spp);
    for (Req* q : pick) {
        const int64_t px = std::min<int64_t>(q->npix - q->next_pixel, room / q->r.spp);
        if (px <= 0) continue;
        take.push_back({q, px});
        room -= px * q->r.spp;
    }
    std::stable_partition(take.begin(), take.end(), [](const std::pair<Req*, int64_t>& t) { return t.first->adjoint; });
    std::vector<Seg> segs;
    int64_t used = 0, n_adj = 0;
    int max_depth = 1;
    bool env = false, any_adj = false;
    for (const auto& t : take) {
        Req* q = t.first;
        const int spp = q->r.spp;
        const int64_t px = t.second;
        Seg s{q, (uint32_t)q->next_pixel, (uint32_t)(q->next_pixel + px)};
        q->r.g_base = s.a * (uint32_t)spp;
        q->r.sid_base = (uint32_t)used;
        segs.push_back(s);
        used += px * spp;
        if (q->adjoint) n_adj = used, any_adj = true;
        q->next_pixel += px;
        max_depth = std::max(max_depth, q->r.max_depth);
        env = env || q->r.env_on;
    }
    if (segs.empty()) return;
    // path records for the compensation segments, when they fit: the replay then reads
    // hits and shadow visibility instead of tracing again
    int64_t rec_need = 0;
    for (const Seg& s : segs)
        if (s.q->adjoint) rec_need += (int64_t)(s.b - s.a) * s.q->r.spp * s.q->r.max_depth;
    const bool replay = any_adj && rec_need <= rec_cap;
    int64_t rec_off = 0;
    const clk::time_point now = clk::now();
    for (const Seg& s : segs)
        if (!s.q->launched) {
            s.q->launched = true;
            s.q->t_launch = now;
        }
    for (const Seg& s : segs) {
        Req* q = s.q;
        if (replay && q->adjoint) {
            q->r.rec = rec + rec_off;
            q->r.rec_g0 = s.a * (uint32_t)q->r.spp;
            rec_off += (int64_t)(s.b - s.a) * q->r.spp * q->r.max_depth;
        } else {
            q->r.rec = nullptr;
        }
        launch_set_desc(l, table, q->slot, q->r);
    }
    // the tree of the wave's scene (every segment's descriptor holds it): closest-hit
    // queries read nothing else of a descriptor, so they run in the one-request form
    const ReqDesc& any = segs[0].q->r;
    // forward over the shared queues
    launch_set_count(l, q.cnt, 0, (uint32_t)used, 1, 4);
    for (const Seg& s : segs) launch_raygen(l, q, s.q->r, table, s.q->slot, s.q->r.g_base, (s.b - s.a) * s.q->r.spp,
                                            false, nullptr);
    int cur = 0;
    // a depth's shadow rays on the side stream beside the next depth's closest hit;
    // shading (both add to the samples' radiance) and the finalize wait for them
    Queues qs = q;
    qs.spill = spill2;
    const Launch ls{side, ctx->grid_cap};
    // (only full-size waves: at 2^20 paths of a small scene, the scene-fit step's waves,
    // the cross-stream waits cost more than the overlap gained: 2.50 -> 2.62 ms)
    const bool side_fwd = side && used >= LOOP_SIDE_MIN_PATHS, side_adj = side && n_adj >= LOOP_SIDE_MIN_PATHS;
    for (int d = 0; d < max_depth; ++d) {
        launch_trace(l, q, cur, any, nullptr, used);   // (empties the queues shading appends to)
        if (side_fwd && d > 0) (void)hipStreamWaitEvent(st, ev_shadow, 0);
        launch_shade(l, q, cur, d, any, table, used);
        if (side_fwd) {
            (void)hipEventRecord(ev_shade, st);
            (void)hipStreamWaitEvent(side, ev_shade, 0);
            launch_shadow(ls, qs, 0, any, table, used, d, true);
            if (env) launch_shadow(ls, qs, 1, any, table, used, d, true);
            (void)hipEventRecord(ev_shadow, side);
        } else {
            launch_shadow(l, q, 0, any, table, used, d, true);
            if (env) launch_shadow(l, q, 1, any, table, used, d, true);
        }
        cur ^= 1;
    }
    if (side_fwd) (void)hipStreamWaitEvent(st, ev_shadow, 0);
    for (const Seg& s : segs) launch_finalize(l, q, s.q->r, table, s.q->slot, s.a, s.b);
    // adjoint replay of the compensation-step segments (a dense prefix of the wave)
    if (any_adj) {
        // compensation paths of one request, replayed from records, with maps the binning
        // buffers hold: the replay runs in the one-request form and its map cotangents are
        // binned and flushed into the request's maps like a single VJP's, instead of one
        // global atomic per texel and channel
        Req* binq = nullptr;
        AdjQueues ab = aq;
        if (replay) {
            for (const Seg& s : segs)
                if (s.q->adjoint) binq = binq == nullptr || binq == s.q ? s.q : (Req*)-1;
            if (binq == (Req*)-1 || !loop_bins_view(tex_bins, tex_bins_cap, 5, 8, binq->r.tw, binq->r.th, ab.tb) ||
                !loop_bins_view(ep_bins, ep_bins_cap, 3, 6, binq->r.Wp, binq->r.Hp, ab.eb)) {
                binq = nullptr;
            } else {   // a fresh histogram for this map size
                ZeroList zl(l);
                zl.add((float*)ab.tb.count, 1);
                zl.add((float*)ab.tb.bins, 3 * (int64_t)MAP_MAX_BINS + 2);
                zl.add((float*)ab.eb.count, 1);
                zl.add((float*)ab.eb.bins, 3 * (int64_t)MAP_MAX_BINS + 2);
                zl.launch();
                ++st_binned;
            }
        }
        for (const Seg& s : segs)
            if (s.q->adjoint) launch_adj_pixel(l, q, aq, s.q->r, s.a, s.b, nullptr);
        // queue sizes: the replay's rotate over their own slots; re-tracing, the
        // closest-hit launch empties the queues shading appends to
        if (binq || replay) launch_set_count(l, q.cnt, REPLAY_CNT, (uint32_t)n_adj, REPLAY_CNT + 1, REPLAY_CNT + 2);
        else launch_set_count(l, q.cnt, 0, (uint32_t)n_adj, 1, 4);
        for (const Seg& s : segs)
            if (s.q->adjoint) launch_adj_raygen(l, q, aq, s.q->r, s.q->slot, s.q->r.g_base, (s.b - s.a) * s.q->r.spp);
        cur = 0;
        for (int d = 0; d < max_depth; ++d) {
            if (binq) {
                launch_adj_replay(l, q, ab, cur, d, binq->r, nullptr, n_adj);
                if ((d + 1) % BIN_DEPTHS == 0 || d == max_depth - 1) launch_map_flush(l, ab, binq->r);
            } else if (replay) {
                launch_adj_replay(l, q, aq, cur, d, any, table, n_adj);
            } else {   // (adjoint shadow rays beside the next closest hit, as in the forward)
                launch_trace(l, q, cur, any, nullptr, n_adj);
                if (side_adj && d > 0) (void)hipStreamWaitEvent(st, ev_shadow, 0);
                launch_adj_shade(l, q, aq, cur, d, any, table, n_adj);
                if (side_adj) {
                    (void)hipEventRecord(ev_shade, st);
                    (void)hipStreamWaitEvent(side, ev_shade, 0);
                    launch_adj_shadow(ls, qs, aq, 0, cur ^ 1, any, table, n_adj);
                    if (env) launch_adj_shadow(ls, qs, aq, 1, cur ^ 1, any, table, n_adj);
                    (void)hipEventRecord(ev_shadow, side);
                } else {
                    launch_adj_shadow(l, q, aq, 0, cur ^ 1, any, table, n_adj);
                    if (env) launch_adj_shadow(l, q, aq, 1, cur ^ 1, any, table, n_adj);
                }
            }
            cur ^= 1;
        }
        if (side_adj && !binq && !replay) (void)hipStreamWaitEvent(st, ev_shadow, 0);
    }
    ++st_waves;
    st_samples += used + n_adj;
    if (any_adj) ++(replay ? st_replayed : st_retraced);
    for (const Seg& s : segs) {
        Req* q = s.q;
        if (q->next_pixel >= q->npix) {
            q->scheduled_all = true;
            if (q->adjoint)
                launch_adj_finish(l, q->r, q->grads.d_proj_image, q->grads.d_albedo, q->grads.d_roughness,
                                  q->grads.d_specular, q->grads.d_scalars, q->r.d_acc);
            (void)hipEventRecord(q->done, st);
        }
    }
    if (hipGetLastError() != hipSuccess) err = "kernel launch failed in the server loop";
}

void dpcs_server_s::run() {
    (void)hipSetDevice(ctx->device);
    Launch l{st, ctx->grid_cap};
    std::deque<hipEvent_t> inflight;
    std::vector<hipEvent_t> ev_pool;
    for (int k = 0; k < 4; ++k) {
        hipEvent_t e;
        (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
        ev_pool.push_back(e);
    }
    size_t ev_next = 0;
    while (true) {
        {
            std::unique_lock<std::mutex> lk(mu);
            admit_locked(l);
            if (stop && queued.empty() && active.empty() && finishing.empty()) break;
            if (active.empty() && finishing.empty())
                cv.wait_for(lk, std::chrono::milliseconds(2));
        }
        // one wave over everything active (the lists only change on this thread)
        bool launched = false;
        {
            std::lock_guard<std::mutex> lk(mu);
            const bool have = std::any_of(active.begin(), active.end(), [](Req* q) { return !q->scheduled_all; });
            if (have) {
                wave(l);
                launched = true;
            }
            for (auto it = active.begin(); it != active.end();) {
                if ((*it)->scheduled_all) {
                    finishing.push_back(*it);
                    it = active.erase(it);
                } else {
                    ++it;
                }
            }
        }
        if (launched) {
            hipEvent_t e = ev_pool[ev_next++ % ev_pool.size()];
            (void)hipEventRecord(e, st);
            inflight.push_back(e);
            // the host waits for each wave before building the next, so a wave takes in
            // whatever arrived while the previous one ran (one or two waves queued behind
            // the running one measured the same saturated throughput, 80 requests/s, and
            // 1-3 ms more p50 latency at 50 requests/s)
            while (!inflight.empty()) {
                (void)hipEventSynchronize(inflight.front());
                inflight.pop_front();
            }
        } else if (!finishing.empty()) {
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        // retire requests whose work has passed on the device
        std::lock_guard<std::mutex> lk(mu);
        for (auto it = finishing.begin(); it != finishing.end();) {
            Req* q = *it;
            const hipError_t e = hipEventQuery(q->done);
            if (e == hipErrorNotReady) {
                ++it;
                continue;
            }
            const clk::time_point t_done = clk::now();
            const double ms = std::chrono::duration<double, std::milli>(t_done - q->t_submit).count();
            auto us = [](clk::time_point a, clk::time_point b) {
                return (int64_t)std::chrono::duration_cast<std::chrono::microseconds>(b - a).count();
            };
            st_wait_us += us(q->t_submit, q->t_admit);
            st_admit_us += us(q->t_admit, q->t_launch);
            st_run_us += us(q->t_launch, t_done);
            const int32_t status = e == hipSuccess && err.empty() ? DPCS_OK : DPCS_E_DEVICE;
            completed.emplace_back(q->id, status, ms);
            ++st_completed;
            arena.release(q->off, q->bytes);
            admitted_bytes -= q->bytes;
            free_slots.push_back(q->slot);
            q->scene->refs.fetch_sub(1);
            (void)hipEventDestroy(q->done);
            (void)hipEventDestroy(q->ready);
            delete q;
            it = finishing.erase(it);
        }
    }
    (void)hipStreamSynchronize(st);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
}

extern "C" dpcs_status dpcs_server_create(dpcs_context ctx, size_t memory_budget_bytes, int32_t max_slots,
                                          dpcs_server* out) {
    if (!ctx || !out || max_slots < 1 || max_slots > 4096) return DPCS_E_INVALID;
    *out = nullptr;
    std::lock_guard<std::recursive_mutex> lk(ctx->mu);
    if (ctx->sticky) return DPCS_E_DEVICE;
    (void)hipSetDevice(ctx->device);
    (void)hipGetLastError();
    auto* s = new dpcs_server_s();
    s->ctx = ctx;
    s->budget = memory_budget_bytes;
    s->max_slots = max_slots;
    // shared wave queues take at most a quarter of the budget
    const size_t per_path = (2 * 80 + 4 + 2 * 52 + 16) + (2 * 144 + 16);
    const int64_t fit = (int64_t)(memory_budget_bytes / 4 / per_path);
    s->cap = std::max<int64_t>(1024, std::min<int64_t>({ctx->capacity, int64_t(1) << 22, fit}));
    s->lat_cap = std::min<int64_t>(s->cap, int64_t(1) << 21);
    const size_t c = (size_t)s->cap;
    // + 256 bytes of alignment slack per part (42 parts); path records for up to 8
    // vertices per path of a wave
    // traversal grids: four resident rounds, but never more workgroups than one per
    // TRACE_TB paths of a wave
    const int tblocks = (int)std::min<int64_t>(trace_grid_cap(ctx->grid_cap, TRACE_ROUNDS), (s->cap + TRACE_TB - 1) / TRACE_TB);
    const size_t spill_bytes = 4 * (size_t)tblocks * TRACE_TB * SPILL;
    const size_t qbytes = c * per_path + 64 * 256 + 2 * spill_bytes + 4 * 8 * c;
    s->shared_bytes = qbytes + sizeof(ReqDesc) * (size_t)max_slots;
    if (s->shared_bytes >= s->budget) {
        delete s;
        return fail(ctx, DPCS_E_INVALID, "memory budget smaller than the shared queues of one wave");
    }
    // binning buffers for one-request compensation waves (records of up to BIN_DEPTHS + 1
    // texture and BIN_DEPTHS E_p entries per path between flushes), when they take at most
    // a quarter of the budget (~1.2 GB for 2^21-path waves)
    s->tex_bins_cap = s->lat_cap * (BIN_DEPTHS + 1);
    s->ep_bins_cap = s->lat_cap * BIN_DEPTHS;
    const size_t bins_bytes = loop_bins_bytes(s->tex_bins_cap, 5, 8) + loop_bins_bytes(s->ep_bins_cap, 3, 6);
    const bool binning = bins_bytes <= s->budget / 4 && s->shared_bytes + bins_bytes < s->budget;
    if (binning) s->shared_bytes += bins_bytes;
    const size_t arena_bytes = s->budget - s->shared_bytes;
    bool ok = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) == hipSuccess;
    if (ok && (hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreateWithFlags(&s->ev_shade, hipEventDisableTiming) != hipSuccess ||
               hipEventCreateWithFlags(&s->ev_shadow, hipEventDisableTiming) != hipSuccess)) {
        (void)hipGetLastError();   // run every wave on one stream
        if (s->side) (void)hipStreamDestroy(s->side);
        if (s->ev_shade) (void)hipEventDestroy(s->ev_shade);
        s->side = nullptr;
        s->ev_shade = nullptr;
        s->ev_shadow = nullptr;
    }
    ok = ok && hipMalloc((void**)&s->table, sizeof(ReqDesc) * max_slots) == hipSuccess;
    ok = ok && hipMalloc(&s->qbuf, qbytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&s->arena_base, arena_bytes) == hipSuccess;
    if (ok && binning) {
        ok = hipMalloc((void**)&s->tex_bins, bins_bytes) == hipSuccess;
        s->ep_bins = ok ? s->tex_bins + loop_bins_bytes(s->tex_bins_cap, 5, 8) : nullptr;
    }
    if (!ok) {
        (void)hipGetLastError();
        if (s->arena_base) (void)hipFree(s->arena_base);
        if (s->table) (void)hipFree(s->table);
        if (s->qbuf) (void)hipFree(s->qbuf);
        if (s->st) (void)hipStreamDestroy(s->st);
        if (s->side) (void)hipStreamDestroy(s->side);
        if (s->ev_shade) (void)hipEventDestroy(s->ev_shade);
        if (s->ev_shadow) (void)hipEventDestroy(s->ev_shadow);
        delete s;
        return fail(ctx, DPCS_E_OOM, "server allocation failed");
    }
    s->arena.reset(arena_bytes);
    // carve the shared queues
    char* b = (char*)s->qbuf;
    auto take = [&](size_t n) {
        char* p = b;
        b += (n + 255) & ~size_t(255);
        return (void*)p;
    };
    for (int k = 0; k < 2; ++k) {
        s->q.po[k] = (PathO*)take(32 * c);
        s->q.pd[k] = (PathD*)take(32 * c);
        s->q.pb[k] = (float4*)take(16 * c);
        s->q.so[k] = (float4*)take(16 * c);
        s->q.sd[k] = (float4*)take(16 * c);
        s->q.sc[k] = (float4*)take(16 * c);
        s->q.st[k] = (float*)take(4 * c);
        s->aq.rl[k] = (float4*)take(16 * c);
        s->aq.puv[k] = (double2*)take(16 * c);
        s->aq.pend[k] = (float2*)take(8 * c);
        s->aq.penda[k] = (float4*)take(16 * c);
        s->aq.sproj[k] = (double2*)take(16 * c);
        s->aq.suv[k] = (double2*)take(16 * c);
        s->aq.sg[k] = (float4*)take(16 * c);
        s->aq.sa[k] = (float4*)take(16 * c);
        s->aq.ss[k] = (float*)take(4 * c);
        s->aq.pn[k] = (float4*)take(16 * c);
        s->aq.pns[k] = (float*)take(4 * c);
    }
    s->q.hit = (int*)take(4 * c);
    s->q.L = (float4*)take(16 * c);
    s->aq.delta = (float4*)take(16 * c);
    s->aq.tb = MapBins{};   // several requests' compensation paths: direct scatter (a
    s->aq.eb = MapBins{};   // wave of one request binds the binning buffers instead)
    s->q.cnt = (uint32_t*)take(4 * (SHADOW_CNT + 4));
    s->q.spill = (int*)take(spill_bytes);
    s->spill2 = (int*)take(spill_bytes);
    s->q.trace_blocks = tblocks;
    s->rec = (uint32_t*)take(4 * 8 * c);
    s->rec_cap = 8 * (int64_t)c;
    s->q.cap = s->cap;
    s->q.stats = nullptr;
    for (int k = max_slots - 1; k >= 0; --k) s->free_slots.push_back(k);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return DPCS_OK;
}

extern "C" dpcs_status dpcs_server_submit(dpcs_server s, const dpcs_request* rq) {
    if (!s || !rq) return DPCS_E_INVALID;
    dpcs_context ctx = s->ctx;
    if (!rq->scene || rq->scene->ctx != ctx || !rq->out_image) return DPCS_E_INVALID;
    if (rq->params.metallic || rq->params.normal_map) return DPCS_E_UNSUPPORTED;   // single-request path only
    if (rq->grads && rq->grads->d_camera) return DPCS_E_UNSUPPORTED;               // likewise
    (void)hipSetDevice(ctx->device);
    auto* q = new Req();
    std::string why;
    if (!fill_desc(ctx, q->r, &rq->params, rq->scene, rq->proj_image, &why)) {
        delete q;
        std::lock_guard<std::mutex> lk(s->mu);
        s->err = why;
        return DPCS_E_INVALID;
    }
    q->adjoint = rq->grads != nullptr;
    if (q->adjoint && !rq->grad_image && !rq->target) {
        delete q;
        return DPCS_E_INVALID;
    }
    q->id = rq->request_id;
    q->scene = rq->scene;
    q->params = rq->params;
    q->proj = rq->proj_image;
    q->out = rq->out_image;
    q->grad = rq->grad_image;
    q->target = rq->target;
    if (q->adjoint) q->grads = *rq->grads;
    q->r.out_image = rq->out_image;
    q->r.grad_image = rq->grad_image;
    q->r.target = rq->grad_image ? nullptr : rq->target;
    q->npix = (int64_t)q->r.Wc * q->r.Hc;
    q->bytes = request_bytes(q->r, q->adjoint);
    q->t_submit = clk::now();
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->st_submitted;
    if (q->bytes + s->shared_bytes > s->budget || q->r.spp > s->cap) {
        ++s->st_rejected;
        delete q;
        return DPCS_E_REJECTED;
    }
    if (s->stop) {
        delete q;
        return DPCS_E_INVALID;
    }
    if (hipEventCreateWithFlags(&q->done, hipEventDisableTiming) != hipSuccess) {
        delete q;
        return DPCS_E_DEVICE;
    }
    if (hipEventCreateWithFlags(&q->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(q->ready, rq->input_stream ? (hipStream_t)rq->input_stream : ctx->stream) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(q->done);
        if (q->ready) (void)hipEventDestroy(q->ready);
        delete q;
        return DPCS_E_DEVICE;
    }
    q->scene->refs.fetch_add(1);
    s->queued.push_back(q);
    s->cv.notify_one();
    return DPCS_OK;
}

extern "C" int32_t dpcs_server_poll(dpcs_server s, uint64_t* ids, int32_t* status, double* latency_ms, int32_t max) {
    if (!s || max <= 0) return 0;
    std::lock_guard<std::mutex> lk(s->mu);
    int32_t n = 0;
    while (n < max && !s->completed.empty()) {
        auto [id, stt, ms] = s->completed.front();
        s->completed.pop_front();
        if (ids) ids[n] = id;
        if (status) status[n] = stt;
        if (latency_ms) latency_ms[n] = ms;
        ++n;
    }
    return n;
}

extern "C" dpcs_status dpcs_server_stats(dpcs_server s, int64_t* o) {   // o: 14 counters
    if (!s || !o) return DPCS_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    o[0] = s->st_submitted;
    o[1] = s->st_completed;
    o[2] = s->st_rejected;
    o[3] = (int64_t)s->active.size() + (int64_t)s->finishing.size();
    o[4] = (int64_t)s->queued.size();
    o[5] = s->st_waves;
    o[6] = s->st_samples;
    o[7] = s->st_peak;
    o[8] = s->st_replayed;
    o[9] = s->st_retraced;
    o[10] = s->st_wait_us;
    o[11] = s->st_admit_us;
    o[12] = s->st_run_us;
    o[13] = s->st_binned;
    return DPCS_OK;
}

extern "C" dpcs_status dpcs_server_destroy(dpcs_server s) {
    if (!s) return DPCS_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->st);
    (void)hipFree(s->arena_base);
    (void)hipFree(s->qbuf);
    (void)hipFree(s->table);
    if (s->tex_bins) (void)hipFree(s->tex_bins);
    (void)hipStreamDestroy(s->st);
    if (s->side) {
        (void)hipStreamSynchronize(s->side);
        (void)hipStreamDestroy(s->side);
        (void)hipEventDestroy(s->ev_shade);
        (void)hipEventDestroy(s->ev_shadow);
    }
    const bool failed = !s->err.empty();
    delete s;
    return failed ? DPCS_E_DEVICE : DPCS_OK;
}

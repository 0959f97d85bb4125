// Serving loop: many robots' maps resident in HBM, scans fused as they arrive.
//
// A scheduler thread keeps n_streams "lanes" (a batch context on its own
// stream each). Whenever a lane is free it takes, in arrival order, every
// queued scan whose map is not running on another lane, up to the batch
// limits, and enqueues them as one batched integration; the other lanes keep
// running meanwhile, so work that arrived later overlaps work already on the
// GPU (continuous batching). A lane's completion is observed by polling its
// event; every scan of the batch is then stamped done. Maps are admitted while
// their eq. 1 storage fits the memory budget.
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <vector>

#include "runtime.h"

using namespace dbtsdf;

namespace {

struct Request {
    uint64_t ticket = 0;
    uint32_t map = 0;
    float pose[16];
    float *pts = nullptr;   // pinned host copy: the points, then (a sweep) the time fractions
    size_t cap = 0;         // floats in pts
    uint64_t n = 0;
    uint64_t t_arrival = 0;
    int kind = -1;          // -1: a plain scan; else a motion-compensated sweep of this dbtsdf_deskew mode
    float pose_end[16];
};

struct MapSlot {
    dbtsdf_grid *grid = nullptr;
    uint64_t bytes = 0;
    bool busy = false;      // in a running batch
    bool removing = false;
};

struct Lane {
    dbtsdf_batch *batch = nullptr;
    hipEvent_t ev = nullptr;
    bool running = false;
    dbtsdf_status status = DBTSDF_OK;
    uint64_t t_launch = 0;
    std::vector<Request> reqs;
    std::vector<dbtsdf_scan_stats> stats;
};

}  // namespace

struct dbtsdf_server {
    dbtsdf_server_config cfg{};
    int device = 0;
    hipStream_t admin = nullptr;
    std::mutex mu;
    std::condition_variable cv_done;
    // a deque: add_map's push_back never moves a slot, so a reference held
    // across a wait that releases mu (remove_map) stays valid
    std::deque<MapSlot> maps;
    std::deque<Request> queue;
    std::vector<Lane> lanes;
    std::deque<dbtsdf_completion> done;
    std::multimap<size_t, float *> pool;   // free pinned buffers by capacity (floats)
    uint64_t admitted = 0, budget = 0;
    uint64_t next_ticket = 1, submitted = 0, completed = 0;
    std::atomic<bool> stop{false};
    std::thread sched;

    float *take_buffer(size_t floats, size_t *cap);
    void give_buffer(float *p, size_t cap) { pool.emplace(cap, p); }
    void loop();
    bool poll_lanes();
    bool launch_free_lanes();
};

float *dbtsdf_server::take_buffer(size_t floats, size_t *cap) {
    auto it = pool.lower_bound(floats);
    if (it != pool.end() && it->first <= 4 * std::max<size_t>(floats, 1024)) {
        float *p = it->second;
        *cap = it->first;
        pool.erase(it);
        return p;
    }
    size_t c = 1024;
    while (c < floats) c <<= 1;
    void *p = nullptr;
    if (hipHostMalloc(&p, c * sizeof(float), hipHostMallocDefault) != hipSuccess) return nullptr;
    *cap = c;
    return (float *)p;
}

bool dbtsdf_server::poll_lanes() {
    bool any = false;
    for (Lane &ln : lanes) {
        if (!ln.running) continue;
        hipError_t q = hipEventQuery(ln.ev);
        if (q == hipErrorNotReady) continue;
        // the batch has finished (or failed): deliver statistics
        dbtsdf_status bs = q == hipSuccess ? dbtsdf_batch_sync(ln.batch) : DBTSDF_ERR_DEVICE;
        if (ln.status != DBTSDF_OK) bs = ln.status;
        const uint64_t t_done = dbtsdf_now_ns();
        std::lock_guard<std::mutex> lk(mu);
        for (size_t i = 0; i < ln.reqs.size(); ++i) {
            Request &r = ln.reqs[i];
            dbtsdf_completion c{};
            c.ticket = r.ticket;
            c.map_id = r.map;
            c.status = (uint32_t)bs;
            c.t_arrival_ns = r.t_arrival;
            c.t_launch_ns = ln.t_launch;
            c.t_done_ns = t_done;
            c.batch_scans = (uint32_t)ln.reqs.size();
            c.stats = ln.stats[i];
            done.push_back(c);
            maps[r.map].busy = false;
            give_buffer(r.pts, r.cap);
            ++completed;
        }
        ln.reqs.clear();
        ln.running = false;
        any = true;
        cv_done.notify_all();
    }
    return any;
}

bool dbtsdf_server::launch_free_lanes() {
    bool any = false;
    for (Lane &ln : lanes) {
        if (ln.running) continue;
        std::vector<Request> pick;
        std::vector<dbtsdf_grid *> grids;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (queue.empty()) break;
            std::unordered_set<uint32_t> blocked;
            uint64_t pts = 0;
            // one launch holds one kind of request (plain scans, or sweeps of
            // one mode): the first picked sets it
            int kind = 0;
            for (auto it = queue.begin(); it != queue.end() && pick.size() < cfg.max_batch_scans;) {
                MapSlot &m = maps[it->map];
                if (m.busy || blocked.count(it->map) || (!pick.empty() && it->kind != kind)) {
                    blocked.insert(it->map);  // keep per-map arrival order
                    ++it;
                    continue;
                }
                kind = it->kind;
                if (!pick.empty() && pts + it->n > cfg.max_batch_points) break;
                pts += it->n;
                pick.push_back(*it);
                it = queue.erase(it);
            }
            for (Request &r : pick) {
                maps[r.map].busy = true;
                grids.push_back(maps[r.map].grid);
            }
        }
        if (pick.empty()) continue;
        const uint32_t n = (uint32_t)pick.size();
        const int kind = pick[0].kind;
        std::vector<float> poses(16 * (size_t)n), poses_end(kind >= 0 ? 16 * (size_t)n : 0);
        std::vector<const float *> ptrs(n), times(n);
        std::vector<uint64_t> counts(n);
        for (uint32_t i = 0; i < n; ++i) {
            std::memcpy(&poses[16 * (size_t)i], pick[i].pose, sizeof(pick[i].pose));
            if (kind >= 0) std::memcpy(&poses_end[16 * (size_t)i], pick[i].pose_end, sizeof(pick[i].pose_end));
            ptrs[i] = pick[i].pts;
            times[i] = pick[i].pts + 3 * pick[i].n;
            counts[i] = pick[i].n;
        }
        ln.stats.assign(n, dbtsdf_scan_stats{});
        ln.t_launch = dbtsdf_now_ns();
        dbtsdf_status s =
            kind < 0 ? dbtsdf_batch_integrate(ln.batch, n, grids.data(), poses.data(), ptrs.data(), counts.data(), 0,
                                              ln.stats.data())
                     : dbtsdf_batch_integrate_deskew(ln.batch, n, grids.data(), poses.data(), poses_end.data(), kind,
                                                     ptrs.data(), times.data(), counts.data(), 0, ln.stats.data());
        hipError_t e = hipSuccess;
        if (s == DBTSDF_OK) e = hipEventRecord(ln.ev, ln.batch->stream);
        ln.reqs = std::move(pick);
        ln.running = true;
        ln.status = s != DBTSDF_OK ? s : (e != hipSuccess ? DBTSDF_ERR_DEVICE : DBTSDF_OK);
        if (s != DBTSDF_OK || e != hipSuccess) {
            // the failure is reported on every scan of the batch at the next poll
            (void)hipEventRecord(ln.ev, ln.batch->stream);
        }
        any = true;
    }
    return any;
}

void dbtsdf_server::loop() {
    (void)hipSetDevice(device);
    while (!stop.load()) {
        bool a = poll_lanes();
        bool b = launch_free_lanes();
        if (!a && !b) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

extern "C" {

dbtsdf_status dbtsdf_server_create(const dbtsdf_server_config *cfg, dbtsdf_server **out) {
    if (!out) {
        set_error("NULL out");
        return DBTSDF_ERR_INVALID_ARG;
    }
    auto s = std::make_unique<dbtsdf_server>();
    dbtsdf_server_config c{};
    if (cfg) c = *cfg;
    if (c.n_streams == 0) c.n_streams = 2;
    if (c.n_streams > 16) {
        set_error("n_streams must be <= 16");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (c.max_batch_scans == 0) c.max_batch_scans = 64;
    if (c.max_batch_points == 0) c.max_batch_points = 4ull << 20;
    if (c.queue_capacity == 0) c.queue_capacity = 4096;
    s->cfg = c;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->admin, hipStreamNonBlocking);
    if (e != hipSuccess) return check_hip(e, "server: device setup");
    size_t free_b = 0, total_b = 0;
    e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return check_hip(e, "server: hipMemGetInfo");
    const uint64_t reserve = 8ull << 30;
    s->budget = c.memory_budget ? c.memory_budget : (free_b > reserve ? free_b - reserve : 0);
    s->lanes.resize(c.n_streams);
    for (Lane &ln : s->lanes) {
        dbtsdf_status st = dbtsdf_batch_create(nullptr, c.use_graph ? 1 : 0, &ln.batch);
        if (st != DBTSDF_OK) return st;
        e = hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming);
        if (e != hipSuccess) return check_hip(e, "server: event");
    }
    dbtsdf_server *raw = s.release();
    raw->sched = std::thread([raw] { raw->loop(); });
    *out = raw;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_server_add_map(dbtsdf_server *s, const dbtsdf_grid_params *params, const dbtsdf_kernel_set *ks,
                                    uint32_t *map_id) {
    if (!s || !params || !ks || !map_id) {
        set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    const uint64_t bytes = dbtsdf_grid_bytes(params);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->admitted + bytes > s->budget) {
            set_error("map does not fit the server's memory budget");
            return DBTSDF_ERR_OUT_OF_MEMORY;
        }
        s->admitted += bytes;  // reserve before allocating
    }
    dbtsdf_grid *g = nullptr;
    dbtsdf_status st = dbtsdf_create_grid(params, ks, s->admin, &g);
    if (st == DBTSDF_OK) st = dbtsdf_sync(g);
    std::lock_guard<std::mutex> lk(s->mu);
    if (st != DBTSDF_OK) {
        s->admitted -= bytes;
        if (g) dbtsdf_destroy_grid(g);
        return st;
    }
    g->external_order = true;
    if (!s->maps.empty() && s->maps[0].grid) {
        // every map of a server shares one tuning so that maps batch together
        const dbtsdf_grid *g0 = s->maps[0].grid;
        g->tuning = g0->tuning;
    }
    MapSlot m;
    m.grid = g;
    m.bytes = bytes;
    s->maps.push_back(m);
    *map_id = (uint32_t)(s->maps.size() - 1);
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_server_remove_map(dbtsdf_server *s, uint32_t map_id) {
    if (!s) return DBTSDF_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    if (map_id >= s->maps.size() || !s->maps[map_id].grid) {
        set_error("unknown map");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (s->maps[map_id].removing) {
        set_error("map is already being removed");
        return DBTSDF_ERR_INVALID_ARG;
    }
    s->maps[map_id].removing = true;
    // the wait releases mu: other threads may add maps meanwhile, so the slot
    // is looked up again by index rather than held across it
    s->cv_done.wait(lk, [&] {
        if (s->maps[map_id].busy) return false;
        for (const Request &r : s->queue)
            if (r.map == map_id) return false;
        return true;
    });
    MapSlot &m = s->maps[map_id];
    dbtsdf_destroy_grid(m.grid);
    m.grid = nullptr;
    s->admitted -= m.bytes;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_server_map_grid(dbtsdf_server *s, uint32_t map_id, dbtsdf_grid **g) {
    if (!s || !g) return DBTSDF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (map_id >= s->maps.size() || !s->maps[map_id].grid) {
        set_error("unknown map");
        return DBTSDF_ERR_INVALID_ARG;
    }
    *g = s->maps[map_id].grid;
    return DBTSDF_OK;
}

static dbtsdf_status submit_impl(dbtsdf_server *s, uint32_t map_id, const float pose[16], const float *pose_end,
                                 int mode, const float *points, const float *times, uint64_t n,
                                 uint64_t t_arrival_ns, uint64_t *ticket) {
    if (!s || !pose || (n && !points) || (pose_end && n && !times)) {
        set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(pose[k]) || (pose_end && !std::isfinite(pose_end[k]))) {
            set_error("pose must be finite");
            return DBTSDF_ERR_INVALID_ARG;
        }
    if (pose_end && mode != DBTSDF_DESKEW_SE3 && mode != DBTSDF_DESKEW_YAW) {
        set_error("unknown deskew mode");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (n > kMaxPointsPerCall) return DBTSDF_ERR_OUT_OF_RANGE;
    std::lock_guard<std::mutex> lk(s->mu);
    if (map_id >= s->maps.size() || !s->maps[map_id].grid || s->maps[map_id].removing) {
        set_error("unknown map");
        return DBTSDF_ERR_INVALID_ARG;
    }
    if (s->queue.size() >= s->cfg.queue_capacity) {
        set_error("server queue is full");
        return DBTSDF_ERR_BUSY;
    }
    Request r;
    r.ticket = s->next_ticket++;
    r.map = map_id;
    std::memcpy(r.pose, pose, sizeof(r.pose));
    r.kind = pose_end ? mode : -1;
    if (pose_end) std::memcpy(r.pose_end, pose_end, sizeof(r.pose_end));
    r.pts = s->take_buffer((pose_end ? 4 : 3) * std::max<uint64_t>(n, 1), &r.cap);
    if (!r.pts) {
        set_error("pinned staging allocation failed");
        return DBTSDF_ERR_OUT_OF_MEMORY;
    }
    if (n) std::memcpy(r.pts, points, 12 * n);
    if (n && pose_end) std::memcpy(r.pts + 3 * n, times, 4 * n);
    r.n = n;
    r.t_arrival = t_arrival_ns;
    s->queue.push_back(r);
    ++s->submitted;
    if (ticket) *ticket = r.ticket;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_server_submit(dbtsdf_server *s, uint32_t map_id, const float pose[16], const float *points,
                                   uint64_t n, uint64_t t_arrival_ns, uint64_t *ticket) {
    return submit_impl(s, map_id, pose, nullptr, 0, points, nullptr, n, t_arrival_ns, ticket);
}

dbtsdf_status dbtsdf_server_submit_sweep(dbtsdf_server *s, uint32_t map_id, const float pose_start[16],
                                         const float pose_end[16], int mode, const float *points, const float *times,
                                         uint64_t n, uint64_t t_arrival_ns, uint64_t *ticket) {
    if (!pose_end) {
        set_error("NULL argument");
        return DBTSDF_ERR_INVALID_ARG;
    }
    return submit_impl(s, map_id, pose_start, pose_end, mode, points, times, n, t_arrival_ns, ticket);
}

dbtsdf_status dbtsdf_server_poll(dbtsdf_server *s, dbtsdf_completion *out, uint32_t max, uint32_t *n_out) {
    if (!s || (max && !out)) return DBTSDF_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    uint32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    if (n_out) *n_out = k;
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_server_drain(dbtsdf_server *s) {
    if (!s) return DBTSDF_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->completed == s->submitted; });
    return DBTSDF_OK;
}

dbtsdf_status dbtsdf_server_memory(const dbtsdf_server *s, uint64_t *admitted, uint64_t *budget) {
    if (!s) return DBTSDF_ERR_INVALID_ARG;
    if (admitted) *admitted = s->admitted;
    if (budget) *budget = s->budget;
    return DBTSDF_OK;
}

void dbtsdf_server_destroy(dbtsdf_server *s) {
    if (!s) return;
    (void)dbtsdf_server_drain(s);
    s->stop.store(true);
    if (s->sched.joinable()) s->sched.join();
    for (Lane &ln : s->lanes) {
        if (ln.batch) dbtsdf_batch_destroy(ln.batch);
        if (ln.ev) (void)hipEventDestroy(ln.ev);
    }
    for (MapSlot &m : s->maps)
        if (m.grid) dbtsdf_destroy_grid(m.grid);
    for (auto &kv : s->pool) (void)hipHostFree(kv.second);
    for (Request &r : s->queue) (void)hipHostFree(r.pts);
    if (s->admin) (void)hipStreamDestroy(s->admin);
    delete s;
}

}  // extern "C"
